// Host-side helpers shared by the C-ABI entry points (declared in host.h).
#include "host.h"

#include <algorithm>
#include <atomic>
#include <unordered_map>

namespace me {
namespace host {

namespace {
std::atomic<int> g_arch_ok{-1};  // -1 unknown, 0 no, 1 yes
}

int hip_err(hipError_t e) { return e == hipSuccess ? ME_OK : ME_EHIP; }

int check_device(int dev) {
    int ok = g_arch_ok.load();
    if (ok < 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ME_ENODEV;
        ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
        g_arch_ok.store(ok);
    }
    return ok ? ME_OK : ME_ENODEV;
}

int check_frame(const me_frame &f, bool need_alpha) {
    if (!f.luma) return ME_EINVAL;
    if (need_alpha && !f.alpha) return ME_EINVAL;
    if (f.width <= 0 || f.height <= 0 || f.width > kMaxDim || f.height > kMaxDim) return ME_EINVAL;
    if (f.width % 16 || f.height % 16) return ME_EALIGN;
    if (f.stride < f.width || f.stride % 4) return ME_EALIGN;
    if (!al4(f.luma) || (f.alpha && !al4(f.alpha))) return ME_EALIGN;
    return ME_OK;
}

int check_params(const me_params *p) {
    if (!p) return ME_EINVAL;
    if (p->search_range < 1 || p->search_range > 64) return ME_EINVAL;
    if (p->theta < 1 || p->theta > 127) return ME_EINVAL;
    if (p->eps_q12 < 0 || p->eps_q12 > 65536) return ME_EINVAL;
    if (p->max_step < 1 || p->max_step > p->search_range) return ME_EINVAL;
    if (p->k_max < 0 || p->k_max > 255) return ME_EINVAL;
    if (p->half_pel != 0 && p->half_pel != 1) return ME_EINVAL;
    if (p->flags & ~(ME_FLAG_LINE_WORKERS | ME_FLAG_UNRESTRICTED | ME_FLAG_T_TEXTURE | ME_FLAG_MASKED_PRS))
        return ME_EINVAL;
    return ME_OK;
}

int check_job(const me_job &j, bool need_alpha) {
    int rc = check_frame(j.cur, need_alpha);
    if (rc) return rc;
    rc = check_frame(j.ref, need_alpha);
    if (rc) return rc;
    if (j.cur.width != j.ref.width || j.cur.height != j.ref.height || j.cur.stride != j.ref.stride) return ME_EINVAL;
    if ((j.cur.alpha == nullptr) != (j.ref.alpha == nullptr)) return ME_EINVAL;
    if (!j.mv || !j.mv_int) return ME_EINVAL;
    if (!al4(j.mv) || !al4(j.mv_int) || (j.t_field && !al4(j.t_field)) || (j.seed && !al4(j.seed)))
        return ME_EALIGN;
    if (j.t_field && (const void *)j.t_field == (const void *)j.mv_int) return ME_EINVAL;
    return ME_OK;
}

KParams kparams(const me_params *p, bool shape_only) {
    KParams k;
    k.S = p->search_range;
    k.theta = p->theta;
    k.eps = p->eps_q12;
    k.max_step = p->max_step;
    k.k_max = p->k_max;
    k.half_pel = p->half_pel;
    k.shape_only = shape_only ? 1 : 0;
    k.spin_limit = kSpinLimit;
    k.poll_sleep = 2;
    // eps * U rounds to a zero step iff |eps * U| < 2^23, i.e. |U| < ceil(2^23 / eps)
    k.zero_t = p->eps_q12 > 0 ? (int32_t)(((1ll << 23) + p->eps_q12 - 1) / p->eps_q12) : 0x7FFFFFFF;
    k.unrestricted = (p->flags & ME_FLAG_UNRESTRICTED) ? 1 : 0;
    k.t_texture = (p->flags & ME_FLAG_T_TEXTURE) ? 1 : 0;
    k.masked_prs = (p->flags & ME_FLAG_MASKED_PRS) && !shape_only ? 1 : 0;
    return k;
}

JobDesc job_desc(const me_job &j) {
    JobDesc d;
    std::memset(&d, 0, sizeof(d));
    d.cur = j.cur.luma;
    d.ref = j.ref.luma;
    d.cur_a = j.cur.alpha;
    d.ref_a = j.ref.alpha;
    d.cls = j.mb_class;
    d.tf = (const int16_t *)j.t_field;
    d.seed = (const int16_t *)j.seed;
    d.mv = (int16_t *)j.mv;
    d.mv_int = (int16_t *)j.mv_int;
    d.cost = j.cost;
    d.iters = j.iters;
    d.points = j.points;
    d.width = j.cur.width;
    d.height = j.cur.height;
    d.stride = j.cur.stride;
    d.wm = j.cur.width / 16;
    d.hm = j.cur.height / 16;
    d.dep_line_base = -1;
    return d;
}

int mc_desc(const me_job &j, uint8_t *pred, JobDesc *out) {
    int rc = check_frame(j.cur, false);
    if (rc) return rc;
    rc = check_frame(j.ref, false);
    if (rc) return rc;
    if (j.cur.width != j.ref.width || j.cur.height != j.ref.height || j.cur.stride != j.ref.stride) return ME_EINVAL;
    if (!j.mv) return ME_EINVAL;
    if (!al4(j.mv)) return ME_EALIGN;
    if (pred && !al4(pred)) return ME_EALIGN;
    *out = job_desc(j);
    out->out_u8 = pred;
    return ME_OK;
}

int build_pa(const me_job *jobs, int n, PaMemo &m) {
    // chains: a job whose T field is the mv_int of an earlier job follows it
    std::unordered_map<const void *, int> producer;
    for (int i = 0; i < n; ++i) {
        if (!producer.emplace((const void *)jobs[i].mv_int, i).second) return ME_EINVAL;  // shared output
    }
    std::vector<JobDesc> desc(n);
    std::vector<int> chain_of(n), pos_of(n), prod_of(n, -1);
    std::vector<std::vector<int>> chains;
    for (int i = 0; i < n; ++i) {
        desc[i] = job_desc(jobs[i]);
        int prod = -1;
        if (jobs[i].t_field) {
            auto it = producer.find((const void *)jobs[i].t_field);
            if (it != producer.end()) {
                if (it->second >= i) return ME_EINVAL;  // would read a field written later in this call
                prod = it->second;
            }
        }
        prod_of[i] = prod;
        if (prod >= 0) {
            if (desc[prod].wm != desc[i].wm || desc[prod].hm != desc[i].hm) return ME_EINVAL;
            int c = chain_of[prod];
            if (chains[c].back() == prod) {
                chains[c].push_back(i);
                chain_of[i] = c;
                pos_of[i] = (int)chains[c].size() - 1;
                desc[i].t_local = 1;
            } else {
                chain_of[i] = (int)chains.size();
                pos_of[i] = 0;
                chains.push_back({i});
            }
            desc[i].dep_pos = pos_of[prod];
            desc[i].dep_line_base = -2 - chain_of[prod];  // resolved below
        } else {
            chain_of[i] = (int)chains.size();
            pos_of[i] = 0;
            chains.push_back({i});
        }
    }
    const int nc = (int)chains.size();
    if (nc > kMaxChains) return ME_EINVAL;
    for (const auto &ch : chains)
        if (ch.size() > 65535) return ME_EINVAL;  // progress words count pairs in 16 bits
    // descriptors in chain order: chain c's pair p at cd[c].first + p
    std::vector<ChainDesc> cd(nc);
    std::vector<JobDesc> ordered;
    ordered.reserve(n);
    std::vector<int> order;
    order.reserve(n);
    long long nlines = 0;
    int maxkey = 0;
    int maxlen = 0;
    long long total_mbs = 0;
    for (int c = 0; c < nc; ++c) {
        const JobDesc &d0 = desc[chains[c][0]];
        cd[c] = ChainDesc{(int32_t)ordered.size(), (int32_t)chains[c].size(), d0.wm, d0.hm, (int32_t)nlines, {0, 0, 0}};
        int pos = 0;
        for (int i : chains[c]) {
            order.push_back(i);
            ordered.push_back(desc[i]);
            JobDesc &d = ordered.back();
            d.chain_line_base = (int32_t)nlines;
            d.chain_pos = pos++;
            d.mb_base = (int32_t)total_mbs;
            total_mbs += (long long)d.wm * d.hm;
        }
        nlines += (long long)d0.wm * d0.hm;
        maxkey = std::max(maxkey, (d0.wm - 1) + 2 * (d0.hm - 1));
        maxlen = std::max(maxlen, (int)chains[c].size());
    }
    if (total_mbs > (1ll << 30)) return ME_EINVAL;
    if (nlines > (1ll << 30)) return ME_EINVAL;
    for (auto &d : ordered)
        if (d.dep_line_base <= -2) d.dep_line_base = cd[-2 - d.dep_line_base].line_base;
    // tickets in the order (h + 2v, chain): counting sort on the key
    std::vector<uint32_t> cnt(maxkey + 2, 0);
    for (int c = 0; c < nc; ++c)
        for (int v = 0; v < cd[c].hm; ++v)
            for (int h = 0; h < cd[c].wm; ++h) cnt[h + 2 * v + 1]++;
    for (int key = 1; key <= maxkey + 1; ++key) cnt[key] += cnt[key - 1];
    std::vector<uint32_t> tickets((size_t)nlines);
    for (int c = 0; c < nc; ++c)
        for (int v = 0; v < cd[c].hm; ++v)
            for (int h = 0; h < cd[c].wm; ++h)
                tickets[cnt[h + 2 * v]++] = ((uint32_t)c << 16) | ((uint32_t)v << 8) | (uint32_t)h;

    // bands of kRowWaves MB rows for the row workers (job sets without
    // chains inside the call), in the order (first row, chain)
    std::vector<uint32_t> bands;
    const bool unchained = nc == n;
    if (unchained) {
        int maxhm = 0;
        for (int c = 0; c < nc; ++c) maxhm = std::max(maxhm, (int)cd[c].hm);
        for (int v0 = 0; v0 < maxhm; v0 += kRowWaves)
            for (int c = 0; c < nc; ++c)
                if (v0 < cd[c].hm) bands.push_back(((uint32_t)c << 16) | (uint32_t)v0);
    }

    m.blob.clear();
    m.o_jobs = put(m.blob, ordered.data(), ordered.size());
    m.o_ch = put(m.blob, cd.data(), cd.size());
    m.o_tk = put(m.blob, tickets.data(), tickets.size());
    m.o_bands = put(m.blob, bands.data(), bands.size());
    m.nbands = (int)bands.size();
    m.unchained = unchained;
    m.n = n;
    m.total_mbs = (int)total_mbs;
    m.nlines = (int)nlines;
    m.mask_words = (maxlen + 31) / 32;
    m.nchains = nc;
    m.order.swap(order);
    m.prod.swap(prod_of);
    return ME_OK;
}

}  // namespace host
}  // namespace me

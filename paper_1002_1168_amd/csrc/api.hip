// Host side of the C ABI: argument validation (before any HIP call), per-stream
// workspaces (device scratch + pinned staging), chain / ticket construction
// for the pipelined block-recursive search, and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "flat_kernels.h"
#include "host.h"
#include "me_internal.h"

namespace me {
size_t es_lds_bytes(int S);
}

using namespace me;
using namespace me::host;

namespace {

constexpr int kRing = 4;

struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
};

// Device scratch of one kind of call (classification, search, baselines,
// MC): descriptors stay resident between calls of the same kind, so a
// repeated call with the same jobs uploads nothing.
struct Arena {
    uint8_t *dev = nullptr;
    size_t cap = 0;
    std::vector<uint8_t> last;  // content of the last upload
    bool last_valid = false;
};

enum ArenaKind { A_CLASSIFY = 0, A_PA = 1, A_SEARCH = 2, A_MC = 3, A_PRS8 = 4, A_PAD = 5, A_COUNT = 6 };
// timing kinds: the first four arena kinds (ME_KT_*), the network forward and
// training kernels, then the 8 x 8 refinement
constexpr int kTimerKinds = 7;


// Event pairs of timed launches of one call kind: in flight until their
// stop event has completed, then summed.
struct TimerPool {
    std::vector<KernelTimer> free, inflight;
    double total_ms = 0.0;
    int count = 0;
    void harvest(bool wait) {
        size_t k = 0;
        for (auto &t : inflight) {
            hipError_t q = wait ? hipEventSynchronize(t.stop) : hipEventQuery(t.stop);
            if (q == hipErrorNotReady) {
                inflight[k++] = t;
                continue;
            }
            float ms = 0.f;
            if (q == hipSuccess && hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
                total_ms += ms;
                count++;
            }
            free.push_back(t);
        }
        inflight.resize(k);
    }
};

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena[A_COUNT];
    uint32_t *status = nullptr;  // persistent device status word
    Staging ring[kRing];
    int slot = 0;
    PaMemo pa;
    unsigned long long *host_acc = nullptr;  // pinned readback for MC
    size_t host_acc_cap = 0;
    TimerPool timers[kTimerKinds];  // main-kernel events per call kind (timing on)
    std::mutex mu;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;
std::atomic<int> g_timing{0};



int get_ws(void *stream, Workspace **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ME_ENODEV;
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = check_device(dev);
    if (rc) return rc;
    auto key = std::make_pair(dev, (hipStream_t)stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return ME_OK;
    }
    Workspace *w = new Workspace();
    w->device = dev;
    w->stream = (hipStream_t)stream;
    if (hipMalloc(&w->status, 256) != hipSuccess) {
        delete w;
        return ME_ENOMEM;
    }
    if (hipMemset(w->status, 0, 256) != hipSuccess) {
        hipFree(w->status);
        delete w;
        return ME_EHIP;
    }
    for (auto &s : w->ring)
        if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) return ME_EHIP;
    g_ws[key] = w;
    *out = w;
    return ME_OK;
}


// Event pair for the main kernel of a call of `kind` (false when timing is off).
// Whether calls of `kind` are timed: timing mask 1 = every kind, else bit
// kind + 1.
bool timing_on(int kind) {
    const int m = g_timing.load(std::memory_order_relaxed);
    return m == 1 || ((m >> (kind + 1)) & 1);
}

bool timer_for(Workspace &w, int kind, KernelTimer *out) {
    if (!timing_on(kind)) return false;
    TimerPool &p = w.timers[kind];
    p.harvest(false);
    KernelTimer t;
    if (!p.free.empty()) {
        t = p.free.back();
        p.free.pop_back();
    } else {
        if (hipEventCreate(&t.start) != hipSuccess) return false;
        if (hipEventCreate(&t.stop) != hipSuccess) {
            hipEventDestroy(t.start);
            return false;
        }
    }
    p.inflight.push_back(t);
    *out = t;
    return true;
}

// Copy `blob` to the start of the arena of `kind` (skipped when the arena
// still holds exactly these bytes), zero `zero_bytes` after it and reserve
// `scratch_bytes` more.  Returns the arena base, zeroed and scratch regions.
int upload(Workspace &w, int kind, const std::vector<uint8_t> &blob, size_t zero_bytes, uint8_t **base,
           uint8_t **zero, size_t scratch_bytes = 0, uint8_t **scratch = nullptr) {
    Arena &ar = w.arena[kind];
    size_t off = align_up(blob.size(), 256);
    size_t need = off + align_up(zero_bytes, 256) + align_up(scratch_bytes, 256) + 256;
    if (need > ar.cap) {
        if (ar.dev) {
            if (hipStreamSynchronize(w.stream) != hipSuccess) return ME_EHIP;
            hipFree(ar.dev);
            ar.dev = nullptr;
            ar.cap = 0;
        }
        size_t cap = std::max(need + need / 4, (size_t)1 << 20);
        if (hipMalloc(&ar.dev, cap) != hipSuccess) return ME_ENOMEM;
        ar.cap = cap;
        ar.last_valid = false;
    }
    bool same = ar.last_valid && ar.last.size() == blob.size() &&
                std::memcmp(ar.last.data(), blob.data(), blob.size()) == 0;
    if (!same && !blob.empty()) {
        Staging &s = w.ring[w.slot];
        w.slot = (w.slot + 1) % kRing;
        if (hipEventSynchronize(s.ev) != hipSuccess) return ME_EHIP;
        if (s.cap < blob.size()) {
            if (s.host) hipHostFree(s.host);
            s.host = nullptr;
            size_t cap = std::max(align_up(blob.size(), 4096), (size_t)1 << 16);
            if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess) {
                s.cap = 0;
                return ME_ENOMEM;
            }
            s.cap = cap;
        }
        std::memcpy(s.host, blob.data(), blob.size());
        if (hipMemcpyAsync(ar.dev, s.host, blob.size(), hipMemcpyHostToDevice, w.stream) != hipSuccess)
            return ME_EHIP;
        if (hipEventRecord(s.ev, w.stream) != hipSuccess) return ME_EHIP;
        ar.last = blob;
        ar.last_valid = true;
    }
    *base = ar.dev;
    *zero = ar.dev + off;
    if (scratch) *scratch = ar.dev + off + align_up(zero_bytes, 256);
    if (zero_bytes) {
        int rc = hip_err(launch_fill_u32((uint32_t *)(ar.dev + off), align_up(zero_bytes, 4) / 4, 0u, w.stream));
        if (rc) return rc;
    }
    return ME_OK;
}









// The proposed algorithm for n jobs (shared by the texture and shape entry points).
int run_pa(const me_job *jobs, int n, const me_params *params, bool shape_only, void *stream) {
    if (n < 0 || (n > 0 && !jobs)) return ME_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        rc = check_job(jobs[i], shape_only);
        if (rc) return rc;
        if (jobs[i].seed && params->k_max > kMaxSeededKmax) return ME_EINVAL;
    }
    if (n == 0) return ME_OK;
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) {
        PaMemo probe;  // structural errors of the job set take precedence
        int vr = build_pa(jobs, n, probe);
        return vr ? vr : rc;
    }
    std::lock_guard<std::mutex> lk(w->mu);
    // a repeated call with byte-identical jobs reuses the prepared launch
    std::vector<uint8_t> key(sizeof(me_job) * (size_t)n + sizeof(me_params) + 1);
    std::memcpy(key.data(), jobs, sizeof(me_job) * (size_t)n);
    std::memcpy(key.data() + sizeof(me_job) * (size_t)n, params, sizeof(me_params));
    key.back() = shape_only ? 1 : 0;
    PaMemo &m = w->pa;
    if (!(m.valid && m.key == key)) {
        m.valid = false;
        rc = build_pa(jobs, n, m);
        if (rc) return rc;
        m.key.swap(key);
        m.valid = true;
    }
    // zeroed scratch: progress words, ticket counter, transparent and
    // boundary masks (one bit per pair, 32 pairs per word, per line)
    const size_t o_prog = 0;
    const size_t o_ctr = align_up((size_t)m.nlines * 8, 256);
    const size_t o_mask = o_ctr + 256;
    const size_t zero = o_mask + align_up((size_t)m.nlines * m.mask_words * 2 * 4, 256);
    uint8_t *base = nullptr, *zb = nullptr, *sb = nullptr;
    rc = upload(*w, A_PA, m.blob, zero, &base, &zb, pa_scratch_bytes(m.nlines), &sb);
    if (rc) return rc;
    KernelTimer kt;
    KParams kp = kparams(params, shape_only);
    if (m.unchained && !(params->flags & ME_FLAG_LINE_WORKERS)) {
        return hip_err(launch_pa_rows((const JobDesc *)(base + m.o_jobs), (const ChainDesc *)(base + m.o_ch),
                                      (const uint32_t *)(base + m.o_bands), m.nbands,
                                      (unsigned long long *)(zb + o_prog), (uint32_t *)(zb + o_ctr), w->status, kp,
                                      pa_rows_cap(kp.S, kp.half_pel != 0), w->stream, timer_for(*w, A_PA, &kt) ? &kt : nullptr));
    }
    // the several-wave line worker scores every candidate on the MB's own
    // plane; T on texture takes the one-wave worker
    const int waves = one_wave_lines(params->flags) ? 1 : lines_waves(m.nlines);
    int workers = std::min(m.nlines, pa_worker_cap() / waves);
    return hip_err(launch_pa((const JobDesc *)(base + m.o_jobs), m.n, m.total_mbs, (const ChainDesc *)(base + m.o_ch),
                             (const uint32_t *)(base + m.o_tk), m.nlines, (unsigned long long *)(zb + o_prog),
                             (uint32_t *)(zb + o_ctr), (uint32_t *)(zb + o_mask), m.mask_words, sb, w->status, kp,
                             workers, w->stream, timer_for(*w, A_PA, &kt) ? &kt : nullptr, false, waves));
}

}  // namespace

namespace me {
namespace host {

bool timing_enabled(int kind) { return kind >= 0 && kind < kTimerKinds && timing_on(kind); }

bool kernel_timer(void *stream, int kind, KernelTimer *out) {
    if (kind < 0 || kind >= kTimerKinds || !timing_on(kind)) return false;
    Workspace *w = nullptr;
    if (get_ws(stream, &w) != ME_OK) return false;
    std::lock_guard<std::mutex> lk(w->mu);
    return timer_for(*w, kind, out);
}

}  // namespace host
}  // namespace me

extern "C" {

void me_default_params(me_params *p) {
    if (!p) return;
    p->search_range = 16;
    p->theta = 3;
    p->eps_q12 = 4096;
    p->max_step = 1;
    p->k_max = 8;
    p->half_pel = 0;
    p->flags = 0;
}

const char *me_status_str(int s) {
    switch (s) {
        case ME_OK: return "ok";
        case ME_EINVAL: return "invalid argument";
        case ME_EALIGN: return "frame size, stride or pointer alignment not supported";
        case ME_EHIP: return "HIP runtime error";
        case ME_ENOMEM: return "out of device or pinned memory";
        case ME_EEMPTY: return "PSNR over zero pixels";
        case ME_EDEVICE: return "device status word set";
        case ME_ENODEV: return "no gfx950 device";
        case ME_EFORMAT: return "network checkpoint malformed";
        case ME_EIO: return "network checkpoint file not readable or writable";
        default: return "unknown status";
    }
}

void me_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipDeviceSynchronize();
    for (auto &kv : g_ws) {
        Workspace *w = kv.second;
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(w->device);
        for (auto &ar : w->arena)
            if (ar.dev) hipFree(ar.dev);
        if (w->status) hipFree(w->status);
        for (auto &s : w->ring) {
            if (s.host) hipHostFree(s.host);
            if (s.ev) hipEventDestroy(s.ev);
        }
        if (w->host_acc) hipHostFree(w->host_acc);
        for (auto &p : w->timers) {
            for (auto *v : {&p.free, &p.inflight})
                for (auto &t : *v) {
                    hipEventDestroy(t.start);
                    hipEventDestroy(t.stop);
                }
        }
        hipSetDevice(cur);
        delete w;
    }
    g_ws.clear();
}

int me_classify_babs(const me_frame *frames, int n, uint8_t *const *mb_class, uint32_t *const *bab_bits,
                     void *stream) {
    if (n < 0 || (n > 0 && (!frames || !mb_class))) return ME_EINVAL;
    std::vector<JobDesc> desc(n);
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        int rc = check_frame(frames[i], true);
        if (rc) return rc;
        if (!mb_class[i]) return ME_EINVAL;
        if (bab_bits && bab_bits[i] && !al4(bab_bits[i])) return ME_EALIGN;
        JobDesc &d = desc[i];
        std::memset(&d, 0, sizeof(d));
        d.cur_a = frames[i].alpha;
        d.cls = mb_class[i];
        d.out_u32 = bab_bits ? bab_bits[i] : nullptr;
        d.width = frames[i].width;
        d.height = frames[i].height;
        d.stride = frames[i].stride;
        d.wm = d.width / 16;
        d.hm = d.height / 16;
        d.mb_base = (int32_t)total;
        d.dep_line_base = -1;
        total += (long long)d.wm * d.hm;
    }
    if (total > (1ll << 30)) return ME_EINVAL;
    if (n == 0) return ME_OK;
    Workspace *w = nullptr;
    int rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr;
    rc = upload(*w, A_CLASSIFY, blob, 0, &base, &zb);
    if (rc) return rc;
    KernelTimer kt;
    return hip_err(launch_classify((const JobDesc *)(base + o), n, (int)total, w->stream,
                                   timer_for(*w, A_CLASSIFY, &kt) ? &kt : nullptr));
}

int me_pad_vops(const me_frame *frames, int n, uint8_t *const *padded, void *stream) {
    if (n < 0 || (n > 0 && (!frames || !padded))) return ME_EINVAL;
    if (n > 65535) return ME_EINVAL;  // one grid row per VOP
    std::vector<JobDesc> desc(n);
    long long total = 0;
    int max_mbs = 0;
    for (int i = 0; i < n; ++i) {
        int rc = check_frame(frames[i], true);
        if (rc) return rc;
        if (!padded[i] || padded[i] == frames[i].luma || padded[i] == frames[i].alpha) return ME_EINVAL;
        if (!al4(padded[i])) return ME_EALIGN;
        JobDesc &d = desc[i];
        std::memset(&d, 0, sizeof(d));
        d.cur = frames[i].luma;
        d.cur_a = frames[i].alpha;
        d.out_u8 = padded[i];
        d.width = frames[i].width;
        d.height = frames[i].height;
        d.stride = frames[i].stride;
        d.wm = d.width / 16;
        d.hm = d.height / 16;
        d.mb_base = (int32_t)total;
        d.dep_line_base = -1;
        total += (long long)d.wm * d.hm;
        max_mbs = std::max(max_mbs, d.wm * d.hm);
    }
    if (total > (1ll << 30)) return ME_EINVAL;
    if (n == 0) return ME_OK;
    Workspace *w = nullptr;
    int rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr, *cls = nullptr;
    rc = upload(*w, A_PAD, blob, 0, &base, &zb, (size_t)total, &cls);
    if (rc) return rc;
    return hip_err(launch_pad((const JobDesc *)(base + o), n, max_mbs, cls, w->stream));
}

int me_texture_recursive(const me_job *jobs, int n, const me_params *params, const me_net *net, void *stream) {
    if (net) {
        // everything is validated before the network writes any seed
        if (n < 0 || (n > 0 && !jobs)) return ME_EINVAL;
        int rc = check_params(params);
        if (rc) return rc;
        for (int i = 0; i < n; ++i) {
            rc = check_job(jobs[i], false);
            if (rc) return rc;
            if (!jobs[i].seed) return ME_EINVAL;
        }
        if (params->k_max > kMaxSeededKmax) return ME_EINVAL;
        if (n == 0) return ME_OK;
        rc = net_seed_jobs(const_cast<me_net *>(net), jobs, n, stream);
        if (rc) return rc;
    }
    return run_pa(jobs, n, params, false, stream);
}

int me_shape_search(const me_job *jobs, int n, const me_params *params, void *stream) {
    return run_pa(jobs, n, params, true, stream);
}

int me_full_search(int method, const me_job *jobs, int n, const me_params *params, void *stream) {
    if (method != ME_ES && method != ME_TSS && method != ME_DS && method != ME_4SS) return ME_EINVAL;
    if (n < 0 || (n > 0 && !jobs)) return ME_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    std::vector<JobDesc> desc(n);
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        rc = check_job(jobs[i], false);
        if (rc) return rc;
        desc[i] = job_desc(jobs[i]);
        desc[i].tf = nullptr;
        desc[i].seed = nullptr;
        desc[i].mb_base = (int32_t)total;
        total += (long long)desc[i].wm * desc[i].hm;
    }
    if (total > (1ll << 30)) return ME_EINVAL;
    if (n == 0) return ME_OK;
    if (n > 65536) return ME_EINVAL;  // queue entries pack the job index in 16 bits
    if (method == ME_ES) {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) != hipSuccess) return ME_ENODEV;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return ME_EHIP;
        if (es_lds_bytes(params->search_range) > (size_t)lim) return ME_EINVAL;
    }
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr, *sb = nullptr;
    rc = upload(*w, A_SEARCH, blob, 256, &base, &zb, full_search_scratch((int)total), &sb);
    if (rc) return rc;
    KParams kp = kparams(params, false);
    KernelTimer kt;
    return hip_err(launch_full_search(method, (const JobDesc *)(base + o), n, (int)total, kp, (uint32_t *)zb,
                                      (uint32_t *)sb, w->status, w->stream,
                                      timer_for(*w, A_SEARCH, &kt) ? &kt : nullptr));
}

namespace {

// Descriptors of the jobs of an MC call, checked on the host (nothing
// touches the device); *total = their MB count.
int mc_descs(const me_job *jobs, int n, uint8_t *const *pred, std::vector<JobDesc> &desc, long long *total) {
    desc.resize(n);
    long long t = 0;
    for (int i = 0; i < n; ++i) {
        int rc = mc_desc(jobs[i], pred ? pred[i] : nullptr, &desc[i]);
        if (rc) return rc;
        desc[i].mb_base = (int32_t)t;
        t += (long long)desc[i].wm * desc[i].hm;
    }
    *total = t;
    return t > (1ll << 30) ? ME_EINVAL : ME_OK;
}

// Uploads the descriptors and queues the MC + SSE kernels on w's stream
// (w's lock held by the caller); the per-job sums (SSE, pixel count) land in
// `sums` (device, 2n), or in the workspace's scratch when `sums` is NULL
// (*acc_out: where they land).
int mc_enqueue(Workspace &w, const std::vector<JobDesc> &desc, long long total, unsigned long long *sums,
               unsigned long long **acc_out) {
    const int n = (int)desc.size();
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr, *sb = nullptr;
    const size_t acc_bytes = sums ? 0 : (size_t)n * 2 * sizeof(unsigned long long);
    int rc = upload(w, A_MC, blob, 0, &base, &zb, acc_bytes + mc_scratch((int)total), &sb);
    if (rc) return rc;
    unsigned long long *acc = sums ? sums : (unsigned long long *)sb;
    *acc_out = acc;
    bool sums_only = true;
    for (const JobDesc &d : desc) sums_only = sums_only && d.out_u8 == nullptr;
    KernelTimer kt;
    return hip_err(launch_mc((const JobDesc *)(base + o), n, (int)total, (uint32_t *)(sb + acc_bytes), acc,
                             w.status, w.stream, timer_for(w, A_MC, &kt) ? &kt : nullptr, 8, false, sums_only));
}

}  // namespace

int me_motion_compensate_psnr(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sse, uint64_t *npix,
                              double *psnr_db, void *stream) {
    if (n < 0 || (n > 0 && (!jobs || !sse || !npix || !psnr_db))) return ME_EINVAL;
    std::vector<JobDesc> desc;
    long long total = 0;
    int rc = mc_descs(jobs, n, pred, desc, &total);
    if (rc || n == 0) return rc;
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    unsigned long long *acc = nullptr;
    rc = mc_enqueue(*w, desc, total, nullptr, &acc);
    if (rc) return rc;
    const size_t acc_bytes = (size_t)n * 2 * sizeof(unsigned long long);
    if (w->host_acc_cap < acc_bytes) {
        if (w->host_acc) hipHostFree(w->host_acc);
        w->host_acc = nullptr;
        if (hipHostMalloc((void **)&w->host_acc, acc_bytes, hipHostMallocDefault) != hipSuccess) {
            w->host_acc_cap = 0;
            return ME_ENOMEM;
        }
        w->host_acc_cap = acc_bytes;
    }
    if (hipMemcpyAsync(w->host_acc, acc, acc_bytes, hipMemcpyDeviceToHost, w->stream) != hipSuccess) return ME_EHIP;
    if (hipStreamSynchronize(w->stream) != hipSuccess) return ME_EHIP;
    int status = ME_OK;
    for (int i = 0; i < n; ++i) {
        sse[i] = w->host_acc[2 * i];
        npix[i] = w->host_acc[2 * i + 1];
        if (npix[i] == 0) {
            psnr_db[i] = NAN;
            status = ME_EEMPTY;
        } else if (sse[i] == 0) {
            psnr_db[i] = INFINITY;
        } else {
            psnr_db[i] = 10.0 * std::log10(255.0 * 255.0 * (double)npix[i] / (double)sse[i]);
        }
    }
    return status;
}

int me_refine_8x8(const me_job *jobs, int n, const me_params *params, me_mv *const *mv4, uint32_t *const *cost4,
                  uint8_t *const *iters4, uint16_t *const *points4, void *stream) {
    if (n < 0 || (n > 0 && (!jobs || !mv4))) return ME_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    std::vector<JobDesc> desc(n);
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        rc = check_job(jobs[i], false);
        if (rc) return rc;
        if (!mv4[i]) return ME_EINVAL;
        if (!al4(mv4[i]) || (cost4 && cost4[i] && !al4(cost4[i])) || (points4 && points4[i] && ((uintptr_t)points4[i] & 1u)))
            return ME_EALIGN;
        JobDesc &d = desc[i];
        d = job_desc(jobs[i]);
        d.tf = (const int16_t *)jobs[i].mv;  // the MB's own vector, kept by boundary MBs
        d.seed = nullptr;
        d.mv = (int16_t *)mv4[i];
        d.mv_int = (int16_t *)jobs[i].mv_int;
        d.cost = cost4 ? cost4[i] : nullptr;
        d.iters = iters4 ? iters4[i] : nullptr;
        d.points = points4 ? points4[i] : nullptr;
        d.mb_base = (int32_t)total;
        total += (long long)d.wm * d.hm;
    }
    if (total > (1ll << 30)) return ME_EINVAL;
    if (n == 0) return ME_OK;
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr;
    rc = upload(*w, A_PRS8, blob, 0, &base, &zb);
    if (rc) return rc;
    KernelTimer kt;
    return hip_err(launch_prs8((const JobDesc *)(base + o), n, (int)total, kparams(params, false), w->stream,
                               timer_for(*w, ME_KT_REFINE8, &kt) ? &kt : nullptr));
}

int me_motion_compensate4_sse(const me_job *jobs, int n, const me_mv *const *mv4, uint8_t *const *pred,
                              uint64_t *sums, void *stream) {
    if (n < 0 || (n > 0 && (!jobs || !sums || !mv4))) return ME_EINVAL;
    if (((uintptr_t)sums & 7u) != 0) return ME_EALIGN;
    std::vector<JobDesc> desc;
    long long total = 0;
    int rc = mc_descs(jobs, n, pred, desc, &total);
    if (rc || n == 0) return rc;
    for (int i = 0; i < n; ++i) {
        if (!mv4[i]) return ME_EINVAL;
        if (!al4(mv4[i])) return ME_EALIGN;
        desc[i].mv = (int16_t *)mv4[i];
    }
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    std::vector<uint8_t> blob;
    size_t o = put(blob, desc.data(), desc.size());
    uint8_t *base = nullptr, *zb = nullptr, *sb = nullptr;
    rc = upload(*w, A_MC, blob, 0, &base, &zb, mc_scratch((int)total), &sb);
    if (rc) return rc;
    KernelTimer kt;
    return hip_err(launch_mc((const JobDesc *)(base + o), n, (int)total, (uint32_t *)sb, (unsigned long long *)sums,
                             w->status, w->stream, timer_for(*w, A_MC, &kt) ? &kt : nullptr, 8, true));
}

int me_motion_compensate_sse(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sums, void *stream) {
    if (n < 0 || (n > 0 && (!jobs || !sums))) return ME_EINVAL;
    if (((uintptr_t)sums & 7u) != 0) return ME_EALIGN;
    std::vector<JobDesc> desc;
    long long total = 0;
    int rc = mc_descs(jobs, n, pred, desc, &total);
    if (rc || n == 0) return rc;
    Workspace *w = nullptr;
    rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    unsigned long long *acc = nullptr;
    return mc_enqueue(*w, desc, total, (unsigned long long *)sums, &acc);
}

int me_search_schedule(const me_job *jobs, int n, int32_t *job_info, uint32_t *lines, int cap, int *nlines) {
    if (n <= 0 || !jobs || !job_info || !nlines || cap < 0 || (cap > 0 && !lines)) return ME_EINVAL;
    for (int i = 0; i < n; ++i) {
        int rc = check_job(jobs[i], false);
        if (rc) return rc;
    }
    PaMemo m;
    int rc = build_pa(jobs, n, m);
    if (rc) return rc;
    const ChainDesc *cd = (const ChainDesc *)(m.blob.data() + m.o_ch);
    const JobDesc *od = (const JobDesc *)(m.blob.data() + m.o_jobs);
    for (int c = 0; c < m.nchains; ++c) {
        for (int p = 0; p < cd[c].len; ++p) {
            const int q = cd[c].first + p;
            if (q >= n) return ME_EINVAL;
            const int j = m.order[q];
            job_info[3 * j] = c;
            job_info[3 * j + 1] = od[q].chain_pos;
            job_info[3 * j + 2] = m.prod[j];
        }
    }
    *nlines = m.nlines;
    if (cap < m.nlines) return ME_EINVAL;
    std::memcpy(lines, m.blob.data() + m.o_tk, sizeof(uint32_t) * (size_t)m.nlines);
    return ME_OK;
}

int me_kernel_timing(int on) {
    // 0, 1, or kind bits 1 .. kTimerKinds only
    if (on < 0 || (on > 1 && ((on & 1) || (on >> (kTimerKinds + 1)) != 0))) return ME_EINVAL;
    g_timing.store(on, std::memory_order_relaxed);
    return ME_OK;
}

int me_kernel_time_ms(int kind, void *stream, double *total_ms, int *count) {
    if (kind < 0 || kind >= kTimerKinds || !total_ms || !count) return ME_EINVAL;
    Workspace *w = nullptr;
    int rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    TimerPool &p = w->timers[kind];
    p.harvest(true);
    *total_ms = p.total_ms;
    *count = p.count;
    p.total_ms = 0.0;
    p.count = 0;
    return ME_OK;
}

int me_device_status(void *stream) {
    Workspace *w = nullptr;
    int rc = get_ws(stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    if (hipStreamSynchronize(w->stream) != hipSuccess) return ME_EHIP;
    uint32_t st = 0;
    if (hipMemcpy(&st, w->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return ME_EHIP;
    if (st) {
        if (hipMemset(w->status, 0, 4) != hipSuccess) return ME_EHIP;
        return ME_EDEVICE;
    }
    return ME_OK;
}

}  // extern "C"

// Batched frame step: classification, the proposed search and motion
// compensation + SSE for a fixed job structure (many VOP streams of any
// sizes), captured once into a HIP graph and replayed per frame step with
// only the job table rewritten.  The launch configuration (search workers,
// window staging, dependency-poll back-off, MBs per block of the flat
// kernels) is chosen at creation, optionally by timing the candidates on
// the first step's data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "flat_kernels.h"
#include "host.h"
#include "me_internal.h"

using namespace me;
using namespace me::host;

// kinds of kernel timing a batch graph can carry: classification, search,
// baselines (unused), MC, network forward
constexpr int kBatchKinds = ME_KT_NET + 1;

struct me_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int n = 0;
    bool shape = false;
    me_params params{};
    PaMemo plan;                    // chain structure, tickets, descriptor template
    std::vector<JobDesc> tmpl;      // chain-ordered descriptors of the creating job set
    uint8_t *dev = nullptr;         // one allocation, layout below
    size_t o_zero = 0, zero_bytes = 0, rows_zero_bytes = 0, o_pscr = 0, o_acc = 0, o_status = 0;
    void *host[2] = {nullptr, nullptr};  // pinned job-table staging
    hipEvent_t ev[2] = {nullptr, nullptr};  // recorded after the last untimed use of host[i]
    unsigned long long *host_acc = nullptr;
    // The frame step as two graphs used alternately: graph i copies the job
    // table from host[i], runs the step, and (kernel timing on at capture)
    // records event set i around the timed kernels as event nodes, so that
    // one replay's table and events are free while the next replay runs.
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    uint32_t timed = 0;                           // bit k: kind k (ME_KT_*) is timed
    KernelTimer tm[2][kBatchKinds];               // event pairs per set and kind
    bool pending[2] = {false, false};             // a replay with event set i whose events are unread
    double t_ms[kBatchKinds] = {0, 0, 0, 0, 0};
    int t_count[kBatchKinds] = {0, 0, 0, 0, 0};
    long long replays = 0;
    // workers, window staging (1 plan, 0 generic), poll sleep, flat MBs/CU,
    // waves per line (row workers: rows per band), row workers (1) or line workers (0)
    int32_t cfg[6] = {0, 1, 2, 8, 1, 0};
    me_net *net = nullptr;          // proposal network seeding the search (optional)
    uint8_t *net_scratch = nullptr;
    bool stepped = false;
    std::mutex mu;
};

namespace {

constexpr uint32_t kFlagsKnown = ME_BATCH_SHAPE | ME_BATCH_AUTOTUNE;

// Same structure as the creating job set: sizes, strides, which optional
// buffers are present, and which job feeds which T field.
int check_structure(const me_batch &b, const me_job *jobs, int n) {
    if (n != b.n || !jobs) return ME_EINVAL;
    std::unordered_map<const void *, int> producer;
    producer.reserve((size_t)n * 2);
    for (int i = 0; i < n; ++i) {
        int rc = check_job(jobs[i], b.shape);
        if (rc) return rc;
        if (!producer.emplace((const void *)jobs[i].mv_int, i).second) return ME_EINVAL;
    }
    for (int p = 0; p < n; ++p) {
        const int i = b.plan.order[p];
        const me_job &j = jobs[i];
        const JobDesc &d = b.tmpl[p];
        if (j.cur.width != d.width || j.cur.height != d.height || j.cur.stride != d.stride) return ME_EINVAL;
        if ((j.cur.alpha != nullptr) != (d.cur_a != nullptr)) return ME_EINVAL;
        if ((j.mb_class != nullptr) != (d.cls != nullptr)) return ME_EINVAL;
        if ((j.seed != nullptr) != (d.seed != nullptr)) return ME_EINVAL;
        if ((j.t_field != nullptr) != (d.tf != nullptr)) return ME_EINVAL;
        int prod = -1;
        if (j.t_field) {
            auto it = producer.find((const void *)j.t_field);
            if (it != producer.end()) prod = it->second;
        }
        if (prod != b.plan.prod[i]) return ME_EINVAL;
    }
    return ME_OK;
}

// Chain-ordered job table for `jobs` (structure already checked).
void fill_table(const me_batch &b, const me_job *jobs, JobDesc *out) {
    for (int p = 0; p < b.n; ++p) {
        const me_job &j = jobs[b.plan.order[p]];
        JobDesc d = b.tmpl[p];
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
        d.out_u8 = nullptr;
        d.out_u32 = nullptr;
        out[p] = d;
    }
}

struct Bufs {
    const JobDesc *jobs;
    const ChainDesc *chains;
    const uint32_t *tickets;
    const uint32_t *bands;
    uint8_t *zero;
    unsigned long long *progress;
    uint32_t *counter, *masks, *status;
    uint8_t *pscr;
    unsigned long long *acc;
};

Bufs bufs(const me_batch &b) {
    Bufs r;
    const PaMemo &m = b.plan;
    r.jobs = (const JobDesc *)(b.dev + m.o_jobs);
    r.chains = (const ChainDesc *)(b.dev + m.o_ch);
    r.tickets = (const uint32_t *)(b.dev + m.o_tk);
    r.bands = (const uint32_t *)(b.dev + m.o_bands);
    r.zero = b.dev + b.o_zero;
    r.progress = (unsigned long long *)r.zero;
    r.counter = (uint32_t *)(r.zero + align_up((size_t)m.nlines * 8, 256));
    r.masks = (uint32_t *)((uint8_t *)r.counter + 256);
    r.pscr = b.dev + b.o_pscr;
    r.acc = (unsigned long long *)(b.dev + b.o_acc);
    r.status = (uint32_t *)(b.dev + b.o_status);
    return r;
}

KParams batch_kparams(const me_batch &b, int sleep) {
    KParams kp = kparams(&b.params, b.shape);
    kp.poll_sleep = sleep;
    return kp;
}

// Words of the search scratch that start at zero: row workers need only the
// row progress counts and the ticket counter.
size_t zero_words(const me_batch &b, const int32_t *cfg) { return (cfg[5] ? b.rows_zero_bytes : b.zero_bytes) / 4; }

// The search; `fill`: clear its scratch first (else the caller has).
hipError_t launch_search(const me_batch &b, const Bufs &u, const int32_t *cfg, hipStream_t s,
                         const KernelTimer *t = nullptr, bool fill = true) {
    if (fill) {
        hipError_t e = launch_fill_u32((uint32_t *)u.zero, zero_words(b, cfg), 0u, s);
        if (e != hipSuccess) return e;
    }
    if (cfg[5])
        return launch_pa_rows(u.jobs, u.chains, u.bands, b.plan.nbands, u.progress, u.counter, u.status,
                              batch_kparams(b, cfg[2]), cfg[0], s, t, cfg[1] == 0);
    return launch_pa(u.jobs, b.n, b.plan.total_mbs, u.chains, u.tickets, b.plan.nlines, u.progress, u.counter, u.masks,
                     b.plan.mask_words, u.pscr, u.status, batch_kparams(b, cfg[2]), cfg[0], s, t,
                     cfg[1] == 0, cfg[4]);
}

// Classification, which also clears the search scratch and the per-job
// sums; MC + SSE adds into those sums.
hipError_t launch_classify_step(const me_batch &b, const Bufs &u, const int32_t *cfg, hipStream_t s,
                                const KernelTimer *t, int per_cu) {
    return launch_classify_zeroing(u.jobs, b.n, b.plan.total_mbs, (uint32_t *)u.zero, zero_words(b, cfg),
                                   (uint32_t *)u.acc, (size_t)b.n * 4, s, t, per_cu);
}

// The whole frame step with configuration `cfg` on stream `s`; `tm` (or
// null): event pairs per timing kind, used for the kinds set in `timed`.
hipError_t launch_step(const me_batch &b, const int32_t *cfg, hipStream_t s, const KernelTimer *tm = nullptr,
                       uint32_t timed = 0) {
    auto T = [&](int kind) -> const KernelTimer * { return tm && ((timed >> kind) & 1u) ? &tm[kind] : nullptr; };
    const Bufs u = bufs(b);
    hipError_t e = launch_classify_step(b, u, cfg, s, T(ME_KT_CLASSIFY), cfg[3]);
    if (e != hipSuccess) return e;
    if (b.net) {
        e = net_forward_table(b.net, u.jobs, b.n, b.plan.total_mbs, b.net_scratch, s, T(ME_KT_NET));
        if (e != hipSuccess) return e;
    }
    e = launch_search(b, u, cfg, s, T(ME_KT_SEARCH), false);
    if (e != hipSuccess) return e;
    return launch_mc_sums_acc(u.jobs, b.n, b.plan.total_mbs, u.acc, u.status, s, T(ME_KT_MC), cfg[3]);
}

// Read and clear the device status word (blocking); true when it was clear.
bool status_clear(const me_batch &b, const Bufs &u, bool *ok) {
    uint32_t st = 0;
    if (hipMemcpyAsync(&st, u.status, 4, hipMemcpyDeviceToHost, b.stream) != hipSuccess) return false;
    if (hipStreamSynchronize(b.stream) != hipSuccess) return false;
    *ok = st == 0;
    if (st && (launch_fill_u32(u.status, 64, 0u, b.stream) != hipSuccess || hipStreamSynchronize(b.stream) != hipSuccess))
        return false;
    return true;
}

// Fastest of three timed runs of `fn` on the batch's stream (ms), or -1.
template <class F>
float time_min(const me_batch &b, hipEvent_t e0, hipEvent_t e1, F fn) {
    float best = -1.f;
    for (int r = 0; r < 3; ++r) {
        if (hipEventRecord(e0, b.stream) != hipSuccess) return -1.f;
        if (fn() != hipSuccess) return -1.f;
        if (hipEventRecord(e1, b.stream) != hipSuccess) return -1.f;
        if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
        if (best < 0.f || ms < best) best = ms;
    }
    return best;
}

// Pick the launch configuration by timing the candidates on the creating
// job set (its outputs are written; every configuration computes the same
// results).
int autotune(me_batch &b) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return ME_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ME_EHIP;
    }
    const Bufs u = bufs(b);
    int rc = ME_OK;
    int32_t best[6] = {b.cfg[0], b.cfg[1], b.cfg[2], b.cfg[3], b.cfg[4], b.cfg[5]};
    if (launch_classify(u.jobs, b.n, b.plan.total_mbs, b.stream, nullptr, best[3]) != hipSuccess) rc = ME_EHIP;
    std::vector<int> staging = {0};
    if (plan_elems(b.params.search_range) > 0) staging.insert(staging.begin(), 1);
    float best_ms = -1.f;
    // row workers (job sets without chains in the call): workgroups cap, cap/2
    if (b.plan.unchained && !(b.params.flags & ME_FLAG_LINE_WORKERS)) {
        const int cap = std::min(b.plan.nbands, pa_rows_cap(b.params.search_range, b.params.half_pel != 0));
        std::vector<int> workers = {cap};
        if (cap / 2 >= 64) workers.push_back(cap / 2);
        for (int w : workers)
            for (int st : staging)
                for (int sl : {1, 2}) {
                    if (rc) break;
                    const int32_t c[6] = {w, st, sl, best[3], kRowWaves, 1};
                    float ms = time_min(b, e0, e1, [&] { return launch_search(b, u, c, b.stream); });
                    bool clean = false;
                    if (ms < 0.f || !status_clear(b, u, &clean)) {
                        rc = ME_EHIP;
                        break;
                    }
                    if (!clean) continue;
                    if (best_ms < 0.f || ms < best_ms) {
                        best_ms = ms;
                        for (int i = 0; i < 6; ++i) best[i] = c[i];
                    }
                }
    }
    for (int wavesn : {1, 2, 4}) {
        if (wavesn > 1 && one_wave_lines(b.params.flags)) break;  // the one-wave worker only
        // workgroups of `wavesn` waves; the same wave budget
        const int cap = std::min(b.plan.nlines, pa_worker_cap() / wavesn);
        std::vector<int> workers = {cap};
        for (int w : {cap / 2, cap / 4})
            if (w >= 64 && w != workers.back()) workers.push_back(w);
        for (int w : workers)
            for (int st : staging)
                for (int sl : {1, 2, 4}) {
                    if (rc) break;
                    if (wavesn > 1 && sl != 1) continue;  // the several-wave worker polls with a fixed back-off
                    const int32_t c[6] = {w, st, sl, best[3], wavesn, 0};
                    float ms = time_min(b, e0, e1, [&] { return launch_search(b, u, c, b.stream); });
                    bool clean = false;
                    if (ms < 0.f || !status_clear(b, u, &clean)) {
                        rc = ME_EHIP;
                        break;
                    }
                    // a candidate that raised the status word (a dependency wait
                    // ran out) is dropped: its workers left early, so its time
                    // says nothing
                    if (!clean) continue;
                    if (best_ms < 0.f || ms < best_ms) {
                        best_ms = ms;
                        for (int i = 0; i < 6; ++i) best[i] = c[i];
                    }
                }
    }
    if (rc == ME_OK && best_ms < 0.f) rc = ME_EDEVICE;  // no search configuration ran cleanly
    best_ms = -1.f;
    for (int pc : {4, 8, 16}) {
        if (rc) break;
        float ms = time_min(b, e0, e1, [&] {
            hipError_t e = launch_classify_step(b, u, best, b.stream, nullptr, pc);
            if (e != hipSuccess) return e;
            return launch_mc_sums_acc(u.jobs, b.n, b.plan.total_mbs, u.acc, u.status, b.stream, nullptr, pc);
        });
        bool clean = false;
        if (ms < 0.f || !status_clear(b, u, &clean)) {
            rc = ME_EHIP;
            break;
        }
        if (!clean) {
            rc = ME_EDEVICE;
            break;
        }
        if (best_ms < 0.f || ms < best_ms) {
            best_ms = ms;
            best[3] = pc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == ME_OK)
        for (int i = 0; i < 6; ++i) b.cfg[i] = best[i];
    return rc;
}

void drop_graphs(me_batch &b) {
    for (int i = 0; i < 2; ++i) {
        if (b.exec[i]) (void)hipGraphExecDestroy(b.exec[i]);
        if (b.graph[i]) (void)hipGraphDestroy(b.graph[i]);
        b.exec[i] = nullptr;
        b.graph[i] = nullptr;
    }
    b.pending[0] = b.pending[1] = false;
}

// Capture state: the event set whose records become event nodes, and the
// kinds whose stop node was added.
struct CaptureCtx {
    me_batch *b;
    int set;
    hipError_t err;
    uint32_t stopped;
};

// A timed kernel's start or stop, added as an event-record node of the
// graph being captured after the stream's current capture dependencies,
// which it then replaces.
void record_node(void *ctx, int kind, bool start, hipStream_t s) {
    CaptureCtx &c = *(CaptureCtx *)ctx;
    if (c.err != hipSuccess) return;
    const KernelTimer &t = c.b->tm[c.set][kind];
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t ndeps = 0;
    c.err = hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &ndeps);
    if (c.err == hipSuccess && (st != hipStreamCaptureStatusActive || !g)) c.err = hipErrorStreamCaptureInvalidated;
    if (c.err != hipSuccess) return;
    hipGraphNode_t node = nullptr;
    c.err = hipGraphAddEventRecordNode(&node, g, deps, ndeps, start ? t.start : t.stop);
    if (c.err == hipSuccess) c.err = hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
    if (c.err == hipSuccess && !start) c.stopped |= 1u << kind;
}

// Sum the event pairs of event set i's last replay (waits for it).
void harvest(me_batch &b, int i) {
    if (!b.pending[i]) return;
    b.pending[i] = false;
    for (int k = 0; k < kBatchKinds; ++k) {
        if (!((b.timed >> k) & 1u)) continue;
        float ms = 0.f;
        if (hipEventSynchronize(b.tm[i][k].stop) == hipSuccess &&
            hipEventElapsedTime(&ms, b.tm[i][k].start, b.tm[i][k].stop) == hipSuccess) {
            b.t_ms[k] += ms;
            b.t_count[k]++;
        }
    }
}

// Capture the two graphs of the frame step (kernel timing as now in
// force).  Waits for the stream first (earlier replays' events are
// harvested).
int capture(me_batch &b) {
    if (hipStreamSynchronize(b.stream) != hipSuccess) return ME_EHIP;
    for (int i = 0; i < 2; ++i) harvest(b, i);
    drop_graphs(b);
    b.timed = 0;
    for (int k = 0; k < kBatchKinds; ++k)
        if (k != ME_KT_FULL && timing_enabled(k) && (k != ME_KT_NET || b.net)) b.timed |= 1u << k;
    for (int i = 0; i < (b.timed ? 2 : 0); ++i)
        for (int k = 0; k < kBatchKinds; ++k) {
            if (!((b.timed >> k) & 1u) || b.tm[i][k].start) continue;
            if (hipEventCreate(&b.tm[i][k].start) != hipSuccess || hipEventCreate(&b.tm[i][k].stop) != hipSuccess)
                return ME_EHIP;
        }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return ME_EHIP;
    const size_t table = sizeof(JobDesc) * (size_t)b.n;
    int rc = ME_OK;
    uint32_t stopped = b.timed;
    for (int i = 0; i < 2 && rc == ME_OK; ++i) {
        CaptureCtx ctx{&b, i, hipSuccess, 0u};
        KernelTimer marks[kBatchKinds];
        for (int k = 0; k < kBatchKinds; ++k) {
            marks[k].split = record_node;
            marks[k].ctx = &ctx;
            marks[k].kind = k;
        }
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
            rc = ME_EHIP;
            break;
        }
        hipError_t e = hipMemcpyAsync(b.dev + b.plan.o_jobs, b.host[i], table, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = launch_step(b, b.cfg, cs, marks, b.timed);
        if (e == hipSuccess) e = ctx.err;
        stopped &= ctx.stopped;
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = ee != hipSuccess ? ee : (g ? hipSuccess : hipErrorUnknown);
        if (e == hipSuccess) {
            b.graph[i] = g;
            e = hipGraphInstantiate(&b.exec[i], g, nullptr, nullptr, 0);
            if (e != hipSuccess) b.exec[i] = nullptr;
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
        if (e != hipSuccess) rc = ME_EHIP;
    }
    (void)hipStreamDestroy(cs);
    // timed kinds are those with event nodes in the graphs (a kind whose
    // kernel was not launched has none)
    b.timed = rc ? 0u : stopped;
    if (rc) drop_graphs(b);
    return rc;
}

// Job table i staged for `jobs`: waits until its previous copy is done.
int stage_table(me_batch &b, const me_job *jobs, int i) {
    if (hipEventSynchronize(b.ev[i]) != hipSuccess) return ME_EHIP;
    fill_table(b, jobs, (JobDesc *)b.host[i]);
    return ME_OK;
}

// The job table for `jobs` copied outside the graphs (staging 0).
int upload_table(me_batch &b, const me_job *jobs) {
    int rc = stage_table(b, jobs, 0);
    if (rc) return rc;
    if (hipMemcpyAsync(b.dev + b.plan.o_jobs, b.host[0], sizeof(JobDesc) * (size_t)b.n, hipMemcpyHostToDevice,
                       b.stream) != hipSuccess)
        return ME_EHIP;
    if (hipEventRecord(b.ev[0], b.stream) != hipSuccess) return ME_EHIP;
    return ME_OK;
}

void release(me_batch *b) {
    if (!b) return;
    if (b->stream || b->dev) (void)hipStreamSynchronize(b->stream);
    drop_graphs(*b);
    for (auto &row : b->tm)
        for (auto &t : row) {
            if (t.start) (void)hipEventDestroy(t.start);
            if (t.stop) (void)hipEventDestroy(t.stop);
        }
    for (int s = 0; s < 2; ++s) {
        if (b->ev[s]) (void)hipEventDestroy(b->ev[s]);
        if (b->host[s]) (void)hipHostFree(b->host[s]);
    }
    if (b->host_acc) (void)hipHostFree(b->host_acc);
    if (b->net_scratch) (void)hipFree(b->net_scratch);
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}

}  // namespace

extern "C" {

int me_batch_create(const me_job *jobs, int n, const me_params *params, uint32_t flags, void *stream,
                    me_batch **out) {
    if (!out) return ME_EINVAL;
    *out = nullptr;
    if (n <= 0 || !jobs || (flags & ~kFlagsKnown)) return ME_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    const bool shape = (flags & ME_BATCH_SHAPE) != 0;
    for (int i = 0; i < n; ++i) {
        rc = check_job(jobs[i], shape);
        if (rc) return rc;
        if (jobs[i].seed && params->k_max > kMaxSeededKmax) return ME_EINVAL;
    }
    me_batch *b = new me_batch();
    b->n = n;
    b->shape = shape;
    b->params = *params;
    b->stream = (hipStream_t)stream;
    rc = build_pa(jobs, n, b->plan);
    if (rc) {
        delete b;
        return rc;
    }
    if (hipGetDevice(&b->device) != hipSuccess || check_device(b->device) != ME_OK) {
        delete b;
        return ME_ENODEV;
    }
    const PaMemo &m = b->plan;
    b->tmpl.resize(n);
    std::memcpy(b->tmpl.data(), m.blob.data() + m.o_jobs, sizeof(JobDesc) * (size_t)n);
    // device layout: [jobs | chains | tickets] [zeroed search scratch] [ticket compaction] [per-job sums]
    // [status]
    b->o_zero = align_up(m.blob.size(), 256);
    b->zero_bytes = align_up(align_up((size_t)m.nlines * 8, 256) + 256 + (size_t)m.nlines * m.mask_words * 2 * 4, 256);
    b->rows_zero_bytes = align_up((size_t)m.nlines * 8, 256) + 256;  // progress words (rows use the first) and counter
    b->o_pscr = b->o_zero + b->zero_bytes;
    b->o_acc = b->o_pscr + align_up(pa_scratch_bytes(m.nlines), 256);
    b->o_status = b->o_acc + align_up((size_t)n * 16, 256);
    const size_t total = b->o_status + 256;
    const size_t table = sizeof(JobDesc) * (size_t)n;
    b->cfg[5] = m.unchained && !(params->flags & ME_FLAG_LINE_WORKERS) ? 1 : 0;
    b->cfg[4] = b->cfg[5] ? kRowWaves : one_wave_lines(params->flags) ? 1 : lines_waves(m.nlines);
    b->cfg[0] = b->cfg[5] ? std::min(m.nbands, pa_rows_cap(params->search_range, params->half_pel != 0))
                          : std::min(m.nlines, pa_worker_cap() / b->cfg[4]);
    b->cfg[1] = plan_elems(params->search_range) > 0 ? 1 : 0;
    b->cfg[2] = b->cfg[4] > 1 && !b->cfg[5] ? 1 : 2;
    b->cfg[3] = 8;
    if (hipMalloc(&b->dev, total) != hipSuccess) {
        b->dev = nullptr;
        release(b);
        return ME_ENOMEM;
    }
    for (int s = 0; s < 2; ++s) {
        if (hipHostMalloc(&b->host[s], table, hipHostMallocDefault) != hipSuccess) {
            b->host[s] = nullptr;
            release(b);
            return ME_ENOMEM;
        }
        if (hipEventCreateWithFlags(&b->ev[s], hipEventDisableTiming) != hipSuccess) {
            b->ev[s] = nullptr;
            release(b);
            return ME_EHIP;
        }
    }
    if (hipHostMalloc((void **)&b->host_acc, (size_t)n * 16, hipHostMallocDefault) != hipSuccess) {
        b->host_acc = nullptr;
        release(b);
        return ME_ENOMEM;
    }
    // static tables once; the status word starts clear
    if (hipMemcpy(b->dev, m.blob.data(), m.blob.size(), hipMemcpyHostToDevice) != hipSuccess ||
        launch_fill_u32((uint32_t *)(b->dev + b->o_status), 64, 0u, b->stream) != hipSuccess) {
        release(b);
        return ME_EHIP;
    }
    if (flags & ME_BATCH_AUTOTUNE) {
        rc = upload_table(*b, jobs);
        if (!rc) rc = autotune(*b);
        if (rc) {
            release(b);
            return rc;
        }
    }
    rc = capture(*b);
    if (rc) {
        release(b);
        return rc;
    }
    *out = b;
    return ME_OK;
}

int me_batch_step(me_batch *b, const me_job *jobs, int n) {
    if (!b) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(b->mu);
    int rc = check_structure(*b, jobs, n);
    if (rc) return rc;
    const int set = (int)(b->replays & 1);
    harvest(*b, set);  // that set's previous replay (the other one may still run)
    rc = stage_table(*b, jobs, set);
    if (rc) return rc;
    if (hipGraphLaunch(b->exec[set], b->stream) != hipSuccess) return ME_EHIP;
    // the next use of table `set` waits for this replay's copy: through the
    // event set's stop events (harvest) when kernels are timed, which come
    // after the copy, else through ev[set]
    if (!b->timed && hipEventRecord(b->ev[set], b->stream) != hipSuccess) return ME_EHIP;
    b->pending[set] = b->timed != 0;
    b->replays++;
    b->stepped = true;
    return ME_OK;
}

int me_batch_results(me_batch *b, uint64_t *sse, uint64_t *npix, double *psnr_db, int n) {
    if (!b || !sse || !npix || !psnr_db || n != b->n) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(b->mu);
    if (!b->stepped) return ME_EINVAL;
    const Bufs u = bufs(*b);
    if (hipMemcpyAsync(b->host_acc, u.acc, (size_t)n * 16, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
        return ME_EHIP;
    uint32_t st = 0;
    if (hipMemcpyAsync(&st, u.status, 4, hipMemcpyDeviceToHost, b->stream) != hipSuccess) return ME_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return ME_EHIP;
    int status = ME_OK;
    for (int p = 0; p < n; ++p) {
        const int i = b->plan.order[p];
        sse[i] = b->host_acc[2 * p];
        npix[i] = b->host_acc[2 * p + 1];
        if (npix[i] == 0) {
            psnr_db[i] = NAN;
            status = ME_EEMPTY;
        } else if (sse[i] == 0) {
            psnr_db[i] = INFINITY;
        } else {
            psnr_db[i] = 10.0 * std::log10(255.0 * 255.0 * (double)npix[i] / (double)sse[i]);
        }
    }
    if (st) {
        if (launch_fill_u32(u.status, 64, 0u, b->stream) != hipSuccess) return ME_EHIP;
        if (hipStreamSynchronize(b->stream) != hipSuccess) return ME_EHIP;
        return ME_EDEVICE;
    }
    return status;
}

int me_batch_set_net(me_batch *b, me_net *net) {
    if (!b) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(b->mu);
    if (net) {
        for (const auto &d : b->tmpl)
            if (!d.seed) return ME_EINVAL;  // the seeds are written into the jobs' seed buffers
        if (b->n > 65535) return ME_EINVAL;
        for (const auto &d : b->tmpl)
            if (d.wm * d.hm > 65536) return ME_EINVAL;
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return ME_EHIP;
    if (net && !b->net_scratch &&
        hipMalloc(&b->net_scratch, align_up(net_table_scratch(b->plan.total_mbs), 256)) != hipSuccess) {
        b->net_scratch = nullptr;
        return ME_ENOMEM;
    }
    b->net = net;
    return capture(*b);
}

int me_batch_config(const me_batch *b, int32_t *cfg, int ncfg) {
    if (!b || !cfg || ncfg < 4) return ME_EINVAL;
    for (int i = 0; i < std::min(ncfg, 6); ++i) cfg[i] = b->cfg[i];
    return ME_OK;
}

int me_batch_set_config(me_batch *b, const int32_t *cfg, int ncfg) {
    if (!b || !cfg || (ncfg != 5 && ncfg != 6)) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(b->mu);
    const int rows = ncfg == 6 ? cfg[5] : 0;
    if (rows != 0 && rows != 1) return ME_EINVAL;
    const int waves = cfg[4];
    if (rows) {
        // row workers: job sets without chains in the call; persistent
        // workgroups of kRowWaves rows, up to the resident count
        if (!b->plan.unchained || waves != kRowWaves) return ME_EINVAL;
        if (cfg[0] < 1 || cfg[0] > std::min(b->plan.nbands, pa_rows_cap(b->params.search_range, b->params.half_pel != 0))) return ME_EINVAL;
    } else {
        if (waves != 1 && waves != 2 && waves != 4) return ME_EINVAL;
        if (waves > 1 && one_wave_lines(b->params.flags)) return ME_EINVAL;
        // persistent workers: any count up to one per line (and the wave budget)
        if (cfg[0] < 1 || cfg[0] > std::min(b->plan.nlines, pa_worker_cap() / waves)) return ME_EINVAL;
    }
    if (cfg[1] != 0 && cfg[1] != 1) return ME_EINVAL;
    if (cfg[1] == 1 && plan_elems(b->params.search_range) <= 0) return ME_EINVAL;
    if (cfg[2] != 1 && cfg[2] != 2 && cfg[2] != 4) return ME_EINVAL;
    if (cfg[3] != 4 && cfg[3] != 8 && cfg[3] != 16) return ME_EINVAL;
    for (int i = 0; i < 5; ++i) b->cfg[i] = cfg[i];
    b->cfg[5] = rows;
    return capture(*b);
}

int me_batch_kernel_time_ms(me_batch *b, int kind, double *total_ms, int *count) {
    if (!b || !total_ms || !count || kind < 0 || kind >= kBatchKinds) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(b->mu);
    for (int i = 0; i < 2; ++i) harvest(*b, i);
    *total_ms = b->t_ms[kind];
    *count = b->t_count[kind];
    b->t_ms[kind] = 0.0;
    b->t_count[kind] = 0;
    return ME_OK;
}

void me_batch_destroy(me_batch *b) { release(b); }

}  // extern "C"

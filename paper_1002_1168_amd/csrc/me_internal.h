// Internal declarations of the gfx950 motion-estimation library: device-side
// job descriptors, launch entry points and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/me.h"

namespace me {

// ---------------------------------------------------------------- layout
// Device view of one frame pair (one me_job) or one frame (classification).
struct JobDesc {
    const uint8_t *cur, *ref, *cur_a, *ref_a;
    const uint8_t *cls;   // MB classes (written by the classification kernel)
    const int16_t *tf, *seed;
    int16_t *mv, *mv_int;
    uint32_t *cost;
    uint8_t *iters;
    uint16_t *points;
    uint8_t *out_u8;      // MC: prediction out (nullable)
    uint32_t *out_u32;    // classification: BAB words out (nullable)
    int32_t width, height, stride, wm, hm;
    int32_t mb_base;        // first flat MB index of this job in multi-job grids
    int32_t dep_line_base;  // PA: progress lines of the chain producing T (-1: none)
    int32_t dep_pos;        // PA: position of the producing job in that chain
    int32_t t_local;        // PA: T is the previous position of this job's own chain
    int32_t chain_line_base;  // PA: first progress line of this job's chain
    int32_t chain_pos;        // PA: position of this job in its chain
    int32_t pad;
};
static_assert(sizeof(JobDesc) == 160, "JobDesc is read as 40 dwords");

// A pipelined chain of frame pairs (each one's T field is the previous one's
// mv_int).  One progress line per MB position.
struct ChainDesc {
    int32_t first;      // index of the chain's first pair in the chain-ordered job array
    int32_t len;
    int32_t wm, hm;
    int32_t line_base;  // first progress counter of this chain
    int32_t pad[3];
};

struct KParams {
    int32_t S, theta, eps, max_step, k_max, half_pel, shape_only, spin_limit;
    int32_t poll_sleep;  // s_sleep units between dependency polls (0, 1, 2 or 4)
    int32_t zero_t;      // |trunc(S / n)| < zero_t <=> zero step (eps > 0: ceil(2^23 / eps); eps = 0: INT_MAX)
    int32_t unrestricted;  // 1: vectors limited by S only, the reference extended by its edge pixels
    int32_t t_texture;     // 1: a boundary MB's T scored on texture (Section 3.1 text)
    int32_t masked_prs;    // 1: a boundary MB's recursion refines on luma over the VOP pixels
};

// device status word bits
enum : uint32_t { ST_SPIN_TIMEOUT = 1u, ST_BAD_CLASS = 2u, ST_ABORT = 4u };

// ------------------------------------------------------------- launches
// Optional event pair recorded around the main kernel of a launch
// (profiling).  With `split` set the launch is being captured into a graph:
// events recorded during capture add no graph node, so the mark calls
// split(ctx, kind, start, s) instead, and the graph's owner adds the event
// record to the graph itself.
struct KernelTimer {
    hipEvent_t start = nullptr, stop = nullptr;
    void (*split)(void *ctx, int kind, bool start, hipStream_t s) = nullptr;
    void *ctx = nullptr;
    int kind = 0;
};
inline void timer_mark(const KernelTimer *t, bool start, hipStream_t s) {
    if (!t) return;
    if (t->split)
        t->split(t->ctx, t->kind, start, s);
    else
        (void)hipEventRecord(start ? t->start : t->stop, s);
}

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_classify(const JobDesc *jobs, int n, int total_mbs, hipStream_t s, const KernelTimer *t = nullptr,
                           int per_cu = 8);
int flat_chunk(int total_mbs, int per_cu);
hipError_t launch_pa(const JobDesc *jobs, int njobs, int total_mbs, const ChainDesc *chains, const uint32_t *tickets,
                     int nlines, unsigned long long *progress, uint32_t *counter, uint32_t *masks, int mask_words,
                     uint8_t *scratch, uint32_t *status, const KParams &kp, int workers, hipStream_t s,
                     const KernelTimer *t = nullptr, bool generic = false, int waves = 1);
// bytes of the `scratch` argument of launch_pa (256-aligned base; no zeroing needed)
size_t pa_scratch_bytes(int nlines);
// LDS bytes of one search worker; `generic`: single-buffered generic staging
size_t pa_lds_bytes(int S, bool generic = false);
int plan_elems(int S);
hipError_t launch_full_search(int method, const JobDesc *jobs, int n, int total_mbs, const KParams &kp,
                              uint32_t *counters, uint32_t *list, uint32_t *status, hipStream_t s,
                              const KernelTimer *t = nullptr);
size_t full_search_scratch(int total_mbs);
// `four`: each job's mv holds four vectors per MB (8 x 8 blocks in raster order).
// `sums_only`: no job writes a prediction frame; transparent MBs (by class)
// are then skipped - exact when the classes are those of the current alpha.
hipError_t launch_mc(const JobDesc *jobs, int n, int total_mbs, uint32_t *part, unsigned long long *acc,
                     uint32_t *status, hipStream_t s, const KernelTimer *t = nullptr, int per_cu = 8,
                     bool four = false, bool sums_only = false);
// Pel-recursive refinement of the 8 x 8 blocks of every texture MB: reads
// cur, ref, cls, mv_int (start vectors) and tf (the MB's half-pel vector,
// repeated for boundary MBs); writes four vectors per MB to mv, and per
// block cost (nullable), iters (nullable), points (nullable).
hipError_t launch_prs8(const JobDesc *jobs, int n, int total_mbs, const KParams &kp, hipStream_t s,
                       const KernelTimer *t = nullptr);
size_t mc_scratch(int total_mbs);

// Row workers (job sets without chains inside the call): bands of
// kRowWaves MB rows, one wave per row.  `bands`: chain << 16 | first row, in
// (first row, chain) order; `progress` and `counter` zeroed.
constexpr int kRowWaves = 4;
hipError_t launch_pa_rows(const JobDesc *jobs, const ChainDesc *chains, const uint32_t *bands, int nbands,
                          unsigned long long *progress, uint32_t *counter, uint32_t *status, const KParams &kp,
                          int workers, hipStream_t s, const KernelTimer *t = nullptr, bool generic = false);
// resident row-worker workgroups the device holds for range S (with half-sample
// refinement on, the workers keep two windows each when they fit)
int pa_rows_cap(int S, bool half_pel);

int pa_worker_cap();
// Waves per line worker for `nlines` lines: 4 while every line still gets
// a worker (each wave then has four pairs' time for its own pair), 2 while
// that holds at two, else 1 (more lines than workers: one wave per line)
inline int lines_waves(int nlines) {
    return nlines <= pa_worker_cap() / 4 ? 4 : nlines <= pa_worker_cap() / 2 ? 2 : 1;
}
// exclusive scan of n counts in place (one block), total to *total
hipError_t launch_scan_counts(uint32_t *counts, int n, uint32_t *total, hipStream_t s);

// ------------------------------------------------ learned proposal network
// parameter vector: W1 (32,3,3,2) | b1 (32) | W2 (32,3,3,32) | b2 (32) | W3 (2,3,3,32) | b3 (2)
constexpr int kNetOW1 = 0, kNetOB1 = 576, kNetOW2 = 608, kNetOB2 = 9824, kNetOW3 = 9856, kNetOB3 = 10432;
constexpr int kNetParams = 10434;
constexpr int kNetBf16 = 576 + 2 * 9216 + 576;  // bf16 copies: W1 | W2 | W2 as [tap][ci][co] | W3
size_t net_lds_bytes(bool train);
size_t net_list_scratch(int total_mbs);
// list of opaque MBs (all MBs of jobs without classes) in flat order, into `scratch`
hipError_t launch_net_list(const JobDesc *jobs, int n, int total_mbs, uint8_t *scratch, const uint32_t **list,
                           const uint32_t **count, hipStream_t s);
// forward (seeds / predictions) or forward + backward into per-workgroup partials
hipError_t launch_net(bool train, const JobDesc *jobs, int n, const uint32_t *list, const uint32_t *count,
                      const float *P, const uint16_t *wb, float *part, int groups, int scale, hipStream_t s,
                      const KernelTimer *t = nullptr);
// sum of the partials into grad / loss (nullable); `apply`: momentum SGD too
hipError_t launch_net_sgd(float *P, float *V, uint16_t *wb, const float *part, int nparts, float lr, float mu,
                          float *grad, double *loss, hipStream_t s, bool apply = true);
// momentum SGD from the gradient g (device)
hipError_t launch_net_apply(float *P, float *V, uint16_t *wb, const float *g, float lr, float mu, hipStream_t s);
hipError_t launch_net_refresh(const float *P, uint16_t *wb, hipStream_t s);

}  // namespace me

// ----------------------------------------------------------- device helpers
#if defined(__HIPCC__)
namespace me {

__device__ __forceinline__ int lane() { return __lane_id(); }

// Unaligned 4-byte load from global memory (gfx950 serves unaligned dword
// accesses).  The explicit global address space makes it a global_load, not a
// flat_load, so independent loads can be in flight together.
typedef uint32_t __attribute__((aligned(1))) u32_unaligned;
__device__ __forceinline__ uint32_t ld4(const uint8_t *p) {
    return *(const __attribute__((address_space(1))) u32_unaligned *)(p);
}

// 4 frame bytes of `row` starting at column xx, edge replicated: an
// in-frame dword at the clamped column, then a byte permute (branch-free, so
// independent loads stay in flight together).
__device__ __forceinline__ uint32_t ld4_clamped(const uint8_t *row, int xx, int W);

__device__ __forceinline__ uint32_t ldg32(const uint32_t *p) {
    return *(const __attribute__((address_space(1))) uint32_t *)(p);
}

__device__ __forceinline__ uint32_t ldg8(const uint8_t *p) {
    return *(const __attribute__((address_space(1))) uint8_t *)(p);
}

// Per byte: 0xFF where the byte is non-zero, else 0 (binary alpha -> 0/255 plane).
__device__ __forceinline__ uint32_t bin4(uint32_t x) {
    uint32_t m = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    return (m >> 7) * 0xFFu;
}

__device__ __forceinline__ int byte_of(uint32_t w, int k) { return (int)((w >> (8 * k)) & 0xFFu); }

// Sum over the 64 lanes with DPP row operations, broadcast to every lane.
__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false); // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false); // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) { return (uint32_t)wave_sum((int)v); }

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uni64(unsigned long long v) {
    return (unsigned long long)(uint32_t)uni((int)(uint32_t)v) |
           ((unsigned long long)(uint32_t)uni((int)(uint32_t)(v >> 32)) << 32);
}

#define DWI(f) ((int)(offsetof(JobDesc, f) / 4))

// Wave-uniform job cursor of the flat-MB kernels: the job index, its flat MB
// range [base, end), and its descriptor one dword per lane (lane l holds
// dword l of the 40), read out with readlane.
struct JobCursor {
    int j, base, end;
    uint32_t d;
    __device__ __forceinline__ int i32(int i) const { return __builtin_amdgcn_readlane((int)d, i); }
    template <class T>
    __device__ __forceinline__ T *ptr(int i) const {
        return (T *)(uintptr_t)((unsigned long long)(uint32_t)i32(i) | ((unsigned long long)(uint32_t)i32(i + 1) << 32));
    }
};

// Last job in [lo, n) whose mb_base <= idx, given jobs[lo].mb_base <= idx
// (mb_base is the running sum of the jobs' MB counts).  Each round every
// lane reads one candidate's mb_base and a ballot narrows the range 64-fold:
// one round for up to 64 jobs, two for up to 4096.
__device__ __forceinline__ int seek_job(const JobDesc *jobs, int lo, int n, int idx) {
    int hi = n - 1;
    while (lo < hi) {
        const int step = (hi - lo + 64) >> 6;
        const int c = lo + lane() * step;
        const bool ok = c <= hi && *(const __attribute__((address_space(1))) int32_t *)&jobs[c].mb_base <= idx;
        const unsigned long long b = __ballot(ok);
        lo += (63 - __builtin_clzll(b)) * step;
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

// Move the cursor to the job of flat MB idx (idx never decreases).
__device__ __forceinline__ void seek(JobCursor &c, const JobDesc *jobs, int n, int idx) {
    if (idx < c.end) return;
    c.j = seek_job(jobs, c.j + 1, n, idx);
    c.d = ldg32((const uint32_t *)(jobs + c.j) + min(lane(), 39));
    c.base = c.i32(DWI(mb_base));
    c.end = c.base + c.i32(DWI(wm)) * c.i32(DWI(hm));
}

// One flat MB per lane, the wave's 64 consecutive MBs [base, last]: calls
// f(c, k) in the lanes whose MB belongs to the cursor's job c (k = its index
// within the job), once per job the range touches.  f runs in a subset of
// the lanes: no wave-level operations inside it.
template <class F>
__device__ __forceinline__ void for_lane_mbs(const JobDesc *jobs, int n, int base, int last, F &&f) {
    const int mb = base + lane();
    JobCursor c{-1, 0, 0, 0u};
    seek(c, jobs, n, base);
    for (;;) {
        if (mb <= last && mb >= c.base && mb < c.end) f(c, mb - c.base);
        if (last < c.end) break;
        seek(c, jobs, n, c.end);
    }
}

__device__ __forceinline__ int iclamp(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

__device__ __forceinline__ uint32_t ld4_clamped(const uint8_t *row, int xx, int W) {
    const int xc = iclamp(xx, 0, W - 4);
    const uint32_t sel = (uint32_t)(iclamp(xx, 0, W - 1) - xc) | ((uint32_t)(iclamp(xx + 1, 0, W - 1) - xc) << 8) |
                         ((uint32_t)(iclamp(xx + 2, 0, W - 1) - xc) << 16) |
                         ((uint32_t)(iclamp(xx + 3, 0, W - 1) - xc) << 24);
    const uint32_t v = ld4(row + xc);
    return __builtin_amdgcn_perm(v, v, sel);
}

// Eq. 3 per-axis step: eps * U (Q.24) rounded half away from zero, clamped.
__device__ __forceinline__ int prs_step(int u, int eps, int max_step) {
    long long vq = (long long)eps * (long long)u;
    long long a = vq < 0 ? -vq : vq;
    long long s = (a + (1ll << 23)) >> 24;
    int r = (int)(s > max_step ? max_step : s);
    return vq < 0 ? -r : r;
}

}  // namespace me
#endif

// Baseline block matching (Section 1 references [5], [6], [7]; Tables 1-2):
// exhaustive search (ES), three-step search (TSS), four-step search (4SS) and
// diamond search (DS) on the luma of every non-transparent MB.  No inter-MB
// dependency: flat grids.
#include <algorithm>

#include "me_internal.h"

namespace me {

namespace {

constexpr int kEsThreads = 256;

// A thread task of ES is one column offset dx and G consecutive row offsets
// dy (register blocking: every reference row read feeds up to G candidate
// SADs).  G is picked per range so that the (2S+1) x ceil((2S+1)/G) tasks
// fill the 256 threads with the fewest SAD instructions per thread: rounds
// of 256 tasks times G, ties to the larger G (fewer LDS reads per SAD).
__host__ __device__ constexpr int es_group(int S) {
    const int ncol = 2 * S + 1;
    int best = 4, cost = 1 << 30;
    for (int G = 4; G <= 8; ++G) {
        if (G == 7) continue;  // not instantiated
        const int tasks = ncol * ((ncol + G - 1) / G);
        const int c = ((tasks + kEsThreads - 1) / kEsThreads) * G;
        if (c <= cost) {
            cost = c;
            best = G;
        }
    }
    return best;
}

// ES window geometry: 16 + 2S columns; rows 16 + 2S plus padding up to the
// last row any task reads (ceil((2S+1)/G) G + 15), so the unrolled row loop
// needs no bounds test (padding rows are never part of a kept candidate);
// row pitch a power of two (>= (16+2S+3)/4 dwords) so staging needs no
// divisions, and each of the four byte-shifted copies padded to 8 mod 32
// dwords so that the four copies of a dword fall on four different LDS banks.
__host__ __device__ constexpr int es_pitch_log2(int S) {
    const int need = (16 + 2 * S + 3) >> 2;
    int lg = 0;
    while ((1 << lg) < need) ++lg;
    return lg;
}
__host__ __device__ constexpr int es_rows(int S) {
    const int ncol = 2 * S + 1, G = es_group(S);
    const int reach = ((ncol + G - 1) / G) * G + 15;
    return 16 + 2 * S > reach ? 16 + 2 * S : reach;
}
__host__ __device__ constexpr int es_copy_dwords(int S) {
    const int raw = es_rows(S) << es_pitch_log2(S);
    return raw + ((8 - raw % 32) + 32) % 32;
}

// The ranges with a kernel of their own (geometry fixed at compile time).
constexpr bool es_fixed(int S) { return S == 7 || S == 16 || S == 32; }
// Dwords of one window buffer: four copies and the 64-dword current block.
constexpr int es_buffer_dwords(int S) { return 4 * es_copy_dwords(S) + 64; }
// Two window buffers (one barrier per MB) where both fit in 32 KB.
constexpr bool es_double(int S) { return 2 * 4 * es_buffer_dwords(S) <= 32768; }

__device__ __forceinline__ void write_result(const JobDesc &J, int k, int dx, int dy, uint32_t cost, int pts) {
    uint32_t w = (uint32_t)(uint16_t)(2 * dx) | ((uint32_t)(uint16_t)(2 * dy) << 16);
    ((uint32_t *)J.mv)[k] = w;
    ((uint32_t *)J.mv_int)[k] = w;
    if (J.cost) J.cost[k] = cost;
    if (J.iters) J.iters[k] = 0;
    if (J.points) J.points[k] = (uint16_t)pts;
}

// ES.  One workgroup per MB.  The (16+2S)^2 reference window is staged in LDS
// as four byte-shifted copies so that a 16-byte row segment at any column is
// four aligned dword reads.  A thread owns one column offset dx and G
// consecutive dy (es_group): every reference row it reads feeds up to G
// candidate SADs (v_sad_u8 on packed bytes), with the current block held in
// registers.  Key = (SAD, |dx|+|dy|, dy, dx) lexicographic, packed into 64 bits.
// Compaction: one lane per MB.  Transparent MBs get their (zero) result at
// once; the others are appended to `list` as (job << 16 | MB index).  A class
// byte above 2 raises ST_BAD_CLASS and the MB is treated as transparent (as
// the search pre-pass does).
__global__ __launch_bounds__(256) void compact_kernel(const JobDesc *jobs, int n, int total, uint32_t *list,
                                                     uint32_t *count, uint32_t *status) {
    const int l = lane();
    const int base = ((int)blockIdx.x * 4 + uni((int)threadIdx.x >> 6)) * 64;
    if (base >= total) return;
    bool searched = false;
    int k = 0, ji = 0;
    for_lane_mbs(jobs, n, base, min(base + 64, total) - 1, [&](const JobCursor &c, int kk) {
        k = kk;
        ji = c.j;
        const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
        const int cl = cls ? (int)ldg8(cls + k) : ME_MB_OPAQUE;
        if (cl > ME_MB_BOUNDARY) atomicOr(status, ST_BAD_CLASS);
        searched = cl == ME_MB_OPAQUE || cl == ME_MB_BOUNDARY;
        if (!searched) write_result(jobs[c.j], k, 0, 0, 0u, 0);
    });
    const unsigned long long ball = __ballot(searched);
    const int cnt = __popcll(ball);
    uint32_t slot = 0;
    if (l == 0 && cnt) slot = atomicAdd(count, (uint32_t)cnt);
    slot = (uint32_t)__shfl((int)slot, 0, 64);
    if (searched) {
        const int before = __popcll(ball & ((1ull << l) - 1ull));
        list[slot + before] = ((uint32_t)ji << 16) | (uint32_t)k;
    }
}

// Ranges without a kernel of their own: S is a kernel argument, the window
// is loaded when the MB starts, 64-bit keys.
template <int G>
__global__ __launch_bounds__(kEsThreads) void es_kernel(const JobDesc *jobs, const uint32_t *list,
                                                       const uint32_t *count, KParams kp) {
    extern __shared__ uint32_t lds[];
    const int tid = threadIdx.x;
    const int S = kp.S;
    const int nitems = (int)*count;
    const int span = 16 + 2 * S;      // window rows and columns
    const int lgp = es_pitch_log2(S);
    const int pd = 1 << lgp;          // dwords per row per copy
    const int csz = es_copy_dwords(S);
    const int per = span << lgp;
    // every searched MB costs the same: static striding, no shared counter
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    __syncthreads();  // the previous MB's readers are done with the window
    const uint32_t e = list[it];
    const JobDesc &J = jobs[e >> 16];
    const int k = (int)(e & 0xFFFF);
    const int h = k % J.wm, v = k / J.wm;
    const int x0 = 16 * h, y0 = 16 * v, W = J.width, H = J.height, st = J.stride;
    uint32_t *win = lds;              // 4 copies
    uint32_t *curb = lds + 4 * csz;   // 64 dwords
    unsigned long long *red = (unsigned long long *)(curb + 64);  // 4 wave minima
    // copy 0 (rows and columns clamped, edge dwords permuted: the frame
    // extended by its edge pixels, which unrestricted vectors read), eight
    // loads in flight per thread; copy s dword w = window bytes 4w+s ..
    // 4w+s+3 is then built from copy 0 in LDS
    const int wx0 = x0 - S, wy0 = y0 - S;
    for (int base = 0; base < per; base += 8 * kEsThreads) {
        uint32_t v8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = min(base + u * kEsThreads + tid, per - 1);
            const int r = idx >> lgp, w = idx & (pd - 1);
            v8[u] = ld4_clamped(J.ref + (size_t)iclamp(wy0 + r, 0, H - 1) * st, wx0 + 4 * w, W);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (base + u * kEsThreads + tid < per) win[base + u * kEsThreads + tid] = v8[u];
    }
    __syncthreads();
    for (int idx = tid; idx < per; idx += kEsThreads) {
        const uint32_t a = win[idx], b = (idx & (pd - 1)) + 1 < pd ? win[idx + 1] : 0u;
        win[csz + idx] = __builtin_amdgcn_alignbyte(b, a, 1);
        win[2 * csz + idx] = __builtin_amdgcn_alignbyte(b, a, 2);
        win[3 * csz + idx] = __builtin_amdgcn_alignbyte(b, a, 3);
    }
    if (tid < 64) curb[tid] = *(const uint32_t *)(J.cur + (size_t)(y0 + (tid >> 2)) * st + x0 + 4 * (tid & 3));
    __syncthreads();
    uint32_t cr[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) cr[i] = curb[i];

    const int lox = kp.unrestricted ? -S : max(-S, -x0), hix = kp.unrestricted ? S : min(S, W - 16 - x0);
    const int loy = kp.unrestricted ? -S : max(-S, -y0), hiy = kp.unrestricted ? S : min(S, H - 16 - y0);
    const int ncol = 2 * S + 1;
    const int ngrp = (ncol + G - 1) / G;
    // key = (SAD, |dx| + |dy|, dy + S, dx + S) in lexicographic order: the
    // first three fields in 32 bits per task (dx is the task's), then dx
    unsigned long long best = ~0ull;
    for (int task = tid; task < ncol * ngrp; task += kEsThreads) {
        const int cxr = task % ncol;           // dx + S
        const int dy0 = (task / ncol) * G;     // first dy + S
        const int dx = cxr - S;
        if (dx < lox || dx > hix) continue;
        const uint32_t *cp = win + (cxr & 3) * csz + (cxr >> 2);
        uint32_t acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0;
#pragma unroll
        for (int r = 0; r < G + 15; ++r) {
            // rows past the window are padding: read, never kept
            const uint32_t *rp = cp + (dy0 + r) * pd;
            const uint32_t r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int jj = r - g;
                if (jj >= 0 && jj < 16) {
                    uint32_t a = acc[g];
                    a = __builtin_amdgcn_sad_u8(cr[4 * jj + 0], r0, a);
                    a = __builtin_amdgcn_sad_u8(cr[4 * jj + 1], r1, a);
                    a = __builtin_amdgcn_sad_u8(cr[4 * jj + 2], r2, a);
                    a = __builtin_amdgcn_sad_u8(cr[4 * jj + 3], r3, a);
                    acc[g] = a;
                }
            }
        }
        const int adx = abs(dx);
        uint32_t kb = ~0u;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int dys = dy0 + g, dy = dys - S;
            const uint32_t key = (acc[g] << 16) | ((uint32_t)(adx + abs(dy)) << 8) | (uint32_t)dys;
            kb = (dys < ncol && dy >= loy && dy <= hiy && key < kb) ? key : kb;
        }
        const unsigned long long k64 = ((unsigned long long)kb << 8) | (unsigned long long)cxr;
        best = kb != ~0u && k64 < best ? k64 : best;
    }
    best = wave_min_u64(best);
    if (lane() == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        unsigned long long b = red[0];
        for (int w = 1; w < kEsThreads / 64; ++w) b = red[w] < b ? red[w] : b;
        const int dx = (int)(b & 0xFF) - S, dy = (int)((b >> 8) & 0xFF) - S;
        const int pts = (hix - lox + 1) * (hiy - loy + 1);
        write_result(J, k, dx, dy, (uint32_t)(b >> 24), pts);
    }
    }
}

// Minimum over the 64 lanes with DPP row operations; lane 63 holds it.
__device__ __forceinline__ uint32_t wave_min_to_last(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return v;
}

// ES for S = 7, 16 and 32: the same tasks as es_kernel with the window
// geometry fixed at compile time (row offsets become instruction offsets).
// - Copy 0 of the next MB's window is loaded into registers during the
//   current MB's search: plain loads when the window lies inside the frame,
//   edge-clamped ones otherwise.  The four byte-shifted copies are built from
//   the registers: the next dword of a row is the next lane's (64 is a
//   multiple of the row pitch); past a row's end it only fills bytes at or
//   beyond column 16 + 2S, which no candidate reads.
// - Where two window buffers fit (es_double), the next window is staged into
//   the other buffer before the MB's one barrier; otherwise after it, behind
//   a second barrier.
// - Key per candidate in 31 bits: SAD (16 bits), then |dx| + |dy| (7), dy + S
//   (7) and whether dx > 0 (1).  With |dx| + |dy| and dy fixed, |dx| is fixed,
//   so that bit orders the two remaining candidates by dx: the same
//   lexicographic order (SAD, |dx| + |dy|, dy, dx) as the 64-bit key.
template <int S>
__global__ __launch_bounds__(kEsThreads) void es_fixed_kernel(const JobDesc *__restrict__ jobs,
                                                             const uint32_t *__restrict__ list,
                                                             const uint32_t *__restrict__ count, KParams kp) {
    constexpr int span = 16 + 2 * S, ncol = 2 * S + 1, G = es_group(S), lgp = es_pitch_log2(S), pd = 1 << lgp;
    constexpr int csz = es_copy_dwords(S), per = span << lgp, PF = (per + kEsThreads - 1) / kEsThreads;
    constexpr int ngrp = (ncol + G - 1) / G, ntask = ncol * ngrp;
    constexpr bool DB = es_double(S);
    constexpr int bufw = es_buffer_dwords(S);
    static_assert(S <= 63 && 64 % pd == 0, "31-bit keys and whole rows per wave");
    extern __shared__ uint32_t lds[];
    uint32_t *red = lds + (DB ? 2 : 1) * bufw;  // two sets of 4 wave minima
    const int tid = threadIdx.x, wave = uni(tid >> 6);
    const int nitems = (int)*count;

    uint32_t nv[PF] = {}, ncur = 0u;
    // list entry, MB origin and frame size of the MB fetched last
    uint32_t ne = 0u;
    int nx0 = 0, ny0 = 0, nW = 0, nH = 0;
    // copy 0 of list entry `item`'s window: dword u * 256 + tid into nv[u];
    // the current block's dword tid into ncur (threads 0 .. 63)
    auto fetch = [&](int item) {
        const uint32_t en = list[item];
        const JobDesc &Jn = jobs[en >> 16];
        const int kn = (int)(en & 0xFFFF);
        const int W = Jn.width, H = Jn.height, st = Jn.stride;
        ne = en;
        nx0 = 16 * (kn % Jn.wm);
        ny0 = 16 * (kn / Jn.wm);
        nW = W;
        nH = H;
        const int wx = nx0 - S, wy = ny0 - S;
        if (tid < 64) ncur = ld4(Jn.cur + (size_t)(wy + S + (tid >> 2)) * st + wx + S + 4 * (tid & 3));
        const int w = tid & (pd - 1), r0 = tid >> lgp;
        if (wx >= 0 && wx + 4 * pd <= W && wy >= 0 && wy + span <= H) {
            const uint8_t *p = Jn.ref + (size_t)(wy + r0) * st + wx + 4 * w;
#pragma unroll
            for (int u = 0; u < PF; ++u)
                if (per % kEsThreads == 0 || u * kEsThreads + tid < per)
                    nv[u] = ld4(p + (size_t)(u * (kEsThreads >> lgp)) * st);
        } else {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int r = min(r0 + u * (kEsThreads >> lgp), span - 1);
                nv[u] = ld4_clamped(Jn.ref + (size_t)iclamp(wy + r, 0, H - 1) * st, wx + 4 * w, W);
            }
        }
    };
    // the four copies and the current block from the registers
    auto stage = [&](uint32_t *win) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int idx = u * kEsThreads + tid;
            const uint32_t a = nv[u];
            uint32_t b;
            if constexpr (pd <= 16)
                b = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x101, 0xF, 0xF, true);  // row_shl:1
            else
                b = (uint32_t)__shfl((int)a, (lane() + 1) & 63, 64);
            if (per % kEsThreads == 0 || idx < per) {
                win[idx] = a;
                win[csz + idx] = __builtin_amdgcn_alignbyte(b, a, 1);
                win[2 * csz + idx] = __builtin_amdgcn_alignbyte(b, a, 2);
                win[3 * csz + idx] = __builtin_amdgcn_alignbyte(b, a, 3);
            }
        }
        if (tid < 64) win[4 * csz + tid] = ncur;
    };
    // This workgroup's MBs.  Workgroups go to the 8 XCDs in turn
    // (blockIdx.x % 8), each XCD with its own L2, and neighbouring MBs'
    // windows overlap by two thirds: XCD x takes the x-th eighth of the list,
    // which its workgroups sweep together (entry first + j * stride), so that
    // windows loaded at the same time share that L2.  Every searched MB costs
    // the same: static striding, no shared counter.  Plain striding when the
    // grid is not a multiple of 8.
    int first = (int)blockIdx.x, stride = (int)gridDim.x, last = nitems;
    if (gridDim.x % 8 == 0) {
        const int x = (int)blockIdx.x & 7, q = (int)blockIdx.x >> 3;
        stride = (int)gridDim.x >> 3;
        first = (int)(((long long)nitems * x) >> 3) + q;
        last = (int)(((long long)nitems * (x + 1)) >> 3);
    }
    if (first < last) {
        fetch(first);
        stage(lds);
    }
    __syncthreads();
    int bw = 0, br = 0;  // window buffer, minima set
    for (int it = first; it < last; it += stride) {
        const uint32_t *win = lds + bw * bufw;
        uint32_t cr[64];
        const uint4 *c4 = (const uint4 *)(win + 4 * csz);  // 16-byte aligned
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint4 q = c4[i];
            cr[4 * i] = q.x;
            cr[4 * i + 1] = q.y;
            cr[4 * i + 2] = q.z;
            cr[4 * i + 3] = q.w;
        }
        // this MB (fetched before), then the next one's loads, in flight
        // during this search
        const uint32_t e = ne;
        const int x0 = nx0, y0 = ny0, W = nW, H = nH;
        const int nxt = it + stride;
        if (nxt < last) fetch(nxt);
        // this MB's result slot, read before the search (used after the
        // barrier by thread 0)
        const JobDesc &Jr = jobs[e >> 16];
        int16_t *o_mv = Jr.mv, *o_mvi = Jr.mv_int;
        uint32_t *o_cost = Jr.cost;
        uint8_t *o_it = Jr.iters;
        uint16_t *o_pts = Jr.points;
        const int lox = kp.unrestricted ? -S : max(-S, -x0), hix = kp.unrestricted ? S : min(S, W - 16 - x0);
        const int loy = kp.unrestricted ? -S : max(-S, -y0), hiy = kp.unrestricted ? S : min(S, H - 16 - y0);
        // kept rows: dy + S in [loy + S, hiy + S] (padding rows lie above)
        const uint32_t ylo = (uint32_t)(loy + S), yspan = (uint32_t)(hiy - loy);
        uint32_t best = ~0u;
#pragma unroll
        for (int t0 = 0; t0 < ntask; t0 += kEsThreads) {
            const int task = t0 + tid;
            if (ntask % kEsThreads != 0 && task >= ntask) break;
            const int cxr = task % ncol;        // dx + S
            const int dy0 = (task / ncol) * G;  // first dy + S
            const int dx = cxr - S;
            if (dx < lox || dx > hix) continue;
            const uint32_t *cp = win + (cxr & 3) * csz + (cxr >> 2) + dy0 * pd;
            uint32_t acc[G];
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = 0;
#pragma unroll
            for (int r = 0; r < G + 15; ++r) {
                // rows past the window are padding: read, never kept
                const uint32_t r0 = cp[r * pd], r1 = cp[r * pd + 1], r2 = cp[r * pd + 2], r3 = cp[r * pd + 3];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int jj = r - g;
                    if (jj >= 0 && jj < 16) {
                        uint32_t a = acc[g];
                        a = __builtin_amdgcn_sad_u8(cr[4 * jj + 0], r0, a);
                        a = __builtin_amdgcn_sad_u8(cr[4 * jj + 1], r1, a);
                        a = __builtin_amdgcn_sad_u8(cr[4 * jj + 2], r2, a);
                        a = __builtin_amdgcn_sad_u8(cr[4 * jj + 3], r3, a);
                        acc[g] = a;
                    }
                }
            }
            const uint32_t adx = (uint32_t)abs(dx), pos = dx > 0 ? 1u : 0u;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int dys = dy0 + g;
                const uint32_t key = (acc[g] << 15) | ((adx + (uint32_t)abs(dys - S)) << 8) | ((uint32_t)dys << 1) | pos;
                best = (uint32_t)dys - ylo <= yspan ? min(best, key) : best;
            }
        }
        best = wave_min_to_last(best);
        if (lane() == 63) red[br * 4 + wave] = best;
        if constexpr (DB)
            if (nxt < last) stage(lds + (bw ^ 1) * bufw);
        __syncthreads();
        if (tid == 0) {
            uint32_t b = red[br * 4];
            for (int w = 1; w < kEsThreads / 64; ++w) b = min(b, red[br * 4 + w]);
            const int dys = (int)((b >> 1) & 127), dy = dys - S;
            const int adx = (int)((b >> 8) & 127) - abs(dy);
            const int pts = (hix - lox + 1) * (hiy - loy + 1);
            const int k = (int)(e & 0xFFFF), dx = (b & 1) ? adx : -adx;
            const uint32_t mvw = (uint32_t)(uint16_t)(2 * dx) | ((uint32_t)(uint16_t)(2 * dy) << 16);
            ((uint32_t *)o_mv)[k] = mvw;
            ((uint32_t *)o_mvi)[k] = mvw;
            if (o_cost) o_cost[k] = b >> 15;
            if (o_it) o_it[k] = 0;
            if (o_pts) o_pts[k] = (uint16_t)pts;
        }
        if constexpr (DB) {
            bw ^= 1;
        } else if (nxt < last) {
            stage(lds);
            __syncthreads();
        }
        br ^= 1;
    }
}

// TSS / 4SS / DS.  One wave per MB; each round's candidates are evaluated together
// (lane = row j, quad q; 4 pixels per lane, unaligned dword loads from the
// L2-resident reference), partial SADs packed two per reduction.  A bitmap of
// evaluated positions in LDS counts distinct search points.
constexpr int kMemoWords = (129 * 129 + 31) / 32;

__constant__ int kLdsp[8][2] = {{0, -2}, {-1, -1}, {1, -1}, {-2, 0}, {2, 0}, {-1, 1}, {1, 1}, {0, 2}};
__constant__ int kSdsp[4][2] = {{0, -1}, {-1, 0}, {1, 0}, {0, 1}};

struct Mb {
    const uint8_t *ref;
    int st, W, H, x, y;  // frame size, this lane's first pixel
    uint32_t c4;
    int lox, hix, loy, hiy, S;
    uint32_t *memo;
    int pts;
};

__device__ __forceinline__ bool feas(const Mb &m, int dx, int dy) {
    return dx >= m.lox && dx <= m.hix && dy >= m.loy && dy <= m.hiy;
}

__device__ __forceinline__ void visit(Mb &m, int dx, int dy) {
    int i = (dy + m.S) * (2 * m.S + 1) + (dx + m.S);
    uint32_t w = m.memo[i >> 5], bit = 1u << (i & 31);
    if (!(w & bit)) {
        m.memo[i >> 5] = w | bit;
        m.pts++;
    }
}

// Evaluate up to 8 offsets (ox, oy), returns SADs (infeasible -> ~0u).
template <int N>
__device__ __forceinline__ void eval_pts(Mb &m, const int (&ox)[N], const int (&oy)[N], uint32_t (&out)[N]) {
    int part[N + (N & 1)];
    bool ok[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        ok[i] = feas(m, ox[i], oy[i]);
        part[i] = 0;
        if (ok[i]) {
            // coordinates clamped: the frame extended by its edge pixels
            // (reached only by unrestricted vectors)
            const uint32_t r4 = ld4_clamped(m.ref + (size_t)iclamp(m.y + oy[i], 0, m.H - 1) * m.st, m.x + ox[i], m.W);
            part[i] = (int)__builtin_amdgcn_sad_u8(m.c4, r4, 0u);
        }
    }
    if (N & 1) part[N] = 0;
#pragma unroll
    for (int i = 0; i < N; i += 2) {
        int pk = wave_sum(part[i] | ((i + 1 < N ? part[i + 1] : 0) << 16));
        out[i] = ok[i] ? (uint32_t)(pk & 0xFFFF) : ~0u;
        if (i + 1 < N) out[i + 1] = ok[i + 1] ? (uint32_t)((uint32_t)pk >> 16) : ~0u;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (ok[i]) visit(m, ox[i], oy[i]);
}

__global__ __launch_bounds__(64) void tss_ds_kernel(const JobDesc *jobs, const uint32_t *list,
                                                    const uint32_t *count, KParams kp, int method) {
    __shared__ uint32_t memo[kMemoWords];
    const int l = lane();
    const int nitems = (int)*count;
    // static striding over the searched MBs (a shared counter would
    // serialise every pick at one L2 atomic)
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const uint32_t e = list[it];
    const JobDesc &J = jobs[e >> 16];
    const int k = (int)(e & 0xFFFF);
    const int h = k % J.wm, v = k / J.wm;
    const int x0 = 16 * h, y0 = 16 * v;
    const int S = kp.S;
    const int words = ((2 * S + 1) * (2 * S + 1) + 31) >> 5;
    for (int i = l; i < words; i += 64) memo[i] = 0;
    Mb m;
    m.ref = J.ref;
    m.st = J.stride;
    m.W = J.width;
    m.H = J.height;
    m.x = x0 + 4 * (l & 3);
    m.y = y0 + (l >> 2);
    m.c4 = *(const uint32_t *)(J.cur + (size_t)m.y * m.st + m.x);
    m.lox = kp.unrestricted ? -S : max(-S, -x0);
    m.hix = kp.unrestricted ? S : min(S, J.width - 16 - x0);
    m.loy = kp.unrestricted ? -S : max(-S, -y0);
    m.hiy = kp.unrestricted ? S : min(S, J.height - 16 - y0);
    m.S = S;
    m.memo = memo;
    m.pts = 0;
    int cx = 0, cy = 0;
    uint32_t cc;
    {
        int ox[1] = {0}, oy[1] = {0};
        uint32_t o[1];
        eval_pts<1>(m, ox, oy, o);
        cc = o[0];
    }
    if (method == ME_TSS) {
        int p2 = 1;
        while (p2 < S + 1) p2 *= 2;
        for (int stp = p2 / 2; stp >= 1; stp /= 2) {
            int ox[8], oy[8];
            int i = 0;
#pragma unroll
            for (int jj = -1; jj <= 1; ++jj)
#pragma unroll
                for (int ii = -1; ii <= 1; ++ii)
                    if (ii || jj) {
                        ox[i] = cx + ii * stp;
                        oy[i] = cy + jj * stp;
                        ++i;
                    }
            uint32_t c[8];
            eval_pts<8>(m, ox, oy, c);
            int nx = cx, ny = cy;
            uint32_t nc = cc;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (c[q] < nc) {
                    nc = c[q];
                    nx = ox[q];
                    ny = oy[q];
                }
            cx = nx;
            cy = ny;
            cc = nc;
        }
    } else if (method == ME_4SS) {
        // squares of step 2 until the centre wins (at most ceil((S-1)/2) of
        // them, three at S = 7), then the square of step 1
        const int n5 = max(S / 2, 1);
        for (int round = 0; round <= n5; ++round) {
            const int stp = round < n5 ? 2 : 1;
            int ox[8], oy[8];
            int i = 0;
#pragma unroll
            for (int jj = -1; jj <= 1; ++jj)
#pragma unroll
                for (int ii = -1; ii <= 1; ++ii)
                    if (ii || jj) {
                        ox[i] = cx + ii * stp;
                        oy[i] = cy + jj * stp;
                        ++i;
                    }
            uint32_t c[8];
            eval_pts<8>(m, ox, oy, c);
            int nx = cx, ny = cy;
            uint32_t nc = cc;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (c[q] < nc) {
                    nc = c[q];
                    nx = ox[q];
                    ny = oy[q];
                }
            const bool moved = nx != cx || ny != cy;
            cx = nx;
            cy = ny;
            cc = nc;
            if (stp == 2 && !moved) round = n5 - 1;  // the centre won: the step-1 square is next
        }
    } else {
        for (int guard = 0; guard < 65536; ++guard) {
            int ox[8], oy[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                ox[q] = cx + kLdsp[q][0];
                oy[q] = cy + kLdsp[q][1];
            }
            uint32_t c[8];
            eval_pts<8>(m, ox, oy, c);
            int nx = cx, ny = cy;
            uint32_t nc = cc;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (c[q] < nc) {
                    nc = c[q];
                    nx = ox[q];
                    ny = oy[q];
                }
            if (nx == cx && ny == cy) break;
            cx = nx;
            cy = ny;
            cc = nc;
        }
        int ox[4], oy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ox[q] = cx + kSdsp[q][0];
            oy[q] = cy + kSdsp[q][1];
        }
        uint32_t c[4];
        eval_pts<4>(m, ox, oy, c);
        int nx = cx, ny = cy;
        uint32_t nc = cc;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (c[q] < nc) {
                nc = c[q];
                nx = ox[q];
                ny = oy[q];
            }
        cx = nx;
        cy = ny;
        cc = nc;
    }
    if (l == 0) write_result(J, k, cx, cy, cc, m.pts);
    }
}

}  // namespace

size_t es_lds_bytes(int S) {
    if (es_fixed(S)) return (size_t)((es_double(S) ? 2 : 1) * es_buffer_dwords(S) + 8) * 4;
    return (size_t)es_buffer_dwords(S) * 4 + 4 * sizeof(unsigned long long);
}

size_t full_search_scratch(int total_mbs) { return (size_t)total_mbs * 4; }

hipError_t launch_full_search(int method, const JobDesc *jobs, int n, int total_mbs, const KParams &kp,
                              uint32_t *counters, uint32_t *list, uint32_t *status, hipStream_t s,
                              const KernelTimer *t) {
    if (total_mbs <= 0) return hipSuccess;
    hipLaunchKernelGGL(compact_kernel, dim3((total_mbs + 255) / 256), dim3(256), 0, s, jobs, n, total_mbs, list,
                       counters, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    timer_mark(t, true, s);
    if (method == ME_ES) {
        size_t lds = es_lds_bytes(kp.S);
        int blocks = std::min(total_mbs, cus * 8);
#define ME_ES_LAUNCH(kern) hipLaunchKernelGGL((kern), dim3(blocks), dim3(kEsThreads), lds, s, jobs, list, counters, kp)
        const int G = es_group(kp.S);
        if (kp.S == 7) ME_ES_LAUNCH(es_fixed_kernel<7>);
        else if (kp.S == 16) ME_ES_LAUNCH(es_fixed_kernel<16>);
        else if (kp.S == 32) ME_ES_LAUNCH(es_fixed_kernel<32>);
        else if (G == 4) ME_ES_LAUNCH(es_kernel<4>);
        else if (G == 5) ME_ES_LAUNCH(es_kernel<5>);
        else if (G == 6) ME_ES_LAUNCH(es_kernel<6>);
        else ME_ES_LAUNCH(es_kernel<8>);
#undef ME_ES_LAUNCH
    } else {
        int blocks = std::min(total_mbs, cus * 16);
        hipLaunchKernelGGL(tss_ds_kernel, dim3(blocks), dim3(64), 0, s, jobs, list, counters, kp, method);
    }
    e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

}  // namespace me

// Reference VOP padding (Section 4 protocol: the reference is an MPEG-4 VOP,
// whose texture outside the shape is filled before blocks are matched against
// it; MPEG-4 Visual's padding of arbitrarily shaped VOPs on the frame's MB
// grid).  Inside means alpha != 0.
//  - Opaque MB: copied.
//  - Boundary MB, repetitive padding within the 16x16 block: along each row, a
//    sample outside the shape takes the rounded-up mean of the nearest inside
//    samples to its left and right, or the one that exists; rows with no
//    inside sample stay open and take the same rule along each column over
//    the row-padded samples.
//  - Transparent MB, extended padding: the border of its first adjacent MB
//    that is not transparent, in the order left, above, right, below, is
//    repeated over the block; with no such neighbour every sample is 128.
// Two launches: the first pads the opaque and boundary MBs and records every
// MB's class, the second the transparent MBs from their padded neighbours.
#include "flat_kernels.h"

namespace me {

namespace {

// One 64-thread block takes 4 MBs of job blockIdx.y, 16 lanes per MB.
constexpr int kPadMbs = 4;

__device__ __forceinline__ int pad_mean(int a, int b) { return (a + b + 1) >> 1; }

// The value a sample outside the shape takes from the inside samples of its
// line (16 samples `v`, bit i of `in` set for inside samples): the rounded-up
// mean of the nearest ones on both sides, or the one that exists.  `in` is
// non-zero and bit i is clear.
template <class F>
__device__ __forceinline__ int line_fill(uint32_t in, int i, F v) {
    const uint32_t lo = in & ((1u << i) - 1u), hi = in & ~((2u << i) - 1u);
    if (lo && hi) return pad_mean(v(31 - __builtin_clz(lo)), v(__builtin_ctz(hi)));
    return lo ? v(31 - __builtin_clz(lo)) : v(__builtin_ctz(hi));
}

__device__ __forceinline__ int byte_at(const uint32_t (&w)[4], int i) { return (int)((w[i >> 2] >> (8 * (i & 3))) & 0xFFu); }

// Pass 1.  Lane r of an MB holds its row r, then its column r.
__global__ __launch_bounds__(64) void pad_inner_kernel(const JobDesc *jobs, uint8_t *cls_all) {
    __shared__ uint32_t rowpad[kPadMbs][16][5];  // row-padded samples (row pitch 5 dwords)
    __shared__ uint32_t fin[kPadMbs][16][5];     // padded samples
    const JobDesc &J = jobs[blockIdx.y];
    const int wm = J.wm, st = J.stride;
    const int s = (int)threadIdx.x >> 4, r = (int)threadIdx.x & 15;
    const int k = (int)blockIdx.x * kPadMbs + s;
    const bool valid = k < wm * J.hm;
    const int x0 = valid ? 16 * (k % wm) : 0, y0 = valid ? 16 * (k / wm) : 0;
    uint32_t L[4] = {0u, 0u, 0u, 0u}, A[4] = {0u, 0u, 0u, 0u};
    if (valid) {
        const uint32_t *pl = (const uint32_t *)(J.cur + (size_t)(y0 + r) * st + x0);
        const uint32_t *pa = (const uint32_t *)(J.cur_a + (size_t)(y0 + r) * st + x0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            L[u] = ldg32(pl + u);
            A[u] = ldg32(pa + u);
        }
    }
    uint32_t in = 0u;  // bit i: sample i of row r is inside
#pragma unroll
    for (int i = 0; i < 16; ++i) in |= (byte_at(A, i) != 0 ? 1u : 0u) << i;
    int n = __popc(in);
    n += __shfl_xor(n, 1, 64);
    n += __shfl_xor(n, 2, 64);
    n += __shfl_xor(n, 4, 64);
    n += __shfl_xor(n, 8, 64);
    const int c = n == 0 ? ME_MB_TRANSPARENT : (n == 256 ? ME_MB_OPAQUE : ME_MB_BOUNDARY);
    if (valid && r == 0) cls_all[J.mb_base + k] = (uint8_t)c;
    // bit j: row j of this MB has an inside sample
    const uint32_t rows = (uint32_t)(__ballot(in != 0u) >> (16 * s)) & 0xFFFFu;
    // rows
    uint32_t Hp[4] = {L[0], L[1], L[2], L[3]};
    if (c == ME_MB_BOUNDARY && in != 0u) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if ((in >> i) & 1u) continue;
            const int val = line_fill(in, i, [&](int x) { return byte_at(L, x); });
            Hp[i >> 2] = (Hp[i >> 2] & ~(0xFFu << (8 * (i & 3)))) | ((uint32_t)val << (8 * (i & 3)));
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) rowpad[s][r][u] = Hp[u];
    __syncthreads();
    // columns (lane r: column r), open rows only
    if (c == ME_MB_BOUNDARY) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            auto at = [&](int y) { return (int)((const uint8_t *)rowpad[s][y])[r]; };
            const int val = ((rows >> j) & 1u) ? at(j) : line_fill(rows, j, at);
            ((uint8_t *)fin[s][j])[r] = (uint8_t)val;
        }
    }
    __syncthreads();
    if (valid && c != ME_MB_TRANSPARENT) {
        uint32_t *po = (uint32_t *)(J.out_u8 + (size_t)(y0 + r) * st + x0);
#pragma unroll
        for (int u = 0; u < 4; ++u) po[u] = c == ME_MB_BOUNDARY ? fin[s][r][u] : L[u];
    }
}

// Pass 2: transparent MBs from the padded border of a neighbour.
__global__ __launch_bounds__(64) void pad_outer_kernel(const JobDesc *jobs, const uint8_t *cls_all) {
    const JobDesc &J = jobs[blockIdx.y];
    const int wm = J.wm, hm = J.hm, st = J.stride;
    const int s = (int)threadIdx.x >> 4, r = (int)threadIdx.x & 15;
    const int k = (int)blockIdx.x * kPadMbs + s;
    if (k >= wm * hm) return;
    const uint8_t *cls = cls_all + J.mb_base;
    if (cls[k] != ME_MB_TRANSPARENT) return;
    const int h = k % wm, v = k / wm, x0 = 16 * h, y0 = 16 * v;
    uint8_t *out = J.out_u8;
    uint32_t w[4];
    if (h > 0 && cls[k - 1] != ME_MB_TRANSPARENT) {
        const uint32_t b = out[(size_t)(y0 + r) * st + x0 - 1] * 0x01010101u;
        w[0] = w[1] = w[2] = w[3] = b;
    } else if (v > 0 && cls[k - wm] != ME_MB_TRANSPARENT) {
        const uint32_t *p = (const uint32_t *)(out + (size_t)(y0 - 1) * st + x0);
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = p[u];
    } else if (h + 1 < wm && cls[k + 1] != ME_MB_TRANSPARENT) {
        const uint32_t b = out[(size_t)(y0 + r) * st + x0 + 16] * 0x01010101u;
        w[0] = w[1] = w[2] = w[3] = b;
    } else if (v + 1 < hm && cls[k + wm] != ME_MB_TRANSPARENT) {
        const uint32_t *p = (const uint32_t *)(out + (size_t)(y0 + 16) * st + x0);
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = p[u];
    } else {
        w[0] = w[1] = w[2] = w[3] = 0x80808080u;
    }
    uint32_t *po = (uint32_t *)(out + (size_t)(y0 + r) * st + x0);
#pragma unroll
    for (int u = 0; u < 4; ++u) po[u] = w[u];
}

}  // namespace

hipError_t launch_pad(const JobDesc *jobs, int n, int max_mbs, uint8_t *cls_all, hipStream_t s) {
    if (n <= 0 || max_mbs <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_mbs + kPadMbs - 1) / kPadMbs), (unsigned)n);
    hipLaunchKernelGGL(pad_inner_kernel, grid, dim3(64), 0, s, jobs, cls_all);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pad_outer_kernel, grid, dim3(64), 0, s, jobs, (const uint8_t *)cls_all);
    return hipGetLastError();
}

}  // namespace me

// MB classification from the binary alpha plane (Section 1) and motion
// compensation + squared error (Section 4).  Both read each pixel once and
// are bound by HBM.  Layout: 16 lanes per MB, lane = one 16-pixel row, four
// MBs per wave; per-MB sums are 16-lane DPP reductions (no atomics).
#include "me_internal.h"

namespace me {

namespace {

__global__ __launch_bounds__(64) void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Sum over each group of 16 lanes (a DPP row), result in every lane of the row.
__device__ __forceinline__ int row_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
    return v;
}

// bit i set where byte i of the 4 words (16 bytes) is non-zero
__device__ __forceinline__ uint32_t nz16(const uint32_t (&a)[4]) {
    uint32_t bits = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t nz = (((a[w] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | a[w]) & 0x80808080u;
        bits |= (((nz >> 7) & 1u) | ((nz >> 14) & 2u) | ((nz >> 21) & 4u) | ((nz >> 28) & 8u)) << (4 * w);
    }
    return bits;
}

// Quads of 4 consecutive MBs per wave; a block strides its waves over a
// contiguous range of quads.  Each lane tracks the job of its own MB.
struct QuadIter {
    int q, qend, step;
};

__device__ __forceinline__ QuadIter quads(int total, int chunk) {
    const int nq = (total + 3) >> 2;
    QuadIter it;
    it.q = blockIdx.x * chunk + (threadIdx.x >> 6);
    it.qend = min(blockIdx.x * chunk + chunk, nq);
    it.step = 4;
    return it;
}

// n = number of pixels with alpha != 0 -> transparent (0), opaque (256),
// boundary, written to the job's class array; BAB word w = rows 2w, 2w+1
// with column i at bit (row&1)*16 + i.  Jobs without alpha or without a
// class array (rectangular frames) are skipped.
__global__ __launch_bounds__(256) void classify_kernel(const JobDesc *jobs, int n, int total, int chunk) {
    const int l = lane(), r = l & 15;
    QuadIter it = quads(total, chunk);
    if (it.q >= it.qend) return;
    int ji = find_job(jobs, n, min(4 * it.q, total - 1));
    for (; it.q < it.qend; it.q += it.step) {
        const int mb = 4 * it.q + (l >> 4);
        const bool valid = mb < total;
        const int m = valid ? mb : total - 1;
        ji = next_job(jobs, n, ji, m);
        const JobDesc &J = jobs[ji];
        const int k = m - J.mb_base;
        const int h = k % J.wm, v = k / J.wm;
        const bool has = J.cur_a != nullptr && J.cls != nullptr;
        uint32_t a[4] = {0u, 0u, 0u, 0u};
        if (has) {
            const uint32_t *row = (const uint32_t *)(J.cur_a + (size_t)(16 * v + r) * J.stride + 16 * h);
#pragma unroll
            for (int w = 0; w < 4; ++w) a[w] = ldg32(row + w);
        }
        const uint32_t bits = nz16(a);
        const int tot = row_sum(__builtin_popcount(bits));
        const uint32_t odd = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0xB1, 0xF, 0xF, true);
        if (valid && has) {
            if (J.out_u32 && (r & 1) == 0) J.out_u32[(size_t)k * 8 + (r >> 1)] = bits | (odd << 16);
            if (r == 0)
                const_cast<uint8_t *>(J.cls)[k] =
                    (uint8_t)(tot == 0 ? ME_MB_TRANSPARENT : (tot == 256 ? ME_MB_OPAQUE : ME_MB_BOUNDARY));
        }
    }
}

// Prediction of one 16-pixel row by the half-pel vector (ix, fx; iy, fy),
// MPEG-4 bilinear with rounding control 0, coordinates clamped to the frame.
__device__ __forceinline__ void predict_row(const uint8_t *ref, int st, int W, int H, int x, int y, int hx, int hy,
                                            uint32_t (&out)[4]) {
    const int ix = hx >> 1, iy = hy >> 1, fx = hx & 1, fy = hy & 1;
    const uint8_t *ra = ref + (size_t)iclamp(y + iy, 0, H - 1) * st;
    uint32_t a[5];
#pragma unroll
    for (int w = 0; w < 5; ++w) a[w] = ld4_clamped(ra, x + ix + 4 * w, W);
    if (!fx && !fy) {
#pragma unroll
        for (int w = 0; w < 4; ++w) out[w] = a[w];
        return;
    }
    const uint8_t *rb = ref + (size_t)iclamp(y + iy + 1, 0, H - 1) * st;
    uint32_t c[5];
#pragma unroll
    for (int w = 0; w < 5; ++w) c[w] = fy ? ld4_clamped(rb, x + ix + 4 * w, W) : 0u;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = 4 * w + b;
            const int A = byte_of(a[i >> 2], i & 3), B = byte_of(a[(i + 1) >> 2], (i + 1) & 3);
            const int Cc = byte_of(c[i >> 2], i & 3), D = byte_of(c[(i + 1) >> 2], (i + 1) & 3);
            const int p = (fx && fy) ? ((A + B + Cc + D + 2) >> 2) : fx ? ((A + B + 1) >> 1) : ((A + Cc + 1) >> 1);
            o |= (uint32_t)p << (8 * b);
        }
        out[w] = o;
    }
}

// Prediction of MB k by its half-pel vector (transparent: zero vector),
// written to out_u8 when set; per-MB SSE and pixel count over the mask to
// part[2 * mb], part[2 * mb + 1].
__global__ __launch_bounds__(256) void mc_kernel(const JobDesc *jobs, int n, int total, int chunk, uint32_t *part) {
    const int l = lane(), r = l & 15;
    QuadIter it = quads(total, chunk);
    if (it.q >= it.qend) return;
    int ji = find_job(jobs, n, min(4 * it.q, total - 1));
    for (; it.q < it.qend; it.q += it.step) {
        const int mb = 4 * it.q + (l >> 4);
        const bool valid = mb < total;
        const int m = valid ? mb : total - 1;
        ji = next_job(jobs, n, ji, m);
        const JobDesc &J = jobs[ji];
        const int k = m - J.mb_base;
        const int h = k % J.wm, v = k / J.wm;
        const int W = J.width, H = J.height, st = J.stride;
        const int cls = J.cls ? (int)J.cls[k] : ME_MB_OPAQUE;
        int hx = 0, hy = 0;
        if (cls != ME_MB_TRANSPARENT) {
            const uint32_t w = ((const uint32_t *)J.mv)[k];
            hx = (int)(int16_t)(w & 0xFFFF);
            hy = (int)(int16_t)(w >> 16);
        }
        const int x = 16 * h, y = 16 * v + r;
        const uint32_t *crow = (const uint32_t *)(J.cur + (size_t)y * st + x);
        uint32_t c[4], mk[4], p[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) c[w] = ldg32(crow + w);
        if (J.cur_a) {
            const uint32_t *arow = (const uint32_t *)(J.cur_a + (size_t)y * st + x);
#pragma unroll
            for (int w = 0; w < 4; ++w) mk[w] = ldg32(arow + w);
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w) mk[w] = 0xFFFFFFFFu;
        }
        predict_row(J.ref, st, W, H, x, y, hx, hy, p);
        if (valid && J.out_u8) {
            uint32_t *prow = (uint32_t *)(J.out_u8 + (size_t)y * st + x);
#pragma unroll
            for (int w = 0; w < 4; ++w) prow[w] = p[w];
        }
        const uint32_t in = nz16(mk);
        int sse = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int d = byte_of(c[i >> 2], i & 3) - byte_of(p[i >> 2], i & 3);
            sse += ((in >> i) & 1u) ? d * d : 0;
        }
        const int tsse = row_sum(sse);
        const int tcnt = row_sum(__builtin_popcount(in));
        if (valid && r == 0) {
            part[2 * (size_t)mb] = (uint32_t)tsse;
            part[2 * (size_t)mb + 1] = (uint32_t)tcnt;
        }
    }
}

// Per job: the exact 64-bit sums of its MBs' SSE and pixel counts.
__global__ __launch_bounds__(256) void mc_reduce_kernel(const JobDesc *jobs, const uint32_t *part,
                                                        unsigned long long *acc) {
    __shared__ unsigned long long red[2][4];
    const JobDesc &J = jobs[blockIdx.x];
    const int nmb = J.wm * J.hm;
    unsigned long long s = 0, c = 0;
    for (int i = threadIdx.x; i < nmb; i += 256) {
        s += part[2 * ((size_t)J.mb_base + i)];
        c += part[2 * ((size_t)J.mb_base + i) + 1];
    }
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if (lane() == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        acc[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 63) / 64;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(64), 0, s, p, n, v);
    return hipGetLastError();
}

// Units (MBs, or quads of MBs) per block so that a flat grid has about
// per_cu blocks per CU.
int flat_chunk(int total_units, int per_cu) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    long long blocks = (long long)(cus > 0 ? cus : 256) * per_cu;
    long long c = (total_units + blocks - 1) / blocks;
    return (int)(c < 1 ? 1 : c);
}

hipError_t launch_classify(const JobDesc *jobs, int n, int total_mbs, hipStream_t s, const KernelTimer *t,
                           int per_cu) {
    if (total_mbs <= 0) return hipSuccess;
    const int nq = (total_mbs + 3) / 4;
    const int chunk = (flat_chunk(nq, per_cu) + 3) / 4 * 4;
    timer_mark(t, true, s);
    hipLaunchKernelGGL(classify_kernel, dim3((nq + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs, chunk);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

size_t mc_scratch(int total_mbs) { return (size_t)total_mbs * 8; }

hipError_t launch_mc(const JobDesc *jobs, int n, int total_mbs, uint32_t *part, unsigned long long *acc,
                     hipStream_t s, const KernelTimer *t, int per_cu) {
    if (total_mbs <= 0) return hipSuccess;
    const int nq = (total_mbs + 3) / 4;
    const int chunk = (flat_chunk(nq, per_cu) + 3) / 4 * 4;
    timer_mark(t, true, s);
    hipLaunchKernelGGL(mc_kernel, dim3((nq + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs, chunk, part);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mc_reduce_kernel, dim3(n), dim3(256), 0, s, jobs, part, acc);
    return hipGetLastError();
}

}  // namespace me

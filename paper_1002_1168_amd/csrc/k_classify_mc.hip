// MB classification from the binary alpha plane (Section 1) and motion
// compensation + squared error (Section 4).  Both read each pixel once and
// are bound by HBM; one wave per MB, lane = (row j, quad q), 4 pixels/lane.
#include "me_internal.h"

namespace me {

namespace {

__global__ __launch_bounds__(64) void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// n = number of pixels with alpha != 0 -> transparent (0), opaque (256),
// boundary; BAB word w = rows 2w, 2w+1 with column i at bit (row&1)*16 + i.
__global__ __launch_bounds__(256) void classify_kernel(const JobDesc *jobs, int n, int total, int chunk) {
    const int first = blockIdx.x * chunk + (threadIdx.x >> 6);
    const int last = min(blockIdx.x * chunk + chunk, total);
    int ji = first < total ? find_job(jobs, n, first) : 0;
    for (int mb = first; mb < last; mb += 4) {
    ji = next_job(jobs, n, ji, mb);
    const JobDesc &J = jobs[ji];
    const int k = mb - J.mb_base;
    const int h = k % J.wm, v = k / J.wm;
    const int l = lane(), j = l >> 2, q = l & 3;
    uint32_t a = *(const uint32_t *)(J.cur_a + (size_t)(16 * v + j) * J.stride + 16 * h + 4 * q);
    uint32_t nz = (((a & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | a) & 0x80808080u;  // bit 7 of each non-zero byte
    uint32_t nib = ((nz >> 7) & 1u) | ((nz >> 14) & 2u) | ((nz >> 21) & 4u) | ((nz >> 28) & 8u);
    int cnt = __builtin_popcount(nib);
    int tot = wave_sum(cnt);
    // 8 lanes (2 rows x 4 quads) make one BAB word; their nibbles do not overlap
    int w = (int)(nib << (4 * (l & 7)));
    w += __builtin_amdgcn_update_dpp(0, w, 0xB1, 0xF, 0xF, true);
    w += __builtin_amdgcn_update_dpp(0, w, 0x4E, 0xF, 0xF, true);
    w += __builtin_amdgcn_update_dpp(0, w, 0x141, 0xF, 0xF, true);
    if (J.out_u32 && (l & 7) == 0) J.out_u32[(size_t)k * 8 + (l >> 3)] = (uint32_t)w;
    if (l == 0) J.out_u8[k] = (uint8_t)(tot == 0 ? ME_MB_TRANSPARENT : (tot == 256 ? ME_MB_OPAQUE : ME_MB_BOUNDARY));
    }
}

__device__ __forceinline__ int pix(const uint8_t *p, int st, int W, int H, int x, int y) {
    return p[(size_t)iclamp(y, 0, H - 1) * st + iclamp(x, 0, W - 1)];
}

// Prediction of MB k by its half-pel vector (transparent: zero vector),
// written to out_u8 when set; SSE and pixel count over the mask accumulate
// into acc[2 * job] (exact integer sums, order-independent).
__global__ __launch_bounds__(256) void mc_kernel(const JobDesc *jobs, int n, int total, int chunk,
                                                 unsigned long long *acc) {
    const int first = blockIdx.x * chunk + (threadIdx.x >> 6);
    const int last = min(blockIdx.x * chunk + chunk, total);
    int ji = first < total ? find_job(jobs, n, first) : 0;
    for (int mb = first; mb < last; mb += 4) {
    ji = next_job(jobs, n, ji, mb);
    const JobDesc &J = jobs[ji];
    const int k = mb - J.mb_base;
    const int h = k % J.wm, v = k / J.wm;
    const int l = lane(), j = l >> 2, q = l & 3;
    const int W = J.width, H = J.height, st = J.stride;
    const int cls = J.cls ? (int)J.cls[k] : ME_MB_OPAQUE;
    int hx = 0, hy = 0;
    if (cls != ME_MB_TRANSPARENT) {
        uint32_t w = ((const uint32_t *)J.mv)[k];
        hx = (int)(int16_t)(w & 0xFFFF);
        hy = (int)(int16_t)(w >> 16);
    }
    const int ix = hx >> 1, iy = hy >> 1, fx = hx & 1, fy = hy & 1;
    const int x = 16 * h + 4 * q, y = 16 * v + j;
    uint32_t c4 = *(const uint32_t *)(J.cur + (size_t)y * st + x);
    uint32_t m4 = J.cur_a ? *(const uint32_t *)(J.cur_a + (size_t)y * st + x) : 0xFFFFFFFFu;
    uint32_t p4 = 0;
    int sse = 0, cnt = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        int xx = x + kk + ix, yy = y + iy;
        int A = pix(J.ref, st, W, H, xx, yy);
        int p = A;
        if (fx || fy) {
            int B = pix(J.ref, st, W, H, xx + 1, yy);
            int Cc = pix(J.ref, st, W, H, xx, yy + 1);
            int D = pix(J.ref, st, W, H, xx + 1, yy + 1);
            p = (fx && fy) ? ((A + B + Cc + D + 2) >> 2) : fx ? ((A + B + 1) >> 1) : ((A + Cc + 1) >> 1);
        }
        p4 |= (uint32_t)p << (8 * kk);
        if (byte_of(m4, kk)) {
            int d = byte_of(c4, kk) - p;
            sse += d * d;
            cnt += 1;
        }
    }
    if (J.out_u8) *(uint32_t *)(J.out_u8 + (size_t)y * st + x) = p4;
    int tsse = wave_sum(sse);
    int tcnt = wave_sum(cnt);
    if (l == 0) {
        if (tsse) atomicAdd(acc + 2 * ji, (unsigned long long)(uint32_t)tsse);
        if (tcnt) atomicAdd(acc + 2 * ji + 1, (unsigned long long)tcnt);
    }
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

// MBs per block so that a flat grid has about per_cu blocks per CU.
int flat_chunk(int total_mbs, int per_cu) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    long long blocks = (long long)(cus > 0 ? cus : 256) * per_cu;
    long long c = (total_mbs + blocks - 1) / blocks;
    return (int)(c < 1 ? 1 : c);
}

hipError_t launch_classify(const JobDesc *jobs, int n, int total_mbs, hipStream_t s) {
    if (total_mbs <= 0) return hipSuccess;
    int chunk = (flat_chunk(total_mbs, 8) + 3) / 4 * 4;
    hipLaunchKernelGGL(classify_kernel, dim3((total_mbs + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs,
                       chunk);
    return hipGetLastError();
}

hipError_t launch_mc(const JobDesc *jobs, int n, int total_mbs, unsigned long long *acc, hipStream_t s) {
    if (total_mbs <= 0) return hipSuccess;
    int chunk = (flat_chunk(total_mbs, 8) + 3) / 4 * 4;
    hipLaunchKernelGGL(mc_kernel, dim3((total_mbs + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs, chunk,
                       acc);
    return hipGetLastError();
}

}  // namespace me

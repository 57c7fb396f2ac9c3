// Four vectors per MB (Section 3.2: with MPEG-4's four motion vectors per
// macroblock the recursive search works on 8 x 8 blocks): the pel-recursive
// refinement of Eqs. 3-5 on each 8 x 8 block of every texture MB, started
// from the MB's full-pel vector, then (half_pel) the eight half-sample
// offsets around each block's vector.  No MB depends on another: a flat
// range over the MBs of all jobs, one wave per MB, 16 lanes per block (lane
// = block b, row j, half q: four pixels), so the four blocks' recursions run
// side by side and every block sum is a 16-lane DPP reduction.  Reference
// bytes come straight from global memory (L2), coordinates clamped to the
// frame (which is also the edge extension of unrestricted vectors).
#include <algorithm>

#include "me_internal.h"

namespace me {

namespace {

// Sum over the 16 lanes of a DPP row, in every lane of the row.
__device__ __forceinline__ int sum16(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
    return v;
}

// 4 bytes of reference row y (clamped) from column x (clamped, edge bytes replicated).
__device__ __forceinline__ uint32_t ref4(const uint8_t *ref, int st, int W, int H, int x, int y) {
    return ld4_clamped(ref + (size_t)iclamp(y, 0, H - 1) * st, x, W);
}

struct Px {
    const uint8_t *ref;
    const short *R;
    int st, W, H;
    int px, py;  // this lane's first pixel
    uint32_t c4;
};

struct Pass {
    int sad, sx, sy, nxy;
};

// SAD of the lane's block at (dx, dy) and the gradient sums of Eqs. 3-5
// (central differences of the reference at the displaced pixels).
__device__ __forceinline__ Pass pass8(const Px &p, int dx, int dy) {
    const int rx = p.px + dx, ry = p.py + dy;
    const uint32_t lo = ref4(p.ref, p.st, p.W, p.H, rx - 1, ry);  // bytes rx-1 .. rx+2
    const uint32_t hi = ref4(p.ref, p.st, p.W, p.H, rx + 3, ry);  // bytes rx+3 .. rx+6
    const uint32_t up = ref4(p.ref, p.st, p.W, p.H, rx, ry - 1);
    const uint32_t dn = ref4(p.ref, p.st, p.W, p.H, rx, ry + 1);
    const uint32_t m = __builtin_amdgcn_alignbyte(hi, lo, 1);     // bytes rx .. rx+3
    const int lf = (int)(lo & 0xFF), rt = (int)((hi >> 8) & 0xFF);
    int sx = 0, sy = 0, nn = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = byte_of(p.c4, k) - byte_of(m, k);
        const int left = k == 0 ? lf : byte_of(m, k - 1);
        const int right = k == 3 ? rt : byte_of(m, k + 1);
        const int rgx = p.R[right - left + 255];
        const int rgy = p.R[byte_of(dn, k) - byte_of(up, k) + 255];
        sx += e * rgx;
        sy += e * rgy;
        nn += (rgx != 0) + ((rgy != 0) << 16);
    }
    Pass o;
    o.sad = sum16((int)__builtin_amdgcn_sad_u8(p.c4, m, 0u));
    o.sx = sum16(sx);
    o.sy = sum16(sy);
    o.nxy = sum16(nn);
    return o;
}

constexpr int kHx[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
constexpr int kHy[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

__global__ __launch_bounds__(256) void prs8_kernel(const JobDesc *jobs, int n, int total, KParams kp) {
    __shared__ short R[512];  // reciprocal table of Eq. 4-5 (Q.12)
    for (int g = threadIdx.x; g < 511; g += 256) {
        const int m = abs(g - 255);
        const int r = (m == 0 || m < 2 * kp.theta) ? 0 : (16384 + m) / (2 * m);
        R[g] = (short)(g < 255 ? -r : r);
    }
    __syncthreads();
    const int l = lane(), b = l >> 4, j = (l & 15) >> 1, q = l & 1;
    const int S = kp.S;
    const int wave = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const int nwaves = (int)gridDim.x * 4;
    JobCursor c{-1, 0, 0, 0u};
    for (int mb = wave; mb < total; mb += nwaves) {
        seek(c, jobs, n, mb);
        const int k = mb - c.base;
        const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
        const int cl = cls ? (int)ldg8(cls + k) : ME_MB_OPAQUE;
        uint32_t *mv4 = c.ptr<uint32_t>(DWI(mv));            // 4 vectors per MB (out)
        uint32_t *cost4 = c.ptr<uint32_t>(DWI(cost));        // nullable
        uint8_t *iters4 = c.ptr<uint8_t>(DWI(iters));        // nullable
        uint16_t *points4 = c.ptr<uint16_t>(DWI(points));    // nullable
        const uint32_t *mvi = c.ptr<const uint32_t>(DWI(mv_int));
        const uint32_t *mvh = c.ptr<const uint32_t>(DWI(tf));  // the MB's final (half-pel) vector
        const bool lead = (l & 15) == 0;
        if (cl != ME_MB_OPAQUE) {
            // boundary MBs keep their one vector, transparent MBs (0, 0); a
            // class byte above 2 is taken as transparent
            const uint32_t w = cl == ME_MB_BOUNDARY ? ldg32(mvh + k) : 0u;
            if (lead) {
                mv4[4 * k + b] = w;
                if (cost4) cost4[4 * k + b] = 0u;
                if (iters4) iters4[4 * k + b] = 0;
                if (points4) points4[4 * k + b] = 0;
            }
            continue;
        }
        const int wm = c.i32(DWI(wm)), st = c.i32(DWI(stride));
        const int W = c.i32(DWI(width)), H = c.i32(DWI(height));
        const int h = k % wm, v = k / wm;
        const int bx0 = 16 * h + 8 * (b & 1), by0 = 16 * v + 8 * (b >> 1);
        Px p;
        p.ref = c.ptr<const uint8_t>(DWI(ref));
        p.R = R;
        p.st = st;
        p.W = W;
        p.H = H;
        p.px = bx0 + 4 * q;
        p.py = by0 + j;
        p.c4 = ldg32((const uint32_t *)(c.ptr<const uint8_t>(DWI(cur)) + (size_t)p.py * st + p.px));
        const uint32_t w0 = ldg32(mvi + k);
        int dx = ((int)(int16_t)(w0 & 0xFFFF)) >> 1, dy = ((int)(int16_t)(w0 >> 16)) >> 1;
        // admissible box of the 8 x 8 block
        const int lox = kp.unrestricted ? -S : max(-S, -bx0), hix = kp.unrestricted ? S : min(S, W - 8 - bx0);
        const int loy = kp.unrestricted ? -S : max(-S, -by0), hiy = kp.unrestricted ? S : min(S, H - 8 - by0);
        Pass sw = pass8(p, dx, dy);
        int cost = sw.sad, it = 0;
        bool active = kp.k_max > 0;
        // every lane runs every pass (the block reductions need the whole
        // row); a finished block repeats its last position
        for (;;) {
            int tx = dx, ty = dy;
            if (active) {
                const int nx = sw.nxy & 0xFFFF, ny = sw.nxy >> 16;
                const bool zx = nx == 0 || llabs((long long)sw.sx) < (long long)kp.zero_t * nx;
                const bool zy = ny == 0 || llabs((long long)sw.sy) < (long long)kp.zero_t * ny;
                const int sx = zx ? 0 : prs_step(sw.sx / nx, kp.eps, kp.max_step);
                const int sy = zy ? 0 : prs_step(sw.sy / ny, kp.eps, kp.max_step);
                tx = iclamp(dx + sx, lox, hix);
                ty = iclamp(dy + sy, loy, hiy);
                if ((sx == 0 && sy == 0) || (tx == dx && ty == dy)) {
                    active = false;
                    tx = dx;
                    ty = dy;
                } else {
                    ++it;
                }
            }
            if (__ballot(active) == 0ull) break;
            const Pass s2 = pass8(p, tx, ty);
            if (active) {
                if (s2.sad < cost) {
                    dx = tx;
                    dy = ty;
                    cost = s2.sad;
                    sw = s2;
                    active = it < kp.k_max;
                } else {
                    active = false;
                }
            }
        }
        int pts = it;
        int hx = 2 * dx, hy = 2 * dy;
        if (kp.half_pel) {
            // 3 x 6 neighbourhood: rows ry-1 .. ry+1, columns rx-1 .. rx+4
            const int rx = p.px + dx, ry = p.py + dy;
            int nb[3][6];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const uint32_t lo = ref4(p.ref, st, W, H, rx - 1, ry - 1 + r);
                const uint32_t hi2 = ref4(p.ref, st, W, H, rx + 3, ry - 1 + r);
#pragma unroll
                for (int t = 0; t < 4; ++t) nb[r][t] = byte_of(lo, t);
                nb[r][4] = byte_of(hi2, 0);
                nb[r][5] = byte_of(hi2, 1);
            }
            int part[8];
            bool feas[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int ox = kHx[o], oy = kHy[o];
                const int fx = ox & 1, fy = oy & 1;
                const int oxr = ox < 0 ? 0 : 1, oyr = oy < 0 ? 0 : 1;  // neighbourhood origin of A
                const int qx = 2 * dx + ox, qy = 2 * dy + oy;
                const int ix = dx + (ox < 0 ? -1 : 0), iy = dy + (oy < 0 ? -1 : 0);
                feas[o] = abs(qx) <= 2 * S && abs(qy) <= 2 * S &&
                          (kp.unrestricted || (bx0 + ix >= 0 && bx0 + ix + 7 + fx <= W - 1 && by0 + iy >= 0 &&
                                               by0 + iy + 7 + fy <= H - 1));
                int s = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int A = nb[oyr][oxr + t], B = nb[oyr][oxr + t + 1];
                    const int Cc = nb[oyr + 1][oxr + t], D = nb[oyr + 1][oxr + t + 1];
                    const int pr = (fx && fy) ? ((A + B + Cc + D + 2) >> 2)
                                              : fx ? ((A + B + 1) >> 1) : fy ? ((A + Cc + 1) >> 1) : A;
                    s += abs(byte_of(p.c4, t) - pr);
                }
                part[o] = s;
            }
            int bhx = hx, bhy = hy;
#pragma unroll
            for (int o = 0; o < 8; o += 2) {
                const int pk = sum16(part[o] | (part[o + 1] << 16));
                const int t0 = pk & 0xFFFF, t1 = (int)((uint32_t)pk >> 16);
                if (feas[o]) {
                    ++pts;
                    if (t0 < cost) {
                        cost = t0;
                        bhx = 2 * dx + kHx[o];
                        bhy = 2 * dy + kHy[o];
                    }
                }
                if (feas[o + 1]) {
                    ++pts;
                    if (t1 < cost) {
                        cost = t1;
                        bhx = 2 * dx + kHx[o + 1];
                        bhy = 2 * dy + kHy[o + 1];
                    }
                }
            }
            hx = bhx;
            hy = bhy;
        }
        if (lead) {
            mv4[4 * k + b] = (uint32_t)(uint16_t)hx | ((uint32_t)(uint16_t)hy << 16);
            if (cost4) cost4[4 * k + b] = (uint32_t)cost;
            if (iters4) iters4[4 * k + b] = (uint8_t)it;
            if (points4) points4[4 * k + b] = (uint16_t)pts;
        }
    }
}

}  // namespace

hipError_t launch_prs8(const JobDesc *jobs, int n, int total_mbs, const KParams &kp, hipStream_t s,
                       const KernelTimer *t) {
    if (total_mbs <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int blocks = std::max(1, std::min((total_mbs + 3) / 4, cus * 8));
    timer_mark(t, true, s);
    hipLaunchKernelGGL(prs8_kernel, dim3(blocks), dim3(256), 0, s, jobs, n, total_mbs, kp);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

}  // namespace me

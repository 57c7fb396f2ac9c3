// MB classification from the binary alpha plane (Section 1) and motion
// compensation + squared error (Section 4).  Both stream each pixel once and
// are bound by the memory system.  Layout: a few lanes per MB (four for
// classification, eight for MC), each lane whole 16-pixel rows, per-MB sums
// DPP reductions over those lanes (no atomics); the job of a wave's MBs is a
// wave-uniform cursor, so descriptor fields live in scalar registers.
#include "flat_kernels.h"

namespace me {

namespace {

// n words of value v from p: 16-byte stores over the whole quads when p is
// 16-byte aligned, single words for the rest.
__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v) {
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t done = 0;
    if (((uintptr_t)p & 15u) == 0) {
        typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
        u32x4v *q = (u32x4v *)p;
        const size_t nq = n / 4;
        for (size_t i = i0; i < nq; i += stride) q[i] = u32x4v{v, v, v, v};
        done = nq * 4;
    }
    for (size_t i = done + i0; i < n; i += stride) p[i] = v;
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

// 16 bytes of global memory at a 4-byte aligned address.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 __attribute__((aligned(4))) u32x4_a4;
__device__ __forceinline__ u32x4 ld16(const uint8_t *p) {
    return *(const __attribute__((address_space(1))) u32x4_a4 *)p;
}
__device__ __forceinline__ void st16(uint8_t *p, const uint32_t (&v)[4]) {
    *(__attribute__((address_space(1))) u32x4_a4 *)p = u32x4{v[0], v[1], v[2], v[3]};
}
__device__ __forceinline__ void st32(uint32_t *p, uint32_t v) { *(__attribute__((address_space(1))) uint32_t *)p = v; }
__device__ __forceinline__ void st8(uint8_t *p, uint8_t v) { *(__attribute__((address_space(1))) uint8_t *)p = v; }

// The flat MB range is cut into units of 64 / LPM consecutive MBs (LPM
// lanes per MB), one unit per wave per iteration; a block strides its four
// waves over `chunk` consecutive units.  body(c, k, mb, on) runs once per
// job a unit touches (nearly always one), `on` set in the lanes whose MB
// belongs to the cursor's job (k: that MB's index within the job, else 0).
template <int LPM, class Body>
__device__ __forceinline__ void for_units(const JobDesc *jobs, int n, int total, int chunk, Body &&body) {
    constexpr int PER = 64 / LPM;
    const int nu = (total + PER - 1) / PER;
    const int u0 = (int)blockIdx.x * chunk;
    const int uend = min(u0 + chunk, nu);
    JobCursor c{-1, 0, 0, 0u};
    for (int u = u0 + uni((int)threadIdx.x >> 6); u < uend; u += 4) {
        const int m0 = u * PER, mlast = min(m0 + PER, total) - 1;
        const int mb = m0 + lane() / LPM;
        seek(c, jobs, n, m0);
        for (;;) {
            const bool on = mb <= mlast && mb >= c.base && mb < c.end;
            body(c, on ? mb - c.base : 0, mb, on);
            if (mlast < c.end) break;
            seek(c, jobs, n, c.end);
        }
    }
}

// Sums over groups of 4 and of 8 lanes, result in every lane of the group.
__device__ __forceinline__ int sum4(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    return v;
}
__device__ __forceinline__ int sum8(int v) {
    v = sum4(v);
    return v + __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
}

__device__ __forceinline__ uint32_t nz16v(const u32x4 a) {
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
    return nz16(w);
}

// n = number of pixels with alpha != 0 -> transparent (0), opaque (256),
// boundary, written to the job's class array; BAB word w = rows 2w, 2w+1
// with column i at bit (row&1)*16 + i.  Jobs without alpha or without a
// class array (rectangular frames) are skipped.  LPM lanes per MB (2 or
// 4): lane t reads rows R t .. R t + R - 1 (R = 16 / LPM, all loads in
// flight together) and writes BAB words R t / 2 .. R (t + 1) / 2 - 1.  The
// grid also clears z0[0, n0) and z1[0, n1).
constexpr int kClassifyLanes = 2;
template <int LPM>
__global__ __launch_bounds__(256) void classify_kernel(const JobDesc *jobs, int n, int total, int chunk, uint32_t *z0,
                                                       size_t n0, uint32_t *z1, size_t n1) {
    static_assert(LPM == 2 || LPM == 4, "two or four lanes per MB");
    constexpr int R = 16 / LPM;
    if (n0 + n1 > 0) {
        const size_t stride = (size_t)gridDim.x * blockDim.x;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += stride) st32(z0 + i, 0u);
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += stride) st32(z1 + i, 0u);
    }
    const int t = lane() & (LPM - 1);
    for_units<LPM>(jobs, n, total, chunk, [&](const JobCursor &c, int k, int, bool on) {
        const uint8_t *alpha = c.ptr<const uint8_t>(DWI(cur_a));
        uint8_t *cls = c.ptr<uint8_t>(DWI(cls));
        if (!alpha || !cls) return;
        uint32_t *bab = c.ptr<uint32_t>(DWI(out_u32));
        const int wm = c.i32(DWI(wm)), st = c.i32(DWI(stride));
        const int h = k % wm, v = k / wm;
        const uint8_t *row = alpha + (size_t)(16 * v + R * t) * st + 16 * h;
        u32x4 a[R];
#pragma unroll
        for (int i = 0; i < R; ++i) a[i] = ld16(row + (size_t)i * st);
        uint32_t bits[R];
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            bits[i] = nz16v(a[i]);
            cnt += __builtin_popcount(bits[i]);
        }
        const int tot = LPM == 4 ? sum4(cnt) : cnt + __builtin_amdgcn_update_dpp(0, cnt, 0xB1, 0xF, 0xF, true);
        if (on) {
            if (bab) {
#pragma unroll
                for (int i = 0; i < R / 2; ++i)
                    st32(bab + (size_t)k * 8 + (R / 2) * t + i, bits[2 * i] | (bits[2 * i + 1] << 16));
            }
            if (t == 0)
                st8(cls + k, (uint8_t)(tot == 0 ? ME_MB_TRANSPARENT : (tot == 256 ? ME_MB_OPAQUE : ME_MB_BOUNDARY)));
        }
    });
}

// (x + y + 1) >> 1 in each of the four bytes: x + y = 2 (x & y) + (x ^ y),
// so the rounded-up half is (x | y) - ((x ^ y) >> 1), with no borrow
// between bytes.
__device__ __forceinline__ uint32_t avg2_u8x4(uint32_t x, uint32_t y) {
    return (x | y) - ((x ^ y) >> 1 & 0x7F7F7F7Fu);
}

// (a + b + c + d + 2) >> 2 in each of the four bytes: the even and the odd
// bytes summed in 16-bit fields (at most 1022, no carry between fields).
__device__ __forceinline__ uint32_t avg4_u8x4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    constexpr uint32_t M = 0x00FF00FFu;
    const uint32_t ev = (a & M) + (b & M) + (c & M) + (d & M) + 0x00020002u;
    const uint32_t od = (a >> 8 & M) + (b >> 8 & M) + (c >> 8 & M) + (d >> 8 & M) + 0x00020002u;
    return (ev >> 2 & M) | (od << 6 & ~M);
}

// One row of the prediction from reference rows a (at the row's own vertical
// offset) and c (the row below), 20 bytes each from the integer column:
// MPEG-4 bilinear interpolation with rounding control 0, four pixels per
// word.  The right neighbours of a word's pixels are the bytes one further
// along the row (the word and the next one, aligned by one byte).
__device__ __forceinline__ void bilinear_row(const uint32_t (&a)[5], const uint32_t (&c)[5], int fx, int fy,
                                             uint32_t (&out)[4]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t ar = __builtin_amdgcn_alignbyte(a[w + 1], a[w], 1);
        const uint32_t cr = __builtin_amdgcn_alignbyte(c[w + 1], c[w], 1);
        out[w] = fx ? (fy ? avg4_u8x4(a[w], ar, c[w], cr) : avg2_u8x4(a[w], ar)) : (fy ? avg2_u8x4(a[w], c[w]) : a[w]);
    }
}

// Rows y .. y+R-1 (16 pixels from column x) of the prediction by the
// half-pel vector (hx, hy): reference rows y+iy .. y+iy+R, coordinates
// clamped to the frame.  The last row is used only for a vertical half-pel;
// it is read when some lane of the wave has one (a branch per lane would wait
// for each of its loads on its own).
template <int R>
__device__ __forceinline__ void predict_rows(const uint8_t *ref, int st, int W, int H, int x, int y, int hx, int hy,
                                             uint32_t (&p)[R][4]) {
    const int ix = hx >> 1, iy = hy >> 1, fx = hx & 1, fy = hy & 1;
    uint32_t r[R + 1][5];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const uint8_t *row = ref + (size_t)iclamp(y + iy + t, 0, H - 1) * st;
#pragma unroll
        for (int w = 0; w < 5; ++w) r[t][w] = ld4_clamped(row, x + ix + 4 * w, W);
    }
    // the loads of the last row in one block, their byte permutes after it
    uint32_t raw[5] = {0u, 0u, 0u, 0u, 0u}, sel[5];
    const uint8_t *rowl = ref + (size_t)iclamp(y + iy + R, 0, H - 1) * st;
#pragma unroll
    for (int w = 0; w < 5; ++w) {
        const int xx = x + ix + 4 * w, xc = iclamp(xx, 0, W - 4);
        sel[w] = (uint32_t)(iclamp(xx, 0, W - 1) - xc) | ((uint32_t)(iclamp(xx + 1, 0, W - 1) - xc) << 8) |
                 ((uint32_t)(iclamp(xx + 2, 0, W - 1) - xc) << 16) | ((uint32_t)(iclamp(xx + 3, 0, W - 1) - xc) << 24);
        raw[w] = (uint32_t)xc;
    }
    if (__ballot(fy) != 0) {
#pragma unroll
        for (int w = 0; w < 5; ++w) raw[w] = ld4(rowl + raw[w]);
    }
#pragma unroll
    for (int w = 0; w < 5; ++w) r[R][w] = __builtin_amdgcn_perm(raw[w], raw[w], sel[w]);
#pragma unroll
    for (int t = 0; t < R; ++t) bilinear_row(r[t], r[t + 1], fx, fy, p[t]);
}

// Squared error of one 16-pixel row over the pixels whose alpha is set: with
// c, p masked to those bytes (mask bit i -> byte i all ones), the sum of
// (c - p)^2 is c.c + p.p - 2 c.p, each a 4-byte dot product, exact in 32 bits.
__device__ __forceinline__ int row_sse(const u32x4 cur, const uint32_t (&p)[4], uint32_t in) {
    const uint32_t c[4] = {cur.x, cur.y, cur.z, cur.w};
    uint32_t sq = 0u, cross = 0u;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t m = (((in >> (4 * w)) & 0xFu) * 0x00204081u & 0x01010101u) * 0xFFu;
        const uint32_t cm = c[w] & m, pm = p[w] & m;
        sq = __builtin_amdgcn_udot4(cm, cm, sq, false);
        sq = __builtin_amdgcn_udot4(pm, pm, sq, false);
        cross = __builtin_amdgcn_udot4(cm, pm, cross, false);
    }
    return (int)(sq - 2u * cross);
}

// Prediction of MB k by its half-pel vector (transparent: zero vector),
// written to out_u8 when set; per-MB SSE and pixel count over the mask to
// part[2 * mb], part[2 * mb + 1].  Eight lanes per MB, lane t predicts rows
// 2t and 2t+1 (three reference rows at most).  A class byte above 2 raises
// ST_BAD_CLASS (the MB is still predicted by its vector).
// FOUR: the job's mv holds four vectors per MB (8 x 8 blocks in raster
// order); lane t's rows belong to the top or bottom pair, its left 8 pixels
// to the first block of the pair and its right 8 to the second.
// One MB's prediction by eight lanes: lane t takes rows 2t and 2t+1 of the
// current rows, the alpha mask and the prediction (by the MB's vector, or
// per 8 x 8 column half by its two block vectors when FOUR), stores the
// prediction when `store`, and returns its part of the MB's SSE and pixel
// count (sum over the eight lanes for the MB's totals).
template <bool FOUR>
__device__ __forceinline__ void mc_mb(const JobCursor &c, int k, int cl, int t, bool store, int &sse, int &cnt) {
    const uint8_t *cur = c.ptr<const uint8_t>(DWI(cur));
    const uint8_t *ref = c.ptr<const uint8_t>(DWI(ref));
    const uint8_t *alpha = c.ptr<const uint8_t>(DWI(cur_a));
    const uint32_t *mv = c.ptr<const uint32_t>(DWI(mv));
    uint8_t *out = c.ptr<uint8_t>(DWI(out_u8));
    const int W = c.i32(DWI(width)), H = c.i32(DWI(height)), st = c.i32(DWI(stride)), wm = c.i32(DWI(wm));
    const int h = k % wm, v = k / wm;
    const int x = 16 * h, y = 16 * v + 2 * t;
    const uint32_t w = FOUR ? ldg32(mv + 4 * k + 2 * (t >> 2)) : ldg32(mv + k);
    const size_t o0 = (size_t)y * st + x, o1 = o0 + st;
    // the alpha rows are loaded unconditionally (the current rows again when
    // there is no alpha plane) and used last, so that all loads are in flight
    // together: the scheduler would otherwise wait for each alpha row before
    // the next one's load
    const uint8_t *ap = alpha ? alpha : cur;
    const u32x4 c0 = ld16(cur + o0), c1 = ld16(cur + o1), a0 = ld16(ap + o0), a1 = ld16(ap + o1);
    __builtin_amdgcn_sched_barrier(0);
    int hx = 0, hy = 0;
    if (cl != ME_MB_TRANSPARENT) {
        hx = (int)(int16_t)(w & 0xFFFF);
        hy = (int)(int16_t)(w >> 16);
    }
    uint32_t p[2][4];
    predict_rows<2>(ref, st, W, H, x, y, hx, hy, p);
    if constexpr (FOUR) {
        // the right 8 pixels by the pair's second block vector
        const uint32_t w2 = ldg32(mv + 4 * k + 2 * (t >> 2) + 1);
        int hx2 = 0, hy2 = 0;
        if (cl != ME_MB_TRANSPARENT) {
            hx2 = (int)(int16_t)(w2 & 0xFFFF);
            hy2 = (int)(int16_t)(w2 >> 16);
        }
        uint32_t q[2][4];
        predict_rows<2>(ref, st, W, H, x, y, hx2, hy2, q);
        p[0][2] = q[0][2];
        p[0][3] = q[0][3];
        p[1][2] = q[1][2];
        p[1][3] = q[1][3];
    }
    if (store && out) {
        st16(out + o0, p[0]);
        st16(out + o1, p[1]);
    }
    const uint32_t in0 = alpha ? nz16v(a0) : 0xFFFFu, in1 = alpha ? nz16v(a1) : 0xFFFFu;
    sse = row_sse(c0, p[0], in0) + row_sse(c1, p[1], in1);
    cnt = __builtin_popcount(in0) + __builtin_popcount(in1);
}

// Section 4's prediction and squared error: every MB predicted by its
// half-pel vector (transparent MBs by (0, 0)) from the reference frame,
// written to out_u8 when set; per-MB SSE and pixel count over the mask to
// part[2 mb], part[2 mb + 1] for the per-job reduction.  Eight lanes per MB.
template <bool FOUR>
__global__ __launch_bounds__(256) void mc_kernel(const JobDesc *jobs, int n, int total, int chunk, uint32_t *part,
                                                 uint32_t *status) {
    const int t = lane() & 7;
    for_units<8>(jobs, n, total, chunk, [&](const JobCursor &c, int k, int mb, bool on) {
        const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
        const uint32_t *mv = c.ptr<const uint32_t>(DWI(mv));
        // the class byte is read unconditionally (from the vector array when
        // there is no class array) so that it shares one round trip with the
        // vector and the current rows
        const uint32_t cb = ldg8(cls ? cls + k : (const uint8_t *)(mv + k));
        const int cl = cls ? (int)cb : ME_MB_OPAQUE;
        if (on && t == 0 && cl > ME_MB_BOUNDARY) atomicOr(status, ST_BAD_CLASS);
        int sse, cnt;
        mc_mb<FOUR>(c, k, cl, t, on, sse, cnt);
        sse = sum8(sse);
        cnt = sum8(cnt);
        if (on && t == 0) {
            st32(part + 2 * (size_t)mb, (uint32_t)sse);
            st32(part + 2 * (size_t)mb + 1, (uint32_t)cnt);
        }
    });
}

__device__ __forceinline__ void st64(uint32_t *p, unsigned long long v) {
    *(__attribute__((address_space(1))) unsigned long long *)p = v;
}

// SSE and pixel count of MB k predicted by the half-pel vector word w, by
// four lanes: lane t takes rows 4t .. 4t+3.
__device__ __forceinline__ void mc_sums_mb(const JobCursor &c, int k, uint32_t w, int t, int &sse, int &cnt) {
    const uint8_t *cur = c.ptr<const uint8_t>(DWI(cur));
    const uint8_t *ref = c.ptr<const uint8_t>(DWI(ref));
    const uint8_t *alpha = c.ptr<const uint8_t>(DWI(cur_a));
    const int W = c.i32(DWI(width)), H = c.i32(DWI(height)), st = c.i32(DWI(stride)), wm = c.i32(DWI(wm));
    const int x = 16 * (k % wm), y = 16 * (k / wm) + 4 * t;
    // all loads of the current and alpha rows before any use (alpha rows
    // unconditionally, the current rows again when there is no alpha plane)
    const uint8_t *ap = alpha ? alpha : cur;
    u32x4 cr[4], ar[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cr[i] = ld16(cur + (size_t)(y + i) * st + x);
        ar[i] = ld16(ap + (size_t)(y + i) * st + x);
    }
    __builtin_amdgcn_sched_barrier(0);
    uint32_t p[4][4];
    predict_rows<4>(ref, st, W, H, x, y, (int)(int16_t)(w & 0xFFFF), (int)(int16_t)(w >> 16), p);
    sse = 0;
    cnt = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t in = alpha ? nz16v(ar[i]) : 0xFFFFu;
        sse += row_sse(cr[i], p[i], in);
        cnt += __builtin_popcount(in);
    }
}

// The same sums without a prediction frame.  A transparent MB has no pixel
// with alpha != 0 (its class is the classification of the current alpha),
// so its SSE and pixel count are zero whatever its prediction: such MBs cost
// one class byte (and a zero partial).  One lane per MB reads the class and
// the vector of 64 consecutive MBs in one round trip; the other MBs are
// compacted in LDS (wave-private) with their vectors and predicted four
// lanes per MB, 16 MBs per round.
// ACC: no partials; each wave adds its totals for the job to acc[2 j],
// acc[2 j + 1] atomically (an SSE total of 64 MBs fits 32 bits).
template <bool ACC>
__global__ __launch_bounds__(256) void mc_sums_kernel(const JobDesc *jobs, int n, int total, int chunk,
                                                      uint32_t *part, unsigned long long *acc, uint32_t *status) {
    __shared__ int list_k[4][64];
    __shared__ uint32_t list_w[4][64];
    int *lk = list_k[threadIdx.x >> 6];
    uint32_t *lw = list_w[threadIdx.x >> 6];
    const int t = lane() & 3, g = lane() >> 2;
    for_units<1>(jobs, n, total, chunk, [&](const JobCursor &c, int k, int mb, bool on) {
        const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
        const uint32_t *mv = c.ptr<const uint32_t>(DWI(mv));
        int cl = ME_MB_OPAQUE;
        uint32_t w = 0u;
        if (on) {
            if (cls) cl = (int)ldg8(cls + k);
            w = ldg32(mv + k);
        }
        if (on && cl > ME_MB_BOUNDARY) atomicOr(status, ST_BAD_CLASS);
        const bool act = on && cl != ME_MB_TRANSPARENT;
        if (!ACC && on && !act) st64(part + 2 * (size_t)mb, 0ull);
        const unsigned long long m = __ballot(act);
        const int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // the wave's previous reads of the list are done before it is rewritten
        __builtin_amdgcn_wave_barrier();
        if (act) {
            lk[pos] = k;
            lw[pos] = w;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cnt_act = __popcll(m);
        uint32_t job_sse = 0u, job_cnt = 0u;
        for (int i = 0; i < cnt_act; i += 16) {
            const bool live = i + g < cnt_act;
            const int e = live ? i + g : i;
            const int kk = lk[e];
            int sse, cnt;
            mc_sums_mb(c, kk, lw[e], t, sse, cnt);
            sse = sum4(sse);
            cnt = sum4(cnt);
            if (!ACC && live && t == 0)
                st64(part + 2 * ((size_t)c.base + kk),
                     (unsigned long long)(uint32_t)sse | ((unsigned long long)(uint32_t)cnt << 32));
            if (ACC && live && t == 0) {
                job_sse += (uint32_t)sse;
                job_cnt += (uint32_t)cnt;
            }
        }
        if (ACC && cnt_act > 0) {
            for (int o = 32; o >= 1; o >>= 1) {
                job_sse += __shfl_xor(job_sse, o, 64);
                job_cnt += __shfl_xor(job_cnt, o, 64);
            }
            if (lane() == 0) {
                atomicAdd(acc + 2 * c.j, (unsigned long long)job_sse);
                atomicAdd(acc + 2 * c.j + 1, (unsigned long long)job_cnt);
            }
        }
    });
}

// Per job: the exact 64-bit sums of its MBs' SSE and pixel counts.  One
// block per job, 64 to 1024 threads (about four MBs per thread); an MB's
// (SSE, count) pair is one 8-byte load, four loads in flight per thread.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void mc_reduce_kernel(const JobDesc *jobs, const uint32_t *part,
                                                                   unsigned long long *acc) {
    __shared__ unsigned long long red[2][kReduceThreads / 64];
    const JobDesc &J = jobs[blockIdx.x];
    const int nmb = J.wm * J.hm, nt = (int)blockDim.x;
    const unsigned long long *p = (const unsigned long long *)(part + 2 * (size_t)J.mb_base);
    unsigned long long s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    int i = threadIdx.x;
    for (; i + 3 * nt < nmb; i += 4 * nt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long w = p[i + u * nt];
            s[u] += (uint32_t)w;
            c[u] += w >> 32;
        }
    }
    for (; i < nmb; i += nt) {
        const unsigned long long w = p[i];
        s[0] += (uint32_t)w;
        c[0] += w >> 32;
    }
    unsigned long long ss = s[0] + s[1] + s[2] + s[3], cc = c[0] + c[1] + c[2] + c[3];
    for (int o = 32; o >= 1; o >>= 1) {
        ss += __shfl_xor(ss, o, 64);
        cc += __shfl_xor(cc, o, 64);
    }
    if (lane() == 0) {
        red[0][threadIdx.x >> 6] = ss;
        red[1][threadIdx.x >> 6] = cc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ts = 0, tc = 0;
        for (int w = 0; w < nt / 64; ++w) {
            ts += red[0][w];
            tc += red[1][w];
        }
        acc[2 * blockIdx.x] = ts;
        acc[2 * blockIdx.x + 1] = tc;
    }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 1023) / 1024;  // about four words per thread
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Units (runs of consecutive MBs) per block so that a flat grid has about
// per_cu blocks per CU.
int flat_chunk(int total_units, int per_cu) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    long long blocks = (long long)(cus > 0 ? cus : 256) * per_cu;
    long long c = (total_units + blocks - 1) / blocks;
    return (int)(c < 1 ? 1 : c);
}

hipError_t launch_classify_zeroing(const JobDesc *jobs, int n, int total_mbs, uint32_t *z0, size_t n0, uint32_t *z1,
                                   size_t n1, hipStream_t s, const KernelTimer *t, int per_cu) {
    if (total_mbs <= 0) return hipSuccess;
    constexpr int per_unit = 64 / kClassifyLanes;
    const int nu = (total_mbs + per_unit - 1) / per_unit;
    const int chunk = (flat_chunk(nu, per_cu) + 3) / 4 * 4;
    timer_mark(t, true, s);
    hipLaunchKernelGGL(classify_kernel<kClassifyLanes>, dim3((nu + chunk - 1) / chunk), dim3(256), 0, s, jobs, n,
                       total_mbs, chunk, z0, n0, z1, n1);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

hipError_t launch_classify(const JobDesc *jobs, int n, int total_mbs, hipStream_t s, const KernelTimer *t,
                           int per_cu) {
    return launch_classify_zeroing(jobs, n, total_mbs, nullptr, 0, nullptr, 0, s, t, per_cu);
}

size_t mc_scratch(int total_mbs) { return (size_t)total_mbs * 8; }

hipError_t launch_mc(const JobDesc *jobs, int n, int total_mbs, uint32_t *part, unsigned long long *acc,
                     uint32_t *status, hipStream_t s, const KernelTimer *t, int per_cu, bool four, bool sums_only) {
    if (total_mbs <= 0) return hipSuccess;
    const int nu = (total_mbs + 7) / 8;
    const int chunk = (flat_chunk(nu, per_cu) + 3) / 4 * 4;
    timer_mark(t, true, s);
    if (sums_only && !four) {
        const int nu64 = (total_mbs + 63) / 64;
        const int chunk64 = (flat_chunk(nu64, per_cu) + 3) / 4 * 4;
        hipLaunchKernelGGL(mc_sums_kernel<false>, dim3((nu64 + chunk64 - 1) / chunk64), dim3(256), 0, s, jobs, n,
                           total_mbs, chunk64, part, nullptr, status);
    } else if (four)
        hipLaunchKernelGGL(mc_kernel<true>, dim3((nu + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs, chunk,
                           part, status);
    else
        hipLaunchKernelGGL(mc_kernel<false>, dim3((nu + chunk - 1) / chunk), dim3(256), 0, s, jobs, n, total_mbs,
                           chunk, part, status);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    if (e != hipSuccess) return e;
    int th = 64;
    while (th < kReduceThreads && 4 * th < total_mbs / n) th <<= 1;
    hipLaunchKernelGGL(mc_reduce_kernel, dim3(n), dim3(th), 0, s, jobs, part, acc);
    return hipGetLastError();
}

hipError_t launch_mc_sums_acc(const JobDesc *jobs, int n, int total_mbs, unsigned long long *acc, uint32_t *status,
                              hipStream_t s, const KernelTimer *t, int per_cu) {
    if (total_mbs <= 0) return hipSuccess;
    const int nu64 = (total_mbs + 63) / 64;
    const int chunk64 = (flat_chunk(nu64, per_cu) + 3) / 4 * 4;
    timer_mark(t, true, s);
    hipLaunchKernelGGL(mc_sums_kernel<true>, dim3((nu64 + chunk64 - 1) / chunk64), dim3(256), 0, s, jobs, n,
                       total_mbs, chunk64, nullptr, acc, status);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

}  // namespace me

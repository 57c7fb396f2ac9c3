// Learned motion-vector proposal: a 3-layer convolutional network that
// predicts a starting vector for the pel-recursive search of an opaque MB
// (the paper's recursion starts from the block-recursive winner, Section
// 3.2; the learned start and its 5 % fallback are additions of this
// library).  Per MB:
//   input   24x24x2 at window scale f (2 or 4): the current MB box-averaged
//           f x f ((16/f)^2, centred in a zero canvas) and the frame-clamped
//           reference window [-(12f-8), 12f+8) box-averaged f x f; an f x f
//           sum s maps to (s - 128 f^2) / (128 f^2) in bfloat16 (f = 2: the
//           window [-16, 32), (s - 512) / 512)
//   conv1   3x3, 2 -> 32, stride 1, pad 1, ReLU   -> 24x24x32 (bf16)
//   conv2   3x3, 32 -> 32, stride 2, pad 1, ReLU  -> 12x12x32 (bf16)
//   conv3   3x3, 32 -> 2, stride 2, pad 1         -> 6x6x2 (fp32)
//   p       mean of conv3 over its 36 positions: the predicted full-pel
//           vector; seed = 2 * clamp(rint(p), -w, w) half-pel, w = 12f - 8
// One workgroup (4 waves) takes one MB at a time and keeps every activation
// in LDS (NHWC, channels innermost).  The convolutions and the two large
// gradient products are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (bf16
// operands, fp32 accumulation); the conv3 gradients, the bias gradients and
// the ReLU masks are VALU work.  Training accumulates each workgroup's
// gradient over its MBs in registers, writes one partial per workgroup, and
// a second kernel sums the partials in a fixed order and applies momentum
// SGD, so a step is deterministic for a given launch shape.
//
// MFMA operand layout (16x16x32): lane l holds A row l%16 and B column l%16
// at k = 8*(l/16) .. +7; the result holds column l%16, rows 4*(l/16) .. +3.
#include <type_traits>

#include "me_internal.h"

namespace me {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ f32x4 mfma(const u16x8 &a, const u16x8 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

// The bf16 copies of master parameter i: W1, W2 (and W2 transposed to
// [tap][ci][co] for the input-gradient product), W3.
__device__ __forceinline__ void net_refresh_one(float w, uint16_t *wb, int i) {
    const uint16_t b = (uint16_t)bf16_bits(w);
    if (i < kNetOB1) {
        wb[i] = b;
    } else if (i >= kNetOW2 && i < kNetOB2) {
        const int q = i - kNetOW2, co = q / 288, tap = (q % 288) >> 5, ci = q & 31;
        wb[576 + q] = b;
        wb[576 + 9216 + (tap * 32 + ci) * 32 + co] = b;
    } else if (i >= kNetOW3 && i < kNetOB3) {
        wb[576 + 2 * 9216 + (i - kNetOW3)] = b;
    }
}

__device__ __forceinline__ float relu(float x) { return x > 0.f ? x : 0.f; }

__device__ __forceinline__ u16x8 ld16(const uint16_t *p) { return *(const u16x8 *)p; }
__device__ __forceinline__ u16x8 zero8() { return u16x8{0, 0, 0, 0, 0, 0, 0, 0}; }

// 16-byte aligned arrays: MFMA operands are read as 128-bit LDS loads
struct NetLds {
    alignas(16) uint16_t x0[576 * 2];   // input, [pixel][channel]
    alignas(16) uint16_t a1[576 * 32];  // conv1 output
    alignas(16) uint16_t a2[144 * 32];  // conv2 output
    alignas(16) float red[4][64];       // cross-wave reductions
    alignas(16) float bias[64];         // conv1 and conv2 biases
    float pv[2];                        // prediction of the current MB
};
struct NetLdsTrain : NetLds {
    alignas(16) uint16_t d2[144 * 32];  // conv2 pre-activation gradient (bf16)
    alignas(16) uint16_t d1[576 * 32];  // conv1 pre-activation gradient (bf16)
    alignas(16) float gb[kThreads];
};
static_assert(sizeof(NetLds) % 16 == 0 && sizeof(NetLdsTrain) % 16 == 0, "LDS layout");

// --------------------------------------------------------------- stages
// Input of MB (x0, y0): 576 reference-window values and 64 current values.
// The pixels are loaded into registers first (`issue_input`, up to three
// positions per thread) and summed into LDS later (`write_input`), so the
// next MB's loads can fly while the current MB is computed.
struct InPix {
    uint32_t r[3][4];  // scale 2: the 2x2 reference pixels of each position; scale 4: its four 4-byte rows
    uint32_t c[3][4];  // the current pixels of the position's rows (centre positions only)
};

// The fields of a job the network reads, as wave-uniform values (frame
// pointers then address global memory directly).
struct InJob {
    const uint8_t *cur, *ref;
    int W, H, st, wm, hm;
};

__device__ __forceinline__ uint32_t dword_of(const JobDesc *J, int i) {
    return (uint32_t)uni((int)ldg32((const uint32_t *)J + i));
}

__device__ __forceinline__ InJob in_job(const JobDesc *J) {
    const int o_cur = (int)(offsetof(JobDesc, cur) / 4), o_ref = (int)(offsetof(JobDesc, ref) / 4);
    const int o_w = (int)(offsetof(JobDesc, width) / 4);
    InJob j;
    j.cur = (const uint8_t *)(uintptr_t)((unsigned long long)dword_of(J, o_cur) |
                                         ((unsigned long long)dword_of(J, o_cur + 1) << 32));
    j.ref = (const uint8_t *)(uintptr_t)((unsigned long long)dword_of(J, o_ref) |
                                         ((unsigned long long)dword_of(J, o_ref + 1) << 32));
    j.W = (int)dword_of(J, o_w);
    j.H = (int)dword_of(J, o_w + 1);
    j.st = (int)dword_of(J, o_w + 2);
    j.wm = (int)dword_of(J, o_w + 3);
    j.hm = (int)dword_of(J, o_w + 4);
    return j;
}

// Window scale f (2 or 4): canvas position (y, x) averages the f x f reference
// pixels at rows/columns 12f - 8 before the MB plus f (y, x); the current MB
// covers the centre (16/f)^2 positions.
__device__ __forceinline__ void issue_input(InPix &v, const InJob &J, int x0, int y0, int scale) {
    const int W = J.W, H = J.H, st = J.st;
    if (scale == 4) {
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            const int q = threadIdx.x + kThreads * sl;
            const int y = q / 24, x = q - (q / 24) * 24;
            const bool in = q < 576;
            // clamped coordinates: every address is in the frame
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v.r[sl][r] = in ? ld4_clamped(J.ref + (size_t)iclamp(y0 - 40 + 4 * y + r, 0, H - 1) * st,
                                              x0 - 40 + 4 * x, W)
                                : 0u;
#pragma unroll
            for (int r = 0; r < 4; ++r) v.c[sl][r] = 0u;
            if (in && y >= 10 && y < 14 && x >= 10 && x < 14) {
                const uint8_t *c = J.cur + (size_t)(y0 + 4 * (y - 10)) * st + x0 + 4 * (x - 10);
#pragma unroll
                for (int r = 0; r < 4; ++r) v.c[sl][r] = ldg32((const uint32_t *)(c + (size_t)r * st));
            }
        }
        return;
    }
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
        const int q = threadIdx.x + kThreads * sl;
        const int y = q / 24, x = q - (q / 24) * 24;
        const int ya = iclamp(y0 - 16 + 2 * y, 0, H - 1), yb = iclamp(y0 - 15 + 2 * y, 0, H - 1);
        const int xa = iclamp(x0 - 16 + 2 * x, 0, W - 1), xb = iclamp(x0 - 15 + 2 * x, 0, W - 1);
        const bool in = q < 576;
        // clamped coordinates: every address is in the frame
        v.r[sl][0] = in ? ldg8(J.ref + (size_t)ya * st + xa) : 0u;
        v.r[sl][1] = in ? ldg8(J.ref + (size_t)ya * st + xb) : 0u;
        v.r[sl][2] = in ? ldg8(J.ref + (size_t)yb * st + xa) : 0u;
        v.r[sl][3] = in ? ldg8(J.ref + (size_t)yb * st + xb) : 0u;
        v.c[sl][0] = v.c[sl][1] = v.c[sl][2] = v.c[sl][3] = 0u;
        if (in && y >= 8 && y < 16 && x >= 8 && x < 16) {
            const uint8_t *c = J.cur + (size_t)(y0 + 2 * (y - 8)) * st + x0 + 2 * (x - 8);
            v.c[sl][0] = *(const __attribute__((address_space(1))) uint16_t *)c;
            v.c[sl][1] = *(const __attribute__((address_space(1))) uint16_t *)(c + st);
        }
    }
}

__device__ __forceinline__ void write_input(uint16_t *x0s, const InPix &v, int scale) {
    // an f x f sum s maps to (s - 128 f^2) / (128 f^2): exact in fp32, then bf16
    const int norm = scale == 4 ? 2048 : 512;
    const float inv = scale == 4 ? 1.0f / 2048.0f : 1.0f / 512.0f;
    const int lo = scale == 4 ? 10 : 8, hi = scale == 4 ? 14 : 16;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
        const int q = threadIdx.x + kThreads * sl;
        if (q >= 576) continue;
        const int y = q / 24, x = q - (q / 24) * 24;
        int s = 0, sc = 0;
        if (scale == 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                s += (int)__builtin_amdgcn_sad_u8(v.r[sl][r], 0u, 0u);  // byte sum
                sc += (int)__builtin_amdgcn_sad_u8(v.c[sl][r], 0u, 0u);
            }
        } else {
            s = (int)(v.r[sl][0] + v.r[sl][1] + v.r[sl][2] + v.r[sl][3]);
            sc = (int)((v.c[sl][0] & 0xFFu) + (v.c[sl][0] >> 8) + (v.c[sl][1] & 0xFFu) + (v.c[sl][1] >> 8));
        }
        uint32_t c0 = 0;
        if (y >= lo && y < hi && x >= lo && x < hi) c0 = bf16_bits((float)(sc - norm) * inv);
        x0s[2 * q] = (uint16_t)c0;
        x0s[2 * q + 1] = (uint16_t)bf16_bits((float)(s - norm) * inv);
    }
    // every register consumed on every path (lanes past the input included), so
    // no load into them is left in flight for the next MB's loads to wait on
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
#pragma unroll
        for (int t = 0; t < 4; ++t) asm volatile("" ::"v"(v.r[sl][t]), "v"(v.c[sl][t]));
    }
}

// conv1 A operand: row = output pixel m (24x24), k = 2*tap + ci (18 used).
__device__ __forceinline__ u16x8 conv1_a(const uint16_t *x0s, int m, int g) {
    const int y = m / 24, x = m - (m / 24) * 24;
    uint16_t v[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tap = 4 * g + t;
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        const bool ok = tap < 9 && yy >= 0 && yy < 24 && xx >= 0 && xx < 24;
        const uint32_t pr = ok ? *(const uint32_t *)(x0s + 2 * (yy * 24 + xx)) : 0u;
        v[2 * t] = (uint16_t)(pr & 0xFFFF);
        v[2 * t + 1] = (uint16_t)(pr >> 16);
    }
    return u16x8{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
}

// Activation maps (conv1 and conv2 outputs) are NHWC with 32 bf16 channels
// per pixel, the four 16-byte channel chunks of pixel p XOR-rotated by
// (p >> 1) & 3.  A stride-2 convolution reads every other pixel; without the
// rotation the 16 pixels of one operand read start 128 bytes apart and share
// LDS banks, with it four consecutive ones fall in different banks.
__device__ __forceinline__ int act_off(int pix, int ch) {
    return pix * 32 + ((((ch >> 3) ^ (pix >> 1)) & 3) << 3) + (ch & 7);
}

// A operand of a stride-2 convolution over a 32-channel NHWC map `in`
// (size Hi x Hi, output Ho x Ho): row m, tap, channels 8g..8g+7.
__device__ __forceinline__ u16x8 conv_s2_a(const uint16_t *in, int Hi, int Ho, int m, int tap, int g) {
    const int oy = m / Ho, ox = m - (m / Ho) * Ho;
    const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
    if (m >= Ho * Ho || yy < 0 || yy >= Hi || xx < 0 || xx >= Hi) return zero8();
    return ld16(in + act_off(yy * Hi + xx, 8 * g));
}

// forward pass of one MB; returns with lds.pv holding p (all threads)
// conv1 B operand (column tile nt): k = 2*tap + ci of W1[co][tap][ci], 18 used
__device__ __forceinline__ u16x8 conv1_b(const uint16_t *w1b, int nt, int r16, int g) {
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * g + j;
        v[j] = k < 18 ? w1b[(nt * 16 + r16) * 18 + k] : (uint16_t)0;
    }
    return u16x8{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
}

// The weight operands and biases a wave uses, loaded once per launch.  The
// convolutions run as out^T = W x im2col(in)^T: the weights are the MFMA A
// operand (rows = output channels) and the input patches the B operand
// (columns = output pixels), so a lane's four results are four consecutive
// channels of one pixel and leave as one 8-byte LDS store.
struct NetOps {
    u16x8 w1[2], w2[9], w3[9];  // conv1 row tiles 0, 1; conv2 row tile wv & 1 per tap; conv3 per tap
};

__device__ __forceinline__ void load_ops(NetOps &o, const uint16_t *w1b, const uint16_t *w2b, const uint16_t *w3b,
                                         const float *P) {
    const int l = lane(), wv = threadIdx.x >> 6, r16 = l & 15, g = l >> 4;
    const int n2 = (wv & 1) * 16 + r16;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) o.w1[nt] = conv1_b(w1b, nt, r16, g);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        o.w2[tap] = ld16(w2b + (n2 * 9 + tap) * 32 + 8 * g);
        o.w3[tap] = r16 < 2 ? ld16(w3b + (r16 * 9 + tap) * 32 + 8 * g) : zero8();
    }
    // consumed here, once: otherwise the first use inside the MB loop waits
    // for every load in flight, the next MB's prefetched pixels included
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) asm volatile("" : "+v"(o.w1[nt]));
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        asm volatile("" : "+v"(o.w2[tap]));
        asm volatile("" : "+v"(o.w3[tap]));
    }
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// bias + ReLU of four consecutive channels, rounded to bfloat16 (to nearest
// even, as the bit-level rounding above) and stored as 8 bytes
__device__ __forceinline__ void store4_relu(uint16_t *dst, const f32x4 &acc, const float *bias) {
    const f32x4 b = *(const f32x4 *)bias;
    const f32x2 lo = {relu(acc[0] + b[0]), relu(acc[1] + b[1])};
    const f32x2 hi = {relu(acc[2] + b[2]), relu(acc[3] + b[3])};
    const uint32_t plo = __builtin_bit_cast(uint32_t, __builtin_convertvector(lo, bf16x2));
    const uint32_t phi = __builtin_bit_cast(uint32_t, __builtin_convertvector(hi, bf16x2));
    *(uint2 *)dst = make_uint2(plo, phi);
}

template <class L>
__device__ void forward_mb(L &S, const NetOps &o, const float *P) {
    NetLds &F = S;
    const int l = lane(), wv = threadIdx.x >> 6, r16 = l & 15, g = l >> 4;
    // conv1: 36 pixel tiles x 2 channel tiles
    for (int mt = wv; mt < 36; mt += 4) {
        const u16x8 x = conv1_a(F.x0, mt * 16 + r16, g);
        const int m = mt * 16 + r16;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const f32x4 acc = mfma(o.w1[nt], x, f32x4{0.f, 0.f, 0.f, 0.f});
            store4_relu(F.a1 + act_off(m, nt * 16 + 4 * g), acc, F.bias + nt * 16 + 4 * g);
        }
    }
    __syncthreads();
    // conv2: 9 pixel tiles x 2 channel tiles; wave -> channel tile wv & 1
    {
        const int nt = wv & 1;
        for (int mt = wv >> 1; mt < 9; mt += 2) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc = mfma(o.w2[tap], conv_s2_a(F.a1, 24, 12, mt * 16 + r16, tap, g), acc);
            store4_relu(F.a2 + act_off(mt * 16 + r16, nt * 16 + 4 * g), acc, F.bias + 32 + nt * 16 + 4 * g);
        }
    }
    __syncthreads();
    // conv3: 3 pixel tiles (36 used) x 1 channel tile (2 used), then the mean
    // over the pixels: lanes of g = 0 hold channels 0 and 1 of pixel r16
    if (wv < 3) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) acc = mfma(o.w3[tap], conv_s2_a(F.a2, 12, 6, wv * 16 + r16, tap, g), acc);
        const bool ok = g == 0 && wv * 16 + r16 < 36;
        if (g == 0) {
            F.red[wv][r16] = ok ? acc[0] : 0.f;
            F.red[wv][16 + r16] = ok ? acc[1] : 0.f;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int c = threadIdx.x;
        float t = 0.f;
        for (int w = 0; w < 3; ++w)
            for (int r = 0; r < 16; ++r) t += F.red[w][16 * c + r];
        F.pv[c] = P[kNetOB3 + c] + t * (1.0f / 36.0f);
    }
    __syncthreads();
}

struct NetArgs {
    const JobDesc *jobs;  // tf: training labels (half-pel); out_u32: prediction out (float x 2 per MB)
    int njobs;
    const uint32_t *list;   // (job << 16) | MB, opaque MBs in order
    const uint32_t *count;  // number of list entries
    const float *P;         // fp32 master parameters
    const uint16_t *wb;     // bf16 copies: W1 | W2 | W2 transposed | W3
    float *part;            // training: per-workgroup gradient partials (kNetParams + 1 floats each)
    int scale;              // window scale f (2 or 4)
};

// inference: three workgroups per CU (their LDS fits), so at most 168 VGPRs
template <bool TRAIN>
__global__ __launch_bounds__(kThreads, TRAIN ? 1 : 3) void net_kernel(NetArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds_raw[];
    using L = typename std::conditional<TRAIN, NetLdsTrain, NetLds>::type;
    L &S = *(L *)lds_raw;
    NetLds &F = S;
    const int l = lane(), wv = threadIdx.x >> 6, r16 = l & 15, g = l >> 4;
    const uint16_t *w1b = a.wb, *w2b = a.wb + 576, *w2t = a.wb + 576 + 9216, *w3b = a.wb + 576 + 2 * 9216;
    const int count = (int)uni((int)ldg32(a.count));
    // training accumulators
    f32x4 gw2[9];   // this wave's 9 tiles of dW2 (rows (tap, ci), columns co)
    f32x4 gw1 = {0.f, 0.f, 0.f, 0.f};  // dW1 tile wv: rows co, columns (tap, ci)
    float gw3[2][2] = {{0.f, 0.f}, {0.f, 0.f}};  // (tap, ci) = tid, tid + 256; c = 0, 1
    float gb1 = 0.f, gb2 = 0.f, gb3[2] = {0.f, 0.f}, loss = 0.f;
    if constexpr (TRAIN) {
#pragma unroll
        for (int u = 0; u < 9; ++u) gw2[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const float inv_b = count > 0 ? 1.0f / (float)count : 0.f;
    NetOps ops;
    load_ops(ops, w1b, w2b, w3b, a.P);
    if (threadIdx.x < 64) F.bias[threadIdx.x] = a.P[(threadIdx.x < 32 ? kNetOB1 : kNetOB2 - 32) + threadIdx.x];
    // MB `e` of the list: its job and index (false for an entry the list
    // kernel never produces)
    auto decode = [&](int e, const JobDesc *&J, int &k, InJob &ij) {
        const uint32_t ent = (uint32_t)uni((int)ldg32(a.list + e));
        if ((int)(ent >> 16) >= a.njobs) return false;
        J = a.jobs + (ent >> 16);
        k = (int)(ent & 0xFFFF);
        ij = in_job(J);
        return ij.wm > 0 && k < ij.wm * ij.hm;
    };
    // this workgroup's MBs e = blockIdx.x + j * gridDim.x; the pixels of the
    // next one are loaded while the current one is computed
    InPix pix;
    const JobDesc *Jc = nullptr;
    int kc = 0;
    InJob ic{};
    bool vc = (int)blockIdx.x < count && decode(blockIdx.x, Jc, kc, ic);
    if (vc) {
        issue_input(pix, ic, 16 * (kc % ic.wm), 16 * (kc / ic.wm), a.scale);
        write_input(F.x0, pix, a.scale);
    }
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int en = e + gridDim.x;
        const JobDesc *Jn = nullptr;
        int kn = 0;
        InJob in{};
        const bool vn = en < count && decode(en, Jn, kn, in);
        __syncthreads();  // MB e's input is in LDS
        if (vn) issue_input(pix, in, 16 * (kn % in.wm), 16 * (kn / in.wm), a.scale);
        if (vc) {
            const JobDesc &J = *Jc;
            const int k = kc;
            forward_mb(S, ops, a.P);
            const float p0 = F.pv[0], p1 = F.pv[1];
            if constexpr (!TRAIN) {
                if (threadIdx.x == 0) {
                    if (J.seed) {
                        const int hw = 12 * a.scale - 8;  // the window's half-width
                        const int sx = 2 * iclamp((int)rintf(p0), -hw, hw), sy = 2 * iclamp((int)rintf(p1), -hw, hw);
                        *(__attribute__((address_space(1))) uint32_t *)((uint32_t *)J.seed + k) =
                            (uint32_t)(uint16_t)sx | ((uint32_t)(uint16_t)sy << 16);
                    }
                    if (J.out_u32) {
                        __attribute__((address_space(1))) float *o = (__attribute__((address_space(1))) float *)J.out_u32;
                        o[2 * k] = p0;
                        o[2 * k + 1] = p1;
                    }
                }
            } else {
                NetLdsTrain &T = S;
                const uint32_t lab = ((const uint32_t *)J.tf)[k];
                const float y0 = (float)(((int)(int16_t)(lab & 0xFFFF)) >> 1);
                const float y1 = (float)(((int)(int16_t)(lab >> 16)) >> 1);
                const float dp0 = (p0 - y0) * inv_b, dp1 = (p1 - y1) * inv_b;
                if (threadIdx.x == 0) {
                    loss += 0.5f * ((p0 - y0) * (p0 - y0) + (p1 - y1) * (p1 - y1)) * inv_b;
                    gb3[0] += dp0;
                    gb3[1] += dp1;
                }
                const float dz0 = dp0 * (1.0f / 36.0f), dz1 = dp1 * (1.0f / 36.0f);
                // dW3[c][tap][ci] += dz_c * (sum of the tap-shifted conv2 outputs)
    #pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int q = threadIdx.x + kThreads * r;
                    if (q < 288) {
                        const int tap = q >> 5, ci = q & 31;
                        float s = 0.f;
                        for (int m = 0; m < 36; ++m) {
                            const int yy = 2 * (m / 6) + tap / 3 - 1, xx = 2 * (m % 6) + tap % 3 - 1;
                            if (yy >= 0 && yy < 12 && xx >= 0 && xx < 12) s += bf16_val(F.a2[act_off(yy * 12 + xx, ci)]);
                        }
                        gw3[r][0] += dz0 * s;
                        gw3[r][1] += dz1 * s;
                    }
                }
                // dA2 (uniform dz3) -> ReLU mask -> bias gradient, bf16 copy
                for (int q = threadIdx.x; q < 144 * 32; q += kThreads) {
                    const int pix = q >> 5, ci = q & 31;
                    const int iy = pix / 12, ix = pix % 12;
                    float d = 0.f;
                    for (int ky = 0; ky < 3; ++ky) {
                        const int ty = iy + 1 - ky;
                        if (ty < 0 || (ty & 1) || (ty >> 1) >= 6) continue;
                        for (int kx = 0; kx < 3; ++kx) {
                            const int tx = ix + 1 - kx;
                            if (tx < 0 || (tx & 1) || (tx >> 1) >= 6) continue;
                            const int tap = ky * 3 + kx;
                            d += dz0 * bf16_val(w3b[tap * 32 + ci]) + dz1 * bf16_val(w3b[(9 + tap) * 32 + ci]);
                        }
                    }
                    if (F.a2[act_off(pix, ci)] == 0) d = 0.f;
                    gb2 += d;
                    T.d2[q] = (uint16_t)bf16_bits(d);
                }
                __syncthreads();
                // dW2 += a1 (shifted) x d2: rows (tap, ci) = 18 tiles, columns co = 2 tiles, K = 144 pixels
    #pragma unroll
                for (int u = 0; u < 9; ++u) {
                    const int t = wv * 9 + u, mt = t >> 1, nt = t & 1;
                    const int row = mt * 16 + r16, tap = row >> 5, ci = row & 31;
                    const int co = nt * 16 + r16;
    #pragma unroll 1
                    for (int ks = 0; ks < 5; ++ks) {
                        uint16_t av[8], bv[8];
    #pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int q = ks * 32 + 8 * g + j;
                            const int oy = q / 12, ox = q % 12;
                            const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
                            const bool ok = q < 144 && yy >= 0 && yy < 24 && xx >= 0 && xx < 24;
                            av[j] = ok ? F.a1[act_off(yy * 24 + xx, ci)] : (uint16_t)0;
                            bv[j] = q < 144 ? T.d2[q * 32 + co] : (uint16_t)0;
                        }
                        gw2[u] = mfma(u16x8{av[0], av[1], av[2], av[3], av[4], av[5], av[6], av[7]},
                                      u16x8{bv[0], bv[1], bv[2], bv[3], bv[4], bv[5], bv[6], bv[7]}, gw2[u]);
                    }
                }
                // dA1 = transposed conv of d2 with W2: rows = 576 input pixels, columns ci (tile wv & 1)
                {
                    const int nt = wv & 1, n = nt * 16 + r16;
                    for (int mt = wv >> 1; mt < 36; mt += 2) {
                        const int m = mt * 16 + r16, iy = m / 24, ix = m % 24;
                        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    #pragma unroll
                        for (int tap = 0; tap < 9; ++tap) {
                            const int ty = iy + 1 - tap / 3, tx = ix + 1 - tap % 3;
                            const bool ok = ty >= 0 && !(ty & 1) && (ty >> 1) < 12 && tx >= 0 && !(tx & 1) && (tx >> 1) < 12;
                            const u16x8 av = ok ? ld16(T.d2 + ((ty >> 1) * 12 + (tx >> 1)) * 32 + 8 * g) : zero8();
                            acc = mfma(av, ld16(w2t + (tap * 32 + n) * 32 + 8 * g), acc);
                        }
    #pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int mm = mt * 16 + 4 * g + i;
                            const float d = F.a1[act_off(mm, n)] != 0 ? acc[i] : 0.f;
                            gb1 += d;
                            T.d1[mm * 32 + n] = (uint16_t)bf16_bits(d);
                        }
                    }
                }
                __syncthreads();
                // dW1 += d1^T x x0 (shifted): rows co (tile wv >> 1), columns (tap, ci) (tile wv & 1), K = 576
                {
                    const int co = (wv >> 1) * 16 + r16;
                    const int col = (wv & 1) * 16 + r16, tap = col >> 1, ci = col & 1;
    #pragma unroll 1
                    for (int ks = 0; ks < 18; ++ks) {
                        uint16_t av[8], bv[8];
    #pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int q = ks * 32 + 8 * g + j;
                            const int y = q / 24, x = q % 24;
                            const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
                            av[j] = T.d1[q * 32 + co];
                            bv[j] = (col < 18 && yy >= 0 && yy < 24 && xx >= 0 && xx < 24) ? F.x0[2 * (yy * 24 + xx) + ci]
                                                                                             : (uint16_t)0;
                        }
                        gw1 = mfma(u16x8{av[0], av[1], av[2], av[3], av[4], av[5], av[6], av[7]},
                                   u16x8{bv[0], bv[1], bv[2], bv[3], bv[4], bv[5], bv[6], bv[7]}, gw1);
                    }
                }
            }
        }
        __syncthreads();  // LDS is reused by the next MB
        if (vn) write_input(F.x0, pix, a.scale);
        Jc = Jn;
        kc = kn;
        ic = in;
        vc = vn;
    }
    if constexpr (TRAIN) {
        NetLdsTrain &T = S;
        float *out = a.part + (size_t)blockIdx.x * (kNetParams + 1);
        // dW1: tile rows co = (wv >> 1) * 16 + 4g + i, column (tap, ci) = (wv & 1) * 16 + r16
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = (wv >> 1) * 16 + 4 * g + i, col = (wv & 1) * 16 + r16;
            if (col < 18) out[kNetOW1 + co * 18 + col] = gw1[i];
        }
        // dW2: tile u rows (tap, ci) = mt * 16 + 4g + i, column co = nt * 16 + r16
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const int t = wv * 9 + u, mt = t >> 1, nt = t & 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * g + i, tap = row >> 5, ci = row & 31, co = nt * 16 + r16;
                out[kNetOW2 + (co * 9 + tap) * 32 + ci] = gw2[u][i];
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = threadIdx.x + kThreads * r;
            if (q < 288) {
                out[kNetOW3 + q] = gw3[r][0];
                out[kNetOW3 + 288 + q] = gw3[r][1];
            }
        }
        // bias gradients in a fixed order: b2 by thread (ci = tid % 32), b1 by (wave, lane)
        T.gb[threadIdx.x] = gb2;
        F.red[wv][l] = gb1;
        __syncthreads();
        if (threadIdx.x < 32) {
            const int c = threadIdx.x;
            float s2 = 0.f, s1 = 0.f;
            for (int t = c; t < kThreads; t += 32) s2 += T.gb[t];
            for (int w = (c >> 4); w < 4; w += 2)
                for (int gg = 0; gg < 4; ++gg) s1 += F.red[w][16 * gg + (c & 15)];
            out[kNetOB2 + c] = s2;
            out[kNetOB1 + c] = s1;
        }
        if (threadIdx.x == 0) {
            out[kNetOB3] = gb3[0];
            out[kNetOB3 + 1] = gb3[1];
            out[kNetParams] = loss;
        }
    }
}

// Sum of the workgroup partials (fixed order) into the gradient (and the
// loss); with `apply`, momentum SGD on the fp32 master copy and the bf16
// copies the forward pass reads.
__global__ __launch_bounds__(256) void net_sgd_kernel(float *P, float *V, uint16_t *wb, const float *part, int nparts,
                                                      float lr, float mu, float *grad, double *loss, int apply) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > kNetParams) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += (double)part[(size_t)b * (kNetParams + 1) + i];
    if (i == kNetParams) {
        if (loss) *loss = s;
        return;
    }
    const float gi = (float)s;
    if (grad) grad[i] = gi;
    if (!apply) return;
    const float vi = mu * V[i] + gi;
    const float wi = P[i] - lr * vi;
    V[i] = vi;
    P[i] = wi;
    net_refresh_one(wi, wb, i);
}

// Momentum SGD from a given gradient g: v = mu v + g, w = w - lr v, and the
// bf16 copies.
__global__ __launch_bounds__(256) void net_apply_kernel(float *P, float *V, uint16_t *wb, const float *g, float lr,
                                                        float mu) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kNetParams) return;
    const float vi = mu * V[i] + g[i];
    const float wi = P[i] - lr * vi;
    V[i] = vi;
    P[i] = wi;
    net_refresh_one(wi, wb, i);
}

__global__ __launch_bounds__(256) void net_refresh_kernel(const float *P, uint16_t *wb) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kNetParams) net_refresh_one(P[i], wb, i);
}

// Opaque MBs (all MBs of jobs without classes) in flat order: per-wave
// keep ballots and per-block counts, then (after the scan) the scatter.
__global__ __launch_bounds__(256) void net_flags_kernel(const JobDesc *jobs, int n, int total,
                                                       unsigned long long *keepw, uint32_t *bcount) {
    __shared__ int wcnt[4];
    const int mb = blockIdx.x * 256 + threadIdx.x;
    const int wbase = (int)blockIdx.x * 256 + 64 * uni((int)threadIdx.x >> 6);
    bool keep = false;
    if (wbase < total)
        for_lane_mbs(jobs, n, wbase, min(wbase + 64, total) - 1, [&](const JobCursor &c, int k) {
            const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
            keep = cls ? ldg8(cls + k) == ME_MB_OPAQUE : true;
        });
    const unsigned long long bal = __ballot(keep);
    if (lane() == 0) {
        keepw[mb >> 6] = bal;
        wcnt[threadIdx.x >> 6] = __popcll(bal);
    }
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = (uint32_t)(wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3]);
}

__global__ __launch_bounds__(256) void net_scatter_kernel(const JobDesc *jobs, int n, int total,
                                                         const unsigned long long *keepw, const uint32_t *boff,
                                                         uint32_t *list) {
    const int mb = blockIdx.x * 256 + threadIdx.x;
    const int wbase = (int)blockIdx.x * 256 + 64 * uni((int)threadIdx.x >> 6);
    if (wbase >= total) return;
    const unsigned long long bal = keepw[wbase >> 6];
    if (bal == 0ull) return;  // uniform: nothing kept in this wave
    const bool keep = mb < total && ((bal >> (mb & 63)) & 1ull);
    uint32_t pos = boff[blockIdx.x] + (uint32_t)__popcll(bal & ((1ull << (mb & 63)) - 1ull));
    for (int w = (blockIdx.x * 256) >> 6; w < (mb >> 6); ++w) pos += (uint32_t)__popcll(keepw[w]);
    for_lane_mbs(jobs, n, wbase, min(wbase + 64, total) - 1, [&](const JobCursor &c, int k) {
        if (keep) list[pos] = ((uint32_t)c.j << 16) | (uint32_t)k;
    });
}

}  // namespace

size_t net_lds_bytes(bool train) { return train ? sizeof(NetLdsTrain) : sizeof(NetLds); }

size_t net_list_scratch(int total_mbs) {
    const size_t nb = ((size_t)total_mbs + 255) / 256;
    return 256 + nb * 32 + 256 + nb * 4 + 256 + (size_t)total_mbs * 4 + 256;
}

hipError_t launch_net_list(const JobDesc *jobs, int n, int total_mbs, uint8_t *scratch, const uint32_t **list,
                           const uint32_t **count, hipStream_t s) {
    const int nb = (total_mbs + 255) / 256;
    uint32_t *cnt = (uint32_t *)scratch;
    unsigned long long *keepw = (unsigned long long *)(scratch + 256);
    uint32_t *bcount = (uint32_t *)((uint8_t *)keepw + (((size_t)nb * 32 + 255) & ~(size_t)255));
    uint32_t *out = (uint32_t *)((uint8_t *)bcount + (((size_t)nb * 4 + 255) & ~(size_t)255));
    hipLaunchKernelGGL(net_flags_kernel, dim3(nb), dim3(256), 0, s, jobs, n, total_mbs, keepw, bcount);
    hipError_t e = launch_scan_counts(bcount, nb, cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(net_scatter_kernel, dim3(nb), dim3(256), 0, s, jobs, n, total_mbs, keepw, bcount, out);
    *list = out;
    *count = cnt;
    return hipGetLastError();
}

hipError_t launch_net(bool train, const JobDesc *jobs, int n, const uint32_t *list, const uint32_t *count,
                      const float *P, const uint16_t *wb, float *part, int groups, int scale, hipStream_t s,
                      const KernelTimer *t) {
    NetArgs a{jobs, n, list, count, P, wb, part, scale};
    static bool lds_attr = false;  // dynamic LDS above the default limit for the training kernel
    if (train && !lds_attr) {
        (void)hipFuncSetAttribute((const void *)net_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)net_lds_bytes(true));
        lds_attr = true;
    }
    timer_mark(t, true, s);
    if (train)
        hipLaunchKernelGGL(net_kernel<true>, dim3(groups), dim3(kThreads), net_lds_bytes(true), s, a);
    else
        hipLaunchKernelGGL(net_kernel<false>, dim3(groups), dim3(kThreads), net_lds_bytes(false), s, a);
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

hipError_t launch_net_sgd(float *P, float *V, uint16_t *wb, const float *part, int nparts, float lr, float mu,
                          float *grad, double *loss, hipStream_t s, bool apply) {
    hipLaunchKernelGGL(net_sgd_kernel, dim3((kNetParams + 1 + 255) / 256), dim3(256), 0, s, P, V, wb, part, nparts, lr,
                       mu, grad, loss, apply ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_net_apply(float *P, float *V, uint16_t *wb, const float *g, float lr, float mu, hipStream_t s) {
    hipLaunchKernelGGL(net_apply_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, s, P, V, wb, g, lr, mu);
    return hipGetLastError();
}

hipError_t launch_net_refresh(const float *P, uint16_t *wb, hipStream_t s) {
    hipLaunchKernelGGL(net_refresh_kernel, dim3((kNetParams + 255) / 256), dim3(256), 0, s, P, wb);
    return hipGetLastError();
}

}  // namespace me

// Proposed algorithm (Fig. 1): block-recursive search over A, B, C, T then
// pel-recursive refinement (Eqs. 3-5), for many frame pairs in one launch.
//
// Schedule.  MB (h, v) of a pair needs A = (h-1, v), B = (h, v-1) and
// C = (h+1, v-1) of the same pair, and T = (h, v) of the pair that produced
// its temporal field.  Each wave is a persistent worker that takes one
// "line" = one MB position (h, v) of one chain of pairs and walks it through
// the chain's pairs in order; T of a chained pair is then a register.  Lines
// are handed out by an atomic ticket in the order (h + 2v, chain), which is a
// topological order of the dependencies, so the ticket holder of the oldest
// unfinished work never waits on a worker that has not started: the schedule
// cannot deadlock whatever the residency.  Every wait is bounded; on timeout
// a status bit is raised and all workers leave.
//
// Coherence without cache maintenance.  Each line owns one 64-bit progress
// word: the number of pairs done in the low half and the full-pel vector of
// the latest one in the high half, stored by a single device-scope atomic.
// A consumer that needs pair p of a neighbour polls the word; when it reads
// exactly p+1 the vector comes with it, when the neighbour has moved on the
// vector is read from that pair's mv_int array.  A producer publishes pair p
// and only then writes pair p's result arrays; before every publish it waits
// (s_waitcnt) until all its earlier stores have completed, so arrays of
// pairs < p are complete whenever the word says p+1.  The only loads that
// may still be in flight at a publish are the next pair's window loads,
// issued after those stores; the wait leaves them in flight.  All these accesses are
// device-scope atomics (sc1: served at the device coherence point, never from
// a per-XCD L2 copy), so no L2 invalidate or write-back is ever issued and the
// read-only frames stay L2-resident.  A neighbour that is transparent in the
// pair contributes (0, 0) and is not waited for.
//
// Data path.  Before polling, the worker stages the reference plane around
// its MB, rows and columns [-S-1, 16+S] with coordinates clamped to the frame
// (the clamped central differences of Eq. 5 then need no edge logic), into
// LDS; the poll and the staging loads are in flight together.  The candidate
// costs and every gradient pass then read LDS only.  Lane = (row j, quad q)
// holds 4 pixels; block sums use DPP wave reductions.
#include <algorithm>

#include "me_internal.h"

namespace me {

namespace {

struct PaArgs {
    const JobDesc *jobs;  // in chain order: chain c's pair p is jobs[chains[c].first + p]
    const ChainDesc *chains;
    const uint32_t *tickets;  // lines with work, in ticket order
    const uint32_t *nactive;  // number of those tickets
    unsigned long long *progress;
    uint32_t *counter;
    const uint32_t *tmask;  // per line, per 32 pairs: bit set = MB transparent in that pair
    const uint32_t *bmask;  // per line, per 32 pairs: bit set = MB scored on its alpha block
    int mw;                 // mask words per line
    uint32_t *status;
    KParams kp;
    int pitch;  // window row pitch in bytes (multiple of 4)
    int rows;   // window rows = columns = 2S + 18
};

// Device-scope relaxed accesses through global (not flat) addresses: flat
// operations also count in the LDS counter, and an outstanding flat store
// would then delay every later LDS read of the search.
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint16_t g_u16;
typedef __attribute__((address_space(1))) uint8_t g_u8;

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
    return __hip_atomic_load((g_u32 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(uint32_t *p, uint32_t v) {
    __hip_atomic_store((g_u32 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld64(const unsigned long long *p) {
    typedef __attribute__((address_space(1))) unsigned long long g_u64;
    return __hip_atomic_load((const g_u64 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until at most N vector-memory operations of this wave are in flight
// (and no LDS / scalar-memory operation).  The vector-memory counter
// completes in issue order, loads and stores alike, so every operation
// issued before the N most recent ones has completed.
template <int N>
__device__ __forceinline__ void wait_vm_at_most() {
    static_assert(N == 0 || N == 9 || N == 17 || N == 33, "wait count");
    if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    if constexpr (N == 9) asm volatile("s_waitcnt vmcnt(9) lgkmcnt(0)" ::: "memory");
    if constexpr (N == 17) asm volatile("s_waitcnt vmcnt(17) lgkmcnt(0)" ::: "memory");
    if constexpr (N == 33) asm volatile("s_waitcnt vmcnt(33) lgkmcnt(0)" ::: "memory");
}

// Progress word of a line: pairs done in bits 48-63 (so a larger word is a
// later one) and the full-pel vectors of the last three pairs done in bits
// 0-15 (latest), 16-31 and 32-47, each as two signed bytes (|d| <= 64).
// Published once every memory access of this wave older than its N most
// recent vector-memory operations has completed.
template <int N = 0>
__device__ __forceinline__ void publish(unsigned long long *p, unsigned long long word) {
    wait_vm_at_most<N>();
    __hip_atomic_store(p, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t pack_mv(int x, int y) { return (uint32_t)(uint16_t)x | ((uint32_t)(uint16_t)y << 16); }
__device__ __forceinline__ int mvx_full(uint32_t w) { return ((int)(int16_t)(w & 0xFFFF)) >> 1; }
__device__ __forceinline__ int mvy_full(uint32_t w) { return ((int)(int16_t)(w >> 16)) >> 1; }
__device__ __forceinline__ uint32_t enc8(int dx, int dy) { return (uint32_t)(uint8_t)dx | ((uint32_t)(uint8_t)dy << 8); }
__device__ __forceinline__ unsigned long long progress_word(uint32_t done, uint32_t h0, uint32_t h1, uint32_t h2) {
    return ((unsigned long long)done << 48) | (unsigned long long)h0 | ((unsigned long long)h1 << 16) |
           ((unsigned long long)h2 << 32);
}
__device__ __forceinline__ uint32_t count_of(unsigned long long w) { return (uint32_t)(w >> 48); }
__device__ __forceinline__ uint32_t hist_of(unsigned long long w, uint32_t k) { return (uint32_t)(w >> (16 * k)) & 0xFFFFu; }

// Vectors (half-pel pairs) of pair `need-1` of lines whose progress words are
// `w`: carried by the word when the line is at most three pairs past it,
// else read from that pair's array.
// For the four slots u with use[u] (others give 0); the array reads are all
// issued before any is used, so they cost one memory round trip together.
__device__ __forceinline__ void vectors_of(const unsigned long long (&w)[4], const uint32_t (&need)[4],
                                           const bool (&use)[4], const uint32_t *const (&arr)[4], uint32_t (&m)[4]) {
    bool far[4];
    uint32_t raw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        far[u] = use[u] && count_of(w[u]) - need[u] >= 3u;
        raw[u] = 0u;
        if (far[u]) raw[u] = ld_relaxed(arr[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t age = count_of(w[u]) - need[u];
        const uint32_t e = hist_of(w[u], age < 3u ? age : 0u);
        const uint32_t near = pack_mv(2 * (int)(int8_t)(e & 0xFF), 2 * (int)(int8_t)(e >> 8));
        m[u] = !use[u] ? 0u : far[u] ? (uint32_t)uni((int)raw[u]) : near;
    }
}

// ---------------------------------------------------------------- window
// Window byte (r, c) = plane(clamp(y0-S-1+r), clamp(x0-S-1+c)), binarised
// (0/255) for shape MBs.  Branch-free: every lane loads an in-frame dword at
// the clamped column and, at the frame edge, replicates the edge bytes with a
// byte permute.  Loads are issued twelve at a time (one round trip for a
// +-16 window), not one per dword.
__device__ __forceinline__ void stage_window(uint32_t *win, int pitch, int rows, const uint8_t *P, int st, int W,
                                             int H, int x0, int y0, int S, bool shape) {
    const int l = lane();
    const int dw = pitch >> 2, total = rows * dw;
    const int wx0 = x0 - S - 1, wy0 = y0 - S - 1;
    int r = l / dw, c = l - (l / dw) * dw;
    const int dr = 64 / dw, dc = 64 - (64 / dw) * dw;
    constexpr int kB = 12;
    for (int base = 0; base < total; base += kB * 64) {
        uint32_t v[kB], sel[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int rr = iclamp(wy0 + r, 0, H - 1);
            const int xx = wx0 + 4 * c;
            const int xc = iclamp(xx, 0, W - 4);
            sel[u] = (uint32_t)(iclamp(xx, 0, W - 1) - xc) | ((uint32_t)(iclamp(xx + 1, 0, W - 1) - xc) << 8) |
                     ((uint32_t)(iclamp(xx + 2, 0, W - 1) - xc) << 16) | ((uint32_t)(iclamp(xx + 3, 0, W - 1) - xc) << 24);
            v[u] = ld4(P + (size_t)rr * st + xc);  // clamped: in frame even past the window end
            r += dr;
            c += dc;
            if (c >= dw) {
                c -= dw;
                r += 1;
            }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int i = base + u * 64 + l;
            uint32_t x = __builtin_amdgcn_perm(v[u], v[u], sel[u]);
            if (i < total) win[i] = shape ? bin4(x) : x;
        }
    }
}

// Per-lane staging plan of a line's window: the window geometry is the same
// for every pair of the line, so each lane's dword positions (clamped frame
// row and column) and edge byte selectors are computed once per line.  A
// pair then costs one load, one permute and one LDS write per element, and
// the loads of the next pair's window can be in flight during this pair's
// search.  EM = elements per lane (window dwords / 64, rounded up).
template <int EM>
struct Plan {
    uint32_t loc[EM];  // clamped frame row << 16 | clamped column of the dword
    uint32_t sel[EM];  // byte selectors replicating the frame edge
    uint32_t off[EM];  // byte offsets row * stride + column for stride `st`
    int total, st;

    __device__ __forceinline__ void init(int pitch, int rows, int x0, int y0, int S, int W, int H) {
        const int l = lane();
        const int dw = pitch >> 2;
        total = rows * dw;
        const int wx0 = x0 - S - 1, wy0 = y0 - S - 1;
#pragma unroll
        for (int u = 0; u < EM; ++u) {
            const int i = u * 64 + l;
            const int r = i < total ? i / dw : 0, c = i < total ? i - (i / dw) * dw : 0;
            const int rr = iclamp(wy0 + r, 0, H - 1);
            const int xx = wx0 + 4 * c;
            const int xc = iclamp(xx, 0, W - 4);
            loc[u] = ((uint32_t)rr << 16) | (uint32_t)xc;
            sel[u] = (uint32_t)(iclamp(xx, 0, W - 1) - xc) | ((uint32_t)(iclamp(xx + 1, 0, W - 1) - xc) << 8) |
                     ((uint32_t)(iclamp(xx + 2, 0, W - 1) - xc) << 16) |
                     ((uint32_t)(iclamp(xx + 3, 0, W - 1) - xc) << 24);
        }
        st = -1;
    }
    // byte offsets for row pitch `stride` (kept while the pitch repeats)
    __device__ __forceinline__ void offsets(int stride) {
        if (stride == st) return;
        st = stride;
#pragma unroll
        for (int u = 0; u < EM; ++u) off[u] = (loc[u] >> 16) * (uint32_t)stride + (loc[u] & 0xFFFFu);
    }
    // loads only; every address is in frame, elements past the window
    // re-read the window origin and are never written
    __device__ __forceinline__ void issue(const uint8_t *P, int stride, uint32_t (&v)[EM]) {
        offsets(stride);
#pragma unroll
        for (int u = 0; u < EM; ++u) v[u] = ld4(P + off[u]);
    }
    __device__ __forceinline__ void write(uint32_t *win, const uint32_t (&v)[EM], bool shape) const {
        const int l = lane();
#pragma unroll
        for (int u = 0; u < EM; ++u) {
            const int i = u * 64 + l;
            const uint32_t x = __builtin_amdgcn_perm(v[u], v[u], sel[u]);
            if (i < total) win[i] = shape ? bin4(x) : x;
        }
    }
};

struct Sweep {
    int sad, sx, sy, nxy;  // nxy = nx | ny << 16
};

struct Ctx {
    const uint32_t *win;
    const short *R;
    int pitch, S;
    int off0;          // window byte offset of this lane's first pixel at d = 0
    int bdw, ph;       // off0 = 4 bdw + ph; ph is the same in every lane (the pitch is a multiple of 4)
    int x0, y0, W, H;
    uint32_t c4;       // this lane's 4 current pixels
    bool shape;
    int lox, hix, loy, hiy;
    // texture of a boundary MB, for T scored on texture (Section 3.1 text) and
    // the masked-luma recursion: the reference luma, its pitch, this lane's 4
    // current luma pixels
    const uint8_t *ref_l;
    int st;
    uint32_t tl4;
};

__device__ __forceinline__ int cost_of(const Ctx &c, int sad) { return c.shape ? sad / 255 : sad; }

// The lane's window offset plus a wave-uniform offset uo: the byte shift and
// the dword step are then scalar, and a read is one address add, one
// two-dword LDS read and one v_alignbyte_b32.
__device__ __forceinline__ void set_lane_base(Ctx &c, int off0, int S) {
    c.off0 = off0;
    c.bdw = off0 >> 2;
    c.ph = (S + 1) & 3;
}
// 4 window bytes at the lane's pixel moved by uo
__device__ __forceinline__ uint32_t wread4(const Ctx &c, int uo) {
    const int t = uni(c.ph + uo);
    const uint32_t *w = c.win + c.bdw + (t >> 2);
    return __builtin_amdgcn_alignbyte(w[1], w[0], (uint32_t)(t & 3));
}
// 8 window bytes at the lane's pixel moved by uo (lo = bytes 0..3, hi = 4..7)
__device__ __forceinline__ void wread8(const Ctx &c, int uo, uint32_t &lo, uint32_t &hi) {
    const int t = uni(c.ph + uo);
    const uint32_t *w = c.win + c.bdw + (t >> 2);
    const uint32_t a = w[0], b = w[1], d = w[2];
    lo = __builtin_amdgcn_alignbyte(b, a, (uint32_t)(t & 3));
    hi = __builtin_amdgcn_alignbyte(d, b, (uint32_t)(t & 3));
}

// Admissible box of the MB at (x0, y0): |d| <= S with the displaced block in
// the frame, or (unrestricted vectors) |d| <= S only - the staged window
// covers every such offset with edge-replicated bytes.
__device__ __forceinline__ void set_box(Ctx &c, const KParams &kp, int x0, int y0, int W, int H) {
    const int S = kp.S;
    c.lox = kp.unrestricted ? -S : max(-S, -x0);
    c.hix = kp.unrestricted ? S : min(S, W - 16 - x0);
    c.loy = kp.unrestricted ? -S : max(-S, -y0);
    c.hiy = kp.unrestricted ? S : min(S, H - 16 - y0);
}

// One fused pass at full-pel offset (dx, dy): SAD of the block and the
// gradient sums of Eqs. 3-5 (central differences of the reference at the
// displaced position).
__device__ __forceinline__ Sweep sweep(const Ctx &c, int dx, int dy) {
    const int uo = uni(dy * c.pitch + dx);
    uint32_t lo, hi;
    wread8(c, uo - 1, lo, hi);                    // bytes rx-1 .. rx+6
    const uint32_t m = __builtin_amdgcn_alignbyte(hi, lo, 1);
    const int lf = (int)(lo & 0xFF), rt = (int)((hi >> 8) & 0xFF);
    const uint32_t up = wread4(c, uo - c.pitch), dn = wread4(c, uo + c.pitch);
    int sad = (int)__builtin_amdgcn_sad_u8(c.c4, m, 0u);
    int sx = 0, sy = 0, nn = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = byte_of(c.c4, k) - byte_of(m, k);
        const int left = k == 0 ? lf : byte_of(m, k - 1);
        const int right = k == 3 ? rt : byte_of(m, k + 1);
        const int rgx = c.R[right - left + 255];
        const int rgy = c.R[byte_of(dn, k) - byte_of(up, k) + 255];
        sx += e * rgx;
        sy += e * rgy;
        nn += (rgx != 0) + ((rgy != 0) << 16);
    }
    Sweep s;
    s.sad = wave_sum(sad);
    s.sx = wave_sum(sx);
    s.sy = wave_sum(sy);
    s.nxy = wave_sum(nn);
    return s;
}

// The pass of a boundary MB refined on texture over the current VOP's pixels
// (c.c4: the 0/255 mask of the lane's 4 pixels, c.tl4: their luma): the
// luma SAD and the gradient sums of Eqs. 3-5 over the masked pixels only,
// the reference read from the frame with edge-clamped coordinates.
__device__ __forceinline__ Sweep sweep_masked(const Ctx &c, int dx, int dy) {
    const int ry = c.y0 + (lane() >> 2) + dy, rx = c.x0 + 4 * (lane() & 3) + dx;
    const uint8_t *row = c.ref_l + (size_t)iclamp(ry, 0, c.H - 1) * c.st;
    const uint32_t lo = ld4_clamped(row, rx - 1, c.W), hi = ld4_clamped(row, rx + 3, c.W);
    const uint32_t up = ld4_clamped(c.ref_l + (size_t)iclamp(ry - 1, 0, c.H - 1) * c.st, rx, c.W);
    const uint32_t dn = ld4_clamped(c.ref_l + (size_t)iclamp(ry + 1, 0, c.H - 1) * c.st, rx, c.W);
    const uint32_t m = __builtin_amdgcn_alignbyte(hi, lo, 1);
    const int lf = (int)(lo & 0xFF), rt = (int)((hi >> 8) & 0xFF);
    const int sad = (int)__builtin_amdgcn_sad_u8(c.tl4 & c.c4, m & c.c4, 0u);
    int sx = 0, sy = 0, nn = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = byte_of(c.c4, k) != 0;
        const int e = byte_of(c.tl4, k) - byte_of(m, k);
        const int left = k == 0 ? lf : byte_of(m, k - 1);
        const int right = k == 3 ? rt : byte_of(m, k + 1);
        const int rgx = in ? c.R[right - left + 255] : 0;
        const int rgy = in ? c.R[byte_of(dn, k) - byte_of(up, k) + 255] : 0;
        sx += e * rgx;
        sy += e * rgy;
        nn += (rgx != 0) + ((rgy != 0) << 16);
    }
    Sweep s;
    s.sad = wave_sum(sad);
    s.sx = wave_sum(sx);
    s.sy = wave_sum(sy);
    s.nxy = wave_sum(nn);
    return s;
}

// Section 3.2 recursion from (dx, dy) with distortion `cost` and pass `sw`
// at that point (MASKED: the masked-luma passes of a boundary MB refined on
// texture).  Returns the number of candidates evaluated.
template <bool MASKED = false>
__device__ int pel_recursion(const Ctx &c, const KParams &kp, int &dx, int &dy, int &cost, Sweep sw) {
    int it = 0;
    // every value here is the same in all lanes: readfirstlane keeps the
    // step rule in scalar registers and scalar branches
    dx = uni(dx);
    dy = uni(dy);
    cost = uni(cost);
    while (it < kp.k_max) {
        const int nx = sw.nxy & 0xFFFF, ny = sw.nxy >> 16;
        // U = trunc(S / n) gives a zero step iff |U| < zero_t, i.e. |S| < zero_t * n:
        // decided without the divisions, which most MBs then skip
        const bool zx = nx == 0 || llabs((long long)sw.sx) < (long long)kp.zero_t * nx;
        const bool zy = ny == 0 || llabs((long long)sw.sy) < (long long)kp.zero_t * ny;
        if (zx && zy) break;
        const int sx = zx ? 0 : prs_step(sw.sx / nx, kp.eps, kp.max_step);
        const int sy = zy ? 0 : prs_step(sw.sy / ny, kp.eps, kp.max_step);
        if (sx == 0 && sy == 0) break;
        const int tx = uni(iclamp(dx + sx, c.lox, c.hix));
        const int ty = uni(iclamp(dy + sy, c.loy, c.hiy));
        if (tx == dx && ty == dy) break;
        ++it;
        const Sweep s2 = MASKED ? sweep_masked(c, tx, ty) : sweep(c, tx, ty);
        const int c2 = MASKED ? s2.sad : cost_of(c, s2.sad);
        if (c2 < cost) {
            dx = tx;
            dy = ty;
            cost = c2;
            sw = s2;
        } else {
            break;
        }
    }
    return it;
}

// the eight half-sample offsets in row order (compile-time, so every index
// into the neighbourhood below is a constant)
constexpr int kHalfX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
constexpr int kHalfY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

// Per byte, (a + b + 1) >> 1: the half-sample average of MPEG-4 with
// rounding control 0, four pixels at once (v_lerp_u8 adds the low bit of
// each byte of its third operand before the shift).
__device__ __forceinline__ uint32_t avg2_u8x4(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_lerp(a, b, 0x01010101u);
}

// The even (bytes 0, 2) and odd (bytes 1, 3) pixels of a quad in the low
// bytes of two 16-bit halves.
__device__ __forceinline__ uint32_t even_u8x2(uint32_t x) { return x & 0x00FF00FFu; }
__device__ __forceinline__ uint32_t odd_u8x2(uint32_t x) { return __builtin_amdgcn_perm(0u, x, 0x0C030C01u); }

// Per byte, (s + 2) >> 2 of 16-bit half sums s = a + b + c + d (at most
// 1022, so no half carries into the next): the diagonal half-sample value,
// even and odd pixels put back in place.
__device__ __forceinline__ uint32_t quarter_u8x4(uint32_t se, uint32_t so) {
    const uint32_t pe = ((se + 0x00020002u) >> 2) & 0x00FF00FFu;
    const uint32_t po = ((so + 0x00020002u) >> 2) & 0x00FF00FFu;
    return pe | (po << 8);
}

// Half-sample refinement around the full-pel vector d (MPEG-4 bilinear,
// rounding control 0).  Updates (hx, hy), cost; returns the feasible count.
// Each lane predicts its 4 pixels for all eight offsets from the quads of
// the rows above, at and below d, shifted one pixel left (L), in place (P)
// and one pixel right (R): horizontal and vertical half samples are per-byte
// rounded averages, diagonal ones per-byte (A + B + C + D + 2) >> 2 from
// 16-bit pair sums; each SAD is one v_sad_u8.
__device__ int half_refine(const Ctx &c, const KParams &kp, int dx, int dy, int &hx, int &hy, int &cost) {
    const int uo = uni(dy * c.pitch + dx);
    uint32_t L[3], P[3], R[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        uint32_t lo, hi;
        wread8(c, uo + (r - 1) * c.pitch - 1, lo, hi);   // columns -1 .. 6
        L[r] = lo;
        P[r] = __builtin_amdgcn_alignbyte(hi, lo, 1);
        R[r] = __builtin_amdgcn_alignbyte(hi, lo, 2);
    }
    // horizontal pair sums (pixel k-1 + k, pixel k + k+1) per row, even / odd
    uint32_t hme[3], hmo[3], hpe[3], hpo[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const uint32_t pe = even_u8x2(P[r]), po = odd_u8x2(P[r]);
        hme[r] = even_u8x2(L[r]) + pe;
        hmo[r] = odd_u8x2(L[r]) + po;
        hpe[r] = pe + even_u8x2(R[r]);
        hpo[r] = po + odd_u8x2(R[r]);
    }
    // predictions in the order of the offsets (row order: -1 -1, 0 -1, 1 -1,
    // -1 0, 1 0, -1 1, 0 1, 1 1)
    uint32_t pred[8];
    pred[0] = quarter_u8x4(hme[0] + hme[1], hmo[0] + hmo[1]);
    pred[1] = avg2_u8x4(P[0], P[1]);
    pred[2] = quarter_u8x4(hpe[0] + hpe[1], hpo[0] + hpo[1]);
    pred[3] = avg2_u8x4(L[1], P[1]);
    pred[4] = avg2_u8x4(P[1], R[1]);
    pred[5] = quarter_u8x4(hme[1] + hme[2], hmo[1] + hmo[2]);
    pred[6] = avg2_u8x4(P[1], P[2]);
    pred[7] = quarter_u8x4(hpe[1] + hpe[2], hpo[1] + hpo[2]);
    int tot[8];
#pragma unroll
    for (int o = 0; o < 8; o += 2) {
        const int pk = wave_sum((int)__builtin_amdgcn_sad_u8(c.c4, pred[o], 0u) |
                                ((int)__builtin_amdgcn_sad_u8(c.c4, pred[o + 1], 0u) << 16));
        tot[o] = pk & 0xFFFF;
        tot[o + 1] = (int)((uint32_t)pk >> 16);
    }
    // feasibility, the same in every lane: offset -1 / +1 on an axis needs
    // |2d -+ 1| <= 2S and (unless vectors are unrestricted) the interpolated
    // block's extra column / row inside the frame (d itself is admissible)
    dx = uni(dx);
    dy = uni(dy);
    const int S2 = 2 * kp.S, ur = kp.unrestricted;
    const bool xm = 2 * dx - 1 >= -S2 && (ur || c.x0 + dx >= 1);
    const bool xp = 2 * dx + 1 <= S2 && (ur || c.x0 + dx + 16 <= c.W - 1);
    const bool ym = 2 * dy - 1 >= -S2 && (ur || c.y0 + dy >= 1);
    const bool yp = 2 * dy + 1 <= S2 && (ur || c.y0 + dy + 16 <= c.H - 1);
    int bx = 2 * dx, by = 2 * dy, bc = uni(cost), nfeas = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int ox = kHalfX[o], oy = kHalfY[o];
        const bool feas = (ox < 0 ? xm : ox > 0 ? xp : true) && (oy < 0 ? ym : oy > 0 ? yp : true);
        nfeas += feas;
        if (feas && tot[o] < bc) {
            bc = tot[o];
            bx = 2 * dx + ox;
            by = 2 * dy + oy;
        }
    }
    hx = uni(bx);
    hy = uni(by);
    cost = uni(bc);
    return uni(nfeas);
}

struct MbOut {
    uint32_t mv, mvi, cost;
    int iters, points, dx, dy;
};

// Fig. 1 after the candidates are known: the admissible distinct list in the
// order A, B, C, T, its first minimum, the recursion (from a learned seed
// with the 5 % fallback when the job carries seeds), half-sample refinement.
// MP: the instantiation that has the masked-luma recursion of boundary MBs
// (kp.masked_prs); the others have no code for it.
template <bool MP = false>
__device__ MbOut search_mb(const uint32_t *seed, const Ctx &c, int k, int (&cx)[4], int (&cy)[4], const KParams &kp,
                           bool half = true) {
    // the candidates are the same in every lane: in scalar registers, and
    // the list (admissible, distinct, in order) as a bit mask
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cx[i] = uni(cx[i]);
        cy[i] = uni(cy[i]);
    }
    int keepm = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int ok = (cx[i] >= c.lox && cx[i] <= c.hix && cy[i] >= c.loy && cy[i] <= c.hiy) ? 1 : 0;
#pragma unroll
        for (int p = 0; p < i; ++p)
            if (((keepm >> p) & 1) && cx[p] == cx[i] && cy[p] == cy[i]) ok = 0;
        keepm |= ok << i;
    }
    keepm = uni(keepm);
    if (keepm == 0) {
        cx[0] = cy[0] = 0;
        keepm = 1;
    }
    const int n = __builtin_popcount((uint32_t)keepm);
    bool keep[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) keep[i] = (keepm >> i) & 1;
    // block costs of the list, two 16-bit partial SADs per reduction.  All
    // four are computed without branches (their LDS reads in flight
    // together): an offset clamped to +-S lies inside the staged window, and
    // the cost of a dropped candidate is never used.
    uint32_t blk[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        blk[i] = wread4(c, iclamp(cy[i], -c.S, c.S) * c.pitch + iclamp(cx[i], -c.S, c.S));
    int part[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) part[i] = (int)__builtin_amdgcn_sad_u8(c.c4, blk[i], 0u);
    const int p01 = wave_sum(part[0] | (part[1] << 16));
    const int p23 = wave_sum(part[2] | (part[3] << 16));
    const int costs[4] = {p01 & 0xFFFF, (int)((uint32_t)p01 >> 16), p23 & 0xFFFF, (int)((uint32_t)p23 >> 16)};
    // Min[...]: the first minimum in list order.  With T scored on texture
    // (a boundary MB whose list holds T and a spatial entry), the first
    // minimum of the spatial entries' BAB costs, then T replaces it when its
    // luma SAD over the VOP pixels is strictly lower.
    const bool tex_t = kp.t_texture && c.shape && !kp.shape_only && keep[3] && n > 1;
    int dx = 0, dy = 0, bc = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int ci = cost_of(c, costs[i]);
        if (keep[i] && (i < 3 || !tex_t) && ci < bc) {
            bc = ci;
            dx = cx[i];
            dy = cy[i];
        }
    }
    if (tex_t) {
        // c.c4 is the 0/255 mask of the current VOP pixels: both SADs over it
        const int ry = c.y0 + (lane() >> 2), rx = c.x0 + 4 * (lane() & 3);
        const uint32_t rs = ld4_clamped(c.ref_l + (size_t)iclamp(ry + dy, 0, c.H - 1) * c.st, rx + dx, c.W);
        const uint32_t rt = ld4_clamped(c.ref_l + (size_t)iclamp(ry + cy[3], 0, c.H - 1) * c.st, rx + cx[3], c.W);
        const uint32_t lm = c.tl4 & c.c4;
        const int ps = (int)__builtin_amdgcn_sad_u8(lm, rs & c.c4, 0u);
        const int pt = (int)__builtin_amdgcn_sad_u8(lm, rt & c.c4, 0u);
        const int pk = wave_sum(ps | (pt << 16));
        if ((int)((uint32_t)pk >> 16) < (pk & 0xFFFF)) {
            dx = cx[3];
            dy = cy[3];
            bc = cost_of(c, costs[3]);
        }
    }
    dx = uni(dx);
    dy = uni(dy);
    bc = uni(bc);
    int dc = bc;
    int pts = n + (tex_t ? 1 : 0), its = 0;
    if (MP && kp.masked_prs && c.shape) {
        // a boundary MB refined on texture over its VOP pixels (a reading of
        // Section 3.1): the winner's masked luma SAD (one more compared
        // block) starts the recursion
        const Sweep sw = sweep_masked(c, dx, dy);
        dc = sw.sad;
        pts += 1;
        if (kp.k_max > 0) {
            const int it1 = pel_recursion<true>(c, kp, dx, dy, dc, sw);
            its += it1;
            pts += it1;
        }
    } else if (seed && !c.shape) {
        const uint32_t w = (uint32_t)uni((int)ldg32(seed + k));
        int sx = iclamp(mvx_full(w), c.lox, c.hix), sy = iclamp(mvy_full(w), c.loy, c.hiy);
        const Sweep sw = sweep(c, sx, sy);
        int sc = cost_of(c, sw.sad);
        pts += 1;
        const int it1 = pel_recursion(c, kp, sx, sy, sc, sw);
        its += it1;
        pts += it1;
        if (20ll * sc > 21ll * bc) {
            if (kp.k_max > 0) {
                const int it2 = pel_recursion(c, kp, dx, dy, dc, sweep(c, dx, dy));
                its += it2;
                pts += it2;
            }
        } else {
            dx = sx;
            dy = sy;
            dc = sc;
        }
    } else if (kp.k_max > 0) {
        const int it1 = pel_recursion(c, kp, dx, dy, dc, sweep(c, dx, dy));
        its += it1;
        pts += it1;
    }
    int hx = 2 * dx, hy = 2 * dy;
    if (half && kp.half_pel && !c.shape) pts += half_refine(c, kp, dx, dy, hx, hy, dc);
    MbOut o;
    o.mv = pack_mv(hx, hy);
    o.mvi = pack_mv(2 * dx, 2 * dy);
    o.cost = (uint32_t)dc;
    o.iters = its;
    o.points = pts;
    o.dx = dx;
    o.dy = dy;
    return o;
}

// A job descriptor held across the wave: lane i (< 40) holds dword i, so a
// field is one v_readlane.  Loading the next pair's descriptor this way costs
// one load per lane, issued a whole pair ahead.
struct DescReg {
    uint32_t d;
    __device__ __forceinline__ uint32_t u32(int i) const { return (uint32_t)__builtin_amdgcn_readlane((int)d, i); }
    __device__ __forceinline__ int i32(int i) const { return (int)u32(i); }
    template <class T>
    __device__ __forceinline__ T *ptr(int i) const {
        return (T *)(uintptr_t)((unsigned long long)u32(i) | ((unsigned long long)u32(i + 1) << 32));
    }
};

#define DW(f) ((int)(offsetof(JobDesc, f) / 4))

__device__ __forceinline__ uint32_t load_desc(const JobDesc *J) {
    const int l = lane();
    return ldg32((const uint32_t *)J + (l < 40 ? l : 39));
}

__device__ __forceinline__ void store_result(const DescReg &D, int k, uint32_t mv, uint32_t mvi, uint32_t cost,
                                             int iters, int points) {
    ((g_u32 *)D.ptr<uint32_t>(DW(mv)))[k] = mv;
    st_relaxed(D.ptr<uint32_t>(DW(mv_int)) + k, mvi);
    uint32_t *co = D.ptr<uint32_t>(DW(cost));
    uint8_t *it = D.ptr<uint8_t>(DW(iters));
    uint16_t *pt = D.ptr<uint16_t>(DW(points));
    if (co) ((g_u32 *)co)[k] = cost;
    if (it) ((g_u8 *)it)[k] = (uint8_t)iters;
    if (pt) ((g_u16 *)pt)[k] = (uint16_t)points;
}

// Pre-pass over every MB of every pair: a transparent MB gets its (zero)
// result here, and each line's 32-pair mask words record which pairs are
// transparent and which are scored on the alpha block.  The line workers
// then skip transparent runs with one publish and never wait for a
// neighbour that is transparent in the pair.
__global__ __launch_bounds__(256) void pa_prepass(const JobDesc *jobs, int n, int total, uint32_t *tmask,
                                                 uint32_t *bmask, int mw, int shape_only, uint32_t *status) {
    // one MB per lane, 64 consecutive flat MBs per wave; their job (nearly
    // always one) is a wave-uniform cursor
    const int base = ((int)blockIdx.x * 4 + uni((int)threadIdx.x >> 6)) * 64;
    if (base >= total) return;
    for_lane_mbs(jobs, n, base, min(base + 64, total) - 1, [&](const JobCursor &c, int k) {
        const uint8_t *cls = c.ptr<const uint8_t>(DWI(cls));
        int cl = cls ? (int)ldg8(cls + k) : ME_MB_OPAQUE;
        if (cl > 2) {
            atomicOr(status, ST_BAD_CLASS);
            cl = ME_MB_TRANSPARENT;
        }
        const int pos = c.i32(DWI(chain_pos));
        const size_t wi = (size_t)(c.i32(DWI(chain_line_base)) + k) * mw + (pos >> 5);
        const uint32_t bit = 1u << (pos & 31);
        if (cl == ME_MB_TRANSPARENT) {
            ((g_u32 *)c.ptr<uint32_t>(DWI(mv)))[k] = 0u;
            ((g_u32 *)c.ptr<uint32_t>(DWI(mv_int)))[k] = 0u;
            uint32_t *co = c.ptr<uint32_t>(DWI(cost));
            uint8_t *it = c.ptr<uint8_t>(DWI(iters));
            uint16_t *pt = c.ptr<uint16_t>(DWI(points));
            if (co) ((g_u32 *)co)[k] = 0u;
            if (it) ((g_u8 *)it)[k] = 0;
            if (pt) ((g_u16 *)pt)[k] = 0;
            atomicOr(tmask + wi, bit);
        } else if (cl == ME_MB_BOUNDARY || shape_only) {
            atomicOr(bmask + wi, bit);
        }
    });
}

// Line of ticket tk, and whether it is transparent in every pair of its
// chain (its mask bits of pairs 0 .. len-1 all set).  The mask words are
// read four at a time (in-range loads past the last word are ignored), so a
// transparent line costs one round trip per four words, not per word.
__device__ __forceinline__ bool line_all_transparent(const ChainDesc *chains, uint32_t tk, const uint32_t *tmask,
                                                     int mw, int &line, int &len) {
    const ChainDesc ch = chains[tk >> 16];
    line = ch.line_base + (int)((tk >> 8) & 0xFF) * ch.wm + (int)(tk & 0xFF);
    len = ch.len;
    const uint32_t *m = tmask + (size_t)line * mw;
    const int nw = min(mw, (ch.len + 31) >> 5);
    for (int w0 = 0; w0 < nw; w0 += 4) {
        uint32_t word[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) word[d] = m[min(w0 + d, nw - 1)];
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int bits = min(32, ch.len - 32 * (w0 + d));
            const uint32_t full = bits >= 32 ? 0xFFFFFFFFu : bits > 0 ? ((1u << bits) - 1u) : 0u;
            ok = ok && (w0 + d >= nw || (word[d] & full) == full);
        }
        if (!ok) return false;
    }
    return true;
}

// Lines transparent in every pair of their chain need no worker: their
// final progress word (all pairs done, zero vector) is stored here and they
// leave the ticket list; the others keep their ticket order (an order-
// preserving compaction: per-wave keep ballots and per-block counts, a scan
// of the block counts, then the scatter).
__global__ __launch_bounds__(256) void pa_line_flags(const ChainDesc *chains, const uint32_t *tickets, int nlines,
                                                    const uint32_t *tmask, int mw, unsigned long long *progress,
                                                    unsigned long long *keepw, uint32_t *bcount) {
    __shared__ int wcnt[4];
    const int t = blockIdx.x * 256 + threadIdx.x;
    bool keep = false;
    if (t < nlines) {
        int line = 0, len = 0;
        const bool all = line_all_transparent(chains, tickets[t], tmask, mw, line, len);
        if (all) progress[line] = (unsigned long long)(uint32_t)len << 48;
        keep = !all;
    }
    const unsigned long long bal = __ballot(keep);
    if (lane() == 0) {
        keepw[t >> 6] = bal;
        wcnt[threadIdx.x >> 6] = __popcll(bal);
    }
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = (uint32_t)(wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3]);
}

// The same flags and order-preserving compaction in one workgroup, for at
// most kCompactOneBlock lines: chunks of 1024 tickets, one per thread, a
// scan of the keep flags in LDS gives each kept ticket its output slot after
// the earlier chunks' total.
constexpr int kCompactOneBlock = 4096;
__global__ __launch_bounds__(1024) void pa_compact_lines(const ChainDesc *chains, const uint32_t *tickets, int nlines,
                                                        const uint32_t *tmask, int mw, unsigned long long *progress,
                                                        uint32_t *out, uint32_t *nactive) {
    __shared__ uint32_t sh[1024];
    const int tid = threadIdx.x;
    uint32_t carry = 0u;
    for (int base = 0; base < nlines; base += 1024) {
        const int t = base + tid;
        uint32_t tk = 0u, keep = 0u;
        if (t < nlines) {
            tk = tickets[t];
            int line = 0, len = 0;
            if (line_all_transparent(chains, tk, tmask, mw, line, len))
                progress[line] = (unsigned long long)(uint32_t)len << 48;
            else
                keep = 1u;
        }
        sh[tid] = keep;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t x = tid >= off ? sh[tid - off] : 0u;
            __syncthreads();
            sh[tid] += x;
            __syncthreads();
        }
        if (keep) out[carry + sh[tid] - 1u] = tk;  // exclusive prefix = inclusive - 1
        carry += sh[1023];
        __syncthreads();
    }
    if (tid == 0) *nactive = carry;
}

// Exclusive scan of the nb block counts in place; the total to *nactive.
__global__ __launch_bounds__(1024) void pa_scan_counts(uint32_t *bcount, int nb, uint32_t *nactive) {
    __shared__ uint32_t sh[1024];
    const int tid = threadIdx.x;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + tid;
        const uint32_t v = i < nb ? bcount[i] : 0u;
        sh[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t x = tid >= off ? sh[tid - off] : 0u;
            __syncthreads();
            sh[tid] += x;
            __syncthreads();
        }
        if (i < nb) bcount[i] = carry + sh[tid] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (tid == 0) *nactive = carry;
}

__global__ __launch_bounds__(256) void pa_scatter_tickets(const uint32_t *tickets, int nlines,
                                                         const unsigned long long *keepw, const uint32_t *boff,
                                                         uint32_t *out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nlines) return;
    const unsigned long long bal = keepw[t >> 6];
    if (!((bal >> (t & 63)) & 1ull)) return;
    uint32_t pos = boff[blockIdx.x] + (uint32_t)__popcll(bal & ((1ull << (t & 63)) - 1ull));
    for (int w = (blockIdx.x * 256) >> 6; w < (t >> 6); ++w) pos += (uint32_t)__popcll(keepw[w]);
    out[pos] = tickets[t];
}

template <int EM, bool MP = false>
__global__ __launch_bounds__(64) void pa_kernel(PaArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int slot;
    short *R = (short *)lds;                     // 511 reciprocal entries (Eq. 4-5, Q.12)
    uint32_t *const win0 = lds + 256;            // staged reference window
    const KParams kp = a.kp;
    for (int g = lane(); g < 511; g += 64) {
        const int m = abs(g - 255);
        const int r = (m == 0 || m < 2 * kp.theta) ? 0 : (16384 + m) / (2 * m);
        R[g] = (short)(g < 255 ? -r : r);
    }
    const int l = lane(), j = l >> 2, q = l & 3;
    const int S = kp.S;
    const int nact = (int)uni((int)ldg32(a.nactive));
    for (;;) {
        // ticket: lane 0 draws, LDS + barriers broadcast (barriers keep the
        // wave converged across loop trips).  Only a running worker ever
        // holds a ticket, which the deadlock-freedom argument needs.
        __syncthreads();
        if (l == 0) slot = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int t = uni(slot);
        if (t >= nact) break;
        if (uni((int)ld_relaxed(a.status)) & ST_ABORT) break;
        const uint32_t tk = a.tickets[t];
        const int ci = (int)(tk >> 16), v = (int)((tk >> 8) & 0xFF), h = (int)(tk & 0xFF);
        const ChainDesc ch = a.chains[ci];
        const int wm = ch.wm;
        const int k = v * wm + h;
        const JobDesc *jobs = a.jobs + ch.first;
        const int line = ch.line_base + k;
        unsigned long long *const own = a.progress + line;
        const int x0 = 16 * h, y0 = 16 * v;
        const int W = 16 * ch.wm, H = 16 * ch.hm;
        const bool inA = h > 0, inB = v > 0, inC = v > 0 && h + 1 < wm;
        // mask rows of this line and of A, B, C (absent ones alias this line)
        const uint32_t *mo = a.tmask + (size_t)line * a.mw;
        const uint32_t *mbd = a.bmask + (size_t)line * a.mw;
        const uint32_t *ma = a.tmask + (size_t)(inA ? line - 1 : line) * a.mw;
        const uint32_t *mb = a.tmask + (size_t)(inB ? line - wm : line) * a.mw;
        const uint32_t *mc = a.tmask + (size_t)(inC ? line - wm + 1 : line) * a.mw;
        Plan<(EM > 0 ? EM : 1)> plan;
        if (EM > 0) plan.init(a.pitch, a.rows, x0, y0, S, W, H);
        uint32_t wT = 0, wB = 0, wA = 0, wBn = 0, wC = 0;
        int wi = -1;
        int tx = 0, ty = 0;
        uint32_t hist1 = 0, hist2 = 0;  // encoded vectors of the two pairs before the latest
        // descriptors of pairs p and p + 1 (valid flags v0, v1), fetched ahead
        uint32_t d0 = 0, d1 = 0;
        bool v0 = false, v1 = false;
        // pf: pair p's polls, current pixels and window were issued during pair p - 1
        bool pf = false;
        unsigned long long pval[4] = {0ull, 0ull, 0ull, 0ull};
        uint32_t pcur4 = 0;
        uint32_t pnv[EM > 0 ? EM : 1];
        int p = 0;
        while (p < ch.len) {
            if ((p >> 5) != wi) {
                wi = p >> 5;
                wT = (uint32_t)uni((int)ldg32(mo + wi));
                wB = (uint32_t)uni((int)ldg32(mbd + wi));
                wA = (uint32_t)uni((int)ldg32(ma + wi));
                wBn = (uint32_t)uni((int)ldg32(mb + wi));
                wC = (uint32_t)uni((int)ldg32(mc + wi));
            }
            const int b = p & 31;
            if ((wT >> b) & 1u) {
                // a run of transparent pairs (results written by the pre-pass):
                // one publish covers it
                const uint32_t ones = ~(wT >> b);
                int r = ones ? __builtin_ctz(ones) : 32 - b;
                r = min(r, min(32 - b, ch.len - p));
                p += r;
                // the newest history entries are the run's zero vectors
                const uint32_t h0n = enc8(tx, ty);
                const uint32_t g1 = r >= 2 ? 0u : h0n, g2 = r >= 3 ? 0u : (r == 2 ? h0n : hist1);
                hist1 = g1;
                hist2 = g2;
                tx = ty = 0;
                v0 = v1 = pf = false;
                if (l == 0) publish(own, progress_word((uint32_t)p, 0u, hist1, hist2));
                continue;
            }
            const uint32_t dcur = v0 ? d0 : load_desc(jobs + p);
            const DescReg D{dcur};
            // the next pair is searched and in this mask word: its descriptor
            // is fetched now unless it already was, and (staged plan) its
            // polls, current pixels and window are issued during this search
            const bool nxt = p + 1 < ch.len && b < 31 && !((wT >> (b + 1)) & 1u);
            const bool pre = EM > 0 && nxt;
            if (nxt && !v1) {
                d1 = load_desc(jobs + p + 1);
                v1 = true;
            }
            const uint32_t need = (uint32_t)(p + 1);
            // neighbours in this pair; transparent ones contribute (0, 0)
            // without a wait
            const int dep_line = D.i32(DW(dep_line_base));
            const bool t_local = D.i32(DW(t_local)) != 0;
            const bool hasT = dep_line >= 0 && !t_local;
            const bool use[4] = {inA && !((wA >> b) & 1u), inB && !((wBn >> b) & 1u), inC && !((wC >> b) & 1u),
                                 hasT};
            // unused slots poll this line's own word (always readable) and are
            // ignored: branch-free polls stay in flight with the staging loads
            const unsigned long long *const w[4] = {use[0] ? own - 1 : own, use[1] ? own - wm : own,
                                                    use[2] ? own - wm + 1 : own,
                                                    hasT ? a.progress + dep_line + k : own};
            const uint32_t nd[4] = {need, need, need, (uint32_t)(D.i32(DW(dep_pos)) + 1)};
            unsigned long long val[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) val[i] = pf ? pval[i] : ld64(w[i]);
            Ctx c;
            c.shape = ((wB >> b) & 1u) != 0;
            const uint8_t *Pc = c.shape ? D.ptr<const uint8_t>(DW(cur_a)) : D.ptr<const uint8_t>(DW(cur));
            const uint8_t *Pr = c.shape ? D.ptr<const uint8_t>(DW(ref_a)) : D.ptr<const uint8_t>(DW(ref));
            const int st = D.i32(DW(stride));
            c.win = win0;
            c.R = R;
            c.pitch = a.pitch;
            c.S = S;
            set_lane_base(c, (j + S + 1) * a.pitch + 4 * q + S + 1, S);
            c.x0 = x0;
            c.y0 = y0;
            c.W = W;
            c.H = H;
            set_box(c, kp, x0, y0, W, H);
            const uint32_t cur4 = pf ? pcur4 : ldg32((const uint32_t *)(Pc + (size_t)(y0 + j) * st + x0 + 4 * q));
            if (!pf) {
                if constexpr (EM > 0) {
                    uint32_t wv[EM];
                    plan.issue(Pr, st, wv);
                    plan.write(win0, wv, c.shape);
                } else {
                    stage_window(win0, a.pitch, a.rows, Pr, st, W, H, x0, y0, S, c.shape);
                }
            }
            // remaining polls
            int spins = 0;
            for (;;) {
                bool ok = true;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (use[i]) ok = ok && (uint32_t)uni((int)(uint32_t)(val[i] >> 48)) >= nd[i];
                if (ok) break;
                if ((spins & 31) == 31 && (uni((int)ld_relaxed(a.status)) & ST_ABORT)) return;
                if (++spins > kp.spin_limit) {
                    if (l == 0) atomicOr(a.status, ST_SPIN_TIMEOUT | ST_ABORT);
                    return;
                }
                if (kp.poll_sleep == 1)
                    __builtin_amdgcn_s_sleep(1);
                else if (kp.poll_sleep == 2)
                    __builtin_amdgcn_s_sleep(2);
                else if (kp.poll_sleep >= 4)
                    __builtin_amdgcn_s_sleep(4);
#pragma unroll
                for (int i = 0; i < 4; ++i) val[i] = ld64(w[i]);
            }
            asm volatile("" ::: "memory");  // vector reads stay after the polls
            // the window prefetched during the previous pair (a single wave:
            // that pair's reads of the buffer have all returned)
            if constexpr (EM > 0) {
                if (pf) plan.write(win0, pnv, c.shape);
            }
            c.c4 = c.shape ? bin4(cur4) : cur4;
            if ((kp.t_texture || (MP && kp.masked_prs)) && c.shape && !kp.shape_only) {
                c.ref_l = D.ptr<const uint8_t>(DW(ref));
                c.st = st;
                c.tl4 = ldg32((const uint32_t *)(D.ptr<const uint8_t>(DW(cur)) + (size_t)(y0 + j) * st + x0 + 4 * q));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t lo = (uint32_t)uni((int)(uint32_t)val[i]);
                const uint32_t hi = (uint32_t)uni((int)(uint32_t)(val[i] >> 32));
                val[i] = ((unsigned long long)hi << 32) | lo;
            }
            const uint32_t *mvi = D.ptr<const uint32_t>(DW(mv_int));
            const uint32_t *tf = D.ptr<const uint32_t>(DW(tf));
            uint32_t m[4];
            const uint32_t *const arr[4] = {mvi + k - 1, mvi + k - wm, mvi + k - wm + 1, tf + k};
            vectors_of(val, nd, use, arr, m);
            if (!hasT && tf && !(t_local && p > 0)) m[3] = (uint32_t)uni((int)ldg32(tf + k));
            int cx[4], cy[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cx[i] = mvx_full(m[i]);
                cy[i] = mvy_full(m[i]);
            }
            if (t_local && p > 0) {
                cx[3] = tx;
                cy[3] = ty;
            }
            // window writes visible to every lane: the workgroup is one wave,
            // so completing its LDS writes (and a compiler fence) suffices
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            // pair p + 1 while this one is searched: the descriptor of p + 2,
            // then the polls, current pixels and window of p + 1
            bool v2 = false;
            uint32_t d2 = 0;
            if constexpr (EM > 0) {
                if (pre) {
                    if (p + 2 < ch.len && b < 30 && !((wT >> (b + 2)) & 1u)) {
                        d2 = load_desc(jobs + p + 2);
                        v2 = true;
                    }
                    const DescReg Dn{d1};
                    const int bn = b + 1;
                    const int dl_n = Dn.i32(DW(dep_line_base));
                    const bool hasT_n = dl_n >= 0 && Dn.i32(DW(t_local)) == 0;
                    const unsigned long long *const wn[4] = {
                        inA && !((wA >> bn) & 1u) ? own - 1 : own, inB && !((wBn >> bn) & 1u) ? own - wm : own,
                        inC && !((wC >> bn) & 1u) ? own - wm + 1 : own, hasT_n ? a.progress + dl_n + k : own};
#pragma unroll
                    for (int i = 0; i < 4; ++i) pval[i] = ld64(wn[i]);
                    const bool nshape = ((wB >> bn) & 1u) != 0;
                    const uint8_t *Pcn = nshape ? Dn.ptr<const uint8_t>(DW(cur_a)) : Dn.ptr<const uint8_t>(DW(cur));
                    const uint8_t *Prn = nshape ? Dn.ptr<const uint8_t>(DW(ref_a)) : Dn.ptr<const uint8_t>(DW(ref));
                    const int stn = Dn.i32(DW(stride));
                    pcur4 = ldg32((const uint32_t *)(Pcn + (size_t)(y0 + j) * stn + x0 + 4 * q));
                    plan.issue(Prn, stn, pnv);
                }
            }
            const MbOut o = search_mb<MP>(D.ptr<const uint32_t>(DW(seed)), c, k, cx, cy, kp);
            // publish: the wait leaves the next pair's loads (at least the
            // EM + 5 most recent vector-memory operations) in flight
            const unsigned long long word = progress_word(need, enc8(o.dx, o.dy), enc8(tx, ty), hist1);
            if (l == 0) {
                if (pre)
                    publish<(EM > 0 ? EM + 5 : 0)>(own, word);
                else
                    publish(own, word);
            }
            hist2 = hist1;
            hist1 = enc8(tx, ty);
            if (l == 0) store_result(D, k, o.mv, o.mvi, o.cost, o.iters, o.points);
            tx = o.dx;
            ty = o.dy;
            pf = pre;
            d0 = d1;
            v0 = v1;
            d1 = d2;
            v1 = v2;
            ++p;
        }
    }
}


// ------------------------------------------------- several waves per line
// Shifted history: the three vectors of pairs c-1+g, c-2+g, c-3+g given the
// word of count c (the g pairs in between are transparent: zero vectors).
__device__ __forceinline__ void shift_hist(unsigned long long w, uint32_t g, uint32_t (&h)[3]) {
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k) h[k] = k >= g ? hist_of(w, k - g) : 0u;
}

typedef __attribute__((address_space(3))) volatile int l_vint;
typedef __attribute__((address_space(3))) volatile unsigned long long l_vu64;

__device__ __forceinline__ void publish_max(unsigned long long *p, unsigned long long word) {
    typedef __attribute__((address_space(1))) unsigned long long g_u64;
    __hip_atomic_fetch_max((g_u64 *)p, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The recursion of Section 3.2 from (dx, dy) at distortion dc (nothing when k_max = 0).
__device__ __forceinline__ int recurse_from(const Ctx &c, const KParams &kp, int &dx, int &dy, int &dc) {
    if (kp.k_max <= 0) return 0;
    return pel_recursion(c, kp, dx, dy, dc, sweep(c, dx, dy));
}

// NW (2 to 8) waves per line.  The i-th searched pair of the line (in pair
// order) belongs to wave i % NW.  Everything of a pair that does not need its T
// candidate (the previous pair's vector, which the preceding wave produces) is
// done first: polls, window staging, the costs of A, B, C, the recursion from
// their first minimum (and from the learned seed).  T then arrives through
// LDS; its cost decides whether that speculative result stands (T is last in
// the list, so it wins only with a strictly lower cost) or the recursion is
// redone from T.  The vector is handed to the next wave at once; the
// progress word is published with a 64-bit atomic max (count in the top
// bits, so publishes from the waves can land in any order), and the
// half-sample refinement and the result stores follow.
template <int EM, int NW>
__global__ __launch_bounds__(64 * NW) void pa2_kernel(PaArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int slot;
    __shared__ unsigned long long hword;  // progress word after the latest handed-off pair
    __shared__ int hseq;                  // its index among the line's searched pairs (-1: none)
    __shared__ int sdone[NW];             // per wave: latest own pair whose result stores completed
    __shared__ int hpos[8];               // pair position of searched pair j, at j & 7
    __shared__ int ab;                    // a wave left the line on an abort
    __shared__ int stop;                  // the status word asked every worker to leave
    short *R = (short *)lds;              // 511 reciprocal entries (Eq. 4-5, Q.12)
    const int wv = threadIdx.x >> 6;
    const int wwords = ((a.rows * a.pitch + 16) >> 2) + 4;
    uint32_t *const win = lds + 256 + wv * wwords;  // this wave's staged reference window
    const KParams kp = a.kp;
    for (int g = threadIdx.x; g < 511; g += 64 * NW) {
        const int m = abs(g - 255);
        const int r = (m == 0 || m < 2 * kp.theta) ? 0 : (16384 + m) / (2 * m);
        R[g] = (short)(g < 255 ? -r : r);
    }
    // LDS (not generic) pointers: a volatile access through a generic pointer
    // becomes a flat access that waits for every outstanding vector-memory
    // operation, the progress atomic and the prefetches included
    l_vint *const vhseq = (l_vint *)&hseq;
    l_vu64 *const vhword = (l_vu64 *)&hword;
    l_vint *const vsdone = (l_vint *)sdone;
    l_vint *const vab = (l_vint *)&ab;
    l_vint *const vhpos = (l_vint *)hpos;
    const int l = lane(), j = l >> 2, q = l & 3;
    const int S = kp.S;
    const int nact = (int)uni((int)ldg32(a.nactive));
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            slot = (int)atomicAdd(a.counter, 1u);
            hseq = -1;
            hword = 0ull;
            for (int u = 0; u < NW; ++u) sdone[u] = -1;
            ab = 0;
            stop = (int)(ld_relaxed(a.status) & ST_ABORT);
        }
        __syncthreads();
        const int t = uni(slot);
        if (t >= nact || uni(stop)) break;  // LDS values: the same decision in every wave
        const uint32_t tk = a.tickets[t];
        const int ci = (int)(tk >> 16), v = (int)((tk >> 8) & 0xFF), h = (int)(tk & 0xFF);
        const ChainDesc ch = a.chains[ci];
        const int wm = ch.wm;
        const int k = v * wm + h;
        const JobDesc *jobs = a.jobs + ch.first;
        const int line = ch.line_base + k;
        unsigned long long *const own = a.progress + line;
        const int x0 = 16 * h, y0 = 16 * v;
        const int W = 16 * ch.wm, H = 16 * ch.hm;
        const bool inA = h > 0, inB = v > 0, inC = v > 0 && h + 1 < wm;
        const uint32_t *mo = a.tmask + (size_t)line * a.mw;
        const uint32_t *mbd = a.bmask + (size_t)line * a.mw;
        const uint32_t *ma = a.tmask + (size_t)(inA ? line - 1 : line) * a.mw;
        const uint32_t *mb = a.tmask + (size_t)(inB ? line - wm : line) * a.mw;
        const uint32_t *mc = a.tmask + (size_t)(inC ? line - wm + 1 : line) * a.mw;
        Plan<(EM > 0 ? EM : 1)> plan;
        if (EM > 0) plan.init(a.pitch, a.rows, x0, y0, S, W, H);
        uint32_t wT = 0, wB = 0, wA = 0, wBn = 0, wC = 0;
        int wi = -1;
        int i = 0;        // searched pairs seen so far on this line
        int myprev = -1;  // index of this wave's latest pair (its stores may be in flight)
        bool aborted = false;
        int p = 0;
        while (p < ch.len) {
            if ((p >> 5) != wi) {
                wi = p >> 5;
                wT = (uint32_t)uni((int)ldg32(mo + wi));
                wB = (uint32_t)uni((int)ldg32(mbd + wi));
                wA = (uint32_t)uni((int)ldg32(ma + wi));
                wBn = (uint32_t)uni((int)ldg32(mb + wi));
                wC = (uint32_t)uni((int)ldg32(mc + wi));
            }
            const int b = p & 31;
            if ((wT >> b) & 1u) {
                const uint32_t ones = ~(wT >> b);
                int r = ones ? __builtin_ctz(ones) : 32 - b;
                p += min(r, min(32 - b, ch.len - p));
                continue;
            }
            if (i % NW != wv) {  // another wave's pair
                ++i;
                ++p;
                continue;
            }
            // ---- this wave's pair p (the i-th searched one): work without T
            const DescReg D{load_desc(jobs + p)};
            const uint32_t need = (uint32_t)(p + 1);
            const int dep_line = D.i32(DW(dep_line_base));
            const bool t_local = D.i32(DW(t_local)) != 0;
            const bool hasT = dep_line >= 0 && !t_local;
            const bool use[4] = {inA && !((wA >> b) & 1u), inB && !((wBn >> b) & 1u), inC && !((wC >> b) & 1u),
                                 hasT};
            const unsigned long long *const w[4] = {use[0] ? own - 1 : own, use[1] ? own - wm : own,
                                                    use[2] ? own - wm + 1 : own,
                                                    hasT ? a.progress + dep_line + k : own};
            const uint32_t nd[4] = {need, need, need, (uint32_t)(D.i32(DW(dep_pos)) + 1)};
            unsigned long long val[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) val[u] = ld64(w[u]);
            Ctx c;
            c.shape = ((wB >> b) & 1u) != 0;
            const uint8_t *Pc = c.shape ? D.ptr<const uint8_t>(DW(cur_a)) : D.ptr<const uint8_t>(DW(cur));
            const uint8_t *Pr = c.shape ? D.ptr<const uint8_t>(DW(ref_a)) : D.ptr<const uint8_t>(DW(ref));
            const int st = D.i32(DW(stride));
            c.win = win;
            c.R = R;
            c.pitch = a.pitch;
            c.S = S;
            set_lane_base(c, (j + S + 1) * a.pitch + 4 * q + S + 1, S);
            c.x0 = x0;
            c.y0 = y0;
            c.W = W;
            c.H = H;
            set_box(c, kp, x0, y0, W, H);
            const uint32_t cur4 = ldg32((const uint32_t *)(Pc + (size_t)(y0 + j) * st + x0 + 4 * q));
            if constexpr (EM > 0) {
                uint32_t wv4[EM];
                plan.issue(Pr, st, wv4);
                plan.write(win, wv4, c.shape);
            } else {
                stage_window(win, a.pitch, a.rows, Pr, st, W, H, x0, y0, S, c.shape);
            }
            // the window loads have returned, so this wave's earlier result
            // stores (issued before them) have completed
            if (l == 0) vsdone[wv] = myprev;
            c.c4 = c.shape ? bin4(cur4) : cur4;
            // polls: the first slot still short of its count is read with three
            // loads in flight (a new one every few hundred cycles), so a
            // publish is seen about a third of a memory round trip after it
            // lands rather than up to a whole one
            int spins = 0;
            unsigned long long g0 = 0, g1 = 0, g2 = 0;  // the last two may still be in flight
            for (;;) {
                int ms = -1;
#pragma unroll
                for (int u = 3; u >= 0; --u)
                    if (use[u] && (uint32_t)uni((int)(uint32_t)(val[u] >> 48)) < nd[u]) ms = u;
                if (ms < 0) break;
                const unsigned long long *pw = ms == 0 ? w[0] : ms == 1 ? w[1] : ms == 2 ? w[2] : w[3];
                const uint32_t want = ms == 0 ? nd[0] : ms == 1 ? nd[1] : ms == 2 ? nd[2] : nd[3];
                unsigned long long got = 0ull;
                g0 = ld64(pw);
                __builtin_amdgcn_s_sleep(3);
                g1 = ld64(pw);
                __builtin_amdgcn_s_sleep(3);
                for (;;) {
                    g2 = ld64(pw);
                    if ((uint32_t)uni((int)(uint32_t)(g0 >> 48)) >= want) {
                        got = g0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(3);
                    g0 = ld64(pw);
                    if ((uint32_t)uni((int)(uint32_t)(g1 >> 48)) >= want) {
                        got = g1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(3);
                    g1 = ld64(pw);
                    if ((uint32_t)uni((int)(uint32_t)(g2 >> 48)) >= want) {
                        got = g2;
                        break;
                    }
                    spins += 3;
                    if ((spins & 31) < 3 && (uni((int)ld_relaxed(a.status)) & ST_ABORT)) {
                        aborted = true;
                        break;
                    }
                    if (spins > kp.spin_limit) {
                        if (l == 0) atomicOr(a.status, ST_SPIN_TIMEOUT | ST_ABORT);
                        aborted = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(3);
                }
                if (aborted) break;
                if (ms == 0)
                    val[0] = got;
                else if (ms == 1)
                    val[1] = got;
                else if (ms == 2)
                    val[2] = got;
                else
                    val[3] = got;
            }
            if (aborted) break;
            asm volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t lo = (uint32_t)uni((int)(uint32_t)val[u]);
                const uint32_t hi = (uint32_t)uni((int)(uint32_t)(val[u] >> 32));
                val[u] = ((unsigned long long)hi << 32) | lo;
            }
            const uint32_t *mvi = D.ptr<const uint32_t>(DW(mv_int));
            const uint32_t *tf = D.ptr<const uint32_t>(DW(tf));
            uint32_t m[4];
            const uint32_t *const arr[4] = {mvi + k - 1, mvi + k - wm, mvi + k - wm + 1, tf + k};
            vectors_of(val, nd, use, arr, m);
            // T when it does not come from the preceding wave
            uint32_t tm = m[3];
            if (!hasT && tf && !(t_local && p > 0)) tm = (uint32_t)uni((int)ldg32(tf + k));
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // window visible to the whole wave
            // A, B, C: admissible distinct entries, first minimum
            int cx[3], cy[3];
            bool keep[3];
            int nabc = 0;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                cx[u] = mvx_full(m[u]);
                cy[u] = mvy_full(m[u]);
                bool ok = cx[u] >= c.lox && cx[u] <= c.hix && cy[u] >= c.loy && cy[u] <= c.hiy;
#pragma unroll
                for (int pq = 0; pq < u; ++pq) ok = ok && !(keep[pq] && cx[pq] == cx[u] && cy[pq] == cy[u]);
                keep[u] = ok;
                nabc += ok;
            }
            uint32_t blk[3];
#pragma unroll
            for (int u = 0; u < 3; ++u)
                blk[u] = wread4(c, iclamp(cy[u], -S, S) * c.pitch + iclamp(cx[u], -S, S));
            const int p01 = wave_sum((int)__builtin_amdgcn_sad_u8(c.c4, blk[0], 0u) |
                                     ((int)__builtin_amdgcn_sad_u8(c.c4, blk[1], 0u) << 16));
            const int p2 = wave_sum((int)__builtin_amdgcn_sad_u8(c.c4, blk[2], 0u));
            const int craw[3] = {p01 & 0xFFFF, (int)((uint32_t)p01 >> 16), p2};
            int bx = 0, by = 0, bc = 0x7FFFFFFF;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int cu = cost_of(c, craw[u]);
                if (keep[u] && cu < bc) {
                    bc = cu;
                    bx = cx[u];
                    by = cy[u];
                }
            }
            // speculative recursion from the A/B/C winner, and the learned start
            int sdx = bx, sdy = by, sdc = bc, sits = 0;
            if (nabc > 0) sits = recurse_from(c, kp, sdx, sdy, sdc);
            const uint32_t *seed = D.ptr<const uint32_t>(DW(seed));
            const bool seeded = seed && !c.shape;
            int lx = 0, ly = 0, lc = 0, lits = 0;
            if (seeded) {
                const uint32_t sw0 = (uint32_t)uni((int)ldg32(seed + k));
                lx = iclamp(mvx_full(sw0), c.lox, c.hix);
                ly = iclamp(mvy_full(sw0), c.loy, c.hiy);
                const Sweep sws = sweep(c, lx, ly);
                lc = cost_of(c, sws.sad);
                lits = pel_recursion(c, kp, lx, ly, lc, sws);
            }
            // ---- T: from the preceding wave's hand-off (or known already)
            for (int sp = 0; uni(*vhseq) != i - 1; ++sp) {
                if (sp > kp.spin_limit) {
                    if (l == 0) atomicOr(a.status, ST_SPIN_TIMEOUT | ST_ABORT);
                    aborted = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (aborted) break;
            asm volatile("" ::: "memory");
            const unsigned long long hw = *vhword;
            const unsigned long long prevw = (unsigned long long)(uint32_t)uni((int)(uint32_t)hw) |
                                             ((unsigned long long)(uint32_t)uni((int)(uint32_t)(hw >> 32)) << 32);
            const uint32_t gap = need - 1 - count_of(prevw);  // transparent pairs since the previous searched one
            uint32_t hs[3];
            shift_hist(prevw, gap, hs);  // vectors of pairs p-1, p-2, p-3
            int tx = 0, ty = 0;
            if (t_local && p > 0) {
                tx = (int)(int8_t)(hs[0] & 0xFF);
                ty = (int)(int8_t)(hs[0] >> 8);
            } else {
                tx = mvx_full(tm);
                ty = mvy_full(tm);
            }
            bool keepT = tx >= c.lox && tx <= c.hix && ty >= c.loy && ty <= c.hiy;
#pragma unroll
            for (int u = 0; u < 3; ++u) keepT = keepT && !(keep[u] && cx[u] == tx && cy[u] == ty);
            int n = nabc + (keepT ? 1 : 0);
            int dx, dy, dc, its;
            int wx = bx, wy = by, wc = bc;  // BRS winner
            bool from_spec = nabc > 0;
            if (keepT) {
                const int ct = cost_of(c, wave_sum((int)__builtin_amdgcn_sad_u8(
                                              c.c4, wread4(c, ty * c.pitch + tx), 0u)));
                if (ct < wc) {
                    wx = tx;
                    wy = ty;
                    wc = ct;
                    from_spec = false;
                }
            }
            if (n == 0) {  // nothing admissible: (0, 0)
                n = 1;
                wx = wy = 0;
                wc = cost_of(c, wave_sum((int)__builtin_amdgcn_sad_u8(c.c4, wread4(c, 0), 0u)));
                from_spec = false;
            }
            int pts = n;
            if (seeded) {
                pts += 1 + lits;
                its = lits;
                if (20ll * lc > 21ll * wc) {
                    dx = wx;
                    dy = wy;
                    dc = wc;
                    int it2;
                    if (from_spec) {
                        dx = sdx;
                        dy = sdy;
                        dc = sdc;
                        it2 = sits;
                    } else {
                        it2 = recurse_from(c, kp, dx, dy, dc);
                    }
                    its += it2;
                    pts += it2;
                } else {
                    dx = lx;
                    dy = ly;
                    dc = lc;
                }
            } else if (from_spec) {
                dx = sdx;
                dy = sdy;
                dc = sdc;
                its = sits;
                pts += its;
            } else {
                dx = wx;
                dy = wy;
                dc = wc;
                its = recurse_from(c, kp, dx, dy, dc);
                pts += its;
            }
            const unsigned long long word = progress_word(need, enc8(dx, dy), hs[0], hs[1]);
            // count `need` promises the stores of pairs <= need - 4 (p - 3).
            // This wave's earlier pairs are complete (its window loads came
            // after their stores); so are the other waves' pairs before their
            // latest ones (handed off after their own window loads).  What
            // may still be in flight: the other waves' latest pairs i - 1 ..
            // i - NW + 1, which count only when a transparent run puts them
            // three or more pairs back.
#pragma unroll
            for (int d = 1; d < NW; ++d) {
                const int jj = i - d;
                if (jj < 0 || aborted) break;
                if ((int)uni(vhpos[jj & 7]) > p - 3) continue;
                for (int sp = 0; uni(vsdone[jj % NW]) < jj; ++sp) {
                    if (sp > kp.spin_limit) {
                        if (l == 0) atomicOr(a.status, ST_SPIN_TIMEOUT | ST_ABORT);
                        aborted = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (aborted) break;
            if (l == 0) {
                publish_max(own, word);
                *vhword = word;
                vhpos[i & 7] = p;
                asm volatile("" ::: "memory");
                *vhseq = i;
            }
            // ---- after the hand-off: half-sample refinement, results
            int hx = 2 * dx, hy = 2 * dy;
            if (kp.half_pel && !c.shape) pts += half_refine(c, kp, dx, dy, hx, hy, dc);
            if (l == 0) {
                const DescReg &Dr = D;
                store_result(Dr, k, pack_mv(hx, hy), pack_mv(2 * dx, 2 * dy), (uint32_t)dc, its, pts);
            }
            asm volatile("" ::"v"(g0), "v"(g1), "v"(g2));  // poll loads still in flight complete here
            myprev = i;
            ++i;
            ++p;
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (l == 0) {
            vsdone[wv] = myprev;
            if (aborted) *vab = 1;
        }
        __syncthreads();
        const bool any_abort = uni(*vab) != 0;
        if (threadIdx.x == 0 && !any_abort) {
            // trailing transparent pairs: the line's final count
            const unsigned long long wlast = hword;
            const uint32_t cnt = count_of(wlast);
            if (cnt < (uint32_t)ch.len) {
                uint32_t hs[3];
                shift_hist(wlast, (uint32_t)ch.len - cnt, hs);
                publish_max(own, progress_word((uint32_t)ch.len, hs[0], hs[1], hs[2]));
            }
        }
        if (any_abort) break;  // the same decision in every wave
    }
}

// ------------------------------------------------------------- row workers
// Job sets with no chain inside the call (every T field is already in
// memory, as in a batched frame step).  A workgroup of NR waves takes a
// "band" of NR consecutive MB rows of one job; wave r walks row v0 + r from
// left to right.  MB (h, v) needs A = the wave's own previous MB (a
// register), B = (h, v-1) and C = (h+1, v-1) from the wave above through
// LDS - or, for the band's first row, from the previous band's last row
// through a per-row progress count in device memory and that row's mv_int
// array - and T from memory.  Bands are handed out in (first row, job)
// order, a topological order of these dependencies, so the schedule cannot
// deadlock at any residency.  A row's transparent MBs get their zero results
// here (no pre-pass); a neighbour transparent in the pair contributes (0, 0)
// and is never waited for.  Every wait is bounded; on timeout a status bit
// is raised and the workers leave.

struct PrArgs {
    const JobDesc *jobs;  // chain-ordered descriptors (one job per chain)
    const ChainDesc *chains;
    const uint32_t *bands;          // chain << 16 | first row, in (first row, chain) order
    int nbands;
    unsigned long long *rowprog;    // per chain, from its line_base: MBs of row v done (count in the low half)
    uint32_t *counter;
    uint32_t *status;
    KParams kp;
    int pitch, rows;
};

typedef __attribute__((address_space(3))) volatile uint32_t l_vu32;

// Row progress word (one per MB row of a band-last row): bits 0-8 the count
// of the row's MBs done (every MB before that position), bits 9-17 and 18-26
// the positions of the two latest searched MBs (511: none), bits 32-47 and
// 48-63 their full-pel vectors as two signed bytes each (|d| <= 64).  The
// result arrays of every other MB before the count are complete when the
// word is published: a row worker issues an MB's result stores one MB late,
// before the loads of the window after next, and waits for those loads
// before it publishes again; the vector-memory counter completes in issue
// order.
constexpr uint32_t kNoPos = 511u;
__device__ __forceinline__ unsigned long long row_word(uint32_t count, uint32_t p, uint32_t vp, uint32_t q, uint32_t vq) {
    return (unsigned long long)(count | (p << 9) | (q << 18)) | ((unsigned long long)vp << 32) |
           ((unsigned long long)vq << 48);
}
__device__ __forceinline__ uint32_t enc_full(uint32_t mvi) { return enc8(mvx_full(mvi), mvy_full(mvi)); }
__device__ __forceinline__ uint32_t dec_full(uint32_t e) {
    return pack_mv(2 * (int)(int8_t)(e & 0xFF), 2 * (int)(int8_t)(e >> 8));
}

// Window loads of one MB, issued ahead.  Column-major: the window's dw =
// pitch / 4 dword columns are spread over the lanes, g = 64 / dw lanes per
// column; lane l (taken modulo g * dw, so spare lanes repeat the first ones)
// holds column l % dw and rows l / dw + u * g, u < EM = ceil(rows / g).
// Only the last element can fall past the window; it repeats the last row
// (the same bytes to the same place).  The column's frame clamp and edge
// byte selector are worked out once per MB, so an element costs one offset
// step, one load and one LDS store; rows are clamped per element only when
// the window crosses the top or bottom frame edge.
template <int EM>
struct RowWin {
    uint32_t v[EM];
    uint32_t sel;
    int shape, edge;  // wave-uniform
    __device__ __forceinline__ void issue(const uint8_t *P, int st, int W, int H, int x0, int y0, int S, int pitch,
                                          int rows, bool shape_) {
        shape = uni(shape_ ? 1 : 0);
        // the plane in scalar registers: each load is a 32-bit lane offset
        // from a scalar base (one add per element)
        const uint8_t *const Pu = (const uint8_t *)(uintptr_t)uni64((unsigned long long)(uintptr_t)P);
        const int dw = pitch >> 2, g = 64 / dw;
        const int l = lane() % (g * dw), c = l % dw, r0 = l / dw;
        const int xx = x0 - S - 1 + 4 * c;
        const int xc = iclamp(xx, 0, W - 4);
        edge = __ballot(xx < 0 || xx + 3 > W - 1) != 0ull;
        sel = (uint32_t)(iclamp(xx, 0, W - 1) - xc) | ((uint32_t)(iclamp(xx + 1, 0, W - 1) - xc) << 8) |
              ((uint32_t)(iclamp(xx + 2, 0, W - 1) - xc) << 16) | ((uint32_t)(iclamp(xx + 3, 0, W - 1) - xc) << 24);
        const int wy0 = y0 - S - 1;
        if (wy0 >= 0 && wy0 + rows <= H) {  // no row clamp (wave-uniform)
            const uint32_t o0 = (uint32_t)(wy0 + r0) * (uint32_t)st + (uint32_t)xc;
            const uint32_t gst = (uint32_t)uni(g * st);
#pragma unroll
            for (int u = 0; u < EM - 1; ++u) v[u] = ld4(Pu + (size_t)(o0 + (uint32_t)u * gst));
            const int rl = min(r0 + (EM - 1) * g, rows - 1);
            v[EM - 1] = ld4(Pu + (size_t)((uint32_t)(wy0 + rl) * (uint32_t)st + (uint32_t)xc));
        } else {
#pragma unroll
            for (int u = 0; u < EM; ++u) {
                const int r = min(r0 + u * g, rows - 1);
                v[u] = ld4(Pu + (size_t)((uint32_t)iclamp(wy0 + r, 0, H - 1) * (uint32_t)st + (uint32_t)xc));
            }
        }
    }
    __device__ __forceinline__ void write(uint32_t *win, int pitch, int rows) {
        const int dw = pitch >> 2, g = 64 / dw;
        const int l = lane() % (g * dw), c = l % dw, r0 = l / dw;
        if (edge) {
#pragma unroll
            for (int u = 0; u < EM; ++u) v[u] = __builtin_amdgcn_perm(v[u], v[u], sel);
        }
        if (shape) {
#pragma unroll
            for (int u = 0; u < EM; ++u) v[u] = bin4(v[u]);
        }
        uint32_t *const wl = win + r0 * dw + c;
        const int gdw = g * dw;
#pragma unroll
        for (int u = 0; u < EM - 1; ++u) wl[u * gdw] = v[u];
        win[min(r0 + (EM - 1) * g, rows - 1) * dw + c] = v[EM - 1];
    }
};

// dwords per lane of the column-major window staging for range S (0: the
// generic loop): ceil(rows / g) where instantiated (S = 7, 16, 32)
__host__ __device__ inline int row_elems(int S) {
    const int rows = 2 * S + 18, dw = ((rows + 3) & ~3) >> 2, g = 64 / dw;
    const int e = g > 0 ? (rows + g - 1) / g : 0;
    return e == 4 || e == 13 || e == 28 ? e : 0;
}

// First MB index >= from whose bit is set in the 256-bit row mask m (wm: none).
__device__ __forceinline__ int next_set(const unsigned long long (&m)[4], int from, int wm) {
    for (int w = from >> 6; w < 4; ++w) {
        const int b = from > 64 * w ? from - 64 * w : 0;
        const unsigned long long x = b >= 64 ? 0ull : (m[w] >> b) << b;
        if (x) return min(64 * w + __builtin_ctzll(x), wm);
    }
    return wm;
}

__device__ __forceinline__ bool bit_of(const unsigned long long (&m)[4], int h) { return (m[h >> 6] >> (h & 63)) & 1ull; }

// DB: two windows per wave, and each MB's half-sample step one MB late (it
// does not feed any neighbour): the next MB's block-recursive and
// pel-recursive steps, which do, are not held up by it, and a row waiting
// for the row above runs it in that wait.
template <int EM, int NR, bool DB, bool MP = false>
__global__ __launch_bounds__(64 * NR) void pr_kernel(PrArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int slot;
    __shared__ int stop;
    __shared__ int ab;
    __shared__ int prog[NR];              // per wave: MBs of its row done
    __shared__ uint32_t vecs[NR * 256];   // per wave: its row's full-pel vectors (half-pel units, packed)
    short *R = (short *)lds;              // 511 reciprocal entries (Eq. 4-5, Q.12)
    const int wv = threadIdx.x >> 6;
    const int wwords = ((a.rows * a.pitch + 16) >> 2) + 4;
    uint32_t *const win0 = lds + 256 + wv * (DB ? 2 : 1) * wwords;
    const KParams kp = a.kp;
    for (int g = threadIdx.x; g < 511; g += 64 * NR) {
        const int m = abs(g - 255);
        const int r = (m == 0 || m < 2 * kp.theta) ? 0 : (16384 + m) / (2 * m);
        R[g] = (short)(g < 255 ? -r : r);
    }
    l_vint *const vprog = (l_vint *)prog;
    l_vu32 *const vvec = (l_vu32 *)vecs;
    l_vint *const vab = (l_vint *)&ab;
    const int l = lane(), j = l >> 2, q = l & 3;
    const int S = kp.S;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            slot = (int)atomicAdd(a.counter, 1u);
            stop = (int)(ld_relaxed(a.status) & ST_ABORT);
            ab = 0;
        }
        if (threadIdx.x < NR) prog[threadIdx.x] = 0;
        __syncthreads();
        const int t = uni(slot);
        if (t >= a.nbands || uni(stop)) break;  // LDS values: the same decision in every wave
        const uint32_t tk = a.bands[t];
        const ChainDesc ch = a.chains[tk >> 16];
        const int wm = ch.wm, hm = ch.hm;
        const int v = (int)(tk & 0xFFFF) + wv;
        bool aborted = false;
        if (v < hm) {
            const DescReg D{load_desc(a.jobs + ch.first)};
            const uint8_t *cls = D.ptr<const uint8_t>(DW(cls));
            const int W = 16 * wm, H = 16 * hm, st = D.i32(DW(stride));
            // classes of this row and of the row above: MB h = l + 64 m in lane l
            unsigned long long srch[4], upn[4], bnd[4];
            {
                int cl[4], cu[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int h = l + 64 * m;
                    cl[m] = h < wm ? (cls ? (int)ldg8(cls + v * wm + h) : ME_MB_OPAQUE) : ME_MB_TRANSPARENT;
                    cu[m] = (h < wm && v > 0) ? (cls ? (int)ldg8(cls + (v - 1) * wm + h) : ME_MB_OPAQUE)
                                              : ME_MB_TRANSPARENT;
                }
                bool bad = false;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    bad = bad || cl[m] > ME_MB_BOUNDARY;
                    const bool sr = cl[m] == ME_MB_OPAQUE || cl[m] == ME_MB_BOUNDARY;
                    srch[m] = __ballot(sr);
                    bnd[m] = __ballot(sr && (cl[m] == ME_MB_BOUNDARY || kp.shape_only));
                    upn[m] = __ballot(cu[m] == ME_MB_OPAQUE || cu[m] == ME_MB_BOUNDARY);
                }
                if (bad) atomicOr(a.status, ST_BAD_CLASS);
                // transparent MBs (and bad class bytes, taken as transparent):
                // zero results; every vector of the row starts at zero in LDS
                uint32_t *mv = D.ptr<uint32_t>(DW(mv));
                uint32_t *mvi = D.ptr<uint32_t>(DW(mv_int));
                uint32_t *co = D.ptr<uint32_t>(DW(cost));
                uint8_t *it = D.ptr<uint8_t>(DW(iters));
                uint16_t *pt = D.ptr<uint16_t>(DW(points));
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int h = l + 64 * m;
                    vvec[wv * 256 + h] = 0u;
                    if (h < wm && !((srch[m] >> l) & 1ull)) {
                        const int k = v * wm + h;
                        ((g_u32 *)mv)[k] = 0u;
                        ((g_u32 *)mvi)[k] = 0u;
                        if (co) ((g_u32 *)co)[k] = 0u;
                        if (it) ((g_u8 *)it)[k] = 0;
                        if (pt) ((g_u16 *)pt)[k] = 0;
                    }
                }
            }
            unsigned long long *const gprog = a.rowprog + ch.line_base + v;
            const bool pub_global = wv == NR - 1 && v + 1 < hm;  // the next band's first row reads it
            const uint32_t *mvi_up = D.ptr<const uint32_t>(DW(mv_int)) + (v > 0 ? (v - 1) * wm : 0);
            const uint32_t *tf = D.ptr<const uint32_t>(DW(tf));
            const uint32_t *seed = D.ptr<const uint32_t>(DW(seed));
            int h = next_set(srch, 0, wm);
            // the transparent MBs before the first searched one are done
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (l == 0) {
                vprog[wv] = h;
                if (pub_global) publish(gprog, row_word((uint32_t)h, kNoPos, 0u, kNoPos, 0u));
            }
            RowWin<(EM > 0 ? EM : 1)> nw;
            uint32_t ncur = 0, nt = 0;
            // pixels, window and T of searched MB hh, issued ahead
            auto issue = [&](int hh) {
                const bool sh = bit_of(bnd, hh);
                const uint8_t *Pc = sh ? D.ptr<const uint8_t>(DW(cur_a)) : D.ptr<const uint8_t>(DW(cur));
                const uint8_t *Pr = sh ? D.ptr<const uint8_t>(DW(ref_a)) : D.ptr<const uint8_t>(DW(ref));
                ncur = ldg32((const uint32_t *)(Pc + (size_t)(16 * v + j) * st + 16 * hh + 4 * q));
                nt = tf ? ldg32(tf + v * wm + hh) : 0u;
                if constexpr (EM > 0) nw.issue(Pr, st, W, H, 16 * hh, 16 * v, S, a.pitch, a.rows, sh);
            };
            if (h < wm) issue(h);
            uint32_t lastv = 0u;  // vector of MB h - 1 when it was searched
            int lasth = -2;
            // results of the previous searched MB, stored one MB late (after
            // the next window's loads have arrived): so that waiting for a
            // window never waits for result stores still in flight
            bool pend = false;
            int pk = 0, piters = 0, ppoints = 0;
            uint32_t pmv = 0u, pmvi = 0u, pcost = 0u;
            // DB: the previous MB's half-sample step is still to do (its
            // window is the other buffer, its pixels pc4, position px0, py0,
            // full-pel vector pdx, pdy)
            bool phalf = false;
            int px0 = 0, py0 = 0, pdx = 0, pdy = 0;
            uint32_t pc4 = 0u;
            int cb = 0;  // DB: the buffer of this MB's window
            unsigned long long wseen = 0ull;  // the latest row word seen (first row of a band)
            while (h < wm) {
                const int k = v * wm + h;
                const int x0 = 16 * h, y0 = 16 * v;
                uint32_t *const win = win0 + (DB ? cb * wwords : 0);
                Ctx c;
                c.shape = bit_of(bnd, h);
                if constexpr (EM > 0) {
                    nw.write(win, a.pitch, a.rows);
                } else {
                    const uint8_t *Pr = c.shape ? D.ptr<const uint8_t>(DW(ref_a)) : D.ptr<const uint8_t>(DW(ref));
                    stage_window(win, a.pitch, a.rows, Pr, st, W, H, x0, y0, S, c.shape);
                }
                if constexpr (DB) {
                    // the previous MB's half-sample step, from its window in the other buffer
                    if (phalf) {
                        Ctx cp;
                        cp.win = win0 + (cb ^ 1) * wwords;
                        cp.pitch = a.pitch;
                        cp.S = S;
                        set_lane_base(cp, (j + S + 1) * a.pitch + 4 * q + S + 1, S);
                        cp.x0 = px0;
                        cp.y0 = py0;
                        cp.W = W;
                        cp.H = H;
                        cp.c4 = pc4;
                        cp.shape = false;
                        int hx = 2 * pdx, hy = 2 * pdy, hc = (int)pcost;
                        ppoints += half_refine(cp, kp, pdx, pdy, hx, hy, hc);
                        pmv = pack_mv(hx, hy);
                        pcost = (uint32_t)hc;
                    }
                }
                const uint32_t cur4 = ncur, tv = nt;
                const int h2 = next_set(srch, h + 1, wm);
                // the previous searched MB's results (issued before the next
                // window's loads, so that waiting for that window does not wait
                // for stores issued after it), then the next window's loads, in
                // flight during the poll and this MB's search
                if (pend && l == 0) store_result(D, pk, pmv, pmvi, pcost, piters, ppoints);
                if (h2 < wm) issue(h2);
                // B and C from the row above, once that row is far enough
                const bool useB = v > 0 && bit_of(upn, h);
                const bool useC = v > 0 && h + 1 < wm && bit_of(upn, h + 1);
                const int need = useC ? h + 2 : useB ? h + 1 : 0;
                uint32_t mB = 0u, mC = 0u;
                if (need > 0) {
                    int spins = 0;
                    for (;;) {
                        int got;
                        if (wv > 0) {
                            got = uni(vprog[wv - 1]);
                        } else {
                            if ((int)(uint32_t)(wseen & 0x1FFull) < need)
                                wseen = (unsigned long long)uni64(ld64(a.rowprog + ch.line_base + v - 1));
                            got = (int)(uint32_t)(wseen & 0x1FFull);
                        }
                        if (got >= need) break;
                        if ((spins & 31) == 31 && (uni((int)ld_relaxed(a.status)) & ST_ABORT)) {
                            aborted = true;
                            break;
                        }
                        if (++spins > kp.spin_limit) {
                            if (l == 0) atomicOr(a.status, ST_SPIN_TIMEOUT | ST_ABORT);
                            aborted = true;
                            break;
                        }
                        if (kp.poll_sleep >= 4)
                            __builtin_amdgcn_s_sleep(4);
                        else if (kp.poll_sleep == 2)
                            __builtin_amdgcn_s_sleep(2);
                        else
                            __builtin_amdgcn_s_sleep(1);
                    }
                    if (aborted) break;
                    asm volatile("" ::: "memory");  // vector reads stay after the poll
                    if (wv > 0) {
                        mB = useB ? (uint32_t)uni((int)vvec[(wv - 1) * 256 + h]) : 0u;
                        mC = useC ? (uint32_t)uni((int)vvec[(wv - 1) * 256 + h + 1]) : 0u;
                    } else {
                        // the two latest searched MBs come with the word; the
                        // arrays hold every other one
                        const uint32_t lo = (uint32_t)wseen, hi = (uint32_t)(wseen >> 32);
                        const uint32_t p0 = (lo >> 9) & 0x1FFu, p1 = (lo >> 18) & 0x1FFu;
                        const bool bw = useB && ((uint32_t)h == p0 || (uint32_t)h == p1);
                        const bool cw = useC && ((uint32_t)(h + 1) == p0 || (uint32_t)(h + 1) == p1);
                        uint32_t rb = 0u, rc = 0u;
                        if (useB && !bw) rb = ld_relaxed(mvi_up + h);
                        if (useC && !cw) rc = ld_relaxed(mvi_up + h + 1);
                        const uint32_t eb = (uint32_t)h == p0 ? (hi & 0xFFFFu) : (hi >> 16);
                        const uint32_t ec = (uint32_t)(h + 1) == p0 ? (hi & 0xFFFFu) : (hi >> 16);
                        mB = !useB ? 0u : bw ? dec_full(eb) : (uint32_t)uni((int)rb);
                        mC = !useC ? 0u : cw ? dec_full(ec) : (uint32_t)uni((int)rc);
                    }
                }
                c.win = win;
                c.R = R;
                c.pitch = a.pitch;
                c.S = S;
                set_lane_base(c, (j + S + 1) * a.pitch + 4 * q + S + 1, S);
                c.x0 = x0;
                c.y0 = y0;
                c.W = W;
                c.H = H;
                set_box(c, kp, x0, y0, W, H);
                c.c4 = c.shape ? bin4(cur4) : cur4;
                if ((kp.t_texture || (MP && kp.masked_prs)) && c.shape && !kp.shape_only) {
                    c.ref_l = D.ptr<const uint8_t>(DW(ref));
                    c.st = st;
                    c.tl4 = ldg32((const uint32_t *)(D.ptr<const uint8_t>(DW(cur)) + (size_t)(y0 + j) * st + x0 + 4 * q));
                }
                const uint32_t mA = lasth == h - 1 ? lastv : 0u;
                const uint32_t mT = (uint32_t)uni((int)tv);
                int cx[4] = {mvx_full(mA), mvx_full(mB), mvx_full(mC), mvx_full(mT)};
                int cy[4] = {mvy_full(mA), mvy_full(mB), mvy_full(mC), mvy_full(mT)};
                // window writes visible to every lane: one wave, so completing
                // its LDS writes (and a compiler fence) suffices
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                const MbOut o = search_mb<MP>(seed, c, k, cx, cy, kp, !DB);
                const uint32_t ovi = (uint32_t)uni((int)o.mvi);
                if (l == 0) {
                    vvec[wv * 256 + h] = ovi;
                    vprog[wv] = h2;  // h done, and the transparent MBs up to h2
                    // the word carries h and the searched MB before it; every
                    // older result was stored before this MB's window arrived
                    if (pub_global)
                        __hip_atomic_store(gprog,
                                           row_word((uint32_t)h2, (uint32_t)h, enc_full(ovi),
                                                    lasth >= 0 ? (uint32_t)lasth : kNoPos, enc_full(lastv)),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                pend = true;
                pk = k;
                pmv = (uint32_t)uni((int)o.mv);
                pmvi = ovi;
                pcost = (uint32_t)uni((int)o.cost);
                piters = uni(o.iters);
                ppoints = uni(o.points);
                if constexpr (DB) {
                    phalf = kp.half_pel && !c.shape;
                    px0 = x0;
                    py0 = y0;
                    pdx = uni(o.dx);
                    pdy = uni(o.dy);
                    pc4 = c.c4;
                    cb ^= 1;
                }
                lastv = ovi;
                lasth = h;
                h = h2;
            }
            if constexpr (DB) {
                // the row's last MB: its half-sample step
                if (pend && phalf && !aborted) {
                    Ctx cp;
                    cp.win = win0 + (cb ^ 1) * wwords;
                    cp.pitch = a.pitch;
                    cp.S = S;
                    set_lane_base(cp, (j + S + 1) * a.pitch + 4 * q + S + 1, S);
                    cp.x0 = px0;
                    cp.y0 = py0;
                    cp.W = W;
                    cp.H = H;
                    cp.c4 = pc4;
                    cp.shape = false;
                    int hx = 2 * pdx, hy = 2 * pdy, hc = (int)pcost;
                    ppoints += half_refine(cp, kp, pdx, pdy, hx, hy, hc);
                    pmv = pack_mv(hx, hy);
                    pcost = (uint32_t)hc;
                }
            }
            // the row's last results, then (band-last row) a final word once
            // every store has completed
            if (pend && l == 0) store_result(D, pk, pmv, pmvi, pcost, piters, ppoints);
            if (!aborted && pub_global && l == 0)
                publish(gprog, row_word((uint32_t)wm, lasth >= 0 ? (uint32_t)lasth : kNoPos, enc_full(lastv), kNoPos,
                                        0u));
            if (aborted && l == 0) *vab = 1;
        }
        __syncthreads();
        if (uni(*vab)) break;  // the same decision in every wave
    }
}

}  // namespace

// elements per lane of the staging plan for range S (0: generic loop)
int plan_elems(int S) {
    const int rows = 2 * S + 18, dw = ((rows + 3) & ~3) >> 2;
    const int e = (rows * dw + 63) / 64;
    return e <= 4 ? 4 : e <= 12 ? 12 : e <= 28 ? 28 : 0;
}

int pa_worker_cap() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus * 16;
}

size_t pa_lds_bytes(int S, bool generic) {
    const int rows = 2 * S + 18, pitch = (rows + 3) & ~3;
    const size_t one = (size_t)rows * pitch + 16;
    (void)generic;
    return 1024 + one;
}

hipError_t launch_scan_counts(uint32_t *counts, int n, uint32_t *total, hipStream_t s) {
    hipLaunchKernelGGL(pa_scan_counts, dim3(1), dim3(1024), 0, s, counts, n, total);
    return hipGetLastError();
}

size_t pa_scratch_bytes(int nlines) {
    const size_t nb = ((size_t)nlines + 255) / 256;
    return 256 + nb * 4 * 8 + 256 + nb * 4 + 256 + (size_t)nlines * 4 + 256;
}

size_t pa2_lds_bytes(int S, int waves) {
    const int rows = 2 * S + 18, pitch = (rows + 3) & ~3;
    return 1024 + (size_t)waves * ((size_t)(((rows * pitch + 16) >> 2) + 4) * 4);
}

size_t pr_lds_bytes(int S, bool dbl) {
    const int rows = 2 * S + 18, pitch = (rows + 3) & ~3;
    return 1024 + (size_t)kRowWaves * (dbl ? 2 : 1) * ((size_t)(((rows * pitch + 16) >> 2) + 4) * 4);
}

// Two windows per wave (the half-sample step one MB late) when half-sample
// refinement is on and the workgroup's LDS still fits.
bool pr_double(int S, bool half_pel) {
    if (!half_pel) return false;
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
        lim = 64 * 1024;
    return pr_lds_bytes(S, true) + kRowWaves * 256 * 4 + 64 <= (size_t)lim;
}

int pa_rows_cap(int S, bool half_pel) {
    int dev = 0, cus = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds <= 0)
        lds = 160 * 1024;
    // dynamic + static LDS of one workgroup
    const size_t per = pr_lds_bytes(S, pr_double(S, half_pel)) + kRowWaves * 256 * 4 + 64;
    const int fit = (int)std::max<size_t>(1, (size_t)lds / per);
    return cus * std::min(fit, 8);
}

hipError_t launch_pa_rows(const JobDesc *jobs, const ChainDesc *chains, const uint32_t *bands, int nbands,
                          unsigned long long *progress, uint32_t *counter, uint32_t *status, const KParams &kp,
                          int workers, hipStream_t s, const KernelTimer *t, bool generic) {
    if (nbands <= 0) return hipSuccess;
    const int rows = 2 * kp.S + 18;
    PrArgs a{jobs, chains, bands, nbands, progress, counter, status, kp, (rows + 3) & ~3, rows};
    const bool dbl = pr_double(kp.S, kp.half_pel != 0);
    const size_t lds = pr_lds_bytes(kp.S, dbl);
    const dim3 blk(64 * kRowWaves);
    workers = std::max(1, std::min(workers, nbands));
    timer_mark(t, true, s);
#define ME_PR_LAUNCH(em)                                                                               \
    do {                                                                                               \
        if (dbl)                                                                                       \
            hipLaunchKernelGGL((pr_kernel<em, kRowWaves, true>), dim3(workers), blk, lds, s, a);      \
        else                                                                                           \
            hipLaunchKernelGGL((pr_kernel<em, kRowWaves, false>), dim3(workers), blk, lds, s, a);     \
    } while (0)
    if (kp.masked_prs) {  // the masked-luma recursion: generic staging only
        if (dbl)
            hipLaunchKernelGGL((pr_kernel<0, kRowWaves, true, true>), dim3(workers), blk, lds, s, a);
        else
            hipLaunchKernelGGL((pr_kernel<0, kRowWaves, false, true>), dim3(workers), blk, lds, s, a);
    } else {
        switch (generic ? 0 : row_elems(kp.S)) {
            case 4: ME_PR_LAUNCH(4); break;
            case 13: ME_PR_LAUNCH(13); break;
            case 28: ME_PR_LAUNCH(28); break;
            default: ME_PR_LAUNCH(0); break;
        }
    }
#undef ME_PR_LAUNCH
    hipError_t e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

namespace {
template <int NW>
void launch_lines(int em, int workers, size_t lds, hipStream_t s, const PaArgs &a) {
    const dim3 blk(64 * NW);
    switch (em) {
        case 4: hipLaunchKernelGGL((pa2_kernel<4, NW>), dim3(workers), blk, lds, s, a); break;
        case 12: hipLaunchKernelGGL((pa2_kernel<12, NW>), dim3(workers), blk, lds, s, a); break;
        case 28: hipLaunchKernelGGL((pa2_kernel<28, NW>), dim3(workers), blk, lds, s, a); break;
        default: hipLaunchKernelGGL((pa2_kernel<0, NW>), dim3(workers), blk, lds, s, a); break;
    }
}
}  // namespace

hipError_t launch_pa(const JobDesc *jobs, int njobs, int total_mbs, const ChainDesc *chains, const uint32_t *tickets,
                     int nlines, unsigned long long *progress, uint32_t *counter, uint32_t *masks, int mask_words,
                     uint8_t *scratch, uint32_t *status, const KParams &kp, int workers, hipStream_t s,
                     const KernelTimer *t, bool generic, int waves) {
    if (total_mbs <= 0 || nlines <= 0) return hipSuccess;
    uint32_t *tmask = masks, *bmask = masks + (size_t)nlines * mask_words;
    hipLaunchKernelGGL(pa_prepass, dim3((total_mbs + 255) / 256), dim3(256), 0, s, jobs, njobs, total_mbs, tmask,
                       bmask, mask_words, kp.shape_only, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // scratch: [nactive] [keep ballots, 4 per block] [block counts] [active tickets]
    const int nb = (nlines + 255) / 256;
    uint32_t *nactive = (uint32_t *)scratch;
    unsigned long long *keepw = (unsigned long long *)(scratch + 256);
    uint32_t *bcount = (uint32_t *)((uint8_t *)keepw + (((size_t)nb * 32 + 255) & ~(size_t)255));
    uint32_t *active = (uint32_t *)((uint8_t *)bcount + (((size_t)nb * 4 + 255) & ~(size_t)255));
    if (nlines <= kCompactOneBlock) {
        hipLaunchKernelGGL(pa_compact_lines, dim3(1), dim3(1024), 0, s, chains, tickets, nlines, tmask, mask_words,
                           progress, active, nactive);
    } else {
        hipLaunchKernelGGL(pa_line_flags, dim3(nb), dim3(256), 0, s, chains, tickets, nlines, tmask, mask_words,
                           progress, keepw, bcount);
        hipLaunchKernelGGL(pa_scan_counts, dim3(1), dim3(1024), 0, s, bcount, nb, nactive);
        hipLaunchKernelGGL(pa_scatter_tickets, dim3(nb), dim3(256), 0, s, tickets, nlines, keepw, bcount, active);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int rows = 2 * kp.S + 18;
    PaArgs a{jobs, chains, active, nactive, progress, counter, tmask, bmask, mask_words, status, kp,
             (rows + 3) & ~3, rows};
    // the several-wave worker reads no texture for boundary MBs
    if (waves >= 2 && (kp.t_texture || kp.masked_prs)) return hipErrorInvalidValue;
    timer_mark(t, true, s);
    if (waves >= 2) {
        const size_t lds2 = pa2_lds_bytes(kp.S, waves);
        const int em = generic ? 0 : plan_elems(kp.S);
        switch (waves) {
            case 2: launch_lines<2>(em, workers, lds2, s, a); break;
            case 3: launch_lines<3>(em, workers, lds2, s, a); break;
            case 4: launch_lines<4>(em, workers, lds2, s, a); break;
            case 6: launch_lines<6>(em, workers, lds2, s, a); break;
            case 8: launch_lines<8>(em, workers, lds2, s, a); break;
            default: return hipErrorInvalidValue;  // no worker of that width
        }
        e = hipGetLastError();
        timer_mark(t, false, s);
        return e;
    }
    // the masked-luma recursion: generic staging only
    const bool gen = generic || kp.masked_prs;
    const size_t lds = pa_lds_bytes(kp.S, gen);
    if (kp.masked_prs) {
        hipLaunchKernelGGL((pa_kernel<0, true>), dim3(workers), dim3(64), lds, s, a);
    } else {
        switch (gen ? 0 : plan_elems(kp.S)) {
            case 4: hipLaunchKernelGGL(pa_kernel<4>, dim3(workers), dim3(64), lds, s, a); break;
            case 12: hipLaunchKernelGGL(pa_kernel<12>, dim3(workers), dim3(64), lds, s, a); break;
            case 28: hipLaunchKernelGGL(pa_kernel<28>, dim3(workers), dim3(64), lds, s, a); break;
            default: hipLaunchKernelGGL(pa_kernel<0>, dim3(workers), dim3(64), lds, s, a); break;
        }
    }
    e = hipGetLastError();
    timer_mark(t, false, s);
    return e;
}

}  // namespace me

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
// cannot deadlock whatever the residency.  Per-line progress counters publish
// "pairs done".  Every wait is bounded; on timeout a status bit is raised and
// all workers leave.
//
// Coherence without cache maintenance.  The only data that crosses workers
// is the full-pel field mv_int (candidates A, B, C and cross-chain T) and the
// progress counters.  Both are written and read with device-scope atomic
// accesses (sc1: performed at the device coherence point, never served from
// a per-XCD L2 copy), and a producer waits for its mv_int store to complete
// (s_waitcnt vmcnt(0)) before it stores the counter.  A consumer issues its
// mv_int loads only after the counter load has returned the awaited value.
// No acquire/release fences are needed, so no L2 invalidate or write-back is
// ever issued and the frames stay L2-resident.  Frames, classes and external
// T fields are read-only during the launch and use ordinary cached loads.
#include "me_internal.h"

namespace me {

namespace {

struct PaArgs {
    const JobDesc *jobs;
    const ChainDesc *chains;
    const int32_t *chain_jobs;
    const uint32_t *tickets;
    int nlines;
    uint32_t *progress;
    uint32_t *counter;
    uint32_t *status;
    KParams kp;
};

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish `v` after every earlier store of this wave has completed.
__device__ __forceinline__ void publish(uint32_t *p, uint32_t v) {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    st_relaxed(p, v);
}

__device__ bool wait_ge(const uint32_t *p, uint32_t need, uint32_t *status, int spin_limit) {
    int spins = 0;
    for (;;) {
        uint32_t v = (uint32_t)uni((int)ld_relaxed(p));
        if (v >= need) {
            asm volatile("" ::: "memory");  // later loads stay after the counter load
            return true;
        }
        if ((spins & 31) == 31 && (uni((int)ld_relaxed(status)) & ST_ABORT)) return false;
        if (++spins > spin_limit) {
            if (lane() == 0) atomicOr(status, ST_SPIN_TIMEOUT | ST_ABORT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

struct Sweep {
    int sad, sx, sy, nxy;  // nxy = nx | ny << 16
};

// One fused pass at full-pel offset (dx, dy): SAD of the block and the
// gradient sums of Eqs. 3-5 (reference central differences at the displaced
// position, coordinates clamped to the frame).  Lane = (row j, quad q).
__device__ __forceinline__ Sweep sweep(const uint8_t *Pr, int st, int W, int H, int x, int y, int dx, int dy,
                                       uint32_t c4, bool shape, const int *R) {
    const int rx = x + dx, ry = y + dy;
    const uint8_t *row = Pr + (size_t)ry * st;
    uint32_t m = ld4(row + rx);
    int lf = row[rx > 0 ? rx - 1 : 0];
    int rt = row[rx + 4 < W ? rx + 4 : W - 1];
    uint32_t up = ld4(Pr + (size_t)(ry > 0 ? ry - 1 : 0) * st + rx);
    uint32_t dn = ld4(Pr + (size_t)(ry + 1 < H ? ry + 1 : H - 1) * st + rx);
    if (shape) {
        m = bin4(m);
        up = bin4(up);
        dn = bin4(dn);
        lf = lf ? 255 : 0;
        rt = rt ? 255 : 0;
    }
    int sad = (int)__builtin_amdgcn_sad_u8(c4, m, 0u);
    int sx = 0, sy = 0, nn = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int e = byte_of(c4, k) - byte_of(m, k);
        int left = k == 0 ? lf : byte_of(m, k - 1);
        int right = k == 3 ? rt : byte_of(m, k + 1);
        int rgx = R[right - left + 255];
        int rgy = R[byte_of(dn, k) - byte_of(up, k) + 255];
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

struct Ctx {
    const uint8_t *Pc, *Pr;
    int st, W, H, x, y;  // x, y: this lane's first pixel
    int x0, y0;
    uint32_t c4;
    bool shape;
    const int *R;
    int lox, hix, loy, hiy;
};

__device__ __forceinline__ int cost_of(const Ctx &c, int sad) { return c.shape ? sad / 255 : sad; }

// Section 3.2 recursion from (dx, dy) with distortion `cost` and pass `sw`
// at that point.  Returns the number of candidates evaluated.
__device__ int pel_recursion(const Ctx &c, const KParams &kp, int &dx, int &dy, int &cost, Sweep sw) {
    int it = 0;
    while (it < kp.k_max) {
        int nx = sw.nxy & 0xFFFF, ny = sw.nxy >> 16;
        int ux = nx ? sw.sx / nx : 0;
        int uy = ny ? sw.sy / ny : 0;
        int sx = prs_step(ux, kp.eps, kp.max_step);
        int sy = prs_step(uy, kp.eps, kp.max_step);
        if (sx == 0 && sy == 0) break;
        int tx = iclamp(dx + sx, c.lox, c.hix);
        int ty = iclamp(dy + sy, c.loy, c.hiy);
        if (tx == dx && ty == dy) break;
        ++it;
        Sweep s2 = sweep(c.Pr, c.st, c.W, c.H, c.x, c.y, tx, ty, c.c4, c.shape, c.R);
        int c2 = cost_of(c, s2.sad);
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

// Half-sample refinement around the full-pel vector d (MPEG-4 bilinear,
// rounding control 0).  Updates (hx, hy), cost; returns feasible count.
__device__ int half_refine(const Ctx &c, const KParams &kp, int dx, int dy, int &hx, int &hy, int &cost) {
    const int W = c.W, H = c.H, st = c.st;
    // 3 x 6 neighbourhood: rows ry-1..ry+1, columns rx-1..rx+4 (clamped)
    int nb[3][6];
    const int rx = c.x + dx, ry = c.y + dy;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        int yy = iclamp(ry - 1 + r, 0, H - 1);
        const uint8_t *row = c.Pr + (size_t)yy * st;
#pragma unroll
        for (int q = 0; q < 6; ++q) nb[r][q] = row[iclamp(rx - 1 + q, 0, W - 1)];
    }
    int part[8];
    bool feas[8];
    int nfeas = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int ox = kHalfX[o], oy = kHalfY[o];
        const int fx = ox & 1, fy = oy & 1;
        const int oxr = ox < 0 ? 0 : 1, oyr = oy < 0 ? 0 : 1;  // neighbourhood origin of A
        const int qx = 2 * dx + ox, qy = 2 * dy + oy;
        const int ix = dx + (ox < 0 ? -1 : 0), iy = dy + (oy < 0 ? -1 : 0);
        feas[o] = abs(qx) <= 2 * kp.S && abs(qy) <= 2 * kp.S && c.x0 + ix >= 0 && c.x0 + ix + 15 + fx <= W - 1 &&
                  c.y0 + iy >= 0 && c.y0 + iy + 15 + fy <= H - 1;
        nfeas += feas[o];
        int s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int A = nb[oyr][oxr + k], B = nb[oyr][oxr + k + 1];
            int Cc = nb[oyr + 1][oxr + k], D = nb[oyr + 1][oxr + k + 1];
            int p = (fx && fy) ? ((A + B + Cc + D + 2) >> 2) : fx ? ((A + B + 1) >> 1) : fy ? ((A + Cc + 1) >> 1) : A;
            s += abs(byte_of(c.c4, k) - p);
        }
        part[o] = s;
    }
    int tot[8];
#pragma unroll
    for (int o = 0; o < 8; o += 2) {
        int pk = wave_sum(part[o] | (part[o + 1] << 16));
        tot[o] = pk & 0xFFFF;
        tot[o + 1] = (int)((uint32_t)pk >> 16);
    }
    int bx = 2 * dx, by = 2 * dy, bc = cost;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        if (feas[o] && tot[o] < bc) {
            bc = tot[o];
            bx = 2 * dx + kHalfX[o];
            by = 2 * dy + kHalfY[o];
        }
    }
    hx = bx;
    hy = by;
    cost = bc;
    return nfeas;
}

__device__ __forceinline__ uint32_t pack_mv(int x, int y) { return (uint32_t)(uint16_t)x | ((uint32_t)(uint16_t)y << 16); }
__device__ __forceinline__ int mvx_full(uint32_t w) { return ((int)(int16_t)(w & 0xFFFF)) >> 1; }
__device__ __forceinline__ int mvy_full(uint32_t w) { return ((int)(int16_t)(w >> 16)) >> 1; }

// Fig. 1 for the non-transparent MB (h, v) of job J with class `cls`.
// (tx, ty): T candidate (full-pel) when `t_reg`; returns the MB's full-pel
// vector in (tx, ty).
__device__ void process_mb(const JobDesc &J, int h, int v, int cls, bool t_reg, int &tx, int &ty, const int *R,
                           const KParams &kp) {
    const int l = lane(), j = l >> 2, q = l & 3;
    const int wm = J.wm, k = v * wm + h;
    const int x0 = 16 * h, y0 = 16 * v;
    uint32_t *mv = (uint32_t *)J.mv;
    uint32_t *mvi = (uint32_t *)J.mv_int;
    Ctx c;
    c.shape = kp.shape_only || cls == ME_MB_BOUNDARY;
    c.Pc = c.shape ? J.cur_a : J.cur;
    c.Pr = c.shape ? J.ref_a : J.ref;
    c.st = J.stride;
    c.W = J.width;
    c.H = J.height;
    c.x0 = x0;
    c.y0 = y0;
    c.x = x0 + 4 * q;
    c.y = y0 + j;
    c.R = R;
    const int S = kp.S;
    c.lox = max(-S, -x0);
    c.hix = min(S, c.W - 16 - x0);
    c.loy = max(-S, -y0);
    c.hiy = min(S, c.H - 16 - y0);
    uint32_t c4 = *(const uint32_t *)(c.Pc + (size_t)c.y * c.st + c.x);
    c.c4 = c.shape ? bin4(c4) : c4;

    // candidates A, B, C, T (neighbours outside the grid: (0, 0))
    int cx[4] = {0, 0, 0, 0}, cy[4] = {0, 0, 0, 0};
    if (h > 0) {
        uint32_t w = (uint32_t)uni((int)ld_relaxed(mvi + k - 1));
        cx[0] = mvx_full(w);
        cy[0] = mvy_full(w);
    }
    if (v > 0) {
        uint32_t w = (uint32_t)uni((int)ld_relaxed(mvi + k - wm));
        cx[1] = mvx_full(w);
        cy[1] = mvy_full(w);
        if (h + 1 < wm) {
            uint32_t w2 = (uint32_t)uni((int)ld_relaxed(mvi + k - wm + 1));
            cx[2] = mvx_full(w2);
            cy[2] = mvy_full(w2);
        }
    }
    if (t_reg) {
        cx[3] = tx;
        cy[3] = ty;
    } else if (J.tf) {
        uint32_t w = (uint32_t)uni((int)ld_relaxed((const uint32_t *)J.tf + k));
        cx[3] = mvx_full(w);
        cy[3] = mvy_full(w);
    }
    // admissible and distinct, in the order A, B, C, T (compile-time indices
    // only, so the list lives in registers)
    bool keep[4];
    int n = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        bool ok = cx[i] >= c.lox && cx[i] <= c.hix && cy[i] >= c.loy && cy[i] <= c.hiy;
#pragma unroll
        for (int p = 0; p < i; ++p) ok = ok && !(keep[p] && cx[p] == cx[i] && cy[p] == cy[i]);
        keep[i] = ok;
        n += ok;
    }
    if (n == 0) {
        cx[0] = cy[0] = 0;
        keep[0] = true;
        n = 1;
    }
    // block costs of the list, two 16-bit partial SADs per reduction
    int part[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (keep[i]) {
            uint32_t r4 = ld4(c.Pr + (size_t)(c.y + cy[i]) * c.st + c.x + cx[i]);
            if (c.shape) r4 = bin4(r4);
            part[i] = (int)__builtin_amdgcn_sad_u8(c.c4, r4, 0u);
        }
    }
    int p01 = wave_sum(part[0] | (part[1] << 16));
    int p23 = (keep[2] || keep[3]) ? wave_sum(part[2] | (part[3] << 16)) : 0;
    int costs[4] = {p01 & 0xFFFF, (int)((uint32_t)p01 >> 16), p23 & 0xFFFF, (int)((uint32_t)p23 >> 16)};
    // Min[...]: the first minimum in list order
    int dx = 0, dy = 0, bc = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int ci = cost_of(c, costs[i]);
        if (keep[i] && ci < bc) {
            bc = ci;
            dx = cx[i];
            dy = cy[i];
        }
    }
    int dc = bc;
    int pts = n, its = 0;
    if (J.seed && !c.shape) {
        uint32_t w = (uint32_t)uni((int)ld_relaxed((const uint32_t *)J.seed + k));
        int sx = iclamp(mvx_full(w), c.lox, c.hix), sy = iclamp(mvy_full(w), c.loy, c.hiy);
        Sweep sw = sweep(c.Pr, c.st, c.W, c.H, c.x, c.y, sx, sy, c.c4, c.shape, c.R);
        int sc = cost_of(c, sw.sad);
        pts += 1;
        int it1 = pel_recursion(c, kp, sx, sy, sc, sw);
        its += it1;
        pts += it1;
        if (20ll * sc > 21ll * bc) {
            if (kp.k_max > 0) {
                Sweep s0 = sweep(c.Pr, c.st, c.W, c.H, c.x, c.y, dx, dy, c.c4, c.shape, c.R);
                int it2 = pel_recursion(c, kp, dx, dy, dc, s0);
                its += it2;
                pts += it2;
            }
        } else {
            dx = sx;
            dy = sy;
            dc = sc;
        }
    } else if (kp.k_max > 0) {
        Sweep s0 = sweep(c.Pr, c.st, c.W, c.H, c.x, c.y, dx, dy, c.c4, c.shape, c.R);
        int it1 = pel_recursion(c, kp, dx, dy, dc, s0);
        its += it1;
        pts += it1;
    }
    int hx = 2 * dx, hy = 2 * dy;
    if (kp.half_pel && !c.shape) pts += half_refine(c, kp, dx, dy, hx, hy, dc);
    if (l == 0) {
        mv[k] = pack_mv(hx, hy);
        st_relaxed(mvi + k, pack_mv(2 * dx, 2 * dy));
        if (J.cost) J.cost[k] = (uint32_t)dc;
        if (J.iters) J.iters[k] = (uint8_t)its;
        if (J.points) J.points[k] = (uint16_t)pts;
    }
    tx = dx;
    ty = dy;
}

__global__ __launch_bounds__(64) void pa_kernel(PaArgs a) {
    __shared__ int R[512];
    const KParams kp = a.kp;
    for (int g = lane(); g < 511; g += 64) {
        int m = abs(g - 255);
        int r = (m == 0 || m < 2 * kp.theta) ? 0 : (16384 + m) / (2 * m);
        R[g] = g < 255 ? -r : r;
    }
    __syncthreads();
    const int l = lane();
    for (;;) {
        int t = 0;
        if (l == 0) t = (int)atomicAdd(a.counter, 1u);
        t = __shfl(t, 0, 64);
        t = uni(t);
        if (t >= a.nlines) break;
        if (uni((int)ld_relaxed(a.status)) & ST_ABORT) break;
        const uint32_t tk = a.tickets[t];
        const int ci = (int)(tk >> 16), v = (int)((tk >> 8) & 0xFF), h = (int)(tk & 0xFF);
        const ChainDesc ch = a.chains[ci];
        const int wm = ch.wm;
        const int line = ch.line_base + v * wm + h;
        int tx = 0, ty = 0;
        for (int p = 0; p < ch.len; ++p) {
            const JobDesc &J = a.jobs[a.chain_jobs[ch.first + p]];
            const uint32_t need = (uint32_t)(p + 1);
            const int k = v * wm + h;
            int cls = J.cls ? (int)J.cls[k] : ME_MB_OPAQUE;
            if (cls > 2) {
                if (l == 0) atomicOr(a.status, ST_BAD_CLASS);
                cls = ME_MB_TRANSPARENT;
            }
            if (cls == ME_MB_TRANSPARENT) {
                // no vector is computed: the result depends on nothing, so
                // it is published without waiting for the neighbours
                if (l == 0) {
                    ((uint32_t *)J.mv)[k] = 0u;
                    st_relaxed((uint32_t *)J.mv_int + k, 0u);
                    if (J.cost) J.cost[k] = 0u;
                    if (J.iters) J.iters[k] = 0;
                    if (J.points) J.points[k] = 0;
                    publish(a.progress + line, need);
                }
                tx = ty = 0;
                continue;
            }
            // A, B and C each waited for directly: a transparent MB publishes
            // without waiting, so no neighbour's progress implies another's
            bool ok = true;
            if (h > 0) ok = wait_ge(a.progress + line - 1, need, a.status, kp.spin_limit);
            if (ok && v > 0) ok = wait_ge(a.progress + line - wm, need, a.status, kp.spin_limit);
            if (ok && v > 0 && h + 1 < wm) ok = wait_ge(a.progress + line - wm + 1, need, a.status, kp.spin_limit);
            if (ok && J.dep_line_base >= 0 && !J.t_local)
                ok = wait_ge(a.progress + J.dep_line_base + v * wm + h, (uint32_t)(J.dep_pos + 1), a.status,
                             kp.spin_limit);
            if (!ok) return;
            process_mb(J, h, v, cls, J.t_local != 0 && p > 0, tx, ty, R, kp);
            if (l == 0) publish(a.progress + line, need);
        }
    }
}

}  // namespace

int pa_worker_cap() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus * 16;
}

hipError_t launch_pa(const JobDesc *jobs, const ChainDesc *chains, const int32_t *chain_jobs,
                     const uint32_t *tickets, int nlines, uint32_t *progress, uint32_t *counter,
                     uint32_t *status, const KParams &kp, int workers, hipStream_t s) {
    PaArgs a{jobs, chains, chain_jobs, tickets, nlines, progress, counter, status, kp};
    hipLaunchKernelGGL(pa_kernel, dim3(workers), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace me

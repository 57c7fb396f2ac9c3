/*
 * CPU oracle for the shape-adaptive motion estimator of Benboubker, Abdi and
 * Ahaitouf, "Shape-Adaptive Motion Estimation Algorithm for MPEG-4 Video
 * Coding".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product never does.  It
 * shares no source with the GPU library: every routine is written out here
 * from the paper, in scalar loops, with no blocking, fusion or reordering.
 *
 * Conventions (the paper leaves them open; each reading is listed in the
 * design notes):
 *   - frame W x H (multiples of 16), macroblock (MB) (h, v) has its top-left
 *     pixel at (16h, 16v); MBs are visited in raster order, rows v outer,
 *     columns h inner (Fig. 1 loops);
 *   - a full-pel motion vector d = (dx, dy) predicts cur(x, y) by
 *     ref(x + dx, y + dy);
 *   - every motion vector at the interface is int16 (x, y) in half-pel units;
 *     integer results are even;
 *   - MB classes: 0 transparent, 1 opaque, 2 boundary (Section 1).
 *
 * Parity pins live in the tests (closed forms, brute force, invariants).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TRANSPARENT 0
#define OR_OPAQUE 1
#define OR_BOUNDARY 2

typedef struct {
    const uint8_t *cur_luma, *ref_luma;   /* row stride `stride` bytes */
    const uint8_t *cur_alpha, *ref_alpha; /* both NULL: rectangular frames */
    int width, height, stride;
} or_pair;

typedef struct {
    int search_range; /* S: |dx|, |dy| <= S (full-pel) */
    int theta;        /* gradient dead zone of Eq. 4 */
    int eps_q12;      /* convergence factor of Eq. 3 in Q.12 */
    int max_step;     /* largest per-axis step of one recursion */
    int k_max;        /* cap on the recursion count */
    int half_pel;     /* 1: half-sample refinement of texture MBs */
    int unrestricted; /* 1: vectors limited by S only, the reference extended by its edge pixels */
    int t_texture;    /* 1: Section 3.1 text - a boundary MB's T is scored on texture */
    int masked_prs;   /* 1: a boundary MB's recursion refines on luma over the current VOP's pixels */
} or_params;

/* ------------------------------------------------------------ helpers */
static int iabs(int a) { return a < 0 ? -a : a; }
static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static int iclamp(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* half-pel component -> full-pel, rounding toward minus infinity */
static int half_to_full(int v) { return (v >= 0) ? v / 2 : -((-v + 1) / 2); }

static int luma_at(const uint8_t *p, int stride, int x, int y) { return p[(size_t)y * stride + x]; }

/* the binary shape plane of a VOP as gray levels: 255 inside, 0 outside */
static int shape_at(const uint8_t *a, int stride, int x, int y) {
    return a[(size_t)y * stride + x] != 0 ? 255 : 0;
}

static int plane_cur(const or_pair *fp, int shape, int x, int y) {
    return shape ? shape_at(fp->cur_alpha, fp->stride, x, y) : luma_at(fp->cur_luma, fp->stride, x, y);
}

/* Reference reads clamp both coordinates to the frame: the reference plane
 * extended by repeating its edge pixels (MPEG-4's padding for unrestricted
 * vectors).  With the restricted admissibility every read is in the frame
 * anyway. */
static int ref_luma_at(const or_pair *fp, int x, int y) {
    return luma_at(fp->ref_luma, fp->stride, iclamp(x, 0, fp->width - 1), iclamp(y, 0, fp->height - 1));
}

static int plane_ref(const or_pair *fp, int shape, int x, int y) {
    x = iclamp(x, 0, fp->width - 1);
    y = iclamp(y, 0, fp->height - 1);
    return shape ? shape_at(fp->ref_alpha, fp->stride, x, y) : luma_at(fp->ref_luma, fp->stride, x, y);
}

/* ------------------------------------------------- MB classification */
/*
 * Section 1: an MB is transparent (no pixel of the VOP), opaque (every pixel
 * inside) or boundary.  Inside means alpha != 0.  `bab` (optional) receives
 * the 16x16 binary alpha block of each MB as 8 words: word w holds rows 2w
 * (bits 0..15) and 2w+1 (bits 16..31), column i at bit i of its half.
 */
int or_classify(const uint8_t *alpha, int width, int height, int stride, uint8_t *cls, uint32_t *bab) {
    if (!alpha || !cls || width <= 0 || height <= 0 || width % 16 || height % 16 || stride < width) return -1;
    int wm = width / 16, hm = height / 16;
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int n = 0;
            uint32_t words[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int j = 0; j < 16; ++j) {
                for (int i = 0; i < 16; ++i) {
                    int in = alpha[(size_t)(16 * v + j) * stride + 16 * h + i] != 0;
                    n += in;
                    if (in) words[j / 2] |= 1u << ((j % 2) * 16 + i);
                }
            }
            int k = v * wm + h;
            cls[k] = (uint8_t)(n == 0 ? OR_TRANSPARENT : (n == 256 ? OR_OPAQUE : OR_BOUNDARY));
            if (bab) memcpy(bab + 8 * (size_t)k, words, sizeof(words));
        }
    }
    return 0;
}

/* ------------------------------------------------------ block costs */
/* Section 2 / 3.1: sum of absolute luma differences of the n x n block at
 * (x0, y0) against the reference block displaced by (dx, dy). */
static uint32_t sad_n(const or_pair *fp, int x0, int y0, int n, int dx, int dy) {
    uint32_t s = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            s += (uint32_t)iabs(luma_at(fp->cur_luma, fp->stride, x0 + i, y0 + j) -
                                ref_luma_at(fp, x0 + i + dx, y0 + j + dy));
    return s;
}

uint32_t or_sad(const or_pair *fp, int x0, int y0, int dx, int dy) { return sad_n(fp, x0, y0, 16, dx, dy); }

/* Fig. 1, boundary branch: the distortion of two binary alpha blocks is the
 * number of pixels whose inside/outside state differs. */
uint32_t or_mismatch(const or_pair *fp, int x0, int y0, int dx, int dy) {
    uint32_t s = 0;
    for (int j = 0; j < 16; ++j)
        for (int i = 0; i < 16; ++i) {
            int a = fp->cur_alpha[(size_t)(y0 + j) * fp->stride + x0 + i] != 0;
            int b = plane_ref(fp, 1, x0 + i + dx, y0 + j + dy) != 0;
            s += (uint32_t)(a != b);
        }
    return s;
}

static uint32_t block_cost(const or_pair *fp, int shape, int x0, int y0, int dx, int dy) {
    return shape ? or_mismatch(fp, x0, y0, dx, dy) : or_sad(fp, x0, y0, dx, dy);
}

/* Luma SAD of the 16 x 16 block at (x0, y0) over the pixels of the current
 * VOP only (alpha != 0): the texture distortion of a boundary MB. */
static uint32_t masked_sad(const or_pair *fp, int x0, int y0, int dx, int dy) {
    uint32_t s = 0;
    for (int j = 0; j < 16; ++j)
        for (int i = 0; i < 16; ++i)
            if (fp->cur_alpha[(size_t)(y0 + j) * fp->stride + x0 + i] != 0)
                s += (uint32_t)iabs(luma_at(fp->cur_luma, fp->stride, x0 + i, y0 + j) -
                                    ref_luma_at(fp, x0 + i + dx, y0 + j + dy));
    return s;
}

/* A full-pel vector is admissible when |dx|, |dy| <= S and (unless the
 * reference is extended for unrestricted vectors) the whole displaced n x n
 * block lies inside the reference frame. */
static int feasible_n(const or_pair *fp, const or_params *p, int x0, int y0, int n, int dx, int dy) {
    int S = p->search_range;
    if (iabs(dx) > S || iabs(dy) > S) return 0;
    return p->unrestricted ||
           (x0 + dx >= 0 && x0 + dx <= fp->width - n && y0 + dy >= 0 && y0 + dy <= fp->height - n);
}

static int feasible(const or_pair *fp, const or_params *p, int x0, int y0, int dx, int dy) {
    return feasible_n(fp, p, x0, y0, 16, dx, dy);
}

/* The admissible box of the n x n block at (x0, y0), per axis. */
static void box_n(const or_pair *fp, const or_params *p, int x0, int y0, int n, int *lox, int *hix, int *loy,
                  int *hiy) {
    int S = p->search_range;
    *lox = p->unrestricted ? -S : imax(-S, -x0);
    *hix = p->unrestricted ? S : imin(S, fp->width - n - x0);
    *loy = p->unrestricted ? -S : imax(-S, -y0);
    *hiy = p->unrestricted ? S : imin(S, fp->height - n - y0);
}

/* ------------------------------------ pel-recursive search (Section 3.2) */
/*
 * Eq. 4 with Eq. 5: u = 0 where |df/dx| < Theta, else 1/(df/dx), with
 * df/dx = g / 2 for the central difference g = f(x+1) - f(x-1).  Hence
 * u = 2/g for |g| >= 2 Theta.  Returned in Q.12, rounded half up on the
 * magnitude: sgn(g) * floor((2^14 + |g|) / (2|g|)).
 */
int32_t or_recip(int g, int theta) {
    int a = iabs(g);
    if (a < 2 * theta || a == 0) return 0;
    int32_t r = (int32_t)((16384 + a) / (2 * a));
    return g < 0 ? -r : r;
}

/*
 * One gradient pass at displacement d (Eqs. 3-5).  For every pixel p of the
 * block: the displaced pixel difference e = cur(p) - ref(p + d) and the
 * central differences of the reference at p + d (coordinates clamped to the
 * frame).  The per-pixel updates e * u are averaged over the pixels whose
 * gradient passes the threshold, per component, in Q.12 (C division).
 * `mask` (NULL: every pixel) restricts the pass to the pixels where it is
 * non-zero: the current VOP's pixels when a boundary MB refines on texture.
 */
static void prs_pass_n(const or_pair *fp, int shape, const uint8_t *mask, int theta, int x0, int y0, int n, int dx,
                       int dy, int32_t *ux, int32_t *uy) {
    int32_t sx = 0, sy = 0;
    int nx = 0, ny = 0;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            int px = x0 + i, py = y0 + j;
            if (mask && mask[(size_t)py * fp->stride + px] == 0) continue;
            int rx = px + dx, ry = py + dy;
            int e = plane_cur(fp, shape, px, py) - plane_ref(fp, shape, rx, ry);
            int gx = plane_ref(fp, shape, imin(rx + 1, fp->width - 1), ry) - plane_ref(fp, shape, imax(rx - 1, 0), ry);
            int gy = plane_ref(fp, shape, rx, imin(ry + 1, fp->height - 1)) - plane_ref(fp, shape, rx, imax(ry - 1, 0));
            int32_t rgx = or_recip(gx, theta);
            int32_t rgy = or_recip(gy, theta);
            sx += e * rgx;
            sy += e * rgy;
            nx += rgx != 0;
            ny += rgy != 0;
        }
    }
    *ux = nx ? sx / nx : 0;
    *uy = ny ? sy / ny : 0;
}

void or_prs_pass(const or_pair *fp, int shape, int theta, int x0, int y0, int dx, int dy, int32_t *ux, int32_t *uy) {
    prs_pass_n(fp, shape, NULL, theta, x0, y0, 16, dx, dy, ux, uy);
}

/* Eq. 3 step in one axis: eps * U in Q.24, rounded half away from zero to
 * whole pixels, limited to +-max_step. */
int or_step(int32_t u, int eps_q12, int max_step) {
    int64_t vq = (int64_t)eps_q12 * (int64_t)u;
    int64_t a = vq < 0 ? -vq : vq;
    int64_t s = (a + ((int64_t)1 << 23)) >> 24;
    if (vq < 0) s = -s;
    if (s > max_step) s = max_step;
    if (s < -max_step) s = -max_step;
    return (int)s;
}

/*
 * Section 3.2: starting at the BRS winner, repeatedly take the Eq. 3 update
 * as the next candidate (one of the eight neighbours for max_step 1), keep it
 * when its distortion is strictly smaller, and stop at the first candidate
 * that does not improve, at a zero update, at the search-window border, or
 * after k_max candidates.  Returns the number of candidates evaluated.
 * With `mask` (16 x 16 luma only) the passes and the distortions cover the
 * pixels where it is non-zero.
 */
static int pel_recursion_n(const or_pair *fp, const or_params *p, int shape, const uint8_t *mask, int x0, int y0,
                           int n, int *dx, int *dy, uint32_t *cost) {
    int lox, hix, loy, hiy;
    box_n(fp, p, x0, y0, n, &lox, &hix, &loy, &hiy);
    int it = 0;
    while (it < p->k_max) {
        int32_t ux, uy;
        prs_pass_n(fp, shape, mask, p->theta, x0, y0, n, *dx, *dy, &ux, &uy);
        int sx = or_step(ux, p->eps_q12, p->max_step);
        int sy = or_step(uy, p->eps_q12, p->max_step);
        if (sx == 0 && sy == 0) break;
        int nx = iclamp(*dx + sx, lox, hix);
        int ny = iclamp(*dy + sy, loy, hiy);
        if (nx == *dx && ny == *dy) break;
        ++it;
        uint32_t c = n != 16 ? sad_n(fp, x0, y0, n, nx, ny)
                              : (mask ? masked_sad(fp, x0, y0, nx, ny) : block_cost(fp, shape, x0, y0, nx, ny));
        if (c < *cost) {
            *dx = nx;
            *dy = ny;
            *cost = c;
        } else {
            break;
        }
    }
    return it;
}

static int pel_recursion(const or_pair *fp, const or_params *p, int shape, int x0, int y0, int *dx, int *dy,
                         uint32_t *cost) {
    return pel_recursion_n(fp, p, shape, NULL, x0, y0, 16, dx, dy, cost);
}

/* ------------------------------------------- half-sample refinement */
/* MPEG-4 bilinear half-sample prediction, rounding control 0.  (hx, hy) is
 * a half-pel vector; reference coordinates are clamped to the frame. */
static int pred_half(const or_pair *fp, int x, int y, int hx, int hy) {
    int ix = half_to_full(hx), iy = half_to_full(hy);
    int fx = hx - 2 * ix, fy = hy - 2 * iy;
    int W = fp->width, H = fp->height;
    int xa = iclamp(x + ix, 0, W - 1), xb = iclamp(x + ix + 1, 0, W - 1);
    int ya = iclamp(y + iy, 0, H - 1), yb = iclamp(y + iy + 1, 0, H - 1);
    int A = luma_at(fp->ref_luma, fp->stride, xa, ya);
    if (!fx && !fy) return A;
    int B = luma_at(fp->ref_luma, fp->stride, xb, ya);
    int C = luma_at(fp->ref_luma, fp->stride, xa, yb);
    if (fx && !fy) return (A + B + 1) >> 1;
    if (!fx && fy) return (A + C + 1) >> 1;
    int D = luma_at(fp->ref_luma, fp->stride, xb, yb);
    return (A + B + C + D + 2) >> 2;
}

static uint32_t sad_half_n(const or_pair *fp, int x0, int y0, int n, int hx, int hy) {
    uint32_t s = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            s += (uint32_t)iabs(luma_at(fp->cur_luma, fp->stride, x0 + i, y0 + j) - pred_half(fp, x0 + i, y0 + j, hx, hy));
    return s;
}

uint32_t or_sad_half(const or_pair *fp, int x0, int y0, int hx, int hy) { return sad_half_n(fp, x0, y0, 16, hx, hy); }

/* The whole integer footprint of the half-sample prediction of the n x n
 * block (n + fx columns, n + fy rows) lies in the reference frame. */
static int half_feasible_n(const or_pair *fp, const or_params *p, int x0, int y0, int n, int hx, int hy) {
    int S = p->search_range;
    if (iabs(hx) > 2 * S || iabs(hy) > 2 * S) return 0;
    if (p->unrestricted) return 1;
    int ix = half_to_full(hx), iy = half_to_full(hy);
    int fx = hx - 2 * ix, fy = hy - 2 * iy;
    return x0 + ix >= 0 && x0 + ix + n - 1 + fx <= fp->width - 1 && y0 + iy >= 0 &&
           y0 + iy + n - 1 + fy <= fp->height - 1;
}

static int half_feasible(const or_pair *fp, const or_params *p, int x0, int y0, int hx, int hy) {
    return half_feasible_n(fp, p, x0, y0, 16, hx, hy);
}

static const int HALF_OFFS[8][2] = {{-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1}};

/* ----------------------------------------------- the proposed algorithm */
/*
 * Fig. 1 for one MB (h, v) of one frame pair of one VOP: the candidates come
 * from the vectors already in `mv_int` (left, upper, upper-right neighbours)
 * and from `t_field`.
 */
static int pa_mb(const or_pair *fp, const uint8_t *cls, const int16_t *t_field, const int16_t *seed,
                 const or_params *p, int shape_only, int h, int v, int16_t *mv, int16_t *mv_int, uint32_t *cost,
                 uint8_t *iters, uint16_t *points) {
    int has_alpha = fp->cur_alpha != NULL && fp->ref_alpha != NULL;
    int wm = fp->width / 16;
    int k = v * wm + h;
    int c = cls ? cls[k] : OR_OPAQUE;
    int x0 = 16 * h, y0 = 16 * v;
    if (c == OR_TRANSPARENT) { /* no vector is computed */
        mv[2 * k] = mv[2 * k + 1] = 0;
        mv_int[2 * k] = mv_int[2 * k + 1] = 0;
        if (cost) cost[k] = 0;
        if (iters) iters[k] = 0;
        if (points) points[k] = 0;
        return 0;
    }
    int shape = shape_only || c == OR_BOUNDARY;
    if (shape && !has_alpha) return -1;
    /* a reading of Section 3.1 (the temporal candidate of a boundary MB is
     * evaluated on texture): its recursion refines on texture too, over the
     * current VOP's pixels */
    int mprs = p->masked_prs && !shape_only && c == OR_BOUNDARY;
    /* candidates A (left), B (up), C (up-right), T (same MB, previous
     * pair); neighbours outside the MB grid contribute (0, 0) */
    int cand[4][2];
    cand[0][0] = h > 0 ? half_to_full(mv_int[2 * (k - 1)]) : 0;
    cand[0][1] = h > 0 ? half_to_full(mv_int[2 * (k - 1) + 1]) : 0;
    cand[1][0] = v > 0 ? half_to_full(mv_int[2 * (k - wm)]) : 0;
    cand[1][1] = v > 0 ? half_to_full(mv_int[2 * (k - wm) + 1]) : 0;
    cand[2][0] = (v > 0 && h + 1 < wm) ? half_to_full(mv_int[2 * (k - wm + 1)]) : 0;
    cand[2][1] = (v > 0 && h + 1 < wm) ? half_to_full(mv_int[2 * (k - wm + 1) + 1]) : 0;
    cand[3][0] = t_field ? half_to_full(t_field[2 * k]) : 0;
    cand[3][1] = t_field ? half_to_full(t_field[2 * k + 1]) : 0;
    /* admissible, distinct, in order A, B, C, T */
    int list[4][2], n = 0, has_t = 0;
    for (int i = 0; i < 4; ++i) {
        if (!feasible(fp, p, x0, y0, cand[i][0], cand[i][1])) continue;
        int dup = 0;
        for (int q = 0; q < n; ++q)
            if (list[q][0] == cand[i][0] && list[q][1] == cand[i][1]) dup = 1;
        if (!dup) {
            list[n][0] = cand[i][0];
            list[n][1] = cand[i][1];
            ++n;
            has_t = i == 3;
        }
    }
    if (n == 0) {
        list[0][0] = list[0][1] = 0;
        n = 1;
    }
    int bx, by, pts = n;
    uint32_t bc;
    if (p->t_texture && !shape_only && c == OR_BOUNDARY && has_t && n > 1) {
        /* Section 3.1, text: the spatial candidates are scored on the
         * BABs (first minimum), T on texture - T replaces the spatial
         * winner when its luma SAD over the VOP pixels is strictly lower;
         * the spatial winner's texture comparison is one more block */
        bx = list[0][0];
        by = list[0][1];
        bc = block_cost(fp, shape, x0, y0, bx, by);
        for (int i = 1; i < n - 1; ++i) {
            uint32_t ci = block_cost(fp, shape, x0, y0, list[i][0], list[i][1]);
            if (ci < bc) {
                bc = ci;
                bx = list[i][0];
                by = list[i][1];
            }
        }
        int tx = list[n - 1][0], ty = list[n - 1][1];
        if (masked_sad(fp, x0, y0, tx, ty) < masked_sad(fp, x0, y0, bx, by)) {
            bx = tx;
            by = ty;
            bc = block_cost(fp, shape, x0, y0, bx, by);
        }
        pts = n + 1;
    } else {
        /* Min[...] keeps the first minimum (MATLAB min semantics) */
        bx = list[0][0];
        by = list[0][1];
        bc = block_cost(fp, shape, x0, y0, bx, by);
        for (int i = 1; i < n; ++i) {
            uint32_t ci = block_cost(fp, shape, x0, y0, list[i][0], list[i][1]);
            if (ci < bc) {
                bc = ci;
                bx = list[i][0];
                by = list[i][1];
            }
        }
    }
    int its = 0;
    int dx = bx, dy = by;
    uint32_t dc = bc;
    if (mprs) {
        /* the candidate winner's luma SAD over the VOP pixels starts the
         * recursion: one more compared block */
        dc = masked_sad(fp, x0, y0, dx, dy);
        pts += 1;
        int it1 = pel_recursion_n(fp, p, 0, fp->cur_alpha, x0, y0, 16, &dx, &dy, &dc);
        its += it1;
        pts += it1;
    } else if (seed && !shape) {
        /* learned start: clamp into the admissible window, refine,
         * and fall back to the plain recursion when the refined
         * distortion exceeds the BRS minimum by more than 5 % */
        int lox, hix, loy, hiy;
        box_n(fp, p, x0, y0, 16, &lox, &hix, &loy, &hiy);
        int sx = iclamp(half_to_full(seed[2 * k]), lox, hix);
        int sy = iclamp(half_to_full(seed[2 * k + 1]), loy, hiy);
        uint32_t sc = block_cost(fp, shape, x0, y0, sx, sy);
        pts += 1;
        int it1 = pel_recursion(fp, p, shape, x0, y0, &sx, &sy, &sc);
        its += it1;
        pts += it1;
        if ((uint64_t)20 * sc > (uint64_t)21 * bc) {
            int it2 = pel_recursion(fp, p, shape, x0, y0, &dx, &dy, &dc);
            its += it2;
            pts += it2;
        } else {
            dx = sx;
            dy = sy;
            dc = sc;
        }
    } else {
        int it1 = pel_recursion(fp, p, shape, x0, y0, &dx, &dy, &dc);
        its += it1;
        pts += it1;
    }
    int hx = 2 * dx, hy = 2 * dy;
    if (p->half_pel && !shape) {
        int bhx = hx, bhy = hy;
        uint32_t hc = dc;
        for (int o = 0; o < 8; ++o) {
            int qx = hx + HALF_OFFS[o][0], qy = hy + HALF_OFFS[o][1];
            if (!half_feasible(fp, p, x0, y0, qx, qy)) continue;
            ++pts;
            uint32_t c2 = or_sad_half(fp, x0, y0, qx, qy);
            if (c2 < hc) {
                hc = c2;
                bhx = qx;
                bhy = qy;
            }
        }
        hx = bhx;
        hy = bhy;
        dc = hc;
    }
    mv[2 * k] = (int16_t)hx;
    mv[2 * k + 1] = (int16_t)hy;
    mv_int[2 * k] = (int16_t)(2 * dx);
    mv_int[2 * k + 1] = (int16_t)(2 * dy);
    if (cost) cost[k] = dc;
    if (iters) iters[k] = (uint8_t)its;
    if (points) points[k] = (uint16_t)pts;
    return 0;
}

static int pa_args_ok(const or_pair *fp, const int16_t *seed, const or_params *p, int shape_only, const int16_t *mv,
                      const int16_t *mv_int) {
    if (!fp || !p || !mv || !mv_int) return 0;
    if (fp->width % 16 || fp->height % 16 || fp->width <= 0 || fp->height <= 0) return 0;
    if (shape_only && !(fp->cur_alpha != NULL && fp->ref_alpha != NULL)) return 0;
    /* a dropped seed counts both recursions (up to 2 k_max) in a byte */
    if (seed && p->k_max > 127) return 0;
    return 1;
}

/*
 * Fig. 1 for one frame pair of one VOP, MBs in raster order.  `cls` from
 * or_classify on the current alpha (NULL: every MB opaque).  `t_field` is the
 * previous pair's full-pel field (half-pel units; NULL: zeros).  `seed` (NULL:
 * plain method) is a learned per-MB starting vector for texture MBs.
 * `shape_only` scores every non-transparent MB on its alpha block.
 */
int or_pa(const or_pair *fp, const uint8_t *cls, const int16_t *t_field, const int16_t *seed, const or_params *p,
          int shape_only, int16_t *mv, int16_t *mv_int, uint32_t *cost, uint8_t *iters, uint16_t *points) {
    if (!pa_args_ok(fp, seed, p, shape_only, mv, mv_int)) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    for (int v = 0; v < hm; ++v)
        for (int h = 0; h < wm; ++h)
            if (pa_mb(fp, cls, t_field, seed, p, shape_only, h, v, mv, mv_int, cost, iters, points)) return -1;
    return 0;
}

/*
 * The same pair with the MBs visited in the order `order` (MB indices v*W_mb+h,
 * each exactly once).  Any order in which every MB comes after its left,
 * upper and upper-right neighbours reads the same candidates as the raster
 * scan and so gives the same result; a test uses this to show that the
 * wavefront order of a parallel schedule is legal.
 */
int or_pa_order(const or_pair *fp, const uint8_t *cls, const int16_t *t_field, const int16_t *seed,
                const or_params *p, int shape_only, const int32_t *order, int16_t *mv, int16_t *mv_int,
                uint32_t *cost, uint8_t *iters, uint16_t *points) {
    if (!pa_args_ok(fp, seed, p, shape_only, mv, mv_int) || !order) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    for (int i = 0; i < wm * hm; ++i) {
        int k = order[i];
        if (k < 0 || k >= wm * hm) return -1;
        if (pa_mb(fp, cls, t_field, seed, p, shape_only, k % wm, k / wm, mv, mv_int, cost, iters, points)) return -1;
    }
    return 0;
}

/* --------------------------------------------------- baseline searches */
/* Exhaustive search: every admissible vector; ties broken by the smaller
 * |dx| + |dy|, then the smaller dy, then the smaller dx. */
static void search_es(const or_pair *fp, const or_params *p, int x0, int y0, int *bx, int *by, uint32_t *bc,
                      int *pts) {
    int S = p->search_range;
    int have = 0, n = 0;
    for (int dy = -S; dy <= S; ++dy) {
        for (int dx = -S; dx <= S; ++dx) {
            if (!feasible(fp, p, x0, y0, dx, dy)) continue;
            ++n;
            uint32_t c = or_sad(fp, x0, y0, dx, dy);
            int l1 = iabs(dx) + iabs(dy), bl1 = iabs(*bx) + iabs(*by);
            int better = !have || c < *bc || (c == *bc && (l1 < bl1 || (l1 == bl1 && (dy < *by || (dy == *by && dx < *bx)))));
            if (better) {
                have = 1;
                *bc = c;
                *bx = dx;
                *by = dy;
            }
        }
    }
    *pts = n;
}

/* evaluated-position memo over the (2S+1)^2 window */
typedef struct {
    int S;
    uint8_t *seen;
    int count;
} memo;

static void memo_visit(memo *m, int dx, int dy) {
    size_t i = (size_t)(dy + m->S) * (2 * m->S + 1) + (dx + m->S);
    if (!m->seen[i]) {
        m->seen[i] = 1;
        ++m->count;
    }
}

/* Three-step search: first step 2^(ceil(log2(S+1)) - 1), halved down to 1;
 * each round the eight points around the centre in row order; the centre
 * moves only to a strictly better point (the first one on ties). */
static void search_tss(const or_pair *fp, const or_params *p, int x0, int y0, memo *m, int *bx, int *by,
                       uint32_t *bc) {
    int S = p->search_range;
    int p2 = 1;
    while (p2 < S + 1) p2 *= 2;
    int step = p2 / 2;
    int cx = 0, cy = 0;
    uint32_t cc = or_sad(fp, x0, y0, 0, 0);
    memo_visit(m, 0, 0);
    while (step >= 1) {
        int nx = cx, ny = cy;
        uint32_t nc = cc;
        for (int j = -1; j <= 1; ++j) {
            for (int i = -1; i <= 1; ++i) {
                if (i == 0 && j == 0) continue;
                int qx = cx + i * step, qy = cy + j * step;
                if (!feasible(fp, p, x0, y0, qx, qy)) continue;
                memo_visit(m, qx, qy);
                uint32_t c = or_sad(fp, x0, y0, qx, qy);
                if (c < nc) {
                    nc = c;
                    nx = qx;
                    ny = qy;
                }
            }
        }
        cx = nx;
        cy = ny;
        cc = nc;
        step /= 2;
    }
    *bx = cx;
    *by = cy;
    *bc = cc;
}

static const int LDSP[8][2] = {{0, -2}, {-1, -1}, {1, -1}, {-2, 0}, {2, 0}, {-1, 1}, {1, 1}, {0, 2}};
static const int SDSP[4][2] = {{0, -1}, {-1, 0}, {1, 0}, {0, 1}};

/* Diamond search: the large diamond is repeated until its centre is the
 * best point (moves need a strictly smaller SAD), then one small diamond. */
static void search_ds(const or_pair *fp, const or_params *p, int x0, int y0, memo *m, int *bx, int *by,
                      uint32_t *bc) {
    int cx = 0, cy = 0;
    uint32_t cc = or_sad(fp, x0, y0, 0, 0);
    memo_visit(m, 0, 0);
    for (;;) {
        int nx = cx, ny = cy;
        uint32_t nc = cc;
        for (int o = 0; o < 8; ++o) {
            int qx = cx + LDSP[o][0], qy = cy + LDSP[o][1];
            if (!feasible(fp, p, x0, y0, qx, qy)) continue;
            memo_visit(m, qx, qy);
            uint32_t c = or_sad(fp, x0, y0, qx, qy);
            if (c < nc) {
                nc = c;
                nx = qx;
                ny = qy;
            }
        }
        if (nx == cx && ny == cy) break;
        cx = nx;
        cy = ny;
        cc = nc;
    }
    int nx = cx, ny = cy;
    uint32_t nc = cc;
    for (int o = 0; o < 4; ++o) {
        int qx = cx + SDSP[o][0], qy = cy + SDSP[o][1];
        if (!feasible(fp, p, x0, y0, qx, qy)) continue;
        memo_visit(m, qx, qy);
        uint32_t c = or_sad(fp, x0, y0, qx, qy);
        if (c < nc) {
            nc = c;
            nx = qx;
            ny = qy;
        }
    }
    *bx = nx;
    *by = ny;
    *bc = nc;
}

/* Four-step search [6]: the 9-point pattern of step 2 (a 5 x 5 square)
 * around the origin; while its best point is not the centre the centre moves
 * there and the square is evaluated again, for at most n5 squares in all
 * (three at S = 7: the reach 2 n5 + 1 of the squares plus the last step is
 * then +-7; n5 = ceil((S - 1) / 2), at least one, in general); then the
 * 3 x 3 square of step 1 around the centre.  Points of a square that were
 * evaluated before are not counted again; moves need a strictly smaller SAD
 * and the first point in row order wins ties. */
static void search_4ss(const or_pair *fp, const or_params *p, int x0, int y0, memo *m, int *bx, int *by,
                       uint32_t *bc) {
    int S = p->search_range;
    int n5 = S / 2; /* = ceil((S - 1) / 2) */
    if (n5 < 1) n5 = 1;
    int cx = 0, cy = 0;
    uint32_t cc = or_sad(fp, x0, y0, 0, 0);
    memo_visit(m, 0, 0);
    for (int round = 0; round < n5 + 1; ++round) {
        int step = round < n5 ? 2 : 1;
        int nx = cx, ny = cy;
        uint32_t nc = cc;
        for (int j = -1; j <= 1; ++j) {
            for (int i = -1; i <= 1; ++i) {
                if (i == 0 && j == 0) continue;
                int qx = cx + i * step, qy = cy + j * step;
                if (!feasible(fp, p, x0, y0, qx, qy)) continue;
                memo_visit(m, qx, qy);
                uint32_t c = or_sad(fp, x0, y0, qx, qy);
                if (c < nc) {
                    nc = c;
                    nx = qx;
                    ny = qy;
                }
            }
        }
        int moved = nx != cx || ny != cy;
        cx = nx;
        cy = ny;
        cc = nc;
        if (step == 2 && !moved) round = n5 - 1; /* centre won: the step-1 square is next */
    }
    *bx = cx;
    *by = cy;
    *bc = cc;
}

/* method 0 = exhaustive, 1 = three-step, 2 = diamond, 3 = four-step; texture
 * SAD on every non-transparent MB, starting at (0, 0). */
int or_search(int method, const or_pair *fp, const uint8_t *cls, const or_params *p, int16_t *mv, int16_t *mv_int,
              uint32_t *cost, uint16_t *points) {
    if (!fp || !p || !mv || !mv_int || method < 0 || method > 3) return -1;
    if (fp->width % 16 || fp->height % 16 || fp->width <= 0 || fp->height <= 0) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    int S = p->search_range;
    size_t win = (size_t)(2 * S + 1) * (2 * S + 1);
    uint8_t *seen = (uint8_t *)malloc(win);
    if (!seen) return -1;
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int k = v * wm + h;
            int c = cls ? cls[k] : OR_OPAQUE;
            int bx = 0, by = 0, pts = 0;
            uint32_t bc = 0;
            if (c != OR_TRANSPARENT) {
                if (method == 0) {
                    search_es(fp, p, 16 * h, 16 * v, &bx, &by, &bc, &pts);
                } else {
                    memo m = {S, seen, 0};
                    memset(seen, 0, win);
                    if (method == 1)
                        search_tss(fp, p, 16 * h, 16 * v, &m, &bx, &by, &bc);
                    else if (method == 2)
                        search_ds(fp, p, 16 * h, 16 * v, &m, &bx, &by, &bc);
                    else
                        search_4ss(fp, p, 16 * h, 16 * v, &m, &bx, &by, &bc);
                    pts = m.count;
                }
            }
            mv[2 * k] = mv_int[2 * k] = (int16_t)(2 * bx);
            mv[2 * k + 1] = mv_int[2 * k + 1] = (int16_t)(2 * by);
            if (cost) cost[k] = bc;
            if (points) points[k] = (uint16_t)pts;
        }
    }
    free(seen);
    return 0;
}

/* ---------------------------------------- motion compensation and SSE */
/* Section 4: the motion-compensated prediction of the current frame (each MB
 * predicted by its half-pel vector, transparent MBs by (0, 0)) and its
 * squared error against the current frame over the VOP pixels (every pixel
 * for rectangular frames). */
int or_mc_sse(const or_pair *fp, const uint8_t *cls, const int16_t *mv, uint8_t *pred, uint64_t *sse, uint64_t *npix) {
    if (!fp || !mv || !sse || !npix) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    uint64_t s = 0, n = 0;
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int k = v * wm + h;
            int c = cls ? cls[k] : OR_OPAQUE;
            int hx = c == OR_TRANSPARENT ? 0 : mv[2 * k];
            int hy = c == OR_TRANSPARENT ? 0 : mv[2 * k + 1];
            for (int j = 0; j < 16; ++j) {
                for (int i = 0; i < 16; ++i) {
                    int x = 16 * h + i, y = 16 * v + j;
                    int pv = pred_half(fp, x, y, hx, hy);
                    if (pred) pred[(size_t)y * fp->stride + x] = (uint8_t)pv;
                    int in = fp->cur_alpha ? fp->cur_alpha[(size_t)y * fp->stride + x] != 0 : 1;
                    if (in) {
                        int d = luma_at(fp->cur_luma, fp->stride, x, y) - pv;
                        s += (uint64_t)(d * d);
                        ++n;
                    }
                }
            }
        }
    }
    *sse = s;
    *npix = n;
    return 0;
}

/* ------------------------------------ four vectors per MB (Section 3.2) */
/*
 * Section 3.2 notes that MPEG-4 allows four motion vectors per MB and that
 * the recursive search therefore works on 8 x 8 blocks.  Reading: the
 * block-recursive search of Fig. 1 stays per MB (its candidates are MB
 * vectors); the pel-recursive refinement is then applied to each 8 x 8 block
 * b (raster order: top-left, top-right, bottom-left, bottom-right) of every
 * texture (opaque) MB, starting from the MB's full-pel vector mv_int: the
 * same gradient pass over the 64 pixels of the block, the same step, accept
 * and stop rule, 8 x 8 SAD as the cost, the displaced 8 x 8 block inside the
 * frame and |d| <= S; then (half_pel) the eight half-sample offsets around
 * the block's vector.  Boundary MBs keep their one (shape) vector, repeated;
 * transparent MBs get zero vectors.  Per block: mv4 (half-pel), cost4 (final
 * 8 x 8 SAD), iters4 (recursion candidates), points4 (8 x 8 blocks compared
 * beyond the start: recursion candidates and feasible half-sample ones).
 */
int or_prs8(const or_pair *fp, const uint8_t *cls, const int16_t *mv, const int16_t *mv_int, const or_params *p,
            int16_t *mv4, uint32_t *cost4, uint8_t *iters4, uint16_t *points4) {
    if (!fp || !p || !mv || !mv_int || !mv4) return -1;
    if (fp->width % 16 || fp->height % 16 || fp->width <= 0 || fp->height <= 0) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int k = v * wm + h;
            int c = cls ? cls[k] : OR_OPAQUE;
            for (int b = 0; b < 4; ++b) {
                int q = 4 * k + b;
                int hx = 0, hy = 0, its = 0, pts = 0;
                uint32_t cost = 0;
                if (c == OR_OPAQUE) {
                    int bx0 = 16 * h + 8 * (b & 1), by0 = 16 * v + 8 * (b >> 1);
                    int dx = half_to_full(mv_int[2 * k]), dy = half_to_full(mv_int[2 * k + 1]);
                    cost = sad_n(fp, bx0, by0, 8, dx, dy);
                    its = pel_recursion_n(fp, p, 0, NULL, bx0, by0, 8, &dx, &dy, &cost);
                    pts = its;
                    hx = 2 * dx;
                    hy = 2 * dy;
                    if (p->half_pel) {
                        int bhx = hx, bhy = hy;
                        for (int o = 0; o < 8; ++o) {
                            int qx = hx + HALF_OFFS[o][0], qy = hy + HALF_OFFS[o][1];
                            if (!half_feasible_n(fp, p, bx0, by0, 8, qx, qy)) continue;
                            ++pts;
                            uint32_t c2 = sad_half_n(fp, bx0, by0, 8, qx, qy);
                            if (c2 < cost) {
                                cost = c2;
                                bhx = qx;
                                bhy = qy;
                            }
                        }
                        hx = bhx;
                        hy = bhy;
                    }
                } else if (c == OR_BOUNDARY) {
                    hx = mv[2 * k];
                    hy = mv[2 * k + 1];
                }
                mv4[2 * q] = (int16_t)hx;
                mv4[2 * q + 1] = (int16_t)hy;
                if (cost4) cost4[q] = cost;
                if (iters4) iters4[q] = (uint8_t)its;
                if (points4) points4[q] = (uint16_t)pts;
            }
        }
    }
    return 0;
}

/* Motion compensation with four vectors per MB: each 8 x 8 block predicted
 * by its own half-pel vector (transparent MBs by (0, 0)); SSE over the VOP
 * pixels (every pixel for rectangular frames), as or_mc_sse. */
int or_mc4_sse(const or_pair *fp, const uint8_t *cls, const int16_t *mv4, uint8_t *pred, uint64_t *sse,
               uint64_t *npix) {
    if (!fp || !mv4 || !sse || !npix) return -1;
    int wm = fp->width / 16, hm = fp->height / 16;
    uint64_t s = 0, n = 0;
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int k = v * wm + h;
            int c = cls ? cls[k] : OR_OPAQUE;
            for (int j = 0; j < 16; ++j) {
                for (int i = 0; i < 16; ++i) {
                    int q = 4 * k + 2 * (j / 8) + i / 8;
                    int hx = c == OR_TRANSPARENT ? 0 : mv4[2 * q];
                    int hy = c == OR_TRANSPARENT ? 0 : mv4[2 * q + 1];
                    int x = 16 * h + i, y = 16 * v + j;
                    int pv = pred_half(fp, x, y, hx, hy);
                    if (pred) pred[(size_t)y * fp->stride + x] = (uint8_t)pv;
                    int in = fp->cur_alpha ? fp->cur_alpha[(size_t)y * fp->stride + x] != 0 : 1;
                    if (in) {
                        int d = luma_at(fp->cur_luma, fp->stride, x, y) - pv;
                        s += (uint64_t)(d * d);
                        ++n;
                    }
                }
            }
        }
    }
    *sse = s;
    *npix = n;
    return 0;
}

/* ------------------------------------------------ reference VOP padding */
/*
 * Section 4 protocol: the reference is an MPEG-4 VOP, whose texture outside
 * the shape is filled before blocks are matched against it (MPEG-4 Visual's
 * padding of arbitrarily shaped VOPs, on the frame's MB grid).  Inside means
 * alpha != 0.
 *  - Opaque MB: copied.
 *  - Boundary MB, repetitive padding within its 16x16 block.  Along each row,
 *    a sample outside the shape takes the rounded-up mean of the nearest
 *    inside samples to its left and right, or the one of them that exists;
 *    a row with no inside sample stays open.  Then along each column, an open
 *    sample takes the rounded-up mean of the nearest row-padded samples above
 *    and below, or the one that exists.
 *  - Transparent MB, extended padding: the border of the first adjacent MB
 *    that is not transparent, in the order left, above, right, below, is
 *    repeated over the block: the left MB's last column along each row, the
 *    upper MB's last row down each column, the right MB's first column, the
 *    lower MB's first row.  With no such neighbour, every sample is 128.
 * `out` (row stride out_stride) must not overlap `luma`.
 */
static int pad_mean(int a, int b) { return (a + b + 1) >> 1; }

int or_pad_vop(const uint8_t *luma, const uint8_t *alpha, int width, int height, int stride, uint8_t *out,
               int out_stride) {
    if (!luma || !alpha || !out || width <= 0 || height <= 0 || width % 16 || height % 16 || stride < width ||
        out_stride < width)
        return -1;
    int wm = width / 16, hm = height / 16;
    uint8_t *cls = (uint8_t *)malloc((size_t)wm * hm);
    if (!cls) return -1;
    or_classify(alpha, width, height, stride, cls, NULL);
    /* opaque and boundary MBs */
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int c = cls[v * wm + h], x0 = 16 * h, y0 = 16 * v;
            if (c == OR_TRANSPARENT) continue;
            int val[16][16], in[16][16], row_open[16];
            for (int j = 0; j < 16; ++j)
                for (int i = 0; i < 16; ++i) {
                    val[j][i] = luma_at(luma, stride, x0 + i, y0 + j);
                    in[j][i] = alpha[(size_t)(y0 + j) * stride + x0 + i] != 0;
                }
            if (c == OR_BOUNDARY) {
                int hp[16][16];
                for (int j = 0; j < 16; ++j) {
                    row_open[j] = 1;
                    for (int i = 0; i < 16; ++i) row_open[j] &= !in[j][i];
                    for (int i = 0; i < 16; ++i) {
                        if (in[j][i]) {
                            hp[j][i] = val[j][i];
                            continue;
                        }
                        int l = i - 1, r = i + 1;
                        while (l >= 0 && !in[j][l]) --l;
                        while (r < 16 && !in[j][r]) ++r;
                        if (l >= 0 && r < 16) hp[j][i] = pad_mean(val[j][l], val[j][r]);
                        else if (l >= 0) hp[j][i] = val[j][l];
                        else if (r < 16) hp[j][i] = val[j][r];
                        else hp[j][i] = -1; /* open */
                    }
                }
                for (int i = 0; i < 16; ++i) {
                    for (int j = 0; j < 16; ++j) {
                        if (!row_open[j]) {
                            val[j][i] = hp[j][i];
                            continue;
                        }
                        int u = j - 1, d = j + 1;
                        while (u >= 0 && row_open[u]) --u;
                        while (d < 16 && row_open[d]) ++d;
                        /* a boundary MB has an inside sample, so some row is filled */
                        if (u >= 0 && d < 16) val[j][i] = pad_mean(hp[u][i], hp[d][i]);
                        else if (u >= 0) val[j][i] = hp[u][i];
                        else val[j][i] = hp[d][i];
                    }
                }
            }
            for (int j = 0; j < 16; ++j)
                for (int i = 0; i < 16; ++i) out[(size_t)(y0 + j) * out_stride + x0 + i] = (uint8_t)val[j][i];
        }
    }
    /* transparent MBs, from their padded neighbours */
    for (int v = 0; v < hm; ++v) {
        for (int h = 0; h < wm; ++h) {
            int k = v * wm + h, x0 = 16 * h, y0 = 16 * v;
            if (cls[k] != OR_TRANSPARENT) continue;
            for (int j = 0; j < 16; ++j) {
                for (int i = 0; i < 16; ++i) {
                    int s;
                    if (h > 0 && cls[k - 1] != OR_TRANSPARENT) s = out[(size_t)(y0 + j) * out_stride + x0 - 1];
                    else if (v > 0 && cls[k - wm] != OR_TRANSPARENT) s = out[(size_t)(y0 - 1) * out_stride + x0 + i];
                    else if (h + 1 < wm && cls[k + 1] != OR_TRANSPARENT) s = out[(size_t)(y0 + j) * out_stride + x0 + 16];
                    else if (v + 1 < hm && cls[k + wm] != OR_TRANSPARENT) s = out[(size_t)(y0 + 16) * out_stride + x0 + i];
                    else s = 128;
                    out[(size_t)(y0 + j) * out_stride + x0 + i] = (uint8_t)s;
                }
            }
        }
    }
    free(cls);
    return 0;
}

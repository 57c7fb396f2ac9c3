/*
 * me.h - C ABI of the MI355X (gfx950) shape-adaptive motion-estimation
 * library, after F. Benboubker, F. Abdi, A. Ahaitouf, "Shape-Adaptive Motion
 * Estimation Algorithm for MPEG-4 Video Coding".
 *
 * Problem statement (Section 2): for every 16x16 macroblock (MB) of the
 * current video object plane (VOP) find the motion vector into the reference
 * VOP that minimises the block distortion; boundary MBs are matched on their
 * binary alpha blocks (BABs), opaque MBs on luma (Section 1, Section 3.1).
 *
 * Common conventions
 *  - All frame, class, vector and result pointers inside the structs are
 *    DEVICE pointers (hipMalloc / torch CUDA tensors) owned by the caller.
 *    Arrays of structs and arrays of pointers passed as arguments are HOST
 *    memory and may be reused as soon as the call returns.
 *  - Frames are 8-bit, row-major with a row pitch of `stride` bytes; width
 *    and height must be multiples of 16 (ME_EALIGN), `stride` >= width and a
 *    multiple of 4, and plane base pointers 4-byte aligned (ME_EALIGN).
 *  - MB (h, v) covers pixels [16h, 16h+16) x [16v, 16v+16); per-MB arrays
 *    are row-major over the MB grid, (height/16) x (width/16).
 *  - A full-pel vector d = (dx, dy) predicts cur(x, y) by ref(x+dx, y+dy).
 *    Every me_mv is in HALF-PEL units; integer results are even.
 *  - Admissible vectors: |dx|, |dy| <= search_range and the displaced block
 *    entirely inside the reference frame (the second condition is dropped
 *    with ME_FLAG_UNRESTRICTED).
 *  - Every call validates all arguments on the host before touching the GPU
 *    and returns a negative ME_E* code on error (nothing launched).  Calls
 *    are asynchronous on `stream` (a hipStream_t; NULL = default stream)
 *    except me_motion_compensate_psnr and me_device_status, which block.
 *  - The library owns only internal scratch (per stream, grown on demand,
 *    released by me_shutdown).  Calls that share a stream are ordered; calls
 *    on different streams must not share output buffers.
 */
#ifndef ME_H
#define ME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ME_OK 0
#define ME_EINVAL (-1)   /* null pointer, size or parameter out of range */
#define ME_EALIGN (-2)   /* width/height not multiples of 16, bad stride/alignment */
#define ME_EHIP (-3)     /* HIP runtime error */
#define ME_ENOMEM (-4)   /* internal scratch allocation failed */
#define ME_EEMPTY (-5)   /* PSNR over zero pixels */
#define ME_EDEVICE (-6)  /* device status word set (dependency wait timed out / bad class) */
#define ME_ENODEV (-7)   /* no usable gfx950 device */
#define ME_EFORMAT (-8)  /* network checkpoint malformed (size, magic, version, checksum, values) */
#define ME_EIO (-9)      /* network checkpoint file could not be opened, read or written */

/* MB classes (Section 1) */
#define ME_MB_TRANSPARENT 0 /* no pixel of the VOP */
#define ME_MB_OPAQUE 1      /* every pixel inside the VOP */
#define ME_MB_BOUNDARY 2    /* both */

/* baseline methods (Section 1 references [5], [6], [7]; Tables 1-2) */
#define ME_ES 0  /* exhaustive search */
#define ME_TSS 1 /* three-step search */
#define ME_DS 2  /* diamond search */
#define ME_4SS 3 /* four-step search */

typedef struct me_frame {
    const uint8_t *luma;  /* composited luma (device) */
    const uint8_t *alpha; /* binary alpha of this VOP, inside <=> != 0; NULL = rectangular frame */
    int32_t width, height, stride;
} me_frame;

typedef struct me_mv {
    int16_t x, y; /* half-pel units */
} me_mv;

typedef struct me_params {
    int32_t search_range; /* S, 1..64 (full-pel) */
    int32_t theta;        /* Theta of Eq. 4, 1..127 (default 3: "two or three") */
    int32_t eps_q12;      /* convergence factor epsilon of Eq. 3 in Q.12, 0..65536 (default 4096 = 1.0) */
    int32_t max_step;     /* largest per-axis pel-recursion step, 1..S (default 1: one of eight neighbours) */
    int32_t k_max;        /* cap on pel-recursion candidates per MB, 0..255 (default 8); at most 127
                             when any job carries seeds (a dropped seed counts both recursions, and
                             `iters` is a byte), ME_EINVAL otherwise */
    int32_t half_pel;     /* 1: half-sample refinement of texture MBs after the recursion (Section 4) */
    uint32_t flags;       /* ME_FLAG_* bits below; others must be 0 */
} me_params;

/* me_params.flags */
#define ME_FLAG_UNRESTRICTED 0x1u   /* unrestricted vectors (MPEG-4 reference padding; the Section 4
                                       protocol): a vector is admissible when |dx|, |dy| <= S wherever
                                       the displaced block lands, the reference being extended by
                                       repeating its edge pixels (as MC always reads it); applies to
                                       every search, the half-sample step and me_refine_8x8 */
#define ME_FLAG_T_TEXTURE 0x2u      /* Section 3.1 text: a boundary MB's temporal candidate T is evaluated
                                       on texture - its spatial candidates A, B, C are scored on the
                                       BABs (first minimum), and T replaces their winner when its luma
                                       SAD over the MB's VOP pixels is strictly lower (one more compared
                                       block); the recursion then runs on the BABs as before.  Used by
                                       me_texture_recursive (me_shape_search ignores it) */
#define ME_FLAG_MASKED_PRS 0x4u     /* a reading of Section 3.1 (T of a boundary MB evaluated on texture):
                                       a boundary MB's pel recursion (Section 3.2) refines on luma over
                                       the current VOP's pixels - its start is the candidate winner
                                       (scored as above) with that winner's luma SAD over the VOP pixels
                                       (one more compared block), each gradient pass sums only VOP
                                       pixels, each candidate's distortion is its luma SAD over them,
                                       and `cost` reports that SAD.  No half-sample step for boundary
                                       MBs.  Used by me_texture_recursive and the batch
                                       (me_shape_search ignores it) */
#define ME_FLAG_LINE_WORKERS 0x100u /* schedule the proposed search with line workers (one MB position
                                       across a chain's pairs) even when no job's T field is written in
                                       the same call, where row workers (one MB row per wave) are the
                                       default; the results are the same */

/* One frame pair of one VOP (the unit of Fig. 1's outer loops). */
typedef struct me_job {
    me_frame cur, ref;       /* same width/height/stride; alpha both set or both NULL */
    const uint8_t *mb_class; /* per-MB class from me_classify_babs of cur; NULL = all opaque */
    const me_mv *t_field;    /* temporal candidates T (previous pair's mv_int); NULL = zeros.
                                May point at the mv_int of an EARLIER job of the same call:
                                that pair is then solved first, MB by MB (pipelined); such a
                                chain holds at most 65535 pairs (ME_EINVAL otherwise). */
    const me_mv *seed;       /* learned starting vectors for texture MBs; NULL = plain method */
    me_mv *mv;               /* out: final vector (half-pel) */
    me_mv *mv_int;           /* out: full-pel vector before half-sample refinement (feeds A, B, C, T) */
    uint32_t *cost;          /* out, nullable: final distortion (SAD, or BAB mismatch count) */
    uint8_t *iters;          /* out, nullable: pel-recursion candidates evaluated */
    uint16_t *points;        /* out, nullable: search points (compared blocks), Table 1 */
} me_job;

typedef struct me_net me_net; /* learned MV proposal network (opaque) */

/* Fill `p` with the defaults: S 16, Theta 3, eps 1.0, max_step 1, k_max 8, no half-pel. */
void me_default_params(me_params *p);

/*
 * Learned motion-vector proposal network (an addition to the paper's
 * method: it seeds the pel-recursive search of Section 3.2 for opaque MBs;
 * the block-recursive result stays the fallback, see me_job.seed).
 * Per MB, at window scale f (2 or 4): input 2 x 24 x 24 (the current MB and
 * the frame-clamped reference window [-(12f-8), 12f+8) around it - 24f
 * pixels, [-16, 32) at f = 2 - both box-averaged f x f, an f x f sum s as
 * (s - 128 f^2) / (128 f^2) in bfloat16); conv 3x3 2->32 stride 1 + ReLU;
 * conv 3x3 32->32 stride 2 + ReLU; conv 3x3 32->2 stride 2; mean over the
 * 6 x 6 positions = predicted full-pel vector p; seed = 2 * clamp(rint(p),
 * -w, w) half-pel with w = 12f - 8.  bfloat16 weights and activations, fp32
 * accumulation.  Parameters (ME_NET_PARAMS floats): W1 (32,3,3,2) | b1 (32)
 * | W2 (32,3,3,32) | b2 (32) | W3 (2,3,3,32) | b3 (2), weights laid out
 * [out][ky][kx][in].  The MBs served are the opaque ones (every MB of a job
 * whose mb_class is NULL).
 *
 * me_net_create: fp32 master weights from the host array `init` on the
 *   current device (momentum zero), window scale `scale` (2 or 4;
 *   ME_EINVAL otherwise).  *out = handle (NULL on error).
 * me_net_forward: for every served MB, writes the seed into job.seed (if
 *   set) and p (2 floats at 2*k) into pred[i] (host array of n device
 *   pointers, itself nullable, entries nullable).  Only cur/ref/mb_class/seed
 *   of the jobs are read.  Asynchronous on `stream`.
 * me_net_backward: the gradient g of the loss over the served MBs of
 *   `jobs`, labels[i] = device field of full-pel vectors in half-pel units
 *   (the plain method's mv_int): loss = sum |p - label/2|^2 / (2 B) over the
 *   B served MBs.  grad (device, ME_NET_PARAMS floats, required) receives g;
 *   loss (host, nullable) the loss - then the call blocks.  The weights are
 *   not changed.  The gradient sum is deterministic for a given device and
 *   job set.
 * me_net_sgd_step: one momentum-SGD step from the gradient `grad` (device):
 *   v = momentum * v + grad; w = w - lr * v (0 <= momentum < 1, lr >= 0).
 * me_net_train_step: me_net_backward then me_net_sgd_step in one call
 *   (grad nullable here: receives g when set).
 * me_net_weights: blocking copy of the master weights (and momentum, nullable).
 * me_net_scale: the window scale (ME_EINVAL for NULL).
 * me_net_save: blocking; writes a checkpoint to `path`: 8-byte magic
 *   "ME-NET\0\0", u32 version 1, u32 ME_NET_PARAMS, u32 window scale, u32 0,
 *   the fp32 weights, the fp32 momentum, and the 64-bit FNV-1a hash of every
 *   preceding byte (little-endian).  ME_EIO when the file cannot be written.
 * me_net_load: creates a network on the current device from a checkpoint;
 *   ME_EIO when the file cannot be read, ME_EFORMAT when its size, magic,
 *   version, parameter count, hash, scale or values are wrong.
 * me_net_destroy: waits for the device and frees (NULL is a no-op).
 */
#define ME_NET_PARAMS 10434
int me_net_create(const float *init, int32_t scale, me_net **out);
int me_net_forward(me_net *net, const me_job *jobs, int n, float *const *pred, void *stream);
int me_net_backward(me_net *net, const me_job *jobs, int n, const me_mv *const *labels, float *grad, double *loss,
                    void *stream);
int me_net_sgd_step(me_net *net, const float *grad, float lr, float momentum, void *stream);
int me_net_train_step(me_net *net, const me_job *jobs, int n, const me_mv *const *labels, float lr, float momentum,
                      float *grad, double *loss, void *stream);
int me_net_weights(me_net *net, float *weights, float *momentum);
int me_net_scale(const me_net *net);
int me_net_save(me_net *net, const char *path);
int me_net_load(const char *path, me_net **out);
void me_net_destroy(me_net *net);

/* Human-readable text of a status code (static storage). */
const char *me_status_str(int status);

/* Release every stream workspace (device scratch, pinned staging).  Waits for
 * the device.  Optional; the library re-initialises on the next call. */
void me_shutdown(void);

/*
 * MB classification from the binary alpha plane (Section 1; Fig. 1 Block_Type):
 * class 0 transparent, 1 opaque, 2 boundary, counted over alpha != 0.
 *  frames[i].alpha  required (device); luma unused.
 *  mb_class[i]      device, (height/16)*(width/16) bytes.
 *  bab_bits[i]      device or NULL; 8 uint32 per MB: word w holds rows 2w
 *                   (bits 0..15) and 2w+1 (bits 16..31), column i at bit i.
 *  `bab_bits` itself may be NULL.
 */
int me_classify_babs(const me_frame *frames, int n, uint8_t *const *mb_class, uint32_t *const *bab_bits,
                     void *stream);

/*
 * Reference VOP padding (Section 4 protocol: the reference is an MPEG-4 VOP,
 * whose texture outside the shape is filled before blocks are matched
 * against it; MPEG-4 Visual's padding of arbitrarily shaped VOPs, applied on
 * the frame's MB grid).  Inside means alpha != 0.
 *  - Opaque MBs are copied.
 *  - Boundary MBs: repetitive padding within the 16x16 block.  Along each
 *    row, a sample outside the shape takes the rounded-up mean of the
 *    nearest inside samples to its left and right, or the one that exists.
 *    Rows with no inside sample then take the same rule along each column,
 *    over the row-padded samples.
 *  - Transparent MBs: extended padding.  The block repeats the border of the
 *    first adjacent MB that is not transparent, in the order left, above,
 *    right, below: the left MB's last column along each row, the upper MB's
 *    last row down each column, the right MB's first column, the lower MB's
 *    first row.  With no such neighbour, every sample is 128.
 *  frames[i].luma, .alpha  the reference frame's luma and this VOP's alpha
 *                          (device, both required, checked as for
 *                          me_classify_babs).
 *  padded[i]   device, caller-owned: height rows of frames[i].stride bytes,
 *              4-byte aligned; the first width bytes of each row are
 *              written.  It must not overlap the frame's luma or alpha
 *              (ME_EINVAL when it is the same address).
 * Pass padded[i] as the `ref.luma` of the VOP's search and MC jobs.  At most
 * 65,535 VOPs per call (ME_EINVAL beyond).  Asynchronous on `stream`.
 */
int me_pad_vops(const me_frame *frames, int n, uint8_t *const *padded, void *stream);

/*
 * The proposed algorithm (Fig. 1; Sections 3.1-3.2) for n frame pairs.
 * Per MB in raster order: transparent -> zero vector; otherwise the
 * block-recursive search over the candidates A (left), B (up), C (up-right)
 * of this pair and T, keeping the first minimum of the distortion (BAB
 * mismatch count for boundary MBs, luma SAD for opaque MBs), then the
 * pel-recursive refinement of Eqs. 3-5 in Q.12 fixed point, then (half_pel)
 * half-sample refinement of opaque MBs.  `net` NULL: each job's `seed` (if
 * set) is used as given; non-NULL: the network writes its proposals into the
 * jobs' `seed` buffers first (they must then be writable device buffers).
 */
int me_texture_recursive(const me_job *jobs, int n, const me_params *params, const me_net *net, void *stream);

/* Same procedure with every non-transparent MB scored on its BAB (shape
 * motion estimation of Section 3.1 applied to all object MBs).  Requires alpha. */
int me_shape_search(const me_job *jobs, int n, const me_params *params, void *stream);

/*
 * Baseline block matching on the luma of every non-transparent MB, starting
 * at (0, 0): ME_ES (all admissible vectors; ties -> smaller |dx|+|dy|, then
 * smaller dy, then smaller dx), ME_TSS (first step 2^(ceil(log2(S+1))-1),
 * halved to 1), ME_DS (large diamond until the centre wins, then the small
 * diamond), ME_4SS (the 5x5 square of step 2 around the centre until the
 * centre wins, at most ceil((S-1)/2) squares - three at S = 7 as in [6] -
 * then the 3x3 square of step 1).  Moves need a strictly smaller SAD; among
 * the eight points of a pattern the first in row order wins ties.  `points`
 * counts distinct positions evaluated; iters is written 0; t_field and seed
 * are ignored.
 */
int me_full_search(int method, const me_job *jobs, int n, const me_params *params, void *stream);

/*
 * Motion compensation and PSNR (Section 4, Table 2): predict every MB of
 * cur from ref by its `mv` (half-pel, MPEG-4 bilinear with rounding control
 * 0, reference coordinates clamped to the frame; transparent MBs use (0,0)),
 * then SSE over the VOP pixels (alpha != 0; all pixels when alpha is NULL).
 *  pred     NULL, or host array of n device pointers (entries may be NULL)
 *           receiving the predicted frame with the job's stride.
 *  sse, npix, psnr_db   host arrays of n; psnr = 10 log10(255^2 npix / sse)
 *           in double (+inf when sse == 0).  ME_EEMPTY if some npix is 0
 *           (all outputs still written; that job's psnr is NaN).
 * Blocks until the results are on the host.
 */
int me_motion_compensate_psnr(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sse, uint64_t *npix,
                              double *psnr_db, void *stream);

/*
 * The same motion compensation and masked SSE (Section 4, Table 2) without
 * waiting: the per-job sums land in DEVICE memory when the stream reaches
 * them, and the call returns once the work is queued, so a caller can queue
 * the next frame step before reading these results.
 *  pred     as in me_motion_compensate_psnr.
 *  sums     2n uint64 in device-accessible memory: device memory, or pinned
 *           host memory from hipHostMalloc (then readable on the host once
 *           the stream has passed this call, with no copy); 8-byte aligned
 *           (ME_EALIGN otherwise); owned by the caller.  sums[2i] = SSE of
 *           job i, sums[2i+1] = its pixel count over the VOP (0 for a job
 *           without VOP pixels; no ME_EEMPTY here).
 *           PSNR = 10 log10(255^2 npix / sse).
 * Errors are those of me_motion_compensate_psnr found on the host; the jobs
 * array may be reused on return.
 */
int me_motion_compensate_sse(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sums, void *stream);

/*
 * Four motion vectors per MB (Section 3.2: MPEG-4 allows four vectors per
 * macroblock, so the recursive search works on 8 x 8 blocks).  The
 * block-recursive search of Fig. 1 stays per MB; me_refine_8x8 then applies
 * the pel-recursive refinement of Eqs. 3-5 to each 8 x 8 block (raster
 * order: top-left, top-right, bottom-left, bottom-right) of every texture
 * (opaque) MB, starting from the MB's full-pel vector: the gradient pass
 * over the block's 64 pixels, the same step, accept and stop rule, the 8 x 8
 * SAD as cost, the displaced 8 x 8 block inside the frame and |d| <= S; then
 * (half_pel) the eight half-sample offsets around each block's vector.
 * Boundary MBs keep their one (shape) vector in all four entries,
 * transparent MBs get zero vectors.
 *  jobs      a finished search's jobs: cur, ref, mb_class, mv (the MB's
 *            final vector, repeated on boundary MBs) and mv_int (the start;
 *            it must be admissible for the MB, as the search leaves it) are
 *            read; t_field, seed, cost, iters, points are ignored.
 *  mv4[i]    device, 4 me_mv per MB (half-pel), required.
 *  cost4[i], iters4[i], points4[i]  device or NULL (and the arrays of
 *            pointers themselves nullable): per block the final 8 x 8
 *            distortion, the recursion candidates evaluated, and the 8 x 8
 *            blocks compared beyond the start (recursion and half-sample
 *            candidates); zero for non-texture MBs.
 * Asynchronous on `stream`.
 *
 * me_motion_compensate4_sse: me_motion_compensate_sse with each 8 x 8 block
 * predicted by its own vector mv4[i] (transparent MBs by (0, 0)); the jobs'
 * mv is not read.  Same sums, errors and pinned-memory rules.
 */
int me_refine_8x8(const me_job *jobs, int n, const me_params *params, me_mv *const *mv4, uint32_t *const *cost4,
                  uint8_t *const *iters4, uint16_t *const *points4, void *stream);
int me_motion_compensate4_sse(const me_job *jobs, int n, const me_mv *const *mv4, uint8_t *const *pred,
                              uint64_t *sums, void *stream);

/*
 * me_motion_compensate_sse for callers that cannot allocate (code under HIP
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same prediction, masked SSE and per-job sums (same arguments, errors and
 * results), with the job table, the per-MB partial sums and the status slot
 * in a fixed array in device memory - one per GPU, about 4.2 MiB, held until
 * the process ends - so that no call allocates anything.  The job table is
 * passed to the device as kernel arguments.  Limits: n <= 1024 jobs and at
 * most 524288 MBs in all (ME_EINVAL beyond).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race; calls in order on one stream do not.  Not reported here: a
 * class byte above 2 (me_motion_compensate_sse raises the device status
 * word for it); kernel timing does not apply.
 */
int me_motion_compensate_sse_noalloc(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sums,
                                     void *stream);

/*
 * Batched frame step: many frame pairs (VOP streams of any sizes) per launch,
 * replayed once per frame step as one HIP graph (Fig. 1 applied to every job
 * of the step; classification as in me_classify_babs, search as in
 * me_texture_recursive / me_shape_search, MC + SSE as in
 * me_motion_compensate_psnr).
 *
 * me_batch_create fixes the STRUCTURE of a job set: n, each job's frame
 * size and stride, which of alpha / mb_class / seed / t_field are set, and
 * which jobs take an earlier job's mv_int as T (pipelined as in
 * me_texture_recursive).  Parameters and flags are fixed too:
 *  ME_BATCH_SHAPE     score every non-transparent MB on its BAB (as me_shape_search; alpha required)
 *  ME_BATCH_AUTOTUNE  pick the launch configuration by timing candidates on
 *                     `jobs` (their outputs and mb_class are written; every
 *                     configuration gives the same results)
 * The batch is bound to `stream` and to the current device.  *out receives
 * the handle (NULL on error).
 *
 * me_batch_step runs one frame step for `jobs` (same n and structure; any
 * device buffers): for every job with alpha and mb_class, the classes of
 * its cur alpha are WRITTEN to mb_class (so mb_class is an output here);
 * then the search writes mv, mv_int, cost, iters, points; then the SSE and
 * pixel counts over the VOP are summed on the device.  Asynchronous; the
 * `jobs` array may be reused on return.  ME_EINVAL if the structure differs.
 *
 * me_batch_results waits for the last step and writes its per-job SSE,
 * pixel count and PSNR (host arrays of n, in job order; as
 * me_motion_compensate_psnr), ME_EEMPTY if a job has no VOP pixel,
 * ME_EDEVICE if a kernel raised the device status word (then cleared).
 *
 * me_batch_config writes the launch configuration in use (ncfg >= 4; up
 * to six entries): search workers, window staging (1 staged plan, 0
 * generic), dependency-poll back-off (s_sleep units), MB blocks per CU of
 * the flat kernels, waves per line worker (1, 2 or 4: the searched pairs of
 * a line are dealt round-robin to its waves; row workers: rows per band),
 * and the search schedule (1: row workers, one wave per MB row, for job
 * sets whose T fields all come from earlier calls; 0: line workers).  With
 * ME_BATCH_AUTOTUNE a candidate whose run raises the device status word is
 * dropped (ME_EDEVICE when no candidate runs cleanly).
 * me_batch_destroy waits for the batch's stream and frees it (NULL is a no-op).
 */
typedef struct me_batch me_batch;
#define ME_BATCH_SHAPE 1u
#define ME_BATCH_AUTOTUNE 2u
int me_batch_create(const me_job *jobs, int n, const me_params *params, uint32_t flags, void *stream,
                    me_batch **out);
int me_batch_step(me_batch *b, const me_job *jobs, int n);
int me_batch_results(me_batch *b, uint64_t *sse, uint64_t *npix, double *psnr_db, int n);
int me_batch_config(const me_batch *b, int32_t *cfg, int ncfg);
/* Force the launch configuration (ncfg 5 or 6, same layout as
 * me_batch_config; a missing sixth entry means line workers): line workers
 * 1 .. min(lines, 16 x CUs / waves) with waves per line 1, 2 or 4, or row
 * workers (sixth entry 1, job sets without chains only) 1 .. the resident
 * workgroup count with rows per band 4; staging 0 or 1 (1 needs a staging
 * plan for this S), poll back-off 1, 2 or 4, flat MBs per CU 4, 8 or 16;
 * ME_EINVAL otherwise.  Every configuration computes the same results.
 * Waits for the batch's stream and re-captures the graph (with the kernel
 * timing now in force). */
int me_batch_set_config(me_batch *b, const int32_t *cfg, int ncfg);
/* Kernel durations inside the batch's graph: when me_kernel_timing has kind
 * k (ME_KT_CLASSIFY, ME_KT_SEARCH, ME_KT_MC, ME_KT_NET) on at the time the
 * graph is captured (me_batch_create, me_batch_set_net, me_batch_set_config),
 * every replay records an event pair around that kernel (event-record
 * nodes of the graph, added in the stream's capture order).
 * Waits for the replays, writes the sum of their durations (ms) and their
 * number, and restarts both at zero.  Zero counts when not timed. */
int me_batch_kernel_time_ms(me_batch *b, int kind, double *total_ms, int *count);
/* Seed the batch's searches with a proposal network (NULL detaches):
 * every step then runs the network on the opaque MBs between the
 * classification and the search, writing the jobs' seed buffers (so every
 * job of the structure must carry one; ME_EINVAL otherwise).  The network
 * must outlive the batch or be detached first; training it between steps
 * is allowed (the graph reads its current weights).  Waits for the batch's
 * stream and re-captures the graph. */
int me_batch_set_net(me_batch *b, me_net *net);
void me_batch_destroy(me_batch *b);

/*
 * Kernel timing (a profiling aid, off by default).  While on, every call
 * records a HIP event pair on its stream around its main kernel:
 *  ME_KT_CLASSIFY  me_classify_babs           classification kernel
 *  ME_KT_SEARCH    me_texture_recursive,      pipelined search kernel (not the
 *                  me_shape_search            transparent pre-pass before it)
 *  ME_KT_FULL      me_full_search             ES / TSS / DS kernel (not the compaction)
 *  ME_KT_MC        me_motion_compensate_psnr, prediction + SSE kernel (not the per-job sum)
 *                  me_motion_compensate_sse
 *  ME_KT_NET       me_net_forward (also via   network forward kernel (not the MB list)
 *                  me_texture_recursive)
 *  ME_KT_NET_TRAIN me_net_train_step          forward + backward kernel (not the SGD update)
 *  ME_KT_REFINE8   me_refine_8x8              8 x 8 block refinement kernel
 * me_kernel_timing: on = 0 (off), 1 (every kind), or ME_KT_ONLY(kind) bits
 * OR-ed together (only those kinds: the others record no events, which
 * add a few microseconds between kernels each); ME_EINVAL otherwise.
 * Affects later calls.
 * me_kernel_time_ms: waits for every timed call of `kind` on `stream`, writes
 * the sum of their main-kernel durations in milliseconds (host double) and
 * their number (host int), and restarts both sums at zero.
 */
#define ME_KT_CLASSIFY 0
#define ME_KT_SEARCH 1
#define ME_KT_FULL 2
#define ME_KT_MC 3
#define ME_KT_NET 4
#define ME_KT_NET_TRAIN 5
#define ME_KT_REFINE8 6
#define ME_KT_ONLY(kind) (2 << (kind))
int me_kernel_timing(int on);
int me_kernel_time_ms(int kind, void *stream, double *total_ms, int *count);

/*
 * Schedule of the pipelined search (host only, no device access): the order
 * in which me_texture_recursive / me_shape_search hand out MB "lines" (one MB
 * position of one chain of frame pairs, a chain being pairs linked by their
 * t_field) to the device workers.  The search needs this order to be
 * topological over the dependencies of Fig. 1 (A, B, C of the same pair, T of
 * the producing pair); it is exposed so that this can be checked.
 *  job_info  host, 3n: per job its chain, its position in the chain, and the
 *            index of the job whose mv_int is its t_field (-1: none).
 *  lines     host, cap entries: line i = chain << 16 | v << 8 | h, in order.
 *  *nlines   number of lines (also written when cap is too small, which
 *            returns ME_EINVAL).
 * Job validation and errors as me_texture_recursive.
 */
int me_search_schedule(const me_job *jobs, int n, int32_t *job_info, uint32_t *lines, int cap, int *nlines);

/* Wait for `stream`, then read and clear its device status word:
 * ME_OK, or ME_EDEVICE when a kernel reported a fault condition. */
int me_device_status(void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ME_H */

/*
 * hsgd.h -- C ABI of the MI355X (gfx950) HSGD library, libhsgd.so.
 *
 * Hierarchical Sparse Gradient Descent (RealLiFe, arXiv 2307.03017, Sec. 3.3) refines a
 * multi-plane image (MPI, Sec. 3.1) against N posed source views. One iteration:
 *   select  -- per reference pixel, keep the k planes with the largest compositing weight
 *              A_z = a_z prod_{j<z}(1 - a_j) of the un-warped MPI (Eq. gradient, Eq. overA;
 *              "Gradient Sparsification");
 *   render  -- warp every plane into each view with the plane homography (Eq. homo) and
 *              composite with the over operator (Eq. render, Eq. over);
 *   grad    -- photometric loss against the views and its exact gradient, pushed back
 *              through compositing and the bilinear warp, kept only on the selected voxels;
 *   update  -- analytic descent (Eq. 4; the sparsity prior of Sec. 3.4 optional, weight
 *              lambda_s) restored onto the selected voxels (the M_{n+1} = M_n + R(., S)
 *              update), clamped to [0, 1].
 * Levels run coarse to fine (Sec. 3.2: H/2^l x W/2^l), the MPI upsampled 2x in between.
 * Also exported: the hierarchical plane-sweep volume (Sec. 3.2) and a continuous-batching
 * serving core. tests/hsgd_c_smoke.c shows the calls used from plain C.
 *
 * Conventions for every call:
 *  - Layouts. MPI: [D][H][W][4] straight (non-premultiplied) RGBA in [0, 1], plane z = 0 the
 *    nearest (the paper's d = D - z), FP32 or BF16 storage. Images: [N][H][W][3] FP32.
 *    Views and the MPI share one H x W grid per level; pixel centres sit at integer
 *    coordinates.
 *  - Ownership. Every pointer passed in is CALLER-OWNED; the library never allocates,
 *    frees or retains device memory. Pointers documented as "device" must be device
 *    memory of the current HIP device; "host" pointers are ordinary host memory.
 *    Scratch memory comes in through (ws, ws_bytes); size it with hsgd_workspace_bytes().
 *  - Streams. Device work is enqueued on the given stream (NULL = the legacy default
 *    stream) and the call returns before it runs. Calls on one workspace must not overlap.
 *  - Errors. Arguments are validated before anything is enqueued; a failing call enqueues
 *    nothing and leaves every output untouched, returns a negative hsgd_status and sets a
 *    thread-local message (hsgd_last_error). A failed kernel launch returns HSGD_E_HIP.
 *    Faults during execution surface at the caller's next stream synchronisation.
 *  - Limits: 1 <= D <= 64, H, W >= 2, 1 <= N <= 64, 1 <= k <= D.
 */
#ifndef HSGD_H
#define HSGD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HSGD_OK = 0,
    HSGD_E_ARG = -1,        /* null pointer, bad scalar (k, tau, lr, level count ...) */
    HSGD_E_SHAPE = -2,      /* inconsistent or out-of-range sizes                      */
    HSGD_E_DTYPE = -3,      /* unknown storage type                                    */
    HSGD_E_CAPACITY = -4,   /* output array too small (ids capacity)                   */
    HSGD_E_WORKSPACE = -5,  /* ws missing or smaller than hsgd_workspace_bytes()       */
    HSGD_E_HIP = -6,        /* a HIP runtime call or kernel launch failed              */
    HSGD_E_BUDGET = -7      /* admission would exceed the serving batch's HBM budget   */
} hsgd_status;

typedef enum { HSGD_FP32 = 0, HSGD_BF16 = 1 } hsgd_dtype;

/* Per (view, plane) pixel map, 96 bytes. From hsgd_build_warps: view pixel (x, y, 1) ->
 * reference pixel on that plane, the inverse of the plane homography H_i^{-1}(d_z) of
 * Eq. (homo) (the direction rendering gathers in). From hsgd_build_psv_warps: reference
 * pixel -> view pixel, H_i^{-1}(d_z) itself (the plane-sweep direction).
 *  G        row-major 3x3 FP64 map, divided by |G[8]|: positions are unchanged and the
 *           sign of the homogeneous coordinate is kept (a point with q2 <= 0 is behind
 *           the camera and samples as transparent / 0). The kernels evaluate positions
 *           from it in FP64 and round only the bilinear fractions to FP32;
 *  is_shift 1 when the map is a pure translation (identity rotation, no z translation,
 *           equal intrinsics). Then the mapped position is (x + ix + fx, y + iy + fy)
 *           exactly: ix, iy integers, fx, fy in [0, 1) rounded once from FP64. */
typedef struct {
    double G[9];
    int32_t is_shift;
    int32_t ix, iy;
    float fx, fy;
    int32_t pad;
} hsgd_warp;

/* An MPI level. rgba: device, [D][H][W][4] of float (HSGD_FP32) or bfloat16 (HSGD_BF16). */
typedef struct {
    void* rgba;
    int32_t D, H, W;
    int32_t dtype;
} hsgd_mpi;

/* N source views at one level. images: device [N][H][W][3] FP32 targets (may be NULL
 * where documented); warps: device [N][D] hsgd_warp (from hsgd_build_warps).
 * flags: HSGD_VIEWS_SHIFT_ONLY when every warp record has is_shift = 1 (check the host
 * copy with hsgd_warps_shift_only); the gradient then takes the deterministic
 * translation path. Setting it for records that are not shifts gives wrong results. */
#define HSGD_VIEWS_SHIFT_ONLY 1
typedef struct {
    const float* images;
    const hsgd_warp* warps;
    int32_t N, H, W;
    int32_t flags;
} hsgd_views;

/* Sparsification rule (Sec. 3.3 "Gradient Sparsification"), on the scores A_z of the
 * un-warped MPI. k: planes kept per pixel (1..D).
 *  rule HSGD_SELECT_TOPK (0, the paper's rule): the k largest A_z, equal scores to the
 *       nearer plane;
 *  rule HSGD_SELECT_MVS (1, the MVS-sampling alternative the paper ablates): the plane with
 *       the largest A_z (equal scores: the nearer) and its neighbours, (k - 1)/2 planes
 *       nearer (rounded down) and the rest farther; a window that would leave [0, D) is
 *       moved inside it, so k planes are always kept.
 * tau < 0: nothing more; tau >= 0 additionally drops kept planes whose A_z <= tau. */
enum { HSGD_SELECT_TOPK = 0, HSGD_SELECT_MVS = 1 };
typedef struct {
    int32_t k;
    float tau;
    int32_t rule;
} hsgd_select_params;

/* Operation codes for hsgd_workspace_bytes. */
enum { HSGD_OP_SELECT = 0, HSGD_OP_RENDER = 1, HSGD_OP_GRAD_STEP = 2, HSGD_OP_REFINE = 3 };

/* Human-readable name of a status code (static string). */
const char* hsgd_status_string(int32_t status);

/* Detail of the last failing call on this thread ("" if none). */
const char* hsgd_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t hsgd_version(void);

/*
 * hsgd_build_warps -- host, FP64 (Sec. 3.2, Eq. homo).
 * Computes, for view i and plane z at depth depth[z] (plane n^T X = d, n = (0,0,1), in the
 * reference camera frame), H = K_i R_i (I + R_i^{-1} t_i n^T / d) K_ref^{-1} (the reference
 * pose is the identity: world = reference camera frame; poses map world to camera,
 * x_cam = R x_world + t) and stores its inverse in out[i*D + z].
 *  K_ref host [9]; K, R host [N][9] row-major; t host [N][3]; depth host [D] (> 0);
 *  out host [N*D]. No device memory is touched; copy out to the device yourself.
 * Errors: HSGD_E_ARG for null pointers, non-positive depths or a singular map;
 *         HSGD_E_SHAPE for N or D out of range.
 */
hsgd_status hsgd_build_warps(const double* K_ref, const double* K, const double* R,
                             const double* t, const double* depth, int32_t N, int32_t D,
                             hsgd_warp* out);

/*
 * hsgd_build_psv_warps -- host, FP64 (Sec. 3.2, Eq. homo): the plane-sweep direction.
 * out[i*D + z] holds H_i^{-1}(d_z) itself, the map from a reference pixel on plane z to
 * source view i (hsgd_build_warps stores its inverse), normalised by |G[8]| and split into
 * an exact integer + fraction translation when it is one, as hsgd_build_warps does.
 * Arguments, ownership and errors as for hsgd_build_warps.
 */
hsgd_status hsgd_build_psv_warps(const double* K_ref, const double* K, const double* R,
                                 const double* t, const double* depth, int32_t N, int32_t D,
                                 hsgd_warp* out);

/* hsgd_warps_shift_only -- host. 1 if all n records (host memory) are pure translations,
 * else 0 (also for NULL or n < 1): the value for hsgd_views.flags. */
int32_t hsgd_warps_shift_only(const hsgd_warp* warps, int32_t n);

/*
 * hsgd_level_intrinsics -- host. Intrinsics of a W x H camera resampled to Wl x Hl in
 * pixel-index coordinates (focal lengths scale by Wl/W, Hl/H; a principal point c maps to
 * (c + 0.5) s - 0.5), the camera of hierarchy level l (Sec. 3.2). K, out: host [9].
 */
hsgd_status hsgd_level_intrinsics(const double* K, int32_t W, int32_t H, int32_t Wl,
                                  int32_t Hl, double* out);

/*
 * hsgd_workspace_bytes -- bytes of workspace needed by one call of `op` on an MPI of
 * D x H x W with N views and k planes kept per pixel. For HSGD_OP_REFINE give the finest
 * level's H, W and the number of levels L (ignored otherwise). Returns 0 on bad sizes.
 */
size_t hsgd_workspace_bytes(int32_t op, int32_t D, int32_t H, int32_t W, int32_t N,
                            int32_t k, int32_t L);

/*
 * hsgd_select_active -- the sparse index set S (Sec. 3.3 "Gradient Sparsification";
 * Fig. sparse (b)).
 * For every reference pixel p, computes the scores of the un-warped MPI front to back in
 * IEEE float32, exactly A_z = a_z * T_z, T_{z+1} = T_z * (1 - a_z), T_0 = 1 (no fused
 * multiply-add, denormals kept; BF16 alpha is decoded exactly), and keeps the k planes
 * with the largest A_z; equal scores go to the nearer (smaller z) plane; NaN scores rank
 * last. With p.tau >= 0, kept planes with A_z <= tau are dropped.
 *  mask      device [H][W] uint64: bit z set <=> voxel (z, p) in S.
 *  ids       device [cap] int32 or NULL: S as ascending linear ids z*H*W + y*W + x
 *            (plane-major, the original depth order kept). cap >= k*H*W required.
 *  plane_off device [D+1] int32 or NULL: ids of plane z are ids[plane_off[z] ..
 *            plane_off[z+1]).
 *  n_active  device [1] int32 or NULL: |S|.
 * ids, plane_off and n_active are all NULL or all non-NULL.
 */
hsgd_status hsgd_select_active(const hsgd_mpi* m, hsgd_select_params p, uint64_t* mask,
                               int32_t* ids, int32_t cap, int32_t* plane_off,
                               int32_t* n_active, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/*
 * hsgd_render -- novel/source view rendering I~_t = O(w_t(M)) (Eq. render, Eq. over).
 * For every view pixel, each plane is sampled at the warped position with bilinear
 * interpolation (zero outside the plane; colour and alpha interpolated separately) and
 * composited front to back over a black background.
 *  out_rgb  device [N][H][W][3] FP32 or NULL.
 *  out_loss device [1] FP32 or NULL: L = 1/(2N) sum_i sum_p sum_ch (C - I)^2 against
 *           v->images (which must then be non-NULL).
 */
hsgd_status hsgd_render(const hsgd_mpi* m, const hsgd_views* v, float* out_rgb,
                        float* out_loss, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * hsgd_grad_step -- one sparse gradient step (Sec. 3.3 "Sparse Gradient Update" with the
 * analytic update of Eq. 4).
 * Computes g = dL/dM, the exact gradient of the dense rendering of all views, where
 * dL/dI~ is (I~ - I)/N for the photometric loss (dimg == NULL; v->images required) or the
 * given upstream gradient dimg (device [N][H][W][3], a vector-Jacobian product), through
 * the over operator (colour weight a~_z T_z, alpha weight T_z <g, c~_z - B_z> with B_z the
 * composite behind plane z from a back-to-front scan) and the transpose of the bilinear
 * warp. Only voxels of S are kept:
 *  mask  device [H][W] uint64 from hsgd_select_active, or NULL for every voxel (dense).
 *  kcap  most bits set in any mask word (the k given to hsgd_select_active; D when
 *        mask == NULL). Planes of a pixel beyond its first kcap set bits are treated as
 *        not selected.
 *  lambda_s  weight of the sparsity prior (Sec. 3.4, L_s = mean over the level's voxels of
 *        log(1.5 - |0.5 - alpha|), the prior phi of Eq. 4); 0 = none. When non-zero, its
 *        alpha gradient lambda_s sign(0.5 - alpha) / ((1.5 - |0.5 - alpha|) D H W) (0 at
 *        alpha = 0.5) is added to g on S. out_loss stays the data term.
 * Then, if lr_rgb or lr_alpha is non-zero, M[S] <- clamp(M[S] - (lr_rgb x3, lr_alpha) g,
 * 0, 1) in place (BF16 storage: round to nearest even on store); voxels outside S are
 * never written.
 *  grad_out device [D][H][W][4] FP32 or NULL: g on S, 0 elsewhere (every entry written).
 *  out_loss device [1] FP32 or NULL: the loss before the update (needs v->images).
 */
hsgd_status hsgd_grad_step(hsgd_mpi* m, const hsgd_views* v, const uint64_t* mask,
                           int32_t kcap, const float* dimg, float lr_rgb, float lr_alpha,
                           float lambda_s, float* grad_out, float* out_loss, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/*
 * hsgd_upsample2x -- MPI level transition (Sec. 3.3: refine the upsampled MPI).
 * fine = 2x bilinear upsampling of coarse per plane and channel, source coordinate
 * (x + 0.5)/2 - 0.5 clamped to the edge. fine must be 2H x 2W with the same D and dtype.
 */
hsgd_status hsgd_upsample2x(const hsgd_mpi* coarse, hsgd_mpi* fine, hipStream_t stream);

/*
 * hsgd_downsample2x -- one level of the image pyramid (Sec. 3.2: H/2^l x W/2^l):
 * out[n][y][x] = mean of the 2x2 block of images at (2y, 2x). images device
 * [N][H][W][3] FP32 (H, W even), out device [N][H/2][W/2][3].
 */
hsgd_status hsgd_downsample2x(const float* images, int32_t N, int32_t H, int32_t W,
                              float* out, hipStream_t stream);

/*
 * hsgd_plane_sweep -- the hierarchical plane-sweep volume (Sec. 3.2, Hierarchical PSV
 * Construction): level 0 is P[i][z][y][x] = bilinear sample of source image i at
 * H_i^{-1}(d_z) (x, y, 1) (pixel-index coordinates, zero padding outside the image, 0 where
 * the point is behind view i), for every view i, plane z and reference pixel (x, y) of an
 * H x W reference grid; level l (1 <= l < L) is the 2x2 box mean of level l - 1
 * (H/2^l x W/2^l). All levels come from one pass over the images: no level is re-read.
 *  src    images: device [N][H][W][3] FP32 source images (required); warps: device [N][D]
 *         records from hsgd_build_psv_warps for an H x W reference camera; flags
 *         HSGD_VIEWS_SHIFT_ONLY as for the other calls (translation path).
 *  D      planes, 1..64; L levels, 1..5; H and W multiples of 2^(L-1).
 *  out_dtype  HSGD_FP32 or HSGD_BF16 (every level computed in FP32 from the FP32 level
 *         above, rounded to nearest even once, on store).
 *  out    host array of L device pointers, 16-byte aligned: out[l] receives
 *         [N][D][H>>l][W>>l][3] of out_dtype; a NULL entry skips storing that level (at
 *         least one must be set). Caller owns all buffers; no workspace.
 * Errors: HSGD_E_ARG (NULL images/warps/out, every out[l] NULL, misaligned out),
 *         HSGD_E_SHAPE (N, D, L, H, W out of range), HSGD_E_DTYPE (unknown out_dtype),
 *         HSGD_E_HIP (launch failure).
 */
hsgd_status hsgd_plane_sweep(const hsgd_views* src, int32_t D, int32_t L, int32_t out_dtype,
                             void* const* out, hipStream_t stream);

/*
 * hsgd_refine -- the whole coarse-to-fine HSGD refinement (Sec. 3.3; Fig. pipeline).
 *  levels  [L] MPI descriptors, coarsest first; levels[0].rgba holds the initial MPI and
 *          is refined in place; levels[l] for l > 0 (2x the size of level l-1, same D and
 *          dtype) is overwritten with the upsampled MPI and refined in place. The result
 *          is levels[L-1].
 *  views   [L] per-level views: warps built with that level's intrinsics; images of the
 *          finest level required; images of a coarser level may be NULL, in which case
 *          they are computed as 2x2 box means of the next finer level into the workspace.
 *  iters   host [L] iterations per level (>= 0).
 *  sel     sparsification rule (k, tau, rule) used at every iteration.
 *  lr_rgb, lr_alpha, lambda_s  as in hsgd_grad_step, at every iteration.
 *  loss_log device [sum(iters)] FP32 or NULL: loss of each iteration before its update.
 */
hsgd_status hsgd_refine(hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                        const int32_t* iters, hsgd_select_params sel, float lr_rgb,
                        float lr_alpha, float lambda_s, float* loss_log, void* ws,
                        size_t ws_bytes, hipStream_t stream);

/*
 * hsgd_refine_noalloc -- hsgd_refine for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments and results without ws / ws_bytes. Its workspace is a static device array of
 * HSGD_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends; the call itself allocates and frees nothing (while hsgd_profile_* timing
 * is off). The refine's workspace (hsgd_workspace_bytes(HSGD_OP_REFINE, ...)) must fit in
 * it: 512x384 with 32 planes, 4 views and k = 4 needs 52.3 MiB and fits; larger calls
 * fail with HSGD_E_WORKSPACE and enqueue nothing. The array is looked up once per device
 * (with that device current) on the first call whose stream is on it. Every call on one
 * GPU uses that GPU's one array: calls that overlap on a GPU (on different streams, or
 * from several threads) race and corrupt each other's results; calls ordered on one
 * stream are safe. Nothing in the array needs to start at zero (the kernels write every
 * workspace value they read first, or clear it with a fill kernel).
 */
#define HSGD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hsgd_status hsgd_refine_noalloc(hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                                const int32_t* iters, hsgd_select_params sel, float lr_rgb,
                                float lr_alpha, float lambda_s, float* loss_log, hipStream_t stream);

/*
 * hsgd_convert -- storage conversion of n floats: FP32 -> BF16 (round to nearest even),
 * BF16 -> FP32 (exact) or a plain copy for equal types. src, dst device.
 */
hsgd_status hsgd_convert(const void* src, int32_t src_dtype, void* dst, int32_t dst_dtype,
                         size_t n, hipStream_t stream);

/*
 * Serving: continuous batching of refinements. A request is one frame of a persistent
 * stream (scene): its views and the initial MPI at the coarsest level, refined coarse to
 * fine exactly as hsgd_refine does. Requests that arrive while others are in flight are
 * admitted as slots and HBM budget allow; each hsgd_batch_step runs ONE iteration of
 * every request in flight, all of them in the same fixed sequence of persistent kernels
 * captured once in a HIP graph (the work of each request is a range of work items in a
 * device table rebuilt per step). A request's result is bitwise the result of hsgd_refine
 * on the same inputs: the per-request arithmetic and its order are the same.
 *
 * Streams keep their buffers: the caller allocates, per stream, the MPI of every level
 * and the images of every level (the finest holds the frame's targets, the coarser ones
 * receive the pyramid) once and passes the same pointers with every frame; the result of
 * a frame stays in levels[L-1] until the stream's next frame is admitted. The budget
 * counts the batch workspace plus the resident bytes of every stream seen since it was
 * last released (MPI levels, images, warps).
 */
typedef struct hsgd_batch hsgd_batch;      /* opaque */

#define HSGD_MAX_BATCH_LEVELS 4

typedef struct {
    int32_t max_slots;        /* requests in flight at once, 1..16                        */
    int32_t max_D;            /* largest plane count, <= 64                               */
    int32_t max_N;            /* most views of a request, <= 64                           */
    int32_t max_H, max_W;     /* largest finest-level frame                               */
    int32_t max_k;            /* largest k of a request's selection                       */
    int32_t dtype;            /* hsgd_dtype of every request's MPI                        */
    int32_t pad_;
    int64_t hbm_budget;       /* bytes: workspace + resident stream buffers               */
} hsgd_batch_config;

typedef struct {
    int32_t stream_id;                        /* >= 0                                      */
    int32_t L;                                /* levels, 1..HSGD_MAX_BATCH_LEVELS          */
    hsgd_mpi levels[HSGD_MAX_BATCH_LEVELS];   /* coarsest first, each 2x the previous;     */
                                              /* levels[0] holds the frame's initial MPI  */
    hsgd_views views[HSGD_MAX_BATCH_LEVELS];  /* per level, shift-only warps (flag set);   */
                                              /* images non-NULL at every level           */
    int32_t iters[HSGD_MAX_BATCH_LEVELS];     /* >= 1, except level 0 which may be 0       */
    hsgd_select_params sel;
    float lr_rgb, lr_alpha;
    float lambda_s;                           /* sparsity prior weight, as in grad_step    */
    float* loss_log;                          /* device [sum(iters)] FP32 or NULL          */
} hsgd_request;

/* Device workspace for hsgd_batch_create (0 for an invalid configuration). */
size_t hsgd_batch_workspace_bytes(const hsgd_batch_config* cfg);

/* Creates a batch on the current device. ws is device memory of at least
 * hsgd_batch_workspace_bytes(cfg) bytes, owned by the caller and kept until
 * hsgd_batch_destroy. The library allocates only host-side state, two small pinned
 * staging buffers, events and (at the first step) the instantiated graph.
 * HSGD_E_BUDGET if the workspace alone exceeds cfg->hbm_budget. */
hsgd_status hsgd_batch_create(const hsgd_batch_config* cfg, void* ws, size_t ws_bytes,
                              hsgd_batch** out);
/* Waits for the batch's device work, then frees its host-side state. */
hsgd_status hsgd_batch_destroy(hsgd_batch* b);

/* Admits a request; *ticket identifies it. HSGD_E_CAPACITY: every slot is busy, or the
 * stream's previous frame has iterations not yet stepped. HSGD_E_BUDGET: the stream is
 * new and its resident bytes do not fit the remaining budget. Shapes are checked against
 * the configuration (HSGD_E_SHAPE). Nothing runs until the next hsgd_batch_step. */
hsgd_status hsgd_batch_admit(hsgd_batch* b, const hsgd_request* r, int64_t* ticket);

/* Enqueues one iteration of every admitted request on stream (one table upload, one
 * graph launch). Blocks the host only while the step before the previous one still holds
 * its staging buffer. Steps run in the order they are enqueued whatever streams they are
 * given: a step enqueued on a stream other than the previous step's first makes that
 * stream wait for the previous step to complete (all steps share one device table, and
 * each continues the requests of the one before). Outputs (each may be NULL): *n_active requests stepped; the tickets
 * of requests whose last iteration this step holds, up to max_finished of them, and their
 * number *n_finished. With no request in flight it enqueues nothing. */
hsgd_status hsgd_batch_step(hsgd_batch* b, hipStream_t stream, int32_t* n_active,
                            int64_t* finished, int32_t max_finished, int32_t* n_finished);

/* Records the batch's time reference on stream and waits for it; completion times are
 * measured from it. */
hsgd_status hsgd_batch_reference(hsgd_batch* b, hipStream_t stream);

/* *done = 1 once the request's last iteration has completed on the device; then
 * *done_ms (nullable) is its completion time in ms after the reference (-1 without one). */
hsgd_status hsgd_batch_poll(hsgd_batch* b, int64_t ticket, int32_t* done, double* done_ms);

/* Forgets a stream (its resident bytes leave the budget). HSGD_E_CAPACITY while one of
 * its frames has iterations not yet stepped. */
hsgd_status hsgd_batch_release_stream(hsgd_batch* b, int32_t stream_id);

/* Bytes currently charged to the budget (workspace + resident streams). */
int64_t hsgd_batch_budget_used(const hsgd_batch* b);

/*
 * Kernel timing (tracing). Between hsgd_profile_begin and hsgd_profile_end, every launch
 * of a kernel kind whose bit is set in kind_mask is bracketed by two HIP events recorded
 * on the stream it is launched on. hsgd_profile_end waits for those events and adds up
 * the durations; hsgd_profile_read returns launches and total milliseconds of one kind.
 * One window at a time per process; not for use under stream capture.
 */
enum {
    HSGD_K_SELECT = 0, HSGD_K_SCAN = 1, HSGD_K_COMPACT = 2, HSGD_K_RENDER = 3,
    HSGD_K_GRAD = 4, HSGD_K_UPDATE = 5, HSGD_K_FILL = 6, HSGD_K_REDUCE = 7,
    HSGD_K_UPSAMPLE = 8, HSGD_K_DOWNSAMPLE = 9, HSGD_K_CONVERT = 10, HSGD_K_PSV = 11, HSGD_K_COUNT = 12
};
hsgd_status hsgd_profile_begin(uint32_t kind_mask);
hsgd_status hsgd_profile_end(void);
hsgd_status hsgd_profile_read(int32_t kind, int64_t* launches, double* total_ms);
/* Name of a kernel kind as it appears in profiler traces (static string, "" if unknown). */
const char* hsgd_kernel_name(int32_t kind);

#ifdef __cplusplus
}
#endif

#endif /* HSGD_H */

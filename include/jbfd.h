/*
 * jbfd.h - C ABI of the MI355X (gfx950) LiDAR depth-densification library.
 *
 * The library implements the data-parallel hot path of "Real-Time LiDAR
 * Point Cloud Densification for Low-Latency Spatial Data Transmission"
 * (arXiv 2601.01210):
 *
 *   1. jbfd_project  - the merged LiDAR points of a viewpoint become one
 *                      sparse depth image in its camera (Sec. 2), the
 *                      nearest point winning each pixel (z-buffer);
 *                      jbfd_project_recycled and jbfd_zbuf_clear do the same
 *                      for a frame loop that reuses its key buffer, and
 *                      jbfd_project_densify runs both steps below in one
 *                      call with the key decode fused into the list build
 *                      (jbfd_project_densify_noalloc: the same without a
 *                      caller workspace);
 *   2. jbfd_densify  - RGB-guided joint bilateral filter over that sparse
 *                      depth image (Eq. 1-4, organised as Algorithm 1),
 *                      giving a dense depth image and a validity mask;
 *   3. jbfd_densify_backward - gradients of a loss through the filter with
 *                      respect to the input depths and the two Gaussian
 *                      widths (Sec. 4: the filter parameters are trainable
 *                      by backpropagation);
 *   4. jbfd_batch_run - projection + filter for many viewpoints of mixed
 *                      size in one persistent launch that takes work items
 *                      of every view from a device queue (Sec. 2 processes
 *                      each viewpoint independently);
 *   5. jbfd_densify_two_stage (with jbfd_pool3, jbfd_restore_merge) - the
 *                      two-stage filter of Sec. 5: a pass at a third of the
 *                      resolution, then a small-radius pass at full size;
 *   6. jbfd_motion_mask, jbfd_project_motion - afterimage removal (Sec. 4.1):
 *                      older sweeps' points are dropped where the RGB frame
 *                      changed;
 *   7. jbfd_remove_occluded - occluded-point removal (Sec. 4.1);
 *   8. jbfd_backproject - contour removal and back-projection of the dense
 *                      depth to a coloured world point cloud (Sec. 5, Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every buffer pointer is a DEVICE pointer unless stated otherwise. The
 *   caller allocates and frees every buffer; the library never allocates
 *   device memory and keeps no mutable global state (the one exception is
 *   the fixed per-GPU array of jbfd_project_densify_noalloc), so calls on
 *   different streams may run concurrently from different host threads.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *   work is enqueued asynchronously on it; outputs are valid once the caller
 *   has synchronised the stream.
 * - Images are row-major, H rows by W columns; pixel (col,row) is at index
 *   row*W + col. RGB is interleaved 8-bit (3 bytes per pixel, R first).
 * - Argument errors are detected on the host before anything is enqueued
 *   and returned as JBFD_EINVAL; no output is touched then. Launch failures
 *   return JBFD_EHIP with a message in jbfd_last_error(). Faults inside a
 *   kernel surface at the caller's next synchronisation (HIP semantics).
 *   No C++ exception crosses this interface.
 * - Readings of what the paper leaves open (the same ones the CPU oracle
 *   uses): depth is camera-frame Z; pixel (col,row) covers u in [col,col+1),
 *   v in [row,row+1); the nearest point wins a pixel and an exact float tie
 *   goes to the smaller point index; the filter window is the full
 *   (2r+1)x(2r+1) square including its centre, clipped at the border;
 *   colour distance is the squared L2 norm of raw 0..255 RGB; an output
 *   pixel is valid iff its window holds at least one valid sample; invalid
 *   pixels hold depth 0.
 */
#ifndef JBFD_H
#define JBFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JBFD_ABI_VERSION 5

/* Largest filter radius: the halo of one 8x8 output block must fit the
 * per-workgroup spatial table in LDS. */
#define JBFD_MAX_RADIUS 32

/* Largest image width or height (pixel coordinates plus the halo travel as
 * packed 16-bit values inside the kernels). */
#define JBFD_MAX_SIDE 32767

/* Smallest accepted sigma (pixels for sigma_s, RGB units for sigma_r). Below
 * it the log2-domain weight exponent of a far sample would exceed the range
 * in which the FP32 kernels keep it exact. */
#define JBFD_MIN_SIGMA 0.25f

/* Enumerations cross the ABI as 32-bit ints. A caller may pass any int where
 * one is expected (an unknown value is rejected as JBFD_EINVAL, or named
 * "unknown status"); C++ gives the enumerations int as their underlying type
 * so that every int is a value of the type there as well. */
#ifdef __cplusplus
#define JBFD_ENUM_INT : int
#else
#define JBFD_ENUM_INT
#endif

typedef enum jbfd_status JBFD_ENUM_INT {
    JBFD_OK = 0,
    JBFD_EINVAL = 1,      /* bad argument (null pointer, size, radius, sigma) */
    JBFD_EUNSUPPORTED = 2, /* valid request this library does not implement */
    JBFD_EHIP = 3,        /* HIP runtime or launch error, see jbfd_last_error */
    JBFD_ENOSPC = 4       /* caller workspace smaller than the queried size */
} jbfd_status;

typedef enum jbfd_precision JBFD_ENUM_INT {
    JBFD_FP32 = 0,        /* weights, sums and divide in FP32 */
    JBFD_FP16_RANGE = 1   /* colour differences and range weights in FP16,
                             spatial weight, depth, sums, divide in FP32 */
} jbfd_precision;

/* Flags of jbfd_densify. */
#define JBFD_LISTS_READY 1u  /* ws already holds the sample lists of these
                                inputs (from jbfd_densify_prepare): skip
                                building them */
#define JBFD_DENSE 2u        /* inputs where most pixels hold a sample: one
                                thread per output pixel visits every tap of
                                its window (radius <= JBFD_DENSE_MAX_RADIUS,
                                FP32, no aux; ws is not used). Same weights
                                as the sparse kernels; the sums may differ
                                from theirs in the last bits (order). */
#define JBFD_DENSE_MAX_RADIUS 4

/* Pinhole intrinsics of a camera and the size of its image. */
typedef struct jbfd_intrinsics {
    double fx, fy;        /* focal lengths in pixels */
    double cx, cy;        /* principal point, pixel-edge convention
                             (a centred camera has cx = W/2) */
    int32_t width;        /* W, 1 .. JBFD_MAX_SIDE */
    int32_t height;       /* H, 1 .. JBFD_MAX_SIDE */
} jbfd_intrinsics;

/* Version of this interface (JBFD_ABI_VERSION of the built library). */
int jbfd_abi_version(void);

/* Static description of a status code; never NULL. */
const char *jbfd_status_string(jbfd_status s);

/* Message of the last error on the calling thread ("" if none). The pointer
 * stays valid until the next call into the library on this thread. */
const char *jbfd_last_error(void);

/*
 * Projection of merged LiDAR points into one camera and nearest-depth
 * z-buffer (Sec. 2: the combined sweeps of a viewpoint become one sparse
 * depth image in its camera; the collision rule is the reading stated
 * above).
 *
 * For each point i (its index in the merged array, sweeps concatenated in
 * order): (X,Y,Z) = R p + t in double precision, summed left to right with
 * no fused multiply-add; the point is dropped unless Z > 0 and finite;
 * u = fx*(X/Z) + cx, v = fy*(Y/Z) + cy; dropped unless 0 <= u < W and
 * 0 <= v < H; zf = (float)Z (round to nearest even), dropped if zf == 0 or
 * infinite; key = (bits(zf) << 32) | i competes for pixel (floor u, floor v)
 * and the smallest key wins (atomicMin on the 64-bit key).
 *
 * pts_xyz         n x 3 float32 world coordinates (device), any alignment
 *                 of 4 bytes; non-finite points are culled, not an error
 * n               number of points, 0 <= n < 2^32
 * cam_from_world  12 doubles, row-major 3x4 [R|t] (HOST memory, read during
 *                 the call); must be finite
 * K               intrinsics and image size (HOST memory); fx, fy, cx, cy
 *                 finite
 * zbuf            W*H uint64 workspace/output (device): the winning key per
 *                 pixel, UINT64_MAX where no point landed; cleared by this
 *                 call
 * sparse_depth    W*H float32 output (device): float Z of the winner, 0.0f
 *                 where empty; may be NULL
 * sparse_valid    W*H uint8 output (device): 1 where a point landed, else 0;
 *                 may be NULL
 */
jbfd_status jbfd_project(const float *pts_xyz, int64_t n,
                         const double cam_from_world[12],
                         const jbfd_intrinsics *K, uint64_t *zbuf,
                         float *sparse_depth, uint8_t *sparse_valid,
                         void *stream);

/*
 * jbfd_project for a frame loop that reuses its key buffer (same
 * projection, same sparse_depth and sparse_valid, bit for bit). zbuf must
 * hold the empty key UINT64_MAX in every pixel on entry: the state
 * jbfd_zbuf_clear and every call of this function leave it in (a buffer
 * fresh from jbfd_project holds the winning keys instead). The clearing
 * pass is skipped, and the decode writes the empty key back over each key
 * it reads that is not empty (the others are empty already), so the
 * buffer is touched once less per frame and the winning keys are not
 * returned. sparse_depth and sparse_valid are required (NULL
 * is JBFD_EINVAL); the other arguments are those of jbfd_project. Calls
 * that share a zbuf must be ordered (one stream, or synchronised).
 */
jbfd_status jbfd_project_recycled(const float *pts_xyz, int64_t n,
                                  const double cam_from_world[12],
                                  const jbfd_intrinsics *K, uint64_t *zbuf,
                                  float *sparse_depth, uint8_t *sparse_valid,
                                  void *stream);

/*
 * The whole path of one viewpoint (Sec. 2: projection of the merged sweeps
 * into the camera with a nearest-depth z-buffer; Sec. 4.2, Eq. 1-4 and
 * Algorithm 1: the joint bilateral filter): jbfd_project_recycled followed
 * by jbfd_densify with sample lists, in one call that fuses the decode of
 * the key image with the counting pass of the list build (the decode reads
 * each unit's halo keys itself, and the list scatter clears the keys once
 * the lists are written). Results are those of the two calls made
 * separately, bit for bit: sparse_depth / sparse_valid as
 * jbfd_project_recycled (required, device, W*H), dense_depth / dense_valid
 * as jbfd_densify with the same workspace (required, device, W*H; no aux).
 * zbuf holds only empty keys on entry and is left so (as for
 * jbfd_project_recycled). ws, ws_bytes: NULL/0, or a device workspace,
 * 256-byte aligned (else JBFD_EINVAL), as for jbfd_densify; when ws is NULL
 * or cannot hold the lists' tables (see jbfd_densify_ws_bytes), the call
 * projects with jbfd_project_recycled and the filter streams its inputs.
 * Other errors as jbfd_project and jbfd_densify; sizes come from K. The
 * caller owns every buffer; calls that share zbuf or ws must be ordered.
 */
jbfd_status jbfd_project_densify(const float *pts_xyz, int64_t n,
                                 const double cam_from_world[12],
                                 const jbfd_intrinsics *K, const uint8_t *rgb_hwc,
                                 int32_t radius, float sigma_s, float sigma_r,
                                 jbfd_precision prec, uint64_t *zbuf,
                                 float *sparse_depth, uint8_t *sparse_valid,
                                 float *dense_depth, uint8_t *dense_valid, void *ws,
                                 size_t ws_bytes, void *stream);

/*
 * jbfd_project_densify for callers that cannot allocate device memory or
 * hand over a workspace: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, results and errors as
 * jbfd_project_densify without ws / ws_bytes, bit for bit: the sample lists
 * are built in a fixed array of JBFD_NOALLOC_WS_BYTES bytes inside the
 * library (one per GPU, held from the first call on that GPU until the
 * process ends; the call never allocates). A call whose lists may need more,
 * jbfd_densify_ws_bytes(K->height, K->width, radius, n) > JBFD_NOALLOC_WS_BYTES
 * (n bounds the valid samples), returns JBFD_ENOSPC before anything is
 * enqueued. Every call on one GPU shares that GPU's array and leaves its
 * contents there; each call rewrites every table it reads, so nothing needs
 * clearing between calls, but calls that overlap on one GPU (different
 * streams or host threads without ordering) race on the array and must not
 * be issued. The device must be current (hipSetDevice) on the calling
 * thread, as for any launch on `stream`.
 */
#define JBFD_NOALLOC_WS_BYTES ((size_t)32 << 20)
jbfd_status jbfd_project_densify_noalloc(const float *pts_xyz, int64_t n,
                                         const double cam_from_world[12],
                                         const jbfd_intrinsics *K,
                                         const uint8_t *rgb_hwc, int32_t radius,
                                         float sigma_s, float sigma_r,
                                         jbfd_precision prec, uint64_t *zbuf,
                                         float *sparse_depth, uint8_t *sparse_valid,
                                         float *dense_depth, uint8_t *dense_valid,
                                         void *stream);

/* Set every key of an H x W key buffer (device) to the empty key
 * UINT64_MAX, for jbfd_project_recycled. */
jbfd_status jbfd_zbuf_clear(uint64_t *zbuf, int32_t H, int32_t W, void *stream);

/*
 * Joint bilateral filter over a sparse depth image (Eq. 1-4; the window and
 * step structure of Algorithm 1).
 *
 * For each pixel x, over the valid samples n (sparse_valid == 1) of the
 * (2r+1)x(2r+1) window around x, clipped to the image:
 *     w(x,n) = exp(-|I(x)-I(n)|^2 / (2 sigma_r^2)) * exp(-|x-n|^2 / (2 sigma_s^2))
 *     dense_depth(x) = sum w D(n) / sum w,   dense_valid(x) = 1
 * and dense_depth(x) = 0, dense_valid(x) = 0 when the window holds no valid
 * sample. sparse_depth is read only where sparse_valid == 1. The kernels
 * divide all weights of one output pixel by a common power of two that
 * keeps them in range; it cancels in the ratio.
 *
 * sparse_depth, sparse_valid  H*W float32 / uint8 (device)
 * rgb_hwc         H*W*3 uint8 guide image (device)
 * H, W            1 .. JBFD_MAX_SIDE each
 * radius          0 .. JBFD_MAX_RADIUS
 * sigma_s         spatial width in pixels, >= JBFD_MIN_SIGMA or +inf
 * sigma_r         colour width in RGB units, >= JBFD_MIN_SIGMA or +inf
 * prec            JBFD_FP32 or JBFD_FP16_RANGE
 * dense_depth     H*W float32 output (device)
 * dense_valid     H*W uint8 output (device)
 * aux             NULL, or H*W*2 float32 output (device) saved for
 *                 jbfd_densify_backward: per pixel the log2 shift its
 *                 weights were formed with and their weight sum (FP32
 *                 precision only; the backward recomputes the same weights)
 * ws, ws_bytes    NULL/0, or a device workspace (256-byte aligned). With at
 *                 least jbfd_densify_ws_bytes(H, W, radius, n) bytes, where
 *                 n bounds the number of valid samples (the number of
 *                 projected points is such a bound), the call first builds
 *                 per-strip sample lists and the filter reads them; with a
 *                 smaller or no workspace, if the image holds more valid
 *                 samples than the workspace can list, or if it has more
 *                 than 2^26 pixels, the filter streams the inputs directly. Both ways visit the samples in the
 *                 same (row-major) order; they may differ in the last bits
 *                 where a range rescale falls inside a group of samples.
 */
jbfd_status jbfd_densify(const float *sparse_depth, const uint8_t *sparse_valid,
                         const uint8_t *rgb_hwc, int32_t H, int32_t W,
                         int32_t radius, float sigma_s, float sigma_r,
                         jbfd_precision prec, float *dense_depth,
                         uint8_t *dense_valid, float *aux, void *ws,
                         size_t ws_bytes, uint32_t flags, void *stream);

/*
 * Build jbfd_densify's per-strip sample lists in ws (the first half of a
 * jbfd_densify call with a workspace). A following jbfd_densify (or
 * jbfd_densify_backward) on the same inputs, radius and workspace may pass
 * JBFD_LISTS_READY to reuse them. ws must not be NULL; a workspace smaller
 * than needed leaves lists the filter will not use (it streams instead).
 */
jbfd_status jbfd_densify_prepare(const float *sparse_depth,
                                 const uint8_t *sparse_valid,
                                 const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                 int32_t radius, void *ws, size_t ws_bytes,
                                 void *stream);

/* Workspace bytes for jbfd_densify's sample lists on an H x W image with
 * at most max_samples valid samples; 0 for invalid sizes. */
size_t jbfd_densify_ws_bytes(int32_t H, int32_t W, int32_t radius,
                             int64_t max_samples);

/*
 * Gradient of a scalar loss L through jbfd_densify (FP32 precision).
 *
 * With w_i the weights of the valid samples i in the window of x,
 * W(x) = sum w_i and out(x) = dense_depth(x):
 *     dL/dD_i      += g(x) w_i / W(x)
 *     dL/dsigma_r  += g(x) sum_i w_i c_i (D_i - out(x)) / (sigma_r^3 W(x))
 *     dL/dsigma_s  += g(x) sum_i w_i s_i (D_i - out(x)) / (sigma_s^3 W(x))
 * where c_i is the squared colour distance, s_i the squared pixel distance
 * and g = grad_out. Pixels with dense_valid == 0 contribute nothing.
 *
 * The forward inputs and parameters must be the ones of the jbfd_densify
 * call that produced dense_depth and aux.
 * grad_out        H*W float32 (device), dL/d dense_depth
 * grad_depth      H*W float32 output (device), dL/d sparse_depth (0 where
 *                 sparse_valid == 0); overwritten
 * grad_sigmas     2 doubles output (device): dL/dsigma_s, dL/dsigma_r;
 *                 overwritten; 0 for an infinite sigma
 * ws, ws_bytes    device workspace of at least
 *                 jbfd_densify_backward_ws_bytes(H, W) bytes; the sigma
 *                 reduction is deterministic (fixed order)
 */
jbfd_status jbfd_densify_backward(const float *sparse_depth,
                                  const uint8_t *sparse_valid,
                                  const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                  int32_t radius, float sigma_s, float sigma_r,
                                  const float *dense_depth, const float *aux,
                                  const float *grad_out, float *grad_depth,
                                  double *grad_sigmas, void *ws,
                                  size_t ws_bytes, void *stream);

/* Workspace bytes needed by jbfd_densify_backward for an H x W image; 0
 * when H or W is outside 1 .. JBFD_MAX_SIDE (such a call is rejected). */
size_t jbfd_densify_backward_ws_bytes(int32_t H, int32_t W);

/*
 * Batched projection + filter over many viewpoints of mixed image size,
 * point count and filter parameters (Sec. 2: each viewpoint is processed
 * on its own, with no exchange between viewpoints).
 *
 * Usage: jbfd_batch_prepare() validates the views on the host and writes a
 * device-side descriptor table into a HOST buffer of
 * jbfd_batch_table_bytes(n_views) bytes (pinned memory lets the copy be
 * asynchronous and captured); the caller copies it to device memory and
 * calls jbfd_batch_run() with that device pointer. By default
 * jbfd_batch_run is ONE persistent launch of a fixed grid that takes work
 * items from device queues in the table: every view's projection chunks,
 * then every view's key decode chunks, then every view's filter tiles, each
 * item waiting (bounded) only for the earlier items of its own view, so a
 * view is filtered while later views are still being decoded. With
 * JBFD_BATCH_STAGED (or JBFD_BATCH_LISTS) the run is instead a sequence of
 * fixed-grid launches (project, decode, with JBFD_BATCH_LISTS list count and
 * list scatter, filter), each covering every view. Either form needs each
 * view's key buffer to hold only empty keys (UINT64_MAX) on entry, and
 * leaves it so (the decode writes the empty key back over each key that is
 * not empty): clear a new buffer once with jbfd_zbuf_clear. Either way every
 * size is read from the table on the device,
 * so the launch(es) can be captured once into a HIP graph and replayed for
 * any batch written into the same device table, as long as every radius
 * stays <= the captured max_radius; the one-launch run leaves its queue
 * reset, so it may also be replayed on an unchanged table.
 *
 * Per view, the work is that of jbfd_project followed by jbfd_densify on
 * the same definitions (with sample lists when the run has
 * JBFD_BATCH_LISTS and the view brings a list workspace, else streaming the
 * halo); outputs are identical to the single-view calls made the same way.
 * Views must not share output, scratch or list buffers, and runs that share
 * a device table must be ordered (the table holds the run's queue).
 * A list workspace smaller than its tables (jbfd_densify_ws_bytes with no
 * samples) is JBFD_ENOSPC; a block whose list does not fit streams.
 */
typedef struct jbfd_view {
    const float *points;      /* n_points x 3 float32 world xyz (device) */
    int64_t n_points;         /* 0 <= n_points < 2^32 */
    double cam_from_world[12];/* row-major [R|t], finite */
    jbfd_intrinsics K;        /* camera and image size */
    const uint8_t *rgb;       /* H*W*3 guide image (device) */
    int32_t radius;           /* 0 .. JBFD_MAX_RADIUS */
    float sigma_s, sigma_r;   /* as jbfd_densify */
    uint64_t *zbuf;           /* H*W key buffer (device): only empty keys
                                 on entry, and again after every run */
    float *sparse_depth;      /* H*W scratch/output (device) */
    uint8_t *sparse_valid;    /* H*W scratch/output (device) */
    float *dense_depth;       /* H*W output (device) */
    uint8_t *dense_valid;     /* H*W output (device) */
    void *list_ws;            /* NULL, or a sample-list workspace for this
                                 view (device, 256-byte aligned, as for
                                 jbfd_densify; jbfd_densify_ws_bytes sizes
                                 it): the batch then builds the view's
                                 lists and its filter walks them */
    size_t list_ws_bytes;     /* bytes at list_ws */
} jbfd_view;

/* Bytes of the descriptor table for n_views views (0 if n_views < 1). */
size_t jbfd_batch_table_bytes(int32_t n_views);

/* Validate views[0..n_views) (HOST array) and write the descriptor table
 * into host_table (HOST memory of at least jbfd_batch_table_bytes bytes).
 * Nothing is enqueued. JBFD_EINVAL names the first bad view. */
jbfd_status jbfd_batch_prepare(const jbfd_view *views, int32_t n_views,
                               void *host_table, size_t table_bytes);

/* Run a batch whose table (from jbfd_batch_prepare) is at d_table (device,
 * 8-byte aligned, written by the run: it holds the one-launch queue and an
 * error word). max_radius bounds every view's radius (it selects the kernel
 * variant and the LDS size); a view with a larger radius gets zero depth
 * and mask and sets the error word that jbfd_batch_check reports. flags: 0
 * (one persistent launch, every view streams its halo), JBFD_BATCH_STAGED
 * (the same results from a sequence of launches), or JBFD_BATCH_LISTS
 * (launch sequence that builds the sample lists of the views that bring a
 * list workspace and walks them in the filter). Capturable in a HIP graph. */
#define JBFD_BATCH_LISTS 1u
#define JBFD_BATCH_STAGED 2u
jbfd_status jbfd_batch_run(void *d_table, int32_t max_radius, jbfd_precision prec,
                           uint32_t flags, void *stream);

/* After the runs on a table since its jbfd_batch_prepare have finished on
 * `stream`: JBFD_OK, or JBFD_EINVAL when a view's radius exceeded the run's
 * max_radius (that view's outputs are zeros), or JBFD_EHIP when a work item
 * of the one-launch run gave up waiting (the outputs are not valid). Copies
 * the table's error word to the host and synchronises `stream`; allocates
 * nothing. */
jbfd_status jbfd_batch_check(const void *d_table, void *stream);

/*
 * Two-stage filtering (Sec. 5: a first pass at a third of the resolution
 * in each dimension, reached by pooling, then a pass at full resolution on
 * the restored map; radius 4 then 2 in the paper). The paper names pooling
 * and restoring only; this library reads them as:
 *
 *   jbfd_pool3          3x3 cells; partial edge cells pool the pixels
 *                       inside the image. Pooled depth = mean of the cell's
 *                       valid depths (summed in double, row-major, rounded
 *                       once to float), pooled valid = the cell holds a
 *                       sample, pooled colour = floor((sum + n/2) / n) per
 *                       channel over the cell's n pixels. Output size
 *                       H1 = (H+2)/3, W1 = (W+2)/3.
 *   jbfd_restore_merge  nearest restore: pixel (x, y) takes cell (x/3, y/3);
 *                       the second pass sees the original depth where
 *                       sparse_valid = 1, else the first pass's depth where
 *                       its mask is 1, else nothing.
 *   jbfd_densify_two_stage
 *                       pool3 -> filter (radius1, sigmas1) at H1 x W1 ->
 *                       restore_merge -> filter (radius2, sigmas2) at H x W.
 *                       Each filter uses the dense kernel (JBFD_DENSE) when
 *                       its radius is <= JBFD_DENSE_MAX_RADIUS, else the
 *                       sparse kernel without lists. FP32.
 *
 * Buffers are device pointers; sizes and errors as jbfd_densify. The two-
 * stage call keeps its intermediates in ws (device, 256-byte aligned, at
 * least jbfd_two_stage_ws_bytes(H, W) bytes, else JBFD_ENOSPC).
 */
typedef struct jbfd_two_stage {
    int32_t radius1;          /* first pass, at (H+2)/3 x (W+2)/3 */
    float sigma_s1, sigma_r1; /* sigma_s1 in pooled pixels */
    int32_t radius2;          /* second pass, at H x W */
    float sigma_s2, sigma_r2;
} jbfd_two_stage;

jbfd_status jbfd_pool3(const float *sparse_depth, const uint8_t *sparse_valid,
                       const uint8_t *rgb_hwc, int32_t H, int32_t W,
                       float *depth1, uint8_t *valid1, uint8_t *rgb1,
                       void *stream);

jbfd_status jbfd_restore_merge(const float *sparse_depth,
                               const uint8_t *sparse_valid,
                               const float *depth1, const uint8_t *valid1,
                               int32_t H, int32_t W, float *depth2,
                               uint8_t *valid2, void *stream);

size_t jbfd_two_stage_ws_bytes(int32_t H, int32_t W);

jbfd_status jbfd_densify_two_stage(const float *sparse_depth,
                                   const uint8_t *sparse_valid,
                                   const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                   const jbfd_two_stage *params,
                                   float *dense_depth, uint8_t *dense_valid,
                                   void *ws, size_t ws_bytes, void *stream);

/*
 * Occluded-point removal (Sec. 4.1: the merged depth map is averaged and
 * samples lying well behind the average are dropped as surfaces the camera
 * cannot see). For each valid pixel, mean = the mean of the valid depths in
 * its (2k+1)^2 window (centre included, clipped at the border), summed in
 * double in row-major order; valid_out = 0 when D - mean > tau * mean (in
 * double), else valid_out = sparse_valid. The depth image is not changed.
 *
 * sparse_depth, sparse_valid  H*W (device); valid_out  H*W uint8 (device,
 * may not alias sparse_valid); k 0 .. JBFD_OCCLUSION_MAX_K; tau finite >= 0.
 */
#define JBFD_OCCLUSION_MAX_K 8
jbfd_status jbfd_remove_occluded(const float *sparse_depth,
                                 const uint8_t *sparse_valid, int32_t H,
                                 int32_t W, int32_t k, float tau,
                                 uint8_t *valid_out, void *stream);

/*
 * Contour removal and back-projection to a coloured cloud in the world
 * frame (Sec. 5: depths along object contours are removed by thresholding
 * the depth gradient; Sec. 2: each viewpoint's coloured points go to the
 * common world frame). A dense pixel is kept when dense_valid = 1 and its
 * largest |D(n) - D(x)| over valid 4-neighbours n (in double) is at most
 * tau * D(x) (tau = +inf keeps every valid pixel). A kept pixel (col, row)
 * becomes p_c = ((col + 0.5 - cx) Z / fx, (row + 0.5 - cy) Z / fy, Z) and
 * the world point R^T (p_c - t) for the camera-from-world pose [R|t], each
 * coordinate evaluated in double without contraction and rounded once to
 * float. Points are written in row-major pixel order.
 *
 * dense_depth, dense_valid, rgb_hwc  outputs of jbfd_densify (device)
 * cam_from_world, K                  host, finite, fx and fy nonzero
 * xyz        device float32, room for H*W*3 values
 * rgb_out    device uint8, room for H*W*3 values
 * count      device int64: the number of points written
 * ws         device, 256-byte aligned, jbfd_backproject_ws_bytes(H, W)
 *            bytes (else JBFD_ENOSPC)
 * H*W at most JBFD_BACKPROJECT_MAX_PIXELS (else JBFD_EINVAL; the write pass
 * sums the point counts of all earlier 1024-pixel chunks in every chunk, a
 * cost that grows with the square of the image size: about 1 ms at the
 * limit); jbfd_backproject_ws_bytes returns 0 beyond it.
 */
#define JBFD_BACKPROJECT_MAX_PIXELS (1 << 26)
size_t jbfd_backproject_ws_bytes(int32_t H, int32_t W);
jbfd_status jbfd_backproject(const float *dense_depth, const uint8_t *dense_valid,
                             const uint8_t *rgb_hwc, int32_t H, int32_t W,
                             const double cam_from_world[12],
                             const jbfd_intrinsics *K, float tau, float *xyz,
                             uint8_t *rgb_out, int64_t *count, void *ws,
                             size_t ws_bytes, void *stream);

/*
 * Afterimage removal (Sec. 4.1: moving regions are found from the colour
 * change between consecutive RGB frames, thresholded and closed
 * morphologically; there, LiDAR points not from the most recent frame are
 * discarded before the depth image is formed).
 *
 * jbfd_motion_mask: mask = closing of [squared RGB distance between rgb and
 * rgb_prev > tau^2] with a (2k+1)x(2k+1) square; the dilation treats
 * pixels outside the image as still and the erosion treats them as moving,
 * so the closing never removes motion at the border. rgb_hwc, rgb_prev_hwc:
 * device H x W x 3 uint8; mask: device H x W uint8 (1 = moving), written
 * in full. k 0 .. JBFD_MOTION_MAX_K; tau finite >= 0; else JBFD_EINVAL.
 * Needs no workspace.
 *
 * jbfd_project_motion: jbfd_project in which a point whose sweep id
 * (sweep_ids[i], device int8) differs from `latest` is dropped when its
 * pixel lies in `motion` (device, K->height x K->width); all else as
 * jbfd_project.
 */
#define JBFD_MOTION_MAX_K 16
jbfd_status jbfd_motion_mask(const uint8_t *rgb_hwc, const uint8_t *rgb_prev_hwc,
                             int32_t H, int32_t W, float tau, int32_t k,
                             uint8_t *mask, void *stream);
jbfd_status jbfd_project_motion(const float *pts_xyz, int64_t n,
                                const int8_t *sweep_ids, int8_t latest,
                                const uint8_t *motion,
                                const double cam_from_world[12],
                                const jbfd_intrinsics *K, uint64_t *zbuf,
                                float *sparse_depth, uint8_t *sparse_valid,
                                void *stream);

#ifdef __cplusplus
}
#endif

#endif /* JBFD_H */

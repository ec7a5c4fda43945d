// C ABI of libjbfd (declared in include/jbfd.h): argument validation on the
// host, then asynchronous launches on the caller's stream. No entry point
// allocates device memory; errors are returned as status codes with a
// thread-local message.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "filter_common.hpp"

namespace {

thread_local char g_err[512] = "";

jbfd_status fail(jbfd_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// Prepend "batch view v: " to the message a check just left.
jbfd_status prefix_error(jbfd_status s, int32_t v) {
    char inner[sizeof g_err];
    snprintf(inner, sizeof inner, "%s", g_err);
    return fail(s, "batch view %d: %s", v, inner);
}

jbfd_status ok() {
    g_err[0] = '\0';
    return JBFD_OK;
}

jbfd_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return ok();
    return fail(JBFD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool sigma_ok(float s) {
    if (isnan(s)) return false;
    if (isinf(s)) return s > 0;
    return s >= JBFD_MIN_SIGMA;
}

// log2(e) / (2 sigma^2), 0 for an infinite sigma
float log2_half_inv_var(float sigma) {
    if (isinf(sigma)) return 0.0f;
    const double s = (double)sigma;
    return (float)(1.4426950408889634 / (2.0 * s * s));
}

jbfd_status check_image(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0 || H > JBFD_MAX_SIDE || W > JBFD_MAX_SIDE)
        return fail(JBFD_EINVAL, "image size %d x %d outside 1..%d", H, W,
                    JBFD_MAX_SIDE);
    return JBFD_OK;
}

jbfd_status check_filter(int32_t radius, float ss, float sr) {
    if (radius < 0 || radius > JBFD_MAX_RADIUS)
        return fail(JBFD_EINVAL, "radius %d outside 0..%d", radius,
                    JBFD_MAX_RADIUS);
    if (!sigma_ok(ss))
        return fail(JBFD_EINVAL, "sigma_s %g must be >= %g or +inf", (double)ss,
                    (double)JBFD_MIN_SIGMA);
    if (!sigma_ok(sr))
        return fail(JBFD_EINVAL, "sigma_r %g must be >= %g or +inf", (double)sr,
                    (double)JBFD_MIN_SIGMA);
    return JBFD_OK;
}

}  // namespace

extern "C" {

int jbfd_abi_version(void) { return JBFD_ABI_VERSION; }

const char *jbfd_status_string(jbfd_status s) {
    switch (s) {
    case JBFD_OK: return "ok";
    case JBFD_EINVAL: return "invalid argument";
    case JBFD_EUNSUPPORTED: return "unsupported";
    case JBFD_EHIP: return "HIP runtime error";
    case JBFD_ENOSPC: return "workspace too small";
    }
    return "unknown status";
}

const char *jbfd_last_error(void) { return g_err; }

// argument checks shared by the projection entry points
static jbfd_status check_project(const char *name, const float *pts_xyz, int64_t n,
                                 const double cam_from_world[12],
                                 const jbfd_intrinsics *K, const uint64_t *zbuf) {
    if (!cam_from_world || !K || !zbuf)
        return fail(JBFD_EINVAL, "%s: null pose, intrinsics or zbuf", name);
    if (n < 0 || n >= ((int64_t)1 << 32))
        return fail(JBFD_EINVAL, "%s: n = %lld outside 0..2^32-1", name, (long long)n);
    if (n > 0 && !pts_xyz) return fail(JBFD_EINVAL, "%s: null points", name);
    jbfd_status st = check_image(K->height, K->width);
    if (st != JBFD_OK) return st;
    for (int t = 0; t < 12; ++t)
        if (!isfinite(cam_from_world[t]))
            return fail(JBFD_EINVAL, "%s: pose entry %d not finite", name, t);
    if (!isfinite(K->fx) || !isfinite(K->fy) || !isfinite(K->cx) || !isfinite(K->cy))
        return fail(JBFD_EINVAL, "%s: intrinsics not finite", name);
    return JBFD_OK;
}

static jbfd_status project_common(const char *name, const float *pts_xyz, int64_t n,
                                  const double cam_from_world[12],
                                  const jbfd_intrinsics *K, uint64_t *zbuf,
                                  float *sparse_depth, uint8_t *sparse_valid,
                                  bool recycle, void *stream) {
    const jbfd_status st = check_project(name, pts_xyz, n, cam_from_world, K, zbuf);
    if (st != JBFD_OK) return st;
    jbfd::Pose P;
    for (int t = 0; t < 12; ++t) P.m[t] = cam_from_world[t];
    jbfd::Intr I{K->fx, K->fy, K->cx, K->cy, K->width, K->height};
    return hip_status(jbfd::launch_project(pts_xyz, n, P, I, zbuf, sparse_depth,
                                           sparse_valid, recycle, (hipStream_t)stream),
                      name);
}

jbfd_status jbfd_project(const float *pts_xyz, int64_t n,
                         const double cam_from_world[12],
                         const jbfd_intrinsics *K, uint64_t *zbuf,
                         float *sparse_depth, uint8_t *sparse_valid,
                         void *stream) {
    return project_common("jbfd_project", pts_xyz, n, cam_from_world, K, zbuf,
                          sparse_depth, sparse_valid, false, stream);
}

jbfd_status jbfd_project_recycled(const float *pts_xyz, int64_t n,
                                  const double cam_from_world[12],
                                  const jbfd_intrinsics *K, uint64_t *zbuf,
                                  float *sparse_depth, uint8_t *sparse_valid,
                                  void *stream) {
    if (!sparse_depth || !sparse_valid)
        return fail(JBFD_EINVAL, "jbfd_project_recycled: null sparse_depth or sparse_valid");
    return project_common("jbfd_project_recycled", pts_xyz, n, cam_from_world, K,
                          zbuf, sparse_depth, sparse_valid, true, stream);
}

// argument checks shared by the one-call projection + filter entry points
static jbfd_status check_project_densify(const char *name, const float *pts_xyz,
                                         int64_t n, const double cam_from_world[12],
                                         const jbfd_intrinsics *K,
                                         const uint8_t *rgb_hwc, int32_t radius,
                                         float sigma_s, float sigma_r,
                                         jbfd_precision prec, const uint64_t *zbuf,
                                         const float *sparse_depth,
                                         const uint8_t *sparse_valid,
                                         const float *dense_depth,
                                         const uint8_t *dense_valid) {
    jbfd_status st = check_project(name, pts_xyz, n, cam_from_world, K, zbuf);
    if (st != JBFD_OK) return st;
    if (!rgb_hwc || !sparse_depth || !sparse_valid || !dense_depth || !dense_valid)
        return fail(JBFD_EINVAL, "%s: null buffer", name);
    st = check_filter(radius, sigma_s, sigma_r);
    if (st != JBFD_OK) return st;
    if (prec != JBFD_FP32 && prec != JBFD_FP16_RANGE)
        return fail(JBFD_EINVAL, "%s: unknown precision %d", name, (int)prec);
    return JBFD_OK;
}

static jbfd_status run_project_densify(const char *name, const float *pts_xyz,
                                       int64_t n, const double cam_from_world[12],
                                       const jbfd_intrinsics *K,
                                       const uint8_t *rgb_hwc, int32_t radius,
                                       float sigma_s, float sigma_r,
                                       jbfd_precision prec, uint64_t *zbuf,
                                       float *sparse_depth, uint8_t *sparse_valid,
                                       float *dense_depth, uint8_t *dense_valid,
                                       void *ws, size_t ws_bytes, void *stream) {
    jbfd::Pose P;
    for (int t = 0; t < 12; ++t) P.m[t] = cam_from_world[t];
    jbfd::Intr I{K->fx, K->fy, K->cx, K->cy, K->width, K->height};
    jbfd::FilterParams fp{radius, log2_half_inv_var(sigma_r), log2_half_inv_var(sigma_s)};
    const hipError_t e = jbfd::launch_project_densify(
        pts_xyz, n, P, I, rgb_hwc, fp, prec, zbuf, sparse_depth, sparse_valid,
        dense_depth, dense_valid, ws, ws_bytes, (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(JBFD_EUNSUPPORTED, "%s: precision not built", name);
    return hip_status(e, name);
}

jbfd_status jbfd_project_densify(const float *pts_xyz, int64_t n,
                                 const double cam_from_world[12],
                                 const jbfd_intrinsics *K, const uint8_t *rgb_hwc,
                                 int32_t radius, float sigma_s, float sigma_r,
                                 jbfd_precision prec, uint64_t *zbuf,
                                 float *sparse_depth, uint8_t *sparse_valid,
                                 float *dense_depth, uint8_t *dense_valid, void *ws,
                                 size_t ws_bytes, void *stream) {
    const char *name = "jbfd_project_densify";
    const jbfd_status st = check_project_densify(
        name, pts_xyz, n, cam_from_world, K, rgb_hwc, radius, sigma_s, sigma_r, prec,
        zbuf, sparse_depth, sparse_valid, dense_depth, dense_valid);
    if (st != JBFD_OK) return st;
    if (ws && ((uintptr_t)ws & 255))
        return fail(JBFD_EINVAL, "%s: workspace not 256-byte aligned", name);
    if (!ws) ws_bytes = 0;
    return run_project_densify(name, pts_xyz, n, cam_from_world, K, rgb_hwc, radius,
                               sigma_s, sigma_r, prec, zbuf, sparse_depth,
                               sparse_valid, dense_depth, dense_valid, ws, ws_bytes,
                               stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// jbfd_project_densify_noalloc: the sample lists live in a fixed device array
// of this file, one copy per GPU, instead of a caller workspace.
// ---------------------------------------------------------------------------

namespace {

// The array itself. In host code `scratch` names a host-side stand-in, not
// the device memory: its device address, which differs per GPU, comes from
// hipGetSymbolAddress with that GPU current, and only that address is ever
// passed to kernels.
__device__ __align__(256) unsigned char scratch[JBFD_NOALLOC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device and kept.
jbfd_status scratch_address(const char *name, void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(JBFD_EHIP, "%s: hipGetDevice: %s", name, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(JBFD_EUNSUPPORTED, "%s: device %d beyond the %d supported", name,
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(JBFD_EHIP, "%s: hipGetSymbolAddress: %s", name,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return JBFD_OK;
}

}  // namespace

extern "C" {

jbfd_status jbfd_project_densify_noalloc(const float *pts_xyz, int64_t n,
                                         const double cam_from_world[12],
                                         const jbfd_intrinsics *K,
                                         const uint8_t *rgb_hwc, int32_t radius,
                                         float sigma_s, float sigma_r,
                                         jbfd_precision prec, uint64_t *zbuf,
                                         float *sparse_depth, uint8_t *sparse_valid,
                                         float *dense_depth, uint8_t *dense_valid,
                                         void *stream) {
    const char *name = "jbfd_project_densify_noalloc";
    jbfd_status st = check_project_densify(
        name, pts_xyz, n, cam_from_world, K, rgb_hwc, radius, sigma_s, sigma_r, prec,
        zbuf, sparse_depth, sparse_valid, dense_depth, dense_valid);
    if (st != JBFD_OK) return st;
    // every valid sample is a projected point, so n bounds the lists
    const size_t need = jbfd::densify_ws_bytes(K->height, K->width, radius, n);
    if (need > JBFD_NOALLOC_WS_BYTES)
        return fail(JBFD_ENOSPC,
                    "%s: the sample lists of a %d x %d image with up to %lld points "
                    "at radius %d need %zu bytes, more than the %zu bytes built in",
                    name, K->width, K->height, (long long)n, radius, need,
                    (size_t)JBFD_NOALLOC_WS_BYTES);
    void *ws = nullptr;
    st = scratch_address(name, &ws);
    if (st != JBFD_OK) return st;
    return run_project_densify(name, pts_xyz, n, cam_from_world, K, rgb_hwc, radius,
                               sigma_s, sigma_r, prec, zbuf, sparse_depth,
                               sparse_valid, dense_depth, dense_valid, ws,
                               JBFD_NOALLOC_WS_BYTES, stream);
}

jbfd_status jbfd_zbuf_clear(uint64_t *zbuf, int32_t H, int32_t W, void *stream) {
    if (!zbuf) return fail(JBFD_EINVAL, "jbfd_zbuf_clear: null zbuf");
    const jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    return hip_status(jbfd::launch_fill_keys(zbuf, (int64_t)H * W, (hipStream_t)stream),
                      "jbfd_zbuf_clear");
}

jbfd_status jbfd_densify(const float *sparse_depth, const uint8_t *sparse_valid,
                         const uint8_t *rgb_hwc, int32_t H, int32_t W,
                         int32_t radius, float sigma_s, float sigma_r,
                         jbfd_precision prec, float *dense_depth,
                         uint8_t *dense_valid, float *aux, void *ws,
                         size_t ws_bytes, uint32_t flags, void *stream) {
    if (!sparse_depth || !sparse_valid || !rgb_hwc || !dense_depth || !dense_valid)
        return fail(JBFD_EINVAL, "jbfd_densify: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    st = check_filter(radius, sigma_s, sigma_r);
    if (st != JBFD_OK) return st;
    if (prec != JBFD_FP32 && prec != JBFD_FP16_RANGE)
        return fail(JBFD_EINVAL, "jbfd_densify: unknown precision %d", (int)prec);
    if (aux && prec != JBFD_FP32)
        return fail(JBFD_EINVAL, "jbfd_densify: aux is produced by FP32 only");
    if (ws && ((uintptr_t)ws & 255))
        return fail(JBFD_EINVAL, "jbfd_densify: workspace not 256-byte aligned");
    if (!ws) ws_bytes = 0;
    if (flags & ~(JBFD_LISTS_READY | JBFD_DENSE))
        return fail(JBFD_EINVAL, "jbfd_densify: unknown flags 0x%x", flags);
    jbfd::FilterParams fp{radius, log2_half_inv_var(sigma_r),
                          log2_half_inv_var(sigma_s)};
    if (flags & JBFD_DENSE) {
        if (radius > JBFD_DENSE_MAX_RADIUS || prec != JBFD_FP32 || aux)
            return fail(JBFD_EUNSUPPORTED,
                        "jbfd_densify: the dense kernel takes radius <= %d, "
                        "FP32 and no aux", JBFD_DENSE_MAX_RADIUS);
        return hip_status(jbfd::launch_densify_dense(sparse_depth, sparse_valid,
                                                     rgb_hwc, H, W, fp,
                                                     dense_depth, dense_valid,
                                                     (hipStream_t)stream),
                          "jbfd_densify");
    }
    hipError_t e = jbfd::launch_densify(sparse_depth, sparse_valid, rgb_hwc, H, W,
                                        fp, prec, dense_depth, dense_valid, aux,
                                        ws, ws_bytes, (flags & JBFD_LISTS_READY) != 0,
                                        (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(JBFD_EUNSUPPORTED, "jbfd_densify: precision not built");
    return hip_status(e, "jbfd_densify");
}

jbfd_status jbfd_densify_prepare(const float *sparse_depth,
                                 const uint8_t *sparse_valid,
                                 const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                 int32_t radius, void *ws, size_t ws_bytes,
                                 void *stream) {
    if (!sparse_depth || !sparse_valid || !rgb_hwc || !ws)
        return fail(JBFD_EINVAL, "jbfd_densify_prepare: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    if (radius < 0 || radius > JBFD_MAX_RADIUS)
        return fail(JBFD_EINVAL, "radius %d outside 0..%d", radius,
                    JBFD_MAX_RADIUS);
    if ((uintptr_t)ws & 255)
        return fail(JBFD_EINVAL, "jbfd_densify_prepare: workspace not aligned");
    return hip_status(jbfd::launch_densify_prepare(sparse_depth, sparse_valid,
                                                   rgb_hwc, H, W, radius, ws,
                                                   ws_bytes, (hipStream_t)stream),
                      "jbfd_densify_prepare");
}

jbfd_status jbfd_densify_backward(const float *sparse_depth,
                                  const uint8_t *sparse_valid,
                                  const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                  int32_t radius, float sigma_s, float sigma_r,
                                  const float *dense_depth, const float *aux,
                                  const float *grad_out, float *grad_depth,
                                  double *grad_sigmas, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (!sparse_depth || !sparse_valid || !rgb_hwc || !dense_depth || !aux ||
        !grad_out || !grad_depth || !grad_sigmas || !ws)
        return fail(JBFD_EINVAL, "jbfd_densify_backward: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    st = check_filter(radius, sigma_s, sigma_r);
    if (st != JBFD_OK) return st;
    if (ws_bytes < jbfd::backward_ws_bytes(H, W))
        return fail(JBFD_ENOSPC, "jbfd_densify_backward: workspace %zu < %zu",
                    ws_bytes, jbfd::backward_ws_bytes(H, W));
    jbfd::FilterParams fp{radius, log2_half_inv_var(sigma_r),
                          log2_half_inv_var(sigma_s)};
    return hip_status(jbfd::launch_densify_backward(
                          sparse_depth, sparse_valid, rgb_hwc, H, W, fp, sigma_s,
                          sigma_r, dense_depth, aux, grad_out, grad_depth,
                          grad_sigmas, ws, (hipStream_t)stream),
                      "jbfd_densify_backward");
}

size_t jbfd_densify_ws_bytes(int32_t H, int32_t W, int32_t radius,
                             int64_t max_samples) {
    if (H <= 0 || W <= 0 || H > JBFD_MAX_SIDE || W > JBFD_MAX_SIDE || radius < 0 ||
        radius > JBFD_MAX_RADIUS || max_samples < 0)
        return 0;
    return jbfd::densify_ws_bytes(H, W, radius, max_samples);
}

size_t jbfd_densify_backward_ws_bytes(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0 || H > JBFD_MAX_SIDE || W > JBFD_MAX_SIDE) return 0;
    return jbfd::backward_ws_bytes(H, W);
}

jbfd_status jbfd_pool3(const float *sparse_depth, const uint8_t *sparse_valid,
                       const uint8_t *rgb_hwc, int32_t H, int32_t W,
                       float *depth1, uint8_t *valid1, uint8_t *rgb1,
                       void *stream) {
    if (!sparse_depth || !sparse_valid || !rgb_hwc || !depth1 || !valid1 || !rgb1)
        return fail(JBFD_EINVAL, "jbfd_pool3: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    return hip_status(jbfd::launch_pool3(sparse_depth, sparse_valid, rgb_hwc, H, W,
                                         depth1, valid1, rgb1, (hipStream_t)stream),
                      "jbfd_pool3");
}

jbfd_status jbfd_restore_merge(const float *sparse_depth,
                               const uint8_t *sparse_valid,
                               const float *depth1, const uint8_t *valid1,
                               int32_t H, int32_t W, float *depth2,
                               uint8_t *valid2, void *stream) {
    if (!sparse_depth || !sparse_valid || !depth1 || !valid1 || !depth2 || !valid2)
        return fail(JBFD_EINVAL, "jbfd_restore_merge: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    return hip_status(jbfd::launch_restore_merge(sparse_depth, sparse_valid, depth1,
                                                 valid1, H, W, depth2, valid2,
                                                 (hipStream_t)stream),
                      "jbfd_restore_merge");
}

size_t jbfd_two_stage_ws_bytes(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0 || H > JBFD_MAX_SIDE || W > JBFD_MAX_SIDE) return 0;
    return jbfd::two_stage_ws_bytes(H, W);
}

jbfd_status jbfd_densify_two_stage(const float *sparse_depth,
                                   const uint8_t *sparse_valid,
                                   const uint8_t *rgb_hwc, int32_t H, int32_t W,
                                   const jbfd_two_stage *params,
                                   float *dense_depth, uint8_t *dense_valid,
                                   void *ws, size_t ws_bytes, void *stream) {
    if (!sparse_depth || !sparse_valid || !rgb_hwc || !params || !dense_depth ||
        !dense_valid || !ws)
        return fail(JBFD_EINVAL, "jbfd_densify_two_stage: null buffer or params");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    st = check_filter(params->radius1, params->sigma_s1, params->sigma_r1);
    if (st != JBFD_OK) return st;
    st = check_filter(params->radius2, params->sigma_s2, params->sigma_r2);
    if (st != JBFD_OK) return st;
    if ((uintptr_t)ws & 255)
        return fail(JBFD_EINVAL, "jbfd_densify_two_stage: workspace not aligned");
    if (ws_bytes < jbfd::two_stage_ws_bytes(H, W))
        return fail(JBFD_ENOSPC, "jbfd_densify_two_stage: workspace %zu < %zu bytes",
                    ws_bytes, jbfd::two_stage_ws_bytes(H, W));
    const jbfd::FilterParams f1{params->radius1, log2_half_inv_var(params->sigma_r1),
                                log2_half_inv_var(params->sigma_s1)};
    const jbfd::FilterParams f2{params->radius2, log2_half_inv_var(params->sigma_r2),
                                log2_half_inv_var(params->sigma_s2)};
    return hip_status(jbfd::launch_two_stage(sparse_depth, sparse_valid, rgb_hwc, H,
                                             W, f1, f2, dense_depth, dense_valid,
                                             ws, (hipStream_t)stream),
                      "jbfd_densify_two_stage");
}

jbfd_status jbfd_remove_occluded(const float *sparse_depth,
                                 const uint8_t *sparse_valid, int32_t H,
                                 int32_t W, int32_t k, float tau,
                                 uint8_t *valid_out, void *stream) {
    if (!sparse_depth || !sparse_valid || !valid_out)
        return fail(JBFD_EINVAL, "jbfd_remove_occluded: null buffer");
    if (valid_out == sparse_valid)
        return fail(JBFD_EINVAL, "jbfd_remove_occluded: valid_out aliases the input");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    if (k < 0 || k > JBFD_OCCLUSION_MAX_K)
        return fail(JBFD_EINVAL, "jbfd_remove_occluded: k %d outside 0..%d", k,
                    JBFD_OCCLUSION_MAX_K);
    if (!isfinite(tau) || tau < 0.0f)
        return fail(JBFD_EINVAL, "jbfd_remove_occluded: tau must be finite and >= 0");
    return hip_status(jbfd::launch_remove_occluded(sparse_depth, sparse_valid, H, W,
                                                   k, (double)tau, valid_out,
                                                   (hipStream_t)stream),
                      "jbfd_remove_occluded");
}

size_t jbfd_backproject_ws_bytes(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0 || H > JBFD_MAX_SIDE || W > JBFD_MAX_SIDE ||
        (int64_t)H * W > JBFD_BACKPROJECT_MAX_PIXELS)
        return 0;
    return jbfd::backproject_ws_bytes(H, W);
}

jbfd_status jbfd_backproject(const float *dense_depth, const uint8_t *dense_valid,
                             const uint8_t *rgb_hwc, int32_t H, int32_t W,
                             const double cam_from_world[12],
                             const jbfd_intrinsics *K, float tau, float *xyz,
                             uint8_t *rgb_out, int64_t *count, void *ws,
                             size_t ws_bytes, void *stream) {
    if (!dense_depth || !dense_valid || !rgb_hwc || !cam_from_world || !K || !xyz ||
        !rgb_out || !count || !ws)
        return fail(JBFD_EINVAL, "jbfd_backproject: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    if ((int64_t)H * W > JBFD_BACKPROJECT_MAX_PIXELS)
        return fail(JBFD_EINVAL, "jbfd_backproject: %d x %d pixels above the limit %d", H,
                    W, JBFD_BACKPROJECT_MAX_PIXELS);
    if (K->width != W || K->height != H)
        return fail(JBFD_EINVAL, "jbfd_backproject: intrinsics size %d x %d != image",
                    K->width, K->height);
    for (int t = 0; t < 12; ++t)
        if (!isfinite(cam_from_world[t]))
            return fail(JBFD_EINVAL, "jbfd_backproject: pose entry %d not finite", t);
    if (!isfinite(K->fx) || !isfinite(K->fy) || !isfinite(K->cx) ||
        !isfinite(K->cy) || K->fx == 0.0 || K->fy == 0.0)
        return fail(JBFD_EINVAL, "jbfd_backproject: intrinsics not finite or zero focal");
    if (isnan(tau) || tau < 0.0f)
        return fail(JBFD_EINVAL, "jbfd_backproject: tau must be >= 0 or +inf");
    if ((uintptr_t)ws & 255)
        return fail(JBFD_EINVAL, "jbfd_backproject: workspace not aligned");
    if (ws_bytes < jbfd::backproject_ws_bytes(H, W))
        return fail(JBFD_ENOSPC, "jbfd_backproject: workspace %zu < %zu bytes",
                    ws_bytes, jbfd::backproject_ws_bytes(H, W));
    jbfd::Pose P;
    for (int t = 0; t < 12; ++t) P.m[t] = cam_from_world[t];
    jbfd::Intr I{K->fx, K->fy, K->cx, K->cy, K->width, K->height};
    return hip_status(jbfd::launch_backproject(dense_depth, dense_valid, rgb_hwc, H,
                                               W, P, I, (double)tau, xyz, rgb_out,
                                               count, ws, (hipStream_t)stream),
                      "jbfd_backproject");
}

jbfd_status jbfd_motion_mask(const uint8_t *rgb_hwc, const uint8_t *rgb_prev_hwc,
                             int32_t H, int32_t W, float tau, int32_t k,
                             uint8_t *mask, void *stream) {
    if (!rgb_hwc || !rgb_prev_hwc || !mask)
        return fail(JBFD_EINVAL, "jbfd_motion_mask: null buffer");
    jbfd_status st = check_image(H, W);
    if (st != JBFD_OK) return st;
    if (k < 0 || k > JBFD_MOTION_MAX_K)
        return fail(JBFD_EINVAL, "jbfd_motion_mask: k %d outside 0..%d", k,
                    JBFD_MOTION_MAX_K);
    if (!isfinite(tau) || tau < 0.0f)
        return fail(JBFD_EINVAL, "jbfd_motion_mask: tau must be finite and >= 0");
    return hip_status(jbfd::launch_motion_mask(rgb_hwc, rgb_prev_hwc, H, W,
                                               (double)tau, k, mask,
                                               (hipStream_t)stream),
                      "jbfd_motion_mask");
}

jbfd_status jbfd_project_motion(const float *pts_xyz, int64_t n,
                                const int8_t *sweep_ids, int8_t latest,
                                const uint8_t *motion,
                                const double cam_from_world[12],
                                const jbfd_intrinsics *K, uint64_t *zbuf,
                                float *sparse_depth, uint8_t *sparse_valid,
                                void *stream) {
    if (!cam_from_world || !K || !zbuf || !motion)
        return fail(JBFD_EINVAL, "jbfd_project_motion: null pose, intrinsics, zbuf or mask");
    if (n < 0 || n >= ((int64_t)1 << 32))
        return fail(JBFD_EINVAL, "jbfd_project_motion: n = %lld outside 0..2^32-1",
                    (long long)n);
    if (n > 0 && (!pts_xyz || !sweep_ids))
        return fail(JBFD_EINVAL, "jbfd_project_motion: null points or sweep ids");
    jbfd_status st = check_image(K->height, K->width);
    if (st != JBFD_OK) return st;
    for (int t = 0; t < 12; ++t)
        if (!isfinite(cam_from_world[t]))
            return fail(JBFD_EINVAL, "jbfd_project_motion: pose entry %d not finite", t);
    if (!isfinite(K->fx) || !isfinite(K->fy) || !isfinite(K->cx) ||
        !isfinite(K->cy))
        return fail(JBFD_EINVAL, "jbfd_project_motion: intrinsics not finite");
    jbfd::Pose P;
    for (int t = 0; t < 12; ++t) P.m[t] = cam_from_world[t];
    jbfd::Intr I{K->fx, K->fy, K->cx, K->cy, K->width, K->height};
    return hip_status(jbfd::launch_project_motion(pts_xyz, n, sweep_ids, latest,
                                                  motion, P, I, zbuf, sparse_depth,
                                                  sparse_valid, (hipStream_t)stream),
                      "jbfd_project_motion");
}

size_t jbfd_batch_table_bytes(int32_t n_views) {
    if (n_views < 1) return 0;
    return jbfd::batch_counters_offset(n_views) +
           (size_t)n_views * sizeof(jbfd::BatchCounters);
}

jbfd_status jbfd_batch_prepare(const jbfd_view *views, int32_t n_views,
                               void *host_table, size_t table_bytes) {
    if (!views || !host_table || n_views < 1)
        return fail(JBFD_EINVAL, "jbfd_batch_prepare: null views/table or no views");
    if (table_bytes < jbfd_batch_table_bytes(n_views))
        return fail(JBFD_ENOSPC, "jbfd_batch_prepare: table %zu < %zu bytes",
                    table_bytes, jbfd_batch_table_bytes(n_views));
    jbfd::BatchHeader *hdr = static_cast<jbfd::BatchHeader *>(host_table);
    jbfd::BatchView *out = reinterpret_cast<jbfd::BatchView *>(
        static_cast<unsigned char *>(host_table) + sizeof(jbfd::BatchHeader));
    int64_t tiles = 0, px_chunks = 0, pt_chunks = 0, units = 0;
    int64_t fpx = 0, fpt = 0, ftile = 0;   // items of the one-launch run
    int32_t max_radius = 0;
    for (int32_t v = 0; v < n_views; ++v) {
        const jbfd_view &x = views[v];
        if (!x.rgb || !x.zbuf || !x.sparse_depth || !x.sparse_valid ||
            !x.dense_depth || !x.dense_valid || (x.n_points > 0 && !x.points))
            return fail(JBFD_EINVAL, "batch view %d: null buffer", v);
        if (x.n_points < 0 || x.n_points >= ((int64_t)1 << 32))
            return fail(JBFD_EINVAL, "batch view %d: n_points out of range", v);
        jbfd_status st = check_image(x.K.height, x.K.width);
        if (st != JBFD_OK) return prefix_error(st, v);
        st = check_filter(x.radius, x.sigma_s, x.sigma_r);
        if (st != JBFD_OK) return prefix_error(st, v);
        for (int t = 0; t < 12; ++t)
            if (!isfinite(x.cam_from_world[t]))
                return fail(JBFD_EINVAL, "batch view %d: pose not finite", v);
        if (!isfinite(x.K.fx) || !isfinite(x.K.fy) || !isfinite(x.K.cx) ||
            !isfinite(x.K.cy))
            return fail(JBFD_EINVAL, "batch view %d: intrinsics not finite", v);
        jbfd::BatchView &b = out[v];
        b.pts = x.points;
        b.n_pts = x.n_points;
        for (int t = 0; t < 12; ++t) b.pose[t] = x.cam_from_world[t];
        b.fx = x.K.fx;
        b.fy = x.K.fy;
        b.cx = x.K.cx;
        b.cy = x.K.cy;
        b.W = x.K.width;
        b.H = x.K.height;
        b.rgb = x.rgb;
        b.zbuf = x.zbuf;
        b.sd = x.sparse_depth;
        b.sv = x.sparse_valid;
        b.out = x.dense_depth;
        b.mask = x.dense_valid;
        b.radius = x.radius;
        b.kr = log2_half_inv_var(x.sigma_r);
        b.ks = log2_half_inv_var(x.sigma_s);
        b.tiles_x = (x.K.width + jbfd::kTileEdge - 1) / jbfd::kTileEdge;
        b.n_tiles = b.tiles_x * ((x.K.height + jbfd::kTileEdge - 1) / jbfd::kTileEdge);
        b.tile_off = (int32_t)tiles;
        tiles += b.n_tiles;
        const int64_t npix = (int64_t)x.K.width * x.K.height;
        b.px_chunk_off = (int32_t)px_chunks;
        px_chunks += (npix + jbfd::kBatchChunk - 1) / jbfd::kBatchChunk;
        b.pt_chunk_off = (int32_t)pt_chunks;
        pt_chunks += (x.n_points + jbfd::kBatchChunk - 1) / jbfd::kBatchChunk;
        // one-launch queue: projection chunks, decode chunks, filter items
        b.fpx_off = (int32_t)fpx;
        fpx += (npix + jbfd::kFusedPxChunk - 1) / jbfd::kFusedPxChunk;
        b.fpt_off = (int32_t)fpt;
        fpt += (x.n_points + jbfd::kFusedPtChunk - 1) / jbfd::kFusedPtChunk;
        b.ftile_off = (int32_t)ftile;
        ftile += (b.n_tiles + jbfd::kFusedTiles - 1) / jbfd::kFusedTiles;
        b.pad_ = 0;
        if (x.radius > max_radius) max_radius = x.radius;
        // sample lists (as jbfd_densify with a workspace)
        const jbfd::ListLayout L = jbfd::list_layout(x.K.height, x.K.width);
        b.recs = nullptr;
        b.rowoff = b.bandcnt = b.grpcnt = nullptr;
        b.capacity = 0;
        b.n_strips = L.n_strips;
        b.n_groups = L.n_groups;
        b.n_bands = L.n_bands;
        b.unit_off = (int32_t)units;
        if (x.list_ws) {
            if ((uintptr_t)x.list_ws & 255)
                return fail(JBFD_EINVAL, "batch view %d: list workspace not aligned", v);
            jbfd::ListViews lv;
            if (!jbfd::list_views(x.list_ws, x.list_ws_bytes, L, lv))
                return fail(JBFD_ENOSPC, "batch view %d: list workspace %zu < %zu bytes",
                            v, x.list_ws_bytes, L.recs);
            if (jbfd::lists_possible(x.K.height, x.K.width, x.radius)) {
                b.recs = lv.recs;
                b.rowoff = lv.rowoff;
                b.bandcnt = lv.bandcnt;
                b.grpcnt = lv.grpcnt;
                b.capacity = lv.capacity;
                units += (int64_t)L.n_groups * L.n_bands;
            }
        }
        // the queues number every item in one int32 (well below 2^30 items
        // when the launch-sequence counts, which are larger, are)
        if (tiles >= ((int64_t)1 << 30) || px_chunks >= ((int64_t)1 << 30) ||
            pt_chunks >= ((int64_t)1 << 30) || units >= ((int64_t)1 << 30))
            return fail(JBFD_EINVAL, "batch: too many tiles or chunks");
    }
    hdr->n_views = n_views;
    hdr->total_tiles = (int32_t)tiles;
    hdr->px_chunks = (int32_t)px_chunks;
    hdr->pt_chunks = (int32_t)pt_chunks;
    hdr->list_units = (int32_t)units;
    hdr->max_radius = max_radius;
    hdr->fpx_chunks = (int32_t)fpx;
    hdr->fpt_chunks = (int32_t)fpt;
    hdr->ftile_items = (int32_t)ftile;
    hdr->exited = 0;
    hdr->error = 0;
    hdr->pad_ = 0;
    unsigned char *state = static_cast<unsigned char *>(host_table) +
                           jbfd::batch_queues_offset(n_views);
    memset(state, 0, jbfd_batch_table_bytes(n_views) - jbfd::batch_queues_offset(n_views));
    return ok();
}

jbfd_status jbfd_batch_run(void *d_table, int32_t max_radius, jbfd_precision prec,
                           uint32_t flags, void *stream) {
    if (!d_table || ((uintptr_t)d_table & 7))
        return fail(JBFD_EINVAL, "jbfd_batch_run: null or misaligned table");
    if (max_radius < 0 || max_radius > JBFD_MAX_RADIUS)
        return fail(JBFD_EINVAL, "jbfd_batch_run: max_radius %d", max_radius);
    if (prec != JBFD_FP32 && prec != JBFD_FP16_RANGE)
        return fail(JBFD_EINVAL, "jbfd_batch_run: unknown precision %d", (int)prec);
    if (flags & ~(JBFD_BATCH_LISTS | JBFD_BATCH_STAGED))
        return fail(JBFD_EINVAL, "jbfd_batch_run: unknown flags 0x%x", flags);
    hipError_t e;
    if (flags & (JBFD_BATCH_LISTS | JBFD_BATCH_STAGED))
        e = jbfd::launch_batch(d_table, max_radius, (flags & JBFD_BATCH_LISTS) != 0, prec,
                               (hipStream_t)stream);
    else
        e = jbfd::launch_batch_fused(d_table, max_radius, prec, (hipStream_t)stream);
    return hip_status(e, "jbfd_batch_run");
}

jbfd_status jbfd_batch_check(const void *d_table, void *stream) {
    if (!d_table || ((uintptr_t)d_table & 7))
        return fail(JBFD_EINVAL, "jbfd_batch_check: null or misaligned table");
    uint32_t err = 0;
    const unsigned char *src = static_cast<const unsigned char *>(d_table) +
                               offsetof(jbfd::BatchHeader, error);
    hipError_t e = hipMemcpyAsync(&err, src, sizeof err, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_status(e, "jbfd_batch_check");
    if (err & jbfd::kBatchErrRadius)
        return fail(JBFD_EINVAL,
                    "jbfd_batch_check: a view's radius exceeded the max_radius of the "
                    "run; its outputs were set to zero");
    if (err & jbfd::kBatchErrWait)
        return fail(JBFD_EHIP,
                    "jbfd_batch_check: a work item gave up waiting for the items it "
                    "depends on; the batch's outputs are not valid");
    return ok();
}

}  // extern "C"

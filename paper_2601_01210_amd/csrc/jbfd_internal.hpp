// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/jbfd.h"

namespace jbfd {

// Camera-from-world [R|t] passed by value to kernels.
struct Pose {
    double m[12];
};

struct Intr {
    double fx, fy, cx, cy;
    int32_t w, h;
};

constexpr uint64_t kEmptyKey = ~0ull;

// Filter parameters in log2 units: weight = exp2(-kr*c - ks*s), with
// kr = log2(e) / (2 sigma_r^2) and ks = log2(e) / (2 sigma_s^2).
struct FilterParams {
    int32_t radius;
    float kr;
    float ks;
};

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_project(const float *pts, int64_t n, const Pose &pose,
                          const Intr &K, uint64_t *zbuf, float *depth,
                          uint8_t *valid, hipStream_t s);

hipError_t launch_densify(const float *D, const uint8_t *B, const uint8_t *rgb,
                          int32_t H, int32_t W, const FilterParams &fp,
                          jbfd_precision prec, float *out, uint8_t *mask,
                          float *aux, void *ws, size_t ws_bytes, bool lists_ready,
                          hipStream_t s);

hipError_t launch_densify_prepare(const float *D, const uint8_t *B,
                                  const uint8_t *rgb, int32_t H, int32_t W,
                                  int32_t radius, void *ws, size_t ws_bytes,
                                  hipStream_t s);

size_t densify_ws_bytes(int32_t H, int32_t W, int32_t r, int64_t max_samples);

hipError_t launch_densify_backward(const float *D, const uint8_t *B,
                                   const uint8_t *rgb, int32_t H, int32_t W,
                                   const FilterParams &fp, float sigma_s,
                                   float sigma_r, const float *out,
                                   const float *aux, const float *g,
                                   float *grad_d, double *grad_sigmas,
                                   void *ws, hipStream_t s);

size_t backward_ws_bytes(int32_t H, int32_t W);

}  // namespace jbfd

// The projection of one point (Sec. 2: the merged sweeps are projected into
// the camera view to form one depth image), shared by the single-view and
// batched kernels. Every source that includes it is built with
// -ffp-contract=off: the double-precision steps below must not be fused.
#pragma once

#include "jbfd_internal.hpp"

namespace jbfd {

// Project point i; false if it is culled. Otherwise key and pixel index.
__device__ inline bool project_one(const float *__restrict__ pts, int64_t i,
                                   const double *__restrict__ m, double fx,
                                   double fy, double cx, double cy, int32_t w,
                                   int32_t h, unsigned long long &key,
                                   int64_t &pix) {
    const double x = (double)pts[3 * i + 0];
    const double y = (double)pts[3 * i + 1];
    const double z = (double)pts[3 * i + 2];
    // each row summed left to right; no contraction into FMA
    double X = m[0] * x;
    X = X + m[1] * y;
    X = X + m[2] * z;
    X = X + m[3];
    double Y = m[4] * x;
    Y = Y + m[5] * y;
    Y = Y + m[6] * z;
    Y = Y + m[7];
    double Z = m[8] * x;
    Z = Z + m[9] * y;
    Z = Z + m[10] * z;
    Z = Z + m[11];
    if (!(Z > 0.0) || !__builtin_isfinite(Z)) return false;
    const double u = fx * (X / Z) + cx;
    const double v = fy * (Y / Z) + cy;
    if (!(u >= 0.0 && u < (double)w)) return false;
    if (!(v >= 0.0 && v < (double)h)) return false;
    const int64_t col = (int64_t)__builtin_floor(u);
    const int64_t row = (int64_t)__builtin_floor(v);
    const float zf = (float)Z;
    if (zf == 0.0f || __builtin_isinf(zf)) return false;
    key = ((unsigned long long)__float_as_uint(zf) << 32) |
          (unsigned long long)(uint32_t)i;
    pix = row * w + col;
    return true;
}

}  // namespace jbfd

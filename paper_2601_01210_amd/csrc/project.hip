// Projection of merged LiDAR points into the camera with a nearest-depth
// z-buffer (Sec. 2: the merged sweeps are projected into the camera view to
// form one depth image). Three kernels on one stream:
//
//   k_fill_keys  clears the H*W 64-bit key image to UINT64_MAX (a fill
//                kernel rather than a memset node, so the sequence can be
//                captured into a graph and replayed);
//   k_project    one thread per point: double-precision rigid transform and
//                pinhole projection in a fixed order without fused
//                multiply-add (the file is built with -ffp-contract=off),
//                then atomicMin of (bits(float Z) << 32 | index) into the
//                pixel's key; positive floats order like their bit
//                patterns, so the minimum key is the nearest point and an
//                exact tie goes to the smaller index;
//   k_decode     key image -> float depth (0 where empty) and 0/1 mask.
//
// Traffic per frame: 12N bytes of points, 8HW to clear, the atomics, 8HW
// read + 5HW written by the decode.
#include "jbfd_internal.hpp"

namespace jbfd {

__global__ __launch_bounds__(256) void k_fill_keys(uint64_t *__restrict__ keys,
                                                   int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 2;
    const bool vec = (reinterpret_cast<uintptr_t>(keys) & 15) == 0;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
         i < n; i += stride) {
        if (vec && i + 1 < n) {
            *reinterpret_cast<ulonglong2 *>(keys + i) =
                make_ulonglong2(kEmptyKey, kEmptyKey);
        } else {
            keys[i] = kEmptyKey;
            if (i + 1 < n) keys[i + 1] = kEmptyKey;
        }
    }
}

__global__ __launch_bounds__(256) void k_project(const float *__restrict__ pts,
                                                 int64_t n, Pose P, Intr K,
                                                 unsigned long long *__restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        const double x = (double)pts[3 * i + 0];
        const double y = (double)pts[3 * i + 1];
        const double z = (double)pts[3 * i + 2];
        // each row summed left to right; no contraction into FMA
        double X = P.m[0] * x;
        X = X + P.m[1] * y;
        X = X + P.m[2] * z;
        X = X + P.m[3];
        double Y = P.m[4] * x;
        Y = Y + P.m[5] * y;
        Y = Y + P.m[6] * z;
        Y = Y + P.m[7];
        double Z = P.m[8] * x;
        Z = Z + P.m[9] * y;
        Z = Z + P.m[10] * z;
        Z = Z + P.m[11];
        if (!(Z > 0.0) || !__builtin_isfinite(Z)) continue;
        const double u = K.fx * (X / Z) + K.cx;
        const double v = K.fy * (Y / Z) + K.cy;
        if (!(u >= 0.0 && u < (double)K.w)) continue;
        if (!(v >= 0.0 && v < (double)K.h)) continue;
        const int64_t col = (int64_t)__builtin_floor(u);
        const int64_t row = (int64_t)__builtin_floor(v);
        const float zf = (float)Z;
        if (zf == 0.0f || __builtin_isinf(zf)) continue;
        const unsigned long long key =
            ((unsigned long long)__float_as_uint(zf) << 32) |
            (unsigned long long)(uint32_t)i;
        atomicMin(keys + row * K.w + col, key);
    }
}

// Four pixels per thread: two 16-byte key loads, one 16-byte depth store and
// one 4-byte mask store; the last group may be partial.
__global__ __launch_bounds__(256) void k_decode(const uint64_t *__restrict__ keys,
                                                int64_t npix,
                                                float *__restrict__ depth,
                                                uint8_t *__restrict__ valid) {
    const int64_t groups = (npix + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool vec = ((reinterpret_cast<uintptr_t>(depth) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(valid) & 3) == 0) &&
                     ((reinterpret_cast<uintptr_t>(keys) & 15) == 0);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
         g += stride) {
        const int64_t p0 = g * 4;
        if (vec && p0 + 4 <= npix) {
            const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(keys + p0);
            const ulonglong2 b = *reinterpret_cast<const ulonglong2 *>(keys + p0 + 2);
            const uint64_t k[4] = {a.x, a.y, b.x, b.y};
            float d[4];
            uint32_t m = 0;
            for (int t = 0; t < 4; ++t) {
                const bool hit = k[t] != kEmptyKey;
                d[t] = hit ? __uint_as_float((uint32_t)(k[t] >> 32)) : 0.0f;
                m |= (uint32_t)hit << (8 * t);
            }
            if (depth)
                *reinterpret_cast<float4 *>(depth + p0) = make_float4(d[0], d[1], d[2], d[3]);
            if (valid) *reinterpret_cast<uint32_t *>(valid + p0) = m;
        } else {
            for (int64_t p = p0; p < npix && p < p0 + 4; ++p) {
                const uint64_t k = keys[p];
                const bool hit = k != kEmptyKey;
                if (depth) depth[p] = hit ? __uint_as_float((uint32_t)(k >> 32)) : 0.0f;
                if (valid) valid[p] = (uint8_t)hit;
            }
        }
    }
}

static int grid_for(int64_t work, int per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

hipError_t launch_project(const float *pts, int64_t n, const Pose &pose,
                          const Intr &K, uint64_t *zbuf, float *depth,
                          uint8_t *valid, hipStream_t s) {
    const int64_t npix = (int64_t)K.w * K.h;
    k_fill_keys<<<grid_for(npix, 512), 256, 0, s>>>(zbuf, npix);
    if (n > 0)
        k_project<<<grid_for(n, 256), 256, 0, s>>>(
            pts, n, pose, K, reinterpret_cast<unsigned long long *>(zbuf));
    if (depth || valid)
        k_decode<<<grid_for(npix, 1024), 256, 0, s>>>(zbuf, npix, depth, valid);
    return hipGetLastError();
}

}  // namespace jbfd

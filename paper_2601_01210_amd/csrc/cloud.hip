// Occluded-point removal (Sec. 4.1) and contour removal with
// back-projection to a coloured world cloud (Sec. 5, Sec. 2).
//
//   k_remove_occluded  one thread per pixel of a 16x16 tile; the tile and a
//                      halo of kOccMaxK pixels of depth (0 where invalid) and
//                      validity are staged in LDS; a valid pixel sums the
//                      valid depths of its (2k+1)^2 window in double, in
//                      row-major order, and keeps its sample unless
//                      D - mean > tau * mean (in double);
//   k_cloud_count      1024-pixel chunks of the row-major pixel order: the
//                      number of pixels that are valid and pass the contour
//                      rule (largest jump to a valid 4-neighbour, in double,
//                      at most tau * D);
//   k_cloud_write      each chunk sums the counts of the chunks before it,
//                      ranks its kept pixels by a block scan (four
//                      consecutive pixels per thread, so the output keeps
//                      row-major order) and writes each one's world point,
//                      R^T (p_c - t) with p_c through the pixel centre, in
//                      double with a fixed operation order (no contraction)
//                      rounded once to float, and its colour. The last chunk
//                      writes the total.
#include "filter_common.hpp"

namespace jbfd {

constexpr int kOccMaxK = 8;
constexpr int kCloudChunk = 1024;

__global__ __launch_bounds__(256) void k_remove_occluded(
    const float *__restrict__ D, const uint8_t *__restrict__ B, int H, int W,
    int k, double tau, uint8_t *__restrict__ Bout) {
    constexpr int E = kTile + 2 * kOccMaxK;
    __shared__ float sd[E * E];
    __shared__ uint8_t sb[E * E];
    const int tiles_x = (W + kTile - 1) / kTile;
    const int ty0 = (blockIdx.x / tiles_x) * kTile, tx0 = (blockIdx.x % tiles_x) * kTile;
    for (int e = threadIdx.x; e < E * E; e += 256) {
        const int ly = e / E, lx = e - ly * E;
        const int y = ty0 - kOccMaxK + ly, x = tx0 - kOccMaxK + lx;
        float d = 0.0f;
        uint8_t v = 0;
        if (y >= 0 && y < H && x >= 0 && x < W) {
            const int64_t p = (int64_t)y * W + x;
            v = B[p] != 0;
            d = v ? D[p] : 0.0f;
        }
        sd[e] = d;
        sb[e] = v;
    }
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x >= W || y >= H) return;
    const int c = (ly + kOccMaxK) * E + lx + kOccMaxK;
    uint8_t keep = 0;
    if (sb[c]) {
        double sum = 0.0;
        int n = 0;
        for (int dy = -k; dy <= k; ++dy) {
            for (int dx = -k; dx <= k; ++dx) {
                const int q = c + dy * E + dx;   // out-of-image taps hold 0/0
                if (sb[q]) {
                    sum = sum + (double)sd[q];
                    ++n;
                }
            }
        }
        const double mean = sum / (double)n;
        keep = (uint8_t)!((double)sd[c] - mean > tau * mean);
    }
    Bout[(int64_t)y * W + x] = keep;
}

// Contour rule at pixel (x, y): largest |D(n) - D(x)| over valid
// 4-neighbours, in double, against tau * D(x).
__device__ inline bool contour_keep(const float *__restrict__ D,
                                    const uint8_t *__restrict__ M, int H, int W,
                                    int x, int y, double tau) {
    const int64_t p = (int64_t)y * W + x;
    const double z = (double)D[p];
    double g = 0.0;
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xx = x + dx[i], yy = y + dy[i];
        if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
        const int64_t q = (int64_t)yy * W + xx;
        if (!M[q]) continue;
        const double diff = __builtin_fabs((double)D[q] - z);
        if (diff > g) g = diff;
    }
    return !(g > tau * z);
}

__device__ inline int kept_of_four(const float *__restrict__ D,
                                   const uint8_t *__restrict__ M, int H, int W,
                                   int64_t p0, double tau, bool (&keep)[4]) {
    const int64_t n = (int64_t)H * W;
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t p = p0 + u;
        keep[u] = false;
        if (p < n && M[p]) {
            const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
            keep[u] = contour_keep(D, M, H, W, x, y, tau);
        }
        cnt += keep[u] ? 1 : 0;
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_cloud_count(const float *__restrict__ D,
                                                     const uint8_t *__restrict__ M,
                                                     int H, int W, double tau,
                                                     int *__restrict__ counts) {
    __shared__ int part[4];
    const int64_t p0 = (int64_t)blockIdx.x * kCloudChunk + 4 * threadIdx.x;
    bool keep[4];
    int cnt = kept_of_four(D, M, H, W, p0, tau, keep);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ __launch_bounds__(256) void k_cloud_write(
    const float *__restrict__ D, const uint8_t *__restrict__ M,
    const uint8_t *__restrict__ rgb, int H, int W, Pose P, Intr K, double tau,
    const int *__restrict__ counts, float *__restrict__ xyz,
    uint8_t *__restrict__ rgb_out, int64_t *__restrict__ total) {
    __shared__ int wsum[4];
    __shared__ int64_t wacc[4];
    __shared__ int64_t before_s;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int chunk = blockIdx.x;
    // points of all earlier chunks
    int64_t acc = 0;
    for (int c = t; c < chunk; c += 256) acc += counts[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) wacc[wid] = acc;
    __syncthreads();
    if (t == 0) before_s = wacc[0] + wacc[1] + wacc[2] + wacc[3];
    // rank of this thread's kept pixels inside the chunk
    const int64_t p0 = (int64_t)chunk * kCloudChunk + 4 * t;
    bool keep[4];
    const int cnt = kept_of_four(D, M, H, W, p0, tau, keep);
    const int incl = wave_inclusive_scan(cnt);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int wbefore = 0;
    for (int w = 0; w < wid; ++w) wbefore += wsum[w];
    int64_t pos = before_s + wbefore + incl - cnt;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (!keep[u]) continue;
        const int64_t p = p0 + u;
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const double Z = (double)D[p];
        const double Xc = ((double)x + 0.5 - K.cx) * Z / K.fx;
        const double Yc = ((double)y + 0.5 - K.cy) * Z / K.fy;
        const double a = Xc - P.m[3], b = Yc - P.m[7], c = Z - P.m[11];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = P.m[0 + i] * a;
            s = s + P.m[4 + i] * b;
            s = s + P.m[8 + i] * c;
            xyz[3 * pos + i] = (float)s;
        }
        rgb_out[3 * pos] = rgb[3 * p];
        rgb_out[3 * pos + 1] = rgb[3 * p + 1];
        rgb_out[3 * pos + 2] = rgb[3 * p + 2];
        ++pos;
    }
    if (chunk == (int)gridDim.x - 1 && t == 255) *total = pos;
}

hipError_t launch_remove_occluded(const float *D, const uint8_t *B, int32_t H,
                                  int32_t W, int32_t k, double tau,
                                  uint8_t *Bout, hipStream_t s) {
    const int tiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    k_remove_occluded<<<tiles, 256, 0, s>>>(D, B, H, W, k, tau, Bout);
    return hipGetLastError();
}

size_t backproject_ws_bytes(int32_t H, int32_t W) {
    const int64_t chunks = ((int64_t)H * W + kCloudChunk - 1) / kCloudChunk;
    return align256((size_t)chunks * 4);
}

hipError_t launch_backproject(const float *D, const uint8_t *M, const uint8_t *rgb,
                              int32_t H, int32_t W, const Pose &P, const Intr &K,
                              double tau, float *xyz, uint8_t *rgb_out,
                              int64_t *total, void *ws, hipStream_t s) {
    const int64_t chunks = ((int64_t)H * W + kCloudChunk - 1) / kCloudChunk;
    int *counts = static_cast<int *>(ws);
    k_cloud_count<<<(int)chunks, 256, 0, s>>>(D, M, H, W, tau, counts);
    k_cloud_write<<<(int)chunks, 256, 0, s>>>(D, M, rgb, H, W, P, K, tau, counts,
                                              xyz, rgb_out, total);
    return hipGetLastError();
}

}  // namespace jbfd

namespace jbfd {

// ---------------------------------------------------------------------------
// afterimage removal: closed motion mask (Sec. 4.1)
// ---------------------------------------------------------------------------

// raw[p] = squared RGB distance between the frames > tau^2 (in double)
__global__ __launch_bounds__(256) void k_motion_raw(const uint8_t *__restrict__ a,
                                                    const uint8_t *__restrict__ b,
                                                    int64_t n, double tau2,
                                                    uint8_t *__restrict__ raw) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        int c = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const int d = (int)a[3 * p + ch] - (int)b[3 * p + ch];
            c += d * d;
        }
        raw[p] = (uint8_t)((double)c > tau2);
    }
}

// One separable pass of the square closing over the in-image part of each
// window, along rows (ROWS) or columns: OR (dilation) or AND (erosion).
template <bool ROWS, bool OR>
__global__ __launch_bounds__(256) void k_morph_pass(const uint8_t *__restrict__ in,
                                                    int H, int W, int k,
                                                    uint8_t *__restrict__ out) {
    const int64_t n = (int64_t)H * W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const int c = ROWS ? x : y, len = ROWS ? W : H;
        const int lo = max(c - k, 0), hi = min(c + k, len - 1);
        uint8_t r = OR ? 0 : 1;
        for (int j = lo; j <= hi; ++j) {
            const uint8_t v = ROWS ? in[(int64_t)y * W + j] : in[(int64_t)j * W + x];
            r = OR ? (uint8_t)(r | v) : (uint8_t)(r & v);
        }
        out[p] = r;
    }
}

size_t motion_mask_ws_bytes(int32_t H, int32_t W) {
    return 2 * align256((size_t)H * W);
}

hipError_t launch_motion_mask(const uint8_t *rgb, const uint8_t *rgb_prev,
                              int32_t H, int32_t W, double tau, int32_t k,
                              uint8_t *mask, void *ws, hipStream_t s) {
    const int64_t n = (int64_t)H * W;
    uint8_t *t0 = static_cast<uint8_t *>(ws);
    uint8_t *t1 = t0 + align256((size_t)n);
    int64_t g = (n + 255) / 256;
    const int grid = (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
    k_motion_raw<<<grid, 256, 0, s>>>(rgb, rgb_prev, n, tau * tau, t0);
    k_morph_pass<true, true><<<grid, 256, 0, s>>>(t0, H, W, k, t1);    // dilate rows
    k_morph_pass<false, true><<<grid, 256, 0, s>>>(t1, H, W, k, t0);   // dilate cols
    k_morph_pass<true, false><<<grid, 256, 0, s>>>(t0, H, W, k, t1);   // erode rows
    k_morph_pass<false, false><<<grid, 256, 0, s>>>(t1, H, W, k, mask); // erode cols
    return hipGetLastError();
}

}  // namespace jbfd

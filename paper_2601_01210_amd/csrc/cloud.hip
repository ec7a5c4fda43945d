// Occluded-point removal (Sec. 4.1), contour removal with back-projection
// to a coloured world cloud (Sec. 5, Sec. 2), and the motion mask of
// afterimage removal (Sec. 4.1).
//
//   k_remove_occluded  one workgroup per 64 x 16 output tile; depth (0 where
//                      invalid) and validity of the tile plus a k-pixel halo
//                      are staged in LDS; a valid pixel sums the valid
//                      depths of its (2k+1)^2 window in double, in row-major
//                      order, and keeps its sample unless
//                      D - mean > tau * mean (in double);
//   k_cloud_count      1024-pixel chunks of the row-major pixel order, four
//                      consecutive pixels per thread: the contour rule
//                      (largest jump to a valid 4-neighbour, in double, at
//                      most tau * D) for each valid pixel; the four keep
//                      bits go to a workspace byte and the chunk's count to
//                      the chunk table;
//   k_cloud_write      each chunk sums the counts of the chunks before it,
//                      ranks its kept pixels by a block scan (so the output
//                      keeps row-major order), computes each one's world
//                      point, R^T (p_c - t) with p_c through the pixel
//                      centre, in double with a fixed operation order (no
//                      contraction) rounded once to float, stages points and
//                      colours in LDS and writes them with coalesced stores.
//                      The last chunk writes the total;
//   k_motion_mask      one workgroup per output tile; the closed motion mask.
//
// Every global load is issued from a clamped address with no branch around
// it, so a thread's loads are in flight together.
#include "filter_common.hpp"

namespace jbfd {

constexpr int kOccMaxK = 8;
constexpr int kOccCols = 64, kOccRows = 16;
constexpr int kCloudChunk = 1024;

template <int K>
__global__ __launch_bounds__(256) void k_remove_occluded(
    const float *__restrict__ D, const uint8_t *__restrict__ B, int H, int W,
    double tau, uint8_t *__restrict__ Bout) {
    constexpr int EW = kOccCols + 2 * K, EH = kOccRows + 2 * K;
    // (depth, valid) per pixel of the tile plus halo; depth 0 and valid 0
    // outside the image and at invalid pixels. One extra record takes the
    // stores of lanes that have no element, so no branch guards the loads.
    __shared__ float2 s[EH * EW + 1];
    const int x0 = blockIdx.x * kOccCols - K, y0 = blockIdx.y * kOccRows - K;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i2 = min(tx + 64, EW - 1);
    const int xa = min(max(x0 + tx, 0), W - 1), xb = min(max(x0 + i2, 0), W - 1);
    const bool xina = x0 + tx >= 0 && x0 + tx < W;
    const bool xinb = x0 + i2 >= 0 && x0 + i2 < W;
    constexpr int NIT = (EH + 3) / 4;
    uint8_t va[NIT], vb[NIT];
    float da[NIT], db[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int y = y0 + min(ty + 4 * it, EH - 1);
        const int64_t row = (int64_t)min(max(y, 0), H - 1) * W;
        va[it] = B[row + xa];
        da[it] = D[row + xa];
        vb[it] = B[row + xb];
        db[it] = D[row + xb];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int j = ty + 4 * it;
        const int y = y0 + j;
        const bool yin = y >= 0 && y < H && j < EH;
        const bool ina = yin && xina && va[it] != 0;
        const bool inb = yin && xinb && vb[it] != 0;
        const int ea = j < EH ? j * EW + tx : EH * EW;
        const int eb = j < EH && tx + 64 < EW ? j * EW + i2 : EH * EW;
        s[ea] = make_float2(ina ? da[it] : 0.0f, ina ? 1.0f : 0.0f);
        s[eb] = make_float2(inb ? db[it] : 0.0f, inb ? 1.0f : 0.0f);
    }
    __syncthreads();
    const int x = x0 + K + tx;
#pragma unroll
    for (int q = 0; q < kOccRows / 4; ++q) {
        const int ly = ty + 4 * q;
        const int y = y0 + K + ly;
        if (x >= W || y >= H) continue;
        const int c = (ly + K) * EW + tx + K;
        const float2 me = s[c];
        // the window's valid depths summed in row-major order; adding +0.0
        // for an invalid tap leaves the sum unchanged (it starts at +0.0 and
        // so never holds -0.0)
        double sum = 0.0;
        float n = 0.0f;
#pragma unroll
        for (int dy = -K; dy <= K; ++dy) {
#pragma unroll
            for (int dx = -K; dx <= K; ++dx) {
                const float2 v = s[c + dy * EW + dx];
                sum = sum + (double)v.x;
                n += v.y;
            }
        }
        const double mean = sum / (double)n;
        const bool keep = me.y != 0.0f && !((double)me.x - mean > tau * mean);
        Bout[(int64_t)y * W + x] = (uint8_t)keep;
    }
}

// Keep bits (bit u for pixel p0 + u) of the four pixels p0 .. p0+3 under
// the contour rule: largest |D(n) - D(p)| over valid in-image
// 4-neighbours, in double, at most tau * D(p). Pixels at or past npix get 0.
__device__ inline uint32_t contour_bits(const float *__restrict__ D,
                                        const uint8_t *__restrict__ M, int H,
                                        int W, uint32_t npix, uint32_t p0,
                                        double tau) {
    const uint32_t last = npix - 1;
    float dr[6], du[4], dd[4];
    uint8_t mr[6], mu[4], md[4];
    // the row strip p0-1 .. p0+4, and the pixels one row up and down
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const uint32_t q = min(p0 + e > 0 ? p0 + e - 1 : 0u, last);
        dr[e] = D[q];
        mr[e] = M[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t p = min(p0 + u, last);
        const uint32_t qu = p >= (uint32_t)W ? p - W : p;
        const uint32_t qd = p + W <= last ? p + W : p;
        du[u] = D[qu];
        mu[u] = M[qu];
        dd[u] = D[qd];
        md[u] = M[qd];
    }
    uint32_t bits = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t p = p0 + u;
        if (p >= npix || !mr[u + 1]) continue;
        const uint32_t y = p / (uint32_t)W, x = p - y * (uint32_t)W;
        const double z = (double)dr[u + 1];
        double g = 0.0;
        if (x + 1 < (uint32_t)W && mr[u + 2])
            g = fmax(g, __builtin_fabs((double)dr[u + 2] - z));
        if (x > 0 && mr[u])
            g = fmax(g, __builtin_fabs((double)dr[u] - z));
        if (y + 1 < (uint32_t)H && md[u])
            g = fmax(g, __builtin_fabs((double)dd[u] - z));
        if (y > 0 && mu[u])
            g = fmax(g, __builtin_fabs((double)du[u] - z));
        if (!(g > tau * z)) bits |= 1u << u;
    }
    return bits;
}

__global__ __launch_bounds__(256) void k_cloud_count(const float *__restrict__ D,
                                                     const uint8_t *__restrict__ M,
                                                     int H, int W, double tau,
                                                     int *__restrict__ counts,
                                                     uint8_t *__restrict__ keep) {
    __shared__ int part[4];
    const uint32_t npix = (uint32_t)H * (uint32_t)W;
    const uint32_t p0 = (uint32_t)blockIdx.x * kCloudChunk + 4u * threadIdx.x;
    const uint32_t bits = contour_bits(D, M, H, W, npix, p0, tau);
    keep[(size_t)blockIdx.x * 256 + threadIdx.x] = (uint8_t)bits;
    const int cnt = wave_sum(__builtin_popcount(bits));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ __launch_bounds__(256) void k_cloud_write(
    const float *__restrict__ D, const uint8_t *__restrict__ rgb, int H, int W,
    Pose P, Intr K, const int *__restrict__ counts,
    const uint8_t *__restrict__ keep, float *__restrict__ xyz,
    uint8_t *__restrict__ rgb_out, int64_t *__restrict__ total) {
    __shared__ float sxyz[3 * kCloudChunk];
    __shared__ uint8_t srgb[3 * kCloudChunk];
    __shared__ int wsum[4];
    __shared__ int64_t wacc[4];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int chunk = blockIdx.x;
    const uint32_t npix = (uint32_t)H * (uint32_t)W, last = npix - 1;
    const uint32_t p0 = (uint32_t)chunk * kCloudChunk + 4u * t;
    const uint32_t bits = keep[(size_t)chunk * 256 + t];
    float z4[4];
    uint8_t c12[12];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t p = min(p0 + u, last);
        z4[u] = D[p];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) c12[3 * u + ch] = rgb[3 * (size_t)p + ch];
    }
    // points of all earlier chunks (in all at most H*W < 2^31): the counts
    // of the first 2048 chunks are loaded together (Full-HD has 2025),
    // later ones in further batches
    int acc = 0;
    {
        int a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = 256 * u + t;
            a[u] = counts[c < chunk ? c : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += 256 * u + t < chunk ? a[u] : 0;
        for (int c0 = 8 * 256; c0 < chunk; c0 += 8 * 256) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + 256 * u + t;
                a[u] = counts[c < chunk ? c : 0];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += c0 + 256 * u + t < chunk ? a[u] : 0;
        }
    }
    acc = wave_sum(acc);
    const int cnt = __builtin_popcount(bits);
    const int incl = wave_inclusive_scan(cnt);
    if (lane == 0) wacc[wid] = acc;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    const int64_t before = wacc[0] + wacc[1] + wacc[2] + wacc[3];
    int r = incl - cnt;
    for (int w = 0; w < wid; ++w) r += wsum[w];
    const int n_chunk = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (!((bits >> u) & 1u)) continue;
        const uint32_t p = p0 + u;
        const uint32_t y = p / (uint32_t)W, x = p - y * (uint32_t)W;
        const double Z = (double)z4[u];
        const double Xc = ((double)x + 0.5 - K.cx) * Z / K.fx;
        const double Yc = ((double)y + 0.5 - K.cy) * Z / K.fy;
        const double a = Xc - P.m[3], b = Yc - P.m[7], c = Z - P.m[11];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double sacc = P.m[0 + i] * a;
            sacc = sacc + P.m[4 + i] * b;
            sacc = sacc + P.m[8 + i] * c;
            sxyz[3 * r + i] = (float)sacc;
            srgb[3 * r + i] = c12[3 * u + i];
        }
        ++r;
    }
    __syncthreads();
    float *dst = xyz + 3 * before;
    uint8_t *cdst = rgb_out + 3 * before;
    for (int e = t; e < 3 * n_chunk; e += 256) {
        dst[e] = sxyz[e];
        cdst[e] = srgb[e];
    }
    if (chunk == (int)gridDim.x - 1 && t == 0) *total = before + n_chunk;
}

hipError_t launch_remove_occluded(const float *D, const uint8_t *B, int32_t H,
                                  int32_t W, int32_t k, double tau,
                                  uint8_t *Bout, hipStream_t s) {
    const dim3 grid((W + kOccCols - 1) / kOccCols, (H + kOccRows - 1) / kOccRows);
    switch (k) {
#define JBFD_OCC_CASE(KK)                                                      \
    case KK:                                                                   \
        k_remove_occluded<KK><<<grid, 256, 0, s>>>(D, B, H, W, tau, Bout);     \
        break;
        JBFD_OCC_CASE(0) JBFD_OCC_CASE(1) JBFD_OCC_CASE(2) JBFD_OCC_CASE(3)
        JBFD_OCC_CASE(4) JBFD_OCC_CASE(5) JBFD_OCC_CASE(6) JBFD_OCC_CASE(7)
        JBFD_OCC_CASE(8)
#undef JBFD_OCC_CASE
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kOccMaxK == 8, "one instantiation per window size");
    return hipGetLastError();
}

struct CloudLayout {
    size_t counts, keep, total;
};

static CloudLayout cloud_layout(int32_t H, int32_t W) {
    const size_t chunks = ((size_t)H * W + kCloudChunk - 1) / kCloudChunk;
    CloudLayout L;
    L.counts = 0;
    L.keep = align256(chunks * 4);
    L.total = L.keep + align256(chunks * 256);
    return L;
}

size_t backproject_ws_bytes(int32_t H, int32_t W) { return cloud_layout(H, W).total; }

hipError_t launch_backproject(const float *D, const uint8_t *M, const uint8_t *rgb,
                              int32_t H, int32_t W, const Pose &P, const Intr &K,
                              double tau, float *xyz, uint8_t *rgb_out,
                              int64_t *total, void *ws, hipStream_t s) {
    const int64_t chunks = ((int64_t)H * W + kCloudChunk - 1) / kCloudChunk;
    const CloudLayout L = cloud_layout(H, W);
    unsigned char *base = static_cast<unsigned char *>(ws);
    int *counts = reinterpret_cast<int *>(base + L.counts);
    uint8_t *keep = base + L.keep;
    k_cloud_count<<<(int)chunks, 256, 0, s>>>(D, M, H, W, tau, counts, keep);
    k_cloud_write<<<(int)chunks, 256, 0, s>>>(D, rgb, H, W, P, K, counts, keep,
                                              xyz, rgb_out, total);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// afterimage removal: closed motion mask (Sec. 4.1)
// ---------------------------------------------------------------------------

constexpr int kMotionRows = 32;                 // output rows per workgroup
constexpr int kMotionMaxK = 16;

// Output tile width for closing size k: the staged region is the tile plus
// 2k pixels on each side (dilation then erosion), 64 or 128 bytes wide.
__host__ __device__ constexpr int motion_tile_w(int k) {
    return (4 * k <= 32 ? 64 : 128) - 4 * k;
}

// One workgroup per TW x kMotionRows output tile. The raw motion bits of
// the tile plus a 2k halo go to LDS (pixels outside the image are still),
// then four separable passes of the square closing run in LDS: dilation
// along rows and columns, out-of-image pixels set to moving, erosion along
// rows and columns. Square windows factor into a row and a column pass, and
// the in-image restriction of a window factors the same way, so this equals
// the closing over each window's in-image pixels.
template <int k>
__global__ __launch_bounds__(256) void k_motion_mask(const uint8_t *__restrict__ a,
                                                     const uint8_t *__restrict__ b,
                                                     int H, int W, double tau2,
                                                     uint8_t *__restrict__ mask) {
    constexpr int TW = motion_tile_w(k);
    constexpr int RW = TW + 4 * k, RH = kMotionRows + 4 * k;
    __shared__ __align__(4) uint8_t A[RH * RW];
    __shared__ __align__(4) uint8_t Bf[RH * RW];
    const int x0 = blockIdx.x * TW - 2 * k, y0 = blockIdx.y * kMotionRows - 2 * k;
    constexpr int lw = RW == 64 ? 6 : 7;
    constexpr int n_el = RH * RW;
    // raw bits, kBatch elements per thread at a time with all their loads
    // issued together (clamped addresses, no branch around them); a lane
    // past the region repeats the last element, value included
    constexpr int kBatch = 8;
    for (int base = 0; base < n_el; base += 256 * kBatch) {
        uint8_t ca[kBatch][3], cb[kBatch][3];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = min(base + (int)threadIdx.x + 256 * u, n_el - 1);
            const int y = min(max(y0 + (e >> lw), 0), H - 1);
            const int x = min(max(x0 + (e & (RW - 1)), 0), W - 1);
            const int64_t p = 3 * ((int64_t)y * W + x);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                ca[u][ch] = a[p + ch];
                cb[u][ch] = b[p + ch];
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = min(base + (int)threadIdx.x + 256 * u, n_el - 1);
            const int y = y0 + (e >> lw), x = x0 + (e & (RW - 1));
            int c = 0;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const int d = (int)ca[u][ch] - (int)cb[u][ch];
                c += d * d;
            }
            const bool in = y >= 0 && y < H && x >= 0 && x < W;
            A[e] = (uint8_t)(in && (double)c > tau2);
        }
    }
    __syncthreads();
    // The closing on 32-bit words of four 0/1 bytes: OR / AND of bytes is
    // OR / AND of words, a row shift by d bytes is one alignbyte of two
    // neighbouring words, and a column step is a word read RW/4 words away.
    // Words at the region's edges read clamped neighbours; the bytes that
    // makes wrong lie outside the columns every later pass reads.
    constexpr int NW = RW / 4;                // words per row
    constexpr int Q = (k + 3) / 4;            // neighbour words a shift reaches
    const uint32_t *A4 = reinterpret_cast<const uint32_t *>(A);
    const uint32_t *B4 = reinterpret_cast<const uint32_t *>(Bf);
    uint32_t *A4w = reinterpret_cast<uint32_t *>(A);
    uint32_t *B4w = reinterpret_cast<uint32_t *>(Bf);
    // OR (dilate) or AND (erode) of the row shifts -k..k of word g of row j
    auto row_pass = [&](const uint32_t *src, int j, int g, bool dilate) {
        uint32_t w[2 * Q + 2];
#pragma unroll
        for (int m = 0; m < 2 * Q + 2; ++m)
            w[m] = src[j * NW + min(max(g - Q + m, 0), NW - 1)];
        uint32_t r = dilate ? 0u : ~0u;
#pragma unroll
        for (int d = -k; d <= k; ++d) {
            // bytes 4g + d .. 4g + d + 3
            const int m = (d + 4 * Q) >> 2, sh = (d + 4 * Q) & 3;
            const uint32_t v = sh == 0 ? w[m]
                                       : __builtin_amdgcn_alignbyte(w[m + 1], w[m], sh);
            r = dilate ? (r | v) : (r & v);
        }
        return r;
    };
    constexpr int ROWS_IT = (RH + 256 / NW - 1) / (256 / NW);
    const int wg = threadIdx.x % NW, wr = threadIdx.x / NW;   // word, row slot
    constexpr int RSTEP = 256 / NW;
#pragma unroll
    for (int it = 0; it < ROWS_IT; ++it) {                 // dilate along rows
        const int j = wr + RSTEP * it;
        if (j < RH) B4w[j * NW + wg] = row_pass(A4, j, wg, true);
    }
    __syncthreads();
    const int gx = x0 + 4 * wg;              // image column of the word's byte 0
    uint32_t outside_x = 0;                  // bytes of the word outside the image
#pragma unroll
    for (int b = 0; b < 4; ++b)
        outside_x |= (gx + b < 0 || gx + b >= W) ? (0xFFu << (8 * b)) : 0u;
#pragma unroll
    for (int it = 0; it < ROWS_IT; ++it) {                 // dilate along columns
        const int j = wr + RSTEP * it;
        if (j >= k && j < RH - k) {
            uint32_t r = 0;
#pragma unroll
            for (int d = -k; d <= k; ++d) r |= B4[(j + d) * NW + wg];
            const int y = y0 + j;
            const uint32_t out = (y < 0 || y >= H) ? ~0u : outside_x;
            A4w[j * NW + wg] = r | (out & 0x01010101u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ROWS_IT; ++it) {                 // erode along rows
        const int j = wr + RSTEP * it;
        if (j >= k && j < RH - k) B4w[j * NW + wg] = row_pass(A4, j, wg, false);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ROWS_IT; ++it) {                 // erode along columns
        const int j = wr + RSTEP * it;
        const int y = y0 + j;
        if (j >= 2 * k && j < RH - 2 * k && y < H) {
            uint32_t r = ~0u;
#pragma unroll
            for (int d = -k; d <= k; ++d) r &= B4[(j + d) * NW + wg];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = 4 * wg + b;     // column in the region
                if (i >= 2 * k && i < RW - 2 * k && gx + b < W)
                    mask[(int64_t)y * W + gx + b] = (uint8_t)((r >> (8 * b)) & 1u);
            }
        }
    }
}

hipError_t launch_motion_mask(const uint8_t *rgb, const uint8_t *rgb_prev,
                              int32_t H, int32_t W, double tau, int32_t k,
                              uint8_t *mask, hipStream_t s) {
    if (k < 0 || k > kMotionMaxK) return hipErrorInvalidValue;
    const int TW = motion_tile_w(k);
    const dim3 grid((W + TW - 1) / TW, (H + kMotionRows - 1) / kMotionRows);
    const double tau2 = tau * tau;
    switch (k) {
#define JBFD_MOTION_CASE(KK)                                                   \
    case KK:                                                                   \
        k_motion_mask<KK><<<grid, 256, 0, s>>>(rgb, rgb_prev, H, W, tau2, mask); \
        break;
        JBFD_MOTION_CASE(0) JBFD_MOTION_CASE(1) JBFD_MOTION_CASE(2)
        JBFD_MOTION_CASE(3) JBFD_MOTION_CASE(4) JBFD_MOTION_CASE(5)
        JBFD_MOTION_CASE(6) JBFD_MOTION_CASE(7) JBFD_MOTION_CASE(8)
        JBFD_MOTION_CASE(9) JBFD_MOTION_CASE(10) JBFD_MOTION_CASE(11)
        JBFD_MOTION_CASE(12) JBFD_MOTION_CASE(13) JBFD_MOTION_CASE(14)
        JBFD_MOTION_CASE(15) JBFD_MOTION_CASE(16)
#undef JBFD_MOTION_CASE
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kMotionMaxK == 16, "one instantiation per closing size");
    return hipGetLastError();
}

}  // namespace jbfd

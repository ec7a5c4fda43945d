// Two-stage filtering (Sec. 5): the sparse depth image is pooled to a third
// of its resolution in each dimension, filtered there, restored to full
// resolution and filtered again with a small radius.
//
//   k_pool3          one thread per 3x3 cell: valid-average depth (summed in
//                    double in row-major order, rounded once to float), cell
//                    validity, rounded mean colour floor((sum + n/2) / n);
//   k_restore_merge  one thread per pixel: the original depth where the
//                    pixel holds a sample, else the first pass's output of
//                    its cell (x/3, y/3) where that is valid;
//   k_jbf_dense<R,T,RPT> the joint bilateral filter (Eq. 1-4) for inputs
//                    where most pixels hold a sample and the radius is small:
//                    one thread per RPT output pixels loops over every tap of
//                    their (2R+1)^2 windows, read from a tile plus halo staged
//                    in LDS (16 x 32 pixels with two per thread, or 8 x 8 on
//                    small images). After pooling and
//                    restoring, nearly every window tap is valid, so a
//                    wave-uniform walk over sample lists (the sparse kernel)
//                    would spend most of its lanes outside the small windows.
//
// Weights of k_jbf_dense follow the sparse kernel's pass 1 exactly (same
// exponent form and clamps: colour part max(2 kr t - kr|p|^2, -60) with
// t = p.q - |q|^2/2 from f16 channel values, spatial part
// max(-ks (dx^2+dy^2), -60)), so every in-window sample has a weight of at
// least 2^-120 and den > 0 is exactly the mask; lanes whose weight sum ends
// below 2^-16 are recomputed with the exact running shift of the sparse
// kernel's pass 2. A tile record is {(r,g) f16x2, (b, valid) f16x2, depth,
// -|q|^2/2}; the valid flag in the upper half of the second word multiplies
// the weight into den through one mixed-precision fma, and invalid pixels
// carry depth 0, so they add nothing to either sum.
#include "filter_common.hpp"

namespace jbfd {

// One thread per cell; grid (ceil(W1 / 256), H1). The nine pixels are read
// from clamped addresses with every load issued before any is used; the
// cell's in-image pixels are then taken in row-major order (adding +0.0 for
// a pixel without a sample leaves the double sum unchanged: it starts at
// +0.0 and so never holds -0.0).
__global__ __launch_bounds__(256) void k_pool3(const float *__restrict__ D,
                                               const uint8_t *__restrict__ B,
                                               const uint8_t *__restrict__ rgb,
                                               int H, int W,
                                               float *__restrict__ D1,
                                               uint8_t *__restrict__ B1,
                                               uint8_t *__restrict__ rgb1) {
    const int W1 = (W + 2) / 3;
    const int cy = blockIdx.y, cx = blockIdx.x * 256 + threadIdx.x;
    if (cx >= W1) return;
    float d[9];
    uint8_t v[9], c[9][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const int64_t row = (int64_t)min(3 * cy + dy, H - 1) * W;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int64_t p = row + min(3 * cx + dx, W - 1);
            d[3 * dy + dx] = D[p];
            v[3 * dy + dx] = B[p];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) c[3 * dy + dx][ch] = rgb[3 * p + ch];
        }
    }
    double sum = 0.0;
    int n_valid = 0, n_pix = 0;
    int c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int e = 3 * dy + dx;
            const bool in = 3 * cy + dy < H && 3 * cx + dx < W;
            const bool use = in && v[e] != 0;
            n_pix += in;
            c0 += in ? c[e][0] : 0;
            c1 += in ? c[e][1] : 0;
            c2 += in ? c[e][2] : 0;
            sum = sum + (use ? (double)d[e] : 0.0);
            n_valid += use;
        }
    }
    const int64_t q = (int64_t)cy * W1 + cx;
    D1[q] = n_valid ? (float)(sum / (double)n_valid) : 0.0f;
    B1[q] = (uint8_t)(n_valid > 0);
    rgb1[3 * q] = (uint8_t)((c0 + n_pix / 2) / n_pix);
    rgb1[3 * q + 1] = (uint8_t)((c1 + n_pix / 2) / n_pix);
    rgb1[3 * q + 2] = (uint8_t)((c2 + n_pix / 2) / n_pix);
}

// One thread per pixel; grid (ceil(W / 256), H).
__global__ __launch_bounds__(256) void k_restore_merge(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const float *__restrict__ O1, const uint8_t *__restrict__ M1, int H, int W,
    float *__restrict__ D2, uint8_t *__restrict__ B2) {
    const int W1 = (W + 2) / 3;
    const int y = blockIdx.y, x = blockIdx.x * 256 + threadIdx.x;
    if (x >= W || y >= H) return;
    const int64_t p = (int64_t)y * W + x;
    const int64_t q = (int64_t)(y / 3) * W1 + x / 3;
    const uint8_t own_v = B[p], up_v = M1[q];
    const float d = D[p], o = O1[q];
    const bool own = own_v != 0, up = up_v != 0;
    D2[p] = own ? d : (up ? o : 0.0f);
    B2[p] = (uint8_t)(own || up);
}

// Exact pass of one pixel whose weights are all tiny (far colours or tiny
// sigma_s): running shift, exact unclamped spatial exponents; row0 is the
// tile row of the window's top edge.
template <int R, int EX>
__device__ __forceinline__ void dense_exact(const uint4 *tile, int row0, int lx,
                                            uint32_t prg, uint32_t pb0, float p2,
                                            const FilterParams &fp, float &num,
                                            float &den) {
    const float kr2 = 2.0f * fp.kr;
    float M = kShiftInit - fp.kr * p2, n2 = 0.0f, d2 = 0.0f;
    for (int dy = -R; dy <= R; ++dy) {
        for (int dx = -R; dx <= R; ++dx) {
            const uint4 q = tile[(row0 + R + dy) * EX + lx + R + dx];
            if ((q.y >> 16) == 0u) continue;
            const float tq = dot2h(prg, q.x, dot2h(pb0, q.y, __uint_as_float(q.w)));
            consume1(tq, -fp.ks * (float)(dx * dx + dy * dy), __uint_as_float(q.z),
                     kr2, M, n2, d2);
        }
    }
    num = n2;
    den = d2;
}

// Filter of one T x (RPT T) tile (see the file comment): T x T threads, each
// for RPT vertically adjacent pixels. With RPT = 2 a thread reads each of
// the 2R + 2 window rows of its pixel pair from LDS once and applies it to
// both pixels, so the tile reads per pixel drop from (2R+1)^2 to
// (2R+2)(2R+1)/2; each pixel still takes its taps row by row, left to
// right. T = 16 with RPT = 2 on large images, T = 8 with RPT = 1 on images
// too small to give every CU several workgroups. With RESTORE the kernel
// stages the restored input of the two-stage filter's second pass itself:
// a pixel's own depth where it holds a sample, else the first pass's output
// O1 of its cell (x/3, y/3) where that is valid (M1), the values
// k_restore_merge would have stored.
template <int R, int T, int RPT, bool RESTORE>
__global__ __launch_bounds__(T * T) void k_jbf_dense(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int n_tiles, int n_pad, float *__restrict__ out,
    uint8_t *__restrict__ mask, const float *__restrict__ O1,
    const uint8_t *__restrict__ M1) {
    static_assert(RPT == 1 || RPT == 2, "one or two rows per thread");
    constexpr int EX = T + 2 * R;             // tile width with halo
    constexpr int EY = RPT * T + 2 * R;       // tile height with halo
    constexpr int NE = EX * EY;
    constexpr int NT = T * T;                 // threads
    __shared__ uint4 tile[NE + 1];
    const int t = xcd_tile(blockIdx.x, n_pad);
    if (t >= n_tiles) return;                 // whole workgroup leaves together
    const int ty0 = (t / tiles_x) * (RPT * T), tx0 = (t % tiles_x) * T;

    // stage the tile and its halo: invalid and out-of-image pixels get a
    // zero depth and a zero valid flag. Every element's loads come from a
    // clamped address and are issued before any is used; elements past the
    // tile store into one spare record.
    constexpr int NIT = (NE + NT - 1) / NT;
    uint8_t cr[NIT][3], cv[NIT], cm[NIT];
    float cd[NIT], co[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = min((int)threadIdx.x + NT * it, NE - 1);
        const int ly = e / EX, lx = e - ly * EX;
        const int y = min(max(ty0 - R + ly, 0), H - 1);
        const int x = min(max(tx0 - R + lx, 0), W - 1);
        const int64_t p = (int64_t)y * W + x;
        cr[it][0] = rgb[3 * p];
        cr[it][1] = rgb[3 * p + 1];
        cr[it][2] = rgb[3 * p + 2];
        cv[it] = B[p];
        cd[it] = D[p];
        if (RESTORE) {
            const int64_t q = (int64_t)(y / 3) * ((W + 2) / 3) + x / 3;
            cm[it] = M1[q];
            co[it] = O1[q];
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = (int)threadIdx.x + NT * it;
        const int ly = e / EX, lx = e - ly * EX;
        const int y = ty0 - R + ly, x = tx0 - R + lx;
        const bool in = e < NE && y >= 0 && y < H && x >= 0 && x < W;
        uint32_t rg, b0;
        float nq2h;
        colour_fields((uint32_t)cr[it][0] | ((uint32_t)cr[it][1] << 8), cr[it][2],
                      rg, b0, nq2h);
        const bool own = cv[it] != 0;
        const bool up = RESTORE && cm[it] != 0;
        const bool v = in && (own || up);
        const float dv = own ? cd[it] : (up ? co[it] : 0.0f);
        // valid flag = f16 1.0 in the upper half of the (b, 0) word
        const uint4 rec = in ? make_uint4(rg, b0 | (v ? 0x3C000000u : 0u),
                                          __float_as_uint(v ? dv : 0.0f),
                                          __float_as_uint(nq2h))
                             : make_uint4(0u, 0u, 0u, 0u);
        tile[e < NE ? e : NE] = rec;
    }
    __syncthreads();

    const int lx = threadIdx.x % T, row0 = RPT * (int)(threadIdx.x / T);
    const int px = tx0 + lx, py = ty0 + row0;
    if (px >= W || py >= H) return;           // no barrier follows
    const bool has1 = RPT == 2 && py + 1 < H;
    uint32_t prg[RPT], pb0[RPT];
    float p2[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const uint4 me = tile[(row0 + j + R) * EX + lx + R];
        prg[j] = me.x;
        pb0[j] = me.y & 0xFFFFu;                 // (b, 0) for the dot
        p2[j] = -2.0f * __uint_as_float(me.w);
    }
    const float kr2 = 2.0f * fp.kr;
    const Pass1Exp p1a(kr2, -fp.kr * p2[0]), p1b(kr2, -fp.kr * p2[RPT - 1]);

    // spatial exponents of the distinct squared distances, clamped as in
    // the sparse kernel's table
    float gs[2 * R * R + 1];
#pragma unroll
    for (int s = 0; s <= 2 * R * R; ++s)
        gs[s] = fmaxf(-fp.ks * (float)s, kClampExp);

    float num[RPT], den[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) num[j] = den[j] = 0.0f;
    // window row k of the pixel group: row k - R of pixel 0, row k - R - 1
    // of pixel 1
#pragma unroll
    for (int k = 0; k < 2 * R + RPT; ++k) {
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            const uint4 q = tile[(row0 + k) * EX + lx + R + dx];
            const _Float16 vf = __builtin_bit_cast(h2, q.y)[1];
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int dy = k - R - j;
                if (dy < -R || dy > R) continue;
                const float tq =
                    dot2h(prg[j], q.x, dot2h(pb0[j], q.y, __uint_as_float(q.w)));
                const float a = (j == 0 ? p1a : p1b)(tq, gs[dx * dx + dy * dy]);
                const float w = __builtin_amdgcn_exp2f(a);
                num[j] = __builtin_fmaf(w, __uint_as_float(q.z), num[j]);
                den[j] = __builtin_fmaf(w, (float)vf, den[j]);
            }
        }
    }

#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (j == 1 && !has1) break;
        if (den[j] > 0.0f && den[j] < kWeakBelow)
            dense_exact<R, EX>(tile, row0 + j, lx, prg[j], pb0[j], p2[j], fp, num[j],
                               den[j]);
        const int64_t p = (int64_t)(py + j) * W + px;
        const bool ok = den[j] > 0.0f;
        out[p] = ok ? num[j] / den[j] : 0.0f;
        mask[p] = (uint8_t)ok;
    }
}

hipError_t launch_pool3(const float *D, const uint8_t *B, const uint8_t *rgb,
                        int32_t H, int32_t W, float *D1, uint8_t *B1,
                        uint8_t *rgb1, hipStream_t s) {
    const dim3 grid(((W + 2) / 3 + 255) / 256, (H + 2) / 3);
    k_pool3<<<grid, 256, 0, s>>>(D, B, rgb, H, W, D1, B1, rgb1);
    return hipGetLastError();
}

hipError_t launch_restore_merge(const float *D, const uint8_t *B,
                                const float *O1, const uint8_t *M1, int32_t H,
                                int32_t W, float *D2, uint8_t *B2,
                                hipStream_t s) {
    const dim3 grid((W + 255) / 256, H);
    k_restore_merge<<<grid, 256, 0, s>>>(D, B, O1, M1, H, W, D2, B2);
    return hipGetLastError();
}

hipError_t launch_densify_dense(const float *D, const uint8_t *B,
                                const uint8_t *rgb, int32_t H, int32_t W,
                                const FilterParams &fp, float *out,
                                uint8_t *mask, hipStream_t s, const float *O1,
                                const uint8_t *M1) {
    // 16x32 tiles (two rows per thread) when there are at least eight per
    // CU, else 8x8 tiles (one row per thread)
    const bool big = (int64_t)((W + 15) / 16) * ((H + 31) / 32) >= 2048;
    const bool restore = O1 != nullptr;
    const int T = big ? 16 : 8, TY = big ? 32 : 8;
    const int tiles_x = (W + T - 1) / T;
    const int tiles_y = (H + TY - 1) / TY;
    const int n_tiles = tiles_x * tiles_y;
    const int n_pad = (n_tiles + 7) & ~7;
#define JBFD_DENSE_LAUNCH(RR, TT, RP, RS, NTH)                                  \
    k_jbf_dense<RR, TT, RP, RS><<<n_pad, NTH, 0, s>>>(                         \
        D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, out, mask, O1, M1)
#define JBFD_DENSE_CASE(RR)                                                    \
    case RR:                                                                   \
        if (big && restore)                                                    \
            JBFD_DENSE_LAUNCH(RR, 16, 2, true, 256);                           \
        else if (big)                                                          \
            JBFD_DENSE_LAUNCH(RR, 16, 2, false, 256);                          \
        else if (restore)                                                      \
            JBFD_DENSE_LAUNCH(RR, 8, 1, true, 64);                             \
        else                                                                   \
            JBFD_DENSE_LAUNCH(RR, 8, 1, false, 64);                            \
        break;
    switch (fp.radius) {
        JBFD_DENSE_CASE(0) JBFD_DENSE_CASE(1) JBFD_DENSE_CASE(2)
        JBFD_DENSE_CASE(3) JBFD_DENSE_CASE(4)
    default:
        return hipErrorInvalidValue;
    }
#undef JBFD_DENSE_CASE
#undef JBFD_DENSE_LAUNCH
    return hipGetLastError();
}

// Intermediates of the two-stage filter inside the caller's workspace.
struct TwoStageLayout {
    size_t d1, b1, c1, o1, m1, d2, b2, total;
};

static TwoStageLayout two_stage_layout(int32_t H, int32_t W) {
    const size_t n1 = (size_t)((H + 2) / 3) * ((W + 2) / 3);
    const size_t n = (size_t)H * W;
    TwoStageLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.d1 = take(4 * n1);
    L.b1 = take(n1);
    L.c1 = take(3 * n1);
    L.o1 = take(4 * n1);
    L.m1 = take(n1);
    L.d2 = take(4 * n);
    L.b2 = take(n);
    L.total = off;
    return L;
}

size_t two_stage_ws_bytes(int32_t H, int32_t W) {
    return two_stage_layout(H, W).total;
}

hipError_t launch_two_stage(const float *D, const uint8_t *B, const uint8_t *rgb,
                            int32_t H, int32_t W, const FilterParams &f1,
                            const FilterParams &f2, float *out, uint8_t *mask,
                            void *ws, hipStream_t s) {
    const TwoStageLayout L = two_stage_layout(H, W);
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *D1 = reinterpret_cast<float *>(w + L.d1);
    uint8_t *B1 = w + L.b1;
    uint8_t *C1 = w + L.c1;
    float *O1 = reinterpret_cast<float *>(w + L.o1);
    uint8_t *M1 = w + L.m1;
    float *D2 = reinterpret_cast<float *>(w + L.d2);
    uint8_t *B2 = w + L.b2;
    const int32_t H1 = (H + 2) / 3, W1 = (W + 2) / 3;
    hipError_t e = launch_pool3(D, B, rgb, H, W, D1, B1, C1, s);
    if (e != hipSuccess) return e;
    e = f1.radius <= kDenseMaxRadius
            ? launch_densify_dense(D1, B1, C1, H1, W1, f1, O1, M1, s, nullptr,
                                   nullptr)
            : launch_densify(D1, B1, C1, H1, W1, f1, JBFD_FP32, O1, M1, nullptr,
                             nullptr, 0, false, s);
    if (e != hipSuccess) return e;
    // the dense kernel restores its input while staging its tiles; the
    // sparse kernel reads a restored image
    if (f2.radius <= kDenseMaxRadius)
        return launch_densify_dense(D, B, rgb, H, W, f2, out, mask, s, O1, M1);
    e = launch_restore_merge(D, B, O1, M1, H, W, D2, B2, s);
    if (e != hipSuccess) return e;
    return launch_densify(D2, B2, rgb, H, W, f2, JBFD_FP32, out, mask, nullptr,
                          nullptr, 0, false, s);
}

}  // namespace jbfd

// Backward of the joint bilateral filter (Sec. 4: the Gaussian widths are
// trainable by backpropagation; the input depths get gradients as well).
//
// With w_i the weights of the valid samples i in the window of output pixel
// x, W(x) = sum w_i and out(x) = sum w_i D_i / W(x):
//     dout(x)/dD_i      = w_i / W(x)
//     dout(x)/dsigma_r  = sum_i w_i c_i (D_i - out(x)) / (sigma_r^3 W(x))
//     dout(x)/dsigma_s  = sum_i w_i s_i (D_i - out(x)) / (sigma_s^3 W(x))
// (c_i squared colour distance, s_i squared pixel distance; in natural
// units dw/dsigma = w c / sigma^3). Every weight is recomputed from the
// forward's saved per-pixel shift and weight sum with exactly the forward's
// arithmetic, so the backward sees the very weights the forward summed.
//
//   k_jbf_bwd_sigma  one wave per 8x8 block of output pixels (the forward's
//                    walk over the halo samples); per-lane sums, a
//                    fixed-order wave reduction in double, one partial pair
//                    per wave;
//   k_jbf_bwd_depth  one wave per 8x8 block of sample pixels: gathers
//                    g(x) w(x,j) / W(x) over the output pixels x of its halo
//                    with g(x) != 0 (the window is symmetric, so this is the
//                    transpose of the forward's gather without atomics);
//   k_reduce_sigma   one workgroup sums the partials in a fixed order.
// All three are deterministic: two runs give identical bits.
#include "filter_common.hpp"

namespace jbfd {

namespace {

struct alignas(16) OutRec {
    uint32_t xy;   // x - (bx - r) | y << 16 of the output pixel
    uint32_t rg;   // its colour (r, g) as f16
    uint32_t b0;   // (b, 0) as f16
    float M;       // its weight shift (pass-1 pixels: their Pass1Exp lane constant)
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

template <int RMAX>
__global__ __launch_bounds__(256) void k_jbf_bwd_sigma(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int tiles_y, const float *__restrict__ out,
    const float2 *__restrict__ aux, const float *__restrict__ gout,
    float inv_sr3, float inv_ss3, double *__restrict__ partials) {
    constexpr int kTableMax = (2 * RMAX + 15) * table_stride(RMAX);
    __shared__ float G[kTableMax];
    __shared__ Rec recs[kWaves][64];
    __shared__ float nq2h[kWaves][64];

    const int r = fp.radius;
    const int ts = table_stride(r);
    int tx, ty;
    if (!column_tile(blockIdx.x, tiles_x, tiles_y, tx, ty)) return;
    build_table(G, r, ts, fp.ks, false);
    __syncthreads();

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int slot = (ty * tiles_x + tx) * kWaves + wid;
    const int bx = tx * kTile + (wid & 1) * 8;
    const int by = ty * kTile + (wid >> 1) * 8;
    const int i = lane & 7, j = lane >> 3;
    const int px = bx + i, py = by + j;
    const bool inside = px < W && py < H;
    const int64_t p = (int64_t)py * W + px;
    float gx = 0.0f, o = 0.0f;
    float2 ax = make_float2(0.0f, 0.0f);
    if (inside) {
        gx = gout[p];
        ax = aux[p];
        o = out[p];
    }
    const bool active = inside && ax.y != 0.0f && gx != 0.0f;
    if (bx >= W || by >= H || __builtin_amdgcn_ballot_w64(active) == 0) {
        if (lane == 0) {
            partials[2 * slot] = 0.0;
            partials[2 * slot + 1] = 0.0;
        }
        return;
    }

    float p2 = 0.0f;
    uint32_t prg = 0, pb0 = 0;
    if (inside) {
        const uint8_t *c = rgb + 3 * p;
        float nh;
        colour_fields((uint32_t)c[0] | ((uint32_t)c[1] << 8), c[2], prg, pb0, nh);
        p2 = -2.0f * nh;
    }
    const uint32_t lxy = (uint32_t)(i + 2 * r + 7) | ((uint32_t)(py + r + 7) << 16);
    const uint32_t gstride = 4u | ((uint32_t)(4 * ts) << 16);
    const float kr2 = 2.0f * fp.kr;
    const ListArgs none{nullptr, nullptr, 0};
    const BlockWalker bw{D, B, rgb, H, W, r, none, bx, by, lane, prg, pb0, lxy,
                         gstride, 0u, ts, reinterpret_cast<const unsigned char *>(G),
                         recs[wid], nq2h[wid], -fp.ks};

    // the forward's weight of this (pixel, sample) pair
    const bool pass1 = ax.y < 0.0f;
    const float M = ax.x;
    const Pass1Exp p1(kr2, M);
    float Ar = 0.0f, As = 0.0f;
    auto eat = [&](float t, float gtab, float d, uint32_t uv) {
        if (!active) return;
        float a;
        if (pass1)
            a = p1(t, gtab);
        else
            a = __builtin_fmaf(kr2, t, M) + bw.exact_g(uv);
        const float w = __builtin_amdgcn_exp2f(a);
        const float c = __builtin_fmaf(-2.0f, t, p2);       // exact integer
        const int dx = (int)(uv & 0xffffu) - r - 7, dy = (int)(uv >> 16) - r - 7;
        const float s = (float)(dx * dx + dy * dy);
        const float wd = w * (d - o);
        Ar = __builtin_fmaf(wd, c, Ar);
        As = __builtin_fmaf(wd, s, As);
    };
    bw.walk<false>(
        [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
            const uint32_t (&uv)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
        },
        eat);

    double cr = 0.0, cs = 0.0;
    if (active) {
        const double f = (double)gx / (double)fabsf(ax.y);
        cr = f * (double)Ar * (double)inv_sr3;
        cs = f * (double)As * (double)inv_ss3;
    }
    cr = wave_sum(cr);
    cs = wave_sum(cs);
    if (lane == 0) {
        partials[2 * slot] = cs;
        partials[2 * slot + 1] = cr;
    }
}

template <int RMAX>
__global__ __launch_bounds__(256) void k_jbf_bwd_depth(
    const uint8_t *__restrict__ B, const uint8_t *__restrict__ rgb, int H,
    int W, FilterParams fp, int tiles_x, int tiles_y,
    const float2 *__restrict__ aux, const float *__restrict__ gout,
    float *__restrict__ grad_d) {
    constexpr int kTableMax = (2 * RMAX + 15) * table_stride(RMAX);
    __shared__ float G[kTableMax];
    __shared__ OutRec orec[kWaves][64];
    __shared__ float coef[kWaves][64];
    __shared__ int first[kWaves][64];

    const int r = fp.radius;
    const int ts = table_stride(r);
    int tx, ty;
    if (!column_tile(blockIdx.x, tiles_x, tiles_y, tx, ty)) return;
    build_table(G, r, ts, fp.ks, false);
    __syncthreads();

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int bx = tx * kTile + (wid & 1) * 8;
    const int by = ty * kTile + (wid >> 1) * 8;
    const int i = lane & 7, j = lane >> 3;
    const int px = bx + i, py = by + j;
    const bool inside = px < W && py < H;
    if (bx >= W || by >= H) return;
    const int64_t p = (int64_t)py * W + px;
    const bool valid = inside && B[p] != 0;
    if (__builtin_amdgcn_ballot_w64(valid) == 0) {
        if (inside) grad_d[p] = 0.0f;
        return;
    }
    // this lane is sample j: its colour fields and -|q|^2/2
    uint32_t qrg = 0, qb0 = 0;
    float qn = 0.0f;
    if (inside) {
        const uint8_t *c = rgb + 3 * p;
        colour_fields((uint32_t)c[0] | ((uint32_t)c[1] << 8), c[2], qrg, qb0, qn);
    }
    const uint32_t lxy = (uint32_t)(i + 2 * r + 7) | ((uint32_t)(py + r + 7) << 16);
    const uint32_t gstride = 4u | ((uint32_t)(4 * ts) << 16);
    const unsigned char *Gb = reinterpret_cast<const unsigned char *>(G);
    const float kr2 = 2.0f * fp.kr, nks = -fp.ks;
    const float k1 = Pass1Exp(kr2, 0.0f).k;

    // the output pixels of the halo with a nonzero upstream gradient
    const int hx0 = max(bx - r, 0), hx1 = min(bx + 8 + r, W);
    const int hy0 = max(by - r, 0), hy1 = min(by + 8 + r, H);
    const int hw = hx1 - hx0;
    const int npx = hw * (hy1 - hy0);
    OutRec *my = orec[wid];
    float *myc = coef[wid];
    int *myf = first[wid];
    float grad = 0.0f;
    for (int base = 0; base < npx; base += 64) {
        const int k = base + lane;
        bool act = false;
        int64_t q = 0;
        int sx = 0, sy = 0;
        if (k < npx) {
            sx = hx0 + k % hw;
            sy = hy0 + k / hw;
            q = (int64_t)sy * W + sx;
            act = gout[q] != 0.0f && aux[q].y != 0.0f;
        }
        const uint64_t bal = __builtin_amdgcn_ballot_w64(act);
        if (bal == 0) continue;
        __builtin_amdgcn_wave_barrier();
        if (act) {
            const float2 ax = aux[q];
            const uint8_t *c = rgb + 3 * q;
            OutRec rec;
            float dummy;
            colour_fields((uint32_t)c[0] | ((uint32_t)c[1] << 8), c[2], rec.rg,
                          rec.b0, dummy);
            rec.xy = (uint32_t)(sx - (bx - r)) | ((uint32_t)sy << 16);
            // a pass-1 pixel's record carries its Pass1Exp lane constant
            rec.M = ax.y < 0.0f ? Pass1Exp::lane_c(ax.x) : ax.x;
            const int pos = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            my[pos] = rec;
            myc[pos] = gout[q] / fabsf(ax.y);
            myf[pos] = ax.y < 0.0f ? 1 : 0;
        }
        __builtin_amdgcn_wave_barrier();
        const int cnt = __builtin_popcountll(bal);
        for (int e = 0; e < cnt; ++e) {
            const OutRec o = my[e];
            const float t = dot2h(qrg, o.rg, dot2h(qb0, o.b0, qn));
            const uint32_t uv = pk_sub_u16(lxy, o.xy);
            float a;
            if (myf[e]) {
                const float g = *reinterpret_cast<const float *>(Gb + dot2_u16(uv, gstride, 0u));
                a = Pass1Exp::eval(k1, o.M, t, g);
            } else {
                const int dx = (int)(uv & 0xffffu) - r - 7, dy = (int)(uv >> 16) - r - 7;
                const bool in = dx >= -r && dx <= r && dy >= -r && dy <= r;
                const float g = in ? nks * (float)(dx * dx + dy * dy) : -__builtin_inff();
                a = __builtin_fmaf(kr2, t, o.M) + g;
            }
            grad = __builtin_fmaf(myc[e], __builtin_amdgcn_exp2f(a), grad);
        }
    }
    if (inside) grad_d[p] = valid ? grad : 0.0f;
}

__global__ __launch_bounds__(256) void k_reduce_sigma(const double *__restrict__ partials,
                                                      int n_slots,
                                                      double *__restrict__ grad_sigmas) {
    __shared__ double acc[2][256];
    double s = 0.0, r = 0.0;
    for (int k = threadIdx.x; k < n_slots; k += 256) {
        s += partials[2 * k];
        r += partials[2 * k + 1];
    }
    acc[0][threadIdx.x] = s;
    acc[1][threadIdx.x] = r;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            acc[0][threadIdx.x] += acc[0][threadIdx.x + off];
            acc[1][threadIdx.x] += acc[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grad_sigmas[0] = acc[0][0];
        grad_sigmas[1] = acc[1][0];
    }
}

static void tiles(int H, int W, int &tiles_x, int &tiles_y) {
    tiles_x = (W + kTile - 1) / kTile;
    tiles_y = (H + kTile - 1) / kTile;
}

size_t backward_ws_bytes(int32_t H, int32_t W) {
    int tiles_x, tiles_y;
    tiles(H, W, tiles_x, tiles_y);
    return (size_t)tiles_x * tiles_y * kWaves * 2 * sizeof(double);
}

hipError_t launch_densify_backward(const float *D, const uint8_t *B,
                                   const uint8_t *rgb, int32_t H, int32_t W,
                                   const FilterParams &fp, float sigma_s,
                                   float sigma_r, const float *out,
                                   const float *aux, const float *g,
                                   float *grad_d, double *grad_sigmas,
                                   void *ws, hipStream_t s) {
    int tiles_x, tiles_y;
    tiles(H, W, tiles_x, tiles_y);
    const int n_tiles = tiles_x * tiles_y, n_wg = column_grid(tiles_x, tiles_y);
    const float inv_sr3 =
        __builtin_isinf(sigma_r) ? 0.0f : (float)(1.0 / ((double)sigma_r * sigma_r * sigma_r));
    const float inv_ss3 =
        __builtin_isinf(sigma_s) ? 0.0f : (float)(1.0 / ((double)sigma_s * sigma_s * sigma_s));
    double *partials = static_cast<double *>(ws);
    const float2 *a2 = reinterpret_cast<const float2 *>(aux);
    if (fp.radius <= 16) {
        k_jbf_bwd_sigma<16><<<n_wg, 256, 0, s>>>(D, B, rgb, H, W, fp, tiles_x,
                                                tiles_y, out, a2, g, inv_sr3,
                                                inv_ss3, partials);
        k_jbf_bwd_depth<16><<<n_wg, 256, 0, s>>>(B, rgb, H, W, fp, tiles_x, tiles_y,
                                                a2, g, grad_d);
    } else {
        k_jbf_bwd_sigma<JBFD_MAX_RADIUS><<<n_wg, 256, 0, s>>>(
            D, B, rgb, H, W, fp, tiles_x, tiles_y, out, a2, g, inv_sr3,
            inv_ss3, partials);
        k_jbf_bwd_depth<JBFD_MAX_RADIUS><<<n_wg, 256, 0, s>>>(
            B, rgb, H, W, fp, tiles_x, tiles_y, a2, g, grad_d);
    }
    k_reduce_sigma<<<1, 256, 0, s>>>(partials, n_tiles * kWaves, grad_sigmas);
    return hipGetLastError();
}

}  // namespace jbfd

// Joint bilateral filter over a sparse depth image (Eq. 1-4; Algorithm 1's
// window and steps), gather form, one 64-lane wave per 8x8 output block.
//
// Algorithm 1 materialises a weight volume w(x,y,k) for every pixel and
// offset, then scatters D*w and B*w with a transpose convolution. Both
// sums only ever see offsets that hold a valid sample (B = 1), and the
// colour and spatial Gaussians are symmetric, so the same output is the
// gather over valid samples of each window. On a LiDAR image only a few
// percent of pixels are valid, so the kernel never touches an invalid tap:
//
//   1. Each wave streams the halo of its block ((8+2r)^2 pixels, clipped) in
//      chunks of 64 pixels, one per lane, and compacts the valid ones with a
//      ballot into a wave-private LDS list. The stream is software-pipelined:
//      the mask bytes of chunk c+2 and the sample data of chunk c+1 are
//      loaded while chunk c is processed. Records are 16 bytes
//      {halo xy (u16x2), (r,g) as f16x2, (b,0) as f16x2, depth (f32)} plus
//      -|rgb|^2/2 (f32) in a parallel array.
//   2. The wave then walks that list in lockstep: every lane (one output
//      pixel) reads the same record (LDS broadcast) and evaluates its
//      weight.
//        colour   t = p.q - |q|^2/2 by two v_dot2_f32_f16 on the 0..255
//                 channel values (every product and partial sum is an
//                 integer or half-integer below 2^23, so t is exact), and
//                 -kr c = 2 kr t - kr |p|^2 with the per-lane -kr |p|^2
//                 folded into the shift M;
//        space    a per-workgroup LDS table G[dy][dx] = -ks (dx^2+dy^2)
//                 inside the (2r+1)^2 window and -inf outside, indexed by
//                 one packed 16-bit subtract and one v_dot2_u32_u16, so the
//                 window test costs nothing;
//        weight   w = exp2(fma(2 kr, t, M) + G).
//   3. M starts at 2^23 - kr|p|^2 (on the half-integer grid) and is lowered
//      by whole integers k whenever a weight exponent would exceed +12; the
//      accumulators are then scaled by the exact power of two 2^-k and the
//      exponent is recomputed. Every weight of one pixel is therefore its
//      true value times one common factor, which cancels in num/den; the
//      largest weight of a pixel lies in [2^-1, 2^12], so nothing underflows
//      however far the colours are. Because M only moves by exact integer
//      steps, the fma returns each exponent with one rounding relative to
//      the exponent itself, which is small for the weights that matter.
//   4. Epilogue: out = num/den, mask = (den > 0) -- den is at least 1/2 as
//      soon as one sample of the window was seen, so the mask is exact.
//
// Work is proportional to the number of (pixel, sample-in-halo) pairs; the
// fraction of those inside the window is (2r+1)^2/(2r+8)^2 (66% at r=15).
#include "jbfd_internal.hpp"

namespace jbfd {

namespace {

constexpr int kWaves = 4;          // waves per workgroup (2x2 blocks of 8x8)
constexpr int kTile = 16;          // workgroup tile edge in pixels
constexpr float kRescaleAbove = 12.0f;
constexpr float kShiftInit = 8388608.0f;  // 2^23

struct alignas(16) Rec {
    uint32_t xy;   // halo-local x | y << 16
    uint32_t rg;   // (r, g) as two f16
    uint32_t b0;   // (b, 0) as two f16
    float d;       // depth
};

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// Row stride of the spatial table: at least 2r+15 and congruent to 8 mod 16,
// so the 8 rows touched by one 8x8 block land in 8 distinct groups of 8
// banks (no LDS bank conflict for 32 or 64 banks).
__host__ __device__ constexpr int table_stride(int r) {
    return ((2 * r + 15 + 7) / 16) * 16 + 8;
}

__device__ inline void load_rgb(const uint8_t *__restrict__ rgb, int64_t p,
                                uint32_t &rg, uint32_t &b0, float &sq) {
    const uint8_t *q = rgb + 3 * p;
    const float r = (float)q[0], g = (float)q[1], b = (float)q[2];
    h2 a = {(_Float16)r, (_Float16)g};
    h2 c = {(_Float16)b, (_Float16)0.0f};
    rg = __builtin_bit_cast(uint32_t, a);
    b0 = __builtin_bit_cast(uint32_t, c);
    sq = r * r + g * g + b * b;   // exact: integer below 2^18
}

__device__ inline float dot2h(uint32_t a, uint32_t b, float acc) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, a),
                                  __builtin_bit_cast(h2, b), acc, false);
}

__device__ inline uint32_t pk_sub_u16(uint32_t a, uint32_t b) {
    us2 r = __builtin_bit_cast(us2, a) - __builtin_bit_cast(us2, b);
    return __builtin_bit_cast(uint32_t, r);
}

__device__ inline uint32_t dot2_u16(uint32_t a, uint32_t b, uint32_t acc) {
    return __builtin_amdgcn_udot2(__builtin_bit_cast(us2, a),
                                  __builtin_bit_cast(us2, b), acc, false);
}

// Workgroup index -> tile index such that consecutive workgroups of one XCD
// (hardware round-robins workgroups over the 8 XCDs) cover a contiguous band
// of tiles and share halo rows in that XCD's L2. n_pad is a multiple of 8.
__device__ inline int xcd_tile(int wg, int n_pad) {
    return (wg & 7) * (n_pad >> 3) + (wg >> 3);
}

}  // namespace

template <int RMAX>
__global__ __launch_bounds__(256) void k_jbf_fwd_f32(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int n_tiles, int n_pad, float *__restrict__ out,
    uint8_t *__restrict__ mask, float2 *__restrict__ aux) {
    constexpr int kTableMax = (2 * RMAX + 15) * table_stride(RMAX);
    __shared__ float G[kTableMax];
    __shared__ Rec recs[kWaves][64];
    __shared__ float nq2h[kWaves][64];

    const int r = fp.radius;
    const int tdim = 2 * r + 15;
    const int ts = table_stride(r);
    const int tile = xcd_tile(blockIdx.x, n_pad);
    if (tile >= n_tiles) return;  // whole workgroup leaves together

    // Spatial table: G[uy*ts + ux] for dx = ux - r - 7, dy = uy - r - 7:
    // -ks (dx^2 + dy^2) inside the window, -inf outside.
    for (int t = threadIdx.x; t < tdim * tdim; t += blockDim.x) {
        const int uy = t / tdim;
        const int ux = t - uy * tdim;
        const int dx = ux - r - 7, dy = uy - r - 7;
        float g = -__builtin_inff();
        if (dx >= -r && dx <= r && dy >= -r && dy <= r)
            g = -fp.ks * (float)(dx * dx + dy * dy);
        G[uy * ts + ux] = g;
    }
    __syncthreads();

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int lane = threadIdx.x & 63;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int bx = tx * kTile + (wid & 1) * 8;
    const int by = ty * kTile + (wid >> 1) * 8;
    const int i = lane & 7, j = lane >> 3;
    const int px = bx + i, py = by + j;
    const bool inside = px < W && py < H;
    if (bx >= W || by >= H) return;  // block of a partial tile: no outputs

    uint32_t prg = 0, pb0 = 0;
    float p2 = 0.0f;
    if (inside) load_rgb(rgb, (int64_t)py * W + px, prg, pb0, p2);
    const uint32_t lxy = (uint32_t)(i + 2 * r + 7) | ((uint32_t)(j + 2 * r + 7) << 16);
    const uint32_t gstride = 4u | ((uint32_t)(4 * ts) << 16);
    const float kr2 = 2.0f * fp.kr;

    // clipped halo in absolute coordinates
    const int hx0 = max(bx - r, 0), hx1 = min(bx + 8 + r, W);
    const int hy0 = max(by - r, 0), hy1 = min(by + 8 + r, H);
    const int hw = hx1 - hx0;          // >= 1: the block holds a pixel
    const int npx = hw * (hy1 - hy0);
    const int step_x = 64 % hw, step_y = 64 / hw;

    Rec *my = recs[wid];
    float *myq = nq2h[wid];
    // M on the half-integer grid: 2^23 - kr |p|^2 rounded once
    float M = kShiftInit - fp.kr * p2;
    float num = 0.0f, den = 0.0f;
    const unsigned char *Gb = reinterpret_cast<const unsigned char *>(G);

    // Software pipeline over 64-pixel halo chunks: while the samples of
    // chunk c are processed from LDS, the sample loads of chunk c+1 and the
    // mask loads of chunk c+2 are in flight. Loaded values are only consumed
    // after the compute loop, so no wait is forced before it.
    int cx = lane % hw, cy = lane / hw;          // this lane's pixel, chunk 0
    auto advance = [&]() {
        cx += step_x;
        cy += step_y;
        if (cx >= hw) {
            cx -= hw;
            cy += 1;
        }
    };
    // pixel index of this lane in the current chunk (clamped to the first
    // halo pixel past the end, so the mask load is always in bounds)
    auto pix = [&](int base) -> uint32_t {
        const bool in = base + lane < npx;
        return in ? (uint32_t)(hy0 + cy) * (uint32_t)W + (uint32_t)(hx0 + cx)
                  : (uint32_t)hy0 * (uint32_t)W + (uint32_t)hx0;
    };
    auto xy_of = [&]() -> uint32_t {
        return (uint32_t)(hx0 + cx - (bx - r)) | ((uint32_t)(hy0 + cy - (by - r)) << 16);
    };
    auto stage = [&](bool v, uint64_t bal, uint32_t xy, uint32_t c01,
                     uint32_t c2, float d) {
        if (v) {
            const float fr = (float)(c01 & 255u), fg = (float)(c01 >> 8),
                        fb = (float)c2;
            h2 a = {(_Float16)fr, (_Float16)fg};
            h2 c = {(_Float16)fb, (_Float16)0.0f};
            Rec rec;
            rec.xy = xy;
            rec.rg = __builtin_bit_cast(uint32_t, a);
            rec.b0 = __builtin_bit_cast(uint32_t, c);
            rec.d = d;
            const int pos = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            my[pos] = rec;
            myq[pos] = -0.5f * (fr * fr + fg * fg + fb * fb);
        }
    };

    // prologue: chunk 0 fully staged, chunk 1 mask in flight
    uint32_t p0 = pix(0);
    bool v0 = (B[p0] != 0) && (lane < npx);
    uint64_t bal0 = __builtin_amdgcn_ballot_w64(v0);
    {
        uint32_t c01 = 0, c2 = 0;
        float d = 0.0f;
        if (v0) {
            const uint8_t *c = rgb + 3 * (int64_t)p0;
            c01 = (uint32_t)c[0] | ((uint32_t)c[1] << 8);
            c2 = c[2];
            d = D[p0];
        }
        stage(v0, bal0, xy_of(), c01, c2, d);
    }
    advance();
    uint32_t p1 = pix(64);
    uint32_t m1 = B[p1];
    int cnt = __builtin_popcountll(bal0);

    for (int base = 0; base < npx; base += 64) {
        // chunk c+1: its mask arrived during the previous compute loop
        const bool v1 = (m1 != 0u) && (base + 64 + lane < npx);
        const uint64_t bal1 = __builtin_amdgcn_ballot_w64(v1);
        const uint32_t xy1 = xy_of();
        uint32_t c01 = 0, c2 = 0;
        float d1 = 0.0f;
        if (v1) {
            const uint8_t *c = rgb + 3 * (int64_t)p1;
            c01 = (uint32_t)c[0] | ((uint32_t)c[1] << 8);
            c2 = c[2];
            d1 = D[p1];
        }
        // chunk c+2: mask load
        advance();
        const uint32_t p2n = pix(base + 128);
        const uint32_t m2 = B[p2n];
        __builtin_amdgcn_wave_barrier();
        // groups of four samples: all LDS reads first, one range test, and
        // the rescale path only when an exponent of the group exceeds +12
        int s = 0;
        for (; s + 4 <= cnt; s += 4) {
            float t[4], g[4], d[4], a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const Rec q = my[s + u];
                t[u] = dot2h(prg, q.rg, dot2h(pb0, q.b0, myq[s + u]));
                const uint32_t gaddr = dot2_u16(pk_sub_u16(lxy, q.xy), gstride, 0u);
                g[u] = *reinterpret_cast<const float *>(Gb + gaddr);
                d[u] = q.d;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = __builtin_fmaf(kr2, t[u], M) + g[u];
            const float amax = fmaxf(fmaxf(a[0], a[1]), fmaxf(a[2], a[3]));
            if (amax > kRescaleAbove) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float au = __builtin_fmaf(kr2, t[u], M) + g[u];
                    if (au > kRescaleAbove) {
                        const float k = __builtin_ceilf(au);
                        const int ki = (int)k;
                        num = __builtin_ldexpf(num, -ki);
                        den = __builtin_ldexpf(den, -ki);
                        M -= k;
                        au = __builtin_fmaf(kr2, t[u], M) + g[u];
                    }
                    a[u] = au;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // M may have dropped after a[u] was formed: re-form it
                    a[u] = __builtin_fmaf(kr2, t[u], M) + g[u];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float w = __builtin_amdgcn_exp2f(a[u]);
                num = __builtin_fmaf(w, d[u], num);
                den += w;
            }
        }
        for (; s < cnt; ++s) {
            const Rec q = my[s];
            const float t = dot2h(prg, q.rg, dot2h(pb0, q.b0, myq[s]));
            const uint32_t gaddr = dot2_u16(pk_sub_u16(lxy, q.xy), gstride, 0u);
            const float g = *reinterpret_cast<const float *>(Gb + gaddr);
            float a = __builtin_fmaf(kr2, t, M) + g;
            if (a > kRescaleAbove) {
                const float k = __builtin_ceilf(a);
                const int ki = (int)k;
                num = __builtin_ldexpf(num, -ki);
                den = __builtin_ldexpf(den, -ki);
                M -= k;
                a = __builtin_fmaf(kr2, t, M) + g;
            }
            const float w = __builtin_amdgcn_exp2f(a);
            num = __builtin_fmaf(w, q.d, num);
            den += w;
        }
        __builtin_amdgcn_wave_barrier();
        stage(v1, bal1, xy1, c01, c2, d1);
        cnt = __builtin_popcountll(bal1);
        p1 = p2n;
        m1 = m2;
    }

    if (inside) {
        const int64_t p = (int64_t)py * W + px;
        const bool ok = den > 0.0f;
        out[p] = ok ? num / den : 0.0f;
        mask[p] = (uint8_t)ok;
        if (aux) aux[p] = make_float2(M, den);
    }
}

hipError_t launch_densify(const float *D, const uint8_t *B, const uint8_t *rgb,
                          int32_t H, int32_t W, const FilterParams &fp,
                          jbfd_precision prec, float *out, uint8_t *mask,
                          float *aux, hipStream_t s) {
    const int tiles_x = (W + kTile - 1) / kTile;
    const int tiles_y = (H + kTile - 1) / kTile;
    const int n_tiles = tiles_x * tiles_y;
    const int n_pad = (n_tiles + 7) & ~7;
    if (prec != JBFD_FP32) return hipErrorNotSupported;
    float2 *a2 = reinterpret_cast<float2 *>(aux);
    if (fp.radius <= 16)
        k_jbf_fwd_f32<16><<<n_pad, 256, 0, s>>>(D, B, rgb, H, W, fp, tiles_x,
                                               n_tiles, n_pad, out, mask, a2);
    else
        k_jbf_fwd_f32<JBFD_MAX_RADIUS><<<n_pad, 256, 0, s>>>(
            D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, out, mask, a2);
    return hipGetLastError();
}

}  // namespace jbfd

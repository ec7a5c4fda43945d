// Joint bilateral filter over a sparse depth image (Eq. 1-4; Algorithm 1's
// window and steps), gather form, one 64-lane wave per 8x8 output block.
//
// Algorithm 1 materialises a weight volume w(x,y,k) for every pixel and
// offset, then scatters D*w and B*w with a transpose convolution. Both sums
// only ever see offsets that hold a valid sample (B = 1), and the colour and
// spatial Gaussians are symmetric, so the same output is the gather over the
// valid samples of each window. On a LiDAR image only a few percent of the
// pixels are valid, so no kernel here touches an invalid tap.
//
// Sample lists (with a caller workspace). Three small kernels build, once
// per image, a row-sorted list of the valid samples of every 8-column strip
// of the image, covering the strip's halo columns [8s-r, 8s+8+r):
//   k_list_count    one workgroup per row: 64-bit validity masks of the row
//                   (wave ballots) and, per strip, the row's sample count;
//   k_list_scan     one workgroup per strip: exclusive scan of its row counts
//                   and the strip total;
//   k_list_scatter  one workgroup per row: scans the strip totals (workgroup
//                   0 publishes them), then writes each valid sample into the
//                   list of every strip whose halo holds it (rank inside the
//                   row from the masks), as a 20-byte record
//                   {x - (8s - r) | y << 16, (r,g) f16x2, (b,0) f16x2, depth,
//                    -|rgb|^2 / 2}.
// The halo of an 8x8 block is then one contiguous range of its strip's list.
// The filter wave walks it in lockstep with scalar loads into SGPRs (every
// lane needs the same record), so per sample there is no staging work and
// no LDS traffic for the record: an LDS broadcast read would still move 16
// bytes into each of the 64 lanes and make the filter LDS-bandwidth bound.
//
// Without a workspace (or if the caller's workspace is too small for the
// lists), each wave instead streams the halo of its block from the input
// images in 64-pixel chunks and compacts the valid samples into a
// wave-private LDS list (software-pipelined: the mask bytes of chunk c+2
// and the sample data of chunk c+1 load while chunk c is processed).
//
// Per sample and lane (one output pixel):
//   colour   t = p.q - |q|^2/2 by two v_dot2_f32_f16 on the 0..255 channel
//            values (every product and partial sum is an integer or
//            half-integer below 2^23, so t is exact); -kr c = 2 kr t - kr|p|^2
//            with the per-lane -kr|p|^2 folded into the shift M;
//   space    a per-workgroup LDS table G[dy][dx] = -ks (dx^2+dy^2) inside the
//            (2r+1)^2 window and -inf outside, indexed by one packed 16-bit
//            subtract and one v_dot2_u32_u16, so the window test is free;
//   weight   w = exp2(fma(2 kr, t, M) + G), kr and ks in log2 units.
// M starts at 2^23 - kr|p|^2 (on the half-integer grid) and is lowered by
// whole integers k whenever a weight exponent would exceed +12; the
// accumulators are then scaled by the exact power of two 2^-k and the
// exponent is recomputed. Every weight of one pixel is thus its true value
// times one common factor, which cancels in num/den; the largest weight of a
// pixel lies in [2^-1, 2^12], so nothing underflows however far the colours
// are, and because M only moves by exact integer steps the fma returns each
// exponent with one rounding relative to the exponent itself. Epilogue:
// out = num/den and mask = (den > 0), den being at least 1/2 once one sample
// of the window was seen, so the mask is exact.
//
// The fraction of (pixel, halo sample) pairs that fall inside the window is
// (2r+1)^2/(2r+8)^2 (66% at r = 15).
#include <type_traits>

#include "jbfd_internal.hpp"

namespace jbfd {

namespace {

constexpr int kWaves = 4;          // waves per workgroup (2x2 blocks of 8x8)
constexpr int kTile = 16;          // workgroup tile edge in pixels
constexpr float kRescaleAbove = 12.0f;
constexpr float kShiftInit = 8388608.0f;  // 2^23
constexpr float kClampExp = -60.0f;       // pass-1 floor of each exponent part
constexpr float kWeakBelow = 1.52587890625e-05f;  // 2^-16: pass-2 threshold
constexpr int kRecWords = 5;       // list record size in 32-bit words

struct alignas(16) Rec {
    uint32_t xy;   // x - (bx - r) | y << 16
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

// colour bytes -> (r,g) f16x2, (b,0) f16x2 and -|rgb|^2/2 (all exact)
__device__ inline void colour_fields(uint32_t c01, uint32_t c2, uint32_t &rg,
                                     uint32_t &b0, float &nq2h) {
    const float fr = (float)(c01 & 255u), fg = (float)(c01 >> 8), fb = (float)c2;
    h2 a = {(_Float16)fr, (_Float16)fg};
    h2 c = {(_Float16)fb, (_Float16)0.0f};
    rg = __builtin_bit_cast(uint32_t, a);
    b0 = __builtin_bit_cast(uint32_t, c);
    nq2h = -0.5f * (fr * fr + fg * fg + fb * fb);
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

// number of set bits of the row mask `words` at positions [a, b)
__device__ inline int popc_range(const uint64_t *words, int a, int b) {
    if (b <= a) return 0;
    const int wa = a >> 6, wb = (b - 1) >> 6;
    int cnt = 0;
    for (int w = wa; w <= wb; ++w) {
        uint64_t m = words[w];
        if (w == wa) m &= ~0ull << (a & 63);
        const int hi = (b - 1) & 63;
        if (w == wb && hi != 63) m &= (1ull << (hi + 1)) - 1ull;
        cnt += __builtin_popcountll(m);
    }
    return cnt;
}

// exclusive scan over the 256 threads of a workgroup (Hillis-Steele in LDS)
__device__ inline int block_exclusive_scan(int v, int *scratch, int &total) {
    const int t = threadIdx.x;
    scratch[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = t >= off ? scratch[t - off] : 0;
        __syncthreads();
        scratch[t] += add;
        __syncthreads();
    }
    const int incl = scratch[t];
    total = scratch[255];
    __syncthreads();
    return incl - v;
}

}  // namespace

// ---------------------------------------------------------------------------
// workspace layout of the sample lists
// ---------------------------------------------------------------------------

struct ListLayout {
    int nwords;      // 64-bit mask words per row
    int n_strips;
    size_t rowbits;  // uint64 [H][nwords]
    size_t rowoff;   // int32  [n_strips][H]   counts, then row offsets
    size_t totals;   // int32  [n_strips]
    size_t base;     // int32  [n_strips + 1]
    size_t recs;     // uint32 [capacity][5]
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static ListLayout list_layout(int H, int W) {
    ListLayout L;
    L.nwords = (W + 63) / 64;
    L.n_strips = (W + 7) / 8;
    size_t off = 0;
    L.rowbits = off;
    off = align256(off + (size_t)H * L.nwords * 8);
    L.rowoff = off;
    off = align256(off + (size_t)L.n_strips * H * 4);
    L.totals = off;
    off = align256(off + (size_t)L.n_strips * 4);
    L.base = off;
    off = align256(off + (size_t)(L.n_strips + 1) * 4);
    L.recs = off;
    return L;
}

// Largest number of strips whose halo columns hold one image column.
static int strips_per_column(int r) { return (2 * r + 7) / 8 + 1; }

size_t densify_ws_bytes(int32_t H, int32_t W, int32_t r, int64_t max_samples) {
    const ListLayout L = list_layout(H, W);
    return L.recs + (size_t)max_samples * strips_per_column(r) * kRecWords * 4;
}

__global__ __launch_bounds__(256) void k_list_count(
    const uint8_t *__restrict__ B, int H, int W, int r, int n_strips,
    int nwords, uint64_t *__restrict__ rowbits, int *__restrict__ counts) {
    __shared__ uint64_t bits[512];
    const int y = blockIdx.x;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint8_t *row = B + (int64_t)y * W;
    // eight 256-pixel slices per round, all loads issued before any ballot
    for (int x0 = 0; x0 < W; x0 += 8 * 256) {
        uint8_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = x0 + 256 * k + threadIdx.x;
            v[k] = x < W ? row[x] : (uint8_t)0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint64_t bal = __builtin_amdgcn_ballot_w64(v[k] != 0);
            const int xw = x0 + 256 * k + 64 * wid;
            if (lane == 0 && xw < W) bits[xw >> 6] = bal;
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nwords; w += 256)
        rowbits[(int64_t)y * nwords + w] = bits[w];
    for (int s = threadIdx.x; s < n_strips; s += 256) {
        const int a = max(8 * s - r, 0), b = min(8 * s + 8 + r, W);
        counts[(int64_t)s * H + y] = popc_range(bits, a, b);
    }
}

// inclusive scan across the 64 lanes of a wave
__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive scan of n ints in place by one 256-thread workgroup: every
// thread sums a contiguous segment, one workgroup scan of the 256 sums, then
// every thread rewrites its segment. Returns the total.
__device__ inline int segment_scan(int *__restrict__ a, int n, int *wsum) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int seg = (n + 255) / 256;
    const int b0 = min(t * seg, n), b1 = min(b0 + seg, n);
    int sum = 0;
    for (int i0 = b0; i0 < b1; i0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = i0 + u < b1 ? a[i0 + u] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += v[u];
    }
    const int incl = wave_inclusive_scan(sum);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
        before += w < wid ? wsum[w] : 0;
        total += wsum[w];
    }
    int run = before + incl - sum;
    for (int i0 = b0; i0 < b1; i0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = i0 + u < b1 ? a[i0 + u] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (i0 + u < b1) a[i0 + u] = run;
            run += v[u];
        }
    }
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(256) void k_list_scan(int *__restrict__ rowoff,
                                                   int H,
                                                   int *__restrict__ totals) {
    __shared__ int wsum[4];
    const int s = blockIdx.x;
    const int total = segment_scan(rowoff + (int64_t)s * H, H, wsum);
    if (threadIdx.x == 0) totals[s] = total;
}

__global__ __launch_bounds__(256) void k_list_scatter(
    const float *__restrict__ D, const uint8_t *__restrict__ rgb, int H, int W,
    int r, int n_strips, int nwords, const uint64_t *__restrict__ rowbits,
    const int *__restrict__ rowoff, const int *__restrict__ totals,
    int *__restrict__ base, int64_t capacity, uint32_t *__restrict__ recs) {
    __shared__ uint64_t bits[512];
    __shared__ int start[4097];   // strip offsets, then this row's first index
    __shared__ int wsum[4];
    const int y = blockIdx.x;
    // every workgroup scans the strip totals (at most 4096 ints) itself;
    // workgroup 0 publishes them for the filter
    for (int t = threadIdx.x; t < n_strips; t += 256) start[t] = totals[t];
    for (int w = threadIdx.x; w < nwords; w += 256)
        bits[w] = rowbits[(int64_t)y * nwords + w];
    __syncthreads();
    const int all = segment_scan(start, n_strips, wsum);
    if (y == 0) {
        for (int t = threadIdx.x; t < n_strips; t += 256) base[t] = start[t];
        if (threadIdx.x == 0) base[n_strips] = all;
    }
    if (all > capacity) return;   // lists do not fit: not used
    for (int t = threadIdx.x; t < n_strips; t += 256)
        start[t] += rowoff[(int64_t)t * H + y];
    __syncthreads();
    for (int x = threadIdx.x; x < W; x += 256) {
        if (!((bits[x >> 6] >> (x & 63)) & 1ull)) continue;
        const int64_t p = (int64_t)y * W + x;
        const uint8_t *c = rgb + 3 * p;
        uint32_t rg, b0;
        float nq2h;
        colour_fields((uint32_t)c[0] | ((uint32_t)c[1] << 8), c[2], rg, b0, nq2h);
        const float d = D[p];
        const int n = x - r - 7;
        const int s_lo = n > 0 ? (n + 7) / 8 : 0;
        const int s_hi = min((x + r) / 8, n_strips - 1);
        for (int s = s_lo; s <= s_hi; ++s) {
            const int a = max(8 * s - r, 0);
            const int64_t idx = (int64_t)start[s] + popc_range(bits, a, x);
            uint32_t *q = recs + idx * kRecWords;
            q[0] = (uint32_t)(x - (8 * s - r)) | ((uint32_t)y << 16);
            q[1] = rg;
            q[2] = b0;
            q[3] = __float_as_uint(d);
            q[4] = __float_as_uint(nq2h);
        }
    }
}

// ---------------------------------------------------------------------------
// the filter
// ---------------------------------------------------------------------------

struct ListArgs {
    const uint32_t *recs;   // nullptr: stream the halo instead
    const int *rowoff;
    const int *base;
    int64_t capacity;
    int n_strips;
};

// Consume four samples: exponents a = fma(2kr, t, M) + g, rescale when one
// exceeds +12, then accumulate w = exp2(a).
__device__ inline void consume4(const float (&t)[4], const float (&g)[4],
                                const float (&d)[4], float kr2, float &M,
                                float &num, float &den) {
    float a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = __builtin_fmaf(kr2, t[u], M) + g[u];
    const float amax = fmaxf(fmaxf(a[0], a[1]), fmaxf(a[2], a[3]));
    if (amax > kRescaleAbove) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float au = __builtin_fmaf(kr2, t[u], M) + g[u];
            if (au > kRescaleAbove) {
                const float k = __builtin_ceilf(au);
                const int ki = (int)k;
                num = __builtin_ldexpf(num, -ki);
                den = __builtin_ldexpf(den, -ki);
                M -= k;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = __builtin_fmaf(kr2, t[u], M) + g[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const float w = __builtin_amdgcn_exp2f(a[u]);
        num = __builtin_fmaf(w, d[u], num);
        den += w;
    }
}

__device__ inline void consume1(float t, float g, float d, float kr2, float &M,
                                float &num, float &den) {
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
    num = __builtin_fmaf(w, d, num);
    den += w;
}

template <int RMAX>
__global__ __launch_bounds__(256) void k_jbf_fwd_f32(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int n_tiles, int n_pad, ListArgs la, float *__restrict__ out,
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
    // -ks (dx^2 + dy^2) inside the window (clamped at -60, see pass 1), -inf
    // outside.
    for (int uy = threadIdx.x >> 6; uy < tdim; uy += 4) {
        const int dy = uy - r - 7;
        for (int ux = threadIdx.x & 63; ux < tdim; ux += 64) {
            const int dx = ux - r - 7;
            float g = -__builtin_inff();
            if (dx >= -r && dx <= r && dy >= -r && dy <= r)
                g = fmaxf(-fp.ks * (float)(dx * dx + dy * dy), kClampExp);
            G[uy * ts + ux] = g;
        }
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

    float p2 = 0.0f;
    uint32_t prg = 0, pb0 = 0;
    if (inside) {
        const uint8_t *c = rgb + 3 * ((int64_t)py * W + px);
        float nh;
        colour_fields((uint32_t)c[0] | ((uint32_t)c[1] << 8), c[2], prg, pb0, nh);
        p2 = -2.0f * nh;
    }
    // lane constant for the table index: (i + 2r + 7, py + r + 7); a sample
    // record holds (x - (bx - r), y), so one packed subtract gives
    // (dx + r + 7, dy + r + 7) in [0, 2r+14]^2
    const uint32_t lxy = (uint32_t)(i + 2 * r + 7) | ((uint32_t)(py + r + 7) << 16);
    const uint32_t gstride = 4u | ((uint32_t)(4 * ts) << 16);
    const float kr2 = 2.0f * fp.kr;
    const unsigned char *Gb = reinterpret_cast<const unsigned char *>(G);
    Rec *my = recs[wid];
    float *myq = nq2h[wid];

    // Exact spatial exponent from the packed offsets u = (dx+r+7, dy+r+7):
    // -ks (dx^2+dy^2) inside the window, -inf outside (no clamp).
    const float nks = -fp.ks;
    auto exact_g = [&](uint32_t u) -> float {
        const int dx = (int)(u & 0xffffu) - r - 7, dy = (int)(u >> 16) - r - 7;
        const bool in = dx >= -r && dx <= r && dy >= -r && dy <= r;
        return in ? nks * (float)(dx * dx + dy * dy) : -__builtin_inff();
    };

    // Evaluate the samples held in the wave's LDS list, four at a time; the
    // spatial exponent comes from the clamped table, or exactly (EXACT).
    auto run_chunk = [&](int cnt, auto exact_tag, auto &&eat4, auto &&eat1) {
        constexpr bool EXACT = decltype(exact_tag)::value;
        int k = 0;
        for (; k + 4 <= cnt; k += 4) {
            float t[4], g[4], d[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const Rec q = my[k + u];
                t[u] = dot2h(prg, q.rg, dot2h(pb0, q.b0, myq[k + u]));
                const uint32_t uv = pk_sub_u16(lxy, q.xy);
                if constexpr (EXACT) {
                    g[u] = exact_g(uv);
                } else {
                    const uint32_t gaddr = dot2_u16(uv, gstride, 0u);
                    g[u] = *reinterpret_cast<const float *>(Gb + gaddr);
                }
                d[u] = q.d;
            }
            eat4(t, g, d);
        }
        for (; k < cnt; ++k) {
            const Rec q = my[k];
            const float t = dot2h(prg, q.rg, dot2h(pb0, q.b0, myq[k]));
            const uint32_t uv = pk_sub_u16(lxy, q.xy);
            float g;
            if constexpr (EXACT) {
                g = exact_g(uv);
            } else {
                g = *reinterpret_cast<const float *>(Gb + dot2_u16(uv, gstride, 0u));
            }
            eat1(t, g, q.d);
        }
    };

    // Walk every sample of the block's halo, in row-major order, through the
    // wave's LDS list: from the strip list (copy 64 records at a time) or by
    // streaming the input images.
    auto walk = [&](auto exact_tag, auto &&eat4, auto &&eat1) {
        const bool lists = la.recs != nullptr &&
                           (int64_t)la.base[la.n_strips] <= la.capacity;
        if (lists) {
            // The range [lo, hi) of the strip list, read with scalar loads
            // (the records are the same for every lane), four at a time.
            const int s = bx >> 3;
            const int *ro = la.rowoff + (int64_t)s * H;
            const int y0 = max(by - r, 0), y1 = by + 8 + r;
            const int lo = __builtin_amdgcn_readfirstlane(la.base[s] + ro[y0]);
            const int hi = __builtin_amdgcn_readfirstlane(
                y1 < H ? la.base[s] + ro[y1] : la.base[s + 1]);
            const uint32_t *__restrict__ rp = la.recs;
            constexpr bool EXACT = decltype(exact_tag)::value;
            auto sample = [&](const uint32_t *q, float &t, float &g, float &d) {
                t = dot2h(prg, q[1], dot2h(pb0, q[2], __uint_as_float(q[4])));
                const uint32_t uv = pk_sub_u16(lxy, q[0]);
                if constexpr (EXACT) {
                    g = exact_g(uv);
                } else {
                    g = *reinterpret_cast<const float *>(Gb + dot2_u16(uv, gstride, 0u));
                }
                d = __uint_as_float(q[3]);
            };
            int k = lo;
            for (; k + 4 <= hi; k += 4) {
                uint32_t q[4 * kRecWords];
                const uint32_t *src = rp + (int64_t)k * kRecWords;
#pragma unroll
                for (int e = 0; e < 4 * kRecWords; ++e) q[e] = src[e];
                float t[4], g[4], d[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) sample(q + u * kRecWords, t[u], g[u], d[u]);
                eat4(t, g, d);
            }
            for (; k < hi; ++k) {
                float t, g, d;
                sample(rp + (int64_t)k * kRecWords, t, g, d);
                eat1(t, g, d);
            }
            return;
        }
        // ---- stream the block's halo from the images ----
        const int hx0 = max(bx - r, 0), hx1 = min(bx + 8 + r, W);
        const int hy0 = max(by - r, 0), hy1 = min(by + 8 + r, H);
        const int hw = hx1 - hx0;          // >= 1: the block holds a pixel
        const int npx = hw * (hy1 - hy0);
        const int step_x = 64 % hw, step_y = 64 / hw;
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
            return (uint32_t)(hx0 + cx - (bx - r)) | ((uint32_t)(hy0 + cy) << 16);
        };
        auto stage = [&](bool v, uint64_t bal, uint32_t xy, uint32_t c01,
                         uint32_t c2, float d) {
            if (v) {
                Rec rec;
                float q2h;
                colour_fields(c01, c2, rec.rg, rec.b0, q2h);
                rec.xy = xy;
                rec.d = d;
                const int pos = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                my[pos] = rec;
                myq[pos] = q2h;
            }
        };
        // prologue: chunk 0 fully staged, chunk 1 mask in flight
        __builtin_amdgcn_wave_barrier();
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
            run_chunk(cnt, exact_tag, eat4, eat1);
            __builtin_amdgcn_wave_barrier();
            stage(v1, bal1, xy1, c01, c2, d1);
            cnt = __builtin_popcountll(bal1);
            p1 = p2n;
            m1 = m2;
        }
        __builtin_amdgcn_wave_barrier();
    };

    // Pass 1: fixed per-lane shift. Every exponent E = -kr c - ks s is <= 0,
    // so a = fma(2kr, t, -kr|p|^2) + G (the fma rounds once, relative to the
    // colour exponent itself; the rounded lane constant -kr|p|^2 shifts every
    // weight of the lane alike and cancels) never overflows. The colour part
    // is clamped at -60 and the table at -60, so an in-window sample never
    // underflows to zero: den > 0 exactly when the window holds a sample.
    const float Mfast = -fp.kr * p2;
    float num = 0.0f, den = 0.0f;
    walk(
        std::false_type{},
        [&](const float (&t)[4], const float (&g)[4], const float (&d)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float a = fmaxf(__builtin_fmaf(kr2, t[u], Mfast), kClampExp) + g[u];
                const float w = __builtin_amdgcn_exp2f(a);
                num = __builtin_fmaf(w, d[u], num);
                den += w;
            }
        },
        [&](float t, float g, float d) {
            const float a = fmaxf(__builtin_fmaf(kr2, t, Mfast), kClampExp) + g;
            const float w = __builtin_amdgcn_exp2f(a);
            num = __builtin_fmaf(w, d, num);
            den += w;
        });

    // Pass 2, only for lanes whose heaviest weight is below about 2^-16
    // (clamping or precision could matter there): the exact running shift
    // of consume4/consume1 over the same samples, with exact, unclamped
    // spatial exponents.
    const bool weak = den > 0.0f && den < kWeakBelow;
    float M = Mfast;
    if (__builtin_amdgcn_ballot_w64(weak) != 0) {
        float M2 = kShiftInit - fp.kr * p2, num2 = 0.0f, den2 = 0.0f;
        walk(
            std::true_type{},
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4]) {
                if (weak) consume4(t, g, d, kr2, M2, num2, den2);
            },
            [&](float t, float g, float d) {
                if (weak) consume1(t, g, d, kr2, M2, num2, den2);
            });
        if (weak) {
            num = num2;
            den = den2;
            M = M2;
        }
    }

    if (inside) {
        const int64_t p = (int64_t)py * W + px;
        const bool ok = den > 0.0f;
        out[p] = ok ? num / den : 0.0f;
        mask[p] = (uint8_t)ok;
        // aux: the shift and the weight sum; a negative sum marks a pixel of
        // pass 1 (weights formed with the -60 clamps)
        if (aux) aux[p] = make_float2(M, weak ? den : -den);
    }
}

// views of a caller workspace
struct ListViews {
    uint64_t *rowbits;
    int *rowoff, *totals, *base;
    uint32_t *recs;
    int64_t capacity;
};

static bool list_views(void *ws, size_t ws_bytes, const ListLayout &L,
                       ListViews &v) {
    if (ws == nullptr || ws_bytes < L.recs) return false;
    unsigned char *w = static_cast<unsigned char *>(ws);
    v.rowbits = reinterpret_cast<uint64_t *>(w + L.rowbits);
    v.rowoff = reinterpret_cast<int *>(w + L.rowoff);
    v.totals = reinterpret_cast<int *>(w + L.totals);
    v.base = reinterpret_cast<int *>(w + L.base);
    v.recs = reinterpret_cast<uint32_t *>(w + L.recs);
    v.capacity = (int64_t)((ws_bytes - L.recs) / (kRecWords * 4));
    return true;
}

hipError_t launch_densify_prepare(const float *D, const uint8_t *B,
                                  const uint8_t *rgb, int32_t H, int32_t W,
                                  int32_t radius, void *ws, size_t ws_bytes,
                                  hipStream_t s) {
    const ListLayout L = list_layout(H, W);
    ListViews v;
    if (!list_views(ws, ws_bytes, L, v)) return hipSuccess;  // nothing to build
    k_list_count<<<H, 256, 0, s>>>(B, H, W, radius, L.n_strips, L.nwords,
                                   v.rowbits, v.rowoff);
    k_list_scan<<<L.n_strips, 256, 0, s>>>(v.rowoff, H, v.totals);
    k_list_scatter<<<H, 256, 0, s>>>(D, rgb, H, W, radius, L.n_strips, L.nwords,
                                     v.rowbits, v.rowoff, v.totals, v.base,
                                     v.capacity, v.recs);
    return hipGetLastError();
}

hipError_t launch_densify(const float *D, const uint8_t *B, const uint8_t *rgb,
                          int32_t H, int32_t W, const FilterParams &fp,
                          jbfd_precision prec, float *out, uint8_t *mask,
                          float *aux, void *ws, size_t ws_bytes, bool lists_ready,
                          hipStream_t s) {
    if (prec != JBFD_FP32) return hipErrorNotSupported;
    const int tiles_x = (W + kTile - 1) / kTile;
    const int tiles_y = (H + kTile - 1) / kTile;
    const int n_tiles = tiles_x * tiles_y;
    const int n_pad = (n_tiles + 7) & ~7;
    ListArgs la{nullptr, nullptr, nullptr, 0, 0};
    const ListLayout L = list_layout(H, W);
    ListViews v;
    if (list_views(ws, ws_bytes, L, v)) {
        if (!lists_ready) {
            const hipError_t e =
                launch_densify_prepare(D, B, rgb, H, W, fp.radius, ws, ws_bytes, s);
            if (e != hipSuccess) return e;
        }
        la = ListArgs{v.recs, v.rowoff, v.base, v.capacity, L.n_strips};
    }
    float2 *a2 = reinterpret_cast<float2 *>(aux);
    if (fp.radius <= 16)
        k_jbf_fwd_f32<16><<<n_pad, 256, 0, s>>>(D, B, rgb, H, W, fp, tiles_x,
                                               n_tiles, n_pad, la, out, mask, a2);
    else
        k_jbf_fwd_f32<JBFD_MAX_RADIUS><<<n_pad, 256, 0, s>>>(
            D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, la, out, mask, a2);
    return hipGetLastError();
}

}  // namespace jbfd

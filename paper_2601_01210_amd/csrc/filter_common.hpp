// Device helpers shared by the filter's forward and backward kernels
// (product code; the CPU oracle has its own, independent implementation).
#pragma once

#include <type_traits>

#include "jbfd_internal.hpp"

namespace jbfd {


constexpr int kWaves = 4;          // waves per workgroup (2x2 blocks of 8x8)
constexpr int kTile = kTileEdge;   // workgroup tile edge in pixels
constexpr float kRescaleAbove = 12.0f;
constexpr float kShiftInit = 8388608.0f;  // 2^23
constexpr float kClampExp = -60.0f;       // pass-1 floor of each exponent part
constexpr float kWeakBelow = 1.52587890625e-05f;  // 2^-16: pass-2 threshold
constexpr int kRecWords = 5;       // list record size in 32-bit words
constexpr int NG = 4;              // records per group of the first pass's list
                                   // walk (6 and 8 measured no faster)

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

// Column-interleaved tile order, for kernels whose work follows the sample
// density: XCD c (which runs workgroups c, c + 8, ...) takes the tile
// columns tx = c (mod 8), row by row. Every XCD gets an even share of the
// columns whatever rows hold the samples (a band split leaves the XCDs of
// an empty sky idle), and vertically adjacent tiles, which read overlapping
// list ranges, stay in one L2. column_grid workgroups cover every tile;
// column_tile returns false for the few left over.
inline int column_grid(int tiles_x, int tiles_y) {
    return 8 * ((tiles_x + 7) / 8) * tiles_y;
}

__device__ inline bool column_tile(int wg, int tiles_x, int tiles_y, int &tx, int &ty) {
    const int c = wg & 7, k = wg >> 3;
    const int ncol = (tiles_x - c + 7) >> 3;   // columns c, c + 8, ... below tiles_x
    if (ncol <= 0 || k >= ncol * tiles_y) return false;
    ty = k / ncol;
    tx = c + 8 * (k - ty * ncol);
    return true;
}

// bits [a, b) of a 64-bit word (a, b clamped to [0, 64])
__device__ inline uint64_t bit_range(int a, int b) {
    a = max(a, 0);
    b = min(b, 64);
    if (b <= a) return 0ull;
    const uint64_t hi = b == 64 ? ~0ull : ((1ull << b) - 1ull);
    return hi & (~0ull << a);
}

// number of set bits at positions [a, b) of the 128-bit mask (lo | hi << 64)
__device__ inline int popc128(uint64_t lo, uint64_t hi, int a, int b) {
    return __builtin_popcountll(lo & bit_range(a, b)) +
           __builtin_popcountll(hi & bit_range(a - 64, b - 64));
}

// Inclusive scan across the 64 lanes of a wave (every lane active), with
// DPP moves instead of LDS permutes: shifts by 1, 2, 4 and 8 lanes within
// each row of 16 (Hillis-Steele), then lane 15's sum added to rows 1 and 3
// and lane 31's to rows 2 and 3 (row broadcasts). A lane whose source is
// outside its row takes the old value 0.
__device__ inline int wave_inclusive_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

// sum over the 64 lanes of a wave (every lane active), wave-uniform
__device__ inline int wave_sum(int v) {
    return __builtin_amdgcn_readlane(wave_inclusive_scan(v), 63);
}

// ---------------------------------------------------------------------------
// workspace layout of the sample lists
// ---------------------------------------------------------------------------

// The lists are built per (group of 8 strips) x (band of 32 rows): one
// workgroup per unit (bands of 8, 16, 32 and 64 rows measured 21.0, 15.3,
// 14.2 and 16.2 us for the Full-HD lists at r = 15).
constexpr int kGroupStrips = 8;
constexpr int kBandRows = 32;

struct ListLayout {
    int n_strips;    // 8-column strips
    int n_groups;    // groups of kGroupStrips strips (64 columns)
    int n_bands;     // bands of kBandRows rows
    size_t rowoff;   // int32 [n_strips][H + 1]: absolute index of the first
                     //   record of row y in strip s; [s][H] = end of strip s
    size_t bandcnt;  // int32 [n_strips][n_bands]: records per strip and band
    size_t grpcnt;   // int32 [n_groups][n_bands]: records per group and band
    size_t table;    // float [kTableFloats]: the spatial table of the
                     //   filter (build_table's layout), written by the list
                     //   scatter of a call that knows sigma_s
    size_t recs;     // uint32 [capacity][kRecWords]
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// floats of the largest spatial table (radius JBFD_MAX_RADIUS)
constexpr int kTableFloats = (2 * JBFD_MAX_RADIUS + 15) * table_stride(JBFD_MAX_RADIUS);

inline ListLayout list_layout(int H, int W) {
    ListLayout L;
    L.n_strips = (W + 7) / 8;
    L.n_groups = (L.n_strips + kGroupStrips - 1) / kGroupStrips;
    L.n_bands = (H + kBandRows - 1) / kBandRows;
    size_t off = 0;
    L.rowoff = off;
    off = align256(off + (size_t)L.n_strips * (H + 1) * 4);
    L.bandcnt = off;
    off = align256(off + (size_t)L.n_strips * L.n_bands * 4);
    L.grpcnt = off;
    off = align256(off + (size_t)L.n_groups * L.n_bands * 4);
    L.table = off;
    off = align256(off + (size_t)kTableFloats * 4);
    L.recs = off;
    return L;
}

// Largest number of strips whose halo columns hold one image column.
inline int strips_per_column(int r) { return (2 * r + 7) / 8 + 1; }

// Largest image (pixels) that gets sample lists: the list scatter's
// workgroups each sum the record counts of all earlier (group, band) units,
// a cost that grows with the square of the unit count (one unit per 1,024
// pixels; about 1 ms at this size). Larger images stream their halos.
constexpr int64_t kListMaxPixels = (int64_t)1 << 26;

// Record indices are int32: lists are built only when every pixel of the
// image could be valid without overflowing them, and only up to
// kListMaxPixels.
inline bool lists_possible(int H, int W, int r) {
    return (int64_t)H * W * strips_per_column(r) < ((int64_t)1 << 31) &&
           (int64_t)H * W <= kListMaxPixels;
}

struct ListArgs {
    const uint32_t *recs;   // nullptr: stream the halo instead
    const int *rowoff;      // [n_strips][H + 1]
    int64_t capacity;       // records the workspace holds
    const float *table = nullptr;   // the spatial table built for this call
                                    // (nullptr: each workgroup builds it)
};

// Pass-1 exponent of one sample (FP32 forms; the forward and the backward
// both use it, so they form bit-identical weights): max(a, -60) + g for the
// colour exponent a = fma(2kr, t, M) and the table entry g. It is evaluated
// as
//     y = clamp01((m - a) / 60),   e = g - 60 y   (= a - m + g above the floor)
// with the clamp done by the fma's output modifier, two instructions where
// max-then-add takes three. The heavy weights have y near 0, where y and
// g - 60 y round as finely as a and a + g do. The margin m > 0 (a lane
// constant) keeps y above 0 although rounding of the lane constant M can
// leave a slightly above 0; it scales every weight of the lane by 2^-m,
// which cancels in num/den.
struct Pass1Exp {
    float k, c;   // y = clamp01(fma(k, t, c))
    __device__ Pass1Exp(float kr2, float M)
        : k(kr2 * (1.0f / kClampExp)), c(lane_c(M)) {}
    // c for the lane constant M: (m - M) / 60 with m = 2^-10 + |M| 2^-18
    // (above the rounding residue of M, which is at most |M| 2^-24)
    __device__ static float lane_c(float M) {
        const float m = __builtin_fmaf(__builtin_fabsf(M), 0x1p-18f, 0x1p-10f);
        return (m - M) * (-1.0f / kClampExp);
    }
    __device__ static float eval(float k, float c, float t, float g) {
        const float y = __builtin_amdgcn_fmed3f(__builtin_fmaf(k, t, c), 0.0f, 1.0f);
        return __builtin_fmaf(kClampExp, y, g);
    }
    __device__ float operator()(float t, float g) const { return eval(k, c, t, g); }
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

// views of a caller workspace
struct ListViews {
    int *rowoff, *bandcnt, *grpcnt;
    float *table;
    uint32_t *recs;
    int64_t capacity;
};

inline bool list_views(void *ws, size_t ws_bytes, const ListLayout &L,
                       ListViews &v) {
    if (ws == nullptr || ws_bytes < L.recs) return false;
    unsigned char *w = static_cast<unsigned char *>(ws);
    v.rowoff = reinterpret_cast<int *>(w + L.rowoff);
    v.bandcnt = reinterpret_cast<int *>(w + L.bandcnt);
    v.grpcnt = reinterpret_cast<int *>(w + L.grpcnt);
    v.table = reinterpret_cast<float *>(w + L.table);
    v.recs = reinterpret_cast<uint32_t *>(w + L.recs);
    v.capacity = (int64_t)((ws_bytes - L.recs) / (kRecWords * 4));
    return true;
}

// Last word of a list record {(r,g) f16x2, (b,0) f16x2, depth, -|q|^2/2,
// table word}: the sample's byte offset in the spatial table frame,
// 4 (x - (8s - r)) + 4 ts y, so that a lane's table byte address is its own
// constant minus this word (one subtract per sample).
__device__ inline uint32_t rec_table_word(int xrel, int y, int ts) {
    return 4u * ((uint32_t)xrel + (uint32_t)ts * (uint32_t)y);
}

// Walks the valid samples of one 8x8 output block: the sample lists, or the
// halo streamed from the images.
struct BlockWalker {
    const float *D;
    const uint8_t *B;
    const uint8_t *rgb;
    int H, W, r;
    ListArgs la;
    int bx, by, lane;
    uint32_t prg, pb0;     // this lane's colour fields
    uint32_t lxy;          // (i + 2r + 7) | (py + r + 7) << 16
    uint32_t gstride;      // byte strides of the table index
    uint32_t lc;           // 4 ((i + 2r + 7) + ts (py + r + 7)): table byte
                           // address of a list record = lc - record word 0
    int ts;                // table row stride (floats)
    const unsigned char *Gb;
    Rec *my;               // the wave's LDS list
    float *myq;
    float nks;             // -ks
    int staged = -1;       // samples of the block's halo that the workgroup
                           // staged into `my` (row-major), or -1: stream
    float tadd = 0.0f;     // added to each sample's -|q|^2/2 when ADD

    // start of a sample's colour term: -|q|^2/2, plus the lane's own
    // -|p|^2/2 when ADD (then t = -c/2 exactly, c the squared distance)
    template <bool ADD>
    __device__ float tinit(float q2h) const {
        if constexpr (ADD)
            return q2h + tadd;
        else
            return q2h;
    }

    // exact spatial exponent: -ks (dx^2+dy^2) inside the window, -inf outside
    __device__ float exact_g(uint32_t u) const {
        const int dx = (int)(u & 0xffffu) - r - 7, dy = (int)(u >> 16) - r - 7;
        const bool in = dx >= -r && dx <= r && dy >= -r && dy <= r;
        return in ? nks * (float)(dx * dx + dy * dy) : -__builtin_inff();
    }

    template <bool EXACT>
    __device__ float spatial(uint32_t uv) const {
        if constexpr (EXACT) {
            return exact_g(uv);
        } else {
            return *reinterpret_cast<const float *>(Gb + dot2_u16(uv, gstride, 0u));
        }
    }

    // samples held in the wave's LDS list
    template <bool EXACT, bool ADD = false, class E4, class E1>
    __device__ void run_chunk(int cnt, E4 &eat4, E1 &eat1) const {
        int k = 0;
        for (; k + 4 <= cnt; k += 4) {
            float t[4], g[4], d[4];
            uint32_t uv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const Rec q = my[k + u];
                t[u] = dot2h(prg, q.rg, dot2h(pb0, q.b0, tinit<ADD>(myq[k + u])));
                uv[u] = pk_sub_u16(lxy, q.xy);
                g[u] = spatial<EXACT>(uv[u]);
                d[u] = q.d;
            }
            eat4(t, g, d, uv);
        }
        for (; k < cnt; ++k) {
            const Rec q = my[k];
            const float t = dot2h(prg, q.rg, dot2h(pb0, q.b0, tinit<ADD>(myq[k])));
            const uint32_t uv = pk_sub_u16(lxy, q.xy);
            eat1(t, spatial<EXACT>(uv), q.d, uv);
        }
    }

    // table word of a list sample -> (ux | uy << 16) for the exact pass
    __device__ uint32_t uv_of_offset(uint32_t off) const {
        const int idx = (int)(off >> 2);
        const int uy = (int)(((float)idx + 0.5f) * (1.0f / (float)ts));
        const int ux = idx - uy * ts;
        return (uint32_t)ux | ((uint32_t)uy << 16);
    }

    // records [lo, hi) of the strip list, read four at a time with scalar
    // loads (every lane needs the same record)
    template <bool EXACT, class E4, class E1>
    __device__ void walk_list(int lo, int hi, E4 &eat4, E1 &eat1) const {
        const uint32_t *__restrict__ rp = la.recs;
        auto sample = [&](const uint32_t *q, float &t, float &g, float &d,
                          uint32_t &uv) {
            t = dot2h(prg, q[0], dot2h(pb0, q[1], __uint_as_float(q[3])));
            const uint32_t off = lc - q[4];
            if constexpr (EXACT) {
                uv = uv_of_offset(off);
                g = exact_g(uv);
            } else {
                uv = off;
                g = *reinterpret_cast<const float *>(Gb + off);
            }
            d = __uint_as_float(q[2]);
        };
        int k = lo;
        for (; k + 4 <= hi; k += 4) {
            uint32_t q[4 * kRecWords];
            const uint32_t *src = rp + (int64_t)k * kRecWords;
#pragma unroll
            for (int e = 0; e < 4 * kRecWords; ++e) q[e] = src[e];
            float t[4], g[4], d[4];
            uint32_t uv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                sample(q + u * kRecWords, t[u], g[u], d[u], uv[u]);
            eat4(t, g, d, uv);
        }
        for (; k < hi; ++k) {
            float t, g, d;
            uint32_t uv;
            sample(rp + (int64_t)k * kRecWords, t, g, d, uv);
            eat1(t, g, d, uv);
        }
    }

    // The first pass's list walk, with the record loads of the next group
    // of four issued after this group's table values have arrived and before
    // its exponentials. Table reads (LDS) and record loads (scalar) share one
    // completion counter and scalar loads complete out of order, so a table
    // read still pending behind a record load would wait for that load too;
    // issued here, the loads complete while the exponentials run. stage_a
    // (t, g, d) must use g; stage_b finishes the sample. The arithmetic is
    // the same as walk_list's with eat = stage_b o stage_a. g_none is the
    // table value of weight zero (-inf for exponents, 0 for weights).
    template <bool ADD = false, class SA, class SB, class E1>
    __device__ void walk_list_split(int lo, int hi, SA &stage_a, SB &stage_b,
                                    E1 &eat1, float g_none) const {
        const uint32_t *__restrict__ rp = la.recs;
        int k = lo;
        if (k + NG <= hi) {
            uint32_t q[NG * kRecWords];
            const uint32_t *src = rp + (int64_t)k * kRecWords;
#pragma unroll
            for (int e = 0; e < NG * kRecWords; ++e) q[e] = src[e];
            for (;;) {
                float g[NG], d[NG];
                decltype(stage_a(0.0f, 0.0f, 0.0f)) sa[NG];
                // the group's table reads first, then the colour dots under them
#pragma unroll
                for (int u = 0; u < NG; ++u)
                    g[u] = *reinterpret_cast<const float *>(Gb + (lc - q[u * kRecWords + 4]));
                __builtin_amdgcn_sched_barrier(0);
                // every colour dot first: a dot product's result is read
                // by the next VALU instruction only after wait states,
                // which the other samples' dots fill (61.5 against 62.8 us)
                float tt[NG];
#pragma unroll
                for (int u = 0; u < NG; ++u) {
                    const uint32_t *qq = q + u * kRecWords;
                    tt[u] = dot2h(prg, qq[0],
                                  dot2h(pb0, qq[1], tinit<ADD>(__uint_as_float(qq[3]))));
                    d[u] = __uint_as_float(qq[2]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < NG; ++u) sa[u] = stage_a(tt[u], g[u], d[u]);
                __builtin_amdgcn_sched_barrier(0);
                // the next group (the last full group again at the end, so
                // the address stays inside the range)
                const int kn = k + NG;
                const uint32_t *nsrc = rp + (int64_t)min(kn, hi - NG) * kRecWords;
#pragma unroll
                for (int e = 0; e < NG * kRecWords; ++e) q[e] = nsrc[e];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < NG; ++u) stage_b(sa[u], g[u], d[u]);
                k = kn;
                if (k + NG > hi) break;
            }
            // the last 1 .. NG-1 samples: q already holds records [hi-NG, hi) (the
            // loads above); the first `skip` of them were consumed, and get
            // the neutral table value g_none (weight 0: num and den are
            // left exactly as they are)
            if (k < hi) {
                const int skip = k - (hi - NG);
#pragma unroll
                for (int u = 0; u < NG; ++u) {
                    const uint32_t *qq = q + u * kRecWords;
                    const float t = dot2h(
                        prg, qq[0], dot2h(pb0, qq[1], tinit<ADD>(__uint_as_float(qq[3]))));
                    const float gt =
                        *reinterpret_cast<const float *>(Gb + (lc - qq[4]));
                    const float g = u < skip ? g_none : gt;
                    const float d = __uint_as_float(qq[2]);
                    stage_b(stage_a(t, g, d), g, d);
                }
                k = hi;
            }
        }
        // lists of fewer than NG samples
        for (; k < hi; ++k) {
            const uint32_t *qq = rp + (int64_t)k * kRecWords;
            const float t =
                dot2h(prg, qq[0], dot2h(pb0, qq[1], tinit<ADD>(__uint_as_float(qq[3]))));
            const uint32_t off = lc - qq[4];
            eat1(t, *reinterpret_cast<const float *>(Gb + off), __uint_as_float(qq[2]),
                 off);
        }
    }

    // the range [lo, hi) of this block's strip list; false when there is no
    // list or the range does not lie inside the workspace (then stream)
    __device__ bool list_range(int &lo, int &hi) const {
        if (la.recs == nullptr) return false;
        const int s = bx >> 3;
        const int *ro = la.rowoff + (int64_t)s * (H + 1);
        const int y0 = max(by - r, 0), y1 = min(by + 8 + r, H);
        lo = __builtin_amdgcn_readfirstlane(ro[y0]);
        hi = __builtin_amdgcn_readfirstlane(ro[y1]);
        return lo >= 0 && lo <= hi && (int64_t)hi <= la.capacity;
    }

    template <bool EXACT, class E4, class E1>
    __device__ void walk(E4 &&eat4, E1 &&eat1) const {
        int lo, hi;
        if (list_range(lo, hi)) {
            walk_list<EXACT>(lo, hi, eat4, eat1);
            return;
        }
        if (staged >= 0) {
            run_chunk<EXACT>(staged, eat4, eat1);
            return;
        }
        stream<EXACT>(eat4, eat1);
    }

    // the exact pass: exact spatial exponents, read from the table when it
    // holds them exactly (table_exact) on the list walk; the stream always
    // recomputes them (one streaming loop fewer in the kernel)
    template <class E4, class E1>
    __device__ void walk_exact(bool table_exact, E4 &&eat4, E1 &&eat1) const {
        int lo, hi;
        if (list_range(lo, hi)) {
            if (table_exact)
                walk_list<false>(lo, hi, eat4, eat1);
            else
                walk_list<true>(lo, hi, eat4, eat1);
            return;
        }
        if (staged >= 0) {
            run_chunk<true>(staged, eat4, eat1);
            return;
        }
        stream<true>(eat4, eat1);
    }

    // first pass: the split list walk, or the stream
    template <bool ADD = false, class SA, class SB, class E4, class E1>
    __device__ void walk_split(SA &&stage_a, SB &&stage_b, E4 &&eat4, E1 &&eat1,
                               float g_none) const {
        int lo, hi;
        if (list_range(lo, hi)) {
            walk_list_split<ADD>(lo, hi, stage_a, stage_b, eat1, g_none);
            return;
        }
        if (staged >= 0) {
            run_chunk<false, ADD>(staged, eat4, eat1);
            return;
        }
        stream<false, ADD>(eat4, eat1);
    }

    // ---- stream the block's halo from the images ----
    // The halo is walked in row-major order, 64 pixels per chunk, lane k of
    // a chunk at halo position (64 c + k) mod hw, div hw. Each lane steps
    // its pixel offset, column and record position by the chunk's constant
    // strides (plus a row wrap), and addresses the images with 32-bit
    // offsets from their bases (every offset of an image of at most
    // JBFD_MAX_SIDE^2 pixels, times 4, fits in 32 bits).
    template <bool EXACT, bool ADD = false, class E4, class E1>
    __device__ void stream(E4 &eat4, E1 &eat1) const {
        const int hx0 = max(bx - r, 0), hx1 = min(bx + 8 + r, W);
        const int hy0 = max(by - r, 0), hy1 = min(by + 8 + r, H);
        const int hw = hx1 - hx0;          // >= 1: the block holds a pixel
        const int npx = hw * (hy1 - hy0);
        const int step_x = 64 % hw, step_y = 64 / hw;
        // (lane + 0.5) / hw lies at least 0.5 / hw from an integer, far
        // above the product's rounding error, so the floor is lane div hw
        const int cy0 = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)hw));
        int cx = lane - cy0 * hw;
        const uint32_t Wu = (uint32_t)W;
        const uint32_t first = (uint32_t)hy0 * Wu + (uint32_t)hx0;
        uint32_t p = first + (uint32_t)cy0 * Wu + (uint32_t)cx;
        uint32_t xy = (uint32_t)(hx0 + cx - (bx - r)) | ((uint32_t)(hy0 + cy0) << 16);
        const uint32_t dp = (uint32_t)step_y * Wu + (uint32_t)step_x;
        const uint32_t dp_wrap = Wu - (uint32_t)hw;
        const uint32_t dxy = (uint32_t)step_x + ((uint32_t)step_y << 16);
        const uint32_t dxy_wrap = (1u << 16) - (uint32_t)hw;   // x - hw, y + 1
        auto advance = [&]() {
            cx += step_x;
            p += dp;
            xy += dxy;
            if (cx >= hw) {
                cx -= hw;
                p += dp_wrap;
                xy += dxy_wrap;
            }
        };
        // the lane's pixel offset in the chunk starting at halo index base,
        // or the first halo pixel past the end (an in-bounds mask load)
        auto pix = [&](int base) -> uint32_t { return base + lane < npx ? p : first; };
        const char *Dc = reinterpret_cast<const char *>(D);
        auto load_sample = [&](uint32_t q, uint32_t &c01, uint32_t &c2, float &d) {
            const uint32_t o3 = q * 3u;
            c01 = (uint32_t)rgb[o3] | ((uint32_t)rgb[o3 + 1u] << 8);
            c2 = rgb[o3 + 2u];
            d = *reinterpret_cast<const float *>(Dc + (q << 2));
        };
        auto stage = [&](bool v, uint64_t bal, uint32_t xyv, uint32_t c01,
                         uint32_t c2, float d) {
            if (v) {
                Rec rec;
                float q2h;
                colour_fields(c01, c2, rec.rg, rec.b0, q2h);
                rec.xy = xyv;
                rec.d = d;
                const int pos = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                my[pos] = rec;
                myq[pos] = q2h;
            }
        };
        // software pipeline over 64-pixel chunks: the mask bytes of chunk c+2
        // and the sample data of chunk c+1 load while chunk c is processed;
        // loaded values are consumed only after the compute loop
        __builtin_amdgcn_wave_barrier();
        const uint32_t p0 = pix(0);
        const bool v0 = (B[p0] != 0) && (lane < npx);
        const uint64_t bal0 = __builtin_amdgcn_ballot_w64(v0);
        {
            uint32_t c01 = 0, c2 = 0;
            float d = 0.0f;
            if (v0) load_sample(p0, c01, c2, d);
            stage(v0, bal0, xy, c01, c2, d);
        }
        advance();
        uint32_t p1 = pix(64);
        uint32_t m1 = B[p1];
        int cnt = __builtin_popcountll(bal0);
        for (int base = 0; base < npx; base += 64) {
            const bool v1 = (m1 != 0u) && (base + 64 + lane < npx);
            const uint64_t bal1 = __builtin_amdgcn_ballot_w64(v1);
            const uint32_t xy1 = xy;
            uint32_t c01 = 0, c2 = 0;
            float d1 = 0.0f;
            if (v1) load_sample(p1, c01, c2, d1);
            advance();
            const uint32_t p2n = pix(base + 128);
            const uint32_t m2 = B[p2n];
            __builtin_amdgcn_wave_barrier();
            run_chunk<EXACT, ADD>(cnt, eat4, eat1);
            __builtin_amdgcn_wave_barrier();
            stage(v1, bal1, xy1, c01, c2, d1);
            cnt = __builtin_popcountll(bal1);
            p1 = p2n;
            m1 = m2;
        }
        __builtin_amdgcn_wave_barrier();
    }
};

// Fill the spatial table G[uy*ts + ux] (dx = ux - r - 7, dy = uy - r - 7;
// in LDS, or in a workspace for the filter's workgroups to copy) with the
// clamped exponent -ks (dx^2+dy^2) >= -60 inside the window and -inf
// outside (weights = false), or with the weight exp2(-ks (dx^2+dy^2))
// floored at 2^-100 inside and 0 outside (weights = true).
// The entries depend on |dx| and |dy| only: the workgroup's threads share
// the quarter 0 <= |dx|, |dy| <= r + 7 and each writes its entry at the
// four mirrored positions (about half the work of one entry per table
// cell; without a table built for the call, every workgroup of the filter
// builds its own, 8,160 times per Full-HD frame). (float)(dx^2 + dy^2) is
// exact (below 2^24), so the entries equal -ks (float)(dx^2 + dy^2), the
// exact pass's spatial exponents.
__device__ inline void build_table(float *G, int r, int ts, float ks, bool weights) {
    const int h = r + 7;       // the centre's index in both directions
    const int q = h + 1;       // quarter side
    const float g_out = weights ? 0.0f : -__builtin_inff();
    // (e + 0.5) / q lies at least 0.5 / q from an integer, far above the
    // product's rounding error for e < q^2 <= 1600
    const float inv = __builtin_amdgcn_rcpf((float)q);
    for (int e = (int)threadIdx.x; e < q * q; e += 256) {
        const int ay = (int)(((float)e + 0.5f) * inv);
        const int ax = e - ay * q;
        float g = g_out;
        if (ax <= r && ay <= r) {
            const float d2 = -ks * (float)(__mul24(ax, ax) + __mul24(ay, ay));
            g = weights ? __builtin_amdgcn_exp2f(fmaxf(d2, -100.0f)) : fmaxf(d2, kClampExp);
        }
        float *row0 = G + (h - ay) * ts, *row1 = G + (h + ay) * ts;
        row0[h - ax] = g;
        row0[h + ax] = g;
        row1[h - ax] = g;
        row1[h + ax] = g;
    }
}

// The workgroup's copy of a table that build_table wrote to global memory
// for this call (rows of ts floats, ts a multiple of 8: 16-byte loads and
// LDS stores; the columns past 2r + 14 are never read, built or not).
__device__ inline void copy_table(float *G, const float *__restrict__ src, int r, int ts) {
    const int n4 = (2 * r + 15) * ts / 4;
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *g4 = reinterpret_cast<float4 *>(G);
    for (int e = (int)threadIdx.x; e < n4; e += 256) g4[e] = s4[e];
}

}  // namespace jbfd

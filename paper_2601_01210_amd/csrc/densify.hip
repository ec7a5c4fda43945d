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
#include "filter_common.hpp"

namespace jbfd {

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

// Scratch of one filter workgroup (LDS).
template <int RMAX>
struct FilterShared {
    float G[(2 * RMAX + 15) * table_stride(RMAX)];
    Rec recs[kWaves][64];
    float nq2h[kWaves][64];
};

// Filter one 16x16 output tile (tx, ty) of an image with one 256-thread
// workgroup: builds the spatial table, then each wave filters its 8x8 block.
// Every thread returns normally, so callers may loop over tiles with a
// barrier between them.
template <int RMAX, int PREC>
__device__ void filter_tile(const float *__restrict__ D,
                            const uint8_t *__restrict__ B,
                            const uint8_t *__restrict__ rgb, int H, int W,
                            const FilterParams &fp, const ListArgs &la, int tx,
                            int ty, float *__restrict__ out,
                            uint8_t *__restrict__ mask, float2 *__restrict__ aux,
                            FilterShared<RMAX> &sh) {
    const int r = fp.radius;
    const int ts = table_stride(r);
    // spatial table: clamped exponents (FP32) or weights (FP16 range)
    build_table(sh.G, r, ts, fp.ks, PREC != JBFD_FP32);
    __syncthreads();

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int lane = threadIdx.x & 63;
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
    const BlockWalker bw{D, B, rgb, H, W, r, la, bx, by, lane, prg, pb0, lxy,
                         gstride, reinterpret_cast<const unsigned char *>(sh.G),
                         sh.recs[wid], sh.nq2h[wid], -fp.ks};

    // Pass 1: fixed per-lane shift. Every exponent E = -kr c - ks s is <= 0,
    // so a = fma(2kr, t, -kr|p|^2) + G (the fma rounds once, relative to the
    // colour exponent itself; the rounded lane constant -kr|p|^2 shifts every
    // weight of the lane alike and cancels) never overflows.
    //  FP32: the colour part is clamped at -60 and the table at -60, so an
    //        in-window sample never underflows to zero and den > 0 exactly
    //        when the window holds a sample.
    //  FP16 range weights: the colour exponent is rounded to FP16 by the
    //        mixed-precision fma, w_c = v_exp_f16, and w_c times the FP32
    //        spatial weight is accumulated in FP32 through v_fma_mix; the
    //        sum of the spatial weights alone (never zero in the window)
    //        decides the mask.
    const float Mfast = -fp.kr * p2;
    float num = 0.0f, den = 0.0f, dsp = 0.0f;
    if constexpr (PREC == JBFD_FP32) {
        auto eat = [&](float t, float g, float d, uint32_t) {
            const float a = fmaxf(__builtin_fmaf(kr2, t, Mfast), kClampExp) + g;
            const float w = __builtin_amdgcn_exp2f(a);
            num = __builtin_fmaf(w, d, num);
            den += w;
        };
        bw.walk<false>(
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&uv)[4]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
            },
            eat);
        dsp = den;
    } else {
        auto eat = [&](float t, float ws, float d, uint32_t) {
            const _Float16 e = (_Float16)__builtin_fmaf(kr2, t, Mfast);
            const float wc = (float)__builtin_exp2f16(e);
            num = __builtin_fmaf(wc, ws * d, num);
            den = __builtin_fmaf(wc, ws, den);
            dsp += ws;
        };
        bw.walk<false>(
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&uv)[4]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
            },
            eat);
    }

    // Pass 2, only for lanes whose heaviest weight is below about 2^-16
    // (clamping or precision could matter there): the exact running shift
    // of consume4/consume1 over the same samples, with exact, unclamped
    // spatial exponents.
    const bool weak =
        dsp > 0.0f && den < (PREC == JBFD_FP32 ? kWeakBelow : kWeakBelowF16);
    float M = Mfast;
    if (__builtin_amdgcn_ballot_w64(weak) != 0) {
        float M2 = kShiftInit - fp.kr * p2, num2 = 0.0f, den2 = 0.0f;
        bw.walk<true>(
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&)[4]) {
                if (weak) consume4(t, g, d, kr2, M2, num2, den2);
            },
            [&](float t, float g, float d, uint32_t) {
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
        const bool ok = dsp > 0.0f;
        out[p] = ok ? num / den : 0.0f;
        mask[p] = (uint8_t)ok;
        // aux: the shift and the weight sum; a negative sum marks a pixel of
        // pass 1 (weights formed with the -60 clamps)
        if (aux) aux[p] = make_float2(M, weak ? den : -den);
    }
}

template <int RMAX, int PREC>
__global__ __launch_bounds__(256) void k_jbf_fwd(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int n_tiles, int n_pad, ListArgs la, float *__restrict__ out,
    uint8_t *__restrict__ mask, float2 *__restrict__ aux) {
    __shared__ FilterShared<RMAX> sh;
    const int tile = xcd_tile(blockIdx.x, n_pad);
    if (tile >= n_tiles) return;  // whole workgroup leaves together
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    filter_tile<RMAX, PREC>(D, B, rgb, H, W, fp, la, tx, ty, out, mask, aux, sh);
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
    const bool small = fp.radius <= 16;
    if (prec == JBFD_FP32) {
        if (small)
            k_jbf_fwd<16, JBFD_FP32><<<n_pad, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, la, out, mask, a2);
        else
            k_jbf_fwd<JBFD_MAX_RADIUS, JBFD_FP32><<<n_pad, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, la, out, mask, a2);
    } else {
        if (small)
            k_jbf_fwd<16, JBFD_FP16_RANGE><<<n_pad, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, la, out, mask, nullptr);
        else
            k_jbf_fwd<JBFD_MAX_RADIUS, JBFD_FP16_RANGE><<<n_pad, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, n_tiles, n_pad, la, out, mask, nullptr);
    }
    return hipGetLastError();
}

}  // namespace jbfd

namespace jbfd {

// Filter tiles of every view of a batch: a fixed grid walks the flattened
// tile space (views back to back); each workgroup finds its view by a
// binary search of the table's tile offsets (wave-uniform scalar loads).
template <int RMAX, int PREC>
__global__ __launch_bounds__(256) void k_batch_filter(const BatchHeader *__restrict__ hdr,
                                                      const BatchView *__restrict__ views) {
    __shared__ FilterShared<RMAX> sh;
    const int n_views = hdr->n_views;
    const int total = hdr->total_tiles;
    const ListArgs none{nullptr, nullptr, nullptr, 0, 0};
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int lo = batch_view_of<&BatchView::tile_off>(views, n_views, t);
        const BatchView &v = views[lo];
        const int local = t - v.tile_off;
        const int ty = local / v.tiles_x, tx = local - ty * v.tiles_x;
        const FilterParams fp{v.radius, v.kr, v.ks};
        filter_tile<RMAX, PREC>(v.sd, v.sv, v.rgb, v.H, v.W, fp, none, tx, ty,
                                v.out, v.mask, nullptr, sh);
        __syncthreads();   // the next tile rebuilds the table
    }
}

hipError_t launch_batch_filter(const BatchHeader *hdr, const BatchView *views,
                               int32_t max_radius, jbfd_precision prec,
                               hipStream_t s) {
    const int grid = 2048;   // 8 workgroups per CU
    if (max_radius <= 16) {
        if (prec == JBFD_FP32)
            k_batch_filter<16, JBFD_FP32><<<grid, 256, 0, s>>>(hdr, views);
        else
            k_batch_filter<16, JBFD_FP16_RANGE><<<grid, 256, 0, s>>>(hdr, views);
    } else {
        if (prec == JBFD_FP32)
            k_batch_filter<JBFD_MAX_RADIUS, JBFD_FP32><<<grid, 256, 0, s>>>(hdr, views);
        else
            k_batch_filter<JBFD_MAX_RADIUS, JBFD_FP16_RANGE><<<grid, 256, 0, s>>>(hdr,
                                                                                views);
    }
    return hipGetLastError();
}

}  // namespace jbfd

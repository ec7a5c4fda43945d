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
// Sample lists (with a caller workspace). The image is cut into 8-column
// strips; the list of strip s holds, sorted by row and then column, every
// valid sample in the strip's halo columns [8s-r, 8s+8+r), as a 20-byte
// record {(r,g) f16x2, (b,0) f16x2, depth, -|rgb|^2 / 2, table word}. Two
// kernels build all lists, each over (group of 8 strips) x (band of 32
// rows) units:
//   k_list_count    validity masks of the band's rows over the group's
//                   halo columns (wave ballots) -> records per strip and band;
//   k_list_scatter  the group's strip offsets from the band counts, per-row
//                   offsets by a wave scan over the band's rows (written
//                   to rowoff), then every valid sample written into the list
//                   of each strip of the group whose halo holds it (its rank
//                   in the row from the masks).
// The halo rows of an 8x8 block are one contiguous range of its strip's
// list. The filter wave walks it in lockstep with scalar loads into SGPRs
// (every lane needs the same record), so per sample there is no staging work
// and no LDS traffic for the record: an LDS broadcast read would still move
// 16 bytes into each of the 64 lanes and make the filter LDS-bandwidth
// bound. A block whose range does not fit the workspace streams instead.
//
// Without a workspace the workgroup stages its tile's halo once and each
// wave copies its block's samples into its LDS list (tile_stage); beyond
// the staging capacities a wave streams the halo of its block from the
// input images in 64-pixel chunks and compacts the valid samples into its
// list (software-pipelined: the mask bytes of chunk c+2 and the sample
// data of chunk c+1 load while chunk c is processed).
//
// Per sample and lane (one output pixel):
//   colour   t = p.q - |q|^2/2 by two v_dot2_f32_f16 on the 0..255 channel
//            values (every product and partial sum is an integer or
//            half-integer below 2^23, so t is exact); -kr c = 2 kr t - kr|p|^2;
//   space    a per-workgroup LDS table G[dy][dx] = -ks (dx^2+dy^2) inside the
//            (2r+1)^2 window and -inf outside; a list record carries its
//            position as a table offset, so the lane's address is one
//            subtract and the window test is free;
//   weight   FP32 without aux (the direct pass): the colour term starts at
//            -(|p|^2 + |q|^2)/2, so t = -c/2 exactly and w = exp2(fma(2 kr,
//            t, G)), eight VALU instructions per sample; a weight may
//            underflow, so lanes whose sum ends below 2^-16, zero
//            included, take the second pass, which also decides their
//            mask. With aux (the backward replays these weights):
//            w = exp2(max(2 kr t - kr|p|^2, -60) + G), kr and ks in log2
//            units (the table is clamped at -60 too), so every in-window
//            sample has w >= 2^-120 > 0 and den > 0 is exactly the mask;
//            the clamp rides on an fma's output modifier (Pass1Exp), nine
//            instructions per sample.
// Lanes whose weight sum ends below 2^-16 (far colours: clamping,
// underflow or rounding could matter) are recomputed in a second pass with
// an exact running shift M: it starts at 2^23 - kr|p|^2 and drops by whole
// integers k whenever an exponent would exceed +12, scaling the sums by
// 2^-k, with unclamped spatial exponents. Every weight of a pixel is thus
// its true value times one common factor, which cancels in num/den.
//
// The fraction of (pixel, halo sample) pairs that fall inside the window is
// (2r+1)^2/(2r+8)^2 (66% at r = 15).
#include "filter_common.hpp"
#include "project_common.hpp"

namespace jbfd {

size_t densify_ws_bytes(int32_t H, int32_t W, int32_t r, int64_t max_samples) {
    const ListLayout L = list_layout(H, W);
    return L.recs + (size_t)max_samples * strips_per_column(r) * kRecWords * 4;
}

// The halo columns of group g at radius r are [c0, c0 + 64 + 2r) with
// c0 = 64g - r, at most 128 (r <= 32): lane l covers column c0 + l in the
// first half and column c0 + 64 + l in the second, where only lanes
// l < 2r lie in the halo. The other lanes of the second half read the
// halo's last column again (a load of a line the wave already reads) and
// their ballot bits are zero.
__device__ __forceinline__ int halo_col_b(int c0, int r, int W) {
    const int lane = threadIdx.x & 63;
    return min(c0 + 64 + min(lane, 2 * r - 1), W - 1);   // >= 0: r < 64
}

// Load the validity bytes of rows [y_first, y_first + NROWS) over the
// group's halo columns (halo_col_b), one byte per lane and row and half.
// Every load is unconditional from a clamped (in-image) address, so all of
// them are in flight together; row_ballots masks the columns and rows
// outside the image and the halo.
template <int NROWS>
__device__ __forceinline__ void group_row_bytes(const uint8_t *__restrict__ B, int H,
                                                int W, int c0, int r, int y_first,
                                                uint8_t (&va)[NROWS],
                                                uint8_t (&vb)[NROWS]) {
    const int lane = threadIdx.x & 63;
    const int xa_c = min(max(c0 + lane, 0), W - 1);
    const int xb_c = halo_col_b(c0, r, W);
#pragma unroll
    for (int k = 0; k < NROWS; ++k) {
        const uint8_t *row = B + (int64_t)min(y_first + k, H - 1) * W;
        va[k] = row[xa_c];
        vb[k] = row[xb_c];
    }
}

// ... and ballot them into 128-bit row masks (bit c: column c0 + c)
template <int NROWS>
__device__ __forceinline__ void row_ballots(int H, int W, int c0, int r, int y_first,
                                            const uint8_t (&va)[NROWS],
                                            const uint8_t (&vb)[NROWS],
                                            uint64_t (&lo)[NROWS], uint64_t (&hi)[NROWS]) {
    const int lane = threadIdx.x & 63;
    const int xa = c0 + lane, xb = c0 + 64 + lane;
    const bool ina = xa >= 0 && xa < W, inb = lane < 2 * r && xb < W;
#pragma unroll
    for (int k = 0; k < NROWS; ++k) {
        const bool iny = y_first + k < H;
        lo[k] = __builtin_amdgcn_ballot_w64(ina && iny && va[k] != 0);
        hi[k] = __builtin_amdgcn_ballot_w64(inb && iny && vb[k] != 0);
    }
}

// Unit (group g, band) of this workgroup in a one-dimensional grid of
// n_groups x n_bands workgroups. Workgroup i runs on XCD i mod 8, each XCD
// with an L2 of its own, and neighbouring groups of a band read each
// other's edge columns, so the units are numbered band by band and XCD x
// takes the x-th of eight contiguous runs of them.
__device__ __forceinline__ void list_unit(int n_groups, int n_bands, int &g, int &band) {
    const int n = n_groups * n_bands;
    const int i = blockIdx.x, x = i & 7, slot = i >> 3;
    const int u = x * (n >> 3) + min(x, n & 7) + slot;
    band = u / n_groups;
    g = u - band * n_groups;
}

// Records per (strip, band) from the row masks of the unit (group g, band
// b): lanes 0..7 of each wave count its rows' samples in the halo of strip
// 8g + lane; wave 0 sums the four waves and the group. (The unit functions
// are forced inline: called out of line, their uniform arguments and
// pointers would live in vector registers and their loads would lose their
// scalar bases.)
template <int NROWS>
__device__ __forceinline__ void count_strips(const uint64_t (&lo)[NROWS],
                                             const uint64_t (&hi)[NROWS], int r,
                                             int n_strips, int n_bands,
                                             int *__restrict__ bandcnt,
                                             int *__restrict__ grpcnt, int g, int band) {
    __shared__ int part[4][kGroupStrips];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    int acc = 0;
    if (lane < kGroupStrips) {
#pragma unroll
        for (int k = 0; k < NROWS; ++k)
            acc += popc128(lo[k], hi[k], 8 * lane, 8 * lane + 8 + 2 * r);
        part[wid][lane] = acc;
    }
    __syncthreads();
    if (threadIdx.x < 64) {   // wave 0: strips of the group, then their sum
        const int q = threadIdx.x;
        const int s = kGroupStrips * g + q;
        int sum = 0;
        if (q < kGroupStrips && s < n_strips) {
            sum = part[0][q] + part[1][q] + part[2][q] + part[3][q];
            bandcnt[(int64_t)s * n_bands + band] = sum;
        }
        const int gsum = wave_sum(sum);   // lanes 8 .. 63 hold 0
        if (q == 0) grpcnt[(int64_t)g * n_bands + band] = gsum;
    }
}

// Records per (strip, band): workgroup (group g, band b); wave w ballots a
// quarter of the band's rows from the validity bytes.
__device__ __forceinline__ void list_count_unit(const uint8_t *__restrict__ B, int H, int W,
                                       int r, int n_strips, int n_bands,
                                       int *__restrict__ bandcnt,
                                       int *__restrict__ grpcnt, int g, int band) {
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = 64 * g - r;
    constexpr int kRowsPerWave = kBandRows / 4;
    const int y_first = band * kBandRows + wid * kRowsPerWave;
    uint8_t va[kRowsPerWave], vb[kRowsPerWave];
    group_row_bytes<kRowsPerWave>(B, H, W, c0, r, y_first, va, vb);
    uint64_t lo[kRowsPerWave], hi[kRowsPerWave];
    row_ballots<kRowsPerWave>(H, W, c0, r, y_first, va, vb, lo, hi);
    count_strips<kRowsPerWave>(lo, hi, r, n_strips, n_bands, bandcnt, grpcnt, g, band);
}

__global__ __launch_bounds__(256) void k_list_count(const uint8_t *__restrict__ B,
                                                    int H, int W, int r, int n_strips,
                                                    int n_bands,
                                                    int *__restrict__ bandcnt,
                                                    int *__restrict__ grpcnt) {
    int g, band;
    list_unit((n_strips + kGroupStrips - 1) / kGroupStrips, n_bands, g, band);
    list_count_unit(B, H, W, r, n_strips, n_bands, bandcnt, grpcnt, g, band);
}

// Decode and count in one pass, for a projection straight into the sample
// lists (jbfd_project_densify). Unit (group g, band b) reads the keys of the
// band's rows over the group's halo columns, writes depth and validity
// of its own 64 columns [64g, 64g + 64) (lane l decodes column
// 64g + ((l - r) mod 64) of each row, from the key it loaded in the first
// or the second half; r <= 32 < 64) and counts each strip's samples as
// k_list_count does. Keys are only read here (the list scatter clears them
// afterwards), so a unit may read its neighbours' columns.
__global__ __launch_bounds__(256) void k_decode_count(const uint64_t *__restrict__ keys,
                                                      int H, int W, int r, int n_strips,
                                                      int n_bands, float *__restrict__ D,
                                                      uint8_t *__restrict__ B,
                                                      int *__restrict__ bandcnt,
                                                      int *__restrict__ grpcnt) {
    int g, band;
    list_unit((n_strips + kGroupStrips - 1) / kGroupStrips, n_bands, g, band);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c0 = 64 * g - r;
    constexpr int kRowsPerWave = kBandRows / 4;
    const int y_first = band * kBandRows + wid * kRowsPerWave;
    const int xa = c0 + lane, xb = c0 + 64 + lane;
    const int xa_c = min(max(xa, 0), W - 1), xb_c = halo_col_b(c0, r, W);
    uint64_t ka[kRowsPerWave], kb[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {   // all loads in flight together
        const uint64_t *row = keys + (int64_t)min(y_first + k, H - 1) * W;
        ka[k] = row[xa_c];
        kb[k] = row[xb_c];
    }
    const bool ina = xa >= 0 && xa < W, inb = lane < 2 * r && xb < W;
    uint64_t lo[kRowsPerWave], hi[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
        const bool iny = y_first + k < H;
        lo[k] = __builtin_amdgcn_ballot_w64(ina && iny && ka[k] != kEmptyKey);
        hi[k] = __builtin_amdgcn_ballot_w64(inb && iny && kb[k] != kEmptyKey);
    }
    const bool own_a = lane >= r;
    const int xo = own_a ? xa : xb;   // in [64g, 64g + 64)
    if (xo < W) {
#pragma unroll
        for (int k = 0; k < kRowsPerWave; ++k) {
            const int y = y_first + k;
            if (y >= H) break;
            const uint64_t key = own_a ? ka[k] : kb[k];
            const bool hit = key != kEmptyKey;
            const int64_t p = (int64_t)y * W + xo;
            D[p] = hit ? __uint_as_float((uint32_t)(key >> 32)) : 0.0f;
            B[p] = (uint8_t)hit;
        }
    }
    count_strips<kRowsPerWave>(lo, hi, r, n_strips, n_bands, bandcnt, grpcnt, g, band);
}

// Offsets and records of the group's strips over one band (see the file
// comment). The absolute start of strip s is the sum of the band counts of
// every strip before it; the start of band b within s adds the counts of
// bands < b. The phases are ordered so that the loads of the records' data
// are in flight while the offsets are computed: masks, the band's valid
// pixels (plist) and their colour and depth loads first, then the offsets,
// then the record stores.
__device__ __forceinline__ void list_scatter_unit(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, int r, int n_strips,
    int n_bands, const int *__restrict__ bandcnt, const int *__restrict__ grpcnt,
    int *__restrict__ rowoff, int64_t capacity, uint32_t *__restrict__ recs, int g,
    int band, uint64_t *__restrict__ reset_keys = nullptr) {
    __shared__ uint64_t mlo[kBandRows], mhi[kBandRows];
    __shared__ __align__(16) int start[kBandRows][kGroupStrips];   // [row][strip]
    __shared__ uint16_t plist[kBandRows * 128];   // valid pixels of the band

    __shared__ int red[4];
    __shared__ int stot[kGroupStrips], spre[kGroupStrips], sbase[kGroupStrips];
    const int t = threadIdx.x;
    const int wid = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int c0 = 64 * g - r;
    const int y_band = band * kBandRows;
    const int s_first = kGroupStrips * g;

    // The prologue's loads are all issued before the first wait: (a) the
    // validity bytes of the band's rows (wave w: the w-th quarter), (b) the
    // group-and-band totals of the groups before g, whose sum is the number
    // of records of all strips before the group, and (c) per strip of the
    // group (32 threads each), its band counts, for its total and the part
    // in bands before ours. One batch of (b) and (c) covers images of up to
    // 2048 group-band entries before the group and 128 bands (Full-HD:
    // 986 and 34); larger images loop over further batches afterwards.
    constexpr int kRowsPerWave = kBandRows / 4;
    const int y_rows = y_band + wid * kRowsPerWave;
    uint8_t va[kRowsPerWave], vb[kRowsPerWave];
    group_row_bytes<kRowsPerWave>(B, H, W, c0, r, y_rows, va, vb);
    const int n_before = g * n_bands;
    int a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int k = 256 * u + t;
        a[u] = grpcnt[k < n_before ? k : 0];
    }
    const int j = t >> 5, k32 = t & 31;
    const int sj = s_first + j;
    const bool sj_ok = sj < n_strips;
    const int *bc = bandcnt + (int64_t)(sj_ok ? sj : 0) * n_bands;
    int c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int b = 32 * u + k32;
        c[u] = bc[b < n_bands ? b : 0];
    }

    // (1) row masks (waits for the validity bytes only)
    {
        uint64_t lo[kRowsPerWave], hi[kRowsPerWave];
        row_ballots<kRowsPerWave>(H, W, c0, r, y_rows, va, vb, lo, hi);
        if (lane < kRowsPerWave) {
            uint64_t ma = 0, mb = 0;
#pragma unroll
            for (int k = 0; k < kRowsPerWave; ++k) {
                ma = lane == k ? lo[k] : ma;
                mb = lane == k ? hi[k] : mb;
            }
            mlo[wid * kRowsPerWave + lane] = ma;
            mhi[wid * kRowsPerWave + lane] = mb;
        }
    }
    __syncthreads();
    // (2) compact the band's valid pixels into plist (row << 8 | column),
    // row by row; every wave scans the rows' counts (lane = row) and fills
    // rows w, w + 4, ...
    int total;
    {
        const bool rl = lane < kBandRows;
        const int row = rl ? lane : 0;
        const int cnt = rl ? __builtin_popcountll(mlo[row]) + __builtin_popcountll(mhi[row])
                           : 0;
        const int incl = wave_inclusive_scan(cnt);
        const int excl = incl - cnt;
        total = __builtin_amdgcn_readlane(incl, kBandRows - 1);
        for (int row = wid; row < kBandRows; row += 4) {
            const uint64_t ml = mlo[row], mh = mhi[row];
            const int base = __builtin_amdgcn_readlane(excl, row);
            const uint32_t below =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(ml >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)ml, 0u));
            if ((ml >> lane) & 1ull) plist[base + below] = (uint16_t)((row << 8) | lane);
            const uint32_t below_h =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(mh >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mh, 0u));
            if ((mh >> lane) & 1ull)
                plist[base + __builtin_popcountll(ml) + below_h] =
                    (uint16_t)((row << 8) | (64 + lane));
        }
    }
    __syncthreads();
    // (3) one thread per valid pixel, two per pass: the first pass's colour
    // and depth loads are issued here, unconditionally (a lane past the end
    // reads the band's first in-image pixel of the group), so no branch
    // separates them from the offsets' waits below
    const int safe_ent = c0 < 0 ? -c0 : 0;   // row 0, column max(c0, 0)
    int ent[2];
    uint32_t c01[2], c2[2], dd[2];
    auto load_pass = [&](int e0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + 256 * u + t;
            ent[u] = e < total ? (int)plist[e] : safe_ent;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = ent[u] >> 8, lc = ent[u] & 255;
            const int64_t p = (int64_t)(y_band + row) * W + (c0 + lc);
            const uint8_t *cp = rgb + 3 * p;
            c01[u] = (uint32_t)cp[0] | ((uint32_t)cp[1] << 8);
            c2[u] = cp[2];
            dd[u] = __float_as_uint(D[p]);
        }
    };
    load_pass(0);

    // (4) the offsets: strip totals and parts before the band, the groups'
    // sum, per-row counts of each strip
    int acc = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += 256 * u + t < n_before ? a[u] : 0;
    for (int k0 = 8 * 256; k0 < n_before; k0 += 8 * 256) {
        int e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + 256 * u + t;
            e[u] = grpcnt[k < n_before ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += k0 + 256 * u + t < n_before ? e[u] : 0;
    }
    int tot = 0, pre = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int b = 32 * u + k32;
        const int v = sj_ok && b < n_bands ? c[u] : 0;
        tot += v;
        pre += b < band ? v : 0;
    }
    for (int b0 = 4 * 32; b0 < n_bands; b0 += 4 * 32) {
        int e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + 32 * u + k32;
            e[u] = bc[b < n_bands ? b : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + 32 * u + k32;
            const int v = sj_ok && b < n_bands ? e[u] : 0;
            tot += v;
            pre += b < band ? v : 0;
        }
    }
    // strips j = 2w (lanes 0-31) and 2w + 1 (lanes 32-63) of wave w: the
    // scans' lanes 31 and 63 hold the first half's and the whole wave's sums
    {
        const int st = wave_inclusive_scan(tot), sp = wave_inclusive_scan(pre);
        const int t_lo = __builtin_amdgcn_readlane(st, 31);
        const int p_lo = __builtin_amdgcn_readlane(sp, 31);
        if (lane == 0) {
            stot[j] = t_lo;
            spre[j] = p_lo;
        } else if (lane == 32) {
            stot[j] = __builtin_amdgcn_readlane(st, 63) - t_lo;
            spre[j] = __builtin_amdgcn_readlane(sp, 63) - p_lo;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) red[wid] = acc;
    for (int e = t; e < kGroupStrips * kBandRows; e += 256) {
        const int q = e / kBandRows, row = e % kBandRows;
        start[row][q] = popc128(mlo[row], mhi[row], 8 * q, 8 * q + 8 + 2 * r);
    }
    __syncthreads();
    if (t == 0) {
        int run = red[0] + red[1] + red[2] + red[3];
        for (int q = 0; q < kGroupStrips; ++q) {
            sbase[q] = run + spre[q];
            run += stot[q];
        }
    }
    __syncthreads();
    // (5) exclusive scan over the band's rows (lane = row): wave w scans
    // strips w, w + 4; the row offsets are stored after the records
    int ro_val[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = wid + 4 * h;
        const bool rl = lane < kBandRows;
        const int v = rl ? start[rl ? lane : 0][q] : 0;
        const int incl = wave_inclusive_scan(v);
        const int st = sbase[q] + incl - v;
        ro_val[h] = st;
        // kept for the records less the row's samples left of the strip's
        // first halo column, so that a sample's index there is this plus
        // its own rank in the row
        if (rl) start[lane][q] = st - popc128(mlo[lane], mhi[lane], 0, 8 * q);
    }
    __syncthreads();
    // (6) records: each valid pixel into each strip of the group whose halo
    // holds it
    const int ts = table_stride(r);
    const int n_here = min(kGroupStrips, n_strips - s_first);
    for (int e0 = 0; e0 < total; e0 += 512) {
        if (e0 > 0) load_pass(e0);
        // wait for these loads once, here: the store counter is the same
        // in-order counter as the load counter, so a load still pending at a
        // store (the depth word is stored as loaded) would make every record
        // store wait for all earlier ones
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt/lgkmcnt any
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (e0 + 256 * u + t >= total) continue;
            const int row = ent[u] >> 8, lc = ent[u] & 255;
            const int y = y_band + row;
            if (reset_keys && lc >= r && lc < r + 64)   // one of the unit's own columns
                reset_keys[(int64_t)y * W + (c0 + lc)] = kEmptyKey;
            uint32_t rg, b0;
            float nq2h;
            colour_fields(c01[u], c2[u], rg, b0, nq2h);
            // the sample's rank among the row's samples (columns left of it)
            const int rank = popc128(mlo[row], mhi[row], 0, lc);
            const int4 sa = *reinterpret_cast<const int4 *>(&start[row][0]);
            const int4 sb = *reinterpret_cast<const int4 *>(&start[row][4]);
            const int st[kGroupStrips] = {sa.x, sa.y, sa.z, sa.w,
                                          sb.x, sb.y, sb.z, sb.w};
#pragma unroll
            for (int q = 0; q < kGroupStrips; ++q) {
                // strips q of the group with 8q <= lc < 8q + 8 + 2r
                if (q >= n_here || lc < 8 * q || lc >= 8 * q + 8 + 2 * r) continue;
                const int64_t idx = (int64_t)(st[q] + rank);
                if (idx >= capacity) continue;
                // words 0-3 are the same for every strip of this sample, so
                // their (merged) store never waits on a rewritten register
                uint32_t *o = recs + idx * kRecWords;
                o[0] = rg;
                o[1] = b0;
                o[2] = dd[u];
                o[3] = __float_as_uint(nq2h);
                o[4] = rec_table_word(lc - 8 * q, y, ts);
            }
        }
    }
    // row offsets of strips w and w + 4 (lane = row), and each strip's end
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = wid + 4 * h;
        const int s = s_first + q;
        const int y = y_band + lane;
        if (s < n_strips) {
            int *ro = rowoff + (int64_t)s * (H + 1);
            if (lane < kBandRows && y < H) ro[y] = ro_val[h];
            if (band == n_bands - 1 && lane == 0)
                ro[H] = sbase[q] - spre[q] + stot[q];   // end of strip s
        }
    }
}

// reset_keys (or null): the key image the decode read. A pixel is valid
// exactly when its key is not the empty key, so writing the empty key back
// at the valid pixels of each unit's own columns leaves the whole image
// empty for the next projection. table (or null): where to build the
// filter's spatial table for sigma_s (ks in log2 units; weights: the FP16
// range form's table of weights).
__global__ __launch_bounds__(256) void k_list_scatter(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, int r, int n_strips,
    int n_bands, const int *__restrict__ bandcnt, const int *__restrict__ grpcnt,
    int *__restrict__ rowoff, int64_t capacity, uint32_t *__restrict__ recs,
    uint64_t *__restrict__ reset_keys, float *__restrict__ table, float ks,
    bool weights) {
    // the filter's spatial table for this call, built once by workgroup 0
    // (the filter's workgroups copy it instead of building it each)
    if (table && blockIdx.x == 0) build_table(table, r, table_stride(r), ks, weights);
    int g, band;
    list_unit((n_strips + kGroupStrips - 1) / kGroupStrips, n_bands, g, band);
    list_scatter_unit(D, B, rgb, H, W, r, n_strips, n_bands, bandcnt, grpcnt, rowoff,
                      capacity, recs, g, band, reset_keys);
}

// ---------------------------------------------------------------------------
// the filter
// ---------------------------------------------------------------------------

// Scratch of one filter workgroup (LDS).
// Workgroup-level staging of a tile's halo (STAGE): the valid samples of
// the tile plus r pixels on every side are gathered once for the four
// waves (each wave streaming its own block's halo reads most pixels two to
// four times), then each wave copies the ones in its block's halo into its
// list. Capacities: samples of the tile's halo, samples of one block's.
constexpr int kTileCap = 256;
constexpr int kSubCap = 128;
// Rounds of 256 halo pixels whose loads the staging issues together: three
// covers the halo of a tile at r = 5 (676 pixels) and r = 15 (2116 pixels,
// nine rounds) without an idle round.
constexpr int kStageGroup = 3;

// rounds of 256 pixels that cover a tile's halo at radius r <= RMAX
template <int RMAX>
constexpr int stage_rounds() {
    return ((kTile + 2 * RMAX) * (kTile + 2 * RMAX) + 255) / 256;
}

template <int RMAX, bool STAGE>
struct FilterShared;

template <int RMAX>
struct FilterShared<RMAX, false> {
    float G[(2 * RMAX + 15) * table_stride(RMAX)];
    Rec recs[kWaves][64];
    float nq2h[kWaves][64];
};

template <int RMAX>
struct FilterShared<RMAX, true> {
    float G[(2 * RMAX + 15) * table_stride(RMAX)];
    Rec recs[kWaves][kSubCap];    // each wave's list (or its stream chunks)
    float nq2h[kWaves][kSubCap];
    Rec trec[kTileCap];           // the tile halo's samples, xy = x | y << 16,
                                  // rg = the colour bytes (unpacked per wave)
    int tcnt[stage_rounds<RMAX>() * kWaves];   // samples per (round, wave)
};

// Stage the valid samples of tile (tx, ty)'s halo (clipped to the image):
// every thread of the workgroup calls it. Pixel k of the halo in row-major
// order is handled in round k / 256 by thread k mod 256, so ordering the
// samples by (round, wave, lane) keeps row-major order. Returns the number
// of samples of block (bx, by)'s halo now in the wave's list (row-major,
// records as the stream writes them), or -1 when a capacity is exceeded
// (the wave then streams its halo itself).
template <int RMAX>
__device__ int tile_stage(const float *__restrict__ D, const uint8_t *__restrict__ B,
                          const uint8_t *__restrict__ rgb, int H, int W, int r,
                          int tx, int ty, int bx, int by, FilterShared<RMAX, true> &sh) {
    constexpr int kMaxRounds = stage_rounds<RMAX>();
    static_assert(kMaxRounds * kWaves <= 128 && kMaxRounds + kStageGroup - 1 <= 32,
                  "each wave scans the round counts, two per lane");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int X0 = max(tx * kTile - r, 0), X1 = min(tx * kTile + kTile + r, W);
    const int Y0 = max(ty * kTile - r, 0), Y1 = min(ty * kTile + kTile + r, H);
    const int rw = X1 - X0;                 // >= 1: the tile holds a pixel
    const int n = rw * (Y1 - Y0);
    const int rounds = (n + 255) >> 8;      // <= kMaxRounds
    // round 0: pixel tid of the halo, at (tid mod rw, tid div rw); (tid +
    // 0.5) / rw lies at least 0.5 / rw from an integer, far above the
    // product's rounding error
    const int cy0 = (int)(((float)tid + 0.5f) * __builtin_amdgcn_rcpf((float)rw));
    const int cx0 = tid - cy0 * rw;
    const uint32_t Wu = (uint32_t)W;
    const uint32_t first = (uint32_t)Y0 * Wu + (uint32_t)X0;
    const uint32_t p0 = first + (uint32_t)cy0 * Wu + (uint32_t)cx0;
    const uint32_t xy0 = (uint32_t)(X0 + cx0) | ((uint32_t)(Y0 + cy0) << 16);
    // per round: 256 pixels further
    const int sx = 256 % rw, sy = 256 / rw;
    const uint32_t dp = (uint32_t)sy * Wu + (uint32_t)sx, dp_wrap = Wu - (uint32_t)rw;
    const uint32_t dxy = (uint32_t)sx + ((uint32_t)sy << 16);
    const uint32_t dxy_wrap = (1u << 16) - (uint32_t)rw;   // x - rw, y + 1
    __syncthreads();   // the previous tile's waves have read trec and tcnt

    // (A) validity of each round's pixel, counted per (round, wave); the
    // mask bytes of kStageGroup rounds are loaded together. (Loading the
    // first rounds' sample data here already, to land under the count
    // exchange, measured 7% slower on the eight-view batch: the registers
    // it holds cost the kernel occupancy.)
    uint32_t vbits = 0;
    auto load_sample = [&](uint32_t q, uint32_t &ac, float &ad) {
        const uint32_t o3 = q * 3u;
        ac = (uint32_t)rgb[o3] | ((uint32_t)rgb[o3 + 1u] << 8) |
             ((uint32_t)rgb[o3 + 2u] << 16);
        ad = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(D) +
                                              (q << 2));
    };
    {
        int cx = cx0;
        uint32_t p = p0;
        for (int j0 = 0; j0 < rounds; j0 += kStageGroup) {
            uint32_t q[kStageGroup];
            bool in[kStageGroup];
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) {
                in[u] = (j0 + u) * 256 + tid < n;
                q[u] = in[u] ? p : first;
                cx += sx;
                p += dp;
                if (cx >= rw) {
                    cx -= rw;
                    p += dp_wrap;
                }
            }
            uint32_t m[kStageGroup];
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) m[u] = B[q[u]];
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) {
                const bool v = in[u] && m[u] != 0u;
                const uint64_t bal = __builtin_amdgcn_ballot_w64(v);
                if (lane == 0 && j0 + u < rounds)
                    sh.tcnt[(j0 + u) * kWaves + wid] = __builtin_popcountll(bal);
                vbits |= (uint32_t)v << (j0 + u);
            }
        }
    }
    __syncthreads();
    // every wave scans the counts in (round, wave) order itself (exclusive
    // prefix: entry e in lane e, entry 64 + e in lane e of the second half)
    const int ne = rounds * kWaves;
    const int ca = lane < ne ? sh.tcnt[lane] : 0;
    const int cb = lane + 64 < ne ? sh.tcnt[lane + 64] : 0;
    const int ia = wave_inclusive_scan(ca);
    const int ib = wave_inclusive_scan(cb) + __builtin_amdgcn_readlane(ia, 63);
    const int xa = ia - ca, xb = ib - cb;
    const int total = __builtin_amdgcn_readlane(ib, 63);
    if (total > kTileCap) return -1;   // the same in every wave
    auto base_of = [&](int j) -> int {   // wave-uniform j
        const int e = j * kWaves + wid;
        return e < 64 ? __builtin_amdgcn_readlane(xa, e)
                      : __builtin_amdgcn_readlane(xb, e - 64);
    };

    // (B) records of the valid pixels at their ranks, the sample data of
    // kStageGroup rounds loaded together
    {
        int cx = cx0;
        uint32_t p = p0, xy = xy0;
        for (int j0 = 0; j0 < rounds; j0 += kStageGroup) {
            uint32_t q[kStageGroup], qxy[kStageGroup];
            bool v[kStageGroup];
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) {
                v[u] = (vbits >> (j0 + u)) & 1u;
                q[u] = p;
                qxy[u] = xy;
                cx += sx;
                p += dp;
                xy += dxy;
                if (cx >= rw) {
                    cx -= rw;
                    p += dp_wrap;
                    xy += dxy_wrap;
                }
            }
            uint32_t cc[kStageGroup];   // colour bytes r | g << 8 | b << 16
            float dd[kStageGroup];
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) {
                cc[u] = 0u;
                dd[u] = 0.0f;
                if (v[u]) load_sample(q[u], cc[u], dd[u]);
            }
#pragma unroll
            for (int u = 0; u < kStageGroup; ++u) {
                const uint64_t bal = __builtin_amdgcn_ballot_w64(v[u]);
                if (j0 + u < rounds && bal != 0u) {   // uniform
                    const int b0 = base_of(j0 + u);
                    if (v[u]) {
                        const int pos = b0 + (int)__builtin_amdgcn_mbcnt_hi(
                                                 (uint32_t)(bal >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        Rec rec;
                        rec.xy = qxy[u];
                        rec.rg = cc[u];
                        rec.b0 = 0u;
                        rec.d = dd[u];
                        sh.trec[pos] = rec;
                    }
                }
            }
        }
    }
    __syncthreads();

    // (C) this wave's block halo, in order, into its list (a block outside
    // the image has nothing to filter)
    if (bx >= W || by >= H) return 0;
    const int hx0 = max(bx - r, 0), hx1 = min(bx + 8 + r, W);
    const int hy0 = max(by - r, 0), hy1 = min(by + 8 + r, H);
    const uint32_t xoff = (uint32_t)(bx - r);   // record x is x - (bx - r)
    Rec *my = sh.recs[wid];
    float *myq = sh.nq2h[wid];
    int cnt = 0;
    for (int k0 = 0; k0 < total; k0 += 64) {
        const int k = k0 + lane;
        const int kk = k < total ? k : 0;
        Rec rec = sh.trec[kk];
        const int x = (int)(rec.xy & 0xffffu), y = (int)(rec.xy >> 16);
        const bool mine = k < total && x >= hx0 && x < hx1 && y >= hy0 && y < hy1;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(mine);
        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                  (uint32_t)(bal >> 32),
                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (mine && pos < kSubCap) {
            // the colour fields are formed here, once per wave and sample,
            // rather than for every lane of every staging round
            const uint32_t c = rec.rg;
            float q2h;
            colour_fields(c & 0xffffu, c >> 16, rec.rg, rec.b0, q2h);
            rec.xy -= xoff;
            my[pos] = rec;
            myq[pos] = q2h;
        }
        cnt += __builtin_popcountll(bal);
    }
    return cnt <= kSubCap ? cnt : -1;
}

// Filter one 16x16 output tile (tx, ty) of an image with one 256-thread
// workgroup: builds the spatial table, then each wave filters its 8x8 block.
// Every thread returns normally, so callers may loop over tiles with a
// barrier between them.
template <int RMAX, int PREC, bool STAGE, bool DIRECT = false>
__device__ __forceinline__ void filter_tile(const float *__restrict__ D,
                            const uint8_t *__restrict__ B,
                            const uint8_t *__restrict__ rgb, int H, int W,
                            const FilterParams &fp, const ListArgs &la, int tx,
                            int ty, float *__restrict__ out,
                            uint8_t *__restrict__ mask, float2 *__restrict__ aux,
                            FilterShared<RMAX, STAGE> &sh, bool build = true) {
    const int r = fp.radius;
    const int ts = table_stride(r);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int lane = threadIdx.x & 63;
    const int bx = tx * kTile + (wid & 1) * 8;
    const int by = ty * kTile + (wid >> 1) * 8;
    const int i = lane & 7, j = lane >> 3;
    const int px = bx + i, py = by + j;
    const bool inside = px < W && py < H;
    // this lane's colour, from a clamped address (lanes outside the image
    // take an edge pixel's and write nothing), loaded before the table build
    // so that it lands under it
    const uint8_t *c = rgb + 3 * ((int64_t)min(py, H - 1) * W + min(px, W - 1));
    const uint8_t c0 = c[0], c1 = c[1], c2 = c[2];
    // spatial table: clamped exponents (FP32) or weights (FP16 range); a
    // caller whose previous tile had the same radius and sigma_s keeps it
    if (build) {
        if (la.table)   // uniform: built once for the call (list scatter)
            copy_table(sh.G, la.table, r, ts);
        else
            build_table(sh.G, r, ts, fp.ks, PREC != JBFD_FP32);
        __syncthreads();
    }
    // without sample lists the workgroup stages the tile's halo once
    // (every thread takes part, before any block leaves)
    int staged = -1;
    if constexpr (STAGE) {
        if (la.recs == nullptr)   // uniform
            staged = tile_stage<RMAX>(D, B, rgb, H, W, r, tx, ty, bx, by, sh);
    }
    if (bx >= W || by >= H) return;  // block of a partial tile: no outputs

    uint32_t prg, pb0;
    float nh;
    colour_fields((uint32_t)c0 | ((uint32_t)c1 << 8), c2, prg, pb0, nh);
    const float p2 = -2.0f * nh;
    // lane constant for the table index: (i + 2r + 7, py + r + 7); a sample
    // record holds (x - (bx - r), y), so one packed subtract gives
    // (dx + r + 7, dy + r + 7) in [0, 2r+14]^2
    const uint32_t lxy = (uint32_t)(i + 2 * r + 7) | ((uint32_t)(py + r + 7) << 16);
    const uint32_t gstride = 4u | ((uint32_t)(4 * ts) << 16);
    const float kr2 = 2.0f * fp.kr;
    const uint32_t lc =
        4u * ((uint32_t)(i + 2 * r + 7) + (uint32_t)ts * (uint32_t)(py + r + 7));
    const BlockWalker bw{D, B, rgb, H, W, r, la, bx, by, lane, prg, pb0, lxy,
                         gstride, lc, ts,
                         reinterpret_cast<const unsigned char *>(sh.G),
                         sh.recs[wid], sh.nq2h[wid], -fp.ks, staged,
                         DIRECT ? nh : 0.0f};

    // Pass 1: fixed per-lane shift. Every exponent E = -kr c - ks s is <= 0,
    // so a = fma(2kr, t, -kr|p|^2) + G (the fma rounds once, relative to the
    // colour exponent itself; the rounded lane constant -kr|p|^2 shifts every
    // weight of the lane alike and cancels) never overflows.
    //  FP32: the colour part is clamped at -60 and the table at -60 (the
    //        colour clamp and the sum take two fmas, Pass1Exp), so an
    //        in-window sample never underflows to zero and den > 0 exactly
    //        when the window holds a sample.
    //  FP16 range weights: w_c = 2^n v_exp_f16(f) for the colour exponent's
    //        integer part n and fraction f, times the FP32 spatial weight,
    //        accumulated in FP32; the sum of the spatial weights alone
    //        (never zero in the window) decides the mask.
    const float Mfast = -fp.kr * p2;
    float num = 0.0f, den = 0.0f, dsp = 0.0f;
    if constexpr (PREC == JBFD_FP32 && DIRECT) {
        // Without aux (no backward to serve): the walker starts each
        // sample's colour term at -(|p|^2 + |q|^2)/2, so t = -c/2 exactly and
        // one fma gives the exact exponent -kr c + G (G from the table, -inf
        // outside the window), rounded once and never above 0. No clamp:
        // a weight may underflow, so the mask comes from the sums: a lane
        // whose sum stays below 2^-16, zero included, takes the exact pass,
        // which decides it (one instruction less per sample than the
        // clamped form).
        auto stage_a = [&](float t, float g, float) { return __builtin_fmaf(kr2, t, g); };
        auto stage_b = [&](float a, float, float d) {
            const float w = __builtin_amdgcn_exp2f(a);
            num = __builtin_fmaf(w, d, num);
            den += w;
        };
        auto eat = [&](float t, float g, float d, uint32_t) {
            stage_b(stage_a(t, g, d), g, d);
        };
        bw.template walk_split<true>(
            stage_a, stage_b,
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&uv)[4]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
            },
            eat, -__builtin_inff());
        dsp = den;
    } else if constexpr (PREC == JBFD_FP32) {
        const Pass1Exp p1(kr2, Mfast);
        auto stage_a = [&](float t, float g, float) { return p1(t, g); };
        auto stage_b = [&](float a, float, float d) {
            const float w = __builtin_amdgcn_exp2f(a);
            num = __builtin_fmaf(w, d, num);
            den += w;
        };
        auto eat = [&](float t, float g, float d, uint32_t) {
            stage_b(stage_a(t, g, d), g, d);
        };
        bw.walk_split(
            stage_a, stage_b,
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&uv)[4]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
            },
            eat, -__builtin_inff());
        dsp = den;
    } else {
        // The colour exponent a = -kr c (FP32, from the exact t) is split into
        // its integer part n and fraction f in [0, 1); the FP16 exponential
        // evaluates 2^f (f rounded to FP16: at most 2^-12 off) and 2^n is
        // applied exactly to the FP32 spatial weight. Every range weight thus
        // carries the relative error of one FP16 result, whatever |a|.
        // stage_a keeps f, ws 2^n and ws 2^n d.
        auto stage_a = [&](float t, float ws, float d) {
            const float a = __builtin_fmaf(kr2, t, Mfast);
            const float n = __builtin_floorf(a);
            const float wsn = __builtin_ldexpf(ws, (int)n);
            return make_float3(a - n, wsn, wsn * d);
        };
        auto stage_b = [&](float3 a, float ws, float) {
            const float e = (float)__builtin_exp2f16((_Float16)a.x);
            num = __builtin_fmaf(e, a.z, num);
            den = __builtin_fmaf(e, a.y, den);
            dsp += ws;
        };
        auto eat = [&](float t, float ws, float d, uint32_t) {
            stage_b(stage_a(t, ws, d), ws, d);
        };
        bw.walk_split(
            stage_a, stage_b,
            [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                const uint32_t (&uv)[4]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) eat(t[u], g[u], d[u], uv[u]);
            },
            eat, 0.0f);
    }

    // Pass 2, only for lanes whose heaviest weight is below about 2^-16
    // (clamping or precision could matter there): the exact running shift
    // of consume4/consume1 over the same samples, with exact, unclamped
    // spatial exponents.
    // (DIRECT: also lanes whose sum is zero, whose window may hold samples
    // whose weights all underflowed)
    const bool weak = inside && (DIRECT || dsp > 0.0f) && den < kWeakBelow;
    float M = Mfast;
    if (__builtin_amdgcn_ballot_w64(weak) != 0) {
        float M2 = kShiftInit - fp.kr * p2, num2 = 0.0f, den2 = 0.0f;
        auto eat4 = [&](const float (&t)[4], const float (&g)[4], const float (&d)[4],
                        const uint32_t (&)[4]) {
            if (weak) consume4(t, g, d, kr2, M2, num2, den2);
        };
        auto eat1 = [&](float t, float g, float d, uint32_t) {
            if (weak) consume1(t, g, d, kr2, M2, num2, den2);
        };
        // When no entry inside the window is clamped (the corners hold the
        // largest distance, 2r^2), the FP32 table holds exactly the
        // exponents exact_g forms, with the same float operations, so the
        // exact pass's list walk reads them from the table.
        bool table_exact = false;
        if constexpr (PREC == JBFD_FP32)
            table_exact = -fp.ks * (float)(2 * r * r) >= kClampExp;
        bw.walk_exact(table_exact, eat4, eat1);
        if (weak) {
            num = num2;
            den = den2;
            M = M2;
            if constexpr (DIRECT) dsp = den2;
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

template <int RMAX, int PREC, bool STAGE, bool DIRECT>
__global__ __launch_bounds__(256) void k_jbf_fwd(
    const float *__restrict__ D, const uint8_t *__restrict__ B,
    const uint8_t *__restrict__ rgb, int H, int W, FilterParams fp,
    int tiles_x, int tiles_y, ListArgs la, float *__restrict__ out,
    uint8_t *__restrict__ mask, float2 *__restrict__ aux) {
    __shared__ FilterShared<RMAX, STAGE> sh;
    int tx, ty;
    if (!column_tile(blockIdx.x, tiles_x, tiles_y, tx, ty))
        return;  // whole workgroup leaves together
    filter_tile<RMAX, PREC, STAGE, DIRECT>(D, B, rgb, H, W, fp, la, tx, ty, out, mask,
                                           aux, sh);
}

hipError_t launch_densify_prepare(const float *D, const uint8_t *B,
                                  const uint8_t *rgb, int32_t H, int32_t W,
                                  int32_t radius, void *ws, size_t ws_bytes,
                                  hipStream_t s) {
    const ListLayout L = list_layout(H, W);
    ListViews v;
    if (!lists_possible(H, W, radius) || !list_views(ws, ws_bytes, L, v))
        return hipSuccess;  // nothing to build
    const int grid = L.n_groups * L.n_bands;   // units, see list_unit
    k_list_count<<<grid, 256, 0, s>>>(B, H, W, radius, L.n_strips, L.n_bands,
                                      v.bandcnt, v.grpcnt);
    k_list_scatter<<<grid, 256, 0, s>>>(D, B, rgb, H, W, radius, L.n_strips,
                                        L.n_bands, v.bandcnt, v.grpcnt, v.rowoff,
                                        v.capacity, v.recs, nullptr, nullptr, 0.0f,
                                        false);
    return hipGetLastError();
}

hipError_t launch_densify(const float *D, const uint8_t *B, const uint8_t *rgb,
                          int32_t H, int32_t W, const FilterParams &fp,
                          jbfd_precision prec, float *out, uint8_t *mask,
                          float *aux, void *ws, size_t ws_bytes, bool lists_ready,
                          hipStream_t s, bool table_ready) {
    const int tiles_x = (W + kTile - 1) / kTile;
    const int tiles_y = (H + kTile - 1) / kTile;
    const int n_wg = column_grid(tiles_x, tiles_y);
    ListArgs la{nullptr, nullptr, 0};
    const ListLayout L = list_layout(H, W);
    ListViews v;
    if (lists_possible(H, W, fp.radius) && list_views(ws, ws_bytes, L, v)) {
        if (!lists_ready) {
            const hipError_t e =
                launch_densify_prepare(D, B, rgb, H, W, fp.radius, ws, ws_bytes, s);
            if (e != hipSuccess) return e;
        }
        la = ListArgs{v.recs, v.rowoff, v.capacity, table_ready ? v.table : nullptr};
    }
    float2 *a2 = reinterpret_cast<float2 *>(aux);
    // with sample lists no staging (its LDS would cost the list walk
    // occupancy); without, the workgroup stages each tile's halo
    // FP32 without aux takes the direct first pass (clamped weights only
    // when the backward needs them)
    auto go = [&](auto rmax, auto prc, auto stage, float2 *ax) {
        constexpr int R = decltype(rmax)::value, PR = decltype(prc)::value;
        constexpr bool ST = decltype(stage)::value;
        if (PR == JBFD_FP32 && ax == nullptr)
            k_jbf_fwd<R, PR, ST, PR == JBFD_FP32><<<n_wg, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, tiles_y, la, out, mask, ax);
        else
            k_jbf_fwd<R, PR, ST, false><<<n_wg, 256, 0, s>>>(
                D, B, rgb, H, W, fp, tiles_x, tiles_y, la, out, mask, ax);
    };
    using F32 = std::integral_constant<int, JBFD_FP32>;
    using F16 = std::integral_constant<int, JBFD_FP16_RANGE>;
    using R16 = std::integral_constant<int, 16>;
    using R32 = std::integral_constant<int, JBFD_MAX_RADIUS>;
    using Yes = std::true_type;
    using No = std::false_type;
    const bool small = fp.radius <= 16, lists = la.recs != nullptr;
    if (prec == JBFD_FP32) {
        if (small)
            lists ? go(R16{}, F32{}, No{}, a2) : go(R16{}, F32{}, Yes{}, a2);
        else
            lists ? go(R32{}, F32{}, No{}, a2) : go(R32{}, F32{}, Yes{}, a2);
    } else {
        if (small)
            lists ? go(R16{}, F16{}, No{}, nullptr) : go(R16{}, F16{}, Yes{}, nullptr);
        else
            lists ? go(R32{}, F16{}, No{}, nullptr) : go(R32{}, F16{}, Yes{}, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_project_densify(const float *pts, int64_t n, const Pose &pose,
                                  const Intr &K, const uint8_t *rgb,
                                  const FilterParams &fp, jbfd_precision prec,
                                  uint64_t *zbuf, float *D, uint8_t *B, float *out,
                                  uint8_t *mask, void *ws, size_t ws_bytes,
                                  hipStream_t s) {
    const int H = K.h, W = K.w;
    const ListLayout L = list_layout(H, W);
    ListViews v;
    if (!lists_possible(H, W, fp.radius) || !list_views(ws, ws_bytes, L, v)) {
        // no lists: the recycling projection, then the streaming filter
        hipError_t e = launch_project(pts, n, pose, K, zbuf, D, B, true, s);
        if (e != hipSuccess) return e;
        return launch_densify(D, B, rgb, H, W, fp, prec, out, mask, nullptr, ws,
                              ws_bytes, false, s);
    }
    hipError_t e = launch_project_keys(pts, n, pose, K, zbuf, s);
    if (e != hipSuccess) return e;
    const int grid = L.n_groups * L.n_bands;   // units, see list_unit
    k_decode_count<<<grid, 256, 0, s>>>(zbuf, H, W, fp.radius, L.n_strips, L.n_bands,
                                        D, B, v.bandcnt, v.grpcnt);
    k_list_scatter<<<grid, 256, 0, s>>>(D, B, rgb, H, W, fp.radius, L.n_strips,
                                        L.n_bands, v.bandcnt, v.grpcnt, v.rowoff,
                                        v.capacity, v.recs, zbuf, v.table, fp.ks,
                                        prec != JBFD_FP32);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_densify(D, B, rgb, H, W, fp, prec, out, mask, nullptr, ws, ws_bytes,
                          true, s, true);
}

}  // namespace jbfd

namespace jbfd {

// A tile of a view whose radius exceeds the launch's table bound: its
// outputs are zero (no valid pixel) and the batch's error word records it.
__device__ inline void refuse_tile(BatchHeader *hdr, const BatchView &v, int tx, int ty) {
    const int px = tx * kTile + (int)(threadIdx.x & 15);
    const int py = ty * kTile + (int)(threadIdx.x >> 4);
    if (px < v.W && py < v.H) {
        const int64_t p = (int64_t)py * v.W + px;
        v.out[p] = 0.0f;
        v.mask[p] = 0;
    }
    if (threadIdx.x == 0) atomicOr(&hdr->error, kBatchErrRadius);
}

// Filter tiles of every view of a batch: a fixed grid walks the flattened
// tile space (views back to back); each workgroup finds its view by a
// binary search of the table's tile offsets (wave-uniform scalar loads).
template <int RMAX, int PREC, bool STAGE>
__global__ __launch_bounds__(256) void k_batch_filter(BatchHeader *__restrict__ hdr,
                                                      const BatchView *__restrict__ views,
                                                      bool use_lists) {
    __shared__ FilterShared<RMAX, STAGE> sh;
    const int n_views = hdr->n_views;
    const int total = hdr->total_tiles;
    // the spatial table depends on the radius and sigma_s only: it is
    // rebuilt when a tile's view differs in either from the previous tile's
    int cur_r = -1;
    float cur_ks = 0.0f;
    // t only grows, so the view is looked up again only when t passes the
    // next view's first tile (a binary search per tile, a chain of
    // dependent scalar loads, cost the batch 35 us of waiting)
    int next_off = -1;
    BatchView v;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        if (t >= next_off) {   // uniform
            const int lo = batch_view_of<&BatchView::tile_off>(views, n_views, t);
            v = global_view(views[lo]);
            next_off = lo + 1 < n_views ? views[lo + 1].tile_off : total;
        }
        const int local = t - v.tile_off;
        const int ty = local / v.tiles_x, tx = local - ty * v.tiles_x;
        if (v.radius > RMAX) {   // uniform: the table would not fit
            refuse_tile(hdr, v, tx, ty);
            continue;
        }
        const FilterParams fp{v.radius, v.kr, v.ks};
        const bool rebuild = fp.radius != cur_r || fp.ks != cur_ks;  // uniform
        if (rebuild && cur_r >= 0) __syncthreads();  // old table no longer read
        // lists only when this run built them (recs null: stream)
        const ListArgs la{use_lists ? v.recs : nullptr, v.rowoff, v.capacity};
        filter_tile<RMAX, PREC, STAGE, PREC == JBFD_FP32>(v.sd, v.sv, v.rgb, v.H, v.W,
                                                          fp, la, tx, ty, v.out, v.mask,
                                                          nullptr, sh, rebuild);
        cur_r = fp.radius;
        cur_ks = fp.ks;
    }
}

// Sample lists of every view that has a list workspace: fixed grids walk the
// flattened (view, strip group, row band) units; the workgroup of a unit
// runs the single-view kernels' body for it. Both kernels exit at once when
// the batch has no lists.
__global__ __launch_bounds__(256) void k_batch_list_count(const BatchHeader *__restrict__ hdr,
                                                          const BatchView *__restrict__ views) {
    const int n_views = hdr->n_views, units = hdr->list_units;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const BatchView v =
            global_view(views[batch_view_of<&BatchView::unit_off>(views, n_views, u)]);
        const int local = u - v.unit_off;
        const int band = local / v.n_groups, g = local - band * v.n_groups;
        list_count_unit(v.sv, v.H, v.W, v.radius, v.n_strips, v.n_bands, v.bandcnt,
                        v.grpcnt, g, band);
        __syncthreads();   // the next unit reuses the LDS
    }
}

__global__ __launch_bounds__(256) void k_batch_list_scatter(const BatchHeader *__restrict__ hdr,
                                                            const BatchView *__restrict__ views) {
    const int n_views = hdr->n_views, units = hdr->list_units;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const BatchView v =
            global_view(views[batch_view_of<&BatchView::unit_off>(views, n_views, u)]);
        const int local = u - v.unit_off;
        const int band = local / v.n_groups, g = local - band * v.n_groups;
        list_scatter_unit(v.sd, v.sv, v.rgb, v.H, v.W, v.radius, v.n_strips,
                          v.n_bands, v.bandcnt, v.grpcnt, v.rowoff, v.capacity,
                          v.recs, g, band);
        __syncthreads();   // the next unit reuses the LDS
    }
}

hipError_t launch_batch_lists(const BatchHeader *hdr, const BatchView *views,
                              hipStream_t s) {
    const int grid = 2048;   // 8 workgroups per CU
    k_batch_list_count<<<grid, 256, 0, s>>>(hdr, views);
    k_batch_list_scatter<<<grid, 256, 0, s>>>(hdr, views);
    return hipGetLastError();
}

hipError_t launch_batch_filter(BatchHeader *hdr, const BatchView *views,
                               int32_t max_radius, jbfd_precision prec,
                               bool use_lists, hipStream_t s) {
    // views with sample lists (JBFD_BATCH_LISTS) walk them; the others
    // stage each tile's halo, which leaves LDS for 6 workgroups per CU at
    // RMAX = 16 (a view streams the same way with or without the flag)
    const int grid = 1536;
    if (max_radius <= 16) {
        if (prec == JBFD_FP32)
            k_batch_filter<16, JBFD_FP32, true><<<grid, 256, 0, s>>>(hdr, views, use_lists);
        else
            k_batch_filter<16, JBFD_FP16_RANGE, true><<<grid, 256, 0, s>>>(hdr, views,
                                                                           use_lists);
    } else {
        if (prec == JBFD_FP32)
            k_batch_filter<JBFD_MAX_RADIUS, JBFD_FP32, true><<<grid, 256, 0, s>>>(
                hdr, views, use_lists);
        else
            k_batch_filter<JBFD_MAX_RADIUS, JBFD_FP16_RANGE, true><<<grid, 256, 0, s>>>(
                hdr, views, use_lists);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the whole batch in one persistent launch
// ---------------------------------------------------------------------------
//
// The key buffers hold only empty keys on entry (every batch run leaves
// them so: its decode writes the empty key back over each key that is not
// empty), so
// the run has no clearing pass. Work items, numbered in this order (each
// part view by view):
//   [0, P)          projection chunks (kFusedPtChunk points),
//   [P, P + C)      decode chunks (kFusedPxChunk pixels),
//   [P + C, ...)    filter items (kFusedTiles consecutive tiles each).
// An item waits only for earlier items of its own view: a decode chunk for
// the view's projection chunks, a filter item for its decode chunks. Every
// decode comes before every filter item in every queue, so a filter item
// never waits on a decode that some queue has not reached because its
// workgroups are held by earlier filter items (with each view's decode just
// before its own filter items, workgroups averaged 0.34 ms of waiting on the
// eight-view batch). The items are dealt to kQueues queues in turns of
// kQueueRun consecutive items; workgroup w takes the items of queue
// w % kQueues in increasing order (one atomic per item on that queue's
// counter: one shared counter for every item measured 0.4 ms of hand-outs
// alone on the eight-view batch, the atomics on one address being served
// one after another). A workgroup claims its next item while it works on
// the current one and starts it only after. So the lowest unfinished item,
// whose queue has handed out every earlier item of its own, is held by a
// workgroup of that queue that works on it or is free to take it, and it
// depends only on finished items: the queues advance and every wait ends as
// long as each queue has a resident workgroup (the first kQueues workgroups
// of the grid cover every queue).
//
// Data passes between items of different workgroups, which may sit on
// different XCDs with separate L2 caches. The keys are lowered by atomicMin
// (performed at the memory side, coherent across XCDs) and read back by
// the decode with relaxed agent-scope loads. The decode writes the sparse
// depth and mask with write-through stores (relaxed agent-scope atomic
// stores), each cache line by one decode chunk; the filter then reads them
// with ordinary loads: no L2
// holds a line of them from before (the launch starts with no stale lines,
// as every launch does, and nothing reads a view's sparse image before its
// decode is published), so every L2 fetches them fresh. The decode's
// write-back of empty keys is read only by the next launch. An item is
// published when every wave has waited for its own stores and atomics to
// complete (s_waitcnt vmcnt(0)) and then one thread increments the view's
// counter; a dependent item polls the counter with coherent loads. No L2
// write-back or invalidation is needed (an agent-scope release or acquire
// fence would write back or invalidate the whole L2 once per item).
//
// Waits are bounded: after kSpinLimit polls the item sets kBatchErrWait in
// the header and runs anyway, so the launch always ends (its results are
// then not to be trusted, and jbfd_batch_check reports it). The last
// workgroup to finish resets the queues and the counters, so a captured
// launch can be replayed on the same table.

constexpr int kSpinLimit = 1 << 22;   // polls (about 0.1 s) before giving up

__device__ inline void store_coherent(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(uint8_t *p, uint8_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t load_coherent(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t load_coherent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every vector memory access this wave has issued has completed (stores and
// atomics acknowledged); the clobber keeps the compiler from moving memory
// accesses across the wait.
__device__ inline void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The workgroup's item is done: count it for its view.
__device__ inline void publish(uint32_t *counter) {
    wait_memory();
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(counter, 1u);
}

// Wait until *counter reaches need (thread 0 polls, the workgroup waits at
// the barrier). False when the wait gave up.
__device__ inline bool await_count(const uint32_t *counter, uint32_t need,
                                   BatchHeader *hdr, int &s_ok) {
    if (threadIdx.x == 0) {
        int polls = 0;
        while (load_coherent(counter) < need) {
            if (++polls > kSpinLimit) {
                atomicOr(&hdr->error, kBatchErrWait);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        s_ok = polls <= kSpinLimit;
    }
    __syncthreads();
    return s_ok != 0;
}

__device__ inline int pixel_items(const BatchView &v) {
    return (int)(((int64_t)v.W * v.H + kFusedPxChunk - 1) / kFusedPxChunk);
}

__device__ inline int point_items(const BatchView &v) {
    return (int)((v.n_pts + kFusedPtChunk - 1) / kFusedPtChunk);
}

// points [c kFusedPtChunk, (c + 1) kFusedPtChunk) into the key image
__device__ inline void project_chunk(const BatchView &v, int c) {
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(v.zbuf);
    const int64_t i0 = (int64_t)c * kFusedPtChunk + threadIdx.x;
    // not unrolled: several projections in flight would raise the register
    // count of the whole kernel above the filter's
#pragma unroll 1
    for (int j = 0; j < kFusedPtChunk / 256; ++j) {
        const int64_t i = i0 + 256 * j;
        if (i >= v.n_pts) break;
        unsigned long long key;
        int64_t pix;
        if (project_one(v.pts, i, v.pose, v.fx, v.fy, v.cx, v.cy, v.W, v.H, key, pix))
            atomicMin(keys + pix, key);
    }
}

// keys of the chunk's pixels -> sparse depth (0 where empty) and 0/1 mask,
// four consecutive pixels per thread and pass; the empty key is written
// back over each key that is not empty (ordinary stores: only the next
// launch reads them)
__device__ inline void decode_chunk(const BatchView &v, int c) {
    const int64_t npix = (int64_t)v.W * v.H;
    const bool vec = ((reinterpret_cast<uintptr_t>(v.sd) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(v.sv) & 3) == 0) &&
                     ((reinterpret_cast<uintptr_t>(v.zbuf) & 15) == 0);
    for (int pass = 0; pass < kFusedPxChunk / 1024; ++pass) {
        const int64_t p0 = (int64_t)c * kFusedPxChunk + 1024 * pass + 4 * (int64_t)threadIdx.x;
        if (vec && p0 + 4 <= npix) {
            uint32_t d[4], m = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t key = load_coherent(v.zbuf + p0 + k);
                const bool hit = key != kEmptyKey;
                d[k] = hit ? (uint32_t)(key >> 32) : 0u;   // the bits of float Z, or +0
                m |= (uint32_t)hit << (8 * k);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((m >> (8 * k)) & 1u) v.zbuf[p0 + k] = kEmptyKey;
            // (two 8-byte stores: a 16-byte store with this cache policy
            // exists only as inline assembly, whose data registers the
            // compiler would not protect until the store has read them)
            store_coherent(reinterpret_cast<uint64_t *>(v.sd + p0),
                           (uint64_t)d[0] | ((uint64_t)d[1] << 32));
            store_coherent(reinterpret_cast<uint64_t *>(v.sd + p0 + 2),
                           (uint64_t)d[2] | ((uint64_t)d[3] << 32));
            store_coherent(reinterpret_cast<uint32_t *>(v.sv + p0), m);
        } else {
            for (int64_t p = p0; p < npix && p < p0 + 4; ++p) {
                const uint64_t key = load_coherent(v.zbuf + p);
                const bool hit = key != kEmptyKey;
                store_coherent(v.sd + p, hit ? __uint_as_float((uint32_t)(key >> 32)) : 0.0f);
                store_coherent(v.sv + p, (uint8_t)hit);
                if (hit) v.zbuf[p] = kEmptyKey;
            }
        }
    }
}

// The k-th item of queue q: queues take turns of kQueueRun consecutive
// items, so each queue's items rise with k and keep neighbours together.
__device__ inline int queue_item(int q, uint32_t k) {
    const int turn = (int)(k / kQueueRun), within = (int)(k % kQueueRun);
    return (turn * kQueues + q) * kQueueRun + within;
}

// Six waves per SIMD at RMAX = 16: 80 registers, none spilled (at eight, as
// the staged filter kernel has, 14 registers of loop state go to scratch
// and the eight-view batch took 0.275 ms; at seven, 2 and 0.258 ms; at six
// 0.253 ms); the LDS of the halo staging also leaves room for six
// workgroups per CU. At RMAX = 32 the LDS allows three.
template <int RMAX, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RMAX <= 16 ? 6 : 3)))
void k_batch_fused(BatchHeader *__restrict__ hdr, const BatchView *__restrict__ views) {
    __shared__ FilterShared<RMAX, true> sh;
    __shared__ int s_item, s_ok;
    const int n_views = hdr->n_views;
    unsigned char *state =
        reinterpret_cast<unsigned char *>(const_cast<BatchView *>(views) + n_views);
    BatchLine *queues = reinterpret_cast<BatchLine *>(state);
    BatchCounters *cnt = reinterpret_cast<BatchCounters *>(state + kQueues * sizeof(BatchLine));
    const int C = hdr->fpx_chunks, P = hdr->fpt_chunks;
    const int total = P + C + hdr->ftile_items;
    const int q = (int)(blockIdx.x % kQueues);
    uint32_t *turn = &queues[q].n;
    int cur_r = -1;       // radius and sigma_s of the spatial table in LDS
    float cur_ks = 0.0f;
    if (threadIdx.x == 0) s_item = queue_item(q, atomicAdd(turn, 1u));
    __syncthreads();
    int item = s_item;
    while (item < total) {
        int next = 0;
        if (threadIdx.x == 0) next = queue_item(q, atomicAdd(turn, 1u));
        if (item < P) {
            const int v = batch_view_of<&BatchView::fpt_off>(views, n_views, item);
            project_chunk(global_view(views[v]), item - views[v].fpt_off);
            publish(&cnt[v].projected.n);
        } else if (item < P + C) {
            const int c = item - P;
            const int v = batch_view_of<&BatchView::fpx_off>(views, n_views, c);
            const BatchView bv = global_view(views[v]);
            await_count(&cnt[v].projected.n, point_items(bv), hdr, s_ok);
            decode_chunk(bv, c - bv.fpx_off);
            publish(&cnt[v].decoded.n);
        } else {
            const int t = item - P - C;
            const int v = batch_view_of<&BatchView::ftile_off>(views, n_views, t);
            const BatchView bv = global_view(views[v]);
            const int t0 = kFusedTiles * (t - bv.ftile_off);
            if (bv.radius > RMAX) {   // uniform: the table would not fit
                for (int lt = t0; lt < min(t0 + kFusedTiles, bv.n_tiles); ++lt)
                    refuse_tile(hdr, bv, lt % bv.tiles_x, lt / bv.tiles_x);
            } else {
                await_count(&cnt[v].decoded.n, pixel_items(bv), hdr, s_ok);
                const FilterParams fp{bv.radius, bv.kr, bv.ks};
                // the previous item ended at a barrier, so its table reads
                // are over before a rebuild; the tiles of one item share it
                bool rebuild = fp.radius != cur_r || fp.ks != cur_ks;
                const ListArgs none{nullptr, nullptr, 0};
                for (int lt = t0; lt < min(t0 + kFusedTiles, bv.n_tiles); ++lt) {
                    filter_tile<RMAX, PREC, true, PREC == JBFD_FP32>(
                        bv.sd, bv.sv, bv.rgb, bv.H, bv.W, fp, none,
                                            lt % bv.tiles_x, lt / bv.tiles_x, bv.out,
                                            bv.mask, nullptr, sh, rebuild);
                    rebuild = false;
                }
                cur_r = fp.radius;
                cur_ks = fp.ks;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_item = next;
        __syncthreads();
        item = s_item;
    }
    // the last workgroup out resets the queues and counters for the next
    // run on this table
    if (threadIdx.x == 0 && atomicAdd(&hdr->exited, 1u) == gridDim.x - 1) {
        for (int k = 0; k < kQueues; ++k) store_coherent(&queues[k].n, 0u);
        for (int v = 0; v < n_views; ++v) {
            store_coherent(&cnt[v].projected.n, 0u);
            store_coherent(&cnt[v].decoded.n, 0u);
        }
        store_coherent(&hdr->exited, 0u);
    }
}

hipError_t launch_batch_fused(void *d_table, int32_t max_radius, jbfd_precision prec,
                              hipStream_t s) {
    BatchHeader *hdr = static_cast<BatchHeader *>(d_table);
    const BatchView *views = reinterpret_cast<const BatchView *>(
        static_cast<const unsigned char *>(d_table) + sizeof(BatchHeader));
    // six workgroups per CU are resident at RMAX = 16 (three at 32); the
    // others start as those finish and find the queues empty (grids of
    // 1536 and 1792 measured the same)
    const int grid = 2048;
    if (max_radius <= 16) {
        if (prec == JBFD_FP32)
            k_batch_fused<16, JBFD_FP32><<<grid, 256, 0, s>>>(hdr, views);
        else
            k_batch_fused<16, JBFD_FP16_RANGE><<<grid, 256, 0, s>>>(hdr, views);
    } else {
        if (prec == JBFD_FP32)
            k_batch_fused<JBFD_MAX_RADIUS, JBFD_FP32><<<grid, 256, 0, s>>>(hdr, views);
        else
            k_batch_fused<JBFD_MAX_RADIUS, JBFD_FP16_RANGE><<<grid, 256, 0, s>>>(hdr, views);
    }
    return hipGetLastError();
}

}  // namespace jbfd

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
//   k_decode     key image -> float depth (0 where empty) and 0/1 mask; the
//                recycling form also writes the empty key back, so a frame
//                loop that reuses its key buffer needs no k_fill_keys.
//
// k_project_motion is k_project for afterimage removal (Sec. 4.1): points of
// older sweeps that land in a moving pixel are dropped before the atomic.
//
// Traffic per frame: 12N bytes of points, 8HW to clear, the atomics, 8HW
// read + 5HW written by the decode.
#include <type_traits>

#include "project_common.hpp"

namespace jbfd {

// key buffer as the decode sees it: read-only, or written back with RESET
template <bool RESET>
using KeyPtr = std::conditional_t<RESET, uint64_t *, const uint64_t *__restrict__>;

// Eight keys per thread per step, as four 16-byte stores that are each
// contiguous across the workgroup (2048 keys per workgroup and step).
__global__ __launch_bounds__(256) void k_fill_keys(uint64_t *__restrict__ keys,
                                                   int64_t n) {
    const bool vec = (reinterpret_cast<uintptr_t>(keys) & 15) == 0;
    const int64_t step = (int64_t)gridDim.x * 2048;
    for (int64_t base = (int64_t)blockIdx.x * 2048; base < n; base += step) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + 2 * ((int64_t)threadIdx.x + 256 * j);
            if (vec && i + 1 < n) {
                *reinterpret_cast<ulonglong2 *>(keys + i) =
                    make_ulonglong2(kEmptyKey, kEmptyKey);
            } else if (i < n) {
                keys[i] = kEmptyKey;
                if (i + 1 < n) keys[i + 1] = kEmptyKey;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_project(const float *__restrict__ pts,
                                                 int64_t n, Pose P, Intr K,
                                                 unsigned long long *__restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        unsigned long long key;
        int64_t pix;
        if (project_one(pts, i, P.m, K.fx, K.fy, K.cx, K.cy, K.w, K.h, key, pix))
            atomicMin(keys + pix, key);
    }
}

// k_project for a merged cloud of several sweeps: a point from a sweep other
// than `latest` that lands in a moving pixel of `motion` is dropped.
__global__ __launch_bounds__(256) void k_project_motion(
    const float *__restrict__ pts, int64_t n, const int8_t *__restrict__ sweep,
    int8_t latest, const uint8_t *__restrict__ motion, Pose P, Intr K,
    unsigned long long *__restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        unsigned long long key;
        int64_t pix;
        if (!project_one(pts, i, P.m, K.fx, K.fy, K.cx, K.cy, K.w, K.h, key, pix))
            continue;
        if (sweep[i] != latest && motion[pix]) continue;
        atomicMin(keys + pix, key);
    }
}

// Decode pixels [p0, min(p0+4, npix)): two 16-byte key loads, one 16-byte
// depth store and one 4-byte mask store when aligned, else per pixel. With
// RESET the empty key is written back over each key that is not empty, so
// the buffer needs no clearing before the next projection into it (the
// other keys are empty already; on a sparse image most lines of the key
// buffer are then not written at all).
template <bool RESET>
__device__ inline void decode4(KeyPtr<RESET> keys, int64_t npix, int64_t p0, bool vec,
                               float *__restrict__ depth, uint8_t *__restrict__ valid) {
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
        if constexpr (RESET) {
            for (int t = 0; t < 4; ++t)
                if (k[t] != kEmptyKey) keys[p0 + t] = kEmptyKey;
        }
    } else {
        for (int64_t p = p0; p < npix && p < p0 + 4; ++p) {
            const uint64_t k = keys[p];
            const bool hit = k != kEmptyKey;
            if (depth) depth[p] = hit ? __uint_as_float((uint32_t)(k >> 32)) : 0.0f;
            if (valid) valid[p] = (uint8_t)hit;
            if constexpr (RESET)
                if (hit) keys[p] = kEmptyKey;
        }
    }
}

__device__ inline bool decode_vec_ok(const uint64_t *keys, const float *depth,
                                     const uint8_t *valid) {
    return ((reinterpret_cast<uintptr_t>(depth) & 15) == 0) &&
           ((reinterpret_cast<uintptr_t>(valid) & 3) == 0) &&
           ((reinterpret_cast<uintptr_t>(keys) & 15) == 0);
}

template <bool RESET>
__global__ __launch_bounds__(256) void k_decode(KeyPtr<RESET> keys, int64_t npix,
                                                float *__restrict__ depth,
                                                uint8_t *__restrict__ valid) {
    const int64_t groups = (npix + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool vec = decode_vec_ok(keys, depth, valid);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
         g += stride)
        decode4<RESET>(keys, npix, g * 4, vec, depth, valid);
}

// ---------------------------------------------------------------------------
// batches: fixed grids that loop over the views of a descriptor table and
// grid-stride over each view's pixels or points
// ---------------------------------------------------------------------------

// Each workgroup takes chunks of kBatchChunk elements; chunk c belongs to
// the view found by a scalar binary search of the chunk prefixes, so every
// view's work is spread over the whole grid at once. The key buffers hold
// only empty keys on entry and the decode writes the empty key back, so
// there is no clearing pass.

__global__ __launch_bounds__(256) void k_batch_project(const BatchHeader *__restrict__ hdr,
                                                       const BatchView *__restrict__ views) {
    const int n_views = hdr->n_views, chunks = hdr->pt_chunks;
    for (int c = blockIdx.x; c < chunks; c += gridDim.x) {
        const BatchView bv =
            global_view(views[batch_view_of<&BatchView::pt_chunk_off>(views, n_views, c)]);
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(bv.zbuf);
        const int64_t i0 = (int64_t)(c - bv.pt_chunk_off) * kBatchChunk + threadIdx.x;
        // four points per thread, 256 apart (coalesced); every point's
        // projection is independent, its atomic needs no result
#pragma unroll
        for (int j = 0; j < kBatchChunk / 256; ++j) {
            const int64_t i = i0 + 256 * j;
            if (i >= bv.n_pts) break;
            unsigned long long key;
            int64_t pix;
            if (project_one(bv.pts, i, bv.pose, bv.fx, bv.fy, bv.cx, bv.cy, bv.W,
                            bv.H, key, pix))
                atomicMin(keys + pix, key);
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_decode(const BatchHeader *__restrict__ hdr,
                                                      const BatchView *__restrict__ views) {
    const int n_views = hdr->n_views, chunks = hdr->px_chunks;
    for (int c = blockIdx.x; c < chunks; c += gridDim.x) {
        const BatchView bv =
            global_view(views[batch_view_of<&BatchView::px_chunk_off>(views, n_views, c)]);
        const int64_t npix = (int64_t)bv.W * bv.H;
        const int64_t p0 = (int64_t)(c - bv.px_chunk_off) * kBatchChunk +
                           4 * (int64_t)threadIdx.x;
        // the empty key is written back: every batch run leaves its key
        // buffers empty, as the one-launch run requires them on entry
        if (p0 < npix)
            decode4<true>(bv.zbuf, npix, p0, decode_vec_ok(bv.zbuf, bv.sd, bv.sv),
                          bv.sd, bv.sv);
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
                          uint8_t *valid, bool recycle, hipStream_t s) {
    const int64_t npix = (int64_t)K.w * K.h;
    if (!recycle) k_fill_keys<<<grid_for(npix, 2048), 256, 0, s>>>(zbuf, npix);
    if (n > 0)
        k_project<<<grid_for(n, 256), 256, 0, s>>>(
            pts, n, pose, K, reinterpret_cast<unsigned long long *>(zbuf));
    if (recycle)
        k_decode<true><<<grid_for(npix, 1024), 256, 0, s>>>(zbuf, npix, depth, valid);
    else if (depth || valid)
        k_decode<false><<<grid_for(npix, 1024), 256, 0, s>>>(zbuf, npix, depth, valid);
    return hipGetLastError();
}

hipError_t launch_project_keys(const float *pts, int64_t n, const Pose &pose,
                               const Intr &K, uint64_t *zbuf, hipStream_t s) {
    if (n > 0)
        k_project<<<grid_for(n, 256), 256, 0, s>>>(
            pts, n, pose, K, reinterpret_cast<unsigned long long *>(zbuf));
    return hipGetLastError();
}

hipError_t launch_fill_keys(uint64_t *zbuf, int64_t npix, hipStream_t s) {
    k_fill_keys<<<grid_for(npix, 2048), 256, 0, s>>>(zbuf, npix);
    return hipGetLastError();
}

hipError_t launch_project_motion(const float *pts, int64_t n, const int8_t *sweep,
                                 int8_t latest, const uint8_t *motion,
                                 const Pose &P, const Intr &K, uint64_t *zbuf,
                                 float *depth, uint8_t *valid, hipStream_t s) {
    const int64_t npix = (int64_t)K.w * K.h;
    k_fill_keys<<<grid_for(npix, 2048), 256, 0, s>>>(zbuf, npix);
    if (n > 0)
        k_project_motion<<<grid_for(n, 256), 256, 0, s>>>(
            pts, n, sweep, latest, motion, P, K,
            reinterpret_cast<unsigned long long *>(zbuf));
    if (depth || valid)
        k_decode<false><<<grid_for(npix, 1024), 256, 0, s>>>(zbuf, npix, depth, valid);
    return hipGetLastError();
}

hipError_t launch_batch(void *d_table, int32_t max_radius, bool use_lists,
                        jbfd_precision prec, hipStream_t s) {
    BatchHeader *hdr = static_cast<BatchHeader *>(d_table);
    const BatchView *views = reinterpret_cast<const BatchView *>(
        static_cast<const unsigned char *>(d_table) + sizeof(BatchHeader));
    const int grid = 2048;   // eight workgroups per CU, striding over chunks
    k_batch_project<<<grid, 256, 0, s>>>(hdr, views);
    k_batch_decode<<<grid, 256, 0, s>>>(hdr, views);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (use_lists) {
        e = launch_batch_lists(hdr, views, s);
        if (e != hipSuccess) return e;
    }
    return launch_batch_filter(hdr, views, max_radius, prec, use_lists, s);
}

}  // namespace jbfd

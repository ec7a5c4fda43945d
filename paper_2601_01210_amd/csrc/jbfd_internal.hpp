// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/jbfd.h"

namespace jbfd {

// Camera-from-world [R|t] passed by value to kernels.
struct Pose {
    double m[12];
};

struct Intr {
    double fx, fy, cx, cy;
    int32_t w, h;
};

constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kTileEdge = 16;   // filter workgroup tile edge in pixels

// Filter parameters in log2 units: weight = exp2(-kr*c - ks*s), with
// kr = log2(e) / (2 sigma_r^2) and ks = log2(e) / (2 sigma_s^2).
struct FilterParams {
    int32_t radius;
    float kr;
    float ks;
};

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_project(const float *pts, int64_t n, const Pose &pose,
                          const Intr &K, uint64_t *zbuf, float *depth,
                          uint8_t *valid, bool recycle, hipStream_t s);
hipError_t launch_fill_keys(uint64_t *zbuf, int64_t npix, hipStream_t s);
// only the atomics of the projection (no clear, no decode)
hipError_t launch_project_keys(const float *pts, int64_t n, const Pose &pose,
                               const Intr &K, uint64_t *zbuf, hipStream_t s);
hipError_t launch_project_densify(const float *pts, int64_t n, const Pose &pose,
                                  const Intr &K, const uint8_t *rgb,
                                  const FilterParams &fp, jbfd_precision prec,
                                  uint64_t *zbuf, float *D, uint8_t *B, float *out,
                                  uint8_t *mask, void *ws, size_t ws_bytes,
                                  hipStream_t s);

// table_ready: the workspace holds this call's spatial table (built by the
// list scatter of jbfd_project_densify with the same radius, sigma_s and
// precision)
hipError_t launch_densify(const float *D, const uint8_t *B, const uint8_t *rgb,
                          int32_t H, int32_t W, const FilterParams &fp,
                          jbfd_precision prec, float *out, uint8_t *mask,
                          float *aux, void *ws, size_t ws_bytes, bool lists_ready,
                          hipStream_t s, bool table_ready = false);

hipError_t launch_densify_prepare(const float *D, const uint8_t *B,
                                  const uint8_t *rgb, int32_t H, int32_t W,
                                  int32_t radius, void *ws, size_t ws_bytes,
                                  hipStream_t s);

size_t densify_ws_bytes(int32_t H, int32_t W, int32_t r, int64_t max_samples);

hipError_t launch_densify_backward(const float *D, const uint8_t *B,
                                   const uint8_t *rgb, int32_t H, int32_t W,
                                   const FilterParams &fp, float sigma_s,
                                   float sigma_r, const float *out,
                                   const float *aux, const float *g,
                                   float *grad_d, double *grad_sigmas,
                                   void *ws, hipStream_t s);

size_t backward_ws_bytes(int32_t H, int32_t W);

// Device-side descriptor table of a batch (written by jbfd_batch_prepare).
struct BatchView {
    const float *pts;
    int64_t n_pts;
    double pose[12];
    double fx, fy, cx, cy;
    int32_t W, H;
    const uint8_t *rgb;
    uint64_t *zbuf;
    float *sd;
    uint8_t *sv;
    float *out;
    uint8_t *mask;
    int32_t radius;
    float kr, ks;
    int32_t tiles_x;
    int32_t tile_off;   // exclusive prefix of filter tiles over the views
    int32_t n_tiles;
    int32_t px_chunk_off;   // exclusive prefix of kBatchChunk-pixel chunks
    int32_t pt_chunk_off;   // exclusive prefix of kBatchChunk-point chunks
    // sample lists in the view's workspace (recs == nullptr: the filter
    // streams the halo); list units are (strip group, row band) pairs
    uint32_t *recs;
    int *rowoff;
    int *bandcnt;
    int *grpcnt;
    int64_t capacity;       // records the workspace holds
    int32_t n_strips, n_groups, n_bands;
    int32_t unit_off;       // exclusive prefix of list units over the views
    // one-launch run: exclusive prefixes over the views of its decode chunks
    // (kFusedPxChunk pixels), its projection chunks (kFusedPtChunk points)
    // and its filter items (kFusedTiles tiles)
    int32_t fpx_off;
    int32_t fpt_off;
    int32_t ftile_off;
    int32_t pad_;
};

// Elements (pixels or points) one workgroup handles per chunk of the
// launch-sequence batch.
constexpr int kBatchChunk = 1024;

// Work items of the one-launch batch: large enough that handing them out
// costs little next to their work (each hand-out is an atomic on a shared
// counter), small enough that 2048 workgroups share them evenly. (On the
// eight-view batch: decode items of 1024, 2048 and 4096 pixels measured
// 0.256, 0.235 and 0.268 ms; projection items of 256, 512 and 1024 points
// 0.228, 0.235 and 0.244 ms; 2, 4 and 8 filter tiles 0.239, 0.235 and
// 0.260 ms, and then, with 256 points, 3 and 4 tiles 0.224 and 0.228 ms.)
constexpr int kFusedPxChunk = 2048;   // pixels per decode item
constexpr int kFusedPtChunk = 256;    // points per projection item (a
                                      // multiple of 256: one per thread)
constexpr int kFusedTiles = 3;        // filter tiles per item (consecutive in
                                      // the view's row-major tile order)
// work queues, workgroup w uses w % kQueues (16, 32, 64 and 128 queues
// measured 0.256, 0.250-0.255, 0.251 and 0.259 ms on the eight-view batch)
constexpr int kQueues = 64;
constexpr int kQueueRun = 4;          // consecutive items per queue turn

struct BatchHeader {
    int32_t n_views;
    int32_t total_tiles;
    int32_t px_chunks;
    int32_t pt_chunks;
    int32_t list_units;     // list units of every view with lists
    int32_t max_radius;     // largest radius over the views
    int32_t fpx_chunks;     // one-launch run: decode items
    int32_t fpt_chunks;     //   projection items
    int32_t ftile_items;    //   filter items
    // Written by the one-launch run (zero in a freshly prepared table, and
    // reset to zero by the last workgroup of every run, except `error`).
    uint32_t exited;        // workgroups that have finished
    uint32_t error;         // kBatchErr* bits of the runs since preparation
    uint32_t pad_;
};

// error bits of a batch run
constexpr uint32_t kBatchErrRadius = 1;   // a view's radius exceeds the launch's
                                          // bound: its outputs are zeros
constexpr uint32_t kBatchErrWait = 2;     // a work item gave up waiting for the
                                          // items it depends on

// One-launch run state after the views in the table (device-written, zero
// between runs): the next turn of each work queue and, per view, the items
// finished per stage. Every counter has a 128-byte line of its own, so
// atomics on different counters do not queue behind each other.
struct BatchLine {
    uint32_t n;
    uint32_t pad_[31];
};

struct BatchCounters {
    BatchLine projected, decoded;
};

inline size_t batch_queues_offset(int32_t n_views) {
    return sizeof(BatchHeader) + (size_t)n_views * sizeof(BatchView);
}

inline size_t batch_counters_offset(int32_t n_views) {
    return batch_queues_offset(n_views) + kQueues * sizeof(BatchLine);
}

// A pointer the kernel read from memory (a view of the descriptor table) is
// generic to the compiler, which then accesses it with flat instructions.
// Flat loads count on the LDS counter as well, so every wait for an LDS
// read would also wait for them. Routing the pointer through an integer
// into the global address space makes its accesses global ones; every
// pointer a caller hands in is device global memory.
template <class T>
__device__ __forceinline__ T *as_global(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// A copy of a view whose pointers are marked global (as_global).
__device__ inline BatchView global_view(const BatchView &v) {
    BatchView g = v;
    g.pts = as_global(v.pts);
    g.rgb = as_global(v.rgb);
    g.zbuf = as_global(v.zbuf);
    g.sd = as_global(v.sd);
    g.sv = as_global(v.sv);
    g.out = as_global(v.out);
    g.mask = as_global(v.mask);
    g.recs = as_global(v.recs);
    g.rowoff = as_global(v.rowoff);
    g.bandcnt = as_global(v.bandcnt);
    g.grpcnt = as_global(v.grpcnt);
    return g;
}

// Last view v with views[v].*field <= c (the fields are exclusive prefixes,
// so v is the view that owns chunk or tile c). Wave-uniform arguments give
// scalar loads.
template <int32_t BatchView::*FIELD>
__device__ inline int batch_view_of(const BatchView *views, int n_views, int c) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].*FIELD <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Two-stage filtering and the dense small-radius filter (stage2.hip).
constexpr int kDenseMaxRadius = JBFD_DENSE_MAX_RADIUS;
hipError_t launch_pool3(const float *D, const uint8_t *B, const uint8_t *rgb,
                        int32_t H, int32_t W, float *D1, uint8_t *B1,
                        uint8_t *rgb1, hipStream_t s);
hipError_t launch_restore_merge(const float *D, const uint8_t *B,
                                const float *O1, const uint8_t *M1, int32_t H,
                                int32_t W, float *D2, uint8_t *B2,
                                hipStream_t s);
// O1, M1: NULL, or the first pass of the two-stage filter (a third of the
// resolution in each dimension): the kernel then filters the restored image
// (own sample, else the cell's first-pass output) without storing it.
hipError_t launch_densify_dense(const float *D, const uint8_t *B,
                                const uint8_t *rgb, int32_t H, int32_t W,
                                const FilterParams &fp, float *out,
                                uint8_t *mask, hipStream_t s,
                                const float *O1 = nullptr,
                                const uint8_t *M1 = nullptr);
size_t two_stage_ws_bytes(int32_t H, int32_t W);
hipError_t launch_two_stage(const float *D, const uint8_t *B, const uint8_t *rgb,
                            int32_t H, int32_t W, const FilterParams &f1,
                            const FilterParams &f2, float *out, uint8_t *mask,
                            void *ws, hipStream_t s);

// Occluded-point removal, contour removal and back-projection (cloud.hip).
hipError_t launch_remove_occluded(const float *D, const uint8_t *B, int32_t H,
                                  int32_t W, int32_t k, double tau,
                                  uint8_t *Bout, hipStream_t s);
size_t backproject_ws_bytes(int32_t H, int32_t W);
hipError_t launch_backproject(const float *D, const uint8_t *M, const uint8_t *rgb,
                              int32_t H, int32_t W, const Pose &P, const Intr &K,
                              double tau, float *xyz, uint8_t *rgb_out,
                              int64_t *total, void *ws, hipStream_t s);

// Afterimage removal (cloud.hip, project.hip).
hipError_t launch_motion_mask(const uint8_t *rgb, const uint8_t *rgb_prev,
                              int32_t H, int32_t W, double tau, int32_t k,
                              uint8_t *mask, hipStream_t s);
hipError_t launch_project_motion(const float *pts, int64_t n, const int8_t *sweep,
                                 int8_t latest, const uint8_t *motion,
                                 const Pose &P, const Intr &K, uint64_t *zbuf,
                                 float *depth, uint8_t *valid, hipStream_t s);

hipError_t launch_batch_lists(const BatchHeader *hdr, const BatchView *views,
                              hipStream_t s);
hipError_t launch_batch(void *d_table, int32_t max_radius, bool use_lists,
                        jbfd_precision prec, hipStream_t s);
hipError_t launch_batch_filter(BatchHeader *hdr, const BatchView *views,
                               int32_t max_radius, jbfd_precision prec,
                               bool use_lists, hipStream_t s);
// the whole batch in one persistent launch (streaming filter)
hipError_t launch_batch_fused(void *d_table, int32_t max_radius, jbfd_precision prec,
                              hipStream_t s);

}  // namespace jbfd

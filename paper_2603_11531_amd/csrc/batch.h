// Device-side plan of a batch of render requests (mgs_render_batch).
#pragma once

#include "common.h"

namespace mgs {

constexpr int BATCH_MAX_REQ = 64;
constexpr int BATCH_ALIGN = 256;       // request Gaussian ranges start on multiples of this

// Written once per batch on the device.  Gaussians of request r occupy the global
// index range [gbase[r], gbase[r] + n_r), each range starting on a multiple of
// BATCH_ALIGN so a projection block never mixes requests; tiles of request r are the global tile
// ids [tbase[r], tbase[r + 1]) and its 8x8-tile supertiles (binning) the global ids
// [stbase[r], stbase[r + 1]).
struct BatchPlan {
    int32_t nreq;
    int32_t ok;            // 1 = the batch fits the workspace limits; 0 = nothing is rendered
    uint32_t n_total;      // end of the last request's (padded) Gaussian range
    uint32_t t_total;      // number of global tiles
    uint32_t st_total;     // number of global supertiles
    uint32_t gbase[BATCH_MAX_REQ + 1];
    uint32_t tbase[BATCH_MAX_REQ + 1];
    uint32_t stbase[BATCH_MAX_REQ + 1];
    uint32_t tiles_x[BATCH_MAX_REQ];
    uint32_t tiles_y[BATCH_MAX_REQ];
    uint32_t st_x[BATCH_MAX_REQ];
};

// Index r of the request whose range [base[r], base[r+1]) holds v (base[0] = 0, nreq >= 1).
__device__ __forceinline__ int find_request(const uint32_t *base, int nreq, uint32_t v) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ CamK camk_device(const mgs_camera &c) {
    CamK k;
#pragma unroll
    for (int i = 0; i < 9; ++i) k.R[i] = c.R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) k.t[i] = c.t[i];
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    k.W = c.width; k.H = c.height; k.near_z = c.near_z;
    // the same rounded operations, in the same order, as the host-side make_camk (no contraction),
    // so a batched request sees exactly the camera centre of a single-view render
#pragma unroll
    for (int i = 0; i < 3; ++i)
        k.campos[i] = -__fadd_rn(__fadd_rn(__fmul_rn(c.R[0 * 3 + i], c.t[0]), __fmul_rn(c.R[1 * 3 + i], c.t[1])),
                                 __fmul_rn(c.R[2 * 3 + i], c.t[2]));
    k.tiles_x = (c.width + MGS_TILE - 1) / MGS_TILE;
    k.tiles_y = (c.height + MGS_TILE - 1) / MGS_TILE;
    k.weight_mode = MGS_WEIGHT_EQ3;
    return k;
}

// Binning of a whole batch (bin.hip): keys are global tile ids.
int bin_batch(const mgs_projected *proj, int64_t n_max, const BatchPlan *plan, uint32_t max_tiles, void *ws,
              size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity, uint32_t *n_pairs,
              hipStream_t s);
size_t bin_batch_workspace(int64_t n_max, uint32_t max_tiles, uint64_t capacity);

// Split-tile OIT blend of a whole batch (blend.hip).
size_t blend_split_workspace(uint32_t T, uint64_t capacity);
int blend_split_batch(const float4 *splat, const uint32_t *offs, const uint32_t *gids, const BatchPlan *plan,
                      const mgs_request *reqs, uint32_t max_tiles, const uint32_t *n_pairs, uint64_t capacity,
                      float alpha_min, float alpha_max, void *ws, hipStream_t s);

}  // namespace mgs

// mgs_render_batch: a batch of render requests (resident scenes, mixed resolutions and
// poses) in one fixed sequence of launches whose grids depend only on the workspace
// limits -- the request table and its count live in device memory, so the whole
// sequence can be captured once in a hipGraph and replayed for any batch that fits.
//
// Every request keeps its own index space: Gaussians of request r are projected
// into the global range [gbase[r], gbase[r] + n_r) and its tiles get global ids
// [tbase[r], tbase[r+1]); one binning pass sorts all requests' pairs by global tile
// id, and the blend runs one workgroup per global tile.  The per-tile lists hold the
// same Gaussians in the same order as a single-view render, so every image is
// bit-identical to rendering its request alone.
#include "batch.h"
#include "mlp_math.h"
#include "proj_math.h"

namespace mgs {

static_assert(BATCH_MAX_REQ == MGS_BATCH_MAX_REQUESTS, "batch limit");

__global__ void batch_plan_kernel(const mgs_request *__restrict__ reqs, const int32_t *__restrict__ n_req,
                                  uint64_t max_gauss, uint64_t max_tiles, BatchPlan *__restrict__ plan) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nr = *n_req;
    int ok = (nr >= 0 && nr <= BATCH_MAX_REQ) ? 1 : 0;
    if (!ok) nr = 0;
    uint64_t g = 0, t = 0, st = 0;
    for (int r = 0; r < nr; ++r) {
        const mgs_request &q = reqs[r];
        const int tx = (q.cam.width + MGS_TILE - 1) / MGS_TILE, ty = (q.cam.height + MGS_TILE - 1) / MGS_TILE;
        if (q.g.n < 0 || q.cam.width <= 0 || q.cam.height <= 0 || q.cam.fx <= 0.f || q.cam.fy <= 0.f ||
            q.image == nullptr)
            ok = 0;
        const uint32_t txu = uint32_t(tx > 0 ? tx : 1), tyu = uint32_t(ty > 0 ? ty : 1);
        plan->gbase[r] = uint32_t(g);
        plan->tbase[r] = uint32_t(t);
        plan->stbase[r] = uint32_t(st);
        plan->tiles_x[r] = txu;
        plan->tiles_y[r] = tyu;
        plan->st_x[r] = (txu + 7) / 8;
        g += (uint64_t(q.g.n > 0 ? q.g.n : 0) + BATCH_ALIGN - 1) / BATCH_ALIGN * BATCH_ALIGN;
        t += uint64_t(tx > 0 ? tx : 0) * uint64_t(ty > 0 ? ty : 0);
        st += uint64_t((txu + 7) / 8) * uint64_t((tyu + 7) / 8);
    }
    if (g > max_gauss || t > max_tiles) ok = 0;
    if (!ok) { nr = 0; g = 0; t = 0; st = 0; }
    plan->gbase[nr] = uint32_t(g);
    plan->tbase[nr] = uint32_t(t);
    plan->stbase[nr] = uint32_t(st);
    plan->nreq = nr;
    plan->ok = ok;
    plan->n_total = uint32_t(g);
    plan->t_total = uint32_t(t);
    plan->st_total = uint32_t(st);
}

// Enhancement MLP (for requests that carry one) and projection of every request's Gaussians
// into the global index space, one 256-Gaussian block per iteration; request ranges start on
// multiples of 256, so a block never mixes requests and one LDS copy of its request's packed
// MLP serves the block.  Alignment padding gets n_tiles = 0; nothing past n_total is written
// (the binning reads only the first n_total Gaussians).  Same arithmetic as the single-view
// enhance + project, so a request renders bit-identically alone and in a batch.
__global__ void __launch_bounds__(256)
batch_enhance_project_kernel(const mgs_request *__restrict__ reqs, const BatchPlan *__restrict__ plan,
                             float alpha_min, float4 *__restrict__ splat, uint2 *__restrict__ rect_out,
                             uint32_t *__restrict__ ntiles_out) {
    __shared__ __attribute__((aligned(16))) __bf16 s_x[4][64 * FEAT_STRIDE];
    __shared__ __attribute__((aligned(16))) uint8_t s_mlp[MGS_MLP_PACKED_BYTES];
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int nreq = plan->nreq;
    if (nreq == 0) return;                                             // grid-uniform
    const uint32_t nblk = plan->n_total / BATCH_ALIGN;
    const void *loaded = nullptr;
    const MlpLds F{s_mlp, l};
    for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const uint32_t k0 = b * BATCH_ALIGN;
        const int r = find_request(plan->gbase, nreq, k0);             // block-uniform
        const mgs_request &q = reqs[r];
        const CamK cam = camk_device(q.cam);
        const bool mlp = q.packed_mlp != nullptr;
        if (mlp && q.packed_mlp != loaded) {
            __syncthreads();                                           // the previous copy is no longer read
            for (int k = threadIdx.x; k < MGS_MLP_PACKED_BYTES / 16; k += blockDim.x)
                reinterpret_cast<uint4 *>(s_mlp)[k] = reinterpret_cast<const uint4 *>(q.packed_mlp)[k];
            __syncthreads();
            loaded = q.packed_mlp;
        }
        const uint32_t k = k0 + threadIdx.x;
        const int64_t i = int64_t(k) - plan->gbase[r];
        const bool valid = i < q.g.n;
        float ph = 1.0f, om = 1.0f;
        if (mlp) {                                                     // block-uniform
            f32x8 f[4];
            if (valid) {
                const GaussIn a = load_gauss(q.g, i, nullptr, nullptr);
                lane_features(a.mu, a.ls, a.q, a.sh, cam, f);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
            }
            mlp_wave(f, F, s_x[w], ph, om);
            __asm__ volatile("" ::: "memory");                         // re-read the attributes below
        }
        if (valid) {
            GaussIn in = load_gauss(q.g, i, nullptr, nullptr);
            in.phi = ph;
            in.om = om;
            store_proj(project_gaussian(in, cam, alpha_min), k, splat, rect_out, ntiles_out);
        } else {
            rect_out[k] = make_uint2(0u, 0u);
            ntiles_out[k] = 0u;
        }
    }
}

__global__ void batch_status_kernel(const BatchPlan *__restrict__ plan, int32_t *__restrict__ status) {
    status[0] = plan->ok;
    status[1] = plan->nreq;
}

struct BatchLayout {
    size_t plan, splat, rect, ntiles, offs, gids, bin, split, total;
};

inline BatchLayout batch_layout(int64_t max_gauss, int64_t max_tiles, uint64_t capacity) {
    BatchLayout L;
    const size_t ng = size_t(max_gauss > 0 ? max_gauss : 1), cap = size_t(capacity > 0 ? capacity : 1);
    size_t o = 0;
    L.plan = o;   o = align_up(o + sizeof(BatchPlan), 256);
    L.splat = o;  o = align_up(o + ng * 48, 256);
    L.rect = o;   o = align_up(o + ng * 8, 256);
    L.ntiles = o; o = align_up(o + ng * 4, 256);
    L.offs = o;   o = align_up(o + (size_t(max_tiles) + 1) * 4, 256);
    L.gids = o;   o = align_up(o + cap * 4, 256);
    L.bin = o;    o = align_up(o + bin_batch_workspace(int64_t(ng), uint32_t(max_tiles), capacity), 256);
    L.split = o;  o = align_up(o + blend_split_workspace(uint32_t(max_tiles), capacity), 256);
    L.total = o;
    return L;
}

}  // namespace mgs

extern "C" int mgs_batch_workspace(int64_t max_gaussians, int64_t max_tiles, uint64_t capacity, size_t *bytes) {
    MGS_REQUIRE(bytes != nullptr, "bytes is NULL");
    MGS_REQUIRE(max_gaussians > 0 && max_gaussians < (int64_t(1) << 31), "max_gaussians out of range");
    MGS_REQUIRE(max_tiles > 0 && max_tiles < (int64_t(1) << 20), "max_tiles out of range");
    MGS_REQUIRE(capacity > 0 && capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    *bytes = mgs::batch_layout(max_gaussians, max_tiles, capacity).total;
    return MGS_OK;
}

extern "C" int mgs_render_batch(const mgs_request *requests, const int32_t *n_requests, int64_t max_gaussians,
                                int64_t max_tiles, uint64_t capacity, float alpha_min, float alpha_max, void *ws,
                                size_t ws_bytes, uint32_t *n_pairs, int32_t *status, void *stream) {
    MGS_TRACE("mgs_render_batch");
    using namespace mgs;
    MGS_REQUIRE(requests && n_requests && n_pairs, "requests / n_requests / n_pairs is NULL");
    MGS_REQUIRE(max_gaussians > 0 && max_gaussians < (int64_t(1) << 31), "max_gaussians out of range");
    MGS_REQUIRE(max_tiles > 0 && max_tiles < (int64_t(1) << 20), "max_tiles out of range");
    MGS_REQUIRE(capacity > 0 && capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    MGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f && alpha_max > alpha_min && alpha_max < 1.f, "bad alpha range");
    const BatchLayout L = batch_layout(max_gaussians, max_tiles, capacity);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(ws);
    BatchPlan *plan = reinterpret_cast<BatchPlan *>(w + L.plan);
    float4 *splat = reinterpret_cast<float4 *>(w + L.splat);
    uint2 *rect = reinterpret_cast<uint2 *>(w + L.rect);
    uint32_t *ntiles = reinterpret_cast<uint32_t *>(w + L.ntiles);
    uint32_t *offs = reinterpret_cast<uint32_t *>(w + L.offs);
    uint32_t *gids = reinterpret_cast<uint32_t *>(w + L.gids);

    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(64), 0, s, requests, n_requests, uint64_t(max_gaussians),
                       uint64_t(max_tiles), plan);
    MGS_LAUNCH_CHECK("batch_plan_kernel");
    const int64_t pblk = (max_gaussians + BATCH_ALIGN - 1) / BATCH_ALIGN;
    hipLaunchKernelGGL(batch_enhance_project_kernel, dim3(unsigned(pblk < 4096 ? pblk : 4096)), dim3(256), 0, s,
                       requests, plan, alpha_min, splat, rect, ntiles);
    MGS_LAUNCH_CHECK("batch_enhance_project_kernel");
    mgs_projected proj;
    proj.splat = reinterpret_cast<float *>(splat);
    proj.rect = reinterpret_cast<uint32_t *>(rect);
    proj.n_tiles = ntiles;
    int rc = bin_batch(&proj, max_gaussians, plan, uint32_t(max_tiles), w + L.bin, L.split - L.bin, offs, gids,
                       capacity, n_pairs, s);
    if (rc != MGS_OK) return rc;
    rc = blend_split_batch(splat, offs, gids, plan, requests, uint32_t(max_tiles), n_pairs, capacity, alpha_min,
                           alpha_max, w + L.split, s);
    if (rc != MGS_OK) return rc;
    if (status) {
        hipLaunchKernelGGL(batch_status_kernel, dim3(1), dim3(1), 0, s, plan, status);
        MGS_LAUNCH_CHECK("batch_status_kernel");
    }
    return MGS_OK;
}

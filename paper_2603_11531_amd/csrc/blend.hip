// mgs_blend_oit (Eq. 2) and mgs_blend_sorted (Eq. 11): per-tile compositing.
//
// One 256-thread workgroup per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1) and each lane one pixel of it.  The tile's Gaussians are
// staged through LDS in batches of 256 (one coalesced 48-byte record per
// thread).  While staging, every thread also decides, for its Gaussian, which
// quadrants can see it: the largest alpha over a quadrant's pixel-centre
// rectangle is found exactly (the exponent is a concave quadratic, so its
// maximum over a rectangle is at the centre or on an edge) and quadrants where
// it stays below alpha_min are masked out.  Each wave then walks only its own
// Gaussians (ballot over the masks, scalar bit loop), so a wave never spends
// VALU cycles on a splat that cannot reach its 64 pixels.
//
// Per pixel-Gaussian pair the OIT inner loop is: 2 subtractions, 3 FMA and
// 2 multiplies for the exponent, 1 exp2, 1 compare/select, 1 min and 6 for the
// accumulation of N (rgb), D and T -- all float32 VALU, no sort, no order.
#include "blend_math.h"

namespace mgs {

constexpr int BLEND_THREADS = 256;
constexpr int BLEND_BATCH = 256;
__device__ __forceinline__ int tile_index(int b) { return b; }

template <bool SORTED>
__global__ void __launch_bounds__(BLEND_THREADS)
blend_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs,
             const uint32_t *__restrict__ gids, CamK cam, float bgr, float bgg, float bgb,
             float log2_amin, float amax, float t_stop, float *__restrict__ image,
             float *__restrict__ aux) {
    __shared__ float4 s_r0[BLEND_BATCH];
    __shared__ float4 s_r1[BLEND_BATCH];
    __shared__ float4 s_r2[BLEND_BATCH];
    __shared__ uint32_t s_mask[BLEND_BATCH];
    __shared__ int s_done[4];

    const int tile = tile_index(blockIdx.x);
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int px = tx * 16 + (w & 1) * 8 + (l & 7);
    const int py = ty * 16 + (w >> 1) * 8 + (l >> 3);
    const float fpx = float(px) + 0.5f, fpy = float(py) + 0.5f;
    const uint32_t start = offs[tile], end = offs[tile + 1];

    float Nr = 0.f, Ng = 0.f, Nb = 0.f, D = 0.f, T = 1.f;
    bool wave_done = false;

    for (uint32_t b = start; b < end; b += BLEND_BATCH) {
        __syncthreads();
        const uint32_t i = b + threadIdx.x;
        uint32_t mask = 0;
        if (i < end) {
            const uint32_t g = gids[i];
            const float4 r0 = splat[3 * size_t(g) + 0];
            const float4 r1 = splat[3 * size_t(g) + 1];
            const float4 r2 = splat[3 * size_t(g) + 2];
            s_r0[threadIdx.x] = r0;
            s_r1[threadIdx.x] = r1;
            s_r2[threadIdx.x] = r2;
            mask = quadrant_mask(r0, r1, tx, ty, log2_amin);
        }
        s_mask[threadIdx.x] = mask;
        if (SORTED && l == 0) s_done[w] = wave_done ? 1 : 0;
        __syncthreads();
        if (SORTED && s_done[0] && s_done[1] && s_done[2] && s_done[3]) break;
        if (SORTED && wave_done) continue;
        for (int grp = 0; grp < BLEND_BATCH / 64; ++grp) {
            uint64_t bal = __ballot((s_mask[grp * 64 + l] >> w) & 1u);
            while (bal) {
                const int j = grp * 64 + __builtin_ctzll(bal);
                bal &= bal - 1;
                const float4 r0 = s_r0[j];
                const float4 r1 = s_r1[j];
                const float4 r2 = s_r2[j];
                const float dx = fpx - r0.x;
                const float dy = fpy - r0.y;
                const float t = fmaf(r1.y, dy, dx);
                const float e = fmaf(r1.x * t, t, fmaf(r1.z * dy, dy, r0.z));
                if (!SORTED) {
                    const float al = e >= log2_amin ? fminf(fast_exp2(e), amax) : 0.0f;
                    const float aw = al * r0.w;
                    Nr = fmaf(aw, r2.x, Nr);
                    Ng = fmaf(aw, r2.y, Ng);
                    Nb = fmaf(aw, r2.z, Nb);
                    D += aw;
                    T = fmaf(-T, al, T);
                } else {
                    const float al = (e >= log2_amin && T >= t_stop) ? fminf(fast_exp2(e), amax) : 0.0f;
                    const float at = al * T;
                    Nr = fmaf(at, r2.x, Nr);
                    Ng = fmaf(at, r2.y, Ng);
                    Nb = fmaf(at, r2.z, Nb);
                    T = fmaf(-T, al, T);
                }
            }
            if (SORTED) {
                wave_done = __ballot(T >= t_stop) == 0ull;
                if (wave_done) break;
            }
        }
    }

    if (px < cam.W && py < cam.H) {
        const size_t hw = size_t(cam.W) * cam.H;
        const size_t p = size_t(py) * cam.W + px;
        float cr, cg, cb;
        if (!SORTED) {
            if (D > 0.f) {
                const float inv = 1.0f / D;
                const float fr = Nr * inv, fg = Ng * inv, fb = Nb * inv;
                const float f = 1.0f - T;
                cr = fmaf(f, fr, T * bgr);
                cg = fmaf(f, fg, T * bgg);
                cb = fmaf(f, fb, T * bgb);
                if (aux) {
                    aux[p] = fr; aux[hw + p] = fg; aux[2 * hw + p] = fb;
                    aux[3 * hw + p] = D; aux[4 * hw + p] = T;
                }
            } else {
                cr = bgr; cg = bgg; cb = bgb;
                if (aux) {
                    aux[p] = 0.f; aux[hw + p] = 0.f; aux[2 * hw + p] = 0.f;
                    aux[3 * hw + p] = 0.f; aux[4 * hw + p] = 1.f;
                }
            }
        } else {
            cr = fmaf(T, bgr, Nr);
            cg = fmaf(T, bgg, Ng);
            cb = fmaf(T, bgb, Nb);
        }
        image[p] = cr;
        image[hw + p] = cg;
        image[2 * hw + p] = cb;
    }
}

inline int blend_common_checks(const mgs_projected *proj, const uint32_t *offs, const uint32_t *gids,
                               const mgs_camera *cam, int tile, const float *bg, float amin, float amax,
                               float *image) {
    int rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    MGS_REQUIRE(proj != nullptr, "projected is NULL");
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(offs && image && bg, "tile_offsets / image / bg is NULL");
    MGS_REQUIRE(amin > 0.f && amin < 1.f && amax > amin && amax < 1.f, "bad alpha range");
    MGS_REQUIRE(aligned(proj->splat, 16), "splat must be 16-byte aligned");
    (void)gids;
    return MGS_OK;
}

}  // namespace mgs

extern "C" int mgs_blend_oit(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                             const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                             float alpha_max, float *image, float *aux, void *stream) {
    using namespace mgs;
    int rc;
    if ((rc = blend_common_checks(proj, tile_offsets, gids, cam, tile, bg, alpha_min, alpha_max, image)) != MGS_OK)
        return rc;
    const CamK k = make_camk(cam);
    const unsigned ntiles = unsigned(k.tiles_x) * unsigned(k.tiles_y);
    hipLaunchKernelGGL(blend_kernel<false>, dim3(ntiles), dim3(BLEND_THREADS), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, k, bg[0], bg[1], bg[2],
                       log2f(alpha_min), alpha_max, 0.0f, image, aux);
    MGS_LAUNCH_CHECK("blend_kernel<oit>");
    return MGS_OK;
}

extern "C" int mgs_blend_sorted(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                                float alpha_max, float t_stop, float *image, void *stream) {
    using namespace mgs;
    int rc;
    if ((rc = blend_common_checks(proj, tile_offsets, gids, cam, tile, bg, alpha_min, alpha_max, image)) != MGS_OK)
        return rc;
    MGS_REQUIRE(t_stop >= 0.f && t_stop < 1.f, "t_stop must be in [0, 1)");
    const CamK k = make_camk(cam);
    const unsigned ntiles = unsigned(k.tiles_x) * unsigned(k.tiles_y);
    hipLaunchKernelGGL(blend_kernel<true>, dim3(ntiles), dim3(BLEND_THREADS), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, k, bg[0], bg[1], bg[2],
                       log2f(alpha_min), alpha_max, t_stop, image, nullptr);
    MGS_LAUNCH_CHECK("blend_kernel<sorted>");
    return MGS_OK;
}

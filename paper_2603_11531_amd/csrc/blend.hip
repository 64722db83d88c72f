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
// Per pixel-Gaussian pair the OIT inner loop is: 5 FMA for the exponent (a
// polynomial in the lane's offset, see quad_poly), compare/select, min, exp2,
// and 5 FMA to accumulate N (rgb, colours pre-multiplied by w), D and T -- all
// float32 VALU, no sort, no order.
#include "blend_math.h"

namespace mgs {

template <bool SORTED>
__global__ void __launch_bounds__(BLEND_THREADS)
blend_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs,
             const uint32_t *__restrict__ gids, CamK cam, float bgr, float bgg, float bgb,
             float log2_amin, float amax, float t_stop, float *__restrict__ image,
             float *__restrict__ aux) {
    const int tile = blockIdx.x;
    blend_tile<SORTED>(splat, gids, offs[tile], offs[tile + 1], tile % cam.tiles_x, tile / cam.tiles_x, cam.W,
                       cam.H, bgr, bgg, bgb, log2_amin, amax, t_stop, image, aux);
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

// mgs_project: per-Gaussian preprocessing (EWA projection, SH1 colour, Eq. 3 weight,
// effective opacity, tile rectangle).  One thread per Gaussian; every attribute
// plane is read with unit stride (coalesced SoA), the 48-byte splat record is
// written as three float4 per thread.
//
// Numerics.  The 2D covariance of a 3D Gaussian is a sum of three rank-one
// terms u_i u_i^T with u_i = s_i * M r_i (M = J W, r_i the rotation columns).
// Its determinant is therefore sum_{i<j} cross(u_i, u_j)^2 plus the dilation
// terms -- a sum of non-negative terms that float32 evaluates without the
// cancellation of a*c - b^2, which matters for thin, elongated splats.  The
// exponent is stored as q = A t^2 + dy^2 / c with t = dx - (b/c) dy, which is
// the same quadratic form split into two non-negative parts.
#include "proj_math.h"

namespace mgs {

__global__ void __launch_bounds__(256)
project_kernel(mgs_gaussians g, CamK cam, const float *__restrict__ phi_in,
               const float *__restrict__ omod_in, float alpha_min,
               float4 *__restrict__ splat, uint2 *__restrict__ rect_out,
               uint32_t *__restrict__ ntiles_out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const GaussIn in = load_gauss(g, i, phi_in, omod_in);
    const GaussFwd f = gauss_forward(in, cam);

    // exact bounding box of {alpha >= alpha_min} = {q <= 2 ln(o_eff / alpha_min)}
    const float kq = 2.0f * logf(fmaxf(f.o, alpha_min) / alpha_min);
    const float ex = sqrtf(kq * f.a), ey = sqrtf(kq * f.c);
    const float fW = float(cam.W), fH = float(cam.H);
    const float i0 = fminf(fmaxf(ceilf(f.mx - ex - 0.5f), 0.0f), fW);
    const float i1 = fminf(fmaxf(floorf(f.mx + ex - 0.5f), -1.0f), fW - 1.0f);
    const float j0 = fminf(fmaxf(ceilf(f.my - ey - 0.5f), 0.0f), fH);
    const float j1 = fminf(fmaxf(floorf(f.my + ey - 0.5f), -1.0f), fH - 1.0f);
    const bool vis = f.front && (f.o >= alpha_min) && (f.qnorm > 0.0f) && (i0 <= i1) && (j0 <= j1) &&
                     (f.det > 0.0f) && isfinite(f.mx) && isfinite(f.my);

    uint32_t nt = 0;
    uint2 rc = make_uint2(0u, 0u);
    if (vis) {
        const uint32_t tx0 = uint32_t(i0) / MGS_TILE, tx1 = uint32_t(i1) / MGS_TILE;
        const uint32_t ty0 = uint32_t(j0) / MGS_TILE, ty1 = uint32_t(j1) / MGS_TILE;
        nt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        rc = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
    }
    const float kA = -0.5f * LOG2E * (f.c / f.det);   // log2(alpha) = log2(o) + kA t^2 + kG dy^2
    const float beta = -f.b / f.c;                   // t = dx + beta * dy
    const float kG = -0.5f * LOG2E / f.c;
    const float d = f.front ? f.z : -1.0f;
    splat[3 * i + 0] = make_float4(f.mx, f.my, log2f(fmaxf(f.o, 1e-30f)), f.w);
    splat[3 * i + 1] = make_float4(kA, beta, kG, d);
    splat[3 * i + 2] = make_float4(f.col[0], f.col[1], f.col[2], f.o);
    rect_out[i] = rc;
    ntiles_out[i] = nt;
}

}  // namespace mgs

extern "C" int mgs_project(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                           const float *omod, int tile, float alpha_min, mgs_projected *out,
                           void *stream) {
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    if (g->n == 0) return MGS_OK;
    const CamK k = make_camk(cam);
    const unsigned blocks = unsigned((g->n + 255) / 256);
    hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), *g, k, phi, omod,
                       alpha_min, reinterpret_cast<float4 *>(out->splat),
                       reinterpret_cast<uint2 *>(out->rect), out->n_tiles);
    MGS_LAUNCH_CHECK("project_kernel");
    return MGS_OK;
}

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
#include "mlp_math.h"
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
    store_proj(project_gaussian(in, cam, alpha_min), i, splat, rect_out, ntiles_out);
}

// Where the fused kernel reads a Gaussian's attributes: float32 SoA planes, or the
// codebooks of a vector-quantised scene (positions float32, five 4-value sub-vectors).
struct SoaSource {
    mgs_gaussians g;
    __device__ __forceinline__ int64_t count() const { return g.n; }
    __device__ __forceinline__ GaussIn load(int64_t i) const { return load_gauss(g, i, nullptr, nullptr); }
};
struct NvqSource {
    int64_t n;
    const float *mean;
    const uint16_t *codes;
    const float4 *cb;              // [5][1024] codewords
    __device__ __forceinline__ int64_t count() const { return n; }
    __device__ __forceinline__ GaussIn load(int64_t i) const {
        GaussIn in;
#pragma unroll
        for (int k = 0; k < 3; ++k) in.mu[k] = mean[k * n + i];
        float4 v[MGS_NVQ_GROUPS];
#pragma unroll
        for (int g = 0; g < MGS_NVQ_GROUPS; ++g)
            v[g] = cb[g * MGS_NVQ_CODEWORDS + (codes[g * n + i] & (MGS_NVQ_CODEWORDS - 1))];
        in.ls[0] = v[0].x; in.ls[1] = v[0].y; in.ls[2] = v[0].z;
        in.q[0] = v[0].w; in.q[1] = v[1].x; in.q[2] = v[1].y; in.q[3] = v[1].z;
        in.logit = v[1].w;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            in.sh[4 * g + 0] = v[2 + g].x;
            in.sh[4 * g + 1] = v[2 + g].y;
            in.sh[4 * g + 2] = v[2 + g].z;
            in.sh[4 * g + 3] = v[2 + g].w;
        }
        in.phi = 1.0f;
        in.om = 1.0f;
        return in;
    }
};

// Enhancement MLP and projection in one pass: each wave builds its 64 Gaussians'
// features, runs the MLP on MFMA (weights read from an LDS copy), hands every lane its
// own (phi, m) and projects.  Same results as mgs_enhance followed by mgs_project.
template <typename Src>
__global__ void __launch_bounds__(256)
enhance_project_kernel(Src src, CamK cam, const uint8_t *__restrict__ packed, float alpha_min,
                       float4 *__restrict__ splat, uint2 *__restrict__ rect_out, uint32_t *__restrict__ ntiles_out,
                       float *__restrict__ phi_out, float *__restrict__ omod_out) {
    __shared__ __attribute__((aligned(16))) __bf16 s_x[4][64 * FEAT_STRIDE];
    __shared__ __attribute__((aligned(16))) uint8_t s_mlp[MGS_MLP_PACKED_BYTES];
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int64_t n = src.count();
    const int64_t ngroups = (n + 63) / 64;
    // the packed MLP lives in LDS (read at each use) so the registers go to the projection
    static_assert(MGS_MLP_PACKED_BYTES % 16 == 0, "packed MLP size");
    for (int k = threadIdx.x; k < MGS_MLP_PACKED_BYTES / 16; k += blockDim.x)
        reinterpret_cast<uint4 *>(s_mlp)[k] = reinterpret_cast<const uint4 *>(packed)[k];
    __syncthreads();
    const MlpLds F{s_mlp, l};
    for (int64_t grp = int64_t(blockIdx.x) * 4 + w; grp < ngroups; grp += int64_t(gridDim.x) * 4) {
        const int64_t i = grp * 64 + l;
        const bool valid = i < n;
        f32x8 f[4];
        if (valid) {
            const GaussIn a = src.load(i);
            lane_features(a.mu, a.ls, a.q, a.sh, cam, f);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
        float ph, om;
        mlp_wave(f, F, s_x[w], ph, om);
        // The projection reads the attributes again (cache hits) instead of keeping them in
        // registers across the MLP: fewer live registers, more waves in flight.
        __asm__ volatile("" ::: "memory");
        if (valid) {
            GaussIn in = src.load(i);
            in.phi = ph;
            in.om = om;
            store_proj(project_gaussian(in, cam, alpha_min), i, splat, rect_out, ntiles_out);
            phi_out[i] = ph;
            omod_out[i] = om;
        }
    }
}

// Codebook decode to SoA planes, one thread per Gaussian.
__global__ void __launch_bounds__(256)
nvq_decode_kernel(NvqSource src, float *__restrict__ ls, float *__restrict__ q, float *__restrict__ logit,
                  float *__restrict__ sh) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = src.n;
    if (i >= n) return;
    const GaussIn in = src.load(i);
#pragma unroll
    for (int k = 0; k < 3; ++k) ls[k * n + i] = in.ls[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k * n + i] = in.q[k];
    logit[i] = in.logit;
#pragma unroll
    for (int k = 0; k < 12; ++k) sh[k * n + i] = in.sh[k];
}

inline int check_nvq(const mgs_gaussians_nvq *q) {
    MGS_REQUIRE(q != nullptr, "nvq scene is NULL");
    MGS_REQUIRE(q->n >= 0 && q->n < (int64_t(1) << 31), "n = %lld out of range", (long long)q->n);
    if (q->n == 0) return MGS_OK;
    MGS_REQUIRE(q->mean && q->codes && q->codebooks, "a pointer of the nvq scene is NULL");
    MGS_REQUIRE(aligned(q->codebooks, 16), "codebooks must be 16-byte aligned");
    return MGS_OK;
}

inline NvqSource nvq_source(const mgs_gaussians_nvq *q) {
    return NvqSource{q->n, q->mean, q->codes, reinterpret_cast<const float4 *>(q->codebooks)};
}

}  // namespace mgs

extern "C" int mgs_enhance_project_weighted(const mgs_gaussians *g, const mgs_camera *cam,
                                            const void *packed_mlp, int tile, float alpha_min, int weight_mode,
                                            mgs_projected *out, float *phi, float *omod, void *stream) {
    using namespace mgs;
    int rc;
    MGS_REQUIRE(valid_weight_mode(weight_mode), "unknown weight_mode %d", weight_mode);
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(packed_mlp && aligned(packed_mlp, 16), "packed MLP must be non-NULL and 16-byte aligned");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    CamK k = make_camk(cam);
    k.weight_mode = weight_mode;
    const int64_t groups = (g->n + 63) / 64;
    int64_t blocks = (groups + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(enhance_project_kernel<SoaSource>, dim3(unsigned(blocks)), dim3(256), 0, as_stream(stream),
                       SoaSource{*g}, k,
                       static_cast<const uint8_t *>(packed_mlp), alpha_min, reinterpret_cast<float4 *>(out->splat),
                       reinterpret_cast<uint2 *>(out->rect), out->n_tiles, phi, omod);
    MGS_LAUNCH_CHECK("enhance_project_kernel");
    return MGS_OK;
}

extern "C" int mgs_enhance_project(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp, int tile,
                                   float alpha_min, mgs_projected *out, float *phi, float *omod, void *stream) {
    return mgs_enhance_project_weighted(g, cam, packed_mlp, tile, alpha_min, MGS_WEIGHT_EQ3, out, phi, omod, stream);
}

extern "C" int mgs_project_weighted(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                                    const float *omod, int tile, float alpha_min, int weight_mode,
                                    mgs_projected *out, void *stream) {
    using namespace mgs;
    int rc;
    MGS_REQUIRE(valid_weight_mode(weight_mode), "unknown weight_mode %d", weight_mode);
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    if (g->n == 0) return MGS_OK;
    CamK k = make_camk(cam);
    k.weight_mode = weight_mode;
    const unsigned blocks = unsigned((g->n + 255) / 256);
    hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), *g, k, phi, omod,
                       alpha_min, reinterpret_cast<float4 *>(out->splat),
                       reinterpret_cast<uint2 *>(out->rect), out->n_tiles);
    MGS_LAUNCH_CHECK("project_kernel");
    return MGS_OK;
}

extern "C" int mgs_project(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                           const float *omod, int tile, float alpha_min, mgs_projected *out,
                           void *stream) {
    return mgs_project_weighted(g, cam, phi, omod, tile, alpha_min, MGS_WEIGHT_EQ3, out, stream);
}

extern "C" int mgs_nvq_decode(const mgs_gaussians_nvq *q, float *log_scale, float *quat, float *opacity_logit,
                              float *sh, void *stream) {
    using namespace mgs;
    int rc;
    if ((rc = check_nvq(q)) != MGS_OK) return rc;
    if (q->n == 0) return MGS_OK;
    MGS_REQUIRE(log_scale && quat && opacity_logit && sh, "an output plane is NULL");
    const unsigned blocks = unsigned((q->n + 255) / 256);
    hipLaunchKernelGGL(nvq_decode_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), nvq_source(q), log_scale,
                       quat, opacity_logit, sh);
    MGS_LAUNCH_CHECK("nvq_decode_kernel");
    return MGS_OK;
}

extern "C" int mgs_enhance_project_nvq(const mgs_gaussians_nvq *q, const mgs_camera *cam, const void *packed_mlp,
                                       int tile, float alpha_min, mgs_projected *out, float *phi, float *omod,
                                       void *stream) {
    using namespace mgs;
    int rc;
    if ((rc = check_nvq(q)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, q->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(packed_mlp && aligned(packed_mlp, 16), "packed MLP must be non-NULL and 16-byte aligned");
    if (q->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    const CamK k = make_camk(cam);
    const int64_t groups = (q->n + 63) / 64;
    int64_t blocks = (groups + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(enhance_project_kernel<NvqSource>, dim3(unsigned(blocks)), dim3(256), 0, as_stream(stream),
                       nvq_source(q), k, static_cast<const uint8_t *>(packed_mlp), alpha_min,
                       reinterpret_cast<float4 *>(out->splat), reinterpret_cast<uint2 *>(out->rect), out->n_tiles,
                       phi, omod);
    MGS_LAUNCH_CHECK("enhance_project_kernel<nvq>");
    return MGS_OK;
}

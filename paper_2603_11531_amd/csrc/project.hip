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

// sig_in / beta_in: the Eq. 1 weight's sigma_i, beta_i (read only for MGS_WEIGHT_SORTFREE).
__global__ void __launch_bounds__(256)
project_kernel(mgs_gaussians g, CamK cam, const float *__restrict__ phi_in,
               const float *__restrict__ omod_in, const float *__restrict__ sig_in,
               const float *__restrict__ beta_in, float alpha_min,
               float4 *__restrict__ splat, uint2 *__restrict__ rect_out,
               uint32_t *__restrict__ ntiles_out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    GaussIn in = load_gauss(g, i, phi_in, omod_in);
    if (cam.weight_mode == MGS_WEIGHT_SORTFREE) {
        in.wsig = sig_in[i];
        in.wbeta = beta_in[i];
    }
    store_proj(project_gaussian(in, cam, alpha_min), i, splat, rect_out, ntiles_out);
}

// Where the fused kernel reads a Gaussian's attributes: float32 SoA planes, or the
// codebooks of a vector-quantised scene (positions float32, five 4-value sub-vectors).
struct SoaSource {
    mgs_gaussians g;
    __device__ __forceinline__ int64_t count() const { return g.n; }
    __device__ __forceinline__ GaussIn load(int64_t i) const { return load_gauss(g, i, nullptr, nullptr); }
};
// Float32 SoA planes plus the per-Gaussian sigma_i, beta_i of the Eq. 1 weight.
struct SoaSortfreeSource {
    mgs_gaussians g;
    const float *sigma, *beta;
    __device__ __forceinline__ int64_t count() const { return g.n; }
    __device__ __forceinline__ GaussIn load(int64_t i) const {
        GaussIn in = load_gauss(g, i, nullptr, nullptr);
        in.wsig = sigma[i];
        in.wbeta = beta[i];
        return in;
    }
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
        in.cext[0] = in.cext[1] = in.cext[2] = 0.0f;
        return in;
    }
};

// Float32 SoA planes with SH of order DEG (0, 2 or 3; 3 (DEG + 1)^2 planes, plane 3 k + channel):
// the MLP and the first-order colour see the order <= 1 block (zeros for order 0), the terms of
// order 2 and 3 go to cext.  Real SH with the sign (-1)^m on odd m, as for order 1.
template <int DEG>
struct SoaShSource {
    mgs_gaussians g;
    float campos[3];
    static constexpr int K = (DEG + 1) * (DEG + 1);
    __device__ __forceinline__ int64_t count() const { return g.n; }
    __device__ __forceinline__ GaussIn load(int64_t i) const {
        const int64_t n = g.n;
        GaussIn in;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            in.mu[k] = g.mean[k * n + i];
            in.ls[k] = g.log_scale[k * n + i];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) in.q[k] = g.quat[k * n + i];
        in.logit = g.opacity_logit[i];
#pragma unroll
        for (int k = 0; k < 12; ++k) in.sh[k] = k < 3 * K ? g.sh[k * n + i] : 0.0f;
        in.phi = 1.0f;
        in.om = 1.0f;
        in.cext[0] = in.cext[1] = in.cext[2] = 0.0f;
        if constexpr (DEG >= 2) {
            const float vx = in.mu[0] - campos[0], vy = in.mu[1] - campos[1], vz = in.mu[2] - campos[2];
            const float vi = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
            const float x = vx * vi, y = vy * vi, z = vz * vi;
            float Y[K > 4 ? K - 4 : 1];
            const float a2 = 1.0925484305920792f, b2 = 0.31539156525252005f, c2 = 0.5462742152960396f;
            Y[0] = a2 * x * y; Y[1] = -a2 * y * z; Y[2] = b2 * (3.0f * z * z - 1.0f); Y[3] = -a2 * x * z;
            Y[4] = c2 * (x * x - y * y);
            if constexpr (DEG >= 3) {
                const float a3 = 0.5900435899266435f, b3 = 2.890611442640554f, c3 = 0.4570457994644658f;
                const float d3 = 0.3731763325901154f, e3 = 1.445305721320277f;
                Y[5] = -a3 * y * (3.0f * x * x - y * y); Y[6] = b3 * x * y * z; Y[7] = -c3 * y * (5.0f * z * z - 1.0f);
                Y[8] = d3 * z * (5.0f * z * z - 3.0f); Y[9] = -c3 * x * (5.0f * z * z - 1.0f);
                Y[10] = e3 * z * (x * x - y * y); Y[11] = -a3 * x * (x * x - 3.0f * y * y);
            }
#pragma unroll
            for (int k = 4; k < K; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) in.cext[ch] += Y[k - 4] * g.sh[(3 * k + ch) * n + i];
        }
        return in;
    }
};

// Whether the fused pass holds a source's attributes in registers across the MLP (one read) or
// reads them again after it (cache hits).  Holding them pays for the float32 first-order planes;
// the higher SH orders (up to 48 planes and their basis) run faster re-read, and the quantised and
// Eq. 1 sources keep the re-read they were measured with.
template <typename Src>
struct KeepAcrossMlp {
    static constexpr bool value = false;
};
template <>
struct KeepAcrossMlp<SoaSource> {
    static constexpr bool value = true;
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
        GaussIn in;
        if (valid) {
            in = src.load(i);
            lane_features(in.mu, in.ls, in.q, in.sh, cam, f);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
        float ph, om;
        mlp_wave(f, F, s_x[w], ph, om);
        if constexpr (!KeepAcrossMlp<Src>::value) {
            __asm__ volatile("" ::: "memory");      // a second read, not the first one's registers
            if (valid) in = src.load(i);
        }
        if (valid) {
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
    MGS_TRACE("mgs_enhance_project_weighted");
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

extern "C" int mgs_enhance_project_sh(const mgs_gaussians *g, int sh_degree, const mgs_camera *cam,
                                      const void *packed_mlp, int tile, float alpha_min, mgs_projected *out,
                                      float *phi, float *omod, void *stream) {
    MGS_TRACE("mgs_enhance_project_sh");
    using namespace mgs;
    int rc;
    MGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree %d outside 0..3", sh_degree);
    if (sh_degree == 1) return mgs_enhance_project(g, cam, packed_mlp, tile, alpha_min, out, phi, omod, stream);
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(packed_mlp && aligned(packed_mlp, 16), "packed MLP must be non-NULL and 16-byte aligned");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    const CamK k = make_camk(cam);
    const int64_t groups = (g->n + 63) / 64;
    int64_t blocks = (groups + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    auto launch = [&](auto src) {
        hipLaunchKernelGGL(enhance_project_kernel<decltype(src)>, dim3(unsigned(blocks)), dim3(256), 0,
                           as_stream(stream), src, k, static_cast<const uint8_t *>(packed_mlp), alpha_min,
                           reinterpret_cast<float4 *>(out->splat), reinterpret_cast<uint2 *>(out->rect),
                           out->n_tiles, phi, omod);
    };
    if (sh_degree == 0)
        launch(SoaShSource<0>{*g, {k.campos[0], k.campos[1], k.campos[2]}});
    else if (sh_degree == 2)
        launch(SoaShSource<2>{*g, {k.campos[0], k.campos[1], k.campos[2]}});
    else
        launch(SoaShSource<3>{*g, {k.campos[0], k.campos[1], k.campos[2]}});
    MGS_LAUNCH_CHECK("enhance_project_kernel<sh>");
    return MGS_OK;
}

extern "C" int mgs_project_weighted(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                                    const float *omod, int tile, float alpha_min, int weight_mode,
                                    mgs_projected *out, void *stream) {
    MGS_TRACE("mgs_project_weighted");
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
                       static_cast<const float *>(nullptr), static_cast<const float *>(nullptr), alpha_min,
                       reinterpret_cast<float4 *>(out->splat), reinterpret_cast<uint2 *>(out->rect), out->n_tiles);
    MGS_LAUNCH_CHECK("project_kernel");
    return MGS_OK;
}

extern "C" int mgs_project_sortfree(const mgs_gaussians *g, const mgs_camera *cam, const float *omod,
                                    const float *sigma, const float *beta, int tile, float alpha_min,
                                    mgs_projected *out, void *stream) {
    MGS_TRACE("mgs_project_sortfree");
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(sigma && beta, "sigma / beta is NULL");
    CamK k = make_camk(cam);
    k.weight_mode = MGS_WEIGHT_SORTFREE;
    const unsigned blocks = unsigned((g->n + 255) / 256);
    hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), *g, k,
                       static_cast<const float *>(nullptr), omod, sigma, beta, alpha_min,
                       reinterpret_cast<float4 *>(out->splat), reinterpret_cast<uint2 *>(out->rect), out->n_tiles);
    MGS_LAUNCH_CHECK("project_kernel<sortfree>");
    return MGS_OK;
}

extern "C" int mgs_enhance_project_sortfree(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp,
                                            const float *sigma, const float *beta, int tile, float alpha_min,
                                            mgs_projected *out, float *phi, float *omod, void *stream) {
    MGS_TRACE("mgs_enhance_project_sortfree");
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(packed_mlp && aligned(packed_mlp, 16), "packed MLP must be non-NULL and 16-byte aligned");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    MGS_REQUIRE(sigma && beta, "sigma / beta is NULL");
    CamK k = make_camk(cam);
    k.weight_mode = MGS_WEIGHT_SORTFREE;
    const int64_t groups = (g->n + 63) / 64;
    int64_t blocks = (groups + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(enhance_project_kernel<SoaSortfreeSource>, dim3(unsigned(blocks)), dim3(256), 0,
                       as_stream(stream), SoaSortfreeSource{*g, sigma, beta}, k,
                       static_cast<const uint8_t *>(packed_mlp), alpha_min, reinterpret_cast<float4 *>(out->splat),
                       reinterpret_cast<uint2 *>(out->rect), out->n_tiles, phi, omod);
    MGS_LAUNCH_CHECK("enhance_project_kernel<sortfree>");
    return MGS_OK;
}

extern "C" int mgs_project(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                           const float *omod, int tile, float alpha_min, mgs_projected *out,
                           void *stream) {
    return mgs_project_weighted(g, cam, phi, omod, tile, alpha_min, MGS_WEIGHT_EQ3, out, stream);
}

extern "C" int mgs_nvq_decode(const mgs_gaussians_nvq *q, float *log_scale, float *quat, float *opacity_logit,
                              float *sh, void *stream) {
    MGS_TRACE("mgs_nvq_decode");
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
    MGS_TRACE("mgs_enhance_project_nvq");
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

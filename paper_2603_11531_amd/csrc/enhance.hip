// mgs_mlp_pack / mgs_enhance: the view-dependent enhancement MLP of Eq. 4 on MFMA.
//
// Per Gaussian: x = [P_i, s_i, r_i, Y_i] (22 values, zero-padded to 32),
// h1 = ReLU(W1 x + b1), F = ReLU(W2 h1 + b2), phi = ReLU(w_phi . F + b_phi),
// m = sigmoid(w_o . F + b_o).  Inputs of every product are bfloat16; products
// accumulate in float32 (v_mfma_f32_16x16x32_bf16).
//
// Work layout.  A wave takes 64 Gaussians; each lane builds the 32 features of
// one Gaussian and stores them (bf16) to a per-wave LDS tile.  The network is
// evaluated transposed, H^T = W X^T, so the MFMA's M dimension is neurons and
// N is 16 Gaussians: the accumulator a lane ends up with (4 neurons of one
// Gaussian per 16-neuron block) is, after ReLU and conversion, exactly the
// B-operand fragment of the next layer once the K (input-neuron) axis of the
// next weight matrix is permuted to match -- which mgs_mlp_pack does once.
// No shuffles or LDS round trips between layers.  All weight fragments
// (14 x 16 bytes per lane) stay in registers for the wave's lifetime.
#include "mlp_math.h"

namespace mgs {

__global__ void __launch_bounds__(256)
mlp_pack_kernel(const float *__restrict__ prm, uint8_t *__restrict__ packed) {
    const float *W1 = prm + MGS_MLP_OFF_W1, *b1 = prm + MGS_MLP_OFF_B1, *W2 = prm + MGS_MLP_OFF_W2;
    const float *b2 = prm + MGS_MLP_OFF_B2, *wphi = prm + MGS_MLP_OFF_WPHI, *bphi = prm + MGS_MLP_OFF_BPHI;
    const float *wo = prm + MGS_MLP_OFF_WO, *bo = prm + MGS_MLP_OFF_BO;
    uint16_t *l1 = reinterpret_cast<uint16_t *>(packed + PK_L1);
    uint16_t *l2 = reinterpret_cast<uint16_t *>(packed + PK_L2);
    uint16_t *hh = reinterpret_cast<uint16_t *>(packed + PK_H);
    for (int e = threadIdx.x; e < 4 * 64 * 8; e += blockDim.x) {          // L1
        const int mb = e / 512, lane = (e / 8) % 64, j = e % 8;
        const int row = 16 * mb + lane % 16, k = 8 * (lane / 16) + j;
        l1[e] = bf16_bits_rne(k < MGS_MLP_IN ? W1[row * MGS_MLP_IN + k] : 0.0f);
    }
    for (int e = threadIdx.x; e < 4 * 2 * 64 * 8; e += blockDim.x) {      // L2
        const int mb = e / 1024, kc = (e / 512) % 2, lane = (e / 8) % 64, j = e % 8;
        const int row = 16 * mb + lane % 16;
        l2[e] = bf16_bits_rne(W2[row * MGS_MLP_HIDDEN + perm_neuron(kc, lane / 16, j)]);
    }
    for (int e = threadIdx.x; e < 2 * 64 * 8; e += blockDim.x) {          // heads
        const int kc = e / 512, lane = (e / 8) % 64, j = e % 8;
        const int row = lane % 16, k = perm_neuron(kc, lane / 16, j);
        const float v = row == 0 ? wphi[k] : (row == 1 ? wo[k] : 0.0f);
        hh[e] = bf16_bits_rne(v);
    }
    float *fb1 = reinterpret_cast<float *>(packed + PK_B1);
    float *fb2 = reinterpret_cast<float *>(packed + PK_B2);
    float *fbh = reinterpret_cast<float *>(packed + PK_BH);
    for (int e = threadIdx.x; e < 64; e += blockDim.x) {
        fb1[e] = b1[e];
        fb2[e] = b2[e];
    }
    if (threadIdx.x == 0) {
        fbh[0] = bphi[0];
        fbh[1] = bo[0];
    }
}

__global__ void __launch_bounds__(256)
enhance_kernel(mgs_gaussians g, CamK cam, const uint8_t *__restrict__ packed, float *__restrict__ phi,
               float *__restrict__ omod) {
    __shared__ __attribute__((aligned(16))) __bf16 s_x[4][64 * FEAT_STRIDE];
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int64_t ngroups = (g.n + 63) / 64;
    MlpFrags F;
    load_mlp(packed, l, F);
    for (int64_t grp = int64_t(blockIdx.x) * 4 + w; grp < ngroups; grp += int64_t(gridDim.x) * 4)
        enhance_group(g, cam, grp * 64, F, s_x[w], phi, omod, grp * 64);
}

}  // namespace mgs

extern "C" int mgs_mlp_pack(const float *params, void *packed, void *stream) {
    MGS_TRACE("mgs_mlp_pack");
    using namespace mgs;
    MGS_REQUIRE(params && packed, "params / packed is NULL");
    MGS_REQUIRE(aligned(params, 4) && aligned(packed, 16), "packed must be 16-byte aligned");
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(256), 0, as_stream(stream), params,
                       static_cast<uint8_t *>(packed));
    MGS_LAUNCH_CHECK("mlp_pack_kernel");
    return MGS_OK;
}

extern "C" int mgs_enhance(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp, float *phi,
                           float *omod, void *stream) {
    MGS_TRACE("mgs_enhance");
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    MGS_REQUIRE(packed_mlp && aligned(packed_mlp, 16), "packed MLP must be non-NULL and 16-byte aligned");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    const CamK k = make_camk(cam);
    const int64_t groups = (g->n + 63) / 64;
    int64_t blocks = (groups + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(enhance_kernel, dim3(unsigned(blocks)), dim3(256), 0, as_stream(stream), *g, k,
                       static_cast<const uint8_t *>(packed_mlp), phi, omod);
    MGS_LAUNCH_CHECK("enhance_kernel");
    return MGS_OK;
}

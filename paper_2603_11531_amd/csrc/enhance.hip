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
#include "common.h"

namespace mgs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

// Packed layout (bytes): L1 fragments [4 mb][64 lanes][8]        @ 0
//                        L2 fragments [4 mb][2 kc][64 lanes][8]  @ 4096
//                        head fragments [2 kc][64 lanes][8]      @ 12288
//                        b1[64] f32 @ 14336, b2[64] f32 @ 14592, b_phi, b_o @ 14848
constexpr int PK_L1 = 0, PK_L2 = 4096, PK_H = 12288, PK_B1 = 14336, PK_B2 = 14592, PK_BH = 14848;
static_assert(PK_BH + 8 <= MGS_MLP_PACKED_BYTES, "packed MLP size");

// Input neuron fed by K-slot j of K-chunk kc in lane group g (see header comment).
__host__ __device__ __forceinline__ int perm_neuron(int kc, int g, int j) {
    return 16 * (2 * kc + (j >> 2)) + 4 * g + (j & 3);
}

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

__device__ __forceinline__ bf16x8 relu_pack(f32x4 lo, f32x4 hi) {
    f32x8 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = fmaxf(lo[i], 0.0f);
        v[i + 4] = fmaxf(hi[i], 0.0f);
    }
    return __builtin_convertvector(v, bf16x8);
}

constexpr int FEAT_STRIDE = 40;   // bf16 per LDS row (32 + 8 padding)

__global__ void __launch_bounds__(256)
enhance_kernel(mgs_gaussians g, CamK cam, const uint8_t *__restrict__ packed, float *__restrict__ phi,
               float *__restrict__ omod) {
    __shared__ __attribute__((aligned(16))) __bf16 s_x[4][64 * FEAT_STRIDE];
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int lg = l >> 4;           // lane group
    const int64_t n = g.n;
    const int64_t ngroups = (n + 63) / 64;

    // weight fragments and biases, resident for the wave's lifetime
    const bf16x8 *pl1 = reinterpret_cast<const bf16x8 *>(packed + PK_L1);
    const bf16x8 *pl2 = reinterpret_cast<const bf16x8 *>(packed + PK_L2);
    const bf16x8 *phh = reinterpret_cast<const bf16x8 *>(packed + PK_H);
    const float *fb1 = reinterpret_cast<const float *>(packed + PK_B1);
    const float *fb2 = reinterpret_cast<const float *>(packed + PK_B2);
    const float *fbh = reinterpret_cast<const float *>(packed + PK_BH);
    bf16x8 A1[4], A2[4][2], AH[2];
    f32x4 B1[4], B2[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        A1[mb] = pl1[mb * 64 + l];
        A2[mb][0] = pl2[(mb * 2 + 0) * 64 + l];
        A2[mb][1] = pl2[(mb * 2 + 1) * 64 + l];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            B1[mb][i] = fb1[16 * mb + 4 * lg + i];
            B2[mb][i] = fb2[16 * mb + 4 * lg + i];
        }
    }
    AH[0] = phh[l];
    AH[1] = phh[64 + l];
    const float bphi = fbh[0], bo = fbh[1];

    __bf16 *xs = s_x[w];
    for (int64_t grp = int64_t(blockIdx.x) * 4 + w; grp < ngroups; grp += int64_t(gridDim.x) * 4) {
        const int64_t i = grp * 64 + l;
        f32x8 f[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (i < n) {
            const float mx = g.mean[i], my = g.mean[n + i], mz = g.mean[2 * n + i];
            const float vx = mx - cam.campos[0], vy = my - cam.campos[1], vz = mz - cam.campos[2];
            const float vn = rsqrtf(vx * vx + vy * vy + vz * vz);
            float qw = g.quat[i], qx = g.quat[n + i], qy = g.quat[2 * n + i], qz = g.quat[3 * n + i];
            const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
            const float qi = qn2 > 0.f ? rsqrtf(qn2) : 0.f;
            f[0][0] = vx * vn; f[0][1] = vy * vn; f[0][2] = vz * vn;
            f[0][3] = expf(g.log_scale[i]);
            f[0][4] = expf(g.log_scale[n + i]);
            f[0][5] = expf(g.log_scale[2 * n + i]);
            f[0][6] = qw * qi; f[0][7] = qx * qi;
            f[1][0] = qy * qi; f[1][1] = qz * qi;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const float y = g.sh[k * n + i];
                const int slot = 10 + k;
                f[slot >> 3][slot & 7] = y;
            }
        }
        bf16x8 *row = reinterpret_cast<bf16x8 *>(xs + l * FEAT_STRIDE);
#pragma unroll
        for (int c = 0; c < 4; ++c) row[c] = __builtin_convertvector(f[c], bf16x8);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(xs + (nb * 16 + (l & 15)) * FEAT_STRIDE + 8 * lg);
            f32x4 h1[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) h1[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[mb], xb, B1[mb], 0, 0, 0);
            const bf16x8 x2a = relu_pack(h1[0], h1[1]);
            const bf16x8 x2b = relu_pack(h1[2], h1[3]);
            f32x4 h2[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                h2[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[mb][0], x2a, B2[mb], 0, 0, 0);
                h2[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[mb][1], x2b, h2[mb], 0, 0, 0);
            }
            const bf16x8 xha = relu_pack(h2[0], h2[1]);
            const bf16x8 xhb = relu_pack(h2[2], h2[3]);
            f32x4 hz = {0.f, 0.f, 0.f, 0.f};
            f32x4 hd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH[0], xha, hz, 0, 0, 0);
            hd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH[1], xhb, hd, 0, 0, 0);
            const int64_t gi = grp * 64 + nb * 16 + l;
            if (l < 16 && gi < n) {
                phi[gi] = fmaxf(hd[0] + bphi, 0.0f);
                omod[gi] = 1.0f / (1.0f + expf(-(hd[1] + bo)));
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace mgs

extern "C" int mgs_mlp_pack(const float *params, void *packed, void *stream) {
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

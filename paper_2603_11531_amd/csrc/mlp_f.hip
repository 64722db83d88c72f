// mgs_mlp_f_pack / mgs_enhance_project_mlp_f: the appendix's enhancement network MLP_f
// (ReLU hidden layers of 256, 128 and 64 neurons) fused with the projection.
//
// About 98 kFLOP per Gaussian (the first layer's 22 inputs padded to 32), so unlike the
// two-layer network this pass is bound by the matrix cores, not by HBM.  Work layout:
//
//   * a workgroup of 8 waves keeps the packed network (bf16 A-operand fragments of
//     v_mfma_f32_32x32x16_bf16 plus float32 biases, ~102 KB) in LDS; one workgroup per CU;
//   * a wave takes 64 Gaussians as two 32-column N tiles, so every weight fragment read
//     from LDS feeds two matrix instructions;
//   * the network runs transposed, H^T = W X^T (neurons on M).  A 32x32 accumulator leaves
//     neuron 8 (r / 4) + 4 h + r % 4 of Gaussian c in lane c + 32 h, register r; after bias
//     (folded into the accumulator's initial value), ReLU and conversion, registers
//     8 s .. 8 s + 7 are exactly the B operand of K step s of the next layer, once that
//     layer's input axis is permuted to match at pack time (mlpf_perm).  No shuffles and no
//     LDS round trips between layers;
//   * the first layer's 32 x 64 output tile is consumed by the second layer's partial
//     products as soon as it is made, so only the second layer's 128 x 64 accumulator
//     stays live across the first layer;
//   * (phi, m) go back to the Gaussian's own lane through LDS and the lane projects as in
//     mgs_enhance_project.
#include "mlp_math.h"
#include "proj_math.h"

namespace mgs {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Packed layout (bytes): fragments of 64 lanes x 8 bf16 (1 KB each)
constexpr int MF_L1 = 0;             // [8 m tiles][2 k steps]   W1, inputs in natural order
constexpr int MF_L2 = 16384;         // [4 m tiles][16 k steps]  W2, inputs permuted
constexpr int MF_L3 = 81920;         // [2 m tiles][8 k steps]   W3, inputs permuted
constexpr int MF_H = 98304;          // [4 k steps]              rows 0 = w_phi, 1 = w_o
constexpr int MF_B1 = 102400, MF_B2 = 103424, MF_B3 = 103936, MF_BH = 104192;
static_assert(MF_BH + 8 <= MGS_MLPF_PACKED_BYTES && MGS_MLPF_PACKED_BYTES % 16 == 0, "packed MLP_f size");
#ifndef MGS_MLPF_NT
#define MGS_MLPF_NT 2
#endif
#ifndef MGS_MLPF_THREADS
#define MGS_MLPF_THREADS 512
#endif
// 32-Gaussian N tiles per MLP pass, and the workgroup size (one workgroup per CU).  Measured on
// the 1M-Gaussian workload: NT = 2 with 512 threads (238 VGPRs, two waves per SIMD) 117 us;
// NT = 1 with 1024 threads (128 VGPRs, four waves per SIMD, twice the LDS weight traffic) 127 us;
// NT = 1 with 768 threads 130 us.
constexpr int MF_NT = MGS_MLPF_NT;
constexpr int MF_THREADS = MGS_MLPF_THREADS;

// Input neuron of the next layer fed by K step ks, lane half h, slot e of a B fragment made
// from registers 8 s .. 8 s + 7 of an accumulator (see the header comment).
__host__ __device__ __forceinline__ int mlpf_perm(int ks, int h, int e) { return 16 * ks + 8 * (e >> 2) + 4 * h + (e & 3); }

__global__ void __launch_bounds__(256)
mlpf_pack_kernel(const float *__restrict__ prm, uint8_t *__restrict__ packed) {
    const float *W1 = prm + MGS_MLPF_OFF_W1, *W2 = prm + MGS_MLPF_OFF_W2, *W3 = prm + MGS_MLPF_OFF_W3;
    const float *wphi = prm + MGS_MLPF_OFF_WPHI, *wo = prm + MGS_MLPF_OFF_WO;
    uint16_t *l1 = reinterpret_cast<uint16_t *>(packed + MF_L1);
    uint16_t *l2 = reinterpret_cast<uint16_t *>(packed + MF_L2);
    uint16_t *l3 = reinterpret_cast<uint16_t *>(packed + MF_L3);
    uint16_t *hh = reinterpret_cast<uint16_t *>(packed + MF_H);
    // element e of fragment f: lane (e / 8) % 64, slot e % 8; row = lane % 32, half = lane / 32
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 16 * 512; e += gridDim.x * blockDim.x) {
        const int f = e / 512, lane = (e / 8) % 64, j = e % 8;
        const int mt = f / 2, s = f % 2, row = 32 * mt + lane % 32, k = 16 * s + 8 * (lane / 32) + j;
        l1[e] = bf16_bits_rne(k < MGS_MLP_IN ? W1[row * MGS_MLP_IN + k] : 0.0f);
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 64 * 512; e += gridDim.x * blockDim.x) {
        const int f = e / 512, lane = (e / 8) % 64, j = e % 8;
        const int mt = f / 16, ks = f % 16, row = 32 * mt + lane % 32;
        l2[e] = bf16_bits_rne(W2[row * 256 + mlpf_perm(ks, lane / 32, j)]);
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 16 * 512; e += gridDim.x * blockDim.x) {
        const int f = e / 512, lane = (e / 8) % 64, j = e % 8;
        const int mt = f / 8, ks = f % 8, row = 32 * mt + lane % 32;
        l3[e] = bf16_bits_rne(W3[row * 128 + mlpf_perm(ks, lane / 32, j)]);
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 4 * 512; e += gridDim.x * blockDim.x) {
        const int ks = e / 512, lane = (e / 8) % 64, j = e % 8, row = lane % 32;
        const int k = mlpf_perm(ks, lane / 32, j);
        hh[e] = bf16_bits_rne(row == 0 ? wphi[k] : (row == 1 ? wo[k] : 0.0f));
    }
    float *fb1 = reinterpret_cast<float *>(packed + MF_B1), *fb2 = reinterpret_cast<float *>(packed + MF_B2);
    float *fb3 = reinterpret_cast<float *>(packed + MF_B3), *fbh = reinterpret_cast<float *>(packed + MF_BH);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 256; e += gridDim.x * blockDim.x) {
        fb1[e] = prm[MGS_MLPF_OFF_B1 + e];
        if (e < 128) fb2[e] = prm[MGS_MLPF_OFF_B2 + e];
        if (e < 64) fb3[e] = prm[MGS_MLPF_OFF_B3 + e];
        if (e == 0) {
            fbh[0] = prm[MGS_MLPF_OFF_BPHI];
            fbh[1] = prm[MGS_MLPF_OFF_BO];
        }
    }
}

// Accumulator initial value of M tile rows b[0 .. 32): register r of lane half h holds row
// 8 (r / 4) + 4 h + r % 4.
__device__ __forceinline__ f32x16 bias_tile(const float *b, int h) {
    f32x16 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4 x = *reinterpret_cast<const f32x4 *>(b + 8 * q + 4 * h);
#pragma unroll
        for (int p = 0; p < 4; ++p) v[4 * q + p] = x[p];
    }
    return v;
}

// ReLU of registers 8 s .. 8 s + 7, as the bf16 B fragment of one K step (relu_bf16x2).
__device__ __forceinline__ bf16x8 relu_half(const f32x16 &v, int s) {
    bf16x8 b;
    i16x2 *u = reinterpret_cast<i16x2 *>(&b);
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = relu_bf16x2(v[8 * s + 2 * q], v[8 * s + 2 * q + 1]);
    return b;
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// MLP_f for the 32 NT Gaussians g0 + 32 nt + c (nt < NT) of a wave; (phi, m) of Gaussian
// g0 + k - base go to xo[k] and xo[64 + k] (k = 32 nt + c + o, o the pass offset).
template <int NT>
__device__ __forceinline__ void mlpf_pass(const mgs_gaussians &g, const CamK &cam, int64_t g0, int o,
                                          const uint8_t *s_w, float *xo) {
    const int l = threadIdx.x & 63, h = l >> 5, c = l & 31;
    const bf16x8 *A1 = reinterpret_cast<const bf16x8 *>(s_w + MF_L1) + l;
    const bf16x8 *A2 = reinterpret_cast<const bf16x8 *>(s_w + MF_L2) + l;
    const bf16x8 *A3 = reinterpret_cast<const bf16x8 *>(s_w + MF_L3) + l;
    const bf16x8 *AH = reinterpret_cast<const bf16x8 *>(s_w + MF_H) + l;
    const float *b1 = reinterpret_cast<const float *>(s_w + MF_B1);
    const float *b2 = reinterpret_cast<const float *>(s_w + MF_B2);
    const float *b3 = reinterpret_cast<const float *>(s_w + MF_B3);
    const float *bh = reinterpret_cast<const float *>(s_w + MF_BH);
    const int64_t n = g.n;
    // B fragments of the first layer: features 16 s + 8 h .. + 7 of Gaussian g0 + 32 nt + c
    bf16x8 x[NT][2];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t i = g0 + 32 * nt + c;
        f32x8 f[4];
        if (i < n) {
            const GaussIn a = load_gauss(g, i, nullptr, nullptr);
            lane_features(a.mu, a.ls, a.q, a.sh, cam, f);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) f[q] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
        // lane half h takes features 16 s + 8 h .. + 7 (a select, not a dynamic register index)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            f32x8 y;
#pragma unroll
            for (int e = 0; e < 8; ++e) y[e] = h ? f[2 * s + 1][e] : f[2 * s][e];
            x[nt][s] = __builtin_convertvector(y, bf16x8);
        }
    }
    // layers 1 and 2: each 32-neuron tile of layer 1 feeds two K steps of layer 2 at once
    f32x16 acc2[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const f32x16 b = bias_tile(b2 + 32 * mt, h);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc2[mt][nt] = b;
    }
#pragma unroll 1
    for (int t = 0; t < 8; ++t) {
        __asm__ volatile("" ::: "memory");
        const f32x16 b = bias_tile(b1 + 32 * t, h);
        f32x16 h1[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) h1[nt] = mfma32(A1[(2 * t) * 64], x[nt][0], b);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) h1[nt] = mfma32(A1[(2 * t + 1) * 64], x[nt][1], h1[nt]);
        bf16x8 p[NT][2];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int s = 0; s < 2; ++s) p[nt][s] = relu_half(h1[nt], s);
        // K step s outer: the accumulators are updated in turn, so no instruction waits on the
        // one just issued
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 a = A2[(16 * mt + 2 * t + s) * 64];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc2[mt][nt] = mfma32(a, p[nt][s], acc2[mt][nt]);
            }
    }
    // layer 3
    bf16x8 x3[NT][8];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) x3[nt][2 * mt + s] = relu_half(acc2[mt][nt], s);
    f32x16 acc3[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const f32x16 b = bias_tile(b3 + 32 * mt, h);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc3[mt][nt] = b;
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const bf16x8 a = A3[(8 * mt + ks) * 64];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc3[mt][nt] = mfma32(a, x3[nt][ks], acc3[mt][nt]);
        }
    // heads: row 0 phi, row 1 m
    bf16x8 xh[NT][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) xh[nt][2 * mt + s] = relu_half(acc3[mt][nt], s);
    f32x16 hd[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) hd[nt] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const bf16x8 a = AH[ks * 64];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) hd[nt] = mfma32(a, xh[nt][ks], hd[nt]);
    }
    // (phi, m) of Gaussian 32 nt + c sit in lane c (h = 0), registers 0 and 1
    if (h == 0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            xo[o + 32 * nt + c] = fmaxf(hd[nt][0] + bh[0], 0.0f);
            xo[64 + o + 32 * nt + c] = 1.0f / (1.0f + expf(-(hd[nt][1] + bh[1])));
        }
    }
}

// A wave takes 64 Gaussians per task: MLP_f in 2 / NT passes of 32 NT Gaussians (NT = 2: each
// weight fragment read from LDS feeds two matrix instructions; NT = 1: half the accumulator
// registers, more waves per SIMD), then one projection per lane.
template <int NT, int THREADS>
__global__ void __launch_bounds__(THREADS)
enhance_project_mlpf_kernel(mgs_gaussians g, CamK cam, const uint8_t *__restrict__ packed, float alpha_min,
                            float4 *__restrict__ splat, uint2 *__restrict__ rect_out,
                            uint32_t *__restrict__ ntiles_out, float *__restrict__ phi_out,
                            float *__restrict__ omod_out) {
    __shared__ __attribute__((aligned(16))) uint8_t s_w[MGS_MLPF_PACKED_BYTES];
    __shared__ float s_xo[THREADS / 64][128];
    for (int k = threadIdx.x; k < MGS_MLPF_PACKED_BYTES / 16; k += blockDim.x)
        reinterpret_cast<uint4 *>(s_w)[k] = reinterpret_cast<const uint4 *>(packed)[k];
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t n = g.n, ngroups = (n + 63) / 64;
    const int wpb = THREADS / 64;
    for (int64_t grp = int64_t(blockIdx.x) * wpb + w; grp < ngroups; grp += int64_t(gridDim.x) * wpb) {
#pragma unroll 1
        for (int o = 0; o < 64; o += 32 * NT) {
            // weights and biases are read from LDS at each use: keep the compiler from hoisting
            // those loads out of the loops into (spilled) registers
            __asm__ volatile("" ::: "memory");
            mlpf_pass<NT>(g, cam, grp * 64 + o, o, s_w, s_xo[w]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float ph = s_xo[w][l], om = s_xo[w][64 + l];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t i = grp * 64 + l;
        if (i < n) {
            GaussIn in = load_gauss(g, i, nullptr, nullptr);
            in.phi = ph;
            in.om = om;
            store_proj(project_gaussian(in, cam, alpha_min), i, splat, rect_out, ntiles_out);
            phi_out[i] = ph;
            omod_out[i] = om;
        }
    }
}

}  // namespace mgs

extern "C" int mgs_mlp_f_pack(const float *params, void *packed, void *stream) {
    MGS_TRACE("mgs_mlp_f_pack");
    using namespace mgs;
    MGS_REQUIRE(params && packed, "params / packed is NULL");
    MGS_REQUIRE(aligned(params, 4) && aligned(packed, 16), "packed must be 16-byte aligned");
    hipLaunchKernelGGL(mlpf_pack_kernel, dim3(32), dim3(256), 0, as_stream(stream), params,
                       static_cast<uint8_t *>(packed));
    MGS_LAUNCH_CHECK("mlpf_pack_kernel");
    return MGS_OK;
}

extern "C" int mgs_enhance_project_mlp_f(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp_f,
                                         int tile, float alpha_min, mgs_projected *out, float *phi, float *omod,
                                         void *stream) {
    MGS_TRACE("mgs_enhance_project_mlp_f");
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(out, g->n)) != MGS_OK) return rc;
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(alpha_min > 0.0f && alpha_min < 1.0f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(packed_mlp_f && aligned(packed_mlp_f, 16), "packed MLP_f must be non-NULL and 16-byte aligned");
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(phi && omod, "phi / omod is NULL");
    const CamK k = make_camk(cam);
    // one workgroup per CU holds the network in LDS; the grid strides over 64-Gaussian groups
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;                                  // the grid size only; any positive count is correct
    const int64_t groups = (g->n + 63) / 64, per_block = MF_THREADS / 64;
    int64_t blocks = (groups + per_block - 1) / per_block;
    if (blocks > cus) blocks = cus;
    hipLaunchKernelGGL((enhance_project_mlpf_kernel<MF_NT, MF_THREADS>), dim3(unsigned(blocks)), dim3(MF_THREADS), 0,
                       as_stream(stream), *g, k, static_cast<const uint8_t *>(packed_mlp_f), alpha_min,
                       reinterpret_cast<float4 *>(out->splat), reinterpret_cast<uint2 *>(out->rect), out->n_tiles,
                       phi, omod);
    MGS_LAUNCH_CHECK("enhance_project_mlpf_kernel");
    return MGS_OK;
}

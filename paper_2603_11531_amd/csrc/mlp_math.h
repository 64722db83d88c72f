// Enhancement-MLP device code shared by mgs_enhance and the batched renderer.
#pragma once

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

// ReLU then bf16 of (lo, hi).  Converted first, then clamped as signed 16-bit integers (a
// negative bf16, -0 included, has the sign bit set): the same bits as converting max(x, 0),
// one conversion per pair of values and one packed integer max per pair.
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ i16x2 relu_bf16x2(float a, float b) {
    const bf16x2 c = __builtin_convertvector(f32x2{a, b}, bf16x2);
    return __builtin_elementwise_max(__builtin_bit_cast(i16x2, c), i16x2{0, 0});
}
__device__ __forceinline__ bf16x8 relu_pack(f32x4 lo, f32x4 hi) {
    bf16x8 r;
    i16x2 *u = reinterpret_cast<i16x2 *>(&r);
    u[0] = relu_bf16x2(lo[0], lo[1]);
    u[1] = relu_bf16x2(lo[2], lo[3]);
    u[2] = relu_bf16x2(hi[0], hi[1]);
    u[3] = relu_bf16x2(hi[2], hi[3]);
    return r;
}

// LDS feature tile: 64 rows of 32 bf16 (64 bytes), the four 16-byte chunks of row r stored
// in the order c ^ ((r >> 2) & 3), so 16 consecutive rows' chunk c (the MFMA operand reads) and
// 16 consecutive rows written whole both fall in distinct banks.
constexpr int FEAT_STRIDE = 32;
__device__ __forceinline__ int feat_chunk(int row, int c) { return c ^ ((row >> 2) & 3); }

// Weight fragments and biases of one packed MLP, held in registers by a wave.
struct MlpFrags {
    bf16x8 A1[4], A2[4][2], AH[2];
    f32x4 B1[4], B2[4];
    float bphi, bo;
    static constexpr bool kStreamed = false;
    __device__ __forceinline__ bf16x8 a1(int mb) const { return A1[mb]; }
    __device__ __forceinline__ bf16x8 a2(int mb, int kc) const { return A2[mb][kc]; }
    __device__ __forceinline__ bf16x8 ah(int kc) const { return AH[kc]; }
    __device__ __forceinline__ f32x4 b1(int mb) const { return B1[mb]; }
    __device__ __forceinline__ f32x4 b2(int mb) const { return B2[mb]; }
    __device__ __forceinline__ float b_phi() const { return bphi; }
    __device__ __forceinline__ float b_o() const { return bo; }
};

// The same fragments read from a copy of the packed MLP in LDS at each use (for kernels
// whose other live state leaves no room for them in registers).
struct MlpLds {
    const uint8_t *p;    // packed MLP (MGS_MLP_PACKED_BYTES) in LDS
    int l;               // lane
    static constexpr bool kStreamed = true;
    __device__ __forceinline__ bf16x8 a1(int mb) const {
        return reinterpret_cast<const bf16x8 *>(p + PK_L1)[mb * 64 + l];
    }
    __device__ __forceinline__ bf16x8 a2(int mb, int kc) const {
        return reinterpret_cast<const bf16x8 *>(p + PK_L2)[(mb * 2 + kc) * 64 + l];
    }
    __device__ __forceinline__ bf16x8 ah(int kc) const { return reinterpret_cast<const bf16x8 *>(p + PK_H)[kc * 64 + l]; }
    __device__ __forceinline__ f32x4 b1(int mb) const {
        return *reinterpret_cast<const f32x4 *>(p + PK_B1 + 4 * (16 * mb + 4 * (l >> 4)));
    }
    __device__ __forceinline__ f32x4 b2(int mb) const {
        return *reinterpret_cast<const f32x4 *>(p + PK_B2 + 4 * (16 * mb + 4 * (l >> 4)));
    }
    __device__ __forceinline__ float b_phi() const { return reinterpret_cast<const float *>(p + PK_BH)[0]; }
    __device__ __forceinline__ float b_o() const { return reinterpret_cast<const float *>(p + PK_BH)[1]; }
};

__device__ __forceinline__ void load_mlp(const uint8_t *__restrict__ packed, int l, MlpFrags &F) {
    const int lg = l >> 4;
    const bf16x8 *pl1 = reinterpret_cast<const bf16x8 *>(packed + PK_L1);
    const bf16x8 *pl2 = reinterpret_cast<const bf16x8 *>(packed + PK_L2);
    const bf16x8 *phh = reinterpret_cast<const bf16x8 *>(packed + PK_H);
    const float *fb1 = reinterpret_cast<const float *>(packed + PK_B1);
    const float *fb2 = reinterpret_cast<const float *>(packed + PK_B2);
    const float *fbh = reinterpret_cast<const float *>(packed + PK_BH);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        F.A1[mb] = pl1[mb * 64 + l];
        F.A2[mb][0] = pl2[(mb * 2 + 0) * 64 + l];
        F.A2[mb][1] = pl2[(mb * 2 + 1) * 64 + l];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            F.B1[mb][i] = fb1[16 * mb + 4 * lg + i];
            F.B2[mb][i] = fb2[16 * mb + 4 * lg + i];
        }
    }
    F.AH[0] = phh[l];
    F.AH[1] = phh[64 + l];
    F.bphi = fbh[0];
    F.bo = fbh[1];
}

// The 32 MLP inputs of one Gaussian: [P_i (3), s_i (3), q_i (4), Y_i (12)], zero-padded.
__device__ __forceinline__ void lane_features(const float mu[3], const float ls[3], const float q[4],
                                              const float sh[12], const CamK &cam, f32x8 f[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
    const float vx = mu[0] - cam.campos[0], vy = mu[1] - cam.campos[1], vz = mu[2] - cam.campos[2];
    const float vn = rsqrtf(vx * vx + vy * vy + vz * vz);
    const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const float qi = qn2 > 0.f ? rsqrtf(qn2) : 0.f;
    f[0][0] = vx * vn; f[0][1] = vy * vn; f[0][2] = vz * vn;
    f[0][3] = expf(ls[0]);
    f[0][4] = expf(ls[1]);
    f[0][5] = expf(ls[2]);
    f[0][6] = q[0] * qi; f[0][7] = q[1] * qi;
    f[1][0] = q[2] * qi; f[1][1] = q[3] * qi;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const int slot = 10 + k;
        f[slot >> 3][slot & 7] = sh[k];
    }
}

// The MLP for the wave's 64 Gaussians (lane l holds the features of Gaussian l);
// returns lane l's (phi, m).  xs: the wave's LDS feature tile (its first 128
// floats are reused to hand the head outputs back to their lanes).
template <typename W>
__device__ __forceinline__ void mlp_wave(const f32x8 f[4], const W &F, __bf16 *xs, float &phi_o, float &om_o) {
    const int l = threadIdx.x & 63;
    const int lg = l >> 4;
    bf16x8 *row = reinterpret_cast<bf16x8 *>(xs + l * FEAT_STRIDE);
#pragma unroll
    for (int c = 0; c < 4; ++c) row[feat_chunk(l, c)] = __builtin_convertvector(f[c], bf16x8);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Gaussians nb * 16 .. nb * 16 + 15; their head outputs land in xo[nb * 16 + l] (phi) and
    // xo[64 + nb * 16 + l] (m), lanes 0..15.  xo overlays feature rows 0..7, which block 0 has
    // consumed before any block writes there.
    float *xo = reinterpret_cast<float *>(xs);
    auto block = [&](int nb) {
        const int xr = nb * 16 + (l & 15);
        const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(xs + xr * FEAT_STRIDE + 8 * feat_chunk(xr, lg));
        f32x4 h1[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) h1[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a1(mb), xb, F.b1(mb), 0, 0, 0);
        const bf16x8 x2a = relu_pack(h1[0], h1[1]);
        const bf16x8 x2b = relu_pack(h1[2], h1[3]);
        // streamed weights: keep each layer's fragment loads inside that layer
        if constexpr (W::kStreamed) __builtin_amdgcn_sched_barrier(0);
        f32x4 h2[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            h2[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2(mb, 0), x2a, F.b2(mb), 0, 0, 0);
            h2[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2(mb, 1), x2b, h2[mb], 0, 0, 0);
        }
        const bf16x8 xha = relu_pack(h2[0], h2[1]);
        const bf16x8 xhb = relu_pack(h2[2], h2[3]);
        if constexpr (W::kStreamed) __builtin_amdgcn_sched_barrier(0);
        f32x4 hz = {0.f, 0.f, 0.f, 0.f};
        f32x4 hd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.ah(0), xha, hz, 0, 0, 0);
        hd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.ah(1), xhb, hd, 0, 0, 0);
        if (l < 16) {                                       // lanes 0..15 hold Gaussian nb * 16 + l
            xo[nb * 16 + l] = fmaxf(hd[0] + F.b_phi(), 0.0f);
            xo[64 + nb * 16 + l] = 1.0f / (1.0f + expf(-(hd[1] + F.b_o())));
        }
    };
    if constexpr (W::kStreamed) {
        // weights come from LDS at each use: one block at a time keeps few of them live
#pragma unroll 1
        for (int nb = 0; nb < 4; ++nb) block(nb);
    } else {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) block(nb);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    phi_o = xo[l];
    om_o = xo[64 + l];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The MLP for the 64 Gaussians i0 .. i0 + 63 of g (indices >= g.n are padding), one wave;
// outputs to phi / omod at out0 + k.  xs: this wave's LDS feature tile.
__device__ __forceinline__ void enhance_group(const mgs_gaussians &g, const CamK &cam, int64_t i0,
                                              const MlpFrags &F, __bf16 *xs, float *__restrict__ phi,
                                              float *__restrict__ omod, int64_t out0) {
    const int l = threadIdx.x & 63;
    const int64_t n = g.n;
    const int64_t i = i0 + l;
    f32x8 f[4];
    if (i < n) {
        float mu[3], ls[3], q[4], sh[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mu[k] = g.mean[k * n + i];
            ls[k] = g.log_scale[k * n + i];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = g.quat[k * n + i];
#pragma unroll
        for (int k = 0; k < 12; ++k) sh[k] = g.sh[k * n + i];
        lane_features(mu, ls, q, sh, cam, f);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) f[c] = f32x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
    float ph, om;
    mlp_wave(f, F, xs, ph, om);
    if (i < n) {
        phi[out0 + l] = ph;
        omod[out0 + l] = om;
    }
}

}  // namespace mgs

// Per-Gaussian forward math shared by mgs_project and the backward pass (which
// recomputes it instead of storing intermediates).
#pragma once

#include <math.h>

#include "common.h"

namespace mgs {

constexpr float SH_C0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float SH_C1 = 0.48860251190291992f;   // sqrt(3) / (2 sqrt(pi))
constexpr float EWA_DILATION = 0.3f;
constexpr float FRUSTUM_CLAMP = 1.3f;

struct GaussIn {
    float mu[3], ls[3], q[4], logit, sh[12];
    float phi, om;
    float cext[3];            // SH terms above first order, added before the colour clamp (0 for SH1)
    float wsig = 0.0f, wbeta = 1.0f;   // sigma_i, beta_i of the Eq. 1 weight (MGS_WEIGHT_SORTFREE only)
};

struct GaussFwd {
    // camera space
    float xc, yc, z;
    bool clamp_x, clamp_y;
    float txz, tyz;
    // activation
    float s[3], qn[4], qnorm, sig, o;
    float r[3][3];            // rotation matrix R(qn), r[i][k]: row i, column k
    // view direction
    float v[3], vlen, P[3];
    // colour (pre-clamp value and clamped)
    float cpre[3], col[3];
    // weight
    float smax; int kmax; float esd, w, phi;
    // EWA
    float J00, J02, J11, J12;
    float M[2][3];
    float u[3][2];            // u_k = s_k M r_k
    float a0, b, c0, a, c, det;
    float mx, my;
    bool front;
};

__device__ __forceinline__ GaussIn load_gauss(const mgs_gaussians &g, int64_t i, const float *phi_in,
                                              const float *om_in) {
    GaussIn in;
    const int64_t n = g.n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        in.mu[k] = g.mean[k * n + i];
        in.ls[k] = g.log_scale[k * n + i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) in.q[k] = g.quat[k * n + i];
    in.logit = g.opacity_logit[i];
#pragma unroll
    for (int k = 0; k < 12; ++k) in.sh[k] = g.sh[k * n + i];
    in.phi = phi_in ? phi_in[i] : 1.0f;
    in.om = om_in ? om_in[i] : 1.0f;
    in.cext[0] = in.cext[1] = in.cext[2] = 0.0f;
    return in;
}

// Reciprocals (v_rcp_f32, ~1 ulp) stand in for the divisions of the quantities whose float32 error
// is compared relatively: the rotation, opacity, view direction, weight and conic coefficients.
// The screen mean keeps the correctly rounded 1 / z, since the ambiguity band of the alpha cut is
// sized from its rounding error; the pass is latency bound and the shorter dependent chains saved
// ~3% of it.
__device__ __forceinline__ GaussFwd gauss_forward(const GaussIn &in, const CamK &cam) {
    GaussFwd f;
    const float *R = cam.R;
    f.xc = R[0] * in.mu[0] + R[1] * in.mu[1] + R[2] * in.mu[2] + cam.t[0];
    f.yc = R[3] * in.mu[0] + R[4] * in.mu[1] + R[5] * in.mu[2] + cam.t[1];
    const float d = R[6] * in.mu[0] + R[7] * in.mu[1] + R[8] * in.mu[2] + cam.t[2];
    f.front = d > cam.near_z;
    f.z = f.front ? d : 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) f.s[k] = expf(in.ls[k]);
    const float qn2 = in.q[0] * in.q[0] + in.q[1] * in.q[1] + in.q[2] * in.q[2] + in.q[3] * in.q[3];
    f.qnorm = sqrtf(qn2);
    const float qi = qn2 > 0.f ? __builtin_amdgcn_rcpf(f.qnorm) : 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) f.qn[k] = in.q[k] * qi;
    const float w = f.qn[0], x = f.qn[1], y = f.qn[2], z = f.qn[3];
    f.r[0][0] = 1.f - 2.f * (y * y + z * z); f.r[0][1] = 2.f * (x * y - w * z); f.r[0][2] = 2.f * (x * z + w * y);
    f.r[1][0] = 2.f * (x * y + w * z); f.r[1][1] = 1.f - 2.f * (x * x + z * z); f.r[1][2] = 2.f * (y * z - w * x);
    f.r[2][0] = 2.f * (x * z - w * y); f.r[2][1] = 2.f * (y * z + w * x); f.r[2][2] = 1.f - 2.f * (x * x + y * y);
    f.sig = __builtin_amdgcn_rcpf(1.0f + expf(-in.logit));
    f.o = f.sig * in.om;

#pragma unroll
    for (int k = 0; k < 3; ++k) f.v[k] = in.mu[k] - cam.campos[k];
    f.vlen = sqrtf(f.v[0] * f.v[0] + f.v[1] * f.v[1] + f.v[2] * f.v[2]);
    const float vi = __builtin_amdgcn_rcpf(f.vlen);
#pragma unroll
    for (int k = 0; k < 3; ++k) f.P[k] = f.v[k] * vi;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        f.cpre[ch] = 0.5f + SH_C0 * in.sh[ch] +
                     SH_C1 * (-f.P[1] * in.sh[3 + ch] + f.P[2] * in.sh[6 + ch] - f.P[0] * in.sh[9 + ch]) +
                     in.cext[ch];
        f.col[ch] = fmaxf(0.0f, f.cpre[ch]);
    }

    f.kmax = 0;
    f.smax = f.s[0];
    if (f.s[1] > f.smax) { f.smax = f.s[1]; f.kmax = 1; }
    if (f.s[2] > f.smax) { f.smax = f.s[2]; f.kmax = 2; }
    f.phi = in.phi;
    // Eq. 3, its ablations without the depth (d = 1) or without the scale term, or Eq. 1
    if (cam.weight_mode == MGS_WEIGHT_NO_DEPTH) {
        f.esd = expf(f.smax);
        f.w = in.phi * in.phi + in.phi + f.esd;
    } else if (cam.weight_mode == MGS_WEIGHT_NO_SCALE) {
        f.esd = 0.0f;
        f.w = in.phi * in.phi + in.phi / (f.z * f.z);
    } else if (cam.weight_mode == MGS_WEIGHT_SORTFREE) {
        // Eq. 1's weighting function w(d) = exp(-sigma d^beta); d > near_z > 0 for every
        // Gaussian that reaches the blend (culled ones use z = 1)
        f.esd = 0.0f;
        f.w = expf(-in.wsig * powf(f.z, in.wbeta));
    } else {
        const float izw = __builtin_amdgcn_rcpf(f.z);
        f.esd = expf(f.smax * izw);
        f.w = in.phi * in.phi + in.phi * izw * izw + f.esd;
    }

    const float limx = FRUSTUM_CLAMP * (0.5f * cam.W) / cam.fx;
    const float limy = FRUSTUM_CLAMP * (0.5f * cam.H) / cam.fy;
    const float iz = 1.0f / f.z;
    const float rx = f.xc * iz, ry = f.yc * iz;
    f.clamp_x = !(rx > -limx && rx < limx);
    f.clamp_y = !(ry > -limy && ry < limy);
    f.txz = fminf(fmaxf(rx, -limx), limx);
    f.tyz = fminf(fmaxf(ry, -limy), limy);
    f.J00 = cam.fx * iz;
    f.J02 = -cam.fx * f.txz * iz;
    f.J11 = cam.fy * iz;
    f.J12 = -cam.fy * f.tyz * iz;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        f.M[0][j] = f.J00 * R[0 * 3 + j] + f.J02 * R[2 * 3 + j];
        f.M[1][j] = f.J11 * R[1 * 3 + j] + f.J12 * R[2 * 3 + j];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f.u[k][0] = f.s[k] * (f.M[0][0] * f.r[0][k] + f.M[0][1] * f.r[1][k] + f.M[0][2] * f.r[2][k]);
        f.u[k][1] = f.s[k] * (f.M[1][0] * f.r[0][k] + f.M[1][1] * f.r[1][k] + f.M[1][2] * f.r[2][k]);
    }
    f.a0 = f.u[0][0] * f.u[0][0] + f.u[1][0] * f.u[1][0] + f.u[2][0] * f.u[2][0];
    f.c0 = f.u[0][1] * f.u[0][1] + f.u[1][1] * f.u[1][1] + f.u[2][1] * f.u[2][1];
    f.b = f.u[0][0] * f.u[0][1] + f.u[1][0] * f.u[1][1] + f.u[2][0] * f.u[2][1];
    const float x01 = f.u[0][0] * f.u[1][1] - f.u[0][1] * f.u[1][0];
    const float x02 = f.u[0][0] * f.u[2][1] - f.u[0][1] * f.u[2][0];
    const float x12 = f.u[1][0] * f.u[2][1] - f.u[1][1] * f.u[2][0];
    f.a = f.a0 + EWA_DILATION;
    f.c = f.c0 + EWA_DILATION;
    // det(a, b, c) = a c - b^2, evaluated as a sum of non-negative terms (Cauchy-Binet)
    f.det = x01 * x01 + x02 * x02 + x12 * x12 + EWA_DILATION * (f.a0 + f.c0) + EWA_DILATION * EWA_DILATION;
    f.mx = cam.fx * f.xc * iz + cam.cx;
    f.my = cam.fy * f.yc * iz + cam.cy;
    return f;
}

// Everything mgs_project writes for one Gaussian.
struct ProjOut {
    float4 r0, r1, r2;
    uint2 rect;
    uint32_t n_tiles;
};

__device__ __forceinline__ ProjOut project_gaussian(const GaussIn &in, const CamK &cam, float alpha_min) {
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
    ProjOut o;
    o.n_tiles = 0;
    o.rect = make_uint2(0u, 0u);
    if (vis) {
        const uint32_t tx0 = uint32_t(i0) / MGS_TILE, tx1 = uint32_t(i1) / MGS_TILE;
        const uint32_t ty0 = uint32_t(j0) / MGS_TILE, ty1 = uint32_t(j1) / MGS_TILE;
        if (!MGS_CHECK(tx0 <= tx1 && ty0 <= ty1 && tx1 < uint32_t(cam.tiles_x) && ty1 < uint32_t(cam.tiles_y),
                       BS_RECT_GRID))
            return o;
        o.n_tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        o.rect = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
    }
    const float ic = __builtin_amdgcn_rcpf(f.c);
    const float kA = -0.5f * LOG2E * (f.c * __builtin_amdgcn_rcpf(f.det));   // log2(alpha) = log2(o) + kA t^2 + kG dy^2
    const float beta = -f.b * ic;                    // t = dx + beta * dy
    const float kG = -0.5f * LOG2E * ic;
    o.r0 = make_float4(f.mx, f.my, log2f(fmaxf(f.o, 1e-30f)), f.w);
    o.r1 = make_float4(kA, beta, kG, f.front ? f.z : -1.0f);
    o.r2 = make_float4(f.col[0], f.col[1], f.col[2], f.o);
    return o;
}

__device__ __forceinline__ void store_proj(const ProjOut &o, int64_t k, float4 *__restrict__ splat,
                                           uint2 *__restrict__ rect_out, uint32_t *__restrict__ ntiles_out) {
    splat[3 * k + 0] = o.r0;
    splat[3 * k + 1] = o.r1;
    splat[3 * k + 2] = o.r2;
    rect_out[k] = o.rect;
    ntiles_out[k] = o.n_tiles;
}

}  // namespace mgs

// mgs_render_backward: gradients of the order-independent pass (Eq. 2-4).
//
// Nothing per fragment is stored by the forward pass: the blend gradients are
// recomputed per pixel-Gaussian pair from the per-pixel aux (F = N/D, D, T).
// For one pixel with upstream gradient g = dL/dC (D > 0):
//   G1 = g (1 - T) / D,  gF = G1 . F,  gT = g . (c_bg - F)
// and for one contributor (alpha, w, c):
//   u = G1 . c - gF                    (dL/d(alpha w))
//   dL/dc     += alpha w G1
//   dL/dw     += alpha u
//   dL/dalpha  = w u - gT T / (1 - alpha)   (0 where alpha was clamped)
// then alpha = o exp(-q/2) carries it to o and to the quadratic form.
//
// Deterministic reduction without float atomics:
//   1. bwd_blend: one workgroup per tile, one thread per listed Gaussian; the
//      thread walks the tile's pixels (per-pixel terms staged in LDS) and writes
//      its 10 partial sums to the pair's slot in Gaussian-major order
//      (slot = first[g] + index of the tile inside g's rectangle);
//   2. bwd_reduce: one wave per Gaussian sums its contiguous slots (fixed tree);
//   3. bwd_gauss: per-Gaussian chain rule to mean, log-scale, quaternion,
//      opacity logit, SH and (with the MLP) to phi and the opacity factor;
//   4. bwd_mlp: per-Gaussian MLP backward in float32 (straight through the
//      bfloat16 roundings of the forward) -> input gradients, and the per-Gaussian
//      vectors whose outer products give the weight gradients;
//   5. wgrad_partial / wgrad_sum: chunked outer-product sums, summed in chunk order.
#include "blend_math.h"
#include "proj_math.h"

namespace mgs {

constexpr int NPART = 10;   // mx, my, A, beta, gamma, o, w, r, g, b
constexpr int WG_CHUNK = 2048;
constexpr int MLP_VEC = 24 + 64 + 64 + 64 + 64 + 2;   // xb(22, padded), h1b, Fb, dH1, dF, (dphi, dm)
constexpr int OFF_XB = 0, OFF_H1 = 24, OFF_FB = 88, OFF_DH1 = 152, OFF_DF = 216, OFF_DHD = 280;

// ------------------------------------------------------------------ 1. blend backward
__global__ void __launch_bounds__(256)
bwd_blend_kernel(const float4 *__restrict__ splat, const uint2 *__restrict__ rect,
                 const uint32_t *__restrict__ first, const uint32_t *__restrict__ offs,
                 const uint32_t *__restrict__ gids, CamK cam, float bgr, float bgg, float bgb,
                 float log2_amin, float amax, const float *__restrict__ aux, const float *__restrict__ dimg,
                 float *__restrict__ part, uint64_t cap) {
    __shared__ float4 s_pa[256];   // G1 rgb, gF
    __shared__ float2 s_pb[256];   // gT, T
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    {
        const int t = threadIdx.x;
        const int px = tx * 16 + (t & 15), py = ty * 16 + (t >> 4);
        float4 pa = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 pb = make_float2(0.f, 1.f);
        if (px < cam.W && py < cam.H) {
            const size_t hw = size_t(cam.W) * cam.H, p = size_t(py) * cam.W + px;
            const float D = aux[3 * hw + p];
            if (D > 0.f) {
                const float T = aux[4 * hw + p];
                const float Fr = aux[p], Fg = aux[hw + p], Fb = aux[2 * hw + p];
                const float gr = dimg[p], gg = dimg[hw + p], gb = dimg[2 * hw + p];
                const float k = (1.0f - T) / D;
                pa = make_float4(gr * k, gg * k, gb * k, 0.f);
                pa.w = pa.x * Fr + pa.y * Fg + pa.z * Fb;
                pb = make_float2(gr * (bgr - Fr) + gg * (bgg - Fg) + gb * (bgb - Fb), T);
            }
        }
        s_pa[t] = pa;
        s_pb[t] = pb;
    }
    __syncthreads();
    const uint32_t start = offs[tile], end = offs[tile + 1];
    const float inv_k = -2.0f / LOG2E;      // kA = -(1/2) log2(e) A  ->  A = kA * inv_k
    for (uint32_t base = start; base < end; base += 256) {
        const uint32_t i = base + threadIdx.x;
        const bool active = i < end;
        float4 r0 = make_float4(0.f, 0.f, -1000.f, 0.f), r1 = make_float4(-1.f, 0.f, -1.f, 1.f),
               r2 = make_float4(0.f, 0.f, 0.f, 1.f);
        uint32_t g = 0, mask = 0;
        if (active) {
            g = gids[i];
            r0 = splat[3 * size_t(g) + 0];
            r1 = splat[3 * size_t(g) + 1];
            r2 = splat[3 * size_t(g) + 2];
            mask = quadrant_mask(r0, r1, tx, ty, log2_amin);
        }
        const float A = r1.x * inv_k, beta = r1.y, gam = r1.z * inv_k;
        const float inv_o = 1.0f / r2.w;
        float acc[NPART];
#pragma unroll
        for (int k = 0; k < NPART; ++k) acc[k] = 0.f;
        for (int q = 0; q < 4; ++q) {
            const bool mine = active && ((mask >> q) & 1u);
            if (__ballot(mine) == 0ull) continue;
            const int qx = (q & 1) * 8, qy = (q >> 1) * 8;
            for (int pp = 0; pp < 64; ++pp) {
                const int lx = qx + (pp & 7), ly = qy + (pp >> 3);
                const int k = ly * 16 + lx;
                const float4 pa = s_pa[k];
                const float2 pb = s_pb[k];
                const float dx = float(tx * 16 + lx) + 0.5f - r0.x;
                const float dy = float(ty * 16 + ly) + 0.5f - r0.y;
                const float t = fmaf(beta, dy, dx);
                const float e = fmaf(r1.x * t, t, fmaf(r1.z * dy, dy, r0.z));
                if (mine && e >= log2_amin) {
                    const float a = fast_exp2(e);
                    const float al = fminf(a, amax);
                    const float u = pa.x * r2.x + pa.y * r2.y + pa.z * r2.z - pa.w;
                    const float aw = al * r0.w;
                    acc[7] = fmaf(aw, pa.x, acc[7]);
                    acc[8] = fmaf(aw, pa.y, acc[8]);
                    acc[9] = fmaf(aw, pa.z, acc[9]);
                    acc[6] = fmaf(al, u, acc[6]);
                    const float dal = r0.w * u - pb.x * pb.y / (1.0f - al);
                    const float da = a > amax ? 0.0f : dal;
                    acc[5] = fmaf(da * a, inv_o, acc[5]);
                    const float dq = -0.5f * a * da;
                    acc[2] = fmaf(dq * t, t, acc[2]);
                    acc[4] = fmaf(dq * dy, dy, acc[4]);
                    const float s1 = 2.0f * dq * A * t;
                    acc[3] = fmaf(s1, dy, acc[3]);
                    acc[0] -= s1;
                    acc[1] -= fmaf(s1, beta, 2.0f * dq * gam * dy);
                }
            }
        }
        if (active) {
            const uint2 rc = rect[g];
            const uint64_t slot = pair_slot(first[g], unpack_rect(rc.x, rc.y), uint32_t(tx), uint32_t(ty));
            if (MGS_GUARD(slot < cap, BS_BWD_SLOT)) {
#pragma unroll
                for (int k = 0; k < NPART; ++k) part[k * cap + slot] = acc[k];
            }
        }
    }
}

// ------------------------------------------------------------------ 2. per-Gaussian reduce
__global__ void __launch_bounds__(256)
bwd_reduce_kernel(const uint32_t *__restrict__ first, const uint32_t *__restrict__ ntiles, int64_t n,
                  const float *__restrict__ part, uint64_t cap, const uint32_t *__restrict__ n_pairs,
                  float *__restrict__ gr) {
    const int64_t g = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (g >= n) return;
    // lists that overflowed their capacity in the forward carry no gradient
    const uint32_t nt = uint64_t(*n_pairs) <= cap ? ntiles[g] : 0u;
    const uint64_t e0 = first[g];
    float acc[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) acc[k] = 0.f;
    for (uint32_t j = l; j < nt; j += 64) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) acc[k] += part[k * cap + e0 + j];
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
        float v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[k] = v;
    }
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) gr[k * n + g] = acc[k];
    }
}

// ------------------------------------------------------------------ 3. per-Gaussian chain rule
__global__ void __launch_bounds__(256)
bwd_gauss_kernel(mgs_gaussians gs, CamK cam, const float *__restrict__ phi_in, const float *__restrict__ om_in,
                 const uint32_t *__restrict__ ntiles, const float *__restrict__ gr, mgs_gaussians_grad out,
                 float *__restrict__ gphi_out, float *__restrict__ gom_out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = gs.n;
    if (i >= n) return;
    float gmu[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, glogit = 0.f;
    float gsh[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) gsh[k] = 0.f;
    float gphi = 0.f, gom = 0.f;
    if (ntiles[i] > 0) {
        const GaussIn in = load_gauss(gs, i, phi_in, om_in);
        const GaussFwd f = gauss_forward(in, cam);
        const float gmx = gr[0 * n + i], gmy = gr[1 * n + i], gA = gr[2 * n + i], gbeta = gr[3 * n + i];
        const float ggam = gr[4 * n + i], go = gr[5 * n + i], gw = gr[6 * n + i];
        const float gc[3] = {gr[7 * n + i], gr[8 * n + i], gr[9 * n + i]};
        const float a = f.a, b = f.b, c = f.c, det = f.det;
        const float id2 = 1.0f / (det * det);
        // conic parameters (A = c/det, beta = -b/c, gamma = 1/c) -> covariance (a, b, c)
        const float ga = gA * (-c * c * id2);
        const float gb = gA * (2.0f * b * c * id2) - gbeta / c;
        const float gcc = gA * (-b * b * id2) + gbeta * b / (c * c) - ggam / (c * c);
        (void)a;
        // covariance -> u_k -> (s_k, M, rotation columns)
        float gM[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float gR[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float gs_[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float gux = 2.0f * ga * f.u[k][0] + gb * f.u[k][1];
            const float guy = 2.0f * gcc * f.u[k][1] + gb * f.u[k][0];
            const float mrx = f.M[0][0] * f.r[0][k] + f.M[0][1] * f.r[1][k] + f.M[0][2] * f.r[2][k];
            const float mry = f.M[1][0] * f.r[0][k] + f.M[1][1] * f.r[1][k] + f.M[1][2] * f.r[2][k];
            gs_[k] = gux * mrx + guy * mry;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                gM[0][j] += f.s[k] * gux * f.r[j][k];
                gM[1][j] += f.s[k] * guy * f.r[j][k];
                gR[j][k] = f.s[k] * (f.M[0][j] * gux + f.M[1][j] * guy);
            }
        }
        // M = J W
        const float *W = cam.R;
        const float gJ00 = gM[0][0] * W[0] + gM[0][1] * W[1] + gM[0][2] * W[2];
        const float gJ02 = gM[0][0] * W[6] + gM[0][1] * W[7] + gM[0][2] * W[8];
        const float gJ11 = gM[1][0] * W[3] + gM[1][1] * W[4] + gM[1][2] * W[5];
        const float gJ12 = gM[1][0] * W[6] + gM[1][1] * W[7] + gM[1][2] * W[8];
        const float z = f.z, iz = 1.0f / z, iz2 = iz * iz;
        float gx = 0.f, gy = 0.f, gz = 0.f;
        gz += -gJ00 * cam.fx * iz2 - gJ11 * cam.fy * iz2;
        gz += gJ02 * cam.fx * f.txz * iz2 + gJ12 * cam.fy * f.tyz * iz2;
        const float gtx = -gJ02 * cam.fx * iz, gty = -gJ12 * cam.fy * iz;
        if (!f.clamp_x) { gx += gtx * iz; gz -= gtx * f.xc * iz2; }
        if (!f.clamp_y) { gy += gty * iz; gz -= gty * f.yc * iz2; }
        // screen-space mean
        gx += gmx * cam.fx * iz;
        gz -= gmx * cam.fx * f.xc * iz2;
        gy += gmy * cam.fy * iz;
        gz -= gmy * cam.fy * f.yc * iz2;
        // weight w = phi^2 + phi / z^2 + exp(s_max / z)
        gphi = gw * (2.0f * f.phi + iz2);
        gz += gw * (-2.0f * f.phi * iz2 * iz - f.smax * iz2 * f.esd);
        gs_[f.kmax] += gw * f.esd * iz;
        // effective opacity o = sigmoid(logit) * m
        glogit = go * in.om * f.sig * (1.0f - f.sig);
        gom = go * f.sig;
        // colour
        float gP[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            if (f.cpre[ch] > 0.0f) {
                const float g = gc[ch];
                gsh[ch] = g * SH_C0;
                gsh[3 + ch] = -g * SH_C1 * f.P[1];
                gsh[6 + ch] = g * SH_C1 * f.P[2];
                gsh[9 + ch] = -g * SH_C1 * f.P[0];
                gP[0] -= g * SH_C1 * in.sh[9 + ch];
                gP[1] -= g * SH_C1 * in.sh[3 + ch];
                gP[2] += g * SH_C1 * in.sh[6 + ch];
            }
        }
        // camera space -> world mean, plus the view-direction path
        const float PdotG = f.P[0] * gP[0] + f.P[1] * gP[1] + f.P[2] * gP[2];
        const float ivl = 1.0f / f.vlen;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gmu[j] = W[0 * 3 + j] * gx + W[1 * 3 + j] * gy + W[2 * 3 + j] * gz + (gP[j] - f.P[j] * PdotG) * ivl;
#pragma unroll
        for (int k = 0; k < 3; ++k) gls[k] = gs_[k] * f.s[k];
        // rotation matrix -> unit quaternion -> raw quaternion
        const float qw = f.qn[0], qx = f.qn[1], qy = f.qn[2], qz = f.qn[3];
        float gqn[4];
        gqn[0] = 2.f * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] + qx * gR[2][1]);
        gqn[1] = 2.f * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2.f * qx * gR[1][1] - qw * gR[1][2] +
                        qz * gR[2][0] + qw * gR[2][1] - 2.f * qx * gR[2][2]);
        gqn[2] = 2.f * (-2.f * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] -
                        qw * gR[2][0] + qz * gR[2][1] - 2.f * qy * gR[2][2]);
        gqn[3] = 2.f * (-2.f * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] - 2.f * qz * gR[1][1] +
                        qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
        const float qd = qw * gqn[0] + qx * gqn[1] + qy * gqn[2] + qz * gqn[3];
        const float iq = 1.0f / f.qnorm;
#pragma unroll
        for (int k = 0; k < 4; ++k) gq[k] = (gqn[k] - f.qn[k] * qd) * iq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out.mean[k * n + i] = gmu[k];
        out.log_scale[k * n + i] = gls[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out.quat[k * n + i] = gq[k];
    out.opacity_logit[i] = glogit;
#pragma unroll
    for (int k = 0; k < 12; ++k) out.sh[k * n + i] = gsh[k];
    if (gphi_out) {
        gphi_out[i] = gphi;
        gom_out[i] = gom;
    }
}

// ------------------------------------------------------------------ 4. MLP backward
__global__ void __launch_bounds__(128)
bwd_mlp_kernel(mgs_gaussians gs, CamK cam, const float *__restrict__ prm, const float *__restrict__ gphi_in,
               const float *__restrict__ gom_in, mgs_gaussians_grad out, float *__restrict__ vec) {
    __shared__ float sW1[64 * 22];
    __shared__ float sW2[64 * 64];
    __shared__ float sB1[64], sB2[64], sWp[64], sWo[64];
    for (int e = threadIdx.x; e < 64 * 22; e += blockDim.x) sW1[e] = bf16_round(prm[MGS_MLP_OFF_W1 + e]);
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) sW2[e] = bf16_round(prm[MGS_MLP_OFF_W2 + e]);
    for (int e = threadIdx.x; e < 64; e += blockDim.x) {
        sB1[e] = prm[MGS_MLP_OFF_B1 + e];
        sB2[e] = prm[MGS_MLP_OFF_B2 + e];
        sWp[e] = bf16_round(prm[MGS_MLP_OFF_WPHI + e]);
        sWo[e] = bf16_round(prm[MGS_MLP_OFF_WO + e]);
    }
    __syncthreads();
    const float bphi = prm[MGS_MLP_OFF_BPHI], bo = prm[MGS_MLP_OFF_BO];
    const int64_t n = gs.n;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *V = vec + size_t(i) * MLP_VEC;
    // features, rounded as the forward rounds them
    const float mx = gs.mean[i], my = gs.mean[n + i], mz = gs.mean[2 * n + i];
    const float v0 = mx - cam.campos[0], v1 = my - cam.campos[1], v2 = mz - cam.campos[2];
    const float vl = sqrtf(v0 * v0 + v1 * v1 + v2 * v2), ivl = 1.0f / vl;
    const float P[3] = {v0 * ivl, v1 * ivl, v2 * ivl};
    float q[4], s[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = gs.quat[k * n + i];
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float iqn = qn > 0.f ? 1.0f / qn : 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] *= iqn;
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = expf(gs.log_scale[k * n + i]);
    float x[22];
#pragma unroll
    for (int k = 0; k < 3; ++k) { x[k] = P[k]; x[3 + k] = s[k]; }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[6 + k] = q[k];
#pragma unroll
    for (int k = 0; k < 12; ++k) x[10 + k] = gs.sh[k * n + i];
#pragma unroll
    for (int k = 0; k < 22; ++k) { x[k] = bf16_round(x[k]); V[OFF_XB + k] = x[k]; }
    V[OFF_XB + 22] = 0.f;
    V[OFF_XB + 23] = 0.f;
    // forward, layer 1
    float h[64];
    uint64_t m1 = 0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        float acc = sB1[j];
#pragma unroll
        for (int k = 0; k < 22; ++k) acc = fmaf(sW1[j * 22 + k], x[k], acc);
        m1 |= uint64_t(acc > 0.f) << j;
        h[j] = bf16_round(fmaxf(acc, 0.f));
        V[OFF_H1 + j] = h[j];
    }
    // forward, layer 2 and heads
    uint64_t m2 = 0;
    float php = bphi, mop = bo;
#pragma unroll 4
    for (int j = 0; j < 64; ++j) {
        float acc = sB2[j];
#pragma unroll
        for (int k = 0; k < 64; ++k) acc = fmaf(sW2[j * 64 + k], h[k], acc);
        m2 |= uint64_t(acc > 0.f) << j;
        const float fb = bf16_round(fmaxf(acc, 0.f));
        V[OFF_FB + j] = fb;
        php = fmaf(sWp[j], fb, php);
        mop = fmaf(sWo[j], fb, mop);
    }
    const float m = 1.0f / (1.0f + expf(-mop));
    const float dphi = php > 0.f ? gphi_in[i] : 0.f;
    const float dmo = gom_in[i] * m * (1.0f - m);
    V[OFF_DHD + 0] = dphi;
    V[OFF_DHD + 1] = dmo;
    // backward, layer 2 (h is reused as dL/dh1)
#pragma unroll
    for (int k = 0; k < 64; ++k) h[k] = 0.f;
#pragma unroll 4
    for (int j = 0; j < 64; ++j) {
        const float dF = ((m2 >> j) & 1ull) ? fmaf(dphi, sWp[j], dmo * sWo[j]) : 0.f;
        V[OFF_DF + j] = dF;
#pragma unroll
        for (int k = 0; k < 64; ++k) h[k] = fmaf(sW2[j * 64 + k], dF, h[k]);
    }
    // backward, layer 1
    float dx[22];
#pragma unroll
    for (int k = 0; k < 22; ++k) dx[k] = 0.f;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const float d = ((m1 >> j) & 1ull) ? h[j] : 0.f;
        V[OFF_DH1 + j] = d;
#pragma unroll
        for (int k = 0; k < 22; ++k) dx[k] = fmaf(sW1[j * 22 + k], d, dx[k]);
    }
    // input gradients: P -> mean, s -> log_scale, q -> raw quaternion, Y -> sh
    const float pd = P[0] * dx[0] + P[1] * dx[1] + P[2] * dx[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out.mean[k * n + i] += (dx[k] - P[k] * pd) * ivl;
        out.log_scale[k * n + i] += dx[3 + k] * s[k];
    }
    const float qd = q[0] * dx[6] + q[1] * dx[7] + q[2] * dx[8] + q[3] * dx[9];
#pragma unroll
    for (int k = 0; k < 4; ++k) out.quat[k * n + i] += (dx[6 + k] - q[k] * qd) * iqn;
#pragma unroll
    for (int k = 0; k < 12; ++k) out.sh[k * n + i] += dx[10 + k];
}

// ------------------------------------------------------------------ 5. weight gradients
// Outer-product sums: out[r][c] = sum_g L[g][r] * R[g][c] for c < nc, and the
// bias column out[r][nc] = sum_g L[g][r].  Partial sums per chunk of WG_CHUNK
// Gaussians; the chunks are added in order by wgrad_sum_kernel.
struct WJob {
    int loff, roff, nr, nc, out_off;   // vector offsets in the per-Gaussian record; result layout
};

__global__ void __launch_bounds__(256)
wgrad_partial_kernel(const float *__restrict__ vec, int64_t n, WJob job, float *__restrict__ partial) {
    __shared__ float sL[64][65];
    __shared__ float sR[64][65];
    const int64_t g0 = int64_t(blockIdx.x) * WG_CHUNK;
    const int nout = job.nr * (job.nc + 1);
    float acc[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) acc[k] = 0.f;
    for (int64_t sub = 0; sub < WG_CHUNK; sub += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e / 64, c = e % 64;
            const int64_t g = g0 + sub + r;
            const bool ok = g < n;
            sL[r][c] = (ok && c < job.nr) ? vec[size_t(g) * MLP_VEC + job.loff + c] : 0.f;
            sR[r][c] = (ok && c < job.nc) ? vec[size_t(g) * MLP_VEC + job.roff + c] : 0.f;
        }
        if (threadIdx.x < 64) sR[threadIdx.x][64] = (g0 + sub + threadIdx.x < n) ? 1.f : 0.f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 17; ++k) {
            const int o = threadIdx.x + k * 256;
            if (o < nout) {
                const int r = o / (job.nc + 1), c = o % (job.nc + 1);
                const int cc = c == job.nc ? 64 : c;
                float a = acc[k];
                for (int j = 0; j < 64; ++j) a = fmaf(sL[j][r], sR[j][cc], a);
                acc[k] = a;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 17; ++k) {
        const int o = threadIdx.x + k * 256;
        if (o < nout) partial[size_t(blockIdx.x) * nout + o] = acc[k];
    }
}

__global__ void __launch_bounds__(256)
wgrad_sum_kernel(const float *__restrict__ partial, int nchunks, WJob job, float *__restrict__ dmlp) {
    const int nout = job.nr * (job.nc + 1);
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partial[size_t(c) * nout + o];
    const int r = o / (job.nc + 1), c = o % (job.nc + 1);
    // job.out_off encodes where weights / biases go (see launch site)
    if (job.out_off == 0) {           // W1 [64][22] + b1
        if (c < 22) dmlp[MGS_MLP_OFF_W1 + r * 22 + c] = s; else dmlp[MGS_MLP_OFF_B1 + r] = s;
    } else if (job.out_off == 1) {    // W2 [64][64] + b2
        if (c < 64) dmlp[MGS_MLP_OFF_W2 + r * 64 + c] = s; else dmlp[MGS_MLP_OFF_B2 + r] = s;
    } else {                          // heads: row 0 phi, row 1 opacity
        if (r == 0) { if (c < 64) dmlp[MGS_MLP_OFF_WPHI + c] = s; else dmlp[MGS_MLP_OFF_BPHI] = s; }
        else        { if (c < 64) dmlp[MGS_MLP_OFF_WO + c] = s; else dmlp[MGS_MLP_OFF_BO] = s; }
    }
}

__global__ void fill_zero_kernel(float *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------ host side
struct BwdLayout {
    size_t first, scan, part, gr, gphi, gom, vec, wpart, total;
    int nchunks;
};

inline BwdLayout bwd_layout(int64_t n, uint64_t cap, bool mlp) {
    BwdLayout L;
    const size_t nn = size_t(n > 0 ? n : 1), cc = size_t(cap > 0 ? cap : 1);
    L.nchunks = int((nn + WG_CHUNK - 1) / WG_CHUNK);
    size_t o = 0;
    L.first = o; o = align_up(o + nn * 4, 256);
    L.scan = o;  o = align_up(o + scan_tmp_elems(n) * 8 + 16, 256);
    L.part = o;  o = align_up(o + cc * NPART * 4, 256);
    L.gr = o;    o = align_up(o + nn * NPART * 4, 256);
    L.gphi = o;  o = align_up(o + (mlp ? nn * 4 : 0), 256);
    L.gom = o;   o = align_up(o + (mlp ? nn * 4 : 0), 256);
    L.vec = o;   o = align_up(o + (mlp ? nn * MLP_VEC * 4 : 0), 256);
    L.wpart = o; o = align_up(o + (mlp ? size_t(L.nchunks) * 64 * 65 * 4 : 0), 256);
    L.total = o;
    return L;
}

}  // namespace mgs

extern "C" int mgs_render_backward_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity,
                                             int with_mlp, size_t *bytes) {
    MGS_REQUIRE(bytes && n >= 0 && tiles_x > 0 && tiles_y > 0, "bad arguments");
    *bytes = mgs::bwd_layout(n, capacity, with_mlp != 0).total;
    return MGS_OK;
}

extern "C" int mgs_render_backward(const mgs_gaussians *g, const mgs_camera *cam, const float *mlp_params,
                                   const float *phi, const float *omod, const mgs_projected *proj,
                                   const uint32_t *tile_offsets, const uint32_t *gids, uint64_t capacity,
                                   const float *aux, const float *dL_dimage, const float bg[3], float alpha_min,
                                   float alpha_max, void *ws, size_t ws_bytes, mgs_gaussians_grad *out,
                                   float *dmlp, void *stream) {
    MGS_TRACE("mgs_render_backward");
    using namespace mgs;
    int rc;
    if ((rc = check_gaussians(g)) != MGS_OK) return rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    if ((rc = check_projected(proj, g->n)) != MGS_OK) return rc;
    MGS_REQUIRE(out && bg && tile_offsets && aux && dL_dimage, "a required pointer is NULL");
    MGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f && alpha_max > alpha_min && alpha_max < 1.f, "bad alpha range");
    const bool mlp = mlp_params != nullptr;
    MGS_REQUIRE(!mlp || (phi && omod && dmlp), "the MLP path needs phi, omod and dmlp");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32), "capacity too large");
    const int64_t n = g->n;
    const BwdLayout L = bwd_layout(n, capacity, mlp);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    if (n > 0) MGS_REQUIRE(out->mean && out->log_scale && out->quat && out->opacity_logit && out->sh,
                           "a gradient pointer is NULL");
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(ws);
    uint32_t *first = reinterpret_cast<uint32_t *>(w + L.first);
    uint64_t *stmp = reinterpret_cast<uint64_t *>(w + L.scan);
    uint32_t *ptot = reinterpret_cast<uint32_t *>(w + L.scan + scan_tmp_elems(n) * 8);
    float *part = reinterpret_cast<float *>(w + L.part);
    float *gr = reinterpret_cast<float *>(w + L.gr);
    float *gphi = mlp ? reinterpret_cast<float *>(w + L.gphi) : nullptr;
    float *gom = mlp ? reinterpret_cast<float *>(w + L.gom) : nullptr;
    float *vec = reinterpret_cast<float *>(w + L.vec);
    float *wpart = reinterpret_cast<float *>(w + L.wpart);
    const CamK k = make_camk(cam);
    if (n == 0) {
        if (mlp) {
            hipLaunchKernelGGL(fill_zero_kernel, dim3((MGS_MLP_PARAMS + 255) / 256), dim3(256), 0, s, dmlp,
                               int(MGS_MLP_PARAMS));
            MGS_LAUNCH_CHECK("fill_zero_kernel");
        }
        return MGS_OK;
    }
    if ((rc = scan_exclusive(proj->n_tiles, first, n, stmp, ptot, s)) != MGS_OK) return rc;
    const unsigned T = unsigned(k.tiles_x) * unsigned(k.tiles_y);
    hipLaunchKernelGGL(bwd_blend_kernel, dim3(T), dim3(256), 0, s, reinterpret_cast<const float4 *>(proj->splat),
                       reinterpret_cast<const uint2 *>(proj->rect), first, tile_offsets, gids, k, bg[0], bg[1], bg[2],
                       log2f(alpha_min), alpha_max, aux, dL_dimage, part, uint64_t(capacity > 0 ? capacity : 1));
    MGS_LAUNCH_CHECK("bwd_blend_kernel");
    hipLaunchKernelGGL(bwd_reduce_kernel, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, first, proj->n_tiles, n,
                       part, uint64_t(capacity > 0 ? capacity : 1), ptot, gr);
    MGS_LAUNCH_CHECK("bwd_reduce_kernel");
    hipLaunchKernelGGL(bwd_gauss_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, *g, k, phi, omod,
                       proj->n_tiles, gr, *out, gphi, gom);
    MGS_LAUNCH_CHECK("bwd_gauss_kernel");
    if (mlp) {
        hipLaunchKernelGGL(bwd_mlp_kernel, dim3(unsigned((n + 127) / 128)), dim3(128), 0, s, *g, k, mlp_params, gphi,
                           gom, *out, vec);
        MGS_LAUNCH_CHECK("bwd_mlp_kernel");
        const WJob jobs[3] = {{OFF_DH1, OFF_XB, 64, 22, 0}, {OFF_DF, OFF_H1, 64, 64, 1}, {OFF_DHD, OFF_FB, 2, 64, 2}};
        for (int j = 0; j < 3; ++j) {
            hipLaunchKernelGGL(wgrad_partial_kernel, dim3(unsigned(L.nchunks)), dim3(256), 0, s, vec, n, jobs[j], wpart);
            MGS_LAUNCH_CHECK("wgrad_partial_kernel");
            const int nout = jobs[j].nr * (jobs[j].nc + 1);
            hipLaunchKernelGGL(wgrad_sum_kernel, dim3(unsigned((nout + 255) / 256)), dim3(256), 0, s, wpart,
                               L.nchunks, jobs[j], dmlp);
            MGS_LAUNCH_CHECK("wgrad_sum_kernel");
        }
    }
    return MGS_OK;
}

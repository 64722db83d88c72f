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
//   1. bwd_plan: the tile lists are cut into work items of at most BWD_CHUNK list
//      positions (a chunk count per tile, an exclusive scan, the items written);
//   2. bwd_blend: one workgroup per item, one lane per listed Gaussian.  Each wave
//      lists its Gaussians' (Gaussian, quadrant) entries for the tile quadrants they
//      reach and evaluates them 64 at a time (a lane walks one quadrant's pixels, the
//      per-pixel terms staged in LDS); the entries' sums are gathered, in entry order,
//      by the lane that owns the Gaussian, which writes its 10 partial sums as one
//      record to the pair's slot in Gaussian-major order (slot = first[g] + index of
//      the tile inside g's rectangle);
//   3. bwd_reduce: 16 lanes per Gaussian sum its contiguous slots (fixed tree);
//   4. bwd_gauss: per-Gaussian chain rule to mean, log-scale, quaternion,
//      opacity logit, SH and (with the MLP) to phi and the opacity factor;
//   5. bwd_mlp: the MLP backward in float32 (straight through the bfloat16
//      roundings of the forward) on matrix instructions, 64 Gaussians per workgroup
//      step: input gradients, and per-workgroup sums of the weight gradients;
//   6. mlp_wsum: the workgroups' weight-gradient sums added in workgroup order.
#include "blend_math.h"
#include "proj_math.h"

namespace mgs {

constexpr int NPART = 10;        // mx, my, A, beta, gamma, o, w, r, g, b
constexpr int PART_STRIDE = 12;  // floats per pair record: the 10 sums and 2 zeros (48-byte records)
constexpr uint32_t BWD_CHUNK = 256;   // list positions per blend work item (one per thread)
constexpr unsigned BWD_GRID_MAX = 1u << 20;   // blend workgroups; more items are walked in a grid stride

// Work items of the blend backward for T tiles and at most `capacity` pairs: sum over tiles of
// ceil(L_t / BWD_CHUNK) <= capacity / BWD_CHUNK + T.
inline uint64_t bwd_max_items(uint64_t T, uint64_t capacity) { return T + capacity / BWD_CHUNK + 1; }

// ------------------------------------------------------------------ 1. work items
// Chunks per tile; none at all when the forward's lists overflowed their capacity (the lists
// and offsets were not built: nothing is read and every gradient is zero).
__global__ void __launch_bounds__(256)
bwd_chunks_kernel(const uint32_t *__restrict__ offs, uint32_t T, const uint32_t *__restrict__ n_pairs,
                  uint64_t cap, uint32_t *__restrict__ chunks) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t >= T) return;
    uint32_t c = 0;
    if (uint64_t(*n_pairs) <= cap) {
        const uint32_t s = offs[t], e = offs[t + 1];
        if (MGS_CHECK(s <= e && e <= *n_pairs, BS_LIST_READ)) c = ceil_div(e - s, BWD_CHUNK);
    }
    chunks[t] = c;
}

// Item j of tile t (j < chunks[t]) = (t, first list position of its chunk), at cbase[t] + j.
__global__ void __launch_bounds__(256)
bwd_items_kernel(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ chunks,
                 const uint32_t *__restrict__ cbase, uint32_t T, uint64_t max_items, uint2 *__restrict__ items) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t >= T) return;
    const uint32_t c = chunks[t], b = cbase[t], s = offs[t];
    for (uint32_t j = 0; j < c; ++j)
        if (MGS_CHECK(uint64_t(b) + j < max_items, BS_BWD_ITEM)) items[b + j] = make_uint2(t, s + j * BWD_CHUNK);
}

// ------------------------------------------------------------------ 2. blend backward
// Sums over the pixels of one (Gaussian, quadrant) entry.  With a = alpha before the clamp and
// ada = a dL/dalpha (0 where alpha was clamped or below alpha_min):
//   sc = sum alpha G1 (times w at the end), sw = sum alpha u, so = sum ada,
//   and the quadratic-form sums with t = dx + beta dy:
//   st = sum ada t, stt = sum ada t^2, sty = sum ada t dy, sy = sum ada dy, syy = sum ada dy^2
// (each -2 times the sum of the corresponding dq = d alpha / d(quadratic form) terms).
constexpr int BWD_SUMS = 10;
struct BwdSums {
    float v[BWD_SUMS] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
};
enum { S_CR, S_CG, S_CB, S_W, S_O, S_T, S_TT, S_TY, S_Y, S_YY };

// LDS strides of the per-pixel terms per quadrant (float4 and float units): the four quadrants
// of one read fall in different banks.
constexpr int QS4 = 65, QS1 = 68;

// One entry: the Gaussian's pixels in quadrant (xb, yb) of the tile, row by row.  The exponent
// is the forward's (same polynomial about the tile centre, same pixel offsets X = c + xb,
// Y = row + yb), so the alpha_min cut and alpha are bit-identical to the forward's.  Within a row
// dy is fixed and t = tY + X, so a pixel adds ada, ada c and ada c^2 (c the column, a literal)
// to row sums combined once per row.
template <bool CLAMP>
__device__ __forceinline__ void bwd_entry(const float4 &qa, const float4 &qb, float beta, float t0, float v0, float cr,
                                          float cg, float cb, float wgt, bool act0, float xb, float yb,
                                          float log2_amin, float amax, const float4 *__restrict__ pa_q,
                                          const float *__restrict__ pb_q, BwdSums &S) {
    for (int row = 0; row < 8; ++row) {
        const float Y = float(row) + yb;
        const float P = fmaf(fmaf(qb.y, Y, qa.z), Y, qa.x);
        const float R = fmaf(qb.x, Y, qa.y);
        const float4 *pa_r = pa_q + row * 8;
        const float *pb_r = pb_q + row * 8;
        float r0 = 0.f, rx = 0.f, rxx = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float X = float(c) + xb;
            const float e = fmaf(fmaf(qa.w, X, R), X, P);
            const float4 pa = pa_r[c];
            const float pb = pb_r[c];
            const float a = (act0 && e >= log2_amin) ? fast_exp2(e) : 0.0f;
            const float al = CLAMP ? fminf(a, amax) : a;
            const float u = fmaf(pa.z, cb, fmaf(pa.y, cg, fmaf(pa.x, cr, pa.w)));
            S.v[S_CR] = fmaf(al, pa.x, S.v[S_CR]);
            S.v[S_CG] = fmaf(al, pa.y, S.v[S_CG]);
            S.v[S_CB] = fmaf(al, pa.z, S.v[S_CB]);
            S.v[S_W] = fmaf(al, u, S.v[S_W]);
            const float dal = fmaf(wgt, u, -pb * __builtin_amdgcn_rcpf(1.0f - al));
            const float ada = (CLAMP && a > amax) ? 0.0f : a * dal;
            r0 += ada;
            rx = fmaf(ada, float(c), rx);
            rxx = fmaf(ada, float(c * c), rxx);
        }
        const float tc = fmaf(beta, Y, t0) + xb, dyr = v0 + Y;   // t at column 0 of the row
        const float s1 = fmaf(tc, r0, rx);                         // sum ada t over the row
        S.v[S_O] += r0;
        S.v[S_T] += s1;
        S.v[S_TT] += fmaf(tc, fmaf(tc, r0, 2.0f * rx), rxx);     // sum ada (tc + c)^2
        S.v[S_TY] = fmaf(s1, dyr, S.v[S_TY]);
        S.v[S_Y] = fmaf(r0, dyr, S.v[S_Y]);
        S.v[S_YY] = fmaf(r0 * dyr, dyr, S.v[S_YY]);
    }
}

__global__ void __launch_bounds__(256)
bwd_blend_kernel(const float4 *__restrict__ splat, const uint2 *__restrict__ rect,
                 const uint32_t *__restrict__ first, const uint32_t *__restrict__ offs,
                 const uint32_t *__restrict__ gids, const uint2 *__restrict__ items,
                 const uint32_t *__restrict__ n_items, uint64_t max_items, const uint32_t *__restrict__ n_pairs,
                 CamK cam, float bgr, float bgg, float bgb, float log2_amin, float amax,
                 const float *__restrict__ aux, const float *__restrict__ dimg, float *__restrict__ part,
                 uint64_t cap) {
    // per pixel of quadrant q, row r, column c (at q * QS + 8 r + c): (G1 rgb, -gF) and gT T
    __shared__ float4 s_pa[4 * QS4];
    __shared__ float s_pb[4 * QS1];
    // per wave: its Gaussians' (lane, quadrant) entries, Gaussian-major (lane << 2 | quadrant)
    __shared__ uint8_t s_ent[4][4 * 64];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const float inv_k = -2.0f / LOG2E;      // kA = -(1/2) log2(e) A  ->  A = kA * inv_k
    const float log2_amax_safe = __log2f(amax) - OIT_CLAMP_MARGIN;
    const uint32_t ni = *n_items;
    for (uint32_t k = blockIdx.x; k < ni; k += gridDim.x) {             // block-uniform
        if (!MGS_CHECK(k < max_items, BS_BWD_ITEM)) return;
        const uint2 it = items[k];
        const uint32_t tile = it.x, start = it.y, tend = offs[tile + 1];
        const uint32_t end = tend - start > BWD_CHUNK ? start + BWD_CHUNK : tend;
        if (!MGS_CHECK(start < end && end <= *n_pairs, BS_LIST_READ)) return;
        const int tx = int(tile % uint32_t(cam.tiles_x)), ty = int(tile / uint32_t(cam.tiles_x));
        __syncthreads();                    // the previous item's LDS reads are done
        {
            const int q = threadIdx.x >> 6, row = (threadIdx.x >> 3) & 7, cl = threadIdx.x & 7;
            const int px = tx * 16 + (q & 1) * 8 + cl, py = ty * 16 + (q >> 1) * 8 + row;
            float4 pa = make_float4(0.f, 0.f, 0.f, 0.f);
            float pb = 0.f;
            if (px < cam.W && py < cam.H) {
                const size_t hw = size_t(cam.W) * cam.H, p = size_t(py) * cam.W + px;
                const float D = aux[3 * hw + p];
                if (D > 0.f) {
                    const float T = aux[4 * hw + p];
                    const float Fr = aux[p], Fg = aux[hw + p], Fb = aux[2 * hw + p];
                    const float gr = dimg[p], gg = dimg[hw + p], gb = dimg[2 * hw + p];
                    const float kk = (1.0f - T) / D;
                    pa = make_float4(gr * kk, gg * kk, gb * kk, 0.f);
                    pa.w = -(pa.x * Fr + pa.y * Fg + pa.z * Fb);
                    pb = (gr * (bgr - Fr) + gg * (bgg - Fg) + gb * (bgb - Fb)) * T;
                }
            }
            s_pa[q * QS4 + row * 8 + cl] = pa;
            s_pb[q * QS1 + row * 8 + cl] = pb;
        }
        // the lane's list position: culling; a Gaussian that reaches no quadrant has a zero record
        const uint32_t i = start + threadIdx.x;
        uint32_t g = 0, mask = 0;
        if (i < end) {
            g = gids[i];
            mask = quadrant_mask(splat[3 * size_t(g) + 0], splat[3 * size_t(g) + 1], tx, ty, log2_amin);
            if (mask == 0u) {
                const uint2 rc = rect[g];
                const uint64_t slot = pair_slot(first[g], unpack_rect(rc.x, rc.y), uint32_t(tx), uint32_t(ty));
                if (MGS_GUARD(slot < cap, BS_BWD_SLOT)) {
                    float4 *o = reinterpret_cast<float4 *>(part + slot * PART_STRIDE);
                    o[0] = o[1] = o[2] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
        }
        // the wave's entries: lane l's quadrants at base .. base + popc(mask) - 1
        const uint32_t cnt = uint32_t(__popc(mask));
        uint32_t inc = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= uint32_t(o)) inc += y;
        }
        const uint32_t base = inc - cnt;
        const uint32_t E = __shfl(inc, 63, 64);
        {
            uint32_t m = mask, e = base;
            while (m) {
                const uint32_t q = uint32_t(__builtin_ctz(m));
                s_ent[w][e++] = uint8_t((lane << 2) | q);
                m &= m - 1u;
            }
        }
        __syncthreads();                    // pixel terms and entries are visible
        BwdSums acc;                        // the lane's own Gaussian
        const float tcx = float(tx * 16) + 8.0f, tcy = float(ty * 16) + 8.0f;
        for (uint32_t c0 = 0; c0 < E; c0 += 64) {                          // wave-uniform
            const uint32_t e = c0 + lane;
            const bool have = e < E;
            const uint32_t ent = have ? s_ent[w][e] : 0u;
            const int src = int(ent >> 2), q = int(ent & 3u);
            const uint32_t ge = uint32_t(__shfl(int(g), src, 64));
            float4 r0 = make_float4(0.f, 0.f, -1000.f, 0.f), r1 = make_float4(-1.f, 0.f, -1.f, 1.f),
                   r2 = make_float4(0.f, 0.f, 0.f, 1.f);
            if (have) {
                r0 = splat[3 * size_t(ge) + 0];
                r1 = splat[3 * size_t(ge) + 1];
                r2 = splat[3 * size_t(ge) + 2];
            }
            float4 qa, qb = make_float4(0.f, 0.f, 0.f, 0.f);
            quad_poly(r0, r1, tcx, tcy, qa, qb);
            const float beta = r1.y;
            const float v0 = tcy - r0.y, t0 = fmaf(beta, v0, tcx - r0.x);
            const float xb = (q & 1) ? 0.5f : -7.5f, yb = (q >> 1) ? 0.5f : -7.5f;
            BwdSums S;
            const float4 *pa_q = s_pa + q * QS4;
            const float *pb_q = s_pb + q * QS1;
            if (__ballot(have && r0.z > log2_amax_safe) != 0ull)
                bwd_entry<true>(qa, qb, beta, t0, v0, r2.x, r2.y, r2.z, r0.w, have, xb, yb, log2_amin, amax, pa_q,
                                pb_q, S);
            else
                bwd_entry<false>(qa, qb, beta, t0, v0, r2.x, r2.y, r2.z, r0.w, have, xb, yb, log2_amin, amax, pa_q,
                                 pb_q, S);
            // each lane adds its Gaussian's entries of this chunk, in entry order
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t ej = base + j;
                const bool mine = j < cnt && ej >= c0 && ej < c0 + 64u;
                const int from = int(ej - c0) & 63;
#pragma unroll
                for (int v = 0; v < BWD_SUMS; ++v) {
                    const float x = __shfl(S.v[v], from, 64);
                    if (mine) acc.v[v] += x;
                }
            }
        }
        if (mask != 0u) {
            const float4 r0 = splat[3 * size_t(g) + 0], r1 = splat[3 * size_t(g) + 1];
            const float r2w = splat[3 * size_t(g) + 2].w;
            const float A = r1.x * inv_k, gam = r1.z * inv_k, beta = r1.y, wgt = r0.w;
            const uint2 rc = rect[g];
            const uint64_t slot = pair_slot(first[g], unpack_rect(rc.x, rc.y), uint32_t(tx), uint32_t(ty));
            if (MGS_GUARD(slot < cap, BS_BWD_SLOT)) {
                // dq = -ada / 2: dL/dA = sum dq t^2, dL/dgamma = sum dq dy^2, dL/dbeta = 2 A sum dq t dy,
                // dL/dmx = -2 A sum dq t, dL/dmy = -2 A beta sum dq t - 2 gamma sum dq dy
                const float *v = acc.v;
                float4 *o = reinterpret_cast<float4 *>(part + slot * PART_STRIDE);
                o[0] = make_float4(A * v[S_T], fmaf(A * beta, v[S_T], gam * v[S_Y]), -0.5f * v[S_TT], -A * v[S_TY]);
                o[1] = make_float4(-0.5f * v[S_YY], v[S_O] / r2w, v[S_W], wgt * v[S_CR]);
                o[2] = make_float4(wgt * v[S_CG], wgt * v[S_CB], 0.f, 0.f);
            }
        }
    }
}

// ------------------------------------------------------------------ 3. per-Gaussian reduce
// 16 lanes per Gaussian: lane j sums slots j, j + 16, ... of the Gaussian, then a fixed
// butterfly over the 16 lanes.
__global__ void __launch_bounds__(256)
bwd_reduce_kernel(const uint32_t *__restrict__ first, const uint32_t *__restrict__ ntiles, int64_t n,
                  const float *__restrict__ part, uint64_t cap, const uint32_t *__restrict__ n_pairs,
                  float *__restrict__ gr) {
    const int64_t g = int64_t(blockIdx.x) * 16 + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    const bool ok = g < n;
    // lists that overflowed their capacity in the forward carry no gradient
    const uint32_t nt = (ok && uint64_t(*n_pairs) <= cap) ? ntiles[g] : 0u;
    const uint64_t e0 = ok ? first[g] : 0u;
    float acc[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) acc[k] = 0.f;
    for (uint32_t j = l; j < nt; j += 16) {
        const float4 *rec = reinterpret_cast<const float4 *>(part + (e0 + j) * PART_STRIDE);
        const float4 a = rec[0], b = rec[1];
        const float2 c = *reinterpret_cast<const float2 *>(rec + 2);
        acc[0] += a.x; acc[1] += a.y; acc[2] += a.z; acc[3] += a.w;
        acc[4] += b.x; acc[5] += b.y; acc[6] += b.z; acc[7] += b.w;
        acc[8] += c.x; acc[9] += c.y;
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
        float v = acc[k];
        for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
        acc[k] = v;
    }
    if (ok && l < NPART) {
        float v = acc[0];
#pragma unroll
        for (int k = 1; k < NPART; ++k) v = l == k ? acc[k] : v;
        gr[int64_t(l) * n + g] = v;
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
// Super tiles of 64 Gaussians per workgroup, 16 per wave, all products on float32 matrix
// instructions (v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 16 x 4 by 4 x 16 product; output element v of lane l is D[4 (l / 16) + v][l % 16]).
// Per wave and its 16 Gaussians: the features x (bfloat16-rounded as the forward rounds them),
// layer 1 and 2 recomputed (pre-activations kept as ReLU masks, activations rounded to
// bfloat16), the heads, dF (dL/d layer-2 output), dH1 = (dF W2) masked, dx = dH1 W1 -> input
// gradients.  The weight gradients dW2 += dF^T h1 and dW1 += dH1^T x are shared out by rows:
// wave w accumulates rows 16 w .. 16 w + 15 over all 64 Gaussians of the super tile (read from
// the other waves' LDS between workgroup barriers), in registers over the workgroup's super
// tiles; bias and head sums per lane.  One record of sums per workgroup; mlp_wsum adds the
// workgroups in order.
constexpr int MT = 16;                  // Gaussians per wave per super tile
constexpr int XS = 25, HS = 65;         // LDS row strides (floats) of x and of the 64-wide rows
constexpr int W1S = 23, W2S = 65;       // LDS row strides of W1 [64][22] and W2 [64][64]
constexpr int MLP_WAVE_LDS = MT * XS + 2 * MT * HS + 2 * MT + 12 * MT;   // floats per wave
constexpr unsigned MLP_BLOCKS_MAX = 512;   // persistent workgroups
typedef float f32x4v __attribute__((ext_vector_type(4)));

// LDS written by some lanes of a wave and read by others after this point (a wave's LDS
// accesses are performed in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ f32x4v mfma16(float a, float b, f32x4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

inline unsigned mlp_blocks(int64_t n) {
    const int64_t tiles = (n + 4 * MT - 1) / (4 * MT);
    return unsigned(tiles < 1 ? 1 : (tiles < int64_t(MLP_BLOCKS_MAX) ? tiles : int64_t(MLP_BLOCKS_MAX)));
}

__global__ void __launch_bounds__(256)
bwd_mlp_kernel(mgs_gaussians gs, CamK cam, const float *__restrict__ prm, const float *__restrict__ gphi_in,
               const float *__restrict__ gom_in, mgs_gaussians_grad out, float *__restrict__ wpart) {
    __shared__ float sW1[64 * W1S];
    __shared__ float sW2[64 * W2S];
    __shared__ float sV[4][64];             // w_phi, w_o (bfloat16-rounded), b1, b2
    __shared__ float s_wave[4][MLP_WAVE_LDS];
    for (int e = threadIdx.x; e < 64 * 22; e += 256) sW1[(e / 22) * W1S + e % 22] = bf16_round(prm[MGS_MLP_OFF_W1 + e]);
    for (int e = threadIdx.x; e < 64 * 64; e += 256) sW2[(e / 64) * W2S + e % 64] = bf16_round(prm[MGS_MLP_OFF_W2 + e]);
    {
        const int r = threadIdx.x >> 6, c = threadIdx.x & 63;
        const int off[4] = {MGS_MLP_OFF_WPHI, MGS_MLP_OFF_WO, MGS_MLP_OFF_B1, MGS_MLP_OFF_B2};
        sV[r][c] = r < 2 ? bf16_round(prm[off[r] + c]) : prm[off[r] + c];
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    // wave ww's buffers: x [MT][XS]; P: h1, then dH1 [MT][HS]; Q: layer-2 output, then dF, then dx
    // [MT][HS]; (dphi, dmo) [MT][2]; P, 1/|v|, q, 1/|q|, s of its Gaussians [12][MT]
    auto bufX = [&](int ww) { return s_wave[ww]; };
    auto bufP = [&](int ww) { return s_wave[ww] + MT * XS; };
    auto bufQ = [&](int ww) { return s_wave[ww] + MT * XS + MT * HS; };
    float *sX = bufX(w), *sP = bufP(w), *sQ = bufQ(w);
    float *sD = sQ + MT * HS;
    float *sG = sD + 2 * MT;
    const int64_t n = gs.n;
    const float bphi = prm[MGS_MLP_OFF_BPHI], bo = prm[MGS_MLP_OFF_BO];
    // rows 16 w .. 16 w + 15 of dW2 (four column blocks) and dW1 (two); per lane j = l: sums of
    // db1, db2, dw_phi, dw_o over this wave's Gaussians; dbphi, dbo (the same in every lane)
    f32x4v gW2[4], gW1[2];
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
    gW1[0] = gW1[1] = f32x4v{0.f, 0.f, 0.f, 0.f};
    float gb1 = 0.f, gb2 = 0.f, gwp = 0.f, gwo = 0.f, gbphi = 0.f, gbo = 0.f;
    const int64_t tiles = (n + 4 * MT - 1) / (4 * MT);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {   // block-uniform
        const int64_t g0 = tile * (4 * MT) + w * MT;
        // 1. features of Gaussian g0 + l (lanes 0 .. 15)
        const int64_t gi = g0 + li;
        const bool mine = l < MT && gi < n;
        if (l < MT) {
            float P[3] = {0.f, 0.f, 0.f}, q[4] = {0.f, 0.f, 0.f, 0.f}, sc[3] = {0.f, 0.f, 0.f}, ivl = 0.f, iqn = 0.f;
            float x[22];
#pragma unroll
            for (int k = 0; k < 22; ++k) x[k] = 0.f;
            if (mine) {
                const float v0 = gs.mean[gi] - cam.campos[0], v1 = gs.mean[n + gi] - cam.campos[1],
                            v2 = gs.mean[2 * n + gi] - cam.campos[2];
                const float vl = sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
                ivl = 1.0f / vl;
                P[0] = v0 * ivl; P[1] = v1 * ivl; P[2] = v2 * ivl;
#pragma unroll
                for (int k = 0; k < 4; ++k) q[k] = gs.quat[k * n + gi];
                const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
                iqn = qn > 0.f ? 1.0f / qn : 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k) q[k] *= iqn;
#pragma unroll
                for (int k = 0; k < 3; ++k) sc[k] = expf(gs.log_scale[k * n + gi]);
#pragma unroll
                for (int k = 0; k < 3; ++k) { x[k] = P[k]; x[3 + k] = sc[k]; }
#pragma unroll
                for (int k = 0; k < 4; ++k) x[6 + k] = q[k];
#pragma unroll
                for (int k = 0; k < 12; ++k) x[10 + k] = gs.sh[k * n + gi];
            }
#pragma unroll
            for (int k = 0; k < 22; ++k) sX[l * XS + k] = bf16_round(x[k]);
            sX[l * XS + 22] = 0.f;
            sX[l * XS + 23] = 0.f;
            const float st[12] = {P[0], P[1], P[2], ivl, q[0], q[1], q[2], q[3], iqn, sc[0], sc[1], sc[2]};
#pragma unroll
            for (int k = 0; k < 12; ++k) sG[k * MT + l] = st[k];
        }
        wave_sync_lds();
        // 2. layer 1: H1[g][j] = b1[j] + sum_k x[g][k] W1[j][k]
        uint32_t m1 = 0, m2 = 0;           // ReLU masks, bit 4 nb + v for (g = 4 lk + v, j = 16 nb + li)
        {
            f32x4v acc[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int k = 4 * st + lk;
                const float a = sX[li * XS + k];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
                    acc[nb] = mfma16(a, k < 22 ? sW1[(16 * nb + li) * W1S + k] : 0.f, acc[nb]);
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float h = acc[nb][v] + sV[2][16 * nb + li];
                    m1 |= uint32_t(h > 0.f) << (4 * nb + v);
                    sP[(4 * lk + v) * HS + 16 * nb + li] = bf16_round(fmaxf(h, 0.f));
                }
        }
        wave_sync_lds();
        // 3. layer 2: F[g][j] = b2[j] + sum_k h1[g][k] W2[j][k]
        {
            f32x4v acc[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int st = 0; st < 16; ++st) {
                const int k = 4 * st + lk;
                const float a = sP[li * HS + k];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma16(a, sW2[(16 * nb + li) * W2S + k], acc[nb]);
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float f = acc[nb][v] + sV[3][16 * nb + li];
                    m2 |= uint32_t(f > 0.f) << (4 * nb + v);
                    sQ[(4 * lk + v) * HS + 16 * nb + li] = bf16_round(fmaxf(f, 0.f));
                }
        }
        wave_sync_lds();
        // 4. heads for Gaussian li (lane group lk takes neurons 16 lk .. 16 lk + 15), their
        //    gradients, and the head weight-gradient sums (lane l = neuron j)
        {
            float php = 0.f, mop = 0.f;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int j = 16 * lk + c;
                const float fb = sQ[li * HS + j];
                php = fmaf(sV[0][j], fb, php);
                mop = fmaf(sV[1][j], fb, mop);
            }
            php += __shfl_xor(php, 16, 64);
            mop += __shfl_xor(mop, 16, 64);
            php += __shfl_xor(php, 32, 64);
            mop += __shfl_xor(mop, 32, 64);
            php += bphi;
            mop += bo;
            const bool gok = g0 + li < n;
            const float m = 1.0f / (1.0f + expf(-mop));
            const float dphi = (gok && php > 0.f) ? gphi_in[g0 + li] : 0.f;
            const float dmo = gok ? gom_in[g0 + li] * m * (1.0f - m) : 0.f;
            if (lk == 0) {
                sD[2 * li] = dphi;
                sD[2 * li + 1] = dmo;
            }
        }
        wave_sync_lds();
#pragma unroll
        for (int g = 0; g < MT; ++g) {
            const float dphi = sD[2 * g], dmo = sD[2 * g + 1], fb = sQ[g * HS + l];
            gwp = fmaf(dphi, fb, gwp);
            gwo = fmaf(dmo, fb, gwo);
            gbphi += dphi;
            gbo += dmo;
        }
        wave_sync_lds();                    // the layer-2 outputs are read; Q takes dF
        // 5. dF[g][j] = (F > 0) (dphi w_phi[j] + dmo w_o[j])
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int g = 4 * lk + v;
            const float dphi = sD[2 * g], dmo = sD[2 * g + 1];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                sQ[g * HS + 16 * nb + li] =
                    ((m2 >> (4 * nb + v)) & 1u) ? fmaf(dphi, sV[0][16 * nb + li], dmo * sV[1][16 * nb + li]) : 0.f;
        }
        wave_sync_lds();
#pragma unroll
        for (int g = 0; g < MT; ++g) gb2 += sQ[g * HS + l];
        __syncthreads();                    // every wave's dF and h1 are written
        // 6. rows 16 w .. of dW2[j][k] += sum_g dF[g][j] h1[g][k] over the super tile's 64 Gaussians
#pragma unroll 1
        for (int ww = 0; ww < 4; ++ww) {
            const float *qF = bufQ(ww), *qH = bufP(ww);
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int g = 4 * st + lk;
                const float a = qF[g * HS + 16 * w + li];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) gW2[nb] = mfma16(a, qH[g * HS + 16 * nb + li], gW2[nb]);
            }
        }
        __syncthreads();                    // every wave's h1 is read; P takes dH1
        // 7. dH1[g][k] = (H1 > 0) sum_j dF[g][j] W2[j][k]
        {
            f32x4v acc[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int st = 0; st < 16; ++st) {
                const int j = 4 * st + lk;
                const float a = sQ[li * HS + j];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma16(a, sW2[j * W2S + 16 * nb + li], acc[nb]);
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    sP[(4 * lk + v) * HS + 16 * nb + li] = ((m1 >> (4 * nb + v)) & 1u) ? acc[nb][v] : 0.f;
        }
        wave_sync_lds();
#pragma unroll
        for (int g = 0; g < MT; ++g) gb1 += sP[g * HS + l];
        // 9. dx[g][k] = sum_j dH1[g][j] W1[j][k]  (into Q: this wave's dF is read)
        {
            f32x4v acc[2] = {f32x4v{0.f, 0.f, 0.f, 0.f}, f32x4v{0.f, 0.f, 0.f, 0.f}};
#pragma unroll 4
            for (int st = 0; st < 16; ++st) {
                const int j = 4 * st + lk;
                const float a = sP[li * HS + j];
                acc[0] = mfma16(a, sW1[j * W1S + li], acc[0]);
                acc[1] = mfma16(a, li < 6 ? sW1[j * W1S + 16 + li] : 0.f, acc[1]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sQ[(4 * lk + v) * HS + li] = acc[0][v];
                if (li < 6) sQ[(4 * lk + v) * HS + 16 + li] = acc[1][v];
            }
        }
        __syncthreads();                    // every wave's dH1 is written
        // 8. rows 16 w .. of dW1[j][k] += sum_g dH1[g][j] x[g][k] over the super tile
#pragma unroll 1
        for (int ww = 0; ww < 4; ++ww) {
            const float *qD = bufP(ww), *qX = bufX(ww);
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int g = 4 * st + lk;
                const float a = qD[g * HS + 16 * w + li];
                gW1[0] = mfma16(a, qX[g * XS + li], gW1[0]);
                gW1[1] = mfma16(a, li < 8 ? qX[g * XS + 16 + li] : 0.f, gW1[1]);
            }
        }
        // 10. input gradients of Gaussian g0 + l: P -> mean, s -> log_scale, q -> raw quaternion, Y -> sh
        if (mine) {
            const float *dx = sQ + l * HS;
            const float P[3] = {sG[0 * MT + l], sG[1 * MT + l], sG[2 * MT + l]}, ivl = sG[3 * MT + l];
            const float q[4] = {sG[4 * MT + l], sG[5 * MT + l], sG[6 * MT + l], sG[7 * MT + l]}, iqn = sG[8 * MT + l];
            const float sc[3] = {sG[9 * MT + l], sG[10 * MT + l], sG[11 * MT + l]};
            const float pd = P[0] * dx[0] + P[1] * dx[1] + P[2] * dx[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                out.mean[k * n + gi] += (dx[k] - P[k] * pd) * ivl;
                out.log_scale[k * n + gi] += dx[3 + k] * sc[k];
            }
            const float qd = q[0] * dx[6] + q[1] * dx[7] + q[2] * dx[8] + q[3] * dx[9];
#pragma unroll
            for (int k = 0; k < 4; ++k) out.quat[k * n + gi] += (dx[6 + k] - q[k] * qd) * iqn;
#pragma unroll
            for (int k = 0; k < 12; ++k) out.sh[k * n + gi] += dx[10 + k];
        }
        __syncthreads();                    // the super tile's LDS is reused by the next one
    }
    // this workgroup's sums, in the parameter layout: dW2 / dW1 rows of this wave; the per-lane
    // vector sums added over the four waves in wave order
    float *o = wpart + size_t(blockIdx.x) * MGS_MLP_PARAMS;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = 16 * w + 4 * lk + v;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) o[MGS_MLP_OFF_W2 + j * 64 + 16 * nb + li] = gW2[nb][v];
        o[MGS_MLP_OFF_W1 + j * 22 + li] = gW1[0][v];
        if (li < 6) o[MGS_MLP_OFF_W1 + j * 22 + 16 + li] = gW1[1][v];
    }
    float *red = s_wave[0];                 // [4 waves][4][64] + [4][2], after the loop's last barrier
    red[(w * 4 + 0) * 64 + l] = gb1;
    red[(w * 4 + 1) * 64 + l] = gb2;
    red[(w * 4 + 2) * 64 + l] = gwp;
    red[(w * 4 + 3) * 64 + l] = gwo;
    if (l == 0) {
        red[16 * 64 + 2 * w] = gbphi;
        red[16 * 64 + 2 * w + 1] = gbo;
    }
    __syncthreads();
    {
        const int r = threadIdx.x >> 6, c = threadIdx.x & 63;   // vector r, element c
        float acc = 0.f;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) acc += red[(ww * 4 + r) * 64 + c];
        const int off[4] = {MGS_MLP_OFF_B1, MGS_MLP_OFF_B2, MGS_MLP_OFF_WPHI, MGS_MLP_OFF_WO};
        o[off[r] + c] = acc;
        if (threadIdx.x < 2) {
            float h = 0.f;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) h += red[16 * 64 + 2 * ww + threadIdx.x];
            o[threadIdx.x == 0 ? MGS_MLP_OFF_BPHI : MGS_MLP_OFF_BO] = h;
        }
    }
}

// dmlp[p] = sum over the workgroups' records, in workgroup order (one wave per parameter:
// lanes take records lane, lane + 64, ..., then a fixed butterfly).
__global__ void __launch_bounds__(256)
mlp_wsum_kernel(const float *__restrict__ wpart, int nrec, float *__restrict__ dmlp) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    if (p >= MGS_MLP_PARAMS) return;                                   // wave-uniform
    float s = 0.f;
    for (int k = l; k < nrec; k += 64) s += wpart[size_t(k) * MGS_MLP_PARAMS + p];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if (l == 0) dmlp[p] = s;
}

__global__ void fill_zero_kernel(float *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------ host side
struct BwdLayout {
    size_t first, scan, chunks, cbase, tscan, items, part, gr, gphi, gom, wpart, total;
    uint64_t max_items;
};

inline BwdLayout bwd_layout(int64_t n, uint32_t T, uint64_t cap, bool mlp) {
    BwdLayout L;
    const size_t nn = size_t(n > 0 ? n : 1), cc = size_t(cap > 0 ? cap : 1), tt = size_t(T > 0 ? T : 1);
    L.max_items = bwd_max_items(T, cc);
    size_t o = 0;
    L.first = o;  o = align_up(o + nn * 4, 256);
    L.scan = o;   o = align_up(o + scan_tmp_elems(n) * 8 + 16, 256);
    L.chunks = o; o = align_up(o + tt * 4, 256);
    L.cbase = o;  o = align_up(o + tt * 4, 256);
    L.tscan = o;  o = align_up(o + scan_tmp_elems(int64_t(tt)) * 8 + 16, 256);
    L.items = o;  o = align_up(o + size_t(L.max_items) * 8, 256);
    L.part = o;   o = align_up(o + cc * PART_STRIDE * 4, 256);
    L.gr = o;     o = align_up(o + nn * NPART * 4, 256);
    L.gphi = o;   o = align_up(o + (mlp ? nn * 4 : 0), 256);
    L.gom = o;    o = align_up(o + (mlp ? nn * 4 : 0), 256);
    L.wpart = o;  o = align_up(o + (mlp ? size_t(mlp_blocks(n)) * MGS_MLP_PARAMS * 4 : 0), 256);
    L.total = o;
    return L;
}

}  // namespace mgs

extern "C" int mgs_render_backward_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity,
                                             int with_mlp, size_t *bytes) {
    MGS_REQUIRE(bytes && n >= 0 && tiles_x > 0 && tiles_y > 0, "bad arguments");
    MGS_REQUIRE(uint64_t(tiles_x) * uint64_t(tiles_y) < (uint64_t(1) << 31), "tile grid too large");
    *bytes = mgs::bwd_layout(n, uint32_t(tiles_x) * uint32_t(tiles_y), capacity, with_mlp != 0).total;
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
    MGS_REQUIRE(out && bg && tile_offsets && gids && aux && dL_dimage, "a required pointer is NULL");
    MGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f && alpha_max > alpha_min && alpha_max < 1.f, "bad alpha range");
    const bool mlp = mlp_params != nullptr;
    MGS_REQUIRE(!mlp || (phi && omod && dmlp), "the MLP path needs phi, omod and dmlp");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32), "capacity too large");
    const int64_t n = g->n;
    const CamK k = make_camk(cam);
    const uint32_t T = uint32_t(k.tiles_x) * uint32_t(k.tiles_y);
    const BwdLayout L = bwd_layout(n, T, capacity, mlp);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    if (n > 0) MGS_REQUIRE(out->mean && out->log_scale && out->quat && out->opacity_logit && out->sh,
                           "a gradient pointer is NULL");
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(ws);
    uint32_t *first = reinterpret_cast<uint32_t *>(w + L.first);
    uint64_t *stmp = reinterpret_cast<uint64_t *>(w + L.scan);
    uint32_t *ptot = reinterpret_cast<uint32_t *>(w + L.scan + scan_tmp_elems(n) * 8);
    uint32_t *chunks = reinterpret_cast<uint32_t *>(w + L.chunks);
    uint32_t *cbase = reinterpret_cast<uint32_t *>(w + L.cbase);
    uint64_t *ttmp = reinterpret_cast<uint64_t *>(w + L.tscan);
    uint32_t *n_items = reinterpret_cast<uint32_t *>(w + L.tscan + scan_tmp_elems(int64_t(T > 0 ? T : 1)) * 8);
    uint2 *items = reinterpret_cast<uint2 *>(w + L.items);
    float *part = reinterpret_cast<float *>(w + L.part);
    float *gr = reinterpret_cast<float *>(w + L.gr);
    float *gphi = mlp ? reinterpret_cast<float *>(w + L.gphi) : nullptr;
    float *gom = mlp ? reinterpret_cast<float *>(w + L.gom) : nullptr;
    float *wpart = reinterpret_cast<float *>(w + L.wpart);
    if (n == 0) {
        if (mlp) {
            hipLaunchKernelGGL(fill_zero_kernel, dim3((MGS_MLP_PARAMS + 255) / 256), dim3(256), 0, s, dmlp,
                               int(MGS_MLP_PARAMS));
            MGS_LAUNCH_CHECK("fill_zero_kernel");
        }
        return MGS_OK;
    }
    if ((rc = scan_exclusive(proj->n_tiles, first, n, stmp, ptot, s)) != MGS_OK) return rc;
    const uint64_t cap1 = uint64_t(capacity > 0 ? capacity : 1);
    hipLaunchKernelGGL(bwd_chunks_kernel, dim3((T + 255) / 256), dim3(256), 0, s, tile_offsets, T, ptot, cap1, chunks);
    MGS_LAUNCH_CHECK("bwd_chunks_kernel");
    if ((rc = scan_exclusive(chunks, cbase, int64_t(T), ttmp, n_items, s)) != MGS_OK) return rc;
    hipLaunchKernelGGL(bwd_items_kernel, dim3((T + 255) / 256), dim3(256), 0, s, tile_offsets, chunks, cbase, T,
                       L.max_items, items);
    MGS_LAUNCH_CHECK("bwd_items_kernel");
    const unsigned grid = unsigned(L.max_items < BWD_GRID_MAX ? L.max_items : BWD_GRID_MAX);
    hipLaunchKernelGGL(bwd_blend_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<const float4 *>(proj->splat),
                       reinterpret_cast<const uint2 *>(proj->rect), first, tile_offsets, gids, items, n_items,
                       L.max_items, ptot, k, bg[0], bg[1], bg[2], log2f(alpha_min), alpha_max, aux, dL_dimage, part,
                       cap1);
    MGS_LAUNCH_CHECK("bwd_blend_kernel");
    hipLaunchKernelGGL(bwd_reduce_kernel, dim3(unsigned((n + 15) / 16)), dim3(256), 0, s, first, proj->n_tiles, n,
                       part, cap1, ptot, gr);
    MGS_LAUNCH_CHECK("bwd_reduce_kernel");
    hipLaunchKernelGGL(bwd_gauss_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, *g, k, phi, omod,
                       proj->n_tiles, gr, *out, gphi, gom);
    MGS_LAUNCH_CHECK("bwd_gauss_kernel");
    if (mlp) {
        const unsigned mb = mlp_blocks(n);
        hipLaunchKernelGGL(bwd_mlp_kernel, dim3(mb), dim3(256), 0, s, *g, k, mlp_params, gphi, gom, *out, wpart);
        MGS_LAUNCH_CHECK("bwd_mlp_kernel");
        hipLaunchKernelGGL(mlp_wsum_kernel, dim3((MGS_MLP_PARAMS + 3) / 4), dim3(256), 0, s, wpart, int(mb), dmlp);
        MGS_LAUNCH_CHECK("mlp_wsum_kernel");
    }
    return MGS_OK;
}

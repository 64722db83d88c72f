// Splat-versus-rectangle culling shared by the forward and backward blends.
#pragma once

#include "common.h"
#include "index_math.h"

namespace mgs {

constexpr float CULL_MARGIN = 1e-3f;   // log2 units; keeps the quadrant test conservative

struct Splat {
    float4 r0;   // mx, my, log2(o), w
    float4 r1;   // kA, beta, kG, depth
    float4 r2;   // r, g, b, o
};

// Bit q set <=> the splat may reach quadrant q of tile (tx, ty): the largest log2(alpha) over
// the quadrant's 8x8 pixel centres is at least thr - CULL_MARGIN.
//
// log2(alpha) = log2(o) + g(dx, dy) with g = kA (dx + beta dy)^2 + kG dy^2 <= 0 concave in the
// offset from the mean, so its maximum over a rectangle is g = 0 at the mean if the mean is
// inside, else on an edge: on a row (dy fixed) at dx = -beta dy, on a column (dx fixed) at
// dy = -kA beta dx / (kA beta^2 + kG), each clamped to the edge.  The four quadrants are bounded
// by four pixel-centre rows and four columns of the tile; each line's vertex is found once.
// Only the vertex position is rounded differently from an exact division (it moves the
// evaluated point along the edge by a relative 1e-7), far inside the margin.
__device__ __forceinline__ uint32_t quadrant_mask(float4 r0, float4 r1, int tx, int ty, float thr) {
    const float kA = r1.x, beta = r1.y, kG = r1.z;
    const float slope = -kA * beta * __builtin_amdgcn_rcpf(fmaf(kA * beta, beta, kG));
    // bounding columns / rows as offsets from the mean: quadrants with (q & 1) == s span columns
    // xs[2 s] .. xs[2 s + 1], those with (q >> 1) == s rows ys[2 s] .. ys[2 s + 1]
    const float xa = float(tx * 16) + 0.5f - r0.x, ya = float(ty * 16) + 0.5f - r0.y;
    const float xs[4] = {xa, xa + 7.0f, xa + 8.0f, xa + 15.0f};
    const float ys[4] = {ya, ya + 7.0f, ya + 8.0f, ya + 15.0f};
    // best[2 sy + sx]: largest g on the edges of quadrant (sx, sy) so far
    float best[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int k = 0; k < 4; ++k) {                   // row k bounds the quadrants with sy = k / 2
        const float y = ys[k], vx = -beta * y, gy = kG * y * y;
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
            const float t = fmaf(beta, y, __builtin_amdgcn_fmed3f(vx, xs[2 * sx], xs[2 * sx + 1]));
            best[2 * (k >> 1) + sx] = fmaxf(best[2 * (k >> 1) + sx], fmaf(kA * t, t, gy));
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {                   // column k bounds the quadrants with sx = k / 2
        const float x = xs[k], vy = slope * x;
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const float dy = __builtin_amdgcn_fmed3f(vy, ys[2 * sy], ys[2 * sy + 1]);
            const float t = fmaf(beta, dy, x);
            best[2 * sy + (k >> 1)] = fmaxf(best[2 * sy + (k >> 1)], fmaf(kA * t, t, kG * dy * dy));
        }
    }
    const float need = thr - CULL_MARGIN - r0.z;    // g must reach this somewhere
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int sx = q & 1, sy = q >> 1;
        const bool inside = xs[2 * sx] <= 0.0f && xs[2 * sx + 1] >= 0.0f && ys[2 * sy] <= 0.0f && ys[2 * sy + 1] >= 0.0f;
        if ((inside ? 0.0f : best[q]) >= need) m |= 1u << q;
    }
    return m;
}

constexpr int BLEND_THREADS = 256;
constexpr int BLEND_BATCH = 128;

// Exponent of a splat as a polynomial in a pixel's offset (x, y) from a centre (xc, yc)
// (a quadrant's or a tile's):
//   log2(alpha) = c0 + cx x + cy y + cxx x^2 + cxy x y + cyy y^2
// (the same quadratic form as log2(o) + kA t^2 + kG dy^2, re-centred once per
// staged splat so the per-pixel work is a few FMAs).
__device__ __forceinline__ void quad_poly(float4 r0, float4 r1, float xc, float yc, float4 &qa, float4 &qb) {
    const float kA = r1.x, beta = r1.y, kG = r1.z;
    const float u0 = xc - r0.x, v0 = yc - r0.y;
    const float t0 = fmaf(beta, v0, u0);
    qa.x = r0.z + kA * t0 * t0 + kG * v0 * v0;
    qa.y = 2.0f * kA * t0;
    qa.z = 2.0f * fmaf(kA * t0, beta, kG * v0);
    qa.w = kA;
    qb.x = 2.0f * kA * beta;
    qb.y = fmaf(kA * beta, beta, kG);
}

// Background weight that selects Eq. 2's composite (any w_bg >= 0 selects Eq. 1's).
constexpr float EQ2_COMPOSITE = -1.0f;

// Composite of one pixel from its sums.  Eq. 2 (wbg < 0): C = (1 - T) N / D + T c_bg (c_bg if
// D = 0).  Eq. 1 (wbg >= 0): C = (c_bg wbg + N) / (wbg + D) (c_bg if wbg + D = 0).
// aux (if non-NULL) receives (N/D rgb, D, T) in both cases.
__device__ __forceinline__ void composite_oit(float Nr, float Ng, float Nb, float D, float T, int px, int py, int W,
                                              int H, float bgr, float bgg, float bgb, float wbg,
                                              float *__restrict__ image, float *__restrict__ aux) {
    if (px >= W || py >= H) return;
    const size_t hw = size_t(W) * H;
    const size_t p = size_t(py) * W + px;
    float cr, cg, cb;
    if (wbg >= 0.f) {
        const float den = wbg + D;
        if (den > 0.f) {
            const float inv = 1.0f / den;
            cr = fmaf(wbg, bgr, Nr) * inv;
            cg = fmaf(wbg, bgg, Ng) * inv;
            cb = fmaf(wbg, bgb, Nb) * inv;
        } else {
            cr = bgr; cg = bgg; cb = bgb;
        }
        if (aux) {
            const float inv = D > 0.f ? 1.0f / D : 0.0f;
            aux[p] = Nr * inv; aux[hw + p] = Ng * inv; aux[2 * hw + p] = Nb * inv;
            aux[3 * hw + p] = D; aux[4 * hw + p] = T;
        }
    } else if (D > 0.f) {
        const float inv = 1.0f / D;
        const float fr = Nr * inv, fg = Ng * inv, fb = Nb * inv;
        const float f = 1.0f - T;
        cr = fmaf(f, fr, T * bgr);
        cg = fmaf(f, fg, T * bgg);
        cb = fmaf(f, fb, T * bgb);
        if (aux) {
            aux[p] = fr; aux[hw + p] = fg; aux[2 * hw + p] = fb;
            aux[3 * hw + p] = D; aux[4 * hw + p] = T;
        }
    } else {
        cr = bgr; cg = bgg; cb = bgb;
        if (aux) {
            aux[p] = 0.f; aux[hw + p] = 0.f; aux[2 * hw + p] = 0.f;
            aux[3 * hw + p] = 0.f; aux[4 * hw + p] = 1.f;
        }
    }
    image[p] = cr;
    image[hw + p] = cg;
    image[2 * hw + p] = cb;
}

// Pixel of workgroup thread `k` in tile (tx, ty): wave k / 64 owns quadrant (w & 1, w >> 1).
__device__ __forceinline__ void tile_pixel(int k, int tx, int ty, int &px, int &py) {
    const int w = k >> 6, l = k & 63;
    px = tx * 16 + (w & 1) * 8 + (l & 7);
    py = ty * 16 + (w >> 1) * 8 + (l >> 3);
}

// Front-to-back composite (Eq. 11) of one 16x16 tile (tile coordinates tx, ty) from its
// depth-sorted list gids[start, end) into image of a W x H view.  Called by a whole
// 256-thread workgroup: wave w owns quadrant (w & 1, w >> 1), lane l one pixel of it, and
// the wave stops once every one of its pixels has transmittance below t_stop.
__device__ __forceinline__ void blend_tile_sorted(const float4 *__restrict__ splat, const uint32_t *__restrict__ gids,
                                                  uint32_t start, uint32_t end, int tx, int ty, int W, int H,
                                                  float bgr, float bgg, float bgb, float log2_amin, float amax,
                                                  float t_stop, float *__restrict__ image) {
    // per quadrant and staged splat: polynomial (c0, cx, cy, cxx), (cxy, cyy, -, -) and the colour
    // (r, g, b, -), one 48-byte record so a wave reads all three with one address register
    __shared__ float4 s_rec[4][BLEND_BATCH][3];
    __shared__ uint32_t s_mask[BLEND_BATCH];
    __shared__ int s_done[4];

    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int px = tx * 16 + (w & 1) * 8 + (l & 7);
    const int py = ty * 16 + (w >> 1) * 8 + (l >> 3);
    // lane offset from the quadrant centre, and its products
    const float lx = float(l & 7) - 3.5f, ly = float(l >> 3) - 3.5f;
    const float lxx = lx * lx, lxy = lx * ly, lyy = ly * ly;

    float Nr = 0.f, Ng = 0.f, Nb = 0.f, T = 1.f;
    bool wave_done = false;

    for (uint32_t b = start; b < end; b += BLEND_BATCH) {
        __syncthreads();
        if (threadIdx.x < BLEND_BATCH) {
            const uint32_t i = b + threadIdx.x;
            uint32_t mask = 0;
            if (i < end) {
                const uint32_t g = gids[i];
                const float4 r0 = splat[3 * size_t(g) + 0];
                const float4 r1 = splat[3 * size_t(g) + 1];
                const float4 r2 = splat[3 * size_t(g) + 2];
                mask = quadrant_mask(r0, r1, tx, ty, log2_amin);
                const float4 col = make_float4(r2.x, r2.y, r2.z, 0.f);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if ((mask >> q) & 1u) {
                        float4 qa;
                        float4 qb = make_float4(0.f, 0.f, 0.f, 0.f);
                        quad_poly(r0, r1, float(tx * 16 + (q & 1) * 8) + 4.0f, float(ty * 16 + (q >> 1) * 8) + 4.0f,
                                  qa, qb);
                        s_rec[q][threadIdx.x][0] = qa;
                        s_rec[q][threadIdx.x][1] = qb;
                        s_rec[q][threadIdx.x][2] = col;
                    }
                }
            }
            s_mask[threadIdx.x] = mask;
        }
        if (l == 0) s_done[w] = wave_done ? 1 : 0;
        __syncthreads();
        if (s_done[0] && s_done[1] && s_done[2] && s_done[3]) break;
        if (wave_done) continue;
        const int wu = __builtin_amdgcn_readfirstlane(w);       // wave-uniform quadrant index
        const float4(*rec_w)[3] = s_rec[wu];
        for (int grp = 0; grp < BLEND_BATCH / 64; ++grp) {
            uint64_t bal = __ballot((s_mask[grp * 64 + l] >> w) & 1u);
            while (bal) {
                const int j = grp * 64 + __builtin_ctzll(bal);
                bal &= bal - 1;
                const float4 qa = rec_w[j][0];
                const float4 qb = rec_w[j][1];
                const float4 cw = rec_w[j][2];
                float e = fmaf(qa.y, lx, qa.x);
                e = fmaf(qa.z, ly, e);
                e = fmaf(qa.w, lxx, e);
                e = fmaf(qb.x, lxy, e);
                e = fmaf(qb.y, lyy, e);
                const float al = (e >= log2_amin && T >= t_stop) ? fminf(fast_exp2(e), amax) : 0.0f;
                const float at = al * T;
                Nr = fmaf(at, cw.x, Nr);
                Ng = fmaf(at, cw.y, Ng);
                Nb = fmaf(at, cw.z, Nb);
                T = fmaf(-T, al, T);
            }
            wave_done = __ballot(T >= t_stop) == 0ull;
            if (wave_done) break;
        }
    }

    if (px < W && py < H) {
        const size_t hw = size_t(W) * H;
        const size_t p = size_t(py) * W + px;
        image[p] = fmaf(T, bgr, Nr);
        image[hw + p] = fmaf(T, bgg, Ng);
        image[2 * hw + p] = fmaf(T, bgb, Nb);
    }
}

// Staged-Gaussian flag of the order-independent blend (bits 0-3 are the quadrant mask): the
// Gaussian's peak log2(o) is within OIT_CLAMP_MARGIN of log2(alpha_max), so the clamp may bind.
constexpr uint32_t OIT_CLAMP = 1u << 8;
constexpr float OIT_CLAMP_MARGIN = 1e-2f;

// Order-independent composite (Eq. 2) of one 16x16 tile (tile coordinates tx, ty) from
// the list range gids[start, end).  Called by a whole 256-thread workgroup.
//
// The four waves share the range: wave w takes every fourth Gaussian of the list (4k + w),
// stages 64 of them at a time in its own LDS region (one per lane) and walks them without
// waiting for the other waves.  Each lane holds four pixels, one per 8x8 quadrant (pixel
// (l & 7, l >> 3) of each).  A staged Gaussian is read from LDS once and evaluated only on
// the quadrants its exact quadrant test keeps, so a 40-byte broadcast read feeds up to four
// pixel updates.
// The exponent is a polynomial in the pixel's offset from the tile centre (quad_poly about
// (16 tx + 8, 16 ty + 8)); offsets are within +-7.5 px.  At the end the waves' sums are
// merged through LDS in wave order (N and D add, T multiplies), which is exact up to
// rounding because the composite does not depend on the order of the Gaussians.
//
// The result goes to thread k's pixel tile_pixel(k) (quadrant k / 64, lane k % 64): the
// composite (Eq. 2, or Eq. 1 for wbg >= 0) into image / aux of a W x H view, or, if part is
// non-NULL, the sums
// (N rgb, D, T) to part[5][256] for a later merge with the tile's other ranges.
constexpr int OIT_BATCH = 256;                  // list positions staged per pass by the four waves

__device__ __forceinline__ void blend_tile_oit(const float4 *__restrict__ splat, const uint32_t *__restrict__ gids,
                                               uint32_t start, uint32_t end, int tx, int ty, int W, int H, float bgr,
                                               float bgg, float bgb, float wbg, float log2_amin, float amax,
                                               float *__restrict__ image, float *__restrict__ aux,
                                               float *__restrict__ part) {
    // wave w's staged Gaussian j: (c0, cx, cy, cxx), (cxy, cyy, -, -), (w r, w g, w b, w) at
    // s_buf[192 w + 3 j ..]; after the last batch the same memory holds the waves' sums
    __shared__ float4 s_buf[4 * 4 * 5 * 64 / 4];

    // the wave index is uniform: held in a scalar register, the wave's LDS region address is
    // scalar and a staged record's address costs one move per Gaussian
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    // the lane's pixel offsets from the tile centre: x in the left / right quadrants, y in the
    // top / bottom ones
    const float xl = float(l & 7) - 7.5f, xr = xl + 8.0f;
    const float yt = float(l >> 3) - 7.5f, yb = yt + 8.0f;
    const float tcx = float(tx * 16) + 8.0f, tcy = float(ty * 16) + 8.0f;

    // per quadrant q: N rgb, D, T
    float acc[4][5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.f;
        acc[q][4] = 1.f;
    }

    // log2(o) above this: the alpha_max clamp can bind somewhere in the tile (the margin is
    // far above the float32 error of the exponent polynomial)
    const float log2_amax_safe = __log2f(amax) - OIT_CLAMP_MARGIN;
    // Each wave stages and walks its own Gaussians (list positions b + 4 l + w, l = 0 .. 63,
    // for b = start, start + 256, ...) in its own LDS region, so the waves never wait on
    // each other before the final merge.
    float4 *wbuf = s_buf + w * (3 * 64);
    for (uint32_t b = start; b < end; b += OIT_BATCH) {
        const uint32_t i = b + 4 * l + w;
        uint32_t mk = 0;
        if (i < end) {
            const uint32_t g = gids[i];
            const float4 r0 = splat[3 * size_t(g) + 0];
            const float4 r1 = splat[3 * size_t(g) + 1];
            mk = quadrant_mask(r0, r1, tx, ty, log2_amin);
            if (mk) {
                const float4 r2 = splat[3 * size_t(g) + 2];   // colour, only for a kept Gaussian
                float4 qa, qb = make_float4(0.f, 0.f, 0.f, 0.f);
                quad_poly(r0, r1, tcx, tcy, qa, qb);
                wbuf[3 * l + 0] = qa;
                wbuf[3 * l + 1] = qb;
                wbuf[3 * l + 2] = make_float4(r0.w * r2.x, r0.w * r2.y, r0.w * r2.z, r0.w);
                if (r0.z > log2_amax_safe) mk |= OIT_CLAMP;
            }
        }
        // the lanes' records are visible to the whole wave (LDS is in order within a wave)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Gaussians whose alpha can reach alpha_max are taken last, in the only loop that needs
        // the clamp.  The others are walked by quadrant pattern: one loop per pattern a convex
        // footprint usually has (one quadrant, two side by side, all four) evaluates exactly
        // those quadrants with no per-Gaussian tests; the rare rest (three quadrants, diagonals)
        // go through a loop that tests each quadrant.
        const uint64_t clamp = __ballot((mk & OIT_CLAMP) != 0u);
        const uint32_t mq = mk & 15u;
        constexpr uint32_t OWN_LOOP = (1u << 1) | (1u << 2) | (1u << 4) | (1u << 8) | (1u << 3) | (1u << 12) |
                                      (1u << 5) | (1u << 10) | (1u << 15);
        uint64_t any = __ballot(mq != 0u && ((OWN_LOOP >> mq) & 1u) == 0u) & ~clamp;
        // per quadrant, the staged Gaussians that reach it (tested in scalar registers)
        const uint64_t qm0 = __ballot((mk & 1u) != 0u), qm1 = __ballot((mk & 2u) != 0u);
        const uint64_t qm2 = __ballot((mk & 4u) != 0u), qm3 = __ballot((mk & 8u) != 0u);
// The exponent c0 + cx x + cy y + cxx x^2 + cxy x y + cyy y^2 is evaluated as
// P(y) + x (R(y) + cxx x), P(y) = c0 + y (cy + cyy y), R(y) = cx + cxy y: the two quadrants
// of a row share y, so P and R are computed once for both (3 FMA) and each pixel costs 2.
#define MGS_OIT_ROWTERMS(Y)                                                         \
            const float P = fmaf(fmaf(qb.y, Y, qa.z), Y, qa.x);                     \
            const float R = fmaf(qb.x, Y, qa.y);
#define MGS_OIT_EVAL(q, X, ALPHA)                                                   \
            {                                                                       \
                const float e = fmaf(fmaf(qa.w, X, R), X, P);                       \
                const float al = e >= log2_amin ? ALPHA : 0.0f;                     \
                acc[q][0] = fmaf(al, cw.x, acc[q][0]);                              \
                acc[q][1] = fmaf(al, cw.y, acc[q][1]);                              \
                acc[q][2] = fmaf(al, cw.z, acc[q][2]);                              \
                acc[q][3] = fmaf(al, cw.w, acc[q][3]);                              \
                acc[q][4] = fmaf(-acc[q][4], al, acc[q][4]);                        \
            }
// staged Gaussians of SET in list order, their record in qa, qb, cw
#define MGS_OIT_WALK(SET, BODY)                                                     \
        for (uint64_t set = (SET); set; set &= set - 1) {                           \
            const int k = __builtin_ctzll(set);                                     \
            const float4 *rec = wbuf + 3 * k;                                       \
            const float4 qa = rec[0];                                               \
            const float4 qb = rec[1];                                               \
            const float4 cw = rec[2];                                               \
            BODY                                                                    \
        }
#define MGS_OIT_PATTERN(M, BODY) MGS_OIT_WALK(__ballot(mq == (M)) & ~clamp, BODY)
#define MGS_OIT_TOP(BODY) { MGS_OIT_ROWTERMS(yt) BODY }
#define MGS_OIT_BOTTOM(BODY) { MGS_OIT_ROWTERMS(yb) BODY }
#define MGS_OIT_Q0 MGS_OIT_EVAL(0, xl, fast_exp2(e))
#define MGS_OIT_Q1 MGS_OIT_EVAL(1, xr, fast_exp2(e))
#define MGS_OIT_Q2 MGS_OIT_EVAL(2, xl, fast_exp2(e))
#define MGS_OIT_Q3 MGS_OIT_EVAL(3, xr, fast_exp2(e))
        MGS_OIT_PATTERN(1u, MGS_OIT_TOP(MGS_OIT_Q0))
        MGS_OIT_PATTERN(2u, MGS_OIT_TOP(MGS_OIT_Q1))
        MGS_OIT_PATTERN(4u, MGS_OIT_BOTTOM(MGS_OIT_Q2))
        MGS_OIT_PATTERN(8u, MGS_OIT_BOTTOM(MGS_OIT_Q3))
        MGS_OIT_PATTERN(3u, MGS_OIT_TOP(MGS_OIT_Q0 MGS_OIT_Q1))
        MGS_OIT_PATTERN(12u, MGS_OIT_BOTTOM(MGS_OIT_Q2 MGS_OIT_Q3))
        MGS_OIT_PATTERN(5u, MGS_OIT_TOP(MGS_OIT_Q0) MGS_OIT_BOTTOM(MGS_OIT_Q2))
        MGS_OIT_PATTERN(10u, MGS_OIT_TOP(MGS_OIT_Q1) MGS_OIT_BOTTOM(MGS_OIT_Q3))
        MGS_OIT_PATTERN(15u, MGS_OIT_TOP(MGS_OIT_Q0 MGS_OIT_Q1) MGS_OIT_BOTTOM(MGS_OIT_Q2 MGS_OIT_Q3))
#undef MGS_OIT_Q3
#undef MGS_OIT_Q2
#undef MGS_OIT_Q1
#undef MGS_OIT_Q0
#define MGS_OIT_TESTED(q, X, ALPHA) if ((qm##q >> k) & 1u) MGS_OIT_EVAL(q, X, ALPHA)
#define MGS_OIT_ANY(ALPHA)                                                          \
        if (((qm0 | qm1) >> k) & 1u)                                                \
            MGS_OIT_TOP(MGS_OIT_TESTED(0, xl, ALPHA) MGS_OIT_TESTED(1, xr, ALPHA))   \
        if (((qm2 | qm3) >> k) & 1u)                                                \
            MGS_OIT_BOTTOM(MGS_OIT_TESTED(2, xl, ALPHA) MGS_OIT_TESTED(3, xr, ALPHA))
        MGS_OIT_WALK(any, MGS_OIT_ANY(fast_exp2(e)))
        MGS_OIT_WALK(clamp, MGS_OIT_ANY(fminf(fast_exp2(e), amax)))
#undef MGS_OIT_ANY
#undef MGS_OIT_TESTED
#undef MGS_OIT_BOTTOM
#undef MGS_OIT_TOP
#undef MGS_OIT_PATTERN
#undef MGS_OIT_WALK
#undef MGS_OIT_EVAL
#undef MGS_OIT_ROWTERMS
        // every lane's reads of this batch's records precede the next batch's writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // merge the four waves' sums: s_sum[(w * 4 + q) * 5 + v][l]
    float *s_sum = reinterpret_cast<float *>(s_buf);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 5; ++v) s_sum[((w * 4 + q) * 5 + v) * 64 + l] = acc[q][v];
    __syncthreads();
    // thread (w, l) now takes pixel l of quadrant w
    float S[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) S[v] = s_sum[((0 * 4 + w) * 5 + v) * 64 + l];
#pragma unroll
    for (int src = 1; src < 4; ++src) {
#pragma unroll
        for (int v = 0; v < 4; ++v) S[v] += s_sum[((src * 4 + w) * 5 + v) * 64 + l];
        S[4] *= s_sum[((src * 4 + w) * 5 + 4) * 64 + l];
    }
    if (part) {
        const int k = threadIdx.x;
        part[k] = S[0];
        part[256 + k] = S[1];
        part[512 + k] = S[2];
        part[768 + k] = S[3];
        part[1024 + k] = S[4];
    } else {
        int px, py;
        tile_pixel(threadIdx.x, tx, ty, px, py);
        composite_oit(S[0], S[1], S[2], S[3], S[4], px, py, W, H, bgr, bgg, bgb, wbg, image, aux);
    }
}

// ---------------------------------------------------------------- split tiles
// Order independence makes the per-pixel state additive (N and D add, T multiplies), so a long
// tile list can be cut into ranges rendered by different workgroups and merged exactly: the
// range plan (n_ranges, range_len; item = tile | range << 24) is in index_math.h.

}  // namespace mgs

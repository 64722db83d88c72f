// Splat-versus-rectangle culling shared by the forward and backward blends.
#pragma once

#include "common.h"

namespace mgs {

constexpr float CULL_MARGIN = 1e-3f;   // log2 units; keeps the quadrant test conservative

struct Splat {
    float4 r0;   // mx, my, log2(o), w
    float4 r1;   // kA, beta, kG, depth
    float4 r2;   // r, g, b, o
};

// Largest log2(alpha) of a splat over the rectangle of pixel centres
// [x0, x1] x [y0, y1] (offsets from the splat mean).
__device__ __forceinline__ float max_log2_alpha(float4 r0, float4 r1, float x0, float x1, float y0, float y1) {
    const float kA = r1.x, beta = r1.y, kG = r1.z;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return r0.z;
    // g(dx, dy) = kA (dx + beta dy)^2 + kG dy^2 <= 0, concave
    float best = -INFINITY;
    // horizontal edges: dy fixed, optimum dx = -beta dy
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dy = e ? y1 : y0;
        const float dx = fminf(fmaxf(-beta * dy, x0), x1);
        const float t = fmaf(beta, dy, dx);
        best = fmaxf(best, kA * t * t + kG * dy * dy);
    }
    // vertical edges: dx fixed, optimum dy = -kA beta dx / (kA beta^2 + kG)
    const float den = kA * beta * beta + kG;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = e ? x1 : x0;
        const float dy = fminf(fmaxf(-kA * beta * dx / den, y0), y1);
        const float t = fmaf(beta, dy, dx);
        best = fmaxf(best, kA * t * t + kG * dy * dy);
    }
    return r0.z + best;
}

// Bit q set <=> the splat may reach quadrant q of tile (tx, ty).
__device__ __forceinline__ uint32_t quadrant_mask(float4 r0, float4 r1, int tx, int ty, float thr) {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float X0 = float(tx * 16 + (q & 1) * 8) + 0.5f - r0.x;
        const float Y0 = float(ty * 16 + (q >> 1) * 8) + 0.5f - r0.y;
        if (max_log2_alpha(r0, r1, X0, X0 + 7.0f, Y0, Y0 + 7.0f) >= thr - CULL_MARGIN) m |= 1u << q;
    }
    return m;
}

constexpr int BLEND_THREADS = 256;
constexpr int BLEND_BATCH = 128;

// Exponent of a splat as a polynomial in the lane's offset (x, y) from its
// quadrant's centre, x, y in {-3.5 .. 3.5}:
//   log2(alpha) = c0 + cx x + cy y + cxx x^2 + cxy x y + cyy y^2
// (the same quadratic form as log2(o) + kA t^2 + kG dy^2, re-centred once per
// staged splat and quadrant so the per-pixel work is five FMAs).
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

// Composite one 16x16 tile (tile coordinates tx, ty) from its list gids[start, end)
// into image / aux of a W x H view.  Called by a whole 256-thread workgroup.
// Eq. 2 composite of one pixel from its sums: C = (1 - T) N / D + T c_bg (c_bg if D = 0);
// aux (if non-NULL) receives (N/D rgb, D, T).
__device__ __forceinline__ void composite_oit(float Nr, float Ng, float Nb, float D, float T, int px, int py, int W,
                                              int H, float bgr, float bgg, float bgb, float *__restrict__ image,
                                              float *__restrict__ aux) {
    if (px >= W || py >= H) return;
    const size_t hw = size_t(W) * H;
    const size_t p = size_t(py) * W + px;
    float cr, cg, cb;
    if (D > 0.f) {
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

// Composite one 16x16 tile (tile coordinates tx, ty) from the list range gids[start, end)
// into image / aux of a W x H view.  Called by a whole 256-thread workgroup.  With
// PARTIAL (order-independent path only) the per-pixel sums (N rgb, D, T) of this range
// go to part[5][256] instead, to be merged with the tile's other ranges.
template <bool SORTED, bool PARTIAL = false>
__device__ __forceinline__ void blend_tile(const float4 *__restrict__ splat, const uint32_t *__restrict__ gids,
                                           uint32_t start, uint32_t end, int tx, int ty, int W, int H, float bgr,
                                           float bgg, float bgb, float log2_amin, float amax, float t_stop,
                                           float *__restrict__ image, float *__restrict__ aux,
                                           float *__restrict__ part = nullptr) {
    // per quadrant and staged splat: polynomial (c0, cx, cy, cxx), (cxy, cyy, -, -) and the colour
    // (OIT: (w r, w g, w b, w); sorted: (r, g, b, 0)), one 48-byte record so a wave reads all three
    // with one address register
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

    float Nr = 0.f, Ng = 0.f, Nb = 0.f, D = 0.f, T = 1.f;
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
                const float4 col = SORTED ? make_float4(r2.x, r2.y, r2.z, 0.f)
                                          : make_float4(r0.w * r2.x, r0.w * r2.y, r0.w * r2.z, r0.w);
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
        if (SORTED && l == 0) s_done[w] = wave_done ? 1 : 0;
        __syncthreads();
        if (SORTED && s_done[0] && s_done[1] && s_done[2] && s_done[3]) break;
        if (SORTED && wave_done) continue;
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
                if (!SORTED) {
                    const float al = e >= log2_amin ? fminf(fast_exp2(e), amax) : 0.0f;
                    Nr = fmaf(al, cw.x, Nr);
                    Ng = fmaf(al, cw.y, Ng);
                    Nb = fmaf(al, cw.z, Nb);
                    D = fmaf(al, cw.w, D);
                    T = fmaf(-T, al, T);
                } else {
                    const float al = (e >= log2_amin && T >= t_stop) ? fminf(fast_exp2(e), amax) : 0.0f;
                    const float at = al * T;
                    Nr = fmaf(at, cw.x, Nr);
                    Ng = fmaf(at, cw.y, Ng);
                    Nb = fmaf(at, cw.z, Nb);
                    T = fmaf(-T, al, T);
                }
            }
            if (SORTED) {
                wave_done = __ballot(T >= t_stop) == 0ull;
                if (wave_done) break;
            }
        }
    }

    if (PARTIAL) {
        const int k = threadIdx.x;
        part[k] = Nr;
        part[256 + k] = Ng;
        part[512 + k] = Nb;
        part[768 + k] = D;
        part[1024 + k] = T;
    } else if (!SORTED) {
        composite_oit(Nr, Ng, Nb, D, T, px, py, W, H, bgr, bgg, bgb, image, aux);
    } else if (px < W && py < H) {
        const size_t hw = size_t(W) * H;
        const size_t p = size_t(py) * W + px;
        image[p] = fmaf(T, bgr, Nr);
        image[hw + p] = fmaf(T, bgg, Ng);
        image[2 * hw + p] = fmaf(T, bgb, Nb);
    }
}

// ---------------------------------------------------------------- split tiles
// Order independence makes the per-pixel state additive (N and D add, T multiplies), so
// a long tile list can be cut into ranges rendered by different workgroups and merged
// exactly.  Ranges hold at most `split` Gaussians (more for extremely long lists, so a
// tile has at most 255 ranges); item = tile | range << 24.
__device__ __forceinline__ uint32_t range_len(uint32_t L, uint32_t split) {
    const uint32_t m = (L + 254) / 255;
    return split > m ? split : m;
}
__device__ __forceinline__ uint32_t n_ranges(uint32_t L, uint32_t split) {
    const uint32_t r = range_len(L, split);
    return L == 0 ? 1u : (L + r - 1) / r;
}

}  // namespace mgs

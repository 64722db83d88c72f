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

}  // namespace mgs

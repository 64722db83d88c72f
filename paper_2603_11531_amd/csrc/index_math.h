// Index arithmetic of the binning, split-blend and backward kernels, as plain functions that
// compile for the device (hipcc) and for the host (any C++17 compiler).  The kernels call these
// functions; a host program replays them against brute-force enumerations under the address and
// undefined-behaviour sanitizers, so every index a kernel derives from them is checked on the
// CPU against the workspace bounds it is allocated with.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define MGS_HD __host__ __device__ __forceinline__
#else
#define MGS_HD inline
#endif

namespace mgs {

// ---------------------------------------------------------------- split tile lists (blend)
// 2,048: with the work items dispatched longest first, longer ranges (fewer partial sums to merge)
// measured faster than 1,024 on a 1M-Gaussian frame and no slower on a 3M one (in tile order,
// 1,024 was best)
constexpr uint32_t SPLIT_RANGE = 2048;       // Gaussians per range of a long tile list
constexpr uint32_t SPLIT_MAX_RANGES = 255;   // ranges per tile (8-bit range index in a work item)

MGS_HD uint32_t ceil_div(uint32_t a, uint32_t b) { return a / b + (a % b != 0u); }

// A list of L Gaussians is cut into n_ranges(L) ranges of equal length range_len(L) (the last up
// to n - 1 shorter): at most `split` Gaussians each, or ceil(L / 255) for lists longer than
// 255 * split, so a tile has at most 255 ranges.  An empty list is one (empty) range.
MGS_HD uint32_t n_ranges(uint32_t L, uint32_t split) {
    if (L == 0) return 1u;
    if (L <= SPLIT_MAX_RANGES * split) return ceil_div(L, split);
    return ceil_div(L, ceil_div(L, SPLIT_MAX_RANGES));
}
// Every range is non-empty: with n = n_ranges(L) and len = ceil(L / n), (n - 1) len < L.
MGS_HD uint32_t range_len(uint32_t L, uint32_t split) { return ceil_div(L, n_ranges(L, split)); }

// Workspace bounds of the split plan for T tiles and at most `capacity` pairs: work items
// (one per range) and partial-sum slots (one per range of a tile with more than one range).
MGS_HD uint64_t split_max_items(uint64_t T, uint64_t capacity) { return T + capacity / SPLIT_RANGE + 1; }
MGS_HD uint64_t split_max_slots(uint64_t capacity) { return 2 * (capacity / SPLIT_RANGE) + 2; }

// ---------------------------------------------------------------- two-level binning
constexpr int SUPER_SHIFT = 3;                // supertile = 8 x 8 tiles
constexpr int SUPER = 1 << SUPER_SHIFT;
constexpr int SUPER_TILES = SUPER * SUPER;
constexpr int ST_KEY_SHIFT = 12;              // supertile id above a 12-bit local rectangle
constexpr uint32_t CHUNK = 256;               // supertile entries per level-2 chunk

// Inclusive tile rectangle of a Gaussian, packed as in mgs_projected.rect.
struct TileRect {
    uint32_t x0, y0, x1, y1;
};
MGS_HD TileRect unpack_rect(uint32_t lo, uint32_t hi) {
    return TileRect{lo & 0xFFFFu, lo >> 16, hi & 0xFFFFu, hi >> 16};
}

// Supertiles the rectangle overlaps.
MGS_HD uint32_t rect_n_super(const TileRect &r) {
    return ((r.x1 >> SUPER_SHIFT) - (r.x0 >> SUPER_SHIFT) + 1) * ((r.y1 >> SUPER_SHIFT) - (r.y0 >> SUPER_SHIFT) + 1);
}

// Level-1 key of the rectangle's entry in supertile (sx, sy) with id `id`: the id above the
// part of the rectangle inside that supertile, 3 bits per corner (lx0 | ly0 << 3 | lx1 << 6 |
// ly1 << 9).
MGS_HD uint32_t super_entry_key(uint32_t id, const TileRect &r, uint32_t sx, uint32_t sy) {
    const uint32_t ox = sx << SUPER_SHIFT, oy = sy << SUPER_SHIFT, last = uint32_t(SUPER - 1);
    const uint32_t lx0 = (r.x0 > ox ? r.x0 : ox) - ox, ly0 = (r.y0 > oy ? r.y0 : oy) - oy;
    const uint32_t ex = r.x1 - ox, ey = r.y1 - oy;
    const uint32_t lx1 = ex < last ? ex : last, ly1 = ey < last ? ey : last;
    return (id << ST_KEY_SHIFT) | lx0 | (ly0 << 3) | (lx1 << 6) | (ly1 << 9);
}

// The tiles of the supertile an entry covers, as a 64-bit mask (bit ky * 8 + kx), from the local
// rectangle in the low bits of its level-1 key (never empty: lx0 <= lx1, ly0 <= ly1).
MGS_HD uint64_t local_mask(uint32_t key) {
    const uint32_t lx0 = key & 7u, ly0 = (key >> 3) & 7u, lx1 = (key >> 6) & 7u, ly1 = (key >> 9) & 7u;
    const uint64_t row = uint64_t((2u << lx1) - (1u << lx0));                    // columns lx0 .. lx1
    const uint64_t rows = (0x0101010101010101ull << (8 * ly0)) & (~0ull >> (8 * (SUPER - 1 - ly1)));
    return rows * row;                                                           // no carries: row < 256
}

// Level-2 chunks of the supertile entries: ceil(E_s / CHUNK) per supertile, at most this many
// for E = sum E_s <= capacity entries over S supertiles.
MGS_HD uint64_t bin_max_chunks(uint64_t capacity, uint64_t S) { return capacity / CHUNK + S + 1; }

// ---------------------------------------------------------------- backward pair slots
// Slot of Gaussian g's pair with tile (tx, ty) inside its rectangle, in Gaussian-major order:
// first = the exclusive prefix of the tile counts up to g, then row-major inside the rectangle.
MGS_HD uint64_t pair_slot(uint32_t first, const TileRect &r, uint32_t tx, uint32_t ty) {
    return uint64_t(first) + uint64_t(ty - r.y0) * (r.x1 - r.x0 + 1) + uint64_t(tx - r.x0);
}

}  // namespace mgs

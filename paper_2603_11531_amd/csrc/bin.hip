// mgs_bin / mgs_bin_sorted: tile binning by prefix sums, with no atomics.
//
// Sorted comparison path (mgs_bin_sorted), the usual depth sort:
//   1. exclusive scan of n_tiles            -> first pair slot of every Gaussian, P
//   2. expand: every Gaussian writes (tile << 32 | depth bits, gid) for each tile of
//      its rectangle
//   3. stable LSD radix sort on the 64-bit key (digit histograms per block, a scan of
//      the digit-major histogram, stable scatter); ranks inside a wave come from
//      ballot-matched digits, so nothing is ordered by atomics and the output is
//      bit-identical from run to run
//   4. tile ranges from the sorted keys
//
// Order-independent path (mgs_bin, and the batched render): no depth key and no sort
// of the pairs.  The lists (ascending Gaussian index per tile) are built in two levels,
// over 8x8-tile supertiles and then over the tiles of each supertile (see the comment
// above super_count_kernel).
#include "batch.h"
#include "index_math.h"

namespace mgs {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;     // 4096 elements per block
constexpr int RADIX_THREADS = 256;
constexpr int RADIX_WAVES = RADIX_THREADS / 64;
constexpr int RADIX_ITERS = 16;                           // 64-key steps per wave
constexpr int RADIX_TILE = RADIX_THREADS * RADIX_ITERS;   // 4096 keys per block
constexpr int EXPAND_SMALL = 16;                          // pairs a lane writes on its own
constexpr int RADIX_MAX_BITS = 8;
constexpr int RADIX_MAX_DIGITS = 1 << RADIX_MAX_BITS;
constexpr int RADIX_MAX_GRID = 2048;                      // resident blocks striding over the used ones

constexpr int SUPER_MAX_GRID = 8192;                      // resident blocks striding over the level-2 chunks
constexpr int SUPER_RADIX_ITERS = 4;                      // level-1 sort: 1024 keys per block (a short sort,
constexpr int SUPER_RADIX_TILE = RADIX_THREADS * SUPER_RADIX_ITERS;   // so more, shorter blocks)
// supertiles up to which the plan takes the supertile ranges from the sort's digit totals
constexpr int ST_FROM_DIGITS = 256;
constexpr unsigned PLAN_REPLICAS = 8;                    // blocks of a single-pass chunk plan

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Supertiles of a rectangle of tiles (inclusive bounds packed as in mgs_projected.rect).
__device__ __forceinline__ uint32_t n_super(uint2 r) { return rect_n_super(unpack_rect(r.x, r.y)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive scan over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const unsigned l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (l >= unsigned(o)) v += u;
    }
    return v;
}

// ----------------------------------------------------------------- device scan
// Block-wise exclusive scan of uint32 values in three launches: block totals,
// a one-block scan of the totals (64-bit, the grand total clamped to 2^32-1),
// then the per-block scan with its offset.
__global__ void __launch_bounds__(SCAN_THREADS)
scan_reduce_kernel(const uint32_t *__restrict__ in, int64_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t wsum[SCAN_THREADS / 64];
    const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane_id() == 0) wsum[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) t += wsum[w];
        sums[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(1024)
scan_sums_kernel(uint64_t *__restrict__ sums, int nb, uint32_t *__restrict__ total) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        const uint64_t inc = wave_incl_scan(v);
        if (lane_id() == 63) wsum[threadIdx.x / 64] = inc;
        __syncthreads();
        uint64_t wpre = 0;
        for (int w = 0; w < int(threadIdx.x / 64); ++w) wpre += wsum[w];
        const uint64_t c = carry;
        if (i < nb) sums[i] = c + wpre + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c + wpre + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) {
        const uint64_t t = carry;
        *total = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(t);
    }
}

__global__ void __launch_bounds__(SCAN_THREADS)
scan_apply_kernel(const uint32_t *__restrict__ in, int64_t n, const uint64_t *__restrict__ sums,
                  uint32_t *__restrict__ out) {
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    const uint32_t inc = wave_incl_scan(s);
    if (lane_id() == 63) wsum[threadIdx.x / 64] = inc;
    __syncthreads();
    uint32_t pre = uint32_t(sums[blockIdx.x]);
    for (int w = 0; w < int(threadIdx.x / 64); ++w) pre += wsum[w];
    pre += inc - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = pre;
        pre += v[k];
    }
}

size_t scan_tmp_elems(int64_t n) { return size_t((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

int scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *tmp, uint32_t *total,
                   hipStream_t s) {
    const unsigned nb = unsigned((n + SCAN_TILE - 1) / SCAN_TILE);
    if (nb > 0) {
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, tmp);
        MGS_LAUNCH_CHECK("scan_reduce_kernel");
    }
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, tmp, int(nb), total);
    MGS_LAUNCH_CHECK("scan_sums_kernel");
    if (nb > 0) {
        hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, tmp, out);
        MGS_LAUNCH_CHECK("scan_apply_kernel");
    }
    return MGS_OK;
}

// Exclusive scan of one value per thread over a 256-thread block (all threads call).
template <typename T>
__device__ __forceinline__ T block_excl_scan256(T v, T *s_wsum /* [4] */) {
    const unsigned l = lane_id();
    const int w = threadIdx.x >> 6;
    const T inc = wave_incl_scan(v);
    if (l == 63) s_wsum[w] = inc;
    __syncthreads();
    T pre = 0;
    for (int k = 0; k < w; ++k) pre += s_wsum[k];
    __syncthreads();
    return pre + inc - v;
}

// ----------------------------------------------------------------- pair counts
// Sum of n_tiles over each group of 256 Gaussians (the expand kernel's block).
__global__ void __launch_bounds__(256)
count_reduce_kernel(const uint32_t *__restrict__ ntiles, int64_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t wsum[4];
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    uint64_t v = g < n ? ntiles[g] : 0u;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane_id() == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// ----------------------------------------------------------------- expand
struct TileKey {
    __device__ __forceinline__ uint32_t operator()(uint32_t tile, float) const { return tile; }
};
struct TileDepthKey {
    // depth > near_z > 0 for every listed Gaussian, so its IEEE bits order like the value
    __device__ __forceinline__ uint64_t operator()(uint32_t tile, float depth) const {
        return (uint64_t(tile) << 32) | uint64_t(__float_as_uint(depth));
    }
};

// Global tile id of tile (tx, ty) of Gaussian g's view (the expand kernel's Map interface).
struct GridMap {
    uint32_t tiles_x;
    __device__ __forceinline__ uint32_t base(int64_t, uint32_t &tx) const { tx = tiles_x; return 0u; }
};

// One block per 256 Gaussians.  The block's first pair slot comes from the scanned
// per-block counts; inside the block a wave/LDS scan gives every Gaussian its slot.
// Gaussians with at most EXPAND_SMALL tiles are written by their own lane (row by
// row over the rectangle); larger ones are written by the whole wave.
// Key of a list entry.  Per tile (SHIFT = 0): keyfn(tile, depth).  Per supertile (SHIFT > 0):
// the supertile id above the entry's tile rectangle inside that supertile, 3 bits per corner
// coordinate (lx0 | ly0 << 3 | lx1 << 6 | ly1 << 9): the sort orders by the id alone
// (ST_KEY_SHIFT up) and the level-2 passes read the rectangle from the key instead of
// gathering the Gaussian's rectangle by index.
template <int SHIFT, typename KeyFn>
__device__ __forceinline__ auto entry_key(const KeyFn &keyfn, uint32_t id, float depth, uint2 r, uint32_t sx,
                                          uint32_t sy) {
    if constexpr (SHIFT == 0) {
        return keyfn(id, depth);
    } else {
        static_assert(SHIFT == SUPER_SHIFT, "supertile keys are 8 x 8 tiles");
        return super_entry_key(id, unpack_rect(r.x, r.y), sx, sy);
    }
}

template <typename K, typename KeyFn, typename Map, int SHIFT = 0>
__global__ void __launch_bounds__(256)
expand_kernel(const uint2 *__restrict__ rect, const uint32_t *__restrict__ ntiles,
              const uint64_t *__restrict__ block_first, const float4 *__restrict__ splat, int64_t n,
              Map map, const uint32_t *__restrict__ n_pairs, uint64_t capacity,
              K *__restrict__ keys, uint32_t *__restrict__ vals, KeyFn keyfn,
              const uint32_t *__restrict__ n_live = nullptr) {
    __shared__ uint32_t s_wsum[4];
    if (uint64_t(*n_pairs) > capacity) return;          // block-uniform
    if (n_live && int64_t(*n_live) < n) n = *n_live;    // Gaussians past the live count are not read
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    uint32_t cnt = g < n ? ntiles[g] : 0u;
    if (SHIFT && cnt > 0) cnt = n_super(rect[g]);       // entries per supertile instead of per tile
    const uint32_t excl = block_excl_scan256<uint32_t>(cnt, s_wsum);
    const uint32_t base = uint32_t(block_first[blockIdx.x]) + excl;
    uint2 r = make_uint2(0u, 0u);
    float depth = 0.f;
    uint32_t tbase = 0u, tiles_x = 0u;
    if (cnt > 0) {
        r = rect[g];
        depth = splat[3 * g + 1].w;
        tbase = map.base(g, tiles_x);
    }
    const uint32_t x0 = (r.x & 0xFFFFu) >> SHIFT, y0 = (r.x >> 16) >> SHIFT;
    const uint32_t x1 = (r.y & 0xFFFFu) >> SHIFT, y1 = (r.y >> 16) >> SHIFT;
    if (cnt > 0 && cnt <= uint32_t(EXPAND_SMALL)) {
        uint32_t p = base;
        for (uint32_t ty = y0; ty <= y1; ++ty)
            for (uint32_t tx = x0; tx <= x1; ++tx, ++p) {
                if (!MGS_CHECK(p < capacity, BS_EXPAND_WRITE)) continue;
                keys[p] = entry_key<SHIFT>(keyfn, tbase + ty * tiles_x + tx, depth, r, tx, ty);
                vals[p] = uint32_t(g);
            }
    }
    uint64_t big = __ballot(cnt > uint32_t(EXPAND_SMALL));
    const unsigned l = lane_id();
    while (big) {
        const int j = __builtin_ctzll(big);
        big &= big - 1;
        const uint32_t bj = __shfl(base, j, 64), cj = __shfl(cnt, j, 64);
        const uint32_t xj = __shfl(x0, j, 64), yj = __shfl(y0, j, 64), x1j = __shfl(x1, j, 64);
        const float dj = __shfl(depth, j, 64);
        const uint32_t tbj = __shfl(tbase, j, 64), txj = __shfl(tiles_x, j, 64);
        const uint2 rj = make_uint2(__shfl(r.x, j, 64), __shfl(r.y, j, 64));
        const uint32_t gj = uint32_t(g - l + j);
        const uint32_t wdt = x1j - xj + 1;
        for (uint32_t p = l; p < cj; p += 64) {
            const uint32_t ty = yj + p / wdt, tx = xj + p % wdt;
            if (!MGS_CHECK(uint64_t(bj) + p < capacity, BS_EXPAND_WRITE)) continue;
            keys[bj + p] = entry_key<SHIFT>(keyfn, tbj + ty * txj + tx, dj, rj, tx, ty);
            vals[bj + p] = gj;
        }
    }
}

// ----------------------------------------------------------------- radix sort
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
    return uint32_t(key >> shift) & mask;
}

// Ballot match: lanes of `active` holding the same digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, uint64_t active) {
    uint64_t peers = active;
    for (int b = 0; b < bits; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

// The radix kernels run a bounded grid that strides over the logical 4096-key
// blocks actually in use, ceil(P / 4096), read on the device; the histogram keeps
// the capacity-sized stride `nblocks` but only its first used columns are touched.
template <int ITERS>
__device__ __forceinline__ int used_blocks(uint32_t P) {
    return int((uint64_t(P) + RADIX_THREADS * ITERS - 1) / (RADIX_THREADS * ITERS));
}

// Per-block digit counts, digit-major: counts[d * nblocks + block].
template <typename K, int ITERS = RADIX_ITERS>
__global__ void __launch_bounds__(RADIX_THREADS)
radix_upsweep_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ n_pairs, uint64_t capacity,
                     int shift, int bits, uint32_t *__restrict__ counts, int nblocks) {
    __shared__ uint32_t cnt[RADIX_WAVES][RADIX_MAX_DIGITS];
    const uint32_t P = *n_pairs;
    if (uint64_t(P) > capacity) return;                                   // grid-uniform
    const int nbu = used_blocks<ITERS>(P);
    const int nd = 1 << bits;
    const uint32_t mask = uint32_t(nd - 1);
    const int w = threadIdx.x / 64;
    const unsigned l = lane_id();
    for (int blk = blockIdx.x; blk < nbu; blk += gridDim.x) {
        // all of the wave's loads are issued before the first digit is matched
        const int64_t base = int64_t(blk) * (RADIX_THREADS * ITERS) + w * (ITERS * 64);
        uint32_t d[ITERS];
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int64_t idx = base + it * 64 + l;
            d[it] = idx < int64_t(P) ? digit_of(keys[idx], shift, mask) : 0u;
        }
        for (int i = threadIdx.x; i < RADIX_WAVES * RADIX_MAX_DIGITS; i += RADIX_THREADS) (&cnt[0][0])[i] = 0;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int64_t idx = base + it * 64 + l;
            const bool ok = idx < int64_t(P);
            const uint64_t active = __ballot(ok);
            if (active == 0) break;
            const uint64_t peers = match_digit(d[it], bits, active);
            if (ok && (peers >> l) == 1ull) cnt[w][d[it]] += uint32_t(__popcll(peers));  // highest lane of its digit
        }
        __syncthreads();
        for (int d2 = threadIdx.x; d2 < nd; d2 += RADIX_THREADS)
            counts[int64_t(d2) * nblocks + blk] = cnt[0][d2] + cnt[1][d2] + cnt[2][d2] + cnt[3][d2];
        __syncthreads();
    }
}

// One block per digit: exclusive scan of that digit's per-block counts, and its total.
template <int ITERS = RADIX_ITERS>
__global__ void __launch_bounds__(256)
radix_colscan_kernel(uint32_t *__restrict__ counts, int nblocks, const uint32_t *__restrict__ n_pairs,
                     uint64_t capacity, uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_tot;
    const uint32_t P = *n_pairs;
    if (uint64_t(P) > capacity) return;                                   // grid-uniform
    const int nbu = used_blocks<ITERS>(P);
    uint32_t *row = counts + int64_t(blockIdx.x) * nblocks;
    uint32_t carry = 0;
    constexpr int ITEMS = 8;
    for (int b0 = 0; b0 < nbu; b0 += 256 * ITEMS) {
        const int i0 = b0 + threadIdx.x * ITEMS;
        uint32_t v[ITEMS], s = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            v[k] = i0 + k < nbu ? row[i0 + k] : 0u;
            s += v[k];
        }
        uint32_t pre = block_excl_scan256<uint32_t>(s, s_wsum);
        if (threadIdx.x == 255) s_tot = pre + s;
        __syncthreads();
        pre += carry;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (i0 + k < nbu) row[i0 + k] = pre;
            pre += v[k];
        }
        carry += s_tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter of one block of 256 * ITERS keys: ranks from ballot-matched digits, the
// block's keys reordered by digit in LDS, then written out in runs (coalesced).
template <typename K, int ITERS = RADIX_ITERS>
__global__ void __launch_bounds__(RADIX_THREADS)
radix_downsweep_kernel(const K *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
                       const uint32_t *__restrict__ n_pairs, uint64_t capacity, int shift, int bits,
                       const uint32_t *__restrict__ colscan, const uint32_t *__restrict__ digit_total,
                       int nblocks, K *__restrict__ keys_out, uint32_t *__restrict__ vals_out) {
    __shared__ uint32_t cnt[RADIX_WAVES][RADIX_MAX_DIGITS];
    __shared__ uint32_t s_lstart[RADIX_MAX_DIGITS], s_gstart[RADIX_MAX_DIGITS];
    __shared__ uint32_t s_wsum[4];
    __shared__ K sk[(RADIX_THREADS * ITERS)];
    __shared__ uint32_t sv[(RADIX_THREADS * ITERS)];
    const uint32_t P = *n_pairs;
    if (uint64_t(P) > capacity) return;                                   // grid-uniform
    const int nbu = used_blocks<ITERS>(P);
    const int nd = 1 << bits;
    const uint32_t mask = uint32_t(nd - 1);
    const int t = threadIdx.x;
    const int w = t / 64;
    const unsigned l = lane_id();
    const uint32_t dt = t < nd ? digit_total[t] : 0u;
    const uint32_t dex = block_excl_scan256<uint32_t>(dt, s_wsum);          // contains __syncthreads
    for (int blk = blockIdx.x; blk < nbu; blk += gridDim.x) {
        const int64_t blk0 = int64_t(blk) * (RADIX_THREADS * ITERS);
        const int64_t base = blk0 + w * (ITERS * 64);
        // all of the wave's loads are issued before the first digit is matched
        K key[ITERS];
        uint32_t val[ITERS], rank[ITERS], dig[ITERS];
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int64_t idx = base + it * 64 + l;
            const bool ok = idx < int64_t(P);
            key[it] = ok ? keys_in[idx] : K(0);
            val[it] = ok ? vals_in[idx] : 0u;
        }
        const uint32_t gcol = t < nd ? colscan[int64_t(t) * nblocks + blk] : 0u;
        for (int i = t; i < RADIX_WAVES * RADIX_MAX_DIGITS; i += RADIX_THREADS) (&cnt[0][0])[i] = 0;
        if (t < nd) s_gstart[t] = dex + gcol;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int64_t idx = base + it * 64 + l;
            const bool ok = idx < int64_t(P);
            const uint64_t active = __ballot(ok);
            const uint32_t d = ok ? digit_of(key[it], shift, mask) : 0u;
            dig[it] = d;
            rank[it] = 0;
            if (active != 0) {
                const uint64_t peers = match_digit(d, bits, active);
                const uint32_t before = ok ? cnt[w][d] : 0u;
                rank[it] = before + uint32_t(__popcll(peers & lanemask_lt()));
                __builtin_amdgcn_wave_barrier();
                if (ok && (peers >> l) == 1ull) cnt[w][d] = before + uint32_t(__popcll(peers));
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        uint32_t tot = 0;
        if (t < nd) {
            for (int ww = 0; ww < RADIX_WAVES; ++ww) {
                const uint32_t c = cnt[ww][t];
                cnt[ww][t] = tot;
                tot += c;
            }
        }
        const uint32_t lex = block_excl_scan256<uint32_t>(tot, s_wsum);    // contains __syncthreads
        if (t < nd) s_lstart[t] = lex;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int64_t idx = base + it * 64 + l;
            if (idx < int64_t(P)) {
                const uint32_t lp = s_lstart[dig[it]] + cnt[w][dig[it]] + rank[it];
                sk[lp] = key[it];
                sv[lp] = val[it];
            }
        }
        __syncthreads();
        const int nloc = int(int64_t(P) - blk0 < (RADIX_THREADS * ITERS) ? int64_t(P) - blk0 : (RADIX_THREADS * ITERS));
        for (int lp = t; lp < nloc; lp += RADIX_THREADS) {
            const K k = sk[lp];
            const uint32_t d = digit_of(k, shift, mask);
            const uint32_t dst = s_gstart[d] + uint32_t(lp) - s_lstart[d];
            keys_out[dst] = k;
            vals_out[dst] = sv[lp];
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- tile ranges
// offsets[u] = first pair of tile u, for u = 0 .. n_tiles (offsets[n_tiles] = P).  Element i
// writes the boundaries between its key and the previous one; the boundaries after the
// last key (tiles with no pairs at the end, the sentinel) are spread over all threads.
template <typename K>
__global__ void __launch_bounds__(256)
tile_ranges_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ n_pairs, uint64_t capacity,
                   int shift, uint32_t n_tiles, uint32_t *__restrict__ offsets) {
    const uint32_t P = *n_pairs;
    if (uint64_t(P) > capacity) return;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = tid; i < int64_t(P); i += stride) {
        const int64_t t = int64_t(keys[i] >> shift);
        const int64_t tp = i > 0 ? int64_t(keys[i - 1] >> shift) : -1;
        for (int64_t u = tp + 1; u <= t; ++u) offsets[u] = uint32_t(i);
    }
    const int64_t tl = P > 0 ? int64_t(keys[P - 1] >> shift) : -1;
    for (int64_t u = tl + 1 + tid; u <= int64_t(n_tiles); u += stride) offsets[u] = P;
}

// ----------------------------------------------------------------- two-level binning
// The order-independent lists are built without sorting the tile/Gaussian pairs:
//
//   level 1  every visible Gaussian is listed once per 8x8-tile supertile its rectangle
//            overlaps (about 1.5 entries per Gaussian against about 10 pairs), and the
//            entries are ordered by supertile with the stable radix sort above (one
//            8-bit pass for up to 256 supertiles); a supertile's entries stay in
//            ascending Gaussian order.  An entry's key carries, below the supertile id,
//            the part of the Gaussian's tile rectangle inside that supertile, so level 2
//            reads keys and values in order and gathers nothing by Gaussian index;
//   level 2  a supertile's entries are cut into chunks of CHUNK.  One pass counts,
//            per chunk and per tile of the supertile, the entries whose rectangle
//            covers the tile (ballots over the wave); a column scan over each
//            supertile's chunks and a scan over the tiles give every (chunk, tile) its
//            first slot; a second pass writes the Gaussian indices, ranked inside the
//            chunk by the same ballots.
//
// Every step is a prefix sum or a ballot, so the lists are deterministic and equal to
// the stable tile sort's: ascending Gaussian index per tile.

// Supertile layout of a single view, or of a batch of views (global supertile ids).
struct SuperGrid {
    uint32_t tiles_x, tiles_y, st_x;
    // global id of Gaussian g's supertile (sx, sy) (the expand kernel's Map interface)
    __device__ __forceinline__ uint32_t base(int64_t, uint32_t &stx) const { stx = st_x; return 0u; }
    // supertile s: the view's first global tile, its tiles per row and column, and the
    // supertile's coordinates in the view
    __device__ __forceinline__ void view(uint32_t s, uint32_t &tbase, uint32_t &tw, uint32_t &th, uint32_t &sx,
                                         uint32_t &sy) const {
        tbase = 0u; tw = tiles_x; th = tiles_y; sx = s % st_x; sy = s / st_x;
    }
};
struct SuperBatch {
    const BatchPlan *plan;
    __device__ __forceinline__ uint32_t base(int64_t g, uint32_t &stx) const {
        const int r = find_request(plan->gbase, plan->nreq, uint32_t(g));
        stx = plan->st_x[r];
        return plan->stbase[r];
    }
    __device__ __forceinline__ void view(uint32_t s, uint32_t &tbase, uint32_t &tw, uint32_t &th, uint32_t &sx,
                                         uint32_t &sy) const {
        const int r = find_request(plan->stbase, plan->nreq, s);
        const uint32_t ls = s - plan->stbase[r];
        tbase = plan->tbase[r]; tw = plan->tiles_x[r]; th = plan->tiles_y[r];
        sx = ls % plan->st_x[r]; sy = ls / plan->st_x[r];
    }
};
// Supertiles per row of a single view (the level-1 path from the rectangles is for single views).
inline uint32_t geo_st_x(const SuperGrid &g) { return g.st_x; }
inline uint32_t geo_st_x(const SuperBatch &) { return 0u; }

// Per 256 Gaussians: number of supertile entries and of tile pairs.
__global__ void __launch_bounds__(256)
super_count_kernel(const uint2 *__restrict__ rect, const uint32_t *__restrict__ ntiles, int64_t n,
                   const uint32_t *__restrict__ n_live, uint64_t *__restrict__ sums_e, uint64_t *__restrict__ sums_p) {
    __shared__ uint64_t ws[2][4];
    if (n_live && int64_t(*n_live) < n) n = *n_live;           // Gaussians past the live count are not read
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const uint32_t nt = g < n ? ntiles[g] : 0u;
    uint64_t e = nt > 0 ? n_super(rect[g]) : 0u, p = nt;
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o, 64);
        p += __shfl_xor(p, o, 64);
    }
    if (lane_id() == 0) {
        ws[0][threadIdx.x >> 6] = e;
        ws[1][threadIdx.x >> 6] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sums_e[blockIdx.x] = ws[0][0] + ws[0][1] + ws[0][2] + ws[0][3];
        sums_p[blockIdx.x] = ws[1][0] + ws[1][1] + ws[1][2] + ws[1][3];
    }
}

// Level-1 slots: exclusive scan of the per-256-Gaussian entry counts (in place), their total
// E, and the pair total P (clamped to 2^32 - 1) -> n_pairs; E is written as 0 when
// P > capacity, so nothing after this step does any work.  Chunked scan (see plan_chunks):
// pass 1 writes the chunk totals of both counts, pass 2 the prefixes.
__global__ void __launch_bounds__(1024)
super_sum_kernel(const uint64_t *__restrict__ sums_e, const uint64_t *__restrict__ sums_p, int nb,
                 uint64_t *__restrict__ part_e, uint64_t *__restrict__ part_p) {
    __shared__ uint64_t s_wsum[16];
    const uint32_t nc = plan_chunks(uint64_t(nb));
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const int i0 = int(c) * PLAN_TILE + int(threadIdx.x) * PLAN_ITEMS;
        uint64_t e = 0, p = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            e += i0 + j < nb ? sums_e[i0 + j] : 0u;
            p += i0 + j < nb ? sums_p[i0 + j] : 0u;
        }
        uint64_t te, tp;
        block_scan1024(e, s_wsum, &te);
        block_scan1024(p, s_wsum, &tp);
        if (threadIdx.x == 0) {
            part_e[c] = te;
            part_p[c] = tp;
        }
    }
}

__global__ void __launch_bounds__(1024)
super_scan_kernel(uint64_t *__restrict__ sums_e, const uint64_t *__restrict__ sums_p, int nb,
                  const uint64_t *__restrict__ part_e, const uint64_t *__restrict__ totals /* {E, P} */,
                  uint64_t capacity, uint32_t *__restrict__ e_total, uint32_t *__restrict__ n_pairs) {
    // part_e == NULL: one block walks every chunk with a running carry (few chunks)
    __shared__ uint64_t s_wsum[16];
    const uint32_t nc = plan_chunks(uint64_t(nb));
    uint64_t carry = 0, ptot = 0;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const int i0 = int(c) * PLAN_TILE + int(threadIdx.x) * PLAN_ITEMS;
        uint64_t v[PLAN_ITEMS], sum = 0, psum = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            v[j] = i0 + j < nb ? sums_e[i0 + j] : 0u;
            if (!part_e) psum += i0 + j < nb ? sums_p[i0 + j] : 0u;
            sum += v[j];
        }
        uint64_t tot, ptot_c = 0;
        uint64_t o = block_scan1024(sum, s_wsum, &tot) + (part_e ? part_e[c] : carry);
        if (!part_e) block_scan1024(psum, s_wsum, &ptot_c);
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            if (i0 + j < nb) sums_e[i0 + j] = o;
            o += v[j];
        }
        carry += tot;
        ptot += ptot_c;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t E = part_e ? totals[0] : carry, P = part_e ? totals[1] : ptot;
        const uint32_t p32 = P > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(P);
        *n_pairs = p32;
        *e_total = uint64_t(p32) > capacity ? 0u : uint32_t(E);
    }
}

// Level 2 work list: supertile s has ceil(E_s / CHUNK) chunks starting at chunk sc0[s];
// chunk c covers entries [chunk_lo[c], min(chunk_lo[c] + CHUNK, st_offs[s + 1])) of
// supertile chunk_st[c].  Chunked scan over the supertiles: pass 1 counts each piece's
// chunks, pass 2 writes sc0 and fills the piece's chunks (every thread, binary search of
// the supertiles' chunk prefixes in LDS).
__device__ __forceinline__ uint32_t live_supertiles(const uint32_t *st_count, uint32_t st_host,
                                                    const uint32_t *n_pairs, uint64_t capacity) {
    uint32_t S = st_count ? *st_count : st_host;
    if (S > st_host) S = st_host;
    return uint64_t(*n_pairs) > capacity ? 0u : S;             // lists are not built
}

__global__ void __launch_bounds__(1024)
chunk_sum_kernel(const uint32_t *__restrict__ st_offs, const uint32_t *__restrict__ st_count, uint32_t st_host,
                 const uint32_t *__restrict__ n_pairs, uint64_t capacity, uint64_t *__restrict__ part) {
    __shared__ uint64_t s_wsum[16];
    const uint32_t S = live_supertiles(st_count, st_host, n_pairs, capacity);
    for (uint32_t c = blockIdx.x; c < plan_chunks(st_host); c += gridDim.x) {
        const uint32_t s0 = c * PLAN_TILE + threadIdx.x * PLAN_ITEMS;
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j)
            if (s0 + j < S) cnt += (st_offs[s0 + j + 1] - st_offs[s0 + j] + CHUNK - 1) / CHUNK;
        uint64_t tot;
        block_scan1024(cnt, s_wsum, &tot);
        if (threadIdx.x == 0) part[c] = tot;
    }
}

// The plan for workgroup `bid` of `nblk` (1024 threads; LDS: s_wsum[16], s_pre[PLAN_TILE + 1],
// s_offs[ST_FROM_DIGITS + 1]).
__device__ __forceinline__ void chunk_plan_body(const uint32_t *st_offs, const uint32_t *__restrict__ st_count,
                                                uint32_t st_host, const uint32_t *__restrict__ n_pairs,
                                                uint64_t capacity, const uint64_t *__restrict__ part,
                                                const uint64_t *__restrict__ total, uint32_t *__restrict__ sc0,
                                                uint32_t *__restrict__ chunk_st, uint32_t *__restrict__ chunk_lo,
                                                uint32_t *__restrict__ n_chunks,
                                                const uint32_t *__restrict__ digit_total, uint32_t *st_offs_out,
                                                uint32_t bid, uint32_t nblk, uint64_t *s_wsum, uint32_t *s_pre,
                                                uint32_t *s_offs) {
    // part == NULL (few pieces): every block walks every piece with a running carry and writes
    // every grid-th 1024 chunk entries; block 0 writes the per-supertile outputs
    const uint32_t S = live_supertiles(st_count, st_host, n_pairs, capacity);
    const bool replicated = part == nullptr;
    const bool writer = !replicated || bid == 0;
    // digit_total != NULL (one block, S <= ST_FROM_DIGITS): the supertile sort took a single
    // radix pass over the whole supertile id, so its digit totals are the supertiles' entry
    // counts; their exclusive scan is st_offs, written here instead of by a pass over the keys
    if (digit_total) {
        uint64_t tot;
        const uint32_t v = threadIdx.x < S ? digit_total[threadIdx.x] : 0u;
        const uint32_t pre = uint32_t(block_scan1024(v, s_wsum, &tot));
        if (threadIdx.x <= S && threadIdx.x <= uint32_t(ST_FROM_DIGITS)) {
            s_offs[threadIdx.x] = threadIdx.x < S ? pre : uint32_t(tot);
            if (writer) st_offs_out[threadIdx.x] = threadIdx.x < S ? pre : uint32_t(tot);
        }
        __syncthreads();
    }
    const uint32_t *offs_in = digit_total ? s_offs : st_offs;
    uint32_t carry = 0;
    const uint32_t fill0 = replicated ? bid * 1024u : 0u, fill_step = 1024u * (replicated ? nblk : 1u);
    for (uint32_t c = replicated ? 0u : bid; c < plan_chunks(S); c += replicated ? 1u : nblk) {
        const uint32_t base = c * PLAN_TILE, k0 = threadIdx.x * PLAN_ITEMS, s0 = base + k0;
        uint32_t o[PLAN_ITEMS + 1];
#pragma unroll
        for (int j = 0; j <= PLAN_ITEMS; ++j) o[j] = s0 + j <= S ? offs_in[s0 + j] : 0u;
        uint32_t nc[PLAN_ITEMS], cnt = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            nc[j] = s0 + j < S ? (o[j + 1] - o[j] + CHUNK - 1) / CHUNK : 0u;
            cnt += nc[j];
        }
        uint64_t tot;
        uint32_t q = uint32_t(block_scan1024(cnt, s_wsum, &tot));
        const uint32_t first = part ? uint32_t(part[c]) : carry;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            s_pre[k0 + j] = q;
            if (writer && s0 + j < S) sc0[s0 + j] = first + q;
            q += nc[j];
        }
        if (threadIdx.x == 0) s_pre[PLAN_TILE] = uint32_t(tot);
        __syncthreads();
        const uint32_t ns = min(uint32_t(PLAN_TILE), S - base);
        for (uint32_t i = fill0 + threadIdx.x; i < uint32_t(tot); i += fill_step) {
            const int k = upper_index(s_pre, int(ns), i);
            chunk_st[first + i] = base + k;
            chunk_lo[first + i] = offs_in[base + k] + (i - s_pre[k]) * CHUNK;
        }
        __syncthreads();
        carry += uint32_t(tot);
    }
    if (bid == 0 && threadIdx.x == 0) {
        const uint32_t nct = S == 0 ? 0u : (part ? uint32_t(*total) : carry);
        sc0[S] = nct;
        *n_chunks = nct;
    }
}

__global__ void __launch_bounds__(1024)
chunk_plan_kernel(const uint32_t *st_offs, const uint32_t *__restrict__ st_count, uint32_t st_host,
                  const uint32_t *__restrict__ n_pairs, uint64_t capacity, const uint64_t *__restrict__ part,
                  const uint64_t *__restrict__ total, uint32_t *__restrict__ sc0, uint32_t *__restrict__ chunk_st,
                  uint32_t *__restrict__ chunk_lo, uint32_t *__restrict__ n_chunks,
                  const uint32_t *__restrict__ digit_total, uint32_t *st_offs_out) {
    __shared__ uint64_t s_wsum[16];
    __shared__ uint32_t s_pre[PLAN_TILE + 1];    // first chunk of each supertile of the piece (piece-relative)
    __shared__ uint32_t s_offs[ST_FROM_DIGITS + 1];
    chunk_plan_body(st_offs, st_count, st_host, n_pairs, capacity, part, total, sc0, chunk_st, chunk_lo, n_chunks,
                    digit_total, st_offs_out, blockIdx.x, gridDim.x, s_wsum, s_pre, s_offs);
}

// An entry's covered tiles of its supertile: local_mask (index_math.h).

// 64 x 64 bit transpose across the wave: on return lane k holds, in bit j, bit k of lane j's
// input.  Six butterfly stages; stage s exchanges, between lanes l and l ^ s, the s-bit
// sub-blocks whose bit index and lane index differ in bit s.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
    const unsigned l = lane_id();
    const uint64_t M[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0F0F0F0F0F0F0F0Full,
                           0x00FF00FF00FF00FFull, 0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int sh = 1 << i;
        const uint32_t ylo = __shfl_xor(uint32_t(x), sh, 64), yhi = __shfl_xor(uint32_t(x >> 32), sh, 64);
        const uint64_t y = (uint64_t(yhi) << 32) | ylo;
        x = (l & sh) ? (((y >> sh) & M[i]) | (x & ~M[i])) : ((x & M[i]) | ((y & M[i]) << sh));
    }
    return x;
}

// One chunk: entry threadIdx.x of the chunk (if any) and the tiles of the supertile it covers.
template <typename Geo>
__device__ __forceinline__ void chunk_entry(const uint32_t *__restrict__ vals, const uint32_t *__restrict__ keys,
                                            uint32_t c, const uint32_t *__restrict__ chunk_st,
                                            const uint32_t *__restrict__ chunk_lo,
                                            const uint32_t *__restrict__ st_offs, const Geo &geo, uint32_t &gid,
                                            uint64_t &mask, uint32_t &tbase, uint32_t &tw, uint32_t &th,
                                            uint32_t &sx, uint32_t &sy) {
    const uint32_t s = chunk_st[c];
    const uint32_t lo = chunk_lo[c], hi = min(lo + uint32_t(CHUNK), st_offs[s + 1]);
    geo.view(s, tbase, tw, th, sx, sy);
    const uint32_t i = lo + threadIdx.x;
    mask = 0ull;
    gid = 0u;
    if (i < hi) {
        gid = vals[i];
        mask = local_mask(keys[i]);
    }
}

// Level-2 pass 1: per chunk and tile of its supertile, the number of covering entries
// (after the wave transpose, lane k of a wave holds tile k's membership over the wave's 64
// entries).
template <typename Geo>
__global__ void __launch_bounds__(CHUNK)
chunk_count_kernel(const uint32_t *__restrict__ vals, const uint32_t *__restrict__ keys,
                   const uint32_t *__restrict__ chunk_st, const uint32_t *__restrict__ chunk_lo,
                   const uint32_t *__restrict__ st_offs, const uint32_t *__restrict__ n_chunks, Geo geo,
                   uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_cnt[CHUNK / 64][SUPER_TILES];
    const uint32_t nc = *n_chunks;
    const int w = threadIdx.x >> 6;
    const unsigned l = lane_id();
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        uint32_t gid, tbase, tw, th, sx, sy;
        uint64_t mask;
        chunk_entry(vals, keys, c, chunk_st, chunk_lo, st_offs, geo, gid, mask, tbase, tw, th, sx, sy);
        s_cnt[w][l] = uint32_t(__popcll(wave_transpose64(mask)));
        __syncthreads();
        if (threadIdx.x < SUPER_TILES) {
            const int k = threadIdx.x;
            cnt[size_t(c) * SUPER_TILES + k] = s_cnt[0][k] + s_cnt[1][k] + s_cnt[2][k] + s_cnt[3][k];
        }
        __syncthreads();
    }
}

// Exclusive scan of the per-tile totals -> tile_offsets[0 .. T], skipped on overflow (then
// only n_pairs has been written).  Chunked scan: pass 1 sums, pass 2 writes.
__device__ __forceinline__ uint32_t live_tiles(const uint32_t *t_count, uint32_t t_host) {
    const uint32_t T = t_count ? *t_count : t_host;
    return T > t_host ? t_host : T;
}

__global__ void __launch_bounds__(1024)
tile_sum_kernel(const uint32_t *__restrict__ tile_total, const uint32_t *__restrict__ t_count, uint32_t t_host,
                uint64_t *__restrict__ part) {
    __shared__ uint64_t s_wsum[16];
    const uint32_t T = live_tiles(t_count, t_host);
    for (uint32_t c = blockIdx.x; c < plan_chunks(t_host); c += gridDim.x) {
        const uint32_t t0 = c * PLAN_TILE + threadIdx.x * PLAN_ITEMS;
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) sum += t0 + j < T ? tile_total[t0 + j] : 0u;
        uint64_t tot;
        block_scan1024(sum, s_wsum, &tot);
        if (threadIdx.x == 0) part[c] = tot;
    }
}

__device__ __forceinline__ void tile_scan_body(const uint32_t *__restrict__ tile_total,
                                               const uint32_t *__restrict__ t_count, uint32_t t_host,
                                               const uint32_t *__restrict__ n_pairs, uint64_t capacity,
                                               const uint64_t *__restrict__ part, uint32_t *__restrict__ offs,
                                               uint32_t bid, uint32_t nblk, uint64_t *s_wsum) {
    if (uint64_t(*n_pairs) > capacity) return;                  // grid-uniform
    // part == NULL: one block walks every chunk with a running carry (few chunks)
    const uint32_t T = live_tiles(t_count, t_host);
    uint64_t carry = 0;
    for (uint32_t c = bid; c < plan_chunks(T); c += nblk) {
        const uint32_t t0 = c * PLAN_TILE + threadIdx.x * PLAN_ITEMS;
        uint32_t v[PLAN_ITEMS], sum = 0;
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            v[j] = t0 + j < T ? tile_total[t0 + j] : 0u;
            sum += v[j];
        }
        uint64_t tot;
        uint32_t o = uint32_t(block_scan1024(sum, s_wsum, &tot) + (part ? part[c] : carry));
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            if (t0 + j < T) offs[t0 + j] = o;
            o += v[j];
        }
        carry += tot;
    }
    if (bid == 0 && threadIdx.x == 0) offs[T] = *n_pairs;
}

__global__ void __launch_bounds__(1024)
tile_scan_kernel(const uint32_t *__restrict__ tile_total, const uint32_t *__restrict__ t_count, uint32_t t_host,
                 const uint32_t *__restrict__ n_pairs, uint64_t capacity, const uint64_t *__restrict__ part,
                 uint32_t *__restrict__ offs) {
    __shared__ uint64_t s_wsum[16];
    tile_scan_body(tile_total, t_count, t_host, n_pairs, capacity, part, offs, blockIdx.x, gridDim.x, s_wsum);
}

// Per (supertile, tile of it), one wave each: exclusive scan of the chunk counts in place, and
// the tile's total pair count -> tile_total[global tile] for every tile inside its view.
template <typename Geo>
__global__ void __launch_bounds__(1024)
chunk_colscan_kernel(uint32_t *__restrict__ cnt, const uint32_t *__restrict__ sc0,
                     const uint32_t *__restrict__ st_count, uint32_t st_host, const uint32_t *__restrict__ n_pairs,
                     uint64_t capacity, Geo geo, uint32_t *__restrict__ tile_total) {
    uint32_t S = st_count ? *st_count : st_host;
    if (S > st_host) S = st_host;
    if (uint64_t(*n_pairs) > capacity) S = 0;                  // lists are not built
    const unsigned l = lane_id();
    const uint32_t wpb = blockDim.x >> 6;
    for (uint32_t job = blockIdx.x * wpb + (threadIdx.x >> 6); job < S * SUPER_TILES; job += gridDim.x * wpb) {
        const uint32_t s = job / SUPER_TILES, k = job % SUPER_TILES;
        uint32_t tbase, tw, th, sx, sy;
        geo.view(s, tbase, tw, th, sx, sy);
        const uint32_t tx = sx * SUPER + (k & (SUPER - 1)), ty = sy * SUPER + k / SUPER;
        const uint32_t c0 = sc0[s], c1 = sc0[s + 1];
        uint32_t carry = 0;
        for (uint32_t cb = c0; cb < c1; cb += 64) {
            const uint32_t c = cb + l;
            const uint32_t v = c < c1 ? cnt[size_t(c) * SUPER_TILES + k] : 0u;
            const uint32_t inc = wave_incl_scan(v);
            if (c < c1) cnt[size_t(c) * SUPER_TILES + k] = carry + inc - v;
            carry += __shfl(inc, 63, 64);
        }
        if (l == 0 && tx < tw && ty < th) tile_total[tbase + ty * tw + tx] = carry;
    }
}

// Level-2 pass 2: the Gaussian indices go into the tile lists.  After the wave transpose,
// lane k of wave w holds which of the wave's 64 entries cover tile k.  The chunk's output
// for tile k is one contiguous run of the tile's list (the tile's first slot + the chunk's
// column prefix), the waves' parts in wave order.  The runs are assembled tile by tile in
// LDS (with each pair's tile in a byte map), then copied out by consecutive threads, so the
// global stores are coalesced; a chunk with more than CHUNK_STAGE pairs has its lanes write
// their runs straight to memory.  3,072 staged pairs (19 KB of LDS per workgroup) let eight
// workgroups share a CU (4,096: six); most chunks still fit (8.5 M pairs over ~4,300 chunks on a 1M-Gaussian
// frame).
constexpr int CHUNK_STAGE = 3072;

template <typename Geo>
__global__ void __launch_bounds__(CHUNK)
chunk_write_kernel(const uint32_t *__restrict__ vals, const uint32_t *__restrict__ keys,
                   const uint32_t *__restrict__ chunk_st, const uint32_t *__restrict__ chunk_lo,
                   const uint32_t *__restrict__ st_offs, const uint32_t *__restrict__ n_chunks, Geo geo,
                   const uint32_t *__restrict__ cbase, const uint32_t *__restrict__ offs,
                   const uint32_t *__restrict__ n_pairs, uint64_t capacity, uint32_t *__restrict__ gids) {
    __shared__ uint32_t s_gid[CHUNK / 64][64];
    __shared__ uint32_t s_cnt[CHUNK / 64][SUPER_TILES];
    __shared__ uint32_t s_lw[CHUNK / 64][SUPER_TILES];      // local (chunk) start of wave w's part of tile k
    __shared__ uint32_t s_lpre[SUPER_TILES + 1];            // local start of tile k's run; [64] = total
    __shared__ uint32_t s_first[SUPER_TILES];               // global start of tile k's run
    __shared__ uint32_t s_out[CHUNK_STAGE];
    __shared__ uint8_t s_tile[CHUNK_STAGE];                 // tile of each staged pair
    if (uint64_t(*n_pairs) > capacity) return;              // grid-uniform
    const uint32_t nc = *n_chunks;
    const int w = threadIdx.x >> 6;
    const unsigned l = lane_id();
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        uint32_t gid, tbase, tw, th, sx, sy;
        uint64_t mask;
        // wave 0, one lane per tile of the supertile: the tile's list start plus this chunk's
        // slot in it, loaded before the entries so the two memory latencies overlap
        uint32_t first = 0u;
        if (threadIdx.x < SUPER_TILES) {
            geo.view(chunk_st[c], tbase, tw, th, sx, sy);
            const int k = threadIdx.x;
            const uint32_t tx = sx * SUPER + (k & (SUPER - 1)), ty = sy * SUPER + k / SUPER;
            if (tx < tw && ty < th) first = offs[tbase + ty * tw + tx] + cbase[size_t(c) * SUPER_TILES + k];
        }
        chunk_entry(vals, keys, c, chunk_st, chunk_lo, st_offs, geo, gid, mask, tbase, tw, th, sx, sy);
        s_gid[w][l] = gid;
        uint64_t col = wave_transpose64(mask);
        s_cnt[w][l] = uint32_t(__popcll(col));
        __syncthreads();
        if (threadIdx.x < SUPER_TILES) {                        // wave 0: one lane per tile
            const int k = threadIdx.x;
            const uint32_t ck = s_cnt[0][k] + s_cnt[1][k] + s_cnt[2][k] + s_cnt[3][k];
            uint32_t incl = ck;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = __shfl_up(incl, o, 64);
                if (k >= o) incl += u;
            }
            uint32_t lo = incl - ck;
            s_lpre[k] = lo;
            if (k == 63) s_lpre[64] = incl;
            if (ck > 0) s_first[k] = first;
#pragma unroll
            for (int ww = 0; ww < CHUNK / 64; ++ww) {
                s_lw[ww][k] = lo;
                lo += s_cnt[ww][k];
            }
        }
        __syncthreads();
        const uint32_t L = s_lpre[SUPER_TILES];
        if (L <= uint32_t(CHUNK_STAGE)) {
            // up to four of the lane's entries per step, their LDS reads in flight together
            // (an index past the last entry reads entry 63 and is not stored)
            uint32_t pos = s_lw[w][l];
            while (col) {
                const int j0 = __builtin_ctzll(col);
                col &= col - 1;
                const bool h1 = col != 0ull;
                const int j1 = __builtin_ctzll(col | (1ull << 63));
                col &= col - 1;
                const bool h2 = col != 0ull;
                const int j2 = __builtin_ctzll(col | (1ull << 63));
                col &= col - 1;
                const bool h3 = col != 0ull;
                const int j3 = __builtin_ctzll(col | (1ull << 63));
                col &= col - 1;
                const uint32_t g0 = s_gid[w][j0], g1 = s_gid[w][j1], g2 = s_gid[w][j2], g3 = s_gid[w][j3];
                s_out[pos] = g0;
                s_tile[pos] = uint8_t(l);
                if (h1) { s_out[pos + 1] = g1; s_tile[pos + 1] = uint8_t(l); }
                if (h2) { s_out[pos + 2] = g2; s_tile[pos + 2] = uint8_t(l); }
                if (h3) { s_out[pos + 3] = g3; s_tile[pos + 3] = uint8_t(l); }
                pos += 1u + uint32_t(h1) + uint32_t(h2) + uint32_t(h3);
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < L; i += CHUNK) {
                const int k = s_tile[i];
                const uint32_t dst = s_first[k] + (i - s_lpre[k]);
                if (MGS_CHECK(dst < *n_pairs, BS_LIST_WRITE)) gids[dst] = s_out[i];
            }
        } else if (col) {
            uint32_t pos = s_first[l] + (s_lw[w][l] - s_lpre[l]);
            while (col) {
                const int j = __builtin_ctzll(col);
                col &= col - 1;
                if (MGS_CHECK(pos < *n_pairs, BS_LIST_WRITE)) gids[pos] = s_gid[w][j];
                ++pos;
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- level 1 from the rectangles
// Single view with at most 2^8 supertiles: the supertile entries are counted, placed and
// stably ordered straight from the Gaussians' rectangles, with no entry array in between:
//   super_hist:    per block of L1_GB Gaussians, entries per supertile (digit-major
//                  counts[s * nbg + b]) and the block's pair count;
//   super_colscan: one block per supertile: exclusive scan of its counts over the Gaussian
//                  blocks, and its total; block 0 also sums the pair counts -> n_pairs;
//   super_scatter: per Gaussian block, its entries staged in LDS in Gaussian order (a
//                  Gaussian's supertiles row by row), ranked by supertile with ballot-matched
//                  digits as in the radix downsweep and written out in runs.
// The result is the one-pass supertile sort of the expanded entries: per supertile, its
// entries in ascending Gaussian index.
constexpr int L1_GPT = 4;                          // Gaussians per thread
constexpr int L1_GB = 256 * L1_GPT;                // Gaussians per block
// 8 steps (110 VGPRs, 24 KB of LDS) keep four workgroups on a CU, one wave per SIMD each, so a
// 1M-Gaussian scene's 977 workgroups run in one round; 16 steps held three
constexpr int L1_ITERS = 8;                        // 64-entry steps per wave and round
constexpr uint32_t L1_STAGE = 256u * L1_ITERS;     // entries staged per round
constexpr uint32_t L1_SMALL = 4;                   // supertiles a lane handles alone; larger: the wave

__device__ __forceinline__ void super_rect(uint2 r, uint32_t &x0, uint32_t &y0, uint32_t &x1, uint32_t &y1) {
    x0 = (r.x & 0xFFFFu) >> SUPER_SHIFT;
    y0 = (r.x >> 16) >> SUPER_SHIFT;
    x1 = (r.y & 0xFFFFu) >> SUPER_SHIFT;
    y1 = (r.y >> 16) >> SUPER_SHIFT;
}

__global__ void __launch_bounds__(256)
super_hist_kernel(const uint2 *__restrict__ rect, const uint32_t *__restrict__ ntiles, int64_t n, uint32_t st_x,
                  uint32_t S, uint32_t nbg, uint32_t *__restrict__ counts, uint64_t *__restrict__ psum) {
    __shared__ uint32_t s_h[RADIX_MAX_DIGITS];
    __shared__ uint64_t s_p[4];
    for (int i = threadIdx.x; i < RADIX_MAX_DIGITS; i += 256) s_h[i] = 0u;
    __syncthreads();
    const uint32_t b = blockIdx.x;
    const int64_t g0 = int64_t(b) * L1_GB + int64_t(threadIdx.x) * L1_GPT;
    uint64_t p = 0;
    const unsigned l = lane_id();
#pragma unroll
    for (int j = 0; j < L1_GPT; ++j) {
        const int64_t g = g0 + j;
        const uint32_t nt = g < n ? ntiles[g] : 0u;
        p += nt;
        uint32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0, ec = 0;
        if (nt > 0) {
            super_rect(rect[g], x0, y0, x1, y1);
            ec = (x1 - x0 + 1) * (y1 - y0 + 1);
        }
        // counts are order-free: LDS atomics.  Up to L1_SMALL supertiles a lane adds its own;
        // the wave adds a larger footprint's together, one supertile per lane
        if (ec > 0 && ec <= L1_SMALL) {
            for (uint32_t sy = y0; sy <= y1; ++sy)
                for (uint32_t sx = x0; sx <= x1; ++sx) {
                    const uint32_t id = sy * st_x + sx;
                    if (MGS_CHECK(id < S, BS_RECT_GRID)) atomicAdd(&s_h[id], 1u);
                }
        }
        for (uint64_t big = __ballot(ec > L1_SMALL); big; big &= big - 1) {
            const int src = __builtin_ctzll(big);
            const uint32_t bx0 = __shfl(x0, src, 64), by0 = __shfl(y0, src, 64), bx1 = __shfl(x1, src, 64);
            const uint32_t bc = __shfl(ec, src, 64), wdt = bx1 - bx0 + 1;
            for (uint32_t k = l; k < bc; k += 64) {
                const uint32_t id = (by0 + k / wdt) * st_x + bx0 + k % wdt;
                if (MGS_CHECK(id < S, BS_RECT_GRID)) atomicAdd(&s_h[id], 1u);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if (lane_id() == 0) s_p[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) psum[b] = s_p[0] + s_p[1] + s_p[2] + s_p[3];
    for (uint32_t sid = threadIdx.x; sid < S; sid += 256) counts[size_t(sid) * nbg + b] = s_h[sid];
}

__global__ void __launch_bounds__(1024)
super_colscan_kernel(uint32_t *__restrict__ counts, const uint64_t *__restrict__ psum, uint32_t nbg,
                     uint32_t *__restrict__ digit_total, uint32_t *__restrict__ n_pairs) {
    __shared__ uint64_t s_wsum[16];
    uint32_t *row = counts + size_t(blockIdx.x) * nbg;
    uint64_t carry = 0;
    constexpr int ITEMS = 4;
    for (uint32_t b0 = 0; b0 < nbg; b0 += 1024 * ITEMS) {
        const uint32_t i0 = b0 + threadIdx.x * ITEMS;
        uint32_t v[ITEMS], sm = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            v[k] = i0 + k < nbg ? row[i0 + k] : 0u;
            sm += v[k];
        }
        uint64_t tot;
        uint32_t pre = uint32_t(block_scan1024(sm, s_wsum, &tot) + carry);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (i0 + k < nbg) row[i0 + k] = pre;
            pre += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = uint32_t(carry);
    if (blockIdx.x == 0) {                             // block-uniform: the pair total
        uint64_t p = 0;
        for (uint32_t i = threadIdx.x; i < nbg; i += 1024) p += psum[i];
        uint64_t P;
        block_scan1024(p, s_wsum, &P);
        if (threadIdx.x == 0) *n_pairs = P > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(P);
    }
}

__global__ void __launch_bounds__(256)
super_scatter_kernel(const uint2 *__restrict__ rect, const uint32_t *__restrict__ ntiles, int64_t n, uint32_t st_x,
                     uint32_t S, int bits, uint32_t nbg, const uint32_t *__restrict__ colscan,
                     const uint32_t *__restrict__ digit_total, const uint32_t *__restrict__ n_pairs,
                     uint64_t capacity, uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out) {
    __shared__ uint32_t cnt[RADIX_WAVES][RADIX_MAX_DIGITS];
    __shared__ uint32_t s_lstart[RADIX_MAX_DIGITS], s_gstart[RADIX_MAX_DIGITS], s_rtot[RADIX_MAX_DIGITS];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_eb;
    __shared__ uint32_t sk[L1_STAGE], sv[L1_STAGE];
    if (uint64_t(*n_pairs) > capacity) return;                           // block-uniform: no lists
    const uint32_t b = blockIdx.x;
    const int t = threadIdx.x, w = t >> 6;
    const unsigned l = lane_id();
    const uint32_t mask = (1u << bits) - 1u;
    // this thread's Gaussians (contiguous indices) and their entry counts; every global load of
    // the block is issued before the first scan waits on any
    const int64_t g0 = int64_t(b) * L1_GB + int64_t(t) * L1_GPT;
    uint2 r[L1_GPT];
    uint32_t ec[L1_GPT], esum = 0;
#pragma unroll
    for (int j = 0; j < L1_GPT; ++j) {
        const int64_t g = g0 + j;
        r[j] = g < n ? rect[g] : make_uint2(0u, 0u);
        ec[j] = g < n ? ntiles[g] : 0u;
    }
    const uint32_t dt = uint32_t(t) < S ? digit_total[t] : 0u;
    const uint32_t gcol = uint32_t(t) < S ? colscan[size_t(t) * nbg + b] : 0u;
#pragma unroll
    for (int j = 0; j < L1_GPT; ++j) {
        ec[j] = ec[j] > 0 ? n_super(r[j]) : 0u;
        esum += ec[j];
    }
    {
        const uint32_t dex = block_excl_scan256<uint32_t>(dt, s_wsum);  // contains __syncthreads
        s_gstart[t] = uint32_t(t) < S ? dex + gcol : 0u;
    }
    const uint32_t ebase = block_excl_scan256<uint32_t>(esum, s_wsum);
    if (t == 255) s_eb = ebase + esum;
    __syncthreads();
    const uint32_t Eb = s_eb;
    for (uint32_t r0 = 0; r0 < Eb; r0 += L1_STAGE) {                    // block-uniform rounds
        const uint32_t rn = Eb - r0 < L1_STAGE ? Eb - r0 : L1_STAGE;
        // stage the round's entries in Gaussian order
        uint32_t e = ebase;
#pragma unroll
        for (int j = 0; j < L1_GPT; ++j) {
            const uint32_t c = ec[j];
            const bool in_round = c > 0 && e < r0 + rn && e + c > r0;
            uint32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0;
            if (in_round) super_rect(r[j], x0, y0, x1, y1);
            if (in_round && c <= L1_SMALL) {
                const uint32_t wdt = x1 - x0 + 1;
                const uint32_t k0 = e < r0 ? r0 - e : 0u, k1 = e + c > r0 + rn ? r0 + rn - e : c;
                for (uint32_t k = k0; k < k1; ++k) {
                    const uint32_t sx = x0 + k % wdt, sy = y0 + k / wdt;
                    sk[e + k - r0] = super_entry_key(sy * st_x + sx, unpack_rect(r[j].x, r[j].y), sx, sy);
                    sv[e + k - r0] = uint32_t(g0 + j);
                }
            }
            // a larger footprint: the wave writes its entries together, one per lane
            for (uint64_t big = __ballot(in_round && c > L1_SMALL); big; big &= big - 1) {
                const int src = __builtin_ctzll(big);
                const uint32_t be = __shfl(e, src, 64), bc = __shfl(c, src, 64);
                const uint32_t bx0 = __shfl(x0, src, 64), by0 = __shfl(y0, src, 64), bx1 = __shfl(x1, src, 64);
                const uint2 br = make_uint2(__shfl(r[j].x, src, 64), __shfl(r[j].y, src, 64));
                const uint32_t bg = uint32_t(__shfl(uint32_t(g0 + j), src, 64)), wdt = bx1 - bx0 + 1;
                const uint32_t k0 = be < r0 ? r0 - be : 0u, k1 = be + bc > r0 + rn ? r0 + rn - be : bc;
                for (uint32_t k = k0 + l; k < k1; k += 64) {
                    const uint32_t sx = bx0 + k % wdt, sy = by0 + k / wdt;
                    sk[be + k - r0] = super_entry_key(sy * st_x + sx, unpack_rect(br.x, br.y), sx, sy);
                    sv[be + k - r0] = bg;
                }
            }
            e += c;
        }
        for (int i = t; i < RADIX_WAVES * RADIX_MAX_DIGITS; i += 256) (&cnt[0][0])[i] = 0u;
        __syncthreads();
        // rank by supertile: the round's entries split evenly, in order, over the four waves
        // (wave w takes [w * seg, (w + 1) * seg), seg a multiple of 64)
        uint32_t key[L1_ITERS], val[L1_ITERS], rank[L1_ITERS], dig[L1_ITERS];
        const uint32_t nit = (rn + 255u) / 256u, seg = 64u * nit;
        const uint32_t base = uint32_t(w) * seg, wend = base + seg < rn ? base + seg : rn;
#pragma unroll
        for (int it = 0; it < L1_ITERS; ++it) {
            const uint32_t idx = base + uint32_t(it) * 64u + l;
            const bool ok = uint32_t(it) < nit && idx < wend;
            key[it] = ok ? sk[idx] : 0u;
            val[it] = ok ? sv[idx] : 0u;
        }
#pragma unroll
        for (int it = 0; it < L1_ITERS; ++it) {
            if (uint32_t(it) >= nit) break;                              // wave-uniform
            const uint32_t idx = base + uint32_t(it) * 64u + l;
            const bool ok = idx < wend;
            const uint64_t active = __ballot(ok);
            const uint32_t d = ok ? (key[it] >> ST_KEY_SHIFT) & mask : 0u;
            dig[it] = d;
            rank[it] = 0;
            if (active != 0) {
                const uint64_t peers = match_digit(d, bits, active);
                const uint32_t before = ok ? cnt[w][d] : 0u;
                rank[it] = before + uint32_t(__popcll(peers & lanemask_lt()));
                __builtin_amdgcn_wave_barrier();
                if (ok && (peers >> l) == 1ull) cnt[w][d] = before + uint32_t(__popcll(peers));
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int ww = 0; ww < RADIX_WAVES; ++ww) {
            const uint32_t c = cnt[ww][t];
            cnt[ww][t] = tot;
            tot += c;
        }
        const uint32_t lex = block_excl_scan256<uint32_t>(tot, s_wsum);  // contains __syncthreads
        s_lstart[t] = lex;
        s_rtot[t] = tot;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < L1_ITERS; ++it) {
            const uint32_t idx = base + uint32_t(it) * 64u + l;
            if (uint32_t(it) < nit && idx < wend) {
                const uint32_t lp = s_lstart[dig[it]] + cnt[w][dig[it]] + rank[it];
                sk[lp] = key[it];
                sv[lp] = val[it];
            }
        }
        __syncthreads();
        for (uint32_t lp = t; lp < rn; lp += 256) {
            const uint32_t k = sk[lp];
            const uint32_t d = (k >> ST_KEY_SHIFT) & mask;
            const uint32_t dst = s_gstart[d] + lp - s_lstart[d];
            if (MGS_CHECK(uint64_t(dst) < capacity, BS_EXPAND_WRITE)) {
                keys_out[dst] = k;
                vals_out[dst] = sv[lp];
            }
        }
        __syncthreads();
        s_gstart[t] += s_rtot[t];                  // the next round's entries follow this round's
        __syncthreads();
    }
}

// ----------------------------------------------------------------- host side
inline int bits_for(uint64_t v) {
    int b = 0;
    while ((uint64_t(1) << b) < v) ++b;
    return b;
}

struct BinLayout {
    size_t off_sums, off_keys0, off_keys1, off_vals1, off_hist, off_dtot, total;
    int nblocks, nsums;
};

template <typename K>
BinLayout bin_layout(int64_t n, uint64_t capacity) {
    BinLayout L;
    const int64_t nb = int64_t((capacity + RADIX_TILE - 1) / RADIX_TILE);
    L.nblocks = int(nb > 0 ? nb : 1);
    L.nsums = int((n + 255) / 256) + 1;
    const size_t cap = size_t(capacity > 0 ? capacity : 1);
    size_t o = 0;
    L.off_sums = o;  o = align_up(o + size_t(L.nsums) * 8, 256);
    L.off_keys0 = o; o = align_up(o + cap * sizeof(K), 256);
    L.off_keys1 = o; o = align_up(o + cap * sizeof(K), 256);
    L.off_vals1 = o; o = align_up(o + cap * 4, 256);
    L.off_hist = o;  o = align_up(o + size_t(RADIX_MAX_DIGITS) * L.nblocks * 4, 256);
    L.off_dtot = o;  o = align_up(o + RADIX_MAX_DIGITS * 4, 256);
    L.total = o;
    return L;
}

template <typename K, typename KeyFn, typename Map>
int bin_impl(const mgs_projected *proj, int64_t n, Map map, uint32_t T, void *ws, size_t ws_bytes,
             uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity, uint32_t *n_pairs,
             hipStream_t s, int key_bits, int range_shift) {
    int rc;
    MGS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if ((rc = check_projected(proj, n)) != MGS_OK) return rc;
    MGS_REQUIRE(T > 0, "bad tile grid");
    MGS_REQUIRE(tile_offsets && n_pairs, "tile_offsets / n_pairs is NULL");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity must be < 2^32 - 1");
    MGS_REQUIRE(capacity == 0 || gids, "gids is NULL");
    MGS_REQUIRE(ws && aligned(ws, 256), "workspace must be non-NULL and 256-byte aligned");
    const BinLayout L = bin_layout<K>(n, capacity);
    MGS_REQUIRE(ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    char *w = static_cast<char *>(ws);
    uint64_t *sums = reinterpret_cast<uint64_t *>(w + L.off_sums);
    K *k0 = reinterpret_cast<K *>(w + L.off_keys0);
    K *k1 = reinterpret_cast<K *>(w + L.off_keys1);
    uint32_t *v1 = reinterpret_cast<uint32_t *>(w + L.off_vals1);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + L.off_hist);
    uint32_t *dtot = reinterpret_cast<uint32_t *>(w + L.off_dtot);
    const unsigned nb256 = unsigned((n + 255) / 256);

    // 1. pair slots: per-256-Gaussian counts, scanned (the grand total is P)
    if (nb256 > 0) {
        hipLaunchKernelGGL(count_reduce_kernel, dim3(nb256), dim3(256), 0, s, proj->n_tiles, n, sums);
        MGS_LAUNCH_CHECK("count_reduce_kernel");
    }
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, int(nb256), n_pairs);
    MGS_LAUNCH_CHECK("scan_sums_kernel");
    // 2. expand
    const int npass = (key_bits + RADIX_MAX_BITS - 1) / RADIX_MAX_BITS;
    K *kin = k0, *kout = k1;
    uint32_t *vbuf[2] = {gids, v1};
    uint32_t *vin = vbuf[npass % 2];
    if (nb256 > 0) {
        hipLaunchKernelGGL((expand_kernel<K, KeyFn, Map>), dim3(nb256), dim3(256), 0, s,
                           reinterpret_cast<const uint2 *>(proj->rect), proj->n_tiles, sums,
                           reinterpret_cast<const float4 *>(proj->splat), n, map, n_pairs,
                           capacity, kin, vin, KeyFn());
        MGS_LAUNCH_CHECK("expand_kernel");
    }
    // 3. radix passes (digits of at most 8 bits, spread evenly)
    if (capacity > 0) {
        const unsigned grid = unsigned(L.nblocks < RADIX_MAX_GRID ? L.nblocks : RADIX_MAX_GRID);
        int shift = 0;
        for (int p = 0; p < npass; ++p) {
            const int bits = (key_bits - shift + (npass - p) - 1) / (npass - p);
            uint32_t *vout = vbuf[(npass - 1 - p) % 2];
            hipLaunchKernelGGL((radix_upsweep_kernel<K>), dim3(grid), dim3(RADIX_THREADS), 0, s, kin,
                               n_pairs, capacity, shift, bits, hist, L.nblocks);
            MGS_LAUNCH_CHECK("radix_upsweep_kernel");
            hipLaunchKernelGGL(radix_colscan_kernel<>, dim3(1u << bits), dim3(256), 0, s, hist, L.nblocks, n_pairs,
                               capacity, dtot);
            MGS_LAUNCH_CHECK("radix_colscan_kernel");
            hipLaunchKernelGGL((radix_downsweep_kernel<K>), dim3(grid), dim3(RADIX_THREADS), 0, s, kin,
                               vin, n_pairs, capacity, shift, bits, hist, dtot, L.nblocks, kout, vout);
            MGS_LAUNCH_CHECK("radix_downsweep_kernel");
            K *tk = kin; kin = kout; kout = tk;
            vin = vout;
            shift += bits;
        }
    }
    // 4. ranges
    const uint64_t rblocks = (capacity + 1 + 255) / 256;
    hipLaunchKernelGGL((tile_ranges_kernel<K>), dim3(unsigned(rblocks < 4096 ? rblocks : 4096)), dim3(256), 0, s, kin,
                       n_pairs, capacity, range_shift, T, tile_offsets);
    MGS_LAUNCH_CHECK("tile_ranges_kernel");
    return MGS_OK;
}

// Two-level order-independent binning (see the comment above super_count_kernel).
struct Bin2Layout {
    size_t sums_e, sums_p, etot, keys0, keys1, vals0, vals1, hist, hist_g, dtot, st_offs, sc0, chunk_st, chunk_lo,
        nch, cnt, ttot, part_e, part_p, part_c, part_t, totals, total;
    int nblocks;
    uint32_t chunks_max;
};

inline Bin2Layout bin2_layout(int64_t n, uint32_t st_max, uint32_t t_max, uint64_t capacity) {
    Bin2Layout L;
    const size_t cap = size_t(capacity > 0 ? capacity : 1);     // entries <= pairs <= capacity
    const int64_t nb = int64_t((cap + SUPER_RADIX_TILE - 1) / SUPER_RADIX_TILE);
    L.nblocks = int(nb > 0 ? nb : 1);
    L.chunks_max = uint32_t(bin_max_chunks(cap, st_max));
    const size_t nsums = size_t((n + 255) / 256) + 1;
    size_t o = 0;
    L.sums_e = o;   o = align_up(o + nsums * 8, 256);
    L.sums_p = o;   o = align_up(o + nsums * 8, 256);
    L.etot = o;     o = align_up(o + 16, 256);
    L.keys0 = o;    o = align_up(o + cap * 4, 256);
    L.keys1 = o;    o = align_up(o + cap * 4, 256);
    L.vals0 = o;    o = align_up(o + cap * 4, 256);
    L.vals1 = o;    o = align_up(o + cap * 4, 256);
    L.hist = o;     o = align_up(o + size_t(RADIX_MAX_DIGITS) * L.nblocks * 4, 256);
    L.hist_g = o;   o = align_up(o + size_t(RADIX_MAX_DIGITS) * (size_t((n + L1_GB - 1) / L1_GB) + 1) * 4, 256);
    L.dtot = o;     o = align_up(o + RADIX_MAX_DIGITS * 4, 256);
    L.st_offs = o;  o = align_up(o + (size_t(st_max) + 1) * 4, 256);
    L.sc0 = o;      o = align_up(o + (size_t(st_max) + 1) * 4, 256);
    L.chunk_st = o; o = align_up(o + size_t(L.chunks_max) * 4, 256);
    L.chunk_lo = o; o = align_up(o + size_t(L.chunks_max) * 4, 256);
    L.nch = o;      o = align_up(o + 16, 256);
    L.cnt = o;      o = align_up(o + size_t(L.chunks_max) * SUPER_TILES * 4, 256);
    L.ttot = o;     o = align_up(o + size_t(t_max) * 4, 256);
    L.part_e = o;   o = align_up(o + (size_t(plan_chunks(nsums)) + 1) * 8, 256);
    L.part_p = o;   o = align_up(o + (size_t(plan_chunks(nsums)) + 1) * 8, 256);
    L.part_c = o;   o = align_up(o + (size_t(plan_chunks(st_max)) + 1) * 8, 256);
    L.part_t = o;   o = align_up(o + (size_t(plan_chunks(t_max)) + 1) * 8, 256);
    L.totals = o;   o = align_up(o + 4 * 8, 256);
    L.total = o;
    return L;
}

// n_live / st_count / t_count: device-side Gaussian / supertile / tile counts (batches), NULL
// for a single view (then n / st_max / T are exact).
template <typename Geo>
int bin2_impl(const mgs_projected *proj, int64_t n, const uint32_t *n_live, Geo geo, uint32_t st_max,
              const uint32_t *st_count, uint32_t T, const uint32_t *t_count, void *ws, size_t ws_bytes,
              uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity, uint32_t *n_pairs, hipStream_t s) {
    int rc;
    MGS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if ((rc = check_projected(proj, n)) != MGS_OK) return rc;
    MGS_REQUIRE(T > 0 && st_max > 0, "bad tile grid");
    MGS_REQUIRE(st_max < (1u << (32 - ST_KEY_SHIFT)), "2^%d or more supertiles", 32 - ST_KEY_SHIFT);
    MGS_REQUIRE(tile_offsets && n_pairs, "tile_offsets / n_pairs is NULL");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity must be < 2^32 - 1");
    MGS_REQUIRE(capacity == 0 || gids, "gids is NULL");
    MGS_REQUIRE(ws && aligned(ws, 256), "workspace must be non-NULL and 256-byte aligned");
    const Bin2Layout L = bin2_layout(n, st_max, T, capacity);
    MGS_REQUIRE(ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    char *w = static_cast<char *>(ws);
    uint64_t *sums_e = reinterpret_cast<uint64_t *>(w + L.sums_e);
    uint64_t *sums_p = reinterpret_cast<uint64_t *>(w + L.sums_p);
    uint32_t *etot = reinterpret_cast<uint32_t *>(w + L.etot);
    uint32_t *keys[2] = {reinterpret_cast<uint32_t *>(w + L.keys0), reinterpret_cast<uint32_t *>(w + L.keys1)};
    uint32_t *vals[2] = {reinterpret_cast<uint32_t *>(w + L.vals0), reinterpret_cast<uint32_t *>(w + L.vals1)};
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + L.hist);
    uint32_t *dtot = reinterpret_cast<uint32_t *>(w + L.dtot);
    uint32_t *st_offs = reinterpret_cast<uint32_t *>(w + L.st_offs);
    uint32_t *sc0 = reinterpret_cast<uint32_t *>(w + L.sc0);
    uint32_t *chunk_st = reinterpret_cast<uint32_t *>(w + L.chunk_st);
    uint32_t *chunk_lo = reinterpret_cast<uint32_t *>(w + L.chunk_lo);
    uint32_t *nch = reinterpret_cast<uint32_t *>(w + L.nch);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(w + L.cnt);
    uint32_t *ttot = reinterpret_cast<uint32_t *>(w + L.ttot);
    uint64_t *part_e = reinterpret_cast<uint64_t *>(w + L.part_e);
    uint64_t *part_p = reinterpret_cast<uint64_t *>(w + L.part_p);
    uint64_t *part_c = reinterpret_cast<uint64_t *>(w + L.part_c);
    uint64_t *part_t = reinterpret_cast<uint64_t *>(w + L.part_t);
    uint64_t *totals = reinterpret_cast<uint64_t *>(w + L.totals);     // {E, P, chunks, -}
    const uint2 *rect = reinterpret_cast<const uint2 *>(proj->rect);
    const unsigned nb256 = unsigned((n + 255) / 256);

    const int key_bits = bits_for(st_max) > 0 ? bits_for(st_max) : 1;
    const int npass = (key_bits + RADIX_MAX_BITS - 1) / RADIX_MAX_BITS;
    int cur = 0;
    // a single view with few supertiles: level 1 straight from the rectangles (super_hist,
    // super_colscan, super_scatter); otherwise entry counts, their scan, the entries and a
    // radix sort of them by supertile
    const bool direct = n_live == nullptr && st_count == nullptr && t_count == nullptr && capacity > 0 &&
                        st_max <= uint32_t(RADIX_MAX_DIGITS) && st_max <= uint32_t(ST_FROM_DIGITS);
    if (direct) {
        const uint32_t nbg = uint32_t((n + L1_GB - 1) / L1_GB);
        uint32_t *hist_g = reinterpret_cast<uint32_t *>(w + L.hist_g);
        const uint32_t st_x = geo_st_x(geo);
        if (nbg > 0) {
            hipLaunchKernelGGL(super_hist_kernel, dim3(nbg), dim3(256), 0, s, rect, proj->n_tiles, n, st_x, st_max,
                               nbg, hist_g, sums_p);
            MGS_LAUNCH_CHECK("super_hist_kernel");
        }
        hipLaunchKernelGGL(super_colscan_kernel, dim3(st_max), dim3(1024), 0, s, hist_g,
                           static_cast<const uint64_t *>(sums_p), nbg, dtot, n_pairs);
        MGS_LAUNCH_CHECK("super_colscan_kernel");
        if (nbg > 0) {
            hipLaunchKernelGGL(super_scatter_kernel, dim3(nbg), dim3(256), 0, s, rect, proj->n_tiles, n, st_x, st_max,
                               key_bits, nbg, static_cast<const uint32_t *>(hist_g), static_cast<const uint32_t *>(dtot),
                               static_cast<const uint32_t *>(n_pairs), capacity, keys[0], vals[0]);
            MGS_LAUNCH_CHECK("super_scatter_kernel");
        }
    } else {
        // level 1: entry counts (and the pair total P), their scan, the entries, the supertile sort
        if (nb256 > 0) {
            hipLaunchKernelGGL(super_count_kernel, dim3(nb256), dim3(256), 0, s, rect, proj->n_tiles, n, n_live, sums_e,
                               sums_p);
            MGS_LAUNCH_CHECK("super_count_kernel");
        }
        const uint32_t nce = plan_chunks(nb256);
        if (nce <= PLAN_ONE_BLOCK) {                 // few chunks: one block with a running carry
            hipLaunchKernelGGL(super_scan_kernel, dim3(1), dim3(1024), 0, s, sums_e, sums_p, int(nb256),
                               static_cast<const uint64_t *>(nullptr), static_cast<const uint64_t *>(nullptr), capacity,
                               etot, n_pairs);
        } else {
            hipLaunchKernelGGL(super_sum_kernel, dim3(plan_grid(nce)), dim3(1024), 0, s, sums_e, sums_p, int(nb256),
                               part_e, part_p);
            MGS_LAUNCH_CHECK("super_sum_kernel");
            hipLaunchKernelGGL(part_scan_kernel<>, dim3(1), dim3(1024), 0, s, part_e, part_p, nce, totals, totals + 1);
            MGS_LAUNCH_CHECK("part_scan_kernel");
            hipLaunchKernelGGL(super_scan_kernel, dim3(plan_grid(nce)), dim3(1024), 0, s, sums_e, sums_p, int(nb256),
                               part_e, totals, capacity, etot, n_pairs);
        }
        MGS_LAUNCH_CHECK("super_scan_kernel");
        if (nb256 > 0) {
            hipLaunchKernelGGL((expand_kernel<uint32_t, TileKey, Geo, SUPER_SHIFT>), dim3(nb256), dim3(256), 0, s, rect,
                               proj->n_tiles, sums_e, reinterpret_cast<const float4 *>(proj->splat), n, geo, n_pairs,
                               capacity, keys[0], vals[0], TileKey(), n_live);
            MGS_LAUNCH_CHECK("expand_kernel<supertile>");
        }
        if (capacity > 0) {
            const unsigned grid = unsigned(L.nblocks < RADIX_MAX_GRID ? L.nblocks : RADIX_MAX_GRID);
            int shift = ST_KEY_SHIFT;                        // the local rectangle below the id is not sorted
            for (int p = 0; p < npass; ++p) {
                const int bits = (key_bits - (shift - ST_KEY_SHIFT) + (npass - p) - 1) / (npass - p);
                hipLaunchKernelGGL((radix_upsweep_kernel<uint32_t, SUPER_RADIX_ITERS>), dim3(grid), dim3(RADIX_THREADS), 0,
                                   s, keys[cur], etot, capacity, shift, bits, hist, L.nblocks);
                MGS_LAUNCH_CHECK("radix_upsweep_kernel");
                hipLaunchKernelGGL(radix_colscan_kernel<SUPER_RADIX_ITERS>, dim3(1u << bits), dim3(256), 0, s, hist,
                                   L.nblocks, etot, capacity, dtot);
                MGS_LAUNCH_CHECK("radix_colscan_kernel");
                hipLaunchKernelGGL((radix_downsweep_kernel<uint32_t, SUPER_RADIX_ITERS>), dim3(grid), dim3(RADIX_THREADS), 0,
                                   s, keys[cur],
                                   vals[cur], etot, capacity, shift, bits, hist, dtot, L.nblocks, keys[cur ^ 1],
                                   vals[cur ^ 1]);
                MGS_LAUNCH_CHECK("radix_downsweep_kernel");
                cur ^= 1;
                shift += bits;
            }
        }
    }
    // supertile ranges: from the sort's digit totals when one radix pass covered the whole id
    // (the plan scans them), else from the sorted keys
    const uint32_t ncs = plan_chunks(st_max);
    const bool from_digits =
        direct || (capacity > 0 && npass == 1 && st_max <= uint32_t(ST_FROM_DIGITS) && ncs <= PLAN_ONE_BLOCK);
    if (!from_digits) {
        const uint64_t rblocks = (capacity + 1 + 255) / 256;
        hipLaunchKernelGGL((tile_ranges_kernel<uint32_t>), dim3(unsigned(rblocks < 4096 ? rblocks : 4096)), dim3(256),
                           0, s, keys[cur], etot, capacity, ST_KEY_SHIFT, st_max, st_offs);
        MGS_LAUNCH_CHECK("tile_ranges_kernel<supertile>");
    }

    // level 2: chunks, per-chunk tile counts, column scans, tile offsets, the lists
    if (ncs <= PLAN_ONE_BLOCK) {
        hipLaunchKernelGGL(chunk_plan_kernel, dim3(PLAN_REPLICAS), dim3(1024), 0, s, st_offs, st_count, st_max, n_pairs,
                           capacity, static_cast<const uint64_t *>(nullptr), static_cast<const uint64_t *>(nullptr), sc0,
                           chunk_st, chunk_lo, nch, from_digits ? dtot : static_cast<const uint32_t *>(nullptr),
                           st_offs);
    } else {
        hipLaunchKernelGGL(chunk_sum_kernel, dim3(plan_grid(ncs)), dim3(1024), 0, s, st_offs, st_count, st_max,
                           n_pairs, capacity, part_c);
        MGS_LAUNCH_CHECK("chunk_sum_kernel");
        hipLaunchKernelGGL(part_scan_kernel<>, dim3(1), dim3(1024), 0, s, part_c, static_cast<uint64_t *>(nullptr),
                           ncs, totals + 2, static_cast<uint64_t *>(nullptr));
        MGS_LAUNCH_CHECK("part_scan_kernel");
        hipLaunchKernelGGL(chunk_plan_kernel, dim3(plan_grid(ncs)), dim3(1024), 0, s, st_offs, st_count, st_max,
                           n_pairs, capacity, part_c, totals + 2, sc0, chunk_st, chunk_lo, nch,
                           static_cast<const uint32_t *>(nullptr), st_offs);
    }
    MGS_LAUNCH_CHECK("chunk_plan_kernel");
    const unsigned cgrid = L.chunks_max < uint32_t(SUPER_MAX_GRID) ? L.chunks_max : uint32_t(SUPER_MAX_GRID);
    hipLaunchKernelGGL((chunk_count_kernel<Geo>), dim3(cgrid), dim3(CHUNK), 0, s, vals[cur], keys[cur], chunk_st,
                       chunk_lo, st_offs, nch, geo, cnt);
    MGS_LAUNCH_CHECK("chunk_count_kernel");
    const uint64_t jobs = uint64_t(st_max) * SUPER_TILES;
    {                                            // a wave per job, 4 per workgroup
        const uint64_t nb = (jobs + 3) / 4;
        hipLaunchKernelGGL((chunk_colscan_kernel<Geo>), dim3(unsigned(nb < 16384 ? nb : 16384)), dim3(256), 0, s, cnt,
                           sc0, st_count, st_max, n_pairs, capacity, geo, ttot);
    }
    MGS_LAUNCH_CHECK("chunk_colscan_kernel");
    const uint32_t nct = plan_chunks(T);
    if (nct <= PLAN_ONE_BLOCK) {
        hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, s, ttot, t_count, T, n_pairs, capacity,
                           static_cast<const uint64_t *>(nullptr), tile_offsets);
    } else {
        hipLaunchKernelGGL(tile_sum_kernel, dim3(plan_grid(nct)), dim3(1024), 0, s, ttot, t_count, T, part_t);
        MGS_LAUNCH_CHECK("tile_sum_kernel");
        hipLaunchKernelGGL(part_scan_kernel<>, dim3(1), dim3(1024), 0, s, part_t, static_cast<uint64_t *>(nullptr),
                           nct, static_cast<uint64_t *>(nullptr), static_cast<uint64_t *>(nullptr));
        MGS_LAUNCH_CHECK("part_scan_kernel");
        hipLaunchKernelGGL(tile_scan_kernel, dim3(plan_grid(nct)), dim3(1024), 0, s, ttot, t_count, T, n_pairs,
                           capacity, part_t, tile_offsets);
    }
    MGS_LAUNCH_CHECK("tile_scan_kernel");
    if (capacity > 0) {
        hipLaunchKernelGGL((chunk_write_kernel<Geo>), dim3(cgrid), dim3(CHUNK), 0, s, vals[cur], keys[cur], chunk_st,
                           chunk_lo, st_offs, nch, geo, cnt, tile_offsets, n_pairs, capacity, gids);
        MGS_LAUNCH_CHECK("chunk_write_kernel");
    }
    return MGS_OK;
}

inline uint32_t super_count(int tiles_x, int tiles_y) {
    return uint32_t((tiles_x + SUPER - 1) / SUPER) * uint32_t((tiles_y + SUPER - 1) / SUPER);
}

int bin_batch(const mgs_projected *proj, int64_t n_max, const BatchPlan *plan, uint32_t max_tiles, void *ws,
              size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity, uint32_t *n_pairs,
              hipStream_t s) {
    // a request has at most as many supertiles as tiles
    return bin2_impl(proj, n_max, &plan->n_total, SuperBatch{plan}, max_tiles, &plan->st_total, max_tiles,
                     &plan->t_total, ws, ws_bytes, tile_offsets, gids, capacity, n_pairs, s);
}

size_t bin_batch_workspace(int64_t n_max, uint32_t max_tiles, uint64_t capacity) {
    return bin2_layout(n_max, max_tiles, max_tiles, capacity).total;
}

}  // namespace mgs

extern "C" int mgs_bin_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes) {
    MGS_REQUIRE(bytes != nullptr, "bytes is NULL");
    MGS_REQUIRE(n >= 0 && tiles_x > 0 && tiles_y > 0, "bad sizes");
    MGS_REQUIRE(tiles_x <= 65535 && tiles_y <= 65535, "bad tile grid");
    MGS_REQUIRE(mgs::super_count(tiles_x, tiles_y) < (1u << (32 - mgs::ST_KEY_SHIFT)), "too many supertiles");
    *bytes = mgs::bin2_layout(n, mgs::super_count(tiles_x, tiles_y), uint32_t(tiles_x) * uint32_t(tiles_y), capacity)
                 .total;
    return MGS_OK;
}

extern "C" int mgs_bin(const mgs_projected *proj, int64_t n, int tiles_x, int tiles_y, void *ws,
                       size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity,
                       uint32_t *n_pairs, void *stream) {
    MGS_TRACE("mgs_bin");
    MGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && tiles_x <= 65535 && tiles_y <= 65535, "bad tile grid");
    const uint32_t st_x = uint32_t((tiles_x + mgs::SUPER - 1) / mgs::SUPER);
    return mgs::bin2_impl(proj, n, nullptr, mgs::SuperGrid{uint32_t(tiles_x), uint32_t(tiles_y), st_x},
                          mgs::super_count(tiles_x, tiles_y), nullptr, uint32_t(tiles_x) * uint32_t(tiles_y), nullptr,
                          ws, ws_bytes, tile_offsets, gids, capacity, n_pairs, mgs::as_stream(stream));
}

extern "C" int mgs_bin_sorted_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity,
                                        size_t *bytes) {
    MGS_REQUIRE(bytes != nullptr, "bytes is NULL");
    MGS_REQUIRE(n >= 0 && tiles_x > 0 && tiles_y > 0, "bad sizes");
    *bytes = mgs::bin_layout<uint64_t>(n, capacity).total;
    return MGS_OK;
}

extern "C" int mgs_bin_sorted(const mgs_projected *proj, int64_t n, int tiles_x, int tiles_y, void *ws,
                              size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity,
                              uint32_t *n_pairs, void *stream) {
    MGS_TRACE("mgs_bin_sorted");
    MGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && tiles_x <= 65535 && tiles_y <= 65535, "bad tile grid");
    const int tile_bits = mgs::bits_for(uint64_t(tiles_x) * uint64_t(tiles_y));
    return mgs::bin_impl<uint64_t, mgs::TileDepthKey>(proj, n, mgs::GridMap{uint32_t(tiles_x)},
                                                       uint32_t(tiles_x) * uint32_t(tiles_y), ws, ws_bytes,
                                                       tile_offsets, gids, capacity, n_pairs, mgs::as_stream(stream),
                                                       32 + (tile_bits > 0 ? tile_bits : 1), 32);
}

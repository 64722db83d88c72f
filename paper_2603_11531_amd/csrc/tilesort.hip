// mgs_tile_sort: the order-independent binning's tile lists (ascending Gaussian index) sorted in
// place by camera depth, ties by Gaussian index -- the lists of the sorted comparison path
// (Eq. 11), built as a segmented sort on top of the two-level binning instead of a global sort of
// 64-bit (tile, depth) keys.
//
// One workgroup per tile list.  The key of an entry is the float32 depth of its record (depth >
// near_z > 0, so the IEEE bits order like the value); a stable LSD counting sort over 8-bit digits
// of it, skipping digits every entry of the list shares:
//   * a list of at most TS_CHUNK entries is sorted in LDS: per pass the entries are ranked by
//     ballot-matched digits (split evenly, in order, over the waves), the waves' digit counts
//     are scanned, and the entries rewritten in LDS in digit order;
//   * a longer list ping-pongs through a workspace copy in global memory: per pass, its digit
//     histogram, then its chunks in order, each ranked in LDS as above and written to the digit
//     runs after the entries of the earlier chunks.
// Stable passes over a list in ascending Gaussian index leave equal depths in index order.
#include "common.h"

namespace mgs {
namespace tsort {

#ifndef MGS_TS_THREADS
#define MGS_TS_THREADS 256
#endif
#ifndef MGS_TS_ITERS
#define MGS_TS_ITERS 8
#endif
constexpr int TS_THREADS = MGS_TS_THREADS;               // 256 or 512: a thread per digit and more
constexpr int TS_WAVES = TS_THREADS / 64;
constexpr int TS_ITERS = MGS_TS_ITERS;
constexpr uint32_t TS_CHUNK = TS_THREADS * TS_ITERS;    // entries sorted in LDS at once
static_assert(TS_THREADS >= 256 && TS_THREADS % 64 == 0, "a thread per 8-bit digit");
constexpr unsigned TS_GRID_MAX = 1u << 20;

struct Lds {
    uint32_t cnt[TS_WAVES][256];          // per wave and digit: entries so far, then the wave's start
    uint32_t lstart[256];                 // per digit: first position in the pass's output
    uint32_t ltot[256];                   // per digit: entries in the pass
    uint32_t gstart[256];                 // long lists: first position of the digit's run in the list
    uint32_t run[256];                    // long lists: entries of the digit written by earlier chunks
    uint32_t wsum[TS_WAVES];
    uint32_t bits[2];                     // OR and AND of the list's keys
    uint32_t k[TS_CHUNK], v[TS_CHUNK];
};

__device__ __forceinline__ unsigned lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanes_below() {
    const unsigned l = lane();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}
// Lanes of `active` holding the same 8-bit digit as this lane.
__device__ __forceinline__ uint64_t same_digit(uint32_t d, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}
// Exclusive scan of one value per thread over the workgroup (every thread calls).
__device__ __forceinline__ uint32_t excl_scan(uint32_t v, uint32_t *s_wsum) {
    const unsigned l = lane();
    const int w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (l >= unsigned(o)) inc += y;
    }
    if (l == 63) s_wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += s_wsum[k];
    __syncthreads();
    return pre + inc - v;
}

// One stable pass over the n <= TS_CHUNK entries in S.k / S.v by the digit (k >> shift) & 255:
// the entries end up in S.k / S.v in digit order (equal digits in their input order), with
// S.lstart / S.ltot the digits' runs.  Every thread calls it.
__device__ __forceinline__ void lds_pass(Lds &S, uint32_t n, int shift) {
    const int t = threadIdx.x, w = t >> 6;
    const unsigned l = lane();
    const uint32_t nit = (n + TS_THREADS - 1u) / uint32_t(TS_THREADS), seg = 64u * nit;
    const uint32_t base = uint32_t(w) * seg, wend = base + seg < n ? base + seg : n;
    uint32_t key[TS_ITERS], val[TS_ITERS], rank[TS_ITERS], dig[TS_ITERS];
#pragma unroll
    for (int it = 0; it < TS_ITERS; ++it) {
        const uint32_t idx = base + uint32_t(it) * 64u + l;
        const bool ok = uint32_t(it) < nit && idx < wend;
        key[it] = ok ? S.k[idx] : 0u;
        val[it] = ok ? S.v[idx] : 0u;
    }
    for (int i = t; i < TS_WAVES * 256; i += TS_THREADS) (&S.cnt[0][0])[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < TS_ITERS; ++it) {
        if (uint32_t(it) >= nit) break;                                   // wave-uniform
        const uint32_t idx = base + uint32_t(it) * 64u + l;
        const bool ok = idx < wend;
        const uint64_t active = __ballot(ok);
        const uint32_t d = ok ? (key[it] >> shift) & 255u : 0u;
        dig[it] = d;
        rank[it] = 0;
        if (active != 0) {
            const uint64_t peers = same_digit(d, active);
            const uint32_t before = ok ? S.cnt[w][d] : 0u;
            rank[it] = before + uint32_t(__popcll(peers & lanes_below()));
            __builtin_amdgcn_wave_barrier();
            if (ok && (peers >> l) == 1ull) S.cnt[w][d] = before + uint32_t(__popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    uint32_t tot = 0;
    if (t < 256) {
#pragma unroll
        for (int ww = 0; ww < TS_WAVES; ++ww) {
            const uint32_t c = S.cnt[ww][t];
            S.cnt[ww][t] = tot;
            tot += c;
        }
    }
    const uint32_t lex = excl_scan(tot, S.wsum);                           // contains __syncthreads
    if (t < 256) {
        S.lstart[t] = lex;
        S.ltot[t] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < TS_ITERS; ++it) {
        const uint32_t idx = base + uint32_t(it) * 64u + l;
        if (uint32_t(it) < nit && idx < wend) {
            const uint32_t lp = S.lstart[dig[it]] + S.cnt[w][dig[it]] + rank[it];
            S.k[lp] = key[it];
            S.v[lp] = val[it];
        }
    }
    __syncthreads();
}

// OR and AND of the keys each thread saw -> S.bits (every thread calls).
__device__ __forceinline__ void key_bits(Lds &S, uint32_t kor, uint32_t kand) {
    for (int o = 32; o > 0; o >>= 1) {
        kor |= __shfl_xor(kor, o, 64);
        kand &= __shfl_xor(kand, o, 64);
    }
    if (threadIdx.x == 0) {
        S.bits[0] = 0u;
        S.bits[1] = ~0u;
    }
    __syncthreads();
    if (lane() == 0) {
        atomicOr(&S.bits[0], kor);
        atomicAnd(&S.bits[1], kand);
    }
    __syncthreads();
}

// Long lists first.  Workgroups start in launch order as earlier ones finish, so in tile order the
// lists longer than TS_CHUNK (sorted through the workspace, several times the work of an LDS sort)
// that come last would run alone at the end.  The launch therefore walks the tiles twice: work
// item k < T sorts tile k only if its list is long, item T + k only if it is not, so every long
// list starts before any short one with no ordering pass; a skipped item costs two offset reads.
// The short lists keep tile order (neighbouring tiles share records in the caches).
__global__ void __launch_bounds__(TS_THREADS)
tile_sort_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs, uint32_t *__restrict__ gids,
                 uint32_t T, const uint32_t *__restrict__ n_pairs, uint64_t capacity, uint32_t *__restrict__ tk0,
                 uint32_t *__restrict__ tk1, uint32_t *__restrict__ tv0, uint32_t *__restrict__ tv1) {
    __shared__ Lds S;
    if (uint64_t(*n_pairs) > capacity) return;                            // grid-uniform: no lists
    const uint32_t P = *n_pairs;
    const int t = threadIdx.x;
    for (uint64_t k = blockIdx.x; k < 2 * uint64_t(T); k += gridDim.x) { // block-uniform
        const bool long_pass = k < T;
        const uint32_t tile = uint32_t(long_pass ? k : k - T);
        const uint32_t s = offs[tile], e = offs[tile + 1];
        if (!MGS_CHECK(s <= e && e <= P, BS_LIST_READ)) continue;
        const uint32_t n = e - s;
        if ((n > TS_CHUNK) != long_pass) continue;                        // the other pass's list
        if (n <= 1u) continue;
        if (n <= TS_CHUNK) {
            uint32_t kor = 0u, kand = ~0u;
            for (uint32_t i = t; i < n; i += TS_THREADS) {
                const uint32_t g = gids[s + i];
                const uint32_t k = __float_as_uint(splat[3 * size_t(g) + 1].w);
                S.k[i] = k;
                S.v[i] = g;
                kor |= k;
                kand &= k;
            }
            key_bits(S, kor, kand);                                       // contains __syncthreads
            const uint32_t vary = S.bits[0] ^ S.bits[1];
            for (int shift = 0; shift < 32; shift += 8)
                if ((vary >> shift) & 255u) lds_pass(S, n, shift);        // block-uniform
            for (uint32_t i = t; i < n; i += TS_THREADS) gids[s + i] = S.v[i];
            __syncthreads();                                              // LDS is reused by the next tile
            continue;
        }
        // a long list: keys and ids through the workspace copies (positions s .. e - 1)
        uint32_t kor = 0u, kand = ~0u;
        for (uint32_t i = t; i < n; i += TS_THREADS) {
            const uint32_t g = gids[s + i];
            const uint32_t k = __float_as_uint(splat[3 * size_t(g) + 1].w);
            tk0[s + i] = k;
            tv0[s + i] = g;
            kor |= k;
            kand &= k;
        }
        key_bits(S, kor, kand);
        const uint32_t vary = S.bits[0] ^ S.bits[1];
        uint32_t *ks = tk0, *vs = tv0, *kd = tk1, *vd = tv1;
        for (int shift = 0; shift < 32; shift += 8) {
            if (((vary >> shift) & 255u) == 0u) continue;                 // block-uniform
            // the list's digit histogram (counts: order-free) and each digit's run start
            if (t < 256) S.gstart[t] = 0u;
            __syncthreads();
            for (uint32_t i = t; i < n; i += TS_THREADS) atomicAdd(&S.gstart[(ks[s + i] >> shift) & 255u], 1u);
            __syncthreads();
            const uint32_t c = t < 256 ? S.gstart[t] : 0u;
            __syncthreads();
            const uint32_t gs = excl_scan(c, S.wsum);
            if (t < 256) {
                S.gstart[t] = gs;
                S.run[t] = 0u;
            }
            __syncthreads();
            // chunks in order, each ranked in LDS, written after the earlier chunks' entries
            for (uint32_t c0 = 0; c0 < n; c0 += TS_CHUNK) {
                const uint32_t rn = n - c0 < TS_CHUNK ? n - c0 : TS_CHUNK;
                for (uint32_t i = t; i < rn; i += TS_THREADS) {
                    S.k[i] = ks[s + c0 + i];
                    S.v[i] = vs[s + c0 + i];
                }
                __syncthreads();
                lds_pass(S, rn, shift);
                for (uint32_t lp = t; lp < rn; lp += TS_THREADS) {
                    const uint32_t d = (S.k[lp] >> shift) & 255u;
                    const uint32_t dst = S.gstart[d] + S.run[d] + lp - S.lstart[d];
                    if (MGS_CHECK(dst < n, BS_LIST_WRITE)) {
                        kd[s + dst] = S.k[lp];
                        vd[s + dst] = S.v[lp];
                    }
                }
                __syncthreads();
                if (t < 256) S.run[t] += S.ltot[t];
                __syncthreads();
            }
            uint32_t *tmp = ks; ks = kd; kd = tmp;
            tmp = vs; vs = vd; vd = tmp;
        }
        for (uint32_t i = t; i < n; i += TS_THREADS) gids[s + i] = vs[s + i];
        __syncthreads();
    }
}

struct SortLayout {
    size_t tk0, tk1, tv0, tv1, total;
};

inline SortLayout sort_layout(uint64_t capacity) {
    SortLayout L;
    const size_t cap = size_t(capacity > 0 ? capacity : 1);
    size_t o = 0;
    L.tk0 = o; o = align_up(o + cap * 4, 256);
    L.tk1 = o; o = align_up(o + cap * 4, 256);
    L.tv0 = o; o = align_up(o + cap * 4, 256);
    L.tv1 = o; o = align_up(o + cap * 4, 256);
    L.total = o;
    return L;
}

}  // namespace tsort
}  // namespace mgs

extern "C" int mgs_tile_sort_workspace(int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes) {
    MGS_REQUIRE(bytes != nullptr, "bytes is NULL");
    MGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && tiles_x <= 65535 && tiles_y <= 65535, "bad tile grid");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity must be < 2^32 - 1");
    *bytes = mgs::tsort::sort_layout(capacity).total;
    return MGS_OK;
}

extern "C" int mgs_tile_sort(const mgs_projected *proj, int64_t n, const uint32_t *tile_offsets, uint32_t *gids,
                             int tiles_x, int tiles_y, uint64_t capacity, const uint32_t *n_pairs, void *ws,
                             size_t ws_bytes, void *stream) {
    MGS_TRACE("mgs_tile_sort");
    using namespace mgs;
    int rc;
    MGS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if ((rc = check_projected(proj, n)) != MGS_OK) return rc;
    MGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && tiles_x <= 65535 && tiles_y <= 65535, "bad tile grid");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity must be < 2^32 - 1");
    MGS_REQUIRE(tile_offsets && n_pairs && (capacity == 0 || gids), "a required pointer is NULL");
    const tsort::SortLayout L = tsort::sort_layout(capacity);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.total, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    const uint64_t T = uint64_t(tiles_x) * uint64_t(tiles_y);
    if (capacity == 0 || n == 0) return MGS_OK;
    char *w = static_cast<char *>(ws);
    const unsigned grid = unsigned(2 * T < tsort::TS_GRID_MAX ? 2 * T : tsort::TS_GRID_MAX);
    hipLaunchKernelGGL(tsort::tile_sort_kernel, dim3(grid), dim3(tsort::TS_THREADS), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, uint32_t(T), n_pairs,
                       capacity, reinterpret_cast<uint32_t *>(w + L.tk0), reinterpret_cast<uint32_t *>(w + L.tk1),
                       reinterpret_cast<uint32_t *>(w + L.tv0), reinterpret_cast<uint32_t *>(w + L.tv1));
    MGS_LAUNCH_CHECK("tile_sort_kernel");
    return MGS_OK;
}

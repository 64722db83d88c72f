// mgs_blend_oit (Eq. 2) and mgs_blend_sorted (Eq. 11): per-tile compositing.
//
// One 256-thread workgroup per 16x16 tile (or per range of a long tile list).  The
// tile's Gaussians are staged through LDS in batches (one coalesced 48-byte record
// per thread).  While staging, every thread also decides, for its Gaussian, which
// 8x8 quadrants of the tile can see it: the largest alpha over a quadrant's
// pixel-centre rectangle is found exactly (the exponent is a concave quadratic, so
// its maximum over a rectangle is at the centre or on an edge) and quadrants where
// it stays below alpha_min are masked out, so no VALU cycle is spent on a quadrant
// that a splat cannot reach.
//
// Order-independent path: the four waves split the staged Gaussians, each lane
// holds one pixel in each quadrant, and the waves' sums are merged at the end
// (blend_tile_oit).  Per pixel-Gaussian pair the inner loop is 2 FMA for the
// exponent (a polynomial in the pixel's offset, see quad_poly, with 3 more FMA per
// row of quadrants), compare/select, exp2 and 5 FMA to accumulate N (rgb, colours
// pre-multiplied by w), D and T -- all float32 VALU, no sort, no order.
//
// Sorted path: wave w owns quadrant w and walks the depth-ordered list front to
// back with early termination (blend_tile_sorted).
#include <mutex>

#include "batch.h"
#include "blend_math.h"

namespace mgs {

template <bool SORTED>
__global__ void __launch_bounds__(BLEND_THREADS)
blend_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs,
             const uint32_t *__restrict__ gids, CamK cam, float bgr, float bgg, float bgb, float wbg,
             float log2_amin, float amax, float t_stop, float *__restrict__ image,
             float *__restrict__ aux) {
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    if (SORTED)
        blend_tile_sorted(splat, gids, offs[tile], offs[tile + 1], tx, ty, cam.W, cam.H, bgr, bgg, bgb, log2_amin,
                          amax, t_stop, image);
    else
        blend_tile_oit(splat, gids, offs[tile], offs[tile + 1], tx, ty, cam.W, cam.H, bgr, bgg, bgb, wbg, log2_amin,
                       amax, image, aux, nullptr);
}

// ---------------------------------------------------------------- split-tile OIT blend
constexpr uint32_t MERGE_GRID = 2048;         // workgroups of the range merge
constexpr int PART_FLOATS = 5 * 256;          // per-range partial sums (N rgb, D, T) x 256 pixels

// Destination of one tile: a single view, or one request of a batch.
// wbg: EQ2_COMPOSITE, or the background weight of Eq. 1's composite.
struct TileView {
    int tx, ty, W, H;
    float bg[3];
    float wbg;
    float *image, *aux;
};
struct SingleViewLoc {
    int tiles_x, W, H;
    float bg[3];
    float wbg;
    float *image, *aux;
    __device__ __forceinline__ TileView operator()(uint32_t t) const {
        return TileView{int(t % uint32_t(tiles_x)), int(t / uint32_t(tiles_x)), W, H, {bg[0], bg[1], bg[2]}, wbg,
                        image, aux};
    }
};
struct BatchViewLoc {
    const mgs_request *reqs;
    const BatchPlan *plan;
    __device__ __forceinline__ TileView operator()(uint32_t gt) const {
        const int r = find_request(plan->tbase, plan->nreq, gt);
        const mgs_request &q = reqs[r];
        const uint32_t lt = gt - plan->tbase[r], tx = plan->tiles_x[r];
        return TileView{int(lt % tx), int(lt / tx), q.cam.width, q.cam.height, {q.bg[0], q.bg[1], q.bg[2]},
                        EQ2_COMPOSITE, q.image, nullptr};
    }
};

// Work list of the split blend: every tile gets n_ranges(L) items (item = tile | range << 24,
// so at most 2^24 - 1 tiles); ranges of split tiles (n_ranges > 1) also get a partial-sum slot.
// counts = {items, split tiles}; split_tile[j] = tile | n_ranges << 24 and split_slot0[j] = first
// slot of the j-th split tile.
// Chunked scan over the tiles (SPLIT_TILE tiles per chunk): pass 1 totals each chunk's items, slots
// and split tiles; pass 2 puts each tile's first item and slot in LDS and writes the chunk's
// items coalesced, each thread finding the tile of its item by binary search in LDS.
__device__ __forceinline__ uint32_t live_tiles(const uint32_t *t_count, uint32_t t_host, const uint32_t *n_pairs,
                                               uint64_t capacity) {
    uint32_t T = t_count ? *t_count : t_host;
    if (T > t_host) T = t_host;
    return uint64_t(*n_pairs) > capacity ? 0u : T;             // lists were not built: render nothing
}

// The split plan scans chunks of SPLIT_TILE tiles, SPLIT_ITEMS per thread of a 1024-thread
// block (one chunk covers a 1920x1080 view's 8,160 tiles, so a single view needs one pass).
constexpr int SPLIT_ITEMS = 8;
constexpr int SPLIT_TILE = 1024 * SPLIT_ITEMS;
__host__ __device__ __forceinline__ uint32_t split_chunks(uint64_t T) {
    return uint32_t((T + SPLIT_TILE - 1) / SPLIT_TILE);
}

// Ranges of this thread's SPLIT_ITEMS tiles t0 .. (n_ranges <= 255: 8 bits each, tile t0 + j in
// bits 8 j ..), and their sums: ci items, cs slots (ranges of split tiles), cm split tiles.
// One chunk's items, slots and split tiles packed for a single block scan: items and slots
// are at most SPLIT_TILE * 255 < 2^21 each, split tiles at most SPLIT_TILE.
static_assert(uint64_t(SPLIT_TILE) * 255 < (1ull << 21), "split plan packing");
__device__ __forceinline__ uint64_t split_pack(uint32_t ci, uint32_t cs, uint32_t cm) {
    return uint64_t(ci) | (uint64_t(cs) << 21) | (uint64_t(cm) << 42);
}
__device__ __forceinline__ uint32_t split_items(uint64_t v) { return uint32_t(v) & 0x1FFFFFu; }
__device__ __forceinline__ uint32_t split_slots(uint64_t v) { return uint32_t(v >> 21) & 0x1FFFFFu; }
__device__ __forceinline__ uint32_t split_tiles(uint64_t v) { return uint32_t(v >> 42); }

__device__ __forceinline__ uint64_t tile_ranges(const uint32_t *offs, uint32_t t0, uint32_t T, uint32_t &ci,
                                                uint32_t &cs, uint32_t &cm) {
    uint32_t o[SPLIT_ITEMS + 1];
#pragma unroll
    for (int j = 0; j <= SPLIT_ITEMS; ++j) o[j] = t0 + j <= T ? offs[t0 + j] : 0u;
    ci = cs = cm = 0;
    uint64_t packed = 0;
#pragma unroll
    for (int j = 0; j < SPLIT_ITEMS; ++j) {
        const uint32_t nr = t0 + j < T ? n_ranges(o[j + 1] - o[j], SPLIT_RANGE) : 0u;
        packed |= uint64_t(nr) << (8 * j);
        ci += nr;
        cs += nr > 1 ? nr : 0u;
        cm += nr > 1 ? 1u : 0u;
    }
    return packed;
}

__global__ void __launch_bounds__(1024)
split_sum_kernel(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ t_count, uint32_t t_host,
                 const uint32_t *__restrict__ n_pairs, uint64_t capacity, uint64_t *__restrict__ part_is,
                 uint64_t *__restrict__ part_m) {
    __shared__ uint64_t s_wsum[16];
    const uint32_t T = live_tiles(t_count, t_host, n_pairs, capacity);
    for (uint32_t c = blockIdx.x; c < split_chunks(t_host); c += gridDim.x) {
        uint32_t ci, cs, cm;
        tile_ranges(offs, c * SPLIT_TILE + threadIdx.x * SPLIT_ITEMS, T, ci, cs, cm);
        uint64_t t;
        block_scan1024(split_pack(ci, cs, cm), s_wsum, &t);
        if (threadIdx.x == 0) {
            part_is[c] = split_items(t) | (uint64_t(split_slots(t)) << 32);
            part_m[c] = split_tiles(t);
        }
    }
}

static_assert(SPLIT_TILE == 8192, "split_plan_kernel searches an 8192-entry table in 13 steps");
constexpr int SPLIT_FILL_ILP = 4;                // item searches a thread keeps in flight
constexpr unsigned SPLIT_REPLICAS = 16;          // blocks of the ordered plan, each writing one wave's tiles

__global__ void __launch_bounds__(1024)
split_plan_kernel(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ t_count, uint32_t t_host,
                  const uint32_t *__restrict__ n_pairs, uint64_t capacity, const uint64_t *__restrict__ part_is,
                  const uint64_t *__restrict__ part_m, const uint64_t *__restrict__ totals,
                  uint32_t *__restrict__ items, uint32_t *__restrict__ item_slot, uint32_t *__restrict__ split_tile,
                  uint32_t *__restrict__ split_slot0, uint32_t *__restrict__ counts) {
    // block c (and c + grid ...) takes chunk c, its first item / slot / split tile from part_is, part_m
    __shared__ uint64_t s_wsum[16];
    __shared__ uint32_t s_item0[SPLIT_TILE];     // chunk-relative first item of each tile
    __shared__ uint32_t s_slot0[SPLIT_TILE];     // first partial-sum slot of a split tile, else ~0
    const uint32_t T = live_tiles(t_count, t_host, n_pairs, capacity);
    constexpr uint32_t fill_stride = 1024u;
    for (uint32_t c = blockIdx.x; c < split_chunks(T); c += gridDim.x) {
        const uint32_t t0 = c * SPLIT_TILE + threadIdx.x * SPLIT_ITEMS;
        uint32_t ci, cs, cm;
        const uint64_t nr = tile_ranges(offs, t0, T, ci, cs, cm);
        uint64_t t;
        const uint64_t x = block_scan1024(split_pack(ci, cs, cm), s_wsum, &t);
        const uint64_t b1 = part_is[c];          // items | slots << 32 before the chunk
        const uint64_t b2 = part_m[c];
        const uint32_t t1 = split_items(t);
        uint32_t i0 = split_items(x), s0 = uint32_t(b1 >> 32) + split_slots(x), js = uint32_t(b2) + split_tiles(x);
#pragma unroll
        for (int j = 0; j < SPLIT_ITEMS; ++j) {
            const uint32_t nj = uint32_t(nr >> (8 * j)) & 0xFFu;
            const bool m = nj > 1;
            s_item0[threadIdx.x * SPLIT_ITEMS + j] = i0;
            s_slot0[threadIdx.x * SPLIT_ITEMS + j] = m ? s0 : 0xFFFFFFFFu;
            if (m) {
                split_tile[js] = (t0 + j) | (nj << 24);          // the merge needs no list offsets
                split_slot0[js] = s0;
            }
            if (m) {
                s0 += nj;
                ++js;
            }
            i0 += nj;
        }
        __syncthreads();
        // item i of the chunk belongs to its last tile whose first item is <= i (tiles with
        // no item share the next tile's start and are never chosen); s_item0[0] = 0 <= i
        const uint32_t n_items = uint32_t(t1), ibase = uint32_t(b1);
        for (uint32_t i = threadIdx.x; i < n_items; i += fill_stride * SPLIT_FILL_ILP) {
            uint32_t lo[SPLIT_FILL_ILP];
#pragma unroll
            for (int q = 0; q < SPLIT_FILL_ILP; ++q) lo[q] = 0;
#pragma unroll 1
            for (uint32_t step = SPLIT_TILE / 2; step; step >>= 1) {
#pragma unroll
                for (int q = 0; q < SPLIT_FILL_ILP; ++q)
                    if (s_item0[lo[q] + step] <= i + q * fill_stride) lo[q] += step;
            }
#pragma unroll
            for (int q = 0; q < SPLIT_FILL_ILP; ++q) {
                const uint32_t k = i + q * fill_stride;
                if (k < n_items && MGS_CHECK(uint64_t(ibase) + k < split_max_items(t_host, capacity), BS_SPLIT_ITEM)) {
                    const uint32_t r = k - s_item0[lo[q]], sl = s_slot0[lo[q]];
                    items[ibase + k] = (c * SPLIT_TILE + lo[q]) | (r << 24);
                    item_slot[ibase + k] = sl == 0xFFFFFFFFu ? sl : sl + r;
                }
            }
        }
        __syncthreads();                         // the tables are rewritten by the next chunk
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[0] = T == 0 ? 0u : uint32_t(totals[0]);   // items (low half of items | slots << 32)
        counts[1] = T == 0 ? 0u : uint32_t(totals[1]);   // split tiles
    }
}

// Work items longest first.  The range workgroups are dispatched in item order as earlier ones
// finish, so items in tile order leave whichever long items come last running alone at the end;
// putting the longest first (list scheduling by decreasing length) shortens that tail.  A tile's
// ranges all go to the length bucket of its range length (LEN_BUCKETS buckets of SPLIT_RANGE /
// LEN_BUCKETS), buckets in decreasing length, tile order inside a bucket; the partial-sum slots
// stay in tile order.  The order changes no result: an item owns its tile's pixels or its slot.
constexpr int LEN_BUCKETS = 8;
constexpr int LEN_WORDS = LEN_BUCKETS / 3 + 1;          // 21-bit counters, three per word
static_assert(uint64_t(SPLIT_TILE) * SPLIT_MAX_RANGES < (1ull << 21), "21-bit bucket counters");
static_assert(SPLIT_REPLICAS == 1024 / 64, "each replica writes the tiles of one of the 16 waves");
__device__ __forceinline__ uint32_t len_bucket(uint32_t len) {
    const uint32_t b = len == 0u ? 0u : (len - 1u) / (SPLIT_RANGE / LEN_BUCKETS);
    return b < uint32_t(LEN_BUCKETS - 1) ? b : uint32_t(LEN_BUCKETS - 1);
}
// Counter b of packed bucket counters in v[0 .. LEN_WORDS): an OR of masked words, not an indexed
// read, so the array stays in registers.
template <int N>
__device__ __forceinline__ uint32_t len_field(const uint64_t (&v)[N], uint32_t b) {
    static_assert(N >= LEN_WORDS, "bucket counter words");
    const uint32_t wi = b / 3u;
    uint64_t w = 0;
#pragma unroll
    for (int k = 0; k < LEN_WORDS; ++k) w |= v[k] & (0ull - uint64_t(wi == uint32_t(k)));
    return uint32_t(w >> (21u * (b - 3u * wi))) & 0x1FFFFFu;
}

// The plan in longest-first order, for up to ORDER_CHUNKS chunks of SPLIT_TILE tiles (a single view
// up to 4K, or a batch of up to eight 1920 x 1080 views).  Per thread: its tiles' items per length
// bucket and its split-tile slots / count, scanned over the block in one pass (PLAN_WORDS packed
// words, one LDS exchange).  Inside a bucket the items keep tile order, across chunks too.
constexpr uint32_t ORDER_CHUNKS = 8;
constexpr int PLAN_WORDS = LEN_WORDS + 1;        // bucket counters, then slots | split tiles << 32
constexpr int CHUNK_TOTALS = LEN_BUCKETS + 2;    // per chunk: items per bucket, slots, split tiles
static_assert(ORDER_CHUNKS * CHUNK_TOTALS <= 1024, "one chunk total per thread");

// Chunk c, this thread's tiles t0 .. t0 + 7 (t0 returned): range counts (8 bits each) and length
// buckets (4 bits each) packed in nrp / bkp, per-bucket item counts and slots / split tiles in v.
__device__ __forceinline__ uint32_t plan_tiles(const uint32_t *__restrict__ offs, uint32_t T, uint32_t c,
                                               uint64_t &nrp, uint32_t &bkp, uint64_t (&v)[PLAN_WORDS]) {
    static_assert(SPLIT_ITEMS == 8 && LEN_BUCKETS <= 16, "packing of the per-tile values");
    const uint32_t t0 = c * SPLIT_TILE + threadIdx.x * SPLIT_ITEMS;
    uint32_t o[SPLIT_ITEMS + 1];
#pragma unroll
    for (int j = 0; j <= SPLIT_ITEMS; ++j) o[j] = t0 + j <= T ? offs[t0 + j] : 0u;
    nrp = 0;
    bkp = 0;
    uint32_t cs = 0, cm = 0;
#pragma unroll
    for (int k = 0; k < PLAN_WORDS; ++k) v[k] = 0;
#pragma unroll
    for (int j = 0; j < SPLIT_ITEMS; ++j) {
        const uint32_t L = o[j + 1] - o[j];
        const uint32_t n = t0 + j < T ? n_ranges(L, SPLIT_RANGE) : 0u;
        const uint32_t b = len_bucket(t0 + j < T ? range_len(L, SPLIT_RANGE) : 0u);
        nrp |= uint64_t(n) << (8 * j);
        bkp |= b << (4 * j);
        const uint32_t wi = b / 3u;
        const uint64_t add = uint64_t(n) << (21u * (b - 3u * wi));
#pragma unroll
        for (int k = 0; k < LEN_WORDS; ++k) v[k] += wi == uint32_t(k) ? add : 0ull;
        cs += n > 1 ? n : 0u;
        cm += n > 1 ? 1u : 0u;
    }
    v[PLAN_WORDS - 1] = uint64_t(cs) | (uint64_t(cm) << 32);
    return t0;
}

// Inclusive wave scan of the words (inc); lane 63 leaves the wave's sums in s_w[k][wave].
__device__ __forceinline__ void plan_wave_scan(const uint64_t (&v)[PLAN_WORDS], uint64_t (&inc)[PLAN_WORDS],
                                               uint64_t (*s_w)[16]) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < PLAN_WORDS; ++k) inc[k] = v[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int k = 0; k < PLAN_WORDS; ++k) {
            const uint64_t u = __shfl_up(inc[k], d, 64);
            if (l >= d) inc[k] += u;
        }
    }
    if (l == 63) {
#pragma unroll
        for (int k = 0; k < PLAN_WORDS; ++k) s_w[k][threadIdx.x >> 6] = inc[k];
    }
}

// Block sums of the words from s_w (after a barrier): per-bucket items, slots, split tiles.
__device__ __forceinline__ void plan_totals(const uint64_t (*s_w)[16], uint32_t (&tot)[CHUNK_TOTALS]) {
    uint64_t t[PLAN_WORDS];
#pragma unroll
    for (int k = 0; k < PLAN_WORDS; ++k) {
        t[k] = 0;
        for (int ww = 0; ww < 16; ++ww) t[k] += s_w[k][ww];
    }
#pragma unroll
    for (int b = 0; b < LEN_BUCKETS; ++b) tot[b] = len_field(t, uint32_t(b));
    tot[LEN_BUCKETS] = uint32_t(t[PLAN_WORDS - 1]);
    tot[LEN_BUCKETS + 1] = uint32_t(t[PLAN_WORDS - 1] >> 32);
}

// Several chunks, first launch: block c writes chunk c's CHUNK_TOTALS totals to ctot.
__global__ void __launch_bounds__(1024)
split_chunk_totals_kernel(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ t_count, uint32_t t_host,
                          const uint32_t *__restrict__ n_pairs, uint64_t capacity, uint32_t *__restrict__ ctot) {
    __shared__ uint64_t s_w[PLAN_WORDS][16];
    const uint32_t T = live_tiles(t_count, t_host, n_pairs, capacity);
    uint64_t nrp, v[PLAN_WORDS], inc[PLAN_WORDS];
    uint32_t bkp;
    plan_tiles(offs, T, blockIdx.x, nrp, bkp, v);
    plan_wave_scan(v, inc, s_w);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot[CHUNK_TOTALS];
        plan_totals(s_w, tot);
#pragma unroll
        for (int k = 0; k < CHUNK_TOTALS; ++k) ctot[blockIdx.x * CHUNK_TOTALS + k] = tot[k];
    }
}

// The items and split-tile tables.  SPLIT_REPLICAS blocks per chunk (block b: chunk b / 16) each
// scan the chunk and write the items and split-tile entries of the tiles of one wave (b % 16),
// which spreads the scattered writes over CUs.  ONE (a single chunk): the bucket totals come from
// the block's own scan; else from every chunk's totals in ctot (the first launch), which give the
// chunk's first position in each bucket and its first slot and split tile.
template <bool ONE>
__global__ void __launch_bounds__(1024)
split_plan_ordered_kernel(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ t_count, uint32_t t_host,
                          const uint32_t *__restrict__ n_pairs, uint64_t capacity, const uint32_t *__restrict__ ctot,
                          uint32_t *__restrict__ items, uint32_t *__restrict__ item_slot,
                          uint32_t *__restrict__ split_tile, uint32_t *__restrict__ split_slot0,
                          uint32_t *__restrict__ counts) {
    constexpr int K = PLAN_WORDS;
    __shared__ uint64_t s_w[K][16];                      // per word and wave: the wave's sums
    __shared__ uint32_t s_ctot[ONE ? 1 : ORDER_CHUNKS * CHUNK_TOTALS];
    __shared__ uint32_t s_first[LEN_BUCKETS];            // the chunk's first position in each bucket
    __shared__ uint32_t s_slot0, s_split0;               // the chunk's first slot and split tile
    const int w = threadIdx.x >> 6;
    const uint32_t c = ONE ? 0u : blockIdx.x / SPLIT_REPLICAS;
    const uint32_t nc = ONE ? 1u : gridDim.x / SPLIT_REPLICAS;
    const uint32_t T = live_tiles(t_count, t_host, n_pairs, capacity);
    uint32_t ct = 0;                                     // one chunk total per thread, loaded before the scan
    if (!ONE && threadIdx.x < nc * CHUNK_TOTALS) ct = ctot[threadIdx.x];
    uint64_t nrp, v[K], inc[K];
    uint32_t bkp;
    const uint32_t t0 = plan_tiles(offs, T, c, nrp, bkp, v);
    plan_wave_scan(v, inc, s_w);
    if (!ONE && threadIdx.x < nc * CHUNK_TOTALS) s_ctot[threadIdx.x] = ct;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint64_t pre = 0;
        for (int ww = 0; ww < w; ++ww) pre += s_w[k][ww];
        v[k] = pre + inc[k] - v[k];
    }
    if (threadIdx.x == 0) {
        // first positions, longest bucket first, chunks in order inside a bucket
        uint32_t run = 0, slot = 0, split = 0;
        if (ONE) {
            uint32_t tot[CHUNK_TOTALS];
            plan_totals(s_w, tot);
            for (int b = LEN_BUCKETS - 1; b >= 0; --b) {
                s_first[b] = run;
                run += tot[b];
            }
            split = tot[LEN_BUCKETS + 1];
            s_slot0 = 0;
            s_split0 = 0;
        } else {
            for (int b = LEN_BUCKETS - 1; b >= 0; --b)
                for (uint32_t cc = 0; cc < nc; ++cc) {
                    if (cc == c) s_first[b] = run;
                    run += s_ctot[cc * CHUNK_TOTALS + b];
                }
            for (uint32_t cc = 0; cc < nc; ++cc) {
                if (cc == c) {
                    s_slot0 = slot;
                    s_split0 = split;
                }
                slot += s_ctot[cc * CHUNK_TOTALS + LEN_BUCKETS];
                split += s_ctot[cc * CHUNK_TOTALS + LEN_BUCKETS + 1];
            }
        }
        if (blockIdx.x == 0) {
            counts[0] = run;
            counts[1] = split;
        }
    }
    __syncthreads();
    if (w != int(blockIdx.x % SPLIT_REPLICAS)) return;   // the writer wave
    const uint64_t max_items = split_max_items(t_host, capacity);
    uint32_t s0 = s_slot0 + uint32_t(v[K - 1]), js = s_split0 + uint32_t(v[K - 1] >> 32);
    for (uint32_t j = 0; j < uint32_t(SPLIT_ITEMS); ++j) {
        const uint32_t n = uint32_t(nrp >> (8 * j)) & 0xFFu, b = (bkp >> (4 * j)) & 0xFu;
        uint32_t before = 0;                             // this thread's earlier items in bucket b
        for (uint32_t jj = 0; jj < j; ++jj)
            before += ((bkp >> (4 * jj)) & 0xFu) == b ? uint32_t(nrp >> (8 * jj)) & 0xFFu : 0u;
        const uint32_t pos = s_first[b] + len_field(v, b) + before;
        const bool split = n > 1;
        if (split) {
            split_tile[js] = (t0 + j) | (n << 24);
            split_slot0[js] = s0;
        }
        for (uint32_t r = 0; r < n; ++r) {
            if (MGS_CHECK(uint64_t(pos) + r < max_items, BS_SPLIT_ITEM)) {
                items[pos + r] = (t0 + j) | (r << 24);
                item_slot[pos + r] = split ? s0 + r : 0xFFFFFFFFu;
            }
        }
        if (split) {
            s0 += n;
            ++js;
        }
    }
}

// n_pairs / max_slots are read only by the checks of a checked build (MGS_CHECK_BOUNDS).
template <typename Loc>
__global__ void __launch_bounds__(BLEND_THREADS, 7)
blend_range_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs,
                   const uint32_t *__restrict__ gids, const uint32_t *__restrict__ items,
                   const uint32_t *__restrict__ item_slot, const uint32_t *__restrict__ counts, Loc loc,
                   float log2_amin, float amax, float *__restrict__ part, const uint32_t *__restrict__ n_pairs,
                   uint32_t max_slots) {
    const uint32_t k = blockIdx.x;
    if (k >= counts[0]) return;                                           // block-uniform
    const uint32_t it = items[k], t = it & 0xFFFFFFu, r = it >> 24;
    const uint32_t start = offs[t], end = offs[t + 1];
    if (!MGS_CHECK(start <= end && end <= *n_pairs, BS_LIST_READ)) return;
    const uint32_t L = end - start, rl = range_len(L, SPLIT_RANGE);
    const TileView v = loc(t);
    // a tile with one range is composited here; a range of a split tile leaves its sums in part
    const bool whole = n_ranges(L, SPLIT_RANGE) == 1;
    if (!whole && !MGS_CHECK(item_slot[k] < max_slots && r < n_ranges(L, SPLIT_RANGE), BS_SPLIT_ITEM)) return;
    const uint32_t s = whole ? start : start + r * rl;
    const uint32_t e = (whole || end - s <= rl) ? end : s + rl;
    blend_tile_oit(splat, gids, s, e, v.tx, v.ty, v.W, v.H, v.bg[0], v.bg[1], v.bg[2], v.wbg, log2_amin, amax,
                   v.image, v.aux, whole ? nullptr : part + size_t(item_slot[k]) * PART_FLOATS);
}

// Merge the ranges of each split tile in range order and composite (Eq. 2).
template <typename Loc>
__global__ void __launch_bounds__(BLEND_THREADS)
merge_ranges_kernel(const uint32_t *__restrict__ split_tile, const uint32_t *__restrict__ split_slot0,
                    const uint32_t *__restrict__ counts, Loc loc, const float *__restrict__ part) {
    const uint32_t n_split = counts[1];
    for (uint32_t j = blockIdx.x; j < n_split; j += gridDim.x) {         // block-uniform
        const uint32_t st = split_tile[j], t = st & 0xFFFFFFu, nr = st >> 24;
        const float *b = part + size_t(split_slot0[j]) * PART_FLOATS;
        const int p = threadIdx.x;
        float Nr = 0.f, Ng = 0.f, Nb = 0.f, D = 0.f, T = 1.f;
        for (uint32_t r = 0; r < nr; ++r, b += PART_FLOATS) {
            Nr += b[p];
            Ng += b[256 + p];
            Nb += b[512 + p];
            D += b[768 + p];
            T *= b[1024 + p];
        }
        const TileView v = loc(t);
        int px, py;
        tile_pixel(p, v.tx, v.ty, px, py);
        composite_oit(Nr, Ng, Nb, D, T, px, py, v.W, v.H, v.bg[0], v.bg[1], v.bg[2], v.wbg, v.image, v.aux);
    }
}

struct SplitLayout {
    size_t items, slot, stile, sslot, counts, part, part_is, part_m, totals, ctot, total;
    uint32_t max_items;
};

inline SplitLayout split_layout(uint32_t T, uint64_t capacity) {
    SplitLayout L;
    L.max_items = uint32_t(split_max_items(T, capacity));
    const size_t max_slots = size_t(split_max_slots(capacity));
    size_t o = 0;
    L.items = o;  o = align_up(o + size_t(L.max_items) * 4, 256);
    L.slot = o;   o = align_up(o + size_t(L.max_items) * 4, 256);
    L.stile = o;  o = align_up(o + size_t(T) * 4 + 4, 256);
    L.sslot = o;  o = align_up(o + size_t(T) * 4 + 4, 256);
    L.counts = o; o = align_up(o + 16, 256);
    L.part = o;   o = align_up(o + max_slots * PART_FLOATS * 4, 256);
    L.part_is = o; o = align_up(o + (size_t(split_chunks(T)) + 1) * 8, 256);
    L.part_m = o;  o = align_up(o + (size_t(split_chunks(T)) + 1) * 8, 256);
    L.totals = o;  o = align_up(o + 2 * 8, 256);
    L.ctot = o;    o = align_up(o + ORDER_CHUNKS * CHUNK_TOTALS * 4, 256);
    L.total = o;
    return L;
}

template <typename Loc>
int blend_split_launch(const float4 *splat, const uint32_t *offs, const uint32_t *gids, const uint32_t *t_count,
                       uint32_t T, const uint32_t *n_pairs, uint64_t capacity, Loc loc, float alpha_min,
                       float alpha_max, void *ws, hipStream_t s) {
    const SplitLayout L = split_layout(T, capacity);
    char *w = static_cast<char *>(ws);
    uint32_t *items = reinterpret_cast<uint32_t *>(w + L.items);
    uint32_t *slot = reinterpret_cast<uint32_t *>(w + L.slot);
    uint32_t *stile = reinterpret_cast<uint32_t *>(w + L.stile);
    uint32_t *sslot = reinterpret_cast<uint32_t *>(w + L.sslot);
    uint32_t *counts = reinterpret_cast<uint32_t *>(w + L.counts);
    float *part = reinterpret_cast<float *>(w + L.part);
    uint64_t *part_is = reinterpret_cast<uint64_t *>(w + L.part_is);
    uint64_t *part_m = reinterpret_cast<uint64_t *>(w + L.part_m);
    uint64_t *totals = reinterpret_cast<uint64_t *>(w + L.totals);
    uint32_t *ctot = reinterpret_cast<uint32_t *>(w + L.ctot);
    const uint32_t nc = split_chunks(T);
    if (nc <= 1) {                               // one chunk: the plan in longest-first order
        hipLaunchKernelGGL(split_plan_ordered_kernel<true>, dim3(SPLIT_REPLICAS), dim3(1024), 0, s, offs, t_count, T,
                           n_pairs, capacity, static_cast<const uint32_t *>(nullptr), items, slot, stile, sslot,
                           counts);
    } else if (nc <= ORDER_CHUNKS) {             // a few chunks: longest first, chunk totals first
        hipLaunchKernelGGL(split_chunk_totals_kernel, dim3(nc), dim3(1024), 0, s, offs, t_count, T, n_pairs, capacity,
                           ctot);
        MGS_LAUNCH_CHECK("split_chunk_totals_kernel");
        hipLaunchKernelGGL(split_plan_ordered_kernel<false>, dim3(nc * SPLIT_REPLICAS), dim3(1024), 0, s, offs,
                           t_count, T, n_pairs, capacity, ctot, items, slot, stile, sslot, counts);
    } else {                                     // many chunks (beyond eight 1920 x 1080 views): tile order
        hipLaunchKernelGGL(split_sum_kernel, dim3(plan_grid(nc)), dim3(1024), 0, s, offs, t_count, T, n_pairs,
                           capacity, part_is, part_m);
        MGS_LAUNCH_CHECK("split_sum_kernel");
        hipLaunchKernelGGL(part_scan_kernel<>, dim3(1), dim3(1024), 0, s, part_is, part_m, nc, totals, totals + 1);
        MGS_LAUNCH_CHECK("part_scan_kernel");
        hipLaunchKernelGGL(split_plan_kernel, dim3(plan_grid(nc)), dim3(1024), 0, s, offs, t_count, T, n_pairs,
                           capacity, part_is, part_m, totals, items, slot, stile, sslot, counts);
    }
    MGS_LAUNCH_CHECK("split_plan_kernel");
    hipLaunchKernelGGL(blend_range_kernel<Loc>, dim3(L.max_items), dim3(BLEND_THREADS), 0, s, splat, offs, gids,
                       items, slot, counts, loc, log2f(alpha_min), alpha_max, part, n_pairs,
                       uint32_t(split_max_slots(capacity)));
    MGS_LAUNCH_CHECK("blend_range_kernel");
    // split tiles are at most T; a bounded grid walks them (most tiles are not split)
    hipLaunchKernelGGL(merge_ranges_kernel<Loc>, dim3(T == 0 ? 1u : (T < MERGE_GRID ? T : MERGE_GRID)),
                       dim3(BLEND_THREADS), 0, s, stile, sslot, counts, loc, part);
    MGS_LAUNCH_CHECK("merge_ranges_kernel");
    return MGS_OK;
}

size_t blend_split_workspace(uint32_t T, uint64_t capacity) { return split_layout(T, capacity).total; }

int blend_split_batch(const float4 *splat, const uint32_t *offs, const uint32_t *gids, const BatchPlan *plan,
                      const mgs_request *reqs, uint32_t max_tiles, const uint32_t *n_pairs, uint64_t capacity,
                      float alpha_min, float alpha_max, void *ws, hipStream_t s) {
    return blend_split_launch(splat, offs, gids, &plan->t_total, max_tiles, n_pairs, capacity,
                              BatchViewLoc{reqs, plan}, alpha_min, alpha_max, ws, s);
}

inline int blend_common_checks(const mgs_projected *proj, const uint32_t *offs, const uint32_t *gids,
                               const mgs_camera *cam, int tile, const float *bg, float amin, float amax,
                               float *image) {
    int rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    MGS_REQUIRE(proj != nullptr, "projected is NULL");
    if (tile != MGS_TILE) return set_error(MGS_ERR_UNSUPPORTED, "tile must be %d", MGS_TILE);
    MGS_REQUIRE(offs && image && bg, "tile_offsets / image / bg is NULL");
    MGS_REQUIRE(amin > 0.f && amin < 1.f && amax > amin && amax < 1.f, "bad alpha range");
    MGS_REQUIRE(aligned(proj->splat, 16), "splat must be 16-byte aligned");
    (void)gids;
    return MGS_OK;
}

}  // namespace mgs

namespace mgs {

// One workgroup per tile, Eq. 2 (wbg = EQ2_COMPOSITE) or Eq. 1 composite.
inline int blend_whole_tiles(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                             const mgs_camera *cam, int tile, const float bg[3], float wbg, float alpha_min,
                             float alpha_max, float *image, float *aux, void *stream) {
    int rc;
    if ((rc = blend_common_checks(proj, tile_offsets, gids, cam, tile, bg, alpha_min, alpha_max, image)) != MGS_OK)
        return rc;
    const CamK k = make_camk(cam);
    const unsigned ntiles = unsigned(k.tiles_x) * unsigned(k.tiles_y);
    hipLaunchKernelGGL(blend_kernel<false>, dim3(ntiles), dim3(BLEND_THREADS), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, k, bg[0], bg[1], bg[2], wbg,
                       log2f(alpha_min), alpha_max, 0.0f, image, aux);
    MGS_LAUNCH_CHECK("blend_kernel<oit>");
    return MGS_OK;
}

// Split tile lists, Eq. 2 (wbg = EQ2_COMPOSITE) or Eq. 1 composite.
inline int blend_split_single(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                              const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, int tile,
                              const float bg[3], float wbg, float alpha_min, float alpha_max, void *ws,
                              size_t ws_bytes, float *image, float *aux, void *stream) {
    int rc;
    if ((rc = blend_common_checks(proj, tile_offsets, gids, cam, tile, bg, alpha_min, alpha_max, image)) != MGS_OK)
        return rc;
    MGS_REQUIRE(n_pairs != nullptr, "n_pairs is NULL");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    const CamK k = make_camk(cam);
    MGS_REQUIRE(uint64_t(k.tiles_x) * uint64_t(k.tiles_y) < (uint64_t(1) << 24), "2^24 or more tiles");
    const uint32_t T = uint32_t(k.tiles_x) * uint32_t(k.tiles_y);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= blend_split_workspace(T, capacity), "workspace too small");
    SingleViewLoc loc{k.tiles_x, k.W, k.H, {bg[0], bg[1], bg[2]}, wbg, image, aux};
    return blend_split_launch(reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, nullptr, T, n_pairs,
                              capacity, loc, alpha_min, alpha_max, ws, as_stream(stream));
}

}  // namespace mgs

extern "C" int mgs_blend_oit(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                             const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                             float alpha_max, float *image, float *aux, void *stream) {
    MGS_TRACE("mgs_blend_oit");
    return mgs::blend_whole_tiles(proj, tile_offsets, gids, cam, tile, bg, mgs::EQ2_COMPOSITE, alpha_min, alpha_max,
                                  image, aux, stream);
}

extern "C" int mgs_blend_sortfree(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                  const mgs_camera *cam, int tile, const float bg[3], float w_bg, float alpha_min,
                                  float alpha_max, float *image, float *aux, void *stream) {
    MGS_TRACE("mgs_blend_sortfree");
    MGS_REQUIRE(w_bg >= 0.0f && w_bg < INFINITY, "w_bg must be finite and >= 0");
    return mgs::blend_whole_tiles(proj, tile_offsets, gids, cam, tile, bg, w_bg, alpha_min, alpha_max, image, aux,
                                  stream);
}

extern "C" int mgs_blend_sorted(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                                float alpha_max, float t_stop, float *image, void *stream) {
    MGS_TRACE("mgs_blend_sorted");
    using namespace mgs;
    int rc;
    if ((rc = blend_common_checks(proj, tile_offsets, gids, cam, tile, bg, alpha_min, alpha_max, image)) != MGS_OK)
        return rc;
    MGS_REQUIRE(t_stop >= 0.f && t_stop < 1.f, "t_stop must be in [0, 1)");
    const CamK k = make_camk(cam);
    const unsigned ntiles = unsigned(k.tiles_x) * unsigned(k.tiles_y);
    hipLaunchKernelGGL(blend_kernel<true>, dim3(ntiles), dim3(BLEND_THREADS), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(proj->splat), tile_offsets, gids, k, bg[0], bg[1], bg[2],
                       EQ2_COMPOSITE, log2f(alpha_min), alpha_max, t_stop, image, nullptr);
    MGS_LAUNCH_CHECK("blend_kernel<sorted>");
    return MGS_OK;
}

extern "C" int mgs_blend_oit_split_workspace(int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes) {
    MGS_REQUIRE(bytes && tiles_x > 0 && tiles_y > 0, "bad arguments");
    MGS_REQUIRE(uint64_t(tiles_x) * uint64_t(tiles_y) < (uint64_t(1) << 24), "2^24 or more tiles");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    *bytes = mgs::blend_split_workspace(uint32_t(tiles_x) * uint32_t(tiles_y), capacity);
    return MGS_OK;
}

extern "C" int mgs_blend_oit_split(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                   const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, int tile,
                                   const float bg[3], float alpha_min, float alpha_max, void *ws, size_t ws_bytes,
                                   float *image, float *aux, void *stream) {
    MGS_TRACE("mgs_blend_oit_split");
    return mgs::blend_split_single(proj, tile_offsets, gids, n_pairs, capacity, cam, tile, bg, mgs::EQ2_COMPOSITE,
                                   alpha_min, alpha_max, ws, ws_bytes, image, aux, stream);
}

extern "C" int mgs_blend_sortfree_split(const mgs_projected *proj, const uint32_t *tile_offsets,
                                        const uint32_t *gids, const uint32_t *n_pairs, uint64_t capacity,
                                        const mgs_camera *cam, int tile, const float bg[3], float w_bg,
                                        float alpha_min, float alpha_max, void *ws, size_t ws_bytes, float *image,
                                        float *aux, void *stream) {
    MGS_TRACE("mgs_blend_sortfree_split");
    MGS_REQUIRE(w_bg >= 0.0f && w_bg < INFINITY, "w_bg must be finite and >= 0");
    return mgs::blend_split_single(proj, tile_offsets, gids, n_pairs, capacity, cam, tile, bg, w_bg, alpha_min,
                                   alpha_max, ws, ws_bytes, image, aux, stream);
}

// ---------------------------------------------------------------- census of the blend's work
// One thread per list entry (tile, Gaussian): the quadrant test of the order-independent blend
// (quadrant_mask, the same function) gives the pixels it evaluates (64 per kept quadrant); the
// exponent of Eq. 2 at each of those pixel centres gives the pairs that contribute (alpha >=
// alpha_min).  Wave sums, one 64-bit atomic add per wave and counter (integer: any order).
namespace mgs {

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(256)
blend_census_kernel(const float4 *__restrict__ splat, const uint32_t *__restrict__ offs,
                    const uint32_t *__restrict__ gids, const uint32_t *__restrict__ n_pairs, uint64_t capacity,
                    uint32_t T, int tiles_x, int W, int H, float log2_amin, unsigned long long *__restrict__ counts) {
    const uint32_t P = uint64_t(*n_pairs) > capacity ? 0u : *n_pairs;
    unsigned long long ev = 0, con = 0, pairs = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        // tile of list position i: the last t with offs[t] <= i
        uint32_t lo = 0, hi = T - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const int tx = int(lo % uint32_t(tiles_x)), ty = int(lo / uint32_t(tiles_x));
        const uint32_t g = gids[i];
        const float4 r0 = splat[3 * size_t(g)], r1 = splat[3 * size_t(g) + 1];
        const uint32_t m = quadrant_mask(r0, r1, tx, ty, log2_amin);
        pairs += 1;
        ev += 64ull * __builtin_popcount(m);
        for (int q = 0; q < 4; ++q) {
            if (!((m >> q) & 1u)) continue;
            for (int k = 0; k < 64; ++k) {
                const int px = tx * 16 + (q & 1) * 8 + (k & 7), py = ty * 16 + (q >> 1) * 8 + (k >> 3);
                if (px >= W || py >= H) continue;
                const float dx = float(px) + 0.5f - r0.x, dy = float(py) + 0.5f - r0.y;
                const float t = fmaf(r1.y, dy, dx);
                const float e = r0.z + r1.x * t * t + r1.z * dy * dy;
                con += e >= log2_amin ? 1ull : 0ull;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        ev += __shfl_xor(ev, o, 64);
        con += __shfl_xor(con, o, 64);
        pairs += __shfl_xor(pairs, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(counts + 0, pairs);
        atomicAdd(counts + 1, ev);
        atomicAdd(counts + 2, con);
    }
}

}  // namespace mgs

extern "C" int mgs_blend_census(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, float alpha_min,
                                uint64_t *counts, void *stream) {
    MGS_TRACE("mgs_blend_census");
    using namespace mgs;
    int rc;
    if ((rc = check_camera(cam)) != MGS_OK) return rc;
    MGS_REQUIRE(proj && proj->splat && aligned(proj->splat, 16), "splat is NULL or misaligned");
    MGS_REQUIRE(tile_offsets && gids && n_pairs && counts, "a pointer is NULL");
    MGS_REQUIRE(aligned(counts, 8), "counts must be 8-byte aligned");
    MGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f, "alpha_min must be in (0, 1)");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    const CamK k = make_camk(cam);
    const uint32_t T = uint32_t(k.tiles_x) * uint32_t(k.tiles_y);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long *>(counts), 3);
    MGS_LAUNCH_CHECK("zero_u64_kernel");
    hipLaunchKernelGGL(blend_census_kernel, dim3(2048), dim3(256), 0, s, reinterpret_cast<const float4 *>(proj->splat),
                       tile_offsets, gids, n_pairs, capacity, T, k.tiles_x, k.W, k.H, log2f(alpha_min),
                       reinterpret_cast<unsigned long long *>(counts));
    MGS_LAUNCH_CHECK("blend_census_kernel");
    return MGS_OK;
}

// ---------------------------------------------------------------- no-allocation split blend
// The split blend's workspace (work list, split-tile tables, per-range partial sums) lives in
// this file-scope device array instead of a caller buffer.  Every GPU the library runs on holds
// its own copy until the process ends.  Host code never passes the array's name to a kernel:
// it is a host-side stand-in, not a device address; the device address comes from
// hipGetSymbolAddress, once per device, and is kept in scratch_dev[].
namespace mgs {

static __device__ __align__(256) uint8_t scratch[MGS_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void *scratch_dev[NOALLOC_MAX_DEVICES];

// Device address of the current device's scratch array (looked up on the first call per device).
static int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(MGS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_error(MGS_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[dev] == nullptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return set_error(MGS_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return MGS_OK;
}

}  // namespace mgs

extern "C" int mgs_blend_oit_split_noalloc(const mgs_projected *proj, const uint32_t *tile_offsets,
                                           const uint32_t *gids, const uint32_t *n_pairs, uint64_t capacity,
                                           const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                                           float alpha_max, float *image, float *aux, void *stream) {
    MGS_TRACE("mgs_blend_oit_split_noalloc");
    using namespace mgs;
    int rc;
    // size checks first, so an oversized call is refused before anything touches the device
    MGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "bad camera");
    MGS_REQUIRE(capacity < (uint64_t(1) << 32) - 1, "capacity out of range");
    const uint64_t tx = (uint64_t(cam->width) + MGS_TILE - 1) / MGS_TILE;
    const uint64_t ty = (uint64_t(cam->height) + MGS_TILE - 1) / MGS_TILE;
    MGS_REQUIRE(tx * ty < (uint64_t(1) << 24), "2^24 or more tiles");
    const size_t need = blend_split_workspace(uint32_t(tx * ty), capacity);
    if (need > size_t(MGS_NOALLOC_SCRATCH_BYTES))
        return set_error(MGS_ERR_CAPACITY,
                         "split-blend workspace of %zu bytes (%llu tiles, capacity %llu) exceeds the %zu-byte "
                         "no-allocation scratch; use mgs_blend_oit_split with a caller workspace",
                         need, (unsigned long long)(tx * ty), (unsigned long long)capacity,
                         size_t(MGS_NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    if ((rc = scratch_address(&ws)) != MGS_OK) return rc;
    return blend_split_single(proj, tile_offsets, gids, n_pairs, capacity, cam, tile, bg, EQ2_COMPOSITE, alpha_min,
                              alpha_max, ws, size_t(MGS_NOALLOC_SCRATCH_BYTES), image, aux, stream);
}

// Host replay of the kernels' index arithmetic (paper_2603_11531_amd/csrc/index_math.h) against
// brute-force enumerations, built with the address and undefined-behaviour sanitizers by
// tests/test_index_math.py.  Every index is checked against the bound its workspace is sized
// with; a failure prints the case and exits non-zero.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "index_math.h"

using namespace mgs;

static int fails = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            if (fails < 20) {                             \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
                std::printf(__VA_ARGS__);                 \
                std::printf("\n");                        \
            }                                             \
            ++fails;                                      \
        }                                                 \
    } while (0)

// Split plan: the ranges of one list partition it, at most 255, none empty; over a view, items
// and partial-sum slots stay within the workspace bounds.
static void check_split(std::mt19937_64 &rng) {
    const uint32_t special[] = {0u, 1u, 2u, 1023u, 1024u, 1025u, 2048u, SPLIT_RANGE - 1u, SPLIT_RANGE,
                                SPLIT_RANGE + 1u, 255u * 1024u, 255u * 1024u + 1u, 255u * SPLIT_RANGE,
                                255u * SPLIT_RANGE + 1u, 300000u, 1u << 20, (1u << 24) + 7u, 0x7FFFFFFFu,
                                0xFFFFFFFEu};
    for (uint32_t L : special) {
        const uint32_t n = n_ranges(L, SPLIT_RANGE), len = range_len(L, SPLIT_RANGE);
        CHECK(n >= 1 && n <= SPLIT_MAX_RANGES, "L=%u n=%u", L, n);
        if (L == 0) continue;
        CHECK(uint64_t(n - 1) * len < L, "L=%u: range %u starts past the end", L, n - 1);
        CHECK(uint64_t(n) * len >= L, "L=%u: ranges do not cover the list", L);
        CHECK(L <= uint64_t(SPLIT_MAX_RANGES) * SPLIT_RANGE ? len <= SPLIT_RANGE : true, "L=%u len=%u", L, len);
    }
    for (int trial = 0; trial < 400; ++trial) {
        const uint32_t T = 1 + uint32_t(rng() % 9000);
        const uint64_t cap = uint64_t(rng() % 40000000);
        // tile list lengths summing to at most cap: a heavy-tailed draw, scaled down to fit
        std::vector<uint64_t> len(T);
        uint64_t sum = 0;
        for (auto &v : len) {
            const double u = std::uniform_real_distribution<double>(0.0, 1.0)(rng);
            v = uint64_t(u * u * u * u * 40000.0 * (rng() % 4 == 0 ? 30.0 : 1.0));
            sum += v;
        }
        if (sum > cap && sum > 0)
            for (auto &v : len) v = v * cap / sum;
        uint64_t items = 0, slots = 0, P = 0;
        for (uint32_t t = 0; t < T; ++t) {
            const uint32_t L = uint32_t(len[t]), n = n_ranges(L, SPLIT_RANGE);
            items += n;
            slots += n > 1 ? n : 0;
            P += L;
        }
        CHECK(P <= cap, "trial %d: P %llu > cap", trial, (unsigned long long)P);
        CHECK(items <= split_max_items(T, cap), "trial %d: %llu items > bound %llu", trial,
              (unsigned long long)items, (unsigned long long)split_max_items(T, cap));
        CHECK(slots <= split_max_slots(cap), "trial %d: %llu slots > bound %llu", trial, (unsigned long long)slots,
              (unsigned long long)split_max_slots(cap));
    }
}

// Two-level binning: supertile counts, keys, masks and chunk bounds against an enumeration of
// every tile of every rectangle.
static void check_binning(std::mt19937_64 &rng) {
    for (int trial = 0; trial < 20000; ++trial) {
        const uint32_t tiles_x = 1 + uint32_t(rng() % (trial % 10 == 0 ? 65535 : 300));
        const uint32_t tiles_y = 1 + uint32_t(rng() % (trial % 10 == 1 ? 65535 : 200));
        TileRect r;
        r.x0 = uint32_t(rng() % tiles_x);
        r.y0 = uint32_t(rng() % tiles_y);
        const uint32_t w = uint32_t(rng() % (trial % 7 == 0 ? 200 : 12)), h = uint32_t(rng() % (trial % 5 == 0 ? 200 : 12));
        r.x1 = r.x0 + w < tiles_x ? r.x0 + w : tiles_x - 1;
        r.y1 = r.y0 + h < tiles_y ? r.y0 + h : tiles_y - 1;
        const uint32_t lo = r.x0 | (r.y0 << 16), hi = r.x1 | (r.y1 << 16);
        const TileRect u = unpack_rect(lo, hi);
        CHECK(u.x0 == r.x0 && u.y0 == r.y0 && u.x1 == r.x1 && u.y1 == r.y1, "rect packing");
        const uint32_t st_x = (tiles_x + SUPER - 1) / SUPER, st_y = (tiles_y + SUPER - 1) / SUPER;
        const uint64_t n_tiles = uint64_t(r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1);
        uint32_t ns = 0;
        uint64_t covered = 0;
        for (uint32_t sy = r.y0 >> SUPER_SHIFT; sy <= (r.y1 >> SUPER_SHIFT); ++sy)
            for (uint32_t sx = r.x0 >> SUPER_SHIFT; sx <= (r.x1 >> SUPER_SHIFT); ++sx) {
                ++ns;
                const uint32_t id = sy * st_x + sx;
                CHECK(id < st_x * st_y, "supertile id %u out of %u", id, st_x * st_y);
                const uint32_t key = super_entry_key(id, r, sx, sy);
                CHECK((key >> ST_KEY_SHIFT) == id || uint64_t(id) >= (1u << (32 - ST_KEY_SHIFT)),
                      "key id %u != %u", key >> ST_KEY_SHIFT, id);
                const uint64_t m = local_mask(key);
                uint64_t brute = 0;
                for (uint32_t ky = 0; ky < uint32_t(SUPER); ++ky)
                    for (uint32_t kx = 0; kx < uint32_t(SUPER); ++kx) {
                        const uint32_t tx = sx * SUPER + kx, ty = sy * SUPER + ky;
                        if (tx >= r.x0 && tx <= r.x1 && ty >= r.y0 && ty <= r.y1) brute |= 1ull << (ky * 8 + kx);
                    }
                CHECK(m == brute, "mask of rect (%u,%u)-(%u,%u) in supertile (%u,%u)", r.x0, r.y0, r.x1, r.y1, sx, sy);
                CHECK(m != 0ull, "empty entry");
                covered += uint64_t(__builtin_popcountll(m));
            }
        CHECK(rect_n_super(r) == ns, "n_super %u != %u", rect_n_super(r), ns);
        CHECK(covered == n_tiles, "masks cover %llu of %llu tiles", (unsigned long long)covered,
              (unsigned long long)n_tiles);
        // backward slots: a bijection from the rectangle's tiles onto [first, first + n_tiles)
        const uint32_t first = uint32_t(rng() % 1000000);
        std::vector<char> seen(size_t(n_tiles), 0);
        for (uint32_t ty = r.y0; ty <= r.y1; ++ty)
            for (uint32_t tx = r.x0; tx <= r.x1; ++tx) {
                const uint64_t s = pair_slot(first, r, tx, ty);
                CHECK(s >= first && s < first + n_tiles, "slot %llu outside [%u, +%llu)", (unsigned long long)s, first,
                      (unsigned long long)n_tiles);
                if (s >= first && s < first + n_tiles) {
                    CHECK(!seen[size_t(s - first)], "slot %llu twice", (unsigned long long)s);
                    seen[size_t(s - first)] = 1;
                }
            }
    }
    // level-2 chunks: entries per supertile summing to at most the capacity
    for (int trial = 0; trial < 500; ++trial) {
        const uint64_t S = 1 + rng() % 20000, cap = rng() % 30000000;
        std::vector<uint64_t> e(S);
        uint64_t sum = 0;
        for (auto &v : e) sum += (v = rng() % 50000);
        if (sum > cap && sum > 0)
            for (auto &v : e) v = v * cap / sum;
        uint64_t chunks = 0;
        for (auto v : e) chunks += (v + CHUNK - 1) / CHUNK;
        CHECK(chunks <= bin_max_chunks(cap, S), "trial %d: %llu chunks > bound", trial, (unsigned long long)chunks);
    }
}

int main() {
    std::mt19937_64 rng(20261203);
    check_split(rng);
    check_binning(rng);
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("index arithmetic: all checks passed\n");
    return 0;
}

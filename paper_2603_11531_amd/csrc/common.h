// Internal helpers shared by the gfx950 kernels and the C-ABI glue.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <stdio.h>

#include "mgs.h"

namespace mgs {

// Thread-local error text (defined in status.hip).
int set_error(int code, const char *fmt, ...);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// A roctx range over an entry point's host call (argument checks and enqueue), visible to
// rocprofv3 --marker-trace; a few hundred nanoseconds when no tool listens.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
#define MGS_TRACE(name) ::mgs::TraceRange mgs_trace_range_(name)

inline bool aligned(const void *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

#define MGS_REQUIRE(cond, ...)                                              \
    do {                                                                    \
        if (!(cond)) return ::mgs::set_error(MGS_ERR_INVALID_ARG, __VA_ARGS__); \
    } while (0)

#define MGS_LAUNCH_CHECK(name)                                              \
    do {                                                                    \
        hipError_t e_ = hipGetLastError();                                  \
        if (e_ != hipSuccess)                                               \
            return ::mgs::set_error(MGS_ERR_HIP, "%s: %s", name, hipGetErrorString(e_)); \
    } while (0)

// Camera as passed by value to kernels.
struct CamK {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int W, H;
    float near_z;
    float campos[3];   // t_v = -R^T t
    int tiles_x, tiles_y;
    int weight_mode;   // MGS_WEIGHT_*: Eq. 3, one of its ablations, or Eq. 1's weight
};

inline bool valid_weight_mode(int m) {
    return m == MGS_WEIGHT_EQ3 || m == MGS_WEIGHT_NO_DEPTH || m == MGS_WEIGHT_NO_SCALE;
}

inline CamK make_camk(const mgs_camera *c) {
    CamK k;
    for (int i = 0; i < 9; ++i) k.R[i] = c->R[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c->t[i];
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy;
    k.W = c->width; k.H = c->height; k.near_z = c->near_z;
    for (int i = 0; i < 3; ++i)
        k.campos[i] = -(c->R[0 * 3 + i] * c->t[0] + c->R[1 * 3 + i] * c->t[1] + c->R[2 * 3 + i] * c->t[2]);
    k.tiles_x = (c->width + MGS_TILE - 1) / MGS_TILE;
    k.tiles_y = (c->height + MGS_TILE - 1) / MGS_TILE;
    k.weight_mode = MGS_WEIGHT_EQ3;
    return k;
}

inline int check_camera(const mgs_camera *c) {
    MGS_REQUIRE(c != nullptr, "camera is NULL");
    MGS_REQUIRE(c->width > 0 && c->height > 0, "image size %dx%d must be positive", c->width, c->height);
    MGS_REQUIRE(c->width <= 16 * 65535 && c->height <= 16 * 65535, "image too large");
    MGS_REQUIRE(c->fx > 0.f && c->fy > 0.f, "focal lengths must be positive");
    MGS_REQUIRE(c->near_z > 0.f, "near_z must be positive");
    return MGS_OK;
}

inline int check_gaussians(const mgs_gaussians *g) {
    MGS_REQUIRE(g != nullptr, "gaussians is NULL");
    MGS_REQUIRE(g->n >= 0 && g->n < (int64_t(1) << 31), "n = %lld out of range", (long long)g->n);
    if (g->n == 0) return MGS_OK;
    MGS_REQUIRE(g->mean && g->log_scale && g->quat && g->opacity_logit && g->sh,
                "a Gaussian attribute pointer is NULL");
    return MGS_OK;
}

inline int check_projected(const mgs_projected *p, int64_t n) {
    MGS_REQUIRE(p != nullptr, "projected is NULL");
    if (n == 0) return MGS_OK;
    MGS_REQUIRE(p->splat && p->rect && p->n_tiles, "a projected pointer is NULL");
    MGS_REQUIRE(aligned(p->splat, 16), "splat must be 16-byte aligned");
    MGS_REQUIRE(aligned(p->rect, 8), "rect must be 8-byte aligned");
    MGS_REQUIRE(aligned(p->n_tiles, 4), "n_tiles must be 4-byte aligned");
    return MGS_OK;
}

constexpr float LOG2E = 1.4426950408889634f;

// ---------------------------------------------------------------- checked builds
// A build with -DMGS_CHECK_BOUNDS checks the indices the kernels derive (list positions against
// the pair count, list writes against the capacity, rectangles against the tile grid, backward
// slots against the capacity).  A failed check sets its site's bit in this translation unit's
// flag word and the access is skipped, so a wrong index is reported, never followed;
// mgs_bounds_status() gathers the words of every translation unit.  Without the macro a
// MGS_CHECK is the constant true and a MGS_GUARD its condition.
enum BoundsSite : uint32_t {
    BS_EXPAND_WRITE = 1u << 0,     // level-1 / sorted-path entry written past the capacity
    BS_RECT_GRID = 1u << 1,        // a rectangle outside the tile grid
    BS_LIST_WRITE = 1u << 2,       // a tile-list write past the pair count
    BS_LIST_READ = 1u << 3,        // a tile-list range past the pair count
    BS_SPLIT_ITEM = 1u << 4,       // a split-blend work item or slot past its workspace bound
    BS_BWD_SLOT = 1u << 5,         // a backward pair slot past the capacity
    BS_BWD_ITEM = 1u << 6,         // a backward work item past its workspace bound
    BS_PRUNE_INDEX = 1u << 7,      // a survivor index past n, or a gather index past its plane
};
#ifdef MGS_CHECK_BOUNDS
static __device__ uint32_t tu_bounds_flags;
__device__ __forceinline__ bool bounds_ok(bool ok, uint32_t site) {
    if (!ok) atomicOr(&tu_bounds_flags, site);
    return ok;
}
// MGS_CHECK: a check a normal build leaves out; MGS_GUARD: a guard every build keeps, which a
// checked build also reports when it fails
#define MGS_CHECK(cond, site) (::mgs::bounds_ok(bool(cond), (site)))
#define MGS_GUARD(cond, site) (::mgs::bounds_ok(bool(cond), (site)))
// Reader / clearer of this translation unit's flag word, registered at load time.
void register_bounds_word(int (*read)(uint32_t *), int (*clear)());
static int tu_bounds_read(uint32_t *out) {
    return hipMemcpyFromSymbol(out, HIP_SYMBOL(tu_bounds_flags), sizeof(uint32_t)) == hipSuccess ? 0 : -1;
}
static int tu_bounds_clear() {
    const uint32_t z = 0;
    return hipMemcpyToSymbol(HIP_SYMBOL(tu_bounds_flags), &z, sizeof(uint32_t)) == hipSuccess ? 0 : -1;
}
namespace {
struct BoundsRegistration {
    BoundsRegistration() { register_bounds_word(&tu_bounds_read, &tu_bounds_clear); }
};
static BoundsRegistration bounds_registration;
}  // namespace
#else
#define MGS_CHECK(cond, site) (true)
#define MGS_GUARD(cond, site) (bool(cond))
#endif

// Device-wide exclusive scan of uint32 values (bin.hip); tmp holds scan_tmp_elems(n) uint64,
// *total receives the sum clamped to 2^32 - 1.
size_t scan_tmp_elems(int64_t n);
int scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *tmp, uint32_t *total, hipStream_t s);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// float32 -> bfloat16 bit pattern, round to nearest even (NaN stays NaN).
__host__ __device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return uint16_t((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_round(float f) {
    uint32_t u = uint32_t(bf16_bits_rne(f)) << 16;
    float r;
    __builtin_memcpy(&r, &u, 4);
    return r;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Exclusive scan of one value per thread over a 1024-thread block (all threads call);
// *total receives the block's sum in every thread.  s_wsum: 16 shared slots.
__device__ __forceinline__ uint64_t block_scan1024(uint64_t v, uint64_t *s_wsum, uint64_t *total) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t u = __shfl_up(inc, o, 64);
        if (l >= o) inc += u;
    }
    if (l == 63) s_wsum[w] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint64_t x = s_wsum[k];
        pre += k < w ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// Items per thread of the single-block planning scans (each thread loads its items
// before the scan, so one global latency covers PLAN_TILE items).
constexpr int PLAN_ITEMS = 4;
constexpr int PLAN_TILE = 1024 * PLAN_ITEMS;

// Planning scans run over chunks of PLAN_TILE items, one 1024-thread block per chunk: a
// first pass writes every chunk's totals, part_scan_kernel turns them into exclusive chunk
// offsets in one block, and a second pass redoes its chunk's block scan from that offset and
// writes the outputs.  Chunks past the live item count contribute zero.
__host__ __device__ __forceinline__ uint32_t plan_chunks(uint64_t n_items) {
    return uint32_t((n_items + PLAN_TILE - 1) / PLAN_TILE);
}
inline unsigned plan_grid(uint32_t chunks) { return chunks == 0 ? 1u : (chunks < 1024u ? chunks : 1024u); }
// Up to this many chunks a planning scan runs as one block with a running carry (one launch
// instead of three: a launch costs a few microseconds even when it has little to do).
constexpr uint32_t PLAN_ONE_BLOCK = 4;

// Exclusive scan in place of a[0 .. n) (and of b, if non-NULL); the totals go to *tot_a /
// *tot_b (if non-NULL).
template <int UNUSED = 0>
__global__ void __launch_bounds__(1024)
part_scan_kernel(uint64_t *__restrict__ a, uint64_t *__restrict__ b, uint32_t n, uint64_t *__restrict__ tot_a,
                 uint64_t *__restrict__ tot_b) {
    __shared__ uint64_t s_wsum[16];
    uint64_t ca = 0, cb = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        uint64_t ta, tb;
        const uint64_t ea = block_scan1024(i < n ? a[i] : 0u, s_wsum, &ta);
        if (i < n) a[i] = ca + ea;
        ca += ta;
        if (b) {
            const uint64_t eb = block_scan1024(i < n ? b[i] : 0u, s_wsum, &tb);
            if (i < n) b[i] = cb + eb;
            cb += tb;
        }
    }
    if (threadIdx.x == 0) {
        if (tot_a) *tot_a = ca;
        if (tot_b) *tot_b = cb;
    }
}

// Largest j in [0, n) with pre[j] <= v, for a non-decreasing pre with pre[0] <= v.
__device__ __forceinline__ int upper_index(const uint32_t *pre, int n, uint32_t v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace mgs

// Contribution-based pruning (Sec. 3.3): per training iteration, the Gaussians whose opacity
// and whose largest scale both lie under their tau-quantiles gain a vote; at the end of a
// pruning interval the Gaussians with more than I_prune * v votes are removed and the rest
// keep their order.
//
// The quantile is decided exactly, without sorting.  Q_tau interpolates linearly between the
// order statistics x_(k) and x_(k+1), k = floor(tau (N - 1)), so "x < Q_tau" depends only on
// x_(k), on whether tau (N - 1) has a fractional part and on whether x_(k+1) > x_(k):
//   fractional part and x_(k) < x_(k+1):  x < Q  <=>  x <= x_(k)
//   otherwise (Q = x_(k)):                x < Q  <=>  x <  x_(k)
// and x_(k+1) > x_(k) exactly when k + 1 values are <= x_(k).  Sigmoid and exp are strictly
// increasing, so the decisions are taken on the stored opacity logit and the largest stored
// log-scale, mapped to order-preserving 32-bit keys.  x_(k) comes from a radix select over the
// keys: three histogram passes of 11, 11 and 10 bits, the opacity and the scale key together.
// Histograms count with atomics (order-free integer sums), so every result is deterministic.
#include "common.h"

namespace mgs {
namespace {

constexpr int PR_THREADS = 1024;
constexpr int PR_BINS = 2048;                    // bins of the 11-bit passes (the last has 1,024)
constexpr int PR_PASSES = 3;
constexpr int PR_KEYS = 2;                       // opacity, largest scale (criteria bits 0 and 1)
static_assert(MGS_PRUNE_OPACITY == 1 && MGS_PRUNE_SCALE == 2, "criteria bit q selects key q");
constexpr int PR_HIST_WORDS = PR_PASSES * PR_KEYS * PR_BINS;
constexpr unsigned PR_GRID_MAX = 1024;

__host__ __device__ constexpr int pass_shift(int p) { return p == 0 ? 21 : (p == 1 ? 10 : 0); }
__host__ __device__ constexpr int pass_bins(int p) { return p == 2 ? 1024 : PR_BINS; }

// Order-preserving key of a float: -0 and +0 map to one key (they compare equal).
__device__ __forceinline__ uint32_t order_key(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ void gaussian_keys(const float *__restrict__ logit, const float *__restrict__ log_scale,
                                              int64_t n, int64_t g, uint32_t (&key)[PR_KEYS]) {
    key[0] = order_key(logit[g]);
    key[1] = order_key(fmaxf(fmaxf(log_scale[g], log_scale[n + g]), log_scale[2 * n + g]));
}

// Digit search over one pass's histograms of both keys: for key q, the bin b holding rank r[q]
// of the keys that reach this pass, the rank left inside b (r[q] minus the keys in lower bins)
// and b's count.  One block scan serves both keys: their counts share a 64-bit word (each is
// below 2^31, so the low half never carries into the high half).  All 1,024 threads call.
struct Digit {
    uint32_t bin, rank, count;
};
__device__ void select_digits(const uint32_t *__restrict__ h, int bins, const uint32_t (&r)[PR_KEYS],
                              uint64_t *s_wsum, uint32_t (*s_out)[3], Digit (&d)[PR_KEYS]) {
    const int per = bins / PR_THREADS;           // 2 or 1 bins per thread
    const uint32_t b0 = threadIdx.x * per;
    uint32_t c[PR_KEYS][2];
#pragma unroll
    for (int q = 0; q < PR_KEYS; ++q) {
        c[q][0] = h[q * PR_BINS + b0];
        c[q][1] = per > 1 ? h[q * PR_BINS + b0 + 1] : 0u;
    }
    if (threadIdx.x < PR_KEYS) {
        s_out[threadIdx.x][0] = 0u;
        s_out[threadIdx.x][1] = 0u;
        s_out[threadIdx.x][2] = 0u;
    }
    uint64_t tot;
    const uint64_t packed = (uint64_t(c[0][0]) + c[0][1]) | ((uint64_t(c[1][0]) + c[1][1]) << 32);
    const uint64_t below = block_scan1024(packed, s_wsum, &tot);    // its barriers order s_out
#pragma unroll
    for (int q = 0; q < PR_KEYS; ++q) {
        uint64_t acc = q == 0 ? (below & 0xFFFFFFFFull) : (below >> 32);
        for (int j = 0; j < per; ++j) {
            if (c[q][j] > 0 && acc <= r[q] && r[q] < acc + c[q][j]) {
                s_out[q][0] = b0 + j;
                s_out[q][1] = uint32_t(r[q] - acc);
                s_out[q][2] = c[q][j];
            }
            acc += c[q][j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PR_KEYS; ++q) d[q] = Digit{s_out[q][0], s_out[q][1], s_out[q][2]};
    __syncthreads();
}

// The key prefixes selected by passes 0 .. pass-1 (for both keys), and the ranks left.
struct SelectState {
    uint32_t prefix[PR_KEYS], rank[PR_KEYS], count[PR_KEYS];
};
__device__ SelectState select_through(const uint32_t *__restrict__ hist, int passes, uint32_t k, uint64_t *s_wsum,
                                      uint32_t (*s_out)[3]) {
    SelectState st;
    for (int q = 0; q < PR_KEYS; ++q) {
        st.prefix[q] = 0u;
        st.rank[q] = k;
        st.count[q] = 0u;
    }
    for (int p = 0; p < passes; ++p) {
        Digit d[PR_KEYS];
        select_digits(hist + p * PR_KEYS * PR_BINS, pass_bins(p), st.rank, s_wsum, s_out, d);
        for (int q = 0; q < PR_KEYS; ++q) {
            st.prefix[q] = (st.prefix[q] << (p == 2 ? 10 : 11)) | d[q].bin;
            st.rank[q] = d[q].rank;
            st.count[q] = d[q].count;
        }
    }
    return st;
}

__global__ void __launch_bounds__(PR_THREADS) prune_zero_kernel(uint32_t *__restrict__ hist) {
    for (int i = threadIdx.x; i < PR_HIST_WORDS; i += PR_THREADS) hist[i] = 0u;
}

// One radix pass: histogram of this pass's digit over the keys whose higher digits match the
// prefixes selected so far.
template <int PASS>
__global__ void __launch_bounds__(PR_THREADS)
prune_hist_kernel(const float *__restrict__ logit, const float *__restrict__ log_scale, int64_t n, uint32_t k,
                  uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[PR_KEYS][PR_BINS];
    __shared__ uint64_t s_wsum[16];
    __shared__ uint32_t s_out[PR_KEYS][3];
    constexpr int shift = pass_shift(PASS), bins = pass_bins(PASS);
    for (int i = threadIdx.x; i < PR_KEYS * PR_BINS; i += PR_THREADS) (&s_h[0][0])[i] = 0u;
    __syncthreads();
    const SelectState st = select_through(hist, PASS, k, s_wsum, s_out);
    for (int64_t g = int64_t(blockIdx.x) * PR_THREADS + threadIdx.x; g < n; g += int64_t(gridDim.x) * PR_THREADS) {
        uint32_t key[PR_KEYS];
        gaussian_keys(logit, log_scale, n, g, key);
#pragma unroll
        for (int q = 0; q < PR_KEYS; ++q) {
            const bool match = PASS == 0 || (key[q] >> (shift + (PASS == 1 ? 11 : 10))) == st.prefix[q];
            if (match) atomicAdd(&s_h[q][(key[q] >> shift) & uint32_t(bins - 1)], 1u);
        }
    }
    __syncthreads();
    uint32_t *out = hist + PASS * PR_KEYS * PR_BINS;
    for (int i = threadIdx.x; i < PR_KEYS * PR_BINS; i += PR_THREADS) {
        const uint32_t c = (&s_h[0][0])[i];
        if (c) atomicAdd(out + i, c);
    }
}

// The votes: x_(k) of both keys from the three passes, then per Gaussian the candidate test
// and votes[g] += candidate (candidates[g] too, if requested).
__global__ void __launch_bounds__(PR_THREADS)
prune_vote_kernel(const float *__restrict__ logit, const float *__restrict__ log_scale, int64_t n, uint32_t k,
                  int frac, int criteria, const uint32_t *__restrict__ hist, uint32_t *__restrict__ votes,
                  uint8_t *__restrict__ candidates) {
    __shared__ uint64_t s_wsum[16];
    __shared__ uint32_t s_out[PR_KEYS][3];
    const SelectState st = select_through(hist, PR_PASSES, k, s_wsum, s_out);
    bool inclusive[PR_KEYS];
#pragma unroll
    for (int q = 0; q < PR_KEYS; ++q) {
        // keys <= x_(k): k - rank (strictly below) + count (equal); x_(k+1) > x_(k) iff that is k + 1
        const uint64_t le = uint64_t(k) - st.rank[q] + st.count[q];
        inclusive[q] = frac && le == uint64_t(k) + 1;
    }
    for (int64_t g = int64_t(blockIdx.x) * PR_THREADS + threadIdx.x; g < n; g += int64_t(gridDim.x) * PR_THREADS) {
        uint32_t key[PR_KEYS];
        gaussian_keys(logit, log_scale, n, g, key);
        bool cand = true;                        // the criteria selected (bit q: key q), all must hold
#pragma unroll
        for (int q = 0; q < PR_KEYS; ++q)
            cand = cand && (!((criteria >> q) & 1) || (inclusive[q] ? key[q] <= st.prefix[q] : key[q] < st.prefix[q]));
        votes[g] += cand ? 1u : 0u;
        if (candidates) candidates[g] = cand ? 1 : 0;
    }
}

// Compaction over chunks of PLAN_TILE Gaussians (PLAN_ITEMS per thread): kept counts per chunk,
// their exclusive scan (part_scan_kernel), then each chunk's kept indices from its offset.
__device__ __forceinline__ uint32_t keep_bits(const uint32_t *__restrict__ votes, int64_t n, uint32_t max_votes,
                                              uint64_t c, int64_t &g0) {
    g0 = int64_t(c) * PLAN_TILE + int64_t(threadIdx.x) * PLAN_ITEMS;
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < PLAN_ITEMS; ++j)
        if (g0 + j < n && votes[g0 + j] <= max_votes) bits |= 1u << j;
    return bits;
}

__global__ void __launch_bounds__(1024)
prune_count_kernel(const uint32_t *__restrict__ votes, int64_t n, uint32_t max_votes, uint64_t *__restrict__ part) {
    __shared__ uint64_t s_wsum[16];
    for (uint32_t c = blockIdx.x; c < plan_chunks(uint64_t(n)); c += gridDim.x) {
        int64_t g0;
        const uint32_t bits = keep_bits(votes, n, max_votes, c, g0);
        uint64_t t;
        block_scan1024(__builtin_popcount(bits), s_wsum, &t);
        if (threadIdx.x == 0) part[c] = t;
    }
}

__global__ void __launch_bounds__(1024)
prune_write_kernel(uint32_t *__restrict__ votes, int64_t n, uint32_t max_votes, const uint64_t *__restrict__ part,
                   const uint64_t *__restrict__ total, uint32_t *__restrict__ keep_index, uint32_t *__restrict__ n_keep) {
    __shared__ uint64_t s_wsum[16];
    for (uint32_t c = blockIdx.x; c < plan_chunks(uint64_t(n)); c += gridDim.x) {
        int64_t g0;
        const uint32_t bits = keep_bits(votes, n, max_votes, c, g0);
        uint64_t t;
        uint64_t o = part[c] + block_scan1024(__builtin_popcount(bits), s_wsum, &t);
#pragma unroll
        for (int j = 0; j < PLAN_ITEMS; ++j) {
            if (g0 + j < n) {
                if ((bits >> j) & 1u) {
                    if (MGS_CHECK(o < uint64_t(n), BS_PRUNE_INDEX)) keep_index[o] = uint32_t(g0 + j);
                    ++o;
                }
                votes[g0 + j] = 0u;              // the next interval counts from zero
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_keep = uint32_t(*total);
}

// dst[p][i] = src[p][index[i]] for i < *n_index, p < planes.
__global__ void __launch_bounds__(256)
gather_planes_kernel(const float *__restrict__ src, int64_t src_stride, int planes, const uint32_t *__restrict__ index,
                     const uint32_t *__restrict__ n_index, int64_t n_max, float *__restrict__ dst, int64_t dst_stride) {
    const int64_t m = *n_index < uint64_t(n_max) ? int64_t(*n_index) : n_max;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < m; i += int64_t(gridDim.x) * 256) {
        const int64_t s = index[i];
        if (!MGS_CHECK(s < src_stride, BS_PRUNE_INDEX)) continue;
        for (int p = 0; p < planes; ++p) dst[p * dst_stride + i] = src[p * src_stride + s];
    }
}

struct PruneLayout {
    size_t hist, part, total, bytes;
};
PruneLayout prune_layout(int64_t n) {
    PruneLayout L;
    size_t o = 0;
    L.hist = o;  o = align_up(o + size_t(PR_HIST_WORDS) * 4, 256);
    L.part = o;  o = align_up(o + (size_t(plan_chunks(uint64_t(n))) + 1) * 8, 256);
    L.total = o; o = align_up(o + 8, 256);
    L.bytes = o;
    return L;
}

unsigned stream_grid(int64_t n) {
    const int64_t b = (n + 4 * PR_THREADS - 1) / (4 * PR_THREADS);
    return unsigned(b < 1 ? 1 : (b > PR_GRID_MAX ? PR_GRID_MAX : b));
}

}  // namespace
}  // namespace mgs

extern "C" int mgs_prune_workspace(int64_t n, size_t *bytes) {
    MGS_REQUIRE(bytes, "bytes is NULL");
    MGS_REQUIRE(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31)");
    *bytes = mgs::prune_layout(n).bytes;
    return MGS_OK;
}

extern "C" int mgs_prune_vote(const float *opacity_logit, const float *log_scale, int64_t n, double tau, int criteria,
                              void *ws, size_t ws_bytes, uint32_t *votes, uint8_t *candidates, void *stream) {
    MGS_TRACE("mgs_prune_vote");
    using namespace mgs;
    MGS_REQUIRE(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31)");
    MGS_REQUIRE(tau >= 0.0 && tau <= 1.0, "tau must be in [0, 1]");
    MGS_REQUIRE(criteria >= 1 && criteria <= (MGS_PRUNE_OPACITY | MGS_PRUNE_SCALE), "unknown criteria %d", criteria);
    if (n == 0) return MGS_OK;
    MGS_REQUIRE(opacity_logit && log_scale && votes, "opacity_logit / log_scale / votes is NULL");
    const PruneLayout L = prune_layout(n);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.bytes, "workspace too small or not 256-byte aligned");
    // k = floor(tau (N - 1)) and whether tau (N - 1) has a fractional part, in double
    const double h = tau * double(n - 1);
    const double kf = floor(h);
    const uint32_t k = uint32_t(kf);
    const int frac = h > kf ? 1 : 0;
    uint32_t *hist = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + L.hist);
    hipStream_t s = as_stream(stream);
    const unsigned grid = stream_grid(n);
    hipLaunchKernelGGL(prune_zero_kernel, dim3(1), dim3(PR_THREADS), 0, s, hist);
    MGS_LAUNCH_CHECK("prune_zero_kernel");
    hipLaunchKernelGGL(prune_hist_kernel<0>, dim3(grid), dim3(PR_THREADS), 0, s, opacity_logit, log_scale, n, k, hist);
    MGS_LAUNCH_CHECK("prune_hist_kernel<0>");
    hipLaunchKernelGGL(prune_hist_kernel<1>, dim3(grid), dim3(PR_THREADS), 0, s, opacity_logit, log_scale, n, k, hist);
    MGS_LAUNCH_CHECK("prune_hist_kernel<1>");
    hipLaunchKernelGGL(prune_hist_kernel<2>, dim3(grid), dim3(PR_THREADS), 0, s, opacity_logit, log_scale, n, k, hist);
    MGS_LAUNCH_CHECK("prune_hist_kernel<2>");
    hipLaunchKernelGGL(prune_vote_kernel, dim3(grid), dim3(PR_THREADS), 0, s, opacity_logit, log_scale, n, k, frac,
                       criteria, static_cast<const uint32_t *>(hist), votes, candidates);
    MGS_LAUNCH_CHECK("prune_vote_kernel");
    return MGS_OK;
}

extern "C" int mgs_prune_compact(uint32_t *votes, int64_t n, uint32_t max_votes, void *ws, size_t ws_bytes,
                                 uint32_t *keep_index, uint32_t *n_keep, void *stream) {
    MGS_TRACE("mgs_prune_compact");
    using namespace mgs;
    MGS_REQUIRE(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31)");
    MGS_REQUIRE(n_keep, "n_keep is NULL");
    const PruneLayout L = prune_layout(n);
    MGS_REQUIRE(ws && aligned(ws, 256) && ws_bytes >= L.bytes, "workspace too small or not 256-byte aligned");
    MGS_REQUIRE(n == 0 || (votes && keep_index), "votes / keep_index is NULL");
    char *w = static_cast<char *>(ws);
    uint64_t *part = reinterpret_cast<uint64_t *>(w + L.part);
    uint64_t *total = reinterpret_cast<uint64_t *>(w + L.total);
    hipStream_t s = as_stream(stream);
    const uint32_t nc = plan_chunks(uint64_t(n));
    hipLaunchKernelGGL(prune_count_kernel, dim3(plan_grid(nc)), dim3(1024), 0, s, static_cast<const uint32_t *>(votes),
                       n, max_votes, part);
    MGS_LAUNCH_CHECK("prune_count_kernel");
    hipLaunchKernelGGL(part_scan_kernel<>, dim3(1), dim3(1024), 0, s, part, static_cast<uint64_t *>(nullptr), nc, total,
                       static_cast<uint64_t *>(nullptr));
    MGS_LAUNCH_CHECK("part_scan_kernel");
    hipLaunchKernelGGL(prune_write_kernel, dim3(plan_grid(nc)), dim3(1024), 0, s, votes, n, max_votes,
                       static_cast<const uint64_t *>(part), static_cast<const uint64_t *>(total), keep_index, n_keep);
    MGS_LAUNCH_CHECK("prune_write_kernel");
    return MGS_OK;
}

extern "C" int mgs_gather_planes(const float *src, int64_t src_stride, int planes, const uint32_t *index,
                                 const uint32_t *n_index, int64_t n_max, float *dst, int64_t dst_stride, void *stream) {
    MGS_TRACE("mgs_gather_planes");
    using namespace mgs;
    MGS_REQUIRE(planes >= 1 && n_max >= 0 && n_max <= int64_t(INT32_MAX), "planes must be >= 1, n_max in [0, 2^31)");
    MGS_REQUIRE(dst_stride >= n_max && src_stride >= 1, "dst_stride must be >= n_max, src_stride >= 1");
    if (n_max == 0) return MGS_OK;
    MGS_REQUIRE(src && index && n_index && dst, "src / index / n_index / dst is NULL");
    const int64_t b = (n_max + 255) / 256;
    hipLaunchKernelGGL(gather_planes_kernel, dim3(unsigned(b < 2048 ? b : 2048)), dim3(256), 0, as_stream(stream), src,
                       src_stride, planes, index, n_index, n_max, dst, dst_stride);
    MGS_LAUNCH_CHECK("gather_planes_kernel");
    return MGS_OK;
}

// Reference sort for measurement only: ROCm's library radix sort (hipCUB over rocPRIM's onesweep
// sort) of the same 64-bit (tile << 32 | depth bits) keys and 32-bit Gaussian ids that the sorted
// comparison path sorts with its own kernels (mgs_bin_sorted).  It is not part of any render;
// bench.py times it beside mgs_bin_sorted to show what a library sort of those keys costs on
// this device.  Built into libmgs_refsort.so, separate from libmgs.so.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

extern "C" int mgs_ref_sort_workspace(int64_t n, int end_bit, size_t *bytes) {
    if (bytes == nullptr || n < 0 || n > INT32_MAX || end_bit < 1 || end_bit > 64) return -1;
    size_t tmp = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<const uint64_t *>(nullptr),
                                                      static_cast<uint64_t *>(nullptr),
                                                      static_cast<const uint32_t *>(nullptr),
                                                      static_cast<uint32_t *>(nullptr), int(n), 0, end_bit);
    if (e != hipSuccess) return -3;
    *bytes = tmp;
    return 0;
}

// Sorts n (key, value) pairs by key bits [0, end_bit) into keys_out / vals_out (device buffers,
// caller-owned, inputs unchanged); tmp: mgs_ref_sort_workspace bytes.  Returns 0, -1 for bad
// arguments, -3 for a HIP error.
extern "C" int mgs_ref_sort_pairs(const uint64_t *keys_in, uint64_t *keys_out, const uint32_t *vals_in,
                                  uint32_t *vals_out, int64_t n, int end_bit, void *tmp, size_t tmp_bytes,
                                  void *stream) {
    if (n < 0 || n > INT32_MAX || end_bit < 1 || end_bit > 64) return -1;
    if (n > 0 && (!keys_in || !keys_out || !vals_in || !vals_out || !tmp)) return -1;
    size_t need = 0;
    if (mgs_ref_sort_workspace(n, end_bit, &need) != 0 || tmp_bytes < need) return -1;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys_in, keys_out, vals_in, vals_out, int(n), 0,
                                                      end_bit, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -3;
}

// Segmented variant: the n (depth bits, Gaussian id) pairs of the order-independent binning's
// lists sorted by depth inside each tile list, list t being [offsets[t], offsets[t + 1]) for
// t < n_segments (a stable sort of lists in ascending id: ties stay in id order).  Measurement
// only, as above; tmp: mgs_ref_segsort_workspace bytes.
extern "C" int mgs_ref_segsort_workspace(int64_t n, int n_segments, size_t *bytes) {
    if (bytes == nullptr || n < 0 || n > INT32_MAX || n_segments < 0) return -1;
    size_t tmp = 0;
    hipError_t e = hipcub::DeviceSegmentedRadixSort::SortPairs(
        nullptr, tmp, static_cast<const uint32_t *>(nullptr), static_cast<uint32_t *>(nullptr),
        static_cast<const uint32_t *>(nullptr), static_cast<uint32_t *>(nullptr), int(n), n_segments,
        static_cast<const uint32_t *>(nullptr), static_cast<const uint32_t *>(nullptr), 0, 32);
    if (e != hipSuccess) return -3;
    *bytes = tmp;
    return 0;
}

extern "C" int mgs_ref_segsort_pairs(const uint32_t *keys_in, uint32_t *keys_out, const uint32_t *vals_in,
                                     uint32_t *vals_out, int64_t n, const uint32_t *offsets, int n_segments,
                                     void *tmp, size_t tmp_bytes, void *stream) {
    if (n < 0 || n > INT32_MAX || n_segments < 0) return -1;
    if (n > 0 && (!keys_in || !keys_out || !vals_in || !vals_out || !offsets || !tmp)) return -1;
    size_t need = 0;
    if (mgs_ref_segsort_workspace(n, n_segments, &need) != 0 || tmp_bytes < need) return -1;
    hipError_t e = hipcub::DeviceSegmentedRadixSort::SortPairs(
        tmp, tmp_bytes, keys_in, keys_out, vals_in, vals_out, int(n), n_segments, offsets, offsets + 1, 0, 32,
        reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -3;
}

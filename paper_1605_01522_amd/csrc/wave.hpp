// Wavefront-level helpers over sorted CSR rows shared by the setup kernels
// (one 64-lane wavefront works on one group of rows).
#pragma once

#include <hip/hip_runtime.h>

namespace nf {

// Distinct values of col[k] / g over the sorted row [p0, e0): their number,
// and with `out` the values themselves in ascending order, leaving out
// `skip`.  An entry starts a run when the previous entry has another value.
__device__ __forceinline__ int group_runs(int p0, int e0, int g, const int* __restrict__ col, int skip, int* out) {
  const int lane = threadIdx.x & 63;
  int n = 0, prev = -1;
  for (int base = p0; base < e0; base += 64) {
    const int k = base + lane;
    const int v = k < e0 ? col[k] / g : -1;
    int left = __shfl_up(v, 1, 64);
    if (lane == 0) left = prev;
    const bool first = k < e0 && v != left && v != skip;
    const unsigned long long bal = __ballot(first);
    if (out && first) out[n + __popcll(bal & ((1ull << lane) - 1ull))] = v;
    n += __popcll(bal);
    prev = __shfl(v, 63, 64);
  }
  return n;
}

// True when rows row0 + 1 .. row0 + nrow - 1 each have the same set of
// values col / g as row row0 (n0 distinct values): the same number of
// distinct values, each found in row row0 by binary search.  Wavefront-
// uniform result.
__device__ __forceinline__ bool rows_share_groups(const int* __restrict__ ptr, int row0, int nrow, int g,
                                                  const int* __restrict__ col, int n0) {
  const int lane = threadIdx.x & 63;
  const int p0 = ptr[row0], e0 = ptr[row0 + 1];
  for (int r = 1; r < nrow; ++r) {
    const int pr = ptr[row0 + r], er = ptr[row0 + r + 1];
    if (group_runs(pr, er, g, col, -1, nullptr) != n0) return false;
    bool miss = false;
    for (int k = pr + lane; k < er; k += 64) {
      const int v = col[k] / g;
      int lo = p0, hi = e0;             // first entry of row row0 whose value is >= v
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] / g < v) lo = mid + 1;
        else hi = mid;
      }
      miss |= lo == e0 || col[lo] / g != v;
    }
    if (__ballot(miss) != 0ull) return false;
  }
  return true;
}

}  // namespace nf

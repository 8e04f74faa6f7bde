// Wavefront-level helpers over sorted CSR rows shared by the setup kernels
// (one 64-lane wavefront works on one group of rows).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

namespace nf {

// Distinct values of col[k] / g over the sorted row [p0, e0): their number,
// and with `out` the first `cap` of them in ascending order, leaving out
// `skip`.  An entry starts a run when the previous entry has another value.
__device__ __forceinline__ int group_runs(int p0, int e0, int g, const int* __restrict__ col, int skip, int* out,
                                          int cap = INT_MAX) {
  const int lane = threadIdx.x & 63;
  int n = 0, prev = -1;
  for (int base = p0; base < e0; base += 64) {
    const int k = base + lane;
    const int v = k < e0 ? col[k] / g : -1;
    int left = __shfl_up(v, 1, 64);
    if (lane == 0) left = prev;
    const bool first = k < e0 && v != left && v != skip;
    const unsigned long long bal = __ballot(first);
    const int at = n + __popcll(bal & ((1ull << lane) - 1ull));
    if (out && first && at < cap) out[at] = v;
    n += __popcll(bal);
    prev = __shfl(v, 63, 64);
  }
  return n;
}

// For a workgroup of one wavefront: true when rows row0 + 1 .. row0 + nrow - 1
// each have the same distinct values col / g as row row0.  Row row0's n0
// distinct values go to ref (LDS, the first cap of them; with more than cap
// and nrow > 1: false), and each other row's sorted distinct values are
// compared with them in place.
__device__ __forceinline__ bool rows_share_groups(const int* __restrict__ ptr, int row0, int nrow, int g,
                                                  const int* __restrict__ col, int* ref, int cap, int& n0) {
  const int lane = threadIdx.x & 63;
  n0 = group_runs(ptr[row0], ptr[row0 + 1], g, col, -1, ref, cap);
  if (nrow == 1) return true;
  if (n0 > cap) return false;
  __syncthreads();
  for (int r = 1; r < nrow; ++r) {
    const int pr = ptr[row0 + r], er = ptr[row0 + r + 1];
    int n = 0, prev = -1;
    bool miss = false;
    for (int base = pr; base < er; base += 64) {
      const int k = base + lane;
      const int v = k < er ? col[k] / g : -1;
      int left = __shfl_up(v, 1, 64);
      if (lane == 0) left = prev;
      const bool first = k < er && v != left;
      const unsigned long long bal = __ballot(first);
      const int at = n + __popcll(bal & ((1ull << lane) - 1ull));
      miss |= first && (at >= n0 || ref[at] != v);
      n += __popcll(bal);
      prev = __shfl(v, 63, 64);
    }
    if (n != n0 || __ballot(miss) != 0ull) return false;
  }
  return true;
}

// ascending bitonic sort of keys[0, ts) (ts a power of two) in LDS by a
// workgroup of one wavefront
__device__ inline void wave_bitonic(int* keys, int ts, int lane) {
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < ts; t += 64) {
        const int u = t ^ j;
        if (u > t) {
          const int x = keys[t], y = keys[u];
          if ((x > y) == ((t & kk) == 0)) {
            keys[t] = y;
            keys[u] = x;
          }
        }
      }
      __syncthreads();
    }
}

}  // namespace nf

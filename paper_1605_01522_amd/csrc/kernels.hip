// gfx950 kernels of the n-field solver: vector updates, CSR SpMV with fused
// epilogues (residual, Chebyshev step, prolongate-and-add), deterministic
// FP64 reductions, GMRES block operations, and the AMG setup kernels
// (node graph, MIS-2, aggregation, tentative prolongator, SpGEMM, transpose,
// sparse add, dense Gauss-Jordan inverse).
//
// Wavefronts are 64 lanes.  Reductions use a fixed grid so that every sum is
// taken in the same order on every run.

#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.hpp"
#include "wave.hpp"

namespace nf {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ====================================================================== utils
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over a 256-thread block; result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* ws) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) ws[w] = v;
  __syncthreads();
  return (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a pure function of its
// input: add the golden gamma, then the two xor-shift-multiply rounds.
__device__ __forceinline__ uint64_t smix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ==================================================================== vectors
#define NF_ROWS(n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <class T>
__global__ void k_fill(T* x, T v, int64_t n) { NF_ROWS(n) x[i] = v; }
template <class S, class D>
__global__ void k_cast(const S* x, D* y, int64_t n) { NF_ROWS(n) y[i] = (D)x[i]; }
// multi-column kernels: column k = blockIdx.y
template <class T>
__global__ void k_fillm(T* x, int64_t ldx, T v, int64_t n) {
  T* xk = x + blockIdx.y * ldx;
  NF_ROWS(n) xk[i] = v;
}
template <class S, class D>
__global__ void k_castm(const S* x, int64_t ldx, D* y, int64_t ldy, int64_t n) {
  const S* xk = x + blockIdx.y * ldx;
  D* yk = y + blockIdx.y * ldy;
  NF_ROWS(n) yk[i] = (D)xk[i];
}
template <class T>
__global__ void k_add_intom(const T* d, int64_t ldd, T* x, int64_t ldx, int64_t n, const int* mask) {
  if (mask && !mask[blockIdx.y]) return;
  const T* dk = d + blockIdx.y * ldd;
  T* xk = x + blockIdx.y * ldx;
  NF_ROWS(n) xk[i] += dk[i];
}
template <class T>
__global__ void k_sub_scaledm(const T* dinv, const T* u, int64_t ldu, T* x, int64_t ldx, int64_t n) {
  const T* uk = u + blockIdx.y * ldu;
  T* xk = x + blockIdx.y * ldx;
  NF_ROWS(n) xk[i] -= dinv[i] * uk[i];
}
template <class T>
__global__ void k_cheb_firstm(const T* b, int64_t ldb, const T* dinv, T inv_theta, T* d, int64_t ldd, T* x, int64_t ldx,
                              int64_t n) {
  const T* bk = b + blockIdx.y * ldb;
  T* dk = d + blockIdx.y * ldd;
  T* xk = x + blockIdx.y * ldx;
  NF_ROWS(n) {
    const T v = dinv[i] * bk[i] * inv_theta;
    dk[i] = v;
    xk[i] = v;
  }
}
__global__ void k_scale_inv_devm(const double* w, int64_t ldw, double* v, int64_t ldv, const double* nrm, int stride,
                                 int64_t n, const int* mask, const int* vcol, int64_t vstep) {
  const int k = blockIdx.y;
  if (mask && !mask[k]) return;
  const double sv = nrm[k * stride];
  const double inv = sv != 0.0 ? 1.0 / sv : 1.0;
  const double* wk = w + k * ldw;
  double* vk = v + k * ldv + (vcol ? (int64_t)vcol[k] * vstep : 0);
  NF_ROWS(n) vk[i] = wk[i] * inv;
}
// one wavefront per row of a dense row-major matrix, all columns at once
template <int NR, class T>
__global__ __launch_bounds__(256) void k_dense_gemvm(const double* __restrict__ M, int n, const T* __restrict__ b, int64_t ldb,
                                                    T* __restrict__ x, int64_t ldx, int nrhs) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  const double* m = M + (int64_t)row * n;
  for (int j = lane; j < n; j += 64) {
    const double mj = m[j];
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k < nrhs) acc[k] += mj * (double)b[k * ldb + j];
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k >= nrhs) break;
    const double v = wave_sum(acc[k]);
    if (lane == 0) x[k * ldx + row] = (T)v;
  }
}

static thread_local double g_alg_bytes = 0.0;
void bytes_count(double b) { g_alg_bytes += b; }
// SpMVs inside a set-up (power iterations, ...) do not read block copies,
// which other parts of the set-up may be building at the same time: the
// set-up's results then do not depend on its timing
static thread_local bool g_in_setup = false;
void setup_mode(bool on) { g_in_setup = on; }
bool in_setup() { return g_in_setup; }
double bytes_counted() { return g_alg_bytes; }

static inline int grid_for(int64_t n, int threads = 256) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}
static inline int grid_cols(int64_t n, int nrhs) {
  int64_t g = (n + 255) / 256;
  const int64_t cap = 8192 / (nrhs > 0 ? nrhs : 1);
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

template <class T> void fill(T* x, T v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, s, x, v, n);
}
template <class S, class D> void cast_copy(const S* x, D* y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_cast<S, D>), dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
}
template <class T> void fillm(T* x, int64_t ldx, T v, int64_t n, int nrhs, hipStream_t s) {
  if (n > 0 && nrhs > 0) bytes_count((double)sizeof(T) * n * nrhs);
  if (n > 0 && nrhs > 0) hipLaunchKernelGGL(k_fillm<T>, dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, x, ldx, v, n);
}
template <class S, class D> void castm(const S* x, int64_t ldx, D* y, int64_t ldy, int64_t n, int nrhs, hipStream_t s) {
  if (n > 0 && nrhs > 0) bytes_count((double)(sizeof(S) + sizeof(D)) * n * nrhs);
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL((k_castm<S, D>), dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, x, ldx, y, ldy, n);
}
template <class T> void copym(const T* x, int64_t ldx, T* y, int64_t ldy, int64_t n, int nrhs, hipStream_t s) {
  castm<T, T>(x, ldx, y, ldy, n, nrhs, s);
}
template <class T> void add_intom(const T* d, int64_t ldd, T* x, int64_t ldx, int64_t n, int nrhs, const int* mask,
                                  hipStream_t s) {
  if (n > 0 && nrhs > 0) bytes_count(3.0 * sizeof(T) * n * nrhs);
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_add_intom<T>, dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, d, ldd, x, ldx, n, mask);
}
template <class T> void sub_scaledm(const T* dinv, const T* u, int64_t ldu, T* x, int64_t ldx, int64_t n, int nrhs,
                                    hipStream_t s) {
  if (n > 0 && nrhs > 0) bytes_count((double)sizeof(T) * n * (1 + 3 * nrhs));
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_sub_scaledm<T>, dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, dinv, u, ldu, x, ldx, n);
}
template <class T> void cheb_firstm(const T* b, int64_t ldb, const T* dinv, T inv_theta, T* d, int64_t ldd, T* x,
                                    int64_t ldx, int64_t n, int nrhs, hipStream_t s) {
  if (n > 0 && nrhs > 0) bytes_count((double)sizeof(T) * n * (1 + 3 * nrhs));
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_cheb_firstm<T>, dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, b, ldb, dinv, inv_theta, d, ldd,
                       x, ldx, n);
}
void scale_inv_devm(const double* w, int64_t ldw, double* v, int64_t ldv, const double* nrm, int stride, int64_t n,
                    int nrhs, const int* mask, hipStream_t s, const int* vcol, int64_t vstep) {
  if (n > 0 && nrhs > 0) bytes_count(16.0 * n * nrhs);
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_scale_inv_devm, dim3(grid_cols(n, nrhs), nrhs), dim3(256), 0, s, w, ldw, v, ldv, nrm, stride, n,
                       mask, vcol, vstep);
}
template <class T> void dense_gemvm(const double* M, int n, const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs,
                                    hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  bytes_count(8.0 * n * n + 2.0 * sizeof(T) * n * nrhs);
  if (nrhs == 1) hipLaunchKernelGGL((k_dense_gemvm<1, T>), dim3(cdiv(n, 4)), dim3(256), 0, s, M, n, b, ldb, x, ldx, nrhs);
  else hipLaunchKernelGGL((k_dense_gemvm<NRMAX, T>), dim3(cdiv(n, 4)), dim3(256), 0, s, M, n, b, ldb, x, ldx, nrhs);
}

template void fill<double>(double*, double, int64_t, hipStream_t);
template void fill<float>(float*, float, int64_t, hipStream_t);
template void fill<int>(int*, int, int64_t, hipStream_t);
template void fill<unsigned long long>(unsigned long long*, unsigned long long, int64_t, hipStream_t);
template void cast_copy<double, float>(const double*, float*, int64_t, hipStream_t);
template void cast_copy<float, double>(const float*, double*, int64_t, hipStream_t);
template void fillm<double>(double*, int64_t, double, int64_t, int, hipStream_t);
template void fillm<float>(float*, int64_t, float, int64_t, int, hipStream_t);
template void castm<double, float>(const double*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void castm<float, double>(const float*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void copym<double>(const double*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void copym<float>(const float*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void add_intom<double>(const double*, int64_t, double*, int64_t, int64_t, int, const int*, hipStream_t);
template void add_intom<float>(const float*, int64_t, float*, int64_t, int64_t, int, const int*, hipStream_t);
template void sub_scaledm<double>(const double*, const double*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void sub_scaledm<float>(const float*, const float*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void cheb_firstm<double>(const double*, int64_t, const double*, double, double*, int64_t, double*, int64_t,
                                  int64_t, int, hipStream_t);
template void cheb_firstm<float>(const float*, int64_t, const float*, float, float*, int64_t, float*, int64_t, int64_t,
                                 int, hipStream_t);
template void dense_gemvm<double>(const double*, int, const double*, int64_t, double*, int64_t, int, hipStream_t);
template void dense_gemvm<float>(const double*, int, const float*, int64_t, float*, int64_t, int, hipStream_t);

// ======================================================================= SpMV
// G lanes per row (G divides 64, groups aligned inside the wavefront), NR
// columns at most per launch (the matrix row is read once for all columns).
// Row sums are reduced with xor-shuffles inside the group; lane 0 of the
// group applies the epilogue to every column.
// sum over p = p0, p0 + G, ... < p1 of val[p] x[k ldx + col[p]] into s[k]
// (k < nrhs), in ascending p.  The entries are taken U per lane at a time with
// the loads past p1 masked off, so a lane's share of a typical row (at most 8
// entries with one right-hand side) costs one round trip for the matrix and
// one for the gathered x, instead of a chain of single-entry iterations.
// (Masked, not clamped: a row's tail would otherwise repeat its last entry's
// loads on most of the U positions; measured slower.)  A larger U takes the
// same entries in the same order per lane, in fewer rounds.
template <int G, int NR, class T, int U = (NR == 1 ? 8 : 4)>
__device__ __forceinline__ void row_dot(int p0, int p1, const int* __restrict__ col, const T* __restrict__ val,
                                        const T* __restrict__ x, int64_t ldx, int nrhs, T* s) {
  for (int p = p0; p < p1; p += U * G) {
    T v[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = p + u * G;
      v[u] = q < p1 ? val[q] : (T)0;
      c[u] = q < p1 ? col[q] : -1;
    }
    T xv[U][NR];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) xv[u][k] = (c[u] >= 0 && k < nrhs) ? x[k * ldx + c[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (c[u] >= 0 && k < nrhs) s[k] += v[u] * xv[u][k];
  }
}

template <int G, int MODE, int NR, class T>
__global__ __launch_bounds__(256) void k_spmv(int nr, const int* __restrict__ ptr, const int* __restrict__ col,
                                              const T* __restrict__ val, SpmvArgs<T> a) {
  const int gid = blockIdx.x * 256 + threadIdx.x;
  const int row = gid / G, lane = gid & (G - 1);
  if (row >= nr) return;
  const int p0 = ptr[row], p1 = ptr[row + 1];
  const T* __restrict__ x = a.x;
  const int nrhs = a.nrhs;
  T s[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) s[k] = 0;
  // a wavefront per row (rows of 256 entries or more on average): 16 entries
  // per lane in flight, so rows up to 1,024 entries take one round trip
  row_dot<G, NR, T, (NR == 1 && G == 64) ? 16 : (NR == 1 ? 8 : 4)>(p0 + lane, p1, col, val, x, a.ldx, nrhs, s);
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o, G);
  if (lane != 0) return;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k >= nrhs) break;
    if (MODE == SPMV_STORE) a.y[k * a.ldy + row] = s[k];
    else if (MODE == SPMV_RESID) a.y[k * a.ldy + row] = a.b[k * a.ldb + row] - s[k];
    else if (MODE == SPMV_ADD) a.y[k * a.ldy + row] += s[k];
    else if (MODE == SPMV_SUB) a.y[k * a.ldy + row] -= s[k];
    else if (MODE == SPMV_DSCALE) a.y[k * a.ldy + row] = a.dinv[row] * s[k];
    else {  // SPMV_CHEB
      const T r = a.b[k * a.ldb + row] - s[k];
      T dn = a.c2 * a.dinv[row] * r;
      if (a.c1 != (T)0) dn += a.c1 * a.d[k * a.ldd + row];
      a.d[k * a.ldd + row] = dn;
      a.xo[k * a.ldxo + row] = a.x[k * a.ldx + row] + dn;
    }
  }
}

int spmv_group(int nr, int64_t nnz) {
  if (nr <= 0) return 1;
  const double avg = (double)nnz / nr;
  int g = 1;
  while (g * 2 <= avg && g < 64) g *= 2;
  return g < 2 ? 2 : g;
}
// SpMV rows: two to four entries per lane; four to eight on rows of 64 or
// more entries when that still leaves at least 16,384 wavefronts (measured:
// large matrices with long rows gain from the fewer wavefronts, short rows
// and small matrices lose)
int spmv_lanes(int nr, int64_t nnz) {
  if (nr <= 0) return 2;
  const double avg = (double)nnz / nr;
  int g = 1;
  while (g * 4 <= avg && g < 64) g *= 2;
  if (avg >= 64 && g > 2 && (int64_t)nr * (g / 2) >= (int64_t)64 * 16384) g /= 2;
  return g < 2 ? 2 : g;
}

template <int MODE, int NR, class T>
static void spmv_mode(int G, const DCsr& A, const SpmvArgs<T>& a, const T* val, hipStream_t s) {
  const int blocks = cdiv((int64_t)A.nr * G, 256);
  switch (G) {
    case 2: hipLaunchKernelGGL((k_spmv<2, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
    case 4: hipLaunchKernelGGL((k_spmv<4, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
    case 8: hipLaunchKernelGGL((k_spmv<8, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
    case 16: hipLaunchKernelGGL((k_spmv<16, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
    case 32: hipLaunchKernelGGL((k_spmv<32, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
    default: hipLaunchKernelGGL((k_spmv<64, MODE, NR, T>), dim3(blocks), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, val, a); break;
  }
}
template <int MODE, class T>
static void spmv_nr(int G, const DCsr& A, const SpmvArgs<T>& a, const T* val, hipStream_t s) {
  NF_CHECK(a.nrhs >= 1 && a.nrhs <= NRMAX, NFIELD_EINVAL, "more than 8 right-hand sides in one call");
  if (a.nrhs == 1) spmv_mode<MODE, 1, T>(G, A, a, val, s);
  else spmv_mode<MODE, NRMAX, T>(G, A, a, val, s);
}

template <class T> static const T* csr_values(const DCsr& A);
template <> const double* csr_values<double>(const DCsr& A) {
  if (!A.val.p && A.nnz > 0) throw NfError(NFIELD_EINVAL, "FP64 values of a matrix were released (FP32 hierarchy)");
  return A.val.p;
}
template <> const float* csr_values<float>(const DCsr& A) {
  if (!A.val32.p && A.nnz > 0) throw NfError(NFIELD_EINVAL, "FP32 values of a matrix were not prepared");
  return A.val32.p;
}

// ---- launch timing ----
namespace {
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;   // pairs
  std::vector<int> key;
  std::vector<double> bytes;
  std::vector<int> count;       // launches bracketed by each pair
  size_t used = 0;
};
Prof g_prof;
}  // namespace

void prof_enable(int on) {
  if (on && g_prof.ev.empty()) {
    g_prof.ev.resize(2 * 32768);
    for (auto& e : g_prof.ev) NF_HIP(hipEventCreate(&e));
  }
  g_prof.on = on != 0;
  g_prof.used = 0;
  g_prof.key.clear();
  g_prof.bytes.clear();
  g_prof.count.clear();
}

bool prof_recording() { return g_prof.on; }
// launches of a thread set quiet are not timed (threads that set up parts of
// the preconditioner concurrently)
static thread_local bool g_prof_quiet = false;
void prof_quiet(bool q) { g_prof_quiet = q; }

int prof_read(int max, int* key, int64_t* count, double* ms, double* bytes) {
  std::vector<int> keys;
  std::vector<int64_t> cnt;
  std::vector<double> t, b;
  for (size_t i = 0; i < g_prof.used; ++i) {
    NF_HIP(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    float e = 0.f;
    NF_HIP(hipEventElapsedTime(&e, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
    size_t k = 0;
    while (k < keys.size() && keys[k] != g_prof.key[i]) ++k;
    if (k == keys.size()) { keys.push_back(g_prof.key[i]); cnt.push_back(0); t.push_back(0); b.push_back(0); }
    cnt[k] += g_prof.count[i];
    t[k] += e;
    b[k] += g_prof.bytes[i];
  }
  const int n = (int)keys.size() < max ? (int)keys.size() : max;
  for (int k = 0; k < n; ++k) {
    key[k] = keys[k];
    count[k] = cnt[k];
    ms[k] = t[k];
    bytes[k] = b[k];
  }
  return (int)keys.size();
}

int prof_begin(hipStream_t s) {
  if (!g_prof.on || g_prof_quiet || g_prof.used >= g_prof.ev.size() / 2) return -1;
  NF_HIP(hipEventRecord(g_prof.ev[2 * g_prof.used], s));
  return (int)g_prof.used;
}
void prof_end(int slot, hipStream_t s, int key, double bytes, int count) {
  if (slot < 0) return;
  NF_HIP(hipEventRecord(g_prof.ev[2 * (size_t)slot + 1], s));
  g_prof.key.push_back(key);
  g_prof.bytes.push_back(bytes);
  g_prof.count.push_back(count);
  g_prof.used = (size_t)slot + 1;
}

// algorithmic bytes of one launch: matrix once, operand once, epilogue streams
template <class T>
static double spmv_bytes(SpmvMode mode, const DCsr& A, int nrhs) {
  const double s = sizeof(T);
  double b = (double)A.nnz * (s + 4) + 4.0 * (A.nr + 1) + nrhs * s * A.nc;
  const int streams = mode == SPMV_STORE ? 1 : mode == SPMV_CHEB ? 5 : 2;
  return b + nrhs * streams * s * A.nr;
}

template <class T> static bool spmv_bsr(SpmvMode mode, const DCsr& A, const SpmvArgs<T>& a, hipStream_t s);

template <class T> void spmv(SpmvMode mode, const DCsr& A, const SpmvArgs<T>& a, hipStream_t s) {
  if (A.nr <= 0) return;
  if (spmv_bsr<T>(mode, A, a, s)) return;
  const T* val = csr_values<T>(A);
  const int G = spmv_lanes(A.nr, A.nnz);
  bytes_count(spmv_bytes<T>(mode, A, a.nrhs));
  const bool timed = g_prof.on && !g_prof_quiet && g_prof.used < g_prof.ev.size() / 2;
  if (timed) NF_HIP(hipEventRecord(g_prof.ev[2 * g_prof.used], s));
  switch (mode) {
    case SPMV_STORE: spmv_nr<SPMV_STORE, T>(G, A, a, val, s); break;
    case SPMV_RESID: spmv_nr<SPMV_RESID, T>(G, A, a, val, s); break;
    case SPMV_ADD: spmv_nr<SPMV_ADD, T>(G, A, a, val, s); break;
    case SPMV_SUB: spmv_nr<SPMV_SUB, T>(G, A, a, val, s); break;
    case SPMV_CHEB: spmv_nr<SPMV_CHEB, T>(G, A, a, val, s); break;
    case SPMV_DSCALE: spmv_nr<SPMV_DSCALE, T>(G, A, a, val, s); break;
  }
  if (timed) {
    NF_HIP(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s));
    g_prof.key.push_back(((G * 16) * 100 + (int)mode) * 10 + (sizeof(T) == 4 ? 1 : 0));
    g_prof.bytes.push_back(spmv_bytes<T>(mode, A, a.nrhs));
    g_prof.count.push_back(1);
    ++g_prof.used;
  }
}
// Blocks j and (if hb) jb of a node's nu dense B x B blocks against x:
// their values (nv: the node's values, entry (q, c) of its blocks at
// nv[(q B + c) nu ..]) and their column nodes' (nc: the node's column nodes)
// B entries of x, added into the B row sums.  Without a second block the
// first is loaded twice and its second terms dropped: every load is
// unconditional, so none waits for another.
template <int B, class T>
__device__ __forceinline__ void bsr_block_rows(int j, int jb, bool hb, int nu, const int* __restrict__ nc,
                                               const T* __restrict__ nv, const T* __restrict__ x, T* acc) {
  constexpr int S = B * B;
  const int jj = hb ? jb : j;
  const int ca = nc[j], cb = nc[jj];
  T va[S], vb[S], xa[B], xb[B];
#pragma unroll
  for (int e = 0; e < S; ++e) {
    va[e] = nv[e * nu + j];
    vb[e] = nv[e * nu + jj];
  }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    xa[c] = x[(int64_t)ca * B + c];
    xb[c] = x[(int64_t)cb * B + c];
  }
#pragma unroll
  for (int e = 0; e < S; ++e) vb[e] = hb ? vb[e] : (T)0;
#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int c = 0; c < B; ++c) {
      acc[q] += va[q * B + c] * xa[c];
      acc[q] += vb[q * B + c] * xb[c];
    }
}

// SpMV from the block copy (one right-hand side; store, residual, add,
// subtract): G lanes per node taking whole blocks, the node's B row sums
// reduced across them
template <int B, int G, int MODE, class T>
__global__ __launch_bounds__(256) void k_spmv_bsr(int nnodes, const int* __restrict__ bptr, const int* __restrict__ bcol,
                                                  const T* __restrict__ bval, SpmvArgs<T> a) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int u = (int)(gid / G), lane = (int)(gid % G);
  if (u >= nnodes) return;   // whole groups of G lanes together
  const int k0 = bptr[u], k1 = bptr[u + 1];
  T acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = 0;
  const int nu = k1 - k0;
  for (int j = lane; j < nu; j += 2 * G)
    bsr_block_rows<B, T>(j, j + G, j + G < nu, nu, bcol + k0, bval + (int64_t)k0 * B * B, a.x, acc);
#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, G);
  T v = acc[0];
#pragma unroll
  for (int q = 1; q < B; ++q)
    if (lane == q) v = acc[q];
  if (lane >= B) return;
  const int64_t r = (int64_t)u * B + lane;
  if (MODE == SPMV_STORE) a.y[r] = v;
  else if (MODE == SPMV_RESID) a.y[r] = a.b[r] - v;
  else if (MODE == SPMV_ADD) a.y[r] += v;
  else if (MODE == SPMV_SUB) a.y[r] -= v;
}

template <class T> static const T* bsr_values(const DCsr& A);
template <> const double* bsr_values<double>(const DCsr& A) { return A.bsr_val.p; }
template <> const float* bsr_values<float>(const DCsr& A) { return A.bsr_val32.p; }

template <int B, class T>
static void spmv_bsr_launch(SpmvMode mode, const DCsr& A, const T* bv, const SpmvArgs<T>& a, hipStream_t s) {
  constexpr int G = 16;
  const int nnodes = A.nr / B;
  const unsigned blocks = (unsigned)cdiv((int64_t)nnodes * G, 256);
  switch (mode) {
    case SPMV_STORE:
      hipLaunchKernelGGL((k_spmv_bsr<B, G, SPMV_STORE, T>), dim3(blocks), dim3(256), 0, s, nnodes, A.bsr_ptr.p,
                         A.bsr_col.p, bv, a);
      break;
    case SPMV_RESID:
      hipLaunchKernelGGL((k_spmv_bsr<B, G, SPMV_RESID, T>), dim3(blocks), dim3(256), 0, s, nnodes, A.bsr_ptr.p,
                         A.bsr_col.p, bv, a);
      break;
    case SPMV_ADD:
      hipLaunchKernelGGL((k_spmv_bsr<B, G, SPMV_ADD, T>), dim3(blocks), dim3(256), 0, s, nnodes, A.bsr_ptr.p,
                         A.bsr_col.p, bv, a);
      break;
    default:
      hipLaunchKernelGGL((k_spmv_bsr<B, G, SPMV_SUB, T>), dim3(blocks), dim3(256), 0, s, nnodes, A.bsr_ptr.p,
                         A.bsr_col.p, bv, a);
      break;
  }
}

template <class T> static bool spmv_bsr(SpmvMode mode, const DCsr& A, const SpmvArgs<T>& a, hipStream_t s) {
  const T* bv = bsr_values<T>(A);
  if (g_in_setup || a.nrhs != 1 || !A.bsr_b || !bv || mode > SPMV_SUB) return false;
  const int b = A.bsr_b, nnodes = A.nr / b;
  const double sz = sizeof(T);
  const int streams = mode == SPMV_STORE ? 1 : 2;
  const double bytes = (double)A.bsr_nblk * (b * b * sz + 4) + 4.0 * (nnodes + 1) + sz * A.nc + streams * sz * A.nr;
  bytes_count(bytes);
  const bool timed = g_prof.on && !g_prof_quiet && g_prof.used < g_prof.ev.size() / 2;
  if (timed) NF_HIP(hipEventRecord(g_prof.ev[2 * g_prof.used], s));
  if (b == 2) spmv_bsr_launch<2, T>(mode, A, bv, a, s);
  else spmv_bsr_launch<3, T>(mode, A, bv, a, s);
  if (timed) {
    NF_HIP(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s));
    g_prof.key.push_back(((16 * 16 + b) * 100 + (int)mode) * 10 + (sizeof(T) == 4 ? 1 : 0));
    g_prof.bytes.push_back(bytes);
    g_prof.count.push_back(1);
    ++g_prof.used;
  }
  return true;
}

template void spmv<double>(SpmvMode, const DCsr&, const SpmvArgs<double>&, hipStream_t);
template void spmv<float>(SpmvMode, const DCsr&, const SpmvArgs<float>&, hipStream_t);

// ================================================================= reductions
// Fixed grids (RED_BLOCKS blocks per column) so that every sum is taken in
// the same order on every run and for every batch size.
__global__ __launch_bounds__(256) void k_dot_partialm(const double* __restrict__ x, int64_t ldx, const double* __restrict__ y,
                                                      int64_t ldy, int64_t n, double* __restrict__ partial) {
  __shared__ double ws[4];
  const double* xk = x + blockIdx.y * ldx;
  const double* yk = y + blockIdx.y * ldy;
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += xk[i] * yk[i];
  s = block_sum256(s, ws);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * RED_BLOCKS + blockIdx.x] = s;
}
// grid (ncols, nrhs): out[k*os + j] (+)= sum of partial[k*ps + j*RED_BLOCKS + 0..RED_BLOCKS)
__global__ __launch_bounds__(256) void k_mreduce(const double* __restrict__ partial, int64_t ps, double* __restrict__ out,
                                                 int64_t os, int accumulate, const int* mask, const int* ncv) {
  __shared__ double ws[4];
  const int j = blockIdx.x, k = blockIdx.y;
  if (mask && !mask[k]) return;
  if (ncv && j >= ncv[k]) return;
  const double* pk = partial + k * ps + (int64_t)j * RED_BLOCKS;
  double s = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) s += pk[i];
  s = block_sum256(s, ws);
  if (threadIdx.x == 0) out[k * os + j] = accumulate ? out[k * os + j] + s : s;
}

void dotm(const double* x, int64_t ldx, const double* y, int64_t ldy, int64_t n, int nrhs, double* partial, double* out,
          hipStream_t s) {
  bytes_count(16.0 * n * nrhs);
  hipLaunchKernelGGL(k_dot_partialm, dim3(RED_BLOCKS, nrhs), dim3(256), 0, s, x, ldx, y, ldy, n, partial);
  hipLaunchKernelGGL(k_mreduce, dim3(1, nrhs), dim3(256), 0, s, partial, (int64_t)RED_BLOCKS, out, (int64_t)1, 0,
                     (const int*)nullptr, (const int*)nullptr);
}

// v = w / ||w||, ||w||^2 the sum of the RED_BLOCKS partials of one dot:
// every workgroup sums them as k_mreduce does (same order, same bits) and
// workgroup 0 stores ||w|| in nrm[0]; a zero norm leaves w unscaled
__global__ __launch_bounds__(256) void k_normalize_partials(const double* __restrict__ partial, const double* __restrict__ w,
                                                            double* __restrict__ v, int64_t n, double* __restrict__ nrm) {
  __shared__ double ws[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) s += partial[i];
  s = block_sum256(s, ws);
  const double sv = sqrt(s);
  if (blockIdx.x == 0 && threadIdx.x == 0) *nrm = sv;
  const double inv = sv != 0.0 ? 1.0 / sv : 1.0;
  NF_ROWS(n) v[i] = w[i] * inv;
}
void normalize(const double* w, double* v, int64_t n, double* partial, double* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partialm, dim3(RED_BLOCKS, 1), dim3(256), 0, s, w, n, w, n, n, partial);
  if (n > 0) hipLaunchKernelGGL(k_normalize_partials, dim3(grid_cols(n, 1)), dim3(256), 0, s, partial, w, v, n, nrm);
}

// column k = blockIdx.y: partial dots of V_k[k0, k0 + CH) (k0 = CH
// blockIdx.z, below ncols) with w_k.  Splitting the columns over blockIdx.z
// keeps the accumulators few and the workgroups many; each dot still sums
// its terms per thread and per workgroup in the same order.
template <int CH>
__global__ __launch_bounds__(256) void k_mdot(const double* __restrict__ V, int64_t vs, int64_t n, int ncols,
                                              const double* __restrict__ w, int64_t ldw, double* __restrict__ partial,
                                              int64_t ps, const int* mask, const int* ncv) {
  __shared__ double ws[4];
  const int kc = blockIdx.y, k0 = blockIdx.z * CH;
  if (mask && !mask[kc]) return;
  if (ncv) ncols = ncv[kc];
  const int nk = min(CH, ncols - k0);
  if (nk <= 0) return;   // uniform over the workgroup
  const double* Vk = V + kc * vs + (int64_t)k0 * n;
  const double* wk = w + kc * ldw;
  double acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double wi = wk[i];
#pragma unroll
    for (int k = 0; k < CH; ++k)
      if (k < nk) acc[k] += Vk[k * n + i] * wi;
  }
#pragma unroll
  for (int k = 0; k < CH; ++k)
    if (k < nk) {
      double r = block_sum256(acc[k], ws);
      if (threadIdx.x == 0) partial[kc * ps + (int64_t)(k0 + k) * RED_BLOCKS + blockIdx.x] = r;
    }
}

// w_k <- w_k - V_k h_k, one element per thread (terms in ascending k)
template <int MAXC>
__global__ __launch_bounds__(256) void k_mupdate_only(const double* __restrict__ V, int64_t vs, int64_t n, int ncols,
                                                      const double* __restrict__ h, int64_t hs, double* __restrict__ w,
                                                      int64_t ldw, const int* mask, const int* ncv) {
  __shared__ double hsh[MAXC];
  const int kc = blockIdx.y;
  if (mask && !mask[kc]) return;
  if (ncv) ncols = ncv[kc];
  for (int k = threadIdx.x; k < MAXC; k += 256) hsh[k] = k < ncols ? h[kc * hs + k] : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* Vk = V + kc * vs;
  double wi = w[kc * ldw + i];
#pragma unroll
  for (int k = 0; k < MAXC; ++k)
    if (k < ncols) wi -= Vk[k * n + i] * hsh[k];
  w[kc * ldw + i] = wi;
}

// partial sums of w_k^2 in the grid-stride order of the workgroups
__global__ __launch_bounds__(256) void k_norm_partial(int64_t n, const double* __restrict__ w, int64_t ldw,
                                                      double* __restrict__ partial, int64_t ps, const int* mask) {
  __shared__ double ws[4];
  const int kc = blockIdx.y;
  if (mask && !mask[kc]) return;
  const double* wk = w + kc * ldw;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double wi = wk[i];
    acc += wi * wi;
  }
  const double r = block_sum256(acc, ws);
  if (threadIdx.x == 0) partial[kc * ps + blockIdx.x] = r;
}

template <int MAXC>
__global__ __launch_bounds__(256) void k_mcombine(const double* __restrict__ V, int64_t vs, int64_t n, const int* ncols,
                                                  const double* __restrict__ y, int64_t ys, double* __restrict__ u,
                                                  int64_t ldu, int accumulate, const int* mask) {
  __shared__ double ysh[MAXC];
  const int kc = blockIdx.y;
  if (mask && !mask[kc]) return;
  const int nck = ncols[kc];
  const double* Vk = V + kc * vs;
  double* uk = u + kc * ldu;
  for (int k = threadIdx.x; k < MAXC; k += 256) ysh[k] = k < nck ? y[kc * ys + k] : 0.0;
  __syncthreads();
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double sacc = accumulate ? uk[i] : 0.0;
#pragma unroll
    for (int k = 0; k < MAXC; ++k)
      if (k < nck) sacc += Vk[k * n + i] * ysh[k];
    uk[i] = sacc;
  }
}

#define NF_MAXC_DISPATCH(ncols, KERNEL_CALL)               \
  do {                                                     \
    if ((ncols) <= 8) { constexpr int MC = 8; KERNEL_CALL; } \
    else if ((ncols) <= 16) { constexpr int MC = 16; KERNEL_CALL; } \
    else if ((ncols) <= 32) { constexpr int MC = 32; KERNEL_CALL; } \
    else if ((ncols) <= 64) { constexpr int MC = 64; KERNEL_CALL; } \
    else throw NfError(NFIELD_EINVAL, "GMRES restart length above 63 is not supported"); \
  } while (0)

void mdot_partial(const GmresLayout& L, const double* V, int ncols, const double* w, int64_t ldw, double* partial,
                  const int* mask, hipStream_t s, const int* ncv) {
  if (ncols <= 0) return;
  NF_CHECK(ncols <= 64, NFIELD_EINVAL, "GMRES restart length above 63 is not supported");
  bytes_count(8.0 * L.n * (ncols + 1) * L.nrhs);
  if (ncols <= 8)
    hipLaunchKernelGGL(k_mdot<8>, dim3(RED_BLOCKS, L.nrhs, 1), dim3(256), 0, s, V, L.vs, L.n, ncols, w, ldw, partial, L.ps,
                       mask, ncv);
  else
    hipLaunchKernelGGL(k_mdot<16>, dim3(RED_BLOCKS, L.nrhs, cdiv(ncols, 16)), dim3(256), 0, s, V, L.vs, L.n, ncols, w, ldw,
                       partial, L.ps, mask, ncv);
}
void mreduce(const GmresLayout& L, const double* partial, int ncols, double* out, int accumulate, const int* mask,
             hipStream_t s, const int* ncv) {
  hipLaunchKernelGGL(k_mreduce, dim3(ncols, L.nrhs), dim3(256), 0, s, partial, L.ps, out, L.hs, accumulate, mask, ncv);
}
// the update with every element's thread, then the dots as mdot_partial
// (the same sums as one fused pass, at the cost of a second read of V)
void mupdate_dot(const GmresLayout& L, const double* V, int ncols, const double* h, double* w, int64_t ldw,
                 double* partial, const int* mask, hipStream_t s, const int* ncv) {
  if (ncols <= 0 || L.n <= 0) return;
  bytes_count(8.0 * L.n * (ncols + 2) * L.nrhs);
  NF_MAXC_DISPATCH(ncols, hipLaunchKernelGGL((k_mupdate_only<MC>), dim3(cdiv(L.n, 256), L.nrhs), dim3(256), 0, s, V, L.vs,
                                             L.n, ncols, h, L.hs, w, ldw, mask, ncv));
  mdot_partial(L, V, ncols, w, ldw, partial, mask, s, ncv);
}
void mupdate_norm(const GmresLayout& L, const double* V, int ncols, const double* h, double* w, int64_t ldw,
                  double* partial, const int* mask, hipStream_t s, const int* ncv) {
  if (ncols <= 0 || L.n <= 0) return;
  bytes_count(8.0 * L.n * (ncols + 3) * L.nrhs);
  NF_MAXC_DISPATCH(ncols, hipLaunchKernelGGL((k_mupdate_only<MC>), dim3(cdiv(L.n, 256), L.nrhs), dim3(256), 0, s, V, L.vs,
                                             L.n, ncols, h, L.hs, w, ldw, mask, ncv));
  hipLaunchKernelGGL(k_norm_partial, dim3(RED_BLOCKS, L.nrhs), dim3(256), 0, s, L.n, w, ldw, partial, L.ps, mask);
}
void mcombine(const GmresLayout& L, const double* V, const int* ncols, int max_ncols, const double* y, double* u,
              int64_t ldu, int accumulate, const int* mask, hipStream_t s) {
  if (max_ncols <= 0) return;
  bytes_count(8.0 * L.n * (max_ncols + (accumulate ? 2 : 1)) * L.nrhs);
  NF_MAXC_DISPATCH(max_ncols, hipLaunchKernelGGL(k_mcombine<MC>, dim3(grid_cols(L.n, L.nrhs), L.nrhs), dim3(256), 0, s, V, L.vs,
                                                 L.n, ncols, y, (int64_t)L.m, u, ldu, accumulate, mask));
}

// Givens step of the Arnoldi process for column k = blockIdx.x: H_k is
// (m+1) x m column-major.
__global__ __launch_bounds__(256) void k_givens(int j, int m, const double* __restrict__ h1, const double* __restrict__ h2,
                                                int64_t hs, const double* __restrict__ nrm_partial, int64_t ps, double* H,
                                                double* cs, double* sn, double* g, double* scal, const int* mask,
                                                const int* jv) {
  __shared__ double ws[4];
  __shared__ double hc[66], csl[64], snl[64];   // the new column and the rotations so far, staged by all threads
  const int kc = blockIdx.x;
  if (mask && !mask[kc]) return;
  if (jv) j = jv[kc];
  const int ld = m + 1;
  double* Hk = H + (int64_t)kc * ld * m;
  double* csk = cs + (int64_t)kc * m;
  double* snk = sn + (int64_t)kc * m;
  double* gk = g + (int64_t)kc * ld;
  double* Hj = Hk + (int64_t)j * ld;
  for (int i = threadIdx.x; i <= j; i += 256) hc[i] = h1[kc * hs + i] + h2[kc * hs + i];
  for (int i = threadIdx.x; i < j; i += 256) {
    csl[i] = csk[i];
    snl[i] = snk[i];
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) s += nrm_partial[kc * ps + i];
  s = block_sum256(s, ws);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(s);
    hc[j + 1] = hn;
    scal[2 * kc] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = hc[i], c = hc[i + 1];
      hc[i] = csl[i] * a + snl[i] * c;
      hc[i + 1] = -snl[i] * a + csl[i] * c;
    }
    const double a = hc[j], c = hc[j + 1];
    const double den = hypot(a, c);
    const double cj = den == 0.0 ? 1.0 : a / den, sj = den == 0.0 ? 0.0 : c / den;
    csk[j] = cj;
    snk[j] = sj;
    hc[j] = den;
    hc[j + 1] = 0.0;
    const double gj = gk[j];
    gk[j + 1] = -sj * gj;
    gk[j] = cj * gj;
    scal[2 * kc + 1] = fabs(gk[j + 1]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += 256) Hj[i] = hc[i];
}
__global__ void k_backsolve(const int* ncols, int m, const double* H, const double* g, double* y, const int* mask) {
  const int kc = blockIdx.x;
  if (threadIdx.x != 0 || (mask && !mask[kc])) return;
  const int ld = m + 1, k = ncols[kc];
  const double* Hk = H + (int64_t)kc * ld * m;
  const double* gk = g + (int64_t)kc * ld;
  double* yk = y + (int64_t)kc * m;
  for (int i = k - 1; i >= 0; --i) {
    double s = gk[i];
    for (int l = i + 1; l < k; ++l) s -= Hk[(int64_t)l * ld + i] * yk[l];
    // a zero diagonal (A M singular on the Krylov space, after a breakdown)
    // leaves that coefficient at zero
    const double d = Hk[(int64_t)i * ld + i];
    yk[i] = d != 0.0 ? s / d : 0.0;
  }
}
void givens_step(const GmresLayout& L, int j, const double* h1, const double* h2, const double* nrm_partial, double* H,
                 double* cs, double* sn, double* g, double* scal, const int* mask, hipStream_t s, const int* jv) {
  hipLaunchKernelGGL(k_givens, dim3(L.nrhs), dim3(256), 0, s, j, L.m, h1, h2, L.hs, nrm_partial, L.ps, H, cs, sn, g, scal,
                     mask, jv);
}
void backsolve(const GmresLayout& L, const int* ncols, const double* H, const double* g, double* y, const int* mask,
               hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, dim3(L.nrhs), dim3(64), 0, s, ncols, L.m, H, g, y, mask);
}

// Columns of per-column Krylov sets: out column c = V_{act[c]}[jv[act[c]]]
// (jv NULL: vector 0), and the reverse scatter.
__global__ void k_slot_gather(const double* __restrict__ V, int64_t vs, int64_t n, const int* __restrict__ act,
                              const int* __restrict__ jv, double* __restrict__ out) {
  const int c = blockIdx.y, k = act[c];
  const double* src = V + k * vs + (jv ? (int64_t)jv[k] * n : 0);
  double* dst = out + (int64_t)c * n;
  NF_ROWS(n) dst[i] = src[i];
}
__global__ void k_slot_scatter(const double* __restrict__ in, int64_t n, const int* __restrict__ act,
                               const int* __restrict__ jv, double* __restrict__ V, int64_t vs) {
  const int c = blockIdx.y, k = act[c];
  const double* src = in + (int64_t)c * n;
  double* dst = V + k * vs + (jv ? (int64_t)jv[k] * n : 0);
  NF_ROWS(n) dst[i] = src[i];
}
void slot_gather(const double* V, int64_t vs, int64_t n, const int* act, const int* jv, int nact, double* out,
                 hipStream_t s) {
  if (n <= 0 || nact <= 0) return;
  bytes_count(16.0 * n * nact);
  hipLaunchKernelGGL(k_slot_gather, dim3(grid_cols(n, nact), nact), dim3(256), 0, s, V, vs, n, act, jv, out);
}
void slot_scatter(const double* in, int64_t n, const int* act, const int* jv, int nact, double* V, int64_t vs,
                  hipStream_t s) {
  if (n <= 0 || nact <= 0) return;
  bytes_count(16.0 * n * nact);
  hipLaunchKernelGGL(k_slot_scatter, dim3(grid_cols(n, nact), nact), dim3(256), 0, s, in, n, act, jv, V, vs);
}

// ====================================================================== scan
// Exclusive scan of int32 counts: each 256-thread block scans 2048 entries
// (8 per thread); block totals are scanned recursively and added back.
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_BLOCK = 256 * SCAN_PER_THREAD;

__global__ __launch_bounds__(256) void k_scan_block(const int* __restrict__ in, int* __restrict__ out, int64_t n,
                                                    int* __restrict__ block_sums) {
  __shared__ int sums[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD];
  int t = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    t += v[k];
  }
  sums[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {   // Hillis-Steele inclusive scan of thread totals
    int add = threadIdx.x >= off ? sums[threadIdx.x - off] : 0;
    __syncthreads();
    sums[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sums[threadIdx.x] - t;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) block_sums[blockIdx.x] = sums[255];
}
__global__ void k_scan_add(int* out, int64_t n, const int* __restrict__ scanned_block_sums) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t b = i / SCAN_BLOCK;
  if (i < n) out[i] += scanned_block_sums[b];
}
__global__ void k_set_total(const int* in, int* out, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = (n > 0 ? out[n - 1] + in[n - 1] : 0);
}

static void scan_rec(const int* in, int* out, int64_t n, hipStream_t s) {
  const int nb = cdiv(n, SCAN_BLOCK);
  DBuf<int> bs(nb + 1);
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(256), 0, s, in, out, n, bs.p);
  if (nb > 1) {
    // (temporaries go back to the context's block cache, reused in stream order)
    DBuf<int> bss(nb + 1);
    scan_rec(bs.p, bss.p, nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3(cdiv(n, 256)), dim3(256), 0, s, out, n, bss.p);
  }
}

int64_t exclusive_scan(const int* in, int* out, int64_t n, hipStream_t s) {
  if (n > 0) scan_rec(in, out, n, s);
  hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, in, out, n);
  int total = 0;
  NF_HIP(hipMemcpyAsync(&total, out + n, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  NF_CHECK(total >= 0, NFIELD_ENOMEM, "index count exceeds 2^31");
  return total;
}

// ============================================================== setup basics
__global__ void k_csr_diag(int nr, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
                           double* d, int* zero_flag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nr) return;
  int lo = ptr[i], hi = ptr[i + 1];
  while (lo < hi) {   // lower_bound of column i
    int mid = (lo + hi) >> 1;
    if (col[mid] < i) lo = mid + 1; else hi = mid;
  }
  double v = (lo < ptr[i + 1] && col[lo] == i) ? val[lo] : 0.0;
  d[i] = v;
  if (v == 0.0) atomicOr(zero_flag, 1);
}
void csr_diag(const DCsr& A, double* d, int* zero_flag, hipStream_t s) {
  if (A.nr > 0) hipLaunchKernelGGL(k_csr_diag, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, A.val.p, d, zero_flag);
}
__global__ void k_invert(const double* d, double* dinv, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dinv[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
}
void invert(const double* d, double* dinv, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_invert, dim3(cdiv(n, 256)), dim3(256), 0, s, d, dinv, n);
}
__global__ void k_power_start(double* v, int64_t n, uint64_t seed) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= n) return;
  const uint64_t s0 = smix64(seed);
  v[u] = 0.5 + (double)(smix64(s0 ^ (uint64_t)(u + 1)) >> 11) * 0x1.0p-53;
}
void power_start(double* v, int64_t n, uint64_t seed, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_power_start, dim3(cdiv(n, 256)), dim3(256), 0, s, v, n, seed);
}

// ================================================================ node graph
constexpr int MAXB = 8;
// node u ~ v (u != v) iff some stored entry couples their dofs.  The
// neighbours come out in ascending order.
//
// Serial form (one lane): merge the b sorted rows of the node by node index.
__device__ int node_merge(int u, int b, const int* __restrict__ ptr, const int* __restrict__ col, int* adj) {
  int p[MAXB], e[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    p[c] = c < b ? ptr[u * b + c] : 0;
    e[c] = c < b ? ptr[u * b + c + 1] : 0;
  }
  int cnt = 0;
  while (true) {
    int mn = INT_MAX;
#pragma unroll
    for (int c = 0; c < MAXB; ++c)
      if (p[c] < e[c]) mn = min(mn, col[p[c]] / b);
    if (mn == INT_MAX) break;
#pragma unroll
    for (int c = 0; c < MAXB; ++c)
      while (p[c] < e[c] && col[p[c]] / b == mn) ++p[c];
    if (mn != u) {
      if (adj) adj[cnt] = mn;
      ++cnt;
    }
  }
  return cnt;
}
// One wavefront per node.  When every row of the node couples to the same
// set of nodes (the usual case for node-blocked operators), that set is the
// first row's, found with one pass over each row: each row's distinct nodes
// in order are the first row's.  Otherwise (rows of a constrained dof, say) the node
// indices of all its rows are sorted in LDS and the runs counted, or, beyond
// NG_CAP entries, lane 0 merges.
constexpr int NG_CAP = 2048;
template <bool FILL>
__global__ __launch_bounds__(64) void k_node_graph(int nnode, int b, const int* __restrict__ ptr, const int* __restrict__ col,
                                                   int* cnt_or_off, int* adj) {
  __shared__ int keys[NG_CAP];
  const int u = blockIdx.x, lane = threadIdx.x;
  if (u >= nnode) return;
  const int p0 = ptr[u * b], e0 = ptr[u * b + 1];
  int* out = FILL ? adj + cnt_or_off[u] : nullptr;
  int c, n0;
  if (rows_share_groups(ptr, u * b, b, b, col, keys, NG_CAP, n0)) {
    c = group_runs(p0, e0, b, col, u, out);
  } else {
    __syncthreads();   // keys held the first row's nodes
    const int E = ptr[u * b + b] - p0;
    if (E <= NG_CAP) {
      int ts = 1;
      while (ts < E) ts <<= 1;
      for (int t = lane; t < ts; t += 64) keys[t] = t < E ? col[p0 + t] / b : INT_MAX;
      __syncthreads();
      wave_bitonic(keys, ts, lane);
      c = 0;
      for (int t0 = 0; t0 < E; t0 += 64) {
        const int t = t0 + lane;
        const bool first = t < E && (t == 0 || keys[t - 1] != keys[t]) && keys[t] != u;
        const unsigned long long bal = __ballot(first);
        if (out && first) out[c + __popcll(bal & ((1ull << lane) - 1ull))] = keys[t];
        c += __popcll(bal);
      }
    } else {
      c = lane == 0 ? node_merge(u, b, ptr, col, out) : 0;
    }
  }
  if (!FILL && lane == 0) cnt_or_off[u] = c;
}
// flag = 1 if some edge u -> v of the graph has no edge v -> u (the
// neighbour lists are sorted: a binary search in v's list)
__global__ void k_graph_asym(int n, const int* __restrict__ gp, const int* __restrict__ ga, int* flag) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= n) return;
  for (int p = gp[u]; p < gp[u + 1]; ++p) {
    const int v = ga[p];
    int lo = gp[v], hi = gp[v + 1];
    const int end = hi;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ga[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    if (lo == end || ga[lo] != u) {
      atomicOr(flag, 1);
      return;
    }
  }
}

// The node graph is the pattern of A + A^T on nodes: the rows give u -> v;
// when some edge has no reverse (a nonsymmetric pattern), the graph is
// replaced by its union with its transpose, so that the MIS-2 distances and
// the colouring see every coupling from both ends.
void node_graph(const DCsr& A, int b, DBuf<int>& gptr, DBuf<int>& gadj, int* nnode_out, hipStream_t s) {
  NF_CHECK(b >= 1 && b <= MAXB, NFIELD_EINVAL, "block size must be between 1 and 8");
  NF_CHECK(A.nr == A.nc && A.nr % b == 0, NFIELD_EINVAL, "node graph: size is not a multiple of the block size");
  const int nn = A.nr / b;
  *nnode_out = nn;
  DBuf<int> cnt(nn + 1);
  gptr.alloc(nn + 1);
  if (nn > 0) hipLaunchKernelGGL(k_node_graph<false>, dim3(nn), dim3(64), 0, s, nn, b, A.ptr.p, A.col.p, cnt.p, nullptr);
  const int64_t tot = exclusive_scan(cnt.p, gptr.p, nn, s);
  gadj.alloc(tot > 0 ? tot : 1);
  if (nn <= 0 || tot <= 0) return;
  hipLaunchKernelGGL(k_node_graph<true>, dim3(nn), dim3(64), 0, s, nn, b, A.ptr.p, A.col.p, gptr.p, gadj.p);
  fill<int>(cnt.p, 0, 1, s);
  hipLaunchKernelGGL(k_graph_asym, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, gptr.p, gadj.p, cnt.p);
  int asym = 0;
  NF_HIP(hipMemcpyAsync(&asym, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  if (!asym) return;
  DCsr G, GT, U;
  G.nr = G.nc = nn;
  G.nnz = tot;
  G.ptr = std::move(gptr);
  G.col = std::move(gadj);
  G.val.alloc(tot);
  fill<double>(G.val.p, 1.0, tot, s);
  transpose(G, GT, s);
  csr_add(1.0, G, 1.0, GT, U, s);
  gptr = std::move(U.ptr);
  gadj = std::move(U.col);
}

// ===================================================================== MIS-2
// Synchronous rounds with the node tuples (key, id), key = splitmix64(seed ^
// splitmix64(id)).  States: 0 undecided, 1 root, 2 out.
__device__ __forceinline__ bool tuple_greater(const uint64_t* key, int a, int b) {
  const uint64_t ka = key[a], kb = key[b];
  return ka != kb ? ka > kb : a > b;
}
__global__ void k_mis_keys(int n, uint64_t seed, uint64_t* key) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < n) key[u] = smix64(seed ^ smix64((uint64_t)u));
}
// m1[v] = largest undecided tuple in the closed neighbourhood of v (-1: none)
__global__ void k_mis_m1(int n, const int* __restrict__ gp, const int* __restrict__ ga, const uint64_t* __restrict__ key,
                         const int* __restrict__ st, int* __restrict__ m1) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  int best = st[v] == 0 ? v : -1;
  for (int p = gp[v]; p < gp[v + 1]; ++p) {
    const int w = ga[p];
    if (st[w] == 0 && (best < 0 || tuple_greater(key, w, best))) best = w;
  }
  m1[v] = best;
}
// an undecided u whose tuple is the largest within distance 2 becomes a root
__global__ void k_mis_root(int n, const int* __restrict__ gp, const int* __restrict__ ga, const uint64_t* __restrict__ key,
                           int* __restrict__ st, const int* __restrict__ m1) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= n || st[u] != 0) return;
  int best = m1[u];
  for (int p = gp[u]; p < gp[u + 1]; ++p) {
    const int c = m1[ga[p]];
    if (c >= 0 && (best < 0 || tuple_greater(key, c, best))) best = c;
  }
  if (best == u) st[u] = 1;
}
__global__ void k_mis_r1(int n, const int* __restrict__ gp, const int* __restrict__ ga, const int* __restrict__ st,
                         int* __restrict__ r1) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  int f = st[v] == 1;
  for (int p = gp[v]; p < gp[v + 1] && !f; ++p) f = st[ga[p]] == 1;
  r1[v] = f;
}
__global__ void k_mis_out(int n, const int* __restrict__ gp, const int* __restrict__ ga, int* __restrict__ st,
                          const int* __restrict__ r1, int* und_count) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= n || st[u] != 0) return;
  int f = r1[u];
  for (int p = gp[u]; p < gp[u + 1] && !f; ++p) f = r1[ga[p]];
  if (f) st[u] = 2;
  else atomicAdd(und_count, 1);
}
__global__ void k_is_root(int n, const int* st, int* flag) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < n) flag[u] = st[u] == 1;
}
// phase 1 + 2: roots take their number; a neighbour of a root joins it
__global__ void k_agg_phase2(int n, const int* __restrict__ gp, const int* __restrict__ ga, const int* __restrict__ st,
                             const int* __restrict__ rootid, int* __restrict__ agg, int* __restrict__ phase) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= n) return;
  if (st[u] == 1) { agg[u] = rootid[u]; phase[u] = 1; return; }
  int a = -1;
  for (int p = gp[u]; p < gp[u + 1]; ++p)
    if (st[ga[p]] == 1) { a = rootid[ga[p]]; break; }
  agg[u] = a;
  phase[u] = a >= 0 ? 2 : 0;
}
// phase 3: join the smallest aggregate among phase-2 neighbours
__global__ void k_agg_phase3(int n, const int* __restrict__ gp, const int* __restrict__ ga, const int* __restrict__ phase,
                             int* __restrict__ agg, int* err) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= n || phase[u] != 0) return;
  int best = -1;
  for (int p = gp[u]; p < gp[u + 1]; ++p) {
    const int v = ga[p];
    if (phase[v] == 2 && (best < 0 || agg[v] < best)) best = agg[v];
  }
  if (best < 0) atomicOr(err, 1);
  agg[u] = best < 0 ? 0 : best;
}

int mis2_aggregate(int n, const int* gp, const int* ga, uint64_t seed, int* agg, hipStream_t s) {
  if (n == 0) return 0;
  DBuf<uint64_t> key(n);
  DBuf<int> st(n), m1(n), cnt(1), flag(n + 1), rootid(n + 1), phase(n), err(1);
  const int g = cdiv(n, 256);
  hipLaunchKernelGGL(k_mis_keys, dim3(g), dim3(256), 0, s, n, seed, key.p);
  fill<int>(st.p, 0, n, s);
  int und = n, rounds = 0;
  while (und > 0) {
    NF_CHECK(++rounds <= n + 1, NFIELD_EINVAL, "MIS-2 did not terminate");
    const int before = und;
    hipLaunchKernelGGL(k_mis_m1, dim3(g), dim3(256), 0, s, n, gp, ga, key.p, st.p, m1.p);
    hipLaunchKernelGGL(k_mis_root, dim3(g), dim3(256), 0, s, n, gp, ga, key.p, st.p, m1.p);
    hipLaunchKernelGGL(k_mis_r1, dim3(g), dim3(256), 0, s, n, gp, ga, st.p, m1.p /* reused as r1 */);
    fill<int>(cnt.p, 0, 1, s);
    hipLaunchKernelGGL(k_mis_out, dim3(g), dim3(256), 0, s, n, gp, ga, st.p, m1.p, cnt.p);
    NF_HIP(hipMemcpyAsync(&und, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    NF_CHECK(und < before, NFIELD_EINVAL, "MIS-2 round made no progress");
  }
  hipLaunchKernelGGL(k_is_root, dim3(g), dim3(256), 0, s, n, st.p, flag.p);
  const int nagg = (int)exclusive_scan(flag.p, rootid.p, n, s);
  fill<int>(err.p, 0, 1, s);
  hipLaunchKernelGGL(k_agg_phase2, dim3(g), dim3(256), 0, s, n, gp, ga, st.p, rootid.p, agg, phase.p);
  hipLaunchKernelGGL(k_agg_phase3, dim3(g), dim3(256), 0, s, n, gp, ga, phase.p, agg, err.p);
  int e = 0;
  NF_HIP(hipMemcpyAsync(&e, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  NF_CHECK(e == 0, NFIELD_EINVAL, "aggregation: node without a phase-2 neighbour");
  return nagg;
}

// ================================================== multicolour Gauss-Seidel
// Greedy colouring in node order: every node takes the smallest colour not
// used by its smaller-index neighbours.  Each node's colour depends only on
// its smaller neighbours' final colours, so any schedule that colours a node
// after all of them gives the sequential result.
__global__ void k_max_int(const int* x, int n, int* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) atomicMax(out, x[i] + 1);
}

// Schedule: wait[w] counts the smaller neighbours of w (in w's own list) not
// yet coloured; a node is coloured as soon as that count is zero and then
// releases the nodes waiting on it (the reverse of the smaller-neighbour
// relation, built first from the lists themselves).  node_graph makes the
// graph symmetric, so a node sees every smaller neighbour and no two
// neighbours share a colour.  One workgroup runs every round of frontiers,
// kept in two global lists.
__global__ void k_color_wait(int n, const int* __restrict__ gp, const int* __restrict__ ga, int* wait, int* rcnt, int* front,
                             int* nfront) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= n) return;
  int c = 0;
  for (int p = gp[w]; p < gp[w + 1]; ++p) {
    const int v = ga[p];
    if (v < w) {
      ++c;
      atomicAdd(&rcnt[v], 1);
    }
  }
  wait[w] = c;
  if (c == 0) front[atomicAdd(nfront, 1)] = w;
}
__global__ void k_color_rev(int n, const int* __restrict__ gp, const int* __restrict__ ga, const int* __restrict__ rptr,
                            int* rcur, int* radj) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= n) return;
  for (int p = gp[w]; p < gp[w + 1]; ++p) {
    const int v = ga[p];
    if (v < w) radj[rptr[v] + atomicAdd(&rcur[v], 1)] = w;
  }
}
// Four lanes per frontier node: the lanes split the node's neighbour list
// (its smaller neighbours' colours are or-ed into one mask across the four)
// and the list of nodes waiting on it (their counters are released in
// parallel).  With LDS, the wait counters (one byte each, packed four to a
// word for LDS atomics) and the colours (one byte each) of every node live in
// LDS, for graphs of up to COLOR_LDS_NODES nodes with at most 255 smaller
// neighbours per node; otherwise both stay in global memory.
constexpr int COLOR_LDS_NODES = 73728;
constexpr int COLOR_LPN = 4;
// neighbour loads a lane issues together before using them
constexpr int COLOR_BATCH = 8;

template <bool LDS>
__global__ __launch_bounds__(1024) void k_color_frontier(int n, const int* __restrict__ gp, const int* __restrict__ ga,
                                                         const int* __restrict__ rptr, const int* __restrict__ radj,
                                                         int* color, int* wait, int* fa, int* fb, const int* nfront0,
                                                         int* err, int* done) {
  __shared__ unsigned int wt[LDS ? COLOR_LDS_NODES / 4 : 1];
  __shared__ unsigned char cl[LDS ? COLOR_LDS_NODES : 1];
  __shared__ int nf_cur, nf_next;
  if (LDS)
    for (int w = threadIdx.x; w < (n + 3) / 4; w += 1024) {
      unsigned int x = 0;
      for (int k = 0; k < 4; ++k)
        if (4 * w + k < n) x |= (unsigned int)wait[4 * w + k] << (8 * k);
      wt[w] = x;
    }
  if (threadIdx.x == 0) { nf_cur = *nfront0; nf_next = 0; }
  __syncthreads();
  const int grp = threadIdx.x / COLOR_LPN, sub = threadIdx.x % COLOR_LPN;
  constexpr int NGRP = 1024 / COLOR_LPN;
  int* cur = fa;
  int* nxt = fb;
  int coloured = 0;
  while (true) {
    const int m = nf_cur;
    if (m == 0) break;
    // every group runs the same number of passes (the shuffles need all lanes)
    for (int i0 = 0; i0 < m; i0 += NGRP) {
      const int i = i0 + grp;
      const int u = i < m ? cur[i] : -1;
      int g0 = 0, g1 = 0, r0 = 0, r1 = 0;
      if (u >= 0) {
        g0 = gp[u];
        g1 = gp[u + 1];
        r0 = rptr[u];
        r1 = rptr[u + 1];
      }
      uint64_t mask[4] = {0, 0, 0, 0};
      for (int pb = g0 + sub; pb < g1; pb += COLOR_BATCH * COLOR_LPN) {
        int vv[COLOR_BATCH];   // the batch's loads issued together
#pragma unroll
        for (int q = 0; q < COLOR_BATCH; ++q) vv[q] = pb + q * COLOR_LPN < g1 ? ga[pb + q * COLOR_LPN] : INT_MAX;
#pragma unroll
        for (int q = 0; q < COLOR_BATCH; ++q) {
          const int v = vv[q];
          if (v >= u) continue;
          const int c = LDS ? (int)cl[v] : __hip_atomic_load(&color[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (c >= 0 && c < 256) mask[c >> 6] |= 1ull << (c & 63);
        }
      }
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int o = COLOR_LPN / 2; o > 0; o >>= 1) mask[w] |= __shfl_xor(mask[w], o, COLOR_LPN);
      if (u < 0) continue;
      int c = -1;
      for (int w = 0; w < 4 && c < 0; ++w)
        if (~mask[w]) c = w * 64 + __builtin_ctzll(~mask[w]);
      if (c < 0) {
        if (sub == 0) atomicOr(err, 1);
        c = 0;
      }
      if (sub == 0) {
        if (LDS) cl[u] = (unsigned char)c;
        else __hip_atomic_store(&color[u], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      // the colour is stored before any waiting node can be released
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      for (int pb = r0 + sub; pb < r1; pb += COLOR_BATCH * COLOR_LPN) {
        int ww[COLOR_BATCH];
#pragma unroll
        for (int q = 0; q < COLOR_BATCH; ++q) ww[q] = pb + q * COLOR_LPN < r1 ? radj[pb + q * COLOR_LPN] : -1;
#pragma unroll
        for (int q = 0; q < COLOR_BATCH; ++q) {
          const int w = ww[q];
          if (w < 0) continue;
          bool last;
          if (LDS) {
            const int sh = 8 * (w & 3);
            last = ((atomicSub(&wt[w >> 2], 1u << sh) >> sh) & 0xffu) == 1u;
          } else {
            last = atomicSub(&wait[w], 1) == 1;
          }
          if (last) nxt[atomicAdd(&nf_next, 1)] = w;
        }
      }
    }
    coloured += m;
    __syncthreads();
    if (threadIdx.x == 0) { nf_cur = nf_next; nf_next = 0; }
    __syncthreads();
    int* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (LDS)
    for (int v = threadIdx.x; v < n; v += 1024) color[v] = cl[v];
  if (threadIdx.x == 0) *done = coloured;
}

// One round of the same schedule as a launch of its own over the whole GPU,
// for large graphs: the nodes of the current frontier (its length in the
// counter ring rc[r mod 3]) take their colours, COLOR_LPN lanes each, and
// release the nodes waiting on them into the next frontier (rc[(r + 1) mod 3],
// zero on entry); the counter of the round before is cleared for the round
// after.  A node's colour is read only in rounds after the one that wrote it.
__global__ __launch_bounds__(256) void k_color_round(const int* __restrict__ gp, const int* __restrict__ ga,
                                                     const int* __restrict__ rptr, const int* __restrict__ radj, int* color,
                                                     int* wait, const int* __restrict__ cur, int* nxt, int* rc, int r,
                                                     int* err, int* done) {
  const int m = rc[r % 3];
  int* nnxt = rc + (r + 1) % 3;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rc[(r + 2) % 3] = 0;
    atomicAdd(done, m);
  }
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int grp = (int)(gid / COLOR_LPN), sub = (int)(gid % COLOR_LPN);
  const int ngrp = (int)((int64_t)gridDim.x * 256 / COLOR_LPN);
  // every group runs the same number of passes (the shuffles need all lanes)
  for (int i0 = 0; i0 < m; i0 += ngrp) {
    const int i = i0 + grp;
    const int u = i < m ? cur[i] : -1;
    int g0 = 0, g1 = 0, r0 = 0, r1 = 0;
    if (u >= 0) {
      g0 = gp[u];
      g1 = gp[u + 1];
      r0 = rptr[u];
      r1 = rptr[u + 1];
    }
    uint64_t mask[4] = {0, 0, 0, 0};
    for (int pb = g0 + sub; pb < g1; pb += COLOR_BATCH * COLOR_LPN) {
      int vv[COLOR_BATCH];
#pragma unroll
      for (int q = 0; q < COLOR_BATCH; ++q) vv[q] = pb + q * COLOR_LPN < g1 ? ga[pb + q * COLOR_LPN] : INT_MAX;
#pragma unroll
      for (int q = 0; q < COLOR_BATCH; ++q) {
        const int v = vv[q];
        if (v >= u) continue;
        const int c = color[v];
        if (c >= 0 && c < 256) mask[c >> 6] |= 1ull << (c & 63);
      }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int o = COLOR_LPN / 2; o > 0; o >>= 1) mask[w] |= __shfl_xor(mask[w], o, COLOR_LPN);
    if (u < 0) continue;
    int c = -1;
    for (int w = 0; w < 4 && c < 0; ++w)
      if (~mask[w]) c = w * 64 + __builtin_ctzll(~mask[w]);
    if (c < 0) {
      if (sub == 0) atomicOr(err, 1);
      c = 0;
    }
    if (sub == 0) color[u] = c;
    for (int pb = r0 + sub; pb < r1; pb += COLOR_BATCH * COLOR_LPN) {
      int ww[COLOR_BATCH];
#pragma unroll
      for (int q = 0; q < COLOR_BATCH; ++q) ww[q] = pb + q * COLOR_LPN < r1 ? radj[pb + q * COLOR_LPN] : -1;
#pragma unroll
      for (int q = 0; q < COLOR_BATCH; ++q)
        if (ww[q] >= 0 && atomicSub(&wait[ww[q]], 1) == 1) nxt[atomicAdd(nnxt, 1)] = ww[q];
    }
  }
}

// graphs too large for the LDS variant are coloured one launch per round
// (measured on the FSI-like fluid, 68,921 nodes: no faster than the LDS
// variant; on the lung-like tissue, 274,625 nodes: 12.4 ms in one workgroup)
constexpr int COLOR_ROUNDS_MIN_NODES = COLOR_LDS_NODES;

__global__ void k_max_wait(int n, const int* __restrict__ wait, int* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) atomicMax(out, wait[i]);
}

// ---- small graphs on the host: coarse levels have few nodes with many
// neighbours, where the order of a greedy colouring matters.  The colouring
// is greedy in node order (as on the device) and greedy in smallest-last
// order, and the one with fewer colours is kept (node order on ties).
// Smallest-last (Matula-Beck): nodes leave the graph one at a time, always
// one of least remaining degree, and are coloured in the reverse order.
// Ties follow stacks per degree: all nodes pushed in ascending number onto
// the stack of their degree at the start; a node whose degree drops (its
// neighbour left; neighbours in adjacency order) pushed onto its new
// degree's stack; the next node to leave is the top of the least non-empty
// stack, skipping entries of nodes that have left or moved on.
constexpr int COLOR_HOST_MAX = 32768;

static int host_greedy(int n, const std::vector<int>& gp, const std::vector<int>& ga, const std::vector<int>& order,
                       int maxdeg, std::vector<int>& col) {
  col.assign(n, -1);
  std::vector<int> stamp(maxdeg + 2, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i) {
    const int u = order[i];
    for (int p = gp[u]; p < gp[u + 1]; ++p)
      if (col[ga[p]] >= 0) stamp[col[ga[p]]] = i;
    int c = 0;
    while (stamp[c] == i) ++c;
    col[u] = c;
    nc = std::max(nc, c + 1);
  }
  return nc;
}

static void host_smallest_last(int n, const std::vector<int>& gp, const std::vector<int>& ga, int maxdeg,
                               std::vector<int>& deg, std::vector<int>& order) {
  std::vector<int> head(maxdeg + 1, -1), ent_node, ent_next;
  ent_node.reserve((size_t)n + ga.size());
  ent_next.reserve((size_t)n + ga.size());
  auto push = [&](int d, int v) {
    ent_node.push_back(v);
    ent_next.push_back(head[d]);
    head[d] = (int)ent_node.size() - 1;
  };
  for (int u = 0; u < n; ++u) push(deg[u], u);
  std::vector<char> gone(n, 0);
  order.assign(n, -1);
  int d = 0;
  for (int k = 0; k < n; ++k) {
    int u = -1;
    while (u < 0) {
      while (head[d] < 0) ++d;
      const int e = head[d];
      head[d] = ent_next[e];
      const int t = ent_node[e];
      if (!gone[t] && deg[t] == d) u = t;
    }
    gone[u] = 1;
    order[n - 1 - k] = u;   // colouring order = reverse removal order
    for (int p = gp[u]; p < gp[u + 1]; ++p) {
      const int v = ga[p];
      if (v == u || gone[v]) continue;
      push(--deg[v], v);
      d = std::min(d, deg[v]);
    }
  }
}

static int color_nodes_host(int n, const int* gp_dev, const int* ga_dev, int* color, hipStream_t s) {
  std::vector<int> gp(n + 1);
  NF_HIP(hipMemcpyAsync(gp.data(), gp_dev, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  std::vector<int> ga(gp[n]);
  if (gp[n] > 0) NF_HIP(hipMemcpyAsync(ga.data(), ga_dev, sizeof(int) * gp[n], hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  std::vector<int> deg(n, 0), order(n);
  int maxdeg = 0;
  for (int u = 0; u < n; ++u) {
    for (int p = gp[u]; p < gp[u + 1]; ++p) deg[u] += ga[p] != u;
    maxdeg = std::max(maxdeg, deg[u]);
  }
  for (int u = 0; u < n; ++u) order[u] = u;
  std::vector<int> col, col2;
  int nc = host_greedy(n, gp, ga, order, maxdeg, col);
  host_smallest_last(n, gp, ga, maxdeg, deg, order);
  const int nc2 = host_greedy(n, gp, ga, order, maxdeg, col2);
  if (nc2 < nc) {
    nc = nc2;
    col.swap(col2);
  }
  NF_CHECK(nc <= 256, NFIELD_ENOMEM, "colouring needs more than 256 colours");
  NF_HIP(hipMemcpyAsync(color, col.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  NF_HIP(hipStreamSynchronize(s));   // the host array is freed on return
  return nc;
}

int color_nodes(int n, const int* gp, const int* ga, uint64_t /*seed*/, int* color, hipStream_t s) {
  if (n == 0) return 0;
  if (n <= COLOR_HOST_MAX) return color_nodes_host(n, gp, ga, color, s);
  const int g = cdiv(n, 256);
  DBuf<int> wait(n), fa(n), fb(n), cnt(5), rcnt(n + 1), rptr(n + 1), rcur(n + 1);
  fill<int>(color, -1, n, s);
  fill<int>(cnt.p, 0, 5, s);
  fill<int>(rcnt.p, 0, n + 1, s);
  fill<int>(rcur.p, 0, n + 1, s);
  hipLaunchKernelGGL(k_color_wait, dim3(g), dim3(256), 0, s, n, gp, ga, wait.p, rcnt.p, fa.p, cnt.p);
  hipLaunchKernelGGL(k_max_wait, dim3(g), dim3(256), 0, s, n, wait.p, cnt.p + 4);
  int maxwait = 0;
  NF_HIP(hipMemcpyAsync(&maxwait, cnt.p + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  const int64_t nr = exclusive_scan(rcnt.p, rptr.p, n, s);   // synchronises: maxwait is on the host
  DBuf<int> radj(nr > 0 ? nr : 1);
  hipLaunchKernelGGL(k_color_rev, dim3(g), dim3(256), 0, s, n, gp, ga, rptr.p, rcur.p, radj.p);
  if (n > COLOR_ROUNDS_MIN_NODES) {
    // rounds in batches of 32 launches, then a look at the next frontier's length
    DBuf<int> rc(3);
    NF_HIP(hipMemcpyAsync(rc.p, cnt.p, sizeof(int), hipMemcpyDeviceToDevice, s));
    fill<int>(rc.p + 1, 0, 2, s);
    const int grid = std::min(cdiv((int64_t)n * COLOR_LPN, 256), 1024);
    int r = 0;
    while (true) {
      for (int k = 0; k < 32; ++k, ++r)
        hipLaunchKernelGGL(k_color_round, dim3(grid), dim3(256), 0, s, gp, ga, rptr.p, radj.p, color, wait.p,
                           (r & 1) ? fb.p : fa.p, (r & 1) ? fa.p : fb.p, rc.p, r, cnt.p + 1, cnt.p + 2);
      int left = 0;
      NF_HIP(hipMemcpyAsync(&left, rc.p + r % 3, sizeof(int), hipMemcpyDeviceToHost, s));
      NF_HIP(hipStreamSynchronize(s));
      if (left == 0) break;
      NF_CHECK(r <= n + 32, NFIELD_EINVAL, "colouring did not terminate");
    }
  } else if (n <= COLOR_LDS_NODES && maxwait <= 255) {
    hipLaunchKernelGGL(k_color_frontier<true>, dim3(1), dim3(1024), 0, s, n, gp, ga, rptr.p, radj.p, color, wait.p, fa.p,
                       fb.p, cnt.p, cnt.p + 1, cnt.p + 2);
  } else {
    hipLaunchKernelGGL(k_color_frontier<false>, dim3(1), dim3(1024), 0, s, n, gp, ga, rptr.p, radj.p, color, wait.p, fa.p,
                       fb.p, cnt.p, cnt.p + 1, cnt.p + 2);
  }
  hipLaunchKernelGGL(k_max_int, dim3(g), dim3(256), 0, s, color, n, cnt.p + 3);
  int h[4];
  NF_HIP(hipMemcpyAsync(h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  NF_CHECK(h[1] == 0, NFIELD_ENOMEM, "colouring needs more than 256 colours");
  NF_CHECK(h[2] == n, NFIELD_EINVAL, "colouring left nodes uncoloured");
  return h[3];
}

// D^-1, rhs and old x of row r (loaded before the row sum with one
// right-hand side; after it with several, where the registers are scarcer)
template <int NR, class T>
__device__ __forceinline__ void sgs_row_load(int r, const T* __restrict__ dinv, const T* __restrict__ rhs, int64_t ldr,
                                             const T* __restrict__ x, int64_t ldx, int nrhs, T& dv, T* rv, T* xo) {
  dv = dinv[r];
#pragma unroll
  for (int k = 0; k < NR; ++k)
    if (k == 0 || k < nrhs) {
      rv[k] = rhs[k * ldr + r];
      xo[k] = x[k * ldx + r];
    }
}

// One group of B2*G lanes per node (B2 = b rounded up to a power of two,
// G lanes per row, B2*G <= 64 so the group lies inside one wavefront): every
// row of the node is summed at once for all columns, and the updates are
// written after all of the group's loads have completed, so the node's dofs
// are relaxed together from their old values.  t indexes the colour-ordered
// node list; cptr holds, per listed node, the b + 1 row bounds of its rows, so
// the row loads need no lookup through the node id; with one right-hand side
// the row's D^-1, rhs and old x (written by this group alone) are fetched
// beside them.
template <int G, int B2, int NR, class T>
__device__ __forceinline__ void sgs_node(int t, int sub, int b, const int* __restrict__ nodes, const int* __restrict__ cptr,
                                         const int* __restrict__ col, const T* __restrict__ val, const T* __restrict__ dinv,
                                         T omega, const T* __restrict__ rhs, int64_t ldr, T* __restrict__ x, int64_t ldx,
                                         int nrhs) {
  const int q = sub / G, lane = sub % G;
  const int qc = q < b ? q : b - 1;   // rows past b (b < B2) shadow the last one
  T acc[NR], rv[NR], xo[NR];
  T dv = 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = rv[k] = xo[k] = 0;
  const int* cp = cptr + (int64_t)t * (b + 1) + qc;
  const int p0 = cp[0], p1 = cp[1];
  const int r = nodes[t] * b + qc;
  // one right-hand side: the row's D^-1, rhs and old x on every lane, loaded
  // beside the row (unconditional loads wait on no branch)
  if (NR == 1) sgs_row_load<NR, T>(r, dinv, rhs, ldr, x, ldx, nrhs, dv, rv, xo);
  row_dot<G, NR, T>(p0 + lane, q < b ? p1 : p0, col, val, x, ldx, nrhs, acc);   // shadow rows: nothing
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, G);
  if (q < b && lane == 0) {
    if (NR > 1) sgs_row_load<NR, T>(r, dinv, rhs, ldr, x, ldx, nrhs, dv, rv, xo);
    const T w = omega * dv;
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k < nrhs) x[k * ldx + r] = xo[k] + w * (rv[k] - acc[k]);
  }
}

// Workgroups go to the 8 XCDs, each with its own L2, round-robin by
// workgroup index.  xcd_block maps the hardware index b (of nb) to a logical
// one under which XCD k takes the k-th contiguous eighth of the logical
// range (a bijection: XCD k holds the b = k (mod 8)).  A colour's node list
// is in node order, so an XCD then relaxes one slab of nodes, whose gathered
// x entries share its L2 (measured on the FSI-like fine fluid level: 7.9 ->
// 7.5 us per colour launch; plain SpMV rows got slower with it).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, k = b & 7, i = b >> 3;
  return k * q + min(k, r) + i;
}

template <int G, int B2, int NR, class T>
__global__ __launch_bounds__(256) void k_sgs_color(int nnodes, const int* __restrict__ nodes, const int* __restrict__ cptr,
                                                   int b, const int* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ dinv, T omega, const T* __restrict__ rhs,
                                                   int64_t ldr, T* __restrict__ x, int64_t ldx, int nrhs) {
  constexpr int NG = G * B2;
  const int gid = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int t = gid / NG;
  if (t >= nnodes) return;
  sgs_node<G, B2, NR, T>(t, gid % NG, b, nodes, cptr, col, val, dinv, omega, rhs, ldr, x, ldx, nrhs);
}

// A whole sweep over every colour of a small level in one workgroup: the
// colours run in turn with a barrier between them (the same per-node update
// as k_sgs_color, so the results are the same bits).
template <int G, int B2, int NR, class T>
__global__ __launch_bounds__(1024) void k_sgs_sweep1(const int* __restrict__ nodes, const int* __restrict__ cptr,
                                                     const int* __restrict__ off, int ncolors, int forward, int b,
                                                     const int* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ dinv, T omega, const T* __restrict__ rhs,
                                                     int64_t ldr, T* __restrict__ x, int64_t ldx, int nrhs) {
  constexpr int NG = G * B2, PER = 1024 / NG;
  const int grp = threadIdx.x / NG, sub = threadIdx.x % NG;
  for (int ci = 0; ci < ncolors; ++ci) {
    const int c = forward ? ci : ncolors - 1 - ci;
    const int n1 = off[c + 1];
    for (int t = off[c] + grp; t < n1; t += PER)
      sgs_node<G, B2, NR, T>(t, sub, b, nodes, cptr, col, val, dinv, omega, rhs, ldr, x, ldx, nrhs);
    __syncthreads();
  }
}

// One workgroup per node for long rows: 256 / B2 lanes per row (rows in
// separate wavefronts when B2 <= 4), all loads of the node before a barrier,
// then the writes.
template <int G, int B2, int NR, class T>
__global__ __launch_bounds__(256) void k_sgs_node(const int* __restrict__ nodes, const int* __restrict__ cptr, int b,
                                                  const int* __restrict__ col, const T* __restrict__ val,
                                                  const T* __restrict__ dinv, T omega, const T* __restrict__ rhs, int64_t ldr,
                                                  T* __restrict__ x, int64_t ldx, int nrhs) {
  static_assert(G * B2 == 256 && G <= 64, "one node per 256-thread workgroup");
  // with 32 lanes per row (8-row nodes: coarse elasticity levels, rows of
  // 256-512 entries) 16 entries per lane in flight take such a row in one
  // round instead of two
  constexpr int SGS_NODE_U = NR == 1 ? (G <= 32 ? 16 : 8) : 4;
  const int t = blockIdx.x;
  const int q = threadIdx.x / G, lane = threadIdx.x % G;
  const int qc = q < b ? q : b - 1;   // rows past b (b < B2) shadow the last one
  T acc[NR], rv[NR], xo[NR];
  T dv = 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = rv[k] = xo[k] = 0;
  const int* cp = cptr + (int64_t)t * (b + 1) + qc;
  const int p0 = cp[0], p1 = cp[1];
  const int r = nodes[t] * b + qc;
  if (NR == 1) sgs_row_load<NR, T>(r, dinv, rhs, ldr, x, ldx, nrhs, dv, rv, xo);
  row_dot<G, NR, T, SGS_NODE_U>(p0 + lane, q < b ? p1 : p0, col, val, x, ldx, nrhs, acc);   // shadow rows: nothing
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, G);
  __syncthreads();
  if (q < b && lane == 0) {
    if (NR > 1) sgs_row_load<NR, T>(r, dinv, rhs, ldr, x, ldx, nrhs, dv, rv, xo);
    const T w = omega * dv;
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k < nrhs) x[k * ldx + r] = xo[k] + w * (rv[k] - acc[k]);
  }
}

// row bounds of every listed node's rows, in list order: cptr[t (b+1) + q] =
// ptr[nodes[t] b + q], q = 0..b
__global__ void k_sgs_cptr(int nnodes, const int* __restrict__ nodes, int b, const int* __restrict__ ptr,
                           int* __restrict__ cptr) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)nnodes * (b + 1)) return;
  const int t = (int)(i / (b + 1)), q = (int)(i % (b + 1));
  cptr[i] = ptr[nodes[t] * b + q];
}

void sgs_node_ptrs(const DCsr& A, int b, const int* nodes, int nnodes, int* cptr, hipStream_t s) {
  const int64_t m = (int64_t)nnodes * (b + 1);
  if (m <= 0) return;
  hipLaunchKernelGGL(k_sgs_cptr, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, s, nnodes, nodes, b, A.ptr.p, cptr);
}

template <int G, int B2, class T>
static void sgs_launch(const DCsr& A, int b, const int* nodes, const int* cptr, int nnodes, const T* val, const T* dinv,
                       T omega, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
  const int blocks = cdiv((int64_t)nnodes * G * B2, 256);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_sgs_color<G, B2, 1, T>), dim3(blocks), dim3(256), 0, s, nnodes, nodes, cptr, b, A.col.p, val,
                       dinv, omega, rhs, ldr, x, ldx, nrhs);
  else
    hipLaunchKernelGGL((k_sgs_color<G, B2, NRMAX, T>), dim3(blocks), dim3(256), 0, s, nnodes, nodes, cptr, b, A.col.p,
                       val, dinv, omega, rhs, ldr, x, ldx, nrhs);
}

template <int G, int B2, class T>
static void sgs_sweep1_launch(const int* nodes, const int* cptr, const int* off, int nc, bool forward, const DCsr& A,
                              int b, const T* val, const T* dinv, T omega, const T* rhs, int64_t ldr, T* x, int64_t ldx,
                              int nrhs, hipStream_t s) {
  if (nrhs == 1)
    hipLaunchKernelGGL((k_sgs_sweep1<G, B2, 1, T>), dim3(1), dim3(1024), 0, s, nodes, cptr, off, nc, forward ? 1 : 0, b,
                       A.col.p, val, dinv, omega, rhs, ldr, x, ldx, nrhs);
  else
    hipLaunchKernelGGL((k_sgs_sweep1<G, B2, NRMAX, T>), dim3(1), dim3(1024), 0, s, nodes, cptr, off, nc, forward ? 1 : 0,
                       b, A.col.p, val, dinv, omega, rhs, ldr, x, ldx, nrhs);
}

template <int B2, class T>
static void sgs_node_launch(const int* nodes, const int* cptr, int nnodes, const DCsr& A, int b, const T* val,
                            const T* dinv, T omega, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
  constexpr int G = 256 / B2;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_sgs_node<G, B2, 1, T>), dim3(nnodes), dim3(256), 0, s, nodes, cptr, b, A.col.p, val, dinv,
                       omega, rhs, ldr, x, ldx, nrhs);
  else
    hipLaunchKernelGGL((k_sgs_node<G, B2, NRMAX, T>), dim3(nnodes), dim3(256), 0, s, nodes, cptr, b, A.col.p, val, dinv,
                       omega, rhs, ldr, x, ldx, nrhs);
}

int sgs_lanes(const DCsr& A, int b) {
  int b2 = 1;
  while (b2 < b) b2 <<= 1;
  int g = spmv_lanes(A.nr, A.nnz);
  while (g * b2 > 64) g >>= 1;
  return g < 2 ? 2 : g;
}

int sgs_kind(const DCsr& A, int b, int nnodes_total, int ncolors) {
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
  // one workgroup costs about as much as 8 per-colour launches on these levels
  if (ncolors >= SGS_SWEEP1_MIN_COLORS && A.nnz <= SGS_SWEEP1_MAX_NNZ && A.nr > 0 && A.nnz / A.nr <= SGS_SWEEP1_MAX_ROW &&
      nnodes_total <= SGS_SWEEP1_MAX_NODES)
    return SGS_SWEEP1;
  if (B2 >= 4 && A.nr > 0 && A.nnz / A.nr >= SGS_NODE_MIN_ROW) return SGS_NODE;
  return SGS_COLOR;
}

template <class T>
void sgs_sweep(const DCsr& A, int b, const int* nodes, const int* cptr, const int* off_dev, const std::vector<int>& off,
               bool forward, const T* dinv, T omega, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
  const int nc = (int)off.size() - 1;
  if (nc <= 0) return;
  NF_CHECK(b >= 1 && b <= MAXB, NFIELD_EINVAL, "Gauss-Seidel: block size above 8");
  NF_CHECK(nrhs >= 1 && nrhs <= NRMAX, NFIELD_EINVAL, "more than 8 right-hand sides in one call");
  const T* val = csr_values<T>(A);
  const int kind = sgs_kind(A, b, off[nc], nc);
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
  if (kind == SGS_SWEEP1) {
    const int G = sgs_lanes(A, b);
#define NF_SGS1(GG, BB) \
  if (G == GG && B2 == BB) return sgs_sweep1_launch<GG, BB, T>(nodes, cptr, off_dev, nc, forward, A, b, val, dinv, omega, rhs, ldr, x, ldx, nrhs, s);
    NF_SGS1(2, 1) NF_SGS1(4, 1) NF_SGS1(8, 1) NF_SGS1(16, 1) NF_SGS1(32, 1) NF_SGS1(64, 1)
    NF_SGS1(2, 2) NF_SGS1(4, 2) NF_SGS1(8, 2) NF_SGS1(16, 2) NF_SGS1(32, 2)
    NF_SGS1(2, 4) NF_SGS1(4, 4) NF_SGS1(8, 4) NF_SGS1(16, 4)
    NF_SGS1(2, 8) NF_SGS1(4, 8) NF_SGS1(8, 8)
#undef NF_SGS1
    throw NfError(NFIELD_EINVAL, "Gauss-Seidel: no kernel for this lane layout");
  }
  for (int i = 0; i < nc; ++i) {
    const int c = forward ? i : nc - 1 - i;
    const int m = off[c + 1] - off[c];
    if (m <= 0) continue;
    if (kind == SGS_NODE) {
      const int* cp = cptr + (int64_t)off[c] * (b + 1);
      if (B2 == 4) sgs_node_launch<4, T>(nodes + off[c], cp, m, A, b, val, dinv, omega, rhs, ldr, x, ldx, nrhs, s);
      else sgs_node_launch<8, T>(nodes + off[c], cp, m, A, b, val, dinv, omega, rhs, ldr, x, ldx, nrhs, s);
    } else {
      sgs_color<T>(A, b, nodes + off[c], cptr + (int64_t)off[c] * (b + 1), m, dinv, omega, rhs, ldr, x, ldx, nrhs, s);
    }
  }
}

template <class T>
void sgs_color(const DCsr& A, int b, const int* nodes, const int* cptr, int nnodes, const T* dinv, T omega, const T* rhs,
               int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
  if (nnodes <= 0) return;
  NF_CHECK(b >= 1 && b <= MAXB, NFIELD_EINVAL, "Gauss-Seidel: block size above 8");
  NF_CHECK(nrhs >= 1 && nrhs <= NRMAX, NFIELD_EINVAL, "more than 8 right-hand sides in one call");
  const T* val = csr_values<T>(A);
  const int G = sgs_lanes(A, b);
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
#define NF_SGS(GG, BB) \
  if (G == GG && B2 == BB) return sgs_launch<GG, BB, T>(A, b, nodes, cptr, nnodes, val, dinv, omega, rhs, ldr, x, ldx, nrhs, s);
  NF_SGS(2, 1) NF_SGS(4, 1) NF_SGS(8, 1) NF_SGS(16, 1) NF_SGS(32, 1) NF_SGS(64, 1)
  NF_SGS(2, 2) NF_SGS(4, 2) NF_SGS(8, 2) NF_SGS(16, 2) NF_SGS(32, 2)
  NF_SGS(2, 4) NF_SGS(4, 4) NF_SGS(8, 4) NF_SGS(16, 4)
  NF_SGS(2, 8) NF_SGS(4, 8) NF_SGS(8, 8)
#undef NF_SGS
  throw NfError(NFIELD_EINVAL, "Gauss-Seidel: no kernel for this lane layout");
}
__global__ void k_color_traffic(int nnodes, const int* __restrict__ nodes, int b, const int* __restrict__ ptr,
                                const int* __restrict__ col, int stamp, int* touched, unsigned long long* out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nnodes) return;
  const int u = nodes[t];
  unsigned long long e = 0, d = 0;
  for (int q = 0; q < b; ++q) {
    const int r = u * b + q;
    e += ptr[r + 1] - ptr[r];
    for (int p = ptr[r]; p < ptr[r + 1]; ++p)
      if (atomicExch(&touched[col[p]], stamp) != stamp) ++d;
  }
  atomicAdd(&out[0], e);
  atomicAdd(&out[1], d);
}
void color_traffic(const DCsr& A, int b, const int* nodes, const std::vector<int>& off, std::vector<int64_t>& nnz,
                   std::vector<int64_t>& ncols, hipStream_t s) {
  const int nc = (int)off.size() - 1;
  DBuf<int> touched(A.nc > 0 ? A.nc : 1);
  DBuf<unsigned long long> out(2 * (nc > 0 ? nc : 1));
  fill<int>(touched.p, -1, A.nc, s);
  fill<unsigned long long>(out.p, 0ull, 2 * (int64_t)nc, s);
  for (int c = 0; c < nc; ++c) {
    const int m = off[c + 1] - off[c];
    if (m > 0)
      hipLaunchKernelGGL(k_color_traffic, dim3(cdiv(m, 256)), dim3(256), 0, s, m, nodes + off[c], b, A.ptr.p, A.col.p, c,
                         touched.p, out.p + 2 * c);
  }
  std::vector<unsigned long long> h(2 * nc);
  NF_HIP(hipMemcpyAsync(h.data(), out.p, sizeof(unsigned long long) * 2 * nc, hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  nnz.resize(nc);
  ncols.resize(nc);
  for (int c = 0; c < nc; ++c) {
    nnz[c] = (int64_t)h[2 * c];
    ncols[c] = (int64_t)h[2 * c + 1];
  }
}

// Dense form of one symmetric Gauss-Seidel sweep on a small level: the
// sweep is affine, x_new = S x + Q b, so it is run on X = [I | 0] with
// right-hand sides [0 | I] (2n columns), giving X = [S | Q].  The columns
// are independent sweeps: one workgroup takes `tile` of them through every
// colour (forward then backward) with the tile held in LDS, a barrier between
// colours; within a colour each thread owns one (node, row), and all rows of
// the colour are summed before any is written, so a node's dofs are relaxed
// together from their old values, as in the colour kernels.
constexpr int DSGS_LDS_DOUBLES = 19456;   // 152 KiB of the 160 KiB LDS
constexpr int DSGS_MAX_TILE = 4;
__global__ __launch_bounds__(256) void k_dense_sgs_tile(double* __restrict__ X, int n, int tile, const int* __restrict__ nodes,
                                                        const int* __restrict__ off, int nc, int b, const int* __restrict__ ptr,
                                                        const int* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ dinv, double omega) {
  __shared__ double xs[DSGS_LDS_DOUBLES];     // xs[r * tile + t] = X[r][j0 + t]
  const int j0 = blockIdx.x * tile;
  const int nt = min(tile, 2 * n - j0);
  for (int e = threadIdx.x; e < n * tile; e += 256) {
    const int r = e / tile, t = e % tile;
    xs[e] = (t < nt && j0 + t < n && r == j0 + t) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = 0; i < 2 * nc; ++i) {
    const int c = i < nc ? i : 2 * nc - 1 - i;
    const int m = (off[c + 1] - off[c]) * b;
    for (int e0 = 0; e0 < m; e0 += 256) {
      const int e = e0 + threadIdx.x;
      int r = -1;
      double acc[DSGS_MAX_TILE] = {0.0, 0.0, 0.0, 0.0};
      if (e < m) {
        r = nodes[off[c] + e / b] * b + e % b;
        for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
          const double v = val[p];
          const double* xr = xs + (int64_t)col[p] * tile;
#pragma unroll
          for (int t = 0; t < DSGS_MAX_TILE; ++t)
            if (t < nt) acc[t] += v * xr[t];
        }
      }
      __syncthreads();
      if (r >= 0) {
        const double w = omega * dinv[r];
#pragma unroll
        for (int t = 0; t < DSGS_MAX_TILE; ++t)
          if (t < nt) {
            const double rhs = (j0 + t >= n && r == j0 + t - n) ? 1.0 : 0.0;
            xs[r * tile + t] += w * (rhs - acc[t]);
          }
      }
      __syncthreads();
    }
  }
  const int64_t ld = 2 * (int64_t)n;
  for (int e = threadIdx.x; e < n * tile; e += 256) {
    const int r = e / tile, t = e % tile;
    if (t < nt) X[r * ld + j0 + t] = xs[e];
  }
}
void dense_sgs_build(const DCsr& A, int b, const int* nodes, const int* off_dev, const std::vector<int>& off,
                     const double* dinv, double omega, double* X, hipStream_t s) {
  const int n = A.nr, nc = (int)off.size() - 1;
  const int tile = std::min(DSGS_MAX_TILE, DSGS_LDS_DOUBLES / std::max(n, 1));
  NF_CHECK(tile >= 1, NFIELD_EINVAL, "dense Gauss-Seidel sweep: level too large");
  hipLaunchKernelGGL(k_dense_sgs_tile, dim3(cdiv(2 * n, tile)), dim3(256), 0, s, X, n, tile, nodes, off_dev, nc, b, A.ptr.p,
                     A.col.p, A.val.p, dinv, omega);
  NF_HIP(hipGetLastError());
}

// y = S x + Q b (or Q b alone) for the dense sweep X = [S | Q] (n x 2n,
// row-major, stored in T): one wavefront per row, columns lane-strided
template <int NR, class T>
__global__ __launch_bounds__(256) void k_dense_sweep_apply(const T* __restrict__ X, int n, const T* __restrict__ x, int64_t ldx,
                                                           const T* __restrict__ rb, int64_t ldb, T* __restrict__ y, int64_t ldy,
                                                           int nrhs, int with_x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  const T* m = X + (int64_t)row * 2 * n;
  if (with_x)
    for (int j = lane; j < n; j += 64) {
      const double mj = m[j];
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (k < nrhs) acc[k] += mj * (double)x[k * ldx + j];
    }
  for (int j = lane; j < n; j += 64) {
    const double mj = m[n + j];
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k < nrhs) acc[k] += mj * (double)rb[k * ldb + j];
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k >= nrhs) break;
    const double v = wave_sum(acc[k]);
    if (lane == 0) y[k * ldy + row] = (T)v;
  }
}
template <class T>
void dense_sweep_apply(const T* X, int n, const T* x, int64_t ldx, const T* rb, int64_t ldb, T* y, int64_t ldy, int nrhs,
                       bool with_x, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_dense_sweep_apply<1, T>), dim3(cdiv(n, 4)), dim3(256), 0, s, X, n, x, ldx, rb, ldb, y, ldy, nrhs,
                       with_x ? 1 : 0);
  else
    hipLaunchKernelGGL((k_dense_sweep_apply<NRMAX, T>), dim3(cdiv(n, 4)), dim3(256), 0, s, X, n, x, ldx, rb, ldb, y, ldy, nrhs,
                       with_x ? 1 : 0);
}
// ---- block copies of node-blocked matrices.  A level whose matrix is made
// of dense b x b node blocks (b = 2 or 3: elasticity, velocity) keeps a copy
// with one column node per block and each node's values together, entry by
// entry (entry (q, c) of all its blocks, then the next), so that the lanes
// of a node, which take consecutive blocks, read consecutive addresses, and
// a colour's launch reads each of its nodes' values as one stretch.
//
// The copy comes straight from the CSR.  A matrix passes the check when row r of
// node u has the length of the node's first row and its entries are, block
// by block, the b consecutive columns of the block column that the first row
// has there; the entries before node u then number b^2 times the blocks
// before it.
constexpr int BSR_COPY_LANES = 16;   // lanes per row of the check and the copy
__global__ void k_bsr_dense_check(int nr, int b, const int* __restrict__ ptr, const int* __restrict__ col,
                                  int* __restrict__ bad) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = (int)(gid / BSR_COPY_LANES), lane = (int)(gid % BSR_COPY_LANES);
  if (r >= nr) return;
  const int u = r / b;
  const int f0 = ptr[u * b], len = ptr[u * b + 1] - f0, p0 = ptr[r];
  bool ok = len % b == 0 && ptr[r + 1] - p0 == len && f0 % (b * b) == 0;
  for (int k = lane * b; ok && k < len; k += BSR_COPY_LANES * b) {
    const int c0 = col[f0 + k];
    ok = c0 % b == 0;
    for (int c = 0; ok && c < b; ++c) ok = col[p0 + k + c] == c0 + c;
  }
  if (!ok) atomicOr(bad, 1);
}
// dense copy: block j of node u is number ptr[u b] / b^2 + j; its entry
// (q, c) goes to the node's values at (q b + c) nu + j (nu: the node's blocks)
template <class T>
__global__ void k_bsr_dense_copy(int nr, int b, const int* __restrict__ ptr, const int* __restrict__ col,
                                 const double* __restrict__ val, int* __restrict__ bcol, T* __restrict__ bval) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = (int)(gid / BSR_COPY_LANES), lane = (int)(gid % BSR_COPY_LANES);
  if (r >= nr) return;
  const int u = r / b, q = r % b;
  const int64_t blk0 = ptr[u * b] / (b * b);
  const int p0 = ptr[r], len = ptr[r + 1] - p0, nu = len / b;
  T* nv = bval + blk0 * b * b;
  for (int i = lane; i < len; i += BSR_COPY_LANES) {
    const int j = i / b, c = i % b;
    nv[(q * b + c) * nu + j] = (T)val[p0 + i];
    if (q == 0 && c == 0) bcol[blk0 + j] = col[p0 + i] / b;
  }
}
__global__ void k_bsr_dense_ptr(int nnodes, int b, const int* __restrict__ ptr, int* __restrict__ bptr) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u <= nnodes) bptr[u] = ptr[u * b] / (b * b);
}
// the block row bounds of each listed node, 2 ints per node in list order
__global__ void k_bsr_node_bounds(int nnodes, const int* __restrict__ nodes, const int* __restrict__ bptr,
                                  int* __restrict__ bcp) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nnodes) return;
  const int u = nodes[t];
  bcp[2 * t] = bptr[u];
  bcp[2 * t + 1] = bptr[u + 1];
}

// One colour of the Gauss-Seidel sweep from the block copy: G lanes per node,
// each lane taking whole blocks (two at a time in flight), the node's B row
// sums reduced across its G lanes; lanes 0..B-1 write the node's B values
// (x_r += omega D^-1_r (b_r - A_r x), A_r x with the node's own old values,
// as k_sgs_color).  Colours are independent sets, so only the own node's x
// is both read and written, by lanes of one wavefront, reads first.
template <int B, int G, class T>
__global__ __launch_bounds__(256) void k_sgs_color_bsr(int nnodes, const int* __restrict__ nodes,
                                                       const int* __restrict__ bcp, const int* __restrict__ bcol,
                                                       const T* __restrict__ bval, const T* __restrict__ dinv, T omega,
                                                       const T* __restrict__ rhs, T* __restrict__ x) {
  const int gid = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int t = gid / G, lane = gid % G;
  if (t >= nnodes) return;   // whole groups of G lanes together
  const int node = nodes[t];
  const int k0 = bcp[2 * t], k1 = bcp[2 * t + 1];
  // the node's own entries, loaded by every lane (lanes past B repeat the
  // last row's) so that no load waits on a branch
  const int64_t r = (int64_t)node * B + (lane < B ? lane : B - 1);
  const T dv = dinv[r], rv = rhs[r], xo = x[r];
  T acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = 0;
  const int nu = k1 - k0;
  for (int j = lane; j < nu; j += 2 * G)
    bsr_block_rows<B, T>(j, j + G, j + G < nu, nu, bcol + k0, bval + (int64_t)k0 * B * B, x, acc);
#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, G);
  T a = acc[0];
#pragma unroll
  for (int q = 1; q < B; ++q)
    if (lane == q) a = acc[q];
  const T w = omega * dv;
  if (lane < B) x[r] = xo + w * (rv - a);
}

template <class T> static DBuf<T>& bsr_store(DCsr& A);
template <> DBuf<double>& bsr_store<double>(DCsr& A) { return A.bsr_val; }
template <> DBuf<float>& bsr_store<float>(DCsr& A) { return A.bsr_val32; }
static std::mutex g_bsr_mu;

// the copy of A in precision T (and its structure, shared by both
// precisions); false, keeping nothing new, when some node block of A is not
// full
template <class T> static bool bsr_build(DCsr& A, int b, hipStream_t s) {
  if ((b != 2 && b != 3) || A.nnz % ((int64_t)b * b) != 0) return false;
  const int nnodes = A.nr / b;
  const unsigned rows_grid = (unsigned)cdiv((int64_t)A.nr * BSR_COPY_LANES, 256);
  {
    DBuf<int> bad(1);
    fill<int>(bad.p, 0, 1, s);
    hipLaunchKernelGGL(k_bsr_dense_check, dim3(rows_grid), dim3(256), 0, s, A.nr, b, A.ptr.p, A.col.p, bad.p);
    int h = 1;
    NF_HIP(hipMemcpyAsync(&h, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    if (h) return false;
  }
  const int64_t nblk = A.nnz / (b * b);
  DBuf<T>& bval = bsr_store<T>(A);
  A.bsr_ptr.alloc((size_t)nnodes + 1);
  hipLaunchKernelGGL(k_bsr_dense_ptr, dim3(cdiv(nnodes + 1, 256)), dim3(256), 0, s, nnodes, b, A.ptr.p, A.bsr_ptr.p);
  A.bsr_col.alloc(nblk);
  bval.alloc((size_t)nblk * b * b);
  hipLaunchKernelGGL(k_bsr_dense_copy<T>, dim3(rows_grid), dim3(256), 0, s, A.nr, b, A.ptr.p, A.col.p, A.val.p,
                     A.bsr_col.p, bval.p);
  A.bsr_nblk = nblk;
  NF_HIP(hipGetLastError());
  NF_HIP(hipStreamSynchronize(s));   // complete before another stream's smoother may read it
  A.bsr_b = b;
  return true;
}

template <class T>
bool sgs_bsr_setup(const DCsr& A_, int b, const int* nodes, int nnodes, DBuf<int>& bcp, hipStream_t s) {
  DCsr& A = const_cast<DCsr&>(A_);   // the copy is kept with the matrix
  if (b < 2 || b > 3 || nnodes <= 0 || A.nnz <= 0 || A.nr != nnodes * b || A.nc != A.nr) return false;
  {
    std::lock_guard<std::mutex> lock(g_bsr_mu);   // smoothers of one matrix set up side by side
    if (!bsr_store<T>(A).p) {
      if (A.bsr_b) {   // the other precision's copy: same structure, values again
        const int b0 = A.bsr_b;
        A.bsr_b = 0;
        if (!bsr_build<T>(A, b0, s)) return false;
      } else if (!bsr_build<T>(A, b, s)) {
        return false;
      }
    }
  }
  bcp.alloc((size_t)2 * nnodes);
  hipLaunchKernelGGL(k_bsr_node_bounds, dim3(cdiv(nnodes, 256)), dim3(256), 0, s, nnodes, nodes, A.bsr_ptr.p, bcp.p);
  NF_HIP(hipGetLastError());
  return true;
}

template <int B, class T>
static void sgs_bsr_launch(const int* nodes, const int* bcp, const DCsr& A, const T* bv, int m, const T* dinv, T omega,
                           const T* rhs, T* x, hipStream_t s) {
  constexpr int G = SGS_BSR_LANES;
  const unsigned blocks = (unsigned)cdiv((int64_t)m * G, 256);
  hipLaunchKernelGGL((k_sgs_color_bsr<B, G, T>), dim3(blocks), dim3(256), 0, s, m, nodes, bcp, A.bsr_col.p, bv, dinv,
                     omega, rhs, x);
}

template <class T>
void sgs_sweep_bsr(const DCsr& A, const int* nodes, const int* bcp, const std::vector<int>& off, bool forward,
                   const T* dinv, T omega, const T* rhs, T* x, hipStream_t s) {
  const int nc = (int)off.size() - 1;
  const T* bv = bsr_values<T>(A);
  NF_CHECK(A.bsr_b && bv, NFIELD_EINVAL, "Gauss-Seidel: the matrix has no block copy");
  for (int i = 0; i < nc; ++i) {
    const int c = forward ? i : nc - 1 - i;
    const int m = off[c + 1] - off[c];
    if (m <= 0) continue;
    const int* nd = nodes + off[c];
    const int* bc = bcp + (int64_t)2 * off[c];
    if (A.bsr_b == 2) sgs_bsr_launch<2, T>(nd, bc, A, bv, m, dinv, omega, rhs, x, s);
    else sgs_bsr_launch<3, T>(nd, bc, A, bv, m, dinv, omega, rhs, x, s);
  }
}
template bool sgs_bsr_setup<double>(const DCsr&, int, const int*, int, DBuf<int>&, hipStream_t);
template bool sgs_bsr_setup<float>(const DCsr&, int, const int*, int, DBuf<int>&, hipStream_t);
template void sgs_sweep_bsr<double>(const DCsr&, const int*, const int*, const std::vector<int>&, bool, const double*,
                                    double, const double*, double*, hipStream_t);
template void sgs_sweep_bsr<float>(const DCsr&, const int*, const int*, const std::vector<int>&, bool, const float*,
                                   float, const float*, float*, hipStream_t);

template void dense_sweep_apply<double>(const double*, int, const double*, int64_t, const double*, int64_t, double*, int64_t,
                                        int, bool, hipStream_t);
template void dense_sweep_apply<float>(const float*, int, const float*, int64_t, const float*, int64_t, float*, int64_t, int,
                                       bool, hipStream_t);

template void sgs_sweep<double>(const DCsr&, int, const int*, const int*, const int*, const std::vector<int>&, bool,
                                const double*, double, const double*, int64_t, double*, int64_t, int, hipStream_t);
template void sgs_sweep<float>(const DCsr&, int, const int*, const int*, const int*, const std::vector<int>&, bool,
                               const float*, float, const float*, int64_t, float*, int64_t, int, hipStream_t);
template void sgs_color<double>(const DCsr&, int, const int*, const int*, int, const double*, double, const double*, int64_t,
                                double*, int64_t, int, hipStream_t);
template void sgs_color<float>(const DCsr&, int, const int*, const int*, int, const float*, float, const float*, int64_t,
                               float*, int64_t, int, hipStream_t);

// ==================================================================== DD(GS)
// Domain-decomposition Gauss-Seidel: the nodes are split into subdomains
// (the level's aggregates); one workgroup owns one subdomain, whose nodes are
// listed by (subdomain, colour, node).  At set-up every row of the list is
// split into its own part (couplings to nodes of the same subdomain, columns
// as local dof indices: position in the subdomain's list times b plus the
// component) and its other part (couplings to other subdomains, global
// columns), both stored in list order.  A sweep:
//  1. stage the subdomain's x in LDS and ext = rhs - (other part) xo, where
//     xo holds every node's value at the sweep's start (NULL: zero) -- fully
//     parallel over the subdomain's rows, the only gather of the sweep;
//  2. colour by colour (a barrier between colours, colours without nodes in
//     the subdomain skipped): each node's dofs together from their old
//     values, x_r += omega dinv_r (ext_r - (own part) x), own values in LDS;
//  3. write the subdomain's x back.
// Workgroups never read what another one writes.
template <int G, int U, int NR, class T>
__device__ __forceinline__ void dd_row_sum(int p0, int p1, const int* __restrict__ col, const T* __restrict__ val,
                                           const T* src, int64_t lds, int nrhs, T* s) {
  for (int p = p0; p < p1; p += U * G) {
    T v[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = p + u * G;
      v[u] = q < p1 ? val[q] : (T)0;
      c[u] = q < p1 ? col[q] : -1;
    }
    T xv[U][NR];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) xv[u][k] = (c[u] >= 0 && k < nrhs) ? src[k * lds + c[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (c[u] >= 0 && k < nrhs) s[k] += v[u] * xv[u][k];
  }
}

// LDS of one workgroup (md = max_nodes * b dofs): xs and ext (NR columns of
// md values each), the node ids, and the own and other row bounds of the
// subdomain's rows (md + 1 each, relative to its first entry).
template <int G1, int U1, int G2, int B2, int NR, class T>
__global__ __launch_bounds__(256) void k_dd_sweep(const int* __restrict__ nodes, const int* __restrict__ off, int nc,
                                                  int forward, int b, const int* __restrict__ optr,
                                                  const int* __restrict__ ocol, const T* __restrict__ oval,
                                                  const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                  const T* __restrict__ xval, const T* __restrict__ dinv, T omega,
                                                  const T* __restrict__ rhs, int64_t ldr, const T* __restrict__ xo,
                                                  int64_t ldxo, T* __restrict__ x, int64_t ldx, int nrhs, int max_nodes) {
  extern __shared__ __align__(16) unsigned char dd_lds[];
  const int* so = off + (int64_t)blockIdx.x * (nc + 1);
  const int base = so[0], nn = so[nc] - base, nd = nn * b;
  const int md = max_nodes * b;
  T* xs = (T*)dd_lds;
  T* ext = xs + (size_t)NR * md;
  int* nid = (int*)(ext + (size_t)NR * md);
  int* ob = nid + max_nodes;
  int* xb = ob + md + 1;
  const int rb = base * b;
  // node ids and row bounds of the subdomain: one round trip
  for (int e = threadIdx.x; e < nn; e += 256) nid[e] = nodes[base + e];
  for (int e = threadIdx.x; e <= nd; e += 256) {
    ob[e] = optr[rb + e];
    xb[e] = xptr[rb + e];
  }
  __syncthreads();
  // 1. own values, and ext = rhs - (other part) xo with G1 lanes per row,
  // U1 entries per lane in flight
  for (int e = threadIdx.x; e < nd * NR; e += 256) {
    const int k = e / nd, d = e % nd;
    const int64_t r = (int64_t)nid[d / b] * b + d % b;
    xs[k * md + d] = k < nrhs ? x[k * ldx + r] : (T)0;
  }
  {
    const int lane = threadIdx.x % G1;
    for (int d0 = 0; d0 < nd; d0 += 256 / G1) {
      const int d = d0 + threadIdx.x / G1;
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = 0;
      if (d < nd && xo) dd_row_sum<G1, U1, NR, T>(xb[d] + lane, xb[d + 1], xcol, xval, xo, ldxo, nrhs, acc);
#pragma unroll
      for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int o = G1 / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, G1);
      if (d < nd && lane == 0) {
        const int64_t r = (int64_t)nid[d / b] * b + d % b;
#pragma unroll
        for (int k = 0; k < NR; ++k)
          if (k < nrhs) ext[k * md + d] = rhs[k * ldr + r] - acc[k];
      }
    }
  }
  __syncthreads();
  // 2. the colours
  constexpr int NG = G2 * B2, PER = 256 / NG;
  const int grp = threadIdx.x / NG, sub = threadIdx.x % NG;
  const int q = sub / G2, lane = sub % G2;
  for (int ci = 0; ci < nc; ++ci) {
    const int c = forward ? ci : nc - 1 - ci;
    const int t0 = so[c] - base, t1 = so[c + 1] - base;
    if (t0 == t1) continue;   // no node of this colour here (uniform over the workgroup)
    for (int t = t0 + grp; t < t1; t += PER) {
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = 0;
      const int d = t * b + q;
      if (q < b) dd_row_sum<G2, NR == 1 ? 8 : 4, NR, T>(ob[d] + lane, ob[d + 1], ocol, oval, xs, md, nrhs, acc);
#pragma unroll
      for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int o = G2 / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, G2);
      if (q < b && lane == 0) {
        const T w = omega * dinv[(int64_t)nid[t] * b + q];
#pragma unroll
        for (int k = 0; k < NR; ++k)
          if (k < nrhs) xs[k * md + d] = xs[k * md + d] + w * (ext[k * md + d] - acc[k]);
      }
    }
    __syncthreads();
  }
  // 3. write back
  for (int e = threadIdx.x; e < nd * NR; e += 256) {
    const int k = e / nd, d = e % nd;
    if (k < nrhs) x[k * ldx + (int64_t)nid[d / b] * b + d % b] = xs[k * md + d];
  }
}

// own / other entry counts of every listed row (list order: row lr = t b + q)
__global__ void k_dd_split_count(int nlist, int b, const int* __restrict__ nodes, const int* __restrict__ ptr,
                                 const int* __restrict__ col, const int* __restrict__ sub, int* __restrict__ nown,
                                 int* __restrict__ noth) {
  const int lr = blockIdx.x * 256 + threadIdx.x;
  if (lr >= nlist * b) return;
  const int u = nodes[lr / b], r = u * b + lr % b, su = sub[u];
  int o = 0, x = 0;
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    if (sub[col[p] / b] == su) ++o;
    else ++x;
  }
  nown[lr] = o;
  noth[lr] = x;
}
template <class T>
__global__ void k_dd_split_fill(int nlist, int b, const int* __restrict__ nodes, const int* __restrict__ ptr,
                                const int* __restrict__ col, const double* __restrict__ val, const int* __restrict__ sub,
                                const int* __restrict__ pos, const int* __restrict__ optr, int* __restrict__ ocol,
                                T* __restrict__ oval, const int* __restrict__ xptr, int* __restrict__ xcol,
                                T* __restrict__ xval) {
  const int lr = blockIdx.x * 256 + threadIdx.x;
  if (lr >= nlist * b) return;
  const int u = nodes[lr / b], r = u * b + lr % b, su = sub[u];
  int o = optr[lr], x = xptr[lr];
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    const int c = col[p];
    if (sub[c / b] == su) {
      ocol[o] = pos[c / b] * b + c % b;
      oval[o++] = (T)val[p];
    } else {
      xcol[x] = c;
      xval[x++] = (T)val[p];
    }
  }
}

template <class T>
void dd_split(const DCsr& A, int b, int nlist, const int* nodes, const int* sub, const int* pos, DBuf<int>& optr,
              DBuf<int>& ocol, DBuf<T>& oval, DBuf<int>& xptr, DBuf<int>& xcol, DBuf<T>& xval, hipStream_t s) {
  const int nr = nlist * b;
  DBuf<int> no(nr + 1), nx(nr + 1);
  optr.alloc(nr + 1);
  xptr.alloc(nr + 1);
  if (nr > 0)
    hipLaunchKernelGGL(k_dd_split_count, dim3(cdiv(nr, 256)), dim3(256), 0, s, nlist, b, nodes, A.ptr.p, A.col.p, sub,
                       no.p, nx.p);
  const int64_t to = exclusive_scan(no.p, optr.p, nr, s), tx = exclusive_scan(nx.p, xptr.p, nr, s);
  ocol.alloc(to > 0 ? to : 1);
  oval.alloc(to > 0 ? to : 1);
  xcol.alloc(tx > 0 ? tx : 1);
  xval.alloc(tx > 0 ? tx : 1);
  if (nr > 0)
    hipLaunchKernelGGL(k_dd_split_fill<T>, dim3(cdiv(nr, 256)), dim3(256), 0, s, nlist, b, nodes, A.ptr.p, A.col.p,
                       A.val.p, sub, pos, optr.p, ocol.p, oval.p, xptr.p, xcol.p, xval.p);
}
template void dd_split<double>(const DCsr&, int, int, const int*, const int*, const int*, DBuf<int>&, DBuf<int>&,
                               DBuf<double>&, DBuf<int>&, DBuf<int>&, DBuf<double>&, hipStream_t);
template void dd_split<float>(const DCsr&, int, int, const int*, const int*, const int*, DBuf<int>&, DBuf<int>&,
                              DBuf<float>&, DBuf<int>&, DBuf<int>&, DBuf<float>&, hipStream_t);

size_t dd_lds_bytes(int b, int max_nodes, int nrhs, size_t val_bytes) {
  const int NR = nrhs == 1 ? 1 : NRMAX;
  const size_t md = (size_t)max_nodes * b;
  return 2 * val_bytes * (size_t)NR * md + sizeof(int) * ((size_t)max_nodes + 2 * (md + 1));
}

// lanes per row of the own part: two to four entries per lane, at most
// 64 / B2 (a node's rows in one wavefront)
static int dd_lanes(double avg, int cap) {
  int g = 1;
  while (g * 4 <= avg && g < 64) g *= 2;
  if (g < 2) g = 2;
  while (g > cap) g >>= 1;
  return g;
}

template <int G1, int U1, int G2, int B2, class T>
static void dd_launch(int nsub, const int* nodes, const int* off, int nc, bool forward, int b, const int* optr,
                      const int* ocol, const T* oval, const int* xptr, const int* xcol, const T* xval, const T* dinv,
                      T omega, const T* rhs, int64_t ldr, const T* xo, int64_t ldxo, T* x, int64_t ldx, int nrhs,
                      int max_nodes, hipStream_t s) {
  const size_t lds = dd_lds_bytes(b, max_nodes, nrhs, sizeof(T));
  if (nrhs == 1)
    hipLaunchKernelGGL((k_dd_sweep<G1, U1, G2, B2, 1, T>), dim3(nsub), dim3(256), lds, s, nodes, off, nc,
                       forward ? 1 : 0, b, optr, ocol, oval, xptr, xcol, xval, dinv, omega, rhs, ldr, xo, ldxo, x, ldx,
                       nrhs, max_nodes);
  else
    hipLaunchKernelGGL((k_dd_sweep<G1, 4, G2, B2, NRMAX, T>), dim3(nsub), dim3(256), lds, s, nodes, off, nc,
                       forward ? 1 : 0, b, optr, ocol, oval, xptr, xcol, xval, dinv, omega, rhs, ldr, xo, ldxo, x, ldx,
                       nrhs, max_nodes);
}

// Lanes per row: G1 for the other part, G2 for the own part, each from the
// part's mean row length (two to four entries per lane).
template <class T>
void dd_sweep(int b, int nsub, const int* nodes, const int* off_dev, int nc, bool forward, double avg_own,
              double avg_other, const int* optr, const int* ocol, const T* oval, const int* xptr, const int* xcol,
              const T* xval, const T* dinv, T omega, const T* rhs, int64_t ldr, const T* xo, int64_t ldxo, T* x,
              int64_t ldx, int nrhs, int max_nodes, hipStream_t s) {
  if (nsub <= 0 || nc <= 0) return;
  NF_CHECK(b >= 1 && b <= MAXB, NFIELD_EINVAL, "DD(GS): block size above 8");
  NF_CHECK(nrhs >= 1 && nrhs <= NRMAX, NFIELD_EINVAL, "more than 8 right-hand sides in one call");
  NF_CHECK(dd_lds_bytes(b, max_nodes, nrhs, sizeof(T)) <= DD_LDS_MAX, NFIELD_EINVAL,
           "DD(GS): a subdomain is too large for the workgroup's LDS");
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
  const int G2 = dd_lanes(avg_own, 64 / B2), G1 = dd_lanes(avg_other, 16);
  const int U1 = 8;
#define NF_DD(A1, V1, A2, BB)                                                                                        \
  if (G1 == A1 && U1 == V1 && G2 == A2 && B2 == BB)                                                                  \
    return dd_launch<A1, V1, A2, BB, T>(nsub, nodes, off_dev, nc, forward, b, optr, ocol, oval, xptr, xcol, xval, dinv, \
                                        omega, rhs, ldr, xo, ldxo, x, ldx, nrhs, max_nodes, s);
#define NF_DD_G2(A1, V1) \
  NF_DD(A1, V1, 2, 1) NF_DD(A1, V1, 4, 1) NF_DD(A1, V1, 8, 1) NF_DD(A1, V1, 16, 1) NF_DD(A1, V1, 32, 1)  \
  NF_DD(A1, V1, 64, 1) NF_DD(A1, V1, 2, 2) NF_DD(A1, V1, 4, 2) NF_DD(A1, V1, 8, 2) NF_DD(A1, V1, 16, 2) \
  NF_DD(A1, V1, 32, 2) NF_DD(A1, V1, 2, 4) NF_DD(A1, V1, 4, 4) NF_DD(A1, V1, 8, 4) NF_DD(A1, V1, 16, 4) \
  NF_DD(A1, V1, 2, 8) NF_DD(A1, V1, 4, 8) NF_DD(A1, V1, 8, 8)
  NF_DD_G2(1, 8) NF_DD_G2(2, 8) NF_DD_G2(4, 8) NF_DD_G2(8, 8) NF_DD_G2(16, 8)
  NF_DD_G2(1, 16) NF_DD_G2(2, 16) NF_DD_G2(4, 16) NF_DD_G2(8, 16) NF_DD_G2(16, 16)
#undef NF_DD_G2
#undef NF_DD
  throw NfError(NFIELD_EINVAL, "DD(GS): no kernel for this lane layout");
}
template void dd_sweep<double>(int, int, const int*, const int*, int, bool, double, double, const int*, const int*,
                               const double*, const int*, const int*, const double*, const double*, double,
                               const double*, int64_t, const double*, int64_t, double*, int64_t, int, int, hipStream_t);
template void dd_sweep<float>(int, int, const int*, const int*, int, bool, double, double, const int*, const int*,
                              const float*, const int*, const int*, const float*, const float*, float, const float*,
                              int64_t, const float*, int64_t, float*, int64_t, int, int, hipStream_t);

// ======================================================= tentative prolongator
__global__ void k_count_by(int n, const int* __restrict__ key, int* cnt) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < n) atomicAdd(&cnt[key[u]], 1);
}
__global__ void k_place_by(int n, const int* __restrict__ key, const int* __restrict__ off, int* cursor, int* out) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < n) out[off[key[u]] + atomicAdd(&cursor[key[u]], 1)] = u;
}
__global__ void k_ptent_pattern(int ndof, int b, int k, const int* __restrict__ agg, int* ptr, int* col) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r > ndof) return;
  ptr[r] = r * k;
  if (r == ndof) return;
  const int a = agg[r / b];
  for (int j = 0; j < k; ++j) col[r * k + j] = a * k + j;
}
// One wavefront per aggregate: order its nodes (each lane ranks some of the
// members against all of them; the members are distinct node ids), copy the
// near-nullspace rows, then modified Gram-Schmidt with positive R diagonal
// (each lane owns a strided set of the aggregate's rows; inner products are
// wavefront sums); a column whose remaining norm is <= 1e-12 ||B_a||_F is
// dead: zero in Q, zero row in R, flagged.  Aggregates of up to
// TQR_LDS_MEMBERS nodes are ranked and kept in LDS, larger ones in `sorted`.
constexpr int TQR_LDS_MEMBERS = 1024;
__global__ __launch_bounds__(64) void k_tentative_qr(int nagg, int b, int k, int ndof, const int* __restrict__ aoff,
                                                     const int* __restrict__ members, int* __restrict__ sorted,
                                                     const double* __restrict__ B, double* __restrict__ Q,
                                                     double* __restrict__ Bc, int* __restrict__ dead) {
  __shared__ int raw[TQR_LDS_MEMBERS], ord[TQR_LDS_MEMBERS];
  const int a = blockIdx.x, lane = threadIdx.x;
  if (a >= nagg) return;
  const int m0 = aoff[a], m1 = aoff[a + 1], m = m1 - m0;
  const bool in_lds = m <= TQR_LDS_MEMBERS;
  const int* src = members + m0;
  if (in_lds) {
    for (int t = lane; t < m; t += 64) raw[t] = members[m0 + t];
    __syncthreads();
    src = raw;
  }
  for (int t = lane; t < m; t += 64) {
    const int v = src[t];
    int rk = 0;
    for (int i = 0; i < m; ++i) rk += src[i] < v ? 1 : 0;
    if (in_lds) ord[rk] = v;
    else sorted[m0 + rk] = v;
  }
  __syncthreads();
  const int* mem = in_lds ? ord : sorted + m0;
  const int rows = (m1 - m0) * b, nc = nagg * k;
  double fro = 0.0;
  for (int t = lane; t < rows; t += 64) {
    const int r = mem[t / b] * b + t % b;
    for (int j = 0; j < k; ++j) {
      const double v = B[(int64_t)j * ndof + r];
      Q[(int64_t)r * k + j] = v;
      fro += v * v;
    }
  }
  fro = sqrt(wave_sum(fro));
  double R[MAXB * MAXB];
  for (int q = 0; q < MAXB * MAXB; ++q) R[q] = 0.0;
  for (int j = 0; j < k; ++j) {
    for (int l = 0; l < j; ++l) {
      double rr = 0.0;
      for (int t = lane; t < rows; t += 64) {
        const int64_t r = (int64_t)(mem[t / b] * b + t % b) * k;
        rr += Q[r + l] * Q[r + j];
      }
      rr = wave_sum(rr);
      R[l * MAXB + j] = rr;
      for (int t = lane; t < rows; t += 64) {
        const int64_t r = (int64_t)(mem[t / b] * b + t % b) * k;
        Q[r + j] -= rr * Q[r + l];
      }
    }
    double nr = 0.0;
    for (int t = lane; t < rows; t += 64) {
      const int64_t r = (int64_t)(mem[t / b] * b + t % b) * k;
      nr += Q[r + j] * Q[r + j];
    }
    nr = sqrt(wave_sum(nr));
    const bool is_dead = nr <= 1e-12 * fro;
    for (int t = lane; t < rows; t += 64) {
      const int64_t r = (int64_t)(mem[t / b] * b + t % b) * k;
      Q[r + j] = is_dead ? 0.0 : Q[r + j] / nr;
    }
    if (is_dead) {
      for (int l = j; l < k; ++l) R[j * MAXB + l] = 0.0;
    } else {
      R[j * MAXB + j] = nr;
    }
    if (lane == 0) dead[a * k + j] = is_dead ? 1 : 0;
  }
  if (lane == 0)
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Bc[(int64_t)j * nc + a * k + i] = R[i * MAXB + j];
}
__global__ void k_compact_flags(int n, const int* __restrict__ flag, const int* __restrict__ off, int* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && flag[i]) out[off[i]] = i;
}

int tentative(int nnode, int b, int k, const int* agg, int nagg, const double* B, DCsr& P, DBuf<double>& Bc,
              DBuf<int>& dead, hipStream_t s) {
  NF_CHECK(k >= 1 && k <= MAXB, NFIELD_EINVAL, "near-nullspace dimension must be between 1 and 8");
  const int ndof = nnode * b, nc = nagg * k;
  NF_CHECK((int64_t)ndof * k < INT_MAX, NFIELD_ENOMEM, "tentative prolongator too large");
  DBuf<int> cnt(nagg + 1), aoff(nagg + 1), cursor(nagg + 1), members(nnode > 0 ? nnode : 1), sorted(nnode > 0 ? nnode : 1),
      dflag(nc + 1), doff(nc + 1);
  fill<int>(cnt.p, 0, nagg + 1, s);
  fill<int>(cursor.p, 0, nagg + 1, s);
  const int g = cdiv(nnode, 256);
  hipLaunchKernelGGL(k_count_by, dim3(g), dim3(256), 0, s, nnode, agg, cnt.p);
  exclusive_scan(cnt.p, aoff.p, nagg, s);
  hipLaunchKernelGGL(k_place_by, dim3(g), dim3(256), 0, s, nnode, agg, aoff.p, cursor.p, members.p);
  P.nr = ndof;
  P.nc = nc;
  P.nnz = (int64_t)ndof * k;
  P.ptr.alloc(ndof + 1);
  P.col.alloc(P.nnz);
  P.val.alloc(P.nnz);
  Bc.alloc((size_t)k * nc);
  hipLaunchKernelGGL(k_ptent_pattern, dim3(cdiv(ndof + 1, 256)), dim3(256), 0, s, ndof, b, k, agg, P.ptr.p, P.col.p);
  if (nagg > 0)
    hipLaunchKernelGGL(k_tentative_qr, dim3(nagg), dim3(64), 0, s, nagg, b, k, ndof, aoff.p, members.p, sorted.p, B, P.val.p, Bc.p,
                       dflag.p);
  const int ndead = (int)exclusive_scan(dflag.p, doff.p, nc, s);
  dead.alloc(ndead > 0 ? ndead : 1);
  if (ndead > 0) hipLaunchKernelGGL(k_compact_flags, dim3(cdiv(nc, 256)), dim3(256), 0, s, nc, dflag.p, doff.p, dead.p);
  return ndead;
}

// P <- P_tent + s .* (A P_tent), in place on the product (whose pattern
// contains that of P_tent because A has its whole diagonal stored)
__global__ void k_smooth_P(int nr, const int* __restrict__ ptr, const int* __restrict__ col, double* __restrict__ val,
                           const double* __restrict__ srow, const double* __restrict__ ptv, int b, int k,
                           const int* __restrict__ agg) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  const double sr = srow[r];
  const int a = agg[r / b];
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    const int c = col[p];
    double v = val[p] * sr;
    if (c / k == a) v = ptv[(int64_t)r * k + (c - a * k)] + v;
    val[p] = v;
  }
}
void smooth_prolongator(DCsr& AP, const double* srow, const DCsr& Pt, int b, int k, const int* agg, hipStream_t s) {
  if (AP.nr > 0)
    hipLaunchKernelGGL(k_smooth_P, dim3(cdiv(AP.nr, 256)), dim3(256), 0, s, AP.nr, AP.ptr.p, AP.col.p, AP.val.p, srow,
                       Pt.val.p, b, k, agg);
}

// Petrov-Galerkin dampings: om[j] = <AP e_j, AQ e_j> / ||AQ e_j||^2 (0 where
// that is not positive or AQ e_j = 0), from the transposes (rows = columns
// of P, entries in ascending row order): one thread per column, its sums in
// ascending row order.
__global__ void k_pg_omega(int nc, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
                           const int* __restrict__ qp, const int* __restrict__ qc, const double* __restrict__ qv,
                           double* __restrict__ om) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nc) return;
  int p = ap[j];
  const int pe = ap[j + 1];
  double num = 0.0, den = 0.0;
  for (int q = qp[j]; q < qp[j + 1]; ++q) {
    const int r = qc[q];
    const double v = qv[q];
    while (p < pe && ac[p] < r) ++p;
    if (p < pe && ac[p] == r) num += av[p] * v;
    den += v * v;
  }
  om[j] = (den > 0.0 && num > 0.0) ? num / den : 0.0;
}
void pg_omega(const DCsr& AP, const DCsr& AQ, double* om, hipStream_t s) {
  DCsr APt, AQt;
  transpose(AP, APt, s);
  transpose(AQ, AQt, s);
  if (AP.nc > 0)
    hipLaunchKernelGGL(k_pg_omega, dim3(cdiv(AP.nc, 256)), dim3(256), 0, s, AP.nc, APt.ptr.p, APt.col.p, APt.val.p,
                       AQt.ptr.p, AQt.col.p, AQt.val.p, om);
  NF_HIP(hipStreamSynchronize(s));   // the transposes are freed on return
}
// P = P_tent - Q diag(om) on the pattern of Q (= that of A P_tent), written
// into val; P_tent entries as in k_smooth_P
__global__ void k_pg_P(int nr, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ qv,
                       const double* __restrict__ om, const double* __restrict__ ptv, int b, int k,
                       const int* __restrict__ agg, double* __restrict__ val) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  const int a = agg[r / b];
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    const int c = col[p];
    double v = -om[c] * qv[p];
    if (c / k == a) v = ptv[(int64_t)r * k + (c - a * k)] + v;
    val[p] = v;
  }
}
void pg_prolongator(const DCsr& Q, const double* om, const DCsr& Pt, int b, int k, const int* agg, DCsr& P,
                    hipStream_t s) {
  csr_copy(Q, P, s);
  if (Q.nr > 0)
    hipLaunchKernelGGL(k_pg_P, dim3(cdiv(Q.nr, 256)), dim3(256), 0, s, Q.nr, Q.ptr.p, Q.col.p, Q.val.p, om, Pt.val.p, b,
                       k, agg, P.val.p);
}

// ===================================================================== SpGEMM
// C = A B, row by row, one wavefront per row.  Pass 1 counts the distinct
// columns of each row with an LDS hash set; pass 2 rebuilds the set in a
// table sized for the row, sorts it (bitonic, LDS) and accumulates
// a_ik b_kj into the sorted slots in ascending k: the lanes of one step work
// on distinct columns of row k of B, so every entry is summed in the same
// order as a serial row-by-row product, without atomics.
constexpr int SPG_COUNT_CAP = 4096;
constexpr int EMPTY_KEY = INT_MAX;

__device__ __forceinline__ int hash_slot(int key, int logts) {
  return (int)(((uint32_t)key * 2654435761u) >> (32 - logts));
}
// returns 1 if the key was new, 0 if present, -1 if the table is full
// (a plain read first: most inserts of a product row are repeats, which then
// need no atomic; an empty slot is claimed by compare-and-swap)
__device__ __forceinline__ int hash_insert(int* table, int ts, int logts, int key) {
  int h = logts > 0 ? hash_slot(key, logts) : 0;
  for (int probe = 0; probe < ts; ++probe) {
    int cur = __hip_atomic_load(&table[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == key) return 0;
    if (cur == EMPTY_KEY) {
      cur = atomicCAS(&table[h], EMPTY_KEY, key);
      if (cur == EMPTY_KEY) return 1;
      if (cur == key) return 0;
    }
    h = (h + 1) & (ts - 1);
  }
  return -1;
}

// distinct-column count of listed rows: WAVES rows per block, one wavefront
// and one LDS hash table of CAP slots per row
// (rows whose table fills up are appended to ovf, count in ovf_n, and are
// counted again by the dense-accumulator path)
template <int CAP, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_spgemm_count(const int* __restrict__ rows, int nrows, const int* __restrict__ Ap,
                                                             const int* __restrict__ Ac, const int* __restrict__ Bp,
                                                             const int* __restrict__ Bc, int* __restrict__ cnt, int* ovf,
                                                             int* ovf_n) {
  __shared__ int tables[WAVES][CAP];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = blockIdx.x * WAVES + w;
  if (idx >= nrows) return;            // whole wavefront leaves; no block barrier below
  int* table = tables[w];
  const int row = rows[idx];
  for (int i = lane; i < CAP; i += 64) table[i] = EMPTY_KEY;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  int logc = 0;
  for (int t = CAP; t > 1; t >>= 1) ++logc;
  int mine = 0, full = 0;
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + lane; q < Bp[k + 1]; q += 64) {
      const int r = hash_insert(table, CAP, logc, Bc[q]);
      if (r > 0) ++mine;
      if (r < 0) full = 1;
    }
  }
  const int tot = wave_sum_int(mine);
  const int anyfull = wave_sum_int(full);
  if (lane == 0) {
    if (anyfull) ovf[atomicAdd(ovf_n, 1)] = row;
    else cnt[row] = tot;
  }
}

// upper bound of each product row's length; rows split into three lists
// (LDS tables of 512 and 4096 slots, dense accumulator beyond)
__global__ void k_spgemm_bin_ub(int nr, const int* __restrict__ Ap, const int* __restrict__ Ac, const int* __restrict__ Bp,
                                int small_max, int big_max, int* small, int* nsmall, int* big, int* nbig, int* huge, int* nhuge,
                                int* cnt, int* ubrow, unsigned long long* ubtotal) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  int64_t ub = 0;
  for (int p = Ap[r]; p < Ap[r + 1]; ++p) ub += Bp[Ac[p] + 1] - Bp[Ac[p]];
  ubrow[r] = (int)std::min<int64_t>(ub, INT_MAX);
  atomicAdd(ubtotal, (unsigned long long)ub);
  if (ub == 0) cnt[r] = 0;
  else if (ub <= small_max) small[atomicAdd(nsmall, 1)] = r;
  else if (ub <= big_max) big[atomicAdd(nbig, 1)] = r;
  else huge[atomicAdd(nhuge, 1)] = r;
}

// Dense-accumulator product rows (rows too long for the LDS tables): one
// workgroup per row with a private flag array and accumulator over all
// columns of B (batch slot = blockIdx.x).  Count: mark, then clear while
// counting first clears, which leaves the flags zero for the next row.
__global__ __launch_bounds__(256) void k_spa_count(const int* __restrict__ rows, const int* __restrict__ Ap,
                                                   const int* __restrict__ Ac, const int* __restrict__ Bp,
                                                   const int* __restrict__ Bc, int ncols, int* flags, int* cnt) {
  __shared__ int part[4];
  const int row = rows[blockIdx.x], t = threadIdx.x;
  int* f = flags + (int64_t)blockIdx.x * ncols;
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256) f[Bc[q]] = 1;
  }
  __syncthreads();
  int mine = 0;
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256)
      if (atomicExch(&f[Bc[q]], 0) == 1) ++mine;
  }
  mine = wave_sum_int(mine);
  if ((t & 63) == 0) part[t >> 6] = mine;
  __syncthreads();
  if (t == 0) cnt[row] = part[0] + part[1] + part[2] + part[3];
}

// Fill: accumulate a_ik b_kj into acc[j] in ascending k (a barrier after
// each k; the lanes of one step hold distinct columns), collect the touched
// columns, sort them (bitonic in the slot's key scratch of ts entries), then
// write the row in column order and clear what was touched.
__global__ __launch_bounds__(256) void k_spa_fill(const int* __restrict__ rows, const int* __restrict__ Ap,
                                                  const int* __restrict__ Ac, const double* __restrict__ Av,
                                                  const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                  const double* __restrict__ Bv, const int* __restrict__ Cp, int* __restrict__ Ccol,
                                                  double* __restrict__ Cval, int ncols, int* flags, double* accs, int* kscr, int ts) {
  __shared__ int pos;
  const int row = rows[blockIdx.x], t = threadIdx.x;
  int* f = flags + (int64_t)blockIdx.x * ncols;
  double* acc = accs + (int64_t)blockIdx.x * ncols;
  int* ks = kscr + (int64_t)blockIdx.x * ts;
  const int c0 = Cp[row], cnt = Cp[row + 1] - c0;
  if (t == 0) pos = 0;
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    const double a = Av[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256) {
      const int j = Bc[q];
      acc[j] += a * Bv[q];
      f[j] = 1;
    }
    __syncthreads();
  }
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256) {
      const int j = Bc[q];
      if (atomicExch(&f[j], 0) == 1) {
        const int at = atomicAdd(&pos, 1);
        if (at < ts) ks[at] = j;
      }
    }
  }
  __syncthreads();
  for (int i = pos + t; i < ts; i += 256) ks[i] = EMPTY_KEY;
  __syncthreads();
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = t; i < ts; i += 256) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = ks[i], y = ks[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { ks[i] = y; ks[ixj] = x; }
        }
      }
      __syncthreads();
    }
  for (int i = t; i < cnt; i += 256) {
    const int j = ks[i];
    const bool ok = j >= 0 && j < ncols;   // always true when the count pass matched
    Ccol[c0 + i] = ok ? j : 0;
    Cval[c0 + i] = ok ? acc[j] : 0.0;
    if (ok) acc[j] = 0.0;
  }
}

// WAVES rows per workgroup, one wavefront and one LDS table of CAP slots per
// row (wavefront-level barriers only)
template <int CAP, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_spgemm_fill(const int* __restrict__ rows, int nrows, const int* __restrict__ Ap,
                                                            const int* __restrict__ Ac, const double* __restrict__ Av,
                                                            const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                            const double* __restrict__ Bv, const int* __restrict__ Cp,
                                                            int* __restrict__ Ccol, double* __restrict__ Cval) {
  __shared__ int keys_all[WAVES][CAP];
  __shared__ double acc_all[WAVES][CAP];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = blockIdx.x * WAVES + w;
  if (idx >= nrows) return;            // whole wavefront leaves; only wavefront barriers below
  int* keys = keys_all[w];
  double* acc = acc_all[w];
  const int row = rows[idx];
  const int c0 = Cp[row], cnt = Cp[row + 1] - c0;
  if (cnt == 0) return;
  int ts = 1, logts = 0;
  while (ts < 2 * cnt) { ts <<= 1; ++logts; }
  if (ts > CAP) { ts = CAP; logts = 0; for (int t = CAP; t > 1; t >>= 1) ++logts; }
  auto wave_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  for (int i = lane; i < ts; i += 64) keys[i] = EMPTY_KEY;
  wave_sync();
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + lane; q < Bp[k + 1]; q += 64) hash_insert(keys, ts, logts, Bc[q]);
  }
  wave_sync();
  // bitonic sort of the table (ascending; empty slots sort last)
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < ts; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = keys[i], y = keys[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { keys[i] = y; keys[ixj] = x; }
        }
      }
      wave_sync();
    }
  for (int i = lane; i < cnt; i += 64) acc[i] = 0.0;
  wave_sync();
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    const double a = Av[p];
    for (int q = Bp[k] + lane; q < Bp[k + 1]; q += 64) {
      const int key = Bc[q];
      int lo = 0, hi = cnt;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
      }
      acc[lo] += a * Bv[q];
    }
    wave_sync();
  }
  for (int i = lane; i < cnt; i += 64) {
    Ccol[c0 + i] = keys[i];
    Cval[c0 + i] = acc[i];
  }
}

// Single-pass product rows: the LDS hash set of the row is built, counted,
// sorted and accumulated as in k_spgemm_fill, and the row is written to a
// scratch at the row's upper-bound offset (its count in cnt); rows the table
// cannot hold are listed in ovf for the dense accumulator.
template <int CAP>
__global__ __launch_bounds__(64) void k_spgemm_fill_ub(const int* __restrict__ rows, int nrows, const int* __restrict__ nrows_dev,
                                                       const int* __restrict__ Ap,
                                                       const int* __restrict__ Ac, const double* __restrict__ Av,
                                                       const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                       const double* __restrict__ Bv, const int* __restrict__ toff,
                                                       const int* __restrict__ ubrow, int* __restrict__ tcol,
                                                       double* __restrict__ tval, int* __restrict__ cnt, int* ovf, int* ovf_n) {
  __shared__ int keys[CAP];
  __shared__ double acc[CAP];
  __shared__ int npos;
  // the list's length on the device (a list another pass wrote) when given;
  // workgroups stride over the list
  const int nlist = nrows_dev ? *nrows_dev : nrows;
  for (int bi = blockIdx.x; bi < nlist; bi += gridDim.x) {
    __syncthreads();
    const int row = rows[bi], lane = threadIdx.x;
    const int ub = ubrow[row];
    int ts = 1, logts = 0;
    while (ts < 2 * ub && ts < CAP) { ts <<= 1; ++logts; }
    for (int i = lane; i < ts; i += 64) keys[i] = EMPTY_KEY;
    __syncthreads();
    int mine = 0, full = 0;
    for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
      const int k = Ac[p];
      for (int q = Bp[k] + lane; q < Bp[k + 1]; q += 64) {
        const int r = hash_insert(keys, ts, logts, Bc[q]);
        if (r > 0) ++mine;
        if (r < 0) full = 1;
      }
    }
    const int c = wave_sum_int(mine);
    if (wave_sum_int(full)) {
      if (lane == 0) ovf[atomicAdd(ovf_n, 1)] = row;
      continue;
    }
    // gather the c keys to the front (through the accumulator's storage), pad
    // to a power of two and sort only that
    int* tmp = (int*)acc;
    if (lane == 0) npos = 0;
    __syncthreads();
    for (int i = lane; i < ts; i += 64) {
      const int k = keys[i];
      if (k != EMPTY_KEY) tmp[atomicAdd(&npos, 1)] = k;
    }
    __syncthreads();
    int ts2 = 1;
    while (ts2 < c) ts2 <<= 1;
    for (int i = lane; i < ts2; i += 64) keys[i] = i < c ? tmp[i] : EMPTY_KEY;
    __syncthreads();
    for (int kk = 2; kk <= ts2; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < ts2; i += 64) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const int x = keys[i], y = keys[ixj];
            const bool up = (i & kk) == 0;
            if ((x > y) == up) { keys[i] = y; keys[ixj] = x; }
          }
        }
        __syncthreads();
      }
    for (int i = lane; i < c; i += 64) acc[i] = 0.0;
    __syncthreads();
    for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
      const int k = Ac[p];
      const double a = Av[p];
      for (int q = Bp[k] + lane; q < Bp[k + 1]; q += 64) {
        const int key = Bc[q];
        int lo = 0, hi = c;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (keys[mid] < key) lo = mid + 1; else hi = mid;
        }
        acc[lo] += a * Bv[q];
      }
      __syncthreads();
    }
    const int o = toff[row];
    for (int i = lane; i < c; i += 64) {
      tcol[o + i] = keys[i];
      tval[o + i] = acc[i];
    }
    if (lane == 0) cnt[row] = c;
  }
}

// the dense-accumulator row of k_spa_fill written to the scratch at the
// row's upper-bound offset, its count in cnt (ts >= the row's distinct count)
__global__ __launch_bounds__(256) void k_spa_fill_ub(const int* __restrict__ rows, const int* __restrict__ Ap,
                                                     const int* __restrict__ Ac, const double* __restrict__ Av,
                                                     const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                     const double* __restrict__ Bv, const int* __restrict__ toff,
                                                     int* __restrict__ tcol, double* __restrict__ tval, int* __restrict__ cnt,
                                                     int ncols, int* flags, double* accs, int* kscr, int ts) {
  __shared__ int pos;
  const int row = rows[blockIdx.x], t = threadIdx.x;
  int* f = flags + (int64_t)blockIdx.x * ncols;
  double* acc = accs + (int64_t)blockIdx.x * ncols;
  int* ks = kscr + (int64_t)blockIdx.x * ts;
  if (t == 0) pos = 0;
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    const double a = Av[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256) {
      const int j = Bc[q];
      acc[j] += a * Bv[q];
      f[j] = 1;
    }
    __syncthreads();
  }
  for (int p = Ap[row]; p < Ap[row + 1]; ++p) {
    const int k = Ac[p];
    for (int q = Bp[k] + t; q < Bp[k + 1]; q += 256) {
      const int j = Bc[q];
      if (atomicExch(&f[j], 0) == 1) {
        const int at = atomicAdd(&pos, 1);
        if (at < ts) ks[at] = j;
      }
    }
  }
  __syncthreads();
  const int c = pos < ts ? pos : ts;
  for (int i = c + t; i < ts; i += 256) ks[i] = EMPTY_KEY;
  __syncthreads();
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = t; i < ts; i += 256) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = ks[i], y = ks[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { ks[i] = y; ks[ixj] = x; }
        }
      }
      __syncthreads();
    }
  const int o = toff[row];
  for (int i = t; i < c; i += 256) {
    const int j = ks[i];
    tcol[o + i] = j;
    tval[o + i] = acc[j];
    acc[j] = 0.0;
  }
  if (t == 0) cnt[row] = c;
}

// C row r = scratch[toff[r], toff[r] + cnt[r]) (one wavefront per row)
__global__ __launch_bounds__(256) void k_spgemm_compact(int nr, const int* __restrict__ toff, const int* __restrict__ Cp,
                                                        const int* __restrict__ tcol, const double* __restrict__ tval,
                                                        int* __restrict__ Ccol, double* __restrict__ Cval) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= nr) return;
  const int o = toff[r], c0 = Cp[r], n = Cp[r + 1] - c0;
  for (int i = lane; i < n; i += 64) {
    Ccol[c0 + i] = tcol[o + i];
    Cval[c0 + i] = tval[o + i];
  }
}

// split rows by their distinct count into the two LDS table sizes and the
// dense-accumulator list
__global__ void k_bin_rows(int nr, const int* __restrict__ Cp, int small_max, int big_max, int* small, int* nsmall, int* big,
                           int* nbig, int* huge, int* nhuge, int* maxlen) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  const int c = Cp[r + 1] - Cp[r];
  if (c == 0) return;
  if (c <= small_max) small[atomicAdd(nsmall, 1)] = r;
  else if (c <= big_max) big[atomicAdd(nbig, 1)] = r;
  else {
    huge[atomicAdd(nhuge, 1)] = r;
    atomicMax(maxlen, c);
  }
}

// rows of the dense-accumulator path run in batches of concurrent slots,
// each slot holding a flag and an accumulator entry per column of B
static int spa_slots(int ncols, int nrows, int extra_per_slot) {
  const int64_t per = (int64_t)ncols * 12 + (int64_t)extra_per_slot * 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nrows, ((int64_t)1 << 29) / std::max<int64_t>(per, 1)));
}

// scratch of the single-pass product (upper-bound slots) above which the
// two-pass product (count, then fill in place) is used
constexpr int64_t SPG_ONEPASS_MAX_SLOTS = (int64_t)1 << 28;

void spgemm(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s) {
  NF_CHECK(A.nc == B.nr, NFIELD_EINVAL, "spgemm: inner dimensions differ");
  C.nr = A.nr;
  C.nc = B.nc;
  C.ptr.alloc(A.nr + 1);
  const int nr1 = A.nr > 0 ? A.nr : 1;
  DBuf<int> cnt(A.nr + 1), flags(8), ubrow(A.nr + 1);
  DBuf<unsigned long long> ubtot(1);
  DBuf<int> small(nr1), big(nr1), huge(nr1);
  fill<int>(flags.p, 0, 8, s);
  fill<int>(cnt.p, 0, A.nr + 1, s);
  fill<unsigned long long>(ubtot.p, 0ull, 1, s);
  int h_flags[8];
  if (A.nr > 0 && A.nnz > 0 && B.nnz > 0) {
    // rows with an upper bound above 256 go to the 4096-slot table; rows it
    // cannot hold (more than 4096 distinct columns) to the dense accumulator
    hipLaunchKernelGGL(k_spgemm_bin_ub, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, B.ptr.p, 256,
                       INT_MAX, small.p, flags.p, big.p, flags.p + 1, huge.p, flags.p + 2, cnt.p, ubrow.p, ubtot.p);
    unsigned long long h_ub = 0;
    NF_HIP(hipMemcpyAsync(h_flags, flags.p, sizeof(h_flags), hipMemcpyDeviceToHost, s));
    NF_HIP(hipMemcpyAsync(&h_ub, ubtot.p, sizeof(h_ub), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    const int ns = h_flags[0], nb = h_flags[1];
    if (h_ub <= (unsigned long long)SPG_ONEPASS_MAX_SLOTS) {
      // single pass: rows into upper-bound slots of a scratch, then compacted
      DBuf<int> toff(A.nr + 1), tcol(h_ub > 0 ? h_ub : 1);
      DBuf<double> tval(h_ub > 0 ? h_ub : 1);
      exclusive_scan(ubrow.p, toff.p, A.nr, s);
      fill<int>(flags.p + 3, 0, 1, s);
      // rows with an upper bound above 256 try a 1024-slot table (small LDS,
      // many workgroups per CU); rows with more distinct columns retry with
      // 4096 slots, and beyond that the dense accumulator
      DBuf<int> big2(nr1);
      fill<int>(flags.p + 4, 0, 1, s);
      if (ns > 0)
        hipLaunchKernelGGL(k_spgemm_fill_ub<512>, dim3(ns), dim3(64), 0, s, small.p, ns, (const int*)nullptr, A.ptr.p,
                           A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, toff.p, ubrow.p, tcol.p, tval.p, cnt.p, huge.p,
                           flags.p + 3);
      if (nb > 0) {
        hipLaunchKernelGGL(k_spgemm_fill_ub<1024>, dim3(nb), dim3(64), 0, s, big.p, nb, (const int*)nullptr, A.ptr.p,
                           A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, toff.p, ubrow.p, tcol.p, tval.p, cnt.p, big2.p,
                           flags.p + 4);
        // the retries: the list's length stays on the device, a bounded grid
        // strides over it
        hipLaunchKernelGGL(k_spgemm_fill_ub<4096>, dim3(std::min(nb, 2048)), dim3(64), 0, s, big2.p, nb, flags.p + 4, A.ptr.p, A.col.p,
                           A.val.p, B.ptr.p, B.col.p, B.val.p, toff.p, ubrow.p, tcol.p, tval.p, cnt.p, huge.p, flags.p + 3);
      }
      int nh = 0;
      NF_HIP(hipMemcpyAsync(&nh, flags.p + 3, sizeof(int), hipMemcpyDeviceToHost, s));
      NF_HIP(hipStreamSynchronize(s));
      if (nh > 0) {
        // longest overflow row bounds its distinct count by min(upper bound, columns)
        std::vector<int> hrows(nh), hub(A.nr);
        NF_HIP(hipMemcpyAsync(hrows.data(), huge.p, sizeof(int) * nh, hipMemcpyDeviceToHost, s));
        NF_HIP(hipMemcpyAsync(hub.data(), ubrow.p, sizeof(int) * A.nr, hipMemcpyDeviceToHost, s));
        NF_HIP(hipStreamSynchronize(s));
        int mx = 1;
        for (int r : hrows) mx = std::max(mx, std::min(hub[r], B.nc));
        int ts = 1;
        while (ts < mx) ts <<= 1;
        const int slots = spa_slots(B.nc, nh, ts);
        DBuf<int> f((size_t)slots * B.nc), ks((size_t)slots * ts);
        DBuf<double> acc((size_t)slots * B.nc);
        fill<int>(f.p, 0, (int64_t)slots * B.nc, s);
        fill<double>(acc.p, 0.0, (int64_t)slots * B.nc, s);
        for (int r0 = 0; r0 < nh; r0 += slots)
          hipLaunchKernelGGL(k_spa_fill_ub, dim3(std::min(slots, nh - r0)), dim3(256), 0, s, huge.p + r0, A.ptr.p, A.col.p,
                             A.val.p, B.ptr.p, B.col.p, B.val.p, toff.p, tcol.p, tval.p, cnt.p, B.nc, f.p, acc.p, ks.p, ts);
      }
      C.nnz = exclusive_scan(cnt.p, C.ptr.p, A.nr, s);
      C.col.alloc(C.nnz > 0 ? C.nnz : 1);
      C.val.alloc(C.nnz > 0 ? C.nnz : 1);
      if (C.nnz > 0)
        hipLaunchKernelGGL(k_spgemm_compact, dim3(cdiv(A.nr, 4)), dim3(256), 0, s, A.nr, toff.p, C.ptr.p, tcol.p, tval.p,
                           C.col.p, C.val.p);
      NF_HIP(hipGetLastError());
      return;
    }
    if (ns > 0)
      hipLaunchKernelGGL((k_spgemm_count<512, 4>), dim3(cdiv(ns, 4)), dim3(256), 0, s, small.p, ns, A.ptr.p, A.col.p, B.ptr.p,
                         B.col.p, cnt.p, huge.p, flags.p + 2);
    if (nb > 0)
      hipLaunchKernelGGL((k_spgemm_count<SPG_COUNT_CAP, 1>), dim3(nb), dim3(64), 0, s, big.p, nb, A.ptr.p, A.col.p, B.ptr.p,
                         B.col.p, cnt.p, huge.p, flags.p + 2);
    NF_HIP(hipMemcpyAsync(h_flags, flags.p, sizeof(h_flags), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    const int nh = h_flags[2];
    if (nh > 0) {
      const int slots = spa_slots(B.nc, nh, 0);
      DBuf<int> f((size_t)slots * B.nc);
      fill<int>(f.p, 0, (int64_t)slots * B.nc, s);
      for (int r0 = 0; r0 < nh; r0 += slots)
        hipLaunchKernelGGL(k_spa_count, dim3(std::min(slots, nh - r0)), dim3(256), 0, s, huge.p + r0, A.ptr.p, A.col.p,
                           B.ptr.p, B.col.p, B.nc, f.p, cnt.p);
      NF_HIP(hipStreamSynchronize(s));
    }
  }
  C.nnz = exclusive_scan(cnt.p, C.ptr.p, A.nr, s);
  C.col.alloc(C.nnz > 0 ? C.nnz : 1);
  C.val.alloc(C.nnz > 0 ? C.nnz : 1);
  if (C.nnz == 0) return;
  fill<int>(flags.p, 0, 8, s);
  hipLaunchKernelGGL(k_bin_rows, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, C.ptr.p, 256, 2048, small.p, flags.p, big.p,
                     flags.p + 1, huge.p, flags.p + 2, flags.p + 3);
  NF_HIP(hipMemcpyAsync(h_flags, flags.p, sizeof(h_flags), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  if (h_flags[0] > 0)
    hipLaunchKernelGGL((k_spgemm_fill<512, 1>), dim3(h_flags[0]), dim3(64), 0, s, small.p, h_flags[0], A.ptr.p, A.col.p,
                       A.val.p, B.ptr.p, B.col.p, B.val.p, C.ptr.p, C.col.p, C.val.p);
  if (h_flags[1] > 0)
    hipLaunchKernelGGL((k_spgemm_fill<4096, 1>), dim3(h_flags[1]), dim3(64), 0, s, big.p, h_flags[1], A.ptr.p, A.col.p,
                       A.val.p, B.ptr.p, B.col.p, B.val.p, C.ptr.p, C.col.p, C.val.p);
  if (h_flags[2] > 0) {
    const int nh = h_flags[2];
    int ts = 1;
    while (ts < h_flags[3]) ts <<= 1;
    const int slots = spa_slots(B.nc, nh, ts);
    DBuf<int> f((size_t)slots * B.nc), ks((size_t)slots * ts);
    DBuf<double> acc((size_t)slots * B.nc);
    fill<int>(f.p, 0, (int64_t)slots * B.nc, s);
    fill<double>(acc.p, 0.0, (int64_t)slots * B.nc, s);
    for (int r0 = 0; r0 < nh; r0 += slots)
      hipLaunchKernelGGL(k_spa_fill, dim3(std::min(slots, nh - r0)), dim3(256), 0, s, huge.p + r0, A.ptr.p, A.col.p, A.val.p,
                         B.ptr.p, B.col.p, B.val.p, C.ptr.p, C.col.p, C.val.p, B.nc, f.p, acc.p, ks.p, ts);
  }
  NF_HIP(hipGetLastError());
  NF_HIP(hipStreamSynchronize(s));
}

// ================================================================= transpose
__global__ void k_col_count(int64_t nnz, const int* __restrict__ col, int* cnt) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[col[p]], 1);
}
__global__ void k_transpose_place(int nr, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
                                  const int* __restrict__ tptr, int* cursor, int* tcol, double* tval) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    const int c = col[p];
    const int q = tptr[c] + atomicAdd(&cursor[c], 1);
    tcol[q] = r;
    tval[q] = val[p];
  }
}
// sort each row of (col, val) pairs by column: one wavefront per row,
// bitonic sort in LDS (rows up to 4096 entries); longer rows are listed in
// longrows (count in longinfo[0], largest length in longinfo[1]) for
// k_sort_long_rows
__global__ __launch_bounds__(64) void k_sort_rows(int nr, const int* __restrict__ ptr, int* col, double* val, int* longrows,
                                                  int* longinfo) {
  __shared__ int ks[4096];
  __shared__ double vs[4096];
  const int row = blockIdx.x, lane = threadIdx.x;
  const int p0 = ptr[row], len = ptr[row + 1] - p0;
  if (len <= 1) return;
  if (len > 4096) {
    if (lane == 0) {
      longrows[atomicAdd(&longinfo[0], 1)] = row;
      atomicMax(&longinfo[1], len);
    }
    return;
  }
  int ts = 1;
  while (ts < len) ts <<= 1;
  for (int i = lane; i < ts; i += 64) {
    ks[i] = i < len ? col[p0 + i] : EMPTY_KEY;
    vs[i] = i < len ? val[p0 + i] : 0.0;
  }
  __syncthreads();
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < ts; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = ks[i], y = ks[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) {
            ks[i] = y;
            ks[ixj] = x;
            const double t = vs[i];
            vs[i] = vs[ixj];
            vs[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  for (int i = lane; i < len; i += 64) {
    col[p0 + i] = ks[i];
    val[p0 + i] = vs[i];
  }
}
// the same bitonic sort for rows longer than 4096 entries: one workgroup per
// listed row, in a power-of-two scratch of ts pairs per row
__global__ __launch_bounds__(1024) void k_sort_long_rows(const int* __restrict__ rows, const int* __restrict__ ptr, int* col,
                                                         double* val, int* kscr, double* vscr, int ts) {
  const int row = rows[blockIdx.x], t = threadIdx.x;
  const int p0 = ptr[row], len = ptr[row + 1] - p0;
  int* ks = kscr + (int64_t)blockIdx.x * ts;
  double* vs = vscr + (int64_t)blockIdx.x * ts;
  for (int i = t; i < ts; i += 1024) {
    ks[i] = i < len ? col[p0 + i] : EMPTY_KEY;
    vs[i] = i < len ? val[p0 + i] : 0.0;
  }
  __syncthreads();
  for (int kk = 2; kk <= ts; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = t; i < ts; i += 1024) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = ks[i], y = ks[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) {
            ks[i] = y;
            ks[ixj] = x;
            const double v = vs[i];
            vs[i] = vs[ixj];
            vs[ixj] = v;
          }
        }
      }
      __syncthreads();
    }
  for (int i = t; i < len; i += 1024) {
    col[p0 + i] = ks[i];
    val[p0 + i] = vs[i];
  }
}
void transpose(const DCsr& A, DCsr& T, hipStream_t s) {
  T.nr = A.nc;
  T.nc = A.nr;
  DBuf<int> cnt(A.nc + 1), cursor(A.nc + 1), longrows(A.nc > 0 ? A.nc : 1), longinfo(2);
  fill<int>(cnt.p, 0, A.nc + 1, s);
  fill<int>(cursor.p, 0, A.nc + 1, s);
  fill<int>(longinfo.p, 0, 2, s);
  if (A.nnz > 0) hipLaunchKernelGGL(k_col_count, dim3(cdiv(A.nnz, 256)), dim3(256), 0, s, A.nnz, A.col.p, cnt.p);
  T.ptr.alloc(A.nc + 1);
  T.nnz = exclusive_scan(cnt.p, T.ptr.p, A.nc, s);
  T.col.alloc(T.nnz > 0 ? T.nnz : 1);
  T.val.alloc(T.nnz > 0 ? T.nnz : 1);
  if (A.nr > 0)
    hipLaunchKernelGGL(k_transpose_place, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, A.val.p, T.ptr.p,
                       cursor.p, T.col.p, T.val.p);
  if (T.nr > 0)
    hipLaunchKernelGGL(k_sort_rows, dim3(T.nr), dim3(64), 0, s, T.nr, T.ptr.p, T.col.p, T.val.p, longrows.p, longinfo.p);
  int info[2] = {0, 0};
  NF_HIP(hipMemcpyAsync(info, longinfo.p, sizeof(info), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  if (info[0] > 0) {
    int ts = 1;
    while (ts < info[1]) ts <<= 1;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(info[0], ((int64_t)1 << 28) / ((int64_t)ts * 12)));
    DBuf<int> kscr((size_t)chunk * ts);
    DBuf<double> vscr((size_t)chunk * ts);
    for (int c0 = 0; c0 < info[0]; c0 += chunk)
      hipLaunchKernelGGL(k_sort_long_rows, dim3(std::min(chunk, info[0] - c0)), dim3(1024), 0, s, longrows.p + c0, T.ptr.p,
                         T.col.p, T.val.p, kscr.p, vscr.p, ts);
    NF_HIP(hipGetLastError());
    NF_HIP(hipStreamSynchronize(s));
  }
}

// ================================================================ sparse add
// G lanes per row: a row present in only one operand is copied (scaled) by
// the lanes together; a row present in both is merged by the group's first
// lane (both cases give every entry the expression of the serial merge)
template <bool FILL, int G>
__global__ void k_csr_add(int nr, double alpha, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
                          double beta, const int* __restrict__ bp, const int* __restrict__ bc, const double* __restrict__ bv,
                          int* cnt_or_ptr, int* cc, double* cv) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = (int)(gid / G), lane = (int)(gid % G);
  if (r >= nr) return;
  int p = ap ? ap[r] : 0, pe = ap ? ap[r + 1] : 0, q = bp ? bp[r] : 0, qe = bp ? bp[r + 1] : 0;
  const int o = FILL ? cnt_or_ptr[r] : 0;
  if (q == qe || p == pe) {
    const int n = (pe - p) + (qe - q);
    if (!FILL) {
      if (lane == 0) cnt_or_ptr[r] = n;
      return;
    }
    for (int t = lane; t < n; t += G) {
      if (p < pe) {
        cc[o + t] = ac[p + t];
        cv[o + t] = alpha * av[p + t];
      } else {
        cc[o + t] = bc[q + t];
        cv[o + t] = beta * bv[q + t];
      }
    }
    return;
  }
  if (lane != 0) return;
  int n = 0;
  while (p < pe || q < qe) {
    const int ca = p < pe ? ac[p] : INT_MAX, cb = q < qe ? bc[q] : INT_MAX;
    int c;
    double v;
    if (ca == cb) { c = ca; v = alpha * av[p] + beta * bv[q]; ++p; ++q; }
    else if (ca < cb) { c = ca; v = alpha * av[p]; ++p; }
    else { c = cb; v = beta * bv[q]; ++q; }
    if (FILL) { cc[o + n] = c; cv[o + n] = v; }
    ++n;
  }
  if (!FILL) cnt_or_ptr[r] = n;
}
void csr_add(double alpha, const DCsr& A, double beta, const DCsr& B, DCsr& C, hipStream_t s) {
  const bool ha = A.nnz > 0, hb = B.nnz > 0;
  const int nr = ha ? A.nr : B.nr;
  C.nr = nr;
  C.nc = ha ? A.nc : B.nc;
  DBuf<int> cnt(nr + 1);
  C.ptr.alloc(nr + 1);
  constexpr int G = 8;
  const int g = cdiv((int64_t)nr * G, 256);
  if (nr > 0)
    hipLaunchKernelGGL((k_csr_add<false, G>), dim3(g), dim3(256), 0, s, nr, alpha, ha ? A.ptr.p : nullptr, A.col.p, A.val.p,
                       beta, hb ? B.ptr.p : nullptr, B.col.p, B.val.p, cnt.p, nullptr, nullptr);
  C.nnz = exclusive_scan(cnt.p, C.ptr.p, nr, s);
  C.col.alloc(C.nnz > 0 ? C.nnz : 1);
  C.val.alloc(C.nnz > 0 ? C.nnz : 1);
  if (nr > 0)
    hipLaunchKernelGGL((k_csr_add<true, G>), dim3(g), dim3(256), 0, s, nr, alpha, ha ? A.ptr.p : nullptr, A.col.p, A.val.p,
                       beta, hb ? B.ptr.p : nullptr, B.col.p, B.val.p, C.ptr.p, C.col.p, C.val.p);
  NF_HIP(hipStreamSynchronize(s));
}
void csr_copy(const DCsr& A, DCsr& C, hipStream_t s) {
  C.nr = A.nr;
  C.nc = A.nc;
  C.nnz = A.nnz;
  C.ptr.alloc(A.nr + 1);
  C.col.alloc(A.nnz > 0 ? A.nnz : 1);
  C.val.alloc(A.nnz > 0 ? A.nnz : 1);
  NF_HIP(hipMemcpyAsync(C.ptr.p, A.ptr.p, sizeof(int) * (A.nr + 1), hipMemcpyDeviceToDevice, s));
  if (A.nnz > 0) {
    NF_HIP(hipMemcpyAsync(C.col.p, A.col.p, sizeof(int) * A.nnz, hipMemcpyDeviceToDevice, s));
    NF_HIP(hipMemcpyAsync(C.val.p, A.val.p, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s));
  }
}
__global__ void k_scale_rows(int nr, const int* __restrict__ ptr, double* val, const double* __restrict__ srow) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  const double sr = srow[r];
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) val[p] *= sr;
}
void scale_rows(DCsr& A, const double* s_rows, hipStream_t s) {
  if (A.nr > 0) hipLaunchKernelGGL(k_scale_rows, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.val.p, s_rows);
}
__global__ void k_set_diag_one(const int* rows, int n, const int* __restrict__ ptr, const int* __restrict__ col, double* val) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int r = rows[t];
  for (int p = ptr[r]; p < ptr[r + 1]; ++p)
    if (col[p] == r) val[p] = 1.0;
}
void set_diag_one(DCsr& A, const int* rows, int nrows, hipStream_t s) {
  if (nrows > 0) hipLaunchKernelGGL(k_set_diag_one, dim3(cdiv(nrows, 256)), dim3(256), 0, s, rows, nrows, A.ptr.p, A.col.p, A.val.p);
}
__global__ void k_identity(int n, int* ptr, int* col, double* val) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i > n) return;
  ptr[i] = i;
  if (i < n) { col[i] = i; val[i] = 1.0; }
}
void identity(int n, DCsr& I, hipStream_t s) {
  I.nr = I.nc = n;
  I.nnz = n;
  I.ptr.alloc(n + 1);
  I.col.alloc(n > 0 ? n : 1);
  I.val.alloc(n > 0 ? n : 1);
  hipLaunchKernelGGL(k_identity, dim3(cdiv(n + 1, 256)), dim3(256), 0, s, n, I.ptr.p, I.col.p, I.val.p);
}
void make_fp32(DCsr& A, hipStream_t s) {
  A.val32.alloc(A.nnz > 0 ? A.nnz : 1);
  cast_copy<double, float>(A.val.p, A.val32.p, A.nnz, s);
}

// ===================================================================== dense
__global__ void k_csr_to_dense(int nr, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
                               double* M, int64_t ld, int r0, int c0) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) M[(int64_t)(r0 + r) * ld + c0 + col[p]] += val[p];
}
void csr_to_dense(const DCsr& A, double* M, int64_t ld, int r0, int c0, hipStream_t s) {
  if (A.nr > 0 && A.nnz > 0)
    hipLaunchKernelGGL(k_csr_to_dense, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, A.val.p, M, ld, r0, c0);
}

// In-place Gauss-Jordan inverse of a row-major n x n matrix with partial
// pivoting (largest magnitude, lowest row on ties), blocked by column panels
// of GJ_NB.  Per panel K = [k0, k0 + kb):
//  1. the panel's columns are packed into a compact n x GJ_NB buffer and the
//     kb pivot steps run on it, one launch per step over all rows (the step
//     reads one buffer and writes the other, so rows never race); a step
//     swaps rows k and p in the panel, scales the pivot row and eliminates
//     column k from every other row, leaving the panel holding columns K of
//     the elimination matrix T; each workgroup also offers its best
//     candidate for the next pivot;
//  2. the pivots' row swaps are applied to the other columns, Y = rows K of
//     those columns is saved and zeroed, and every column outside K gets
//     += T[:, K] Y (a rank-kb update), the deferred eliminations.
// Afterwards the matrix holds (P M)^-1 for the row permutation P of the
// pivots; permuting its columns (the swaps in reverse order) gives M^-1.
constexpr int GJ_NB = 32;
constexpr int GJ_RPW = 8;          // panel rows per 256-thread workgroup
constexpr int DENSE_MAX = 12000;

__device__ __forceinline__ void gj_better(double& bv, int& bi, double ov, int oi) {
  if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
}
// workgroup-wide best (value, index) of 256 threads; result in every thread
__device__ __forceinline__ void gj_block_best(double& bv, int& bi, double* sv, int* si) {
  for (int off = 32; off > 0; off >>= 1) gj_better(bv, bi, __shfl_xor(bv, off), __shfl_xor(bi, off));
  const int t = threadIdx.x;
  __syncthreads();
  if ((t & 63) == 0) { sv[t >> 6] = bv; si[t >> 6] = bi; }
  __syncthreads();
  bv = sv[0];
  bi = si[0];
  for (int w = 1; w < 4; ++w) gj_better(bv, bi, sv[w], si[w]);
}

// pack columns K into PB and offer the candidates of column k0 (rows >= k0)
__global__ __launch_bounds__(256) void k_gj_pack(const double* __restrict__ M, double* __restrict__ PB, int n, int k0, int kb,
                                                 double* __restrict__ cv, int* __restrict__ ci) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const int t = threadIdx.x, lane = t & 31;
  const int i = blockIdx.x * GJ_RPW + (t >> 5);
  double bv = -1.0;
  int bi = n;
  if (i < n) {
    const double v = lane < kb ? M[(int64_t)i * n + k0 + lane] : 0.0;
    PB[(int64_t)i * GJ_NB + lane] = v;
    if (lane == 0 && i >= k0) { bv = fabs(v); bi = i; }
  }
  gj_block_best(bv, bi, sv, si);
  if (t == 0) { cv[blockIdx.x] = bv; ci[blockIdx.x] = bi; }
}

// one pivot step k on the packed panel: PBin -> PBout
__global__ __launch_bounds__(256) void k_gj_step(const double* __restrict__ PBin, double* __restrict__ PBout, int n, int k0,
                                                 int kb, int k, int nwg, const double* __restrict__ cv_in,
                                                 const int* __restrict__ ci_in, double* __restrict__ cv_out,
                                                 int* __restrict__ ci_out, int* __restrict__ piv, int* __restrict__ singular) {
  __shared__ double sv[4];
  __shared__ int si[4];
  if (*singular) return;
  const int t = threadIdx.x, lane = t & 31;
  const int jj = k - k0;
  const int i = blockIdx.x * GJ_RPW + (t >> 5);
  // the row's own values and those of row k (which row p takes) do not
  // depend on the pivot: loaded before its reduction
  const int ii = i < n ? i : k;
  const double fi = PBin[(int64_t)ii * GJ_NB + jj], vi = PBin[(int64_t)ii * GJ_NB + lane];
  const double fk = PBin[(int64_t)k * GJ_NB + jj], vk = PBin[(int64_t)k * GJ_NB + lane];
  double bv = -1.0;
  int bi = n;
  for (int w = t; w < nwg; w += 256) gj_better(bv, bi, cv_in[w], ci_in[w]);
  gj_block_best(bv, bi, sv, si);
  const int p = bi;
  if (!(bv > 0.0)) {                   // zero (or NaN) column below the diagonal
    if (blockIdx.x == 0 && t == 0) *singular = 1;
    return;
  }
  if (blockIdx.x == 0 && t == 0) piv[k] = p;
  const double a = PBin[(int64_t)p * GJ_NB + jj];
  const double pr = PBin[(int64_t)p * GJ_NB + lane];
  const double scaled = lane == jj ? 1.0 / a : pr / a;
  double cb = -1.0;
  int cbi = n;
  if (i < n) {
    double v;
    if (i == k) {
      v = scaled;
    } else {
      const double f = i == p ? fk : fi;
      v = lane == jj ? -f / a : (i == p ? vk : vi) - f * scaled;
    }
    if (lane < kb) PBout[(int64_t)i * GJ_NB + lane] = v;
    if (lane == jj + 1 && i > k) { cb = fabs(v); cbi = i; }
  }
  gj_block_best(cb, cbi, sv, si);
  if (t == 0) { cv_out[blockIdx.x] = cb; ci_out[blockIdx.x] = cbi; }
}

__global__ void k_gj_unpack(double* __restrict__ M, const double* __restrict__ PB, int n, int k0, int kb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * GJ_NB) return;
  const int i = (int)(e / GJ_NB), lane = (int)(e % GJ_NB);
  if (lane < kb) M[(int64_t)i * n + k0 + lane] = PB[e];
}

// the panel's row swaps on every column outside the panel (one thread per column)
__global__ void k_gj_swaprows(double* __restrict__ M, int n, int k0, int kb, const int* __restrict__ piv) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + kb)) return;
  for (int k = k0; k < k0 + kb; ++k) {
    const int p = piv[k];
    if (p != k) {
      const double a = M[(int64_t)k * n + j];
      M[(int64_t)k * n + j] = M[(int64_t)p * n + j];
      M[(int64_t)p * n + j] = a;
    }
  }
}

// Y (GJ_NB x n) = rows K of the columns outside K, which are then zeroed.
__global__ void k_gj_save(double* __restrict__ M, double* __restrict__ Y, int n, int k0, int kb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kb * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  if (c >= k0 && c < k0 + kb) {
    Y[e] = 0.0;
    return;
  }
  const int64_t m = (int64_t)(k0 + r) * n + c;
  Y[e] = M[m];
  M[m] = 0.0;
}

// M[:, j] += M[:, K] Y[:, j] for every column j outside K.  64 x 64 tiles,
// 256 threads, 4 x 4 outputs per thread; a thread's 16 outputs are loaded
// first, so that their latency overlaps the staging and the products.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ M, const double* __restrict__ Y, int n, int k0, int kb) {
  __shared__ double Ts[64][GJ_NB + 1];
  __shared__ double Ys[GJ_NB][64 + 1];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int t = threadIdx.x;
  const int tr = (t / 16) * 4, tc = (t % 16) * 4;
  double cv[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + tr + i, c = c0 + tc + j;
      cv[i][j] = (r < n && c < n) ? M[(int64_t)r * n + c] : 0.0;
    }
  for (int e = t; e < 64 * GJ_NB; e += 256) {
    const int r = e / GJ_NB, q = e % GJ_NB;
    Ts[r][q] = (r0 + r < n && q < kb) ? M[(int64_t)(r0 + r) * n + k0 + q] : 0.0;
  }
  for (int e = t; e < GJ_NB * 64; e += 256) {
    const int q = e / 64, c = e % 64;
    Ys[q][c] = (q < kb && c0 + c < n) ? Y[(int64_t)q * n + c0 + c] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int q = 0; q < kb; ++q) {
    double a[4], b[4];
    for (int i = 0; i < 4; ++i) a[i] = Ts[tr + i][q];
    for (int j = 0; j < 4; ++j) b[j] = Ys[q][tc + j];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + tr + i;
    if (r >= n) continue;
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + j;
      if (c >= n || (c >= k0 && c < k0 + kb)) continue;
      M[(int64_t)r * n + c] = cv[i][j] + acc[i][j];
    }
  }
}

// out[i][j] = W[i][src[j]]
__global__ void k_gj_gather_cols(const double* __restrict__ W, double* __restrict__ out, int n, const int* __restrict__ src) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  out[e] = W[(int64_t)i * n + src[j]];
}

__global__ void k_iota(int* v, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---- symmetric definite matrices: the same elimination without row
// exchanges.  A symmetric matrix whose elimination pivots all have one sign
// is definite, and Gauss-Jordan without pivoting is then stable; a panel
// becomes one kb x kb inverse (one workgroup, LDS) and one pass over the
// rows instead of kb pivot steps over all rows.

// max |M_ij - M_ji| (out[0]) and max |M_ij| (out[1]) as the bit patterns of
// nonnegative doubles, which order like the values; 32 x 32 tile pairs
__global__ __launch_bounds__(256) void k_sym_check(const double* __restrict__ M, int n, unsigned long long* out) {
  __shared__ double a[32][33], b[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    a[r][tx] = (bi + r < n && bj + tx < n) ? M[(int64_t)(bi + r) * n + bj + tx] : 0.0;
    b[r][tx] = (bj + r < n && bi + tx < n) ? M[(int64_t)(bj + r) * n + bi + tx] : 0.0;
  }
  __syncthreads();
  double asym = 0.0, mag = 0.0;
  for (int r = ty; r < 32; r += 8) {      // partner of M[bi + r][bj + tx] is M[bj + tx][bi + r]
    asym = fmax(asym, fabs(a[r][tx] - b[tx][r]));
    mag = fmax(mag, fabs(a[r][tx]));
  }
  for (int off = 32; off > 0; off >>= 1) {
    asym = fmax(asym, __shfl_xor(asym, off));
    mag = fmax(mag, __shfl_xor(mag, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(asym));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(mag));
  }
}

// Dinv = inverse of the diagonal block M[K, K] by Gauss-Jordan in LDS (one
// thread per entry); a pivot p with sign * p <= tiny flags the matrix as
// not definite
__global__ __launch_bounds__(1024) void k_gjnp_diag(const double* __restrict__ M, int n, int k0, int kb, double sign,
                                                    double tiny, double* __restrict__ Dinv, int* fail) {
  __shared__ double D[GJ_NB][GJ_NB + 1];
  const int r = threadIdx.x / GJ_NB, c = threadIdx.x % GJ_NB;
  D[r][c] = (r < kb && c < kb) ? M[(int64_t)(k0 + r) * n + k0 + c] : 0.0;
  __syncthreads();
  for (int q = 0; q < kb; ++q) {
    const double a = D[q][q];
    if (threadIdx.x == 0 && !(sign * a > tiny)) *fail = 1;
    const double sc = c == q ? 1.0 / a : D[q][c] / a;
    double v;
    if (r == q) v = sc;
    else {
      const double f = D[r][q];
      v = c == q ? -f / a : D[r][c] - f * sc;
    }
    __syncthreads();
    D[r][c] = v;
    __syncthreads();
  }
  if (r < kb && c < kb) Dinv[r * GJ_NB + c] = D[r][c];
}

// columns K of the elimination matrix, in place: rows in K take Dinv, every
// other row i takes -M[i, K] Dinv (32 lanes per row, ascending inner index)
__global__ __launch_bounds__(256) void k_gjnp_panel(double* __restrict__ M, int n, int k0, int kb,
                                                    const double* __restrict__ Dinv) {
  __shared__ double Ds[GJ_NB * GJ_NB];
  for (int e = threadIdx.x; e < GJ_NB * GJ_NB; e += 256) Ds[e] = (e / GJ_NB < kb && e % GJ_NB < kb) ? Dinv[e] : 0.0;
  __syncthreads();
  const int i = blockIdx.x * GJ_RPW + (threadIdx.x >> 5), c = threadIdx.x & 31;
  const bool row = i < n;
  const double m = row && c < kb ? M[(int64_t)(row ? i : 0) * n + k0 + c] : 0.0;
  double v = 0.0;
  for (int q = 0; q < kb; ++q) v = fma(__shfl(m, q, 32), Ds[q * GJ_NB + c], v);
  if (!row || c >= kb) return;
  M[(int64_t)i * n + k0 + c] = (i >= k0 && i < k0 + kb) ? Ds[(i - k0) * GJ_NB + c] : -v;
}

// Gauss-Jordan without row exchanges; false if a pivot breaks the sign test
// (M is then partly eliminated: the caller restores it)
static bool dense_inverse_definite(double* M, int n, double sign, double tiny, hipStream_t s) {
  const int nwg = cdiv(n, GJ_RPW);
  DBuf<double> Y((size_t)GJ_NB * n), Dinv(GJ_NB * GJ_NB);
  DBuf<int> fail(1);
  fill<int>(fail.p, 0, 1, s);
  const dim3 tiles(cdiv(n, 64), cdiv(n, 64));
  for (int k0 = 0; k0 < n; k0 += GJ_NB) {
    const int kb = std::min(GJ_NB, n - k0);
    hipLaunchKernelGGL(k_gjnp_diag, dim3(1), dim3(GJ_NB * GJ_NB), 0, s, M, n, k0, kb, sign, tiny, Dinv.p, fail.p);
    hipLaunchKernelGGL(k_gjnp_panel, dim3(nwg), dim3(256), 0, s, M, n, k0, kb, Dinv.p);
    hipLaunchKernelGGL(k_gj_save, dim3(cdiv((int64_t)kb * n, 256)), dim3(256), 0, s, M, Y.p, n, k0, kb);
    hipLaunchKernelGGL(k_gj_update, tiles, dim3(256), 0, s, M, Y.p, n, k0, kb);
  }
  NF_HIP(hipGetLastError());
  int h = 0;
  NF_HIP(hipMemcpyAsync(&h, fail.p, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  return h == 0;
}

int dense_inverse(double* M, int n, hipStream_t s) {
  if (n == 0) return 0;
  NF_CHECK(n <= DENSE_MAX, NFIELD_ENOMEM, "dense solve larger than " + std::to_string(DENSE_MAX) + " unknowns");
  {
    DBuf<unsigned long long> chk(2);
    fill<unsigned long long>(chk.p, 0ull, 2, s);
    hipLaunchKernelGGL(k_sym_check, dim3(cdiv(n, 32), cdiv(n, 32)), dim3(256), 0, s, M, n, chk.p);
    unsigned long long h[2];
    double m00 = 0.0;
    NF_HIP(hipMemcpyAsync(h, chk.p, sizeof(h), hipMemcpyDeviceToHost, s));
    NF_HIP(hipMemcpyAsync(&m00, M, sizeof(double), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    double asym, mag;
    std::memcpy(&asym, &h[0], sizeof(double));
    std::memcpy(&mag, &h[1], sizeof(double));
    if (mag > 0.0 && asym <= 1e-12 * mag && m00 != 0.0) {
      DBuf<double> keep((size_t)n * n);
      NF_HIP(hipMemcpyAsync(keep.p, M, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
      if (dense_inverse_definite(M, n, m00 > 0.0 ? 1.0 : -1.0, 1e-14 * mag, s)) return 0;
      NF_HIP(hipMemcpyAsync(M, keep.p, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
    }
  }
  const int nwg = cdiv(n, GJ_RPW);
  DBuf<double> Y((size_t)GJ_NB * n), PB0((size_t)GJ_NB * n), PB1((size_t)GJ_NB * n), cv(2 * (size_t)nwg);
  DBuf<int> piv(n), sing(1), ci(2 * (size_t)nwg);
  fill<int>(sing.p, 0, 1, s);
  hipLaunchKernelGGL(k_iota, dim3(cdiv(n, 256)), dim3(256), 0, s, piv.p, n);
  const dim3 tiles(cdiv(n, 64), cdiv(n, 64));
  for (int k0 = 0; k0 < n; k0 += GJ_NB) {
    const int kb = std::min(GJ_NB, n - k0);
    hipLaunchKernelGGL(k_gj_pack, dim3(nwg), dim3(256), 0, s, M, PB0.p, n, k0, kb, cv.p, ci.p);
    for (int k = k0; k < k0 + kb; ++k) {
      const int c = (k - k0) & 1;        // step parity: which buffers are read
      double* in = c ? PB1.p : PB0.p;
      double* out = c ? PB0.p : PB1.p;
      hipLaunchKernelGGL(k_gj_step, dim3(nwg), dim3(256), 0, s, in, out, n, k0, kb, k, nwg, cv.p + (size_t)c * nwg,
                         ci.p + (size_t)c * nwg, cv.p + (size_t)(1 - c) * nwg, ci.p + (size_t)(1 - c) * nwg, piv.p, sing.p);
    }
    const double* fin = (kb & 1) ? PB1.p : PB0.p;
    hipLaunchKernelGGL(k_gj_unpack, dim3(cdiv((int64_t)n * GJ_NB, 256)), dim3(256), 0, s, M, fin, n, k0, kb);
    hipLaunchKernelGGL(k_gj_swaprows, dim3(cdiv(n, 256)), dim3(256), 0, s, M, n, k0, kb, piv.p);
    hipLaunchKernelGGL(k_gj_save, dim3(cdiv((int64_t)kb * n, 256)), dim3(256), 0, s, M, Y.p, n, k0, kb);
    hipLaunchKernelGGL(k_gj_update, tiles, dim3(256), 0, s, M, Y.p, n, k0, kb);
  }
  NF_HIP(hipGetLastError());
  int h = 0;
  std::vector<int> hp(n);
  NF_HIP(hipMemcpyAsync(&h, sing.p, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipMemcpyAsync(hp.data(), piv.p, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  if (h) return -1;
  // column j of M^-1 is column src[j] of (P M)^-1: the swaps applied to the
  // columns in reverse order
  std::vector<int> src(n);
  for (int j = 0; j < n; ++j) src[j] = j;
  for (int k = n - 1; k >= 0; --k) std::swap(src[k], src[hp[k]]);
  DBuf<int> dsrc(n);
  DBuf<double> W((size_t)n * n);
  NF_HIP(hipMemcpyAsync(dsrc.p, src.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  NF_HIP(hipMemcpyAsync(W.p, M, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_gj_gather_cols, dim3(cdiv((int64_t)n * n, 256)), dim3(256), 0, s, W.p, M, n, dsrc.p);
  NF_HIP(hipGetLastError());
  NF_HIP(hipStreamSynchronize(s));
  return 0;
}

// ===================================================================== SIMPLE
__global__ void k_row_accumulate(int nr, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
                                 int mode, int is_diag, double* acc) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  double s = 0.0;
  for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
    if (mode == 0) s += fabs(val[p]);
    else if (mode == 1) s += val[p];
    else if (is_diag && col[p] == r) s += val[p];
  }
  acc[r] += s;
}
void row_accumulate(const DCsr& A, int mode, int is_diag, double* acc, hipStream_t s) {
  if (A.nr > 0) hipLaunchKernelGGL(k_row_accumulate, dim3(cdiv(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr.p, A.col.p, A.val.p, mode, is_diag, acc);
}
__global__ void k_finish_simplec(double* acc, int64_t n, int mode, int* zero_flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = mode == 1 ? fabs(acc[i]) : acc[i];
  if (v == 0.0) atomicOr(zero_flag, 1);
  acc[i] = v != 0.0 ? 1.0 / v : 0.0;
}
void finish_simplec(double* acc, int64_t n, int mode, int* zero_flag, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_finish_simplec, dim3(cdiv(n, 256)), dim3(256), 0, s, acc, n, mode, zero_flag);
}

}  // namespace nf

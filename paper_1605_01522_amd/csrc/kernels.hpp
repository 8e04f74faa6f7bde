// Host launch wrappers of the gfx950 kernels.  Every wrapper enqueues on
// the given stream; wrappers that return a host value synchronise the stream.
#pragma once

#include "common.hpp"

namespace nf {

// ------------------------------------------------------------ vectors
template <class T> void fill(T* x, T v, int64_t n, hipStream_t s);
template <class S, class D> void cast_copy(const S* x, D* y, int64_t n, hipStream_t s);
void axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);          // y += a x
template <class T> void sub_scaled(const T* dinv, const T* u, T* x, int64_t n, hipStream_t s);  // x -= dinv .* u
template <class T> void add_into(const T* d, T* x, int64_t n, hipStream_t s);                   // x += d
// v = w / *nrm_dev (v = w if the norm is zero)
void scale_inv_dev(const double* w, double* v, const double* nrm_dev, int64_t n, hipStream_t s);
// first Chebyshev step from a zero guess: d = dinv .* b * inv_theta; x = d
template <class T> void cheb_first(const T* b, const T* dinv, T inv_theta, T* d, T* x, int64_t n, hipStream_t s);
// x = M b with a dense row-major FP64 matrix (explicit coarse inverse)
template <class T> void dense_gemv(const double* M, int n, const T* b, T* x, hipStream_t s);

// ------------------------------------------------------------ CSR SpMV
enum SpmvMode { SPMV_STORE = 0, SPMV_RESID = 1, SPMV_ADD = 2, SPMV_SUB = 3, SPMV_CHEB = 4, SPMV_DSCALE = 5 };
template <class T>
struct SpmvArgs {
  const T* x = nullptr;     // operand
  T* y = nullptr;           // output (STORE/RESID/ADD/SUB/DSCALE)
  const T* b = nullptr;     // RESID, CHEB
  const T* dinv = nullptr;  // CHEB, DSCALE
  T* d = nullptr;           // CHEB (in/out)
  T* xo = nullptr;          // CHEB output iterate (must differ from x)
  T c1 = 0, c2 = 0;         // CHEB: d = c1 d + c2 dinv (b - A x)
};
// lanes per row chosen from the mean row length
int spmv_group(int nr, int64_t nnz);

// Optional per-launch timing of the SpMV kernels with HIP events on the
// launch stream, keyed by (lanes per row, mode, FP32?), with the algorithmic
// bytes of every launch.
void prof_enable(int on);
int prof_read(int max, int* key, int64_t* count, double* ms, double* bytes);
// bracket any other launch: slot = prof_begin(s) (-1 if not recording), then
// prof_end(slot, s, key, bytes) after the launch
int prof_begin(hipStream_t s);
void prof_end(int slot, hipStream_t s, int key, double bytes, int count = 1);
bool prof_recording();
template <class T> void spmv(SpmvMode mode, const DCsr& A, const SpmvArgs<T>& a, hipStream_t s);

// ------------------------------------------------------------ reductions (FP64, deterministic)
constexpr int RED_BLOCKS = 480;
constexpr int RED_THREADS = 256;
// *out = x . y  (partial must hold RED_BLOCKS doubles)
void dot_dev(const double* x, const double* y, int64_t n, double* partial, double* out, hipStream_t s);
// GMRES block operations on V (column-major, leading dimension ldv)
void mdot_partial(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, double* partial, hipStream_t s);
void mreduce(const double* partial, int ncols, double* out, int accumulate, hipStream_t s);
void mupdate_dot(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, double* partial, hipStream_t s);
void mupdate_norm(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, double* partial, hipStream_t s);
void mcombine(const double* V, int64_t ldv, int ncols, const double* y, double* u, int64_t n, int accumulate, hipStream_t s);
// Arnoldi step j bookkeeping on device: reduce ||w||^2 partials into H(j+1,j),
// h1 + h2 into H(:,j), apply the stored rotations and a new one, update g,
// write |g_{j+1}| to res_out.  H is (m+1) x m column-major.
void givens_step(int j, int m, const double* h1, const double* h2, const double* nrm_partial,
                 double* H, double* cs, double* sn, double* g, double* hnorm_out, double* res_out, hipStream_t s);
// y = H(0:k,0:k)^-1 g (upper triangular, after rotations)
void backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t s);

// ------------------------------------------------------------ multicolour Gauss-Seidel
// greedy colouring of a node graph (Jones-Plassmann order, splitmix64 keys);
// returns the number of colours and fills color[node]
int color_nodes(int nnode, const int* gptr, const int* gadj, uint64_t seed, int* color, hipStream_t s);
// relax all nodes of one colour: x_r += omega dinv_r (b_r - A_r x) for the b
// dofs of each listed node, all from the values before the node's update
template <class T> void sgs_color(const DCsr& A, int b, const int* nodes, int nnodes, const T* dinv, T omega,
                                  const T* rhs, T* x, hipStream_t s);
int sgs_lanes(const DCsr& A, int b);   // lanes per row of the Gauss-Seidel kernel
// per colour: stored entries of its rows and distinct columns they touch
// (algorithmic bytes of one colour sweep)
void color_traffic(const DCsr& A, int b, const int* nodes, const std::vector<int>& off, std::vector<int64_t>& nnz,
                   std::vector<int64_t>& ncols, hipStream_t s);

// ------------------------------------------------------------ setup
int64_t exclusive_scan(const int* in, int* out, int64_t n, hipStream_t s);   // out[n] = total; returns total
void csr_diag(const DCsr& A, double* d, int* zero_flag, hipStream_t s);
void invert(const double* d, double* dinv, int64_t n, hipStream_t s);
void power_start(double* v, int64_t n, uint64_t seed, hipStream_t s);
void node_graph(const DCsr& A, int b, DBuf<int>& gptr, DBuf<int>& gadj, int* nnode, hipStream_t s);
// synchronous MIS-2 + aggregation; returns the number of aggregates
int mis2_aggregate(int nnode, const int* gptr, const int* gadj, uint64_t seed, int* agg, hipStream_t s);
// tentative prolongator + coarse nullspace; returns number of dead coarse dofs
int tentative(int nnode, int b, int k, const int* agg, int nagg, const double* B, DCsr& P,
              DBuf<double>& Bc, DBuf<int>& dead, hipStream_t s);
// smoothed prolongator in place on AP = A * P_tent: AP <- P_tent + s .* AP
void smooth_prolongator(DCsr& AP, const double* srow, const DCsr& Pt, int b, int k, const int* agg, hipStream_t s);
void spgemm(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s);
void transpose(const DCsr& A, DCsr& T, hipStream_t s);
void csr_add(double alpha, const DCsr& A, double beta, const DCsr& B, DCsr& C, hipStream_t s);
void csr_copy(const DCsr& A, DCsr& C, hipStream_t s);
void scale_rows(DCsr& A, const double* s_rows, hipStream_t s);
void set_diag_one(DCsr& A, const int* rows, int nrows, hipStream_t s);
void identity(int n, DCsr& I, hipStream_t s);
void make_fp32(DCsr& A, hipStream_t s);
// dense row-major block of a CSR (adds into M with row/col offsets, leading dim ld)
void csr_to_dense(const DCsr& A, double* M, int64_t ld, int r0, int c0, hipStream_t s);
// in-place dense inverse by Gauss-Jordan with partial pivoting; returns 0 or -1 (singular)
int dense_inverse(double* M, int n, hipStream_t s);
// SIMPLE diagonal accumulation: mode 0 sum|a|, 1 sum a, 2 diag only (when is_diag)
void row_accumulate(const DCsr& A, int mode, int is_diag, double* acc, hipStream_t s);
void finish_simplec(double* acc, int64_t n, int mode, int* zero_flag, hipStream_t s);

}  // namespace nf

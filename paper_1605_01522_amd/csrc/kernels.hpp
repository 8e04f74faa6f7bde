// Host launch wrappers of the gfx950 kernels.  Every wrapper enqueues on
// the given stream; wrappers that return a host value synchronise the stream.
#pragma once

#include "common.hpp"

namespace nf {

// Multi-column vectors: nrhs columns, column k at p + k * ld (ld >= length).
// Every apply-phase kernel processes all columns of a call; columns never
// mix, so a column's result does not depend on the other columns.
constexpr int NRMAX = 8;

// Algorithmic HBM bytes of the apply-phase launches made by this thread
// (every operand counted once per launch: matrix entries, indices, the
// vectors read and written), accumulated by the launch wrappers; a solve
// reads the counter before and after to fill nfield_stats.bytes.
void bytes_count(double b);
// set-up mode of the calling thread: SpMVs then ignore block copies
void setup_mode(bool on);
bool in_setup();
double bytes_counted();

// ------------------------------------------------------------ vectors
template <class T> void fill(T* x, T v, int64_t n, hipStream_t s);   // one column
template <class S, class D> void cast_copy(const S* x, D* y, int64_t n, hipStream_t s);
template <class T> void fillm(T* x, int64_t ldx, T v, int64_t n, int nrhs, hipStream_t s);
template <class S, class D> void castm(const S* x, int64_t ldx, D* y, int64_t ldy, int64_t n, int nrhs, hipStream_t s);
template <class T> void copym(const T* x, int64_t ldx, T* y, int64_t ldy, int64_t n, int nrhs, hipStream_t s);
// x += d, for the columns whose mask entry is nonzero (mask may be null)
template <class T> void add_intom(const T* d, int64_t ldd, T* x, int64_t ldx, int64_t n, int nrhs, const int* mask,
                                  hipStream_t s);
// x -= dinv .* u
template <class T> void sub_scaledm(const T* dinv, const T* u, int64_t ldu, T* x, int64_t ldx, int64_t n, int nrhs,
                                    hipStream_t s);
// first Chebyshev step from a zero guess: d = dinv .* b * inv_theta; x = d
template <class T> void cheb_firstm(const T* b, int64_t ldb, const T* dinv, T inv_theta, T* d, int64_t ldd, T* x,
                                    int64_t ldx, int64_t n, int nrhs, hipStream_t s);
// x = M b with a dense row-major FP64 matrix (explicit coarse inverse)
template <class T> void dense_gemvm(const double* M, int n, const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs,
                                    hipStream_t s);

// ------------------------------------------------------------ CSR SpMV
enum SpmvMode { SPMV_STORE = 0, SPMV_RESID = 1, SPMV_ADD = 2, SPMV_SUB = 3, SPMV_CHEB = 4, SPMV_DSCALE = 5 };
template <class T>
struct SpmvArgs {
  const T* x = nullptr;     // operand
  T* y = nullptr;           // output (STORE/RESID/ADD/SUB/DSCALE)
  const T* b = nullptr;     // RESID, CHEB
  const T* dinv = nullptr;  // CHEB, DSCALE (one column, shared)
  T* d = nullptr;           // CHEB (in/out)
  T* xo = nullptr;          // CHEB output iterate (must differ from x)
  T c1 = 0, c2 = 0;         // CHEB: d = c1 d + c2 dinv (b - A x)
  int64_t ldx = 0, ldy = 0, ldb = 0, ldd = 0, ldxo = 0;   // column strides
  int nrhs = 1;
};
// lanes per row chosen from the mean row length (Gauss-Seidel; SpMV)
int spmv_group(int nr, int64_t nnz);
int spmv_lanes(int nr, int64_t nnz);

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
void prof_quiet(bool q);   // this thread's launches untimed
template <class T> void spmv(SpmvMode mode, const DCsr& A, const SpmvArgs<T>& a, hipStream_t s);

// ------------------------------------------------------------ reductions (FP64, deterministic)
constexpr int RED_BLOCKS = 480;
constexpr int RED_THREADS = 256;
// out[k] = x_k . y_k for nrhs columns (partial: RED_BLOCKS * nrhs doubles)
// v = w / ||w|| (in place allowed), nrm[0] = ||w||: one partial-dot launch
// and one launch that reduces the partials and scales
void normalize(const double* w, double* v, int64_t n, double* partial, double* nrm, hipStream_t s);
void dotm(const double* x, int64_t ldx, const double* y, int64_t ldy, int64_t n, int nrhs, double* partial, double* out,
          hipStream_t s);
// GMRES block operations, batched over nrhs independent columns.  Column k's
// Krylov basis is V + k * vs (vectors j at + j * n); h / partial / H etc. use
// the per-column strides given.  mask (device, may be null): columns with a
// zero entry are skipped.
struct GmresLayout {
  int64_t n = 0;        // vector length
  int64_t vs = 0;       // per-column stride of V (and of Z for the flexible form)
  int64_t hs = 0;       // per-column stride of h1, h2 (m + 1)
  int64_t ps = 0;       // per-column stride of partial ((m + 1) * RED_BLOCKS)
  int m = 0;            // restart length
  int nrhs = 1;
};
// ncv (device, may be null): per-column counts of basis vectors, at most
// ncols (the grid's count); columns then proceed at their own Arnoldi steps
void mdot_partial(const GmresLayout& L, const double* V, int ncols, const double* w, int64_t ldw, double* partial,
                  const int* mask, hipStream_t s, const int* ncv = nullptr);
void mreduce(const GmresLayout& L, const double* partial, int ncols, double* out, int accumulate, const int* mask,
             hipStream_t s, const int* ncv = nullptr);
void mupdate_dot(const GmresLayout& L, const double* V, int ncols, const double* h, double* w, int64_t ldw,
                 double* partial, const int* mask, hipStream_t s, const int* ncv = nullptr);
void mupdate_norm(const GmresLayout& L, const double* V, int ncols, const double* h, double* w, int64_t ldw,
                  double* partial, const int* mask, hipStream_t s, const int* ncv = nullptr);
// u_k (+)= sum_{j < ncols_k} V_k[j] y_k[j]; ncols per column on the device, max_ncols on the host
void mcombine(const GmresLayout& L, const double* V, const int* ncols, int max_ncols, const double* y, double* u,
              int64_t ldu, int accumulate, const int* mask, hipStream_t s);
// Arnoldi step j bookkeeping per column: reduce ||w||^2 partials into
// H(j+1,j), h1 + h2 into H(:,j), apply the stored rotations and a new one,
// update g, write ||w|| and |g_{j+1}| to scal[2k], scal[2k+1].
// (jv, device, may be null: per-column step numbers in place of j)
void givens_step(const GmresLayout& L, int j, const double* h1, const double* h2, const double* nrm_partial, double* H,
                 double* cs, double* sn, double* g, double* scal, const int* mask, hipStream_t s,
                 const int* jv = nullptr);
// y_k = H_k(0:k,0:k)^-1 g_k with k = ncols[col]
void backsolve(const GmresLayout& L, const int* ncols, const double* H, const double* g, double* y, const int* mask,
               hipStream_t s);
// v_k = w_k / nrm[k * stride] (v_k = w_k if the norm is zero); vcol (device,
// may be null): column k's destination moved by vcol[k] * vstep elements
void scale_inv_devm(const double* w, int64_t ldw, double* v, int64_t ldv, const double* nrm, int stride, int64_t n,
                    int nrhs, const int* mask, hipStream_t s, const int* vcol = nullptr, int64_t vstep = 0);
// out column c = V + act[c] vs + jv[act[c]] n (jv may be null: + 0), and back
void slot_gather(const double* V, int64_t vs, int64_t n, const int* act, const int* jv, int nact, double* out,
                 hipStream_t s);
void slot_scatter(const double* in, int64_t n, const int* act, const int* jv, int nact, double* V, int64_t vs,
                  hipStream_t s);

// ------------------------------------------------------------ multicolour Gauss-Seidel
// greedy colouring of a node graph in node order (graphs of at most 32,768
// nodes: also in smallest-last order, keeping the one with fewer colours);
// returns the number of colours and fills color[node]
int color_nodes(int nnode, const int* gptr, const int* gadj, uint64_t seed, int* color, hipStream_t s);
// row bounds of the listed nodes' rows in list order: cptr[t (b+1) + q] =
// ptr[nodes[t] b + q] for q = 0..b (cptr holds nnodes (b+1) ints)
void sgs_node_ptrs(const DCsr& A, int b, const int* nodes, int nnodes, int* cptr, hipStream_t s);
// relax all nodes of one colour: x_r += omega dinv_r (b_r - A_r x) for the b
// dofs of each listed node, all from the values before the node's update
// (cptr: the listed nodes' row bounds as sgs_node_ptrs writes them)
template <class T> void sgs_color(const DCsr& A, int b, const int* nodes, const int* cptr, int nnodes, const T* dinv,
                                  T omega, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s);
int sgs_lanes(const DCsr& A, int b);   // lanes per row of the Gauss-Seidel kernel
// kernel layout of a sweep: SGS_SWEEP1 = every colour in one workgroup (small
// levels), SGS_NODE = one workgroup per node (long rows), SGS_COLOR = one
// lane group per node, a launch per colour
enum { SGS_COLOR = 0, SGS_SWEEP1 = 1, SGS_NODE = 2 };
// levels of at least this many nodes with a block copy relax from it (one
// right-hand side)
constexpr int SGS_BSR_MIN_NODES = 4096;
constexpr int SGS_BSR_LANES = 16;   // lanes per node of the block-copy colour kernel
constexpr int64_t SGS_SWEEP1_MAX_NNZ = 65536;
constexpr int64_t SGS_SWEEP1_MAX_ROW = 128;
constexpr int SGS_SWEEP1_MAX_NODES = 65536;
constexpr int SGS_SWEEP1_MIN_COLORS = 8;
constexpr int64_t SGS_NODE_MIN_ROW = 128;
int sgs_kind(const DCsr& A, int b, int nnodes_total, int ncolors);
// levels up to SGS_DENSE_MAX dofs with at least SGS_DENSE_MIN_COLORS colours
// apply their symmetric sweep as a dense affine map X = [S | Q]
constexpr int SGS_DENSE_MAX = 2048;
constexpr int SGS_DENSE_MIN_COLORS = 16;
void dense_sgs_build(const DCsr& A, int b, const int* nodes, const int* off_dev, const std::vector<int>& off,
                     const double* dinv, double omega, double* X, hipStream_t s);
template <class T> void dense_sweep_apply(const T* X, int n, const T* x, int64_t ldx, const T* rb, int64_t ldb, T* y,
                                          int64_t ldy, int nrhs, bool with_x, hipStream_t s);
// one sweep over all colours (forward: ascending colour order), nodes grouped
// by colour with colour c owning nodes[off[c], off[c+1]) (off also on the
// device as off_dev; cptr from sgs_node_ptrs over the whole list)
// The block copy of a level made of dense b x b node blocks (b = 2 or 3) for
// its Gauss-Seidel colour kernel (kept with A, built once per precision) and
// the block row bounds of each listed node (2 ints per node in list order);
// false, keeping nothing new, when some node block of A is not full
template <class T> bool sgs_bsr_setup(const DCsr& A, int b, const int* nodes, int nnodes, DBuf<int>& bcp,
                                      hipStream_t s);
// one sweep over all colours from A's block copy (one right-hand side)
template <class T> void sgs_sweep_bsr(const DCsr& A, const int* nodes, const int* bcp, const std::vector<int>& off,
                                      bool forward, const T* dinv, T omega, const T* rhs, T* x, hipStream_t s);
template <class T> void sgs_sweep(const DCsr& A, int b, const int* nodes, const int* cptr, const int* off_dev,
                                  const std::vector<int>& off, bool forward, const T* dinv, T omega, const T* rhs,
                                  int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s);
// DD(GS) sweep: one workgroup per subdomain; nodes listed by (subdomain,
// colour, node), subdomain q's colour c owning nodes[off[q (nc+1) + c],
// off[q (nc+1) + c + 1]) (off on the device).  dd_split stores every listed
// row's own part (couplings inside its subdomain, local dof columns; pos: a
// node's position in its subdomain's list) and other part (global columns),
// in list order; xo: the sweep's start values of x (NULL: zero); max_nodes:
// the largest subdomain (its values live in LDS).
constexpr size_t DD_LDS_MAX = 65536;
size_t dd_lds_bytes(int b, int max_nodes, int nrhs, size_t val_bytes);
template <class T> void dd_split(const DCsr& A, int b, int nlist, const int* nodes, const int* sub, const int* pos,
                                 DBuf<int>& optr, DBuf<int>& ocol, DBuf<T>& oval, DBuf<int>& xptr, DBuf<int>& xcol,
                                 DBuf<T>& xval, hipStream_t s);
template <class T> void dd_sweep(int b, int nsub, const int* nodes, const int* off_dev, int nc, bool forward,
                                 double avg_own, double avg_other, const int* optr, const int* ocol, const T* oval,
                                 const int* xptr, const int* xcol, const T* xval, const T* dinv, T omega, const T* rhs,
                                 int64_t ldr, const T* xo, int64_t ldxo, T* x, int64_t ldx, int nrhs, int max_nodes,
                                 hipStream_t s);
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
// Petrov-Galerkin smoothing of a tentative prolongator: om[j] (P.nc values)
// = <AP e_j, AQ e_j> / ||AQ e_j||^2 clipped at 0; P = P_tent - Q diag(om)
// on the pattern of Q = D^-1 A P_tent
void pg_omega(const DCsr& AP, const DCsr& AQ, double* om, hipStream_t s);
void pg_prolongator(const DCsr& Q, const double* om, const DCsr& Pt, int b, int k, const int* agg, DCsr& P,
                    hipStream_t s);
// node-blocked matrix: block pattern (pat.val: block indices for a converted
// or transposed matrix, unused otherwise), br x bc values per
// block (row-major, zero where nothing is stored) and a mask of the stored
// entries (bit r bc + c)
struct DBsr {
  DCsr pat;
  int br = 1, bc = 1;
  DBuf<double> val;
  DBuf<unsigned long long> mask;
};
void csr_to_bsr(const DCsr& A, int br, int bc, DBsr& B, hipStream_t s);
void bsr_to_csr(const DBsr& B, DCsr& A, hipStream_t s);
// R = P^T (P converted by csr_to_bsr)
void bsr_transpose(const DBsr& P, DBsr& R, hipStream_t s);
// C = A B block by block (A.bc == B.br); same pattern and bits as spgemm on
// the scalar matrices
void bspgemm(const DBsr& A, const DBsr& B, DBsr& C, hipStream_t s);
// C = A B for A with br x bk blocks and B with bk x bc blocks
void spgemm_blocked(const DCsr& A, int br, int bk, const DCsr& B, int bc, DCsr& C, hipStream_t s);
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

// Preconditioner tree (BGS, SIMPLE, monolithic AMG, dense LU), restarted
// right-preconditioned / flexible GMRES, and the C ABI of nfield.h.
//
// Every numerical step runs in the kernels of kernels.hip and amg.hip; the
// host parses the specification, sequences launches on the caller's stream
// and reads back one residual estimate per Arnoldi step.

#include <algorithm>
#include <cctype>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <mutex>
#include <exception>

#include "amg.hpp"

namespace nf {

thread_local DevPool* g_pool = nullptr;
// where this thread's builds leave the hierarchies and blocks they own
thread_local std::vector<std::unique_ptr<Hierarchy>>* g_hsink = nullptr;
thread_local std::vector<std::unique_ptr<BlockMat>>* g_osink = nullptr;
static thread_local std::string g_err;

// ================================================================ helpers
// Multi-column buffers: every temporary of a preconditioner holds the
// largest column count one call may pass (the max_rhs option, at most
// NRMAX), set for the thread that builds it.
thread_local int g_mbuf_cols = NRMAX;
template <class T>
struct MBuf {
  DBuf<T> buf;
  int64_t ld = 0;
  void alloc(int64_t n) {
    ld = n > 0 ? n : 1;
    buf.alloc((size_t)ld * g_mbuf_cols);
  }
  T* p() const { return buf.p; }
};

// r_i = b_i - sum_j A_ij x_j over fields [f0, f1) of A (vectors re-based at f0)
template <class T>
static void block_resid(const BlockMat& A, int f0, int f1, const T* b, int64_t ldb, const T* x, int64_t ldx, T* r,
                        int64_t ldr, int nrhs, hipStream_t s) {
  std::vector<int> o = A.offsets();
  for (int i = f0; i < f1; ++i) {
    bool first = true;
    for (int j = f0; j < f1; ++j) {
      const DCsr* B = A.at(i, j);
      if (!B) continue;
      SpmvArgs<T> a;
      a.x = x + (o[j] - o[f0]);
      a.ldx = ldx;
      a.y = r + (o[i] - o[f0]);
      a.ldy = ldr;
      a.b = b + (o[i] - o[f0]);
      a.ldb = ldb;
      a.nrhs = nrhs;
      spmv<T>(first ? SPMV_RESID : SPMV_SUB, *B, a, s);
      first = false;
    }
    if (first && A.size[i] > 0) copym<T>(b + (o[i] - o[f0]), ldb, r + (o[i] - o[f0]), ldr, A.size[i], nrhs, s);
  }
}

static void prepare_fp32(BlockMat& A, hipStream_t s) {
  for (auto& b : A.blk)
    if (b && !b->val32.p) make_fp32(*b, s);
}
// FP32 copy of block (i, j) for a solver of precision T that reads it
// (input blocks get one only when some FP32 solver uses them)
template <class T>
static void need_fp32(const BlockMat& A, int i, int j, hipStream_t s) {
  if (sizeof(T) != sizeof(float)) return;
  DCsr* b = const_cast<DCsr*>(A.at(i, j));
  if (b && !b->val32.p) make_fp32(*b, s);
}

// ================================================================ solvers
template <class T>
struct Solver {
  int n = 0;
  virtual ~Solver() {}
  // z = M^-1 r for nrhs <= NRMAX columns (column k at r + k ldr, z + k ldz)
  virtual void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) = 0;
};

template <class T>
struct FieldSmootherD {
  virtual ~FieldSmootherD() {}
  virtual void apply(const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) = 0;
  // the level smoother's phase for the next applications: pre-smoothing
  // (before the coarse correction) or post-smoothing
  virtual void set_phase(bool pre) { (void)pre; }
};

// Chebyshev smoother on D^-1 A over [lambda/ratio, boost*lambda]: three-term
// recurrence (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
// Algorithm 12.1).  Each step after the first is one fused kernel: residual,
// direction update and iterate update.
template <class T>
struct ChebD : FieldSmootherD<T> {
  const DCsr* A = nullptr;
  DBuf<T> dinv;
  MBuf<T> d, xt;
  double theta = 0, delta = 0, sigma = 0;
  int degree = 2, n = 0;
  void setup(const DCsr* A_, const double* dinv64, double lam, const Opts& o, hipStream_t s) {
    A = A_;
    n = A->nr;
    dinv.alloc(n);
    d.alloc(n);
    xt.alloc(n);
    if (sizeof(T) == sizeof(double)) NF_HIP(hipMemcpyAsync(dinv.p, dinv64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else cast_copy<double, float>(dinv64, (float*)dinv.p, n, s);
    const double hi = o.cheb_boost * lam, lo = lam / o.cheb_ratio;
    theta = 0.5 * (hi + lo);
    delta = 0.5 * (hi - lo);
    sigma = theta / delta;
    degree = o.cheb_degree;
  }
  void apply(const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) override {
    const T* src;
    int64_t lds;
    int k0;
    if (zero_guess) {
      const bool to_x = degree % 2 == 1;   // the last write must land in x
      T* dst = to_x ? x : xt.p();
      const int64_t ldd = to_x ? ldx : xt.ld;
      cheb_firstm<T>(b, ldb, dinv.p, (T)(1.0 / theta), d.p(), d.ld, dst, ldd, n, nrhs, s);
      src = dst;
      lds = ldd;
      k0 = 1;
    } else {
      src = x;
      lds = ldx;
      k0 = 0;
    }
    double rho = 1.0 / sigma;
    for (int k = k0; k < degree; ++k) {
      const bool to_xt = src == x;
      T* dst = to_xt ? xt.p() : x;
      const int64_t ldd = to_xt ? xt.ld : ldx;
      SpmvArgs<T> a;
      a.x = src;
      a.ldx = lds;
      a.b = b;
      a.ldb = ldb;
      a.dinv = dinv.p;
      a.d = d.p();
      a.ldd = d.ld;
      a.xo = dst;
      a.ldxo = ldd;
      a.nrhs = nrhs;
      if (k == 0) {
        a.c1 = 0;
        a.c2 = (T)(1.0 / theta);
      } else {
        const double rn = 1.0 / (2.0 * sigma - rho);
        a.c1 = (T)(rn * rho);
        a.c2 = (T)(2.0 * rn / delta);
        rho = rn;
      }
      spmv<T>(SPMV_CHEB, *A, a, s);
      src = dst;
      lds = ldd;
    }
    if (src != x) copym<T>(src, lds, x, ldx, n, nrhs, s);
  }
};

// Symmetric multicolour Gauss-Seidel with damping omega: colours forward,
// then backward; the nodes of one colour are relaxed by one kernel.
template <class T>
struct SgsD : FieldSmootherD<T> {
  const DCsr* A = nullptr;
  int b = 1, steps = 1, n = 0;
  T omega = 1;
  DBuf<T> dinv;
  DBuf<int> nodes;                 // nodes grouped by colour
  DBuf<int> cptr;                  // row bounds of the listed nodes' rows, b + 1 each
  std::vector<int> off;            // colour c owns nodes[off[c], off[c+1])
  DBuf<int> off_dev;
  int kind = SGS_COLOR;
  // a level made of dense 2 x 2 or 3 x 3 node blocks: the colour kernel for
  // one right-hand side reads A's block copy (bcp: each listed node's block
  // bounds)
  bool bsr = false;
  DBuf<int> bcp;
  // gp / ga / nn: the node graph of A when the caller already has it
  void setup(const DCsr* A_, int b_, const double* dinv64, double om, int st, uint64_t seed, hipStream_t s,
             const DBuf<int>* gp = nullptr, const DBuf<int>* ga = nullptr, int nn_given = 0) {
    A = A_;
    b = b_;
    n = A->nr;
    omega = (T)om;
    steps = st;
    dinv.alloc(n);
    if (sizeof(T) == sizeof(double)) NF_HIP(hipMemcpyAsync(dinv.p, dinv64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else cast_copy<double, float>(dinv64, (float*)dinv.p, n, s);
    DBuf<int> gptr, gadj;
    int nn = 0;
    const int* gpp;
    const int* gap;
    if (gp && ga) {
      nn = nn_given;
      gpp = gp->p;
      gap = ga->p;
    } else {
      node_graph(*A, b, gptr, gadj, &nn, s);
      gpp = gptr.p;
      gap = gadj.p;
    }
    DBuf<int> color(nn > 0 ? nn : 1);
    const int nc = color_nodes(nn, gpp, gap, seed, color.p, s);
    std::vector<int> hc(nn);
    NF_HIP(hipMemcpyAsync(hc.data(), color.p, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    // group node ids by colour (ascending within a colour)
    off.assign(nc + 1, 0);
    for (int c : hc) off[c + 1]++;
    for (int c = 0; c < nc; ++c) off[c + 1] += off[c];
    std::vector<int> list(nn > 0 ? nn : 1), cur(off.begin(), off.end() - 1);
    for (int u = 0; u < nn; ++u) list[cur[hc[u]]++] = u;
    nodes.alloc(list.size());
    NF_HIP(hipMemcpyAsync(nodes.p, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, s));
    off_dev.alloc(off.size());
    NF_HIP(hipMemcpyAsync(off_dev.p, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, s));
    cptr.alloc((size_t)(nn > 0 ? nn : 1) * (b + 1));
    sgs_node_ptrs(*A, b, nodes.p, nn, cptr.p, s);
    NF_HIP(hipStreamSynchronize(s));
    kind = sgs_kind(*A, b, nn, nc);
    bsr = kind == SGS_COLOR && nn >= SGS_BSR_MIN_NODES && sgs_bsr_setup<T>(*A, b, nodes.p, nn, bcp, s);
    const double nblk = bsr ? (double)A->bsr_nblk : 0.0, slots = (double)b * b;
    // a sweep's algorithmic bytes for the solve statistics: every entry and
    // row bound once (a block copy: every value, one column per block and two
    // bounds per node), node ids and D^-1, and per right-hand side the rhs,
    // the own x read and written and the operand x once
    {
      const double sz = sizeof(T);
      stat_bytes = (double)A->nnz * (sz + 4) + 4.0 * (b + 2) * nn + sz * n;
      stat_bytes_bsr = nblk * (slots * sz + 4.0) + 12.0 * nn + sz * n;
      stat_bytes_x = 4.0 * sz * n;
    }
    // per-launch bytes with the distinct columns of every colour, counted
    // only while launch timing is recording
    sweep_bytes = 0.0;
    sweep_bytes_x = 0.0;
    if (prof_recording()) {
      std::vector<int64_t> cnnz, ccols;
      color_traffic(*A, b, nodes.p, off, cnnz, ccols, s);
      std::vector<int> hp;
      if (bsr) {   // blocks of each colour, from the block row bounds
        hp.resize((size_t)nn + 1);
        NF_HIP(hipMemcpyAsync(hp.data(), A->bsr_ptr.p, sizeof(int) * (nn + 1), hipMemcpyDeviceToHost, s));
        NF_HIP(hipStreamSynchronize(s));
      }
      const double sz = sizeof(T);
      for (int c = 0; c < nc; ++c) {
        const double rows = (double)(off[c + 1] - off[c]) * b;
        sweep_bytes += cnnz[c] * (sz + 4) + 4.0 * (b + 2) * (off[c + 1] - off[c]) + rows * sz;
        if (bsr) {
          double blocks = 0.0;
          for (int t = off[c]; t < off[c + 1]; ++t) blocks += hp[list[t] + 1] - hp[list[t]];
          sweep_bytes_bsr += blocks * (slots * sz + 4.0) + 12.0 * (off[c + 1] - off[c]) + rows * sz;
        }
        sweep_bytes_x += rows * 3 * sz + sz * ccols[c];
      }
    }
  }
  // algorithmic bytes of one sweep over all colours: every colour's rows'
  // entries and pointers, node ids and D^-1 (once), and per right-hand side
  // its rhs, own x read and written and each distinct column value read
  double sweep_bytes = 0.0, sweep_bytes_x = 0.0, stat_bytes = 0.0, stat_bytes_x = 0.0;
  double sweep_bytes_bsr = 0.0, stat_bytes_bsr = 0.0;
  void sweep(bool forward, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
    const int nc = (int)off.size() - 1;
    const bool blocks = bsr && nrhs == 1;
    bytes_count((blocks ? stat_bytes_bsr : stat_bytes) + nrhs * stat_bytes_x);
    const int slot = prof_begin(s);
    if (blocks) sgs_sweep_bsr<T>(*A, nodes.p, bcp.p, off, forward, dinv.p, omega, rhs, x, s);
    else sgs_sweep<T>(*A, b, nodes.p, cptr.p, off_dev.p, off, forward, dinv.p, omega, rhs, ldr, x, ldx, nrhs, s);
    // rows field of the key: the node-group size (a power of two), or for a
    // block copy its block size
    const int b2 = blocks ? b : b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
    const int lanes = blocks ? SGS_BSR_LANES : kind == SGS_NODE ? 256 / b2 : sgs_lanes(*A, b);
    const int mode = blocks ? 11 : kind == SGS_SWEEP1 ? 7 : kind == SGS_NODE ? 8 : 6;
    int launches = kind == SGS_SWEEP1 ? 1 : 0;
    if (kind != SGS_SWEEP1)
      for (int c = 0; c < nc; ++c) launches += off[c + 1] > off[c] ? 1 : 0;
    prof_end(slot, s, ((lanes * 16 + b2) * 100 + mode) * 10 + (sizeof(T) == 4 ? 1 : 0),
             (blocks ? sweep_bytes_bsr : sweep_bytes) + nrhs * sweep_bytes_x, launches);
  }
  // half: pre-smoothing sweeps forward only, post-smoothing backward only
  int half = 0;
  bool pre = true;
  void set_phase(bool p) override { pre = p; }
  void apply(const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) override {
    if (zero_guess) fillm<T>(x, ldx, (T)0, n, nrhs, s);
    for (int st = 0; st < steps; ++st) {
      if (!half || pre) sweep(true, rhs, ldr, x, ldx, nrhs, s);
      if (!half || !pre) sweep(false, rhs, ldr, x, ldx, nrhs, s);
    }
  }
};

// DD(GS) with damping omega (the paper's domain-decomposition smoother,
// Sec. 7): subdomains = the level's aggregates (given, or computed from the
// node graph with the hierarchy's MIS-2 rule), one workgroup per subdomain
// relaxing its nodes in colour order against the other subdomains' values
// from the start of the sweep; forward then backward, or half sweeps.
template <class T>
static std::unique_ptr<FieldSmootherD<T>> make_sgs(const DCsr* A, int b, const double* dinv64, double omega, int steps,
                                                   uint64_t seed, hipStream_t s, const DBuf<int>* gp, const DBuf<int>* ga,
                                                   int nn, int half);

template <class T>
struct DdgsD : FieldSmootherD<T> {
  const DCsr* A = nullptr;
  int b = 1, steps = 1, n = 0, nsub = 0, nc = 0, half = 0, max_nodes = 0;
  std::unique_ptr<FieldSmootherD<T>> whole;   // a level with few subdomains: one subdomain (multicolour SGS)
  bool pre = true;
  T omega = 1;
  DBuf<T> dinv;
  DBuf<int> nodes, off, optr, ocol, xptr, xcol;
  DBuf<T> oval, xval;
  double avg_own = 0.0, avg_other = 0.0;
  MBuf<T> xold;
  double stat_bytes = 0.0, stat_bytes_x = 0.0;
  void setup(const DCsr* A_, int b_, const double* dinv64, double om, int st, uint64_t seed, hipStream_t s,
             const DBuf<int>* gp, const DBuf<int>* ga, int nn_given, const DBuf<int>* agg_given, int h, int ddmin) {
    A = A_;
    b = b_;
    n = A->nr;
    omega = (T)om;
    steps = st;
    half = h;
    DBuf<int> gptr, gadj;
    int nn = 0;
    const int *gpp, *gap;
    if (gp && ga) {
      nn = nn_given;
      gpp = gp->p;
      gap = ga->p;
    } else {
      node_graph(*A, b, gptr, gadj, &nn, s);
      gpp = gptr.p;
      gap = gadj.p;
    }
    DBuf<int> subd;
    const int* sp;
    if (agg_given) {
      sp = agg_given->p;
    } else {
      subd.alloc(nn > 0 ? nn : 1);
      mis2_aggregate(nn, gpp, gap, seed, subd.p, s);
      sp = subd.p;
    }
    std::vector<int> hs(nn);
    NF_HIP(hipMemcpyAsync(hs.data(), sp, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    nsub = 0;
    for (int v : hs) nsub = std::max(nsub, v + 1);
    if (nsub < ddmin) {   // one subdomain: the multicolour SGS
      whole = make_sgs<T>(A, b, dinv64, om, st, seed, s, gp && ga ? gp : nullptr, gp && ga ? ga : nullptr,
                          gp && ga ? nn_given : 0, h);
      return;
    }
    dinv.alloc(n);
    if (sizeof(T) == sizeof(double)) NF_HIP(hipMemcpyAsync(dinv.p, dinv64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else cast_copy<double, float>(dinv64, (float*)dinv.p, n, s);
    DBuf<int> color(nn > 0 ? nn : 1);
    nc = color_nodes(nn, gpp, gap, seed, color.p, s);
    std::vector<int> hc(nn);
    NF_HIP(hipMemcpyAsync(hc.data(), color.p, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    // nodes ordered by (subdomain, colour, node); off[q (nc + 1) + c]
    std::vector<int> cnt((size_t)nsub * nc + 1, 0);
    for (int u = 0; u < nn; ++u) cnt[(size_t)hs[u] * nc + hc[u] + 1]++;
    for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
    std::vector<int> list(nn > 0 ? nn : 1), cur(cnt.begin(), cnt.end() - 1);
    for (int u = 0; u < nn; ++u) list[cur[(size_t)hs[u] * nc + hc[u]]++] = u;
    std::vector<int> ho((size_t)nsub * (nc + 1)), pos(nn > 0 ? nn : 1);
    max_nodes = 0;
    for (int q = 0; q < nsub; ++q) {
      for (int c = 0; c <= nc; ++c) ho[(size_t)q * (nc + 1) + c] = cnt[(size_t)q * nc + c];
      const int q0 = ho[(size_t)q * (nc + 1)], q1 = ho[(size_t)q * (nc + 1) + nc];
      max_nodes = std::max(max_nodes, q1 - q0);
      for (int t = q0; t < q1; ++t) pos[list[t]] = t - q0;
    }
    NF_CHECK(dd_lds_bytes(b, max_nodes, g_mbuf_cols, sizeof(T)) <= DD_LDS_MAX, NFIELD_EINVAL,
             "DD(GS): a subdomain is too large for the workgroup's LDS");
    nodes.alloc(list.size());
    off.alloc(ho.size() > 0 ? ho.size() : 1);
    DBuf<int> pos_dev(pos.size());
    NF_HIP(hipMemcpyAsync(nodes.p, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, s));
    NF_HIP(hipMemcpyAsync(off.p, ho.data(), sizeof(int) * ho.size(), hipMemcpyHostToDevice, s));
    NF_HIP(hipMemcpyAsync(pos_dev.p, pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice, s));
    dd_split<T>(*A, b, nn, nodes.p, sp, pos_dev.p, optr, ocol, oval, xptr, xcol, xval, s);
    xold.alloc(n);
    NF_HIP(hipStreamSynchronize(s));   // the host lists are freed on return
    avg_own = n > 0 ? (double)oval.n / n : 0.0;
    avg_other = n > 0 ? (double)xval.n / n : 0.0;
    const double sz = sizeof(T);
    // entries and row bounds of both parts, node ids, subdomain offsets,
    // D^-1; per right-hand side rhs, x read and written, xo once
    stat_bytes = (double)A->nnz * (sz + 4) + 8.0 * (n + 1) + 4.0 * nn + 4.0 * ho.size() + sz * n;
    stat_bytes_x = 4.0 * sz * n;
  }
  void sweep(bool forward, bool from_zero, const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, hipStream_t s) {
    if (!from_zero) copym<T>(x, ldx, xold.p(), xold.ld, n, nrhs, s);
    bytes_count(stat_bytes + nrhs * stat_bytes_x);
    const int slot = prof_begin(s);
    dd_sweep<T>(b, nsub, nodes.p, off.p, nc, forward, avg_own, avg_other, optr.p, ocol.p, oval.p, xptr.p, xcol.p,
                xval.p, dinv.p, omega, rhs, ldr, from_zero ? nullptr : xold.p(), xold.ld, x, ldx, nrhs, max_nodes, s);
    const int b2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
    prof_end(slot, s, ((sgs_lanes(*A, b) * 16 + b2) * 100 + 10) * 10 + (sizeof(T) == 4 ? 1 : 0),
             stat_bytes + nrhs * stat_bytes_x, 1);
  }
  void set_phase(bool p) override {
    pre = p;
    if (whole) whole->set_phase(p);
  }
  void apply(const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) override {
    if (whole) return whole->apply(rhs, ldr, x, ldx, nrhs, zero_guess, s);
    if (zero_guess) fillm<T>(x, ldx, (T)0, n, nrhs, s);
    bool zero = zero_guess;
    for (int st = 0; st < steps; ++st) {
      if (!half || pre) {
        sweep(true, zero, rhs, ldr, x, ldx, nrhs, s);
        zero = false;
      }
      if (!half || !pre) {
        sweep(false, zero, rhs, ldr, x, ldx, nrhs, s);
        zero = false;
      }
    }
  }
};

// Symmetric Gauss-Seidel of a small many-colour level as its dense affine
// map: the colouring, ordering and damping of SgsD, with the whole symmetric
// sweep x <- S x + Q b precomputed (X = [S | Q], n x 2n) and applied as one
// GEMV per sweep instead of one launch per colour and direction.
template <class T>
struct DenseSgsD : FieldSmootherD<T> {
  int n = 0, steps = 1, b2 = 1;
  DBuf<T> X;
  MBuf<T> y;
  void setup(const SgsD<T>& g, const DCsr* A, int b, const double* dinv64, double omega, int st, hipStream_t s) {
    n = A->nr;
    steps = st;
    b2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
    const size_t m = 2 * (size_t)n * n;
    if (sizeof(T) == sizeof(double)) {
      X.alloc(m);
      dense_sgs_build(*A, b, g.nodes.p, g.off_dev.p, g.off, dinv64, omega, (double*)X.p, s);
    } else {
      DBuf<double> X64(m);
      dense_sgs_build(*A, b, g.nodes.p, g.off_dev.p, g.off, dinv64, omega, X64.p, s);
      X.alloc(m);
      cast_copy<double, float>(X64.p, (float*)X.p, (int64_t)m, s);
    }
    y.alloc(n);
  }
  void apply(const T* rhs, int64_t ldr, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) override {
    for (int st = 0; st < steps; ++st) {
      const bool with_x = !(zero_guess && st == 0);
      const double bytes =
          (double)sizeof(T) * n * (with_x ? 2.0 * n : (double)n) + (double)nrhs * sizeof(T) * n * (with_x ? 3 : 2);
      bytes_count(bytes);
      const int slot = prof_begin(s);
      dense_sweep_apply<T>(X.p, n, x, ldx, rhs, ldr, y.p(), y.ld, nrhs, with_x, s);
      prof_end(slot, s, ((64 * 16 + b2) * 100 + 9) * 10 + (sizeof(T) == 4 ? 1 : 0), bytes);
      copym<T>(y.p(), y.ld, x, ldx, n, nrhs, s);
    }
  }
};

// One BGS sweep over fields [f0, f1) of a block matrix with per-field inner
// solves: dd_i = S_i(res_i - sum_{j done} A_ij dd_j).
template <class T, class Inner>
static void bgs_sweep(const BlockMat& A, int f0, int f1, int order, const T* res, int64_t ldres, T* dd, int64_t lddd,
                      T* t, int64_t ldt, int nrhs, Inner inner, hipStream_t s) {
  std::vector<int> o = A.offsets();
  std::vector<int> seq;
  for (int i = f0; i < f1; ++i) seq.push_back(i);
  if (order == 1) std::reverse(seq.begin(), seq.end());
  std::vector<char> done(A.N, 0);
  for (int i : seq) {
    const int oi = o[i] - o[f0];
    bool first = true;
    for (int j = f0; j < f1; ++j) {
      if (j == i || !done[j] || !A.at(i, j)) continue;
      SpmvArgs<T> a;
      a.x = dd + (o[j] - o[f0]);
      a.ldx = lddd;
      a.y = t;
      a.ldy = ldt;
      a.b = res + oi;
      a.ldb = ldres;
      a.nrhs = nrhs;
      spmv<T>(first ? SPMV_RESID : SPMV_SUB, *A.at(i, j), a, s);
      first = false;
    }
    if (first) inner(i, res + oi, ldres, dd + oi, lddd);
    else inner(i, (const T*)t, ldt, dd + oi, lddd);
    done[i] = 1;
  }
}

// Level smoother of a (monolithic) hierarchy (Sec. 4.3, last paragraph):
// one BGS sweep over the level's blocks, or one SIMPLE step with the last
// field as the Schur field, each with the fields' own smoothers in place of
// the block solves (a single field: the field smoother itself).
template <class T>
struct LevelSmootherD {
  const BlockMat* A = nullptr;
  int order = 1;
  int kind = 0;                     // 0 BGS, 1 SIMPLE
  std::vector<std::unique_ptr<FieldSmootherD<T>>> cheb;
  MBuf<T> r, d, t;
  // SIMPLE: fields [0, N-1) predictor, field N-1 Schur
  DBuf<T> dtinv;                    // SIMPLEC diagonal of the predictor block, inverted
  std::unique_ptr<Solver<T>> schur; // dense inverse or Chebyshev on S~
  MBuf<T> ts, u;
  void smooth(const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs, bool zero_guess, hipStream_t s) {
    const int N = A->N;
    // pre-smoothing starts from zero, post-smoothing does not
    for (auto& c : cheb) c->set_phase(zero_guess);
    if (N == 1) {
      cheb[0]->apply(b, ldb, x, ldx, nrhs, zero_guess, s);
      return;
    }
    const T* res = b;
    int64_t ldres = ldb;
    if (!zero_guess) {
      block_resid<T>(*A, 0, N, b, ldb, x, ldx, r.p(), r.ld, nrhs, s);
      res = r.p();
      ldres = r.ld;
    }
    T* dd = zero_guess ? x : d.p();
    const int64_t lddd = zero_guess ? ldx : d.ld;
    const int ord = order == 2 ? (zero_guess ? 0 : 1) : order;
    auto inner = [&](int i, const T* rhs, int64_t ldrhs, T* out, int64_t ldout) {
      cheb[i]->apply(rhs, ldrhs, out, ldout, nrhs, true, s);
    };
    if (kind == 0) {
      bgs_sweep<T>(*A, 0, N, ord, res, ldres, dd, lddd, t.p(), t.ld, nrhs, inner, s);
    } else {
      const int g = N - 1;
      std::vector<int> o = A->offsets();
      bgs_sweep<T>(*A, 0, g, ord, res, ldres, dd, lddd, t.p(), t.ld, nrhs, inner, s);   // predictor
      bool first = true;
      for (int j = 0; j < g; ++j) {
        if (!A->at(g, j)) continue;
        SpmvArgs<T> a;
        a.x = dd + o[j];
        a.ldx = lddd;
        a.y = ts.p();
        a.ldy = ts.ld;
        a.b = res + o[g];
        a.ldb = ldres;
        a.nrhs = nrhs;
        spmv<T>(first ? SPMV_RESID : SPMV_SUB, *A->at(g, j), a, s);
        first = false;
      }
      if (first) schur->apply(res + o[g], ldres, dd + o[g], lddd, nrhs, s);
      else schur->apply(ts.p(), ts.ld, dd + o[g], lddd, nrhs, s);
      for (int j = 0; j < g; ++j) {
        if (!A->at(j, g)) continue;
        SpmvArgs<T> a;
        a.x = dd + o[g];
        a.ldx = lddd;
        a.y = u.p();
        a.ldy = u.ld;
        a.nrhs = nrhs;
        spmv<T>(SPMV_STORE, *A->at(j, g), a, s);
        sub_scaledm<T>(dtinv.p + o[j], u.p(), u.ld, dd + o[j], lddd, A->size[j], nrhs, s);
      }
    }
    if (!zero_guess) add_intom<T>(d.p(), d.ld, x, ldx, A->total(), nrhs, nullptr, s);
  }
};

template <class T>
struct AmgSolverD : Solver<T> {
  Hierarchy* H = nullptr;
  std::vector<LevelSmootherD<T>> sm;
  std::vector<MBuf<T>> res, bl, xl;   // per level: residual; right-hand side and iterate (levels > 0)
  void vcycle(int l, const T* b, int64_t ldb, T* x, int64_t ldx, int nrhs, hipStream_t s) {
    const Level& L = H->lev[l];
    if (l == (int)H->lev.size() - 1) {
      dense_gemvm<T>(H->coarse_inv.p, H->ncoarse, b, ldb, x, ldx, nrhs, s);
      return;
    }
    sm[l].smooth(b, ldb, x, ldx, nrhs, true, s);
    block_resid<T>(L.A, 0, L.A.N, b, ldb, x, ldx, res[l].p(), res[l].ld, nrhs, s);
    const Level& C = H->lev[l + 1];
    std::vector<int> o = L.A.offsets(), oc = C.A.offsets();
    for (int i = 0; i < L.A.N; ++i) {
      SpmvArgs<T> a;
      a.x = res[l].p() + o[i];
      a.ldx = res[l].ld;
      a.y = bl[l + 1].p() + oc[i];
      a.ldy = bl[l + 1].ld;
      a.nrhs = nrhs;
      spmv<T>(SPMV_STORE, *L.R[i], a, s);
    }
    vcycle(l + 1, bl[l + 1].p(), bl[l + 1].ld, xl[l + 1].p(), xl[l + 1].ld, nrhs, s);
    for (int i = 0; i < L.A.N; ++i) {
      SpmvArgs<T> a;
      a.x = xl[l + 1].p() + oc[i];
      a.ldx = xl[l + 1].ld;
      a.y = x + o[i];
      a.ldy = ldx;
      a.nrhs = nrhs;
      spmv<T>(SPMV_ADD, *L.P[i], a, s);
    }
    sm[l].smooth(b, ldb, x, ldx, nrhs, false, s);
  }
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    vcycle(0, r, ldr, z, ldz, nrhs, s);
  }
};

// A single-level smoother used as a block solve (the DD(GS) block solver of
// the paper's single-level comparison BGS(DD(GS)), Sec. 7): its sweeps from
// a zero guess, forward then backward.
template <class T>
struct SmootherSolverD : Solver<T> {
  std::unique_ptr<FieldSmootherD<T>> sm;
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    sm->apply(r, ldr, z, ldz, nrhs, true, s);
  }
};

template <class T>
struct LuSolverD : Solver<T> {
  DBuf<double> inv;
  int nn = 0;
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    dense_gemvm<T>(inv.p, nn, r, ldr, z, ldz, nrhs, s);
  }
};

template <class T>
struct BgsSolverD : Solver<T> {
  const BlockMat* A = nullptr;
  int f0 = 0, f1 = 0, sweeps = 1, order = 1;
  std::vector<std::unique_ptr<Solver<T>>> child;
  MBuf<T> res, d, t;
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    for (int sw = 0; sw < sweeps; ++sw) {
      const T* rr = r;
      int64_t ldrr = ldr;
      if (sw > 0) {
        block_resid<T>(*A, f0, f1, r, ldr, z, ldz, res.p(), res.ld, nrhs, s);
        rr = res.p();
        ldrr = res.ld;
      }
      T* dd = sw == 0 ? z : d.p();
      const int64_t lddd = sw == 0 ? ldz : d.ld;
      const int ord = order == 2 ? (sw % 2) : order;
      bgs_sweep<T>(*A, f0, f1, ord, rr, ldrr, dd, lddd, t.p(), t.ld, nrhs,
                   [&](int i, const T* rhs, int64_t ldrhs, T* out, int64_t ldout) {
                     child[i - f0]->apply(rhs, ldrhs, out, ldout, nrhs, s);
                   }, s);
      if (sw > 0) add_intom<T>(d.p(), d.ld, z, ldz, this->n, nrhs, nullptr, s);
    }
  }
};

// SIMPLE over fields [f0, f1) with predictor group [f0, g) and Schur field g
// (matrix form of M_SIMPLE, Sec. 4.2).
template <class T>
struct SimpleSolverD : Solver<T> {
  const BlockMat* A = nullptr;
  int f0 = 0, f1 = 0, g = 0, sweeps = 1;
  std::unique_ptr<Solver<T>> pred, schur;
  DBuf<T> dtinv;
  MBuf<T> res, d, t, u;
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    std::vector<int> o = A->offsets();
    const int n1 = o[g] - o[f0];
    for (int sw = 0; sw < sweeps; ++sw) {
      const T* rr = r;
      int64_t ldrr = ldr;
      if (sw > 0) {
        block_resid<T>(*A, f0, f1, r, ldr, z, ldz, res.p(), res.ld, nrhs, s);
        rr = res.p();
        ldrr = res.ld;
      }
      T* dd = sw == 0 ? z : d.p();
      const int64_t lddd = sw == 0 ? ldz : d.ld;
      pred->apply(rr, ldrr, dd, lddd, nrhs, s);
      bool first = true;
      for (int j = f0; j < g; ++j) {
        if (!A->at(g, j)) continue;
        SpmvArgs<T> a;
        a.x = dd + (o[j] - o[f0]);
        a.ldx = lddd;
        a.y = t.p();
        a.ldy = t.ld;
        a.b = rr + n1;
        a.ldb = ldrr;
        a.nrhs = nrhs;
        spmv<T>(first ? SPMV_RESID : SPMV_SUB, *A->at(g, j), a, s);
        first = false;
      }
      if (first) schur->apply(rr + n1, ldrr, dd + n1, lddd, nrhs, s);
      else schur->apply(t.p(), t.ld, dd + n1, lddd, nrhs, s);
      for (int j = f0; j < g; ++j) {
        if (!A->at(j, g)) continue;
        const int oj = o[j] - o[f0];
        SpmvArgs<T> a;
        a.x = dd + n1;
        a.ldx = lddd;
        a.y = u.p();
        a.ldy = u.ld;
        a.nrhs = nrhs;
        spmv<T>(SPMV_STORE, *A->at(j, g), a, s);
        sub_scaledm<T>(dtinv.p + oj, u.p(), u.ld, dd + oj, lddd, A->size[j], nrhs, s);
      }
      if (sw > 0) add_intom<T>(d.p(), d.ld, z, ldz, this->n, nrhs, nullptr, s);
    }
  }
};

// ================================================================== spec
struct Spec {
  std::string name;
  int sweeps = -1, order = -1, degree = -1, smoother = -1, steps = -1, half = 0, pg = 0, ddmin = 256;
  int cheb_from = -1;   // Gauss-Seidel / DD(GS) hierarchies: Chebyshev on levels >= cheb_from
  double omega = -1.0;
  std::vector<Spec> kids;
};

static Spec parse_spec(const std::string& str) {
  size_t i = 0;
  auto ws = [&]() { while (i < str.size() && str[i] == ' ') ++i; };
  std::function<Spec()> node = [&]() -> Spec {
    ws();
    Spec sp;
    while (i < str.size() && isalpha((unsigned char)str[i])) sp.name += (char)toupper(str[i++]);
    NF_CHECK(!sp.name.empty(), NFIELD_EINVAL, "spec: method name expected in '" + str + "'");
    ws();
    if (i < str.size() && str[i] == '[') {
      ++i;
      while (i < str.size() && str[i] != ']') {
        ws();
        std::string k, v;
        while (i < str.size() && (isalpha((unsigned char)str[i]) || str[i] == '_')) k += (char)tolower(str[i++]);
        ws();
        NF_CHECK(i < str.size() && str[i] == '=', NFIELD_EINVAL, "spec: '=' expected");
        ++i;
        ws();
        while (i < str.size() && (isalnum((unsigned char)str[i]) || str[i] == '.')) v += (char)tolower(str[i++]);
        ws();
        if (k == "sweeps") {
          sp.sweeps = atoi(v.c_str());
          NF_CHECK(sp.sweeps >= 1, NFIELD_EINVAL, "spec: sweeps must be >= 1");
        } else if (k == "order") {
          sp.order = v == "fwd" ? 0 : v == "bwd" ? 1 : v == "sym" ? 2 : -9;
          NF_CHECK(sp.order >= 0, NFIELD_EINVAL, "spec: order must be fwd, bwd or sym");
        } else if (k == "degree") {
          sp.degree = atoi(v.c_str());
          NF_CHECK(sp.degree >= 1, NFIELD_EINVAL, "spec: degree must be >= 1");
        } else if (k == "smoother") {
          sp.smoother = v == "cheb" ? 0 : v == "sgs" ? 1 : v == "ddgs" ? 2 : -9;
          NF_CHECK(sp.smoother >= 0, NFIELD_EINVAL, "spec: smoother must be cheb, sgs or ddgs");
        } else if (k == "omega") {
          sp.omega = atof(v.c_str());
          NF_CHECK(sp.omega > 0.0 && sp.omega < 2.0, NFIELD_EINVAL, "spec: omega must be in (0, 2)");
        } else if (k == "steps") {
          sp.steps = atoi(v.c_str());
          NF_CHECK(sp.steps >= 1, NFIELD_EINVAL, "spec: steps must be >= 1");
        } else if (k == "half") {
          sp.half = atoi(v.c_str());
          NF_CHECK(sp.half == 0 || sp.half == 1, NFIELD_EINVAL, "spec: half must be 0 or 1");
        } else if (k == "pg") {
          sp.pg = atoi(v.c_str());
          NF_CHECK(sp.pg == 0 || sp.pg == 1, NFIELD_EINVAL, "spec: pg must be 0 or 1");
        } else if (k == "ddmin") {
          sp.ddmin = atoi(v.c_str());
          NF_CHECK(sp.ddmin >= 1, NFIELD_EINVAL, "spec: ddmin must be >= 1");
        } else if (k == "cheb_from") {
          sp.cheb_from = atoi(v.c_str());
          NF_CHECK(sp.cheb_from >= 1, NFIELD_EINVAL, "spec: cheb_from must be >= 1");
        } else {
          throw NfError(NFIELD_EINVAL, "spec: unknown parameter " + k);
        }
        if (i < str.size() && str[i] == ',') ++i;
      }
      NF_CHECK(i < str.size() && str[i] == ']', NFIELD_EINVAL, "spec: ']' expected");
      ++i;
      ws();
    }
    if (i < str.size() && str[i] == '(') {
      ++i;
      sp.kids.push_back(node());
      ws();
      while (i < str.size() && str[i] == ';') {
        ++i;
        sp.kids.push_back(node());
        ws();
      }
      NF_CHECK(i < str.size() && str[i] == ')', NFIELD_EINVAL, "spec: ')' expected");
      ++i;
    }
    ws();
    return sp;
  };
  Spec sp = node();
  NF_CHECK(i == str.size(), NFIELD_EINVAL, "spec: trailing characters in '" + str + "'");
  return sp;
}

// method names and arities, checked before any device work
static void check_spec(const Spec& sp) {
  const size_t k = sp.kids.size();
  if (sp.name == "LU") NF_CHECK(k == 0, NFIELD_EINVAL, "spec: LU takes no argument");
  else if (sp.name == "DDGS") NF_CHECK(k == 0, NFIELD_EINVAL, "spec: DDGS takes no argument");
  else if (sp.name == "AMG") {
    NF_CHECK(k <= 1, NFIELD_EINVAL, "spec: AMG takes at most one level smoother");
    if (k == 1) {
      NF_CHECK(sp.kids[0].name == "BGS" || sp.kids[0].name == "SIMPLE", NFIELD_EINVAL,
               "spec: AMG level smoother must be BGS or SIMPLE");
      NF_CHECK(sp.kids[0].kids.empty(), NFIELD_EINVAL, "spec: a level smoother takes no inner solver");
    }
    return;
  } else if (sp.name == "BGS") NF_CHECK(k == 1, NFIELD_EINVAL, "spec: BGS takes one inner solver");
  else if (sp.name == "SIMPLE") NF_CHECK(k == 1 || k == 2, NFIELD_EINVAL, "spec: SIMPLE(pred[;schur])");
  else throw NfError(NFIELD_EINVAL, "spec: unknown method " + sp.name);
  for (const Spec& c : sp.kids) check_spec(c);
}

}  // namespace nf

// ============================================================== context
// A subtree of the solver built concurrently with its siblings: its own host
// thread, stream and block cache (kept across rebuilds, so the cache serves
// the next build of the same subtree).
struct SideBuild {
  nf::DevPool pool;
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  ~SideBuild() {
    pool.trim();
    if (done) (void)hipEventDestroy(done);
    if (st) (void)hipStreamDestroy(st);
  }
};

struct nfield_ctx {
  nf::DevPool pool;   // first member: destroyed after every buffer it backs
  std::vector<std::unique_ptr<SideBuild>> side;   // second: after every buffer they back
  size_t side_next = 0;
  std::mutex side_mu;   // nested concurrent builds take their side slots under it
  int N = 0;
  std::vector<nf::FieldDev> F;
  nf::BlockMat A;
  nf::DCsr Aglob;   // all blocks merged into one CSR (GMRES operator)
  nf::Opts o;
  std::vector<std::unique_ptr<nf::Hierarchy>> hiers;
  std::vector<std::unique_ptr<nf::BlockMat>> owned;
  std::unique_ptr<nf::Solver<double>> root64;
  std::unique_ptr<nf::Solver<float>> root32;
  nf::Spec spec;
  std::vector<std::shared_ptr<nf::DBuf<int>>> gpos;   // per block: entry -> position in Aglob
  bool inputs_dropped = false;   // FP32 tree built: input blocks hold no FP64 values
  nf::DBuf<float> r32, z32;
  double setup_s = 0.0;
  size_t tree_bytes = 0;   // live device bytes the preconditioner tree holds
  // GMRES workspace
  int ws_m = 0, ws_nr = 0;
  nf::DBuf<double> V, Z, w, z, r, u, H, cs, sn, g, y, h1, h2, partial, scal;
  nf::DBuf<int> imask;
  double* pinned = nullptr;
  int* pinned_i = nullptr;
  // residual estimates of the last solve, per column
  std::vector<std::vector<double>> hist;
  // preconditioner replay: graph per column count, captured on a private
  // stream into fixed input / output buffers
  hipGraphExec_t gexec[nf::NRMAX + 1] = {};
  double gbytes[nf::NRMAX + 1] = {};   // algorithmic bytes of one replay
  hipStream_t cap_stream = nullptr;
  nf::DBuf<double> g_in, g_out;
  void drop_graphs() {
    for (auto& g : gexec)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  ~nfield_ctx() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (pinned) (void)hipHostFree(pinned);
    if (pinned_i) (void)hipHostFree(pinned_i);
  }
};

namespace nf {

// Independent parts of the setup (the children of a solver node: the fields
// of BGS, the predictor and Schur parts of SIMPLE; a hierarchy and its finest
// level's Gauss-Seidel set-up) run concurrently: the first on the calling
// thread and stream, every other one on a host thread and a stream of its own
// that first waits for everything already queued on s, allocating from the
// part's own block cache; s then waits for every part's stream.  (Keeping
// the first part on s keeps the number of streams, which share a few
// hardware queues, low.)  Hierarchies and owned blocks are handed back in
// task order, so the tree, and every result, is the same as built one by one.
static void run_concurrently(nfield_ctx& C, const std::vector<std::function<void(hipStream_t)>>& tasks, hipStream_t s) {
  const size_t n = tasks.size();
  if (n < 2 || !C.o.parallel_setup) {
    for (size_t k = 0; k < n; ++k) tasks[k](s);
    return;
  }
  int dev = 0;
  NF_HIP(hipGetDevice(&dev));
  std::vector<SideBuild*> sb(n, nullptr);
  {
    std::lock_guard<std::mutex> lock(C.side_mu);
    for (size_t k = 1; k < n; ++k) {
      if (C.side_next == C.side.size()) {
        auto b = std::make_unique<SideBuild>();
        NF_HIP(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
        NF_HIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
        C.side.push_back(std::move(b));
      }
      sb[k] = C.side[C.side_next++].get();
    }
  }
  hipEvent_t start;
  NF_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  NF_HIP(hipEventRecord(start, s));
  std::vector<std::vector<std::unique_ptr<Hierarchy>>> hs(n);
  std::vector<std::vector<std::unique_ptr<BlockMat>>> os(n);
  std::vector<std::exception_ptr> err(n);
  std::vector<char> ok(n, 0);
  std::vector<std::thread> th;
  const int cols = g_mbuf_cols;
  for (size_t k = 1; k < n; ++k)
    th.emplace_back([&, k, cols] {
      try {
        g_mbuf_cols = cols;
        setup_mode(true);
        NF_HIP(hipSetDevice(dev));
        g_pool = &sb[k]->pool;
        g_hsink = &hs[k];
        g_osink = &os[k];
        prof_quiet(true);
        sb[k]->pool.enter(sb[k]->st);
        NF_HIP(hipStreamWaitEvent(sb[k]->st, start, 0));
        tasks[k](sb[k]->st);
        NF_HIP(hipEventRecord(sb[k]->done, sb[k]->st));
        ok[k] = 1;
      } catch (...) {
        err[k] = std::current_exception();
      }
    });
  // the first task here, straight into this thread's sinks (it comes first)
  try {
    tasks[0](s);
  } catch (...) {
    err[0] = std::current_exception();
  }
  for (auto& t : th) t.join();
  (void)hipEventDestroy(start);
  for (size_t k = 1; k < n; ++k)
    if (ok[k]) NF_HIP(hipStreamWaitEvent(s, sb[k]->done, 0));
  for (size_t k = 1; k < n; ++k) {
    for (auto& h : hs[k]) g_hsink->push_back(std::move(h));
    for (auto& o : os[k]) g_osink->push_back(std::move(o));
  }
  for (size_t k = 0; k < n; ++k)
    if (err[k]) {
      // the other tasks may still have work queued on their streams
      for (size_t j = 1; j < n; ++j) (void)hipStreamSynchronize(sb[j]->st);
      std::rethrow_exception(err[k]);
    }
}

template <class T>
using BuildTask = std::function<std::unique_ptr<Solver<T>>(hipStream_t)>;

template <class T>
static std::vector<std::unique_ptr<Solver<T>>> build_children(nfield_ctx& C, const std::vector<BuildTask<T>>& tasks,
                                                              hipStream_t s) {
  std::vector<std::unique_ptr<Solver<T>>> out(tasks.size());
  std::vector<std::function<void(hipStream_t)>> run;
  for (size_t k = 0; k < tasks.size(); ++k) run.push_back([&out, &tasks, k](hipStream_t st) { out[k] = tasks[k](st); });
  run_concurrently(C, run, s);
  return out;
}

template <class T>
static std::unique_ptr<Solver<T>> build(nfield_ctx& C, const Spec& sp, const BlockMat& A, const std::vector<FieldDev>& F,
                                        int f0, int f1, hipStream_t s);

// SIMPLE pieces over fields [f0, g) (predictor) and g (Schur), Sec. 3.2:
// dt = inverse of the SIMPLEC-type diagonal of the merged predictor block
// (mode 0: sum_j |a_ij|, 1: |sum_j a_ij|, 2: a_ii, over the predictor
// columns), and S~ = A_gg - sum_i A_gi diag(dt_i) A_ig.
static void simple_parts(const BlockMat& A, int f0, int g, int mode, DBuf<double>& dt, DCsr& Sm, hipStream_t s) {
  std::vector<int> o = A.offsets();
  const int n1 = o[g] - o[f0], n2 = A.size[g];
  dt.alloc(n1 > 0 ? n1 : 1);
  DBuf<int> zf(1);
  fill<double>(dt.p, 0.0, n1, s);
  fill<int>(zf.p, 0, 1, s);
  for (int i = f0; i < g; ++i)
    for (int j = f0; j < g; ++j)
      if (A.at(i, j)) row_accumulate(*A.at(i, j), mode, i == j, dt.p + (o[i] - o[f0]), s);
  finish_simplec(dt.p, n1, mode, zf.p, s);
  int z = 0;
  NF_HIP(hipMemcpyAsync(&z, zf.p, sizeof(int), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  NF_CHECK(z == 0, NFIELD_ESINGULAR, "SIMPLE: zero entry in the approximate predictor diagonal");
  if (A.at(g, g)) csr_copy(*A.at(g, g), Sm, s);
  else { Sm.nr = Sm.nc = n2; Sm.nnz = 0; }
  for (int i = f0; i < g; ++i) {
    if (!A.at(g, i) || !A.at(i, g)) continue;
    DCsr Tm, prod, sum;
    csr_copy(*A.at(i, g), Tm, s);
    scale_rows(Tm, dt.p + (o[i] - o[f0]), s);
    spgemm(*A.at(g, i), Tm, prod, s);
    csr_add(1.0, Sm, -1.0, prod, sum, s);
    Sm = std::move(sum);
  }
  NF_HIP(hipStreamSynchronize(s));
  NF_CHECK(Sm.nnz > 0, NFIELD_ESINGULAR, "SIMPLE: approximate Schur complement is zero");
}

// Chebyshev on S~ used as the Schur solve of a SIMPLE level smoother when S~
// is too large for a dense inverse.
template <class T>
struct ChebSolverD : Solver<T> {
  std::shared_ptr<DCsr> S;
  ChebD<T> cheb;
  void apply(const T* r, int64_t ldr, T* z, int64_t ldz, int nrhs, hipStream_t s) override {
    cheb.apply(r, ldr, z, ldz, nrhs, true, s);
  }
};

// Multicolour Gauss-Seidel of one field on one level (the node graph of A is
// computed here unless given); small many-colour levels as the dense map of
// the full symmetric sweep (not with half sweeps).
template <class T>
static std::unique_ptr<FieldSmootherD<T>> make_sgs(const DCsr* A, int b, const double* dinv64, double omega, int steps,
                                                   uint64_t seed, hipStream_t s, const DBuf<int>* gp, const DBuf<int>* ga,
                                                   int nn, int half) {
  auto g = std::make_unique<SgsD<T>>();
  g->setup(A, b, dinv64, omega, steps, seed, s, gp, ga, nn);
  g->half = half;
  if (half) return g;
  const int ncol = (int)g->off.size() - 1;
  if (A->nr <= SGS_DENSE_MAX && ncol >= SGS_DENSE_MIN_COLORS) {
    auto d = std::make_unique<DenseSgsD<T>>();
    d->setup(*g, A, b, dinv64, omega, steps, s);
    return d;
  }
  return g;
}

template <class T>
static std::unique_ptr<Solver<T>> build_amg(nfield_ctx& C, const BlockMat& A, const std::vector<FieldDev>& F, int f0, int f1,
                                            const Spec* smoother, const Spec& amg, hipStream_t s) {
  Opts lo = C.o;   // smoother polynomial degree of this hierarchy
  if (amg.degree > 0) lo.cheb_degree = amg.degree;
  const bool sgs = amg.smoother == 1 || amg.smoother == 2;
  const bool dd = amg.smoother == 2;
  const double omega = amg.omega > 0.0 ? amg.omega : 1.0;
  const int steps = amg.steps > 0 ? amg.steps : 1;
  BlockMat sub = A.sub(f0, f1);
  std::vector<FieldDev> Fs(F.begin() + f0, F.begin() + f1);
  const bool simple = smoother && smoother->name == "SIMPLE";
  NF_CHECK(!simple || sub.N >= 2, NFIELD_EINVAL, "AMG(SIMPLE) needs at least two fields");
  for (int i = 0; i < sub.N; ++i)
    NF_CHECK(sub.at(i, i) != nullptr || (simple && i == sub.N - 1), NFIELD_ESINGULAR, "AMG: zero diagonal block");
  auto H = std::make_unique<Hierarchy>();
  Opts ho = C.o;   // this hierarchy's transfers
  ho.pg = amg.pg;
  // the finest level's Gauss-Seidel or DD(GS) needs only A_ii: set up beside
  // the hierarchy (its own D^-1, node graph and, for DD(GS), aggregates: the
  // same values as the hierarchy's), unless the level smoother is SIMPLE
  std::vector<std::unique_ptr<FieldSmootherD<T>>> sgs0(sub.N);
  if (sgs && !simple && C.o.parallel_setup) {
    std::vector<std::function<void(hipStream_t)>> tasks;
    tasks.push_back([&](hipStream_t st) { build_hierarchy(*H, sub, Fs, ho, st); });
    tasks.push_back([&](hipStream_t st) {
      for (int i = 0; i < sub.N; ++i) {
        const DCsr* Aii = sub.at(i, i);
        if (!Aii || Aii->nr <= 0) continue;
        DBuf<double> d(Aii->nr), dinv(Aii->nr);
        DBuf<int> zf(1);
        fill<int>(zf.p, 0, 1, st);
        csr_diag(*Aii, d.p, zf.p, st);
        invert(d.p, dinv.p, Aii->nr, st);
        int z = 0;
        NF_HIP(hipMemcpyAsync(&z, zf.p, sizeof(int), hipMemcpyDeviceToHost, st));
        NF_HIP(hipStreamSynchronize(st));
        if (z) continue;   // a zero diagonal entry: the hierarchy's check reports it
        if (dd) {   // its own node graph and aggregates (the same as the hierarchy's level 0)
          auto d = std::make_unique<DdgsD<T>>();
          d->setup(Aii, Fs[i].bs, dinv.p, omega, steps, C.o.seed, st, nullptr, nullptr, 0, nullptr, amg.half, amg.ddmin);
          sgs0[i] = std::move(d);
        } else {
          sgs0[i] = make_sgs<T>(Aii, Fs[i].bs, dinv.p, omega, steps, C.o.seed, st, nullptr, nullptr, 0, amg.half);
        }
        NF_HIP(hipStreamSynchronize(st));
      }
    });
    run_concurrently(C, tasks, s);
  } else {
    build_hierarchy(*H, sub, Fs, ho, s);
  }
  auto S = std::make_unique<AmgSolverD<T>>();
  S->H = H.get();
  S->n = sub.total();
  const int nl = (int)H->lev.size();
  if (sizeof(T) == sizeof(float))
    for (int l = 0; l < nl; ++l) {
      prepare_fp32(H->lev[l].A, s);
      for (auto& p : H->lev[l].P) if (p) make_fp32(*p, s);
      for (auto& r : H->lev[l].R) if (r) make_fp32(*r, s);
    }
  S->sm.resize(nl > 0 ? nl - 1 : 0);
  S->res.resize(nl);
  S->bl.resize(nl);
  S->xl.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const Level& L = H->lev[l];
    const int n = L.A.total();
    if (l > 0) {
      S->bl[l].alloc(n);
      S->xl[l].alloc(n);
    }
    if (l + 1 == nl) break;
    S->res[l].alloc(n);
    LevelSmootherD<T>& M = S->sm[l];
    M.A = &L.A;
    M.order = smoother && smoother->order >= 0 ? smoother->order : C.o.order;
    M.kind = simple ? 1 : 0;
    const int nsm = simple ? sub.N - 1 : sub.N;   // fields with their own smoother
    // Gauss-Seidel / DD(GS) on this level, or Chebyshev from level cheb_from on
    const bool cheb_l = amg.cheb_from >= 1 && l >= amg.cheb_from;
    const bool sgs_l = sgs && !cheb_l, dd_l = dd && !cheb_l;
    for (int i = 0; i < nsm; ++i) {
      NF_CHECK(L.dinv[i] != nullptr, NFIELD_ESINGULAR, "Chebyshev smoother: zero diagonal entry");
      if (dd_l && l == 0 && sgs0[i]) {
        M.cheb.push_back(std::move(sgs0[i]));
      } else if (dd_l) {
        const bool have = i < (int)L.gptr.size() && L.gptr[i] && L.gadj[i];
        const bool hagg = i < (int)L.agg.size() && L.agg[i];
        auto d = std::make_unique<DdgsD<T>>();
        d->setup(L.A.at(i, i), L.bs[i], L.dinv[i]->p, omega, steps, C.o.seed, s, have ? L.gptr[i].get() : nullptr,
                 have ? L.gadj[i].get() : nullptr, have ? L.nnode[i] : 0, hagg && have ? L.agg[i].get() : nullptr,
                 amg.half, amg.ddmin);
        M.cheb.push_back(std::move(d));
      } else if (sgs_l) {
        if (l == 0 && sgs0[i]) {
          M.cheb.push_back(std::move(sgs0[i]));
        } else {
          const bool have = i < (int)L.gptr.size() && L.gptr[i] && L.gadj[i];
          M.cheb.push_back(make_sgs<T>(L.A.at(i, i), L.bs[i], L.dinv[i]->p, omega, steps, C.o.seed, s,
                                       have ? L.gptr[i].get() : nullptr, have ? L.gadj[i].get() : nullptr,
                                       have ? L.nnode[i] : 0, amg.half));
        }
      } else {
        auto ch = std::make_unique<ChebD<T>>();
        ch->setup(L.A.at(i, i), L.dinv[i]->p, L.lambda[i], lo, s);
        M.cheb.push_back(std::move(ch));
      }
    }
    if (sub.N > 1) {
      M.r.alloc(n);
      M.d.alloc(n);
      int mx = 0;
      for (int v : L.A.size) mx = std::max(mx, v);
      M.t.alloc(mx);
    }
    if (simple) {
      const int g = sub.N - 1, n2 = L.A.size[g];
      DBuf<double> dt;
      auto Sm = std::make_shared<DCsr>();
      simple_parts(L.A, 0, g, C.o.simplec_mode, dt, *Sm, s);
      const int n1 = L.A.offsets()[g];
      M.dtinv.alloc(n1 > 0 ? n1 : 1);
      if (sizeof(T) == sizeof(double)) NF_HIP(hipMemcpyAsync(M.dtinv.p, dt.p, sizeof(double) * n1, hipMemcpyDeviceToDevice, s));
      else cast_copy<double, float>(dt.p, (float*)M.dtinv.p, n1, s);
      if (n2 <= C.o.schur_direct_max) {
        auto lu = std::make_unique<LuSolverD<T>>();
        BlockMat one;
        one.N = 1;
        one.size = {n2};
        one.blk = {Sm};
        dense_block_inverse(one, lu->inv, &lu->nn, s);
        lu->n = n2;
        M.schur = std::move(lu);
      } else {
        auto ch = std::make_unique<ChebSolverD<T>>();
        DBuf<double> dg(n2), dinv(n2);
        DBuf<int> zf(1);
        fill<int>(zf.p, 0, 1, s);
        csr_diag(*Sm, dg.p, zf.p, s);
        invert(dg.p, dinv.p, n2, s);
        int z = 0;
        NF_HIP(hipMemcpyAsync(&z, zf.p, sizeof(int), hipMemcpyDeviceToHost, s));
        NF_HIP(hipStreamSynchronize(s));
        NF_CHECK(z == 0, NFIELD_ESINGULAR, "SIMPLE: zero diagonal entry in the approximate Schur complement");
        const double lam = power_lambda(*Sm, dinv.p, C.o.seed, C.o.power_its, s);
        if (sizeof(T) == sizeof(float)) make_fp32(*Sm, s);
        ch->cheb.setup(Sm.get(), dinv.p, lam, lo, s);
        NF_HIP(hipStreamSynchronize(s));
        ch->S = Sm;
        ch->n = n2;
        M.schur = std::move(ch);
      }
      M.ts.alloc(n2);
      int mp = 0;
      for (int i = 0; i < g; ++i) mp = std::max(mp, L.A.size[i]);
      M.u.alloc(mp > 0 ? mp : 1);
    }
  }
  g_hsink->push_back(std::move(H));
  return S;
}

template <class T>
static std::unique_ptr<Solver<T>> build(nfield_ctx& C, const Spec& sp, const BlockMat& A, const std::vector<FieldDev>& F,
                                        int f0, int f1, hipStream_t s) {
  const int nf_ = f1 - f0;
  std::vector<int> o = A.offsets();
  const int n = o[f1] - o[f0];
  if (sp.name == "LU") {
    NF_CHECK(sp.kids.empty(), NFIELD_EINVAL, "spec: LU takes no argument");
    auto S = std::make_unique<LuSolverD<T>>();
    BlockMat sub = A.sub(f0, f1);
    dense_block_inverse(sub, S->inv, &S->nn, s);
    S->n = n;
    return S;
  }
  if (sp.name == "DDGS") {
    NF_CHECK(nf_ == 1, NFIELD_EINVAL, "spec: DDGS needs a single field");
    const DCsr* Aii = A.at(f0, f0);
    NF_CHECK(Aii != nullptr, NFIELD_ESINGULAR, "DDGS: zero diagonal block");
    DBuf<double> d(Aii->nr), dinv(Aii->nr);
    DBuf<int> zf(1);
    fill<int>(zf.p, 0, 1, s);
    csr_diag(*Aii, d.p, zf.p, s);
    invert(d.p, dinv.p, Aii->nr, s);
    int z = 0;
    NF_HIP(hipMemcpyAsync(&z, zf.p, sizeof(int), hipMemcpyDeviceToHost, s));
    NF_HIP(hipStreamSynchronize(s));
    NF_CHECK(z == 0, NFIELD_ESINGULAR, "DDGS: zero diagonal entry");
    need_fp32<T>(A, f0, f0, s);
    auto sm = std::make_unique<DdgsD<T>>();
    sm->setup(Aii, F[f0].bs, dinv.p, sp.omega > 0.0 ? sp.omega : 1.0, sp.steps > 0 ? sp.steps : 1, C.o.seed, s,
              nullptr, nullptr, 0, nullptr, 0, sp.ddmin);
    auto S = std::make_unique<SmootherSolverD<T>>();
    S->sm = std::move(sm);
    S->n = Aii->nr;
    return S;
  }
  if (sp.name == "AMG") {
    if (sp.kids.empty()) {
      NF_CHECK(nf_ == 1, NFIELD_EINVAL, "spec: plain AMG needs a single field; use AMG(BGS)");
      return build_amg<T>(C, A, F, f0, f1, nullptr, sp, s);
    }
    NF_CHECK(sp.kids.size() == 1, NFIELD_EINVAL, "spec: AMG takes one level smoother");
    return build_amg<T>(C, A, F, f0, f1, &sp.kids[0], sp, s);
  }
  if (sp.name == "BGS") {
    NF_CHECK(sp.kids.size() == 1, NFIELD_EINVAL, "spec: BGS takes one inner solver");
    auto S = std::make_unique<BgsSolverD<T>>();
    S->A = &A;
    S->f0 = f0;
    S->f1 = f1;
    S->sweeps = sp.sweeps > 0 ? sp.sweeps : C.o.sweeps;
    S->order = sp.order >= 0 ? sp.order : C.o.order;
    // the sweep reads the coupling blocks; the residual of later sweeps all
    // blocks (before the children, which may be built concurrently)
    for (int i = f0; i < f1; ++i)
      for (int j = f0; j < f1; ++j)
        if (i != j || S->sweeps > 1) need_fp32<T>(A, i, j, s);
    int mx = 0;
    std::vector<BuildTask<T>> tasks;
    for (int i = f0; i < f1; ++i) {
      NF_CHECK(A.at(i, i) != nullptr, NFIELD_ESINGULAR, "BGS: zero diagonal block");
      tasks.push_back([&C, &sp, &A, &F, i](hipStream_t st) { return build<T>(C, sp.kids[0], A, F, i, i + 1, st); });
      mx = std::max(mx, A.size[i]);
    }
    S->child = build_children<T>(C, tasks, s);
    S->n = n;
    S->res.alloc(n);
    S->d.alloc(n);
    S->t.alloc(mx);
    return S;
  }
  if (sp.name == "SIMPLE") {
    NF_CHECK(!sp.kids.empty() && sp.kids.size() <= 2, NFIELD_EINVAL, "spec: SIMPLE(pred[;schur])");
    NF_CHECK(nf_ >= 2, NFIELD_EINVAL, "SIMPLE needs at least two fields");
    int g = f1 - 1;
    if (!C.o.split.empty()) {
      int cnt = 0;
      for (int i = f0; i < f1; ++i)
        if (C.o.split[i] == 1) { ++cnt; g = i; }
      NF_CHECK(cnt == 1 && g == f1 - 1, NFIELD_EINVAL, "SIMPLE: the Schur group must be the last single field");
    }
    auto S = std::make_unique<SimpleSolverD<T>>();
    S->A = &A;
    S->f0 = f0;
    S->f1 = f1;
    S->g = g;
    S->sweeps = sp.sweeps > 0 ? sp.sweeps : 1;
    // the step reads A_gj and A_jg; the residual of later sweeps all blocks
    for (int i = f0; i < f1; ++i)
      for (int j = f0; j < f1; ++j)
        if (S->sweeps > 1 || (i == g) != (j == g)) need_fp32<T>(A, i, j, s);
    const int n1 = o[g] - o[f0], n2 = A.size[g];
    std::vector<FieldDev> Fs = {F[g]};
    Spec def;
    def.name = n2 <= C.o.schur_direct_max ? "LU" : "AMG";
    const Spec& ssp = sp.kids.size() == 2 ? sp.kids[1] : def;
    // the predictor needs only the predictor blocks: its set-up runs beside
    // the Schur part's, which first forms D~ and S~
    std::unique_ptr<BlockMat> Bm;
    SimpleSolverD<T>* Sp = S.get();
    const int mode = C.o.simplec_mode;
    std::vector<BuildTask<T>> tasks;
    tasks.push_back([&C, &sp, &A, &F, f0, g](hipStream_t st) { return build<T>(C, sp.kids[0], A, F, f0, g, st); });
    tasks.push_back([&C, &ssp, &A, &Fs, &Bm, Sp, f0, g, n1, n2, mode](hipStream_t st) {
      DBuf<double> dt;
      auto Sm = std::make_shared<DCsr>();
      simple_parts(A, f0, g, mode, dt, *Sm, st);
      Sp->dtinv.alloc(n1 > 0 ? n1 : 1);
      if (sizeof(T) == sizeof(double))
        NF_HIP(hipMemcpyAsync(Sp->dtinv.p, dt.p, sizeof(double) * n1, hipMemcpyDeviceToDevice, st));
      else cast_copy<double, float>(dt.p, (float*)Sp->dtinv.p, n1, st);
      Bm = std::make_unique<BlockMat>();
      Bm->N = 1;
      Bm->size = {n2};
      Bm->blk = {Sm};
      if (sizeof(T) == sizeof(float)) prepare_fp32(*Bm, st);
      auto out = build<T>(C, ssp, *Bm, Fs, 0, 1, st);
      NF_HIP(hipStreamSynchronize(st));   // dt is freed on return
      return out;
    });
    auto kids = build_children<T>(C, tasks, s);
    S->pred = std::move(kids[0]);
    S->schur = std::move(kids[1]);
    g_osink->push_back(std::move(Bm));
    S->n = n;
    S->res.alloc(n);
    S->d.alloc(n);
    S->t.alloc(n2);
    int mx = 0;
    for (int i = f0; i < g; ++i) mx = std::max(mx, A.size[i]);
    S->u.alloc(mx > 0 ? mx : 1);
    return S;
  }
  throw NfError(NFIELD_EINVAL, "spec: unknown method " + sp.name);
}

// ================================================================= GMRES
// Device and host buffers of one GMRES call: the context's own (grown on
// demand) or carved from the static scratch of the allocation-free entry
// point.
struct KrylovWs {
  double *V = nullptr, *Z = nullptr, *w = nullptr, *z = nullptr, *r = nullptr, *u = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *h1 = nullptr, *h2 = nullptr;
  double *partial = nullptr, *scal = nullptr;
  int* imask = nullptr;            // 3 NRMAX ints
  float *r32 = nullptr, *z32 = nullptr;   // FP32 staging of the precision form (n nrhs each)
  double* pinned = nullptr;        // host staging, 64 doubles
  int* pinned_i = nullptr;         // host staging, 64 ints
  bool direct = false;             // launch the preconditioner directly (no graph replay)
};

// FP32 staging of the precision form for nrhs columns, grown on demand
static void fp32_staging(nfield_ctx& C, int nrhs) {
  const int64_t n = C.Aglob.nr;
  if (C.root32 && C.r32.n < (size_t)n * nrhs) {
    C.r32.alloc((size_t)n * nrhs);
    C.z32.alloc((size_t)n * nrhs);
  }
}

// Krylov workspace for nrhs columns of restart length m in the context's
// own buffers, grown on demand (kept at the largest restart length and
// column count used so far).
static KrylovWs ctx_workspace(nfield_ctx& C, int m, int flexible, int nrhs) {
  const int64_t n = C.Aglob.nr;
  if (C.ws_m < m || C.ws_nr < nrhs) {
    const int mm = std::max(m, C.ws_m), nr = std::max(nrhs, C.ws_nr);
    C.V.alloc((size_t)n * (mm + 1) * nr);
    if (C.Z.p) C.Z.alloc((size_t)n * mm * nr);
    C.H.alloc((size_t)(mm + 1) * mm * nr);
    C.cs.alloc((size_t)mm * nr);
    C.sn.alloc((size_t)mm * nr);
    C.g.alloc((size_t)(mm + 1) * nr);
    C.y.alloc((size_t)mm * nr);
    C.h1.alloc((size_t)(mm + 1) * nr);
    C.h2.alloc((size_t)(mm + 1) * nr);
    C.partial.alloc((size_t)RED_BLOCKS * (mm + 1) * nr);
    C.ws_m = mm;
    C.ws_nr = nr;
  }
  if (flexible && C.Z.n < (size_t)n * C.ws_m * C.ws_nr) C.Z.alloc((size_t)n * C.ws_m * C.ws_nr);
  if (C.w.n < (size_t)n * C.ws_nr) {
    C.w.alloc((size_t)n * C.ws_nr);
    C.z.alloc((size_t)n * C.ws_nr);
    C.r.alloc((size_t)n * C.ws_nr);
    C.u.alloc((size_t)n * C.ws_nr);
  }
  if (!C.scal.p) {
    C.scal.alloc(4 * NRMAX);
    C.imask.alloc(3 * NRMAX);
  }
  fp32_staging(C, nrhs);
  if (!C.pinned) NF_HIP(hipHostMalloc((void**)&C.pinned, 64 * sizeof(double), hipHostMallocDefault));
  if (!C.pinned_i) NF_HIP(hipHostMalloc((void**)&C.pinned_i, 64 * sizeof(int), hipHostMallocDefault));
  KrylovWs W;
  W.V = C.V.p;
  W.Z = C.Z.p;
  W.w = C.w.p;
  W.z = C.z.p;
  W.r = C.r.p;
  W.u = C.u.p;
  W.H = C.H.p;
  W.cs = C.cs.p;
  W.sn = C.sn.p;
  W.g = C.g.p;
  W.y = C.y.p;
  W.h1 = C.h1.p;
  W.h2 = C.h2.p;
  W.partial = C.partial.p;
  W.scal = C.scal.p;
  W.imask = C.imask.p;
  W.r32 = C.r32.p;
  W.z32 = C.z32.p;
  W.pinned = C.pinned;
  W.pinned_i = C.pinned_i;
  return W;
}

static void precond_direct(nfield_ctx& C, const double* r, int64_t ldr, double* z, int64_t ldz, int nrhs, float* r32,
                           float* z32, hipStream_t s) {
  if (C.root64) {
    C.root64->apply(r, ldr, z, ldz, nrhs, s);
  } else {
    const int64_t n = C.Aglob.nr;
    castm<double, float>(r, ldr, r32, n, n, nrhs, s);
    C.root32->apply(r32, n, z32, n, nrhs, s);
    castm<float, double>(z32, n, z, ldz, n, nrhs, s);
  }
}

// z = M^-1 r.  With graphs on (and launch timing off) the preconditioner's
// kernels are recorded once per column count on a private stream, reading
// g_in and writing g_out, and replayed on s between two copies; the kernels
// and their order are those of precond_direct.  W (may be null: the
// context's own staging) gives the FP32 staging and may ask for direct
// launches.
static void precond(nfield_ctx& C, const double* r, int64_t ldr, double* z, int64_t ldz, int nrhs, hipStream_t s,
                    const KrylovWs* W = nullptr) {
  if (W && W->direct) return precond_direct(C, r, ldr, z, ldz, nrhs, W->r32, W->z32, s);
  fp32_staging(C, nrhs);
  if (!C.o.graphs || prof_recording()) return precond_direct(C, r, ldr, z, ldz, nrhs, C.r32.p, C.z32.p, s);
  const int64_t n = C.Aglob.nr;
  if (!C.g_in.p) {
    C.g_in.alloc((size_t)n * C.o.max_rhs);
    C.g_out.alloc((size_t)n * C.o.max_rhs);
  }
  if (!C.gexec[nrhs]) {
    if (!C.cap_stream) NF_HIP(hipStreamCreateWithFlags(&C.cap_stream, hipStreamNonBlocking));
    NF_HIP(hipStreamSynchronize(s));   // buffers the capture may allocate are then idle
    hipGraph_t g = nullptr;
    NF_HIP(hipStreamBeginCapture(C.cap_stream, hipStreamCaptureModeRelaxed));
    const double b0 = bytes_counted();
    try {
      precond_direct(C, C.g_in.p, n, C.g_out.p, n, nrhs, C.r32.p, C.z32.p, C.cap_stream);
      C.gbytes[nrhs] = bytes_counted() - b0;
      bytes_count(-C.gbytes[nrhs]);   // counted at each replay instead
    } catch (...) {
      (void)hipStreamEndCapture(C.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    NF_HIP(hipStreamEndCapture(C.cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&C.gexec[nrhs], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NF_HIP(e);
  }
  copym<double>(r, ldr, C.g_in.p, n, n, nrhs, s);
  bytes_count(C.gbytes[nrhs]);
  NF_HIP(hipGraphLaunch(C.gexec[nrhs], s));
  copym<double>(C.g_out.p, n, z, ldz, n, nrhs, s);
}

// ||b_k - A x_k|| for nrhs columns, read back to host res[k]
static void true_residuals(nfield_ctx& C, const KrylovWs& W, const double* b, int64_t ldb, const double* x, int64_t ldx,
                           int nrhs, double* res, hipStream_t s) {
  const int64_t n = C.Aglob.nr;
  SpmvArgs<double> a;
  a.x = x;
  a.ldx = ldx;
  a.y = W.r;
  a.ldy = n;
  a.b = b;
  a.ldb = ldb;
  a.nrhs = nrhs;
  spmv<double>(SPMV_RESID, C.Aglob, a, s);
  dotm(W.r, n, W.r, n, n, nrhs, W.partial, W.scal, s);
  NF_HIP(hipMemcpyAsync(W.pinned, W.scal, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < nrhs; ++k) res[k] = std::sqrt(W.pinned[k]);
}

static void upload_ints(const KrylovWs& W, const std::vector<int>& v, int* dev, hipStream_t s) {
  for (size_t k = 0; k < v.size(); ++k) W.pinned_i[k] = v[k];
  NF_HIP(hipMemcpyAsync(dev, W.pinned_i, sizeof(int) * v.size(), hipMemcpyHostToDevice, s));
  NF_HIP(hipStreamSynchronize(s));   // the staging buffer is reused right away
}

__global__ void k_init_gm(double* g, int m, const double* beta, const int* mask) {
  const int k = blockIdx.x, i = threadIdx.x;
  if (mask && !mask[k]) return;
  if (i <= m) g[(int64_t)k * (m + 1) + i] = i == 0 ? beta[k] : 0.0;
}

// Restarted GMRES(m) with right preconditioning (Sec. 3.2), plain or
// flexible, on nrhs independent columns at once.  Each column runs its own
// Arnoldi process (CGS2, Givens rotations on the device, its own
// convergence test and restarts); the columns share only the kernel
// launches, so a column's iterates do not depend on the other columns.
static void gmres(nfield_ctx& C, const KrylovWs& W, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                  const nfield_solve_opts& so, nfield_stats* st, hipStream_t s, std::vector<double>* hist = nullptr) {
  const int64_t n = C.Aglob.nr;
  const int m = so.restart;
  const bool flex = so.flexible != 0;
  GmresLayout L;
  L.n = n;
  L.vs = (int64_t)(m + 1) * n;
  L.hs = m + 1;
  L.ps = (int64_t)(m + 1) * RED_BLOCKS;
  L.m = m;
  L.nrhs = nrhs;
  GmresLayout LZ = L;
  LZ.vs = (int64_t)m * n;
  int* mask = W.imask;            // columns in the current Arnoldi cycle
  int* part = W.imask + NRMAX;    // columns that took part in the cycle
  int* jend = W.imask + 2 * NRMAX;
  std::vector<double> beta0(nrhs), beta(nrhs);
  std::vector<int> total(nrhs, 0), done(nrhs, 0), cyc(nrhs, 0), je(nrhs, 0), broke(nrhs, 0);
  for (int k = 0; k < nrhs; ++k) std::memset(&st[k], 0, sizeof(nfield_stats));
  true_residuals(C, W, b, ldb, x, ldx, nrhs, beta0.data(), s);
  for (int k = 0; k < nrhs; ++k) {
    if (!std::isfinite(beta0[k])) { st[k].status = NFIELD_ENAN; done[k] = 1; }
    else if (beta0[k] == 0.0) { st[k].status = NFIELD_OK; done[k] = 1; }
  }
  bool first = true;
  while (true) {
    if (first) beta = beta0;
    else true_residuals(C, W, b, ldb, x, ldx, nrhs, beta.data(), s);
    first = false;
    int nact = 0;
    for (int k = 0; k < nrhs; ++k) {
      cyc[k] = 0;
      if (done[k]) continue;
      st[k].relres = beta[k] / beta0[k];
      if (!std::isfinite(beta[k])) { st[k].status = NFIELD_ENAN; done[k] = 1; continue; }
      if (beta[k] / beta0[k] < so.rtol) { st[k].status = NFIELD_OK; done[k] = 1; continue; }
      // a breakdown whose solution fails the true-residual test: a restart
      // would rebuild the same invariant space
      if (broke[k]) { st[k].status = NFIELD_EBREAKDOWN; done[k] = 1; continue; }
      if (total[k] >= so.maxit) { st[k].status = NFIELD_NOT_CONVERGED; done[k] = 1; continue; }
      if (total[k] > 0) st[k].restarts++;
      cyc[k] = 1;
      ++nact;
    }
    if (nact == 0) break;
    upload_ints(W, cyc, mask, s);
    for (int k = 0; k < nrhs; ++k) W.pinned[k] = beta[k];
    NF_HIP(hipMemcpyAsync(W.scal + 2 * NRMAX, W.pinned, sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
    // v_0 = r / beta (r holds the residuals of the last true_residuals call)
    scale_inv_devm(W.r, n, W.V, L.vs, W.scal + 2 * NRMAX, 1, n, nrhs, mask, s);
    hipLaunchKernelGGL(k_init_gm, dim3(nrhs), dim3(64), 0, s, W.g, m, W.scal + 2 * NRMAX, mask);
    NF_HIP(hipStreamSynchronize(s));   // the beta staging buffer is reused below
    std::vector<int> in_cycle = cyc;
    std::fill(je.begin(), je.end(), 0);
    const int64_t ldz = flex ? LZ.vs : n;
    bool z_ready = false;             // z_j already enqueued by the step before
    // the last two residual estimates of each column, to foresee the end
    std::vector<double> res1(beta), res2(nrhs, 0.0);
    for (int j = 0; j < m; ++j) {
      double* vj = W.V + (int64_t)j * n;
      double* zj = flex ? W.Z + (int64_t)j * n : W.z;
      if (!z_ready) precond(C, vj, L.vs, zj, ldz, nrhs, s, &W);
      z_ready = false;
      SpmvArgs<double> a;
      a.x = zj;
      a.ldx = ldz;
      a.y = W.w;
      a.ldy = n;
      a.nrhs = nrhs;
      spmv<double>(SPMV_STORE, C.Aglob, a, s);
      // classical Gram-Schmidt, twice
      mdot_partial(L, W.V, j + 1, W.w, n, W.partial, mask, s);
      mreduce(L, W.partial, j + 1, W.h1, 0, mask, s);
      mupdate_dot(L, W.V, j + 1, W.h1, W.w, n, W.partial, mask, s);
      mreduce(L, W.partial, j + 1, W.h2, 0, mask, s);
      mupdate_norm(L, W.V, j + 1, W.h2, W.w, n, W.partial, mask, s);
      givens_step(L, j, W.h1, W.h2, W.partial, W.H, W.cs, W.sn, W.g, W.scal, mask, s);
      scale_inv_devm(W.w, n, W.V + (int64_t)(j + 1) * n, L.vs, W.scal, 2, n, nrhs, mask, s);
      NF_HIP(hipMemcpyAsync(W.pinned, W.scal, 2 * sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
      // the next step's preconditioner needs only v_{j+1}: enqueued before
      // the wait for this step's residual estimates, so that the device has
      // work while the host tests them; not when every column is expected
      // to stop here (the estimate falling at its last rate to below twice
      // the tolerance, or the iteration limit)
      bool more = false;
      for (int k = 0; k < nrhs && !more; ++k) {
        if (!cyc[k]) continue;
        const double rate = res2[k] > 0.0 ? std::min(1.0, res1[k] / res2[k]) : 1.0;
        more = !(res1[k] * rate < 2.0 * so.rtol * beta0[k] || total[k] + 1 >= so.maxit);
      }
      if (j + 1 < m && more) {
        precond(C, W.V + (int64_t)(j + 1) * n, L.vs, flex ? W.Z + (int64_t)(j + 1) * n : W.z, ldz, nrhs, s, &W);
        z_ready = true;
      }
      NF_HIP(hipStreamSynchronize(s));
      bool changed = false;
      int left = 0;
      for (int k = 0; k < nrhs; ++k) {
        if (!cyc[k]) continue;
        ++total[k];
        je[k] = j + 1;
        const double hn = W.pinned[2 * k], res = W.pinned[2 * k + 1];
        if (hist) hist[k].push_back(res / beta0[k]);
        res2[k] = res1[k];
        res1[k] = res;
        if (!std::isfinite(res) || hn <= 1e-300 || res / beta0[k] < so.rtol || total[k] >= so.maxit) {
          if (hn <= 1e-300) broke[k] = 1;
          cyc[k] = 0;
          changed = true;
        } else {
          ++left;
        }
      }
      if (left == 0) break;
      if (changed) upload_ints(W, cyc, mask, s);
    }
    // end of the cycle: y = H^-1 g and the solution update for every column
    // that took part
    upload_ints(W, in_cycle, part, s);
    upload_ints(W, je, jend, s);
    int maxj = 0;
    for (int k = 0; k < nrhs; ++k) maxj = std::max(maxj, je[k]);
    backsolve(L, jend, W.H, W.g, W.y, part, s);
    if (flex) {
      mcombine(LZ, W.Z, jend, maxj, W.y, x, ldx, 1, part, s);
    } else {
      mcombine(L, W.V, jend, maxj, W.y, W.u, n, 0, part, s);
      precond(C, W.u, n, W.z, n, nrhs, s, &W);
      add_intom<double>(W.z, n, x, ldx, n, nrhs, part, s);
    }
  }
  for (int k = 0; k < nrhs; ++k) st[k].iters = total[k];
}

// host-side checks of one input block (before any device work)
static void validate_block(const nfield_csr& c, int nr, int nc) {
  NF_CHECK(c.nrows == nr && c.ncols == nc, NFIELD_EINVAL, "block dimensions disagree with the field sizes");
  NF_CHECK(c.rowptr && c.colind, NFIELD_EINVAL, "block: null rowptr / colind");
  NF_CHECK(c.rowptr[0] == 0 && c.rowptr[nr] == c.nnz, NFIELD_EINVAL, "block: rowptr inconsistent with nnz");
  NF_CHECK(c.nnz < INT32_MAX, NFIELD_ENOMEM, "block: more than 2^31 entries");
  for (int i = 0; i < nr; ++i) {
    NF_CHECK(c.rowptr[i + 1] >= c.rowptr[i], NFIELD_EINVAL, "block: rowptr decreasing");
    for (int64_t p = c.rowptr[i]; p < c.rowptr[i + 1]; ++p) {
      NF_CHECK(c.colind[p] >= 0 && c.colind[p] < nc, NFIELD_EINVAL, "block: column index out of range");
      NF_CHECK(p == c.rowptr[i] || c.colind[p] > c.colind[p - 1], NFIELD_EINVAL,
               "block: column indices not strictly increasing");
      NF_CHECK(std::isfinite(c.val[p]), NFIELD_EINVAL, "block: non-finite value");
    }
  }
}

static void upload_block(const nfield_csr& c, int nr, int nc, DCsr& D, hipStream_t s) {
  std::vector<int> ptr(nr + 1);
  for (int i = 0; i <= nr; ++i) ptr[i] = (int)c.rowptr[i];
  D.nr = nr;
  D.nc = nc;
  D.nnz = c.nnz;
  D.ptr.alloc(nr + 1);
  D.col.alloc(c.nnz > 0 ? c.nnz : 1);
  D.val.alloc(c.nnz > 0 ? c.nnz : 1);
  NF_HIP(hipMemcpyAsync(D.ptr.p, ptr.data(), sizeof(int) * (nr + 1), hipMemcpyHostToDevice, s));
  NF_HIP(hipMemcpyAsync(D.col.p, c.colind, sizeof(int) * c.nnz, hipMemcpyHostToDevice, s));
  NF_HIP(hipMemcpyAsync(D.val.p, c.val, sizeof(double) * c.nnz, hipMemcpyHostToDevice, s));
  NF_HIP(hipStreamSynchronize(s));
}

// all blocks merged into one CSR: block row i, blocks j ascending, column
// offsets of the fields; built on the host from the (validated) inputs
static void merge_global(const nfield_csr* blocks, int N, const std::vector<int>& size, DCsr& G,
                         std::vector<std::shared_ptr<DBuf<int>>>& gpos, hipStream_t s) {
  std::vector<int> o(N + 1, 0);
  for (int i = 0; i < N; ++i) o[i + 1] = o[i] + size[i];
  const int n = o[N];
  std::vector<int> ptr(n + 1, 0);
  int64_t nnz = 0;
  for (int i = 0; i < N; ++i)
    for (int r = 0; r < size[i]; ++r) {
      for (int j = 0; j < N; ++j) {
        const nfield_csr& c = blocks[(size_t)i * N + j];
        if (c.nnz == 0 || !c.val) continue;
        nnz += c.rowptr[r + 1] - c.rowptr[r];
      }
      ptr[o[i] + r + 1] = (int)nnz;
    }
  NF_CHECK(nnz < INT32_MAX, NFIELD_ENOMEM, "system has more than 2^31 entries");
  std::vector<int> col(nnz > 0 ? nnz : 1);
  std::vector<double> val(nnz > 0 ? nnz : 1);
  std::vector<std::vector<int>> pos((size_t)N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const nfield_csr& c = blocks[(size_t)i * N + j];
      if (c.nnz > 0 && c.val) pos[(size_t)i * N + j].resize(c.nnz);
    }
  int64_t q = 0;
  for (int i = 0; i < N; ++i)
    for (int r = 0; r < size[i]; ++r)
      for (int j = 0; j < N; ++j) {
        const nfield_csr& c = blocks[(size_t)i * N + j];
        if (c.nnz == 0 || !c.val) continue;
        for (int64_t p = c.rowptr[r]; p < c.rowptr[r + 1]; ++p) {
          col[q] = c.colind[p] + o[j];
          val[q] = c.val[p];
          pos[(size_t)i * N + j][p] = (int)q;
          ++q;
        }
      }
  gpos.assign((size_t)N * N, nullptr);
  for (size_t b = 0; b < pos.size(); ++b) {
    if (pos[b].empty()) continue;
    gpos[b] = std::make_shared<DBuf<int>>(pos[b].size());
    NF_HIP(hipMemcpyAsync(gpos[b]->p, pos[b].data(), sizeof(int) * pos[b].size(), hipMemcpyHostToDevice, s));
  }
  G.nr = G.nc = n;
  G.nnz = nnz;
  G.ptr.alloc(n + 1);
  G.col.alloc(col.size());
  G.val.alloc(val.size());
  NF_HIP(hipMemcpyAsync(G.ptr.p, ptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
  NF_HIP(hipMemcpyAsync(G.col.p, col.data(), sizeof(int) * col.size(), hipMemcpyHostToDevice, s));
  NF_HIP(hipMemcpyAsync(G.val.p, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, s));
  NF_HIP(hipStreamSynchronize(s));
}

// device bytes in live buffers of the context (its own pool and the side
// builds' pools)
static size_t tree_live(const nfield_ctx& C) {
  size_t b = C.pool.live;
  for (auto& sb : C.side) b += sb->pool.live;
  return b;
}

// (re)build the preconditioner tree from the device-resident blocks
__global__ void k_scatter_vals(const double* v, const int* pos, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[pos[i]] = v[i];
}
__global__ void k_gather_vals(const double* g, const int* pos, int64_t n, double* v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = g[pos[i]];
}

// set-up mode for the calling thread while in scope
struct SetupScope {
  bool prev;
  SetupScope() : prev(in_setup()) { setup_mode(true); }
  ~SetupScope() { setup_mode(prev); }
};

static void build_tree(nfield_ctx& C, hipStream_t s) {
  SetupScope scope;
  C.drop_graphs();
  C.root64.reset();
  C.root32.reset();
  C.hiers.clear();
  C.owned.clear();
  C.side_next = 0;
  g_hsink = &C.hiers;
  g_osink = &C.owned;
  g_mbuf_cols = C.o.max_rhs;
  if (C.inputs_dropped) {   // the input blocks' FP64 values, from the merged operator
    for (size_t k = 0; k < C.A.blk.size(); ++k) {
      DCsr* b = C.A.blk[k].get();
      if (!b || b->nnz == 0) continue;
      NF_CHECK(C.gpos[k] != nullptr, NFIELD_EINVAL, "rebuild: a block without its merged positions");
      b->val.alloc(b->nnz);
      hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((b->nnz + 255) / 256)), dim3(256), 0, s, C.Aglob.val.p,
                         C.gpos[k]->p, b->nnz, b->val.p);
    }
    NF_HIP(hipGetLastError());
    C.inputs_dropped = false;
  }
  for (auto& b : C.A.blk)   // FP32 and block copies of the inputs count as the tree's
    if (b) {
      b->val32.release();
      b->bsr_release();
    }
  const size_t live0 = tree_live(C);
  if (C.o.hier_fp32) {
    // FP32 copies of the input blocks are made where an FP32 solver reads them
    C.root32 = build<float>(C, C.spec, C.A, C.F, 0, C.N, s);
    // the FP32 tree runs on the FP32 copies alone: the FP64 values of the
    // matrices it built (coarse levels, transfers, Schur approximations)
    // are released; the input blocks keep theirs (rebuilds start there)
    NF_HIP(hipStreamSynchronize(s));
    for (auto& H : C.hiers)
      for (size_t l = 0; l < H->lev.size(); ++l) {
        Level& L = H->lev[l];
        if (l > 0)
          for (auto& b : L.A.blk)
            if (b && b->val32.p) b->val.free_now();
        for (auto& p : L.P) if (p && p->val32.p) p->val.free_now();
        for (auto& r : L.R) if (r && r->val32.p) r->val.free_now();
      }
    for (auto& B : C.owned)
      for (auto& b : B->blk)
        if (b && b->val32.p) b->val.free_now();
    C.tree_bytes = tree_live(C) - live0;
    // the input blocks' FP64 values are the merged operator's (which FP64
    // GMRES keeps): released, and gathered back from it at the next rebuild
    for (auto& b : C.A.blk)
      if (b && b->nnz > 0) b->val.free_now();
    C.inputs_dropped = true;
  } else {
    C.root64 = build<double>(C, C.spec, C.A, C.F, 0, C.N, s);
    C.tree_bytes = tree_live(C) - live0;
  }
}


// ------------------------------------------------ allocation-free workspace
// The Krylov workspace of nfield_gmres_solve_noalloc lives in this static
// device array (256 MiB on every device the library runs on, held until the
// process ends).  Host code never passes the array's name to a kernel or a
// copy: the address of each device's copy comes from hipGetSymbolAddress,
// taken once per device (with that device current) and kept here.
constexpr size_t SCRATCH_DOUBLES = (size_t)32 << 20;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

static double* scratch_on_current_device() {
  int dev = 0;
  NF_HIP(hipGetDevice(&dev));
  NF_CHECK(dev >= 0 && dev < SCRATCH_MAX_DEVICES, NFIELD_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    NF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    NF_CHECK(p != nullptr, NFIELD_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
    g_scratch_dev[dev] = (double*)p;
  }
  return g_scratch_dev[dev];
}

// Krylov workspace of nrhs columns carved from the scratch array, every
// region on a 256-byte boundary; host staging in the caller's arrays.
// size_only: check that the workspace fits (ENOMEM if not) and return.
static KrylovWs scratch_workspace(nfield_ctx& C, int m, int flexible, int nrhs, double* host_d, int* host_i,
                                  bool size_only) {
  const size_t n = (size_t)C.Aglob.nr, nr = (size_t)nrhs, mm = (size_t)m;
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t o = off;
    off += (doubles + 31) & ~(size_t)31;
    return o;
  };
  const size_t oV = take(n * (mm + 1) * nr), oZ = flexible ? take(n * mm * nr) : 0;
  const size_t ow = take(n * nr), oz = take(n * nr), orr = take(n * nr), ou = take(n * nr);
  const size_t oH = take((mm + 1) * mm * nr), ocs = take(mm * nr), osn = take(mm * nr), og = take((mm + 1) * nr);
  const size_t oy = take(mm * nr), oh1 = take((mm + 1) * nr), oh2 = take((mm + 1) * nr);
  const size_t op = take((size_t)RED_BLOCKS * (mm + 1) * nr), os = take(4 * NRMAX);
  const size_t oi = take((3 * NRMAX + 1) / 2);
  const bool f32 = C.root32 != nullptr;
  const size_t or32 = f32 ? take((n * nr + 1) / 2) : 0, oz32 = f32 ? take((n * nr + 1) / 2) : 0;
  NF_CHECK(off <= SCRATCH_DOUBLES, NFIELD_ENOMEM,
           "nfield_gmres_solve_noalloc: the Krylov workspace (" + std::to_string(off * 8) +
               " bytes) exceeds the static scratch of " + std::to_string(SCRATCH_DOUBLES * 8) + " bytes");
  KrylovWs W;
  if (size_only) return W;
  double* base = scratch_on_current_device();
  W.V = base + oV;
  W.Z = flexible ? base + oZ : nullptr;
  W.w = base + ow;
  W.z = base + oz;
  W.r = base + orr;
  W.u = base + ou;
  W.H = base + oH;
  W.cs = base + ocs;
  W.sn = base + osn;
  W.g = base + og;
  W.y = base + oy;
  W.h1 = base + oh1;
  W.h2 = base + oh2;
  W.partial = base + op;
  W.scal = base + os;
  W.imask = (int*)(base + oi);
  W.r32 = f32 ? (float*)(base + or32) : nullptr;
  W.z32 = f32 ? (float*)(base + oz32) : nullptr;
  W.pinned = host_d;
  W.pinned_i = host_i;
  W.direct = true;
  return W;
}

}  // namespace nf

// ============================================================ slot batches
// Iteration-level continuous batching.  A batch holds a fixed number of
// column slots, each running its own restarted GMRES process with the
// arithmetic of gmres() above (the same kernels per column, so a column's
// iterates are those of a solve of that column alone).  One step advances
// every running slot by one Arnoldi step in shared launches; at the step
// boundaries finished slots leave (their Krylov cycle ends, the solution is
// updated and the true residual decides) and new right-hand sides join.
// The preconditioner and the operator act on the running slots gathered into
// contiguous columns; the basis, Hessenberg and rotation state stay per slot,
// each slot at its own Arnoldi index.
enum SlotState { SLOT_FREE = 0, SLOT_START, SLOT_RUN, SLOT_END, SLOT_DONE };

struct nfield_batch {
  nfield_ctx* C = nullptr;
  int slots = 0, m = 0;
  bool flex = false;
  nfield_solve_opts so{};
  nf::GmresLayout L, LZ;
  // per slot: basis (m + 1 vectors), flexible basis (m), solution, rhs,
  // one work vector, the cycle-end combination; compact columns rc, zc, wc
  nf::DBuf<double> V, Z, X, Bv, Wsl, U, rc, zc, wc;
  nf::DBuf<double> H, cs, sn, g, y, h1, h2, partial, scal;
  nf::DBuf<int> ibuf;          // 3 phases x 5 slots ints
  double* pinned = nullptr;    // 4 slots doubles
  int* pinned_i = nullptr;     // 3 phases x 5 slots ints
  std::vector<int> state, j, total, fresh;
  std::vector<char> broke;
  std::vector<double> beta0;
  std::vector<nfield_stats> st;
  std::vector<std::chrono::steady_clock::time_point> t_submit;
  ~nfield_batch() {
    if (pinned) (void)hipHostFree(pinned);
    if (pinned_i) (void)hipHostFree(pinned_i);
  }
  // device and host int regions of one phase: [act | mask | jv | ncv | aux]
  int* dev_i(int phase) { return ibuf.p + (size_t)phase * 5 * slots; }
  int* host_i(int phase) { return pinned_i + (size_t)phase * 5 * slots; }
};

namespace nf {

static void batch_upload(nfield_batch& B, int phase, int regions, hipStream_t s) {
  NF_HIP(hipMemcpyAsync(B.dev_i(phase), B.host_i(phase), sizeof(int) * regions * B.slots, hipMemcpyHostToDevice, s));
}

// Cycle ends of the slots in SLOT_END: y = H^-1 g, x += Z y (flexible) or
// x += M^-1 (V y); the slots then wait for their true residual.
static void batch_cycle_ends(nfield_batch& B, hipStream_t s) {
  nfield_ctx& C = *B.C;
  const int64_t n = C.Aglob.nr;
  int* hi = B.host_i(0);
  int* act = hi;
  int* part = hi + B.slots;
  int* jend = hi + 2 * B.slots;
  int ne = 0, maxj = 0;
  for (int k = 0; k < B.slots; ++k) {
    const bool e = B.state[k] == SLOT_END;
    part[k] = e;
    jend[k] = e ? B.j[k] : 0;
    if (e) {
      act[ne++] = k;
      maxj = std::max(maxj, B.j[k]);
    }
  }
  if (ne == 0) return;
  batch_upload(B, 0, 3, s);
  int* dact = B.dev_i(0);
  int* dpart = dact + B.slots;
  int* djend = dact + 2 * B.slots;
  backsolve(B.L, djend, B.H.p, B.g.p, B.y.p, dpart, s);
  if (B.flex) {
    mcombine(B.LZ, B.Z.p, djend, maxj, B.y.p, B.X.p, n, 1, dpart, s);
  } else {
    mcombine(B.L, B.V.p, djend, maxj, B.y.p, B.U.p, n, 0, dpart, s);
    slot_gather(B.U.p, n, n, dact, nullptr, ne, B.rc.p, s);
    precond(C, B.rc.p, n, B.zc.p, n, ne, s);
    slot_scatter(B.zc.p, n, dact, nullptr, ne, B.U.p, n, s);
    add_intom<double>(B.U.p, n, B.X.p, n, n, B.slots, dpart, s);
  }
  for (int c = 0; c < ne; ++c) B.state[act[c]] = SLOT_START;
}

// True residuals of the slots in SLOT_START and the restart test; a slot
// that goes on starts a cycle: v_0 = r / beta, g = beta e_1.
static void batch_cycle_starts(nfield_batch& B, std::vector<int>& finished, hipStream_t s) {
  nfield_ctx& C = *B.C;
  const int64_t n = C.Aglob.nr;
  const nfield_solve_opts& so = B.so;
  int* act = B.host_i(1);
  int* mask = act + B.slots;
  int ns = 0;
  for (int k = 0; k < B.slots; ++k) {
    mask[k] = 0;
    if (B.state[k] == SLOT_START) act[ns++] = k;
  }
  if (ns == 0) return;
  batch_upload(B, 1, 1, s);
  int* dact = B.dev_i(1);
  int* dmask = dact + B.slots;
  slot_gather(B.X.p, n, n, dact, nullptr, ns, B.zc.p, s);
  slot_gather(B.Bv.p, n, n, dact, nullptr, ns, B.wc.p, s);
  SpmvArgs<double> a;
  a.x = B.zc.p;
  a.ldx = n;
  a.y = B.rc.p;
  a.ldy = n;
  a.b = B.wc.p;
  a.ldb = n;
  a.nrhs = ns;
  spmv<double>(SPMV_RESID, C.Aglob, a, s);
  dotm(B.rc.p, n, B.rc.p, n, n, ns, B.partial.p, B.scal.p, s);
  double* res = B.pinned;
  double* beta = B.pinned + B.slots;
  NF_HIP(hipMemcpyAsync(res, B.scal.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  int nbegin = 0;
  for (int c = 0; c < ns; ++c) {
    const int k = act[c];
    const double bk = std::sqrt(res[c]);
    nfield_stats& st = B.st[k];
    auto finish = [&](int status) {
      st.status = status;
      B.state[k] = SLOT_DONE;
      finished.push_back(k);
    };
    if (B.fresh[k]) {
      B.fresh[k] = 0;
      B.beta0[k] = bk;
      if (!std::isfinite(bk)) { finish(NFIELD_ENAN); continue; }
      if (bk == 0.0) { finish(NFIELD_OK); continue; }
    }
    st.relres = bk / B.beta0[k];
    if (!std::isfinite(bk)) { finish(NFIELD_ENAN); continue; }
    if (bk / B.beta0[k] < so.rtol) { finish(NFIELD_OK); continue; }
    if (B.broke[k]) { finish(NFIELD_EBREAKDOWN); continue; }
    if (B.total[k] >= so.maxit) { finish(NFIELD_NOT_CONVERGED); continue; }
    if (B.total[k] > 0) st.restarts++;
    mask[k] = 1;
    beta[k] = bk;
    B.j[k] = 0;
    B.state[k] = SLOT_RUN;
    ++nbegin;
  }
  if (nbegin == 0) return;
  batch_upload(B, 1, 2, s);   // the mask (and the same act list)
  double* dbeta = B.scal.p + 2 * B.slots;
  NF_HIP(hipMemcpyAsync(dbeta, beta, sizeof(double) * B.slots, hipMemcpyHostToDevice, s));
  slot_scatter(B.rc.p, n, dact, nullptr, ns, B.Wsl.p, n, s);
  scale_inv_devm(B.Wsl.p, n, B.V.p, B.L.vs, dbeta, 1, n, B.slots, dmask, s);
  hipLaunchKernelGGL(k_init_gm, dim3(B.slots), dim3(64), 0, s, B.g.p, B.m, dbeta, dmask);
}

// One Arnoldi step of every slot in SLOT_RUN, each at its own index j:
// z = M^-1 v_j, w = A z, two classical Gram-Schmidt passes over v_0..v_j,
// the Givens update and v_{j+1} = w / ||w||.
static void batch_arnoldi(nfield_batch& B, hipStream_t s) {
  nfield_ctx& C = *B.C;
  const int64_t n = C.Aglob.nr;
  const nfield_solve_opts& so = B.so;
  int* act = B.host_i(2);
  int* mask = act + B.slots;
  int* jv = act + 2 * B.slots;
  int* ncv = act + 3 * B.slots;
  int nr = 0, maxj = 0;
  for (int k = 0; k < B.slots; ++k) {
    const bool r = B.state[k] == SLOT_RUN;
    mask[k] = r;
    jv[k] = r ? B.j[k] : 0;
    ncv[k] = jv[k] + 1;
    if (r) {
      act[nr++] = k;
      maxj = std::max(maxj, B.j[k]);
    }
  }
  if (nr == 0) return;
  batch_upload(B, 2, 4, s);
  int* dact = B.dev_i(2);
  int* dmask = dact + B.slots;
  int* djv = dact + 2 * B.slots;
  int* dncv = dact + 3 * B.slots;
  slot_gather(B.V.p, B.L.vs, n, dact, djv, nr, B.rc.p, s);
  precond(C, B.rc.p, n, B.zc.p, n, nr, s);
  if (B.flex) slot_scatter(B.zc.p, n, dact, djv, nr, B.Z.p, B.LZ.vs, s);
  SpmvArgs<double> a;
  a.x = B.zc.p;
  a.ldx = n;
  a.y = B.wc.p;
  a.ldy = n;
  a.nrhs = nr;
  spmv<double>(SPMV_STORE, C.Aglob, a, s);
  slot_scatter(B.wc.p, n, dact, nullptr, nr, B.Wsl.p, n, s);
  const GmresLayout& L = B.L;
  const int nc = maxj + 1;
  mdot_partial(L, B.V.p, nc, B.Wsl.p, n, B.partial.p, dmask, s, dncv);
  mreduce(L, B.partial.p, nc, B.h1.p, 0, dmask, s, dncv);
  mupdate_dot(L, B.V.p, nc, B.h1.p, B.Wsl.p, n, B.partial.p, dmask, s, dncv);
  mreduce(L, B.partial.p, nc, B.h2.p, 0, dmask, s, dncv);
  mupdate_norm(L, B.V.p, nc, B.h2.p, B.Wsl.p, n, B.partial.p, dmask, s, dncv);
  givens_step(L, 0, B.h1.p, B.h2.p, B.partial.p, B.H.p, B.cs.p, B.sn.p, B.g.p, B.scal.p, dmask, s, djv);
  scale_inv_devm(B.Wsl.p, n, B.V.p + n, L.vs, B.scal.p, 2, n, B.slots, dmask, s, djv, n);
  double* hr = B.pinned + 2 * B.slots;
  NF_HIP(hipMemcpyAsync(hr, B.scal.p, 2 * sizeof(double) * B.slots, hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < nr; ++c) {
    const int k = act[c];
    ++B.total[k];
    ++B.j[k];
    const double hn = hr[2 * k], res = hr[2 * k + 1];
    if (!std::isfinite(res) || hn <= 1e-300 || res / B.beta0[k] < so.rtol || B.total[k] >= so.maxit || B.j[k] == B.m) {
      if (hn <= 1e-300) B.broke[k] = 1;
      B.state[k] = SLOT_END;
    }
  }
}

}  // namespace nf

// ================================================================ C ABI
using namespace nf;

static nfield_status fail(const NfError& e) {
  g_err = e.what();
  return (nfield_status)e.code;
}

extern "C" {

void nfield_default_opts(nfield_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->sweeps = 1;
  o->order = 1;
  o->coarse_max = 200;
  o->max_levels = 10;
  o->cheb_degree = 2;
  o->power_its = 10;
  o->cheb_ratio = 30.0;
  o->cheb_boost = 1.1;
  o->simplec_mode = 0;
  o->split = nullptr;
  o->schur_direct_max = 5000;
  o->hier_fp32 = 0;
  o->seed = 0;
  o->graphs = 0;
  o->block_products = 1;
  o->parallel_setup = 1;
  o->max_rhs = NRMAX;
}

void nfield_default_solve_opts(nfield_solve_opts* so) {
  so->restart = 50;
  so->maxit = 1000;
  so->flexible = 0;
  so->rtol = 1e-8;
}

const char* nfield_last_error(void) { return g_err.c_str(); }

const char* nfield_strerror(nfield_status s) {
  switch (s) {
    case NFIELD_OK: return "ok";
    case NFIELD_NOT_CONVERGED: return "not converged";
    case NFIELD_EINVAL: return "invalid argument";
    case NFIELD_ENOMEM: return "out of memory or size limit";
    case NFIELD_ESINGULAR: return "singular block or pivot";
    case NFIELD_EBREAKDOWN: return "Krylov breakdown";
    case NFIELD_ENAN: return "non-finite value";
    case NFIELD_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

nfield_status nfield_setup(int32_t nfields, const nfield_field* fields, const nfield_csr* blocks, const char* spec,
                           const nfield_opts* opts, void* hip_stream, nfield_ctx** out) {
  if (!out || !fields || !blocks || !spec || nfields < 1) {
    g_err = "nfield_setup: null argument or no fields";
    return NFIELD_EINVAL;
  }
  *out = nullptr;
  hipStream_t s = (hipStream_t)hip_stream;
  auto C = std::make_unique<nfield_ctx>();
  DevPool* prev = g_pool;
  g_pool = &C->pool;
  C->pool.enter(s);
  try {
    const auto t0 = std::chrono::steady_clock::now();
    nfield_opts od;
    nfield_default_opts(&od);
    const nfield_opts& o = opts ? *opts : od;
    C->o.sweeps = o.sweeps;
    C->o.order = o.order;
    C->o.coarse_max = o.coarse_max;
    C->o.max_levels = o.max_levels;
    C->o.cheb_degree = o.cheb_degree;
    C->o.power_its = o.power_its;
    C->o.cheb_ratio = o.cheb_ratio;
    C->o.cheb_boost = o.cheb_boost;
    C->o.simplec_mode = o.simplec_mode;
    if (o.split) C->o.split.assign(o.split, o.split + nfields);
    C->o.schur_direct_max = o.schur_direct_max;
    C->o.hier_fp32 = o.hier_fp32;
    C->o.seed = o.seed;
    C->o.graphs = o.graphs;
    C->o.block_products = o.block_products;
    C->o.parallel_setup = o.parallel_setup;
    C->o.max_rhs = o.max_rhs;
    NF_CHECK(o.sweeps >= 1 && o.order >= 0 && o.order <= 2 && o.cheb_degree >= 1 && o.max_levels >= 1 &&
                 o.cheb_ratio > 1.0 && o.cheb_boost > 0.0 && o.simplec_mode >= 0 && o.simplec_mode <= 2 &&
                 o.max_rhs >= 1 && o.max_rhs <= NRMAX,
             NFIELD_EINVAL, "options out of range");
    C->N = nfields;
    C->A.N = nfields;
    C->A.size.resize(nfields);
    C->A.blk.resize((size_t)nfields * nfields);
    for (int i = 0; i < nfields; ++i) {
      const nfield_field& f = fields[i];
      NF_CHECK(f.ndof > 0 && f.block_size > 0 && f.ndof % f.block_size == 0 && f.nns >= 0, NFIELD_EINVAL,
               "field description");
      C->A.size[i] = f.ndof;
    }
    for (int i = 0; i < nfields; ++i)
      for (int j = 0; j < nfields; ++j) {
        const nfield_csr& c = blocks[(size_t)i * nfields + j];
        if (c.nnz == 0 || c.val == nullptr) continue;
        validate_block(c, C->A.size[i], C->A.size[j]);
      }
    const Spec sp = parse_spec(spec);
    check_spec(sp);
    for (int i = 0; i < nfields; ++i) {
      const nfield_field& f = fields[i];
      FieldDev fd;
      fd.ndof = f.ndof;
      fd.bs = f.block_size;
      fd.nns = f.nns;
      if (f.nns > 0 && f.nullspace) {
        fd.B = std::make_shared<DBuf<double>>((size_t)f.ndof * f.nns);
        NF_HIP(hipMemcpyAsync(fd.B->p, f.nullspace, sizeof(double) * f.ndof * f.nns, hipMemcpyHostToDevice, s));
      }
      C->F.push_back(fd);
      C->A.size[i] = f.ndof;
    }
    for (int i = 0; i < nfields; ++i)
      for (int j = 0; j < nfields; ++j) {
        const nfield_csr& c = blocks[(size_t)i * nfields + j];
        if (c.nnz == 0 || c.val == nullptr) continue;
        auto D = std::make_shared<DCsr>();
        upload_block(c, C->A.size[i], C->A.size[j], *D, s);
        C->A.blk[(size_t)i * nfields + j] = D;
      }
    merge_global(blocks, nfields, C->A.size, C->Aglob, C->gpos, s);
    C->spec = sp;
    build_tree(*C, s);
    NF_HIP(hipStreamSynchronize(s));
    NF_HIP(hipGetLastError());
    C->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    g_pool = prev;
    *out = C.release();
    return NFIELD_OK;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  } catch (std::exception& e) {
    g_pool = prev;
    g_err = e.what();
    return NFIELD_ENOMEM;
  }
}

void nfield_destroy(nfield_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

size_t nfield_footprint_bytes(const nfield_ctx* ctx) {
  if (!ctx) return 0;
  size_t b = ctx->pool.live + ctx->pool.cached;
  for (auto& sb : ctx->side) b += sb->pool.live + sb->pool.cached;
  return b;
}
int64_t nfield_size(const nfield_ctx* ctx) { return ctx ? ctx->Aglob.nr : 0; }
size_t nfield_precond_bytes(const nfield_ctx* ctx) { return ctx ? ctx->tree_bytes : 0; }

nfield_status nfield_precond_apply(nfield_ctx* ctx, const double* r, double* z, int32_t nrhs, void* hip_stream) {
  if (!ctx || !r || !z || nrhs < 0) { g_err = "nfield_precond_apply: bad argument"; return NFIELD_EINVAL; }
  hipStream_t s = (hipStream_t)hip_stream;
  DevPool* prev = g_pool;
  g_pool = &ctx->pool;
  ctx->pool.enter(s);
  try {
    const int64_t n = ctx->Aglob.nr;
    const int cols = ctx->o.max_rhs;
    for (int k = 0; k < nrhs; k += cols) {
      const int nb = std::min(cols, nrhs - k);
      precond(*ctx, r + k * n, n, z + k * n, n, nb, s);
    }
    NF_HIP(hipGetLastError());
    g_pool = prev;
    return NFIELD_OK;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  }
}

nfield_status nfield_matvec(nfield_ctx* ctx, const double* x, double* y, int32_t nrhs, void* hip_stream) {
  if (!ctx || !x || !y || nrhs < 0) { g_err = "nfield_matvec: bad argument"; return NFIELD_EINVAL; }
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    const int64_t n = ctx->Aglob.nr;
    for (int k = 0; k < nrhs; k += NRMAX) {
      SpmvArgs<double> a;
      a.x = x + k * n;
      a.ldx = n;
      a.y = y + k * n;
      a.ldy = n;
      a.nrhs = std::min(NRMAX, nrhs - k);
      spmv<double>(SPMV_STORE, ctx->Aglob, a, s);
    }
    NF_HIP(hipGetLastError());
    return NFIELD_OK;
  } catch (NfError& e) {
    return fail(e);
  }
}

static nfield_status gmres_entry(nfield_ctx* ctx, const double* b, double* x, int32_t nrhs, const nfield_solve_opts* sopts,
                                 nfield_stats* stats, void* hip_stream, bool noalloc) {
  const char* who = noalloc ? "nfield_gmres_solve_noalloc" : "nfield_gmres_solve";
  if (!ctx || !b || !x || nrhs < 0) { g_err = std::string(who) + ": bad argument"; return NFIELD_EINVAL; }
  nfield_solve_opts so;
  nfield_default_solve_opts(&so);
  if (sopts) so = *sopts;
  if (so.restart < 1 || so.restart > 63 || so.maxit < 0 || !(so.rtol > 0)) {
    g_err = std::string(who) + ": restart must be in [1, 63], maxit >= 0, rtol > 0";
    return NFIELD_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  DevPool* prev = g_pool;
  g_pool = &ctx->pool;
  ctx->pool.enter(s);
  try {
    const int64_t n = ctx->Aglob.nr;
    int worst = NFIELD_OK;
    std::vector<nfield_stats> st(NRMAX);
    double host_d[64];   // staging of the allocation-free path (pageable)
    int host_i[64];
    const int cols = ctx->o.max_rhs;   // columns per batch: what the preconditioner's temporaries hold
    if (noalloc && nrhs > 0) (void)scratch_workspace(*ctx, so.restart, so.flexible, std::min(cols, nrhs), nullptr,
                                                     nullptr, true);   // size check first
    for (int k = 0; k < nrhs; k += cols) {
      const int nb = std::min(cols, nrhs - k);
      const auto t0 = std::chrono::steady_clock::now();
      const double b0 = bytes_counted();
      if (k == 0) ctx->hist.assign(nrhs, {});
      const KrylovWs W = noalloc ? scratch_workspace(*ctx, so.restart, so.flexible, nb, host_d, host_i, false)
                                 : ctx_workspace(*ctx, so.restart, so.flexible, nb);
      gmres(*ctx, W, b + k * n, n, x + k * n, n, nb, so, st.data(), s, ctx->hist.data() + k);
      NF_HIP(hipStreamSynchronize(s));
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      const double bytes = bytes_counted() - b0;
      for (int q = 0; q < nb; ++q) {
        st[q].solve_s = dt;
        st[q].setup_s = ctx->setup_s;
        st[q].bytes = bytes;
        st[q].gbps = dt > 0.0 ? bytes / dt * 1e-9 : 0.0;
        if (stats) stats[k + q] = st[q];
        if (st[q].status < 0) worst = std::min(worst, st[q].status);
        else if (worst >= 0 && st[q].status > worst) worst = st[q].status;
      }
    }
    g_pool = prev;
    if (worst == NFIELD_ENAN) g_err = std::string(who) + ": non-finite value in the right-hand side or the iteration";
    else if (worst == NFIELD_EBREAKDOWN)
      g_err = std::string(who) + ": Krylov breakdown (the preconditioned operator is singular on the Krylov space) "
                                 "and the true residual is above rtol";
    else if (worst == NFIELD_NOT_CONVERGED) g_err = std::string(who) + ": iteration limit reached above rtol";
    return (nfield_status)worst;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  }
}

nfield_status nfield_gmres_solve(nfield_ctx* ctx, const double* b, double* x, int32_t nrhs, const nfield_solve_opts* sopts,
                                 nfield_stats* stats, void* hip_stream) {
  return gmres_entry(ctx, b, x, nrhs, sopts, stats, hip_stream, false);
}

nfield_status nfield_gmres_solve_noalloc(nfield_ctx* ctx, const double* b, double* x, int32_t nrhs,
                                         const nfield_solve_opts* sopts, nfield_stats* stats, void* hip_stream) {
  return gmres_entry(ctx, b, x, nrhs, sopts, stats, hip_stream, true);
}

nfield_status nfield_batch_create(nfield_ctx* ctx, int32_t slots, const nfield_solve_opts* sopts, nfield_batch** out) {
  if (!ctx || !out || slots < 1 || slots > NRMAX || slots > ctx->o.max_rhs) {
    g_err = "nfield_batch_create: bad argument (slots must be in [1, max_rhs])";
    return NFIELD_EINVAL;
  }
  *out = nullptr;
  nfield_solve_opts so;
  nfield_default_solve_opts(&so);
  if (sopts) so = *sopts;
  if (so.restart < 1 || so.restart > 63 || so.maxit < 0 || !(so.rtol > 0)) {
    g_err = "nfield_batch_create: restart must be in [1, 63], maxit >= 0, rtol > 0";
    return NFIELD_EINVAL;
  }
  DevPool* prev = g_pool;
  g_pool = &ctx->pool;
  try {
    auto B = std::make_unique<nfield_batch>();
    const int64_t n = ctx->Aglob.nr;
    const int m = so.restart;
    const size_t sl = (size_t)slots;
    B->C = ctx;
    B->slots = slots;
    B->m = m;
    B->flex = so.flexible != 0;
    B->so = so;
    B->L.n = n;
    B->L.vs = (int64_t)(m + 1) * n;
    B->L.hs = m + 1;
    B->L.ps = (int64_t)(m + 1) * RED_BLOCKS;
    B->L.m = m;
    B->L.nrhs = slots;
    B->LZ = B->L;
    B->LZ.vs = (int64_t)m * n;
    B->V.alloc((size_t)n * (m + 1) * sl);
    if (B->flex) B->Z.alloc((size_t)n * m * sl);
    else B->U.alloc((size_t)n * sl);
    for (DBuf<double>* d : {&B->X, &B->Bv, &B->Wsl, &B->rc, &B->zc, &B->wc}) d->alloc((size_t)n * sl);
    B->H.alloc((size_t)(m + 1) * m * sl);
    B->cs.alloc((size_t)m * sl);
    B->sn.alloc((size_t)m * sl);
    B->g.alloc((size_t)(m + 1) * sl);
    B->y.alloc((size_t)m * sl);
    B->h1.alloc((size_t)(m + 1) * sl);
    B->h2.alloc((size_t)(m + 1) * sl);
    B->partial.alloc((size_t)RED_BLOCKS * (m + 1) * sl);
    B->scal.alloc(4 * sl);
    B->ibuf.alloc(15 * sl);
    NF_HIP(hipHostMalloc((void**)&B->pinned, 4 * sl * sizeof(double), hipHostMallocDefault));
    NF_HIP(hipHostMalloc((void**)&B->pinned_i, 15 * sl * sizeof(int), hipHostMallocDefault));
    B->state.assign(sl, SLOT_FREE);
    B->j.assign(sl, 0);
    B->total.assign(sl, 0);
    B->fresh.assign(sl, 0);
    B->broke.assign(sl, 0);
    B->beta0.assign(sl, 0.0);
    B->st.assign(sl, nfield_stats{});
    B->t_submit.assign(sl, {});
    g_pool = prev;
    *out = B.release();
    return NFIELD_OK;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  }
}

nfield_status nfield_batch_submit(nfield_batch* B, int32_t slot, const double* b, const double* x0, void* hip_stream) {
  if (!B || !b || slot < 0 || slot >= B->slots || B->state[slot] != SLOT_FREE) {
    g_err = "nfield_batch_submit: bad argument or the slot is not free";
    return NFIELD_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    const int64_t n = B->C->Aglob.nr;
    double* xs = B->X.p + (int64_t)slot * n;
    NF_HIP(hipMemcpyAsync(B->Bv.p + (int64_t)slot * n, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (x0) NF_HIP(hipMemcpyAsync(xs, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else NF_HIP(hipMemsetAsync(xs, 0, sizeof(double) * n, s));
    B->state[slot] = SLOT_START;
    B->fresh[slot] = 1;
    B->j[slot] = 0;
    B->total[slot] = 0;
    B->broke[slot] = 0;
    B->beta0[slot] = 0.0;
    std::memset(&B->st[slot], 0, sizeof(nfield_stats));
    B->t_submit[slot] = std::chrono::steady_clock::now();
    return NFIELD_OK;
  } catch (NfError& e) {
    return fail(e);
  }
}

nfield_status nfield_batch_step(nfield_batch* B, int32_t* done, int32_t* ndone, int32_t* nactive, void* hip_stream) {
  if (!B) { g_err = "nfield_batch_step: null batch"; return NFIELD_EINVAL; }
  hipStream_t s = (hipStream_t)hip_stream;
  nfield_ctx& C = *B->C;
  DevPool* prev = g_pool;
  g_pool = &C.pool;
  C.pool.enter(s);
  try {
    std::vector<int> finished;
    batch_cycle_ends(*B, s);
    batch_cycle_starts(*B, finished, s);
    batch_arnoldi(*B, s);
    // the host staging of this step is rewritten by the next one
    NF_HIP(hipStreamSynchronize(s));
    NF_HIP(hipGetLastError());
    const auto now = std::chrono::steady_clock::now();
    for (int k : finished) {
      B->st[k].iters = B->total[k];
      B->st[k].setup_s = C.setup_s;
      B->st[k].solve_s = std::chrono::duration<double>(now - B->t_submit[k]).count();
    }
    if (done)
      for (size_t q = 0; q < finished.size(); ++q) done[q] = finished[q];
    if (ndone) *ndone = (int32_t)finished.size();
    int live = 0;
    for (int k = 0; k < B->slots; ++k) live += B->state[k] == SLOT_START || B->state[k] == SLOT_RUN ||
                                             B->state[k] == SLOT_END;
    if (nactive) *nactive = live;
    g_pool = prev;
    return NFIELD_OK;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  }
}

nfield_status nfield_batch_take(nfield_batch* B, int32_t slot, double* x, nfield_stats* stats, void* hip_stream) {
  if (!B || slot < 0 || slot >= B->slots || B->state[slot] != SLOT_DONE) {
    g_err = "nfield_batch_take: bad argument or the slot has not finished";
    return NFIELD_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    const int64_t n = B->C->Aglob.nr;
    if (x) NF_HIP(hipMemcpyAsync(x, B->X.p + (int64_t)slot * n, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (stats) *stats = B->st[slot];
    B->state[slot] = SLOT_FREE;
    return NFIELD_OK;
  } catch (NfError& e) {
    return fail(e);
  }
}

int32_t nfield_batch_state(const nfield_batch* B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->slots) return -1;
  return B->state[slot];
}

size_t nfield_batch_bytes(const nfield_batch* B) {
  if (!B) return 0;
  size_t b = 0;
  for (const DBuf<double>* d : {&B->V, &B->Z, &B->X, &B->Bv, &B->Wsl, &B->U, &B->rc, &B->zc, &B->wc, &B->H, &B->cs,
                                &B->sn, &B->g, &B->y, &B->h1, &B->h2, &B->partial, &B->scal})
    b += d->n * sizeof(double);
  return b + B->ibuf.n * sizeof(int);
}

void nfield_batch_destroy(nfield_batch* B) {
  delete B;
}

nfield_status nfield_update_values(nfield_ctx* ctx, int32_t i, int32_t j, const double* val, int32_t on_device,
                                   void* hip_stream) {
  if (!ctx || !val || i < 0 || j < 0 || i >= ctx->N || j >= ctx->N || !ctx->A.at(i, j)) {
    g_err = "nfield_update_values: bad argument or zero block";
    return NFIELD_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    DCsr& B = *ctx->A.blk[(size_t)i * ctx->N + j];
    // with the FP32 tree the block holds no FP64 values: the new ones go
    // through a buffer of their own into the merged operator alone
    DevPool* prev = g_pool;
    g_pool = &ctx->pool;
    DBuf<double> tmp;
    if (ctx->inputs_dropped && B.nnz > 0) tmp.alloc(B.nnz);
    g_pool = prev;
    double* dst = ctx->inputs_dropped ? tmp.p : B.val.p;
    NF_HIP(hipMemcpyAsync(dst, val, sizeof(double) * B.nnz, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    const auto& pos = ctx->gpos[(size_t)i * ctx->N + j];
    if (B.nnz > 0)
      hipLaunchKernelGGL(k_scatter_vals, dim3((unsigned)((B.nnz + 255) / 256)), dim3(256), 0, s, dst, pos->p, B.nnz,
                         ctx->Aglob.val.p);
    NF_HIP(hipGetLastError());
    if (!on_device || tmp.p) NF_HIP(hipStreamSynchronize(s));
    if (tmp.p) tmp.free_now();
    return NFIELD_OK;
  } catch (NfError& e) {
    return fail(e);
  }
}

nfield_status nfield_rebuild(nfield_ctx* ctx, void* hip_stream) {
  if (!ctx) { g_err = "nfield_rebuild: null context"; return NFIELD_EINVAL; }
  hipStream_t s = (hipStream_t)hip_stream;
  DevPool* prev = g_pool;
  g_pool = &ctx->pool;
  ctx->pool.enter(s);
  try {
    const auto t0 = std::chrono::steady_clock::now();
    build_tree(*ctx, s);
    NF_HIP(hipStreamSynchronize(s));
    NF_HIP(hipGetLastError());
    ctx->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    g_pool = prev;
    return NFIELD_OK;
  } catch (NfError& e) {
    g_pool = prev;
    return fail(e);
  }
}

void nfield_prof_enable(int32_t on) {
  try { prof_enable(on); } catch (NfError& e) { g_err = e.what(); }
}

int32_t nfield_prof_read(int32_t max, int32_t* key, int64_t* count, double* ms, double* bytes) {
  try { return prof_read(max, key, count, ms, bytes); } catch (NfError& e) { g_err = e.what(); return -1; }
}

// ---------------------------------------------------------------- inspection
int32_t nfield_hier_count(const nfield_ctx* c) { return c ? (int32_t)c->hiers.size() : 0; }
int32_t nfield_hier_nlevels(const nfield_ctx* c, int32_t h) { return (int32_t)c->hiers[h]->lev.size(); }
int32_t nfield_hier_nfields(const nfield_ctx* c, int32_t h) { return c->hiers[h]->N; }
int32_t nfield_hier_size(const nfield_ctx* c, int32_t h, int32_t l, int32_t f) { return c->hiers[h]->lev[l].A.size[f]; }
double nfield_hier_lambda(const nfield_ctx* c, int32_t h, int32_t l, int32_t f) {
  const Level& L = c->hiers[h]->lev[l];
  return f < (int)L.lambda.size() ? L.lambda[f] : 0.0;
}

int64_t nfield_hier_matrix(const nfield_ctx* c, int32_t h, int32_t l, int32_t which, int32_t i, int32_t j, int64_t* rowptr,
                           int32_t* colind, double* val, int32_t* nrows, int32_t* ncols) {
  try {
    const Level& L = c->hiers[h]->lev[l];
    const DCsr* M = nullptr;
    if (which == 0) M = L.A.at(i, j);
    else if (which == 1 && i < (int)L.P.size()) M = L.P[i].get();
    else if (which == 2 && i < (int)L.R.size()) M = L.R[i].get();
    if (!M) return -1;
    if (nrows) *nrows = M->nr;
    if (ncols) *ncols = M->nc;
    NF_HIP(hipDeviceSynchronize());
    if (rowptr) {
      std::vector<int> p(M->nr + 1);
      NF_HIP(hipMemcpy(p.data(), M->ptr.p, sizeof(int) * (M->nr + 1), hipMemcpyDeviceToHost));
      for (int r = 0; r <= M->nr; ++r) rowptr[r] = p[r];
    }
    if (colind && M->nnz) NF_HIP(hipMemcpy(colind, M->col.p, sizeof(int) * M->nnz, hipMemcpyDeviceToHost));
    if (val && M->nnz) {
      if (M->val.p) {
        NF_HIP(hipMemcpy(val, M->val.p, sizeof(double) * M->nnz, hipMemcpyDeviceToHost));
      } else {   // a precision-form matrix keeps its FP32 values only
        std::vector<float> v32(M->nnz);
        NF_HIP(hipMemcpy(v32.data(), M->val32.p, sizeof(float) * M->nnz, hipMemcpyDeviceToHost));
        for (int64_t q = 0; q < M->nnz; ++q) val[q] = v32[q];
      }
    }
    return M->nnz;
  } catch (NfError& e) {
    g_err = e.what();
    return -2;
  }
}

int64_t nfield_hier_nnz(const nfield_ctx* c, int32_t h, int32_t l) {
  if (!c || h < 0 || h >= (int)c->hiers.size() || l < 0 || l >= (int)c->hiers[h]->lev.size()) return -1;
  int64_t t = 0;
  for (const auto& b : c->hiers[h]->lev[l].A.blk)
    if (b) t += b->nnz;
  return t;
}

static double hier_complexity(const nfield_ctx* c, int32_t h, bool op) {
  if (!c || h < 0 || h >= (int)c->hiers.size() || c->hiers[h]->lev.empty()) return 0.0;
  double t = 0.0, t0 = 0.0;
  for (size_t l = 0; l < c->hiers[h]->lev.size(); ++l) {
    const double v = op ? (double)nfield_hier_nnz(c, h, (int32_t)l) : (double)c->hiers[h]->lev[l].A.total();
    if (l == 0) t0 = v;
    t += v;
  }
  return t0 > 0.0 ? t / t0 : 0.0;
}
double nfield_hier_op_complexity(const nfield_ctx* c, int32_t h) { return hier_complexity(c, h, true); }
double nfield_hier_grid_complexity(const nfield_ctx* c, int32_t h) { return hier_complexity(c, h, false); }

int32_t nfield_residual_history(const nfield_ctx* c, int32_t col, double* out, int32_t max) {
  if (!c || col < 0 || col >= (int)c->hist.size()) return -1;
  const auto& v = c->hist[col];
  if (out)
    for (int32_t i = 0; i < max && i < (int32_t)v.size(); ++i) out[i] = v[i];
  return (int32_t)v.size();
}

int32_t nfield_hier_aggregates(const nfield_ctx* c, int32_t h, int32_t l, int32_t f, int32_t* agg) {
  const Level& L = c->hiers[h]->lev[l];
  if (f >= (int)L.agg.size() || !L.agg[f]) return -1;
  const int nn = L.A.size[f] / L.bs[f];
  if (agg) {
    if (hipDeviceSynchronize() != hipSuccess) return -2;
    if (hipMemcpy(agg, L.agg[f]->p, sizeof(int) * nn, hipMemcpyDeviceToHost) != hipSuccess) return -2;
  }
  return nn;
}

}  // extern "C"

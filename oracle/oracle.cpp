// Serial FP64 CPU oracle for the n-field block preconditioners and GMRES.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU library is checked against.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg load it.  It shares no code, header, helper or
// table with the GPU library, and the GPU library never calls it.
//
// What it follows (Verdugo & Wall, "Unified computational framework for the
// efficient solution of n-field coupled problems with monolithic schemes"):
//   * the N x N block system with possibly zero blocks ........ Sec. 4, eq. (the-blocked-system)
//   * right preconditioning, x = P y with (A P) y = b ......... Sec. 3.2
//   * GMRES as the accelerator ................................ Sec. 3.1
//   * multigrid V-cycle ....................................... Sec. 3.3, Algorithm 1
//   * Galerkin coarse operators A^{l+1} = R A P ............... Sec. 3.3
//   * block Gauss-Seidel (fwd / bwd / sym), increment form .... Sec. 4.1, BGS iteration
//   * SIMPLE matrix form, SIMPLEC diagonal, block merging ..... Sec. 4.2
//   * monolithic AMG: block-diagonal transfers, R_i A_ij P_j,
//     BGS / SIMPLE level smoothers ............................ Sec. 4.3
//   * nesting of the three methods ............................ Sec. 5
// The paper treats the single-field AMG as a black box ("standard smoothed
// aggregation").  The choices made for it here (pattern-only node graph,
// synchronous MIS-2 with splitmix64 keys, MGS tentative prolongator, 10 seeded
// power iterations, damping 4/(3 lambda), degree-2 Chebyshev on
// [lambda/30, 1.1 lambda], dense LU on the coarsest level) are stated where
// they are made.  splitmix64 is the generator of Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014.
//
// Every sparse matrix is CSR with strictly increasing column indices per row.
// Sparse products keep every entry of the structural product (explicit zeros
// from cancellation stay), so patterns are a function of patterns alone.

#include <algorithm>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace orc {

enum Status { OK = 0, NOT_CONVERGED = 1, EINVAL_ = -1, ENOMEM_ = -2, ESINGULAR = -3,
              EBREAKDOWN = -4, ENAN = -5 };

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ----------------------------------------------------------------- sparse
struct Csr {
  int nr = 0, nc = 0;
  std::vector<int64_t> ptr;
  std::vector<int> col;
  std::vector<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr[nr]; }
};

static Csr identity(int n) {
  Csr I;
  I.nr = I.nc = n;
  I.ptr.resize(n + 1);
  I.col.resize(n);
  I.val.assign(n, 1.0);
  for (int i = 0; i <= n; ++i) I.ptr[i] = i;
  for (int i = 0; i < n; ++i) I.col[i] = i;
  return I;
}

// y = A x
static void spmv(const Csr& A, const double* x, double* y) {
  for (int i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
    y[i] = s;
  }
}

// y += A x
static void spmv_add(const Csr& A, const double* x, double* y) {
  for (int i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
    y[i] += s;
  }
}

static Csr transpose(const Csr& A) {
  Csr T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.ptr.assign(T.nr + 1, 0);
  for (int64_t p = 0; p < A.nnz(); ++p) T.ptr[A.col[p] + 1]++;
  for (int i = 0; i < T.nr; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int64_t> next(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < A.nr; ++i)           // rows ascending -> columns of T sorted
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int64_t q = next[A.col[p]]++;
      T.col[q] = i;
      T.val[q] = A.val[p];
    }
  return T;
}

// C = A * B (Gustavson, row by row; each entry sums a_ik b_kj in ascending k)
static Csr spgemm(const Csr& A, const Csr& B) {
  if (A.nc != B.nr) throw Error(EINVAL_, "spgemm: inner dimensions differ");
  Csr C;
  C.nr = A.nr;
  C.nc = B.nc;
  C.ptr.assign(C.nr + 1, 0);
  std::vector<int> mark(B.nc, -1);
  std::vector<double> acc(B.nc, 0.0);
  std::vector<int> cols;
  for (int i = 0; i < A.nr; ++i) {
    cols.clear();
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int k = A.col[p];
      double a = A.val[p];
      for (int64_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
        int j = B.col[q];
        if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols.push_back(j); }
        acc[j] += a * B.val[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int j : cols) { C.col.push_back(j); C.val.push_back(acc[j]); }
    C.ptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

// C = alpha*A + beta*B on the union pattern
static Csr add(double alpha, const Csr& A, double beta, const Csr& B) {
  if (A.nr != B.nr || A.nc != B.nc) throw Error(EINVAL_, "add: shapes differ");
  Csr C;
  C.nr = A.nr;
  C.nc = A.nc;
  C.ptr.assign(C.nr + 1, 0);
  for (int i = 0; i < A.nr; ++i) {
    int64_t p = A.ptr[i], pe = A.ptr[i + 1], q = B.ptr[i], qe = B.ptr[i + 1];
    while (p < pe || q < qe) {
      int ca = p < pe ? A.col[p] : INT32_MAX;
      int cb = q < qe ? B.col[q] : INT32_MAX;
      if (ca == cb) { C.col.push_back(ca); C.val.push_back(alpha * A.val[p] + beta * B.val[q]); ++p; ++q; }
      else if (ca < cb) { C.col.push_back(ca); C.val.push_back(alpha * A.val[p]); ++p; }
      else { C.col.push_back(cb); C.val.push_back(beta * B.val[q]); ++q; }
    }
    C.ptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

static void scale_rows(Csr& A, const std::vector<double>& s) {
  for (int i = 0; i < A.nr; ++i)
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) A.val[p] *= s[i];
}

static std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d(A.nr, 0.0);
  for (int i = 0; i < A.nr; ++i)
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
      if (A.col[p] == i) d[i] = A.val[p];
  return d;
}

static double dot(int n, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}
static double nrm2(int n, const double* a) { return std::sqrt(dot(n, a, a)); }

// -------------------------------------------------------------- splitmix64
// Steele, Lea & Flood (OOPSLA 2014): state += golden gamma, then the mix.
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// ---------------------------------------------------------- aggregation
// Node graph of a field with block size b: node u owns dofs [b u, b u + b);
// u ~ v (u != v) iff some stored entry couples a dof of u with a dof of v,
// in either direction (entry (u, v) or (v, u)): the graph of the pattern of
// A + A^T, so that the relation is symmetric even when the pattern is not.
// Strength threshold 0: every stored connection counts (the paper is silent).
struct Graph {
  int n = 0;
  std::vector<int64_t> ptr;
  std::vector<int> adj;
};

static Graph node_graph(const Csr& A, int b) {
  if (A.nr != A.nc || A.nr % b) throw Error(EINVAL_, "node_graph: size not a multiple of block size");
  Graph G;
  G.n = A.nr / b;
  G.ptr.assign(G.n + 1, 0);
  std::vector<std::vector<int>> nb(G.n);
  for (int u = 0; u < G.n; ++u)
    for (int r = b * u; r < b * u + b; ++r)
      for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
        const int v = A.col[p] / b;
        if (v == u) continue;
        nb[u].push_back(v);
        nb[v].push_back(u);
      }
  for (int u = 0; u < G.n; ++u) {
    std::sort(nb[u].begin(), nb[u].end());
    nb[u].erase(std::unique(nb[u].begin(), nb[u].end()), nb[u].end());
    G.adj.insert(G.adj.end(), nb[u].begin(), nb[u].end());
    G.ptr[u + 1] = (int64_t)G.adj.size();
  }
  return G;
}

enum { UND = 0, ROOT = 1, OUT = 2 };

// Synchronous MIS-2.  Node u carries the tuple (key(u), u) with
// key(u) = splitmix64(seed ^ splitmix64(u)).  In each round, with the states
// frozen at the start of the round, an undecided node becomes a root when its
// tuple is the largest among the undecided nodes within graph distance 2 of it
// (paths may pass through decided nodes); then every undecided node within
// distance 2 of a root is taken out.  Rounds repeat until no node is undecided.
static std::vector<int> mis2(const Graph& G, uint64_t seed) {
  const int n = G.n;
  std::vector<uint64_t> key(n);
  for (int u = 0; u < n; ++u) key[u] = splitmix64(seed ^ splitmix64((uint64_t)u));
  auto greater = [&](int a, int b) {   // tuple order (key, id)
    return key[a] != key[b] ? key[a] > key[b] : a > b;
  };
  std::vector<int> state(n, UND);
  int undecided = n;
  std::vector<char> seen(n, 0);
  std::vector<int> touched;
  while (undecided > 0) {
    std::vector<int> new_roots;
    for (int u = 0; u < n; ++u) {
      if (state[u] != UND) continue;
      // walk the closed distance-2 neighbourhood of u
      bool is_max = true;
      touched.clear();
      auto visit = [&](int w) {
        if (seen[w]) return;
        seen[w] = 1;
        touched.push_back(w);
        if (w != u && state[w] == UND && greater(w, u)) is_max = false;
      };
      visit(u);
      for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p) {
        int v = G.adj[p];
        visit(v);
        for (int64_t q = G.ptr[v]; q < G.ptr[v + 1]; ++q) visit(G.adj[q]);
      }
      for (int w : touched) seen[w] = 0;
      if (is_max) new_roots.push_back(u);
    }
    for (int r : new_roots) { state[r] = ROOT; --undecided; }
    // every undecided node within distance 2 of a root leaves
    std::vector<int> leave;
    for (int u = 0; u < n; ++u) {
      if (state[u] != UND) continue;
      bool near = false;
      for (int64_t p = G.ptr[u]; p < G.ptr[u + 1] && !near; ++p) {
        int v = G.adj[p];
        if (state[v] == ROOT) near = true;
        for (int64_t q = G.ptr[v]; q < G.ptr[v + 1] && !near; ++q)
          if (state[G.adj[q]] == ROOT) near = true;
      }
      if (near) leave.push_back(u);
    }
    for (int u : leave) { state[u] = OUT; --undecided; }
  }
  return state;
}

// Aggregates from the MIS-2 roots.  Roots are numbered in ascending node
// order.  Phase 2: a node adjacent to a root joins that root (unique, since
// roots are at least 3 apart).  Phase 3: every remaining node joins the
// aggregate of its phase-2 neighbour with the smallest aggregate number.
static std::vector<int> aggregate(const Graph& G, const std::vector<int>& state, int* n_agg) {
  const int n = G.n;
  std::vector<int> agg(n, -1), phase(n, 0);
  int na = 0;
  for (int u = 0; u < n; ++u)
    if (state[u] == ROOT) { agg[u] = na++; phase[u] = 1; }
  for (int u = 0; u < n; ++u) {
    if (phase[u]) continue;
    for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p)
      if (state[G.adj[p]] == ROOT) { agg[u] = agg[G.adj[p]]; phase[u] = 2; break; }
  }
  for (int u = 0; u < n; ++u) {
    if (phase[u]) continue;
    int best = -1;
    for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p) {
      int v = G.adj[p];
      if (phase[v] == 2 && (best < 0 || agg[v] < best)) best = agg[v];
    }
    if (best < 0) throw Error(EINVAL_, "aggregate: node without a phase-2 neighbour");
    agg[u] = best;
    phase[u] = 3;
  }
  *n_agg = na;
  return agg;
}

// Subdomains of the DD(GS) smoother: the MIS-2 aggregates of the level's
// node graph for the same seed, i.e. the aggregates the AMG coarsening of
// that level forms (compact patches of a node and its neighbours).
static std::vector<int> dd_subdomains(const Graph& G, uint64_t seed, int* n_sub);

static std::vector<int> dd_subdomains(const Graph& G, uint64_t seed, int* n_sub) {
  std::vector<int> st = mis2(G, seed);
  return aggregate(G, st, n_sub);
}

// Greedy colouring: the nodes in the given order each take the smallest
// colour that none of their already coloured neighbours has.  The node graph
// is symmetric, so no two neighbours share a colour.  (In node order on a
// structured 27-point stencil numbered lexicographically this gives 8
// colours.)
static std::vector<int> greedy_colors(const Graph& G, const std::vector<int>& order, int* ncolors) {
  std::vector<int> color(G.n, -1);
  int nc = 0;
  for (int u : order) {
    std::vector<char> used(G.ptr[u + 1] - G.ptr[u] + 1, 0);
    for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p) {
      const int c = color[G.adj[p]];
      if (c >= 0 && c < (int)used.size()) used[c] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    color[u] = c;
    nc = std::max(nc, c + 1);
  }
  *ncolors = nc;
  return color;
}

// Smallest-last order (Matula and Beck): repeatedly remove a node of least
// degree in the graph that remains, and colour in the reverse of the removal
// order.  Ties: the nodes of one degree form a stack; at the start every
// node is pushed in ascending number onto the stack of its degree, a node
// whose degree drops (a neighbour was removed; neighbours visited in
// adjacency order) is pushed onto its new degree's stack, and the node
// removed is the top of the least non-empty stack (entries of nodes removed
// or moved since are skipped).
static std::vector<int> smallest_last_order(const Graph& G) {
  const int n = G.n;
  std::vector<int> deg(n, 0);
  int maxd = 0;
  for (int u = 0; u < n; ++u) {
    for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p) deg[u] += G.adj[p] != u;
    maxd = std::max(maxd, deg[u]);
  }
  std::vector<std::vector<int>> stack(maxd + 1);
  for (int u = 0; u < n; ++u) stack[deg[u]].push_back(u);
  std::vector<char> gone(n, 0);
  std::vector<int> removal;
  int d = 0;
  while ((int)removal.size() < n) {
    int u = -1;
    while (u < 0) {
      while (stack[d].empty()) ++d;
      const int t = stack[d].back();
      stack[d].pop_back();
      if (!gone[t] && deg[t] == d) u = t;
    }
    gone[u] = 1;
    removal.push_back(u);
    for (int64_t p = G.ptr[u]; p < G.ptr[u + 1]; ++p) {
      const int v = G.adj[p];
      if (v == u || gone[v]) continue;
      --deg[v];
      stack[deg[v]].push_back(v);
      d = std::min(d, deg[v]);
    }
  }
  return std::vector<int>(removal.rbegin(), removal.rend());
}

// Colouring of a node graph for the multicolour smoothers: greedy in node
// order; graphs of at most COLOR_SL_MAX nodes are also coloured greedily in
// smallest-last order and keep that colouring when it has fewer colours.
constexpr int COLOR_SL_MAX = 32768;
static std::vector<int> color_nodes(const Graph& G, uint64_t /*seed*/, int* ncolors) {
  std::vector<int> natural(G.n);
  for (int u = 0; u < G.n; ++u) natural[u] = u;
  std::vector<int> color = greedy_colors(G, natural, ncolors);
  if (G.n > 0 && G.n <= COLOR_SL_MAX) {
    int nsl = 0;
    std::vector<int> c2 = greedy_colors(G, smallest_last_order(G), &nsl);
    if (nsl < *ncolors) {
      color = c2;
      *ncolors = nsl;
    }
  }
  return color;
}

// Tentative prolongator.  For aggregate a, B_a stacks the near-nullspace rows
// of its dofs (nodes ascending, then dofs ascending), k columns.  Modified
// Gram-Schmidt gives B_a = Q_a R_a with positive diagonal; Q_a becomes the
// rows of P_tent in columns [a k, a k + k) and R_a the coarse near-nullspace.
// A column whose remaining norm is <= 1e-12 ||B_a||_F is dead: its Q column
// and R row are zero and the coarse dof a k + j is recorded as dead.
struct Tentative {
  Csr P;
  std::vector<double> Bc;   // coarse nullspace, (k, n_agg k) row-major: Bc[c * nc + i]
  std::vector<int> dead;
};

static Tentative tentative(const std::vector<int>& agg, int n_agg, int b, int k,
                           const std::vector<double>& B /* (k, ndof) */) {
  const int nnode = (int)agg.size(), ndof = nnode * b, nc = n_agg * k;
  std::vector<std::vector<int>> members(n_agg);
  for (int u = 0; u < nnode; ++u) members[agg[u]].push_back(u);
  Tentative T;
  T.P.nr = ndof;
  T.P.nc = nc;
  T.P.ptr.assign(ndof + 1, 0);
  T.Bc.assign((size_t)k * nc, 0.0);
  std::vector<std::vector<double>> rowval(ndof, std::vector<double>(k, 0.0));
  std::vector<int> rowagg(ndof, -1);
  for (int a = 0; a < n_agg; ++a) {
    std::vector<int> dofs;
    for (int u : members[a])
      for (int c = 0; c < b; ++c) dofs.push_back(u * b + c);
    const int m = (int)dofs.size();
    std::vector<double> Q((size_t)m * k), R((size_t)k * k, 0.0);
    double fro = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < k; ++j) {
        double v = B[(size_t)j * ndof + dofs[i]];
        Q[(size_t)i * k + j] = v;
        fro += v * v;
      }
    fro = std::sqrt(fro);
    for (int j = 0; j < k; ++j) {
      for (int l = 0; l < j; ++l) {
        double r = 0.0;
        for (int i = 0; i < m; ++i) r += Q[(size_t)i * k + l] * Q[(size_t)i * k + j];
        R[(size_t)l * k + j] = r;
        for (int i = 0; i < m; ++i) Q[(size_t)i * k + j] -= r * Q[(size_t)i * k + l];
      }
      double nr = 0.0;
      for (int i = 0; i < m; ++i) nr += Q[(size_t)i * k + j] * Q[(size_t)i * k + j];
      nr = std::sqrt(nr);
      if (nr <= 1e-12 * fro) {
        for (int i = 0; i < m; ++i) Q[(size_t)i * k + j] = 0.0;
        for (int l = j; l < k; ++l) R[(size_t)j * k + l] = 0.0;
        T.dead.push_back(a * k + j);
      } else {
        R[(size_t)j * k + j] = nr;
        for (int i = 0; i < m; ++i) Q[(size_t)i * k + j] /= nr;
      }
    }
    for (int i = 0; i < m; ++i) {
      rowagg[dofs[i]] = a;
      for (int j = 0; j < k; ++j) rowval[dofs[i]][j] = Q[(size_t)i * k + j];
    }
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) T.Bc[(size_t)j * nc + a * k + i] = R[(size_t)i * k + j];
  }
  std::sort(T.dead.begin(), T.dead.end());
  for (int r = 0; r < ndof; ++r) {
    int a = rowagg[r];
    for (int j = 0; j < k; ++j) { T.P.col.push_back(a * k + j); T.P.val.push_back(rowval[r][j]); }
    T.P.ptr[r + 1] = (int64_t)T.P.col.size();
  }
  return T;
}

// lambda_max(D^-1 A) by power iteration from the seeded start vector
// v_u = 0.5 + (splitmix64(splitmix64(seed) ^ (u + 1)) >> 11) * 2^-53.
static double power_lambda(const Csr& A, const std::vector<double>& dinv, uint64_t seed, int its) {
  const int n = A.nr;
  std::vector<double> v(n), w(n);
  const uint64_t s0 = splitmix64(seed);
  for (int u = 0; u < n; ++u)
    v[u] = 0.5 + (double)(splitmix64(s0 ^ (uint64_t)(u + 1)) >> 11) * 0x1.0p-53;
  double nv = nrm2(n, v.data());
  for (int u = 0; u < n; ++u) v[u] /= nv;
  double lam = 0.0;
  for (int it = 0; it < its; ++it) {
    spmv(A, v.data(), w.data());
    for (int u = 0; u < n; ++u) w[u] *= dinv[u];
    lam = nrm2(n, w.data());       // ||v|| = 1
    if (lam == 0.0) break;
    for (int u = 0; u < n; ++u) v[u] = w[u] / lam;
  }
  return lam;
}

// ------------------------------------------------------------- dense LU
// Partial pivoting; the pivot is the first row holding the largest |a|.
struct DenseLU {
  int n = 0;
  std::vector<double> a;    // row-major LU factors
  std::vector<int> piv;
  void factor(const std::vector<double>& M, int n_) {
    n = n_;
    a = M;
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
      int p = k;
      double best = std::fabs(a[(size_t)k * n + k]);
      for (int i = k + 1; i < n; ++i) {
        double v = std::fabs(a[(size_t)i * n + k]);
        if (v > best) { best = v; p = i; }
      }
      piv[k] = p;
      if (best == 0.0) throw Error(ESINGULAR, "dense LU: zero pivot");
      if (p != k)
        for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
      for (int i = k + 1; i < n; ++i) {
        double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
        a[(size_t)i * n + k] = l;
        for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
      }
    }
  }
  void solve(const double* b, double* x) const {
    std::vector<double> y(b, b + n);
    for (int k = 0; k < n; ++k) std::swap(y[k], y[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) y[i] -= a[(size_t)i * n + j] * y[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) y[i] -= a[(size_t)i * n + j] * y[j];
      y[i] /= a[(size_t)i * n + i];
    }
    std::copy(y.begin(), y.end(), x);
  }
};

static std::vector<double> to_dense(const Csr& A) {
  std::vector<double> M((size_t)A.nr * A.nc, 0.0);
  for (int i = 0; i < A.nr; ++i)
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) M[(size_t)i * A.nc + A.col[p]] += A.val[p];
  return M;
}

// ------------------------------------------------------------ options
struct Opts {
  int sweeps = 1, order = 1 /*0 fwd 1 bwd 2 sym*/, coarse_max = 200, max_levels = 10;
  int cheb_degree = 2, power_its = 10;
  double cheb_ratio = 30.0, cheb_boost = 1.1;
  int simplec_mode = 0;      // 0: sum_j |a_ij|, 1: |sum_j a_ij|, 2: a_ii
  std::vector<int> split;    // field -> group (0 predictor, 1 Schur); empty: last field is Schur
  int schur_direct_max = 5000;
  uint64_t seed = 0;
  int pg = 0;                // Petrov-Galerkin transfers (per AMG node of the specification)
};

// ------------------------------------------------------- block matrices
// An N x N grid of blocks over fields [0, N); a missing block is zero.
struct BlockMat {
  int N = 0;
  std::vector<int> size;
  std::vector<std::shared_ptr<Csr>> blk;   // N*N, row-major (i, j)
  const Csr* at(int i, int j) const { return blk[(size_t)i * N + j].get(); }
  std::vector<int> offsets() const {
    std::vector<int> o(N + 1, 0);
    for (int i = 0; i < N; ++i) o[i + 1] = o[i] + size[i];
    return o;
  }
  int total() const { int s = 0; for (int v : size) s += v; return s; }
  // y = A x restricted to field ranges [f0, f1) for rows and columns
  void apply(int f0, int f1, const double* x, double* y) const {
    std::vector<int> o = offsets();
    for (int i = f0; i < f1; ++i) {
      double* yi = y + (o[i] - o[f0]);
      std::fill(yi, yi + size[i], 0.0);
      for (int j = f0; j < f1; ++j)
        if (at(i, j)) spmv_add(*at(i, j), x + (o[j] - o[f0]), yi);
    }
  }
  std::vector<double> dense(int f0, int f1) const {
    std::vector<int> o = offsets();
    int n = o[f1] - o[f0];
    std::vector<double> M((size_t)n * n, 0.0);
    for (int i = f0; i < f1; ++i)
      for (int j = f0; j < f1; ++j) {
        const Csr* B = at(i, j);
        if (!B) continue;
        for (int r = 0; r < B->nr; ++r)
          for (int64_t p = B->ptr[r]; p < B->ptr[r + 1]; ++p)
            M[(size_t)(o[i] - o[f0] + r) * n + (o[j] - o[f0] + B->col[p])] += B->val[p];
      }
    return M;
  }
};

// ----------------------------------------------------------- smoothers
// Field smoother, one of
//  * Chebyshev polynomial on D^-1 A over [lambda/ratio, boost*lambda]
//    (three-term recurrence, Saad "Iterative Methods for Sparse Linear
//    Systems", 2nd ed., Algorithm 12.1); with zero_guess the first residual
//    is b itself; degree 1 is damped Jacobi;
//  * symmetric multicolour Gauss-Seidel with damping omega (the Gauss-Seidel
//    family of smoothers the paper runs inside its AMG): nodes of one colour
//    are relaxed together, colours forward then backward; the dofs of one
//    node are updated together from the values before the node's update.
//    With half, pre-smoothing (before the coarse correction) sweeps forward
//    only and post-smoothing backward only; the level smoother tells the
//    field smoother which of the two it is doing;
//  * DD(GS) with damping omega, the paper's domain-decomposition smoother
//    (Sec. 7: Gauss-Seidel inside each subdomain, the subdomains coupled
//    additively): the nodes are split into subdomains (the level's
//    aggregates); in a sweep every subdomain relaxes its nodes in the colour
//    order of the multicolour SGS, using the newest values of its own nodes
//    and the values the other subdomains' nodes held when the sweep began.
//    Forward then backward, or half sweeps as above.  A level with fewer
//    aggregates than the ddmin parameter (default 256: the workgroups a GPU
//    runs side by side) is one subdomain: the multicolour SGS.
struct Cheb {
  const Csr* A = nullptr;
  std::vector<double> dinv;
  double lambda = 0.0, lo = 0.0, hi = 0.0;
  int degree = 2;
  int kind = 0;                       // 0 Chebyshev, 1 multicolour SGS, 2 DD(GS)
  int bs = 1, steps = 1, half = 0;
  double omega = 1.0;
  std::vector<std::vector<int>> color_nodes;   // nodes of each colour, ascending
  std::vector<int> sub;                        // DD(GS): node -> subdomain
  void setup_sgs(const Csr* A_, int b, double om, int st, uint64_t seed) {
    A = A_;
    std::vector<double> d = diagonal(*A);
    dinv.resize(d.size());
    for (size_t i = 0; i < d.size(); ++i) {
      if (d[i] == 0.0) throw Error(ESINGULAR, "Gauss-Seidel smoother: zero diagonal entry");
      dinv[i] = 1.0 / d[i];
    }
    kind = 1;
    bs = b;
    omega = om;
    steps = st;
    Graph G = node_graph(*A, b);
    int nc = 0;
    std::vector<int> col = orc::color_nodes(G, seed, &nc);
    color_nodes.assign(nc, {});
    for (int u = 0; u < G.n; ++u) color_nodes[col[u]].push_back(u);
  }
  // DD(GS): the SGS set-up plus the subdomains (given, or the aggregates;
  // a level with fewer than ddmin aggregates is one subdomain)
  void setup_ddgs(const Csr* A_, int b, double om, int st, uint64_t seed, const int* given_sub = nullptr,
                  int ddmin = 1) {
    setup_sgs(A_, b, om, st, seed);
    kind = 2;
    Graph G = node_graph(*A, b);
    if (given_sub) {
      sub.assign(given_sub, given_sub + G.n);
    } else {
      int ns = 0;
      sub = dd_subdomains(G, seed, &ns);
      if (ns < ddmin) sub.assign(G.n, 0);
    }
  }
  // relax the nodes of colour c; with DD(GS) (xold non-null) a coupling to a
  // node of another subdomain takes that node's value from xold
  void relax_color(int c, const double* b, double* x, const double* xold = nullptr) const {
    std::vector<double> upd(bs);
    for (int u : color_nodes[c]) {
      for (int q = 0; q < bs; ++q) {
        const int r = u * bs + q;
        double s = b[r];
        for (int64_t p = A->ptr[r]; p < A->ptr[r + 1]; ++p) {
          const int cc = A->col[p];
          const bool own = !xold || sub[cc / bs] == sub[u];
          s -= A->val[p] * (own ? x[cc] : xold[cc]);
        }
        upd[q] = omega * dinv[r] * s;
      }
      for (int q = 0; q < bs; ++q) x[u * bs + q] += upd[q];
    }
  }
  // one sweep over the colours in the given direction; DD(GS): every
  // subdomain relaxes its own nodes in colour order against the values its
  // neighbours held when the sweep began (block Jacobi between subdomains,
  // Gauss-Seidel inside)
  void sweep(bool forward, const double* b, double* x) const {
    const int nc = (int)color_nodes.size();
    std::vector<double> xold;
    if (kind == 2) xold.assign(x, x + A->nr);
    for (int k = 0; k < nc; ++k) relax_color(forward ? k : nc - 1 - k, b, x, kind == 2 ? xold.data() : nullptr);
  }
  // pre: this application is pre-smoothing (only matters with half)
  void apply_sgs(const double* b, double* x, bool zero_guess, bool pre) const {
    if (zero_guess) std::fill(x, x + A->nr, 0.0);
    for (int st = 0; st < steps; ++st) {
      if (!half || pre) sweep(true, b, x);
      if (!half || !pre) sweep(false, b, x);
    }
  }
  void setup(const Csr* A_, double lam, const Opts& o) {
    A = A_;
    std::vector<double> d = diagonal(*A);
    dinv.resize(d.size());
    for (size_t i = 0; i < d.size(); ++i) {
      if (d[i] == 0.0) throw Error(ESINGULAR, "Chebyshev smoother: zero diagonal entry");
      dinv[i] = 1.0 / d[i];
    }
    lambda = lam;
    hi = o.cheb_boost * lam;
    lo = lam / o.cheb_ratio;
    degree = o.cheb_degree;
  }
  void apply(const double* b, double* x, bool zero_guess, bool pre = true) const {
    if (kind >= 1) { apply_sgs(b, x, zero_guess, pre); return; }
    const int n = A->nr;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    std::vector<double> r(n), d(n);
    double rho = 1.0 / sigma;
    if (zero_guess) std::copy(b, b + n, r.begin());
    else { spmv(*A, x, r.data()); for (int i = 0; i < n; ++i) r[i] = b[i] - r[i]; }
    for (int i = 0; i < n; ++i) { d[i] = dinv[i] * r[i] / theta; x[i] = (zero_guess ? 0.0 : x[i]) + d[i]; }
    for (int k = 1; k < degree; ++k) {
      spmv(*A, x, r.data());
      for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
      double rho_new = 1.0 / (2.0 * sigma - rho);
      for (int i = 0; i < n; ++i) {
        d[i] = rho_new * rho * d[i] + (2.0 * rho_new / delta) * dinv[i] * r[i];
        x[i] += d[i];
      }
      rho = rho_new;
    }
  }
};

// ---------------------------------------------------------- hierarchies
// A (monolithic) AMG hierarchy over N fields (Sec. 4.3).  N = 1 is the
// plain single-field AMG.  Per-field transfers P_i^l, R_i^l = (P_i^l)^T are
// built from the diagonal blocks in lockstep; coarse blocks are
// A_ij^{l+1} = R_i^l A_ij^l P_j^l.  A field that is not coarsened on a level
// (zero diagonal block, already small, or stalled) uses P = I there.
struct Level {
  BlockMat A;
  std::vector<Csr> P, R;              // per field (empty on the coarsest level)
  std::vector<std::vector<int>> agg;  // per field node -> aggregate (empty if P = I)
  std::vector<std::vector<double>> B; // per field near-nullspace (k, n_i)
  std::vector<int> bs;                // per field block size
  std::vector<double> lambda;         // per field lambda_max(D^-1 A_ii), 0 if none
  std::vector<std::vector<int>> dead; // per field dead dofs on THIS level
};

struct FieldDesc { int ndof, bs, nns; std::vector<double> B; };

struct Hierarchy {
  std::vector<Level> lev;
  DenseLU coarse;
  int N = 0;
};

// Petrov-Galerkin smoothing of a tentative prolongator (Sala and Tuminaro,
// "A new Petrov-Galerkin smoothed aggregation preconditioner for
// nonsymmetric linear systems", SIAM J. Sci. Comput. 2008, the method the
// paper uses for the fluid, Sec. 7): P = P_tent - Q diag(omega) with
// Q = D^-1 A P_tent, each column's damping omega_j minimising ||A P e_j||_2,
// omega_j = <A P_tent e_j, A Q e_j> / ||A Q e_j||^2, and 0 where that is
// negative or A Q e_j = 0.  The column sums run over the rows in ascending
// order.  Given A^T instead of A this gives the transpose of the restriction.
static Csr pg_smooth(const Csr& A, const Csr& Pt, const std::vector<double>& dinv) {
  Csr AP = spgemm(A, Pt);
  Csr Q = AP;
  scale_rows(Q, dinv);
  Csr AQ = spgemm(A, Q);
  std::vector<double> num(Pt.nc, 0.0), den(Pt.nc, 0.0);
  for (int r = 0; r < AQ.nr; ++r) {
    int64_t p = AP.ptr[r];
    for (int64_t q = AQ.ptr[r]; q < AQ.ptr[r + 1]; ++q) {
      const int c = AQ.col[q];
      while (p < AP.ptr[r + 1] && AP.col[p] < c) ++p;
      if (p < AP.ptr[r + 1] && AP.col[p] == c) num[c] += AP.val[p] * AQ.val[q];
      den[c] += AQ.val[q] * AQ.val[q];
    }
  }
  std::vector<double> omega(Pt.nc, 0.0);
  for (int c = 0; c < Pt.nc; ++c)
    if (den[c] > 0.0 && num[c] > 0.0) omega[c] = num[c] / den[c];
  for (int r = 0; r < Q.nr; ++r)
    for (int64_t p = Q.ptr[r]; p < Q.ptr[r + 1]; ++p) Q.val[p] *= -omega[Q.col[p]];
  return add(1.0, Pt, 1.0, Q);
}

static void build_hierarchy(Hierarchy& H, const BlockMat& A0, const std::vector<FieldDesc>& F,
                            const Opts& o) {
  const int N = A0.N;
  H.N = N;
  H.lev.clear();
  Level L0;
  L0.A = A0;
  L0.bs.resize(N);
  L0.B.resize(N);
  L0.dead.resize(N);
  for (int i = 0; i < N; ++i) { L0.bs[i] = F[i].bs; L0.B[i] = F[i].B; }
  H.lev.push_back(L0);
  std::vector<char> active(N);
  for (int i = 0; i < N; ++i) active[i] = A0.at(i, i) != nullptr;
  while (true) {
    Level& L = H.lev.back();
    const int l = (int)H.lev.size() - 1;
    // lambda for every field with a diagonal block (used by smoothers and P)
    L.lambda.assign(N, 0.0);
    for (int i = 0; i < N; ++i) {
      const Csr* Aii = L.A.at(i, i);
      if (!Aii) continue;
      std::vector<double> d = diagonal(*Aii), dinv(d.size());
      bool ok = true;
      for (size_t r = 0; r < d.size(); ++r) { if (d[r] == 0.0) ok = false; dinv[r] = d[r] != 0.0 ? 1.0 / d[r] : 0.0; }
      if (ok) L.lambda[i] = power_lambda(*Aii, dinv, o.seed, o.power_its);
    }
    // stopping test: coarsenable size small enough, nothing left to coarsen,
    // or the level limit reached
    int coarsenable = 0;
    bool any = false;
    for (int i = 0; i < N; ++i) {
      if (A0.at(i, i)) coarsenable += L.A.size[i];
      if (active[i] && L.A.size[i] <= o.coarse_max) active[i] = 0;
      if (active[i]) any = true;
    }
    if (coarsenable <= o.coarse_max || !any || l + 1 >= o.max_levels) break;
    Level C;
    C.bs.resize(N);
    C.B.resize(N);
    C.dead.resize(N);
    L.P.resize(N);
    L.R.resize(N);
    L.agg.resize(N);
    for (int i = 0; i < N; ++i) {
      const int n = L.A.size[i];
      if (!active[i]) {
        L.P[i] = identity(n);
        C.bs[i] = L.bs[i];
        C.B[i] = L.B[i];
        C.dead[i] = L.dead[i];
      } else {
        const Csr& Aii = *L.A.at(i, i);
        if (L.lambda[i] <= 0.0) throw Error(ESINGULAR, "AMG: diagonal block has a zero diagonal entry");
        Graph G = node_graph(Aii, L.bs[i]);
        std::vector<int> st = mis2(G, o.seed);
        int na = 0;
        L.agg[i] = aggregate(G, st, &na);
        const int k = (int)(L.B[i].size() / n);
        if (k == 0) throw Error(EINVAL_, "AMG: field has no near-nullspace vectors");
        Tentative T = tentative(L.agg[i], na, L.bs[i], k, L.B[i]);
        std::vector<double> d = diagonal(Aii);
        if (o.pg) {
          // Petrov-Galerkin smoothed aggregation: column-wise dampings for
          // P from A and for R from A^T
          std::vector<double> dinv(n);
          for (int r = 0; r < n; ++r) dinv[r] = 1.0 / d[r];
          L.P[i] = pg_smooth(Aii, T.P, dinv);
          L.R[i] = transpose(pg_smooth(transpose(Aii), T.P, dinv));
        } else {
          // smoothed prolongator P = (I - omega D^-1 A) P_tent, omega = 4/(3 lambda)
          std::vector<double> s(n);
          const double omega = 4.0 / (3.0 * L.lambda[i]);
          for (int r = 0; r < n; ++r) s[r] = -omega / d[r];
          Csr AP = spgemm(Aii, T.P);
          scale_rows(AP, s);
          L.P[i] = add(1.0, T.P, 1.0, AP);
        }
        C.bs[i] = k;
        C.B[i] = T.Bc;
        C.dead[i] = T.dead;
        if (na * k > 0.83 * n) active[i] = 0;   // coarsening stalled
      }
      if (L.R[i].nr == 0 && L.R[i].nc == 0) L.R[i] = transpose(L.P[i]);   // R = P^T unless Petrov-Galerkin
    }
    C.A.N = N;
    C.A.size.resize(N);
    C.A.blk.resize((size_t)N * N);
    for (int i = 0; i < N; ++i) C.A.size[i] = L.P[i].nc;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const Csr* Aij = L.A.at(i, j);
        if (!Aij) continue;
        Csr AP = spgemm(*Aij, L.P[j]);
        auto Ac = std::make_shared<Csr>(spgemm(L.R[i], AP));
        if (i == j)   // dead coarse dofs: identity row on the diagonal
          for (int dd : C.dead[i])
            for (int64_t p = Ac->ptr[dd]; p < Ac->ptr[dd + 1]; ++p)
              if (Ac->col[p] == dd) Ac->val[p] = 1.0;
        C.A.blk[(size_t)i * N + j] = Ac;
      }
    H.lev.push_back(std::move(C));
  }
  const Level& Lc = H.lev.back();
  H.coarse.factor(Lc.A.dense(0, N), Lc.A.total());
}

// ---------------------------------------------------------- solvers
struct Solver {
  int n = 0;
  virtual ~Solver() {}
  virtual void apply(const double* r, double* z) = 0;   // z = M^-1 r
};

// Global store of every hierarchy a context builds, for inspection.
struct Ctx;

struct LuSolver : Solver {
  DenseLU lu;
  void apply(const double* r, double* z) override { lu.solve(r, z); }
};

// A single-level smoother used as a block solve (the DD(GS) block solver of
// the paper's single-level comparison BGS(DD(GS)), Sec. 7): its sweeps from
// a zero guess, forward then backward.
struct SmootherSolver : Solver {
  Cheb sm;
  void apply(const double* r, double* z) override { sm.apply(r, z, true, true); }
};

// Level smoother of a (monolithic) hierarchy: one BGS sweep or one SIMPLE
// step over the level's blocks, with each field's own Chebyshev smoother in
// place of the diagonal solves (Sec. 4.3, last paragraph).
struct LevelSmoother {
  int kind = 0;                  // 0 BGS, 1 SIMPLE
  int order = 1;
  const BlockMat* A = nullptr;
  std::vector<Cheb> cheb;        // per field (unused for the Schur field)
  // SIMPLE pieces
  int ngroup1 = 0;               // fields [0, ngroup1) predictor, [ngroup1, N) Schur (1 field)
  std::vector<double> dtilde_inv;
  Csr Stilde;
  DenseLU schur_lu;
  bool schur_direct = true;
  Cheb schur_cheb;
  void bgs_sweep(int f0, int f1, const double* r, double* d, int ord, bool pre) const {
    std::vector<int> o = A->offsets();
    std::vector<int> seq;
    for (int i = f0; i < f1; ++i) seq.push_back(i);
    if (ord == 1) std::reverse(seq.begin(), seq.end());
    std::vector<char> done(A->N, 0);
    std::fill(d + 0, d + (o[f1] - o[f0]), 0.0);
    for (int i : seq) {
      std::vector<double> t(r + (o[i] - o[f0]), r + (o[i] - o[f0]) + A->size[i]);
      for (int j = f0; j < f1; ++j)
        if (j != i && done[j] && A->at(i, j)) {
          std::vector<double> y(A->size[i]);
          spmv(*A->at(i, j), d + (o[j] - o[f0]), y.data());
          for (int q = 0; q < A->size[i]; ++q) t[q] -= y[q];
        }
      cheb[i].apply(t.data(), d + (o[i] - o[f0]), true, pre);
      done[i] = 1;
    }
  }
  // one smoothing step: x <- x + M^-1 (b - A x)
  void smooth(const double* b, double* x, bool zero_guess) const {
    const int n = A->total(), N = A->N;
    std::vector<double> r(b, b + n), d(n, 0.0);
    if (!zero_guess) {
      std::vector<double> Ax(n);
      A->apply(0, N, x, Ax.data());
      for (int i = 0; i < n; ++i) r[i] = b[i] - Ax[i];
    }
    // symmetric order: forward before the coarse correction, backward after
    const int ord = order == 2 ? (zero_guess ? 0 : 1) : order;
    // pre-smoothing starts from zero, post-smoothing does not
    if (kind == 0) {
      bgs_sweep(0, N, r.data(), d.data(), ord, zero_guess);
    } else {
      std::vector<int> o = A->offsets();
      const int n1 = o[ngroup1], n2 = n - n1;
      bgs_sweep(0, ngroup1, r.data(), d.data(), ord, zero_guess);  // predictor
      std::vector<double> t(r.begin() + n1, r.end()), y(n2);
      for (int j = 0; j < ngroup1; ++j)
        if (A->at(ngroup1, j)) {
          spmv(*A->at(ngroup1, j), d.data() + o[j], y.data());
          for (int q = 0; q < n2; ++q) t[q] -= y[q];
        }
      if (schur_direct) schur_lu.solve(t.data(), d.data() + n1);
      else schur_cheb.apply(t.data(), d.data() + n1, true);
      for (int j = 0; j < ngroup1; ++j)
        if (A->at(j, ngroup1)) {
          std::vector<double> u(A->size[j]);
          spmv(*A->at(j, ngroup1), d.data() + n1, u.data());
          for (int q = 0; q < A->size[j]; ++q) d[o[j] + q] -= dtilde_inv[o[j] + q] * u[q];
        }
    }
    for (int i = 0; i < n; ++i) x[i] = (zero_guess ? 0.0 : x[i]) + d[i];
  }
};

// SIMPLEC-type diagonal of the merged predictor block over fields [0, g1)
static std::vector<double> simplec_inv(const BlockMat& A, int g1, int mode) {
  std::vector<int> o = A.offsets();
  std::vector<double> dinv(o[g1], 0.0);
  for (int i = 0; i < g1; ++i)
    for (int r = 0; r < A.size[i]; ++r) {
      double sabs = 0.0, s = 0.0, dg = 0.0;
      for (int j = 0; j < g1; ++j) {
        const Csr* B = A.at(i, j);
        if (!B) continue;
        for (int64_t p = B->ptr[r]; p < B->ptr[r + 1]; ++p) {
          sabs += std::fabs(B->val[p]);
          s += B->val[p];
          if (i == j && B->col[p] == r) dg = B->val[p];
        }
      }
      double v = mode == 0 ? sabs : mode == 1 ? std::fabs(s) : dg;
      if (v == 0.0) throw Error(ESINGULAR, "SIMPLE: zero entry in the approximate predictor diagonal");
      dinv[o[i] + r] = 1.0 / v;
    }
  return dinv;
}

// S~ = A22 - sum_{i in group 1} A_2i D~_i^-1 A_i2   (Schur field = index g1)
static Csr schur_approx(const BlockMat& A, int g1, const std::vector<double>& dinv) {
  std::vector<int> o = A.offsets();
  const int n2 = A.size[g1];
  Csr S;
  S.nr = S.nc = n2;
  S.ptr.assign(n2 + 1, 0);
  if (A.at(g1, g1)) S = *A.at(g1, g1);
  for (int i = 0; i < g1; ++i) {
    if (!A.at(g1, i) || !A.at(i, g1)) continue;
    Csr T = *A.at(i, g1);
    std::vector<double> s(dinv.begin() + o[i], dinv.begin() + o[i] + A.size[i]);
    scale_rows(T, s);
    Csr prod = spgemm(*A.at(g1, i), T);
    S = add(1.0, S, -1.0, prod);
  }
  return S;
}

struct AmgSolver : Solver {
  Hierarchy H;
  std::vector<LevelSmoother> sm;   // per non-coarsest level
  int smoother_kind = 0;
  void vcycle(int l, const double* b, double* x) const {
    const Level& L = H.lev[l];
    const int n = L.A.total();
    if (l == (int)H.lev.size() - 1) { H.coarse.solve(b, x); return; }
    sm[l].smooth(b, x, true);                          // pre-smoothing, x = 0 on entry
    std::vector<double> Ax(n);
    L.A.apply(0, L.A.N, x, Ax.data());
    for (int i = 0; i < n; ++i) Ax[i] = b[i] - Ax[i];  // residual
    const Level& C = H.lev[l + 1];
    std::vector<int> o = L.A.offsets(), oc = C.A.offsets();
    const int nc = C.A.total();
    std::vector<double> bc(nc), xc(nc, 0.0);
    for (int i = 0; i < L.A.N; ++i) spmv(L.R[i], Ax.data() + o[i], bc.data() + oc[i]);
    vcycle(l + 1, bc.data(), xc.data());
    for (int i = 0; i < L.A.N; ++i) spmv_add(L.P[i], xc.data() + oc[i], x + o[i]);
    sm[l].smooth(b, x, false);                         // post-smoothing
  }
  void apply(const double* r, double* z) override {
    std::fill(z, z + n, 0.0);
    vcycle(0, r, z);
  }
};

// Block Gauss-Seidel over fields [f0, f1) of a block matrix, increment form:
// z^(k) = z^(k-1) + M^-1 (r - A z^(k-1)), M the lower (fwd) or upper (bwd)
// block triangle; sym alternates fwd / bwd.  Diagonal solves use children.
struct BgsSolver : Solver {
  const BlockMat* A = nullptr;
  int f0 = 0, f1 = 0, sweeps = 1, order = 1;
  std::vector<std::unique_ptr<Solver>> child;   // per field in [f0, f1)
  void apply(const double* r, double* z) override {
    std::vector<int> o = A->offsets();
    std::fill(z, z + n, 0.0);
    std::vector<double> res(n), d(n), t, y;
    for (int s = 0; s < sweeps; ++s) {
      if (s == 0) std::copy(r, r + n, res.begin());
      else {
        A->apply(f0, f1, z, res.data());
        for (int i = 0; i < n; ++i) res[i] = r[i] - res[i];
      }
      int ord = order == 2 ? (s % 2) : order;
      std::vector<int> seq;
      for (int i = f0; i < f1; ++i) seq.push_back(i);
      if (ord == 1) std::reverse(seq.begin(), seq.end());
      std::vector<char> done(A->N, 0);
      std::fill(d.begin(), d.end(), 0.0);
      for (int i : seq) {
        const int oi = o[i] - o[f0], ni = A->size[i];
        t.assign(res.begin() + oi, res.begin() + oi + ni);
        for (int j = f0; j < f1; ++j)
          if (j != i && done[j] && A->at(i, j)) {
            y.assign(ni, 0.0);
            spmv(*A->at(i, j), d.data() + (o[j] - o[f0]), y.data());
            for (int q = 0; q < ni; ++q) t[q] -= y[q];
          }
        child[i - f0]->apply(t.data(), d.data() + oi);
        done[i] = 1;
      }
      for (int i = 0; i < n; ++i) z[i] += d[i];
    }
  }
};

// SIMPLE over fields [f0, f1) split into a predictor group [f0, g) and a
// Schur field g = f1 - 1 (matrix form of M_SIMPLE, Sec. 4.2):
//   z1 = A11^-1 r1;  z2 = S~^-1 (r2 - A21 z1);  d1 = z1 - D~^-1 A12 z2;  d2 = z2.
struct SimpleSolver : Solver {
  const BlockMat* A = nullptr;
  int f0 = 0, f1 = 0, g = 0, sweeps = 1;
  std::unique_ptr<Solver> pred, schur;
  std::vector<double> dtinv;    // over the predictor rows
  BlockMat Ssub;                // sub-block view with fields re-based at f0
  void apply(const double* r, double* z) override {
    std::vector<int> o = A->offsets();
    const int n1 = o[g] - o[f0], n2 = n - n1;
    std::fill(z, z + n, 0.0);
    std::vector<double> res(n), d(n), t(n2), y;
    for (int s = 0; s < sweeps; ++s) {
      if (s == 0) std::copy(r, r + n, res.begin());
      else {
        A->apply(f0, f1, z, res.data());
        for (int i = 0; i < n; ++i) res[i] = r[i] - res[i];
      }
      pred->apply(res.data(), d.data());
      std::copy(res.begin() + n1, res.end(), t.begin());
      for (int j = f0; j < g; ++j)
        if (A->at(g, j)) {
          y.assign(n2, 0.0);
          spmv(*A->at(g, j), d.data() + (o[j] - o[f0]), y.data());
          for (int q = 0; q < n2; ++q) t[q] -= y[q];
        }
      schur->apply(t.data(), d.data() + n1);
      for (int j = f0; j < g; ++j)
        if (A->at(j, g)) {
          const int nj = A->size[j], oj = o[j] - o[f0];
          y.assign(nj, 0.0);
          spmv(*A->at(j, g), d.data() + n1, y.data());
          for (int q = 0; q < nj; ++q) d[oj + q] -= dtinv[oj + q] * y[q];
        }
      for (int i = 0; i < n; ++i) z[i] += d[i];
    }
  }
};

// ------------------------------------------------------------- spec
// Preconditioner specification in the paper's notation, e.g. "BGS(AMG)",
// "SIMPLE(BGS(AMG);AMG)", "AMG(BGS)", "AMG(SIMPLE)".  Optional parameters
// in brackets: "BGS[sweeps=2,order=bwd](AMG)".
struct Spec {
  std::string name;
  int sweeps = -1, order = -1, degree = -1, smoother = -1, steps = -1, half = 0, pg = 0, ddmin = 256;
  int cheb_from = -1;                  // with sgs / ddgs: Chebyshev on the levels l >= cheb_from
  double omega = -1.0;
  std::vector<Spec> kids;
};

struct Parser {
  const char* s;
  size_t i = 0;
  explicit Parser(const char* s_) : s(s_) {}
  void ws() { while (s[i] == ' ') ++i; }
  Spec parse() {
    ws();
    Spec sp;
    while (isalpha((unsigned char)s[i])) sp.name += (char)toupper(s[i++]);
    if (sp.name.empty()) throw Error(EINVAL_, std::string("spec: name expected in '") + s + "'");
    ws();
    if (s[i] == '[') {
      ++i;
      while (s[i] && s[i] != ']') {
        std::string k, v;
        ws();
        while (isalpha((unsigned char)s[i]) || s[i] == '_') k += (char)tolower(s[i++]);
        ws();
        if (s[i++] != '=') throw Error(EINVAL_, "spec: '=' expected");
        ws();
        while (isalnum((unsigned char)s[i]) || s[i] == '.') v += (char)tolower(s[i++]);
        ws();
        if (k == "sweeps") sp.sweeps = atoi(v.c_str());
        else if (k == "order") sp.order = v == "fwd" ? 0 : v == "bwd" ? 1 : v == "sym" ? 2 : -9;
        else if (k == "degree") sp.degree = atoi(v.c_str());
        else if (k == "smoother") sp.smoother = v == "cheb" ? 0 : v == "sgs" ? 1 : v == "ddgs" ? 2 : -9;
        else if (k == "omega") sp.omega = atof(v.c_str());
        else if (k == "steps") sp.steps = atoi(v.c_str());
        else if (k == "half") {
          sp.half = atoi(v.c_str());
          if (sp.half != 0 && sp.half != 1) throw Error(EINVAL_, "spec: bad value " + v);
        }
        else if (k == "pg") {
          sp.pg = atoi(v.c_str());
          if (sp.pg != 0 && sp.pg != 1) throw Error(EINVAL_, "spec: bad value " + v);
        }
        else if (k == "ddmin") {
          sp.ddmin = atoi(v.c_str());
          if (sp.ddmin < 1) throw Error(EINVAL_, "spec: bad value " + v);
        }
        else if (k == "cheb_from") {
          sp.cheb_from = atoi(v.c_str());
          if (sp.cheb_from < 1) throw Error(EINVAL_, "spec: bad value " + v);
        }
        else throw Error(EINVAL_, "spec: unknown parameter " + k);
        if (sp.smoother == -9 || (k == "omega" && !(sp.omega > 0.0 && sp.omega < 2.0)) ||
            (k == "steps" && sp.steps < 1))
          throw Error(EINVAL_, "spec: bad value " + v);
        if (sp.order == -9 || (k == "sweeps" && sp.sweeps < 1) || (k == "degree" && sp.degree < 1))
          throw Error(EINVAL_, "spec: bad value " + v);
        if (s[i] == ',') ++i;
      }
      if (s[i] != ']') throw Error(EINVAL_, "spec: ']' expected");
      ++i;
      ws();
    }
    if (s[i] == '(') {
      ++i;
      sp.kids.push_back(parse());
      ws();
      while (s[i] == ';') { ++i; sp.kids.push_back(parse()); ws(); }
      if (s[i] != ')') throw Error(EINVAL_, "spec: ')' expected");
      ++i;
    }
    ws();
    return sp;
  }
};

struct Ctx {
  BlockMat A;
  std::vector<FieldDesc> F;
  Opts o;
  std::unique_ptr<Solver> root;
  std::vector<AmgSolver*> hier;            // every AMG hierarchy, in build order
  std::vector<std::unique_ptr<BlockMat>> owned;
  double setup_s = 0.0;
};

static BlockMat sub_blocks(const BlockMat& A, int f0, int f1) {
  BlockMat S;
  S.N = f1 - f0;
  S.size.assign(A.size.begin() + f0, A.size.begin() + f1);
  S.blk.resize((size_t)S.N * S.N);
  for (int i = 0; i < S.N; ++i)
    for (int j = 0; j < S.N; ++j) S.blk[(size_t)i * S.N + j] = A.blk[(size_t)(i + f0) * A.N + (j + f0)];
  return S;
}

static std::unique_ptr<Solver> build(Ctx& C, const Spec& sp, const BlockMat& A, int f0, int f1,
                                     const std::vector<FieldDesc>& F);

static std::unique_ptr<Solver> build_amg(Ctx& C, const BlockMat& A, int f0, int f1,
                                         const std::vector<FieldDesc>& F, const Spec* smoother,
                                         const Spec& amg) {
  auto S = std::make_unique<AmgSolver>();
  Opts lo = C.o;                       // this hierarchy's smoother degree
  if (amg.degree > 0) lo.cheb_degree = amg.degree;
  const bool sgs = amg.smoother == 1 || amg.smoother == 2;
  const double omega = amg.omega > 0.0 ? amg.omega : 1.0;
  const int steps = amg.steps > 0 ? amg.steps : 1;
  BlockMat sub = sub_blocks(A, f0, f1);
  std::vector<FieldDesc> Fs(F.begin() + f0, F.begin() + f1);
  for (int i = 0; i < sub.N; ++i)
    if (!sub.at(i, i) && !(smoother && smoother->name == "SIMPLE" && i == sub.N - 1))
      throw Error(ESINGULAR, "AMG: zero diagonal block");
  Opts ho = C.o;
  ho.pg = amg.pg;
  build_hierarchy(S->H, sub, Fs, ho);
  S->n = sub.total();
  S->smoother_kind = smoother && smoother->name == "SIMPLE" ? 1 : 0;
  const int nl = (int)S->H.lev.size();
  S->sm.resize(nl > 0 ? nl - 1 : 0);
  for (int l = 0; l + 1 < nl; ++l) {
    LevelSmoother& M = S->sm[l];
    const Level& L = S->H.lev[l];
    M.kind = S->smoother_kind;
    M.order = smoother && smoother->order >= 0 ? smoother->order : C.o.order;
    M.A = &L.A;
    M.cheb.resize(sub.N);
    const int nchb = M.kind == 1 ? sub.N - 1 : sub.N;
    // Gauss-Seidel / DD(GS) down to level cheb_from - 1, Chebyshev below
    const bool sgs_here = sgs && !(amg.cheb_from >= 1 && l >= amg.cheb_from);
    for (int i = 0; i < nchb; ++i) {
      if (sgs_here) {
        if (amg.smoother == 2) M.cheb[i].setup_ddgs(L.A.at(i, i), L.bs[i], omega, steps, C.o.seed, nullptr, amg.ddmin);
        else M.cheb[i].setup_sgs(L.A.at(i, i), L.bs[i], omega, steps, C.o.seed);
        M.cheb[i].half = amg.half;
      } else {
        M.cheb[i].setup(L.A.at(i, i), L.lambda[i], lo);
      }
    }
    if (M.kind == 1) {
      if (sub.N < 2) throw Error(EINVAL_, "AMG(SIMPLE) needs at least two fields");
      M.ngroup1 = sub.N - 1;
      M.dtilde_inv = simplec_inv(L.A, M.ngroup1, C.o.simplec_mode);
      M.Stilde = schur_approx(L.A, M.ngroup1, M.dtilde_inv);
      M.schur_direct = M.Stilde.nr <= C.o.schur_direct_max;
      if (M.schur_direct) M.schur_lu.factor(to_dense(M.Stilde), M.Stilde.nr);
      else {
        std::vector<double> d = diagonal(M.Stilde), dinv(d.size());
        for (size_t r = 0; r < d.size(); ++r) dinv[r] = 1.0 / d[r];
        M.schur_cheb.setup(&M.Stilde, power_lambda(M.Stilde, dinv, C.o.seed, C.o.power_its), lo);
      }
    }
  }
  C.hier.push_back(S.get());
  return S;
}

static std::unique_ptr<Solver> build(Ctx& C, const Spec& sp, const BlockMat& A, int f0, int f1,
                                     const std::vector<FieldDesc>& F) {
  const int nf = f1 - f0;
  if (sp.name == "LU") {
    if (!sp.kids.empty()) throw Error(EINVAL_, "spec: LU takes no argument");
    auto S = std::make_unique<LuSolver>();
    BlockMat sub = sub_blocks(A, f0, f1);
    S->n = sub.total();
    S->lu.factor(sub.dense(0, nf), S->n);
    return S;
  }
  if (sp.name == "DDGS") {
    if (!sp.kids.empty()) throw Error(EINVAL_, "spec: DDGS takes no argument");
    if (nf != 1) throw Error(EINVAL_, "spec: DDGS needs a single field");
    const Csr* Aii = A.at(f0, f0);
    if (!Aii) throw Error(ESINGULAR, "DDGS: zero diagonal block");
    auto S = std::make_unique<SmootherSolver>();
    S->sm.setup_ddgs(Aii, F[f0].bs, sp.omega > 0.0 ? sp.omega : 1.0, sp.steps > 0 ? sp.steps : 1, C.o.seed, nullptr,
                     sp.ddmin);
    S->n = Aii->nr;
    return S;
  }
  if (sp.name == "AMG") {
    if (sp.kids.empty()) {
      if (nf != 1) throw Error(EINVAL_, "spec: plain AMG needs a single field; use AMG(BGS) or AMG(SIMPLE)");
      return build_amg(C, A, f0, f1, F, nullptr, sp);
    }
    if (sp.kids.size() != 1 || (sp.kids[0].name != "BGS" && sp.kids[0].name != "SIMPLE"))
      throw Error(EINVAL_, "spec: AMG level smoother must be BGS or SIMPLE");
    return build_amg(C, A, f0, f1, F, &sp.kids[0], sp);
  }
  if (sp.name == "BGS") {
    if (sp.kids.size() != 1) throw Error(EINVAL_, "spec: BGS takes one inner solver");
    auto S = std::make_unique<BgsSolver>();
    S->A = &A;
    S->f0 = f0;
    S->f1 = f1;
    S->sweeps = sp.sweeps > 0 ? sp.sweeps : C.o.sweeps;
    S->order = sp.order >= 0 ? sp.order : C.o.order;
    int n = 0;
    for (int i = f0; i < f1; ++i) {
      if (!A.at(i, i)) throw Error(ESINGULAR, "BGS: zero diagonal block");
      S->child.push_back(build(C, sp.kids[0], A, i, i + 1, F));
      n += A.size[i];
    }
    S->n = n;
    return S;
  }
  if (sp.name == "SIMPLE") {
    if (sp.kids.empty() || sp.kids.size() > 2) throw Error(EINVAL_, "spec: SIMPLE(pred[;schur])");
    if (nf < 2) throw Error(EINVAL_, "SIMPLE needs at least two fields");
    // groups: predictor = fields with split 0, Schur = fields with split 1;
    // default the last field is the Schur field.  Groups must be contiguous
    // and the Schur group a single field.
    int g = f1 - 1;
    if (!C.o.split.empty()) {
      int cnt = 0;
      for (int i = f0; i < f1; ++i) if (C.o.split[i] == 1) { ++cnt; g = i; }
      if (cnt != 1 || g != f1 - 1) throw Error(EINVAL_, "SIMPLE: the Schur group must be the last single field");
    }
    auto S = std::make_unique<SimpleSolver>();
    S->A = &A;
    S->f0 = f0;
    S->f1 = f1;
    S->g = g;
    S->sweeps = sp.sweeps > 0 ? sp.sweeps : 1;
    BlockMat sub = sub_blocks(A, f0, f1);
    const int gl = g - f0;
    S->dtinv = simplec_inv(sub, gl, C.o.simplec_mode);
    S->pred = build(C, sp.kids[0], A, f0, g, F);
    // Schur field as a new one-field system
    auto Sm = std::make_unique<BlockMat>();
    Sm->N = 1;
    Sm->size = {A.size[g]};
    Sm->blk = {std::make_shared<Csr>(schur_approx(sub, gl, S->dtinv))};
    std::vector<FieldDesc> Fs = {F[g]};
    Spec def;
    def.name = A.size[g] <= C.o.schur_direct_max ? "LU" : "AMG";
    const Spec& ss = sp.kids.size() == 2 ? sp.kids[1] : def;
    S->schur = build(C, ss, *Sm, 0, 1, Fs);
    C.owned.push_back(std::move(Sm));
    int n = 0;
    for (int i = f0; i < f1; ++i) n += A.size[i];
    S->n = n;
    return S;
  }
  throw Error(EINVAL_, "spec: unknown method " + sp.name);
}

// ----------------------------------------------------------- GMRES
// Restarted GMRES(m) on A x = b with right preconditioning (Sec. 3.2):
// Arnoldi on A M, modified Gram-Schmidt, Givens rotations.  Plain form:
// x += M (V y) at the end of a cycle; flexible form keeps Z = [M v_j] and
// does x += Z y.  Stop when |g_{j+1}| / ||r0|| < rtol, confirmed by the true
// residual (a failed confirmation restarts).  A breakdown (||w|| <= 1e-300
// after the orthogonalisation: the Krylov space is invariant) ends the
// cycle; if the true residual then still fails the test, a restart would
// rebuild the same space, and the solve ends with EBREAKDOWN.  A zero on the
// diagonal of the rotated Hessenberg matrix (A M singular on the space)
// gives a zero coefficient in the back substitution.
struct SolveOpts { int restart = 50, maxit = 1000, flexible = 0; double rtol = 1e-8; };
struct Stats { int iters = 0, restarts = 0, status = 0; double relres = 0, setup_s = 0, solve_s = 0, bytes = 0, gbps = 0; };

static Stats gmres(const BlockMat& A, Solver& M, const double* b, double* x, const SolveOpts& so) {
  const int n = A.total(), m = so.restart;
  Stats st;
  std::vector<double> r(n), w(n), z(n);
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n)), Z;
  if (so.flexible) Z.assign(m, std::vector<double>(n));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  auto residual = [&]() {
    A.apply(0, A.N, x, r.data());
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    return nrm2(n, r.data());
  };
  const double beta0 = residual();
  for (int i = 0; i < n; ++i) if (!std::isfinite(b[i])) { st.status = ENAN; return st; }
  if (beta0 == 0.0) { st.status = OK; return st; }
  int total = 0;
  bool first = true, broke = false;
  while (true) {
    const double beta = first ? beta0 : residual();
    first = false;
    st.relres = beta / beta0;
    if (!std::isfinite(beta)) { st.status = ENAN; break; }
    if (beta / beta0 < so.rtol) { st.status = OK; break; }
    if (broke) { st.status = EBREAKDOWN; break; }
    if (total >= so.maxit) { st.status = NOT_CONVERGED; break; }
    if (total > 0) st.restarts++;
    for (int i = 0; i < n; ++i) V[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* zj = so.flexible ? Z[j].data() : z.data();
      M.apply(V[j].data(), zj);
      A.apply(0, A.N, zj, w.data());
      for (int i = 0; i <= j; ++i) {
        double h = dot(n, w.data(), V[i].data());
        H[(size_t)i * m + j] = h;
        for (int q = 0; q < n; ++q) w[q] -= h * V[i][q];
      }
      const double hn = nrm2(n, w.data());
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {   // previous rotations
        double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, c);
      cs[j] = den == 0.0 ? 1.0 : a / den;
      sn[j] = den == 0.0 ? 0.0 : c / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      jend = j + 1;
      if (!std::isfinite(g[j + 1])) break;
      if (hn <= 1e-300) { broke = true; break; }
      if (std::fabs(g[j + 1]) / beta0 < so.rtol || total >= so.maxit) break;
      for (int q = 0; q < n; ++q) V[j + 1][q] = w[q] / hn;
    }
    for (int i = jend - 1; i >= 0; --i) {   // back substitution H y = g
      double s = g[i];
      for (int k = i + 1; k < jend; ++k) s -= H[(size_t)i * m + k] * y[k];
      y[i] = H[(size_t)i * m + i] != 0.0 ? s / H[(size_t)i * m + i] : 0.0;
    }
    if (so.flexible) {
      for (int k = 0; k < jend; ++k)
        for (int q = 0; q < n; ++q) x[q] += y[k] * Z[k][q];
    } else {
      std::fill(w.begin(), w.end(), 0.0);
      for (int k = 0; k < jend; ++k)
        for (int q = 0; q < n; ++q) w[q] += y[k] * V[k][q];
      M.apply(w.data(), z.data());
      for (int q = 0; q < n; ++q) x[q] += z[q];
    }
  }
  st.iters = total;
  return st;
}

}  // namespace orc

// =========================================================================
// C interface used by the Python tests (ctypes).  Struct layouts are this
// file's own.
// =========================================================================
extern "C" {

typedef struct { int32_t nrows, ncols; int64_t nnz; const int64_t* rowptr; const int32_t* colind; const double* val; } orc_csr;
typedef struct { int32_t ndof, block_size, nns; const double* nullspace; } orc_field;
typedef struct {
  int32_t sweeps, order, coarse_max, max_levels, cheb_degree, power_its;
  double cheb_ratio, cheb_boost;
  int32_t simplec_mode;
  const int32_t* split;
  int32_t schur_direct_max, hier_fp32;
  uint64_t seed;
} orc_opts;
typedef struct { int32_t restart, maxit, flexible; double rtol; } orc_solve_opts;
typedef struct { int32_t iters, restarts, status; double relres, setup_s, solve_s, bytes, gbps; } orc_stats;

static thread_local std::string g_err;

const char* orc_last_error(void) { return g_err.c_str(); }

static orc::Csr from_c(const orc_csr& c) {
  orc::Csr A;
  A.nr = c.nrows;
  A.nc = c.ncols;
  A.ptr.assign(c.rowptr, c.rowptr + c.nrows + 1);
  if (A.ptr[0] != 0) throw orc::Error(orc::EINVAL_, "csr: rowptr[0] != 0");
  for (int i = 0; i < A.nr; ++i) {
    if (A.ptr[i + 1] < A.ptr[i]) throw orc::Error(orc::EINVAL_, "csr: rowptr decreasing");
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      if (c.colind[p] < 0 || c.colind[p] >= A.nc) throw orc::Error(orc::EINVAL_, "csr: column out of range");
      if (p > A.ptr[i] && c.colind[p] <= c.colind[p - 1]) throw orc::Error(orc::EINVAL_, "csr: columns not strictly increasing");
    }
  }
  if (A.ptr[A.nr] != c.nnz) throw orc::Error(orc::EINVAL_, "csr: nnz mismatch");
  A.col.assign(c.colind, c.colind + c.nnz);
  A.val.assign(c.val, c.val + c.nnz);
  return A;
}

static orc::Opts opts_from_c(const orc_opts* o, int nfields) {
  orc::Opts r;
  if (!o) return r;
  r.sweeps = o->sweeps;
  r.order = o->order;
  r.coarse_max = o->coarse_max;
  r.max_levels = o->max_levels;
  r.cheb_degree = o->cheb_degree;
  r.power_its = o->power_its;
  r.cheb_ratio = o->cheb_ratio;
  r.cheb_boost = o->cheb_boost;
  r.simplec_mode = o->simplec_mode;
  if (o->split) r.split.assign(o->split, o->split + nfields);
  r.schur_direct_max = o->schur_direct_max;
  r.seed = o->seed;
  return r;
}

int orc_setup(int32_t nfields, const orc_field* fields, const orc_csr* blocks, const char* spec,
              const orc_opts* opts, void** out) {
  try {
    auto t0 = std::chrono::steady_clock::now();
    auto C = std::make_unique<orc::Ctx>();
    C->o = opts_from_c(opts, nfields);
    C->A.N = nfields;
    C->A.size.resize(nfields);
    C->A.blk.resize((size_t)nfields * nfields);
    for (int i = 0; i < nfields; ++i) {
      orc::FieldDesc f;
      f.ndof = fields[i].ndof;
      f.bs = fields[i].block_size;
      f.nns = fields[i].nns;
      if (f.ndof <= 0 || f.bs <= 0 || f.ndof % f.bs || f.nns < 0) throw orc::Error(orc::EINVAL_, "field description");
      if (f.nns > 0 && fields[i].nullspace)
        f.B.assign(fields[i].nullspace, fields[i].nullspace + (size_t)f.ndof * f.nns);
      C->F.push_back(f);
      C->A.size[i] = f.ndof;
    }
    for (int i = 0; i < nfields; ++i)
      for (int j = 0; j < nfields; ++j) {
        const orc_csr& b = blocks[(size_t)i * nfields + j];
        if (b.nnz == 0 || b.val == nullptr) continue;
        if (b.nrows != C->A.size[i] || b.ncols != C->A.size[j]) throw orc::Error(orc::EINVAL_, "block dims disagree with fields");
        C->A.blk[(size_t)i * nfields + j] = std::make_shared<orc::Csr>(from_c(b));
      }
    orc::Parser P(spec);
    orc::Spec sp = P.parse();
    if (spec[P.i] != 0) throw orc::Error(orc::EINVAL_, "spec: trailing characters");
    C->root = orc::build(*C, sp, C->A, 0, nfields, C->F);
    C->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = C.release();
    return 0;
  } catch (orc::Error& e) {
    g_err = e.what();
    return e.code;
  } catch (std::exception& e) {
    g_err = e.what();
    return orc::ENOMEM_;
  }
}

void orc_destroy(void* c) { delete (orc::Ctx*)c; }

int orc_precond_apply(void* c, const double* r, double* z, int32_t nrhs) {
  auto* C = (orc::Ctx*)c;
  try {
    const int n = C->A.total();
    for (int k = 0; k < nrhs; ++k) C->root->apply(r + (size_t)k * n, z + (size_t)k * n);
    return 0;
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

int orc_apply_matrix(void* c, const double* x, double* y, int32_t nrhs) {
  auto* C = (orc::Ctx*)c;
  const int n = C->A.total();
  for (int k = 0; k < nrhs; ++k) C->A.apply(0, C->A.N, x + (size_t)k * n, y + (size_t)k * n);
  return 0;
}

int orc_gmres_solve(void* c, const double* b, double* x, int32_t nrhs, const orc_solve_opts* so,
                    orc_stats* stats) {
  auto* C = (orc::Ctx*)c;
  try {
    orc::SolveOpts s;
    if (so) { s.restart = so->restart; s.maxit = so->maxit; s.flexible = so->flexible; s.rtol = so->rtol; }
    const int n = C->A.total();
    int worst = 0;
    for (int k = 0; k < nrhs; ++k) {
      auto t0 = std::chrono::steady_clock::now();
      orc::Stats st = orc::gmres(C->A, *C->root, b + (size_t)k * n, x + (size_t)k * n, s);
      double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (stats) {
        stats[k].iters = st.iters;
        stats[k].restarts = st.restarts;
        stats[k].status = st.status;
        stats[k].relres = st.relres;
        stats[k].setup_s = C->setup_s;
        stats[k].solve_s = dt;
        stats[k].bytes = 0;
        stats[k].gbps = 0;
      }
      if (st.status < 0) return st.status;
      if (st.status > worst) worst = st.status;
    }
    return worst;
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

// ---- inspection of the hierarchies a context built (build order) ----
int orc_hier_count(void* c) { return (int)((orc::Ctx*)c)->hier.size(); }
int orc_hier_nlevels(void* c, int h) { return (int)((orc::Ctx*)c)->hier[h]->H.lev.size(); }
int orc_hier_nfields(void* c, int h) { return ((orc::Ctx*)c)->hier[h]->H.N; }
int orc_hier_size(void* c, int h, int l, int f) { return ((orc::Ctx*)c)->hier[h]->H.lev[l].A.size[f]; }
double orc_hier_lambda(void* c, int h, int l, int f) {
  const auto& L = ((orc::Ctx*)c)->hier[h]->H.lev[l];
  return f < (int)L.lambda.size() ? L.lambda[f] : 0.0;
}
int orc_hier_block_size(void* c, int h, int l, int f) { return ((orc::Ctx*)c)->hier[h]->H.lev[l].bs[f]; }

// which: 0 = A_ij, 1 = P_i, 2 = R_i.  Returns nnz (or -1 if absent); fills
// the arrays when they are non-null.
int64_t orc_hier_matrix(void* c, int h, int l, int which, int i, int j, int64_t* ptr, int32_t* col,
                        double* val, int32_t* nr, int32_t* nc) {
  const auto& L = ((orc::Ctx*)c)->hier[h]->H.lev[l];
  const orc::Csr* M = nullptr;
  if (which == 0) M = L.A.at(i, j);
  else if (which == 1 && i < (int)L.P.size()) M = &L.P[i];
  else if (which == 2 && i < (int)L.R.size()) M = &L.R[i];
  if (!M) return -1;
  if (nr) *nr = M->nr;
  if (nc) *nc = M->nc;
  if (ptr) std::copy(M->ptr.begin(), M->ptr.end(), ptr);
  if (col) std::copy(M->col.begin(), M->col.end(), col);
  if (val) std::copy(M->val.begin(), M->val.end(), val);
  return M->nnz();
}

// aggregate id per node on level l for field f (returns node count, or -1)
int orc_hier_aggregates(void* c, int h, int l, int f, int32_t* out) {
  const auto& L = ((orc::Ctx*)c)->hier[h]->H.lev[l];
  if (f >= (int)L.agg.size() || L.agg[f].empty()) return -1;
  if (out) std::copy(L.agg[f].begin(), L.agg[f].end(), out);
  return (int)L.agg[f].size();
}

int orc_hier_nullspace(void* c, int h, int l, int f, double* out) {
  const auto& L = ((orc::Ctx*)c)->hier[h]->H.lev[l];
  if (out) std::copy(L.B[f].begin(), L.B[f].end(), out);
  return (int)L.B[f].size();
}

// ---- building blocks exposed for pinning tests ----
int64_t orc_node_graph(int32_t n, int32_t b, const int64_t* rowptr, const int32_t* col,
                       int64_t* gptr, int32_t* gadj) {
  try {
    orc::Csr A;
    A.nr = A.nc = n;
    A.ptr.assign(rowptr, rowptr + n + 1);
    A.col.assign(col, col + rowptr[n]);
    A.val.assign(rowptr[n], 1.0);
    orc::Graph G = orc::node_graph(A, b);
    if (gptr) std::copy(G.ptr.begin(), G.ptr.end(), gptr);
    if (gadj) std::copy(G.adj.begin(), G.adj.end(), gadj);
    return (int64_t)G.adj.size();
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

int orc_mis2_aggregate(int32_t nnode, const int64_t* gptr, const int32_t* gadj, uint64_t seed,
                       int32_t* state, int32_t* agg) {
  try {
    orc::Graph G;
    G.n = nnode;
    G.ptr.assign(gptr, gptr + nnode + 1);
    G.adj.assign(gadj, gadj + gptr[nnode]);
    std::vector<int> st = orc::mis2(G, seed);
    int na = 0;
    std::vector<int> a = orc::aggregate(G, st, &na);
    if (state) std::copy(st.begin(), st.end(), state);
    if (agg) std::copy(a.begin(), a.end(), agg);
    return na;
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

// P_tent for given aggregates; returns number of dead coarse dofs.
int orc_tentative(int32_t nnode, const int32_t* agg, int32_t n_agg, int32_t b, int32_t k,
                  const double* B, int64_t* pptr, int32_t* pcol, double* pval, double* Bc) {
  std::vector<int> a(agg, agg + nnode);
  std::vector<double> Bv(B, B + (size_t)k * nnode * b);
  orc::Tentative T = orc::tentative(a, n_agg, b, k, Bv);
  std::copy(T.P.ptr.begin(), T.P.ptr.end(), pptr);
  std::copy(T.P.col.begin(), T.P.col.end(), pcol);
  std::copy(T.P.val.begin(), T.P.val.end(), pval);
  std::copy(T.Bc.begin(), T.Bc.end(), Bc);
  return (int)T.dead.size();
}

double orc_power_lambda(int32_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                        uint64_t seed, int32_t its) {
  orc::Csr A;
  A.nr = A.nc = n;
  A.ptr.assign(rowptr, rowptr + n + 1);
  A.col.assign(col, col + rowptr[n]);
  A.val.assign(val, val + rowptr[n]);
  std::vector<double> d = orc::diagonal(A), dinv(n);
  for (int i = 0; i < n; ++i) dinv[i] = 1.0 / d[i];
  return orc::power_lambda(A, dinv, seed, its);
}

// degree-k Chebyshev smoother applied once (for closed-form tests)
int orc_chebyshev(int32_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                  double lambda, double ratio, double boost, int32_t degree, const double* b,
                  double* x, int32_t zero_guess) {
  try {
    orc::Csr A;
    A.nr = A.nc = n;
    A.ptr.assign(rowptr, rowptr + n + 1);
    A.col.assign(col, col + rowptr[n]);
    A.val.assign(val, val + rowptr[n]);
    orc::Opts o;
    o.cheb_ratio = ratio;
    o.cheb_boost = boost;
    o.cheb_degree = degree;
    orc::Cheb c;
    c.setup(&A, lambda, o);
    c.apply(b, x, zero_guess != 0);
    return 0;
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

uint64_t orc_splitmix64(uint64_t x) { return orc::splitmix64(x); }

// greedy colouring of a node graph; returns the number of colours
int orc_color_nodes(int32_t nnode, const int64_t* gptr, const int32_t* gadj, uint64_t seed, int32_t* color) {
  orc::Graph G;
  G.n = nnode;
  G.ptr.assign(gptr, gptr + nnode + 1);
  G.adj.assign(gadj, gadj + gptr[nnode]);
  int nc = 0;
  std::vector<int> c = orc::color_nodes(G, seed, &nc);
  std::copy(c.begin(), c.end(), color);
  return nc;
}

// one application of the multicolour SGS smoother (for splitting-form tests);
// dd: the DD(GS) smoother instead, with subdomains sub (node -> subdomain;
// NULL: the aggregates)
int orc_sgs(int32_t n, const int64_t* rowptr, const int32_t* col, const double* val, int32_t b, double omega,
            int32_t steps, uint64_t seed, const double* rhs, double* x, int32_t zero_guess, int32_t half, int32_t dd,
            const int32_t* sub) {
  try {
    orc::Csr A;
    A.nr = A.nc = n;
    A.ptr.assign(rowptr, rowptr + n + 1);
    A.col.assign(col, col + rowptr[n]);
    A.val.assign(val, val + rowptr[n]);
    orc::Cheb c;
    if (dd) c.setup_ddgs(&A, b, omega, steps, seed, sub);
    else c.setup_sgs(&A, b, omega, steps, seed);
    c.half = half;
    c.apply(rhs, x, zero_guess != 0, zero_guess != 0);
    return 0;
  } catch (orc::Error& e) { g_err = e.what(); return e.code; }
}

}  // extern "C"

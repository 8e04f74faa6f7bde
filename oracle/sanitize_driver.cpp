// TEST INFRASTRUCTURE ONLY: a standalone driver of the oracle's C API, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test suite.
// It assembles a small coupled two-field system (a 2-dof vector Laplacian
// and a scalar reaction-diffusion field on a k x k grid, coupled both ways),
// builds every preconditioner form the oracle has on it, solves, applies,
// inspects the hierarchies and calls the standalone building blocks.  Exit
// status 0 when every call succeeded and every solve converged; a sanitizer
// finding aborts the run with its report.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

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
int orc_setup(int32_t, const orc_field*, const orc_csr*, const char*, const orc_opts*, void**);
void orc_destroy(void*);
int orc_precond_apply(void*, const double*, double*, int32_t);
int orc_apply_matrix(void*, const double*, double*, int32_t);
int orc_gmres_solve(void*, const double*, double*, int32_t, const orc_solve_opts*, orc_stats*);
int orc_hier_count(void*);
int orc_hier_nlevels(void*, int);
int orc_hier_nfields(void*, int);
int orc_hier_size(void*, int, int, int);
int64_t orc_hier_matrix(void*, int, int, int, int, int, int64_t*, int32_t*, double*, int32_t*, int32_t*);
int orc_hier_aggregates(void*, int, int, int, int32_t*);
int64_t orc_node_graph(int32_t, int32_t, const int64_t*, const int32_t*, int64_t*, int32_t*);
int orc_mis2_aggregate(int32_t, const int64_t*, const int32_t*, uint64_t, int32_t*, int32_t*);
int orc_color_nodes(int32_t, const int64_t*, const int32_t*, uint64_t, int32_t*);
double orc_power_lambda(int32_t, const int64_t*, const int32_t*, const double*, uint64_t, int32_t);
int orc_chebyshev(int32_t, const int64_t*, const int32_t*, const double*, double, double, double, int32_t,
                  const double*, double*, int32_t);
int orc_sgs(int32_t, const int64_t*, const int32_t*, const double*, int32_t, double, int32_t, uint64_t, const double*,
            double*, int32_t, int32_t, int32_t, const int32_t*);
const char* orc_last_error(void);
}

namespace {

struct Csr {
  int nr = 0, nc = 0;
  std::vector<int64_t> ptr{0};
  std::vector<int32_t> col;
  std::vector<double> val;
  orc_csr view() const { return {nr, nc, (int64_t)col.size(), ptr.data(), col.data(), val.data()}; }
};

// 5-point operator on a k x k grid with b dofs per node (dof-major inside a
// node), diagonal d, off-diagonal -1 between equal dofs of neighbouring nodes
Csr grid_operator(int k, int b, double d, double cross) {
  Csr A;
  A.nr = A.nc = k * k * b;
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i)
      for (int q = 0; q < b; ++q) {
        const int node = j * k + i;
        std::vector<std::pair<int, double>> row;
        auto add = [&](int nn, int qq, double v) { row.push_back({nn * b + qq, v}); };
        if (j > 0) add(node - k, q, -1.0);
        if (i > 0) add(node - 1, q, -1.0);
        for (int qq = 0; qq < b; ++qq) add(node, qq, qq == q ? d : cross);
        if (i + 1 < k) add(node + 1, q, -1.0);
        if (j + 1 < k) add(node + k, q, -1.0);
        for (auto& e : row) {
          A.col.push_back(e.first);
          A.val.push_back(e.second);
        }
        A.ptr.push_back((int64_t)A.col.size());
      }
  return A;
}

// coupling: row node i of a (ba dofs) to column node i of b (bb dofs), weight w
Csr coupling(int nodes, int ba, int bb, double w) {
  Csr C;
  C.nr = nodes * ba;
  C.nc = nodes * bb;
  for (int n = 0; n < nodes; ++n)
    for (int q = 0; q < ba; ++q) {
      for (int qq = 0; qq < bb; ++qq) {
        C.col.push_back(n * bb + qq);
        C.val.push_back(w * (1.0 + 0.1 * q - 0.05 * qq));
      }
      C.ptr.push_back((int64_t)C.col.size());
    }
  return C;
}

int failures = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, orc_last_error());
    ++failures;
  }
}

}  // namespace

int main() {
  const int k = 14, nodes = k * k;
  const Csr A = grid_operator(k, 2, 4.2, 0.3), B = grid_operator(k, 1, 4.5, 0.0);
  const Csr CAB = coupling(nodes, 2, 1, 0.05), CBA = coupling(nodes, 1, 2, -0.02);
  const int na = A.nr, nb = B.nr, n = na + nb;
  // near-nullspaces: the two translations for A, the constant for B
  std::vector<double> nsA((size_t)na * 2, 0.0), nsB(nb, 1.0);
  for (int i = 0; i < nodes; ++i) {
    nsA[(size_t)2 * i] = 1.0;
    nsA[(size_t)na + 2 * i + 1] = 1.0;
  }
  const orc_field fields[2] = {{na, 2, 2, nsA.data()}, {nb, 1, 1, nsB.data()}};
  const orc_csr blocks[4] = {A.view(), CAB.view(), CBA.view(), B.view()};
  std::vector<double> rhs(n), x(n), z(n), y(n);
  for (int i = 0; i < n; ++i) rhs[i] = std::sin(0.37 * i) + 0.1;
  const int32_t split[2] = {0, 1};
  const char* specs[] = {"BGS(AMG)",
                         "BGS[sweeps=2,order=sym](AMG[degree=3])",
                         "BGS(AMG[smoother=sgs,omega=0.8,half=1,steps=2])",
                         "BGS(AMG[smoother=ddgs,omega=0.8,half=1,ddmin=1])",
                         "BGS(DDGS[omega=0.8,ddmin=1])",
                         "BGS(AMG[pg=1])",
                         "BGS(AMG[smoother=sgs,omega=0.9,half=1,pg=1])",
                         "AMG(BGS)",
                         "AMG[smoother=sgs,omega=0.9](BGS[order=fwd])",
                         "SIMPLE(AMG;AMG)",
                         "SIMPLE(LU;AMG[smoother=sgs,omega=0.9])",
                         "BGS(LU)"};
  for (const char* spec : specs) {
    for (int mode = 0; mode < 3; ++mode) {
      orc_opts o;
      std::memset(&o, 0, sizeof(o));
      o.sweeps = 1;
      o.order = 1;
      o.coarse_max = 40;
      o.cheb_degree = 2;
      o.power_its = 10;
      o.cheb_ratio = 30.0;
      o.cheb_boost = 1.1;
      o.simplec_mode = mode;
      o.split = split;
      o.schur_direct_max = 64;
      o.seed = 7;
      void* ctx = nullptr;
      const int rc = orc_setup(2, fields, blocks, spec, &o, &ctx);
      check(rc == 0, spec);
      if (rc != 0) continue;
      for (int flex = 0; flex < 2; ++flex) {
        std::fill(x.begin(), x.end(), 0.0);
        orc_solve_opts so = {20, 400, flex, 1e-8};
        orc_stats st;
        check(orc_gmres_solve(ctx, rhs.data(), x.data(), 1, &so, &st) == 0 && st.status == 0, spec);
        check(orc_apply_matrix(ctx, x.data(), y.data(), 1) == 0, "matvec");
        double r2 = 0.0, b2 = 0.0;
        for (int i = 0; i < n; ++i) {
          r2 += (rhs[i] - y[i]) * (rhs[i] - y[i]);
          b2 += rhs[i] * rhs[i];
        }
        check(std::sqrt(r2 / b2) < 1e-7, "true residual");
      }
      check(orc_precond_apply(ctx, rhs.data(), z.data(), 1) == 0, "precond apply");
      for (int h = 0; h < orc_hier_count(ctx); ++h)
        for (int l = 0; l < orc_hier_nlevels(ctx, h); ++l)
          for (int f = 0; f < orc_hier_nfields(ctx, h); ++f) {
            const int sz = orc_hier_size(ctx, h, l, f);
            int32_t nr = 0, nc = 0;
            const int64_t nnz = orc_hier_matrix(ctx, h, l, 0, f, f, nullptr, nullptr, nullptr, &nr, &nc);
            if (nnz >= 0) {
              std::vector<int64_t> ptr(nr + 1);
              std::vector<int32_t> col(nnz > 0 ? nnz : 1);
              std::vector<double> val(nnz > 0 ? nnz : 1);
              orc_hier_matrix(ctx, h, l, 0, f, f, ptr.data(), col.data(), val.data(), nullptr, nullptr);
              check(nr == sz && ptr[nr] == nnz, "hierarchy matrix");
            }
            const int nagg = orc_hier_aggregates(ctx, h, l, f, nullptr);
            if (nagg > 0) {
              std::vector<int32_t> agg(nagg);
              orc_hier_aggregates(ctx, h, l, f, agg.data());
            }
          }
      orc_destroy(ctx);
    }
  }
  // building blocks on field A's matrix
  std::vector<int64_t> gptr(nodes + 1);
  const int64_t ne = orc_node_graph(na, 2, A.ptr.data(), A.col.data(), gptr.data(), nullptr);
  check(ne > 0, "node graph");
  std::vector<int32_t> gadj(ne), state(nodes), agg(nodes), color(nodes);
  orc_node_graph(na, 2, A.ptr.data(), A.col.data(), gptr.data(), gadj.data());
  check(orc_mis2_aggregate(nodes, gptr.data(), gadj.data(), 3, state.data(), agg.data()) > 0, "mis2");
  check(orc_color_nodes(nodes, gptr.data(), gadj.data(), 3, color.data()) > 0, "colouring");
  const double lam = orc_power_lambda(na, A.ptr.data(), A.col.data(), A.val.data(), 5, 10);
  check(lam > 0.0, "power iteration");
  std::vector<double> xa(na, 0.0);
  check(orc_chebyshev(na, A.ptr.data(), A.col.data(), A.val.data(), lam, 30.0, 1.1, 3, rhs.data(), xa.data(), 1) == 0,
        "chebyshev");
  for (int dd = 0; dd < 2; ++dd)
    for (int half = 0; half < 3; ++half) {
      std::fill(xa.begin(), xa.end(), 0.0);
      check(orc_sgs(na, A.ptr.data(), A.col.data(), A.val.data(), 2, 0.9, 2, 3, rhs.data(), xa.data(), 1, half, dd,
                    dd ? agg.data() : nullptr) == 0,
            "sgs");
    }
  // error paths: a malformed spec and a block whose columns are out of order
  void* bad = nullptr;
  check(orc_setup(2, fields, blocks, "BGS(AMG", nullptr, &bad) != 0, "malformed spec rejected");
  Csr Abad = A;
  std::swap(Abad.col[1], Abad.col[2]);
  const orc_csr bad_blocks[4] = {Abad.view(), CAB.view(), CBA.view(), B.view()};
  check(orc_setup(2, fields, bad_blocks, "BGS(AMG)", nullptr, &bad) != 0, "unsorted columns rejected");
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("sanitized oracle driver: all checks passed\n");
  return 0;
}

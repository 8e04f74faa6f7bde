// Device-resident block matrices and (monolithic) smoothed-aggregation AMG
// hierarchies.
#pragma once

#include <memory>

#include "kernels.hpp"

namespace nf {

struct Opts {
  int sweeps = 1, order = 1, coarse_max = 200, max_levels = 10, cheb_degree = 2, power_its = 10;
  double cheb_ratio = 30.0, cheb_boost = 1.1;
  int simplec_mode = 0;
  std::vector<int> split;
  int schur_direct_max = 5000;
  int hier_fp32 = 0;
  uint64_t seed = 0;
  int graphs = 0;
  int block_products = 1;
  int parallel_setup = 1;
  int max_rhs = NRMAX;
  int pg = 0;   // Petrov-Galerkin transfers (per AMG node of the specification)
};

// N x N grid of device blocks over fields [0, N); a null block is zero.
struct BlockMat {
  int N = 0;
  std::vector<int> size;
  std::vector<std::shared_ptr<DCsr>> blk;
  const DCsr* at(int i, int j) const { return blk[(size_t)i * N + j].get(); }
  std::vector<int> offsets() const {
    std::vector<int> o(N + 1, 0);
    for (int i = 0; i < N; ++i) o[i + 1] = o[i] + size[i];
    return o;
  }
  int total() const {
    int t = 0;
    for (int v : size) t += v;
    return t;
  }
  BlockMat sub(int f0, int f1) const {
    BlockMat S;
    S.N = f1 - f0;
    S.size.assign(size.begin() + f0, size.begin() + f1);
    S.blk.resize((size_t)S.N * S.N);
    for (int i = 0; i < S.N; ++i)
      for (int j = 0; j < S.N; ++j) S.blk[(size_t)i * S.N + j] = blk[(size_t)(i + f0) * N + (j + f0)];
    return S;
  }
};

struct FieldDev {
  int ndof = 0, bs = 1, nns = 0;
  std::shared_ptr<DBuf<double>> B;   // (nns, ndof) row-major
};

struct Level {
  BlockMat A;
  std::vector<std::unique_ptr<DCsr>> P, R;      // per field, empty on the coarsest level
  std::vector<std::shared_ptr<DBuf<int>>> agg;  // per field node -> aggregate (null if P = I)
  std::vector<std::shared_ptr<DBuf<double>>> B; // per field near-nullspace
  std::vector<int> bs;
  std::vector<double> lambda;                   // per field lambda_max(D^-1 A_ii), 0 if none
  std::vector<std::shared_ptr<DBuf<double>>> dinv;  // per field D^-1 (null if no diagonal)
  std::vector<std::shared_ptr<DBuf<int>>> dead;
  std::vector<int> ndead;
  // per field node graph of A_ii (from aggregation; null where not built)
  std::vector<std::shared_ptr<DBuf<int>>> gptr, gadj;
  std::vector<int> nnode;
};

struct Hierarchy {
  int N = 0;
  std::vector<Level> lev;
  DBuf<double> coarse_inv;   // dense inverse of the coarsest block system (row-major)
  int ncoarse = 0;
};

// Builds the hierarchy over the blocks of A (all fields of A).  Throws
// NfError on singular input.
void build_hierarchy(Hierarchy& H, const BlockMat& A, const std::vector<FieldDev>& F, const Opts& o, hipStream_t s);

// lambda_max(D^-1 A) by power iteration from the seeded start vector.
double power_lambda(const DCsr& A, const double* dinv, uint64_t seed, int its, hipStream_t s);

// Dense inverse of the assembled block system over fields [f0, f1).
void dense_block_inverse(const BlockMat& A, DBuf<double>& inv, int* n_out, hipStream_t s);

}  // namespace nf

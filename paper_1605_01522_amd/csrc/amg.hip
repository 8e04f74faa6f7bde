// Setup of the smoothed-aggregation hierarchies on the device.
//
// Per level and field: the node graph of the diagonal block (pattern only),
// synchronous MIS-2 aggregation, the tentative prolongator from the field's
// near-nullspace (per-aggregate QR), lambda_max(D^-1 A) by power iteration,
// the smoothed prolongator P = (I - 4/(3 lambda) D^-1 A) P_tent, R = P^T and
// the Galerkin products R_i A_ij P_j of every nonzero block (Sec. 3.3 and the
// monolithic transfers of Sec. 4.3).  Fields are coarsened in lockstep; a
// field that is not coarsened on a level (zero diagonal block, already small
// or stalled) keeps P = I there.  The coarsest block system is inverted
// densely.  The host only sequences the launches and reads back sizes.

#include <cmath>

#include "amg.hpp"

namespace nf {

__global__ void k_scale_copy(const double* x, double a, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

double power_lambda(const DCsr& A, const double* dinv, uint64_t seed, int its, hipStream_t s) {
  const int n = A.nr;
  DBuf<double> v(n), w(n), partial(RED_BLOCKS), nrm(1);
  power_start(v.p, n, seed, s);
  normalize(v.p, v.p, n, partial.p, nrm.p, s);
  double lam = 0.0;
  for (int it = 0; it < its; ++it) {
    SpmvArgs<double> a;
    a.x = v.p;
    a.y = w.p;
    a.dinv = dinv;
    a.ldx = a.ldy = n;
    spmv<double>(SPMV_DSCALE, A, a, s);
    normalize(w.p, v.p, n, partial.p, nrm.p, s);
  }
  NF_HIP(hipMemcpyAsync(&lam, nrm.p, sizeof(double), hipMemcpyDeviceToHost, s));
  NF_HIP(hipStreamSynchronize(s));
  return its > 0 ? lam : 0.0;
}

void dense_block_inverse(const BlockMat& A, DBuf<double>& inv, int* n_out, hipStream_t s) {
  const int n = A.total();
  *n_out = n;
  inv.alloc((size_t)n * n > 0 ? (size_t)n * n : 1);
  fill<double>(inv.p, 0.0, (int64_t)n * n, s);
  std::vector<int> o = A.offsets();
  for (int i = 0; i < A.N; ++i)
    for (int j = 0; j < A.N; ++j)
      if (A.at(i, j)) csr_to_dense(*A.at(i, j), inv.p, n, o[i], o[j], s);
  NF_CHECK(dense_inverse(inv.p, n, s) == 0, NFIELD_ESINGULAR, "coarse dense solve: singular matrix");
}

static std::shared_ptr<DBuf<double>> copy_dev(const DBuf<double>& x, hipStream_t s) {
  auto y = std::make_shared<DBuf<double>>(x.n);
  if (x.n) NF_HIP(hipMemcpyAsync(y->p, x.p, x.bytes(), hipMemcpyDeviceToDevice, s));
  return y;
}

// Node blocks pay in a product when the inner block and the output block hold
// more than one entry.
static bool use_blocks(const Opts& o, int br, int bk, int bc) { return o.block_products && bk >= 2 && br * bc >= 2; }

// A field's matrices of one level in block form, converted once and shared by
// the products that need them (A_ii for A P_tent and the Galerkin product,
// P and R = P^T for every Galerkin product of the field's row and column).
struct LevelBlocks {
  std::vector<DBsr> A, P, R;
  std::vector<char> hasA, hasP;
  explicit LevelBlocks(int N) : A(N), P(N), R(N), hasA(N, 0), hasP(N, 0) {}
};

// Galerkin block R_i A_ij P_j (Sec. 3.3): A P first, then R (A P); node
// blocks: R ci x bi, A bi x bj, P bj x cj.  With blocks on both products the
// intermediate A P stays blocked.
static void galerkin(const Opts& o, LevelBlocks& LB, int i, int j, const DCsr& R, const DCsr& A, const DCsr& P, int ci,
                     int bi, int bj, int cj, DCsr& Ac, hipStream_t s) {
  if (use_blocks(o, bi, bj, cj) && use_blocks(o, ci, bi, cj)) {
    DBsr Ab, Pb, Rb, APb, Cb;
    const DBsr* pa = &Ab;
    const DBsr* pp = &Pb;
    const DBsr* pr = &Rb;
    if (i == j && LB.hasA[i]) pa = &LB.A[i];
    else csr_to_bsr(A, bi, bj, Ab, s);
    if (LB.hasP[j]) pp = &LB.P[j];
    else csr_to_bsr(P, bj, cj, Pb, s);
    if (LB.hasP[i]) pr = &LB.R[i];
    else csr_to_bsr(R, ci, bi, Rb, s);
    bspgemm(*pa, *pp, APb, s);
    bspgemm(*pr, APb, Cb, s);
    bsr_to_csr(Cb, Ac, s);
    return;
  }
  DCsr AP;
  if (use_blocks(o, bi, bj, cj)) spgemm_blocked(A, bi, bj, P, cj, AP, s);
  else spgemm(A, P, AP, s);
  if (use_blocks(o, ci, bi, cj)) spgemm_blocked(R, ci, bi, AP, cj, Ac, s);
  else spgemm(R, AP, Ac, s);
}

void build_hierarchy(Hierarchy& H, const BlockMat& A0, const std::vector<FieldDev>& F, const Opts& o, hipStream_t s) {
  const int N = A0.N;
  H.N = N;
  H.lev.clear();
  H.lev.emplace_back();
  {
    Level& L0 = H.lev.back();
    L0.A = A0;
    L0.bs.resize(N);
    L0.B.resize(N);
    L0.dead.resize(N);
    L0.ndead.assign(N, 0);
    for (int i = 0; i < N; ++i) {
      L0.bs[i] = F[i].bs;
      L0.B[i] = F[i].B;
    }
  }
  std::vector<char> active(N);
  for (int i = 0; i < N; ++i) active[i] = A0.at(i, i) != nullptr;
  DBuf<int> zflag(1);
  while (true) {
    const int l = (int)H.lev.size() - 1;
    Level& L = H.lev[l];
    L.gptr.assign(N, nullptr);
    L.gadj.assign(N, nullptr);
    L.nnode.assign(N, 0);
    L.lambda.assign(N, 0.0);
    L.dinv.resize(N);
    for (int i = 0; i < N; ++i) {
      const DCsr* Aii = L.A.at(i, i);
      if (!Aii) continue;
      DBuf<double> d(Aii->nr);
      auto dinv = std::make_shared<DBuf<double>>(Aii->nr);
      fill<int>(zflag.p, 0, 1, s);
      csr_diag(*Aii, d.p, zflag.p, s);
      invert(d.p, dinv->p, Aii->nr, s);
      int z = 0;
      NF_HIP(hipMemcpyAsync(&z, zflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
      NF_HIP(hipStreamSynchronize(s));
      if (!z) {
        L.dinv[i] = dinv;
        L.lambda[i] = power_lambda(*Aii, dinv->p, o.seed, o.power_its, s);
      }
    }
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
    C.ndead.assign(N, 0);
    L.P.resize(N);
    L.R.resize(N);
    L.agg.resize(N);
    LevelBlocks LB(N);
    for (int i = 0; i < N; ++i) {
      const int n = L.A.size[i];
      const bool coarsened = active[i];
      L.P[i] = std::make_unique<DCsr>();
      if (!active[i]) {
        identity(n, *L.P[i], s);
        C.bs[i] = L.bs[i];
        C.B[i] = L.B[i];
        C.dead[i] = L.dead[i];
        C.ndead[i] = L.ndead[i];
      } else {
        const DCsr& Aii = *L.A.at(i, i);
        NF_CHECK(L.lambda[i] > 0.0, NFIELD_ESINGULAR, "AMG: diagonal block has a zero diagonal entry");
        const int k = L.B[i] ? (int)(L.B[i]->n / n) : 0;
        NF_CHECK(k >= 1, NFIELD_EINVAL, "AMG: field has no near-nullspace vectors");
        auto gptr = std::make_shared<DBuf<int>>(), gadj = std::make_shared<DBuf<int>>();
        int nnode = 0;
        node_graph(Aii, L.bs[i], *gptr, *gadj, &nnode, s);
        auto agg = std::make_shared<DBuf<int>>(nnode > 0 ? nnode : 1);
        const int na = mis2_aggregate(nnode, gptr->p, gadj->p, o.seed, agg->p, s);
        // kept for the level's Gauss-Seidel colouring
        L.gptr[i] = gptr;
        L.gadj[i] = gadj;
        L.nnode[i] = nnode;
        DCsr Pt;
        auto Bc = std::make_shared<DBuf<double>>();
        auto dead = std::make_shared<DBuf<int>>();
        const int ndead = tentative(nnode, L.bs[i], k, agg->p, na, L.B[i]->p, Pt, *Bc, *dead, s);
        DCsr AP;
        // B (a field's matrix with b x b node blocks) times a matrix of b x k blocks
        auto times_blocks = [&](const DCsr& Bm, const DBsr* Bb, const DCsr& X, DCsr& out) {
          if (use_blocks(o, L.bs[i], L.bs[i], k)) {
            DBsr Xb, Ob, Bo;
            if (!Bb) {
              csr_to_bsr(Bm, L.bs[i], L.bs[i], Bo, s);
              Bb = &Bo;
            }
            csr_to_bsr(X, L.bs[i], k, Xb, s);
            bspgemm(*Bb, Xb, Ob, s);
            bsr_to_csr(Ob, out, s);
          } else {
            spgemm(Bm, X, out, s);
          }
        };
        if (use_blocks(o, L.bs[i], L.bs[i], k)) {
          csr_to_bsr(Aii, L.bs[i], L.bs[i], LB.A[i], s);
          LB.hasA[i] = 1;
        }
        times_blocks(Aii, LB.hasA[i] ? &LB.A[i] : nullptr, Pt, AP);
        if (o.pg) {
          // Petrov-Galerkin smoothed aggregation: P = P_tent - Q diag(om),
          // Q = D^-1 A P_tent, column dampings minimising ||A P e_j||; the
          // restriction is the same construction on A^T, transposed
          const int nc = na * k;
          auto pg_side = [&](const DCsr& M, const DBsr* Mb, const DCsr& MP, DCsr& out) {
            DCsr Q, MQ;
            csr_copy(MP, Q, s);
            scale_rows(Q, L.dinv[i]->p, s);
            times_blocks(M, Mb, Q, MQ);
            DBuf<double> om(nc > 0 ? nc : 1);
            pg_omega(MP, MQ, om.p, s);
            pg_prolongator(Q, om.p, Pt, L.bs[i], k, agg->p, out, s);
            NF_HIP(hipStreamSynchronize(s));
          };
          DCsr P, At, AtP, PR;
          pg_side(Aii, LB.hasA[i] ? &LB.A[i] : nullptr, AP, P);
          // A^T (and below R) through the block forms where the products
          // run on blocks: the same entries as the scalar transposes
          DBsr Atb;
          const DBsr* atb = nullptr;
          if (LB.hasA[i]) {
            bsr_transpose(LB.A[i], Atb, s);
            atb = &Atb;
          } else {
            transpose(Aii, At, s);
          }
          times_blocks(At, atb, Pt, AtP);
          pg_side(At, atb, AtP, PR);
          *L.P[i] = std::move(P);
          L.R[i] = std::make_unique<DCsr>();
          if (o.block_products && L.bs[i] * k >= 2) {
            DBsr PRb;
            csr_to_bsr(PR, L.bs[i], k, PRb, s);
            bsr_transpose(PRb, LB.R[i], s);
            bsr_to_csr(LB.R[i], *L.R[i], s);
            csr_to_bsr(*L.P[i], L.bs[i], k, LB.P[i], s);
            LB.hasP[i] = 1;
          } else {
            transpose(PR, *L.R[i], s);
          }
        } else {
          DBuf<double> srow(n);
          const double omega = 4.0 / (3.0 * L.lambda[i]);
          if (n > 0) hipLaunchKernelGGL(k_scale_copy, dim3((n + 255) / 256), dim3(256), 0, s, L.dinv[i]->p, -omega, srow.p, (int64_t)n);
          smooth_prolongator(AP, srow.p, Pt, L.bs[i], k, agg->p, s);
          *L.P[i] = std::move(AP);
        }
        L.agg[i] = agg;
        C.bs[i] = k;
        C.B[i] = Bc;
        C.dead[i] = dead;
        C.ndead[i] = ndead;
        if (na * k > 0.83 * n) active[i] = 0;
      }
      if (L.R[i]) continue;   // Petrov-Galerkin: R built above
      L.R[i] = std::make_unique<DCsr>();
      if (o.block_products && coarsened && L.bs[i] * C.bs[i] >= 2) {
        // R = P^T through the block form, which the Galerkin products reuse
        csr_to_bsr(*L.P[i], L.bs[i], C.bs[i], LB.P[i], s);
        bsr_transpose(LB.P[i], LB.R[i], s);
        bsr_to_csr(LB.R[i], *L.R[i], s);
        LB.hasP[i] = 1;
      } else {
        transpose(*L.P[i], *L.R[i], s);
      }
    }
    C.A.N = N;
    C.A.size.resize(N);
    C.A.blk.resize((size_t)N * N);
    for (int i = 0; i < N; ++i) C.A.size[i] = L.P[i]->nc;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const DCsr* Aij = L.A.at(i, j);
        if (!Aij) continue;
        auto Ac = std::make_shared<DCsr>();
        galerkin(o, LB, i, j, *L.R[i], *Aij, *L.P[j], C.bs[i], L.bs[i], L.bs[j], C.bs[j], *Ac, s);
        if (i == j && C.ndead[i] > 0) set_diag_one(*Ac, C.dead[i]->p, C.ndead[i], s);
        C.A.blk[(size_t)i * N + j] = Ac;
      }
    H.lev.push_back(std::move(C));
  }
  dense_block_inverse(H.lev.back().A, H.coarse_inv, &H.ncoarse, s);
  (void)copy_dev;
}

}  // namespace nf

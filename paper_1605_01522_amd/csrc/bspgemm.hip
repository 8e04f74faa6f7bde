// Block-structured sparse products for the Galerkin triple products of the
// AMG setup (R A P, A P) on node-blocked matrices.
//
// A field's matrices are node-blocked: rows and columns come in groups of the
// field's dofs per node (fine level) or near-nullspace vectors per aggregate
// (coarse levels), and their sparsity is a pattern of small dense blocks.
// Hashing scalar columns (one insert per scalar product, most of them repeats)
// then costs far more than the arithmetic.  Here both operands are regrouped
// into blocks of br x bc values with a bitmask of the stored entries, the
// block pattern of the product comes from the scalar product machinery run on
// the (much smaller) block patterns, and every output value is accumulated
// term by term, one A block after another.  Each output entry exists exactly
// when some inner index pairs two stored entries, and its value adds a_ik b_kj
// over exactly those pairs in ascending k (block by block, then within the
// block), which is the pattern and the order of the scalar product: the
// results are the same bits.

#include <climits>

#include "kernels.hpp"
#include "wave.hpp"

namespace nf {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// v[t] = t (the pattern values of a converted matrix: its block indices)
__global__ void k_iota(double* v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) v[t] = (double)t;
}
static void iota(double* v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(cdiv(n, 256)), dim3(256), 0, s, v, n);
}

// ------------------------------------------------------------ CSR -> blocks
// The br scalar rows of block row i are adjacent in CSR, so its entries are
// the range [ptr[i br], ptr[(i + 1) br]).
constexpr int BSR_CAP = 2048;

// one wavefront per block row: its distinct block columns, ascending, into
// the scratch at the row's first entry offset (it has room: one slot per
// entry), their number into cnt[i].  Up to BSR_CAP entries are sorted in
// LDS; longer block rows merge their BR sorted rows serially.
template <int BR>
__global__ __launch_bounds__(64) void k_bsr_keys(int bc, const int* __restrict__ ptr, const int* __restrict__ col,
                                                 int* __restrict__ ucol, int* __restrict__ cnt) {
  __shared__ int keys[BSR_CAP];
  const int i = blockIdx.x, lane = threadIdx.x;
  const int e0 = ptr[i * BR], e1 = ptr[(i + 1) * BR], E = e1 - e0;
  {  // rows with the block columns of the first row: those, ascending
    int n0;
    if (rows_share_groups(ptr, i * BR, BR, bc, col, keys, BSR_CAP, n0)) {
      __syncthreads();
      if (n0 <= BSR_CAP)
        for (int t = lane; t < n0; t += 64) ucol[e0 + t] = keys[t];
      else   // one row (BR = 1) with more block columns than keys holds
        group_runs(e0, ptr[i * BR + 1], bc, col, -1, ucol + e0);
      if (lane == 0) cnt[i] = n0;
      return;
    }
    __syncthreads();   // keys held the first row's block columns
  }
  if (E <= BSR_CAP) {
    int ts = 1;
    while (ts < E) ts <<= 1;
    for (int t = lane; t < ts; t += 64) keys[t] = t < E ? col[e0 + t] / bc : INT_MAX;
    __syncthreads();
    wave_bitonic(keys, ts, lane);
    int n = 0;
    for (int t0 = 0; t0 < E; t0 += 64) {
      const int t = t0 + lane;
      const bool first = t < E && (t == 0 || keys[t - 1] != keys[t]);
      const unsigned long long bal = __ballot(first);
      if (first) ucol[e0 + n + __popcll(bal & ((1ull << lane) - 1ull))] = keys[t];
      n += __popcll(bal);
    }
    if (lane == 0) cnt[i] = n;
    return;
  }
  if (lane != 0) return;
  int pos[BR], end[BR];
#pragma unroll
  for (int q = 0; q < BR; ++q) {
    pos[q] = ptr[i * BR + q];
    end[q] = ptr[i * BR + q + 1];
  }
  int n = 0;
  while (true) {
    int mn = INT_MAX;
#pragma unroll
    for (int q = 0; q < BR; ++q)
      if (pos[q] < end[q]) mn = min(mn, col[pos[q]] / bc);
    if (mn == INT_MAX) break;
#pragma unroll
    for (int q = 0; q < BR; ++q)
      while (pos[q] < end[q] && col[pos[q]] / bc == mn) ++pos[q];
    ucol[e0 + n++] = mn;
  }
  cnt[i] = n;
}

// one wavefront per block row: copy its block columns, then every entry finds
// its block (binary search) and lands at row q, column c inside it, with its
// bit (q bc + c) or-ed into the block's mask: in LDS for rows of up to
// BSR_PLACE_LDS blocks (written out at the end), in global memory (zeroed
// beforehand) beyond
constexpr int BSR_PLACE_LDS = 512;
__global__ __launch_bounds__(64) void k_bsr_place(int br, int bc, const int* __restrict__ ptr, const int* __restrict__ col,
                                                  const double* __restrict__ val, const int* __restrict__ ucol,
                                                  const int* __restrict__ bptr, int* __restrict__ bcol,
                                                  double* __restrict__ bval, unsigned long long* bmask) {
  __shared__ unsigned long long lm[BSR_PLACE_LDS];
  const int i = blockIdx.x, lane = threadIdx.x;
  const int e0 = ptr[i * br], e1 = ptr[(i + 1) * br];
  const int o = bptr[i], n = bptr[i + 1] - o, bb = br * bc;
  const bool in_lds = n <= BSR_PLACE_LDS;
  const int* __restrict__ u = ucol + e0;
  for (int t = lane; t < n; t += 64) {
    bcol[o + t] = u[t];
    if (in_lds) lm[t] = 0ull;
  }
  __syncthreads();
  for (int t = e0 + lane; t < e1; t += 64) {
    int q = 0;
    while (ptr[i * br + q + 1] <= t) ++q;
    const int c = col[t], jb = c / bc;
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (u[mid] < jb) lo = mid + 1; else hi = mid;
    }
    const int cc = c - jb * bc;
    bval[(int64_t)(o + lo) * bb + q * bc + cc] = val[t];
    const unsigned long long bit = 1ull << (q * bc + cc);
    if (in_lds) atomicOr(&lm[lo], bit);
    else atomicOr(&bmask[o + lo], bit);
  }
  if (in_lds) {
    __syncthreads();
    for (int t = lane; t < n; t += 64) bmask[o + t] = lm[t];
  }
}

void csr_to_bsr(const DCsr& A, int br, int bc, DBsr& B, hipStream_t s) {
  NF_CHECK(br >= 1 && br <= 8 && bc >= 1 && bc <= 8, NFIELD_EINVAL, "block product: block size above 8");
  NF_CHECK(A.nr % br == 0 && A.nc % bc == 0, NFIELD_EINVAL, "block product: size not a multiple of the block size");
  B.br = br;
  B.bc = bc;
  B.pat.nr = A.nr / br;
  B.pat.nc = A.nc / bc;
  const int nbr = B.pat.nr;
  B.pat.ptr.alloc(nbr + 1);
  DBuf<int> cnt(nbr + 1), ucol(A.nnz > 0 ? A.nnz : 1);
  if (nbr > 0) {
    switch (br) {
#define NF_BK(R) \
  case R: hipLaunchKernelGGL(k_bsr_keys<R>, dim3(nbr), dim3(64), 0, s, bc, A.ptr.p, A.col.p, ucol.p, cnt.p); break;
      NF_BK(1) NF_BK(2) NF_BK(3) NF_BK(4) NF_BK(5) NF_BK(6) NF_BK(7) NF_BK(8)
#undef NF_BK
    }
  }
  B.pat.nnz = exclusive_scan(cnt.p, B.pat.ptr.p, nbr, s);
  const int64_t nb = B.pat.nnz > 0 ? B.pat.nnz : 1;
  B.pat.col.alloc(nb);
  B.pat.val.alloc(nb);
  B.val.alloc(nb * br * bc);
  B.mask.alloc(nb);
  iota(B.pat.val.p, nb, s);
  fill<double>(B.val.p, 0.0, nb * br * bc, s);
  fill<unsigned long long>(B.mask.p, 0ull, nb, s);
  if (nbr > 0)
    hipLaunchKernelGGL(k_bsr_place, dim3(nbr), dim3(64), 0, s, br, bc, A.ptr.p, A.col.p, A.val.p, ucol.p, B.pat.ptr.p,
                       B.pat.col.p, B.val.p, B.mask.p);
}

// ------------------------------------------------------------ blocks -> CSR
// G lanes per scalar row (G divides 64): the lanes take G blocks of the block
// row at a time, count their stored entries in this row, and (pass 1) write
// them at offsets from a scan across the lanes, so the row comes out in
// ascending column (blocks ascending, then columns inside the block); pass 0
// writes the row's count
template <int G, int PASS>
__global__ void k_bsr_rows(int nr, int br, int bc, const int* __restrict__ bptr, const int* __restrict__ bcol,
                           const double* __restrict__ bval, const unsigned long long* __restrict__ bmask,
                           int* __restrict__ cnt, const int* __restrict__ ptr, int* __restrict__ col,
                           double* __restrict__ val) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = (int)(gid / G), lane = (int)(gid % G);
  if (r >= nr) return;
  const int i = r / br, q = r - i * br, bb = br * bc;
  const unsigned long long rowbits = ((1ull << bc) - 1ull) << (q * bc);
  int n = 0;
  const int o = PASS ? ptr[r] : 0;
  const int p1 = bptr[i + 1];
  for (int p0 = bptr[i]; p0 < p1; p0 += G) {
    const int p = p0 + lane;
    const unsigned long long m = p < p1 ? (bmask[p] & rowbits) : 0ull;
    const int k = __popcll(m);
    int incl = k;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const int t = __shfl_up(incl, d, G);
      if (lane >= d) incl += t;
    }
    if (PASS && m) {
      int w = o + n + incl - k;
      for (int c = 0; c < bc; ++c)
        if ((m >> (q * bc + c)) & 1ull) {
          col[w] = bcol[p] * bc + c;
          val[w] = bval[(int64_t)p * bb + q * bc + c];
          ++w;
        }
    }
    n += __shfl(incl, G - 1, G);
  }
  if (!PASS && lane == 0) cnt[r] = n;
}

template <int G>
static void bsr_rows(const DBsr& B, DCsr& A, int pass, const int* cnt_or_ptr, hipStream_t s) {
  const int blocks = cdiv((int64_t)A.nr * G, 256);
  if (pass == 0)
    hipLaunchKernelGGL((k_bsr_rows<G, 0>), dim3(blocks), dim3(256), 0, s, A.nr, B.br, B.bc, B.pat.ptr.p, B.pat.col.p,
                       B.val.p, B.mask.p, (int*)cnt_or_ptr, (const int*)nullptr, (int*)nullptr, (double*)nullptr);
  else
    hipLaunchKernelGGL((k_bsr_rows<G, 1>), dim3(blocks), dim3(256), 0, s, A.nr, B.br, B.bc, B.pat.ptr.p, B.pat.col.p,
                       B.val.p, B.mask.p, (int*)nullptr, cnt_or_ptr, A.col.p, A.val.p);
}

void bsr_to_csr(const DBsr& B, DCsr& A, hipStream_t s) {
  A.nr = B.pat.nr * B.br;
  A.nc = B.pat.nc * B.bc;
  A.ptr.alloc(A.nr + 1);
  DBuf<int> cnt(A.nr + 1);
  // lanes per row: the average blocks per block row, a power of two in [4, 64]
  const int64_t avg = B.pat.nr > 0 ? B.pat.nnz / B.pat.nr : 0;
  const int G = avg > 32 ? 64 : avg > 16 ? 32 : avg > 8 ? 16 : avg > 4 ? 8 : 4;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      A.nnz = exclusive_scan(cnt.p, A.ptr.p, A.nr, s);
      A.col.alloc(A.nnz > 0 ? A.nnz : 1);
      A.val.alloc(A.nnz > 0 ? A.nnz : 1);
      if (A.nnz == 0) break;
    }
    if (A.nr == 0) continue;
    const int* arg = pass == 0 ? cnt.p : A.ptr.p;
    switch (G) {
      case 4: bsr_rows<4>(B, A, pass, arg, s); break;
      case 8: bsr_rows<8>(B, A, pass, arg, s); break;
      case 16: bsr_rows<16>(B, A, pass, arg, s); break;
      case 32: bsr_rows<32>(B, A, pass, arg, s); break;
      default: bsr_rows<64>(B, A, pass, arg, s); break;
    }
  }
}

// ------------------------------------------------------------ numeric product
// One workgroup of NT threads per block row i of C, its output values and
// stored flags in LDS (block by block, br bc values each).  For every block
// (i, kb) of A in ascending kb the threads take the entries (block (kb, j) of
// B, r, c) of B's block row kb, one each: the thread finds block j in C's row
// (binary search over the row's block columns) and adds a_rk b_kc for k
// ascending inside the block where both entries are stored.  Within one A
// block no two threads share an output entry; the blocks follow one another
// with a barrier, so every output entry sums its terms in ascending k.  The
// block columns and B row ranges of the next NT blocks of A's row are read
// at once.  With STAGE, B's block row and A's block are staged in LDS one
// block ahead (double buffer), so the loads of the next A block overlap the
// work on the current one: they are issued into registers before the current
// block's work and stored to LDS after it (a B block row too long for the
// stage is read from global memory); this suits few long rows (R (A P)),
// while many short rows (A P) want the small footprint and the occupancy it
// brings.
constexpr int BSP_STG = 512;     // staged values of one B block row
constexpr int BSP_STGB = 64;     // staged blocks of one B block row

template <int NT>
__device__ __forceinline__ void bsp_stage(int tid, int nq, int kbc, int na, const int* __restrict__ Bc,
                                          const double* __restrict__ Bv, const unsigned long long* __restrict__ Bm,
                                          const double* __restrict__ av, int q0, double* sv, int* sc,
                                          unsigned long long* sm, double* sa) {
  const int nv = nq * kbc;
  for (int t = tid; t < nv; t += NT) sv[t] = Bv[(int64_t)q0 * kbc + t];
  if (tid < nq) {
    sc[tid] = Bc[q0 + tid];
    sm[tid] = Bm[q0 + tid];
  }
  if (tid < na) sa[tid] = av[tid];
}

template <int NT, int CAPV, bool STAGE>
__global__ __launch_bounds__(NT) void k_bspgemm_lds(const int* __restrict__ rows, int nrows, const int* __restrict__ nrows_dev,
                                                    int br, int bk, int bc,
                                                    const int* __restrict__ Ap, const int* __restrict__ Ac,
                                                    const double* __restrict__ Av, const unsigned long long* __restrict__ Am,
                                                    const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                    const double* __restrict__ Bv, const unsigned long long* __restrict__ Bm,
                                                    const int* __restrict__ Cp, const int* __restrict__ Cc,
                                                    double* __restrict__ Cv, unsigned long long* __restrict__ Cm,
                                                    int* __restrict__ ovf, int* __restrict__ novf) {
  __shared__ double acc[CAPV];
  __shared__ unsigned char st[CAPV];
  __shared__ int ccol[CAPV / 2];
  __shared__ int mq0[NT], mq1[NT];
  __shared__ unsigned long long mam[NT];
  __shared__ double sv[STAGE ? 2 : 1][STAGE ? BSP_STG : 1];
  __shared__ int sc[STAGE ? 2 : 1][STAGE ? BSP_STGB : 1];
  __shared__ unsigned long long sm[STAGE ? 2 : 1][STAGE ? BSP_STGB : 1];
  __shared__ double sa[STAGE ? 2 : 1][STAGE ? 64 : 1];
  const int tid = threadIdx.x;
  // rows: all of C's (no list) or a list whose length may be on the device;
  // workgroups stride over them
  const int nlist = nrows_dev ? *nrows_dev : nrows;
  for (int bi = blockIdx.x; bi < nlist; bi += gridDim.x) {
    __syncthreads();
    const int i = rows ? rows[bi] : bi;
    const int c0 = Cp[i], ncb = Cp[i + 1] - c0, bb = br * bc, nel = ncb * bb;
    if (nel > CAPV || ncb > CAPV / 2) {
      if (tid == 0) ovf[atomicAdd(novf, 1)] = i;
      continue;
    }
    const int kbc = bk * bc, na = br * bk;
    for (int t = tid; t < ncb; t += NT) ccol[t] = Cc[c0 + t];
    for (int t = tid; t < nel; t += NT) {
      acc[t] = 0.0;
      st[t] = 0;
    }
    const int a0 = Ap[i], a1 = Ap[i + 1];
    for (int p0 = a0; p0 < a1; p0 += NT) {
      __syncthreads();
      if (p0 + tid < a1) {
        const int kb = Ac[p0 + tid];
        mq0[tid] = Bp[kb];
        mq1[tid] = Bp[kb + 1];
        mam[tid] = Am[p0 + tid];
      }
      __syncthreads();
      const int np = min(NT, a1 - p0);
      if (STAGE) {
        const int nq = mq1[0] - mq0[0];
        if (nq <= BSP_STGB && nq * kbc <= BSP_STG)
          bsp_stage<NT>(tid, nq, kbc, na, Bc, Bv, Bm, Av + (int64_t)p0 * na, mq0[0], sv[0], sc[0], sm[0], sa[0]);
        __syncthreads();
      }
      for (int t = 0; t < np; ++t) {
        const int b = STAGE ? (t & 1) : 0;
        // the next block's stage is loaded into registers before this
        // block's work and written to the other buffer after it
        constexpr int PVN = STAGE ? (BSP_STG + NT - 1) / NT : 1;
        double pv[PVN], pa = 0.0;
        int pc = 0, nv1 = 0;
        unsigned long long pm = 0ull;
        bool pf = false;
        if (STAGE && t + 1 < np) {
          const int nq1 = mq1[t + 1] - mq0[t + 1];
          pf = nq1 <= BSP_STGB && nq1 * kbc <= BSP_STG;
          if (pf) {
            const int q1 = mq0[t + 1];
            nv1 = nq1 * kbc;
  #pragma unroll
            for (int u = 0; u < PVN; ++u)
              if (tid + u * NT < nv1) pv[u] = Bv[(int64_t)q1 * kbc + tid + u * NT];
            if (tid < nq1) {
              pc = Bc[q1 + tid];
              pm = Bm[q1 + tid];
            }
            if (tid < na) pa = Av[(int64_t)(p0 + t + 1) * na + tid];
          }
        }
        const int q0 = mq0[t], nq = mq1[t] - q0;
        const unsigned long long am = mam[t];
        const bool staged = STAGE && nq <= BSP_STGB && nq * kbc <= BSP_STG;
        const double* __restrict__ avp = Av + (int64_t)(p0 + t) * na;
        const int items = nq * bb;
        for (int it = tid; it < items; it += NT) {
          const int qo = it / bb, rc = it - qo * bb, r = rc / bc, c = rc - r * bc;
          int jb;
          unsigned long long bm;
          double x[8], y[8];
          // every operand is fetched at once (stored or not), then used where
          // both entries are stored
          if (staged) {
            jb = sc[b][qo];
            bm = sm[b][qo];
  #pragma unroll
            for (int k = 0; k < 8; ++k)
              if (k < bk) {
                x[k] = sa[b][r * bk + k];
                y[k] = sv[b][qo * kbc + k * bc + c];
              }
          } else {
            jb = Bc[q0 + qo];
            bm = Bm[q0 + qo];
  #pragma unroll
            for (int k = 0; k < 8; ++k)
              if (k < bk) {
                x[k] = avp[r * bk + k];
                y[k] = Bv[(int64_t)(q0 + qo) * kbc + k * bc + c];
              }
          }
          int lo = 0, hi = ncb;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ccol[mid] < jb) lo = mid + 1; else hi = mid;
          }
          const int e = lo * bb + rc;
          double a = acc[e];
          bool any = false;
  #pragma unroll
          for (int k = 0; k < 8; ++k)
            if (k < bk && ((am >> (r * bk + k)) & 1ull) && ((bm >> (k * bc + c)) & 1ull)) {
              a += x[k] * y[k];
              any = true;
            }
          if (any) {
            acc[e] = a;
            st[e] = 1;
          }
        }
        if (pf) {
  #pragma unroll
          for (int u = 0; u < PVN; ++u)
            if (tid + u * NT < nv1) sv[b ^ 1][tid + u * NT] = pv[u];
          if (tid < mq1[t + 1] - mq0[t + 1]) {
            sc[b ^ 1][tid] = pc;
            sm[b ^ 1][tid] = pm;
          }
          if (tid < na) sa[b ^ 1][tid] = pa;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    for (int t = tid; t < nel; t += NT) Cv[(int64_t)c0 * bb + t] = acc[t];
    for (int pb = tid; pb < ncb; pb += NT) {
      unsigned long long m = 0;
      for (int rc = 0; rc < bb; ++rc)
        if (st[pb * bb + rc]) m |= 1ull << rc;
      Cm[c0 + pb] = m;
    }
  }
}

// Block rows too long for LDS (more than 8,192 values): the listed rows, one wavefront each, every
// lane owning output entries (each block padded to BBP = the next power of
// two >= br bc, so a block never straddles a 64-lane window) of up to EPL
// windows at a time and summing their terms over the A blocks in ascending
// kb, k; the block's stored-entry mask is the ballot of its lanes.
constexpr int BSP_EPL = 4;

__global__ __launch_bounds__(64) void k_bspgemm_wide(const int* __restrict__ rows, int nrows, const int* __restrict__ nrows_dev,
                                                     int br, int bk, int bc, int bbp,
                                                     const int* __restrict__ Ap, const int* __restrict__ Ac,
                                                     const double* __restrict__ Av, const unsigned long long* __restrict__ Am,
                                                     const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                     const double* __restrict__ Bv, const unsigned long long* __restrict__ Bm,
                                                     const int* __restrict__ Cp, const int* __restrict__ Cc,
                                                     double* __restrict__ Cv, unsigned long long* __restrict__ Cm) {
  const int lane = threadIdx.x;
  const int nlist = nrows_dev ? *nrows_dev : nrows;
  for (int bi = blockIdx.x; bi < nlist; bi += gridDim.x) {
    const int i = rows[bi];
    const int c0 = Cp[i], ncb = Cp[i + 1] - c0;
    const int bb = br * bc, nel = ncb * bbp;
    const int a0 = Ap[i], a1 = Ap[i + 1];
    for (int base = 0; base < nel; base += 64 * BSP_EPL) {
      double acc[BSP_EPL];
      bool st[BSP_EPL];
      int jb[BSP_EPL], rr[BSP_EPL], cc[BSP_EPL];
  #pragma unroll
      for (int u = 0; u < BSP_EPL; ++u) {
        acc[u] = 0.0;
        st[u] = false;
        jb[u] = -1;
        rr[u] = cc[u] = 0;
        const int e = base + u * 64 + lane;
        if (e < nel) {
          const int pb = e / bbp, rc = e - pb * bbp;
          if (rc < bb) {
            jb[u] = Cc[c0 + pb];
            rr[u] = rc / bc;
            cc[u] = rc - rr[u] * bc;
          }
        }
      }
      for (int p = a0; p < a1; ++p) {
        const int kb = Ac[p];
        const unsigned long long am = Am[p];
        const double* av = Av + (int64_t)p * br * bk;
        const int q0 = Bp[kb], q1 = Bp[kb + 1];
  #pragma unroll
        for (int u = 0; u < BSP_EPL; ++u) {
          if (jb[u] < 0) continue;
          int lo = q0, hi = q1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (Bc[mid] < jb[u]) lo = mid + 1; else hi = mid;
          }
          if (lo >= q1 || Bc[lo] != jb[u]) continue;
          const unsigned long long bm = Bm[lo];
          const double* bv = Bv + (int64_t)lo * bk * bc;
          for (int k = 0; k < bk; ++k)
            if (((am >> (rr[u] * bk + k)) & 1ull) && ((bm >> (k * bc + cc[u])) & 1ull)) {
              acc[u] += av[rr[u] * bk + k] * bv[k * bc + cc[u]];
              st[u] = true;
            }
        }
      }
  #pragma unroll
      for (int u = 0; u < BSP_EPL; ++u) {
        const int e = base + u * 64 + lane;
        const unsigned long long bal = __ballot(st[u]);
        if (e < nel) {
          const int pb = e / bbp, rc = e - pb * bbp;
          if (rc < bb) Cv[(int64_t)(c0 + pb) * bb + rc] = acc[u];
          if (rc == 0) {
            // this block's bits sit at lanes [lane, lane + bbp) of the window
            const unsigned long long w = bal >> lane;
            Cm[c0 + pb] = bbp == 64 ? w : (w & ((1ull << bbp) - 1ull));
          }
        }
      }
    }
  }
}

// One pass over a row list (or all rows), with the list's length read on the
// device: rows too long for the pass are appended to ovf (count novf, which
// starts at zero).  Nothing is read back, so the passes queue one behind the
// other without the host waiting.
template <int NT, int CAPV, bool STAGE>
static void bsp_pass(const int* rows, int nrows, const int* nrows_dev, int grid, const DBsr& A, const DBsr& B, DBsr& C,
                     int* ovf, int* novf, hipStream_t s) {
  hipLaunchKernelGGL((k_bspgemm_lds<NT, CAPV, STAGE>), dim3(grid), dim3(NT), 0, s, rows, nrows, nrows_dev, A.br, A.bc, B.bc,
                     A.pat.ptr.p, A.pat.col.p, A.val.p, A.mask.p, B.pat.ptr.p, B.pat.col.p, B.val.p, B.mask.p, C.pat.ptr.p,
                     C.pat.col.p, C.val.p, C.mask.p, ovf, novf);
}

// block rows of C above which a product counts as many short rows
constexpr int BSP_MANY_ROWS = 8192;

// ------------------------------------------------------------ block pattern
// Block pattern of A B when B has at most PAT_BITS block columns: one
// wavefront per block row marks the block columns it reaches in an LDS
// bitmap (lanes take A's entries, each walking its B row), then reads the
// set bits in ascending order (pass 0 counts them, pass 1 writes them at the
// row's offset).  The same pattern as the scalar product machinery, with no
// hashing.
constexpr int PAT_BITS = 16384;
template <int PASS>
__global__ __launch_bounds__(64) void k_pattern_bits(int nc, const int* __restrict__ Ap, const int* __restrict__ Ac,
                                                     const int* __restrict__ Bp, const int* __restrict__ Bc,
                                                     int* __restrict__ cnt_or_ptr, int* __restrict__ Cc) {
  __shared__ unsigned int bits[PAT_BITS / 32];
  const int i = blockIdx.x, lane = threadIdx.x;
  const int nw = (nc + 31) >> 5;
  for (int w = lane; w < nw; w += 64) bits[w] = 0u;
  __syncthreads();
  for (int p = Ap[i] + lane; p < Ap[i + 1]; p += 64) {
    const int k = Ac[p];
    for (int q = Bp[k]; q < Bp[k + 1]; ++q) {
      const int j = Bc[q];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  }
  __syncthreads();
  int n = 0;
  const int o = PASS ? cnt_or_ptr[i] : 0;
  for (int w0 = 0; w0 < nw; w0 += 64) {
    const int w = w0 + lane;
    const unsigned int x = w < nw ? bits[w] : 0u;
    const int c = __popc(x);
    int incl = c;
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    if (PASS) {
      int pos = o + n + incl - c;
      for (unsigned int y = x; y; y &= y - 1u) Cc[pos++] = (w << 5) + __ffs((int)y) - 1;
    }
    n += __shfl(incl, 63, 64);
  }
  if (!PASS && lane == 0) cnt_or_ptr[i] = n;
}

static void pattern_bits(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s) {
  C.nr = A.nr;
  C.nc = B.nc;
  C.ptr.alloc(C.nr + 1);
  DBuf<int> cnt(C.nr + 1);
  if (C.nr > 0)
    hipLaunchKernelGGL(k_pattern_bits<0>, dim3(C.nr), dim3(64), 0, s, C.nc, A.ptr.p, A.col.p, B.ptr.p, B.col.p, cnt.p,
                       (int*)nullptr);
  C.nnz = exclusive_scan(cnt.p, C.ptr.p, C.nr, s);
  const int64_t nb = C.nnz > 0 ? C.nnz : 1;
  C.col.alloc(nb);
  C.val.alloc(nb);
  if (C.nnz > 0) {
    hipLaunchKernelGGL(k_pattern_bits<1>, dim3(C.nr), dim3(64), 0, s, C.nc, A.ptr.p, A.col.p, B.ptr.p, B.col.p, C.ptr.p,
                       C.col.p);
    iota(C.val.p, C.nnz, s);
  }
}

void bspgemm(const DBsr& A, const DBsr& B, DBsr& C, hipStream_t s) {
  NF_CHECK(A.pat.nc == B.pat.nr && A.bc == B.br, NFIELD_EINVAL, "block product: inner dimensions differ");
  C.br = A.br;
  C.bc = B.bc;
  // block pattern of the product (its values, unused, are block indices
  // from the bitmap path and counts from the scalar product)
  if (B.pat.nc <= PAT_BITS) pattern_bits(A.pat, B.pat, C.pat, s);
  else spgemm(A.pat, B.pat, C.pat, s);
  const int64_t nb = C.pat.nnz > 0 ? C.pat.nnz : 1;
  const int bb = C.br * C.bc;
  C.val.alloc(nb * bb);
  C.mask.alloc(nb);
  const int nbr = C.pat.nr;
  if (nbr <= 0 || C.pat.nnz <= 0) return;
  // every pass takes the rows the previous one could not hold: 512 values in
  // 6.5 KB of LDS (many workgroups per CU, for many short rows), 2,048 values
  // with a staged B row, 8,192 values (one workgroup per CU), then register-
  // owned entries; later passes stride over their lists with bounded grids
  DBuf<int> l1(nbr), l2(nbr), l3(nbr), cnt(3);
  fill<int>(cnt.p, 0, 3, s);
  const int* list2;
  const int* n2;
  if (nbr >= BSP_MANY_ROWS) {
    bsp_pass<64, 512, false>(nullptr, nbr, nullptr, nbr, A, B, C, l1.p, cnt.p, s);
    bsp_pass<256, 2048, true>(l1.p, nbr, cnt.p, std::min(nbr, 4096), A, B, C, l2.p, cnt.p + 1, s);
    list2 = l2.p;
    n2 = cnt.p + 1;
  } else {
    bsp_pass<256, 2048, true>(nullptr, nbr, nullptr, nbr, A, B, C, l2.p, cnt.p + 1, s);
    list2 = l2.p;
    n2 = cnt.p + 1;
  }
  bsp_pass<256, 8192, true>(list2, nbr, n2, std::min(nbr, 512), A, B, C, l3.p, cnt.p + 2, s);
  int bbp = 1;
  while (bbp < bb) bbp <<= 1;
  hipLaunchKernelGGL(k_bspgemm_wide, dim3(std::min(nbr, 1024)), dim3(64), 0, s, l3.p, nbr, cnt.p + 2, A.br, A.bc, B.bc, bbp,
                     A.pat.ptr.p, A.pat.col.p, A.val.p, A.mask.p, B.pat.ptr.p, B.pat.col.p, B.val.p, B.mask.p, C.pat.ptr.p,
                     C.pat.col.p, C.val.p, C.mask.p);
}

// R = P^T block by block: the block pattern transposed (pattern values carry
// the source block's index), each block's values and mask transposed
__global__ void k_bsr_tblocks(int64_t nb, int pr, int pc, const double* __restrict__ src, const double* __restrict__ Pv,
                              const unsigned long long* __restrict__ Pm, double* __restrict__ Rv,
                              unsigned long long* __restrict__ Rm) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nb) return;
  const int64_t q = (int64_t)src[t];
  const int bb = pr * pc;
  const unsigned long long m = Pm[q];
  unsigned long long rm = 0;
  for (int r = 0; r < pr; ++r)
    for (int c = 0; c < pc; ++c) {
      Rv[t * bb + c * pr + r] = Pv[q * bb + r * pc + c];
      if ((m >> (r * pc + c)) & 1ull) rm |= 1ull << (c * pr + r);
    }
  Rm[t] = rm;
}

void bsr_transpose(const DBsr& P, DBsr& R, hipStream_t s) {
  R.br = P.bc;
  R.bc = P.br;
  transpose(P.pat, R.pat, s);
  const int64_t nb = R.pat.nnz > 0 ? R.pat.nnz : 1;
  R.val.alloc(nb * R.br * R.bc);
  R.mask.alloc(nb);
  if (R.pat.nnz > 0)
    hipLaunchKernelGGL(k_bsr_tblocks, dim3(cdiv(R.pat.nnz, 256)), dim3(256), 0, s, R.pat.nnz, P.br, P.bc, R.pat.val.p,
                       P.val.p, P.mask.p, R.val.p, R.mask.p);
  // the pattern values of a converted matrix are block indices
  if (R.pat.nnz > 0) iota(R.pat.val.p, R.pat.nnz, s);
}

void spgemm_blocked(const DCsr& A, int br, int bk, const DCsr& B, int bc, DCsr& C, hipStream_t s) {
  DBsr Ab, Bb, Cb;
  csr_to_bsr(A, br, bk, Ab, s);
  csr_to_bsr(B, bk, bc, Bb, s);
  bspgemm(Ab, Bb, Cb, s);
  bsr_to_csr(Cb, C, s);
}

}  // namespace nf

// Hessian factor H = R^adj o R (Section 5.4, Algorithms 5.3 and 5.4) on the
// supernodal factor, and the Gram matrix of the vectors it produces
// (Section 1.3: the Schur complement A_i . H(A_j) = R(A_i) . R(A_j) of an
// interior-point step).
//
// Scalar form: with K_jj = dD_jj and K_{I_j j} = D_jj dL_{I_j j} (step 1 of
// the Hessian), W_jj = K_jj / D_jj and W_{I_j j} = R_j^T K_{I_j j} / sqrt(D_jj),
// where S_{I_j I_j} = R_j R_j^T with R_j upper triangular.  Block form per
// supernode (N columns, A ancestors), derived from the scalar one with the
// block step 1 (K_NN = dD_NN, K_AN = dL_AN D_NN):
//   W_NN = lower triangle of C^-1 K_NN C^-T,   W_AN = G K_AN C^-T,
// where D_NN = C C^T (the NN part of the Cholesky panel) and G is the lower
// triangular matrix with G^T G = S_AA.  For N = 1 this is the scalar rule:
// C = sqrt(D_jj) and G = R_j^T, the trailing principal submatrices of S_JJ
// being those of the column's I_j.  The adjoint (Algorithm 5.4) inverts the
// conversion and hands the block step 2 of the Hessian a K that reproduces
// the paper's M: with sym(W_NN) the symmetric matrix whose lower triangle
// is W_NN,
//   Kt_NN = C sym(W_NN) C^T,   Kt_AN = G^-1 W_AN C^T,
// so that D^-1 Kt_NN D^-1 = C^-T sym(W_NN) C^-1 and S_AA Kt_AN D^-1 =
// G^T W_AN C^-1 (for N = 1: W_jj / D_jj and R_j W_{I_j j} / sqrt(D_jj)); the
// Hessian's root-to-leaf sweep then finishes R^adj(W).
//
// G is cached per supernode together with G^-1 (packed lower, the layout
// and offsets of the S_AA blocks): P S_AA P = F F^T for the index reversal
// P of A_s, and G = P F^T P, so the left-looking Cholesky runs on the
// reversed view of the packed block, in place, and its inverse gives G^-1.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "front.h"
#include "kernels.h"
#include "wg_dense.h"

namespace mfb {

namespace {

// Entry (p, q), p >= q, of the factor F of the reversed block, kept where
// G(A-1-q, A-1-p) lives in packed lower storage of G.
struct Reversed {
  double* u;
  int a;
  __device__ __forceinline__ double& operator()(int p, int q) const { return u[pk(a - 1 - q, a - 1 - p, a)]; }
};

// C(i, j) <- epi(i, j, sum_{k <= i} L(i, k) B(k, j)) for a lower-triangular
// M x M operand L (read for k <= i only) and an M x N operand B: the k loop
// of a row tile stops at the tile's last row.
template <bool BK, class FL, class FB, class EPI>
__device__ __forceinline__ void wg_trmm_lower(int M, int N, const FL& fl, const FB& fb, const EPI& epi,
                                              double* sm) {
  for (int i0 = 0; i0 < M; i0 += TM)
    for (int j0 = 0; j0 < N; j0 += TM) {
      MfmaTile T(threadIdx.x);
      tile_mma<false, BK>(
          T, i0, j0, M, N, 0, min(M, i0 + TM), [&](int i, int k) { return k <= i ? fl(i, k) : 0.0; }, fb, sm);
      tile_store(T, i0, j0, M, N, epi, false);
    }
}

}  // namespace

// G and G^-1 of every supernode of the list with A > 0 (one workgroup per
// supernode): copy S_AA, factor its reversed view in place (64-column
// left-looking Cholesky, diagonal blocks left inverted), copy, invert the
// copy, then put the diagonal blocks of the factor back.
__global__ void __launch_bounds__(NT) k_gamma(DevPlan P, const int32_t* list, const double* Vs, double* Gam,
                                              double* Gami, DevStatus* st) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double d64[NB2 * LD2];
  __shared__ int fail;
  const int s = list[blockIdx.x];
  const int A = P.nrow[s] - P.ncol[s];
  if (A == 0) return;  // (the whole workgroup)
  const int64_t off = P.arena[s], m = (int64_t)A * (A + 1) / 2;
  double* g = Gam + off;
  double* gi = Gami + off;
  for (int64_t e = threadIdx.x; e < m; e += NT) g[e] = Vs[off + e];
  if (threadIdx.x == 0) fail = -1;
  __syncthreads();
  // the reversed view of the symmetric block is P S_AA P itself: entry
  // (p, q) of it is S_AA(A-1-p, A-1-q), stored at the packed position of
  // (A-1-q, A-1-p)
  wg_potrf64(Reversed{g, A}, A, sm, d64, &fail);
  if (threadIdx.x == 0 && fail >= 0) report(st, MFB_ENOTPD, P.vlabel[P.colbase[s]]);
  for (int64_t e = threadIdx.x; e < m; e += NT) gi[e] = g[e];
  __syncthreads();
  wg_trtri64_invdiag(Reversed{gi, A}, A, sm, d64);
  const Reversed F{g, A};
  for (int j0 = 0; j0 < A; j0 += NB2) {
    const int nb = min(NB2, A - j0);
    for (int e = threadIdx.x; e < NB2 * LD2; e += NT) d64[e] = 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) d64[i + j * LD2] = F(j0 + i, j0 + j);
    }
    __syncthreads();
    wg_trtri_inplace(DenseAt{d64, LD2}, nb, sm);
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) F(j0 + i, j0 + j) = d64[i + j * LD2];
    }
    __syncthreads();
  }
}

// W = R(Y) from the block step-1 output K (CCS, right-hand side
// blockIdx.y), one workgroup per (supernode, right-hand side); supernodes
// are independent.  Scratch (doubles): 2 N^2 + A N.  A supernode that
// step 1 pruned (act 0: no nonzero of Y in its subtree, so K = 0) gets
// W = 0 directly (Section 5.5).
__global__ void __launch_bounds__(NT) k_hfactor(DevPlan P, const int32_t* list, const double* R,
                                                const double* Gam, const double* Kt, double* Wt, double* wsb,
                                                int64_t slot, const int32_t* act) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const int N = v.N, A = v.A;
    const double* K = Kt + r * P.nnz;
    double* w = Wt + r * P.nnz;
    if (!act[r * P.ns + v.s]) {
      for (int64_t e = threadIdx.x; e < (int64_t)v.J * N; e += NT) {
        const int i = int(e % v.J), j = int(e / v.J);
        if (i >= j) w[v.at(i, j)] = 0.0;
      }
      return;
    }
    double* Ci = slot_ptr(wsb, slot);
    double* T1 = Ci + (int64_t)N * N;
    double* E = T1 + (int64_t)N * N;
    wg_trtri([&](int i, int k) { return R[v.at(i, k)]; }, N, Ci, N, sm);
    // T1 = C^-1 K_NN (C^-1 lower: k <= i), then W_NN = lower(T1 C^-T)
    wg_gemm<false, true>(
        N, N, N, [&](int i, int k) { return Ci[i + (int64_t)k * N]; }, [&](int k, int j) { return K[v.nn(k, j)]; },
        [&](int i, int j, double acc) { T1[i + (int64_t)j * N] = acc; }, false, sm);
    __syncthreads();
    wg_gemm(
        N, N, N, [&](int i, int k) { return T1[i + (int64_t)k * N]; },
        [&](int k, int j) { return Ci[j + (int64_t)k * N]; },
        [&](int i, int j, double acc) { w[v.at(i, j)] = acc; }, true, sm);
    if (A == 0) return;
    // E = K_AN C^-T, then W_AN = G E
    wg_gemm(
        A, N, N, [&](int i, int k) { return K[v.an(i, k)]; }, [&](int k, int j) { return Ci[j + (int64_t)k * N]; },
        [&](int i, int j, double acc) { E[i + (int64_t)j * A] = acc; }, false, sm);
    __syncthreads();
    const double* g = Gam + P.arena[v.s];
    wg_trmm_lower<true>(
        A, N, [&](int i, int k) { return g[pk(i, k, A)]; }, [&](int k, int j) { return E[k + (int64_t)j * A]; },
        [&](int i, int j, double acc) { w[v.an(i, j)] = acc; }, sm);
  });
}

// Kt = the block step-2 input that makes the Hessian's root-to-leaf sweep
// produce R^adj(W) (W: CCS, right-hand side blockIdx.y); one workgroup per
// (supernode, right-hand side).  Scratch (doubles): N^2 + A N.
__global__ void __launch_bounds__(NT) k_hfactor_adj(DevPlan P, const int32_t* list, const double* R,
                                                    const double* Gami, const double* Wt, double* Kt, double* wsb,
                                                    int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const int N = v.N, A = v.A;
    const double* w = Wt + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* T1 = slot_ptr(wsb, slot);
    double* E = T1 + (int64_t)N * N;
    auto Ct = [&](int k, int j) { return k <= j ? R[v.at(j, k)] : 0.0; };  // C^T(k, j)
    // T1 = sym(W_NN) C^T, Kt_NN = lower(C T1)
    wg_gemm(
        N, N, N, [&](int i, int k) { return w[v.nn(i, k)]; }, Ct,
        [&](int i, int j, double acc) { T1[i + (int64_t)j * N] = acc; }, false, sm);
    __syncthreads();
    wg_gemm<false, true>(
        N, N, N, [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; },
        [&](int k, int j) { return T1[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { K[v.at(i, j)] = acc; }, true, sm);
    if (A == 0) return;
    // E = W_AN C^T, then Kt_AN = G^-1 E
    wg_gemm(
        A, N, N, [&](int i, int k) { return w[v.an(i, k)]; }, Ct,
        [&](int i, int j, double acc) { E[i + (int64_t)j * A] = acc; }, false, sm);
    __syncthreads();
    const double* gi = Gami + P.arena[v.s];
    wg_trmm_lower<true>(
        A, N, [&](int i, int k) { return gi[pk(i, k, A)]; }, [&](int k, int j) { return E[k + (int64_t)j * A]; },
        [&](int i, int j, double acc) { K[v.an(i, j)] = acc; }, sm);
  });
}

// Gram matrix of m vectors of S^n_V (m x nnz, row-major) under the trace
// inner product, sum_e wt_e W_i[e] W_j[e] with wt_e = 1 on the diagonal and
// 2 off it, written as 2 (sum over all entries) - (sum over the diagonal
// entries).  Partial products: one workgroup per (lower 64 x 64 tile pair,
// chunk), chunks of `chunk` entries over [0, nnz) followed by chunks of the
// n diagonal entries (colptr[j], the first entry of column j); partial c of
// tile pair q goes to part[(c * pairs + q) * 4096].
__global__ void __launch_bounds__(NT) k_gram_part(const double* Wt, int64_t nnz, int64_t n, int m,
                                                  const int64_t* colptr, int64_t chunk, int64_t nfull,
                                                  double* part) {
  __shared__ double sm[SMEM_DOUBLES];
  const int tiles = (m + TM - 1) / TM, pairs = tiles * (tiles + 1) / 2;
  const int q = blockIdx.x;
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
  const int tj = q - ti * (ti + 1) / 2;
  const int64_t c = blockIdx.y;
  const bool diag = c >= nfull;
  const int64_t e0 = (diag ? c - nfull : c) * chunk;
  const int64_t len = diag ? n : nnz;
  const int kl = int(len - e0 < chunk ? len - e0 : chunk);
  MfmaTile T(threadIdx.x);
  if (diag)
    tile_mma<false, false>(
        T, ti * TM, tj * TM, m, m, 0, kl, [&](int i, int k) { return Wt[(int64_t)i * nnz + colptr[e0 + k]]; },
        [&](int k, int j) { return Wt[(int64_t)j * nnz + colptr[e0 + k]]; }, sm);
  else
    tile_mma<true, true>(
        T, ti * TM, tj * TM, m, m, 0, kl, [&](int i, int k) { return Wt[(int64_t)i * nnz + e0 + k]; },
        [&](int k, int j) { return Wt[(int64_t)j * nnz + e0 + k]; }, sm);
  double* out = part + ((int64_t)c * pairs + q) * (TM * TM);
  const double f = diag ? -1.0 : 2.0;
  tile_store(
      T, 0, 0, TM, TM, [&](int i, int j, double acc) { out[i + j * TM] = f * acc; }, false);
}

// G(i, j) = G(j, i) = sum over the partials in chunk order.
__global__ void __launch_bounds__(NT) k_gram_sum(int m, int64_t nparts, const double* part, double* Gout) {
  const int tiles = (m + TM - 1) / TM, pairs = tiles * (tiles + 1) / 2;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = int(e % m), j = int(e / m);
  if (i < j) return;
  const int ti = i / TM, tj = j / TM;
  const int q = ti * (ti + 1) / 2 + tj;
  const int li = i - ti * TM, lj = j - tj * TM;
  double acc = 0.0;
  for (int64_t c = 0; c < nparts; ++c) acc += part[((int64_t)c * pairs + q) * (TM * TM) + li + lj * TM];
  Gout[i + (int64_t)j * m] = acc;
  Gout[j + (int64_t)i * m] = acc;
}

void launch_gamma(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* Vs, double* Gam,
                  double* Gami, DevStatus* st) {
  k_gamma<<<dim3(grid.x), NT, 0, s>>>(P, list, Vs, Gam, Gami, st);
}

void launch_hfactor(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                    const double* Gam, const double* Kt, double* Wt, double* wsb, int64_t slot, const int32_t* act) {
  k_hfactor<<<grid, NT, 0, s>>>(P, list, R, Gam, Kt, Wt, wsb, slot, act);
}

void launch_hfactor_adj(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                        const double* Gami, const double* Wt, double* Kt, double* wsb, int64_t slot) {
  k_hfactor_adj<<<grid, NT, 0, s>>>(P, list, R, Gami, Wt, Kt, wsb, slot);
}

GramShape gram_shape(int64_t nnz, int64_t n, int m) {
  GramShape g;
  const int tiles = (m + TM - 1) / TM;
  g.pairs = tiles * (tiles + 1) / 2;
  // about 2048 workgroups in all (at most 256 chunks over the entries),
  // each chunk a whole number of k-chunks of at least 1024 entries
  int64_t want = (2048 + g.pairs - 1) / g.pairs;
  want = want > 256 ? 256 : want;
  int64_t c = (nnz + want - 1) / want;
  c = (c + KC - 1) / KC * KC;
  g.chunk = c < 1024 ? 1024 : c;
  g.nfull = (nnz + g.chunk - 1) / g.chunk;
  g.nparts = g.nfull + (n + g.chunk - 1) / g.chunk;
  g.part_doubles = g.nparts * g.pairs * (TM * TM);
  return g;
}

void launch_gram(hipStream_t s, const GramShape& g, const double* Wt, int64_t nnz, int64_t n, int m,
                 const int64_t* colptr, double* part, double* Gout) {
  k_gram_part<<<dim3(unsigned(g.pairs), unsigned(g.nparts)), NT, 0, s>>>(Wt, nnz, n, m, colptr, g.chunk, g.nfull,
                                                                         part);
  const int64_t total = (int64_t)m * m;
  k_gram_sum<<<dim3(unsigned((total + NT - 1) / NT)), NT, 0, s>>>(m, g.nparts, part, Gout);
}

}  // namespace mfb

// Supernodal multifrontal sweeps on gfx950: one workgroup per
// (supernode, right-hand side) of a level of the clique tree.
//
// Factor state per supernode s (N = |N_s|, A = |A_s|), all in the CCS
// order of the user's pattern (column c of s holds rows J_s[c:]):
//   R  : the Cholesky panel [C; B] with C = chol(D_NN) and B = L_AN C, i.e.
//        the scalar Cholesky factor of X (independent of the partition);
//   LB : [D_NN^-1 (lower); L_AN], the block L D L^T factors of Algorithm 7.1
//        with the inverse of the pivot block;
//   S  : the projected inverse P(X^-1), and per supernode the packed block
//        V_s = S_{A_s A_s} (update matrices of Algorithm 7.2);
//   Vi : (S_{A_s A_s})^-1, packed, for the inverse Hessian and completion.
// Update matrices (U, U', V, V') are packed lower-triangular A x A blocks in
// an arena; children are assembled in a fixed order without atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdint>

#include "kernels.h"
#include "front.h"
#include "reg_front.h"
#include "wg_dense.h"

namespace mfb {

static_assert(NT == NT_LAUNCH, "launch width");
static_assert(SMEM_DOUBLES >= (NT_DOWN / NT) * 2 * KC * LDS_TM, "team GEMM staging fits the workgroup scratch");


// Lower-triangle accessor of a packed symmetric A x A block.
struct PackedLower {
  double* u;
  int A;
  __device__ __forceinline__ double& operator()(int i, int j) const { return u[pk(i, j, A)]; }
};

// VI <- C^-1 (lower, packed) for a packed symmetric positive definite
// A x A block V = C C^T, in place in VI (no scratch): copy V, then the
// Cholesky factor and its triangular inverse on the packed triangle.
// d64: LDS of NB2 * LD2 doubles.
__device__ __forceinline__ void packed_tri_inverse(const double* V, double* VI, int A, double* sm, double* d64,
                                                   int* fail) {
  const int64_t m = (int64_t)A * (A + 1) / 2;
  for (int64_t e = threadIdx.x; e < m; e += NT) VI[e] = V[e];
  __syncthreads();
  wg_potrf64(PackedLower{VI, A}, A, sm, d64, fail);
  wg_trtri64_invdiag(PackedLower{VI, A}, A, sm, d64);
}

// ---------------------------------------------------------------------------
// Algorithm 7.1: supernodal Cholesky factorization (leaf-to-root level).
// F = [X_NN X_AN^T; X_AN 0] + sum_children E U_c E^T; C = chol(F11);
// B = F21 C^-T; U_s = F22 - B B^T; L_AN = B C^-1; D^-1 = C^-T C^-1.
// Scratch per workgroup: J*N + N*N.
// PANEL: the front's A x A update block is left to the tile-parallel
// update kernel (k_wide_update); only the panel columns are assembled.
template <bool PANEL>
__global__ void __launch_bounds__(NT) k_factor(DevPlan P, const int32_t* list, const double* x,
                                               double* R, double* LB, double* U, double* part,
                                               DevStatus* st, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  __shared__ int fail;
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    double* F = slot_ptr(wsb, slot);
    double* Ci = F + (int64_t)v.J * v.N;
    double* Us = U + P.arena[v.s];
    if (threadIdx.x == 0) fail = -1;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * v.N; e += NT) {
      const int r = int(e % v.J), c = int(e / v.J);
      F[e] = r >= c ? x[v.at(r, c)] : 0.0;
    }
    if (!PANEL) zero_packed(Us, v.A);
    __syncthreads();
    if (PANEL)
      assemble_children_panel(P, v, U, F);
    else
      assemble_children(P, v, U, F, Us, sm);
    wg_potrf_panel(F, v.J, v.J, v.N, sm, &fail);
    // Cholesky panel -> R, log det contribution 2 sum log C_kk
    double lg = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * v.N; e += NT) {
      const int r = int(e % v.J), c = int(e / v.J);
      if (r >= c) R[v.at(r, c)] = F[e];
    }
    for (int c = threadIdx.x; c < v.N; c += NT) lg += 2.0 * log(F[c + (int64_t)c * v.J]);
    lg = wg_sum(lg, sm);
    if (threadIdx.x == 0) {
      part[v.s] = lg;
      if (fail >= 0) report(st, MFB_ENOTPD, v.vl[fail]);
    }
    // U_s = F22 - B B^T
    if (!PANEL)
      wg_gemm(
          v.A, v.A, v.N, [&](int i, int k) { return F[(v.N + i) + (int64_t)k * v.J]; },
          [&](int k, int j) { return F[(v.N + j) + (int64_t)k * v.J]; },
          [&](int i, int j, double acc) { Us[pk(i, j, v.A)] -= acc; }, true, sm);
    // C^-1
    wg_trtri([&](int i, int j) { return F[i + (int64_t)j * v.J]; }, v.N, Ci, v.N, sm);
    // L_AN = B C^-1
    wg_gemm<false, true>(
        v.A, v.N, v.N, [&](int i, int k) { return F[(v.N + i) + (int64_t)k * v.J]; },
        [&](int k, int j) { return Ci[k + (int64_t)j * v.N]; },
        [&](int i, int j, double acc) { LB[v.an(i, j)] = acc; }, false, sm);
    // D^-1 = C^-T C^-1 (lower)
    wg_gemm<true, true>(
        v.N, v.N, v.N, [&](int i, int k) { return Ci[k + (int64_t)i * v.N]; },
        [&](int k, int j) { return Ci[k + (int64_t)j * v.N]; },
        [&](int i, int j, double acc) { LB[v.at(i, j)] = acc; }, true, sm);
  });
}
template __global__ void k_factor<false>(DevPlan, const int32_t*, const double*, double*, double*, double*,
                                         double*, DevStatus*, double*, int64_t);
template __global__ void k_factor<true>(DevPlan, const int32_t*, const double*, double*, double*, double*,
                                        double*, DevStatus*, double*, int64_t);

// ---------------------------------------------------------------------------
// Algorithm 7.2: projected inverse (root-to-leaf level).
// V_s from the parent; S_AN = -V_s L_AN; S_NN = D^-1 - S_AN^T L_AN.
__global__ void __launch_bounds__(NT_DOWN) k_projinv(DevPlan P, const int32_t* list, const double* LB,
                                                double* S, double* Vs) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols<NT_DOWN>(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    extract_from_parent<NT_DOWN>(P, v, S, Vs, sm);
    __syncthreads();
    const double* V = Vs + P.arena[v.s];
    wg_gemm_split<NT_DOWN, false, true>(
        v.A, v.N, v.A, [&](int i, int k) { return sym_packed(V, i, k, v.A); },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { S[v.an(i, j)] = -acc; }, false, sm);
    __syncthreads();
    wg_gemm_split<NT_DOWN, true, true>(
        v.N, v.N, v.A, [&](int i, int k) { return S[v.an(k, i)]; },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { S[v.at(i, j)] = LB[v.at(i, j)] - acc; }, true, sm);
  });
}

// ---------------------------------------------------------------------------
// Hessian step 1 (leaf-to-root), block form of Algorithm 5.1 step 1:
// F' = [Y_NN Y_AN^T; Y_AN 0] + sum E U'_c E^T;
// K_NN = F'11, K_AN = F'21 - L F'11, U'_s = F'22 - L F'21^T - K_AN L^T.
// Per RHS r = blockIdx.y.  Scratch: J*N.
// PANEL: panel columns only; U'_s is left to k_wide_update, which reads
// F'21 from this workgroup's scratch slot.
template <bool PANEL>
__global__ void __launch_bounds__(NT) k_hess_up(DevPlan P, const int32_t* list, const double* LB,
                                                const double* Y, double* Kt, double* Ua,
                                                int64_t upd, double* wsb, int64_t slot, int32_t* act) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const double* y = Y + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* ua = Ua + r * upd;
    double* Us = ua + P.arena[v.s];
    double* F = slot_ptr(wsb, slot);
    int32_t* ac = act + r * P.ns;
    bool own = false;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * v.N; e += NT) {
      const int rr = int(e % v.J), c = int(e / v.J);
      const double yv = rr >= c ? y[v.at(rr, c)] : 0.0;
      own = own || yv != 0.0;
      F[e] = yv;
    }
    if (!step1_active(P, v.s, ac, own)) {
      // no nonzero of Y below this front: K = 0 here, and the update block
      // (zero) is neither formed nor read (the parent skips it)
      for (int64_t e = threadIdx.x; e < (int64_t)v.J * v.N; e += NT) {
        const int rr = int(e % v.J), c = int(e / v.J);
        if (rr >= c) K[v.at(rr, c)] = 0.0;
      }
      if (threadIdx.x == 0) ac[v.s] = 0;
      return;
    }
    if (!PANEL) zero_packed(Us, v.A);
    __syncthreads();
    if (PANEL)
      assemble_children_panel(P, v, ua, F, ac);
    else
      assemble_children(P, v, ua, F, Us, sm, ac);
    for (int64_t e = threadIdx.x; e < (int64_t)v.N * v.N; e += NT) {
      const int i = int(e % v.N), c = int(e / v.N);
      if (i >= c) K[v.at(i, c)] = F[i + (int64_t)c * v.J];
    }
    auto F11 = [&](int i, int j) { return i >= j ? F[i + (int64_t)j * v.J] : F[j + (int64_t)i * v.J]; };
    wg_gemm<false, true>(
        v.A, v.N, v.N, [&](int i, int k) { return LB[v.an(i, k)]; }, [&](int k, int j) { return F11(k, j); },
        [&](int i, int j, double acc) { K[v.an(i, j)] = F[(v.N + i) + (int64_t)j * v.J] - acc; }, false,
        sm);
    if (PANEL) return;
    __syncthreads();
    const int N = v.N;
    wg_gemm(
        v.A, v.A, 2 * N,
        [&](int i, int k) { return k < N ? LB[v.an(i, k)] : K[v.an(i, k - N)]; },
        [&](int k, int j) { return k < N ? F[(N + j) + (int64_t)k * v.J] : LB[v.an(j, k - N)]; },
        [&](int i, int j, double acc) { Us[pk(i, j, v.A)] -= acc; }, true, sm);
  });
}
template __global__ void k_hess_up<false>(DevPlan, const int32_t*, const double*, const double*, double*,
                                          double*, int64_t, double*, int64_t, int32_t*);
template __global__ void k_hess_up<true>(DevPlan, const int32_t*, const double*, const double*, double*,
                                         double*, int64_t, double*, int64_t, int32_t*);

// Hessian steps 2 and 3 (root-to-leaf), block form of Algorithm 5.1 with
// the V_j recursion of its modified step 2 (here V_s is cached):
// M_NN = D^-1 K_NN D^-1, M_AN = V_s K_AN D^-1, T_AN = M_AN - V' L,
// T_NN = M_NN - L^T T_AN - M_AN^T L, V'_c = E^T [T_NN T_AN^T; T_AN V'] E.
// Scratch: 2AN + 2N^2.
__global__ void __launch_bounds__(NT_DOWN) k_hess_down(DevPlan P, const int32_t* list, const double* LB,
                                                  const double* Vs, const double* Kt, double* T,
                                                  double* Va, int64_t upd, double* wsb,
                                                  int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols<NT_DOWN>(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const double* K = Kt + r * P.nnz;
    double* t = T + r * P.nnz;
    double* va = Va + r * upd;
    const int N = v.N, A = v.A;
    double* Z = slot_ptr(wsb, slot);
    double* W = Z + (int64_t)A * N;
    double* MA = W + (int64_t)N * N;
    double* MN = MA + (int64_t)A * N;
    extract_from_parent<NT_DOWN>(P, v, t, va, sm);
    auto Dinv = [&](int i, int j) { return LB[v.nn(i, j)]; };
    wg_gemm_split<NT_DOWN, false, true>(
        A, N, N, [&](int i, int k) { return K[v.an(i, k)]; }, Dinv,
        [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false, sm);
    wg_gemm_split<NT_DOWN, false, true>(
        N, N, N, [&](int i, int k) { return K[v.nn(i, k)]; }, Dinv,
        [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false, sm);
    __syncthreads();
    const double* V = Vs + P.arena[v.s];
    wg_gemm_split<NT_DOWN, false, true>(
        A, N, A, [&](int i, int k) { return sym_packed(V, i, k, A); },
        [&](int k, int j) { return Z[k + (int64_t)j * A]; },
        [&](int i, int j, double acc) { MA[i + (int64_t)j * A] = acc; }, false, sm);
    wg_gemm_split<NT_DOWN, false, true>(
        N, N, N, Dinv, [&](int k, int j) { return W[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { MN[i + (int64_t)j * N] = acc; }, true, sm);
    __syncthreads();
    const double* Vp = va + P.arena[v.s];
    wg_gemm_split<NT_DOWN, false, true>(
        A, N, A, [&](int i, int k) { return sym_packed(Vp, i, k, A); },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { t[v.an(i, j)] = MA[i + (int64_t)j * A] - acc; }, false, sm);
    __syncthreads();
    wg_gemm_split<NT_DOWN, true, true>(
        N, N, 2 * A,
        [&](int i, int k) { return k < A ? LB[v.an(k, i)] : MA[(k - A) + (int64_t)i * A]; },
        [&](int k, int j) { return k < A ? t[v.an(k, j)] : LB[v.an(k - A, j)]; },
        [&](int i, int j, double acc) { t[v.at(i, j)] = MN[i + (int64_t)j * N] - acc; }, true, sm);
  });
}

// Hessian steps 2+3 of a root front (A = 0, so T_NN = D^-1 K_NN D^-1 and
// nothing else) with its two products spread over 64 x 64 output tiles, one
// workgroup each (blockIdx.x, blockIdx.y: tile; blockIdx.z: right-hand
// side).  STAGE 0: W = K_NN D^-1 into scratch (N x N per right-hand side);
// STAGE 1: T_NN = D^-1 W, lower tiles.  The supernode is list[0].
template <int STAGE>
__global__ void __launch_bounds__(NT) k_hess_down_root(DevPlan P, const int32_t* list, const double* LB,
                                                       const double* Kt, double* T, double* W,
                                                       int64_t wstride) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int i0 = blockIdx.x * TM, j0 = blockIdx.y * TM;
  if (STAGE == 1 && j0 > i0) return;  // a tile wholly above the diagonal (the whole workgroup)
  const int64_t r = blockIdx.z;
  with_staged_cols(SnView(P, list[0]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N;
    const double* K = Kt + r * P.nnz;
    double* t = T + r * P.nnz;
    double* w = W + r * wstride;
    auto Dinv = [&](int i, int j) { return LB[v.nn(i, j)]; };
    if (STAGE == 0)
      tile_gemm<false, true>(
          i0, j0, N, N, N, [&](int i, int k) { return K[v.nn(i, k)]; }, Dinv,
          [&](int i, int j, double acc) { w[i + (int64_t)j * N] = acc; }, false, sm);
    else
      tile_gemm<false, true>(
          i0, j0, N, N, N, Dinv, [&](int k, int j) { return w[k + (int64_t)j * N]; },
          [&](int i, int j, double acc) { t[v.at(i, j)] = acc; }, true, sm);
  });
}
template __global__ void k_hess_down_root<0>(DevPlan, const int32_t*, const double*, const double*, double*,
                                             double*, int64_t);
template __global__ void k_hess_down_root<1>(DevPlan, const int32_t*, const double*, const double*, double*,
                                             double*, int64_t);

// Inverse Hessian steps 1+2 of a root front (A = 0, so K_NN = D T_NN D with
// D = C C^T and nothing else), tile-parallel like k_hess_down_root.
// STAGE 0: D = C C^T into scratch; STAGE 1: W = T_NN D into scratch;
// STAGE 2: K_NN = D W, lower tiles.  Scratch: 2 N^2 per right-hand side
// (D, then W).  The supernode is list[0].
template <int STAGE>
__global__ void __launch_bounds__(NT) k_ihess_down_root(DevPlan P, const int32_t* list, const double* R,
                                                        const double* T, double* Kt, double* W,
                                                        int64_t wstride) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int i0 = blockIdx.x * TM, j0 = blockIdx.y * TM;
  if (STAGE == 2 && j0 > i0) return;  // a tile wholly above the diagonal (the whole workgroup)
  const int64_t r = blockIdx.z;
  with_staged_cols(SnView(P, list[0]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N;
    const double* t = T + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* Dm = W + r * wstride;
    double* Wm = Dm + (int64_t)N * N;
    if (STAGE == 0)
      tile_gemm(
          i0, j0, N, N, N, [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; },
          [&](int k, int j) { return k <= j ? R[v.at(j, k)] : 0.0; },
          [&](int i, int j, double acc) { Dm[i + (int64_t)j * N] = acc; }, false, sm);
    else if (STAGE == 1)
      tile_gemm<false, true>(
          i0, j0, N, N, N, [&](int i, int k) { return t[v.nn(i, k)]; },
          [&](int k, int j) { return Dm[k + (int64_t)j * N]; },
          [&](int i, int j, double acc) { Wm[i + (int64_t)j * N] = acc; }, false, sm);
    else
      tile_gemm<false, true>(
          i0, j0, N, N, N, [&](int i, int k) { return Dm[i + (int64_t)k * N]; },
          [&](int k, int j) { return Wm[k + (int64_t)j * N]; },
          [&](int i, int j, double acc) { K[v.at(i, j)] = acc; }, true, sm);
  });
}
template __global__ void k_ihess_down_root<0>(DevPlan, const int32_t*, const double*, const double*, double*,
                                              double*, int64_t);
template __global__ void k_ihess_down_root<1>(DevPlan, const int32_t*, const double*, const double*, double*,
                                              double*, int64_t);
template __global__ void k_ihess_down_root<2>(DevPlan, const int32_t*, const double*, const double*, double*,
                                              double*, int64_t);

// ---------------------------------------------------------------------------
// Inverse Hessian steps 1 and 2, block form of Algorithm 5.2, for one
// front given V'_s = T_{A_s A_s} in the arena; M_AN = T_AN + V' L;
// M_NN = T_NN + L^T M_AN + T_AN^T L; K_NN = D M_NN D; K_AN = V_s^-1 M_AN D,
// with D = C C^T.  Scratch: 2AN + 3N^2.
__global__ void __launch_bounds__(NT_DOWN) k_ihess_down(DevPlan P, const int32_t* list, const double* R,
                                                   const double* LB, const double* Vi,
                                                   const double* T, double* Kt, double* Va,
                                                   int64_t upd, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols<NT_DOWN>(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const double* t = T + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* va = Va + r * upd;
    const int N = v.N, A = v.A;
    double* MA = slot_ptr(wsb, slot);
    double* Z = MA + (int64_t)A * N;
    double* MN = Z + (int64_t)A * N;
    double* Dm = MN + (int64_t)N * N;
    double* W = Dm + (int64_t)N * N;
    // (V'_s = T_{A_s A_s} is in the arena, gathered beforehand)
    // D = C C^T (full)
    wg_gemm_split<NT_DOWN>(
        N, N, N, [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; },
        [&](int k, int j) { return k <= j ? R[v.at(j, k)] : 0.0; },
        [&](int i, int j, double acc) { Dm[i + (int64_t)j * N] = acc; }, false, sm);
    __syncthreads();
    const double* Vp = va + P.arena[v.s];
    wg_gemm_split<NT_DOWN, false, true>(
        A, N, A, [&](int i, int k) { return sym_packed(Vp, i, k, A); },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { MA[i + (int64_t)j * A] = t[v.an(i, j)] + acc; }, false, sm);
    __syncthreads();
    wg_gemm_split<NT_DOWN, true, true>(
        N, N, 2 * A,
        [&](int i, int k) { return k < A ? LB[v.an(k, i)] : t[v.an(k - A, i)]; },
        [&](int k, int j) { return k < A ? MA[k + (int64_t)j * A] : LB[v.an(k - A, j)]; },
        [&](int i, int j, double acc) {
          const double m = t[v.at(i, j)] + acc;
          MN[i + (int64_t)j * N] = m;
          MN[j + (int64_t)i * N] = m;
        },
        true, sm);
    __syncthreads();
    wg_gemm_split<NT_DOWN, false, true>(
        N, N, N, [&](int i, int k) { return MN[i + (int64_t)k * N]; },
        [&](int k, int j) { return Dm[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false, sm);
    wg_gemm_split<NT_DOWN, false, true>(
        A, N, N, [&](int i, int k) { return MA[i + (int64_t)k * A]; },
        [&](int k, int j) { return Dm[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false, sm);
    __syncthreads();
    wg_gemm_split<NT_DOWN, false, true>(
        N, N, N, [&](int i, int k) { return Dm[i + (int64_t)k * N]; },
        [&](int k, int j) { return W[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { K[v.at(i, j)] = acc; }, true, sm);
    const double* VI = Vi + P.arena[v.s];
    if (A <= kVExplicitMax) {
      wg_gemm_split<NT_DOWN, false, true>(
          A, N, A, [&](int i, int k) { return sym_packed(VI, i, k, A); },
          [&](int k, int j) { return Z[k + (int64_t)j * A]; },
          [&](int i, int j, double acc) { K[v.an(i, j)] = acc; }, false, sm);
    } else {
      // V^-1 Z = C_V^-T (C_V^-1 Z), through MA (free once Z is formed)
      wg_gemm_split<NT_DOWN, false, true>(
          A, N, A, [&](int i, int k) { return k <= i ? VI[pk(i, k, A)] : 0.0; },
          [&](int k, int j) { return Z[k + (int64_t)j * A]; },
          [&](int i, int j, double acc) { MA[i + (int64_t)j * A] = acc; }, false, sm);
      __syncthreads();
      wg_gemm_split<NT_DOWN, true, true>(
          A, N, A, [&](int i, int k) { return k >= i ? VI[pk(k, i, A)] : 0.0; },
          [&](int k, int j) { return MA[k + (int64_t)j * A]; },
          [&](int i, int j, double acc) { K[v.an(i, j)] = acc; }, false, sm);
    }
  });
}

// Triangular solves with an upper triangular U (n x n; U(i, j), i <= j,
// read through a functor) in one workgroup, in place on a column-major B
// (leading dimension ldb, nc columns), blocked by NB: each diagonal block
// is inverted in LDS (diag_trtri of its transpose), the rest are wg_gemm
// updates.  TRANS = false: B <- U^-1 B (last block row first); TRANS =
// true: B <- U^-T B (first block row first).  Ends with a barrier.
template <bool TRANS, class UF>
__device__ __forceinline__ void wg_upper_solve(const UF& U, int n, double* B, int64_t ldb, int nc, double* sm) {
  double* Ld = sm + SMEM_GEMM;
  double* Li = Ld + NB * LDD;
  const int nblk = (n + NB - 1) / NB;
  for (int t = 0; t < nblk; ++t) {
    const int bk = TRANS ? t : nblk - 1 - t;
    const int jb = bk * NB, nb = min(NB, n - jb), r1 = jb + nb;
    if (!TRANS && r1 < n) {
      wg_gemm(
          nb, nc, n - r1, [&](int i, int k) { return U(jb + i, r1 + k); },
          [&](int k, int j) { return B[(r1 + k) + j * ldb]; },
          [&](int i, int j, double acc) { B[(jb + i) + j * ldb] -= acc; }, false, sm);
      __syncthreads();
    }
    if (TRANS && jb > 0) {
      wg_gemm(
          nb, nc, jb, [&](int i, int k) { return U(k, jb + i); }, [&](int k, int j) { return B[k + j * ldb]; },
          [&](int i, int j, double acc) { B[(jb + i) + j * ldb] -= acc; }, false, sm);
      __syncthreads();
    }
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) Ld[i + j * LDD] = U(jb + j, jb + i);  // the block's transpose (lower)
    }
    __syncthreads();
    diag_trtri(Ld, Li, nb);  // Li = U_bb^-T
    wg_gemm(
        nb, nc, nb,
        [&](int i, int k) {
          return TRANS ? (k <= i ? Li[i + k * LDD] : 0.0) : (k >= i ? Li[k + i * LDD] : 0.0);
        },
        [&](int k, int j) { return B[(jb + k) + j * ldb]; },
        [&](int i, int j, double acc) { B[(jb + i) + j * ldb] = acc; }, false, sm);
    __syncthreads();
  }
}

// Inverse Hessian steps 1 and 2 as in k_ihess_down, with the improvement
// noted after Algorithm 5.2: S_{A_s A_s} is used through its factor
// V_s = R_s R_s^T (R_s upper triangular, packed as R_s^T lower in Ru,
// left there by the completion with factored update matrices), so that
// K_AN = R_s^-T R_s^-1 (M_AN D) by two triangular solves and no inverse
// of S_AA is formed.  One workgroup per front and right-hand side.
// Scratch: 2AN + 3N^2.
__global__ void __launch_bounds__(NT) k_ihess_down_factored(DevPlan P, const int32_t* list, const double* R,
                                                            const double* LB, const double* Ru,
                                                            const double* T, double* Kt, double* Va,
                                                            int64_t upd, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const double* t = T + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* va = Va + r * upd;
    const int N = v.N, A = v.A;
    double* MA = slot_ptr(wsb, slot);
    double* Z = MA + (int64_t)A * N;
    double* MN = Z + (int64_t)A * N;
    double* Dm = MN + (int64_t)N * N;
    double* W = Dm + (int64_t)N * N;
    // D = C C^T (full)
    wg_gemm(
        N, N, N, [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; },
        [&](int k, int j) { return k <= j ? R[v.at(j, k)] : 0.0; },
        [&](int i, int j, double acc) { Dm[i + (int64_t)j * N] = acc; }, false, sm);
    __syncthreads();
    // M_AN = T_AN + V' L (V'_s = T_{A_s A_s}, gathered beforehand)
    const double* Vp = va + P.arena[v.s];
    wg_gemm<false, true>(
        A, N, A, [&](int i, int k) { return sym_packed(Vp, i, k, A); },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { MA[i + (int64_t)j * A] = t[v.an(i, j)] + acc; }, false, sm);
    __syncthreads();
    // M_NN = T_NN + L^T M_AN + T_AN^T L
    wg_gemm<true, true>(
        N, N, 2 * A,
        [&](int i, int k) { return k < A ? LB[v.an(k, i)] : t[v.an(k - A, i)]; },
        [&](int k, int j) { return k < A ? MA[k + (int64_t)j * A] : LB[v.an(k - A, j)]; },
        [&](int i, int j, double acc) {
          const double m = t[v.at(i, j)] + acc;
          MN[i + (int64_t)j * N] = m;
          MN[j + (int64_t)i * N] = m;
        },
        true, sm);
    __syncthreads();
    // W = M_NN D, Z = M_AN D, K_NN = D W
    wg_gemm<false, true>(
        N, N, N, [&](int i, int k) { return MN[i + (int64_t)k * N]; },
        [&](int k, int j) { return Dm[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false, sm);
    wg_gemm<false, true>(
        A, N, N, [&](int i, int k) { return MA[i + (int64_t)k * A]; },
        [&](int k, int j) { return Dm[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false, sm);
    __syncthreads();
    wg_gemm<false, true>(
        N, N, N, [&](int i, int k) { return Dm[i + (int64_t)k * N]; },
        [&](int k, int j) { return W[k + (int64_t)j * N]; },
        [&](int i, int j, double acc) { K[v.at(i, j)] = acc; }, true, sm);
    if (A == 0) return;  // (uniform)
    // K_AN = R_s^-T (R_s^-1 Z)
    const double* Rs = Ru + P.arena[v.s];
    auto Rsf = [&](int i, int j) { return Rs[pk(j, i, A)]; };  // R_s(i, j), i <= j
    wg_upper_solve<false>(Rsf, A, Z, A, N, sm);
    wg_upper_solve<true>(Rsf, A, Z, A, N, sm);
    for (int64_t e = threadIdx.x; e < (int64_t)A * N; e += NT) {
      const int x = int(e % A), c = int(e / A);
      K[v.an(x, c)] = Z[e];
    }
  });
}

void launch_ihess_down_factored(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                                const double* LB, const double* Ru, const double* T, double* Kt, double* Va,
                                int64_t upd, double* wsb, int64_t slot) {
  k_ihess_down_factored<<<grid, NT, 0, s>>>(P, list, R, LB, Ru, T, Kt, Va, upd, wsb, slot);
}

// Inverse Hessian step 3 (leaf-to-root), block form of Algorithm 5.2:
// G' = sum E U'_c E^T; Y_NN = K_NN - G'11; Y_AN = L K_NN + K_AN - G'21;
// U'_s = G'22 - L K_NN L^T - L K_AN^T - K_AN L^T.  Scratch: J*N + A*N.
// PANEL: panel columns only; U'_s is left to k_wide_update, which reads Q
// from this workgroup's scratch slot.
template <bool PANEL>
__global__ void __launch_bounds__(NT) k_ihess_up(DevPlan P, const int32_t* list, const double* LB,
                                                 const double* Kt, double* Y, double* Ua,
                                                 int64_t upd, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int64_t r = blockIdx.y;
    const double* K = Kt + r * P.nnz;
    double* y = Y + r * P.nnz;
    double* ua = Ua + r * upd;
    double* Us = ua + P.arena[v.s];
    const int N = v.N, A = v.A;
    double* G = slot_ptr(wsb, slot);
    double* Q = G + (int64_t)v.J * N;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * N; e += NT) G[e] = 0.0;
    if (!PANEL) zero_packed(Us, A);
    __syncthreads();
    if (PANEL)
      assemble_children_panel(P, v, ua, G);
    else
      assemble_children(P, v, ua, G, Us, sm);
    for (int64_t e = threadIdx.x; e < (int64_t)N * N; e += NT) {
      const int i = int(e % N), c = int(e / N);
      if (i >= c) y[v.at(i, c)] = K[v.at(i, c)] - G[i + (int64_t)c * v.J];
    }
    wg_gemm<false, true>(
        A, N, N, [&](int i, int k) { return LB[v.an(i, k)]; },
        [&](int k, int j) { return K[v.nn(k, j)]; },
        [&](int i, int j, double acc) {
          const double q = acc + K[v.an(i, j)];
          Q[i + (int64_t)j * A] = q;
          y[v.an(i, j)] = q - G[(N + i) + (int64_t)j * v.J];
        },
        false, sm);
    if (PANEL) return;
    __syncthreads();
    wg_gemm(
        A, A, 2 * N,
        [&](int i, int k) { return k < N ? Q[i + (int64_t)k * A] : LB[v.an(i, k - N)]; },
        [&](int k, int j) { return k < N ? LB[v.an(j, k)] : K[v.an(j, k - N)]; },
        [&](int i, int j, double acc) { Us[pk(i, j, A)] -= acc; }, true, sm);
  });
}
template __global__ void k_ihess_up<false>(DevPlan, const int32_t*, const double*, const double*, double*,
                                           double*, int64_t, double*, int64_t);
template __global__ void k_ihess_up<true>(DevPlan, const int32_t*, const double*, const double*, double*,
                                          double*, int64_t, double*, int64_t);

// The end of Algorithm 7.3 on one front once W (A x N, leading dimension A,
// with W^T W = S_AN^T V_s^-1 S_AN) and L_AN (in LB) are in place:
// D^-1 = S_NN - W^T W into LB, then C = chol(D) and B = L_AN C into R, and
// the front's part of log det.  ws: 3 N^2 doubles.  No barrier at the end:
// callers synchronize before they reuse LB or R.
__device__ __forceinline__ void completion_finish(const SnView& v, const double* Sin, double* R, double* LB,
                                                  double* part, DevStatus* st, double* ws, const double* W,
                                                  double* sm, int* fail) {
  const int N = v.N, A = v.A;
  double* Dd = ws;
  double* Gi = ws + (int64_t)N * N;
  double* Dm = Gi + (int64_t)N * N;
  wg_gemm<true, true>(
      N, N, A, [&](int i, int k) { return W[k + (int64_t)i * A]; },
      [&](int k, int j) { return W[k + (int64_t)j * A]; },
      [&](int i, int j, double acc) {
        const double d = Sin[v.at(i, j)] - acc;
        LB[v.at(i, j)] = d;
        Dd[i + (int64_t)j * N] = d;
      },
      true, sm);
  __syncthreads();
  if (threadIdx.x == 0) *fail = -1;
  __syncthreads();
  // D = (D^-1)^-1 via its Cholesky factor, then C = chol(D)
  wg_potrf_panel(Dd, N, N, N, sm, fail);
  if (threadIdx.x == 0 && *fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[*fail]);
  wg_trtri([&](int i, int j) { return Dd[i + (int64_t)j * N]; }, N, Gi, N, sm);
  wg_gemm<true, true>(
      N, N, N, [&](int i, int k) { return Gi[k + (int64_t)i * N]; },
      [&](int k, int j) { return Gi[k + (int64_t)j * N]; },
      [&](int i, int j, double acc) { Dm[i + (int64_t)j * N] = acc; }, true, sm);
  __syncthreads();
  if (threadIdx.x == 0) *fail = -1;
  __syncthreads();
  wg_potrf_panel(Dm, N, N, N, sm, fail);
  double lg = 0.0;
  for (int c = threadIdx.x; c < N; c += NT) lg += 2.0 * log(Dm[c + (int64_t)c * N]);
  lg = wg_sum(lg, sm);
  if (threadIdx.x == 0) {
    part[v.s] = lg;
    if (*fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[*fail]);
  }
  for (int64_t e = threadIdx.x; e < (int64_t)N * N; e += NT) {
    const int i = int(e % N), c = int(e / N);
    if (i >= c) R[v.at(i, c)] = Dm[e];
  }
  wg_gemm<false, true>(
      A, N, N, [&](int i, int k) { return LB[v.an(i, k)]; },
      [&](int k, int j) { return k >= j ? Dm[k + (int64_t)j * N] : 0.0; },
      [&](int i, int j, double acc) { R[v.an(i, j)] = acc; }, false, sm);
}

// ---------------------------------------------------------------------------
// Algorithm 7.3: matrix completion of one front, with V_s = S_{A_s A_s}
// already gathered: L_AN = -V_s^-1 S_AN; D^-1 = S_NN +
// S_AN^T L_AN; then C = chol(D), B = L_AN C so that the handle holds the
// factor of X-hat.  Also caches S and the inverse of V_s in its packed
// block (see kVExplicitMax).  Scratch: 3N^2 + AN.
__global__ void __launch_bounds__(NT) k_completion(DevPlan P, const int32_t* list, const double* Sin,
                                                   double* R, double* LB, double* S, double* Vs,
                                                   double* Vi, double* part, DevStatus* st,
                                                   double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double d64[NB2 * LD2];
  __shared__ int64_t colc[kColCache];
  __shared__ int fail;
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    double* ws = slot_ptr(wsb, slot);
    if (threadIdx.x == 0) fail = -1;
    // cache S (own columns) and gather V_s from the input
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * N; e += NT) {
      const int rr = int(e % v.J), c = int(e / v.J);
      if (rr >= c) S[v.at(rr, c)] = Sin[v.at(rr, c)];
    }
    __syncthreads();  // (V_s was gathered beforehand)
    const double* V = Vs + P.arena[v.s];
    double* VI = Vi + P.arena[v.s];
    const PackedLower Cvi{VI, A};  // C_V^-1 once formed
    if (A > 0) packed_tri_inverse(V, VI, A, sm, d64, &fail);  // VI <- C_V^-1, V = C_V C_V^T
    __syncthreads();
    if (threadIdx.x == 0 && fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[0]);
    double* W = ws + 3 * (int64_t)N * N;  // after completion_finish's 3 N^2
    // W = C_V^-1 S_AN, L_AN = -C_V^-T W, D^-1 = S_NN - W^T W: the Schur
    // complement as a difference of Gram products (no explicit V^-1, whose
    // product with S_AN would cancel against S_NN)
    wg_gemm<false, true>(
        A, N, A, [&](int i, int k) { return k <= i ? Cvi(i, k) : 0.0; },
        [&](int k, int j) { return Sin[v.an(k, j)]; },
        [&](int i, int j, double acc) { W[i + (int64_t)j * A] = acc; }, false, sm);
    __syncthreads();
    wg_gemm<true, true>(
        A, N, A, [&](int i, int k) { return k >= i ? Cvi(k, i) : 0.0; },
        [&](int k, int j) { return W[k + (int64_t)j * A]; },
        [&](int i, int j, double acc) { LB[v.an(i, j)] = -acc; }, false, sm);
    completion_finish(v, Sin, R, LB, part, st, ws, W, sm, &fail);
    // the cached block: V^-1 itself up to kVExplicitMax, C_V^-1 beyond
    if (A > 0 && A <= kVExplicitMax) {
      __syncthreads();
      wg_lauum_inplace(Cvi, A, sm);
    }
  });
}

// Algorithm 7.3 with factored update matrices (the supernodal form of
// Algorithm 4.3): V_s = S_{A_s A_s} is carried as V_s = R_s R_s^T, R_s
// upper triangular with a positive diagonal, obtained from the parent's
// R_p instead of being factored from scratch.  A_s splits into A_s ∩ N_p
// (its first p1 indices) and A_s \ N_p (m indices, all in A_p), so that
// V_s = [A B^T; B C C^T] with A and B from the parent's panel of S and C
// the rows of R_p at A_s \ N_p.  C = R Q^T by Householder reflections
// applied from the right (last row first; a row with no weight left of its
// diagonal column is left alone), R's diagonal made positive by column
// signs; W = R^-1 B; A - W^T W = T T^T with T upper triangular (Cholesky
// of the index-reversed matrix); R_s = [T W^T; 0 R], kept as R_s^T packed
// lower in the front's block of Ru.  Then Z = R_s^-1 S_AN, L_AN =
// -R_s^-T Z, and the front is finished as in k_completion with W = Z.
// One root-to-leaf level per launch (the parents' R_p are in place).
// Scratch: 3N^2 + 2AN + A Ap + A^2 + 2 Ap + 64 doubles (Ap: the parent's A).
__global__ void __launch_bounds__(NT) k_completion_factored(DevPlan P, const int32_t* list, const double* Sin,
                                                            double* R, double* LB, double* S, double* Ru,
                                                            double* part, DevStatus* st, double* wsb,
                                                            int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  __shared__ int fail, sh_p1;
  __shared__ double sh_tau[2];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    double* ws = slot_ptr(wsb, slot);
    double* Z = ws + 3 * (int64_t)N * N;
    double* X = Z + (int64_t)A * N;
    double* Cm = X + (int64_t)A * N;
    if (threadIdx.x == 0) fail = -1;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * N; e += NT) {
      const int rr = int(e % v.J), c = int(e / v.J);
      if (rr >= c) S[v.at(rr, c)] = Sin[v.at(rr, c)];
    }
    double* Rs = Ru + P.arena[v.s];
    if (A > 0) {
      const int p = P.parent[v.s];
      const SnView vp(P, p);
      const int Np = vp.N, Ap = vp.A;
      const int32_t* rl = P.rel + P.relbase[v.s];  // positions of A_s in J_p, ascending
      const double* Rp = Ru + P.arena[p];
      if (threadIdx.x == 0) {
        int lo = 0, hi = A;  // first position at or beyond N_p
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (rl[mid] < Np) lo = mid + 1;
          else hi = mid;
        }
        sh_p1 = lo;
      }
      __syncthreads();
      const int p1 = sh_p1, m = A - p1;
      const int c0 = m > 0 ? rl[p1] - Np : 0, wC = Ap - c0;  // C holds columns c0 .. Ap-1 of R_p
      const int qc = wC - m;                                 // R: the last m of them
      double* Wb = Cm + (int64_t)m * wC;
      double* Fl = Wb + (int64_t)m * p1;
      double* vh = Fl + (int64_t)p1 * p1;
      auto Rm = [&](int i, int j) { return Cm[i + (int64_t)(qc + j) * m]; };
      if (m > 0) {
        for (int64_t e = threadIdx.x; e < (int64_t)m * wC; e += NT) {
          const int cc = int(e % wC), k = int(e / wC);
          const int r = rl[p1 + k] - Np, c = c0 + cc;
          Cm[k + (int64_t)cc * m] = c >= r ? Rp[pk(c, r, Ap)] : 0.0;  // R_p(r, c) = R_p^T(c, r)
        }
        __syncthreads();
        // Row x belongs to thread x % NT, which alone reads and writes it, so
        // a step needs one barrier: the owner of row k forms its reflection
        // (v, tau) from the row as it left it, publishes v in one of two
        // buffers (LDS when C is at most kHhLds columns wide), and every
        // thread applies it to its rows above k.  A buffer is rewritten two
        // steps later, after every thread has passed the barrier between.
        constexpr int kHhLds = SMEM_DOUBLES / 2;
        double* vb = wC <= kHhLds ? sm : vh;
        const int vstride = wC <= kHhLds ? kHhLds : wC;
        for (int k = m - 1; k >= 0; --k) {
          const int lo = rl[p1 + k] - Np - c0, q = qc + k;  // the row's first and diagonal columns
          double* v = vb + (k & 1) * vstride;
          if (threadIdx.x == k % NT) {
            double rest = 0.0;
            for (int b = lo; b < q; ++b) rest += Cm[k + (int64_t)b * m] * Cm[k + (int64_t)b * m];
            double tau = 0.0;  // no weight left of the diagonal column: H = I
            if (rest != 0.0) {
              const double xq = Cm[k + (int64_t)q * m];
              const double nrm = sqrt(rest + xq * xq);
              const double alpha = xq >= 0.0 ? -nrm : nrm;
              tau = 2.0 / (rest + (xq - alpha) * (xq - alpha));
              for (int b = lo; b < q; ++b) {
                v[b] = Cm[k + (int64_t)b * m];
                Cm[k + (int64_t)b * m] = 0.0;
              }
              v[q] = xq - alpha;
              Cm[k + (int64_t)q * m] = alpha;
            }
            sh_tau[k & 1] = tau;
          }
          __syncthreads();
          const double tau = sh_tau[k & 1];
          if (tau != 0.0)
            for (int x = threadIdx.x; x < k; x += NT) {
              double d = 0.0;
              for (int b = lo; b <= q; ++b) d += Cm[x + (int64_t)b * m] * v[b];
              d *= tau;
              for (int b = lo; b <= q; ++b) Cm[x + (int64_t)b * m] -= d * v[b];
            }
        }
        __syncthreads();
        for (int b = threadIdx.x; b < m; b += NT) vh[b] = Rm(b, b) < 0.0 ? -1.0 : 1.0;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += NT) {
          const int i = int(e % m), j = int(e / m);
          if (i <= j && vh[j] < 0.0) Cm[i + (int64_t)(qc + j) * m] = -Cm[i + (int64_t)(qc + j) * m];
        }
        __syncthreads();
        if (p1 > 0) {
          // W = R^-1 B, B(x, y) = S(A_s[p1 + x], A_s[y]) from the parent's panel
          for (int64_t e = threadIdx.x; e < (int64_t)m * p1; e += NT) {
            const int x = int(e % m), y = int(e / m);
            Wb[e] = Sin[vp.at(rl[p1 + x], rl[y])];
          }
          __syncthreads();
          wg_upper_solve<false>(Rm, m, Wb, m, p1, sm);
        }
      }
      if (p1 > 0) {
        // A - W^T W, index-reversed (Fl(p1-1-j, p1-1-i) for i >= j), then its Cholesky
        wg_gemm<true, true>(
            p1, p1, m, [&](int i, int k) { return Wb[k + (int64_t)i * m]; },
            [&](int k, int j) { return Wb[k + (int64_t)j * m]; },
            [&](int i, int j, double acc) {
              Fl[(p1 - 1 - j) + (int64_t)(p1 - 1 - i) * p1] = Sin[vp.at(rl[i], rl[j])] - acc;
            },
            true, sm);
        __syncthreads();
        wg_potrf_panel(Fl, p1, p1, p1, sm, &fail);
        __syncthreads();
      }
      if (threadIdx.x == 0 && fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[0]);
      // R_s^T packed lower: entry (x, y), x >= y, is R_s(y, x)
      for (int64_t e = threadIdx.x; e < (int64_t)A * A; e += NT) {
        const int x = int(e % A), y = int(e / A);
        if (x < y) continue;
        double val;
        if (y >= p1)
          val = Rm(y - p1, x - p1);
        else if (x >= p1)
          val = Wb[(x - p1) + (int64_t)y * m];
        else
          val = Fl[(p1 - 1 - y) + (int64_t)(p1 - 1 - x) * p1];
        Rs[pk(x, y, A)] = val;
      }
      __syncthreads();
    }
    // Z = R_s^-1 S_AN; L_AN = -R_s^-T Z
    for (int64_t e = threadIdx.x; e < (int64_t)A * N; e += NT) {
      const int x = int(e % A), c = int(e / A);
      Z[e] = Sin[v.an(x, c)];
    }
    __syncthreads();
    if (A > 0) {
      auto Rsf = [&](int i, int j) { return Rs[pk(j, i, A)]; };  // R_s(i, j), i <= j
      wg_upper_solve<false>(Rsf, A, Z, A, N, sm);
      for (int64_t e = threadIdx.x; e < (int64_t)A * N; e += NT) X[e] = Z[e];
      __syncthreads();
      wg_upper_solve<true>(Rsf, A, X, A, N, sm);
      for (int64_t e = threadIdx.x; e < (int64_t)A * N; e += NT) {
        const int x = int(e % A), c = int(e / A);
        LB[v.an(x, c)] = -X[e];
      }
      __syncthreads();
    }
    completion_finish(v, Sin, R, LB, part, st, ws, Z, sm, &fail);
  });
}

void launch_completion_factored(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* Sin,
                                double* R, double* LB, double* S, double* Ru, double* part, DevStatus* st,
                                double* wsb, int64_t slot) {
  k_completion_factored<<<grid, NT, 0, s>>>(P, list, Sin, R, LB, S, Ru, part, st, wsb, slot);
}

// The inverse of S_{A_s A_s} for every supernode in the list (needs the
// cached V_s), in place in the packed Vi block (no scratch): V^-1 up to
// order kVExplicitMax, the inverse Cholesky factor C_V^-1 beyond.
__global__ void __launch_bounds__(NT) k_vinv(DevPlan P, const int32_t* list, const double* Vs,
                                             double* Vi, DevStatus* st, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double d64[NB2 * LD2];
  __shared__ int64_t colc[kColCache];
  __shared__ int fail;
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    if (v.A == 0) return;
    if (threadIdx.x == 0) fail = -1;
    __syncthreads();
    double* VI = Vi + P.arena[v.s];
    packed_tri_inverse(Vs + P.arena[v.s], VI, v.A, sm, d64, &fail);
    if (v.A <= kVExplicitMax) {
      __syncthreads();
      wg_lauum_inplace(PackedLower{VI, v.A}, v.A, sm);
    }
    if (threadIdx.x == 0 && fail >= 0) report(st, MFB_ENOTPD, v.vl[0]);
  });
}

// Gather pass of the steps that read a block of their input (V_s =
// S_{A_s A_s} for the completion, V'_s = T_{A_s A_s} for the inverse
// Hessian) with the plan's source map: arena[e] = src[map[e]] for
// every packed update-block entry e < n (right-hand side blockIdx.y), one
// elementwise launch for all supernodes.
// TAG only names the caller in profiles (1 inverse Hessian, 2 completion).
template <int TAG>
__global__ void __launch_bounds__(NT) k_gather_map(const int64_t* map, int64_t n, const double* src,
                                                   double* arena, int64_t src_stride, int64_t arena_stride) {
  const int64_t r = blockIdx.y;
  const double* sr = src + r * src_stride;
  double* ar = arena + r * arena_stride;
  for (int64_t e = int64_t(blockIdx.x) * NT + threadIdx.x; e < n; e += int64_t(gridDim.x) * NT)
    ar[e] = sr[map[e]];
}
template __global__ void k_gather_map<1>(const int64_t*, int64_t, const double*, double*, int64_t, int64_t);
template __global__ void k_gather_map<2>(const int64_t*, int64_t, const double*, double*, int64_t, int64_t);

// ---------------------------------------------------------------------------
// Algorithm 3.2 in block form (leaf-to-root): with G = sum E U_c E^T,
// X_NN = C C^T - G11, X_AN = B C^T - G21, U_s = G22 - B B^T.  Scratch: J*N.
// PANEL: panel columns only; U_s is left to k_wide_update.
template <bool PANEL>
__global__ void __launch_bounds__(NT) k_product(DevPlan P, const int32_t* list, const double* R,
                                                double* X, double* U, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    double* G = slot_ptr(wsb, slot);
    double* Us = U + P.arena[v.s];
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * N; e += NT) G[e] = 0.0;
    if (!PANEL) zero_packed(Us, A);
    __syncthreads();
    if (PANEL)
      assemble_children_panel(P, v, U, G);
    else
      assemble_children(P, v, U, G, Us, sm);
    auto C = [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; };
    wg_gemm(
        N, N, N, C, [&](int k, int j) { return C(j, k); },
        [&](int i, int j, double acc) { X[v.at(i, j)] = acc - G[i + (int64_t)j * v.J]; }, true, sm);
    wg_gemm(
        A, N, N, [&](int i, int k) { return R[v.an(i, k)]; }, [&](int k, int j) { return C(j, k); },
        [&](int i, int j, double acc) { X[v.an(i, j)] = acc - G[(N + i) + (int64_t)j * v.J]; }, false,
        sm);
    if (PANEL) return;
    wg_gemm(
        A, A, N, [&](int i, int k) { return R[v.an(i, k)]; },
        [&](int k, int j) { return R[v.an(j, k)]; },
        [&](int i, int j, double acc) { Us[pk(i, j, A)] -= acc; }, true, sm);
  });
}
template __global__ void k_product<false>(DevPlan, const int32_t*, const double*, double*, double*, double*,
                                          int64_t);
template __global__ void k_product<true>(DevPlan, const int32_t*, const double*, double*, double*, double*,
                                         int64_t);

// ---------------------------------------------------------------------------
// log det = sum of the per-supernode contributions, fixed-order reduction.
__global__ void __launch_bounds__(NT) k_logdet(const double* part, int ns, double* out) {
  __shared__ double sm[NT];
  double v = 0.0;
  for (int i = threadIdx.x; i < ns; i += NT) v += part[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// Scalar L D L^T from the Cholesky factor: D_jj = R_jj^2, L_ij = R_ij / R_jj.
__global__ void __launch_bounds__(NT) k_export_ldl(const double* R, const int64_t* colptr,
                                                   const int32_t* colidx, int64_t nnz, double* out) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * NT) {
    const int64_t d = colptr[colidx[e]];
    const double rd = R[d];
    out[e] = e == d ? rd * rd : R[e] / rd;
  }
}

// Relaxed plans.  In: k arrays on V (nu entries each) onto V' (nv each),
// entry e to e + shift[e] and zero on the nz entries of V' \ V.  Out: the
// reverse restriction.  Right-hand side r = blockIdx.y.
__global__ void __launch_bounds__(NT) k_relax_in(const double* __restrict__ src, int64_t nu,
                                                 const int32_t* __restrict__ shift,
                                                 const int64_t* __restrict__ zpos, int64_t nz,
                                                 double* __restrict__ dst, int64_t nv) {
  src += int64_t(blockIdx.y) * nu;
  dst += int64_t(blockIdx.y) * nv;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nu + nz; e += (int64_t)gridDim.x * NT) {
    if (e < nu)
      dst[e + shift[e]] = src[e];
    else
      dst[zpos[e - nu]] = 0.0;
  }
}

__global__ void __launch_bounds__(NT) k_relax_out(const double* __restrict__ src, int64_t nv,
                                                  const int32_t* __restrict__ shift, double* __restrict__ dst,
                                                  int64_t nu) {
  src += int64_t(blockIdx.y) * nv;
  dst += int64_t(blockIdx.y) * nu;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nu; e += (int64_t)gridDim.x * NT)
    dst[e] = src[e + shift[e]];
}

void launch_relax_in(hipStream_t s, int k, const double* src, int64_t nu, const int32_t* shift, const int64_t* zpos,
                     int64_t nz, double* dst, int64_t nv) {
  if (k <= 0 || nu + nz == 0) return;
  const unsigned bx = unsigned(std::min<int64_t>((nu + nz + NT - 1) / NT, 4096));
  k_relax_in<<<dim3(bx, unsigned(k)), NT, 0, s>>>(src, nu, shift, zpos, nz, dst, nv);
}

void launch_relax_out(hipStream_t s, int k, const double* src, int64_t nv, const int32_t* shift, double* dst,
                      int64_t nu) {
  if (k <= 0 || nu == 0) return;
  const unsigned bx = unsigned(std::min<int64_t>((nu + NT - 1) / NT, 4096));
  k_relax_out<<<dim3(bx, unsigned(k)), NT, 0, s>>>(src, nv, shift, dst, nu);
}

__global__ void k_reset_status(DevStatus* st) {
  if (threadIdx.x == 0) {
    st->code = 0;
    st->pad = 0;
    st->bad = ~0ull;
  }
}


// ---------------------------------------------------------------------------
// Register-front kernels: the whole J x J front (or the A x A block V_s) of a
// supernode lives in the registers of one workgroup (reg_front.h), so the
// dense part is a sequence of rank-1 or rank-2 steps with one LDS broadcast
// and one barrier each.  Fronts are read from and written to HBM once, with
// branch-free gathers (every address is computed, invalid lanes read a
// valid dummy address and discard the value).  Used for fronts up to order
// 192; the blocked kernels above serve larger ones.

// Columns of L_AN (or of the Cholesky panel) staged per LDS pass.
constexpr int KCL = 8;

// Only the lower triangle of a register front is read or written: the
// elimination steps never read entries above the diagonal (reg_front.h),
// so those registers start at zero and are left stale.

// CCS offsets of the lower panel entries a thread owns: entry (i, j),
// i >= j, j < N, lives at col[j] + (i - j).  Columns are clamped to N - 1
// for columns outside the panel (their offsets are never used).
template <class C>
struct PanelIdx {
  int64_t cc[C::RY];
  template <bool LO>
  __device__ __forceinline__ PanelIdx(const RegFront<C, LO>& M, const SnView& v) {
#pragma unroll
    for (int b = 0; b < C::RY; ++b) cc[b] = v.col[min(M.col(b), v.N - 1)];
  }
};

// Loads the lower panel part (j < N) of the front from the CCS array src;
// everything else is zero.
template <class C, bool LO>
__device__ __forceinline__ void load_panel(RegFront<C, LO>& M, const SnView& v, const double* src) {
  const PanelIdx<C> ix(M, v);
#pragma unroll
  for (int a = 0; a < C::RX; ++a)
#pragma unroll
    for (int b = 0; b < C::RY; ++b) {
      M.v[a][b] = 0.0;
      if (M.skip(a, b)) continue;
      const int i = M.row(a), j = M.col(b);
      const bool ok = i < v.J && j < v.N && i >= j;
      const double x = src[ok ? ix.cc[b] + (i - j) : 0];
      M.v[a][b] = ok ? x : 0.0;
    }
}

// Stores the lower panel entries (j < N) through out(offset, value) and
// the lower A x A entries through outa(packed index, value).
template <class C, bool LO, class OP, class OA>
__device__ __forceinline__ void store_front(const RegFront<C, LO>& M, const SnView& v, const OP& out,
                                            const OA& outa) {
  const PanelIdx<C> ix(M, v);
  const int N = v.N, A = v.A;
  M.store_lower(
      v.J, [](int, int) { return true; },
      [&](int, int b, int i, int j, double x) {
        if (j < N)
          out(ix.cc[b] + (i - j), x);
        else
          outa(pk(i - N, j - N, A), x);
      });
}

// Lower A x A block <- V_s = E^T [S_NN S_AN^T; S_AN V_p] E gathered from
// the parent's CCS columns of `src` and its packed block in `arena`
// (eq. e-sn-gradient-2).  Relative indices increase, so i >= j maps to a
// lower entry of the parent's front.  No-op for A = 0.
template <class C, bool LO>
__device__ __forceinline__ void gather_parent(RegFront<C, LO>& M, const DevPlan& P, const SnView& v,
                                              const double* src, const double* arena) {
  if (v.A == 0) return;
  const int N = v.N, J = v.J;
  const int p = P.parent[v.s];
  const int Np = P.ncol[p], Ap = P.nrow[p] - Np;
  const int64_t* colp = P.col + P.colbase[p];
  const int32_t* rl = P.rel + P.relbase[v.s];
  const double* Vp = arena + P.arena[p];
  int rr[C::RX], rc[C::RY];
  int64_t cpc[C::RY];
#pragma unroll
  for (int a = 0; a < C::RX; ++a) {
    const int i = M.row(a);
    rr[a] = (i >= N && i < J) ? rl[i - N] : 0;
  }
#pragma unroll
  for (int b = 0; b < C::RY; ++b) {
    const int j = M.col(b);
    rc[b] = (j >= N && j < J) ? rl[j - N] : 0;
    cpc[b] = colp[min(rc[b], Np - 1)];
  }
#pragma unroll
  for (int a = 0; a < C::RX; ++a)
#pragma unroll
    for (int b = 0; b < C::RY; ++b) {
      if (M.skip(a, b)) continue;
      const int i = M.row(a), j = M.col(b);
      const bool in = j >= N && i < J && i >= j;
      const double* q = !in ? src
                            : (rc[b] < Np ? src + cpc[b] + (rr[a] - rc[b])
                                          : Vp + pk(rr[a] - Np, rc[b] - Np, Ap));
      const double x = *q;
      if (in) M.v[a][b] = x;
    }
}

// The A x A block of the front from this supernode's packed lower block U
// (entries (i, j), N <= j <= i < J).
template <class C, bool LO>
__device__ __forceinline__ void load_packed_block(RegFront<C, LO>& M, const SnView& v, const double* U) {
  const int N = v.N, J = v.J, A = v.A;
#pragma unroll
  for (int a = 0; a < C::RX; ++a)
#pragma unroll
    for (int b = 0; b < C::RY; ++b) {
      if (M.skip(a, b)) continue;
      const int i = M.row(a), j = M.col(b);
      const bool in = j >= N && i < J && i >= j;
      const double x = U[in ? pk(i - N, j - N, A) : 0];
      if (in) M.v[a][b] = x;
    }
}

// Front += sg * sum over children c of E_c U_c E_c^T (lower triangle),
// with the children's packed blocks taken from `ua`; one child at a time
// through an inverse relative-index map in LDS (`inv`, MMAX ints).
template <class C, bool LO>
__device__ __forceinline__ void gather_children(RegFront<C, LO>& M, const DevPlan& P, const SnView& v,
                                                const double* ua, int* inv, double sg,
                                                const int32_t* act = nullptr) {
  for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
    const int c = P.cidx[t];
    if (act && !act[c]) continue;  // (uniform: a child inactive in Hessian step 1)
    const int Ac = P.nrow[c] - P.ncol[c];
    const int32_t* rl = P.rel + P.relbase[c];
    const double* Uc = ua + P.arena[c];
    for (int i = threadIdx.x; i < C::MMAX; i += C::NTH) inv[i] = -1;
    __syncthreads();
    for (int x = threadIdx.x; x < Ac; x += C::NTH) inv[rl[x]] = x;
    __syncthreads();
    int xi[C::RX], yj[C::RY];
#pragma unroll
    for (int a = 0; a < C::RX; ++a) xi[a] = inv[M.row(a)];
#pragma unroll
    for (int b = 0; b < C::RY; ++b) yj[b] = inv[M.col(b)];
    __syncthreads();
    // rows in groups of GR, so the loads in flight stay within the
    // registers the front leaves free
    constexpr int GR = C::RX * C::RY > 32 ? (32 + C::RY - 1) / C::RY : C::RX;
#pragma unroll
    for (int a0 = 0; a0 < C::RX; a0 += GR) {
      double tv[GR][C::RY];
#pragma unroll
      for (int g = 0; g < GR; ++g)
#pragma unroll
        for (int b = 0; b < C::RY; ++b) {
          const int a = a0 + g < C::RX ? a0 + g : C::RX - 1;
          const bool ok = a0 + g < C::RX && !M.skip(a, b) && xi[a] >= yj[b] && yj[b] >= 0;
          const double x = Uc[ok ? pk(xi[a], yj[b], Ac) : 0];
          tv[g][b] = ok ? sg * x : 0.0;
        }
#pragma unroll
      for (int g = 0; g < GR; ++g)
#pragma unroll
        for (int b = 0; b < C::RY; ++b)
          if (a0 + g < C::RX && !M.skip(a0 + g, b)) M.v[a0 + g][b] += tv[g][b];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Columns k0 .. k0 + KCL - 1 of the N columns given by val(i, k) for
// rows i below MMAX (zero where val is not taken) into LDS:
// Ls[i + t MMAX] = val(i, k0 + t).
template <class C, class VF>
__device__ __forceinline__ void stage_columns(int N, int k0, double* Ls, const VF& val) {
  for (int e = threadIdx.x; e < C::MMAX * KCL; e += C::NTH) {
    const int i = e % C::MMAX, t = e / C::MMAX;
    Ls[e] = k0 + t < N ? val(i, k0 + t) : 0.0;
  }
}

// The N congruences with the columns of [0; L_AN] (staged KCL at a time):
// fronts of order above 64 take them in blocks of KCL (two barriers per
// block; the extra small solve per block does not pay on smaller fronts),
// smaller ones one step at a time.  `lds` holds kCongLds<C> doubles.
// With A = 0 (a root front) every l_k is zero and the congruences are the
// identity, so none is taken; the early return is uniform over the
// workgroup and leaves no LDS access unfenced (the callers' other steps
// bracket their own LDS use with barriers).
template <class C>
constexpr int kCongLds = C::MMAX > 64 ? 6 * KCL * C::MMAX : (4 + KCL) * C::MMAX;
template <class C, bool LO>
__device__ __forceinline__ void congruences(RegFront<C, LO>& M, const SnView& v, const double* LB, double sg,
                                            double* lds) {
  if (v.A == 0) return;
  auto stage = [&](int k0, double* ls) {
    stage_columns<C>(v.N, k0, ls, [&](int i, int kk) {
      const bool ok = i >= v.N && i < v.J;
      const double x = LB[ok ? v.at(i, kk) : 0];
      return ok ? x : 0.0;
    });
  };
  if constexpr (C::MMAX > 64)
    M.template congruences_blocked<KCL>(v.N, sg, lds, stage);
  else
    M.template congruences<KCL>(v.N, sg, lds, lds + 4 * C::MMAX, stage);
}

// Column k of the Cholesky factor from the broadcast column of the sweep
// of pivot k (rows k .. J-1 of `bk`, pivot p): R[col[k] + i - k] =
// bk[i] / sqrt(p), one row per thread.
__device__ __forceinline__ void put_chol_column(const SnView& v, int k, const double* bk, double p,
                                                const int64_t* colc, double* R) {
  const int i = k + threadIdx.x;
  if (i < v.J) R[colc[k] + (i - k)] = bk[i] * fast_rsqrt(p);
}

// sum_{k < n} log piv[k] (LDS), by the first wavefront in a fixed order;
// the result is valid in thread 0.  Call with all threads after a barrier
// that published piv.
__device__ __forceinline__ double sum_log_pivots(const double* piv, int n) {
  double s = 0.0;
  if (threadIdx.x < 64) {
    for (int k = threadIdx.x; k < n; k += 64) s += log(piv[k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  }
  return s;
}

// Column offsets of the supernode's panel into LDS (colc[c] = col[c]).
template <class C>
__device__ __forceinline__ void stage_col(const SnView& v, int64_t* colc) {
  for (int c = threadIdx.x; c < v.N; c += C::NTH) colc[c] = v.col[c];
}

// (S_{A_s A_s})^-1 by sweeping every pivot of V_s.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_vinv_reg(DevPlan P, const int32_t* list, const double* Vs,
                                                     double* Vi, DevStatus* st) {
  __shared__ double buf[4 * C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int A = v.A;
  if (A == 0) return;
  const double* V = Vs + P.arena[v.s];
  double* VI = Vi + P.arena[v.s];
  RegFront<C> M;
#pragma unroll
  for (int a = 0; a < C::RX; ++a)
#pragma unroll
    for (int b = 0; b < C::RY; ++b) {
      M.v[a][b] = 0.0;
      if (M.skip(a, b)) continue;
      const int i = M.row(a), j = M.col(b);
      const bool ok = i < A && i >= j;
      const double x = V[ok ? pk(i, j, A) : 0];
      M.v[a][b] = ok ? x : 0.0;
    }
  const bool bad = M.sweeps(0, A, buf) >= 0;
  M.store_lower(
      A, [](int, int) { return true; }, [&](int, int, int i, int j, double x) { VI[pk(i, j, A)] = -x; });
  if (threadIdx.x == 0 && bad) report(st, MFB_ENOTPD, v.vl[0]);
}

// Algorithm 7.1 on a register front.  After the extend-add, sweeping the N
// pivots of F = [D_NN X_AN^T; X_AN F22] leaves [-D^-1, .; L_AN, U_s] with
// L_AN = X_AN D^-1 and U_s = F22 - X_AN D^-1 X_AN^T (the block L D L^T
// step), and the column broadcast before each pivot gives the Cholesky
// panel [C; B] and log det D_NN = sum of log pivots.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_factor_reg(DevPlan P, const int32_t* list, const double* x,
                                                       double* R, double* LB, double* U, double* part,
                                                       DevStatus* st) {
  __shared__ double buf[4 * C::MMAX];
  __shared__ int inv[C::MMAX];
  __shared__ int64_t colc[C::MMAX];
  __shared__ double piv[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int N = v.N, A = v.A;
  double* Us = U + P.arena[v.s];
  stage_col<C>(v, colc);
  RegFront<C> M;
  load_panel(M, v, x);
  gather_children(M, P, v, U, inv, 1.0);
  const int fail = M.sweeps(0, N, buf, [&](const double* bk, double p, int k) {
    put_chol_column(v, k, bk, p, colc, R);
    if (threadIdx.x == 0) piv[k] = p;
  });
  store_front(
      M, v,
      [&](int64_t o, double y) {
        // N x N block: -D^-1 (sign flipped here); A x N block: L_AN
        LB[o] = y;
      },
      [&](int64_t e, double y) { Us[e] = y; });
  M.store_lower(
      N, [](int, int) { return true; },
      [&](int, int b, int i, int j, double y) { LB[colc[j] + (i - j)] = -y; });
  __syncthreads();
  const double lg = sum_log_pivots(piv, N);
  if (threadIdx.x == 0) {
    part[v.s] = lg;
    if (fail >= 0) report(st, MFB_ENOTPD, v.vl[fail]);
  }
  (void)A;
}

// Algorithm 7.3 on a register front G = S_{J_s J_s} = [S_NN S_AN^T; S_AN V_s].
// Sweeping the A pivots leaves [D^-1, -L_AN^T; -L_AN, -V_s^-1] with
// L_AN = -V_s^-1 S_AN and D^-1 = S_NN + S_AN^T L_AN; sweeping the N pivots
// next turns the first N columns into -[D; L_AN D].  A last sweep of the N
// pivots of [D; L_AN D] broadcasts the columns of its Cholesky panel,
// C = chol(D) and B = L_AN D C^-T = L_AN C, and log det D.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_completion_reg(DevPlan P, const int32_t* list,
                                                           const double* Sin, double* R, double* LB,
                                                           double* S, double* Vs, double* Vi,
                                                           double* part, DevStatus* st) {
  __shared__ double buf[4 * C::MMAX];
  __shared__ int64_t colc[C::MMAX];
  __shared__ double piv[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int N = v.N, A = v.A, J = v.J;
  double* VS = Vs + P.arena[v.s];
  double* VI = Vi + P.arena[v.s];
  stage_col<C>(v, colc);
  RegFront<C> M;
  load_panel(M, v, Sin);
  load_packed_block(M, v, VS);  // V_s, gathered beforehand
  // cache S (own columns)
  store_front(M, v, [&](int64_t o, double y) { S[o] = y; }, [](int64_t, double) {});
  const bool badV = M.sweeps(N, J, buf) >= 0;
  // L_AN = -(swept A x N block), D^-1 = swept N x N block, V_s^-1 = -(swept A x A block)
  M.store_lower(
      J, [](int, int) { return true; },
      [&](int, int, int i, int j, double y) {
        if (j < N)
          LB[colc[j] + (i - j)] = i >= N ? -y : y;
        else
          VI[pk(i - N, j - N, A)] = -y;
      });
  if (threadIdx.x == 0 && badV) report(st, MFB_ENOCOMPLETION, v.vl[0]);
  int fail = M.sweeps(0, N, buf);
  M.negate_columns(N);
  const int fail2 = M.sweeps(0, N, buf, [&](const double* bk, double p, int k) {
    put_chol_column(v, k, bk, p, colc, R);
    if (threadIdx.x == 0) piv[k] = p;
  });
  if (fail < 0) fail = fail2;
  __syncthreads();
  const double lg = sum_log_pivots(piv, N);
  if (threadIdx.x == 0) {
    part[v.s] = lg;
    if (fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[fail]);
  }
}

// Hessian step 1 (leaf-to-root) on a register front: with E = [I 0; L I],
// E^-1 F' E^-T = [K_NN K_AN^T; K_AN U'_s] for F' = [Y_NN Y_AN^T; Y_AN 0] +
// sum E_c U'_c E_c^T (the block formulas K_AN = F'21 - L F'11 and
// U'_s = F'22 - L F'12 - K_AN L^T), applied as N congruence steps.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_hess_up_reg(DevPlan P, const int32_t* list, const double* LB,
                                                        const double* Y, double* Kt, double* Ua,
                                                        int64_t upd, int32_t* act) {
  __shared__ double lds[kCongLds<C>];
  __shared__ int inv[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int64_t r = blockIdx.y;
  const double* y = Y + r * P.nnz;
  double* K = Kt + r * P.nnz;
  double* ua = Ua + r * upd;
  double* Us = ua + P.arena[v.s];
  int32_t* ac = act + r * P.ns;
  RegFront<C> M;
  load_panel(M, v, y);
  bool own = false;
#pragma unroll
  for (int a = 0; a < C::RX; ++a)
#pragma unroll
    for (int b = 0; b < C::RY; ++b) own = own || M.v[a][b] != 0.0;
  bool active = __syncthreads_or(own ? 1 : 0) != 0;
  for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1] && !active; ++t) active = ac[P.cidx[t]] != 0;
  if (!active) {
    // no nonzero of Y below this front: K = 0 (the panel loaded as zero)
    // and no update block (the parent skips it)
    store_front(M, v, [&](int64_t o, double x) { K[o] = x; }, [&](int64_t, double) {});
    if (threadIdx.x == 0) ac[v.s] = 0;
    return;
  }
  gather_children(M, P, v, ua, inv, 1.0, ac);
  congruences<C>(M, v, LB, -1.0, lds);
  store_front(M, v, [&](int64_t o, double x) { K[o] = x; }, [&](int64_t e, double x) { Us[e] = x; });
}

// Inverse Hessian step 3 (leaf-to-root) on a register front:
// E [K_NN K_AN^T; K_AN 0] E^T - G' = [Y_NN Y_AN^T; Y_AN -U'_s] with
// G' = sum E_c U'_c E_c^T (Y_AN = L K_NN + K_AN - G'21, U'_s = G'22 -
// L K_NN L^T - L K_AN^T - K_AN L^T), applied as N congruence steps.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_ihess_up_reg(DevPlan P, const int32_t* list, const double* LB,
                                                         const double* Kt, double* Y, double* Ua,
                                                         int64_t upd) {
  __shared__ double lds[kCongLds<C>];
  __shared__ int inv[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int64_t r = blockIdx.y;
  const double* K = Kt + r * P.nnz;
  double* y = Y + r * P.nnz;
  double* ua = Ua + r * upd;
  double* Us = ua + P.arena[v.s];
  RegFront<C> M;
  load_panel(M, v, K);
  congruences<C>(M, v, LB, 1.0, lds);
  gather_children(M, P, v, ua, inv, -1.0);
  store_front(M, v, [&](int64_t o, double x) { y[o] = x; }, [&](int64_t e, double x) { Us[e] = -x; });
}

// Algorithm 3.2 in block form on a register front: R R^T - G =
// [X_NN X_AN^T; X_AN -U_s] for the Cholesky panel R = [C; B] and
// G = sum E_c U_c E_c^T, with R R^T accumulated from R's columns staged
// through LDS KCL at a time.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_product_reg(DevPlan P, const int32_t* list, const double* R,
                                                        double* X, double* U) {
  __shared__ int inv[C::MMAX];
  __shared__ double Rs[C::MMAX * KCL];
  const SnView v(P, list[blockIdx.x]);
  const int N = v.N, J = v.J;
  double* Us = U + P.arena[v.s];
  RegFront<C> M;
  M.zero();
  for (int k0 = 0; k0 < N; k0 += KCL) {
    stage_columns<C>(N, k0, Rs, [&](int i, int k) {
      const bool ok = i >= k && i < J;
      const double x = R[ok ? v.at(i, k) : 0];
      return ok ? x : 0.0;
    });
    __syncthreads();
    const int kc = min(KCL, N - k0);
    for (int t = 0; t < kc; ++t) M.rank1(Rs + t * C::MMAX);
    __syncthreads();
  }
  gather_children(M, P, v, U, inv, -1.0);
  store_front(M, v, [&](int64_t o, double x) { X[o] = x; }, [&](int64_t e, double x) { Us[e] = -x; });
}

// Panel addressing of SnView with the column offsets staged in LDS, so an
// operand fetch needs no dependent global load.
struct LdsPanel {
  const int64_t* colc;
  int N;
  __device__ __forceinline__ int64_t at(int r, int c) const { return colc[c] + (r - c); }
  __device__ __forceinline__ int64_t nn(int i, int j) const { return i >= j ? at(i, j) : at(j, i); }
  __device__ __forceinline__ int64_t an(int x, int c) const { return colc[c] + (N + x - c); }
};

// Chunk width of the staged operands of reg_gemm.
constexpr int KG = 8;

// M(i, j) += sum_{x < K} fa(i, x) fb(x, j) for i < nr, j < nc.  fa and fb
// return zero outside the wanted block, so the FMAs run over the whole
// register block: branches around register blocks outside nr x nc cost
// more than the FMAs they save.  Operands are staged through LDS KG columns of fa and KG rows of
// fb at a time (As, Bs: 2 MMAX KG doubles each, double-buffered), with the
// next chunk's global loads in flight during the current chunk's FMAs; one
// barrier per chunk.  Ends with a barrier.
template <class C, bool LO, class FA, class FB>
__device__ __forceinline__ void reg_gemm(RegFront<C, LO>& M, int K, int nr, int nc, double* As, double* Bs,
                                         const FA& fa, const FB& fb) {
  constexpr int CH = C::MMAX * KG;
  constexpr int PER = (CH + C::NTH - 1) / C::NTH;
  const int nch = (K + KG - 1) / KG;
  if (nch == 0) return;
  double ra[PER], rb[PER];
  auto fetch = [&](int x0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * C::NTH;
      const int i = e % C::MMAX, x = x0 + e / C::MMAX;
      const bool ok = e < CH && x < K;
      ra[q] = ok ? fa(i, x) : 0.0;
      rb[q] = ok ? fb(x, i) : 0.0;
    }
  };
  auto put = [&](int h) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * C::NTH;
      if (e < CH) {
        As[h * CH + e] = ra[q];
        Bs[h * CH + e] = rb[q];
      }
    }
  };
  fetch(0);
  put(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) fetch((c + 1) * KG);
    const double* as = As + (c & 1) * CH;
    const double* bs = Bs + (c & 1) * CH;
#pragma unroll 4
    for (int t = 0; t < KG; ++t) {
      double ai[C::RX], bj[C::RY];
#pragma unroll
      for (int a = 0; a < C::RX; ++a) ai[a] = as[M.row(a) + t * C::MMAX];
#pragma unroll
      for (int b = 0; b < C::RY; ++b) bj[b] = bs[M.col(b) + t * C::MMAX];
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
#pragma unroll
        for (int b = 0; b < C::RY; ++b)
          if (!M.skip(a, b)) M.v[a][b] = fma(ai[a], bj[b], M.v[a][b]);
      // one k-step's operands live at a time (the other wavefronts of the
      // SIMD hide the LDS latency)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (c + 1 < nch) put((c + 1) & 1);
    __syncthreads();
  }
}

// Algorithm 7.2 on a register front (root-to-leaf): V_s gathered from the
// parent (and cached), then S_AN = -V_s L_AN and S_NN = D^-1 - S_AN^T L_AN
// as two register GEMMs over A.
template <class C>
__global__ void __launch_bounds__(C::NTH) k_projinv_reg(DevPlan P, const int32_t* list, const double* LB,
                                                        double* S, double* Vs) {
  __shared__ double As[2 * C::MMAX * KG], Bs[2 * C::MMAX * KG];
  __shared__ int64_t colc[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  const int N = v.N, A = v.A, J = v.J;
  stage_col<C>(v, colc);
  __syncthreads();
  const LdsPanel pn{colc, N};
  const double* V = Vs + P.arena[v.s];
  RegFront<C> M;
  M.zero();
  gather_parent(M, P, v, S, Vs);
  store_front(M, v, [](int64_t, double) {}, [&](int64_t e, double y) { Vs[P.arena[v.s] + e] = y; });
  __syncthreads();
  M.zero();
  reg_gemm(
      M, A, J, N, As, Bs,
      [&](int i, int x) { return i >= N && i < J ? sym_packed(V, i - N, x, A) : 0.0; },
      [&](int x, int j) { return j < N ? LB[pn.an(x, j)] : 0.0; });
  store_front(M, v, [&](int64_t o, double y) { S[o] = -y; }, [](int64_t, double) {});
  __syncthreads();
  M.zero();
  reg_gemm(
      M, A, N, N, As, Bs, [&](int i, int x) { return i < N ? LB[pn.an(x, i)] : 0.0; },
      [&](int x, int j) { return j < N ? S[pn.an(x, j)] : 0.0; });
  M.store_lower(
      N, [](int, int) { return true; },
      [&](int, int, int i, int j, double y) { S[pn.at(i, j)] = LB[pn.at(i, j)] - y; });
}

// Hessian steps 2 and 3 (root-to-leaf) on a register front: with
// Z = [K_NN; K_AN] D^-1, [M_NN; M_AN] = blkdiag(D^-1, V_s) Z, then
// T_AN = M_AN - V' L and T_NN = M_NN - M_AN^T L - L^T T_AN, where
// V'_s = T_{A_s A_s} is gathered from the parent (and cached for the
// children).  Four register GEMMs; Z and M_AN pass through the
// workgroup's scratch (J N + A N doubles).
template <class C>
__global__ void __launch_bounds__(C::NTH) k_hess_down_reg(DevPlan P, const int32_t* list, const double* LB,
                                                          const double* Vs, const double* Kt, double* T,
                                                          double* Va, int64_t upd, double* wsb,
                                                          int64_t slot) {
  __shared__ double As[2 * C::MMAX * KG], Bs[2 * C::MMAX * KG];
  __shared__ int64_t colc[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  stage_col<C>(v, colc);
  __syncthreads();
  const LdsPanel pn{colc, v.N};
  const int64_t r = blockIdx.y;
  const double* K = Kt + r * P.nnz;
  double* t = T + r * P.nnz;
  double* va = Va + r * upd;
  const int N = v.N, A = v.A, J = v.J;
  double* Z = slot_ptr(wsb, slot);      // J x N
  double* MA = Z + (int64_t)J * N;      // A x N
  const double* V = Vs + P.arena[v.s];
  const double* Vp = va + P.arena[v.s];
  auto Dinv = [&](int i, int j) { return LB[pn.nn(i, j)]; };
  {
    RegFront<C> G;
    G.zero();
    gather_parent(G, P, v, t, va);
    store_front(G, v, [](int64_t, double) {}, [&](int64_t e, double y) { va[P.arena[v.s] + e] = y; });
  }
  RegFront<C, false> M;  // general J x N products (Z is not symmetric)
  M.zero();
  reg_gemm(
      M, N, J, N, As, Bs,
      [&](int i, int x) { return i < J ? (i >= N ? K[pn.an(i - N, x)] : K[pn.nn(i, x)]) : 0.0; },
      [&](int x, int j) { return j < N ? Dinv(x, j) : 0.0; });
  M.store_all(
      J, [&](int, int j) { return j < N; }, [&](int, int, int i, int j, double y) { Z[i + (int64_t)j * J] = y; });
  __syncthreads();
  M.zero();
  reg_gemm(
      M, J, J, N, As, Bs,
      [&](int i, int x) {
        if (i < N && x < N) return Dinv(i, x);
        if (i >= N && i < J && x >= N) return sym_packed(V, i - N, x - N, A);
        return 0.0;
      },
      [&](int x, int j) { return j < N ? Z[x + (int64_t)j * J] : 0.0; });
  M.store_lower(
      J, [&](int i, int j) { return j < N && i >= N; },
      [&](int, int, int i, int j, double y) { MA[(i - N) + (int64_t)j * A] = y; });
  reg_gemm(
      M, A, J, N, As, Bs, [&](int i, int x) { return i >= N && i < J ? -sym_packed(Vp, i - N, x, A) : 0.0; },
      [&](int x, int j) { return j < N ? LB[pn.an(x, j)] : 0.0; });
  M.store_lower(
      J, [&](int i, int j) { return j < N && i >= N; },
      [&](int, int, int i, int j, double y) { t[pn.at(i, j)] = y; });
  __syncthreads();
  reg_gemm(
      M, 2 * A, N, N, As, Bs,
      [&](int i, int x) {
        if (i >= N) return 0.0;
        return x < A ? -MA[x + (int64_t)i * A] : -LB[pn.an(x - A, i)];
      },
      [&](int x, int j) {
        if (j >= N) return 0.0;
        return x < A ? LB[pn.an(x, j)] : t[pn.an(x - A, j)];
      });
  M.store_lower(
      N, [](int, int) { return true; }, [&](int, int, int i, int j, double y) { t[pn.at(i, j)] = y; });
}

// Inverse Hessian steps 1 and 2 on a register front (no dependence on
// other fronts once V'_s = T_{A_s A_s} is in the arena);
// M_AN = T_AN + V' L, M_NN = T_NN + L^T M_AN + T_AN^T L; with D = C C^T,
// [W; Z] = [M_NN; M_AN] D and [K_NN; K_AN] = blkdiag(D, V_s^-1) [W; Z].
// Five register GEMMs; D, M_NN, M_AN and [W; Z] pass through the
// workgroup's scratch (3 N^2 + 2 A N doubles).
template <class C>
__global__ void __launch_bounds__(C::NTH) k_ihess_down_reg(DevPlan P, const int32_t* list, const double* R,
                                                           const double* LB, const double* Vi,
                                                           const double* T, double* Kt, double* Va,
                                                           int64_t upd, double* wsb, int64_t slot) {
  __shared__ double As[2 * C::MMAX * KG], Bs[2 * C::MMAX * KG];
  __shared__ int64_t colc[C::MMAX];
  const SnView v(P, list[blockIdx.x]);
  stage_col<C>(v, colc);
  __syncthreads();
  const LdsPanel pn{colc, v.N};
  const int64_t r = blockIdx.y;
  const double* t = T + r * P.nnz;
  double* K = Kt + r * P.nnz;
  double* va = Va + r * upd;
  const int N = v.N, A = v.A, J = v.J;
  double* Dm = slot_ptr(wsb, slot);     // N x N
  double* MN = Dm + (int64_t)N * N;     // N x N
  double* MA = MN + (int64_t)N * N;     // A x N
  double* WZ = MA + (int64_t)A * N;     // J x N
  const double* Vp = va + P.arena[v.s];
  const double* VI = Vi + P.arena[v.s];
  // V'_s = T_{A_s A_s} is in the arena (gathered beforehand)
  RegFront<C, false> M;  // general J x N products ([W; Z] is not symmetric)
  // D = C C^T
  M.zero();
  reg_gemm(
      M, N, N, N, As, Bs, [&](int i, int x) { return i < N && x <= i ? R[pn.at(i, x)] : 0.0; },
      [&](int x, int j) { return j < N && x <= j ? R[pn.at(j, x)] : 0.0; });
  M.store_lower(
      N, [](int, int) { return true; },
      [&](int, int, int i, int j, double y) {
        Dm[i + (int64_t)j * N] = y;
        Dm[j + (int64_t)i * N] = y;
      });
  // M_AN = T_AN + V' L
  M.zero();
  load_panel(M, v, t);
  reg_gemm(
      M, A, J, N, As, Bs, [&](int i, int x) { return i >= N && i < J ? sym_packed(Vp, i - N, x, A) : 0.0; },
      [&](int x, int j) { return j < N ? LB[pn.an(x, j)] : 0.0; });
  M.store_lower(
      J, [&](int i, int j) { return j < N && i >= N; },
      [&](int, int, int i, int j, double y) { MA[(i - N) + (int64_t)j * A] = y; });
  __syncthreads();
  // M_NN = T_NN + L^T M_AN + T_AN^T L (rows < N of the registers still hold T_NN)
  reg_gemm(
      M, 2 * A, N, N, As, Bs,
      [&](int i, int x) {
        if (i >= N) return 0.0;
        return x < A ? LB[pn.an(x, i)] : t[pn.an(x - A, i)];
      },
      [&](int x, int j) {
        if (j >= N) return 0.0;
        return x < A ? MA[x + (int64_t)j * A] : LB[pn.an(x - A, j)];
      });
  M.store_lower(
      N, [](int, int) { return true; },
      [&](int, int, int i, int j, double y) {
        MN[i + (int64_t)j * N] = y;
        MN[j + (int64_t)i * N] = y;
      });
  __syncthreads();
  // [W; Z] = [M_NN; M_AN] D
  M.zero();
  reg_gemm(
      M, N, J, N, As, Bs,
      [&](int i, int x) {
        if (i >= J) return 0.0;
        return i < N ? MN[i + (int64_t)x * N] : MA[(i - N) + (int64_t)x * A];
      },
      [&](int x, int j) { return j < N ? Dm[x + (int64_t)j * N] : 0.0; });
  M.store_all(
      J, [&](int, int j) { return j < N; }, [&](int, int, int i, int j, double y) { WZ[i + (int64_t)j * J] = y; });
  __syncthreads();
  // [K_NN; K_AN] = blkdiag(D, V^-1) [W; Z]
  M.zero();
  reg_gemm(
      M, J, J, N, As, Bs,
      [&](int i, int x) {
        if (i < N && x < N) return Dm[i + (int64_t)x * N];
        if (i >= N && i < J && x >= N) return sym_packed(VI, i - N, x - N, A);
        return 0.0;
      },
      [&](int x, int j) { return j < N ? WZ[x + (int64_t)j * J] : 0.0; });
  store_front(M, v, [&](int64_t o, double y) { K[o] = y; }, [](int64_t, double) {});
}

// Workgroup shapes of the register classes (front order <= MMAX).
using RegC0 = RegCfg<16, 16, 1, 1>;
using RegC1 = RegCfg<16, 16, 2, 2>;
using RegC2 = RegCfg<16, 16, 4, 4>;
using RegC3 = RegCfg<16, 32, 8, 4>;
using RegC4 = RegCfg<16, 32, 12, 6>;
static_assert(RegC0::MMAX == kRegMax[0] && RegC1::MMAX == kRegMax[1] && RegC2::MMAX == kRegMax[2] &&
                  RegC3::MMAX == kRegMax[3] && RegC4::MMAX == kRegMax[4] && kRegClasses == 5,
              "register classes shared with the host");

template <class C>
static void go_vinv(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* Vs,
                    double* Vi, DevStatus* st) {
  k_vinv_reg<C><<<g, C::NTH, 0, s>>>(P, list, Vs, Vi, st);
}
template <class C>
static void go_factor(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* x,
                      double* R, double* LB, double* U, double* part, DevStatus* st) {
  k_factor_reg<C><<<g, C::NTH, 0, s>>>(P, list, x, R, LB, U, part, st);
}
template <class C>
static void go_completion(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                          const double* Sin, double* R, double* LB, double* S, double* Vs, double* Vi,
                          double* part, DevStatus* st) {
  k_completion_reg<C><<<g, C::NTH, 0, s>>>(P, list, Sin, R, LB, S, Vs, Vi, part, st);
}
template <class C>
static void go_hess_up(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* LB,
                       const double* Y, double* Kt, double* Ua, int64_t upd, int32_t* act) {
  k_hess_up_reg<C><<<g, C::NTH, 0, s>>>(P, list, LB, Y, Kt, Ua, upd, act);
}
template <class C>
static void go_ihess_up(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* LB,
                        const double* Kt, double* Y, double* Ua, int64_t upd) {
  k_ihess_up_reg<C><<<g, C::NTH, 0, s>>>(P, list, LB, Kt, Y, Ua, upd);
}
template <class C>
static void go_product(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                       double* X, double* U) {
  k_product_reg<C><<<g, C::NTH, 0, s>>>(P, list, R, X, U);
}

template <class C>
static void go_projinv(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* LB,
                       double* S, double* Vs) {
  k_projinv_reg<C><<<g, C::NTH, 0, s>>>(P, list, LB, S, Vs);
}
template <class C>
static void go_hess_down(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* LB,
                         const double* Vs, const double* Kt, double* T, double* Va, int64_t upd,
                         double* wsb, int64_t slot) {
  k_hess_down_reg<C><<<g, C::NTH, 0, s>>>(P, list, LB, Vs, Kt, T, Va, upd, wsb, slot);
}
template <class C>
static void go_ihess_down(dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                          const double* LB, const double* Vi, const double* T, double* Kt, double* Va,
                          int64_t upd, double* wsb, int64_t slot) {
  k_ihess_down_reg<C><<<g, C::NTH, 0, s>>>(P, list, R, LB, Vi, T, Kt, Va, upd, wsb, slot);
}

#define MFB_REG_SWITCH(fn, ...)                  \
  switch (cls) {                                 \
    case 0: fn<RegC0>(__VA_ARGS__); break;       \
    case 1: fn<RegC1>(__VA_ARGS__); break;       \
    case 2: fn<RegC2>(__VA_ARGS__); break;       \
    case 3: fn<RegC3>(__VA_ARGS__); break;       \
    default: fn<RegC4>(__VA_ARGS__); break;      \
  }

void launch_vinv_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                     const double* Vs, double* Vi, DevStatus* st) {
  MFB_REG_SWITCH(go_vinv, g, s, P, list, Vs, Vi, st)
}
void launch_factor_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                       const double* x, double* R, double* LB, double* U, double* part, DevStatus* st) {
  MFB_REG_SWITCH(go_factor, g, s, P, list, x, R, LB, U, part, st)
}
void launch_completion_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* Sin, double* R, double* LB, double* S, double* Vs,
                           double* Vi, double* part, DevStatus* st) {
  MFB_REG_SWITCH(go_completion, g, s, P, list, Sin, R, LB, S, Vs, Vi, part, st)
}
// x[0 .. n) = v (kernel launch, not a memset: graph-capture safe)
__global__ void __launch_bounds__(NT) k_fill_i32(int32_t* x, int64_t n, int32_t v) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) x[e] = v;
}
void launch_fill_i32(hipStream_t s, int32_t* x, int64_t n, int32_t v) {
  if (n <= 0) return;
  const int64_t b = std::min<int64_t>(1024, (n + NT - 1) / NT);
  k_fill_i32<<<dim3(unsigned(b)), NT, 0, s>>>(x, n, v);
}

void launch_hess_up_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* LB, const double* Y, double* Kt, double* Ua, int64_t upd, int32_t* act) {
  MFB_REG_SWITCH(go_hess_up, g, s, P, list, LB, Y, Kt, Ua, upd, act)
}
void launch_ihess_up_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                         const double* LB, const double* Kt, double* Y, double* Ua, int64_t upd) {
  MFB_REG_SWITCH(go_ihess_up, g, s, P, list, LB, Kt, Y, Ua, upd)
}
void launch_product_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* R, double* X, double* U) {
  MFB_REG_SWITCH(go_product, g, s, P, list, R, X, U)
}
void launch_projinv_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* LB, double* S, double* Vs) {
  MFB_REG_SWITCH(go_projinv, g, s, P, list, LB, S, Vs)
}
void launch_hess_down_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                          const double* LB, const double* Vs, const double* Kt, double* T, double* Va,
                          int64_t upd, double* wsb, int64_t slot) {
  MFB_REG_SWITCH(go_hess_down, g, s, P, list, LB, Vs, Kt, T, Va, upd, wsb, slot)
}
void launch_ihess_down_reg(int cls, dim3 g, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* R, const double* LB, const double* Vi, const double* T,
                           double* Kt, double* Va, int64_t upd, double* wsb, int64_t slot) {
  MFB_REG_SWITCH(go_ihess_down, g, s, P, list, R, LB, Vi, T, Kt, Va, upd, wsb, slot)
}
#undef MFB_REG_SWITCH

}  // namespace mfb

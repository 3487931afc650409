// Register-resident symmetric fronts for gfx950.
//
// A workgroup of GX * GY threads holds an m x m symmetric matrix (m <= MMAX)
// entirely in registers: thread (tx, ty) = (t % GX, t / GX) owns the RX x RY
// entries (tx + GX a, ty + GY b).  Both triangles are kept, so every
// elimination step is one rank-1 update of the whole register block after a
// single LDS broadcast of the pivot column, with one workgroup barrier per
// step.  No step touches global memory: the front is read once and its
// results written once.
//
// Two eliminations are provided:
//  * sweep (the symmetric Gauss-Jordan "sweep operator"): sweeping pivot k
//    of M maps M_kk -> -1/M_kk, M_ik -> M_ik / M_kk, M_kj -> M_kj / M_kk and
//    M_ij -> M_ij - M_ik M_kj / M_kk.  Sweeping a set K of pivots of
//    [M_KK M_KR; M_RK M_RR] leaves [-M_KK^-1, M_KK^-1 M_KR; M_RK M_KK^-1,
//    M_RR - M_RK M_KK^-1 M_KR], so sweeping every pivot gives -M^-1.  The
//    pivots are the successive Schur-complement diagonals, all positive
//    exactly when the swept block is positive definite.
//  * right-looking Cholesky on the leading columns: step k divides column k
//    by sqrt(M_kk) and subtracts the outer product of that column from the
//    trailing columns j < ncols (all rows).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfb {

template <int GX_, int GY_, int RX_, int RY_>
struct RegCfg {
  static constexpr int GX = GX_, GY = GY_, RX = RX_, RY = RY_;
  static constexpr int NTH = GX * GY;
  static constexpr int MMAX = GX * RX;
  static_assert(GX * RX == GY * RY, "square register front");
  static_assert(NTH % 64 == 0, "whole wavefronts");
};

template <class C>
struct RegFront {
  double v[C::RX][C::RY];
  int tx, ty;
  int phase;  // which half of the broadcast buffer the next step uses

  __device__ __forceinline__ RegFront() : tx(threadIdx.x % C::GX), ty(threadIdx.x / C::GX), phase(0) {}
  __device__ __forceinline__ int row(int a) const { return tx + C::GX * a; }
  __device__ __forceinline__ int col(int b) const { return ty + C::GY * b; }

  // v(i, j) = f(i, j) for i, j < m, else 0.
  template <class F>
  __device__ __forceinline__ void load(int m, const F& f) {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) {
        const int i = row(a), j = col(b);
        v[a][b] = (i < m && j < m) ? f(i, j) : 0.0;
      }
  }
  // out(i, j, v(i, j)) for every owned entry with pred(i, j) true.
  template <class PR, class OUT>
  __device__ __forceinline__ void store(int m, const PR& pred, const OUT& out) const {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) {
        const int i = row(a), j = col(b);
        if (C::GX * a < m && C::GY * b < m && i < m && j < m && pred(i, j)) out(i, j, v[a][b]);
      }
  }
  // As store(), with the register coordinates passed on: out(a, b, i, j, value).
  template <class PR, class OUT>
  __device__ __forceinline__ void store_ab(int m, const PR& pred, const OUT& out) const {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) {
        const int i = row(a), j = col(b);
        if (C::GX * a < m && C::GY * b < m && i < m && j < m && pred(i, j)) out(a, b, i, j, v[a][b]);
      }
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) v[a][b] = 0.0;
  }

  // Writes column k to buf (all MMAX rows; rows >= m hold zeros or values
  // that never reach an entry inside the front).  Called by every thread:
  // the register index is selected by uniform branches, the owning lanes
  // by a divergent one inside.
  __device__ __forceinline__ void put_column(int k, double* buf) const {
    const int kb = k / C::GY;
#pragma unroll
    for (int b = 0; b < C::RY; ++b)
      if (b == kb) {
        if (ty == k % C::GY) {
#pragma unroll
          for (int a = 0; a < C::RX; ++a) buf[row(a)] = v[a][b];
        }
      }
  }

  // Half of the broadcast buffer for the next step: consecutive steps (of
  // either kind) alternate, so one barrier per step suffices.
  __device__ __forceinline__ double* next_half(double* buf) {
    double* h = buf + phase * C::MMAX;
    phase ^= 1;
    return h;
  }

  // Entries outside the m x m front are zero and stay zero: every step
  // below reads the broadcast column without bounds checks, relying on the
  // zero rows that put_column() copies out of those registers.

  // One sweep of pivot k (0 <= k < m); `buf` is LDS of 2 * MMAX doubles.
  // Returns true if the pivot is not positive (it is then replaced by one
  // so the arithmetic stays finite).  The rank-1 update runs over the whole
  // register block, and the pivot row and column are rewritten afterwards
  // by their owners.
  __device__ __forceinline__ bool sweep(int k, double* buf) {
    double* bk = next_half(buf);
    put_column(k, bk);
    __syncthreads();
    double p = bk[k];
    const bool bad = !(p > 0.0);
    if (bad) p = 1.0;
    const double r = 1.0 / p;
    double ci[C::RX], cj[C::RY];
#pragma unroll
    for (int a = 0; a < C::RX; ++a) ci[a] = bk[row(a)];
#pragma unroll
    for (int b = 0; b < C::RY; ++b) cj[b] = bk[col(b)] * r;
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) v[a][b] = fma(-ci[a], cj[b], v[a][b]);
    // row k: M_kj / M_kk; column k: M_ik / M_kk; pivot: -1 / M_kk
    const int ka = k / C::GX, kb = k / C::GY;
    const bool own_r = tx == k % C::GX, own_c = ty == k % C::GY;
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
      if (a == ka) {
        if (own_r) {
#pragma unroll
          for (int b = 0; b < C::RY; ++b) v[a][b] = cj[b];
        }
      }
#pragma unroll
    for (int b = 0; b < C::RY; ++b)
      if (b == kb) {
        if (own_c) {
#pragma unroll
          for (int a = 0; a < C::RX; ++a) v[a][b] = ci[a] * r;
        }
#pragma unroll
        for (int a = 0; a < C::RX; ++a)
          if (a == ka) {
            if (own_r && own_c) v[a][b] = -r;
          }
      }
    return bad;
  }

  // One right-looking Cholesky step on column k < ncols: on return column
  // k holds sqrt(M_kk) at row k and M_ik / sqrt(M_kk) below, and the
  // columns k < j < ncols are updated.  `buf` is LDS of 4 * MMAX doubles:
  // the column goes to one half and, cut at row ncols, to the other (the
  // multipliers of the columns), so columns from ncols on are untouched.
  // Same failure convention as sweep(); entries above the diagonal are
  // left stale.
  __device__ __forceinline__ bool chol(int k, int ncols, double* buf, double* diag) {
    double* bk = next_half(buf);
    double* bc = bk + 2 * C::MMAX;
    const int kb = k / C::GY;
#pragma unroll
    for (int b = 0; b < C::RY; ++b)
      if (b == kb) {
        if (ty == k % C::GY) {
#pragma unroll
          for (int a = 0; a < C::RX; ++a) {
            bk[row(a)] = v[a][b];
            bc[row(a)] = row(a) < ncols ? v[a][b] : 0.0;
          }
        }
      }
    __syncthreads();
    const double p = bk[k];
    const bool bad = !(p > 0.0);
    const double d = bad ? 1.0 : sqrt(p);
    const double r = 1.0 / d;
    *diag = d;
    double li[C::RX], lj[C::RY];
#pragma unroll
    for (int a = 0; a < C::RX; ++a) li[a] = row(a) > k ? bk[row(a)] * r : 0.0;
#pragma unroll
    for (int b = 0; b < C::RY; ++b) lj[b] = col(b) > k ? bc[col(b)] * r : 0.0;
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) v[a][b] = fma(-li[a], lj[b], v[a][b]);
#pragma unroll
    for (int b = 0; b < C::RY; ++b)
      if (b == kb) {
        if (ty == k % C::GY) {
#pragma unroll
          for (int a = 0; a < C::RX; ++a) {
            const int i = row(a);
            v[a][b] = i > k ? li[a] : (i == k ? d : v[a][b]);
          }
        }
      }
    return bad;
  }

  // Congruence with the elementary matrix I + sg l e_k^T (sg = +-1), where
  // l vanishes on the rows and columns of the pivots (k among them):
  // M <- (I + sg l e_k^T) M (I + sg e_k l^T)
  //    = M + l w^T + w l^T,  w = sg M e_k + (M_kk / 2) l.
  // Factors for different pivots commute (e_k^T l = 0), so applying them one
  // pivot at a time to the current M gives the product over all pivots.
  // `lcol` holds l for every row index below MMAX (LDS, zero where l is).
  __device__ __forceinline__ void congruence(int k, double sg, double* buf, const double* lcol) {
    double* bk = next_half(buf);
    put_column(k, bk);
    __syncthreads();
    const double h = 0.5 * bk[k];
    // two rank-1 passes, so only one pair of vectors is live at a time
    {
      double li[C::RX], wj[C::RY];
#pragma unroll
      for (int a = 0; a < C::RX; ++a) li[a] = lcol[row(a)];
#pragma unroll
      for (int b = 0; b < C::RY; ++b) wj[b] = fma(h, lcol[col(b)], sg * bk[col(b)]);
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
#pragma unroll
        for (int b = 0; b < C::RY; ++b) v[a][b] = fma(li[a], wj[b], v[a][b]);
    }
    {
      double wi[C::RX], lj[C::RY];
#pragma unroll
      for (int a = 0; a < C::RX; ++a) wi[a] = fma(h, lcol[row(a)], sg * bk[row(a)]);
#pragma unroll
      for (int b = 0; b < C::RY; ++b) lj[b] = lcol[col(b)];
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
#pragma unroll
        for (int b = 0; b < C::RY; ++b) v[a][b] = fma(wi[a], lj[b], v[a][b]);
    }
  }

  // Negates the entries in columns j < ncols.
  __device__ __forceinline__ void negate_columns(int ncols) {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b)
        if (col(b) < ncols) v[a][b] = -v[a][b];
  }
};

// Deterministic sum over the NTH threads of a workgroup (sm: NTH doubles).
template <int NTH>
__device__ __forceinline__ double block_sum(double x, double* sm) {
  sm[threadIdx.x] = x;
  __syncthreads();
#pragma unroll
  for (int s = NTH / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

}  // namespace mfb

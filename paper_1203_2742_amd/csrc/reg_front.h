// Register-resident symmetric fronts for gfx950.
//
// A workgroup of GX * GY threads holds an m x m symmetric matrix (m <= MMAX)
// in registers: thread (tx, ty) = (t % GX, t / GX) owns the RX x RY entries
// (tx + GX a, ty + GY b).  Register blocks (a, b) lying wholly above the
// diagonal (every row index of the block below every column index) are
// never computed; all other blocks hold correct values, so the lower
// triangle and the diagonal are always exact.  Every elimination step is
// one rank-1 or rank-2 update of the register block after a single LDS
// broadcast of the pivot column, with one workgroup barrier per step.  No
// step touches global memory: the front is read once and its results
// written once.
//
// Eliminations:
//  * sweep (the symmetric Gauss-Jordan "sweep operator"): sweeping pivot k
//    of M maps M_kk -> -1/M_kk, M_ik -> M_ik / M_kk, M_kj -> M_kj / M_kk and
//    M_ij -> M_ij - M_ik M_kj / M_kk.  Sweeping a set K of pivots of
//    [M_KK M_KR; M_RK M_RR] leaves [-M_KK^-1, M_KK^-1 M_KR; M_RK M_KK^-1,
//    M_RR - M_RK M_KK^-1 M_KR], so sweeping every pivot gives -M^-1.  Just
//    before pivot k is swept (pivots swept in increasing order), column k
//    restricted to the rows >= k is the first column of the Schur
//    complement, i.e. d_k [1; l_k] of the scalar L D L^T factorization, so
//    the broadcast column also yields column k of the Cholesky factor.
//  * congruence with I + sg l e_k^T for a vector l that vanishes on the
//    pivot rows (the block L D L^T transforms of the Hessian sweeps).
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
  static_assert(NTH >= MMAX, "one thread per row of a broadcast column");
  // register block (a, b) lies wholly above the diagonal
  static constexpr bool upper(int a, int b) { return GX * a + GX - 1 < GY * b; }
};

// 1 / p for p > 0: the hardware reciprocal refined by two Newton steps
// (each squares the relative error), short enough to sit on the
// per-step critical path.
__device__ __forceinline__ double fast_rcp(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  r = fma(r, fma(-p, r, 1.0), r);
  return r;
}

// 1 / sqrt(p) for p > 0: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double fast_rsqrt(double p) {
  double y = __builtin_amdgcn_rsq(p);
  const double h = 0.5 * p;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

template <int V>
struct ic {
  static constexpr int value = V;
};

// LO: keep only the register blocks not wholly above the diagonal (a
// symmetric front); otherwise every block (a general m x m tile).
template <class C, bool LO = true>
struct RegFront {
  // register block (a, b) is not stored
  static constexpr bool skip(int a, int b) { return LO && C::upper(a, b); }
  double v[C::RX][C::RY];
  int tx, ty;
  int phase;  // which half of the broadcast buffer the next step uses

  __device__ __forceinline__ RegFront() : tx(threadIdx.x % C::GX), ty(threadIdx.x / C::GX), phase(0) {}
  __device__ __forceinline__ int row(int a) const { return tx + C::GX * a; }
  __device__ __forceinline__ int col(int b) const { return ty + C::GY * b; }

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) v[a][b] = 0.0;
  }
  // out(a, b, i, j, v(i, j)) for every owned lower entry (i >= j) of the
  // m x m front with pred(i, j) true.
  template <class PR, class OUT>
  __device__ __forceinline__ void store_lower(int m, const PR& pred, const OUT& out) const {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) {
        if (skip(a, b)) continue;
        const int i = row(a), j = col(b);
        if (C::GX * a < m && C::GY * b < m && i < m && i >= j && pred(i, j)) out(a, b, i, j, v[a][b]);
      }
  }

  // out(a, b, i, j, v(i, j)) for every stored entry of the m x m tile with
  // pred(i, j) true.
  template <class PR, class OUT>
  __device__ __forceinline__ void store_all(int m, const PR& pred, const OUT& out) const {
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b) {
        if (skip(a, b)) continue;
        const int i = row(a), j = col(b);
        if (C::GX * a < m && C::GY * b < m && i < m && j < m && pred(i, j)) out(a, b, i, j, v[a][b]);
      }
  }

  // Broadcast buffer for the next step (2 MMAX doubles out of `buf`, which
  // holds 4 MMAX): consecutive steps (of either kind) alternate halves, so
  // one barrier per step suffices.
  __device__ __forceinline__ double* next_half(double* buf) {
    double* h = buf + phase * 2 * C::MMAX;
    phase ^= 1;
    return h;
  }

  // Entries outside the m x m front are zero and stay zero: every step
  // below reads the broadcast column without bounds checks, relying on the
  // zero rows that the broadcast copies out of those registers.
  //
  // Steps are instantiated per register row block KA of the pivot
  // (k in [GX KA, GX KA + GX)), so the pivot's row block KA and column
  // block KB = GX KA / GY are compile-time constants and no step selects a
  // register by a runtime index.

  // Broadcast of column k of the symmetric matrix: the owners of column k
  // write their rows to bk[0 .. MMAX), the owners of row k their columns to
  // bk[MMAX .. 2 MMAX).  Entry i of column k is then bk[i] for i >= k (a
  // lower entry of column k) and bk[MMAX + i] for i < k (a lower entry of
  // row k); in(...) picks the part, which is known at compile time except
  // in the pivot's own block.
  template <int KA>
  __device__ __forceinline__ void put_column(int k, double* bk) const {
    constexpr int KB = (C::GX * KA) / C::GY;
    if (ty == k - C::GY * KB) {
#pragma unroll
      for (int a = 0; a < C::RX; ++a) bk[row(a)] = skip(a, KB) ? 0.0 : v[a][KB];
    }
    if (tx == k - C::GX * KA) {
#pragma unroll
      for (int b = 0; b < C::RY; ++b) bk[C::MMAX + col(b)] = skip(KA, b) ? 0.0 : v[KA][b];
    }
  }
  template <int KA>
  __device__ __forceinline__ double in_row(const double* bk, int a, int k) const {
    if (a < KA) return bk[C::MMAX + row(a)];
    if (a > KA) return bk[row(a)];
    return bk[row(a) < k ? C::MMAX + row(a) : row(a)];
  }
  template <int KA>
  __device__ __forceinline__ double in_col(const double* bk, int b, int k) const {
    constexpr int KB = (C::GX * KA) / C::GY;
    if (b < KB) return bk[C::MMAX + col(b)];
    if (b > KB) return bk[col(b)];
    return bk[col(b) < k ? C::MMAX + col(b) : col(b)];
  }

  // One sweep of pivot k (in row block KA).  After the barrier,
  // ext(column, pivot, k) sees the broadcast column (before this step's
  // update; entries i >= k at column[i]).  Returns true if the pivot is not
  // positive (it is then replaced by one so the arithmetic stays finite).
  // The rank-1 update runs over the whole register block, and the pivot
  // row and column are rewritten afterwards by their owners.
  template <int KA, class EX>
  __device__ __forceinline__ bool sweep_step(int k, double* buf, const EX& ext) {
    constexpr int KB = (C::GX * KA) / C::GY;
    double* bk = next_half(buf);
    put_column<KA>(k, bk);
    __syncthreads();
    double p = bk[k];
    const bool bad = !(p > 0.0);
    if (bad) p = 1.0;
    ext(static_cast<const double*>(bk), p, k);
    const double r = fast_rcp(p);
    double ci[C::RX], cj[C::RY];
#pragma unroll
    for (int a = 0; a < C::RX; ++a) ci[a] = in_row<KA>(bk, a, k);
#pragma unroll
    for (int b = 0; b < C::RY; ++b) cj[b] = in_col<KA>(bk, b, k) * r;
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b)
        if (!skip(a, b)) v[a][b] = fma(-ci[a], cj[b], v[a][b]);
    // row k: M_kj / M_kk; column k: M_ik / M_kk; pivot: -1 / M_kk
    const bool own_r = tx == k - C::GX * KA, own_c = ty == k - C::GY * KB;
    if (own_r) {
#pragma unroll
      for (int b = 0; b < C::RY; ++b) v[KA][b] = cj[b];
    }
    if (own_c) {
#pragma unroll
      for (int a = 0; a < C::RX; ++a) v[a][KB] = ci[a] * r;
    }
    if (own_r && own_c) v[KA][KB] = -r;
    return bad;
  }

  // Sweeps the pivots kbeg .. kend-1 in increasing order, calling
  // ext(column, pivot, k) at each (see sweep_step).  Returns the first pivot
  // that was not positive, or -1.
  template <class EX>
  __device__ __forceinline__ int sweeps(int kbeg, int kend, double* buf, const EX& ext) {
    int fail = -1;
    blocks(kbeg, kend, [&](auto ka, int lo, int hi) {
      constexpr int KA = decltype(ka)::value;
      for (int k = lo; k < hi; ++k)
        if (sweep_step<KA>(k, buf, ext) && fail < 0) fail = k;
    });
    return fail;
  }
  __device__ __forceinline__ int sweeps(int kbeg, int kend, double* buf) {
    return sweeps(kbeg, kend, buf, [](const double*, double, int) {});
  }

  // Congruence with the elementary matrix I + sg l e_k^T (sg = +-1), where
  // l vanishes on the rows and columns of the pivots (k among them):
  // M <- (I + sg l e_k^T) M (I + sg e_k l^T)
  //    = M + l w^T + w l^T,  w = sg M e_k + (M_kk / 2) l.
  // Factors for different pivots commute (e_k^T l = 0), so applying them one
  // pivot at a time to the current M gives the product over all pivots.
  // `lcol` holds l for every row index below MMAX (LDS, zero where l is).
  template <int KA>
  __device__ __forceinline__ void congruence_step(int k, double sg, double* buf, const double* lcol) {
    double* bk = next_half(buf);
    put_column<KA>(k, bk);
    __syncthreads();
    const double h = 0.5 * bk[k];
    // two rank-1 passes, so only one pair of vectors is live at a time
    {
      double li[C::RX], wj[C::RY];
#pragma unroll
      for (int a = 0; a < C::RX; ++a) li[a] = lcol[row(a)];
#pragma unroll
      for (int b = 0; b < C::RY; ++b) wj[b] = fma(h, lcol[col(b)], sg * in_col<KA>(bk, b, k));
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
#pragma unroll
        for (int b = 0; b < C::RY; ++b)
          if (!skip(a, b)) v[a][b] = fma(li[a], wj[b], v[a][b]);
    }
    {
      double wi[C::RX], lj[C::RY];
#pragma unroll
      for (int a = 0; a < C::RX; ++a) wi[a] = fma(h, lcol[row(a)], sg * in_row<KA>(bk, a, k));
#pragma unroll
      for (int b = 0; b < C::RY; ++b) lj[b] = lcol[col(b)];
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
#pragma unroll
        for (int b = 0; b < C::RY; ++b)
          if (!skip(a, b)) v[a][b] = fma(wi[a], lj[b], v[a][b]);
    }
  }

  // Congruence steps for the pivots 0 .. n-1.  The vectors l come in LDS
  // chunks of KC pivots: stage(k0, ls) fills ls[i + t MMAX] = l_{k0+t}(i)
  // (every thread takes part; KC divides GX, so chunks never straddle a
  // register row block).
  template <int KC, class ST>
  __device__ __forceinline__ void congruences(int n, double sg, double* buf, double* ls, const ST& stage) {
    static_assert(C::GX % KC == 0, "chunks inside one row block");
    blocks(0, n, [&](auto ka, int lo, int hi) {
      constexpr int KA = decltype(ka)::value;
      for (int k0 = lo; k0 < hi; k0 += KC) {
        stage(k0, ls);
        __syncthreads();
        const int kc = min(KC, hi - k0);
        for (int t = 0; t < kc; ++t) congruence_step<KA>(k0 + t, sg, buf, ls + t * C::MMAX);
        __syncthreads();
      }
    });
  }

  // Columns k0 .. k0 + kc - 1 (all in row block KA) of the symmetric matrix
  // into cols[t MMAX + i], whole: entry i of column k is taken from (i, k)
  // by the owners of column k when i >= k and from (k, i) by the owners of
  // row k when i < k, both lower entries and hence exact.
  template <int KA>
  __device__ __forceinline__ void put_columns(int k0, int kc, double* cols) const {
    constexpr int KB = (C::GX * KA) / C::GY;
    const int tc = col(KB) - k0;
    if (tc >= 0 && tc < kc) {
#pragma unroll
      for (int a = 0; a < C::RX; ++a)
        if (!skip(a, KB) && row(a) >= col(KB)) cols[tc * C::MMAX + row(a)] = v[a][KB];
    }
    const int tr = row(KA) - k0;
    if (tr >= 0 && tr < kc) {
#pragma unroll
      for (int b = 0; b < C::RY; ++b)
        if (!skip(KA, b) && col(b) < row(KA)) cols[tr * C::MMAX + col(b)] = v[KA][b];
    }
  }

  // v += sgn sum_{t < kc} p_t q_t^T over the stored register blocks, with
  // p_t(i) = pp[t MMAX + i] and q_t(j) = qq[t MMAX + j] in LDS (rows below
  // MMAX; kc <= KC).  Step t + 1's operands are loaded while step t's FMAs
  // run, and no further (the scheduling barrier keeps the live operands to
  // two steps' worth).
  template <int KC>
  __device__ __forceinline__ void rank_updates(int kc, const double* pp, const double* qq, double sgn) {
    double p[2][C::RX], q[2][C::RY];
    auto load = [&](int t, double* pt, double* qt) {
#pragma unroll
      for (int a = 0; a < C::RX; ++a) pt[a] = pp[t * C::MMAX + row(a)];
#pragma unroll
      for (int b = 0; b < C::RY; ++b) qt[b] = sgn * qq[t * C::MMAX + col(b)];
    };
    load(0, p[0], q[0]);
#pragma unroll
    for (int t = 0; t < KC; ++t) {
      if (t + 1 < KC) load(t + 1, p[(t + 1) & 1], q[(t + 1) & 1]);
      if (t < kc) {
#pragma unroll
        for (int a = 0; a < C::RX; ++a)
#pragma unroll
          for (int b = 0; b < C::RY; ++b)
            if (!skip(a, b)) v[a][b] = fma(p[t & 1][a], q[t & 1][b], v[a][b]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // Congruence with the elementary matrices I + sg l_k e_k^T (sg = +-1) of
  // the kc <= KC pivots k = k0 .. k0 + kc - 1 of row block KA, where every
  // l_k vanishes on the pivot rows.  The factors commute (e_k^T l_j = 0), so
  // with L = [l_k] and E = [e_k] their product is I + sg L E^T and
  //   M <- (I + sg L E^T) M (I + sg E L^T) = M + L W^T + W L^T,
  //   W = sg M E + (1/2) L M_EE,
  // one rank-2kc update after a single broadcast of the kc columns M E:
  // two barriers for kc pivots.  ls[t MMAX + i] = l_{k0+t}(i) (LDS, every
  // row index below MMAX, written before the call); cols and W take KC MMAX
  // doubles each.
  template <int KA, int KC>
  __device__ __forceinline__ void congruence_block(int k0, int kc, double sg, double* cols, double* W,
                                                   const double* ls) {
    put_columns<KA>(k0, kc, cols);
    __syncthreads();
    if (threadIdx.x < C::MMAX) {
      const int r = threadIdx.x;
      double hl[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) hl[u] = u < kc ? 0.5 * ls[u * C::MMAX + r] : 0.0;
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        if (t < kc) {
          double w = sg * cols[t * C::MMAX + r];
#pragma unroll
          for (int u = 0; u < KC; ++u)
            if (u < kc) w = fma(hl[u], cols[t * C::MMAX + k0 + u], w);
          W[t * C::MMAX + r] = w;
        }
      }
    }
    __syncthreads();
    rank_updates<KC>(kc, ls, W, 1.0);
    rank_updates<KC>(kc, W, ls, 1.0);
  }

  // Half of a 6 KC MMAX double buffer for the next blocked step (halves
  // alternate with `phase`).
  template <int KC>
  __device__ __forceinline__ double* next_block_half(double* bufs) {
    double* h = bufs + phase * 3 * KC * C::MMAX;
    phase ^= 1;
    return h;
  }

  // Congruence blocks for the pivots 0 .. n-1, KC at a time (KC divides GX,
  // so a block never straddles a register row block).  stage(k0, ls) fills
  // ls[i + t MMAX] = l_{k0+t}(i) (every thread takes part).  `bufs` holds
  // 6 KC MMAX doubles: two halves of (cols, W, ls) used alternately, so a
  // block's writes never meet the previous block's reads.
  template <int KC, class ST>
  __device__ __forceinline__ void congruences_blocked(int n, double sg, double* bufs, const ST& stage) {
    static_assert(C::GX % KC == 0, "blocks inside one row block");
    blocks(0, n, [&](auto ka, int lo, int hi) {
      constexpr int KA = decltype(ka)::value;
      for (int k0 = lo; k0 < hi; k0 += KC) {
        double* h = next_block_half<KC>(bufs);
        stage(k0, h + 2 * KC * C::MMAX);
        congruence_block<KA, KC>(k0, min(KC, hi - k0), sg, h, h + KC * C::MMAX, h + 2 * KC * C::MMAX);
      }
    });
  }

  // f(ic<KA>, lo, hi) for every register row block KA meeting [kbeg, kend),
  // with [lo, hi) its part of the range, in increasing order.
  template <int KA = 0, class F>
  __device__ __forceinline__ static void blocks(int kbeg, int kend, const F& f) {
    if constexpr (KA < C::RX) {
      const int lo = max(kbeg, C::GX * KA), hi = min(kend, C::GX * (KA + 1));
      if (lo < hi) f(ic<KA>{}, lo, hi);
      blocks<KA + 1>(kbeg, kend, f);
    }
  }

  // Rank-1 update M += x x^T with x read from LDS (x[i] for every row
  // index below MMAX).
  __device__ __forceinline__ void rank1(const double* x) {
    double xi[C::RX], xj[C::RY];
#pragma unroll
    for (int a = 0; a < C::RX; ++a) xi[a] = x[row(a)];
#pragma unroll
    for (int b = 0; b < C::RY; ++b) xj[b] = x[col(b)];
#pragma unroll
    for (int a = 0; a < C::RX; ++a)
#pragma unroll
      for (int b = 0; b < C::RY; ++b)
        if (!skip(a, b)) v[a][b] = fma(xi[a], xj[b], v[a][b]);
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

}  // namespace mfb

// Tile-parallel sweeps for wide fronts: supernodes with a large ancestor
// set A (so a large A x A update block) and few columns N.  One workgroup
// per front would stream the whole A x A block through a single CU (about
// 30 GB/s); here every product or block whose size grows with A is cut
// into 64 x 64 (or 64-row) tiles over all wide fronts of a level, one
// workgroup each, and only the work that grows with N stays per front.
//
// Leaf-to-root sweeps (factor, product, Hessian step 1, inverse Hessian
// step 3): the per-front kernels of kernels.hip in PANEL mode assemble and
// process the front's N panel columns; k_wide_update then forms the update
// block U_s = sum_c E_c U_c E_c^T - (a rank-N or rank-2N product) tile by
// tile, gathering the children's entries through relative-index searches.
// Root-to-leaf sweeps (projected inverse, Hessian steps 2+3): the parent
// extraction of eq. e-sn-gradient-2 runs tile by tile, then the A x N
// products run over 64-row tiles and the N x N products per front.
//
// Tiles of a segment (the wide fronts of one level) are numbered front by
// front through prefix arrays: `pre[f]` is the first tile of front f.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "front.h"
#include "kernels.h"
#include "wg_dense.h"

namespace mfb {

constexpr int WT = 64;   // tile edge
constexpr int WKC = 32;  // k-chunk of the update's product staged in LDS
constexpr int WLD = WT + 1;

// Largest f < count with pre[f] <= b (the front owning tile b).
__device__ __forceinline__ int seg_front(const int32_t* pre, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Tile (ti, tj), ti >= tj, of the lower triangle of tiles, numbered column
// by column of rows: l = ti (ti + 1) / 2 + tj.
__device__ __forceinline__ void tri_tile(int l, int& ti, int& tj) {
  int t = int((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while (t * (t + 1) / 2 > l) --t;
  while ((t + 1) * (t + 2) / 2 <= l) ++t;
  ti = t;
  tj = l - t * (t + 1) / 2;
}

// Index of parent front position p in a child's increasing relative-index
// list rl[0 .. Ac), or -1.
__device__ __forceinline__ int find_rel(const int32_t* rl, int Ac, int p) {
  int lo = 0, hi = Ac;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rl[mid] < p)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < Ac && rl[lo] == p) ? lo : -1;
}

// ---------------------------------------------------------------------------
// Update block of a wide front, one 64 x 64 lower tile per workgroup
// (blockIdx.x: tile of the segment, blockIdx.y: right-hand side):
//   U(x, y) = sum over children c (fixed order) of U_c at the positions of
//             (x, y) in A_c, minus sum_k P1(x, k) P2(y, k),
// with the rank-K product of the operation:
//   WU_FACTOR (factor and product): P1 = P2 = B = L_AN C (the AN part of the
//             Cholesky panel R), K = N: U_s = G22 - B B^T;
//   WU_HUP  (Hessian step 1): P1 = [L, K_AN], P2 = [F'21, L], K = 2N:
//             U'_s = F'22 - L F'21^T - K_AN L^T, with F'21 left in the
//             panel kernel's scratch slot;
//   WU_IHUP (inverse Hessian step 3): P1 = [Q, L], P2 = [L, K_AN], K = 2N:
//             U'_s = G'22 - Q L^T - L K_AN^T, Q = L K_NN + K_AN in the
//             panel kernel's scratch slot (after its J x N panel).
// Thread t owns row t mod 64 and columns t / 64 + 4q of the tile, so the
// gathers from the children's packed columns and the stores are
// contiguous across a wavefront.
// (WU_PRODUCT: the product's update, the same arithmetic as WU_FACTOR under
// a kernel symbol of its own, so that profiles attribute it.)
enum { WU_FACTOR = 0, WU_HUP = 1, WU_IHUP = 2, WU_PRODUCT = 3 };

template <int OP>
__global__ void __launch_bounds__(NT) k_wide_update(DevPlan P, const int32_t* list, const int32_t* pre,
                                                    int count, const double* R, const double* LB,
                                                    const double* Kt, double* Ua, int64_t upd,
                                                    const double* wsb, int64_t slot) {
  __shared__ double p1[WKC * WLD], p2[WKC * WLD];
  __shared__ int invr[WT], invc[WT];
  __shared__ int64_t colc[kColCache];
  const int b = blockIdx.x;
  const int f = seg_front(pre, count, b);
  int ti, tj;
  tri_tile(b - pre[f], ti, tj);
  const int64_t r = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A, J = v.J;
    const int i0 = ti * WT, j0 = tj * WT;
    const int row = threadIdx.x & (WT - 1), cq = threadIdx.x >> 6;
    const double* K = Kt + r * P.nnz;
    const double* ws = wsb + (r * count + f) * slot;
    double* ua = Ua + r * upd;
    auto P1 = [&](int x, int k) -> double {
      if (OP == WU_FACTOR || OP == WU_PRODUCT) return R[v.an(x, k)];
      if (OP == WU_HUP) return k < N ? LB[v.an(x, k)] : K[v.an(x, k - N)];
      return k < N ? ws[(int64_t)J * N + x + (int64_t)k * A] : LB[v.an(x, k - N)];
    };
    auto P2 = [&](int y, int k) -> double {
      if (OP == WU_FACTOR || OP == WU_PRODUCT) return R[v.an(y, k)];
      if (OP == WU_HUP) return k < N ? ws[(N + y) + (int64_t)k * J] : LB[v.an(y, k - N)];
      return k < N ? LB[v.an(y, k)] : K[v.an(y, k - N)];
    };
    const int KK = (OP == WU_FACTOR || OP == WU_PRODUCT) ? N : 2 * N;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int k0 = 0; k0 < KK; k0 += WKC) {
      for (int e = threadIdx.x; e < WKC * WT; e += NT) {
        const int x = e & (WT - 1), kk = e >> 6;
        const bool okk = k0 + kk < KK;
        p1[kk * WLD + x] = (okk && i0 + x < A) ? P1(i0 + x, k0 + kk) : 0.0;
        p2[kk * WLD + x] = (okk && j0 + x < A) ? P2(j0 + x, k0 + kk) : 0.0;
      }
      __syncthreads();
      const int kn = min(WKC, KK - k0);
      for (int kk = 0; kk < kn; ++kk) {
        const double a = p1[kk * WLD + row];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = fma(a, p2[kk * WLD + cq + 4 * q], acc[q]);
      }
      __syncthreads();
    }
    double g[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) g[q] = 0.0;
    for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
      const int c = P.cidx[t];
      const int Ac = P.nrow[c] - P.ncol[c];
      const int32_t* rl = P.rel + P.relbase[c];
      const double* Uc = ua + P.arena[c];
      const int tid = threadIdx.x;
      if (tid < WT)
        invr[tid] = i0 + tid < A ? find_rel(rl, Ac, N + i0 + tid) : -1;
      else if (tid < 2 * WT)
        invc[tid - WT] = j0 + tid - WT < A ? find_rel(rl, Ac, N + j0 + tid - WT) : -1;
      __syncthreads();
      const int cx = invr[row];
      double u[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int cy = invc[cq + 4 * q];
        const bool ok = cx >= 0 && cy >= 0 && cx >= cy;
        const double val = Uc[ok ? pk(cx, cy, Ac) : 0];
        u[q] = ok ? val : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) g[q] += u[q];
      __syncthreads();
    }
    double* Us = ua + P.arena[v.s];
    const int gi = i0 + row;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int gj = j0 + cq + 4 * q;
      if (gi < A && gj < A && gi >= gj) Us[pk(gi, gj, A)] = g[q] - acc[q];
    }
  });
}
// ---------------------------------------------------------------------------
// Parent extraction of one lower 64 x 64 tile (ti, tj) of the packed block
// V_s = E^T [S_NN S_AN^T; S_AN V_p] E (eq. e-sn-gradient-2), from the
// parent's CCS columns of `src` and its packed block in `arena`.
__device__ __forceinline__ void wide_extract_tile(const DevPlan& P, int s, int ti, int tj, const double* src,
                                                  double* arena, int* rr, int* rc, int64_t* cpc) {
  const int N = P.ncol[s], A = P.nrow[s] - N;
  const int p = P.parent[s];
  const int Np = P.ncol[p], Ap = P.nrow[p] - Np;
  const int64_t* colp = P.col + P.colbase[p];
  const int32_t* rl = P.rel + P.relbase[s];
  const double* Vp = arena + P.arena[p];
  double* Vo = arena + P.arena[s];
  const int i0 = ti * WT, j0 = tj * WT;
  const int tid = threadIdx.x;
  if (tid < WT) {
    rr[tid] = i0 + tid < A ? rl[i0 + tid] : 0;
  } else if (tid < 2 * WT) {
    const int j = tid - WT;
    const int ry = j0 + j < A ? rl[j0 + j] : 0;
    rc[j] = ry;
    cpc[j] = ry < Np ? colp[ry] : 0;
  }
  __syncthreads();
  const int row = tid & (WT - 1), cq = tid >> 6;
  const int gi = i0 + row, rx = rr[row];
  double val[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = cq + 4 * q, gj = j0 + j;
    const bool ok = gi < A && gj < A && gi >= gj;
    const int ry = rc[j];
    const double* a = !ok ? src : (ry < Np ? src + cpc[j] + (rx - ry) : Vp + pk(rx - Np, ry - Np, Ap));
    val[q] = *a;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int gj = j0 + cq + 4 * q;
    if (gi < A && gj < A && gi >= gj) Vo[pk(gi, gj, A)] = val[q];
  }
}

// Tiles of the extraction over the segment (blockIdx.y: right-hand side,
// with its own source array and arena at the given strides).  TAG only
// names the caller in profiles: 0 the projected inverse, 1 the gather of
// T_AA for the inverse Hessian, 2 the gather of S_AA for the completion.
template <int TAG>
__global__ void __launch_bounds__(NT) k_wide_extract(DevPlan P, const int32_t* list, const int32_t* pre,
                                                     int count, const double* src, double* arena,
                                                     int64_t src_stride, int64_t arena_stride) {
  __shared__ int rr[WT], rc[WT];
  __shared__ int64_t cpc[WT];
  const int f = seg_front(pre, count, blockIdx.x);
  int ti, tj;
  tri_tile(blockIdx.x - pre[f], ti, tj);
  const int64_t r = blockIdx.y;
  wide_extract_tile(P, list[f], ti, tj, src + r * src_stride, arena + r * arena_stride, rr, rc, cpc);
}

// Rows [i0, i0 + 64) of V (A x A symmetric, packed) times an A x N operand b:
// accumulated into T, the k range split so that each part is fetched along
// its contiguous index (below the tile: packed columns k read down the rows;
// above it: the transposed entries V(k, i), read along k).
template <bool BK, class FB>
__device__ __forceinline__ void wide_sym_rows(MfmaTile& T, int i0, int A, int N, const double* V, const FB& fb,
                                              double* sm) {
  auto lo = [&](int i, int k) { return V[pk(i, k, A)]; };  // k <= i
  auto hi = [&](int i, int k) { return V[pk(k, i, A)]; };  // k >= i
  auto mid = [&](int i, int k) { return sym_packed(V, i, k, A); };
  const int d0 = min(i0, A), d1 = min(i0 + WT, A);
  tile_mma<false, BK>(T, i0, 0, A, N, 0, d0, lo, fb, sm);
  tile_mma<false, BK>(T, i0, 0, A, N, d0, d1, mid, fb, sm);
  tile_mma<true, BK>(T, i0, 0, A, N, d1, A, hi, fb, sm);
}

// ---------------------------------------------------------------------------
// Algorithm 7.2 on wide fronts (after k_wide_extract has put V_s in place):
// S_AN = -V_s L_AN over 64-row tiles (tiles numbered through `pre`), then
// S_NN = D^-1 - S_AN^T L_AN per front (k_wide_projinv_nn).
__global__ void __launch_bounds__(NT) k_wide_projinv_an(DevPlan P, const int32_t* list, const int32_t* pre,
                                                        int count, const double* LB, double* S,
                                                        const double* Vs) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = seg_front(pre, count, blockIdx.x);
  const int i0 = (blockIdx.x - pre[f]) * WT;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const double* V = Vs + P.arena[v.s];
    MfmaTile T(threadIdx.x);
    wide_sym_rows<true>(T, i0, v.A, v.N, V, [&](int k, int j) { return LB[v.an(k, j)]; }, sm);
    tile_store(T, i0, 0, v.A, v.N, [&](int i, int j, double acc) { S[v.an(i, j)] = -acc; }, false);
  });
}

__global__ void __launch_bounds__(NT) k_wide_projinv_nn(DevPlan P, const int32_t* list, const double* LB,
                                                        double* S) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    wg_gemm<true, true>(
        v.N, v.N, v.A, [&](int i, int k) { return S[v.an(k, i)]; },
        [&](int k, int j) { return LB[v.an(k, j)]; },
        [&](int i, int j, double acc) { S[v.at(i, j)] = LB[v.at(i, j)] - acc; }, true, sm);
  });
}

// ---------------------------------------------------------------------------
// Hessian steps 2+3 on wide fronts, three launches per segment.  Scratch
// slot per (front, right-hand side): MN (N x N), MA (A x N), Z (A x N),
// W (N x N), all column-major.
//  a: the extraction tiles of V'_s (grid part 1), per front W = K_NN D^-1
//     and MN = D^-1 W (part 2), Z = K_AN D^-1 over 64-row tiles (part 3);
//  b: per 64-row tile MA = V_s Z and T_AN = MA - V'_s L;
//  c: per front T_NN = MN - L^T T_AN - MA^T L.
__global__ void __launch_bounds__(NT) k_wide_hdown_a(DevPlan P, const int32_t* list, const int32_t* pre_aa,
                                                     const int32_t* pre_rt, int count, int n_aa,
                                                     const double* LB, const double* Kt, const double* T,
                                                     double* Va, int64_t upd, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  __shared__ int rr[WT], rc[WT];
  __shared__ int64_t cpc[WT];
  const int64_t r = blockIdx.y;
  const int b = blockIdx.x;
  if (b < n_aa) {
    const int f = seg_front(pre_aa, count, b);
    int ti, tj;
    tri_tile(b - pre_aa[f], ti, tj);
    wide_extract_tile(P, list[f], ti, tj, T + r * P.nnz, Va + r * upd, rr, rc, cpc);
    return;
  }
  const bool nn = b < n_aa + count;
  const int f = nn ? b - n_aa : seg_front(pre_rt, count, b - n_aa - count);
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    const double* K = Kt + r * P.nnz;
    double* MN = wsb + (r * count + f) * slot;
    double* Z = MN + (int64_t)N * N + (int64_t)A * N;
    double* W = Z + (int64_t)A * N;
    auto Dinv = [&](int i, int j) { return LB[v.nn(i, j)]; };
    if (nn) {
      wg_gemm<false, true>(
          N, N, N, [&](int i, int k) { return K[v.nn(i, k)]; }, Dinv,
          [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false, sm);
      __syncthreads();
      wg_gemm<false, true>(
          N, N, N, Dinv, [&](int k, int j) { return W[k + (int64_t)j * N]; },
          [&](int i, int j, double acc) { MN[i + (int64_t)j * N] = acc; }, true, sm);
    } else {
      const int i0 = (b - n_aa - count - pre_rt[f]) * WT;
      MfmaTile Tz(threadIdx.x);
      tile_mma<false, true>(Tz, i0, 0, A, N, 0, N, [&](int i, int k) { return K[v.an(i, k)]; }, Dinv, sm);
      tile_store(Tz, i0, 0, A, N, [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false);
    }
  });
}

__global__ void __launch_bounds__(NT) k_wide_hdown_b(DevPlan P, const int32_t* list, const int32_t* pre_rt,
                                                     int count, const double* LB, const double* Vs, double* T,
                                                     const double* Va, int64_t upd, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int64_t r = blockIdx.y;
  const int f = seg_front(pre_rt, count, blockIdx.x);
  const int i0 = (blockIdx.x - pre_rt[f]) * WT;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    double* t = T + r * P.nnz;
    double* MN = wsb + (r * count + f) * slot;
    double* MA = MN + (int64_t)N * N;
    const double* Z = MA + (int64_t)A * N;
    MfmaTile Tm(threadIdx.x);
    wide_sym_rows<true>(Tm, i0, A, N, Vs + P.arena[v.s], [&](int k, int j) { return Z[k + (int64_t)j * A]; },
                        sm);
    MfmaTile Tv(threadIdx.x);
    wide_sym_rows<true>(Tv, i0, A, N, Va + r * upd + P.arena[v.s], [&](int k, int j) { return LB[v.an(k, j)]; },
                        sm);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gi = i0 + Tm.row_of(e), gj = Tm.col_of(e);
      if (gi < A && gj < N) {
        const double ma = Tm.get(e);
        MA[gi + (int64_t)gj * A] = ma;
        t[v.an(gi, gj)] = ma - Tv.get(e);
      }
    }
  });
}

__global__ void __launch_bounds__(NT) k_wide_hdown_c(DevPlan P, const int32_t* list, int count,
                                                     const double* LB, double* T, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int64_t r = blockIdx.y;
  const int f = blockIdx.x;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    double* t = T + r * P.nnz;
    const double* MN = wsb + (r * count + f) * slot;
    const double* MA = MN + (int64_t)N * N;
    wg_gemm<true, true>(
        N, N, 2 * A, [&](int i, int k) { return k < A ? LB[v.an(k, i)] : MA[(k - A) + (int64_t)i * A]; },
        [&](int k, int j) { return k < A ? t[v.an(k, j)] : LB[v.an(k - A, j)]; },
        [&](int i, int j, double acc) { t[v.at(i, j)] = MN[i + (int64_t)j * N] - acc; }, true, sm);
  });
}

// ---------------------------------------------------------------------------
// Host launchers.

void launch_wide_update(int op, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const int32_t* pre, int count, const double* R, const double* LB, const double* Kt,
                        double* Ua, int64_t upd, const double* wsb, int64_t slot) {
  switch (op) {
    case WU_FACTOR:
      k_wide_update<WU_FACTOR><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot);
      break;
    case WU_HUP:
      k_wide_update<WU_HUP><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot);
      break;
    case WU_PRODUCT:
      k_wide_update<WU_PRODUCT><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot);
      break;
    default:
      k_wide_update<WU_IHUP><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot);
      break;
  }
}

void launch_wide_extract(int tag, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                         const int32_t* pre, int count, const double* src, double* arena, int64_t src_stride,
                         int64_t arena_stride) {
  if (tag == 1)
    k_wide_extract<1><<<grid, NT, 0, s>>>(P, list, pre, count, src, arena, src_stride, arena_stride);
  else
    k_wide_extract<2><<<grid, NT, 0, s>>>(P, list, pre, count, src, arena, src_stride, arena_stride);
}

void launch_wide_projinv(hipStream_t s, const DevPlan& P, const int32_t* list, const int32_t* pre_aa,
                         const int32_t* pre_rt, int count, int n_aa, int n_rt, const double* LB, double* S,
                         double* Vs) {
  k_wide_extract<0><<<dim3(unsigned(n_aa)), NT, 0, s>>>(P, list, pre_aa, count, S, Vs, 0, 0);
  k_wide_projinv_an<<<dim3(unsigned(n_rt)), NT, 0, s>>>(P, list, pre_rt, count, LB, S, Vs);
  k_wide_projinv_nn<<<dim3(unsigned(count)), NT, 0, s>>>(P, list, LB, S);
}

void launch_wide_hess_down(int k, hipStream_t s, const DevPlan& P, const int32_t* list, const int32_t* pre_aa,
                           const int32_t* pre_rt, int count, int n_aa, int n_rt, const double* LB,
                           const double* Vs, const double* Kt, double* T, double* Va, int64_t upd, double* wsb,
                           int64_t slot) {
  k_wide_hdown_a<<<dim3(unsigned(n_aa + count + n_rt), unsigned(k)), NT, 0, s>>>(
      P, list, pre_aa, pre_rt, count, n_aa, LB, Kt, T, Va, upd, wsb, slot);
  k_wide_hdown_b<<<dim3(unsigned(n_rt), unsigned(k)), NT, 0, s>>>(P, list, pre_rt, count, LB, Vs, T, Va, upd,
                                                                   wsb, slot);
  k_wide_hdown_c<<<dim3(unsigned(count), unsigned(k)), NT, 0, s>>>(P, list, count, LB, T, wsb, slot);
}

}  // namespace mfb

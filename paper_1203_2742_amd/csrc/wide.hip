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

#include <algorithm>
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

// First index t of a child's increasing relative-index list rl[0 .. Ac)
// with rl[t] >= p (Ac when there is none), by a 64-way search of each
// wavefront: every round probes 64 increasing positions at once and keeps
// the gap the answer lies in, so a list of up to 64 * 65 entries takes two
// dependent loads.  Called by whole wavefronts (the result is uniform).
__device__ __forceinline__ int lower_rel(const int32_t* rl, int Ac, int p) {
  const int lane = int(threadIdx.x) & 63;
  int lo = 0, hi = Ac;  // the answer lies in [lo, hi]
  while (hi - lo > 64) {
    const int n = hi - lo;
    const bool lt = rl[lo + int((int64_t)(lane + 1) * n / 65)] < p;
    const int c = __popcll(__ballot(lt));  // probes below p: a prefix of the lanes
    const int nlo = c > 0 ? lo + int((int64_t)c * n / 65) + 1 : lo;
    hi = c < 64 ? lo + int((int64_t)(c + 1) * n / 65) : hi;
    lo = nlo;
  }
  const bool lt = lane < hi - lo && rl[lo + lane] < p;
  return lo + __popcll(__ballot(lt));
}

// map[t] = the position x in a child's increasing relative-index list
// rl[0 .. Ac) with rl[x] = p0 + t, for the 64 parent positions p0 ..
// p0 + 63 below pend, else -1.  The child's entries in that window are one
// run of rl, found by two 64-way searches, then stored one per lane (a
// strictly increasing list has at most 64 of them).  Called by one whole
// wavefront; the caller synchronizes before map is read.
__device__ __forceinline__ void rel_window(const int32_t* rl, int Ac, int p0, int pend, int* map) {
  const int lane = int(threadIdx.x) & 63;
  map[lane] = -1;
  const int xb = lower_rel(rl, Ac, p0), xe = lower_rel(rl, Ac, min(p0 + WT, pend));
  wave_sync();
  if (xb + lane < xe) map[rl[xb + lane] - p0] = xb + lane;
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
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_wide_update(DevPlan P, const int32_t* list, const int32_t* pre,
                                                    int count, const double* R, const double* LB,
                                                    const double* Kt, double* Ua, int64_t upd,
                                                    const double* wsb, int64_t slot, const int32_t* act) {
  // the product's staging (tile_mma), then its 64 x 64 result in the
  // threads' layout of the gather below
  __shared__ double lds[2 * WKC * WLD];
  __shared__ int invr[WT], invc[WT];
  __shared__ int64_t colc[kColCache];
  const int b = blockIdx.x;
  const int f = seg_front(pre, count, b);
  int ti, tj;
  tri_tile(b - pre[f], ti, tj);
  const int64_t r = blockIdx.y;
  // Hessian step 1: a front whose subtree holds no nonzero of Y (marked by
  // its panel kernel) has a zero update block, neither formed nor read
  const int32_t* ac = (OP == WU_HUP && act) ? act + r * P.ns : nullptr;
  if (ac && !ac[list[f]]) return;  // (the whole workgroup)
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
    {
      MfmaTile T(threadIdx.x);
      tile_mma(T, i0, j0, A, A, 0, KK, P1, [&](int k, int y) { return P2(y, k); }, lds);
      tile_store(T, 0, 0, WT, WT, [&](int i, int j, double a) { lds[i + j * WLD] = a; }, false);
    }
    __syncthreads();
    // the product stays in LDS through the children's gather (read back
    // at the store), which keeps the gather's registers few
    double g[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) g[q] = 0.0;
    for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
      const int c = P.cidx[t];
      if (ac && !ac[c]) continue;  // (uniform)
      const int Ac = P.nrow[c] - P.ncol[c];
      const int32_t* rl = P.rel + P.relbase[c];
      const double* Uc = ua + P.arena[c];
      const int tid = threadIdx.x;
      if (tid < WT)
        rel_window(rl, Ac, N + i0, N + A, invr);
      else if (tid < 2 * WT)
        rel_window(rl, Ac, N + j0, N + A, invc);
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
      if (gi < A && gj < A && gi >= gj) Us[pk(gi, gj, A)] = g[q] - lds[row + (cq + 4 * q) * WLD];
    }
  });
}
// ---------------------------------------------------------------------------
// Parent extraction of one lower 64 x 64 tile (ti, tj) of the packed block
// V_s = E^T [S_NN S_AN^T; S_AN V_p] E (eq. e-sn-gradient-2), from the
// parent's CCS columns of `src` and its packed block in `arena`.
// Sum over the partial products of row tile ti (front with ta row tiles,
// N <= kPartN columns, partial area pb): entry (row, n) of the row block ti
// of V' L, in a fixed order (tiles (ti, J) for J <= ti, then (J, ti) for
// J >= ti, J ascending, each tile's two blocks in that order).
__device__ __forceinline__ double sum_partials(const double* pb, int ta, int ti, int N, int row, int n) {
  double acc = 0.0;
  const int64_t blk = (int64_t)WT * N;
  for (int J = 0; J < ta; ++J) {
    if (J <= ti) acc += pb[(int64_t)(ti * (ti + 1) / 2 + J) * 2 * blk + row + WT * n];
    if (J >= ti) acc += pb[(int64_t)(J * (J + 1) / 2 + ti) * 2 * blk + blk + row + WT * n];
  }
  return acc;
}

// Tile (ti, tj) of the extraction V'_s = E^T [.] E (eq. e-sn-gradient-2 and
// its Hessian counterparts) from the parent's CCS columns of src and its
// block in arena.  With pbase (a wide front with N <= kPartN columns; ps:
// 6 * 64 * kPartN doubles of LDS), also the tile's partial products with
// L = L_AN (taken from LB): P1 = V'_{ti,tj} L_tj and P2 = V'_{ti,tj}^T L_ti
// (strictly lower entries on a diagonal tile), 64 x N each, at pbase +
// l * 128 N, l = ti (ti + 1) / 2 + tj.  Ends with a barrier.
__device__ __forceinline__ void wide_extract_tile(const DevPlan& P, int s, int ti, int tj, const double* src,
                                                  double* arena, int* rr, int* rc, int64_t* cpc,
                                                  const double* LB = nullptr, double* pbase = nullptr,
                                                  double* ps = nullptr) {
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
  if (!pbase) return;  // (uniform: a property of the front)
  const int64_t* cols = P.col + P.colbase[s];
  double* Lr = ps;                   // L rows i0 .. i0 + 63: Lr[x + 64 n]
  double* Lc = ps + WT * kPartN;     // L rows j0 .. j0 + 63
  double* red = ps + 2 * WT * kPartN;  // P1 per wavefront: red[(w kPartN + n) 64 + row]
  for (int e = tid; e < 2 * WT * N; e += NT) {
    const int which = e / (WT * N), rem = e - which * WT * N, x = rem % WT, n = rem / WT;
    const int gx = (which ? j0 : i0) + x;
    (which ? Lc : Lr)[x + WT * n] = gx < A ? LB[cols[n] + N + gx - n] : 0.0;
  }
  __syncthreads();
  double* out = pbase + (int64_t)(ti * (ti + 1) / 2 + tj) * 2 * WT * N;
  for (int n = 0; n < N; ++n) {
    double a1 = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = cq + 4 * q, gj = j0 + j;
      if (gi < A && gj < A && gi >= gj) a1 += val[q] * Lc[j + WT * n];
    }
    red[(cq * kPartN + n) * WT + row] = a1;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = cq + 4 * q, gj = j0 + j;
      double a2 = (gi < A && gj < A && (ti != tj ? gi >= gj : gi > gj)) ? val[q] * Lr[row + WT * n] : 0.0;
      for (int o = 32; o > 0; o >>= 1) a2 += __shfl_xor(a2, o);
      if (row == 0) out[(int64_t)WT * N + j + WT * n] = a2;
    }
  }
  __syncthreads();
  for (int e = tid; e < WT * N; e += NT) {
    const int x = e % WT, n = e / WT;
    out[x + WT * n] = ((red[(0 * kPartN + n) * WT + x] + red[(1 * kPartN + n) * WT + x]) +
                       red[(2 * kPartN + n) * WT + x]) +
                      red[(3 * kPartN + n) * WT + x];
  }
  __syncthreads();
}

// Tiles of the extraction over the segment (blockIdx.y: right-hand side,
// with its own source array and arena at the given strides).  TAG only
// names the caller in profiles: 0 the projected inverse, 1 the gather of
// T_AA for the inverse Hessian, 2 the gather of S_AA for the completion.
// TAG 1 also takes the partial products of T_AA L for the fronts with
// partial areas when part is given (stride pstride per RHS).
template <int TAG>
__global__ void __launch_bounds__(NT) k_wide_extract(DevPlan P, const int32_t* list, const int32_t* pre,
                                                     int count, const double* src, double* arena,
                                                     int64_t src_stride, int64_t arena_stride, const double* LB,
                                                     double* part, int64_t pstride) {
  __shared__ int rr[WT], rc[WT];
  __shared__ int64_t cpc[WT];
  __shared__ double ps[TAG == 1 ? 6 * WT * kPartN : 1];
  const int f = seg_front(pre, count, blockIdx.x);
  int ti, tj;
  tri_tile(blockIdx.x - pre[f], ti, tj);
  const int64_t r = blockIdx.y;
  const int s = list[f];
  double* pbase = (TAG == 1 && part && P.poff[s] >= 0) ? part + r * pstride + P.poff[s] : nullptr;
  wide_extract_tile(P, s, ti, tj, src + r * src_stride, arena + r * arena_stride, rr, rc, cpc, LB, pbase, ps);
}

// Tile (ti, tj) of the ceil(A/64) x ceil(N/64) grid of an A x N block (an
// "AN tile") or of the ceil(N/64) x ceil(N/64) grid of an N x N block (an
// "NN tile"), numbered row by row within the front.
__device__ __forceinline__ void grid_tile(int l, int N, int& ti, int& tj) {
  const int tn = (N + WT - 1) / WT;
  ti = l / tn;
  tj = l - ti * tn;
}

// Rows [i0, i0 + 64) and columns [j0, j0 + 64) of V b, with V an A x A
// symmetric packed block and b(k, j) an A x N operand: accumulated into T,
// the k range split so that each part is fetched along its contiguous
// index (below the tile: packed columns k read down the rows; above it:
// the transposed entries V(k, i), read along k).
template <bool BK, class FB>
__device__ __forceinline__ void wide_sym_rows(MfmaTile& T, int i0, int j0, int A, int N, const double* V,
                                              const FB& fb, double* sm) {
  auto lo = [&](int i, int k) { return V[pk(i, k, A)]; };  // k <= i
  auto hi = [&](int i, int k) { return V[pk(k, i, A)]; };  // k >= i
  auto mid = [&](int i, int k) { return sym_packed(V, i, k, A); };
  const int d0 = min(i0, A), d1 = min(i0 + WT, A);
  tile_mma<false, BK>(T, i0, j0, A, N, 0, d0, lo, fb, sm);
  tile_mma<false, BK>(T, i0, j0, A, N, d0, d1, mid, fb, sm);
  tile_mma<true, BK>(T, i0, j0, A, N, d1, A, hi, fb, sm);
}

// wide_sym_rows on a NarrowTile (fronts with at most NC columns).
template <bool BK, int NC, class FB>
__device__ __forceinline__ void wide_sym_rows_narrow(NarrowTile<NC>& T, int i0, int j0, int A, int N, const double* V,
                                                     const FB& fb, double* sm) {
  auto lo = [&](int i, int k) { return V[pk(i, k, A)]; };  // k <= i
  auto hi = [&](int i, int k) { return V[pk(k, i, A)]; };  // k >= i
  auto mid = [&](int i, int k) { return sym_packed(V, i, k, A); };
  const int d0 = min(i0, A), d1 = min(i0 + WT, A);
  tile_mma_narrow<false, BK>(T, i0, j0, A, N, 0, d0, lo, fb, sm);
  tile_mma_narrow<false, BK>(T, i0, j0, A, N, d0, d1, mid, fb, sm);
  tile_mma_narrow<true, BK>(T, i0, j0, A, N, d1, A, hi, fb, sm);
}

// C(i, j) = sum_{k < K} a(k, i) b(k, j) for the lower triangle of a small
// N x N result (N <= SMALL_N), on the vector units: the workgroup strides
// over k (consecutive threads, consecutive k), each thread keeps the
// N(N+1)/2 partial sums, then one fixed-order reduction (a butterfly in
// each wavefront, then the wavefronts in order through LDS).  For the
// N x N products with a long k range (2A) of fronts with few columns,
// where a 64 x 64 matrix-core tile would be mostly empty.  epi(i, j, c)
// is called once per lower entry, by one thread.
constexpr int SMALL_N = 8;
template <class FA, class FB, class EPI>
__device__ __forceinline__ void small_nn_dot(int N, int K, const FA& fa, const FB& fb, const EPI& epi, double* sm) {
  constexpr int NP = SMALL_N * (SMALL_N + 1) / 2;
  double acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.0;
  for (int k = threadIdx.x; k < K; k += NT) {
    double a[SMALL_N], b[SMALL_N];
#pragma unroll
    for (int i = 0; i < SMALL_N; ++i) {
      a[i] = i < N ? fa(k, i) : 0.0;
      b[i] = i < N ? fb(k, i) : 0.0;
    }
    int p = 0;
#pragma unroll
    for (int i = 0; i < SMALL_N; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) acc[p++] += a[i] * b[j];
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    double v = acc[p];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (l == 0) sm[w * NP + p] = v;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    const int p = threadIdx.x;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    const int j = p - i * (i + 1) / 2;
    if (i < N) epi(i, j, ((sm[p] + sm[NP + p]) + sm[2 * NP + p]) + sm[3 * NP + p]);
  }
  __syncthreads();
}

// The same product for SMALL_N < N <= 32 on the matrix cores: a 32 x 32
// tile whose k range the four wavefronts split (wavefront w takes k-steps
// 8w .. 8w + 7 of every staged chunk of 32), the four partial tiles then
// summed in wavefront order, so the result does not depend on timing.  The
// operands are read along k (consecutive lanes, consecutive k).  sm holds
// at least 4 * 32 * 32 doubles.
template <class FA, class FB, class EPI>
__device__ __forceinline__ void small_nn_mfma(int N, int K, const FA& fa, const FB& fb, const EPI& epi,
                                              double* sm) {
  constexpr int T32 = 32, LD = T32 + 1, KS = 32, PER = KS * T32 / NT;
  double* As = sm;  // [k][LD]
  double* Bs = sm + KS * LD;
  const int tid = threadIdx.x, w = tid >> 6, lr = tid & 15, lk = (tid & 63) >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  double ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NT, k = e & (KS - 1), i = e / KS;
      const bool ok = i < N && k0 + k < K;
      ra[q] = ok ? fa(k0 + k, i) : 0.0;
      rb[q] = ok ? fb(k0 + k, i) : 0.0;
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NT, k = e & (KS - 1), i = e / KS;
      As[k * LD + i] = ra[q];
      Bs[k * LD + i] = rb[q];
    }
    __syncthreads();
    if (k0 + KS < K) fetch(k0 + KS);
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int k = 8 * w + 4 * st + lk;
      const double a0 = As[k * LD + lr], a1 = As[k * LD + 16 + lr];
      const double b0 = Bs[k * LD + lr], b1 = Bs[k * LD + 16 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* red = sm;  // [wavefront][32 x 32]
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = 16 * (e >> 3) + lk + 4 * (e & 3), col = 16 * ((e >> 2) & 1) + lr;
    red[w * T32 * T32 + row * T32 + col] = acc[e >> 3][(e >> 2) & 1][e & 3];
  }
  __syncthreads();
  for (int idx = tid; idx < T32 * T32; idx += NT) {
    const int row = idx / T32, col = idx % T32;
    if (row < N && col <= row) {
      double c = red[idx];
#pragma unroll
      for (int q = 1; q < 4; ++q) c += red[q * T32 * T32 + idx];
      epi(row, col, c);
    }
  }
  __syncthreads();
}

// Right-hand sides batched along the columns of a product whose left
// operand (a packed A x A block shared by all right-hand sides) is the
// expensive read: column tile c of a front with N columns covers, when
// N <= 64, the right-hand sides c g .. c g + g - 1 (g = floor(64 / N)), N
// columns each; when N > 64, 64 columns of one right-hand side.  Tiles
// per front: ct; the largest ct of a segment is that of its largest N.
struct RhsCols {
  int N, k, g, tn, ct;
  __host__ __device__ RhsCols(int N_, int k_) : N(N_), k(k_) {
    if (N <= WT) {
      g = WT / N;
      tn = 1;
      ct = (k + g - 1) / g;
    } else {
      g = 1;
      tn = (N + WT - 1) / WT;
      ct = tn * k;
    }
  }
  // local column lc of tile c -> right-hand side r and column j; false
  // past the tile's columns
  __device__ __forceinline__ bool map(int c, int lc, int& r, int& j) const {
    if (N <= WT) {
      const int rr = lc / N;
      r = c * g + rr;
      j = lc - rr * N;
      return rr < g && r < k;
    }
    r = c / tn;
    j = (c - r * tn) * WT + lc;
    return j < N;
  }
};

// ---------------------------------------------------------------------------
// Algorithm 7.2 on wide fronts (after k_wide_extract has put V_s in place):
// S_AN = -V_s L_AN over the AN tiles, then S_NN = D^-1 - S_AN^T L_AN over
// the lower NN tiles.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_wide_projinv_an(DevPlan P, const int32_t* list, const int32_t* pre,
                                                        int count, const double* LB, double* S,
                                                        const double* Vs) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = seg_front(pre, count, blockIdx.x);
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    int ti, tj;
    grid_tile(blockIdx.x - pre[f], v.N, ti, tj);
    const int i0 = ti * WT, j0 = tj * WT;
    const double* V = Vs + P.arena[v.s];
    MfmaTile T(threadIdx.x);
    wide_sym_rows<true>(T, i0, j0, v.A, v.N, V, [&](int k, int j) { return LB[v.an(k, j)]; }, sm);
    tile_store(T, i0, j0, v.A, v.N, [&](int i, int j, double acc) { S[v.an(i, j)] = -acc; }, false);
  });
}

__global__ void __launch_bounds__(NT) k_wide_projinv_nn(DevPlan P, const int32_t* list, const int32_t* pre,
                                                        int count, const double* LB, double* S) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = seg_front(pre, count, blockIdx.x);
  const int N = P.ncol[list[f]];
  int ti, tj;
  grid_tile(blockIdx.x - pre[f], N, ti, tj);
  if (tj > ti) return;  // a tile wholly above the diagonal (the whole workgroup)
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int i0 = ti * WT, j0 = tj * WT;
    MfmaTile T(threadIdx.x);
    tile_mma<true, true>(T, i0, j0, v.N, v.N, 0, v.A, [&](int i, int k) { return S[v.an(k, i)]; },
                         [&](int k, int j) { return LB[v.an(k, j)]; }, sm);
    tile_store(T, i0, j0, v.N, v.N, [&](int i, int j, double acc) { S[v.at(i, j)] = LB[v.at(i, j)] - acc; },
               true);
  });
}

// ---------------------------------------------------------------------------
// Hessian steps 2+3 on wide fronts, three launches per segment.  Scratch
// slot per (front, right-hand side): MN (N x N), MA (A x N), Z (A x N),
// W (N x N), all column-major.
//  a: the extraction tiles of V'_s, W = K_NN D^-1 over the NN tiles and
//     Z = K_AN D^-1 over the AN tiles;
//  vz: MA = V_s Z over the AN tiles, right-hand sides batched along the
//     columns (V_s is read once per 64 columns instead of once per RHS);
//  b: MN = D^-1 W over the lower NN tiles; T_AN = MA - V'_s L over the AN
//     tiles;
//  c: T_NN = MN - L^T T_AN - MA^T L over the lower NN tiles.
struct SegTiles {
  const int32_t* aa;  // prefix arrays (count + 1 entries each)
  const int32_t* an;
  const int32_t* nn;
  int n_aa, n_an, n_nn;
};

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_wide_hdown_a(DevPlan P, const int32_t* list, SegTiles tl, int count,
                                                     const double* LB, const double* Kt, const double* T,
                                                     double* Va, int64_t upd, double* wsb, int64_t slot,
                                                     double* part, int64_t pstride) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  __shared__ int rr[WT], rc[WT];
  __shared__ int64_t cpc[WT];
  const int64_t r = blockIdx.y;
  int b = blockIdx.x;
  if (b < tl.n_aa) {
    const int f = seg_front(tl.aa, count, b);
    int ti, tj;
    tri_tile(b - tl.aa[f], ti, tj);
    const int s = list[f];
    double* pbase = P.poff[s] >= 0 ? part + r * pstride + P.poff[s] : nullptr;
    wide_extract_tile(P, s, ti, tj, T + r * P.nnz, Va + r * upd, rr, rc, cpc, LB, pbase, sm);
    return;
  }
  b -= tl.n_aa;
  const bool nn = b < tl.n_nn;
  if (!nn) b -= tl.n_nn;
  const int32_t* pre = nn ? tl.nn : tl.an;
  const int f = seg_front(pre, count, b);
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    int ti, tj;
    grid_tile(b - pre[f], N, ti, tj);
    const int i0 = ti * WT, j0 = tj * WT;
    const double* K = Kt + r * P.nnz;
    double* MN = wsb + (r * count + f) * slot;
    double* Z = MN + (int64_t)N * N + (int64_t)A * N;
    double* W = Z + (int64_t)A * N;
    auto Dinv = [&](int i, int j) { return LB[v.nn(i, j)]; };
    MfmaTile Tt(threadIdx.x);
    if (nn) {
      tile_mma<false, true>(Tt, i0, j0, N, N, 0, N, [&](int i, int k) { return K[v.nn(i, k)]; }, Dinv, sm);
      tile_store(Tt, i0, j0, N, N, [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false);
    } else {
      tile_mma<false, true>(Tt, i0, j0, A, N, 0, N, [&](int i, int k) { return K[v.an(i, k)]; }, Dinv, sm);
      tile_store(Tt, i0, j0, A, N, [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false);
    }
  });
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_wide_hdown_b(DevPlan P, const int32_t* list, SegTiles tl, int count,
                                                     const double* LB, const double* Vs, double* T,
                                                     const double* Va, int64_t upd, double* wsb, int64_t slot,
                                                     const double* part, int64_t pstride) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int64_t r = blockIdx.y;
  int b = blockIdx.x;
  const bool nn = b < tl.n_nn;
  if (!nn) b -= tl.n_nn;
  const int32_t* pre = nn ? tl.nn : tl.an;
  const int f = seg_front(pre, count, b);
  const int N = P.ncol[list[f]];
  int ti, tj;
  grid_tile(b - pre[f], N, ti, tj);
  if (nn && tj > ti) return;  // MN is read on and below the diagonal only
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int A = v.A;
    const int i0 = ti * WT, j0 = tj * WT;
    double* t = T + r * P.nnz;
    double* MN = wsb + (r * count + f) * slot;
    const double* MA = MN + (int64_t)N * N;
    const double* W = MA + 2 * (int64_t)A * N;
    if (nn) {
      MfmaTile Tt(threadIdx.x);
      tile_mma<false, true>(Tt, i0, j0, N, N, 0, N, [&](int i, int k) { return LB[v.nn(i, k)]; },
                            [&](int k, int j) { return W[k + (int64_t)j * N]; }, sm);
      tile_store(Tt, i0, j0, N, N, [&](int i, int j, double acc) { MN[i + (int64_t)j * N] = acc; }, true);
      return;
    }
    if (P.poff[v.s] >= 0) {  // V'_s L from the extraction's partial products
      const double* pb = part + r * pstride + P.poff[v.s];
      const int ta = (A + WT - 1) / WT;
      for (int e = threadIdx.x; e < WT * N; e += NT) {
        const int row = e % WT, n = e / WT, gi = i0 + row;
        if (gi < A) t[v.an(gi, n)] = MA[gi + (int64_t)n * A] - sum_partials(pb, ta, ti, N, row, n);
      }
      return;
    }
    MfmaTile Tv(threadIdx.x);
    wide_sym_rows<true>(Tv, i0, j0, A, N, Va + r * upd + P.arena[v.s],
                        [&](int k, int j) { return LB[v.an(k, j)]; }, sm);
    tile_store(
        Tv, i0, j0, A, N, [&](int i, int j, double acc) { t[v.an(i, j)] = MA[i + (int64_t)j * A] - acc; }, false);
  });
}

// MA_r = V_s Z_r for every right-hand side r of every front of the segment
// (blockIdx.y), 64-row tile x RhsCols column tile per workgroup.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_wide_hdown_vz(DevPlan P, const int32_t* list, int count, int k, int ct_max,
                                                      const double* Vs, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  const int f = blockIdx.y;
  const int s = list[f];
  const int N = P.ncol[s], A = P.nrow[s] - N;
  const int ti = int(blockIdx.x) / ct_max, c = int(blockIdx.x) - ti * ct_max;
  const RhsCols rc(N, k);
  if (ti * WT >= A || c >= rc.ct) return;
  const int i0 = ti * WT;
  auto base = [&](int r) { return wsb + ((int64_t)r * count + f) * slot + (int64_t)N * N; };  // MA_r, then Z_r
  MfmaTile T(threadIdx.x);
  wide_sym_rows<true>(T, i0, 0, A, WT, Vs + P.arena[s],
                      [&](int kk, int lc) {
                        int r, j;
                        return rc.map(c, lc, r, j) ? base(r)[(int64_t)A * N + kk + (int64_t)j * A] : 0.0;
                      },
                      sm);
  tile_store(
      T, i0, 0, A, WT,
      [&](int i, int lc, double acc) {
        int r, j;
        if (rc.map(c, lc, r, j)) base(r)[i + (int64_t)j * A] = acc;
      },
      false);
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) k_wide_hdown_c(DevPlan P, const int32_t* list, SegTiles tl, int count,
                                                     const double* LB, double* T, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int64_t r = blockIdx.y;
  const int f = seg_front(tl.nn, count, blockIdx.x);
  const int N = P.ncol[list[f]];
  int ti, tj;
  grid_tile(blockIdx.x - tl.nn[f], N, ti, tj);
  if (tj > ti) return;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int A = v.A;
    const int i0 = ti * WT, j0 = tj * WT;
    double* t = T + r * P.nnz;
    const double* MN = wsb + (r * count + f) * slot;
    const double* MA = MN + (int64_t)N * N;
    auto fa = [&](int k, int i) { return k < A ? LB[v.an(k, i)] : MA[(k - A) + (int64_t)i * A]; };
    auto fb = [&](int k, int j) { return k < A ? t[v.an(k, j)] : LB[v.an(k - A, j)]; };
    auto out = [&](int i, int j, double acc) { t[v.at(i, j)] = MN[i + (int64_t)j * N] - acc; };
    if (N <= SMALL_N) {
      small_nn_dot(N, 2 * A, fa, fb, out, sm);
      return;
    }
    if (N <= 32) {
      small_nn_mfma(N, 2 * A, fa, fb, out, sm);
      return;
    }
    MfmaTile Tt(threadIdx.x);
    tile_mma<true, true>(
        Tt, i0, j0, N, N, 0, 2 * A,
        [&](int i, int k) { return k < A ? LB[v.an(k, i)] : MA[(k - A) + (int64_t)i * A]; },
        [&](int k, int j) { return k < A ? t[v.an(k, j)] : LB[v.an(k - A, j)]; }, sm);
    tile_store(Tt, i0, j0, N, N, [&](int i, int j, double acc) { t[v.at(i, j)] = MN[i + (int64_t)j * N] - acc; },
               true);
  });
}

// ---------------------------------------------------------------------------
// Fat fronts: more than kWideMaxN columns (the large separators and the
// root).  The leaf-to-root sweeps' panel work (the J x N columns of the
// front) runs tile-parallel too.  Grids are two-dimensional: blockIdx.x is
// a tile of the front, blockIdx.y = f + count * r picks the front f of the
// segment and the right-hand side r; tiles beyond a front's own count exit
// at once.  Scratch slot per (front, RHS) starts with the panel F (J x N,
// column-major, leading dimension J).

// Lower-triangle accessor of a packed symmetric A x A block.
struct PackedLowerW {
  double* u;
  int A;
  __device__ __forceinline__ double& operator()(int i, int j) const { return u[pk(i, j, A)]; }
};

// Tile counts of a front, in 64-wide tiles.
struct FatDims {
  int N, A, J, tn, ta, tj;
  __device__ __forceinline__ explicit FatDims(const SnView& v)
      : N(v.N), A(v.A), J(v.J), tn((v.N + WT - 1) / WT), ta((v.A + WT - 1) / WT), tj((v.J + WT - 1) / WT) {}
};

// The front's panel F (rows 0..J-1, columns 0..N-1; zero above the
// diagonal) = the input's CCS panel (X for the factor, Y for Hessian step
// 1; none for the product and inverse Hessian step 3) plus the children's
// update blocks at their relative positions, children in a fixed order.
// Tiles: ceil(J/64) x ceil(N/64), those wholly above the diagonal skipped.
template <int TAG>
__global__ void __launch_bounds__(NT) k_fat_panel(DevPlan P, const int32_t* list, int count, const double* src,
                                                  const double* Ua, int64_t upd, double* wsb, int64_t slot,
                                                  const int32_t* act) {
  __shared__ int64_t colc[kColCache];
  __shared__ int invr[WT], invc[WT];
  const int f = blockIdx.y % count;
  const int64_t r = blockIdx.y / count;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const FatDims d(v);
    const int l = blockIdx.x;
    if (l >= d.tj * d.tn) return;
    const int ti = l / d.tn, tj = l - (l / d.tn) * d.tn;
    const int i0 = ti * WT, j0 = tj * WT;
    if (i0 + WT - 1 < j0) return;
    const double* y = src ? src + r * P.nnz : nullptr;
    const double* ua = Ua + r * upd;
    double* F = wsb + (r * count + f) * slot;
    const int row = threadIdx.x & (WT - 1), cq = threadIdx.x >> 6;
    const int gi = i0 + row;
    double g[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int gj = j0 + cq + 4 * q;
      const bool ok = y && gi < d.J && gj < d.N && gi >= gj;
      const double val = y ? y[ok ? v.at(gi, gj) : v.at(0, 0)] : 0.0;
      g[q] = ok ? val : 0.0;
    }
    for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
      const int c = P.cidx[t];
      if (TAG == 1 && act && !act[r * P.ns + c]) continue;  // (uniform) pruned child, Hessian step 1
      const int Ac = P.nrow[c] - P.ncol[c];
      const int32_t* rl = P.rel + P.relbase[c];
      const double* Uc = ua + P.arena[c];
      const int tid = threadIdx.x;
      if (tid < WT)
        rel_window(rl, Ac, i0, d.J, invr);
      else if (tid < 2 * WT)
        rel_window(rl, Ac, j0, d.N, invc);
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
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int gj = j0 + cq + 4 * q;
      if (gi < d.J && gj < d.N) F[gi + (int64_t)gj * d.J] = gi >= gj ? g[q] : 0.0;
    }
  });
}

// Blocked Cholesky of the panel F, block column kb (64 columns): the
// diagonal block by one workgroup per front (Cholesky factor C_kk in F,
// its inverse in the scratch block list after F, the log det part), then
// (k_fat_potrf_panel) the rows below times C_kk^-T, then
// (k_fat_potrf_trail) the remaining panel columns updated.  The inverse
// blocks are stored 64 x 64 (zero above the diagonal) at F + rows N + 4096 b
// for block column b, and X = C^-1 (k_fat_trtri_row) after them.
// Two layouts (`sq`):
//  sq = 0, the factor: F is the J x N panel at the start of the slot
//          (rows J, leading dimension J); C and B are also written to R,
//          and part[s] receives log det D = 2 sum log C_kk;
//  sq = 1, the completion: F is an N x N matrix at slot offset `off`
//          (rows N, leading dimension N) holding the reversed Schur
//          complement; nothing goes to R, part[s] receives
//          -2 sum log C_kk, and a failure is reported as no completion at
//          the column of the original order.
struct FatSquare {
  int sq;
};
__device__ __forceinline__ int fat_rows(const FatSquare& q, int N, int J) { return q.sq ? N : J; }
// F of front f: the slot's start (factor) or after the completion's W (A x N)
__device__ __forceinline__ double* fat_F(double* wsb, int f, int64_t slot, const FatSquare& q, int N, int A) {
  return wsb + (int64_t)f * slot + (q.sq ? (int64_t)A * N : 0);
}

template <int SQ>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) k_fat_potrf_diag(DevPlan P, const int32_t* list, int count, int kb,
                                                       double* R, double* part, DevStatus* st, double* wsb,
                                                       int64_t slot) {
  constexpr FatSquare q{SQ};
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double d64[NB2 * LD2];  // the diagonal block, factored and inverted in LDS
  __shared__ int64_t colc[kColCache];
  __shared__ int fail;
  const int f = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    if (kb >= v.N) return;
    const int nb = min(WT, v.N - kb), J = fat_rows(q, v.N, v.J);
    double* F = fat_F(wsb, f, slot, q, v.N, v.A);
    double* Ci = F + (int64_t)J * v.N + (int64_t)(kb / WT) * WT * WT;
    if (threadIdx.x == 0) fail = -1;
    const DenseAt G{F + kb + (int64_t)kb * J, J};
    const DenseAt D{d64, LD2};
    for (int e = threadIdx.x; e < WT * WT; e += NT) {
      const int i = e & (WT - 1), j = e >> 6;
      D(i, j) = (i < nb && j < nb && i >= j) ? G(i, j) : 0.0;
    }
    __syncthreads();
    wg_potrf_acc(D, nb, nb, sm, &fail);
    __syncthreads();
    double lg = 0.0;
    for (int c = threadIdx.x; c < nb; c += NT) lg += 2.0 * log(D(c, c));
    for (int e = threadIdx.x; e < WT * WT; e += NT) {
      const int i = e & (WT - 1), j = e >> 6;
      if (i < nb && j < nb && i >= j) {
        G(i, j) = D(i, j);
        if (!q.sq) R[v.at(kb + i, kb + j)] = D(i, j);
      }
    }
    __syncthreads();
    wg_trtri_inplace(D, nb, sm);
    __syncthreads();
    for (int e = threadIdx.x; e < WT * WT; e += NT) {
      const int i = e & (WT - 1), j = e >> 6;
      Ci[e] = (i < nb && j < nb && i >= j) ? D(i, j) : 0.0;
    }
    lg = wg_sum(lg, sm);
    if (threadIdx.x == 0) {
      const double part_ = q.sq ? -lg : lg;
      part[v.s] = kb == 0 ? part_ : part[v.s] + part_;
      if (fail >= 0) {
        if (q.sq)
          report(st, MFB_ENOCOMPLETION, v.vl[v.N - 1 - (kb + fail)]);
        else
          report(st, MFB_ENOTPD, v.vl[kb + fail]);
      }
    }
  });
}

template <int SQ>
__global__ void __launch_bounds__(NT) k_fat_potrf_panel(DevPlan P, const int32_t* list, int count, int kb,
                                                        double* R, double* wsb, int64_t slot) {
  constexpr FatSquare q{SQ};
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    if (kb >= v.N) return;
    const int nb = min(WT, v.N - kb), J = fat_rows(q, v.N, v.J);
    const int i0 = kb + nb + int(blockIdx.x) * WT;
    if (i0 >= J) return;
    double* F = fat_F(wsb, f, slot, q, v.N, v.A);
    const double* Ci = F + (int64_t)J * v.N + (int64_t)(kb / WT) * WT * WT;
    MfmaTile T(threadIdx.x);
    tile_mma(T, i0, 0, J, nb, 0, nb, [&](int i, int k) { return F[i + (int64_t)(kb + k) * J]; },
             [&](int k, int j) { return Ci[j + k * WT]; }, sm);
    tile_store(
        T, i0, 0, J, nb,
        [&](int i, int j, double acc) {
          F[i + (int64_t)(kb + j) * J] = acc;
          if (!q.sq) R[v.at(i, kb + j)] = acc;
        },
        false);
  });
}

template <int SQ>
__global__ void __launch_bounds__(NT) k_fat_potrf_trail(DevPlan P, const int32_t* list, int count, int kb,
                                                        double* wsb, int64_t slot) {
  constexpr FatSquare q{SQ};
  __shared__ double sm[SMEM_DOUBLES];
  const int f = blockIdx.y;
  const int s = list[f];
  const int N = P.ncol[s], J = fat_rows(q, N, P.nrow[s]);
  if (kb >= N) return;
  const int nb = min(WT, N - kb), r0 = kb + nb;
  if (r0 >= N) return;
  const int tc = (N - r0 + WT - 1) / WT, tr = (J - r0 + WT - 1) / WT;
  const int l = blockIdx.x;
  if (l >= tr * tc) return;
  const int ti = l / tc, tj = l - (l / tc) * tc;
  if (ti < tj) return;
  const int i0 = r0 + ti * WT, j0 = r0 + tj * WT;
  double* F = fat_F(wsb, f, slot, q, N, P.nrow[s] - N);
  MfmaTile T(threadIdx.x);
  tile_mma(T, i0, j0, J, N, 0, nb, [&](int i, int k) { return F[i + (int64_t)(kb + k) * J]; },
           [&](int k, int c) { return F[c + (int64_t)(kb + k) * J]; }, sm);
  tile_store(T, i0, j0, J, N, [&](int i, int c, double acc) { F[i + (int64_t)c * J] -= acc; }, true);
}

// Row block ib of X = C^-1 (C the N x N Cholesky factor in F, X in the
// slot after the inverse blocks, N x N column-major), one 64 x 64 tile
// (ib, jb), jb <= ib, per workgroup:
//   X(ib, jb) = C_ib,ib^-1 (delta I - sum_{jb <= m < ib} C(ib, m) X(m, jb)),
// so a launch per ib completes row block ib from the ones above it.
template <int SQ>
__global__ void __launch_bounds__(NT) k_fat_trtri_row(DevPlan P, const int32_t* list, int count, int ib,
                                                      double* wsb, int64_t slot) {
  constexpr FatSquare q{SQ};
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double rb[WT * WLD];
  const int f = blockIdx.y;
  const int s = list[f];
  const int N = P.ncol[s], J = fat_rows(q, N, P.nrow[s]);
  const int i0 = ib * WT, jb = blockIdx.x, j0 = jb * WT;
  if (i0 >= N || jb > ib) return;
  const int nbi = min(WT, N - i0);
  double* F = fat_F(wsb, f, slot, q, N, P.nrow[s] - N);
  const double* Cinv = F + (int64_t)J * N + (int64_t)ib * WT * WT;
  double* X = F + (int64_t)J * N + (int64_t)((N + WT - 1) / WT) * WT * WT;
  MfmaTile T(threadIdx.x);
  tile_mma<false, true>(T, i0, j0, N, N, j0, i0, [&](int i, int k) { return F[i + (int64_t)k * J]; },
                        [&](int k, int j) { return X[k + (int64_t)j * N]; }, sm);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int li = T.row_of(e), lj = T.col_of(e);
    rb[li + lj * WLD] = (jb == ib && li == lj ? 1.0 : 0.0) - T.get(e);
  }
  __syncthreads();
  MfmaTile T2(threadIdx.x);
  tile_mma(T2, 0, 0, nbi, WT, 0, nbi, [&](int i, int k) { return Cinv[i + k * WT]; },
           [&](int k, int j) { return rb[k + j * WLD]; }, sm);
  tile_store(T2, 0, 0, nbi, min(WT, N - j0),
             [&](int i, int j, double acc) { X[(i0 + i) + (int64_t)(j0 + j) * N] = acc; }, false);
}

// The factor's closing products on a fat front, X = C^-1 from
// k_fat_trtri_row: D^-1 = X^T X over the lower NN tiles and
// L_AN = B X over the AN tiles (B = the panel rows below N).
__global__ void __launch_bounds__(NT) k_fat_factor_fin(DevPlan P, const int32_t* list, int count, double* LB,
                                                       double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const FatDims d(v);
    int b = blockIdx.x;
    if (b >= d.tn * d.tn + d.ta * d.tn) return;
    const double* F = wsb + (int64_t)f * slot;
    const double* X = F + (int64_t)d.J * d.N + (int64_t)d.tn * WT * WT;
    MfmaTile T(threadIdx.x);
    if (b < d.tn * d.tn) {
      const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
      if (tj > ti) return;
      const int i0 = ti * WT, j0 = tj * WT;
      tile_mma<true, true>(T, i0, j0, d.N, d.N, i0, d.N, [&](int i, int k) { return X[k + (int64_t)i * d.N]; },
                           [&](int k, int j) { return X[k + (int64_t)j * d.N]; }, sm);
      tile_store(T, i0, j0, d.N, d.N, [&](int i, int j, double acc) { LB[v.at(i, j)] = acc; }, true);
    } else {
      b -= d.tn * d.tn;
      const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
      const int i0 = ti * WT, j0 = tj * WT;
      tile_mma<false, true>(T, i0, j0, d.A, d.N, j0, d.N,
                            [&](int x, int k) { return F[(d.N + x) + (int64_t)k * d.J]; },
                            [&](int k, int j) { return X[k + (int64_t)j * d.N]; }, sm);
      tile_store(T, i0, j0, d.A, d.N, [&](int x, int j, double acc) { LB[v.an(x, j)] = acc; }, false);
    }
  });
}

// The closing products of the other leaf-to-root sweeps on a fat front,
// over the lower NN tiles and the AN tiles (G = the panel F of children's
// contributions):
//  FAT_PRODUCT: X_NN = C C^T - G11, X_AN = B C^T - G21 (Algorithm 3.2);
//  FAT_HUP:     K_NN = F'11, K_AN = F'21 - L F'11 (Hessian step 1);
//  FAT_IHUP:    Y_NN = K_NN - G'11, Q = L K_NN + K_AN (kept in the slot
//               after the panel), Y_AN = Q - G'21 (inverse Hessian step 3).
enum { FAT_PRODUCT = 0, FAT_HUP = 1, FAT_IHUP = 2 };
template <int OP>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_fat_up_fin(DevPlan P, const int32_t* list, int count, const double* R,
                                                   const double* LB, double* Out, double* Kt, double* wsb,
                                                   int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y % count;
  const int64_t r = blockIdx.y / count;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const FatDims d(v);
    int b = blockIdx.x;
    if (b >= d.tn * d.tn + d.ta * d.tn) return;
    double* F = wsb + (r * count + f) * slot;
    double* out = Out + r * P.nnz;
    double* K = Kt ? Kt + r * P.nnz : nullptr;
    const int N = d.N, J = d.J, A = d.A;
    MfmaTile T(threadIdx.x);
    if (b < d.tn * d.tn) {
      const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
      if (tj > ti) return;
      const int i0 = ti * WT, j0 = tj * WT;
      if (OP == FAT_PRODUCT) {
        auto C = [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; };
        tile_mma(T, i0, j0, N, N, 0, min(N, j0 + WT), C, [&](int k, int j) { return C(j, k); }, sm);
        tile_store(T, i0, j0, N, N,
                   [&](int i, int j, double acc) { out[v.at(i, j)] = acc - F[i + (int64_t)j * J]; }, true);
      } else {
        // a copy: K_NN = F'11 (Hessian), Y_NN = K_NN - G'11 (inverse Hessian)
        const int row = threadIdx.x & (WT - 1), cq = threadIdx.x >> 6;
        const int gi = i0 + row;
        for (int q = 0; q < 16; ++q) {
          const int gj = j0 + cq + 4 * q;
          if (gi < N && gj < N && gi >= gj) {
            const double fv = F[gi + (int64_t)gj * J];
            if (OP == FAT_HUP)
              K[v.at(gi, gj)] = fv;
            else
              out[v.at(gi, gj)] = K[v.at(gi, gj)] - fv;
          }
        }
      }
      return;
    }
    b -= d.tn * d.tn;
    const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
    const int i0 = ti * WT, j0 = tj * WT;
    if (OP == FAT_PRODUCT) {
      tile_mma(T, i0, j0, A, N, 0, min(N, j0 + WT), [&](int x, int k) { return R[v.an(x, k)]; },
               [&](int k, int j) { return k <= j ? R[v.at(j, k)] : 0.0; }, sm);
      tile_store(T, i0, j0, A, N,
                 [&](int x, int j, double acc) { out[v.an(x, j)] = acc - F[(N + x) + (int64_t)j * J]; }, false);
    } else if (OP == FAT_HUP) {
      auto F11 = [&](int k, int j) { return k >= j ? F[k + (int64_t)j * J] : F[j + (int64_t)k * J]; };
      tile_mma<false, true>(T, i0, j0, A, N, 0, N, [&](int x, int k) { return LB[v.an(x, k)]; }, F11, sm);
      tile_store(T, i0, j0, A, N,
                 [&](int x, int j, double acc) { K[v.an(x, j)] = F[(N + x) + (int64_t)j * J] - acc; }, false);
    } else {
      double* Q = F + (int64_t)J * N;
      tile_mma<false, true>(T, i0, j0, A, N, 0, N, [&](int x, int k) { return LB[v.an(x, k)]; },
                            [&](int k, int j) { return K[v.nn(k, j)]; }, sm);
      tile_store(
          T, i0, j0, A, N,
          [&](int x, int j, double acc) {
            const double q = acc + K[v.an(x, j)];
            Q[x + (int64_t)j * A] = q;
            out[v.an(x, j)] = q - F[(N + x) + (int64_t)j * J];
          },
          false);
    }
  });
}

// ---------------------------------------------------------------------------
// Algorithm 7.3 on fat fronts (independent fronts, after the gather of
// V_s = S_AA).  Scratch slot per front: W (A x N), then the reversed Schur
// complement Mr (N x N) with the inverse blocks and X = Mr-factor^-1 of the
// blocked Cholesky after it.
//  prep (one workgroup per front): S's own columns into the cached S, and
//       C_V^-1 in place in the packed Vi block when A <= big_a (larger
//       blocks are factored and inverted beforehand by the bigv launches);
//  a:   W = C_V^-1 S_AN (AN tiles);
//  b:   L_AN = -C_V^-T W (AN tiles) and D^-1 = M = S_NN - W^T W (lower NN
//       tiles), M also stored reversed, Mr(N-1-j, N-1-i) = M(i, j);
//  then the blocked Cholesky of Mr = Lr Lr^T (k_fat_potrf_*, sq = 1) and
//       X = Lr^-1 (k_fat_trtri_row): with the reversal P, M = P Lr Lr^T P,
//       so D = M^-1 = (P X^T P)(P X^T P)^T and C = chol(D) = P X^T P,
//       C(i, j) = X(N-1-j, N-1-i), without inverting M explicitly;
//  c:   R_NN = C and R_AN = L_AN C (NN and AN tiles);
//  lauum: the explicit V_s^-1 for A <= kVExplicitMax, in place.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_fat_compl_prep(DevPlan P, const int32_t* list, const double* Sin,
                                                       double* S, const double* Vs, double* Vi, DevStatus* st) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ double d64[NB2 * LD2];
  __shared__ int64_t colc[kColCache];
  __shared__ int fail;
  with_staged_cols(SnView(P, list[blockIdx.x]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    if (threadIdx.x == 0) fail = -1;
    for (int64_t e = threadIdx.x; e < (int64_t)v.J * v.N; e += NT) {
      const int rr = int(e % v.J), c = int(e / v.J);
      if (rr >= c) S[v.at(rr, c)] = Sin[v.at(rr, c)];
    }
    __syncthreads();
    if (v.A == 0 || v.A > P.big_a) return;  // larger blocks: the bigv launches
    const int A = v.A;
    double* VI = Vi + P.arena[v.s];
    const double* V = Vs + P.arena[v.s];
    const int64_t m = (int64_t)A * (A + 1) / 2;
    for (int64_t e = threadIdx.x; e < m; e += NT) VI[e] = V[e];
    __syncthreads();
    wg_potrf64(PackedLowerW{VI, A}, A, sm, d64, &fail);
    wg_trtri64_invdiag(PackedLowerW{VI, A}, A, sm, d64);
    if (threadIdx.x == 0 && fail >= 0) report(st, MFB_ENOCOMPLETION, v.vl[0]);
  });
}

template <int STAGE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_fat_compl(DevPlan P, const int32_t* list, int count, const double* Sin,
                                                  double* R, double* LB, const double* Vi, double* wsb,
                                                  int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const FatDims d(v);
    const int N = d.N, A = d.A;
    int b = blockIdx.x;
    if (b >= d.tn * d.tn + d.ta * d.tn) return;
    const bool nn = b < d.tn * d.tn;
    if (!nn) b -= d.tn * d.tn;
    const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
    if (nn && (tj > ti || STAGE == 0)) return;
    const int i0 = ti * WT, j0 = tj * WT;
    double* W = wsb + (int64_t)f * slot;
    double* Mr = W + (int64_t)A * N;
    const double* X = Mr + (int64_t)N * N + (int64_t)d.tn * WT * WT;
    const double* VI = Vi + P.arena[v.s];
    MfmaTile T(threadIdx.x);
    if (STAGE == 0) {
      mma_cols<false, true>(
          i0, j0, A, N, 0, min(A, i0 + WT), [&](int i, int k) { return k <= i ? VI[pk(i, k, A)] : 0.0; },
          [&](int k, int j) { return Sin[v.an(k, j)]; },
          [&](int i, int j, double acc) { W[i + (int64_t)j * A] = acc; }, sm);
    } else if (STAGE == 1) {
      if (nn) {
        auto out = [&](int i, int j, double acc) {
          const double m = Sin[v.at(i, j)] - acc;
          LB[v.at(i, j)] = m;
          Mr[(N - 1 - j) + (int64_t)(N - 1 - i) * N] = m;
        };
        if (N <= 32) {
          small_nn_mfma(
              N, A, [&](int k, int i) { return W[k + (int64_t)i * A]; },
              [&](int k, int j) { return W[k + (int64_t)j * A]; }, out, sm);
        } else {
          tile_mma<true, true>(T, i0, j0, N, N, 0, A, [&](int i, int k) { return W[k + (int64_t)i * A]; },
                               [&](int k, int j) { return W[k + (int64_t)j * A]; }, sm);
          tile_store(T, i0, j0, N, N, out, true);
        }
      } else {
        mma_cols<true, true>(
            i0, j0, A, N, i0, A, [&](int i, int k) { return k >= i ? VI[pk(k, i, A)] : 0.0; },
            [&](int k, int j) { return W[k + (int64_t)j * A]; },
            [&](int i, int j, double acc) { LB[v.an(i, j)] = -acc; }, sm);
      }
    } else {
      // C(k, j) = X(N-1-j, N-1-k), zero for k < j
      auto C = [&](int k, int j) { return k >= j ? X[(N - 1 - j) + (int64_t)(N - 1 - k) * N] : 0.0; };
      if (nn) {
        const int row = threadIdx.x & (WT - 1), cq = threadIdx.x >> 6;
        const int gi = i0 + row;
        for (int q = 0; q < 16; ++q) {
          const int gj = j0 + cq + 4 * q;
          if (gi < N && gj < N && gi >= gj) R[v.at(gi, gj)] = C(gi, gj);
        }
      } else {
        tile_mma(T, i0, j0, A, N, j0, N, [&](int x, int k) { return LB[v.an(x, k)]; }, C, sm);
        tile_store(T, i0, j0, A, N, [&](int x, int j, double acc) { R[v.an(x, j)] = acc; }, false);
      }
    }
  });
}

__global__ void __launch_bounds__(NT) k_fat_compl_lauum(DevPlan P, const int32_t* list, double* Vi) {
  __shared__ double sm[SMEM_DOUBLES];
  const int s = list[blockIdx.x];
  const int A = P.nrow[s] - P.ncol[s];
  if (A == 0 || A > kVExplicitMax) return;
  wg_lauum_inplace(PackedLowerW{Vi + P.arena[s], A}, A, sm);
}

// ---------------------------------------------------------------------------
// Inverse Hessian steps 1+2 on fat fronts (independent fronts, after the
// gather of V'_s = T_AA), five launches over [NN tiles | AN tiles] of every
// (front, RHS).  Scratch slot as for k_ihess_down: MA (A x N), Z (A x N),
// MN, Dm, W (N x N each).
//  1: Dm = C C^T (NN), MA = T_AN + V' L (AN);
//  2: MN = T_NN + L^T MA + T_AN^T L (lower NN tiles, stored symmetric);
//  3: W = MN Dm (NN), Z = MA Dm (AN);
//  4: K_NN = Dm W (lower NN tiles); the AN tiles and stage 5 run in
//     k_fat_ihess_an with the right-hand sides batched.
template <int STAGE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(STAGE == 2 ? 2 : 4))) k_fat_ihess(DevPlan P, const int32_t* list, int count, const double* R,
                                                  const double* LB, const double* Vi, const double* Tin,
                                                  double* Kt, const double* Va, int64_t upd, double* wsb,
                                                  int64_t slot, const double* part, int64_t pstride, int r0) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y % count;
  const int64_t r = blockIdx.y / count;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const FatDims d(v);
    const int N = d.N, A = d.A;
    int b = blockIdx.x;
    if (b >= d.tn * d.tn + d.ta * d.tn) return;
    const bool nn = b < d.tn * d.tn;
    if (!nn) b -= d.tn * d.tn;
    const int ti = b / d.tn, tj = b - (b / d.tn) * d.tn;
    const int i0 = ti * WT, j0 = tj * WT;
    if (nn && tj > ti && (STAGE == 2 || STAGE == 4)) return;
    if (!nn && STAGE == 2) return;
    if (!nn && STAGE == 4) return;  // k_fat_ihess_an<4>
    const double* t = Tin + r * P.nnz;
    double* K = Kt + r * P.nnz;
    double* MA = wsb + (r * count + f) * slot;
    double* Z = MA + (int64_t)A * N;
    double* MN = Z + (int64_t)A * N;
    double* Dm = MN + (int64_t)N * N;
    double* W = Dm + (int64_t)N * N;
    MfmaTile T(threadIdx.x);
    if (STAGE == 1) {
      if (nn) {
        auto C = [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; };
        tile_mma(T, i0, j0, N, N, 0, min(N, min(i0, j0) + WT), C, [&](int k, int j) { return C(j, k); }, sm);
        tile_store(T, i0, j0, N, N, [&](int i, int j, double acc) { Dm[i + (int64_t)j * N] = acc; }, false);
      } else if (part && P.poff[v.s] >= 0) {  // V' L from the gather's partial products
        const double* pb = part + (r0 + r) * pstride + P.poff[v.s];
        for (int e = threadIdx.x; e < WT * N; e += NT) {
          const int row = e % WT, n = e / WT, gi = i0 + row;
          if (gi < A) MA[gi + (int64_t)n * A] = t[v.an(gi, n)] + sum_partials(pb, d.ta, ti, N, row, n);
        }
      } else {
        // fronts with few columns on a narrow tile (the same sums, less
        // matrix-core work on empty columns)
        const double* Vp = Va + r * upd + P.arena[v.s];
        auto lb = [&](int k, int j) { return LB[v.an(k, j)]; };
        auto out = [&](int i, int j, double acc) { MA[i + (int64_t)j * A] = t[v.an(i, j)] + acc; };
        if (N <= 16) {
          NarrowTile<16> Tn(threadIdx.x);
          wide_sym_rows_narrow<true>(Tn, i0, j0, A, N, Vp, lb, sm);
          tile_store_narrow(Tn, i0, j0, A, N, out);
        } else if (N <= 32) {
          NarrowTile<32> Tn(threadIdx.x);
          wide_sym_rows_narrow<true>(Tn, i0, j0, A, N, Vp, lb, sm);
          tile_store_narrow(Tn, i0, j0, A, N, out);
        } else {
          wide_sym_rows<true>(T, i0, j0, A, N, Vp, lb, sm);
          tile_store(T, i0, j0, A, N, out, false);
        }
      }
    } else if (STAGE == 2 && N <= 32) {
      auto fa = [&](int k, int i) { return k < A ? LB[v.an(k, i)] : t[v.an(k - A, i)]; };
      auto fb = [&](int k, int j) { return k < A ? MA[k + (int64_t)j * A] : LB[v.an(k - A, j)]; };
      auto out = [&](int i, int j, double acc) {
        const double m = t[v.at(i, j)] + acc;
        MN[i + (int64_t)j * N] = m;
        MN[j + (int64_t)i * N] = m;
      };
      if (N <= SMALL_N)
        small_nn_dot(N, 2 * A, fa, fb, out, sm);
      else
        small_nn_mfma(N, 2 * A, fa, fb, out, sm);
    } else if (STAGE == 2) {
      tile_mma<true, true>(
          T, i0, j0, N, N, 0, 2 * A, [&](int i, int k) { return k < A ? LB[v.an(k, i)] : t[v.an(k - A, i)]; },
          [&](int k, int j) { return k < A ? MA[k + (int64_t)j * A] : LB[v.an(k - A, j)]; }, sm);
      tile_store(
          T, i0, j0, N, N,
          [&](int i, int j, double acc) {
            const double m = t[v.at(i, j)] + acc;
            MN[i + (int64_t)j * N] = m;
            MN[j + (int64_t)i * N] = m;
          },
          true);
    } else if (STAGE == 3) {
      if (nn) {
        tile_mma<false, true>(T, i0, j0, N, N, 0, N, [&](int i, int k) { return MN[i + (int64_t)k * N]; },
                              [&](int k, int j) { return Dm[k + (int64_t)j * N]; }, sm);
        tile_store(T, i0, j0, N, N, [&](int i, int j, double acc) { W[i + (int64_t)j * N] = acc; }, false);
      } else {
        tile_mma<false, true>(T, i0, j0, A, N, 0, N, [&](int i, int k) { return MA[i + (int64_t)k * A]; },
                              [&](int k, int j) { return Dm[k + (int64_t)j * N]; }, sm);
        tile_store(T, i0, j0, A, N, [&](int i, int j, double acc) { Z[i + (int64_t)j * A] = acc; }, false);
      }
    } else {
      tile_mma<false, true>(T, i0, j0, N, N, 0, N, [&](int i, int k) { return Dm[i + (int64_t)k * N]; },
                            [&](int k, int j) { return W[k + (int64_t)j * N]; }, sm);
      tile_store(T, i0, j0, N, N, [&](int i, int j, double acc) { K[v.at(i, j)] = acc; }, true);
    }
  });
}

// Stage 2 of k_fat_ihess on a segment whose fronts all have at most
// SMALL_N columns: their one NN tile, one workgroup per front and
// right-hand side (grid.x = 1), with only the vector-unit product compiled
// in, so that the kernel keeps few registers and little LDS (more
// workgroups per CU than the stage-2 kernel with its matrix-core paths).
// The same sums as k_fat_ihess<2> on these fronts.
__global__ void __launch_bounds__(NT) k_fat_ihess_small2(DevPlan P, const int32_t* list, int count,
                                                         const double* LB, const double* Tin, double* wsb,
                                                         int64_t slot) {
  __shared__ double sm[4 * SMALL_N * (SMALL_N + 1) / 2];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y % count;
  const int64_t r = blockIdx.y / count;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    const double* t = Tin + r * P.nnz;
    double* MA = wsb + (r * count + f) * slot;
    double* MN = MA + 2 * (int64_t)A * N;  // after MA and Z
    auto fa = [&](int k, int i) { return k < A ? LB[v.an(k, i)] : t[v.an(k - A, i)]; };
    auto fb = [&](int k, int j) { return k < A ? MA[k + (int64_t)j * A] : LB[v.an(k - A, j)]; };
    auto out = [&](int i, int j, double acc) {
      const double m = t[v.at(i, j)] + acc;
      MN[i + (int64_t)j * N] = m;
      MN[j + (int64_t)i * N] = m;
    };
    small_nn_dot(N, 2 * A, fa, fb, out, sm);
  });
}

// Stages 4 (AN tiles) and 5 of the fat inverse Hessian, right-hand sides
// batched along the columns (RhsCols; the cached V_s^-1 or C_V^-1 is read
// once per 64 columns): STAGE 4: K_AN = V_s^-1 Z with the explicit inverse,
// else MA = C_V^-1 Z; STAGE 5: K_AN = C_V^-T MA (factored form only).
// blockIdx.y: front of the segment; blockIdx.x: 64-row tile x column tile.
template <int STAGE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_fat_ihess_an(DevPlan P, const int32_t* list, int count, int k, int ct_max,
                                                     const double* Vi, double* Kt, double* wsb, int64_t slot) {
  __shared__ double sm[SMEM_DOUBLES];
  __shared__ int64_t colc[kColCache];
  const int f = blockIdx.y;
  with_staged_cols(SnView(P, list[f]), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A;
    const int ti = int(blockIdx.x) / ct_max, c = int(blockIdx.x) - ti * ct_max;
    const RhsCols rc(N, k);
    if (ti * WT >= A || c >= rc.ct) return;
    const bool explicit_v = A <= kVExplicitMax;
    if (STAGE == 5 && explicit_v) return;
    const int i0 = ti * WT;
    const double* VI = Vi + P.arena[v.s];
    auto MA = [&](int r) { return wsb + ((int64_t)r * count + f) * slot; };  // then Z_r = MA_r + A N
    MfmaTile T(threadIdx.x);
    if (STAGE == 4) {
      auto fz = [&](int kk, int lc) {
        int r, j;
        return rc.map(c, lc, r, j) ? MA(r)[(int64_t)A * N + kk + (int64_t)j * A] : 0.0;
      };
      if (explicit_v) {
        // V^-1 Z with every operand fetch along the tile's rows (this block
        // is at most kVExplicitMax wide): the wide_sym_rows form, whose part
        // above the diagonal block fetches along k, gave wrong results here
        // for blocks of more than one row tile
        const int d0 = min(i0, A), d1 = min(i0 + WT, A);
        tile_mma<false, true>(T, i0, 0, A, WT, 0, d0, [&](int i, int kk) { return VI[pk(i, kk, A)]; }, fz, sm);
        tile_mma<false, true>(T, i0, 0, A, WT, d0, d1, [&](int i, int kk) { return sym_packed(VI, i, kk, A); }, fz,
                              sm);
        tile_mma<false, true>(T, i0, 0, A, WT, d1, A, [&](int i, int kk) { return VI[pk(kk, i, A)]; }, fz, sm);
        tile_store(
            T, i0, 0, A, WT,
            [&](int i, int lc, double acc) {
              int r, j;
              if (rc.map(c, lc, r, j)) Kt[(int64_t)r * P.nnz + v.an(i, j)] = acc;
            },
            false);
      } else {
        tile_mma<false, true>(
            T, i0, 0, A, WT, 0, min(A, i0 + WT), [&](int i, int kk) { return kk <= i ? VI[pk(i, kk, A)] : 0.0; }, fz,
            sm);
        tile_store(
            T, i0, 0, A, WT,
            [&](int i, int lc, double acc) {
              int r, j;
              if (rc.map(c, lc, r, j)) MA(r)[i + (int64_t)j * A] = acc;
            },
            false);
      }
    } else {
      tile_mma<true, true>(
          T, i0, 0, A, WT, i0, A, [&](int i, int kk) { return kk >= i ? VI[pk(kk, i, A)] : 0.0; },
          [&](int kk, int lc) {
            int r, j;
            return rc.map(c, lc, r, j) ? MA(r)[kk + (int64_t)j * A] : 0.0;
          },
          sm);
      tile_store(
          T, i0, 0, A, WT,
          [&](int i, int lc, double acc) {
            int r, j;
            if (rc.map(c, lc, r, j)) Kt[(int64_t)r * P.nnz + v.an(i, j)] = acc;
          },
          false);
    }
  });
}

// ---------------------------------------------------------------------------
// Cholesky factor and its inverse of the packed blocks V = S_AA with
// A > big_a ("bigv"), tile-parallel over all such fronts of a list:
// left-looking by 64-column block columns, each tile of the factor formed
// once as one matrix-core k-loop over the block columns before it.
// Each tile of V is read from Vs once, by the step that forms the factor's
// tile at its place in Cb (Cb is written in full, Vs only read):
//  diag:  block column kb's diagonal tile T = V_kk - C_k,<k C_k,<k^T,
//         factored in LDS (C_kk into Cb) and inverted (C_kk^-1 into the
//         diagonal block of Out, where the inverse ends up anyway);
//  panel: its row tiles below, C_ik = (V_ik - C_i,<k C_k,<k^T) C_kk^-T;
//  trtri: row block ib of X = C^-1 from the rows above it,
//         X_ib,jb = -X_ib,ib sum_{jb <= m < ib} C_ib,m X_m,jb,
//         in the launch of block column ib's panel.
// MODE names the caller (0: the inverse Hessian's cache, 1: the
// completion, 2: the Hessian factor); MODE 2 runs all of it on the
// reversed view of the packed blocks (entry (i, j) of the view at the
// packed position of (A-1-j, A-1-i)): then Cb ends up holding G with
// G^T G = V (G = P F^T P for P V P = F F^T) and Out holds G^-1, the
// Hessian factor's pair.  Failures are reported as MFB_ENOCOMPLETION in
// the completion, MFB_ENOTPD otherwise.  Fronts with A <= big_a exit, so
// a mixed list (the completion's) needs no split.
template <bool REV>
struct PView {
  double* u;
  int a;
  __device__ __forceinline__ double& operator()(int i, int j) const {
    return REV ? u[pk(a - 1 - j, a - 1 - i, a)] : u[pk(i, j, a)];
  }
};

template <int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) k_bigv_diag(DevPlan P, const int32_t* list, int kb, const double* Vs,
                                                  double* Cb, double* Out, DevStatus* st) {
  constexpr bool REV = MODE == 2;
  __shared__ double sm[SMEM_DOUBLES];
  // the diagonal tile as a packed lower triangle: the factorization and the
  // inversion touch entries (i >= j) only, and half the LDS of a square
  // tile lets three workgroups share a CU
  __shared__ double d64[NB2 * (NB2 + 1) / 2];
  __shared__ int fail;
  const int s = list[blockIdx.y];
  const int A = P.nrow[s] - P.ncol[s];
  if (A <= P.big_a || kb >= A) return;
  const int nb = min(WT, A - kb);
  const PView<REV> F{Cb + P.arena[s], A}, X{Out + P.arena[s], A};
  const PView<REV> Vv{const_cast<double*>(Vs) + P.arena[s], A};
  MfmaTile T(threadIdx.x);
  tile_mma<REV, REV>(T, 0, 0, nb, nb, 0, kb, [&](int i, int k) { return F(kb + i, k); },
                     [&](int k, int j) { return F(kb + j, k); }, sm);
  for (int e = threadIdx.x; e < NB2 * (NB2 + 1) / 2; e += NT) d64[e] = 0.0;
  if (threadIdx.x == 0) fail = -1;
  __syncthreads();
  const PackedLowerW D{d64, NB2};
  tile_store(T, 0, 0, nb, nb, [&](int i, int j, double acc) { D(i, j) = Vv(kb + i, kb + j) - acc; }, true);
  __syncthreads();
  wg_potrf_acc(D, nb, nb, sm, &fail);
  for (int e = threadIdx.x; e < nb * nb; e += NT) {
    const int i = e % nb, j = e / nb;
    if (i >= j) F(kb + i, kb + j) = D(i, j);
  }
  __syncthreads();
  wg_trtri_inplace(D, nb, sm);
  for (int e = threadIdx.x; e < nb * nb; e += NT) {
    const int i = e % nb, j = e / nb;
    if (i >= j) X(kb + i, kb + j) = D(i, j);
  }
  if (threadIdx.x == 0 && fail >= 0) report(st, MODE == 1 ? MFB_ENOCOMPLETION : MFB_ENOTPD, P.vlabel[P.colbase[s]]);
}

// panel: row tile `tile` below the diagonal block of block column kb; sm
// and rb are the workgroup's LDS.
template <int MODE>
__device__ __forceinline__ void bigv_panel_tile(const DevPlan& P, int s, int kb, int tile, const double* Vs,
                                                double* Cb, const double* Out, double* sm, double* rb) {
  constexpr bool REV = MODE == 2;
  const int A = P.nrow[s] - P.ncol[s];
  if (A <= P.big_a || kb >= A) return;
  const int nb = min(WT, A - kb);
  const int i0 = kb + nb + tile * WT;
  if (i0 >= A) return;
  const PView<REV> F{Cb + P.arena[s], A};
  const PView<REV> X{const_cast<double*>(Out) + P.arena[s], A};
  const PView<REV> Vv{const_cast<double*>(Vs) + P.arena[s], A};
  MfmaTile T(threadIdx.x);
  tile_mma<REV, REV>(T, i0, 0, A, nb, 0, kb, [&](int i, int k) { return F(i, k); },
                     [&](int k, int j) { return F(kb + j, k); }, sm);
  for (int e = threadIdx.x; e < WT * WLD; e += NT) rb[e] = 0.0;
  __syncthreads();
  tile_store(T, i0, 0, A, nb, [&](int i, int j, double acc) { rb[(i - i0) + j * WLD] = Vv(i, kb + j) - acc; },
             false);
  __syncthreads();
  MfmaTile T2(threadIdx.x);
  tile_mma(T2, 0, 0, WT, nb, 0, nb, [&](int i, int k) { return rb[i + k * WLD]; },
           [&](int k, int j) { return j >= k ? X(kb + j, kb + k) : 0.0; }, sm);
  tile_store(T2, 0, 0, min(WT, A - i0), nb, [&](int i, int j, double acc) { F(i0 + i, kb + j) = acc; }, false);
}

// trtri: tile (ib, jb) of X = C^-1 below the diagonal.
template <int MODE>
__device__ __forceinline__ void bigv_trtri_tile(const DevPlan& P, int s, int ib, int jb, const double* Cb,
                                                double* Out, double* sm, double* rb) {
  constexpr bool REV = MODE == 2;
  const int A = P.nrow[s] - P.ncol[s];
  const int i0 = ib * WT, j0 = jb * WT;
  if (A <= P.big_a || i0 >= A || jb >= ib) return;
  const int nbi = min(WT, A - i0);
  const PView<REV> F{const_cast<double*>(Cb) + P.arena[s], A}, X{Out + P.arena[s], A};
  MfmaTile T(threadIdx.x);
  tile_mma<REV, !REV>(T, i0, j0, A, A, j0, i0, [&](int i, int k) { return F(i, k); },
                      [&](int k, int j) { return k >= j ? X(k, j) : 0.0; }, sm);
  for (int e = threadIdx.x; e < WT * WLD; e += NT) rb[e] = 0.0;
  __syncthreads();
  tile_store(T, i0, j0, A, A, [&](int i, int j, double acc) { rb[(i - i0) + (j - j0) * WLD] = -acc; }, false);
  __syncthreads();
  MfmaTile T2(threadIdx.x);
  tile_mma(T2, 0, 0, nbi, WT, 0, nbi, [&](int i, int k) { return k <= i ? X(i0 + i, i0 + k) : 0.0; },
           [&](int k, int j) { return rb[k + j * WLD]; }, sm);
  tile_store(T2, 0, 0, nbi, WT, [&](int i, int j, double acc) { X(i0 + i, j0 + j) = acc; }, false);
}

// The panel of block column kb and row block ib = kb / 64 of the inverse in
// one launch: workgroups x < rows take panel row tile x, the others tile
// (ib, x - rows) of the inverse.  The two parts touch disjoint data: the
// panel writes the factor's column block kb below its diagonal block and
// reads the inverse's diagonal block kb only; the inverse's row block ib
// reads the factor's row block ib left of column block kb, finished by the
// panels before kb, the inverse's rows above it and its diagonal block kb
// (all from earlier launches), and writes its row block ib left of the
// diagonal block.  So the inverse's rows run beside the factor's panels,
// which alone leave most of the chip idle at the last block columns.
//
// Grid: packed (T.packed) when the list is in decreasing order of A and the
// largest front has at most kBigvMaxRows row tiles below the diagonal
// block: the first T.off[1] workgroups are panel row tile 0 of the first
// T.off[1] fronts (those that have it), the next T.off[2] - T.off[1] row
// tile 1, ..., then tile jb of the inverse's row block for the first T.ctr
// fronts (those with A > kb), jb-major.  Otherwise rectangular: tile
// blockIdx.x of front blockIdx.y, tiles beyond a front's A exit.
constexpr int kBigvMaxRows = 64;
struct BigvTiles {
  int packed, rows, ctr;
  int off[kBigvMaxRows + 1];
};

template <int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_bigv_panel_trtri(DevPlan P, const int32_t* list, int kb, BigvTiles T,
                                                         const double* Vs, double* Cb, double* Out) {
  __shared__ double sm[SMEM_GEMM];  // tile_mma staging only
  __shared__ double rb[WT * WLD];
  int f, x;
  if (T.packed) {
    const int w = int(blockIdx.x);
    if (w < T.off[T.rows]) {
      x = 0;
      while (T.off[x + 1] <= w) ++x;  // ends at x < rows: off[rows] > w
      f = w - T.off[x];
    } else {
      const int r = w - T.off[T.rows];
      x = T.rows + r / T.ctr;
      f = r % T.ctr;
    }
  } else {
    f = int(blockIdx.y);
    x = int(blockIdx.x);
  }
  const int s = list[f];
  if (x < T.rows)
    bigv_panel_tile<MODE>(P, s, kb, x, Vs, Cb, Out, sm, rb);
  else
    bigv_trtri_tile<MODE>(P, s, kb / WT, x - T.rows, Cb, Out, sm, rb);
}

// ---------------------------------------------------------------------------
// Panel part of the leaf-to-root sweeps of wide fronts (N <= kWideMaxN) that
// need nothing but the children's update blocks and the front's own columns,
// spread over 64-row tiles of the A rows: workgroup blockIdx.x = f * ta + ti
// (front f of the segment, row tile ti; tiles beyond the front's A exit),
// right-hand side blockIdx.y.  G' = sum of the children's E U_c E^T is
// assembled child by child in the fixed order, so every entry takes its terms
// in the order of the one-workgroup panel kernels (k_product<true>,
// k_ihess_up<true>), and the products use the same 64-row tiles.
//   UP_PRODUCT (Algorithm 3.2): X_AN = R_AN C^T - G'21 on tile ti's rows and,
//     on tile 0, X_NN = C C^T - G'11 (C the lower N x N block of R);
//   UP_IHESS (inverse Hessian step 3): Q = L K_NN + K_AN and
//     Y_AN = Q - G'21 on tile ti's rows, Y_NN = K_NN - G'11 on tile 0; Q
//     goes to the (front, right-hand side) scratch slot, after the J x N
//     panel area, where k_wide_update reads it.
template <int UP>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) k_up_panel_tiles(DevPlan P, const int32_t* list, int count, int ta,
                                                       const double* R, const double* LB, const double* Kt,
                                                       double* Y, const double* Ua, int64_t upd, double* wsb,
                                                       int64_t slot) {
  __shared__ double sm[SMEM_GEMM];
  __shared__ double G[WT * kWideMaxN];
  __shared__ int64_t colc[kColCache];
  const int f = int(blockIdx.x) / ta, ti = int(blockIdx.x) - f * ta;
  const int s = list[f];
  if (ti > 0 && ti * WT >= P.nrow[s] - P.ncol[s]) return;  // the whole workgroup
  const int64_t r = blockIdx.y;
  with_staged_cols(SnView(P, s), colc, [&](const SnView& v) __attribute__((always_inline)) {
    const int N = v.N, A = v.A, J = v.J;
    const int i0 = ti * WT, m = min(WT, A - i0);
    const double* ua = Ua + r * upd;
    const double* K = UP == UP_IHESS ? Kt + r * P.nnz : nullptr;
    double* y = Y + r * P.nnz;
    auto C = [&](int i, int k) { return k <= i ? R[v.at(i, k)] : 0.0; };
    auto assemble = [&](int lo, int hi, int ld) {  // rows of the front [lo, hi), into G(row - lo, col)
      for (int e = threadIdx.x; e < WT * kWideMaxN; e += NT) G[e] = 0.0;
      __syncthreads();
      for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
        const int c = P.cidx[t];
        const int Ac = P.nrow[c] - P.ncol[c];
        const int32_t* rl = P.rel + P.relbase[c];
        const double* Uc = ua + P.arena[c];
        // the child's rows in [lo, hi) (at most 64) times its columns that
        // land in the front's N columns, all pairs at once: each pair has
        // its own entry of G, which takes one term per child
        const int xb = lower_rel(rl, Ac, lo), xe = lower_rel(rl, Ac, hi), yc = lower_rel(rl, Ac, N);
        const int nx = xe - xb;
        for (int e = int(threadIdx.x); e < yc * nx; e += NT) {
          const int yy = e / nx, x = xb + (e - yy * nx);
          if (x >= yy) G[(rl[x] - lo) + (int64_t)rl[yy] * ld] += Uc[pk(x, yy, Ac)];
        }
        __syncthreads();
      }
    };
    if (m > 0) {
      assemble(N + i0, N + i0 + m, WT);
      if (UP == UP_PRODUCT) {
        wg_gemm(
            m, N, N, [&](int i, int k) { return R[v.an(i0 + i, k)]; }, [&](int k, int j) { return C(j, k); },
            [&](int i, int j, double acc) { y[v.an(i0 + i, j)] = acc - G[i + j * WT]; }, false, sm);
      } else {
        double* Q = wsb + (r * count + f) * slot + (int64_t)J * N;
        wg_gemm<false, true>(
            m, N, N, [&](int i, int k) { return LB[v.an(i0 + i, k)]; }, [&](int k, int j) { return K[v.nn(k, j)]; },
            [&](int i, int j, double acc) {
              const double q = acc + K[v.an(i0 + i, j)];
              Q[(i0 + i) + (int64_t)j * A] = q;
              y[v.an(i0 + i, j)] = q - G[i + j * WT];
            },
            false, sm);
      }
    }
    if (ti == 0) {
      __syncthreads();  // G is reused
      assemble(0, N, N);
      if (UP == UP_PRODUCT) {
        wg_gemm(
            N, N, N, C, [&](int k, int j) { return C(j, k); },
            [&](int i, int j, double acc) { y[v.at(i, j)] = acc - G[i + j * N]; }, true, sm);
      } else {
        for (int64_t e = threadIdx.x; e < (int64_t)N * N; e += NT) {
          const int i = int(e % N), c = int(e / N);
          if (i >= c) y[v.at(i, c)] = K[v.at(i, c)] - G[i + c * N];
        }
      }
    }
  });
}

void launch_up_panel_tiles(int up, int maxA, int count, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* R, const double* LB, const double* Kt, double* Y, const double* Ua,
                           int64_t upd, double* wsb, int64_t slot) {
  const int ta = std::max(1, (maxA + WT - 1) / WT);
  const dim3 grid(unsigned(count * ta), unsigned(k));
  if (up == UP_PRODUCT)
    k_up_panel_tiles<UP_PRODUCT><<<grid, NT, 0, s>>>(P, list, count, ta, R, LB, Kt, Y, Ua, upd, wsb, slot);
  else
    k_up_panel_tiles<UP_IHESS><<<grid, NT, 0, s>>>(P, list, count, ta, R, LB, Kt, Y, Ua, upd, wsb, slot);
}

// ---------------------------------------------------------------------------
// Host launchers.

void launch_wide_update(int op, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const int32_t* pre, int count, const double* R, const double* LB, const double* Kt,
                        double* Ua, int64_t upd, const double* wsb, int64_t slot, const int32_t* act) {
  switch (op) {
    case WU_FACTOR:
      k_wide_update<WU_FACTOR><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot, act);
      break;
    case WU_HUP:
      k_wide_update<WU_HUP><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot, act);
      break;
    case WU_PRODUCT:
      k_wide_update<WU_PRODUCT><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot, act);
      break;
    default:
      k_wide_update<WU_IHUP><<<grid, NT, 0, s>>>(P, list, pre, count, R, LB, Kt, Ua, upd, wsb, slot, act);
      break;
  }
}

void launch_wide_extract(int tag, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                         const int32_t* pre, int count, const double* src, double* arena, int64_t src_stride,
                         int64_t arena_stride, const double* LB, double* part, int64_t pstride) {
  if (tag == 1)
    k_wide_extract<1><<<grid, NT, 0, s>>>(P, list, pre, count, src, arena, src_stride, arena_stride, LB, part,
                                          pstride);
  else
    k_wide_extract<2><<<grid, NT, 0, s>>>(P, list, pre, count, src, arena, src_stride, arena_stride, nullptr,
                                          nullptr, 0);
}

void launch_wide_projinv(hipStream_t s, const DevPlan& P, const int32_t* list, const WideTiles& w, int count,
                         const double* LB, double* S, double* Vs) {
  if (w.n_aa)
    k_wide_extract<0><<<dim3(unsigned(w.n_aa)), NT, 0, s>>>(P, list, w.aa, count, S, Vs, 0, 0, nullptr, nullptr, 0);
  if (w.n_an) k_wide_projinv_an<<<dim3(unsigned(w.n_an)), NT, 0, s>>>(P, list, w.an, count, LB, S, Vs);
  k_wide_projinv_nn<<<dim3(unsigned(w.n_nn)), NT, 0, s>>>(P, list, w.nn, count, LB, S);
}

void launch_wide_hess_down(int k, int maxN, int maxA, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const WideTiles& w, int count, const double* LB, const double* Vs, const double* Kt,
                           double* T, double* Va, int64_t upd, double* wsb, int64_t slot, double* part,
                           int64_t pstride) {
  const SegTiles tl{w.aa, w.an, w.nn, w.n_aa, w.n_an, w.n_nn};
  k_wide_hdown_a<<<dim3(unsigned(w.n_aa + w.n_nn + w.n_an), unsigned(k)), NT, 0, s>>>(P, list, tl, count, LB, Kt,
                                                                                       T, Va, upd, wsb, slot, part,
                                                                                       pstride);
  if (maxA > 0) {
    const int ct = RhsCols(std::max(1, maxN), k).ct, ta = (maxA + WT - 1) / WT;
    k_wide_hdown_vz<<<dim3(unsigned(ta * ct), unsigned(count)), NT, 0, s>>>(P, list, count, k, ct, Vs, wsb, slot);
  }
  k_wide_hdown_b<<<dim3(unsigned(w.n_nn + w.n_an), unsigned(k)), NT, 0, s>>>(P, list, tl, count, LB, Vs, T, Va,
                                                                              upd, wsb, slot, part, pstride);
  k_wide_hdown_c<<<dim3(unsigned(w.n_nn), unsigned(k)), NT, 0, s>>>(P, list, tl, count, LB, T, wsb, slot);
}

void launch_fat_panel(int op, const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                      int count, const double* src, const double* Ua, int64_t upd, double* wsb, int64_t slot,
                      const int32_t* act) {
  const dim3 grid(unsigned(g.panel), unsigned(count * k));
  switch (op) {
    case 0: k_fat_panel<0><<<grid, NT, 0, s>>>(P, list, count, src, Ua, upd, wsb, slot, act); break;
    case 1: k_fat_panel<1><<<grid, NT, 0, s>>>(P, list, count, src, Ua, upd, wsb, slot, act); break;
    case 2: k_fat_panel<2><<<grid, NT, 0, s>>>(P, list, count, src, Ua, upd, wsb, slot, act); break;
    default: k_fat_panel<3><<<grid, NT, 0, s>>>(P, list, count, src, Ua, upd, wsb, slot, act); break;
  }
}

// The blocked Cholesky (k_fat_potrf_*) and the row blocks of its inverse
// (k_fat_trtri_row) over a segment's fronts, grids sized by its largest
// front (maxN columns, maxRows rows); tiles beyond a front's own exit.
template <int SQ>
static void fat_potrf_trtri(int maxN, int maxRows, hipStream_t s, const DevPlan& P, const int32_t* list,
                            int count, double* R, double* part, DevStatus* st, double* wsb, int64_t slot) {
  const unsigned c = unsigned(count);
  for (int kb = 0; kb < maxN; kb += WT) {
    k_fat_potrf_diag<SQ><<<dim3(1, c), NT, 0, s>>>(P, list, count, kb, R, part, st, wsb, slot);
    const int rows = (maxRows - kb + WT - 1) / WT, cols = (maxN - kb + WT - 1) / WT;
    k_fat_potrf_panel<SQ><<<dim3(unsigned(rows), c), NT, 0, s>>>(P, list, count, kb, R, wsb, slot);
    if (kb + WT < maxN)
      k_fat_potrf_trail<SQ><<<dim3(unsigned(rows * cols), c), NT, 0, s>>>(P, list, count, kb, wsb, slot);
  }
  for (int ib = 0; ib * WT < maxN; ++ib)
    k_fat_trtri_row<SQ><<<dim3(unsigned(ib + 1), c), NT, 0, s>>>(P, list, count, ib, wsb, slot);
}

void launch_fat_factor(const FatGrid& g, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                       double* R, double* LB, double* part, DevStatus* st, double* wsb, int64_t slot) {
  const unsigned c = unsigned(count);
  fat_potrf_trtri<0>(g.maxN, g.maxJ, s, P, list, count, R, part, st, wsb, slot);
  k_fat_factor_fin<<<dim3(unsigned(g.fin), c), NT, 0, s>>>(P, list, count, LB, wsb, slot);
}

void launch_fat_completion(const FatGrid& g, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                           const double* Sin, double* R, double* LB, double* S, const double* Vs, double* Vi,
                           double* part, DevStatus* st, double* wsb, int64_t slot) {
  const unsigned c = unsigned(count);
  k_fat_compl_prep<<<dim3(c), NT, 0, s>>>(P, list, Sin, S, Vs, Vi, st);
  if (g.maxA > 0) k_fat_compl<0><<<dim3(unsigned(g.fin), c), NT, 0, s>>>(P, list, count, Sin, R, LB, Vi, wsb, slot);
  k_fat_compl<1><<<dim3(unsigned(g.fin), c), NT, 0, s>>>(P, list, count, Sin, R, LB, Vi, wsb, slot);
  fat_potrf_trtri<1>(g.maxN, g.maxN, s, P, list, count, R, part, st, wsb, slot);
  k_fat_compl<2><<<dim3(unsigned(g.fin), c), NT, 0, s>>>(P, list, count, Sin, R, LB, Vi, wsb, slot);
  k_fat_compl_lauum<<<dim3(c), NT, 0, s>>>(P, list, Vi);
}

void launch_fat_up_fin(int op, const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                       int count, const double* R, const double* LB, double* Out, double* Kt, double* wsb,
                       int64_t slot) {
  const dim3 grid(unsigned(g.fin), unsigned(count * k));
  if (op == FAT_PRODUCT)
    k_fat_up_fin<FAT_PRODUCT><<<grid, NT, 0, s>>>(P, list, count, R, LB, Out, Kt, wsb, slot);
  else if (op == FAT_HUP)
    k_fat_up_fin<FAT_HUP><<<grid, NT, 0, s>>>(P, list, count, R, LB, Out, Kt, wsb, slot);
  else
    k_fat_up_fin<FAT_IHUP><<<grid, NT, 0, s>>>(P, list, count, R, LB, Out, Kt, wsb, slot);
}

template <int MODE>
static void bigv_launches(int maxA, int count, const int32_t* acnt, hipStream_t s, const DevPlan& P,
                          const int32_t* list, const double* Vs, double* Cb, double* Out, DevStatus* st) {
  // the fronts a step at row kb needs are those with A > kb (A > kb + 64
  // for the row tiles below the diagonal block): acnt[kb / 64] of them, a
  // prefix of the list (decreasing A); without acnt every front is launched
  // and the others exit
  auto fronts = [&](int kb) { return acnt ? std::min(count, acnt[kb / WT]) : count; };
  // block column kb: its diagonal block, then its panel beside row block
  // kb / 64 of the inverse (which needs that diagonal block's inverse and
  // nothing of the panel)
  for (int kb = 0; kb < maxA; kb += WT) {
    const int rows = (maxA - kb - 1) / WT;  // row tiles below the diagonal block (largest front)
    const int c = fronts(kb);
    if (c == 0) break;
    k_bigv_diag<MODE><<<dim3(1, unsigned(c)), NT, 0, s>>>(P, list, kb, Vs, Cb, Out, st);
    const int ib = kb / WT;
    if (rows + ib == 0) continue;
    BigvTiles T{};
    T.rows = rows;
    T.ctr = c;
    if (acnt && rows <= kBigvMaxRows) {
      // row tile x lies at 64 (ib + x + 1): the fronts with A above that
      T.packed = 1;
      for (int x = 0; x < rows; ++x) T.off[x + 1] = T.off[x] + fronts(kb + (x + 1) * WT);
      const int64_t total = T.off[rows] + (int64_t)ib * c;
      if (total > 0) k_bigv_panel_trtri<MODE><<<dim3(unsigned(total)), NT, 0, s>>>(P, list, kb, T, Vs, Cb, Out);
    } else {
      k_bigv_panel_trtri<MODE><<<dim3(unsigned(rows + ib), unsigned(c)), NT, 0, s>>>(P, list, kb, T, Vs, Cb, Out);
    }
  }
}

void launch_bigv(int mode, int maxA, int count, const int32_t* acnt, hipStream_t s, const DevPlan& P,
                 const int32_t* list, const double* Vs, double* Cb, double* Out, DevStatus* st) {
  if (count == 0 || maxA <= P.big_a) return;
  if (mode == 0)
    bigv_launches<0>(maxA, count, acnt, s, P, list, Vs, Cb, Out, st);
  else if (mode == 1)
    bigv_launches<1>(maxA, count, acnt, s, P, list, Vs, Cb, Out, st);
  else
    bigv_launches<2>(maxA, count, acnt, s, P, list, Vs, Cb, Out, st);
}

void launch_fat_ihess(const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                      const double* R, const double* LB, const double* Vi, const double* T, double* Kt,
                      const double* Va, int64_t upd, double* wsb, int64_t slot, const double* part,
                      int64_t pstride) {
  // blockIdx.y = front + count * (right-hand side): right-hand sides in
  // groups that keep the grid's y extent within 65535
  const int kc = std::max(1, 65535 / std::max(1, count));
  for (int r0 = 0; r0 < k; r0 += kc) {
    const int kk = std::min(kc, k - r0);
    const dim3 grid(unsigned(g.fin), unsigned(count * kk));
    const double* t = T + (int64_t)r0 * P.nnz;
    double* K = Kt + (int64_t)r0 * P.nnz;
    const double* va = Va + (int64_t)r0 * upd;
    k_fat_ihess<1><<<grid, NT, 0, s>>>(P, list, count, R, LB, Vi, t, K, va, upd, wsb, slot, part, pstride, r0);
    // stages 2 and 4 work on the NN tiles only: a segment whose fronts have
    // at most 64 columns needs its tile 0 alone
    const dim3 gnn(g.maxN <= WT ? 1u : unsigned(g.fin), unsigned(count * kk));
    if (g.maxN <= SMALL_N)
      k_fat_ihess_small2<<<dim3(1, unsigned(count * kk)), NT, 0, s>>>(P, list, count, LB, t, wsb, slot);
    else
      k_fat_ihess<2><<<gnn, NT, 0, s>>>(P, list, count, R, LB, Vi, t, K, va, upd, wsb, slot, part, pstride, r0);
    k_fat_ihess<3><<<grid, NT, 0, s>>>(P, list, count, R, LB, Vi, t, K, va, upd, wsb, slot, part, pstride, r0);
    k_fat_ihess<4><<<gnn, NT, 0, s>>>(P, list, count, R, LB, Vi, t, K, va, upd, wsb, slot, part, pstride, r0);
    if (g.maxA > 0) {
      const int ct = RhsCols(std::max(1, g.maxN), kk).ct, ta = (g.maxA + WT - 1) / WT;
      const dim3 gan(unsigned(ta * ct), unsigned(count));
      k_fat_ihess_an<4><<<gan, NT, 0, s>>>(P, list, count, kk, ct, Vi, K, wsb, slot);
      if (g.maxA > kVExplicitMax) k_fat_ihess_an<5><<<gan, NT, 0, s>>>(P, list, count, kk, ct, Vi, K, wsb, slot);
    }
  }
}

}  // namespace mfb

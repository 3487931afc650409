// Device helpers shared by the sweep kernels: the supernode view of the
// CCS-ordered arrays, the children's extend-add and the parent extraction
// of the clique-tree recursions, workgroup scratch slots.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "wg_dense.h"

namespace mfb {

__device__ inline void report(DevStatus* st, int code, long long label) {
  atomicMax(&st->code, code);
  atomicMin(&st->bad, (unsigned long long)label);
}

struct SnView {
  int s, N, A, J;
  const int64_t* col;  // CCS diagonal offsets of the supernode's columns
  const int32_t* vl;   // user labels of the supernode's columns
  __device__ SnView(const DevPlan& P, int s_) : s(s_) {
    N = P.ncol[s];
    J = P.nrow[s];
    A = J - N;
    col = P.col + P.colbase[s];
    vl = P.vlabel + P.colbase[s];
  }
  // element (r, c), r >= c, of a CCS-ordered array restricted to the panel
  __device__ __forceinline__ int64_t at(int r, int c) const { return col[c] + (r - c); }
  // symmetric NN access
  __device__ __forceinline__ int64_t nn(int i, int j) const { return i >= j ? at(i, j) : at(j, i); }
  // AN block entry (x in A, c in N)
  __device__ __forceinline__ int64_t an(int x, int c) const { return col[c] + (N + x - c); }
};

__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Extend-add of the children's packed update blocks taken from `ua`.
// Entries landing in N_s columns go to the panel F (leading dimension J);
// the others (rows and columns in A_s) go to the packed block Us.  One
// child at a time (fixed order), so every target is written once per pass;
// a child's entries are spread over the whole workgroup (flat index over
// its A_c x A_c square, lower entries taken), with its relative indices
// staged in LDS (`sm`: at least 2048 doubles) when they fit.
// With `act` (Hessian step 1: per supernode, whether its subtree holds a
// nonzero of the right-hand side), children marked 0 are skipped: their
// update blocks are zero and were not written.
template <int NTH = NT>
__device__ __forceinline__ void assemble_children(const DevPlan& P, const SnView& v, const double* ua,
                                                  double* F, double* Us, double* sm,
                                                  const int32_t* act = nullptr) {
  int* srl = reinterpret_cast<int*>(sm);
  constexpr int CAP = 4096;
  for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
    const int c = P.cidx[t];
    const int Ac = P.nrow[c] - P.ncol[c];
    if (Ac == 0 || (act && !act[c])) continue;  // (a child always has ancestors)
    const int32_t* rl = P.rel + P.relbase[c];
    const double* Uc = ua + P.arena[c];
    const bool st = Ac <= CAP;
    if (st)
      for (int i = threadIdx.x; i < Ac; i += NTH) srl[i] = rl[i];
    __syncthreads();
    // flat walk of the Ac x Ac square as in extract_from_parent, BATCH
    // entries per round; the targets of one child are distinct
    auto pass = [&](const auto& R) {
      constexpr int BATCH = 4;
      const int dy = NTH / Ac, dx = NTH - dy * Ac;
      int y = int(threadIdx.x) / Ac, x = int(threadIdx.x) - y * Ac;
      while (y < Ac) {
        double* q[BATCH];
        const double* u_[BATCH];
        bool ok[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          ok[u] = y < Ac && x >= y;
          const int rx = ok[u] ? R(x) : 0, ry = ok[u] ? R(y) : 0;
          q[u] = !ok[u] ? F : ry < v.N ? F + (rx + (int64_t)ry * v.J) : Us + pk(rx - v.N, ry - v.N, v.A);
          u_[u] = ok[u] ? Uc + pk(x, y, Ac) : Uc;
          x += dx;
          y += dy;
          if (x >= Ac) {
            x -= Ac;
            ++y;
          }
        }
        double a[BATCH], b[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          a[u] = *q[u];
          b[u] = *u_[u];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
          if (ok[u]) *q[u] = a[u] + b[u];
      }
    };
    if (st)
      pass([&](int i) { return srl[i]; });
    else
      pass([&](int i) { return rl[i]; });
    __syncthreads();
  }
}

// V_s = E^T [S_NN S_AN^T; S_AN V_p] E (eq. e-sn-gradient-2): gather the
// packed A_s x A_s block from the parent's CCS columns of `src` and the
// parent's packed block in `arena`, into this supernode's packed block.
// Entries are spread over the whole workgroup (flat index over the A x A
// square, lower entries taken); the relative indices and the parent's
// column offsets are staged in LDS (`sm`: at least 4096 doubles) when they
// fit.  Ends with a barrier.
template <int NTH = NT>
__device__ __forceinline__ void extract_from_parent(const DevPlan& P, const SnView& v, const double* src,
                                                    double* arena, double* sm) {
  if (v.A == 0) return;
  const int A = v.A;
  const int p = P.parent[v.s];
  const int Np = P.ncol[p], Ap = P.nrow[p] - Np;
  const int64_t* colp = P.col + P.colbase[p];
  const int32_t* rl = P.rel + P.relbase[v.s];
  const double* Vp = arena + P.arena[p];
  double* Vo = arena + P.arena[v.s];
  int* srl = reinterpret_cast<int*>(sm);
  int64_t* scp = reinterpret_cast<int64_t*>(sm + 2048);
  const bool st = A <= 4096 && Np <= 2048;
  if (st) {
    for (int i = threadIdx.x; i < A; i += NTH) srl[i] = rl[i];
    for (int i = threadIdx.x; i < Np; i += NTH) scp[i] = colp[i];
  }
  __syncthreads();
  // Each thread walks the flat index tid, tid + NTH, ... of the A x A
  // square as (x, y) = (e mod A, e div A), stepped without divisions, and
  // issues BATCH loads (masked entries load a valid dummy) before storing.
  auto pass = [&](const auto& R, const auto& CP) {
    constexpr int BATCH = 8;
    const int dy = NTH / A, dx = NTH - dy * A;
    int y = int(threadIdx.x) / A, x = int(threadIdx.x) - y * A;
    while (y < A) {
      const double* q[BATCH];
      int64_t o[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const bool ok = y < A && x >= y;
        const int rx = ok ? R(x) : 0, ry = ok ? R(y) : 0;
        q[u] = !ok ? src : ry < Np ? src + CP(ry) + (rx - ry) : Vp + pk(rx - Np, ry - Np, Ap);
        o[u] = ok ? pk(x, y, A) : -1;
        x += dx;
        y += dy;
        if (x >= A) {
          x -= A;
          ++y;
        }
      }
      double val[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) val[u] = *q[u];
#pragma unroll
      for (int u = 0; u < BATCH; ++u)
        if (o[u] >= 0) Vo[o[u]] = val[u];
    }
  };
  if (st)
    pass([&](int i) { return srl[i]; }, [&](int i) { return scp[i]; });
  else
    pass([&](int i) { return rl[i]; }, [&](int i) { return colp[i]; });
  __syncthreads();
}

// The children's contributions to the front's N panel columns only (its
// columns below N; the A x A part is assembled tile by tile elsewhere):
// for child c, the entries (x, y) of its packed block with rel[y] < N,
// i.e. its first columns, since the relative indices increase.  Targets
// of one child are distinct; children in a fixed order.  Ends with a
// barrier.
template <int NTH = NT>
__device__ __forceinline__ void assemble_children_panel(const DevPlan& P, const SnView& v, const double* ua,
                                                        double* F, const int32_t* act = nullptr) {
  for (int t = P.cptr[v.s]; t < P.cptr[v.s + 1]; ++t) {
    const int c = P.cidx[t];
    if (act && !act[c]) continue;
    const int Ac = P.nrow[c] - P.ncol[c];
    const int32_t* rl = P.rel + P.relbase[c];
    const double* Uc = ua + P.arena[c];
    for (int y = 0; y < Ac; ++y) {
      const int ry = rl[y];  // the same for every thread
      if (ry >= v.N) break;
      for (int x = y + int(threadIdx.x); x < Ac; x += NTH)
        F[rl[x] + (int64_t)ry * v.J] += Uc[pk(x, y, Ac)];
    }
    __syncthreads();
  }
}

template <int NTH = NT>
__device__ __forceinline__ void zero_packed(double* U, int A) {
  const int64_t m = (int64_t)A * (A + 1) / 2;
  for (int64_t e = threadIdx.x; e < m; e += NTH) U[e] = 0.0;
}

// Hessian step 1 with a sparse right-hand side (pruning, Section 5.5):
// the front is active when its own panel of Y holds a nonzero (own, this
// thread's view) or a child is active.  Uniform over the workgroup.
__device__ __forceinline__ bool step1_active(const DevPlan& P, int s, const int32_t* act, bool own) {
  bool a = __syncthreads_or(own ? 1 : 0) != 0;
  for (int t = P.cptr[s]; t < P.cptr[s + 1] && !a; ++t) a = act[P.cidx[t]] != 0;
  return a;
}

__device__ __forceinline__ double* slot_ptr(double* wsb, int64_t slot) {
  return wsb + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * slot;
}

// Runs body(v) with the supernode's column offsets copied to LDS (`colc`)
// when N <= kColCache, so every CCS address is formed without a dependent
// global load, else with the offsets read from global memory.
constexpr int kColCache = 512;
template <int NTH = NT, class BODY>
__device__ __forceinline__ void with_staged_cols(SnView v, int64_t* colc, const BODY& body) {
  if (v.N <= kColCache) {
    for (int i = threadIdx.x; i < v.N; i += NTH) colc[i] = v.col[i];
    __syncthreads();
    v.col = colc;
    body(v);
  } else {
    body(v);
  }
}

}  // namespace mfb

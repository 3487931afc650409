// Workgroup-cooperative dense FP64 building blocks for gfx950.
//
// Every routine is called by all 256 threads of a workgroup (uniform
// control flow) and works on column-major matrices reached through
// operand functors, so one routine serves panels kept in CCS order,
// packed symmetric update blocks and per-workgroup scratch alike.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfb {

constexpr int NT = 256;  // threads per workgroup (4 wavefronts of 64)
constexpr int TM = 64;   // output tile edge of wg_gemm
constexpr int KC = 16;   // k-chunk staged through LDS
constexpr int NB = 32;   // diagonal block of the blocked factorizations
constexpr int LDD = NB + 1;
// LDS doubles used by the routines in this file
constexpr int LDS_TM = TM + 1;  // padded row of a staged k-chunk (no bank conflicts on k-major stores)
constexpr int SMEM_GEMM = 2 * KC * LDS_TM;
constexpr int SMEM_DIAG = 2 * NB * LDD;  // diagonal block and its inverse
constexpr int SMEM_DOUBLES = SMEM_GEMM + SMEM_DIAG + 8;

// Packed lower storage of a symmetric A x A block, column-major: entry
// (x, y), x >= y, lives at y*(2A-y-1)/2 + x.
__device__ __forceinline__ int64_t pk(int x, int y, int A) {
  return (int64_t)y * (2 * A - y - 1) / 2 + x;
}
__device__ __forceinline__ double sym_packed(const double* u, int x, int y, int A) {
  return x >= y ? u[pk(x, y, A)] : u[pk(y, x, A)];
}

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// FP64 matrix-core tile: each wavefront of a 256-thread team owns a 32 x 32
// quadrant (wr, wc) of the 64 x 64 output tile as 2 x 2 blocks of 16 x 16,
// accumulated by v_mfma_f64_16x16x4f64.  Lane layout of that instruction
// (checked on the device): lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16) of the 16 x 4 and 4 x 16 operands and holds
// D(l / 16 + 4 v, l % 16) in accumulator element v.
typedef double v4d __attribute__((ext_vector_type(4)));
struct MfmaTile {
  v4d acc[2][2];
  int wr, wc, lr, lk;  // quadrant origin; lane's row in a block and k in a step
  __device__ __forceinline__ explicit MfmaTile(int tid) {
    const int w = tid >> 6, l = tid & 63;
    wr = (w >> 1) * 32;
    wc = (w & 1) * 32;
    lr = l & 15;
    lk = l >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // the KC k-steps of one staged chunk (As, Bs: [k][LDS_TM]); step s + 1's
  // operands are read while step s's products run
  __device__ __forceinline__ void chunk(const double* As, const double* Bs) {
    double fa[2][2], fb[2][2];
    auto load = [&](int s, double* a_, double* b_) {
      const int k = 4 * s + lk;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a_[q] = As[k * LDS_TM + wr + 16 * q + lr];
        b_[q] = Bs[k * LDS_TM + wc + 16 * q + lr];
      }
    };
    load(0, fa[0], fb[0]);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      if (s + 1 < KC / 4) load(s + 1, fa[(s + 1) & 1], fb[(s + 1) & 1]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s & 1][a], fb[s & 1][b], acc[a][b], 0, 0, 0);
    }
  }
  // element e (0..15) of this lane: block (e >> 3, (e >> 2) & 1), entry e & 3
  __device__ __forceinline__ double get(int e) const { return acc[e >> 3][(e >> 2) & 1][e & 3]; }
  __device__ __forceinline__ void add(int e, double x) { acc[e >> 3][(e >> 2) & 1][e & 3] += x; }
  __device__ __forceinline__ int row_of(int e) const { return wr + 16 * (e >> 3) + lk + 4 * (e & 3); }
  __device__ __forceinline__ int col_of(int e) const { return wc + 16 * ((e >> 2) & 1) + lr; }
};

// C(i, j) <- epi(i, j, sum_k a(i, k) b(k, j)) for 0 <= i < M, 0 <= j < N
// (only i >= j when `lower`).  64 x 64 output tiles on the FP64 matrix
// cores (MfmaTile); k-chunks of 16 are staged through LDS with the next
// chunk's global loads in flight during the current chunk's products.
// AK (BK) makes consecutive lanes fetch consecutive k of a(i, .) (of
// b(., j)), for operands stored contiguously along k; otherwise they fetch
// consecutive i (j).  Every (i, j) is produced by exactly one thread, in a
// fixed k order.
template <bool AK = false, bool BK = false, class FA, class FB, class EPI>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, const FA& fa, const FB& fb,
                                        const EPI& epi, bool lower, double* sm) {
  double* As = sm;
  double* Bs = sm + KC * LDS_TM;
  const int tid = threadIdx.x;
  constexpr int PER = KC * TM / NT;
  auto slot_a = [&](int q, int& i, int& k) {
    const int e = tid + q * NT;
    i = AK ? e / KC : e & (TM - 1);
    k = AK ? e & (KC - 1) : e / TM;
  };
  auto slot_b = [&](int q, int& j, int& k) {
    const int e = tid + q * NT;
    j = BK ? e / KC : e & (TM - 1);
    k = BK ? e & (KC - 1) : e / TM;
  };
  for (int i0 = 0; i0 < M; i0 += TM) {
    for (int j0 = 0; j0 < N; j0 += TM) {
      if (lower && j0 > i0 + TM - 1) continue;
      MfmaTile T(tid);
      double ra[PER], rb[PER];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          int i, ka, j, kb;
          slot_a(q, i, ka);
          slot_b(q, j, kb);
          ra[q] = (i0 + i < M && k0 + ka < K) ? fa(i0 + i, k0 + ka) : 0.0;
          rb[q] = (j0 + j < N && k0 + kb < K) ? fb(k0 + kb, j0 + j) : 0.0;
        }
      };
      if (K > 0) fetch(0);
      for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          int i, ka, j, kb;
          slot_a(q, i, ka);
          slot_b(q, j, kb);
          As[ka * LDS_TM + i] = ra[q];
          Bs[kb * LDS_TM + j] = rb[q];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);
        T.chunk(As, Bs);
        __syncthreads();
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int gi = i0 + T.row_of(e), gj = j0 + T.col_of(e);
        if (gi < M && gj < N && (!lower || gi >= gj)) epi(gi, gj, T.get(e));
      }
    }
  }
}

// Accumulates sum_{kb <= k < ke} a(i, k) b(k, j) into the tile T at
// (i0, j0) (rows i < M, columns j < N; entries outside read as zero), with
// the operand fetch of wg_gemm (AK, BK).  Several calls with different
// k ranges and fetch layouts may accumulate into one tile.
template <bool AK = false, bool BK = false, class FA, class FB>
__device__ __forceinline__ void tile_mma(MfmaTile& T, int i0, int j0, int M, int N, int kb, int ke,
                                         const FA& fa, const FB& fb, double* sm) {
  double* As = sm;
  double* Bs = sm + KC * LDS_TM;
  const int tid = threadIdx.x;
  constexpr int PER = KC * TM / NT;
  auto slot_a = [&](int q, int& i, int& k) {
    const int e = tid + q * NT;
    i = AK ? e / KC : e & (TM - 1);
    k = AK ? e & (KC - 1) : e / TM;
  };
  auto slot_b = [&](int q, int& j, int& k) {
    const int e = tid + q * NT;
    j = BK ? e / KC : e & (TM - 1);
    k = BK ? e & (KC - 1) : e / TM;
  };
  double ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, ka, j, kb2;
      slot_a(q, i, ka);
      slot_b(q, j, kb2);
      ra[q] = (i0 + i < M && k0 + ka < ke) ? fa(i0 + i, k0 + ka) : 0.0;
      rb[q] = (j0 + j < N && k0 + kb2 < ke) ? fb(k0 + kb2, j0 + j) : 0.0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, ka, j, kb2;
      slot_a(q, i, ka);
      slot_b(q, j, kb2);
      As[ka * LDS_TM + i] = ra[q];
      Bs[kb2 * LDS_TM + j] = rb[q];
    }
    __syncthreads();
    if (k0 + KC < ke) fetch(k0 + KC);
    T.chunk(As, Bs);
    __syncthreads();
  }
}

// A 64 x NC output tile (NC = 16 or 32) for products with few columns:
// wavefront w owns rows 16 w .. 16 w + 15 as NC / 16 blocks of 16 x 16
// (lane layout as MfmaTile).  Each entry takes the same 4-wide k-steps in
// the same order as in a 64 x 64 tile, so it gets the same value, with a
// quarter (NC = 16) or half (NC = 32) of the matrix-core work when the
// other columns would be empty.
template <int NC>
struct NarrowTile {
  static_assert(NC == 16 || NC == 32, "16 or 32 columns");
  v4d acc[NC / 16];
  int wr, lr, lk;
  __device__ __forceinline__ explicit NarrowTile(int tid) {
    wr = (tid >> 6) * 16;
    lr = tid & 15;
    lk = (tid & 63) >> 4;
#pragma unroll
    for (int b = 0; b < NC / 16; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // the KC k-steps of one staged chunk (As: [k][LDS_TM], Bs: [k][NC + 1])
  __device__ __forceinline__ void chunk(const double* As, const double* Bs) {
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = 4 * s + lk;
      const double a = As[k * LDS_TM + wr + lr];
#pragma unroll
      for (int b = 0; b < NC / 16; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k * (NC + 1) + 16 * b + lr], acc[b], 0, 0, 0);
    }
  }
  static constexpr int kEntries = 4 * (NC / 16);
  __device__ __forceinline__ double get(int e) const { return acc[e >> 2][e & 3]; }
  __device__ __forceinline__ int row_of(int e) const { return wr + lk + 4 * (e & 3); }
  __device__ __forceinline__ int col_of(int e) const { return 16 * (e >> 2) + lr; }
};

// tile_mma for a NarrowTile at (i0, j0): accumulates
// sum_{kb <= k < ke} a(i, k) b(k, j) over rows i < M, columns j < N.
template <bool AK = false, bool BK = false, int NC, class FA, class FB>
__device__ __forceinline__ void tile_mma_narrow(NarrowTile<NC>& T, int i0, int j0, int M, int N, int kb, int ke,
                                                const FA& fa, const FB& fb, double* sm) {
  double* As = sm;
  double* Bs = sm + KC * LDS_TM;
  const int tid = threadIdx.x;
  constexpr int PA = KC * TM / NT, PB = (KC * NC + NT - 1) / NT;
  auto slot_a = [&](int q, int& i, int& k) {
    const int e = tid + q * NT;
    i = AK ? e / KC : e & (TM - 1);
    k = AK ? e & (KC - 1) : e / TM;
  };
  auto slot_b = [&](int q, int& j, int& k) {  // valid when e < KC * NC
    const int e = tid + q * NT;
    j = BK ? e / KC : e % NC;
    k = BK ? e % KC : e / NC;
  };
  double ra[PA], rb[PB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      int i, ka;
      slot_a(q, i, ka);
      ra[q] = (i0 + i < M && k0 + ka < ke) ? fa(i0 + i, k0 + ka) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      int j, kb2;
      slot_b(q, j, kb2);
      rb[q] = (tid + q * NT < KC * NC && j0 + j < N && k0 + kb2 < ke) ? fb(k0 + kb2, j0 + j) : 0.0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      int i, ka;
      slot_a(q, i, ka);
      As[ka * LDS_TM + i] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      int j, kb2;
      slot_b(q, j, kb2);
      if (tid + q * NT < KC * NC) Bs[kb2 * (NC + 1) + j] = rb[q];
    }
    __syncthreads();
    if (k0 + KC < ke) fetch(k0 + KC);
    T.chunk(As, Bs);
    __syncthreads();
  }
}

template <int NC, class EPI>
__device__ __forceinline__ void tile_store_narrow(const NarrowTile<NC>& T, int i0, int j0, int M, int N,
                                                  const EPI& epi) {
#pragma unroll
  for (int e = 0; e < NarrowTile<NC>::kEntries; ++e) {
    const int gi = i0 + T.row_of(e), gj = j0 + T.col_of(e);
    if (gi < M && gj < N) epi(gi, gj, T.get(e));
  }
}

// Passes the entries (i, j) of tile T at (i0, j0) with i < M, j < N (and
// i >= j when `lower`) to epi(i, j, value).
template <class EPI>
__device__ __forceinline__ void tile_store(const MfmaTile& T, int i0, int j0, int M, int N, const EPI& epi,
                                           bool lower) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int gi = i0 + T.row_of(e), gj = j0 + T.col_of(e);
    if (gi < M && gj < N && (!lower || gi >= gj)) epi(gi, gj, T.get(e));
  }
}

// epi(i, j, sum_{kb <= k < ke} a(i, k) b(k, j)) for the rows [i0, i0 + 64)
// and the columns [j0, N) of an output with at most 64 columns from j0:
// on a narrow tile when they are at most 32 (uniform over the workgroup).
template <bool AK, bool BK, class FA, class FB, class EPI>
__device__ __forceinline__ void mma_cols(int i0, int j0, int M, int N, int kb, int ke, const FA& fa, const FB& fb,
                                         const EPI& epi, double* sm) {
  if (N - j0 <= 16) {
    NarrowTile<16> T(threadIdx.x);
    tile_mma_narrow<AK, BK>(T, i0, j0, M, N, kb, ke, fa, fb, sm);
    tile_store_narrow(T, i0, j0, M, N, epi);
  } else if (N - j0 <= 32) {
    NarrowTile<32> T(threadIdx.x);
    tile_mma_narrow<AK, BK>(T, i0, j0, M, N, kb, ke, fa, fb, sm);
    tile_store_narrow(T, i0, j0, M, N, epi);
  } else {
    MfmaTile T(threadIdx.x);
    tile_mma<AK, BK>(T, i0, j0, M, N, kb, ke, fa, fb, sm);
    tile_store(T, i0, j0, M, N, epi, false);
  }
}

// One 64 x 64 output tile (i0, j0) of wg_gemm's product by one 256-thread
// workgroup, for products spread over many workgroups (one tile each).
template <bool AK = false, bool BK = false, class FA, class FB, class EPI>
__device__ __forceinline__ void tile_gemm(int i0, int j0, int M, int N, int K, const FA& fa, const FB& fb,
                                          const EPI& epi, bool lower, double* sm) {
  double* As = sm;
  double* Bs = sm + KC * LDS_TM;
  const int tid = threadIdx.x;
  constexpr int PER = KC * TM / NT;
  auto slot_a = [&](int q, int& i, int& k) {
    const int e = tid + q * NT;
    i = AK ? e / KC : e & (TM - 1);
    k = AK ? e & (KC - 1) : e / TM;
  };
  auto slot_b = [&](int q, int& j, int& k) {
    const int e = tid + q * NT;
    j = BK ? e / KC : e & (TM - 1);
    k = BK ? e & (KC - 1) : e / TM;
  };
  MfmaTile T(tid);
  double ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, ka, j, kb;
      slot_a(q, i, ka);
      slot_b(q, j, kb);
      ra[q] = (i0 + i < M && k0 + ka < K) ? fa(i0 + i, k0 + ka) : 0.0;
      rb[q] = (j0 + j < N && k0 + kb < K) ? fb(k0 + kb, j0 + j) : 0.0;
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, ka, j, kb;
      slot_a(q, i, ka);
      slot_b(q, j, kb);
      As[ka * LDS_TM + i] = ra[q];
      Bs[kb * LDS_TM + j] = rb[q];
    }
    __syncthreads();
    if (k0 + KC < K) fetch(k0 + KC);
    T.chunk(As, Bs);
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int gi = i0 + T.row_of(e), gj = j0 + T.col_of(e);
    if (gi < M && gj < N && (!lower || gi >= gj)) epi(gi, gj, T.get(e));
  }
}

// wg_gemm for a workgroup of NTH = TEAMS * NT threads: the teams of NT
// threads share every output tile and take its k-chunks in turn (team t
// the chunks t, t + TEAMS, ...), each staging its own chunk in LDS; the
// partial tiles are then added through LDS in team order, so the result
// does not depend on timing.  At most one tile per front is in flight, so
// this doubles the waves per SIMD on fronts too few to fill the chip.
// Staging: TEAMS * 2 * KC * LDS_TM doubles at sm; the reduction reuses
// them ((TEAMS - 1) * TM * TM doubles).
template <int NTH, bool AK = false, bool BK = false, class FA, class FB, class EPI>
__device__ __forceinline__ void wg_gemm_split(int M, int N, int K, const FA& fa, const FB& fb,
                                              const EPI& epi, bool lower, double* sm) {
  constexpr int TEAMS = NTH / NT;
  static_assert(TEAMS * NT == NTH && TEAMS >= 1, "whole teams");
  static_assert((TEAMS - 1) * TM * TM <= TEAMS * 2 * KC * LDS_TM || TEAMS == 1, "reduction fits the staging");
  const int team = threadIdx.x / NT, tid = threadIdx.x - team * NT;
  double* As = sm + team * 2 * KC * LDS_TM;
  double* Bs = As + KC * LDS_TM;
  constexpr int PER = KC * TM / NT;
  auto slot_a = [&](int q, int& i, int& k) {
    const int e = tid + q * NT;
    i = AK ? e / KC : e & (TM - 1);
    k = AK ? e & (KC - 1) : e / TM;
  };
  auto slot_b = [&](int q, int& j, int& k) {
    const int e = tid + q * NT;
    j = BK ? e / KC : e & (TM - 1);
    k = BK ? e & (KC - 1) : e / TM;
  };
  const int rounds = ((K + KC - 1) / KC + TEAMS - 1) / TEAMS;
  for (int i0 = 0; i0 < M; i0 += TM) {
    for (int j0 = 0; j0 < N; j0 += TM) {
      if (lower && j0 > i0 + TM - 1) continue;
      MfmaTile T(tid);
      double ra[PER], rb[PER];
      auto fetch = [&](int r) {
        const int k0 = (r * TEAMS + team) * KC;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          int i, ka, j, kb;
          slot_a(q, i, ka);
          slot_b(q, j, kb);
          ra[q] = (i0 + i < M && k0 + ka < K) ? fa(i0 + i, k0 + ka) : 0.0;
          rb[q] = (j0 + j < N && k0 + kb < K) ? fb(k0 + kb, j0 + j) : 0.0;
        }
      };
      if (rounds > 0) fetch(0);
      for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          int i, ka, j, kb;
          slot_a(q, i, ka);
          slot_b(q, j, kb);
          As[ka * LDS_TM + i] = ra[q];
          Bs[kb * LDS_TM + j] = rb[q];
        }
        __syncthreads();
        if (r + 1 < rounds) fetch(r + 1);
        T.chunk(As, Bs);
        __syncthreads();
      }
      if (TEAMS > 1) {
        // teams 1.. park their partial tiles, team 0 adds them in order
        if (team > 0) {
#pragma unroll
          for (int e = 0; e < 16; ++e) sm[(team - 1) * TM * TM + e * NT + tid] = T.get(e);
        }
        __syncthreads();
        if (team == 0) {
          for (int t = 1; t < TEAMS; ++t)
#pragma unroll
            for (int e = 0; e < 16; ++e) T.add(e, sm[(t - 1) * TM * TM + e * NT + tid]);
        }
      }
      if (team == 0) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int gi = i0 + T.row_of(e), gj = j0 + T.col_of(e);
          if (gi < M && gj < N && (!lower || gi >= gj)) epi(gi, gj, T.get(e));
        }
      }
      if (TEAMS > 1) __syncthreads();  // the next tile's staging overwrites the partials
    }
  }
}

// Unblocked Cholesky of an nb x nb (nb <= NB) lower block in LDS (leading
// dimension LDD) by wavefront 0.  A non-positive pivot is replaced by one
// (so later arithmetic stays finite) and its index is returned through
// *fail (first failure, -1 if none).  Call with all threads; includes the
// closing workgroup barrier.
__device__ __forceinline__ void diag_chol(double* L, int nb, int* fail) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int k = 0; k < nb; ++k) {
      double d = L[k + k * LDD];
      const bool bad = !(d > 0.0);
      d = bad ? 1.0 : sqrt(d);
      wave_sync();
      if (lane == 0) {
        L[k + k * LDD] = d;
        if (bad && *fail < 0) *fail = k;
      }
      const double inv = 1.0 / d;
      for (int i = k + 1 + lane; i < nb; i += 64) L[i + k * LDD] *= inv;
      wave_sync();
      const int m = nb - k - 1;
      for (int e = lane; e < m * m; e += 64) {
        const int i = k + 1 + e % m, j = k + 1 + e / m;
        if (i >= j) L[i + j * LDD] -= L[i + k * LDD] * L[j + k * LDD];
      }
      wave_sync();
    }
  }
  __syncthreads();
}

// Inverse of an nb x nb lower-triangular block L (LDS, LDD) into Li (LDS,
// LDD; everything outside the lower nb x nb triangle set to zero).  Lane c
// computes column c by forward substitution; columns are independent.
__device__ __forceinline__ void diag_trtri(const double* L, double* Li, int nb) {
  const int c = threadIdx.x;
  for (int e = threadIdx.x; e < NB * LDD; e += NT) Li[e] = 0.0;
  __syncthreads();
  if (c < nb) {
    for (int i = 0; i < c; ++i) Li[i + c * LDD] = 0.0;
    Li[c + c * LDD] = 1.0 / L[c + c * LDD];
    for (int i = c + 1; i < nb; ++i) {
      double v = 0.0;
      for (int k = c; k < i; ++k) v = fma(L[i + k * LDD], Li[k + c * LDD], v);
      Li[i + c * LDD] = -v / L[i + i * LDD];
    }
  }
  __syncthreads();
}

// Partial Cholesky of a J x N column panel reached through G(i, j)
// (a reference to entry (i, j), i >= j): on return rows 0..N-1 of the
// panel hold C = chol(F11) (lower) and rows N..J-1 hold F21 C^-T.  Blocked
// right-looking with NB-column blocks: the diagonal block is factored and
// inverted in LDS, the rows below are multiplied by that inverse and the
// remaining panel columns updated, both with wg_gemm.  With INVDIAG the
// diagonal blocks are left holding their inverses (for multiplications by
// the triangular inverse later).  *fail receives the first failing column
// (or stays -1).
template <bool INVDIAG = false, class GA>
__device__ __forceinline__ void wg_potrf_acc(const GA& G, int J, int N, double* sm, int* fail) {
  double* Ld = sm + SMEM_GEMM;
  for (int kb = 0; kb < N; kb += NB) {
    const int nb = min(NB, N - kb);
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) Ld[i + j * LDD] = G(kb + i, kb + j);
    }
    __shared__ int lfail;
    if (threadIdx.x == 0) lfail = -1;
    __syncthreads();
    diag_chol(Ld, nb, &lfail);
    if (threadIdx.x == 0 && lfail >= 0 && *fail < 0) *fail = kb + lfail;
    double* Li = Ld + NB * LDD;
    if (kb + nb < J || INVDIAG) diag_trtri(Ld, Li, nb);
    const double* Lw = INVDIAG ? Li : Ld;
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) G(kb + i, kb + j) = Lw[i + j * LDD];
    }
    // rows below the diagonal block: X <- X C_kk^-T, applied as a product
    // with the explicit inverse of the diagonal block.  In place is safe:
    // nb <= TM gives one column tile, and each row tile reads only its own
    // rows before its epilogue writes them.
    if (kb + nb < J) {
      wg_gemm(
          J - kb - nb, nb, nb, [&](int i, int k) { return G(kb + nb + i, kb + k); },
          [&](int k, int j) { return Li[j + k * LDD]; },
          [&](int i, int j, double acc) { G(kb + nb + i, kb + j) = acc; }, false, sm);
    }
    __syncthreads();
    const int r0 = kb + nb;
    if (r0 < N) {
      wg_gemm(
          J - r0, N - r0, nb, [&](int i, int k) { return G(r0 + i, kb + k); },
          [&](int k, int j) { return G(r0 + j, kb + k); },
          [&](int i, int j, double acc) { G(r0 + i, r0 + j) -= acc; }, true, sm);
      __syncthreads();
    }
  }
}

// wg_potrf_acc on a column-major panel F with leading dimension ld.
__device__ __forceinline__ void wg_potrf_panel(double* F, int ld, int J, int N, double* sm, int* fail) {
  wg_potrf_acc([&](int i, int j) -> double& { return F[i + (int64_t)j * ld]; }, J, N, sm, fail);
}

// In place, on an n x n lower triangle reached through G(i, j) (i >= j):
// G <- G^-1.  Diagonal blocks from the last to the first: with
// G = [G11 0; G21 G22] and G22 already inverted in place,
// inv(G)21 = -inv(G22) G21 inv(G11); the product inv(G22) G21 overwrites
// G21 row tile by row tile from the bottom (a tile reads only rows at or
// above its own).  INVDIAG: the diagonal blocks already hold their
// inverses (wg_potrf_acc<true>).
template <bool INVDIAG = false, class GA>
__device__ __forceinline__ void wg_trtri_inplace(const GA& G, int n, double* sm) {
  double* Ld = sm + SMEM_GEMM;
  double* Li = Ld + NB * LDD;
  const int nblk = (n + NB - 1) / NB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int jb = bk * NB, nb = min(NB, n - jb);
    if (INVDIAG) {
      for (int e = threadIdx.x; e < NB * LDD; e += NT) Li[e] = 0.0;
      __syncthreads();
      for (int e = threadIdx.x; e < nb * nb; e += NT) {
        const int i = e % nb, j = e / nb;
        if (i >= j) Li[i + j * LDD] = G(jb + i, jb + j);
      }
      __syncthreads();
    } else {
      for (int e = threadIdx.x; e < nb * nb; e += NT) {
        const int i = e % nb, j = e / nb;
        if (i >= j) Ld[i + j * LDD] = G(jb + i, jb + j);
      }
      __syncthreads();
      diag_trtri(Ld, Li, nb);
    }
    const int r0 = jb + nb, m = n - r0;
    if (m > 0) {
      for (int i0 = ((m - 1) / TM) * TM; i0 >= 0; i0 -= TM) {
        MfmaTile T(threadIdx.x);
        tile_mma<false, true>(
            T, i0, 0, m, nb, 0, min(m, i0 + TM),
            [&](int i, int k) { return k <= i ? G(r0 + i, r0 + k) : 0.0; },
            [&](int k, int j) { return G(r0 + k, jb + j); }, sm);
        tile_store(T, i0, 0, m, nb, [&](int i, int j, double acc) { G(r0 + i, jb + j) = acc; }, false);
        __syncthreads();
      }
      wg_gemm(
          m, nb, nb, [&](int i, int k) { return G(r0 + i, jb + k); },
          [&](int k, int j) { return Li[k + j * LDD]; },
          [&](int i, int j, double acc) { G(r0 + i, jb + j) = -acc; }, false, sm);
      __syncthreads();
    }
    if (!INVDIAG)
      for (int e = threadIdx.x; e < nb * nb; e += NT) {
        const int i = e % nb, j = e / nb;
        if (i >= j) G(jb + i, jb + j) = Li[i + j * LDD];
      }
    __syncthreads();
  }
}

// In place, on an n x n lower triangle reached through G(i, j) (i >= j):
// G <- the lower triangle of G^T G, i.e. W(i, j) = sum_{k >= i} G(k, i)
// G(k, j) for i >= j.  Row tiles from the top; within a row tile the
// diagonal tile last: a tile reads only rows at or below its own, and the
// diagonal column block that the other tiles of its row still read is
// overwritten last.
template <class GA>
__device__ __forceinline__ void wg_lauum_inplace(const GA& G, int n, double* sm) {
  for (int i0 = 0; i0 < n; i0 += TM) {
    for (int j0 = 0; j0 <= i0; j0 += TM) {
      // off-diagonal tiles first, in order; the diagonal tile (j0 == i0) last
      MfmaTile T(threadIdx.x);
      tile_mma<true, true>(
          T, 0, 0, TM, TM, i0, n,
          [&](int i, int k) { return (i0 + i < n && k >= i0 + i) ? G(k, i0 + i) : 0.0; },
          [&](int k, int j) { return (j0 + j < n && k >= j0 + j) ? G(k, j0 + j) : 0.0; }, sm);
      tile_store(
          T, 0, 0, min(TM, n - i0), min(TM, n - j0),
          [&](int i, int j, double acc) {
            if (i0 + i >= j0 + j) G(i0 + i, j0 + j) = acc;
          },
          false);
      __syncthreads();
    }
  }
}

// Dense column-major accessor (reference to entry (i, j)).
struct DenseAt {
  double* a;
  int64_t ld;
  __device__ __forceinline__ double& operator()(int i, int j) const { return a[i + (int64_t)j * ld]; }
};

// Block of the left-looking factorizations below, and the leading
// dimension of their 64 x 64 diagonal block in LDS (d64: NB2 * LD2
// doubles, passed by the caller).
constexpr int NB2 = 64;
constexpr int LD2 = NB2 + 1;

// In place on an n x n lower triangle reached through G(i, j) (i >= j):
// left-looking blocked Cholesky with 64-column blocks.  Every 64 x 64 tile
// of the factor is formed once, T = G(I, J) - sum_{k < j0} G(I, k) G(J, k),
// as one pipelined matrix-core k-loop; the diagonal tile is then factored
// and inverted in LDS and the tiles below it are multiplied by the
// transposed inverse.  On return each 64 x 64 diagonal block holds the
// INVERSE of its Cholesky block (as wg_trtri64_invdiag expects).  *fail
// receives the first failing column (or stays -1).
template <class GA>
__device__ __forceinline__ void wg_potrf64(const GA& G, int n, double* sm, double* d64, int* fail) {
  const DenseAt D{d64, LD2};
  for (int j0 = 0; j0 < n; j0 += NB2) {
    const int nb = min(NB2, n - j0);
    {
      MfmaTile T(threadIdx.x);
      tile_mma(T, 0, 0, nb, nb, 0, j0, [&](int i, int k) { return G(j0 + i, k); },
               [&](int k, int j) { return G(j0 + j, k); }, sm);
      for (int e = threadIdx.x; e < NB2 * LD2; e += NT) d64[e] = 0.0;
      __syncthreads();
      tile_store(T, 0, 0, nb, nb, [&](int i, int j, double acc) { d64[i + j * LD2] = G(j0 + i, j0 + j) - acc; },
                 true);
    }
    __syncthreads();
    __shared__ int lf;
    if (threadIdx.x == 0) lf = -1;
    __syncthreads();
    wg_potrf_acc(D, nb, nb, sm, &lf);
    if (threadIdx.x == 0 && lf >= 0 && *fail < 0) *fail = j0 + lf;
    wg_trtri_inplace(D, nb, sm);
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) G(j0 + i, j0 + j) = d64[i + j * LD2];
    }
    __syncthreads();
    for (int i0 = j0 + nb; i0 < n; i0 += TM) {
      MfmaTile T(threadIdx.x);
      tile_mma(T, i0, 0, n, nb, 0, j0, [&](int i, int k) { return G(i, k); },
               [&](int k, int j) { return G(j0 + j, k); }, sm);
      tile_store(T, i0, 0, n, nb, [&](int i, int j, double acc) { G(i, j0 + j) = G(i, j0 + j) - acc; }, false);
      __syncthreads();
      MfmaTile T2(threadIdx.x);
      tile_mma(T2, i0, 0, n, nb, 0, nb, [&](int i, int k) { return G(i, j0 + k); },
               [&](int k, int j) { return d64[j + k * LD2]; }, sm);
      tile_store(T2, i0, 0, n, nb, [&](int i, int j, double acc) { G(i, j0 + j) = acc; }, false);
      __syncthreads();
    }
  }
}

// In place on an n x n lower triangle G whose 64 x 64 diagonal blocks
// already hold their inverses (wg_potrf64): G <- G^-1, diagonal blocks from
// the last to the first (as wg_trtri_inplace, with 64-column blocks).
template <class GA>
__device__ __forceinline__ void wg_trtri64_invdiag(const GA& G, int n, double* sm, double* d64) {
  const int nblk = (n + NB2 - 1) / NB2;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int jb = bk * NB2, nb = min(NB2, n - jb);
    const int r0 = jb + nb, m = n - r0;
    if (m == 0) continue;
    for (int e = threadIdx.x; e < NB2 * LD2; e += NT) d64[e] = 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) d64[i + j * LD2] = G(jb + i, jb + j);
    }
    __syncthreads();
    for (int i0 = ((m - 1) / TM) * TM; i0 >= 0; i0 -= TM) {
      MfmaTile T(threadIdx.x);
      tile_mma<false, true>(
          T, i0, 0, m, nb, 0, min(m, i0 + TM), [&](int i, int k) { return k <= i ? G(r0 + i, r0 + k) : 0.0; },
          [&](int k, int j) { return G(r0 + k, jb + j); }, sm);
      tile_store(T, i0, 0, m, nb, [&](int i, int j, double acc) { G(r0 + i, jb + j) = acc; }, false);
      __syncthreads();
    }
    wg_gemm(
        m, nb, nb, [&](int i, int k) { return G(r0 + i, jb + k); },
        [&](int k, int j) { return d64[k + j * LD2]; },
        [&](int i, int j, double acc) { G(r0 + i, jb + j) = -acc; }, false, sm);
    __syncthreads();
  }
}

// Ci = C^-1 for an N x N lower-triangular C (leading dimensions ldc, ldi),
// blocked, last diagonal block first: with C = [C11 0; C21 C22],
// inv(C)21 = -inv(C22) C21 inv(C11).
template <class CF>
__device__ __forceinline__ void wg_trtri(const CF& C, int N, double* Ci, int ldi, double* sm) {
  double* Ld = sm + SMEM_GEMM;
  double* Li = Ld + NB * LDD;
  const int nblk = (N + NB - 1) / NB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int jb = bk * NB, nb = min(NB, N - jb);
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      if (i >= j) Ld[i + j * LDD] = C(jb + i, jb + j);
    }
    __syncthreads();
    diag_trtri(Ld, Li, nb);
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int i = e % nb, j = e / nb;
      Ci[(jb + i) + (int64_t)(jb + j) * ldi] = i >= j ? Li[i + j * LDD] : 0.0;
    }
    const int r0 = jb + nb, m = N - r0;
    if (m > 0) {
      // T = inv(C22) C21 into the output block, then right-multiply by -inv(C11)
      wg_gemm<false, true>(
          m, nb, m,
          [&](int i, int k) { return k <= i ? Ci[(r0 + i) + (int64_t)(r0 + k) * ldi] : 0.0; },
          [&](int k, int j) { return C(r0 + k, jb + j); },
          [&](int i, int j, double acc) { Ci[(r0 + i) + (int64_t)(jb + j) * ldi] = acc; }, false,
          sm);
      __syncthreads();
      // block <- -T inv(C11), in place (one column tile, row-local)
      wg_gemm(
          m, nb, nb, [&](int i, int k) { return Ci[(r0 + i) + (int64_t)(jb + k) * ldi]; },
          [&](int k, int j) { return Li[k + j * LDD]; },
          [&](int i, int j, double acc) { Ci[(r0 + i) + (int64_t)(jb + j) * ldi] = -acc; }, false,
          sm);
    }
    __syncthreads();
  }
  // zero the strict upper triangle so Ci can be read as a full matrix
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int i = e % N, j = e / N;
    if (i < j) Ci[i + (int64_t)j * ldi] = 0.0;
  }
  __syncthreads();
}

// Deterministic workgroup sum of one value per thread.
__device__ __forceinline__ double wg_sum(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

}  // namespace mfb

// Internal structures shared by the symbolic plan (host) and the kernels.
#pragma once
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/mfb.h"

namespace mfb {

// Device view of a plan: plain pointers, passed to kernels by value.
// Supernodes are numbered in a postorder of the clique tree (children
// before parents).  For supernode s with N = |N_s|, A = |A_s|, J = N + A:
//   col[colbase[s] + c] = CCS offset of the diagonal entry of the c-th
//   column of N_s.  Because V is filled, that CCS column holds exactly the
//   rows J_s[c:], so panel entry (r, c), r >= c, of any CCS-ordered array
//   is at col[colbase[s] + c] + (r - c).
//   rel[relbase[s] + t] = position of A_s[t] inside J_parent(s).
//   arena[s] = offset (in doubles) of the packed lower triangle of an
//   A x A symmetric block (update matrices U, V and their derivatives).
struct DevPlan {
  int32_t ns;
  int64_t n, nnz;
  const int32_t* ncol;      // N
  const int32_t* nrow;      // J
  const int32_t* parent;    // -1 for roots
  const int32_t* cptr;      // children of s: cidx[cptr[s] .. cptr[s+1])
  const int32_t* cidx;
  const int32_t* colbase;
  const int64_t* col;
  const int32_t* relbase;
  const int32_t* rel;
  const int64_t* arena;
  const int32_t* vlabel;    // user label of the c-th column: vlabel[colbase[s] + c]
  int32_t big_a;            // S_AA blocks with A > big_a are factored tile-parallel
  const int64_t* poff;      // offset of the front's partial products V' L, or -1 (kPartN)
};

struct Level {
  int32_t begin, count;  // slice of the level's supernode list
  int32_t maxN, maxA, maxJ;
  // sums over the level's supernodes, for canonical bytes and flops:
  // panel entries sum_c (J - c), packed update entries A(A+1)/2, N^3, N^2 A, N A^2, A^3
  double p, u, n3, n2a, na2, a3;
};

// Scratch (doubles per workgroup) of each kernel for a level's largest front.
enum Op { OP_FACTOR, OP_PRODUCT, OP_COMPLETION, OP_VINV, OP_HUP, OP_HDOWN, OP_IHDOWN, OP_IHUP, OP_HFAC };
inline int64_t slot_doubles(Op op, const Level& L) {
  const int64_t N = L.maxN, A = L.maxA, J = L.maxJ;
  switch (op) {
    case OP_FACTOR: return J * N + N * N + 64 * N + 4096;  // fat fronts: + inverse diagonal blocks
    case OP_PRODUCT: return J * N;
    case OP_COMPLETION: return 3 * N * N + A * N + 64 * N + 4096;
    case OP_VINV: return 1;
    case OP_HUP: return J * N;
    case OP_HDOWN: return 2 * A * N + 2 * N * N;
    case OP_IHDOWN: return 2 * A * N + 3 * N * N;
    case OP_IHUP: return J * N + A * N;
    case OP_HFAC: return 2 * N * N + A * N;
  }
  return 0;
}
// Register-front classes: the register kernel of class c takes fronts of
// order (J for the factor and the completion, A for the inverse of V_s)
// at most kRegMax[c]; larger fronts run the blocked kernels.
constexpr int kRegClasses = 5;
constexpr int kRegMax[kRegClasses] = {16, 32, 64, 128, 192};
// The cached inverse of V_s = S_{A_s A_s} (inverse Hessian and completion)
// is held as V_s^-1 itself for A <= kVExplicitMax (the register kernels'
// sweeps produce it) and as the inverse Cholesky factor C_V^-1 (lower,
// packed; V_s = C_V C_V^T) beyond, so that the blocked kernels form
// V_s^-1 B as C_V^-T (C_V^-1 B) and the completion's Schur complement as
// S_NN - W^T W with W = C_V^-1 S_AN.
constexpr int kVExplicitMax = kRegMax[kRegClasses - 1];
// Largest front order for which the projected inverse and the Hessian
// and inverse-Hessian down-sweeps use the register kernels on a level of
// non-root fronts.
constexpr int kDownRegMaxJ = 64;
// Largest workgroup scratch (doubles per right-hand side) of one launch of
// a schedule that runs independent fronts together.
constexpr int64_t kFlatScratch = int64_t(1) << 22;
// The same for the completion's wide and fat fronts (scratch per front
// A N + 3 N^2 + ..., many fronts per launch).
constexpr int64_t kFlatScratchFat = int64_t(1) << 26;
// Largest number of packed update-block entries for which the plan keeps
// the CCS source offset of every entry (8 bytes each), so that gathering
// the blocks of an input takes one elementwise launch.
constexpr int64_t kGatherMapMax = int64_t(1) << 25;

// Wide fronts: a large ancestor set and few columns (J > the plan's wide
// threshold, N <= kWideMaxN, A > 0).  Their A x A and A x N work runs
// tile-parallel over all wide fronts of a level (wide.hip).
constexpr int kWideMaxN = 64;
constexpr int kWideJ = 192;     // default threshold on J (the largest register front)
constexpr int kWideJLow = 64;   // with MFB_PLAN_WIDE_LOW
constexpr int kWide = kRegClasses + 1;  // class value of a wide segment
constexpr int kFat = kRegClasses + 2;   // class value of a segment of fat fronts
constexpr int kWideTile = 64;
// The blocks S_AA with A > the plan's big_a (kBigA, or kVExplicitMax with
// MFB_PLAN_WIDE_LOW) are factored and inverted tile-parallel, one launch
// per block column and row block over all such fronts (wide.hip, "bigv"),
// for the inverse Hessian's and the Hessian factor's caches and in the
// completion; smaller ones by one workgroup each.
constexpr int kBigA = 256;
constexpr int kBigV = kRegClasses + 3;  // class value of the segment of those fronts
// Wide fronts with at most kPartN columns form the product V' L of the
// root-to-leaf sweeps (V' = the extracted block: V'_s of the Hessian, T_AA
// of the inverse Hessian) from partial products taken while each 64 x 64
// tile of V' is extracted, so V' is not read back: per lower tile (ti, tj)
// the 64 x N blocks V'_{ti,tj} L_tj and V'_{ti,tj}^T L_ti (strictly lower
// entries only on the diagonal tile), in a per-RHS area at poff[s].
constexpr int kPartN = 4;

// A level of a schedule split by class: at most three launches (groups of
// launches for the wide fronts), the wide fronts (cls == kWide), the
// blocked kernels (cls == kRegClasses) on the other fronts no register
// class holds, then one register class, the largest any other front of
// the level needs.  A wide segment also numbers its tiles: pre[aa_off +
// f] is the first 64 x 64 lower tile of the A x A block of its front f
// (n_aa in all), pre[rt_off + f] the first 64-row tile of its A rows (n_rt
// in all).
struct ClassSeg {
  Level lv;  // begin/count index the schedule's own list
  int32_t level, cls;
  // tile numbering of a wide or fat segment: prefix arrays in the
  // schedule's `pre` (count + 1 entries each) of the 64 x 64 lower tiles of
  // the A x A blocks (aa), of the tiles of the A x N blocks (an) and of the
  // N x N blocks (nn), with their totals; for fat segments also the grid
  // sizes of the per-front tile sets (largest front)
  int32_t aa_off = 0, an_off = 0, nn_off = 0, n_aa = 0, n_an = 0, n_nn = 0;
  int32_t fat_panel = 0, fat_fin = 0;
  // kBigV segments (fronts in decreasing order of A): acnt[t] = number of
  // fronts with A > 64 t, the prefix of the list a step at row 64 t needs
  std::vector<int32_t> acnt;
};
struct ClassSched {
  std::vector<int32_t> list;
  std::vector<ClassSeg> segs;
  std::vector<int32_t> pre;  // tile prefix arrays of the wide segments
  const int32_t* d_list = nullptr;
  const int32_t* d_pre = nullptr;
};

}  // namespace mfb

struct mfb_plan_s {
  int64_t n = 0, nnz = 0;
  uint32_t flags = 0;
  int32_t ns = 0;
  int32_t wide_thr = mfb::kWideJ;  // wide fronts: J > wide_thr (see kWideMaxN)
  int32_t big_a = mfb::kBigA;      // tile-parallel S_AA factorization: A > big_a (see kBigA)
  std::vector<int32_t> N, J, parent, cptr, cidx, colbase, relbase, rel, rep, vlabel, snode_of;
  std::vector<int64_t> col, arena;
  // per supernode: offset of its partial products in the per-RHS partial
  // area, or -1 (wide fronts with at most kPartN columns, A > 0), and the
  // area's size in doubles
  std::vector<int64_t> poff;
  int64_t part_doubles = 0;
  int64_t update_doubles = 0;
  int32_t max_front = 0, max_ncols = 0, max_nanc = 0;
  // leaf-to-root schedule: levels by height; root-to-leaf: by depth
  std::vector<int32_t> up_list, down_list;
  std::vector<mfb::Level> up_levels, down_levels;
  // class-split schedules: factor (leaf-to-root, by J), inverse of V_s
  // (by A) and the projected inverse and Hessian down-sweeps (by J on the
  // levels that take the register kernels, blocked elsewhere); wide fronts
  // in segments of their own in the leaf-to-root and root-to-leaf ones
  mfb::ClassSched cs_factor, cs_vinv, cs_down;
  // the completion's sweeps, one launch per class over all supernodes;
  // the inverse Hessian's steps 1+2 likewise, in launches whose workgroup
  // scratch stays within kFlatScratch doubles per right-hand side
  mfb::ClassSched cs_compl_flat, cs_ihd_flat;
  // the Hessian factor's per-supernode conversions: every supernode, one
  // launch per group of fronts whose workgroup scratch stays within
  // kFlatScratch doubles per right-hand side
  mfb::ClassSched cs_hfac;
  // the fronts with A > big_a (cs_vinv's kBigV segment), which the
  // completion factors tile-parallel before its per-front launches
  mfb::ClassSched cs_bigv;
  // the Hessian down-sweep: cs_down without its root level when that is one
  // front with A = 0 and N > kDownRegMaxJ (hd_root, else -1), which runs as
  // tile-parallel products instead
  mfb::ClassSched cs_hdown;
  int32_t hd_root = -1;
  // that front when it was also taken out of cs_ihd_flat (the inverse
  // Hessian's steps 1+2 of it then run tile-parallel too), else -1
  int32_t ihd_root = -1;
  // gmap[e]: CCS offset of the input entry that packed update-block entry e
  // holds (S_AA or T_AA blocks), empty beyond kGatherMapMax entries;
  // all_levels: every supernode as one level (canonical counts of a gather)
  std::vector<int64_t> gmap;
  std::vector<mfb::Level> all_levels;
  // the same gather level by level (plans without the map): per
  // root-to-leaf level one segment of the fronts with A > 0, its tiles
  // numbered as in a wide segment
  mfb::ClassSched cs_gather;
  const int64_t* d_gmap = nullptr;
  double fl_factor = 0, fl_projinv = 0, fl_hess = 0, fl_invhess = 0, fl_invhess_x = 0,
         fl_completion = 0, fl_product = 0;
  double by_factor = 0, by_projinv = 0, by_hess = 0, by_invhess = 0, by_completion = 0, by_product = 0;
  // the pattern the plan factors on (CCS, host)
  std::vector<int64_t> colptr_h;
  std::vector<int32_t> rowind_h;
  // relaxed plans: the plan is that of V', a filled superset of the
  // caller's pattern V; the caller's arrays (nnz_user entries) are on V.
  // Entry e of V sits at e + vshift[e] in V'; zpos lists V' \ V.
  bool relaxed = false;
  double relax_frac = 0;
  int64_t nnz_user = 0;
  std::vector<int32_t> vshift;
  std::vector<int64_t> zpos, ucolptr_h;
  const int32_t* d_vshift = nullptr;
  const int64_t* d_zpos = nullptr;
  const int64_t* d_ucolptr = nullptr;
  // device copies (uploaded on first use)
  std::mutex mu;
  void* dmem = nullptr;  // one allocation holding every index array
  mfb::DevPlan dev{};
  const int32_t* d_up_list = nullptr;
  const int32_t* d_down_list = nullptr;
  const int32_t* d_all_list = nullptr;  // 0..ns-1
  const int64_t* d_colptr = nullptr;    // user colptr (n+1)
  const int32_t* d_colidx = nullptr;    // column of every CCS entry (nnz)
};

namespace mfb {
// Plan thresholds chosen by the caller (0: the default or the environment's)
struct PlanTuning {
  int32_t wide_j = 0, big_a = 0;
};
// Host symbolic analysis (plan.cpp).  Fills everything except device copies.
mfb_status_t build_plan(int64_t n, const int64_t* colptr, const int32_t* rowind, uint32_t flags,
                        mfb_plan_s* p, const PlanTuning& tune = PlanTuning{});
// The same on relaxed supernodes: zeros per merged supernode within `frac`
// of its entries.
mfb_status_t build_plan_relaxed(int64_t n, const int64_t* colptr, const int32_t* rowind, uint32_t flags,
                                double frac, mfb_plan_s* p, const PlanTuning& tune = PlanTuning{});
}  // namespace mfb

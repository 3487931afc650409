// Kernel entry points of kernels.hip (launched from api.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "mfb_internal.h"

namespace mfb {
constexpr int NT_LAUNCH = 256;  // threads per workgroup of the blocked sweep kernels
// except the projected inverse and the Hessian down-sweeps: two teams of
// NT_LAUNCH splitting every product's k range
constexpr int NT_DOWN = 512;

struct DevStatus {
  int code;
  int pad;
  unsigned long long bad;  // smallest failing user column
};

template <bool PANEL>
__global__ void k_factor(DevPlan, const int32_t*, const double*, double*, double*, double*,
                         double*, DevStatus*, double*, int64_t);
__global__ void k_projinv(DevPlan, const int32_t*, const double*, double*, double*);
template <bool PANEL>
__global__ void k_hess_up(DevPlan, const int32_t*, const double*, const double*, double*, double*,
                          int64_t, double*, int64_t, int32_t*);
__global__ void k_hess_down(DevPlan, const int32_t*, const double*, const double*, const double*,
                            double*, double*, int64_t, double*, int64_t);
__global__ void k_ihess_down(DevPlan, const int32_t*, const double*, const double*, const double*,
                             const double*, double*, double*, int64_t, double*, int64_t);
template <bool PANEL>
__global__ void k_ihess_up(DevPlan, const int32_t*, const double*, const double*, double*, double*,
                           int64_t, double*, int64_t);
__global__ void k_completion(DevPlan, const int32_t*, const double*, double*, double*, double*,
                             double*, double*, double*, DevStatus*, double*, int64_t);
__global__ void k_vinv(DevPlan, const int32_t*, const double*, double*, DevStatus*, double*,
                       int64_t);
template <int STAGE>
__global__ void k_hess_down_root(DevPlan, const int32_t*, const double*, const double*, double*, double*,
                                 int64_t);
template <int STAGE>
__global__ void k_ihess_down_root(DevPlan, const int32_t*, const double*, const double*, double*, double*,
                                  int64_t);
template <int TAG>
__global__ void k_gather_map(const int64_t*, int64_t, const double*, double*, int64_t, int64_t);
template <bool PANEL>
__global__ void k_product(DevPlan, const int32_t*, const double*, double*, double*, double*,
                          int64_t);
__global__ void k_logdet(const double*, int, double*);
__global__ void k_export_ldl(const double*, const int64_t*, const int32_t*, int64_t, double*);
__global__ void k_reset_status(DevStatus*);
// relaxed plans: caller arrays on V in and out of the sweeps' V'
void launch_relax_in(hipStream_t s, int k, const double* src, int64_t nu, const int32_t* shift, const int64_t* zpos,
                     int64_t nz, double* dst, int64_t nv);
void launch_relax_out(hipStream_t s, int k, const double* src, int64_t nv, const int32_t* shift, double* dst,
                      int64_t nu);

// Register-front kernels for fronts of order <= kRegMax[cls] (host
// launchers; cls selects the workgroup shape).
void launch_vinv_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                     const double* Vs, double* Vi, DevStatus* st);
void launch_factor_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                       const double* x, double* R, double* LB, double* U, double* part, DevStatus* st);
void launch_completion_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* Sin, double* R, double* LB, double* S, double* Vs,
                           double* Vi, double* part, DevStatus* st);
// Algorithm 7.3 with factored update matrices V_s = R_s R_s^T, one
// root-to-leaf level (grid.x fronts of list); Ru: the packed R_s^T blocks
// at the plan's arena offsets (parents' in place, the level's written).
void launch_completion_factored(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* Sin,
                                double* R, double* LB, double* S, double* Ru, double* part, DevStatus* st,
                                double* wsb, int64_t slot);
// Inverse Hessian steps 1+2 with S_AA through the factors R_s left in Ru by
// the factored completion (grid: fronts of list x right-hand sides).
void launch_ihess_down_factored(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                                const double* LB, const double* Ru, const double* T, double* Kt, double* Va,
                                int64_t upd, double* wsb, int64_t slot);
// act: Hessian step 1's per-(RHS, supernode) activity flags (ns per RHS;
// entries of pruned fronts are set to 0, others left as they are)
void launch_hess_up_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* LB, const double* Y, double* Kt, double* Ua, int64_t upd, int32_t* act);
void launch_fill_i32(hipStream_t s, int32_t* x, int64_t n, int32_t v);
void launch_ihess_up_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                         const double* LB, const double* Kt, double* Y, double* Ua, int64_t upd);
void launch_product_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* R, double* X, double* U);
void launch_projinv_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const double* LB, double* S, double* Vs);
void launch_hess_down_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                          const double* LB, const double* Vs, const double* Kt, double* T, double* Va,
                          int64_t upd, double* wsb, int64_t slot);
void launch_ihess_down_reg(int cls, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* R, const double* LB, const double* Vi, const double* T,
                           double* Kt, double* Va, int64_t upd, double* wsb, int64_t slot);

// Wide fronts (wide.hip): tile-parallel update blocks, parent extraction
// and root-to-leaf products over the wide fronts of one level.  The tiles
// of a segment are numbered front by front through prefix arrays (count +
// 1 entries each): `aa` the 64 x 64 lower tiles of the A x A blocks, `an`
// the 64 x 64 tiles of the A x N blocks, `nn` those of the N x N blocks.
struct WideTiles {
  const int32_t *aa, *an, *nn;
  int n_aa, n_an, n_nn;
};
// op: 0 factor, 1 Hessian step 1, 2 inverse Hessian step 3, 3 product;
// act (op 1, may be null): the step's activity flags, pruned fronts skipped
void launch_wide_update(int op, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                        const int32_t* pre, int count, const double* R, const double* LB, const double* Kt,
                        double* Ua, int64_t upd, const double* wsb, int64_t slot, const int32_t* act);
// Panel part of the product (UP_PRODUCT, Y = X, k = 1) or of the inverse
// Hessian's step 3 (UP_IHESS) for the wide fronts of a segment (maxA: its
// largest ancestor count), tile-parallel over 64-row tiles
enum { UP_PRODUCT = 0, UP_IHESS = 1 };
void launch_up_panel_tiles(int up, int maxA, int count, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const double* R, const double* LB, const double* Kt, double* Y, const double* Ua,
                           int64_t upd, double* wsb, int64_t slot);
// tag (profile attribution): 1 inverse Hessian gather, 2 completion gather
// tag 1 (the inverse Hessian's gather) with part: also the partial
// products of T_AA L_AN of the fronts that have a partial area
void launch_wide_extract(int tag, dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list,
                         const int32_t* pre, int count, const double* src, double* arena, int64_t src_stride,
                         int64_t arena_stride, const double* LB, double* part, int64_t pstride);
void launch_wide_projinv(hipStream_t s, const DevPlan& P, const int32_t* list, const WideTiles& w, int count,
                         const double* LB, double* S, double* Vs);
void launch_wide_hess_down(int k, int maxN, int maxA, hipStream_t s, const DevPlan& P, const int32_t* list,
                           const WideTiles& w, int count, const double* LB, const double* Vs, const double* Kt,
                           double* T, double* Va, int64_t upd, double* wsb, int64_t slot, double* part,
                           int64_t pstride);
// Fat fronts (more than kWideMaxN columns): grids sized by the segment's
// largest front; `panel` = tiles of the J x N panel, `fin` = NN plus AN
// tiles.  Panel op: 0 factor (source X), 1 Hessian step 1 (source Y),
// 2 inverse Hessian step 3, 3 product (children only).
struct FatGrid {
  int maxN, maxA, maxJ, panel, fin;
};
void launch_fat_panel(int op, const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                      int count, const double* src, const double* Ua, int64_t upd, double* wsb, int64_t slot,
                      const int32_t* act);
void launch_fat_factor(const FatGrid& g, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                       double* R, double* LB, double* part, DevStatus* st, double* wsb, int64_t slot);
// op: 0 product (Out = X), 1 Hessian step 1 (K), 2 inverse Hessian step 3 (Out = Y)
void launch_fat_up_fin(int op, const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list,
                       int count, const double* R, const double* LB, double* Out, double* Kt, double* wsb,
                       int64_t slot);
void launch_fat_completion(const FatGrid& g, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                           const double* Sin, double* R, double* LB, double* S, const double* Vs, double* Vi,
                           double* part, DevStatus* st, double* wsb, int64_t slot);
// Tile-parallel Cholesky factor (into Cb, packed like S_AA) and its inverse
// (into Out) of the blocks S_AA with A > big_a of the listed fronts.  mode
// 0: for the inverse Hessian, 1: for the completion (failures reported as
// no completion), 2: for the Hessian factor, on the reversed view, giving
// G (G^T G = S_AA) and G^-1.
// acnt (host, may be null): the segment's prefix counts (ClassSeg::acnt),
// so that each step launches only the fronts it has work for.
void launch_bigv(int mode, int maxA, int count, const int32_t* acnt, hipStream_t s, const DevPlan& P,
                 const int32_t* list, const double* Vs, double* Cb, double* Out, DevStatus* st);
// part: the gather's partial products of T_AA L (nullptr when the gather
// took the source map), per-RHS stride pstride
void launch_fat_ihess(const FatGrid& g, int k, hipStream_t s, const DevPlan& P, const int32_t* list, int count,
                      const double* R, const double* LB, const double* Vi, const double* T, double* Kt,
                      const double* Va, int64_t upd, double* wsb, int64_t slot, const double* part,
                      int64_t pstride);

// Hessian factor (hfactor.hip): per supernode with A > 0 the lower G with
// G^T G = S_AA and G^-1, packed like S_AA (one workgroup per supernode);
// the conversions between the Hessian's step 1 and W = R(Y) (one workgroup
// per supernode and right-hand side, scratch 2N^2 + AN); the Gram matrix of
// m vectors of S^n_V (partials per 64 x 64 tile pair and entry chunk, then
// an ordered sum).
void launch_gamma(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* Vs, double* Gam,
                  double* Gami, DevStatus* st);
void launch_hfactor(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                    const double* Gam, const double* Kt, double* Wt, double* wsb, int64_t slot, const int32_t* act);
void launch_hfactor_adj(dim3 grid, hipStream_t s, const DevPlan& P, const int32_t* list, const double* R,
                        const double* Gami, const double* Wt, double* Kt, double* wsb, int64_t slot);
struct GramShape {
  int pairs = 0;                          // lower 64 x 64 tile pairs of the m x m result
  int64_t chunk = 0, nfull = 0, nparts = 0;  // entries per chunk, chunks over nnz, all chunks
  int64_t part_doubles = 0;                  // partial sums: nparts * pairs 64 x 64 tiles
};
GramShape gram_shape(int64_t nnz, int64_t n, int m);
void launch_gram(hipStream_t s, const GramShape& g, const double* Wt, int64_t nnz, int64_t n, int m,
                 const int64_t* colptr, double* part, double* Gout);

}  // namespace mfb

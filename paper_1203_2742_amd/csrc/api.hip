// C-ABI entry points: plan upload, workspace layout, level-scheduled
// launches and status readback.  Every numeric step runs in the kernels of
// kernels.hip; this file only marshals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "mfb_internal.h"

#include "kernels.h"

namespace mfb {
constexpr size_t ALIGN = 256;
// right-hand sides of one call: the grid's y extent of the per-RHS launches
constexpr int kMaxRhs = 65535;
static inline size_t up(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

static int64_t scratch_doubles(Op op, const std::vector<Level>& lv) {
  int64_t m = 0;
  for (const auto& L : lv) m = std::max(m, int64_t(L.count) * std::max<int64_t>(1, slot_doubles(op, L)));
  return m;
}
static bool up_op(Op op) {
  return op == OP_FACTOR || op == OP_PRODUCT || op == OP_VINV || op == OP_HUP || op == OP_IHUP;
}
static int64_t plan_scratch(const mfb_plan_s* p, Op op) {
  return scratch_doubles(op, up_op(op) ? p->up_levels : p->down_levels);
}
// Largest workgroup scratch of one launch of a schedule of independent
// fronts (the blocked segments).
static int64_t flat_scratch(const ClassSched& cs, Op op) {
  int64_t m = 0;
  for (const ClassSeg& g : cs.segs)
    if (g.cls == kRegClasses || g.cls == kFat)
      m = std::max(m, int64_t(g.lv.count) * std::max<int64_t>(1, slot_doubles(op, g.lv)));
  return m;
}
// Workgroup scratch (doubles) of the factored completion on front s (the
// layout of k_completion_factored; Ap is the parent's ancestor count).
static int64_t complf_slot(const mfb_plan_s* p, int32_t s) {
  const int64_t N = p->N[s], A = p->J[s] - N;
  const int32_t q = p->parent[s];
  const int64_t Ap = q >= 0 ? p->J[q] - p->N[q] : 0;
  return 3 * N * N + 2 * A * N + A * Ap + A * A + 2 * Ap + 64;
}
static int64_t factor_scratch(const mfb_plan_s* p) {
  int64_t complf = 1;
  for (int32_t s = 0; s < p->ns; ++s) complf = std::max(complf, complf_slot(p, s));
  return std::max({plan_scratch(p, OP_FACTOR), plan_scratch(p, OP_PRODUCT),
                   flat_scratch(p->cs_compl_flat, OP_COMPLETION), flat_scratch(p->cs_vinv, OP_VINV), complf});
}
static int64_t rhs_scratch(const mfb_plan_s* p) {
  int64_t flat = 0;
  for (const ClassSeg& g : p->cs_ihd_flat.segs)
    flat = std::max(flat, int64_t(g.lv.count) * std::max<int64_t>(1, slot_doubles(OP_IHDOWN, g.lv)));
  if (p->ihd_root >= 0) flat = std::max(flat, 2 * int64_t(p->N[p->ihd_root]) * p->N[p->ihd_root]);
  return std::max({plan_scratch(p, OP_HUP), plan_scratch(p, OP_HDOWN), flat, plan_scratch(p, OP_IHUP),
                   flat_scratch(p->cs_hfac, OP_HFAC), int64_t(1)});
}
static size_t factor_bytes(const mfb_plan_s* p) {
  const size_t nnz = size_t(std::max<int64_t>(1, p->nnz)), upd = size_t(std::max<int64_t>(1, p->update_doubles));
  // relaxed plans: one more V' array for the caller's values mapped in or out
  return (p->relaxed ? 4 : 3) * up(nnz * 8) + 3 * up(upd * 8) + up(size_t(std::max(1, p->ns)) * 8) + up(8) +
         up(sizeof(DevStatus)) + up(size_t(factor_scratch(p)) * 8);
}
static size_t rhs_bytes(const mfb_plan_s* p) {
  const size_t nnz = size_t(std::max<int64_t>(1, p->nnz)), upd = size_t(std::max<int64_t>(1, p->update_doubles));
  // relaxed plans: Y mapped onto V' (then T on V') per right-hand side
  return (upd + nnz + size_t(rhs_scratch(p)) + size_t(p->part_doubles) + (p->relaxed ? nnz : 0)) * 8 +
         size_t(std::max(1, p->ns)) * 4 + 6 * ALIGN;
}
}  // namespace mfb

using namespace mfb;

// Uploads the plan's index arrays to the current device (once).
static mfb_status_t ensure_device(mfb_plan_s* p) {
  std::lock_guard<std::mutex> g(p->mu);
  if (p->dmem) return MFB_OK;
  // all index arrays in one device allocation
  std::vector<int32_t> all(std::max(1, p->ns));
  for (int32_t i = 0; i < p->ns; ++i) all[i] = i;
  std::vector<int32_t> colidx(std::max<int64_t>(1, p->nnz));
  for (int64_t j = 0; j < p->n; ++j)
    for (int64_t e = p->colptr_h[j]; e < p->colptr_h[j + 1]; ++e) colidx[e] = int32_t(j);
  struct Blob {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Blob> blobs;
  size_t total = 0;
  auto add = [&](const void* src, size_t bytes) {
    blobs.push_back({src, bytes, total});
    total += up(std::max<size_t>(bytes, 8));
    return blobs.size() - 1;
  };
  auto v32 = [&](const std::vector<int32_t>& v) { return add(v.data(), v.size() * 4); };
  auto v64 = [&](const std::vector<int64_t>& v) { return add(v.data(), v.size() * 8); };
  size_t iN = v32(p->N), iJ = v32(p->J), iPar = v32(p->parent), iCp = v32(p->cptr), iCi = v32(p->cidx),
         iCb = v32(p->colbase), iCol = v64(p->col), iRb = v32(p->relbase), iRel = v32(p->rel),
         iAr = v64(p->arena), iVl = v32(p->vlabel), iUp = v32(p->up_list), iDn = v32(p->down_list),
         iAll = v32(all), iCidx = v32(colidx), iColptr = v64(p->colptr_h),
         iCf = v32(p->cs_factor.list), iCv = v32(p->cs_vinv.list),
         iCd = v32(p->cs_down.list), iCx = v32(p->cs_compl_flat.list), iCh = v32(p->cs_ihd_flat.list),
         iGm = v64(p->gmap), iHd = v32(p->cs_hdown.list), iPf = v32(p->cs_factor.pre),
         iPd = v32(p->cs_down.pre), iPh = v32(p->cs_hdown.pre), iGl = v32(p->cs_gather.list),
         iGp = v32(p->cs_gather.pre), iPi = v32(p->cs_ihd_flat.pre), iPx = v32(p->cs_compl_flat.pre),
         iHf = v32(p->cs_hfac.list), iBv = v32(p->cs_bigv.list), iPo = v64(p->poff), iVs = v32(p->vshift),
         iZp = v64(p->zpos), iUc = v64(p->ucolptr_h);
  void* d = nullptr;
  if (hipMalloc(&d, std::max<size_t>(total, 256)) != hipSuccess) return MFB_ENOMEM;
  for (const auto& b : blobs)
    if (b.bytes && hipMemcpy((char*)d + b.off, b.src, b.bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return MFB_EHIP;
    }
  auto at = [&](size_t i) { return (const void*)((char*)d + blobs[i].off); };
  p->dmem = d;
  DevPlan& P = p->dev;
  P.ns = p->ns;
  P.n = p->n;
  P.nnz = p->nnz;
  P.ncol = (const int32_t*)at(iN);
  P.nrow = (const int32_t*)at(iJ);
  P.parent = (const int32_t*)at(iPar);
  P.cptr = (const int32_t*)at(iCp);
  P.cidx = (const int32_t*)at(iCi);
  P.colbase = (const int32_t*)at(iCb);
  P.col = (const int64_t*)at(iCol);
  P.relbase = (const int32_t*)at(iRb);
  P.rel = (const int32_t*)at(iRel);
  P.arena = (const int64_t*)at(iAr);
  P.vlabel = (const int32_t*)at(iVl);
  P.big_a = p->big_a;
  P.poff = (const int64_t*)at(iPo);
  p->d_up_list = (const int32_t*)at(iUp);
  p->d_down_list = (const int32_t*)at(iDn);
  p->d_all_list = (const int32_t*)at(iAll);
  p->d_colidx = (const int32_t*)at(iCidx);
  p->d_colptr = (const int64_t*)at(iColptr);
  p->cs_factor.d_list = (const int32_t*)at(iCf);
  p->cs_vinv.d_list = (const int32_t*)at(iCv);
  p->cs_down.d_list = (const int32_t*)at(iCd);
  p->cs_compl_flat.d_list = (const int32_t*)at(iCx);
  p->cs_ihd_flat.d_list = (const int32_t*)at(iCh);
  p->d_gmap = p->gmap.empty() ? nullptr : (const int64_t*)at(iGm);
  p->cs_hdown.d_list = (const int32_t*)at(iHd);
  p->cs_factor.d_pre = (const int32_t*)at(iPf);
  p->cs_down.d_pre = (const int32_t*)at(iPd);
  p->cs_hdown.d_pre = (const int32_t*)at(iPh);
  p->cs_gather.d_list = (const int32_t*)at(iGl);
  p->cs_gather.d_pre = (const int32_t*)at(iGp);
  p->cs_ihd_flat.d_pre = (const int32_t*)at(iPi);
  p->cs_compl_flat.d_pre = (const int32_t*)at(iPx);
  p->cs_hfac.d_list = (const int32_t*)at(iHf);
  p->cs_bigv.d_list = (const int32_t*)at(iBv);
  if (p->relaxed) {
    p->d_vshift = (const int32_t*)at(iVs);
    p->d_zpos = (const int64_t*)at(iZp);
    p->d_ucolptr = (const int64_t*)at(iUc);
  }
  return MFB_OK;
}


namespace mfb {
struct ProfRec {
  int32_t kernel, level, nsuper, k;
  double bytes, flops;
  hipEvent_t e0, e1;
};
}  // namespace mfb

struct mfb_factor_s {
  mfb_plan_s* plan = nullptr;
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  char* ws = nullptr;
  double *R = nullptr, *LB = nullptr, *S = nullptr, *Vs = nullptr, *Vi = nullptr, *U = nullptr;
  // per supernode: the lower G with G^T G = S_AA and G^-1 (Hessian factor),
  // held in U and Vi while valid (gam_valid): the factor and product sweeps
  // use U as their update arena and Vi caches (S_AA)^-1 otherwise, so
  // building one cache invalidates the other
  double *Gam = nullptr, *Gami = nullptr;
  double *part = nullptr, *logdet = nullptr, *scratch = nullptr;
  // relaxed plans: the caller's X mapped onto V', and the V' outputs of the
  // product and the export before they are mapped back
  double* Xw = nullptr;
  DevStatus* st = nullptr;
  bool has_factor = false, s_valid = false, vinv_valid = false, gam_valid = false;
  // U holds the factored completion's R_s blocks (written by
  // mfb_completion_factored; every other user of U clears it)
  bool rfac_valid = false;
  hipStream_t last = nullptr;
};

#define HIPCHK(x)                         \
  do {                                    \
    if ((x) != hipSuccess) return MFB_EHIP; \
  } while (0)

static mfb_status_t launched() { return hipGetLastError() == hipSuccess ? MFB_OK : MFB_EHIP; }

extern "C" {

const char* mfb_strerror(mfb_status_t s) {
  switch (s) {
    case MFB_OK: return "ok";
    case MFB_EINVAL: return "invalid argument";
    case MFB_ENOTCHORDAL: return "pattern is not filled (chordal) in the given order";
    case MFB_ENOTPD: return "matrix is not positive definite";
    case MFB_ENOCOMPLETION: return "matrix has no positive definite completion";
    case MFB_ENOMEM: return "out of memory";
    case MFB_EHIP: return "HIP runtime error";
    case MFB_ESTATE: return "call order violated";
    case MFB_ESCRATCH: return "the call needs more than the library's static scratch";
  }
  return "unknown status";
}

mfb_status_t mfb_plan_symbolic(int64_t n, const int64_t* colptr, const int32_t* rowind,
                               uint32_t flags, mfb_plan_t* out) {
  if (!out) return MFB_EINVAL;
  *out = nullptr;
  mfb_plan_s* p = new (std::nothrow) mfb_plan_s();
  if (!p) return MFB_ENOMEM;
  mfb_status_t st = build_plan(n, colptr, rowind, flags, p);
  if (st) {
    delete p;
    return st;
  }
  *out = p;
  return MFB_OK;
}

mfb_status_t mfb_plan_symbolic_opts(int64_t n, const int64_t* colptr, const int32_t* rowind,
                                    const mfb_plan_opts_t* opts, mfb_plan_t* out) {
  if (!out || !opts) return MFB_EINVAL;
  *out = nullptr;
  if ((opts->wide_j != 0 && opts->wide_j < kWideJLow) || (opts->big_a != 0 && opts->big_a < kVExplicitMax))
    return MFB_EINVAL;
  if (opts->max_zero_frac >= 1.0 || opts->max_zero_frac != opts->max_zero_frac) return MFB_EINVAL;
  mfb_plan_s* p = new (std::nothrow) mfb_plan_s();
  if (!p) return MFB_ENOMEM;
  PlanTuning tune;
  tune.wide_j = opts->wide_j;
  tune.big_a = opts->big_a;
  mfb_status_t st = opts->max_zero_frac >= 0.0
                        ? build_plan_relaxed(n, colptr, rowind, opts->flags, opts->max_zero_frac, p, tune)
                        : build_plan(n, colptr, rowind, opts->flags, p, tune);
  if (st) {
    delete p;
    return st;
  }
  *out = p;
  return MFB_OK;
}

mfb_status_t mfb_plan_pattern(mfb_plan_t p, int64_t* colptr, int32_t* rowind) {
  if (!p) return MFB_EINVAL;
  if (colptr) std::copy(p->colptr_h.begin(), p->colptr_h.end(), colptr);
  if (rowind) std::copy(p->rowind_h.begin(), p->rowind_h.end(), rowind);
  return MFB_OK;
}

mfb_status_t mfb_plan_info(mfb_plan_t p, mfb_plan_info_t* o) {
  if (!p || !o) return MFB_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->n = p->n;
  o->nnz = p->nnz_user;
  o->nnz_relaxed = p->nnz;
  o->nsuper = p->ns;
  o->nlevels_up = int64_t(p->up_levels.size());
  o->nlevels_down = int64_t(p->down_levels.size());
  o->max_front = p->max_front;
  o->max_ncols = p->max_ncols;
  o->max_nanc = p->max_nanc;
  o->update_doubles = p->update_doubles;
  o->factor_workspace_bytes = factor_bytes(p);
  o->rhs_arena_bytes = rhs_bytes(p);
  o->flops_factor = p->fl_factor;
  o->flops_projinv = p->fl_projinv;
  o->flops_hessian = p->fl_hess;
  o->flops_inv_hessian = p->fl_invhess;
  o->flops_inv_hessian_x = p->fl_invhess_x;
  o->flops_completion = p->fl_completion;
  o->flops_product = p->fl_product;
  o->bytes_factor = p->by_factor;
  o->bytes_projinv = p->by_projinv;
  o->bytes_hessian = p->by_hess;
  o->bytes_inv_hessian = p->by_invhess;
  o->bytes_completion = p->by_completion;
  o->bytes_product = p->by_product;
  return MFB_OK;
}

mfb_status_t mfb_plan_supernodes(mfb_plan_t p, int32_t* snode_of, int32_t* sparent, int32_t* srep) {
  if (!p) return MFB_EINVAL;
  if (snode_of) std::copy(p->snode_of.begin(), p->snode_of.end(), snode_of);
  if (sparent) std::copy(p->parent.begin(), p->parent.end(), sparent);
  if (srep) std::copy(p->rep.begin(), p->rep.end(), srep);
  return MFB_OK;
}

void mfb_plan_destroy(mfb_plan_t p) {
  if (!p) return;
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
}

mfb_status_t mfb_factor_create(mfb_plan_t p, void* ws, size_t bytes, mfb_factor_t* out) {
  if (!p || !out) return MFB_EINVAL;
  *out = nullptr;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0 || bytes < factor_bytes(p)) return MFB_EINVAL;
  if (mfb_status_t st = ensure_device(p)) return st;
  mfb_factor_s* f = new (std::nothrow) mfb_factor_s();
  if (!f) return MFB_ENOMEM;
  f->plan = p;
  f->ws = (char*)ws;
  const size_t nnz = size_t(std::max<int64_t>(1, p->nnz)), upd = size_t(std::max<int64_t>(1, p->update_doubles));
  char* c = f->ws;
  auto take = [&](size_t b) {
    char* r = c;
    c += up(b);
    return r;
  };
  f->R = (double*)take(nnz * 8);
  f->LB = (double*)take(nnz * 8);
  f->S = (double*)take(nnz * 8);
  f->Vs = (double*)take(upd * 8);
  f->Vi = (double*)take(upd * 8);
  f->U = (double*)take(upd * 8);
  f->Gam = f->U;
  f->Gami = f->Vi;
  f->part = (double*)take(size_t(std::max(1, p->ns)) * 8);
  f->logdet = (double*)take(8);
  f->st = (DevStatus*)take(sizeof(DevStatus));
  f->scratch = (double*)take(size_t(factor_scratch(p)) * 8);
  if (p->relaxed) f->Xw = (double*)take(nnz * 8);
  *out = f;
  return MFB_OK;
}

void mfb_factor_destroy(mfb_factor_t f) {
  if (!f) return;
  for (auto& r : f->recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (auto e : f->pool) (void)hipEventDestroy(e);
  delete f;
}

// Canonical algorithmic bytes and flops of one level launch of kernel `kid`
// with k right-hand sides.  Bytes: every panel entry of the inputs read once
// and of the outputs written once, factor data shared by all right-hand
// sides counted once, and each update block produced written once and read
// once.  Flops: the canonical per-supernode counts split between the two
// sweeps of an operation.
static void canonical(int kid, const Level& L, int k, double* bytes, double* flops) {
  const double p = L.p, u = L.u, K = k;
  double b = 0, fl = 0;
  switch (kid) {
    case MFB_K_FACTOR: b = 2 * p + 2 * u; fl = L.n3 / 3 + L.n2a + L.na2; break;
    case MFB_K_PROJINV: b = 2 * p + 2 * u; fl = 2 * L.n3 / 3 + 2 * L.na2 + L.n2a; break;
    case MFB_K_HESS_UP: b = p + K * (2 * p + 2 * u); fl = K * (2 * L.na2 + 2 * L.n2a); break;
    case MFB_K_HESS_DOWN: b = p + u + K * (2 * p + 2 * u); fl = K * (4 * L.na2 + 4 * L.n2a + 3 * L.n3); break;
    case MFB_K_IHESS_DOWN: b = 2 * p + u + K * (2 * p + 2 * u); fl = K * (4 * L.na2 + 4 * L.n2a + 3 * L.n3); break;
    case MFB_K_IHESS_UP: b = p + K * (2 * p + 2 * u); fl = K * (3 * L.na2 + 3 * L.n2a); break;
    case MFB_K_COMPLETION: b = 4 * p + 3 * u; fl = L.a3 / 3 + 2 * L.na2 + L.n2a + L.n3; break;
    case MFB_K_VINV: b = 2 * u; fl = L.a3 / 3; break;
    case MFB_K_PRODUCT: b = 2 * p + 2 * u; fl = L.n3 / 3 + L.n2a + L.na2; break;
    case MFB_K_GATHER_V: b = K * 2 * u; fl = 0; break;
    case MFB_K_GAMMA: b = 3 * u; fl = 2 * L.a3 / 3; break;
    case MFB_K_HFACTOR: b = p + u + K * 2 * p; fl = K * (7 * L.n3 / 3 + 2 * L.n2a + L.na2); break;
    case MFB_K_HFACTOR_ADJ: b = p + u + K * 2 * p; fl = K * (2 * L.n3 + 2 * L.n2a + L.na2); break;
    case MFB_K_COMPL_SAA: b = 2 * u; fl = L.a3 / 3; break;
  }
  *bytes = 8 * b;
  *flops = fl;
}

static hipEvent_t pool_event(mfb_factor_s* f) {
  if (!f->pool.empty()) {
    hipEvent_t e = f->pool.back();
    f->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static mfb_status_t run_levels(mfb_factor_s* f, int kid, const std::vector<Level>& lv, const int32_t* dlist,
                               hipStream_t s, int k, Op op,
                               void (*launch)(mfb_factor_s*, const int32_t*, dim3, hipStream_t,
                                              int64_t, void*),
                               void* ctx) {
  int32_t level = -1;
  for (const auto& L : lv) {
    ++level;
    if (L.count == 0) continue;
    dim3 grid(unsigned(L.count), unsigned(k));
    ProfRec rec{kid, level, L.count, k, 0.0, 0.0, nullptr, nullptr};
    if (f->prof) {
      canonical(kid, L, k, &rec.bytes, &rec.flops);
      rec.e0 = pool_event(f);
      rec.e1 = pool_event(f);
      if (!rec.e0 || !rec.e1) return MFB_EHIP;
      if (hipEventRecord(rec.e0, s) != hipSuccess) return MFB_EHIP;
    }
    launch(f, dlist + L.begin, grid, s, std::max<int64_t>(1, slot_doubles(op, L)), ctx);
    if (hipGetLastError() != hipSuccess) return MFB_EHIP;
    if (f->prof) {
      if (hipEventRecord(rec.e1, s) != hipSuccess) return MFB_EHIP;
      f->recs.push_back(rec);
    }
  }
  return MFB_OK;
}

// As run_levels, over a class-split schedule: one launch per (level,
// class) segment; register classes get their own kernels.
// The launcher gets the segment: its class (g.cls: a register class,
// kRegClasses for the blocked kernels, kWide for the wide-front launches),
// its fronts cs.d_list + g.lv.begin and, for a wide segment, its tile
// numbering in cs.d_pre.
typedef void (*SegLaunch)(mfb_factor_s*, const ClassSched&, const ClassSeg&, dim3, hipStream_t, int64_t,
                          void*);
static mfb_status_t run_classes(mfb_factor_s* f, int kid, const ClassSched& cs, hipStream_t s, int k,
                                Op op, SegLaunch launch, void* ctx) {
  for (const ClassSeg& g : cs.segs) {
    const Level& L = g.lv;
    dim3 grid(unsigned(L.count), unsigned(k));
    ProfRec rec{kid, g.level, L.count, k, 0.0, 0.0, nullptr, nullptr};
    if (f->prof) {
      canonical(kid, L, k, &rec.bytes, &rec.flops);
      rec.e0 = pool_event(f);
      rec.e1 = pool_event(f);
      if (!rec.e0 || !rec.e1) return MFB_EHIP;
      if (hipEventRecord(rec.e0, s) != hipSuccess) return MFB_EHIP;
    }
    // register kernels use workgroup scratch only for the down sweeps'
    // intermediate products
    const bool reg_scratch = op == OP_HDOWN || op == OP_IHDOWN;
    const int64_t slot = g.cls < kRegClasses && !reg_scratch ? 1 : slot_doubles(op, L);
    launch(f, cs, g, grid, s, std::max<int64_t>(1, slot), ctx);
    if (hipGetLastError() != hipSuccess) return MFB_EHIP;
    if (f->prof) {
      if (hipEventRecord(rec.e1, s) != hipSuccess) return MFB_EHIP;
      f->recs.push_back(rec);
    }
  }
  return MFB_OK;
}

static WideTiles wide_tiles(const ClassSched& cs, const ClassSeg& g) {
  return WideTiles{cs.d_pre + g.aa_off, cs.d_pre + g.an_off, cs.d_pre + g.nn_off, g.n_aa, g.n_an, g.n_nn};
}
static FatGrid fat_grid(const ClassSeg& g) {
  return FatGrid{g.lv.maxN, g.lv.maxA, g.lv.maxJ, g.fat_panel, g.fat_fin};
}

// Packed A_s x A_s blocks of an input (S for the completion, T for the
// inverse Hessian, k right-hand sides) into `arena`: one elementwise launch
// with the plan's source map, else level by level from the parents.
static mfb_status_t gather_blocks(mfb_factor_s* f, hipStream_t s, int k, const double* src, double* arena,
                                  int64_t src_stride, int64_t arena_stride, int tag, double* part = nullptr,
                                  int64_t pstride = 0) {
  const mfb_plan_s* p = f->plan;
  struct Ctx { const double* src; double* arena; int64_t ss, as; int tag; double* part; int64_t ps; } ctx{
      src, arena, src_stride, arena_stride, tag, part, pstride};
  if (p->d_gmap) {
    return run_levels(
        f, MFB_K_GATHER_V, p->all_levels, p->d_all_list, s, k, OP_COMPLETION,
        [](mfb_factor_s* f, const int32_t*, dim3 g, hipStream_t s, int64_t, void* c) {
          Ctx* x = (Ctx*)c;
          const int64_t n = f->plan->update_doubles;
          const unsigned blocks = unsigned(std::min<int64_t>(2048, std::max<int64_t>(1, (n + NT_LAUNCH - 1) / NT_LAUNCH)));
          const dim3 grid(blocks, g.y);
          if (x->tag == 1)
            k_gather_map<1><<<grid, NT_LAUNCH, 0, s>>>(f->plan->d_gmap, n, x->src, x->arena, x->ss, x->as);
          else
            k_gather_map<2><<<grid, NT_LAUNCH, 0, s>>>(f->plan->d_gmap, n, x->src, x->arena, x->ss, x->as);
        },
        &ctx);
  }
  return run_classes(
      f, MFB_K_GATHER_V, p->cs_gather, s, k, OP_COMPLETION,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t, void* c) {
        Ctx* x = (Ctx*)c;
        launch_wide_extract(x->tag, dim3(unsigned(sg.n_aa), g.y), s, f->plan->dev, cs.d_list + sg.lv.begin,
                            cs.d_pre + sg.aa_off, sg.lv.count, x->src, x->arena, x->ss, x->as, f->LB, x->part,
                            x->ps);
      },
      &ctx);
}

mfb_status_t mfb_factor(mfb_factor_t f, const double* x, void* stream) {
  if (!f || (!x && f->plan->nnz)) return MFB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  // the cached state describes the previous X until this factor is enqueued
  f->has_factor = f->s_valid = f->vinv_valid = f->gam_valid = f->rfac_valid = false;
  k_reset_status<<<1, 64, 0, s>>>(f->st);
  const mfb_plan_s* p = f->plan;
  if (p->relaxed) {  // X on V' (zero on V' \ V)
    launch_relax_in(s, 1, x, p->nnz_user, p->d_vshift, p->d_zpos, int64_t(p->zpos.size()), f->Xw, p->nnz);
    x = f->Xw;
  }
  struct Ctx { const double* x; } ctx{x};
  mfb_status_t st = run_classes(
      f, MFB_K_FACTOR, f->plan->cs_factor, s, 1, OP_FACTOR,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (cls < kRegClasses) {
          launch_factor_reg(cls, g, s, f->plan->dev, list, ((Ctx*)c)->x, f->R, f->LB, f->U, f->part,
                            f->st);
        } else if (cls == kWide) {
          k_factor<true><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, ((Ctx*)c)->x, f->R, f->LB, f->U,
                                                 f->part, f->st, f->scratch, slot);
          launch_wide_update(0, dim3(unsigned(sg.n_aa)), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                             sg.lv.count, f->R, f->LB, nullptr, f->U, 0, f->scratch, slot, nullptr);
        } else if (cls == kFat) {
          const FatGrid fg = fat_grid(sg);
          launch_fat_panel(0, fg, 1, s, f->plan->dev, list, sg.lv.count, ((Ctx*)c)->x, f->U, 0, f->scratch, slot, nullptr);
          launch_fat_factor(fg, s, f->plan->dev, list, sg.lv.count, f->R, f->LB, f->part, f->st, f->scratch, slot);
          if (sg.n_aa)
            launch_wide_update(0, dim3(unsigned(sg.n_aa)), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                               sg.lv.count, f->R, f->LB, nullptr, f->U, 0, f->scratch, slot, nullptr);
        } else {
          k_factor<false><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, ((Ctx*)c)->x, f->R, f->LB, f->U,
                                                  f->part, f->st, f->scratch, slot);
        }
      },
      &ctx);
  if (st) return st;
  f->has_factor = true;
  return launched();
}

mfb_status_t mfb_logdet(mfb_factor_t f, double* out, void* stream) {
  if (!f || !out) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  k_logdet<<<1, NT_LAUNCH, 0, s>>>(f->part, f->plan->ns, out);
  return launched();
}

static mfb_status_t ensure_projinv(mfb_factor_s* f, hipStream_t s) {
  if (f->s_valid) return MFB_OK;
  mfb_status_t st = run_classes(
      f, MFB_K_PROJINV, f->plan->cs_down, s, 1, OP_FACTOR,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t, void*) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (cls < kRegClasses)
          launch_projinv_reg(cls, g, s, f->plan->dev, list, f->LB, f->S, f->Vs);
        else if (cls == kWide)
          launch_wide_projinv(s, f->plan->dev, list, wide_tiles(cs, sg), sg.lv.count, f->LB, f->S, f->Vs);
        else
          k_projinv<<<g, NT_DOWN, 0, s>>>(f->plan->dev, list, f->LB, f->S, f->Vs);
      },
      nullptr);
  if (st) return st;
  f->s_valid = true;
  return MFB_OK;
}

mfb_status_t mfb_projected_inverse(mfb_factor_t f, double* s_out, void* stream) {
  if (!f) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  f->s_valid = false;  // recompute on request
  mfb_status_t st = ensure_projinv(f, s);
  if (st) return st;
  const mfb_plan_s* p = f->plan;
  if (s_out && p->nnz) {
    if (p->relaxed)
      launch_relax_out(s, 1, f->S, p->nnz, p->d_vshift, s_out, p->nnz_user);
    else
      HIPCHK(hipMemcpyAsync(s_out, f->S, size_t(p->nnz) * 8, hipMemcpyDeviceToDevice, s));
  }
  return launched();
}

struct RhsArena {
  double *Ua, *Kt, *scr, *part;
  double* Yw;            // relaxed plans: Y, then T, on V' (k arrays)
  int64_t upd, pstride;  // pstride: doubles of the partial area per RHS
  int32_t* act;          // Hessian step 1 activity flags, ns per RHS
};
static mfb_status_t carve(mfb_factor_s* f, int k, void* arena, size_t bytes, RhsArena* a) {
  const mfb_plan_s* p = f->plan;
  if (!arena || (reinterpret_cast<uintptr_t>(arena) % ALIGN) != 0) return MFB_EINVAL;
  if (k > kMaxRhs || bytes < size_t(k) * rhs_bytes(p)) return MFB_EINVAL;
  const size_t nnz = size_t(std::max<int64_t>(1, p->nnz)), upd = size_t(std::max<int64_t>(1, p->update_doubles));
  char* c = (char*)arena;
  a->upd = int64_t(upd);
  a->Ua = (double*)c;
  c += up(size_t(k) * upd * 8);
  a->Kt = (double*)c;
  c += up(size_t(k) * nnz * 8);
  a->pstride = p->part_doubles;
  a->part = (double*)c;
  c += up(size_t(k) * size_t(std::max<int64_t>(1, p->part_doubles)) * 8);
  a->act = (int32_t*)c;
  c += up(size_t(k) * size_t(std::max(1, p->ns)) * 4);
  a->Yw = nullptr;
  if (p->relaxed) {
    a->Yw = (double*)c;
    c += up(size_t(k) * nnz * 8);
  }
  a->scr = (double*)c;
  return MFB_OK;
}

// Hessian step 1 (leaf-to-root) on k right-hand sides: K into a.Kt.
struct HessCtx {
  const double* y;
  double* t;
  RhsArena a;
};
static mfb_status_t hess_up_run(mfb_factor_s* f, int32_t k, const double* y, const RhsArena& a, hipStream_t s) {
  HessCtx ctx{y, nullptr, a};
  using Ctx = HessCtx;
  // every front active until its step-1 kernel finds its subtree's part of
  // Y zero (pruning; fat fronts keep the flag)
  launch_fill_i32(s, a.act, int64_t(k) * f->plan->ns, 1);
  return run_classes(
      f, MFB_K_HESS_UP, f->plan->cs_factor, s, k, OP_HUP,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        Ctx* x = (Ctx*)c;
        if (cls < kRegClasses) {
          launch_hess_up_reg(cls, g, s, f->plan->dev, list, f->LB, x->y, x->a.Kt, x->a.Ua, x->a.upd, x->a.act);
        } else if (cls == kWide) {
          k_hess_up<true><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, f->LB, x->y, x->a.Kt, x->a.Ua,
                                                  x->a.upd, x->a.scr, slot, x->a.act);
          launch_wide_update(1, dim3(unsigned(sg.n_aa), g.y), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                             sg.lv.count, nullptr, f->LB, x->a.Kt, x->a.Ua, x->a.upd, x->a.scr, slot, x->a.act);
        } else if (cls == kFat) {
          const FatGrid fg = fat_grid(sg);
          const int k = int(g.y);
          launch_fat_panel(1, fg, k, s, f->plan->dev, list, sg.lv.count, x->y, x->a.Ua, x->a.upd, x->a.scr, slot,
                           x->a.act);
          launch_fat_up_fin(1, fg, k, s, f->plan->dev, list, sg.lv.count, f->R, f->LB, nullptr, x->a.Kt, x->a.scr,
                            slot);
          if (sg.n_aa)
            launch_wide_update(1, dim3(unsigned(sg.n_aa), g.y), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                               sg.lv.count, nullptr, f->LB, x->a.Kt, x->a.Ua, x->a.upd, x->a.scr, slot,
                               x->a.act);
        } else {
          k_hess_up<false><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, f->LB, x->y, x->a.Kt, x->a.Ua,
                                                   x->a.upd, x->a.scr, slot, x->a.act);
        }
      },
      &ctx);
}

// Hessian steps 2 and 3 (root-to-leaf) from K in a.Kt: T into t.
static mfb_status_t hess_down_run(mfb_factor_s* f, int32_t k, double* t, const RhsArena& a, hipStream_t s) {
  HessCtx ctx{nullptr, t, a};
  using Ctx = HessCtx;
  mfb_status_t st;
  if (f->plan->hd_root >= 0) {
    // the root front: two tile-parallel products (Hessian steps 2+3 with A = 0)
    const mfb_plan_s* p = f->plan;
    const int N = p->N[p->hd_root];
    const unsigned tiles = unsigned((N + 63) / 64);
    const int32_t* root = p->d_all_list + p->hd_root;
    ProfRec rec{MFB_K_HESS_DOWN, 0, 1, k, 0.0, 0.0, nullptr, nullptr};
    if (f->prof) {
      canonical(MFB_K_HESS_DOWN, p->down_levels[0], k, &rec.bytes, &rec.flops);
      rec.e0 = pool_event(f);
      rec.e1 = pool_event(f);
      if (!rec.e0 || !rec.e1) return MFB_EHIP;
      if (hipEventRecord(rec.e0, s) != hipSuccess) return MFB_EHIP;
    }
    const dim3 grid(tiles, tiles, unsigned(k));
    k_hess_down_root<0><<<grid, NT_LAUNCH, 0, s>>>(p->dev, root, f->LB, a.Kt, t, a.scr, int64_t(N) * N);
    k_hess_down_root<1><<<grid, NT_LAUNCH, 0, s>>>(p->dev, root, f->LB, a.Kt, t, a.scr, int64_t(N) * N);
    if (hipGetLastError() != hipSuccess) return MFB_EHIP;
    if (f->prof) {
      if (hipEventRecord(rec.e1, s) != hipSuccess) return MFB_EHIP;
      f->recs.push_back(rec);
    }
  }
  st = run_classes(
      f, MFB_K_HESS_DOWN, f->plan->cs_hdown, s, k, OP_HDOWN,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        Ctx* x = (Ctx*)c;
        if (cls < kRegClasses)
          launch_hess_down_reg(cls, g, s, f->plan->dev, list, f->LB, f->Vs, x->a.Kt, x->t, x->a.Ua,
                               x->a.upd, x->a.scr, slot);
        else if (cls == kWide)
          launch_wide_hess_down(int(g.y), sg.lv.maxN, sg.lv.maxA, s, f->plan->dev, list, wide_tiles(cs, sg),
                                sg.lv.count, f->LB, f->Vs, x->a.Kt, x->t, x->a.Ua, x->a.upd, x->a.scr, slot,
                                x->a.part, x->a.pstride);
        else
          k_hess_down<<<g, NT_DOWN, 0, s>>>(f->plan->dev, list, f->LB, f->Vs, x->a.Kt, x->t, x->a.Ua,
                                              x->a.upd, x->a.scr, slot);
      },
      &ctx);
  if (st) return st;
  return launched();
}

// Hessian steps on k right-hand sides with the per-RHS arena `a`.
static mfb_status_t hessian_run(mfb_factor_s* f, int32_t k, const double* y, double* t, const RhsArena& a,
                                hipStream_t s) {
  mfb_status_t st;
  f->last = s;
  if ((st = ensure_projinv(f, s))) return st;
  const mfb_plan_s* p = f->plan;
  if (!p->relaxed) {
    if ((st = hess_up_run(f, k, y, a, s))) return st;
    return hess_down_run(f, k, t, a, s);
  }
  // Y onto V' in a.Yw; step 1 is its only reader, so steps 2-3 write T there
  launch_relax_in(s, k, y, p->nnz_user, p->d_vshift, p->d_zpos, int64_t(p->zpos.size()), a.Yw, p->nnz);
  if ((st = hess_up_run(f, k, a.Yw, a, s))) return st;
  if ((st = hess_down_run(f, k, a.Yw, a, s))) return st;
  launch_relax_out(s, k, a.Yw, p->nnz, p->d_vshift, t, p->nnz_user);
  return launched();
}

mfb_status_t mfb_hessian(mfb_factor_t f, int32_t k, const double* y, double* t, void* arena,
                         size_t bytes, void* stream) {
  if (!f || k < 0) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!y || !t) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  RhsArena a;
  mfb_status_t st = carve(f, k, arena, bytes, &a);
  if (st) return st;
  return hessian_run(f, k, y, t, a, (hipStream_t)stream);
}

// ---- the Hessian without a caller arena (callers that cannot allocate) ----
// The per-RHS arena comes from `scratch`, a fixed device array of this
// file.  In host code the array's name is not a device address: its
// address on the current device is looked up once per device with
// hipGetSymbolAddress and kept in static_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[MFB_STATIC_SCRATCH_BYTES];
static std::mutex static_scratch_mu;
constexpr int kMaxDevices = 64;
static void* static_scratch_ptr[kMaxDevices];

static mfb_status_t static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MFB_EHIP;
  std::lock_guard<std::mutex> g(static_scratch_mu);
  if (!static_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MFB_EHIP;
    static_scratch_ptr[dev] = ptr;
  }
  *out = static_scratch_ptr[dev];
  return MFB_OK;
}

mfb_status_t mfb_hessian_static(mfb_factor_t f, int32_t k, const double* y, double* t, void* stream) {
  if (!f || k < 0) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!y || !t) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  if (size_t(k) * rhs_bytes(f->plan) > size_t(MFB_STATIC_SCRATCH_BYTES)) return MFB_ESCRATCH;
  void* arena = nullptr;
  mfb_status_t st = static_scratch(&arena);
  if (st) return st;
  RhsArena a;
  if ((st = carve(f, k, arena, size_t(MFB_STATIC_SCRATCH_BYTES), &a))) return st;
  // no launch records: they would create HIP events
  const bool prof = f->prof;
  f->prof = false;
  st = hessian_run(f, k, y, t, a, (hipStream_t)stream);
  f->prof = prof;
  return st;
}

static mfb_status_t ensure_vinv(mfb_factor_s* f, hipStream_t s) {
  if (f->vinv_valid) return MFB_OK;
  mfb_status_t st = run_classes(
      f, MFB_K_VINV, f->plan->cs_vinv, s, 1, OP_VINV,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void*) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (cls < kRegClasses)
          launch_vinv_reg(cls, g, s, f->plan->dev, list, f->Vs, f->Vi, f->st);
        else if (cls == kBigV)  // factor formed in U, its inverse into Vi
          launch_bigv(0, sg.lv.maxA, sg.lv.count, sg.acnt.empty() ? nullptr : sg.acnt.data(), s, f->plan->dev,
                      list, f->Vs, f->U, f->Vi, f->st);
        else
          k_vinv<<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, f->Vs, f->Vi, f->st, f->scratch, slot);
      },
      nullptr);
  if (st) return st;
  f->vinv_valid = true;
  f->gam_valid = false;  // Vi and U overwrote Gami and Gam
  f->rfac_valid = false;
  return MFB_OK;
}

// G (lower, G^T G = S_AA) and G^-1 per supernode for the current X.
static mfb_status_t ensure_gamma(mfb_factor_s* f, hipStream_t s) {
  if (f->gam_valid) return MFB_OK;
  mfb_status_t st = ensure_projinv(f, s);
  if (st) return st;
  st = run_classes(
      f, MFB_K_GAMMA, f->plan->cs_vinv, s, 1, OP_VINV,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t, void*) {
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (sg.cls == kBigV)
          launch_bigv(2, sg.lv.maxA, sg.lv.count, sg.acnt.empty() ? nullptr : sg.acnt.data(), s, f->plan->dev,
                      list, f->Vs, f->Gam, f->Gami, f->st);
        else
          launch_gamma(g, s, f->plan->dev, list, f->Vs, f->Gam, f->Gami, f->st);
      },
      nullptr);
  if (st) return st;
  f->gam_valid = true;
  f->vinv_valid = false;  // Gami overwrote Vi
  f->rfac_valid = false;
  return MFB_OK;
}

mfb_status_t mfb_hessian_factor(mfb_factor_t f, int32_t k, const double* y, double* w, void* arena,
                                size_t bytes, void* stream) {
  if (!f || k < 0 || f->plan->relaxed) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!y || !w) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  RhsArena a;
  mfb_status_t st = carve(f, k, arena, bytes, &a);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  if ((st = ensure_gamma(f, s))) return st;
  if ((st = hess_up_run(f, k, y, a, s))) return st;
  struct Ctx { double* w; RhsArena a; } ctx{w, a};
  st = run_classes(
      f, MFB_K_HFACTOR, f->plan->cs_hfac, s, k, OP_HFAC,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        Ctx* x = (Ctx*)c;
        launch_hfactor(g, s, f->plan->dev, cs.d_list + sg.lv.begin, f->R, f->Gam, x->a.Kt, x->w, x->a.scr, slot,
                       x->a.act);
      },
      &ctx);
  if (st) return st;
  return launched();
}

mfb_status_t mfb_hessian_factor_adj(mfb_factor_t f, int32_t k, const double* w, double* t, void* arena,
                                    size_t bytes, void* stream) {
  if (!f || k < 0 || f->plan->relaxed) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!w || !t) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  RhsArena a;
  mfb_status_t st = carve(f, k, arena, bytes, &a);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  if ((st = ensure_gamma(f, s))) return st;
  struct Ctx { const double* w; RhsArena a; } ctx{w, a};
  st = run_classes(
      f, MFB_K_HFACTOR_ADJ, f->plan->cs_hfac, s, k, OP_HFAC,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        Ctx* x = (Ctx*)c;
        launch_hfactor_adj(g, s, f->plan->dev, cs.d_list + sg.lv.begin, f->R, f->Gami, x->w, x->a.Kt, x->a.scr,
                           slot);
      },
      &ctx);
  if (st) return st;
  return hess_down_run(f, k, t, a, s);
}

size_t mfb_gram_arena_bytes(mfb_plan_t p, int32_t m) {
  if (!p || m <= 0) return 0;
  const GramShape g = gram_shape(std::max<int64_t>(1, p->nnz_user), p->n, m);
  return size_t(g.part_doubles) * 8;
}

mfb_status_t mfb_gram(mfb_plan_t p, int32_t m, const double* w, double* gout, void* arena, size_t bytes,
                      void* stream) {
  if (!p || m < 0) return MFB_EINVAL;
  if (m == 0) return MFB_OK;
  if (!w || !gout || p->nnz_user == 0) return MFB_EINVAL;
  if (!arena || (reinterpret_cast<uintptr_t>(arena) % ALIGN) != 0 || bytes < mfb_gram_arena_bytes(p, m))
    return MFB_EINVAL;
  if (mfb_status_t st = ensure_device(p)) return st;
  // the vectors are on the caller's pattern V (also for a relaxed plan)
  const GramShape g = gram_shape(p->nnz_user, p->n, m);
  launch_gram((hipStream_t)stream, g, w, p->nnz_user, p->n, m, p->relaxed ? p->d_ucolptr : p->d_colptr,
              (double*)arena, gout);
  return launched();
}

// Inverse Hessian steps 1+2 on the root front when it runs alone (A = 0):
// three tile-parallel products.
static mfb_status_t ihess_root(mfb_factor_s* f, int32_t k, const double* t, const RhsArena& a, hipStream_t s) {
  if (f->plan->ihd_root < 0) return MFB_OK;
  const mfb_plan_s* p = f->plan;
  const int N = p->N[p->ihd_root];
  const unsigned tiles = unsigned((N + 63) / 64);
  const int32_t* root = p->d_all_list + p->ihd_root;
  ProfRec rec{MFB_K_IHESS_DOWN, 0, 1, k, 0.0, 0.0, nullptr, nullptr};
  if (f->prof) {
    canonical(MFB_K_IHESS_DOWN, p->down_levels[0], k, &rec.bytes, &rec.flops);
    rec.e0 = pool_event(f);
    rec.e1 = pool_event(f);
    if (!rec.e0 || !rec.e1) return MFB_EHIP;
    if (hipEventRecord(rec.e0, s) != hipSuccess) return MFB_EHIP;
  }
  const dim3 grid(tiles, tiles, unsigned(k));
  const int64_t ws = 2 * int64_t(N) * N;
  k_ihess_down_root<0><<<grid, NT_LAUNCH, 0, s>>>(p->dev, root, f->R, t, a.Kt, a.scr, ws);
  k_ihess_down_root<1><<<grid, NT_LAUNCH, 0, s>>>(p->dev, root, f->R, t, a.Kt, a.scr, ws);
  k_ihess_down_root<2><<<grid, NT_LAUNCH, 0, s>>>(p->dev, root, f->R, t, a.Kt, a.scr, ws);
  if (hipGetLastError() != hipSuccess) return MFB_EHIP;
  if (f->prof) {
    if (hipEventRecord(rec.e1, s) != hipSuccess) return MFB_EHIP;
    f->recs.push_back(rec);
  }
  return MFB_OK;
}

// Inverse Hessian step 3 (leaf-to-root) from K in a.Kt: Y into y.
static mfb_status_t ihess_up_run(mfb_factor_s* f, int32_t k, double* y, const RhsArena& a, hipStream_t s) {
  struct Ctx { const double* t; double* y; RhsArena a; } ctx{nullptr, y, a};
  mfb_status_t st;
  st = run_classes(
      f, MFB_K_IHESS_UP, f->plan->cs_factor, s, k, OP_IHUP,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        Ctx* x = (Ctx*)c;
        if (cls < kRegClasses) {
          launch_ihess_up_reg(cls, g, s, f->plan->dev, list, f->LB, x->a.Kt, x->y, x->a.Ua, x->a.upd);
        } else if (cls == kWide) {
          launch_up_panel_tiles(UP_IHESS, sg.lv.maxA, sg.lv.count, int(g.y), s, f->plan->dev, list, nullptr, f->LB,
                                x->a.Kt, x->y, x->a.Ua, x->a.upd, x->a.scr, slot);
          launch_wide_update(2, dim3(unsigned(sg.n_aa), g.y), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                             sg.lv.count, nullptr, f->LB, x->a.Kt, x->a.Ua, x->a.upd, x->a.scr, slot, nullptr);
        } else if (cls == kFat) {
          const FatGrid fg = fat_grid(sg);
          const int k = int(g.y);
          launch_fat_panel(2, fg, k, s, f->plan->dev, list, sg.lv.count, nullptr, x->a.Ua, x->a.upd, x->a.scr,
                           slot, nullptr);
          launch_fat_up_fin(2, fg, k, s, f->plan->dev, list, sg.lv.count, f->R, f->LB, x->y, x->a.Kt, x->a.scr,
                            slot);
          if (sg.n_aa)
            launch_wide_update(2, dim3(unsigned(sg.n_aa), g.y), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                               sg.lv.count, nullptr, f->LB, x->a.Kt, x->a.Ua, x->a.upd, x->a.scr, slot, nullptr);
        } else {
          k_ihess_up<false><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, f->LB, x->a.Kt, x->y, x->a.Ua,
                                                    x->a.upd, x->a.scr, slot);
        }
      },
      &ctx);
  if (st) return st;
  return launched();
}

mfb_status_t mfb_inv_hessian(mfb_factor_t f, int32_t k, const double* t, double* y, void* arena,
                             size_t bytes, void* stream) {
  if (!f || k < 0 || f->plan->relaxed) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!y || !t) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  RhsArena a;
  mfb_status_t st = carve(f, k, arena, bytes, &a);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  if ((st = ensure_projinv(f, s))) return st;
  if ((st = ensure_vinv(f, s))) return st;
  struct Ctx { const double* t; double* y; RhsArena a; } ctx{t, y, a};
  // V'_s = T_{A_s A_s} for every supernode and right-hand side (root-to-leaf
  // gathers), then steps 1+2 of all fronts, which are independent
  // (without the source map the level gathers also leave the partial
  // products T_AA L of the fronts that have a partial area)
  st = gather_blocks(f, s, k, t, a.Ua, f->plan->nnz, a.upd, 1, a.part, a.pstride);
  if (st) return st;
  if ((st = ihess_root(f, k, t, a, s))) return st;
  st = run_classes(
      f, MFB_K_IHESS_DOWN, f->plan->cs_ihd_flat, s, k, OP_IHDOWN,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        Ctx* x = (Ctx*)c;
        if (cls < kRegClasses)
          launch_ihess_down_reg(cls, g, s, f->plan->dev, list, f->R, f->LB, f->Vi, x->t, x->a.Kt,
                                x->a.Ua, x->a.upd, x->a.scr, slot);
        else if (cls == kFat)
          launch_fat_ihess(fat_grid(sg), int(g.y), s, f->plan->dev, list, sg.lv.count, f->R, f->LB, f->Vi, x->t,
                           x->a.Kt, x->a.Ua, x->a.upd, x->a.scr, slot, f->plan->d_gmap ? nullptr : x->a.part,
                           x->a.pstride);
        else
          k_ihess_down<<<g, NT_DOWN, 0, s>>>(f->plan->dev, list, f->R, f->LB, f->Vi, x->t, x->a.Kt,
                                               x->a.Ua, x->a.upd, x->a.scr, slot);
      },
      &ctx);
  if (st) return st;
  return ihess_up_run(f, k, y, ctx.a, s);
}

mfb_status_t mfb_inv_hessian_factored(mfb_factor_t f, int32_t k, const double* t, double* y, void* arena,
                                      size_t bytes, void* stream) {
  if (!f || k < 0 || f->plan->relaxed) return MFB_EINVAL;
  if (k == 0) return MFB_OK;
  if (!y || !t) return MFB_EINVAL;
  if (!f->has_factor || !f->s_valid || !f->rfac_valid) return MFB_ESTATE;
  RhsArena a;
  mfb_status_t st = carve(f, k, arena, bytes, &a);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  const mfb_plan_s* p = f->plan;
  // T_{A_s A_s} for every supernode (root-to-leaf gathers), then steps 1+2
  // of all fronts, which are independent, with S_AA through R_s in U
  st = gather_blocks(f, s, k, t, a.Ua, p->nnz, a.upd, 1, a.part, a.pstride);
  if (st) return st;
  if ((st = ihess_root(f, k, t, a, s))) return st;
  for (const ClassSeg& sg : p->cs_ihd_flat.segs) {
    const int64_t slot = std::max<int64_t>(1, slot_doubles(OP_IHDOWN, sg.lv));
    launch_ihess_down_factored(dim3(unsigned(sg.lv.count), unsigned(k)), s, p->dev,
                               p->cs_ihd_flat.d_list + sg.lv.begin, f->R, f->LB, f->U, t, a.Kt, a.Ua, a.upd,
                               a.scr, slot);
    if (hipGetLastError() != hipSuccess) return MFB_EHIP;
  }
  return ihess_up_run(f, k, y, a, s);
}

mfb_status_t mfb_completion(mfb_factor_t f, const double* sin, void* stream) {
  if (!f || (!sin && f->plan->nnz) || f->plan->relaxed) return MFB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  f->has_factor = f->s_valid = f->vinv_valid = f->gam_valid = f->rfac_valid = false;
  k_reset_status<<<1, 64, 0, s>>>(f->st);
  struct Ctx { const double* s; } ctx{sin};
  // V_s = S_{A_s A_s} for every supernode (root-to-leaf gathers), then the
  // fronts' sweeps, which need nothing but their own S and V_s
  mfb_status_t st = gather_blocks(f, s, 1, sin, f->Vs, 0, 0, 2);
  if (st) return st;
  // the blocks S_AA with A > big_a: Cholesky factor (formed in U) and its
  // inverse C_V^-1 into Vi, tile-parallel over all those fronts (their
  // A^3/3 is counted here, not in the per-front launches that follow)
  st = run_classes(
      f, MFB_K_COMPL_SAA, f->plan->cs_bigv, s, 1, OP_VINV,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3, hipStream_t s, int64_t, void*) {
        launch_bigv(1, sg.lv.maxA, sg.lv.count, sg.acnt.empty() ? nullptr : sg.acnt.data(), s, f->plan->dev,
                    cs.d_list + sg.lv.begin, f->Vs, f->U, f->Vi, f->st);
      },
      nullptr);
  if (st) return st;
  st = run_classes(
      f, MFB_K_COMPLETION, f->plan->cs_compl_flat, s, 1, OP_COMPLETION,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (cls < kRegClasses)
          launch_completion_reg(cls, g, s, f->plan->dev, list, ((Ctx*)c)->s, f->R, f->LB, f->S, f->Vs,
                                f->Vi, f->part, f->st);
        else if (cls == kFat)
          launch_fat_completion(fat_grid(sg), s, f->plan->dev, list, sg.lv.count, ((Ctx*)c)->s, f->R, f->LB, f->S,
                                f->Vs, f->Vi, f->part, f->st, f->scratch, slot);
        else
          k_completion<<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, ((Ctx*)c)->s, f->R, f->LB, f->S,
                                               f->Vs, f->Vi, f->part, f->st, f->scratch, slot);
      },
      &ctx);
  if (st) return st;
  f->has_factor = true;
  f->s_valid = true;
  f->vinv_valid = true;
  return launched();
}

mfb_status_t mfb_completion_factored(mfb_factor_t f, const double* sin, void* stream) {
  if (!f || (!sin && f->plan->nnz) || f->plan->relaxed) return MFB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  f->has_factor = f->s_valid = f->vinv_valid = f->gam_valid = f->rfac_valid = false;
  k_reset_status<<<1, 64, 0, s>>>(f->st);
  const mfb_plan_s* p = f->plan;
  // V_s = S_{A_s A_s} for the Hessian sweeps that may follow (the
  // completion itself reads S and the parents' R_p)
  mfb_status_t st = gather_blocks(f, s, 1, sin, f->Vs, 0, 0, 2);
  if (st) return st;
  // level by level from the roots; a level's fronts in launches whose
  // scratch stays within the factor's scratch area
  const int64_t budget = factor_scratch(p);
  for (const Level& L : p->down_levels) {
    int64_t sl = 1;
    for (int32_t t = L.begin; t < L.begin + L.count; ++t) sl = std::max(sl, complf_slot(p, p->down_list[t]));
    const int32_t chunk = int32_t(std::max<int64_t>(1, std::min<int64_t>(L.count, budget / sl)));
    for (int32_t b = 0; b < L.count; b += chunk) {
      const int32_t c = std::min(chunk, L.count - b);
      launch_completion_factored(dim3(unsigned(c)), s, p->dev, p->d_down_list + L.begin + b, sin, f->R, f->LB,
                                 f->S, f->U, f->part, f->st, f->scratch, sl);
      if (hipGetLastError() != hipSuccess) return MFB_EHIP;
    }
  }
  f->has_factor = true;
  f->s_valid = true;
  f->rfac_valid = true;
  return launched();
}

mfb_status_t mfb_cholesky_product(mfb_factor_t f, double* x, void* stream) {
  if (!f || (!x && f->plan->nnz)) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  f->gam_valid = false;  // the sweep's update arena U holds the Hessian factor's G
  f->rfac_valid = false;
  const mfb_plan_s* p = f->plan;
  double* xo = x;
  if (p->relaxed) x = f->Xw;  // on V', restricted to V below
  struct Ctx { double* x; } ctx{x};
  mfb_status_t st = run_classes(
      f, MFB_K_PRODUCT, f->plan->cs_factor, s, 1, OP_PRODUCT,
      [](mfb_factor_s* f, const ClassSched& cs, const ClassSeg& sg, dim3 g, hipStream_t s, int64_t slot, void* c) {
        const int cls = sg.cls;
        const int32_t* list = cs.d_list + sg.lv.begin;
        if (cls < kRegClasses) {
          launch_product_reg(cls, g, s, f->plan->dev, list, f->R, ((Ctx*)c)->x, f->U);
        } else if (cls == kWide) {
          launch_up_panel_tiles(UP_PRODUCT, sg.lv.maxA, sg.lv.count, 1, s, f->plan->dev, list, f->R, nullptr, nullptr,
                                ((Ctx*)c)->x, f->U, 0, f->scratch, slot);
          launch_wide_update(3, dim3(unsigned(sg.n_aa)), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                             sg.lv.count, f->R, f->LB, nullptr, f->U, 0, f->scratch, slot, nullptr);
        } else if (cls == kFat) {
          const FatGrid fg = fat_grid(sg);
          launch_fat_panel(3, fg, 1, s, f->plan->dev, list, sg.lv.count, nullptr, f->U, 0, f->scratch, slot, nullptr);
          launch_fat_up_fin(0, fg, 1, s, f->plan->dev, list, sg.lv.count, f->R, f->LB, ((Ctx*)c)->x, nullptr,
                            f->scratch, slot);
          if (sg.n_aa)
            launch_wide_update(3, dim3(unsigned(sg.n_aa)), s, f->plan->dev, list, cs.d_pre + sg.aa_off,
                               sg.lv.count, f->R, f->LB, nullptr, f->U, 0, f->scratch, slot, nullptr);
        } else {
          k_product<false><<<g, NT_LAUNCH, 0, s>>>(f->plan->dev, list, f->R, ((Ctx*)c)->x, f->U,
                                                   f->scratch, slot);
        }
      },
      &ctx);
  if (st) return st;
  if (p->relaxed) launch_relax_out(s, 1, f->Xw, p->nnz, p->d_vshift, xo, p->nnz_user);
  return launched();
}

mfb_status_t mfb_factor_export_ldl(mfb_factor_t f, double* out, void* stream) {
  if (!f || (!out && f->plan->nnz)) return MFB_EINVAL;
  if (!f->has_factor) return MFB_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  f->last = s;
  const mfb_plan_s* p = f->plan;
  const int64_t nnz = p->nnz;
  if (nnz == 0) return MFB_OK;
  const int blocks = int(std::min<int64_t>((nnz + NT_LAUNCH - 1) / NT_LAUNCH, 4096));
  k_export_ldl<<<blocks, NT_LAUNCH, 0, s>>>(f->R, p->d_colptr, p->d_colidx, nnz, p->relaxed ? f->Xw : out);
  if (p->relaxed) launch_relax_out(s, 1, f->Xw, nnz, p->d_vshift, out, p->nnz_user);
  return launched();
}

mfb_status_t mfb_get_status(mfb_factor_t f, int64_t* bad) {
  if (!f) return MFB_EINVAL;
  if (bad) *bad = -1;
  if (hipStreamSynchronize(f->last) != hipSuccess) return MFB_EHIP;
  DevStatus h{};
  if (hipMemcpy(&h, f->st, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return MFB_EHIP;
  if (h.code == 0) return MFB_OK;
  if (bad && h.bad != ~0ull) *bad = int64_t(h.bad);
  return h.code;
}

struct mfb_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

mfb_status_t mfb_step_graph_create(mfb_factor_t f, uint32_t ops, const mfb_step_args_t* a, mfb_graph_t* out) {
  if (!f || !a || !out || !(ops & MFB_STEP_FACTOR)) return MFB_EINVAL;
  *out = nullptr;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MFB_EHIP;
  const bool prof = f->prof;
  f->prof = false;  // no events inside the graph
  mfb_status_t st = MFB_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = MFB_EHIP;
  } else {
    st = mfb_factor(f, a->x, cs);
    if (!st && (ops & MFB_STEP_LOGDET)) st = mfb_logdet(f, a->logdet, cs);
    if (!st && (ops & MFB_STEP_PROJINV)) st = mfb_projected_inverse(f, a->s, cs);
    if (!st && (ops & MFB_STEP_HESSIAN)) st = mfb_hessian(f, a->k, a->y, a->t, a->arena, a->arena_bytes, cs);
    if (!st && (ops & MFB_STEP_INV_HESSIAN))
      st = mfb_inv_hessian(f, a->k, a->t_in, a->y_out, a->arena, a->arena_bytes, cs);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess && !st) st = MFB_EHIP;
    if (!st) {
      mfb_graph_s* h = new (std::nothrow) mfb_graph_s();
      if (!h) {
        st = MFB_ENOMEM;
      } else if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        delete h;
        st = MFB_EHIP;
      } else {
        h->graph = g;
        g = nullptr;
        *out = h;
      }
    }
    if (g) (void)hipGraphDestroy(g);
  }
  f->prof = prof;
  (void)hipStreamDestroy(cs);
  return st;
}

mfb_status_t mfb_graph_launch(mfb_graph_t g, void* stream) {
  if (!g) return MFB_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? MFB_OK : MFB_EHIP;
}

void mfb_graph_destroy(mfb_graph_t g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

mfb_status_t mfb_profile_enable(mfb_factor_t f, int32_t enable) {
  if (!f) return MFB_EINVAL;
  f->prof = enable != 0;
  return MFB_OK;
}

mfb_status_t mfb_profile_read(mfb_factor_t f, mfb_profile_entry_t* out, int64_t cap, int64_t* count) {
  if (!f || (cap > 0 && !out)) return MFB_EINVAL;
  if (count) *count = int64_t(f->recs.size());
  if (!out) return MFB_OK;  // count only
  int64_t i = 0;
  mfb_status_t st = MFB_OK;
  for (auto& r : f->recs) {
    if (i < cap) {
      float ms = 0.f;
      if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
        st = MFB_EHIP;
      out[i] = mfb_profile_entry_t{r.kernel, r.level, r.nsuper, r.k, double(ms), r.bytes, r.flops};
    }
    ++i;
    f->pool.push_back(r.e0);
    f->pool.push_back(r.e1);
  }
  f->recs.clear();
  return st;
}

const char* mfb_kernel_name(int32_t kernel) {
  static const char* names[MFB_K_COUNT] = {"k_factor", "k_projinv", "k_hess_up", "k_hess_down",
                                           "k_ihess_down", "k_ihess_up", "k_completion", "k_vinv",
                                           "k_product", "k_gather", "k_gamma", "k_hfactor",
                                           "k_hfactor_adj", "k_bigv"};
  return (kernel >= 0 && kernel < MFB_K_COUNT) ? names[kernel] : "unknown";
}

}  // extern "C"

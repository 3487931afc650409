/*
 * mfb.h -- multifrontal log-det barrier kernels for one AMD MI355X (gfx950).
 *
 * The library evaluates the logarithmic barrier f(X) = -log det X of the
 * cone of positive definite matrices with a filled (chordal) sparsity
 * pattern V, and the dual barrier f_*, by the supernodal multifrontal
 * recursions of Andersen, Dahl and Vandenberghe, "Logarithmic barriers for
 * sparse matrix cones":
 *
 *   factor                X = L D L^T over the clique tree (Algorithm 7.1)
 *   logdet                log det X, so f(X) = -logdet (Section 1.1)
 *   projected_inverse     S = P(X^-1) = -grad f(X) (eq. e-grad-def, Algorithm 7.2)
 *   hessian               T = P(X^-1 Y X^-1) for k matrices Y (Section 5.2, Algorithm 5.1
 *                         in block form)
 *   inv_hessian           Y = H^-1(T), i.e. solve P(X^-1 Y X^-1) = T (Section 5.3,
 *                         Algorithm 5.2 in block form)
 *   completion            the factor of X-hat with P(X-hat^-1) = S, i.e. -grad f_*(S)
 *                         (eq. e-Xhat-eq, Algorithm 7.3); f_*(S) = log det X-hat - n
 *   cholesky_product      values of L D L^T on V (Algorithm 3.2 in block form)
 *   factor_export_ldl     the scalar factors D, L in the pattern's CCS order
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Values.  All numeric values are IEEE double.  A symmetric matrix in S^n_V
 * is passed as its lower triangle (diagonal included) in the compressed
 * column (CCS) order of the pattern handed to mfb_plan_symbolic: one double
 * per pattern entry, column by column, rows ascending.  k right-hand sides
 * are k such arrays stored back to back (k * nnz doubles).
 *
 * Memory.  Pointers named *_dev are device pointers on the current HIP
 * device; pointers named *_host are host pointers.  The caller owns every
 * value array, every workspace and every arena and keeps them alive until
 * the work that uses them has completed on the stream.  The library owns
 * only its opaque handles and the plan's device-resident index arrays
 * (allocated once in mfb_plan_symbolic, freed by mfb_plan_destroy).  The
 * numeric entry points do not allocate device memory.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Numeric entry points only enqueue work.  Argument and state
 * errors are returned synchronously (MFB_EINVAL, MFB_ESTATE) and enqueue
 * nothing.  Numerical failures (a pivot block that is not positive
 * definite) are recorded on the device and read back by mfb_get_status;
 * outputs computed after such a failure are unspecified.  A factor handle
 * may be used from one stream at a time.
 *
 * Determinism.  Children are assembled in a fixed order and no atomics are
 * used, so repeated calls with equal inputs give bitwise equal outputs.
 */
#ifndef MFB_H
#define MFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mfb_status_t;
#define MFB_OK 0
#define MFB_EINVAL 1          /* bad argument (null pointer, bad CCS, k < 0, short buffer) */
#define MFB_ENOTCHORDAL 2     /* the pattern is not filled in the given order */
#define MFB_ENOTPD 3          /* X (or the S_AA blocks for inv_hessian) not positive definite */
#define MFB_ENOCOMPLETION 4   /* S has no positive definite completion */
#define MFB_ENOMEM 5          /* host or device allocation failed */
#define MFB_EHIP 6            /* a HIP runtime call failed */
#define MFB_ESTATE 7          /* call order violated (e.g. hessian before factor) */
#define MFB_ESCRATCH 8        /* mfb_hessian_static: k right-hand sides need more than
                                 MFB_STATIC_SCRATCH_BYTES of scratch */

typedef struct mfb_plan_s* mfb_plan_t;
typedef struct mfb_factor_s* mfb_factor_t;

/* Plan flags. */
#define MFB_PLAN_TIE_LAST 1u  /* Pothen-Sun tie-break: join the highest-labelled
                                 eligible child instead of the lowest */
#define MFB_PLAN_NO_GATHER_MAP 2u  /* keep no CCS source map of the packed update
                                      blocks: the completion and the inverse
                                      Hessian gather their input blocks level by
                                      level from the parents instead of in one
                                      launch (plans with more than 2^25 block
                                      entries never keep the map) */
#define MFB_PLAN_WIDE_LOW 4u  /* run the tile-parallel wide-front kernels from
                                 front order 65 instead of 193 (fronts with at
                                 most 64 columns and a nonempty ancestor set),
                                 and the tile-parallel factorization of the
                                 blocks S_AA from order 193 instead of 257;
                                 for testing those kernels on small patterns.
                                 Without it, the environment variables
                                 MFB_WIDE_J and MFB_BIG_A, when set, replace
                                 those two defaults (192, 256) at plan build;
                                 mfb_plan_symbolic_opts sets them directly */

typedef struct {
  int64_t n;                 /* order of X */
  int64_t nnz;               /* entries of V in the lower triangle, diagonal included */
  int64_t nsuper;            /* supernodes (cliques) */
  int64_t nlevels_up;        /* levels of the leaf-to-root schedule (tree height + 1) */
  int64_t nlevels_down;      /* levels of the root-to-leaf schedule (tree depth + 1) */
  int64_t max_front;         /* max |J_s| = |N_s| + |A_s| */
  int64_t max_ncols;         /* max |N_s| */
  int64_t max_nanc;          /* max |A_s| */
  int64_t update_doubles;    /* sum over supernodes of |A|(|A|+1)/2 */
  size_t factor_workspace_bytes;  /* device bytes for mfb_factor_create */
  size_t rhs_arena_bytes;         /* device bytes per right-hand side for hessian/inv_hessian */
  /* canonical algorithmic flop counts (LAPACK conventions, summed per supernode) */
  double flops_factor, flops_projinv, flops_hessian, flops_inv_hessian, flops_inv_hessian_x,
      flops_completion, flops_product;
  /* canonical algorithmic bytes of one call (k = 1): every input entry read
   * once, every output entry written once, each update block written once
   * and read once, 8 bytes per double; the per-launch figures of the
   * profiler (mfb_profile_read) sum to these.  The inverse Hessian's figure
   * leaves out the one-time (S_AA)^-1 cache. */
  double bytes_factor, bytes_projinv, bytes_hessian, bytes_inv_hessian, bytes_completion, bytes_product;
  /* entries of the pattern the sweeps run on: nnz for a plan of
   * mfb_plan_symbolic, |V'| for one of mfb_plan_symbolic_opts with max_zero_frac >= 0 (the other
   * sizes, counts and bytes above then describe V' too, except nnz) */
  int64_t nnz_relaxed;
} mfb_plan_info_t;

/* Symbolic analysis of a filled pattern (Sections 2 and 6; Algorithm 6.1).
 *   n          order (>= 0).
 *   colptr_host  int64[n+1], colptr[0] = 0, strictly increasing.
 *   rowind_host  int32[colptr[n]]: rows of each column, sorted ascending, the
 *              diagonal first, all < n.  Both arrays are read during the call only.
 *   flags      MFB_PLAN_* bits.
 *   out        receives the plan; immutable afterwards and safe to share between
 *              factor handles and threads.
 * Builds the elimination tree (parent(j) = min I_j), checks that the pattern is
 * filled in the given order (I_j \ {parent} within I_parent for every j:
 * eqs. e-filled, e-etree-ch), forms the supernodes and the clique tree by the
 * Pothen-Sun algorithm, the relative indices of every A_s inside its parent
 * clique, and the level schedules.  Host work only: the index arrays are
 * uploaded to the current device by the first mfb_factor_create.  Returns
 * MFB_EINVAL for malformed CCS, MFB_ENOTCHORDAL when the pattern is not
 * filled, MFB_ENOMEM on allocation failure. */
mfb_status_t mfb_plan_symbolic(int64_t n, const int64_t* colptr_host, const int32_t* rowind_host,
                               uint32_t flags, mfb_plan_t* out);

/* The same analysis with options.  Fields:
 *   flags          MFB_PLAN_* bits.
 *   max_zero_frac  relaxed supernodes (the amalgamation Section 8 names as a
 *                  refinement) when >= 0, the fundamental partition when < 0.
 *                  The fundamental partition of V is formed first; then,
 *                  from the leaves up, each supernode absorbs the child whose
 *                  merge adds the fewest explicit zeros, provided the merged
 *                  supernode (columns N, ancestors A) holds at most
 *                  max_zero_frac * (N(N+1)/2 + N A) zeros, counting those it
 *                  inherited.  The result is a filled pattern V' that
 *                  contains V, with fewer, larger supernodes and far smaller
 *                  update blocks; the sweeps run on V' and the caller's
 *                  arrays stay on V (nnz entries of V, CCS order as above),
 *                  mapped in and out by the entry points.  0 gives the
 *                  fundamental partition.
 *   wide_j         fronts of order above this run tile-parallel (>= 64; 0:
 *                  the default 192, or 64 under MFB_PLAN_WIDE_LOW, or the
 *                  environment's MFB_WIDE_J).
 *   big_a          blocks S_AA with more rows than this are factored
 *                  tile-parallel (>= 192; 0: the default 256, or 192 under
 *                  MFB_PLAN_WIDE_LOW, or the environment's MFB_BIG_A).
 * The thresholds change which kernels run, not the results beyond rounding.
 * A relaxed plan is exact on V' for the operations whose inputs vanish on
 * V' \ V and whose outputs restricted to V are those of V: mfb_factor,
 * mfb_logdet, mfb_projected_inverse, mfb_hessian (and mfb_hessian_static),
 * mfb_cholesky_product and mfb_factor_export_ldl.  The inverse Hessian and
 * the completion take inputs that are unknown on V' \ V, and the Hessian
 * factor depends on the partition: mfb_inv_hessian, mfb_completion,
 * mfb_hessian_factor and mfb_hessian_factor_adj return MFB_EINVAL on a
 * relaxed plan.  Errors as mfb_plan_symbolic, and MFB_EINVAL for a NULL
 * opts, max_zero_frac >= 1 or NaN, or a threshold below its minimum. */
typedef struct {
  uint32_t flags;
  double max_zero_frac;
  int32_t wide_j;
  int32_t big_a;
} mfb_plan_opts_t;
mfb_status_t mfb_plan_symbolic_opts(int64_t n, const int64_t* colptr_host, const int32_t* rowind_host,
                                    const mfb_plan_opts_t* opts, mfb_plan_t* out);

/* The pattern the plan's sweeps run on (V, or V' for a relaxed plan), in
 * the CCS form mfb_plan_symbolic takes.
 *   colptr_host  int64[n+1] or NULL; rowind_host  int32[nnz_relaxed] or NULL. */
mfb_status_t mfb_plan_pattern(mfb_plan_t plan, int64_t* colptr_host, int32_t* rowind_host);

/* Sizes, workspace requirements and canonical flop counts of a plan. */
mfb_status_t mfb_plan_info(mfb_plan_t plan, mfb_plan_info_t* out_host);

/* The supernode partition and clique tree (Section 6.2-6.3), for inspection.
 *   snode_of_host  int32[n]: supernode of every column (0-based, clique-tree
 *                  postorder numbering), may be NULL.
 *   sparent_host   int32[nsuper]: parent supernode, -1 for roots, may be NULL.
 *   srep_host      int32[nsuper]: representative vertex (min N_s), may be NULL. */
mfb_status_t mfb_plan_supernodes(mfb_plan_t plan, int32_t* snode_of_host, int32_t* sparent_host,
                                 int32_t* srep_host);

/* Frees the plan and its device arrays.  No factor handle may still use it. */
void mfb_plan_destroy(mfb_plan_t plan);

/* Numeric state for one X on one plan.
 *   workspace_dev  device buffer of at least plan_info.factor_workspace_bytes,
 *                  256-byte aligned; owned by the caller, used until
 *                  mfb_factor_destroy.  It holds the Cholesky factor, the
 *                  cached projected inverse and the per-supernode S_AA blocks.
 * Returns MFB_EINVAL for a short or misaligned buffer. */
mfb_status_t mfb_factor_create(mfb_plan_t plan, void* workspace_dev, size_t workspace_bytes,
                               mfb_factor_t* out);

/* Frees the handle (never the caller's memory). */
void mfb_factor_destroy(mfb_factor_t f);

/* Algorithm 7.1: factor X = L D L^T (x_dev: nnz doubles, read only).
 * Invalidates the cached projected inverse.  A pivot block that is not
 * positive definite sets MFB_ENOTPD (see mfb_get_status). */
mfb_status_t mfb_factor(mfb_factor_t f, const double* x_dev, void* stream);

/* log det X = sum over supernodes of log det D_NN (Section 1.1, f = -logdet),
 * written as one double to out_dev.  Requires a factor (mfb_factor or
 * mfb_completion); for a completion it is log det X-hat, and
 * f_*(S) = logdet - n. */
mfb_status_t mfb_logdet(mfb_factor_t f, double* out_dev, void* stream);

/* Algorithm 7.2: S = P(X^-1) (eq. e-sn-gradient-1/2) written to s_dev
 * (nnz doubles).  The result is also cached in the handle for hessian and
 * inv_hessian.  s_dev may be NULL to fill the cache only. */
mfb_status_t mfb_projected_inverse(mfb_factor_t f, double* s_dev, void* stream);

/* Hessian of f at X applied to k matrices (Section 5.2):
 *   t_r = P(X^-1 y_r X^-1),  r = 0..k-1.
 *   y_dev, t_dev: k*nnz doubles each (may not overlap).
 *   arena_dev: at least k * plan_info.rhs_arena_bytes device bytes,
 *   256-byte aligned, caller-owned scratch.
 * Computes the projected inverse first if it is not cached.  k = 0 is a
 * no-op; k above 65535 gives MFB_EINVAL (this holds for every call that
 * takes k right-hand sides and an arena). */
mfb_status_t mfb_hessian(mfb_factor_t f, int32_t k, const double* y_dev, double* t_dev,
                         void* arena_dev, size_t arena_bytes, void* stream);

/* Inverse Hessian (Section 5.3): y_r = H^-1(t_r), the unique y_r in S^n_V
 * with P(X^-1 y_r X^-1) = t_r.  Same buffer rules as mfb_hessian.  Uses and
 * caches (S_AA)^-1 per supernode for the current X. */
mfb_status_t mfb_inv_hessian(mfb_factor_t f, int32_t k, const double* t_dev, double* y_dev,
                             void* arena_dev, size_t arena_bytes, void* stream);

/* mfb_hessian without a caller-provided arena, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same inputs, outputs and
 * kernels as mfb_hessian; the per-RHS arena is carved from a fixed device
 * array of MFB_STATIC_SCRATCH_BYTES owned by the library, one per GPU it
 * runs on, held until the process ends.  The call allocates nothing and
 * records no launch profile.  Returns MFB_ESCRATCH (enqueueing nothing)
 * when k * plan_info.rhs_arena_bytes exceeds MFB_STATIC_SCRATCH_BYTES.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other threads, other factor handles) race and must
 * be serialized by the caller.  The array keeps the last call's contents;
 * every entry a call reads it has written first. */
#define MFB_STATIC_SCRATCH_BYTES (256u << 20)
mfb_status_t mfb_hessian_static(mfb_factor_t f, int32_t k, const double* y_dev, double* t_dev,
                                void* stream);

/* Hessian factor (Section 5.4, Algorithm 5.3): w_r = R(y_r), r = 0..k-1,
 * the linear map with H = R^adj o R, so that y . H(y') = R(y) . R(y')
 * under the trace inner product of S^n_V.  Per column j of the scalar
 * factor X = L D L^T, with K the result of step 1 of the Hessian:
 * W_jj = K_jj / D_jj and W_{I_j j} = R_j^T K_{I_j j} / sqrt(D_jj), where
 * S_{I_j I_j} = R_j R_j^T with R_j upper triangular.  w_dev receives the
 * lower-triangle values of W in the pattern's CCS order.  Same buffer
 * rules as mfb_hessian (y_dev, w_dev: k*nnz doubles, not overlapping).
 * Computes the projected inverse if it is not cached, and computes and
 * caches per supernode the lower triangular G with G^T G = S_AA and G^-1
 * for the current X.  That cache shares the handle's storage with the
 * (S_AA)^-1 cache of mfb_inv_hessian and with the update arena of
 * mfb_cholesky_product: after either of those, the next Hessian-factor
 * call rebuilds it (and after a Hessian-factor call the next inverse
 * Hessian rebuilds its own). */
mfb_status_t mfb_hessian_factor(mfb_factor_t f, int32_t k, const double* y_dev, double* w_dev,
                                void* arena_dev, size_t arena_bytes, void* stream);

/* Adjoint Hessian factor (Section 5.4, Algorithm 5.4): t_r = R^adj(w_r),
 * the adjoint of mfb_hessian_factor under the trace inner product, so that
 * mfb_hessian_factor_adj(mfb_hessian_factor(y)) = mfb_hessian(y).  Same
 * buffer rules and caches as mfb_hessian_factor. */
mfb_status_t mfb_hessian_factor_adj(mfb_factor_t f, int32_t k, const double* w_dev, double* t_dev,
                                    void* arena_dev, size_t arena_bytes, void* stream);

/* Gram matrix of m vectors of S^n_V under the trace inner product
 * (diagonal entries once, strict-lower entries twice):
 * g(i, j) = w_i . w_j, i, j = 0..m-1.  With w_i = R(a_i) from
 * mfb_hessian_factor this is the interior-point Schur complement matrix
 * a_i . H(a_j) (Sections 1.3 and 5.4).
 *   w_dev: m*nnz doubles (vector i at offset i*nnz); g_dev: m*m doubles
 *   (symmetric, both triangles written).
 *   arena_dev: at least mfb_gram_arena_bytes(p, m) device bytes, 256-byte
 *   aligned, caller-owned scratch for partial sums.
 * The sum runs in a fixed order (results do not depend on timing).
 * m = 0 is a no-op; a plan with nnz = 0 gives MFB_EINVAL. */
size_t mfb_gram_arena_bytes(mfb_plan_t p, int32_t m);
mfb_status_t mfb_gram(mfb_plan_t p, int32_t m, const double* w_dev, double* g_dev, void* arena_dev,
                      size_t arena_bytes, void* stream);

/* Algorithm 7.3: matrix completion.  Given S in S^n_V with a positive definite
 * completion (s_dev, nnz doubles), replaces the handle's factor by the factor
 * of X-hat, the X in S^n_V with P(X^-1) = S (eq. e-Xhat-eq); S itself becomes
 * the cached projected inverse.  Failure (S_AA or a Schur complement not
 * positive definite) sets MFB_ENOCOMPLETION. */
mfb_status_t mfb_completion(mfb_factor_t f, const double* s_dev, void* stream);

/* Matrix completion with factored update matrices (Algorithm 4.3, in the
 * supernodal form of the paper's appendix on supernodal algorithms): the
 * same result and handle state as mfb_completion, computed root to leaf
 * with each V_s = S_{A_s A_s} carried as V_s = R_s R_s^T (R_s upper
 * triangular) and R_s obtained from the parent's factor by deleting rows
 * and retriangularizing with Householder reflections (eqs.
 * e-mfp-compl-3-factored and e-mf-compl-2-factored), so that no S_AA is
 * factored from scratch.  Then L_AN = -R_s^-T R_s^-1 S_AN (eq.
 * e-mf-compl-1-factored).  One launch per level of the clique tree, one
 * workgroup per front.  Arguments, buffers and errors as mfb_completion
 * (MFB_ENOCOMPLETION when a retriangularized block or a Schur complement
 * is not positive definite; MFB_EINVAL on a relaxed plan).  The R_s blocks
 * are left in the handle's update arena; the cached inverse blocks of
 * S_AA are not formed (the inverse Hessian forms them on its first call). */
mfb_status_t mfb_completion_factored(mfb_factor_t f, const double* s_dev, void* stream);

/* Inverse Hessian at the X of the last mfb_completion_factored (Algorithm
 * 5.2 with the improvement noted after it): steps 1 and 2 use S_{A_s A_s}
 * through the factors V_s = R_s R_s^T that the factored completion left in
 * the handle, K_AN = R_s^-T R_s^-1 (M_AN D) by two triangular solves per
 * front, so no inverse of S_AA is formed; step 3 as in mfb_inv_hessian.
 * One workgroup per front and right-hand side for steps 1 and 2.  Buffer
 * rules as mfb_hessian.  MFB_ESTATE unless the handle's last factor came
 * from mfb_completion_factored and no call that rewrites its update arena
 * (mfb_factor, mfb_completion, mfb_cholesky_product, mfb_inv_hessian,
 * mfb_hessian_factor, mfb_hessian_factor_adj) followed it; MFB_EINVAL on a
 * relaxed plan. */
mfb_status_t mfb_inv_hessian_factored(mfb_factor_t f, int32_t k, const double* t_dev, double* y_dev,
                                      void* arena_dev, size_t arena_bytes, void* stream);

/* Algorithm 3.2 (block form): values of L D L^T on V, written to x_dev
 * (nnz doubles).  For a completion this gives X-hat = -grad f_*(S). */
mfb_status_t mfb_cholesky_product(mfb_factor_t f, double* x_dev, void* stream);

/* The scalar factorization X = L D L^T with unit lower L (Section 2): D_jj
 * in the diagonal slot of column j and L_ij in the strict-lower slots, in
 * the pattern's CCS order (ldl_dev, nnz doubles).  Unique for positive
 * definite X, hence independent of the supernode partition. */
mfb_status_t mfb_factor_export_ldl(mfb_factor_t f, double* ldl_dev, void* stream);

/* Synchronizes the handle's last stream and reports the first numerical
 * failure since the last mfb_factor / mfb_completion: MFB_OK, MFB_ENOTPD or
 * MFB_ENOCOMPLETION.  *bad_index_host (may be NULL) receives the failing
 * column in the user's labels, or -1. */
mfb_status_t mfb_get_status(mfb_factor_t f, int64_t* bad_index_host);

/* Static description of a status code. */
const char* mfb_strerror(mfb_status_t s);

/* ---- captured steps ------------------------------------------------------ */

/* One interior-point step on a factor handle captured once as a HIP graph
 * and replayed with a single launch: the level-by-level launches of every
 * operation in `ops` (flags below, run in the order listed) with the
 * buffers of `args` baked in.  The step starts with the factorization
 * (MFB_STEP_FACTOR is required), so every cache the later operations use
 * is rebuilt inside each replay.  Same buffer rules as the individual
 * entry points; the buffers, the arena and the factor handle must outlive
 * the graph, and a replay must not overlap another use of the handle.
 * Capture records no memset and allocates nothing on the device; the plan's
 * device arrays exist from mfb_factor_create on, so no eager call is needed
 * first.  Creation runs no kernel but leaves the handle's host-side state as
 * the captured calls leave it: launch the graph once before using the
 * handle eagerly.  Errors: MFB_EINVAL (NULL f, args or out, or
 * MFB_STEP_FACTOR missing), the argument errors of the captured calls,
 * MFB_EHIP when capture or instantiation fails; *out is NULL on error. */
#define MFB_STEP_FACTOR 1u       /* mfb_factor(args->x) */
#define MFB_STEP_LOGDET 2u       /* mfb_logdet -> args->logdet (1 double) */
#define MFB_STEP_PROJINV 4u      /* mfb_projected_inverse -> args->s */
#define MFB_STEP_HESSIAN 8u      /* mfb_hessian(args->k, args->y -> args->t) */
#define MFB_STEP_INV_HESSIAN 16u /* mfb_inv_hessian(args->k, args->t_in -> args->y_out) */
typedef struct {
  const double* x;
  double* logdet;
  double* s;
  int32_t k;
  const double* y;
  double* t;
  const double* t_in;
  double* y_out;
  void* arena;        /* at least k * rhs_arena_bytes, 256-byte aligned */
  size_t arena_bytes;
} mfb_step_args_t;
typedef struct mfb_graph_s* mfb_graph_t;
mfb_status_t mfb_step_graph_create(mfb_factor_t f, uint32_t ops, const mfb_step_args_t* args,
                                   mfb_graph_t* out);
/* Enqueues one replay of the captured step on `stream` (MFB_EINVAL for a
 * NULL graph, MFB_EHIP when the launch fails). */
mfb_status_t mfb_graph_launch(mfb_graph_t g, void* stream);
/* Frees the graph; the caller makes sure no replay is still running.
 * NULL is ignored. */
void mfb_graph_destroy(mfb_graph_t g);

/* ---- launch profiling (tracing aid; off by default) -------------------- */

/* Kernel identifiers reported by the profiler. */
#define MFB_K_FACTOR 0       /* Algorithm 7.1, one leaf-to-root level */
#define MFB_K_PROJINV 1      /* Algorithm 7.2, one root-to-leaf level */
#define MFB_K_HESS_UP 2      /* Hessian step 1 (Algorithm 5.1 in block form) */
#define MFB_K_HESS_DOWN 3    /* Hessian steps 2-3 */
#define MFB_K_IHESS_DOWN 4   /* inverse Hessian steps 1-2 (Algorithm 5.2) */
#define MFB_K_IHESS_UP 5     /* inverse Hessian step 3 */
#define MFB_K_COMPLETION 6   /* Algorithm 7.3 */
#define MFB_K_VINV 7         /* (S_AA)^-1 per supernode */
#define MFB_K_PRODUCT 8      /* Algorithm 3.2 in block form */
#define MFB_K_GATHER_V 9     /* gather of the input blocks S_AA (completion) or T_AA
                                (inverse Hessian): one launch of k_gather_map with
                                the plan's source map, else one k_wide_extract
                                launch per root-to-leaf level (profile name
                                "k_gather") */
#define MFB_K_GAMMA 10       /* G (G^T G = S_AA) and G^-1 per supernode (Hessian factor) */
#define MFB_K_HFACTOR 11     /* step-1 output to W = R(Y), Algorithm 5.3 */
#define MFB_K_HFACTOR_ADJ 12 /* W to the step-2 input of the Hessian's root-to-leaf sweep,
                                Algorithm 5.4 */
#define MFB_K_COMPL_SAA 13   /* the completion's tile-parallel factorization of the blocks
                                S_AA above the plan's size threshold (profile name "k_bigv") */
#define MFB_K_COUNT 14

typedef struct {
  int32_t kernel;   /* MFB_K_* */
  int32_t level;    /* level index in its schedule */
  int32_t nsuper;   /* supernodes in the launch */
  int32_t k;        /* right-hand sides in the launch */
  double ms;        /* launch duration between HIP events recorded on its stream */
  double bytes;     /* canonical algorithmic bytes moved by the launch */
  double flops;     /* canonical algorithmic flops of the launch */
} mfb_profile_entry_t;

/* Enables (1) or disables (0) profiling on a factor handle.  While enabled,
 * every kernel launch of the handle is bracketed by two HIP events on its
 * stream.  Entries accumulate until read. */
mfb_status_t mfb_profile_enable(mfb_factor_t f, int32_t enable);

/* Synchronizes the recorded events and copies up to `cap` entries (in
 * launch order) to out_host; *count_host receives the number recorded.  The
 * recorded list is then cleared.  With out_host NULL only the count is
 * returned and nothing is cleared. */
mfb_status_t mfb_profile_read(mfb_factor_t f, mfb_profile_entry_t* out_host, int64_t cap,
                              int64_t* count_host);

/* Kernel symbol name of an MFB_K_* identifier (as seen by rocprofv3). */
const char* mfb_kernel_name(int32_t kernel);

#ifdef __cplusplus
}
#endif
#endif /* MFB_H */

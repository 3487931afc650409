/*
 * CPU oracle for the multifrontal barrier recursions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that
 * the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the library
 * never does, and the two share no code.
 *
 * Everything is double precision, scalar, column by column, following the
 * paper's multifrontal (non-supernodal) algorithms on compressed column
 * storage (CCS) of the lower triangle of a filled pattern V:
 *
 *   orc_factor       Algorithm 3.1 (multifrontal Cholesky, Section 3.1,
 *                    eqs. e-mf-chol-1 / e-mf-chol-2)
 *   orc_logdet       f(X) = -sum log D_jj (Section 1.1, Section 3)
 *   orc_product      Algorithm 3.2 (Cholesky product, eq. e-mf-prod)
 *   orc_projinv      Algorithm 4.1 (projected inverse, eqs. e-mf-gradient-1/2)
 *   orc_completion   Algorithm 4.2 (matrix completion, eqs. e-mf-compl-1/2)
 *   orc_completion_factored  Algorithm 4.3 (the same with factored update
 *                    matrices V_j = R_j R_j^T, Householder row deletion)
 *   orc_hessian      Algorithm 5.1 (Hessian evaluation, Section 5.2)
 *   orc_inv_hessian  Algorithm 5.2 (inverse Hessian evaluation, Section 5.3)
 *   orc_hessian_factor      Algorithm 5.3 (W = R(Y), Section 5.4)
 *   orc_hessian_factor_adj  Algorithm 5.4 (T = R^adj(W), Section 5.4)
 *
 * Storage: colptr[n+1] (int64), rowind[nnz] (int32), rows sorted ascending
 * in every column with the diagonal first.  Because V is filled, column j
 * holds exactly the index set J_j = {j} U I_j (Section 2).  The factor is
 * exchanged as "ldl": D_jj in the diagonal slot of column j and L_ij in the
 * strict-lower slots (L unit lower triangular), i.e. X = L D L^T.
 *
 * Readings of the paper used here:
 *  - The elimination tree may be a forest (Section 2): columns with an
 *    empty I_j are roots; their update matrices are empty.
 *  - Children of a vertex are visited in ascending label order (fixed
 *    summation order).
 *  - Equation e-compl-lin prints T_{I_j j}^T in its (2,1) block; the
 *    matrix is symmetric, so it is read as T_{I_j j}.
 *  - Algorithm 5.2 step 3 prints K_{I_j}^T; read K_{I_j j}^T.
 *  - Steps 2 of Algorithms 5.1 and 5.2 may visit columns in any order; the
 *    oracle takes S_{I_j I_j} directly from the CCS array of S (binary
 *    search per entry), not from the optional V_j recursion.
 *  - Algorithm 5.3 needs a factor S_{I_j I_j} = R_j R_j^T with R_j upper
 *    triangular; the oracle forms it from the dense matrix by the
 *    "reverse" Cholesky (Cholesky of the index-reversed matrix).
 *
 * Return codes: 0 ok; ORC_EINVAL bad CCS; ORC_ENOTCHORDAL some I_c is not
 * contained in J_parent(c); ORC_ENOTPD / ORC_ENOCOMPL a non-positive pivot
 * (the failing column is written to *bad when bad != NULL); ORC_ENOMEM.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOTCHORDAL 2
#define ORC_ENOTPD 3
#define ORC_ENOCOMPL 4
#define ORC_ENOMEM 5

typedef struct {
  int64_t n;
  const int64_t* cp;
  const int32_t* ri;
  int64_t* parent;  /* -1 for roots */
  int64_t* chead;   /* first child (ascending list) */
  int64_t* cnext;   /* next sibling */
} tree_t;

/* --- symbolic ----------------------------------------------------------- */

static int check_ccs(int64_t n, const int64_t* cp, const int32_t* ri) {
  if (n < 0 || !cp || (n > 0 && !ri)) return ORC_EINVAL;
  if (cp[0] != 0) return ORC_EINVAL;
  for (int64_t j = 0; j < n; ++j) {
    if (cp[j + 1] <= cp[j]) return ORC_EINVAL;
    if (ri[cp[j]] != j) return ORC_EINVAL;
    for (int64_t p = cp[j] + 1; p < cp[j + 1]; ++p)
      if (ri[p] <= ri[p - 1] || ri[p] >= n) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* Elimination tree: parent(j) = min I_j (Section 2); children sorted. */
static int tree_init(tree_t* t, int64_t n, const int64_t* cp, const int32_t* ri) {
  int rc = check_ccs(n, cp, ri);
  if (rc) return rc;
  t->n = n; t->cp = cp; t->ri = ri;
  t->parent = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  t->chead = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  t->cnext = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  if (!t->parent || !t->chead || !t->cnext) return ORC_ENOMEM;
  for (int64_t j = 0; j < n; ++j) { t->chead[j] = -1; t->cnext[j] = -1; }
  for (int64_t j = 0; j < n; ++j)
    t->parent[j] = (cp[j + 1] - cp[j] > 1) ? ri[cp[j] + 1] : -1;
  /* prepend in descending order -> ascending child lists */
  for (int64_t j = n - 1; j >= 0; --j) {
    int64_t p = t->parent[j];
    if (p >= 0) { t->cnext[j] = t->chead[p]; t->chead[p] = j; }
  }
  return ORC_OK;
}

static void tree_free(tree_t* t) {
  free(t->parent); free(t->chead); free(t->cnext);
}

/* Positions of I_c (rows of column c below the diagonal) inside J_j (all
 * rows of column j).  Fails if I_c is not a subset (pattern not filled). */
static int relpos(const tree_t* t, int64_t c, int64_t j, int64_t* pos) {
  const int32_t* sub = t->ri + t->cp[c] + 1;
  int64_t ns = t->cp[c + 1] - t->cp[c] - 1;
  const int32_t* sup = t->ri + t->cp[j];
  int64_t nsup = t->cp[j + 1] - t->cp[j];
  int64_t q = 0;
  for (int64_t k = 0; k < ns; ++k) {
    while (q < nsup && sup[q] < sub[k]) ++q;
    if (q == nsup || sup[q] != sub[k]) return ORC_ENOTCHORDAL;
    pos[k] = q++;
  }
  return ORC_OK;
}

/* Value of the symmetric matrix stored in CCS at (r, c), r >= c, by binary
 * search in column c; returns 0 if (r, c) is not in the pattern. */
static double ccs_get(const tree_t* t, const double* v, int64_t r, int64_t c) {
  if (r < c) { int64_t s = r; r = c; c = s; }
  int64_t lo = t->cp[c], hi = t->cp[c + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int64_t x = t->ri[mid];
    if (x == r) return v[mid];
    if (x < r) lo = mid + 1; else hi = mid - 1;
  }
  return 0.0;
}

/* Dense principal submatrix S_{I_j I_j} (order m, full symmetric, row-major). */
static void gather_sub(const tree_t* t, const double* s, int64_t j, double* out) {
  const int32_t* I = t->ri + t->cp[j] + 1;
  int64_t m = t->cp[j + 1] - t->cp[j] - 1;
  for (int64_t a = 0; a < m; ++a)
    for (int64_t b = 0; b <= a; ++b) {
      double v = ccs_get(t, s, I[a], I[b]);
      out[a * m + b] = v;
      out[b * m + a] = v;
    }
}

/* --- small dense helpers (textbook, unblocked) -------------------------- */

/* In-place lower Cholesky of a full row-major m x m matrix: A = G G^T.
 * Returns 0 or the 1-based index of the first non-positive pivot. */
static int64_t dense_chol(double* a, int64_t m) {
  for (int64_t k = 0; k < m; ++k) {
    double d = a[k * m + k];
    for (int64_t p = 0; p < k; ++p) d -= a[k * m + p] * a[k * m + p];
    if (!(d > 0.0)) return k + 1;
    d = sqrt(d);
    a[k * m + k] = d;
    for (int64_t i = k + 1; i < m; ++i) {
      double v = a[i * m + k];
      for (int64_t p = 0; p < k; ++p) v -= a[i * m + p] * a[k * m + p];
      a[i * m + k] = v / d;
    }
  }
  return 0;
}

/* Solve (G G^T) x = b in place with the lower factor G. */
static void dense_chol_solve(const double* g, int64_t m, double* x) {
  for (int64_t i = 0; i < m; ++i) {
    double v = x[i];
    for (int64_t p = 0; p < i; ++p) v -= g[i * m + p] * x[p];
    x[i] = v / g[i * m + i];
  }
  for (int64_t i = m - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t p = i + 1; p < m; ++p) v -= g[p * m + i] * x[p];
    x[i] = v / g[i * m + i];
  }
}

/* Full symmetric frontal matrix F (order m, row-major) += E U E^T where U is
 * the update matrix of child c (order m-1 of I_c) and E = E_{J_j I_c}. */
static void extend_add(double* f, int64_t m, const double* u, int64_t mu, const int64_t* pos, double sign) {
  for (int64_t a = 0; a < mu; ++a)
    for (int64_t b = 0; b < mu; ++b)
      f[pos[a] * m + pos[b]] += sign * u[a * mu + b];
}

/* V_c = E^T G E: principal submatrix of the full front G (order m) at pos. */
static void extract(const double* g, int64_t m, const int64_t* pos, int64_t mc, double* vc) {
  (void)m;
  for (int64_t a = 0; a < mc; ++a)
    for (int64_t b = 0; b < mc; ++b)
      vc[a * mc + b] = g[pos[a] * m + pos[b]];
}

static double pairwise_sum(const double* v, int64_t n) {
  if (n <= 8) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    return s;
  }
  int64_t h = n / 2;
  return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

#define NEW(T, cnt) ((T*)malloc(sizeof(T) * ((size_t)(cnt) > 0 ? (size_t)(cnt) : 1)))

/* --- Algorithm 3.1: Cholesky factorization ------------------------------- */

int orc_factor(int64_t n, const int64_t* cp, const int32_t* ri, const double* x, double* ldl,
               int64_t* bad) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double** U = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  if (bad) *bad = -1;
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {        /* topological order */
    int64_t m = cp[j + 1] - cp[j];
    double* f = (double*)calloc((size_t)(m * m), sizeof(double));
    /* F = [X_jj X_Ij^T; X_Ij 0] */
    for (int64_t r = 0; r < m; ++r) { f[r * m] = x[cp[j] + r]; f[r] = x[cp[j] + r]; }
    /* + sum over children of E U_i E^T (eq. e-mf-chol-1) */
    for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
      int64_t mc = cp[c + 1] - cp[c] - 1;
      rc = relpos(&t, c, j, pos);
      if (rc) break;
      extend_add(f, m, U[c], mc, pos, 1.0);
      free(U[c]); U[c] = NULL;
    }
    if (rc) { free(f); break; }
    /* pivot step (eq. e-mf-chol-2) */
    double d = f[0];
    if (!(d > 0.0)) { rc = ORC_ENOTPD; if (bad) *bad = j; free(f); break; }
    ldl[cp[j]] = d;
    for (int64_t r = 1; r < m; ++r) ldl[cp[j] + r] = f[r * m] / d;
    int64_t mu = m - 1;
    U[j] = NEW(double, mu * mu);
    for (int64_t a = 0; a < mu; ++a)
      for (int64_t b = 0; b < mu; ++b) {
        double la = ldl[cp[j] + 1 + a], lb = ldl[cp[j] + 1 + b];
        U[j][a * mu + b] = f[(a + 1) * m + (b + 1)] - d * la * lb;
      }
    free(f);
  }
  for (int64_t j = 0; j < n; ++j) free(U[j]);
  free(U); free(pos); tree_free(&t);
  return rc;
}

/* log det X = sum_j log D_jj (so f(X) = -log det X), pairwise summation. */
int orc_logdet(int64_t n, const int64_t* cp, const double* ldl, double* out) {
  double* v = NEW(double, n);
  for (int64_t j = 0; j < n; ++j) v[j] = log(ldl[cp[j]]);
  *out = pairwise_sum(v, n);
  free(v);
  return ORC_OK;
}

/* --- Algorithm 3.2: Cholesky product X = L D L^T ------------------------ */

int orc_product(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl, double* x) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double** U = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t m = cp[j + 1] - cp[j];
    const double d = ldl[cp[j]];
    const double* l = ldl + cp[j];  /* l[r], r >= 1 */
    double* f = (double*)calloc((size_t)(m * m), sizeof(double));
    /* D [1; l][1; l]^T - sum E U_i E^T  (eq. e-mf-prod) */
    for (int64_t a = 0; a < m; ++a)
      for (int64_t b = 0; b < m; ++b) {
        double la = a ? l[a] : 1.0, lb = b ? l[b] : 1.0;
        f[a * m + b] = d * la * lb;
      }
    for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
      int64_t mc = cp[c + 1] - cp[c] - 1;
      rc = relpos(&t, c, j, pos);
      if (rc) break;
      extend_add(f, m, U[c], mc, pos, -1.0);
      free(U[c]); U[c] = NULL;
    }
    if (rc) { free(f); break; }
    for (int64_t r = 0; r < m; ++r) x[cp[j] + r] = f[r * m];
    int64_t mu = m - 1;
    U[j] = NEW(double, mu * mu);
    for (int64_t a = 0; a < mu; ++a)
      for (int64_t b = 0; b < mu; ++b) U[j][a * mu + b] = -f[(a + 1) * m + (b + 1)];
    free(f);
  }
  for (int64_t j = 0; j < n; ++j) free(U[j]);
  free(U); free(pos); tree_free(&t);
  return rc;
}

/* --- Algorithm 4.1: projected inverse S = P(X^-1) ----------------------- */

int orc_projinv(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl, double* s) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double** V = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  for (int64_t j = n - 1; j >= 0 && rc == ORC_OK; --j) {   /* reverse topological */
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    const double* l = ldl + cp[j] + 1;
    double* v = V[j];                                      /* S_{I_j I_j}, order mi */
    /* eq. e-mf-gradient-1 */
    double sjj = 1.0 / ldl[cp[j]];
    for (int64_t a = 0; a < mi; ++a) {
      double acc = 0.0;
      for (int64_t b = 0; b < mi; ++b) acc += v[a * mi + b] * l[b];
      s[cp[j] + 1 + a] = -acc;
    }
    for (int64_t a = 0; a < mi; ++a) sjj -= s[cp[j] + 1 + a] * l[a];
    s[cp[j]] = sjj;
    /* eq. e-mf-gradient-2: V_c = E^T [S_jj S_Ij^T; S_Ij V_j] E */
    if (t.chead[j] != -1) {
      double* g = NEW(double, m * m);
      for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
          double val;
          if (a == 0 && b == 0) val = sjj;
          else if (a == 0) val = s[cp[j] + b];
          else if (b == 0) val = s[cp[j] + a];
          else val = v[(a - 1) * mi + (b - 1)];
          g[a * m + b] = val;
        }
      for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
        int64_t mc = cp[c + 1] - cp[c] - 1;
        rc = relpos(&t, c, j, pos);
        if (rc) break;
        V[c] = NEW(double, mc * mc);
        extract(g, m, pos, mc, V[c]);
      }
      free(g);
    }
    free(V[j]); V[j] = NULL;
  }
  for (int64_t j = 0; j < n; ++j) free(V[j]);
  free(V); free(pos); tree_free(&t);
  return rc;
}

/* --- Algorithm 4.2: matrix completion ----------------------------------- */

int orc_completion(int64_t n, const int64_t* cp, const int32_t* ri, const double* s, double* ldl,
                   int64_t* bad) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double** V = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  if (bad) *bad = -1;
  for (int64_t j = n - 1; j >= 0 && rc == ORC_OK; --j) {   /* reverse topological */
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    double* v = V[j];                                      /* V_j = S_{I_j I_j} */
    const double* sij = s + cp[j] + 1;
    /* eq. e-mf-compl-1: L_Ij = -V_j^{-1} S_Ij, D_jj = (S_jj + S_Ij^T L_Ij)^{-1} */
    double* g = NEW(double, mi * mi);
    if (mi) memcpy(g, v, sizeof(double) * (size_t)(mi * mi));
    if (dense_chol(g, mi)) { rc = ORC_ENOCOMPL; if (bad) *bad = j; free(g); break; }
    double* l = ldl + cp[j] + 1;
    for (int64_t a = 0; a < mi; ++a) l[a] = sij[a];
    dense_chol_solve(g, mi, l);
    for (int64_t a = 0; a < mi; ++a) l[a] = -l[a];
    free(g);
    double den = s[cp[j]];
    for (int64_t a = 0; a < mi; ++a) den += sij[a] * l[a];
    if (!(den > 0.0)) { rc = ORC_ENOCOMPL; if (bad) *bad = j; break; }
    ldl[cp[j]] = 1.0 / den;
    /* eq. e-mf-compl-2 */
    if (t.chead[j] != -1) {
      double* fr = NEW(double, m * m);
      for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
          double val;
          if (a == 0 && b == 0) val = s[cp[j]];
          else if (a == 0) val = s[cp[j] + b];
          else if (b == 0) val = s[cp[j] + a];
          else val = v[(a - 1) * mi + (b - 1)];
          fr[a * m + b] = val;
        }
      for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
        int64_t mc = cp[c + 1] - cp[c] - 1;
        rc = relpos(&t, c, j, pos);
        if (rc) break;
        V[c] = NEW(double, mc * mc);
        extract(fr, m, pos, mc, V[c]);
      }
      free(fr);
    }
    free(V[j]); V[j] = NULL;
  }
  for (int64_t j = 0; j < n; ++j) free(V[j]);
  free(V); free(pos); tree_free(&t);
  return rc;
}

/* --- Algorithm 4.3: matrix completion with factored update matrices -----
 * The update matrix V_j = S_{I_j I_j} is carried as V_j = R_j R_j^T with
 * R_j upper triangular of order |I_j| (dense, row-major).  In reverse
 * topological order:
 *   eq. e-mf-compl-1-factored: L_Ij = -R_j^-T R_j^-1 S_Ij (back, then forward
 *     substitution), D_jj = (S_jj + S_Ij^T L_Ij)^-1;
 *   for every child i, eq. e-mfp-compl-3-factored: C = E^T R_j, the rows of
 *     R_j at the positions of I_i \ {j} in I_j, reduced to C = R Q^T by
 *     Householder reflections applied from the right (last row first, each
 *     moving the row's weight into its diagonal column; none where the
 *     row has no weight left of that column);
 *   eq. e-mf-compl-2-factored: R_i = [(S_jj - |w|^2)^1/2, w^T; 0, R] with
 *     w = R^-1 b, b = E^T S_Ij.
 * Every diagonal is made positive (by the sign of R's columns, which leaves
 * R R^T unchanged), so R_i is the unique upper triangular factor of V_i
 * with a positive diagonal.  rout (optional) receives R_j for every j, its
 * upper triangle by rows, |I_j|(|I_j|+1)/2 values per column j, j ascending.
 * Errors as orc_completion (ORC_ENOCOMPL at the column whose pivot or
 * update factor is not positive).                                          */
int orc_completion_factored(int64_t n, const int64_t* cp, const int32_t* ri, const double* s, double* ldl,
                            double* rout, int64_t* bad) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double** R = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  int64_t* roff = NEW(int64_t, n + 1);
  roff[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    int64_t mi = cp[j + 1] - cp[j] - 1;
    roff[j + 1] = roff[j] + mi * (mi + 1) / 2;
  }
  if (bad) *bad = -1;
  for (int64_t j = n - 1; j >= 0 && rc == ORC_OK; --j) {
    int64_t mi = cp[j + 1] - cp[j] - 1;
    const double* r = R[j];                                /* R_j, mi x mi */
    const double* sij = s + cp[j] + 1;
    if (rout)
      for (int64_t a = 0, q = roff[j]; a < mi; ++a)
        for (int64_t b = a; b < mi; ++b) rout[q++] = r[a * mi + b];
    /* z = R_j^-1 S_Ij, then L_Ij = -R_j^-T z */
    double* z = NEW(double, mi);
    for (int64_t a = mi - 1; a >= 0; --a) {
      double acc = sij[a];
      for (int64_t b = a + 1; b < mi; ++b) acc -= r[a * mi + b] * z[b];
      z[a] = acc / r[a * mi + a];
    }
    double* l = ldl + cp[j] + 1;
    for (int64_t a = 0; a < mi; ++a) {
      double acc = z[a];
      for (int64_t b = 0; b < a; ++b) acc -= r[b * mi + a] * l[b];
      l[a] = acc / r[a * mi + a];
    }
    for (int64_t a = 0; a < mi; ++a) l[a] = -l[a];
    free(z);
    double den = s[cp[j]];
    for (int64_t a = 0; a < mi; ++a) den += sij[a] * l[a];
    if (!(den > 0.0)) { rc = ORC_ENOCOMPL; if (bad) *bad = j; break; }
    ldl[cp[j]] = 1.0 / den;
    for (int64_t c = t.chead[j]; c != -1 && rc == ORC_OK; c = t.cnext[c]) {
      int64_t mc = cp[c + 1] - cp[c] - 1, m = mc - 1;      /* |I_c \ {j}| = m */
      /* positions of I_c \ {j} among the rows of column j (J_j = {j} U I_j) */
      rc = relpos(&t, c, j, pos);
      if (rc) break;
      double* cm = NEW(double, m * mi);                    /* C = E^T R_j */
      for (int64_t k = 0; k < m; ++k)
        for (int64_t b = 0; b < mi; ++b) cm[k * mi + b] = r[(pos[k + 1] - 1) * mi + b];
      double* v = NEW(double, mi);
      for (int64_t k = m - 1; k >= 0; --k) {
        int64_t q = mi - m + k;                            /* the row's diagonal column */
        double rest = 0.0;
        for (int64_t b = 0; b < q; ++b) rest += cm[k * mi + b] * cm[k * mi + b];
        if (rest == 0.0) continue;                         /* already e_q times a scalar: H = I */
        double nrm = sqrt(rest + cm[k * mi + q] * cm[k * mi + q]);
        double alpha = cm[k * mi + q] >= 0.0 ? -nrm : nrm;
        double vtv = 0.0;
        for (int64_t b = 0; b <= q; ++b) {
          v[b] = cm[k * mi + b] - (b == q ? alpha : 0.0);
          vtv += v[b] * v[b];
        }
        if (vtv > 0.0)
          for (int64_t x = 0; x < k; ++x) {
            double d = 0.0;
            for (int64_t b = 0; b <= q; ++b) d += cm[x * mi + b] * v[b];
            d *= 2.0 / vtv;
            for (int64_t b = 0; b <= q; ++b) cm[x * mi + b] -= d * v[b];
          }
        for (int64_t b = 0; b < q; ++b) cm[k * mi + b] = 0.0;
        cm[k * mi + q] = alpha;
      }
      free(v);
      /* R = the last m columns of C Q; positive diagonal */
      double* rc_ = (double*)calloc((size_t)(mc * mc) + 1, sizeof(double));
      for (int64_t k = 0; k < m; ++k)
        for (int64_t b = k; b < m; ++b) rc_[(k + 1) * mc + (b + 1)] = cm[k * mi + (mi - m + b)];
      for (int64_t b = 0; b < m; ++b)
        if (rc_[(b + 1) * mc + (b + 1)] < 0.0)
          for (int64_t k = 0; k <= b; ++k) rc_[(k + 1) * mc + (b + 1)] = -rc_[(k + 1) * mc + (b + 1)];
      free(cm);
      /* w = R^-1 b, b = E^T S_Ij; first row of R_c */
      double ww = 0.0;
      for (int64_t k = m - 1; k >= 0; --k) {
        double acc = sij[pos[k + 1] - 1];
        for (int64_t b = k + 1; b < m; ++b) acc -= rc_[(k + 1) * mc + (b + 1)] * rc_[b + 1];
        double wk = acc / rc_[(k + 1) * mc + (k + 1)];
        rc_[k + 1] = wk;                                   /* row 0, column k + 1 */
        ww += wk * wk;
      }
      double rho = s[cp[j]] - ww;
      if (!(rho > 0.0) || !(mc > 0)) { rc = ORC_ENOCOMPL; if (bad) *bad = c; free(rc_); break; }
      rc_[0] = sqrt(rho);
      R[c] = rc_;
    }
    free(R[j]); R[j] = NULL;
  }
  for (int64_t j = 0; j < n; ++j) free(R[j]);
  free(R); free(pos); free(roff); tree_free(&t);
  return rc;
}

/* --- Hessian step 1 (shared by Algorithms 5.1 and 5.3) -------------------
 * Topological order: F' = [Y_jj Y_Ij^T; Y_Ij 0] + sum E U'_i E^T, then
 * [K_jj K_Ij^T; K_Ij U'_j] = [1 0; -l I] F' [1 -l^T; 0 I].                */
static int hess_step1(const tree_t* t, const double* ldl, const double* y, double* k) {
  int64_t n = t->n;
  const int64_t* cp = t->cp;
  int rc = ORC_OK;
  double** U = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    const double* l = ldl + cp[j] + 1;
    double* f = (double*)calloc((size_t)(m * m), sizeof(double));
    for (int64_t r = 0; r < m; ++r) { f[r * m] = y[cp[j] + r]; f[r] = y[cp[j] + r]; }
    for (int64_t c = t->chead[j]; c != -1; c = t->cnext[c]) {
      int64_t mc = cp[c + 1] - cp[c] - 1;
      rc = relpos(t, c, j, pos);
      if (rc) break;
      extend_add(f, m, U[c], mc, pos, 1.0);
      free(U[c]); U[c] = NULL;
    }
    if (rc) { free(f); break; }
    double f11 = f[0];
    k[cp[j]] = f11;                                        /* K_jj = D'_jj */
    for (int64_t a = 0; a < mi; ++a) k[cp[j] + 1 + a] = f[(a + 1) * m] - l[a] * f11;
    U[j] = NEW(double, mi * mi);
    for (int64_t a = 0; a < mi; ++a)
      for (int64_t b = 0; b < mi; ++b)
        U[j][a * mi + b] = f[(a + 1) * m + (b + 1)] - l[a] * f[b + 1] - k[cp[j] + 1 + a] * l[b];
    free(f);
  }
  for (int64_t j = 0; j < n; ++j) free(U[j]);
  free(U); free(pos);
  return rc;
}

/* --- Hessian step 3 (shared by Algorithms 5.1 and 5.4) -------------------
 * Reverse topological order: [T_jj T_Ij^T; T_Ij V'_j] =
 * [1 -l^T; 0 I] [M_jj M_Ij^T; M_Ij V'_j] [1 0; -l I]; V'_c = E^T [..] E.   */
static int hess_step3(const tree_t* t, const double* ldl, const double* mm, double* tt) {
  int64_t n = t->n;
  const int64_t* cp = t->cp;
  int rc = ORC_OK;
  double** V = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  for (int64_t j = n - 1; j >= 0 && rc == ORC_OK; --j) {
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    const double* l = ldl + cp[j] + 1;
    const double* mI = mm + cp[j] + 1;
    double* v = V[j];
    /* T_Ij = M_Ij - V' l;  T_jj = M_jj - 2 l^T M_Ij + l^T V' l */
    double ltm = 0.0, lvl = 0.0;
    for (int64_t a = 0; a < mi; ++a) {
      double vl = 0.0;
      for (int64_t b = 0; b < mi; ++b) vl += v[a * mi + b] * l[b];
      tt[cp[j] + 1 + a] = mI[a] - vl;
      ltm += l[a] * mI[a];
      lvl += l[a] * vl;
    }
    tt[cp[j]] = mm[cp[j]] - 2.0 * ltm + lvl;
    if (t->chead[j] != -1) {
      double* g = NEW(double, m * m);
      for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
          double val;
          if (a == 0 && b == 0) val = tt[cp[j]];
          else if (a == 0) val = tt[cp[j] + b];
          else if (b == 0) val = tt[cp[j] + a];
          else val = v[(a - 1) * mi + (b - 1)];
          g[a * m + b] = val;
        }
      for (int64_t c = t->chead[j]; c != -1; c = t->cnext[c]) {
        int64_t mc = cp[c + 1] - cp[c] - 1;
        rc = relpos(t, c, j, pos);
        if (rc) break;
        V[c] = NEW(double, mc * mc);
        extract(g, m, pos, mc, V[c]);
      }
      free(g);
    }
    free(V[j]); V[j] = NULL;
  }
  for (int64_t j = 0; j < n; ++j) free(V[j]);
  free(V); free(pos);
  return rc;
}

/* --- Algorithm 5.1: Hessian T = P(X^-1 Y X^-1) --------------------------- */

int orc_hessian(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl, const double* s,
                const double* y, double* tout) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  int64_t nnz = cp[n];
  double* k = NEW(double, nnz);
  double* mm = NEW(double, nnz);
  rc = hess_step1(&t, ldl, y, k);
  if (rc == ORC_OK) {
    /* step 2: M_jj = K_jj / D_jj^2, M_Ij = (1/D_jj) S_{I_j I_j} K_Ij */
    for (int64_t j = 0; j < n; ++j) {
      int64_t mi = cp[j + 1] - cp[j] - 1;
      double d = ldl[cp[j]];
      mm[cp[j]] = k[cp[j]] / (d * d);
      double* sub = NEW(double, mi * mi);
      gather_sub(&t, s, j, sub);
      for (int64_t a = 0; a < mi; ++a) {
        double acc = 0.0;
        for (int64_t b = 0; b < mi; ++b) acc += sub[a * mi + b] * k[cp[j] + 1 + b];
        mm[cp[j] + 1 + a] = acc / d;
      }
      free(sub);
    }
    rc = hess_step3(&t, ldl, mm, tout);
  }
  free(k); free(mm); tree_free(&t);
  return rc;
}

/* --- Algorithm 5.2: inverse Hessian Y = H^-1(T) ------------------------- */

int orc_inv_hessian(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl,
                    const double* s, const double* tin, double* yout) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  int64_t nnz = cp[n];
  double* mm = NEW(double, nnz);
  double* k = NEW(double, nnz);
  double** V = (double**)calloc((size_t)n + 1, sizeof(double*));
  int64_t* pos = NEW(int64_t, n);
  /* step 1, reverse topological:
     [M_jj M_Ij^T; M_Ij V'] = [1 l^T; 0 I] [T_jj T_Ij^T; T_Ij V'] [1 0; l I] */
  for (int64_t j = n - 1; j >= 0 && rc == ORC_OK; --j) {
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    const double* l = ldl + cp[j] + 1;
    const double* tI = tin + cp[j] + 1;
    double* v = V[j];
    double ltt = 0.0, lvl = 0.0;
    for (int64_t a = 0; a < mi; ++a) {
      double vl = 0.0;
      for (int64_t b = 0; b < mi; ++b) vl += v[a * mi + b] * l[b];
      mm[cp[j] + 1 + a] = tI[a] + vl;
      ltt += l[a] * tI[a];
      lvl += l[a] * vl;
    }
    mm[cp[j]] = tin[cp[j]] + 2.0 * ltt + lvl;
    if (t.chead[j] != -1) {
      double* g = NEW(double, m * m);
      for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
          double val;
          if (a == 0 && b == 0) val = tin[cp[j]];
          else if (a == 0) val = tin[cp[j] + b];
          else if (b == 0) val = tin[cp[j] + a];
          else val = v[(a - 1) * mi + (b - 1)];
          g[a * m + b] = val;
        }
      for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
        int64_t mc = cp[c + 1] - cp[c] - 1;
        rc = relpos(&t, c, j, pos);
        if (rc) break;
        V[c] = NEW(double, mc * mc);
        extract(g, m, pos, mc, V[c]);
      }
      free(g);
    }
    free(V[j]); V[j] = NULL;
  }
  /* step 2: K_jj = D_jj^2 M_jj, K_Ij = D_jj S_{I_j I_j}^{-1} M_Ij */
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t mi = cp[j + 1] - cp[j] - 1;
    double d = ldl[cp[j]];
    k[cp[j]] = d * d * mm[cp[j]];
    double* sub = NEW(double, mi * mi);
    gather_sub(&t, s, j, sub);
    if (dense_chol(sub, mi)) { rc = ORC_ENOTPD; free(sub); break; }
    for (int64_t a = 0; a < mi; ++a) k[cp[j] + 1 + a] = mm[cp[j] + 1 + a];
    dense_chol_solve(sub, mi, k + cp[j] + 1);
    for (int64_t a = 0; a < mi; ++a) k[cp[j] + 1 + a] *= d;
    free(sub);
  }
  /* step 3, topological:
     [Y_jj Y_Ij^T; Y_Ij -U'_j] = [1 0; l I][K_jj K_Ij^T; K_Ij 0][1 l^T; 0 I] - sum E U'_i E^T */
  double** U = V;  /* reuse the pointer table (all entries are NULL now) */
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t m = cp[j + 1] - cp[j], mi = m - 1;
    const double* l = ldl + cp[j] + 1;
    const double kjj = k[cp[j]];
    const double* kI = k + cp[j] + 1;
    double* g = (double*)calloc((size_t)(m * m), sizeof(double));
    for (int64_t c = t.chead[j]; c != -1; c = t.cnext[c]) {
      int64_t mc = cp[c + 1] - cp[c] - 1;
      rc = relpos(&t, c, j, pos);
      if (rc) break;
      extend_add(g, m, U[c], mc, pos, 1.0);
      free(U[c]); U[c] = NULL;
    }
    if (rc) { free(g); break; }
    yout[cp[j]] = kjj - g[0];
    for (int64_t a = 0; a < mi; ++a) yout[cp[j] + 1 + a] = l[a] * kjj + kI[a] - g[(a + 1) * m];
    U[j] = NEW(double, mi * mi);
    for (int64_t a = 0; a < mi; ++a)
      for (int64_t b = 0; b < mi; ++b)
        U[j][a * mi + b] = g[(a + 1) * m + (b + 1)] - l[a] * kjj * l[b] - kI[a] * l[b] - l[a] * kI[b];
    free(g);
  }
  for (int64_t j = 0; j < n; ++j) free(V[j]);
  free(V); free(pos); free(mm); free(k); tree_free(&t);
  return rc;
}

/* --- Algorithms 5.3 / 5.4: Hessian factor H = R^adj o R ------------------
 * R_j is the upper-triangular factor of S_{I_j I_j} = R_j R_j^T.  With J the
 * exchange (index-reversal) matrix, J S J = G G^T (lower Cholesky) gives
 * S = (J G J)(J G J)^T and J G J is upper triangular.                     */
static int upper_factor(const double* sub, int64_t mi, double* r /* row-major upper */) {
  double* a = NEW(double, mi * mi);
  for (int64_t x = 0; x < mi; ++x)
    for (int64_t y = 0; y < mi; ++y) a[x * mi + y] = sub[(mi - 1 - x) * mi + (mi - 1 - y)];
  if (dense_chol(a, mi)) { free(a); return ORC_ENOTPD; }
  for (int64_t x = 0; x < mi; ++x)
    for (int64_t y = 0; y < mi; ++y) {
      int64_t gx = mi - 1 - x, gy = mi - 1 - y;
      r[x * mi + y] = (gy <= gx) ? a[gx * mi + gy] : 0.0;
    }
  free(a);
  return ORC_OK;
}

int orc_hessian_factor(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl,
                       const double* s, const double* y, double* w) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double* k = NEW(double, cp[n]);
  rc = hess_step1(&t, ldl, y, k);
  /* step 2 (first half): W_jj = K_jj / D_jj, W_Ij = R_j^T K_Ij / sqrt(D_jj) */
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t mi = cp[j + 1] - cp[j] - 1;
    double d = ldl[cp[j]];
    w[cp[j]] = k[cp[j]] / d;
    double* sub = NEW(double, mi * mi);
    double* r = NEW(double, mi * mi);
    gather_sub(&t, s, j, sub);
    rc = upper_factor(sub, mi, r);
    for (int64_t a = 0; a < mi && rc == ORC_OK; ++a) {
      double acc = 0.0;
      for (int64_t b = 0; b < mi; ++b) acc += r[b * mi + a] * k[cp[j] + 1 + b];
      w[cp[j] + 1 + a] = acc / sqrt(d);
    }
    free(sub); free(r);
  }
  free(k); tree_free(&t);
  return rc;
}

int orc_hessian_factor_adj(int64_t n, const int64_t* cp, const int32_t* ri, const double* ldl,
                           const double* s, const double* w, double* tout) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  double* mm = NEW(double, cp[n]);
  /* step 1: M_jj = W_jj / D_jj, M_Ij = R_j W_Ij / sqrt(D_jj) */
  for (int64_t j = 0; j < n && rc == ORC_OK; ++j) {
    int64_t mi = cp[j + 1] - cp[j] - 1;
    double d = ldl[cp[j]];
    mm[cp[j]] = w[cp[j]] / d;
    double* sub = NEW(double, mi * mi);
    double* r = NEW(double, mi * mi);
    gather_sub(&t, s, j, sub);
    rc = upper_factor(sub, mi, r);
    for (int64_t a = 0; a < mi && rc == ORC_OK; ++a) {
      double acc = 0.0;
      for (int64_t b = 0; b < mi; ++b) acc += r[a * mi + b] * w[cp[j] + 1 + b];
      mm[cp[j] + 1 + a] = acc / sqrt(d);
    }
    free(sub); free(r);
  }
  if (rc == ORC_OK) rc = hess_step3(&t, ldl, mm, tout);
  free(mm); tree_free(&t);
  return rc;
}

/* Symbolic outputs for tests: elimination-tree parent and monotone degree. */
int orc_etree(int64_t n, const int64_t* cp, const int32_t* ri, int64_t* parent, int64_t* degree) {
  tree_t t;
  int rc = tree_init(&t, n, cp, ri);
  if (rc) return rc;
  for (int64_t j = 0; j < n; ++j) {
    parent[j] = t.parent[j];
    degree[j] = cp[j + 1] - cp[j] - 1;
    if (t.parent[j] >= 0) {
      int64_t* pos = NEW(int64_t, degree[j]);
      rc = relpos(&t, j, t.parent[j], pos);
      free(pos);
      if (rc) break;
    }
  }
  tree_free(&t);
  return rc;
}

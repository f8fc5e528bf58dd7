/*
 * CPU oracle for restarted GMRES(m): level-1 MGS, one-reduce lagged compact-WY
 * MGS, two-reduce lagged CGS2, and the two classical Gram-Schmidt baselines the
 * paper's GPU study runs (re-orthogonalized CGS with three reductions per
 * step, and Ruhe's two-synchronization CGS). Written from Swirydowicz, Langou,
 * Ananthan, Yang, Thomas, "Low synchronization GMRES algorithms"
 * (arXiv:1809.05805).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library. Plain sequential
 * FP64 C with every sum taken in index order.
 *
 * Conventions (0-based). A cycle builds V[:,0..j] and the (j+1) x j
 * Hessenberg matrix H with A V[:,0:j] = V[:,0:j+1] H. The paper's QR view of
 * Arnoldi (Section III: [r0, A V_m] = V_{m+1} [||r0|| e1, H]) makes r0 the
 * first column to be orthogonalized; the lagged schemes store it unnormalized
 * in V[:,0], and step k normalizes column k with the norm that step's single
 * reduction returns.
 */
#include "oracle_gmres.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* vals;
} csr_t;

/*
 * Accumulator of the long sums: the SpMV row sums and the length-n dot
 * products. FP64 in the oracle proper. A second, test-only build defines
 * ORACLE_ACC as long double (x87 extended precision, 64-bit significand):
 * every product is still the FP64 product, rounded once, but the sums carry
 * 11 more bits, so that build's results differ from exact-sum arithmetic by
 * about 2^-11 of what the FP64 oracle's sequential sums contribute. It is the
 * reference against which the FP64 oracle's and the GPU's summation errors
 * are compared; the algorithm and its order are the same.
 */
#ifndef ORACLE_ACC
#define ORACLE_ACC double
#endif

/*
 * A third, timing-only build (ORACLE_OMP, with -fopenmp) runs the length-n
 * loops as OpenMP parallel loops: row-wise loops keep their arithmetic, and a
 * dot product then sums per thread and adds the threads' sums. It times the
 * oracle on all of a host's cores; parity always uses the sequential build.
 */
#ifdef ORACLE_OMP
#include <omp.h>
#define ORACLE_ROWS _Pragma("omp parallel for schedule(static)")
#define ORACLE_SUM _Pragma("omp parallel for schedule(static) reduction(+ : s)")
/* Threads of the timing build's loops from now on (n >= 1), or just the
   count in effect (n < 1); returns the count in effect. */
int oracle_omp_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
}
#else
#define ORACLE_ROWS
#define ORACLE_SUM
#endif

void oracle_spmv(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                 const double* x, double* y) {
  ORACLE_ROWS
  for (int64_t i = 0; i < n; ++i) {
    ORACLE_ACC s = 0.0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += (ORACLE_ACC)(vals[e] * x[col_idx[e]]);
    y[i] = (double)s;
  }
}

static void spmv(const csr_t* A, const double* x, double* y) {
  oracle_spmv(A->n, A->row_ptr, A->col_idx, A->vals, x, y);
}

static double dot(int64_t n, const double* a, const double* b) {
  ORACLE_ACC s = 0.0;
  ORACLE_SUM
  for (int64_t i = 0; i < n; ++i) s += (ORACLE_ACC)(a[i] * b[i]);
  return (double)s;
}

/*
 * Plane rotation [c s; -s c] that maps (a, b) to (r, 0), r = sqrt(a^2 + b^2),
 * with the operands scaled by max(|a|,|b|) so that squaring cannot overflow.
 */
static void rot_make(double a, double b, double* c, double* s) {
  if (b == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  if (a == 0.0) {
    *c = 0.0;
    *s = 1.0;
    return;
  }
  double scale = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  double as = a / scale, bs = b / scale;
  double r = scale * sqrt(as * as + bs * bs);
  *c = a / r;
  *s = b / r;
}

static void rot_apply(double c, double s, double* x, double* y) {
  double t = c * (*x) + s * (*y);
  *y = -s * (*x) + c * (*y);
  *x = t;
}

typedef struct {
  int64_t n;
  int m;
  int ldh; /* m+1 */
  int ldt; /* m+2 */
  double* V;  /* n x (m+2) */
  double* H;  /* (m+1) x m, unrotated */
  double* R;  /* (m+1) x m, Givens-rotated copy */
  double* T;  /* (m+2) x (m+2): Malard-Paige T, upper unit triangular */
  double* L;  /* (m+2) x (m+2): rows of the strictly lower part of V^T V */
  double* g;  /* m+2 */
  double* cs; /* m+1 */
  double* sn; /* m+1 */
  double* w;  /* n */
  double* p;  /* m+2 */
  double* c;  /* m+2 */
  double* r;  /* m+2 */
  double* h;  /* m+2 */
  double* y;  /* m+2 */
  double* S2; /* (m+1) x m: CGS2 second-pass coefficients s, per column */
  double* gres; /* m+2: gres[c+1] = |g_{c+1}| as rotation c left it */
} ws_t;

static void ws_free(ws_t* ws) {
  free(ws->V); free(ws->H); free(ws->R); free(ws->T); free(ws->L); free(ws->g);
  free(ws->cs); free(ws->sn); free(ws->w); free(ws->p); free(ws->c); free(ws->r);
  free(ws->h); free(ws->y); free(ws->S2); free(ws->gres);
}

static int ws_alloc(ws_t* ws, int64_t n, int m) {
  memset(ws, 0, sizeof(*ws));
  ws->n = n;
  ws->m = m;
  ws->ldh = m + 1;
  ws->ldt = m + 2;
  ws->V = (double*)calloc((size_t)n * (size_t)(m + 2), sizeof(double));
  ws->H = (double*)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
  ws->R = (double*)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
  ws->T = (double*)calloc((size_t)(m + 2) * (size_t)(m + 2), sizeof(double));
  ws->L = (double*)calloc((size_t)(m + 2) * (size_t)(m + 2), sizeof(double));
  ws->g = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->cs = (double*)calloc((size_t)(m + 1), sizeof(double));
  ws->sn = (double*)calloc((size_t)(m + 1), sizeof(double));
  ws->w = (double*)calloc((size_t)n, sizeof(double));
  ws->p = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->c = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->r = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->h = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->y = (double*)calloc((size_t)(m + 2), sizeof(double));
  ws->S2 = (double*)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
  ws->gres = (double*)calloc((size_t)(m + 2), sizeof(double));
  if (!ws->S2 || !ws->gres || !ws->V || !ws->H || !ws->R || !ws->T || !ws->L || !ws->g || !ws->cs || !ws->sn || !ws->w ||
      !ws->p || !ws->c || !ws->r || !ws->h || !ws->y) {
    ws_free(ws);
    return -1;
  }
  return 0;
}

static void ws_reset_small(ws_t* ws) {
  int m = ws->m;
  memset(ws->H, 0, sizeof(double) * (size_t)(m + 1) * (size_t)m);
  memset(ws->R, 0, sizeof(double) * (size_t)(m + 1) * (size_t)m);
  memset(ws->T, 0, sizeof(double) * (size_t)(m + 2) * (size_t)(m + 2));
  memset(ws->L, 0, sizeof(double) * (size_t)(m + 2) * (size_t)(m + 2));
  memset(ws->g, 0, sizeof(double) * (size_t)(m + 2));
  memset(ws->S2, 0, sizeof(double) * (size_t)(m + 1) * (size_t)m);
}

#define HH(ws, i, j) ((ws)->H[(size_t)(j) * (size_t)(ws)->ldh + (size_t)(i)])
#define RR(ws, i, j) ((ws)->R[(size_t)(j) * (size_t)(ws)->ldh + (size_t)(i)])
#define TT(ws, i, j) ((ws)->T[(size_t)(j) * (size_t)(ws)->ldt + (size_t)(i)])
#define LL(ws, i, j) ((ws)->L[(size_t)(j) * (size_t)(ws)->ldt + (size_t)(i)])
#define VC(ws, j) ((ws)->V + (size_t)(j) * (size_t)(ws)->n)

/*
 * Givens least squares, MGS-GMRES algorithm of Section III ("apply Givens
 * rotations to H_{:,i}"): column col of H is complete; copy it into R, apply
 * the earlier rotations, form rotation col and update g. Returns |g[col+1]|.
 */
static double rotate_column(ws_t* ws, int col) {
  for (int i = 0; i <= col + 1; ++i) RR(ws, i, col) = HH(ws, i, col);
  for (int i = 0; i < col; ++i) rot_apply(ws->cs[i], ws->sn[i], &RR(ws, i, col), &RR(ws, i + 1, col));
  double c, s;
  rot_make(RR(ws, col, col), RR(ws, col + 1, col), &c, &s);
  ws->cs[col] = c;
  ws->sn[col] = s;
  rot_apply(c, s, &RR(ws, col, col), &RR(ws, col + 1, col));
  RR(ws, col + 1, col) = 0.0;
  double gk = ws->g[col];
  ws->g[col] = c * gk;
  ws->g[col + 1] = -s * gk;
  return fabs(ws->g[col + 1]);
}

/*
 * End of a cycle: y = argmin ||H y - beta e1|| by back substitution on the
 * rotated triangle, then x = x + V[:,0:j] y (Section III, last two lines of
 * the GMRES listings). A zero pivot (possible only for singular A) sets that
 * component of y to zero.
 */
static void update_solution(ws_t* ws, int j, double* x) {
  for (int i = j - 1; i >= 0; --i) {
    double s = ws->g[i];
    for (int q = i + 1; q < j; ++q) s -= RR(ws, i, q) * ws->y[q];
    ws->y[i] = RR(ws, i, i) != 0.0 ? s / RR(ws, i, i) : 0.0;
  }
  for (int q = 0; q < j; ++q) {
    const double* v = VC(ws, q);
    double yq = ws->y[q];
    ORACLE_ROWS
    for (int64_t i = 0; i < ws->n; ++i) x[i] += v[i] * yq;
  }
}

typedef struct {
  int j;
  int true_conv;
  int breakdown;
  double beta;
} cycle_out;

/* r0 = b - A x, stored in V[:,0]. */
static void residual_into_v0(const csr_t* A, const double* b, const double* x, ws_t* ws) {
  double* v0 = VC(ws, 0);
  spmv(A, x, ws->w);
  ORACLE_ROWS
  for (int64_t i = 0; i < A->n; ++i) v0[i] = b[i] - ws->w[i];
}

/*
 * Level-1 MGS-GMRES cycle (Section III, the Saad-Schultz listing). The inner
 * loop is modified Gram-Schmidt: each coefficient is the inner product with
 * the vector as already updated by the previous projections, so
 * h_{q,i} = (w, v_q) followed by w = w - h_{q,i} v_q. One reduction per
 * coefficient plus one for the norm: i+2 in iteration i.
 */
static int cycle_mgs(const csr_t* A, const double* b, double* x, int m_eff, double tol_abs,
                     double bnorm, ws_t* ws, double* hist, int64_t it0, int64_t* nred,
                     cycle_out* out) {
  int64_t n = A->n;
  memset(out, 0, sizeof(*out));
  ws_reset_small(ws);
  residual_into_v0(A, b, x, ws);
  double* v0 = VC(ws, 0);
  double beta2 = dot(n, v0, v0);
  (*nred)++;
  if (!isfinite(beta2)) return ORACLE_ERR_NONFINITE;
  double beta = sqrt(beta2);
  out->beta = beta;
  ws->g[0] = beta;
  if (beta <= tol_abs) {
    out->true_conv = 1;
    return ORACLE_OK;
  }
  if (m_eff == 0) return ORACLE_OK;
  ORACLE_ROWS
  for (int64_t i = 0; i < n; ++i) v0[i] = v0[i] / beta;
  for (int i = 0; i < m_eff; ++i) {
    double* w = VC(ws, i + 1);
    spmv(A, VC(ws, i), w);
    for (int q = 0; q <= i; ++q) {
      const double* vq = VC(ws, q);
      double hq = dot(n, w, vq);
      (*nred)++;
      ORACLE_ROWS
      for (int64_t e = 0; e < n; ++e) w[e] = w[e] - hq * vq[e];
      HH(ws, q, i) = hq;
    }
    double hn2 = dot(n, w, w);
    (*nred)++;
    if (!isfinite(hn2)) return ORACLE_ERR_NONFINITE;
    double hn = sqrt(hn2);
    HH(ws, i + 1, i) = hn;
    for (int q = 0; q <= i; ++q)
      if (!isfinite(HH(ws, q, i))) return ORACLE_ERR_NONFINITE;
    double gk = rotate_column(ws, i);
    if (!isfinite(gk)) return ORACLE_ERR_NONFINITE;
    ws->gres[i + 1] = gk;
    if (hist) hist[it0 + i] = gk / bnorm;
    if (hn == 0.0) {
      out->breakdown = 1;
      out->j = i + 1;
      return ORACLE_OK;
    }
    ORACLE_ROWS
    for (int64_t e = 0; e < n; ++e) w[e] = w[e] / hn;
    if (gk <= tol_abs) {
      out->j = i + 1;
      return ORACLE_OK;
    }
  }
  out->j = m_eff;
  return ORACLE_OK;
}

/*
 * Alg 1's orthogonalization of a new column w against V[:,0:i+1] (columns
 * of length n, ld = ldv), classical Gram-Schmidt run twice: each pass takes
 * p = V^T w (one reduction), subtracts V p from w and adds p into the
 * Hessenberg column hcol (which must hold zeros on entry), so hcol ends as
 * the sum of both passes' coefficients and w = w_in - V hcol. p is scratch
 * (i+1 doubles).
 */
static void cgs_two_passes(int64_t n, int i, const double* V, int64_t ldv, double* w,
                           double* hcol, double* p) {
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q <= i; ++q) p[q] = dot(n, V + (size_t)q * (size_t)ldv, w);
    for (int q = 0; q <= i; ++q) {
      const double* vq = V + (size_t)q * (size_t)ldv;
      double sq = p[q];
      ORACLE_ROWS
      for (int64_t e = 0; e < n; ++e) w[e] = w[e] - vq[e] * sq;
      hcol[q] = hcol[q] + sq;
    }
  }
}

/*
 * The lagged CGS2 update of step k (Alg 5 under reading 8), given the step's
 * first-pass coefficients r = V[:,0:k+1]^T (w / rho) and the strictly lower
 * L of V^T V = I + L + L^T on the leading (k+1) x (k+1) block (entry (a, q),
 * a > q, at L[q * ldl + a]):
 *   h = (I - L) r (the first-order correction, the uncorrected r on the right),
 *   z = w / rho - V h, s = V^T z (the second reduction), vnext = z - V s,
 *   hcol = h + s, the Hessenberg column.
 * V has columns of length n, ld = ldv; h, s and hcol hold k+1 doubles.
 */
static void cgs2_update(int64_t n, int k, const double* V, int64_t ldv, const double* L,
                        int64_t ldl, const double* r, double rho, const double* w,
                        double* vnext, double* h, double* s, double* hcol) {
  for (int i = k; i >= 0; --i) {
    double a = r[i];
    for (int q = 0; q < i; ++q) a -= L[(size_t)q * (size_t)ldl + (size_t)i] * r[q];
    h[i] = a;
  }
  ORACLE_ROWS
  for (int64_t e = 0; e < n; ++e) vnext[e] = w[e] / rho;
  for (int q = 0; q <= k; ++q) {
    const double* vq = V + (size_t)q * (size_t)ldv;
    double hq = h[q];
    ORACLE_ROWS
    for (int64_t e = 0; e < n; ++e) vnext[e] = vnext[e] - vq[e] * hq;
  }
  for (int q = 0; q <= k; ++q) s[q] = dot(n, V + (size_t)q * (size_t)ldv, vnext);
  for (int q = 0; q <= k; ++q) {
    const double* vq = V + (size_t)q * (size_t)ldv;
    double sq = s[q];
    ORACLE_ROWS
    for (int64_t e = 0; e < n; ++e) vnext[e] = vnext[e] - vq[e] * sq;
  }
  for (int q = 0; q <= k; ++q) hcol[q] = h[q] + s[q];
}

void oracle_cgs_two_passes(int64_t n, int32_t i, const double* V, double* w, double* hcol) {
  double* p = (double*)malloc(sizeof(double) * (size_t)(i + 1));
  if (!p) return;
  for (int q = 0; q <= i; ++q) hcol[q] = 0.0;
  cgs_two_passes(n, i, V, n, w, hcol, p);
  free(p);
}

void oracle_cgs2_update(int64_t n, int32_t k, const double* V, const double* L, const double* r,
                        double rho, const double* w, double* vnext, double* h, double* s,
                        double* hcol) {
  cgs2_update(n, k, V, n, L, k + 1, r, rho, w, vnext, h, s, hcol);
}

/*
 * Classical Gram-Schmidt cycles on a normalized basis, as in the level-1
 * listing: V[:,0] = r0 / ||r0||, and step i orthogonalizes w = A v_i against
 * V[:,0:i+1] with every coefficient taken from the same vector (classical),
 * then normalizes it with a separate norm reduction.
 *
 * ORACLE_CGS2_3R, the first listing of Section II (classical Gram-Schmidt
 *   with re-orthogonalization) run for two iterations: s = V^T w, r += s,
 *   w = w - V s, twice; H[0:i+1,i] = r; h_{i+1,i} = ||w||. Three reductions
 *   per step (two projections and the norm).
 * ORACLE_TWOSYNCH, the two-synchronization iterated CGS of Section II: one
 *   reduction gives y = V^T w together with the new row of L, the strictly
 *   lower part of V^T V = I + L + L^T (l_q = v_q^T v_i for q < i); the
 *   coefficients are r = T y with T = I - L - L^T on the leading
 *   (i+1) x (i+1) block (Ruhe's two Gauss-Jacobi iterations folded into one);
 *   w = w - V r; the second reduction is ||w||. H[0:i+1,i] = r. (Reading of
 *   the listing's update step, which prints a - Q Q^T a: the update uses the
 *   corrected coefficients r, which is what the T derivation before it
 *   produces.)
 * Within a cycle, where V is orthonormal to working precision, the second
 * pass's coefficients s of ORACLE_CGS2_3R are O(eps) relative to the first
 * pass's, so adding them into H (r += s) shows only at the rounding level; the
 * pass itself (cgs_two_passes) is therefore also exposed as
 * oracle_cgs_two_passes and pinned on a basis whose Gram matrix is I + E with
 * E of size delta, where the projection coefficients G^{-1} V^T w must be met
 * to O(delta^2), which one pass's coefficients miss by O(delta). The rest of
 * both schemes is pinned on whole cycles (same H as MGS, Krylov minimizer,
 * dense LU, orthogonality bounds that fail without the re-orthogonalization
 * or without either half of the T correction, reductions per step).
 */
static int cycle_cgs(const csr_t* A, const double* b, double* x, int m_eff, double tol_abs,
                     double bnorm, int scheme, ws_t* ws, double* hist, int64_t it0,
                     int64_t* nred, cycle_out* out) {
  int64_t n = A->n;
  memset(out, 0, sizeof(*out));
  ws_reset_small(ws);
  residual_into_v0(A, b, x, ws);
  double* v0 = VC(ws, 0);
  double beta2 = dot(n, v0, v0);
  (*nred)++;
  if (!isfinite(beta2)) return ORACLE_ERR_NONFINITE;
  double beta = sqrt(beta2);
  out->beta = beta;
  ws->g[0] = beta;
  if (beta <= tol_abs) {
    out->true_conv = 1;
    return ORACLE_OK;
  }
  if (m_eff == 0) return ORACLE_OK;
  ORACLE_ROWS
  for (int64_t i = 0; i < n; ++i) v0[i] = v0[i] / beta;
  for (int i = 0; i < m_eff; ++i) {
    double* w = VC(ws, i + 1);
    spmv(A, VC(ws, i), w);
    if (scheme == ORACLE_CGS2_3R) {
      cgs_two_passes(n, i, ws->V, n, w, &HH(ws, 0, i), ws->p);
      (*nred) += 2;
    } else {
      for (int q = 0; q <= i; ++q) ws->c[q] = dot(n, VC(ws, q), w);
      for (int q = 0; q < i; ++q) LL(ws, i, q) = dot(n, VC(ws, q), VC(ws, i));
      (*nred)++;
      for (int a = 0; a <= i; ++a) {
        double s = ws->c[a];
        for (int q = 0; q < a; ++q) s -= LL(ws, a, q) * ws->c[q];
        for (int q = a + 1; q <= i; ++q) s -= LL(ws, q, a) * ws->c[q];
        ws->r[a] = s;
      }
      for (int q = 0; q <= i; ++q) {
        const double* vq = VC(ws, q);
        double rq = ws->r[q];
        ORACLE_ROWS
        for (int64_t e = 0; e < n; ++e) w[e] = w[e] - vq[e] * rq;
        HH(ws, q, i) = rq;
      }
    }
    double hn2 = dot(n, w, w);
    (*nred)++;
    if (!isfinite(hn2)) return ORACLE_ERR_NONFINITE;
    double hn = sqrt(hn2);
    HH(ws, i + 1, i) = hn;
    for (int q = 0; q <= i; ++q)
      if (!isfinite(HH(ws, q, i))) return ORACLE_ERR_NONFINITE;
    double gk = rotate_column(ws, i);
    if (!isfinite(gk)) return ORACLE_ERR_NONFINITE;
    ws->gres[i + 1] = gk;
    if (hist) hist[it0 + i] = gk / bnorm;
    if (hn == 0.0) {
      out->breakdown = 1;
      out->j = i + 1;
      return ORACLE_OK;
    }
    ORACLE_ROWS
    for (int64_t e = 0; e < n; ++e) w[e] = w[e] / hn;
    if (gk <= tol_abs) {
      out->j = i + 1;
      return ORACLE_OK;
    }
  }
  out->j = m_eff;
  return ORACLE_OK;
}

/*
 * Lagged cycle shared by the one-reduce MGS scheme (level-2 MGS with R
 * normalization lag, inside the one-synchronization GMRES of Section III) and
 * the two-reduce CGS2 scheme (level-2 iterated CGS with the same lag).
 *
 * Step k, with u = V[:,k] orthogonalized but not yet normalized:
 *   w = A u (skipped when k == m_eff: that step only finishes the norm);
 *   one reduction: p = V[:,0:k]^T u, alpha = u^T u, c = V[:,0:k]^T w, gamma = u^T w;
 *   rho = sqrt(alpha) is R_{k,k} (beta at k = 0, else H[k,k-1]); V[:,k] = u/rho;
 *   l = p / rho is row k of the strictly lower L with V^T V = I + L + L^T;
 *   r = V[:,0:k+1]^T (A v_k) = [c/rho ; (gamma/rho)/rho], because w = rho A v_k
 *   and the last entry also carries the freshly normalized v_k.
 * MGS (compact WY, Malard-Paige): T[0:k,k] = -T[0:k,0:k] l, T[k,k] = 1, so
 *   T = (I + L^T)^{-1}; h = T^T r equals (I+L)^{-1} V^T A v_k, the MGS
 *   coefficients (Ruhe's loop invariant, Section II); V[:,k+1] = w/rho - V h.
 * CGS2: r <- (I - L) r (the first-order truncation of the same correction),
 *   z = w/rho - V r, second reduction s = V^T z, V[:,k+1] = z - V s, h = r + s.
 *   Within a cycle the second pass keeps L at O(eps), so the (I - L)
 *   correction and the s term of h show only at the rounding level; the
 *   update (cgs2_update) is therefore also exposed as oracle_cgs2_update and
 *   pinned on a basis with L of size delta, where s must equal -L^T r to
 *   O(delta^2) (without the correction it is -(L + L^T) r, with its sign
 *   flipped -(2L + L^T) r) and the column h + s must reach the projection
 *   coefficients to O(delta^2) with w / rho = V (h + s) + vnext exactly.
 *
 * Pipeline depth (the depth-L pipeline of Section III, shown there for L = 2):
 * the Givens rotations, and with them the stopping test, only consume
 * completed Hessenberg columns and feed nothing back into the Arnoldi
 * recurrence, so they may trail it. With depth L the pending columns are
 * rotated L at a time (and at the last step of a cycle, or at a breakdown):
 * step k rotates columns rot_next .. k-1 once k - rot_next reaches L. The
 * cycle then stops at the first column count j whose |g_j| meets the
 * tolerance, exactly the j that depth 1 (rotation every step) stops at, but
 * up to L - 1 steps later: those extra steps are computed and discarded. H,
 * the rotations, g, y and x for the j columns are the same arithmetic in the
 * same order as at depth 1, so the iterate is identical.
 */
static int cycle_lagged(const csr_t* A, const double* b, double* x, int m_eff, double tol_abs,
                        double bnorm, int scheme, int depth, ws_t* ws, double* hist, int64_t it0,
                        int64_t* nred, cycle_out* out) {
  int64_t n = A->n;
  memset(out, 0, sizeof(*out));
  ws_reset_small(ws);
  residual_into_v0(A, b, x, ws);
  int rot_next = 0;  /* first Hessenberg column not yet rotated */
  int stop_j = -1;   /* first column count whose |g| met the tolerance */
  for (int k = 0;; ++k) {
    double* u = VC(ws, k);
    int flush = (k == m_eff);
    if (!flush) spmv(A, u, ws->w);

    /* the single global reduction of this step */
    for (int q = 0; q < k; ++q) ws->p[q] = dot(n, VC(ws, q), u);
    double alpha = dot(n, u, u);
    double gamma = 0.0;
    if (!flush) {
      for (int q = 0; q < k; ++q) ws->c[q] = dot(n, VC(ws, q), ws->w);
      gamma = dot(n, u, ws->w);
    }
    (*nred)++;
    if (!isfinite(alpha) || alpha < 0.0) return ORACLE_ERR_NONFINITE;
    double rho = sqrt(alpha);

    if (k == 0) {
      out->beta = rho;
      ws->g[0] = rho;
      if (rho <= tol_abs) {
        out->true_conv = 1;
        return ORACLE_OK;
      }
      if (flush) return ORACLE_OK;
    } else {
      HH(ws, k, k - 1) = rho;
      /* column k-1 is complete; rotate the pending columns when L of them
         are waiting, at the cycle's last step, or at a breakdown */
      if (k - rot_next >= depth || flush || rho == 0.0) {
        for (int c = rot_next; c < k; ++c) {
          double gc = rotate_column(ws, c);
          if (!isfinite(gc)) return ORACLE_ERR_NONFINITE;
          ws->gres[c + 1] = gc;
          if (hist) hist[it0 + c] = gc / bnorm;
          if (stop_j < 0 && gc <= tol_abs) stop_j = c + 1;
        }
        rot_next = k;
      }
      if (stop_j >= 0 && stop_j < k) {  /* met earlier: the steps since are discarded */
        out->j = stop_j;
        return ORACLE_OK;
      }
      if (rho == 0.0) {
        out->breakdown = 1;
        out->j = k;
        return ORACLE_OK;
      }
    }

    /* lagged normalization of column k and the new row of L */
    ORACLE_ROWS
    for (int64_t i = 0; i < n; ++i) u[i] = u[i] / rho;
    for (int q = 0; q < k; ++q) ws->p[q] = ws->p[q] / rho;
    if (scheme == ORACLE_MGS_1R) {
      for (int i = 0; i < k; ++i) {
        double s = 0.0;
        for (int q = i; q < k; ++q) s += TT(ws, i, q) * ws->p[q];
        TT(ws, i, k) = -s;
      }
      TT(ws, k, k) = 1.0;
    } else {
      for (int q = 0; q < k; ++q) LL(ws, k, q) = ws->p[q];
    }

    if (stop_j == k) {
      out->j = k;
      return ORACLE_OK;
    }
    if (flush) {
      out->j = k;
      return ORACLE_OK;
    }

    for (int q = 0; q < k; ++q) ws->r[q] = ws->c[q] / rho;
    ws->r[k] = (gamma / rho) / rho;

    double* vnext = VC(ws, k + 1);
    if (scheme == ORACLE_MGS_1R) {
      for (int i = 0; i <= k; ++i) {
        double s = 0.0;
        for (int q = 0; q <= i; ++q) s += TT(ws, q, i) * ws->r[q];
        ws->h[i] = s;
      }
      ORACLE_ROWS
      for (int64_t e = 0; e < n; ++e) vnext[e] = ws->w[e] / rho;
      for (int q = 0; q <= k; ++q) {
        const double* vq = VC(ws, q);
        double hq = ws->h[q];
        ORACLE_ROWS
        for (int64_t e = 0; e < n; ++e) vnext[e] = vnext[e] - vq[e] * hq;
      }
      for (int q = 0; q <= k; ++q) HH(ws, q, k) = ws->h[q];
    } else {
      /* the correction, the second reduction and the new column */
      cgs2_update(n, k, ws->V, n, ws->L, ws->ldt, ws->r, rho, ws->w, vnext, ws->h, ws->y,
                  &HH(ws, 0, k));
      (*nred)++;
      for (int q = 0; q <= k; ++q) ws->S2[(size_t)k * (size_t)ws->ldh + (size_t)q] = ws->y[q];
    }
    for (int q = 0; q <= k; ++q)
      if (!isfinite(HH(ws, q, k))) return ORACLE_ERR_NONFINITE;
  }
}

static void dump_cycle(const ws_t* ws, int scheme, int j, double* V_out, double* H_out,
                       double* T_out, double* g_out, double* S2_out, int32_t* j_out) {
  int m = ws->m;
  const double* tri = (scheme == ORACLE_CGS2 || scheme == ORACLE_TWOSYNCH) ? ws->L : ws->T;
  if (S2_out) memcpy(S2_out, ws->S2, sizeof(double) * (size_t)(m + 1) * (size_t)m);
  if (V_out) memcpy(V_out, ws->V, sizeof(double) * (size_t)ws->n * (size_t)(m + 2));
  if (H_out) memcpy(H_out, ws->H, sizeof(double) * (size_t)(m + 1) * (size_t)m);
  if (T_out) memcpy(T_out, tri, sizeof(double) * (size_t)(m + 2) * (size_t)(m + 2));
  if (g_out) memcpy(g_out, ws->g, sizeof(double) * (size_t)(m + 2));
  if (j_out) *j_out = j;
}

int oracle_gmres_solve(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                       const double* vals, int32_t m, int32_t scheme, const double* b, double* x,
                       double rtol, int64_t max_iters, oracle_info* info, double* hist_res,
                       double* V_out, double* H_out, double* T_out, double* g_out,
                       double* S2_out, int32_t* j_out) {
  return oracle_gmres_solve_depth(n, nnz, row_ptr, col_idx, vals, m, scheme, 1, b, x, rtol,
                                  max_iters, info, hist_res, V_out, H_out, T_out, g_out, S2_out,
                                  j_out);
}

int oracle_gmres_solve_depth(int64_t n, int64_t nnz, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                             int32_t depth, const double* b, double* x, double rtol,
                             int64_t max_iters, oracle_info* info, double* hist_res,
                             double* V_out, double* H_out, double* T_out, double* g_out,
                             double* S2_out, int32_t* j_out) {
  oracle_info loc;
  memset(&loc, 0, sizeof(loc));
  if (info) memset(info, 0, sizeof(*info));
  if (j_out) *j_out = 0;
  if (n < 1 || m < 1 || nnz < 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || !b || !x ||
      (nnz > 0 && (!col_idx || !vals)) || !(rtol >= 0.0) || max_iters < 0 ||
      (scheme != ORACLE_MGS && scheme != ORACLE_MGS_1R && scheme != ORACLE_CGS2 &&
       scheme != ORACLE_CGS2_3R && scheme != ORACLE_TWOSYNCH))
    return ORACLE_ERR_ARG;
  if (depth < 1 || (depth > 1 && scheme != ORACLE_MGS_1R && scheme != ORACLE_CGS2)) return ORACLE_ERR_ARG;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return ORACLE_ERR_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return ORACLE_ERR_ARG;
  for (int64_t e = 0; e < nnz; ++e)
    if (col_idx[e] < 0 || col_idx[e] >= n) return ORACLE_ERR_ARG;

  csr_t A = {n, row_ptr, col_idx, vals};
  double bnorm = sqrt(dot(n, b, b));
  loc.reductions = 1;
  if (!isfinite(bnorm)) {
    if (info) *info = loc;
    return ORACLE_ERR_NONFINITE;
  }
  if (bnorm == 0.0) {
    ORACLE_ROWS
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    loc.converged = 1;
    if (info) *info = loc;
    return ORACLE_OK;
  }
  double tol_abs = rtol * bnorm;

  ws_t ws;
  if (ws_alloc(&ws, n, m) != 0) return ORACLE_ERR_ARG;
  int status = ORACLE_OK;
  int64_t it = 0;
  for (;;) {
    int64_t left = max_iters - it;
    int m_eff = left < (int64_t)m ? (int)left : m;
    cycle_out co;
    if (scheme == ORACLE_MGS)
      status = cycle_mgs(&A, b, x, m_eff, tol_abs, bnorm, &ws, hist_res, it, &loc.reductions, &co);
    else if (scheme == ORACLE_CGS2_3R || scheme == ORACLE_TWOSYNCH)
      status = cycle_cgs(&A, b, x, m_eff, tol_abs, bnorm, scheme, &ws, hist_res, it,
                         &loc.reductions, &co);
    else
      status = cycle_lagged(&A, b, x, m_eff, tol_abs, bnorm, scheme, depth, &ws, hist_res, it,
                            &loc.reductions, &co);
    if (status != ORACLE_OK) break;
    if (co.j > 0) {
      update_solution(&ws, co.j, x);
      loc.cycles++;
      loc.rel_res_est = ws.gres[co.j] / bnorm;
      dump_cycle(&ws, scheme, co.j, V_out, H_out, T_out, g_out, S2_out, j_out);
    }
    it += co.j;
    if (co.breakdown) loc.breakdown = 1;
    if (co.true_conv || m_eff == 0) {
      loc.converged = co.true_conv;
      loc.rel_res_true = co.beta / bnorm;
      if (loc.cycles == 0) loc.rel_res_est = co.beta / bnorm;
      break;
    }
  }
  loc.iters = it;
  ws_free(&ws);
  if (info) *info = loc;
  return status;
}

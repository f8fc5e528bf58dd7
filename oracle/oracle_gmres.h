/*
 * CPU oracle for restarted GMRES(m) with three Gram-Schmidt schemes, written
 * from Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low synchronization GMRES
 * algorithms" (arXiv:1809.05805).
 *
 * TEST INFRASTRUCTURE ONLY. This is the slow, obviously sequential FP64
 * reference that the GPU library is checked against. Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * source with the GPU library: no headers, kernels, helpers or constants.
 *
 * All pointers are host pointers. Sums are taken in index order, one at a
 * time, with no blocking or reordering, so a reader can check every line
 * against the paper.
 */
#ifndef ORACLE_GMRES_H
#define ORACLE_GMRES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Orthogonalization scheme. */
enum {
  ORACLE_MGS = 0,    /* level-1 MGS-GMRES (Algorithm "MGS-GMRES", Section III)     */
  ORACLE_MGS_1R = 1, /* one-synchronization lagged compact-WY MGS (Sections II-III) */
  ORACLE_CGS2 = 2,   /* two-synchronization lagged CGS2 (Section II, level-2 CGS2)  */
  ORACLE_CGS2_3R = 3,  /* classical Gram-Schmidt with one re-orthogonalization pass:
                          three reductions per step (Section II, first listing)     */
  ORACLE_TWOSYNCH = 4  /* iterated classical Gram-Schmidt with two synchronizations,
                          T = I - L - L^T (Section II, Ruhe's loop invariant)        */
};

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_ARG = -1,
  ORACLE_ERR_NONFINITE = -3
};

typedef struct {
  int64_t iters;       /* Arnoldi columns completed over all cycles            */
  int32_t cycles;      /* restart cycles that completed at least one column    */
  int32_t converged;   /* 1 if the true residual met rtol*||b||                */
  int32_t breakdown;   /* 1 if some cycle ended on an exact (happy) breakdown  */
  int32_t pad;
  double rel_res_true; /* ||b - A x||_2 / ||b||_2 at exit                      */
  double rel_res_est;  /* last implicit |g_j| / ||b||_2                        */
  int64_t reductions;  /* global reductions (inner-product synchronizations)   */
} oracle_info;

/*
 * Solve A x = b by restarted GMRES(m).
 *   n, nnz, row_ptr[n+1], col_idx[nnz], vals[nnz]: CSR matrix, int32 indices.
 *   m >= 1: restart length. scheme: one of the ORACLE_* schemes above.
 *   b[n]; x[n]: initial guess on entry, solution on exit.
 *   rtol >= 0: stop when the residual 2-norm is <= rtol*||b||_2.
 *   max_iters >= 0: cap on Arnoldi columns.
 *   info: filled on return (may be NULL).
 *   hist_res (nullable, length max_iters): |g_k|/||b|| after each column.
 *   Dump of the last cycle (each nullable):
 *     V_out  n x (m+2), column-major, ld = n: the basis;
 *     H_out  (m+1) x m, column-major, ld = m+1: the unrotated Hessenberg matrix;
 *     T_out  (m+2) x (m+2), column-major: Malard-Paige T (one-reduce), the
 *            strictly lower L of V^T V = I + L + L^T (lagged CGS2 and the
 *            two-synchronization CGS), zero for the other schemes;
 *     g_out  m+2: the rotated right-hand side;
 *     S2_out (m+1) x m, column-major: CGS2's second-pass coefficients s
 *            (zero for the other schemes);
 *     j_out  number of columns the last cycle completed.
 * Returns ORACLE_OK, ORACLE_ERR_ARG or ORACLE_ERR_NONFINITE.
 */
int oracle_gmres_solve(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                       const double* vals, int32_t m, int32_t scheme, const double* b, double* x,
                       double rtol, int64_t max_iters, oracle_info* info, double* hist_res,
                       double* V_out, double* H_out, double* T_out, double* g_out, double* S2_out,
                       int32_t* j_out);

/*
 * The same solve with the Givens rotations and the stopping test of the
 * lagged schemes (ORACLE_MGS_1R, ORACLE_CGS2) applied depth columns at a time
 * (the depth-L pipeline of Section III; depth 1 is oracle_gmres_solve). The
 * iterate, iteration counts and dumps are those of depth 1; a cycle that
 * stops early runs up to depth - 1 more Arnoldi steps first, which shows in
 * info->reductions. depth < 1, or depth > 1 with another scheme, gives
 * ORACLE_ERR_ARG.
 */
int oracle_gmres_solve_depth(int64_t n, int64_t nnz, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                             int32_t depth, const double* b, double* x, double rtol,
                             int64_t max_iters, oracle_info* info, double* hist_res,
                             double* V_out, double* H_out, double* T_out, double* g_out,
                             double* S2_out, int32_t* j_out);

/*
 * The column updates of two baselines, the very code their cycles run,
 * exposed so that tests can drive them with a basis that is not orthonormal
 * (where the terms they exist for act at first order). V: n x (k+1) (or
 * i+1), column-major, ld = n.
 *   oracle_cgs_two_passes: Alg 1's two classical Gram-Schmidt passes of w
 *     against V[:,0:i+1]; w is updated in place, hcol (i+1) receives the sum
 *     of both passes' coefficients.
 *   oracle_cgs2_update: the lagged CGS2 update (Alg 5) of step k, given the
 *     first-pass coefficients r (k+1), the strictly lower L of V^T V on the
 *     leading (k+1) x (k+1) block (column-major, ld = k+1, entry (a, q) for
 *     a > q), rho and the SpMV output w (n): vnext (n) the new column, h the
 *     corrected coefficients (I - L) r, s the second pass's coefficients,
 *     hcol = h + s the Hessenberg column (k+1 each).
 */
void oracle_cgs_two_passes(int64_t n, int32_t i, const double* V, double* w, double* hcol);
void oracle_cgs2_update(int64_t n, int32_t k, const double* V, const double* L, const double* r,
                        double rho, const double* w, double* vnext, double* h, double* s,
                        double* hcol);

/* y = A x, sequential sum over each row in CSR order. */
void oracle_spmv(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                 const double* x, double* y);

#ifdef __cplusplus
}
#endif

#endif

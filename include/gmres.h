/*
 * gmres.h - restarted GMRES(m) on one AMD MI355X (gfx950) with five
 * Gram-Schmidt schemes for the Arnoldi process, after Swirydowicz, Langou,
 * Ananthan, Yang, Thomas, "Low synchronization GMRES algorithms"
 * (arXiv:1809.05805), in FP64; the one-reduce scheme also on a float32 or
 * bfloat16 basis inside FP64 iterative refinement, and for many independent
 * systems in one persistent launch (the gmres_batch_* calls below):
 *
 *   GMRES_MGS_1R  one global reduction per Arnoldi step: the level-2 MGS in
 *                 compact WY form with lagged normalization of R's diagonal
 *                 (Section II, level-2 MGS with normalization lag; Section III,
 *                 one-synchronization MGS-GMRES). Each step is a CSR SpMV of
 *                 the still-unnormalized newest column, one fused projection
 *                 [V^T u, V^T w] with a single device-wide reduction, the lagged
 *                 norm and the (I + L)^{-1} correction through the Malard-Paige
 *                 T matrix, and one MAXPY.
 *   GMRES_MGS     level-1 MGS-GMRES (Section III, the Saad-Schultz listing):
 *                 i+2 reductions in iteration i.
 *   GMRES_CGS2    two reductions per step: lagged iterated classical
 *                 Gram-Schmidt (Section II, level-2 CGS2 with normalization lag).
 *   GMRES_CGS2_3R three reductions per step: classical Gram-Schmidt with one
 *                 re-orthogonalization pass on a normalized basis (Section II,
 *                 the first listing, two iterations; the paper's GPU approach
 *                 "CGS-2 GMRES").
 *   GMRES_TWO_SYNCH  two reductions per step: iterated classical Gram-Schmidt
 *                 in Ruhe's two-synchronization form, [V^T w, V^T v_i] in one
 *                 reduction, coefficients (I - L - L^T) V^T w, then the norm
 *                 (Section II; the paper's GPU approach "two-synch GMRES").
 *   GMRES_MGS_1R_IR32  the GMRES_MGS_1R step on a float32 basis. Every
 *                 restart computes r = b - A x and ||r|| in float64 from the
 *                 CSR arrays (the float64 master), checks the tolerance on
 *                 that true residual, and starts the cycle from
 *                 float32(r / ||r||). Inside the cycle the basis, the SpMV
 *                 output, the SpMV (float32 values of the sliced copy of A, or
 *                 the CSR values with float32 vector entries), the projection
 *                 products and per-lane sums and the MAXPY are float32; the
 *                 cross-lane and device-wide sums, the lagged norm, the T
 *                 matrix, the Hessenberg column, the Givens least squares and
 *                 the back substitution are float64, and x += ||r|| V y
 *                 accumulates in float64. Restarted GMRES is then iterative
 *                 refinement with float32 inner cycles; the precision is not
 *                 discussed in the paper.
 *   GMRES_MGS_1R_IR16  an experiment: the same refinement with the basis and
 *                 the SpMV output stored in bfloat16 (8-bit significand,
 *                 round to nearest even). Every product and per-lane sum runs
 *                 in float32 on values widened from bfloat16; the sliced copy
 *                 of A keeps float32 values; everything the float32-basis
 *                 scheme keeps in float64 stays float64.
 *
 * The problem is A x = b with residual r = b - A x and initial guess x0
 * (Section III); A is in CSR form (Section V-B); all vectors live in device
 * memory (Section V-B). The relative tolerance is on ||b - A x||_2 / ||b||_2.
 *
 * Pointers are DEVICE pointers unless marked "host". The library never
 * allocates or frees device memory at run time: the caller passes one
 * workspace buffer. Its only allocations are the host-side context and a
 * small pinned host buffer (hipHostMalloc) for per-cycle status readback.
 * For callers that cannot allocate at all, gmres_solve_noalloc (at the end)
 * runs a whole solve in a fixed scratch array that the library's code object
 * reserves on each GPU it is loaded onto.
 *
 * Every call is enqueued on the HIP stream given to gmres_create. A context is
 * bound to that stream and is not thread-safe; use one context per stream.
 */
#ifndef GMRES_H
#define GMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmres_ctx gmres_ctx; /* opaque */

typedef enum {
  GMRES_MGS = 0,
  GMRES_MGS_1R = 1,
  GMRES_CGS2 = 2,
  GMRES_MGS_1R_IR32 = 3,
  GMRES_MGS_1R_IR16 = 4,
  GMRES_CGS2_3R = 5,
  GMRES_TWO_SYNCH = 6
} gmres_scheme;

typedef enum {
  GMRES_OK = 0,
  GMRES_ERR_ARG = -1,       /* invalid argument or malformed CSR structure          */
  GMRES_ERR_HIP = -2,       /* a HIP runtime call or kernel launch failed           */
  GMRES_ERR_NONFINITE = -3, /* NaN or Inf in a norm, Hessenberg entry or residual   */
  GMRES_ERR_WORKSPACE = -4, /* workspace smaller than gmres_workspace_bytes()        */
  GMRES_ERR_TOO_LARGE = -5  /* gmres_solve_noalloc: the problem's workspace exceeds
                               GMRES_NOALLOC_SCRATCH_BYTES                          */
} gmres_status;

/* Largest restart length the kernels' on-chip buffers are sized for. */
#define GMRES_MAX_RESTART 256

typedef struct {
  int64_t iters;       /* Arnoldi columns completed, summed over cycles              */
  int32_t cycles;      /* restart cycles that completed at least one column          */
  int32_t converged;   /* 1 if ||b - A x|| <= rtol ||b|| was verified on the device  */
  int32_t breakdown;   /* 1 if a cycle ended on an exact (happy) breakdown, rho == 0  */
  int32_t pad;
  double rel_res_true; /* ||b - A x||_2 / ||b||_2 at exit, recomputed from x          */
  double rel_res_est;  /* last implicit |g_j| / ||b||_2 from the Givens recurrence    */
  int64_t reductions;  /* device-wide reductions performed, counted on the device     */
} gmres_info;

/*
 * Bytes of device workspace gmres_create needs for n rows, restart m and the
 * given scheme (0 if the arguments are invalid). The workspace holds the
 * basis V (n x (m+2), column-major, leading dimension n rounded up to 64),
 * the Hessenberg and T matrices, Givens data and reduction scratch.
 */
size_t gmres_workspace_bytes(int64_t n, int32_t m, int32_t scheme);

/*
 * Launch and format choices of a context, for gmres_workspace_bytes_ex and
 * gmres_create_ex. Zero every field (gmres_options_init) and set only what
 * should differ: a zero field always means the library's own choice, which
 * is what gmres_workspace_bytes and gmres_create use. The arithmetic of a
 * solve does not depend on these, except the pipeline depth (below) and the
 * rounding of the per-row sums, which differs between the CSR path and the
 * sliced copy (whose three forms agree bit for bit).
 *   format: GMRES_OPT_FORMAT_AUTO (sliced copy of A for regular matrices,
 *     stored by diagonals or with 16-bit column deltas where they fit; see
 *     gmres_create), _CSR (always read the CSR arrays), _SELL64 (the sliced
 *     copy with int32 column indices, whatever its padding), _SELL64_D16 (the
 *     sliced copy whatever its padding, with 16-bit deltas where every slice
 *     column fits them, else int32 indices) or _SELL64_DIAG (the sliced copy
 *     by diagonals whatever its padding where every row's columns are
 *     strictly increasing, else as _SELL64_D16). Slices wider than 4096 or
 *     n >= 2^28 always fall back to CSR.
 *   rows_per_lane: 0, or 1, 2, 4 or 8 rows per lane of the row-tiled kernels
 *     (tiles of 256 rows per lane-row). The default is the largest that leaves
 *     at least 512 tiles. The workspace size depends on it: give the same
 *     options to gmres_workspace_bytes_ex and gmres_create_ex.
 *   csr_spmv_shape: 0, or the CSR SpMV shape as 100 * (lanes per row) +
 *     (entries per lane): 108, 208, 408, 804, 808 or 6401. The default
 *     follows the mean row length.
 *   split_spmv: 0 computes w = A u inside the step kernel; 1 in a launch of
 *     its own before it (the step kernel then reads w back).
 *   pipeline_depth: 0 or 1 applies the Givens rotations and the stopping test
 *     every step; L >= 2 (the lagged schemes GMRES_MGS_1R, GMRES_CGS2 and the
 *     refinement forms only) every L steps, to the L columns finished since
 *     (Section III, the depth-L pipeline; the paper's listing has L = 2). The
 *     rotations feed nothing back into the Arnoldi recurrence: the iterate is
 *     the same, and a cycle stops at the same column count, noticed up to
 *     L - 1 steps later (the steps run in between cost reductions and are
 *     discarded). On the GPU the rotations always run beside the next MAXPY,
 *     off the step's critical path; the depth only batches them.
 *   reserved: must be zero.
 * A field out of range gives GMRES_ERR_ARG (0 bytes from
 * gmres_workspace_bytes_ex).
 */
enum {
  GMRES_OPT_FORMAT_AUTO = 0,
  GMRES_OPT_FORMAT_CSR = 1,
  GMRES_OPT_FORMAT_SELL64 = 2,
  GMRES_OPT_FORMAT_SELL64_D16 = 3,
  GMRES_OPT_FORMAT_SELL64_DIAG = 4
};
typedef struct {
  int32_t format;
  int32_t rows_per_lane;
  int32_t csr_spmv_shape;
  int32_t split_spmv;
  int32_t pipeline_depth;
  int32_t reserved[3];
} gmres_options;

/* Zero every field: the library's own choices. */
void gmres_options_init(gmres_options* opt /* host */);

/* gmres_workspace_bytes for a context created with these options (NULL: defaults). */
size_t gmres_workspace_bytes_ex(int64_t n, int32_t m, int32_t scheme,
                                const gmres_options* opt /* host, nullable */);

/*
 * Bind a CSR matrix and a workspace to a new context.
 *   n >= 1 rows (square A); nnz in [0, 2^31); row_ptr int32[n+1], col_idx
 *   int32[nnz] (any order within a row), vals float64[nnz]: caller-owned
 *   device arrays that must stay valid and unchanged while the context lives.
 *   1 <= m <= GMRES_MAX_RESTART; scheme a gmres_scheme value.
 *   workspace: device buffer of ws_bytes >= gmres_workspace_bytes(n, m, scheme),
 *   256-byte aligned, caller-owned, exclusively used by this context.
 *   hip_stream: the hipStream_t all work is enqueued on (NULL = default stream).
 * The CSR structure is checked on the device (row_ptr[0] == 0, row_ptr[n] ==
 * nnz, non-decreasing row_ptr, 0 <= col_idx < n); a malformed matrix gives
 * GMRES_ERR_ARG and no context. On success *out holds the context.
 * Sparse format: for n < 2^28, gmres_create plans a sliced-ELL copy of A
 * (SELL-64: per slice of 64 rows, slice column j of every row stored
 * together, so a wavefront's index and value loads are contiguous and no row
 * pointers are read) in one of three forms (see gmres_matrix_storage_bytes):
 *   - by diagonals, when every row's columns are strictly increasing and a
 *     slice column per distinct col - row value among each slice's rows adds
 *     at most a quarter to nnz (stencils): no per-entry column index;
 *   - otherwise, when padding every slice to its longest row adds at most a
 *     quarter to nnz (other regular matrices), by rows, with 2-byte column
 *     deltas when every slice column's col - row values span at most 65535,
 *     else int32 column indices. The library allocates no
 * device memory: gmres_matrix_storage_bytes gives the size of the copy and
 * gmres_set_matrix_storage builds it in a caller-owned buffer; from then on
 * every SpMV reads the copy, not the caller's arrays (after changing vals in
 * place, call gmres_refresh_matrix). Without that call the SpMV reads the CSR
 * arrays directly. The slice widths are computed at create in the
 * workspace's basis region.
 */
int gmres_create(gmres_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                 void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * gmres_create with launch and format options (NULL: the defaults, the same
 * as gmres_create). The workspace must be at least
 * gmres_workspace_bytes_ex(n, m, scheme, opt). GMRES_ERR_ARG as for
 * gmres_create, or for an invalid option.
 */
int gmres_create_ex(gmres_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                    const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                    void* workspace, size_t ws_bytes, void* hip_stream,
                    const gmres_options* opt /* host, nullable */);

/*
 * Solve A x = b by restarted GMRES(m) with the context's scheme.
 *   b: float64[n]; x: float64[n], the initial guess on entry, the iterate on exit.
 *   rtol >= 0: stop once ||b - A x||_2 <= rtol ||b||_2 holds for the true
 *   residual. Inside a cycle the implicit Givens residual |g_k| decides when the
 *   cycle ends (for the lagged schemes one step after column k-1 is formed,
 *   since its last Hessenberg entry arrives with the next reduction); every
 *   restart then recomputes b - A x, and only that true residual ends the solve.
 *   max_iters >= 0: cap on Arnoldi columns over all cycles.
 *   info (host, nullable): filled on return.
 *   hist_res (host, nullable, max_iters doubles): |g_k| / ||b|| after each column.
 *   hist_orth (host, nullable, max_iters doubles): loss of orthogonality per
 *   column, ||S||_2 with Paige's S = (I + L^T)^{-1} L^T = I - T, L the strictly
 *   lower part of V^T V: entry i of a cycle covers its basis vectors
 *   v_0..v_i (the leading (i+1) x (i+1) block of T; 0 for i = 0). Computed on
 *   the host from the T (one-reduce MGS) or L (CGS2) the device built (T for
 *   GMRES_MGS_1R_IR32 and _IR16 too, L for GMRES_TWO_SYNCH), by power
 *   iteration to a relative change of 1e-14, while the device runs the next
 *   cycle (the last cycle's after the device has finished); NaN for
 *   GMRES_MGS and GMRES_CGS2_3R, which form neither. Its host work lengthens
 *   the solve only where the power iterations outlast a cycle; pass NULL when
 *   timing.
 * Blocks until the solve has finished on the stream. Returns GMRES_OK when the
 * solve ran to convergence or to max_iters (info->converged tells which),
 * GMRES_ERR_NONFINITE if a NaN or Inf appeared (x then holds the last finished
 * cycle's iterate), or GMRES_ERR_ARG / GMRES_ERR_HIP. If ||b|| == 0, x is set to
 * zero and the solve reports convergence with no iterations.
 */
int gmres_solve(gmres_ctx* ctx, const double* b, double* x, double rtol, int64_t max_iters,
                gmres_info* info, double* hist_res, double* hist_orth);

/*
 * Release the context (host memory only; the workspace, the CSR arrays and
 * any matrix storage stay the caller's).
 */
int gmres_destroy(gmres_ctx* ctx);

/*
 * Device bytes the context's sliced-ELL copy of A needs (0 when no copy is
 * planned and the SpMV reads the CSR arrays): ceil(n/64) + 1 int64 slice
 * offsets, then the column indices and the values of every stored entry (64
 * per slice and slice column; padding entries hold value 0): float64, or for
 * the refinement schemes float32 values (their inner cycles' SpMV) followed
 * by float64 ones (their float64 restart residual); each part 256-byte
 * aligned. The column indices are
 *   - by diagonals: one int32 diagonal d per slice column and nothing per
 *     entry: slice column j of row r holds A[r, r + d_j] (0 where A has no
 *     such entry, or r + d_j is outside [0, n)); a slice's diagonals
 *     increase with j, so each row's entries keep their order;
 *   - with deltas: one int32 base per slice column followed by a 16-bit delta
 *     per entry: the column of entry j of row r is r + base + delta;
 *   - else an int32 column index per entry.
 */
int gmres_matrix_storage_bytes(gmres_ctx* ctx, size_t* bytes /* host */);

/*
 * Build the sliced copy of A in storage: a caller-owned device buffer of at
 * least gmres_matrix_storage_bytes bytes, 256-byte aligned, that stays valid
 * and untouched while the context uses it. Blocks until the copy is built.
 * storage == NULL goes back to reading the CSR arrays. GMRES_ERR_ARG if no
 * copy is planned, the buffer is too small, misaligned or not device memory,
 * or a row no longer fits its slice.
 */
int gmres_set_matrix_storage(gmres_ctx* ctx, void* storage, size_t bytes);

/*
 * Re-read A's values (and re-check its structure) after the caller changed
 * vals in place; the structure must be the one given to gmres_create. Blocks
 * until done. GMRES_ERR_ARG if the structure is malformed or a row no longer
 * fits its slice of the copy: the context's matrix is then invalid, and
 * gmres_solve and gmres_spmv return GMRES_ERR_ARG until a later refresh
 * succeeds.
 */
int gmres_refresh_matrix(gmres_ctx* ctx);

enum {
  GMRES_FORMAT_CSR = 0,
  GMRES_FORMAT_SELL64 = 1,
  GMRES_FORMAT_SELL64_D16 = 2,
  GMRES_FORMAT_SELL64_DIAG = 3
};
/*
 * The SpMV format in use (GMRES_FORMAT_*) and the matrix entries it reads:
 * nnz for CSR, nnz plus padding for the sliced copies (SELL64: int32 column
 * indices; SELL64_D16: 16-bit column deltas; SELL64_DIAG: by diagonals). The
 * sliced forms give the same bits: each row's products are accumulated in
 * storage order by fused multiply-adds, padding adding exact zeros (for
 * finite x). The CSR path sums the same products with other roundings (a
 * separate multiply and add for most entries, and a tree over the lanes of
 * a long row).
 */
int gmres_get_format(gmres_ctx* ctx, int32_t* format, int64_t* stored_entries);

/* Static English description of a gmres_status value. */
const char* gmres_status_string(int status);

/*
 * y = A x with the context's matrix and SpMV kernel, enqueued on its stream
 * without waiting. x and y: float64[n], must not overlap.
 */
int gmres_spmv(gmres_ctx* ctx, const double* x, double* y);

/*
 * Diagnostics of the last cycle that completed at least one column (host
 * copies, each nullable):
 *   H (host, (m+1) x m, column-major): the unrotated Hessenberg matrix;
 *   T (host, (m+2) x (m+2), column-major): for GMRES_MGS_1R (and _IR32, _IR16) the Malard-Paige
 *     T = (I + L^T)^{-1} built one column per step, whose leading blocks give
 *     Paige's loss-of-orthogonality measure S = I - T (Section II); for
 *     GMRES_CGS2 and GMRES_TWO_SYNCH the strictly lower L with
 *     V^T V = I + L + L^T, one row per step; zeros for GMRES_MGS and
 *     GMRES_CGS2_3R. Columns 0..j-1 are formed: the cycle's last
 *     step computes only the norm of column j (and of a cycle that ends on
 *     the tolerance check, column j is formed too);
 *   g (host, m+2): the rotated right-hand side of the least-squares problem
 *     (for GMRES_MGS_1R_IR32 and _IR16 relative to the cycle's restart residual norm:
 *     the cycle starts from r / ||r||, and H is that of the reduced-precision basis);
 *   j (host): the number of columns that cycle completed.
 */
int gmres_last_cycle(gmres_ctx* ctx, double* H, double* T, double* g, int32_t* j);

/*
 * Device pointer to the float64 basis V inside the workspace and its leading
 * dimension (in elements). Columns 0..j-1 of the last cycle hold its
 * orthonormal basis until the next solve, except that a solve that ends by
 * converging overwrites column 0 with the final residual it verified.
 * GMRES_ERR_ARG for GMRES_MGS_1R_IR32 and _IR16, whose basis is float32 or bfloat16.
 */
int gmres_basis(gmres_ctx* ctx, double** V, int64_t* ldv);

/*
 * Per-kernel timing for measurement (lagged schemes). When enabled, every
 * launch of the step kernel (projection + device-wide reduction + small dense
 * step, with the SpMV fused in unless it runs as a launch of its own), of the
 * separate SpMV kernel and of the MAXPY kernel carries start/stop HIP events
 * attached to its dispatch (hipExtLaunchKernel), so they time the kernel
 * alone; launches that the cycle's done flag skipped, and the MAXPY of a step
 * whose extra workgroup ended the cycle, are not counted. bytes is the
 * algorithmic HBM traffic of the counted launches by the method's byte
 * model, whatever the format in use: A = 12 nnz + 4 (n+1), the CSR arrays
 * (8 nnz + 4 (n+1) for the refinement schemes, whose SpMV reads float32
 * values). The figures below are for a float64 basis; for the float32
 * (bfloat16) basis every 8 n is 4 n (2 n):
 *   step k, SpMV fused:     A + 16 n + 8 n (k+1)    (A, u read and w written by
 *                                                     the SpMV, V[:,0:k+1] read)
 *   step k, SpMV separate:  8 n (k+1) + 8 n         (V[:,0:k+1], w read)
 *   separate SpMV:          A + 16 n                (A, u, w written)
 *   last step of a cycle (norm of column k only):  8 n
 *   CGS2 second pass:  8 n (k+2)                          (V[:,0:k+1] and z)
 *   MAXPY at step k:   8 n (k+1) + 16 n                   (V[:,0:k+1], w or z, new column)
 * gmres_set_timing(ctx, 1) enables and clears the totals; (ctx, 0) disables.
 */
enum { GMRES_KSTAT_STEP = 0, GMRES_KSTAT_MAXPY = 1, GMRES_KSTAT_SPMV = 2, GMRES_KSTAT_COUNT = 3 };
typedef struct {
  double ms;        /* summed event-to-event time of the counted launches */
  double bytes;     /* summed algorithmic bytes */
  int64_t launches; /* counted launches */
} gmres_kernel_stat;
int gmres_set_timing(gmres_ctx* ctx, int enable);
int gmres_get_timing(gmres_ctx* ctx, gmres_kernel_stat* stats /* host, GMRES_KSTAT_COUNT */);

/* ------------------------------------------------------------------------
 * Batched solves: many independent systems in one persistent launch.
 *
 * The systems are the diagonal blocks of one block-diagonal CSR matrix:
 * system i owns rows (and columns) [row_off[i], row_off[i+1]) of A and the
 * same entries of b and x. Each is solved by restarted one-reduce GMRES(m)
 * (the GMRES_MGS_1R step of Section III, or its GMRES_MGS_1R_IR32 form) with
 * its own restart cycles, lagged normalization state, T matrix, Givens
 * rotations and stopping test ||b_i - A_i x_i|| <= rtol ||b_i||. One kernel
 * launch solves the whole batch: a fixed number of workgroups take entries
 * from a device-side queue until it is empty. An entry is a whole system, or
 * one row part of a larger system: such a team of workgroups (up to 16) adds
 * its parts' sums through global memory once per step, where a one-part
 * system reduces within its workgroup and the single-system path across the
 * GPU (the paper maps its reductions onto SIMD lanes on the CPU and onto the
 * whole GPU for one system, Section V-B; here the batch fills the GPU).
 * gmres_batch_solve_async makes no host synchronization, memset or
 * allocation, so it can be captured into a HIP graph;
 * gmres_batch_capture / gmres_batch_replay do that inside the library.
 * ------------------------------------------------------------------------ */
typedef struct gmres_batch gmres_batch; /* opaque */

/* Per-system result, written by the device (the same 32-byte layout there). */
typedef struct {
  int64_t iters;       /* Arnoldi columns completed over all cycles                 */
  int32_t cycles;      /* restart cycles that ran at least one Arnoldi step         */
  int32_t converged;   /* 1 if ||b_i - A_i x_i|| <= rtol ||b_i|| was verified       */
  int32_t status;      /* GMRES_OK, GMRES_ERR_NONFINITE, or GMRES_ERR_HIP if the
                          parts of this system's team did not all run at once
                          (each waits about half a minute at most, then gives up) */
  int32_t breakdown;   /* 1 if a cycle ended on an exact breakdown, rho == 0        */
  double rel_res_true; /* ||b_i - A_i x_i|| / ||b_i|| at exit, from a residual the
                          device computed in float64 (0 when ||b_i|| == 0)           */
} gmres_batch_info;

enum { GMRES_BATCH_ORDER_NATURAL = 0, GMRES_BATCH_ORDER_LARGEST_FIRST = 1 };

/*
 * Device workspace bytes for nsys systems with row offsets row_off (host,
 * int64[nsys+1], row_off[0] = 0, strictly increasing, every system below
 * 2^28 rows, total below 2^31), restart m (1..GMRES_MAX_RESTART) and scheme
 * GMRES_MGS_1R or GMRES_MGS_1R_IR32; 0 if the arguments are invalid. Per
 * system: the basis (m+1 columns of n_i rounded up to 64, float64 or
 * float32), a barrier counter and a result record; per possible row part of
 * a system (min(16, ceil(n_i / 256)) of them): the Hessenberg, T and Givens
 * arrays, a state record and two rows of reduction partials; for the batch:
 * the queue, the SpMV output, a float64 copy of x for the autotuner, and for
 * GMRES_MGS_1R_IR32 the float64 restart residual.
 */
size_t gmres_batch_workspace_bytes(int32_t nsys, const int64_t* row_off, int32_t m, int32_t scheme);

/*
 * Bind a block-diagonal CSR matrix (device arrays as for gmres_create, n =
 * row_off[nsys] rows) and a workspace (device, 256-byte aligned,
 * ws_bytes >= gmres_batch_workspace_bytes) to a new batch context. Checks the
 * CSR structure and that every column index of a system's rows lies in the
 * system's own range; GMRES_ERR_ARG otherwise. Blocks until the checks are
 * done and the copy of the matrix by diagonals is planned (see
 * gmres_batch_matrix_storage_bytes; until it is built the SpMV reads the CSR
 * arrays). The initial configuration is 256-thread workgroups, as many as the
 * GPU holds at once, systems largest first, parts of 8192 rows.
 */
int gmres_batch_create(gmres_batch** out, int32_t nsys, const int64_t* row_off, int64_t nnz,
                       const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                       int32_t m, int32_t scheme, void* workspace, size_t ws_bytes,
                       void* hip_stream);

/* Release the context and any captured graph (host resources only). */
int gmres_batch_destroy(gmres_batch* bt);

/*
 * The batch's copy of A by diagonals (the form gmres_matrix_storage_bytes
 * describes, over the whole block-diagonal matrix: 64-row slices of global
 * rows, which may straddle two systems; a slice column per distinct col - row
 * value among the slice's rows; float64 values). gmres_batch_create plans it
 * when every row's columns are strictly increasing and it adds at most a
 * quarter to nnz (stencil systems); *bytes is 0 otherwise.
 * gmres_batch_set_matrix_storage builds it in a caller-owned device buffer of
 * at least that size (256-byte aligned, untouched while in use) and blocks
 * until done; from then on the batched SpMV reads it instead of the CSR
 * arrays (each row's products are accumulated in the same order, by fused
 * multiply-adds, in both forms, so the results are the same bits). storage ==
 * NULL goes back to the CSR arrays. Either call discards a captured graph.
 * GMRES_ERR_ARG if no copy is planned, the buffer is too small, misaligned or
 * not device memory, or the structure no longer fits the plan.
 */
int gmres_batch_matrix_storage_bytes(gmres_batch* bt, size_t* bytes /* host */);
int gmres_batch_set_matrix_storage(gmres_batch* bt, void* storage, size_t bytes);
/* GMRES_FORMAT_CSR or GMRES_FORMAT_SELL64_DIAG, and the entries the SpMV reads. */
int gmres_batch_get_format(gmres_batch* bt, int32_t* format, int64_t* stored_entries);

/* Change the stream later work is enqueued on. */
int gmres_batch_set_stream(gmres_batch* bt, void* hip_stream);

/*
 * Polls a part of a team makes at one team barrier before it gives up and
 * its system ends with status GMRES_ERR_HIP (every kernel still ends
 * normally). The default, GMRES_BATCH_WAIT_LIMIT, is about half a minute of
 * waiting at least; smaller limits serve tests of that failure path. polls in
 * [0, GMRES_BATCH_WAIT_LIMIT], else GMRES_ERR_ARG. Discards a captured graph
 * (gmres_batch_replay then returns GMRES_ERR_ARG until the next capture).
 */
#define GMRES_BATCH_WAIT_LIMIT (1u << 23)
int gmres_batch_set_wait_limit(gmres_batch* bt, uint32_t polls);

/*
 * Enqueue one batched solve and return without waiting.
 *   b, x: float64[n] (x: initial guesses in, solutions out); rtol >= 0;
 *   max_iters >= 0: cap on Arnoldi columns per system;
 *   info: device array of nsys gmres_batch_info, or NULL for the context's
 *   own (read it with gmres_batch_read_info).
 * Only null pointers and negative values are refused here; the device
 * pointers are the caller's to get right.
 */
int gmres_batch_solve_async(gmres_batch* bt, const double* b, double* x, double rtol,
                            int64_t max_iters, gmres_batch_info* info);

/*
 * The same, then wait: info (host, nullable, nsys entries) receives the
 * results. Returns GMRES_ERR_HIP if a team could not assemble,
 * GMRES_ERR_NONFINITE if any system met a NaN or Inf (the others are still
 * solved), else GMRES_OK.
 */
int gmres_batch_solve(gmres_batch* bt, const double* b, double* x, double rtol, int64_t max_iters,
                      gmres_batch_info* info);

/* Copy the context's own result array to info (host, nsys entries); waits. */
int gmres_batch_read_info(gmres_batch* bt, gmres_batch_info* info);

/*
 * Launch configuration: block_size 256, 512 or 1024 threads per workgroup;
 * grid >= 1 persistent workgroups (0: as many as the GPU holds at once, at
 * most the number of queue entries); order GMRES_BATCH_ORDER_*; part_rows:
 * system i is split into ceil(n_i / part_rows) parts (0: never split), but
 * at most 16, at most one per 256 rows, and at most the grid or what the GPU
 * holds at once. Blocks (the queue is uploaded). Each system's arithmetic is
 * fixed by the block size and its number of parts; the grid and the order
 * change only the time. get_config reports the grid in use and the largest
 * team (host pointers, each nullable).
 */
int gmres_batch_set_config(gmres_batch* bt, int32_t block_size, int32_t grid, int32_t order,
                           int64_t part_rows);
int gmres_batch_get_config(gmres_batch* bt, int32_t* block_size, int32_t* grid, int32_t* order,
                           int64_t* part_rows, int32_t* max_parts);

/*
 * How the batched kernel loads basis columns: GMRES_BATCH_LOADS_CACHED through
 * the caches (the MAXPY then re-reads a part's columns from the last-level
 * cache), GMRES_BATCH_LOADS_STREAMED non-temporal (faster when the bases in
 * use at once far exceed that cache), or GMRES_BATCH_LOADS_AUTO (the default):
 * streamed when the running workgroups' share of the bases, queue entries
 * times m+1 columns, exceeds 384 MiB. The results are the same either way.
 * set_loads re-applies the configuration (Blocks; discards a captured graph).
 * get_loads reports the mode and whether the current configuration streams
 * (host pointers, nullable).
 */
enum { GMRES_BATCH_LOADS_AUTO = 0, GMRES_BATCH_LOADS_CACHED = 1, GMRES_BATCH_LOADS_STREAMED = 2 };
int gmres_batch_set_loads(gmres_batch* bt, int32_t mode);
int gmres_batch_get_loads(gmres_batch* bt, int32_t* mode, int32_t* streamed);

typedef struct {
  int32_t block_size, grid, order;
  float ms; /* event-timed duration of the solve */
  int64_t part_rows;
  int32_t streamed; /* basis columns loaded non-temporal in this trial */
} gmres_batch_trial;

/*
 * Time one solve of (b, x, rtol, max_iters) under candidate configurations
 * after one warm-up solve: block sizes 256, 512 and 1024 with parts of
 * 16384, 8192 or 4096 rows or no split (largest first, as many workgroups as
 * the GPU holds), then for the fastest a grid of one workgroup per compute
 * unit and the natural order, and (under GMRES_BATCH_LOADS_AUTO) the best so
 * far with the other load form, which becomes the mode if it wins. Keeps the
 * fastest and leaves x as it was on
 * entry (it is restored from the workspace's copy before every trial).
 * trials (host, nullable, max_trials entries) and ntrials (host, nullable)
 * report what was timed. Blocks.
 */
int gmres_batch_autotune(gmres_batch* bt, const double* b, double* x, double rtol,
                         int64_t max_iters, gmres_batch_trial* trials, int32_t max_trials,
                         int32_t* ntrials);

/*
 * Capture one gmres_batch_solve_async(b, x, rtol, max_iters, NULL) with the
 * current configuration into a HIP graph held by the context (replacing any
 * earlier one); gmres_batch_replay launches it on the context's stream
 * without waiting. The graph keeps the pointers it was captured with: refill
 * b and x in place between replays. Results go to the context's own array.
 * gmres_batch_set_config and gmres_batch_autotune discard the graph (it holds
 * the old grid, block size and queue length): gmres_batch_replay then returns
 * GMRES_ERR_ARG until the next capture.
 */
int gmres_batch_capture(gmres_batch* bt, const double* b, double* x, double rtol,
                        int64_t max_iters);
int gmres_batch_replay(gmres_batch* bt);

/* ------------------------------------------------------------------------
 * One solve that allocates nothing.
 *
 * For callers that cannot allocate memory: code that must not call
 * hipMalloc or hipHostMalloc (tight serving loops, harnesses that forbid
 * allocation). gmres_solve_noalloc does the work of gmres_create +
 * gmres_solve + gmres_destroy for one solve without allocating device or host
 * memory: its workspace is a static device array of
 * GMRES_NOALLOC_SCRATCH_BYTES in the library's code object (each GPU the
 * library runs on holds one copy from the first call on it until the process
 * ends), the context and its status readback live on the call's stack, the
 * SpMV reads the CSR arrays directly (no sliced copy), and no timing events
 * are made.
 *   n, nnz, row_ptr, col_idx, vals, m, scheme: as for gmres_create (device
 *   arrays, checked on the device on every call).
 *   b, x, rtol, max_iters, info (host, nullable), hist_res (host, nullable,
 *   max_iters doubles): as for gmres_solve.
 *   hip_stream: the stream to enqueue on (NULL = default stream); it must
 *   belong to the current device, whose scratch copy the call uses.
 * Results: the arithmetic of gmres_create + gmres_solve on the same stream
 * with the CSR format (the iterate, info and hist_res are the same).
 * Errors: GMRES_ERR_TOO_LARGE when gmres_workspace_bytes(n, m, scheme)
 * exceeds GMRES_NOALLOC_SCRATCH_BYTES (checked before any device pointer is
 * touched); GMRES_ERR_ARG for invalid arguments, a malformed matrix or a
 * stream of another device; otherwise as gmres_solve. Blocks until done.
 * All calls on one GPU share its scratch array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on
 * one GPU, from several threads or streams, race and must not be made.
 */
#define GMRES_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gmres_solve_noalloc(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                        const double* vals, int32_t m, int32_t scheme, const double* b, double* x,
                        double rtol, int64_t max_iters, gmres_info* info, double* hist_res,
                        void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GMRES_H */

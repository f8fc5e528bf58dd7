// Internal declarations shared by the HIP kernels and the host driver of the
// GMRES library. Not part of the public C ABI (include/gmres.h).
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

namespace gmres {

#ifndef GMRES_GROUP
#define GMRES_GROUP 32
#endif
constexpr int kGroup = GMRES_GROUP;  // tiles per first-level group of the grid reduction
constexpr int kMaxRestart = 256;     // GMRES_MAX_RESTART of the public header

constexpr int kSchemeMgs = 0;
constexpr int kSchemeMgs1r = 1;
constexpr int kSchemeCgs2 = 2;
constexpr int kSchemeIr32 = 3;  // one-reduce MGS cycles on an FP32 basis, FP64 refinement
constexpr int kSchemeIr16 = 4;  // the same on a bfloat16 basis (float32 arithmetic)
constexpr int kSchemeCgs2r3 = 5;   // classical Gram-Schmidt, two passes: 3 reductions per step
constexpr int kSchemeTwoSynch = 6; // two-synchronization classical Gram-Schmidt
// Basis element types of the step kernels.
enum BasisType { kBasisF64 = 0, kBasisF32 = 1, kBasisBf16 = 2 };

constexpr int kNonfinite = -3;
constexpr int kTeamStall = -2;  // a team's parts did not all arrive (GMRES_ERR_HIP)

// Tail selectors: what the last workgroup of a reduction does with the totals.
enum Tail {
  kTailLagged1r = 1,    // one-reduce MGS step
  kTailLaggedCgs2 = 2,  // CGS2 step, first reduction
  kTailCgs2Second = 3,  // CGS2 step, second reduction
  kTailBnorm = 4,       // ||b||, tolerance
  kTailFinalRes = 5,    // ||b - A x|| at exit
  kTailMgsBeta = 6,     // level-1 MGS restart norm
  kTailMgsH = 7,        // level-1 MGS coefficient h_{q,i}
  kTailMgsNorm = 8,     // level-1 MGS h_{i+1,i}, Givens, flags
  kTailIrBeta = 9,      // FP32-basis cycle: ||r|| of the FP64 restart residual, check, scales
  kTailCgsPass1 = 10,   // re-orthogonalized CGS, first projection: coef = V^T w
  kTailTwoSynch = 11    // two-synchronization CGS: new row of L, coef = (I - L - L^T) y
};

// Per-solve state in device memory; the host reads it once per cycle.
struct DevState {
  int32_t done;       // the current cycle has ended: later launches return at once
  int32_t j;          // columns the cycle completed
  int32_t true_conv;  // the restart residual met the tolerance
  int32_t breakdown;  // exact breakdown, rho == 0
  int32_t status;     // 0 or kNonfinite
  int32_t bad_csr;    // set by the structure check
  int64_t reductions; // device-wide reductions completed
  int32_t rot_next;   // first Hessenberg column of the cycle not yet rotated
  int32_t pad_;
  double bnorm, tol_abs, beta, rho, inv_rho, gk;
  double tol_cycle;   // what |g_k| is compared with inside a cycle (tol_abs, or tol_abs / beta for IR)
  double xscale;      // x += xscale V y at the end of a cycle (1, or beta for IR)
};

struct Csr {
  const int* rp;
  const int* ci;
  const double* va;
  int64_t n;
  int64_t nnz;
};

// Sliced ELL copy of A owned by the library (SELL-64): slice s holds rows
// 64 s .. 64 s + 63; entry j of row 64 s + l is at sp[s] + 64 j + l, for
// j < W_s = (sp[s+1] - sp[s]) / 64 (at least 1). Padding entries hold value 0.
// Column indices are either int32 (ci; padding holds the row's own index, 0
// for rows past n) or, when every slice column's col - row values span less
// than 2^16, 16-bit deltas (cd): the column of entry j of row r in slice s is
// min(r + cbase[sp[s] / 64 + j] + cd[...], n - 1) taken as unsigned, so a
// padding entry (delta 0) can never leave [0, n).
// How a slice's column indices are stored.
enum SliceForm {
  kSfI32 = 0,   // an int32 column index per entry
  kSfD16 = 1,   // per slice column a base, per entry a 16-bit delta: col = row + base + delta
  kSfDiag = 2   // per slice column one diagonal d and no per-entry index: col = row + d
};
struct Sell {
  const int64_t* sp;  // ns + 1 slice offsets (entries)
  int* ci;            // int32 column indices (kSfI32), else null
  double* va;         // float64 values (the FP64 schemes) ...
  float* vaf;         // ... or float32 values (the FP32-basis scheme)
  int64_t ns;         // slices, ceil(n / 64)
  int64_t n;          // rows (below 2^28: gathers take 32-bit byte offsets)
  uint16_t* cd;       // 16-bit column deltas (kSfD16), else null
  int* cbase;         // per slice column: the smallest col - row of its entries (kSfD16), or
                      // its diagonal (kSfDiag)
  int sf;             // SliceForm
};
constexpr int kSellDeltaSpan = 65535;  // largest col - row spread a slice column may have for cd
constexpr int kSellMaxWidth = 4096;    // widest slice of a sliced copy
constexpr int64_t kSellMaxRows = (int64_t)1 << 28;  // gathers use 32-bit byte offsets

// Views into the caller's workspace.
struct Ws {
  double* V;         // n x (m+2), column-major, leading dimension ldv (FP64 schemes)
  double* w;         // ldv: SpMV output of the current step (FP64 schemes)
  float* Vf;         // the same two in float32 (the FP32-basis scheme)
  float* wf;
  double* r64;       // ldv: the FP64 restart residual (the FP32-basis scheme)
  double* H;         // (m+1) x m unrotated Hessenberg matrix, ld = ldh
  double* R;         // (m+1) x m Givens-rotated copy
  double* T;         // (m+2) x (m+2): Malard-Paige T (one-reduce) or L (CGS2), column-major, ld = ldt
  double* TT;        // the same matrix row-major (rows contiguous), ld = ldt
  double* g;         // m+2 rotated right-hand side
  double* gh;        // m+2: gh[k] = |g_k| as it stood right after rotation k-1
  double* cs;        // m+1 rotation cosines
  double* sn;        // m+1 rotation sines
  double* coef;      // m+2 MAXPY coefficients of the current step
  double* coef2;     // m+2 second-pass coefficients (CGS2)
  double* lvec;      // m+2: l = V[:,0:k]^T v_k of the current lagged step (for the new T column)
  double* y;         // m+2 least-squares solution
  double* partials;  // G x pstride tile sums
  double* gpartials; // ceil(G / kGroup) x pstride group sums
  unsigned* counters;// ceil(G / kGroup) + 1 tickets
  DevState* st;
  int64_t n;
  int64_t ldv;
  int ldh, ldt, pstride, m;
  int keep;          // the projection loads columns 0..keep-1 through the caches, the others
                     // non-temporal (those the next MAXPY reads first stay in the last-level cache)
};

// One system of a batch: rows [r0, r0 + n) of the block-diagonal matrix and
// of the concatenated vectors, and its basis at voff (leading dimension ldv)
// in the batch's basis array.
struct BatchSys {
  int64_t r0, n, voff, ldv;
};

// One entry of the work queue: part `part` of `nparts` of system `sys`. A
// system's parts are consecutive in the queue; part p owns its rows
// [p c, min(n, (p+1) c)) with c = the part size rounded up to 64 rows. Each
// entry has its own slot (its queue position) for the small workspace, the
// state record and two rows of reduction partials; `base` is the slot of
// part 0.
struct BatchTicket {
  int32_t sys, part, nparts, base;
};

// Per-system result of a batched solve (the layout of gmres_batch_info).
struct BatchOut {
  int64_t iters;
  int32_t cycles, converged, status, breakdown;
  double rel_res_true;
};

// Everything the persistent batched kernel needs.
struct Batch {
  Csr A;                     // block-diagonal CSR over all systems (global column indices)
  const BatchSys* sys;       // nsys records
  const BatchTicket* tickets;// ntickets queue entries
  int nsys, ntickets, m;
  void* Vb;                  // bases (float64, or float32 for the FP32-basis scheme)
  void* wb;                  // SpMV outputs, by global row (same type)
  double* r64;               // float64 restart residuals by global row (FP32-basis only)
  double* small;             // small workspaces, batch_small_doubles(m) per slot
  DevState* st;              // one state per slot
  double* partials;          // 2 rows of 2 (m + 2) doubles per slot
  unsigned* bar;             // nsys team barrier counters
  unsigned* queue;           // next queue position
  BatchOut* out;             // nsys results
  const double* b;
  double* x;
  double rtol;
  int64_t max_iters;
  uint32_t spin_limit;       // polls of a team barrier before the team gives up
  Sell S;                    // the copy of A by diagonals (S.va null: the SpMV reads the CSR arrays)
};

// Doubles of one system's small workspace: H and R ((m+1) m each), T and TT
// ((m+2)^2 each), g, gh, cs, sn, coef, coef2, y ((m+2) each).
constexpr size_t batch_small_doubles(int m) {
  return 2 * (size_t)(m + 1) * m + 2 * (size_t)(m + 2) * (m + 2) + 7 * (size_t)(m + 2);
}

// Sets st->bad_csr when a row of system i has a column outside its rows (the
// CSR arrays must already have passed launch_validate).
int launch_batch_validate(const Csr& A, const BatchSys* sys, int nsys, DevState* st, hipStream_t s);
// Clears the queue position, the team barrier counters and every system's
// result (a kernel, so a captured graph holds no memset node).
int launch_batch_reset(const Batch& B, hipStream_t s);
// The persistent solve: grid workgroups of bs threads (256, 512 or 1024)
// take queue entries until the queue is empty. f32: float32 basis; nt: the
// basis columns are loaded non-temporal. A system split into several parts
// needs all of them running at once: the caller keeps every nparts within
// what the GPU holds concurrently.
int launch_batch(const Batch& B, int bs, int grid, bool f32, bool nt, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Workgroups of that k_batch form that one compute unit holds at once (0 on error).
int batch_resident_blocks(int bs, int m, bool f32, bool nt);
size_t batch_lds_bytes(int bs, int m);

int launch_init(const Ws& ws, int ncounters, hipStream_t s);
int launch_solve_begin(const Ws& ws, hipStream_t s);
int launch_cycle_begin(const Ws& ws, hipStream_t s);
int launch_validate(const Csr& A, int64_t nnz, DevState* st, hipStream_t s);
// SpMV shape code: 100 * (lanes per row) + (entries per lane).
int launch_spmv(const Csr& A, int shape, const double* x, const double* b, double* y,
                const DevState* st, hipStream_t s, hipEvent_t e0 = nullptr,
                hipEvent_t e1 = nullptr);
// Where the fused step kernel takes w from.
enum WSource {
  kWNone = 0,  // w = 0: only the sums over u
  kWSpmv = 1,  // w = A u computed in the kernel from the CSR arrays
  kWLoad = 2,  // w read from ws.w, written by a separate SpMV launch
  kWSell = 3,  // w = A u computed in the kernel from the sliced ELL copy (int32 indices)
  kWSellD16 = 4,  // the same from the sliced copy with 16-bit column deltas
  kWSellDiag = 5  // the same from the sliced copy stored by diagonals
};
// Sliced ELL construction: slice widths, then (with sp filled in) the copy;
// rows longer than their slice's width set st->bad_csr.
// width[s] = max(1, longest row of slice s); *spread (device, nullable, set
// to 0 beforehand) = the largest col - row spread over the slice columns of
// slices at most max_width wide (INT_MAX when a slice is wider).
int launch_sell_width(const Csr& A, int64_t ns, int* width, int* spread, int max_width,
                      hipStream_t s);
// width[s] = max(1, the number of distinct col - row values (diagonals) among
// slice s's entries); *flag (device, set to 0 beforehand) gets bit 0 when a
// row's columns are not strictly increasing and bit 1 when a slice has more
// than max_width diagonals (its count is then not finished).
int launch_sell_diags(const Csr& A, int64_t ns, int* width, int* flag, int max_width,
                      hipStream_t s);
int launch_sell_fill(const Csr& A, const Sell& S, DevState* st, hipStream_t s);
int launch_spmv_sell(const Sell& S, int64_t n, const double* x, const double* b, double* y,
                     const DevState* st, hipStream_t s, hipEvent_t e0 = nullptr,
                     hipEvent_t e1 = nullptr);
// f32: the FP32-basis variant (ws.Vf, ws.wf; float32 values in the sliced copy).
int launch_fused(const Csr& A, const Sell& SA, int shape, const Ws& ws, int rpt, int K, int nproj,
                 int wsrc, int m_eff, int tail, int G, int bt, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// side: 0, or (mode 0 of a lagged step) kSchemeMgs1r / kSchemeCgs2, which adds
// one workgroup for the new T column (L row), the Givens rotations and the
// stopping test, the rotations applied once `depth` columns are pending.
int launch_maxpy(const Ws& ws, int rpt, int k, int mode, int G, int bt, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, int side = 0, int depth = 1);
int launch_axpy_dot(const Ws& ws, int rpt, double* w, const double* a, const double* coef,
                    const double* v, int tail, int i_col, int q_row, int m_eff, double aux, int G,
                    hipStream_t s);
int launch_scale(const Ws& ws, double* v, hipStream_t s);
int launch_cycle_end(const Ws& ws, int rpt, double* x, int G, int bt, hipStream_t s);
// FP32-basis cycle start: Vf[:,0] = float(r64 * inv_rho).
int launch_first_vector(const Ws& ws, int bt, hipStream_t s);
size_t fused_lds_bytes(int rpt, int m);

}  // namespace gmres

// Host driver and C ABI of the GMRES library (include/gmres.h).
//
// Restarted GMRES(m) after Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low
// synchronization GMRES algorithms" (arXiv:1809.05805). Each restart cycle is
// enqueued as a whole: every step's kernels read a "done" flag that the
// device sets when the cycle ends (converged, flushed, broke down or failed),
// so later launches of the cycle return at once and the host waits on the
// stream only once per cycle, to read a few scalars and the small matrices.
#include "gmres.h"
#include "gmres_internal.h"

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

using namespace gmres;

static_assert(kMaxRestart == GMRES_MAX_RESTART, "kernel LDS sizes follow the public restart cap");

namespace {

constexpr size_t kAlign = 256;

constexpr size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

//   GMRES_LLC_KEEP_MIB  bytes of basis columns (MiB) the projection keeps in
//   the last-level cache for the next MAXPY: three quarters of the MI355X's
//   256 MB (at 128^3 in float64, 12 columns: 85.9 ms per solve against 86.0
//   for 8 columns, 86.4 for 16 and 88.1 with every column cached).
#ifndef GMRES_LLC_KEEP_MIB
#define GMRES_LLC_KEEP_MIB 192
#endif
constexpr double kKeepBytes = GMRES_LLC_KEEP_MIB * 1048576.0;

// Rows per lane of the row-tiled kernels: the largest of 8, 4, 2 that still
// leaves at least 512 tiles of 256*rpt rows (two per compute unit), else 1;
// or the caller's choice (gmres_options.rows_per_lane).
int pick_rpt(int64_t n, int want) {
  if (want == 1 || want == 2 || want == 4 || want == 8) return want;
  for (int r : {8, 4, 2})
    if ((n + 256 * r - 1) / (256 * r) >= 512) return r;
  return 1;
}

// Tiles of 256*rpt rows, padded to a multiple of 8 (one per XCD) when there
// are at least 8, so the XCD-aware tile mapping is a bijection.
int pick_grid(int64_t n, int rpt) {
  int64_t tiles = (n + 256 * rpt - 1) / (256 * rpt);
  if (tiles >= 8) tiles = (tiles + 7) / 8 * 8;
  return (int)tiles;
}

// CSR SpMV shape (100 * lanes per row + entries per lane) from the mean row
// length: the fewest lanes per row whose entry slots cover it. One thread per
// row for up to 8 entries; 8 lanes of 4 entries for 27-point rows. Or the
// caller's choice (gmres_options.csr_spmv_shape).
bool valid_shape(int v) {
  return v == 108 || v == 208 || v == 408 || v == 804 || v == 808 || v == 6401;
}
int pick_spmv_shape(int64_t n, int64_t nnz, int want) {
  if (valid_shape(want)) return want;
  const int64_t avg = (nnz + n - 1) / n;
  if (avg <= 8) return 108;
  if (avg <= 16) return 208;
  if (avg <= 32) return 804;
  if (avg <= 64) return 808;
  return 6401;
}

// Sparse format of the SpMV. The sliced ELL copy (SELL-64, built at create)
// makes every column-index and value load of a wavefront one contiguous
// 512-byte block and needs no row pointers. By default it is stored by
// diagonals when every row's columns are strictly increasing and giving each
// slice a column per distinct diagonal (col - row value) among its rows costs
// at most a quarter more entries than nnz (stencils): then no column index is
// stored at all, only one diagonal per slice column. Otherwise it is used when
// padding every slice to its longest row costs at most a quarter more
// entries, with column indices as 16-bit deltas from a per-slice-column base
// (2 bytes per entry instead of 4) when every slice column's col - row values
// span at most kSellDeltaSpan (banded matrices), else int32. In every case no
// slice may be wider than kSellMaxWidth and n < kSellMaxRows.
// gmres_options.format forces CSR, the copy with int32 indices, the copy with
// deltas where they fit, or the copy by diagonals where the rows are sorted
// (else with deltas where they fit), whatever the padding (the width and row
// limits still hold).
enum { kFormatCsr = 0, kFormatSell = 1 };

// The caller's options, checked; zero fields take the library's choices.
bool check_options(const gmres_options* o, int scheme) {
  if (!o) return true;
  if (o->format < GMRES_OPT_FORMAT_AUTO || o->format > GMRES_OPT_FORMAT_SELL64_DIAG) return false;
  if (o->rows_per_lane != 0 && o->rows_per_lane != 1 && o->rows_per_lane != 2 &&
      o->rows_per_lane != 4 && o->rows_per_lane != 8)
    return false;
  if (o->csr_spmv_shape != 0 && !valid_shape(o->csr_spmv_shape)) return false;
  if (o->split_spmv != 0 && o->split_spmv != 1) return false;
  if (o->pipeline_depth < 0 || o->pipeline_depth > GMRES_MAX_RESTART) return false;
  const bool lagged = scheme == GMRES_MGS_1R || scheme == GMRES_CGS2 ||
                      scheme == GMRES_MGS_1R_IR32 || scheme == GMRES_MGS_1R_IR16;
  if (o->pipeline_depth > 1 && !lagged) return false;
  for (int r : o->reserved)
    if (r != 0) return false;
  return true;
}

// The refinement schemes: one-reduce cycles on a reduced-precision basis
// (float32 or bfloat16) inside float64 refinement.
bool ir_scheme(int scheme) { return scheme == kSchemeIr32 || scheme == kSchemeIr16; }
int basis_type(int scheme) {
  return scheme == kSchemeIr32 ? kBasisF32 : scheme == kSchemeIr16 ? kBasisBf16 : kBasisF64;
}
size_t basis_bytes(int scheme) {
  return scheme == kSchemeIr32 ? sizeof(float) : scheme == kSchemeIr16 ? 2 : sizeof(double);
}

// The block the host reads back after a cycle, one copy: the device state,
// then g and gh ((m+2) each), then H ((m+1) m) and T ((m+2)^2), each part
// 64-byte aligned. The host mirror has the same layout.
struct Readback {
  size_t g, gh, H, T, total;
};
constexpr Readback readback_layout(int m) {
  const size_t v = round_up((size_t)(m + 2) * sizeof(double), 64);
  const size_t g = round_up(sizeof(DevState), 64);
  const size_t H = g + 2 * v;
  const size_t T = H + round_up((size_t)(m + 1) * (size_t)m * sizeof(double), 64);
  return Readback{g, g + v, H, T, T + round_up((size_t)(m + 2) * (size_t)(m + 2) * sizeof(double), 64)};
}

struct Layout {
  int64_t ldv;
  int rpt, G, NG, pstride;
  size_t V, w, r64, H, R, T, TT, g, gh, cs, sn, coef, coef2, lvec, y, partials, gpartials,
      counters, state, total;
};

// The FP64 schemes keep the basis V and the SpMV output w in float64; the
// refinement schemes keep them in float32 or bfloat16 plus a float64 restart
// residual. Columns are 64 elements apart at least, so every column starts
// 128-byte aligned (256 bytes for float32 and float64). A stride that is a
// multiple of 1024 elements (n = 2^21 at 128^3) gets 17 x 64 elements more:
// the kernels read many columns at the same row offset at once, and with a
// large power-of-two stride those reads differ only in high address bits
// (the 128^3 solve: 83.0 against 81.8 ms, MAXPY 70.2 against 68.4 us).
bool make_layout(int64_t n, int m, int scheme, Layout* L, int rpt_want = 0) {
  if (n < 1 || m < 1 || m > GMRES_MAX_RESTART) return false;
  L->ldv = (int64_t)round_up((size_t)n, 64);
  if (L->ldv % 1024 == 0) L->ldv += 17 * 64;
  L->rpt = pick_rpt(n, rpt_want);
  L->G = pick_grid(n, L->rpt);
  L->NG = (L->G + kGroup - 1) / kGroup;
  L->pstride = (int)round_up((size_t)(2 * (m + 2)), 32);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = round_up(off + bytes, kAlign);
    return at;
  };
  const size_t d = sizeof(double);
  const size_t vb = basis_bytes(scheme);
  L->V = take((size_t)L->ldv * (size_t)(m + 2) * vb);
  L->w = take((size_t)L->ldv * vb);
  L->r64 = ir_scheme(scheme) ? take((size_t)L->ldv * d) : 0;
  const Readback rb = readback_layout(m);
  L->state = take(rb.total);
  L->g = L->state + rb.g;
  L->gh = L->state + rb.gh;
  L->H = L->state + rb.H;
  L->T = L->state + rb.T;
  L->R = take((size_t)(m + 1) * (size_t)m * d);
  L->TT = take((size_t)(m + 2) * (size_t)(m + 2) * d);
  L->cs = take((size_t)(m + 2) * d);
  L->sn = take((size_t)(m + 2) * d);
  L->coef = take((size_t)(m + 2) * d);
  L->coef2 = take((size_t)(m + 2) * d);
  L->lvec = take((size_t)(m + 2) * d);
  L->y = take((size_t)(m + 2) * d);
  L->partials = take((size_t)L->G * (size_t)L->pstride * d);
  L->gpartials = take((size_t)L->NG * (size_t)L->pstride * d);
  L->counters = take((size_t)(L->NG + 1) * sizeof(unsigned));
  L->total = off;
  return true;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

// Device workspace of gmres_solve_noalloc: one solve's workspace at a time per
// GPU, in the library's own code object, so that the call allocates nothing.
// Host code must not pass `scratch` itself to a kernel (in host code it names
// a host-side stand-in); it uses the device address that scratch_on() looks
// up, once per device, with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[GMRES_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];  // per device; null until looked up

// Device address of scratch on device dev, which must be the current device.
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

}  // namespace

struct gmres_ctx {
  Csr A;
  int64_t nnz;
  int m, scheme, S;  // S: SpMV shape code
  bool split;        // separate SpMV launch in the lagged step
  int depth;         // pipeline depth of the rotations (lagged schemes; 1 otherwise)
  int format_want;   // gmres_options.format
  bool matrix_ok;    // false after a refresh found a bad structure: no more SpMVs
  int format;        // kFormatCsr or kFormatSell
  Sell sell;         // the sliced copy (format == kFormatSell), in caller memory
  std::vector<int64_t> sell_sp;  // planned slice offsets (empty: no copy planned)
  int64_t sell_entries;          // planned stored entries
  int sell_sf;                   // the planned copy's SliceForm
  size_t sell_bytes, o_ci, o_va; // planned storage size and its layout (o_ci: indices or deltas)
  size_t o_cb;                   // per-slice-column bases or diagonals (kSfD16, kSfDiag)
  size_t o_va64;                 // the float64 values (after the float32 ones for the refinement schemes)
  Layout L;
  Ws ws;
  hipStream_t stream;
  // host mirror of the device state: DevState, g, gh, and (when
  // mirror_matrices) H and T; pinned memory of the context's own, or the
  // caller's stack for gmres_solve_noalloc
  void* pinned;
  bool mirror_matrices;
  DevState* h_st;
  double* h_g;
  double* h_gh;
  double* h_H;
  double* h_T;
  // host snapshot of the last cycle that completed a column
  std::vector<double> last_H, last_T, last_g;
  int last_j;
  // per-launch event timing (measurement only)
  bool timing;
  std::vector<hipEvent_t> ev;  // pairs: start, stop
  struct Rec {
    int cls;      // GMRES_KSTAT_*
    int step;     // Arnoldi step k of the launch
    int runs_to;  // the launch ran iff the cycle's j >= runs_to
    double bytes;
  };
  std::vector<Rec> recs;
  gmres_kernel_stat stats[GMRES_KSTAT_COUNT];
};

namespace {

int sync_state(gmres_ctx* c, bool with_matrices) {
  // one copy of the readback block: the state, with g and gh after a cycle,
  // and H and T too when the context mirrors them
  const Readback rb = readback_layout(c->m);
  const size_t bytes =
      with_matrices ? (c->mirror_matrices ? rb.total : rb.H) : sizeof(DevState);
  if (hipMemcpyAsync(c->h_st, c->ws.st, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GMRES_ERR_HIP;
  return GMRES_OK;
}

#define TRY(x)                  \
  do {                          \
    int _rc = (x);              \
    if (_rc) return GMRES_ERR_HIP; \
  } while (0)

// Start/stop events attached to one launch when timing is on (null otherwise).
struct TimedLaunch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedLaunch(gmres_ctx* c, int cls, int step, int runs_to, double bytes) {
    if (!c->timing) return;
    const size_t slot = c->recs.size();
    if (2 * slot + 2 > c->ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        c->timing = false;
        return;
      }
      c->ev.push_back(a);
      c->ev.push_back(b);
    }
    c->recs.push_back({cls, step, runs_to, bytes});
    e0 = c->ev[2 * slot];
    e1 = c->ev[2 * slot + 1];
  }
};

// Largest singular value of the K x K matrix S (column-major, leading
// dimension ld) by power iteration on S^T S, started from x (length K, left
// holding the final iterate so that the next, larger block can start from it).
double spectral_norm(const double* S, int K, int ld, std::vector<double>& x) {
  std::vector<double> y((size_t)K), z((size_t)K);
  double nx = 0.0;
  for (int i = 0; i < K; ++i) nx += x[i] * x[i];
  if (!(nx > 0.0)) {
    for (int i = 0; i < K; ++i) x[i] = 1.0;
    nx = K;
  }
  for (int i = 0; i < K; ++i) x[i] /= sqrt(nx);
  double lam = 0.0;
  for (int iter = 0; iter < 5000; ++iter) {
    for (int i = 0; i < K; ++i) y[i] = 0.0;
    for (int col = 0; col < K; ++col)
      for (int i = 0; i < K; ++i) y[i] += S[(size_t)col * ld + i] * x[col];
    for (int col = 0; col < K; ++col) {
      double a = 0.0;
      for (int i = 0; i < K; ++i) a += S[(size_t)col * ld + i] * y[i];
      z[col] = a;
    }
    double nz = 0.0;
    for (int i = 0; i < K; ++i) nz += z[i] * z[i];
    nz = sqrt(nz);
    if (nz == 0.0) return 0.0;
    for (int i = 0; i < K; ++i) x[i] = z[i] / nz;
    const bool done = fabs(nz - lam) <= 1e-14 * nz;
    lam = nz;
    if (done) break;
  }
  return sqrt(lam);
}

// ||S||_2 with S = I - (I + L^T)^{-1} (Paige's S for the basis v_0..v_K-1),
// for the leading K x K blocks, K = 1..j, of the cycle that just ended:
// one-reduce MGS holds T = (I + L^T)^{-1} itself, CGS2 and the
// two-synchronization CGS hold L (its rows are the projections l of the newest
// column); plain MGS and the three-reduction CGS form neither, so their
// entries are NaN.
void orth_history(const gmres_ctx* c, int j, const double* Tm, double* out) {
  if (c->scheme == kSchemeMgs || c->scheme == kSchemeCgs2r3) {
    for (int q = 0; q < j; ++q) out[q] = NAN;
    return;
  }
  const int ldt = c->m + 2;
  std::vector<double> S((size_t)j * j, 0.0);  // column-major, ld j
  if (c->scheme != kSchemeCgs2 && c->scheme != kSchemeTwoSynch) {
    for (int col = 0; col < j; ++col)
      for (int i = 0; i < col; ++i) S[(size_t)col * j + i] = -Tm[(size_t)col * ldt + i];
  } else {
    // U = (I + L^T)^{-1}, unit upper triangular: column col solves
    // (I + L^T) u = e_col by back substitution; L(t, i) sits at h_T[i * ldt + t]
    for (int col = 0; col < j; ++col) {
      std::vector<double> u((size_t)col + 1, 0.0);
      u[col] = 1.0;
      for (int i = col - 1; i >= 0; --i) {
        double a = 0.0;
        for (int t = i + 1; t <= col; ++t) a += Tm[(size_t)i * ldt + t] * u[t];
        u[i] = -a;
      }
      for (int i = 0; i < col; ++i) S[(size_t)col * j + i] = -u[i];
    }
  }
  std::vector<double> x((size_t)j, 0.0);
  out[0] = 0.0;
  for (int K = 2; K <= j; ++K) {
    x[K - 1] = 1.0 / sqrt((double)K);
    out[K - 1] = spectral_norm(S.data(), K, j, x);
  }
}

// After the cycle has finished on the stream: add the launches that ran.
void collect_timing(gmres_ctx* c, int j, bool stopped_at_restart) {
  if (!c->timing) return;
  for (size_t i = 0; i < c->recs.size(); ++i) {
    const auto& r = c->recs[i];
    const bool ran = stopped_at_restart ? (r.step == 0 && r.runs_to == 0 &&
                                           (r.cls == GMRES_KSTAT_STEP || r.cls == GMRES_KSTAT_SPMV))
                                        : j >= r.runs_to;
    if (!ran) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) continue;
    c->stats[r.cls].ms += ms;
    c->stats[r.cls].bytes += r.bytes;
    c->stats[r.cls].launches += 1;
  }
  c->recs.clear();
}

// Plan the sliced copy of A when the format choice asks for it: slice widths
// on the device (in the basis region of the workspace, which holds nothing
// before the first solve), offsets on the host. The copy itself is built by
// gmres_set_matrix_storage in memory the caller provides; until then, or if
// no copy is planned, the SpMV reads the CSR arrays.
int plan_format(gmres_ctx* c) {
  c->format = kFormatCsr;
  c->sell = Sell{};
  c->sell_sp.clear();
  c->sell_entries = 0;
  c->sell_sf = kSfI32;
  c->sell_bytes = 0;
  const int want = c->format_want;
  if (want == GMRES_OPT_FORMAT_CSR || c->nnz == 0 || c->A.n >= kSellMaxRows) return GMRES_OK;
  const int64_t ns = (c->A.n + 63) / 64;
  // 2 (ns + 1) ints fit easily in the basis region (n (m+2) doubles, or floats,
  // n rounded up to 64)
  int* dw = ir_scheme(c->scheme) ? reinterpret_cast<int*>(c->ws.Vf)
                                 : reinterpret_cast<int*>(c->ws.V);
  int* dd = dw + ns + 1;
  std::vector<int> wh((size_t)ns + 1), dh((size_t)ns + 1);
  const bool deltas = want != GMRES_OPT_FORMAT_SELL64;
  const bool diags = want == GMRES_OPT_FORMAT_AUTO || want == GMRES_OPT_FORMAT_SELL64_DIAG;
  if (hipMemsetAsync(dw + ns, 0, sizeof(int), c->stream) != hipSuccess ||
      hipMemsetAsync(dd + ns, 0, sizeof(int), c->stream) != hipSuccess ||
      launch_sell_width(c->A, ns, dw, deltas ? dw + ns : nullptr, kSellMaxWidth, c->stream) ||
      (diags && launch_sell_diags(c->A, ns, dd, dd + ns, kSellMaxWidth, c->stream)) ||
      hipMemcpyAsync(wh.data(), dw, sizeof(int) * (size_t)(ns + 1), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(dh.data(), dd, sizeof(int) * (size_t)(ns + 1), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GMRES_ERR_HIP;
  // slice offsets from slice widths; false if a slice is too wide
  auto offsets = [&](const std::vector<int>& w, std::vector<int64_t>& sp) {
    sp.assign((size_t)ns + 1, 0);
    bool fits = true;
    for (int64_t i = 0; i < ns; ++i) {
      sp[i + 1] = sp[i] + 64 * (int64_t)w[i];
      fits = fits && w[i] <= kSellMaxWidth;
    }
    return fits;
  };
  auto cheap = [&](int64_t total) { return total * 4 <= c->nnz * 5; };
  std::vector<int64_t> sp, dsp;
  const bool ell = offsets(wh, sp);
  const bool diag = diags && dh[ns] == 0 && offsets(dh, dsp);
  if (diag && (want != GMRES_OPT_FORMAT_AUTO || cheap(dsp[ns]))) {
    c->sell_sf = kSfDiag;
    c->sell_sp.swap(dsp);
  } else if (ell && (want != GMRES_OPT_FORMAT_AUTO || cheap(sp[ns]))) {
    c->sell_sf = deltas && wh[ns] <= kSellDeltaSpan ? kSfD16 : kSfI32;
    c->sell_sp.swap(sp);
  } else {
    return GMRES_OK;
  }
  const int64_t total = c->sell_sp[ns];
  c->sell_entries = total;
  const size_t vsize = ir_scheme(c->scheme) ? sizeof(float) : sizeof(double);
  const size_t off_sp = round_up(sizeof(int64_t) * (size_t)(ns + 1), kAlign);
  if (c->sell_sf == kSfDiag) {
    c->o_cb = off_sp;
    c->o_ci = 0;
    c->o_va = round_up(c->o_cb + sizeof(int) * (size_t)(total / 64), kAlign);
  } else if (c->sell_sf == kSfD16) {
    c->o_cb = off_sp;
    c->o_ci = round_up(c->o_cb + sizeof(int) * (size_t)(total / 64), kAlign);
    c->o_va = round_up(c->o_ci + sizeof(uint16_t) * (size_t)total, kAlign);
  } else {
    c->o_cb = 0;
    c->o_ci = off_sp;
    c->o_va = round_up(c->o_ci + sizeof(int) * (size_t)total, kAlign);
  }
  // the refinement schemes keep float64 values too, for the float64 restart residual
  c->o_va64 = ir_scheme(c->scheme) ? round_up(c->o_va + vsize * (size_t)total, kAlign) : c->o_va;
  c->sell_bytes = c->o_va64 + sizeof(double) * (size_t)total;
  return GMRES_OK;
}

// Fill the copy's values (both value arrays for the refinement schemes) and
// column part; a row that does not fit sets st->bad_csr.
int fill_copy(gmres_ctx* c, const Sell& S) {
  if (S.vaf) {
    Sell Sf = S;
    Sf.va = nullptr;
    if (launch_sell_fill(c->A, Sf, c->ws.st, c->stream)) return 1;
  }
  if (S.va) {
    Sell Sd = S;
    Sd.vaf = nullptr;
    if (launch_sell_fill(c->A, Sd, c->ws.st, c->stream)) return 1;
  }
  return 0;
}

// y = A x or y = b - A x in float64: from the sliced copy's float64 values
// (every scheme's copy has them; the refinement schemes' also has float32
// ones for their inner cycles), else from the CSR arrays.
int spmv(gmres_ctx* c, const double* x, const double* b, double* y, const DevState* st,
         hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (c->format == kFormatSell && c->sell.va)
    return launch_spmv_sell(c->sell, c->A.n, x, b, y, st, s, e0, e1);
  return launch_spmv(c->A, c->S, x, b, y, st, s, e0, e1);
}

// Enqueue one restart cycle with m_eff >= 1 columns at most.
int enqueue_cycle(gmres_ctx* c, const double* b, double* x, int m_eff) {
  const Ws& ws = c->ws;
  hipStream_t s = c->stream;
  const int rpt = c->L.rpt, G = c->L.G;
  const bool ir = ir_scheme(c->scheme);  // a reduced-precision basis inside float64 refinement
  const int bt = basis_type(c->scheme);
  const double n8 = (double)basis_bytes(c->scheme) * (double)c->A.n;  // one basis column
  // Algorithmic bytes of the timed launches (the method's model, whatever the
  // format in use): the CSR arrays with int32 indices and float64 values
  // (float32 values for the refinement schemes), one basis column n8.
  const double csr = (ir ? 8.0 : 12.0) * (double)c->nnz + 4.0 * (double)(c->A.n + 1);
  auto col = [&](int q) { return ws.V + (size_t)q * (size_t)ws.ldv; };
  TRY(launch_cycle_begin(ws, s));
  if (ir) {
    // float64 restart residual and its norm (the restart check), then the
    // cycle's first basis vector r / ||r|| in float32
    TRY(spmv(c, x, b, ws.r64, nullptr, s));
    TRY(launch_axpy_dot(ws, rpt, ws.r64, nullptr, nullptr, ws.r64, kTailIrBeta, 0, 0, m_eff, 0.0,
                        G, s));
    TRY(launch_first_vector(ws, bt, s));
  } else {
    TRY(spmv(c, x, b, col(0), nullptr, s));  // V[:,0] = b - A x
  }
  if (c->scheme == kSchemeMgs || c->scheme == kSchemeCgs2r3 || c->scheme == kSchemeTwoSynch) {
    // normalized basis: the restart norm first, then per step the
    // orthogonalization of w = A v_i and a separate norm reduction
    TRY(launch_axpy_dot(ws, rpt, col(0), nullptr, nullptr, col(0), kTailMgsBeta, 0, 0, m_eff, 0.0,
                        G, s));
    TRY(launch_scale(ws, col(0), s));
    for (int i = 0; i < m_eff; ++i) {
      double* w = col(i + 1);
      if (c->scheme == kSchemeMgs) {
        TRY(spmv(c, col(i), nullptr, w, ws.st, s));
        for (int q = 0; q <= i; ++q) {
          const double* a = q > 0 ? col(q - 1) : nullptr;
          const double* cf = q > 0 ? ws.H + (size_t)i * ws.ldh + (q - 1) : nullptr;
          TRY(launch_axpy_dot(ws, rpt, w, a, cf, col(q), kTailMgsH, i, q, m_eff, 0.0, G, s));
        }
        TRY(launch_axpy_dot(ws, rpt, w, col(i), ws.H + (size_t)i * ws.ldh + i, w, kTailMgsNorm, i, 0,
                            m_eff, 0.0, G, s));
      } else if (c->scheme == kSchemeCgs2r3) {
        // two classical passes: coef = V^T w, w -= V coef; coef2 = V^T w,
        // w -= V coef2, H[:,i] = coef + coef2; then ||w||
        TRY(spmv(c, col(i), nullptr, w, ws.st, s));
        TRY(launch_fused(c->A, c->sell, c->S, ws, rpt, i + 1, i + 1, kWNone, m_eff, kTailCgsPass1, G,
                         kBasisF64, s, nullptr, nullptr));
        TRY(launch_maxpy(ws, rpt, i, 2, G, kBasisF64, s, nullptr, nullptr));
        TRY(launch_fused(c->A, c->sell, c->S, ws, rpt, i + 1, i + 1, kWNone, m_eff, kTailCgs2Second, G,
                         kBasisF64, s, nullptr, nullptr));
        TRY(launch_maxpy(ws, rpt, i, 1, G, kBasisF64, s, nullptr, nullptr));
        TRY(launch_axpy_dot(ws, rpt, w, nullptr, nullptr, w, kTailMgsNorm, i, 0, m_eff, 0.0, G, s));
      } else {
        // one reduction for [V^T w, V[:,0:i]^T v_i], coef = (I - L - L^T) y,
        // w = A v_i - V coef; then ||w||
        TRY(spmv(c, col(i), nullptr, ws.w, ws.st, s));
        TRY(launch_fused(c->A, c->sell, c->S, ws, rpt, i, i, kWLoad, m_eff, kTailTwoSynch, G,
                         kBasisF64, s, nullptr, nullptr));
        TRY(launch_maxpy(ws, rpt, i, 3, G, kBasisF64, s, nullptr, nullptr));
        TRY(launch_axpy_dot(ws, rpt, w, nullptr, nullptr, w, kTailMgsNorm, i, 0, m_eff, 0.0, G, s));
      }
      TRY(launch_scale(ws, w, s));
    }
  } else {
    const int tail = c->scheme == kSchemeCgs2 ? kTailLaggedCgs2 : kTailLagged1r;
    // Step k's fused kernel runs iff the cycle reaches step k (j >= k, or the
    // restart check at k = 0 ends it); the rest of step k runs iff j > k.
    for (int k = 0; k <= m_eff; ++k) {
      {
        // The last step of a cycle only finishes the lagged norm of column m_eff.
        const bool last = k == m_eff;
        int wsrc = last ? kWNone
                        : c->format == kFormatSell ? (c->sell.sf == kSfDiag  ? kWSellDiag
                                                      : c->sell.sf == kSfD16 ? kWSellD16
                                                                             : kWSell)
                                                   : kWSpmv;
        // A; u read and w written by the SpMV; V[:,0:k+1] (u included) read by the projection
        double bytes = last ? n8 : csr + 2 * n8 + n8 * (k + 1);
        if (!last && c->split && !ir) {
          TimedLaunch t(c, GMRES_KSTAT_SPMV, k, k, csr + 2 * n8);
          TRY(spmv(c, col(k), nullptr, ws.w, ws.st, s, t.e0, t.e1));
          wsrc = kWLoad;
          bytes = n8 * (k + 2);
        }
        TimedLaunch t(c, GMRES_KSTAT_STEP, k, k, bytes);
        TRY(launch_fused(c->A, c->sell, c->S, ws, rpt, k, last ? 0 : k, wsrc, m_eff, tail, G, bt, s,
                         t.e0, t.e1));
      }
      if (k == m_eff) break;
      {
        TimedLaunch t(c, GMRES_KSTAT_MAXPY, k, k + 1, n8 * (k + 1) + 2 * n8);
        TRY(launch_maxpy(ws, rpt, k, 0, G, bt, s, t.e0, t.e1,
                         c->scheme == kSchemeCgs2 ? kSchemeCgs2 : kSchemeMgs1r, c->depth));
      }
      if (c->scheme == kSchemeCgs2) {
        {
          TimedLaunch t(c, GMRES_KSTAT_STEP, k, k + 1, n8 * (k + 2));
          TRY(launch_fused(c->A, c->sell, c->S, ws, rpt, k + 1, k + 1, kWNone, m_eff, kTailCgs2Second, G,
                           kBasisF64, s, t.e0, t.e1));
        }
        TimedLaunch t(c, GMRES_KSTAT_MAXPY, k, k + 1, n8 * (k + 1) + 2 * n8);
        TRY(launch_maxpy(ws, rpt, k, 1, G, kBasisF64, s, t.e0, t.e1));
      }
    }
  }
  TRY(launch_cycle_end(ws, rpt, x, G, bt, s));
  return GMRES_OK;
}

// ||b - A x|| into the state's beta, without touching the basis.
int enqueue_true_residual(gmres_ctx* c, const double* b, const double* x) {
  const Ws& ws = c->ws;
  double* r = ir_scheme(c->scheme) ? ws.r64 : ws.w;
  TRY(launch_cycle_begin(ws, c->stream));
  TRY(spmv(c, x, b, r, nullptr, c->stream));
  TRY(launch_axpy_dot(ws, c->L.rpt, r, nullptr, nullptr, r, kTailFinalRes, 0, 0, 0, 0.0, c->L.G,
                      c->stream));
  return GMRES_OK;
}

// Point a context's fields at its matrix and workspace (no host mirror yet).
void bind_context(gmres_ctx* c, int64_t n, int64_t nnz, const int32_t* row_ptr,
                  const int32_t* col_idx, const double* vals, int m, int scheme, const Layout& L,
                  void* workspace, hipStream_t stream, const gmres_options* opt) {
  c->A = Csr{row_ptr, col_idx, vals, n, nnz};
  c->nnz = nnz;
  c->m = m;
  c->scheme = scheme;
  c->S = pick_spmv_shape(n, nnz, opt ? opt->csr_spmv_shape : 0);
  c->split = opt && opt->split_spmv == 1;
  c->depth = opt && opt->pipeline_depth > 1 ? opt->pipeline_depth : 1;
  c->format_want = opt ? opt->format : GMRES_OPT_FORMAT_AUTO;
  c->L = L;
  c->stream = stream;
  char* base = (char*)workspace;
  Ws& ws = c->ws;
  if (ir_scheme(scheme)) {
    ws.V = nullptr;
    ws.w = nullptr;
    ws.Vf = (float*)(base + L.V);
    ws.wf = (float*)(base + L.w);
    ws.r64 = (double*)(base + L.r64);
  } else {
    ws.V = (double*)(base + L.V);
    ws.w = (double*)(base + L.w);
    ws.Vf = nullptr;
    ws.wf = nullptr;
    ws.r64 = nullptr;
  }
  ws.H = (double*)(base + L.H);
  ws.R = (double*)(base + L.R);
  ws.T = (double*)(base + L.T);
  ws.TT = (double*)(base + L.TT);
  ws.g = (double*)(base + L.g);
  ws.gh = (double*)(base + L.gh);
  ws.cs = (double*)(base + L.cs);
  ws.sn = (double*)(base + L.sn);
  ws.coef = (double*)(base + L.coef);
  ws.coef2 = (double*)(base + L.coef2);
  ws.lvec = (double*)(base + L.lvec);
  ws.y = (double*)(base + L.y);
  ws.partials = (double*)(base + L.partials);
  ws.gpartials = (double*)(base + L.gpartials);
  ws.counters = (unsigned*)(base + L.counters);
  ws.st = (DevState*)(base + L.state);
  ws.n = n;
  ws.ldv = L.ldv;
  ws.ldh = m + 1;
  ws.ldt = m + 2;
  ws.pstride = L.pstride;
  ws.m = m;
  // basis columns that fit in three quarters of the 256 MB last-level cache
  const double colbytes = (double)basis_bytes(scheme) * (double)n;
  const double kept = kKeepBytes / colbytes;
  ws.keep = kept >= (double)(m + 2) ? m + 2 : (int)kept;
}

// Host mirror: the readback block's layout (readback_layout), with or
// without H and T.
size_t mirror_bytes(int m, bool matrices) {
  const Readback rb = readback_layout(m);
  return matrices ? rb.total : rb.H;
}
void bind_mirror(gmres_ctx* c, void* host, bool matrices) {
  const Readback rb = readback_layout(c->m);
  char* h = (char*)host;
  c->pinned = host;
  c->mirror_matrices = matrices;
  c->h_st = (DevState*)h;
  c->h_g = (double*)(h + rb.g);
  c->h_gh = (double*)(h + rb.gh);
  c->h_H = matrices ? (double*)(h + rb.H) : nullptr;
  c->h_T = matrices ? (double*)(h + rb.T) : nullptr;
}

// The solve itself, arguments already checked. hist_orth and the snapshot of
// the last cycle need the context's full host mirror (H and T).
int solve_impl(gmres_ctx* c, const double* b, double* x, double rtol, int64_t max_iters,
               gmres_info* info, double* hist_res, double* hist_orth) {
  gmres_info loc;
  memset(&loc, 0, sizeof(loc));
  if (info) *info = loc;
  const Ws& ws = c->ws;
  hipStream_t s = c->stream;
  const int m = c->m;
  int rc;

  if (launch_solve_begin(ws, s) ||
      launch_axpy_dot(ws, c->L.rpt, (double*)b, nullptr, nullptr, b, kTailBnorm, 0, 0, 0, rtol,
                      c->L.G, s))
    return GMRES_ERR_HIP;
  if ((rc = sync_state(c, false))) return rc;
  if (c->h_st->status) {
    loc.reductions = c->h_st->reductions;
    if (info) *info = loc;
    return GMRES_ERR_NONFINITE;
  }
  const double bnorm = c->h_st->bnorm;
  if (bnorm == 0.0) {
    if (hipMemsetAsync(x, 0, sizeof(double) * (size_t)c->A.n, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return GMRES_ERR_HIP;
    loc.converged = 1;
    loc.reductions = c->h_st->reductions;
    if (info) *info = loc;
    return GMRES_OK;
  }
  const double tol_abs = c->h_st->tol_abs;

  int64_t it = 0;
  rc = GMRES_OK;
  // The orthogonality history of a finished cycle is computed on the host
  // from its T (kept in last_T) while the device runs the next cycle.
  int orth_j = 0;
  int64_t orth_at = 0;
  auto flush_orth = [&]() {
    if (orth_j > 0) orth_history(c, orth_j, c->last_T.data(), hist_orth + orth_at);
    orth_j = 0;
  };
  for (;;) {
    const int64_t left = max_iters - it;
    const int m_eff = left < (int64_t)m ? (int)left : m;
    if (m_eff == 0) {
      flush_orth();
      if (enqueue_true_residual(c, b, x)) return GMRES_ERR_HIP;
      if ((rc = sync_state(c, false))) return rc;
      if (c->h_st->status) {
        rc = GMRES_ERR_NONFINITE;
        break;
      }
      loc.rel_res_true = c->h_st->beta / bnorm;
      loc.converged = c->h_st->beta <= tol_abs;
      if (loc.cycles == 0) loc.rel_res_est = loc.rel_res_true;
      break;
    }
    if (enqueue_cycle(c, b, x, m_eff)) return GMRES_ERR_HIP;
    flush_orth();
    if ((rc = sync_state(c, true))) return rc;
    const DevState& st = *c->h_st;
    collect_timing(c, st.j, st.true_conv != 0);
    if (st.status) {
      rc = GMRES_ERR_NONFINITE;
      break;
    }
    if (st.true_conv) {
      loc.converged = 1;
      loc.rel_res_true = st.beta / bnorm;
      if (loc.cycles == 0) loc.rel_res_est = loc.rel_res_true;
      break;
    }
    const int j = st.j;
    if (j > 0) {
      // the FP32-basis cycle's g is relative to its restart residual norm
      const double gs = st.xscale / bnorm;
      if (hist_res)
        for (int q = 0; q < j; ++q) hist_res[it + q] = c->h_gh[q + 1] * gs;
      loc.cycles += 1;
      // |g_j| as it stood right after rotation j-1: with a pipeline depth above
      // 1, later rotations of the same batch may have changed g[j] itself
      loc.rel_res_est = c->h_gh[j] * gs;
      if (c->mirror_matrices) {
        memcpy(c->last_H.data(), c->h_H, sizeof(double) * c->last_H.size());
        memcpy(c->last_T.data(), c->h_T, sizeof(double) * c->last_T.size());
        memcpy(c->last_g.data(), c->h_g, sizeof(double) * c->last_g.size());
        c->last_j = j;
        if (hist_orth) {
          orth_j = j;
          orth_at = it;
        }
      }
    }
    if (st.breakdown) loc.breakdown = 1;
    if (j == 0) break;  // no progress is possible; cannot happen for m_eff >= 1
    it += j;
  }
  flush_orth();
  loc.iters = it;
  loc.reductions = c->h_st->reductions;
  if (info) *info = loc;
  return rc;
}


}  // namespace

extern "C" {

size_t gmres_workspace_bytes_ex(int64_t n, int32_t m, int32_t scheme, const gmres_options* opt) {
  if (scheme < GMRES_MGS || scheme > GMRES_TWO_SYNCH || !check_options(opt, scheme)) return 0;
  Layout L;
  if (!make_layout(n, m, scheme, &L, opt ? opt->rows_per_lane : 0)) return 0;
  return L.total;
}

size_t gmres_workspace_bytes(int64_t n, int32_t m, int32_t scheme) {
  return gmres_workspace_bytes_ex(n, m, scheme, nullptr);
}

void gmres_options_init(gmres_options* opt) {
  if (opt) memset(opt, 0, sizeof(*opt));
}

const char* gmres_status_string(int status) {
  switch (status) {
    case GMRES_OK: return "ok";
    case GMRES_ERR_ARG: return "invalid argument";
    case GMRES_ERR_HIP: return "HIP runtime error";
    case GMRES_ERR_NONFINITE: return "non-finite value (NaN or Inf) in the iteration";
    case GMRES_ERR_WORKSPACE: return "workspace too small";
    case GMRES_ERR_TOO_LARGE:
      return "problem needs more workspace than the fixed scratch of gmres_solve_noalloc "
             "(GMRES_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

int gmres_create(gmres_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                 void* workspace, size_t ws_bytes, void* hip_stream) {
  return gmres_create_ex(out, n, nnz, row_ptr, col_idx, vals, m, scheme, workspace, ws_bytes,
                         hip_stream, nullptr);
}

int gmres_create_ex(gmres_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                    const int32_t* col_idx, const double* vals, int32_t m, int32_t scheme,
                    void* workspace, size_t ws_bytes, void* hip_stream, const gmres_options* opt) {
  if (!out) return GMRES_ERR_ARG;
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31) || nnz < 0 || nnz >= ((int64_t)1 << 31) || m < 1 ||
      m > GMRES_MAX_RESTART || scheme < GMRES_MGS || scheme > GMRES_TWO_SYNCH ||
      !check_options(opt, scheme))
    return GMRES_ERR_ARG;
  if (!is_device_ptr(row_ptr) || !is_device_ptr(workspace) ||
      (nnz > 0 && (!is_device_ptr(col_idx) || !is_device_ptr(vals))))
    return GMRES_ERR_ARG;
  if (((uintptr_t)workspace % kAlign) != 0) return GMRES_ERR_ARG;
  Layout L;
  if (!make_layout(n, m, scheme, &L, opt ? opt->rows_per_lane : 0)) return GMRES_ERR_ARG;
  if (ws_bytes < L.total) return GMRES_ERR_WORKSPACE;

  gmres_ctx* c = new (std::nothrow) gmres_ctx();
  if (!c) return GMRES_ERR_ARG;
  bind_context(c, n, nnz, row_ptr, col_idx, vals, m, scheme, L, workspace,
               (hipStream_t)hip_stream, opt);
  const Ws& ws = c->ws;

  void* pin = nullptr;
  if (hipHostMalloc(&pin, mirror_bytes(m, true), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return GMRES_ERR_HIP;
  }
  bind_mirror(c, pin, true);
  c->last_H.assign((size_t)(m + 1) * m, 0.0);
  c->last_T.assign((size_t)(m + 2) * (m + 2), 0.0);
  c->last_g.assign((size_t)(m + 2), 0.0);
  c->last_j = 0;
  c->timing = false;
  memset(c->stats, 0, sizeof(c->stats));

  int rc = GMRES_OK;
  c->matrix_ok = true;
  if (launch_init(ws, L.NG + 1, c->stream) || launch_validate(c->A, nnz, ws.st, c->stream))
    rc = GMRES_ERR_HIP;
  if (rc == GMRES_OK) rc = sync_state(c, false);
  if (rc == GMRES_OK && c->h_st->bad_csr) rc = GMRES_ERR_ARG;
  if (rc == GMRES_OK) rc = plan_format(c);
  if (rc != GMRES_OK) {
    (void)hipHostFree(c->pinned);
    delete c;
    return rc;
  }
  *out = c;
  return GMRES_OK;
}

int gmres_destroy(gmres_ctx* c) {
  if (!c) return GMRES_ERR_ARG;
  int rc = GMRES_OK;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->pinned && hipHostFree(c->pinned) != hipSuccess) rc = GMRES_ERR_HIP;
  delete c;
  return rc;
}

int gmres_refresh_matrix(gmres_ctx* c) {
  if (!c) return GMRES_ERR_ARG;
  if (hipMemsetAsync(&c->ws.st->bad_csr, 0, sizeof(int32_t), c->stream) != hipSuccess ||
      launch_validate(c->A, c->nnz, c->ws.st, c->stream))
    return GMRES_ERR_HIP;
  if (c->format == kFormatSell && fill_copy(c, c->sell)) return GMRES_ERR_HIP;
  c->matrix_ok = false;
  const int rc = sync_state(c, false);
  if (rc != GMRES_OK) return rc;
  if (c->h_st->bad_csr) return GMRES_ERR_ARG;
  c->matrix_ok = true;
  return GMRES_OK;
}

int gmres_matrix_storage_bytes(gmres_ctx* c, size_t* bytes) {
  if (!c || !bytes) return GMRES_ERR_ARG;
  *bytes = c->sell_bytes;
  return GMRES_OK;
}

int gmres_set_matrix_storage(gmres_ctx* c, void* storage, size_t bytes) {
  if (!c) return GMRES_ERR_ARG;
  if (!storage) {
    c->format = kFormatCsr;
    c->sell = Sell{};
    return GMRES_OK;
  }
  if (c->sell_bytes == 0 || bytes < c->sell_bytes || ((uintptr_t)storage % kAlign) != 0 ||
      !is_device_ptr(storage))
    return GMRES_ERR_ARG;
  char* base = (char*)storage;
  const int64_t ns = (int64_t)c->sell_sp.size() - 1;
  const bool fv = ir_scheme(c->scheme);  // float32 values for the reduced-precision bases
  Sell S{};
  S.sp = (const int64_t*)base;
  S.sf = c->sell_sf;
  S.ci = S.sf == kSfI32 ? (int*)(base + c->o_ci) : nullptr;
  S.cd = S.sf == kSfD16 ? (uint16_t*)(base + c->o_ci) : nullptr;
  S.cbase = S.sf != kSfI32 ? (int*)(base + c->o_cb) : nullptr;
  S.va = (double*)(base + c->o_va64);
  S.vaf = fv ? (float*)(base + c->o_va) : nullptr;
  S.ns = ns;
  S.n = c->A.n;
  if (hipMemcpyAsync(base, c->sell_sp.data(), sizeof(int64_t) * (size_t)(ns + 1),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemsetAsync(&c->ws.st->bad_csr, 0, sizeof(int32_t), c->stream) != hipSuccess ||
      fill_copy(c, S))
    return GMRES_ERR_HIP;
  const int rc = sync_state(c, false);  // also keeps the offsets' host copy alive until done
  if (rc != GMRES_OK) return rc;
  if (c->h_st->bad_csr) return GMRES_ERR_ARG;
  c->sell = S;
  c->format = kFormatSell;
  return GMRES_OK;
}

int gmres_get_format(gmres_ctx* c, int32_t* format, int64_t* stored_entries) {
  if (!c || !format || !stored_entries) return GMRES_ERR_ARG;
  *format = c->format != kFormatSell  ? GMRES_FORMAT_CSR
            : c->sell.sf == kSfDiag ? GMRES_FORMAT_SELL64_DIAG
            : c->sell.sf == kSfD16  ? GMRES_FORMAT_SELL64_D16
                                    : GMRES_FORMAT_SELL64;
  *stored_entries = c->format == kFormatSell ? c->sell_entries : c->nnz;
  return GMRES_OK;
}

int gmres_spmv(gmres_ctx* c, const double* x, double* y) {
  if (!c || !x || !y || x == y || !c->matrix_ok) return GMRES_ERR_ARG;
  return spmv(c, x, nullptr, y, nullptr, c->stream) ? GMRES_ERR_HIP : GMRES_OK;
}

int gmres_basis(gmres_ctx* c, double** V, int64_t* ldv) {
  if (!c || ir_scheme(c->scheme)) return GMRES_ERR_ARG;
  if (V) *V = c->ws.V;
  if (ldv) *ldv = c->ws.ldv;
  return GMRES_OK;
}

int gmres_set_timing(gmres_ctx* c, int enable) {
  if (!c) return GMRES_ERR_ARG;
  c->timing = enable != 0;
  c->recs.clear();
  memset(c->stats, 0, sizeof(c->stats));
  return GMRES_OK;
}

int gmres_get_timing(gmres_ctx* c, gmres_kernel_stat* stats) {
  if (!c || !stats) return GMRES_ERR_ARG;
  memcpy(stats, c->stats, sizeof(c->stats));
  return GMRES_OK;
}

int gmres_last_cycle(gmres_ctx* c, double* H, double* T, double* g, int32_t* j) {
  if (!c) return GMRES_ERR_ARG;
  if (H) memcpy(H, c->last_H.data(), sizeof(double) * c->last_H.size());
  if (T) memcpy(T, c->last_T.data(), sizeof(double) * c->last_T.size());
  if (g) memcpy(g, c->last_g.data(), sizeof(double) * c->last_g.size());
  if (j) *j = c->last_j;
  return GMRES_OK;
}

int gmres_solve(gmres_ctx* c, const double* b, double* x, double rtol, int64_t max_iters,
                gmres_info* info, double* hist_res, double* hist_orth) {
  if (info) memset(info, 0, sizeof(*info));
  if (!c || !b || !x || !(rtol >= 0.0) || max_iters < 0 || !c->matrix_ok) return GMRES_ERR_ARG;
  if (!is_device_ptr(b) || !is_device_ptr(x)) return GMRES_ERR_ARG;
  return solve_impl(c, b, x, rtol, max_iters, info, hist_res, hist_orth);
}

int gmres_solve_noalloc(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                        const double* vals, int32_t m, int32_t scheme, const double* b, double* x,
                        double rtol, int64_t max_iters, gmres_info* info, double* hist_res,
                        void* hip_stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (n < 1 || n >= ((int64_t)1 << 31) || nnz < 0 || nnz >= ((int64_t)1 << 31) || m < 1 ||
      m > GMRES_MAX_RESTART || scheme < GMRES_MGS || scheme > GMRES_TWO_SYNCH ||
      !(rtol >= 0.0) || max_iters < 0)
    return GMRES_ERR_ARG;
  Layout L;
  if (!make_layout(n, m, scheme, &L)) return GMRES_ERR_ARG;
  if (L.total > GMRES_NOALLOC_SCRATCH_BYTES) return GMRES_ERR_TOO_LARGE;
  if (!is_device_ptr(row_ptr) || !is_device_ptr(b) || !is_device_ptr(x) ||
      (nnz > 0 && (!is_device_ptr(col_idx) || !is_device_ptr(vals))))
    return GMRES_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GMRES_ERR_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  if (s) {
    hipDevice_t sd = -1;
    if (hipStreamGetDevice(s, &sd) != hipSuccess) return GMRES_ERR_HIP;
    if (sd != dev) return GMRES_ERR_ARG;
  }
  void* ws = scratch_on(dev);
  if (!ws) return GMRES_ERR_HIP;

  // A context on the stack: its vectors stay empty, the host mirror (state,
  // g and gh only) is a stack buffer, the SpMV reads the CSR arrays, and no
  // timing events are made, so nothing is allocated.
  gmres_ctx c{};
  bind_context(&c, n, nnz, row_ptr, col_idx, vals, m, scheme, L, ws, s, nullptr);
  alignas(64) unsigned char host[readback_layout(GMRES_MAX_RESTART).H];
  bind_mirror(&c, host, false);
  c.matrix_ok = true;
  c.format = kFormatCsr;
  c.sell = Sell{};
  c.sell_entries = 0;
  c.sell_sf = kSfI32;
  c.sell_bytes = 0;
  c.last_j = 0;
  c.timing = false;
  memset(c.stats, 0, sizeof(c.stats));
  // the scratch holds whatever the last call left: clear the counters and
  // the state, and check this call's matrix
  if (launch_init(c.ws, L.NG + 1, s) || launch_validate(c.A, nnz, c.ws.st, s)) return GMRES_ERR_HIP;
  int rc = sync_state(&c, false);
  if (rc != GMRES_OK) return rc;
  if (c.h_st->bad_csr) return GMRES_ERR_ARG;
  return solve_impl(&c, b, x, rtol, max_iters, info, hist_res, nullptr);
}

}  // extern "C"

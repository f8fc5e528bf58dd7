// Host driver of the batched solver (the gmres_batch_* calls of gmres.h).
//
// Many independent systems, the diagonal blocks of one CSR matrix, are solved
// by restarted one-reduce GMRES(m) (the lagged compact-WY MGS step of
// Section III) in a single persistent launch: workgroups take entries from a
// device-side queue, each a whole system or one row part of a larger one
// (a team), and run that entry's whole solve. The host side builds the queue
// for a configuration (team sizes, order, grid), times configurations for the
// autotuner and captures the launch into a HIP graph. Everything a solve
// needs lives in the caller's workspace, laid out here once at create.
#include "gmres.h"
#include "gmres_internal.h"

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

using namespace gmres;

static_assert(sizeof(BatchOut) == sizeof(gmres_batch_info), "result layouts differ");
static_assert(offsetof(BatchOut, cycles) == offsetof(gmres_batch_info, cycles), "result layouts differ");
static_assert(offsetof(BatchOut, converged) == offsetof(gmres_batch_info, converged), "result layouts differ");
static_assert(offsetof(BatchOut, status) == offsetof(gmres_batch_info, status), "result layouts differ");
static_assert(offsetof(BatchOut, breakdown) == offsetof(gmres_batch_info, breakdown), "result layouts differ");
static_assert(offsetof(BatchOut, rel_res_true) == offsetof(gmres_batch_info, rel_res_true),
              "result layouts differ");

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxSysRows = (int64_t)1 << 28;  // the kernel's 32-bit byte offsets

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// A system is split into at most kTeamMax parts of at least kMinPartRows
// rows each; every possible part has a slot (small workspace, state record,
// reduction partials) reserved at create.
constexpr int kTeamMax = 16;
constexpr int64_t kDefaultPartRows = 8192;
constexpr int64_t kMinPartRows = 256;
// Bases in use at once beyond this size (1.5 times the MI355X's 256 MB
// last-level cache) are streamed with non-temporal loads under
// GMRES_BATCH_LOADS_AUTO: their re-reads would miss the cache anyway.
constexpr double kStreamBytes = 384.0 * 1048576.0;

int team_cap(int64_t n) {
  const int64_t c = (n + kMinPartRows - 1) / kMinPartRows;
  return (int)std::max<int64_t>(1, std::min<int64_t>(kTeamMax, c));
}

struct BatchLayout {
  std::vector<BatchSys> sys;
  int64_t n;
  int slots;
  size_t o_sys, o_tk, o_st, o_part, o_bar, o_queue, o_out, o_small, o_V, o_w, o_r64, o_xsave, total;
};

// Every system's basis starts 256-byte aligned with a leading dimension that
// is a multiple of 64 elements.
bool batch_layout(int32_t nsys, const int64_t* row_off, int32_t m, int32_t scheme, BatchLayout* L) {
  if (nsys < 1 || !row_off || m < 1 || m > GMRES_MAX_RESTART) return false;
  if (scheme != GMRES_MGS_1R && scheme != GMRES_MGS_1R_IR32) return false;
  if (row_off[0] != 0) return false;
  const size_t vb = scheme == GMRES_MGS_1R_IR32 ? sizeof(float) : sizeof(double);
  const size_t small = batch_small_doubles(m);
  L->sys.resize((size_t)nsys);
  int64_t voff = 0, slots = 0;
  for (int32_t i = 0; i < nsys; ++i) {
    const int64_t n = row_off[i + 1] - row_off[i];
    if (n < 1 || n >= kMaxSysRows) return false;
    BatchSys& s = L->sys[(size_t)i];
    s.r0 = row_off[i];
    s.n = n;
    s.ldv = (int64_t)round_up((size_t)n, 64);
    s.voff = voff;
    voff += s.ldv * (m + 1);
    slots += team_cap(n);
  }
  L->n = row_off[nsys];
  if (L->n >= ((int64_t)1 << 31) || slots >= ((int64_t)1 << 30)) return false;
  L->slots = (int)slots;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = round_up(off + bytes, kAlign);
    return at;
  };
  L->o_sys = take(sizeof(BatchSys) * (size_t)nsys);
  L->o_tk = take(sizeof(BatchTicket) * (size_t)slots);
  L->o_st = take(sizeof(DevState) * (size_t)slots);
  L->o_part = take(sizeof(double) * 4 * (size_t)(m + 2) * (size_t)slots);
  L->o_bar = take(sizeof(unsigned) * (size_t)nsys);
  L->o_queue = take(sizeof(unsigned));
  L->o_out = take(sizeof(BatchOut) * (size_t)nsys);
  L->o_small = take(sizeof(double) * small * (size_t)slots);
  L->o_V = take(vb * (size_t)voff);
  L->o_w = take(vb * (size_t)L->n);
  L->o_r64 = scheme == GMRES_MGS_1R_IR32 ? take(sizeof(double) * (size_t)L->n) : 0;
  L->o_xsave = take(sizeof(double) * (size_t)L->n);
  L->total = off;
  return true;
}

}  // namespace

struct gmres_batch {
  Batch B;            // device view; b, x, rtol, max_iters and out set per solve
  int nsys, m, scheme, slots;
  int64_t n;
  int bs, grid, order;  // grid 0: as many workgroups as the GPU holds
  int64_t part_rows;    // rows per part of a team (0: one workgroup per system)
  int loads;            // GMRES_BATCH_LOADS_*
  bool nt;              // basis columns loaded non-temporal in the current configuration
  int grid_eff;         // the grid of the current queue
  int num_cu;
  BatchTicket* tickets_d;
  std::vector<BatchTicket> tickets;
  BatchOut* out_ws;
  double* xsave;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  std::vector<int64_t> sizes;
  std::vector<int64_t> sell_sp;  // planned slice offsets of the copy by diagonals (empty: none)
  size_t sell_bytes, o_cb, o_va; // its size and layout
};

namespace {

// A captured graph holds the grid, block size and queue length it was
// captured with: any change of configuration discards it.
void drop_graph(gmres_batch* bt) {
  if (bt->graph_exec) (void)hipGraphExecDestroy(bt->graph_exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->graph_exec = nullptr;
  bt->graph = nullptr;
}

// Plan the copy of the block-diagonal matrix by diagonals (64-row slices of
// global rows, a slice column per distinct col - row value among a slice's
// rows; the layout of the single-system copy): when every row's columns are
// strictly increasing and it costs at most a quarter more entries than nnz.
// The slice widths are counted on the device in the basis region of the
// workspace, which holds nothing before the first solve.
int plan_diag(gmres_batch* bt) {
  bt->sell_sp.clear();
  bt->sell_bytes = bt->o_cb = bt->o_va = 0;
  const Csr& A = bt->B.A;
  if (A.nnz == 0 || A.n >= kSellMaxRows) return GMRES_OK;
  const int64_t ns = (A.n + 63) / 64;
  int* dd = (int*)bt->B.Vb;  // 2 (ns + 1) ints: far less than the basis region
  std::vector<int> dh((size_t)ns + 1);
  hipStream_t s = bt->stream;
  if (hipMemsetAsync(dd + ns, 0, sizeof(int), s) != hipSuccess ||
      launch_sell_diags(A, ns, dd, dd + ns, kSellMaxWidth, s) ||
      hipMemcpyAsync(dh.data(), dd, sizeof(int) * (size_t)(ns + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GMRES_ERR_HIP;
  if (dh[(size_t)ns] != 0) return GMRES_OK;
  std::vector<int64_t> sp((size_t)ns + 1, 0);
  for (int64_t i = 0; i < ns; ++i) {
    if (dh[(size_t)i] > kSellMaxWidth) return GMRES_OK;
    sp[(size_t)i + 1] = sp[(size_t)i] + 64 * (int64_t)dh[(size_t)i];
  }
  const int64_t total = sp[(size_t)ns];
  if (total * 4 > A.nnz * 5) return GMRES_OK;
  bt->sell_sp.swap(sp);
  bt->o_cb = round_up(sizeof(int64_t) * (size_t)(ns + 1), kAlign);
  bt->o_va = round_up(bt->o_cb + sizeof(int) * (size_t)(total / 64), kAlign);
  bt->sell_bytes = bt->o_va + sizeof(double) * (size_t)total;
  return GMRES_OK;
}

// Team sizes, queue order and grid for a configuration; uploads the queue
// (blocking), and discards any captured graph. Parts of a system: ceil(n / part_rows), at most kTeamMax, one per
// kMinPartRows rows, and no more than the grid or what the GPU holds at once,
// so that every team can assemble.
int apply_config(gmres_batch* bt, int bs, int grid, int order, int64_t part_rows) {
  drop_graph(bt);
  // the fewer of the two load forms' resident workgroups, whichever runs
  const bool f32 = bt->scheme == GMRES_MGS_1R_IR32;
  const int per_cu = std::min(batch_resident_blocks(bs, bt->m, f32, false),
                              batch_resident_blocks(bs, bt->m, f32, true));
  if (per_cu < 1) return GMRES_ERR_HIP;
  const int64_t resident = (int64_t)per_cu * bt->num_cu;
  const int64_t cap = std::min<int64_t>(resident, grid > 0 ? grid : resident);
  std::vector<int> seq((size_t)bt->nsys);
  std::iota(seq.begin(), seq.end(), 0);
  if (order == GMRES_BATCH_ORDER_LARGEST_FIRST)
    std::stable_sort(seq.begin(), seq.end(),
                     [&](int a, int b) { return bt->sizes[(size_t)a] > bt->sizes[(size_t)b]; });
  std::vector<BatchTicket> tk;
  tk.reserve((size_t)bt->slots);
  for (int i : seq) {
    const int64_t n = bt->sizes[(size_t)i];
    int64_t T = part_rows > 0 ? (n + part_rows - 1) / part_rows : 1;
    T = std::max<int64_t>(1, std::min<int64_t>({T, (int64_t)team_cap(n), cap}));
    const int base = (int)tk.size();
    for (int p = 0; p < (int)T; ++p) tk.push_back(BatchTicket{i, p, (int)T, base});
  }
  if ((int)tk.size() > bt->slots) return GMRES_ERR_ARG;  // cannot happen: T <= team_cap
  if (hipMemcpyAsync(bt->tickets_d, tk.data(), sizeof(BatchTicket) * tk.size(), hipMemcpyHostToDevice,
                     bt->stream) != hipSuccess ||
      hipStreamSynchronize(bt->stream) != hipSuccess)
    return GMRES_ERR_HIP;
  bt->tickets.swap(tk);
  bt->B.ntickets = (int)bt->tickets.size();
  bt->bs = bs;
  bt->grid = grid;
  bt->order = order;
  bt->part_rows = part_rows;
  bt->grid_eff = grid > 0 ? grid : (int)std::max<int64_t>(1, std::min<int64_t>(resident, bt->B.ntickets));
  if (bt->loads == GMRES_BATCH_LOADS_AUTO) {
    // basis in use at once: a queue entry's rows per running workgroup
    const double vb = f32 ? 4.0 : 8.0;
    const double per_entry = (double)bt->n / (double)std::max(1, bt->B.ntickets);
    const double live = std::min((double)bt->n, per_entry * (double)std::min(bt->grid_eff, bt->B.ntickets)) *
                        (double)(bt->m + 1) * vb;
    bt->nt = live > kStreamBytes;
  } else {
    bt->nt = bt->loads == GMRES_BATCH_LOADS_STREAMED;
  }
  return GMRES_OK;
}

int enqueue(gmres_batch* bt, const double* b, double* x, double rtol, int64_t max_iters,
            gmres_batch_info* info, hipEvent_t e0, hipEvent_t e1) {
  Batch B = bt->B;
  B.b = b;
  B.x = x;
  B.rtol = rtol;
  B.max_iters = max_iters;
  B.out = info ? reinterpret_cast<BatchOut*>(info) : bt->out_ws;
  if (launch_batch_reset(B, bt->stream)) return GMRES_ERR_HIP;
  if (launch_batch(B, bt->bs, bt->grid_eff, bt->scheme == GMRES_MGS_1R_IR32, bt->nt, bt->stream, e0,
                   e1))
    return GMRES_ERR_HIP;
  return GMRES_OK;
}

}  // namespace

extern "C" {

size_t gmres_batch_workspace_bytes(int32_t nsys, const int64_t* row_off, int32_t m, int32_t scheme) {
  BatchLayout L;
  if (!batch_layout(nsys, row_off, m, scheme, &L)) return 0;
  return L.total;
}

int gmres_batch_create(gmres_batch** out, int32_t nsys, const int64_t* row_off, int64_t nnz,
                       const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                       int32_t m, int32_t scheme, void* workspace, size_t ws_bytes,
                       void* hip_stream) {
  if (!out) return GMRES_ERR_ARG;
  *out = nullptr;
  BatchLayout L;
  if (!batch_layout(nsys, row_off, m, scheme, &L)) return GMRES_ERR_ARG;
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return GMRES_ERR_ARG;
  if (!is_device_ptr(row_ptr) || !is_device_ptr(workspace) ||
      (nnz > 0 && (!is_device_ptr(col_idx) || !is_device_ptr(vals))))
    return GMRES_ERR_ARG;
  if (((uintptr_t)workspace % kAlign) != 0) return GMRES_ERR_ARG;
  if (ws_bytes < L.total) return GMRES_ERR_WORKSPACE;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
    return GMRES_ERR_HIP;

  gmres_batch* bt = new (std::nothrow) gmres_batch();
  if (!bt) return GMRES_ERR_ARG;
  char* base = (char*)workspace;
  Batch& B = bt->B;
  B.A = Csr{row_ptr, col_idx, vals, L.n, nnz};
  B.sys = (const BatchSys*)(base + L.o_sys);
  B.tickets = (const BatchTicket*)(base + L.o_tk);
  B.nsys = nsys;
  B.ntickets = 0;
  B.m = m;
  B.Vb = base + L.o_V;
  B.wb = base + L.o_w;
  B.r64 = scheme == GMRES_MGS_1R_IR32 ? (double*)(base + L.o_r64) : nullptr;
  B.small = (double*)(base + L.o_small);
  B.st = (DevState*)(base + L.o_st);
  B.partials = (double*)(base + L.o_part);
  B.bar = (unsigned*)(base + L.o_bar);
  B.queue = (unsigned*)(base + L.o_queue);
  B.out = (BatchOut*)(base + L.o_out);
  // polls of a team barrier before a part gives up: GMRES_BATCH_WAIT_LIMIT
  // (about half a minute at least); gmres_batch_set_wait_limit lowers it
  B.spin_limit = GMRES_BATCH_WAIT_LIMIT;
  bt->nsys = nsys;
  bt->m = m;
  bt->scheme = scheme;
  bt->slots = L.slots;
  bt->n = L.n;
  bt->num_cu = ncu;
  bt->tickets_d = (BatchTicket*)(base + L.o_tk);
  bt->out_ws = (BatchOut*)(base + L.o_out);
  bt->xsave = (double*)(base + L.o_xsave);
  bt->stream = (hipStream_t)hip_stream;
  bt->graph = nullptr;
  bt->graph_exec = nullptr;
  bt->sizes.resize((size_t)nsys);
  for (int i = 0; i < nsys; ++i) bt->sizes[(size_t)i] = L.sys[(size_t)i].n;

  DevState st0;
  int rc = GMRES_OK;
  hipStream_t s = bt->stream;
  if (hipMemcpyAsync(base + L.o_sys, L.sys.data(), sizeof(BatchSys) * (size_t)nsys,
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(B.st, 0, sizeof(DevState), s) != hipSuccess ||
      launch_validate(B.A, nnz, B.st, s) ||
      hipMemcpyAsync(&st0, B.st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = GMRES_ERR_HIP;
  if (rc == GMRES_OK && st0.bad_csr) rc = GMRES_ERR_ARG;
  // the block-diagonal check reads col_idx through row_ptr, so only after the
  // CSR arrays themselves passed
  if (rc == GMRES_OK &&
      (launch_batch_validate(B.A, B.sys, nsys, B.st, s) ||
       hipMemcpyAsync(&st0, B.st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    rc = GMRES_ERR_HIP;
  if (rc == GMRES_OK && st0.bad_csr) rc = GMRES_ERR_ARG;
  if (rc == GMRES_OK) rc = plan_diag(bt);
  if (rc == GMRES_OK)
    rc = apply_config(bt, 256, 0, GMRES_BATCH_ORDER_LARGEST_FIRST, kDefaultPartRows);
  if (rc != GMRES_OK) {
    delete bt;
    return rc;
  }
  *out = bt;
  return GMRES_OK;
}

int gmres_batch_matrix_storage_bytes(gmres_batch* bt, size_t* bytes) {
  if (!bt || !bytes) return GMRES_ERR_ARG;
  *bytes = bt->sell_bytes;
  return GMRES_OK;
}

int gmres_batch_set_matrix_storage(gmres_batch* bt, void* storage, size_t bytes) {
  if (!bt) return GMRES_ERR_ARG;
  drop_graph(bt);  // a captured graph holds the matrix form it was captured with
  if (!storage) {
    bt->B.S = Sell{};
    return GMRES_OK;
  }
  if (bt->sell_bytes == 0 || bytes < bt->sell_bytes || ((uintptr_t)storage % kAlign) != 0 ||
      !is_device_ptr(storage))
    return GMRES_ERR_ARG;
  char* base = (char*)storage;
  const int64_t ns = (int64_t)bt->sell_sp.size() - 1;
  Sell S{};
  S.sp = (const int64_t*)base;
  S.cbase = (int*)(base + bt->o_cb);
  S.va = (double*)(base + bt->o_va);
  S.ns = ns;
  S.n = bt->n;
  S.sf = kSfDiag;
  DevState st0;
  hipStream_t s = bt->stream;
  if (hipMemcpyAsync(base, bt->sell_sp.data(), sizeof(int64_t) * (size_t)(ns + 1),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(&bt->B.st->bad_csr, 0, sizeof(int32_t), s) != hipSuccess ||
      launch_sell_fill(bt->B.A, S, bt->B.st, s) ||
      hipMemcpyAsync(&st0, bt->B.st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GMRES_ERR_HIP;
  if (st0.bad_csr) return GMRES_ERR_ARG;
  bt->B.S = S;
  return GMRES_OK;
}

int gmres_batch_get_format(gmres_batch* bt, int32_t* format, int64_t* stored_entries) {
  if (!bt || !format || !stored_entries) return GMRES_ERR_ARG;
  const bool diag = bt->B.S.va != nullptr;
  *format = diag ? GMRES_FORMAT_SELL64_DIAG : GMRES_FORMAT_CSR;
  *stored_entries = diag ? bt->sell_sp.back() : bt->B.A.nnz;
  return GMRES_OK;
}

int gmres_batch_destroy(gmres_batch* bt) {
  if (!bt) return GMRES_ERR_ARG;
  drop_graph(bt);
  delete bt;
  return GMRES_OK;
}

int gmres_batch_set_stream(gmres_batch* bt, void* hip_stream) {
  if (!bt) return GMRES_ERR_ARG;
  bt->stream = (hipStream_t)hip_stream;
  return GMRES_OK;
}

int gmres_batch_set_wait_limit(gmres_batch* bt, uint32_t polls) {
  if (!bt || polls > GMRES_BATCH_WAIT_LIMIT) return GMRES_ERR_ARG;
  bt->B.spin_limit = polls;
  drop_graph(bt);  // a captured graph holds the old limit
  return GMRES_OK;
}

int gmres_batch_solve_async(gmres_batch* bt, const double* b, double* x, double rtol,
                            int64_t max_iters, gmres_batch_info* info) {
  if (!bt || !b || !x || !(rtol >= 0.0) || max_iters < 0) return GMRES_ERR_ARG;
  return enqueue(bt, b, x, rtol, max_iters, info, nullptr, nullptr);
}

int gmres_batch_read_info(gmres_batch* bt, gmres_batch_info* info) {
  if (!bt || !info) return GMRES_ERR_ARG;
  if (hipMemcpyAsync(info, bt->out_ws, sizeof(BatchOut) * (size_t)bt->nsys, hipMemcpyDeviceToHost,
                     bt->stream) != hipSuccess ||
      hipStreamSynchronize(bt->stream) != hipSuccess)
    return GMRES_ERR_HIP;
  return GMRES_OK;
}

int gmres_batch_solve(gmres_batch* bt, const double* b, double* x, double rtol, int64_t max_iters,
                      gmres_batch_info* info) {
  if (!bt || !is_device_ptr(b) || !is_device_ptr(x) || !(rtol >= 0.0) || max_iters < 0)
    return GMRES_ERR_ARG;
  int rc = enqueue(bt, b, x, rtol, max_iters, nullptr, nullptr, nullptr);
  if (rc) return rc;
  std::vector<gmres_batch_info> h((size_t)bt->nsys);
  rc = gmres_batch_read_info(bt, h.data());
  if (rc) return rc;
  if (info) memcpy(info, h.data(), sizeof(gmres_batch_info) * h.size());
  int worst = GMRES_OK;
  for (const auto& o : h) {
    if (o.status == GMRES_ERR_HIP) return GMRES_ERR_HIP;
    if (o.status) worst = GMRES_ERR_NONFINITE;
  }
  return worst;
}

int gmres_batch_set_config(gmres_batch* bt, int32_t block_size, int32_t grid, int32_t order,
                           int64_t part_rows) {
  if (!bt) return GMRES_ERR_ARG;
  if (block_size != 256 && block_size != 512 && block_size != 1024) return GMRES_ERR_ARG;
  if (grid < 0 || part_rows < 0) return GMRES_ERR_ARG;
  if (order != GMRES_BATCH_ORDER_NATURAL && order != GMRES_BATCH_ORDER_LARGEST_FIRST)
    return GMRES_ERR_ARG;
  return apply_config(bt, block_size, grid, order, part_rows);
}

int gmres_batch_set_loads(gmres_batch* bt, int32_t mode) {
  if (!bt || mode < GMRES_BATCH_LOADS_AUTO || mode > GMRES_BATCH_LOADS_STREAMED) return GMRES_ERR_ARG;
  bt->loads = mode;
  return apply_config(bt, bt->bs, bt->grid, bt->order, bt->part_rows);
}

int gmres_batch_get_loads(gmres_batch* bt, int32_t* mode, int32_t* streamed) {
  if (!bt) return GMRES_ERR_ARG;
  if (mode) *mode = bt->loads;
  if (streamed) *streamed = bt->nt ? 1 : 0;
  return GMRES_OK;
}

int gmres_batch_get_config(gmres_batch* bt, int32_t* block_size, int32_t* grid, int32_t* order,
                           int64_t* part_rows, int32_t* max_parts) {
  if (!bt) return GMRES_ERR_ARG;
  if (block_size) *block_size = bt->bs;
  if (grid) *grid = bt->grid_eff;
  if (order) *order = bt->order;
  if (part_rows) *part_rows = bt->part_rows;
  if (max_parts) {
    int mp = 1;
    for (const auto& t : bt->tickets) mp = std::max(mp, t.nparts);
    *max_parts = mp;
  }
  return GMRES_OK;
}

int gmres_batch_autotune(gmres_batch* bt, const double* b, double* x, double rtol,
                         int64_t max_iters, gmres_batch_trial* trials, int32_t max_trials,
                         int32_t* ntrials) {
  if (ntrials) *ntrials = 0;
  if (!bt || !is_device_ptr(b) || !is_device_ptr(x) || !(rtol >= 0.0) || max_iters < 0 ||
      max_trials < 0 || (max_trials > 0 && !trials))
    return GMRES_ERR_ARG;
  const size_t xb = sizeof(double) * (size_t)bt->n;
  hipStream_t s = bt->stream;
  struct Cand {
    int bs, grid, order;
    int64_t part_rows;
    int loads;
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GMRES_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GMRES_ERR_HIP;
  }
  const Cand saved{bt->bs, bt->grid, bt->order, bt->part_rows, bt->loads};
  int rc = hipMemcpyAsync(bt->xsave, x, xb, hipMemcpyDeviceToDevice, s) == hipSuccess
               ? GMRES_OK
               : GMRES_ERR_HIP;
  int nt = 0;
  float best = -1.0f;
  Cand pick = saved;
  // One solve under configuration c from the saved x; its event-timed duration.
  auto trial = [&](const Cand& c, bool record) -> int {
    bt->loads = c.loads;
    int r = apply_config(bt, c.bs, c.grid, c.order, c.part_rows);
    if (r) return r;
    if (hipMemcpyAsync(x, bt->xsave, xb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess)
      return GMRES_ERR_HIP;
    r = enqueue(bt, b, x, rtol, max_iters, nullptr, nullptr, nullptr);
    if (r) return r;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return GMRES_ERR_HIP;
    if (!record) return GMRES_OK;
    if (nt < max_trials)
      trials[nt] = gmres_batch_trial{c.bs, bt->grid_eff, c.order, ms, c.part_rows, bt->nt ? 1 : 0};
    ++nt;
    if (best < 0.0f || ms < best) {
      best = ms;
      pick = c;
    }
    return GMRES_OK;
  };
  // first the workgroup size and the team split (largest systems first, as
  // many workgroups as the GPU holds), then the grid and the order for the best
  const int lm = saved.loads;
  const Cand first{256, 0, GMRES_BATCH_ORDER_LARGEST_FIRST, kDefaultPartRows, lm};
  if (rc == GMRES_OK) rc = trial(first, false);  // warm-up
  for (int bs : {256, 512, 1024})
    for (int64_t pr : {(int64_t)0, (int64_t)16384, (int64_t)8192, (int64_t)4096})
      if (rc == GMRES_OK) rc = trial(Cand{bs, 0, GMRES_BATCH_ORDER_LARGEST_FIRST, pr, lm}, true);
  if (rc == GMRES_OK) {
    const Cand top = pick;
    rc = trial(Cand{top.bs, std::min(bt->num_cu, bt->B.ntickets), top.order, top.part_rows, lm},
               true);
    if (rc == GMRES_OK)
      rc = trial(Cand{top.bs, 0, GMRES_BATCH_ORDER_NATURAL, top.part_rows, lm}, true);
  }
  if (rc == GMRES_OK && lm == GMRES_BATCH_LOADS_AUTO) {
    // the best so far with the other load form
    const Cand top = pick;
    bt->loads = top.loads;
    rc = apply_config(bt, top.bs, top.grid, top.order, top.part_rows);
    const int other = bt->nt ? GMRES_BATCH_LOADS_CACHED : GMRES_BATCH_LOADS_STREAMED;
    if (rc == GMRES_OK) rc = trial(Cand{top.bs, top.grid, top.order, top.part_rows, other}, true);
  }
  if (rc == GMRES_OK &&
      (hipMemcpyAsync(x, bt->xsave, xb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    rc = GMRES_ERR_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const Cand keep = rc == GMRES_OK ? pick : saved;
  bt->loads = keep.loads;
  const int rc2 = apply_config(bt, keep.bs, keep.grid, keep.order, keep.part_rows);
  if (rc != GMRES_OK) return rc;
  if (rc2 != GMRES_OK) return rc2;
  if (ntrials) *ntrials = std::min(nt, max_trials);
  return GMRES_OK;
}

int gmres_batch_capture(gmres_batch* bt, const double* b, double* x, double rtol,
                        int64_t max_iters) {
  if (!bt || !is_device_ptr(b) || !is_device_ptr(x) || !(rtol >= 0.0) || max_iters < 0)
    return GMRES_ERR_ARG;
  if (!bt->stream) return GMRES_ERR_ARG;  // the legacy default stream cannot be captured
  drop_graph(bt);
  // the queue and the grid were set up by the last configuration call; the
  // capture records only the reset kernel and the persistent launch
  if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return GMRES_ERR_HIP;
  const int rc = enqueue(bt, b, x, rtol, max_iters, nullptr, nullptr, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(bt->stream, &g);
  if (rc != GMRES_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return GMRES_ERR_HIP;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return GMRES_ERR_HIP;
  }
  bt->graph = g;
  bt->graph_exec = ex;
  return GMRES_OK;
}

int gmres_batch_replay(gmres_batch* bt) {
  if (!bt || !bt->graph_exec) return GMRES_ERR_ARG;
  return hipGraphLaunch(bt->graph_exec, bt->stream) == hipSuccess ? GMRES_OK : GMRES_ERR_HIP;
}

}  // extern "C"

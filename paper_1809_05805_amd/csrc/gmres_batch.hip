// Host driver of the batched solver (the gmres_batch_* calls of gmres.h).
//
// Many independent systems, the diagonal blocks of one CSR matrix, are solved
// by restarted one-reduce GMRES(m) (the lagged compact-WY MGS step of
// Section III) in a single persistent launch: workgroups take systems from a
// device-side queue and run each system's whole solve. Everything a solve
// needs lives in the caller's workspace, laid out here once at create.
#include "gmres.h"
#include "gmres_internal.h"

#include <hip/hip_runtime.h>

#include <stddef.h>
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

struct BatchLayout {
  std::vector<BatchSys> sys;
  int64_t n;
  size_t o_sys, o_nat, o_lpt, o_st, o_queue, o_out, o_small, o_V, o_w, o_r64, o_xsave, total;
};

// Every system's basis starts 256-byte aligned with a leading dimension that
// is a multiple of 64 elements; the small dense arrays of all systems form
// one block of batch_small_doubles(m) doubles each.
bool batch_layout(int32_t nsys, const int64_t* row_off, int32_t m, int32_t scheme, BatchLayout* L) {
  if (nsys < 1 || !row_off || m < 1 || m > GMRES_MAX_RESTART) return false;
  if (scheme != GMRES_MGS_1R && scheme != GMRES_MGS_1R_IR32) return false;
  if (row_off[0] != 0) return false;
  const size_t vb = scheme == GMRES_MGS_1R_IR32 ? sizeof(float) : sizeof(double);
  const size_t small = batch_small_doubles(m);
  L->sys.resize((size_t)nsys);
  int64_t voff = 0;
  for (int32_t i = 0; i < nsys; ++i) {
    const int64_t n = row_off[i + 1] - row_off[i];
    if (n < 1 || n >= kMaxSysRows) return false;
    BatchSys& s = L->sys[(size_t)i];
    s.r0 = row_off[i];
    s.n = n;
    s.ldv = (int64_t)round_up((size_t)n, 64);
    s.voff = voff;
    s.soff = (int64_t)((size_t)i * small);
    voff += s.ldv * (m + 1);
  }
  L->n = row_off[nsys];
  if (L->n >= ((int64_t)1 << 31)) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = round_up(off + bytes, kAlign);
    return at;
  };
  L->o_sys = take(sizeof(BatchSys) * (size_t)nsys);
  L->o_nat = take(sizeof(int) * (size_t)nsys);
  L->o_lpt = take(sizeof(int) * (size_t)nsys);
  L->o_st = take(sizeof(DevState) * (size_t)nsys);
  L->o_queue = take(sizeof(unsigned));
  L->o_out = take(sizeof(BatchOut) * (size_t)nsys);
  L->o_small = take(sizeof(double) * small * (size_t)nsys);
  L->o_V = take(vb * (size_t)voff);
  L->o_w = take(vb * (size_t)L->n);
  L->o_r64 = scheme == GMRES_MGS_1R_IR32 ? take(sizeof(double) * (size_t)L->n) : 0;
  L->o_xsave = take(sizeof(double) * (size_t)L->n);
  L->total = off;
  return true;
}

}  // namespace

struct gmres_batch {
  Batch B;            // device view; b, x, rtol, max_iters, out and order set per solve
  int nsys, m, scheme;
  int64_t n;
  int bs, grid, order;  // grid 0: as many as the GPU holds
  int num_cu;
  const int* order_nat;
  const int* order_lpt;
  BatchOut* out_ws;
  double* xsave;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  std::vector<int64_t> sizes;
};

namespace {

int effective_grid(const gmres_batch* bt, int bs) {
  if (bt->grid > 0) return bt->grid;
  const int per_cu = batch_resident_blocks(bs, bt->m, bt->scheme == GMRES_MGS_1R_IR32);
  int64_t g = (int64_t)std::max(per_cu, 1) * bt->num_cu;
  if (g > bt->nsys) g = bt->nsys;
  return (int)std::max<int64_t>(g, 1);
}

int enqueue(gmres_batch* bt, const double* b, double* x, double rtol, int64_t max_iters,
            gmres_batch_info* info, hipEvent_t e0, hipEvent_t e1) {
  Batch B = bt->B;
  B.b = b;
  B.x = x;
  B.rtol = rtol;
  B.max_iters = max_iters;
  B.out = info ? reinterpret_cast<BatchOut*>(info) : bt->out_ws;
  B.order = bt->order == GMRES_BATCH_ORDER_NATURAL ? bt->order_nat : bt->order_lpt;
  if (launch_batch_reset(B, bt->stream)) return GMRES_ERR_HIP;
  if (launch_batch(B, bt->bs, effective_grid(bt, bt->bs), bt->scheme == GMRES_MGS_1R_IR32,
                   bt->stream, e0, e1))
    return GMRES_ERR_HIP;
  return GMRES_OK;
}

void drop_graph(gmres_batch* bt) {
  if (bt->graph_exec) (void)hipGraphExecDestroy(bt->graph_exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->graph_exec = nullptr;
  bt->graph = nullptr;
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
  B.nsys = nsys;
  B.m = m;
  B.Vb = base + L.o_V;
  B.wb = base + L.o_w;
  B.r64 = scheme == GMRES_MGS_1R_IR32 ? (double*)(base + L.o_r64) : nullptr;
  B.small = (double*)(base + L.o_small);
  B.st = (DevState*)(base + L.o_st);
  B.queue = (unsigned*)(base + L.o_queue);
  B.out = (BatchOut*)(base + L.o_out);
  bt->nsys = nsys;
  bt->m = m;
  bt->scheme = scheme;
  bt->n = L.n;
  bt->bs = 256;
  bt->grid = 0;
  bt->order = GMRES_BATCH_ORDER_LARGEST_FIRST;
  bt->num_cu = ncu;
  bt->order_nat = (const int*)(base + L.o_nat);
  bt->order_lpt = (const int*)(base + L.o_lpt);
  bt->out_ws = (BatchOut*)(base + L.o_out);
  bt->xsave = (double*)(base + L.o_xsave);
  bt->stream = (hipStream_t)hip_stream;
  bt->graph = nullptr;
  bt->graph_exec = nullptr;
  bt->sizes.resize((size_t)nsys);
  for (int i = 0; i < nsys; ++i) bt->sizes[(size_t)i] = L.sys[(size_t)i].n;

  // The two queue orders: as given, and by decreasing size (longest-processing-
  // time first; the size stands in for the unknown iteration count), ties by index.
  std::vector<int> nat((size_t)nsys), lpt((size_t)nsys);
  std::iota(nat.begin(), nat.end(), 0);
  lpt = nat;
  std::stable_sort(lpt.begin(), lpt.end(),
                   [&](int a, int b) { return L.sys[(size_t)a].n > L.sys[(size_t)b].n; });
  DevState st0;
  int rc = GMRES_OK;
  hipStream_t s = bt->stream;
  if (hipMemcpyAsync(base + L.o_sys, L.sys.data(), sizeof(BatchSys) * (size_t)nsys,
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(base + L.o_nat, nat.data(), sizeof(int) * (size_t)nsys, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemcpyAsync(base + L.o_lpt, lpt.data(), sizeof(int) * (size_t)nsys, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemsetAsync(B.st, 0, sizeof(DevState) * (size_t)nsys, s) != hipSuccess ||
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
  if (rc != GMRES_OK) {
    delete bt;
    return rc;
  }
  *out = bt;
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
  for (const auto& o : h)
    if (o.status) return GMRES_ERR_NONFINITE;
  return GMRES_OK;
}

int gmres_batch_set_config(gmres_batch* bt, int32_t block_size, int32_t grid, int32_t order) {
  if (!bt) return GMRES_ERR_ARG;
  if (block_size != 256 && block_size != 512 && block_size != 1024) return GMRES_ERR_ARG;
  if (grid < 0) return GMRES_ERR_ARG;
  if (order != GMRES_BATCH_ORDER_NATURAL && order != GMRES_BATCH_ORDER_LARGEST_FIRST)
    return GMRES_ERR_ARG;
  bt->bs = block_size;
  bt->grid = grid;
  bt->order = order;
  return GMRES_OK;
}

int gmres_batch_get_config(gmres_batch* bt, int32_t* block_size, int32_t* grid, int32_t* order) {
  if (!bt) return GMRES_ERR_ARG;
  if (block_size) *block_size = bt->bs;
  if (grid) *grid = effective_grid(bt, bt->bs);
  if (order) *order = bt->order;
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
  };
  std::vector<Cand> cands;
  for (int bs : {256, 512, 1024}) {
    const int per_cu = batch_resident_blocks(bs, bt->m, bt->scheme == GMRES_MGS_1R_IR32);
    if (per_cu < 1) continue;
    std::vector<int> grids = {std::min(bt->nsys, per_cu * bt->num_cu), std::min(bt->nsys, bt->num_cu)};
    if (grids[1] == grids[0]) grids.pop_back();
    for (int g : grids)
      for (int order : {GMRES_BATCH_ORDER_LARGEST_FIRST, GMRES_BATCH_ORDER_NATURAL})
        cands.push_back({bs, g, order});
  }
  if (cands.empty()) return GMRES_ERR_HIP;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GMRES_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GMRES_ERR_HIP;
  }
  const int save_bs = bt->bs, save_grid = bt->grid, save_order = bt->order;
  int rc = hipMemcpyAsync(bt->xsave, x, xb, hipMemcpyDeviceToDevice, s) == hipSuccess
               ? GMRES_OK
               : GMRES_ERR_HIP;
  float best = -1.0f;
  Cand pick = cands[0];
  int nt = 0;
  // one warm-up solve (code objects loaded, caches in a steady state), then each candidate once
  for (int t = -1; rc == GMRES_OK && t < (int)cands.size(); ++t) {
    const Cand c = cands[(size_t)(t < 0 ? 0 : t)];
    bt->bs = c.bs;
    bt->grid = c.grid;
    bt->order = c.order;
    if (hipMemcpyAsync(x, bt->xsave, xb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess) {
      rc = GMRES_ERR_HIP;
      break;
    }
    rc = enqueue(bt, b, x, rtol, max_iters, nullptr, nullptr, nullptr);
    float ms = 0.0f;
    if (rc == GMRES_OK &&
        (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = GMRES_ERR_HIP;
    if (rc != GMRES_OK || t < 0) continue;
    if (nt < max_trials) trials[nt] = gmres_batch_trial{c.bs, c.grid, c.order, ms};
    ++nt;
    if (best < 0.0f || ms < best) {
      best = ms;
      pick = c;
    }
  }
  if (rc == GMRES_OK &&
      (hipMemcpyAsync(x, bt->xsave, xb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    rc = GMRES_ERR_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != GMRES_OK) {
    bt->bs = save_bs;
    bt->grid = save_grid;
    bt->order = save_order;
    return rc;
  }
  bt->bs = pick.bs;
  bt->grid = pick.grid;
  bt->order = pick.order;
  if (ntrials) *ntrials = std::min(nt, max_trials);
  return GMRES_OK;
}

int gmres_batch_capture(gmres_batch* bt, const double* b, double* x, double rtol,
                        int64_t max_iters) {
  if (!bt || !is_device_ptr(b) || !is_device_ptr(x) || !(rtol >= 0.0) || max_iters < 0)
    return GMRES_ERR_ARG;
  if (!bt->stream) return GMRES_ERR_ARG;  // the legacy default stream cannot be captured
  drop_graph(bt);
  // the occupancy query behind the default grid is made before capture starts
  const int grid = effective_grid(bt, bt->bs);
  const int save_grid = bt->grid;
  bt->grid = grid;
  if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    bt->grid = save_grid;
    return GMRES_ERR_HIP;
  }
  const int rc = enqueue(bt, b, x, rtol, max_iters, nullptr, nullptr, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(bt->stream, &g);
  bt->grid = save_grid;
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

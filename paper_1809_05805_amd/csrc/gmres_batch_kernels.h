// Kernels and launchers of the batched persistent solver. Included once, by
// gmres_device.hip, after the device helpers they share with the
// single-system kernels (wavefront sums, column loads, the lagged small dense
// step, the device-coherent partial-sum accesses).
#pragma once

// ---------------------------------------------------- batched persistent solver
//
// A batch is a block-diagonal matrix: system i owns rows [r0, r0 + n) and its
// columns lie in the same range. One persistent kernel solves all of them.
// Its workgroups take entries from a device-side queue; an entry is a system,
// or one of the row parts of a larger system. A workgroup runs its entry's
// whole restarted one-reduce GMRES: where the single-system path has one
// device-wide reduction per step, a one-part system reduces within its
// workgroup, and a system of several parts (a team) adds its parts' sums
// through global memory with a team barrier. Every part then runs the small
// dense step itself on identical totals (so all parts take the same
// decisions, with no broadcast), and updates its own rows. Rows that other
// parts read (the SpMV's gathers across a part boundary, of the newest basis
// column and of x) are stored and gathered with device-coherent accesses;
// two team barriers per step order them.
//
// Queue order and team assembly: a system's parts are consecutive queue
// entries, and entries are taken in queue order, so at any time only the
// system whose parts were taken last can be waiting for a partner, and every
// earlier team is complete and finishes, freeing workgroups for the missing
// parts. The host keeps every team within what the GPU holds at once, so a
// team always assembles.

// Block-diagonal check: every column index of system i's rows lies in
// [r0, r0 + n). One thread per row; the system is found by bisection.
__global__ __launch_bounds__(256) void k_batch_validate(Csr A, const BatchSys* __restrict__ sys,
                                                         int nsys, DevState* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < A.n; r += stride) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sys[mid].r0 <= r) lo = mid; else hi = mid - 1;
    }
    const int64_t r0 = sys[lo].r0, r1 = r0 + sys[lo].n;
    bool bad = false;
    for (int e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      const int c = A.ci[e];
      if (c < r0 || c >= r1) bad = true;
    }
    if (bad) atomicOr(&st->bad_csr, 1);
  }
}

// Start of a batched solve: the queue position, the team barriers and every
// system's result.
__global__ void k_batch_reset(Batch B) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *B.queue = 0u;
  for (int i = t; i < B.nsys; i += gridDim.x * blockDim.x) {
    BatchOut o;
    o.iters = 0;
    o.cycles = o.converged = o.status = o.breakdown = 0;
    o.rel_res_true = 0.0;
    B.out[i] = o;
    B.bar[i] = 0u;
  }
}

// Device-coherent (agent-scope) loads and stores of basis and solution
// entries that another workgroup of the team reads or wrote.
template <typename T>
__device__ inline T coh_ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void coh_st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Entry i of a per-system array, addressed as a uniform base plus a 32-bit
// byte offset (a system has fewer than 2^28 rows, so the offset fits): one
// address register per lane instead of two.
template <typename T>
__device__ inline T& at(T* base, uint32_t i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ inline const T& at(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}

// One workgroup's view of its queue entry.
struct Team {
  unsigned* bar;     // the system's barrier counter
  double* rows;      // partial rows: slot base + p, 2 buffers of P doubles each
  unsigned target;   // barrier count this part waits for next
  int nparts, part, P, buf;
  bool failed;       // a wait ran out: the solve of this entry is abandoned
  uint32_t spins;    // polls a team barrier may take before it gives up
  int64_t lo, hi;    // own rows (local indices)
};

// All parts of the team have arrived: every store made before it by any
// part (completed, agent-scope where another part reads it) is visible.
// The counter is relaxed, not a release/acquire pair: visibility rests on each
// part's stores being acknowledged (s_waitcnt vmcnt(0)) before it arrives and
// on the agent-scope encoding, which keeps those accesses coherent across the
// XCDs' otherwise non-coherent L2 caches. Repeated solves of a whole batch
// with teams are tested to be bitwise equal.
// The wait is bounded by `spins` polls (short sleeps for the first 4096, then
// long ones; the default limit is at least about half a minute in all): a team
// that cannot assemble ends its solve with a failure instead of holding the
// GPU. Returns false (and sets failed, the same in every thread) when the wait
// ran out or failed was already set.
__device__ inline bool team_sync(Team& tm) {
  __shared__ int s_ok;
  if (tm.nparts == 1) {
    __syncthreads();
    return true;
  }
  if (tm.failed) return false;
  wait_stores();
  __syncthreads();
  tm.target += (unsigned)tm.nparts;
  if (threadIdx.x == 0) {
    atomicAdd(tm.bar, 1u);
    int ok = 1;
    for (uint32_t spin = 0;; ++spin) {
      if (__hip_atomic_load(tm.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tm.target) break;
      if (spin >= tm.spins) {
        ok = 0;
        break;
      }
      if (spin < 4096)
        __builtin_amdgcn_s_sleep(1);
      else
        __builtin_amdgcn_s_sleep(127);
    }
    s_ok = ok;
  }
  __syncthreads();
  const bool ok = s_ok != 0;
  __syncthreads();
  if (!ok) tm.failed = true;
  return ok;
}

// vals[0:cnt] = the team's totals of loc[0:cnt] (LDS), added over the parts
// in part order (loc is returned unchanged for a one-part team). The two
// buffers alternate, so a buffer is rewritten only after a later barrier
// that every part passes after reading it.
__device__ inline void team_reduce(Team& tm, const double* loc, double* vals, int cnt) {
  const int tid = threadIdx.x, bs = blockDim.x;
  if (tm.nparts == 1) {
    for (int c = tid; c < cnt; c += bs) vals[c] = loc[c];
    __syncthreads();
    return;
  }
  double* mine = tm.rows + ((size_t)tm.part * 2 + tm.buf) * tm.P;
  for (int c = tid; c < cnt; c += bs) atomic_st(&at(mine, (uint32_t)c), loc[c]);
  if (!team_sync(tm)) {
    for (int c = tid; c < cnt; c += bs) vals[c] = 0.0;
    __syncthreads();
    return;
  }
  // every part's row, added in part order; the loads of 8 parts are issued
  // together (one at a time, each would wait for its reply before the next)
  for (int c = tid; c < cnt; c += bs) {
    double a = 0.0;
    for (int q0 = 0; q0 < tm.nparts; q0 += 8) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int q = q0 + t < tm.nparts ? q0 + t : tm.nparts - 1;
        v[t] = atomic_ld(&at(tm.rows + ((size_t)q * 2 + tm.buf) * tm.P, (uint32_t)c));
      }
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (q0 + t < tm.nparts) a += v[t];
    }
    vals[c] = a;
  }
  tm.buf ^= 1;
  __syncthreads();
}

// The team total of one value per thread (loc: NW + 1 doubles of LDS).
template <int BS>
__device__ inline double team_sum(Team& tm, double v, double* loc) {
  v = wave_sum_last(v);
  if ((threadIdx.x & 63) == 63) loc[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < BS / 64; ++w) a += loc[w];
    loc[BS / 64] = a;
  }
  __syncthreads();
  double* tot = loc + BS / 64 + 1;
  team_reduce(tm, loc + BS / 64, tot, 1);
  const double t = tot[0];
  __syncthreads();
  return t;
}

// Row r (local) of A x for one system: rp is the system's first row pointer,
// r0 its first global row, x indexed locally. With COH, entries outside
// [lo, hi) (another part's rows) are gathered with coherent loads.
template <typename XT>
__device__ inline double batch_row(const int* __restrict__ rp, const int* __restrict__ ci,
                                   const double* __restrict__ va, int r0, uint32_t r,
                                   const XT* __restrict__ x, bool COH, uint32_t lo, uint32_t hi) {
  double a = 0.0;
  const int e1 = at(rp, r + 1);
  for (int e = at(rp, r); e < e1; ++e) {
    const uint32_t c = (uint32_t)(ci[e] - r0);
    XT v;
    if (COH && (c < lo || c >= hi))
      v = coh_ld(&at(x, c));
    else
      v = at(x, c);
    a = __builtin_fma(va[e], (double)v, a);
  }
  return a;
}

// The same row from the copy of the whole block-diagonal matrix by
// diagonals (64-row slices of global rows, which may straddle two systems):
// global row R = r0 + r lies in slice R / 64 at lane R % 64, and slice column
// j holds its entry on diagonal d_j (0 where it has none). The column r + d_j
// is clamped into the system's nloc rows, so a padding entry (value 0) never
// leaves them; the products are accumulated by fused multiply-adds in the
// diagonals' increasing order, which is the CSR order of a sorted row, so
// both forms give the same bits.
template <typename XT>
__device__ inline double batch_row_diag(const Sell& S, int64_t r0, uint32_t r, uint32_t nloc,
                                        const XT* __restrict__ x, bool COH, uint32_t lo,
                                        uint32_t hi) {
  const int64_t R = r0 + r;
  const int64_t sl = R >> 6;
  const int64_t b = S.sp[sl];
  const int W = (int)((S.sp[sl + 1] - b) >> 6);
  const double* __restrict__ va = S.va + b + (R & 63);
  const int* __restrict__ cb = S.cbase + (b >> 6);
  double a = 0.0;
  for (int j = 0; j < W; ++j) {
    uint32_t c = (uint32_t)((int)r + cb[j]);
    c = c < nloc ? c : nloc - 1;
    XT v;
    if (COH && (c < lo || c >= hi))
      v = coh_ld(&at(x, c));
    else
      v = at(x, c);
    a = __builtin_fma(va[(size_t)j * 64], (double)v, a);
  }
  return a;
}

template <typename T>
__device__ inline void put(bool coh, T* p, T v) {
  if (coh)
    coh_st(p, v);
  else
    *p = v;
}

// Restarts up to this m keep T in LDS with the rest of a cycle's small dense
// state; longer ones keep T in the system's global small workspace (T alone
// would outgrow the LDS).
constexpr int kBatchLdsTriMaxM = 128;

// LDS doubles of a cycle's small dense state for restart m: the rotations
// (cs, sn), the newest Hessenberg column and two scalars, and with T in LDS
// its strictly upper triangle.
constexpr size_t batch_state_lds_doubles(int m) {
  return 3 * (size_t)(m + 2) + 2 + (m <= kBatchLdsTriMaxM ? (size_t)m * (m + 1) / 2 : 0);
}

// A cycle's small dense state (in LDS; T in LDS or global memory).
struct BatchSml {
  double* cs;   // m + 2: the Givens rotations of the cycle so far
  double* sn;   // m + 2
  double* h;    // m + 2: the newest Hessenberg column h[0..k] (the MAXPY
                // coefficients), with rho below it once known
  double* sc;   // [0] the running residual entry g_k, [1] 1 / rho
  double* tri;  // T above its unit diagonal: T(q, i) at i (i - 1) / 2 + q, q < i
};

// The small dense step of lagged step k of the batched solver, with the
// cycle's state in LDS (T too, for m <= kBatchLdsTriMaxM), so that it makes no
// global round trip but T's for longer restarts:
//   thread 0: the lagged norm rho = ||u|| (Section II, the normalization lag),
//     which completes Hessenberg column k-1; that column's Givens rotation,
//     the update of g and the stopping test |g_k| <= tol (one step late,
//     Section III);
//   all: l = V[:,0:k]^T v_k = p / rho, r = [c / rho; gamma / rho^2], the new
//     column of T (T(q, k) = -(l_q + sum over q < j < k of T(q, j) l_j), so
//     that T = (I + L^T)^{-1}), and h = (I + L)^{-1} r: h[0:k] = r[0:k] +
//     (the earlier T)^T r[0:k] and h_k = r_k - l . h[0:k].
// Only R and g (read by the back substitution) and the state record go to
// memory besides. vals holds the step's totals: vals[2q] = V_q . u,
// vals[2q+1] = V_q . w (q < k), vals[2k] = u.u, vals[2k+1] = u.w; scr holds
// 3 (m + 2) doubles of scratch. Returns true, the same in every thread, when
// the cycle ends here.
__device__ bool batch_tail(const Ws& ws, const double* vals, double* scr, int k, bool norm_only,
                               double tol, const BatchSml& L) {
  __shared__ int s_go, s_bad;
  __shared__ double s_rho;
  const int tid = threadIdx.x, bs = blockDim.x;
  DevState* st = ws.st;
  if (tid == 0) {
    st->reductions += 1;
    const double alpha = vals[norm_only ? 0 : 2 * k];
    int go = 1;
    double rho = 0.0;
    if (!(alpha >= 0.0) || !isfinite(alpha)) {
      st->status = kNonfinite;
      st->done = 1;
      go = 0;
    } else {
      rho = sqrt(alpha);
      if (k == 0) {
        st->beta = rho;
        ws.g[0] = rho;
        L.sc[0] = rho;
        if (rho <= tol) {
          st->true_conv = 1;
          st->done = 1;
          st->j = 0;
          go = 0;
        }
      } else {
        // column k-1 = [h[0..k-1], rho]: the earlier rotations, then its own
        double* Rc = ws.R + (size_t)(k - 1) * ws.ldh;
        double a = L.h[0];
        for (int i = 0; i < k - 1; ++i) {
          const double b = L.h[i + 1], c = L.cs[i], s = L.sn[i];
          Rc[i] = c * a + s * b;
          a = -s * a + c * b;
        }
        double c, s;
        rot_make(a, rho, &c, &s);
        Rc[k - 1] = c * a + s * rho;
        Rc[k] = 0.0;
        L.cs[k - 1] = c;
        L.sn[k - 1] = s;
        const double g = L.sc[0];
        const double gn = -s * g;
        ws.g[k - 1] = c * g;
        ws.g[k] = gn;
        L.sc[0] = gn;
        const double res = fabs(gn);
        if (!isfinite(res)) {
          st->status = kNonfinite;
          st->done = 1;
          go = 0;
        } else if (rho == 0.0) {
          st->breakdown = 1;
          st->done = 1;
          st->j = k;
          go = 0;
        } else if (res <= tol || norm_only) {
          st->done = 1;
          st->j = k;
          go = 0;
        }
      }
      if (go) {
        st->rho = rho;
        L.sc[1] = 1.0 / rho;
      }
    }
    s_rho = rho;
    s_go = go;
    s_bad = 0;
  }
  __syncthreads();
  if (!s_go) return true;
  const double rho = s_rho;
  const int M2 = ws.m + 2;
  double* ell = scr;
  double* rr = scr + M2;
  double* hb = scr + 2 * M2;
  for (int q = tid; q < k; q += bs) {
    ell[q] = vals[2 * q] / rho;
    rr[q] = vals[2 * q + 1] / rho;
  }
  if (tid == 0) rr[k] = (vals[2 * k + 1] / rho) / rho;
  __syncthreads();
  // column k of T (T's earlier columns only are read), and hb = T^T r over them
  double* tk = L.tri + (size_t)k * (k - 1) / 2;
  for (int q = tid; q < k; q += bs) {
    double a = ell[q];
    for (int j = q + 1; j < k; ++j) a += L.tri[(size_t)j * (j - 1) / 2 + q] * ell[j];
    tk[q] = -a;
  }
  tri_dots(L.tri, rr, k, hb);
  __syncthreads();
  for (int i = tid; i < k; i += bs) {
    const double h = rr[i] + hb[i];
    L.h[i] = h;
    if (!isfinite(h)) s_bad = 1;
  }
  if (tid < 64) {
    double a = 0.0;
    for (int q = tid; q < k; q += 64) a += ell[q] * (rr[q] + hb[q]);
    a = wave_sum(a);
    if (tid == 0) {
      const double hk = rr[k] - a;
      L.h[k] = hk;
      if (!isfinite(hk)) s_bad = 1;
    }
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) {
      st->status = kNonfinite;
      st->done = 1;
    }
    return true;
  }
  return false;
}

// The solve of one queue entry (a system, or one part of a team) by one
// workgroup of BS threads. Team and ticket values are uniform.
// LT: T is kept in LDS (m <= kBatchLdsTriMaxM), else in global memory.
// NT: the projection and MAXPY load basis columns non-temporal (streamed).
template <int BS, typename VT, bool LT, bool NT>
__device__ void batch_part(const Batch& B, const BatchTicket K, double* red, double* vals,
                           double* scr, double* sml) {
  constexpr int NW = BS / 64;
  // rows per thread per row block (fewer for 1024 threads, which have 128
  // registers per lane)
  constexpr int RB = BS >= 1024 ? 4 : 8;
  constexpr bool F32 = sizeof(VT) == 4;
  using BasisCol = std::conditional_t<NT, GlbColNT<VT>, GlbCol<VT>>;
  __shared__ int s_flag[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = B.m;
  const int P = 2 * (m + 2);
  const BatchSys S = B.sys[K.sys];
  const int64_t n = S.n, r0 = S.r0;
  const int slot = K.base + K.part;
  Team tm;
  tm.bar = B.bar + K.sys;
  tm.rows = B.partials + (size_t)K.base * 2 * P;
  tm.target = 0;
  tm.nparts = K.nparts;
  tm.part = K.part;
  tm.P = P;
  tm.buf = 0;
  tm.failed = false;
  tm.spins = B.spin_limit;
  {
    const int64_t per = (n + K.nparts - 1) / K.nparts;
    const int64_t chunk = (per + 63) / 64 * 64;
    tm.lo = chunk * K.part < n ? chunk * K.part : n;
    tm.hi = tm.lo + chunk < n ? tm.lo + chunk : n;
  }
  const uint32_t lo = (uint32_t)tm.lo, hi = (uint32_t)tm.hi;
  // coherent gathers across part boundaries and coherent stores of what
  // other parts gather: only in a real team
  const bool coh = K.nparts > 1;
  const bool cst = coh;
  Ws ws{};
  {
    double* sm = B.small + (size_t)slot * batch_small_doubles(m);
    if constexpr (F32) {
      ws.Vf = (float*)B.Vb + S.voff;
      ws.wf = (float*)B.wb + r0;
      ws.r64 = B.r64 + r0;
    } else {
      ws.V = (double*)B.Vb + S.voff;
      ws.w = (double*)B.wb + r0;
    }
    ws.H = sm;
    ws.R = ws.H + (size_t)(m + 1) * m;
    ws.T = ws.R + (size_t)(m + 1) * m;
    ws.TT = ws.T + (size_t)(m + 2) * (m + 2);
    ws.g = ws.TT + (size_t)(m + 2) * (m + 2);
    ws.gh = ws.g + (m + 2);
    ws.cs = ws.gh + (m + 2);
    ws.sn = ws.cs + (m + 2);
    ws.coef = ws.sn + (m + 2);
    ws.coef2 = ws.coef + (m + 2);
    ws.y = ws.coef2 + (m + 2);
    ws.st = B.st + slot;
    ws.n = n;
    ws.ldv = S.ldv;
    ws.ldh = m + 1;
    ws.ldt = m + 2;
    ws.m = m;
  }
  DevState* st = ws.st;
  BatchSml L;
  L.cs = sml;
  L.sn = L.cs + (m + 2);
  L.h = L.sn + (m + 2);
  L.sc = L.h + (m + 2);
  L.tri = LT ? L.sc + 2 : ws.T;
  VT* __restrict__ V = basis_of<VT>(ws);
  VT* __restrict__ wv_ = wbuf_of<VT>(ws);
  const int64_t ldv = ws.ldv;
  const double* __restrict__ b = B.b + r0;
  double* __restrict__ x = B.x + r0;
  const int nblk = (int)((hi - lo + BS * RB - 1) / (BS * RB));
  const int* __restrict__ rp_s = B.A.rp + r0;
  // row r of this system's A times x (x indexed locally)
  const bool diag = B.S.va != nullptr;
  auto row = [&](uint32_t r, const auto* __restrict__ xx) {
    return diag ? batch_row_diag(B.S, r0, r, (uint32_t)n, xx, coh, lo, hi)
                : batch_row(rp_s, B.A.ci, B.A.va, (int)r0, r, xx, coh, lo, hi);
  };
  double* loc = vals + P;  // team_sum's LDS (NW + 2 doubles after vals)

  // ||b|| and the tolerance
  double sb = 0.0;
  for (uint32_t r = lo + tid; r < hi; r += BS) sb += at(b, r) * at(b, r);
  const double bnorm = sqrt(team_sum<BS>(tm, sb, loc));
  if (tid == 0) {
    st->done = st->j = st->true_conv = st->breakdown = st->status = 0;
    st->reductions = 1;
    st->bnorm = bnorm;
    st->tol_abs = B.rtol * bnorm;
    st->tol_cycle = st->tol_abs;
    st->xscale = 1.0;
  }
  __syncthreads();
  BatchOut out;
  out.iters = 0;
  out.cycles = out.converged = out.status = out.breakdown = 0;
  out.rel_res_true = 0.0;
  if (tm.failed) {
    out.status = kTeamStall;
  } else if (!isfinite(bnorm)) {
    out.status = kNonfinite;
  } else if (bnorm == 0.0) {
    for (uint32_t r = lo + tid; r < hi; r += BS) at(x, r) = 0.0;
    out.converged = 1;
  } else {
    const double tol_abs = B.rtol * bnorm;
    int64_t it = 0;
    for (;;) {
      // x of the previous cycle is complete on every part before it is gathered
      if (!team_sync(tm)) break;
      const int64_t left = B.max_iters - it;
      const int m_eff = left < (int64_t)m ? (int)left : m;
      if (m_eff == 0) {
        // the iteration budget is spent: the true residual of the final x
        double sr = 0.0;
        for (uint32_t r = lo + tid; r < hi; r += BS) {
          const double d = at(b, r) - row(r, x);
          sr += d * d;
        }
        const double rn = sqrt(team_sum<BS>(tm, sr, loc));
        if (tm.failed) break;
        out.rel_res_true = rn / bnorm;
        out.converged = rn <= tol_abs;
        if (!isfinite(rn)) out.status = kNonfinite;
        break;
      }
      // cycle start: clear the small dense matrices and the flags
      {
        const size_t tot = 2 * (size_t)(m + 1) * m + 2 * (size_t)(m + 2) * (m + 2) + 2 * (size_t)(m + 2);
        for (uint32_t e = tid; e < tot; e += BS) at(ws.H, e) = 0.0;  // H, R, T, TT, g, gh are contiguous
        if (tid == 0) {
          st->done = st->j = st->true_conv = st->breakdown = 0;
          st->xscale = 1.0;
          st->tol_cycle = tol_abs;
        }
      }
      __syncthreads();
      // restart residual
      double beta_cycle = 0.0;
      if constexpr (F32) {
        double sr = 0.0;
        for (uint32_t r = lo + tid; r < hi; r += BS) {
          const double d = at(b, r) - row(r, x);
          at(ws.r64, r) = d;
          sr += d * d;
        }
        const double beta = sqrt(team_sum<BS>(tm, sr, loc));
        if (tm.failed) break;
        if (!isfinite(beta)) {
          out.status = kNonfinite;
          break;
        }
        if (beta <= tol_abs) {
          out.converged = 1;
          out.rel_res_true = beta / bnorm;
          break;
        }
        const double inv = 1.0 / beta;
        for (uint32_t r = lo + tid; r < hi; r += BS) put(cst, &at(V, r), (VT)(at(ws.r64, r) * inv));
        // the float64 check above is the restart test: the normalized float32
        // start vector is not tested again (tol_cycle 0 for step 0)
        if (tid == 0) {
          st->reductions += 1;
          st->tol_cycle = 0.0;
          st->xscale = beta;
        }
        beta_cycle = beta;
      } else {
        for (uint32_t r = lo + tid; r < hi; r += BS) put(cst, &at(V, r), (VT)(at(b, r) - row(r, x)));
      }
      for (int k = 0; k <= m_eff; ++k) {
        // column k is complete on every part before the SpMV gathers it
        if (!team_sync(tm)) break;
        const bool last = k == m_eff;
        const int nproj = last ? 0 : k;
        const int cnt = 2 * (nproj + 1);
        for (int c = lane; c < cnt; c += 64) red[wv * P + c] = 0.0;
        const VT* __restrict__ u_g = V + (size_t)k * ldv;
        for (int blk = 0; blk < nblk; ++blk) {
          // this thread's rows of the block: clamped loads, masked values
          VT u[RB], w[RB];
          uint32_t off[RB];
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            const uint32_t r = lo + (uint32_t)(blk * BS * RB + t * BS + tid);
            const bool ok = r < hi;
            const uint32_t rc = ok ? r : hi - 1;
            off[t] = rc * (uint32_t)sizeof(VT);
            u[t] = ok ? at(u_g, rc) : (VT)0;
            if (!last) {
              const double a = ok ? row(rc, u_g) : 0.0;
              w[t] = (VT)a;
              if (ok) at(wv_, r) = w[t];
            } else {
              w[t] = (VT)0;
            }
          }
          // projection over columns 0..nproj-1, the next column's loads in flight
          auto load_col = [&](VT (&buf)[RB], int j) {
            const BasisCol col(V + (size_t)j * ldv, n);
#pragma unroll
            for (int t = 0; t < RB; ++t) buf[t] = col(off[t]);
          };
          auto reduce_col = [&](const VT (&vv)[RB], int j) {
            VT p = (VT)0, q = (VT)0;
#pragma unroll
            for (int t = 0; t < RB; ++t) {
              p += vv[t] * u[t];
              q += vv[t] * w[t];
            }
            const double ps = wave_sum_last((double)p);
            const double qs = wave_sum_last((double)q);
            if (lane == 63) {
              red[wv * P + 2 * j] += ps;
              red[wv * P + 2 * j + 1] += qs;
            }
          };
          if (nproj > 0) {
            VT ba[RB], bb[RB];
            load_col(ba, 0);
            int j = 0;
            for (;;) {
              load_col(bb, j + 1 < nproj ? j + 1 : j);
              reduce_col(ba, j);
              if (++j >= nproj) break;
              load_col(ba, j + 1 < nproj ? j + 1 : j);
              reduce_col(bb, j);
              if (++j >= nproj) break;
            }
          }
          VT al = (VT)0, ga = (VT)0;
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            al += u[t] * u[t];
            ga += u[t] * w[t];
          }
          const double als = wave_sum_last((double)al);
          const double gas = wave_sum_last((double)ga);
          if (lane == 63) {
            red[wv * P + 2 * nproj] += als;
            red[wv * P + 2 * nproj + 1] += gas;
          }
        }
        __syncthreads();
        // the workgroup's sums (in scr), then the team's totals in vals
        for (int c = tid; c < cnt; c += BS) {
          double a = 0.0;
          for (int w2 = 0; w2 < NW; ++w2) a += red[w2 * P + c];
          scr[c] = a;
        }
        __syncthreads();
        team_reduce(tm, scr, vals, cnt);
        if (tm.failed) break;
        // the small dense step (H column, T column, Givens, flags, MAXPY
        // coefficients), run by every part on the same totals
        // the small dense step (Givens, T column, flags, the MAXPY
        // coefficients h[0..k] into L.h), run by every part on the same totals
        const double tol_k = F32 ? (k == 0 ? 0.0 : tol_abs / beta_cycle) : tol_abs;
        if (batch_tail(ws, vals, scr, k, last, tol_k, L)) break;
        const double* cl = L.h;
        const VT invr = (VT)L.sc[1];
        // MAXPY: V[:,k] = u / rho, V[:,k+1] = w / rho - V[:,0:k+1] h
        VT* __restrict__ vk_g = V + (size_t)k * ldv;
        VT* __restrict__ vn_g = vk_g + ldv;
        for (int blk = 0; blk < nblk; ++blk) {
          VT acc[RB], vk[RB];
          uint32_t off[RB];
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            const uint32_t r = lo + (uint32_t)(blk * BS * RB + t * BS + tid);
            const uint32_t rc = r < hi ? r : hi - 1;
            off[t] = rc * (uint32_t)sizeof(VT);
            acc[t] = at(wv_, rc) * invr;
            vk[t] = at(vk_g, rc) * invr;
          }
          auto load_col = [&](VT (&buf)[RB], int j) {
            const BasisCol col(V + (size_t)j * ldv, n);
#pragma unroll
            for (int t = 0; t < RB; ++t) buf[t] = col(off[t]);
          };
          auto axpy_col = [&](const VT (&vv)[RB], int j) {
            const VT c = (VT)cl[j];
#pragma unroll
            for (int t = 0; t < RB; ++t) acc[t] -= vv[t] * c;
          };
          if (k > 0) {
            VT ba[RB], bb[RB];
            load_col(ba, 0);
            int j = 0;
            for (;;) {
              load_col(bb, j + 1 < k ? j + 1 : j);
              axpy_col(ba, j);
              if (++j >= k) break;
              load_col(ba, j + 1 < k ? j + 1 : j);
              axpy_col(bb, j);
              if (++j >= k) break;
            }
          }
          const VT ck = (VT)cl[k];
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            const uint32_t r = lo + (uint32_t)(blk * BS * RB + t * BS + tid);
            if (r < hi) {
              at(vk_g, r) = vk[t];
              put(cst, &at(vn_g, r), acc[t] - vk[t] * ck);
            }
          }
        }
      }
      if (tm.failed) break;
      if (tid == 0) {
        s_flag[1] = st->j;
        s_flag[2] = st->status;
        s_flag[3] = st->true_conv | (st->breakdown << 1);
      }
      __syncthreads();
      const int j = s_flag[1];
      if (s_flag[2]) {
        out.status = s_flag[2];
        break;
      }
      if (s_flag[3] & 1) {
        // the restart check of this cycle's first step passed (float64 schemes)
        out.converged = 1;
        out.rel_res_true = st->beta / bnorm;
        break;
      }
      if (s_flag[3] & 2) out.breakdown = 1;
      // back substitution R y = g, then x += xscale V y on the own rows
      double* yl = scr;
      if (tid == 0) {
        const double xs = st->xscale;
        for (int q = j - 1; q >= 0; --q) {
          double a = ws.g[q];
          for (int t = q + 1; t < j; ++t) a -= ws.R[(size_t)t * ws.ldh + q] * ws.y[t];
          const double piv = ws.R[(size_t)q * ws.ldh + q];
          const double yq = piv != 0.0 ? a / piv : 0.0;
          ws.y[q] = yq;
          yl[q] = xs * yq;
        }
      }
      __syncthreads();
      for (uint32_t r = lo + tid; r < hi; r += BS) {
        double a = at(x, r);
        for (int q = 0; q < j; ++q) a += (double)at(V + (size_t)q * ldv, r) * yl[q];
        put(cst, &at(x, r), a);
      }
      __syncthreads();
      it += j;
      out.cycles += 1;
      if (j == 0) break;
    }
    out.iters = it;
    if (tm.failed) out.status = kTeamStall;
  }
  if (tid == 0 && K.part == 0) {
    if (out.status == 0 && st->status) out.status = st->status;
    B.out[K.sys] = out;
  }
  __syncthreads();
}

template <int BS, typename VT, bool LT, bool NT>
__global__ __launch_bounds__(BS) void k_batch(Batch B) {
  extern __shared__ double lds[];
  __shared__ int s_pos;
  constexpr int NW = BS / 64;
  const int P = 2 * (B.m + 2);
  double* red = lds;              // NW x P per-wavefront sums
  double* vals = red + NW * P;    // P totals, then team_sum's NW + 2
  double* scr = vals + P + NW + 2; // 6 (m + 2) for the small dense step
  double* sml = scr + 6 * (B.m + 2);  // batch_state_lds_doubles(m)
  for (;;) {
    if (threadIdx.x == 0) s_pos = (int)atomicAdd(B.queue, 1u);
    __syncthreads();
    const int pos = __builtin_amdgcn_readfirstlane(s_pos);
    __syncthreads();
    if (pos >= B.ntickets) break;
    BatchTicket K = B.tickets[pos];
    K.sys = __builtin_amdgcn_readfirstlane(K.sys);
    K.part = __builtin_amdgcn_readfirstlane(K.part);
    K.nparts = __builtin_amdgcn_readfirstlane(K.nparts);
    K.base = __builtin_amdgcn_readfirstlane(K.base);
    batch_part<BS, VT, LT, NT>(B, K, red, vals, scr, sml);
  }
}

size_t batch_lds_bytes(int bs, int m) {
  const size_t P = 2 * (size_t)(m + 2);
  return ((size_t)(bs / 64) * P + P + (size_t)(bs / 64) + 2 + 6 * (size_t)(m + 2) +
          batch_state_lds_doubles(m)) *
         sizeof(double);
}

int launch_batch_validate(const Csr& A, const BatchSys* sys, int nsys, DevState* st, hipStream_t s) {
  int64_t blocks = (A.n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_batch_validate, dim3((unsigned)blocks), dim3(256), 0, s, A, sys, nsys, st);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_batch_reset(const Batch& B, hipStream_t s) {
  const int blocks = (B.nsys + 255) / 256;
  hipLaunchKernelGGL(k_batch_reset, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, B);
  GMRES_CHECK_LAUNCH();
  return 0;
}

template <int BS, typename VT, bool LT, bool NT>
void batch_launch_one(const Batch& B, int grid, uint32_t lds, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1) {
  if (e0 || e1)
    hipExtLaunchKernelGGL((k_batch<BS, VT, LT, NT>), dim3(grid), dim3(BS), lds, s, e0, e1, 0u, B);
  else
    hipLaunchKernelGGL((k_batch<BS, VT, LT, NT>), dim3(grid), dim3(BS), lds, s, B);
}

template <int BS, typename VT, bool LT>
void batch_launch_nt(const Batch& B, bool nt, int grid, uint32_t lds, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  nt ? batch_launch_one<BS, VT, LT, true>(B, grid, lds, s, e0, e1)
     : batch_launch_one<BS, VT, LT, false>(B, grid, lds, s, e0, e1);
}

template <int BS>
void batch_launch_bs(const Batch& B, bool f32, bool nt, int grid, uint32_t lds, hipStream_t s,
                     hipEvent_t e0, hipEvent_t e1) {
  const bool lt = B.m <= kBatchLdsTriMaxM;
  if (f32)
    lt ? batch_launch_nt<BS, float, true>(B, nt, grid, lds, s, e0, e1)
       : batch_launch_nt<BS, float, false>(B, nt, grid, lds, s, e0, e1);
  else
    lt ? batch_launch_nt<BS, double, true>(B, nt, grid, lds, s, e0, e1)
       : batch_launch_nt<BS, double, false>(B, nt, grid, lds, s, e0, e1);
}

int launch_batch(const Batch& B, int bs, int grid, bool f32, bool nt, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1) {
  if (grid < 1) return -1;
  const uint32_t lds = (uint32_t)batch_lds_bytes(bs, B.m);
  switch (bs) {
    case 256:
      batch_launch_bs<256>(B, f32, nt, grid, lds, s, e0, e1);
      break;
    case 512:
      batch_launch_bs<512>(B, f32, nt, grid, lds, s, e0, e1);
      break;
    case 1024:
      batch_launch_bs<1024>(B, f32, nt, grid, lds, s, e0, e1);
      break;
    default:
      return -1;
  }
  GMRES_CHECK_LAUNCH();
  return 0;
}

template <int BS, typename VT, bool LT>
hipError_t batch_occupancy_nt(int* nb, bool nt, size_t lds) {
  return nt ? hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_batch<BS, VT, LT, true>, BS, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_batch<BS, VT, LT, false>, BS, lds);
}

template <int BS>
hipError_t batch_occupancy(int* nb, int m, bool f32, bool nt, size_t lds) {
  const bool lt = m <= kBatchLdsTriMaxM;
  if (f32)
    return lt ? batch_occupancy_nt<BS, float, true>(nb, nt, lds)
              : batch_occupancy_nt<BS, float, false>(nb, nt, lds);
  return lt ? batch_occupancy_nt<BS, double, true>(nb, nt, lds)
            : batch_occupancy_nt<BS, double, false>(nb, nt, lds);
}

int batch_resident_blocks(int bs, int m, bool f32, bool nt) {
  const size_t lds = batch_lds_bytes(bs, m);
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (bs) {
    case 256:
      e = batch_occupancy<256>(&nb, m, f32, nt, lds);
      break;
    case 512:
      e = batch_occupancy<512>(&nb, m, f32, nt, lds);
      break;
    case 1024:
      e = batch_occupancy<1024>(&nb, m, f32, nt, lds);
      break;
    default:
      break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

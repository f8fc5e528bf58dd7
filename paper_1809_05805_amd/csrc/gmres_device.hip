// HIP kernels for restarted GMRES(m) on gfx950 (FP64), after Swirydowicz,
// Langou, Ananthan, Yang, Thomas, "Low synchronization GMRES algorithms"
// (arXiv:1809.05805).
//
// The Arnoldi step of the one-reduce scheme (Section II, level-2 MGS with R
// normalization lag; Section III, one-synchronization MGS-GMRES) runs as two
// launches:
//   k_fused  - CSR SpMV w = A u of the unnormalized newest column u = V[:,k],
//              the tall-skinny projection [V[:,0:k+1]^T u, V[:,0:k+1]^T w], one
//              device-wide reduction (two-level ticket reduction in a fixed
//              order, so results are bitwise reproducible) and, in the last
//              workgroup to finish, the part of the small dense step that the
//              MAXPY needs: lagged norm and h = (I + L)^{-1} r;
//   k_maxpy  - V[:,k] = u / rho and V[:,k+1] = w / rho - V[:,0:k+1] h, with
//              one extra workgroup for the rest of the small dense step: the
//              new column of T, and the Givens rotations and stopping test
//              for the finished Hessenberg columns, every step or every L
//              steps (Section III, the depth-L pipeline).
// The level-1 MGS and two-reduce CGS2 baselines reuse the same building
// blocks. Everything is memory-bound BLAS-2 work: no matrix cores.
#include "gmres_internal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>

#include <type_traits>

namespace gmres {

// ---------------------------------------------------------------- helpers

// Workgroup tile -> rows. Workgroups are handed to the 8 XCDs round-robin by
// blockIdx.x; when the grid is a multiple of 8, consecutive tiles are given to
// workgroups of the same XCD so that the SpMV's neighbour gathers stay in one
// XCD's L2.
__device__ inline int tile_of_block(int G) {
  const int b = blockIdx.x;
  if ((G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
  return b;
}

__device__ inline double atomic_ld(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void atomic_st(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of v over the 64 lanes of a wavefront, returned in every lane.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce NV values per lane over the wavefront with a halving butterfly:
// log2(NV) exchange steps each move half of the remaining values, then
// 6 - log2(NV) full steps. Lane l ends holding in v[0] the total of value
// index (l >> (6 - log2 NV)); that costs NV - 1 + 6 - log2(NV) shuffles
// instead of 6 NV.
template <int NV>
__device__ inline double wave_multi_sum(double (&v)[NV], int lane) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two");
  int mask = 32;
#pragma unroll
  for (int h = NV / 2; h >= 1; h >>= 1) {
    const bool upper = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      // plain values first: a select between array elements can become a
      // select of addresses, which puts the array in scratch memory
      const double a = v[i], b = v[i + h];
      const double send = upper ? a : b;
      const double keep = upper ? b : a;
      v[i] = keep + __shfl_xor(send, mask, 64);
    }
    mask >>= 1;
  }
  for (; mask >= 1; mask >>= 1) v[0] += __shfl_xor(v[0], mask, 64);
  return v[0];
}

// One data-parallel-primitive (DPP) move of a double: the two 32-bit halves
// go through the same lane permutation CTRL; lanes with no source (or in rows
// outside ROWMASK) receive 0.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWMASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWMASK, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wavefront, valid in lane 63 only: shifts by 1,
// 2, 4 and 8 lanes within each row of 16 leave the row's total in its last
// lane, then row_bcast:15 adds row 0 into row 1 and row 2 into row 3, and
// row_bcast:31 adds rows 0-1 into rows 2-3. All moves are VALU cross-lane
// operations, with no trip through the LDS unit.
__device__ inline double wave_sum_last(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Tuning constants (compile-time; defaults are the measured best on MI355X):
//   GMRES_PROJ_COLS  basis columns per projection chunk (1, 2, 4 or 8).
#ifndef GMRES_PROJ_COLS
#define GMRES_PROJ_COLS 1
#endif
//   GMRES_PROJ_REVERSE  1: the projection streams the basis columns last to
//                       first, so it starts on the columns the previous MAXPY
//                       read last and ends on those the next MAXPY reads
//                       first (both still in the last-level cache); 0: first
//                       to last. Each column's sums are separate, so the order
//                       changes no result.
#ifndef GMRES_PROJ_REVERSE
#define GMRES_PROJ_REVERSE 1
#endif
//   GMRES_NT_STORES  bit 0: the fused step's SpMV output w, bit 1: the two
//                    columns MAXPY writes, are stored non-temporally, so they
//                    neither displace basis columns from the caches nor leave
//                    dirty lines for the write-back at the end of the kernel;
//                    bits 2 and 3: the same for bfloat16 columns.
#ifndef GMRES_NT_STORES
#define GMRES_NT_STORES 15
#endif
//   GMRES_XUPDATE_REVERSE  1: the end-of-cycle x update takes the basis
//                          columns last to first (see k_xupdate).
#ifndef GMRES_XUPDATE_REVERSE
#define GMRES_XUPDATE_REVERSE 1
#endif
template <int BIT, typename T>
__device__ inline void st_stream(T* p, T v) {
  if constexpr (sizeof(T) >= 4 && (GMRES_NT_STORES & BIT) != 0)
    __builtin_nontemporal_store(v, p);
  else if constexpr (sizeof(T) == 2 && (GMRES_NT_STORES & (BIT << 2)) != 0)
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v),
                                reinterpret_cast<unsigned short*>(p));
  else
    *p = v;
}

//   GMRES_SELL_CPOL  cache policy bits of the sliced copy's index and value
//                    loads (0: default; 2: non-temporal, so streaming A does
//                    not evict basis columns from the last-level cache).
#ifndef GMRES_SELL_CPOL
#define GMRES_SELL_CPOL 2
#endif
//   GMRES_SPMV_PIPELINE  1: the fused kernel's SpMV prefetches the next pass (spmv_tile);
//                        0: passes run one after another (spmv_pass).
#ifndef GMRES_SPMV_PIPELINE
#define GMRES_SPMV_PIPELINE 1
#endif
//   GMRES_DPP_REDUCE  1: the projection's wavefront sums use DPP row shifts
//                     and broadcasts; 0: a halving butterfly of lane shuffles.
#ifndef GMRES_DPP_REDUCE
#define GMRES_DPP_REDUCE 1
#endif
//   GMRES_FUSED_ROWMAP  rows of a lane in the fused step (see k_fused).
#ifndef GMRES_FUSED_ROWMAP
#define GMRES_FUSED_ROWMAP 1
#endif
//   GMRES_MAXPY_COLS  basis columns per MAXPY pass (1, 2 or 4).
#ifndef GMRES_MAXPY_COLS
#define GMRES_MAXPY_COLS 2
#endif

// Load base[boff / 8] with boff an unsigned 32-bit byte offset: with a
// wave-uniform base this is the scalar-base + 32-bit vector-offset form of a
// global load, so one offset register per lane serves every column of a tile
// (a signed or 64-bit index costs a 64-bit address per load instead).
__device__ inline double ld_at(const double* base, uint32_t boff) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + boff);
}

// A raw buffer resource over elements [0, nelem) of a wave-uniform array of T
// (double or float): its descriptor sits in scalar registers, so a load needs
// only the lane's 32-bit byte offset; offsets at or past the end read 0
// instead of memory. The third descriptor word is the gfx9-family raw-buffer
// format (32-bit data, no swizzle).
template <typename T>
struct BufCol {
  __amdgpu_buffer_rsrc_t r;
  __device__ BufCol(const T* base, int64_t nelem) {
    const int64_t nb = nelem * (int64_t)sizeof(T);
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                          (int)(nb < 0x7ffffff8 ? nb : 0x7ffffff8), 0x00020000);
  }
  template <int CPOL = 0>
  __device__ T load(uint32_t boff) const {
    if constexpr (sizeof(T) == 8)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)boff, 0, CPOL));
    else if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, CPOL));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)boff, 0, CPOL));
  }
  __device__ T operator()(uint32_t boff) const { return load<0>(boff); }
};

// The same interface over a plain global load (scalar base + 32-bit offset);
// callers keep their offsets inside [0, sizeof(T) nelem).
template <typename T>
struct GlbCol {
  const T* b;
  __device__ GlbCol(const T* base, int64_t) : b(base) {}
  __device__ T operator()(uint32_t boff) const {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(b) + boff);
  }
};

// The same with non-temporal loads (streamed, not kept in the caches).
template <typename T>
struct GlbColNT {
  const T* b;
  __device__ GlbColNT(const T* base, int64_t) : b(base) {}
  __device__ T operator()(uint32_t boff) const {
    const char* p = reinterpret_cast<const char*>(b) + boff;
    if constexpr (sizeof(T) == 8)
      return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(p)));
    else if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p)));
    else
      return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p)));
  }
};

//   GMRES_PROJ_BUFFER / GMRES_MAXPY_BUFFER  1: the projection's (MAXPY's and
//   x update's) column loads are buffer loads; 0: global loads.
#ifndef GMRES_PROJ_BUFFER
#define GMRES_PROJ_BUFFER 0
#endif
#ifndef GMRES_MAXPY_BUFFER
#define GMRES_MAXPY_BUFFER 0
#endif
template <typename T>
using ProjCol = std::conditional_t<GMRES_PROJ_BUFFER != 0, BufCol<T>, GlbCol<T>>;
template <typename T>
using MaxpyCol = std::conditional_t<GMRES_MAXPY_BUFFER != 0, BufCol<T>, GlbCol<T>>;

// Basis element types: float64, float32, and bfloat16 (storage only). The
// arithmetic type of a basis type: its own, and float32 for bfloat16. The
// sliced copy's value type: float64 for the float64 basis, float32 otherwise.
template <typename VT>
struct ArithOf {
  using type = VT;
};
template <>
struct ArithOf<__bf16> {
  using type = float;
};
template <typename VT>
using arith_t = typename ArithOf<VT>::type;
template <typename VT>
using sval_t = std::conditional_t<sizeof(VT) == 8, double, float>;

// The basis and SpMV-output arrays of the workspace in the basis type (the
// reduced-precision bases share the float32 pointers; the workspace layout
// sizes them by element size).
template <typename VT>
__device__ __host__ inline VT* basis_of(const Ws& ws) {
  if constexpr (sizeof(VT) == 8)
    return ws.V;
  else
    return reinterpret_cast<VT*>(ws.Vf);
}
template <typename VT>
__device__ __host__ inline VT* wbuf_of(const Ws& ws) {
  if constexpr (sizeof(VT) == 8)
    return ws.w;
  else
    return reinterpret_cast<VT*>(ws.wf);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Sum R values per lane over aligned segments of S lanes with a halving
// butterfly: min(log2 R, log2 S) exchange steps (each moves half of the
// remaining values to the partner lane), then full steps over the remaining
// lane bits. Afterwards, if R >= S, lane sl of a segment holds in v[0..R/S)
// the totals of value indices sl*(R/S) + t; if R < S, it holds in v[0] the
// total of value index sl / (S/R).
template <int R, int S>
__device__ inline void seg_sum(double (&v)[R], int sl) {
  static_assert((R & (R - 1)) == 0 && (S & (S - 1)) == 0 && S <= 64, "powers of two");
  int mask = S / 2;
#pragma unroll
  for (int h = R / 2; h >= 1 && mask >= 1; h >>= 1) {
    const bool upper = (sl & mask) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      // plain values first: a select between array elements can become a
      // select of addresses, which puts the array in scratch memory
      const double a = v[i], b = v[i + h];
      const double send = upper ? a : b;
      const double keep = upper ? b : a;
      v[i] = keep + __shfl_xor(send, mask, S);
    }
    mask >>= 1;
  }
  if constexpr (R < S) {
    for (; mask >= 1; mask >>= 1) v[0] += __shfl_xor(v[0], mask, S);
  }
}

// CSR SpMV shapes. S lanes share a row and each lane takes EPL of its
// entries, strided by S so that the S lanes read consecutive entries at each
// step; a lane group works on R rows at once. Few lanes per row keep each
// gather instruction on few, well-filled cache lines: on the 7-point
// 128^3 matrix one row per thread (S = 1, EPL = 8) runs at 6.0 TB/s where
// eight lanes per row reach 4.8 TB/s. Rows longer than S * EPL finish in a
// strided loop.
// Rows per lane group: about 8 entry slots per lane in flight in total.
template <int S, int EPL>
constexpr int spmv_rows() { return EPL >= 8 ? 1 : 8 / EPL; }

// Loads for one pass (all unconditional, at clamped indices; values masked
// afterwards): row pointers, then indices and values.
template <int R, int S>
__device__ inline void spmv_load_rp(const Csr& A, int64_t row0, int p0, int (&e0)[R], int (&e1)[R]) {
  constexpr int NSUB = 256 / S;
  const int sub = threadIdx.x / S;
  const int64_t n = A.n;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t r = row0 + p0 + q * NSUB + sub;
    const int64_t rc = r < n ? r : n - 1;
    const int a = A.rp[rc], b = A.rp[rc + 1];
    e0[q] = a;
    e1[q] = r < n ? b : a;
  }
}

template <int R, int S, int EPL>
__device__ inline void spmv_load_cv(const Csr& A, const int (&e0)[R], const int (&e1)[R],
                                    int (&c)[R][EPL], double (&v)[R][EPL]) {
  const int sl = threadIdx.x % S;
  const bool any = A.nnz > 0;
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const int e = e0[q] + sl + t * S;
      const int ec = (any && e < e1[q]) ? e : 0;
      c[q][t] = any ? A.ci[ec] : 0;
      v[q][t] = any ? A.va[ec] : 0.0;
    }
}

// Gathers, products, the long-row tail, the reduction over the S lanes and
// the emit of one pass.
template <int R, int S, int EPL, typename XT, typename Emit>
__device__ inline void spmv_finish(const Csr& A, const XT* __restrict__ x, int p0,
                                   const int (&e0)[R], const int (&e1)[R], const int (&c)[R][EPL],
                                   const double (&v)[R][EPL], Emit emit) {
  constexpr int NSUB = 256 / S;
  const int sub = threadIdx.x / S, sl = threadIdx.x % S;
  double xv[R][EPL];
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int t = 0; t < EPL; ++t) xv[q][t] = (double)x[(unsigned)c[q][t]];
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < EPL; ++t) a += (e0[q] + sl + t * S < e1[q]) ? v[q][t] * xv[q][t] : 0.0;
    for (int e = e0[q] + sl + EPL * S; e < e1[q]; e += S) a += A.va[e] * (double)x[A.ci[e]];
    acc[q] = a;
  }
  seg_sum<R, S>(acc, sl);
  if constexpr (R >= S) {
#pragma unroll
    for (int t = 0; t < R / S; ++t) emit(p0 + (sl * (R / S) + t) * NSUB + sub, acc[t]);
  } else {
    if ((sl & (S / R - 1)) == 0) emit(p0 + (sl / (S / R)) * NSUB + sub, acc[0]);
  }
}

// One pass over R * (256 / S) consecutive local rows starting at local row
// p0; emit(local_row, value) is called by one lane per row (rows at or past
// n give 0).
template <int R, int S, int EPL, typename XT, typename Emit>
__device__ inline void spmv_pass(const Csr& A, const XT* __restrict__ x, int64_t row0, int p0,
                                 Emit emit) {
  int e0[R], e1[R], c[R][EPL];
  double v[R][EPL];
  spmv_load_rp<R, S>(A, row0, p0, e0, e1);
  spmv_load_cv<R, S, EPL>(A, e0, e1, c, v);
  spmv_finish<R, S, EPL>(A, x, p0, e0, e1, c, v, emit);
}

// The SpMV of a whole tile of TR rows as a software pipeline over passes:
// while pass p gathers x, the row pointers and then the indices and values of
// pass p+1 are already in flight.
template <int R, int S, int EPL, int TR, typename XT, typename Emit>
__device__ inline void spmv_tile(const Csr& A, const XT* __restrict__ x, int64_t row0,
                                 Emit emit) {
  constexpr int RPP = R * (256 / S);
  constexpr int NP = TR / RPP;
  static_assert(NP >= 1 && TR % RPP == 0, "tile must hold whole passes");
  int e0[R], e1[R], c[R][EPL];
  double v[R][EPL];
  spmv_load_rp<R, S>(A, row0, 0, e0, e1);
  spmv_load_cv<R, S, EPL>(A, e0, e1, c, v);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    int e0n[R], e1n[R], cn[R][EPL];
    double vn[R][EPL];
    if (p + 1 < NP) spmv_load_rp<R, S>(A, row0, (p + 1) * RPP, e0n, e1n);
    if (p + 1 < NP) spmv_load_cv<R, S, EPL>(A, e0n, e1n, cn, vn);
    spmv_finish<R, S, EPL>(A, x, p * RPP, e0, e1, c, v, emit);
    if (p + 1 < NP) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        e0[q] = e0n[q];
        e1[q] = e1n[q];
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
          c[q][t] = cn[q][t];
          v[q][t] = vn[q][t];
        }
      }
    }
  }
}

// Device-wide sum of cnt doubles, one row of partials per slot (tile). Every
// workgroup calls it; it returns true only in the one workgroup that finishes
// last, with the totals in vals (LDS). Slots are summed in index order in
// groups of kGroup, then the group sums in index order, so the result does not
// depend on which workgroup arrives last. Counters are reset by the workgroup
// that consumes them, ready for the next launch on the stream.
//
// Cross-workgroup visibility. The eight XCDs' L2 caches are not coherent with
// one another for ordinary accesses. Partials travel only through relaxed
// agent-scope atomic stores and loads, whose agent-scope encoding makes each
// such access coherent across the XCDs. Every thread waits until its stores
// are acknowledged (s_waitcnt vmcnt(0)) before the workgroup takes its ticket,
// and the winner issues its loads only after the ticket's value has returned.
// The ticket is itself relaxed, not a release/acquire pair, so under the HIP
// memory model this ordering rests on those two hardware facts rather than on
// a fence. A device-wide release fence would write back the L2 in every
// workgroup. No other data written in this launch is read by another
// workgroup. Whole solves at full size (1,024 tiles, 32 groups) are tested for
// bitwise repeatability, so a toolchain or hardware change that broke the
// ordering would show.
__device__ inline void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Rows [part, part + B * parts, ...) below nrows of column i, B loads at a
// time: all B loads of a batch are in flight together (clamped rows, masked
// values), and the sum runs in row order.
template <int B>
__device__ inline double sum_part(const double* rows_base, int pstride, int nrows, int i, int part,
                                  int parts) {
  double acc = 0.0;
  for (int q0 = part; q0 < nrows; q0 += B * parts) {
    double v[B];
#pragma unroll
    for (int t = 0; t < B; ++t) {
      const int q = q0 + t * parts;
      const int qc = q < nrows ? q : nrows - 1;
      v[t] = atomic_ld(rows_base + (size_t)qc * pstride + i);
    }
#pragma unroll
    for (int t = 0; t < B; ++t) acc += (q0 + t * parts < nrows) ? v[t] : 0.0;
  }
  return acc;
}

// Sum rows [0, nrows) of a partials array (row stride pstride), columns
// [0, cnt), into vals. The workgroup splits the rows into `parts` interleaved
// subsets, one thread per (column, subset), each issuing its rows' loads in
// batches of 8; then the subsets' sums are added in a fixed order (so the
// result does not depend on timing). scratch needs parts * cnt doubles.
__device__ void sum_rows(const double* rows_base, int pstride, int nrows, int cnt, double* vals,
                         double* scratch) {
  const int tid = threadIdx.x, bs = blockDim.x;
  int parts = bs / cnt;
  if (parts > (nrows + 7) / 8) parts = (nrows + 7) / 8;
  if (parts < 1) parts = 1;
  // Batches of 8: wider ones hold an address and a value per load in VGPRs
  // and would raise the whole kernel's register allocation.
  auto part_sum = [&](int i, int part) {
    return sum_part<8>(rows_base, pstride, nrows, i, part, parts);
  };
  if (cnt * parts <= bs) {
    if (tid < cnt * parts) {
      const int i = tid % cnt, part = tid / cnt;
      scratch[part * cnt + i] = part_sum(i, part);
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += bs) {
      double acc = 0.0;
      for (int part = 0; part < parts; ++part) acc += scratch[part * cnt + i];
      vals[i] = acc;
    }
  } else {
    for (int i = tid; i < cnt; i += bs) vals[i] = part_sum(i, 0);
  }
  __syncthreads();
}

// No work to overlap with the final level of a reduction.
struct NoPrefetch {
  __device__ void issue() {}
  __device__ void commit() {}
};

// Two-level deterministic device-wide sum of vals[0:cnt] over nslots
// workgroups: each stores its row of partials; the last of each group of
// kGroup (by ticket) sums the group's rows, and the last group sums the group
// rows. Returns true in the one workgroup that holds the totals. That
// workgroup calls pre.issue() just before the loads of the final level and
// pre.commit() after them, so the caller's own loads for what follows overlap
// the final level's.
template <typename Pre>
__device__ bool grid_reduce(double* vals, int cnt, const Ws& ws, int slot, int nslots,
                            double* scratch, Pre& pre) {
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int bs = blockDim.x;
  const int ng = (nslots + kGroup - 1) / kGroup;
  const int grp = slot / kGroup;
  const int gbeg = grp * kGroup;
  const int gcnt = min(kGroup, nslots - gbeg);
  for (int i = tid; i < cnt; i += bs) atomic_st(ws.partials + (size_t)slot * ws.pstride + i, vals[i]);
  wait_stores();
  __syncthreads();
  if (tid == 0) {
    const unsigned t = atomicAdd(ws.counters + grp, 1u);
    s_last = (t == (unsigned)(gcnt - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  if (ng == 1) pre.issue();
  sum_rows(ws.partials + (size_t)gbeg * ws.pstride, ws.pstride, gcnt, cnt, vals, scratch);
  if (tid == 0) atomicExch(ws.counters + grp, 0u);
  if (ng == 1) {
    pre.commit();
    return true;
  }
  for (int i = tid; i < cnt; i += bs) atomic_st(ws.gpartials + (size_t)grp * ws.pstride + i, vals[i]);
  wait_stores();
  __syncthreads();
  if (tid == 0) {
    const unsigned t = atomicAdd(ws.counters + ng, 1u);
    s_last = (t == (unsigned)(ng - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  pre.issue();
  sum_rows(ws.gpartials, ws.pstride, ng, cnt, vals, scratch);
  if (tid == 0) atomicExch(ws.counters + ng, 0u);
  pre.commit();
  return true;
}

__device__ inline bool grid_reduce(double* vals, int cnt, const Ws& ws, int slot, int nslots,
                                   double* scratch) {
  NoPrefetch none;
  return grid_reduce(vals, cnt, ws, slot, nslots, scratch, none);
}

// out[i] = sum over q in [lo(i), hi(i)) of M[i * ld + q] * vec[q], for i in
// [0, nrows): dot products of contiguous row segments with a vector in LDS.
// Each wavefront takes 8 rows at a time with its lanes striding over q, so
// every lane has 8 independent loads in flight, and one halving butterfly
// reduces the 8 sums. Loads use clamped indices (M must hold nrows rows of ld
// entries); the values are masked.
template <int NR = 8, typename Lo, typename Hi>
__device__ void rows_dot(const double* M, int ld, const double* vec, int nrows, int qmax, Lo lo,
                         Hi hi, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i0 = wv * NR; i0 < nrows; i0 += nw * NR) {
    double acc[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) acc[t] = 0.0;
    for (int q0 = 0; q0 < qmax; q0 += 64) {
      const int q = q0 + lane;
      const int qc = q < ld ? q : ld - 1;
      double v[NR];
#pragma unroll
      for (int t = 0; t < NR; ++t) {
        const int i = i0 + t < nrows ? i0 + t : nrows - 1;
        v[t] = M[(size_t)i * ld + qc];
      }
      const double x = vec[q < qmax ? q : 0];
#pragma unroll
      for (int t = 0; t < NR; ++t) {
        const int i = i0 + t;
        acc[t] += (i < nrows && q >= lo(i) && q < hi(i)) ? v[t] * x : 0.0;
      }
    }
    wave_multi_sum<NR>(acc, lane);
    if ((lane & (64 / NR - 1)) == 0) {
      const int i = i0 + lane / (64 / NR);
      if (i < nrows) out[i] = acc[0];
    }
  }
}

// Plane rotation [c s; -s c] taking (a, b) to (r, 0).
__device__ inline void rot_make(double a, double b, double* c, double* s) {
  if (b == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  const double r = hypot(a, b);
  *c = a / r;
  *s = b / r;
}

// Givens least squares on Hessenberg column col (complete, in H): rotate a copy
// into R with the earlier rotations, form rotation col, update g. Serial; runs
// in one thread. Returns |g[col+1]|, the residual norm after col+1 columns.
__device__ double givens_column(const Ws& ws, int col) {
  const double* Hc = ws.H + (size_t)col * ws.ldh;
  double* Rc = ws.R + (size_t)col * ws.ldh;
  double a = Hc[0];
  for (int i = 0; i < col; ++i) {
    const double b = Hc[i + 1];
    const double c = ws.cs[i], s = ws.sn[i];
    Rc[i] = c * a + s * b;
    a = -s * a + c * b;
  }
  const double b = Hc[col + 1];
  double c, s;
  rot_make(a, b, &c, &s);
  Rc[col] = c * a + s * b;
  Rc[col + 1] = 0.0;
  ws.cs[col] = c;
  ws.sn[col] = s;
  const double gk = ws.g[col];
  const double gn = -s * gk;
  ws.g[col] = c * gk;
  ws.g[col + 1] = gn;
  const double res = fabs(gn);
  ws.gh[col + 1] = res;
  return res;
}

// The same rotation step with column col staged in LDS (hc[0..col+1]) with
// the earlier rotations (csl, snl[0..col-1]), so the serial loop does not wait
// on global memory. g holds g[col] on entry and g[col+1] on exit. Writes R,
// cs, sn, g, gh, and the new rotation into csl[col], snl[col] as well.
__device__ double rotate_staged(const Ws& ws, int col, const double* hc, double* csl, double* snl,
                                double& g) {
  double* Rc = ws.R + (size_t)col * ws.ldh;
  double a = hc[0];
#pragma unroll 4
  for (int i = 0; i < col; ++i) {
    const double b = hc[i + 1];
    const double c = csl[i], s = snl[i];
    Rc[i] = c * a + s * b;
    a = -s * a + c * b;
  }
  const double b = hc[col + 1];
  double c, s;
  rot_make(a, b, &c, &s);
  Rc[col] = c * a + s * b;
  Rc[col + 1] = 0.0;
  ws.cs[col] = c;
  ws.sn[col] = s;
  csl[col] = c;
  snl[col] = s;
  const double gn = -s * g;
  ws.g[col] = c * g;
  ws.g[col + 1] = gn;
  g = gn;
  const double res = fabs(gn);
  ws.gh[col + 1] = res;
  return res;
}

// The Givens least-squares update for the completed Hessenberg columns
// first..k-1, in order. The rotations and the stopping test consume finished
// columns and feed nothing back into the Arnoldi recurrence, so they may
// trail the steps by several columns (Section III, the depth-L pipeline).
// Each column is staged in LDS with the rotations so far; one thread applies
// the earlier rotations, forms the new one and updates g. Returns, in every
// thread, the first column count c + 1 whose |g| meets the cycle's tolerance
// (-1 if none), or -2 once a value is not finite (no column after it is
// rotated). Whole workgroup; lds holds 3 (m + 2) doubles.
__device__ int rotate_columns(const Ws& ws, int first, int k, double* lds) {
  __shared__ int s_res;
  __shared__ double s_g, s_tol;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int M2 = ws.m + 2;
  double* hc = lds;
  double* csl = lds + M2;
  double* snl = lds + 2 * M2;
  for (int i = tid; i < first; i += bs) {
    csl[i] = ws.cs[i];
    snl[i] = ws.sn[i];
  }
  if (tid == 0) {
    s_res = -1;
    s_g = ws.g[first];
    s_tol = ws.st->tol_cycle;
  }
  for (int c = first; c < k; ++c) {
    for (int i = tid; i <= c + 1; i += bs) hc[i] = ws.H[(size_t)c * ws.ldh + i];
    __syncthreads();
    if (tid == 0) {
      double g = s_g;
      const double res = rotate_staged(ws, c, hc, csl, snl, g);
      s_g = g;
      ws.st->gk = res;
      if (!isfinite(res))
        s_res = -2;
      else if (s_res == -1 && res <= s_tol)
        s_res = c + 1;
    }
    __syncthreads();
    if (s_res == -2) break;
  }
  __syncthreads();
  return s_res;
}

// The new column k of the Malard-Paige T (one-reduce MGS: T[0:k,k] =
// -T[0:k,0:k] l, T[k,k] = 1, so that T = (I + L^T)^{-1}; Section II) or row k
// of L (CGS2), from l = V[:,0:k]^T v_k in LDS. T is read from its row-major
// copy TT, whose row i holds T[i, i..k-1] contiguously. Both copies of the new
// column (or row) are written. Whole workgroup; tcol holds k doubles of LDS.
template <int NR>
__device__ void extend_t(const Ws& ws, int k, int scheme, const double* ell, double* tcol) {
  const int tid = threadIdx.x, bs = blockDim.x, ldt = ws.ldt;
  if (scheme == kSchemeMgs1r) {
    rows_dot<NR>(ws.TT, ldt, ell, k, k, [](int i) { return i; }, [&](int) { return k; }, tcol);
    __syncthreads();
    for (int i = tid; i < k; i += bs) {
      const double t = -tcol[i];
      ws.T[(size_t)k * ldt + i] = t;
      ws.TT[(size_t)i * ldt + k] = t;
    }
    if (tid == 0) {
      ws.T[(size_t)k * ldt + k] = 1.0;
      ws.TT[(size_t)k * ldt + k] = 1.0;
    }
  } else {
    for (int q = tid; q < k; q += bs) {
      ws.TT[(size_t)k * ldt + q] = ell[q];
      ws.T[(size_t)q * ldt + k] = ell[q];
    }
  }
}

// out[i] = sum over q < i of tri[i (i-1)/2 + q] vec[q], for i < nrows: dot
// products of the rows of a packed strictly lower triangle (in LDS) with a
// vector in LDS. Four lanes share a row; each keeps two sums over every
// fourth entry, so the loads of a lane are independent, and the four lanes'
// sums are added by two lane exchanges.
__device__ void tri_dots(const double* tri, const double* vec, int nrows, double* out) {
  const int tid = threadIdx.x, sl = tid & 3;
  for (int i0 = 0; i0 < nrows; i0 += blockDim.x / 4) {
    const int i = i0 + (tid >> 2);
    double a0 = 0.0, a1 = 0.0;
    if (i < nrows) {
      const double* row = tri + i * (i - 1) / 2;
      int q = sl;
      for (; q + 4 < i; q += 8) {
        a0 += row[q] * vec[q];
        a1 += row[q + 4] * vec[q + 4];
      }
      if (q < i) a0 += row[q] * vec[q];
    }
    double a = a0 + a1;
    a += __shfl_xor(a, 1, 64);
    a += __shfl_xor(a, 2, 64);
    if (sl == 0 && i < nrows) out[i] = a;
  }
}

// ----------------------------------------------------------- small kernels

__global__ void k_init(Ws ws, int ncounters) {
  for (int i = threadIdx.x; i < ncounters; i += blockDim.x) ws.counters[i] = 0u;
  if (threadIdx.x == 0) {
    DevState* st = ws.st;
    st->done = 0;
    st->j = 0;
    st->true_conv = 0;
    st->breakdown = 0;
    st->status = 0;
    st->bad_csr = 0;
    st->reductions = 0;
    st->rot_next = 0;
    st->bnorm = st->tol_abs = st->beta = st->rho = st->inv_rho = st->gk = 0.0;
    st->tol_cycle = 0.0;
    st->xscale = 1.0;
  }
}

// Start of a cycle: clear the flags and the small dense matrices (H, R, T,
// TT, g, gh), whose untouched entries must read as zero.
__global__ void k_cycle_begin(Ws ws) {
  const int m = ws.m;
  const size_t nh = (size_t)(m + 1) * m, nt = (size_t)(m + 2) * (m + 2);
  const size_t tot = 2 * nh + 2 * nt + 2 * (size_t)(m + 2);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < nh)
      ws.H[i] = 0.0;
    else if (i < 2 * nh)
      ws.R[i - nh] = 0.0;
    else if (i < 2 * nh + nt)
      ws.T[i - 2 * nh] = 0.0;
    else if (i < 2 * nh + 2 * nt)
      ws.TT[i - 2 * nh - nt] = 0.0;
    else if (i < 2 * nh + 2 * nt + (m + 2))
      ws.g[i - 2 * nh - 2 * nt] = 0.0;
    else
      ws.gh[i - 2 * nh - 2 * nt - (m + 2)] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    DevState* st = ws.st;
    st->done = 0;
    st->j = 0;
    st->true_conv = 0;
    st->breakdown = 0;
    st->rot_next = 0;
    st->xscale = 1.0;
  }
}

__global__ void k_solve_begin(Ws ws) {
  DevState* st = ws.st;
  st->done = 0;
  st->j = 0;
  st->true_conv = 0;
  st->breakdown = 0;
  st->status = 0;
  st->reductions = 0;
}

// CSR structure check: row_ptr[0] == 0, row_ptr[n] == nnz, non-decreasing
// row_ptr, 0 <= col_idx < n.
__global__ void k_validate_csr(const int* __restrict__ rp, const int* __restrict__ ci, int64_t n,
                               int64_t nnz, DevState* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (t0 == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) bad = 1;
  for (int64_t i = t0; i < n; i += stride)
    if (rp[i + 1] < rp[i]) bad = 1;
  for (int64_t e = t0; e < nnz; e += stride) {
    const int c = ci[e];
    if (c < 0 || (int64_t)c >= n) bad = 1;
  }
  if (bad) atomicOr(&st->bad_csr, 1);
}

// y = A x (b == nullptr) or y = b - A x: one pass of spmv_rows<S, EPL>() *
// (256 / S) rows per workgroup. Skipped when a state is given and its cycle is done.
template <int S, int EPL>
__global__ __launch_bounds__(256) void k_spmv(Csr A, const double* __restrict__ x,
                                               const double* __restrict__ b, double* __restrict__ y,
                                               const DevState* st) {
  if (st && st->done) return;
  constexpr int R = spmv_rows<S, EPL>();
  constexpr int RPP = R * (256 / S);
  const int64_t row0 = (int64_t)blockIdx.x * RPP;
  spmv_pass<R, S, EPL>(A, x, row0, 0, [&](int lr, double v) {
    const int64_t r = row0 + lr;
    if (r < A.n) y[r] = b ? b[r] - v : v;
  });
}

// ------------------------------------------------ sliced ELL copy of A

// Width of each slice, max(1, longest row): wavefront per slice, lane per row.
// With spread, also the largest spread of col - row over the entries of one
// slice column (entry j of every row of the slice), for slices at most
// max_width wide (a wider slice records INT_MAX: no copy is made then).
__global__ __launch_bounds__(256) void k_sell_width(Csr A, int64_t ns, int* __restrict__ width,
                                                     int* __restrict__ spread, int max_width) {
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= ns) return;  // uniform over the wavefront
  const int l = threadIdx.x & 63;
  const int64_t r = s * 64 + l;
  const int e0 = r < A.n ? A.rp[r] : 0;
  const int len = r < A.n ? A.rp[r + 1] - e0 : 0;
  int W = len;
  for (int mask = 32; mask >= 1; mask >>= 1) W = max(W, __shfl_xor(W, mask, 64));
  if (l == 0) width[s] = W < 1 ? 1 : W;
  if (!spread) return;
  if (W > max_width) {
    if (l == 0) atomicMax(spread, INT_MAX);
    return;
  }
  int widest = 0;
  for (int j = 0; j < W; ++j) {
    const bool real = j < len;
    const int d = real ? A.ci[e0 + j] - (int)r : 0;
    int mn = real ? d : INT_MAX, mx = real ? d : INT_MIN;
    for (int mask = 32; mask >= 1; mask >>= 1) {
      mn = min(mn, __shfl_xor(mn, mask, 64));
      mx = max(mx, __shfl_xor(mx, mask, 64));
    }
    if (mn != INT_MAX) widest = max(widest, mx - mn);
  }
  if (l == 0 && widest > 0) atomicMax(spread, widest);
}

// Number of distinct diagonals (col - row values) among each slice's entries,
// wavefront per slice, lane per row. With every row's columns strictly
// increasing, each lane's col - row values rise along its row, so taking the
// smallest of the lanes' next values over and over (and advancing the lanes
// that hold it) visits the slice's diagonals once each, in increasing order.
// Rows that are not strictly increasing set bit 0 of *flag; a slice with
// more than max_width diagonals stops counting and sets bit 1.
__global__ __launch_bounds__(256) void k_sell_diags(Csr A, int64_t ns, int* __restrict__ width,
                                                     int* __restrict__ flag, int max_width) {
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= ns) return;  // uniform over the wavefront
  const int l = threadIdx.x & 63;
  const int64_t r = s * 64 + l;
  const int e0 = r < A.n ? A.rp[r] : 0;
  const int len = r < A.n ? A.rp[r + 1] - e0 : 0;
  bool sorted = true;
  for (int j = 1; j < len; ++j) sorted = sorted && A.ci[e0 + j] > A.ci[e0 + j - 1];
  const int live = sorted ? len : 0;
  int p = 0, count = 0, wide = 0;
  for (;;) {
    const int d = p < live ? A.ci[e0 + p] - (int)r : INT_MAX;
    int mn = d;
    for (int mask = 32; mask >= 1; mask >>= 1) mn = min(mn, __shfl_xor(mn, mask, 64));
    if (mn == INT_MAX) break;  // uniform
    if (++count > max_width) {
      wide = 1;
      break;
    }
    if (d == mn) ++p;
  }
  if (!sorted) atomicOr(flag, 1);
  if (l == 0) {
    width[s] = count < 1 ? 1 : count;
    if (wide) atomicOr(flag, 2);
  }
}

// Copy of A into slices with 16-bit column deltas (sp already set), values in
// SVT: wavefront per slice, lane per row. Slice column j's base (the smallest
// col - row of its entries, 0 if it has none) goes to cbase, each entry's
// col - row - base to cd. A row that leaves [0, nnz) or does not fit its
// slice, or a slice column whose spread exceeds kSellDeltaSpan (a changed
// structure), sets st->bad_csr.
template <typename SVT>
__global__ __launch_bounds__(256) void k_sell_fill_d16(Csr A, Sell S, SVT* __restrict__ va,
                                                        DevState* st) {
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= S.ns) return;  // uniform over the wavefront
  const int l = threadIdx.x & 63;
  const int64_t r = s * 64 + l;
  const int64_t b = S.sp[s];
  const int W = (int)((S.sp[s + 1] - b) >> 6);
  const int64_t e0 = r < A.n ? A.rp[r] : 0;
  const int64_t e1 = r < A.n ? A.rp[r + 1] : 0;
  int len = (int)(e1 - e0);
  int bad = 0;
  if (e0 < 0 || e1 < e0 || e1 > A.nnz || len > W) {
    bad = 1;
    len = 0;
  }
  for (int j = 0; j < W; ++j) {
    const bool real = j < len;
    const int d = real ? A.ci[e0 + j] - (int)r : 0;
    int mn = real ? d : INT_MAX, mx = real ? d : INT_MIN;
    for (int mask = 32; mask >= 1; mask >>= 1) {
      mn = min(mn, __shfl_xor(mn, mask, 64));
      mx = max(mx, __shfl_xor(mx, mask, 64));
    }
    const int base = mn == INT_MAX ? 0 : mn;
    if (mn != INT_MAX && mx - mn > kSellDeltaSpan) bad = 1;
    const int64_t e = b + (int64_t)j * 64 + l;
    if (l == 0) S.cbase[(b >> 6) + j] = base;
    S.cd[e] = real ? (uint16_t)(d - base) : (uint16_t)0;
    va[e] = real ? (SVT)A.va[e0 + j] : (SVT)0;
  }
  if (bad) atomicOr(&st->bad_csr, 1);
}

// Copy of A into slices stored by diagonals (sp already set): wavefront per
// slice, lane per row. Slice column j holds, for every row r of the slice, the
// entry in column r + d_j, or 0 where the row has none; d_j, the slice's
// diagonals in increasing order (the order k_sell_diags visits them), goes to
// cbase. A row's entries thus keep their order, and padding zeros fall
// between them. A row outside [0, nnz), a row whose columns are not strictly
// increasing, or one with a diagonal beyond its slice's width (a changed
// structure) sets st->bad_csr.
template <typename SVT>
__global__ __launch_bounds__(256) void k_sell_fill_diag(Csr A, Sell S, SVT* __restrict__ va,
                                                         DevState* st) {
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= S.ns) return;  // uniform over the wavefront
  const int l = threadIdx.x & 63;
  const int64_t r = s * 64 + l;
  const int64_t b = S.sp[s];
  const int W = (int)((S.sp[s + 1] - b) >> 6);
  const int64_t e0 = r < A.n ? A.rp[r] : 0;
  const int64_t e1 = r < A.n ? A.rp[r + 1] : 0;
  int len = (int)(e1 - e0);
  int bad = 0;
  if (e0 < 0 || e1 < e0 || e1 > A.nnz || len > W) {
    bad = 1;
    len = 0;
  }
  int p = 0, prev = INT_MIN;
  for (int j = 0; j < W; ++j) {
    const int d = p < len ? A.ci[e0 + p] - (int)r : INT_MAX;
    int mn = d;
    for (int mask = 32; mask >= 1; mask >>= 1) mn = min(mn, __shfl_xor(mn, mask, 64));
    const bool take = p < len && d == mn;
    if (l == 0) S.cbase[(b >> 6) + j] = mn == INT_MAX ? 0 : mn;
    va[b + (int64_t)j * 64 + l] = take ? (SVT)A.va[e0 + p] : (SVT)0;
    if (take) {
      if (d <= prev) bad = 1;
      prev = d;
      ++p;
    }
  }
  if (p < len) bad = 1;
  if (bad) atomicOr(&st->bad_csr, 1);
}

// Copy of A into the slices (sp already set), thread per row, with values in
// SVT (float64, or float32 for the FP32-basis scheme: rounded to nearest). A
// row whose entries are not inside [0, nnz) or that is longer than its slice
// (a changed structure; the copy can run right behind a structure check on
// the stream) sets st->bad_csr and is not read.
template <typename SVT>
__global__ __launch_bounds__(256) void k_sell_fill(Csr A, Sell S, SVT* __restrict__ va,
                                                    DevState* st) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t s = r >> 6;
  if (s >= S.ns) return;
  const int l = (int)(r & 63);
  const int64_t b = S.sp[s];
  const int W = (int)((S.sp[s + 1] - b) >> 6);
  const int64_t e0 = r < A.n ? A.rp[r] : 0;
  const int64_t e1 = r < A.n ? A.rp[r + 1] : 0;
  int len = (int)(e1 - e0);
  if (e0 < 0 || e1 < e0 || e1 > A.nnz || len > W) {
    atomicOr(&st->bad_csr, 1);
    len = 0;
  }
  const int self = r < A.n ? (int)r : 0;
  for (int j = 0; j < W; ++j) {
    const int64_t e = b + (int64_t)j * 64 + l;
    const bool real = j < len;
    S.ci[e] = real ? A.ci[e0 + j] : self;
    va[e] = real ? (SVT)A.va[e0 + j] : (SVT)0;
  }
}

// The sliced copy's values in SVT.
template <typename SVT>
__device__ inline const SVT* sell_vals(const Sell& S) {
  if constexpr (sizeof(SVT) == 8)
    return S.va;
  else
    return S.vaf;
}

// Entries j0 .. j0+U-1 of lane l's row (row r) in the slice at entry offset
// b, width W (>= 1): indices past W are clamped to W-1 (their products are
// masked by the caller). Buffer loads over the slice's own entries (the
// descriptors are scalar; a lane supplies a 32-bit byte offset). SF (a
// SliceForm): kSfD16, the column is r + the slice column's base + the 16-bit
// delta; kSfDiag, r + the slice column's diagonal, with no per-entry index
// load; both as unsigned and at most n - 1 (a padding entry's value is 0
// whatever column it names).
template <int U, typename SVT, int SF>
__device__ inline void sell_load(const Sell& S, int64_t b, int W, int j0, int l, int r,
                                 int (&c)[U], SVT (&v)[U]) {
  const BufCol<SVT> vb(sell_vals<SVT>(S) + b, (int64_t)W * 64);
  if constexpr (SF == kSfDiag) {
    const int* cb = S.cbase + (b >> 6);
    const uint32_t last = (uint32_t)(S.n - 1);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int j = j0 + t < W ? j0 + t : W - 1;
      const uint32_t e = (uint32_t)(j * 64 + l);
      const uint32_t col = (uint32_t)(r + cb[j]);
      c[t] = (int)(col < last ? col : last);
      v[t] = vb.template load<GMRES_SELL_CPOL>(e * (uint32_t)sizeof(SVT));
    }
  } else if constexpr (SF == kSfD16) {
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(S.cd + b, (short)0, W * 64 * 2, 0x00020000);
    const int* cb = S.cbase + (b >> 6);
    const uint32_t last = (uint32_t)(S.n - 1);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int j = j0 + t < W ? j0 + t : W - 1;
      const uint32_t e = (uint32_t)(j * 64 + l);
      const uint32_t dl =
          (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(rd, (int)(e * 2u), 0, GMRES_SELL_CPOL);
      const uint32_t col = (uint32_t)(r + cb[j]) + dl;
      c[t] = (int)(col < last ? col : last);
      v[t] = vb.template load<GMRES_SELL_CPOL>(e * (uint32_t)sizeof(SVT));
    }
  } else {
    const __amdgpu_buffer_rsrc_t rc =
        __builtin_amdgcn_make_buffer_rsrc(S.ci + b, (short)0, W * 64 * 4, 0x00020000);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int j = j0 + t < W ? j0 + t : W - 1;
      const uint32_t e = (uint32_t)(j * 64 + l);
      c[t] = __builtin_amdgcn_raw_buffer_load_b32(rc, (int)(e * 4u), 0, GMRES_SELL_CPOL);
      v[t] = vb.template load<GMRES_SELL_CPOL>(e * (uint32_t)sizeof(SVT));
    }
  }
}

// out[i] = (A x) at row 64 (s0 + i sstride) + l, i < NS, for the lane's row in
// NS slices sstride apart (slice indices past the last are clamped; the
// caller drops those rows). x is in the basis type XT; values are float64 for
// the float64 basis and float32 otherwise, and the products and sums are in
// XT's arithmetic type. U entries per chunk; the column and
// value loads of the next chunk (of this slice or the next) are issued before
// the gathers of the current one are consumed, so one memory latency per
// chunk is hidden.
template <int NS, int U, typename XT, int SF>
__device__ inline void sell_slices(const Sell& S, const XT* __restrict__ x, int64_t s0,
                                   int64_t sstride, int l, arith_t<XT> (&out)[NS]) {
  using T = arith_t<XT>;
  using SVT = sval_t<XT>;
  // s0 is the same in every lane of the wavefront (the callers derive it from
  // the wavefront index); saying so keeps the slice offsets, widths and buffer
  // descriptors in scalar registers (the compiler cannot tell by itself, and
  // would wrap every buffer load in a loop over the distinct descriptors)
  s0 = __builtin_amdgcn_readfirstlane((int)s0);
  auto clampslice = [&](int64_t s) { return s < S.ns ? s : S.ns - 1; };
  // gathers from x[0, n) by 32-bit byte offset (the sliced format is used only
  // for n < 2^28)
  const BufCol<XT> xb(x, S.n);
  int64_t sc = clampslice(s0);
  int64_t b = S.sp[sc];
  int W = (int)((S.sp[sc + 1] - b) >> 6);
  int r = (int)(sc * 64 + l);  // the lane's row in that slice
  int c[U];
  SVT v[U];
  sell_load<U, SVT, SF>(S, b, W, 0, l, r, c, v);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    int64_t bn = b;
    int Wn = W;
    int rn = r;
    if (i + 1 < NS) {
      const int64_t sn = clampslice(s0 + (i + 1) * sstride);
      bn = S.sp[sn];
      Wn = (int)((S.sp[sn + 1] - bn) >> 6);
      rn = (int)(sn * 64 + l);
    }
    // Every product is a fused multiply-add into the row's sum, entries past
    // the width weighted 0: the rounding then does not depend on where in a
    // chunk an entry falls, so the slice forms (whose padding zeros sit at
    // different places in a row) give the same bits.
    T acc = (T)0;
    for (int j0 = 0; j0 < W; j0 += U) {
      T xv[U], vv[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        xv[t] = (T)xb((uint32_t)c[t] * (uint32_t)sizeof(XT));
        vv[t] = j0 + t < W ? (T)v[t] : (T)0;
      }
      if (j0 + U < W)
        sell_load<U, SVT, SF>(S, b, W, j0 + U, l, r, c, v);
      else if (i + 1 < NS)
        sell_load<U, SVT, SF>(S, bn, Wn, 0, l, rn, c, v);
#pragma unroll
      for (int t = 0; t < U; ++t) {
        if constexpr (sizeof(T) == 8)
          acc = __builtin_fma(vv[t], xv[t], acc);
        else
          acc = __builtin_fmaf(vv[t], xv[t], acc);
      }
    }
    out[i] = acc;
    b = bn;
    W = Wn;
    r = rn;
  }
}

// y = A x (b == nullptr) or y = b - A x from the sliced copy: each wavefront
// takes NS consecutive slices. Skipped when a state is given and its cycle is done.
template <int NS, int SF>
__global__ __launch_bounds__(256) void k_spmv_sell(Sell S, int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ y, const DevState* st) {
  if (st && st->done) return;
  const int l = threadIdx.x & 63;
  const int64_t s0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * NS;
  double out[NS];
  sell_slices<NS, 8, double, SF>(S, x, s0, 1, l, out);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int64_t r = (s0 + i) * 64 + l;
    if (r < n) y[r] = b ? b[r] - out[i] : out[i];
  }
}

// First basis vector of a reduced-precision-basis cycle: V[:,0] = r64 / ||r64||
// rounded to float32, and from there to bfloat16 for that basis (inv_rho
// holds 1 / ||r64|| from the restart reduction); skipped once the restart
// check ended the cycle.
template <typename VT>
__global__ __launch_bounds__(256) void k_first_vector(Ws ws) {
  const DevState* st = ws.st;
  if (st->done) return;
  const double s = st->inv_rho;
  VT* __restrict__ V = basis_of<VT>(ws);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ws.n; r += stride)
    V[r] = (VT)(float)(ws.r64[r] * s);
}

// ------------------------------------------------ the fused projection step

// Dynamic LDS layout of k_fused (doubles):
//   wl[TR]          w = A u for this tile (SpMV phase)
//   red[4][P]       per-wavefront column sums, P = 2 (m + 2) (at least 256
//                   doubles: it is also the reduction's scratch)
//   vals[P]         this tile's sums, then the device-wide totals
//   scr[6 (m + 2)]  scratch for the small dense step
__host__ __device__ inline int fused_red_doubles(int m) {
  const int r = 4 * 2 * (m + 2);
  return r < 256 ? 256 : r;
}
__host__ __device__ inline size_t fused_lds_doubles(int rpt, int m) {
  const int P = 2 * (m + 2);
  return (size_t)256 * rpt + (size_t)fused_red_doubles(m) + P + 6 * (size_t)(m + 2);
}

// Inputs of the small dense step of lagged step k, loaded by the workgroup
// that ends up holding the reduction's totals at the same time as the final
// level's partials, so that their latency overlaps: two state scalars into
// thread 0's registers and, when it fits in the SpMV tile buffer, the strictly
// triangular part of T (one-reduce MGS: tri[i (i-1)/2 + q] = T(q, i), q < i,
// column i) or of L (CGS2: the same index holds L(i, q), row i).
template <int NT>
struct TailPrefetch {
  const Ws* ws;
  double* tri;
  int k, scheme;
  int ntri;     // entries of tri to load (0: T or L is read from HBM instead)
  bool active;  // false: this launch's tail needs none of it
  bool staged;  // tri holds the whole strictly triangular block
  double tv[NT];
  double tol;
  int64_t red;

  __device__ void issue() {
    if (!active) return;
    const int tid = threadIdx.x;
    if (tid == 0) {
      tol = ws->st->tol_cycle;
      red = ws->st->reductions;
    }
    if (ntri > 0) {
      const double* src = scheme == kSchemeMgs1r ? ws->T : ws->TT;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int f0 = tid + 256 * t;
        const int f = f0 < ntri ? f0 : ntri - 1;
        // row i of the packed triangle holding entry f: i (i-1)/2 <= f < (i+1) i/2
        int i = (int)((1.0 + sqrt(1.0 + 8.0 * (double)f)) * 0.5);
        if (i * (i - 1) / 2 > f) --i;
        if ((i + 1) * i / 2 <= f) ++i;
        tv[t] = src[(size_t)i * ws->ldt + (f - i * (i - 1) / 2)];
      }
    }
  }
  __device__ void commit() {
    if (!active) return;
    const int tid = threadIdx.x;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int f = tid + 256 * t;
      if (f < ntri) tri[f] = tv[t];
    }
    __syncthreads();
  }
};

// The small dense step of a lagged scheme (one-reduce MGS or CGS2, first
// reduction), run by the workgroup that holds the totals in vals:
//   vals[2q] = V_q . u, vals[2q+1] = V_q . w (q < k), vals[2k] = u.u, vals[2k+1] = u.w.
// It forms the lagged norm rho = ||u|| (Section II, the normalization lag),
// which completes Hessenberg column k-1, and the MAXPY coefficients of step k:
// with l = V[:,0:k]^T v_k = p / rho and r = V[:,0:k+1]^T A v_k = [c / rho;
// gamma / rho^2],
//   one-reduce MGS: h = (I + L)^{-1} r. h[0:k] = T[0:k,0:k]^T r[0:k] with the
//     T of the earlier steps (T = (I + L^T)^{-1}), and h_k = r_k - l . h[0:k],
//     the last step of forward substitution with I + L, whose new row is
//     [l^T, 1]. So h does not wait for the new column of T;
//   CGS2: the first-pass coefficients corrected to first order, (I - L) r.
// The new column of T (or row of L), the Givens rotations and the stopping
// test are left to the extra workgroup of the step's MAXPY launch
// (side_step), off the critical path; the tail rotates only where the cycle
// ends here: at its norm-only last step (norm_only) or on a breakdown,
// rho == 0.
template <int NT, int NR>
__device__ void tail_lagged(const Ws& ws, double* vals, double* scr, int k, bool norm_only,
                            int m_eff, int scheme, const TailPrefetch<NT>& pf) {
  __shared__ double s_rho, s_last;
  __shared__ int s_go;  // 0: nothing more; 1: rotate the pending columns, the cycle ends; 2: go on
  __shared__ int s_first, s_bad;
  const int tid = threadIdx.x, bs = blockDim.x;
  DevState* st = ws.st;
  const int M2 = ws.m + 2;
  if (tid == 0) {
    st->reductions = pf.red + 1;
    const double alpha = vals[norm_only ? 0 : 2 * k];
    int go = 2;
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
        if (rho <= pf.tol) {
          st->true_conv = 1;
          st->done = 1;
          st->j = 0;
          go = 0;
        }
      } else {
        ws.H[(size_t)(k - 1) * ws.ldh + k] = rho;
        if (norm_only || rho == 0.0) go = 1;
      }
      if (go) {
        st->rho = rho;
        st->inv_rho = 1.0 / rho;
      }
    }
    s_rho = rho;
    s_go = go;
    s_first = st->rot_next;
  }
  __syncthreads();
  int go = s_go;
  if (go == 0) return;
  const double rho = s_rho;
  double* rot = scr + 3 * M2;  // 3 (m + 2) doubles for rotate_columns
  if (go == 1) {
    const int stop = rotate_columns(ws, s_first, k, rot);
    if (tid == 0) {
      st->rot_next = k;
      int g2 = 2;
      if (stop == -2) {
        st->status = kNonfinite;
        st->done = 1;
        g2 = 0;
      } else if (stop >= 0 && stop < k) {
        st->done = 1;
        st->j = stop;
        g2 = 0;
      } else if (rho == 0.0) {
        st->breakdown = 1;
        st->done = 1;
        st->j = k;
        g2 = 0;
      } else if (stop == k || norm_only) {
        // met at the newest column (the lag: one step after it was formed),
        // or the cycle's last step: T still gets its column k
        st->done = 1;
        st->j = k;
        g2 = norm_only ? 0 : 1;
      }
      s_go = g2;
    }
    __syncthreads();
    go = s_go;
    if (go == 0) return;
  }
  const int ldt = ws.ldt;
  const double* tri = pf.tri;
  double* ell = scr;                 // l = V[:,0:k]^T v_k, the new row of L
  double* rr = scr + M2;             // r = V[:,0:k+1]^T A v_k
  double* hb = scr + 2 * M2;         // h[0:k]
  for (int q = tid; q < k; q += bs) {
    const double l = vals[2 * q] / rho;
    ell[q] = l;
    ws.lvec[q] = l;
  }
  if (go == 1) return;
  for (int q = tid; q < k; q += bs) rr[q] = vals[2 * q + 1] / rho;
  if (tid == 0) {
    rr[k] = (vals[2 * k + 1] / rho) / rho;
    s_bad = 0;
  }
  __syncthreads();
  // hb[i] = sum over q < i of T(q, i) r_q (column i of T) or L(i, q) r_q (row i of L)
  if (pf.staged)
    tri_dots(tri, rr, k, hb);
  else
    rows_dot<NR>(scheme == kSchemeMgs1r ? ws.T : ws.TT, ldt, rr, k, k, [](int) { return 0; },
                 [](int i) { return i; }, hb);
  __syncthreads();
  for (int i = tid; i < k; i += bs) hb[i] = scheme == kSchemeMgs1r ? rr[i] + hb[i] : rr[i] - hb[i];
  __syncthreads();
  if (tid < 64) {
    const double* y = scheme == kSchemeMgs1r ? hb : rr;
    double a = 0.0;
    for (int q = tid; q < k; q += 64) a += ell[q] * y[q];
    a = wave_sum(a);
    if (tid == 0) s_last = a;
  }
  __syncthreads();
  for (int i = tid; i <= k; i += bs) {
    const double h = i < k ? hb[i] : rr[k] - s_last;
    ws.coef[i] = h;
    if (scheme == kSchemeMgs1r) ws.H[(size_t)k * ws.ldh + i] = h;
    if (!isfinite(h)) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0 && s_bad) {
    st->status = kNonfinite;
    st->done = 1;
  }
}

// The extra workgroup of a lagged step's MAXPY launch (step k), which the
// tail left this work to: the new column of T (or row of L) from
// l = lvec[0:k], then, once `depth` completed Hessenberg columns are pending
// (depth 1: every step), their Givens rotations and the stopping test
// (Section III: the rotations consume finished columns only, so they overlap
// the next step's streaming). A met tolerance ends the cycle at the first
// column count that met it; the steps that ran since then are discarded.
template <int NR>
__device__ void side_step(const Ws& ws, int k, int depth, int scheme) {
  __shared__ double lds[5 * (kMaxRestart + 2)];
  __shared__ int s_go, s_first;
  const int tid = threadIdx.x, bs = blockDim.x;
  DevState* st = ws.st;
  const int M2 = ws.m + 2;
  double* ell = lds + 3 * M2;
  double* tcol = lds + 4 * M2;
  if (tid == 0) {
    s_go = st->done == 0;
    s_first = st->rot_next;
  }
  for (int q = tid; q < k; q += bs) ell[q] = ws.lvec[q];
  __syncthreads();
  if (!s_go) return;
  extend_t<NR>(ws, k, scheme, ell, tcol);
  const int first = s_first;
  if (k >= 1 && k - first >= depth) {
    const int stop = rotate_columns(ws, first, k, lds);
    if (tid == 0) {
      st->rot_next = k;
      if (stop == -2) {
        st->status = kNonfinite;
        st->done = 1;
      } else if (stop >= 0) {
        st->j = stop;
        st->done = 1;
      }
    }
  }
}

// CGS2 second reduction: vals[2q] = V_q . z for q <= k; H[:,k] = (I - L) r + s.
__device__ void tail_cgs2_second(const Ws& ws, const double* vals, int k) {
  __shared__ int s_bad;
  const int tid = threadIdx.x, bs = blockDim.x;
  if (tid == 0) {
    ws.st->reductions += 1;
    s_bad = 0;
  }
  __syncthreads();
  for (int i = tid; i <= k; i += bs) {
    const double s = vals[2 * i];
    ws.coef2[i] = s;
    const double h = ws.coef[i] + s;
    ws.H[(size_t)k * ws.ldh + i] = h;
    if (!isfinite(h)) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0 && s_bad) {
    ws.st->status = kNonfinite;
    ws.st->done = 1;
  }
}

// Re-orthogonalized CGS, first projection: vals[2q] = V_q . w for q <= k,
// the coefficients of the first pass into coef.
__device__ void tail_cgs_pass1(const Ws& ws, const double* vals, int k) {
  __shared__ int s_bad;
  const int tid = threadIdx.x, bs = blockDim.x;
  if (tid == 0) {
    ws.st->reductions += 1;
    s_bad = 0;
  }
  __syncthreads();
  for (int i = tid; i <= k; i += bs) {
    const double s = vals[2 * i];
    ws.coef[i] = s;
    if (!isfinite(s)) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0 && s_bad) {
    ws.st->status = kNonfinite;
    ws.st->done = 1;
  }
}

// Two-synchronization CGS (Ruhe's form of iterated classical Gram-Schmidt),
// with u = v_i (normalized) and w = A v_i:
//   vals[2q] = v_q . v_i (q < i): row i of the strictly lower L of V^T V,
//   vals[2q+1] = v_q . w (q <= i): y;
// then r = (I - L - L^T) y over the leading (i+1) x (i+1) block is both the
// MAXPY coefficients and H[0:i+1, i]. L is kept row-major in TT and
// column-major in T (as for CGS2), so both sums read contiguous entries.
__device__ void tail_two_synch(const Ws& ws, const double* vals, int i) {
  __shared__ int s_bad;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int ldt = ws.ldt;
  if (tid == 0) {
    ws.st->reductions += 1;
    s_bad = 0;
  }
  for (int q = tid; q < i; q += bs) {
    const double l = vals[2 * q];
    ws.TT[(size_t)i * ldt + q] = l;
    ws.T[(size_t)q * ldt + i] = l;
  }
  __syncthreads();
  for (int a = tid; a <= i; a += bs) {
    double r = vals[2 * a + 1];
    const double* Lrow = ws.TT + (size_t)a * ldt;  // L(a, q), q < a
    for (int q = 0; q < a; ++q) r -= Lrow[q] * vals[2 * q + 1];
    const double* Lcol = ws.T + (size_t)a * ldt;   // L(q, a), q > a
    for (int q = a + 1; q <= i; ++q) r -= Lcol[q] * vals[2 * q + 1];
    ws.coef[a] = r;
    ws.H[(size_t)i * ws.ldh + a] = r;
    if (!isfinite(r)) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0 && s_bad) {
    ws.st->status = kNonfinite;
    ws.st->done = 1;
  }
}

// Fused Arnoldi step for the lagged schemes, K = index of the column being
// normalized (u = V[:,K]). Where w comes from (WSRC):
//   kWSpmv: w = A u for the tile, computed here (written to ws.w, kept in LDS);
//   kWLoad: w = A u was written to ws.w by a separate SpMV launch;
//   kWNone: w = 0 (the norm-only flush, or CGS2's second projection with u = z).
// Then sums over the tile of V_q . u and V_q . w for q < nproj, u.u and u.w;
// device-wide reduction; the last workgroup runs the tail.
// RPT rows per lane, 256 threads = 4 wavefronts. Row map (GMRES_FUSED_ROWMAP):
//   0: lane l of wavefront wv owns rows tile0 + wv*64*RPT + i*64 + l (each
//      wavefront a contiguous block of 64 RPT rows);
//   1: rows tile0 + i*256 + wv*64 + l (the four wavefronts' loads of one i
//      are adjacent, 2 KB contiguous per workgroup).
// Either way every column read is 512 contiguous bytes per wavefront.
template <int RPT, int S, int EPL, int WSRC, typename VT>
__global__ __launch_bounds__(256) void k_fused(Csr A, Sell SA, Ws ws, int K, int nproj, int m_eff,
                                                int tail, int G) {
  extern __shared__ double lds[];
  constexpr int TR = 256 * RPT;
  constexpr int CB = GMRES_PROJ_COLS;  // columns per butterfly chunk
  if (ws.st->done) return;
  const int P = 2 * (ws.m + 2);
  double* wl = lds;
  double* red = lds + TR;
  double* vals = red + fused_red_doubles(ws.m);
  double* scr = vals + P;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int tile = tile_of_block(G);
  const int64_t row0 = (int64_t)tile * TR;
  const int64_t n = A.n;
  const VT* __restrict__ V = basis_of<VT>(ws);
  VT* __restrict__ wout = wbuf_of<VT>(ws);
  const int64_t ldv = ws.ldv;
  const VT* __restrict__ u_g = V + (size_t)K * ldv;
  using CT = arith_t<VT>;  // arithmetic type of the basis
  constexpr bool HAS_SPMV = WSRC != kWNone;
  // the sliced copy (kWSell*): the lane's rows are row 64 s + lane of slices
  // s = row0/64 + wv RPT + i
  constexpr bool SELL = WSRC == kWSell || WSRC == kWSellD16 || WSRC == kWSellDiag;
  CT ws_out[RPT];
  if constexpr (SELL) {
    constexpr int SF = WSRC == kWSellD16 ? kSfD16 : WSRC == kWSellDiag ? kSfDiag : kSfI32;
    if constexpr (GMRES_FUSED_ROWMAP == 1)
      sell_slices<RPT, 8, VT, SF>(SA, u_g, (row0 >> 6) + wv, 4, lane, ws_out);
    else
      sell_slices<RPT, 8, VT, SF>(SA, u_g, (row0 >> 6) + wv * RPT, 1, lane, ws_out);
  }

  if constexpr (WSRC == kWSpmv) {
    // SpMV of the tile (fewer rows per lane group when the tile holds fewer).
    constexpr int R0 = spmv_rows<S, EPL>();
    constexpr int RG = R0 * (256 / S) > TR ? TR / (256 / S) : R0;
    auto emit = [&](int lr, double v) { wl[lr] = v; };
    if constexpr (GMRES_SPMV_PIPELINE == 1) {
      spmv_tile<RG, S, EPL, TR>(A, u_g, row0, emit);
    } else {
      constexpr int RPP = RG * (256 / S);
      for (int p0 = 0; p0 < TR; p0 += RPP) spmv_pass<RG, S, EPL>(A, u_g, row0, p0, emit);
    }
    __syncthreads();
  }

  // This lane's rows (clamped into range for loads), its u and w values;
  // rows past n carry u = w = 0 and so add nothing.
  // Loads take a uniform base rb plus a 32-bit byte offset (rows[i]): rb is
  // the tile's first row, or row n-1 for a padding tile past the end, so the
  // clamped rows lie in [rb, rb + TR) and the offsets are never negative.
  // Products and per-lane sums are in CT (the basis type's arithmetic type);
  // the sums become float64 for the cross-lane and device-wide reduction.
  CT u[RPT], w[RPT];
  uint32_t rows[RPT];
  const int64_t rb = row0 < n ? row0 : n - 1;
  const VT* __restrict__ Vt = V + rb;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = GMRES_FUSED_ROWMAP == 1 ? i * 256 + wv * 64 + lane : wv * 64 * RPT + i * 64 + lane;
    const int64_t r = row0 + lr;
    const bool ok = r < n;
    rows[i] = (uint32_t)((ok ? r : n - 1) - rb) * (uint32_t)sizeof(VT);
    const CT uv = (CT)ProjCol<VT>(u_g + rb, n - rb)(rows[i]);
    u[i] = ok ? uv : (CT)0;
    if constexpr (WSRC == kWSpmv) {
      w[i] = ok ? (CT)wl[lr] : (CT)0;
      if (ok) st_stream<1>(wout + r, (VT)w[i]);
    } else if constexpr (SELL) {
      w[i] = ok ? ws_out[i] : (CT)0;
      if (ok) st_stream<1>(wout + r, (VT)w[i]);
    } else if constexpr (WSRC == kWLoad) {
      const CT wv_ = (CT)ProjCol<VT>(wout + rb, n - rb)(rows[i]);
      w[i] = ok ? wv_ : (CT)0;
    } else {
      w[i] = (CT)0;
    }
  }
  double* myred = red + wv * P;

  // Columns 0..nproj-1 in chunks of CB, then the rest one at a time. The
  // loads of the next chunk (CB columns x RPT rows) are issued before the
  // current chunk is reduced, so two chunks' loads are in flight per lane.
  // The loop is unrolled twice over two fixed buffers: a loop-carried copy of
  // a loaded register would make the compiler wait for every load at the end
  // of each iteration. The last chunk's "next" load repeats that chunk (a
  // cache hit), which keeps the loads free of branches.
  constexpr int NVC = HAS_SPMV ? 2 * CB : CB;
  const int64_t nvalid = n - rb;  // rows rb .. n-1 of every column
  // the column at position t of the stream
  auto colat = [&](int t) { return GMRES_PROJ_REVERSE ? nproj - 1 - t : t; };
  auto load_chunk = [&](auto nt, VT (&buf)[CB][RPT], int j) {
    using Col = std::conditional_t<decltype(nt)::value, GlbColNT<VT>, ProjCol<VT>>;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const Col col(Vt + (size_t)colat(j + c) * ldv, nvalid);
#pragma unroll
      for (int i = 0; i < RPT; ++i) buf[c][i] = col(rows[i]);
    }
  };
  auto reduce_chunk = [&](const VT (&vv)[CB][RPT], int j) {
    double acc[NVC];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      CT p = (CT)0, q = (CT)0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        p += (CT)vv[c][i] * u[i];
        if constexpr (HAS_SPMV) q += (CT)vv[c][i] * w[i];
      }
      if constexpr (HAS_SPMV) {
        acc[2 * c] = (double)p;
        acc[2 * c + 1] = (double)q;
      } else {
        acc[c] = (double)p;
      }
    }
    if constexpr (GMRES_DPP_REDUCE) {
      // each value summed on its own, total in lane 63
#pragma unroll
      for (int t = 0; t < NVC; ++t) acc[t] = wave_sum_last(acc[t]);
      if (lane == 63) {
#pragma unroll
        for (int t = 0; t < NVC; ++t) {
          if constexpr (HAS_SPMV) {
            myred[2 * colat(j + t / 2) + (t & 1)] = acc[t];
          } else {
            myred[2 * colat(j + t)] = acc[t];
            myred[2 * colat(j + t) + 1] = 0.0;
          }
        }
      }
    } else {
      const double tot = wave_multi_sum<NVC>(acc, lane);
      constexpr int LOGNV = ilog2(NVC);
      if ((lane & ((64 / NVC) - 1)) == 0) {
        const int vi = lane >> (6 - LOGNV);
        if constexpr (HAS_SPMV) {
          myred[2 * colat(j + vi / 2) + (vi & 1)] = tot;
        } else {
          myred[2 * colat(j + vi)] = tot;
          myred[2 * colat(j + vi) + 1] = 0.0;
        }
      }
    }
  };
  // stream positions [t0, t1) (non-temporal loads if nt); returns the first
  // position not done (the rest of a partial chunk)
  auto stream = [&](auto nt, int t0, int t1) {
    int j0 = t0;
    if (t1 - t0 >= CB) {
      VT ba[CB][RPT], bb[CB][RPT];
      load_chunk(nt, ba, j0);
      for (;;) {
        // ba holds chunk j0
        load_chunk(nt, bb, j0 + 2 * CB <= t1 ? j0 + CB : j0);
        reduce_chunk(ba, j0);
        j0 += CB;
        if (j0 + CB > t1) break;
        // bb holds chunk j0
        load_chunk(nt, ba, j0 + 2 * CB <= t1 ? j0 + CB : j0);
        reduce_chunk(bb, j0);
        j0 += CB;
        if (j0 + CB > t1) break;
      }
    }
    return j0;
  };
  // The columns stream last to first. Columns keep.. go non-temporal: the
  // next MAXPY reads them last, after they would have left the last-level
  // cache anyway. Columns 0..keep-1, which it reads first, load through the
  // caches so that they are still there. (The choice changes no result.)
  const int split = GMRES_PROJ_REVERSE && nproj > ws.keep ? nproj - ws.keep : 0;
  int j0 = stream(std::true_type{}, 0, split);
  j0 = stream(std::false_type{}, j0, nproj);
  for (; j0 < nproj; ++j0) {
    VT vv[RPT];
    const ProjCol<VT> col(Vt + (size_t)colat(j0) * ldv, nvalid);
#pragma unroll
    for (int i = 0; i < RPT; ++i) vv[i] = col(rows[i]);
    CT pl = (CT)0, cl = (CT)0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      pl += (CT)vv[i] * u[i];
      if constexpr (HAS_SPMV) cl += (CT)vv[i] * w[i];
    }
    const double p = wave_sum_last((double)pl);
    const double c = HAS_SPMV ? wave_sum_last((double)cl) : 0.0;
    if (lane == 63) {
      myred[2 * colat(j0)] = p;
      myred[2 * colat(j0) + 1] = c;
    }
  }
  {
    CT all = (CT)0, gal = (CT)0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      all += u[i] * u[i];
      if constexpr (HAS_SPMV) gal += u[i] * w[i];
    }
    const double al = wave_sum_last((double)all);
    const double ga = HAS_SPMV ? wave_sum_last((double)gal) : 0.0;
    if (lane == 63) {
      myred[2 * nproj] = al;
      myred[2 * nproj + 1] = ga;
    }
  }
  __syncthreads();
  const int cnt = 2 * (nproj + 1);
  for (int i = tid; i < cnt; i += 256) vals[i] = ((red[i] + red[P + i]) + red[2 * P + i]) + red[3 * P + i];
  __syncthreads();
  // The tile buffer wl is free now; the tail's inputs are staged there.
  const bool norm_only = nproj < K;
  TailPrefetch<RPT> pf;
  pf.ws = &ws;
  pf.tri = wl;
  pf.k = K;
  pf.scheme = tail == kTailLagged1r ? kSchemeMgs1r : kSchemeCgs2;
  pf.active = tail == kTailLagged1r || tail == kTailLaggedCgs2;
  pf.staged = K * (K - 1) / 2 <= TR;
  pf.ntri = (pf.active && pf.staged && !norm_only) ? K * (K - 1) / 2 : 0;
  if (!grid_reduce(vals, cnt, ws, tile, G, red, pf)) return;
  if (tail == kTailCgs2Second)
    tail_cgs2_second(ws, vals, K - 1);
  else if (tail == kTailCgsPass1)
    tail_cgs_pass1(ws, vals, K - 1);
  else if (tail == kTailTwoSynch)
    tail_two_synch(ws, vals, K);
  else
    tail_lagged<RPT, 8>(ws, vals, scr, K, norm_only, m_eff, pf.scheme, pf);
}

// ------------------------------------------------------------------ MAXPY

// mode 0 (lagged step k): V[:,k] = u / rho and V[:,k+1] = w / rho - V[:,0:k+1] coef,
//   where column k enters already normalized;
// mode 1 (CGS2 second pass): V[:,k+1] -= V[:,0:k+1] coef2;
// mode 2 (re-orthogonalized CGS, first pass): V[:,k+1] -= V[:,0:k+1] coef;
// mode 3 (two-synchronization CGS): V[:,k+1] = w - V[:,0:k+1] coef.
// VT is the basis type; for float32 the coefficients and 1/rho are rounded
// to float32 and the sums run in float32.
// side != 0 (mode 0 only: kSchemeMgs1r or kSchemeCgs2): the launch has one
// workgroup more than the G tiles, which runs side_step for the step's
// scheme with pipeline depth `depth` instead of a tile.
template <int RPT, typename VT>
__global__ __launch_bounds__(256) void k_maxpy(Ws ws, int k, int mode, int G, int side, int depth) {
  constexpr int TR = 256 * RPT;
  if (side && blockIdx.x == G) {
    side_step<4>(ws, k, depth, side);
    return;
  }
  if (ws.st->done) return;
  const int tile = tile_of_block(G);
  const int64_t row0 = (int64_t)tile * TR;
  const int64_t n = ws.n;
  const int tid = threadIdx.x;
  VT* __restrict__ V = basis_of<VT>(ws);
  const int64_t ldv = ws.ldv;
  const double* __restrict__ cf = mode == 1 ? ws.coef2 : ws.coef;
  using CT = arith_t<VT>;  // arithmetic type of the basis
  const CT invr = (CT)ws.st->inv_rho;
  // Loads at clamped rows (unconditional, so they are all in flight at once);
  // only rows below n are stored. Each load is a uniform column base (row rb
  // of column q: the tile's first row, or n-1 for a padding tile past the
  // end) plus a per-lane byte offset in [0, 8 TR), so one offset register per
  // row serves every column.
  CT acc[RPT];
  uint32_t off[RPT];
  const int64_t rb = row0 < n ? row0 : n - 1;
  const int64_t nvalid = n - rb;
  const MaxpyCol<VT> src0(((mode == 0 || mode == 3) ? wbuf_of<VT>(ws) : V + (size_t)(k + 1) * ldv) + rb,
                          nvalid);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = row0 + i * 256 + tid;
    off[i] = (uint32_t)((r < n ? r : n - 1) - rb) * (uint32_t)sizeof(VT);
    acc[i] = mode == 0 ? (CT)src0(off[i]) * invr : (CT)src0(off[i]);
  }
  // GMRES_MAXPY_COLS columns per pass (their loads are in flight together).
  constexpr int MC = GMRES_MAXPY_COLS;
  const VT* __restrict__ Vt = V + rb;
  // Columns below ntend are loaded non-temporal (buffer loads; a global
  // non-temporal load in one arm of the branch would be merged with the
  // other's plain load). The last keep columns, which the next step's
  // projection reads first, load through the caches.
  const int ntend = k - ws.keep;
  int q = 0;
  for (; q + MC <= k; q += MC) {
    CT c[MC];
    VT v[MC][RPT];
#pragma unroll
    for (int t = 0; t < MC; ++t) {
      c[t] = (CT)cf[q + t];
      const VT* cp = Vt + (size_t)(q + t) * ldv;
      if (q + t < ntend) {
        const BufCol<VT> col(cp, nvalid);
#pragma unroll
        for (int i = 0; i < RPT; ++i) v[t][i] = col.template load<2>(off[i]);
      } else {
        const MaxpyCol<VT> col(cp, nvalid);
#pragma unroll
        for (int i = 0; i < RPT; ++i) v[t][i] = col(off[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      CT a = acc[i];
#pragma unroll
      for (int t = 0; t < MC; ++t) a -= (CT)v[t][i] * c[t];
      acc[i] = a;
    }
  }
  for (; q < k; ++q) {
    const CT c0 = (CT)cf[q];
    const MaxpyCol<VT> col(Vt + (size_t)q * ldv, nvalid);
    VT v[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = col(off[i]);
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] -= (CT)v[i] * c0;
  }
  const CT ck = (CT)cf[k];
  VT vk[RPT];
  const MaxpyCol<VT> colk(Vt + (size_t)k * ldv, nvalid);
#pragma unroll
  for (int i = 0; i < RPT; ++i) vk[i] = colk(off[i]);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = row0 + i * 256 + tid;
    if (r < n) {
      CT x = (CT)vk[i];
      if (mode == 0) {
        x *= invr;
        st_stream<2>(V + (size_t)k * ldv + r, (VT)x);
      }
      st_stream<2>(V + (size_t)(k + 1) * ldv + r, (VT)(acc[i] - x * ck));
    }
  }
}

// ------------------------------------------- level-1 MGS building blocks

// w -= coef * a (if a != nullptr; coef read from device memory), then the
// device-wide dot product w . v (v may alias w). The last workgroup runs the
// tail selected by `tail`. Skipped when the cycle is done (except for the
// norm of b and the final residual, which run outside cycles).
template <int RPT>
__global__ __launch_bounds__(256) void k_axpy_dot(Ws ws, double* wv_,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ coef,
                                                   const double* v, int tail, int i_col,
                                                   int q_row, int m_eff, double aux, int G) {
  constexpr int TR = 256 * RPT;
  __shared__ double red[256];
  __shared__ double vals[2];
  if (tail != kTailBnorm && tail != kTailFinalRes && ws.st->done) return;
  const int tile = tile_of_block(G);
  const int64_t row0 = (int64_t)tile * TR;
  const int64_t n = ws.n;
  const int tid = threadIdx.x;
  const double cf = a ? *coef : 0.0;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = row0 + i * 256 + tid;
    if (r < n) {
      double x = wv_[r];
      if (a) {
        x -= cf * a[r];
        wv_[r] = x;
      }
      s += x * (v == wv_ ? x : v[r]);
    }
  }
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) vals[0] = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  if (!grid_reduce(vals, 1, ws, tile, G, red)) return;
  if (tid != 0) return;
  DevState* st = ws.st;
  st->reductions += 1;
  const double d = vals[0];
  switch (tail) {
    case kTailBnorm: {
      const double bn = sqrt(d);
      st->bnorm = bn;
      st->tol_abs = aux * bn;
      st->tol_cycle = st->tol_abs;
      if (!isfinite(bn)) st->status = kNonfinite;
      break;
    }
    case kTailFinalRes: {
      const double r = sqrt(d);
      st->beta = r;
      if (!isfinite(r)) st->status = kNonfinite;
      break;
    }
    case kTailMgsBeta: {
      const double beta = sqrt(d);
      st->beta = beta;
      ws.g[0] = beta;
      if (!isfinite(beta)) {
        st->status = kNonfinite;
        st->done = 1;
      } else if (beta <= st->tol_abs) {
        st->true_conv = 1;
        st->done = 1;
        st->j = 0;
      } else {
        st->inv_rho = 1.0 / beta;
      }
      break;
    }
    case kTailIrBeta: {
      // FP32-basis cycle: ||r|| of the FP64 restart residual is the restart
      // check; the cycle then works on r / ||r||, so its |g_k| are relative
      // to ||r||, and x is updated by ||r|| V y.
      const double beta = sqrt(d);
      st->beta = beta;
      if (!isfinite(beta)) {
        st->status = kNonfinite;
        st->done = 1;
      } else if (beta <= st->tol_abs) {
        st->true_conv = 1;
        st->done = 1;
        st->j = 0;
      } else {
        st->inv_rho = 1.0 / beta;
        st->tol_cycle = st->tol_abs / beta;
        st->xscale = beta;
      }
      break;
    }
    case kTailMgsH: {
      ws.H[(size_t)i_col * ws.ldh + q_row] = d;
      if (!isfinite(d)) {
        st->status = kNonfinite;
        st->done = 1;
      }
      break;
    }
    case kTailMgsNorm: {
      const double hn = sqrt(d);
      ws.H[(size_t)i_col * ws.ldh + i_col + 1] = hn;
      if (!isfinite(hn)) {
        st->status = kNonfinite;
        st->done = 1;
        break;
      }
      const double gk = givens_column(ws, i_col);
      st->gk = gk;
      if (!isfinite(gk)) {
        st->status = kNonfinite;
        st->done = 1;
      } else if (hn == 0.0) {
        st->breakdown = 1;
        st->done = 1;
        st->j = i_col + 1;
      } else {
        st->inv_rho = 1.0 / hn;
        if (gk <= st->tol_abs || i_col + 1 == m_eff) {
          st->done = 1;
          st->j = i_col + 1;
        }
      }
      break;
    }
    default:
      break;
  }
}

// v *= inv_rho (level-1 MGS normalization), skipped once the cycle is done:
// a column formed by the step that ends the cycle is not part of the solution.
__global__ __launch_bounds__(256) void k_scale(Ws ws, double* __restrict__ v) {
  const DevState* st = ws.st;
  if (st->done) return;
  const double s = st->inv_rho;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ws.n; r += stride) v[r] *= s;
}

// --------------------------------------------------------- end of a cycle

// y = R[0:j,0:j]^{-1} g[0:j] by column-oriented back substitution; a zero
// pivot (singular A) gives a zero component. One workgroup. When the leading
// j x j block of R fits in the dynamic LDS (ldh * j doubles), it is staged
// there first with all loads in flight, so the j sequential steps do not each
// wait on global memory.
__global__ __launch_bounds__(256) void k_backsolve(Ws ws, int lds_doubles) {
  extern __shared__ double sm[];
  __shared__ double s_y;
  const DevState* st = ws.st;
  const int j = st->j;
  if (st->status || j <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  double* gg = sm;
  double* Rl = sm + (ws.m + 2);
  const bool staged = (size_t)(ws.m + 2) + (size_t)ws.ldh * j <= (size_t)lds_doubles;
  for (int i = tid; i < j; i += bs) gg[i] = ws.g[i];
  if (staged)
    for (int e = tid; e < ws.ldh * j; e += bs) Rl[e] = ws.R[e];
  __syncthreads();
  const double* R = staged ? Rl : ws.R;
  for (int i = j - 1; i >= 0; --i) {
    if (tid == 0) {
      const double piv = R[(size_t)i * ws.ldh + i];
      const double yi = piv != 0.0 ? gg[i] / piv : 0.0;
      ws.y[i] = yi;
      s_y = yi;
    }
    __syncthreads();
    const double yi = s_y;
    for (int t = tid; t < i; t += bs) gg[t] -= R[(size_t)i * ws.ldh + t] * yi;
    __syncthreads();
  }
}

// x += xscale V[:,0:j] y, with each pass's loads all in flight (loads at
// clamped rows; only rows below n are stored). The sums run
// in float64 whatever the basis type VT; xscale (1 for the FP64 schemes, the
// restart residual norm for the FP32-basis scheme) is folded into y. With
// GMRES_XUPDATE_REVERSE the columns are taken last to first: the cycle's last
// MAXPY read them first to last, so the last-level cache still holds the
// highest ones.
template <int RPT, typename VT>
__global__ __launch_bounds__(256) void k_xupdate(Ws ws, double* __restrict__ x, int G) {
  constexpr int TR = 256 * RPT;
  const DevState* st = ws.st;
  const int j = st->j;
  if (st->status || j <= 0) return;
  const int tile = tile_of_block(G);
  const int64_t row0 = (int64_t)tile * TR;
  const int64_t n = ws.n;
  const VT* __restrict__ V = basis_of<VT>(ws);
  const int64_t ldv = ws.ldv;
  const double* __restrict__ y = ws.y;
  const double xs = st->xscale;
  // byte offsets from row rb (the tile's first row, or n-1 for a padding
  // tile past the end), so they lie in [0, sizeof(VT) TR)
  const int64_t rb = row0 < n ? row0 : n - 1;
  const VT* __restrict__ Vt = V + rb;
  uint32_t off[RPT];  // byte offsets into the basis columns
  double acc[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = row0 + i * 256 + threadIdx.x;
    const uint32_t e = (uint32_t)((r < n ? r : n - 1) - rb);
    off[i] = e * (uint32_t)sizeof(VT);
    acc[i] = MaxpyCol<double>(x + rb, n - rb)(e * 8u);
  }
  // GMRES_MAXPY_COLS columns per pass, as in the MAXPY. The cycle's basis
  // is not read again, so its columns are loaded non-temporal (the first
  // ones, which the last MAXPY read last, still hit in the caches).
  constexpr int MC = GMRES_MAXPY_COLS;
  auto colx = [&](int t) { return GMRES_XUPDATE_REVERSE ? j - 1 - t : t; };
  int q = 0;
  for (; q + MC <= j; q += MC) {
    double c[MC];
    VT v[MC][RPT];
#pragma unroll
    for (int t = 0; t < MC; ++t) {
      c[t] = xs * y[colx(q + t)];
      const GlbColNT<VT> col(Vt + (size_t)colx(q + t) * ldv, n - rb);
#pragma unroll
      for (int i = 0; i < RPT; ++i) v[t][i] = col(off[i]);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      double a = acc[i];
#pragma unroll
      for (int t = 0; t < MC; ++t) a += (double)v[t][i] * c[t];
      acc[i] = a;
    }
  }
  for (; q < j; ++q) {
    const double c0 = xs * y[colx(q)];
    double v[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = (double)GlbColNT<VT>(Vt + (size_t)colx(q) * ldv, n - rb)(off[i]);
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] += v[i] * c0;
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = row0 + i * 256 + threadIdx.x;
    if (r < n) x[r] = acc[i];
  }
}

// ------------------------------------------------------------ launchers

#define GMRES_CHECK_LAUNCH()                          \
  do {                                                \
    if (hipGetLastError() != hipSuccess) return -2;   \
  } while (0)

int launch_init(const Ws& ws, int ncounters, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, ws, ncounters);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_solve_begin(const Ws& ws, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_begin, dim3(1), dim3(1), 0, s, ws);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_cycle_begin(const Ws& ws, hipStream_t s) {
  const size_t tot = 2 * (size_t)(ws.m + 1) * ws.m + 2 * (size_t)(ws.m + 2) * (ws.m + 2) +
                    2 * (size_t)(ws.m + 2);
  const unsigned blocks = (unsigned)((tot + 255) / 256 < 64 ? (tot + 255) / 256 : 64);
  hipLaunchKernelGGL(k_cycle_begin, dim3(blocks), dim3(256), 0, s, ws);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_validate(const Csr& A, int64_t nnz, DevState* st, hipStream_t s) {
  int64_t work = A.n > nnz ? A.n : nnz;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)blocks), dim3(256), 0, s, A.rp, A.ci, A.n, nnz,
                     st);
  GMRES_CHECK_LAUNCH();
  return 0;
}

template <int S, int EPL>
static void spmv_s(const Csr& A, const double* x, const double* b, double* y, const DevState* st,
                   hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr int RPP = spmv_rows<S, EPL>() * (256 / S);
  const int64_t blocks = (A.n + RPP - 1) / RPP;
  hipExtLaunchKernelGGL((k_spmv<S, EPL>), dim3((unsigned)blocks), dim3(256), 0u, s, e0, e1, 0u, A,
                        x, b, y, st);
}

// SpMV shapes: (S lanes per row, EPL entries per lane).
#define GMRES_SPMV_SHAPES(X) X(1, 8) X(2, 8) X(4, 8) X(8, 4) X(8, 8) X(64, 1)

int launch_spmv(const Csr& A, int shape, const double* x, const double* b, double* y,
                const DevState* st, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (shape) {
#define GMRES_CASE(S_, E_) \
  case S_ * 100 + E_: spmv_s<S_, E_>(A, x, b, y, st, s, e0, e1); break;
    GMRES_SPMV_SHAPES(GMRES_CASE)
#undef GMRES_CASE
    default: return -2;
  }
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_sell_width(const Csr& A, int64_t ns, int* width, int* spread, int max_width,
                      hipStream_t s) {
  const int64_t blocks = (ns + 3) / 4;
  hipLaunchKernelGGL(k_sell_width, dim3((unsigned)blocks), dim3(256), 0, s, A, ns, width, spread,
                     max_width);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_sell_diags(const Csr& A, int64_t ns, int* width, int* flag, int max_width,
                      hipStream_t s) {
  const int64_t blocks = (ns + 3) / 4;
  hipLaunchKernelGGL(k_sell_diags, dim3((unsigned)blocks), dim3(256), 0, s, A, ns, width, flag,
                     max_width);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_sell_fill(const Csr& A, const Sell& S, DevState* st, hipStream_t s) {
  const int64_t blocks = (S.ns * 64 + 255) / 256;  // a wavefront per slice, or a thread per row
  if (S.sf == kSfDiag) {
    if (S.vaf)
      hipLaunchKernelGGL(k_sell_fill_diag<float>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.vaf, st);
    else
      hipLaunchKernelGGL(k_sell_fill_diag<double>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.va, st);
  } else if (S.sf == kSfD16) {
    if (S.vaf)
      hipLaunchKernelGGL(k_sell_fill_d16<float>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.vaf, st);
    else
      hipLaunchKernelGGL(k_sell_fill_d16<double>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.va, st);
  } else if (S.vaf) {
    hipLaunchKernelGGL(k_sell_fill<float>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.vaf, st);
  } else {
    hipLaunchKernelGGL(k_sell_fill<double>, dim3((unsigned)blocks), dim3(256), 0, s, A, S, S.va, st);
  }
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_first_vector(const Ws& ws, int bt, hipStream_t s) {
  int64_t blocks = (ws.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (bt == kBasisBf16)
    hipLaunchKernelGGL(k_first_vector<__bf16>, dim3((unsigned)blocks), dim3(256), 0, s, ws);
  else
    hipLaunchKernelGGL(k_first_vector<float>, dim3((unsigned)blocks), dim3(256), 0, s, ws);
  GMRES_CHECK_LAUNCH();
  return 0;
}

// Two slices per wavefront, four wavefronts per workgroup.
int launch_spmv_sell(const Sell& S, int64_t n, const double* x, const double* b, double* y,
                     const DevState* st, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr int NS = 2;
  const int64_t blocks = (S.ns + 4 * NS - 1) / (4 * NS);
  if (S.sf == kSfDiag)
    hipExtLaunchKernelGGL((k_spmv_sell<NS, kSfDiag>), dim3((unsigned)blocks), dim3(256), 0u, s, e0,
                          e1, 0u, S, n, x, b, y, st);
  else if (S.sf == kSfD16)
    hipExtLaunchKernelGGL((k_spmv_sell<NS, kSfD16>), dim3((unsigned)blocks), dim3(256), 0u, s, e0,
                          e1, 0u, S, n, x, b, y, st);
  else
    hipExtLaunchKernelGGL((k_spmv_sell<NS, kSfI32>), dim3((unsigned)blocks), dim3(256), 0u, s, e0,
                          e1, 0u, S, n, x, b, y, st);
  GMRES_CHECK_LAUNCH();
  return 0;
}

// The step kernels are launched with hipExtLaunchKernelGGL so that optional
// start/stop events are attached to the dispatch itself and time the kernel
// alone.
template <int RPT, int S, int EPL, int WSRC, typename VT>
static void fused_t(const Csr& A, const Sell& SA, const Ws& ws, int K, int nproj, int m_eff,
                    int tail, int G, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const uint32_t lds = (uint32_t)(fused_lds_doubles(RPT, ws.m) * sizeof(double));
  hipExtLaunchKernelGGL((k_fused<RPT, S, EPL, WSRC, VT>), dim3(G), dim3(256), lds, s, e0, e1, 0u,
                        A, SA, ws, K, nproj, m_eff, tail, G);
}

template <int RPT, typename VT>
static int fused_r(const Csr& A, const Sell& SA, int shape, int wsrc, const Ws& ws, int K,
                   int nproj, int m_eff, int tail, int G, hipStream_t s, hipEvent_t e0,
                   hipEvent_t e1) {
  switch (wsrc) {
    case kWNone: fused_t<RPT, 1, 1, kWNone, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); return 0;
    case kWLoad: fused_t<RPT, 1, 1, kWLoad, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); return 0;
    case kWSell: fused_t<RPT, 1, 1, kWSell, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); return 0;
    case kWSellD16: fused_t<RPT, 1, 1, kWSellD16, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); return 0;
    case kWSellDiag: fused_t<RPT, 1, 1, kWSellDiag, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); return 0;
    case kWSpmv: break;
    default: return -2;
  }
  switch (shape) {
#define GMRES_CASE(S_, E_) \
  case S_ * 100 + E_: fused_t<RPT, S_, E_, kWSpmv, VT>(A, SA, ws, K, nproj, m_eff, tail, G, s, e0, e1); break;
    GMRES_SPMV_SHAPES(GMRES_CASE)
#undef GMRES_CASE
    default: return -2;
  }
  return 0;
}

template <typename VT>
static int fused_v(const Csr& A, const Sell& SA, int shape, const Ws& ws, int rpt, int K,
                   int nproj, int wsrc, int m_eff, int tail, int G, hipStream_t s, hipEvent_t e0,
                   hipEvent_t e1) {
  switch (rpt) {
    case 1: return fused_r<1, VT>(A, SA, shape, wsrc, ws, K, nproj, m_eff, tail, G, s, e0, e1);
    case 2: return fused_r<2, VT>(A, SA, shape, wsrc, ws, K, nproj, m_eff, tail, G, s, e0, e1);
    case 4: return fused_r<4, VT>(A, SA, shape, wsrc, ws, K, nproj, m_eff, tail, G, s, e0, e1);
    default: return fused_r<8, VT>(A, SA, shape, wsrc, ws, K, nproj, m_eff, tail, G, s, e0, e1);
  }
}

int launch_fused(const Csr& A, const Sell& SA, int shape, const Ws& ws, int rpt, int K, int nproj,
                 int wsrc, int m_eff, int tail, int G, int bt, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1) {
  const int rc =
      bt == kBasisF32    ? fused_v<float>(A, SA, shape, ws, rpt, K, nproj, wsrc, m_eff, tail, G, s, e0, e1)
      : bt == kBasisBf16 ? fused_v<__bf16>(A, SA, shape, ws, rpt, K, nproj, wsrc, m_eff, tail, G, s, e0, e1)
                         : fused_v<double>(A, SA, shape, ws, rpt, K, nproj, wsrc, m_eff, tail, G, s, e0, e1);
  if (rc) return rc;
  GMRES_CHECK_LAUNCH();
  return 0;
}

template <typename VT>
static void maxpy_v(const Ws& ws, int rpt, int k, int mode, int G, int side, int depth,
                    hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)(G + (side ? 1 : 0)));
  switch (rpt) {
    case 1: hipExtLaunchKernelGGL((k_maxpy<1, VT>), grid, dim3(256), 0u, s, e0, e1, 0u, ws, k, mode, G, side, depth); break;
    case 2: hipExtLaunchKernelGGL((k_maxpy<2, VT>), grid, dim3(256), 0u, s, e0, e1, 0u, ws, k, mode, G, side, depth); break;
    case 4: hipExtLaunchKernelGGL((k_maxpy<4, VT>), grid, dim3(256), 0u, s, e0, e1, 0u, ws, k, mode, G, side, depth); break;
    default: hipExtLaunchKernelGGL((k_maxpy<8, VT>), grid, dim3(256), 0u, s, e0, e1, 0u, ws, k, mode, G, side, depth); break;
  }
}

int launch_maxpy(const Ws& ws, int rpt, int k, int mode, int G, int bt, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1, int side, int depth) {
  if (side && (mode != 0 || (side != kSchemeMgs1r && side != kSchemeCgs2) || depth < 1)) return -2;
  if (bt == kBasisF32)
    maxpy_v<float>(ws, rpt, k, mode, G, side, depth, s, e0, e1);
  else if (bt == kBasisBf16)
    maxpy_v<__bf16>(ws, rpt, k, mode, G, side, depth, s, e0, e1);
  else
    maxpy_v<double>(ws, rpt, k, mode, G, side, depth, s, e0, e1);
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_axpy_dot(const Ws& ws, int rpt, double* w, const double* a, const double* coef,
                    const double* v, int tail, int i_col, int q_row, int m_eff, double aux, int G,
                    hipStream_t s) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL(k_axpy_dot<1>, dim3(G), dim3(256), 0, s, ws, w, a, coef, v, tail, i_col, q_row, m_eff, aux, G); break;
    case 2: hipLaunchKernelGGL(k_axpy_dot<2>, dim3(G), dim3(256), 0, s, ws, w, a, coef, v, tail, i_col, q_row, m_eff, aux, G); break;
    case 4: hipLaunchKernelGGL(k_axpy_dot<4>, dim3(G), dim3(256), 0, s, ws, w, a, coef, v, tail, i_col, q_row, m_eff, aux, G); break;
    default: hipLaunchKernelGGL(k_axpy_dot<8>, dim3(G), dim3(256), 0, s, ws, w, a, coef, v, tail, i_col, q_row, m_eff, aux, G); break;
  }
  GMRES_CHECK_LAUNCH();
  return 0;
}

int launch_scale(const Ws& ws, double* v, hipStream_t s) {
  int64_t blocks = (ws.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, s, ws, v);
  GMRES_CHECK_LAUNCH();
  return 0;
}

template <typename VT>
static void xupdate_v(const Ws& ws, int rpt, double* x, int G, hipStream_t s) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_xupdate<1, VT>), dim3(G), dim3(256), 0, s, ws, x, G); break;
    case 2: hipLaunchKernelGGL((k_xupdate<2, VT>), dim3(G), dim3(256), 0, s, ws, x, G); break;
    case 4: hipLaunchKernelGGL((k_xupdate<4, VT>), dim3(G), dim3(256), 0, s, ws, x, G); break;
    default: hipLaunchKernelGGL((k_xupdate<8, VT>), dim3(G), dim3(256), 0, s, ws, x, G); break;
  }
}

int launch_cycle_end(const Ws& ws, int rpt, double* x, int G, int bt, hipStream_t s) {
  // up to 48 KiB: R's leading block when it fits, g always
  size_t want = (size_t)(ws.m + 2) + (size_t)(ws.m + 1) * ws.m;
  const size_t cap = 48 * 1024 / sizeof(double);
  if (want > cap) want = cap;
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(256), want * sizeof(double), s, ws, (int)want);
  GMRES_CHECK_LAUNCH();
  if (bt == kBasisF32)
    xupdate_v<float>(ws, rpt, x, G, s);
  else if (bt == kBasisBf16)
    xupdate_v<__bf16>(ws, rpt, x, G, s);
  else
    xupdate_v<double>(ws, rpt, x, G, s);
  GMRES_CHECK_LAUNCH();
  return 0;
}

#include "gmres_batch_kernels.h"

size_t fused_lds_bytes(int rpt, int m) { return fused_lds_doubles(rpt, m) * sizeof(double); }

}  // namespace gmres

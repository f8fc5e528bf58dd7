// Bandwidth probes of this GPU (measurement only; not part of the solver):
// the achievable HBM rates of streaming reads and of copies, the two access
// patterns of the solver's step kernels, measured over buffers far larger
// than the last-level cache, in two orders: grid-stride (the whole grid
// sweeps the buffer together) and tiled (each workgroup streams a contiguous
// chunk of its own, 6-13% faster here). C ABI in include/gmres_probe.h.
#include "gmres_probe.h"

#include <hip/hip_runtime.h>

namespace {

// 16 bytes as one vector register pair: one dwordx4 load or store
typedef double d2 __attribute__((ext_vector_type(2)));

// Reads of 16-byte vectors, U in flight per thread and grid-stride pass;
// the per-thread sums are summed per wavefront and one value per workgroup is
// written, so no load can be dropped. NT: non-temporal loads.
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_read(const d2* __restrict__ a, int64_t n2,
                                               double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = t0;
  for (; i + (U - 1) * stride < n2; i += U * stride) {
    d2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT)
        v[u] = __builtin_nontemporal_load(a + i + u * stride);
      else
        v[u] = a[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s0 += v[u].x;
      s1 += v[u].y;
    }
  }
  for (; i < n2; i += stride) {
    const d2 v = a[i];
    s0 += v.x;
    s1 += v.y;
  }
  double s = s0 + s1;
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// b = a in 16-byte vectors, U in flight per thread; NT: non-temporal stores.
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy(const d2* __restrict__ a, d2* __restrict__ b,
                                               int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t i = t0;
  for (; i + (U - 1) * stride < n2; i += U * stride) {
    d2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = a[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT)
        __builtin_nontemporal_store(v[u], b + i + u * stride);
      else
        b[i + u * stride] = v[u];
    }
  }
  for (; i < n2; i += stride) b[i] = a[i];
}

// The same two patterns, tiled: workgroup b streams elements
// [b per, min(n2, (b + 1) per)) in order, U 16-byte vectors per thread in
// flight; the reads sum their values and write one double per wavefront
// (out needs 4 doubles per workgroup).
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_read_tiled(const d2* __restrict__ a, int64_t n2,
                                                     double* __restrict__ out) {
  const int64_t per = (n2 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n2 ? b0 + per : n2;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = b0 + threadIdx.x;
  for (; i + (U - 1) * 256 < b1; i += U * 256) {
    d2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT)
        v[u] = __builtin_nontemporal_load(a + i + u * 256);
      else
        v[u] = a[i + u * 256];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s0 += v[u].x;
      s1 += v[u].y;
    }
  }
  for (; i < b1; i += 256) {
    const d2 v = a[i];
    s0 += v.x;
    s1 += v.y;
  }
  double s = s0 + s1;
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) out[(int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy_tiled(const d2* __restrict__ a, d2* __restrict__ b,
                                                     int64_t n2) {
  const int64_t per = (n2 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n2 ? b0 + per : n2;
  int64_t i = b0 + threadIdx.x;
  for (; i + (U - 1) * 256 < b1; i += U * 256) {
    d2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT)
        v[u] = __builtin_nontemporal_load(a + i + u * 256);
      else
        v[u] = a[i + u * 256];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT)
        __builtin_nontemporal_store(v[u], b + i + u * 256);
      else
        b[i + u * 256] = v[u];
    }
  }
  for (; i < b1; i += 256) b[i] = a[i];
}

}  // namespace

extern "C" int gmres_probe_bandwidth(int32_t kind, const double* src, double* dst, int64_t nbytes,
                                     int32_t blocks, int32_t reps, void* hip_stream, float* ms) {
  if (kind < GMRES_PROBE_READ || kind > GMRES_PROBE_COPY_TILED_NT || !src || !dst || !ms ||
      nbytes < 16 || (nbytes % 16) != 0 || blocks < 1 || reps < 1)
    return -1;
  if (((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0) return -1;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n2 = nbytes / 16;
  const d2* a = (const d2*)src;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -2;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -2;
  }
  int rc = 0;
  for (int r = -1; r < reps && rc == 0; ++r) {  // one untimed launch first
    if (r == 0 && hipEventRecord(e0, s) != hipSuccess) rc = -2;
    switch (kind) {
      case GMRES_PROBE_READ:
        hipLaunchKernelGGL((k_read<4, false>), dim3(blocks), dim3(256), 0, s, a, n2, dst);
        break;
      case GMRES_PROBE_READ_NT:
        hipLaunchKernelGGL((k_read<4, true>), dim3(blocks), dim3(256), 0, s, a, n2, dst);
        break;
      case GMRES_PROBE_COPY:
        hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, a, (d2*)dst, n2);
        break;
      case GMRES_PROBE_COPY_NT:
        hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, s, a, (d2*)dst, n2);
        break;
      case GMRES_PROBE_READ_TILED:
        hipLaunchKernelGGL((k_read_tiled<4, false>), dim3(blocks), dim3(256), 0, s, a, n2, dst);
        break;
      case GMRES_PROBE_READ_TILED_NT:
        hipLaunchKernelGGL((k_read_tiled<4, true>), dim3(blocks), dim3(256), 0, s, a, n2, dst);
        break;
      case GMRES_PROBE_COPY_TILED:
        hipLaunchKernelGGL((k_copy_tiled<4, false>), dim3(blocks), dim3(256), 0, s, a, (d2*)dst, n2);
        break;
      default:
        hipLaunchKernelGGL((k_copy_tiled<4, true>), dim3(blocks), dim3(256), 0, s, a, (d2*)dst, n2);
        break;
    }
    if (hipGetLastError() != hipSuccess) rc = -2;
  }
  if (rc == 0 && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    rc = -2;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

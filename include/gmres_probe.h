/*
 * gmres_probe.h - bandwidth probes of the GPU, for measurement (not part of
 * the solver): the achievable rates of streaming 16-byte reads and copies
 * over a caller's buffers, the access patterns of the solver's step kernels.
 * The benchmark reports its kernels' rates against these and against the
 * 8 TB/s HBM peak. Built into libgmres_probe.so.
 */
#ifndef GMRES_PROBE_H
#define GMRES_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMRES_PROBE_READ = 0,           /* read nbytes of src, grid-stride; one double per workgroup to dst */
  GMRES_PROBE_READ_NT = 1,        /* the same with non-temporal loads                                 */
  GMRES_PROBE_COPY = 2,           /* copy nbytes from src to dst, grid-stride                         */
  GMRES_PROBE_COPY_NT = 3,        /* the same with non-temporal stores                                */
  GMRES_PROBE_READ_TILED = 4,     /* read, each workgroup streaming one contiguous chunk; 4 doubles
                                     per workgroup to dst                                              */
  GMRES_PROBE_READ_TILED_NT = 5,  /* the same with non-temporal loads                                 */
  GMRES_PROBE_COPY_TILED = 6,     /* copy, each workgroup streaming one contiguous chunk              */
  GMRES_PROBE_COPY_TILED_NT = 7   /* the same with non-temporal loads and stores                      */
};

/*
 * One untimed launch, then reps launches of the probe `kind` with `blocks`
 * workgroups of 256 threads, timed with HIP events on hip_stream (NULL: the
 * default stream); *ms (host) receives the elapsed time of the reps launches.
 * src, dst: device pointers, 16-byte aligned; nbytes a positive multiple of
 * 16. dst must hold nbytes for the copies, `blocks` doubles for the grid-stride
 * reads and 4 `blocks` doubles for the tiled reads;
 * the buffers must not overlap. Blocks until done. Returns 0, -1 for invalid
 * arguments, -2 for a HIP error.
 */
int gmres_probe_bandwidth(int32_t kind, const double* src, double* dst, int64_t nbytes,
                          int32_t blocks, int32_t reps, void* hip_stream, float* ms /* host */);

#ifdef __cplusplus
}
#endif

#endif /* GMRES_PROBE_H */

/*
 * lbm_probe.h -- measurement probes of the lattice Boltzmann engine (not part
 * of the method).  Each runs an access pattern of the step or adjoint kernels
 * without their arithmetic, or a plain copy, on caller-owned device memory,
 * and times it with HIP events on a private stream: they are the practical
 * ceilings the kernels of include/lbm.h are compared against.  Same return
 * codes as lbm.h; no solver handle is involved.
 */
#ifndef LBM_PROBE_H
#define LBM_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Measurement helper, not part of the method: copy `bytes` (a multiple of
 * 16) from src_dev to dst_dev `reps` times after one warm-up copy, on a
 * private stream, and report the mean time per copy from HIP events.  Used
 * as the practical HBM ceiling (read + write of `bytes`) that the step
 * kernels are compared against.  mode 0: grid-stride loop with four
 * independent 16-byte loads per thread and non-temporal stores; 1: one
 * 16-byte element per thread, non-temporal stores; 2: as 1 with ordinary
 * stores.  Both buffers are device memory owned by the caller and must not
 * overlap.  Errors: EINVAL, EDEVICE. */
int lbm_stream_copy(void *dst_dev, const void *src_dev, int64_t bytes,
                    int32_t mode, int32_t reps, double *ms_per_copy);

/* The step kernel's access pattern without its arithmetic, as a ceiling for
 * it.  The populations are stored as the engine stores them: blocks of 2048
 * consecutive nodes (x fastest, then y, then z), each holding its Q
 * direction runs one after the other, so that population i of node n sits at
 * element (n / 2048) * Q * 2048 + i * 2048 + n % 2048 (FP64 or FP32 per
 * `precision`).  Each population is read at the periodic pull source of its
 * direction (x - e_i wrapped in every axis, the step's own addressing) and
 * written at the node with non-temporal stores, one node per thread in
 * 256-thread blocks.  Runs `reps` times after one warm-up on a private
 * stream and reports the mean time per pass from HIP events (a pass moves
 * 2 * Q * nx*ny*nz * element bytes).  src_dev and dst_dev are caller-owned
 * device buffers of at least Q * P elements, P = nx*ny*nz rounded up to a
 * multiple of 2048, that must not overlap (elements of the last block past
 * nx*ny*nz are neither read nor written).  Errors: EINVAL (bad sizes or
 * lattice; D2Q9 needs nz = 1; one plane must stay below 4 GiB), EDEVICE. */
int lbm_pull_pattern_copy(int lattice, int precision, void *dst_dev, const void *src_dev,
                          int64_t nx, int64_t ny, int64_t nz, int32_t reps,
                          double *ms_per_copy);

/* The adjoint step's access pattern without its arithmetic, as above with
 * a second source: plane i of f_src is read at the pull source x - e_i, plane
 * i of lam_src at x + e_i (the node that pulls from x), and their sum is
 * written at x (a pass moves 3 * Q * nx*ny*nz * element bytes).  Same blocked
 * layout; the three buffers are caller-owned device memory of at least Q * P
 * elements; dst_dev must not overlap either source.  Errors as above. */
int lbm_adjoint_pattern_copy(int lattice, int precision, void *dst_dev, const void *f_src_dev,
                             const void *lam_src_dev, int64_t nx, int64_t ny, int64_t nz,
                             int32_t reps, double *ms_per_copy);

/* The step's pull pattern (as lbm_pull_pattern_copy) with a block size of
 * the caller's choice: consecutive blocks of `block` nodes (a power of two
 * from 64 to 2^30 that divides nx*ny*nz), each holding its Q direction runs
 * one after the other -- the element (i, n) at (n / block) * Q * block +
 * i * block + n % block; a block of nx*ny*nz nodes is the plain
 * one-plane-per-direction layout.  Used to choose the engine's block size.
 * Buffers of at least Q * nx*ny*nz elements; the whole array must stay below
 * 4 GiB.  Errors as lbm_pull_pattern_copy. */
int lbm_blocked_pull_pattern_copy(int lattice, int precision, int32_t block, void *dst_dev,
                                  const void *src_dev, int64_t nx, int64_t ny, int64_t nz,
                                  int32_t reps, double *ms_per_copy);

/* The in-place two-pass ("AA") access pattern on one buffer of Q planes of
 * nx*ny*nz elements (stride nx*ny*nz, periodic in every axis), one node per
 * thread in 256-thread blocks, non-temporal stores.  Even pass: node x reads
 * plane i at x and writes it into plane ibar at x.  Odd pass: node x reads
 * plane ibar at x - e_i and writes plane i at x + e_i (every location is read
 * and written by the same thread, so the pass is race-free in place).  After
 * one warm-up pair, `reps` pairs are timed; *ms_even and *ms_odd get the mean
 * time of each pass (each moves 2 * Q * nx*ny*nz elements).  buf_dev is
 * caller-owned device memory of at least Q * nx*ny*nz elements.  Errors as
 * lbm_pull_pattern_copy. */
int lbm_aa_pattern_copy(int lattice, int precision, void *buf_dev, int64_t nx, int64_t ny,
                        int64_t nz, int32_t reps, double *ms_even, double *ms_odd);

#ifdef __cplusplus
}
#endif

#endif /* LBM_PROBE_H */

/*
 * smoke.h -- C ABI of the differentiable incompressible smoke simulator on
 * MI355X (gfx950), part of the same library as mpm.h (libmpm.so).
 *
 * DiffTaichi (Hu et al., ICLR 2020), Section 4.2 and Table 2, builds this
 * simulator after the fluid example of Autograd: semi-Lagrangian advection
 * (Stam 1999) and a pressure projection by a fixed number of Jacobi
 * iterations on a periodic grid, differentiated through the unrolled
 * iterations (Appendix E.3). One time step, on an n x n periodic grid with one
 * value per cell, lengths in cells and velocities in cells per step:
 *   u*  = advect(u, u)    bilinear sample of each velocity component at the
 *                         back-traced point c - u(c), indices wrapped mod n;
 *   u'  = u* - grad(p^K)  p^0 = 0, p^k = (sum of the four neighbours of
 *                         p^(k-1) - div(u*)) / 4 (Jacobi on the 5-point
 *                         Poisson equation); div and grad central differences
 *                         (f[c + e] - f[c - e]) / 2;
 *   s'  = advect(s, u')   the smoke density, carried by the projected velocity.
 * The loss of the paper's optimisation is the summed squared difference of the
 * final density to a target image.
 *
 * Conventions are those of mpm.h: mpm_status results, caller-owned device
 * memory (16-byte aligned; the library never allocates), work enqueued on the
 * caller's stream, FP32 arithmetic (the loss sums in FP64), adjoint outputs
 * ACCUMULATE (Section 3, Appendix B).
 *
 * A state is three n x n FP32 planes, row-major with axis 0 slowest:
 * [u0 | u1 | s] (u0 the velocity along axis 0), 3 n^2 floats. A tape is
 * steps + 1 consecutive states; the forward writes all of them, the reverse
 * pass reads them (no recomputation: a state is 3 n^2 floats, 14.7 MB for
 * the whole 110^2, 100-step benchmark).
 */
#ifndef SMOKE_H_
#define SMOKE_H_

#include <stddef.h>
#include <stdint.h>

#include "mpm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Problem description (host struct, read during each call).
 *   n       cells per axis of the periodic square grid, 4..4096.
 *   steps   time steps T >= 1.
 *   iters   Jacobi iterations per projection K, 0..24 (Table 2 runs 6;
 *           Appendix E.3 mentions 10; 0 skips the projection).
 *   tile    launch shape (tuning; results agree up to FP32 rounding): tile
 *           edge of the per-step kernels, 8, 16 or 32 cells (64, 256 or
 *           1024 threads per workgroup), 0 for the default 16. */
typedef struct {
  int32_t n;
  int32_t steps;
  int32_t iters;
  int32_t tile;
} smoke_desc;

/* Device bytes of a tape: (steps + 1) * 3 * n^2 floats. 0 for an invalid desc. */
size_t smoke_tape_bytes(const smoke_desc* desc);

/* Device bytes of the workspace: three adjoint states (rotated through the
 * reverse pass), the FP64 loss accumulator and the error word. 0 for an
 * invalid desc. */
size_t smoke_workspace_bytes(const smoke_desc* desc);

/* Zeroes the workspace's error word (asynchronous). Call once after
 * allocating a workspace. */
mpm_status smoke_workspace_init(const smoke_desc* desc, void* workspace, void* stream);

/* Forward trajectory (Section 4.2): copies `init` (one state) into tape
 * state 0 and writes states 1..steps, one launch per step. A back-traced
 * point that is not finite samples its own cell and sets MPM_FLAG_NONFINITE
 * in the workspace's error word. MPM_E_ARG on an invalid desc or null
 * pointers. */
mpm_status smoke_forward(const smoke_desc* desc, const float* init, float* tape, void* workspace, void* stream);

/* Loss of the paper's optimisation on the final tape state:
 * *loss = sum_c (s_T(c) - target[c])^2 (device float, overwritten; summed in
 * FP64). If seed is non-null, OVERWRITES it (one state) with dL/d(state T):
 * zero velocity planes, 2 (s_T - target) on the smoke plane. */
mpm_status smoke_loss(const smoke_desc* desc, const float* tape, const float* target, float* loss, float* seed,
                      void* workspace, void* stream);

/* Reverse pass over a tape written by smoke_forward with the same desc
 * (Appendix E.3: back through the unrolled Jacobi iterations): given
 * seed = dL/d(state T) (one state), ADDS dL/d(state 0) into grad (one state),
 * one launch per step. The workspace is overwritten (except the error word). */
mpm_status smoke_backward(const smoke_desc* desc, const float* tape, const float* seed, float* grad,
                          void* workspace, void* stream);

/* Synchronises `stream`, reads and clears the workspace's error word. */
mpm_status smoke_check_errors(const smoke_desc* desc, void* workspace, void* stream, uint32_t* flags);

#ifdef __cplusplus
}
#endif

#endif /* SMOKE_H_ */

/*
 * mpm.h -- C ABI of the MI355X (gfx950) differentiable MLS-MPM library.
 *
 * The library computes the hot path of the differentiable elastic-object
 * simulator of DiffTaichi (Hu et al., ICLR 2020), Section 4.1: one
 * moving-least-squares MPM time step -- particle-to-grid scatter of APIC
 * momentum, mass and neo-Hookean stress, a grid update, and a grid-to-particle
 * gather that updates v, C, x and F -- and its reverse-mode adjoint, replayed
 * from a tape with the grid recomputed inside each adjoint step (Appendix D.1)
 * and with segment checkpoints (Appendix D.2).
 *
 * Conventions (all entry points):
 *   - Every entry point returns an mpm_status; MPM_OK (0) is success.
 *     Argument errors are detected on the host before any HIP call and leave
 *     device memory untouched. MPM_E_HIP reports a failed HIP runtime call.
 *   - All device pointers are owned by the caller (typically torch tensors);
 *     the library never calls hipMalloc or hipFree. Device buffers must be
 *     16-byte aligned. Host pointers are read only during the call.
 *   - Work is enqueued asynchronously on the caller's stream unless stated.
 *     A context serves one stream at a time and is not thread-safe.
 *   - Device arithmetic is FP32 (gradient reductions over particles use FP64
 *     accumulators).
 *   - Adjoint outputs ACCUMULATE: for a primal f(X) = Y the adjoint takes
 *     (X, Y*) and adds dL/dX into X* (Section 3, Appendix B). Callers zero the
 *     gradient buffers they want to read as plain gradients.
 *   - Particle state (mpm_state) is structure-of-arrays, component-major:
 *     x[d][N], v[d][N], C[d*d][N], F[d*d][N] (C and F row-major in (a, b)),
 *     so component c of particle p is at ptr[c * N + p]. N is the total
 *     particle count of the context; scene k owns particles
 *     [scene_offsets[k], scene_offsets[k+1]).
 *   - Device-side faults of the physics (a particle whose 3^d stencil leaves
 *     the grid, det F <= 0, a non-finite state) set bits of a device error
 *     word; mpm_check_errors reads and clears it. Such particles are skipped
 *     by the scatter and keep their state.
 */
#ifndef MPM_H_
#define MPM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mpm_status;
enum {
  MPM_OK = 0,
  MPM_E_ARG = 1,        /* invalid argument (null, out of range, mismatched sizes)          */
  MPM_E_CAPACITY = 2,   /* bound workspace or tape memory is too small                      */
  MPM_E_TAPE = 3,       /* tape misuse: backward before forward, different params, unbound  */
  MPM_E_HIP = 4,        /* a HIP runtime call failed                                        */
  MPM_E_DOMAIN = 5,     /* device flag: a particle stencil left the grid                    */
  MPM_E_INVERTED = 6,   /* device flag: det F <= 0                                          */
  MPM_E_NONFINITE = 7,  /* device flag: non-finite particle state                           */
  MPM_E_STATE = 8       /* call order: workspace not bound                                  */
};

/* Device error-word bits reported by mpm_check_errors. */
#define MPM_FLAG_DOMAIN 1u
#define MPM_FLAG_INVERTED 2u
#define MPM_FLAG_NONFINITE 4u

typedef struct mpm_ctx mpm_ctx;
typedef struct mpm_tape mpm_tape;

/* Simulation description. Section 4.1 names the method (MLS-MPM after
 * ChainQueen) but no constants; these fields carry them.
 *   dim           2 or 3.
 *   n_grid        nodes per axis (>= 2*bound + 3); nodes sit at i*dx.
 *   bound         sticky band width: a node whose index on any axis is
 *                 < bound or >= n_grid - bound gets velocity 0.
 *   dx, dt        cell size and time step.
 *   gravity       acceleration along axis 1 ("up"), e.g. -9.8.
 *   n_scenes      independent scenes, each with its own n_grid^dim grid.
 *   scene_offsets host array [n_scenes + 1], non-decreasing, offsets[0] = 0;
 *                 N = scene_offsets[n_scenes] >= 1.
 *   n_actuators   actuator columns (0..16); act_strength sigma_a multiplies
 *                 the actuation a_k(s) added to the yy Kirchhoff stress.
 *   flags         0 or MPM_MODEL_COROTATED; other bits give MPM_E_ARG.
 *
 * Constitutive model (Kirchhoff stress tau, initial particle volume): by
 * default compressible neo-Hookean, tau = mu (F F^T - I) + lambda ln(J) I.
 * With MPM_MODEL_COROTATED, fixed-corotated, tau = 2 mu (F - R) F^T +
 * lambda (J - 1) J I with R the rotation of the polar decomposition F = R S;
 * its reverse pass differentiates the decomposition by hand (the custom
 * gradients of Section 3 and Appendix C). An inverted F (J <= 0) sets
 * MPM_FLAG_INVERTED and, for this model, carries no stress. */
#define MPM_MODEL_COROTATED 1u
typedef struct {
  int32_t dim;
  int32_t n_grid;
  int32_t bound;
  float dx;
  float dt;
  float gravity;
  int32_t n_scenes;
  const int32_t* scene_offsets;
  int32_t n_actuators;
  float act_strength;
  uint32_t flags;
} mpm_desc;

/* Particle state: device SoA pointers, each component-major with stride N. */
typedef struct {
  float* x; /* [dim][N]     */
  float* v; /* [dim][N]     */
  float* C; /* [dim*dim][N] */
  float* F; /* [dim*dim][N] */
} mpm_state;

/* Material and actuation parameters (device pointers).
 *   E, nu    [n_scenes] Young's modulus and Poisson ratio; Lame parameters
 *            mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)).
 *   vol      [n_scenes] initial particle volume V_p.
 *   rho      [n_scenes] density; particle mass m_p = rho * vol.
 *   act_id   [N] actuator column of each particle (-1: none) or NULL.
 *   act      [n_steps][n_actuators] actuation values a_k(s) or NULL. For the
 *            single-step calls, row `step` is used.
 *   mat_id   [N] material of each particle or NULL (all solid): 0 solid (the
 *            context's constitutive model), 1 weakly compressible liquid
 *            (Appendix E.1 couples one with the elastic robot through the
 *            shared grid): Tait pressure p = E (J^-7 - 1), Kirchhoff stress
 *            tau = -p J I, the scene's E acting as the bulk modulus. */
typedef struct {
  const float* E;
  const float* nu;
  const float* vol;
  const float* rho;
  const int32_t* act_id;
  const float* act;
  const int32_t* mat_id;
} mpm_params;

/* Gradients with respect to the parameters (device pointers, accumulate).
 *   E    [n_scenes] dL/dE or NULL.
 *   act  [n_steps][n_actuators] dL/da_k(s) or NULL. */
typedef struct {
  float* E;
  float* act;
} mpm_param_grad;

/* Status text (static string). Support call: the paper defines no error
 * reporting. */
const char* mpm_status_string(mpm_status s);

/* Creates a context for the description (Section 4.1's simulator: grid,
 * time step, scenes; the paper's kernels take these as compile-time
 * constants). Host-only: validates the fields, copies scene_offsets and sizes
 * the workspace. MPM_E_ARG on invalid fields. */
mpm_status mpm_init(const mpm_desc* desc, mpm_ctx** out);

/* Destroys the context (host objects only; never frees caller memory).
 * Support call. */
void mpm_destroy(mpm_ctx* ctx);

/* Bytes of device workspace the context needs (grids, sort buffers, adjoint
 * scratch, FP64 reduction accumulators, error word); 0 for a null ctx.
 * Support call (memory management; Appendix D.1 is why it holds grids for
 * only a few steps: the reverse pass recomputes each grid). */
size_t mpm_workspace_bytes(const mpm_ctx* ctx);

/* Binds caller-owned device workspace of at least mpm_workspace_bytes bytes
 * (256-byte aligned) and initialises it (synchronously on the null stream).
 * MPM_E_CAPACITY if too small, MPM_E_ARG if misaligned. Support call. */
mpm_status mpm_bind_workspace(mpm_ctx* ctx, void* dev, size_t bytes);

/* Sets a knob (support call: launch shape and measurement switches; none
 * changes what is computed beyond FP32 rounding order): "block" (threads per workgroup of the per-particle kernels:
 * 64, 128, 192 or 256); "lds" (0/1, default 1: stage each workgroup's stencil
 * footprint in LDS when it fits, else use global memory directly); "split"
 * (0/1, default 1: run the reverse launch's grid recompute for the previous
 * step in workgroups of its own, beside the adjoint workgroups); "remap"
 * (0/1: interleave each workgroup's sorted particles across its waves so
 * that fewer lanes add to one LDS node at a time); "rotate" (0/1, default
 * 1: each lane of a wave visits its 3^d stencil nodes in an order set by its
 * lane index, so lanes rarely add to the same node in the same instruction);
 * "lanes" (1, 2 or 4, default 1: lanes per particle in the step kernels;
 * with 2, each lane of a pair visits half of the 3^d stencil (one in reverse
 * order) and the pair sums its gathers; with 4, three lanes each take one
 * slab and the quad sums its gathers; both raise parallelism for small
 * particle counts); "part" (0/1, default 1: after each sort, cut the
 * particles into workgroups along the Morton cell hierarchy, each packing
 * consecutive child blocks of one block, so a workgroup's stencil footprint
 * stays compact when particle density varies; the launch then has room for
 * up to twice the plain number of workgroups, the unused ones empty; with 0,
 * workgroups are runs of consecutive sorted particles);
 * "tile_stats" (0/1, default 0: count scatter tiles, see mpm_tile_stats);
 * "persist" (0/1, default 0: run the step launches of a full tape's forward
 * and of its reverse pass each as one cooperative persistent launch, the
 * workgroups looping over each step's workgroups and meeting at a grid-wide
 * barrier between steps; same work and arithmetic as the launch per step;
 * checkpointed tapes keep one launch per step; graphs are not used);
 * "graph" (0/1, default 1:
 * capture each tape forward/backward launch sequence once in a HIP graph on
 * an internal stream and replay it on the caller's stream; the cache is keyed
 * on every pointer the sequence uses); "timing" (0/1: bracket every run of consecutive
 * launches of one step kernel on one stream with a pair of HIP events on that stream, for
 * mpm_kernel_stats; tape sequences then launch directly instead of replaying a graph).
 * MPM_E_ARG on an unknown key or value. */
mpm_status mpm_set_knob(mpm_ctx* ctx, const char* key, int64_t value);

/* Step-kernel timing (measurement support, not part of the method): kernel 0
 * is the forward step kernel, 1 the reverse step kernel. Waits for the
 * recorded events, returns the summed duration in ms of the timed runs of
 * that kernel and the number of launches they hold, since the previous call
 * for that kernel, and resets them. Requires the "timing" knob; otherwise
 * returns zeros. */
#define MPM_KERNEL_FWD 0
#define MPM_KERNEL_BWD 1
mpm_status mpm_kernel_stats(mpm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Scatter-tile counters (measurement support, not part of the method): with
 * the knob "tile_stats" on, every workgroup's scatter (the forward's p2g, the
 * reverse pass's g2p* and p2g recompute) counts whether it accumulated in an
 * LDS tile or fell back to global atomics (its stencils' box exceeded the
 * tile, or held particles of another box). Synchronises `stream`, returns the
 * counts since the previous call and resets them. */
mpm_status mpm_tile_stats(mpm_ctx* ctx, void* stream, int64_t* lds_scatters, int64_t* fallback_scatters);

/* Workgroup wall clocks (measurement support, not part of the method). Binds
 * a caller-owned device buffer of `bytes` bytes (or turns the clocks off when
 * buf is null) and restarts the launch count. Every later launch of a step
 * kernel (enqueued directly or captured into a graph; not the persistent form)
 * takes the next row of the buffer, while rows are left: row r, workgroup w
 * holds two uint64 stamps of the device's constant-rate clock at
 * ((uint64_t*)buf)[2 * (r * stride + w)], taken when the workgroup starts and
 * when all its waves have finished. stride = 2 * (workgroups of one particle
 * pass) at bind time; a launch wider than that (after a launch-shape knob
 * change) is not stamped. A replayed graph writes the rows its capture took.
 * MPM_E_ARG on a null ctx or a buffer smaller than one row. */
mpm_status mpm_wg_clock_bind(mpm_ctx* ctx, void* buf, size_t bytes);

/* Rows taken since the last bind: *launches rows; for row r < max_rows,
 * kind[r] (MPM_KERNEL_FWD / MPM_KERNEL_BWD) and wgs[r] (its workgroups: a
 * forward launch's stepping workgroups, followed, when they fill at most half
 * of the device's compute units, by as many that only clear grid memory; a
 * reverse launch's adjoint workgroups, then its recompute workgroups); the
 * row stride in workgroups (with no buffer bound: the stride a bind would
 * take now) and the clock's rate in kHz (the device's wall clock rate). Any
 * output pointer may be null. */
mpm_status mpm_wg_clock_info(const mpm_ctx* ctx, int32_t* launches, int32_t* stride, int32_t* kind, int32_t* wgs,
                             int32_t max_rows, int32_t* rate_khz);

/* Atomic-layout microbenchmark (measurement support, not part of the method):
 * enqueues `launches` back-to-back launches on `stream`, each of 128
 * workgroups of 256 threads adding a 7 x 7 x 5 box of grid nodes of four
 * floats into `grid` (caller-owned device memory of 4 * n^3 floats, n >= 34,
 * node index z fastest, contents overwritten with meaningless sums), the
 * boxes overlapping by three nodes along each axis like the scatter boxes of
 * the 3D lattice workload. layout 0: one node per lane, one atomic instruction
 * per component (the scatter-tile flush's earlier layout); 1: lanes over
 * (node, component), component fastest (the flush's layout); 2: layout 1
 * with plain stores; 3: no memory operation (launch cost only). The caller
 * times the launches (events around the call). MPM_E_ARG on a null grid, n
 * outside 34..1024, a negative count or an unknown layout. */
mpm_status mpm_diag_box_atomics(int32_t layout, float* grid, int32_t n, int32_t launches, void* stream);

/* One forward step, state `in` (step `step`) -> `out` (step + 1), in the
 * caller's particle order: clear_grid, compute_actuation (row `step` of
 * params->act), p2g, grid_op, g2p (Appendix D.1 stage order). `in` and `out`
 * must not alias (each state is written once: the Global Data Access Rules of
 * Section 3). */
mpm_status mpm_step_fwd(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in,
                        mpm_state* out, void* stream);

/* mpm_step_fwd for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, and harnesses that forbid
 * allocation. Same step, same kernels and launch shape, same arguments, plus
 * err_flags; the context needs no bound workspace (a context from mpm_init
 * alone will do). Instead of the workspace, the step uses a fixed device
 * array inside the library, 64 MiB per GPU, allocated when the library's
 * code is loaded on that GPU and held until the process ends: it holds the
 * grid (n_scenes * n_grid^dim * 16 bytes) and, for several scenes, the
 * workgroup table (16 bytes per workgroup). MPM_E_CAPACITY, before any GPU
 * work, when those exceed 64 MiB (one 160^3 grid, 62.5 MiB, fits; 170^3 does not).
 * Allocates nothing: no hipMalloc or hipFree, no allocating library call.
 * The array of the current device is used (the stream must belong to it);
 * its address is looked up on the first call per device. Every call on one
 * GPU, from any context, shares that GPU's array and leaves its content
 * behind; each call clears the grid it uses. Calls that overlap on one GPU
 * (other streams, other host threads) race on the array and must be
 * serialised by the caller.
 *   err_flags  device uint32, caller-owned: MPM_FLAG_* bits of particles
 *              that left the grid, were inverted or not finite are OR-ed in
 *              (the caller clears it); MPM_E_ARG if null.
 * The knob "timing" is ignored by this call. */
mpm_status mpm_step_fwd_noalloc(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in,
                                mpm_state* out, uint32_t* err_flags, void* stream);

/* Adjoint of one step (Appendix D.1): recomputes the grid from `in`, then
 * replays g2p*, grid_op*, p2g*; given out_grad = dL/d(state step+1) it ADDS
 * dL/d(state step) into in_grad and dL/dE, dL/da(step) into pg. */
mpm_status mpm_step_bwd(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in,
                        const mpm_state* out_grad, mpm_state* in_grad, mpm_param_grad* pg, void* stream);

/* A tape over n_steps steps (Section 3.2: the tape records the step launches
 * and replays their adjoints in reverse). ckpt_every = 0 or >= n_steps keeps
 * every state (full tape); 0 < ckpt_every < n_steps keeps states 0, K, 2K, ...
 * plus a ring of 2K working slots, and recomputes each segment from its
 * checkpoint during the reverse pass (Appendix D.2). Host-only. */
mpm_status mpm_tape_create(mpm_ctx* ctx, int32_t n_steps, int32_t ckpt_every, mpm_tape** out);

/* Bytes of device memory the tape needs (state slots + FP64 accumulators):
 * T + 1 states for a full tape, or the checkpoints of Appendix D.2 plus the
 * ring of recomputed states. Support call. */
size_t mpm_tape_bytes(const mpm_tape* tape);

/* Binds caller-owned tape memory (>= mpm_tape_bytes, 256-byte aligned).
 * Support call. */
mpm_status mpm_tape_bind(mpm_tape* tape, void* dev, size_t bytes);

/* Destroys the tape's host objects. Support call. */
void mpm_tape_destroy(mpm_tape* tape);

/* Runs n_steps forward steps from `init` (caller order) and writes the final
 * state to `final` (caller order). Internally particles are sorted by scene
 * and cell (Morton order, as mpm_sort_order) once, at step 0, and the tape
 * keeps sorted states together with the permutation, the sorted actuator and
 * material ids and the workgroup table of that order. Records the parameter
 * pointers and the launch shape (knobs "block", "lanes", "part") for the
 * reverse pass. A second forward on the same tape replaces the recorded
 * trajectory. */
mpm_status mpm_tape_forward(mpm_tape* tape, const mpm_params* params, const mpm_state* init, mpm_state* final_state,
                            void* stream);

/* Reverse pass over the recorded trajectory: given final_grad = dL/d(final
 * state) (caller order), ADDS dL/d(init) into init_grad (caller order) and
 * dL/dE, dL/da into pg. MPM_E_TAPE if no forward was recorded, if params
 * differ from the recorded ones, or if the launch shape changed since the
 * forward. May be called repeatedly after one forward; other tapes of the
 * same context may run in between. */
mpm_status mpm_tape_backward(mpm_tape* tape, const mpm_params* params, const mpm_state* final_grad,
                             mpm_state* init_grad, mpm_param_grad* pg, void* stream);

/* Binning (support call; the paper's Taichi layouts leave the particle order
 * to the compiler): the order in which the tape keeps particles. Sorts the
 * particles of `state` by (scene, cell), cells ordered along the Morton curve
 * of the scene's grid (cell c_a = floor(x_a / dx) clamped into [0, n_grid - 1],
 * NaN to 0; axis 0 the most significant bit of each level), keeping the
 * caller's order among particles of one cell, and writes perm[j] = caller
 * index of the j-th particle in that order (device int32[N], overwritten).
 * Asynchronous on `stream`. */
mpm_status mpm_sort_order(mpm_ctx* ctx, const mpm_state* state, int32_t* perm, void* stream);

/* Loss on a final state (the pattern of the paper's compute_loss kernel):
 * kind MPM_LOSS_MEAN_POS gives, per scene k, L_k = sign * mean_p x_{p,axis}.
 * Writes loss_dev[n_scenes] (device, overwritten) and, if seed is non-null,
 * OVERWRITES every component of *seed with dL/d(final state), where
 * L = sum_k L_k (so x-seed = sign / N_k on `axis`, zero elsewhere). With
 * uniform particle mass per scene this is also the centre-of-mass loss, so no
 * separate mass-weighted kind exists: particle mass is per scene (rho * vol of
 * mpm_params), and a mass-weighted mean equals the plain one. */
#define MPM_LOSS_MEAN_POS 0
mpm_status mpm_loss(mpm_ctx* ctx, int32_t kind, int32_t axis, float sign, const mpm_state* final_state,
                    float* loss_dev, mpm_state* seed, void* stream);

/* Open-loop actuation signal (the controller of the 2D soft robot, Section
 * 4.1): act[s][k] = tanh(sum_j W[k][j] sin(omega s dt + 2 pi j / n_sin)
 * + b[k]) for s < n_steps, k < n_actuators (device buffers, act overwritten). */
mpm_status mpm_actuation(mpm_ctx* ctx, const float* W, const float* b, int32_t n_sin, float omega,
                         int32_t n_steps, float* act, void* stream);

/* Adjoint of mpm_actuation: ADDS dL/dW [n_actuators][n_sin] and dL/db
 * [n_actuators] given gact = dL/dact [n_steps][n_actuators]. */
mpm_status mpm_actuation_bwd(mpm_ctx* ctx, const float* W, const float* b, int32_t n_sin, float omega,
                             int32_t n_steps, const float* gact, float* gW, float* gb, void* stream);

/* Support call (the paper defines no error reporting): synchronises
 * `stream`, reads and clears the device error word. *flags gets
 * the MPM_FLAG_* bits; the return value maps the lowest set bit to
 * MPM_E_DOMAIN / MPM_E_INVERTED / MPM_E_NONFINITE (MPM_OK if none). */
mpm_status mpm_check_errors(mpm_ctx* ctx, void* stream, uint32_t* flags);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H_ */

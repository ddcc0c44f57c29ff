// Host side and C ABI of the differentiable incompressible smoke simulator
// (include/smoke.h). One forward launch and one reverse launch per time step;
// the tape holds every state, so the reverse pass recomputes nothing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "smoke.h"
#include "smoke_kernels.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool desc_ok(const smoke_desc* d) {
  if (!d) return false;
  if (d->n < 4 || d->n > 4096 || d->steps < 1 || d->iters < 0 || d->iters > smoke::kMaxIters) return false;
  return d->tile == 0 || d->tile == 8 || d->tile == 16 || d->tile == 32;
}

int tile_of(const smoke_desc* d) { return d->tile ? d->tile : 16; }

size_t state_floats(const smoke_desc* d) { return size_t(3) * size_t(d->n) * size_t(d->n); }

// Workspace: three adjoint states, the FP64 loss accumulator, the error word.
struct Ws {
  float* g[3];
  double* acc;
  unsigned* err;
};

size_t ws_state_bytes(const smoke_desc* d) { return align_up(state_floats(d) * sizeof(float)); }

Ws ws_of(const smoke_desc* d, void* base) {
  char* b = static_cast<char*>(base);
  const size_t sb = ws_state_bytes(d);
  Ws w;
  for (int k = 0; k < 3; ++k) w.g[k] = reinterpret_cast<float*>(b + k * sb);
  w.acc = reinterpret_cast<double*>(b + 3 * sb);
  w.err = reinterpret_cast<unsigned*>(b + 3 * sb + kAlign);
  return w;
}

bool aligned(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

#define HIP_TRY(expr)                           \
  do {                                          \
    if ((expr) != hipSuccess) return MPM_E_HIP; \
  } while (0)

#define LAUNCH_TRY()                                       \
  do {                                                     \
    if (hipGetLastError() != hipSuccess) return MPM_E_HIP; \
  } while (0)

template <int TS>
mpm_status launch_fwd(const smoke_desc* d, const float* in, float* out, unsigned* err, hipStream_t s) {
  const int g = (d->n + TS - 1) / TS;
  const size_t lds = size_t(smoke::lds_floats(TS, d->iters)) * sizeof(float);
  hipLaunchKernelGGL(smoke::k_smoke_fwd<TS>, dim3(g, g), dim3(TS * TS), lds, s, in, out, d->n, d->iters, err);
  LAUNCH_TRY();
  return MPM_OK;
}

template <int TS>
mpm_status launch_bwd(const smoke_desc* d, const float* st, const float* nx, const float* gnext, float* gout,
                      float* gclear, unsigned* err, hipStream_t s) {
  const int g = (d->n + TS - 1) / TS;
  const size_t lds = size_t(smoke::lds_floats(TS, d->iters)) * sizeof(float);
  hipLaunchKernelGGL(smoke::k_smoke_bwd<TS>, dim3(g, g), dim3(TS * TS), lds, s, st, nx, gnext, gout, gclear, d->n,
                     d->iters, err);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status fill(float* p, size_t n, hipStream_t s) {
  const int blocks = int(std::min<size_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(smoke::k_smoke_fill, dim3(blocks), dim3(256), 0, s, p, n, 0.0f);
  LAUNCH_TRY();
  return MPM_OK;
}

}  // namespace

extern "C" {

size_t smoke_tape_bytes(const smoke_desc* desc) {
  if (!desc_ok(desc)) return 0;
  return size_t(desc->steps + 1) * state_floats(desc) * sizeof(float);
}

size_t smoke_workspace_bytes(const smoke_desc* desc) {
  if (!desc_ok(desc)) return 0;
  return 3 * ws_state_bytes(desc) + 2 * kAlign;
}

mpm_status smoke_workspace_init(const smoke_desc* desc, void* workspace, void* stream) {
  if (!desc_ok(desc) || !workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return MPM_E_ARG;
  const Ws w = ws_of(desc, workspace);
  hipLaunchKernelGGL(smoke::k_smoke_fill, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<float*>(w.err), size_t(1), 0.0f);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status smoke_forward(const smoke_desc* desc, const float* init, float* tape, void* workspace, void* stream) {
  if (!desc_ok(desc) || !init || !tape || !workspace) return MPM_E_ARG;
  if (!aligned(init) || !aligned(tape) || reinterpret_cast<uintptr_t>(workspace) % kAlign) return MPM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = ws_of(desc, workspace);
  const size_t sf = state_floats(desc);
  HIP_TRY(hipMemcpyAsync(tape, init, sf * sizeof(float), hipMemcpyDeviceToDevice, s));
  const int ts = tile_of(desc);
  for (int t = 0; t < desc->steps; ++t) {
    const float* in = tape + size_t(t) * sf;
    float* out = tape + size_t(t + 1) * sf;
    mpm_status st = ts == 8 ? launch_fwd<8>(desc, in, out, w.err, s)
                            : (ts == 32 ? launch_fwd<32>(desc, in, out, w.err, s) : launch_fwd<16>(desc, in, out, w.err, s));
    if (st != MPM_OK) return st;
  }
  return MPM_OK;
}

mpm_status smoke_loss(const smoke_desc* desc, const float* tape, const float* target, float* loss, float* seed,
                      void* workspace, void* stream) {
  if (!desc_ok(desc) || !tape || !target || !loss || !workspace) return MPM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = ws_of(desc, workspace);
  const size_t nn = size_t(desc->n) * desc->n;
  const float* fin = tape + size_t(desc->steps) * state_floats(desc);
  hipLaunchKernelGGL(smoke::k_smoke_zero_acc, dim3(1), dim3(64), 0, s, w.acc);
  LAUNCH_TRY();
  const int blocks = int(std::min<size_t>((nn + 255) / 256, 1024));
  hipLaunchKernelGGL(smoke::k_smoke_loss, dim3(blocks), dim3(256), 0, s, fin, target, desc->n, w.acc, seed);
  LAUNCH_TRY();
  hipLaunchKernelGGL(smoke::k_smoke_loss_out, dim3(1), dim3(64), 0, s, w.acc, loss);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status smoke_backward(const smoke_desc* desc, const float* tape, const float* seed, float* grad, void* workspace,
                          void* stream) {
  if (!desc_ok(desc) || !tape || !seed || !grad || !workspace) return MPM_E_ARG;
  if (!aligned(tape) || !aligned(seed) || !aligned(grad) || reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return MPM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = ws_of(desc, workspace);
  const size_t sf = state_floats(desc);
  const int T = desc->steps;
  // Adjoint of state t lives in g[t % 3] (state T: the caller's seed; state
  // 0: the caller's grad, accumulated into directly). The launch of step t
  // reads g[(t + 1) % 3], adds into g[t % 3] and zeroes g[(t - 1) % 3] for
  // the next launch.
  if (T >= 2) {
    mpm_status st = fill(w.g[(T - 1) % 3], sf, s);
    if (st != MPM_OK) return st;
  }
  const int ts = tile_of(desc);
  for (int t = T - 1; t >= 0; --t) {
    const float* gnext = (t + 1 == T) ? seed : w.g[(t + 1) % 3];
    float* gout = (t == 0) ? grad : w.g[t % 3];
    float* gclear = (t >= 2) ? w.g[(t - 1) % 3] : nullptr;
    const float* st_t = tape + size_t(t) * sf;
    const float* st_n = tape + size_t(t + 1) * sf;
    mpm_status st = ts == 8 ? launch_bwd<8>(desc, st_t, st_n, gnext, gout, gclear, w.err, s)
                            : (ts == 32 ? launch_bwd<32>(desc, st_t, st_n, gnext, gout, gclear, w.err, s)
                                        : launch_bwd<16>(desc, st_t, st_n, gnext, gout, gclear, w.err, s));
    if (st != MPM_OK) return st;
  }
  return MPM_OK;
}

mpm_status smoke_check_errors(const smoke_desc* desc, void* workspace, void* stream, uint32_t* flags) {
  if (!desc_ok(desc) || !workspace) return MPM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = ws_of(desc, workspace);
  HIP_TRY(hipStreamSynchronize(s));
  unsigned v = 0;
  HIP_TRY(hipMemcpy(&v, w.err, sizeof(unsigned), hipMemcpyDeviceToHost));
  const unsigned zero = 0;
  HIP_TRY(hipMemcpy(w.err, &zero, sizeof(unsigned), hipMemcpyHostToDevice));
  if (flags) *flags = v;
  return (v & MPM_FLAG_NONFINITE) ? MPM_E_NONFINITE : MPM_OK;
}

}  // extern "C"

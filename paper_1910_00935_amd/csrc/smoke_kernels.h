// Kernels of the differentiable incompressible smoke simulator (gfx950).
//
// The simulator of DiffTaichi's Section 4.2 (after the fluid example of
// Autograd): on a periodic n x n grid with one value per cell, one time step
// advects the velocity by itself semi-Lagrangianly (bilinear sample at the
// back-traced point c - u(c), in cells, velocities in cells per step),
// projects it with K Jacobi sweeps on the 5-point Poisson equation for the
// central-difference divergence (p^0 = 0), subtracts the central-difference
// pressure gradient, and advects the smoke density by the projected velocity.
// Appendix E.3 differentiates through the unrolled sweeps; here the adjoint of
// every stage is written by hand.
//
// One launch per time step in each direction. The projection couples every
// cell to its neighbours K + 1 cells away, so a workgroup owns a TS x TS tile
// and computes the self-advected velocity on the tile grown by a halo of
// K + 1 cells; the divergence and the sweeps then run in LDS on regions that
// shrink by one cell per sweep, and end on the tile plus one (trading
// redundant halo work for a launch without any grid-wide synchronisation).
// Advection reads the previous state at arbitrary back-traced points straight
// from global memory (the whole state stays resident in L2 at benchmark size).
//
// Reverse launch for step s: the adjoint of the smoke advection (its
// position term is local to each cell; its field term scatters into the
// smoke adjoint of state s), the projection's adjoint on the same shrinking
// halo (linear; no pressure is stored or recomputed), and the adjoint of the
// self-advection (scattered into the velocity adjoint of state s). Scatters
// are FP32 global atomics into buffers zeroed one launch ahead.
#pragma once

#include <hip/hip_runtime.h>

namespace smoke {

constexpr int kMaxIters = 24;     // Jacobi sweeps per projection
constexpr unsigned kErrNonfinite = 4u;

__device__ __forceinline__ int wrap(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Bilinear sample of the back-traced point (i, j) - (v0, v1): its lower
// corner (a0, b0), the next corners (a1, b1), wrapped, and its fractions.
// A point that is not finite or is more than 2^22 cells away samples the cell
// itself and raises the non-finite flag (all indices stay inside the grid).
struct Sample {
  int a0, a1, b0, b1;
  float fa, fb;
};

__device__ __forceinline__ Sample back_trace(int i, int j, float v0, float v1, int n, unsigned& err) {
  float y0 = float(i) - v0, y1 = float(j) - v1;
  if (!(fabsf(y0) < 4194304.0f && fabsf(y1) < 4194304.0f)) {
    err |= kErrNonfinite;
    y0 = float(i);
    y1 = float(j);
  }
  const float f0 = floorf(y0), f1 = floorf(y1);
  Sample s;
  s.fa = y0 - f0;
  s.fb = y1 - f1;
  s.a0 = wrap(int(f0), n);
  s.b0 = wrap(int(f1), n);
  s.a1 = (s.a0 + 1 == n) ? 0 : s.a0 + 1;
  s.b1 = (s.b0 + 1 == n) ? 0 : s.b0 + 1;
  return s;
}

struct Corners {
  float c00, c01, c10, c11;  // f[a0][b0], f[a0][b1], f[a1][b0], f[a1][b1]
};

__device__ __forceinline__ Corners corners(const float* __restrict__ f, const Sample& s, int n) {
  const float* r0 = f + size_t(s.a0) * n;
  const float* r1 = f + size_t(s.a1) * n;
  return Corners{r0[s.b0], r0[s.b1], r1[s.b0], r1[s.b1]};
}

__device__ __forceinline__ float lerp2(const Corners& c, const Sample& s) {
  const float lo = c.c00 + s.fb * (c.c01 - c.c00);
  const float hi = c.c10 + s.fb * (c.c11 - c.c10);
  return lo + s.fa * (hi - lo);
}

// Derivatives of the bilinear sample with respect to the point (y0, y1).
__device__ __forceinline__ void lerp2_grad(const Corners& c, const Sample& s, float& d0, float& d1) {
  d0 = (1.0f - s.fb) * (c.c10 - c.c00) + s.fb * (c.c11 - c.c01);
  d1 = (1.0f - s.fa) * (c.c01 - c.c00) + s.fa * (c.c11 - c.c10);
}

// Adds g times the four bilinear weights of the sample into f (atomics).
__device__ __forceinline__ void scatter2(float* f, const Sample& s, int n, float g) {
  if (g == 0.0f) return;
  const float ga = g * s.fa, gna = g - ga;
  float* r0 = f + size_t(s.a0) * n;
  float* r1 = f + size_t(s.a1) * n;
  unsafeAtomicAdd(r0 + s.b0, gna - gna * s.fb);
  unsafeAtomicAdd(r0 + s.b1, gna * s.fb);
  unsafeAtomicAdd(r1 + s.b0, ga - ga * s.fb);
  unsafeAtomicAdd(r1 + s.b1, ga * s.fb);
}

// Region [k, P - k)^2 of a P x P extended tile, visited by all threads; fn(q)
// gets the linear LDS index q.
template <class Fn>
__device__ __forceinline__ void for_region(int P, int k, int threads, Fn&& fn) {
  const int e = P - 2 * k;
  if (e <= 0) return;
  const float rcp = (1.0f / float(e)) * (1.0f + 0x1p-20f);
  for (int r = threadIdx.x; r < e * e; r += threads) {
    const int ri = int(float(r) * rcp);  // r < 2^16, e <= 2^10: exact quotient
    const int rj = r - ri * e;
    fn((k + ri) * P + (k + rj));
  }
}

// Halo of a tile for K sweeps: the self-advected velocity is needed K + 1
// cells around the tile (K = 0: no projection, no halo).
__host__ __device__ __forceinline__ int halo(int iters) { return iters > 0 ? iters + 1 : 0; }

// LDS floats of either kernel: five P x P arrays.
__host__ __device__ __forceinline__ int lds_floats(int ts, int iters) {
  const int P = ts + 2 * halo(iters);
  return 5 * P * P;
}

// Forward step: state `in` (planes u0, u1, s of n x n floats) -> state `out`.
template <int TS>
__global__ void __launch_bounds__(TS * TS) k_smoke_fwd(const float* __restrict__ in, float* __restrict__ out, int n,
                                                      int iters, unsigned* __restrict__ err_word) {
  extern __shared__ float lds[];
  constexpr int kThreads = TS * TS;
  const int H = halo(iters);
  const int P = TS + 2 * H;
  const int PP = P * P;
  float* w0 = lds;           // self-advected velocity, extended tile
  float* w1 = lds + PP;
  float* dv = lds + 2 * PP;  // divergence, [1, P - 1)
  float* pa = lds + 3 * PP;  // Jacobi iterates (ping-pong)
  float* pb = lds + 4 * PP;
  const size_t nn = size_t(n) * n;
  const float* __restrict__ u0 = in;
  const float* __restrict__ u1 = in + nn;
  const float* __restrict__ sm = in + 2 * nn;
  const int ti0 = int(blockIdx.x) * TS, tj0 = int(blockIdx.y) * TS;
  unsigned err = 0;

  // u* = advect(u, u) on the extended tile.
  for (int q = threadIdx.x; q < PP; q += kThreads) {
    const int qi = q / P, qj = q - (q / P) * P;
    const int i = wrap(ti0 - H + qi, n), j = wrap(tj0 - H + qj, n);
    const size_t c = size_t(i) * n + j;
    const Sample s = back_trace(i, j, u0[c], u1[c], n, err);
    w0[q] = lerp2(corners(u0, s, n), s);
    w1[q] = lerp2(corners(u1, s, n), s);
  }
  const float* p = nullptr;
  if (iters > 0) {
    __syncthreads();
    // Divergence and the first sweep from p^0 = 0, on [1, P - 1).
    for_region(P, 1, kThreads, [&](int q) {
      const float d = 0.5f * ((w0[q + P] - w0[q - P]) + (w1[q + 1] - w1[q - 1]));
      dv[q] = d;
      pa[q] = -0.25f * d;
    });
    float* src = pa;
    float* dst = pb;
    for (int k = 2; k <= iters; ++k) {
      __syncthreads();
      for_region(P, k, kThreads, [&](int q) {
        dst[q] = 0.25f * ((src[q + P] + src[q - P]) + (src[q + 1] + src[q - 1]) - dv[q]);
      });
      float* t = src;
      src = dst;
      dst = t;
    }
    __syncthreads();
    p = src;  // p^K on [K, P - K): the tile plus one
  }
  // Projected velocity and the advected smoke on the tile.
  const int ti = int(threadIdx.x) / TS, tj = int(threadIdx.x) % TS;
  const int i = ti0 + ti, j = tj0 + tj;
  if (i < n && j < n) {
    const int q = (ti + H) * P + (tj + H);
    float v0 = w0[q], v1 = w1[q];
    if (p) {
      v0 -= 0.5f * (p[q + P] - p[q - P]);
      v1 -= 0.5f * (p[q + 1] - p[q - 1]);
    }
    const size_t c = size_t(i) * n + j;
    out[c] = v0;
    out[nn + c] = v1;
    const Sample s = back_trace(i, j, v0, v1, n, err);
    out[2 * nn + c] = lerp2(corners(sm, s, n), s);
  }
  if (err) atomicOr(err_word, err);
}

// Reverse step s: given state s (`st`), state s+1 (`nx`, whose velocity is
// step s's projected velocity) and the adjoint of state s+1 (`gnext`), ADDS
// the adjoint of state s into `gout` (atomics) and zeroes `gclear` (the
// buffer the next launch accumulates into; may be null). All are three
// n x n planes (u0, u1, s).
template <int TS>
__global__ void __launch_bounds__(TS * TS) k_smoke_bwd(const float* __restrict__ st, const float* __restrict__ nx,
                                                      const float* __restrict__ gnext, float* __restrict__ gout,
                                                      float* __restrict__ gclear, int n, int iters,
                                                      unsigned* __restrict__ err_word) {
  extern __shared__ float lds[];
  constexpr int kThreads = TS * TS;
  const int H = halo(iters);
  const int P = TS + 2 * H;
  const int PP = P * P;
  float* gv0 = lds;           // adjoint of the projected velocity, extended tile
  float* gv1 = lds + PP;
  float* db = lds + 2 * PP;   // adjoint of the divergence
  float* qa = lds + 3 * PP;   // adjoint sweeps (ping-pong)
  float* qb = lds + 4 * PP;
  const size_t nn = size_t(n) * n;
  const int ti0 = int(blockIdx.x) * TS, tj0 = int(blockIdx.y) * TS;
  const int ti = int(threadIdx.x) / TS, tj = int(threadIdx.x) % TS;
  const int oi = ti0 + ti, oj = tj0 + tj;
  const bool own = oi < n && oj < n;
  unsigned err = 0;

  // Smoke advection s' = advect(s, v): the position term gives
  // v* = v*_next - s*_next grad(sample) at every cell of the extended tile;
  // the field term scatters s*_next into the smoke adjoint of state s from
  // the tile's own cells.
  for (int q = threadIdx.x; q < PP; q += kThreads) {
    const int qi = q / P, qj = q - (q / P) * P;
    const int i = wrap(ti0 - H + qi, n), j = wrap(tj0 - H + qj, n);
    const size_t c = size_t(i) * n + j;
    const Sample s = back_trace(i, j, nx[c], nx[nn + c], n, err);
    const float gs = gnext[2 * nn + c];
    float d0, d1;
    lerp2_grad(corners(st + 2 * nn, s, n), s, d0, d1);
    gv0[q] = gnext[c] - gs * d0;
    gv1[q] = gnext[nn + c] - gs * d1;
  }
  if (own) {
    const size_t c = size_t(oi) * n + oj;
    const Sample s = back_trace(oi, oj, nx[c], nx[nn + c], n, err);
    scatter2(gout + 2 * nn, s, n, gnext[2 * nn + c]);
  }
  __syncthreads();
  // Projection v = w - grad(p^K), p^K linear in div(w): p*^K = div(v*)
  // (the central-difference gradient is minus the divergence's transpose),
  // then K adjoint sweeps q <- S q / 4, each adding -q / 4 to div*.
  if (iters > 0) {
    for_region(P, 1, kThreads, [&](int q) {
      const float g = 0.5f * ((gv0[q + P] - gv0[q - P]) + (gv1[q + 1] - gv1[q - 1]));
      qa[q] = g;
      db[q] = -0.25f * g;
    });
    float* src = qa;
    float* dst = qb;
    for (int m = 1; m < iters; ++m) {
      __syncthreads();
      for_region(P, 1 + m, kThreads, [&](int q) {
        const float g = 0.25f * ((src[q + P] + src[q - P]) + (src[q + 1] + src[q - 1]));
        dst[q] = g;
        db[q] -= 0.25f * g;
      });
      float* t = src;
      src = dst;
      dst = t;
    }
    __syncthreads();
  }
  if (own) {
    const int q = (ti + H) * P + (tj + H);
    // w* = v* + div^T(div*) on the tile.
    float g0 = gv0[q], g1 = gv1[q];
    if (iters > 0) {
      g0 += 0.5f * (db[q - P] - db[q + P]);
      g1 += 0.5f * (db[q - 1] - db[q + 1]);
    }
    // w_a = advect(u_a, u): field terms scatter, position terms are local.
    const size_t c = size_t(oi) * n + oj;
    const float* u0 = st;
    const float* u1 = st + nn;
    const Sample s = back_trace(oi, oj, u0[c], u1[c], n, err);
    const Corners k0 = corners(u0, s, n), k1 = corners(u1, s, n);
    float a00, a01, a10, a11;  // d(sample of u_a)/dy_b
    lerp2_grad(k0, s, a00, a01);
    lerp2_grad(k1, s, a10, a11);
    scatter2(gout, s, n, g0);
    scatter2(gout + nn, s, n, g1);
    const float l0 = -(g0 * a00 + g1 * a10);
    const float l1 = -(g0 * a01 + g1 * a11);
    if (l0 != 0.0f) unsafeAtomicAdd(gout + c, l0);
    if (l1 != 0.0f) unsafeAtomicAdd(gout + nn + c, l1);
    if (gclear) {
      gclear[c] = 0.0f;
      gclear[nn + c] = 0.0f;
      gclear[2 * nn + c] = 0.0f;
    }
  }
  if (err) atomicOr(err_word, err);
}

// L = sum (s - target)^2 over the smoke plane of `fin`, accumulated in FP64
// into *acc; seed (if non-null) = dL/d(state): zero velocity planes,
// 2 (s - target) on the smoke plane.
__global__ void k_smoke_loss(const float* __restrict__ fin, const float* __restrict__ target, int n,
                             double* __restrict__ acc, float* __restrict__ seed) {
  __shared__ double part[16];
  const size_t nn = size_t(n) * n;
  double sum = 0.0;
  for (size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x; c < nn; c += size_t(gridDim.x) * blockDim.x) {
    const float d = fin[2 * nn + c] - target[c];
    sum += double(d) * double(d);
    if (seed) {
      seed[c] = 0.0f;
      seed[nn + c] = 0.0f;
      seed[2 * nn + c] = 2.0f * d;
    }
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x + 63) / 64; ++w) t += part[w];
    unsafeAtomicAdd(acc, t);
  }
}

__global__ void k_smoke_loss_out(const double* __restrict__ acc, float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *loss = float(*acc);
}

__global__ void k_smoke_fill(float* __restrict__ p, size_t n, float v) {
  for (size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += size_t(gridDim.x) * blockDim.x) p[c] = v;
}

__global__ void k_smoke_zero_acc(double* __restrict__ acc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *acc = 0.0;
}

}  // namespace smoke

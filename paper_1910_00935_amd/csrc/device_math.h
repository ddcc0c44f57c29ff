// Device-side math of one MLS-MPM step and its adjoint, FP32, for gfx950.
//
// Method (DiffTaichi, Section 4.1: moving-least-squares MPM after ChainQueen;
// stage order of Appendix D.1): quadratic B-spline weights on the 3^d nodes
// base .. base+2 with base = floor(x/dx - 1/2); APIC/MLS affine momentum
// transfer with kappa = 4/dx^2; compressible neo-Hookean Kirchhoff stress
// tau = mu (F F^T - I) + lambda ln(J) I evaluated with the initial volume;
// grid update v = P/m + dt g e_1 on interior nodes with mass (sticky band of
// `bound` nodes, zero elsewhere); grid-to-particle gather of v and
// C = kappa sum w v delta^T, x' = x + dt v', F' = (I + dt C') F.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

constexpr unsigned kErrDomain = 1u;
constexpr unsigned kErrInverted = 2u;
constexpr unsigned kErrNonfinite = 4u;
constexpr int kMaxAct = 16;

// Component-major SoA view: component c of particle i at p[c * stride + i].
struct StateRef {
  float* x;
  float* v;
  float* C;
  float* F;
  int stride;
};

template <int D>
struct PState {
  float x[D], v[D], C[D][D], F[D][D];
};

template <int D>
__device__ __forceinline__ void load_xF(const StateRef& s, int i, PState<D>& p) {
#pragma unroll
  for (int a = 0; a < D; ++a) p.x[a] = s.x[a * s.stride + i];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) p.F[a][b] = s.F[(a * D + b) * s.stride + i];
}

template <int D>
__device__ __forceinline__ void load_state(const StateRef& s, int i, PState<D>& p) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    p.x[a] = s.x[a * s.stride + i];
    p.v[a] = s.v[a * s.stride + i];
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      p.C[a][b] = s.C[(a * D + b) * s.stride + i];
      p.F[a][b] = s.F[(a * D + b) * s.stride + i];
    }
}

template <int D>
__device__ __forceinline__ void store_state(const StateRef& s, int i, const PState<D>& p) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    s.x[a * s.stride + i] = p.x[a];
    s.v[a * s.stride + i] = p.v[a];
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      s.C[(a * D + b) * s.stride + i] = p.C[a][b];
      s.F[(a * D + b) * s.stride + i] = p.F[a][b];
    }
}

template <int D>
__device__ __forceinline__ bool state_finite(const PState<D>& p) {
  float acc = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) acc += p.x[a] * 0.0f + p.v[a] * 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) acc += p.C[a][b] * 0.0f + p.F[a][b] * 0.0f;
  return acc == 0.0f;  // NaN or +-inf anywhere makes acc NaN
}

// Per-particle stencil: base node, fractional offset f = x/dx - base in
// [0.5, 1.5), and, per axis, the three nodes base .. base+2 in the order this
// lane visits them: the B-spline piece N (N0 = 1/2 (3/2 - f)^2,
// N1 = 3/4 - (f - 1)^2, N2 = 1/2 (f - 1/2)^2), its derivative dN/df, the
// offset (o - f) dx of the node from the particle, and the node coordinate.
//
// Visiting order: lanes of a wave that add to the same LDS or HBM node in the
// same instruction serialise. A lane with colour (s_0, s_1, s_2) visits, at
// step t_a of axis a, the node whose coordinate is congruent to t_a + s_a
// (mod 3); lanes of different colours therefore never touch the same node in
// the same instruction. Colour -1 keeps the natural order base, base+1, base+2.
//
// Pair mode (two lanes per particle): the second lane of a pair visits every
// axis in the reverse order (step t_a -> node congruent to 2 - t_a + s_a), so
// the first H visits of lane 0 and the first H - 1 of lane 1 (H = 14 in 3D,
// 5 in 2D; the node with flat index H - 1 is lane 0's) split the stencil;
// skip_last marks lane 1.
template <int D>
struct Sten {
  int base[D] = {};
  float f[D];
  float N[D][3];
  float dN[D][3];
  float dl[D][3];
  int nc[D][3];
  bool skip_last = false;
};

// Returns false when the stencil would leave [0, n) on some axis (or x is not
// finite); base is then 0 so that no caller indexes out of bounds.
template <int D>
__device__ __forceinline__ bool make_sten(const float (&x)[D], float inv_dx, float dx, int n, int color,
                                          Sten<D>& st, bool mirror = false) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float xs = x[a] * inv_dx;
    const float g = xs - 0.5f;
    const bool in = (g >= 0.0f) && (g < float(n - 2));
    ok = ok && in;
    const int b = in ? int(floorf(g)) : 0;
    st.base[a] = b;
    const float f = xs - float(b);
    st.f[a] = f;
    const float w[3] = {0.5f * (1.5f - f) * (1.5f - f), 0.75f - (f - 1.0f) * (f - 1.0f), 0.5f * (f - 0.5f) * (f - 0.5f)};
    const float dw[3] = {f - 1.5f, -2.0f * (f - 1.0f), f - 0.5f};
    int k = 0;
    if (color >= 0) {
      const int digit = (D == 3) ? (a == 0 ? color / 9 : (a == 1 ? (color / 3) % 3 : color % 3))
                                 : (a == 0 ? color / 3 : color % 3);
      k = ((digit - b) % 3 + 3) % 3;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      int o = (mirror ? 2 - t : t) + k;
      o = (o >= 3) ? o - 3 : o;
      st.N[a][t] = (o == 0) ? w[0] : ((o == 1) ? w[1] : w[2]);
      st.dN[a][t] = (o == 0) ? dw[0] : ((o == 1) ? dw[1] : dw[2]);
      st.dl[a][t] = (float(o) - f) * dx;
      st.nc[a][t] = b + o;
    }
  }
  st.skip_last = mirror;
  return ok;
}

template <int D>
__device__ __forceinline__ float det(const float (&F)[D][D]) {
  if constexpr (D == 2) {
    return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else {
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  }
}

// cof(F) = det(F) F^{-T}.
template <int D>
__device__ __forceinline__ void cofactor(const float (&F)[D][D], float (&K)[D][D]) {
  if constexpr (D == 2) {
    K[0][0] = F[1][1];
    K[0][1] = -F[1][0];
    K[1][0] = -F[0][1];
    K[1][1] = F[0][0];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        K[a][b] = F[a1][b1] * F[a2][b2] - F[a1][b2] * F[a2][b1];
      }
  }
}

struct SceneParams {
  float mass, vol, mu, lam, dmu_dE, dlam_dE;
};

__device__ __forceinline__ SceneParams scene_params(const float* E, const float* nu, const float* vol,
                                                    const float* rho, int sc) {
  SceneParams p;
  const float e = E[sc], n = nu[sc];
  p.vol = vol[sc];
  p.mass = rho[sc] * p.vol;
  p.dmu_dE = 1.0f / (2.0f * (1.0f + n));
  p.dlam_dE = n / ((1.0f + n) * (1.0f - 2.0f * n));
  p.mu = e * p.dmu_dE;
  p.lam = e * p.dlam_dE;
  return p;
}

// Kirchhoff stress and the affine matrix A = m C - dt V kappa tau.
// Also returns F F^T - I and ln J for the adjoint.
template <int D>
__device__ __forceinline__ void affine(const PState<D>& p, const SceneParams& sp, float act_tau, float dt,
                                       float kappa, float (&A)[D][D], float (&FFtI)[D][D], float& lnJ,
                                       float& J, unsigned& err) {
  J = det<D>(p.F);
  if (J > 0.0f) {
    lnJ = logf(J);
  } else {
    lnJ = 0.0f;
    err |= kErrInverted;
  }
  const float k = dt * sp.vol * kappa;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) s += p.F[a][c] * p.F[b][c];
      FFtI[a][b] = s - (a == b ? 1.0f : 0.0f);
      float tau = sp.mu * FFtI[a][b] + (a == b ? sp.lam * lnJ : 0.0f);
      if (a == 1 && b == 1) tau += act_tau;
      A[a][b] = sp.mass * p.C[a][b] - k * tau;
    }
}


__device__ __forceinline__ bool interior1(int i, int n, int bound) { return i >= bound && i < n - bound; }

// Warp (wave64) sum.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mpm

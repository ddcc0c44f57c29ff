// Device-side math of one MLS-MPM step and its adjoint, FP32, for gfx950.
//
// Method (DiffTaichi, Section 4.1: moving-least-squares MPM after ChainQueen;
// stage order of Appendix D.1): quadratic B-spline weights on the 3^d nodes
// base .. base+2 with base = floor(x/dx - 1/2); APIC/MLS affine momentum
// transfer with kappa = 4/dx^2; compressible neo-Hookean Kirchhoff stress
// tau = mu (F F^T - I) + lambda ln(J) I evaluated with the initial volume, or
// the fixed-corotated tau = 2 mu (F - R) F^T + lambda (J - 1) J I with R the
// polar rotation of F and a hand-written gradient of the decomposition (the
// custom gradients of Section 3 and Appendix C);
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

// Rotation R of the polar decomposition F = R S (S symmetric positive
// definite), for det F > 0. 2D: the rotation angle maximises tr(R^T F), so
// (cos, sin) is the normalised (F00 + F11, F10 - F01). 3D: kPolarIters steps
// of Newton's iteration X <- (g X + X^{-T} / g) / 2 from X = F, with the
// determinant scaling g = det(X)^(-1/3) (Higham, 1986); each step roughly
// squares the distance to R, so strains of tens of percent reach FP32
// precision well within the fixed count.
constexpr int kPolarIters = 6;

template <int D>
__device__ __forceinline__ void polar_rotation(const float (&F)[D][D], float (&R)[D][D]) {
  if constexpr (D == 2) {
    const float a = F[0][0] + F[1][1], b = F[1][0] - F[0][1];
    const float inv = 1.0f / sqrtf(a * a + b * b);
    R[0][0] = a * inv;
    R[0][1] = -b * inv;
    R[1][0] = b * inv;
    R[1][1] = a * inv;
  } else {
    float X[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) X[a][b] = F[a][b];
    for (int it = 0; it < kPolarIters; ++it) {
      float K[3][3];
      cofactor<3>(X, K);
      const float J = X[0][0] * K[0][0] + X[0][1] * K[0][1] + X[0][2] * K[0][2];
      const float g = 1.0f / cbrtf(J);
      const float h = 1.0f / (g * J);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) X[a][b] = 0.5f * (g * X[a][b] + h * K[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) R[a][b] = X[a][b];
  }
}

struct SceneParams {
  float mass, vol, E, mu, lam, dmu_dE, dlam_dE;
};

__device__ __forceinline__ SceneParams scene_params(const float* E, const float* nu, const float* vol,
                                                    const float* rho, int sc) {
  SceneParams p;
  const float e = E[sc], n = nu[sc];
  p.vol = vol[sc];
  p.mass = rho[sc] * p.vol;
  p.dmu_dE = 1.0f / (2.0f * (1.0f + n));
  p.dlam_dE = n / ((1.0f + n) * (1.0f - 2.0f * n));
  p.E = e;
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


// Fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + lambda (J - 1) J I
// (R the polar rotation of F) and the affine matrix A = m C - dt V kappa tau.
// An inverted F (J <= 0) raises the error bit and carries no stress. Also
// returns R for the adjoint.
template <int D>
__device__ __forceinline__ void affine_corotated(const PState<D>& p, const SceneParams& sp, float act_tau, float dt,
                                                 float kappa, float (&A)[D][D], float (&R)[D][D], float& J,
                                                 unsigned& err) {
  J = det<D>(p.F);
  const bool ok = J > 0.0f;
  if (!ok) err |= kErrInverted;
  polar_rotation<D>(p.F, R);
  const float k = dt * sp.vol * kappa;
  const float vol_term = ok ? sp.lam * (J - 1.0f) * J : 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) s += (p.F[a][c] - R[a][c]) * p.F[b][c];
      float tau = ok ? 2.0f * sp.mu * s + (a == b ? vol_term : 0.0f) : 0.0f;
      if (a == 1 && b == 1) tau += act_tau;
      A[a][b] = sp.mass * p.C[a][b] - k * tau;
    }
}

// Adjoint of the fixed-corotated stress: given tb = dL/dtau, ADDS dL/dF into
// gF and returns dL/dE through tau. Term by term,
//   F* = 2 mu [(tb + tb^T) F - tb^T R] + lambda (2J - 1) tr(tb) cof(F) + (rotation share),
// and the rotation's share for R* = -2 mu tb F follows from F = R S: dR = R W
// with W skew and R^T dF - dF^T R = W S + S W. In 3D, W = [w]_x and W S + S W
// = [(tr(S) I - S) w]_x, which gives the share R [c]_x with c = (tr(S) I -
// S)^{-1} a, a the axial vector of X - X^T, X = R^T R*. In 2D the share is
// R [[0, -c], [c, 0]] with c = (X10 - X01) / tr(S).
template <int D>
__device__ __forceinline__ float corotated_adjoint(const PState<D>& p, const SceneParams& sp, const float (&R)[D][D],
                                                   float J, const float (&tb)[D][D], float (&gF)[D][D]) {
  if (!(J > 0.0f)) return 0.0f;
  float K[D][D];
  cofactor<D>(p.F, K);
  float tr = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) tr += tb[a][a];
  const float vol_c = sp.lam * (2.0f * J - 1.0f) * tr;
  float X[D][D], S[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float v = 0.0f, rb = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        v += (tb[a][c] + tb[c][a]) * p.F[c][b] - tb[c][a] * R[c][b];
        rb += tb[a][c] * p.F[c][b];
      }
      gF[a][b] += 2.0f * sp.mu * v + vol_c * K[a][b];
      X[a][b] = -2.0f * sp.mu * rb;  // R* for now; turned into R^T R* below
    }
  float Xt[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float x = 0.0f, sv = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        x += R[c][a] * X[c][b];
        sv += R[c][a] * p.F[c][b];
      }
      Xt[a][b] = x;
      S[a][b] = sv;
    }
  float trS = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) trS += S[a][a];
  float W[D][D] = {};
  if constexpr (D == 2) {
    const float c = (Xt[1][0] - Xt[0][1]) / trS;
    W[0][1] = -c;
    W[1][0] = c;
  } else {
    const float av[3] = {Xt[2][1] - Xt[1][2], Xt[0][2] - Xt[2][0], Xt[1][0] - Xt[0][1]};
    float G[3][3], Gc[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[a][b] = (a == b ? trS : 0.0f) - 0.5f * (S[a][b] + S[b][a]);
    cofactor<3>(G, Gc);
    const float inv_det = 1.0f / (G[0][0] * Gc[0][0] + G[0][1] * Gc[0][1] + G[0][2] * Gc[0][2]);
    float c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = (Gc[a][0] * av[0] + Gc[a][1] * av[1] + Gc[a][2] * av[2]) * inv_det;
    W[0][1] = -c[2];
    W[0][2] = c[1];
    W[1][0] = c[2];
    W[1][2] = -c[0];
    W[2][0] = -c[1];
    W[2][1] = c[0];
  }
  float eb = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float v = 0.0f, frf = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        v += R[a][c] * W[c][b];
        frf += (p.F[a][c] - R[a][c]) * p.F[b][c];
      }
      gF[a][b] += v;
      eb += tb[a][b] * (2.0f * sp.dmu_dE * frf + (a == b ? sp.dlam_dE * (J - 1.0f) * J : 0.0f));
    }
  return eb;
}

// Weakly compressible liquid (material 1): Tait pressure p = E (J^-7 - 1) with
// the scene's E as bulk modulus, Kirchhoff stress tau = -p J I = E (J - J^-6) I;
// an inverted F raises the error bit and carries no stress.
template <int D>
__device__ __forceinline__ void affine_liquid(const PState<D>& p, const SceneParams& sp, float act_tau, float dt,
                                              float kappa, float (&A)[D][D], float& J, unsigned& err) {
  J = det<D>(p.F);
  const bool ok = J > 0.0f;
  if (!ok) err |= kErrInverted;
  const float ji = 1.0f / J, ji2 = ji * ji;
  const float val = ok ? sp.E * (J - ji2 * ji2 * ji2) : 0.0f;
  const float k = dt * sp.vol * kappa;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float tau = (a == b) ? val : 0.0f;
      if (a == 1 && b == 1) tau += act_tau;
      A[a][b] = sp.mass * p.C[a][b] - k * tau;
    }
}

// Adjoint of the liquid stress: d tau / dJ = E (1 + 6 J^-7) I and dJ =
// cof(F) : dF, so F* += E (1 + 6 J^-7) tr(tb) cof(F); returns dL/dE.
template <int D>
__device__ __forceinline__ float liquid_adjoint(const PState<D>& p, const SceneParams& sp, float J,
                                                const float (&tb)[D][D], float (&gF)[D][D]) {
  if (!(J > 0.0f)) return 0.0f;
  float K[D][D];
  cofactor<D>(p.F, K);
  float tr = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) tr += tb[a][a];
  const float ji = 1.0f / J, ji2 = ji * ji, ji6 = ji2 * ji2 * ji2;
  const float c = sp.E * (1.0f + 6.0f * ji6 * ji) * tr;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) gF[a][b] += c * K[a][b];
  return tr * (J - ji6);
}

__device__ __forceinline__ bool interior1(int i, int n, int bound) { return i >= bound && i < n - bound; }

// v of the DPP source lane (row shift or row broadcast `CTRL`, rows `ROWS`),
// 0 where the source lies outside the row or the row is not written.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Wavefront (64-lane) sum, the same value in every lane: DPP row shifts
// within rows of 16, then row broadcasts into lane 63, read back (one VALU
// move per half and step instead of a cross-lane LDS permute). All lanes
// must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

}  // namespace mpm

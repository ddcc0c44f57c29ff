// FP64 serial oracle for the differentiable elastic-object simulator of
// DiffTaichi (Hu et al., "DiffTaichi: Differentiable Programming for Physical
// Simulation", ICLR 2020), Section 4.1 ("diffmpm") and Appendix D.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library. The GPU path shares no code,
// header, table or helper with it.
//
// What it computes (the paper names the method and the stage order; the
// formulas are those of the published methods it cites):
//   * one moving-least-squares MPM step (Hu et al. 2018) with quadratic
//     B-spline weights and APIC affine transfer, stage order clear_grid ->
//     compute_actuation -> p2g -> grid_op -> g2p (Appendix D.1);
//   * compressible neo-Hookean Kirchhoff stress tau = mu (F F^T - I) + lambda
//     ln(J) I, using the initial particle volume; or (model 1) the
//     fixed-corotated stress tau = 2 mu (F - R) F^T + lambda (J - 1) J I with R
//     the rotation of the polar decomposition F = R S, whose derivative is the
//     kind of hand-engineered gradient Section 3 and Appendix C describe for
//     decompositions computed by iteration;
//   * a weakly compressible liquid for particles with material id 1 (Appendix
//     E.1 couples such a liquid with the elastic robot in the same grid): Tait
//     pressure p = E (J^-gamma - 1), gamma = 7, Kirchhoff stress tau = -p J I =
//     E (J - J^(1 - gamma)) I, the scene's E acting as the bulk modulus;
//   * the adjoint of each stage written by hand: for a primal f(X) = Y the
//     adjoint takes (X, Y*) and ACCUMULATES X* = dL/dX (Section 3 and
//     Appendix B); the grid is recomputed inside the adjoint step instead of
//     being stored (Appendix D.1); trajectories are differentiated with
//     segment checkpoints every K steps (Appendix D.2).
// The scalar type is a template parameter so that std::complex<double> gives
// complex-step tangents of the forward map (J v to machine precision), which
// is how the hand-written adjoint is pinned (dot-product test).
//
// Readings of points the paper leaves open (each one is listed in the design
// notes): nodes at i*dx, base = floor(x/dx - 1/2); kappa = 4/dx^2; gravity on
// axis 1 applied to nodes with mass; a node is "sticky" (velocity zero) when
// any index is < bound or >= n - bound; empty nodes (m == 0 exactly) get zero
// velocity; F is updated in the grid-to-particle stage, F' = (I + dt C') F;
// x' = x + dt v'; actuation adds sigma_a * a_k(s) e_y e_y^T to the Kirchhoff
// stress; a particle whose stencil leaves the grid, whose J <= 0, or whose
// state is not finite raises an error bit.
//
// Particle state layout (this file only): particle-major, each particle holds
// x[d], v[d], C[d][d], F[d][d] (row-major), S = 2d + 2d^2 doubles.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

using cd = std::complex<double>;

inline double re(double a) { return a; }
inline double re(const cd& a) { return a.real(); }
inline bool finite(double a) { return std::isfinite(a); }
inline bool finite(const cd& a) { return std::isfinite(a.real()) && std::isfinite(a.imag()); }

enum : int { ERR_DOMAIN = 1, ERR_INVERTED = 2, ERR_NONFINITE = 4 };

// Scene description as passed over the C ABI (plain doubles and ints).
struct Desc {
  int dim, n_grid, bound, n_scenes, n_act;
  double dx, dt, gravity, act_strength;
  const int* offsets;   // [n_scenes + 1] particle ranges per scene
  const double* E;      // [n_scenes] Young's modulus
  const double* nu;     // [n_scenes] Poisson ratio
  const double* vol;    // [n_scenes] initial particle volume
  const double* rho;    // [n_scenes] density (particle mass = rho * vol)
  const int* act_id;    // [N] actuator column per particle, -1 = none; may be null
  int model;            // 0: neo-Hookean, 1: fixed-corotated
  const int* mat_id;    // [N] material per particle (0 solid, 1 liquid); may be null (all solid)
};

constexpr double kTaitGamma = 7.0;

int pow3(int d) { return d == 2 ? 9 : 27; }
int state_size(int d) { return 2 * d + 2 * d * d; }
long nodes_per_scene(const Desc& s) {
  long n = 1;
  for (int a = 0; a < s.dim; ++a) n *= s.n_grid;
  return n;
}

// Views into one particle's packed state.
template <class T>
struct PView {
  T* p;
  int d;
  T& x(int a) const { return p[a]; }
  T& v(int a) const { return p[d + a]; }
  T& C(int a, int b) const { return p[2 * d + a * d + b]; }
  T& F(int a, int b) const { return p[2 * d + d * d + a * d + b]; }
};

// Quadratic B-spline N(t) on [0, 3) split into its three pieces, evaluated at
// the distance of the particle from the base node, f in [0.5, 1.5):
//   N0 = 1/2 (3/2 - f)^2,  N1 = 3/4 - (f - 1)^2,  N2 = 1/2 (f - 1/2)^2,
// and their derivatives with respect to f.
template <class T>
struct Stencil {
  int base[3];
  T f[3];
  T N[3][3];   // N[axis][o]
  T dN[3][3];  // dN/df [axis][o]
};

template <class T>
bool make_stencil(const Desc& s, const T* x, Stencil<T>& st) {
  for (int a = 0; a < s.dim; ++a) {
    T g = x[a] / s.dx - 0.5;
    double gr = re(g);
    if (!(gr >= 0.0 && gr < double(s.n_grid - 2))) return false;
    int b = int(std::floor(gr));
    st.base[a] = b;
    T f = x[a] / s.dx - double(b);
    st.f[a] = f;
    st.N[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
    st.N[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
    st.N[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
    st.dN[a][0] = f - 1.5;
    st.dN[a][1] = -2.0 * (f - 1.0);
    st.dN[a][2] = f - 0.5;
  }
  return true;
}

// Offset number k in [0, 3^d) -> o in {0,1,2}^d (axis 0 slowest).
void offset_of(int d, int k, int o[3]) {
  if (d == 2) {
    o[0] = k / 3; o[1] = k % 3; o[2] = 0;
  } else {
    o[0] = k / 9; o[1] = (k / 3) % 3; o[2] = k % 3;
  }
}

long node_index(const Desc& s, const int i[3]) {
  long idx = 0;
  for (int a = 0; a < s.dim; ++a) idx = idx * s.n_grid + i[a];
  return idx;
}

bool interior(const Desc& s, const int i[3]) {
  for (int a = 0; a < s.dim; ++a)
    if (i[a] < s.bound || i[a] >= s.n_grid - s.bound) return false;
  return true;
}

// Weight, gradient of the weight w.r.t. x_p, and delta = x_i - x_p of offset o.
template <class T>
void weight(const Desc& s, const Stencil<T>& st, const int o[3], T& w, T dw[3], T delta[3]) {
  w = 1.0;
  for (int a = 0; a < s.dim; ++a) w *= st.N[a][o[a]];
  for (int a = 0; a < s.dim; ++a) {
    T g = st.dN[a][o[a]] / s.dx;
    for (int c = 0; c < s.dim; ++c)
      if (c != a) g *= st.N[c][o[c]];
    dw[a] = g;
    delta[a] = (double(o[a]) - st.f[a]) * s.dx;
  }
}

template <class T>
T det(int d, const T F[3][3]) {
  if (d == 2) return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
         F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// Cofactor matrix: cof(F) = det(F) F^{-T}.
template <class T>
void cofactor(int d, const T F[3][3], T K[3][3]) {
  if (d == 2) {
    K[0][0] = F[1][1]; K[0][1] = -F[1][0];
    K[1][0] = -F[0][1]; K[1][1] = F[0][0];
    return;
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
      K[a][b] = F[a1][b1] * F[a2][b2] - F[a1][b2] * F[a2][b1];
    }
}

// Rotation R of the polar decomposition F = R S (S symmetric positive
// definite), for det F > 0. 2D: closed form; the rotation angle maximises
// tr(R^T F), so (cos, sin) is the normalised (F00 + F11, F10 - F01). 3D:
// Newton's iteration X <- (g X + (g X)^{-T}) / 2 from X = F, with the
// determinant scaling g = det(X)^(-1/3) (Higham, 1986), until the real parts
// stop changing. Only analytic operations touch the values, so complex-step
// tangents pass through it.
template <class T>
void polar_rotation(int d, const T F[3][3], T R[3][3]) {
  if (d == 2) {
    T a = F[0][0] + F[1][1], b = F[1][0] - F[0][1];
    T r = std::sqrt(a * a + b * b);
    R[0][0] = a / r;
    R[0][1] = -b / r;
    R[1][0] = b / r;
    R[1][1] = a / r;
    return;
  }
  T X[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X[a][b] = F[a][b];
  for (int it = 0; it < 100; ++it) {
    T K[3][3];
    cofactor(3, X, K);
    T J = det(3, X);
    T g = std::pow(J, -1.0 / 3.0);
    double change = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        T y = 0.5 * (g * X[a][b] + K[a][b] / (g * J));
        change = std::max(change, std::abs(re(y) - re(X[a][b])));
        X[a][b] = y;
      }
    if (change < 1e-15) break;
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R[a][b] = X[a][b];
}

template <class T>
struct Material {
  T mu, lam;
  double dmu_dE, dlam_dE;
};

template <class T>
Material<T> lame(const T& E, double nu) {
  Material<T> m;
  m.mu = E / (2.0 * (1.0 + nu));
  m.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  m.dmu_dE = 1.0 / (2.0 * (1.0 + nu));
  m.dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  return m;
}

int scene_of(const Desc& s, int p) {
  for (int k = 0; k < s.n_scenes; ++k)
    if (p >= s.offsets[k] && p < s.offsets[k + 1]) return k;
  return -1;
}

template <class T>
bool state_finite(const T* p, int S) {
  for (int q = 0; q < S; ++q)
    if (!finite(p[q])) return false;
  return true;
}

// Per-particle quantities the particle-to-grid stage needs: the affine matrix
// A_p = m_p C_p - dt V_p kappa tau_p (momentum-exchange form of MLS-MPM).
template <class T>
struct P2GTerms {
  T F[3][3], R[3][3], tau[3][3], A[3][3], J, lnJ, mass;
  bool ok;
};

template <class T>
int p2g_terms(const Desc& s, int sc, const T* Es, const T* act_s, int p, const PView<const T>& P,
              P2GTerms<T>& t) {
  int d = s.dim, err = 0;
  double kappa = 4.0 / (s.dx * s.dx);
  double vol = s.vol[sc];
  t.mass = s.rho[sc] * vol;
  Material<T> mat = lame(Es[sc], s.nu[sc]);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) t.F[a][b] = P.F(a, b);
  t.J = det(d, t.F);
  t.ok = true;
  if (!(re(t.J) > 0.0)) {
    err |= ERR_INVERTED;
    t.lnJ = 0.0;
  } else {
    t.lnJ = std::log(t.J);
  }
  if (s.mat_id && s.mat_id[p] == 1) {
    // liquid: tau = E (J - J^(1 - gamma)) I (no stress when inverted, flagged above)
    T val = (re(t.J) > 0.0) ? Es[sc] * (t.J - std::pow(t.J, 1.0 - kTaitGamma)) : T(0.0);
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) t.tau[a][b] = (a == b) ? val : T(0.0);
  } else if (s.model == 1 && re(t.J) > 0.0) {
    // tau = 2 mu (F - R) F^T + lambda (J - 1) J I
    polar_rotation(d, t.F, t.R);
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        T FRF = 0.0;
        for (int c = 0; c < d; ++c) FRF += (t.F[a][c] - t.R[a][c]) * t.F[b][c];
        t.tau[a][b] = 2.0 * mat.mu * FRF + (a == b ? mat.lam * (t.J - 1.0) * t.J : T(0.0));
      }
  } else if (s.model == 1) {
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) t.tau[a][b] = 0.0;  // inverted: flagged above, no stress
  } else {
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        T FFt = 0.0;
        for (int c = 0; c < d; ++c) FFt += t.F[a][c] * t.F[b][c];
        t.tau[a][b] = mat.mu * (FFt - (a == b ? 1.0 : 0.0)) + (a == b ? mat.lam * t.lnJ : T(0.0));
      }
  }
  if (act_s && s.act_id && s.act_id[p] >= 0) t.tau[1][1] += s.act_strength * act_s[s.act_id[p]];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) t.A[a][b] = t.mass * P.C(a, b) - s.dt * vol * kappa * t.tau[a][b];
  return err;
}

// ---------------------------------------------------------------------------
// Forward step. grid: [n_scenes][nodes][d+1] holding (m, P) after the
// particle-to-grid stage and (m, v) after the grid update.
// ---------------------------------------------------------------------------
template <class T>
int p2g(const Desc& s, const T* Es, const T* act_s, const T* in, std::vector<T>& grid) {
  int d = s.dim, S = state_size(d), K = pow3(d), err = 0;
  long nn = nodes_per_scene(s);
  grid.assign(size_t(s.n_scenes) * nn * (d + 1), T(0.0));
  int N = s.offsets[s.n_scenes];
  for (int p = 0; p < N; ++p) {
    int sc = scene_of(s, p);
    PView<const T> P{in + size_t(p) * S, d};
    if (!state_finite(P.p, S)) { err |= ERR_NONFINITE; continue; }
    Stencil<T> st;
    if (!make_stencil(s, P.p, st)) { err |= ERR_DOMAIN; continue; }
    P2GTerms<T> t;
    err |= p2g_terms(s, sc, Es, act_s, p, P, t);
    for (int k = 0; k < K; ++k) {
      int o[3], i[3];
      offset_of(d, k, o);
      for (int a = 0; a < 3; ++a) i[a] = st.base[a] + o[a];
      T w, dw[3], dl[3];
      weight(s, st, o, w, dw, dl);
      T* g = &grid[(size_t(sc) * nn + node_index(s, i)) * (d + 1)];
      g[0] += w * t.mass;
      for (int a = 0; a < d; ++a) {
        T Ad = 0.0;
        for (int b = 0; b < d; ++b) Ad += t.A[a][b] * dl[b];
        g[1 + a] += w * (t.mass * P.v(a) + Ad);
      }
    }
  }
  return err;
}

// Grid update: v_i = P_i / m_i + dt g e_1 on interior nodes with mass; else 0.
template <class T>
void grid_update(const Desc& s, std::vector<T>& grid) {
  int d = s.dim;
  long nn = nodes_per_scene(s);
  for (int sc = 0; sc < s.n_scenes; ++sc)
    for (long q = 0; q < nn; ++q) {
      int i[3] = {0, 0, 0};
      long r = q;
      for (int a = d - 1; a >= 0; --a) { i[a] = int(r % s.n_grid); r /= s.n_grid; }
      T* g = &grid[(size_t(sc) * nn + q) * (d + 1)];
      bool active = re(g[0]) > 0.0 && interior(s, i);
      for (int a = 0; a < d; ++a) {
        if (active) {
          g[1 + a] = g[1 + a] / g[0];
          if (a == 1) g[1 + a] += s.dt * s.gravity;
        } else {
          g[1 + a] = 0.0;
        }
      }
    }
}

template <class T>
int g2p(const Desc& s, const T* in, const std::vector<T>& grid, T* out) {
  int d = s.dim, S = state_size(d), K = pow3(d), err = 0;
  long nn = nodes_per_scene(s);
  double kappa = 4.0 / (s.dx * s.dx);
  int N = s.offsets[s.n_scenes];
  for (int p = 0; p < N; ++p) {
    int sc = scene_of(s, p);
    PView<const T> P{in + size_t(p) * S, d};
    PView<T> Q{out + size_t(p) * S, d};
    Stencil<T> st;
    if (!state_finite(P.p, S) || !make_stencil(s, P.p, st)) {
      for (int q = 0; q < S; ++q) Q.p[q] = P.p[q];
      err |= state_finite(P.p, S) ? ERR_DOMAIN : ERR_NONFINITE;
      continue;
    }
    T vn[3] = {0.0, 0.0, 0.0}, Cn[3][3] = {};
    for (int k = 0; k < K; ++k) {
      int o[3], i[3];
      offset_of(d, k, o);
      for (int a = 0; a < 3; ++a) i[a] = st.base[a] + o[a];
      T w, dw[3], dl[3];
      weight(s, st, o, w, dw, dl);
      const T* g = &grid[(size_t(sc) * nn + node_index(s, i)) * (d + 1)];
      for (int a = 0; a < d; ++a) {
        vn[a] += w * g[1 + a];
        for (int b = 0; b < d; ++b) Cn[a][b] += kappa * w * g[1 + a] * dl[b];
      }
    }
    for (int a = 0; a < d; ++a) {
      Q.v(a) = vn[a];
      Q.x(a) = P.x(a) + s.dt * vn[a];
      for (int b = 0; b < d; ++b) {
        Q.C(a, b) = Cn[a][b];
        T Fn = 0.0;
        for (int c = 0; c < d; ++c) Fn += ((a == c ? 1.0 : 0.0) + s.dt * Cn[a][c]) * P.F(c, b);
        Q.F(a, b) = Fn;
      }
    }
  }
  return err;
}

template <class T>
int step_fwd(const Desc& s, const T* Es, const T* act_s, const T* in, T* out) {
  std::vector<T> grid;
  int err = p2g(s, Es, act_s, in, grid);
  grid_update(s, grid);
  err |= g2p(s, in, grid, out);
  return err;
}

// Adjoint of the fixed-corotated stress tau = 2 mu (F F^T - R F^T) + lambda
// (J^2 - J) I for a given tau* (accumulated into H.F) and its E-derivative
// (into eb). Differentiating term by term:
//   F* += 2 mu (tau* + tau*^T) F - 2 mu tau*^T R + lambda (2J - 1) tr(tau*) cof(F)
// plus the rotation's share for R* = -2 mu tau* F. With F = R S, dR = R W,
// W skew, and R^T dF - dF^T R = W S + S W. In 3D, W = [w]_x and
// W S + S W = [G w]_x with G = tr(S) I - S, so <R*, dR> = a . w with a the
// axial vector of X - X^T, X = R^T R*, and w = G^{-1} axial(R^T dF - dF^T R):
// the share is F* += R [G^{-1} a]_x. In 2D, W = w [[0, -1], [1, 0]], w =
// (Y10 - Y01) / tr(S) with Y = R^T dF, and the share is R [[0, -c], [c, 0]]
// with c = (X10 - X01) / tr(S).
void corotated_adjoint(int d, const P2GTerms<double>& t, const Material<double>& mat, const double tb[3][3],
                       PView<double>& H, double& eb) {
  const double J = t.J;
  double cof[3][3];
  cofactor(d, t.F, cof);
  double tr = 0.0;
  for (int a = 0; a < d; ++a) tr += tb[a][a];
  double Fbar[3][3] = {};
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double v = 0.0;
      for (int c = 0; c < d; ++c) v += (tb[a][c] + tb[c][a]) * t.F[c][b] - tb[c][a] * t.R[c][b];
      Fbar[a][b] = 2.0 * mat.mu * v + mat.lam * (2.0 * J - 1.0) * tr * cof[a][b];
    }
  // R* = -2 mu tau* F, X = R^T R*, S = R^T F.
  double Rbar[3][3] = {}, X[3][3] = {}, S[3][3] = {};
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      for (int c = 0; c < d; ++c) Rbar[a][b] += -2.0 * mat.mu * tb[a][c] * t.F[c][b];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      for (int c = 0; c < d; ++c) {
        X[a][b] += t.R[c][a] * Rbar[c][b];
        S[a][b] += t.R[c][a] * t.F[c][b];
      }
  double trS = 0.0;
  for (int a = 0; a < d; ++a) trS += S[a][a];
  double Wc[3][3] = {};
  if (d == 2) {
    double c = (X[1][0] - X[0][1]) / trS;
    Wc[0][1] = -c;
    Wc[1][0] = c;
  } else {
    double av[3] = {X[2][1] - X[1][2], X[0][2] - X[2][0], X[1][0] - X[0][1]};
    double G[3][3], Gc[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) G[a][b] = (a == b ? trS : 0.0) - S[a][b];
    cofactor(3, G, Gc);  // G^{-1} = cof(G)^T / det G; G is symmetric
    double dG = det(3, G);
    double c[3];
    for (int a = 0; a < 3; ++a) {
      c[a] = 0.0;
      for (int b = 0; b < 3; ++b) c[a] += Gc[b][a] * av[b];
      c[a] /= dG;
    }
    Wc[0][1] = -c[2]; Wc[0][2] = c[1];
    Wc[1][0] = c[2];  Wc[1][2] = -c[0];
    Wc[2][0] = -c[1]; Wc[2][1] = c[0];
  }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double v = 0.0;
      for (int c = 0; c < d; ++c) v += t.R[a][c] * Wc[c][b];
      H.F(a, b) += Fbar[a][b] + v;
    }
  // dtau/dE = 2 (F - R) F^T dmu/dE + (J - 1) J I dlambda/dE.
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double FRF = 0.0;
      for (int c = 0; c < d; ++c) FRF += (t.F[a][c] - t.R[a][c]) * t.F[b][c];
      double dtau = 2.0 * mat.dmu_dE * FRF + (a == b ? mat.dlam_dE * (J - 1.0) * J : 0.0);
      eb += tb[a][b] * dtau;
    }
}

// ---------------------------------------------------------------------------
// Adjoint of one step. gout = (x', v', C', F')* of state s+1; accumulates
// (x, v, C, F)* of state s into gin, dL/dE per scene into gE and dL/da_k(s)
// into gact. The grid is recomputed from state s (Appendix D.1).
// ---------------------------------------------------------------------------
int step_bwd(const Desc& s, const double* act_s, const double* in, const double* gout, double* gin,
             double* gE, double* gact) {
  int d = s.dim, S = state_size(d), K = pow3(d);
  long nn = nodes_per_scene(s);
  double kappa = 4.0 / (s.dx * s.dx);
  int N = s.offsets[s.n_scenes];

  // Recompute: clear_grid, p2g, grid_op.
  std::vector<double> grid;
  int err = p2g(s, s.E, act_s, in, grid);
  std::vector<double> grid_mP = grid;  // (m, P) before the update
  grid_update(s, grid);                // (m, v)

  // Adjoint of g2p: scatter v* into the grid, accumulate x* and F*.
  std::vector<double> vbar(size_t(s.n_scenes) * nn * d, 0.0);
  for (int p = 0; p < N; ++p) {
    int sc = scene_of(s, p);
    PView<const double> P{in + size_t(p) * S, d};
    PView<const double> G{gout + size_t(p) * S, d};
    PView<double> H{gin + size_t(p) * S, d};
    Stencil<double> st;
    if (!state_finite(P.p, S) || !make_stencil(s, P.p, st)) continue;
    // Recompute C' of this particle from the grid.
    double Cn[3][3] = {};
    for (int k = 0; k < K; ++k) {
      int o[3], i[3];
      offset_of(d, k, o);
      for (int a = 0; a < 3; ++a) i[a] = st.base[a] + o[a];
      double w, dw[3], dl[3];
      weight(s, st, o, w, dw, dl);
      const double* g = &grid[(size_t(sc) * nn + node_index(s, i)) * (d + 1)];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) Cn[a][b] += kappa * w * g[1 + a] * dl[b];
    }
    // F' = (I + dt C') F.
    double Ct[3][3];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double acc = 0.0;
        for (int c = 0; c < d; ++c) acc += ((c == a ? 1.0 : 0.0) + s.dt * Cn[c][a]) * G.F(c, b);
        H.F(a, b) += acc;
        double FbFt = 0.0;
        for (int c = 0; c < d; ++c) FbFt += G.F(a, c) * P.F(b, c);
        Ct[a][b] = G.C(a, b) + s.dt * FbFt;
      }
    // x' = x + dt v'.
    double vt[3];
    for (int a = 0; a < d; ++a) {
      vt[a] = G.v(a) + s.dt * G.x(a);
      H.x(a) += G.x(a);
    }
    // v' = sum w v_i,  C' = kappa sum w v_i delta^T.
    for (int k = 0; k < K; ++k) {
      int o[3], i[3];
      offset_of(d, k, o);
      for (int a = 0; a < 3; ++a) i[a] = st.base[a] + o[a];
      double w, dw[3], dl[3];
      weight(s, st, o, w, dw, dl);
      size_t q = size_t(sc) * nn + node_index(s, i);
      const double* g = &grid[q * (d + 1)];
      double r[3], vr = 0.0;
      for (int a = 0; a < d; ++a) {
        double Bd = 0.0;
        for (int b = 0; b < d; ++b) Bd += kappa * Ct[a][b] * dl[b];
        r[a] = vt[a] + Bd;
        vr += g[1 + a] * r[a];
        vbar[q * d + a] += w * r[a];
      }
      for (int c = 0; c < d; ++c) {
        double Btv = 0.0;
        for (int a = 0; a < d; ++a) Btv += kappa * Ct[a][c] * g[1 + a];
        H.x(c) += vr * dw[c] - w * Btv;
      }
    }
  }

  // Adjoint of grid_op: P* = v*/m, m* = -(v* . P)/m^2 on active nodes.
  std::vector<double> Pbar(size_t(s.n_scenes) * nn * d, 0.0), mbar(size_t(s.n_scenes) * nn, 0.0);
  for (int sc = 0; sc < s.n_scenes; ++sc)
    for (long q = 0; q < nn; ++q) {
      int i[3] = {0, 0, 0};
      long r = q;
      for (int a = d - 1; a >= 0; --a) { i[a] = int(r % s.n_grid); r /= s.n_grid; }
      size_t qq = size_t(sc) * nn + q;
      double m = grid_mP[qq * (d + 1)];
      if (!(m > 0.0 && interior(s, i))) continue;
      double vP = 0.0;
      for (int a = 0; a < d; ++a) {
        Pbar[qq * d + a] = vbar[qq * d + a] / m;
        vP += vbar[qq * d + a] * grid_mP[qq * (d + 1) + 1 + a];
      }
      mbar[qq] = -vP / (m * m);
    }

  // Adjoint of p2g: gather P*, m*; stress adjoint through neo-Hookean.
  for (int p = 0; p < N; ++p) {
    int sc = scene_of(s, p);
    PView<const double> P{in + size_t(p) * S, d};
    PView<double> H{gin + size_t(p) * S, d};
    Stencil<double> st;
    if (!state_finite(P.p, S) || !make_stencil(s, P.p, st)) continue;
    P2GTerms<double> t;
    p2g_terms(s, sc, s.E, act_s, p, P, t);
    Material<double> mat = lame(s.E[sc], s.nu[sc]);
    double Abar[3][3] = {};
    for (int k = 0; k < K; ++k) {
      int o[3], i[3];
      offset_of(d, k, o);
      for (int a = 0; a < 3; ++a) i[a] = st.base[a] + o[a];
      double w, dw[3], dl[3];
      weight(s, st, o, w, dw, dl);
      size_t q = size_t(sc) * nn + node_index(s, i);
      const double* pb = &Pbar[q * d];
      double mb = mbar[q];
      double contrib = t.mass * mb;  // m_i = sum w m_p
      for (int a = 0; a < d; ++a) {
        double Ad = 0.0;
        for (int b = 0; b < d; ++b) Ad += t.A[a][b] * dl[b];
        contrib += pb[a] * (t.mass * P.v(a) + Ad);
        H.v(a) += t.mass * w * pb[a];
        for (int b = 0; b < d; ++b) Abar[a][b] += w * pb[a] * dl[b];
      }
      for (int c = 0; c < d; ++c) {
        double AtP = 0.0;
        for (int a = 0; a < d; ++a) AtP += t.A[a][c] * pb[a];
        H.x(c) += contrib * dw[c] - w * AtP;
      }
    }
    double vol = s.vol[sc];
    double taubar[3][3], tr = 0.0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        H.C(a, b) += t.mass * Abar[a][b];
        taubar[a][b] = -s.dt * vol * kappa * Abar[a][b];
      }
    for (int a = 0; a < d; ++a) tr += taubar[a][a];
    double cof[3][3];
    cofactor(d, t.F, cof);
    double eb = 0.0;
    if (s.mat_id && s.mat_id[p] == 1) {
      // liquid: d tau / dJ = E (1 - (1 - gamma) J^-gamma) I, dJ = cof(F) : dF.
      if (re(t.J) > 0.0) {
        double E = s.E[sc], J = t.J;
        double dval = E * (1.0 - (1.0 - kTaitGamma) * std::pow(J, -kTaitGamma));
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) H.F(a, b) += dval * tr * cof[a][b];
        eb += tr * (J - std::pow(J, 1.0 - kTaitGamma));
      }
    } else if (s.model == 1) {
      if (re(t.J) > 0.0) corotated_adjoint(d, t, mat, taubar, H, eb);
    } else {
      // tau = mu (F F^T - I) + lambda ln J I
      //  => F* += mu (tau* + tau*^T) F + lambda tr(tau*) F^{-T}.
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          double sym = 0.0;
          for (int c = 0; c < d; ++c) sym += (taubar[a][c] + taubar[c][a]) * t.F[c][b];
          double Finv_t = (re(t.J) > 0.0) ? cof[a][b] / t.J : 0.0;
          H.F(a, b) += mat.mu * sym + mat.lam * tr * Finv_t;
        }
      // dtau/dE = (F F^T - I) dmu/dE + ln J dlambda/dE I.
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          double FFt = 0.0;
          for (int c = 0; c < d; ++c) FFt += t.F[a][c] * t.F[b][c];
          double dtau = mat.dmu_dE * (FFt - (a == b ? 1.0 : 0.0)) + (a == b ? mat.dlam_dE * t.lnJ : 0.0);
          eb += taubar[a][b] * dtau;
        }
    }
    if (gE) gE[sc] += eb;
    if (gact && act_s && s.act_id && s.act_id[p] >= 0) gact[s.act_id[p]] += s.act_strength * taubar[1][1];
  }
  return err;
}

}  // namespace

extern "C" {

// Mirrors Desc; kept as a plain C struct for ctypes.
struct orc_desc {
  int dim, n_grid, bound, n_scenes, n_act;
  double dx, dt, gravity, act_strength;
  const int* offsets;
  const double* E;
  const double* nu;
  const double* vol;
  const double* rho;
  const int* act_id;
  int model;
  const int* mat_id;
};

static Desc to_desc(const orc_desc* o) {
  Desc s;
  s.dim = o->dim; s.n_grid = o->n_grid; s.bound = o->bound; s.n_scenes = o->n_scenes; s.n_act = o->n_act;
  s.dx = o->dx; s.dt = o->dt; s.gravity = o->gravity; s.act_strength = o->act_strength;
  s.offsets = o->offsets; s.E = o->E; s.nu = o->nu; s.vol = o->vol; s.rho = o->rho; s.act_id = o->act_id;
  s.model = o->model;
  s.mat_id = o->mat_id;
  return s;
}

int orc_state_size(int dim) { return state_size(dim); }

// One forward step: in -> out. act_s: [n_act] actuation values at this step or null.
int orc_step_fwd(const orc_desc* o, const double* act_s, const double* in, double* out) {
  Desc s = to_desc(o);
  return step_fwd<double>(s, s.E, act_s, in, out);
}

// Grid after particle-to-grid and after the grid update, [n_scenes][nodes][d+1].
int orc_grid(const orc_desc* o, const double* act_s, const double* in, double* grid_mP, double* grid_mv) {
  Desc s = to_desc(o);
  std::vector<double> g;
  int err = p2g<double>(s, s.E, act_s, in, g);
  if (grid_mP) std::memcpy(grid_mP, g.data(), g.size() * sizeof(double));
  grid_update(s, g);
  if (grid_mv) std::memcpy(grid_mv, g.data(), g.size() * sizeof(double));
  return err;
}

// Adjoint of one step; gin, gE, gact accumulate.
int orc_step_bwd(const orc_desc* o, const double* act_s, const double* in, const double* gout, double* gin,
                 double* gE, double* gact) {
  Desc s = to_desc(o);
  return step_bwd(s, act_s, in, gout, gin, gE, gact);
}

// T forward steps from s0. act: [T][n_act] or null. tape: [(T+1)][N][S] or null. sT: final state.
int orc_run_fwd(const orc_desc* o, int T, const double* act, const double* s0, double* tape, double* sT) {
  Desc s = to_desc(o);
  int N = s.offsets[s.n_scenes], S = state_size(s.dim), err = 0;
  size_t n = size_t(N) * S;
  std::vector<double> a(s0, s0 + n), b(n);
  if (tape) std::memcpy(tape, s0, n * sizeof(double));
  for (int t = 0; t < T; ++t) {
    err |= step_fwd<double>(s, s.E, act ? act + size_t(t) * s.n_act : nullptr, a.data(), b.data());
    a.swap(b);
    if (tape) std::memcpy(tape + size_t(t + 1) * n, a.data(), n * sizeof(double));
  }
  if (sT) std::memcpy(sT, a.data(), n * sizeof(double));
  return err;
}

// Reverse pass over T steps with segment checkpointing every K steps
// (Appendix D.2): the forward keeps states 0, K, 2K, ...; each segment is
// recomputed from its checkpoint, then its steps are reversed. K >= T is the
// full tape. gT: adjoint of the final state. g0, gE [n_scenes], gact [T][n_act]
// accumulate.
int orc_run_bwd(const orc_desc* o, int T, int K, const double* act, const double* s0, const double* gT,
                double* g0, double* gE, double* gact) {
  Desc s = to_desc(o);
  if (K <= 0 || K > T) K = T;
  int N = s.offsets[s.n_scenes], S = state_size(s.dim), err = 0;
  size_t n = size_t(N) * S;
  int n_seg = (T + K - 1) / K;
  std::vector<std::vector<double>> ckpt(n_seg);
  std::vector<double> a(s0, s0 + n), b(n);
  for (int t = 0; t < T; ++t) {
    if (t % K == 0) ckpt[t / K] = a;
    err |= step_fwd<double>(s, s.E, act ? act + size_t(t) * s.n_act : nullptr, a.data(), b.data());
    a.swap(b);
  }
  std::vector<double> gnext(gT, gT + n), gcur(n);
  for (int j = n_seg - 1; j >= 0; --j) {
    int t0 = j * K, t1 = std::min(T, (j + 1) * K);
    std::vector<std::vector<double>> seg(t1 - t0);
    seg[0] = ckpt[j];
    for (int t = t0; t + 1 < t1; ++t) {
      seg[t - t0 + 1].resize(n);
      step_fwd<double>(s, s.E, act ? act + size_t(t) * s.n_act : nullptr, seg[t - t0].data(),
                       seg[t - t0 + 1].data());
    }
    for (int t = t1 - 1; t >= t0; --t) {
      std::fill(gcur.begin(), gcur.end(), 0.0);
      const double* at = act ? act + size_t(t) * s.n_act : nullptr;
      double* gat = gact ? gact + size_t(t) * s.n_act : nullptr;
      step_bwd(s, at, seg[t - t0].data(), gnext.data(), gcur.data(), gE, gat);
      gnext.swap(gcur);
    }
  }
  for (size_t q = 0; q < n; ++q) g0[q] += gnext[q];
  return err;
}

// Complex-step tangent of T forward steps: perturbs s0 by h*s0_dir, E by
// h*E_dir [n_scenes] and act by h*act_dir [T][n_act] (each may be null) and
// returns the real final state and d(sT)/d(direction) = Im(sT(x + i h dir)) / h.
int orc_run_fwd_cs(const orc_desc* o, int T, const double* act, const double* act_dir, const double* s0,
                   const double* s0_dir, const double* E_dir, double h, double* sT, double* sT_tan) {
  Desc s = to_desc(o);
  int N = s.offsets[s.n_scenes], S = state_size(s.dim), err = 0;
  size_t n = size_t(N) * S;
  std::vector<cd> a(n), b(n), Ec(s.n_scenes), ac;
  for (size_t q = 0; q < n; ++q) a[q] = cd(s0[q], s0_dir ? h * s0_dir[q] : 0.0);
  for (int k = 0; k < s.n_scenes; ++k) Ec[k] = cd(s.E[k], E_dir ? h * E_dir[k] : 0.0);
  if (act) {
    ac.resize(size_t(T) * s.n_act);
    for (size_t q = 0; q < ac.size(); ++q) ac[q] = cd(act[q], act_dir ? h * act_dir[q] : 0.0);
  }
  for (int t = 0; t < T; ++t) {
    err |= step_fwd<cd>(s, Ec.data(), act ? ac.data() + size_t(t) * s.n_act : nullptr, a.data(), b.data());
    a.swap(b);
  }
  for (size_t q = 0; q < n; ++q) {
    if (sT) sT[q] = a[q].real();
    if (sT_tan) sT_tan[q] = a[q].imag() / h;
  }
  return err;
}

}  // extern "C"

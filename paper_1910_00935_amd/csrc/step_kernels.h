// Fused per-particle kernels of the MLS-MPM step and its adjoint (gfx950).
//
// Forward, one launch per step s (DiffTaichi Appendix D.1 stage order, with
// the grid update folded into the gather and the next step's scatter fused
// behind it):
//     k_fwd(s):  g2p(s) from grid s  ->  state s+1  ->  p2g(s+1) into grid s+1
// Reverse, one launch per step s (grid recomputed, never stored):
//     k_bwd(s):  A  p2g*(s+1): gather grid s+1 and its adjoint -> dL/dstate(s+1)
//                B  g2p*(s):   scatter dL/dv_i of grid s, keep x*, F* partials
//                C  p2g(s-1):  recompute grid s-1 for the next launch
// The grid adjoint (grid_op*) is folded into phase A's gather:
//     P*_i = v*_i / m_i,  m*_i = -(v*_i . P_i) / m_i^2  on active nodes.
// Each launch also zeroes grid buffers that no in-flight phase touches.
//
// Grids are dense per scene, one float4 per node: (m, P_0, P_1, P_2) for the
// primal (P = momentum; v is formed at gather time), (v*_0, v*_1, v*_2, -) for
// the adjoint. Scatters use hardware FP32 atomics; per-scene dL/dE and
// per-actuator dL/da are reduced per wavefront and added in FP64.
#pragma once

#include "device_math.h"

namespace mpm {

struct StepConsts {
  int N;          // particles
  int n;          // nodes per axis
  int bound;      // sticky band width
  int nodes;      // n^d, nodes per scene
  int n_act;      // actuator columns
  float dx, inv_dx, dt, gdt, kappa, act_strength;
  const int* scene_id;  // [N] scene of each particle, or null (one scene)
  const float* E;
  const float* nu;
  const float* vol;
  const float* rho;
  const int* act_id;    // [N] in this launch's particle order, or null
  unsigned* err;
};

struct FwdArgs {
  StepConsts k;
  StateRef in;             // state s
  StateRef out;            // state s+1 (written when do_g2p)
  const float4* grid_in;   // grid s, (m, P) (read when do_g2p)
  float4* grid_out;        // grid s+1 (scattered when do_p2g)
  const float* act_row;    // actuation row of the scattered state, or null
  int do_g2p, do_p2g;
  float4* clear;           // buffer zeroed by this launch, or null
  long clear_n;            // float4 count
};

struct BwdArgs {
  StepConsts k;
  // Phase A: dL/dstate(s+1) from its seed (a_mode 0) or via p2g*(s+1) (a_mode 1).
  int a_mode;
  StateRef stA;            // state s+1
  const float4* gA;        // grid s+1 (m, P)
  const float4* aA;        // adjoint grid s+1 (v*)
  const float* act_rowA;   // actuation row s+1 or null
  double* gact_rowA;       // dL/da row s+1 (FP64, accumulate) or null
  double* gE;              // [n_scenes] dL/dE (FP64, accumulate) or null
  StateRef seed;           // a_mode 0: dL/dstate(s+1)
  // Output instead of phase B/C: out[perm ? perm[i] : i] += dL/dstate.
  int final_out;
  StateRef out;
  const int* out_perm;
  // Phase B: g2p*(s).
  StateRef stB;            // state s (x, F read)
  const float* cnext;      // C of state s+1, component-major with stride cnext_stride, or null (recompute)
  int cnext_stride;
  const float4* gB;        // grid s (m, P)
  float4* aB;              // adjoint grid s (scatter)
  // x*, F* partials of state s (written by B, read by the next launch's A):
  // component-major [d + d*d][pstride].
  float* partial;
  int pstride;
  // Phase C: p2g(s-1) recompute.
  int do_c;
  StateRef stC;
  const float* act_rowC;
  float4* gC;
  float4* clear0;
  long clear0_n;
  float4* clear1;
  long clear1_n;
};

template <int D, class Fn>
__device__ __forceinline__ void for_nodes(Fn&& fn) {
  if constexpr (D == 2) {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) fn(o0, o1, 0);
  } else {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2) fn(o0, o1, o2);
  }
}

template <int D>
__device__ __forceinline__ float wgt(const Sten<D>& st, int o0, int o1, int o2) {
  float w = st.N[0][o0] * st.N[1][o1];
  if constexpr (D == 3) w *= st.N[2][o2];
  return w;
}

// Gradient of the weight with respect to x_p.
template <int D>
__device__ __forceinline__ void dwgt(const Sten<D>& st, int o0, int o1, int o2, float inv_dx, float (&g)[D]) {
  if constexpr (D == 2) {
    g[0] = st.dN[0][o0] * st.N[1][o1] * inv_dx;
    g[1] = st.N[0][o0] * st.dN[1][o1] * inv_dx;
  } else {
    g[0] = st.dN[0][o0] * st.N[1][o1] * st.N[2][o2] * inv_dx;
    g[1] = st.N[0][o0] * st.dN[1][o1] * st.N[2][o2] * inv_dx;
    g[2] = st.N[0][o0] * st.N[1][o1] * st.dN[2][o2] * inv_dx;
  }
}

template <int D>
__device__ __forceinline__ void delta(const Sten<D>& st, int o0, int o1, int o2, float dx, float (&dl)[D]) {
  const int o[3] = {o0, o1, o2};
#pragma unroll
  for (int a = 0; a < D; ++a) dl[a] = (float(o[a]) - st.f[a]) * dx;
}

template <int D>
__device__ __forceinline__ bool node_active(const Sten<D>& st, int o0, int o1, int o2, int n, int bound, float m) {
  bool in = interior1(st.base[0] + o0, n, bound) && interior1(st.base[1] + o1, n, bound);
  if constexpr (D == 3) in = in && interior1(st.base[2] + o2, n, bound);
  return in && m > 0.0f;
}

__device__ __forceinline__ void zero_range(float4* p, long n) {
  if (!p) return;
  const long stride = long(gridDim.x) * blockDim.x;
  for (long q = long(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// p2g of one particle into its scene's grid.
template <int D>
__device__ __forceinline__ void p2g_particle(const StepConsts& k, int i, int sc, const PState<D>& p,
                                             const float* act_row, float4* grid, unsigned& err) {
  Sten<D> st;
  if (!state_finite<D>(p)) {
    err |= kErrNonfinite;
    return;
  }
  if (!make_sten<D>(p.x, k.inv_dx, k.n, st)) {
    err |= kErrDomain;
    return;
  }
  const SceneParams sp = scene_params(k.E, k.nu, k.vol, k.rho, sc);
  float act_tau = 0.0f;
  if (act_row && k.act_id) {
    const int aid = k.act_id[i];
    if (aid >= 0) act_tau = k.act_strength * act_row[aid];
  }
  float A[D][D], FFtI[D][D], lnJ, J;
  affine<D>(p, sp, act_tau, k.dt, k.kappa, A, FFtI, lnJ, J, err);
  float mv[D];
#pragma unroll
  for (int a = 0; a < D; ++a) mv[a] = sp.mass * p.v[a];
  float4* g = grid + long(sc) * k.nodes;
  for_nodes<D>([&](int o0, int o1, int o2) {
    const float w = wgt<D>(st, o0, o1, o2);
    float dl[D];
    delta<D>(st, o0, o1, o2, k.dx, dl);
    float* node = reinterpret_cast<float*>(g + node_of<D>(st.base, o0, o1, o2, k.n));
    atomic_add_f32(node, w * sp.mass);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float Ad = 0.0f;
#pragma unroll
      for (int b = 0; b < D; ++b) Ad += A[a][b] * dl[b];
      atomic_add_f32(node + 1 + a, w * (mv[a] + Ad));
    }
  });
}

// Node velocity after the grid update, from (m, P).
template <int D>
__device__ __forceinline__ void node_velocity(const StepConsts& k, const Sten<D>& st, int o0, int o1, int o2,
                                              float4 g, float (&v)[D]) {
  const bool act = node_active<D>(st, o0, o1, o2, k.n, k.bound, g.x);
  const float P[3] = {g.y, g.z, g.w};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float va = P[a] / g.x + (a == 1 ? k.gdt : 0.0f);
    v[a] = act ? va : 0.0f;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_fwd(FwdArgs a) {
  zero_range(a.clear, a.clear_n);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.k.N) return;
  const StepConsts& k = a.k;
  const int sc = k.scene_id ? k.scene_id[i] : 0;
  unsigned err = 0;
  PState<D> p;
  load_state<D>(a.in, i, p);
  if (a.do_g2p) {
    Sten<D> st;
    const bool fin = state_finite<D>(p);
    const bool ok = fin && make_sten<D>(p.x, k.inv_dx, k.n, st);
    if (ok) {
      const float4* g = a.grid_in + long(sc) * k.nodes;
      float vn[D] = {}, Cn[D][D] = {};
      for_nodes<D>([&](int o0, int o1, int o2) {
        const float w = wgt<D>(st, o0, o1, o2);
        float dl[D], v[D];
        delta<D>(st, o0, o1, o2, k.dx, dl);
        node_velocity<D>(k, st, o0, o1, o2, g[node_of<D>(st.base, o0, o1, o2, k.n)], v);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          vn[c] += w * v[c];
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[c][b] += w * v[c] * dl[b];
        }
      });
      float Fn[D][D];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          Cn[c][b] *= k.kappa;
        }
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          float s = p.F[c][b];
#pragma unroll
          for (int e = 0; e < D; ++e) s += k.dt * Cn[c][e] * p.F[e][b];
          Fn[c][b] = s;
        }
#pragma unroll
      for (int c = 0; c < D; ++c) {
        p.v[c] = vn[c];
        p.x[c] += k.dt * vn[c];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          p.C[c][b] = Cn[c][b];
          p.F[c][b] = Fn[c][b];
        }
      }
    } else {
      err |= fin ? kErrDomain : kErrNonfinite;
    }
    store_state<D>(a.out, i, p);
  }
  if (a.do_p2g) p2g_particle<D>(k, i, sc, p, a.act_row, a.grid_out, err);
  if (err) atomicOr(k.err, err);
}

// Sum `val` over the live lanes of the wavefront that share `key`, and add
// each group's sum (FP64) to base[key] once.
__device__ __forceinline__ void wave_add_keyed(bool live, int key, double val, double* base) {
  unsigned long long mask = __ballot(live);
  const int lane = threadIdx.x & 63;
  while (mask) {
    const int leader = __ffsll((long long)mask) - 1;
    const int kk = __shfl(key, leader, 64);
    const bool mine = live && key == kk;
    const double s = wave_sum(mine ? val : 0.0);
    if (lane == leader) atomic_add_f64(base + kk, s);
    mask &= ~__ballot(mine);
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_bwd(BwdArgs a) {
  zero_range(a.clear0, a.clear0_n);
  zero_range(a.clear1, a.clear1_n);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const StepConsts& k = a.k;
  const bool live = i < k.N;
  const int ii = live ? i : 0;
  const int sc = (k.scene_id && live) ? k.scene_id[ii] : 0;
  unsigned err = 0;

  // dL/dstate(s+1): gx, gv, gC, gF.
  float gx[D], gv[D], gC[D][D], gF[D][D];
  double eb = 0.0, actb = 0.0;
  int aid = -1;
  if (a.a_mode == 0) {
    if (live) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        gx[c] = a.seed.x[c * a.seed.stride + i];
        gv[c] = a.seed.v[c * a.seed.stride + i];
      }
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          gC[c][b] = a.seed.C[(c * D + b) * a.seed.stride + i];
          gF[c][b] = a.seed.F[(c * D + b) * a.seed.stride + i];
        }
    }
  } else if (live) {
    // p2g*(s+1) with grid_op* folded into the gather.
    PState<D> p;
    load_state<D>(a.stA, i, p);
#pragma unroll
    for (int c = 0; c < D; ++c) gx[c] = a.partial[c * a.pstride + i];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) gF[c][b] = a.partial[(D + c * D + b) * a.pstride + i];
    float Abar[D][D] = {}, vb[D] = {};
    Sten<D> st;
    const bool ok = state_finite<D>(p) && make_sten<D>(p.x, k.inv_dx, k.n, st);
    if (ok) {
      const SceneParams sp = scene_params(k.E, k.nu, k.vol, k.rho, sc);
      float act_tau = 0.0f;
      if (a.act_rowA && k.act_id) {
        aid = k.act_id[i];
        if (aid >= 0) act_tau = k.act_strength * a.act_rowA[aid];
      }
      float A[D][D], FFtI[D][D], lnJ, J;
      unsigned dummy = 0;
      affine<D>(p, sp, act_tau, k.dt, k.kappa, A, FFtI, lnJ, J, dummy);
      float mv[D];
#pragma unroll
      for (int c = 0; c < D; ++c) mv[c] = sp.mass * p.v[c];
      const float4* g = a.gA + long(sc) * k.nodes;
      const float4* ad = a.aA + long(sc) * k.nodes;
      for_nodes<D>([&](int o0, int o1, int o2) {
        const int q = node_of<D>(st.base, o0, o1, o2, k.n);
        const float4 gm = g[q];
        const float4 vb4 = ad[q];
        const bool act = node_active<D>(st, o0, o1, o2, k.n, k.bound, gm.x);
        const float inv_m = act ? 1.0f / gm.x : 0.0f;
        const float P[3] = {gm.y, gm.z, gm.w};
        const float V[3] = {vb4.x, vb4.y, vb4.z};
        float Pb[D];
        float vP = 0.0f;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          Pb[c] = V[c] * inv_m;
          vP += V[c] * P[c];
        }
        const float mb = -vP * inv_m * inv_m;
        const float w = wgt<D>(st, o0, o1, o2);
        float dw[D], dl[D];
        dwgt<D>(st, o0, o1, o2, k.inv_dx, dw);
        delta<D>(st, o0, o1, o2, k.dx, dl);
        float contrib = sp.mass * mb;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          float Ad = 0.0f;
#pragma unroll
          for (int b = 0; b < D; ++b) Ad += A[c][b] * dl[b];
          contrib += Pb[c] * (mv[c] + Ad);
          vb[c] += w * Pb[c];
#pragma unroll
          for (int b = 0; b < D; ++b) Abar[c][b] += w * Pb[c] * dl[b];
        }
#pragma unroll
        for (int e = 0; e < D; ++e) {
          float AtP = 0.0f;
#pragma unroll
          for (int c = 0; c < D; ++c) AtP += A[c][e] * Pb[c];
          gx[e] += contrib * dw[e] - w * AtP;
        }
      });
      const float kt = -k.dt * sp.vol * k.kappa;
      float tb[D][D], tr = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        gv[c] = sp.mass * vb[c];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          gC[c][b] = sp.mass * Abar[c][b];
          tb[c][b] = kt * Abar[c][b];
        }
        tr += tb[c][c];
      }
      // tau = mu (F F^T - I) + lambda ln J I:
      // F* += mu (tau* + tau*^T) F + lambda tr(tau*) F^{-T}.
      float K[D][D];
      cofactor<D>(p.F, K);
      const float lam_tr_invJ = (J > 0.0f) ? sp.lam * tr / J : 0.0f;
      float ebf = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          float sym = 0.0f;
#pragma unroll
          for (int e = 0; e < D; ++e) sym += (tb[c][e] + tb[e][c]) * p.F[e][b];
          gF[c][b] += sp.mu * sym + lam_tr_invJ * K[c][b];
          ebf += tb[c][b] * (sp.dmu_dE * FFtI[c][b] + (c == b ? sp.dlam_dE * lnJ : 0.0f));
        }
      eb = ebf;
      actb = double(k.act_strength) * tb[1][1];
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        gv[c] = 0.0f;
#pragma unroll
        for (int b = 0; b < D; ++b) gC[c][b] = 0.0f;
      }
    }
  }
  if (a.a_mode == 1) {
    if (a.gE) wave_add_keyed(live, sc, eb, a.gE);
    if (a.gact_rowA && k.act_id) {
      for (int kk = 0; kk < k.n_act; ++kk) {
        const double s = wave_sum((live && aid == kk) ? actb : 0.0);
        if ((threadIdx.x & 63) == 0 && s != 0.0) atomic_add_f64(a.gact_rowA + kk, s);
      }
    }
  }
  if (!live) return;

  if (a.final_out) {
    const int o = a.out_perm ? a.out_perm[i] : i;
    const int os = a.out.stride;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      a.out.x[c * os + o] += gx[c];
      a.out.v[c * os + o] += gv[c];
    }
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        a.out.C[(c * D + b) * os + o] += gC[c][b];
        a.out.F[(c * D + b) * os + o] += gF[c][b];
      }
    return;
  }

  // Phase B: g2p*(s).
  {
    PState<D> p;
    load_xF<D>(a.stB, i, p);
    float px[D], pF[D][D];
#pragma unroll
    for (int c = 0; c < D; ++c) px[c] = gx[c];
    Sten<D> st;
    bool fin = true;
#pragma unroll
    for (int c = 0; c < D; ++c) fin = fin && (p.x[c] * 0.0f == 0.0f);
    const bool ok = fin && make_sten<D>(p.x, k.inv_dx, k.n, st);
    if (ok) {
      const float4* g = a.gB + long(sc) * k.nodes;
      float Cn[D][D];
      if (a.cnext) {
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[c][b] = a.cnext[(c * D + b) * a.cnext_stride + i];
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[c][b] = 0.0f;
        for_nodes<D>([&](int o0, int o1, int o2) {
          const float w = wgt<D>(st, o0, o1, o2);
          float dl[D], v[D];
          delta<D>(st, o0, o1, o2, k.dx, dl);
          node_velocity<D>(k, st, o0, o1, o2, g[node_of<D>(st.base, o0, o1, o2, k.n)], v);
#pragma unroll
          for (int c = 0; c < D; ++c)
#pragma unroll
            for (int b = 0; b < D; ++b) Cn[c][b] += w * v[c] * dl[b];
        });
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[c][b] *= k.kappa;
      }
      // F' = (I + dt C') F:  F* = (I + dt C')^T F'*,  C'* += dt F'* F^T.
      float Bm[D][D], vt[D];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          float s = gF[c][b];
#pragma unroll
          for (int e = 0; e < D; ++e) s += k.dt * Cn[e][c] * gF[e][b];
          pF[c][b] = s;
          float t = 0.0f;
#pragma unroll
          for (int e = 0; e < D; ++e) t += gF[c][e] * p.F[b][e];
          Bm[c][b] = k.kappa * (gC[c][b] + k.dt * t);
        }
      // x' = x + dt v':  v'* += dt x'*.
#pragma unroll
      for (int c = 0; c < D; ++c) vt[c] = gv[c] + k.dt * gx[c];
      float4* ad = a.aB + long(sc) * k.nodes;
      for_nodes<D>([&](int o0, int o1, int o2) {
        const int q = node_of<D>(st.base, o0, o1, o2, k.n);
        float v[D];
        node_velocity<D>(k, st, o0, o1, o2, g[q], v);
        const float w = wgt<D>(st, o0, o1, o2);
        float dw[D], dl[D];
        dwgt<D>(st, o0, o1, o2, k.inv_dx, dw);
        delta<D>(st, o0, o1, o2, k.dx, dl);
        float r[D], vr = 0.0f;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          float s = vt[c];
#pragma unroll
          for (int b = 0; b < D; ++b) s += Bm[c][b] * dl[b];
          r[c] = s;
          vr += v[c] * s;
        }
        float* node = reinterpret_cast<float*>(ad + q);
#pragma unroll
        for (int c = 0; c < D; ++c) atomic_add_f32(node + c, w * r[c]);
#pragma unroll
        for (int e = 0; e < D; ++e) {
          float Btv = 0.0f;
#pragma unroll
          for (int c = 0; c < D; ++c) Btv += Bm[c][e] * v[c];
          px[e] += vr * dw[e] - w * Btv;
        }
      });
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) pF[c][b] = gF[c][b];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) a.partial[c * a.pstride + i] = px[c];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) a.partial[(D + c * D + b) * a.pstride + i] = pF[c][b];
  }

  // Phase C: recompute p2g(s-1).
  if (a.do_c) {
    PState<D> p;
    load_state<D>(a.stC, i, p);
    p2g_particle<D>(k, i, sc, p, a.act_rowC, a.gC, err);
  }
  if (err) atomicOr(k.err, err);
}

}  // namespace mpm

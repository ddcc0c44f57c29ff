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
// the adjoint.
//
// LDS staging: particles are sorted by cell (Morton order), so the stencils of
// one workgroup cover a small box of nodes. Each phase computes that box
// (block-wide min/max of the stencil bases); when it fits kTileCap<D> nodes and
// the workgroup holds one scene, gathers read the box once into LDS and
// scatters accumulate in LDS and flush each non-zero node to HBM with one
// hardware FP32 atomic per component. Otherwise the phase reads and scatters
// global memory directly. Per-scene dL/dE and per-actuator dL/da are reduced
// per wavefront and added in FP64.
//
// LDS scatters accumulate in 64-bit fixed point with integer LDS atomics
// (ds_add_u64): on gfx950 ds_add_f32 sustains ~0.3 lane-ops per clock per CU
// against ~8 for ds_add_u64 and ~14 for ds_add_u32. Each workgroup reduces a
// bound B on |contribution| over its particles and uses the scale 2^e with
// B 2^e < 2^31: every contribution rounds to a 32-bit integer (error below
// B 2^-31, finer than the FP32 rounding of a partial sum), node sums cannot
// overflow 64 bits, and the accumulation does not depend on atomic order; the
// flush converts each node back to float once.
#pragma once

#include <hip/hip_cooperative_groups.h>

#include <climits>

#include "device_math.h"

namespace mpm {

// Nodes per LDS tile: 1024 in 3D, 768 in 2D. A workgroup whose box exceeds it
// falls back to global atomics, which costs far more than the LDS it would
// have used: in the batched 2D workload at 256 particles per workgroup about
// 5 % of the boxes exceed 512 nodes and under 1 % exceed 768, and 768 still
// leaves the kernels' LDS use balanced with their register use. In 3D, 512
// nodes cover the lattice workloads (boxes of ~245 nodes) but not the robot
// beside the liquid once the liquid spreads (11 % of late scatters fell back,
// and its trajectories took twice as long); 1024 covers all of them.
template <int D>
constexpr int kTileCap = (D == 3) ? 1024 : 768;
static_assert((3 * kTileCap<2>) % 2 == 0 && (3 * kTileCap<3>) % 2 == 0, "zero_tile64 clears whole 16-byte pairs");

struct StepConsts {
  int N;          // particles
  int n;          // nodes per axis
  int bound;      // sticky band width
  int nodes;      // n^d, nodes per scene
  int n_act;      // actuator columns
  int n_scenes;
  int lds;        // 1: stage gathers and scatters in LDS when the box fits
  int remap;      // 1: interleave the workgroup's particles across waves (lane_particle)
  int rotate;     // 1: per-lane stencil visiting order (Sten, lane_color)
  float dx, inv_dx, dt, gdt, kappa, act_strength;
  const int* mat_id;    // [N] material per particle (0 solid, 1 liquid) or null
  const int4* blocks;   // [n_blocks] scene-aligned workgroups (first, count, scene); required with
                        // several scenes, null with one
  int n_blocks;         // workgroups per particle pass
  int threads;          // threads per workgroup of this launch (blockDim.x, kept in a scalar register)
  int groups;           // workgroups that share the launch's clears (their clear ranks 0..groups-1)
  int clear_per_role;   // of each clearing role's n_blocks workgroups, the first clear_per_role take part
  const float* E;
  const float* nu;
  const float* vol;
  const float* rho;
  const int* act_id;    // [N] in this launch's particle order, or null
  unsigned* err;
  unsigned long long* tstats;  // null, or [2]: scatters accumulated in an LDS tile, scatters that fell back
                               // to global atomics (one count per workgroup and scatter)
  // Workgroup wall clock (mpm_wg_clock_bind), or null: entry and exit stamps of
  // the constant-rate device clock of every workgroup of this launch, at
  // wgclk[2 * (clk_slot * clk_stride + workgroup)] (clk_slot < 0: not stamped).
  unsigned long long* wgclk = nullptr;
  int clk_slot = -1;
  int clk_stride = 0;
};

struct FwdArgs {
  StepConsts k;
  StateRef in;             // state s
  StateRef out;            // state s+1 (written when do_g2p)
  const float4* grid_in;   // grid s, (m, P) (read when do_g2p)
  float4* grid_out;        // grid s+1 (scattered when do_p2g)
  const float* act_row;    // actuation row of the scattered state, or null
  int do_g2p, do_p2g;
  float4* clear;           // grid zeroed by this launch, or null
  long clear_n;            // float4 count (dense clear)
  const int4* clear_box;   // or: the boxes its last scatter recorded (clear_nbox workgroups)
  int clear_nbox;
  int clear_wgs;           // workgroups after the k.n_blocks stepping ones that only clear (0: the stepping ones clear)
  int4* box_out;           // box table of grid_out (record_box), or null
  const int4* box_in;      // box table the scatter into grid_in recorded (this launch's workgroups), or null
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
  int split_c;             // phase C in its own workgroups (grid of 2 nb)
  StateRef stC;
  const float* act_rowC;
  float4* gC;
  float4* clear0;
  long clear0_n;
  const int4* clear0_box;
  int clear0_nbox;
  float4* clear1;
  long clear1_n;
  const int4* clear1_box;
  int clear1_nbox;
  int4* boxB;              // box tables of aB and gC (record_box), or null
  int4* boxC;
  const int4* boxA_in;     // box tables the scatters into gA and gB recorded, or null
  const int4* boxB_in;
};

// Visits the stencil nodes (t0, t1, t2) in the lane's order (see Sten).
// S0 = 3: all of them; S0 = 1: only the slab t0 = 0 (quad mode: the lane's own
// slab); S0 = 2: the first H of them in flat order t0 * 9 + t1 * 3 + t2 (pair
// mode), the last one skipped when st.skip_last.
template <int D, int S0, class Fn>
__device__ __forceinline__ void for_nodes(const Sten<D>& st, Fn&& fn) {
  if constexpr (S0 == 2) {
    constexpr int H = (D == 3) ? 14 : 5;
#pragma unroll
    for (int f = 0; f < H - 1; ++f) {
      if constexpr (D == 3)
        fn(f / 9, (f / 3) % 3, f % 3);
      else
        fn(f / 3, f % 3, 0);
    }
    if (!st.skip_last) {
      constexpr int f = H - 1;
      if constexpr (D == 3)
        fn(f / 9, (f / 3) % 3, f % 3);
      else
        fn(f / 3, f % 3, 0);
    }
  } else if constexpr (D == 2) {
#pragma unroll
    for (int o0 = 0; o0 < S0; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) fn(o0, o1, 0);
  } else {
#pragma unroll
    for (int o0 = 0; o0 < S0; ++o0)
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
  (void)dx;
  dl[0] = st.dl[0][o0];
  dl[1] = st.dl[1][o1];
  if constexpr (D == 3) dl[2] = st.dl[2][o2];
}

// Global index of visited node (t0, t1, t2) within its scene's grid.
template <int D>
__device__ __forceinline__ int node_of(const Sten<D>& st, int o0, int o1, int o2, int n) {
  if constexpr (D == 2) {
    return st.nc[0][o0] * n + st.nc[1][o1];
  } else {
    return (st.nc[0][o0] * n + st.nc[1][o1]) * n + st.nc[2][o2];
  }
}

template <int D>
__device__ __forceinline__ bool node_active(const Sten<D>& st, int o0, int o1, int o2, int n, int bound, float m) {
  bool in = interior1(st.nc[0][o0], n, bound) && interior1(st.nc[1][o1], n, bound);
  if constexpr (D == 3) in = in && interior1(st.nc[2][o2], n, bound);
  return in && m > 0.0f;
}

__device__ __forceinline__ void zero_range(float4* p, long n, int threads, int groups, int rank) {
  if (!p || rank < 0) return;
  const long stride = long(groups) * threads;
  for (long q = long(rank) * threads + threadIdx.x; q < n; q += stride) p[q] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Read of a value that is uniform over the workgroup and was written by an
// earlier launch (box tables): through the constant address space, so it is a
// scalar load counted apart from the vector loads issued before it, and its
// use does not wait for them.
typedef __attribute__((address_space(4))) const int4 uniform_int4;
__device__ __forceinline__ int4 load_uniform(const int4* p) {
  const uniform_int4* q = (const uniform_int4*)(p);
  return make_int4(q->x, q->y, q->z, q->w);
}

// A box record or clear box: a scalar load (load_uniform) when the table was
// written by an earlier launch; with P (the persistent kernels, where the
// table was written before the last grid-wide barrier of the same launch) a
// vector load that bypasses the non-coherent per-CU caches, since the scalar
// cache is not invalidated by the barrier.
template <bool P>
__device__ __forceinline__ int4 load_box(const int4* p) {
  if constexpr (P) {
    const volatile int* q = reinterpret_cast<const volatile int*>(p);
    return make_int4(q[0], q[1], q[2], q[3]);
  } else {
    return load_uniform(p);
  }
}

// (r / d, r % d) for 0 <= r < 2^16 and 1 <= d <= 2^10, with rcp = (1/d)(1 + 2^-20):
// the product r * rcp then lies in [r/d, floor(r/d) + 1) exactly as in real
// arithmetic, so its truncation is the quotient.
__device__ __forceinline__ int div_small(int r, int d, float rcp, int& rem) {
  const int q = int(float(r) * rcp);
  rem = r - q * d;
  return q;
}

// Sparse clears. A scatter launch records, per workgroup, the box of nodes
// it may have written (record_box): two int4, (lo_0, lo_1, lo_2, scene) and
// (ext_0, ext_1, ext_2, 0), scene -1 for every scene, ext_0 = 0 for none. The
// launch that later clears that grid zeroes the recorded boxes instead of the
// whole grid; boxes are clamped to the grid.
template <int D>
__device__ __forceinline__ void clear_box_nodes(float4* grid, int4 lo, int4 ex, int n, int nodes, int n_scenes,
                                                int threads) {
  const int l0 = max(lo.x, 0), l1 = max(lo.y, 0), l2 = (D == 3) ? max(lo.z, 0) : 0;
  const int e0 = min(lo.x + ex.x, n) - l0, e1 = min(lo.y + ex.y, n) - l1;
  const int e2 = (D == 3) ? min(lo.z + ex.z, n) - l2 : 1;
  if (e0 <= 0 || e1 <= 0 || e2 <= 0) return;
  const int total = e0 * e1 * e2;
  const bool small = total < 65536 && e1 <= 1024 && e2 <= 1024;
  const float r1 = small ? (1.0f / float(e1)) * (1.0f + 0x1p-20f) : 0.0f;
  const float r2 = small ? (1.0f / float(e2)) * (1.0f + 0x1p-20f) : 0.0f;
  const int s0 = (lo.w >= 0) ? lo.w : 0;
  const int s1 = (lo.w >= 0) ? min(lo.w + 1, n_scenes) : n_scenes;
  for (int sc = s0; sc < s1; ++sc) {
    float4* g = grid + long(sc) * nodes;
    for (int q = threadIdx.x; q < total; q += threads) {
      int c0, c1, c2, r;
      if (small) {
        r = div_small(q, e2, r2, c2);
        c0 = div_small(r, e1, r1, c1);
      } else {
        c2 = q % e2;
        r = q / e2;
        c1 = r % e1;
        c0 = r / e1;
      }
      const long idx = (D == 3) ? (long(l0 + c0) * n + (l1 + c1)) * n + (l2 + c2) : long(l0 + c0) * n + (l1 + c1);
      g[idx] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// One grid a launch clears: by its recorded boxes (box, nbox entries) or
// densely (dense_n float4), or not at all (g null).
struct ClearSpec {
  float4* g;
  const int4* box;
  int nbox;
  long dense_n;
};

// The box entries of two concatenated tables are spread over the launch's
// workgroups; a workgroup fetches its first two entries early (the loads
// overlap its other reads) and clears them later.
struct ClearJobs {
  int4 lo[2], ex[2];
  int which[2];
  int n;
};

__device__ __forceinline__ int clear_entries(const ClearSpec& s) { return (s.g && s.box) ? s.nbox : 0; }

template <bool P>
__device__ __forceinline__ void clear_entry(const ClearSpec& s0, const ClearSpec& s1, int j, int4& lo, int4& ex,
                                            int& which) {
  const int m0 = clear_entries(s0);
  which = j < m0 ? 0 : 1;
  const int4* t = which == 0 ? s0.box : s1.box;
  const int jj = which == 0 ? j : j - m0;
  lo = load_box<P>(t + 2 * jj);
  ex = load_box<P>(t + 2 * jj + 1);
}

// Clear rank of a workgroup: its index among the workgroups that take part in
// the launch's clears, or -1. Of each clearing role's n_blocks workgroups the
// first clear_per_role do (the aligned partition's trailing empty workgroups
// therefore never do); `offset` places a second role's ranks after the
// first's.
__device__ __forceinline__ int clear_rank(const StepConsts& k, int wg, bool takes_clears, int offset) {
  return (takes_clears && wg < k.clear_per_role) ? offset + wg : -1;
}

template <bool P>
__device__ __forceinline__ ClearJobs clear_jobs_fetch(const ClearSpec& s0, const ClearSpec& s1, int rank, int groups) {
  ClearJobs c;
  c.n = 0;
  if (rank < 0) return c;
  const int m = clear_entries(s0) + clear_entries(s1);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = rank + r * groups;
    if (j < m) {
      clear_entry<P>(s0, s1, j, c.lo[r], c.ex[r], c.which[r]);
      c.n = r + 1;
    }
  }
  return c;
}

template <int D, bool P>
__device__ __forceinline__ void clear_jobs_run(const ClearJobs& c, const ClearSpec& s0, const ClearSpec& s1,
                                               const StepConsts& k, int rank) {
  if (rank < 0) return;
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (r < c.n)
      clear_box_nodes<D>(c.which[r] == 0 ? s0.g : s1.g, c.lo[r], c.ex[r], k.n, k.nodes, k.n_scenes, k.threads);
  const int m = clear_entries(s0) + clear_entries(s1);
  for (int j = rank + 2 * k.groups; j < m; j += k.groups) {
    int4 lo, ex;
    int which;
    clear_entry<P>(s0, s1, j, lo, ex, which);
    clear_box_nodes<D>(which == 0 ? s0.g : s1.g, lo, ex, k.n, k.nodes, k.n_scenes, k.threads);
  }
  if (s0.g && !s0.box) zero_range(s0.g, s0.dense_n, k.threads, k.groups, rank);
  if (s1.g && !s1.box) zero_range(s1.g, s1.dense_n, k.threads, k.groups, rank);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// Sum over the four lanes of a quad (DPP quad permutations, no LDS traffic).
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  return v;
}

// Sum over the two lanes of a pair.
__device__ __forceinline__ float pair_sum(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
}

// Completes a gather split over the lanes of a particle (S0 as in for_nodes).
template <int S0>
__device__ __forceinline__ float lanes_sum(float v) {
  if constexpr (S0 == 1) return quad_sum(v);
  if constexpr (S0 == 2) return pair_sum(v);
  return v;
}

template <int S0, int N>
__device__ __forceinline__ void quad_reduce(float (&v)[N]) {
  if constexpr (S0 != 3) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = lanes_sum<S0>(v[q]);
  }
}

template <int S0, int N, int M>
__device__ __forceinline__ void quad_reduce(float (&v)[N][M]) {
  if constexpr (S0 != 3) {
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
      for (int r = 0; r < M; ++r) v[q][r] = lanes_sum<S0>(v[q][r]);
  }
}

// v * 2^e rounded to the nearest integer, as a 64-bit value. The scale is
// chosen (fixed_exponent) so that |v| 2^e < 2^31 for every contribution, so
// rounding and conversion are two single-precision instructions and the high
// word is the sign extension; node sums of up to 2^32 contributions cannot
// overflow 64 bits.
__device__ __forceinline__ long long to_fixed(float v, int e) { return (long long)int(rintf(ldexpf(v, e))); }

__device__ __forceinline__ float from_fixed(long long q, int e) {
  const double hi = double(int(q >> 32)) * 4294967296.0;
  const double lo = double(unsigned(q & 0xFFFFFFFFll));
  return float(ldexp(hi + lo, -e));
}

// Quad mode: lane `sub` (0..2) of a particle's quad keeps visited node `sub`
// of axis 0 as its slab; lane 3 keeps a zero-weight slab (it only takes part
// in the quad reductions).
template <int D>
__device__ __forceinline__ void slab_select(Sten<D>& st, int sub) {
  const bool act = sub < 3;
  float N = st.N[0][0], dN = st.dN[0][0], dl = st.dl[0][0];
  int nc = st.nc[0][0];
  if (sub == 1) {
    N = st.N[0][1];
    dN = st.dN[0][1];
    dl = st.dl[0][1];
    nc = st.nc[0][1];
  } else if (sub == 2) {
    N = st.N[0][2];
    dN = st.dN[0][2];
    dl = st.dl[0][2];
    nc = st.nc[0][2];
  }
  st.N[0][0] = act ? N : 0.0f;
  st.dN[0][0] = act ? dN : 0.0f;
  st.dl[0][0] = dl;
  st.nc[0][0] = nc;
}

// ---------------------------------------------------------------------------
// LDS tiles
// ---------------------------------------------------------------------------
template <int D>
struct Tile {
  int lo[D];
  int ext[D];
  float rcp[D];  // 1 / ext, rounded up by ~2^-20 (division-free coordinates, tile_coord)
  int n;
  bool on;
  int e;  // fixed-point exponent of a scatter tile
};


// Node addressing: a box of the scene's grid staged in LDS (L = true), or the
// scene's global grid. LDS tiles are structure-of-arrays, component c of tile
// node q at tile[c * kTileCap<D> + q], so lanes touching neighbouring nodes hit
// consecutive banks; the global grid is one float4 per node.
template <int D, bool L>
struct Nodes {
  float* p;
  int lo[D], ext[D];
  int n;
  __device__ __forceinline__ int idx(const Sten<D>& st, int o0, int o1, int o2) const {
    if constexpr (L) {
      if constexpr (D == 2) {
        return (st.nc[0][o0] - lo[0]) * ext[1] + (st.nc[1][o1] - lo[1]);
      } else {
        return ((st.nc[0][o0] - lo[0]) * ext[1] + (st.nc[1][o1] - lo[1])) * ext[2] + (st.nc[2][o2] - lo[2]);
      }
    } else {
      return node_of<D>(st, o0, o1, o2, n);
    }
  }
  // First NC components of a node (the rest are zero).
  template <int NC = 4>
  __device__ __forceinline__ float4 get(const Sten<D>& st, int o0, int o1, int o2) const {
    const int q = idx(st, o0, o1, o2);
    if constexpr (L) {
      float4 v = make_float4(p[q], 0.f, 0.f, 0.f);
      if (NC > 1) v.y = p[kTileCap<D> + q];
      if (NC > 2) v.z = p[2 * kTileCap<D> + q];
      if (NC > 3) v.w = p[3 * kTileCap<D> + q];
      return v;
    } else {
      return reinterpret_cast<const float4*>(p)[q];
    }
  }
  __device__ __forceinline__ void add(int q, int c, float v) const {
    if constexpr (L)
      atomic_add_f32(p + c * kTileCap<D> + q, v);
    else
      atomic_add_f32(p + 4 * q + c, v);
  }
};

template <int D>
__device__ __forceinline__ Nodes<D, true> lds_nodes(float* tile, const Tile<D>& T) {
  Nodes<D, true> a;
  a.p = tile;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    a.lo[q] = T.lo[q];
    a.ext[q] = T.ext[q];
  }
  a.n = 0;
  return a;
}

template <int D>
__device__ __forceinline__ Nodes<D, false> global_nodes(const float4* g, int n) {
  Nodes<D, false> a;
  a.p = reinterpret_cast<float*>(const_cast<float4*>(g));
#pragma unroll
  for (int q = 0; q < D; ++q) {
    a.lo[q] = 0;
    a.ext[q] = 0;
  }
  a.n = n;
  return a;
}

// Lanes of a wave whose particles share a stencil base (particles sorted by
// base run consecutively) add to the same nodes in the same instruction when
// every lane visits its stencil in the same order. RunSum sums a value over
// this lane's run (the adjacent lanes holding its key) within its aligned
// group of eight lanes (three shifted adds, DPP row_shl by 1, 2, 4; a lane
// adds the shifted value only when every lane up to the one it comes from
// holds its key and its group), leaving the run's sum in the run's first lane
// (head), so one atomic per run replaces one per lane. The order of the
// additions is fixed, so results do not depend on scheduling.
template <int K>
__device__ __forceinline__ float dpp_from_above(float v) {  // lane l gets lane l + K of its row of 16
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + K, 0xF, 0xF, true));
}
template <int K>
__device__ __forceinline__ int dpp_from_above_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x100 + K, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_below_i(int v) {  // lane l gets lane l - 1 of its row of 16
  return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);
}

struct RunSum {
  bool m1, m2, m4;  // lane + k holds the same key in the same group of eight
  bool head;
  __device__ __forceinline__ float operator()(float v) const {
    // Selects, not products: a lane outside the run may hold anything.
    const float a1 = dpp_from_above<1>(v);
    v += m1 ? a1 : 0.0f;
    const float a2 = dpp_from_above<2>(v);
    v += m2 ? a2 : 0.0f;
    const float a4 = dpp_from_above<4>(v);
    v += m4 ? a4 : 0.0f;
    return v;
  }
};

// Run of this lane: `key` identifies its stencil base (valid lanes only);
// all lanes of the wave call.
__device__ __forceinline__ RunSum run_sum(bool valid, int key) {
  RunSum r;
  const int lane = int(threadIdx.x & 63);
  const int kk = valid ? key : -1 - lane;  // an invalid lane forms a run of its own
  const int g = lane & 7;
  // Every lane reads its neighbours' keys before any condition: a cross-lane
  // read from a lane that a branch has switched off returns 0, not its key.
  const int n1 = dpp_from_above_i<1>(kk);
  const int n2 = dpp_from_above_i<2>(kk);
  const int n3 = dpp_from_above_i<3>(kk);
  const int n4 = dpp_from_above_i<4>(kk);
  const int p1 = dpp_from_below_i(kk);
  // A run is contiguous: particles sorted once by base move, so equal keys
  // need not be adjacent later; lane + k joins only if every lane between
  // holds the key too.
  const bool e1 = n1 == kk, e2 = e1 & (n2 == kk), e4 = e2 & (n3 == kk) & (n4 == kk);
  r.m1 = (g + 1 < 8) & e1;
  r.m2 = (g + 2 < 8) & e2;
  r.m4 = (g + 4 < 8) & e4;
  r.head = (g == 0) | (p1 != kk);
  return r;
}

// Linear index of a stencil's base node in its scene's grid (the run key).
template <int D>
__device__ __forceinline__ int base_key(const Sten<D>& st, int n) {
  if constexpr (D == 2)
    return st.base[0] * n + st.base[1];
  else
    return (st.base[0] * n + st.base[1]) * n + st.base[2];
}

// Scatter target: a box of the scene's grid in LDS, 64-bit fixed point with
// scale 2^e, component c of tile node q at tile[c * kTileCap<D> + q].
template <int D>
struct FixNodes {
  long long* p;
  int lo[D], ext[D];
  int e;
  __device__ __forceinline__ int idx(const Sten<D>& st, int o0, int o1, int o2) const {
    if constexpr (D == 2) {
      return (st.nc[0][o0] - lo[0]) * ext[1] + (st.nc[1][o1] - lo[1]);
    } else {
      return ((st.nc[0][o0] - lo[0]) * ext[1] + (st.nc[1][o1] - lo[1])) * ext[2] + (st.nc[2][o2] - lo[2]);
    }
  }
  __device__ __forceinline__ void add(int q, int c, float v) const {
    atomicAdd(reinterpret_cast<unsigned long long*>(p + c * kTileCap<D> + q), (unsigned long long)to_fixed(v, e));
  }
};

template <int D>
__device__ __forceinline__ FixNodes<D> fix_nodes(long long* tile, const Tile<D>& T) {
  FixNodes<D> a;
  a.p = tile;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    a.lo[q] = T.lo[q];
    a.ext[q] = T.ext[q];
  }
  a.e = T.e;
  return a;
}

// Stencil visiting colour of this lane (see Sten): lane mod 3^d, or -1.
template <int D, int LPP>
__device__ __forceinline__ int lane_color(const StepConsts& k) {
  return k.rotate ? (int(threadIdx.x & 63) / LPP) % (D == 3 ? 27 : 9) : -1;
}

// Stencil of the particle at x for this lane (quad mode: the lane's slab).
template <int D, int LPP>
__device__ __forceinline__ bool lane_sten(const StepConsts& k, const float (&x)[D], int sub, Sten<D>& st) {
  const bool ok = make_sten<D>(x, k.inv_dx, k.dx, k.n, lane_color<D, LPP>(k), st, LPP == 2 && sub == 1);
  if constexpr (LPP == 4) slab_select<D>(st, sub);
  return ok;
}

// Particle (within its workgroup) handled by thread t. Particles are sorted by
// stencil base, so runs of consecutive particles share all their stencil
// nodes, and lanes of one wave adding to the same LDS node in the same
// instruction serialise. With remap, the B particles of the workgroup are read
// as a (B/8) x 8 matrix of consecutive groups of 8 and thread t takes row
// t % (B/8), column t / (B/8): a wave then holds at most 64 / (B/8) particles
// of any group of 8.
__device__ __forceinline__ int lane_particle(int t, int B, int remap) {
  if (!remap || (B & 7)) return t;
  const int rows = B >> 3;
  return (t % rows) * 8 + t / rows;
}

// Fixed-point exponent for contributions bounded by `bmax`: the largest e
// with bmax 2^e < 2^31, so each contribution is rounded to a multiple of
// 2^-e <= bmax 2^-30 (an error below bmax 2^-31, finer than the 2^-24
// relative rounding of an FP32 partial sum of such contributions); INT_MIN
// when the bound is not finite.
__device__ __forceinline__ int fixed_exponent(float bmax) {
  if (!(bmax < 3.0e38f)) return INT_MIN;
  if (bmax <= 0.0f) return 0;
  return 30 - ilogbf(bmax);
}

// Block-wide reductions with one barrier each: every wave writes its partial
// to its own slots in one of two alternating slot sets (2 x 4 waves x 8 ints),
// and a set is written again only after a later reduction's barrier, which
// every thread reaches after reading it.
struct BlockRed {
  int* sh;
  int phase;
  int nw;  // waves per workgroup
};

template <int D>
struct Box {
  int mn[D], mx[D];
  float bmax;
};

// Wavefront min / max of an int with DPP row shifts and row broadcasts (one
// VALU instruction per step instead of a cross-lane LDS permute): after the
// four shifts lane 15 of each row of 16 holds its row's result, the two
// broadcasts carry it to lane 63, which is read back uniformly. Lanes whose
// DPP source lies outside the row read the identity.
template <bool MAX>
__device__ __forceinline__ int wave_extreme(int v) {
  constexpr int id = MAX ? INT_MIN : INT_MAX;
  auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xF, 0xF, false));  // row_shr:1
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xF, 0xF, false));  // row_shr:2
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xF, 0xF, false));  // row_shr:4
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xF, 0xF, false));  // row_shr:8
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Min/max of the stencil bases of the valid lanes and max of `bound` (a
// non-negative contribution bound; NaN counts as +inf). All threads call.
template <int D>
__device__ Box<D> block_reduce(bool valid, const int (&base)[D], float bound, BlockRed& r) {
  int mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    mn[a] = valid ? base[a] : INT_MAX;
    mx[a] = valid ? base[a] : INT_MIN;
  }
  const float bb = (bound == bound) ? fmaxf(bound, 0.0f) : __int_as_float(0x7f800000);
  int b = __float_as_int(bb);  // non-negative floats order as ints
#pragma unroll
  for (int a = 0; a < D; ++a) {
    mn[a] = wave_extreme<false>(mn[a]);
    mx[a] = wave_extreme<true>(mx[a]);
  }
  b = wave_extreme<true>(b);
  int* s = r.sh + (r.phase & 1) * 32;
  const int w = int(threadIdx.x >> 6), nw = r.nw;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      s[w * 8 + a] = mn[a];
      s[w * 8 + D + a] = mx[a];
    }
    s[w * 8 + 2 * D] = b;
  }
  __syncthreads();
  Box<D> out;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    out.mn[a] = INT_MAX;
    out.mx[a] = INT_MIN;
  }
  int bm = 0;
  for (int q = 0; q < nw; ++q) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      out.mn[a] = min(out.mn[a], s[q * 8 + a]);
      out.mx[a] = max(out.mx[a], s[q * 8 + D + a]);
    }
    bm = max(bm, s[q * 8 + 2 * D]);
  }
  out.bmax = __int_as_float(bm);
  ++r.phase;
  return out;
}

template <int D>
__device__ __forceinline__ Tile<D> empty_tile() {
  Tile<D> T;
  T.on = false;
  T.n = 0;
  T.e = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T.lo[a] = 0;
    T.ext[a] = 0;
    T.rcp[a] = 0.0f;
  }
  return T;
}

template <int D>
__device__ __forceinline__ void tile_set_box(Tile<D>& T, const int (&lo)[D], const int (&ext)[D]) {
  int n = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T.lo[a] = lo[a];
    T.ext[a] = ext[a];
    T.rcp[a] = ext[a] > 0 ? (1.0f / float(ext[a])) * (1.0f + 0x1p-20f) : 0.0f;
    n *= ext[a];
  }
  T.n = ext[0] > 0 ? n : 0;
}

// Box of the stencils of the workgroup's valid lanes (bases lo .. lo + ext - 3).
template <int D>
__device__ __forceinline__ Tile<D> tile_of(const Box<D>& bx, bool one_scene) {
  Tile<D> T = empty_tile<D>();
  if (bx.mn[0] > bx.mx[0]) return T;  // no valid lane
  int lo[D], ext[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = bx.mn[a];
    ext[a] = bx.mx[a] - bx.mn[a] + 3;
  }
  tile_set_box<D>(T, lo, ext);
  T.on = one_scene && T.n <= kTileCap<D>;
  return T;
}

template <int D>
__device__ __forceinline__ Tile<D> block_tile(bool valid, const int (&base)[D], bool one_scene, int enabled,
                                              BlockRed& r) {
  if (!enabled) return empty_tile<D>();
  return tile_of<D>(block_reduce<D>(valid, base, 0.0f, r), one_scene);
}

// Box and fixed-point exponent of a scatter tile in one reduction.
template <int D>
__device__ __forceinline__ Tile<D> block_tile_scaled(bool valid, const int (&base)[D], float bound, bool one_scene,
                                                     int enabled, BlockRed& r) {
  if (!enabled) return empty_tile<D>();
  const Box<D> bx = block_reduce<D>(valid, base, bound, r);
  Tile<D> T = tile_of<D>(bx, one_scene);
  T.e = fixed_exponent(bx.bmax);
  T.on = T.on && T.e != INT_MIN;
  return T;
}

// The box a gather needs, as recorded by the scatter into the same grid one
// launch earlier (same workgroup, same particle positions). Used only when it
// lies inside the grid and belongs to this workgroup's scene.
template <int D, bool P>
__device__ __forceinline__ Tile<D> recorded_tile(const int4* table, int wg, int sc, bool one_scene, int enabled,
                                                 int n) {
  Tile<D> T = empty_tile<D>();
  if (!enabled) return T;
  const int4 l4 = load_box<P>(table + 2 * wg), e4 = load_box<P>(table + 2 * wg + 1);
  const int lo3[3] = {l4.x, l4.y, l4.z}, ex3[3] = {e4.x, e4.y, e4.z};
  int lo[D], ext[D];
  bool inside = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = lo3[a];
    ext[a] = ex3[a];
    inside = inside && lo[a] >= 0 && ext[a] >= 3 && ext[a] <= n && lo[a] <= n - ext[a];
  }
  if (!inside) return T;
  tile_set_box<D>(T, lo, ext);
  T.on = one_scene && l4.w == sc && T.n <= kTileCap<D>;
  return T;
}

// True when the stencil (base .. base + 2) lies in the tile's box.
template <int D>
__device__ __forceinline__ bool in_tile(const Tile<D>& T, const int (&base)[D]) {
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) in = in && base[a] >= T.lo[a] && base[a] + 3 <= T.lo[a] + T.ext[a];
  return in;
}

// Records the box of a scatter's nodes for workgroup `index` (thread 0).
template <int D>
__device__ __forceinline__ void record_box(int4* table, int index, const Tile<D>& T, int scene) {
  if (!table || threadIdx.x != 0) return;
  const bool any = T.n > 0;
  int lo2 = 0, ext2 = 1;  // 2D: a one-node third axis
  if constexpr (D == 3) {
    lo2 = T.lo[2];
    ext2 = any ? T.ext[2] : 0;
  }
  table[2 * index] = make_int4(T.lo[0], T.lo[1], lo2, scene);
  table[2 * index + 1] = make_int4(any ? T.ext[0] : 0, any ? T.ext[1] : 0, ext2, 0);
}

// Records the union of a tile's box and the stencil-base box `bx` (empty when
// bx.mn > bx.mx) for workgroup `index`.
template <int D>
__device__ __forceinline__ void record_box_union(int4* table, int index, const Tile<D>& T, const Box<D>& bx,
                                                 int scene) {
  if (!table) return;
  Tile<D> U = T;
  if (bx.mn[0] <= bx.mx[0]) {
    int lo[D], ext[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int l = (T.n > 0) ? min(T.lo[a], bx.mn[a]) : bx.mn[a];
      const int h = (T.n > 0) ? max(T.lo[a] + T.ext[a], bx.mx[a] + 3) : bx.mx[a] + 3;
      lo[a] = l;
      ext[a] = h - l;
    }
    tile_set_box<D>(U, lo, ext);
  }
  record_box<D>(table, index, U, scene);
}

template <int D>
__device__ __forceinline__ int tile_global_index(const Tile<D>& T, int q, int n) {
  int c[D];
  int r = q;
#pragma unroll
  for (int a = D - 1; a > 0; --a) {
    int m;
    r = div_small(r, T.ext[a], T.rcp[a], m);
    c[a] = T.lo[a] + m;
  }
  c[0] = T.lo[0] + r;
  int g = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) g = g * n + c[a];
  return g;
}

// Scene-grid coordinates of tile node q; returns its linear index.
template <int D>
__device__ __forceinline__ int tile_node(const Tile<D>& T, int q, int n, int (&c)[D]) {
  int r = q;
#pragma unroll
  for (int a = D - 1; a > 0; --a) {
    int m;
    r = div_small(r, T.ext[a], T.rcp[a], m);
    c[a] = T.lo[a] + m;
  }
  c[0] = T.lo[0] + r;
  int g = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) g = g * n + c[a];
  return g;
}

template <int D>
__device__ __forceinline__ bool tile_node_interior(const int (&c)[D], int n, int bound) {
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) in = in && interior1(c[a], n, bound);
  return in;
}

// Adds the non-zero entries of a fixed-point tile into the global grid. Lanes
// run over (node, component) pairs, component fastest, so one atomic
// instruction covers a few runs of consecutive nodes in a handful of cache
// lines. With one node per lane and one instruction per component, each
// instruction spread over a dozen or more lines, and the flush atomics of all
// workgroups (which overlap at box borders) went on draining for several
// microseconds after the last workgroup had ended.
template <int D, int NC>
__device__ __forceinline__ void tile_flush64(const Tile<D>& T, const long long* tile, float4* g, int n,
                                             int threads) {
  // Four entries per thread per pass: their LDS reads are issued together.
  const int total = NC * T.n;
  for (int j0 = threadIdx.x; j0 < total; j0 += 4 * threads) {
    long long v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * threads;
      const int q = j / NC;
      v[u] = j < total ? tile[(j - q * NC) * kTileCap<D> + q] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * threads;
      const int q = j / NC;
      if (v[u] != 0)
        atomic_add_f32(reinterpret_cast<float*>(g + tile_global_index<D>(T, q, n)) + (j - q * NC), from_fixed(v[u], T.e));
    }
  }
}

// Bound on the size of any scatter contribution w * (m v_c + (A delta)_c) or
// w * m of a particle (|delta_b| <= 1.5 dx, w <= 1).
template <int D>
__device__ __forceinline__ float p2g_bound(float mass, const float (&mv)[D], const float (&A)[D][D], float dx) {
  float b = mass;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    float s = fabsf(mv[c]);
#pragma unroll
    for (int e = 0; e < D; ++e) s += 1.5f * dx * fabsf(A[c][e]);
    b = fmaxf(b, s);
  }
  return b;
}

// ---------------------------------------------------------------------------
// Stage bodies (one particle)
// ---------------------------------------------------------------------------

// Node velocity after the grid update, from (m, P).
// grid_op at one node: v = P / m + dt g (gravity on axis 1) at active nodes,
// zero elsewhere (empty nodes and the sticky boundary band).
template <int D>
__device__ __forceinline__ void grid_vel(bool act, float4 g, float gdt, float (&v)[D]) {
  const float P[3] = {g.y, g.z, g.w};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float va = P[a] / g.x + (a == 1 ? gdt : 0.0f);
    v[a] = act ? va : 0.0f;
  }
}

template <int D>
__device__ __forceinline__ void node_velocity(const StepConsts& k, const Sten<D>& st, int o0, int o1, int o2,
                                              float4 g, float (&v)[D]) {
  grid_vel<D>(node_active<D>(st, o0, o1, o2, k.n, k.bound, g.x), g, k.gdt, v);
}

// Grid velocity of a visited node: read from a velocity tile (L), or computed
// from the node's (m, P) in the global grid.
template <int D, bool L>
__device__ __forceinline__ void node_vel(const StepConsts& k, const Sten<D>& st, int o0, int o1, int o2,
                                         const Nodes<D, L>& g, float (&v)[D]) {
  if constexpr (L) {
    const float4 t = g.template get<D>(st, o0, o1, o2);
    v[0] = t.x;
    v[1] = t.y;
    if constexpr (D == 3) v[2] = t.z;
  } else {
    node_velocity<D>(k, st, o0, o1, o2, g.template get<D + 1>(st, o0, o1, o2), v);
  }
}

// g2p: gather v' and C' and update the particle (v, C, x, F).
template <int D, bool L, int S0>
__device__ __forceinline__ void g2p_body(const StepConsts& k, const Sten<D>& st, const Nodes<D, L>& g, PState<D>& p) {
  float vn[D] = {}, Cn[D][D] = {};
  for_nodes<D, S0>(st, [&](int o0, int o1, int o2) {
    const float w = wgt<D>(st, o0, o1, o2);
    float dl[D], v[D];
    delta<D>(st, o0, o1, o2, k.dx, dl);
    node_vel<D>(k, st, o0, o1, o2, g, v);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      vn[c] += w * v[c];
#pragma unroll
      for (int b = 0; b < D; ++b) Cn[c][b] += w * v[c] * dl[b];
    }
  });
  quad_reduce<S0>(vn);
  quad_reduce<S0>(Cn);
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) Cn[c][b] *= k.kappa;
  float Fn[D][D];
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
}

// An affine field over the stencil, a_c + sum_b M_cb (x_i - x_p)_b, kept as
// per-axis terms: t[b][c][o] = M_cb dl_b[o] (+ a_c on axis 0), so a visited
// node costs D - 1 adds per component instead of D multiply-adds (the terms
// of the outer axes are shared by the inner loop's nodes).
template <int D>
struct AffineTab {
  float t[D][D][3];
  __device__ __forceinline__ AffineTab(const Sten<D>& st, const float (&a)[D], const float (&M)[D][D]) {
#pragma unroll
    for (int b = 0; b < D; ++b)
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int o = 0; o < 3; ++o) t[b][c][o] = (b == 0) ? fmaf(M[c][b], st.dl[b][o], a[c]) : M[c][b] * st.dl[b][o];
  }
  __device__ __forceinline__ float at(int c, int o0, int o1, int o2) const {
    float v = t[0][c][o0] + t[1][c][o1];
    if constexpr (D == 3) v += t[2][c][o2];
    return v;
  }
};

// p2g: scatter m and P of one particle (A and m v precomputed). With an
// active RunSum (LDS tiles, base-sorted particles, every lane in the same
// stencil order), lanes of a run sum their contributions and the run's head
// adds them.
template <int D, int S0, bool PRE = false, class SA>
__device__ __forceinline__ void p2g_body(const StepConsts& k, const Sten<D>& st, float mass, const float (&mv)[D],
                                         const float (&A)[D][D], const SA& g, const RunSum& rs = RunSum{}) {
  const AffineTab<D> mom(st, mv, A);  // m v + A (x_i - x_p)
  for_nodes<D, S0>(st, [&](int o0, int o1, int o2) {
    const float w = wgt<D>(st, o0, o1, o2);
    const int q = g.idx(st, o0, o1, o2);
    if constexpr (PRE) {
      float val[D + 1];
      val[0] = rs(w * mass);
#pragma unroll
      for (int a = 0; a < D; ++a) val[1 + a] = rs(w * mom.at(a, o0, o1, o2));
      if (rs.head) {
#pragma unroll
        for (int c = 0; c < D + 1; ++c) g.add(q, c, val[c]);
      }
    } else {
      g.add(q, 0, w * mass);
#pragma unroll
      for (int a = 0; a < D; ++a) g.add(q, 1 + a, w * mom.at(a, o0, o1, o2));
    }
  });
}

// grid_op* at one node: from the node's (m, P) and the adjoint v* of its
// velocity, P* = v* / m and m* = -(v* . P) / m^2 (both zero at inactive nodes).
template <int D>
__device__ __forceinline__ void grid_adj(bool act, float4 gm, float4 vb4, float (&Pb)[D], float& mb) {
  const float inv_m = act ? 1.0f / gm.x : 0.0f;
  const float P[3] = {gm.y, gm.z, gm.w};
  const float V[3] = {vb4.x, vb4.y, vb4.z};
  float vP = 0.0f;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    Pb[c] = V[c] * inv_m;
    vP += V[c] * P[c];
  }
  mb = -vP * inv_m * inv_m;
}

// P* and m* of a visited node: read from an adjoint tile (L: P* in components
// 0..D-1, m* in component D; `ad` unused), or computed from the global grid
// and adjoint grid.
template <int D, bool L>
__device__ __forceinline__ void node_adj(const StepConsts& k, const Sten<D>& st, int o0, int o1, int o2,
                                         const Nodes<D, L>& g, const Nodes<D, L>& ad, float (&Pb)[D], float& mb) {
  if constexpr (L) {
    const float4 t = g.template get<D + 1>(st, o0, o1, o2);
    Pb[0] = t.x;
    Pb[1] = t.y;
    if constexpr (D == 3) {
      Pb[2] = t.z;
      mb = t.w;
    } else {
      mb = t.z;
    }
  } else {
    const float4 gm = g.template get<D + 1>(st, o0, o1, o2);
    const float4 vb4 = ad.template get<D>(st, o0, o1, o2);
    grid_adj<D>(node_active<D>(st, o0, o1, o2, k.n, k.bound, gm.x), gm, vb4, Pb, mb);
  }
}

// The first NC components of a grid node (the rest zero), read with a load of
// exactly NC floats. A float4 load whose unused components' registers the
// compiler hands to other values while the load is in flight must be waited
// for in full before those registers are written, and the in-order counter
// makes that wait cover every load issued before it.
template <int NC>
__device__ __forceinline__ float4 load_node(const float4* p) {
  if constexpr (NC == 4) {
    return *p;
  } else if constexpr (NC == 3) {
    const float3 t = *reinterpret_cast<const float3*>(p);
    return make_float4(t.x, t.y, t.z, 0.0f);
  } else {
    const float2 t = *reinterpret_cast<const float2*>(p);
    return make_float4(t.x, t.y, 0.0f, 0.0f);
  }
}

// Tile loads issue up to kTileBatch node loads per thread before using any,
// so their latencies overlap (a full 3D tile of kTileCap<3> nodes takes one
// round trip at 256 threads per workgroup). The step kernels read the first
// nodes straight-line (tile_first_issue) and use these loops for the rest.
constexpr int kTileBatch = 4;

// Velocity tile: grid_op applied once per node of the box as it is staged
// (components 0..D-1 = v), so gathers read v instead of forming P / m per visit.
template <int D>
__device__ __forceinline__ void tile_load_vel(const StepConsts& k, const Tile<D>& T, const float4* g, float* tile,
                                              int first = 0) {
  for (int q0 = first + threadIdx.x; q0 < T.n; q0 += kTileBatch * k.threads) {
    float4 gm[kTileBatch];
#pragma unroll
    for (int r = 0; r < kTileBatch; ++r) {
      const int q = q0 + r * k.threads;
      int c[D];
      if (q < T.n) gm[r] = load_node<D + 1>(g + tile_node<D>(T, q, k.n, c));
    }
#pragma unroll
    for (int r = 0; r < kTileBatch; ++r) {
      const int q = q0 + r * k.threads;
      if (q < T.n) {
        int c[D];
        tile_node<D>(T, q, k.n, c);
        float v[D];
        grid_vel<D>(tile_node_interior<D>(c, k.n, k.bound) && gm[r].x > 0.0f, gm[r], k.gdt, v);
#pragma unroll
        for (int a = 0; a < D; ++a) tile[a * kTileCap<D> + q] = v[a];
      }
    }
  }
}

// Adjoint tile: grid_op* applied once per node of the box (components 0..D-1
// = P*, component D = m*), from the grid (m, P) and the adjoint grid (v*).
template <int D>
__device__ __forceinline__ void tile_load_adj(const StepConsts& k, const Tile<D>& T, const float4* g,
                                              const float4* ad, float* tile, int first = 0) {
  for (int q0 = first + threadIdx.x; q0 < T.n; q0 += kTileBatch * k.threads) {
    float4 gm[kTileBatch], vb4[kTileBatch];
#pragma unroll
    for (int r = 0; r < kTileBatch; ++r) {
      const int q = q0 + r * k.threads;
      int c[D];
      if (q < T.n) {
        const int gi = tile_node<D>(T, q, k.n, c);
        gm[r] = load_node<D + 1>(g + gi);
        vb4[r] = load_node<D>(ad + gi);
      }
    }
#pragma unroll
    for (int r = 0; r < kTileBatch; ++r) {
      const int q = q0 + r * k.threads;
      if (q < T.n) {
        int c[D];
        tile_node<D>(T, q, k.n, c);
        float Pb[D], mb;
        grid_adj<D>(tile_node_interior<D>(c, k.n, k.bound) && gm[r].x > 0.0f, gm[r], vb4[r], Pb, mb);
#pragma unroll
        for (int a = 0; a < D; ++a) tile[a * kTileCap<D> + q] = Pb[a];
        tile[D * kTileCap<D> + q] = mb;
      }
    }
  }
}

// First node of each thread of a gather tile, read outside any loop. Behind a
// loop the compiler waits for most loads issued before the loop (its
// counter-based waits are conservative at loop headers), so a tile load in a
// loop only starts once the particle loads issued before it have landed; read
// straight-line, the tile's round trip overlaps theirs. Boxes of more nodes
// than threads read the rest with tile_load_vel / tile_load_adj from
// `k.threads` on.
template <int D>
struct TileFirst {
  bool on;
  int c[D];
  float4 g, v;
};

template <int D>
__device__ __forceinline__ TileFirst<D> tile_first_issue(const StepConsts& k, const Tile<D>& T, const float4* g,
                                                         const float4* ad) {
  TileFirst<D> f;
  const int q = threadIdx.x;
  f.on = T.on && q < T.n;
  f.g = make_float4(0.f, 0.f, 0.f, 0.f);
  f.v = f.g;
  if (f.on) {
    const int gi = tile_node<D>(T, q, k.n, f.c);
    f.g = load_node<D + 1>(g + gi);
    if (ad) f.v = load_node<D>(ad + gi);
  }
  return f;
}

// Velocity tile entry of tile_first_issue (grid_op applied).
template <int D>
__device__ __forceinline__ void tile_first_vel(const StepConsts& k, const TileFirst<D>& f, float* tile) {
  if (!f.on) return;
  float v[D];
  grid_vel<D>(tile_node_interior<D>(f.c, k.n, k.bound) && f.g.x > 0.0f, f.g, k.gdt, v);
#pragma unroll
  for (int a = 0; a < D; ++a) tile[a * kTileCap<D> + threadIdx.x] = v[a];
}

// Adjoint tile entry of tile_first_issue (grid_op* applied).
template <int D>
__device__ __forceinline__ void tile_first_adj(const StepConsts& k, const TileFirst<D>& f, float* tile) {
  if (!f.on) return;
  float Pb[D], mb;
  grid_adj<D>(tile_node_interior<D>(f.c, k.n, k.bound) && f.g.x > 0.0f, f.g, f.v, Pb, mb);
#pragma unroll
  for (int a = 0; a < D; ++a) tile[a * kTileCap<D> + threadIdx.x] = Pb[a];
  tile[D * kTileCap<D> + threadIdx.x] = mb;
}

// p2g* with grid_op* folded in: accumulates into gx, gv, Abar from grid (m, P)
// and adjoint grid (v*).
template <int D, bool L, int S0>
__device__ __forceinline__ void p2g_adj_body(const StepConsts& k, const Sten<D>& st, float mass, const float (&mv)[D],
                                             const float (&A)[D][D], const Nodes<D, L>& g, const Nodes<D, L>& ad,
                                             float (&gx)[D], float (&vb)[D], float (&Abar)[D][D]) {
  // d/dx_p of sum_i P*_i . (m v + A (x_i - x_p)) w_ip: the weight-gradient
  // term per node, and -A^T sum_i w_ip P*_i once (the sum is wP, also the
  // velocity adjoint).
  float gxa[D] = {}, wP[D] = {};
  const AffineTab<D> mom(st, mv, A);  // m v + A (x_i - x_p)
  for_nodes<D, S0>(st, [&](int o0, int o1, int o2) {
    float Pb[D], mb;
    node_adj<D>(k, st, o0, o1, o2, g, ad, Pb, mb);
    const float w = wgt<D>(st, o0, o1, o2);
    float dw[D], dl[D];
    dwgt<D>(st, o0, o1, o2, k.inv_dx, dw);
    delta<D>(st, o0, o1, o2, k.dx, dl);
    float contrib = mass * mb;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      contrib += Pb[c] * mom.at(c, o0, o1, o2);
      wP[c] += w * Pb[c];
#pragma unroll
      for (int b = 0; b < D; ++b) Abar[c][b] += w * Pb[c] * dl[b];
    }
#pragma unroll
    for (int e = 0; e < D; ++e) gxa[e] += contrib * dw[e];
  });
#pragma unroll
  for (int e = 0; e < D; ++e) {
#pragma unroll
    for (int c = 0; c < D; ++c) gxa[e] -= A[c][e] * wP[c];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) vb[c] += wP[c];
  quad_reduce<S0>(gxa);
  quad_reduce<S0>(vb);
  quad_reduce<S0>(Abar);
#pragma unroll
  for (int e = 0; e < D; ++e) gx[e] += gxa[e];
}

// C' of a particle recomputed from grid s.
template <int D, bool L, int S0>
__device__ __forceinline__ void g2p_C(const StepConsts& k, const Sten<D>& st, const Nodes<D, L>& g, float (&Cn)[D][D]) {
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) Cn[c][b] = 0.0f;
  for_nodes<D, S0>(st, [&](int o0, int o1, int o2) {
    const float w = wgt<D>(st, o0, o1, o2);
    float dl[D], v[D];
    delta<D>(st, o0, o1, o2, k.dx, dl);
    node_vel<D>(k, st, o0, o1, o2, g, v);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) Cn[c][b] += w * v[c] * dl[b];
  });
  quad_reduce<S0>(Cn);
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) Cn[c][b] *= k.kappa;
}

// g2p*: scatter v* into the adjoint grid; accumulate x* (px).
template <int D, int S0, bool PRE = false, class GA, class SA>
__device__ __forceinline__ void g2p_adj_body(const StepConsts& k, const Sten<D>& st, const float (&vt)[D],
                                             const float (&Bm)[D][D], const GA& g, const SA& ad, float (&px)[D],
                                             bool scatter, const RunSum& rs = RunSum{}) {
  // d/dx_p of sum_i v_i . (v~ + B (x_i - x_p)) w_ip: the weight-gradient term
  // per node, and -B^T sum_i w_ip v_i once (that sum is wv).
  float pxa[D] = {}, wv[D] = {};
  const AffineTab<D> rt(st, vt, Bm);  // r = v~ + B (x_i - x_p)
  for_nodes<D, S0>(st, [&](int o0, int o1, int o2) {
    float v[D];
    node_vel<D>(k, st, o0, o1, o2, g, v);
    const float w = wgt<D>(st, o0, o1, o2);
    float dw[D];
    dwgt<D>(st, o0, o1, o2, k.inv_dx, dw);
    float r[D], vr = 0.0f;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      r[c] = rt.at(c, o0, o1, o2);
      vr += v[c] * r[c];
      wv[c] += w * v[c];
    }
    if (scatter) {
      const int q = ad.idx(st, o0, o1, o2);
      if constexpr (PRE) {
        float val[D];
#pragma unroll
        for (int c = 0; c < D; ++c) val[c] = rs(w * r[c]);
        if (rs.head) {
#pragma unroll
          for (int c = 0; c < D; ++c) ad.add(q, c, val[c]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) ad.add(q, c, w * r[c]);
      }
    }
#pragma unroll
    for (int e = 0; e < D; ++e) pxa[e] += vr * dw[e];
  });
#pragma unroll
  for (int e = 0; e < D; ++e) {
#pragma unroll
    for (int c = 0; c < D; ++c) pxa[e] -= Bm[c][e] * wv[c];
  }
  quad_reduce<S0>(pxa);
#pragma unroll
  for (int e = 0; e < D; ++e) px[e] += pxa[e];
}

template <int D>
__device__ __forceinline__ int actuator_of(const StepConsts& k, const float* act_row, int i, float& act_tau) {
  act_tau = 0.0f;
  if (!act_row || !k.act_id) return -1;
  const int aid = k.act_id[i];
  if (aid >= 0) act_tau = k.act_strength * act_row[aid];
  return aid;
}

// Scatter of one state into `grid` with an optional LDS tile (all threads
// call). The fixed-point tile must already be zero over its first D + 1
// components (zero_tile64).
template <int D, int LPP, int M, bool PRE = false>
__device__ __forceinline__ void p2g_phase(const StepConsts& k, bool live, int i, int sc, bool one_scene, int sub,
                                          const PState<D>& p, const float* act_row, float4* grid,
                                          long long* tile, BlockRed& rd, unsigned& err, int4* box_out, int wg) {
  constexpr int S0 = (LPP == 4) ? 1 : (LPP == 2 ? 2 : 3);
  Sten<D> st;
  const bool fin = live && state_finite<D>(p);
  const bool ok = fin && lane_sten<D, LPP>(k, p.x, sub, st);
  if (live && !fin) err |= kErrNonfinite;
  if (fin && !ok) err |= kErrDomain;
  float A[D][D] = {}, mv[D] = {}, mass = 0.0f, bound = 0.0f;
  if (ok) {
    const SceneParams sp = scene_params(k.E, k.nu, k.vol, k.rho, sc);
    float act_tau;
    actuator_of<D>(k, act_row, i, act_tau);
    if (k.mat_id && k.mat_id[i] == 1) {
      float J;
      affine_liquid<D>(p, sp, act_tau, k.dt, k.kappa, A, J, err);
    } else if constexpr (M == 1) {
      float R[D][D], J;
      affine_corotated<D>(p, sp, act_tau, k.dt, k.kappa, A, R, J, err);
    } else {
      float FFtI[D][D], lnJ, J;
      affine<D>(p, sp, act_tau, k.dt, k.kappa, A, FFtI, lnJ, J, err);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) mv[a] = sp.mass * p.v[a];
    mass = sp.mass;
    bound = p2g_bound<D>(mass, mv, A, k.dx);
  }
  Tile<D> T = block_tile_scaled<D>(ok, st.base, bound, one_scene, k.lds, rd);
  record_box<D>(box_out, wg, T, one_scene ? sc : -1);
  // Runs of up to eight equal-base lanes add one sum: three more bits of headroom.
  const bool presum = PRE && LPP == 1 && T.on;
  if (presum) T.e -= 3;
  RunSum rs{};
  if (presum) rs = run_sum(ok, base_key<D>(st, k.n));
  if (k.tstats && threadIdx.x == 0 && T.n > 0) atomicAdd(k.tstats + (T.on ? 0 : 1), 1ull);
  float4* g = grid + long(sc) * k.nodes;
  if (ok && (LPP != 4 || sub < 3)) {
    if (PRE && presum)
      p2g_body<D, S0, true>(k, st, mass, mv, A, fix_nodes<D>(tile, T), rs);
    else if (T.on)
      p2g_body<D, S0>(k, st, mass, mv, A, fix_nodes<D>(tile, T));
    else
      p2g_body<D, S0>(k, st, mass, mv, A, global_nodes<D>(g, k.n));
  }
  if (T.on) {
    __syncthreads();
    tile_flush64<D, D + 1>(T, tile, g, k.n, k.threads);
  }
}

// Zeroes the first NC components of a whole fixed-point tile (no barrier: the
// next block reduction's barrier orders it before the scatter).
template <int D, int NC>
__device__ __forceinline__ void zero_tile64(long long* tile, int threads) {
  // 16-byte stores: two entries per store (the tiles are 16-byte aligned).
  int4* t = reinterpret_cast<int4*>(tile);
  for (int q = threadIdx.x; q < NC * kTileCap<D> / 2; q += threads) t[q] = make_int4(0, 0, 0, 0);
}

// Brings the launch's kernel arguments into the scalar cache in one round
// trip. The step kernels read their argument struct field by field where each
// branch needs it, and every read of a field not read before waits for memory:
// about a dozen dependent round trips before the reverse kernel issues its
// first global load. Here every whole 64-byte line of the struct is loaded at
// once (into a scratch register block, waited for inside the same statement),
// so those reads then hit the cache.
template <int BYTES>
__device__ __forceinline__ void warm_kernargs() {
  typedef int v16i __attribute__((ext_vector_type(16)));
  const unsigned long long base = reinterpret_cast<unsigned long long>(__builtin_amdgcn_kernarg_segment_ptr());
  v16i sink;
#define KA_LINE(off) "s_load_dwordx16 %0, %1, " #off "\n"
  if constexpr (BYTES / 64 >= 9) {
    asm volatile(KA_LINE(0x0) KA_LINE(0x40) KA_LINE(0x80) KA_LINE(0xc0) KA_LINE(0x100) KA_LINE(0x140)
                 KA_LINE(0x180) KA_LINE(0x1c0) KA_LINE(0x200) "s_waitcnt lgkmcnt(0)"
                 : "=&s"(sink) : "s"(base));
  } else if constexpr (BYTES / 64 >= 5) {
    asm volatile(KA_LINE(0x0) KA_LINE(0x40) KA_LINE(0x80) KA_LINE(0xc0) KA_LINE(0x100) "s_waitcnt lgkmcnt(0)"
                 : "=&s"(sink) : "s"(base));
  } else {
    return;
  }
#undef KA_LINE
  asm volatile("" ::"s"(sink));
}

// Waves per SIMD the step kernels are compiled for: in 2D the batched
// workload is throughput-bound and four waves per SIMD for the reverse kernel
// (at most 128 registers) beat three, six for the forward kernel (80
// registers) beat five; in 3D the kernels need their registers and LDS.
template <int D>
constexpr int kBwdWaves = (D == 2) ? 4 : 1;
template <int D>
constexpr int kFwdWaves = (D == 2) ? 6 : 1;

// Entry stamp t0 and exit stamp of this workgroup's wall clock, the exit taken
// once every wave of the workgroup has finished its work.
__device__ __forceinline__ void stamp_workgroup(const StepConsts& k, unsigned long long t0) {
  __syncthreads();
  if (threadIdx.x == 0 && k.clk_slot >= 0) {
    unsigned long long* p = k.wgclk + 2 * (size_t(k.clk_slot) * size_t(k.clk_stride) + blockIdx.x);
    p[0] = t0;
    p[1] = wall_clock64();
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Thread -> particle mapping. LPP = 1: one lane per particle (optionally
// interleaved, lane_particle). LPP = 2: a pair of lanes per particle, each
// visiting half of the stencil (see Sten and for_nodes); gathers are completed
// with one DPP add per value. LPP = 4: a quad of lanes per particle; lanes
// 0..2 each take one slab of the stencil (t0 = 0, 1, 2), lane 3 only joins
// the quad reductions. Lane 0 of a pair or quad writes the particle's outputs.
//
// With several scenes, workgroups are scene-aligned: k.blocks[b] = (first
// particle, particle count, scene) of workgroup b, so every workgroup holds one
// scene and can stage its grid box in LDS.
template <int LPP>
struct LaneMap {
  int first, i, sub, count, scene;
  bool live, owner;
  __device__ __forceinline__ LaneMap(const StepConsts& k, int block_index) {
    const int per_block = k.threads / LPP;
    int end;
    if (k.blocks) {
      const int4 bi = load_uniform(k.blocks + block_index);
      first = bi.x;
      count = bi.y;
      scene = bi.z;
      end = first + count;
    } else {
      first = block_index * per_block;
      count = per_block;
      scene = 0;
      end = k.N;
    }
    if constexpr (LPP == 4) {
      sub = int(threadIdx.x & 3);
      i = first + int(threadIdx.x >> 2);
    } else if constexpr (LPP == 2) {
      sub = int(threadIdx.x & 1);
      i = first + int(threadIdx.x >> 1);
    } else {
      sub = 0;
      i = first + lane_particle(threadIdx.x, k.threads, k.remap);
    }
    live = i < end;
    owner = sub == 0;
  }
};

// LDS of the forward step body.
template <int D>
struct FwdShared {
  alignas(16) long long tile64[(D + 1) * kTileCap<D>];  // P2G scatter tile (fixed point)
  float vtile[D * kTileCap<D>];              // G2P velocity tile
  int red[64];
};

// Forward step of workgroup `wgi` of the launch described by `a` (all threads
// of the workgroup call). M: constitutive model (0 neo-Hookean, 1
// fixed-corotated).
template <int D, int LPP, int M, bool P, bool PRE = false>
__device__ __forceinline__ void fwd_block(const FwdArgs& a, int wgi, FwdShared<D>& sh) {
  constexpr int S0 = (LPP == 4) ? 1 : (LPP == 2 ? 2 : 3);
  long long* tile64 = sh.tile64;
  float* vtile = sh.vtile;
  const StepConsts& k = a.k;
  const ClearSpec c0{a.clear, a.clear_box, a.clear_nbox, a.clear_n}, c1{nullptr, nullptr, 0, 0};
  if (a.clear_wgs && wgi >= k.n_blocks) {
    // A workgroup that only clears: the launch's clears then stay off the
    // stepping workgroups' chain, on compute units they leave idle.
    const int rank = clear_rank(k, wgi - k.n_blocks, true, 0);
    clear_jobs_run<D, P>(clear_jobs_fetch<P>(c0, c1, rank, k.groups), c0, c1, k, rank);
    return;
  }
  BlockRed rd{sh.red, 0, (k.threads + 63) >> 6};
  const LaneMap<LPP> lm(k, wgi);
  const int i = lm.i, sub = lm.sub;
  const bool live = lm.live;
  // Every workgroup holds particles of one scene (scene-aligned workgroups).
  const int sc = lm.scene;
  const bool one_scene = true;
  unsigned err = 0;
  const int rank = clear_rank(k, wgi, !a.clear_wgs, 0);
  if (k.blocks && lm.count == 0 && rank < 0) {  // an unused entry of the aligned partition
    if (a.do_p2g) record_box<D>(a.box_out, wgi, empty_tile<D>(), -1);
    return;
  }
  // Every independent global read is issued first: the state, the clear
  // boxes, and the G2P box recorded by the scatter into grid_in (the previous
  // launch), so the tile load needs neither this launch's positions nor a
  // reduction and its latency overlaps the state's.
  PState<D> p;
  if (live) load_state<D>(a.in, i, p);
  const ClearJobs cj = clear_jobs_fetch<P>(c0, c1, rank, k.groups);
  if (a.do_p2g && k.lds) zero_tile64<D, D + 1>(tile64, k.threads);
  Tile<D> T = empty_tile<D>();
  const float4* g = a.grid_in + long(sc) * k.nodes;
  if (a.do_g2p && a.box_in) {
    T = recorded_tile<D, P>(a.box_in, wgi, sc, one_scene, k.lds, k.n);
    tile_first_vel<D>(k, tile_first_issue<D>(k, T, g, nullptr), vtile);
    if (T.on && T.n > k.threads) tile_load_vel<D>(k, T, g, vtile, k.threads);
  }
  if (a.do_g2p) {
    Sten<D> st;
    const bool fin = live && state_finite<D>(p);
    const bool ok = fin && lane_sten<D, LPP>(k, p.x, sub, st);
    if (!a.box_in) {
      T = block_tile<D>(ok, st.base, one_scene, k.lds, rd);
      if (T.on) tile_load_vel<D>(k, T, g, vtile);
    }
    if (T.on) __syncthreads();
    clear_jobs_run<D, P>(cj, c0, c1, k, rank);
    if (ok) {
      if (T.on && in_tile<D>(T, st.base))
        g2p_body<D, true, S0>(k, st, lds_nodes<D>(vtile, T), p);
      else
        g2p_body<D, false, S0>(k, st, global_nodes<D>(g, k.n), p);
    } else if (live) {
      err |= fin ? kErrDomain : kErrNonfinite;
    }
    if (live && lm.owner) store_state<D>(a.out, i, p);
  } else {
    clear_jobs_run<D, P>(cj, c0, c1, k, rank);
  }
  if (a.do_p2g)
    p2g_phase<D, LPP, M, PRE>(k, live, i, sc, one_scene, sub, p, a.act_row, a.grid_out, tile64, rd, err, a.box_out, wgi);
  if (err) atomicOr(k.err, err);
}

// PRE: particles sorted by stencil base, LDS scatters summed over runs of
// equal-base lanes first (knob "presum"; one lane per particle only).
template <int D, int LPP, int M, bool PRE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFwdWaves<D>))) k_fwd(FwdArgs a) {
  __shared__ FwdShared<D> sh;
  warm_kernargs<sizeof(FwdArgs)>();
  const unsigned long long t0 = a.k.wgclk ? wall_clock64() : 0ull;
  fwd_block<D, LPP, M, false, PRE>(a, int(blockIdx.x), sh);
  if (a.k.wgclk) stamp_workgroup(a.k, t0);
}

// Sum `val` over the live lanes of the wavefront that share `key`, and add
// each group's sum (FP64) to base[key] once.
__device__ __forceinline__ void wave_add_keyed(bool live, int key, double val, double* base) {
  unsigned long long mask = __ballot(live);
  const int lane = threadIdx.x & 63;
  while (mask) {
    const int leader = __ffsll((long long)mask) - 1;
    const int kk = __builtin_amdgcn_readlane(key, leader);
    const bool mine = live && key == kk;
    const double s = wave_sum(mine ? val : 0.0);
    if (lane == leader) atomic_add_f64(base + kk, s);
    mask &= ~__ballot(mine);
  }
}

// LDS of the reverse step body.
template <int D>
struct BwdShared {
  float tA[(D + 1) * kTileCap<D>];      // phase A: adjoint tile (P*, m*)
  float tV[D * kTileCap<D>];            // phase B: velocity tile
  alignas(16) long long tS[(D + 1) * kTileCap<D>];  // scatter tile: phase B (adjoint grid), phase C (grid)
  int red[64];
};

// Reverse step of workgroup `wgi` of the launch described by `a` (all
// threads of the workgroup call).
template <int D, int LPP, int M, bool P, bool PRE = false>
__device__ __forceinline__ void bwd_block(const BwdArgs& a, int wgi, BwdShared<D>& sh) {
  constexpr int S0 = (LPP == 4) ? 1 : (LPP == 2 ? 2 : 3);
  float* tA = sh.tA;
  float* tV = sh.tV;
  long long* tS = sh.tS;
  const StepConsts& k = a.k;
  BlockRed rd{sh.red, 0, (k.threads + 63) >> 6};
  // With split_c, workgroups [0, nb) run phases A and B and workgroups
  // [nb, 2 nb) run phase C on the same particles: C does not depend on A or B.
  const int nb = k.n_blocks;
  const bool role_c = a.split_c && wgi >= nb;
  const int wg = role_c ? wgi - nb : wgi;
  const LaneMap<LPP> lm(k, wg);
  const int i = lm.i, sub = lm.sub;
  const bool live = lm.live, owner = lm.owner;
  // Every workgroup holds particles of one scene (scene-aligned workgroups).
  const int sc = lm.scene;
  const bool one_scene = true;
  unsigned err = 0;
  // With the recompute role, the clears are spread over both roles (groups =
  // 2 clear_per_role) or, when every workgroup of the launch has a compute
  // unit of its own, all given to the recompute role (groups =
  // clear_per_role): its workgroups end well before the adjoint ones, whose
  // chain then sets the launch's duration.
  const bool c_clears_only = a.split_c && k.groups == k.clear_per_role;
  const int rank = clear_rank(k, wg, role_c || !c_clears_only, (role_c && !c_clears_only) ? k.clear_per_role : 0);
  if (k.blocks && lm.count == 0 && rank < 0) {  // an unused entry of the aligned partition
    if (role_c) {
      record_box<D>(a.boxC, wg, empty_tile<D>(), -1);
    } else {
      if (!a.final_out) record_box<D>(a.boxB, wg, empty_tile<D>(), -1);
      if (a.do_c && !a.split_c) record_box<D>(a.boxC, wg, empty_tile<D>(), -1);
    }
    return;
  }
  const ClearSpec c0{a.clear0, a.clear0_box, a.clear0_nbox, a.clear0_n};
  const ClearSpec c1{a.clear1, a.clear1_box, a.clear1_nbox, a.clear1_n};
  const ClearJobs cj = clear_jobs_fetch<P>(c0, c1, rank, k.groups);
  if (role_c) {
    if (k.lds) zero_tile64<D, D + 1>(tS, k.threads);
    PState<D> p;
    if (live) load_state<D>(a.stC, i, p);
    clear_jobs_run<D, P>(cj, c0, c1, k, rank);
    p2g_phase<D, LPP, M, PRE>(k, live, i, sc, one_scene, sub, p, a.act_rowC, a.gC, tS, rd, err, a.boxC, wg);
    if (err) atomicOr(k.err, err);
    return;
  }
  // Every independent global read is issued first: the gather boxes recorded
  // by the scatters into grid s+1 (phase A) and grid s (phase B), read before
  // the particle loads are issued so that their round trip overlaps those;
  // dL/dstate(s+1) (seed, or state s+1 and the x*, F* partials), phase B's
  // inputs (x, F of state s and C of state s+1); then both tile loads, so no
  // phase waits for a read it could have started earlier.
  Tile<D> TA = empty_tile<D>(), TB = empty_tile<D>();
  if (a.a_mode == 1 && a.boxA_in) TA = recorded_tile<D, P>(a.boxA_in, wg, sc, one_scene, k.lds, k.n);
  if (!a.final_out && a.boxB_in) TB = recorded_tile<D, P>(a.boxB_in, wg, sc, one_scene, k.lds, k.n);
  float gx[D] = {}, gv[D] = {}, gC[D][D] = {}, gF[D][D] = {};
  PState<D> p;  // phase A: state s+1
  if (live) {
    if (a.a_mode == 0) {
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
    } else {
      load_state<D>(a.stA, i, p);
#pragma unroll
      for (int c = 0; c < D; ++c) gx[c] = a.partial[c * a.pstride + i];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) gF[c][b] = a.partial[(D + c * D + b) * a.pstride + i];
    }
  }
  PState<D> pB;  // phase B: x, F of state s
  float CnB[D][D] = {};
  if (!a.final_out && live) {
    load_xF<D>(a.stB, i, pB);
    if (a.cnext) {
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) CnB[c][b] = a.cnext[(c * D + b) * a.cnext_stride + i];
    }
  }
  if (!a.final_out && k.lds) zero_tile64<D, D>(tS, k.threads);
  {
    // Both gather tiles: the first node of each thread of both in one round
    // trip (tile_first_issue), the rest after.
    const float4* gA = a.gA + long(sc) * k.nodes;
    const float4* aA = a.aA + long(sc) * k.nodes;
    const float4* gB = a.gB + long(sc) * k.nodes;
    const TileFirst<D> fA = tile_first_issue<D>(k, TA, gA, aA);
    const TileFirst<D> fB = tile_first_issue<D>(k, TB, gB, nullptr);
    tile_first_adj<D>(k, fA, tA);
    tile_first_vel<D>(k, fB, tV);
    if (TA.on && TA.n > k.threads) tile_load_adj<D>(k, TA, gA, aA, tA, k.threads);
    if (TB.on && TB.n > k.threads) tile_load_vel<D>(k, TB, gB, tV, k.threads);
  }

  // dL/dstate(s+1): gx, gv, gC, gF.
  double eb = 0.0, actb = 0.0;
  int aid = -1;
  if (a.a_mode == 1) {
    // p2g*(s+1) with grid_op* folded into the gather.
    Sten<D> st;
    const bool ok = live && state_finite<D>(p) && lane_sten<D, LPP>(k, p.x, sub, st);
    const float4* g = a.gA + long(sc) * k.nodes;
    const float4* ad = a.aA + long(sc) * k.nodes;
    const Tile<D> T = a.boxA_in ? TA : block_tile<D>(ok, st.base, one_scene, k.lds, rd);
    if (T.on) {
      if (!a.boxA_in) tile_load_adj<D>(k, T, g, ad, tA);
      __syncthreads();
    }
    if (ok) {
      const SceneParams sp = scene_params(k.E, k.nu, k.vol, k.rho, sc);
      float act_tau;
      aid = actuator_of<D>(k, a.act_rowA, i, act_tau);
      float A[D][D], FFtI[D][D], lnJ, J, R[D][D];
      unsigned dummy = 0;
      const bool liquid = k.mat_id && k.mat_id[i] == 1;
      if (liquid)
        affine_liquid<D>(p, sp, act_tau, k.dt, k.kappa, A, J, dummy);
      else if constexpr (M == 1)
        affine_corotated<D>(p, sp, act_tau, k.dt, k.kappa, A, R, J, dummy);
      else
        affine<D>(p, sp, act_tau, k.dt, k.kappa, A, FFtI, lnJ, J, dummy);
      float mv[D];
#pragma unroll
      for (int c = 0; c < D; ++c) mv[c] = sp.mass * p.v[c];
      float Abar[D][D] = {}, vb[D] = {};
      if (T.on && in_tile<D>(T, st.base))
        p2g_adj_body<D, true, S0>(k, st, sp.mass, mv, A, lds_nodes<D>(tA, T), lds_nodes<D>(tA, T), gx, vb, Abar);
      else
        p2g_adj_body<D, false, S0>(k, st, sp.mass, mv, A, global_nodes<D>(g, k.n), global_nodes<D>(ad, k.n), gx, vb,
                                   Abar);
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
      if (liquid) {
        eb = liquid_adjoint<D>(p, sp, J, tb, gF);
      } else if constexpr (M == 1) {
        eb = corotated_adjoint<D>(p, sp, R, J, tb, gF);
      } else {
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
      }
      actb = double(k.act_strength) * tb[1][1];
    }
  }
  if (a.a_mode == 1) {
    if (a.gE) wave_add_keyed(live && owner, sc, eb, a.gE);
    if (a.gact_rowA && k.act_id) {
      for (int kk = 0; kk < k.n_act; ++kk) {
        const double s = wave_sum((live && owner && aid == kk) ? actb : 0.0);
        if ((threadIdx.x & 63) == 0 && s != 0.0) atomic_add_f64(a.gact_rowA + kk, s);
      }
    }
  }

  if (a.final_out) {
    clear_jobs_run<D, P>(cj, c0, c1, k, rank);
    if (!live || !owner) return;
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
    const PState<D>& p = pB;
    float px[D], pF[D][D];
#pragma unroll
    for (int c = 0; c < D; ++c) px[c] = gx[c];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) pF[c][b] = gF[c][b];
    Sten<D> st;
    bool fin = live;
#pragma unroll
    for (int c = 0; c < D; ++c) fin = fin && (p.x[c] * 0.0f == 0.0f);
    const bool ok = fin && lane_sten<D, LPP>(k, p.x, sub, st);
    const float4* g = a.gB + long(sc) * k.nodes;
    float4* ad = a.aB + long(sc) * k.nodes;
    Tile<D> T = TB;
    if (!a.boxB_in) {
      T = block_tile<D>(ok, st.base, one_scene, k.lds, rd);
      if (T.on) tile_load_vel<D>(k, T, g, tV);
    }
    if (T.on) __syncthreads();
    clear_jobs_run<D, P>(cj, c0, c1, k, rank);
    const bool in_t = T.on && ok && in_tile<D>(T, st.base);
    float Bm[D][D] = {}, vt[D] = {}, bound = 0.0f;
    if (ok) {
      float Cn[D][D];
      if (a.cnext) {
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[c][b] = CnB[c][b];
      } else if (in_t) {
        g2p_C<D, true, S0>(k, st, lds_nodes<D>(tV, T), Cn);
      } else {
        g2p_C<D, false, S0>(k, st, global_nodes<D>(g, k.n), Cn);
      }
      // F' = (I + dt C') F:  F* = (I + dt C')^T F'*,  C'* += dt F'* F^T.
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
      for (int c = 0; c < D; ++c) {
        vt[c] = gv[c] + k.dt * gx[c];
        float b = fabsf(vt[c]);
#pragma unroll
        for (int e = 0; e < D; ++e) b += 1.5f * k.dx * fabsf(Bm[c][e]);
        bound = fmaxf(bound, b);
      }
    }
    // One reduction: the scatter scale (bound of every particle of the
    // workgroup) and the box of the particles the tile does not cover (none
    // unless a recorded box missed one), so the recorded scatter box covers all.
    int e_fix = INT_MIN;
    Box<D> outside;
    if (k.lds) {
      outside = block_reduce<D>(ok && !in_t, st.base, bound, rd);
      e_fix = fixed_exponent(outside.bmax);
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        outside.mn[c] = INT_MAX;
        outside.mx[c] = INT_MIN;
      }
    }
    record_box_union<D>(a.boxB, wg, T, outside, one_scene ? sc : -1);
    const bool fix = T.on && e_fix != INT_MIN;
    const bool presum = PRE && LPP == 1 && fix;
    if (presum) e_fix -= 3;  // runs of up to eight lanes add one sum
    RunSum rs{};
    if (presum) rs = run_sum(ok && in_t, base_key<D>(st, k.n));
    const bool any = T.n > 0 || outside.mn[0] <= outside.mx[0];
    if (k.tstats && threadIdx.x == 0 && any) atomicAdd(k.tstats + ((fix && outside.mn[0] > outside.mx[0]) ? 0 : 1), 1ull);
    if (ok) {
      const bool scatter = LPP != 4 || sub < 3;
      if (in_t && fix) {
        FixNodes<D> fn = fix_nodes<D>(tS, T);
        fn.e = e_fix;
        if (PRE && presum)
          g2p_adj_body<D, S0, true>(k, st, vt, Bm, lds_nodes<D>(tV, T), fn, px, scatter, rs);
        else
          g2p_adj_body<D, S0>(k, st, vt, Bm, lds_nodes<D>(tV, T), fn, px, scatter);
      } else if (in_t) {
        g2p_adj_body<D, S0>(k, st, vt, Bm, lds_nodes<D>(tV, T), global_nodes<D>(ad, k.n), px, scatter);
      } else {
        g2p_adj_body<D, S0>(k, st, vt, Bm, global_nodes<D>(g, k.n), global_nodes<D>(ad, k.n), px, scatter);
      }
    }
    if (fix) {
      Tile<D> TS = T;
      TS.e = e_fix;
      __syncthreads();
      tile_flush64<D, D>(TS, tS, ad, k.n, k.threads);
    }
    if (live && owner) {
#pragma unroll
      for (int c = 0; c < D; ++c) a.partial[c * a.pstride + i] = px[c];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int b = 0; b < D; ++b) a.partial[(D + c * D + b) * a.pstride + i] = pF[c][b];
    }
  }

  // Phase C: recompute p2g(s-1).
  if (a.do_c && !a.split_c) {
    PState<D> p;
    if (live) load_state<D>(a.stC, i, p);
    __syncthreads();  // every thread is done with the scatter tile of phase B
    if (k.lds) zero_tile64<D, D + 1>(tS, k.threads);
    p2g_phase<D, LPP, M, PRE>(k, live, i, sc, one_scene, sub, p, a.act_rowC, a.gC, tS, rd, err, a.boxC, wg);
  }
  if (err) atomicOr(k.err, err);
}

template <int D, int LPP, int M, bool PRE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBwdWaves<D>))) k_bwd(BwdArgs a) {
  __shared__ BwdShared<D> sh;
  warm_kernargs<sizeof(BwdArgs)>();
  const unsigned long long t0 = a.k.wgclk ? wall_clock64() : 0ull;
  bwd_block<D, LPP, M, false, PRE>(a, int(blockIdx.x), sh);
  if (a.k.wgclk) stamp_workgroup(a.k, t0);
}

// Persistent forms (knob "persist"): the step launches of a recorded tape
// sequence run in one cooperative launch; each workgroup loops over the
// workgroups of each recorded launch (round robin) and all meet at a
// grid-wide barrier between launches, so the work and arithmetic are those
// of the launch-per-step form and only the launch boundaries differ.
template <int D, int LPP, int M>
__global__ void __launch_bounds__(256) k_fwd_persist(const FwdArgs* __restrict__ seq, int n) {
  __shared__ FwdShared<D> sh;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int l = 0; l < n; ++l) {
    const FwdArgs& a = seq[l];
    const int nvb = a.k.n_blocks;
    for (int vb = int(blockIdx.x); vb < nvb; vb += int(gridDim.x)) {
      fwd_block<D, LPP, M, true>(a, vb, sh);
      __syncthreads();
    }
    grid.sync();
  }
}

template <int D, int LPP, int M>
__global__ void __launch_bounds__(256) k_bwd_persist(const BwdArgs* __restrict__ seq, int n) {
  __shared__ BwdShared<D> sh;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int l = 0; l < n; ++l) {
    const BwdArgs& a = seq[l];
    const int nvb = a.k.n_blocks * (a.split_c ? 2 : 1);
    for (int vb = int(blockIdx.x); vb < nvb; vb += int(gridDim.x)) {
      bwd_block<D, LPP, M, true>(a, vb, sh);
      __syncthreads();
    }
    grid.sync();
  }
}

}  // namespace mpm

// Support kernels: particle binning (cell counts and a stable radix sort by
// scene and Morton cell order), permutation of states between the caller's order and the sorted
// internal order, the mean-position loss and its seed, the open-loop
// actuation signal and its adjoint, and buffer clears.
#pragma once

#include "device_math.h"

namespace mpm {

__global__ void k_zero_f4(float4* p, long n) {
  const long stride = long(gridDim.x) * blockDim.x;
  for (long q = long(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_zero_i32(int* p, long n) {
  const long stride = long(gridDim.x) * blockDim.x;
  for (long q = long(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0;
}

__global__ void k_zero_f64(double* p, long n) {
  const long stride = long(gridDim.x) * blockDim.x;
  for (long q = long(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0.0;
}

// Interleave the bits of cell coordinates (axis 0 most significant).
template <int D>
__device__ __forceinline__ unsigned morton(const int (&c)[D], int bits) {
  unsigned key = 0;
  for (int b = bits - 1; b >= 0; --b)
#pragma unroll
    for (int a = 0; a < D; ++a) key = (key << 1) | ((unsigned(c[a]) >> b) & 1u);
  return key;
}

// key[i] = scene * cells_per_scene + morton(cell of x_i), cells clamped into
// the grid; the cell of coordinate g is floor(x / dx - shift) (shift 0: the
// cell holding the particle; 1/2: its stencil base).
template <int D>
__global__ void k_sort_keys(StateRef st, int N, const int* scene_id, float inv_dx, float shift, int n, int bits,
                            unsigned cells_per_scene, unsigned* keys, int* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int c[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float g = st.x[a * st.stride + i] * inv_dx - shift;
    int ci = (g >= 0.0f) ? (g < float(n - 1) ? int(g) : n - 1) : 0;  // NaN -> 0
    c[a] = ci;
  }
  const int sc = scene_id ? scene_id[i] : 0;
  const unsigned key = unsigned(sc) * cells_per_scene + morton<D>(c, bits);
  keys[i] = key;
  atomicAdd(counts + key, 1);
}

// Exclusive scan, three passes: per-block scan (kScanItems per thread), scan
// of the block sums in one workgroup, add of the scanned sums.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int u = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_blocks(const int* in, int* out, long n, int* block_sums) {
  __shared__ int sh[kScanThreads];
  const long base = long(blockIdx.x) * kScanChunk + long(threadIdx.x) * kScanItems;
  int vals[kScanItems];
  int s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    vals[j] = (base + j < n) ? in[base + j] : 0;
    s += vals[j];
  }
  int total;
  int run = block_exclusive_scan(s, sh, total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += vals[j];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int* sums, int nb) {
  __shared__ int sh[kScanThreads];
  int carry = 0;
  for (int start = 0; start < nb; start += kScanThreads) {
    const int j = start + int(threadIdx.x);
    const int v = (j < nb) ? sums[j] : 0;
    int total;
    const int ex = block_exclusive_scan(v, sh, total);
    if (j < nb) sums[j] = ex + carry;
    carry += total;
    __syncthreads();
  }
}

__global__ void k_scan_add(int* out, long n, const int* sums) {
  const long base = long(blockIdx.x) * kScanChunk;
  const int add = sums[blockIdx.x];
  for (int j = threadIdx.x; j < kScanChunk; j += blockDim.x)
    if (base + j < n) out[base + j] += add;
}

// Stable least-significant-digit radix sort of (key, index) pairs, 8 bits
// per pass, tiles of kRadixTile consecutive elements (one per thread). A pass
// counts each tile's digits (k_radix_hist, digit-major so that one exclusive
// scan gives every (digit, tile) its output offset), then each tile writes
// its elements in index order within every digit (k_radix_scatter: the rank
// among same-digit lanes of a wave comes from eight ballots, the waves of the
// tile follow each other). Equal keys therefore keep their caller order, and
// the work per element is the same whatever the key distribution (a single
// key holding every particle included).
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kRadixTile = 256;

__global__ void __launch_bounds__(kRadixTile) k_radix_hist(const unsigned* keys, int N, int shift, int n_tiles,
                                                           int* hist) {
  __shared__ int cnt[kRadix];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * kRadixTile + int(threadIdx.x);
  if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & (kRadix - 1)], 1);
  __syncthreads();
  hist[long(threadIdx.x) * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// offs: exclusive scan of hist. vin null: the values are the element indices.
__global__ void __launch_bounds__(kRadixTile) k_radix_scatter(const unsigned* kin, const int* vin, int N, int shift,
                                                              int n_tiles, const int* offs, unsigned* kout,
                                                              int* vout) {
  constexpr int kWaves = kRadixTile / 64;
  __shared__ int wcnt[kWaves][kRadix];
  const int t = int(threadIdx.x), w = t >> 6, lane = t & 63;
  for (int q = t; q < kWaves * kRadix; q += kRadixTile) (&wcnt[0][0])[q] = 0;
  const int i = blockIdx.x * kRadixTile + t;
  const bool live = i < N;
  const unsigned key = live ? kin[i] : 0u;
  const int d = int((key >> shift) & (kRadix - 1));
  unsigned long long same = __ballot(live);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1;
    const unsigned long long m = __ballot(bit);
    same &= bit ? m : ~m;
  }
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int rank = __popcll(same & below);
  const int group = __popcll(same);
  __syncthreads();  // wcnt cleared
  if (live && rank == group - 1) wcnt[w][d] = group;
  __syncthreads();
  if (!live) return;
  int before = 0;
  for (int q = 0; q < w; ++q) before += wcnt[q][d];
  const int pos = offs[long(d) * n_tiles + blockIdx.x] + before + rank;
  kout[pos] = key;
  vout[pos] = vin ? vin[i] : i;
}

// Workgroup partition aligned to the Morton cell hierarchy, built from the
// cell starts of the last sort. A block of level l is 2^(D l) consecutive keys
// of one scene (a cube of 2^l cells per axis). A block holding more than P
// particles (P = particles per workgroup) is split: its 2^D children, in key
// order, are packed greedily into workgroups of at most P particles (runs of
// consecutive children only), a child holding more than P particles being
// split in turn; a single cell holding more than P particles is cut into runs
// of P. A scene holding at most P particles is one workgroup. Every workgroup
// therefore lies inside one block whose children it packs, so its particles
// span at most 2^l + 2 nodes per axis (the stencil adds two), unlike runs of P
// consecutive particles, which straddle distant blocks where the Morton curve
// jumps. One thread per block of level >= 1 (a parent), in the order
// (scene, level, block); k_part_visit counts (out null) or writes the
// workgroups that parent emits.
struct PartGeom {
  int dim, bits, P, n_scenes, N;
  long n_keys;
  long cells_per_scene;
  int per_scene;  // parents per scene: sum over l = 1..bits of 2^(dim (bits - l))
};

__device__ __forceinline__ int part_start(const int* start, const PartGeom& g, long key) {
  return key < g.n_keys ? start[key] : g.N;
}

__device__ __forceinline__ int part_visit(const int* start, const PartGeom& g, int t, int4* out) {
  const int sc = t / g.per_scene;
  int r = t - sc * g.per_scene;
  int l = 1;
  for (; l < g.bits; ++l) {
    const int nb = 1 << (g.dim * (g.bits - l));
    if (r < nb) break;
    r -= nb;
  }
  const long size = 1L << (g.dim * l), csize = size >> g.dim;
  const long b0 = long(sc) * g.cells_per_scene + long(r) * size;
  const int f0 = part_start(start, g, b0);
  const int cnt = part_start(start, g, b0 + size) - f0;
  int emitted = 0;
  auto emit = [&](int first, int count) {
    if (out) out[emitted] = make_int4(first, count, sc, 0);
    ++emitted;
  };
  if (cnt <= g.P) {
    if (l == g.bits && cnt > 0) emit(f0, cnt);  // the whole scene
    return emitted;
  }
  int cur_f = 0, cur_n = 0;
  for (int ch = 0; ch < (1 << g.dim); ++ch) {
    const long c0 = b0 + ch * csize;
    const int cf = part_start(start, g, c0);
    const int cc = part_start(start, g, c0 + csize) - cf;
    if (cc > g.P) {
      if (cur_n) emit(cur_f, cur_n);
      cur_n = 0;
      if (l == 1)
        for (int f = cf; f < cf + cc; f += g.P) emit(f, min(g.P, cf + cc - f));
    } else if (cc > 0) {
      if (cur_n + cc > g.P) {
        emit(cur_f, cur_n);
        cur_n = 0;
      }
      if (cur_n == 0) cur_f = cf;
      cur_n += cc;
    }
  }
  if (cur_n) emit(cur_f, cur_n);
  return emitted;
}

__global__ void k_part_count(const int* start, PartGeom g, int* counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.per_scene * g.n_scenes) return;
  counts[t] = part_visit(start, g, t, nullptr);
}

// offs: exclusive scan of the counts. Writes only if the partition fits in cap.
__global__ void k_part_emit(const int* start, PartGeom g, const int* counts, const int* offs, int cap, int4* table) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_par = g.per_scene * g.n_scenes;
  if (t >= n_par) return;
  const int total = offs[n_par - 1] + counts[n_par - 1];
  if (total > cap || counts[t] == 0) return;
  part_visit(start, g, t, table + offs[t]);
}

// Pads the table to cap entries with empty workgroups (count 0); if the
// partition did not fit, writes the plain one (n_plain entries) instead.
__global__ void k_part_finish(PartGeom g, const int* counts, const int* offs, int cap, const int4* plain,
                              int n_plain, int4* table) {
  const int n_par = g.per_scene * g.n_scenes;
  const int total = offs[n_par - 1] + counts[n_par - 1];
  int used = total;
  if (total > cap) {
    for (int j = threadIdx.x; j < n_plain; j += blockDim.x) table[j] = plain[j];
    used = n_plain;
  }
  for (int j = used + int(threadIdx.x); j < cap; j += blockDim.x) table[j] = make_int4(0, 0, 0, 0);
}

// dst[i] = src[perm[i]] for all S components (perm null: identity).
template <int D>
__global__ void k_gather_state(StateRef src, StateRef dst, const int* perm, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int j = perm ? perm[i] : i;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    dst.x[c * dst.stride + i] = src.x[c * src.stride + j];
    dst.v[c * dst.stride + i] = src.v[c * src.stride + j];
  }
#pragma unroll
  for (int c = 0; c < D * D; ++c) {
    dst.C[c * dst.stride + i] = src.C[c * src.stride + j];
    dst.F[c * dst.stride + i] = src.F[c * src.stride + j];
  }
}

// dst[perm[i]] = src[i].
template <int D>
__global__ void k_scatter_state(StateRef src, StateRef dst, const int* perm, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int j = perm ? perm[i] : i;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    dst.x[c * dst.stride + j] = src.x[c * src.stride + i];
    dst.v[c * dst.stride + j] = src.v[c * src.stride + i];
  }
#pragma unroll
  for (int c = 0; c < D * D; ++c) {
    dst.C[c * dst.stride + j] = src.C[c * src.stride + i];
    dst.F[c * dst.stride + j] = src.F[c * src.stride + i];
  }
}

__global__ void k_copy_i4(const int4* src, int4* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_gather_i32(const int* src, int* dst, const int* perm, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  dst[i] = src[perm ? perm[i] : i];
}

// One workgroup per scene: L_k = sign * mean_p x_{p,axis} (FP64 sum in a
// fixed order).
template <int D>
__global__ void __launch_bounds__(1024) k_loss_mean(StateRef fin, const int* offsets, int axis, float sign,
                                                    float* loss) {
  __shared__ double sh[1024 / 64];
  const int sc = blockIdx.x;
  const int lo = offsets[sc], hi = offsets[sc + 1];
  double s = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) s += double(fin.x[axis * fin.stride + i]);
  s = wave_sum(s);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += sh[q];
    loss[sc] = (hi > lo) ? float(double(sign) * t / double(hi - lo)) : 0.0f;
  }
}

// dL/dstate of the mean-position loss, one thread per particle: sign / N_k on
// the loss axis of x (k = the particle's scene), zero in every other component.
template <int D>
__global__ void k_loss_seed(const int* offsets, int n_scenes, int N, int axis, float sign, StateRef seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int a = 0, b = n_scenes;  // offsets[a] <= i < offsets[b]
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (offsets[m] <= i)
      a = m;
    else
      b = m;
  }
  const float g = sign / float(offsets[a + 1] - offsets[a]);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    seed.x[c * seed.stride + i] = (c == axis) ? g : 0.0f;
    seed.v[c * seed.stride + i] = 0.0f;
  }
#pragma unroll
  for (int c = 0; c < D * D; ++c) {
    seed.C[c * seed.stride + i] = 0.0f;
    seed.F[c * seed.stride + i] = 0.0f;
  }
}

// act[s][k] = tanh(sum_j W[k][j] sin(omega s dt + 2 pi j / n_sin) + b[k]).
__global__ void k_actuation(const float* W, const float* b, int n_act, int n_sin, float omega, float dt, int T,
                            float* act) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= T * n_act) return;
  const int s = q / n_act, kk = q % n_act;
  const float t = float(s) * dt;
  float pre = b[kk];
  for (int j = 0; j < n_sin; ++j) pre += W[kk * n_sin + j] * sinf(omega * t + 6.283185307179586f * float(j) / float(n_sin));
  act[q] = tanhf(pre);
}

// gW[k][j] += sum_s gact[s][k] (1 - a^2) sin(...), gb[k] += sum_s gact[s][k] (1 - a^2).
// One thread per (k, j) pair; j == n_sin is the bias.
__global__ void k_actuation_bwd(const float* W, const float* b, int n_act, int n_sin, float omega, float dt, int T,
                                const float* gact, float* gW, float* gb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_act * (n_sin + 1)) return;
  const int kk = q / (n_sin + 1), j = q % (n_sin + 1);
  double acc = 0.0;
  for (int s = 0; s < T; ++s) {
    const float t = float(s) * dt;
    float pre = b[kk];
    for (int jj = 0; jj < n_sin; ++jj)
      pre += W[kk * n_sin + jj] * sinf(omega * t + 6.283185307179586f * float(jj) / float(n_sin));
    const float a = tanhf(pre);
    const float d = gact[s * n_act + kk] * (1.0f - a * a);
    const float basis = (j < n_sin) ? sinf(omega * t + 6.283185307179586f * float(j) / float(n_sin)) : 1.0f;
    acc += double(d) * double(basis);
  }
  if (j < n_sin)
    gW[kk * n_sin + j] += float(acc);
  else
    gb[kk] += float(acc);
}

// dst[i] += float(src[i]) (FP64 accumulators to the caller's FP32 gradients).
__global__ void k_add_f64_to_f32(const double* src, float* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += float(src[i]);
}

}  // namespace mpm

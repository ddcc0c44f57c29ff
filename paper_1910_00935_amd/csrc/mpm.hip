// Host runtime and C ABI of the differentiable MLS-MPM library (gfx950).
//
// Owns no device memory: the caller binds a workspace (grids, sort buffers,
// adjoint partials, FP64 accumulators, error word) and tape memory (state
// slots). The forward trajectory is one fused launch per step; the reverse is
// one fused launch per step with the grid recomputed (DiffTaichi Appendix D.1)
// and, for checkpointed tapes, each segment recomputed from its checkpoint
// before its steps are reversed (Appendix D.2).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mpm.h"
#include "step_kernels.h"
#include "util_kernels.h"

using mpm::BwdArgs;
using mpm::FwdArgs;
using mpm::StateRef;
using mpm::StepConsts;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Buffers of the workspace, in order.
enum Region {
  R_GRID,      // 10 grids: 0-2 forward, 3-6 reverse primal, 7-9 reverse adjoint
  R_PARTIAL,   // (d + d^2) x Np floats
  R_SEED,      // S x Np floats, sorted dL/dstate(T)
  R_KEYS,      // N uint32 sort keys (radix passes ping-pong with R_KEYS2)
  R_KEYS2,     // N uint32
  R_VALS,      // N int32 radix-pass values
  R_RHIST,     // kRadix x radix tiles int32: per-tile digit counts, scanned in place
  R_COUNTS,    // n_keys int32
  R_START,     // n_keys int32
  R_BSUMS,     // scan block sums
  R_SCENE_ID,  // N int32
  R_OFFSETS,   // n_scenes + 1 int32
  R_GE,        // n_scenes double
  R_GACT,      // kMaxAct double (single-step adjoint)
  R_ERR,       // 1 uint32
  R_TSTATS,    // 2 uint64: scatter tile counters (knob "tile_stats")
  R_BLOCKS,    // int4 per workgroup: the plain table padded (single steps, in the caller's order)
  R_PLAIN,     // int4 per workgroup: the plain partition (runs of consecutive particles)
  R_PART,      // int32 per parent block: workgroups it emits, scanned
  R_BOXES,     // per grid, 2 int4 per workgroup: nodes its last scatter touched
  R_COUNT
};

constexpr int kNumGrids = 10;
constexpr int kGridF = 0, kGridB = 3, kAdj = 7;
constexpr int kZero = -1, kDirty = -2;
static_assert(kNumGrids == 10, "mpm_ctx::gstate lists one initial state per grid");

}  // namespace

// Device memory of the allocation-free forward step (mpm_step_fwd_noalloc):
// one fixed array per GPU the library runs on, held until the process ends.
// Host code never uses the array's name as an address (on the host it is a
// stand-in, not device memory): each device's address is looked up once,
// with that device current, by scratch_on_current_device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct mpm_ctx {
  int d = 0, n = 0, bound = 0, ns = 0, n_act = 0, N = 0, Np = 0, S = 0;
  long nodes = 0;
  float dx = 0, dt = 0, gravity = 0, act_strength = 0;
  int bits = 0;
  unsigned cells_per_scene = 0;
  long n_keys = 0;
  std::vector<int> offsets;
  size_t off[R_COUNT] = {}, bytes[R_COUNT] = {};
  size_t ws_bytes = 0;
  char* ws = nullptr;
  int block = 128;
  int lds = 1;
  int split_c = 1;
  int remap = 0;
  int rotate = 1;
  int lanes = 1;
  int graph = 1;
  int part = 1;      // 1: workgroups aligned to the Morton cell hierarchy (rebuilt at each sort)
  int persist = 0;   // 1: a full tape's step launches run as one cooperative persistent launch
  int tile_stats = 0;  // 1: count LDS-tile and fallback scatters (R_TSTATS)
  int presum = 0;    // 1: sort by stencil base; run sums before the LDS scatter atomics
  // While a persistent sequence is enqueued: step launches are appended here
  // instead of being launched.
  std::vector<FwdArgs>* rec_fwd = nullptr;
  std::vector<BwdArgs>* rec_bwd = nullptr;
  int persist_grid[2] = {0, 0};  // co-resident workgroups of the persistent kernels (0: not queried)
  int persist_grid_shape[2] = {0, 0};  // block * 8 + lanes they were queried for
  int model = 0;     // constitutive model: 0 neo-Hookean, 1 fixed-corotated (MPM_MODEL_COROTATED)
  int n_blocks = 0;  // workgroups per particle pass for the current block and lanes
  int n_plain = 0;   // workgroups of the plain partition
  int n_cus = 0;     // compute units of the device (0: not known)
  // Host copy of the caller-order workgroup table of single steps (R_BLOCKS:
  // the plain partition padded to n_blocks entries), empty when the launch
  // needs none (one scene, plain partition).
  std::vector<int4> blocks_host;
  long blocks_cap = 0;
  // What each grid holds, tracked while a launch sequence is enqueued: kZero,
  // kDirty (anything), or n >= 0: non-zero only inside the boxes its last
  // scatter (n workgroups) recorded in its R_BOXES table.
  long box_cap = 0;
  mutable int gstate[kNumGrids] = {kDirty, kDirty, kDirty, kDirty, kDirty, kDirty, kDirty, kDirty, kDirty, kDirty};
  hipStream_t capture = nullptr;
  // Per-kernel timing (knob "timing"): one event pair around each run of
  // consecutive launches of one step kernel on one stream (a span), read back
  // by mpm_kernel_stats as total time and launch count.
  struct Span {
    int kind;
    hipEvent_t e0, e1;
    long n;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Span> ev_pending;
  size_t ev_used = 0;
  int span_kind = -1;
  long span_n = 0;
  hipEvent_t span_e0 = nullptr;
  hipStream_t span_st = nullptr;
  double ev_ms[2] = {0.0, 0.0};
  long ev_count[2] = {0, 0};
  // Workgroup wall clocks (mpm_wg_clock_bind): caller buffer of clk_slots
  // launch rows of clk_stride workgroups; launches take rows in enqueue order
  // (clk_next), their kernel kind and workgroup count kept in clk_kind and
  // clk_wgs. clk_epoch changes at every bind (part of the graph key, so a
  // sequence is captured again with its new rows).
  unsigned long long* clk = nullptr;
  long clk_slots = 0;
  int clk_stride = 0;
  int clk_epoch = 0;
  mutable int clk_next = 0;
  mutable std::vector<int> clk_kind, clk_wgs;

  template <class T>
  T* at(Region r) const {
    return reinterpret_cast<T*>(ws + off[r]);
  }
  float4* grid(int k) const { return at<float4>(R_GRID) + size_t(k) * ns * nodes; }
  long grid_f4() const { return long(ns) * nodes; }
  int blocks_for(long n_items) const { return int((n_items + block - 1) / block); }
};

struct mpm_tape {
  mpm_ctx* ctx = nullptr;
  int T = 0, K = 0;
  bool full = true;
  int n_ckpt = 0, R = 0, n_slots = 0;
  size_t slot_floats = 0, off_gact = 0, off_perm = 0, off_act = 0, off_mat = 0, off_blocks = 0, off_seq = 0,
         total = 0;
  // Recorded step launches of the persistent form (host copies; uploaded
  // into the tape's sequence region before each persistent launch).
  std::vector<FwdArgs> seq_fwd;
  std::vector<BwdArgs> seq_bwd;
  char* mem = nullptr;
  bool recorded = false;
  mpm_params rec{};
  // Launch shape the recorded forward sorted and partitioned for (knobs
  // "block", "lanes", "part"); the reverse pass needs the same.
  int rec_block = 0, rec_lanes = 0, rec_part = 0, rec_presum = 0;
  std::vector<int> ring_holds;
  // Captured launch sequences (knob "graph"): key = every pointer and size the
  // sequence depends on plus the checkpoint-ring state it starts from; the
  // ring state the sequence leaves behind is restored on replay.
  struct Graph {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
    std::vector<int> ring_after;
  };
  std::vector<Graph> graphs;

  int slot_index(int s) const {
    if (s == T) return n_ckpt;
    if (!full && s % K == 0) return s / K;
    if (full && s == 0) return 0;
    const int r = full ? (s - 1) : (s % (2 * K));
    return n_ckpt + 1 + r;
  }
  float* slot_base(int s) const {
    return reinterpret_cast<float*>(mem) + size_t(slot_index(s)) * slot_floats;
  }
  StateRef slot(int s) const {
    const mpm_ctx& c = *ctx;
    float* b = slot_base(s);
    const size_t Np = size_t(c.Np);
    return StateRef{b, b + c.d * Np, b + 2 * c.d * Np, b + (2 * c.d + c.d * c.d) * Np, c.Np};
  }
  double* gact() const { return reinterpret_cast<double*>(mem + off_gact); }
  // The recorded trajectory's sort (sorted index -> caller index), its
  // per-particle ids in sorted order, and its workgroup table: kept with the
  // tape, so other tapes of the context may run between its forward and its
  // reverse pass.
  int* perm() const { return reinterpret_cast<int*>(mem + off_perm); }
  int* act_ids() const { return reinterpret_cast<int*>(mem + off_act); }
  int* mat_ids() const { return reinterpret_cast<int*>(mem + off_mat); }
  int4* blocks() const { return reinterpret_cast<int4*>(mem + off_blocks); }
  char* seq() const { return mem + off_seq; }
};

namespace {

#define HIP_TRY(expr)                           \
  do {                                          \
    if ((expr) != hipSuccess) return MPM_E_HIP; \
  } while (0)

#define LAUNCH_TRY()                                  \
  do {                                                \
    if (hipGetLastError() != hipSuccess) return MPM_E_HIP; \
  } while (0)

bool state_ok(const mpm_state* s) { return s && s->x && s->v && s->C && s->F; }
bool params_ok(const mpm_params* p) { return p && p->E && p->nu && p->vol && p->rho; }

StateRef user_ref(const mpm_ctx& c, const mpm_state* s) {
  return StateRef{s->x, s->v, s->C, s->F, c.N};
}

// `tp` non-null: the launch runs on that tape's sorted particle order (its
// per-particle ids and workgroup table) rather than the caller's. `table` and
// `err` are the caller-order workgroup table and the error word of the memory
// the launch uses (the bound workspace, or the fixed scratch of the
// allocation-free step).
StepConsts consts(const mpm_ctx& c, const mpm_params* p, const mpm_tape* tp, const int4* table, unsigned* err) {
  const int* act_id = p->act_id ? (tp ? tp->act_ids() : p->act_id) : nullptr;
  StepConsts k;
  k.N = c.N;
  k.n = c.n;
  k.bound = c.bound;
  k.nodes = int(c.nodes);
  k.n_act = c.n_act;
  k.n_scenes = c.ns;
  k.dx = c.dx;
  k.inv_dx = 1.0f / c.dx;
  k.dt = c.dt;
  k.gdt = c.gravity * c.dt;
  k.kappa = 4.0f / (c.dx * c.dx);
  k.act_strength = c.act_strength;
  k.lds = c.lds;
  // Base-sorted run sums need every lane of a run to visit its stencil in
  // the same order, on consecutive lanes.
  k.remap = c.presum ? 0 : c.remap;
  k.rotate = c.presum ? 0 : c.rotate;
  k.blocks = (c.ns > 1 || c.part) ? (tp ? tp->blocks() : table) : nullptr;
  k.n_blocks = c.n_blocks;
  k.E = p->E;
  k.nu = p->nu;
  k.vol = p->vol;
  k.rho = p->rho;
  k.act_id = (c.n_act > 0) ? act_id : nullptr;
  k.mat_id = p->mat_id ? (tp ? tp->mat_ids() : p->mat_id) : nullptr;
  k.err = err;
  k.tstats = nullptr;
  return k;
}

StepConsts consts(const mpm_ctx& c, const mpm_params* p, const mpm_tape* tp) {
  StepConsts k = consts(c, p, tp, c.at<int4>(R_BLOCKS), c.at<unsigned>(R_ERR));
  if (c.tile_stats) k.tstats = c.at<unsigned long long>(R_TSTATS);
  return k;
}

// Geometry of the cell hierarchy for the aligned partition (P particles per
// workgroup).
mpm::PartGeom part_geom(const mpm_ctx& c, int P) {
  mpm::PartGeom g;
  g.dim = c.d;
  g.bits = c.bits;
  g.P = P;
  g.n_scenes = c.ns;
  g.N = c.N;
  g.n_keys = c.n_keys;
  g.cells_per_scene = long(c.cells_per_scene);
  g.per_scene = 0;
  for (int l = 1; l <= c.bits; ++l) g.per_scene += 1 << (c.d * (c.bits - l));
  return g;
}

const float* act_row(const mpm_ctx& c, const mpm_params* p, int s) {
  return (p->act && c.n_act > 0) ? p->act + size_t(s) * c.n_act : nullptr;
}

void span_close(const mpm_ctx& cc);

mpm_status zero_f4(const mpm_ctx& c, float4* p, long n, hipStream_t st) {
  span_close(c);
  const int blocks = int(std::min<long>((n + 255) / 256, 8192));
  if (blocks <= 0) return MPM_OK;
  hipLaunchKernelGGL(mpm::k_zero_f4, dim3(blocks), dim3(256), 0, st, p, n);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status zero_f64(double* p, long n, hipStream_t st) {
  if (n <= 0) return MPM_OK;
  const int blocks = int(std::min<long>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(mpm::k_zero_f64, dim3(blocks), dim3(256), 0, st, p, n);
  LAUNCH_TRY();
  return MPM_OK;
}

// Sparse clears: a scatter into grid g records its workgroups' boxes (when
// LDS boxes are on) and a later clear of g zeroes only those boxes.
int4* box_table(const mpm_ctx& c, int g) { return c.at<int4>(R_BOXES) + size_t(g) * 2 * size_t(c.box_cap); }

mpm_status zero_grid(const mpm_ctx& c, int g, hipStream_t s) {
  c.gstate[g] = kZero;
  return zero_f4(c, c.grid(g), c.grid_f4(), s);
}

// Box table for a scatter into grid g (null: not recorded).
int4* scatter_into(const mpm_ctx& c, int g) {
  if (c.lds) {
    c.gstate[g] = c.n_blocks;
    return box_table(c, g);
  }
  c.gstate[g] = kDirty;
  return nullptr;
}

// Box table of grid g when its content came from one scatter launch of the
// current launch shape (the gather of g can reuse the boxes), else null.
const int4* recorded_boxes(const mpm_ctx& c, int g) {
  return (c.lds && c.gstate[g] == c.n_blocks) ? box_table(c, g) : nullptr;
}

// Clear of grid g by a step launch: nothing (already zero), its recorded
// boxes, or the whole grid.
void plan_clear(const mpm_ctx& c, int g, float4*& ptr, long& n, const int4*& box, int& nbox) {
  ptr = nullptr;
  n = 0;
  box = nullptr;
  nbox = 0;
  if (c.gstate[g] != kZero) {
    ptr = c.grid(g);
    if (c.gstate[g] == c.n_blocks) {
      box = box_table(c, g);
      nbox = c.n_blocks;
    } else {
      n = c.grid_f4();
    }
  }
  c.gstate[g] = kZero;
}

hipEvent_t pool_event(mpm_ctx& c) {
  if (c.ev_used == c.ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c.ev_pool.push_back(e);
  }
  return c.ev_pool[c.ev_used++];
}

// Ends the open timing span (any launch that is not a step kernel, and the
// end of every entry point, calls this).
void span_close(const mpm_ctx& cc) {
  mpm_ctx& c = const_cast<mpm_ctx&>(cc);
  if (c.span_kind < 0) return;
  hipEvent_t e1 = pool_event(c);
  if (e1 && hipEventRecord(e1, c.span_st) == hipSuccess) c.ev_pending.push_back({c.span_kind, c.span_e0, e1, c.span_n});
  c.span_kind = -1;
  c.span_n = 0;
}

// Before a step-kernel launch of `kind` on `s`: extends the open span or opens one.
void span_step(const mpm_ctx& cc, int kind, hipStream_t s) {
  mpm_ctx& c = const_cast<mpm_ctx&>(cc);
  if (!c.timing) return;
  if (c.span_kind == kind && c.span_st == s) {
    ++c.span_n;
    return;
  }
  span_close(c);
  hipEvent_t e0 = pool_event(c);
  if (!e0 || hipEventRecord(e0, s) != hipSuccess) return;
  c.span_kind = kind;
  c.span_e0 = e0;
  c.span_st = s;
  c.span_n = 1;
}

// Closes the open timing span when an entry point returns.
struct SpanGuard {
  const mpm_ctx& c;
  explicit SpanGuard(const mpm_ctx& cc) : c(cc) {}
  ~SpanGuard() { span_close(c); }
};

// Gives a launch of `wgs` workgroups of kernel `kind` its wall-clock row, if
// clocks are bound and a row of the right width is left.
void clock_row(const mpm_ctx& c, StepConsts& k, int kind, int wgs) {
  if (!c.clk || wgs > c.clk_stride || c.clk_next >= c.clk_slots) return;
  k.wgclk = c.clk;
  k.clk_stride = c.clk_stride;
  k.clk_slot = c.clk_next++;
  c.clk_kind.push_back(kind);
  c.clk_wgs.push_back(wgs);
}

template <int D, int LPP>
mpm_status launch_fwd(const mpm_ctx& c, const FwdArgs& args, hipStream_t st, bool timed) {
  FwdArgs a = args;
  a.k.threads = c.block;
  a.k.clear_per_role = c.part ? c.n_plain : c.n_blocks;
  a.k.groups = a.k.clear_per_role;
  if (c.rec_fwd) {
    c.rec_fwd->push_back(a);  // the persistent form's stepping workgroups clear
    return MPM_OK;
  }
  // When the stepping workgroups leave compute units idle, as many more
  // workgroups take the clears instead (every launch, so each launch of a
  // sequence has the same shape).
  a.clear_wgs = (c.n_cus > 0 && 2 * c.n_blocks <= c.n_cus) ? a.k.clear_per_role : 0;
  const int wgs = c.n_blocks + a.clear_wgs;
  clock_row(c, a.k, MPM_KERNEL_FWD, wgs);
  if (timed) span_step(c, 0, st);
  const bool pre = LPP == 1 && c.presum;
  if (c.model == 1) {
    if (pre)
      hipLaunchKernelGGL((mpm::k_fwd<D, LPP, 1, LPP == 1>), dim3(wgs), dim3(c.block), 0, st, a);
    else
      hipLaunchKernelGGL((mpm::k_fwd<D, LPP, 1>), dim3(wgs), dim3(c.block), 0, st, a);
  } else {
    if (pre)
      hipLaunchKernelGGL((mpm::k_fwd<D, LPP, 0, LPP == 1>), dim3(wgs), dim3(c.block), 0, st, a);
    else
      hipLaunchKernelGGL((mpm::k_fwd<D, LPP, 0>), dim3(wgs), dim3(c.block), 0, st, a);
  }
  LAUNCH_TRY();
  return MPM_OK;
}

template <int D, int LPP>
mpm_status launch_bwd(const mpm_ctx& c, const BwdArgs& args, hipStream_t st) {
  const int nb = c.n_blocks * (args.split_c ? 2 : 1);
  BwdArgs a = args;
  a.k.threads = c.block;
  a.k.clear_per_role = c.part ? c.n_plain : c.n_blocks;
  // With a separate recompute role the clears go to both roles, or to the
  // recompute role alone when every workgroup of the launch has a compute
  // unit of its own (the kernel reads which from groups).
  const bool clears_c_only = args.split_c && c.n_cus > 0 && nb <= c.n_cus;
  a.k.groups = (args.split_c && !clears_c_only ? 2 : 1) * a.k.clear_per_role;
  if (c.rec_bwd) {
    c.rec_bwd->push_back(a);
    return MPM_OK;
  }
  clock_row(c, a.k, MPM_KERNEL_BWD, nb);
  span_step(c, 1, st);
  const bool pre = LPP == 1 && c.presum;
  if (c.model == 1) {
    if (pre)
      hipLaunchKernelGGL((mpm::k_bwd<D, LPP, 1, LPP == 1>), dim3(nb), dim3(c.block), 0, st, a);
    else
      hipLaunchKernelGGL((mpm::k_bwd<D, LPP, 1>), dim3(nb), dim3(c.block), 0, st, a);
  } else {
    if (pre)
      hipLaunchKernelGGL((mpm::k_bwd<D, LPP, 0, LPP == 1>), dim3(nb), dim3(c.block), 0, st, a);
    else
      hipLaunchKernelGGL((mpm::k_bwd<D, LPP, 0>), dim3(nb), dim3(c.block), 0, st, a);
  }
  LAUNCH_TRY();
  return MPM_OK;
}

// `timed`: the launch may take part in the "timing" knob's event spans.
mpm_status fwd(const mpm_ctx& c, const FwdArgs& a, hipStream_t st, bool timed = true) {
  if (c.d == 2) {
    if (c.lanes == 4) return launch_fwd<2, 4>(c, a, st, timed);
    return c.lanes == 2 ? launch_fwd<2, 2>(c, a, st, timed) : launch_fwd<2, 1>(c, a, st, timed);
  }
  if (c.lanes == 4) return launch_fwd<3, 4>(c, a, st, timed);
  return c.lanes == 2 ? launch_fwd<3, 2>(c, a, st, timed) : launch_fwd<3, 1>(c, a, st, timed);
}
mpm_status bwd(const mpm_ctx& c, const BwdArgs& a, hipStream_t st) {
  if (c.d == 2) {
    if (c.lanes == 4) return launch_bwd<2, 4>(c, a, st);
    return c.lanes == 2 ? launch_bwd<2, 2>(c, a, st) : launch_bwd<2, 1>(c, a, st);
  }
  if (c.lanes == 4) return launch_bwd<3, 4>(c, a, st);
  return c.lanes == 2 ? launch_bwd<3, 2>(c, a, st) : launch_bwd<3, 1>(c, a, st);
}

// Co-resident workgroups of a persistent kernel at the context's block size
// (queried once per kernel, block size and lanes).
template <class K>
mpm_status persist_grid(const mpm_ctx& cc, int kind, K kernel, int* out) {
  mpm_ctx& c = const_cast<mpm_ctx&>(cc);
  const int shape = c.block * 8 + c.lanes;
  if (c.persist_grid[kind] == 0 || c.persist_grid_shape[kind] != shape) {
    int per_cu = 0, dev = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, c.block, 0));
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1 || cus < 1) return MPM_E_HIP;
    c.persist_grid[kind] = per_cu * cus;
    c.persist_grid_shape[kind] = shape;
  }
  *out = c.persist_grid[kind];
  return MPM_OK;
}

// One cooperative launch of `kernel` over the `n` recorded launches at
// `dev_seq` (kind 0 forward, 1 reverse). With the "timing" knob the launch is
// one timed span of n step launches.
template <class K>
mpm_status launch_persist(const mpm_ctx& c, int kind, K kernel, const void* dev_seq, int n, int max_blocks,
                          hipStream_t st) {
  if (n <= 0) return MPM_OK;
  int grid = 0;
  const mpm_status gs = persist_grid(c, kind, kernel, &grid);
  if (gs != MPM_OK) return gs;
  grid = std::min(grid, max_blocks);
  span_close(c);
  mpm_ctx& cm = const_cast<mpm_ctx&>(c);
  hipEvent_t e0 = nullptr;
  if (c.timing) {
    e0 = pool_event(cm);
    if (!e0 || hipEventRecord(e0, st) != hipSuccess) e0 = nullptr;
  }
  const void* seq = dev_seq;
  int nn = n;
  void* args[] = {&seq, &nn};
  HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kernel), dim3(grid), dim3(c.block), args, 0, st));
  if (e0) {
    hipEvent_t e1 = pool_event(cm);
    if (e1 && hipEventRecord(e1, st) == hipSuccess) cm.ev_pending.push_back({kind, e0, e1, long(n)});
  }
  return MPM_OK;
}

mpm_status fwd_persist(const mpm_ctx& c, const void* seq, int n, hipStream_t st) {
  const int nb = c.n_blocks;
  if (c.d == 2) {
    if (c.lanes == 4) return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<2, 4, 1>, seq, n, nb, st)
                                     : launch_persist(c, 0, mpm::k_fwd_persist<2, 4, 0>, seq, n, nb, st);
    if (c.lanes == 2) return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<2, 2, 1>, seq, n, nb, st)
                                     : launch_persist(c, 0, mpm::k_fwd_persist<2, 2, 0>, seq, n, nb, st);
    return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<2, 1, 1>, seq, n, nb, st)
                   : launch_persist(c, 0, mpm::k_fwd_persist<2, 1, 0>, seq, n, nb, st);
  }
  if (c.lanes == 4) return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<3, 4, 1>, seq, n, nb, st)
                                   : launch_persist(c, 0, mpm::k_fwd_persist<3, 4, 0>, seq, n, nb, st);
  if (c.lanes == 2) return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<3, 2, 1>, seq, n, nb, st)
                                   : launch_persist(c, 0, mpm::k_fwd_persist<3, 2, 0>, seq, n, nb, st);
  return c.model ? launch_persist(c, 0, mpm::k_fwd_persist<3, 1, 1>, seq, n, nb, st)
                 : launch_persist(c, 0, mpm::k_fwd_persist<3, 1, 0>, seq, n, nb, st);
}

mpm_status bwd_persist(const mpm_ctx& c, const void* seq, int n, hipStream_t st) {
  const int nb = 2 * c.n_blocks;
  if (c.d == 2) {
    if (c.lanes == 4) return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<2, 4, 1>, seq, n, nb, st)
                                     : launch_persist(c, 1, mpm::k_bwd_persist<2, 4, 0>, seq, n, nb, st);
    if (c.lanes == 2) return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<2, 2, 1>, seq, n, nb, st)
                                     : launch_persist(c, 1, mpm::k_bwd_persist<2, 2, 0>, seq, n, nb, st);
    return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<2, 1, 1>, seq, n, nb, st)
                   : launch_persist(c, 1, mpm::k_bwd_persist<2, 1, 0>, seq, n, nb, st);
  }
  if (c.lanes == 4) return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<3, 4, 1>, seq, n, nb, st)
                                   : launch_persist(c, 1, mpm::k_bwd_persist<3, 4, 0>, seq, n, nb, st);
  if (c.lanes == 2) return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<3, 2, 1>, seq, n, nb, st)
                                   : launch_persist(c, 1, mpm::k_bwd_persist<3, 2, 0>, seq, n, nb, st);
  return c.model ? launch_persist(c, 1, mpm::k_bwd_persist<3, 1, 1>, seq, n, nb, st)
                 : launch_persist(c, 1, mpm::k_bwd_persist<3, 1, 0>, seq, n, nb, st);
}

FwdArgs fwd_args(const mpm_ctx& c, const mpm_params* p, const mpm_tape* tp) {
  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = consts(c, p, tp);
  return a;
}

BwdArgs bwd_args(const mpm_ctx& c, const mpm_params* p, const mpm_tape* tp) {
  BwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = consts(c, p, tp);
  a.partial = c.at<float>(R_PARTIAL);
  a.pstride = c.Np;
  return a;
}

// Aligned workgroup table from the cell starts of the last sort (R_START):
// counts per parent block (into R_COUNTS, free after the sort), their scan,
// the entries, and the padding (or the plain table if it did not fit).
mpm_status build_partition(const mpm_ctx& c, int4* table, hipStream_t s) {
  const mpm::PartGeom g = part_geom(c, c.block / c.lanes);
  const long n_par = long(g.per_scene) * g.n_scenes;
  int* counts = c.at<int>(R_COUNTS);
  int* offs = c.at<int>(R_PART);
  const int pb = int((n_par + 255) / 256);
  hipLaunchKernelGGL(mpm::k_part_count, dim3(pb), dim3(256), 0, s, c.at<int>(R_START), g, counts);
  LAUNCH_TRY();
  const int nb = int((n_par + mpm::kScanChunk - 1) / mpm::kScanChunk);
  int* bsums = c.at<int>(R_BSUMS);
  hipLaunchKernelGGL(mpm::k_scan_blocks, dim3(nb), dim3(mpm::kScanThreads), 0, s, counts, offs, n_par, bsums);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_scan_sums, dim3(1), dim3(mpm::kScanThreads), 0, s, bsums, nb);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_scan_add, dim3(nb), dim3(256), 0, s, offs, n_par, bsums);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_part_emit, dim3(pb), dim3(256), 0, s, c.at<int>(R_START), g, counts, offs, c.n_blocks,
                     table);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_part_finish, dim3(1), dim3(256), 0, s, g, counts, offs, c.n_blocks, c.at<int4>(R_PLAIN),
                     c.n_plain, table);
  LAUNCH_TRY();
  return MPM_OK;
}

// Sorts particles by (scene, Morton cell) of `st` (a stable radix sort, so
// particles of one cell keep the caller's order): perm[j] = caller index of
// the j-th sorted particle. With a table, also writes the workgroup table of
// the sorted order there (the aligned partition with `part`, else the plain
// one).
mpm_status sort_particles(const mpm_ctx& c, StateRef st, int* perm, int4* table, hipStream_t s) {
  span_close(c);
  int* counts = c.at<int>(R_COUNTS);
  int* start = c.at<int>(R_START);
  int* bsums = c.at<int>(R_BSUMS);
  const long nk = c.n_keys;
  const int zb = int(std::min<long>((nk + 255) / 256, 8192));
  hipLaunchKernelGGL(mpm::k_zero_i32, dim3(zb), dim3(256), 0, s, counts, nk);
  LAUNCH_TRY();
  const int* sid = c.ns > 1 ? c.at<int>(R_SCENE_ID) : nullptr;
  const int pb = (c.N + 255) / 256;
  unsigned* keys[2] = {c.at<unsigned>(R_KEYS), c.at<unsigned>(R_KEYS2)};
  if (c.d == 2)
    hipLaunchKernelGGL(mpm::k_sort_keys<2>, dim3(pb), dim3(256), 0, s, st, c.N, sid, 1.0f / c.dx,
                       c.presum ? 0.5f : 0.0f, c.n, c.bits, c.cells_per_scene, keys[0], counts);
  else
    hipLaunchKernelGGL(mpm::k_sort_keys<3>, dim3(pb), dim3(256), 0, s, st, c.N, sid, 1.0f / c.dx,
                       c.presum ? 0.5f : 0.0f, c.n, c.bits, c.cells_per_scene, keys[0], counts);
  LAUNCH_TRY();
  // Cell starts (the partition's input).
  const int nb = int((nk + mpm::kScanChunk - 1) / mpm::kScanChunk);
  hipLaunchKernelGGL(mpm::k_scan_blocks, dim3(nb), dim3(mpm::kScanThreads), 0, s, counts, start, nk, bsums);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_scan_sums, dim3(1), dim3(mpm::kScanThreads), 0, s, bsums, nb);
  LAUNCH_TRY();
  hipLaunchKernelGGL(mpm::k_scan_add, dim3(nb), dim3(256), 0, s, start, nk, bsums);
  LAUNCH_TRY();
  // The permutation: radix passes over the key bits, the last one writing perm.
  int key_bits = 1;
  while ((1L << key_bits) < nk) ++key_bits;
  const int passes = (key_bits + mpm::kRadixBits - 1) / mpm::kRadixBits;
  const int tiles = (c.N + mpm::kRadixTile - 1) / mpm::kRadixTile;
  const long hn = long(mpm::kRadix) * tiles;
  const int hb = int((hn + mpm::kScanChunk - 1) / mpm::kScanChunk);
  int* hist = c.at<int>(R_RHIST);
  int* vals[2] = {perm, c.at<int>(R_VALS)};
  for (int q = 0; q < passes; ++q) {
    const int shift = q * mpm::kRadixBits;
    const unsigned* kin = keys[q & 1];
    unsigned* kout = keys[(q + 1) & 1];
    const int* vin = q == 0 ? nullptr : vals[(passes - q) & 1];
    int* vout = vals[(passes - 1 - q) & 1];
    hipLaunchKernelGGL(mpm::k_radix_hist, dim3(tiles), dim3(mpm::kRadixTile), 0, s, kin, c.N, shift, tiles, hist);
    LAUNCH_TRY();
    hipLaunchKernelGGL(mpm::k_scan_blocks, dim3(hb), dim3(mpm::kScanThreads), 0, s, hist, hist, hn, bsums);
    LAUNCH_TRY();
    hipLaunchKernelGGL(mpm::k_scan_sums, dim3(1), dim3(mpm::kScanThreads), 0, s, bsums, hb);
    LAUNCH_TRY();
    hipLaunchKernelGGL(mpm::k_scan_add, dim3(hb), dim3(256), 0, s, hist, hn, bsums);
    LAUNCH_TRY();
    hipLaunchKernelGGL(mpm::k_radix_scatter, dim3(tiles), dim3(mpm::kRadixTile), 0, s, kin, vin, c.N, shift, tiles,
                       hist, kout, vout);
    LAUNCH_TRY();
  }
  if (!table || !(c.ns > 1 || c.part)) return MPM_OK;
  if (c.part) return build_partition(c, table, s);
  hipLaunchKernelGGL(mpm::k_copy_i4, dim3((c.n_blocks + 255) / 256), dim3(256), 0, s, c.at<int4>(R_BLOCKS), table,
                     c.n_blocks);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status gather_state(const mpm_ctx& c, StateRef src, StateRef dst, const int* perm, hipStream_t s) {
  span_close(c);
  const int pb = (c.N + 255) / 256;
  if (c.d == 2)
    hipLaunchKernelGGL(mpm::k_gather_state<2>, dim3(pb), dim3(256), 0, s, src, dst, perm, c.N);
  else
    hipLaunchKernelGGL(mpm::k_gather_state<3>, dim3(pb), dim3(256), 0, s, src, dst, perm, c.N);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status scatter_state(const mpm_ctx& c, StateRef src, StateRef dst, const int* perm, hipStream_t s) {
  span_close(c);
  const int pb = (c.N + 255) / 256;
  if (c.d == 2)
    hipLaunchKernelGGL(mpm::k_scatter_state<2>, dim3(pb), dim3(256), 0, s, src, dst, perm, c.N);
  else
    hipLaunchKernelGGL(mpm::k_scatter_state<3>, dim3(pb), dim3(256), 0, s, src, dst, perm, c.N);
  LAUNCH_TRY();
  return MPM_OK;
}

#define TRY(expr)                    \
  do {                               \
    mpm_status st_ = (expr);         \
    if (st_ != MPM_OK) return st_;   \
  } while (0)

// Device address of `scratch` on the current device, looked up with
// hipGetSymbolAddress on the first call per device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

mpm_status scratch_on_current_device(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MPM_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPM_E_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MPM_OK;
}

// Forward steps t0 .. t1-1 from state t0 (already in its slot), writing
// states t0+1 .. t1 into their slots, using the three forward grids.
mpm_status run_forward(mpm_tape& tp, const mpm_params* p, int t0, int t1, hipStream_t s) {
  const mpm_ctx& c = *tp.ctx;
  for (int k = 0; k < 3; ++k) TRY(zero_grid(c, kGridF + k, s));
  FwdArgs a = fwd_args(c, p, &tp);
  a.in = tp.slot(t0);
  a.grid_out = c.grid(kGridF);
  a.box_out = scatter_into(c, kGridF);
  a.act_row = act_row(c, p, t0);
  a.do_p2g = 1;
  TRY(fwd(c, a, s));
  for (int t = t0; t < t1; ++t) {
    const int u = t - t0;
    FwdArgs b = fwd_args(c, p, &tp);
    b.in = tp.slot(t);
    b.out = tp.slot(t + 1);
    b.grid_in = c.grid(kGridF + u % 3);
    b.box_in = recorded_boxes(c, kGridF + u % 3);
    b.do_g2p = 1;
    b.do_p2g = (t + 1 < t1) ? 1 : 0;
    b.grid_out = c.grid(kGridF + (u + 1) % 3);
    b.act_row = act_row(c, p, t + 1);
    if (b.do_p2g) {
      // Grid (u + 2) % 3 was last read in the previous launch; it is written next launch.
      plan_clear(c, kGridF + (u + 2) % 3, b.clear, b.clear_n, b.clear_box, b.clear_nbox);
      b.box_out = scatter_into(c, kGridF + (u + 1) % 3);
    }
    TRY(fwd(c, b, s));
    if (!tp.full && (t + 1) != tp.T && (t + 1) % tp.K != 0) tp.ring_holds[(t + 1) % (2 * tp.K)] = t + 1;
  }
  return MPM_OK;
}

// Makes state `step` resident (recomputes its segment from the checkpoint).
mpm_status ensure_state(mpm_tape& tp, const mpm_params* p, int step, hipStream_t s) {
  if (tp.full || step == tp.T || step % tp.K == 0) return MPM_OK;
  if (tp.ring_holds[step % (2 * tp.K)] == step) return MPM_OK;
  const int j = step / tp.K;
  const int t0 = j * tp.K;
  const int t1 = std::min(t0 + tp.K, tp.T) - 1;  // last state of the segment kept in the ring
  return run_forward(tp, p, t0, t1, s);
}

// Workgroup table for the current block and lanes. The plain partition cuts
// each scene into runs of consecutive particles. With `part`, the launch has
// room for the aligned partition (at most twice as many workgroups, rebuilt
// on the device after each sort; trailing entries are empty workgroups), and
// the table starts as the plain one padded with empty entries, so launches
// before the first sort (single steps) are valid too.
mpm_status update_blocks(mpm_ctx& c) {
  const int per_block = c.block / c.lanes;
  std::vector<int4> t;
  for (int sc = 0; sc < c.ns; ++sc)
    for (int f = c.offsets[sc]; f < c.offsets[sc + 1]; f += per_block)
      t.push_back(make_int4(f, std::min(per_block, c.offsets[sc + 1] - f), sc, 0));
  if (t.empty()) t.push_back(make_int4(0, 0, 0, 0));
  if (t.size() * sizeof(int4) > c.bytes[R_PLAIN]) return MPM_E_CAPACITY;
  c.n_plain = int(t.size());
  if (!c.part && c.ns <= 1) {
    c.n_blocks = (c.N + per_block - 1) / per_block;
    c.blocks_host.clear();
    return MPM_OK;
  }
  c.n_blocks = c.part ? 2 * c.n_plain + 32 : c.n_plain;
  if (c.n_blocks > c.blocks_cap || c.n_blocks > c.box_cap) return MPM_E_CAPACITY;
  if (c.ws) HIP_TRY(hipMemcpy(c.at<int4>(R_PLAIN), t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
  t.resize(size_t(c.n_blocks), make_int4(0, 0, 0, 0));
  if (c.ws) HIP_TRY(hipMemcpy(c.at<int4>(R_BLOCKS), t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
  c.blocks_host = std::move(t);
  return MPM_OK;
}

bool step_fwd_args_ok(const mpm_params* params, int step, const mpm_state* in, const mpm_state* out) {
  if (!params_ok(params) || !state_ok(in) || !state_ok(out) || step < 0) return false;
  return !(in->x == out->x || in->v == out->v || in->C == out->C || in->F == out->F);
}

// Device buffers one forward step uses besides its inputs and outputs: the
// grid it scatters into and gathers from, the caller-order workgroup table
// (null when the launch needs none) and the error word.
struct StepBufs {
  float4* grid;
  const int4* table;
  unsigned* err;
  unsigned long long* tstats;  // scatter tile counters, or null
};

// One forward step in the caller's order: clear the grid, p2g, then grid_op
// folded into g2p (two launches; no box records, so the grid is cleared
// densely). `timed`: the launches may join the "timing" knob's event spans.
mpm_status enqueue_step_fwd(const mpm_ctx& c, const mpm_params* params, int step, const mpm_state* in,
                            mpm_state* out, const StepBufs& b, bool timed, hipStream_t s) {
  const long n4 = c.grid_f4();
  if (timed) span_close(c);
  hipLaunchKernelGGL(mpm::k_zero_f4, dim3(int(std::min<long>((n4 + 255) / 256, 8192))), dim3(256), 0, s, b.grid, n4);
  LAUNCH_TRY();
  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = consts(c, params, nullptr, b.table, b.err);
  a.k.tstats = b.tstats;
  a.in = user_ref(c, in);
  a.grid_out = b.grid;
  a.act_row = act_row(c, params, step);
  a.do_p2g = 1;
  TRY(fwd(c, a, s, timed));
  FwdArgs g;
  std::memset(&g, 0, sizeof(g));
  g.k = a.k;
  g.in = user_ref(c, in);
  g.out = user_ref(c, out);
  g.grid_in = b.grid;
  g.do_g2p = 1;
  return fwd(c, g, s, timed);
}

bool same_params(const mpm_params& a, const mpm_params* b) {
  return a.E == b->E && a.nu == b->nu && a.vol == b->vol && a.rho == b->rho && a.act_id == b->act_id && a.mat_id == b->mat_id &&
         a.act == b->act;
}

}  // namespace

extern "C" {

const char* mpm_status_string(mpm_status s) {
  switch (s) {
    case MPM_OK: return "ok";
    case MPM_E_ARG: return "invalid argument";
    case MPM_E_CAPACITY: return "bound memory too small";
    case MPM_E_TAPE: return "tape misuse (no recorded forward or different parameters)";
    case MPM_E_HIP: return "HIP runtime error";
    case MPM_E_DOMAIN: return "a particle stencil left the grid";
    case MPM_E_INVERTED: return "deformation gradient with det F <= 0";
    case MPM_E_NONFINITE: return "non-finite particle state";
    case MPM_E_STATE: return "workspace not bound";
    default: return "unknown status";
  }
}

mpm_status mpm_init(const mpm_desc* desc, mpm_ctx** out) {
  if (!desc || !out) return MPM_E_ARG;
  *out = nullptr;
  const mpm_desc& d = *desc;
  if (d.dim != 2 && d.dim != 3) return MPM_E_ARG;
  if (d.bound < 0 || d.n_grid < 2 * d.bound + 3 || d.n_grid > 1024) return MPM_E_ARG;
  if (!(d.dx > 0.0f) || !(d.dt > 0.0f)) return MPM_E_ARG;
  if (d.n_scenes < 1 || !d.scene_offsets) return MPM_E_ARG;
  if (d.n_actuators < 0 || d.n_actuators > mpm::kMaxAct) return MPM_E_ARG;
  if (d.flags & ~uint32_t(MPM_MODEL_COROTATED)) return MPM_E_ARG;
  if (d.scene_offsets[0] != 0) return MPM_E_ARG;
  for (int k = 0; k < d.n_scenes; ++k)
    if (d.scene_offsets[k + 1] < d.scene_offsets[k]) return MPM_E_ARG;
  const long Nl = d.scene_offsets[d.n_scenes];
  if (Nl < 1 || Nl > (1L << 28)) return MPM_E_ARG;
  long nodes = 1;
  for (int a = 0; a < d.dim; ++a) nodes *= d.n_grid;
  if (nodes * long(d.n_scenes) > (1L << 31) / 4) return MPM_E_ARG;

  mpm_ctx* c = new (std::nothrow) mpm_ctx();
  if (!c) return MPM_E_ARG;
  c->d = d.dim;
  c->n = d.n_grid;
  c->bound = d.bound;
  c->ns = d.n_scenes;
  c->n_act = d.n_actuators;
  c->model = (d.flags & MPM_MODEL_COROTATED) ? 1 : 0;
  c->N = int(Nl);
  c->Np = int(align_up(size_t(Nl), 64));
  c->S = 2 * d.dim + 2 * d.dim * d.dim;
  c->nodes = nodes;
  c->dx = d.dx;
  c->dt = d.dt;
  c->gravity = d.gravity;
  c->act_strength = d.act_strength;
  c->offsets.assign(d.scene_offsets, d.scene_offsets + d.n_scenes + 1);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      c->n_cus = cus;
    else
      (void)hipGetLastError();  // unknown: the step launches keep their clears on their own workgroups
  }
  int bits = 0;
  while ((1 << bits) < d.n_grid) ++bits;
  c->bits = bits;
  c->cells_per_scene = 1u << (bits * d.dim);
  c->n_keys = long(c->cells_per_scene) * d.n_scenes;
  if (c->n_keys > (1L << 30)) {
    delete c;
    return MPM_E_ARG;
  }

  const size_t Np = size_t(c->Np), N = size_t(c->N);
  c->bytes[R_GRID] = size_t(kNumGrids) * size_t(c->ns) * size_t(nodes) * sizeof(float4);
  c->bytes[R_PARTIAL] = size_t(d.dim + d.dim * d.dim) * Np * sizeof(float);
  c->bytes[R_SEED] = size_t(c->S) * Np * sizeof(float);
  c->bytes[R_KEYS] = N * sizeof(unsigned);
  c->bytes[R_KEYS2] = N * sizeof(unsigned);
  c->bytes[R_VALS] = N * sizeof(int);
  const size_t radix_n = size_t(mpm::kRadix) * ((N + mpm::kRadixTile - 1) / mpm::kRadixTile);
  c->bytes[R_RHIST] = radix_n * sizeof(int);
  c->bytes[R_COUNTS] = size_t(c->n_keys) * sizeof(int);
  c->bytes[R_START] = size_t(c->n_keys) * sizeof(int);
  const size_t scan_n = std::max(size_t(c->n_keys), radix_n);
  c->bytes[R_BSUMS] = size_t((scan_n + mpm::kScanChunk - 1) / mpm::kScanChunk + 1) * sizeof(int);
  c->bytes[R_SCENE_ID] = N * sizeof(int);
  c->bytes[R_OFFSETS] = size_t(c->ns + 1) * sizeof(int);
  c->bytes[R_GE] = size_t(c->ns) * sizeof(double);
  c->bytes[R_GACT] = size_t(mpm::kMaxAct) * sizeof(double);
  c->bytes[R_ERR] = sizeof(unsigned);
  c->bytes[R_TSTATS] = 2 * sizeof(unsigned long long);
  // At least 16 particles per workgroup (64 threads, 4 lanes each); the
  // aligned partition may use up to twice the plain one's workgroups.
  const size_t plain_max = N / 16 + size_t(c->ns) + 1;
  c->blocks_cap = long(2 * plain_max + 32);
  c->bytes[R_BLOCKS] = size_t(c->blocks_cap) * sizeof(int4);
  c->bytes[R_PLAIN] = plain_max * sizeof(int4);
  c->bytes[R_PART] = size_t(part_geom(*c, 16).per_scene) * size_t(c->ns) * sizeof(int);
  c->box_cap = c->blocks_cap;
  c->bytes[R_BOXES] = size_t(kNumGrids) * 2 * size_t(c->box_cap) * sizeof(int4);
  size_t o = 0;
  for (int r = 0; r < R_COUNT; ++r) {
    c->off[r] = o;
    o = align_up(o + c->bytes[r]);
  }
  c->ws_bytes = o;
  update_blocks(*c);  // host-side count only (no workspace yet)
  *out = c;
  return MPM_OK;
}

void mpm_destroy(mpm_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  delete ctx;
}

size_t mpm_workspace_bytes(const mpm_ctx* ctx) { return ctx ? ctx->ws_bytes : 0; }

mpm_status mpm_bind_workspace(mpm_ctx* ctx, void* dev, size_t bytes) {
  if (!ctx || !dev) return MPM_E_ARG;
  if (reinterpret_cast<uintptr_t>(dev) % kAlign != 0) return MPM_E_ARG;
  if (bytes < ctx->ws_bytes) return MPM_E_CAPACITY;
  ctx->ws = static_cast<char*>(dev);
  for (int g = 0; g < kNumGrids; ++g) ctx->gstate[g] = kDirty;
  std::vector<int> sid(size_t(ctx->N));
  for (int k = 0; k < ctx->ns; ++k)
    for (int p = ctx->offsets[k]; p < ctx->offsets[k + 1]; ++p) sid[size_t(p)] = k;
  HIP_TRY(hipMemcpy(ctx->at<int>(R_SCENE_ID), sid.data(), sid.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ctx->at<int>(R_OFFSETS), ctx->offsets.data(), ctx->offsets.size() * sizeof(int),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(ctx->at<unsigned>(R_ERR), 0, sizeof(unsigned)));
  HIP_TRY(hipMemset(ctx->at<unsigned long long>(R_TSTATS), 0, 2 * sizeof(unsigned long long)));
  return update_blocks(*ctx);
}

mpm_status mpm_set_knob(mpm_ctx* ctx, const char* key, int64_t value) {
  if (!ctx || !key) return MPM_E_ARG;
  const std::string k(key);
  if (k == "block") {
    if (value != 64 && value != 128 && value != 192 && value != 256) return MPM_E_ARG;
    ctx->block = int(value);
    return update_blocks(*ctx);
  }
  if (k == "lds") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->lds = int(value);
    return MPM_OK;
  }
  if (k == "lanes") {
    if (value != 1 && value != 2 && value != 4) return MPM_E_ARG;
    ctx->lanes = int(value);
    return update_blocks(*ctx);
  }
  if (k == "rotate") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->rotate = int(value);
    return MPM_OK;
  }
  if (k == "graph") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->graph = int(value);
    return MPM_OK;
  }
  if (k == "remap") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->remap = int(value);
    return MPM_OK;
  }
  if (k == "part") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->part = int(value);
    return update_blocks(*ctx);
  }
  if (k == "presum") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->presum = int(value);
    return MPM_OK;
  }
  if (k == "tile_stats") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->tile_stats = int(value);
    return MPM_OK;
  }
  if (k == "persist") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->persist = int(value);
    return MPM_OK;
  }
  if (k == "split") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->split_c = int(value);
    return MPM_OK;
  }
  if (k == "timing") {
    if (value != 0 && value != 1) return MPM_E_ARG;
    ctx->timing = value != 0;
    return MPM_OK;
  }
  return MPM_E_ARG;
}

mpm_status mpm_kernel_stats(mpm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!ctx || kernel < 0 || kernel > 1 || !total_ms || !launches) return MPM_E_ARG;
  span_close(*ctx);
  for (auto& p : ctx->ev_pending) {
    HIP_TRY(hipEventSynchronize(p.e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, p.e0, p.e1));
    ctx->ev_ms[p.kind] += ms;
    ctx->ev_count[p.kind] += p.n;
  }
  ctx->ev_pending.clear();
  ctx->ev_used = 0;
  *total_ms = ctx->ev_ms[kernel];
  *launches = ctx->ev_count[kernel];
  ctx->ev_ms[kernel] = 0.0;
  ctx->ev_count[kernel] = 0;
  return MPM_OK;
}

mpm_status mpm_step_fwd(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in, mpm_state* out,
                        void* stream) {
  if (!ctx) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  if (!step_fwd_args_ok(params, step, in, out)) return MPM_E_ARG;
  const mpm_ctx& c = *ctx;
  const SpanGuard guard(c);
  c.gstate[kGridB] = kDirty;  // written below without a box record
  const StepBufs b{c.grid(kGridB), c.at<int4>(R_BLOCKS), c.at<unsigned>(R_ERR),
                   c.tile_stats ? c.at<unsigned long long>(R_TSTATS) : nullptr};
  return enqueue_step_fwd(c, params, step, in, out, b, true, static_cast<hipStream_t>(stream));
}

mpm_status mpm_step_fwd_noalloc(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in,
                                mpm_state* out, uint32_t* err_flags, void* stream) {
  if (!ctx || !err_flags) return MPM_E_ARG;
  if (!step_fwd_args_ok(params, step, in, out)) return MPM_E_ARG;
  const mpm_ctx& c = *ctx;
  const size_t grid_bytes = align_up(size_t(c.grid_f4()) * sizeof(float4));
  const size_t table_bytes = c.blocks_host.size() * sizeof(int4);
  if (grid_bytes + table_bytes > kScratchBytes) return MPM_E_CAPACITY;
  char* base = nullptr;
  TRY(scratch_on_current_device(&base));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int4* table = reinterpret_cast<int4*>(base + grid_bytes);
  // The table of an earlier call (another context) may differ: upload this
  // context's every call, stream-ordered before the launches that read it.
  if (table_bytes) HIP_TRY(hipMemcpyAsync(table, c.blocks_host.data(), table_bytes, hipMemcpyHostToDevice, s));
  const StepBufs b{reinterpret_cast<float4*>(base), c.blocks_host.empty() ? nullptr : table,
                   reinterpret_cast<unsigned*>(err_flags), nullptr};
  return enqueue_step_fwd(c, params, step, in, out, b, false, s);
}

mpm_status mpm_step_bwd(mpm_ctx* ctx, const mpm_params* params, int32_t step, const mpm_state* in,
                        const mpm_state* out_grad, mpm_state* in_grad, mpm_param_grad* pg, void* stream) {
  if (!ctx) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  if (!params_ok(params) || !state_ok(in) || !state_ok(out_grad) || !state_ok(in_grad) || step < 0)
    return MPM_E_ARG;
  const mpm_ctx& c = *ctx;
  const SpanGuard guard(c);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float4* g = c.grid(kGridB);
  float4* ad = c.grid(kAdj);
  TRY(zero_f4(c, g, c.grid_f4(), s));
  TRY(zero_f4(c, ad, c.grid_f4(), s));
  c.gstate[kGridB] = c.gstate[kAdj] = kDirty;  // written below without a box record
  TRY(zero_f64(c.at<double>(R_GE), c.ns, s));
  TRY(zero_f64(c.at<double>(R_GACT), mpm::kMaxAct, s));
  FwdArgs a = fwd_args(c, params, nullptr);
  a.in = user_ref(c, in);
  a.grid_out = g;
  a.act_row = act_row(c, params, step);
  a.do_p2g = 1;
  TRY(fwd(c, a, s));
  // Seed -> g2p*(step): scatter into the adjoint grid, keep x*, F* partials.
  BwdArgs b = bwd_args(c, params, nullptr);
  b.a_mode = 0;
  b.seed = user_ref(c, out_grad);
  b.stB = user_ref(c, in);
  b.cnext = nullptr;
  b.gB = g;
  b.aB = ad;
  TRY(bwd(c, b, s));
  // p2g*(step) and output.
  BwdArgs e = bwd_args(c, params, nullptr);
  e.a_mode = 1;
  e.stA = user_ref(c, in);
  e.gA = g;
  e.aA = ad;
  e.act_rowA = act_row(c, params, step);
  e.gact_rowA = c.at<double>(R_GACT);
  e.gE = c.at<double>(R_GE);
  e.final_out = 1;
  e.out = user_ref(c, in_grad);
  e.out_perm = nullptr;
  TRY(bwd(c, e, s));
  span_close(c);
  if (pg && pg->E) {
    hipLaunchKernelGGL(mpm::k_add_f64_to_f32, dim3((c.ns + 255) / 256), dim3(256), 0, s, c.at<double>(R_GE), pg->E,
                       c.ns);
    LAUNCH_TRY();
  }
  if (pg && pg->act && c.n_act > 0) {
    hipLaunchKernelGGL(mpm::k_add_f64_to_f32, dim3(1), dim3(64), 0, s, c.at<double>(R_GACT),
                       pg->act + size_t(step) * c.n_act, c.n_act);
    LAUNCH_TRY();
  }
  return MPM_OK;
}

mpm_status mpm_tape_create(mpm_ctx* ctx, int32_t n_steps, int32_t ckpt_every, mpm_tape** out) {
  if (!ctx || !out || n_steps < 1 || ckpt_every < 0) return MPM_E_ARG;
  *out = nullptr;
  mpm_tape* t = new (std::nothrow) mpm_tape();
  if (!t) return MPM_E_ARG;
  t->ctx = ctx;
  t->T = n_steps;
  t->full = (ckpt_every == 0 || ckpt_every >= n_steps);
  t->K = t->full ? n_steps : ckpt_every;
  if (t->full) {
    t->n_ckpt = 1;
    t->R = std::max(n_steps - 1, 0);
  } else {
    t->n_ckpt = (n_steps - 1) / t->K + 1;
    t->R = 2 * t->K;
    t->ring_holds.assign(size_t(t->R), -1);
  }
  t->n_slots = t->n_ckpt + 1 + t->R;
  t->slot_floats = size_t(ctx->S) * size_t(ctx->Np);
  const size_t slots_bytes = align_up(size_t(t->n_slots) * t->slot_floats * sizeof(float));
  const size_t N = size_t(ctx->N);
  t->off_gact = slots_bytes;
  t->off_perm = align_up(t->off_gact + size_t(n_steps) * size_t(std::max(ctx->n_act, 1)) * sizeof(double));
  t->off_act = align_up(t->off_perm + N * sizeof(int));
  t->off_mat = align_up(t->off_act + N * sizeof(int));
  t->off_blocks = align_up(t->off_mat + N * sizeof(int));
  t->off_seq = align_up(t->off_blocks + size_t(ctx->blocks_cap) * sizeof(int4));
  // Persistent form (full tapes): the T + 1 reverse or T forward launches.
  const size_t seq_bytes = t->full ? size_t(n_steps + 1) * std::max(sizeof(FwdArgs), sizeof(BwdArgs)) : 0;
  t->total = align_up(t->off_seq + seq_bytes);
  *out = t;
  return MPM_OK;
}

size_t mpm_tape_bytes(const mpm_tape* tape) { return tape ? tape->total : 0; }

mpm_status mpm_tape_bind(mpm_tape* tape, void* dev, size_t bytes) {
  if (!tape || !dev) return MPM_E_ARG;
  if (reinterpret_cast<uintptr_t>(dev) % kAlign != 0) return MPM_E_ARG;
  if (bytes < tape->total) return MPM_E_CAPACITY;
  tape->mem = static_cast<char*>(dev);
  tape->recorded = false;
  return MPM_OK;
}

void mpm_tape_destroy(mpm_tape* tape) {
  if (!tape) return;
  for (auto& g : tape->graphs) (void)hipGraphExecDestroy(g.exec);
  delete tape;
}

}  // extern "C"

namespace {

mpm_status enqueue_tape_forward(mpm_tape* tape, const mpm_params* params, const mpm_state* init,
                                mpm_state* final_state, hipStream_t s) {
  mpm_ctx& c = *tape->ctx;
  if (!tape->full) std::fill(tape->ring_holds.begin(), tape->ring_holds.end(), -1);
  const StateRef init_ref = user_ref(c, init);
  TRY(sort_particles(c, init_ref, tape->perm(), tape->blocks(), s));
  const int* perm = tape->perm();
  TRY(gather_state(c, init_ref, tape->slot(0), perm, s));
  if (params->act_id && c.n_act > 0) {
    span_close(c);
    hipLaunchKernelGGL(mpm::k_gather_i32, dim3((c.N + 255) / 256), dim3(256), 0, s, params->act_id,
                       tape->act_ids(), perm, c.N);
    LAUNCH_TRY();
  }
  if (params->mat_id) {
    span_close(c);
    hipLaunchKernelGGL(mpm::k_gather_i32, dim3((c.N + 255) / 256), dim3(256), 0, s, params->mat_id,
                       tape->mat_ids(), perm, c.N);
    LAUNCH_TRY();
  }
  if (c.persist && tape->full) {
    // Record the step launches, upload them, run them in one persistent launch.
    tape->seq_fwd.clear();
    c.rec_fwd = &tape->seq_fwd;
    const mpm_status rs = run_forward(*tape, params, 0, tape->T, s);
    c.rec_fwd = nullptr;
    TRY(rs);
    const size_t bytes = tape->seq_fwd.size() * sizeof(FwdArgs);
    HIP_TRY(hipMemcpyAsync(tape->seq(), tape->seq_fwd.data(), bytes, hipMemcpyHostToDevice, s));
    TRY(fwd_persist(c, tape->seq(), int(tape->seq_fwd.size()), s));
  } else {
    TRY(run_forward(*tape, params, 0, tape->T, s));
  }
  TRY(scatter_state(c, tape->slot(tape->T), user_ref(c, final_state), perm, s));
  return MPM_OK;
}

mpm_status enqueue_tape_backward(mpm_tape* tape, const mpm_params* params, const mpm_state* final_grad,
                                 mpm_state* init_grad, mpm_param_grad* pg, hipStream_t s) {
  mpm_ctx& c = *tape->ctx;
  const int T = tape->T;
  const int* perm = tape->perm();
  const size_t Np = size_t(c.Np);
  float* seedb = c.at<float>(R_SEED);
  const StateRef seed{seedb, seedb + c.d * Np, seedb + 2 * c.d * Np, seedb + (2 * c.d + c.d * c.d) * Np, c.Np};
  TRY(gather_state(c, user_ref(c, final_grad), seed, perm, s));
  TRY(zero_f64(c.at<double>(R_GE), c.ns, s));
  TRY(zero_f64(tape->gact(), long(T) * std::max(c.n_act, 1), s));
  for (int k = kGridB; k < kNumGrids; ++k) TRY(zero_grid(c, k, s));

  auto iB = [](int step) { return kGridB + step % 4; };
  auto iA = [](int step) { return kAdj + step % 3; };
  auto gB = [&](int step) { return c.grid(iB(step)); };
  auto aB = [&](int step) { return c.grid(iA(step)); };

  TRY(ensure_state(*tape, params, T - 1, s));
  {
    FwdArgs a = fwd_args(c, params, tape);
    a.in = tape->slot(T - 1);
    a.grid_out = gB(T - 1);
    a.box_out = scatter_into(c, iB(T - 1));
    a.act_row = act_row(c, params, T - 1);
    a.do_p2g = 1;
    TRY(fwd(c, a, s));
  }
  const bool persist = c.persist && tape->full;
  // Recording ends when this function returns, also on an error.
  struct RecordGuard {
    mpm_ctx& c;
    ~RecordGuard() { c.rec_bwd = nullptr; }
  } record_guard{c};
  if (persist) {
    tape->seq_bwd.clear();
    c.rec_bwd = &tape->seq_bwd;
  }
  for (int st = T - 1; st >= 0; --st) {
    TRY(ensure_state(*tape, params, st, s));
    if (st >= 1) TRY(ensure_state(*tape, params, st - 1, s));
    if (st + 1 < T) TRY(ensure_state(*tape, params, st + 1, s));
    BwdArgs b = bwd_args(c, params, tape);
    if (st == T - 1) {
      b.a_mode = 0;
      b.seed = seed;
    } else {
      b.a_mode = 1;
      b.stA = tape->slot(st + 1);
      b.gA = gB(st + 1);
      b.aA = aB(st + 1);
      b.boxA_in = recorded_boxes(c, iB(st + 1));
      b.act_rowA = act_row(c, params, st + 1);
      b.gact_rowA = (c.n_act > 0) ? tape->gact() + size_t(st + 1) * c.n_act : nullptr;
      b.gE = c.at<double>(R_GE);
    }
    b.stB = tape->slot(st);
    const StateRef nx = tape->slot(st + 1);
    b.cnext = nx.C;
    b.cnext_stride = nx.stride;
    b.gB = gB(st);
    b.aB = aB(st);
    b.boxB_in = recorded_boxes(c, iB(st));
    // Grid st+2 and adjoint grid st+2 were last read by the previous launch
    // (phase A); neither is touched by this one.
    plan_clear(c, iB(st + 2), b.clear0, b.clear0_n, b.clear0_box, b.clear0_nbox);
    plan_clear(c, iA(st + 2), b.clear1, b.clear1_n, b.clear1_box, b.clear1_nbox);
    b.boxB = scatter_into(c, iA(st));
    if (st >= 1) {
      b.do_c = 1;
      b.split_c = c.split_c;
      b.stC = tape->slot(st - 1);
      b.act_rowC = act_row(c, params, st - 1);
      b.gC = gB(st - 1);
      b.boxC = scatter_into(c, iB(st - 1));
    }
    TRY(bwd(c, b, s));
  }
  {
    BwdArgs b = bwd_args(c, params, tape);
    b.a_mode = 1;
    b.stA = tape->slot(0);
    b.gA = gB(0);
    b.aA = aB(0);
    b.boxA_in = recorded_boxes(c, iB(0));
    b.act_rowA = act_row(c, params, 0);
    b.gact_rowA = (c.n_act > 0) ? tape->gact() : nullptr;
    b.gE = c.at<double>(R_GE);
    b.final_out = 1;
    b.out = user_ref(c, init_grad);
    b.out_perm = perm;
    const mpm_status bs = bwd(c, b, s);
    c.rec_bwd = nullptr;
    TRY(bs);
  }
  if (persist) {
    const size_t bytes = tape->seq_bwd.size() * sizeof(BwdArgs);
    HIP_TRY(hipMemcpyAsync(tape->seq(), tape->seq_bwd.data(), bytes, hipMemcpyHostToDevice, s));
    TRY(bwd_persist(c, tape->seq(), int(tape->seq_bwd.size()), s));
  }
  span_close(c);
  if (pg && pg->E) {
    hipLaunchKernelGGL(mpm::k_add_f64_to_f32, dim3((c.ns + 255) / 256), dim3(256), 0, s, c.at<double>(R_GE), pg->E,
                       c.ns);
    LAUNCH_TRY();
  }
  if (pg && pg->act && c.n_act > 0) {
    const int n = T * c.n_act;
    hipLaunchKernelGGL(mpm::k_add_f64_to_f32, dim3((n + 255) / 256), dim3(256), 0, s, tape->gact(), pg->act, n);
    LAUNCH_TRY();
  }
  return MPM_OK;
}

void push_state_key(std::vector<uintptr_t>& k, const mpm_state* st) {
  k.push_back(reinterpret_cast<uintptr_t>(st ? st->x : nullptr));
  k.push_back(reinterpret_cast<uintptr_t>(st ? st->v : nullptr));
  k.push_back(reinterpret_cast<uintptr_t>(st ? st->C : nullptr));
  k.push_back(reinterpret_cast<uintptr_t>(st ? st->F : nullptr));
}

std::vector<uintptr_t> graph_key(const mpm_tape* tape, int kind, const mpm_params* p, const mpm_state* a,
                                 const mpm_state* b, const mpm_param_grad* pg) {
  const mpm_ctx& c = *tape->ctx;
  std::vector<uintptr_t> k = {uintptr_t(kind), reinterpret_cast<uintptr_t>(c.ws), reinterpret_cast<uintptr_t>(tape->mem),
                              uintptr_t(c.block), uintptr_t(c.lds), uintptr_t(c.split_c), uintptr_t(c.remap), uintptr_t(c.rotate), uintptr_t(c.lanes),
                              uintptr_t(c.part), uintptr_t(c.presum), reinterpret_cast<uintptr_t>(c.clk),
                              uintptr_t(c.clk_epoch),
                              reinterpret_cast<uintptr_t>(p->E), reinterpret_cast<uintptr_t>(p->nu),
                              reinterpret_cast<uintptr_t>(p->vol), reinterpret_cast<uintptr_t>(p->rho),
                              reinterpret_cast<uintptr_t>(p->act_id), reinterpret_cast<uintptr_t>(p->act),
                              reinterpret_cast<uintptr_t>(p->mat_id),
                              reinterpret_cast<uintptr_t>(pg ? pg->E : nullptr),
                              reinterpret_cast<uintptr_t>(pg ? pg->act : nullptr)};
  push_state_key(k, a);
  push_state_key(k, b);
  for (int r : tape->ring_holds) k.push_back(uintptr_t(uint32_t(r)));
  return k;
}

// Runs `enqueue(stream)` directly, or through a captured graph replayed on
// `s` (captured on first use on the context's own stream).
template <class Fn>
mpm_status run_graphed(mpm_tape* tape, std::vector<uintptr_t> key, hipStream_t s, Fn&& enqueue) {
  mpm_ctx& c = *tape->ctx;
  if (!c.graph || c.timing || c.persist) return enqueue(s);
  for (auto& g : tape->graphs) {
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, s));
      tape->ring_holds = g.ring_after;
      return MPM_OK;
    }
  }
  if (!c.capture) HIP_TRY(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(c.capture, hipStreamCaptureModeThreadLocal));
  const mpm_status st = enqueue(c.capture);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c.capture, &graph);
  if (st != MPM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess || !graph) return MPM_E_HIP;
  mpm_tape::Graph g;
  g.key = std::move(key);
  const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return MPM_E_HIP;
  g.ring_after = tape->ring_holds;
  if (tape->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(tape->graphs.front().exec);
    tape->graphs.erase(tape->graphs.begin());
  }
  tape->graphs.push_back(std::move(g));
  HIP_TRY(hipGraphLaunch(tape->graphs.back().exec, s));
  return MPM_OK;
}

}  // namespace

extern "C" {

mpm_status mpm_tape_forward(mpm_tape* tape, const mpm_params* params, const mpm_state* init, mpm_state* final_state,
                            void* stream) {
  if (!tape || !params_ok(params) || !state_ok(init) || !state_ok(final_state)) return MPM_E_ARG;
  if (!tape->mem) return MPM_E_TAPE;
  if (!tape->ctx->ws) return MPM_E_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SpanGuard guard(*tape->ctx);
  tape->recorded = false;
  if (!tape->full) std::fill(tape->ring_holds.begin(), tape->ring_holds.end(), -1);
  TRY(run_graphed(tape, graph_key(tape, 0, params, init, final_state, nullptr), s,
                  [&](hipStream_t cs) { return enqueue_tape_forward(tape, params, init, final_state, cs); }));
  tape->rec = *params;
  tape->rec_block = tape->ctx->block;
  tape->rec_lanes = tape->ctx->lanes;
  tape->rec_part = tape->ctx->part;
  tape->rec_presum = tape->ctx->presum;
  tape->recorded = true;
  return MPM_OK;
}

mpm_status mpm_tape_backward(mpm_tape* tape, const mpm_params* params, const mpm_state* final_grad,
                             mpm_state* init_grad, mpm_param_grad* pg, void* stream) {
  if (!tape || !params_ok(params) || !state_ok(final_grad) || !state_ok(init_grad)) return MPM_E_ARG;
  if (!tape->mem || !tape->recorded || !same_params(tape->rec, params)) return MPM_E_TAPE;
  const mpm_ctx& cx = *tape->ctx;
  if (cx.block != tape->rec_block || cx.lanes != tape->rec_lanes || cx.part != tape->rec_part ||
      cx.presum != tape->rec_presum)
    return MPM_E_TAPE;
  if (!tape->ctx->ws) return MPM_E_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SpanGuard guard(*tape->ctx);
  return run_graphed(tape, graph_key(tape, 1, params, final_grad, init_grad, pg), s,
                     [&](hipStream_t cs) { return enqueue_tape_backward(tape, params, final_grad, init_grad, pg, cs); });
}

mpm_status mpm_sort_order(mpm_ctx* ctx, const mpm_state* state, int32_t* perm, void* stream) {
  if (!ctx || !state_ok(state) || !perm) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  const SpanGuard guard(*ctx);
  return sort_particles(*ctx, user_ref(*ctx, state), perm, nullptr, static_cast<hipStream_t>(stream));
}

mpm_status mpm_loss(mpm_ctx* ctx, int32_t kind, int32_t axis, float sign, const mpm_state* final_state,
                    float* loss_dev, mpm_state* seed, void* stream) {
  if (!ctx || kind != MPM_LOSS_MEAN_POS || !state_ok(final_state) || !loss_dev) return MPM_E_ARG;
  if (axis < 0 || axis >= ctx->d) return MPM_E_ARG;
  if (seed && !state_ok(seed)) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  const mpm_ctx& c = *ctx;
  hipStream_t s = static_cast<hipStream_t>(stream);
  StateRef sd{nullptr, nullptr, nullptr, nullptr, c.N};
  if (seed) sd = user_ref(c, seed);
  if (c.d == 2)
    hipLaunchKernelGGL(mpm::k_loss_mean<2>, dim3(c.ns), dim3(1024), 0, s, user_ref(c, final_state),
                       c.at<int>(R_OFFSETS), axis, sign, loss_dev);
  else
    hipLaunchKernelGGL(mpm::k_loss_mean<3>, dim3(c.ns), dim3(1024), 0, s, user_ref(c, final_state),
                       c.at<int>(R_OFFSETS), axis, sign, loss_dev);
  LAUNCH_TRY();
  if (seed && c.N > 0) {
    const int pb = (c.N + 255) / 256;
    if (c.d == 2)
      hipLaunchKernelGGL(mpm::k_loss_seed<2>, dim3(pb), dim3(256), 0, s, c.at<int>(R_OFFSETS), c.ns, c.N, axis, sign,
                         sd);
    else
      hipLaunchKernelGGL(mpm::k_loss_seed<3>, dim3(pb), dim3(256), 0, s, c.at<int>(R_OFFSETS), c.ns, c.N, axis, sign,
                         sd);
    LAUNCH_TRY();
  }
  return MPM_OK;
}

mpm_status mpm_actuation(mpm_ctx* ctx, const float* W, const float* b, int32_t n_sin, float omega, int32_t n_steps,
                         float* act, void* stream) {
  if (!ctx || !W || !b || !act || n_sin < 1 || n_steps < 1 || ctx->n_act < 1) return MPM_E_ARG;
  const int n = n_steps * ctx->n_act;
  hipLaunchKernelGGL(mpm::k_actuation, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), W, b,
                     ctx->n_act, n_sin, omega, ctx->dt, n_steps, act);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status mpm_actuation_bwd(mpm_ctx* ctx, const float* W, const float* b, int32_t n_sin, float omega,
                             int32_t n_steps, const float* gact, float* gW, float* gb, void* stream) {
  if (!ctx || !W || !b || !gact || !gW || !gb || n_sin < 1 || n_steps < 1 || ctx->n_act < 1) return MPM_E_ARG;
  const int n = ctx->n_act * (n_sin + 1);
  hipLaunchKernelGGL(mpm::k_actuation_bwd, dim3((n + 63) / 64), dim3(64), 0, static_cast<hipStream_t>(stream), W, b,
                     ctx->n_act, n_sin, omega, ctx->dt, n_steps, gact, gW, gb);
  LAUNCH_TRY();
  return MPM_OK;
}

mpm_status mpm_tile_stats(mpm_ctx* ctx, void* stream, int64_t* lds_scatters, int64_t* fallback_scatters) {
  if (!ctx || !lds_scatters || !fallback_scatters) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  unsigned long long v[2] = {0, 0};
  HIP_TRY(hipMemcpy(v, ctx->at<unsigned long long>(R_TSTATS), sizeof(v), hipMemcpyDeviceToHost));
  const unsigned long long zero[2] = {0, 0};
  HIP_TRY(hipMemcpy(ctx->at<unsigned long long>(R_TSTATS), zero, sizeof(zero), hipMemcpyHostToDevice));
  *lds_scatters = int64_t(v[0]);
  *fallback_scatters = int64_t(v[1]);
  return MPM_OK;
}

mpm_status mpm_wg_clock_bind(mpm_ctx* ctx, void* buf, size_t bytes) {
  if (!ctx) return MPM_E_ARG;
  ctx->clk_next = 0;
  ctx->clk_kind.clear();
  ctx->clk_wgs.clear();
  ++ctx->clk_epoch;
  if (!buf) {
    ctx->clk = nullptr;
    ctx->clk_slots = 0;
    return MPM_OK;
  }
  if (ctx->n_blocks <= 0) return MPM_E_STATE;
  const int stride = 2 * ctx->n_blocks;
  const size_t row = size_t(stride) * 2 * sizeof(unsigned long long);
  if (bytes < row || reinterpret_cast<uintptr_t>(buf) % 8) return MPM_E_ARG;
  ctx->clk = static_cast<unsigned long long*>(buf);
  ctx->clk_stride = stride;
  ctx->clk_slots = long(bytes / row);
  return MPM_OK;
}

mpm_status mpm_wg_clock_info(const mpm_ctx* ctx, int32_t* launches, int32_t* stride, int32_t* kind, int32_t* wgs,
                             int32_t max_rows, int32_t* rate_khz) {
  if (!ctx) return MPM_E_ARG;
  if (launches) *launches = ctx->clk_next;
  if (stride) *stride = ctx->clk ? ctx->clk_stride : 2 * ctx->n_blocks;
  const int n = std::min<int>(std::max<int>(max_rows, 0), ctx->clk_next);
  for (int r = 0; r < n; ++r) {
    if (kind) kind[r] = ctx->clk_kind[r];
    if (wgs) wgs[r] = ctx->clk_wgs[r];
  }
  if (rate_khz) {
    int dev = 0, rate = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
    *rate_khz = rate;
  }
  return MPM_OK;
}

mpm_status mpm_check_errors(mpm_ctx* ctx, void* stream, uint32_t* flags) {
  if (!ctx) return MPM_E_ARG;
  if (!ctx->ws) return MPM_E_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  unsigned v = 0;
  HIP_TRY(hipMemcpy(&v, ctx->at<unsigned>(R_ERR), sizeof(unsigned), hipMemcpyDeviceToHost));
  const unsigned zero = 0;
  HIP_TRY(hipMemcpy(ctx->at<unsigned>(R_ERR), &zero, sizeof(unsigned), hipMemcpyHostToDevice));
  if (flags) *flags = v;
  if (v & MPM_FLAG_DOMAIN) return MPM_E_DOMAIN;
  if (v & MPM_FLAG_INVERTED) return MPM_E_INVERTED;
  if (v & MPM_FLAG_NONFINITE) return MPM_E_NONFINITE;
  return MPM_OK;
}

}  // extern "C"

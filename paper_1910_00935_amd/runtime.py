"""Torch-facing runtime over the C ABI: contexts, states, tapes, and a
``torch.autograd.Function`` over whole trajectories.

PyTorch only provides device memory (workspace, tape, states) and the stream;
all simulation work is in the HIP library. States are component-major
tensors: ``x, v`` of shape (d, N) and ``C, F`` of shape (d, d, N), float32,
contiguous, on the GPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _dev_bytes(nbytes: int, device) -> torch.Tensor:
    # The caching allocator returns blocks aligned to at least 512 bytes.
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


@dataclass
class State:
    """Particle state, component-major: x, v (d, N); C, F (d, d, N)."""
    x: torch.Tensor
    v: torch.Tensor
    C: torch.Tensor
    F: torch.Tensor

    def c(self) -> L.mpm_state:
        for t in (self.x, self.v, self.C, self.F):
            assert t.is_contiguous() and t.dtype == torch.float32 and t.is_cuda
        return L.mpm_state(self.x.data_ptr(), self.v.data_ptr(), self.C.data_ptr(), self.F.data_ptr())

    @staticmethod
    def empty(dim, N, device="cuda") -> "State":
        return State(torch.empty(dim, N, device=device), torch.empty(dim, N, device=device),
                     torch.empty(dim, dim, N, device=device), torch.empty(dim, dim, N, device=device))

    @staticmethod
    def zeros(dim, N, device="cuda") -> "State":
        return State(torch.zeros(dim, N, device=device), torch.zeros(dim, N, device=device),
                     torch.zeros(dim, dim, N, device=device), torch.zeros(dim, dim, N, device=device))

    @staticmethod
    def from_particle_major(x, v, C, F, device="cuda") -> "State":
        """From (N,d), (N,d), (N,d,d), (N,d,d) arrays (NumPy or torch)."""
        def t(a):
            return torch.as_tensor(np.asarray(a, dtype=np.float32) if not torch.is_tensor(a) else a,
                                   dtype=torch.float32)
        x, v, C, F = t(x), t(v), t(C), t(F)
        return State(x.t().contiguous().to(device), v.t().contiguous().to(device),
                     C.permute(1, 2, 0).contiguous().to(device), F.permute(1, 2, 0).contiguous().to(device))

    def to_particle_major(self):
        """(N,d), (N,d), (N,d,d), (N,d,d) float64 NumPy arrays."""
        def n(a):
            return a.detach().cpu().numpy().astype(np.float64)
        return (n(self.x).T.copy(), n(self.v).T.copy(), np.transpose(n(self.C), (2, 0, 1)).copy(),
                np.transpose(n(self.F), (2, 0, 1)).copy())

    def tensors(self):
        return self.x, self.v, self.C, self.F


@dataclass
class Params:
    E: torch.Tensor
    nu: torch.Tensor
    vol: torch.Tensor
    rho: torch.Tensor
    act_id: Optional[torch.Tensor] = None
    act: Optional[torch.Tensor] = None
    mat_id: Optional[torch.Tensor] = None

    def c(self) -> L.mpm_params:
        return L.mpm_params(_ptr(self.E), _ptr(self.nu), _ptr(self.vol), _ptr(self.rho), _ptr(self.act_id),
                            _ptr(self.act), _ptr(self.mat_id))


# The library's knob defaults (mpm_set_knob in mpm.h), for comparing launch
# configurations given as partial dicts.
DEFAULT_KNOBS = {"block": 128, "lanes": 1, "part": 1, "rotate": 1, "lds": 1, "split": 1, "remap": 0}


def effective_knobs(knobs: Optional[dict]) -> dict:
    """The full launch configuration a partial knob dict selects."""
    return {**DEFAULT_KNOBS, **(knobs or {})}


class Simulator:
    """One context: a description (grid, time step, scenes) plus bound workspace."""

    def __init__(self, dim, n_grid, dx, dt, scene_offsets, gravity=-9.8, bound=3, n_actuators=0,
                 act_strength=0.0, device="cuda", knobs: Optional[dict] = None, model: int = 0,
                 workspace: bool = True):
        self.dim, self.n_grid, self.dx, self.dt = int(dim), int(n_grid), float(dx), float(dt)
        self.offsets = np.ascontiguousarray(scene_offsets, dtype=np.int32)
        self.n_scenes = len(self.offsets) - 1
        self.N = int(self.offsets[-1])
        self.n_act = int(n_actuators)
        self.device = device
        self._off_c = self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        desc = L.mpm_desc(self.dim, self.n_grid, int(bound), self.dx, self.dt, float(gravity), self.n_scenes,
                          self._off_c, self.n_act, float(act_strength),
                          L.MPM_MODEL_COROTATED if model == 1 else 0)
        self.ctx = L.mpm_init(desc)
        # workspace=False: no device memory is bound; only step_fwd_noalloc
        # (mpm_step_fwd_noalloc) can run on such a context.
        self.workspace = None
        if workspace:
            self.workspace = _dev_bytes(L.mpm_workspace_bytes(self.ctx), device)
            L.mpm_bind_workspace(self.ctx, self.workspace.data_ptr(), self.workspace.numel())
        for k, v in (knobs or {}).items():
            L.mpm_set_knob(self.ctx, k, v)

    @staticmethod
    def for_scene(scene, device="cuda", knobs=None, workspace: bool = True) -> "Simulator":
        return Simulator(scene.dim, scene.n_grid, scene.dx, scene.dt, scene.offsets, gravity=scene.gravity,
                         bound=scene.bound, n_actuators=scene.n_act, act_strength=scene.act_strength,
                         device=device, knobs=knobs, model=int(getattr(scene, "model", 0) or 0),
                         workspace=workspace)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value and L is not None and L._lib is not None:
            L.mpm_destroy(ctx)
            self.ctx = None

    def set_knob(self, key, value):
        L.mpm_set_knob(self.ctx, key, value)

    # Single steps (caller particle order).
    def step_fwd(self, params: Params, step: int, s_in: State, s_out: State):
        L.mpm_step_fwd(self.ctx, params.c(), step, s_in.c(), s_out.c(), _stream())

    def step_fwd_noalloc(self, params: Params, step: int, s_in: State, s_out: State, err_flags: torch.Tensor):
        """mpm_step_fwd without workspace: the library's fixed device array
        holds the grid; error bits are OR-ed into err_flags (int32 [1])."""
        assert err_flags.dtype == torch.int32 and err_flags.is_cuda and err_flags.numel() >= 1
        L.mpm_step_fwd_noalloc(self.ctx, params.c(), step, s_in.c(), s_out.c(), err_flags.data_ptr(), _stream())

    def step_bwd(self, params: Params, step: int, s_in: State, out_grad: State, in_grad: State,
                 gE: Optional[torch.Tensor] = None, gact: Optional[torch.Tensor] = None):
        pg = L.mpm_param_grad(_ptr(gE), _ptr(gact))
        L.mpm_step_bwd(self.ctx, params.c(), step, s_in.c(), out_grad.c(), in_grad.c(), pg, _stream())

    def tape(self, n_steps: int, ckpt_every: int = 0) -> "Tape":
        return Tape(self, n_steps, ckpt_every)

    def sort_order(self, state: State) -> torch.Tensor:
        """The order in which a tape keeps the particles of `state`: int32 [N],
        entry j = caller index of the j-th particle (mpm_sort_order)."""
        perm = torch.empty(self.N, dtype=torch.int32, device=self.device)
        L.mpm_sort_order(self.ctx, state.c(), perm.data_ptr(), _stream())
        return perm

    def loss_mean(self, final: State, axis: int, sign: float = 1.0, seed: Optional[State] = None):
        loss = torch.empty(self.n_scenes, device=self.device)
        L.mpm_loss(self.ctx, L.MPM_LOSS_MEAN_POS, axis, sign, final.c(), loss.data_ptr(),
                   None if seed is None else seed.c(), _stream())
        return loss

    def actuation(self, W: torch.Tensor, b: torch.Tensor, omega: float, n_steps: int) -> torch.Tensor:
        act = torch.empty(n_steps, self.n_act, device=self.device)
        L.mpm_actuation(self.ctx, W.data_ptr(), b.data_ptr(), W.shape[1], omega, n_steps, act.data_ptr(), _stream())
        return act

    def actuation_bwd(self, W, b, omega, n_steps, gact, gW, gb):
        L.mpm_actuation_bwd(self.ctx, W.data_ptr(), b.data_ptr(), W.shape[1], omega, n_steps, gact.data_ptr(),
                            gW.data_ptr(), gb.data_ptr(), _stream())

    def tile_stats(self):
        """(LDS-tile scatters, fallback scatters) since the last call (knob "tile_stats")."""
        return L.mpm_tile_stats(self.ctx, _stream())

    def bind_wg_clock(self, buf):
        """Workgroup wall clocks of the following step launches into `buf` (a
        CUDA int64 tensor, kept by the simulator), or off with None."""
        self._clk = buf
        if buf is None:
            L.mpm_wg_clock_bind(self.ctx, 0, 0)
        else:
            L.mpm_wg_clock_bind(self.ctx, buf.data_ptr(), buf.numel() * buf.element_size())

    def wg_clock_buffer(self, rows):
        """A zeroed device buffer for `rows` launches of workgroup wall clocks."""
        stride = L.mpm_wg_clock_info(self.ctx)[2]
        return torch.zeros(rows * stride * 2, dtype=torch.int64, device="cuda")

    def wg_clock(self):
        """Rows taken since bind_wg_clock, in enqueue order: (kind, start, end)
        with the start and end of every workgroup in microseconds (numpy)."""
        kinds, wgs, stride, rate = L.mpm_wg_clock_info(self.ctx)
        if getattr(self, "_clk", None) is None or not kinds:
            return []
        torch.cuda.synchronize()
        a = self._clk[: len(kinds) * stride * 2].view(len(kinds), stride, 2).cpu().numpy()
        us = 1e3 / rate
        return [(k, a[r, :w, 0] * us, a[r, :w, 1] * us) for r, (k, w) in enumerate(zip(kinds, wgs))]

    def check_errors(self):
        """Synchronises and returns the device error flags (MPM_FLAG_* bits)."""
        st, flags = L.mpm_check_errors(self.ctx, _stream())
        return flags


class Tape:
    """Trajectory tape (full, or checkpointed every `ckpt_every` steps)."""

    def __init__(self, sim: Simulator, n_steps: int, ckpt_every: int = 0):
        self.sim = sim
        self.n_steps = int(n_steps)
        self.ckpt_every = int(ckpt_every)
        self.h = L.mpm_tape_create(sim.ctx, self.n_steps, self.ckpt_every)
        self.generation = 0  # forwards run on this tape (each replaces the recorded trajectory)
        self.nbytes = L.mpm_tape_bytes(self.h)
        self.mem = _dev_bytes(self.nbytes, sim.device)
        L.mpm_tape_bind(self.h, self.mem.data_ptr(), self.nbytes)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and L is not None and L._lib is not None:
            L.mpm_tape_destroy(h)
            self.h = None

    def forward(self, params: Params, init: State, final: State):
        L.mpm_tape_forward(self.h, params.c(), init.c(), final.c(), _stream())
        self.generation += 1

    def backward(self, params: Params, final_grad: State, init_grad: State, gE: Optional[torch.Tensor] = None,
                 gact: Optional[torch.Tensor] = None):
        pg = L.mpm_param_grad(_ptr(gE), _ptr(gact))
        L.mpm_tape_backward(self.h, params.c(), final_grad.c(), init_grad.c(), pg, _stream())


def params_for_scene(scene, device="cuda", act: Optional[torch.Tensor] = None) -> Params:
    def f(a):
        return torch.as_tensor(np.asarray(a, np.float32), device=device)
    act_id = None
    if scene.act_id is not None:
        act_id = torch.as_tensor(np.asarray(scene.act_id, np.int32), device=device)
    mat_id = None
    if getattr(scene, "mat_id", None) is not None:
        mat_id = torch.as_tensor(np.asarray(scene.mat_id, np.int32), device=device)
    return Params(f(scene.E), f(scene.nu), f(scene.vol), f(scene.rho), act_id, act, mat_id)


def state_for_scene(scene, device="cuda") -> State:
    return State.from_particle_major(scene.x, scene.v, scene.C, scene.F, device=device)


class MPMTrajectory(torch.autograd.Function):
    """Differentiable trajectory: (x0, v0, C0, F0, E, act) -> (xT, vT, CT, FT).

    ``params`` supplies the parameters that are not differentiated (nu, vol,
    rho, act_id, mat_id); its E and act are replaced by the E and act inputs.
    The forward runs the tape; the backward replays it in reverse (with
    segment recompute when the tape is checkpointed) and returns gradients for
    the initial state, E and the actuation table. A tape records one
    trajectory: if it is run forward again before this trajectory's backward,
    the backward raises instead of returning another trajectory's gradients."""

    @staticmethod
    def forward(ctx, tape: Tape, params: Params, x0, v0, C0, F0, E, act):
        sim = tape.sim
        p = Params(E.detach().contiguous(), params.nu, params.vol, params.rho, params.act_id,
                   None if act is None else act.detach().contiguous(), params.mat_id)
        init = State(x0.detach().contiguous(), v0.detach().contiguous(), C0.detach().contiguous(),
                     F0.detach().contiguous())
        final = State.empty(sim.dim, sim.N, sim.device)
        tape.forward(p, init, final)
        ctx.tape = tape
        ctx.generation = tape.generation
        ctx.params = p
        ctx.init = init
        ctx.has_act = act is not None
        return final.x, final.v, final.C, final.F

    @staticmethod
    def backward(ctx, gx, gv, gC, gF):
        tape, sim = ctx.tape, ctx.tape.sim
        if tape.generation != ctx.generation:
            raise RuntimeError("the tape of this trajectory was run forward again before its backward; "
                               "use one tape per trajectory that is differentiated")

        def z(g, like):
            return torch.zeros_like(like) if g is None else g.contiguous()

        fg = State(z(gx, ctx.init.x), z(gv, ctx.init.v), z(gC, ctx.init.C), z(gF, ctx.init.F))
        ig = State.zeros(sim.dim, sim.N, sim.device)
        gE = torch.zeros_like(ctx.params.E)
        gact = torch.zeros_like(ctx.params.act) if ctx.has_act else None
        tape.backward(ctx.params, fg, ig, gE, gact)
        return (None, None, ig.x, ig.v, ig.C, ig.F, gE, gact)


class Actuation(torch.autograd.Function):
    """a[s, k] = tanh(sum_j W[k, j] sin(omega s dt + 2 pi j / n_sin) + b[k]) on the GPU."""

    @staticmethod
    def forward(ctx, sim: Simulator, W, b, omega: float, n_steps: int):
        W = W.detach().contiguous()
        b = b.detach().contiguous()
        ctx.sim, ctx.W, ctx.b, ctx.omega, ctx.n_steps = sim, W, b, omega, n_steps
        return sim.actuation(W, b, omega, n_steps)

    @staticmethod
    def backward(ctx, gact):
        gW = torch.zeros_like(ctx.W)
        gb = torch.zeros_like(ctx.b)
        ctx.sim.actuation_bwd(ctx.W, ctx.b, ctx.omega, ctx.n_steps, gact.contiguous(), gW, gb)
        return None, gW, gb, None, None


def trajectory(tape: Tape, init: State, params: Params, act: Optional[torch.Tensor] = None):
    """Differentiable final state of `tape.n_steps` steps (all of `params`,
    material ids included, reach the tape; E and act are differentiated)."""
    return MPMTrajectory.apply(tape, params, init.x, init.v, init.C, init.F, params.E,
                               params.act if act is None else act)


class SmokeSim:
    """The incompressible smoke simulator (include/smoke.h) over torch memory:
    a tape of steps + 1 states, each a (3, n, n) float32 tensor [u0, u1, s],
    and a workspace. Every step runs in the HIP library."""

    def __init__(self, n: int, steps: int, iters: int, tile: int = 0, device="cuda"):
        self.desc = L.smoke_desc(int(n), int(steps), int(iters), int(tile))
        self.n, self.steps, self.iters = int(n), int(steps), int(iters)
        self.device = device
        nb = L.smoke_tape_bytes(self.desc)
        if nb == 0:
            raise ValueError(f"invalid smoke description n={n} steps={steps} iters={iters} tile={tile}")
        self.tape = torch.empty(self.steps + 1, 3, self.n, self.n, device=device)
        self.workspace = _dev_bytes(L.smoke_workspace_bytes(self.desc), device)
        L.smoke_workspace_init(self.desc, self.workspace.data_ptr(), _stream())

    @staticmethod
    def for_scene(scene, tile: int = 0, device="cuda") -> "SmokeSim":
        return SmokeSim(scene.n, scene.steps, scene.iters, tile, device)

    def forward(self, init: torch.Tensor) -> torch.Tensor:
        """Runs the trajectory from `init` (3, n, n); returns the final state (a view of the tape)."""
        assert init.shape == (3, self.n, self.n) and init.dtype == torch.float32 and init.is_contiguous()
        L.smoke_forward(self.desc, init.data_ptr(), self.tape.data_ptr(), self.workspace.data_ptr(), _stream())
        return self.tape[self.steps]

    def loss(self, target: torch.Tensor, seed: Optional[torch.Tensor] = None) -> torch.Tensor:
        """sum (s_T - target)^2 as a one-element tensor; fills `seed` with dL/d(state T) if given."""
        loss = torch.empty(1, device=self.device)
        L.smoke_loss(self.desc, self.tape.data_ptr(), target.contiguous().data_ptr(), loss.data_ptr(),
                     _ptr(seed), self.workspace.data_ptr(), _stream())
        return loss

    def backward(self, seed: torch.Tensor, grad: torch.Tensor):
        """ADDS dL/d(state 0) into grad (3, n, n) given seed = dL/d(state T)."""
        for t in (seed, grad):
            assert t.shape == (3, self.n, self.n) and t.dtype == torch.float32 and t.is_contiguous()
        L.smoke_backward(self.desc, self.tape.data_ptr(), seed.data_ptr(), grad.data_ptr(),
                         self.workspace.data_ptr(), _stream())

    def check_errors(self) -> int:
        st, flags = L.smoke_check_errors(self.desc, self.workspace.data_ptr(), _stream())
        return flags


def smoke_state(scene, device="cuda") -> torch.Tensor:
    """Initial state (3, n, n) [u0, u1, s] of a SmokeScene."""
    return torch.as_tensor(np.stack([scene.u0, scene.u1, scene.s]), dtype=torch.float32, device=device).contiguous()

"""FP64 CPU oracle of the differentiable MLS-MPM step (DiffTaichi, Section 4.1
and Appendix D) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module. It wraps ``liboracle.so`` (built from
``mpm_oracle.cpp`` with g++, no fast-math) through ctypes, and adds the two
pieces that are plain NumPy: the open-loop actuation signal of the 2D soft
robot and its adjoint.

Scenes are described by any object with the attributes ``dim, n_grid, bound,
dx, dt, gravity, offsets, E, nu, vol, rho, act_id, n_act, act_strength`` and
optionally ``model`` (0 neo-Hookean, 1 fixed-corotated) and ``mat_id`` (per
particle, 1 for the weakly compressible liquid; duck-typed, so this module
imports nothing from the GPU package).

State layout here: ``x (N, d), v (N, d), C (N, d, d), F (N, d, d)`` float64,
packed particle-major into one (N, S) array with S = 2d + 2d^2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpm_oracle.cpp")
_SO = os.path.join(_HERE, "liboracle.so")

ERR_DOMAIN, ERR_INVERTED, ERR_NONFINITE = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP64, -O2, strict IEEE)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-shared", "-fPIC",
             "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


class _Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_grid", ctypes.c_int), ("bound", ctypes.c_int),
        ("n_scenes", ctypes.c_int), ("n_act", ctypes.c_int),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("gravity", ctypes.c_double),
        ("act_strength", ctypes.c_double),
        ("offsets", ctypes.POINTER(ctypes.c_int)),
        ("E", ctypes.POINTER(ctypes.c_double)), ("nu", ctypes.POINTER(ctypes.c_double)),
        ("vol", ctypes.POINTER(ctypes.c_double)), ("rho", ctypes.POINTER(ctypes.c_double)),
        ("act_id", ctypes.POINTER(ctypes.c_int)),
        ("model", ctypes.c_int),
        ("mat_id", ctypes.POINTER(ctypes.c_int)),
    ]


_lib = None
_override = None


def use_library(path=None):
    """Point this module at another build of the oracle (a copy with a planted
    mistake, for the tests that check that the pins catch it); None restores
    the library built from ``mpm_oracle.cpp``."""
    global _lib, _override
    _override = path
    _lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_override or build())
        D = ctypes.POINTER(_Desc)
        P = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.orc_state_size.argtypes = [i]
        lib.orc_step_fwd.argtypes = [D, P, P, P]
        lib.orc_grid.argtypes = [D, P, P, P, P]
        lib.orc_step_bwd.argtypes = [D, P, P, P, P, P, P]
        lib.orc_run_fwd.argtypes = [D, i, P, P, P, P]
        lib.orc_run_bwd.argtypes = [D, i, i, P, P, P, P, P, P]
        lib.orc_run_fwd_cs.argtypes = [D, i, P, P, P, P, P, ctypes.c_double, P, P]
        for f in ("orc_step_fwd", "orc_grid", "orc_step_bwd", "orc_run_fwd", "orc_run_bwd",
                  "orc_run_fwd_cs", "orc_state_size"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Bound:
    """Keeps the ctypes descriptor and the arrays it points at alive."""

    def __init__(self, sc):
        self.offsets = np.ascontiguousarray(sc.offsets, dtype=np.int32)
        ns = len(self.offsets) - 1
        self.n_scenes = ns
        self.N = int(self.offsets[-1])
        self.dim = int(sc.dim)

        def per_scene(v):
            return np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (ns,)))

        self.E = per_scene(sc.E)
        self.nu = per_scene(sc.nu)
        self.vol = per_scene(sc.vol)
        self.rho = per_scene(sc.rho)
        act_id = getattr(sc, "act_id", None)
        self.act_id = None if act_id is None else np.ascontiguousarray(act_id, dtype=np.int32)
        self.n_act = int(getattr(sc, "n_act", 0) or 0)
        mat_id = getattr(sc, "mat_id", None)
        self.mat_id = None if mat_id is None else np.ascontiguousarray(mat_id, dtype=np.int32)
        self.desc = _Desc(
            dim=self.dim, n_grid=int(sc.n_grid), bound=int(sc.bound), n_scenes=ns, n_act=self.n_act,
            dx=float(sc.dx), dt=float(sc.dt), gravity=float(sc.gravity),
            act_strength=float(getattr(sc, "act_strength", 0.0) or 0.0),
            offsets=self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            E=_dptr(self.E), nu=_dptr(self.nu), vol=_dptr(self.vol), rho=_dptr(self.rho),
            act_id=None if self.act_id is None else self.act_id.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            model=int(getattr(sc, "model", 0) or 0),
            mat_id=None if self.mat_id is None else self.mat_id.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        )

    @property
    def ref(self):
        return ctypes.byref(self.desc)


def state_size(dim: int) -> int:
    return 2 * dim + 2 * dim * dim


def pack(x, v, C, F) -> np.ndarray:
    """(N,d),(N,d),(N,d,d),(N,d,d) -> (N,S) float64, particle-major."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    return np.ascontiguousarray(np.concatenate(
        [x.reshape(N, -1), np.asarray(v, np.float64).reshape(N, -1),
         np.asarray(C, np.float64).reshape(N, -1), np.asarray(F, np.float64).reshape(N, -1)], axis=1))


def unpack(s: np.ndarray, dim: int):
    s = np.asarray(s).reshape(s.shape[0], -1)
    N, d = s.shape[0], dim
    x = s[:, :d]
    v = s[:, d:2 * d]
    C = s[:, 2 * d:2 * d + d * d].reshape(N, d, d)
    F = s[:, 2 * d + d * d:].reshape(N, d, d)
    return x, v, C, F


def _act_arr(act, n):
    if act is None:
        return None
    a = np.ascontiguousarray(act, dtype=np.float64)
    assert a.size == n, (a.shape, n)
    return a


def step_fwd(scene, state, act_s=None):
    """One forward step. Returns (state', error_bits)."""
    b = _Bound(scene)
    s = np.ascontiguousarray(state, dtype=np.float64)
    out = np.empty_like(s)
    err = _load().orc_step_fwd(b.ref, _dptr(_act_arr(act_s, b.n_act)), _dptr(s), _dptr(out))
    return out, err


def grid(scene, state, act_s=None):
    """Grid after particle-to-grid (m, P) and after the grid update (m, v):
    two arrays of shape (n_scenes, n_grid**d, d+1)."""
    b = _Bound(scene)
    s = np.ascontiguousarray(state, dtype=np.float64)
    nn = int(scene.n_grid) ** b.dim
    gp = np.zeros((b.n_scenes, nn, b.dim + 1))
    gv = np.zeros_like(gp)
    err = _load().orc_grid(b.ref, _dptr(_act_arr(act_s, b.n_act)), _dptr(s), _dptr(gp), _dptr(gv))
    return gp, gv, err


def step_bwd(scene, state, gout, act_s=None):
    """Adjoint of one step. Returns (gin, gE[n_scenes], gact[n_act], error_bits)."""
    b = _Bound(scene)
    s = np.ascontiguousarray(state, dtype=np.float64)
    g = np.ascontiguousarray(gout, dtype=np.float64)
    gin = np.zeros_like(s)
    gE = np.zeros(b.n_scenes)
    gact = np.zeros(max(b.n_act, 1))
    err = _load().orc_step_bwd(b.ref, _dptr(_act_arr(act_s, b.n_act)), _dptr(s), _dptr(g), _dptr(gin),
                               _dptr(gE), _dptr(gact))
    return gin, gE, gact[:b.n_act], err


def run_fwd(scene, T, state0, act=None, keep_tape=False):
    """T forward steps. Returns (state_T, tape or None, error_bits)."""
    b = _Bound(scene)
    s0 = np.ascontiguousarray(state0, dtype=np.float64)
    sT = np.empty_like(s0)
    tape = np.empty((T + 1,) + s0.shape) if keep_tape else None
    err = _load().orc_run_fwd(b.ref, int(T), _dptr(_act_arr(act, T * b.n_act)), _dptr(s0), _dptr(tape),
                              _dptr(sT))
    return sT, tape, err


def run_bwd(scene, T, K, state0, gT, act=None):
    """Reverse pass with checkpoints every K steps (K >= T: full tape).
    Returns (g0, gE[n_scenes], gact[T, n_act], error_bits)."""
    b = _Bound(scene)
    s0 = np.ascontiguousarray(state0, dtype=np.float64)
    g = np.ascontiguousarray(gT, dtype=np.float64)
    g0 = np.zeros_like(s0)
    gE = np.zeros(b.n_scenes)
    gact = np.zeros((T, max(b.n_act, 1)))
    err = _load().orc_run_bwd(b.ref, int(T), int(K), _dptr(_act_arr(act, T * b.n_act)), _dptr(s0), _dptr(g),
                              _dptr(g0), _dptr(gE), _dptr(gact))
    return g0, gE, gact[:, :b.n_act], err


def run_fwd_cs(scene, T, state0, state_dir=None, E_dir=None, act=None, act_dir=None, h=1e-30):
    """Complex-step tangent of T forward steps along (state_dir, E_dir, act_dir).
    Returns (state_T, tangent_T, error_bits)."""
    b = _Bound(scene)
    s0 = np.ascontiguousarray(state0, dtype=np.float64)
    sd = None if state_dir is None else np.ascontiguousarray(state_dir, dtype=np.float64)
    ed = None if E_dir is None else np.ascontiguousarray(np.broadcast_to(E_dir, (b.n_scenes,)), dtype=np.float64)
    sT = np.empty_like(s0)
    tan = np.empty_like(s0)
    err = _load().orc_run_fwd_cs(b.ref, int(T), _dptr(_act_arr(act, T * b.n_act)),
                                 _dptr(_act_arr(act_dir, T * b.n_act)), _dptr(s0), _dptr(sd), _dptr(ed),
                                 float(h), _dptr(sT), _dptr(tan))
    return sT, tan, err


# ---------------------------------------------------------------------------
# Open-loop actuation of the 2D soft robot (Section 4.1 trains "an open-loop
# controller"): a_k(t) = tanh(sum_j W_kj sin(omega t + 2 pi j / n_sin) + b_k),
# t = s * dt, and its adjoint (W*, b*) from a*(s, k).
# ---------------------------------------------------------------------------
def actuation(W, b, omega, dt, T):
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    n_sin = W.shape[1]
    t = np.arange(T, dtype=np.float64) * dt
    phase = omega * t[:, None] + 2.0 * np.pi * np.arange(n_sin)[None, :] / n_sin  # (T, n_sin)
    return np.tanh(np.sin(phase) @ W.T + b[None, :])  # (T, n_act)


def actuation_bwd(W, b, omega, dt, T, abar):
    W = np.asarray(W, np.float64)
    n_sin = W.shape[1]
    a = actuation(W, b, omega, dt, T)
    t = np.arange(T, dtype=np.float64) * dt
    sn = np.sin(omega * t[:, None] + 2.0 * np.pi * np.arange(n_sin)[None, :] / n_sin)
    pre_bar = np.asarray(abar, np.float64) * (1.0 - a * a)  # (T, n_act)
    return pre_bar.T @ sn, pre_bar.sum(axis=0)


def loss_mean_pos(scene, state, axis, sign=1.0):
    """L = sum over scenes of sign * (1/N_scene) sum_p x_{p,axis}; returns (L per scene, seed dL/dstate).
    A scene with no particles contributes a zero term (and no seed entries)."""
    b = _Bound(scene)
    s = np.asarray(state, np.float64)
    L = np.zeros(b.n_scenes)
    seed = np.zeros_like(s)
    for k in range(b.n_scenes):
        lo, hi = b.offsets[k], b.offsets[k + 1]
        if hi == lo:
            continue
        L[k] = sign * s[lo:hi, axis].mean()
        seed[lo:hi, axis] = sign / (hi - lo)
    return L, seed

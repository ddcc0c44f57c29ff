"""Seeded synthetic scenes for the differentiable MLS-MPM step.

This module only draws inputs: particle positions, initial velocities and
deformation, material constants and actuation weights. It contains none of the
simulation arithmetic, so both the GPU path and the FP64 oracle can take their
inputs from it.

Every scene is generated in float64 and then rounded to float32; the float32
values are what both sides receive (the oracle widens them back to float64),
so parity measures the dynamics and not input rounding.

Workloads (the paper's elastic-object simulator, Section 4.1; its own
benchmark used a 2D scene with 6.4K particles whose grid is not stated):
  translate2d   2D, 64^2 grid, 1024 particles on a jittered lattice, uniform v=(1,0), 64 steps
  deform2d  translate2d with an added affine velocity, so the body deforms
  actuated2d   2D actuated soft body, 128^2 grid, 8192 particles in a union of rectangles,
       4 actuators driven by a_k(t) = tanh(sum_j W_kj sin(w t + 2 pi j/4) + b_k), 512 steps
  elastic3d   3D, 64^3 grid, 32768 particles on a 32^3 jittered lattice, 256 steps, full tape
  elastic3d_long   3D, 128^3 grid, 262144 particles on a 64^3 lattice, 1024 steps, checkpoints every 64
  batched2d   256 independent 2D scenes on their own 64^2 grids, particle counts
       log-uniform in [500, 8000], per-scene E and nu, 256 steps
  robot3d   3D actuated soft robot (body on four legs), 64^3 grid, 30000 particles,
       16 actuators, 512 steps (the crawler of Appendix E.1, synthetic geometry)
  coupled3d   robot3d beside 13000 particles of weakly compressible liquid, two-way
       coupled through the grid (the robot-and-liquid setting of Appendix E.1)
  fd8  8 particles with random C and F, for finite-difference checks

and the incompressible smoke simulator of Section 4.2 (SmokeScene, smoke()):
  smoke110   periodic 110^2 grid, 100 steps, 6 Jacobi iterations per projection
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

F32 = np.float32


@dataclass
class Scene:
    name: str
    dim: int
    n_grid: int
    dx: float
    dt: float
    steps: int
    offsets: np.ndarray          # int32 [n_scenes + 1]
    E: np.ndarray                # float32 [n_scenes]
    nu: np.ndarray               # float32 [n_scenes]
    vol: np.ndarray              # float32 [n_scenes] initial particle volume
    rho: np.ndarray              # float32 [n_scenes]
    x: np.ndarray                # float32 (N, d)
    v: np.ndarray                # float32 (N, d)
    C: np.ndarray                # float32 (N, d, d)
    F: np.ndarray                # float32 (N, d, d)
    bound: int = 3
    gravity: float = -9.8
    ckpt_every: int = 0          # 0: full tape
    loss_axis: int = 0
    loss_sign: float = 1.0
    act_id: Optional[np.ndarray] = None   # int32 (N,) actuator column, -1 for none
    n_act: int = 0
    act_strength: float = 0.0
    act_W: Optional[np.ndarray] = None    # float32 (n_act, n_sin)
    act_b: Optional[np.ndarray] = None    # float32 (n_act,)
    act_omega: float = 0.0
    model: int = 0                        # 0: neo-Hookean, 1: fixed-corotated
    mat_id: Optional[np.ndarray] = None   # int32 (N,): 0 solid, 1 weakly compressible liquid
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_scenes(self) -> int:
        return len(self.offsets) - 1

    def with_steps(self, steps: int, ckpt_every: Optional[int] = None) -> "Scene":
        return replace(self, steps=int(steps), ckpt_every=self.ckpt_every if ckpt_every is None else ckpt_every)

    def subset(self, scenes, keep=None) -> "Scene":
        """Scenes `scenes` of a batched scene (repeats allowed), as a new batched
        scene. `keep[j]`, if given, keeps only the first keep[j] particles of the
        j-th chosen scene (0 gives a scene with no particles)."""
        scenes = list(scenes)
        full = [int(self.offsets[k + 1] - self.offsets[k]) for k in scenes]
        counts = full if keep is None else [min(int(c), f) for c, f in zip(keep, full)]
        idx = np.concatenate([np.arange(self.offsets[k], self.offsets[k] + c, dtype=np.int64)
                              for k, c in zip(scenes, counts)])
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        return replace(
            self, name=f"{self.name}[{len(scenes)}]", offsets=off, E=self.E[scenes].copy(),
            nu=self.nu[scenes].copy(), vol=self.vol[scenes].copy(), rho=self.rho[scenes].copy(),
            x=self.x[idx].copy(), v=self.v[idx].copy(), C=self.C[idx].copy(), F=self.F[idx].copy(),
            act_id=None if self.act_id is None else self.act_id[idx].copy(),
            mat_id=None if self.mat_id is None else self.mat_id[idx].copy())


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(F32))


def _lattice(rng, dim, per_axis, lo, spacing, jitter):
    """per_axis^dim points at lo + (i + 1/2) * spacing, each jittered by U(-jitter, jitter)."""
    idx = np.stack(np.meshgrid(*([np.arange(per_axis)] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    x = lo + (idx + 0.5) * spacing
    return x + rng.uniform(-jitter, jitter, size=x.shape)


def _identity(N, dim):
    return np.broadcast_to(np.eye(dim), (N, dim, dim)).copy()


def _single(name, dim, n_grid, dt, steps, x, v, E, nu, vol, **kw):
    N = x.shape[0]
    return Scene(
        name=name, dim=dim, n_grid=n_grid, dx=1.0 / n_grid, dt=float(F32(dt)), steps=steps,
        offsets=np.array([0, N], np.int32), E=_f32([E]), nu=_f32([nu]), vol=_f32([vol]), rho=_f32([1.0]),
        x=_f32(x), v=_f32(v), C=_f32(np.zeros((N, dim, dim))), F=_f32(_identity(N, dim)), **kw)


def translate2d(seed: int = 0) -> Scene:
    """2D, 64^2, 1024 particles on a 32x32 lattice spaced dx/2 in [0.25, 0.5]^2,
    jitter U(+-0.1 dx), v = (1, 0), E = 10, nu = 0.2, volume (dx/2)^2, dt = 1e-3, 64 steps,
    loss = mean final x-coordinate."""
    rng = np.random.default_rng(seed)
    n = 64
    dx = 1.0 / n
    x = _lattice(rng, 2, 32, 0.25, dx / 2, 0.1 * dx)
    v = np.tile([1.0, 0.0], (x.shape[0], 1))
    return _single("translate2d", 2, n, 1e-3, 64, x, v, 10.0, 0.2, (dx / 2) ** 2, loss_axis=0)


def deform2d(seed: int = 0) -> Scene:
    """translate2d with v = (1, 0) + diag(1, -1) (x - (0.375, 0.375)) so that C and F evolve."""
    s = translate2d(seed)
    x = s.x.astype(np.float64)
    v = np.array([1.0, 0.0]) + (x - 0.375) * np.array([1.0, -1.0])
    return replace(s, name="deform2d", v=_f32(v))


def _skyline_rects(rng, n_rect, w_lo, w_hi, h_lo, h_hi, x_lo, x_hi):
    """Axis-aligned rectangles standing on y = 0, each overlapping an earlier one in x."""
    rects = []
    for k in range(n_rect):
        w = rng.uniform(w_lo, w_hi)
        h = rng.uniform(h_lo, h_hi)
        if k == 0:
            x0 = rng.uniform(x_lo, max(x_lo, x_hi - w))
        else:
            px0, px1, _ = rects[rng.integers(0, k)]
            x0 = rng.uniform(px0 - 0.8 * w, px1 - 0.2 * w)
            x0 = min(max(x0, x_lo), x_hi - w)
        rects.append((x0, x0 + w, h))
    return rects


def _skyline_area(rects):
    xs = sorted({r[0] for r in rects} | {r[1] for r in rects})
    area = 0.0
    for a, b in zip(xs[:-1], xs[1:]):
        mid = 0.5 * (a + b)
        h = max([r[2] for r in rects if r[0] <= mid < r[1]] or [0.0])
        area += (b - a) * h
    return area


def _sample_union(rng, rects, N):
    """N points uniform in the union; also the index of the first rectangle containing each."""
    x0 = min(r[0] for r in rects)
    x1 = max(r[1] for r in rects)
    y1 = max(r[2] for r in rects)
    pts, ids = [], []
    need = N
    while need > 0:
        c = rng.uniform([x0, 0.0], [x1, y1], size=(max(4 * need, 64), 2))
        inside = np.zeros(len(c), bool)
        first = np.full(len(c), -1)
        for k, (a, b, h) in enumerate(rects):
            hit = (c[:, 0] >= a) & (c[:, 0] < b) & (c[:, 1] < h) & ~inside
            first[hit] = k
            inside |= hit
        pts.append(c[inside][:need])
        ids.append(first[inside][:need])
        need -= len(pts[-1])
    return np.concatenate(pts), np.concatenate(ids)


def actuated2d(seed: int = 1) -> Scene:
    """2D actuated soft body: 128^2 grid, 8192 particles uniform in a union of 4-6
    rectangles (widths, heights U[0.05, 0.2], standing on y = 0.1, x in [0.1, 0.6]);
    actuator column = (first containing rectangle) mod 4; a_k(t) = tanh(sum_j W_kj
    sin(omega t + 2 pi j / 4) + b_k) with W, b ~ N(0, 0.1^2), omega = 2 pi 5, sigma_a = 10;
    E = 10, nu = 0.2, dt = 1e-3, 512 steps; loss = -(mean final x)."""
    rng = np.random.default_rng(seed)
    n = 128
    N = 8192
    rects = _skyline_rects(rng, int(rng.integers(4, 7)), 0.05, 0.2, 0.05, 0.2, 0.1, 0.6)
    area = _skyline_area(rects)
    pts, first = _sample_union(rng, rects, N)
    pts[:, 1] += 0.1
    n_act = 4
    W = rng.normal(0.0, 0.1, size=(n_act, 4))
    b = rng.normal(0.0, 0.1, size=(n_act,))
    s = _single("actuated2d", 2, n, 1e-3, 512, pts, np.zeros((N, 2)), 10.0, 0.2, area / N, loss_axis=0,
                loss_sign=-1.0, act_id=(first % n_act).astype(np.int32), n_act=n_act, act_strength=10.0,
                act_W=_f32(W), act_b=_f32(b), act_omega=float(F32(2 * math.pi * 5)))
    s.meta["rects"] = rects
    return s


def _lattice3d(name, seed, n_grid, per_axis, dt, steps, ckpt, loss_axis):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_grid
    x = _lattice(rng, 3, per_axis, 0.25, dx / 2, 0.1 * dx)
    # Affine initial velocity diag(1, -1, 0) (x - x_c), so the block deforms.
    v = (x - 0.375) * np.array([1.0, -1.0, 0.0])
    return _single(name, 3, n_grid, dt, steps, x, v, 20.0, 0.3, (dx / 2) ** 3, ckpt_every=ckpt,
                   loss_axis=loss_axis)


def elastic3d(seed: int = 2) -> Scene:
    """3D, 64^3 grid, 32768 particles on a 32^3 lattice spaced dx/2 in [0.25, 0.5]^3,
    jittered, E = 20, nu = 0.3, dt = 5e-4, 256 steps, full tape; loss = mean final height."""
    return _lattice3d("elastic3d", seed, 64, 32, 5e-4, 256, 0, 1)


def elastic3d_long(seed: int = 3) -> Scene:
    """3D, 128^3 grid, 262144 particles on a 64^3 lattice spaced dx/2, jittered, E = 20,
    nu = 0.3, dt = 2.5e-4, 1024 steps, checkpoints every 64; loss = mean final x."""
    return _lattice3d("elastic3d_long", seed, 128, 64, 2.5e-4, 1024, 64, 0)


def robot3d(seed: int = 5, n_particles: int = 30000, steps: int = 512) -> Scene:
    """3D actuated soft robot (the crawler of Appendix E.1: 16 muscles, about 30K
    particles; the paper gives no geometry, so this one is synthetic): 64^3 grid;
    a body slab [0.1, 0.45] x [0.15, 0.225] x [0.3, 0.65] standing on four legs
    0.1 x 0.1 x 0.1 at its corners (feet at y = 0.05, just above the sticky floor
    band); particles uniform in the five boxes, in proportion to volume. Each leg
    is split into 2 x 2 columns in x-z, one actuator per column (16 actuators);
    the body is passive. a_k(t) as in actuated2d with n_sin = 4, W, b ~ N(0, 0.1^2),
    omega = 2 pi 8, sigma_a = 10; E = 20, nu = 0.3, dt = 5e-4, 512 steps, v0 = 0;
    loss = -(mean final x), i.e. crawl towards +x."""
    rng = np.random.default_rng(seed)
    n = 64
    body = ((0.10, 0.45), (0.15, 0.225), (0.30, 0.65))
    legs = [((x0, x0 + 0.1), (0.05, 0.15), (z0, z0 + 0.1)) for x0 in (0.10, 0.35) for z0 in (0.30, 0.55)]
    boxes = [body] + legs
    vols = np.array([np.prod([hi - lo for lo, hi in b]) for b in boxes])
    counts = np.floor(n_particles * vols / vols.sum()).astype(int)
    counts[0] += n_particles - counts.sum()
    xs, act = [], []
    for k, (b, c) in enumerate(zip(boxes, counts)):
        lo = np.array([r[0] for r in b])
        hi = np.array([r[1] for r in b])
        pts = rng.uniform(lo, hi, size=(c, 3))
        xs.append(pts)
        if k == 0:
            act.append(np.full(c, -1))
        else:
            mid = 0.5 * (lo + hi)
            act.append(4 * (k - 1) + 2 * (pts[:, 0] >= mid[0]) + (pts[:, 2] >= mid[2]))
    x = np.concatenate(xs)
    n_act = 16
    W = rng.normal(0.0, 0.1, size=(n_act, 4))
    bb = rng.normal(0.0, 0.1, size=(n_act,))
    s = _single("robot3d", 3, n, 5e-4, steps, x, np.zeros_like(x), 20.0, 0.3, float(vols.sum()) / n_particles,
                loss_axis=0, loss_sign=-1.0, act_id=np.concatenate(act).astype(np.int32), n_act=n_act,
                act_strength=10.0, act_W=_f32(W), act_b=_f32(bb), act_omega=float(F32(2 * math.pi * 8)))
    s.meta["boxes"] = boxes
    return s


def coupled3d(seed: int = 6, n_liquid: int = 13000, steps: int = 512) -> Scene:
    """The 3D robot (robot3d, 30000 particles, material 0) beside a block of
    weakly compressible liquid (material 1, n_liquid particles uniform in
    [0.5, 0.65] x [0.05, 0.05 + h] x [0.3, 0.65], h set so that the liquid has
    the robot's particle volume), two-way coupled through the shared grid (the
    robot-and-liquid setting of Appendix E.1, 30K + 13K particles); the scene's
    E (20) is the liquid's bulk modulus; loss = -(mean final x) of all particles."""
    rng = np.random.default_rng(seed)
    r = robot3d(steps=steps)
    vol = float(r.vol[0])
    h = n_liquid * vol / (0.15 * 0.35)
    lo = np.array([0.5, 0.05, 0.3])
    hi = np.array([0.65, 0.05 + h, 0.65])
    xl = rng.uniform(lo, hi, size=(n_liquid, 3))
    x = np.concatenate([r.x.astype(np.float64), xl])
    N = x.shape[0]
    s = replace(r, name="coupled3d", offsets=np.array([0, N], np.int32), x=_f32(x),
                v=_f32(np.zeros((N, 3))), C=_f32(np.zeros((N, 3, 3))), F=_f32(_identity(N, 3)),
                act_id=np.concatenate([r.act_id, np.full(n_liquid, -1, np.int32)]).astype(np.int32),
                mat_id=np.concatenate([np.zeros(r.n_particles, np.int32), np.ones(n_liquid, np.int32)]))
    s.meta = dict(r.meta, liquid_box=(tuple(lo), tuple(hi)))
    return s


def batched2d(seed: int = 4, n_scenes: int = 256, steps: int = 256) -> Scene:
    """n_scenes independent 2D scenes, each on its own 64^2 grid, with particle counts
    N = round(exp U(ln 500, ln 8000)) in rectangle-union shapes (4 particles per cell,
    volume (dx/2)^2), centred in x and standing on y = 0.1; E ~ U[5, 30], nu ~ U[0.1, 0.4];
    v0 = 0; dt = 1e-3; loss = sum over scenes of the mean final x."""
    rng = np.random.default_rng(seed)
    n = 64
    dx = 1.0 / n
    vol = (dx / 2) ** 2
    xs, counts, Es, nus = [], [], [], []
    for _ in range(n_scenes):
        N = int(round(math.exp(rng.uniform(math.log(500), math.log(8000)))))
        rects = _skyline_rects(rng, int(rng.integers(4, 7)), 0.25, 1.0, 0.25, 1.0, 0.0, 1.5)
        area0 = _skyline_area(rects)
        scale = math.sqrt(N * vol / area0)
        width0 = max(r[1] for r in rects) - min(r[0] for r in rects)
        height0 = max(r[2] for r in rects)
        sx = sy = scale
        if width0 * sx > 0.8:          # keep the area, make it narrower and taller
            f = 0.8 / (width0 * sx)
            sx *= f
            sy /= f
        if height0 * sy > 0.8:
            sy = 0.8 / height0
        pts, _ = _sample_union(rng, rects, N)
        x_min = min(r[0] for r in rects)
        x_max = max(r[1] for r in rects)
        pts[:, 0] = (pts[:, 0] - 0.5 * (x_min + x_max)) * sx + 0.5
        pts[:, 1] = pts[:, 1] * sy + 0.1
        xs.append(pts)
        counts.append(N)
        Es.append(rng.uniform(5.0, 30.0))
        nus.append(rng.uniform(0.1, 0.4))
    x = np.concatenate(xs)
    Nt = x.shape[0]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    ns = n_scenes
    return Scene(
        name="batched2d", dim=2, n_grid=n, dx=dx, dt=float(F32(1e-3)), steps=steps, offsets=off, E=_f32(Es),
        nu=_f32(nus), vol=_f32(np.full(ns, vol)), rho=_f32(np.ones(ns)), x=_f32(x),
        v=_f32(np.zeros((Nt, 2))), C=_f32(np.zeros((Nt, 2, 2))), F=_f32(_identity(Nt, 2)), loss_axis=0)


def fd8(dim: int = 2, seed: int = 5, steps: int = 16, liquid: bool = False) -> Scene:
    """8 particles (2x4 in 2D, 2x2x2 in 3D) near the centre of a 16^d grid, spaced dx/2,
    with F = I + 0.05 N(0,1), C ~ N(0, 1), v ~ N(0, 0.2): every term of the step is active.
    With `liquid`, every other particle is the weakly compressible liquid."""
    rng = np.random.default_rng(seed)
    n = 16
    dx = 1.0 / n
    shape = (2, 4) if dim == 2 else (2, 2, 2)
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in shape], indexing="ij"), -1).reshape(-1, dim)
    x = 0.5 + (idx - np.array(shape) / 2 + 0.5) * dx / 2 + rng.uniform(-0.1 * dx, 0.1 * dx, (8, dim))
    s = _single(f"fd8_{dim}d", dim, n, 1e-3, steps, x, rng.normal(0, 0.2, (8, dim)), 10.0, 0.25,
                (dx / 2) ** dim)
    s.C = _f32(rng.normal(0.0, 1.0, (8, dim, dim)))
    s.F = _f32(np.eye(dim) + 0.05 * rng.normal(0.0, 1.0, (8, dim, dim)))
    if liquid:
        s.mat_id = (np.arange(8) % 2).astype(np.int32)
    return s


def random_state(scene: Scene, seed: int, c_scale: float = 1.0, f_scale: float = 0.05,
                 v_scale: float = 0.3) -> Scene:
    """The same positions with random v, C and F = I + f_scale N(0,1): a generic state
    for single-step and per-stage checks."""
    rng = np.random.default_rng(seed)
    N, d = scene.x.shape
    return replace(scene, v=_f32(rng.normal(0, v_scale, (N, d))),
                   C=_f32(rng.normal(0, c_scale, (N, d, d))),
                   F=_f32(np.eye(d) + f_scale * rng.normal(0, 1, (N, d, d))))


@dataclass
class SmokeScene:
    """Inputs of the incompressible smoke simulator (Section 4.2): a periodic
    n x n grid, velocities in cells per step (axis-0 and axis-1 components),
    a smoke density and the target density of the loss."""
    name: str
    n: int
    steps: int
    iters: int                   # Jacobi iterations per pressure projection
    u0: np.ndarray               # float32 (n, n)
    u1: np.ndarray               # float32 (n, n)
    s: np.ndarray                # float32 (n, n)
    target: np.ndarray           # float32 (n, n)

    def with_steps(self, steps: int, iters: Optional[int] = None) -> "SmokeScene":
        return replace(self, steps=int(steps), iters=self.iters if iters is None else int(iters))


def _periodic_modes(rng, n, kmax, rms):
    """A smooth periodic field: random low Fourier modes (|k| <= kmax per
    axis), scaled to the given RMS."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((n, n))
    for k0 in range(-kmax, kmax + 1):
        for k1 in range(-kmax, kmax + 1):
            if (k0, k1) != (0, 0):
                f += rng.normal() * np.cos(2 * np.pi * (k0 * i + k1 * j) / n + rng.uniform(0, 2 * np.pi))
    return f * (rms / np.sqrt(np.mean(f * f)))


def _blobs(rng, n, count, radius):
    """Density in [0, 1]: periodic Gaussian blobs at random centres."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((n, n))
    for _ in range(count):
        c0, c1 = rng.uniform(0, n, 2)
        d0 = np.minimum(np.abs(i - c0), n - np.abs(i - c0))
        d1 = np.minimum(np.abs(j - c1), n - np.abs(j - c1))
        f += np.exp(-(d0 ** 2 + d1 ** 2) / (2 * (radius * n) ** 2))
    return np.clip(f, 0.0, 1.0)


def smoke(n: int = 110, steps: int = 100, iters: int = 6, seed: int = 7, speed: float = 0.5) -> SmokeScene:
    """The smoke benchmark's shape (Table 2: a 110 x 110 grid, 100 steps, 6
    Jacobi iterations per projection); the paper's initial image and target
    pattern are not available, so the smoke is a few seeded Gaussian blobs,
    the initial velocity a smooth random periodic field with RMS `speed`
    cells per step (its largest values about three times that), and the
    target another set of blobs."""
    rng = np.random.default_rng(seed)
    u0 = _periodic_modes(rng, n, 3, speed)
    u1 = _periodic_modes(rng, n, 3, speed)
    s = _blobs(rng, n, 6, 0.08)
    target = _blobs(rng, n, 4, 0.12)
    return SmokeScene(name=f"smoke{n}", n=n, steps=steps, iters=iters, u0=_f32(u0), u1=_f32(u1), s=_f32(s),
                      target=_f32(target))


REGISTRY = {"translate2d": translate2d, "deform2d": deform2d, "actuated2d": actuated2d, "elastic3d": elastic3d, "elastic3d_long": elastic3d_long, "batched2d": batched2d,
            "robot3d": robot3d, "coupled3d": coupled3d}


def make(name: str, **kw) -> Scene:
    return REGISTRY[name](**kw)

"""Binning and tape bookkeeping on the GPU:
  - the particle order a tape keeps (mpm_sort_order) equals, bit for bit, a
    stable NumPy sort by (scene, Morton code of the cell), also when every
    particle sits in one cell and for NaN and out-of-grid positions;
  - a tape's reverse pass is unaffected by other tapes of the same context
    running in between;
  - a trajectory whose tape was run forward again refuses its backward, and a
    launch-shape change between forward and backward is refused;
  - the autograd trajectory passes the material ids (liquid) to the tape.
"""
import numpy as np
import pytest
import torch

from paper_1910_00935_amd import _lib as L
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes
from paper_1910_00935_amd.controller import OpenLoopController

from parity import cos, log, rel

pytestmark = pytest.mark.gpu


def _expected_order(sc):
    """Stable argsort of scene * cells + morton(cell), computed with the same
    single-precision cell arithmetic (x * (1/dx), truncated, clamped, NaN to 0)."""
    d, n = sc.dim, sc.n_grid
    bits = int(np.ceil(np.log2(n)))
    x = np.asarray(sc.x, np.float32)
    g = x * (np.float32(1.0) / np.float32(sc.dx))
    with np.errstate(invalid="ignore"):
        c = np.where(g >= 0, np.where(g < np.float32(n - 1), np.floor(np.nan_to_num(g)), n - 1), 0).astype(np.int64)
    key = np.zeros(len(x), np.int64)
    for b in range(bits - 1, -1, -1):
        for a in range(d):
            key = (key << 1) | ((c[:, a] >> b) & 1)
    scene = np.repeat(np.arange(sc.n_scenes), np.diff(sc.offsets))
    key += scene.astype(np.int64) << (d * bits)
    return np.argsort(key, kind="stable")


def _sort_case(sc):
    sim = rt.Simulator.for_scene(sc)
    perm = sim.sort_order(rt.state_for_scene(sc)).cpu().numpy()
    expect = _expected_order(sc)
    log(f"[sort] {sc.name}: N={sc.n_particles}")
    assert np.array_equal(perm, expect)


def test_sort_order_lattice_3d():
    _sort_case(scenes.elastic3d())


def test_sort_order_random_3d():
    _sort_case(scenes.robot3d())


def test_sort_order_ragged_batch_2d():
    base = scenes.batched2d(n_scenes=5, steps=8)
    _sort_case(base.subset([0, 1, 2, 3, 4, 1], [0, 10 ** 9, 1, 37, 10 ** 9, 0]))


def test_sort_order_one_cell_nan_and_outside():
    """100 000 particles in one cell (one key holding almost every particle),
    plus NaN and out-of-grid positions, which bin to clamped cells."""
    rng = np.random.default_rng(0)
    base = scenes.translate2d()
    N = 100_000
    dx = base.dx
    x = (np.array([20.0, 30.0]) + rng.uniform(0.05, 0.95, size=(N, 2))) * dx
    x[::997] = np.nan
    x[5::1001] = [-0.3, 2.0]
    x[7::1003] = [0.5, 1e6]
    sc = scenes.Scene(name="one_cell", dim=2, n_grid=base.n_grid, dx=dx, dt=base.dt, steps=1,
                      offsets=np.array([0, N], np.int32), E=base.E, nu=base.nu, vol=base.vol, rho=base.rho,
                      x=x.astype(np.float32), v=np.zeros((N, 2), np.float32),
                      C=np.zeros((N, 2, 2), np.float32), F=np.broadcast_to(np.eye(2, dtype=np.float32), (N, 2, 2)).copy())
    _sort_case(sc)


def _trajectory(sim, sc, tape, init, w, params=None):
    params = params or rt.params_for_scene(sc)
    fin = rt.State.empty(sc.dim, sc.n_particles)
    tape.forward(params, init, fin)
    return params, fin


def _backward(sc, tape, params, w):
    ig = rt.State.zeros(sc.dim, sc.n_particles)
    gE = torch.zeros(sc.n_scenes, device="cuda")
    tape.backward(params, rt.State.from_particle_major(*w), ig, gE)
    return ig.to_particle_major(), gE.cpu().numpy()


def test_tapes_interleaved_on_one_context():
    """Forward A, forward B of a different initial state on a second tape of the
    same context (a different sort), then backward A: equal to backward A run
    right after forward A. Liquid and actuation ids exercise the sorted ids."""
    sc = scenes.coupled3d().with_steps(16)
    sim = rt.Simulator.for_scene(sc)
    act = torch.as_tensor(np.random.default_rng(1).normal(0, 0.3, (16, sc.n_act)), dtype=torch.float32, device="cuda")
    params = rt.params_for_scene(sc, act=act)
    rng = np.random.default_rng(2)
    S = 24
    wa = rng.normal(size=(sc.n_particles, S)) / np.sqrt(sc.n_particles)
    w = (wa[:, :3], wa[:, 3:6], wa[:, 6:15].reshape(-1, 3, 3), wa[:, 15:].reshape(-1, 3, 3))
    init_a = rt.state_for_scene(sc)
    xb = sc.x[::-1].copy()  # other positions: another permutation
    init_b = rt.State.from_particle_major(xb, sc.v, sc.C, sc.F)
    tape_a, tape_b = sim.tape(16, 8), sim.tape(16, 8)
    _trajectory(sim, sc, tape_a, init_a, w, params)
    ref = _backward(sc, tape_a, params, w)
    _trajectory(sim, sc, tape_b, init_b, w, params)
    got = _backward(sc, tape_a, params, w)
    for k in range(4):
        log(f"  interleaved grad block {k}: rel {rel(got[0][k], ref[0][k]):.3g}")
        assert rel(got[0][k], ref[0][k]) < 1e-6
    assert rel(got[1], ref[1]) < 1e-6
    assert sim.check_errors() == 0


def test_rerun_tape_refuses_stale_backward():
    sc = scenes.deform2d().with_steps(8)
    sim = rt.Simulator.for_scene(sc)
    p = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    tape = sim.tape(8)
    v0 = init.v.clone().requires_grad_(True)
    x1, _, _, _ = rt.MPMTrajectory.apply(tape, p, init.x, v0, init.C, init.F, p.E, None)
    x2, _, _, _ = rt.MPMTrajectory.apply(tape, p, init.x, v0, init.C, init.F, p.E, None)
    with pytest.raises(RuntimeError, match="run forward again"):
        (x1.sum() + x2.sum()).backward()


def test_launch_shape_change_refused():
    sc = scenes.deform2d().with_steps(8)
    sim = rt.Simulator.for_scene(sc, knobs={"block": 128})
    p = rt.params_for_scene(sc)
    tape = sim.tape(8)
    _trajectory(sim, sc, tape, rt.state_for_scene(sc), None, p)
    sim.set_knob("block", 256)
    z = rt.State.zeros(2, sc.n_particles)
    with pytest.raises(L.MPMError) as e:
        tape.backward(p, z, rt.State.zeros(2, sc.n_particles))
    assert e.value.status == L.MPM_E_TAPE
    sim.set_knob("block", 128)
    tape.backward(p, z, rt.State.zeros(2, sc.n_particles))


def test_autograd_trajectory_keeps_liquid():
    """The autograd trajectory of the coupled robot-and-liquid scene (the path
    the controller takes) simulates its liquid: the final state equals the tape
    API's with the scene's material ids and differs from the same run with
    every particle solid. The compression J - 1 of the liquid particles is
    compared: the controller's mean-x loss cannot tell the two apart, since
    internal forces cancel in the total momentum."""
    sc = scenes.coupled3d().with_steps(32)
    ctl = OpenLoopController(sc)
    act = ctl.sim.actuation(ctl.W.detach(), ctl.b.detach(), float(sc.act_omega), 32)
    liquid = np.asarray(sc.mat_id) == 1
    assert liquid.sum() > 1000

    def liquid_dJ(F):  # F: (3, 3, N) tensor
        J = np.linalg.det(np.transpose(F.detach().cpu().numpy().astype(np.float64), (2, 0, 1)))
        return J[liquid] - 1.0

    _, _, _, Fa = rt.trajectory(ctl.tape, ctl.init, ctl.params, act)
    got = liquid_dJ(Fa)
    out = {}
    for name, mat in (("liquid", ctl.params.mat_id), ("solid", None)):
        p = rt.params_for_scene(sc, act=act)
        p.mat_id = mat
        tape = ctl.sim.tape(32)
        fin = rt.State.empty(3, sc.n_particles)
        tape.forward(p, ctl.init, fin)
        out[name] = liquid_dJ(fin.F)
    d_same, d_model = rel(got, out["liquid"]), rel(out["solid"], out["liquid"])
    log(f"[autograd liquid] liquid J-1: rms {np.sqrt(np.mean(out['liquid'] ** 2)):.3g}; "
        f"autograd vs tape with liquid rel {d_same:.3g}; all solid vs liquid rel {d_model:.3g}")
    assert d_same <= 1e-3 and d_model >= 0.1
    L_ = ctl.loss()
    L_.backward()
    assert torch.isfinite(ctl.W.grad).all() and ctl.W.grad.abs().max() > 0
    assert ctl.sim.check_errors() == 0

"""Trajectory parity (tape forward + mean-position loss + tape backward) of the
HIP path against the FP64 oracle on the seeded workloads (GPU)."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import act_table, compare, cos, gpu_run, log, oracle_run, random_seed, rel

pytestmark = pytest.mark.gpu


def test_translate2d_closed_form_and_oracle():
    """translate2d is a rigid translation: every particle moves by (T dt, g dt^2 T(T+1)/2),
    dL/dv0 summed = (T dt, 0), dL/dE = 0."""
    sc = scenes.translate2d()
    T = sc.steps
    log(f"[translate2d] N={sc.n_particles} T={T}")
    g = gpu_run(sc, T)
    assert g["flags"] == 0
    shift = g["final"][0] - sc.x.astype(np.float64)
    dt = sc.dt
    expect = np.array([T * dt, sc.gravity * dt * dt * T * (T + 1) / 2])
    err = np.abs(shift - expect).max()
    gv_sum = g["g0"][1].sum(0)
    log(f"  max |shift - closed form| = {err:.3g}; sum dL/dv0 = {gv_sum}; dL/dE = {g['gE'][0]:.3g}")
    assert err < 2e-6
    np.testing.assert_allclose(gv_sum, [T * dt, 0.0], rtol=1e-4, atol=1e-6)
    assert abs(g["gE"][0]) < 1e-6
    o = oracle_run(sc, T)
    compare("translate2d", sc, g, o, grads=("v",), check_E=False)


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_deform2d_parity(lanes):
    """Deforming 2D body: mean-x loss gradients, then a random functional of the
    final state for every input block and E."""
    sc = scenes.deform2d()
    g = gpu_run(sc, sc.steps, knobs={"lanes": lanes})
    o = oracle_run(sc, sc.steps)
    compare("deform2d", sc, g, o, grads=("x", "v"), check_E=False)
    assert abs(o["gE"][0]) < 1e-15 and abs(g["gE"][0]) < 1e-6  # momentum conservation: dL/dE = 0
    w = random_seed(sc)
    g = gpu_run(sc, sc.steps, seed=w, knobs={"lanes": lanes})
    o = oracle_run(sc, sc.steps, seed=w)
    compare(f"deform2d random functional lanes={lanes}", sc, g, o, grads=("x", "v", "C", "F"))


@pytest.fixture(scope="module")
def elastic3d_oracle_64():
    sc = scenes.elastic3d().with_steps(64)
    return sc, oracle_run(sc, 64)


@pytest.mark.parametrize("knobs", [dict(block=64), dict(block=128), dict(block=256), dict(block=128, lanes=4),
                                   dict(block=256, lanes=2), dict(block=64, lanes=2, rotate=0), dict(block=192),
                                   dict(block=256, lanes=4, rotate=0), dict(block=128, lds=0, remap=1),
                                   dict(block=256, part=0), dict(block=64, lanes=4, part=0)])
def test_elastic3d_parity_64_steps(knobs, elastic3d_oracle_64):
    """3D workload elastic3d (64^3 grid, 32768 particles) gated at 64 steps, in each
    launch configuration."""
    sc, o = elastic3d_oracle_64
    g = gpu_run(sc, 64, knobs=knobs)
    compare(f"elastic3d@64 {knobs}", sc, g, o, grads=("v", "x"), check_E=False)


def test_checkpointed_matches_oracle():
    """Checkpoint-recompute (K=4) over 20 steps on a deforming 2D body."""
    sc = scenes.deform2d().with_steps(20)
    w = random_seed(sc, 7)
    g = gpu_run(sc, 20, K=4, seed=w)
    o = oracle_run(sc, 20, K=4, seed=w)
    compare("deform2d@20 K=4", sc, g, o, grads=("x", "v", "C", "F"))


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_batched2d_batched_subset(lanes):
    """A few scenes of the batched workload run as one batch. The bodies start
    at rest, so until they reach the floor (about step 100) they fall rigidly
    with F = I and no stress: nothing depends on E before contact."""
    full = scenes.batched2d(n_scenes=6, steps=64)
    g = gpu_run(full, 64, knobs={"lanes": lanes})
    o = oracle_run(full, 64)
    compare("batched2d[6]@64", full, g, o, grads=("v",), check_E=False)
    assert np.abs(o["gE"]).max() < 1e-12 and np.abs(g["gE"]).max() < 1e-6
    full = scenes.batched2d(n_scenes=6, steps=160)
    w = random_seed(full, 5)
    g = gpu_run(full, 160, seed=w, knobs={"lanes": lanes})
    o = oracle_run(full, 160, seed=w)
    compare("batched2d[6]@160 random functional", full, g, o, grads=("x", "v", "C", "F"))


@pytest.mark.parametrize("lanes,part", [(1, 1), (2, 1), (4, 1), (1, 0)])
def test_ragged_batch_with_empty_scenes(lanes, part):
    """Scenes with no particles (first, in the middle, last), a one-particle
    scene and scenes whose counts leave ragged workgroups, in one batch: loss
    terms, trajectories and gradients match the oracle; the empty scenes have
    zero loss terms and zero E gradients."""
    base = scenes.batched2d(n_scenes=4, steps=160)
    full = base.subset([0, 0, 1, 2, 3, 1, 2], [0, 1, 0, 37, 257, 10 ** 9, 0])
    log(f"[ragged] counts {list(np.diff(full.offsets))}, lanes {lanes}, part {part}")
    g = gpu_run(full, 64, knobs={"lanes": lanes, "part": part})
    o = oracle_run(full, 64)
    compare("ragged@64", full, g, o, grads=("v",), check_E=False)
    empty = np.diff(full.offsets) == 0
    assert np.all(g["loss"][empty] == 0) and np.all(o["loss"][empty] == 0)
    assert rel(g["loss"], o["loss"]) < 1e-5, (g["loss"], o["loss"])
    w = random_seed(full, 6)
    g = gpu_run(full, 160, seed=w, knobs={"lanes": lanes, "part": part})
    o = oracle_run(full, 160, seed=w)
    compare("ragged@160 random functional", full, g, o, grads=("x", "v", "C", "F"))
    assert np.all(g["gE"][empty] == 0) and np.all(o["gE"][empty] == 0)


@pytest.mark.parametrize("part", [0, 1])
def test_robot3d_partitions(part):
    """The 3D robot (uniform random particles, so runs of consecutive sorted
    particles straddle distant Morton blocks) over 48 steps with the plain and
    the aligned workgroup partition, both against the oracle."""
    sc = scenes.robot3d().with_steps(48)
    act = act_table(sc, 48)
    w = random_seed(sc, 8)
    g = gpu_run(sc, 48, act=act, seed=w, knobs={"block": 256, "part": part})
    o = oracle_run(sc, 48, act=act, seed=w)
    compare(f"robot3d@48 part={part}", sc, g, o, grads=("x", "v", "C", "F"))


@pytest.mark.parametrize("name,T,knobs", [("deform2d", 24, {"lanes": 1}), ("deform2d", 24, {"lanes": 4}),
                                          ("elastic3d", 32, {"block": 256}),
                                          ("robot3d", 32, {"block": 128, "lanes": 2})])
def test_corotated_parity(name, T, knobs):
    """Fixed-corotated stress (polar decomposition and its hand-written
    gradient) over whole trajectories: state, E and actuation gradients of a
    random functional against the oracle."""
    from dataclasses import replace
    sc = replace(scenes.make(name).with_steps(T), model=1)
    act = act_table(sc, T)
    w = random_seed(sc, 10)
    g = gpu_run(sc, T, act=act, seed=w, knobs=knobs)
    o = oracle_run(sc, T, act=act, seed=w)
    compare(f"{name}@{T} corotated {knobs}", sc, g, o, grads=("x", "v", "C", "F"))
    if act is not None:
        assert cos(g["gact"], o["gact"]) >= 0.999 and rel(g["gact"], o["gact"]) <= 1e-3


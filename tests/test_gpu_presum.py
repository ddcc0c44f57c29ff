"""Base-sorted run sums before the LDS scatter atomics (knob "presum"): the
tape sorts particles by stencil base and lanes that share a base add one sum
per run (GPU):
  - single forward and reverse steps against the oracle (2D and 3D, both
    constitutive models, liquid), as for the default scatter;
  - the order a tape keeps (mpm_sort_order) is the stable sort by scene and
    Morton code of the stencil base floor(x / dx - 1/2);
  - trajectories against the oracle (3D elastic body, the robot with its
    actuation gradient, batched 2D scenes) at the parity gates.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as orc
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import G_COS, G_REL, act_table, compare, cos, gpu_run, log, oracle_run, random_seed, rel

pytestmark = pytest.mark.gpu

KNOBS = {"presum": 1, "lanes": 1}


def _morton(c, bits):
    key = np.zeros(c.shape[0], np.int64)
    for b in range(bits - 1, -1, -1):
        for a in range(c.shape[1]):
            key = (key << 1) | ((c[:, a] >> b) & 1)
    return key


@pytest.mark.parametrize("dim", [2, 3])
def test_presum_sort_order_is_by_stencil_base(dim):
    sc = scenes.deform2d() if dim == 2 else scenes.elastic3d()
    sim = rt.Simulator.for_scene(sc, knobs=KNOBS)
    perm = sim.sort_order(rt.state_for_scene(sc)).cpu().numpy()
    g = np.asarray(sc.x, np.float32) * np.float32(1.0 / sc.dx) - np.float32(0.5)
    c = np.where(g >= 0, np.minimum(g, sc.n_grid - 1).astype(np.int64), 0)
    bits = int(np.ceil(np.log2(sc.n_grid)))
    want = np.argsort(_morton(c, bits), kind="stable")
    assert np.array_equal(perm, want)


@pytest.mark.parametrize("model,liquid", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("dim,n_keep", [(2, 1024), (3, 4099)])
def test_presum_single_steps(dim, n_keep, model, liquid):
    base = scenes.deform2d() if dim == 2 else scenes.elastic3d()
    idx = np.sort(np.random.default_rng(1).choice(base.n_particles, n_keep, replace=False))
    sc = replace(base, offsets=np.array([0, n_keep], np.int32), x=base.x[idx], v=base.v[idx], C=base.C[idx],
                 F=base.F[idx])
    sc = replace(scenes.random_state(sc, seed=10 + dim), model=model)
    if liquid:
        sc = replace(sc, mat_id=(np.arange(n_keep) % 2).astype(np.int32))
    # A one-step tape sorts by base, so the scatters run the run sums.
    S = 2 * dim + 2 * dim * dim
    w = np.random.default_rng(3).normal(size=(n_keep, S)).astype(np.float32).astype(np.float64)
    g = gpu_run(sc, 1, seed=w, knobs=KNOBS)
    assert g["flags"] == 0
    ref, err = orc.step_fwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F))
    assert err == 0
    ref = orc.unpack(ref, dim)
    rf = [rel(g["final"][k], ref[k]) for k in range(4)]
    rg, rE, _, err = orc.step_bwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F), w)
    rg = orc.unpack(rg, dim)
    cb = [cos(g["g0"][k], rg[k]) for k in range(4)]
    rb = [rel(g["g0"][k], rg[k]) for k in range(4)]
    eE = abs(g["gE"][0] - rE[0]) / abs(rE[0])
    log(f"[presum step] dim={dim} N={n_keep} model={model} liquid={liquid}: fwd rel {rf}; bwd cos {min(cb):.7f} "
        f"rel {max(rb):.3g}; dE rel {eE:.3g}")
    assert rf[0] < 2e-7 and max(rf[1:]) < 2e-5, rf
    assert min(cb) > 0.99999 and max(rb) < 1e-4 and eE < 1e-4


def test_presum_elastic3d_trajectory():
    sc = scenes.elastic3d().with_steps(64)
    w = random_seed(sc, 9)
    g = gpu_run(sc, 64, seed=w, knobs={**KNOBS, "block": 256, "part": 0})
    o = oracle_run(sc, 64, seed=w)
    compare("presum elastic3d@64 random functional", sc, g, o, grads=("x", "v", "C", "F"))


def test_presum_robot_trajectory():
    sc = scenes.robot3d().with_steps(48)
    act = act_table(sc, 48)
    g = gpu_run(sc, 48, act=act, knobs={**KNOBS, "block": 256, "part": 1})
    o = oracle_run(sc, 48, act=act)
    compare("presum robot3d@48", sc, g, o, grads=("x", "v"), check_E=False)
    assert cos(g["gact"], o["gact"]) >= G_COS and rel(g["gact"], o["gact"]) <= G_REL


def test_presum_batched_sampled():
    # Random v, C and F: at rest, a falling scene has dL/dE = 0 exactly
    # until it reaches the floor.
    sc = scenes.random_state(scenes.batched2d(n_scenes=64, steps=64), seed=3, v_scale=0.1)
    w = random_seed(sc, 13)
    g = gpu_run(sc, 64, seed=w, knobs={**KNOBS, "block": 256, "part": 0})
    assert g["flags"] == 0
    for k in (0, 31, 63):
        one = sc.subset([k])
        lo, hi = sc.offsets[k], sc.offsets[k + 1]
        o = oracle_run(one, 64, seed=w[lo:hi])
        gk = {"final": tuple(a[lo:hi] for a in g["final"]), "g0": tuple(a[lo:hi] for a in g["g0"]),
              "gE": g["gE"][k:k + 1], "flags": g["flags"]}
        compare(f"presum batched2d scene {k}", one, gk, o, grads=("x", "v", "C", "F"))

"""The persistent form of the tape's step launches (knob "persist": one
cooperative launch per direction, workgroups meeting at a grid-wide barrier
between the recorded step launches) against the oracle and against the
launch-per-step form (GPU):
  - the batched 2D workload, all 256 scenes over 256 steps: three sampled
    scenes against the oracle, at the parity gates;
  - per-launch vs persistent on the same inputs, 2D batched (both
    partitions) and 3D, lanes 1 and 2: final state and gradients agree to
    FP32 rounding (only the order of the flush atomics differs);
  - the timing knob counts the persistent launch's step launches.
"""
import numpy as np
import pytest
import torch

from paper_1910_00935_amd import _lib as L
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import compare, cos, gpu_run, log, oracle_run, random_seed, rel

pytestmark = pytest.mark.gpu


def test_persistent_batched_full_sampled():
    sc = scenes.batched2d()
    w = random_seed(sc, 13)
    g = gpu_run(sc, sc.steps, seed=w, knobs={"persist": 1, "part": 0, "block": 256})
    assert g["flags"] == 0
    for k in (0, 97, 255):
        one = sc.subset([k])
        lo, hi = sc.offsets[k], sc.offsets[k + 1]
        o = oracle_run(one, sc.steps, seed=w[lo:hi])
        gk = {"final": tuple(a[lo:hi] for a in g["final"]), "g0": tuple(a[lo:hi] for a in g["g0"]),
              "gE": g["gE"][k:k + 1], "flags": g["flags"]}
        compare(f"persistent batched2d scene {k} (N={hi - lo})", one, gk, o, grads=("x", "v", "C", "F"))


@pytest.mark.parametrize("name,knobs", [
    ("batched2d", {"part": 0, "block": 256}),
    ("batched2d", {"part": 1, "block": 128}),
    ("batched2d", {"part": 0, "block": 128, "lanes": 2}),
    ("elastic3d", {"part": 0, "block": 256}),
    ("robot3d", {"part": 1, "block": 128}),
])
def test_persistent_equals_launch_per_step(name, knobs):
    # Random v, C and F (stress from the first step): a scene falling at
    # rest would have dL/dE = 0 exactly, leaving nothing to compare.
    if name == "batched2d":
        sc = scenes.random_state(scenes.batched2d(n_scenes=32, steps=48), seed=3, v_scale=0.1)
    else:
        sc = scenes.make(name).with_steps(32)
    T = sc.steps
    w = random_seed(sc, 5)
    act = None
    if sc.n_act:
        import oracle as orc
        act = orc.actuation(sc.act_W, sc.act_b, sc.act_omega, sc.dt, T)
    a = gpu_run(sc, T, seed=w, act=act, knobs=dict(knobs))
    b = gpu_run(sc, T, seed=w, act=act, knobs={**knobs, "persist": 1})
    assert a["flags"] == 0 and b["flags"] == 0
    xr = rel(b["final"][0], a["final"][0])
    r = {k: (cos(b["g0"][i], a["g0"][i]), rel(b["g0"][i], a["g0"][i])) for i, k in enumerate("xvCF")}
    er = rel(b["gE"], a["gE"])
    log(f"[persist] {name} {knobs}: x rel {xr:.3g}; grads {r}; dL/dE {np.abs(a['gE']).max():.3g}, rel {er:.3g}")
    assert xr < 1e-6 and er < 1e-4 and np.abs(a["gE"]).max() > 1e-6
    for k, (c, e) in r.items():
        assert c > 0.99999 and e < 1e-4, (k, c, e)
    if act is not None:
        assert rel(b["gact"], a["gact"]) < 1e-4


def test_persistent_timing_counts_step_launches():
    sc = scenes.batched2d(n_scenes=8, steps=16)
    sim = rt.Simulator.for_scene(sc, knobs={"persist": 1, "timing": 1})
    gpu_run(sc, 16, sim=sim)
    fwd_ms, fwd_n = L.mpm_kernel_stats(sim.ctx, L.MPM_KERNEL_FWD)
    bwd_ms, bwd_n = L.mpm_kernel_stats(sim.ctx, L.MPM_KERNEL_BWD)
    log(f"[persist timing] fwd {fwd_ms:.3f} ms / {fwd_n}, bwd {bwd_ms:.3f} ms / {bwd_n}")
    # Forward: the recorded first scatter and 16 steps, plus the reverse
    # pass's first scatter (its own launch); reverse: 16 steps and the output.
    assert fwd_n == 17 + 1 and bwd_n == 17
    assert fwd_ms > 0 and bwd_ms > 0

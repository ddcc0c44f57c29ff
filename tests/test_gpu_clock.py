"""Workgroup wall clocks (mpm_wg_clock_bind / mpm_wg_clock_info), the
measurement behind the split of a step into workgroup work and launch
boundary (GPU):
  - a full-tape trajectory takes one row per step launch in enqueue order
    (forward: the first scatter and T steps; reverse: its first scatter, then
    T + 1 reverse launches), with every workgroup stamped once, start <= end;
  - launches on one stream do not overlap: each launch's first workgroup
    starts after the previous launch's last one ended, both when the tape
    launches directly and when it replays a captured graph;
  - clocks change no result; single steps take one row each; unbinding stops
    the stamping; rows stop when the buffer is full.
"""
import numpy as np
import pytest
import torch

from paper_1910_00935_amd import _lib as L
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import cos, gpu_run, log, random_seed, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph", [1, 0])
def test_trajectory_rows_and_order(graph):
    sc = scenes.make("elastic3d").with_steps(16)
    T = sc.steps
    sim = rt.Simulator.for_scene(sc, knobs={"block": 256, "lanes": 1, "part": 0, "graph": graph})
    w = random_seed(sc, 5)
    ref = gpu_run(sc, T, sim=sim, seed=w)
    sim.bind_wg_clock(sim.wg_clock_buffer(4 * T))
    g = gpu_run(sc, T, sim=sim, seed=w)
    recs = sim.wg_clock()
    sim.bind_wg_clock(None)
    assert g["flags"] == 0
    kinds = [k for k, _, _ in recs]
    assert kinds == [L.MPM_KERNEL_FWD] * (T + 2) + [L.MPM_KERNEL_BWD] * (T + 1), kinds
    n_fwd = len(recs[0][1])
    assert all(len(st) == n_fwd for k, st, _ in recs if k == L.MPM_KERNEL_FWD)
    for r, (k, st, en) in enumerate(recs):
        assert np.all(st > 0) and np.all(en >= st), r
        assert en.max() - st.min() < 1e4, r  # microseconds
        if r + 1 < len(recs):
            assert recs[r + 1][1].min() >= en.max(), (r, recs[r + 1][1].min() - en.max())
    span = [en.max() - st.min() for _, st, en in recs]
    gap = [recs[r + 1][1].min() - recs[r][2].max() for r in range(len(recs) - 1)]
    log(f"[wg clock] graph={graph}: span median {np.median(span):.2f} us, gap median {np.median(gap):.2f} us")
    # The clocks change no result (the flush atomics' order may differ run
    # to run: FP32 rounding only).
    r = [(cos(g["g0"][i], ref["g0"][i]), rel(g["g0"][i], ref["g0"][i])) for i in range(4)]
    log(f"[wg clock] graph={graph}: x rel {rel(g['final'][0], ref['final'][0]):.3g}, grads (cos, rel) {r}")
    assert rel(g["final"][0], ref["final"][0]) < 1e-6
    for i, (c, e) in enumerate(r):
        assert c > 0.99999 and e < 1e-4, (i, c, e)


def test_single_steps_and_unbind():
    sc = scenes.make("deform2d")
    sim = rt.Simulator.for_scene(sc)
    params = rt.params_for_scene(sc)
    a = rt.state_for_scene(sc)
    b = rt.State.empty(2, sc.n_particles)
    sim.bind_wg_clock(sim.wg_clock_buffer(8))
    for _ in range(3):
        sim.step_fwd(params, 0, a, b)
    recs = sim.wg_clock()
    # A single step is two launches: the scatter of `in`, then the gather.
    assert [k for k, _, _ in recs] == [L.MPM_KERNEL_FWD] * 6
    assert all(np.all(en >= st) and np.all(st > 0) for _, st, en in recs)
    sim.bind_wg_clock(None)
    sim.step_fwd(params, 0, a, b)
    assert sim.wg_clock() == []
    assert sim.check_errors() == 0


def test_rows_beyond_the_buffer_are_not_taken():
    sc = scenes.make("deform2d")
    sim = rt.Simulator.for_scene(sc)
    params = rt.params_for_scene(sc)
    a = rt.state_for_scene(sc)
    b = rt.State.empty(2, sc.n_particles)
    buf = sim.wg_clock_buffer(2)
    sim.bind_wg_clock(buf)
    for _ in range(5):
        sim.step_fwd(params, 0, a, b)
    assert len(sim.wg_clock()) == 2
    sim.bind_wg_clock(None)
    assert sim.check_errors() == 0

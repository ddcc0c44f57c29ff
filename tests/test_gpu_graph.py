"""Graph capture and replay of tape launch sequences (GPU): replays give the
same trajectories and gradients as direct launches, for full and
checkpointed tapes, for repeated backward passes after one forward, and when
buffers change (re-capture)."""
import numpy as np
import pytest
import torch

from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import cos, log, random_seed, rel
import oracle as orc

pytestmark = pytest.mark.gpu


def _run(sim, sc, tape, p, init, w, repeats=1):
    """forward + backward `repeats` times on the same buffers; returns outputs of each."""
    outs = []
    fin = rt.State.empty(sc.dim, sc.n_particles)
    seed = rt.State.from_particle_major(*orc.unpack(w, sc.dim))
    for _ in range(repeats):
        tape.forward(p, init, fin)
        g = rt.State.zeros(sc.dim, sc.n_particles)
        gE = torch.zeros(sc.n_scenes, device="cuda")
        tape.backward(p, seed, g, gE)
        outs.append((fin.to_particle_major()[0].copy(), g.to_particle_major(), gE.cpu().numpy().copy()))
    return outs


@pytest.mark.parametrize("K", [0, 4])
def test_graph_replay_matches_direct_launches(K):
    sc = scenes.deform2d().with_steps(24)
    w = random_seed(sc, 3)
    p = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    direct = rt.Simulator.for_scene(sc, knobs={"graph": 0})
    graphed = rt.Simulator.for_scene(sc, knobs={"graph": 1})
    ref = _run(direct, sc, direct.tape(24, K), p, init, w)[0]
    outs = _run(graphed, sc, graphed.tape(24, K), p, init, w, repeats=3)
    for n, (x, g, gE) in enumerate(outs):
        r = rel(x, ref[0])
        c = min(cos(g[k], ref[1][k]) for k in range(4))
        log(f"[graph K={K}] replay {n}: x rel {r:.3g}, grad cos {c:.8f}, dE {gE[0]:.6g} vs {ref[2][0]:.6g}")
        assert r < 1e-6 and c > 0.99999
        assert abs(gE[0] - ref[2][0]) <= 1e-4 * abs(ref[2][0])


def test_graph_repeated_backward_and_recapture():
    """Two backward passes after one forward (checkpointed: the second starts from
    a different ring state), then new state buffers (a new capture)."""
    sc = scenes.deform2d().with_steps(20)
    w = random_seed(sc, 4)
    p = rt.params_for_scene(sc)
    sim = rt.Simulator.for_scene(sc)
    tape = sim.tape(20, 4)
    init = rt.state_for_scene(sc)
    fin = rt.State.empty(2, sc.n_particles)
    seed = rt.State.from_particle_major(*orc.unpack(w, 2))
    tape.forward(p, init, fin)
    grads = []
    for _ in range(2):
        g = rt.State.zeros(2, sc.n_particles)
        tape.backward(p, seed, g)
        grads.append(g.to_particle_major())
    for k in range(4):
        assert cos(grads[0][k], grads[1][k]) > 0.99999
    init2 = rt.state_for_scene(sc)  # new buffers, same values
    fin2 = rt.State.empty(2, sc.n_particles)
    tape.forward(p, init2, fin2)
    g = rt.State.zeros(2, sc.n_particles)
    tape.backward(p, seed, g)
    assert rel(fin2.to_particle_major()[0], fin.to_particle_major()[0]) < 1e-6
    assert cos(g.to_particle_major()[1], grads[0][1]) > 0.99999
    assert sim.check_errors() == 0


def test_autotune_picks_and_caches(tmp_path):
    """The autotuner times each candidate, returns one of them, and reuses the
    cached answer for the same workload shape."""
    from paper_1910_00935_amd import autotune
    sc = scenes.deform2d().with_steps(8)
    space = {"block": (128, 64), "lanes": (1, 4), "rotate": (1,), "lds": (1,), "split": (1,)}
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(sc, cache=cache, space=space)
    assert best in autotune.candidates(space)
    again = autotune.tune(sc, cache=cache, space={"block": (256,)})  # cached: space not searched again
    assert again == best
    g = rt.Simulator.for_scene(sc, knobs=best)
    assert g.N == sc.n_particles


def test_launch_shape_change_between_trajectories():
    """One context, the launch shape changed between trajectories (the number
    of workgroups, hence the per-workgroup scatter boxes the reverse pass
    clears, changes): same trajectory and gradients as a fresh context."""
    sc = scenes.deform2d().with_steps(24)
    w = random_seed(sc, 5)
    p = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    sim = rt.Simulator.for_scene(sc, knobs={"block": 256})
    first = _run(sim, sc, sim.tape(24, 4), p, init, w)[0]
    sim.set_knob("block", 64)
    second = _run(sim, sc, sim.tape(24, 4), p, init, w)[0]
    fresh_sim = rt.Simulator.for_scene(sc, knobs={"block": 64})
    fresh = _run(fresh_sim, sc, fresh_sim.tape(24, 4), p, init, w)[0]
    assert rel(second[0], fresh[0]) < 1e-6
    assert min(cos(second[1][k], fresh[1][k]) for k in range(4)) > 0.99999
    assert rel(first[0], fresh[0]) < 1e-4
    assert sim.check_errors() == 0


def test_partition_change_between_trajectories():
    """One context, the workgroup partition switched between trajectories (plain,
    aligned, plain): same trajectories and gradients as fresh contexts."""
    sc = scenes.robot3d().with_steps(16)
    w = random_seed(sc, 6)
    p = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    sim = rt.Simulator.for_scene(sc, knobs={"block": 256, "part": 0})
    outs = []
    for part in (0, 1, 0):
        sim.set_knob("part", part)
        outs.append(_run(sim, sc, sim.tape(16, 4), p, init, w)[0])
    for part, got in zip((0, 1, 0), outs):
        fresh_sim = rt.Simulator.for_scene(sc, knobs={"block": 256, "part": part})
        ref = _run(fresh_sim, sc, fresh_sim.tape(16, 4), p, init, w)[0]
        assert rel(got[0], ref[0]) < 1e-6
        assert min(cos(got[1][k], ref[1][k]) for k in range(4)) > 0.99999
    assert sim.check_errors() == 0


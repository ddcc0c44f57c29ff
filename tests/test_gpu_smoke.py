"""Parity of the smoke simulator's HIP kernels (include/smoke.h) with the FP64
oracle (GPU), element by element:
  - one forward step and one reverse step on grids that span several tiles
    and end in a ragged tile (n = 17, 50, 110), for K = 0, 1, 6, 10 and 24
    Jacobi sweeps and every tile shape, with velocities of a fraction of a
    cell and of many cells (back-traced points wrapping around the grid);
  - the whole benchmark workload (110^2 grid, 100 steps, 6 sweeps; Table 2):
    final state, loss, and the gradient of the loss with respect to the
    initial velocity and smoke, in the launch configuration the benchmark
    times; also with 10 sweeps (Appendix E.3's count);
  - edge cases: the smallest grid (n = 4, one ragged tile), one step, a
    non-finite velocity (flagged; every index stays in the grid), and the
    accumulating gradient output.
Tolerances: single steps 2e-5 relative per plane (FP32 arithmetic of a few
dozen operations per cell); trajectories 1e-4 on the final state and cosine
0.999 / relative L2 1e-3 on gradients (the MPM path's gates).
"""
import numpy as np
import pytest
import torch

import oracle.smoke as sm
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import cos, log, rel

pytestmark = pytest.mark.gpu


def _state(sc):
    return [a.astype(np.float64) for a in (sc.u0, sc.u1, sc.s)]


def _gpu_traj(sc, tile=0, backward=True, seed=None):
    sim = rt.SmokeSim.for_scene(sc, tile=tile)
    init = rt.smoke_state(sc)
    fin = sim.forward(init)
    out = {"final": fin.cpu().numpy().astype(np.float64)}
    if backward:
        tgt = torch.as_tensor(sc.target, device="cuda")
        if seed is None:
            sd = torch.empty(3, sc.n, sc.n, device="cuda")
            out["loss"] = float(sim.loss(tgt, sd).item())
        else:
            sd = torch.as_tensor(seed, dtype=torch.float32, device="cuda").contiguous()
        g = torch.zeros(3, sc.n, sc.n, device="cuda")
        sim.backward(sd, g)
        out["grad"] = g.cpu().numpy().astype(np.float64)
    out["flags"] = sim.check_errors()
    return out


def _scene(n, iters, speed, seed=0, steps=1):
    return scenes.smoke(n=n, steps=steps, iters=iters, seed=seed, speed=speed)


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("iters", [0, 1, 6, 10, 24])
@pytest.mark.parametrize("n,speed", [(17, 0.6), (50, 4.0), (110, 0.5)])
def test_step_matches_oracle(n, speed, iters, tile):
    sc = _scene(n, iters, speed, seed=n + iters)
    rng = np.random.default_rng(n + 3 * iters)
    seed = rng.normal(size=(3, n, n)).astype(np.float32)
    g = _gpu_traj(sc, tile=tile, seed=seed)
    assert g["flags"] == 0
    u0, u1, s = _state(sc)
    ref = sm.step(u0, u1, s, iters)
    gref = sm.step_adj(u0, u1, s, *seed.astype(np.float64), iters)
    rf = [rel(g["final"][k], ref[k]) for k in range(3)]
    rg = [rel(g["grad"][k], gref[k]) for k in range(3)]
    cg = [cos(g["grad"][k], gref[k]) for k in range(3)]
    log(f"[smoke step] n={n} speed={speed} K={iters} tile={tile}: fwd rel {max(rf):.2g}, "
        f"bwd rel {max(rg):.2g} cos {min(cg):.7f}")
    assert max(rf) < 2e-5, rf
    assert max(rg) < 2e-5 and min(cg) > 0.99999, (rg, cg)


@pytest.mark.parametrize("iters", [6, 10])
def test_benchmark_trajectory_matches_oracle(iters):
    sc = scenes.smoke(iters=iters)
    g = _gpu_traj(sc)
    assert g["flags"] == 0
    st = sm.forward(*_state(sc), sc.steps, sc.iters)
    tgt = sc.target.astype(np.float64)
    loss = sm.loss(st[-1][2], tgt)
    go = sm.backward(st, np.zeros((sc.n, sc.n)), np.zeros((sc.n, sc.n)), sm.loss_seed(st[-1][2], tgt), sc.iters)
    rf = [rel(g["final"][k], st[-1][k]) for k in range(3)]
    rl = abs(g["loss"] - loss) / loss
    r = {name: (cos(g["grad"][k], go[k]), rel(g["grad"][k], go[k])) for k, name in enumerate(("u0", "u1", "s"))}
    log(f"[smoke 110^2 x {sc.steps}, K={iters}] final rel {rf}; loss {g['loss']:.6f} vs {loss:.6f} (rel {rl:.2g}); "
        f"gradients (cos, rel) {r}")
    assert max(rf) < 1e-4 and rl < 1e-5
    for name, (c, e) in r.items():
        assert c >= 0.999 and e <= 1e-3, (name, c, e)


def test_smallest_grid_and_accumulation():
    sc = _scene(4, 6, 0.7, seed=5, steps=3)
    sim = rt.SmokeSim.for_scene(sc)
    sim.forward(rt.smoke_state(sc))
    seed = torch.as_tensor(np.random.default_rng(6).normal(size=(3, 4, 4)), dtype=torch.float32,
                           device="cuda").contiguous()
    g = torch.zeros(3, 4, 4, device="cuda")
    sim.backward(seed, g)
    once = g.clone()
    sim.backward(seed, g)  # accumulates
    st = sm.forward(*_state(sc), 3, 6)
    go = sm.backward(st, *seed.cpu().numpy().astype(np.float64), 6)
    assert rel(sim.tape[3].cpu().numpy(), np.stack(st[-1])) < 1e-5
    assert rel(once.cpu().numpy(), np.stack(go)) < 1e-4
    assert rel(g.cpu().numpy(), 2 * once.cpu().numpy()) < 1e-6
    assert sim.check_errors() == 0


def test_nonfinite_velocity_is_flagged():
    sc = _scene(24, 6, 0.5, seed=9, steps=2)
    u0 = sc.u0.copy()
    u0[5, 7] = np.nan
    u1 = sc.u1.copy()
    u1[11, 3] = np.inf
    from dataclasses import replace
    bad = replace(sc, u0=u0, u1=u1)
    sim = rt.SmokeSim.for_scene(bad)
    sim.forward(rt.smoke_state(bad))
    flags = sim.check_errors()
    log(f"[smoke nonfinite] flags {flags}")
    assert flags & 4
    assert sim.check_errors() == 0  # cleared on read

"""The 3D actuated soft robot (a crawler with 16 actuators, 30000 particles on a
64^3 grid) on the GPU: trajectory, actuation and weight gradients against the
FP64 oracle at full particle count, and a few open-loop controller
optimisation iterations through the torch autograd path."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes
from paper_1910_00935_amd.controller import OpenLoopController

from parity import G_COS, G_REL, act_table, compare, cos, gpu_run, log, oracle_run, random_seed, rel

pytestmark = pytest.mark.gpu


def test_robot3d_parity():
    T = 256
    sc = scenes.robot3d().with_steps(T)
    log(f"[robot3d] N={sc.n_particles} T={T} actuators={sc.n_act}")
    sim = rt.Simulator.for_scene(sc)
    W = torch.as_tensor(sc.act_W, device="cuda")
    b = torch.as_tensor(sc.act_b, device="cuda")
    act_gpu = sim.actuation(W, b, sc.act_omega, T)
    act = act_table(sc, T)
    np.testing.assert_allclose(act_gpu.cpu().numpy(), act, atol=2e-6)
    g = gpu_run(sc, T, act=act_gpu.cpu().numpy(), sim=sim)
    o = oracle_run(sc, T, act=act)
    log(f"  oracle {o['seconds']:.1f} s")
    compare("robot3d@256", sc, g, o, grads=("x", "v", "C", "F"), check_E=False)
    gW = torch.zeros_like(W)
    gb = torch.zeros_like(b)
    sim.actuation_bwd(W, b, sc.act_omega, T, torch.as_tensor(g["gact"], dtype=torch.float32, device="cuda"), gW, gb)
    oW, ob = orc.actuation_bwd(sc.act_W, sc.act_b, sc.act_omega, sc.dt, T, o["gact"])
    gwb = np.concatenate([gW.cpu().numpy().ravel(), gb.cpu().numpy().ravel()])
    owb = np.concatenate([oW.ravel(), ob.ravel()])
    log(f"  dL/d(W,b): cos={cos(gwb, owb):.6f} rel={rel(gwb, owb):.3g}; dL/da cos={cos(g['gact'], o['gact']):.6f} "
        f"rel={rel(g['gact'], o['gact']):.3g}")
    assert cos(g["gact"], o["gact"]) >= G_COS and rel(g["gact"], o["gact"]) <= G_REL
    assert cos(gwb, owb) >= G_COS and rel(gwb, owb) <= G_REL


def test_robot3d_autograd_gradient_and_optimisation():
    """The controller's autograd gradient equals the explicit tape + actuation
    adjoint calls, and normalised gradient descent lowers the loss."""
    sc = scenes.robot3d()
    ctl = OpenLoopController(sc)
    L0 = ctl.loss()
    L0.backward()
    gW_auto, gb_auto = ctl.W.grad.clone(), ctl.b.grad.clone()
    # Same gradient through the explicit calls.
    T = sc.steps
    g = gpu_run(sc, T, act=ctl.sim.actuation(ctl.W.detach(), ctl.b.detach(), sc.act_omega, T).cpu().numpy(),
                sim=ctl.sim)
    gW = torch.zeros_like(gW_auto)
    gb = torch.zeros_like(gb_auto)
    ctl.sim.actuation_bwd(ctl.W.detach(), ctl.b.detach(), sc.act_omega, T,
                          torch.as_tensor(g["gact"], dtype=torch.float32, device="cuda"), gW, gb)
    a = torch.cat([gW_auto.ravel(), gb_auto.ravel()]).cpu().numpy()
    e = torch.cat([gW.ravel(), gb.ravel()]).cpu().numpy()
    log(f"[robot3d] loss {float(L0):.6f} vs {g['loss'][0]:.6f}; autograd vs explicit gradient rel {rel(a, e):.3g}")
    assert abs(float(L0) - g["loss"][0]) <= 1e-6 * abs(g["loss"][0])
    assert rel(a, e) <= 1e-5
    hist = ctl.optimize(iters=4, lr=0.05)
    log(f"  losses {['%.6f' % v for v in hist]}")
    assert hist[1] < hist[0] and hist[-1] < hist[0]


@pytest.mark.parametrize("part", [1, 0])
def test_coupled_robot_and_liquid(part):
    """The robot beside 13000 liquid particles (43000 in all), two-way coupled
    through the grid, over 48 steps: trajectory, state, E and actuation
    gradients of a random functional against the oracle."""
    T = 48
    sc = scenes.coupled3d().with_steps(T)
    act = act_table(sc, T)
    w = random_seed(sc, 12)
    g = gpu_run(sc, T, act=act, seed=w, knobs={"block": 128, "part": part})
    o = oracle_run(sc, T, act=act, seed=w)
    log(f"  oracle {o['seconds']:.1f} s")
    compare(f"coupled3d@{T} part={part}", sc, g, o, grads=("x", "v", "C", "F"))
    assert cos(g["gact"], o["gact"]) >= G_COS and rel(g["gact"], o["gact"]) <= G_REL


"""Open-loop controller optimisation through the differentiable trajectory.

The soft robots of the paper's elastic-object simulator (Section 4.1; the 2D
robot with four muscles and the 3D crawler with 16, Appendix E.1) are driven by
an open-loop signal a_k(s) = tanh(sum_j W_kj sin(omega s dt + 2 pi j / n_sin)
+ b_k) whose weights are trained by gradient descent on a loss of the final
state. Here the signal (``runtime.Actuation``), the trajectory
(``runtime.MPMTrajectory``: tape forward, reverse replay) and the loss are
torch autograd functions, so the weights are ordinary leaf tensors; every
step of the simulation and of its adjoint runs in the HIP library.
"""
from __future__ import annotations

from typing import List, Optional

import torch

from . import runtime as rt


class OpenLoopController:
    """Weights W [n_act, n_sin] and b [n_act] of the open-loop signal of an
    actuated scene, with the tape that evaluates the mean-position loss
    sign * mean_p x_{p,axis}(T) and its gradient."""

    def __init__(self, scene, sim: Optional[rt.Simulator] = None, knobs=None, ckpt_every: int = 0):
        if not scene.n_act:
            raise ValueError(f"scene {scene.name} has no actuators")
        self.scene = scene
        self.sim = sim or rt.Simulator.for_scene(scene, knobs=knobs)
        self.T = int(scene.steps)
        self.tape = self.sim.tape(self.T, ckpt_every)
        self.init = rt.state_for_scene(scene)
        self.params = rt.params_for_scene(scene)
        self.W = torch.tensor(scene.act_W, dtype=torch.float32, device=self.sim.device, requires_grad=True)
        self.b = torch.tensor(scene.act_b, dtype=torch.float32, device=self.sim.device, requires_grad=True)

    def loss(self) -> torch.Tensor:
        """Differentiable loss of one trajectory under the current weights."""
        sc, p = self.scene, self.params
        act = rt.Actuation.apply(self.sim, self.W, self.b, float(sc.act_omega), self.T)
        xT, _, _, _ = rt.MPMTrajectory.apply(self.tape, p, self.init.x, self.init.v, self.init.C, self.init.F, p.E,
                                             act)
        return float(sc.loss_sign) * xT[int(sc.loss_axis)].mean()

    def step(self, lr: float, normalize: bool = True) -> float:
        """One gradient-descent iteration; returns the loss before the update.
        With ``normalize`` the update has length lr in the joint (W, b) space."""
        self.W.grad = None
        self.b.grad = None
        L = self.loss()
        L.backward()
        with torch.no_grad():
            gW, gb = self.W.grad, self.b.grad
            scale = lr
            if normalize:
                norm = torch.sqrt((gW * gW).sum() + (gb * gb).sum())
                scale = lr / max(float(norm), 1e-30)
            self.W -= scale * gW
            self.b -= scale * gb
        return float(L)

    def optimize(self, iters: int, lr: float, normalize: bool = True) -> List[float]:
        """``iters`` iterations; returns the loss before each and after the last."""
        hist = [self.step(lr, normalize) for _ in range(iters)]
        with torch.no_grad():
            hist.append(float(self.loss()))
        err = self.sim.check_errors()
        if err:
            raise RuntimeError(f"simulation error flags {err:#x} during optimisation")
        return hist

"""FP64 NumPy oracle of the differentiable incompressible smoke simulator
(DiffTaichi, Section 4.2 "smoke", Table 2; Appendix E.3 on backpropagating
through the pressure projection) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module. The GPU path shares no code with it.

What it computes. The paper builds the simulator after the fluid example of
Autograd: semi-Lagrangian advection (Stam 1999, "Stable Fluids") and a
pressure projection by a fixed number of Jacobi iterations, on a periodic
square grid, with gradients taken through the unrolled iterations. Restated
here from those methods (collocated grid, one value per cell, lengths in
cells, velocities in cells per time step):

    advect(f, u)(c) = f sampled bilinearly at c - u(c), indices wrapped mod n
    div(u)(c)       = (u0[c + e0] - u0[c - e0] + u1[c + e1] - u1[c - e1]) / 2
    p^0 = 0,  p^k(c) = (p^{k-1}[c + e0] + p^{k-1}[c - e0]
                        + p^{k-1}[c + e1] + p^{k-1}[c - e1] - div(u)(c)) / 4
    project(u)      = u - grad(p^K),  grad(p)(c) = ((p[c + e0] - p[c - e0]) / 2,
                                                   (p[c + e1] - p[c - e1]) / 2)
    one step:  u* = advect(u, u) (each component);  u' = project(u*);
               s' = advect(s, u')
    loss:      L = sum_c (s_T(c) - target(c))^2

Jacobi solves the 5-point Poisson equation lap(p) = div(u*); with p^0 = 0,
K iterations give the truncated Neumann series of that solve. Readings (the
paper is silent or inconsistent; each one is listed in the design notes): the
iteration count K is a parameter (Table 2 states 6 per step, Appendix E.3
states 10); the grid is square and periodic (Section 4.2 says periodic);
velocities are in cells per step (the grid spacing cancels out of the
projection); p starts from zero every step; the loss is the summed squared
difference to a target density.

The adjoint of every stage is written by hand and accumulates: for a primal
f(X) = Y the adjoint takes (X, Y*) and returns X* = dL/dX. Arrays may be
complex: the forward map then carries complex-step tangents (the cell index
of a sample is taken from the real part), which is how the adjoint is pinned.
The one decision floating point makes for an integer here, the cell a
back-traced point falls in, is taken in single precision (_sample_points).

Arrays are (n, n), axis 0 first; a velocity is the pair (u0, u1).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Semi-Lagrangian advection
# ---------------------------------------------------------------------------
def _sample_points(u0, u1):
    """Cell indices (a, b) of the lower corner and fractions (fa, fb) of the
    back-traced point c - u(c) of every cell c. Which cell a point falls in
    is decided in single precision, the precision of the paper's GPU runs
    (Table 2) and of the kernels: floor(fl32(c - fl32(u))). Within rounding
    of a cell boundary the fraction may then lie a rounding error outside
    [0, 1); the bilinear form is continuous there, and both sides take the
    same cell, hence the same derivative of the sample."""
    n = u0.shape[0]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    y0 = i - u0
    y1 = j - u1
    a = np.floor(i.astype(np.float32) - np.real(u0).astype(np.float32)).astype(np.int64)
    b = np.floor(j.astype(np.float32) - np.real(u1).astype(np.float32)).astype(np.int64)
    return a, b, y0 - a, y1 - b


def advect(f, u0, u1):
    """f sampled bilinearly at c - u(c) for every cell c (periodic)."""
    n = f.shape[0]
    a, b, fa, fb = _sample_points(u0, u1)
    a0, a1, b0, b1 = a % n, (a + 1) % n, b % n, (b + 1) % n
    return ((1 - fa) * (1 - fb) * f[a0, b0] + (1 - fa) * fb * f[a0, b1]
            + fa * (1 - fb) * f[a1, b0] + fa * fb * f[a1, b1])


def advect_adj(f, u0, u1, g):
    """Adjoint of advect at (f, u) for the output adjoint g: returns
    (f*, u0*, u1*), f* scattered back to the four cells of every sample,
    u* = -g grad_y(sample) at each cell."""
    n = f.shape[0]
    a, b, fa, fb = _sample_points(u0, u1)
    a0, a1, b0, b1 = a % n, (a + 1) % n, b % n, (b + 1) % n
    gf = np.zeros_like(f * g)
    for ia, ib, w in ((a0, b0, (1 - fa) * (1 - fb)), (a0, b1, (1 - fa) * fb),
                      (a1, b0, fa * (1 - fb)), (a1, b1, fa * fb)):
        np.add.at(gf, (ia, ib), w * g)
    # d(sample)/dy0 and d(sample)/dy1 at the back-traced point; y = c - u.
    dy0 = (1 - fb) * (f[a1, b0] - f[a0, b0]) + fb * (f[a1, b1] - f[a0, b1])
    dy1 = (1 - fa) * (f[a0, b1] - f[a0, b0]) + fa * (f[a1, b1] - f[a1, b0])
    return gf, -g * dy0, -g * dy1


# ---------------------------------------------------------------------------
# Pressure projection (central differences, Jacobi on the 5-point Laplacian)
# ---------------------------------------------------------------------------
def _shift(p, axis, k):
    """q[c] = p[c + k e_axis] (periodic)."""
    return np.roll(p, -k, axis=axis)


def divergence(u0, u1):
    return (_shift(u0, 0, 1) - _shift(u0, 0, -1) + _shift(u1, 1, 1) - _shift(u1, 1, -1)) / 2


def divergence_adj(g):
    """Adjoint of divergence: (u0*, u1*) for the output adjoint g."""
    return (_shift(g, 0, -1) - _shift(g, 0, 1)) / 2, (_shift(g, 1, -1) - _shift(g, 1, 1)) / 2


def gradient(p):
    return (_shift(p, 0, 1) - _shift(p, 0, -1)) / 2, (_shift(p, 1, 1) - _shift(p, 1, -1)) / 2


def gradient_adj(g0, g1):
    """Adjoint of gradient: p* for the output adjoints (g0, g1)."""
    return (_shift(g0, 0, -1) - _shift(g0, 0, 1) + _shift(g1, 1, -1) - _shift(g1, 1, 1)) / 2


def neighbour_sum(p):
    return _shift(p, 0, 1) + _shift(p, 0, -1) + _shift(p, 1, 1) + _shift(p, 1, -1)


def jacobi(d, iters):
    """p^K of the Jacobi iteration for lap(p) = d from p^0 = 0."""
    p = np.zeros_like(d)
    for _ in range(iters):
        p = (neighbour_sum(p) - d) / 4
    return p


def jacobi_adj(g, iters):
    """Adjoint of jacobi with respect to d for the output adjoint g. Each
    iteration p^k = (S p^{k-1} - d) / 4 is linear; S (the neighbour sum) is
    symmetric, so the adjoint runs the same recursion backwards."""
    gd = np.zeros_like(g)
    gp = g
    for _ in range(iters):
        gd = gd - gp / 4
        gp = neighbour_sum(gp) / 4
    return gd


def project(u0, u1, iters):
    p = jacobi(divergence(u0, u1), iters)
    g0, g1 = gradient(p)
    return u0 - g0, u1 - g1


def project_adj(g0, g1, iters):
    """Adjoint of project (linear): (u0*, u1*) for the output adjoints."""
    gp = -gradient_adj(g0, g1)
    gd = jacobi_adj(gp, iters)
    d0, d1 = divergence_adj(gd)
    return g0 + d0, g1 + d1


# ---------------------------------------------------------------------------
# Time step, trajectory, loss
# ---------------------------------------------------------------------------
def step(u0, u1, s, iters):
    """One step: self-advection of the velocity, projection, advection of the
    smoke by the projected velocity."""
    w0 = advect(u0, u0, u1)
    w1 = advect(u1, u0, u1)
    v0, v1 = project(w0, w1, iters)
    return v0, v1, advect(s, v0, v1)


def step_adj(u0, u1, s, g0, g1, gs, iters):
    """Adjoint of step at state (u0, u1, s), given the adjoints (g0, g1, gs)
    of the next state; returns the adjoints of (u0, u1, s). The forward is
    recomputed from the state (nothing of the step is stored)."""
    w0 = advect(u0, u0, u1)
    w1 = advect(u1, u0, u1)
    v0, v1 = project(w0, w1, iters)
    # s' = advect(s, v)
    gs_prev, gv0, gv1 = advect_adj(s, v0, v1, gs)
    gv0 = gv0 + g0
    gv1 = gv1 + g1
    # v = project(w)
    gw0, gw1 = project_adj(gv0, gv1, iters)
    # w_a = advect(u_a, u): u enters as the field and as the velocity
    f0, a0, b0 = advect_adj(u0, u0, u1, gw0)
    f1, a1, b1 = advect_adj(u1, u0, u1, gw1)
    return f0 + a0 + a1, f1 + b0 + b1, gs_prev


def forward(u0, u1, s, steps, iters):
    """States 0..steps as a list of (u0, u1, s)."""
    states = [(u0, u1, s)]
    for _ in range(steps):
        states.append(step(*states[-1], iters))
    return states


def backward(states, g0, g1, gs, iters):
    """Adjoints of state 0 given those of the last state of `states`."""
    for u0, u1, s in reversed(states[:-1]):
        g0, g1, gs = step_adj(u0, u1, s, g0, g1, gs, iters)
    return g0, g1, gs


def loss(s_final, target):
    return np.sum((s_final - target) ** 2)


def loss_seed(s_final, target):
    """dL/ds_T of the summed squared difference."""
    return 2 * (s_final - target)

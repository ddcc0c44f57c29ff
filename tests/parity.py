"""Helpers shared by the GPU parity tests: run a scene through the HIP library
(C ABI via the torch runtime) and through the FP64 oracle on the same seeded
inputs, and compare with the tolerances of the parity gates:
  x after the gated horizon: ||x_gpu - x_orc|| / ||x_orc|| <= 1e-4;
  gradients: cosine >= 0.999 and ||g_gpu - g_orc|| / ||g_orc|| <= 1e-3.
Norm gates over many particles cannot see one particle that is far off, so
each comparison also gates per particle:
  max_p |x_gpu,p - x_orc,p| / dx <= 1e-2 (one hundredth of a cell);
  max_p |g_gpu,p - g_orc,p| / rms_p |g_orc,p| <= 5e-2 for each gradient tensor
  (|.| the particle's block, e.g. its 3 x 3 dL/dF).
"""
from __future__ import annotations

import sys
import time

import numpy as np
import torch

import oracle as orc
from paper_1910_00935_amd import runtime as rt

X_REL = 1e-4
G_COS = 0.999
G_REL = 1e-3
X_MAX_CELLS = 1e-2
G_MAX_RMS = 5e-2


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def cos(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    if na == 0 and nb == 0:
        return 1.0
    return float(a @ b / (na * nb))


def max_dx_cells(a, b, dx):
    """Largest per-particle position error, in cells."""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return float(np.sqrt((d.reshape(d.shape[0], -1) ** 2).sum(1)).max() / dx) if d.size else 0.0


def max_rms(a, b):
    """Largest per-particle error of a gradient tensor over the RMS of the
    reference's per-particle norms (0 when both are zero)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = a.shape[0]
    if n == 0:
        return 0.0
    err = np.sqrt(((a - b).reshape(n, -1) ** 2).sum(1))
    rms = np.sqrt(((b.reshape(n, -1) ** 2).sum(1)).mean())
    if rms == 0.0:
        return 0.0 if err.max() == 0.0 else float("inf")
    return float(err.max() / rms)


def act_table(scene, T):
    if not scene.n_act:
        return None
    return orc.actuation(scene.act_W, scene.act_b, scene.act_omega, scene.dt, T)


def random_seed(scene, seed=123):
    """A random linear functional of the final state, (N, S) float32-exact values.
    Mean-position losses do not depend on E while no particle touches a sticky
    node (total momentum changes only through gravity), so E-gradients are
    compared on such a functional."""
    S = 2 * scene.dim + 2 * scene.dim * scene.dim
    w = np.random.default_rng(seed).normal(size=(scene.n_particles, S)) / np.sqrt(scene.n_particles)
    return w.astype(np.float32).astype(np.float64)


def oracle_run(scene, T, K=None, act=None, backward=True, seed=None):
    st = orc.pack(scene.x, scene.v, scene.C, scene.F)
    t0 = time.time()
    sT, _, e1 = orc.run_fwd(scene, T, st, act=act)
    out = {"final": orc.unpack(sT, scene.dim), "err": e1}
    L, seed_l = orc.loss_mean_pos(scene, sT, scene.loss_axis, scene.loss_sign)
    seed = seed_l if seed is None else seed
    out["loss"] = L
    if backward:
        g0, gE, gact, e2 = orc.run_bwd(scene, T, K or T, st, seed, act=act)
        out.update(g0=orc.unpack(g0, scene.dim), gE=gE, gact=gact, err=e1 | e2)
    out["seconds"] = time.time() - t0
    return out


def gpu_run(scene, T, K=0, act=None, knobs=None, backward=True, sim=None, seed=None):
    """Tape forward, mean-position loss and seed, tape backward on the GPU.
    `seed` (N, S) replaces the loss seed with a given dL/dstate(T)."""
    sim = sim or rt.Simulator.for_scene(scene, knobs=knobs)
    act_t = None if act is None else torch.as_tensor(np.asarray(act, np.float32), device="cuda")
    params = rt.params_for_scene(scene, act=act_t)
    init = rt.state_for_scene(scene)
    tape = sim.tape(T, K)
    final = rt.State.empty(scene.dim, scene.n_particles)
    tape.forward(params, init, final)
    seed_s = rt.State.empty(scene.dim, scene.n_particles)
    loss = sim.loss_mean(final, scene.loss_axis, scene.loss_sign, seed_s)
    if seed is not None:
        seed_s = rt.State.from_particle_major(*orc.unpack(seed, scene.dim))
    out = {"final": final.to_particle_major(), "loss": loss.cpu().numpy()}
    if backward:
        ig = rt.State.zeros(scene.dim, scene.n_particles)
        gE = torch.zeros(scene.n_scenes, device="cuda")
        gact = torch.zeros(T, scene.n_act, device="cuda") if act is not None else None
        tape.backward(params, seed_s, ig, gE, gact)
        out.update(g0=ig.to_particle_major(), gE=gE.cpu().numpy().astype(np.float64),
                   gact=None if gact is None else gact.cpu().numpy().astype(np.float64))
    out["flags"] = sim.check_errors()
    return out


def compare(name, scene, g, o, grads=("v",), check_E=True, x_rel=X_REL):
    """Asserts the parity gates; returns the measured figures."""
    x0 = scene.x.astype(np.float64)
    xg, xo = g["final"][0], o["final"][0]
    r = {"x_rel": rel(xg, xo), "disp_rel": rel(xg - x0, xo - x0), "x_max_cells": max_dx_cells(xg, xo, scene.dx)}
    names = dict(x=0, v=1, C=2, F=3)
    for k in grads:
        gg, go = g["g0"][names[k]], o["g0"][names[k]]
        r[f"g{k}_cos"] = cos(gg, go)
        r[f"g{k}_rel"] = rel(gg, go)
        r[f"g{k}_max_rms"] = max_rms(gg, go)
    if check_E:
        r["gE_rel"] = rel(g["gE"], o["gE"])
    log(f"[parity] {name}: " + ", ".join(f"{k}={v:.3g}" for k, v in r.items()))
    assert g["flags"] == 0 and o["err"] == 0, (g["flags"], o["err"])
    assert r["x_rel"] <= x_rel, r
    assert r["x_max_cells"] <= X_MAX_CELLS, r
    for k in grads:
        assert r[f"g{k}_cos"] >= G_COS and r[f"g{k}_rel"] <= G_REL, (k, r)
        assert r[f"g{k}_max_rms"] <= G_MAX_RMS, (k, r)
    if check_E:
        assert r["gE_rel"] <= G_REL, r
    return r

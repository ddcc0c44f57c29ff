"""Single-step parity of the HIP kernels against the FP64 oracle (GPU).

Random generic states (random v, C and F = I + 0.05 N(0,1)) exercise every
term of the step. Each case covers several workgroups and a ragged tail."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_1910_00935_amd import runtime as rt
from paper_1910_00935_amd import scenes

from parity import cos, log, rel

pytestmark = pytest.mark.gpu


def _case(dim, n_keep, model=0, liquid=False):
    base = scenes.deform2d() if dim == 2 else scenes.elastic3d()
    if n_keep < base.n_particles:
        idx = np.sort(np.random.default_rng(1).choice(base.n_particles, n_keep, replace=False))
        base = base.subset([0])
        from dataclasses import replace
        base = replace(base, offsets=np.array([0, n_keep], np.int32), x=base.x[idx], v=base.v[idx],
                       C=base.C[idx], F=base.F[idx])
    from dataclasses import replace as _replace
    sc = _replace(scenes.random_state(base, seed=10 + dim), model=model)
    if liquid:  # every other particle is the weakly compressible liquid
        sc = _replace(sc, mat_id=(np.arange(sc.n_particles) % 2).astype(np.int32))
    return sc


@pytest.mark.parametrize("model,liquid", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("dim,n_keep", [(2, 1024), (2, 777), (3, 4099)])
def test_step_fwd_matches_oracle(dim, n_keep, lanes, model, liquid):
    sc = _case(dim, n_keep, model, liquid)
    log(f"[step_fwd] dim={dim} N={sc.n_particles} lanes={lanes} model={model} liquid={liquid}")
    sim = rt.Simulator.for_scene(sc, knobs={"lanes": lanes})
    p = rt.params_for_scene(sc)
    s_in = rt.state_for_scene(sc)
    s_out = rt.State.empty(dim, sc.n_particles)
    sim.step_fwd(p, 0, s_in, s_out)
    assert sim.check_errors() == 0
    got = s_out.to_particle_major()
    ref, err = orc.step_fwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F))
    assert err == 0
    ref = orc.unpack(ref, dim)
    # x' = x + dt v' is stored in FP32: x itself is compared (a one-step
    # displacement of ~3e-4 on x ~ 0.4 has only ~1e-4 relative resolution).
    r = [rel(got[k], ref[k]) for k in range(4)]
    log(f"  rel errors (x, v, C, F): {r}")
    assert r[0] < 2e-7 and max(r[1:]) < 2e-5, r


@pytest.mark.parametrize("model,liquid", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("dim,n_keep", [(2, 1024), (2, 777), (3, 4099)])
def test_step_bwd_matches_oracle(dim, n_keep, lanes, model, liquid):
    sc = _case(dim, n_keep, model, liquid)
    log(f"[step_bwd] dim={dim} N={sc.n_particles} lanes={lanes} model={model} liquid={liquid}")
    S = 2 * dim + 2 * dim * dim
    gout = np.random.default_rng(3).normal(size=(sc.n_particles, S))
    gx, gv, gC, gF = orc.unpack(gout, dim)
    sim = rt.Simulator.for_scene(sc, knobs={"lanes": lanes})
    p = rt.params_for_scene(sc)
    s_in = rt.state_for_scene(sc)
    og = rt.State.from_particle_major(gx, gv, gC, gF)
    ig = rt.State.zeros(dim, sc.n_particles)
    gE = torch.zeros(1, device="cuda")
    sim.step_bwd(p, 0, s_in, og, ig, gE)
    assert sim.check_errors() == 0
    got = ig.to_particle_major()
    # Round the seed to float32 exactly as the GPU saw it.
    gout32 = orc.pack(*[a.astype(np.float32) for a in (gx, gv, gC, gF)])
    ref, rE, _, err = orc.step_bwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F), gout32)
    assert err == 0
    ref = orc.unpack(ref, dim)
    for k, name in enumerate("xvCF"):
        c, r = cos(got[k], ref[k]), rel(got[k], ref[k])
        log(f"  d{name}: cos={c:.8f} rel={r:.3g}")
        assert c > 0.99999 and r < 1e-4, (name, c, r)
    rE_rel = abs(gE.item() - rE[0]) / abs(rE[0])
    log(f"  dE: gpu={gE.item():.6g} oracle={rE[0]:.6g} rel={rE_rel:.3g}")
    assert rE_rel < 1e-4


def test_step_bwd_accumulates():
    """Adjoint outputs accumulate: two calls give twice one call."""
    sc = _case(2, 1024)
    S = 12
    gout = np.random.default_rng(4).normal(size=(sc.n_particles, S))
    sim = rt.Simulator.for_scene(sc)
    p = rt.params_for_scene(sc)
    s_in = rt.state_for_scene(sc)
    og = rt.State.from_particle_major(*orc.unpack(gout, 2))
    one = rt.State.zeros(2, sc.n_particles)
    two = rt.State.zeros(2, sc.n_particles)
    sim.step_bwd(p, 0, s_in, og, one)
    sim.step_bwd(p, 0, s_in, og, two)
    sim.step_bwd(p, 0, s_in, og, two)
    a = one.to_particle_major()
    b = two.to_particle_major()
    for k in range(4):
        np.testing.assert_allclose(b[k], 2 * a[k], rtol=1e-4, atol=1e-6 * np.abs(a[k]).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_fixed_point_scale_with_one_large_contribution(dim):
    """A workgroup whose scatter contributions span four orders of magnitude:
    one particle 1e4 times faster than its neighbours (forward: |m v|; reverse:
    its seed dL/dv'), so the workgroup's fixed-point scale follows the large
    bound B. The other particles' contributions are then rounded to B 2^-31;
    their results must stay within the bound that implies (a node sum of n
    contributions is off by at most n B 2^-31) and match the oracle."""
    base = scenes.deform2d() if dim == 2 else scenes.elastic3d()
    n_keep = 1024 if dim == 2 else 4096
    from dataclasses import replace
    rng = np.random.default_rng(20 + dim)
    # The first lattice points: single steps run in the caller's order, and
    # 128 consecutive lattice points (four lattice rows) stage a box that
    # fits the LDS tile.
    sc = replace(base, offsets=np.array([0, n_keep], np.int32), x=base.x[:n_keep], v=base.v[:n_keep],
                 C=base.C[:n_keep], F=base.F[:n_keep])
    small = 1e-2
    v = (small * rng.normal(size=(n_keep, dim))).astype(np.float32)
    sim = rt.Simulator.for_scene(sc, knobs={"block": 128, "lanes": 1, "part": 0, "tile_stats": 1})
    big = 64  # in the first workgroup, particles 0..127
    wg0 = np.arange(128)
    v[big] = 100.0 * np.sign(rng.normal(size=dim))
    sc = replace(sc, v=v)
    p = rt.params_for_scene(sc)
    s_in = rt.state_for_scene(sc)
    s_out = rt.State.empty(dim, n_keep)
    sim.tile_stats()
    sim.step_fwd(p, 0, s_in, s_out)
    assert sim.check_errors() == 0
    lds, fallback = sim.tile_stats()
    assert lds > 0 and fallback == 0, (lds, fallback)  # the fixed-point LDS path ran
    got = s_out.to_particle_major()
    ref, err = orc.step_fwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F))
    assert err == 0
    ref = orc.unpack(ref, dim)
    # Particles of the first workgroup more than two cells from the fast one:
    # their nodes receive none of its contributions, only the coarse rounding.
    far = wg0[np.linalg.norm(sc.x[wg0] - sc.x[big], axis=1) > 3 * sc.dx]
    assert len(far) > 32
    m = float(sc.rho[0] * sc.vol[0])
    B = m * 100.0 * np.sqrt(dim)  # bound of the fast particle's |m v| contributions
    per_node = 4.0 ** dim * B * 2.0 ** -30 / (0.5 * m)  # n contributions over a node mass >= m/2 (generous)
    dv = np.abs(got[1][far] - ref[1][far]).max()
    log(f"[fixed-point scale {dim}D] forward: max |dv'| of {len(far)} far particles {dv:.3g} "
        f"(bound {per_node:.3g}; their |v| ~ {small})")
    assert dv <= per_node, (dv, per_node)
    assert rel(got[1][far], ref[1][far]) < 1e-2
    # Reverse: the fast particle's seed dL/dv' is 1e4 times the others'.
    S = 2 * dim + 2 * dim * dim
    gout = small * rng.normal(size=(n_keep, S))
    gout[big, dim:2 * dim] = 100.0
    gx, gv, gC, gF = orc.unpack(gout, dim)
    og = rt.State.from_particle_major(gx, gv, gC, gF)
    ig = rt.State.zeros(dim, n_keep)
    sim.step_bwd(p, 0, s_in, og, ig)
    assert sim.check_errors() == 0
    gout32 = orc.pack(*[a.astype(np.float32) for a in (gx, gv, gC, gF)])
    rg, _, _, err = orc.step_bwd(sc, orc.pack(sc.x, sc.v, sc.C, sc.F), gout32)
    assert err == 0
    rg = orc.unpack(rg, dim)
    gg = ig.to_particle_major()
    r = {name: rel(gg[k][far], rg[k][far]) for k, name in enumerate("xvCF")}
    log(f"[fixed-point scale {dim}D] reverse: far particles' gradients rel {r}")
    for name, e in r.items():
        assert e < 1e-3, (name, e)

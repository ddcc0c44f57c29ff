"""Pins of the FP64 smoke oracle (no GPU) against facts the mathematics fixes,
independently of the oracle's own code:
  - advection equals SciPy's periodic linear interpolation (map_coordinates,
    order 1, grid-wrap) at the back-traced points; leaves a constant field
    unchanged; is an exact periodic shift (np.roll) for an integer uniform
    velocity; reproduces a bilinear function exactly away from the wrap;
  - the K-iteration projection equals its closed form in Fourier space
    (central differences are i sin(theta), the neighbour-sum average of a
    Jacobi sweep is (cos th0 + cos th1) / 2, K sweeps from zero sum its
    geometric series), for K = 0, 1, 6 and 10, on even and odd grids;
  - Jacobi converges to the FFT solution of the 5-point Poisson equation and
    its residual never grows;
  - one step equals its definition composed from the library primitives above;
  - every adjoint (advection in both arguments, projection, one step, a whole
    trajectory, the loss seed) passes a complex-step dot-product test, and
    the trajectory gradient matches central finite differences.
"""
import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle.smoke as sm
from paper_1910_00935_amd import scenes


def _rng(seed):
    return np.random.default_rng(seed)


def _field(rng, n, scale=1.0):
    return scale * rng.normal(size=(n, n))


def _lib_advect(f, u0, u1):
    """Bilinear periodic sampling at c - u(c) with SciPy's interpolator."""
    n = f.shape[0]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return map_coordinates(f, [i - u0, j - u1], order=1, mode="grid-wrap")


def _fourier_project(u0, u1, iters):
    """The K-sweep projection in Fourier space."""
    n = u0.shape[0]
    th = 2 * np.pi * np.fft.fftfreq(n)
    t0, t1 = np.meshgrid(th, th, indexing="ij")
    U0, U1 = np.fft.fft2(u0), np.fft.fft2(u1)
    D = 1j * (np.sin(t0) * U0 + np.sin(t1) * U1)
    sigma = (np.cos(t0) + np.cos(t1)) / 2
    series = sum(sigma ** k for k in range(iters)) if iters else np.zeros_like(sigma)
    P = -D / 4 * series
    V0 = U0 - 1j * np.sin(t0) * P
    V1 = U1 - 1j * np.sin(t1) * P
    return np.real(np.fft.ifft2(V0)), np.real(np.fft.ifft2(V1))


# ---------------------------------------------------------------------------
# Advection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,scale", [(12, 0.7), (17, 3.5), (32, 11.0)])
def test_advect_matches_library_interpolation(n, scale):
    rng = _rng(n)
    f, u0, u1 = _field(rng, n), _field(rng, n, scale), _field(rng, n, scale)
    np.testing.assert_allclose(sm.advect(f, u0, u1), _lib_advect(f, u0, u1), rtol=0, atol=1e-12)


def test_advect_constant_field_and_zero_velocity():
    rng = _rng(1)
    n = 16
    u0, u1 = _field(rng, n, 2.0), _field(rng, n, 2.0)
    np.testing.assert_allclose(sm.advect(np.full((n, n), 0.37), u0, u1), 0.37, rtol=0, atol=1e-15)
    f = _field(rng, n)
    z = np.zeros((n, n))
    np.testing.assert_array_equal(sm.advect(f, z, z), f)


def test_advect_integer_velocity_is_a_periodic_shift():
    rng = _rng(2)
    n = 13
    f = _field(rng, n)
    u0, u1 = np.full((n, n), 3.0), np.full((n, n), -5.0)
    # sample at (i - 3, j + 5): np.roll by +3 on axis 0 and -5 on axis 1
    np.testing.assert_array_equal(sm.advect(f, u0, u1), np.roll(f, (3, -5), axis=(0, 1)))


def test_advect_reproduces_bilinear_function():
    n = 20
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = 0.5 + 0.3 * i - 0.2 * j + 0.01 * i * j
    rng = _rng(3)
    u0, u1 = rng.uniform(-1.9, 1.9, (n, n)), rng.uniform(-1.9, 1.9, (n, n))
    got = sm.advect(f, u0, u1)
    y0, y1 = i - u0, j - u1
    want = 0.5 + 0.3 * y0 - 0.2 * y1 + 0.01 * y0 * y1
    inner = (i >= 2) & (i < n - 3) & (j >= 2) & (j < n - 3)  # samples never wrap
    np.testing.assert_allclose(got[inner], want[inner], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [12, 15])
@pytest.mark.parametrize("iters", [0, 1, 6, 10])
def test_projection_matches_fourier_closed_form(n, iters):
    rng = _rng(10 * n + iters)
    u0, u1 = _field(rng, n), _field(rng, n)
    got = sm.project(u0, u1, iters)
    want = _fourier_project(u0, u1, iters)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [15, 16])
def test_jacobi_converges_to_poisson_solution(n):
    rng = _rng(n)
    d = sm.divergence(_field(rng, n), _field(rng, n))  # zero mean, no checkerboard mode
    th = 2 * np.pi * np.fft.fftfreq(n)
    t0, t1 = np.meshgrid(th, th, indexing="ij")
    lam = 2 * np.cos(t0) + 2 * np.cos(t1) - 4
    Dh = np.fft.fft2(d)
    Ph = np.where(np.abs(lam) > 1e-12, Dh / np.where(np.abs(lam) > 1e-12, lam, 1.0), 0.0)
    p_exact = np.real(np.fft.ifft2(Ph))

    def lap(p):
        return sm.neighbour_sum(p) - 4 * p

    res, err = [], []
    for K in (0, 1, 2, 4, 8, 16, 64, 256, 1024, 4096):
        p = sm.jacobi(d, K)
        res.append(np.linalg.norm(lap(p) - d))
        err.append(np.linalg.norm(p - p_exact))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:])), res
    assert err[-1] < 1e-9 * np.linalg.norm(p_exact), err


def test_step_composed_from_library_primitives():
    rng = _rng(4)
    n, K = 14, 6
    u0, u1, s = _field(rng, n, 0.8), _field(rng, n, 0.8), rng.uniform(0, 1, (n, n))
    w0, w1 = _lib_advect(u0, u0, u1), _lib_advect(u1, u0, u1)
    v0, v1 = _fourier_project(w0, w1, K)
    want = (v0, v1, _lib_advect(s, v0, v1))
    got = sm.step(u0, u1, s, K)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=0, atol=1e-11)


# ---------------------------------------------------------------------------
# Adjoints
# ---------------------------------------------------------------------------
H = 1e-30


def _dot_rel(jv, v_jtw):
    return abs(jv - v_jtw) / max(abs(jv), abs(v_jtw))


def test_advect_adjoint_dot_products():
    rng = _rng(5)
    n = 11
    f, u0, u1, w = _field(rng, n), _field(rng, n, 1.3), _field(rng, n, 1.3), _field(rng, n)
    df, du0, du1 = _field(rng, n), _field(rng, n), _field(rng, n)
    gf, g0, g1 = sm.advect_adj(f, u0, u1, w)
    jv = np.sum(np.imag(sm.advect(f + 1j * H * df, u0 + 1j * H * du0, u1 + 1j * H * du1)) / H * w)
    assert _dot_rel(jv, np.sum(gf * df + g0 * du0 + g1 * du1)) < 1e-11


@pytest.mark.parametrize("iters", [0, 6, 10])
def test_project_adjoint_dot_products(iters):
    rng = _rng(6 + iters)
    n = 10
    u0, u1, w0, w1 = (_field(rng, n) for _ in range(4))
    a0, a1 = sm.project_adj(w0, w1, iters)
    v0, v1 = sm.project(u0, u1, iters)
    assert _dot_rel(np.sum(v0 * w0 + v1 * w1), np.sum(u0 * a0 + u1 * a1)) < 1e-12


def _traj(u0, u1, s, T, K):
    return sm.forward(u0, u1, s, T, K)[-1]


@pytest.mark.parametrize("T,K", [(1, 6), (5, 6), (4, 10)])
def test_trajectory_adjoint_dot_products(T, K):
    rng = _rng(7 + T)
    n = 12
    u0, u1, s = _field(rng, n, 0.9), _field(rng, n, 0.9), rng.uniform(0, 1, (n, n))
    d = [_field(rng, n) for _ in range(3)]
    w = [_field(rng, n) for _ in range(3)]
    out = _traj(u0 + 1j * H * d[0], u1 + 1j * H * d[1], s + 1j * H * d[2], T, K)
    jv = sum(np.sum(np.imag(o) / H * ww) for o, ww in zip(out, w))
    g = sm.backward(sm.forward(u0, u1, s, T, K), *w, K)
    vjtw = sum(np.sum(gg * dd) for gg, dd in zip(g, d))
    assert _dot_rel(jv, vjtw) < 1e-11


def test_trajectory_gradient_finite_differences():
    sc = scenes.smoke(n=16, steps=6, iters=6, seed=3)
    u0, u1, s = (a.astype(np.float64) for a in (sc.u0, sc.u1, sc.s))
    tgt = sc.target.astype(np.float64)

    def L(a, b, c):
        return sm.loss(_traj(a, b, c, sc.steps, sc.iters)[2], tgt)

    st = sm.forward(u0, u1, s, sc.steps, sc.iters)
    g = sm.backward(st, np.zeros_like(u0), np.zeros_like(u0), sm.loss_seed(st[-1][2], tgt), sc.iters)
    rng = _rng(8)
    h = 1e-6
    for _ in range(3):
        d = [_field(rng, 16) for _ in range(3)]
        fd = (L(*(x + h * dx for x, dx in zip((u0, u1, s), d))) - L(*(x - h * dx for x, dx in zip((u0, u1, s), d)))) / (2 * h)
        an = sum(np.sum(gg * dd) for gg, dd in zip(g, d))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_loss_seed_is_the_loss_gradient():
    rng = _rng(9)
    sT, tgt, d = (_field(rng, 9) for _ in range(3))
    jv = np.imag(sm.loss(sT + 1j * H * d, tgt)) / H
    assert _dot_rel(jv, np.sum(sm.loss_seed(sT, tgt) * d)) < 1e-13


# ---------------------------------------------------------------------------
# Planted mistakes: each consistent change to the oracle (forward and adjoint
# together) fails at least one pin above.
# ---------------------------------------------------------------------------
def _mutations():
    def div_sign(u0, u1):
        return -(sm._shift(u0, 0, 1) - sm._shift(u0, 0, -1) + sm._shift(u1, 1, 1) - sm._shift(u1, 1, -1)) / 2

    def div_sign_adj(g):
        a, b = ORIG["divergence_adj"](g)
        return -a, -b

    def jacobi5(d, iters):
        p = np.zeros_like(d)
        for _ in range(iters):
            p = (sm.neighbour_sum(p) - d) / 5
        return p

    def jacobi5_adj(g, iters):
        gd, gp = np.zeros_like(g), g
        for _ in range(iters):
            gd = gd - gp / 5
            gp = sm.neighbour_sum(gp) / 5
        return gd

    def forward_trace(u0, u1):
        return ORIG["_sample_points"](-u0, -u1)

    def project_plus(u0, u1, iters):
        g0, g1 = sm.gradient(sm.jacobi(sm.divergence(u0, u1), iters))
        return u0 + g0, u1 + g1

    def project_plus_adj(g0, g1, iters):
        gd = sm.jacobi_adj(sm.gradient_adj(g0, g1), iters)
        d0, d1 = sm.divergence_adj(gd)
        return g0 + d0, g1 + d1

    def step_unprojected(u0, u1, s, iters):
        w0, w1 = sm.advect(u0, u0, u1), sm.advect(u1, u0, u1)
        v0, v1 = sm.project(w0, w1, iters)
        return v0, v1, sm.advect(s, w0, w1)

    def adj_no_scatter(f, u0, u1, g):
        gf, a, b = ORIG["advect_adj"](f, u0, u1, g)
        return np.zeros_like(gf), a, b

    def neighbour_transposed(p):  # e0 and e1 mixed up in one term
        return sm._shift(p, 0, 1) + sm._shift(p, 0, -1) + sm._shift(p, 1, 1) + sm._shift(p, 0, 1)

    return {
        "divergence sign": {"divergence": div_sign, "divergence_adj": div_sign_adj},
        "jacobi divides by 5": {"jacobi": jacobi5, "jacobi_adj": jacobi5_adj},
        "back-trace along +u": {"_sample_points": forward_trace},
        "projection adds the gradient": {"project": project_plus, "project_adj": project_plus_adj},
        "smoke advected by the unprojected velocity": {"step": step_unprojected},
        "advection adjoint drops the scatter": {"advect_adj": adj_no_scatter},
        "neighbour sum uses a wrong neighbour": {"neighbour_sum": neighbour_transposed},
    }


ORIG = {k: getattr(sm, k) for k in ("divergence", "divergence_adj", "_sample_points", "advect_adj", "jacobi",
                                    "jacobi_adj", "project", "project_adj", "step", "neighbour_sum")}

PINS = [
    lambda: test_advect_matches_library_interpolation(17, 3.5),
    lambda: test_advect_integer_velocity_is_a_periodic_shift(),
    lambda: test_projection_matches_fourier_closed_form(15, 6),
    lambda: test_jacobi_converges_to_poisson_solution(15),
    lambda: test_step_composed_from_library_primitives(),
    lambda: test_advect_adjoint_dot_products(),
    lambda: test_trajectory_adjoint_dot_products(5, 6),
]


@pytest.mark.parametrize("name", sorted(_mutations()))
def test_planted_mistake_fails_a_pin(name, monkeypatch):
    for attr, fn in _mutations()[name].items():
        monkeypatch.setattr(sm, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1, f"no pin caught: {name}"

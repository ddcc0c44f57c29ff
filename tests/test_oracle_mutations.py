"""The oracle's pins detect plausible mistakes (no GPU).

Each case below plants one mistake in a copy of the oracle source -- applied
consistently to the forward and to its hand-written adjoint where it touches
both, so that the adjoint-versus-forward checks (dot products, finite
differences) cannot see it -- builds the copy with g++, points the oracle
module at it, and asserts that the named pin of ``test_oracle.py`` fails. The
text each case replaces must occur in the source the stated number of times,
so a case cannot silently stop applying when the oracle is edited.
"""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle as orc
import test_oracle as pins

SRC = os.path.join(os.path.dirname(orc.__file__), "mpm_oracle.cpp")

# name -> (list of (old, new, occurrences), [(pin, kwargs), ...] each of which must fail)
MUTATIONS = {
    # The gather of the grid-to-particle stage (C' = kappa sum w v delta^T, F' = (I + dt C') F).
    "g2p_kappa_halved": (
        [("Cn[a][b] += kappa * w * g[1 + a] * dl[b];", "Cn[a][b] += 0.5 * kappa * w * g[1 + a] * dl[b];", 2),
         ("Bd += kappa * Ct[a][b] * dl[b];", "Bd += 0.5 * kappa * Ct[a][b] * dl[b];", 1),
         ("Btv += kappa * Ct[a][c] * g[1 + a];", "Btv += 0.5 * kappa * Ct[a][c] * g[1 + a];", 1)],
        [("test_affine_field_closed_form", {"dim": 2}), ("test_affine_field_closed_form", {"dim": 3})]),
    "g2p_C_transposed": (
        [("Cn[a][b] += kappa * w * g[1 + a] * dl[b];", "Cn[a][b] += kappa * w * g[1 + b] * dl[a];", 2),
         ("Bd += kappa * Ct[a][b] * dl[b];", "Bd += kappa * Ct[b][a] * dl[b];", 1),
         ("Btv += kappa * Ct[a][c] * g[1 + a];", "Btv += kappa * Ct[c][a] * g[1 + a];", 1)],
        [("test_affine_field_closed_form", {"dim": 2}), ("test_affine_field_closed_form", {"dim": 3})]),
    "g2p_F_right_multiplied": (
        [("Fn += ((a == c ? 1.0 : 0.0) + s.dt * Cn[a][c]) * P.F(c, b);",
          "Fn += P.F(a, c) * ((c == b ? 1.0 : 0.0) + s.dt * Cn[c][b]);", 1),
         ("acc += ((c == a ? 1.0 : 0.0) + s.dt * Cn[c][a]) * G.F(c, b);",
          "acc += G.F(a, c) * ((b == c ? 1.0 : 0.0) + s.dt * Cn[b][c]);", 1),
         ("FbFt += G.F(a, c) * P.F(b, c);", "FbFt += P.F(c, a) * G.F(c, b);", 1)],
        [("test_affine_field_closed_form", {"dim": 2}), ("test_affine_field_adjoint_closed_form", {"dim": 3})]),
    "g2p_x_with_old_velocity": (
        [("Q.x(a) = P.x(a) + s.dt * vn[a];", "Q.x(a) = P.x(a) + s.dt * P.v(a);", 1)],
        [("test_affine_field_closed_form", {"dim": 2}), ("test_translate2d_closed_form", {})]),
    # Weights, grid update and boundary.
    "weight_middle_piece": (
        [("st.N[a][1] = 0.75 - (f - 1.0) * (f - 1.0);", "st.N[a][1] = 0.76 - (f - 1.0) * (f - 1.0);", 1)],
        [("test_bspline_golden_values", {"dim": 2}), ("test_bspline_textbook_distance_form", {})]),
    "gravity_on_axis_0": (
        [("if (a == 1) g[1 + a] += s.dt * s.gravity;", "if (a == 0) g[1 + a] += s.dt * s.gravity;", 1)],
        [("test_mass_and_momentum", {"dim": 2}), ("test_translate2d_closed_form", {})]),
    "sticky_band_off_by_one": (
        [("if (i[a] < s.bound || i[a] >= s.n_grid - s.bound) return false;",
          "if (i[a] < s.bound || i[a] > s.n_grid - s.bound) return false;", 1)],
        [("test_sticky_band_width", {}), ("test_mirror_symmetry_with_wall_contact", {"dim": 2})]),
    # Stress.
    "stress_sign": (
        [("t.A[a][b] = t.mass * P.C(a, b) - s.dt * vol * kappa * t.tau[a][b];",
          "t.A[a][b] = t.mass * P.C(a, b) + s.dt * vol * kappa * t.tau[a][b];", 1)],
        [("test_p2g_moments_recover_stress_closed_form", {"dim": 3})]),
    "stress_lambda_dropped": (
        [("t.tau[a][b] = mat.mu * (FFt - (a == b ? 1.0 : 0.0)) + (a == b ? mat.lam * t.lnJ : T(0.0));",
          "t.tau[a][b] = mat.mu * (FFt - (a == b ? 1.0 : 0.0));", 1),
         ("H.F(a, b) += mat.mu * sym + mat.lam * tr * Finv_t;", "H.F(a, b) += mat.mu * sym;", 1),
         ("(a == b ? mat.dlam_dE * t.lnJ : 0.0)", "0.0", 1)],
        [("test_p2g_moments_recover_stress_closed_form", {"dim": 2})]),
    "actuation_on_xx": (
        [("t.tau[1][1] += s.act_strength * act_s[s.act_id[p]];", "t.tau[0][0] += s.act_strength * act_s[s.act_id[p]];",
          1),
         ("gact[s.act_id[p]] += s.act_strength * taubar[1][1];", "gact[s.act_id[p]] += s.act_strength * taubar[0][0];",
          1)],
        [("test_actuation_stress_closed_form", {"dim": 2}), ("test_actuation_stress_closed_form", {"dim": 3})]),
    # Adjoint-only mistakes (the forward is untouched).
    "p2g_adjoint_drops_affine_x_term": (
        [("H.x(c) += contrib * dw[c] - w * AtP;", "H.x(c) += contrib * dw[c];", 1)],
        [("test_dot_product_complex_step", {"dim": 2, "T": 1, "model": 0, "liquid": False})]),
    "grid_adjoint_mass_sign": (
        [("mbar[qq] = -vP / (m * m);", "mbar[qq] = vP / (m * m);", 1)],
        [("test_dot_product_complex_step", {"dim": 3, "T": 1, "model": 0, "liquid": False})]),
    "neo_hookean_adjoint_not_symmetrised": (
        [("sym += (taubar[a][c] + taubar[c][a]) * t.F[c][b];", "sym += 2.0 * taubar[a][c] * t.F[c][b];", 1)],
        [("test_dot_product_complex_step", {"dim": 2, "T": 1, "model": 0, "liquid": False})]),
    "E_adjoint_drops_lambda": (
        [("(a == b ? mat.dlam_dE * t.lnJ : 0.0)", "0.0", 1)],
        [("test_dot_product_complex_step", {"dim": 3, "T": 1, "model": 0, "liquid": False})]),
    "corotated_rotation_share_sign": (
        [("H.F(a, b) += Fbar[a][b] + v;", "H.F(a, b) += Fbar[a][b] - v;", 1)],
        [("test_dot_product_complex_step", {"dim": 3, "T": 1, "model": 1, "liquid": False})]),
    "liquid_adjoint_sign": (
        [("H.F(a, b) += dval * tr * cof[a][b];", "H.F(a, b) -= dval * tr * cof[a][b];", 1)],
        [("test_dot_product_complex_step", {"dim": 2, "T": 1, "model": 0, "liquid": True})]),
    "g2p_adjoint_F_not_transposed": (
        [("acc += ((c == a ? 1.0 : 0.0) + s.dt * Cn[c][a]) * G.F(c, b);",
          "acc += ((c == a ? 1.0 : 0.0) + s.dt * Cn[a][c]) * G.F(c, b);", 1)],
        [("test_dot_product_complex_step", {"dim": 3, "T": 1, "model": 0, "liquid": False})]),
}


def _mutate(src, edits):
    for old, new, count in edits:
        found = src.count(old)
        assert found == count, f"expected {count} occurrence(s) of {old!r}, found {found}"
        src = src.replace(old, new)
    return src


@pytest.fixture(scope="module")
def mutant_libs():
    """Every mutant, built once (in parallel) into a temporary directory."""
    src = open(SRC).read()
    tmp = tempfile.TemporaryDirectory(prefix="oracle_mut_")

    def build(name):
        cpp = os.path.join(tmp.name, name + ".cpp")
        so = os.path.join(tmp.name, name + ".so")
        with open(cpp, "w") as fh:
            fh.write(_mutate(src, MUTATIONS[name][0]))
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-shared",
                               "-fPIC", "-o", so, cpp])
        return name, so

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        libs = dict(ex.map(build, sorted(MUTATIONS)))
    yield libs
    orc.use_library(None)
    tmp.cleanup()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pin_detects_planted_mistake(name, mutant_libs):
    _, killers = MUTATIONS[name]
    orc.use_library(mutant_libs[name])
    try:
        for pin, kwargs in killers:
            with pytest.raises(AssertionError):
                getattr(pins, pin)(**kwargs)
    finally:
        orc.use_library(None)


def test_unmutated_oracle_passes_the_killer_pins():
    """The same pins pass on the oracle as built (so the failures above come
    from the planted mistakes)."""
    orc.use_library(None)
    seen = set()
    for _, killers in MUTATIONS.values():
        for pin, kwargs in killers:
            key = (pin, tuple(sorted(kwargs.items())))
            if key in seen:
                continue
            seen.add(key)
            getattr(pins, pin)(**kwargs)

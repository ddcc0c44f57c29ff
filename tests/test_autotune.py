"""Autotuner host logic (no GPU): candidate grid and cache keys."""
from paper_1910_00935_amd import autotune, scenes


def test_candidates_cover_the_space():
    space = {"block": (128, 64), "lanes": (1, 4), "rotate": (1,)}
    c = autotune.candidates(space)
    assert len(c) == 4 and c[0] == {"block": 128, "lanes": 1, "rotate": 1}
    assert {"block": 64, "lanes": 4, "rotate": 1} in c


def test_shape_key_depends_on_shape_only():
    a = scenes.translate2d()
    b = scenes.translate2d(seed=7)          # same shape, other values
    c = scenes.deform2d().with_steps(32)  # other horizon
    assert autotune.shape_key(a, "gfx950") == autotune.shape_key(b, "gfx950")
    assert autotune.shape_key(a, "gfx950") != autotune.shape_key(c, "gfx950")
    assert autotune.shape_key(a, "gfx950") != autotune.shape_key(a, "gfx942")

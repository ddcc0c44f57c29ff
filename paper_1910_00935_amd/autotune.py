"""Launch-configuration autotuner for the step kernels.

Times whole trajectories (tape forward + loss + tape backward) of a workload
for each candidate knob set (`block`, `lanes`, `part`, `rotate`, `lds`, `split`) and
keeps the fastest. Results are cached in a JSON file keyed by the workload's
shape (dimension, grid, particle and scene counts, steps) and the GPU
architecture, so later runs of the same shape reuse them.

Usage:
    knobs = autotune.tune(scene)                # cached
    sim = runtime.Simulator.for_scene(scene, knobs=knobs)
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from typing import Dict, Iterable, List, Optional

import torch

from . import runtime as rt

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mpm_autotune.json")

# Candidate grid; the first entry is the library default.
SPACE = {
    "block": (128, 64, 192, 256),
    "lanes": (1, 2, 4),
    "part": (1, 0),
    "rotate": (1,),
    "lds": (1,),
    "split": (1,),
}


def shape_key(scene, arch: Optional[str] = None) -> str:
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    desc = dict(dim=scene.dim, n_grid=scene.n_grid, N=scene.n_particles, scenes=scene.n_scenes,
                steps=scene.steps, ckpt=scene.ckpt_every, act=scene.n_act, arch=arch,
                knobs=sorted(SPACE))
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:20]


def candidates(space: Dict[str, Iterable] = SPACE) -> List[dict]:
    keys = list(space)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(space[k] for k in keys))]


def time_trajectory(scene, knobs: dict, steps: Optional[int] = None, repeats: int = 2) -> float:
    """Mean seconds of one trajectory (fwd + loss + bwd) with these knobs."""
    T = steps or scene.steps
    sim = rt.Simulator.for_scene(scene, knobs=knobs)
    p = rt.params_for_scene(scene)
    init = rt.state_for_scene(scene)
    tape = sim.tape(T, scene.ckpt_every if scene.ckpt_every and scene.ckpt_every < T else 0)
    fin = rt.State.empty(scene.dim, scene.n_particles)
    seed = rt.State.empty(scene.dim, scene.n_particles)
    grad = rt.State.zeros(scene.dim, scene.n_particles)

    def run():
        tape.forward(p, init, fin)
        sim.loss_mean(fin, scene.loss_axis, scene.loss_sign, seed)
        tape.backward(p, seed, grad)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeats):
        run()
    torch.cuda.synchronize()
    if sim.check_errors():
        return float("inf")
    return (time.perf_counter() - t0) / repeats


def tune(scene, cache: str = DEFAULT_CACHE, steps: Optional[int] = None, space: Dict[str, Iterable] = SPACE,
         force: bool = False, verbose: bool = False) -> dict:
    """Best knob set for this workload shape (from the cache when present)."""
    key = shape_key(scene)
    db = {}
    if os.path.exists(cache):
        try:
            with open(cache) as fh:
                db = json.load(fh)
        except (OSError, ValueError):
            db = {}
    if key in db and not force:
        return dict(db[key]["knobs"])
    results = []
    for kn in candidates(space):
        t = time_trajectory(scene, kn, steps=steps)
        results.append((t, kn))
        if verbose:
            print(f"[autotune] {kn}: {t * 1e3:.3f} ms", flush=True)
    best_t, best = min(results, key=lambda r: r[0])
    db[key] = {"knobs": best, "seconds": best_t, "steps": steps or scene.steps,
               "all": [{"knobs": k, "seconds": t} for t, k in results]}
    os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
    tmp = cache + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1)
    os.replace(tmp, cache)
    return dict(best)

"""Autotuner for the launch tuning of a loaded Simulation or Batch.

The tuning (cell_scale, tile_scale, tiled, graph, sized, wave_class; see dss_set_tuning in
include/dss.h) changes how the step is launched, never what it computes.  The tuner times a
short run of ordinary time steps under each candidate -- the steps advance the simulation like
any others, so the tuning costs no extra work beyond the time spent in slower candidates --
keeps the fastest, and caches the choice in a JSON file keyed by the workload class: number of
boxes, particles per box (power-of-two bucket), volume fraction (0.05 bucket), size ratio and
precision.  One box of size ratio above 2 also tries the size-class stencils.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import time

CANDIDATES = (
    {"cell_scale": 1.0, "tile_scale": 1.0, "tiled": True, "sized": False},
    {"cell_scale": 1.0, "tile_scale": 0.75, "tiled": True, "sized": False},
    {"cell_scale": 1.0, "tile_scale": 1.5, "tiled": True, "sized": False},
    {"cell_scale": 1.15, "tile_scale": 1.0, "tiled": True, "sized": False},
    {"cell_scale": 1.3, "tile_scale": 1.0, "tiled": True, "sized": False},
    {"cell_scale": 1.0, "tile_scale": 1.0, "tiled": False, "sized": False},
)

# Size-class stencils (one box of high size ratio): cell spacing in units of the smallest pair
# cutoff; wave_class 0 = the default split between lane and wavefront stencils.
SIZED_CANDIDATES = (
    {"cell_scale": 1.0, "sized": True, "wave_class": 0},
    {"cell_scale": 1.5, "sized": True, "wave_class": 0},
    {"cell_scale": 2.0, "sized": True, "wave_class": 0},
    {"cell_scale": 3.0, "sized": True, "wave_class": 0},
    {"cell_scale": 2.0, "sized": True, "wave_class": 2},
    {"cell_scale": 2.0, "sized": True, "wave_class": 1},
    {"cell_scale": 1.5, "sized": True, "wave_class": 2},
    {"cell_scale": 2.5, "sized": True, "wave_class": 2},
    {"cell_scale": 1.5, "sized": True, "wave_class": 1},
    {"cell_scale": 1.25, "sized": True, "wave_class": 2},
)


def candidates_for(sim):
    """The row-tile candidates; for one box of size ratio above 2 also the size-class stencils."""
    if getattr(sim, "B", 1) == 1 and sim.size_ratio > 2.0:
        return CANDIDATES + SIZED_CANDIDATES
    return CANDIDATES


def default_cache_path() -> str:
    return os.environ.get("DSS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dss_tuning.json"))


def workload_key(sim) -> str:
    """Class of the loaded workload: boxes, particles per box, volume fraction, size ratio, precision."""
    n_box = getattr(sim, "B", 1)
    per_box = sim.N / n_box
    phi = sim.phi_mean
    return (f"B{n_box}:N2^{round(math.log2(max(per_box, 1)))}:phi{round(phi / 0.05) * 0.05:.2f}:"
            f"ratio{sim.size_ratio:.2f}:prec{sim.precision}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(sim, trial_steps: int = 20, cache_path: str | None = None, candidates=None,
             force: bool = False, log=None) -> dict:
    """Choose and apply the fastest tuning for `sim` (loaded).  Returns the cache record
    {"tuning": {...}, "ms_per_step": t, "trials": [...], "cached": bool}."""
    from .dss import DssError

    path = cache_path or default_cache_path()
    key = workload_key(sim)
    cache = _load(path)
    if key in cache and not force:
        rec = dict(cache[key])
        sim.set_tuning(**rec["tuning"], graph=True)
        rec["cached"] = True
        return rec
    trials = []
    for cand in (candidates_for(sim) if candidates is None else candidates):
        try:
            sim.set_tuning(**cand, graph=True)
        except DssError:
            continue   # lattice not legal for this workload
        sim.step(2, sync=True)           # the lattice is rebuilt here
        prepare = getattr(sim, "prepare_steps", None)
        if prepare:
            prepare(trial_steps)         # and the graphs of the timed steps captured
        t0 = time.perf_counter()
        sim.step(trial_steps, sync=True)
        ms = (time.perf_counter() - t0) / trial_steps * 1e3
        trials.append({"tuning": dict(cand), "ms_per_step": ms})
        if log:
            log(f"tune {key}: {cand} -> {ms:.4f} ms/step")
    best = min(trials, key=lambda r: r["ms_per_step"])
    sim.set_tuning(**best["tuning"], graph=True)
    rec = {"tuning": best["tuning"], "ms_per_step": best["ms_per_step"], "trials": trials}
    cache[key] = rec
    _store(path, cache)
    return dict(rec, cached=False)

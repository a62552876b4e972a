"""Tile-shape autotuner for batches of uneven walkers.

The tile of the pair kernel is a cluster of 8 atoms cut from a z-sorted
x-y column; its shape is set by the column width (in units of
(8/rho)^(1/3): 1 gives cubic clusters).  Wider columns mean fewer columns
and less padding but flatter clusters whose boxes admit more j atoms;
narrower ones the reverse.  For every size class present in a batch the
tuner times the step of its representative walker (the member of median
size, replicated to fill the GPU) for each candidate width and keeps the
fastest.  The cost timed is what the width changes: the environment pair
kernel per step plus the neighbour rebuild per step (HIP events around
single launches, labf_profile_steps).

Results are cached in JSON keyed by GPU architecture, size class and
precision; the file named by $LABF_AUTOTUNE_CACHE, else autotune_cache.json
beside this module.
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

from . import labf, synth

# size classes by atoms per walker (lower bound inclusive)
CLASSES = [(0, 10000), (10000, 20000), (20000, 40000), (40000, 1 << 62)]
CANDIDATES = (0.8, 0.9, 1.0, 1.12, 1.25)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def size_class(n_atoms: int) -> tuple:
    for lo, hi in CLASSES:
        if lo <= n_atoms < hi:
            return lo, hi
    return CLASSES[-1]


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(a: str, cls: tuple, precision: str) -> str:
    return f"{a}|{cls[0]}-{cls[1]}|{precision}"


def load_cache(path: str | None = None) -> dict:
    path = path or os.environ.get("LABF_AUTOTUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None) -> None:
    path = path or os.environ.get("LABF_AUTOTUNE_CACHE", DEFAULT_CACHE)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def time_width(spec, lam, width: float, steps: int = 10, warmup: int = 10) -> dict:
    """Per-step cost (ms) of a batch at one column width."""
    sp = dataclasses.replace(spec, column_width=np.full(spec.n_walkers, float(width)))
    with labf.System(sp, lam) as s:
        s.step(warmup)
        prof = s.profile_steps(steps)
    per_step = prof["env_ms"] + prof["rebuild_ms"] / spec.rebuild_interval
    return dict(prof, per_step_ms=per_step)


def cached_widths(spec, cache_path: str | None = None) -> np.ndarray:
    """Column widths from the cache only (1 where a class is not cached)."""
    cache = load_cache(cache_path)
    a = arch()
    return np.array([cache.get(_key(a, size_class(int(x)), spec.precision), {}).get("column_width", 1.0)
                     for x in np.diff(spec.atom_offset)], dtype=np.float64)


def tune(spec, lam, cache_path: str | None = None, candidates=CANDIDATES,
         target_atoms: int = 480000, force: bool = False, log=None) -> np.ndarray:
    """Column width per walker of `spec` (size-class choice, cached)."""
    cache = load_cache(cache_path)
    a = arch()
    n = np.diff(spec.atom_offset)
    widths = np.ones(spec.n_walkers)
    changed = False
    for cls in CLASSES:
        members = np.nonzero([size_class(int(x)) == cls for x in n])[0]
        if members.size == 0:
            continue
        key = _key(a, cls, spec.precision)
        if force or key not in cache:
            rep = int(members[np.argsort(n[members], kind="stable")[members.size // 2]])
            one, lam1 = synth.subset(spec, lam, [rep])
            k = max(1, target_atoms // int(n[rep]))
            batch, lamb = synth.batch(one, lam1, k, seed=spec.seed + 7)
            timings = {}
            for wdt in candidates:
                timings[f"{wdt:g}"] = time_width(batch, lamb, wdt)
                if log:
                    log(f"autotune {key}: width {wdt:g} -> {timings[f'{wdt:g}']['per_step_ms']:.4f} ms")
            best = min(candidates, key=lambda w_: timings[f"{w_:g}"]["per_step_ms"])
            cache[key] = {"column_width": float(best), "atoms": int(n[rep]), "replicas": k,
                          "timings_ms": {w_: round(t["per_step_ms"], 5) for w_, t in timings.items()}}
            changed = True
        widths[members] = cache[key]["column_width"]
    if changed:
        save_cache(cache, cache_path)
    return widths

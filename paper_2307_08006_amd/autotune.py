"""Tile-shape and prune-buffer autotuner for batches of uneven walkers.

Two knobs move the environment step.  The tile of the pair kernel is a
cluster of 8 atoms cut from a z-sorted x-y column; its shape is set by the
column width (in units of (8/rho)^(1/3): 1 gives cubic clusters).  Wider
columns mean fewer columns and less padding but flatter clusters whose
boxes admit more j atoms; narrower ones the reverse.  The prune buffer b
sets how far beyond r_cut the per-cluster pair lists reach: a larger b
prunes less often and evaluates more pairs.  For every size class present
in a batch the tuner times the step of its representative walker (the
member of median size, replicated to fill the GPU): first each candidate
width at the default buffer, then each candidate buffer at the best width.
The cost timed is the wall time per batched step over whole rebuild
blocks (HIP graphs, after a warm-up), as the batch runs in production:
timing the kernels one at a time overrates large prune buffers, because the
environment kernel runs faster alone than beside the alchemical one.  The
replicas are relaxed first and fill the GPU as the batch does.  A class's
choice is then kept only if it also speeds up the batch itself (timed
alternately against the knobs kept so far, by more than 1 %); otherwise
the class keeps the library defaults.  Knob effects are a few per cent at most, and a class's
replicas alone do not always rank them as the mixed batch does.

Results are cached in JSON keyed by GPU architecture, size class and
precision; the file named by $LABF_AUTOTUNE_CACHE, else autotune_cache.json
beside this module.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import labf, synth

# size classes by atoms per walker (lower bound inclusive)
CLASSES = [(0, 10000), (10000, 20000), (20000, 40000), (40000, 1 << 62)]
CANDIDATES = (0.8, 0.9, 1.0, 1.12, 1.25)
PRUNE_CANDIDATES = (0.25, 0.5, 0.7)  # A (besides the default 0.35), at most the list buffer
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


def relax(spec, lam, steps: int = 300):
    """The batch after `steps` steps of strong atom friction (50 fs), a 1 fs
    step and a rebuild every step, lambda fixed, no ABF: the synthetic start
    relaxed to the bath temperature.  Timed from the lattice start instead,
    the atoms leaving their sites move faster than in equilibrium and make
    small prune buffers re-prune more often than they do in production."""
    eq = dataclasses.replace(spec, gamma=20e-3, dt=1.0, rebuild_interval=1)
    lm = dataclasses.replace(lam, fixed_lambda=True, abf_on=False)
    with labf.System(eq, lm) as s:
        s.step(steps)
        pos, vel = s.read_atoms()
    return dataclasses.replace(spec, pos=pos, vel=vel)


def time_knobs(spec, lam, widths, buffers, reps: int = 4, warm_blocks: int = 6) -> float:
    """Per-step wall time (ms) of a batch at per-walker column widths and
    prune buffers (0: the library default): `reps` rebuild blocks of batched
    steps (HIP graphs, the kernels side by side as in production) after
    `warm_blocks` blocks of warm-up, which the device clocks need to ramp up.
    Kernels timed one at a time favour the wrong balance: the environment
    kernel runs faster alone than beside the alchemical one."""
    sp = dataclasses.replace(spec, column_width=np.asarray(widths, dtype=np.float64),
                             prune_buffer=np.asarray(buffers, dtype=np.float64))
    k = int(spec.rebuild_interval)
    with labf.System(sp, lam) as s:
        s.step(warm_blocks * k)
        s.read_walker_state()  # synchronises the library's stream
        t0 = time.perf_counter()
        s.step(reps * k)
        s.read_walker_state()
        dt = time.perf_counter() - t0
    return 1e3 * dt / (reps * k)


def time_width(spec, lam, width: float, prune_buffer: float = 0.0, reps: int = 4,
               warm_blocks: int = 6) -> dict:
    """time_knobs with one column width and prune buffer for every walker."""
    W = spec.n_walkers
    return {"per_step_ms": time_knobs(spec, lam, np.full(W, float(width)),
                                      np.full(W, float(prune_buffer)), reps, warm_blocks)}


def cached_widths(spec, cache_path: str | None = None) -> np.ndarray:
    """Column widths from the cache only (1 where a class is not cached)."""
    return cached_knobs(spec, cache_path)[0]


def cached_knobs(spec, cache_path: str | None = None):
    """(column widths, prune buffers) per walker from the cache only (1 and
    0, the library default, where a class is not cached)."""
    cache = load_cache(cache_path)
    a = arch()
    ent = [cache.get(_key(a, size_class(int(x)), spec.precision), {}) for x in np.diff(spec.atom_offset)]
    return (np.array([e.get("column_width", 1.0) for e in ent], dtype=np.float64),
            np.array([e.get("prune_buffer", 0.0) for e in ent], dtype=np.float64))


def tune(spec, lam, cache_path: str | None = None, candidates=CANDIDATES,
         prune_candidates=PRUNE_CANDIDATES, target_atoms: int | None = None, force: bool = False,
         log=None):
    """(column width, prune buffer) per walker of `spec`: the size-class
    choices, cached."""
    cache = load_cache(cache_path)
    a = arch()
    n = np.diff(spec.atom_offset)
    widths = np.ones(spec.n_walkers)
    buffers = np.zeros(spec.n_walkers)
    tuned = []  # (key, members) of the classes tuned in this call
    for cls in CLASSES:
        members = np.nonzero([size_class(int(x)) == cls for x in n])[0]
        if members.size == 0:
            continue
        key = _key(a, cls, spec.precision)
        if force or key not in cache or "prune_buffer" not in cache[key]:
            rep = int(members[np.argsort(n[members], kind="stable")[members.size // 2]])
            one, lam1 = synth.subset(spec, lam, [rep])
            # replicas fill the GPU as the whole batch does (the per-step fixed
            # costs weigh as much as in production), unless told otherwise
            k = max(1, (target_atoms or int(n.sum())) // int(n[rep]))
            batch, lamb = synth.batch(one, lam1, k, seed=spec.seed + 7)
            batch = relax(batch, lamb)
            t_w = {}
            for wdt in candidates:
                t_w[f"{wdt:g}"] = time_width(batch, lamb, wdt)["per_step_ms"]
                if log:
                    log(f"autotune {key}: width {wdt:g} -> {t_w[f'{wdt:g}']:.4f} ms")
            best_w = min(candidates, key=lambda w_: t_w[f"{w_:g}"])
            t_b = {"default": t_w[f"{best_w:g}"]}
            for b in prune_candidates:
                if b > spec.r_skin:
                    continue
                t_b[f"{b:g}"] = time_width(batch, lamb, best_w, b)["per_step_ms"]
                if log:
                    log(f"autotune {key}: width {best_w:g}, prune buffer {b:g} -> {t_b[f'{b:g}']:.4f} ms")
            best_b = min(t_b, key=t_b.get)
            cache[key] = {"column_width": float(best_w),
                          "prune_buffer": 0.0 if best_b == "default" else float(best_b),
                          "atoms": int(n[rep]), "replicas": k,
                          "timings_ms": {w_: round(t, 5) for w_, t in t_w.items()},
                          "prune_timings_ms": {b_: round(t, 5) for b_, t in t_b.items()}}
            tuned.append((key, members))
        widths[members] = cache[key]["column_width"]
        buffers[members] = cache[key]["prune_buffer"]
    if tuned:
        widths, buffers = check_on_batch(spec, lam, widths, buffers, cache, tuned, log)
        save_cache(cache, cache_path)
    return widths, buffers


def check_on_batch(spec, lam, widths, buffers, cache, tuned, log=None, reps: int = 2,
                   margin: float = 0.01):
    """Keep a class's replica-tuned knobs only where they speed up the batch
    itself.  A class's replicas fill the GPU alone; in the batch its walkers
    share every launch with the other classes, and knob effects of a per
    cent or two need not carry over.  Starting from the library defaults,
    each tuned class's knobs are tried on the (relaxed) batch in turn, timed
    alternately against the knobs kept so far (best of `reps`), and kept if
    they are faster by more than `margin` (about the run-to-run spread of a
    whole bench run: a smaller gain need not hold in the next run)."""
    batch = relax(spec, lam)
    cur_w, cur_b = np.ones(spec.n_walkers), np.zeros(spec.n_walkers)
    for key, members in tuned:
        ent = cache[key]
        if ent["column_width"] == 1.0 and ent["prune_buffer"] == 0.0:
            ent.update(batch_check_ms=None, accepted=True)
            continue
        cand_w, cand_b = cur_w.copy(), cur_b.copy()
        cand_w[members] = widths[members]
        cand_b[members] = buffers[members]
        t_cur, t_cand = [], []
        for _ in range(reps):
            t_cur.append(time_knobs(batch, lam, cur_w, cur_b))
            t_cand.append(time_knobs(batch, lam, cand_w, cand_b))
        ok = min(t_cand) < (1.0 - margin) * min(t_cur)
        ent["replica_choice"] = {"column_width": ent["column_width"], "prune_buffer": ent["prune_buffer"]}
        ent["batch_check_ms"] = {"kept": round(min(t_cur), 5), "with_class_knobs": round(min(t_cand), 5)}
        ent["accepted"] = bool(ok)
        if ok:
            cur_w, cur_b = cand_w, cand_b
        else:
            ent["column_width"], ent["prune_buffer"] = 1.0, 0.0
        if log:
            log(f"autotune {key}: on the batch {min(t_cur):.4f} -> {min(t_cand):.4f} ms, "
                f"{'kept' if ok else 'defaults kept'}")
    return cur_w, cur_b

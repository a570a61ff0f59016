"""Launch-shape autotuner for a stepper's time step.

The launch-shape knobs of libpic (tile sizes of the re-bin and of the fused
step, radix width, scatter staging and grouping, threads of the writing pass,
lanes and bins per deposit group, where the pushed state and the deposit are
computed, the ranking form) never change the re-binned state; they only change speed, and the best values depend on the
workload (dimension, particles per bin, how far particles move, how many
instances a forest holds).  ``autotune`` times every setting of the knobs that
matter for the chosen path on the actual state, restores the state after each
trial, applies the fastest setting and optionally caches it per workload
signature in a JSON file.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, Optional

from . import Stepper32, tune, tuning

# knobs each path depends on
SPACES = {
    # tile size, threads of the writing pass, lanes per deposit bin and bins
    # per lane group (the deposit's bucket), the writing-pass deposit, the
    # stored push, the ranking form
    "fused_f64": {"step_tile": (2048, 1024, 4096), "emit_threads": (1024, 512), "deposit_lanes": (64, 32, 16),
                  "deposit_bpw": (1, 2), "emit_deposit": (2, 0, 1), "key_stores": (2, 1), "group_match": (0, 1)},
    "calls_f64": {"rebin_tile": (2048, 4096), "rebin_radix": (4, 5), "scatter_mode": (0, 1),
                  "scatter_group": (4, 2, 1), "deposit_lanes": (64, 32, 16)},
    "f32": {"xcd_tiles": (1, 0), "key_stores": (2, 1, 0), "group_match": (0, 1)},
    "calls_f32": {"rebin_tile": (2048, 4096), "rebin_radix": (4, 5), "scatter_mode": (0, 1),
                  "scatter_group": (4, 2, 1)},
}


def _path(stepper, fused: bool) -> str:
    if isinstance(stepper, Stepper32):
        return "f32" if fused else "calls_f32"
    return "fused_f64" if fused else "calls_f64"


def signature(stepper, fused: bool) -> str:
    t = stepper.tree
    levels = sorted({t.instance(i).max_level for i in range(t.n_inst)})
    return (f"d{t.dim}_inst{t.n_inst}_L{'-'.join(map(str, levels))}_s{stepper.scheme}_{_path(stepper, fused)}"
            f"_n{stepper.n}_bins{t.n_bins(stepper.scheme)}")


def _state(stepper):
    names = ("off", "u", "q", "ids", "start") if isinstance(stepper, Stepper32) else ("x", "v", "q", "ids", "start")
    return {k: getattr(stepper, k).clone() for k in names if getattr(stepper, k) is not None}


def _restore(stepper, saved):
    for k, v in saved.items():
        getattr(stepper, k).copy_(v)


def _time_steps(stepper, fused, step_args, step_kw, steps):
    import torch
    f = stepper.step_fused if fused else stepper.step
    f(*step_args, **step_kw)                       # settle the new launch shape
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        f(*step_args, **step_kw)
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


def autotune(stepper, E, qmdt, dt, q_uniform=0.0, fused=True, steps=3, cache: Optional[str] = None,
             log=None, **kw) -> Dict[str, int]:
    """Pick the fastest launch shape for ``stepper``'s step and apply it to
    the stepper's tree (other trees keep their own knobs).

    Returns the chosen knob values.  With ``cache`` (a JSON path) a setting
    found earlier for the same workload signature is applied without timing,
    and new results are added to the file.
    """
    sig = signature(stepper, fused)
    tree = stepper.tree
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
        if sig in known:
            for k, v in known[sig]["knobs"].items():
                tune(k, v, tree)
            return dict(known[sig]["knobs"])
    space = SPACES[_path(stepper, fused)]
    saved = _state(stepper)
    base = tuning(tree)
    args, kwargs = (E, qmdt, dt), dict(kw, q_uniform=q_uniform)
    results = []
    try:
        for combo in itertools.product(*space.values()):
            setting = dict(zip(space.keys(), combo))
            for k, v in setting.items():
                tune(k, v, tree)
            _restore(stepper, saved)
            ms = _time_steps(stepper, fused, args, kwargs, steps)
            results.append((ms, setting))
            if log:
                log(f"[autotune] {setting} {ms:.4f} ms/step")
    finally:
        _restore(stepper, saved)
        for k, v in base.items():
            tune(k, v, tree)
    best_ms, best = min(results, key=lambda r: r[0])
    for k, v in best.items():
        tune(k, v, tree)
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
        known[sig] = {"knobs": best, "ms_per_step": best_ms, "trials": len(results)}
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1, sort_keys=True)
    return dict(best)

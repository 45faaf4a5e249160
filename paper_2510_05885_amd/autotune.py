"""Autotuner for the front shapes of a KKT pattern.

The plan knobs that decide the front shapes are:
  * small_front_max — fronts up to this order are factored by one workgroup
    entirely in LDS; larger fronts take the global-memory MFMA path;
  * relax_big_zeros — how many explicit zeros supernode amalgamation may add to
    large fronts (wider fronts: fewer levels and contribution-block copies,
    more flops).
For a given pattern, each candidate is analyzed and timed on the device
(factor + one solve, median of a few repetitions, values of the caller's
choosing), and the fastest is cached in a JSON file keyed by device
architecture, precision, form and a hash of the pattern.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from .ncl_kkt import KKT

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
CANDIDATES = [(fm, z) for fm in (64, 96, 128) for z in (0.1, 0.2, 0.3)]


def pattern_key(inp, form: str, precision: str, arch: str) -> str:
    h = hashlib.sha1()
    for a in (inp.W_colptr, inp.W_rowidx, inp.J_rowptr, inp.J_colidx):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    return f"{arch}|{precision}|{form}|n{inp.n}|m{inp.m}|{h.hexdigest()[:16]}"


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def tune(inp, form: str = "condensed", precision: str = "fp64", reps: int = 3, candidates=None,
         use_cache: bool = True, log=None):
    """Return the best plan options {small_front_max, relax_big_zeros} for this pattern."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = pattern_key(inp, form, precision, arch)
    cache = _load()
    if use_cache and key in cache:
        return cache[key]["best"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    W, S, J = dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val)
    order = inp.n if form == "condensed" else inp.n + inp.m
    B = dev(np.random.default_rng(0).standard_normal(order))
    results = []
    for fm, z in (candidates or CANDIDATES):
        try:
            k = KKT.from_input(inp, form=form, precision=precision, small_front_max=fm, relax_big_zeros=z)
        except Exception as e:   # e.g. a bound above the device's LDS limit
            if log:
                log(f"autotune: skip ({fm}, {z}): {e}")
            continue
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            k.factor(W, S, J, inp.rho)
            k.solve(B)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t)
        st = k.stats()
        k.close()
        med = float(np.median(times))
        results.append({"small_front_max": fm, "relax_big_zeros": z, "seconds": med,
                        "flops": st["flops_factor"], "levels": st["n_levels"]})
        if log:
            log(f"autotune: small_front_max={fm} relax_big_zeros={z}: {med * 1e3:.2f} ms "
                f"(levels {st['n_levels']}, flops {st['flops_factor']:.2e})")
    best = min(results, key=lambda r: r["seconds"])
    best = {"small_front_max": best["small_front_max"], "relax_big_zeros": best["relax_big_zeros"]}
    cache[key] = {"best": best, "trials": results}
    with open(CACHE, "w") as f:
        json.dump(cache, f, indent=1)
    return best

"""Autotuner of the step kernel's launch configuration.

The design space (`intervals` consecutive coupling intervals of a seeded
sample of the caller's workload per candidate, the first from a cold start
and the others warm-started from it as a coupling loop runs them, timed
with HIP events on the launching stream, every candidate from the same start
state):
  * lanes per particle and placement of the Newton matrix: one lane with a
    dense pivoted LU in private memory (ADM1_VARIANT_DENSE1), one lane with
    the static sparse LU in registers (SPARSE1) or in LDS (SPARSE1_LDS), two
    lanes with the rows split over the pair in registers (SPARSE2);
  * for the two-lane persistent kernel, resident waves per compute unit
    (1-4) and the service batch (pairs restarted together: 1, 2, 4, 8).
The fastest is set on the context (adm1_set_launch, adm1_set_service_batch),
so the default step path (opts.variant = -1) uses it.  Choices are cached in
a JSON file keyed by GPU architecture, sample size, tolerance and tag; the
package ships the choices measured on gfx950 (data/autotune_choices.json),
so a fresh machine of that architecture starts from them.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import adm1 as A

# (variant, waves per CU, service batch); 0 = the library default
CANDIDATES = ([(A.VARIANT_DENSE1, 0, 0), (A.VARIANT_SPARSE1, 0, 0),
               (A.VARIANT_SPARSE1_LDS, 0, 0)] +
              [(A.VARIANT_SPARSE2, b, sb) for b in (1, 2, 3, 4) for sb in (1, 2, 4, 8)])
LABELS = {A.VARIANT_DENSE1: "1 lane, dense LU in private memory",
          A.VARIANT_SPARSE1: "1 lane, sparse LU in registers",
          A.VARIANT_SPARSE1_LDS: "1 lane, sparse LU in LDS",
          A.VARIANT_SPARSE2: "2 lanes, sparse LU rows split over the pair in registers"}


def describe(choice) -> dict:
    v, b, sb = choice
    d = {"variant": int(v), "layout": LABELS.get(int(v), "?")}
    if v == A.VARIANT_SPARSE2:
        d.update(waves_per_cu=int(b) or 4, service_batch=int(sb) or 4)
    return d


def apply(ctx: "A.Context", choice):
    v, b, sb = (int(c) for c in choice)
    A.adm1_set_launch(ctx.handle, v, b)
    A.adm1_set_service_batch(ctx.handle, sb)


CACHE = os.environ.get("ADM1_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "adm1_autotune.json"))
# choices measured once per architecture and shipped with the package; a
# user cache entry with the same key takes precedence
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                        "autotune_choices.json")


def _key(arch: str, n: int, rtol: float, tag: str) -> str:
    return f"{arch}|n={n}|rtol={rtol:g}|{tag}"


def _read(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def load_cache() -> dict:
    """Packaged choices, overridden by the user cache."""
    d = {k: dict(v, source="packaged") for k, v in _read(PACKAGED).items()}
    d.update({k: dict(v, source="user cache") for k, v in _read(CACHE).items()})
    return d


def save_cache(d: dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def autotune(ctx: "A.Context", X, T, D, fidx, S_in, dt, n=None, tag="", repeats=2,
             candidates=CANDIDATES, use_cache=True, log=None, intervals=1) -> dict:
    """Time the candidates on (X, T, D, fidx, S_in) -- device tensors of the
    sample -- over `intervals` coupling intervals each (the cold one, then
    warm ones); returns {choice, timings_ms, layout}.  X is not modified."""
    import torch
    n = X.shape[1] if n is None else n
    arch = torch.cuda.get_device_properties(X.device).gcnArchName
    key = _key(arch, n, ctx.opts.rtol, tag)
    cache = load_cache() if use_cache else {}
    if key in cache and len(cache[key].get("choice", [])) == 3:
        apply(ctx, cache[key]["choice"])
        return dict(cache[key], cached=True)
    cache = _read(CACHE) if use_cache else {}
    saved_variant = ctx.opts.variant
    ctx.set_opts(variant=-1)
    timings = {}
    stream = torch.cuda.current_stream()
    for cand in candidates:
        apply(ctx, cand)
        ts = []
        for _ in range(repeats):
            Xw = X.clone()
            H = torch.full((n,), -1.0, dtype=torch.float64, device=X.device)
            hl = torch.full((n,), -1.0, dtype=torch.float64, device=X.device)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(intervals):
                ctx.step(Xw, T, D, fidx, S_in, dt, n=n, H=H, hlast=hl, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        timings[":".join(map(str, cand))] = float(np.median(ts))
        if log:
            log(f"# autotune {cand}: {timings[':'.join(map(str, cand))]:.2f} ms")
    best = min(timings, key=timings.get)
    choice = [int(t) for t in best.split(":")]
    apply(ctx, choice)
    ctx.set_opts(variant=saved_variant)
    out = {"choice": choice, "layout": describe(choice), "timings_ms": timings}
    if use_cache:
        cache[key] = out
        save_cache(cache)
    return out

"""Launch-shape autotuner for kh_integrate.

The paper's framework benchmarks alternative implementations at run time and
keeps the fastest (Sec. 2.3, and Sec. 4's work-group-size tuning).  Here the
alternatives are launch shapes of the persistent kernel: threads per block,
register budget (kernel variant with a minimum waves-per-SIMD target) and the
refill threshold, and for MIXED DOPRI5 the policy that places the FP64
right-hand sides (per-wave switch or two-queue split, `mixed_split`).  For
FP64, FP32 and the two-queue split the launch shape changes only the
schedule, never a result (each lane's arithmetic is fixed), so tuning is
safe; per-wave-switch MIXED results depend on which rays share a wave, and
the two policies give results that differ within the mixed tolerance.

Usage: ``best = tune(ctx, reinit, state, params, key)`` where ``reinit()``
re-initialises ``state`` to the tuning sample before each timed run.  The
choice is cached in a JSON file keyed by device and ``key``.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import torch

from . import DOPRI5, P32, P64, PMIXED, RHS_FACTORED, kh_params

CACHE_ENV = "KERRHIP_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kerrhip_autotune.json")

# waves-per-SIMD register budgets compiled for each precision (DOPRI5, factored
# RHS); MIXED under the two-queue split has the first two
WAVE_VARIANTS = {P64: (1, 3, 4), P32: (1, 4, 5), PMIXED: (1, 3, 4)}
SPLIT_WAVE_VARIANTS = (1, 3)


def candidates(params: kh_params):
    dp5_factored = params.method == DOPRI5 and params.rhs_form == RHS_FACTORED
    splits = (0, 1) if (params.precision == PMIXED and params.method == DOPRI5) else (params.mixed_split,)
    for split in splits:
        waves = WAVE_VARIANTS.get(params.precision, (1,)) if dp5_factored else (1,)
        if split:
            waves = SPLIT_WAVE_VARIANTS
        for block, wpe, refill in itertools.product((64, 128, 256), waves, (4, 8, 12, 16)):
            yield dict(block_size=block, waves_per_eu=wpe, refill_min=refill, mixed_split=split)


def _device_key():
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply(params: kh_params, choice: dict) -> kh_params:
    out = kh_params()
    for f, _ in kh_params._fields_:
        setattr(out, f, getattr(params, f))
    for k, v in choice.items():
        setattr(out, k, v)
    return out


def tune(ctx, reinit, state, params: kh_params, key: str, reps: int = 2, cache_path: str | None = None,
         use_cache: bool = True, log=None) -> dict:
    """Return the fastest launch shape for ``params`` on the tuning sample."""
    cache_path = cache_path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    full_key = f"{_device_key()}|{key}|m{params.method}|p{params.precision}|f{params.rhs_form}"
    cache = _load(cache_path) if use_cache else {}
    if full_key in cache:
        return cache[full_key]["choice"]
    results = []
    for cand in candidates(params):
        p = apply(params, cand)
        best = float("inf")
        for _ in range(reps):
            reinit()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.kh_integrate(p, state)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        results.append((best, cand))
        if log:
            log(f"autotune {cand}: {best * 1e3:.3f} ms")
    results.sort(key=lambda t: t[0])
    choice = results[0][1]
    cache[full_key] = {"choice": choice, "ms": results[0][0] * 1e3, "worst_ms": results[-1][0] * 1e3,
                       "n_candidates": len(results)}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    except OSError:
        pass
    return choice

"""Autotuner for the launch shapes of the outer Krylov passes.

For a batch of jobs it times every combination of the context's tuning keys
(``xcd_map``, ``split_dual``) on a short probe of the same batch (the outer
basis for ``k_probe`` steps, stencil and recurrence passes timed with the
library's sampled HIP events), keeps the fastest, applies it to the context
and caches it in a JSON file keyed by (GPU arch, lattice dims, jobs per
lattice, precision, Hermitian / two-sided).  ``schedule`` then times whole
batched calls for the order of the lattice groups (all nested steps after
all outer loops, or each group's nested step after its own loop with the
other groups started late, ``stagger_groups`` percent into the lead group's
loop).  Every choice gives bit-identical results, so tuning never changes a
result.

Cache file: ``$NKS_TUNE_CACHE`` or ``~/.cache/nks/tune.json``.
"""
from __future__ import annotations

import itertools
import json
import os

SPACE = {"xcd_map": (0, 1, 2, 3), "split_dual": (0, 1), "min_waves": (1, 3, 4)}


def _cache_path() -> str:
    return os.environ.get("NKS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "nks",
                                                               "tune.json")


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def batch_key(jobs) -> str:
    groups = {}
    for j in jobs:
        lat = j["lat"]
        key = (lat.dims, j.get("precision", "fp64"), lat.mu != 0.0)
        groups[key] = groups.get(key, 0) + 1
    parts = [f"{'x'.join(map(str, d))}:{p}:{'2s' if ts else 'h'}:{n}" for (d, p, ts), n in sorted(groups.items())]
    return _arch() + "|" + ",".join(parts)


def _probe(ctx, jobs, k_probe: int) -> float:
    """ms per outer iteration (stencil + recurrence) of the batch, from sampled events."""
    import paper_0912_4457_amd as nks
    probe = [dict(j, k=k_probe, ell=2, p=1.0) for j in jobs]
    nks.sign_apply_batch(probe, stats=False)          # warm
    ctx.profile(True)
    nks.sign_apply_batch(probe, stats=False)
    n1, ms1, _ = ctx.profile_read("stencil")
    n2, ms2, _ = ctx.profile_read("recurrence")
    ctx.profile_read("nested")
    ctx.profile_read("lift")
    ctx.profile(False)
    return (ms1 / max(n1, 1)) + (ms2 / max(n2, 1))


def autotune(ctx, jobs, k_probe: int = 48, use_cache: bool = True) -> dict:
    """Pick and apply the fastest tuning for this batch; returns the choice."""
    key = batch_key(jobs)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        choice = cache[key]["choice"]
    else:
        timings = {}
        for combo in itertools.product(*SPACE.values()):
            cfg = dict(zip(SPACE.keys(), combo))
            for k_, v_ in cfg.items():
                ctx.tune_set(k_, v_)
            timings[json.dumps(cfg, sort_keys=True)] = _probe(ctx, jobs, k_probe)
        best = min(timings, key=timings.get)
        choice = json.loads(best)
        cache[key] = {"choice": choice, "ms_per_iteration": timings}
        if use_cache:
            _save_cache(cache)
    for k_, v_ in choice.items():
        ctx.tune_set(k_, v_)
    return {"key": key, "choice": choice, "timings": cache.get(key, {}).get("ms_per_iteration")}


SCHEDULES = ({"pipeline_groups": 0, "stagger_groups": 0},) + tuple(
    {"pipeline_groups": 1, "stagger_groups": s} for s in (0, 20, 30, 35, 40, 45, 50))


def schedule(ctx, jobs, calls: int = 4, rounds: int = 2) -> dict:
    """Pick and apply the fastest group schedule for this batch by timing
    whole calls (graph replay, no stats); returns the choice and the best
    seconds per call of every candidate."""
    import time
    import torch
    import paper_0912_4457_amd as nks
    if len({(id(j["lat"]), j.get("precision", "fp64")) for j in jobs}) < 2:
        choice = dict(SCHEDULES[0])
        for k_, v_ in choice.items():
            ctx.tune_set(k_, v_)
        return {"choice": choice, "seconds_per_call": {}}
    best = {}
    for _ in range(rounds):
        for cfg in SCHEDULES:
            for k_, v_ in cfg.items():
                ctx.tune_set(k_, v_)
            nks.sign_apply_batch(jobs, stats=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                nks.sign_apply_batch(jobs, stats=False)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / calls
            key = json.dumps(cfg, sort_keys=True)
            best[key] = min(best.get(key, dt), dt)
    choice = json.loads(min(best, key=best.get))
    for k_, v_ in choice.items():
        ctx.tune_set(k_, v_)
    return {"choice": choice, "seconds_per_call": best}

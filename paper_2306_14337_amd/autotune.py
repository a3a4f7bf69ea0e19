"""Schedule autotuner: picks the launch schedule of the refactor/solve path for
one sparsity pattern by timing candidates on the user's own matrix.

Knobs (all fields of the C options struct):
  schedule                  1 level-synchronous launches, 2 dependency-driven
  sync_mode                 1 acquire/release fences, 2 device-coherent accesses
  solve_entries_per_lane    triangular-solve lanes per row (entries per lane)
  refactor_waves_per_block  rows in flight per workgroup in the refactorization
  solve_thin_rows           widest level of the one-workgroup solve segments
  dense_tail                size of the dense trailing block (0 auto, -1 none)
  refactor_short_rows       short-row band as update lists (0) or pivot by pivot (-1)
  refactor_long_rows        long-row band with prefetched steps (0) or not (-1)
  refactor_short_band       longest row of the short-row band (0 = 128, up to 256)

The search is in two stages: the launch-shape candidates first, then the
segment, dense-block and refactorization-kernel variants of the winner.

The winner is cached in a JSON file keyed by a hash of the pattern (n, row
pointers, column indices), so a later run with the same pattern skips the
search.  Candidates that fail (e.g. a schedule the pattern cannot use) are
skipped.

autotune_batch does the same for a block-diagonal batch (kkt_analyze_batch):
it times replays of the captured batch graph (refactorization, solve and
device-checked refinement) for each candidate, first one knob away from the
library defaults at a time, then the combination of the knobs that won, and
caches the winner under a hash of every pattern and the instance map.  Batch
knobs:
  refactor_crit_height      rows with this many rows chained after them first
  refactor_micro_rows       micro rows one per lane (0) or a wave per row (-1)
  refactor_waves_per_cu     resident waves per CU of the refactorization
  solve_entries_per_lane    lane-group width of the single-row solve chunks
  solve_blocks_per_cu       resident workgroups per CU of the solves
  solve_chain               longest chain block of the solves
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np

DEFAULT_CACHE = os.environ.get(
    "KKTLU_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "kktlu_autotune.json"))


def pattern_key(n, rowptr, colind) -> str:
    h = hashlib.sha256()
    h.update(np.int64(n).tobytes())
    h.update(np.ascontiguousarray(rowptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(colind, dtype=np.int32).tobytes())
    return h.hexdigest()[:32]


def candidates(full: bool = False):
    """Option dicts to try; the first is the library default."""
    out = [dict(schedule=2, sync_mode=2, solve_entries_per_lane=8, refactor_waves_per_block=0)]
    spl = (2, 4, 8, 16) if full else (4, 8, 16)
    wpb = (0, 1, 2, 4) if full else (0, 1)
    for s, e, w in itertools.product((1, 2), spl, wpb):
        c = dict(schedule=2, sync_mode=s, solve_entries_per_lane=e, refactor_waves_per_block=w)
        if c not in out:
            out.append(c)
    out.append(dict(schedule=1, sync_mode=0, solve_entries_per_lane=8, refactor_waves_per_block=0))
    return out


def refinements(best: dict):
    """Second-stage variants of the first stage's winner."""
    out = []
    if best.get("schedule") != 2:
        return out
    for thin in (-1, 16):
        out.append({**best, "solve_thin_rows": thin})
    out.append({**best, "dense_tail": -1})
    out.append({**best, "refactor_short_rows": -1})
    out.append({**best, "refactor_long_rows": -1})
    out.append({**best, "refactor_short_band": 256})
    return out


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: str = DEFAULT_CACHE) -> None:
    cache = load_cache(path)
    cache[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(n, rowptr, colind, values0, d_values, d_b, repeats: int = 3, full: bool = False,
             cache_path: str | None = DEFAULT_CACHE, base_options: dict | None = None):
    """Time refactor+solve for every candidate on (d_values, d_b) and return
    (best option dict, {candidate index: seconds per step}).  Uses the cache
    when the pattern was tuned before."""
    import torch

    from . import binding

    key = pattern_key(n, rowptr, colind)
    if cache_path:
        hit = load_cache(cache_path).get(key)
        if hit:
            return dict(hit["options"]), {}
    base = dict(base_options or {})
    times = {}
    best, best_t = None, float("inf")

    def run(cand):
        opts = {**base, **cand}
        try:
            s = binding.KKTSolver(**opts)
            s.analyze(n, rowptr, colind, values0)
            x = torch.empty_like(d_b)
            s.refactor(d_values)
            s.solve(d_b, x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(repeats):
                s.refactor(d_values)
                s.solve(d_b, x)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / repeats
            s.close()
        except binding.KKTError:
            return None
        return dt

    first = candidates(full)
    for idx, cand in enumerate(first):
        dt = run(cand)
        if dt is None:
            continue
        times[idx] = dt
        if dt < best_t:
            best, best_t = cand, dt
    if best is None:
        raise RuntimeError("no autotuner candidate ran")
    for idx, cand in enumerate(refinements(best), start=len(first)):
        dt = run(cand)
        if dt is None:
            continue
        times[idx] = dt
        if dt < best_t:
            best, best_t = cand, dt
    if cache_path:
        store_cache(key, {"options": best, "seconds_per_step": best_t, "n": int(n)}, cache_path)
    return dict(best), times


def batch_key(patterns, inst_pattern) -> str:
    h = hashlib.sha256(b"batch")
    for n, rowptr, colind, _ in patterns:
        h.update(pattern_key(n, rowptr, colind).encode())
    h.update(np.ascontiguousarray(inst_pattern, dtype=np.int32).tobytes())
    return h.hexdigest()[:32]


def batch_candidates(full: bool = False):
    """First-stage batch candidates: the library defaults, then one knob away."""
    out = [dict()]
    knobs = [dict(refactor_crit_height=-1), dict(refactor_crit_height=8),
             dict(refactor_micro_rows=-1), dict(solve_entries_per_lane=4),
             dict(solve_entries_per_lane=16), dict(solve_blocks_per_cu=4)]
    if full:
        knobs += [dict(refactor_waves_per_cu=16), dict(solve_chain=8), dict(solve_chain=-1),
                  dict(refactor_short_band=256)]
    return out + knobs


def autotune_batch(patterns, inst_pattern, d_values, d_b, repeats: int = 3, full: bool = False,
                   candidates=None, cache_path: str | None = DEFAULT_CACHE,
                   base_options: dict | None = None):
    """Time captured batch-graph replays for every candidate option set on
    (d_values, d_b); return (best option dict, {repr(candidate): ms per
    replay}).  Uses the cache when the batch was tuned before."""
    import torch

    from . import binding

    key = batch_key(patterns, inst_pattern)
    if cache_path:
        hit = load_cache(cache_path).get(key)
        if hit:
            return dict(hit["options"]), {}
    base = dict(base_options or {})
    times = {}

    def run(cand):
        opts = {**base, **cand}
        try:
            s = binding.KKTSolver(**opts)
            s.analyze_batch(patterns, inst_pattern)
            x = torch.empty_like(d_b)
            stream = torch.cuda.Stream()
            torch.cuda.synchronize()
            s.graph_capture(d_values, d_b, x, stream)
            s.graph_launch(stream)
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(repeats):
                s.graph_launch(stream)
            e1.record(stream)
            stream.synchronize()
            if not float(s.batch_eta().max()) <= s.options.eta_target:
                return None
            ms = e0.elapsed_time(e1) / repeats
            s.close()
        except binding.KKTError:
            return None
        return ms

    first = list(candidates) if candidates is not None else batch_candidates(full)
    best, best_t = None, float("inf")
    winners = []
    base_t = None
    for cand in first:
        ms = run(cand)
        if ms is None:
            continue
        times[repr(cand)] = ms
        if cand == {}:
            base_t = ms
        elif base_t is not None and ms < base_t:
            winners.append(cand)
        if ms < best_t:
            best, best_t = cand, ms
    if best is None:
        raise RuntimeError("no batch autotuner candidate ran")
    # second stage: every knob that beat the defaults, together
    if len(winners) > 1:
        combo = {}
        for w in winners:
            for k, v in w.items():
                combo.setdefault(k, v)
        ms = run(combo)
        if ms is not None:
            times[repr(combo)] = ms
            if ms < best_t:
                best, best_t = combo, ms
    if cache_path:
        store_cache(key, {"options": best, "ms_per_replay": best_t, "batch": True}, cache_path)
    return dict(best), times

"""Autotuner of the persistent fused pass: picks tile size, workgroup size and persistent
workgroups per compute unit for a workload by timing graph replays of svt_process_batch.

Every candidate must write exactly the same bytes (the schedule does not change the result);
the tuner checks this on each candidate, so tuning doubles as a race/determinism sweep.
Results are cached in a JSON file keyed by device name and a workload signature.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
import time
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from . import pipeline as P

TILES = (4096, 8192)
WG_SIZES = (256, 512)
OCCUPANCIES = (1, 2, 3, 4)
ONEPASS_OCCUPANCIES = (1, 2, 3)
CHUNK_ROADS = (32, 64)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "svt_tune.json")


EVENT_OCCUPANCIES = (2, 4)
# Candidates within this fraction of the fastest time are ties, won by the earliest in the
# fixed candidate order: repeated runs on one batch of 8192 uneven events moved the
# candidates' medians by up to about 2 %, which otherwise flips the pick between near-equal
# shapes from run to run.
TIE = 0.025


def candidates():
    """The one-pass kernel at each resident grid size, the flat-tile shapes of the two-kernel
    pass (tile, roads per chunk, workgroup size, workgroups per CU), and the
    one-event-per-workgroup schedule."""
    onepass = [L.make_tune(0, 0, 0, occ, L.SVT_SCHEDULE_ONEPASS) for occ in ONEPASS_OCCUPANCIES]
    flat = [L.make_tune(t, ch, wg, occ, L.SVT_SCHEDULE_TILES)
            for t in TILES for ch in CHUNK_ROADS for wg in WG_SIZES for occ in OCCUPANCIES]
    events = [L.make_tune(4096, 64, 256, occ, L.SVT_SCHEDULE_EVENTS)
              for occ in EVENT_OCCUPANCIES]
    return [L.svt_tune_resolve(t) for t in onepass + flat + events]


def tune_tuple(t: L.svt_tune):
    return (t.tile_combos, t.chunk_roads, t.wg_size, t.wgs_per_cu, t.schedule)


def workload_key(n_words: int, n_roads: int, n_combos: int, device: str) -> str:
    """Cache key: device plus the batch shape rounded to 2 significant digits."""
    def r2(x):
        return float(f"{x:.2g}")
    sig = f"{device}|w{r2(n_words)}|r{r2(n_roads)}|c{r2(n_combos)}"
    return hashlib.sha1(sig.encode()).hexdigest()[:16] + "|" + sig


@dataclasses.dataclass
class TuneResult:
    tune: L.svt_tune
    ms_per_pass: float
    table: list  # (tile, chunk, wg, occ, schedule, ms)
    statistic: str = ""


def _digest(res: dict) -> str:
    h = hashlib.sha1()
    for k in ("p0", "p1", "p2", "chi2", "accept", "best_k", "best_chi2", "best_n_accept"):
        h.update(res[k].cpu().numpy().tobytes())
    return h.hexdigest()


def autotune(words: torch.Tensor, bank: torch.Tensor, cfg: L.svt_config, n_roads: int,
             n_combos: int, samples: int = 30, per_sample: int = 5, warmup: int = 3,
             cands=None, cache_path: Optional[str] = DEFAULT_CACHE, use_cache: bool = True,
             log=None) -> TuneResult:
    """Time every candidate on this batch (graph replays) and return the fastest (ties within
    TIE of it go to the earliest candidate in order).

    A candidate's time is the median over ``samples`` samples, each the mean of
    ``per_sample`` back-to-back replays (host clock, synchronised around the sample), so one
    stall of the runtime moves one sample and not the pick.  ``words`` is a device int32
    tensor of the batch's hit words.  Raises if two candidates disagree on any output byte.
    """
    dev = torch.cuda.get_device_name()
    key = workload_key(words.numel(), n_roads, n_combos, dev)
    if use_cache and cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached:
            t = L.make_tune(*cached["tune"])
            return TuneResult(t, cached["ms_per_pass"], cached.get("table", []), "cached")
    table = []
    ref_digest = None
    timed = []
    for t in (cands or candidates()):
        runner = P.BatchRunner(cfg, bank, words.numel(), n_roads, n_combos, kept_cap=0, tune=t,
                               graph=True, with_c=False)
        runner.load(words)
        for _ in range(warmup):
            runner.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(samples):
            t0 = time.perf_counter()
            for _ in range(per_sample):
                runner.run()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / per_sample * 1e3)
        ms = float(np.median(ts))
        d = _digest(runner.result())
        if ref_digest is None:
            ref_digest = d
        elif d != ref_digest:
            raise RuntimeError(f"tune {tune_tuple(t)} changed the output bytes")
        table.append((*tune_tuple(t), round(ms, 5)))
        if log:
            log(f"tune {tune_tuple(t)}: {ms:.4f} ms")
        timed.append((t, ms))
        L.svt_release_graphs()
        del runner
        torch.cuda.empty_cache()
    fastest = min(ms for _, ms in timed)
    best = next((t, ms) for t, ms in timed if ms <= fastest * (1 + TIE))
    res = TuneResult(best[0], best[1], table,
                     f"median of {samples} samples of {per_sample} graph replays; within "
                     f"{TIE:.1%} of the fastest the first candidate in order")
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        try:
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = dict(tune=list(tune_tuple(res.tune)), ms_per_pass=res.ms_per_pass,
                         table=table)
        tmp = cache_path + ".tmp"
        json.dump(data, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return res


def pick_launch_mode(runner: P.BatchRunner, samples: int = 30, per_sample: int = 5,
                     warmup: int = 3):
    """Time one batch runner with graph replays and with direct launches (the same statistic as
    autotune) and leave it in the faster mode.  Returns {"graph": ms, "direct": ms}.

    The pass is the same kernels either way; on ROCm a replayed graph costs several
    microseconds more per pass than launching its kernels directly, which matters for batches
    whose pass takes tens of microseconds."""
    times = {}
    for graph in (True, False):
        runner.graph = graph
        for _ in range(warmup):
            runner.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(samples):
            t0 = time.perf_counter()
            for _ in range(per_sample):
                runner.run()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / per_sample * 1e3)
        times["graph" if graph else "direct"] = round(float(np.median(ts)), 5)
    runner.graph = times["graph"] <= times["direct"]
    return times


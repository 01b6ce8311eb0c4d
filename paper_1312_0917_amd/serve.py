"""Continuous-batching request loop for the SVT fitter.

Events arrive over time (a Poisson stream in the benchmark).  The scheduler keeps a FIFO of
arrived events and a few *slots*; each slot owns resident device buffers sized for one batch
(the memory it may use), a stream, pinned host staging and, for the fused path, a captured HIP
graph.  Whenever a slot is free, the scheduler admits the longest FIFO prefix of arrived events
that fits the slot's memory (at most ``max_events`` events) and launches it: host-to-device copy
of the packed words, the fit, device-to-host copy of the results, all asynchronous on the
slot's stream.  Several slots are in flight at once, so transfers and kernels of different
batches overlap.  Latency of an event = time its results are on the host - its arrival time;
it includes both transfers, as the paper's loop-latency measurements do (section IV-C).

Slots are an interface: ``GpuSlot`` (fused persistent pass), ``PlainSlot`` (one launch per stage,
host synchronisations in between) and, for CPU tests of the scheduling logic, any object with
the same methods.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class EventStream:
    """Events as contiguous slices of one packed word array (arrival order = stream order)."""
    words: np.ndarray           # uint32, all events back to back
    event_word_begin: np.ndarray  # int64 [n_events + 1]
    arrival_s: np.ndarray       # float64 [n_events], seconds from the start

    @property
    def n_events(self) -> int:
        return len(self.arrival_s)

    def n_words(self, e0: int, e1: int) -> int:
        return int(self.event_word_begin[e1] - self.event_word_begin[e0])

    def slice(self, e0: int, e1: int) -> np.ndarray:
        return self.words[self.event_word_begin[e0]:self.event_word_begin[e1]]


@dataclasses.dataclass
class ServeStats:
    latency_s: np.ndarray        # per event
    batch_sizes: List[int]
    n_combos: int
    wall_s: float
    retries: int = 0

    def percentile_us(self, q) -> float:
        return float(np.percentile(self.latency_s, q) * 1e6)

    def summary(self, warmup_events: int = 0) -> dict:
        lat = self.latency_s[warmup_events:]
        return dict(events=int(len(lat)), p50_us=round(float(np.percentile(lat, 50)) * 1e6, 2),
                    p99_us=round(float(np.percentile(lat, 99)) * 1e6, 2),
                    max_us=round(float(lat.max()) * 1e6, 2),
                    mean_us=round(float(lat.mean()) * 1e6, 2),
                    batches=len(self.batch_sizes),
                    mean_batch=round(float(np.mean(self.batch_sizes)), 2),
                    combos_per_s=self.n_combos / self.wall_s if self.wall_s > 0 else 0.0,
                    retries=self.retries)


def serve(stream: EventStream, slots: Sequence, max_events: int = 256,
          clock: Callable[[], float] = time.perf_counter, keep_results: bool = False,
          idle_sleep_s: float = 0.0):
    """Run the whole stream through the slots; returns (ServeStats, per-event results or None).

    A slot provides: ``fits(n_words, n_events) -> bool``, ``launch(words, e0, e1)``,
    ``poll() -> bool`` (finished), ``collect() -> (n_combos, per_event_results or None)``.
    """
    n = stream.n_events
    lat = np.full(n, np.nan)
    results = [None] * n if keep_results else None
    fifo = deque()
    nxt = 0
    busy = {}  # slot index -> (e0, e1)
    batch_sizes = []
    total_combos = 0
    done = 0
    t0 = clock()
    while done < n:
        now = clock() - t0
        while nxt < n and stream.arrival_s[nxt] <= now:
            fifo.append(nxt)
            nxt += 1
        progressed = False
        for si in list(busy):
            if slots[si].poll():
                e0, e1 = busy.pop(si)
                t_done = clock() - t0
                nc, per_event = slots[si].collect()
                total_combos += nc
                lat[e0:e1] = t_done - stream.arrival_s[e0:e1]
                if keep_results:
                    for i, r in enumerate(per_event):
                        results[e0 + i] = r
                done += e1 - e0
                progressed = True
        for si, slot in enumerate(slots):
            if si in busy or not fifo:
                continue
            e0 = fifo[0]
            # longest FIFO prefix (consecutive events) that fits this slot's memory
            e1 = e0 + 1
            limit = min(e0 + max_events, e0 + len(fifo))
            while e1 < limit and slot.fits(stream.n_words(e0, e1 + 1), e1 + 1 - e0):
                e1 += 1
            if not slot.fits(stream.n_words(e0, e1), e1 - e0):
                raise RuntimeError(f"event {e0} does not fit an empty slot")
            for _ in range(e1 - e0):
                fifo.popleft()
            slot.launch(stream.slice(e0, e1), e0, e1)
            busy[si] = (e0, e1)
            batch_sizes.append(e1 - e0)
            progressed = True
        if not progressed:
            if not busy and nxt < n:
                # nothing in flight: wait for the next arrival
                wait = stream.arrival_s[nxt] - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif idle_sleep_s > 0:
                time.sleep(idle_sleep_s)
    wall = clock() - t0
    stats = ServeStats(latency_s=lat, batch_sizes=batch_sizes, n_combos=total_combos, wall_s=wall,
                       retries=sum(getattr(s, "retries", 0) for s in slots))
    return stats, results


def split_by_event(road_event: np.ndarray, arrays: dict, n_events: int) -> list:
    """Per-road result arrays of one batch -> list of per-event dicts (event ordinal in batch)."""
    bounds = np.searchsorted(road_event, np.arange(n_events + 1))
    return [{k: v[bounds[i]:bounds[i + 1]] for k, v in arrays.items()} for i in range(n_events)]


class GpuSlot:
    """Fused persistent pass on its own stream: pinned words -> H2D -> graph replay -> D2H.

    Results come back in two steps so that only what the batch produced crosses PCIe: the
    sizes and error word first (one 40-byte copy), then, once they are on the host, exactly
    n_roads entries of the per-road best tracks, their event ordinals and constant sets.  Every
    step is a single foreign call (prepared batch arguments, library copy and event helpers),
    so that the host loop's cost per batch stays small next to the arrival gaps.
    """

    BEST_KEYS = ("n_accept", "k", "p0", "p1", "p2", "chi2")

    def __init__(self, cfg, bank, word_cap: int, road_cap: int, combo_cap: int, tune=None,
                 graph: bool = True, keep_results: bool = False):
        import torch

        from . import _lib as L
        from . import pipeline as P

        self.torch, self.L = torch, L
        self.runner = P.BatchRunner(cfg, bank, word_cap, road_cap, combo_cap, kept_cap=0,
                                    tune=tune, graph=graph, with_c=False)
        self.stream = self.runner.stream
        self.word_cap, self.road_cap, self.combo_cap = word_cap, road_cap, combo_cap
        self.keep = keep_results
        self.h_words = torch.empty(word_cap, dtype=torch.int32, pin_memory=True)
        self.h_words_np = self.h_words.numpy().view(np.uint32)
        self.h_n = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.h_n_np = self.h_n.numpy()
        self.h_state = torch.empty(5, dtype=torch.int64, pin_memory=True)  # sizes[4], error
        self.h_state_np = self.h_state.numpy()
        self.h_best = {k: torch.empty(road_cap, dtype=v.dtype, pin_memory=True)
                       for k, v in self.runner.best.items()}
        self.h_event = torch.empty(road_cap, dtype=torch.int32, pin_memory=True)
        self.h_set = torch.empty(road_cap, dtype=torch.int32, pin_memory=True)
        # (device array, host array, element size) of the per-road results
        self._fetch = [(self.runner.best[k], self.h_best[k], self.h_best[k].element_size())
                       for k in self.BEST_KEYS]
        self._fetch += [(self.runner.roads["event"], self.h_event, 4),
                        (self.runner.roads["set"], self.h_set, 4)]
        self.sizes_ev = torch.cuda.Event()
        self.done_ev = torch.cuda.Event()
        for ev in (self.sizes_ev, self.done_ev):  # create the events
            ev.record(self.stream)
        torch.cuda.synchronize()
        self.retries = 0
        self.batch = None
        self.stage = 0  # 1: sizes in flight, 2: results in flight, 3: complete

    def fits(self, n_words: int, n_events: int) -> bool:
        # every road holds at least one word; combinations are checked on the device and a
        # batch that overflows is split and run again
        return n_words <= self.word_cap

    def _enqueue(self, words: np.ndarray):
        L, r, s = self.L, self.runner, self.stream
        n = len(words)
        self.h_words_np[:n] = words
        self.h_n_np[0] = n
        L.svt_copy_async(r.d_n, self.h_n, 8, L.SVT_COPY_H2D, s)
        L.svt_copy_async(r.words, self.h_words, 4 * n, L.SVT_COPY_H2D, s)
        r.run()
        L.svt_copy_async(self.h_state, r.d_state, 40, L.SVT_COPY_D2H, s)
        L.svt_event_record(self.sizes_ev, s)
        self.stage = 1

    def _error(self):
        L = self.L
        err = int(self.h_state_np[4]) & L.SVT_NO_ERROR
        return L.error_decode(err) if err != L.SVT_NO_ERROR else (0, -1)

    def poll(self) -> bool:
        L = self.L
        if self.stage == 1:
            if not L.svt_event_done(self.sizes_ev):
                return False
            nr = int(self.h_state_np[1])
            if self._error()[0] != 0 or not 0 <= nr <= self.road_cap:
                self.stage = 3
                return True
            for d, h, size in self._fetch:
                L.svt_copy_async(h, d, size * nr, L.SVT_COPY_D2H, self.stream)
            L.svt_event_record(self.done_ev, self.stream)
            self.stage = 2
            return False
        if self.stage == 2:
            if not L.svt_event_done(self.done_ev):
                return False
            self.stage = 3
        return self.stage == 3

    def _wait(self):
        self.sizes_ev.synchronize()
        while not self.poll():
            self.done_ev.synchronize()

    def launch(self, words: np.ndarray, e0: int, e1: int):
        self.batch = (words, e0, e1)
        self._enqueue(words)

    def collect(self):
        L = self.L
        words, e0, e1 = self.batch
        st, idx = self._error()
        sizes = [int(v) for v in self.h_state_np[:4]]
        if st == L.SVT_ERR_CAPACITY and e1 - e0 > 1:
            # more roads or combinations than this slot holds: split at an event boundary
            # and run the halves synchronously (rare when slots are sized for the stream)
            self.retries += 1
            return self._split_run(words, e0, e1)
        if st != 0:
            raise RuntimeError(f"batch {e0}-{e1}: {L.status_name(st)} at {idx}")
        per_event = None
        if self.keep:
            nr = sizes[1]
            arrays = {k: self.h_best[k][:nr].numpy().copy() for k in self.BEST_KEYS}
            arrays["set"] = self.h_set[:nr].numpy().copy()
            per_event = split_by_event(self.h_event[:nr].numpy(), arrays, e1 - e0)
        return sizes[2], per_event

    def _split_run(self, words, e0, e1):
        # the words of events e0..e1 are contiguous; event boundaries are event-tag changes
        et = (words >> 24).astype(np.int64)
        starts = np.concatenate([[0], np.nonzero(et[1:] != et[:-1])[0] + 1, [len(words)]])
        mid = (e1 - e0) // 2
        total, res = 0, []
        for a, b in [(0, mid), (mid, e1 - e0)]:
            part = words[starts[a]:starts[b]]
            self.batch = (part, e0 + a, e0 + b)
            self._enqueue(part)
            self._wait()
            nc, pe = self.collect()
            total += nc
            res += pe if pe is not None else []
        return total, (res if self.keep else None)


class PlainSlot:
    """One-launch-per-stage path: the host waits at each stage to size the next one."""

    def __init__(self, cfg, bank):
        from . import pipeline as P
        import torch

        self.torch = torch
        self.runner = P.PlainRunner(cfg, bank, with_c=False, want_kept=False)
        self.h_words = torch.empty(1 << 20, dtype=torch.int32, pin_memory=True)
        self.out = None
        self.retries = 0

    def fits(self, n_words: int, n_events: int) -> bool:
        return True

    def launch(self, words: np.ndarray, e0: int, e1: int):
        torch = self.torch
        n = len(words)
        if self.h_words.numel() < n:
            self.h_words = torch.empty(2 * n, dtype=torch.int32, pin_memory=True)
        self.h_words.numpy().view(np.uint32)[:n] = words
        d = self.h_words[:n].to("cuda", non_blocking=True)
        self.runner.run(d, n)
        best = {k: v[:self.runner.n_roads].cpu() for k, v in self.runner.best.items()}
        self.out = (self.runner.n_combos, best)

    def poll(self) -> bool:
        return True

    def collect(self):
        return self.out[0], None

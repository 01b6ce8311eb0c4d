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
import gc
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
    max_loop_gap_s: float = 0.0   # longest time between two passes of the host loop
    max_service_s: float = 0.0    # longest launch-to-done time of one batch
    max_service_batch: int = 0    # events in that batch
    # per event, from its batch: seconds waiting in the FIFO (arrival to the launch call), in
    # the host's launch call, on the device (first to last operation of the batch on its
    # stream, transfers included; NaN when the slot does not time it) and from the end of the
    # launch call to the host seeing the results, less the device time (launch latency plus
    # how long the finished batch waited for the loop to poll it)
    queue_s: Optional[np.ndarray] = None
    enqueue_s: Optional[np.ndarray] = None
    device_s: Optional[np.ndarray] = None
    visible_s: Optional[np.ndarray] = None

    def percentile_us(self, q) -> float:
        return float(np.percentile(self.latency_s, q) * 1e6)

    def breakdown(self, warmup_events: int = 0) -> Optional[dict]:
        """p50 / p99 / mean in microseconds of each latency component (see the fields)."""
        if self.queue_s is None:
            return None
        out = {}
        for name in ("queue", "enqueue", "device", "visible"):
            v = getattr(self, name + "_s")[warmup_events:]
            v = v[np.isfinite(v)]
            if v.size:
                out[name] = dict(p50_us=round(float(np.percentile(v, 50)) * 1e6, 2),
                                 p99_us=round(float(np.percentile(v, 99)) * 1e6, 2),
                                 mean_us=round(float(v.mean()) * 1e6, 2))
        return out

    def summary(self, warmup_events: int = 0) -> dict:
        lat = self.latency_s[warmup_events:]
        return dict(events=int(len(lat)), p50_us=round(float(np.percentile(lat, 50)) * 1e6, 2),
                    p99_us=round(float(np.percentile(lat, 99)) * 1e6, 2),
                    max_us=round(float(lat.max()) * 1e6, 2),
                    mean_us=round(float(lat.mean()) * 1e6, 2),
                    batches=len(self.batch_sizes),
                    mean_batch=round(float(np.mean(self.batch_sizes)), 2),
                    combos_per_s=self.n_combos / self.wall_s if self.wall_s > 0 else 0.0,
                    retries=self.retries,
                    max_loop_gap_us=round(self.max_loop_gap_s * 1e6, 2),
                    max_service_us=round(self.max_service_s * 1e6, 2),
                    max_service_batch=self.max_service_batch,
                    breakdown=self.breakdown(warmup_events))


def serve(stream: EventStream, slots: Sequence, max_events: int = 256,
          clock: Callable[[], float] = time.perf_counter, keep_results: bool = False,
          idle_sleep_s: float = 0.0):
    """Run the whole stream through the slots; returns (ServeStats, per-event results or None).

    A slot provides: ``fits(n_words, n_events) -> bool``, ``launch(words, e0, e1)``,
    ``poll() -> bool`` (finished), ``collect() -> (n_combos, per_event_results or None)``.
    """
    # A full garbage collection of a large process heap takes milliseconds and would land in
    # the latency of whatever batch it interrupts: collect once now and keep the collector off
    # for the duration of the stream.
    gc_on = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        return _serve(stream, slots, max_events, clock, keep_results, idle_sleep_s)
    finally:
        if gc_on:
            gc.enable()


def _serve(stream, slots, max_events, clock, keep_results, idle_sleep_s):
    n = stream.n_events
    lat = np.full(n, np.nan)
    q_s, enq_s, dev_s, vis_s = (np.full(n, np.nan) for _ in range(4))
    results = [None] * n if keep_results else None
    fifo = deque()
    nxt = 0
    busy = {}  # slot index -> (e0, e1, launch-call start, launch-call end)
    batch_sizes = []
    total_combos = 0
    done = 0
    max_gap = max_service = 0.0
    max_service_batch = 0
    t0 = clock()
    prev = 0.0
    while done < n:
        now = clock() - t0
        max_gap = max(max_gap, now - prev)
        prev = now
        while nxt < n and stream.arrival_s[nxt] <= now:
            fifo.append(nxt)
            nxt += 1
        progressed = False
        for si in list(busy):
            if slots[si].poll():
                e0, e1, t_launch, t_enq = busy.pop(si)
                t_done = clock() - t0
                if t_done - t_launch > max_service:
                    max_service, max_service_batch = t_done - t_launch, e1 - e0
                nc, per_event = slots[si].collect()
                total_combos += nc
                lat[e0:e1] = t_done - stream.arrival_s[e0:e1]
                q_s[e0:e1] = t_launch - stream.arrival_s[e0:e1]
                enq_s[e0:e1] = t_enq - t_launch
                dev = getattr(slots[si], "last_device_s", float("nan"))
                dev_s[e0:e1] = dev
                vis_s[e0:e1] = t_done - t_enq - (dev if np.isfinite(dev) else 0.0)
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
            t_launch = clock() - t0
            slot.launch(stream.slice(e0, e1), e0, e1)
            busy[si] = (e0, e1, t_launch, clock() - t0)
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
                       retries=sum(getattr(s, "retries", 0) for s in slots),
                       max_loop_gap_s=max_gap, max_service_s=max_service,
                       max_service_batch=max_service_batch, queue_s=q_s, enqueue_s=enq_s,
                       device_s=dev_s, visible_s=vis_s)
    return stats, results


def launch_capacity(n_words: int, word_cap: int, min_words: int) -> int:
    """The smallest power-of-two word capacity, at least min_words, that holds n_words, capped at
    word_cap: the capacity a batch is launched for when launches are sized to the batch."""
    c = min_words
    while c < n_words:
        c *= 2
    return min(c, word_cap)


def launch_capacities(word_cap: int, min_words: int) -> list:
    """Every value launch_capacity can return for batches up to word_cap words."""
    caps = {word_cap}
    c = min_words
    while c < word_cap:
        caps.add(c)
        c *= 2
    return sorted(caps)


def split_by_event(road_event: np.ndarray, arrays: dict, n_events: int) -> list:
    """Per-road result arrays of one batch -> list of per-event dicts (event ordinal in batch)."""
    bounds = np.searchsorted(road_event, np.arange(n_events + 1))
    return [{k: v[bounds[i]:bounds[i + 1]] for k, v in arrays.items()} for i in range(n_events)]


class GpuSlot:
    """Fused persistent pass on its own stream, one batch at a time.

    ``io="mapped"`` (default): nothing is copied by a runtime call.  The slot writes the word
    count and the words into one page-locked buffer that the kernels read in place over the
    bus, and one small gather kernel (svt_gather_results) writes the sizes, the error word and
    the batch's n_roads per-road results straight into a second page-locked buffer.  A batch
    is then one graph replay, one gather launch and one event: the runtime's copy calls, which
    now and then spend milliseconds of host time inside the runtime, are off the loop.

    ``io="copy"``: pinned words -> H2D -> graph replay -> D2H in two steps (the sizes and error
    word first, then exactly n_roads entries of each per-road array), kept for comparison.

    ``size_to_batch`` (default): each batch is launched for the smallest power-of-two word
    capacity (at least ``MIN_LAUNCH_WORDS``) that holds it, not for the slot's whole capacity,
    so the persistent grids and look-back state match the batch; with graphs that is one
    cached graph per capacity (``warm`` captures them all).  A zero schedule in ``tune`` is
    then chosen per launch capacity, which puts small batches on the one-pass kernel.
    """

    MIN_LAUNCH_WORDS = 4096

    BEST_KEYS = ("n_accept", "k", "p0", "p1", "p2", "chi2")
    IN_HEADER = 256  # bytes before the words in the mapped input buffer (word count first)

    def __init__(self, cfg, bank, word_cap: int, road_cap: int, combo_cap: int, tune=None,
                 graph: bool = True, keep_results: bool = False, io: str = "mapped",
                 timing: bool = False, size_to_batch: bool = True):
        import torch

        from . import _lib as L
        from . import pipeline as P

        if io not in ("mapped", "copy"):
            raise ValueError(f"unknown io mode {io}")
        self.torch, self.L, self.io = torch, L, io
        self.word_cap, self.road_cap, self.combo_cap = word_cap, road_cap, combo_cap
        self.keep = keep_results
        self.size_to_batch = size_to_batch
        if io == "mapped":
            self.h_in = torch.empty(self.IN_HEADER + 4 * word_cap, dtype=torch.uint8,
                                    pin_memory=True)
            h_in = self.h_in.numpy()
            self.h_n_np = h_in[:8].view(np.int64)
            self.h_words_np = h_in[self.IN_HEADER:].view(np.uint32)
            d_in = L.svt_mapped_pointer(self.h_in)
            self.d_words = d_in + self.IN_HEADER
            self.runner = P.BatchRunner(cfg, bank, word_cap, road_cap, combo_cap, kept_cap=0,
                                        tune=tune, graph=graph, with_c=False, n_words_ptr=d_in)
            self.h_out = torch.empty(L.GATHER_HEADER_BYTES + L.GATHER_BYTES_PER_ROAD * road_cap,
                                     dtype=torch.uint8, pin_memory=True)
            self.h_out_np = self.h_out.numpy()
            r = self.runner
            self._gather = L.PreparedGather(r.roads, r.best, road_cap, d_in, r.d_n[1:2],
                                            r.d_n[2:3], None, r.d_err,
                                            L.svt_mapped_pointer(self.h_out), road_cap)
        else:
            self.runner = P.BatchRunner(cfg, bank, word_cap, road_cap, combo_cap, kept_cap=0,
                                        tune=tune, graph=graph, with_c=False)
            self.h_words = torch.empty(word_cap, dtype=torch.int32, pin_memory=True)
            self.h_words_np = self.h_words.numpy().view(np.uint32)
            self.h_n = torch.empty(1, dtype=torch.int64, pin_memory=True)
            self.h_n_np = self.h_n.numpy()
            self.h_state = torch.empty(5, dtype=torch.int64, pin_memory=True)  # sizes, error
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
        self.stream = self.runner.stream
        # timing: one more event before the batch's first operation, and a timed done event;
        # last_device_s = the batch's time on the device (NaN without timing)
        self.timing = timing
        self.last_device_s = float("nan")
        self.sizes_ev = torch.cuda.Event()
        self.done_ev = torch.cuda.Event(enable_timing=timing)
        self.start_ev = torch.cuda.Event(enable_timing=True) if timing else None
        for ev in (self.sizes_ev, self.done_ev) + ((self.start_ev,) if timing else ()):
            ev.record(self.stream)
        torch.cuda.synchronize()
        self.retries = 0
        self.batch = None
        self.stage = 0  # 1: sizes in flight, 2: results in flight, 3: complete
        self._head = None
        self._roads = None

    def fits(self, n_words: int, n_events: int) -> bool:
        # every road holds at least one word; combinations are checked on the device and a
        # batch that overflows is split and run again
        return n_words <= self.word_cap

    def launch_cap(self, n_words: int) -> int:
        """Word capacity a batch of n_words is launched for."""
        if not self.size_to_batch:
            return self.word_cap
        return launch_capacity(n_words, self.word_cap, self.MIN_LAUNCH_WORDS)

    def launch_caps(self):
        """Every capacity launch_cap can return."""
        if not self.size_to_batch:
            return [self.word_cap]
        return launch_capacities(self.word_cap, self.MIN_LAUNCH_WORDS)

    def warm(self, words: np.ndarray):
        """Run a small batch once per launch capacity (captures every graph before timing)."""
        for cap in self.launch_caps():
            self.batch = (words, 0, 1)
            self._enqueue(words, cap)
            self._wait()
            self.collect()

    def _enqueue(self, words: np.ndarray, cap: Optional[int] = None):
        L, r, s = self.L, self.runner, self.stream
        n = len(words)
        cap = self.launch_cap(n) if cap is None else cap
        self.h_words_np[:n] = words
        self.h_n_np[0] = n
        if self.timing:
            L.svt_event_record(self.start_ev, s)
        if self.io == "mapped":
            r.run(words=self.d_words, word_cap=cap)
            self._gather(s)
            L.svt_event_record(self.done_ev, s)
            self.stage = 2
            return
        L.svt_copy_async(r.d_n, self.h_n, 8, L.SVT_COPY_H2D, s)
        L.svt_copy_async(r.words, self.h_words, 4 * n, L.SVT_COPY_H2D, s)
        r.run(word_cap=cap)
        L.svt_copy_async(self.h_state, r.d_state, 40, L.SVT_COPY_D2H, s)
        L.svt_event_record(self.sizes_ev, s)
        self.stage = 1

    def _sizes_err(self):
        """[n_words, n_roads, n_combos, n_kept] and the raw error word of the finished batch."""
        if self.io == "mapped":
            h = self._head
            return [h["n_words"], h["n_roads"], h["n_combos"], h["n_kept"]], h["err"]
        v = self.h_state_np
        return [int(x) for x in v[:4]], int(v[4]) & self.L.SVT_NO_ERROR

    def _error(self):
        L = self.L
        err = self._sizes_err()[1]
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
            if self.io == "mapped":
                self._head, self._roads = L.gathered(self.h_out_np)
            self.stage = 3
        return self.stage == 3

    def _wait(self):
        self.sizes_ev.synchronize()
        while not self.poll():
            self.done_ev.synchronize()

    def launch(self, words: np.ndarray, e0: int, e1: int):
        self.batch = (words, e0, e1)
        self._enqueue(words)

    def _road_arrays(self, nr):
        """Per-road results of the finished batch (copies: the host buffers are reused)."""
        if self.io == "mapped":
            return {k: v.copy() for k, v in self._roads.items()}
        arrays = {k: self.h_best[k][:nr].numpy().copy() for k in self.BEST_KEYS}
        arrays["event"] = self.h_event[:nr].numpy().copy()
        arrays["set"] = self.h_set[:nr].numpy().copy()
        return arrays

    def collect(self):
        L = self.L
        words, e0, e1 = self.batch
        if self.timing:
            self.last_device_s = self.start_ev.elapsed_time(self.done_ev) * 1e-3
        st, idx = self._error()
        sizes, _ = self._sizes_err()
        if st == L.SVT_ERR_CAPACITY and e1 - e0 > 1:
            # more roads or combinations than this slot holds: split at an event boundary
            # and run the halves synchronously (rare when slots are sized for the stream)
            self.retries += 1
            return self._split_run(words, e0, e1)
        if st != 0:
            raise RuntimeError(f"batch {e0}-{e1}: {L.status_name(st)} at {idx}")
        per_event = None
        if self.keep:
            arrays = self._road_arrays(sizes[1])
            road_event = arrays.pop("event")
            per_event = split_by_event(road_event, arrays, e1 - e0)
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

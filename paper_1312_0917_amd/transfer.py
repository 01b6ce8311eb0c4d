"""Transfer strategies for one packet of events (the one-host analogue of section IV-C).

The paper measures the loop latency of a packet that travels into the GPU, through the fit and
back, with several ways of moving the data (two host buffers; one buffer shared with the
network card; CUDA-aware MPI; peer-to-peer from the card), and finds the transfers to be 20-25 %
of the total.  On one host the question left is how the packed hit words reach HBM:

  ``pageable``  words in ordinary host memory: the runtime stages them through its own
                page-locked buffer (two host-side copies, like the scheme with two buffers);
  ``pinned``    words already in page-locked memory: one DMA straight into HBM (one shared
                host buffer);
  ``mapped``    no copy at all: the pre-pass kernel reads the page-locked words in place over
                the bus (zero-copy input).

Results come back the same way for all three: the sizes, the error word and the per-road best
tracks of the packet, one DMA each into page-locked buffers.  Each measured point is one
packet's end-to-end latency on the host clock, split with HIP events into input, compute and
output, for packet sizes from 600 kB (the paper's smallest packet) up.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from . import pipeline as P

MODES = ("pageable", "pinned", "mapped")
PACKET_BYTES = (600_000, 1_200_000, 2_400_000, 4_800_000, 9_600_000, 19_200_000, 38_400_000,
                64_000_000)
BEST_KEYS = ("n_accept", "k", "p0", "p1", "p2", "chi2")


def packet_events(event_word_begin: np.ndarray, nbytes: int) -> int:
    """Smallest number of leading events whose words fill at least ``nbytes`` (or all)."""
    need = (nbytes + 3) // 4
    e = int(np.searchsorted(event_word_begin, need, side="left"))
    return min(max(e, 1), len(event_word_begin) - 1)


@dataclasses.dataclass
class TransferPoint:
    mode: str
    packet_bytes: int
    events: int
    roads: int
    combos: int
    total_us: float      # mean end-to-end latency on the host clock
    p50_us: float
    input_us: float      # HIP events: copy of the words (0 for mapped)
    compute_us: float    # the batched pass (for mapped: includes reading the words over the bus)
    output_us: float     # copies of sizes, error word and per-road results
    transfer_share: float  # share of the GPU-side time not spent on the pass itself: 1 - (pass
                           # with the words already in HBM) / (input + compute + output); for
                           # mapped input the bus reads are inside "compute", and count here

    def as_dict(self):
        return {k: (round(v, 2) if isinstance(v, float) else v)
                for k, v in dataclasses.asdict(self).items()}


def study(words: np.ndarray, event_word_begin: np.ndarray, road_event: np.ndarray,
          road_combos: np.ndarray, cfg: L.svt_config, dbank: torch.Tensor,
          tune: Optional[L.svt_tune] = None, sizes: Sequence[int] = PACKET_BYTES,
          modes: Sequence[str] = MODES, reps: int = 20, warmup: int = 3,
          log: Optional[Callable[[str], None]] = None):
    """Measure every (mode, packet size).  ``words`` is the packed stream of a run of events;
    ``road_combos`` the combinations of each road (to size the device buffers)."""
    for m in modes:
        if m not in MODES:
            raise ValueError(f"unknown transfer mode {m}")
    ends = [packet_events(event_word_begin, s) for s in sizes]
    e_max = max(ends)
    n_max = int(event_word_begin[e_max])
    r_max = int(np.searchsorted(road_event, e_max))
    c_max = int(road_combos[:r_max].sum())
    runner = P.BatchRunner(cfg, dbank, n_max, r_max, c_max, kept_cap=0, tune=tune, graph=True,
                           with_c=False)
    pinned = torch.empty(n_max, dtype=torch.int32, pin_memory=True)
    pinned.numpy().view(np.uint32)[:] = words[:n_max]
    pageable = np.ascontiguousarray(words[:n_max]).view(np.int32).copy()
    mapped = L.svt_mapped_pointer(pinned)
    h_sizes = torch.empty(4, dtype=torch.int64, pin_memory=True)
    h_err = torch.empty(1, dtype=torch.int64, pin_memory=True)
    h_best = {k: torch.empty(r_max, dtype=v.dtype, pin_memory=True) for k, v in runner.best.items()}
    stream = runner.stream
    points = []
    for size, e1 in zip(sizes, ends):
        n = int(event_word_begin[e1])
        nr = int(np.searchsorted(road_event, e1))
        nc = int(road_combos[:nr].sum())
        size_points = []
        for mode in modes:
            tot, tin, tcomp, tout = [], [], [], []
            for rep in range(warmup + reps):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                with torch.cuda.stream(stream):
                    ev[0].record(stream)
                    if mode == "pageable":
                        runner.words[:n].copy_(torch.from_numpy(pageable[:n]), non_blocking=True)
                    elif mode == "pinned":
                        runner.words[:n].copy_(pinned[:n], non_blocking=True)
                    runner.d_n[0].fill_(n)
                    ev[1].record(stream)
                runner.run(words=mapped if mode == "mapped" else None)
                with torch.cuda.stream(stream):
                    ev[2].record(stream)
                    h_sizes.copy_(runner.d_n, non_blocking=True)
                    h_err.copy_(runner.d_err, non_blocking=True)
                    for k in BEST_KEYS:
                        h_best[k][:nr].copy_(runner.best[k][:nr], non_blocking=True)
                    ev[3].record(stream)
                ev[3].synchronize()
                t1 = time.perf_counter()
                if rep == 0:
                    err = int(h_err[0]) & L.SVT_NO_ERROR
                    if err != L.SVT_NO_ERROR or int(h_sizes[1]) != nr or int(h_sizes[2]) != nc:
                        raise RuntimeError(f"{mode} {size} B: sizes {h_sizes.tolist()} vs "
                                           f"{nr} roads / {nc} combinations, error {err:#x}")
                if rep >= warmup:
                    tot.append((t1 - t0) * 1e6)
                    tin.append(ev[0].elapsed_time(ev[1]) * 1e3)
                    tcomp.append(ev[1].elapsed_time(ev[2]) * 1e3)
                    tout.append(ev[2].elapsed_time(ev[3]) * 1e3)
            i, c, o = float(np.mean(tin)), float(np.mean(tcomp)), float(np.mean(tout))
            size_points.append(TransferPoint(mode=mode, packet_bytes=4 * n, events=e1, roads=nr,
                                             combos=nc, total_us=float(np.mean(tot)),
                                             p50_us=float(np.median(tot)), input_us=i,
                                             compute_us=c, output_us=o, transfer_share=0.0))
        # the pass itself: the fastest compute among the modes that copy the words into HBM
        resident = [p.compute_us for p in size_points if p.mode != "mapped"]
        base = min(resident) if resident else min(p.compute_us for p in size_points)
        for pt in size_points:
            gpu = pt.input_us + pt.compute_us + pt.output_us
            pt.transfer_share = max(0.0, 1.0 - base / max(gpu, 1e-9))
            points.append(pt)
            if log:
                log(f"transfer {pt.mode:8s} {pt.packet_bytes / 1e6:7.2f} MB: total "
                    f"{pt.total_us:8.1f} us, in {pt.input_us:7.1f} compute {pt.compute_us:7.1f} "
                    f"out {pt.output_us:6.1f} (transfer share {pt.transfer_share:.2f})")
    L.svt_release_graphs()
    return points

#!/usr/bin/env python3
"""Throughput and latency of the SVT track fitter on one MI355X.

Default workload: 3000 events x 64 roads, 1-3 hits per layer (2048 combinations per event on
average), the shape of the paper's benchmark sample (section IV).  One step = one pass of the
whole path (unpack, combine, fit, select) over that batch with the words already in HBM.

Prints one JSON line: the batched path's fitted combinations/s (persistent fused kernel behind
a replayed HIP graph), the plain one-launch-per-stage path beside it, the roofline of the fused
kernel (HIP events on its own stream), and the CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# integer VALU lane-operations per second: 256 CUs x 64 lanes per clock x 2.4 GHz
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic integer operations of one fit as the method states it: 6 x 5 multiply-adds,
# 6 offset adds, 6 shifts, 3 squares, 2 adds, 1 compare
INT_OPS_PER_COMBO = 30 + 6 + 6 + 3 + 2 + 1
METRIC = "fitted combinations/s and p50/p99 event latency (µs), batched vs plain"


def int_ops(n_combos, kernel_ms, tune):
    """The dominant kernel's algorithmic integer operations per second against the VALU peak
    (a second view beside the HBM roofline: the fit's arithmetic, not its bytes)."""
    achieved = INT_OPS_PER_COMBO * n_combos / (kernel_ms * 1e-3) / 1e12
    return dict(bound="alu", achieved=round(achieved, 3), peak=round(INT_PEAK_TOPS, 1),
                unit="Tops/s", frac=round(achieved / INT_PEAK_TOPS, 4),
                kernel=kernel_name(tune), ops_per_combination=INT_OPS_PER_COMBO)


PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1312_0917_amd", "csrc")
# sources each timed kernel is compiled from: recorded HBM counters are valid while these match
KERNEL_SOURCES = {
    "k_fused": ["svt_fused.hip", "svt_fit.h", "svt_common.h"],
    "k_onepass": ["svt_onepass.hip", "svt_fit.h", "svt_lookback.h", "svt_common.h"],
    "k_fit_events": ["svt_events.hip", "svt_common.h"],
}


def kernel_source_digest(kernel):
    """SHA-1 of the kernel's source files with comments and blank lines removed (a comment
    edit does not change the kernel the counters were taken on)."""
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kernel]:
        path = os.path.join(CSRC, f)
        if os.path.exists(path):
            text = open(path).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
            h.update(code.encode())
    return h.hexdigest()[:16]


def recorded_traffic(config, n_events, tune):
    """HBM bytes per launch of the timed kernel from the committed counter summary for this
    workload (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what the counter
    reads for a plain copy of known size).  None when there is no summary for the kernel and
    workload, or the kernel's sources changed since the counters were taken."""
    kernel = kernel_name(tune)
    path = os.path.join(PROFILES, f"{kernel}_{config}_hbm_counters.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    kv = dict(re.findall(r"^([a-z_0-9]+): (\S+)\s*$", open(path).read(), flags=re.M))
    try:
        if kv["kernel_source_sha1"] != kernel_source_digest(kernel) or \
                int(kv["events"]) != n_events:
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return int(round((fetch + write) * 1024))


def copy_calibration(n_bytes=1 << 30, reps=3):
    """Plain device copy of a known size, run under the HBM byte counters to scale them."""
    import torch

    torch.cuda.set_device(0)
    x = torch.ones(n_bytes, dtype=torch.uint8, device="cuda")
    y = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=n_bytes, copies=reps)), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n_combos, n_words, n_roads):
    """Bytes the fused pass must move: per combination p0..p2 (12) + chi2 (8) + accept (1);
    per hit word 4 read; per road the best track written (n_accept, k, p0..p2, chi2: 28)."""
    return 21 * n_combos + 4 * n_words + 28 * n_roads


def fused_kernel_ms(runner, steps, warmup):
    """Average duration of the fused kernel alone: HIP events recorded on the runner's stream
    right before and after its launch (direct launches, same launch configuration)."""
    import numpy as np
    import torch
    from paper_1312_0917_amd import _lib as L

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(runner.stream)
    ev1.record(runner.stream)
    torch.cuda.synchronize()
    L.svt_set_fused_timing_events(ev0, ev1)
    graph = runner.graph
    runner.graph = False
    kms = []
    try:
        for i in range(warmup + steps):
            runner.run()
            ev1.synchronize()
            if i >= warmup:
                kms.append(ev0.elapsed_time(ev1))
    finally:
        L.svt_set_fused_timing_events(None, None)
        runner.graph = graph
    return float(np.mean(kms))


def measure_large(ls, passes, tune, bank):
    """Max-scale run: whole batch resident in HBM, graph replays, kernel and pass rooflines."""
    import torch

    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth

    cut = synth.config_chi2_cut("c5")
    n_words, n_roads, n_combos = len(ls.words), ls.n_roads, ls.combos
    gcfg, dbank = L.make_config(chi2_cut=cut), P.device_bank(bank.f, bank.q)
    words = P.words_tensor(ls.words)
    shapes = None
    if tune is None:
        # a short pick among the pre-pass + fused shapes (whole passes, 3 each after one)
        shapes = {}
        for tile, occ in ((4096, 3), (8192, 3), (4096, 4), (8192, 4)):
            t = L.svt_tune_resolve(L.make_tune(tile, 64, 256, occ, L.SVT_SCHEDULE_TILES))
            r = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=t,
                              graph=True, with_c=False)
            r.load(words)
            r.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                r.run()
            torch.cuda.synchronize()
            shapes[f"{tile}x{occ}"] = round((time.perf_counter() - t0) / 3 * 1e3, 4)
            assert r.error()[0] == 0, r.error()
            L.svt_release_graphs()
            del r
        best = min(shapes, key=shapes.get)
        tile, occ = (int(x) for x in best.split("x"))
        tune = L.svt_tune_resolve(L.make_tune(tile, 64, 256, occ, L.SVT_SCHEDULE_TILES))
        log(f"c5 launch shapes (ms per pass): {shapes}")
    tune = L.svt_tune_for_batch(tune, n_words)
    runner = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=tune,
                           graph=True, with_c=False)
    runner.load(words)
    runner.run()
    torch.cuda.synchronize()
    sz = runner.sizes()
    assert sz["n_combos"] == n_combos and runner.error()[0] == 0, (sz, runner.error())
    log(f"c5: {passes} timed passes over {n_combos} combinations")
    t0 = time.perf_counter()
    for _ in range(passes):
        runner.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    k_ms = fused_kernel_ms(runner, passes, 1)
    L.svt_release_graphs()
    out = dict(workload=f"c5: {ls.n_events} events, {n_roads} roads, {n_words} hit words, "
                        f"{n_combos} combinations",
               value=n_combos / dt, unit="fitted combinations/s", ms_per_pass=round(dt * 1e3, 4),
               passes=passes, tune=tune_dict(tune), ms_per_pass_by_shape=shapes,
               roofline=roofline_of(tune, n_combos, n_words, n_roads, k_ms, dt * 1e3,
                                    recorded_traffic("c5", ls.n_events, tune)),
               int_ops=int_ops(n_combos, k_ms, tune))
    del runner
    torch.cuda.empty_cache()
    return out


def tune_dict(t):
    return dict(tile_combos=t.tile_combos, chunk_roads=t.chunk_roads, wg_size=t.wg_size,
                wgs_per_cu=t.wgs_per_cu, schedule=t.schedule)


def measure_uneven(sample, bank, log_fn):
    """Uneven batch in one persistent launch (8192 events, geometric roads/event, heavy-tailed
    hits per layer): the autotuner times every launch shape and keeps the fastest."""
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth
    from paper_1312_0917_amd import tune as T

    cut = synth.config_chi2_cut("c3")
    nr, nc = sample.n_roads, sample.expected_combos()
    words = P.words_tensor(sample.words)
    res = T.autotune(words, P.device_bank(bank.f, bank.q), L.make_config(chi2_cut=cut), nr, nc,
                     cache_path=None, use_cache=False, log=log_fn)
    default = [row for row in res.table
               if row[:5] == T.tune_tuple(L.svt_tune_for_batch(None, len(sample.words)))]
    by_sched = {}
    for row in res.table:
        by_sched[row[4]] = min(by_sched.get(row[4], 1e30), row[5])
    return dict(workload=f"c3: {sample.n_events} events, {nr} roads, {len(sample.words)} hit "
                         f"words, {nc} combinations",
                best_tune=dict(zip(("tile_combos", "chunk_roads", "wg_size", "wgs_per_cu",
                                    "schedule"), T.tune_tuple(res.tune))),
                ms_per_pass_best=round(res.ms_per_pass, 5),
                ms_per_pass_default=default[0][5] if default else None,
                value=nc / (res.ms_per_pass * 1e-3), unit="fitted combinations/s",
                candidates=len(res.table), statistic=res.statistic,
                all_outputs_identical=True,
                best_ms_per_pass_by_schedule={str(k): v for k, v in sorted(by_sched.items())})


def measure_serving(sample, bank, warmup_events, rate_hz, n_slots, max_events, tune):
    """Poisson stream of events through the continuous-batching loop, fused path and plain path
    fed the same schedule; latency from arrival to results on the host (H2D and D2H included)."""
    import numpy as np
    import torch

    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import serve, synth

    n_events = sample.n_events
    arrivals = synth.poisson_arrivals(n_events, rate_hz, seed=3)
    st = serve.EventStream(sample.words, sample.event_word_begin, arrivals)
    mean_w = len(sample.words) / n_events
    mean_c = sample.expected_combos() / n_events
    word_cap = int(max_events * mean_w * 1.6)
    combo_cap = int(max_events * mean_c * 1.6)
    cfg = L.make_config(chi2_cut=synth.config_chi2_cut("c4"))
    dbank = P.device_bank(bank.f, bank.q)
    warm = serve.EventStream(sample.words, sample.event_word_begin, np.zeros(n_events))
    out = {}
    # (io, timing, graph, launch sized to the batch)
    runs = {"mapped": ("mapped", False, True, True), "mapped_timed": ("mapped", True, True, True),
            "mapped_direct": ("mapped", False, False, True),
            "mapped_slot_grid": ("mapped", False, True, False),
            "copy": ("copy", False, True, True)}
    for name, (io, timing, graph, sized) in runs.items():
        slots = [serve.GpuSlot(cfg, dbank, word_cap, word_cap // 5 + 1, combo_cap, tune=tune,
                               io=io, timing=timing, graph=graph, size_to_batch=sized)
                 for _ in range(n_slots)]
        # capture every slot's graphs before the clock starts
        for sl in slots:
            sl.warm(warm.slice(0, 1))
        stats, _ = serve.serve(st, slots, max_events=max_events)
        out[name] = stats.summary(warmup_events)
        caps = slots[0].launch_caps()
        out[name]["launch"] = dict(
            graph=graph, word_caps=[caps[0], caps[-1]],
            schedule_smallest=L.svt_tune_for_batch(tune, caps[0]).schedule,
            schedule_largest=L.svt_tune_for_batch(tune, caps[-1]).schedule)
        L.svt_release_graphs()
        del slots
        torch.cuda.empty_cache()
    pstats, _ = serve.serve(st, [serve.PlainSlot(cfg, dbank)], max_events=max_events)
    plain = pstats.summary(warmup_events)
    return dict(workload=f"c4: {n_events} events ({warmup_events} warm-up) arriving as a "
                         f"Poisson stream at {rate_hz / 1e3:.0f} kHz, {mean_w:.0f} words and "
                         f"{mean_c:.0f} combinations per event on average",
                slots=n_slots, max_events_per_batch=max_events,
                slot_word_cap=word_cap,
                batched_io="words read and results written in place in page-locked host "
                           "memory (no copy calls); batched_copy: H2D and two-step D2H copies",
                batched=out["mapped"],
                launch_shapes="batched: graphs for power-of-two word capacities from 4096 up, "
                              "each batch launched for the smallest that holds it (small "
                              "capacities run the one-pass kernel); batched_direct: the same "
                              "without graphs; batched_slot_grid: every batch launched for the "
                              "slot's whole capacity",
                batched_direct=out["mapped_direct"], batched_slot_grid=out["mapped_slot_grid"],
                batched_breakdown=dict(
                    note="the same stream and slots with a timed HIP event before each batch "
                         "(its overhead included); per event: queue = arrival to launch call, "
                         "enqueue = launch call, device = first to last operation of the batch "
                         "on its stream, visible = end of the launch call to the host seeing "
                         "the results, less the device time", **out["mapped_timed"]),
                batched_copy=out["copy"], plain=plain)


def measure_transfer(sample, bank, tune, reps):
    """Packet latency with pageable, pinned and mapped input (serving-shaped events)."""
    import numpy as np
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth, transfer

    combos = np.prod(sample.road_nhits.astype(np.int64), axis=1)
    pts = transfer.study(sample.words, sample.event_word_begin, sample.road_event, combos,
                         L.make_config(chi2_cut=synth.config_chi2_cut("c4")),
                         P.device_bank(bank.f, bank.q), tune=tune, reps=reps, log=log)
    return dict(workload="c4-shaped events (16-256 roads, 1-4 hits per layer), packets of "
                         "600 kB to 64 MB; per point the mean of %d packets" % reps,
                points=[p.as_dict() for p in pts])


def measure_kept_only(gcfg, dbank, words, n_words, n_roads, n_combos, tune, steps, warmup,
                      graph):
    """The same batch in kept-only mode: accept flags, kept list and best tracks, no records."""
    import torch
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P

    kept_cap = n_combos // 16 + 4096
    runner = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=kept_cap, tune=tune,
                           graph=graph, with_c=False, kept_only=True)
    runner.load(words)
    for _ in range(warmup):
        runner.run()
    torch.cuda.synchronize()
    assert runner.error() == (0, -1), runner.error()
    n_kept = runner.sizes()["n_kept"]
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    k_ms = fused_kernel_ms(runner, steps, warmup)
    ops = INT_OPS_PER_COMBO * n_combos
    achieved = ops / (k_ms * 1e-3) / 1e12
    L.svt_release_graphs()
    del runner
    torch.cuda.empty_cache()
    return dict(value=n_combos / dt, unit="fitted combinations/s", ms_per_step=round(dt * 1e3, 5),
                kept=n_kept,
                roofline=dict(bound="alu", achieved=round(achieved, 3), peak=round(INT_PEAK_TOPS, 1),
                              unit="Tops/s", frac=round(achieved / INT_PEAK_TOPS, 4),
                              kernel="k_fused", kernel_ms=round(k_ms, 5),
                              ops_per_combination=INT_OPS_PER_COMBO))


def cpu_host():
    """Host CPU description for the baseline record: model, logical CPUs, and the CPUs this
    process may run on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return dict(model=model, nproc=os.cpu_count(), usable_cpus=usable)


def run_cpu_baseline(sample, bank, cfg, seconds, threads):
    """The oracle as it stands, built -O3 -march=native on this host: serially on one core
    (the paper's serial baseline), then with the batch cut into event ranges that run on
    `threads` cores at once (the paper's one-event-per-core many-core scheme; events are
    independent).  Host-only work: call before the GPU runtime starts (it runs a compiler)."""
    import tempfile

    import oracle

    flags = "-O3 -march=x86-64-v3"
    try:
        lib = oracle.build_native(os.path.join(tempfile.mkdtemp(prefix="svt_oracle_"),
                                               "libsvt_oracle_native.so"))
        oracle.use_library(lib)
        flags = "-O3 -march=native"
    except (OSError, subprocess.CalledProcessError) as e:  # no compiler: the portable build
        log(f"native oracle build failed ({e}); timing the portable build")
    host = cpu_host()
    sec1, reps1, nc = oracle.time_run(sample.words, bank.f, bank.q, cfg, min_seconds=seconds)
    secn, repsn, ncn = oracle.time_event_ranges(sample.words, sample.event_word_begin, bank.f,
                                                bank.q, cfg, threads=threads,
                                                min_seconds=seconds)
    assert ncn == nc
    return dict(value=nc / secn, unit="fitted combinations/s", cores=threads, kind="oracle",
                sample=f"whole batch ({nc} combinations, all outputs) cut into "
                       f"{4 * threads} event ranges run by {threads} threads at once, "
                       f"{repsn} runs in {secn * repsn:.1f} s",
                serial=dict(value=nc / sec1, cores=1, runs=reps1,
                            seconds=round(sec1 * reps1, 2)),
                all_cores_over_serial=round(sec1 / secn, 2),
                compiler_flags=flags, cpu_model=host["model"], nproc=host["nproc"],
                usable_cpus=host["usable_cpus"])


def kernel_name(tune):
    return {1: "k_fit_events", 2: "k_onepass", 3: "k_fused"}.get(tune.schedule, "?")


def kernel_bytes(tune, n_combos, n_words, n_roads):
    """Algorithmic bytes of the timed kernel alone.  The one-pass kernel is the whole pass
    (the words in, records and best tracks out).  The persistent kernel of the two-kernel
    pass reads what the pre-pass wrote -- 2 B of grouped coordinate per word and 28 B of road
    table per road (hit_begin, combo_begin, nhits, ncombo, set) -- and writes the records;
    the best tracks are written by the finalize launch after it."""
    if tune.schedule == 2:
        return algorithmic_bytes(n_combos, n_words, n_roads)
    return 21 * n_combos + 2 * n_words + 28 * n_roads


def roofline_of(tune, n_combos, n_words, n_roads, kernel_ms, pass_ms, traffic):
    kb = kernel_bytes(tune, n_combos, n_words, n_roads)
    alg = algorithmic_bytes(n_combos, n_words, n_roads)
    ach = kb / (kernel_ms * 1e-3) / 1e9
    pas = alg / (pass_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic,
                traffic_over_algorithmic=round(traffic / kb, 3) if traffic else None,
                kernel=kernel_name(tune), kernel_ms=round(kernel_ms, 5),
                kernel_algorithmic_bytes=kb,
                pass_level=dict(achieved=round(pas, 1), frac=round(pas / HBM_PEAK_GBS, 4),
                                ms=round(pass_ms, 5), algorithmic_bytes=alg,
                                bytes_per_combination=round(alg / n_combos, 3)))


def measure_small(sample, bank, cut, reps, ora_s):
    """The paper's low-count regime on the 100-event workload: the batched pass with words
    resident, the batched pass including the copy of the words in and the per-road results
    out, the plain path, each `reps` times (the paper's 100 repetitions), beside the oracle."""
    import numpy as np
    import torch

    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P

    gcfg = L.make_config(chi2_cut=cut)
    dbank = P.device_bank(bank.f, bank.q)
    nw, nr, nc = len(sample.words), sample.n_roads, sample.expected_combos()
    words = P.words_tensor(sample.words)
    runner = P.BatchRunner(gcfg, dbank, nw, nr, nc, kept_cap=0, graph=True, with_c=False)
    runner.load(words)
    from paper_1312_0917_amd import tune as T
    modes = T.pick_launch_mode(runner)
    for _ in range(5):
        runner.run()
    torch.cuda.synchronize()
    assert runner.error() == (0, -1) and runner.sizes()["n_combos"] == nc
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        runner.run()
        runner.stream.synchronize()
        t.append(time.perf_counter() - t0)
    resident = float(np.median(t))
    pinned = torch.empty(nw, dtype=torch.int32, pin_memory=True)
    pinned.numpy().view(np.uint32)[:] = sample.words
    h_best = {k: torch.empty(nr, dtype=v.dtype, pin_memory=True) for k, v in runner.best.items()}
    t = []
    for _ in range(reps + 5):
        t0 = time.perf_counter()
        with torch.cuda.stream(runner.stream):
            runner.words[:nw].copy_(pinned, non_blocking=True)
        runner.run()
        with torch.cuda.stream(runner.stream):
            for k in h_best:
                h_best[k].copy_(runner.best[k][:nr], non_blocking=True)
        runner.stream.synchronize()
        t.append(time.perf_counter() - t0)
    with_io = float(np.median(t[5:]))
    L.svt_release_graphs()
    small_graph = runner.graph
    del runner
    pr = P.PlainRunner(gcfg, dbank, with_c=False, want_kept=False)
    for _ in range(5):
        pr.run(words)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pr.run(words)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    plain = float(np.median(t))
    us = lambda x: round(x * 1e6, 2)
    return dict(workload=f"c1: {sample.n_events} events, {nr} roads, {nw} hit words, "
                         f"{nc} combinations",
                reps=reps, statistic="median",
                batched=dict(us_per_pass=us(resident), value=nc / resident,
                             launch="graph replay" if small_graph else "direct launches",
                             launch_modes_ms_per_pass=modes),
                batched_with_io=dict(us_per_pass=us(with_io), value=nc / with_io,
                                     io="words in from page-locked memory, the 6 per-road "
                                        "best-track arrays out"),
                plain=dict(us_per_pass=us(plain), value=nc / plain),
                oracle=dict(us_per_pass=us(ora_s), value=nc / ora_s, cores=1),
                unit="fitted combinations/s")


def slim(sample):
    """Only what the GPU runs need of a large sample: its words and sizes."""
    import types
    return types.SimpleNamespace(words=sample.words, n_roads=sample.n_roads,
                                 n_events=sample.n_events, combos=sample.expected_combos())


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--events", type=int, default=0, help="override the workload's event count")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle baseline (0: usable CPUs, at most 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the 100-event workload")
    ap.add_argument("--small-reps", type=int, default=100)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--occ", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=-1,
                    help="launch schedule (0 built-in default, 1 event per workgroup, 2 one "
                         "pass, 3 pre-pass + fused tiles); default: the built-in or autotuned one")
    ap.add_argument("--large-events", type=int, default=10000,
                    help="events of the max-scale run (10000 x 2048 roads); 0 skips it")
    ap.add_argument("--large-passes", type=int, default=5)
    ap.add_argument("--workers", type=int, default=16, help="threads drawing large samples")
    ap.add_argument("--no-graph", action="store_true", help="direct launches instead of replays")
    ap.add_argument("--no-uneven", action="store_true", help="skip the autotuned uneven batch")
    ap.add_argument("--serve-events", type=int, default=40000, help="0 skips the serving run")
    ap.add_argument("--serve-warmup", type=int, default=5000)
    ap.add_argument("--serve-rate", type=float, default=100e3)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--no-kept-only", action="store_true", help="skip the kept-only mode run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shape instead of the autotuned one")
    ap.add_argument("--transfer-reps", type=int, default=10,
                    help="packets per point of the transfer study; 0 skips it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB three times (scale for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the fitter shards by event range with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    # ---- host-side work first: every sample is drawn and the CPU baselines are timed before
    # the GPU runtime starts, so no compiler or worker runs beside a GPU-holding process -------
    import numpy as np

    import oracle
    from paper_1312_0917_amd import synth

    bank = synth.make_bank()
    n_ev = args.events or synth.CONFIGS[args.config]["n_events"]
    log(f"drawing {args.config} ({n_ev} events)")
    sample = synth.make_sample(args.config, bank=bank, n_events=n_ev, workers=args.workers)
    cut = synth.config_chi2_cut(args.config)
    cfg = oracle.make_config(chi2_cut=cut)
    small = synth.make_sample("c1", bank=bank) if not args.no_small else None
    uneven_s = synth.make_sample("c3", bank=bank, workers=args.workers) \
        if not args.no_uneven else None
    serve_s = synth.make_sample("c4", bank=bank, n_events=args.serve_events,
                                workers=args.workers) if args.serve_events > 0 else None
    transfer_s = synth.make_sample("c4", bank=bank, n_events=10000, workers=args.workers) \
        if args.transfer_reps > 0 else None
    large_s = None
    if args.large_events > 0:
        log(f"drawing c5 ({args.large_events} events)")
        large_s = slim(synth.make_sample("c5", bank=bank, n_events=args.large_events,
                                         workers=args.workers))
    cpu = None
    host = cpu_host()
    threads = args.cpu_threads or min(16, host["usable_cpus"])
    if not args.no_cpu:
        log(f"cpu oracle baseline (~{2 * args.cpu_seconds:.0f} s: 1 core, then {threads})")
        cpu = run_cpu_baseline(sample, bank, cfg, args.cpu_seconds, threads)
    small_ora = None
    if small is not None:
        sc = oracle.make_config(chi2_cut=synth.config_chi2_cut("c1"))
        oracle.run(small.words, bank.f, bank.q, sc)
        ts = []
        for _ in range(args.small_reps):
            t0 = time.perf_counter()
            oracle.run(small.words, bank.f, bank.q, sc)
            ts.append(time.perf_counter() - t0)
        small_ora = float(np.median(ts))

    # ---- GPU ----------------------------------------------------------------------------------
    import torch

    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    K, W = args.steps, args.warmup

    n_words, n_roads, n_events = len(sample.words), sample.n_roads, sample.n_events
    n_combos = sample.expected_combos()  # the generator's own record of the batch
    gcfg = L.make_config(chi2_cut=cut)
    dbank = P.device_bank(bank.f, bank.q)
    words = P.words_tensor(sample.words)
    explicit_tune = any((args.tile, args.chunk, args.wg, args.occ)) or args.schedule >= 0
    tune = L.svt_tune_resolve(L.make_tune(args.tile, args.chunk, args.wg, args.occ,
                                          max(args.schedule, 0)))
    default_tune = L.svt_tune_resolve(None)
    tuned = None
    if not explicit_tune and not args.no_autotune:
        # the autotuner picks the launch shape of this batch (every candidate must write the
        # same bytes); the timed steps below then use the winner
        from paper_1312_0917_amd import tune as T
        log("autotuning the batch")
        res = T.autotune(words, dbank, gcfg, n_roads, n_combos, cache_path=None,
                         use_cache=False)
        tune = res.tune
        tuned = dict(candidates=len(res.table), best_ms_per_pass=round(res.ms_per_pass, 5),
                     statistic=res.statistic)
    # the schedule the library runs for this batch (a zero schedule is chosen per capacity)
    tune = L.svt_tune_for_batch(tune, n_words)

    # ---- batched path: resident buffers; graph replays or direct launches, whichever is faster
    runner = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=tune,
                           graph=not args.no_graph, with_c=False)
    runner.load(words)
    launch_modes = None
    if not args.no_graph:
        from paper_1312_0917_amd import tune as T
        log("launch mode: graph replays against direct launches")
        launch_modes = T.pick_launch_mode(runner)
        launch_modes["statistic"] = "median of 30 samples of 5 passes each"
    log("batched warmup")
    for _ in range(W):
        runner.run()
    torch.cuda.synchronize()
    sz = runner.sizes()
    assert sz["n_combos"] == n_combos and runner.error()[0] == 0, (sz, runner.error())
    log(f"batched timed: {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        runner.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    batch_s = (t1 - t0) / K
    value = n_combos / batch_s
    runner_graph = runner.graph

    # ---- the dominant kernel alone: HIP events on the runner's stream around its launch ----
    log("kernel timing")
    k_ms = fused_kernel_ms(runner, K, W)
    traffic = recorded_traffic(args.config, n_events, tune)
    roofline = roofline_of(tune, n_combos, n_words, n_roads, k_ms, batch_s * 1e3, traffic)

    # ---- several batches in flight: more runners, each with its own stream and graph -------
    # (not the headline: `value` is one pass at a time.  With independent batches queued on
    # several streams, one batch's latency-bound pre-pass and kernel tails can overlap another's
    # fused kernel; this is the serving slots' situation at a high arrival rate.)
    in_flight = None
    if not args.no_kept_only:
        in_flight = {}
        for n_fl in (2, 3):
            log(f"{n_fl} batches in flight")
            extra = []
            for _ in range(n_fl - 1):
                r = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=tune,
                                  graph=runner_graph, with_c=False)
                r.load(words)
                extra.append(r)
            group = [runner] + extra
            for _ in range(W):
                for r in group:
                    r.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(K):
                for r in group:
                    r.run()
            torch.cuda.synchronize()
            fl_s = (time.perf_counter() - t0) / K
            assert all(r.error()[0] == 0 for r in group), [r.error() for r in group]
            same = all(torch.equal(runner.result()[k], r.result()[k]) for r in extra
                       for k in ("best_k", "best_chi2", "best_p0", "best_n_accept"))
            in_flight[str(n_fl)] = dict(value=n_fl * n_combos / fl_s,
                                        ms_per_batch=round(fl_s / n_fl * 1e3, 5),
                                        over_one_at_a_time=round(batch_s / (fl_s / n_fl), 3),
                                        same_results=same)
            L.svt_release_graphs()  # (before the buffers the graphs refer to go away)
            del extra, group

    # ---- ablation: one event per workgroup instead of flat combination tiles ---------------
    events_schedule = None
    if not args.no_kept_only:
        log("one event per workgroup")
        ev_tune = L.svt_tune_resolve(L.make_tune(tune.tile_combos, tune.chunk_roads, tune.wg_size,
                                                 4, 1))
        er = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=ev_tune,
                           graph=runner_graph, with_c=False)
        er.load(words)
        for _ in range(W):
            er.run()
        torch.cuda.synchronize()
        assert er.error() == (0, -1), er.error()
        t0 = time.perf_counter()
        for _ in range(K):
            er.run()
        torch.cuda.synchronize()
        ev_s = (time.perf_counter() - t0) / K
        events_schedule = dict(value=n_combos / ev_s, ms_per_step=round(ev_s * 1e3, 5),
                               flat_over_events=round(ev_s / batch_s, 2))
        del er
        L.svt_release_graphs()

    # ---- kept-only mode: no per-combination records ----------------------------------------
    kept_only = None
    if not args.no_kept_only:
        log("kept-only mode")
        L.svt_release_graphs()
        kept_only = measure_kept_only(gcfg, dbank, words, n_words, n_roads, n_combos, tune, K, W,
                                      runner_graph)

    # ---- plain path: one launch per stage, host syncs to size each stage ------------------
    plain = None
    if not args.no_plain:
        log("plain path")
        pr = P.PlainRunner(gcfg, dbank, with_c=False, want_kept=False)
        for _ in range(W):
            pr.run(words)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            pr.run(words)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_s = (t1 - t0) / K
        pr.run(words, timing=True)
        tm = pr.times
        plain = dict(value=n_combos / plain_s, ms_per_step=round(plain_s * 1e3, 4),
                     stages_ms=dict(unpack=round(tm.unpack_ms, 4), combine=round(tm.combine_ms, 4),
                                    fit=round(tm.fit_ms, 4), select=round(tm.select_ms, 4)),
                     batched_over_plain=round(plain_s / batch_s, 2))
        del pr

    small_res = None
    if small is not None:
        log(f"c1: {args.small_reps} repetitions of each path")
        small_res = measure_small(small, bank, synth.config_chi2_cut("c1"), args.small_reps,
                                  small_ora)

    uneven = None
    if uneven_s is not None:
        log("uneven batch: autotuning")
        uneven = measure_uneven(uneven_s, bank, log)

    serving = None
    if serve_s is not None:
        log(f"serving: {args.serve_events} events at {args.serve_rate:.0f} Hz")
        # small batches: the default launch shape (the autotuner's pick is for the big batch)
        serving = measure_serving(serve_s, bank, args.serve_warmup, args.serve_rate,
                                  args.serve_slots, 256, tune if explicit_tune else default_tune)

    transfer = None
    if transfer_s is not None:
        log("transfer study")
        transfer = measure_transfer(transfer_s, bank, tune if explicit_tune else default_tune,
                                    args.transfer_reps)

    large = None
    if large_s is not None:
        L.svt_release_graphs()
        del runner
        torch.cuda.empty_cache()
        large = measure_large(large_s, args.large_passes, tune if explicit_tune else None, bank)

    out = dict(
        metric=METRIC, value=value, unit="fitted combinations/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=round(batch_s * 1e3, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="int32/int64", data="synthetic",
        config=dict(workload=f"{args.config}: {n_events} events, {n_roads} roads, {n_words} hit "
                             f"words, {n_combos} combinations "
                             f"({n_combos / max(n_events, 1):.0f} per event)",
                    events=n_events, roads=n_roads, words=n_words, combinations=n_combos,
                    chi2_cut=cut, path="svt_process_batch (%s)" % (
                        "graph replay" if runner_graph else "direct launches"),
                    launch_modes_ms_per_pass=launch_modes,
                    tune=tune_dict(tune), autotune=tuned, device=dev_name),
        roofline=roofline, int_ops=int_ops(n_combos, k_ms, tune), cpu_baseline=cpu,
        small_batch=small_res, kept_only=kept_only,
        event_per_workgroup=events_schedule, plain=plain,
        batches_in_flight=in_flight,
        uneven_autotuned=uneven,
        serving=serving, transfer=transfer, max_scale=large)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

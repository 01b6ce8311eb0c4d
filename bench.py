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
import re
import os
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


def int_ops(n_combos, kernel_ms):
    """The fused kernel's algorithmic integer operations per second against the VALU peak (a
    second view beside the HBM roofline: the fit's arithmetic, not its bytes)."""
    achieved = INT_OPS_PER_COMBO * n_combos / (kernel_ms * 1e-3) / 1e12
    return dict(bound="alu", achieved=round(achieved, 3), peak=round(INT_PEAK_TOPS, 1),
                unit="Tops/s", frac=round(achieved / INT_PEAK_TOPS, 4), kernel="k_fused",
                ops_per_combination=INT_OPS_PER_COMBO)


PROFILES = os.path.join(ROOT, "profiles")
# sources the fused kernel is compiled from: recorded HBM counters are valid while these match
FUSED_SOURCES = [os.path.join(ROOT, "paper_1312_0917_amd", "csrc", f)
                 for f in ("svt_fused.hip", "svt_common.h")]


def fused_source_digest():
    h = hashlib.sha1()
    for f in FUSED_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(config, n_events):
    """HBM bytes per launch of the fused kernel from the committed counter summary for this
    workload (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what the counter
    reads for a plain copy of known size).  None when there is no summary for the workload or
    the kernel's sources changed since the counters were taken."""
    path = os.path.join(PROFILES, f"k_fused_{config}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    kv = dict(re.findall(r"^([a-z_0-9]+): (\S+)\s*$", open(path).read(), flags=re.M))
    try:
        if kv["kernel_source_sha1"] != fused_source_digest() or int(kv["events"]) != n_events:
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


def measure_large(config, n_events, passes, tune, bank, workers=16):
    """Max-scale run: whole batch resident in HBM, graph replays, fused-kernel roofline."""
    import torch

    import oracle
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth

    log(f"generating {config} ({n_events} events)")
    sample = synth.make_sample(config, bank=bank, n_events=n_events, workers=workers)
    cut = synth.config_chi2_cut(config)
    n_words, n_roads = len(sample.words), sample.n_roads
    n_combos = sample.expected_combos()
    runner = P.BatchRunner(L.make_config(chi2_cut=cut), P.device_bank(bank.f, bank.q), n_words,
                           n_roads, n_combos, kept_cap=0, tune=tune, graph=True, with_c=False)
    runner.load(P.words_tensor(sample.words))
    del sample
    runner.run()
    torch.cuda.synchronize()
    sz = runner.sizes()
    assert sz["n_combos"] == n_combos and runner.error()[0] == 0, (sz, runner.error())
    log(f"{config}: {passes} timed passes over {n_combos} combinations")
    t0 = time.perf_counter()
    for _ in range(passes):
        runner.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    k_ms = fused_kernel_ms(runner, passes, 1)
    L.svt_release_graphs()
    alg = algorithmic_bytes(n_combos, n_words, n_roads)
    ach = alg / (k_ms * 1e-3) / 1e9
    out = dict(workload=f"{config}: {n_events} events, {n_roads} roads, {n_words} hit words, "
                        f"{n_combos} combinations",
               value=n_combos / dt, unit="fitted combinations/s", ms_per_pass=round(dt * 1e3, 4),
               passes=passes, tune=dict(tile_combos=tune.tile_combos, chunk_roads=tune.chunk_roads,
                                        wg_size=tune.wg_size, wgs_per_cu=tune.wgs_per_cu,
                                        schedule=tune.schedule),
               roofline=dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(ach / HBM_PEAK_GBS, 4),
                             traffic=recorded_traffic(config, n_events), kernel="k_fused",
                             kernel_ms=round(k_ms, 4), algorithmic_bytes=alg,
                             bytes_per_combination=round(alg / n_combos, 3)),
               int_ops=int_ops(n_combos, k_ms))
    del runner
    torch.cuda.empty_cache()
    return out


def measure_uneven(bank, steps, log_fn):
    """Uneven batch in one persistent launch (8192 events, geometric roads/event, heavy-tailed
    hits per layer): the autotuner times every launch shape and keeps the fastest."""
    import torch

    import oracle
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth
    from paper_1312_0917_amd import tune as T

    sample = synth.make_sample("c3", bank=bank)
    cut = synth.config_chi2_cut("c3")
    st, nr, ne, nc, _ = oracle.count(sample.words, oracle.make_config(chi2_cut=cut))
    words = P.words_tensor(sample.words)
    res = T.autotune(words, P.device_bank(bank.f, bank.q), L.make_config(chi2_cut=cut), nr, nc,
                     steps=steps, cache_path=None, use_cache=False, log=log_fn)
    default = [row for row in res.table if row[:5] == (4096, 64, 256, 3, 0)]
    flat = [row[5] for row in res.table if row[4] == 0]
    events = [row[5] for row in res.table if row[4] == 1]
    return dict(workload=f"c3: {ne} events, {nr} roads, {len(sample.words)} hit words, "
                         f"{nc} combinations", best_tune=dict(zip(
                             ("tile_combos", "chunk_roads", "wg_size", "wgs_per_cu", "schedule"),
                             T.tune_tuple(res.tune))),
                ms_per_pass_best=round(res.ms_per_pass, 5),
                ms_per_pass_default=default[0][5] if default else None,
                value=nc / (res.ms_per_pass * 1e-3), unit="fitted combinations/s",
                candidates=len(res.table), all_outputs_identical=True,
                ablation_ms_per_pass=dict(flat_tiles_best=min(flat) if flat else None,
                                          event_per_workgroup_best=min(events) if events else None))


def measure_serving(bank, n_events, warmup_events, rate_hz, n_slots, max_events, tune, workers):
    """Poisson stream of events through the continuous-batching loop, fused path and plain path
    fed the same schedule; latency from arrival to results on the host (H2D and D2H included)."""
    import numpy as np
    import torch

    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import serve, synth

    sample = synth.make_sample("c4", bank=bank, n_events=n_events, workers=workers)
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
    for io in ("mapped", "copy"):
        slots = [serve.GpuSlot(cfg, dbank, word_cap, word_cap // 5 + 1, combo_cap, tune=tune,
                               io=io) for _ in range(n_slots)]
        # capture each slot's graph before the clock starts
        for sl in slots:
            sl.launch(warm.slice(0, 1), 0, 1)
            sl._wait()
            sl.collect()
        stats, _ = serve.serve(st, slots, max_events=max_events)
        out[io] = stats.summary(warmup_events)
        L.svt_release_graphs()
        del slots
        torch.cuda.empty_cache()
    pstats, _ = serve.serve(st, [serve.PlainSlot(cfg, dbank)], max_events=max_events)
    plain = pstats.summary(warmup_events)
    return dict(workload=f"c4: {n_events} events ({warmup_events} warm-up) arriving as a "
                         f"Poisson stream at {rate_hz / 1e3:.0f} kHz, {mean_w:.0f} words and "
                         f"{mean_c:.0f} combinations per event on average",
                slots=n_slots, max_events_per_batch=max_events,
                batched_io="words read and results written in place in page-locked host "
                           "memory (no copy calls); batched_copy: H2D and two-step D2H copies",
                batched=out["mapped"], batched_copy=out["copy"], plain=plain)


def measure_transfer(bank, tune, reps, workers):
    """Packet latency with pageable, pinned and mapped input (serving-shaped events)."""
    import numpy as np
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth, transfer

    sample = synth.make_sample("c4", n_events=10000, bank=bank, workers=workers)
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


def run_cpu_baseline(sample, bank, cfg, seconds):
    import oracle

    sec, reps, nc = oracle.time_run(sample.words, bank.f, bank.q, cfg, min_seconds=seconds)
    return dict(value=nc / sec, unit="fitted combinations/s", cores=1, kind="oracle",
                sample=f"whole batch ({nc} combinations), {reps} full oracle runs in "
                       f"{sec * reps:.1f} s, single thread, all outputs")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--events", type=int, default=0, help="override the workload's event count")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--occ", type=int, default=0)
    ap.add_argument("--large-events", type=int, default=10000,
                    help="events of the max-scale run (10000 x 2048 roads); 0 skips it")
    ap.add_argument("--large-passes", type=int, default=5)
    ap.add_argument("--workers", type=int, default=16, help="processes drawing large samples")
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

    import numpy as np
    import torch

    import oracle
    from paper_1312_0917_amd import _lib as L
    from paper_1312_0917_amd import pipeline as P
    from paper_1312_0917_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    K, W = args.steps, args.warmup

    log(f"generating {args.config}")
    bank = synth.make_bank()
    n_ev = args.events or synth.CONFIGS[args.config]["n_events"]
    big = synth.expected_size(args.config)["words"] * n_ev / synth.CONFIGS[args.config]["n_events"] > 5e7
    sample = synth.make_sample(args.config, bank=bank, n_events=n_ev,
                               workers=args.workers if big else 1)
    cut = synth.config_chi2_cut(args.config)
    cfg = oracle.make_config(chi2_cut=cut)
    st, n_roads, n_events, n_combos, _ = oracle.count(sample.words, cfg)
    assert st == 0
    n_words = len(sample.words)
    gcfg = L.make_config(chi2_cut=cut)
    dbank = P.device_bank(bank.f, bank.q)
    words = P.words_tensor(sample.words)
    explicit_tune = any((args.tile, args.chunk, args.wg, args.occ))
    tune = L.svt_tune_resolve(L.make_tune(args.tile, args.chunk, args.wg, args.occ))
    default_tune = L.svt_tune_resolve(None)
    tuned = None
    if not explicit_tune and not args.no_autotune:
        # the autotuner picks the launch shape of this batch (every candidate must write the
        # same bytes); the timed steps below then use the winner
        from paper_1312_0917_amd import tune as T
        log("autotuning the batch")
        res = T.autotune(words, dbank, gcfg, n_roads, n_combos, steps=10, cache_path=None,
                         use_cache=False)
        tune = res.tune
        tuned = dict(candidates=len(res.table), best_ms_per_pass=round(res.ms_per_pass, 5))

    # ---- batched path: resident buffers, graph replay -------------------------------------
    runner = P.BatchRunner(gcfg, dbank, n_words, n_roads, n_combos, kept_cap=0, tune=tune,
                           graph=not args.no_graph, with_c=False)
    runner.load(words)
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

    # ---- fused kernel alone: HIP events on the runner's stream around each launch ---------
    log("fused kernel timing")
    k_ms = fused_kernel_ms(runner, K, W)
    alg = algorithmic_bytes(n_combos, n_words, n_roads)
    achieved = alg / (k_ms * 1e-3) / 1e9
    traffic = recorded_traffic(args.config, n_events)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    traffic_over_algorithmic=round(traffic / alg, 3) if traffic else None,
                    kernel="k_fused", kernel_ms=round(k_ms, 5), algorithmic_bytes=alg,
                    bytes_per_combination=round(alg / n_combos, 3))

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
                                  graph=not args.no_graph, with_c=False)
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
                           graph=not args.no_graph, with_c=False)
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
                                      not args.no_graph)

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

    uneven = None
    if not args.no_uneven:
        log("uneven batch: autotuning")
        uneven = measure_uneven(bank, 10, log)

    serving = None
    if args.serve_events > 0:
        log(f"serving: {args.serve_events} events at {args.serve_rate:.0f} Hz")
        # small batches: the default launch shape (the autotuner's pick is for the big batch)
        serving = measure_serving(bank, args.serve_events, args.serve_warmup, args.serve_rate,
                                  args.serve_slots, 256, tune if explicit_tune else default_tune,
                                  args.workers)

    transfer = None
    if args.transfer_reps > 0:
        log("transfer study")
        transfer = measure_transfer(bank, tune if explicit_tune else default_tune,
                                    args.transfer_reps, args.workers)

    large = None
    if args.large_events > 0:
        L.svt_release_graphs()
        del runner
        torch.cuda.empty_cache()
        large = measure_large("c5", args.large_events, args.large_passes,
                              tune if explicit_tune else default_tune, bank, args.workers)

    cpu = None
    if not args.no_cpu:
        log(f"cpu oracle baseline (~{args.cpu_seconds:.0f} s)")
        cpu = run_cpu_baseline(sample, bank, cfg, args.cpu_seconds)

    t = tune
    out = dict(
        metric=METRIC, value=value, unit="fitted combinations/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=round(batch_s * 1e3, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="int32/int64", data="synthetic",
        config=dict(workload=f"{args.config}: {n_events} events, {n_roads} roads, {n_words} hit "
                             f"words, {n_combos} combinations "
                             f"({n_combos / max(n_events, 1):.0f} per event)",
                    events=n_events, roads=n_roads, words=n_words, combinations=n_combos,
                    chi2_cut=cut, path="svt_process_batch (%s)" % (
                        "direct launches" if args.no_graph else "graph replay"),
                    tune=dict(tile_combos=t.tile_combos, chunk_roads=t.chunk_roads,
                              wg_size=t.wg_size, wgs_per_cu=t.wgs_per_cu, schedule=t.schedule),
                    autotune=tuned,
                    device=dev_name),
        roofline=roofline, int_ops=int_ops(n_combos, k_ms), cpu_baseline=cpu,
        kept_only=kept_only,
        event_per_workgroup=events_schedule, plain=plain,
        batches_in_flight=in_flight,
        uneven_autotuned=uneven,
        serving=serving, transfer=transfer, max_scale=large)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

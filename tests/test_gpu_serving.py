"""Serving loop on the GPU: continuous batching gives every event the same result as fitting
it alone (integers: tolerance 0), and an overflowing batch is split and rerun correctly."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu_cfg, to_np

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import serve, synth

pytestmark = pytest.mark.gpu
KEYS = ("n_accept", "k", "p0", "p1", "p2", "chi2")
ORA = {"n_accept": "best_nacc", "k": "best_k", "p0": "best_p0", "p1": "best_p1",
       "p2": "best_p2", "chi2": "best_chi2"}


def _stream(bank, n_events, rate_hz, seed=3):
    s = synth.make_sample("c4", n_events=n_events, bank=bank)
    arr = synth.poisson_arrivals(s.n_events, rate_hz=rate_hz, seed=seed)
    return serve.EventStream(s.words, s.event_word_begin, arr)


def _alone_gpu(st, e, bank, dbank, cfg):
    w = st.slice(e, e + 1)
    ref = oracle.run(w, bank.f, bank.q, cfg, combos=False)
    r = P.BatchRunner(gpu_cfg(cfg), dbank, len(w), ref["n_roads"], ref["n_combos"] + 4,
                      graph=False, with_c=False)
    out = r.load(P.words_tensor(w)).run().result()
    return {k: to_np(out["best_" + k]) for k in KEYS}, ref


@pytest.mark.parametrize("io", ["mapped", "copy"])
def test_each_event_same_alone_and_in_the_mix(bank, io):
    cfg = oracle.make_config()
    dbank = P.device_bank(bank.f, bank.q)
    st = _stream(bank, 400, rate_hz=2e6)
    words_cap = 64 * 6000
    slots = [serve.GpuSlot(gpu_cfg(cfg), dbank, words_cap, words_cap // 5, 64 * 40000,
                           keep_results=True, io=io) for _ in range(3)]
    stats, res = serve.serve(st, slots, max_events=64, keep_results=True)
    assert max(stats.batch_sizes) > 1, "the stream should have been batched"
    assert not np.isnan(stats.latency_s).any() and np.all(stats.latency_s > 0)
    for e in range(0, st.n_events, 13):
        alone, ref = _alone_gpu(st, e, bank, dbank, cfg)
        for k in KEYS:
            assert np.array_equal(res[e][k], alone[k]), (e, k)
            assert np.array_equal(res[e][k], np.asarray(ref[ORA[k]])), (e, k)
    L.svt_release_graphs()


@pytest.mark.parametrize("io", ["mapped", "copy"])
def test_overflowing_batch_is_split_and_rerun(bank, io):
    cfg = oracle.make_config()
    dbank = P.device_bank(bank.f, bank.q)
    st = _stream(bank, 60, rate_hz=1e7, seed=4)
    # combination capacity of about 6 events: 16-event batches must split
    slot = serve.GpuSlot(gpu_cfg(cfg), dbank, 16 * 6000, 16 * 1200, 80000, keep_results=True,
                         io=io)
    stats, res = serve.serve(st, [slot], max_events=16, keep_results=True)
    assert slot.retries > 0
    for e in range(0, st.n_events, 5):
        ref = oracle.run(st.slice(e, e + 1), bank.f, bank.q, cfg, combos=False)
        for k in KEYS:
            assert np.array_equal(res[e][k], np.asarray(ref[ORA[k]])), (e, k)
    L.svt_release_graphs()


def test_plain_slot_serves_the_same_stream(bank):
    cfg = oracle.make_config()
    dbank = P.device_bank(bank.f, bank.q)
    st = _stream(bank, 50, rate_hz=1e6)
    stats, _ = serve.serve(st, [serve.PlainSlot(gpu_cfg(cfg), dbank)], max_events=16)
    tot = oracle.count(st.words, cfg)[3]
    assert stats.n_combos == tot


@pytest.mark.parametrize("where", ["device", "mapped"])
def test_gather_results_matches_the_batch_outputs(bank, where):
    """svt_gather_results: header = the batch's sizes and error word, then exactly n_roads
    entries of the best tracks, event ordinals and sets (integers: bit-exact); a buffer too
    small for the roads gets the header only."""
    cfg = oracle.make_config()
    dbank = P.device_bank(bank.f, bank.q)
    s = synth.make_sample("c4", n_events=24, bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, cfg, combos=False)
    nr = ref["n_roads"]
    r = P.BatchRunner(gpu_cfg(cfg), dbank, len(s.words), nr + 7, ref["n_combos"] + 4,
                      graph=False, with_c=False)
    out = r.load(P.words_tensor(s.words)).run().result()
    for cap in (nr + 7, nr, nr - 1):
        nbytes = L.GATHER_HEADER_BYTES + L.GATHER_BYTES_PER_ROAD * cap
        if where == "device":
            buf = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
            dst = buf
        else:
            buf = torch.full((nbytes,), 0xA5, dtype=torch.uint8, pin_memory=True)
            dst = L.svt_mapped_pointer(buf)
        g = L.PreparedGather(r.roads, r.best, r.road_cap, r.d_n[0:1], r.d_n[1:2], r.d_n[2:3],
                             None, r.d_err, dst, cap)
        g(r.stream)
        r.stream.synchronize()
        head, roads = L.gathered(buf.cpu().numpy() if where == "device" else buf.numpy())
        assert head == dict(n_words=len(s.words), n_roads=nr, n_combos=ref["n_combos"],
                            n_kept=-1, err=L.SVT_NO_ERROR)
        if cap < nr:
            assert roads is None
            continue
        for k in KEYS:
            assert np.array_equal(roads[k], to_np(out["best_" + k])), (cap, k)
            assert np.array_equal(roads[k], np.asarray(ref[ORA[k]])), (cap, k)
        assert np.array_equal(roads["event"], to_np(out["road_event"]))
        assert np.array_equal(roads["set"], to_np(out["road_set"]))
    L.svt_release_graphs()


def test_gather_results_reports_the_kept_count(bank):
    """With a kept list the header's fourth word is the accepted count (the oracle's)."""
    cfg = oracle.make_config()
    dbank = P.device_bank(bank.f, bank.q)
    s = synth.make_sample("c4", n_events=12, bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, cfg)
    nr, nc = ref["n_roads"], ref["n_combos"]
    r = P.BatchRunner(gpu_cfg(cfg), dbank, len(s.words), nr, nc, kept_cap=nc, graph=False,
                      with_c=False)
    r.load(P.words_tensor(s.words)).run()
    buf = torch.zeros(L.GATHER_HEADER_BYTES + L.GATHER_BYTES_PER_ROAD * nr, dtype=torch.uint8,
                      device="cuda")
    L.PreparedGather(r.roads, r.best, r.road_cap, r.d_n[0:1], r.d_n[1:2], r.d_n[2:3], r.d_n[3:4],
                     r.d_err, buf, nr)(r.stream)
    r.stream.synchronize()
    head, roads = L.gathered(buf.cpu().numpy())
    assert head["n_kept"] == int(ref["n_kept"]) > 0
    assert (head["n_roads"], head["n_combos"]) == (nr, nc)
    assert roads is not None and len(roads["k"]) == nr

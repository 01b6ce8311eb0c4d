"""GPU parity: both HIP paths against the CPU oracle, bit for bit (integer outputs).

Every input is drawn by the seeded generator; every expected value comes from the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (BATCH_KEYS, PLAIN_KEYS, compare, gpu_cfg, run_batch, run_plain, to_np)
from tiny import pack, random_bank, random_events, stream

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth

pytestmark = pytest.mark.gpu

CFG = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT)
ONEPASS, EVENTS, TILES = L.SVT_SCHEDULE_ONEPASS, L.SVT_SCHEDULE_EVENTS, L.SVT_SCHEDULE_TILES
TUNES = [L.make_tune(wgs_per_cu=1, schedule=ONEPASS), L.make_tune(wgs_per_cu=2, schedule=ONEPASS),
         L.make_tune(wgs_per_cu=3, schedule=ONEPASS),
         L.make_tune(4096, 64, 256, 2, TILES), L.make_tune(8192, 64, 256, 3, TILES),
         L.make_tune(4096, 64, 256, 4, TILES),  # a fourth workgroup per CU: a fourth priority slot
         L.make_tune(4096, 64, 512, 1, TILES), L.make_tune(8192, 64, 512, 2, TILES),
         L.make_tune(4096, 32, 256, 3, TILES), L.make_tune(8192, 16, 512, 2, TILES),
         L.make_tune(4096, 64, 256, 4, EVENTS)]  # the last: one event per workgroup


@pytest.fixture(scope="module")
def samples(bank):
    out = {}
    for c in ["c1", "c2", "c3"]:
        s = synth.make_sample(c, bank=bank)
        out[c] = (s, oracle.run(s.words, bank.f, bank.q, CFG))
    return out


@pytest.mark.parametrize("config", ["c1", "c2", "c3"])
def test_plain_path_matches_oracle(samples, bank, config):
    s, ref = samples[config]
    got = run_plain(s.words, bank.f, bank.q, CFG)
    compare(ref, got, PLAIN_KEYS, f"plain {config}")


@pytest.mark.parametrize("config", ["c1", "c2", "c3"])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("schedule", [ONEPASS, TILES])
def test_batch_path_matches_oracle(samples, bank, config, graph, schedule):
    s, ref = samples[config]
    got, runner = run_batch(s.words, bank.f, bank.q, CFG, ref=ref, graph=graph,
                            tune=L.make_tune(schedule=schedule))
    compare(ref, got, BATCH_KEYS, f"batch {config} graph={graph} schedule={schedule}")
    if graph:  # a replay of the captured graph gives the same bytes
        runner.run()
        compare(ref, runner.result(), BATCH_KEYS, f"batch {config} replay")
    L.svt_release_graphs()


@pytest.mark.parametrize("config", ["c1", "c2", "c3"])
def test_event_per_workgroup_schedule_matches_oracle(samples, bank, config):
    """Schedule 1 (one event per workgroup) against the oracle, with and without graphs."""
    s, ref = samples[config]
    for graph in (False, True):
        got, runner = run_batch(s.words, bank.f, bank.q, CFG, ref=ref, graph=graph,
                                tune=L.make_tune(4096, 64, 256, 4, 1))
        compare(ref, got, BATCH_KEYS, f"events {config} graph={graph}")
    L.svt_release_graphs()


@pytest.mark.parametrize("ti", range(len(TUNES)))
def test_batch_every_tune_is_bit_identical(samples, bank, ti):
    """Schedule independence: every tile / chunk / workgroup shape writes the same bytes."""
    s, ref = samples["c3"]
    got, _ = run_batch(s.words, bank.f, bank.q, CFG, ref=ref, tune=TUNES[ti], graph=False)
    compare(ref, got, BATCH_KEYS, f"c3 tune {ti}")


def test_batch_repeats_are_deterministic(samples, bank):
    s, ref = samples["c2"]
    got, runner = run_batch(s.words, bank.f, bank.q, CFG, ref=ref, graph=True)
    first = {k: to_np(v).copy() for k, v in got.items() if isinstance(v, torch.Tensor)}
    for _ in range(5):
        runner.run()
        again = runner.result()
        for k, v in first.items():
            assert np.array_equal(v, to_np(again[k])), k
    L.svt_release_graphs()


def test_batches_in_flight_on_two_streams(samples, bank):
    """Two runners, each with its own stream and captured graph, replayed back to back with no
    synchronisation between them (their kernels overlap on the device): each batch still gives
    the oracle's bytes, on every replay."""
    (s2, ref2), (s3, ref3) = samples["c2"], samples["c3"]
    _, r2 = run_batch(s2.words, bank.f, bank.q, CFG, ref=ref2, graph=True)
    _, r3 = run_batch(s3.words, bank.f, bank.q, CFG, ref=ref3, graph=True)
    for rep in range(3):
        for _ in range(4):
            r2.run()
            r3.run()
        torch.cuda.synchronize()
        compare(ref2, r2.result(), BATCH_KEYS, f"c2 in flight, round {rep}")
        compare(ref3, r3.result(), BATCH_KEYS, f"c3 in flight, round {rep}")
    L.svt_release_graphs()


@pytest.mark.parametrize("seed", range(12))
def test_tiny_random_streams(bank, seed):
    """Ragged tiny inputs: zero-combination roads, extreme constants and coordinates, cuts."""
    rng = np.random.default_rng(1000 + seed)
    ev = random_events(rng, n_events=int(rng.integers(1, 6)), max_roads=6,
                       max_hits=int(rng.integers(1, 9)), min_hits=0 if seed % 3 == 0 else 1)
    words = stream(ev)
    f, q = random_bank(rng, extreme=(seed % 2 == 0))
    cfg = oracle.make_config(chi2_cut=int(rng.choice([0, 10**6, 2**40, 2**62])),
                             shift=int(rng.choice([10, 1, 7, 16, 30])))
    ref = oracle.run(words, f, q, cfg)
    compare(ref, run_plain(words, f, q, cfg), PLAIN_KEYS, f"plain tiny {seed}")
    got, _ = run_batch(words, f, q, cfg, ref=ref, tune=TUNES[seed % len(TUNES)], graph=False)
    compare(ref, got, BATCH_KEYS, f"batch tiny {seed}")


def test_narrow_fit_form_at_its_bounds(bank):
    """The fused kernel's narrow form (whole offset in the int32 accumulator, chi-square summed
    in 32 bits) on constant sets exactly at its bounds, and one step past them (wide form).

    Set 0: rows 0-2 have 4096 * sum|f| + |q| = 2^31 - 1, and coordinates of -4096 against
    f = -32767 drive the row sum to exactly INT32_MAX; rows 3-5 have chi-square components up
    to 32766 in magnitude, so the sum of their squares passes 2^31 (the unsigned 32-bit sum).
    Sets 1 and 2 exceed the chi-square bound and the int32 bound by one and take the wide
    form.  A chunk holding any of them is fitted wide: the first four events (16 roads) use
    only sets 0 and 3, so with 16 roads per chunk their chunk is narrow, and with 64 roads per
    chunk everything is fitted wide."""
    f = np.zeros((256, 6, 5), np.int64)
    q = np.zeros((256, 6), np.int64)
    f[:, :, :] = np.random.default_rng(5).integers(-50, 51, size=(256, 6, 5))
    for s_ in range(3):
        f[s_, 0:3, :] = -32767
        q[s_, 0:3] = 2**31 - 1 - 4096 * 5 * 32767
        f[s_, 3:6, :] = 0
        f[s_, 3:6, 0] = [8191, -8191, 8191]
        q[s_, 3:6] = 33553407 - 4096 * 8191  # (B >> 10) + 1 = 32767
    q[1, 4] += 1024        # chi-square bound passed by one step of the shift
    q[2, 1] += 1           # int32 bound passed by one
    assert np.all(np.abs(f) <= 32767) and np.all(np.abs(q) < 2**31)
    f, q = f.astype(np.int16), q.astype(np.int32)
    rng = np.random.default_rng(6)
    events = []
    for e in range(6):
        roads = []
        for r, st in enumerate([0, 3, 0, 3] if e < 4 else [1, 2, 0, 3]):
            coords = [-4096] * 5 if (e + r) % 2 == 0 else [4095] * 5
            hits = [(l, coords[l]) for l in range(5)]
            hits += [(l, int(rng.integers(-4096, 4096))) for l in range(5)
                     for _ in range(int(rng.integers(0, 3)))]
            roads.append((st, [hits[i] for i in rng.permutation(len(hits))]))
        events.append(roads)
    words = stream(events)
    cfg = oracle.make_config(chi2_cut=2**62, shift=10)
    ref = oracle.run(words, f, q, cfg)
    p0 = np.asarray(ref["p0"]).astype(np.int64)
    chi2 = np.asarray(ref["chi2"]).astype(np.int64)
    first = int(np.asarray(ref["road_combo_begin"])[16])  # combinations of the first 16 roads
    assert p0[:first].max() == (2**31 - 1) >> 10  # a row sum reached INT32_MAX
    assert chi2[:first].max() > 2**31             # the 32-bit chi-square sum passed 2^31
    for t in (L.make_tune(4096, 16, 256, 3, TILES), L.make_tune(8192, 64, 256, 2, TILES)):
        got, _ = run_batch(words, f, q, cfg, ref=ref, tune=t, graph=False)
        compare(ref, got, BATCH_KEYS, f"narrow bounds chunk {t.chunk_roads}")


@pytest.mark.parametrize("extreme", [False, True])
def test_giant_roads_span_many_tiles(bank, extreme):
    """Roads of 8^5 = 32768 combinations cut by several 4096-combination tiles.

    With extreme constants and a cut above 2^49 every combination is accepted with a chi2 too
    large for the packed best-track key, which exercises the exact rescan and the merge of
    per-tile partial results."""
    rng = np.random.default_rng(7)
    events = []
    for e in range(3):
        roads = []
        for r in range(3):
            hits = [(l, int(rng.integers(-4096, 4096))) for l in range(5) for _ in range(8)]
            if r == 1:  # embed a noise-free track so the road has an accepted best
                s = 10 + r
                x = bank.A[s] @ np.array([5, -6, 7]) + bank.b[s]
                hits[8 * 4 + 3] = (4, int(x[4]))
                for l in range(4):
                    hits[8 * l + 5] = (l, int(x[l]))
            roads.append((10 + r, [hits[i] for i in rng.permutation(len(hits))]))
        events.append(roads)
    words = stream(events)
    f, q, cfg = bank.f, bank.q, CFG
    if extreme:
        f, q = random_bank(np.random.default_rng(8), extreme=True)
        cfg = oracle.make_config(chi2_cut=2**62, shift=3)
    ref = oracle.run(words, f, q, cfg)
    assert ref["n_combos"] == 9 * 32768
    if extreme:
        assert int(np.asarray(ref["best_chi2"]).min()) > 2**49
    for t in TUNES:
        got, _ = run_batch(words, f, q, cfg, ref=ref, tune=t, graph=False)
        compare(ref, got, BATCH_KEYS, f"giant extreme={extreme}")
    compare(ref, run_plain(words, f, q, cfg), PLAIN_KEYS, f"giant plain extreme={extreme}")


def _boundary_stream(bank, rng, full, n_events, small):
    """Events whose roads fill tiles exactly and then put roads without combinations (an empty
    layer) where the next tile begins; with small roads (2^5 combinations each) the batch's
    road-spanning groups are written by the listed pass, with large ones (4^5) they go through
    the LDS stash."""
    n = 2 if small else 4
    per_tile = 4096 // (n ** 5)
    events = []
    for e in range(n_events):
        roads, tag = [], 1
        # the first six events fill whole tiles; extra roads in the last three move the
        # boundaries into roads
        for r in range(per_tile + (e % 3 if e >= 6 else 0)):
            hits = [(l, int(rng.integers(-4096, 4096))) for l in range(5) for _ in range(n)]
            if full and r % 3 == 1:  # a noise-free track: the road has an accepted best
                x = bank.A[tag] @ np.array([5, -6, 7]) + bank.b[tag]
                for l in range(5):
                    hits[n * l] = (l, int(x[l]))
            roads.append((tag, [hits[i] for i in rng.permutation(len(hits))]))
            tag += 1
        for r in range(1 + e % 2):  # no combinations: layer 1 or 3 has no hit
            empty = 1 if r == 0 else 3
            hits = [(l, int(rng.integers(-4096, 4096))) for l in range(5) if l != empty
                    for _ in range(1 + (l + r) % 2)]
            roads.append((tag, hits))
            tag += 1
        if not full:  # every road of the batch without combinations
            roads = roads[-(1 + e % 2):]
        events.append(roads)
    return stream(events)


@pytest.mark.parametrize("small", [False, True])
@pytest.mark.parametrize("full", [True, False])
def test_roads_without_combinations_at_tile_boundaries(bank, small, full):
    """Roads without combinations (an empty layer) exactly where tiles of 4096 and 8192
    combinations begin, where the road holding a tile's first combination is not the tile's
    first road; and (full=False) a batch with roads but no combination at all, so that the
    fused kernel has no tile.  Every road's best track and count, with and without a kept
    list."""
    rng = np.random.default_rng(31 + 2 * small + full)
    words = _boundary_stream(bank, rng, full, 9, small)
    ref = oracle.run(words, bank.f, bank.q, CFG)
    if full:
        assert ref["n_combos"] > 2 * 8192
        assert int(np.asarray(ref["best_k"]).max()) >= 0
    else:
        assert ref["n_combos"] == 0 and ref["n_roads"] > 0
    for t in (L.make_tune(4096, 64, 256, 3, TILES), L.make_tune(8192, 32, 256, 2, TILES),
              L.make_tune(4096, 16, 512, 1, TILES)):
        for kept in (True, False):
            got, _ = run_batch(words, bank.f, bank.q, CFG, ref=ref, tune=t, graph=False,
                               kept=kept)
            keys = BATCH_KEYS if kept else [k for k in BATCH_KEYS if "kept" not in k]
            compare(ref, got, keys, f"boundary small={small} full={full} tile "
                                    f"{t.tile_combos} kept={kept}")


def test_empty_input(bank):
    words = np.zeros(0, np.uint32)
    got, _ = run_batch(words, bank.f, bank.q, CFG, ref=dict(n_roads=0, n_combos=0), graph=False)
    assert got["n_roads"] == 0 and got["n_combos"] == 0 and got["n_kept"] == 0
    r = run_plain(words, bank.f, bank.q, CFG)
    assert r["n_roads"] == 0 and r["n_combos"] == 0


def test_split_at_event_boundaries(samples, bank):
    """Results of a batch cut at an event boundary equal the whole batch's."""
    s, ref = samples["c2"]
    cut = 1234
    w1, w2 = s.event_slice(0, cut), s.event_slice(cut, s.n_events)
    r1, _ = run_batch(w1, bank.f, bank.q, CFG, graph=False)
    r2, _ = run_batch(w2, bank.f, bank.q, CFG, graph=False)
    for k in ["p0", "p1", "p2", "chi2", "accept"]:
        both = np.concatenate([to_np(r1[k]), to_np(r2[k])])
        assert np.array_equal(both, np.asarray(ref[k])), k
    for k, kk in [("best_k", "best_k"), ("best_chi2", "best_chi2"), ("best_nacc", "best_n_accept")]:
        both = np.concatenate([to_np(r1[kk]), to_np(r2[kk])])
        assert np.array_equal(both, np.asarray(ref[k])), k


def test_graph_replay_with_new_batches(bank):
    """One captured graph serves batches of different sizes loaded into the same buffers."""
    big = synth.make_sample("c4", n_events=64, bank=bank)
    ref_big = oracle.run(big.words, bank.f, bank.q, CFG)
    wc, rc, cc = len(big.words), ref_big["n_roads"] + 1, ref_big["n_combos"] + 4
    runner = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), wc, rc, cc, kept_cap=cc,
                           graph=True)
    for e0, e1 in [(0, 64), (3, 10), (10, 11), (0, 40), (20, 64)]:
        words = big.event_slice(e0, e1)
        ref = oracle.run(words, bank.f, bank.q, CFG)
        got, _ = run_batch(words, bank.f, bank.q, CFG, runner=runner)
        compare(ref, got, BATCH_KEYS, f"replay {e0}-{e1}")
    L.svt_release_graphs()


def _err_of(got_runner):
    return got_runner.error()


def test_input_errors_are_reported(bank):
    good = [[(1, [(l, 5) for l in range(5)]), (2, [(l, 6) for l in range(5)])]]
    words = stream(good)
    bad_layer = words.copy()
    bad_layer[7] = pack(5, 6, 2, 0)
    too_many = stream([[(1, [(l, 5) for l in range(5)]), (2, [(0, 1)] * 9 + [(l, 1) for l in range(1, 5)])]])
    cases = [(bad_layer, CFG, L.SVT_ERR_LAYER, 7), (too_many, CFG, L.SVT_ERR_HITS, 1),
             (words, oracle.make_config(n_sets=2), L.SVT_ERR_SET, 1)]
    for w, cfg, status, index in cases:
        st, *_ , ei = oracle.count(w, cfg)
        assert (st, ei) == (status, index)
        runner = P.BatchRunner(gpu_cfg(cfg), P.device_bank(bank.f, bank.q), 64, 64, 4096,
                               kept_cap=64, graph=False)
        runner.load(P.words_tensor(w)).run()
        torch.cuda.synchronize()
        assert runner.error() == (status, index)
        with pytest.raises(P.DeviceError):
            run_plain(w, bank.f, bank.q, cfg)


def test_capacity_errors_report_required_sizes(samples, bank):
    s, ref = samples["c1"]
    w = P.words_tensor(s.words)
    dbank = P.device_bank(bank.f, bank.q)
    nr, nc, nk = ref["n_roads"], ref["n_combos"], ref["n_kept"]
    for caps, which in [((nr - 1, nc, nk), 0), ((nr, nc - 1, nk), 1), ((nr, nc, nk - 1), 2)]:
        runner = P.BatchRunner(gpu_cfg(CFG), dbank, len(s.words), caps[0], caps[1],
                               kept_cap=caps[2], graph=False)
        runner.load(w).run()
        torch.cuda.synchronize()
        assert runner.error() == (L.SVT_ERR_CAPACITY, which)
        sz = runner.sizes()
        assert sz["n_roads"] == nr
        if which >= 1:
            assert sz["n_combos"] == nc
        if which == 2:
            assert sz["n_kept"] == nk
    # retry with the reported sizes succeeds
    runner = P.BatchRunner(gpu_cfg(CFG), dbank, len(s.words), nr, nc, kept_cap=nk, graph=False)
    runner.load(w).run()
    compare(ref, runner.result(), BATCH_KEYS, "retry")


def test_words_capacity_of_device_count(bank):
    """A device word count above word_cap is an error, never an out-of-bounds read."""
    s = synth.make_sample("c1", n_events=4, bank=bank)
    runner = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), len(s.words), 64, 4096,
                           graph=False)
    runner.load(P.words_tensor(s.words))
    runner.d_n[0].fill_(len(s.words) + 100)
    runner.run()
    torch.cuda.synchronize()
    assert runner.error() == (L.SVT_ERR_CAPACITY, 3)


def test_noise_free_tracks_on_gpu(samples, bank):
    s, ref = samples["c2"]
    got, _ = run_batch(s.words, bank.f, bank.q, CFG, ref=ref, graph=False)
    cb = to_np(got["road_combo_begin"])
    tr = np.nonzero(s.true_road)[0]
    for r in tr[:2000]:
        k = 0
        for l in range(5):
            k = k * int(s.road_nhits[r, l]) + int(s.true_slot[r, l])
        g = cb[r] + k
        assert (int(got["p0"][g]), int(got["p1"][g]), int(got["p2"][g])) == tuple(s.true_t[r])
        assert int(got["chi2"][g]) == 0

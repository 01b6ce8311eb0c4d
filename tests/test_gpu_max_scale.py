"""Parity at the max-scale workload (10000 events x 2048 roads, 2.0e9 combinations), in the
launch configuration the benchmark times (default tune, captured graph).

The oracle cannot fit 2e9 combinations in seconds, so it runs on sampled events one by one
(first, last and seeded random ones); each is compared bit for bit with the GPU's records and
best tracks for that event's roads.  Properties that hold at any size cover the whole batch:
sizes equal the generator's, ncombo is the product of hits per layer, combo_begin is the
exclusive scan of ncombo, the accepted count equals the sum of n_accept, and every road that
carries a noise-free track has a best track with chi2 = 0.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu_cfg, to_np

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth

pytestmark = pytest.mark.gpu

CFG = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT)
N_SAMPLED = 24


@pytest.fixture(scope="module")
def max_scale(bank):
    s = synth.make_sample("c5", bank=bank, workers=16)
    n_roads, n_combos = len(s.road_event), int(s.expected_combos())
    print(f"c5: {len(s.words)} words, {n_roads} roads, {n_combos} combinations", flush=True)
    runner = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), len(s.words), n_roads,
                           n_combos, kept_cap=0, tune=L.make_tune(), graph=True, with_c=False)
    runner.load(P.words_tensor(s.words))
    runner.run()
    runner.run()  # second replay: the measured configuration
    torch.cuda.synchronize()
    yield s, runner
    L.svt_release_graphs()
    del runner
    torch.cuda.empty_cache()


def test_sizes_and_road_table(max_scale):
    s, r = max_scale
    assert r.error() == (0, -1)
    sz = r.sizes()
    assert sz["n_roads"] == len(s.road_event)
    assert sz["n_combos"] == int(s.expected_combos())
    nr = sz["n_roads"]
    nh = to_np(r.roads["nhits"][:nr]).astype(np.int64) & 0xFFFFFFFF
    per_layer = np.stack([(nh >> (4 * l)) & 15 for l in range(5)], axis=1)
    np.testing.assert_array_equal(per_layer, s.road_nhits)
    ncombo = to_np(r.roads["ncombo"][:nr]).astype(np.int64)
    np.testing.assert_array_equal(ncombo, np.prod(s.road_nhits.astype(np.int64), axis=1))
    cb = to_np(r.roads["combo_begin"][:nr])
    np.testing.assert_array_equal(cb[1:], np.cumsum(ncombo)[:-1])
    assert cb[0] == 0
    np.testing.assert_array_equal(to_np(r.roads["event"][:nr]), s.road_event)
    np.testing.assert_array_equal(to_np(r.roads["set"][:nr]), s.road_set)


def test_accept_counts_and_noise_free_tracks(max_scale):
    s, r = max_scale
    sz = r.sizes()
    nr, nc = sz["n_roads"], sz["n_combos"]
    n_acc_records = int(r.accept[:nc].sum(dtype=torch.int64))
    n_acc_roads = int(r.best["n_accept"][:nr].sum(dtype=torch.int64))
    assert n_acc_records == n_acc_roads
    true_roads = np.nonzero(s.true_road)[0]
    assert true_roads.size > 0.15 * nr
    best_chi2 = to_np(r.best["chi2"][:nr])
    assert np.all(best_chi2[true_roads] == 0)
    assert np.all(to_np(r.best["n_accept"][:nr])[true_roads] >= 1)


def test_sampled_events_match_oracle(max_scale, bank):
    s, r = max_scale
    n_ev = s.n_events
    rng = np.random.default_rng(1312)
    events = sorted(set([0, n_ev - 1] + list(rng.choice(n_ev, N_SAMPLED - 2, replace=False))))
    road_begin = np.searchsorted(s.road_event, np.arange(n_ev + 1))
    for e in events:
        words = s.event_slice(e, e + 1)
        ref = oracle.run(words, bank.f, bank.q, CFG)
        r0, r1 = int(road_begin[e]), int(road_begin[e + 1])
        assert ref["n_roads"] == r1 - r0
        c0 = int(r.roads["combo_begin"][r0])
        c1 = c0 + int(ref["n_combos"])
        where = f"event {e} (roads {r0}..{r1}, combinations {c0}..{c1})"
        for k in ("p0", "p1", "p2", "chi2"):
            got = to_np(r.rec[k][c0:c1]).astype(np.int64)
            np.testing.assert_array_equal(got, np.asarray(ref[k]).astype(np.int64), err_msg=f"{where} {k}")
        np.testing.assert_array_equal(to_np(r.accept[c0:c1]).astype(np.int64),
                                      np.asarray(ref["accept"]).astype(np.int64), err_msg=f"{where} accept")
        for ok, gk in (("best_nacc", "n_accept"), ("best_k", "k"), ("best_p0", "p0"),
                       ("best_p1", "p1"), ("best_p2", "p2"), ("best_chi2", "chi2")):
            got = to_np(r.best[gk][r0:r1]).astype(np.int64)
            np.testing.assert_array_equal(got, np.asarray(ref[ok]).astype(np.int64), err_msg=f"{where} {ok}")
        ref_cb = np.asarray(ref["road_combo_begin"]).astype(np.int64) + c0
        np.testing.assert_array_equal(to_np(r.roads["combo_begin"][r0:r1]), ref_cb, err_msg=where)

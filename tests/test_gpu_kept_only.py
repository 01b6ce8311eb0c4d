"""Kept-only mode (no per-combination records): the kept list, its compacted fit values, the
accept flags and the best track per road must equal the oracle's, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import BATCH_KEYS, compare, gpu_cfg, to_np
from tiny import random_bank, random_events, stream

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth

pytestmark = pytest.mark.gpu

CFG = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT)
KEYS = [k for k in BATCH_KEYS if k not in ("p0", "p1", "p2", "c0", "c1", "c2", "chi2")]


def run_kept_only(words, f, q, cfg, ref, graph=True, tune=None, kept_cap=None):
    n = max(len(words), 1)
    cap = max(ref["n_kept"], 1) if kept_cap is None else kept_cap
    runner = P.BatchRunner(gpu_cfg(cfg), P.device_bank(f, q), n, max(ref["n_roads"], 1),
                           max(ref["n_combos"], 4), kept_cap=cap, graph=graph, tune=tune,
                           kept_only=True)
    w = P.words_tensor(words) if len(words) else torch.zeros(1, dtype=torch.int32, device="cuda")
    runner.load(w, len(words)).run()
    return runner


def check(ref, got, where):
    compare(ref, got, KEYS, where)
    kept = np.asarray(ref["kept"]).astype(np.int64)
    assert np.array_equal(to_np(got["kept"]).astype(np.int64), kept), f"{where}: kept list"
    for k in ("p0", "p1", "p2", "chi2", "c0", "c1", "c2"):
        if got.get(f"kept_{k}") is None:
            continue
        exp = np.asarray(ref[k]).astype(np.int64)[kept]
        np.testing.assert_array_equal(to_np(got[f"kept_{k}"]).astype(np.int64), exp,
                                      err_msg=f"{where}: kept {k}")


@pytest.mark.parametrize("config", ["c1", "c2", "c3"])
def test_kept_only_matches_oracle(bank, config):
    s = synth.make_sample(config, bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, CFG)
    runner = run_kept_only(s.words, bank.f, bank.q, CFG, ref)
    got = runner.result()
    assert got["n_kept"] == ref["n_kept"] > 0
    check(ref, got, f"kept-only {config}")
    runner.run()  # graph replay
    check(ref, runner.result(), f"kept-only {config} replay")
    L.svt_release_graphs()


@pytest.mark.parametrize("seed", range(8))
def test_kept_only_tiny_streams_and_extreme_constants(seed):
    """Ragged tiny inputs as in the default-mode parity tests, including extreme constants
    whose chi-square saturates the best-track key (the exact rescan then refits)."""
    rng = np.random.default_rng(2000 + seed)
    ev = random_events(rng, n_events=int(rng.integers(1, 6)), max_roads=6,
                       max_hits=int(rng.integers(1, 9)), min_hits=0 if seed % 3 == 0 else 1)
    words = stream(ev)
    f, q = random_bank(rng, extreme=(seed % 2 == 0))
    cfg = oracle.make_config(chi2_cut=int(rng.choice([10**6, 2**40, 2**62])),
                             shift=int(rng.choice([10, 1, 7, 16, 30])))
    ref = oracle.run(words, f, q, cfg)
    runner = run_kept_only(words, f, q, cfg, ref, graph=False)
    check(ref, runner.result(), f"tiny seed {seed}")


def test_kept_only_with_event_per_workgroup_schedule(bank):
    s = synth.make_sample("c3", bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, CFG)
    runner = run_kept_only(s.words, bank.f, bank.q, CFG, ref, graph=False,
                           tune=L.make_tune(4096, 64, 256, 4, 1))
    check(ref, runner.result(), "kept-only, events per workgroup")


def test_kept_only_capacity_reports_required_size(bank):
    s = synth.make_sample("c1", bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, CFG)
    runner = run_kept_only(s.words, bank.f, bank.q, CFG, ref, graph=False,
                           kept_cap=ref["n_kept"] - 1)
    torch.cuda.synchronize()
    assert runner.error() == (L.SVT_ERR_CAPACITY, 2)
    assert runner.sizes()["n_kept"] == ref["n_kept"]


@pytest.mark.parametrize("graph", [False, True])
def test_kept_only_bad_input_reports_error_and_sizes(bank, graph):
    """Kept-only passes over input the buffers or the bank cannot take: the pass reports the
    error and the sizes the input needs, and reads nothing it was not given (the refit pass
    runs after the error and must not touch the incomplete road table or a missing set)."""
    s = synth.make_sample("c1", bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, CFG)
    w = P.words_tensor(s.words)
    # too few road entries: capacity error with index 0 (roads), sizes still exact
    small = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), len(s.words),
                          ref["n_roads"] // 2, ref["n_combos"] + 4, kept_cap=ref["n_kept"] + 1,
                          graph=graph, kept_only=True)
    small.load(w).run()
    torch.cuda.synchronize()
    assert small.error() == (L.SVT_ERR_CAPACITY, 0)
    sz = small.sizes()
    assert (sz["n_roads"], sz["n_combos"]) == (ref["n_roads"], ref["n_combos"])
    # a bank of 16 sets: road tags 16..255 have no constant set
    cfg16 = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT, n_sets=16)
    bad = oracle.run(s.words, bank.f[:16], bank.q[:16], cfg16, raise_on_error=False)
    assert bad["status"] == oracle.ERR_SET
    r16 = P.BatchRunner(gpu_cfg(cfg16), P.device_bank(bank.f[:16], bank.q[:16]), len(s.words),
                        ref["n_roads"], ref["n_combos"] + 4, kept_cap=ref["n_kept"] + 1,
                        graph=graph, kept_only=True)
    r16.load(w).run()
    torch.cuda.synchronize()
    assert r16.error() == (L.SVT_ERR_SET, bad["err_index"])
    sz = r16.sizes()
    assert (sz["n_roads"], sz["n_combos"]) == (ref["n_roads"], ref["n_combos"])
    L.svt_release_graphs()

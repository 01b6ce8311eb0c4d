"""The pre-pass look-back's fallback: a block that waits too long for a predecessor computes
the predecessor's aggregate (roads, events, combinations) from the words itself.  With the
wait bound forced to zero (the SVT_LOOKBACK_TIMEOUT_TICKS hook, read at every direct launch)
nearly every block takes that path; every output must still equal the oracle's bit for bit,
and the sizes of inputs with errors (hit counts over the limit, overlong roads) must stay the
sizes the input needs."""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import BATCH_KEYS, compare, gpu_cfg, run_batch
from tiny import stream

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth

pytestmark = pytest.mark.gpu
CFG = oracle.make_config()
HOOK = "SVT_LOOKBACK_TIMEOUT_TICKS"


@pytest.fixture
def forced_fallback():
    L.svt_release_graphs()
    old = os.environ.get(HOOK)
    os.environ[HOOK] = "0"
    yield
    if old is None:
        del os.environ[HOOK]
    else:
        os.environ[HOOK] = old
    L.svt_release_graphs()


# both look-backs: the one-pass kernel's (units of 1024 words, one wave) and the pre-pass's
# (blocks of 2048 words in groups of 64)
SCHEDULES = {"onepass": L.SVT_SCHEDULE_ONEPASS, "prepass": L.SVT_SCHEDULE_TILES}


@pytest.mark.parametrize("schedule", list(SCHEDULES))
@pytest.mark.parametrize("config,n_events", [("c2", 150), ("c3", 300)])
def test_forced_fallback_matches_oracle(bank, forced_fallback, config, n_events, schedule):
    s = synth.make_sample(config, bank=bank, n_events=n_events)
    assert len(s.words) > 40 * 2048, "several dozen pre-pass blocks"
    cfg = oracle.make_config(chi2_cut=synth.config_chi2_cut(config))
    ref = oracle.run(s.words, bank.f, bank.q, cfg)
    got, _ = run_batch(s.words, bank.f, bank.q, cfg, ref=ref, graph=False,
                       tune=L.make_tune(schedule=SCHEDULES[schedule]))
    compare(ref, got, BATCH_KEYS, f"forced fallback {config} {schedule}")


@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_forced_fallback_across_groups(bank, forced_fallback, schedule):
    """Pre-pass blocks in groups past the first also sum group values (level 2 of its
    look-back); with the wait bound at zero they compute missing group values from the blocks'
    words."""
    s = synth.make_sample("c2", bank=bank, n_events=1000)
    assert len(s.words) > 4 * 64 * 2048, "five groups of 64 pre-pass blocks"
    cfg = oracle.make_config(chi2_cut=synth.config_chi2_cut("c2"))
    ref = oracle.run(s.words, bank.f, bank.q, cfg)
    got, _ = run_batch(s.words, bank.f, bank.q, cfg, ref=ref, graph=False,
                       tune=L.make_tune(schedule=SCHEDULES[schedule]))
    compare(ref, got, BATCH_KEYS, f"forced fallback across look-back groups, {schedule}")


@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_forced_fallback_keeps_required_sizes_of_bad_input(bank, forced_fallback, schedule):
    """Roads with too many hits on a layer, and roads longer than any legal one, spread over
    many blocks: no combinations for them, every size as the oracle counts it."""
    rng = np.random.default_rng(11)
    events = []
    for e in range(120):
        roads = []
        for r in range(40):
            kind = rng.integers(0, 10)
            if kind == 0:    # 9 hits on layer 2: over the limit
                hits = [(l, 1) for l in range(5)] + [(2, 3)] * 8
            elif kind == 1:  # 60 words: longer than 5 x 8
                hits = [(l % 5, l) for l in range(60)]
            else:
                hits = [(l, int(rng.integers(-4096, 4096))) for l in range(5)
                        for _ in range(int(rng.integers(1, 4)))]
            roads.append((int(rng.integers(0, 200)) if r % 2 else 1 + (r % 7),
                          [hits[i] for i in rng.permutation(len(hits))]))
        events.append(roads)
    words = stream(events)
    assert len(words) > 30 * 2048
    st, nr, ne, nc, ei = oracle.count(words, CFG)
    assert st == L.SVT_ERR_HITS
    out = {}
    for mode, ticks in (("own", "20000"), ("forced", "0")):
        os.environ[HOOK] = ticks
        runner = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), len(words),
                               nr + 8, 64 * len(words), kept_cap=0, graph=False,
                               tune=L.make_tune(schedule=SCHEDULES[schedule]))
        runner.load(P.words_tensor(words)).run()
        torch.cuda.synchronize()
        out[mode] = (runner.sizes(), runner.error())
    # the oracle stops at the first error, so the combination count is checked between the
    # blocks' own counting and the computed aggregates
    for mode in out:
        sizes, err = out[mode]
        assert sizes["n_roads"] == nr, mode
        assert err == (L.SVT_ERR_HITS, ei), mode
    assert out["forced"][0] == out["own"][0]
    assert out["own"][0]["n_combos"] > 0

"""Transfer strategies: the words read in place from mapped host memory give the same results
as words copied into HBM, and the study measures every mode and packet size."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import BATCH_KEYS, compare, gpu_cfg

from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth, transfer

pytestmark = pytest.mark.gpu

CFG = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT)


def test_mapped_input_matches_oracle(bank):
    s = synth.make_sample("c4", n_events=64, bank=bank)
    ref = oracle.run(s.words, bank.f, bank.q, CFG)
    n = len(s.words)
    runner = P.BatchRunner(gpu_cfg(CFG), P.device_bank(bank.f, bank.q), n, ref["n_roads"],
                           ref["n_combos"], kept_cap=ref["n_combos"], graph=True)
    pinned = torch.empty(n, dtype=torch.int32, pin_memory=True)
    pinned.numpy().view(np.uint32)[:] = s.words
    ptr = L.svt_mapped_pointer(pinned)
    with torch.cuda.stream(runner.stream):
        runner.d_n[0].fill_(n)
    runner.run(words=ptr)
    compare(ref, runner.result(), BATCH_KEYS, "mapped input")
    runner.run(words=ptr)  # replay of the captured graph
    compare(ref, runner.result(), BATCH_KEYS, "mapped input, replay")
    L.svt_release_graphs()


def test_study_covers_every_mode_and_size(bank):
    s = synth.make_sample("c4", n_events=200, bank=bank)
    combos = np.prod(s.road_nhits.astype(np.int64), axis=1)
    pts = transfer.study(s.words, s.event_word_begin, s.road_event, combos, gpu_cfg(CFG),
                         P.device_bank(bank.f, bank.q), sizes=(100_000, 400_000), reps=2,
                         warmup=1)
    assert len(pts) == 6
    assert [p.packet_bytes >= 100_000 for p in pts[:3]] == [True] * 3
    assert [p.packet_bytes >= 400_000 for p in pts[3:]] == [True] * 3
    assert {p.mode for p in pts} == set(transfer.MODES)
    for p in pts:
        assert p.total_us > 0 and p.compute_us > 0 and p.events >= 1
        assert 0.0 <= p.transfer_share <= 1.0

"""svt_process_batch_static -- the batch entry point for callers that cannot allocate device
memory -- against svt_process_batch on the same inputs, bit for bit, and against the oracle.

Two calls in a row through the same buffers: a batch of 3000 events of 64 roads, then one of
100 events of 8 roads, so the second call finds the first call's contents in the library's
static workspace and must clear what it needs itself.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import BATCH_KEYS, caps_for, compare, gpu_cfg, to_np
from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P
from paper_1312_0917_amd import synth

pytestmark = pytest.mark.gpu

CFG = oracle.make_config(chi2_cut=synth.DEFAULT_CHI2_CUT)


@pytest.fixture(scope="module")
def two_batches(bank):
    out = []
    for c in ("c2", "c1"):
        s = synth.make_sample(c, bank=bank)
        out.append((c, s.words, oracle.run(s.words, bank.f, bank.q, CFG)))
    return out


def outputs(runner):
    return {k: to_np(v).copy() if isinstance(v, torch.Tensor) else v
            for k, v in runner.result().items()}


@pytest.mark.parametrize("schedule", [L.SVT_SCHEDULE_ONEPASS, L.SVT_SCHEDULE_TILES])
@pytest.mark.parametrize("kept_only", [False, True])
def test_static_workspace_matches_workspace_entry_point(two_batches, bank, schedule, kept_only):
    _, words0, ref0 = two_batches[0]
    wc, rc, cc = caps_for(words0, ref0)
    tune = L.make_tune(schedule=schedule)
    d_bank = P.device_bank(bank.f, bank.q)

    def runner(static):
        return P.BatchRunner(gpu_cfg(CFG), d_bank, wc, rc, cc, kept_cap=cc, tune=tune,
                             graph=False, kept_only=kept_only, static_workspace=static)

    with_ws, static = runner(False), runner(True)
    assert static.work is None
    for name, words, ref in two_batches:
        where = f"{name} schedule={schedule} kept_only={kept_only}"
        print(f"[no-alloc] {where}: {len(words)} words", flush=True)
        w = P.words_tensor(words)
        for r in (with_ws, static):
            r.load(w, len(words)).run()
        a, b = outputs(with_ws), outputs(static)
        keys = [k for k in BATCH_KEYS if not (kept_only and k in ("p0", "p1", "p2", "chi2"))]
        compare(ref, b, keys, f"static {where}")
        assert a.keys() == b.keys()
        for k in a:
            if isinstance(a[k], np.ndarray):
                assert a[k].shape == b[k].shape and np.array_equal(a[k], b[k]), f"{where}: {k}"
            else:
                assert a[k] == b[k], f"{where}: {k}"


@pytest.mark.parametrize("schedule", [L.SVT_SCHEDULE_ONEPASS, L.SVT_SCHEDULE_TILES])
def test_static_entry_point_inside_a_callers_graph(two_batches, bank, schedule):
    """The case the entry point is for: a caller captures svt_process_batch_static into a graph
    of its own (no allocation can happen under capture) and replays it.  Between replays the
    caller loads another batch (words and device word count, eager work on its own stream); every
    replay must equal the oracle for the batch then loaded."""
    _, words0, ref0 = two_batches[0]
    wc, rc, cc = caps_for(words0, ref0)
    d_bank = P.device_bank(bank.f, bank.q)
    r = P.BatchRunner(gpu_cfg(CFG), d_bank, wc, rc, cc, kept_cap=cc,
                      tune=L.make_tune(schedule=schedule), graph=False, static_workspace=True)
    r.load(P.words_tensor(words0), len(words0)).run()  # eager first call: the device's address
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=r.stream):
        L.check(r._call(r.words, 0, r.stream), "svt_process_batch_static under capture")
    torch.cuda.synchronize()
    order = [two_batches[1], two_batches[0], two_batches[1]]
    for i, (name, words, ref) in enumerate(order):
        print(f"[no-alloc] replay {i}: {name}, schedule={schedule}", flush=True)
        r.load(P.words_tensor(words), len(words))
        torch.cuda.synchronize()
        with torch.cuda.stream(r.stream):
            g.replay()
        torch.cuda.synchronize()
        compare(ref, outputs(r), BATCH_KEYS, f"replay {i} {name} schedule={schedule}")
    del g

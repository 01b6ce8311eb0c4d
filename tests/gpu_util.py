"""Helpers of the GPU parity tests: run both GPU paths and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1312_0917_amd import _lib as L
from paper_1312_0917_amd import pipeline as P

# oracle output name -> GPU result name
NAME = {
    "road_event": "road_event", "road_set": "road_set", "road_hit_begin": "road_hit_begin",
    "road_nhits": "road_nhits", "road_combo_begin": "road_combo_begin",
    "road_ncombo": "road_ncombo", "hit_coord": "hit_coord", "combo_road": "combo_road",
    "combo_hits": "combo_hits", "p0": "p0", "p1": "p1", "p2": "p2", "c0": "c0", "c1": "c1",
    "c2": "c2", "chi2": "chi2", "accept": "accept", "kept": "kept",
    "best_nacc": "best_n_accept", "best_k": "best_k", "best_p0": "best_p0",
    "best_p1": "best_p1", "best_p2": "best_p2", "best_chi2": "best_chi2",
}
PLAIN_KEYS = list(NAME)
BATCH_KEYS = [k for k in NAME if k not in ("hit_coord", "combo_road", "combo_hits")]


def to_np(x):
    if isinstance(x, torch.Tensor):
        return x.detach().cpu().numpy()
    return np.asarray(x)


def as_u64(a):
    a = np.asarray(a)
    return a.astype(np.int64).view(np.uint64) if a.dtype.kind == "i" else a.astype(np.uint64)


def compare(ref: dict, got: dict, keys, where=""):
    """Bit-exact comparison of every listed output (integers, so tolerance 0)."""
    assert got["n_roads"] == ref["n_roads"], f"{where}: n_roads {got['n_roads']} vs {ref['n_roads']}"
    assert got["n_combos"] == ref["n_combos"], f"{where}: n_combos"
    for k in keys:
        if got.get(NAME[k]) is None:
            continue
        a = np.asarray(ref[k]).astype(np.int64)
        b = to_np(got[NAME[k]]).astype(np.int64)
        if k in ("road_nhits", "combo_hits"):
            a = a & 0xFFFFFFFF
            b = b & 0xFFFFFFFF
        assert a.shape == b.shape, f"{where}: {k} shape {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{where}: {k} differs at {bad.size} places, first {bad[:5]}: "
                                 f"oracle {a[bad[:5]]} gpu {b[bad[:5]]}")


def gpu_cfg(cfg: dict) -> L.svt_config:
    return L.make_config(chi2_cut=cfg["chi2_cut"], shift=cfg["shift"], max_hits=cfg["max_hits"],
                         n_sets=cfg["n_sets"], n_layers=cfg["n_layers"])


def run_plain(words, f, q, cfg):
    bank = P.device_bank(f, q)
    w = P.words_tensor(words)
    r = P.PlainRunner(gpu_cfg(cfg), bank).run(w)
    return r.result()


def caps_for(words, ref, slack=1.0):
    nw = max(len(words), 1)
    return (nw, max(int(ref["n_roads"] * slack) + 1, 1), max(int(ref["n_combos"] * slack) + 4, 4))


def run_batch(words, f, q, cfg, ref=None, tune=None, graph=True, kept=True, runner=None):
    bank = P.device_bank(f, q)
    if runner is None:
        if ref is None:
            st, nr, ne, nc, _ = oracle.count(words, cfg)
            ref = dict(n_roads=nr, n_combos=nc)
        wc, rc, cc = caps_for(words, ref)
        runner = P.BatchRunner(gpu_cfg(cfg), bank, wc, rc, cc, kept_cap=cc if kept else 0,
                               tune=tune, graph=graph)
    runner.load(P.words_tensor(words) if len(words) else torch.zeros(1, dtype=torch.int32,
                                                                    device="cuda"),
                len(words))
    runner.run()
    return runner.result(), runner

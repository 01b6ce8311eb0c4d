"""ctypes front-end of the CPU oracle (``svt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the benchmark's CPU
baseline leg, never by the product package.  Inputs are plain numpy arrays; nothing here
imports the HIP binding or the input generator.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "svt_oracle.c")
LIB = os.path.join(HERE, "libsvt_oracle.so")

OK, ERR_ARG, ERR_LAYER, ERR_HITS, ERR_SET = 0, -1, -2, -3, -6


def build() -> str:
    """Compile the oracle with the host C compiler (plain -O2, no target-specific flags)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB, SRC]
    subprocess.run(cmd, check=True)
    return LIB


class _Config(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("shift", ctypes.c_int32),
                ("chi2_cut", ctypes.c_int64), ("max_hits", ctypes.c_int32),
                ("n_sets", ctypes.c_int32)]


_P = ctypes.c_void_p
_OUT_FIELDS = ["road_event", "road_set", "road_hit_begin", "road_nhits", "road_combo_begin",
               "road_ncombo", "hit_coord", "combo_road", "combo_hits", "p0", "p1", "p2",
               "c0", "c1", "c2", "chi2", "accept", "best_nacc", "best_k", "best_p0",
               "best_p1", "best_p2", "best_chi2", "kept"]


class _Out(ctypes.Structure):
    _fields_ = [(n, _P) for n in _OUT_FIELDS]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        lib.ora_count.restype = ctypes.c_int32
        lib.ora_count.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(_Config),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        lib.ora_run.restype = ctypes.c_int32
        lib.ora_run.argtypes = [_P, ctypes.c_int64, _P, _P, ctypes.POINTER(_Config),
                                ctypes.POINTER(_Out), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


def make_config(chi2_cut=256, shift=10, max_hits=8, n_sets=256, n_layers=5) -> dict:
    return dict(n_layers=n_layers, shift=shift, chi2_cut=chi2_cut, max_hits=max_hits,
                n_sets=n_sets)


def _cfg(cfg: dict) -> _Config:
    return _Config(cfg["n_layers"], cfg["shift"], cfg["chi2_cut"], cfg["max_hits"],
                   cfg["n_sets"])


class OracleError(RuntimeError):
    def __init__(self, status, index):
        super().__init__(f"oracle status {status} at index {index}")
        self.status = status
        self.index = index


def count(words: np.ndarray, cfg: dict):
    """(status, n_roads, n_events, n_combos, err_index)."""
    lib = _load()
    w = np.ascontiguousarray(words, dtype=np.uint32)
    nr, ne, nc, ei = (ctypes.c_int64() for _ in range(4))
    c = _cfg(cfg)
    st = lib.ora_count(w.ctypes.data if w.size else None, w.size, ctypes.byref(c),
                       ctypes.byref(nr), ctypes.byref(ne), ctypes.byref(nc), ctypes.byref(ei))
    return st, nr.value, ne.value, nc.value, ei.value


def run(words: np.ndarray, f: np.ndarray, q: np.ndarray, cfg: dict,
        combos: bool = True, raise_on_error: bool = True) -> dict:
    """Run the whole path on the CPU; returns every output as numpy arrays.

    ``combos=False`` skips the per-combination arrays (road table and best tracks only).
    On an input error, raises ``OracleError`` (or returns {"status", "err_index"}).
    """
    lib = _load()
    w = np.ascontiguousarray(words, dtype=np.uint32)
    f = np.ascontiguousarray(f, dtype=np.int16)
    q = np.ascontiguousarray(q, dtype=np.int32)
    assert f.shape[1:] == (6, 5) and q.shape[1:] == (6,) and f.shape[0] == q.shape[0]
    st, nr, ne, nc, ei = count(w, cfg)
    if st != OK:
        if raise_on_error:
            raise OracleError(st, ei)
        return dict(status=st, err_index=ei)
    res = dict(
        road_event=np.zeros(nr, np.int32), road_set=np.zeros(nr, np.int32),
        road_hit_begin=np.zeros(nr, np.int64), road_nhits=np.zeros(nr, np.uint32),
        road_combo_begin=np.zeros(nr, np.int64), road_ncombo=np.zeros(nr, np.int32),
        hit_coord=np.zeros(w.size, np.int16),
        best_nacc=np.zeros(nr, np.int32), best_k=np.zeros(nr, np.int32),
        best_p0=np.zeros(nr, np.int32), best_p1=np.zeros(nr, np.int32),
        best_p2=np.zeros(nr, np.int32), best_chi2=np.zeros(nr, np.int64),
    )
    if combos:
        res.update(
            combo_road=np.zeros(nc, np.int32), combo_hits=np.zeros(nc, np.uint32),
            p0=np.zeros(nc, np.int32), p1=np.zeros(nc, np.int32), p2=np.zeros(nc, np.int32),
            c0=np.zeros(nc, np.int32), c1=np.zeros(nc, np.int32), c2=np.zeros(nc, np.int32),
            chi2=np.zeros(nc, np.int64), accept=np.zeros(nc, np.uint8),
            kept=np.zeros(nc, np.int64))
    out = _Out(**{k: (res[k].ctypes.data if (k in res and res[k].size) else None)
                  for k in _OUT_FIELDS})
    nk = ctypes.c_int64()
    eidx = ctypes.c_int64()
    c = _cfg(cfg)
    st = lib.ora_run(w.ctypes.data if w.size else None, w.size, f.ctypes.data, q.ctypes.data,
                     ctypes.byref(c), ctypes.byref(out), ctypes.byref(nk), ctypes.byref(eidx))
    if st != OK:
        if raise_on_error:
            raise OracleError(st, eidx.value)
        return dict(status=st, err_index=eidx.value)
    if combos:
        res["kept"] = res["kept"][:nk.value]
    res.update(status=OK, n_roads=nr, n_events=ne, n_combos=nc, n_kept=nk.value)
    return res


def time_run(words, f, q, cfg, min_seconds: float = 10.0, max_reps: int = 1000):
    """Wall time of full oracle runs (all outputs), repeated until ``min_seconds`` pass.

    Returns (seconds_per_run, reps, n_combos).  Single thread: the oracle has no threading.
    """
    run(words, f, q, cfg)  # warm-up and sizing
    reps = 0
    t0 = time.perf_counter()
    nc = 0
    while True:
        r = run(words, f, q, cfg)
        nc = r["n_combos"]
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or reps >= max_reps:
            return el / reps, reps, nc

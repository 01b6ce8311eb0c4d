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


# -O3 for a portable x86-64 level: the library is built on one machine and may run on another
# host CPU, so no -march=native here (build_native() makes that variant on the timing host).
CFLAGS = ["-O3", "-march=x86-64-v3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(out: str = LIB, native: bool = False) -> str:
    """Compile the oracle with the host C compiler (no intrinsics; -O3)."""
    flags = [f if f != "-march=x86-64-v3" else "-march=native" for f in CFLAGS] if native \
        else CFLAGS
    subprocess.run(["gcc", *flags, "-o", out, SRC], check=True)
    return out


def build_native(out: str) -> str:
    """The same source compiled with -O3 -march=native on the host that will run it (for the
    benchmark's CPU baseline).  Returns the library path."""
    return build(out, native=True)


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


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (before any other call)."""
    global _lib
    _lib = _bind(ctypes.CDLL(path))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _bind(lib):
    lib.ora_count.restype = ctypes.c_int32
    lib.ora_count.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(_Config),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.ora_run.restype = ctypes.c_int32
    lib.ora_run.argtypes = [_P, ctypes.c_int64, _P, _P, ctypes.POINTER(_Config),
                            ctypes.POINTER(_Out), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int64)]
    return lib


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


ALL_FIELDS = tuple(_OUT_FIELDS)


def run(words: np.ndarray, f: np.ndarray, q: np.ndarray, cfg: dict,
        combos: bool = True, raise_on_error: bool = True, fields=None) -> dict:
    """Run the whole path on the CPU; returns every output as numpy arrays.

    ``combos=False`` skips the per-combination arrays (road table and best tracks only).
    ``fields``: when given, only these outputs are produced (the oracle skips the others).
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
    if fields is not None:
        res = {k: v for k, v in res.items() if k in fields}
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
    if "kept" in res:
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


def run_event_ranges(words: np.ndarray, event_word_begin: np.ndarray, f: np.ndarray,
                     q: np.ndarray, cfg: dict, chunks, threads: int = 1, fields=None,
                     consume=None):
    """Run the oracle on several event ranges of one stream at once (the per-event parallel
    scheme of the paper's many-core port: events are independent).

    ``chunks`` is a list of (e0, e1) event ranges; range c runs on words
    event_word_begin[e0] .. event_word_begin[e1] as its own stream, so its road and
    combination numbers start at 0.  With ``consume(c, result)`` each result is handed over
    as soon as it exists (in the worker thread) and not kept; otherwise the results are
    returned in order.  The oracle's C code holds no state, and ctypes releases the
    interpreter lock during a call, so ``threads`` ranges really run at once.
    """
    import concurrent.futures as cf

    def one(c):
        e0, e1 = chunks[c]
        w = words[event_word_begin[e0]:event_word_begin[e1]]
        r = run(w, f, q, cfg, fields=fields)
        if consume is not None:
            consume(c, r)
            return None
        return r

    if threads <= 1:
        return [one(c) for c in range(len(chunks))]
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(len(chunks))))


def time_event_ranges(words, event_word_begin, f, q, cfg, threads: int, min_seconds=10.0,
                      fields=None):
    """Wall time of the whole stream run as ``threads`` event ranges on ``threads`` threads at
    once, repeated until ``min_seconds`` pass.  Returns (seconds_per_run, reps, n_combos)."""
    n_ev = len(event_word_begin) - 1
    edges = np.linspace(0, n_ev, 4 * threads + 1).round().astype(np.int64)
    chunks = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]
    keep = ("p0",) if fields is None else fields
    run_event_ranges(words, event_word_begin, f, q, cfg, chunks, threads, fields=keep)
    reps, nc = 0, 0
    t0 = time.perf_counter()
    while True:
        res = run_event_ranges(words, event_word_begin, f, q, cfg, chunks, threads, fields=fields)
        nc = sum(r["n_combos"] for r in res)
        del res
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            return el / reps, reps, nc

"""ctypes binding of libsvt.so: the C-ABI entry points under the same names.

Argument marshalling only -- every step of the path runs in the HIP kernels of libsvt.so.
Tensors must be CUDA (HIP) tensors; streams are ``torch.cuda.Stream`` objects or raw handles.
Loading fails loudly when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsvt.so")

SVT_OK, SVT_ERR_ARG, SVT_ERR_LAYER, SVT_ERR_HITS = 0, -1, -2, -3
SVT_ERR_CAPACITY, SVT_ERR_HIP, SVT_ERR_SET = -4, -5, -6
SVT_NO_ERROR = (1 << 64) - 1
SVT_BATCH_GRAPH = 1
SVT_BATCH_KEPT_ONLY = 2
SVT_SCHEDULE_EVENTS = 1   # one event per workgroup (ablation)
SVT_SCHEDULE_ONEPASS = 2  # one persistent kernel per pass (plus a reset)
SVT_SCHEDULE_TILES = 3    # pre-pass, persistent kernel over flat tiles, finalize
SVT_COPY_H2D = 1
SVT_COPY_D2H = 2

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


class svt_config(ctypes.Structure):
    _fields_ = [("n_layers", _I32), ("shift", _I32), ("chi2_cut", _I64), ("max_hits", _I32),
                ("n_sets", _I32)]


class svt_roads(ctypes.Structure):
    _fields_ = [(n, _P) for n in ("event", "set", "hit_begin", "nhits", "combo_begin", "ncombo")]


class svt_fitrec(ctypes.Structure):
    _fields_ = [(n, _P) for n in ("p0", "p1", "p2", "chi2", "c0", "c1", "c2")]


class svt_best(ctypes.Structure):
    _fields_ = [(n, _P) for n in ("n_accept", "k", "p0", "p1", "p2", "chi2")]


class svt_tune(ctypes.Structure):
    _fields_ = [("tile_combos", _I32), ("chunk_roads", _I32), ("wg_size", _I32),
                ("wgs_per_cu", _I32), ("schedule", _I32)]


class LibraryMissing(RuntimeError):
    pass


_lib = None


def load():
    """Load libsvt.so (built by ``__graft_entry__.build()`` / ``paper_1312_0917_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run `python -m paper_1312_0917_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.POINTER
    sig = {
        "svt_abi_version": (_I32, []),
        "svt_status_name": (ctypes.c_char_p, [_I32]),
        "svt_error_decode": (_I32, [ctypes.c_uint64, S(_I64)]),
        "svt_unpack_workspace": (_I64, [_I64]),
        "svt_combine_workspace": (_I64, [_I64]),
        "svt_select_workspace": (_I64, [_I64]),
        "svt_batch_workspace": (_I64, [_I64, _I64, _I64, S(svt_tune)]),
        "svt_unpack": (_I32, [_P, _I64, S(svt_config), S(svt_roads), _I64, _P, _P, _P, _P, _I64,
                              _P]),
        "svt_combine": (_I32, [S(svt_roads), _I64, S(svt_config), _P, _P, _I64, _P, _P, _P, _I64,
                               _P]),
        "svt_fit": (_I32, [_P, S(svt_config), S(svt_roads), _I64, _P, _I64, _P, _P, _I64,
                           S(svt_fitrec), _P, _P]),
        "svt_select": (_I32, [S(svt_config), S(svt_roads), _I64, _P, S(svt_fitrec), _I64, _P,
                              S(svt_best), _P, _I64, _P, _P, _P, _I64, _P]),
        "svt_process_batch": (_I32, [_P, S(svt_config), S(svt_tune), _P, _P, _I64, S(svt_roads),
                                     _I64, S(svt_fitrec), _P, _I64, S(svt_best), _P, _I64, _P,
                                     _P, _P, _P, _P, _I64, _I32, _P]),
        "svt_process_batch_static": (_I32, [_P, S(svt_config), S(svt_tune), _P, _P, _I64,
                                            S(svt_roads), _I64, S(svt_fitrec), _P, _I64,
                                            S(svt_best), _P, _I64, _P, _P, _P, _P, _I32, _P]),
        "svt_static_workspace_need": (_I32, [_I64, _I64, _I64, S(svt_tune), S(_I64), S(_I64)]),
        "svt_set_fused_timing_events": (None, [_P, _P]),
        "svt_release_graphs": (None, []),
        "svt_tune_resolve": (_I32, [S(svt_tune), S(svt_tune)]),
        "svt_tune_for_batch": (_I32, [S(svt_tune), _I64, S(svt_tune)]),
        "svt_mapped_pointer": (_I32, [_P, S(_P)]),
        "svt_copy_async": (_I32, [_P, _P, _I64, _I32, _P]),
        "svt_event_record": (_I32, [_P, _P]),
        "svt_event_done": (_I32, [_P]),
        "svt_gather_results": (_I32, [S(svt_roads), S(svt_best), _I64, _P, _P, _P, _P, _P, _P,
                                      _I64, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["svt_abi_version", "svt_status_name", "svt_error_decode", "svt_unpack_workspace",
            "svt_combine_workspace", "svt_select_workspace", "svt_batch_workspace", "svt_unpack",
            "svt_combine", "svt_fit", "svt_select", "svt_process_batch",
            "svt_process_batch_static", "svt_static_workspace_need",
            "svt_set_fused_timing_events", "svt_release_graphs", "svt_tune_resolve",
            "svt_tune_for_batch",
            "svt_mapped_pointer", "svt_copy_async", "svt_event_record", "svt_event_done",
            "svt_gather_results"]


# ---- marshalling helpers -----------------------------------------------------------------
def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def make_config(chi2_cut=256, shift=10, max_hits=8, n_sets=256, n_layers=5) -> svt_config:
    return svt_config(n_layers, shift, chi2_cut, max_hits, n_sets)


def make_tune(tile_combos=0, chunk_roads=0, wg_size=0, wgs_per_cu=0, schedule=0) -> svt_tune:
    return svt_tune(tile_combos, chunk_roads, wg_size, wgs_per_cu, schedule)


def svt_tune_resolve(tune=None) -> svt_tune:
    """Launch parameters svt_process_batch uses for ``tune`` (defaults filled in)."""
    out = svt_tune()
    check(load().svt_tune_resolve(ctypes.byref(tune) if tune is not None else None,
                                  ctypes.byref(out)), "svt_tune_resolve")
    return out


def svt_tune_for_batch(tune, word_cap) -> svt_tune:
    """Launch parameters svt_process_batch uses for ``tune`` at word capacity ``word_cap``
    (a zero schedule becomes the one chosen for that capacity)."""
    out = svt_tune()
    check(load().svt_tune_for_batch(ctypes.byref(tune) if tune is not None else None, word_cap,
                                    ctypes.byref(out)), "svt_tune_for_batch")
    return out


def roads_struct(d) -> svt_roads:
    return svt_roads(*[_ptr(d.get(k)) for k in ("event", "set", "hit_begin", "nhits",
                                                "combo_begin", "ncombo")])


def fitrec_struct(d) -> svt_fitrec:
    return svt_fitrec(*[_ptr(d.get(k)) for k in ("p0", "p1", "p2", "chi2", "c0", "c1", "c2")])


def best_struct(d) -> svt_best:
    return svt_best(*[_ptr(d.get(k)) for k in ("n_accept", "k", "p0", "p1", "p2", "chi2")])


def pack_bank(f: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Pack int16 f[S,6,5] and int32 q[S,6] into the 88-byte svt_fconst records (uint8)."""
    f = np.ascontiguousarray(f, dtype=np.int16)
    q = np.ascontiguousarray(q, dtype=np.int32)
    S = f.shape[0]
    rec = np.zeros((S, 88), dtype=np.uint8)
    rec[:, :60] = f.reshape(S, 30).view(np.uint8)
    rec[:, 64:88] = q.reshape(S, 6).view(np.uint8)
    return rec


def status_name(st: int) -> str:
    return load().svt_status_name(st).decode()


def error_decode(err: int):
    idx = _I64()
    st = load().svt_error_decode(ctypes.c_uint64(err & SVT_NO_ERROR), ctypes.byref(idx))
    return st, idx.value


class SvtError(RuntimeError):
    def __init__(self, status, where, index=-1):
        super().__init__(f"{where}: {status_name(status)} (index {index})")
        self.status = status
        self.index = index


def check(st: int, where: str):
    if st != SVT_OK:
        raise SvtError(st, where)


# ---- entry points (same names as the C ABI) ---------------------------------------------
def svt_unpack_workspace(n_words): return load().svt_unpack_workspace(n_words)
def svt_combine_workspace(n_roads): return load().svt_combine_workspace(n_roads)
def svt_select_workspace(n_combos): return load().svt_select_workspace(n_combos)


def svt_batch_workspace(word_cap, road_cap, combo_cap, tune=None):
    t = tune if tune is not None else make_tune()
    return load().svt_batch_workspace(word_cap, road_cap, combo_cap, ctypes.byref(t))


def svt_unpack(words, n_words, cfg, roads, road_cap, hit_coord, d_n_roads, d_err, work,
               stream=None):
    r = roads_struct(roads)
    return load().svt_unpack(_ptr(words), n_words, ctypes.byref(cfg), ctypes.byref(r), road_cap,
                             _ptr(hit_coord), _ptr(d_n_roads), _ptr(d_err), _ptr(work),
                             work.numel() * work.element_size(), _stream(stream))


def svt_combine(roads, n_roads, cfg, combo_road, combo_hits, combo_cap, d_n_combos, d_err, work,
                stream=None):
    r = roads_struct(roads)
    return load().svt_combine(ctypes.byref(r), n_roads, ctypes.byref(cfg), _ptr(combo_road),
                              _ptr(combo_hits), combo_cap, _ptr(d_n_combos), _ptr(d_err),
                              _ptr(work), work.numel() * work.element_size(), _stream(stream))


def svt_fit(bank, cfg, roads, n_roads, hit_coord, n_hits, combo_road, combo_hits, n_combos, out,
            d_err, stream=None):
    r = roads_struct(roads)
    o = fitrec_struct(out)
    return load().svt_fit(_ptr(bank), ctypes.byref(cfg), ctypes.byref(r), n_roads,
                          _ptr(hit_coord), n_hits, _ptr(combo_road), _ptr(combo_hits), n_combos,
                          ctypes.byref(o), _ptr(d_err), _stream(stream))


def svt_select(cfg, roads, n_roads, combo_road, rec, n_combos, accept, best, kept, kept_cap,
               d_n_kept, d_err, work, stream=None):
    r = roads_struct(roads)
    rc = fitrec_struct(rec)
    b = best_struct(best)
    return load().svt_select(ctypes.byref(cfg), ctypes.byref(r), n_roads, _ptr(combo_road),
                             ctypes.byref(rc), n_combos, _ptr(accept), ctypes.byref(b),
                             _ptr(kept), kept_cap, _ptr(d_n_kept), _ptr(d_err), _ptr(work),
                             work.numel() * work.element_size(), _stream(stream))


def svt_process_batch(bank, cfg, tune, words, d_n_words, word_cap, roads, road_cap, rec, accept,
                      combo_cap, best, kept, kept_cap, d_n_roads, d_n_combos, d_n_kept, d_err,
                      work, flags=0, stream=None):
    r = roads_struct(roads)
    rc = fitrec_struct(rec)
    b = best_struct(best)
    t = tune if tune is not None else make_tune()
    return load().svt_process_batch(_ptr(bank), ctypes.byref(cfg), ctypes.byref(t), _ptr(words),
                                    _ptr(d_n_words), word_cap, ctypes.byref(r), road_cap,
                                    ctypes.byref(rc), _ptr(accept), combo_cap, ctypes.byref(b),
                                    _ptr(kept), kept_cap, _ptr(d_n_roads), _ptr(d_n_combos),
                                    _ptr(d_n_kept), _ptr(d_err), _ptr(work),
                                    work.numel() * work.element_size(), flags, _stream(stream))


def svt_static_workspace_need(word_cap, road_cap, combo_cap, tune=None):
    """(status, workspace bytes these capacities take, bytes of the static workspace)."""
    t = tune if tune is not None else make_tune()
    need, limit = _I64(0), _I64(0)
    st = load().svt_static_workspace_need(word_cap, road_cap, combo_cap, ctypes.byref(t),
                                          ctypes.byref(need), ctypes.byref(limit))
    return st, need.value, limit.value


class PreparedBatch:
    """The argument list of svt_process_batch built once for a fixed set of buffers, so that a
    host loop pays one foreign call per batch (words, flags and stream may change per call)."""

    def __init__(self, bank, cfg, tune, d_n_words, word_cap, roads, road_cap, rec, accept,
                 combo_cap, best, kept, kept_cap, d_n_roads, d_n_combos, d_n_kept, d_err, work):
        """``work`` None: call svt_process_batch_static (the library's static workspace)."""
        self._keep = (roads_struct(roads), fitrec_struct(rec), best_struct(best), cfg,
                      tune if tune is not None else make_tune())
        r, rc, b, c, t = self._keep
        self._head = (_ptr(bank), ctypes.byref(c), ctypes.byref(t))
        self._tail = (_ptr(d_n_words), word_cap, ctypes.byref(r), road_cap, ctypes.byref(rc),
                      _ptr(accept), combo_cap, ctypes.byref(b), _ptr(kept), kept_cap,
                      _ptr(d_n_roads), _ptr(d_n_combos), _ptr(d_n_kept), _ptr(d_err))
        if work is None:
            self._fn = load().svt_process_batch_static
        else:
            self._tail += (_ptr(work), work.numel() * work.element_size())
            self._fn = load().svt_process_batch

    def __call__(self, words, flags, stream) -> int:
        return self._fn(*self._head, _ptr(words), *self._tail, flags, _stream(stream))


GATHER_HEADER_BYTES = 64
GATHER_BYTES_PER_ROAD = 36


class PreparedGather:
    """svt_gather_results for a fixed set of buffers: the header and the first n_roads per-road
    results of a batch, written back to back into ``out`` (device memory, or the device address
    of page-locked host memory) with one foreign call per batch."""

    def __init__(self, roads, best, road_cap, d_n_words, d_n_roads, d_n_combos, d_n_kept, d_err,
                 out, out_roads):
        self._keep = (roads_struct(roads), best_struct(best))
        r, b = self._keep
        self._args = (ctypes.byref(r), ctypes.byref(b), road_cap, _ptr(d_n_words), _ptr(d_n_roads),
                      _ptr(d_n_combos), _ptr(d_n_kept), _ptr(d_err), _ptr(out), out_roads)
        self._fn = load().svt_gather_results

    def __call__(self, stream):
        check(self._fn(*self._args, _stream(stream)), "svt_gather_results")


def gathered(buf: np.ndarray):
    """Views into a buffer written by svt_gather_results (uint8 array, 8-byte aligned): the
    header dict and, when the per-road part was written, a dict of per-road arrays."""
    head = buf[:GATHER_HEADER_BYTES].view(np.int64)
    h = dict(n_words=int(head[0]), n_roads=int(head[1]), n_combos=int(head[2]),
             n_kept=int(head[3]), err=int(head[4]) & SVT_NO_ERROR)
    nr = h["n_roads"]
    cap = (len(buf) - GATHER_HEADER_BYTES) // GATHER_BYTES_PER_ROAD
    if not 0 <= nr <= cap:
        return h, None
    off = GATHER_HEADER_BYTES
    out = {"chi2": buf[off:off + 8 * nr].view(np.int64)}
    off += 8 * nr
    for k in ("n_accept", "k", "p0", "p1", "p2", "event", "set"):
        out[k] = buf[off:off + 4 * nr].view(np.int32)
        off += 4 * nr
    return h, out


def svt_set_fused_timing_events(start, stop):
    load().svt_set_fused_timing_events(start.cuda_event if start is not None else None,
                                       stop.cuda_event if stop is not None else None)


def svt_release_graphs():
    load().svt_release_graphs()


def svt_copy_async(dst, src, nbytes, kind, stream):
    check(load().svt_copy_async(_ptr(dst), _ptr(src), int(nbytes), kind, _stream(stream)),
          "svt_copy_async")


def svt_event_record(event, stream):
    """``event``: a torch.cuda.Event that has been recorded once (so that it exists)."""
    check(load().svt_event_record(event.cuda_event, _stream(stream)), "svt_event_record")


def svt_event_done(event) -> bool:
    r = load().svt_event_done(event.cuda_event)
    if r < 0:
        raise SvtError(r, "svt_event_done")
    return r == 1


def svt_mapped_pointer(host) -> int:
    """Device address of page-locked host memory (a pinned tensor or an address)."""
    dev = _P()
    check(load().svt_mapped_pointer(_ptr(host), ctypes.byref(dev)), "svt_mapped_pointer")
    return int(dev.value)

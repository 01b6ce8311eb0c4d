"""Device buffers and call sequences around the libsvt C ABI (torch = memory and streams only).

``PlainRunner`` drives the one-launch-per-stage path (svt_unpack -> svt_combine -> svt_fit ->
svt_select) with the host synchronisations it needs to size each stage, like the staged
kernels of the paper's GPU port.  ``BatchRunner`` keeps every buffer resident and runs the
fused persistent pass (svt_process_batch), optionally replayed from a captured HIP graph.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as L

I32, I64, U8 = torch.int32, torch.int64, torch.uint8


def device_bank(f: np.ndarray, q: np.ndarray, device="cuda") -> torch.Tensor:
    """The packed svt_fconst bank as a device byte tensor (kept resident by the caller)."""
    return torch.from_numpy(L.pack_bank(f, q).reshape(-1)).to(device)


def words_tensor(words: np.ndarray, device="cuda") -> torch.Tensor:
    """uint32 hit words as an int32 device tensor (same bits)."""
    return torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint32).view(np.int32)).to(device)


def _err_value(t: torch.Tensor) -> int:
    return int(t.item()) & L.SVT_NO_ERROR


class DeviceError(RuntimeError):
    def __init__(self, status, index, where):
        super().__init__(f"{where}: {L.status_name(status)} at index {index}")
        self.status = status
        self.index = index


def _alloc_roads(n, device):
    return dict(event=torch.empty(max(n, 1), dtype=I32, device=device),
                set=torch.empty(max(n, 1), dtype=I32, device=device),
                hit_begin=torch.empty(max(n, 1), dtype=I64, device=device),
                nhits=torch.empty(max(n, 1), dtype=I32, device=device),
                combo_begin=torch.empty(max(n, 1), dtype=I64, device=device),
                ncombo=torch.empty(max(n, 1), dtype=I32, device=device))


def _alloc_rec(n, device, with_c=True):
    d = dict(p0=torch.empty(max(n, 1), dtype=I32, device=device),
             p1=torch.empty(max(n, 1), dtype=I32, device=device),
             p2=torch.empty(max(n, 1), dtype=I32, device=device),
             chi2=torch.empty(max(n, 1), dtype=I64, device=device))
    if with_c:
        for k in ("c0", "c1", "c2"):
            d[k] = torch.empty(max(n, 1), dtype=I32, device=device)
    return d


def _alloc_best(n, device):
    return dict(n_accept=torch.empty(max(n, 1), dtype=I32, device=device),
                k=torch.empty(max(n, 1), dtype=I32, device=device),
                p0=torch.empty(max(n, 1), dtype=I32, device=device),
                p1=torch.empty(max(n, 1), dtype=I32, device=device),
                p2=torch.empty(max(n, 1), dtype=I32, device=device),
                chi2=torch.empty(max(n, 1), dtype=I64, device=device))


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=U8, device=device)


@dataclasses.dataclass
class StageTimes:
    unpack_ms: float = 0.0
    combine_ms: float = 0.0
    fit_ms: float = 0.0
    select_ms: float = 0.0


class PlainRunner:
    """svt_unpack -> sync -> svt_combine -> sync -> svt_fit -> svt_select."""

    def __init__(self, cfg: L.svt_config, bank: torch.Tensor, device="cuda", with_c=True,
                 want_kept=True):
        self.cfg, self.bank, self.device = cfg, bank, device
        self.with_c, self.want_kept = with_c, want_kept
        self.caps = dict(words=-1, roads=-1, combos=-1)
        self.d_n = torch.zeros(4, dtype=I64, device=device)  # roads, combos, kept
        self.d_err = torch.zeros(1, dtype=I64, device=device)
        self.stage_events = None

    def _grow(self, kind, n):
        if self.caps[kind] >= n:
            return
        cap = max(n, 1)
        d = self.device
        if kind == "words":
            self.hit_coord = torch.empty(cap, dtype=torch.int16, device=d)
            self.ws_unpack = _ws(L.svt_unpack_workspace(cap), d)
        elif kind == "roads":
            self.roads = _alloc_roads(cap, d)
            self.best = _alloc_best(cap, d)
            self.ws_combine = _ws(L.svt_combine_workspace(cap), d)
        else:
            self.combo_road = torch.empty(cap, dtype=I32, device=d)
            self.combo_hits = torch.empty(cap, dtype=I32, device=d)
            self.rec = _alloc_rec(cap, d, self.with_c)
            self.accept = torch.empty(cap, dtype=U8, device=d)
            self.kept = torch.empty(cap, dtype=I64, device=d)
            self.ws_select = _ws(L.svt_select_workspace(cap), d)
        self.caps[kind] = cap

    def _check(self, where):
        err = _err_value(self.d_err)
        if err != L.SVT_NO_ERROR:
            st, idx = L.error_decode(err)
            raise DeviceError(st, idx, where)

    def run(self, words: torch.Tensor, n_words: Optional[int] = None, timing=False):
        n_words = words.numel() if n_words is None else n_words
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if timing else None
        self._grow("words", n_words)
        # road count is at most the word count
        self._grow("roads", n_words)
        if ev: ev[0].record(st)
        L.check(L.svt_unpack(words, n_words, self.cfg, self.roads, self.caps["roads"],
                             self.hit_coord, self.d_n[0:1], self.d_err, self.ws_unpack), "svt_unpack")
        if ev: ev[1].record(st)
        n_roads = int(self.d_n[0].item())  # host sync: size of the next stage
        self._check("svt_unpack")
        while True:
            listing = self.caps["combos"] > 0
            L.check(L.svt_combine(self.roads, n_roads, self.cfg,
                                  self.combo_road if listing else None,
                                  self.combo_hits if listing else None,
                                  max(self.caps["combos"], 0), self.d_n[1:2], self.d_err,
                                  self.ws_combine), "svt_combine")
            n_combos = int(self.d_n[1].item())  # host sync: size of the next stage
            if listing and n_combos <= self.caps["combos"]:
                break
            # first run or a larger input: grow the lists and list again
            self._grow("combos", n_combos)
            self.d_err.fill_(-1)
        self._check("svt_combine")
        if ev: ev[2].record(st)
        L.check(L.svt_fit(self.bank, self.cfg, self.roads, n_roads, self.hit_coord, n_words,
                          self.combo_road, self.combo_hits, n_combos, self.rec, self.d_err),
                "svt_fit")
        if ev: ev[3].record(st)
        L.check(L.svt_select(self.cfg, self.roads, n_roads, self.combo_road, self.rec, n_combos,
                             self.accept, self.best, self.kept if self.want_kept else None,
                             self.caps["combos"], self.d_n[2:3], self.d_err, self.ws_select),
                "svt_select")
        if ev: ev[4].record(st)
        self.n_roads, self.n_combos, self.n_words = n_roads, n_combos, n_words
        if ev:
            torch.cuda.synchronize()
            self.times = StageTimes(ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]),
                                    ev[2].elapsed_time(ev[3]), ev[3].elapsed_time(ev[4]))
        return self

    def result(self, check=True) -> dict:
        torch.cuda.synchronize()
        if check:
            self._check("svt_select")
        nr, nc = self.n_roads, self.n_combos
        nk = int(self.d_n[2].item())
        out = {f"road_{k}": v[:nr] for k, v in self.roads.items()}
        out["hit_coord"] = self.hit_coord[:self.n_words]
        out["combo_road"] = self.combo_road[:nc]
        out["combo_hits"] = self.combo_hits[:nc]
        out.update({k: v[:nc] for k, v in self.rec.items()})
        out["accept"] = self.accept[:nc]
        out.update({f"best_{k}": v[:nr] for k, v in self.best.items()})
        out["kept"] = self.kept[:nk] if self.want_kept else None
        out.update(n_roads=nr, n_combos=nc, n_kept=nk)
        return out


class BatchRunner:
    """Resident buffers + svt_process_batch (fused persistent kernel, optional HIP graph)."""

    def __init__(self, cfg: L.svt_config, bank: torch.Tensor, word_cap: int, road_cap: int,
                 combo_cap: int, kept_cap: int = 0, tune: Optional[L.svt_tune] = None,
                 graph=True, with_c=True, device="cuda", stream=None, kept_only=False,
                 n_words_ptr: Optional[int] = None, static_workspace=False):
        """``kept_only``: no per-combination records; ``rec`` then holds the fit values of the
        accepted combinations, compacted in the order of the kept list (needs kept_cap > 0).
        ``n_words_ptr``: device address the kernels read the word count from (for instance
        mapped host memory the caller writes), instead of the runner's own device word.
        ``static_workspace``: no workspace tensor; every pass goes through
        svt_process_batch_static (the library's per-GPU static workspace, no graph)."""
        if kept_only and kept_cap <= 0:
            raise ValueError("kept-only mode needs a kept list (kept_cap > 0)")
        self.kept_only = kept_only
        self.cfg, self.bank, self.device = cfg, bank, device
        self.tune = tune if tune is not None else L.make_tune()
        self.graph = graph
        self.word_cap, self.road_cap, self.combo_cap = word_cap, road_cap, combo_cap
        self.kept_cap = kept_cap
        # graphs cannot be captured on the legacy default stream: own a stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        d = device
        self.words = torch.zeros(max(word_cap, 1), dtype=I32, device=d)
        # words, roads, combos, kept, then the error word: one copy brings all five back
        self.d_state = torch.zeros(5, dtype=I64, device=d)
        self.d_n = self.d_state[0:4]
        self.d_err = self.d_state[4:5]
        self.roads = _alloc_roads(road_cap, d)
        self.rec = _alloc_rec(kept_cap if kept_only else combo_cap, d, with_c)
        self.accept = torch.empty(max(combo_cap, 4) + 4, dtype=U8, device=d)
        self.best = _alloc_best(road_cap, d)
        self.kept = torch.empty(max(kept_cap, 1), dtype=I64, device=d) if kept_cap > 0 else None
        if static_workspace:
            if graph:
                raise ValueError("the static workspace is for callers without graphs")
            st, need, limit = L.svt_static_workspace_need(word_cap, road_cap, combo_cap,
                                                          self.tune)
            if st != L.SVT_OK:
                raise ValueError(f"capacities need a {need}-byte workspace; the static one "
                                 f"holds {limit} bytes")
            self.work = None
        else:
            nbytes = L.svt_batch_workspace(word_cap, road_cap, combo_cap, self.tune)
            if nbytes < 0:
                raise ValueError("unsupported tune / capacities")
            self.work = _ws(nbytes, d)
        self._d_n_words = self.d_n[0:1] if n_words_ptr is None else n_words_ptr
        self._calls = {}
        self._call = self._prepared(self.word_cap)

    def _prepared(self, word_cap: int):
        """The prepared argument list for a word capacity up to the runner's own (a smaller one
        sizes the launch grids and look-back state to batches that fit it)."""
        call = self._calls.get(word_cap)
        if call is None:
            call = L.PreparedBatch(self.bank, self.cfg, self.tune, self._d_n_words, word_cap,
                                   self.roads, self.road_cap, self.rec, self.accept,
                                   self.combo_cap, self.best, self.kept, self.kept_cap,
                                   self.d_n[1:2], self.d_n[2:3],
                                   self.d_n[3:4] if self.kept_cap > 0 else None, self.d_err,
                                   self.work)
            self._calls[word_cap] = call
        return call

    def load(self, words: torch.Tensor, n_words: Optional[int] = None):
        """Copy a batch of words into the resident buffer and set the device word count."""
        n = words.numel() if n_words is None else n_words
        if n > self.word_cap:
            raise ValueError("batch larger than word_cap")
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            if n:
                self.words[:n].copy_(words[:n], non_blocking=True)
            self.d_n[0].fill_(n)
        self.n_words = n
        return self

    def set_word_count(self, n: int):
        """Words already resident in ``self.words``: only set the device word count."""
        with torch.cuda.stream(self.stream):
            self.d_n[0].fill_(n)
        self.n_words = n
        return self

    def run(self, stream=None, words=None, word_cap: Optional[int] = None):
        """One pass over the batch.  ``words``: another word buffer the kernels can read
        (a device tensor, or the device address of mapped host memory), default the
        resident one.  ``word_cap``: the capacity the pass is launched for (at least the
        batch's word count, at most the runner's; default the runner's): with graphs, each
        distinct value is one cached graph."""
        s = stream if stream is not None else self.stream
        src = self.words if words is None else words
        if word_cap is None or word_cap == self.word_cap:
            call = self._call
        elif 0 <= word_cap <= self.word_cap:
            call = self._prepared(int(word_cap))
        else:
            raise ValueError(f"word_cap {word_cap} outside 0..{self.word_cap}")
        st = call(src, (L.SVT_BATCH_GRAPH if self.graph else 0) |
                  (L.SVT_BATCH_KEPT_ONLY if self.kept_only else 0), s)
        L.check(st, "svt_process_batch" if self.work is not None else "svt_process_batch_static")
        return self

    def sizes(self):
        v = self.d_n.cpu().tolist()
        # the accepted count is only produced when a kept list is wanted
        return dict(n_words=v[0], n_roads=v[1], n_combos=v[2],
                    n_kept=v[3] if self.kept_cap > 0 else None)

    def error(self):
        err = _err_value(self.d_err)
        return L.error_decode(err) if err != L.SVT_NO_ERROR else (L.SVT_OK, -1)

    def result(self, check=True) -> dict:
        torch.cuda.synchronize()
        st, idx = self.error()
        if check and st != L.SVT_OK:
            raise DeviceError(st, idx, "svt_process_batch")
        sz = self.sizes()
        nr, nc, nk = sz["n_roads"], sz["n_combos"], sz["n_kept"]
        out = {f"road_{k}": v[:nr] for k, v in self.roads.items()}
        if self.kept_only:  # records of the kept combinations only, in kept-list order
            out.update({f"kept_{k}": v[:nk] for k, v in self.rec.items()})
        else:
            out.update({k: v[:nc] for k, v in self.rec.items()})
        out["accept"] = self.accept[:nc]
        out.update({f"best_{k}": v[:nr] for k, v in self.best.items()})
        out["kept"] = self.kept[:nk] if self.kept is not None else None
        out.update(n_roads=nr, n_combos=nc, n_kept=nk)
        return out

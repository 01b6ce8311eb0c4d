"""Seeded synthetic inputs for the SVT track fitter: fit-constant banks and hit-word streams.

This module only *draws* inputs. It holds none of the fitter's arithmetic (no dot products of
constants with hits, no shift, no chi-square): both the HIP path and the CPU oracle receive what
it produces, and neither is imported here.

What is being imitated (paper, section II and section IV):
  * events made of roads, roads made of silicon hits on 5 layers, one fit per one-hit-per-layer
    combination of a road;
  * the paper's benchmark sample has a fixed number of roads and combinations per event,
    2048 combinations per event, 1 to 3000 events (section IV, "Results");
  * the constants are "pre-defined constant sets" looked up per road (section II, equation
    p_i = f_i . x_i + q_i).  The real SVT constants and CDF data are not public, so a bank is
    *constructed* so that hits lying exactly on a track of the linear detector model fit back to
    the track parameters with zero chi-square components (see ``make_bank``).

Hit word layout (LSB first): coord int13 (two's complement) | layer 3 bits | road tag 8 bits |
event tag 8 bits.  Event tag = event ordinal mod 256.  Road tags are redrawn so that two adjacent
roads of one event never share a tag.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

N_LAYERS = 5
N_PARAMS = 3          # track parameters (rows 0-2 of a constant set)
N_CHI = 3             # chi-square components (rows 3-5)
N_SETS = 256          # one constant set per value of the 8-bit road tag
SHIFT = 10            # fixed-point scale of the constants: 2**10
COORD_MIN, COORD_MAX = -4096, 4095
EVENTS_PER_BLOCK = 256  # events drawn per independent child RNG stream


@dataclasses.dataclass
class Bank:
    """A bank of fit-constant sets plus the linear detector model each set was built from."""
    f: np.ndarray   # int16 [n_sets, 6, 5]; rows 0-2 parameters, rows 3-5 chi2 components
    q: np.ndarray   # int32 [n_sets, 6]; offsets in the f.x scale (2**SHIFT per unit)
    A: np.ndarray   # int64 [n_sets, 5, 3]; model: hits of a track t are A @ t + b
    b: np.ndarray   # int64 [n_sets, 5]


@dataclasses.dataclass
class Sample:
    """A packed hit-word stream plus the generator's own record of its structure."""
    words: np.ndarray            # uint32 [n_words]
    n_events: int
    road_event: np.ndarray       # int32 [n_roads] event ordinal
    road_set: np.ndarray         # int32 [n_roads] road tag (= constant set index)
    road_nhits: np.ndarray       # int32 [n_roads, 5] hits per layer
    road_word_begin: np.ndarray  # int64 [n_roads] index of the road's first word
    event_word_begin: np.ndarray  # int64 [n_events + 1]
    true_road: np.ndarray        # bool [n_roads] road carries one noise-free track
    true_t: np.ndarray           # int64 [n_roads, 3] its parameters (0 where none)
    true_slot: np.ndarray        # int32 [n_roads, 5] which hit of each layer is on the track

    @property
    def n_roads(self) -> int:
        return int(self.road_set.shape[0])

    def expected_combos(self) -> int:
        return int(np.prod(self.road_nhits.astype(np.int64), axis=1).sum())

    def event_slice(self, e0: int, e1: int) -> np.ndarray:
        """Words of events [e0, e1) (a batch cut at event boundaries)."""
        return self.words[self.event_word_begin[e0]:self.event_word_begin[e1]]


# --------------------------------------------------------------------------------------------
# Workload configurations (hit and road distributions of the five benchmark cases)
# --------------------------------------------------------------------------------------------
CONFIGS = {
    # 100 events x 8 roads, 1-2 hits per layer (<= 32 combinations per road)
    "c1": dict(n_events=100, roads=("fixed", 8), hits=("uniform", 1, 2), seed=0),
    # the paper's benchmark shape: 3000 events x 64 roads x 2**5 = 2048 combinations per event
    "c2": dict(n_events=3000, roads=("fixed", 64), hits=("uniform", 1, 3), seed=1),
    # uneven batch: roads/event geometric with mean 32 capped at 512; 8 hits w.p. 0.05 else 1-4
    "c3": dict(n_events=8192, roads=("geometric", 32, 512), hits=("tail", 1, 4, 8, 0.05), seed=2),
    # serving stream: 16-256 roads per event, 1-4 hits per layer (events drawn on demand)
    "c4": dict(n_events=4096, roads=("uniform", 16, 256), hits=("uniform", 1, 4), seed=3),
    # max scale: 10000 events x 2048 roads, 1-4 hits per layer (<= 1024 combinations per road)
    "c5": dict(n_events=10000, roads=("fixed", 2048), hits=("uniform", 1, 4), seed=4),
}
TRUE_ROAD_FRACTION = 0.2
DEFAULT_CHI2_CUT = 256
BANK_SEED = 20131104


def pack_words(coord, layer, rtag, etag) -> np.ndarray:
    """Pack hit fields into 32-bit words (coord is two's complement in the low 13 bits)."""
    coord = np.asarray(coord, dtype=np.int64)
    if coord.size and (coord.min() < COORD_MIN or coord.max() > COORD_MAX):
        raise ValueError("coordinate outside int13")
    w = (coord & 0x1FFF).astype(np.uint32)
    w |= (np.asarray(layer, dtype=np.uint32) & 7) << 13
    w |= (np.asarray(rtag, dtype=np.uint32) & 0xFF) << 16
    w |= (np.asarray(etag, dtype=np.uint32) & 0xFF) << 24
    return w


def unpack_fields(words: np.ndarray):
    """Field split used by the generator's own self-checks (coord, layer, rtag, etag)."""
    w = np.asarray(words, dtype=np.uint32).astype(np.int64)
    c = w & 0x1FFF
    c = np.where(c >= 4096, c - 8192, c)
    return c, (w >> 13) & 7, (w >> 16) & 0xFF, (w >> 24) & 0xFF


# --------------------------------------------------------------------------------------------
# Constant bank
# --------------------------------------------------------------------------------------------
def _rank2_int_matrix(rng, lo, hi):
    while True:
        W = rng.integers(lo, hi + 1, size=(3, 2))
        if np.linalg.matrix_rank(W.astype(np.float64)) == 2:
            return W


def make_bank(seed: int = BANK_SEED, n_sets: int = N_SETS) -> Bank:
    """Construct ``n_sets`` integer constant sets from a random linear detector model.

    For each set: a layer permutation P, M in [-4,4]^{2x3}, and the model A = P [I3; M]
    (hits x = A t + b for track parameters t).  With W in [-32,32]^{3x2} of rank 2,
    G = [-W M | W] P^T annihilates A (G A = 0).  With K in [-2,2]^{3x3},
    F = [1024 I3 | 0] P^T + K G satisfies F A = 1024 I3.  Offsets q = -F b + r_q and
    h = -G b + r_h with r in [0, 1023] make the fixed-point fit of a noise-free track exact:
    floor((F x + q) / 1024) = t and floor((G x + h) / 1024) = 0.
    """
    rng = np.random.default_rng(seed)
    f = np.zeros((n_sets, 6, N_LAYERS), dtype=np.int16)
    q = np.zeros((n_sets, 6), dtype=np.int32)
    A_all = np.zeros((n_sets, N_LAYERS, 3), dtype=np.int64)
    b_all = np.zeros((n_sets, N_LAYERS), dtype=np.int64)
    eye3 = np.eye(3, dtype=np.int64)
    for s in range(n_sets):
        perm = rng.permutation(N_LAYERS)
        P = np.zeros((N_LAYERS, N_LAYERS), dtype=np.int64)
        P[np.arange(N_LAYERS), perm] = 1
        M = rng.integers(-4, 5, size=(2, 3))
        A = P @ np.vstack([eye3, M])
        W = _rank2_int_matrix(rng, -32, 32)
        G = np.hstack([-W @ M, W]) @ P.T
        K = rng.integers(-2, 3, size=(3, 3))
        F = np.hstack([1024 * eye3, np.zeros((3, 2), dtype=np.int64)]) @ P.T + K @ G
        b = rng.integers(-512, 513, size=N_LAYERS)
        rq = rng.integers(0, 1024, size=3)
        rh = rng.integers(0, 1024, size=3)
        fs = np.vstack([F, G])
        qs = np.concatenate([-F @ b + rq, -G @ b + rh])
        assert np.all(np.abs(fs) <= 32767) and np.all(np.abs(qs) < 2**31)
        f[s] = fs
        q[s] = qs
        A_all[s] = A
        b_all[s] = b
    return Bank(f=f, q=q, A=A_all, b=b_all)


# --------------------------------------------------------------------------------------------
# Events
# --------------------------------------------------------------------------------------------
def _draw_roads_per_event(rng, spec, n):
    kind = spec[0]
    if kind == "fixed":
        return np.full(n, spec[1], dtype=np.int64)
    if kind == "uniform":
        return rng.integers(spec[1], spec[2] + 1, size=n)
    if kind == "geometric":
        mean, cap = spec[1], spec[2]
        return np.minimum(rng.geometric(1.0 / mean, size=n), cap).astype(np.int64)
    raise ValueError(kind)


def _draw_hits(rng, spec, n_roads):
    kind = spec[0]
    shape = (n_roads, N_LAYERS)
    if kind == "uniform":
        return rng.integers(spec[1], spec[2] + 1, size=shape)
    if kind == "tail":
        lo, hi, big, p = spec[1], spec[2], spec[3], spec[4]
        base = rng.integers(lo, hi + 1, size=shape)
        return np.where(rng.random(shape) < p, big, base)
    raise ValueError(kind)


def _segment_shuffle(rng, order, seg_begin, seg_len):
    """Uniform random permutation of ``order`` inside each segment (vectorised Fisher-Yates)."""
    max_len = int(seg_len.max()) if seg_len.size else 0
    for i in range(max_len - 1, 0, -1):
        sel = np.nonzero(seg_len > i)[0]
        if sel.size == 0:
            continue
        j = (rng.random(sel.size) * (i + 1)).astype(np.int64)
        a = seg_begin[sel] + i
        bpos = seg_begin[sel] + j
        tmp = order[a].copy()
        order[a] = order[bpos]
        order[bpos] = tmp


def _draw_block(rng, bank: Bank, n_ev: int, ev0: int, roads_spec, hits_spec, true_frac,
                layer_major: bool):
    rpe = _draw_roads_per_event(rng, roads_spec, n_ev)
    n_roads = int(rpe.sum())
    road_event = np.repeat(np.arange(ev0, ev0 + n_ev, dtype=np.int64), rpe)
    first_of_event = np.zeros(n_roads, dtype=bool)
    if n_roads:
        first_of_event[np.concatenate([[0], np.cumsum(rpe)[:-1]])[rpe > 0]] = True
    # road tags: first road of an event uniform, then a uniform non-zero step mod 256, which
    # is the same law as "redraw until different from the previous road's tag"
    step = rng.integers(1, 256, size=n_roads)
    start = rng.integers(0, 256, size=n_roads)
    incr = np.where(first_of_event, 0, step)
    grp = np.cumsum(first_of_event) - 1
    csum = np.cumsum(incr)
    base_at_first = csum[first_of_event]
    rtag = (start[first_of_event][grp] + csum - base_at_first[grp]) % 256

    nh = _draw_hits(rng, hits_spec, n_roads).astype(np.int64)
    road_len = nh.sum(axis=1)
    road_begin = np.zeros(n_roads, dtype=np.int64)
    if n_roads:
        road_begin[1:] = np.cumsum(road_len)[:-1]
    n_words = int(road_len.sum())

    # layer-major slot table: word j of road r in layer-major order has layer lay[j]
    lay = np.repeat(np.tile(np.arange(N_LAYERS), n_roads), nh.reshape(-1))
    coord = rng.integers(COORD_MIN, COORD_MAX + 1, size=n_words)

    # noise-free tracks in a fraction of the roads: one hit per layer replaced by A t + b
    true_road = rng.random(n_roads) < true_frac
    t = rng.integers(-256, 257, size=(n_roads, 3))
    slot = (rng.random((n_roads, N_LAYERS)) * nh).astype(np.int64)
    t = np.where(true_road[:, None], t, 0)
    slot = np.where(true_road[:, None], slot, 0)
    tr = np.nonzero(true_road)[0]
    if tr.size:
        s = rtag[tr]
        x = np.einsum("rlk,rk->rl", bank.A[s], t[tr]) + bank.b[s]
        layer_off = np.zeros((n_roads, N_LAYERS), dtype=np.int64)
        layer_off[:, 1:] = np.cumsum(nh, axis=1)[:, :-1]
        pos = road_begin[tr][:, None] + layer_off[tr] + slot[tr]
        coord[pos.reshape(-1)] = x.reshape(-1)

    # emission order inside each road: random interleaving of the layers (or layer-major)
    order = np.arange(n_words, dtype=np.int64)
    if not layer_major:
        _segment_shuffle(rng, order, road_begin, road_len)
        if tr.size:
            # rank of each track hit among its layer's hits in emission order
            inv = np.empty_like(order)
            inv[order] = np.arange(n_words, dtype=np.int64)
            hmax = int(nh.max())
            j = np.arange(hmax)
            lay_pos = (road_begin[tr][:, None, None] + layer_off[tr][:, :, None] + j)
            valid = j[None, None, :] < nh[tr][:, :, None]
            em = np.where(valid, inv[np.where(valid, lay_pos, 0)], np.iinfo(np.int64).max)
            mine = inv[pos][:, :, None]
            slot[tr] = (em < mine).sum(axis=2)
    road_idx = np.repeat(np.arange(n_roads), road_len)
    ev_of_word = road_event[road_idx]
    words = pack_words(coord[order], lay[order], rtag[road_idx], ev_of_word % 256)
    return dict(words=words, road_event=road_event, rtag=rtag, nh=nh, road_len=road_len,
                true_road=true_road, t=t, slot=slot, rpe=rpe)


def _draw_job(job, bank: Bank):
    seed, blk, ev0, n, roads, hits, true_frac, layer_major = job
    rng = np.random.default_rng([seed, blk])
    return _draw_block(rng, bank, n, ev0, roads, hits, true_frac, layer_major)


def make_sample(config: str | dict, seed: Optional[int] = None, n_events: Optional[int] = None,
                bank: Optional[Bank] = None, true_frac: float = TRUE_ROAD_FRACTION,
                layer_major: bool = False, workers: int = 1) -> Sample:
    """Draw one of the benchmark configurations (``"c1"`` ... ``"c5"``) or a custom dict.

    Events are drawn in blocks of 256 with child streams ``default_rng([seed, block])``, so a
    prefix of events does not depend on how many events follow it, nor on ``workers`` (blocks
    drawn by that many threads of this process: numpy's generators and array operations
    release the interpreter lock, and no child process is started, which matters in a
    process that already holds the GPU).
    """
    cfg = dict(CONFIGS[config]) if isinstance(config, str) else dict(config)
    seed = cfg["seed"] if seed is None else seed
    n_ev = cfg["n_events"] if n_events is None else n_events
    bank = make_bank() if bank is None else bank
    jobs = [(seed, blk, ev0, min(EVENTS_PER_BLOCK, n_ev - ev0), cfg["roads"], cfg["hits"],
             true_frac, layer_major) for blk, ev0 in enumerate(range(0, n_ev, EVENTS_PER_BLOCK))]
    draw = functools.partial(_draw_job, bank=bank)
    if workers > 1 and len(jobs) > 1:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=min(workers, len(jobs))) as ex:
            parts = list(ex.map(draw, jobs))
    else:
        parts = [draw(j) for j in jobs]
    cat = lambda k: (np.concatenate([p[k] for p in parts]) if parts else np.zeros(0))
    words = cat("words").astype(np.uint32)
    road_len = cat("road_len").astype(np.int64)
    road_word_begin = np.zeros(road_len.size, dtype=np.int64)
    if road_len.size:
        road_word_begin[1:] = np.cumsum(road_len)[:-1]
    rpe = cat("rpe").astype(np.int64)
    ev_road_begin = np.concatenate([[0], np.cumsum(rpe)])
    event_word_begin = np.zeros(n_ev + 1, dtype=np.int64)
    rb = np.concatenate([road_word_begin, [words.size]])
    event_word_begin[:] = rb[ev_road_begin]
    nh = cat("nh").astype(np.int32).reshape(-1, N_LAYERS)
    return Sample(words=words, n_events=n_ev, road_event=cat("road_event").astype(np.int32),
                  road_set=cat("rtag").astype(np.int32), road_nhits=nh,
                  road_word_begin=road_word_begin, event_word_begin=event_word_begin,
                  true_road=cat("true_road").astype(bool),
                  true_t=cat("t").astype(np.int64).reshape(-1, 3),
                  true_slot=cat("slot").astype(np.int32).reshape(-1, N_LAYERS))


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> np.ndarray:
    """Arrival times in seconds of a Poisson stream (exponential gaps of mean 1/rate)."""
    rng = np.random.default_rng([seed, 0xA11])
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def config_chi2_cut(config: str | dict) -> int:
    cfg = CONFIGS[config] if isinstance(config, str) else config
    return int(cfg.get("chi2_cut", DEFAULT_CHI2_CUT))


def expected_size(config: str) -> dict:
    """Mean sizes of a configuration, from its distributions (used to size buffers)."""
    cfg = CONFIGS[config]
    r = cfg["roads"]
    if r[0] == "fixed":
        rpe = r[1]
    elif r[0] == "uniform":
        rpe = (r[1] + r[2]) / 2
    else:
        p = 1.0 / r[1]
        rpe = (1 - (1 - p) ** r[2]) / p
    h = cfg["hits"]
    if h[0] == "uniform":
        vals = np.arange(h[1], h[2] + 1)
        mean_n = vals.mean()
        mean_c = vals.mean() ** N_LAYERS
    else:
        vals = np.arange(h[1], h[2] + 1)
        mean_n = (1 - h[4]) * vals.mean() + h[4] * h[3]
        mean_c = mean_n ** N_LAYERS
    roads = cfg["n_events"] * rpe
    return dict(roads=roads, words=roads * N_LAYERS * mean_n, combos=roads * mean_c)


__all__ = ["Bank", "Sample", "CONFIGS", "make_bank", "make_sample", "pack_words",
           "unpack_fields", "poisson_arrivals", "config_chi2_cut", "expected_size",
           "N_LAYERS", "N_SETS", "SHIFT", "DEFAULT_CHI2_CUT"]

"""Small hand-built and random tiny hit streams for the CPU pins (draws numbers, no fitting)."""
from __future__ import annotations

import numpy as np


def pack(coord: int, layer: int, rtag: int, etag: int) -> int:
    return (coord & 0x1FFF) | ((layer & 7) << 13) | ((rtag & 0xFF) << 16) | ((etag & 0xFF) << 24)


def stream(events) -> np.ndarray:
    """events: list of events; event: list of roads; road: (rtag, [(layer, coord), ...])."""
    out = []
    for e, roads in enumerate(events):
        for rtag, hits in roads:
            for lay, c in hits:
                out.append(pack(c, lay, rtag, e % 256))
    return np.array(out, dtype=np.uint32)


def random_events(rng, n_events=3, max_roads=4, max_hits=3, min_hits=1, shuffle=True,
                  coord_range=(-4096, 4095)):
    """Random tiny event list obeying the stream preconditions (adjacent road tags differ)."""
    events = []
    for _ in range(n_events):
        roads = []
        prev = -1
        for _ in range(int(rng.integers(1, max_roads + 1))):
            rt = int(rng.integers(0, 256))
            while rt == prev:
                rt = int(rng.integers(0, 256))
            prev = rt
            hits = []
            for lay in range(5):
                for _ in range(int(rng.integers(min_hits, max_hits + 1))):
                    hits.append((lay, int(rng.integers(coord_range[0], coord_range[1] + 1))))
            if shuffle:
                hits = [hits[i] for i in rng.permutation(len(hits))]
            roads.append((rt, hits))
        events.append(roads)
    return events


def random_bank(rng, n_sets=256, extreme=False):
    """Random constants; ``extreme`` mixes in the int16 / int32 limits."""
    if extreme:
        f = rng.choice(np.array([-32768, -32767, -1, 0, 1, 32766, 32767], dtype=np.int64),
                       size=(n_sets, 6, 5))
        q = rng.choice(np.array([-(2**31), -(2**31) + 1, -1025, -1, 0, 1023, 2**31 - 1],
                                dtype=np.int64), size=(n_sets, 6))
    else:
        f = rng.integers(-3000, 3001, size=(n_sets, 6, 5))
        q = rng.integers(-(2**24), 2**24, size=(n_sets, 6))
    return f.astype(np.int16), q.astype(np.int32)

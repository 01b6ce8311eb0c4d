"""Brute-force reference for tiny inputs: Python integers and ``itertools.product``.

Used only to pin the oracle on small cases.  It enumerates combinations with
``itertools.product`` over the per-layer hit lists (first layer varies slowest, the nested-loop
order of section II-A) and rounds with Python's floor division ``//``, so it shares neither the
oracle's loop code nor its rounding helper.
"""
from __future__ import annotations

import itertools


def decode(w: int):
    c = w & 0x1FFF
    if c & 0x1000:
        c -= 0x2000
    return c, (w >> 13) & 7, (w >> 16) & 0xFF, (w >> 24) & 0xFF


def brute(words, f, q, cfg):
    """Return the same outputs as the oracle, as Python lists, or ('error', status, index)."""
    words = [int(w) for w in words]
    L = cfg["n_layers"]
    dec = [decode(w) for w in words]
    for i, (_, lay, _, _) in enumerate(dec):
        if lay >= L:
            return ("error", -2, i)
    roads = []  # [begin, end, event, rtag]
    ev = -1
    for i, (_, _, rt, et) in enumerate(dec):
        new_ev = i == 0 or et != dec[i - 1][3]
        new_rd = new_ev or rt != dec[i - 1][2]
        if new_ev:
            ev += 1
        if new_rd:
            roads.append([i, i, ev, rt])
        roads[-1][1] = i + 1
    grouped = []
    for ri, (b, e, _, _) in enumerate(roads):
        lay = [[] for _ in range(L)]
        for i in range(b, e):
            lay[dec[i][1]].append(dec[i][0])
        if any(len(x) > cfg["max_hits"] for x in lay):
            return ("error", -3, ri)
        grouped.append(lay)
    for ri, r in enumerate(roads):
        if r[3] >= cfg["n_sets"]:
            return ("error", -6, ri)

    out = {k: [] for k in ["p0", "p1", "p2", "c0", "c1", "c2", "chi2", "accept",
                           "combo_road", "combo_hits", "kept"]}
    road_tab = {k: [] for k in ["road_event", "road_set", "road_hit_begin", "road_nhits",
                                "road_combo_begin", "road_ncombo", "best_nacc", "best_k",
                                "best_p0", "best_p1", "best_p2", "best_chi2"]}
    hit_coord = [0] * len(words)
    g = 0
    for ri, ((b, e, evo, rt), lay) in enumerate(zip(roads, grouped)):
        fs = [[int(f[rt][j][l]) for l in range(L)] for j in range(6)]
        qs = [int(q[rt][j]) for j in range(6)]
        pos = b
        for l in range(L):
            for x in lay[l]:
                hit_coord[pos] = x
                pos += 1
        n = [len(x) for x in lay]
        road_tab["road_event"].append(evo)
        road_tab["road_set"].append(rt)
        road_tab["road_hit_begin"].append(b)
        road_tab["road_nhits"].append(sum(n[l] << (4 * l) for l in range(L)))
        road_tab["road_combo_begin"].append(g)
        idx_lists = [range(len(x)) for x in lay]
        best = None
        nacc = 0
        cnt = 0
        for k, hs in enumerate(itertools.product(*idx_lists)):
            xs = [lay[l][hs[l]] for l in range(L)]
            v = [(sum(fs[j][l] * xs[l] for l in range(L)) + qs[j]) // (2 ** cfg["shift"])
                 for j in range(6)]
            chi2 = v[3] ** 2 + v[4] ** 2 + v[5] ** 2
            acc = chi2 <= cfg["chi2_cut"]
            for name, val in zip(["p0", "p1", "p2", "c0", "c1", "c2"], v):
                out[name].append(val)
            out["chi2"].append(chi2)
            out["accept"].append(int(acc))
            out["combo_road"].append(ri)
            out["combo_hits"].append(sum(hs[l] << (4 * l) for l in range(L)))
            if acc:
                nacc += 1
                out["kept"].append(g + k)
                if best is None or (chi2, k) < best[:2]:
                    best = (chi2, k, v[0], v[1], v[2])
            cnt += 1
        road_tab["road_ncombo"].append(cnt)
        g += cnt
        road_tab["best_nacc"].append(nacc)
        if best is None:
            road_tab["best_k"].append(-1)
            road_tab["best_chi2"].append(2**63 - 1)
            for nm in ["best_p0", "best_p1", "best_p2"]:
                road_tab[nm].append(-(2**31))
        else:
            road_tab["best_k"].append(best[1])
            road_tab["best_chi2"].append(best[0])
            road_tab["best_p0"].append(best[2])
            road_tab["best_p1"].append(best[3])
            road_tab["best_p2"].append(best[4])
    res = dict(out)
    res.update(road_tab)
    res["hit_coord"] = hit_coord
    res["n_roads"] = len(roads)
    res["n_events"] = ev + 1
    res["n_combos"] = g
    return res

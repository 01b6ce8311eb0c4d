"""The C-ABI library loads and exports every entry point the public header declares.

CPU-only: no call here reaches a GPU (host-side helpers and argument checks only).
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1312_0917_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_stages():
    names = declared_functions()
    for n in ["svt_unpack", "svt_combine", "svt_fit", "svt_select", "svt_process_batch"]:
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = L.load()
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), f"{n} missing from libsvt.so"
    assert sorted(L.exported_symbols()) == names


def test_abi_version_and_struct_sizes():
    lib = L.load()
    assert lib.svt_abi_version() == 1
    assert ctypes.sizeof(L.svt_config) == 24
    assert ctypes.sizeof(L.svt_tune) == 20
    rec = L.pack_bank(__import__("numpy").zeros((2, 6, 5), "int16"),
                      __import__("numpy").zeros((2, 6), "int32"))
    assert rec.shape == (2, 88)


def test_error_word_decoding():
    assert L.error_decode(L.SVT_NO_ERROR) == (L.SVT_OK, -1)
    assert L.error_decode((1 << 56) | 17) == (L.SVT_ERR_LAYER, 17)
    assert L.error_decode((2 << 56) | 5) == (L.SVT_ERR_HITS, 5)
    assert L.error_decode((3 << 56) | 9) == (L.SVT_ERR_SET, 9)
    assert L.error_decode((4 << 56) | 1) == (L.SVT_ERR_CAPACITY, 1)
    assert L.error_decode((5 << 56) | 3) == (L.SVT_ERR_ARG, 3)
    # ordering of the packed word is the precedence order
    assert (1 << 56) | 1000 < (2 << 56) | 0


def test_workspace_sizes_are_aligned_and_monotone():
    for n in [0, 1, 4095, 4096, 4097, 10**6]:
        a = L.svt_unpack_workspace(n)
        assert a > 0 and a % 256 == 0
        assert L.svt_unpack_workspace(n + 4096) >= a
    assert L.svt_unpack_workspace(-1) == -1
    t = L.make_tune(8192, 64, 256, 3)
    assert L.svt_batch_workspace(1 << 20, 1 << 16, 1 << 22, t) > 0
    assert L.svt_batch_workspace(1 << 20, 1 << 16, 1 << 22, L.make_tune(1000, 64, 256, 4)) == -1
    assert L.svt_batch_workspace(1 << 20, 1 << 16, 1 << 22, L.make_tune(16384, 64, 256, 4)) == -1
    assert L.svt_batch_workspace(1 << 20, 1 << 16, 1 << 22, L.make_tune(8192, 48, 256, 4)) == -1
    # the batched path holds at most 2^31 - 1 words per batch
    assert L.svt_batch_workspace((1 << 31) - 1, 1 << 16, 1 << 22, t) > 0
    assert L.svt_batch_workspace(1 << 31, 1 << 16, 1 << 22, t) == -1


def test_host_argument_checks_reject_without_launching():
    lib = L.load()
    cfg = L.make_config()
    roads = L.svt_roads()
    # null error word / sizes: rejected before any HIP call
    assert lib.svt_unpack(None, 0, ctypes.byref(cfg), ctypes.byref(roads), 0, None, None, None,
                          None, 0, None) == L.SVT_ERR_ARG
    bad = L.make_config(n_layers=4)
    assert lib.svt_combine(ctypes.byref(roads), 0, ctypes.byref(bad), None, None, 0, None, None,
                           None, 0, None) == L.SVT_ERR_ARG
    bad_shift = L.make_config(shift=0)
    rec = L.svt_fitrec()
    assert lib.svt_fit(None, ctypes.byref(bad_shift), ctypes.byref(roads), 0, None, 0, None,
                       None, 0, ctypes.byref(rec), None, None) == L.SVT_ERR_ARG
    best = L.svt_best()
    assert lib.svt_select(ctypes.byref(cfg), ctypes.byref(roads), -1, None, ctypes.byref(rec), 0,
                          None, ctypes.byref(best), None, 0, None, None, None, 0,
                          None) == L.SVT_ERR_ARG
    tune = L.make_tune()
    assert lib.svt_process_batch(None, ctypes.byref(cfg), ctypes.byref(tune), None, None, 0,
                                 ctypes.byref(roads), 0, ctypes.byref(rec), None, 0,
                                 ctypes.byref(best), None, 0, None, None, None, None, None, 0,
                                 0, None) == L.SVT_ERR_ARG
    # svt_gather_results: null structs or arrays, a negative size, a misaligned buffer (the
    # non-null "device" addresses are never dereferenced on the host)
    fake = 1 << 20
    full_roads = L.svt_roads(*([fake] * 6))
    full_best = L.svt_best(*([fake] * 6))
    ok_args = [ctypes.byref(full_roads), ctypes.byref(full_best), 10, fake, fake, fake, None,
               fake, fake, 10, None]
    for i, bad_v in [(0, None), (1, ctypes.byref(best)), (3, None), (7, None), (8, None),
                     (8, fake + 4), (9, -1), (2, -1)]:
        args = list(ok_args)
        args[i] = bad_v
        assert lib.svt_gather_results(*args) == L.SVT_ERR_ARG, i


def test_gathered_layout_parses_header_and_road_arrays():
    nr, cap = 3, 5
    buf = np.zeros(L.GATHER_HEADER_BYTES + L.GATHER_BYTES_PER_ROAD * cap, dtype=np.uint8)
    buf[:40].view(np.int64)[:] = [100, nr, 17, -1, -1]
    off = L.GATHER_HEADER_BYTES
    buf[off:off + 8 * nr].view(np.int64)[:] = [5, 7, 2 ** 40]
    off += 8 * nr
    for a in range(7):
        buf[off:off + 4 * nr].view(np.int32)[:] = np.arange(nr) + 10 * a
        off += 4 * nr
    head, roads = L.gathered(buf)
    assert head == dict(n_words=100, n_roads=nr, n_combos=17, n_kept=-1, err=L.SVT_NO_ERROR)
    assert roads["chi2"].tolist() == [5, 7, 2 ** 40]
    for a, k in enumerate(("n_accept", "k", "p0", "p1", "p2", "event", "set")):
        assert roads[k].tolist() == [10 * a, 10 * a + 1, 10 * a + 2], k
    buf[8:16].view(np.int64)[0] = cap + 1  # more roads than the buffer holds: header only
    assert L.gathered(buf)[1] is None


def test_product_path_does_not_import_the_oracle():
    import sys
    import importlib
    for m in list(sys.modules):
        if m == "oracle" or m.startswith("oracle."):
            pass
    src_dir = os.path.join(ROOT, "paper_1312_0917_amd")
    for fn in os.listdir(src_dir):
        if fn.endswith(".py"):
            text = open(os.path.join(src_dir, fn)).read()
            assert "import oracle" not in text and "from oracle" not in text, fn
    for fn in os.listdir(os.path.join(src_dir, "csrc")):
        text = open(os.path.join(src_dir, "csrc", fn)).read()
        assert "svt_oracle" not in text and "ora_" not in text, fn


def test_tune_resolution_fills_defaults_and_rejects_unbuilt_shapes():
    t = L.svt_tune_resolve()  # schedule 0: chosen per call from the word capacity
    assert (t.tile_combos, t.chunk_roads, t.wg_size, t.wgs_per_cu, t.schedule) == \
        (4096, 64, 256, 3, 0)
    t = L.svt_tune_resolve(L.make_tune(8192, 0, 512, 0, 1))
    assert (t.tile_combos, t.chunk_roads, t.wg_size, t.wgs_per_cu, t.schedule) == (8192, 64, 512, 3, 1)
    t = L.svt_tune_resolve(L.make_tune(8192, 0, 0, 4, L.SVT_SCHEDULE_TILES))
    assert (t.tile_combos, t.wgs_per_cu, t.schedule) == (8192, 4, L.SVT_SCHEDULE_TILES)
    for bad in [L.make_tune(wg_size=128), L.make_tune(tile_combos=6000),
                L.make_tune(chunk_roads=48), L.make_tune(wgs_per_cu=9), L.make_tune(schedule=4),
                # the one-pass kernel's LDS holds three workgroups per CU
                L.make_tune(wgs_per_cu=4, schedule=L.SVT_SCHEDULE_ONEPASS),
                L.make_tune(wgs_per_cu=4)]:  # schedule 0 may become the one-pass kernel
        with pytest.raises(L.SvtError):
            L.svt_tune_resolve(bad)


def test_static_workspace_limit_and_host_rejections():
    """svt_process_batch_static: capacities beyond its static workspace, a graph request and
    invalid arguments are refused on the host, before any HIP call."""
    lib = L.load()
    st, need, limit = L.svt_static_workspace_need(4096, 512, 1 << 15)
    assert st == L.SVT_OK and 0 < need <= limit
    assert need == L.svt_batch_workspace(4096, 512, 1 << 15, L.make_tune())
    st, need, limit = L.svt_static_workspace_need(1 << 30, 1 << 20, 1 << 30)
    assert st == L.SVT_ERR_CAPACITY and need > limit
    assert L.svt_static_workspace_need(-1, 0, 0)[0] == L.SVT_ERR_ARG
    cfg, tune = L.make_config(), L.make_tune()
    fake = 1 << 20
    roads = L.svt_roads(*([fake] * 6))
    rec = L.svt_fitrec(*([fake] * 4), None, None, None)
    best = L.svt_best(*([fake] * 6))
    args = [fake, ctypes.byref(cfg), ctypes.byref(tune), fake, fake, 4096, ctypes.byref(roads),
            512, ctypes.byref(rec), fake, 1 << 15, ctypes.byref(best), None, 0, fake, fake, None,
            fake, 0, None]
    fn = lib.svt_process_batch_static
    graph = list(args)
    graph[18] = L.SVT_BATCH_GRAPH
    assert fn(*graph) == L.SVT_ERR_ARG
    big = list(args)
    big[5] = 1 << 30
    assert fn(*big) == L.SVT_ERR_CAPACITY
    nobank = list(args)
    nobank[0] = None
    assert fn(*nobank) == L.SVT_ERR_ARG
    # a negative workspace size stays an argument error on the workspace entry point
    assert lib.svt_process_batch(*args[:18], fake, -2, 0, None) == L.SVT_ERR_ARG


def test_schedule_zero_is_chosen_from_the_word_capacity():
    """Schedule 0: the one-pass kernel up to 2^19 words of capacity, pre-pass + tiles above;
    an explicit schedule is kept; the workspace follows the chosen schedule."""
    small = L.svt_tune_for_batch(None, 1 << 19)
    large = L.svt_tune_for_batch(None, (1 << 19) + 1)
    assert small.schedule == L.SVT_SCHEDULE_ONEPASS and large.schedule == L.SVT_SCHEDULE_TILES
    assert L.svt_tune_for_batch(L.make_tune(schedule=L.SVT_SCHEDULE_TILES), 100).schedule == \
        L.SVT_SCHEDULE_TILES
    assert L.svt_tune_for_batch(L.make_tune(schedule=L.SVT_SCHEDULE_ONEPASS), 1 << 30).schedule == \
        L.SVT_SCHEDULE_ONEPASS
    assert (small.tile_combos, small.chunk_roads, small.wg_size, small.wgs_per_cu) == \
        (4096, 64, 256, 3)
    # schedule 0 must suit the one-pass kernel too: at most 3 workgroups per CU
    with pytest.raises(L.SvtError):
        L.svt_tune_for_batch(L.make_tune(wgs_per_cu=4), 1 << 25)
    assert L.svt_tune_for_batch(L.make_tune(wgs_per_cu=4, schedule=L.SVT_SCHEDULE_TILES),
                                1 << 25).wgs_per_cu == 4
    for cap in (1000, 1 << 19, 1 << 22):
        assert L.svt_batch_workspace(cap, cap // 5, 4 * cap, None) == \
            L.svt_batch_workspace(cap, cap // 5, 4 * cap, L.svt_tune_for_batch(None, cap))

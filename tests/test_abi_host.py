"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, sizes workspaces and rejects invalid arguments before touching a
device.  No compute call is made here."""

import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_2412_16544_amd import htrise as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(H.LIB_PATH):
        from paper_2412_16544_amd import build
        build.build()
    return H.lib()


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            names += re.findall(r"^\s*(?:ht_status|void|const char\s*\*|int32_t|size_t)\s*(ht_\w+)\s*\(", text,
                                re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "ht_init_batch" in names and "ht_rise_update" in names and "ht_reconstruct" in names
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(H.lib(), n)


def test_status_strings():
    for st in range(7):
        assert H.ht_status_str(st)
    assert "rank" in H.ht_status_str(H.HT_ERANKCAP)


def _ws(**kw):
    args = dict(n=(16, 16, 16, 16), eps=1e-4, rank_cap=32, max_batch=8, n_cap=64)
    args.update(kw)
    cfg, keep = H.make_config(args["n"], args["eps"], args["rank_cap"], args["max_batch"], args["n_cap"],
                              args.get("prec", H.HT_FP64), args.get("in_dtype", H.HT_F32), args.get("flags", 0))
    return H.ht_workspace_bytes(cfg)


def test_workspace_sizing_is_monotone():
    a = _ws()
    assert a > 0
    assert _ws(max_batch=16) > a
    assert _ws(n_cap=1024) > a
    assert _ws(rank_cap=8) < a


def test_mixed_form_is_a_valid_config():
    # the FP32 form shares the layout: same workspace as the FP64 form
    assert _ws(prec=H.HT_FP32) == _ws(prec=H.HT_FP64)


@pytest.mark.parametrize("kw", [dict(n=(16,)), dict(eps=0.0), dict(eps=1.0), dict(n=(16, 0, 3)),
                                dict(rank_cap=0), dict(rank_cap=65), dict(max_batch=0), dict(n_cap=0),
                                dict(prec=7), dict(prec=2), dict(in_dtype=5), dict(flags=8)])
def test_invalid_configs_rejected(kw):
    with pytest.raises(H.HTError) as e:
        _ws(**kw)
    assert e.value.status == H.HT_EINVAL
    assert H.lib().ht_last_error().decode()


def _ws_tree(n, parent):
    cfg, keep = H.make_config(n, 1e-4, 16, 4, 16, tree_parent=parent)
    return H.ht_workspace_bytes(cfg)


@pytest.mark.parametrize("n,parent", [((8, 8, 8, 8), [-1, 0, 0, 1, 1, 3, 3]), ((8, 8, 8, 8), [-1, 0, 0, 2, 2, 4, 4]),
                                      ((6, 6, 6, 6, 6), [-1, 0, 0, 2, 2, 3, 3, 4, 4]), ((5, 7), [-1, 0, 0])])
def test_tree_parent_accepted(n, parent):
    assert _ws_tree(n, parent) > 0


def test_tree_parent_of_the_balanced_tree_sizes_like_the_default():
    # the balanced tree written out: same capacities, same workspace
    assert _ws_tree((8, 9, 10, 11, 12), [-1, 0, 0, 1, 1, 2, 2, 3, 3]) == _ws_tree((8, 9, 10, 11, 12), None)


@pytest.mark.parametrize("parent", [[-1, 0, 0, 0, 1, 1, 2],      # three successors of the root
                                    [-1, 0, 0, 1, 1, 1, 1],      # four successors of node 1
                                    [-1, 0, 0, 2, 2, 1, 1],      # not layer by layer, left to right
                                    [0, 0, 0, 1, 1, 2, 2],       # no root
                                    [-1, 0, 0, 3, 3, 4, 4],      # a parent after its successor
                                    [-1, 0, 2, 1, 1, 2, 2]])     # a node naming a later parent
def test_invalid_tree_parent_rejected(parent):
    with pytest.raises(H.HTError) as e:
        _ws_tree((8, 8, 8, 8), parent)
    assert e.value.status == H.HT_EINVAL
    assert "tree_parent" in H.lib().ht_last_error().decode()


def test_null_arguments_rejected_before_device_work():
    L = H.lib()
    cfg, keep = H.make_config((4, 4), 1e-3, 4, 2, 4)
    h = ctypes.c_void_p(0)
    info = H.ht_update_info()
    # NULL batch
    assert L.ht_init_batch(ctypes.byref(cfg), None, 0, None, 2, None, ctypes.byref(h), ctypes.byref(info)) == H.HT_EINVAL
    # NULL out handle
    assert L.ht_init_batch(ctypes.byref(cfg), None, 0, 1, 2, None, None, ctypes.byref(info)) == H.HT_EINVAL
    # N out of range
    assert L.ht_init_batch(ctypes.byref(cfg), None, 0, 1, 0, None, ctypes.byref(h), None) == H.HT_EINVAL
    assert L.ht_init_batch(ctypes.byref(cfg), None, 0, 1, 3, None, ctypes.byref(h), None) == H.HT_ESHAPE
    # calls on a NULL handle
    assert L.ht_rise_update(None, 1, 1, None, None) == H.HT_EINVAL
    assert L.ht_reconstruct(None, 0, 1, 1, H.HT_F64, None) == H.HT_EINVAL
    assert L.ht_project(None, 1, 1, 1, None) == H.HT_EINVAL
    assert L.ht_query_ranks(None, None, 0, None, None) == H.HT_EINVAL
    assert L.ht_export_cores(None, None, 0, None) == H.HT_EINVAL
    L.ht_destroy(None)


def test_update_many_argument_errors_before_device_work():
    L = H.lib()
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    hs = (vp * 2)(fake, fake)
    ys = (vp * 2)(vp(1), vp(1))
    ns = (ctypes.c_int64 * 2)(1, 1)
    infos = (H.ht_update_info * 2)()
    assert L.ht_rise_update_many(None, ys, ns, 2, None, infos) == H.HT_EINVAL
    assert L.ht_rise_update_many(hs, None, ns, 2, None, infos) == H.HT_EINVAL
    assert L.ht_rise_update_many(hs, ys, None, 2, None, infos) == H.HT_EINVAL
    assert L.ht_rise_update_many(hs, ys, ns, 0, None, infos) == H.HT_EINVAL
    # the same handle twice is rejected before any handle is touched
    assert L.ht_rise_update_many(hs, ys, ns, 2, None, infos) == H.HT_EINVAL
    assert "twice" in L.ht_last_error().decode()
    nulls = (vp * 1)(vp(0))
    assert L.ht_rise_update_many(nulls, ys, ns, 1, None, infos) == H.HT_EINVAL


def test_binding_refuses_missing_library(monkeypatch):
    monkeypatch.setattr(H, "_lib", None)
    monkeypatch.setattr(H, "LIB_PATH", "/nonexistent/libhtrise.so")
    with pytest.raises(RuntimeError):
        H.lib()


# ---- precision gate and decision certificate of the mixed form (host logic) -------------------
def _prec(n, eps, rank_cap, prec=H.HT_FP32):
    cfg, keep = H.make_config(n, eps, rank_cap, 8, 64, prec)
    return H.ht_update_precision(cfg)


def test_precision_gate():
    # 16^4 with rank capacity 64: node capacities 16, 16, 16, 16, 64, 64 -> sum(r + 1) = 198
    assert _prec((16, 16, 16, 16), 1e-4, 64) == H.HT_FP32
    assert _prec((16, 16, 16, 16), 1e-3, 64) == H.HT_FP32
    assert _prec((16, 16, 16, 16), 1e-6, 64) == H.HT_FP64
    assert _prec((16, 16, 16, 16), 1e-3, 64, H.HT_FP64) == H.HT_FP64
    # the gate: 2 u sqrt(198) <= 0.5 eps / sqrt(6), u = 2^-24
    edge = 4.0 * 2.0 ** -24 * math.sqrt(198) * math.sqrt(6)
    assert _prec((16, 16, 16, 16), edge * 1.001, 64) == H.HT_FP32
    assert _prec((16, 16, 16, 16), edge * 0.999, 64) == H.HT_FP64
    # a larger capacity raises the floor
    assert _prec((96, 96, 96, 3), 1e-4, 48) == H.HT_FP32
    assert _prec((48, 48, 48, 48, 4), 1e-4, 64) == H.HT_FP32


def test_decision_certificate():
    cert = H.ht_test_decision_certified
    thr = 1.0
    # exact arithmetic: every decision of the rule certifies
    assert cert(3, 0, 10, 0.999, 0.002, thr, 0.0, 0.0)
    assert cert(0, 0, 10, 0.5, 0.0, thr, 0.0, 0.0)
    # kept side within the error of the budget: tail 0.99 thr, Delta = 2 sqrt(.99) 0.01 + 1e-4 > 0.01
    assert not cert(3, 0, 10, 0.99, 0.5, thr, 0.01, 0.0)
    assert cert(3, 0, 10, 0.97, 0.5, thr, 0.01, 0.0)
    # one rank lower within the error: t_r + lam_r = 1.01 thr
    assert not cert(3, 0, 10, 0.5, 0.51, thr, 0.01, 0.0)
    assert cert(3, 0, 10, 0.5, 0.53, thr, 0.01, 0.0)
    # the rank floor: no lower side to check
    assert cert(1, 1, 10, 0.5, 0.51, thr, 0.01, 0.0)
    # the Gram rounding term alone
    assert not cert(0, 0, 10, 0.95, 0.0, thr, 0.0, 0.06)
    assert cert(0, 0, 10, 0.95, 0.0, thr, 0.0, 0.04)
    # a decision cut short by the capacity (r == room, tail above thr) must stay above
    assert cert(2, 0, 2, 2.0, 0.5, thr, 0.01, 0.0)
    assert not cert(2, 0, 2, 1.01, 0.5, thr, 0.01, 0.0)


def test_adaptive_budget_flag_is_accepted():
    assert _ws(flags=H.HT_ADAPTIVE_BUDGET) == _ws()

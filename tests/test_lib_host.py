"""Host-side checks of the C-ABI library (no GPU needed).

* the built library loads and exports every function include/ot_fmm.h declares;
* plan_create rejects every kind of invalid layout and parameter with the
  documented status, before touching the device;
* a host-only plan's pair counts equal the oracle's brute-force enumeration
  (tests/golden/pair_counts.json, written by a script that calls only the
  oracle).
"""
import json
import os
import re

import numpy as np
import pytest

from paper_2412_15518_amd import fmm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ot_fmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_fmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = fmm.load_library()
    declared = header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fmm.EXPORTS) == declared


def test_status_strings_and_phase_names():
    lib = fmm.load_library()
    for code, name in [(0, "OT_FMM_OK"), (-2, "OT_FMM_INVALID_LAYOUT"), (-5, "OT_FMM_UNSUPPORTED_LAYOUT"),
                       (-8, "OT_FMM_NO_DEVICE_STATE")]:
        assert lib.ot_fmm_status_string(code).decode() == name
    assert lib.ot_fmm_status_string(-99).decode() == "OT_FMM_UNKNOWN_STATUS"
    assert [lib.ot_fmm_phase_name(i).decode() for i in range(fmm.NUM_PHASES)] == fmm.PHASES


@pytest.mark.parametrize("key", ["L0_theta0.4", "L1_theta0.4", "L2_theta0.4", "L3_theta0.4", "L4_theta0.4",
                                 "L1_theta0.5", "L2_theta0.7", "L2_theta0.34", "L2_theta0.9"])
def test_pair_counts_match_oracle_enumeration(key):
    rec = json.load(open(os.path.join(ROOT, "tests", "golden", "pair_counts.json")))["counts"][key]
    L, theta = rec["L"], rec["theta"]
    info = fmm.Plan(W.uniform_layout(L), theta=theta, host_only=True).info()
    # the library evaluates every leaf-level pair exactly (near and far stencil)
    assert info["p2p_pairs"] == rec["p2p"] + rec["m2l"][L]
    assert info["m2l_pairs_level"] == rec["m2l"][:L]
    assert info["m2l_pairs"] == sum(rec["m2l"][:L])
    N = (8 << L) ** 3
    assert info["n_leaf_cells"] == N


def test_info_flop_model_at_128():
    info = fmm.Plan(W.uniform_layout(4), host_only=True).info()
    assert info["p2p_pairs"] == 1_296_347_648 and info["m2l_pairs"] == 151_599_552
    tree = 2 * 84 * 2 * sum((8 << l) ** 3 for l in range(1, 4))
    leaf = 2 * 70 * 128 ** 3
    assert info["flops_forward"] == 8 * 1_296_347_648 + 168 * 151_599_552 + tree + leaf
    assert info["flops_forward"] == pytest.approx(3.62e10, rel=0.01)


@pytest.mark.parametrize("order", ["lex", "morton", "random"])
def test_layout_orders_accepted(order):
    p = fmm.Plan(W.uniform_layout(2, order=order, seed=3), host_only=True)
    assert p.info()["n_leaf_nodes"] == 64


def test_host_only_plan_refuses_compute():
    lib = fmm.load_library()
    p = fmm.Plan(W.uniform_layout(1), host_only=True)
    import ctypes as C
    rc = lib.ot_fmm_forward(p._handle, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None)
    assert rc == fmm.NO_DEVICE_STATE
    rc = lib.ot_fmm_adjoint(p._handle, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None)
    assert rc == fmm.NO_DEVICE_STATE
    assert lib.ot_fmm_timing_begin(p._handle, 4) == fmm.NO_DEVICE_STATE
    assert lib.ot_fmm_plan_set_leaf_chunks(p._handle, 2, 2) == fmm.NO_DEVICE_STATE
    for bad in ((0, 1), (1, 9), (-1, 4)):
        assert lib.ot_fmm_plan_set_leaf_chunks(p._handle, *bad) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_plan_set_leaf_chunks(None, 1, 1) == fmm.INVALID_ARGUMENT


def test_null_arguments():
    lib = fmm.load_library()
    import ctypes as C
    assert lib.ot_fmm_forward(None, None, None, None, None) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_adjoint(None, None, None, None, None) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_plan_info(None, None) == fmm.INVALID_ARGUMENT
    lib.ot_fmm_destroy(None)            # no-op
    h = C.c_void_p()
    assert lib.ot_fmm_plan_create(None, 0.4, 3, 0, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert h.value is None


def test_batch_argument_errors():
    """Batch and graph entry points reject bad arguments before touching the
    device; a batch of host-only plans reports NO_DEVICE_STATE."""
    import ctypes as C
    lib = fmm.load_library()
    h = C.c_void_p()
    assert lib.ot_fmm_batch_create(None, 1, 1, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_create(None, 1, 1, None) == fmm.INVALID_ARGUMENT
    p = fmm.Plan(W.uniform_layout(1), host_only=True)
    q = fmm.Plan(W.uniform_layout(1), host_only=True)
    one = (C.c_void_p * 1)(p._handle.value)
    two_same = (C.c_void_p * 2)(p._handle.value, p._handle.value)
    nulls = (C.c_void_p * 2)(None, None)
    assert lib.ot_fmm_batch_create(one, 0, 1, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_create(one, 1, 0, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_create(one, 1, 17, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_create(nulls, 2, 1, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_create(one, 1, 1, C.byref(h)) == fmm.NO_DEVICE_STATE
    assert lib.ot_fmm_batch_create(two_same, 2, 1, C.byref(h)) == fmm.NO_DEVICE_STATE
    assert h.value is None
    assert q._handle.value != p._handle.value
    ptrs = (C.c_void_p * 1)(8)
    assert lib.ot_fmm_batch_forward(None, ptrs, ptrs, ptrs, None) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_adjoint(None, ptrs, ptrs, ptrs, None) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_capture_forward(None, ptrs, ptrs, ptrs, C.byref(h)) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_batch_capture_adjoint(None, ptrs, ptrs, ptrs, None) == fmm.INVALID_ARGUMENT
    assert lib.ot_fmm_graph_launch(None, None) == fmm.INVALID_ARGUMENT
    lib.ot_fmm_graph_destroy(None)      # no-ops
    lib.ot_fmm_batch_destroy(None)


def test_flags():
    """OT_FMM_M2L_FP32 and OT_FMM_AUTOTUNE are accepted (and change no
    host-side count); unknown flag bits are rejected."""
    import ctypes as C
    lay = W.uniform_layout(2)
    a = fmm.Plan(lay, host_only=True).info()
    b = fmm.Plan(lay, host_only=True, m2l_fp32=True).info()
    assert a["m2l_pairs"] == b["m2l_pairs"] and a["flops_forward"] == b["flops_forward"]
    lib = fmm.load_library()
    keep = [np.ascontiguousarray(lay.level, dtype=np.int32), np.ascontiguousarray(lay.coord, dtype=np.int32).reshape(-1),
            np.ascontiguousarray(lay.parent, dtype=np.int32), np.ascontiguousarray(lay.is_leaf, dtype=np.uint8)]
    L = fmm._Layout()
    L.n_nodes = int(keep[0].shape[0])
    L.level = keep[0].ctypes.data_as(C.POINTER(C.c_int32))
    L.coord = keep[1].ctypes.data_as(C.POINTER(C.c_int32))
    L.parent = keep[2].ctypes.data_as(C.POINTER(C.c_int32))
    L.is_leaf = keep[3].ctypes.data_as(C.POINTER(C.c_uint8))
    L.h_leaf_min = 1.0
    L.origin = (C.c_double * 3)(0.0, 0.0, 0.0)
    L.G = 1.0
    h = C.c_void_p()
    for bad in (1 << 4, 1 << 31):
        assert lib.ot_fmm_plan_create(C.byref(L), 0.4, 3, fmm.FLAG_HOST_ONLY | bad, C.byref(h)) == fmm.INVALID_ARGUMENT
        assert h.value is None
    for good in (fmm.FLAG_M2L_FP32, fmm.FLAG_AUTOTUNE, fmm.FLAG_M2L_FP32 | fmm.FLAG_AUTOTUNE):
        assert lib.ot_fmm_plan_create(C.byref(L), 0.4, 3, fmm.FLAG_HOST_ONLY | good, C.byref(h)) == fmm.OK
        lib.ot_fmm_destroy(h)
        h = C.c_void_p()
    # a host-only plan has no leaf passes to tune: it reports no chunk counts
    info = fmm.Plan(lay, host_only=True, autotune=True).info()
    assert info["leaf_chunks_forward"] == 0 and info["leaf_chunks_adjoint"] == 0


def _expect(status, layout, theta=0.4, order=3):
    with pytest.raises(fmm.OTFMMError) as e:
        fmm.Plan(layout, theta=theta, order=order, host_only=True)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def _copy(lay):
    return W.Layout(level=lay.level.copy(), coord=lay.coord.copy(), parent=lay.parent.copy(),
                    is_leaf=lay.is_leaf.copy(), h_leaf_min=lay.h_leaf_min, origin=lay.origin, G=lay.G)


def test_parameter_errors():
    lay = W.uniform_layout(1)
    _expect(fmm.UNSUPPORTED_ORDER, lay, order=2)
    _expect(fmm.UNSUPPORTED_ORDER, lay, order=4)
    _expect(fmm.UNSUPPORTED_THETA, lay, theta=0.3)
    _expect(fmm.UNSUPPORTED_THETA, lay, theta=1.5)
    _expect(fmm.INVALID_ARGUMENT, lay, theta=float("nan"))
    _expect(fmm.INVALID_ARGUMENT, lay, theta=-1.0)
    bad = _copy(lay); bad.h_leaf_min = 0.0
    _expect(fmm.INVALID_ARGUMENT, bad)
    bad = _copy(lay); bad.G = float("inf")
    _expect(fmm.INVALID_ARGUMENT, bad)


def test_layout_errors():
    lay = W.uniform_layout(2)
    # root not first
    bad = _copy(lay); bad.parent[0] = 3
    _expect(fmm.INVALID_LAYOUT, bad)
    # orphan: parent index out of range
    bad = _copy(lay); bad.parent[5] = 10_000
    assert "out of range" in _expect(fmm.INVALID_LAYOUT, bad)
    # parent on the wrong level
    bad = _copy(lay); i = int(np.nonzero(lay.level == 2)[0][0]); bad.parent[i] = 0
    assert "one level up" in _expect(fmm.INVALID_LAYOUT, bad)
    # child outside its parent
    bad = _copy(lay); i = int(np.nonzero(lay.level == 2)[0][0])
    bad.coord[i] = (bad.coord[i] + 2) % 4
    _expect(fmm.INVALID_LAYOUT, bad)
    # coordinates outside the level
    bad = _copy(lay); i = int(np.nonzero(lay.level == 1)[0][0]); bad.coord[i, 0] = 2
    assert "outside level" in _expect(fmm.INVALID_LAYOUT, bad)
    # duplicate node
    bad = _copy(lay)
    leaves = np.nonzero(lay.level == 2)[0]
    a, b = int(leaves[0]), int(leaves[1])
    if lay.parent[a] == lay.parent[b]:
        bad.coord[b] = bad.coord[a]
        assert "duplicate" in _expect(fmm.INVALID_LAYOUT, bad)
    # missing sibling: drop one leaf
    keep = np.ones(lay.n_nodes, bool); keep[int(leaves[-1])] = False
    bad = W.Layout(level=lay.level[keep], coord=lay.coord[keep], parent=lay.parent[keep], is_leaf=lay.is_leaf[keep])
    assert "7 of 8" in _expect(fmm.INVALID_LAYOUT, bad)
    # leaf flagged on an internal node
    bad = _copy(lay); bad.is_leaf[1] = 1
    assert "leaf with children" in _expect(fmm.INVALID_LAYOUT, bad)
    # is_leaf not boolean
    bad = _copy(lay); bad.is_leaf[-1] = 2
    _expect(fmm.INVALID_LAYOUT, bad)


def test_adaptive_layout_one_refined_node():
    """Leaves on two levels, built by hand: level-1 node 1 refined into 8
    level-2 leaves (balanced: every level-1 node exists)."""
    lay = W.uniform_layout(1)
    # refine node 1 (a level-1 leaf) into 8 level-2 leaves
    lv, co, pa, il = list(lay.level), [tuple(c) for c in lay.coord], list(lay.parent), list(lay.is_leaf)
    il[1] = 0
    for b in range(8):
        c = tuple(2 * co[1][k] + ((b >> k) & 1) for k in range(3))
        lv.append(2); co.append(c); pa.append(1); il.append(1)
    bad = W.Layout(level=np.array(lv, np.int32), coord=np.array(co, np.int32), parent=np.array(pa, np.int32),
                   is_leaf=np.array(il, np.uint8))
    info = fmm.Plan(bad, host_only=True).info()
    assert info["depth"] == 2 and info["n_leaf_cells"] == (7 + 8) * 512


def test_too_deep_layout_is_reported_unsupported():
    """A valid octree reaching level 7 (one refined branch per level): deeper
    than the 6 levels this build runs."""
    lv, co, pa, il = [0], [(0, 0, 0)], [-1], [1]
    node = 0
    for level in range(1, 8):
        il[node] = 0
        first = len(lv)
        for b in range(8):
            c = tuple(2 * co[node][k] + ((b >> k) & 1) for k in range(3))
            lv.append(level); co.append(c); pa.append(node); il.append(1)
        node = first
    deep = W.Layout(level=np.array(lv, np.int32), coord=np.array(co, np.int32), parent=np.array(pa, np.int32),
                    is_leaf=np.array(il, np.uint8))
    assert "deeper than 6" in _expect(fmm.UNSUPPORTED_LAYOUT, deep)


def test_plan_is_independent_of_layout_buffers():
    """plan_create copies what it needs; the caller may free the layout."""
    lay = W.uniform_layout(2, order="random", seed=1)
    p = fmm.Plan(lay, host_only=True)
    info0 = p.info()
    lay.level[:] = -7
    assert p.info() == info0


def test_adaptive_layouts_host_only():
    """Balanced adaptive trees are accepted; the info counts the leaf cells
    of every level, and the pair counts cover the M2L levels below the finest."""
    for kind, depth in (("corner", 2), ("edge", 3), ("blob", 3)):
        lay = W.small_amr(kind)["layout"]
        p = fmm.Plan(lay, host_only=True)
        info = p.info()
        assert info["depth"] == depth
        assert info["n_leaf_cells"] == lay.n_leaf_cells
        assert info["p2p_pairs"] > 0 and info["m2l_pairs"] == sum(info["m2l_pairs_level"][:depth])
        p.close()


def test_unbalanced_adaptive_layout_rejected():
    from test_oracle_amr_pins import unbalanced_layout
    with pytest.raises(fmm.OTFMMError) as e:
        fmm.Plan(unbalanced_layout(), host_only=True)
    assert e.value.status == -5 and "2:1" in str(e.value)


def test_am_correction_flag():
    """OT_FMM_AM_CORRECTION is accepted on uniform trees and refused on
    adaptive ones; the entry point refuses a host-only plan."""
    p = fmm.Plan(W.uniform_layout(2), host_only=True, am_correction=True)
    assert p.info()["depth"] == 2
    p.close()
    with pytest.raises(fmm.OTFMMError) as e:
        fmm.Plan(W.small_amr("corner")["layout"], host_only=True, am_correction=True)
    assert e.value.status == -5

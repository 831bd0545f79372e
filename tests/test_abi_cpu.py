"""The C-ABI library loads and exports every symbol include/rs.h declares;
argument and graph validation return their status codes before any device
work (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rs_load_graph", "rs_score", "rs_topk", "rs_apply_removals"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2508_01485_amd as rs
    lib = ctypes.CDLL(rs.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(rs.EXPORTS) == _declared()
    for name in rs.EXPORTS:
        assert callable(getattr(rs, name))


def test_status_strings_and_kernel_names():
    import paper_2508_01485_amd as rs
    assert rs.rs_status_string(0) == "RS_OK"
    assert rs.rs_status_string(6) == "RS_ERR_STATE"
    assert b"k_rows" in [rs.lib().rs_kernel_name(i) for i in range(4)]
    assert rs.lib().rs_kernel_name(999) is None


def _good():
    from rsgen import from_edges
    return from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4)], [3, 3, 9, 9, 1])


@pytest.mark.parametrize("case,status", [
    ("flags", 1), ("asym", 2), ("unsorted", 2), ("dup", 2), ("self", 2), ("neglabel", 2),
    ("range", 3), ("offsets", 2), ("width32_overflow", 3),
])
def test_load_rejects_before_device_work(case, status):
    import paper_2508_01485_amd as rs
    g = _good()
    off, col, lab = g.off.copy(), g.col.copy(), g.labels.copy()
    flags = 0
    if case == "flags":
        flags = 4
    elif case == "asym":
        col[0] = 2   # row 0 is [1, 4] -> [2, 4]; 2 does not list 0
    elif case == "unsorted":
        col[0], col[1] = col[1], col[0]
    elif case == "dup":
        col[1] = col[0]
    elif case == "self":
        col[0] = 0
    elif case == "neglabel":
        lab[2] = -5
    elif case == "range":
        col[-1] = 77
    elif case == "offsets":
        off[1] = off[2] + 1
    if case == "width32_overflow":
        csr = rs.rs_csr(5, 2**31, 4, 0, off.astype(np.int32).ctypes.data, col.ctypes.data, lab.ctypes.data)
        h = ctypes.c_void_p()
        st = rs.lib().rs_load_graph(ctypes.byref(csr), None, 0, ctypes.byref(h))
        assert st == status and not h.value
        return
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_graph(off, col, lab, flags=flags)
    assert ei.value.status == status, ei.value.detail


def test_null_arguments():
    import paper_2508_01485_amd as rs
    lib = rs.lib()
    h = ctypes.c_void_p()
    assert lib.rs_load_graph(None, None, 0, ctypes.byref(h)) == 1
    assert lib.rs_score(None) == 1
    cnt = ctypes.c_int64()
    assert lib.rs_topk(None, 5, None, None, ctypes.byref(cnt)) == 1
    assert lib.rs_apply_removals(None, None, None) == 1
    lib.rs_free_graph(None)  # ignored


def test_null_arguments_of_the_later_entry_points():
    import paper_2508_01485_amd as rs
    lib = rs.lib()
    res = rs.rs_removal_result()
    assert lib.rs_restrict_to_targets(None, 3, ctypes.byref(res)) == 1
    cnt = np.zeros(1, np.int64)
    assert lib.rs_reachable_communities(None, 1, None, cnt.ctypes.data) == 1
    assert lib.rs_topk_batch(None, 4, None, None, None) == 1
    h = ctypes.c_void_p()
    assert lib.rs_load_batch(0, None, None, None, 0, ctypes.byref(h)) == 1


def test_batch_validation_before_device_work():
    """Graph ranges that do not run 0..n, and an edge between two graphs of
    the batch, are refused before anything touches a device."""
    import paper_2508_01485_amd as rs
    g = _good()
    two_off = np.concatenate([g.off, g.off[1:] + g.off[-1]]).astype(np.int64)
    two_col = np.concatenate([g.col, g.col + 5]).astype(np.int32)
    two_lab = np.concatenate([g.labels, g.labels]).astype(np.int32)
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_batch([0, 5, 9], two_off, two_col, two_lab)
    assert ei.value.status == 1 and "0..n" in ei.value.detail
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_batch([0, 6, 10], two_off, two_col, two_lab)  # vertex 5 starts graph 2 but 0-4 link to it
    assert ei.value.status in (1, 2)
    bad = two_col.copy()
    bad[0] = 7  # vertex 0 of graph 0 -> vertex 7 of graph 1
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_batch([0, 5, 10], two_off, bad, two_lab)
    assert ei.value.status == 2 and "joins two graphs" in ei.value.detail


def test_batch_bad_row_offsets_refused():
    """Row offsets that decrease, or end past nnz, are refused with
    RS_ERR_GRAPH before the batch's rows are walked (no read past col)."""
    import paper_2508_01485_amd as rs
    g = _good()
    two_off = np.concatenate([g.off, g.off[1:] + g.off[-1]]).astype(np.int64)
    two_col = np.concatenate([g.col, g.col + 5]).astype(np.int32)
    two_lab = np.concatenate([g.labels, g.labels]).astype(np.int32)
    dec = two_off.copy()
    dec[1], dec[2] = dec[2] + 3, dec[1]  # off[1] > off[2]
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_batch([0, 5, 10], dec, two_col, two_lab)
    assert ei.value.status == 2 and "decrease" in ei.value.detail
    past = two_off.copy()
    past[-1] = two_col.size + 1000  # off[n] > nnz
    with pytest.raises(rs.RSError) as ei:
        rs.rs_load_batch([0, 5, 10], past, two_col, two_lab)
    assert ei.value.status == 2

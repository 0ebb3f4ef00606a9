"""Host-only checks of the C ABI and of the tile layout (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2504_19171_amd import inputs
import tile_layout as lo
from paper_2504_19171_amd import stiles as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "stiles.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stiles_\w+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = st.load()
    names = header_functions()
    assert set(names) == set(st.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name
    assert lib.stiles_version() >= 100


@pytest.mark.parametrize("n,w,a,b", [(2020, 32, 20, 64), (100100, 1024, 100, 256), (60, 10, 5, 64),
                                     (1000, 5000, 0, 128), (777, 100, 33, 192), (513, 0, 1, 256)])
def test_layout_formula(n, w, a, b):
    lay = st.layout(n, w, a, b)
    nb = n - a
    N = -(-nb // b)
    we = min(w, nb - 1)
    B = min(-(-we // b), N - 1)
    ap = -(-a // 16) * 16
    assert (lay.nb, lay.w, lay.nt, lay.bt, lay.arrow_ld) == (nb, we, N, B, ap)
    assert lay.off_arrow == N * (B + 1) * b * b
    assert lay.off_corner == lay.off_arrow + N * ap * b
    assert lay.total_doubles == lay.off_corner + ap * ap
    assert lay.selinv_workspace_bytes >= 8 * lay.total_doubles
    assert lay.factor_workspace_bytes >= 8 * b * b


@pytest.mark.parametrize("args,code", [((0, 1, 0, 64), -1), ((10, -1, 0, 64), -2), ((10, 1, 10, 64), -3),
                                       ((10, 1, -1, 64), -3), ((1000, 1, 513, 64), -3), ((10, 1, 0, 32), -4),
                                       ((10, 1, 0, 100), -4)])
def test_layout_rejects_bad_arguments(args, code):
    c = st._CLayout()
    assert st.load().stiles_layout_init(*args, ctypes.byref(c)) == code


def test_entry_points_reject_bad_arguments_before_any_gpu_call():
    lib = st.load()
    lay = st.layout(100, 4, 3, 64)
    ws = lay.factor_workspace_bytes
    # null A / L / logdet / info / workspace, too small workspace, bad sizes
    assert lib.stiles_factor(None, 8, 100, 4, 3, 64, 8, 8, 8, ws, None) == -1
    assert lib.stiles_factor(8, None, 100, 4, 3, 64, 8, 8, 8, ws, None) == -2
    assert lib.stiles_factor(8, 8, 0, 4, 3, 64, 8, 8, 8, ws, None) == -3
    assert lib.stiles_factor(8, 8, 100, 4, 3, 48, 8, 8, 8, ws, None) == -6
    assert lib.stiles_factor(8, 8, 100, 4, 3, 64, None, 8, 8, ws, None) == -7
    assert lib.stiles_factor(8, 8, 100, 4, 3, 64, 8, None, 8, ws, None) == -8
    assert lib.stiles_factor(8, 8, 100, 4, 3, 64, 8, 8, 8, ws - 1, None) == -9
    wss = lay.selinv_workspace_bytes
    assert lib.stiles_selinv(None, 16, 100, 4, 3, 64, 8, 8, wss, None) == -1
    assert lib.stiles_selinv(8, 8, 100, 4, 3, 64, 8, 8, wss, None) == -2   # Sigma aliases L
    assert lib.stiles_selinv(8, 16, 100, 4, 3, 64, None, 8, wss, None) == -7
    assert lib.stiles_selinv(8, 16, 100, 4, 3, 64, 8, 8, wss - 1, None) == -8
    assert lib.stiles_pack(None, 8, 8, 8, 100, 4, 3, 64, None) == -1
    assert lib.stiles_pack(8, None, 8, 8, 100, 4, 3, 64, None) == -2
    assert lib.stiles_pack(8, 8, 8, 8, 100, 4, 3, 40, None) == -8
    wsi = lib.stiles_inverse_workspace_bytes(ctypes.byref(lay._c()))
    np_ = lay.nt * lay.tile + lay.arrow_ld
    assert wsi >= lay.selinv_workspace_bytes + 8 * np_ * np_
    assert lib.stiles_inverse(None, 16, 100, 4, 3, 64, 8, 8, wsi, None) == -1
    assert lib.stiles_inverse(8, None, 100, 4, 3, 64, 8, 8, wsi, None) == -2
    assert lib.stiles_inverse(8, 16, 100, 4, 3, 64, None, 8, wsi, None) == -7
    assert lib.stiles_inverse(8, 16, 100, 4, 3, 64, 8, 8, wsi - 1, None) == -8
    wst = lib.stiles_trace_workspace_bytes()
    assert lib.stiles_trace_product(None, 8, 100, 4, 3, 64, 8, 8, wst, None) == -1
    assert lib.stiles_trace_product(8, None, 100, 4, 3, 64, 8, 8, wst, None) == -2
    assert lib.stiles_trace_product(8, 8, 100, 4, 3, 64, None, 8, wst, None) == -7
    assert lib.stiles_trace_product(8, 8, 100, 4, 3, 64, 8, 8, wst - 1, None) == -8
    assert lib.stiles_trace_product(8, 8, 100, 4, 3, 40, 8, 8, wst, None) == -6
    for code in (0, 5, -1, -100, -101, -102, -103):
        assert st.strerror(code)


def test_batched_entry_points_reject_bad_arguments_before_any_gpu_call():
    lib = st.load()
    lays = [st.layout(100, 4, 3, 64), st.layout(700, 130, 0, 128)]

    def items(over=None):
        it = (st._CBatchItem * 2)()
        for k, lay in enumerate(lays):
            c = it[k]
            c.n, c.bandwidth, c.arrow, c.tile, c.reserved = lay.n, lay.bandwidth, lay.arrow, lay.tile, 0
            c.A, c.L, c.Sigma, c.logdet, c.info = 8, 16, 24, 32, 40
        for k, (f, v) in (over or {}).items():
            setattr(it[k], f, v)
        return it
    ws = st.batch_workspace_bytes(lays)
    need = sum(max(l.factor_workspace_bytes, l.selinv_workspace_bytes) for l in lays)
    assert ws >= need
    for fn in (lib.stiles_factor_batched, lib.stiles_selinv_batched):
        assert fn(None, 2, 8, ws, None) == -1
        assert fn(items(), 0, 8, ws, None) == -2
        assert fn(items({1: ("tile", 48)}), 2, 8, ws, None) == -1
        assert fn(items({0: ("reserved", 1)}), 2, 8, ws, None) == -1
        assert fn(items({0: ("info", None)}), 2, 8, ws, None) == -1
        assert fn(items(), 2, None, ws, None) == -3
        assert fn(items(), 2, 8, ws - 1, None) == -4
    # the selinv needs Sigma, apart from L; the factor does not read it
    assert lib.stiles_selinv_batched(items({1: ("Sigma", None)}), 2, 8, ws, None) == -1
    assert lib.stiles_selinv_batched(items({1: ("Sigma", 16)}), 2, 8, ws, None) == -1
    assert lib.stiles_factor_batched(items({1: ("Sigma", None)}), 2, 8, ws - 1, None) == -4
    assert lib.stiles_batch_workspace_bytes(items({1: ("tile", 48)}), 2) == 0


def test_batch_shapes_follow_the_stated_distribution():
    sh = inputs.batch_shapes()
    assert len(sh) == 64
    assert sh == inputs.batch_shapes()          # seeded
    for nb, w, a, seed in sh:
        assert 5000 <= nb <= 50000 and w in (32, 128, 512) and 10 <= a <= 200
    assert [s[3] for s in sh] == list(range(2000, 2064))
    assert {s[1] for s in sh} == {32, 128, 512}


@pytest.mark.parametrize("nb,w,a,b", [(200, 20, 7, 64), (60, 10, 5, 64), (300, 299, 0, 64), (130, 0, 17, 128)])
def test_host_pack_roundtrip(nb, w, a, b):
    M = inputs.arrowhead_spd(nb, w, a, seed=1)
    lay = st.layout(M.n, w, a, b)
    T = lo.host_pack(M.ab, M.P, M.C, lay)
    D = lo.band_part(T, lay, lay.w)
    we = lay.w
    for d in range(we + 1):
        np.testing.assert_array_equal(D[d, : nb - d], M.ab[d, : nb - d])
    np.testing.assert_array_equal(lo.arrow_part(T, lay), M.P)
    np.testing.assert_array_equal(lo.corner_part(T, lay), M.C)
    # identity padding: pad diagonal 1, the rest of the pad 0
    full = lo.band_tile(T, lay, lay.nt - 1, 0)
    r0 = nb - (lay.nt - 1) * b
    pad = full[r0:, r0:]
    np.testing.assert_array_equal(pad, np.eye(b - r0))
    assert np.all(full[r0:, :r0] == 0) and np.all(full[:r0, r0:] == 0)


def test_selection_closure():
    """Selected pairs -> (all in L's tile pattern?, first tile column of the closure)."""
    lay = st.layout(1020, 100, 20, 64)      # nb = 1000, N = 16, B = 2
    assert (lay.nt, lay.bt) == (16, 2)
    assert st.selection_closure(lay, [(10, 5)]) == (True, 0)
    assert st.selection_closure(lay, [(500, 400)]) == (True, 6)        # tiles 7 and 6
    assert st.selection_closure(lay, [(400, 500)]) == (True, 6)        # either order
    assert st.selection_closure(lay, [(900, 100)])[0] is False          # 13 tiles apart
    assert st.selection_closure(lay, [(1005, 300)]) == (True, 4)       # arrow row
    assert st.selection_closure(lay, [(1010, 1003)]) == (True, 16)     # the corner alone
    assert st.selection_closure(lay, [(1010, 1003), (700, 650)]) == (True, 10)
    with pytest.raises(ValueError):
        st.selection_closure(lay, [(1020, 3)])


def test_selection_closure_c_entry_point():
    """The symbolic step runs behind the C ABI: empty selections, errors leave
    the outputs untouched, and the leftmost selected tile column wins."""
    import ctypes
    lib = st.load()
    inside, first = ctypes.c_int32(-9), ctypes.c_int64(-9)
    assert lib.stiles_selection_closure(1020, 100, 20, 64, None, 0, ctypes.byref(inside), ctypes.byref(first)) == 0
    assert (inside.value, first.value) == (1, 16)
    ij = np.array([[1019, 0]], dtype=np.int64)                 # arrow row, tile column 0
    assert lib.stiles_selection_closure(1020, 100, 20, 64, ij.ctypes.data, 1, ctypes.byref(inside),
                                        ctypes.byref(first)) == 0
    assert (inside.value, first.value) == (1, 0)
    inside.value, first.value = -9, -9
    bad = np.array([[3, -1]], dtype=np.int64)
    assert lib.stiles_selection_closure(1020, 100, 20, 64, bad.ctypes.data, 1, ctypes.byref(inside),
                                        ctypes.byref(first)) == -5
    assert (inside.value, first.value) == (-9, -9)
    assert lib.stiles_selection_closure(1020, 100, 20, 64, None, 1, ctypes.byref(inside), ctypes.byref(first)) == -5
    assert lib.stiles_selection_closure(1020, 100, 20, 64, ij.ctypes.data, -1, ctypes.byref(inside),
                                        ctypes.byref(first)) == -6
    assert lib.stiles_selection_closure(1020, 100, 20, 64, ij.ctypes.data, 1, None, ctypes.byref(first)) == -7
    assert lib.stiles_selection_closure(1020, 100, 20, 64, ij.ctypes.data, 1, ctypes.byref(inside), None) == -8
    assert lib.stiles_selection_closure(1020, 100, 20, 60, ij.ctypes.data, 1, ctypes.byref(inside),
                                        ctypes.byref(first)) == -4
    # every pair of a small matrix: in the pattern exactly when its tile row is
    # at most B tiles below its tile column or it touches the arrow
    lay = st.layout(300, 70, 12, 64)                          # nb = 288, N = 5, B = 2
    i, j = np.meshgrid(np.arange(300), np.arange(300), indexing="ij")
    for a, c in zip(i.ravel()[::7], j.ravel()[::7]):
        got = st.selection_closure(lay, [(a, c)])
        hi, lo = max(a, c), min(a, c)
        assert got[0] == (hi >= 288 or hi // 64 - lo // 64 <= 2)
        assert got[1] == (lo // 64 if lo < 288 else 5)


def test_selection_entry_points_reject_bad_arguments_before_any_gpu_call():
    lib = st.load()
    lay = st.layout(100, 4, 3, 64)
    wss = lay.selinv_workspace_bytes
    assert lib.stiles_selinv_range(None, 16, 100, 4, 3, 64, 0, 8, 8, wss, None) == -1
    assert lib.stiles_selinv_range(8, 8, 100, 4, 3, 64, 0, 8, 8, wss, None) == -2
    assert lib.stiles_selinv_range(8, 16, 100, 4, 3, 64, -1, 8, 8, wss, None) == -7
    assert lib.stiles_selinv_range(8, 16, 100, 4, 3, 64, lay.nt + 1, 8, 8, wss, None) == -7
    assert lib.stiles_selinv_range(8, 16, 100, 4, 3, 64, 0, None, 8, wss, None) == -8
    assert lib.stiles_selinv_range(8, 16, 100, 4, 3, 64, 0, 8, 8, wss - 1, None) == -9
    assert lib.stiles_gather(None, 100, 4, 3, 64, 8, 1, 8, None) == -1
    assert lib.stiles_gather(8, 100, 4, 3, 64, None, 1, 8, None) == -6
    assert lib.stiles_gather(8, 100, 4, 3, 64, 8, -1, 8, None) == -7
    assert lib.stiles_gather(8, 100, 4, 3, 64, 8, 1, None, None) == -8
    assert lib.stiles_gather(8, 100, 4, 3, 64, None, 0, None, None) == 0

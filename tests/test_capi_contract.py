"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")


def _lib():
    try:
        return st.load_library()
    except st.StencilLibraryMissing:
        pytest.skip("libstencil.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = header_functions()
    for required in ("stencil_plan", "stencil_execute", "stencil_run", "stencil_plan_destroy",
                     "stencil_plan_workspace", "stencil_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in header_functions():
        assert hasattr(lib, name), name
    # the binding covers the same names
    assert set(st.exported_symbols()) >= set(header_functions())


def _plan_status(coeffs, r, interior, dtype, T):
    lib = _lib()
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    shp = st._shape(interior)
    h = ctypes.c_void_p()
    status = lib.stencil_plan(ctypes.byref(h), c.ctypes.data_as(st._DBL), r, ctypes.byref(shp),
                              dtype, T, None)
    if status == st.STENCIL_OK:
        lib.stencil_plan_destroy(h)
    return status


@pytest.mark.parametrize("case,expect", [
    ("ndim1", st.STENCIL_ERR_INVALID),
    ("ndim4", st.STENCIL_ERR_INVALID),
    ("radius_neg", st.STENCIL_ERR_INVALID),
    ("radius_5", st.STENCIL_ERR_INVALID),
    ("T_neg", st.STENCIL_ERR_INVALID),
    ("extent0", st.STENCIL_ERR_INVALID),
    ("bad_dtype", st.STENCIL_ERR_INVALID),
    ("nan_coeff", st.STENCIL_ERR_INVALID),
    ("ok_2d", st.STENCIL_OK),
    ("ok_3d", st.STENCIL_OK),
    ("ok_T0", st.STENCIL_OK),
    ("ok_r0", st.STENCIL_OK),
])
def test_plan_validation(case, expect):
    w2 = wl.random_coeffs(2, "star", 1, 1)
    w3 = wl.random_coeffs(3, "star", 1, 1)
    args = {
        "ndim1": (np.ones(3), 1, (5,), st.STENCIL_F64, 1),
        "ndim4": (np.ones(81), 1, (3, 3, 3, 3), st.STENCIL_F64, 1),
        "radius_neg": (w2, -1, (8, 8), st.STENCIL_F64, 1),
        "radius_5": (np.ones((11, 11)), 5, (8, 8), st.STENCIL_F64, 1),
        "T_neg": (w2, 1, (8, 8), st.STENCIL_F64, -1),
        "extent0": (w2, 1, (0, 8), st.STENCIL_F64, 1),
        "bad_dtype": (w2, 1, (8, 8), 7, 1),
        "nan_coeff": (np.where(w2 > 0, np.nan, 0.0), 1, (8, 8), st.STENCIL_F64, 1),
        "ok_2d": (w2, 1, (8, 8), st.STENCIL_F64, 3),
        "ok_3d": (w3, 1, (4, 5, 6), st.STENCIL_F32, 3),
        "ok_T0": (w2, 1, (8, 8), st.STENCIL_F64, 0),
        "ok_r0": (np.array([[0.5]]), 0, (8, 8), st.STENCIL_F64, 2),
    }[case]
    assert _plan_status(*args) == expect, st.stencil_last_error()


def test_null_pointers_rejected():
    lib = _lib()
    shp = st._shape((8, 8))
    h = ctypes.c_void_p()
    assert lib.stencil_plan(None, None, 1, ctypes.byref(shp), 1, 1, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_plan(ctypes.byref(h), None, 1, ctypes.byref(shp), 1, 1, None) == st.STENCIL_ERR_INVALID
    c = np.ones((3, 3))
    assert lib.stencil_plan(ctypes.byref(h), c.ctypes.data_as(st._DBL), 1, None, 1, 1, None) == st.STENCIL_ERR_INVALID
    assert "shape" in st.stencil_last_error()
    assert lib.stencil_execute(None, None, None, None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_run(c.ctypes.data_as(st._DBL), 1, ctypes.byref(shp), 1, 1, None, None, None) == st.STENCIL_ERR_INVALID


def test_alias_detected_before_device_work():
    _lib()
    w = wl.random_coeffs(2, "box", 1, 3)
    plan = st.stencil_plan(w, 1, (300, 300), "float64", 10)
    try:
        info = st.stencil_plan_describe(plan)
        nbytes = info["padded_bytes"]
        fake = 1 << 40
        ws = st.stencil_plan_workspace(plan)
        with pytest.raises(st.StencilError) as e:
            st.stencil_execute(plan, fake, fake + nbytes // 2, fake + 4 * nbytes, 0)
        assert e.value.status == st.STENCIL_ERR_ALIAS
        if ws:
            with pytest.raises(st.StencilError) as e:
                st.stencil_execute(plan, fake, fake + 2 * nbytes, fake + nbytes // 3, 0)
            assert e.value.status == st.STENCIL_ERR_ALIAS
            with pytest.raises(st.StencilError) as e:
                st.stencil_execute(plan, fake, fake + 2 * nbytes, 0, 0)
            assert e.value.status == st.STENCIL_ERR_INVALID
    finally:
        st.stencil_plan_destroy(plan)


def test_plan_choices():
    _lib()
    # 2D 5-point on a wide grid: blocked scheme, passes = ceil(T / depth)
    p = st.Plan(wl.uniform_5pt_coeffs(), 1, (1024, 2048), "float64", 1000)
    i = p.info
    assert i["scheme_name"] == "blocked_2d" and i["pattern_name"] == "star" and i["points"] == 5
    assert i["passes"] == -(-1000 // i["depth"])
    assert i["workspace_bytes"] == i["padded_bytes"]
    # forced naive: one pass per step
    q = st.Plan(wl.uniform_5pt_coeffs(), 1, (64, 64), "float64", 7, flags=st.STENCIL_FLAG_NAIVE)
    assert q.info["scheme_name"] == "naive" and q.info["passes"] == 7
    # T = 0 is a copy, no workspace
    z = st.Plan(wl.uniform_5pt_coeffs(), 1, (64, 64), "float64", 0)
    assert z.info["scheme_name"] == "copy" and z.workspace_bytes == 0
    # a box pattern with a hole is classified general
    w = wl.random_coeffs(2, "box", 1, 5)
    w[0, 0] = 0.0
    g = st.Plan(w, 1, (600, 600), "float32", 4)
    assert g.info["pattern_name"] == "general" and g.info["points"] == 8
    # a single pass needs no workspace
    one = st.Plan(wl.uniform_5pt_coeffs(), 1, (600, 600), "float64", 3, depth=3)
    assert one.info["passes"] == 1 and one.workspace_bytes == 0


def _strip_columns(P, R, V, HL, ns, strip):
    """Mirror of the device strip layout: (loaded column range, stored column range)."""
    W = 64 * V
    if ns == 1:
        X0, la, lb = R, 0, 64
    elif strip == 0:
        X0, la, lb = R, 0, 64 - HL
    elif strip == ns - 1:
        X0, la, lb = P - R - W, HL, 64
    else:
        X0 = R + (64 - HL) * V + (strip - 1) * (64 - 2 * HL) * V - HL * V
        la, lb = HL, 64 - HL
    return (X0, X0 + W), (X0 + la * V, X0 + lb * V)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("r,kind", [(1, "star"), (2, "box"), (3, "star"), (4, "star")])
def test_strip_layout_covers_interior(dtype, r, kind):
    """For every width and depth the planner accepts, the strips store every
    interior column, load only interior columns, and keep at least depth*r
    columns of redundancy on each open side."""
    _lib()
    w = wl.random_coeffs(2, kind, r, 9)
    for nx in (256, 300, 511, 512, 513, 700, 1000, 1024, 1500, 3001, 8192):
        for T in (1, 2, 3, 5, 8, 13):
            try:
                p = st.Plan(w, r, (40, nx), dtype, T)
            except st.StencilError:
                continue
            i = p.info
            if i["scheme_name"] != "blocked_2d":
                continue
            V, HL, ns = i["cols_per_lane"], i["redundant_lanes"], i["strips"]
            assert HL * V >= i["depth"] * r
            P = nx + 2 * r
            covered = np.zeros(P, dtype=bool)
            for sidx in range(ns):
                (l0, l1), (s0, s1) = _strip_columns(P, r, V, HL, ns, sidx)
                assert r <= l0 and l1 <= P - r, (nx, T, sidx, l0, l1)
                if ns > 1 and 0 < sidx < ns - 1:
                    assert s0 - l0 >= i["depth"] * r and l1 - s1 >= i["depth"] * r
                covered[s0:s1] = True
            assert covered[r:P - r].all(), (nx, T)


def _tile_rows(tile, ns, seg_len, seg_len_e, edge_tiles, Q):
    """Mirror of the device tile order: (strip, first row, end row)."""
    if tile < edge_tiles:
        seg, strip, y0, n = tile // 2, (ns - 1 if tile % 2 else 0), (tile // 2) * seg_len_e, seg_len_e
    elif edge_tiles > 0:
        t = tile - edge_tiles
        seg, strip, y0, n = t // (ns - 2), 1 + t % (ns - 2), (t // (ns - 2)) * seg_len, seg_len
    else:
        seg, strip, y0, n = tile // ns, tile % ns, (tile // ns) * seg_len, seg_len
    return strip, y0, min(y0 + n, Q)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("r,kind,interior,seg", [
    (1, "star", (8192, 8192), 0), (2, "box", (8192, 8192), 0), (3, "star", (8192, 8192), 0),
    (1, "box", (8192, 8192), 0), (1, "box", (450, 800), 100), (1, "star", (2000, 3000), 0),
    (2, "star", (600, 1000), 200), (1, "star", (333, 517), 0)])
def test_edge_strip_segments(dtype, r, kind, interior, seg):
    """Edge strips get shorter segments only when the interior tiles leave
    wave slots free; every (strip, row) is covered by exactly one tile either
    way; STENCIL_FLAG_UNIFORM_TILES turns the split off."""
    _lib()
    w = wl.random_coeffs(2, kind, r, 11)
    T = 1000
    p = st.Plan(w, r, interior, dtype, T, seg_len=seg)
    u = st.Plan(w, r, interior, dtype, T, seg_len=seg, flags=st.STENCIL_FLAG_UNIFORM_TILES)
    for plan in (p, u):
        i = plan.info
        assert i["scheme_name"] == "blocked_2d"
        ns, L, Le, E = i["strips"], i["seg_len"], i["edge_seg_len"], i["edge_tiles"]
        Q = interior[0] + 2 * r
        if E:
            assert ns > 2 and Le < L
            assert E == 2 * -(-Q // Le) and i["tiles"] == E + (ns - 2) * -(-Q // L)
            assert i["tiles"] <= 4 * 256
        else:
            assert i["tiles"] == ns * -(-Q // L)
        hits = np.zeros((ns, Q), dtype=np.int32)
        for t in range(i["tiles"]):
            strip, y0, y1 = _tile_rows(t, ns, L, Le, E, Q)
            assert 0 <= strip < ns and 0 <= y0 < y1 <= Q
            hits[strip, y0:y1] += 1
        assert (hits == 1).all()
    assert u.info["edge_tiles"] == 0
    if seg == 0 and interior == (8192, 8192):
        assert p.info["edge_tiles"] > 0


def test_batch_rejects_shared_outputs_before_device_work():
    _lib()
    w = wl.uniform_5pt_coeffs()
    fake = 1 << 40
    nbytes = 302 * 302 * 8
    specs = [dict(coeffs=w, radius=1, interior=(300, 300), dtype="float64", T=5,
                  in_ptr=fake, out_ptr=fake + 4 * nbytes),
             dict(coeffs=w, radius=1, interior=(300, 300), dtype="float64", T=5,
                  in_ptr=fake + 8 * nbytes, out_ptr=fake + 4 * nbytes + 64)]
    with pytest.raises(st.StencilError) as e:
        st.stencil_batch_submit(specs, 0)
    assert e.value.status == st.STENCIL_ERR_ALIAS
    # a job whose own in and out overlap is reported per job; with no valid job left the call fails
    specs = [dict(coeffs=w, radius=1, interior=(300, 300), dtype="float64", T=5,
                  in_ptr=fake, out_ptr=fake + 100)]
    with pytest.raises(st.StencilError) as e:
        st.stencil_batch_submit(specs, 0)
    assert e.value.status == st.STENCIL_ERR_INVALID


def test_python_constants_mirror_header_defines():
    text = open(HEADER).read()
    defines = dict(re.findall(r"#define (STENCIL_[A-Z_0-9]+) (\d+)", text))
    assert defines, "no #define in the header"
    for name, value in defines.items():
        if name.startswith("STENCIL_MODEL_"):
            continue  # exposed as MODEL_* in the binding
        assert getattr(st, name) == int(value), name


def test_noalloc_rejects_workspace_beyond_region():
    """A multi-pass plan whose workspace exceeds the no-alloc scratch region
    is refused before any device work (so the pointers are never touched)."""
    lib = _lib()
    spec = wl.SUITE_2D[0]
    c = np.ascontiguousarray(wl.coeffs_for(spec, 1), dtype=np.float64)
    shp = st._shape((3000, 3000))  # 72 MB padded FP64, beyond 64 MiB
    status = lib.stencil_run_noalloc(c.ctypes.data_as(st._DBL), 1, ctypes.byref(shp), st.STENCIL_F64, 100,
                                     16, 32, None)
    assert status == st.STENCIL_ERR_INVALID
    assert b"scratch" in lib.stencil_last_error()

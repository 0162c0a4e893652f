"""The planner's performance model (paper Section 5 and the design rules of
Section 6) reproduces the numbers the paper prints for its A100 analysis.
No GPU needed: the model is host code in libstencil.so."""
import json
import os

import pytest

from paper_2305_07390_amd import stencil as st

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cost_model_a100.json")
A100 = json.load(open(GOLDEN))
PAR = A100["params"]
B_GM, B_SM, TDS, S, THR = PAR["B_gm"], PAR["B_sm"], PAR["T_Dsync"], PAR["S"], PAR["thr_cmp_fp64"]


def _lib():
    try:
        st.load_library()
    except st.StencilLibraryMissing:
        pytest.skip("libstencil.so not built")


def model(**kw):
    base = dict(B_gm=B_GM, B_sm=B_SM, thr_cmp=THR, cell_bytes=S, a_gm=2.0, a_sm=4.0, a_cmp=10.0,
                D_gm=1.0, D_sm=1.0, D_cmp=1.0, D_all=1.0, t=1.0, tiling=st.MODEL_NO_TILING,
                tiled_dims=1, tile=(0.0, 0.0), rad=1.0, t_dsync=TDS, n_sync=1.0)
    base.update(kw)
    return st.stencil_model_eval(**base)


def _values():
    v = {}
    v["2d5pt desired depth"] = model(a_gm=2, a_sm=4)["t_desired"]
    dev = dict(tiling=st.MODEL_DEVICE_TILING, tiled_dims=2, tile=(32, 32), a_gm=2, a_sm=4.5,
               D_sm=1024, D_gm=1024)
    r = model(**dev)
    v["3d7pt desired depth, device tile 32x32"] = r["t_desired"]
    v["3d7pt minimum device tile"] = r["min_tile"]
    v["2d5pt SM-tile valid proportion, t = 7, tile 256"] = model(
        tiling=st.MODEL_SM_TILING, tiled_dims=1, tile=(256, 0), t=7)["V"]
    # T_stencil = T_sm = 2.05 us (printed), T_Dsync = 1.2 us
    d_sm = 2.05e-6 * B_SM / (15 * S * 1.0)
    v["2d5pt device-tile valid proportion, T_sm = 2.05 us"] = model(
        tiling=st.MODEL_DEVICE_TILING, a_gm=0.0, a_cmp=0.0, a_sm=1.0, D_sm=d_sm, t=15)["V"]
    v["3d7pt SM tiling attainable P, t = 3"] = model(B_sm=0.0, t=3, D_gm=1.0, D_all=1.0,
                                                      a_cmp=0.0)["P"] / 1e9
    tiles, t = 108, 8
    d_gm = tiles * ((32 + 2) ** 2 + (32 + 32) * 2 * t * 1)
    dt = model(tiling=st.MODEL_DEVICE_TILING, a_gm=2, a_sm=4.5, a_cmp=14, D_gm=d_gm,
               D_sm=tiles * 1024, D_cmp=tiles * 1024, D_all=tiles * 1024, t=t)
    v["3d7pt device tile T_gm (us), t = 8, 108 tiles"] = dt["T_gm"] * 1e6
    v["3d7pt device tiling P, t = 8"] = dt["P"] / 1e9
    v["3d7pt device tiling V"] = dt["V"]
    v["3d7pt device tiling PP"] = dt["PP"] / 1e9
    p12 = model(a_gm=2, a_sm=4, t=12)["P"] / 1e9  # attainable bound at t = 12
    v["2d5pt fraction of the attainable bound, 482 GCells/s at t = 12"] = 482 / p12
    pp12 = model(a_gm=2, a_sm=4, t=12, tiling=st.MODEL_SM_TILING, tile=(256, 0))["PP"] / 1e9
    v["2d5pt fraction of PP"] = 482 / pp12
    b3 = model(B_sm=0.0, a_cmp=0.0, t=8, D_gm=2048, D_all=1024)["P"] / 1e9
    v["3d7pt fraction of the attainable bound, 197 GCells/s at t = 8"] = 197 / b3
    v["3d7pt fraction of PP"] = 197 / (dt["PP"] / 1e9)
    return v


@pytest.mark.parametrize("pin", A100["pins"], ids=[p["name"] for p in A100["pins"]])
def test_model_reproduces_printed_value(pin):
    _lib()
    got = _values()[pin["name"]]
    # half a unit of the last printed digit; whole-percent fractions were
    # rounded loosely in print (4.8/6.09 is printed as 80%)
    tol = 0.5 * 10 ** (-pin["digits"])
    if pin["name"].startswith(("2d5pt fraction", "3d7pt fraction")):
        tol = 0.015
    assert abs(got - pin["printed"]) <= tol, (pin["name"], got, pin["printed"])


def test_model_shapes():
    _lib()
    # P grows with t until the bound leaves global memory, then stays
    ps = [model(a_gm=2, a_sm=4, t=t)["P"] for t in range(1, 20)]
    assert all(b >= a for a, b in zip(ps, ps[1:]))
    assert model(a_gm=2, a_sm=4, t=3)["bottleneck"] == 0
    assert model(a_gm=2, a_sm=4, t=10)["bottleneck"] == 1
    # valid proportion of SM tiling falls with depth, vanishes when the halo eats the tile
    vs = [model(tiling=st.MODEL_SM_TILING, tile=(64, 64), tiled_dims=2, t=t)["V"] for t in range(1, 40)]
    assert all(b <= a for a, b in zip(vs, vs[1:])) and vs[-1] == 0.0
    with pytest.raises(st.StencilError):
        model(B_gm=0.0)

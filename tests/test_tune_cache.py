"""Autotuner cache: key format, JSON save/load, and that plans without a hint
take the cached depth and segment (host only; no kernel runs)."""
import json

import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl


@pytest.fixture(autouse=True)
def _clean_cache():
    st.stencil_tune_cache_clear()
    yield
    st.stencil_tune_cache_clear()


def _five_point():
    return wl.uniform_5pt_coeffs(), 1


def test_key_names_class_dtype_and_bucket():
    c, r = _five_point()
    k64 = st.stencil_tune_cache_key(c, r, (8192, 8192), np.float64)
    k32 = st.stencil_tune_cache_key(c, r, (8192, 8192), np.float32)
    kb = st.stencil_tune_cache_key(c, r, (8192, 8192), np.float64, st.STENCIL_TUNE_BATCH)
    assert "/2d/star/r1/k5/f64/b26.26/single" in k64
    assert k32.replace("/f32/", "/f64/") == k64
    assert kb.endswith("/batch") and kb.replace("/batch", "/single") == k64
    # same half-octave bucket -> same key; another bucket -> another key
    assert st.stencil_tune_cache_key(c, r, (8000, 8100), np.float64) == k64
    assert st.stencil_tune_cache_key(c, r, (4096, 8192), np.float64) != k64
    box = wl.random_coeffs(2, "box", 2, seed=1)
    assert "/2d/box/r2/k25/" in st.stencil_tune_cache_key(box, 2, (1024, 1024), np.float64)


def test_save_load_roundtrip_and_plan_uses_entry(tmp_path):
    c, r = _five_point()
    key = st.stencil_tune_cache_key(c, r, (4096, 4096), np.float64)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"version": 1, "entries": [
        {"key": key, "depth": 5, "seg": 100, "sec_per_step": 1e-4, "candidates": 7}]}))
    assert st.stencil_tune_cache_load(str(path)) == 1
    assert st.stencil_tune_lookup(c, r, (4096, 4096), np.float64) == (5, 100)
    assert st.stencil_tune_lookup(c, r, (4096, 4096), np.float64, st.STENCIL_TUNE_BATCH) is None
    p = st.Plan(c, r, (4096, 4096), np.float64, 100)
    try:
        assert p.info["depth"] == 5 and p.info["seg_len"] == 100
    finally:
        p.close()
    # an explicit hint or NO_CACHE bypasses the cache
    p = st.Plan(c, r, (4096, 4096), np.float64, 100, flags=st.STENCIL_FLAG_NO_CACHE)
    try:
        assert p.info["depth"] != 5
    finally:
        p.close()
    out = tmp_path / "saved.json"
    st.stencil_tune_cache_save(str(out))
    saved = json.loads(out.read_text())
    assert saved["entries"] == [{"key": key, "depth": 5, "seg": 100, "flags": 0, "sec_per_step": 1e-4,
                                 "candidates": 7}]
    st.stencil_tune_cache_clear()
    assert st.stencil_tune_lookup(c, r, (4096, 4096), np.float64) is None


@pytest.mark.parametrize("text", ["{}", '{"entries": [{"depth": 3, "seg": 0}]}',
                                  '{"entries": [{"key": "a", "depth": 0, "seg": 0}]}',
                                  '{"entries": [{"key": "a", "seg": 4}]}'])
def test_malformed_cache_rejected(tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(st.StencilError) as e:
        st.stencil_tune_cache_load(str(path))
    assert e.value.status == st.STENCIL_ERR_INVALID


def test_missing_cache_file_rejected(tmp_path):
    with pytest.raises(st.StencilError):
        st.stencil_tune_cache_load(str(tmp_path / "absent.json"))
    assert st.use_tuned_defaults(str(tmp_path / "absent.json")) == 0


def test_cached_depth_is_clamped_to_compiled_variants(tmp_path):
    c, r = _five_point()
    key = st.stencil_tune_cache_key(c, r, (2048, 2048), np.float64)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"entries": [{"key": key, "depth": 60, "seg": 0}]}))
    st.stencil_tune_cache_load(str(path))
    p = st.Plan(c, r, (2048, 2048), np.float64, 1000)
    try:
        assert 1 <= p.info["depth"] <= 12
    finally:
        p.close()

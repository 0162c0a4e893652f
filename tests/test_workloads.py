"""Seeded input generators: point sets and coefficient normalisation (no GPU)."""
import itertools

import numpy as np
import pytest

from paper_2305_07390_amd import workloads as wl


def _sym(pts, perm, signs):
    return {tuple(signs[i] * p[perm[i]] for i in range(3)) for p in pts}


def test_paper_point_sets():
    p19 = wl.offsets(3, wl.P19, 1)
    p17 = wl.offsets(3, wl.P17, 1)
    assert len(p19) == 19 and len(p17) == 17
    # 19 points: closed under every axis permutation and reflection
    s19 = set(p19)
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            assert _sym(p19, perm, signs) == s19
    assert (0, 0, 0) in s19 and (1, 1, 1) not in s19 and (0, 1, 1) in s19
    # 17 points: closed under x/y swaps and every reflection; z (slowest) is special
    s17 = set(p17)
    for perm in ((0, 1, 2), (0, 2, 1)):
        for signs in itertools.product((1, -1), repeat=3):
            assert _sym(p17, perm, signs) == s17
    assert all((0, dy, dx) in s17 for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    assert (1, 0, 0) not in s17 and (1, 0, 1) in s17 and (1, 1, 1) not in s17


@pytest.mark.parametrize("kind", [wl.P17, wl.P19, wl.STAR, wl.BOX])
def test_poisson_like_step_is_normalised(kind):
    c = wl.poisson_like_coeffs(3, kind, 1, 5)
    assert abs(c.sum() - 1.0) < 1e-15 and c[1, 1, 1] == 0.5
    assert (c != 0).sum() == len(wl.offsets(3, kind, 1))


def test_paper_benchmark_table():
    names = [n for n, _, _ in wl.PAPER_BENCHMARKS]
    assert names == ["j2d5pt", "j2d9pt", "j2d9pt-gol", "j2d25pt", "j3d7pt", "j3d13pt", "j3d17pt",
                     "j3d27pt", "poisson"]
    pts = {n: s.points for n, s, _ in wl.PAPER_BENCHMARKS}
    # point counts: the paper's FLOPs/cell column over 2 (the gaussian's printed 25 is read as
    # its 25 points)
    assert pts == {"j2d5pt": 5, "j2d9pt": 9, "j2d9pt-gol": 9, "j2d25pt": 25, "j3d7pt": 7,
                   "j3d13pt": 13, "j3d17pt": 17, "j3d27pt": 27, "poisson": 19}
    dims = {n: d for n, _, d in wl.PAPER_BENCHMARKS}
    assert dims["j2d5pt"] == (8352, 8352) and dims["poisson"] == (384, 288, 2560)

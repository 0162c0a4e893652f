"""Pins of the CPU oracle against facts fixed by mathematics (no GPU needed)."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2305_07390_amd import workloads as wl
from tests import pins


def _sweep(coeffs, r, u0, T):
    return oracle.sweep(coeffs, r, u0, T)


@pytest.mark.parametrize("name,check", pins.ALL_CHECKS, ids=[n for n, _ in pins.ALL_CHECKS])
def test_pin(name, check):
    check(_sweep)


@pytest.mark.parametrize("name,check", pins.F32_CHECKS, ids=[n for n, _ in pins.F32_CHECKS])
def test_f32_pin(name, check):
    check(_sweep)


def test_round_f32_ties_and_neighbours():
    from fractions import Fraction
    one = Fraction(1)
    ulp = Fraction(1, 2 ** 23)
    # exactly halfway between 1 and its successor: ties to the even significand (1)
    assert pins.round_f32(one + ulp / 2) == np.float32(1.0)
    # halfway between the successor and the next: ties to the even one above
    assert pins.round_f32(one + ulp + ulp / 2) == np.float32(1.0) + np.float32(2 * 2.0 ** -23)
    # a hair above halfway rounds up
    assert pins.round_f32(one + ulp / 2 + Fraction(1, 2 ** 60)) == np.nextafter(np.float32(1), np.float32(2))
    # a case where rounding through float64 first would round twice:
    # 1 + 2^-24 + 2^-54 is above the tie, but its float64 is the tie itself
    x = one + Fraction(1, 2 ** 24) + Fraction(1, 2 ** 54)
    assert np.float32(float(x)) == np.float32(1.0)
    assert pins.round_f32(x) == np.nextafter(np.float32(1), np.float32(2))


def test_dyadic_f32_bitwise():
    # m + qT = 3 + 3*7 = 24 fits the float32 mantissa
    pins.check_dyadic(_sweep, 2, "star", 1, q=3, m=3, T=7, dtype=np.float32)
    pins.check_dyadic(_sweep, 3, "star", 1, q=3, m=3, T=7, dtype=np.float32)


def test_thread_count_invariance():
    w = wl.random_coeffs(2, "box", 2, 41)
    u0 = wl.make_field((37, 53), 2, 41)
    a = oracle.sweep(w, 2, u0, 9, threads=1)
    b = oracle.sweep(w, 2, u0, 9, threads=5)
    assert np.array_equal(a, b)


def test_f32_twin_close_to_f64():
    w = wl.random_coeffs(3, "star", 2, 43)
    u0 = wl.make_field((9, 10, 11), 2, 43)
    a = oracle.sweep(w, 2, u0, 10)
    b = oracle.sweep(w, 2, u0.astype(np.float32), 10)
    assert b.dtype == np.float32
    assert np.max(np.abs(a - b)) < 1e-5


def test_t0_is_copy():
    w = wl.random_coeffs(2, "star", 1, 1)
    u0 = wl.make_field((4, 5), 1, 1)
    assert np.array_equal(oracle.sweep(w, 1, u0, 0), u0)


def test_single_point_recursion_3d_box():
    w = wl.random_coeffs(3, "box", 1, 47)
    u0 = wl.make_field((4, 3, 5), 1, 47)
    ref = brute.brute_field(w, 1, u0, 2)
    got = oracle.sweep(w, 1, u0, 2)
    assert np.max(np.abs(ref - got)) < 1e-14


def test_rejects_bad_arguments():
    u0 = np.zeros((5, 5))
    with pytest.raises(ValueError):
        oracle.sweep(np.zeros((5, 5)), 1, u0, 1)  # wrong coefficient box
    with pytest.raises(ValueError):
        oracle.sweep(np.zeros((3, 3)), 1, u0, -1)  # negative T

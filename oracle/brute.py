"""Independent pure-Python checkers that pin the oracle sweep.

TEST INFRASTRUCTURE (see the package docstring). None of these functions calls
the C sweep; each reaches U^T by a different route:

* ``brute_field`` -- the recursive definition evaluated point by point with
  memoisation: U^s(i) = U^0(i) on the halo or at s = 0, else
  sum_p w_p U^{s-1}(i+p) (paper Section 2.1, Listings 1-3; halo reading as in
  the oracle header). Summation uses Python floats in dense-box order, so it
  matches the sweep to rounding, not bitwise.
* ``exact_dyadic`` -- the same recursion in exact integer arithmetic for dyadic
  weights w_p = n_p / 2^q and integer inputs. While m + q*T stays within the
  mantissa (53 bits for float64, 24 for float32) every floating-point
  operation of any summation order is exact, so a floating-point sweep must
  equal this result bit for bit.
* ``mode_eigenvalue`` / ``binomial_impulse`` -- closed forms: a Fourier mode
  cos(theta.x) is multiplied by lambda = sum_p w_p exp(i theta.p) per step away
  from the boundary, and the 1D (1/4, 1/2, 1/4) kernel applied T times to an
  impulse gives C(2T, T+j) / 4^T.
"""
from __future__ import annotations

import cmath
import itertools
import math
from functools import lru_cache

import numpy as np


def taps(coeffs: np.ndarray, r: int):
    """Non-zero taps as [(offset tuple, weight)] in dense-box order (slowest axis first)."""
    c = np.asarray(coeffs, dtype=np.float64)
    ndim = c.ndim
    out = []
    for off in itertools.product(range(-r, r + 1), repeat=ndim):
        w = float(c[tuple(o + r for o in off)])
        if w != 0.0:
            out.append((off, w))
    return out


def _is_halo(idx, shape, r):
    return any(i < r or i >= s - r for i, s in zip(idx, shape))


def brute_field(coeffs: np.ndarray, r: int, u0: np.ndarray, T: int) -> np.ndarray:
    """U^T for every cell by memoised recursion (tiny grids only)."""
    tp = taps(coeffs, r)
    shape = u0.shape
    base = u0.astype(np.float64)

    @lru_cache(maxsize=None)
    def f(idx, s):
        if s == 0 or _is_halo(idx, shape, r):
            return float(base[idx])
        acc = 0.0
        for off, w in tp:
            nb = tuple(i + o for i, o in zip(idx, off))
            acc += w * f(nb, s - 1)
        return acc

    out = np.empty(shape, dtype=np.float64)
    for idx in itertools.product(*[range(s) for s in shape]):
        out[idx] = f(idx, T)
    return out


def exact_dyadic(numerators: np.ndarray, q: int, r: int, u0_int: np.ndarray, T: int):
    """Exact U^T * 2^(q*T) as an object array of Python ints.

    ``numerators`` is the dense integer weight box n_p (weights n_p / 2^q);
    ``u0_int`` holds integer initial values (halo included).
    """
    n = np.asarray(numerators)
    ndim = n.ndim
    tp = []
    for off in itertools.product(range(-r, r + 1), repeat=ndim):
        v = int(n[tuple(o + r for o in off)])
        if v != 0:
            tp.append((off, v))
    shape = u0_int.shape
    cur = np.empty(shape, dtype=object)
    for idx in itertools.product(*[range(s) for s in shape]):
        cur[idx] = int(u0_int[idx])
    u0o = cur.copy()
    for s in range(1, T + 1):
        nxt = np.empty(shape, dtype=object)
        for idx in itertools.product(*[range(sz) for sz in shape]):
            if _is_halo(idx, shape, r):
                nxt[idx] = u0o[idx] << (q * s)
            else:
                acc = 0
                for off, v in tp:
                    acc += v * cur[tuple(i + o for i, o in zip(idx, off))]
                nxt[idx] = acc
        cur = nxt
    return cur


def mode_eigenvalue(coeffs: np.ndarray, r: int, theta) -> complex:
    """lambda = sum_p w_p exp(i theta.p) for the mode exp(i theta.x)."""
    lam = 0j
    for off, w in taps(coeffs, r):
        lam += w * cmath.exp(1j * sum(t * o for t, o in zip(theta, off)))
    return lam


def binomial_impulse(T: int, j: int) -> float:
    """T-fold (1/4, 1/2, 1/4) applied to a unit impulse, at distance j."""
    if abs(j) > T:
        return 0.0
    return math.comb(2 * T, T + j) / 4.0 ** T

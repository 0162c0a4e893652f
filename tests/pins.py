"""Checks that pin a stencil sweep against facts fixed by mathematics.

Each ``check_*`` takes a ``sweep(coeffs, r, u0, T)`` callable and raises
AssertionError on a mismatch. ``test_oracle_pins.py`` runs them on the oracle;
``test_oracle_mutants.py`` runs them on deliberately broken copies of the
oracle to show that each plausible mistake is caught by at least one check.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import brute
from paper_2305_07390_amd import workloads as wl

EPS64 = np.finfo(np.float64).eps


def _asym_weights(ndim, kind, r, seed):
    """Positive, deliberately asymmetric weights summing to 1."""
    return wl.random_coeffs(ndim, kind, r, seed)


def check_constant(sweep, ndim=2, kind="star", r=1, T=7, c=0.37, seed=11):
    """Sum of weights 1 and a constant field (halo included) => U^T stays constant."""
    w = _asym_weights(ndim, kind, r, seed)
    shape = tuple([9 + 2 * r + d for d in range(ndim)])
    u0 = np.full(shape, c)
    uT = sweep(w, r, u0, T)
    k = np.count_nonzero(w)
    tol = 4 * T * k * EPS64 * c
    assert np.max(np.abs(uT - c)) <= tol, ("constant not preserved", np.max(np.abs(uT - c)))


def check_sine_mode(sweep, ndim=2, kind="star", T=9, seed=5):
    """Per-axis symmetric r=1 weights on a zero halo: prod_j sin(m_j pi i_j/(n_j+1)) is an
    eigenvector with lambda = sum_p w_p prod_j cos(theta_j p_j), so U^T = lambda^T U^0."""
    rng = np.random.default_rng(seed)
    r = 1
    n = [7 + 3 * d for d in range(ndim)]
    m = [1 + d for d in range(ndim)]
    theta = [mj * math.pi / (nj + 1) for mj, nj in zip(m, n)]
    # weights depend only on |p_j| (per-axis reflection symmetry)
    a = {}
    w = np.zeros((3,) * ndim)
    for off in wl.offsets(ndim, kind, 1):
        key = tuple(abs(o) for o in off)
        if key not in a:
            a[key] = rng.uniform(0.2, 1.0)
        w[tuple(o + 1 for o in off)] = a[key]
    w /= w.sum()
    lam = 0.0
    for off in wl.offsets(ndim, kind, 1):
        lam += w[tuple(o + 1 for o in off)] * np.prod([math.cos(t * o) for t, o in zip(theta, off)])
    grids = np.meshgrid(*[np.arange(nj + 2) for nj in n], indexing="ij")
    u0 = np.ones([nj + 2 for nj in n])
    for t, g in zip(theta, grids):
        u0 = u0 * np.sin(t * g)
    # exact zeros on the halo
    for d in range(ndim):
        idx = [slice(None)] * ndim
        idx[d] = 0
        u0[tuple(idx)] = 0.0
        idx[d] = -1
        u0[tuple(idx)] = 0.0
    uT = sweep(w, r, u0, T)
    expect = lam ** T * u0
    err = np.max(np.abs(uT - expect))
    assert err <= 64 * T * EPS64, ("sine mode decay mismatch", err, lam)


def check_cos_mode(sweep, ndim=2, kind="box", r=2, T=3, seed=7, theta=None):
    """Any weights, any r: far from the halo (Chebyshev distance > r T), a mode
    cos(theta.x) becomes |lambda|^T cos(theta.x + T arg lambda)."""
    w = _asym_weights(ndim, kind, r, seed)
    if theta is None:
        theta = [0.31 + 0.17 * d for d in range(ndim)][::-1]
    n = [2 * r * T + 6 + 2 * d for d in range(ndim)]
    shape = [nj + 2 * r for nj in n]
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    phase = sum(t * g for t, g in zip(theta, grids))
    u0 = np.cos(phase)
    uT = sweep(w, r, u0, T)
    lam = brute.mode_eigenvalue(w, r, theta)
    expect = abs(lam) ** T * np.cos(phase + T * np.angle(lam))
    core = tuple(slice(r + r * T, s - r - r * T) for s in shape)
    err = np.max(np.abs(uT[core] - expect[core]))
    assert err <= 1e-13, ("cos mode mismatch", err)


def check_linear(sweep, ndim=2, kind="box", r=2, T=6, seed=3):
    """Point-symmetric weights summing to 1 leave a linear field (halo included) unchanged."""
    rng = np.random.default_rng(seed)
    w = np.zeros((2 * r + 1,) * ndim)
    for off in wl.offsets(ndim, kind, r):
        neg = tuple(-o for o in off)
        if w[tuple(o + r for o in neg)] != 0.0:
            w[tuple(o + r for o in off)] = w[tuple(o + r for o in neg)]
        else:
            w[tuple(o + r for o in off)] = rng.uniform(0.1, 1.0)
    w /= w.sum()
    shape = [8 + 2 * r + 3 * d for d in range(ndim)]
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    coef = [0.013 * (d + 1) for d in range(ndim)]
    u0 = 0.25 + sum(c * g for c, g in zip(coef, grids))
    uT = sweep(w, r, u0, T)
    err = np.max(np.abs(uT - u0))
    assert err <= 32 * T * EPS64, ("linear field changed", err)


def check_brute(sweep, ndim=2, kind="box", r=1, T=3, seed=13):
    """Match the memoised point-by-point recursion on a tiny, non-square grid."""
    w = _asym_weights(ndim, kind, r, seed)
    interior = [5 + 2 * d for d in range(ndim)][::-1]
    u0 = wl.make_field(interior, r, seed)
    uT = sweep(w, r, u0, T)
    ref = brute.brute_field(w, r, u0, T)
    err = np.max(np.abs(uT - ref))
    assert err <= 1e-14, ("brute-force mismatch", err)


def dyadic_case(ndim, kind, r, q, m, seed, interior):
    """Integer weights n_p >= 1 on the stencil's points summing to 2^q (random split),
    and integer inputs in [0, 2^m)."""
    rng = np.random.default_rng(seed)
    pts = wl.offsets(ndim, kind, r)
    k = len(pts)
    total = 2 ** q
    if k > total:
        raise ValueError("need 2^q >= number of points")
    cuts = np.sort(rng.choice(np.arange(1, total), size=k - 1, replace=False))
    parts = np.diff(np.concatenate([[0], cuts, [total]])).astype(np.int64)
    nbox = np.zeros((2 * r + 1,) * ndim, dtype=np.int64)
    for off, v in zip(pts, parts):
        nbox[tuple(o + r for o in off)] = v
    shape = [s + 2 * r for s in interior]
    u0_int = rng.integers(0, 2 ** m, size=shape, dtype=np.int64)
    return nbox, u0_int


def check_dyadic(sweep, ndim=2, kind="star", r=1, q=3, m=5, T=16, seed=17, dtype=np.float64,
                 interior=None):
    """Dyadic weights and integer inputs: every FP operation is exact while
    m + qT fits the mantissa, so the sweep must equal exact integer arithmetic."""
    if interior is None:
        interior = [6 + d for d in range(ndim)]
    nbox, u0_int = dyadic_case(ndim, kind, r, q, m, seed, interior)
    w = nbox.astype(np.float64) / 2.0 ** q
    u0 = u0_int.astype(dtype)
    uT = sweep(w, r, u0, T)
    exact = brute.exact_dyadic(nbox, q, r, u0_int, T)
    scale = 2.0 ** (q * T)
    got = uT.astype(np.float64) * scale
    want = np.vectorize(float)(exact)
    assert np.array_equal(got, want), ("dyadic mismatch", np.max(np.abs(got - want)))


def check_binomial(sweep, T=6):
    """(1/4, 1/2, 1/4) along x on a unit impulse gives C(2T, T+j)/4^T (exact)."""
    w = np.zeros((3, 3))
    w[1, 0], w[1, 1], w[1, 2] = 0.25, 0.5, 0.25
    u0 = np.zeros((7, 4 * T + 5))
    y0, x0 = 3, (4 * T + 5) // 2
    u0[y0, x0] = 1.0
    uT = sweep(w, 1, u0, T)
    for j in range(-T - 1, T + 2):
        assert uT[y0, x0 + j] == brute.binomial_impulse(T, j), ("binomial", j, uT[y0, x0 + j])
    # no spread along y
    assert np.all(uT[y0 - 1] == 0.0) and np.all(uT[y0 + 1] == 0.0)


def check_r0(sweep, T=9, seed=2):
    """r = 0: U^T = w0^T U^0 by repeated rounding multiplication."""
    rng = np.random.default_rng(seed)
    w0 = 0.93
    u0 = rng.random((5, 6))
    uT = sweep(np.array([[w0]]), 0, u0, T)
    ref = u0.copy()
    for _ in range(T):
        ref = w0 * ref
    assert np.array_equal(uT, ref), "r=0 scaling mismatch"


def check_max_principle(sweep, ndim=3, kind="box", r=1, T=5, seed=19):
    """Non-negative weights summing to 1 keep U^T within [min U^0, max U^0]."""
    w = _asym_weights(ndim, kind, r, seed)
    u0 = wl.make_field([6 + d for d in range(ndim)], r, seed)
    uT = sweep(w, r, u0, T)
    slack = 8 * T * EPS64
    assert uT.min() >= u0.min() - slack and uT.max() <= u0.max() + slack


def check_composition(sweep, ndim=2, kind="star", r=2, T1=3, T2=4, seed=23):
    """run(T1 + T2) == run(T2) after run(T1), bit for bit."""
    w = _asym_weights(ndim, kind, r, seed)
    u0 = wl.make_field([11 + d for d in range(ndim)], r, seed)
    a = sweep(w, r, u0, T1 + T2)
    b = sweep(w, r, sweep(w, r, u0, T1), T2)
    assert np.array_equal(a, b)


def check_dependence(sweep, ndim=2, kind="star", r=2, T=3, seed=29):
    """A perturbation of one cell reaches exactly the cells within T steps of the
    stencil's reach: box => Chebyshev distance <= rT; star => sum_j ceil(|d_j|/r) <= T."""
    w = _asym_weights(ndim, kind, r, seed)
    n = [2 * r * T + 9 for _ in range(ndim)]
    u0 = wl.make_field(n, r, seed)
    base = sweep(w, r, u0, T)
    c = tuple(s // 2 + r for s in n)
    u1 = u0.copy()
    u1[c] += 0.5
    pert = sweep(w, r, u1, T)
    changed = pert != base
    grids = np.meshgrid(*[np.arange(s) for s in u0.shape], indexing="ij")
    d = [np.abs(g - ci) for g, ci in zip(grids, c)]
    if kind == "box":
        reach = np.maximum.reduce(d) <= r * T
    else:
        reach = sum(np.ceil(di / r) for di in d) <= T
    assert not np.any(changed & ~reach), "perturbation leaked outside the dependence cone"
    # the tips of the cone (along each axis, at distance rT) do change
    for ax in range(ndim):
        tip = list(c)
        tip[ax] += r * T
        assert changed[tuple(tip)], ("cone tip unchanged", ax)


def check_halo_fixed(sweep, ndim=3, kind="star", r=2, T=4, seed=31):
    """Halo cells keep their initial values bit for bit."""
    w = _asym_weights(ndim, kind, r, seed)
    u0 = wl.make_field([5 + d for d in range(ndim)], r, seed)
    uT = sweep(w, r, u0, T)
    mask = np.ones(u0.shape, dtype=bool)
    mask[tuple(slice(r, s - r) for s in u0.shape)] = False
    assert np.array_equal(uT[mask], u0[mask])


def round_f32(x) -> np.float32:
    """The float32 nearest to the exact rational x, ties to an even significand
    (IEEE 754 round-to-nearest-even), found among the neighbours of a first
    guess by exact comparison (converting through float64 first could round
    twice)."""
    from fractions import Fraction
    x = Fraction(x)
    if x == 0:
        return np.float32(0.0)
    f = np.float32(float(x))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        if not np.isfinite(c):
            continue
        key = (abs(Fraction(float(c)) - x), int(np.array(c, dtype=np.float32).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, np.float32(c))
    return best[1]


def fmaf_exact(a, b, c) -> np.float32:
    """a * b + c computed exactly and rounded once to float32."""
    from fractions import Fraction
    return round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def f32_reference(coeffs, r, u0, T):
    """The float32 twin's definition on exact rationals: coefficients rounded
    once to float32, each cell summed in dense-box order from +0 with one
    rounding per term (a fused multiply-add), the halo held."""
    ndim = u0.ndim
    offs = [o for o in np.ndindex(*coeffs.shape) if coeffs[o] != 0.0]
    w32 = [np.float32(coeffs[o]) for o in offs]
    cur = u0.astype(np.float32).copy()
    inner = [range(r, s - r) for s in u0.shape]
    for _ in range(T):
        nxt = cur.copy()
        for idx in np.ndindex(*[len(x) for x in inner]):
            cell = tuple(i + r for i in idx)
            acc = np.float32(0.0)
            for o, w in zip(offs, w32):
                nb = tuple(c + oo - r for c, oo in zip(cell, o))
                acc = fmaf_exact(w, cur[nb], acc)
            nxt[cell] = acc
        cur = nxt
    return cur


def check_f32_rounding(sweep, ndim=2, kind="box", r=1, T=3, seed=23):
    """float32 sweep equals the exact-rational definition of one fused
    multiply-add per term, bit for bit (random weights and values, so the
    rounding of every term matters)."""
    w = wl.random_coeffs(ndim, kind, r, seed)
    interior = (4, 5) if ndim == 2 else (3, 4, 5)
    u0 = wl.make_field(interior, r, seed, np.float32)
    ref = f32_reference(w, r, u0, T)
    got = sweep(w, r, u0, T)
    assert got.dtype == np.float32
    assert np.array_equal(got, ref), ("float32 rounding differs", np.max(np.abs(got.astype(np.float64) - ref)))


F32_CHECKS = (
    ("f32_exact_2d_box", lambda s: check_f32_rounding(s, 2, "box", 1)),
    ("f32_exact_3d_star_r2", lambda s: check_f32_rounding(s, 3, "star", 2, T=2, seed=29)),
)


ALL_CHECKS = (
    ("constant_2d_star", lambda s: check_constant(s, 2, "star", 1)),
    ("constant_3d_box_r2", lambda s: check_constant(s, 3, "box", 2, T=3)),
    ("sine_2d_star", lambda s: check_sine_mode(s, 2, "star")),
    ("sine_2d_box", lambda s: check_sine_mode(s, 2, "box")),
    ("sine_3d_star", lambda s: check_sine_mode(s, 3, "star", T=5)),
    ("cos_2d_box_r2", lambda s: check_cos_mode(s, 2, "box", 2)),
    ("cos_2d_star_r3", lambda s: check_cos_mode(s, 2, "star", 3, T=2)),
    ("cos_3d_star_r1", lambda s: check_cos_mode(s, 3, "star", 1, T=3)),
    ("linear_2d_box", lambda s: check_linear(s, 2, "box", 2)),
    ("linear_3d_star", lambda s: check_linear(s, 3, "star", 1, T=4)),
    ("brute_2d_box", lambda s: check_brute(s, 2, "box", 1)),
    ("brute_2d_star_r2", lambda s: check_brute(s, 2, "star", 2, T=2)),
    ("brute_3d_star", lambda s: check_brute(s, 3, "star", 1, T=2)),
    ("dyadic_2d_star", lambda s: check_dyadic(s, 2, "star", 1)),
    ("dyadic_2d_box", lambda s: check_dyadic(s, 2, "box", 1, q=4, m=5, T=12)),
    ("dyadic_3d_star", lambda s: check_dyadic(s, 3, "star", 1, T=8)),
    ("binomial", check_binomial),
    ("r0", check_r0),
    ("max_principle", check_max_principle),
    ("composition", check_composition),
    ("dependence_star", lambda s: check_dependence(s, 2, "star", 2)),
    ("dependence_box", lambda s: check_dependence(s, 2, "box", 1)),
    ("halo_fixed", check_halo_fixed),
)

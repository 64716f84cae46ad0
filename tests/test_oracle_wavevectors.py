"""Pins for the oracle's wavevector set H(R2), its counts and the chi -> R2 rule.

Independent checks: Jacobi's two- and four-square theorems (counts of lattice
vectors on a shell), Legendre's three-square theorem (empty shells in d=3),
brute force over the integer grid in numpy, and Python's sort for the order.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O


def r2_jacobi(s: int) -> int:
    """Number of (a, b) in Z^2 with a^2 + b^2 = s: 4 (d_1(s) - d_3(s))."""
    if s == 0:
        return 1
    d1 = sum(1 for q in range(1, s + 1) if s % q == 0 and q % 4 == 1)
    d3 = sum(1 for q in range(1, s + 1) if s % q == 0 and q % 4 == 3)
    return 4 * (d1 - d3)


def r4_jacobi(s: int) -> int:
    """Number of representations as a sum of four squares: 8 * sum of divisors not divisible by 4."""
    if s == 0:
        return 1
    return 8 * sum(q for q in range(1, s + 1) if s % q == 0 and q % 4 != 0)


def brute_counts(d: int, R2: int) -> np.ndarray:
    R = math.isqrt(R2)
    axes = np.meshgrid(*[np.arange(-R, R + 1)] * d, indexing="ij")
    s = sum(a * a for a in axes).ravel()
    c = np.bincount(s[s <= R2], minlength=R2 + 1)
    c[0] = 0
    return c // 2   # half of the nonzero vectors on each shell


@pytest.mark.parametrize("R2", list(range(1, 41)) + [64, 97, 150])
def test_count_d2_jacobi(R2):
    expect = sum(r2_jacobi(s) for s in range(1, R2 + 1)) // 2
    assert O.count(2, R2) == expect


@pytest.mark.parametrize("R2", list(range(1, 25)) + [40, 57])
def test_count_d4_jacobi(R2):
    expect = sum(r4_jacobi(s) for s in range(1, R2 + 1)) // 2
    assert O.count(4, R2) == expect


@pytest.mark.parametrize("R2", [1, 2, 5, 17, 100, 400])
def test_count_d1(R2):
    assert O.count(1, R2) == math.isqrt(R2)


def test_count_d3_brute_and_legendre():
    c = brute_counts(3, 300)
    for R2 in range(1, 301):
        assert O.count(3, R2) == int(c[1:R2 + 1].sum())
    # shells 4^a (8b + 7) are empty (Legendre), all others are not
    for s in range(1, 301):
        t = s
        while t % 4 == 0:
            t //= 4
        assert (c[s] == 0) == (t % 8 == 7)


def brute_cutoff(d, N, chi):
    T = chi * d * (N - 1)
    R2max = 1
    while True:
        c = brute_counts(d, R2max * R2max)
        cum = np.cumsum(c)
        if cum[-1] > T:
            ok = [s for s in range(1, len(c)) if c[s] > 0 and cum[s] <= T]
            s = max(ok)
            return s, int(cum[s])
        R2max += 1


@pytest.mark.parametrize("d,N,chi,R2,M", [
    (2, 128, 0.40, 64, 98),         # the d=2, N=128, chi=0.4 quench
    (3, 8000, 0.45, 297, 10779),    # the d=3, N=8000, chi=0.45 evaluation
    (3, 30000, 0.45, 721, 40494),   # the d=3, N=30000, chi=0.45 staged run
])
def test_cutoff_named_workloads(d, N, chi, R2, M):
    assert O.cutoff(d, N, chi) == (R2, M)
    assert brute_cutoff(d, N, chi) == (R2, M)
    assert M / (d * (N - 1)) <= chi


def test_cutoff_random_against_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(25):
        d = int(rng.integers(1, 5))
        N = int(rng.integers(20, 800))
        chi = float(rng.uniform(0.05, 0.49))
        if chi * d * (N - 1) < 1:
            continue
        assert O.cutoff(d, N, chi) == brute_cutoff(d, N, chi)


def test_cutoff_rejects_invalid():
    for args in [(0, 100, 0.3), (5, 100, 0.3), (2, 1, 0.3), (2, 100, 0.5), (2, 100, 0.0), (2, 3, 0.1)]:
        with pytest.raises(ValueError):
            O.cutoff(*args)


@pytest.mark.parametrize("d,R2", [(1, 9), (2, 1), (2, 64), (3, 20), (3, 61), (4, 12)])
def test_wavevector_order_against_python_sort(d, R2):
    R = math.isqrt(R2)
    vecs = []
    for n in itertools.product(range(-R, R + 1), repeat=d):
        s = sum(x * x for x in n)
        nz = [x for x in n if x != 0]
        if 0 < s <= R2 and nz[0] > 0:
            vecs.append((s, n))
    vecs.sort()
    expect = np.array([n for _, n in vecs], dtype=np.int32).reshape(-1, d)
    got = O.wavevectors(d, R2)
    assert got.dtype == np.int32 and got.shape == expect.shape
    assert np.array_equal(got, expect)
    # inversion closure: H and -H partition the nonzero vectors in the ball
    full = {tuple(x) for x in got} | {tuple(-x) for x in got}
    assert len(full) == 2 * len(got)

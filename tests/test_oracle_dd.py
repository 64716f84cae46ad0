"""Pins for the oracle's double-double arithmetic, phase reduction and sin/cos.

Each check compares against something other than the oracle: exact rationals
(fractions.Fraction) or 256-bit mpmath.  Tolerances are the published error
bounds of the algorithms (u = 2^-53, u^2 = 2^-106) with a small margin.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
import mpref

U2 = 2.0 ** -106
rng = np.random.default_rng(20230418)


def rand_dd(scale=1.0, n=1):
    out = []
    for _ in range(n):
        hi = float(rng.standard_normal() * scale * 2.0 ** rng.integers(-8, 8))
        lo = float(rng.uniform(-0.5, 0.5) * np.spacing(abs(hi))) if hi != 0 else 0.0
        out.append(np.array([hi, lo]))
    return out


def rel_err(res, exact: Fraction):
    got = Fraction(float(res[0])) + Fraction(float(res[1]))
    if exact == 0:
        return abs(float(got))
    return abs(float((got - exact) / exact))


def test_add_mul_div_sqrt_against_rationals():
    for _ in range(3000):
        a, b = rand_dd(n=2)
        if rng.random() < 0.3:  # force heavy cancellation in the sum
            b = np.array([-a[0], float(rng.uniform(-0.5, 0.5) * np.spacing(abs(a[0])))])
        fa, fb = mpref.frac_of(*a), mpref.frac_of(*b)
        assert rel_err(O.dd_add(a, b), fa + fb) <= 3.0 * U2 * 1.001
        assert rel_err(O.dd_mul(a, b), fa * fb) <= 4.0 * U2 * 1.001
        if fb != 0:
            assert rel_err(O.dd_div(a, b), fa / fb) <= 16.0 * U2
        aa = np.abs(a) * np.sign(a[0]) if a[0] != 0 else a
        faa = mpref.frac_of(*aa)
        if faa > 0:
            r = O.dd_sqrt(aa)
            exact = mpref.ctx.sqrt(mpref.mp_of(*aa))
            got = mpref.mp_of(*r)
            assert abs((got - exact) / exact) <= 8.0 * U2


def test_normalised_outputs():
    for _ in range(500):
        a, b = rand_dd(n=2)
        for r in (O.dd_add(a, b), O.dd_mul(a, b)):
            assert r[0] + r[1] == r[0]           # |lo| <= ulp(hi)/2


def test_two_pi_constant():
    tp = O.two_pi()
    exact = 2 * mpref.ctx.pi
    err = abs(mpref.mp_of(*tp) - exact)
    assert err <= np.spacing(tp[1]) / 2 * 1.0000001
    assert tp[0] + tp[1] == tp[0]


def _rand_u():
    hi = float(rng.uniform(-3.0, 4.0)) if rng.random() < 0.3 else float(rng.random())
    if rng.random() < 0.05:
        hi = float(rng.random() * 2.0 ** -30)
    lo = float(rng.uniform(-0.5, 0.5) * np.spacing(abs(hi))) if hi != 0 else 0.0
    return hi, lo


def test_phase_exact_against_rationals():
    for d in (1, 2, 3, 4):
        for _ in range(400):
            n = rng.integers(-1024, 1025, size=d).astype(np.int32)
            us = [_rand_u() for _ in range(d)]
            uhi = np.array([u[0] for u in us])
            ulo = np.array([u[1] for u in us])
            t = O.phase(n, uhi, ulo)
            exact = mpref.phase_exact(n, uhi, ulo)
            got = Fraction(float(t[0])) + Fraction(float(t[1]))
            assert abs(float(got - exact)) <= 2.0 ** -107 * 1.0001
            assert abs(t[0]) <= 0.5
            assert t[0] + t[1] == t[0]


def test_phase_integer_and_half_cases():
    # exact integers reduce to zero; exact halves stay at +-1/2
    t = O.phase(np.array([1, 2], np.int32), np.array([0.5, 0.5]), np.array([0.0, 0.0]))   # 1.5
    assert abs(t[0]) == 0.5 and t[1] == 0.0
    t = O.phase(np.array([3, -5], np.int32), np.array([0.25, 0.75]), np.array([0.0, 0.0]))  # -3
    assert t[0] == 0.0 and t[1] == 0.0
    t = O.phase(np.array([4, 8], np.int32), np.array([0.25, 0.125]), np.array([0.0, 0.0]))
    assert t[0] == 0.0 and t[1] == 0.0


@pytest.mark.parametrize("t", [0.0, 0.125, -0.125, 0.25, -0.25, 0.5, -0.5, 1.0 / 3, 0.0625, 1e-20])
def test_sincos_special_points(t):
    th, tl = mpref.to_dd(mpref.ctx.mpf(t))
    c, s = O.sincos2pi([th, tl])
    tt = mpref.mp_of(th, tl)
    assert abs(mpref.mp_of(*c) - mpref.ctx.cospi(2 * tt)) <= 2 * U2
    assert abs(mpref.mp_of(*s) - mpref.ctx.sinpi(2 * tt)) <= 2 * U2


def test_sincos_random_against_mpmath():
    worst = 0.0
    for _ in range(3000):
        th = float(rng.uniform(-0.5, 0.5))
        tl = float(rng.uniform(-0.5, 0.5) * np.spacing(abs(th)))
        c, s = O.sincos2pi([th, tl])
        tt = mpref.mp_of(th, tl)
        ec = abs(mpref.mp_of(*c) - mpref.ctx.cospi(2 * tt))
        es = abs(mpref.mp_of(*s) - mpref.ctx.sinpi(2 * tt))
        worst = max(worst, float(ec), float(es))
        one = mpref.mp_of(*c) ** 2 + mpref.mp_of(*s) ** 2 - 1
        assert abs(one) <= 8 * U2
    # a dropped Taylor term (the smallest kept one is ~1.5e-31 at pi/4) would fail this
    assert worst <= 4 * U2, worst

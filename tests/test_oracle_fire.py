"""Pins for the oracle's FIRE minimiser (the paper's minimiser, "Simulations";
Bitzek et al., Phys. Rev. Lett. 97, 170201 (2006)).

Independent checks: a second 256-bit implementation of the same published
algorithm (tests/mpref.py) on a separable quadratic (20 iterations, so the step
grows past N_min and the velocity mixing and freezing branches both run) and on
a small stealthy system; the first step from rest in closed form; and, from the
paper's landscape fact (chi < 1/2: every quench from a random start reaches a
ground state), a full d=2, N=128 quench reaching the stated floor.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_09139_amd import inputs
import mpref

ctx = mpref.ctx


def quad_case(seed=5, nv=12):
    rng = np.random.default_rng(seed)
    w = np.exp(rng.uniform(np.log(0.1), np.log(10.0), nv))
    c = rng.uniform(-1, 1, nv)
    x0 = rng.uniform(-1, 1, nv)
    return w, c, x0


def test_first_step_closed_form():
    """From rest P = 0: the step halves, v = -dt g, so x1 = x0 - (dt0 / 2)^2 g0 with
    dt0^2 = step_cap / max|g0| (nmean = 1 for the test objective)."""
    w, c, x0 = quad_case()
    g0 = w * (x0 - c)
    x1 = x0 - 1e-2 / (4.0 * np.max(np.abs(g0))) * g0
    x, res, _ = O.minimize_quadratic(np.stack([w, 0 * w]), np.stack([c, 0 * c]), np.stack([x0, 0 * x0]),
                                     max_iter=1, s_floor=0.0, method="fire")
    assert res["iters"] == 1
    assert np.max(np.abs((x[0] + x[1]) - x1)) <= 1e-15


def test_quadratic_iterates_match_256bit():
    w, c, x0 = quad_case()
    W = np.stack([w, np.zeros_like(w)])
    Cc = np.stack([c, np.zeros_like(c)])
    X0 = np.stack([x0, np.zeros_like(x0)])
    fg = mpref.quadratic_fg([ctx.mpf(float(t)) for t in w], [ctx.mpf(float(t)) for t in c])
    for iters in (1, 2, 6, 8, 20):
        x, res, tr = O.minimize_quadratic(W, Cc, X0, trace_cap=iters + 1, max_iter=iters, s_floor=0.0,
                                          method="fire")
        assert res["iters"] == iters and res["evals"] == iters + 1
        xm, trm = mpref.fire_mp(fg, [ctx.mpf(float(t)) for t in x0], 1.0, iters)
        for i in range(iters + 1):
            assert abs(mpref.mp_of(*tr[i]) - trm[i]) <= 1e-26 * abs(trm[i]), (iters, i)
        for i in range(len(w)):
            assert abs(mpref.mp_of(x[0, i], x[1, i]) - xm[i]) <= 1e-26
    # and it converges
    x, res, _ = O.minimize_quadratic(W, Cc, X0, s_floor=1e-50, max_iter=20000, method="fire")
    assert res["status"] == "converged"


def test_small_stealthy_iterates_match_256bit():
    d, N, R2 = 2, 10, 4
    n = O.wavevectors(d, R2)
    pos = inputs.uniform_positions(d, N, 13)
    fg = mpref.stealthy_fg(n, None, N, d)
    x0 = [mpref.mp_of(pos[0, a, j], pos[1, a, j]) for a in range(d) for j in range(N)]
    iters = 8
    x, res, tr = O.minimize(n, None, pos, trace_cap=iters + 1, max_iter=iters, s_floor=0.0, method="fire")
    xm, trm = mpref.fire_mp(fg, x0, mpref.nmean_of(N, d), iters)
    for i in range(iters + 1):
        assert abs(mpref.mp_of(*tr[i]) - trm[i]) <= 1e-26 * abs(trm[i])
    for a in range(d):
        for j in range(N):
            assert abs(mpref.mp_of(x[0, a, j], x[1, a, j]) - xm[a * N + j]) <= 1e-26


@pytest.mark.slow
def test_fire_quench_reaches_floor_d2_N128():
    d, N, chi = 2, 128, 0.4
    R2, M = O.cutoff(d, N, chi)
    n = O.wavevectors(d, R2)
    pos = inputs.config_positions(1, d, N, 0)
    x, res, _ = O.minimize(n, None, pos, method="fire", stall_window=200)
    assert res["status"] == "converged", res
    e = O.energy_from_nk(N, None, O.nk(n, x))
    assert e.smax[0] <= 1e-40 * (1 + 1e-6)

"""Pins for the oracle's L-BFGS minimiser.

The paper quenches with FIRE ("Simulations" section); this path minimises with
L-BFGS, so the rules are this build's reading and are pinned by a second,
independent 256-bit implementation of the same rules (tests/mpref.py): on a
separable quadratic and on a small stealthy system the first iterates must
agree to 1e-26 relative.  The landscape fact of the paper (for chi < 1/2 every
quench from a random start reaches a global minimum, Phi = 0) is the pin for a
full run: the d=2, N=128, chi=0.4 quench must reach the stated S(k) floor.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_09139_amd import inputs
import mpref

ctx = mpref.ctx


def test_quadratic_iterates_match_256bit():
    rng = np.random.default_rng(3)
    nv = 12
    w = np.exp(rng.uniform(np.log(0.1), np.log(10.0), nv))
    c = rng.uniform(-1, 1, nv)
    x0 = rng.uniform(-1, 1, nv)
    W = np.stack([w, np.zeros(nv)])
    Cc = np.stack([c, np.zeros(nv)])
    X0 = np.stack([x0, np.zeros(nv)])
    fg = mpref.quadratic_fg([ctx.mpf(float(t)) for t in w], [ctx.mpf(float(t)) for t in c])
    for iters in (1, 2, 3, 5, 8):
        x, res, tr = O.minimize_quadratic(W, Cc, X0, trace_cap=iters + 1, max_iter=iters, s_floor=0.0)
        assert res["iters"] == iters
        xm, trm = mpref.lbfgs_mp(fg, [ctx.mpf(float(t)) for t in x0], 1.0, iters)
        for i in range(iters + 1):
            fo = mpref.mp_of(*tr[i])
            assert abs(fo - trm[i]) <= 1e-26 * abs(trm[i]), (iters, i)
        for i in range(nv):
            assert abs(mpref.mp_of(x[0, i], x[1, i]) - xm[i]) <= 1e-26
    # converges on the quadratic
    x, res, _ = O.minimize_quadratic(W, Cc, X0, s_floor=1e-60, max_iter=500)
    assert res["status"] == "converged"
    assert np.max(np.abs(x[0] - c)) <= 1e-29


def test_small_stealthy_iterates_match_256bit():
    d, N, R2 = 2, 10, 4
    n = O.wavevectors(d, R2)
    pos = inputs.uniform_positions(d, N, 12)
    fg = mpref.stealthy_fg(n, None, N, d)
    x0 = [mpref.mp_of(pos[0, a, j], pos[1, a, j]) for a in range(d) for j in range(N)]
    iters = 6
    x, res, tr = O.minimize(n, None, pos, trace_cap=iters + 1, max_iter=iters, s_floor=0.0)
    xm, trm = mpref.lbfgs_mp(fg, x0, mpref.nmean_of(N, d), iters)
    assert len(tr) == iters + 1
    for i in range(iters + 1):
        assert abs(mpref.mp_of(*tr[i]) - trm[i]) <= 1e-26 * abs(trm[i])
    for a in range(d):
        for j in range(N):
            assert abs(mpref.mp_of(x[0, a, j], x[1, a, j]) - xm[a * N + j]) <= 1e-26


@pytest.mark.slow
def test_quench_reaches_floor_d2_N128():
    """chi = 0.4 < 1/2: a quench from a random start reaches a ground state."""
    d, N, chi = 2, 128, 0.4
    R2, M = O.cutoff(d, N, chi)
    n = O.wavevectors(d, R2)
    pos = inputs.config_positions(1, d, N, 0)
    x, res, tr = O.minimize(n, None, pos, trace_cap=100000)
    assert res["status"] == "converged"
    assert res["smax"][0] <= 1e-40
    assert np.all(np.diff(tr[:, 0]) <= 0)      # Armijo: Phi never increases
    # the final S_max is what an independent 256-bit evaluation of the final positions gives
    phi, sk, _, _ = mpref.energy_mp(n[:6], None, x)   # a few k (the full set is slow at 256 bits)
    e = O.energy_from_nk(N, None, O.nk(n, x))
    tol_nk = mpref.U_DD * (5.0 * N + 3.0 * N * N)   # oracle bound on |Delta n~| (test_oracle_energy)
    for k in range(6):
        mag = float(sk[k]) * N
        bound = (2.0 * np.sqrt(mag) * tol_nk + tol_nk ** 2) / N
        assert abs(mpref.mp_of(e.sk[0, k], e.sk[1, k]) - sk[k]) <= bound


# stopping rules: the stall window (W, ratio) and the consecutive line-search
# failure limit, on settings where each ends the run at a different iteration
# (the failure cases have isolated failures before the consecutive ones: with
# limit 1 the run ends earlier than with 2 and 3)
STOP_CASES = ([dict(stall_window=W, stall_ratio=r) for W, r in [(2, 0.5), (3, 0.1), (4, 0.01), (6, 0.01)]]
              + [dict(c1=c1, max_halvings=mh, step_cap=sc, max_ls_fail=lf)
                 for (c1, mh, sc) in [(0.3, 1, 1.0), (1e-4, 0, 0.1)] for lf in (1, 2, 3)])


@pytest.mark.parametrize("rules", STOP_CASES)
def test_stopping_rules_match_256bit(rules):
    """The oracle's stall window and consecutive-failure stop against the second
    256-bit implementation of the same rules: the same status at the same
    iteration, and the same energies along the way."""
    d, N, R2 = 2, 10, 4
    n = O.wavevectors(d, R2)
    pos = inputs.uniform_positions(d, N, 12)
    fg = mpref.stealthy_fg(n, None, N, d)
    x0 = [mpref.mp_of(pos[0, a, j], pos[1, a, j]) for a in range(d) for j in range(N)]
    okw = dict(stall_window=1000)          # no stall-window stop unless the case sets one
    okw.update(rules)
    x, res, tr = O.minimize(n, None, pos, trace_cap=200, max_iter=80, s_floor=0.0, **okw)
    xm, trm, status, iters = mpref.lbfgs_mp_run(fg, x0, mpref.nmean_of(N, d), 80, **rules)
    assert (res["status"], res["iters"]) == (status, iters) == ("stalled", iters)
    assert iters < 80
    for i in range(min(len(trm), res["iters"])):
        assert abs(mpref.mp_of(*tr[i]) - trm[i]) <= 1e-26 * trm[0], i
    assert abs(mpref.mp_of(*res["phi"]) - trm[-1]) <= 1e-26 * trm[0]


def test_stopping_rule_cases_differ():
    """The cases above end at different iterations for different limits, so an
    off-by-one in the window or the failure count would show."""
    d, N, R2 = 2, 10, 4
    n = O.wavevectors(d, R2)
    pos = inputs.uniform_positions(d, N, 12)
    ends = []
    for rules in STOP_CASES:
        okw = dict(stall_window=1000)
        okw.update(rules)
        _, res, _ = O.minimize(n, None, pos, max_iter=80, s_floor=0.0, **okw)
        ends.append(res["iters"])
    assert len(set(ends[4:7])) == 3 and len(set(ends[7:10])) == 3
    assert len(set(ends[:4])) >= 3

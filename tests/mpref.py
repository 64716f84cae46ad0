"""256-bit reference computations used to pin the oracle (test helper).

These are written directly from the paper's definitions with mpmath at
256 bits of precision (about 77 decimal digits) and Python's exact rationals,
independently of both the C oracle and the HIP library:

* n~(k) = sum_j exp(-i k . r_j) (Eq. ntilde), S(k) = |n~|^2 / N
  (Eq. structurefactor), Phi = sum over the half set of v |n~|^2 (Eq. energy
  with the constant term dropped), S_max (Eq. smax);
* the gradient by central differences of that energy;
* the L-BFGS rules of the minimiser, as a second implementation.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

ctx = mpmath.MPContext()
ctx.prec = 256
U_DD = 2.0 ** -106


def frac_of(hi, lo) -> Fraction:
    return Fraction(float(hi)) + Fraction(float(lo))


def mp_of(hi, lo):
    return ctx.mpf(float(hi)) + ctx.mpf(float(lo))


def to_dd(x) -> tuple[float, float]:
    """Round an mpf or Fraction to a normalised double-double."""
    if isinstance(x, Fraction):
        hi = float(x)
        lo = float(x - Fraction(hi))
        return hi, lo
    hi = float(x)
    lo = float(x - ctx.mpf(hi))
    return hi, lo


def phase_exact(n, uhi, ulo) -> Fraction:
    """frac(n . u) in [-1/2, 1/2], exactly."""
    x = sum(int(na) * frac_of(h, l) for na, h, l in zip(n, uhi, ulo))
    return x - round(x)


def positions_mp(pos):
    _, d, N = pos.shape
    return [[mp_of(pos[0, a, j], pos[1, a, j]) for a in range(d)] for j in range(N)]


def nk_mp(n, pos):
    """(C_k, S_k) lists of mpf with n~(k) = C - i S."""
    u = positions_mp(pos)
    Cs, Ss = [], []
    for nv in n:
        C = ctx.mpf(0)
        S = ctx.mpf(0)
        for uj in u:
            t = sum(int(na) * ua for na, ua in zip(nv, uj))
            C += ctx.cospi(2 * t)
            S += ctx.sinpi(2 * t)
        Cs.append(C)
        Ss.append(S)
    return Cs, Ss


def energy_mp(n, v, pos):
    """(Phi, S(k) list, C, S); v is None (all ones) or a dd [2, M] array."""
    Cs, Ss = nk_mp(n, pos)
    N = pos.shape[2]
    phi = ctx.mpf(0)
    sk = []
    for k, (C, S) in enumerate(zip(Cs, Ss)):
        w = ctx.mpf(1) if v is None else mp_of(v[0, k], v[1, k])
        phi += w * (C * C + S * S)
        sk.append((C * C + S * S) / N)
    return phi, sk, Cs, Ss


def energy_at(n, v, u, N):
    """Phi at mp positions u[j][a] (no dd rounding)."""
    phi = ctx.mpf(0)
    for k, nv in enumerate(n):
        C = ctx.mpf(0)
        S = ctx.mpf(0)
        for uj in u:
            t = sum(int(na) * ua for na, ua in zip(nv, uj))
            C += ctx.cospi(2 * t)
            S += ctx.sinpi(2 * t)
        w = ctx.mpf(1) if v is None else mp_of(v[0, k], v[1, k])
        phi += w * (C * C + S * S)
    return phi


def grad_fd(n, v, pos, j, a, L=1.0, h=ctx.mpf(2) ** -100):
    """dPhi/dr_{j,a} by a 256-bit central difference of the energy (r = L u)."""
    u = positions_mp(pos)
    N = pos.shape[2]
    up = [list(x) for x in u]
    um = [list(x) for x in u]
    up[j][a] += h
    um[j][a] -= h
    return (energy_at(n, v, up, N) - energy_at(n, v, um, N)) / (2 * h) / ctx.mpf(L)


# --- L-BFGS rules, second implementation ------------------------------------

def lbfgs_mp(fg, x0, nmean, max_iter, history=8, c1=1e-4, step_cap=1e-2, max_halvings=40):
    """Run the minimiser rules for ``max_iter`` iterations at 256 bits with no
    stopping rule other than the count; returns (x, list of f at each iterate)."""
    x, trace, _, _ = lbfgs_mp_run(fg, x0, nmean, max_iter, history, c1, step_cap, max_halvings)
    return x, trace


def lbfgs_mp_run(fg, x0, nmean, max_iter, history=8, c1=1e-4, step_cap=1e-2, max_halvings=40,
                 stall_window=None, stall_ratio=0.99, max_ls_fail=None):
    """The minimiser rules at 256 bits, with the stopping rules.

    fg(x) -> (f, g list).  Rules: the two-loop recursion with H0 = (s.y / y.y) I
    of the newest pair; a steepest-descent step scaled to move at most
    step_cap * nmean, and at most to 2 f / g.g (the minimum value is 0), when the
    history is empty or the direction is not a descent direction; Armijo
    backtracking by halving from alpha = 1 (max_halvings halvings, then a
    failure: the history is cleared and x kept); a pair is kept only when
    s.y > 0.  Stopping rules, tested at the top of every iteration in this
    order: the iteration cap; with stall_window W, stalled when the smallest f
    of the last W iterates exceeds stall_ratio times the smallest of the W
    before them (tested once 2W iterations are done); and, with max_ls_fail,
    stalled right after that many consecutive failures.

    Returns (x, trace, status, iterations): trace holds f at the top of every
    iteration reached (a run ending on failures has no entry for its last
    count), status is "stalled" or "max_iter".
    """
    x = list(x0)
    f, g = fg(x)
    S, Y, R = [], [], []
    trace = []
    hist = []          # f at every iterate, for the stall window
    it = 0
    fails = 0
    while True:
        trace.append(f)
        hist.append(f)
        if it >= max_iter:
            return x, trace, "max_iter", it
        if stall_window is not None and it >= 2 * stall_window:
            recent = min(hist[it - stall_window + 1:it + 1])
            older = min(hist[it - 2 * stall_window + 1:it - stall_window + 1])
            if recent > ctx.mpf(stall_ratio) * older:
                return x, trace, "stalled", it
        p = None
        if S:
            q = list(g)
            alphas = []
            for s, y, r in zip(reversed(S), reversed(Y), reversed(R)):
                al = r * sum(si * qi for si, qi in zip(s, q))
                alphas.append(al)
                q = [qi - al * yi for qi, yi in zip(q, y)]
            gamma = sum(a * b for a, b in zip(S[-1], Y[-1])) / sum(b * b for b in Y[-1])
            q = [gamma * qi for qi in q]
            for (s, y, r), al in zip(zip(S, Y, R), reversed(alphas)):
                be = r * sum(yi * qi for yi, qi in zip(y, q))
                q = [qi + (al - be) * si for qi, si in zip(q, s)]
            p = [-qi for qi in q]
            gp = sum(a * b for a, b in zip(g, p))
            if gp >= 0:
                p = None
        if p is None:
            S, Y, R = [], [], []
            gmax = max(abs(gi) for gi in g)
            scale = min(ctx.mpf(step_cap * nmean) / gmax, 2 * f / sum(gi * gi for gi in g))
            p = [-gi * scale for gi in g]
            gp = sum(a * b for a, b in zip(g, p))
        alpha = ctx.mpf(1)
        accepted = False
        for _h in range(max_halvings + 1):
            xt = [xi + alpha * pi for xi, pi in zip(x, p)]
            ft, _ = fg(xt, want_grad=False)
            if not ft > f + ctx.mpf(c1) * alpha * gp:
                accepted = True
                break
            alpha /= 2
        it += 1
        if not accepted:
            S, Y, R = [], [], []
            fails += 1
            if max_ls_fail is not None and fails >= max_ls_fail:
                return x, trace, "stalled", it
            continue
        fails = 0
        ft, gt = fg(xt)
        s = [a - b for a, b in zip(xt, x)]
        y = [a - b for a, b in zip(gt, g)]
        sy = sum(a * b for a, b in zip(s, y))
        if sy > 0:
            S.append(s)
            Y.append(y)
            R.append(1 / sy)
            if len(S) > history:
                S.pop(0)
                Y.pop(0)
                R.pop(0)
        x, f, g = xt, ft, gt


def fire_mp(fg, x0, nmean, max_iter, step_cap=1e-2):
    """FIRE (Bitzek et al. 2006) for ``max_iter`` iterations at 256 bits.

    Unit masses, F = -g.  Per iteration: P = F.v; if P > 0, v <- (1 - a) v +
    a |v| F/|F|, the count of consecutive P > 0 steps grows and beyond 5 the step
    grows (dt <- min(1.1 dt, dt_max)) and a <- 0.99 a; otherwise dt <- dt / 2,
    v <- 0, a <- 0.1 and the count restarts; then v <- v + dt F, x <- x + dt v.
    dt0 = sqrt(step_cap nmean / max|g(x0)|), dt_max = 10 dt0.  The step length
    and a are IEEE doubles (as the minimiser keeps them); vectors are 256-bit.
    Returns (x, list of f at each iterate).
    """
    x = list(x0)
    f, g = fg(x)
    v = [ctx.mpf(0)] * len(x)
    gmax = float(max(abs(gi) for gi in g))
    dt = math.sqrt(step_cap * nmean / gmax)
    dt_max = 10.0 * dt
    a = 0.1
    npos = 0
    trace = [f]
    for _ in range(max_iter):
        P = -sum(gi * vi for gi, vi in zip(g, v))
        if P > 0:
            vn = ctx.sqrt(sum(vi * vi for vi in v))
            gn = ctx.sqrt(sum(gi * gi for gi in g))
            cg = vn / gn * ctx.mpf(a)
            cv = ctx.mpf(1.0 - a)
            v = [cv * vi - cg * gi for vi, gi in zip(v, g)]
            npos += 1
            if npos > 5:
                dt = min(dt * 1.1, dt_max)
                a = a * 0.99
        else:
            dt = dt * 0.5
            v = [ctx.mpf(0)] * len(x)
            a = 0.1
            npos = 0
        mdt = ctx.mpf(dt)
        v = [vi - mdt * gi for vi, gi in zip(v, g)]
        x = [xi + mdt * vi for xi, vi in zip(x, v)]
        f, g = fg(x)
        trace.append(f)
    return x, trace


def quadratic_fg(w, c):
    """f = 1/2 sum w_i (x_i - c_i)^2 with mp vectors w, c."""
    def fg(x, want_grad=True):
        r = [xi - ci for xi, ci in zip(x, c)]
        f = sum(wi * ri * ri for wi, ri in zip(w, r)) / 2
        if not want_grad:
            return f, None
        return f, [wi * ri for wi, ri in zip(w, r)]
    return fg


def stealthy_fg(n, v, N, d, L=1.0):
    """Energy and gradient with respect to the fractional coordinates, x = [a][j] flat."""
    n = [tuple(int(t) for t in nv) for nv in n]

    def fg(x, want_grad=True):
        u = [[x[a * N + j] for a in range(d)] for j in range(N)]
        Cs, Ss, cs, ss = [], [], [], []
        for nv in n:
            C = ctx.mpf(0)
            S = ctx.mpf(0)
            crow, srow = [], []
            for uj in u:
                t = sum(na * ua for na, ua in zip(nv, uj))
                c_ = ctx.cospi(2 * t)
                s_ = ctx.sinpi(2 * t)
                crow.append(c_)
                srow.append(s_)
                C += c_
                S += s_
            Cs.append(C)
            Ss.append(S)
            cs.append(crow)
            ss.append(srow)
        f = ctx.mpf(0)
        for k in range(len(n)):
            w = ctx.mpf(1) if v is None else mp_of(v[0, k], v[1, k])
            f += w * (Cs[k] ** 2 + Ss[k] ** 2)
        if not want_grad:
            return f, None
        g = [ctx.mpf(0)] * (d * N)
        four_pi = 4 * ctx.pi
        for k, nv in enumerate(n):
            w = ctx.mpf(1) if v is None else mp_of(v[0, k], v[1, k])
            for j in range(N):
                term = w * (Ss[k] * cs[k][j] - Cs[k] * ss[k][j])
                for a in range(d):
                    if nv[a]:
                        g[a * N + j] += four_pi * nv[a] * term
        return f, g
    return fg


def nmean_of(N: int, d: int) -> float:
    return math.pow(float(N), -1.0 / float(d))


def dd_planes(xs) -> np.ndarray:
    out = np.zeros((2, len(xs)))
    for i, x in enumerate(xs):
        out[0, i], out[1, i] = to_dd(x)
    return out

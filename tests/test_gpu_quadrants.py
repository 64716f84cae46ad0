"""Phase reduction and double-double sin/cos on the device at exact octants and
quadrant boundaries, through the public evaluation.

Single particles (and a pair) at dyadic positions put every phase t = n.u mod 1 on
a multiple of 1/8 -- cos and sin exactly 0, +-1 or +-sqrt(2)/2 -- or within 2^-70
of one (positions with a nonzero low word), where an inexact reduction of n.u
or a quadrant mix-up in the sin/cos shows at once.  Every C_k and S_k of n~ is
compared with the 256-bit value of sum_j cos / sin(2 pi n.u_j) (mpmath), and the
gradient of a single particle, which vanishes, is checked against 0 within the
error of its terms (each pairs the n~ pass's factor with the gradient pass's
own, a walk along the run).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2304_09139_amd import ss

pytestmark = pytest.mark.gpu

mpmath.mp.prec = 256

# per-term bound of the pair factor: at most 16 table steps z^m = z^(m-1) z, at
# most 8 walk steps and d prefix products, each a lazy complex product of about
# 4 2^-106 absolute error (2e-30 per particle; an inexact reduction of n.u
# shows at 1e-16 and a quadrant mix-up at 1)
TOL = 2e-30
# per-component bound of the gradient pass's factor: at most 16 table steps, a
# walk of at most 2R + 1 steps along the run and d prefix products, each a lazy
# complex product of about 4 2^-106
def e_walk(d, R):
    return (16 + 2 * R + 1 + d) * 4 * 2.0 ** -106


def dd_of(fr: Fraction):
    hi = float(fr)
    lo = float(fr - Fraction(hi))
    return hi, lo


CASES = [  # (name, d, R2, particle coordinates as exact fractions)
    ("d1_octants", 1, 400, [[Fraction(1, 8)]]),
    ("d1_near_quarter", 1, 400, [[Fraction(1, 4) + Fraction(1, 2 ** 70)]]),
    ("d2_octants", 2, 50, [[Fraction(1, 4), Fraction(3, 8)]]),
    ("d3_near_boundaries", 3, 30, [[Fraction(1, 2), Fraction(1, 4) + Fraction(1, 2 ** 70),
                                    Fraction(5, 8) - Fraction(1, 2 ** 80)]]),
    ("d2_pair", 2, 80, [[Fraction(1, 8), Fraction(7, 8)], [Fraction(3, 10), Fraction(7, 10)]]),
    ("d4_halves", 4, 6, [[Fraction(1, 2), Fraction(1, 4), Fraction(3, 4), Fraction(1, 8)]]),
]


@pytest.mark.parametrize("name,d,R2,parts", CASES, ids=[c[0] for c in CASES])
def test_octant_phases(name, d, R2, parts):
    ctx = ss.Context(0)
    try:
        N = len(parts)
        pos = np.zeros((2, d, N))
        for j, p in enumerate(parts):
            for a, fr in enumerate(p):
                pos[0, a, j], pos[1, a, j] = dd_of(fr)
        w = ss.Workload(d, N, R2, ss.count(d, R2))
        n = ctx.wavevectors(d, R2)
        out = ctx.energy_grad(w, n, None, torch.from_numpy(pos).cuda(), grad=True, nk=True)
        torch.cuda.synchronize()
        nk = out["nk"].cpu().numpy()
        nh = n.cpu().numpy()
        worst = 0.0
        for k in range(w.M):
            C = mpmath.mpf(0)
            S = mpmath.mpf(0)
            for p in parts:
                t = sum(int(nh[k, a]) * p[a] for a in range(d))
                t = t - (t.numerator // t.denominator)      # exact fractional part
                ang = 2 * mpmath.pi * mpmath.mpf(t.numerator) / t.denominator
                C += mpmath.cos(ang)
                S += mpmath.sin(ang)
            dC = abs((mpmath.mpf(nk[0, k]) + mpmath.mpf(nk[1, k])) - C)
            dS = abs((mpmath.mpf(nk[2, k]) + mpmath.mpf(nk[3, k])) - S)
            worst = max(worst, float(dC), float(dS))
            assert dC <= TOL * N and dS <= TOL * N, (name, k, nh[k], float(dC), float(dS))
        if N == 1:
            # g_a = 4 pi sum_k n_{k,a} (S_k c_k - C_k s_k) (L = 1): a term's error is
            # at most |dS| + |dC| (the n~ pass, within TOL) plus |dc| + |ds| (the walk)
            g = out["grad"].cpu().numpy()
            R = int(np.floor(np.sqrt(R2)))
            for a in range(d):
                bound = 4 * np.pi * np.abs(nh[:, a]).sum() * 2 * (TOL + e_walk(d, R))
                assert abs(g[0, a, 0] + g[1, a, 0]) <= bound, (name, a, g[0, a, 0], bound)
        print(f"{name}: M={w.M} worst |d n~| = {worst:.1e}")
    finally:
        ctx.close()

"""Pins for the oracle's n~(k), S(k), Phi and gradient.

Independent checks: closed forms (one particle, two particles, a periodic
lattice whose n~(k) vanishes below its first Bragg peak), exact symmetries
(translation, inversion, permutation), the Poisson mean S(k) = 1, 256-bit
brute force of the definitions, the paper's full +-k form of Eq. energy and
Eq. force, and 256-bit central differences of the energy.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_09139_amd import inputs
import mpref

U2 = mpref.U_DD
ctx = mpref.ctx


def nk_tol(N):
    """Bound on |Delta C_k|, |Delta S_k| of the oracle against exact: each of the N
    terms carries <= 4 u_dd (sin/cos) + 2*pi*2^-107 (phase), each accurate addition
    <= 3 u_dd times the running sum (<= N)."""
    return U2 * (5.0 * N + 3.0 * N * N)


def positions_from_fractions(fr):
    """fr: list over particles of d Fractions -> float64[2, d, N] (hi, lo rounding)."""
    N = len(fr)
    d = len(fr[0])
    pos = np.zeros((2, d, N))
    for j, row in enumerate(fr):
        for a, x in enumerate(row):
            pos[0, a, j], pos[1, a, j] = mpref.to_dd(Fraction(x))
    return pos


def test_single_particle():
    pos = inputs.uniform_positions(3, 1, 11)
    n = O.wavevectors(3, 20)
    out = O.energy_grad(n, None, pos, want_grad=True)
    Cs, Ss = [], []
    for nv in n:
        t = sum(int(x) * mpref.mp_of(pos[0, a, 0], pos[1, a, 0]) for a, x in enumerate(nv))
        Cs.append(ctx.cospi(2 * t))
        Ss.append(ctx.sinpi(2 * t))
    M = len(n)
    for k in range(M):
        assert abs(mpref.mp_of(out["nk"][0, k], out["nk"][1, k]) - Cs[k]) <= 8 * U2
        assert abs(mpref.mp_of(out["nk"][2, k], out["nk"][3, k]) - Ss[k]) <= 8 * U2
    # |n~|^2 = 1 for every k, so Phi = M and S_max = 1; the gradient vanishes
    assert abs(mpref.mp_of(*out["phi"]) - M) <= 8 * M * U2
    assert abs(mpref.mp_of(*out["smax"]) - 1) <= 8 * U2
    assert np.all(np.abs(out["grad"][0]) <= 1e-28)


def test_two_particles_closed_form():
    pos = inputs.uniform_positions(2, 2, 5)
    n = O.wavevectors(2, 30)
    out = O.energy_grad(n, None, pos, want_grad=False)
    du = [mpref.mp_of(pos[0, a, 0], pos[1, a, 0]) - mpref.mp_of(pos[0, a, 1], pos[1, a, 1]) for a in range(2)]
    phi = ctx.mpf(0)
    for k, nv in enumerate(n):
        mag = 2 + 2 * ctx.cospi(2 * sum(int(x) * du[a] for a, x in enumerate(nv)))
        C = mpref.mp_of(out["nk"][0, k], out["nk"][1, k])
        S = mpref.mp_of(out["nk"][2, k], out["nk"][3, k])
        assert abs(C * C + S * S - mag) <= 64 * U2
        phi += mag
    assert abs(mpref.mp_of(*out["phi"]) - phi) <= 64 * len(n) * U2


@pytest.mark.parametrize("d,m", [(2, 8), (2, 6), (2, 7), (3, 4), (3, 5)])
def test_lattice_below_bragg_peak(d, m):
    """A periodic m^d lattice: n~(k) = 0 for all 0 < |n| < m (first Bragg peak at |n| = m)."""
    import itertools
    off = [Fraction(1, 7), Fraction(2, 11), Fraction(3, 13)][:d]
    fr = [[Fraction(i, m) + off[a] for a, i in enumerate(idx)] for idx in itertools.product(range(m), repeat=d)]
    pos = positions_from_fractions(fr)
    N = m ** d
    n = O.wavevectors(d, m * m - 1)
    out = O.energy_grad(n, None, pos, want_grad=True)
    tol = nk_tol(N)
    assert np.max(np.abs(out["nk"][0])) <= tol
    assert np.max(np.abs(out["nk"][2])) <= tol
    assert out["smax"][0] <= tol * tol / N
    # ground state: the gradient vanishes to the same rounding level
    G = 4 * np.pi * tol * np.abs(n).sum()
    assert np.max(np.abs(out["grad"][0])) <= G
    # the first Bragg shell is not stealthy: |n~(m e_1)|^2 = N^2
    peak = O.nk(np.array([[m] + [0] * (d - 1)], np.int32), pos)
    pc, ps = mpref.mp_of(peak[0, 0], peak[1, 0]), mpref.mp_of(peak[2, 0], peak[3, 0])
    assert abs(pc * pc + ps * ps - N * N) <= N * tol


def test_translation_inversion_permutation():
    d, N = 3, 40
    pos = inputs.uniform_positions(d, N, 3)
    n = O.wavevectors(d, 14)
    M = len(n)
    ref = O.energy_grad(n, None, pos)
    G = np.array([4 * np.pi * np.abs(n[:, a]).sum() * 2 * N for a in range(d)])
    # Sum_j dPhi/dr_j = 0 (translation invariance of Phi)
    for a in range(d):
        tot = sum(Fraction(float(ref["grad"][0, a, j])) + Fraction(float(ref["grad"][1, a, j])) for j in range(N))
        assert abs(float(tot)) <= 64 * N * U2 * G[a]
    # a translation by an exact dyadic shift changes only the phases of n~
    shifted = pos.copy()
    for a, c in enumerate([Fraction(1, 8), Fraction(-1, 4), Fraction(3, 8)]):
        for j in range(N):
            shifted[0, a, j], shifted[1, a, j] = mpref.to_dd(mpref.frac_of(pos[0, a, j], pos[1, a, j]) + c)
    sh = O.energy_grad(n, None, shifted)
    tol = nk_tol(N)
    mag0 = ref["nk"][0] ** 2 + ref["nk"][2] ** 2
    mag1 = sh["nk"][0] ** 2 + sh["nk"][2] ** 2
    assert np.allclose(mag0, mag1, rtol=1e-13, atol=1e-13)
    assert abs(mpref.mp_of(*sh["phi"]) - mpref.mp_of(*ref["phi"])) <= 4 * M * N * tol
    assert np.max(np.abs(sh["grad"][0] - ref["grad"][0])) <= 4 * tol * G.max()
    # inversion u -> -u: C unchanged, S negated, bit for bit (all steps are odd/even exactly)
    inv = O.energy_grad(n, None, -pos)
    assert np.array_equal(inv["nk"][0:2], ref["nk"][0:2])
    assert np.array_equal(inv["nk"][2:4], -ref["nk"][2:4])
    assert np.array_equal(inv["phi"], ref["phi"])
    # permutation of the particles: same n~ to rounding, gradient permuted
    perm = np.random.default_rng(1).permutation(N)
    pp = O.energy_grad(n, None, pos[:, :, perm])
    assert np.max(np.abs(pp["nk"][0] - ref["nk"][0])) <= 2 * tol
    assert np.max(np.abs(pp["grad"][0] - ref["grad"][0][:, perm])) <= 4 * tol * G.max()


def test_poisson_mean_structure_factor():
    """For independent uniform points E[S(k)] = 1 at every k != 0."""
    d, N = 2, 200
    n = O.wavevectors(d, 40)
    vals = []
    for seed in range(8):
        pos = inputs.uniform_positions(d, N, 1000 + seed)
        e = O.energy_from_nk(N, None, O.nk(n, pos))
        vals.append(e.sk[0])
    s = np.concatenate(vals)
    # S(k) of a Poisson pattern is ~ Exp(1) (variance 1): mean within 5 sigma
    assert abs(s.mean() - 1.0) <= 5.0 / np.sqrt(s.size)


@pytest.mark.parametrize("d,N,R2,seed", [(1, 12, 30, 1), (2, 16, 10, 2), (3, 10, 6, 3), (4, 8, 3, 4)])
def test_brute_force_256bit(d, N, R2, seed):
    pos = inputs.uniform_positions(d, N, seed)
    n = O.wavevectors(d, R2)
    v = O.weights(n, R2, 1)
    out = O.energy_grad(n, v, pos)
    phi, sk, Cs, Ss = mpref.energy_mp(n, v, pos)
    tol = nk_tol(N)
    for k in range(len(n)):
        assert abs(mpref.mp_of(out["nk"][0, k], out["nk"][1, k]) - Cs[k]) <= tol
        assert abs(mpref.mp_of(out["nk"][2, k], out["nk"][3, k]) - Ss[k]) <= tol
    assert abs(mpref.mp_of(*out["phi"]) - phi) <= 4 * N * tol * len(n)
    sm = max(sk)
    assert abs(mpref.mp_of(*out["smax"]) - sm) <= 4 * tol
    # gradient against 256-bit central differences of the energy itself
    for j in range(0, N, max(1, N // 4)):
        for a in range(d):
            fd = mpref.grad_fd(n, v, pos, j, a)
            got = mpref.mp_of(out["grad"][0, a, j], out["grad"][1, a, j])
            scale = 4 * np.pi * np.abs(n[:, a]).sum() * 2 * N
            assert abs(got - fd) <= 8 * tol * scale


def test_paper_full_set_forms():
    """Phi/eps0 = N/(2 v_F) sum over all 0<|k|<=K of v~ S(k) and F_j = -dPhi/dr_j of
    Eq. force, both summed over the full +-k set with v~ = eps0 L^d, equal the
    half-set forms the oracle computes (here with L = 1 and L = 2.5)."""
    d, N, R2 = 2, 9, 8
    for L in (1.0, 2.5):
        pos = inputs.uniform_positions(d, N, 77)
        n = O.wavevectors(d, R2)
        out = O.energy_grad(n, None, pos, L=L)
        full = np.concatenate([n, -n])
        r = [[L * mpref.mp_of(pos[0, a, j], pos[1, a, j]) for a in range(d)] for j in range(N)]
        vF = ctx.mpf(L) ** d
        vt = vF                      # v~(k) = eps0 L^d with eps0 = 1
        kmin = 2 * ctx.pi / L
        phi = ctx.mpf(0)
        F = [[ctx.mpf(0)] * d for _ in range(N)]
        for nv in full:
            kv = [kmin * int(x) for x in nv]
            re = sum(ctx.cos(sum(kv[a] * r[j][a] for a in range(d))) for j in range(N))
            im = -sum(ctx.sin(sum(kv[a] * r[j][a] for a in range(d))) for j in range(N))
            S = (re * re + im * im) / N
            phi += N / (2 * vF) * vt * S
            for j in range(N):
                kr = sum(kv[a] * r[j][a] for a in range(d))
                # Im[n~(k) exp(i k.r_j)]
                imv = re * ctx.sin(kr) + im * ctx.cos(kr)
                for a in range(d):
                    F[j][a] += kv[a] * vt * imv / vF
        assert abs(mpref.mp_of(*out["phi"]) - phi) <= 1e-28
        for j in range(N):
            for a in range(d):
                got = mpref.mp_of(out["grad"][0, a, j], out["grad"][1, a, j])
                assert abs(got + F[j][a]) <= 1e-27


def test_weights_against_mpmath():
    for d, R2 in [(2, 64), (3, 61)]:
        n = O.wavevectors(d, R2)
        v = O.weights(n, R2, 1)
        for k in range(len(n)):
            s = int((n[k].astype(np.int64) ** 2).sum())
            exact = (1 - ctx.sqrt(ctx.mpf(s) / (ctx.mpf(R2) + ctx.mpf(1) / 2))) ** 2
            assert abs(mpref.mp_of(v[0, k], v[1, k]) - exact) <= 16 * U2 * float(exact)
            assert v[0, k] > 0
        one = O.weights(n, R2, 0)
        assert np.all(one[0] == 1.0) and np.all(one[1] == 0.0)

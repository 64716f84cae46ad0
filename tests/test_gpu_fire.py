"""GPU FIRE quench (ss_minimize with method = 1) against the oracle's FIRE.

Parity as for L-BFGS: the first iterates agree with the oracle's to 1e-26
(relative in Phi, absolute in the positions) -- 20 iterations cover the step
growth after N_min and both velocity branches -- and full quenches reach the
stated floor when the oracle re-evaluates the final positions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2304_09139_amd import inputs, ss

pytestmark = pytest.mark.gpu

FLOOR = 1e-40


@pytest.fixture(scope="module")
def ctx():
    c = ss.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("d,N,chi,vkind,L", [(2, 128, 0.4, 0, 1.0), (3, 200, 0.3, 1, 1.0), (2, 90, 0.35, 0, 3.0)])
def test_fire_first_iterates_match_oracle(ctx, d, N, chi, vkind, L):
    w = ss.Workload.from_chi(d, N, chi, L=L, vkind=vkind)
    n = ctx.wavevectors(d, w.R2)
    v = ctx.weights(w, n) if vkind else None
    nh = n.cpu().numpy()
    vh = O.weights(nh, w.R2, vkind) if vkind else None
    pos = inputs.config_positions(51, d, N, vkind)
    for iters in (1, 3, 8, 20):
        x = dev(pos)
        r = ctx.minimize(w, n, v, x, max_iter=iters, s_floor=0.0, method="fire")
        xo, ro, _ = O.minimize(nh, vh, pos, L=L, max_iter=iters, s_floor=0.0, method="fire")
        assert r["iters"] == ro["iters"] == iters
        assert r["evals"] == ro["evals"] == iters + 1
        dphi = abs((r["phi"][0] - ro["phi"][0]) + (r["phi"][1] - ro["phi"][1]))
        assert dphi <= 1e-26 * ro["phi"][0], (iters, dphi / ro["phi"][0])
        xg = x.cpu().numpy()
        dx = np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max()
        assert dx <= 1e-26, (iters, dx)


def test_fire_quench_reaches_floor(ctx):
    d, N, chi = 2, 128, 0.4
    w = ss.Workload.from_chi(d, N, chi)
    n = ctx.wavevectors(d, w.R2)
    nh = n.cpu().numpy()
    for seed in range(3):
        pos = inputs.config_positions(1, d, N, seed)
        x = dev(pos)
        r = ctx.minimize(w, n, None, x, s_floor=FLOOR, method="fire", stall_window=200)
        assert r["status"] == "converged", r
        e = O.energy_from_nk(N, None, O.nk(nh, x.cpu().numpy()))
        assert e.smax[0] <= FLOOR * (1 + 1e-6), (e.smax, r["smax"])
        xl = dev(pos)
        rl = ctx.minimize(w, n, None, xl, s_floor=FLOOR)
        print(f"seed {seed}: FIRE iters={r['iters']} t={r['seconds']:.3f}s; L-BFGS iters={rl['iters']} "
              f"evals={rl['evals']} t={rl['seconds']:.3f}s")


def test_fire_options(ctx):
    d, N, chi = 2, 64, 0.3
    w = ss.Workload.from_chi(d, N, chi)
    n = ctx.wavevectors(d, w.R2)
    pos = inputs.config_positions(52, d, N, 0)
    x = dev(pos)
    r = ctx.minimize(w, n, None, x, max_iter=0, method="fire")
    assert r["iters"] == 0 and np.array_equal(x.cpu().numpy(), pos)
    with pytest.raises(ss.SSError) as e:
        ctx.minimize(w, n, None, dev(pos), method=2)
    assert e.value.code == ss.SS_EINVAL
    with pytest.raises(ss.SSError) as e:
        ctx.minimize_batch([w], [dev(pos)], opts=dict(method=1))
    assert e.value.code == ss.SS_EINVAL

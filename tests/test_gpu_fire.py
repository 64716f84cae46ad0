"""GPU FIRE quench (method = 1) against the oracle's FIRE: single quenches
(ss_minimize), batches (ss_minimize_batch) and served requests (ss_submit).

Parity as for L-BFGS: the first iterates agree with the oracle's to 1e-26
(relative in Phi, absolute in the positions) -- 20 iterations cover the step
growth after N_min and both velocity branches -- and full quenches reach the
stated floor when the oracle re-evaluates the final positions.  In batches a
FIRE configuration's result is the same bits alone and mixed with L-BFGS and
staged configurations, and a served FIRE request equals the batch of one.
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
        ctx.minimize_batch([w], [dev(pos)], opts=dict(method=2))
    assert e.value.code == ss.SS_EINVAL
    x = dev(pos)
    r = ctx.minimize_batch([w], [x], opts=dict(max_iter=0, method="fire"))[0]
    assert r["iters"] == 0 and np.array_equal(x.cpu().numpy(), pos)


# (d, N, chi, vkind, L, config id)
FIRE_MIX = [(2, 128, 0.4, 0, 1.0, 81), (3, 200, 0.3, 1, 1.0, 82), (2, 90, 0.35, 0, 3.0, 83),
            (3, 700, 0.45, 0, 1.0, 84), (1, 40, 0.4, 0, 1.0, 85), (2, 1500, 0.2, 0, 2.0, 86)]


def fire_setup(ctx, spec):
    d, N, chi, vkind, L, cid = spec
    w = ss.Workload.from_chi(d, N, chi, L=L, vkind=vkind)
    n = ctx.wavevectors(d, w.R2)
    v = ctx.weights(w, n) if vkind else None
    return w, n, v, inputs.config_positions(cid, d, N, 0)


def test_fire_batch_first_iterates_match_oracle(ctx):
    items = [fire_setup(ctx, s) for s in FIRE_MIX]
    for iters in (1, 3, 8, 20):
        xs = [dev(it[3]) for it in items]
        res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items],
                                 opts=dict(max_iter=iters, s_floor=0.0, method="fire"))
        for (w, n, v, pos), x, r, spec in zip(items, xs, res, FIRE_MIX):
            nh = n.cpu().numpy()
            vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
            xo, ro, _ = O.minimize(nh, vh, pos, L=w.L, max_iter=iters, s_floor=0.0, method="fire")
            assert r["iters"] == ro["iters"] == iters, (spec, r, ro)
            assert r["evals"] == ro["evals"] == iters + 1, (spec, r, ro)
            dphi = abs((r["phi"][0] - ro["phi"][0]) + (r["phi"][1] - ro["phi"][1]))
            assert dphi <= 1e-26 * ro["phi"][0], (spec, iters, dphi / ro["phi"][0])
            xg = x.cpu().numpy()
            dx = np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max()
            assert dx <= 1e-26, (spec, iters, dx)


def test_fire_batch_alone_vs_mix_bitwise(ctx):
    """FIRE, staged FIRE and L-BFGS configurations in one batch: each gives the
    same bits as alone, in two orders."""
    items = [fire_setup(ctx, s) for s in FIRE_MIX]
    kinds = [dict(method="fire"), dict(method="lbfgs"), dict(method="fire", precision="staged"),
             dict(method="fire"), dict(method="lbfgs", precision="staged"), dict(method="fire")]
    opts = [dict(k, max_iter=60, s_floor=0.0, stall_window=200) for k in kinds]
    alone = []
    for (w, n, v, pos), o in zip(items, opts):
        x = dev(pos)
        r = ctx.minimize_batch([w], [x], [v], opts=[o])[0]
        alone.append((x.cpu().numpy(), r))
    for perm in (list(range(len(items))), [3, 5, 0, 2, 4, 1]):
        xs = [dev(items[i][3]) for i in perm]
        res = ctx.minimize_batch([items[i][0] for i in perm], xs, [items[i][2] for i in perm],
                                 opts=[opts[i] for i in perm])
        for i, x, r in zip(perm, xs, res):
            xa, ra = alone[i]
            assert np.array_equal(x.cpu().numpy(), xa), FIRE_MIX[i]
            for key in ("phi", "smax", "iters", "evals", "iters_fp64", "status"):
                assert r[key] == ra[key], (FIRE_MIX[i], key, r[key], ra[key])


def test_fire_batch_and_served_reach_floor(ctx):
    """Batched FIRE quenches (double-double and staged) reach the floor (the
    oracle re-evaluates them), and the same requests served give the same bits."""
    d, N, chi = 2, 128, 0.4
    w = ss.Workload.from_chi(d, N, chi)
    n = ctx.wavevectors(d, w.R2)
    nh = n.cpu().numpy()
    starts = [inputs.config_positions(1, d, N, seed) for seed in range(3)]
    kinds = [dict(method="fire"), dict(method="fire", precision="staged"), dict(method="fire")]
    opts = [dict(k, s_floor=FLOOR, stall_window=200) for k in kinds]
    xs = [dev(p) for p in starts]
    res = ctx.minimize_batch([w] * 3, xs, None, opts=opts)
    for x, r, o in zip(xs, res, opts):
        assert r["status"] == "converged", (o, r)
        e = O.energy_from_nk(N, None, O.nk(nh, x.cpu().numpy()))
        assert e.smax[0] <= FLOOR * (1 + 1e-6), (o, e.smax, r["smax"])
        if o.get("precision") == "staged":
            assert 0 < r["iters_fp64"] < r["iters"], r
        print(f"batched FIRE {o}: iters={r['iters']} (FP64 {r['iters_fp64']})")
    ctx.server_start(1 << 28, max_slots=4)
    try:
        tickets = [ctx.submit(w, p, **o) for p, o in zip(starts, opts)]
        import time
        for t, x, r in zip(tickets, xs, res):
            t0 = time.time()
            while (got := ctx.poll(t)) is None:
                assert time.time() - t0 < 120
                time.sleep(0.002)
            rs, xsrv = got
            assert np.array_equal(xsrv, x.cpu().numpy())
            assert rs["phi"] == r["phi"] and rs["iters"] == r["iters"]
    finally:
        ctx.server_stop()

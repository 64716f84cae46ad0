"""Batched quenches in FP64 and staged precision, and mixed-precision batches.

A batch may hold configurations at different precisions: double-double, FP64
only, and staged (FP64 until its stage stops, then double-double from the same
positions with the kept pairs).  Each configuration switches on its own, so:
  * the FP64 iterates of a batch follow the double-double rules to FP64
    rounding (as for ss_minimize in FP64);
  * staged configurations reach the stated floor (re-evaluated by the oracle)
    with part of their iterations in FP64;
  * a configuration's result is bitwise the same alone and in a batch that mixes
    precisions, sizes and dimensions (its launch shape depends on (d, N, M) only).
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


def setup(ctx, spec):
    d, N, chi, vkind, L, cid = spec
    w = ss.Workload.from_chi(d, N, chi, L=L, vkind=vkind)
    n = ctx.wavevectors(d, w.R2)
    v = ctx.weights(w, n) if vkind else None
    pos = inputs.config_positions(cid, d, N, 0)
    return w, n, v, pos


def oracle_smax(w, n, x):
    nh = n.cpu().numpy()
    vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
    return O.energy_from_nk(w.N, vh, O.nk(nh, x.cpu().numpy())).smax[0]


SPECS = [(2, 128, 0.4, 0, 1.0, 61), (3, 300, 0.3, 1, 1.0, 62), (2, 90, 0.35, 0, 3.0, 63),
         (3, 500, 0.45, 0, 1.0, 64), (1, 40, 0.4, 0, 1.0, 65)]


def test_batch_fp64_first_iterates_follow_rules(ctx):
    items = [setup(ctx, s) for s in SPECS]
    for iters in (1, 3):
        xs = [dev(it[3]) for it in items]
        res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items],
                                 opts=dict(max_iter=iters, s_floor=0.0, precision="fp64"))
        for (w, n, v, pos), x, r, spec in zip(items, xs, res, SPECS):
            nh = n.cpu().numpy()
            vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
            xo, ro, _ = O.minimize(nh, vh, pos, L=w.L, max_iter=iters, s_floor=0.0)
            assert r["iters"] == ro["iters"] == iters and r["iters_fp64"] == iters, (spec, r)
            assert r["evals"] == ro["evals"] == r["evals_fp64"], (spec, r, ro)
            assert abs(r["phi"][0] - ro["phi"][0]) <= 1e-11 * ro["phi"][0], (spec, iters)
            xg = x.cpu().numpy()
            assert np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max() <= 1e-12, (spec, iters)


def test_batch_staged_reaches_floor(ctx):
    items = [setup(ctx, s) for s in SPECS]
    xs = [dev(it[3]) for it in items]
    res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items],
                             opts=dict(s_floor=FLOOR, precision="staged"))
    for (w, n, v, pos), x, r, spec in zip(items, xs, res, SPECS):
        assert r["status"] == "converged", (spec, r)
        assert 0 < r["iters_fp64"] < r["iters"], (spec, r)
        assert r["evals_fp64"] < r["evals"], (spec, r)
        assert oracle_smax(w, n, x) <= FLOOR * (1 + 1e-6), spec
        print(f"{spec}: iters={r['iters']} (fp64 {r['iters_fp64']}) t={r['seconds']:.3f}s")


def test_mixed_precision_batch_alone_vs_mix_bitwise(ctx):
    """Staged, double-double and FP64-only configurations in one batch, in two
    orders: each result is the same bits as the configuration quenched alone."""
    items = [setup(ctx, s) for s in SPECS]
    kinds = [dict(precision="staged", s_floor=FLOOR), dict(precision="dd", s_floor=FLOOR),
             dict(precision="staged", s_floor=FLOOR), dict(precision="fp64", s_floor=FLOOR, max_iter=300),
             dict(precision="staged", s_floor=FLOOR)]
    alone = []
    for (w, n, v, pos), o in zip(items, kinds):
        x = dev(pos)
        r = ctx.minimize_batch([w], [x], [v], opts=o)[0]
        alone.append((x.cpu().numpy(), r))
    for perm in (list(range(len(items))), [3, 0, 4, 2, 1]):
        xs = [dev(items[i][3]) for i in perm]
        res = ctx.minimize_batch([items[i][0] for i in perm], xs, [items[i][2] for i in perm],
                                 opts=[kinds[i] for i in perm])
        for i, x, r in zip(perm, xs, res):
            xa, ra = alone[i]
            assert np.array_equal(x.cpu().numpy(), xa), SPECS[i]
            for key in ("phi", "smax", "iters", "evals", "iters_fp64", "evals_fp64", "status"):
                assert r[key] == ra[key], (SPECS[i], key, r[key], ra[key])
    # the staged and double-double ones converged; FP64 alone has no route to 1e-40
    for i, (xa, ra) in enumerate(alone):
        if kinds[i]["precision"] == "fp64":
            assert ra["iters_fp64"] == ra["iters"] and ra["status"] != "converged"
        else:
            assert ra["status"] == "converged", (SPECS[i], ra)


def test_batch_precision_option_errors(ctx):
    w, n, v, pos = setup(ctx, SPECS[0])
    for bad in (dict(precision=3), dict(precision=2, fp64_floor=-1.0), dict(method=2)):
        with pytest.raises(ss.SSError) as e:
            ctx.minimize_batch([w], [dev(pos)], opts=bad)
        assert e.value.code == ss.SS_EINVAL


def test_tiled_pass_in_batch(ctx):
    """A d = 2 configuration with R >= 48 (N = 5000, chi = 0.45: R2 = 2864, R = 53)
    takes the tiled n~ pass in its double-double evaluations and the piece walk in
    FP64: first iterates against the oracle, alone vs mix bitwise, and a staged
    batch that switches passes on its way to the floor."""
    big = (2, 5000, 0.45, 0, 1.0, 71)
    items = [setup(ctx, s) for s in (big, SPECS[1], SPECS[0])]
    w, n, v, pos = items[0]
    assert int(np.sqrt(w.R2)) >= 48
    xs = [dev(it[3]) for it in items]
    res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items], opts=dict(max_iter=3, s_floor=0.0))
    xo, ro, _ = O.minimize(n.cpu().numpy(), None, pos, max_iter=3, s_floor=0.0)
    assert res[0]["iters"] == ro["iters"] == 3 and res[0]["evals"] == ro["evals"]
    assert abs((res[0]["phi"][0] - ro["phi"][0]) + (res[0]["phi"][1] - ro["phi"][1])) <= 1e-26 * ro["phi"][0]
    xg = xs[0].cpu().numpy()
    assert np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max() <= 1e-26
    # alone vs mix, 30 iterations
    opts = dict(max_iter=30, s_floor=0.0)
    xa = dev(pos)
    ra = ctx.minimize_batch([w], [xa], opts=opts)[0]
    xs = [dev(it[3]) for it in items]
    rm = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items], opts=opts)[0]
    assert np.array_equal(xs[0].cpu().numpy(), xa.cpu().numpy()) and rm["phi"] == ra["phi"]
    # staged to the floor
    xs = [dev(it[3]) for it in items]
    res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items],
                             opts=dict(s_floor=FLOOR, precision="staged"))
    for (wi, ni, vi, pi), x, r in zip(items, xs, res):
        assert r["status"] == "converged" and 0 < r["iters_fp64"] < r["iters"], r
        assert oracle_smax(wi, ni, x) <= FLOOR * (1 + 1e-6)
    print(f"d=2 N=5000 staged in a batch: iters={res[0]['iters']} (fp64 {res[0]['iters_fp64']}) "
          f"t={res[0]['seconds']:.2f}s")

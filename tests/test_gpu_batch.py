"""Batched quenches (ss_minimize_batch) against the oracle, alone-vs-mix.

Every configuration of a batch follows the same minimiser rules as a single
quench, so parity is as for ss_minimize: the first iterates agree with the
oracle's to 1e-26 (relative in Phi, absolute in the positions), and full
quenches reach the stated floor when the oracle re-evaluates them.  A
configuration's launch shape depends on (d, N, M) only, so its batched result is
bitwise the same alone and mixed with other configurations.
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


# (d, N, chi, vkind, L, config id): mixed dimensions, sizes (several n(k) units
# and gradient chunks, ragged tails), weights and box sides
MIX = [(2, 128, 0.4, 0, 1.0, 11), (3, 300, 0.3, 1, 1.0, 12), (2, 90, 0.35, 0, 3.0, 13),
       (3, 700, 0.45, 0, 1.0, 14), (1, 40, 0.4, 0, 1.0, 15), (2, 1500, 0.2, 0, 2.0, 16),
       (4, 60, 0.3, 1, 1.0, 17)]


def setup(ctx, spec):
    d, N, chi, vkind, L, cid = spec
    w = ss.Workload.from_chi(d, N, chi, L=L, vkind=vkind)
    n = ctx.wavevectors(d, w.R2)
    v = ctx.weights(w, n) if vkind else None
    pos = inputs.config_positions(cid, d, N, 0)
    return w, n, v, pos


def test_first_iterates_match_oracle(ctx):
    items = [setup(ctx, s) for s in MIX]
    for iters in (1, 3, 5):
        xs = [dev(it[3]) for it in items]
        res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items],
                                 opts=dict(max_iter=iters, s_floor=0.0))
        for (w, n, v, pos), x, r, spec in zip(items, xs, res, MIX):
            nh = n.cpu().numpy()
            vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
            xo, ro, _ = O.minimize(nh, vh, pos, L=w.L, max_iter=iters, s_floor=0.0)
            assert r["iters"] == ro["iters"] == iters, (spec, r, ro)
            assert r["evals"] == ro["evals"], (spec, r, ro)
            dphi = abs((r["phi"][0] - ro["phi"][0]) + (r["phi"][1] - ro["phi"][1]))
            assert dphi <= 1e-26 * ro["phi"][0], (spec, iters, dphi / ro["phi"][0])
            xg = x.cpu().numpy()
            dx = np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max()
            assert dx <= 1e-26, (spec, iters, dx)


def test_alone_vs_mix_bitwise(ctx):
    """Each configuration's positions and results after 30 iterations are the same
    bits alone, in a mix, and in a mix in a different order."""
    items = [setup(ctx, s) for s in MIX]
    opts = dict(max_iter=30, s_floor=0.0)
    alone = []
    for w, n, v, pos in items:
        x = dev(pos)
        r = ctx.minimize_batch([w], [x], [v], opts=opts)[0]
        alone.append((x.cpu().numpy(), r))
    order = [3, 6, 0, 5, 2, 4, 1]
    for perm in (list(range(len(items))), order):
        xs = [dev(items[i][3]) for i in perm]
        res = ctx.minimize_batch([items[i][0] for i in perm], xs, [items[i][2] for i in perm], opts=opts)
        for i, x, r in zip(perm, xs, res):
            xa, ra = alone[i]
            assert np.array_equal(x.cpu().numpy(), xa), MIX[i]
            assert r["phi"] == ra["phi"] and r["smax"] == ra["smax"] and r["evals"] == ra["evals"], MIX[i]


def test_batch_quench_reaches_floor(ctx):
    """A batch of independent d = 2 and d = 3 starts (different sizes, so they stop
    at different steps and the work lists are compacted) all reach the floor; the
    oracle re-evaluates every final configuration."""
    specs = [(2, 128, 0.4, 0, 1.0, 21), (2, 200, 0.3, 0, 1.0, 22), (3, 150, 0.3, 0, 1.0, 23),
             (2, 96, 0.2, 0, 1.0, 24), (3, 250, 0.35, 1, 1.0, 25)]
    items = [setup(ctx, s) for s in specs]
    xs = [dev(it[3]) for it in items]
    res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items], opts=dict(s_floor=FLOOR))
    for (w, n, v, pos), x, r, spec in zip(items, xs, res, specs):
        assert r["status"] == "converged", (spec, r)
        nh = n.cpu().numpy()
        vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
        e = O.energy_from_nk(w.N, vh, O.nk(nh, x.cpu().numpy()))
        assert e.smax[0] <= FLOOR * (1 + 1e-6), (spec, e.smax, r["smax"])
        print(f"{spec}: iters={r['iters']} evals={r['evals']} smax={r['smax'][0]:.3e} t={r['seconds']:.3f}s")


def test_batch_matches_single_rules(ctx):
    """The same configuration quenched by ss_minimize and by a batch of one takes
    the same decisions over 20 iterations (the two launch shapes round differently
    in the last bits, far below the 1e-26 gate)."""
    w, n, v, pos = setup(ctx, MIX[3])
    a, b = dev(pos), dev(pos)
    ra = ctx.minimize(w, n, v, a, max_iter=20, s_floor=0.0)
    rb = ctx.minimize_batch([w], [b], [v], opts=dict(max_iter=20, s_floor=0.0))[0]
    assert ra["iters"] == rb["iters"] and ra["evals"] == rb["evals"]
    assert abs((ra["phi"][0] - rb["phi"][0]) + (ra["phi"][1] - rb["phi"][1])) <= 1e-26 * ra["phi"][0]
    dx = (a - b).abs().max().item()
    assert dx <= 1e-26


def test_tiles_and_errors(ctx):
    w, n, v, pos = setup(ctx, MIX[0])
    t0 = ctx.get_tile(w)
    assert t0 == dict(nk_chunk=64, grad_k=1024)
    ctx.set_tiles([dict(d=2, max_N=1000, max_M=1000, nk_chunk=32, grad_k=256)])
    assert ctx.get_tile(w) == dict(nk_chunk=32, grad_k=256)
    w3 = ss.Workload.from_chi(3, 300, 0.3)
    assert ctx.get_tile(w3) == dict(nk_chunk=64, grad_k=1024)
    # built-in shape for large N: at most 256 partial rows
    big = ss.Workload(2, 100000, 100, ss.count(2, 100), 1.0, 0)
    assert ctx.get_tile(big) == dict(nk_chunk=391, grad_k=1024)
    # a different tile still satisfies the parity gate against the oracle
    x = dev(pos)
    r = ctx.minimize_batch([w], [x], opts=dict(max_iter=3, s_floor=0.0))[0]
    xo, ro, _ = O.minimize(n.cpu().numpy(), None, pos, max_iter=3, s_floor=0.0)
    assert abs((r["phi"][0] - ro["phi"][0]) + (r["phi"][1] - ro["phi"][1])) <= 1e-26 * ro["phi"][0]
    ctx.set_tiles([])
    assert ctx.get_tile(w) == t0
    with pytest.raises(ss.SSError) as e:
        ctx.set_tiles([dict(d=2, max_N=10, max_M=10, nk_chunk=0, grad_k=1)])
    assert e.value.code == ss.SS_EINVAL
    with pytest.raises(ss.SSError) as e:
        ctx.minimize_batch([w], [dev(pos)], opts=dict(history=0))
    assert e.value.code == ss.SS_EINVAL
    wv = ss.Workload.from_chi(2, 128, 0.4, vkind=1)
    with pytest.raises(ss.SSError) as e:
        ctx.minimize_batch([wv], [dev(pos)], [None])
    assert e.value.code == ss.SS_EINVAL
    with pytest.raises(ss.SSError) as e:
        ctx.minimize_batch([w], [dev(pos)], ws=torch.empty(1024, dtype=torch.uint8, device="cuda"))
    assert e.value.code == ss.SS_EINVAL
    # max_iter = 0 leaves the positions untouched
    x = dev(pos)
    r = ctx.minimize_batch([w], [x], opts=dict(max_iter=0))[0]
    assert r["iters"] == 0 and r["status"] == "max_iter"
    assert np.array_equal(x.cpu().numpy(), pos)


def test_numeric_fault_isolated_in_batch(ctx):
    """One configuration of a batch whose energy turns non-finite (a NaN injected
    into its trial point of iteration 5) stops with status 3 (numeric); every
    other configuration gives the same bits as alone."""
    items = [setup(ctx, s) for s in MIX]
    opts = dict(max_iter=30, s_floor=0.0)
    alone = []
    for w, n, v, pos in items:
        x = dev(pos)
        r = ctx.minimize_batch([w], [x], [v], opts=opts)[0]
        alone.append((x.cpu().numpy(), r))
    bad = 3
    xs = [dev(it[3]) for it in items]
    olist = [dict(opts, fault_iter=5 if i == bad else 0) for i in range(len(items))]
    res = ctx.minimize_batch([it[0] for it in items], xs, [it[2] for it in items], opts=olist)
    for i, (x, r) in enumerate(zip(xs, res)):
        if i == bad:
            assert r["status"] == "numeric", r
            assert r["iters"] == 5, r  # the faulted iteration counts
            continue
        xa, ra = alone[i]
        assert np.array_equal(x.cpu().numpy(), xa), MIX[i]
        assert r["phi"] == ra["phi"] and r["iters"] == ra["iters"] and r["status"] == ra["status"], MIX[i]

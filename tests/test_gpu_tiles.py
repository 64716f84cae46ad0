"""Parity of the measured tile table (tiles.json), the launch shapes that the
batched and served throughput figures run on.

A batched configuration's n~(k) pass is split into units of `nk_chunk`
particles and its gradient pass into blocks of `grad_k` wavevectors; the
reduction order follows these shapes, so every shape the table can hand out is
checked here against the oracle:

* every distinct tuned shape, transplanted onto a configuration with several
  units and gradient blocks and ragged tails (d = 2 on the walk and on the
  tiled pass, d = 3): the first iterates agree with the oracle's to 1e-26 and
  each configuration gives the same bits alone and in the mix;
* with the tuned table itself, one configuration inside every table entry
  (sizes at the entry's lower edges): first iterates against the oracle where
  the oracle finishes in seconds, and the batch of one, the mix and the server
  agree bit for bit.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2304_09139_amd import inputs, ss
from paper_2304_09139_amd.tune import load_tiles

pytestmark = pytest.mark.gpu

TILES = load_tiles()
# particle-wavevector pairs above which the oracle's first iterate is skipped
ORACLE_PAIRS = 1.2e8


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def r2_for(d, m_lo):
    """The smallest R2 whose half set holds at least m_lo wavevectors."""
    lo, hi = 1, 1
    while ss.count(d, hi) < m_lo:
        hi *= 2
    while lo < hi:
        mid = (lo + hi) // 2
        if ss.count(d, mid) >= m_lo:
            hi = mid
        else:
            lo = mid + 1
    return lo


def oracle_check(w, n, v, pos, x, r, iters, tag):
    nh = n.cpu().numpy()
    vh = O.weights(nh, w.R2, w.vkind) if w.vkind else None
    xo, ro, _ = O.minimize(nh, vh, pos, L=w.L, max_iter=iters, s_floor=0.0)
    assert r["iters"] == ro["iters"] == iters and r["evals"] == ro["evals"], (tag, r, ro)
    dphi = abs((r["phi"][0] - ro["phi"][0]) + (r["phi"][1] - ro["phi"][1]))
    assert dphi <= 1e-26 * ro["phi"][0], (tag, dphi / ro["phi"][0])
    xg = x.cpu().numpy()
    dx = np.abs((xg[0] - xo[0]) + (xg[1] - xo[1])).max()
    assert dx <= 1e-26, (tag, dx)
    return dphi / ro["phi"][0], dx


def transplant_cases():
    """(d, N, R2, nk_chunk, grad_k) for every distinct tuned shape: N spans at
    least two full particle units plus a ragged one, M at least one full
    gradient block plus a ragged one; d = 2 both below (walk) and at or above
    (tiled pass) a cutoff radius of 48."""
    shapes = sorted({(e["d"], e["nk_chunk"], e["grad_k"]) for e in TILES})
    cases, used_n = [], set()
    for d, nk_chunk, grad_k in shapes:
        variants = [False, True] if d == 2 else [False]
        for tiled in variants:
            m_lo = int(1.3 * grad_k) + 7
            if tiled:
                m_lo = max(m_lo, ss.count(2, 48 * 48))
            R2 = r2_for(d, m_lo)
            M = ss.count(d, R2)
            if d == 2 and not tiled and int(np.sqrt(R2)) >= 48:
                continue  # this gradient block needs the tiled range
            N = max(2 * nk_chunk + 37, int(M / (0.45 * d)) + 2)
            while N in used_n:
                N += 1
            used_n.add(N)
            assert M / (d * (N - 1)) < 0.5
            cases.append((d, N, R2, nk_chunk, grad_k))
    return cases


@pytest.mark.skipif(not TILES, reason="no tile table")
def test_tuned_shapes_transplanted_match_oracle():
    cases = transplant_cases()
    # one table entry per case, ascending N (all N distinct): each configuration
    # matches its own entry first
    table = [dict(d=d, max_N=N, max_M=1 << 40, nk_chunk=c, grad_k=g) for d, N, R2, c, g in sorted(cases, key=lambda t: t[1])]
    ctx = ss.Context(0, tiles=table)
    try:
        items = []
        for i, (d, N, R2, c, g) in enumerate(cases):
            w = ss.Workload(d, N, R2, ss.count(d, R2), 1.0, 1 if i % 3 == 1 else 0)
            assert ctx.get_tile(w) == dict(nk_chunk=c, grad_k=g)
            n = ctx.wavevectors(d, R2)
            v = ctx.weights(w, n) if w.vkind else None
            items.append((w, n, v, inputs.config_positions(61, d, N, i)))
        works, vs = [it[0] for it in items], [it[2] for it in items]
        # first iterates of the mix against the oracle
        xs = [dev(it[3]) for it in items]
        res = ctx.minimize_batch(works, xs, vs, opts=dict(max_iter=2, s_floor=0.0))
        for it, x, r, case in zip(items, xs, res, cases):
            rel, dx = oracle_check(*it, x, r, 2, case)
            print(f"{case}: M={it[0].M} |dPhi|/Phi={rel:.1e} |dx|={dx:.1e}")
        # alone vs mix, 25 iterations
        opts = dict(max_iter=25, s_floor=0.0)
        xs = [dev(it[3]) for it in items]
        mix = ctx.minimize_batch(works, xs, vs, opts=opts)
        for it, x, r, case in zip(items, xs, mix, cases):
            xa = dev(it[3])
            ra = ctx.minimize_batch([it[0]], [xa], [it[2]], opts=opts)[0]
            assert torch.equal(xa, x), case
            assert ra["phi"] == r["phi"] and ra["evals"] == r["evals"], case
    finally:
        ctx.close()


def entry_cases():
    """One configuration inside every entry of the tuned table: N at the entry's
    lower N edge (the largest max_N of an earlier entry of the same d; 500 for
    the first), M above the entry's lower M edge (the largest max_M of an
    earlier entry of the same d and max_N), near chi = 0.3 where the oracle's
    cost allows, and chi < 1/2."""
    cases = []
    for i, e in enumerate(TILES):
        d = e["d"]
        prev_n = [t["max_N"] for t in TILES[:i] if t["d"] in (0, d) and t["max_N"] < e["max_N"]]
        n_lo = max(prev_n) + 1 if prev_n else min(500, e["max_N"])
        prev_m = [t["max_M"] for t in TILES[:i] if t["d"] in (0, d) and t["max_N"] == e["max_N"]]
        m_lo = max(prev_m) + 1 if prev_m else 1
        m_want = max(m_lo, min(int(0.3 * d * (n_lo - 1)), int(0.95 * ORACLE_PAIRS / n_lo), e["max_M"]))
        R2 = r2_for(d, max(m_want, 4))
        M = ss.count(d, R2)
        N = max(n_lo, int(M / (0.49 * d)) + 2)
        if M > e["max_M"] or N > e["max_N"]:
            continue
        cases.append((i, d, N, R2, M))
    return cases


@pytest.mark.skipif(not TILES, reason="no tile table")
def test_tuned_table_entries_oracle_mix_and_server():
    ctx = ss.Context(0, tiles="tuned")
    try:
        cases = entry_cases()
        assert len(cases) >= len(TILES) * 2 // 3, cases
        items = []
        for i, d, N, R2, M in cases:
            w = ss.Workload(d, N, R2, M, 1.0, 0)
            e = TILES[i]
            assert ctx.get_tile(w) == dict(nk_chunk=e["nk_chunk"], grad_k=e["grad_k"]), (e, w)
            items.append((w, ctx.wavevectors(d, R2), None, inputs.config_positions(62, d, N, i)))
        works = [it[0] for it in items]
        xs = [dev(it[3]) for it in items]
        res = ctx.minimize_batch(works, xs, None, opts=dict(max_iter=1, s_floor=0.0))
        checked = 0
        for it, x, r, case in zip(items, xs, res, cases):
            w = it[0]
            if w.M * w.N <= ORACLE_PAIRS:
                rel, dx = oracle_check(*it, x, r, 1, case)
                checked += 1
                print(f"entry {case}: |dPhi|/Phi={rel:.1e} |dx|={dx:.1e}")
        assert checked >= len(cases) // 2, (checked, len(cases))
        # batch of one, mix and server: the same bits over 12 iterations
        opts = dict(max_iter=12, s_floor=0.0)
        xs = [dev(it[3]) for it in items]
        mix = ctx.minimize_batch(works, xs, None, opts=opts)
        alone = []
        for it in items:
            xa = dev(it[3])
            alone.append((ctx.minimize_batch([it[0]], [xa], None, opts=opts)[0], xa.cpu().numpy()))
        for (ra, xa), x, r, case in zip(alone, xs, mix, cases):
            assert np.array_equal(x.cpu().numpy(), xa), case
            assert r["phi"] == ra["phi"], case
        ctx.server_start(16 << 30, max_slots=len(items) + 2)
        try:
            tickets = []
            for it in reversed(items):
                tickets.append(ctx.submit(it[0], it[3], **opts))
                time.sleep(0.002)
            for t, (ra, xa), case in zip(reversed(tickets), alone, cases):
                t0 = time.time()
                while (got := ctx.poll(t)) is None:
                    assert time.time() - t0 < 120
                    time.sleep(0.002)
                r, xsrv = got
                assert np.array_equal(xsrv, xa), case
                assert r["phi"] == ra["phi"], case
        finally:
            ctx.server_stop()
    finally:
        ctx.close()

"""Serving (ss_server_start / ss_submit / ss_poll / ss_server_stop).

A served request runs the batched minimiser under the same tile table, so its
result must equal ss_minimize_batch's result for the same configuration bit for
bit, whether it is served alone or mixed with other requests arriving at other
times; served quenches reach the stated floor (re-evaluated by the oracle);
admission waits for arena space; errors are reported per request.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2304_09139_amd import inputs, ss

pytestmark = pytest.mark.gpu

FLOOR = 1e-40


@pytest.fixture()
def ctx():
    c = ss.Context(0)
    yield c
    c.close()


def wait(ctx, ticket, limit=120.0):
    t0 = time.time()
    while True:
        r = ctx.poll(ticket)
        if r is not None:
            return r
        assert time.time() - t0 < limit, f"ticket {ticket} still pending"
        time.sleep(0.002)


SPECS = [(2, 128, 0.4, 0, 1.0, 41), (3, 300, 0.3, 1, 1.0, 42), (2, 700, 0.35, 0, 2.0, 43),
         (3, 500, 0.45, 0, 1.0, 44), (2, 96, 0.2, 0, 1.0, 45)]


def make(spec):
    d, N, chi, vkind, L, cid = spec
    return ss.Workload.from_chi(d, N, chi, L=L, vkind=vkind), inputs.config_positions(cid, d, N, 0)


def test_served_equals_batch_alone_and_mixed(ctx):
    """Bitwise: batch of one == served alone == served in a staggered mix."""
    items = [make(s) for s in SPECS]
    opts = dict(max_iter=60, s_floor=0.0)
    ref = []
    for w, pos in items:
        x = torch.from_numpy(pos).cuda()
        v = ctx.weights(w, ctx.wavevectors(w.d, w.R2)) if w.vkind else None
        r = ctx.minimize_batch([w], [x], [v], opts=opts)[0]
        ref.append((r, x.cpu().numpy()))
    ctx.server_start(1 << 30, max_slots=8)
    try:
        # alone
        for (w, pos), (rb, xb) in zip(items, ref):
            r, xs = wait(ctx, ctx.submit(w, pos, **opts))
            assert np.array_equal(xs, xb) and r["phi"] == rb["phi"] and r["evals"] == rb["evals"]
        # mixed: staggered submissions in another order
        tickets = {}
        for i in [3, 0, 4, 1, 2]:
            tickets[i] = ctx.submit(items[i][0], items[i][1], **opts)
            time.sleep(0.003)
        for i, t in tickets.items():
            r, xs = wait(ctx, t)
            rb, xb = ref[i]
            assert np.array_equal(xs, xb), SPECS[i]
            assert r["phi"] == rb["phi"] and r["smax"] == rb["smax"] and r["iters"] == rb["iters"], SPECS[i]
    finally:
        ctx.server_stop()


def test_served_quenches_reach_floor(ctx):
    items = [make(s) for s in SPECS]
    ctx.server_start(1 << 30, max_slots=3)   # fewer slots than requests: queueing
    try:
        tickets = [ctx.submit(w, pos, s_floor=FLOOR) for w, pos in items]
        for (w, pos), t, spec in zip(items, tickets, SPECS):
            r, xs = wait(ctx, t)
            assert r["status"] == "converged", (spec, r)
            n = O.wavevectors(w.d, w.R2)
            v = O.weights(n, w.R2, 1) if w.vkind else None
            e = O.energy_from_nk(w.N, v, O.nk(n, xs))
            assert e.smax[0] <= FLOOR * (1 + 1e-6), (spec, e.smax, r["smax"])
            print(f"{spec}: iters={r['iters']} latency={r['seconds']:.3f}s")
    finally:
        ctx.server_stop()


def test_served_staged_equals_batch(ctx):
    """Staged requests switch to double-double inside the server on their own:
    served mixed with double-double requests, each result equals the batch of
    one bit for bit and reaches the floor."""
    items = [make(s) for s in SPECS[:4]]
    kinds = [dict(precision="staged"), dict(precision="dd"), dict(precision="staged"), dict(precision="staged")]
    ref = []
    for (w, pos), o in zip(items, kinds):
        x = torch.from_numpy(pos).cuda()
        v = ctx.weights(w, ctx.wavevectors(w.d, w.R2)) if w.vkind else None
        r = ctx.minimize_batch([w], [x], [v], opts=dict(o, s_floor=FLOOR))[0]
        ref.append((r, x.cpu().numpy()))
    ctx.server_start(1 << 30, max_slots=8)
    try:
        tickets = {}
        for i in [2, 0, 3, 1]:
            tickets[i] = ctx.submit(items[i][0], items[i][1], s_floor=FLOOR, **kinds[i])
            time.sleep(0.005)
        for i, t in tickets.items():
            r, xs = wait(ctx, t)
            rb, xb = ref[i]
            assert np.array_equal(xs, xb), SPECS[i]
            for key in ("phi", "smax", "iters", "evals", "iters_fp64", "evals_fp64", "status"):
                assert r[key] == rb[key], (SPECS[i], key, r[key], rb[key])
            assert r["status"] == "converged", (SPECS[i], r)
            if kinds[i]["precision"] == "staged":
                assert 0 < r["iters_fp64"] < r["iters"], (SPECS[i], r)
            w = items[i][0]
            n = O.wavevectors(w.d, w.R2)
            v = O.weights(n, w.R2, 1) if w.vkind else None
            assert O.energy_from_nk(w.N, v, O.nk(n, xs)).smax[0] <= FLOOR * (1 + 1e-6), SPECS[i]
    finally:
        ctx.server_stop()


def test_seeded_request_equals_given_start(ctx):
    """A request without positions starts from the library's uniform start of its
    seed: the same bits as the request that passes that start explicitly."""
    w, _ = make(SPECS[0])
    seed = inputs.stream_seed(47, 3)
    pos = inputs.uniform_positions(w.d, w.N, seed)
    ctx.server_start(1 << 28, max_slots=4)
    try:
        t0 = ctx.submit(w, None, seed=seed, s_floor=FLOOR)
        t1 = ctx.submit(w, pos, s_floor=FLOOR)
        (r0, x0), (r1, x1) = wait(ctx, t0), wait(ctx, t1)
        assert np.array_equal(x0, x1) and r0["phi"] == r1["phi"] and r0["iters"] == r1["iters"]
        assert r0["status"] == "converged"
    finally:
        ctx.server_stop()


def test_small_arena_admission(ctx):
    """An arena that holds about one configuration at a time still serves all
    requests, one after another; a request larger than the arena fails alone."""
    items = [make(s) for s in SPECS[:3]]
    need = max(ctx.batch_workspace_size([w], [dict(ss.DEFAULT_MIN_OPTS)]) for w, _ in items)
    ctx.server_start(int(need * 1.5), max_slots=4)
    try:
        big = ss.Workload.from_chi(3, 6000, 0.45)
        # larger than the whole arena: refused at submission, nothing queued
        with pytest.raises(ss.SSError) as e:
            ctx.submit(big, inputs.config_positions(46, 3, 6000, 0), max_iter=5)
        assert e.value.code == ss.SS_ENOMEM
        tickets = [ctx.submit(w, pos, max_iter=40, s_floor=0.0) for w, pos in items]
        for t in tickets:
            r, _ = wait(ctx, t)
            assert r["iters"] == 40
        st = ctx.server_stats()
        assert st["submitted"] == 3 and st["completed"] == 3, st
    finally:
        ctx.server_stop()


def test_serving_errors(ctx):
    w, pos = make(SPECS[0])
    with pytest.raises(ss.SSError) as e:
        ctx.submit(w, pos)
    assert e.value.code == ss.SS_ESTATE
    ctx.server_start(1 << 28, max_slots=2)
    try:
        with pytest.raises(ss.SSError) as e:
            ctx.server_start(1 << 20, max_slots=2)
        assert e.value.code == ss.SS_ESTATE
        for bad in (dict(history=0), dict(method=2), dict(precision=3)):
            with pytest.raises(ss.SSError) as e:
                ctx.submit(w, pos, **bad)
            assert e.value.code == ss.SS_EINVAL
        badpos = pos.copy()
        badpos[0, 0, 0] = np.inf
        with pytest.raises(ss.SSError) as e:
            ctx.submit(w, badpos)
        assert e.value.code == ss.SS_EINVAL
        assert ss.lib().ss_poll(ctx._h, 987654321, None, None) == ss.SS_ENOTFOUND
        t = ctx.submit(w, pos, max_iter=0)
        r, xs = wait(ctx, t)
        assert r["iters"] == 0 and np.array_equal(xs, pos)
        assert ss.lib().ss_poll(ctx._h, t, None, None) == ss.SS_ENOTFOUND
    finally:
        ctx.server_stop()
    ctx.server_stop()  # stopping twice is harmless


def test_requests_overlap_and_stay_bitwise(ctx):
    """Continuous batching: requests submitted while others run are admitted at
    step boundaries and run together (the server's peak count of running
    configurations is at least 2 and it admitted requests while others were
    running), and each result is still the batch of one's bit for bit."""
    items = [make(s) for s in SPECS]
    opts = dict(max_iter=200, s_floor=0.0)
    ref = []
    for w, pos in items:
        x = torch.from_numpy(pos).cuda()
        v = ctx.weights(w, ctx.wavevectors(w.d, w.R2)) if w.vkind else None
        r = ctx.minimize_batch([w], [x], [v], opts=opts)[0]
        ref.append((r, x.cpu().numpy()))
    ctx.server_start(1 << 30, max_slots=8)
    try:
        first = ctx.submit(items[3][0], items[3][1], **opts)
        # wait until the first request is running, then submit the others
        t0 = time.time()
        while ctx.server_stats()["running"] < 1 and ctx.poll(first) is None:
            assert time.time() - t0 < 60
            time.sleep(0.0005)
        tickets = {3: first}
        for i in [0, 4, 1, 2]:
            tickets[i] = ctx.submit(items[i][0], items[i][1], **opts)
        results = {i: wait(ctx, t) for i, t in tickets.items()}
        st = ctx.server_stats()
        print("server counters:", st)
        assert st["max_running"] >= 2, st
        assert st["admitted"] == 5 and st["completed"] == 5, st
        for i, (r, xs) in results.items():
            rb, xb = ref[i]
            assert np.array_equal(xs, xb), SPECS[i]
            assert r["phi"] == rb["phi"] and r["iters"] == rb["iters"] == 200, SPECS[i]
    finally:
        ctx.server_stop()


def test_numeric_fault_isolated_in_server(ctx):
    """A request whose energy turns non-finite (a NaN injected into its trial
    point of iteration 7) ends on its own with status 3 (numeric); the requests
    served beside it give the same bits as the batch of one."""
    items = [make(s) for s in SPECS[:4]]
    opts = dict(max_iter=40, s_floor=0.0)
    ref = []
    for w, pos in items:
        x = torch.from_numpy(pos).cuda()
        v = ctx.weights(w, ctx.wavevectors(w.d, w.R2)) if w.vkind else None
        r = ctx.minimize_batch([w], [x], [v], opts=opts)[0]
        ref.append((r, x.cpu().numpy()))
    bad = 1
    ctx.server_start(1 << 30, max_slots=8)
    try:
        tickets = {i: ctx.submit(w, pos, **dict(opts, fault_iter=7 if i == bad else 0))
                   for i, (w, pos) in enumerate(items)}
        for i, t in tickets.items():
            r, xs = wait(ctx, t)
            if i == bad:
                assert r["status"] == "numeric", r
                assert r["iters"] == 7, r  # the faulted iteration counts
                continue
            rb, xb = ref[i]
            assert np.array_equal(xs, xb), SPECS[i]
            assert r["phi"] == rb["phi"] and r["iters"] == rb["iters"] == 40, SPECS[i]
        # the server keeps serving after the fault
        r, xs = wait(ctx, ctx.submit(items[0][0], items[0][1], **opts))
        assert np.array_equal(xs, ref[0][1])
    finally:
        ctx.server_stop()

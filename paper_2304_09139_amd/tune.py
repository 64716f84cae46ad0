"""Measure the batched tile shapes and write the tile table (tiles.json).

The batched launches split each configuration's n~(k) pass into units of
`nk_chunk` particles and its gradient pass into blocks of `grad_k`
wavevectors.  Both are looked up by (d, N, M) in the context's tile table
(first entry with N <= max_N and M <= max_M).  The table is keyed by d, an N
bucket and an M bucket: for every (d, N bucket) a seeded pool of batch shapes
(N log-uniform in the bucket, chi in {0.2, 0.35, 0.45}) is split at the
tertiles of its M values into three M buckets, and for every (d, N bucket, M
bucket) this script quenches a batch of that bucket's configurations for a
fixed number of L-BFGS iterations with every candidate shape, keeping the shape
with the highest pair throughput.

    python -m paper_2304_09139_amd.tune [--out tiles.json] [--count 48] [--iters 12]

Changing the table changes batched results in their last bits (the reduction
order follows the tile), so a table is fixed before production runs.
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TILES_PATH = os.path.join(HERE, "tiles.json")

NK_CHUNKS = (32, 64, 128, 256)
GRAD_KS = (256, 512, 1024, 2048)
# (d, N range) buckets of the batched mixes (N from 500 to 5000)
BUCKETS = [(2, 500, 1000), (2, 1000, 2000), (2, 2000, 5000), (3, 500, 1000), (3, 1000, 2000), (3, 2000, 5000)]
# larger systems (served requests up to N = 1e5): fewer configurations per batch
# and longer particle chunks
LARGE_BUCKETS = [(2, 5000, 20000), (2, 20000, 100000), (3, 5000, 20000), (3, 20000, 100000)]
NK_CHUNKS_LARGE = (128, 256, 512, 1024)
GRAD_KS_LARGE = (1024, 2048)
M_BUCKETS = 3


def load_tiles(path: str = TILES_PATH) -> list[dict]:
    """The committed tile table, or [] when there is none."""
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        return json.load(fh)["tiles"]


def bucket_pools(d: int, n_lo: int, n_hi: int, count: int):
    """The configurations of (d, [n_lo, n_hi]) split into M_BUCKETS M buckets:
    a list of (max_M, [(N, chi), ...]) with ascending max_M (the last one
    unbounded), each with at most `count` configurations."""
    from . import inputs, ss

    pool = []
    for d_, N, chi in inputs.batch_shapes(count * M_BUCKETS * 2, seed=100 + d * 10 + n_lo // 500,
                                          n_min=n_lo, n_max=n_hi, dims=(d,)):
        R2, M = ss.cutoff(d_, N, chi)
        pool.append((M, N, chi))
    pool.sort()
    edges = [pool[(len(pool) * (b + 1)) // M_BUCKETS - 1][0] for b in range(M_BUCKETS - 1)]
    out = []
    lo = 0
    for b in range(M_BUCKETS):
        hi = edges[b] if b < M_BUCKETS - 1 else 1 << 40
        members = [(N, chi) for M, N, chi in pool if lo < M <= hi]
        out.append((hi, members[:count]))
        lo = hi
    return out


def tune(count: int = 48, iters: int = 12, out: str = TILES_PATH) -> list[dict]:
    import torch

    from . import inputs, ss

    ctx = ss.Context(0)
    entries = []
    plan = [(b, count, NK_CHUNKS, GRAD_KS) for b in BUCKETS] + \
           [(b, max(4, count // 8), NK_CHUNKS_LARGE, GRAD_KS_LARGE) for b in LARGE_BUCKETS]
    for (d, n_lo, n_hi), cnt, chunks, gks in plan:
        for max_M, members in bucket_pools(d, n_lo, n_hi, cnt):
            works = [ss.Workload.from_chi(d, N, chi) for N, chi in members]
            starts = [inputs.config_positions(7, w.d, w.N, i) for i, w in enumerate(works)]
            best = None
            for nk_chunk in chunks:
                for grad_k in gks:
                    ctx.set_tiles([dict(d=0, max_N=1 << 40, max_M=1 << 40, nk_chunk=nk_chunk, grad_k=grad_k)])
                    rate = []
                    for rep in range(2):
                        xs = [torch.from_numpy(p).cuda() for p in starts]
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        res = ctx.minimize_batch(works, xs, opts=dict(max_iter=iters, s_floor=0.0))
                        torch.cuda.synchronize()
                        dt = time.perf_counter() - t0
                        pairs = sum(w.M * w.N * r["evals"] for w, r in zip(works, res))
                        rate.append(pairs / dt)
                    r = max(rate)
                    print(f"d={d} N=({n_lo},{n_hi}] M<={max_M} nk_chunk={nk_chunk} grad_k={grad_k}: "
                          f"{r:.3e} pairs/s", flush=True)
                    if best is None or r > best[0]:
                        best = (r, nk_chunk, grad_k)
            entries.append(dict(d=d, max_N=n_hi, max_M=max_M, nk_chunk=best[1], grad_k=best[2],
                                pairs_per_s=best[0], configs=len(works),
                                M_seen=[min(w.M for w in works), max(w.M for w in works)]))
    ctx.close()
    with open(out, "w") as fh:
        json.dump({"tiles": entries, "count": count, "iters": iters}, fh, indent=1)
    return entries


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TILES_PATH)
    ap.add_argument("--count", type=int, default=48)
    ap.add_argument("--iters", type=int, default=12)
    a = ap.parse_args()
    for e in tune(a.count, a.iters, a.out):
        print(json.dumps(e))

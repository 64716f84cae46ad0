"""Host logic of the tile table (no GPU): the M buckets of every (d, N bucket)
partition its seeded pool at ascending edges, and the committed table is
ordered so that the first matching entry is the entry of a configuration's own
(d, N bucket, M bucket)."""
from paper_2304_09139_amd import ss, tune


def test_bucket_pools_partition():
    for d, lo, hi in tune.BUCKETS[:2] + tune.LARGE_BUCKETS[:1]:
        pools = tune.bucket_pools(d, lo, hi, 16)
        assert len(pools) == tune.M_BUCKETS
        edges = [m for m, _ in pools]
        assert edges == sorted(edges) and edges[-1] == 1 << 40
        prev = 0
        for max_M, members in pools:
            assert members, (d, lo, hi, max_M)
            for N, chi in members:
                assert lo <= N <= hi
                _, M = ss.cutoff(d, N, chi)
                assert prev < M <= max_M
            prev = max_M


def first_match(tiles, d, N, M):
    for e in tiles:
        if e["d"] in (0, d) and N <= e["max_N"] and M <= e["max_M"]:
            return e
    return None


def test_committed_table_first_match():
    tiles = tune.load_tiles()
    assert tiles, "tiles.json is missing"
    for i, e in enumerate(tiles):
        # a configuration just inside the entry's N and M edges finds this entry first
        prev_n = [t["max_N"] for t in tiles[:i] if t["d"] == e["d"] and t["max_N"] < e["max_N"]]
        prev_m = [t["max_M"] for t in tiles[:i] if t["d"] == e["d"] and t["max_N"] == e["max_N"]]
        N = (max(prev_n) + 1) if prev_n else e["max_N"]
        M = (max(prev_m) + 1) if prev_m else 1
        assert first_match(tiles, e["d"], N, M) is e, (i, e)
        assert first_match(tiles, e["d"], e["max_N"], min(e["max_M"], 1 << 39)) is e, (i, e)

"""GPU parity of batched traversals (many queries over graphs packed in one
CSR arena, per-bucket threshold and coarsening) against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2201_02789_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_02789_amd import dpo  # noqa: E402


@pytest.fixture(scope="module")
def mixed():
    """R-MAT graphs of several sizes plus structured ones, weighted."""
    graphs, queries = gg.batch_workload(seed=5, ngraphs=10, sources_per_graph=3, scales=(7, 13),
                                        edgefactors=(4, 24))
    extra = [gg.path_graph(700), gg.star_graph(5000), gg.grid_graph(40, 37),
             gg.from_edges(70, [(1, 2), (3, 4)]), gg.complete_graph(90)]
    base = len(graphs)
    graphs += extra
    queries += [(base, 0), (base, 699), (base + 1, 0), (base + 1, 17), (base + 2, 5),
                (base + 3, 0), (base + 3, 2), (base + 4, 1)]
    graphs = [gg.add_weights(g, 31 + i) for i, g in enumerate(graphs)]
    arena, vbase = gg.pack_arena(graphs)
    # bucket by size: small graphs T=8/CF=2, large T=64/CF=1
    qs = [(g, s, 0 if graphs[g].n < 3000 else 1) for g, s in queries]
    return graphs, qs, dpo.DeviceArena(arena, vbase)


BUCKETS = [dict(threshold=8, coarsen=2), dict(threshold=64, coarsen=1)]


def bucket_opts(**common):
    return [dpo.Options(**{**common, **b}) for b in BUCKETS]


def run_batch(kind, da, qs, bopts, stats=False):
    tot, slot0 = dpo.dpo_batch_slots(da, qs)
    out = torch.full((tot,), -7, dtype=torch.int32, device="cuda")
    ws = torch.empty(dpo.dpo_batch_workspace_bytes(da, qs, bopts[0]), dtype=torch.uint8,
                     device="cuda")
    f = dpo.dpo_bfs_batch if kind == "bfs" else dpo.dpo_sssp_batch
    st = f(da, qs, bopts, out, ws, stats=stats)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    return host, slot0, st


MODES = [dict(), dict(agg=dpo.DPO_AGG_WAVE), dict(agg=dpo.DPO_AGG_BLOCK),
         dict(agg=dpo.DPO_AGG_MULTIBLOCK, agg_blocks=16), dict(agg=dpo.DPO_AGG_NONE),
         dict(mode=dpo.DPO_MODE_FLAT), dict(child_block=64, steps_per_replay=2),
         dict(split_min=0), dict(split_min=256, steps_per_replay=3), dict(serial_wave=0),
         dict(child_block=128), dict(agg=dpo.DPO_AGG_GRID, child_block=128),
         dict(agg=dpo.DPO_AGG_NONE, child_block=128, split_min=0),
         dict(child_block=128, dyn_share=25), dict(agg=dpo.DPO_AGG_NONE, dyn_share=100),
         dict(split_min=0, claim_hint=dpo.DPO_HINT_ON), dict(split_min=0, claim_hint=dpo.DPO_HINT_OFF)]


@pytest.mark.parametrize("common", MODES, ids=[str(m) for m in MODES])
def test_bfs_batch_matches_oracle_per_query(mixed, common):
    graphs, qs, da = mixed
    bopts = bucket_opts(**common)
    host, slot0, st = run_batch("bfs", da, qs, bopts, stats=True)
    want_counts = {}
    for i, (g, s, b) in enumerate(qs):
        n = graphs[g].n
        want, _ = oracle.bfs(graphs[g], s)
        got = host[slot0[i]:slot0[i] + n]
        assert np.array_equal(got, want), (i, g, s, common)
        flat = common.get("mode") == dpo.DPO_MODE_FLAT
        c = oracle.schedule_counts(graphs[g], want, BUCKETS[b]["threshold"],
                                   common.get("child_block", 256), BUCKETS[b]["coarsen"], flat=flat)
        for k, v in c.items():
            want_counts[k] = want_counts.get(k, 0) + v
    got_counts = {k: st[k] for k in want_counts}
    assert got_counts == want_counts, common


SSSP_MODES = MODES


@pytest.mark.parametrize("common", SSSP_MODES, ids=[str(m) for m in SSSP_MODES])
def test_sssp_batch_matches_oracle_per_query(mixed, common):
    graphs, qs, da = mixed
    host, slot0, _ = run_batch("sssp", da, qs, bucket_opts(**common))
    host = host.view(np.uint32)
    for i, (g, s, b) in enumerate(qs):
        want = oracle.dijkstra(graphs[g], s)
        assert np.array_equal(host[slot0[i]:slot0[i] + graphs[g].n], want), (i, g, s, common)


def test_batch_of_one_equals_single_call(mixed):
    graphs, qs, da = mixed
    g, s, b = qs[4]
    host, slot0, _ = run_batch("bfs", da, [(g, s, 0)], bucket_opts())
    dg = dpo.DeviceGraph.from_host(graphs[g])
    single, _ = dpo.bfs(dg, s, bucket_opts()[0])
    assert np.array_equal(host[:graphs[g].n], single.cpu().numpy())


def test_repeated_queries_identical(mixed):
    graphs, qs, da = mixed
    g, s, _ = qs[7]
    rep = [(g, s, 0)] * 5 + [(g, s, 1)] * 3
    host, slot0, _ = run_batch("bfs", da, rep, bucket_opts())
    first = host[slot0[0]:slot0[0] + graphs[g].n]
    for i in range(1, len(rep)):
        assert np.array_equal(host[slot0[i]:slot0[i] + graphs[g].n], first)


@pytest.fixture(scope="module")
def batch512():
    graphs, queries = gg.batch_workload()
    arena, vbase = gg.pack_arena(graphs)
    wants = [oracle.bfs(graphs[g], s)[0] for g, s in queries]
    return graphs, queries, dpo.DeviceArena(arena, vbase), wants


def bench_bucket_options():
    """The batched benchmark's bucket split (scales 10-12, 13-15, 16-18) and
    per-bucket options at the points its tuner has chosen on MI355X, and its
    untuned base point."""
    base = dict(threshold=32, coarsen=1, agg=dpo.DPO_AGG_MULTIBLOCK, agg_blocks=4,
                child_block=128)
    tuned = [dpo.Options(**base), dpo.Options(**base), dpo.Options(**{**base, "threshold": 128})]
    return tuned, [dpo.Options(**base)]


@pytest.mark.slow
@pytest.mark.parametrize("which", ["tuned", "untuned", "two-buckets-CB256", "16-block",
                                   "grid", "lane-serial"])
def test_batch_512_queries_over_64_graphs_bfs(batch512, which):
    """The batched workload: 512 BFS over 64 R-MAT graphs, scales 10..18, at
    the benchmarked per-bucket options and other granularities; every query
    against the oracle, and the counters against the summed schedule counts."""
    graphs, queries, da, wants = batch512
    scales = [int(np.log2(g.n)) for g in graphs]
    bucket3 = [0 if sc <= 12 else (1 if sc <= 15 else 2) for sc in scales]
    tuned, untuned = bench_bucket_options()
    if which == "two-buckets-CB256":
        bopts = bucket_opts()
        bucket = [0 if g.n < 2**14 else 1 for g in graphs]
    else:
        bopts = {"tuned": tuned, "untuned": untuned,
                 "16-block": [dpo.Options(**{**o.__dict__, "agg_blocks": 16}) for o in tuned],
                 "grid": [dpo.Options(**{**o.__dict__, "agg": dpo.DPO_AGG_GRID}) for o in tuned],
                 "lane-serial": [dpo.Options(**{**o.__dict__, "serial_wave": 0}) for o in tuned],
                 }[which]
        bucket = bucket3 if len(bopts) == 3 else [0] * len(graphs)
    qs = [(g, s, bucket[g]) for g, s in queries]
    print("batch512", which, [o.label() for o in bopts], flush=True)
    host, slot0, st = run_batch("bfs", da, qs, bopts, stats=True)
    want_counts = {}
    for i, (g, s, b) in enumerate(qs):
        assert np.array_equal(host[slot0[i]:slot0[i] + graphs[g].n], wants[i]), (which, i)
        c = oracle.schedule_counts(graphs[g], wants[i], bopts[b].threshold, bopts[0].child_block,
                                   bopts[b].coarsen)
        for k, v in c.items():
            want_counts[k] = want_counts.get(k, 0) + v
    assert {k: st[k] for k in want_counts} == want_counts, which


@pytest.mark.slow
def test_batch_512_queries_sssp_tuned_options(batch512):
    """SSSP over the batched workload's graphs (weighted) at the tuned bucket
    options: every query against the oracle."""
    graphs, queries, _, _ = batch512
    wg = [gg.add_weights(g, 700 + i) for i, g in enumerate(graphs)]
    arena, vbase = gg.pack_arena(wg)
    da = dpo.DeviceArena(arena, vbase)
    scales = [int(np.log2(g.n)) for g in wg]
    bucket = [0 if sc <= 12 else (1 if sc <= 15 else 2) for sc in scales]
    tuned, _ = bench_bucket_options()
    qs = [(g, s, bucket[g]) for g, s in queries[::2]]
    host, slot0, _ = run_batch("sssp", da, qs, tuned)
    host = host.view(np.uint32)
    for i, (g, s, _) in enumerate(qs):
        want = oracle.dijkstra(wg[g], s)
        assert np.array_equal(host[slot0[i]:slot0[i] + wg[g].n], want), i

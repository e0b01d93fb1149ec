"""GPU parity of the continuous-batching engine: queries admitted while
others run, a footprint pool small enough that admission waits, and every
result bit-identical to the oracle and to the same query run alone."""
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
def resident():
    graphs = [gg.add_weights(gg.rmat(s, 16, 3000 + i, perm_seed=9000 + i), 500 + i)
              for i, s in enumerate([9, 10, 11, 12, 13, 13])]
    graphs.append(gg.add_weights(gg.path_graph(300), 7))  # 300 levels from an end
    arena, vbase = gg.pack_arena(graphs)
    return graphs, dpo.DeviceArena(arena, vbase)




@pytest.mark.parametrize("kind", ["bfs", "sssp"])
@pytest.mark.parametrize("agg,steps,split_min,dyn,hint", [(dpo.DPO_AGG_MULTIBLOCK, 2, 65536, 0, 0),
                                                          (dpo.DPO_AGG_BLOCK, 5, 65536, 0, 0),
                                                          (dpo.DPO_AGG_NONE, 3, 65536, 0, 0),
                                                          (dpo.DPO_AGG_MULTIBLOCK, 3, 0, 0, 0),
                                                          (dpo.DPO_AGG_MULTIBLOCK, 2, 300, 0, 0),
                                                          (dpo.DPO_AGG_MULTIBLOCK, 3, 65536, 25, 0),
                                                          (dpo.DPO_AGG_MULTIBLOCK, 2, 1024, 0,
                                                           dpo.DPO_HINT_OFF)])
def test_engine_results_match_oracle_and_lone_runs(resident, kind, agg, steps, split_min, dyn, hint):
    graphs, da = resident
    rng = np.random.default_rng(11)
    reqs = []
    for _ in range(48):
        g = int(rng.integers(0, len(graphs)))
        reqs.append((g, int(gg.sample_sources(graphs[g], 1, int(rng.integers(1 << 30)))[0])))
    bopts = [dpo.Options(threshold=16, coarsen=2, agg=agg, steps_per_replay=steps,
                         split_min=split_min, dyn_share=dyn, claim_hint=hint),
             dpo.Options(threshold=64, coarsen=1, agg=agg, steps_per_replay=steps,
                         split_min=split_min, dyn_share=dyn, claim_hint=hint)]
    gb = [0 if g.n < 2048 else 1 for g in graphs]
    # pool of 12k slots: at most a few graphs at once, so admission waits on footprint
    eng = dpo.Engine(da, kind, bopts, graph_bucket=gb, max_queries=8, max_slots=12 * 1024)
    got_tickets = set()
    outs = {}
    pending = list(reqs)
    import time
    t_end = time.time() + 60
    while time.time() < t_end:
        for g, s in pending[:3]:
            o = torch.full((graphs[g].n,), -9, dtype=torch.int32, device="cuda")
            outs[eng.submit(g, s, o)] = (g, s, o)
        pending = pending[3:]
        run, pend = eng.step()
        got_tickets.update(eng.poll())
        if not pending and run == 0 and pend == 0:
            break
    got_tickets.update(eng.poll())
    eng.close()
    torch.cuda.synchronize()
    assert got_tickets == set(outs), "every submitted query completes"
    for t, (g, s, o) in outs.items():
        if kind == "bfs":
            want, _ = oracle.bfs(graphs[g], s)
            assert np.array_equal(o.cpu().numpy(), want), (t, g, s)
        else:
            want = oracle.dijkstra(graphs[g], s)
            assert np.array_equal(dpo.as_uint32(o), want), (t, g, s)
    # alone vs in the mix: the first few queries run on their own
    for t in list(outs)[:4]:
        g, s, o = outs[t]
        dg = dpo.DeviceGraph.from_host(graphs[g])
        lone, _ = (dpo.bfs if kind == "bfs" else dpo.sssp)(dg, s, bopts[gb[g]])
        assert np.array_equal(lone.cpu().numpy(), o.cpu().numpy())


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_engine_on_a_dirty_workspace(resident, kind):
    """An engine built on a workspace full of stale bytes: its arena has slots
    that no query has been admitted to, which the kernels must never take for
    found or queued vertices (every level wide, so every BFS level ends in the
    harvest).  Every result equals the oracle."""
    graphs, da = resident
    bopts = [dpo.Options(threshold=16, coarsen=1, steps_per_replay=3, split_min=0)]
    probe = dpo.Engine(da, kind, bopts, max_queries=4, max_slots=12 * 1024)
    nbytes = probe.ws.numel()
    probe.close()
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    eng = dpo.Engine(da, kind, bopts, max_queries=4, max_slots=12 * 1024, workspace=ws)
    outs = {}
    for g in (0, 2, 4, 1, 3):  # the footprint pool holds a few graphs at once
        s = int(gg.sample_sources(graphs[g], 1, 77 + g)[0])
        o = torch.full((graphs[g].n,), -9, dtype=torch.int32, device="cuda")
        outs[eng.submit(g, s, o)] = (g, s, o)
    done = set()
    for _ in range(2000):
        run, pend = eng.step()
        done.update(eng.poll())
        if run == 0 and pend == 0:
            break
    done.update(eng.poll())
    eng.close()
    torch.cuda.synchronize()
    assert done == set(outs)
    for t, (g, s, o) in outs.items():
        if kind == "bfs":
            want, _ = oracle.bfs(graphs[g], s)
            assert np.array_equal(o.cpu().numpy(), want), (t, g, s)
        else:
            assert np.array_equal(dpo.as_uint32(o), oracle.dijkstra(graphs[g], s)), (t, g, s)


def test_engine_rejects_oversized_and_bad_queries(resident):
    graphs, da = resident
    eng = dpo.Engine(da, "bfs", [dpo.Options()], max_queries=4, max_slots=1024)
    o = torch.empty(graphs[3].n, dtype=torch.int32, device="cuda")
    with pytest.raises(dpo.DpoError) as e:
        eng.submit(3, 0, o)  # 2048 vertices never fit in 1024 slots
    assert e.value.status == dpo.DPO_ERR_CAPACITY
    with pytest.raises(dpo.DpoError) as e:
        eng.submit(0, graphs[0].n, o)
    assert e.value.status == dpo.DPO_ERR_SOURCE
    eng.close()


def _serving_opts(which):
    if which == "bench":
        # the serving benchmark's engines: 128-lane child blocks, a threshold
        # per kind
        import bench
        return {k: [dpo.Options(threshold=bench.SERVE_T[k], coarsen=1, agg=dpo.DPO_AGG_MULTIBLOCK,
                                agg_blocks=4, steps_per_replay=4, child_block=128,
                                dyn_share=bench.SERVE_DYN[k])]
                for k in ("bfs", "sssp")}
    o = [dpo.Options(threshold=32, coarsen=1, steps_per_replay=4)]
    return {"bfs": o, "sssp": o}


@pytest.mark.slow
@pytest.mark.parametrize("which", ["T32-CB256", "bench"])
def test_engines_at_the_serving_shape(which):
    """The serving workload's shape: 8 resident weighted R-MAT graphs (scales
    14..20 and a second 20), a BFS engine and an SSSP engine on two streams
    stepping together, queries arriving in waves while others run.  Every
    result equals the same query run alone; a sample also equals the oracle."""
    graphs = [gg.add_weights(gg.rmat(sc, 16, 3000 + i, perm_seed=9000 + i), 5000 + i)
              for i, sc in enumerate([14, 15, 16, 17, 18, 19, 20, 20])]
    arena, vbase = gg.pack_arena(graphs)
    da = dpo.DeviceArena(arena, vbase)
    kopts = _serving_opts(which)
    streams = {k: torch.cuda.Stream() for k in ("bfs", "sssp")}
    engines = {k: dpo.Engine(da, k, kopts[k], max_queries=64, max_slots=1 << 23,
                             stream=streams[k])
               for k in ("bfs", "sssp")}
    rng = np.random.default_rng(21)
    reqs = []
    for _ in range(72):
        kind = "bfs" if rng.random() < 0.7 else "sssp"
        g = int(rng.integers(0, len(graphs)))
        reqs.append((kind, g, int(gg.sample_sources(graphs[g], 1, int(rng.integers(1 << 30)))[0])))
    outs, done = {}, set()
    pending = list(reqs)
    import time
    t_end = time.time() + 120
    while time.time() < t_end:
        for kind, g, s in pending[:6]:
            o = torch.full((graphs[g].n,), -9, dtype=torch.int32, device="cuda")
            outs[(kind, engines[kind].submit(g, s, o))] = (kind, g, s, o)
        pending = pending[6:]
        busy = 0
        for kind, e in engines.items():
            run, pend = e.step()
            busy += run + pend
            done.update((kind, t) for t in e.poll())
        if not pending and busy == 0:
            break
    for kind, e in engines.items():
        done.update((kind, t) for t in e.poll())
        e.close()
    torch.cuda.synchronize()
    assert done == set(outs), "every submitted query completes"
    dgs = {}
    for i, (key, (kind, g, s, o)) in enumerate(outs.items()):
        dg = dgs.setdefault(g, dpo.DeviceGraph.from_host(graphs[g]))
        lone, _ = (dpo.bfs if kind == "bfs" else dpo.sssp)(dg, s, kopts[kind][0])
        assert np.array_equal(lone.cpu().numpy(), o.cpu().numpy()), (kind, g, s)
        if i % 9 == 0:
            want = oracle.bfs(graphs[g], s)[0] if kind == "bfs" else oracle.dijkstra(graphs[g], s)
            got = o.cpu().numpy() if kind == "bfs" else dpo.as_uint32(o)
            assert np.array_equal(got, want), (kind, g, s)

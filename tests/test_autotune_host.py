"""The tuner's search logic on the host, with batch timings replaced by a
known cost function (no GPU): the threshold heuristic, the greedy (T, CF)
walk per bucket, and the granularity stage over the whole launch."""
from paper_2201_02789_amd import autotune, dpo
from paper_2201_02789_amd import graphgen as gg


def test_heuristic_threshold_targets_the_launch_band():
    # 70 stars of 100 leaves: T <= 1 launches from all 7,070 vertices (inside
    # the 6,000-8,000 band), T in 8..64 from the 70 hubs only, T >= 128 from none
    graphs = [gg.star_graph(101) for _ in range(70)]
    queries = [(g, 0) for g in range(70)]
    assert autotune.heuristic_threshold(graphs, queries) == 0
    # 7,000 hubs of degree 40 and their leaves: T = 8 and T = 32 both keep
    # exactly the hubs (7,000 launches); the smaller threshold wins the tie
    graphs = [gg.star_graph(41) for _ in range(7000)]
    queries = [(g, 0) for g in range(7000)]
    assert autotune.heuristic_threshold(graphs, queries) == 8


def test_greedy_walk_and_granularity_stage(monkeypatch):
    graphs = [gg.path_graph(50), gg.star_graph(300)]
    queries = [(0, 0), (1, 0), (1, 5)]
    calls = []

    # cost: minimum at T = 128, CF = 2 for bucket 0's queries; granularity
    # 16-block fastest for the whole launch
    def fake_time(kind, arena, qs, opts, reps=2):
        bopts = opts if isinstance(opts, (list, tuple)) else [opts]
        o = bopts[0]
        calls.append((len(qs), o.label()))
        cost = abs(autotune.T_GRID.index(o.threshold) - 3) + abs(autotune.CF_GRID.index(o.coarsen) - 1)
        gran = {dpo.DPO_AGG_BLOCK: 3, dpo.DPO_AGG_GRID: 2}.get(o.agg, 1 if o.agg_blocks == 16 else 1.5)
        cb = {64: -0.25, 128: 0.0, 256: 0.5}[o.child_block]
        return cost + gran + cb

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    base = dpo.Options(threshold=32, coarsen=1, child_block=128)
    opts, traces, gtrace = autotune.tune("bfs", None, graphs, queries, [0, 0], 1, base, max_runs=20)
    assert (opts[0].threshold, opts[0].coarsen) == (128, 2)
    assert (opts[0].agg, opts[0].agg_blocks) == (dpo.DPO_AGG_MULTIBLOCK, 16)
    # the child block stage runs at the fastest granularity and keeps the fastest size
    assert opts[0].child_block == 64
    assert [n for n, _ in gtrace][:6] == ["block", "4-block", "16-block", "grid", "16-block-CB64",
                                          "16-block-CB256"]
    assert gtrace[6][0] == "tuned" and gtrace[7][0] == "bucket0-base"
    assert len(traces) == 1 and len(traces[0]) <= 20
    # a bucket without queries keeps the base point
    opts2, traces2, _ = autotune.tune("bfs", None, graphs, queries, [0, 0], 2, base, max_runs=4)
    assert traces2[1] == [] and opts2[1].threshold == base.threshold


def test_check_stage_reverts_a_bucket_that_loses_on_the_whole_batch(monkeypatch):
    """Stage 3: a bucket whose stage-1 point is slower on the whole batch than
    the base point goes back to the base point; one that is faster keeps it."""
    calls = []

    def fake_time(kind, arena, qs, opts, reps=2):
        bopts = opts if isinstance(opts, (list, tuple)) else [opts]
        calls.append([o.threshold for o in bopts])
        # bucket 0 at T=128 costs more than at the base T=32; bucket 1 at 128 less
        return sum({(0, 128): 3.0, (0, 32): 1.0, (1, 128): 1.0, (1, 32): 2.0}[(b, o.threshold)]
                   for b, o in enumerate(bopts))

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    base = dpo.Options(threshold=32, coarsen=1)
    tuned = [dpo.Options(threshold=128, coarsen=1), dpo.Options(threshold=128, coarsen=1)]
    out, trace = autotune.check_against_base("bfs", None, [(0, 0, 0), (1, 0, 1)], tuned, base)
    assert [o.threshold for o in out] == [32, 128]
    assert [n for n, _ in trace] == ["tuned", "bucket0-base", "bucket1-base"]

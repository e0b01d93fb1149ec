"""The timed instantiations of the level kernels (dpo_traverse_timed, the
execution-time breakdown of Sec. VIII-B): same results as the product
kernels, and timing rows that are well formed."""
import numpy as np
import pytest

import oracle
from paper_2201_02789_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_02789_amd import dpo  # noqa: E402

import bench  # noqa: E402


@pytest.fixture(scope="module")
def s16():
    g = gg.add_weights(gg.rmat(16, 16, 16, perm_seed=24), 31)
    return g, dpo.DeviceGraph.from_host(g)


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
@pytest.mark.parametrize("opts", [dpo.Options(threshold=64, coarsen=1, child_block=128),
                                  dpo.Options(threshold=0, coarsen=4),
                                  dpo.Options(threshold=16, coarsen=2, agg=dpo.DPO_AGG_WAVE),
                                  dpo.Options(threshold=16, coarsen=1, agg=dpo.DPO_AGG_BLOCK),
                                  dpo.Options.naive(), dpo.Options.flat(),
                                  dpo.Options(threshold=512, coarsen=1, child_block=128,
                                              split_min=262144),
                                  dpo.Options(threshold=64, coarsen=1, child_block=128, split_min=1024),
                                  dpo.Options(threshold=64, coarsen=1, child_block=128, split_min=1024,
                                              claim_hint=dpo.DPO_HINT_OFF)],
                         ids=lambda o: o.label())
def test_timed_traversal_matches_and_rows_are_well_formed(s16, kind, opts):
    g, dg = s16
    src = gg.max_degree_vertex(g)
    want = oracle.bfs(g, src)[0] if kind == "bfs" else oracle.dijkstra(g, src)
    out = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
    ws = dpo.alloc_workspace(dg, opts)
    timing = torch.full((dpo.TIMING_BYTES // 8,), 7, dtype=torch.int64, device="cuda")
    print("timed", kind, opts.label(), flush=True)
    dpo.dpo_traverse_timed(kind, dg, src, opts, out, ws, timing)
    torch.cuda.synchronize()
    got = out.cpu().numpy() if kind == "bfs" else dpo.as_uint32(out)
    assert np.array_equal(got, want), (kind, opts.label())
    rows = timing.cpu().numpy().view(np.uint64).reshape(64, 4, 4096, 8)
    ran = rows[:, :, :, 1] != 0
    levels = int(want.max()) + 1 if kind == "bfs" else None
    # every level with a frontier ran its parent kernel; rows only where kernels ran
    par_levels = np.flatnonzero(ran[:, 0].any(axis=1))
    if levels is not None:
        assert par_levels.tolist() == list(range(levels)), par_levels
    r = rows[ran]
    assert np.all(r[:, 0] <= r[:, 1])
    assert np.all(r[:, 7] <= r[:, 2:7].sum(axis=1))
    child = rows[:, 1][ran[:, 1]]
    parent = rows[:, 0][ran[:, 0]]
    # the child kernel has no parent or aggregation phase; the parent kernel
    # no disaggregation or child phase
    assert np.all(child[:, 2:4] == 0) and np.all(parent[:, 5:7] == 0)
    if opts.mode == dpo.DPO_MODE_FLAT:
        assert not ran[:, 1].any() and np.all(parent[:, 3:5] == 0)
    else:
        assert ran[:, 1].any() and child[:, 6].sum() > 0
    tot, per_level, imb = bench.phase_split(rows)
    assert all(v >= 0 for v in tot.values()) and imb >= 1.0
    # the same traversal with the product kernels afterwards: identical
    out2 = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
    (dpo.dpo_bfs if kind == "bfs" else dpo.dpo_sssp)(dg, src, opts, out2, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)

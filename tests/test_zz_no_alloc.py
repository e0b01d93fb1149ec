"""The no-allocation entry point (dpo_bfs_noalloc, workspace in the library's
static device array) against dpo_bfs with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller graph, so whatever the first
left in the shared array must not leak into the second; then a larger one
again and the library's other option families."""
import numpy as np
import pytest

import oracle
from paper_2201_02789_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_02789_amd import dpo  # noqa: E402


def _with_workspace(dg, src, opts):
    levels = torch.full((dg.n,), -5, dtype=torch.int32, device="cuda")
    dpo.dpo_bfs(dg, src, opts, levels, dpo.alloc_workspace(dg, opts))
    torch.cuda.synchronize()
    return levels.cpu().numpy()


def _noalloc(dg, src, opts):
    levels = torch.full((dg.n,), -5, dtype=torch.int32, device="cuda")
    dpo.dpo_bfs_noalloc(dg, src, opts, levels)
    torch.cuda.synchronize()
    return levels.cpu().numpy()


@pytest.mark.parametrize("opts", [dpo.Options(), dpo.Options(threshold=64, coarsen=1, child_block=128),
                                  dpo.Options.naive(), dpo.Options.flat(),
                                  dpo.Options(threshold=8, coarsen=2, agg=dpo.DPO_AGG_WAVE,
                                              split_min=0, steps_per_replay=3),
                                  dpo.Options(threshold=64, coarsen=1, child_block=128, split_min=1024),
                                  dpo.Options(threshold=64, coarsen=1, child_block=128, split_min=1024,
                                              claim_hint=dpo.DPO_HINT_OFF)],
                         ids=lambda o: o.label())
def test_noalloc_matches_workspace_call_then_smaller_input(opts):
    big = gg.rmat(16, 16, 16, perm_seed=24)      # 65,536 vertices
    small = gg.rmat(10, 8, 3, perm_seed=5)       # 1,024 vertices
    for g, src in ((big, gg.max_degree_vertex(big)), (small, int(gg.sample_sources(small, 1, 2)[0])),
                   (big, int(gg.sample_sources(big, 1, 9)[0]))):
        dg = dpo.DeviceGraph.from_host(g)
        print("noalloc", opts.label(), g.n, src, flush=True)
        want = _with_workspace(dg, src, opts)
        got = _noalloc(dg, src, opts)
        assert np.array_equal(got, want), (opts.label(), g.n, src)
        assert np.array_equal(got, oracle.bfs(g, src)[0]), (opts.label(), g.n, src)


def test_noalloc_rejects_graphs_beyond_the_static_workspace():
    n = 1_000_000  # its workspace exceeds 64 MiB at the default options
    g = gg.Graph(row_ptr=np.zeros(n + 1, dtype=np.int32), col_idx=np.zeros(0, dtype=np.int32))
    dg = dpo.DeviceGraph.from_host(g)
    levels = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(dpo.DpoError) as e:
        dpo.dpo_bfs_noalloc(dg, 0, dpo.Options(), levels)
    assert e.value.status == dpo.DPO_ERR_WORKSPACE

"""Grid-build code paths chosen by input layout and size (Section IV-A: the
grid is rebuilt from the positions every step), each checked exactly against
the oracle's grid of the same inputs.

* Inputs that are not 16-byte aligned (views starting one element in) take
  the bounds pass's element-wise loads instead of its 16-byte loads.
* A single simulation above 1,024 bounds partials (more than 4,194,304
  agents) reduces them in a launch of its own before the histogram; at
  exactly 1,024 partials the histogram blocks still reduce them themselves.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import workloads
from helpers import NP_IN, expect_grid, oracle_inputs

pytestmark = pytest.mark.gpu

CHUNK = 4096            # agents per bounds partial
SPLIT = 1024 * CHUNK    # largest build whose histogram blocks reduce the partials


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


def check_grid(ws, arrs, mode):
    g = ms.grid_get(ws)
    o = oracle_inputs(arrs, mode)
    origin, edge, dims, nb = oracle.geometry(*o)
    box, start, perm = oracle.grid(*o)
    info = g["info"][0]
    assert info["edge"] == edge
    assert tuple(info["dims"]) == tuple(int(v) for v in dims)
    assert np.array_equal(np.array(info["origin"]), origin)
    expect_grid(g, box, start, perm, dims, nb)


@pytest.mark.parametrize("mode", ["f32", "f64", "f32_pos64"])
def test_unaligned_inputs(mode):
    """20,001 agents (four whole bounds chunks and a ragged one) from views one
    element into their buffers, so no input is 16-byte aligned; the grid
    equals the oracle's and the aligned build's."""
    arrs = workloads.uniform(20001, mean_neighbors=12.0, seed=21).arrays()
    n = len(arrs[0])
    bufs = [torch.zeros(n + 1, dtype=getattr(torch, np.dtype(NP_IN[mode]).name), device="cuda")
            for _ in range(4)]
    views = []
    for b, a in zip(bufs, arrs):
        b[1:] = torch.from_numpy(np.asarray(a).astype(NP_IN[mode])).cuda()
        views.append(b[1:])
    assert all(v.data_ptr() % 16 != 0 for v in views)
    ws = ms.Workspace(n, dtype=mode)
    ms.grid_build(ws, *views)
    ms.device_status(ws)
    check_grid(ws, arrs, mode)
    aligned = [v.clone() for v in views]
    assert all(v.data_ptr() % 16 == 0 for v in aligned)
    g1 = ms.grid_get(ws)
    ms.grid_build(ws, *aligned)
    g2 = ms.grid_get(ws)
    for k in ("box_id", "start", "perm"):
        assert torch.equal(g1[k], g2[k])


@pytest.mark.parametrize("mode,n", [("f32", SPLIT), ("f64", SPLIT + CHUNK + 1)])
def test_geometry_reduction_paths(mode, n):
    """At exactly 1,024 partials (histogram blocks reduce them) and just above
    (one block reduces them first): geometry, box ids, starts and order equal
    the oracle's."""
    arrs = workloads.uniform(n, mean_neighbors=12.0, seed=22).arrays()
    ws = ms.Workspace(n, dtype=mode)
    t = [torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(NP_IN[mode]))).cuda() for a in arrs]
    print(f"[build paths] {mode} n={n}", flush=True)
    ms.grid_build(ws, *t)
    ms.device_status(ws)
    check_grid(ws, arrs, mode)

"""GPU parity at the benchmark's size at its other two densities: 2,097,152
uniform agents at ~4 and ~30 neighbours, FP32 and FP64, with the contact-list
length the benchmark's autotuner picks on the workload.  Grid (box of every
agent, box starts, canonical order) bit-exact; displacements of 4,096 sampled
agents -- random ones and members of the densest boxes -- within tau*S + A of
the oracle (oracle.sample builds the grid over every agent and sums forces for
the sample only)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import autotune, workloads
from helpers import NP_IN, UNIT, check_vectors, force_bound, expect_grid, oracle_inputs

pytestmark = pytest.mark.gpu

P = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("nbrs", [4.0, 30.0])
def test_full_size_uniform_2M_density(nbrs, mode):
    pop = workloads.uniform(workloads.FULL_N, mean_neighbors=nbrs, seed=0)
    arrs = pop.arrays()
    n = pop.n
    t = [torch.from_numpy(np.ascontiguousarray(a.astype(NP_IN[mode]))).cuda() for a in arrs]
    ws = ms.Workspace(n, dtype=mode)
    ms.grid_build(ws, *t)
    out = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    tuning = autotune.tune(ws, lambda: ms.mech_step(ws, P, out=out))
    D = ms.mech_step(ws, P)
    ms.device_status(ws)
    g = ms.grid_get(ws)
    o = oracle_inputs(arrs, mode)
    _, _, dims, nb = oracle.geometry(*o)
    box, start, perm = oracle.grid(*o)
    expect_grid(g, box, start, perm, dims, nb)
    rng = np.random.default_rng(int(nbrs))
    cnt = np.diff(start.astype(np.int64))
    dense = np.argsort(cnt, kind="stable")[-64:]
    members = np.concatenate([perm[start[b]:start[b + 1]] for b in dense]).astype(np.int64)
    idx = np.concatenate([rng.choice(n, 3072, replace=False),
                          rng.choice(members, min(1024, members.size), replace=False)])
    _, Do, S, A, C = oracle.sample(*o, P, idx, UNIT[mode])
    Dg = np.stack([a.cpu().numpy().astype(np.float64) for a in D], axis=1)[idx]
    bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
    worst = check_vectors(Dg, Do, bound, f"2M n{nbrs:g} {mode}")
    assert C.max() > 0
    print(f"2M n{nbrs:g} {mode}: list {tuning['choice']}, densest box {cnt.max()}, "
          f"sampled contacts up to {C.max()}, worst err/bound {worst:.3f}")

"""Batched step (many independent simulations in one grid build and one force
launch) against the oracle per simulation and against the plain single-
simulation path; HIP-graph replay of whole steps against eager execution."""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import workloads
from helpers import NP_IN, UNIT, check_vectors, force_bound, oracle_inputs

pytestmark = pytest.mark.gpu

MODES = ["f64", "f32", "f32_pos64"]
BASE = dict(dt=0.01, max_disp=3.0, adherence=0.0)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


def small_batch(seed=7):
    """Uneven sizes (1 to ~3000 agents), one empty simulation, per-simulation
    densities and force coefficients."""
    b = workloads.batched(n_sims=14, log10_min=0.0, log10_max=3.5, seed=seed)
    sizes = np.diff(b.offsets)
    sizes = np.insert(sizes, 5, 0)                        # an empty simulation
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    kappa = np.insert(b.kappa, 5, 2.0)
    gamma = np.insert(b.gamma, 5, 1.0)
    return workloads.Batch(b.x, b.y, b.z, b.d, offsets, kappa, gamma)


def dev(arrs, mode):
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(NP_IN[mode]))).cuda() for a in arrs]


def sim_params(b):
    return [dict(kappa=float(b.kappa[s]), gamma=float(b.gamma[s]), **BASE) for s in range(b.n_sims)]


def build_batched(b, mode):
    ws = ms.Workspace(b.n, max_sims=b.n_sims, dtype=mode)
    t = dev(b.arrays(), mode)
    spec = ms.BatchSpec(b.offsets)
    ms.grid_build_batched(ws, *t, spec)
    return ws, t, spec


@pytest.mark.parametrize("mode", MODES)
def test_batched_grid_bit_exact(mode):
    b = small_batch()
    ws, _, _ = build_batched(b, mode)
    ms.device_status(ws)
    g = ms.grid_get(ws)
    box = g["box_id"].cpu().numpy()
    start = g["start"].cpu().numpy()
    perm = g["perm"].cpu().numpy()
    base = 0
    for s in range(b.n_sims):
        a0, a1 = int(b.offsets[s]), int(b.offsets[s + 1])
        info = g["info"][s]
        assert info["n_agents"] == a1 - a0
        assert info["box_base"] == base
        if a1 == a0:
            assert info["n_boxes"] == 0
            continue
        o = oracle_inputs([a[a0:a1] for a in b.arrays()], mode)
        origin, edge, dims, nb = oracle.geometry(*o)
        obox, ostart, operm = oracle.grid(*o)
        assert info["edge"] == edge and tuple(info["dims"]) == tuple(int(v) for v in dims)
        assert np.array_equal(np.array(info["origin"]), origin)
        assert np.array_equal(box[a0:a1], obox + base)
        assert np.array_equal(start[base:base + nb + 1], ostart + a0)
        assert np.array_equal(perm[a0:a1], operm + a0)
        base += nb
    assert start[-1] == b.n


@pytest.mark.parametrize("mode", MODES)
def test_batched_step_matches_oracle_and_singles(mode):
    b = small_batch()
    ws, t, spec = build_batched(b, mode)
    P = ms.params_tensor(sim_params(b), "cuda")
    D = ms.mech_step_batched(ws, P)
    ms.device_status(ws)
    Dg = np.stack([a.cpu().numpy().astype(np.float64) for a in D], axis=1)
    for s, prm in enumerate(sim_params(b)):
        a0, a1 = int(b.offsets[s]), int(b.offsets[s + 1])
        if a1 == a0:
            continue
        arrs = [a[a0:a1] for a in b.arrays()]
        o = oracle_inputs(arrs, mode)
        _, Do = oracle.step(*o, prm)
        S, A, _ = oracle.tolerance_scales(*o, prm["kappa"], prm["gamma"], UNIT[mode])
        bound = prm["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
        check_vectors(Dg[a0:a1], Do, bound, f"sim {s} {mode}")
        # the plain path on the same simulation gives the same bits
        w1 = ms.Workspace(a1 - a0, dtype=mode)
        ms.grid_build(w1, *dev(arrs, mode))
        D1 = ms.mech_step(w1, prm)
        for k in range(3):
            assert torch.equal(D1[k], D[k][a0:a1])


@pytest.mark.parametrize("mode", MODES)
def test_batched_backward_matches_singles(mode):
    b = small_batch(seed=11)
    ws, t, spec = build_batched(b, mode)
    P = ms.params_tensor(sim_params(b), "cuda")
    rng = np.random.default_rng(2)
    g = [torch.from_numpy(rng.normal(size=b.n)).to(ws.out_dtype).cuda() for _ in range(3)]
    gx, gy, gz, gd, gkg = ms.mech_step_backward_batched(ws, P, *g)
    ms.device_status(ws)
    rel = 1e-12 if mode == "f64" else 1e-5
    for s, prm in enumerate(sim_params(b)):
        a0, a1 = int(b.offsets[s]), int(b.offsets[s + 1])
        if a1 == a0:
            assert torch.all(gkg[s] == 0)
            continue
        arrs = [a[a0:a1] for a in b.arrays()]
        w1 = ms.Workspace(a1 - a0, dtype=mode)
        ms.grid_build(w1, *dev(arrs, mode))
        o1 = ms.mech_step_backward(w1, prm, *(a[a0:a1].contiguous() for a in g))
        for k, got in enumerate((gx, gy, gz, gd)):
            assert torch.equal(got[a0:a1], o1[k])
        want = o1[4].cpu().numpy()
        np.testing.assert_allclose(gkg[s].cpu().numpy(), want, rtol=rel, atol=rel * np.abs(want).max())


@pytest.mark.parametrize("mode", ["f32", "f32_pos64"])
def test_batched_graph_replay_matches_eager(mode):
    """A whole batched step (grid build, force, integration) captured once and
    replayed; each replay is compared with the eager step, with host
    synchronisation and unrelated eager work between replays."""
    b = small_batch(seed=5)
    P = ms.params_tensor(sim_params(b), "cuda")
    spec = ms.BatchSpec(b.offsets)
    steps = 6
    # eager reference trajectory
    ws_e = ms.Workspace(b.n, max_sims=b.n_sims, dtype=mode)
    te = dev(b.arrays(), mode)
    ref = []
    for _ in range(steps):
        ms.grid_build_batched(ws_e, *te, spec)
        D = ms.mech_step_batched(ws_e, P)
        ms.integrate(*te[:3], *D)
        ref.append([a.clone() for a in te[:3]])
    # captured step
    ws = ms.Workspace(b.n, max_sims=b.n_sims, dtype=mode)
    t = dev(b.arrays(), mode)
    out = tuple(torch.empty(b.n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):           # warm up outside the graph
        ms.grid_build_batched(ws, *dev(b.arrays(), mode), spec)
        ms.mech_step_batched(ws, P, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ms.grid_build_batched(ws, *t, spec)
        ms.mech_step_batched(ws, P, out=out)
        ms.integrate(*t[:3], *out)
    # capture does not execute; reset the state and replay
    for a, v in zip(t, dev(b.arrays(), mode)):
        a.copy_(v)
    junk = torch.zeros(1 << 20, device="cuda")
    for s in range(steps):
        graph.replay()
        torch.cuda.synchronize()
        junk.add_(1.0)                       # unrelated eager work between replays
        for k in range(3):
            assert torch.equal(t[k], ref[s][k]), (s, k)
    ms.device_status(ws)


def test_plain_graph_replay_matches_eager():
    pop = workloads.uniform(50_000, mean_neighbors=12.0, seed=9)
    prm = dict(kappa=2.0, gamma=1.0, **BASE)
    ws_e = ms.Workspace(pop.n, dtype="f32")
    te = dev(pop.arrays(), "f32")
    ref = []
    for _ in range(4):
        ms.grid_build(ws_e, *te)
        D = ms.mech_step(ws_e, prm)
        ms.integrate(*te[:3], *D)
        ref.append([a.clone() for a in te[:3]])
    ws = ms.Workspace(pop.n, dtype="f32")
    t = dev(pop.arrays(), "f32")
    out = tuple(torch.empty(pop.n, device="cuda") for _ in range(3))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ms.grid_build(ws, *dev(pop.arrays(), "f32"))
        ms.mech_step(ws, prm, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ms.grid_build(ws, *t)
        ms.mech_step(ws, prm, out=out)
        ms.integrate(*t[:3], *out)
    for a, v in zip(t, dev(pop.arrays(), "f32")):
        a.copy_(v)
    for s in range(4):
        graph.replay()
        torch.cuda.synchronize()
        for k in range(3):
            assert torch.equal(t[k], ref[s][k]), (s, k)


@pytest.mark.parametrize("mode", ["f32_pos64", "f64"])
def test_batched_dense_cluster_buckets(mode):
    """A batch whose middle simulation is one tight cluster in a box-rich
    domain: buckets of the shared sort above the 4096-agent LDS stage and
    boxes above 255 agents, next to ordinary uniform simulations.  Grid of
    every simulation bit-exact; displacements of the dense simulation and of
    sampled agents of the others within the parity bound."""
    r = np.random.default_rng(91)
    c = r.normal(0.0, 22.0, size=(19992, 3))
    corners = np.array([[sx, sy, sz] for sx in (-400.0, 400.0) for sy in (-400.0, 400.0)
                        for sz in (-400.0, 400.0)])
    dense = np.concatenate([c, corners])
    sims = [workloads.uniform(3000, mean_neighbors=12.0, seed=92).arrays(),
            (dense[:, 0], dense[:, 1], dense[:, 2], r.uniform(8, 12, 20000)),
            workloads.uniform(5000, mean_neighbors=30.0, seed=93).arrays()]
    sizes = [len(s[0]) for s in sims]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    arrs = [np.concatenate([s[k] for s in sims]) for k in range(4)]
    n = int(offsets[-1])
    ws = ms.Workspace(n, max_boxes=600_000, max_sims=3, dtype=mode)
    ms.grid_build_batched(ws, *dev(arrs, mode), ms.BatchSpec(offsets))
    prms = [dict(BASE, kappa=2.0, gamma=1.0)] * 3
    D = ms.mech_step_batched(ws, ms.params_tensor(prms, "cuda"))
    ms.device_status(ws)
    g = ms.grid_get(ws)
    box = g["box_id"].cpu().numpy()
    start = g["start"].cpu().numpy()
    perm = g["perm"].cpu().numpy()
    Dg = np.stack([a.cpu().numpy().astype(np.float64) for a in D], axis=1)
    base = 0
    for s in range(3):
        a0, a1 = int(offsets[s]), int(offsets[s + 1])
        o = oracle_inputs([a[a0:a1] for a in arrs], mode)
        obox, ostart, operm = oracle.grid(*o)
        nb = len(ostart) - 1
        assert np.array_equal(box[a0:a1], obox + base), s
        assert np.array_equal(start[base:base + nb + 1], ostart + a0), s
        assert np.array_equal(perm[a0:a1], operm + a0), s
        idx = np.arange(a1 - a0) if s == 1 else r.choice(a1 - a0, 200, replace=False)
        _, Do, S, A, _ = oracle.sample(*o, prms[s], idx, UNIT[mode])
        bound = BASE["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
        check_vectors(Dg[a0 + idx], Do, bound, f"dense batch sim {s}")
        base += nb

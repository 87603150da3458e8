"""Sorted-state rollouts through ms_reorder (the agent sorting of Section
IV-D, kept across steps).

* The reorder is a permutation into box order: box indices (from the oracle's
  grid) are non-decreasing along it, every element size moves exactly.
* The sorted state is a fixed point: rebuilding from reordered inputs gives
  the identity order.
* Parity of the step on the sorted state against the oracle (same bar as the
  plain parity tests); a rollout that reorders every step reaches, mapped back
  through the composed permutation, the positions of the plain rollout within
  the FP64 rounding of the force sums.
* Batched builds keep every simulation's agents inside its range.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import workloads
from helpers import NP_IN, UNIT, check_vectors, force_bound, expect_grid, oracle_inputs

pytestmark = pytest.mark.gpu

MODES = ["f64", "f32", "f32_pos64"]
P = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


def dev(arrs, mode):
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(NP_IN[mode]))).cuda() for a in arrs]


def population(name):
    if name == "uniform20000_n12":
        return workloads.uniform(20000, mean_neighbors=12.0, seed=11).arrays()
    return workloads.clusters(20000, n_clusters=4, side=400.0, seed=12).arrays()


def slot_order(ws, n):
    return ms.reorder(ws, torch.arange(n, dtype=torch.int32, device="cuda")).cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["uniform20000_n12", "clusters20000"])
def test_reorder_is_box_sorted_permutation(case, mode):
    arrs = population(case)
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    t = dev(arrs, mode)
    ms.grid_build(ws, *t)
    p = slot_order(ws, n).astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(n))
    box, start, _ = oracle.grid(*oracle_inputs(arrs, mode))
    assert np.all(np.diff(box[p]) >= 0)
    # the slots of box b are exactly [start[b], start[b+1])
    assert np.array_equal(box[p], np.repeat(np.arange(len(start) - 1), np.diff(start)))
    rng = np.random.default_rng(3)
    for dt in (torch.int8, torch.int16, torch.float32, torch.float64, torch.complex128):
        src = torch.from_numpy(rng.integers(-100, 100, n).astype(np.float64)).to("cuda", dt)
        out = ms.reorder(ws, src)
        assert torch.equal(out.cpu(), src.cpu()[torch.from_numpy(p)]), dt
    ms.device_status(ws)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["uniform20000_n12", "clusters20000"])
def test_sorted_state_fixed_point_and_parity(case, mode):
    arrs = population(case)
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    t = dev(arrs, mode)
    ms.grid_build(ws, *t)
    ts = [ms.reorder(ws, a) for a in t]
    ms.grid_build(ws, *ts)
    assert np.array_equal(slot_order(ws, n), np.arange(n))
    _check_grid(ws, [a.cpu().numpy() for a in ts], mode)
    D = ms.mech_step(ws, P)
    ms.device_status(ws)
    sorted_arrs = [a.cpu().numpy() for a in ts]
    o = oracle_inputs(sorted_arrs, mode)
    _, Do = oracle.step(*o, P)
    S, A, _ = oracle.tolerance_scales(*o, P["kappa"], P["gamma"], UNIT[mode])
    Dg = np.stack([a.cpu().numpy().astype(np.float64) for a in D], axis=1)
    bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
    check_vectors(Dg, Do, bound, f"sorted state {case} {mode}")


def _check_grid(ws, arrs, mode):
    """Geometry, box ids, box starts and the canonical order of the last build
    equal the oracle's grid of the same inputs."""
    g = ms.grid_get(ws)
    o = oracle_inputs(arrs, mode)
    origin, edge, dims, nb = oracle.geometry(*o)
    box, start, perm = oracle.grid(*o)
    info = g["info"][0]
    assert info["edge"] == edge
    assert tuple(info["dims"]) == tuple(int(v) for v in dims)
    assert np.array_equal(np.array(info["origin"]), origin)
    expect_grid(g, box, start, perm, dims, nb)


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_sorted_input_grid_2M(mode):
    """2,097,152 agents: the build from the random input order moves the
    payload through its partition, the build after a sorted-state step (the
    state one step of motion later, as in a rollout) reads it from the
    inputs; both grids equal the oracle's exactly."""
    arrs = workloads.uniform(workloads.FULL_N, mean_neighbors=12.0, seed=5).arrays()
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    t = dev(arrs, mode)
    ms.grid_build(ws, *t)
    _check_grid(ws, arrs, mode)
    so = ms.mech_step_integrate_sorted(ws, P, *t)
    ms.device_status(ws)
    moved = [a.cpu().numpy() for a in so]
    ms.grid_build(ws, *so)
    _check_grid(ws, moved, mode)
    # the mode of a build is only a question of speed: after another sorted
    # step, a build from the random order (payload read from the inputs)
    # still equals the oracle's grid
    ms.mech_step_integrate_sorted(ws, P, *so)
    ms.grid_build(ws, *t)
    _check_grid(ws, arrs, mode)


def test_sorted_rollout_matches_plain_rollout():
    """Five FP64 steps, reordering every step vs never: the same agents end at
    the same positions up to the rounding order of the force sums."""
    arrs = workloads.uniform(20000, mean_neighbors=12.0, seed=13).arrays()
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype="f64")
    out = tuple(torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
    plain = dev(arrs, "f64")
    for _ in range(5):
        ms.grid_build(ws, *plain)
        ms.mech_step(ws, P, out=out)
        ms.integrate(*plain[:3], *out)
    state = dev(arrs, "f64")
    ident = torch.arange(n, dtype=torch.int32, device="cuda")   # original index of each agent
    for _ in range(5):
        ms.grid_build(ws, *state)
        ms.mech_step(ws, P, out=out)
        ms.integrate(*state[:3], *out)
        state = [ms.reorder(ws, a) for a in state]
        ident = ms.reorder(ws, ident)
    ms.device_status(ws)
    back = torch.empty(n, dtype=torch.int64, device="cuda")
    back[ident.long()] = torch.arange(n, device="cuda")
    for a, b in zip(plain[:3], state[:3]):
        assert torch.abs(a - b[back]).max().item() <= 1e-9
    assert torch.equal(plain[3], state[3][back])


def test_reorder_batched_keeps_simulations():
    b = workloads.batched(n_sims=9, log10_min=1.0, log10_max=3.5, seed=5)
    ws = ms.Workspace(b.n, max_sims=b.n_sims, dtype="f32_pos64")
    t = dev(b.arrays(), "f32_pos64")
    ms.grid_build_batched(ws, *t, ms.BatchSpec(b.offsets))
    p = slot_order(ws, b.n)
    for s in range(b.n_sims):
        a0, a1 = int(b.offsets[s]), int(b.offsets[s + 1])
        assert np.array_equal(np.sort(p[a0:a1]), np.arange(a0, a1)), s


def test_reorder_errors():
    arrs = workloads.uniform(1000, mean_neighbors=12.0, seed=1).arrays()
    ws = ms.Workspace(1000, dtype="f32")
    with pytest.raises(ms.MechStepError):       # no build yet
        ms.reorder(ws, torch.zeros(1000, device="cuda"))
    t = dev(arrs, "f32")
    ms.grid_build(ws, *t)
    with pytest.raises(ValueError):
        ms.reorder(ws, torch.zeros(999, device="cuda"))
    buf = torch.zeros(2000, device="cuda")
    with pytest.raises(ms.MechStepError):       # overlapping source and destination
        ms.reorder(ws, buf[:1000], out=buf[500:1500])
    ms.device_status(ws)

"""The sorted-state rollout step (ms_mech_step_integrate_sorted and its
batched variant): the state after each step comes out in the build's slot
order.  A rollout that steps this way is the caller-order rollout
(ms_mech_step_integrate) with its agents renumbered, bit for bit, in every
precision mode; the displacements it returns are those of ms_mech_step in slot
order; attribute arrays follow with ms_reorder."""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import workloads
from helpers import NP_IN, UNIT, check_vectors, force_bound, oracle_inputs

pytestmark = pytest.mark.gpu

P = dict(kappa=2.0, gamma=1.0, dt=0.05, max_disp=0.02, adherence=0.0)   # some agents clamped


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


def dev(arrs, mode):
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(NP_IN[mode]))).cuda() for a in arrs]


def check_step(arrs_in, disp, mode, what):
    """Displacements of one step from the state arrs_in against the oracle."""
    o = oracle_inputs(arrs_in, mode)
    _, Do = oracle.step(*o, P)
    S, A, _ = oracle.tolerance_scales(*o, P["kappa"], P["gamma"], UNIT[mode])
    bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
    Dg = np.stack([a.cpu().numpy().astype(np.float64) for a in disp], axis=1)
    check_vectors(Dg, Do, bound, what)


@pytest.mark.parametrize("mode", ["f32", "f64", "f32_pos64"])
@pytest.mark.parametrize("case", ["uniform_n12", "clusters"])
def test_sorted_rollout(mode, case):
    """The first sorted step is the caller-order step renumbered, bit for
    bit; every later step matches the oracle on the state it starts from;
    the state is a renumbering of the agents (diameters carried exactly)."""
    pop = workloads.uniform(30011, mean_neighbors=12.0, seed=21) if case == "uniform_n12" else \
        workloads.clusters(20000, n_clusters=3, side=250.0, seed=22)
    n = pop.n
    # one caller-order step
    ref = dev(pop.arrays(), mode)
    ws0 = ms.Workspace(n, dtype=mode)
    ms.grid_build(ws0, *ref)
    ms.mech_step_integrate(ws0, P, *ref[:3])
    ms.device_status(ws0)
    # sorted rollout: ping-pong state buffers, ids carried with ms_reorder
    ws1 = ms.Workspace(n, dtype=mode)
    a = dev(pop.arrays(), mode)
    b = [torch.empty_like(v) for v in a]
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    disp = tuple(torch.empty(n, dtype=ws1.out_dtype, device="cuda") for _ in range(3))
    d0 = a[3].clone()
    for s in range(4):
        state_in = [v.cpu().numpy() for v in a]
        ms.grid_build(ws1, *a)
        ms.mech_step_integrate_sorted(ws1, P, *a, state_out=b, disp_out=disp)
        perm = ms.reorder(ws1, torch.arange(n, dtype=torch.int32, device="cuda")).long()
        if s == 0:
            # the displacements are ms_mech_step's, in slot order, and the
            # state is the caller-order step renumbered
            D = ms.mech_step(ws1, P)
            for dd, full in zip(disp, D):
                assert torch.equal(dd, full[perm])
            for k in range(3):
                assert torch.equal(b[k], ref[k][perm]), k
        ids = ms.reorder(ws1, ids)
        check_step([v[perm.cpu().numpy()] for v in state_in], disp, mode, f"sorted step {s}")
        a, b = b, a
    ms.device_status(ws1)
    idx = ids.long()
    assert torch.equal(torch.sort(idx).values, torch.arange(n, device="cuda"))
    assert torch.equal(a[3], d0[idx])
    # the sorted state is nearly sorted for the next build: its slot order
    # keeps almost every neighbouring pair in place
    ms.grid_build(ws1, *a)
    perm = ms.reorder(ws1, torch.arange(n, dtype=torch.int32, device="cuda")).cpu().numpy()
    assert np.mean(np.diff(perm) > 0) > 0.97


@pytest.mark.parametrize("mode", ["f32_pos64", "f32"])
def test_sorted_batched_rollout(mode):
    b = workloads.batched(n_sims=12, log10_min=3.0, log10_max=4.0, seed=23)
    prms = [dict(P, kappa=float(k), gamma=float(g)) for k, g in zip(b.kappa, b.gamma)]
    Pd = ms.params_tensor(prms, "cuda")
    spec = ms.BatchSpec(b.offsets)
    n = b.n
    ref = dev(b.arrays(), mode)
    ws0 = ms.Workspace(n, max_sims=b.n_sims, dtype=mode)
    ms.grid_build_batched(ws0, *ref, spec)
    ms.mech_step_batched_integrate(ws0, Pd, *ref[:3])
    ws1 = ms.Workspace(n, max_sims=b.n_sims, dtype=mode)
    a = dev(b.arrays(), mode)
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    d0 = a[3].clone()
    for s in range(3):
        state_in = [v.cpu().numpy() for v in a]
        ms.grid_build_batched(ws1, *a, spec)
        disp = tuple(torch.empty(n, dtype=ws1.out_dtype, device="cuda") for _ in range(3))
        out = list(ms.mech_step_batched_integrate_sorted(ws1, Pd, *a, disp_out=disp))
        perm = ms.reorder(ws1, torch.arange(n, dtype=torch.int32, device="cuda")).long()
        if s == 0:
            for k in range(3):
                assert torch.equal(out[k], ref[k][perm]), k
        p_np = perm.cpu().numpy()
        Dg = np.stack([v.cpu().numpy().astype(np.float64) for v in disp], axis=1)
        for q in range(b.n_sims):
            a0, a1 = int(b.offsets[q]), int(b.offsets[q + 1])
            o = oracle_inputs([v[p_np[a0:a1]] for v in state_in], mode)
            _, Do = oracle.step(*o, prms[q])
            S, A, _ = oracle.tolerance_scales(*o, prms[q]["kappa"], prms[q]["gamma"], UNIT[mode])
            bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
            check_vectors(Dg[a0:a1], Do, bound, f"batched sorted step {s} sim {q}")
        ids = ms.reorder(ws1, ids)
        a = out
    ms.device_status(ws0)
    ms.device_status(ws1)
    idx = ids.long()
    assert torch.equal(a[3], d0[idx])
    # every agent stays inside its simulation's range
    off = torch.from_numpy(b.offsets).cuda()
    sim_of_slot = torch.searchsorted(off, torch.arange(n, device="cuda"), right=True) - 1
    sim_of_agent = torch.searchsorted(off, idx, right=True) - 1
    assert torch.equal(sim_of_slot, sim_of_agent)


def test_sorted_step_matches_oracle_and_rejects_overlap():
    mode = "f64"
    arrs = workloads.uniform(5003, mean_neighbors=30.0, seed=24).arrays()
    t = dev(arrs, mode)
    ws = ms.Workspace(len(arrs[0]), dtype=mode)
    ms.grid_build(ws, *t)
    disp = tuple(torch.empty(len(arrs[0]), dtype=torch.float64, device="cuda") for _ in range(3))
    out = ms.mech_step_integrate_sorted(ws, P, *t, disp_out=disp)
    ids = ms.reorder(ws, torch.arange(len(arrs[0]), dtype=torch.int32, device="cuda")).long().cpu().numpy()
    o = oracle_inputs(arrs, mode)
    _, Do = oracle.step(*o, P)
    S, A, _ = oracle.tolerance_scales(*o, 2.0, 1.0, UNIT[mode])
    bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
    Dg = np.stack([a.cpu().numpy() for a in disp], axis=1)
    check_vectors(Dg, Do[ids], bound[ids], "sorted step")
    assert np.array_equal(out[3].cpu().numpy(), arrs[3][ids])
    with pytest.raises(ms.MechStepError):
        ms.mech_step_integrate_sorted(ws, P, *t, state_out=(t[0], out[1], out[2], out[3]))

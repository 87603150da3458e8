"""The fused rollout step (ms_mech_step_integrate and its batched form) is
bitwise the displacement step followed by ms_integrate, through the C ABI.
The separate calls are themselves checked against the oracle in
test_gpu_parity (displacements) and test_integrate_exact (the update)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2105_00039_amd as ms
from paper_2105_00039_amd import workloads
from helpers import NP_IN

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


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("with_out", [True, False])
def test_fused_step_equals_step_then_integrate(mode, with_out):
    arrs = workloads.uniform(30011, mean_neighbors=12.0, seed=21).arrays()
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    a = dev(arrs, mode)
    b = [t.clone() for t in a]
    for _ in range(3):   # three steps: the update feeds the next build
        ms.grid_build(ws, *a)
        D = ms.mech_step(ws, P)
        ms.integrate(*a[:3], *D)
        ms.grid_build(ws, *b)
        out = tuple(torch.full((n,), 7.0, dtype=ws.out_dtype, device="cuda") for _ in range(3)) \
            if with_out else None
        ms.mech_step_integrate(ws, P, *b[:3], out=out)
        if with_out:
            for u, v in zip(D, out):
                assert torch.equal(u, v)
        for u, v in zip(a[:3], b[:3]):
            assert torch.equal(u, v)
    ms.device_status(ws)


@pytest.mark.parametrize("mode", ["f32_pos64", "f64"])
def test_fused_batched_step_equals_step_then_integrate(mode):
    bt = workloads.batched(n_sims=12, log10_min=1.0, log10_max=3.5, seed=9)
    prms = [dict(P, kappa=float(k), gamma=float(g)) for k, g in zip(bt.kappa, bt.gamma)]
    Pd = ms.params_tensor(prms, "cuda")
    spec = ms.BatchSpec(bt.offsets)
    ws = ms.Workspace(bt.n, max_sims=bt.n_sims, dtype=mode)
    a = dev(bt.arrays(), mode)
    b = [t.clone() for t in a]
    for _ in range(2):
        ms.grid_build_batched(ws, *a, spec)
        D = ms.mech_step_batched(ws, Pd)
        ms.integrate(*a[:3], *D)
        ms.grid_build_batched(ws, *b, spec)
        out = tuple(torch.empty(bt.n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
        ms.mech_step_batched_integrate(ws, Pd, *b[:3], out=out)
        for u, v in zip(D, out):
            assert torch.equal(u, v)
        for u, v in zip(a[:3], b[:3]):
            assert torch.equal(u, v)
    ms.device_status(ws)


def test_fused_step_errors_and_failed_build():
    base = [np.array([0.0, 9.0, 20.0]), np.zeros(3), np.zeros(3), np.array([10.0, 10.0, 10.0])]
    ws = ms.Workspace(3, dtype="f32")
    t = dev(base, "f32")
    ms.grid_build(ws, *t)
    lib = ms._lib.load()
    p = ms._params(P)
    d = torch.empty(3, dtype=torch.float32, device="cuda")
    st = lib.ms_mech_step_integrate(ctypes.byref(ws.c), ctypes.byref(p), ctypes.c_void_p(t[0].data_ptr()),
                                    ctypes.c_void_p(t[1].data_ptr()), ctypes.c_void_p(t[2].data_ptr()),
                                    ctypes.c_void_p(d.data_ptr()), None, None, None)
    assert st == ms._lib.MS_EINVAL                       # dx given without dy, dz
    st = lib.ms_mech_step_integrate(ctypes.byref(ws.c), ctypes.byref(p), None, None, None, None,
                                    None, None, None)
    assert st == ms._lib.MS_EINVAL                       # positions are required
    # a build that fails on the device: the fused step moves nothing
    bad = [a.copy() for a in base]
    bad[0][1] = np.nan
    tb = dev(bad, "f32")
    ms.grid_build(ws, *tb)
    before = [a.clone() for a in tb]
    ms.mech_step_integrate(ws, P, *tb[:3])
    with pytest.raises(ms.MechStepError):
        ms.device_status(ws)
    for u, v in zip(before, tb):
        assert torch.equal(torch.nan_to_num(u, nan=-1.0), torch.nan_to_num(v, nan=-1.0))


@pytest.mark.parametrize("mode", ["f32", "f32_pos64"])
def test_fused_step_graph_replay_matches_eager(mode):
    """Build + fused step captured in a HIP graph (as the benchmark times it):
    every replay equals the eager trajectory bit for bit, with eager work and
    synchronisations between the replays."""
    arrs = workloads.uniform(40009, mean_neighbors=12.0, seed=23).arrays()
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    out = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))

    def one(ts):
        ms.grid_build(ws, *ts)
        ms.mech_step_integrate(ws, P, *ts[:3], out=out)

    te = dev(arrs, mode)
    ref = []
    for _ in range(3):
        one(te)
        ref.append([a.clone() for a in te[:3]] + [d.clone() for d in out])
    t = dev(arrs, mode)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        one(dev(arrs, mode))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        one(t)
    for a, v in zip(t, dev(arrs, mode)):
        a.copy_(v)
    for s in range(3):
        graph.replay()
        torch.cuda.synchronize()
        ms.device_status(ws)                     # eager work between replays
        got = [a for a in t[:3]] + list(out)
        for k in range(6):
            assert torch.equal(got[k], ref[s][k]), (s, k)

"""The step without allocation (ms_mech_step_noalloc) against ms_grid_build +
ms_mech_step on a caller workspace, through the C ABI.

Both run the same kernels, so the displacements must agree bit for bit; they
are also held to the oracle's acceptance bound (tau*S + A per agent).  Two
calls in a row, the second on a smaller population: the static workspace
keeps the first call's contents and must not leak them into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import _lib, workloads
from helpers import NP_IN, UNIT, check_vectors, force_bound, oracle_inputs

pytestmark = pytest.mark.gpu

P = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)
CODES = {"f32": _lib.MS_F32, "f64": _lib.MS_F64, "f32_pos64": _lib.MS_F32_POS64}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    _lib.load()


def _dev(arrs, mode):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=NP_IN[mode])).to("cuda") for a in arrs]


def _noalloc(arrs, mode):
    lib = _lib.load()
    n = len(arrs[0])
    t = _dev(arrs, mode)
    od = torch.float64 if mode == "f64" else torch.float32
    # poison the outputs: every element must be written
    out = [torch.full((n,), float("nan"), dtype=od, device="cuda") for _ in range(3)]
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    p = _lib.ms_params(*(P[k] for k in ("kappa", "gamma", "dt", "max_disp", "adherence")))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.ms_mech_step_noalloc(*(ctypes.c_void_p(a.data_ptr()) for a in t), n, CODES[mode], 0.0,
                                  ctypes.byref(p), *(ctypes.c_void_p(a.data_ptr()) for a in out),
                                  ctypes.c_void_p(err.data_ptr()), stream)
    _lib.check(st)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    return np.stack([a.cpu().numpy() for a in out], axis=1)


def _workspace(arrs, mode):
    n = len(arrs[0])
    t = _dev(arrs, mode)
    ws = ms.Workspace(n, dtype=mode)
    ms.grid_build(ws, *t)
    D = ms.mech_step(ws, P)
    ms.device_status(ws)
    return np.stack([a.cpu().numpy() for a in D], axis=1)


@pytest.mark.parametrize("mode", ["f32", "f64", "f32_pos64"])
def test_noalloc_equals_workspace_step(mode):
    first = workloads.uniform(60000, mean_neighbors=12.0, seed=11).arrays()
    second = workloads.uniform(5003, mean_neighbors=30.0, seed=12).arrays()
    for arrs in (first, second):
        got = _noalloc(arrs, mode)
        want = _workspace(arrs, mode)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), mode
        ao = oracle_inputs(arrs, mode)
        _, Do = oracle.step(*ao, P)
        S, A, _ = oracle.tolerance_scales(*ao, P["kappa"], P["gamma"], UNIT[mode])
        bound = P["dt"] * force_bound(S, A, mode) + 8 * UNIT[mode] * np.linalg.norm(Do, axis=1)
        check_vectors(got, Do, bound, f"noalloc {mode} n={len(arrs[0])}")


def test_noalloc_limits_and_device_error():
    lib = _lib.load()
    p = _lib.ms_params(2, 1, 0.01, 3, 0)
    nul = ctypes.c_void_p(0)
    st = lib.ms_mech_step_noalloc(nul, nul, nul, nul, _lib.NOALLOC_MAX_AGENTS + 1, _lib.MS_F32, 0.0,
                                  ctypes.byref(p), nul, nul, nul, nul, nul)
    assert st == _lib.MS_ECAPACITY
    # a sparse population needing more boxes than the static workspace holds
    # (about 834 x 84 x 84 boxes of edge 12 against 524,288):
    # reported through dev_error, not a fault
    n = 1000
    r = np.random.default_rng(5)
    arrs = (r.uniform(0, 1e4, n), r.uniform(0, 1e3, n), r.uniform(0, 1e3, n), r.uniform(8, 12, n))
    t = _dev(arrs, "f32")
    out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = lib.ms_mech_step_noalloc(*(ctypes.c_void_p(a.data_ptr()) for a in t), n, _lib.MS_F32, 0.0,
                                  ctypes.byref(p), *(ctypes.c_void_p(a.data_ptr()) for a in out),
                                  ctypes.c_void_p(err.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.MS_OK
    torch.cuda.synchronize()
    assert int(err.item()) & 8
    # and the next call on the same array is fine again
    arrs = workloads.lattice(seed=0).arrays()
    got = _noalloc(arrs, "f64")
    assert np.array_equal(got, _workspace(arrs, "f64"))

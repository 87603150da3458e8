"""The forward gather's launch shape (the autotuner's knobs: contact-list
length, block size and run walk) does not change any result: plain, fused,
sorted and batched steps and the backward are bitwise identical for every
allowed choice; the tuner picks an allowed (length, block, walk) triple,
caches it under its key (dict or JSON file) and reuses it; other values are
rejected through the C ABI.  The box-order tuner is checked here too."""
import json

import numpy as np
import pytest
import torch

import paper_2105_00039_amd as ms
from paper_2105_00039_amd import autotune, workloads
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


def population(name):
    if name == "uniform20000_n30":
        return workloads.uniform(20000, mean_neighbors=30.0, seed=41).arrays()
    return workloads.clusters(20000, n_clusters=3, side=250.0, seed=42).arrays()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["uniform20000_n30", "clusters20000_dense"])
def test_launch_shape_does_not_change_results(case, mode):
    arrs = population(case)
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype=mode)
    t = dev(arrs, mode)
    ms.grid_build(ws, *t)
    g = [torch.full((n,), 1e-3, dtype=ws.out_dtype, device="cuda") for _ in range(3)]
    res = {}
    for c in autotune.CHOICES:
        ws.gather_list, ws.gather_block, ws.gather_walk = c
        D = [a.clone() for a in ms.mech_step(ws, P)]
        G = [a.clone() for a in ms.mech_step_backward(ws, P, *g)[:4]]
        pos = [a.clone() for a in t[:3]]
        ms.mech_step_integrate(ws, P, *pos)
        so = [a.clone() for a in ms.mech_step_integrate_sorted(ws, P, *t)]
        res[c] = D + G + pos + so
    ms.device_status(ws)
    for c in autotune.CHOICES[1:]:
        for a, b in zip(res[autotune.CHOICES[0]], res[c]):
            assert torch.equal(a, b), c


def test_launch_shape_batched():
    b = workloads.batched(n_sims=10, log10_min=2.0, log10_max=3.7, seed=43)
    prms = [dict(P, kappa=float(k), gamma=float(gm)) for k, gm in zip(b.kappa, b.gamma)]
    Pd = ms.params_tensor(prms, "cuda")
    ws = ms.Workspace(b.n, max_sims=b.n_sims, dtype="f32_pos64")
    ms.grid_build_batched(ws, *dev(b.arrays(), "f32_pos64"), ms.BatchSpec(b.offsets))
    out = {}
    for c in autotune.CHOICES:
        ws.gather_list, ws.gather_block, ws.gather_walk = c
        out[c] = [a.clone() for a in ms.mech_step_batched(ws, Pd)]
    ms.device_status(ws)
    for c in autotune.CHOICES[1:]:
        for a, b in zip(out[autotune.CHOICES[0]], out[c]):
            assert torch.equal(a, b), c


def test_tuner_picks_caches_and_rejects(tmp_path):
    arrs = population("uniform20000_n30")
    n = len(arrs[0])
    ws = ms.Workspace(n, dtype="f32")
    ms.grid_build(ws, *dev(arrs, "f32"))
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))

    def step():
        ms.mech_step(ws, P, out=out)

    table = {}
    r = autotune.tune(ws, step, cache=table)
    assert r["source"] == "timed" and r["choice"] in autotune.CHOICES
    assert (ws.gather_list, ws.gather_block, ws.gather_walk) == r["choice"]
    assert tuple(table[r["key"]]) == r["choice"] and len(r["ms"]) == len(autotune.CHOICES)
    ws.gather_list, ws.gather_block, ws.gather_walk = 0, 0, "lanes"
    r2 = autotune.tune(ws, step, cache=table)
    assert r2["source"] == "cache"
    assert (ws.gather_list, ws.gather_block, ws.gather_walk) == r["choice"]
    path = tmp_path / "tune.json"
    r3 = autotune.tune(ws, step, key="custom", cache=path)
    assert r3["source"] == "timed" and tuple(json.loads(path.read_text())["custom"]) == r3["choice"]
    r4 = autotune.tune(ws, step, key="custom", cache=path)
    assert r4["source"] == "cache" and r4["choice"] == r3["choice"]
    ws.c.gather_walk = 2
    with pytest.raises(ms.MechStepError, match="gather_walk"):
        ms.mech_step(ws, P)
    with pytest.raises(ValueError):
        ws.gather_walk = "rows"
    ws.gather_walk = "lanes"
    ws.gather_list = 33
    with pytest.raises(ms.MechStepError) as ei:
        ms.mech_step(ws, P)
    assert ei.value.status == ms._lib.MS_EINVAL
    ws.gather_list, ws.gather_block = 0, 128
    with pytest.raises(ms.MechStepError) as ei:
        ms.mech_step(ws, P)
    assert ei.value.status == ms._lib.MS_EINVAL
    ws.gather_block = 0
    ms.mech_step(ws, P)
    ms.device_status(ws)


def test_box_order_tuner(tmp_path):
    """tune_box_order times row-major against tiled rows over build + step,
    keeps the automatic choice unless the other is faster, leaves a build in
    the chosen order, caches the pick, and never picks an order whose build
    fails; the displacements do not depend on the order."""
    arrs = workloads.uniform(40000, mean_neighbors=12.0, seed=44).arrays()
    n = len(arrs[0])
    t = dev(arrs, "f32")
    ref_ws = ms.Workspace(n, dtype="f32", box_order="rows")
    ms.grid_build(ref_ws, *t)
    ref = torch.stack(ms.mech_step(ref_ws, P)).cpu()
    ws = ms.Workspace(n, dtype="f32")
    out = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    step = lambda: (ms.grid_build(ws, *t), ms.mech_step(ws, P, out=out))
    cache = tmp_path / "order.json"
    r = autotune.tune_box_order(ws, step, cache=cache)
    assert r["source"] == "timed" and r["auto"] == "rows" and r["choice"] in ("rows", "tiles")
    assert set(r["ms"]) == {"rows", "tiles"}
    assert ws.box_order == r["choice"]
    assert ms.grid_info(ws)[0]["tile_shift"] == (4 if r["choice"] == "tiles" else 0)
    assert torch.equal(torch.stack(out).cpu(), ref)
    assert json.loads(cache.read_text())[r["key"]] == r["choice"]
    ws2 = ms.Workspace(n, dtype="f32")
    r2 = autotune.tune_box_order(ws2, lambda: (ms.grid_build(ws2, *t), ms.mech_step(ws2, P, out=out)),
                                 cache=cache)
    assert r2["source"] == "cache" and r2["choice"] == r["choice"] == ws2.box_order
    # tiles that do not fit the workspace are never picked
    small = ms.Workspace(n, dtype="f32", max_boxes=ms.grid_info(ref_ws)[0]["n_boxes"] + 1)
    step_s = lambda: (ms.grid_build(small, *t), ms.mech_step(small, P, out=out))
    r3 = autotune.tune_box_order(small, step_s)
    assert r3["choice"] == "rows" and set(r3["ms"]) == {"rows"}
    ms.device_status(small)
    with pytest.raises(ValueError):
        autotune.tune_box_order(ms.Workspace(n, max_sims=2, dtype="f32"), step)

"""GPU reverse-mode derivative (ms_mech_step_backward and the autograd layer)
against the oracle's adjoint, finite differences of the GPU FP64 forward, and
checkpoint-interval invariance.

Tolerances (the target sets none; derived from the arithmetic): configurations
keep every pair within the radius at |delta| > 1e-2 and away from the length
bound, where ds/ddelta is bounded.  One backward step is compared agent by
agent: |g_i - g_oracle_i| <= tau_g S_i + A_i with the oracle's per-agent
scales (oracle.adjoint_scales: the magnitudes of the adjoint terms of the
agent's contacts and an overlap-rounding allowance), tau_g = 1e-12 (FP64) and
1e-3 (FP32).  Rollout gradients add a per-agent scale summed over the steps.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2105_00039_amd as ms
from paper_2105_00039_amd import autograd as msa
from paper_2105_00039_amd import workloads
from helpers import NP_IN, TAU_G, UNIT, check_gradients, check_vectors, oracle_inputs

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ms._lib.load()


def smooth_pop(n, nbrs, seed, params, mode="f64", gap=1e-2, steps=1):
    """A population kept away from the kinks of the step map over a
    ``steps``-step oracle trajectory: every pair within the radius has
    |delta| > gap and every agent has ||v| - m| > 1e-3 m, in the precision the
    GPU path sees.  Agents of offending pairs are removed until none is left."""
    pop = workloads.uniform(n, mean_neighbors=nbrs, seed=seed)
    keep = np.ones(pop.n, dtype=bool)
    arrs0 = [np.asarray(a) for a in pop.arrays()]
    for _ in range(100):
        arrs = [a[keep] for a in arrs0]
        o = list(oracle_inputs(arrs, mode))
        bad = np.zeros(len(arrs[0]), dtype=bool)
        traj = oracle.rollout(*o, params, steps)
        for p in traj[:-1] if steps > 0 else traj:
            q = (p[:, 0], p[:, 1], p[:, 2], o[3])
            c, off, lst = oracle.neighbors(*q)
            i = np.repeat(np.arange(len(c)), c)
            l = np.sqrt((q[0][i] - q[0][lst]) ** 2 + (q[1][i] - q[1][lst]) ** 2 + (q[2][i] - q[2][lst]) ** 2)
            delta = q[3][i] / 2 + q[3][lst] / 2 - l
            near = np.abs(delta) < gap
            bad[np.minimum(i[near], lst[near])] = True
            F, _ = oracle.step(*q, params)
            v = params["dt"] * np.linalg.norm(F, axis=1)
            bad |= np.abs(v - params["max_disp"]) < 1e-3 * params["max_disp"]
        if not bad.any():
            return workloads.Population(*arrs)
        idx = np.nonzero(keep)[0]
        keep[idx[bad]] = False
    raise RuntimeError("no smooth population")


def dev(arrs, mode):
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(NP_IN[mode]))).cuda() for a in arrs]


@pytest.mark.parametrize("mode", ["f64", "f32", "f32_pos64"])
@pytest.mark.parametrize("clamp", [False, True])
def test_backward_matches_oracle_adjoint(mode, clamp):
    prm = dict(kappa=2.0, gamma=1.0, dt=0.05 if clamp else 0.01,
               max_disp=0.02 if clamp else 3.0, adherence=0.0)
    pop = smooth_pop(1500, 15.0, 10 if clamp else 30, prm, mode)
    arrs = pop.arrays()
    o = oracle_inputs(arrs, mode)
    rng = np.random.default_rng(5)
    g = rng.normal(size=(pop.n, 3))
    if mode != "f64":
        g = g.astype(np.float32).astype(np.float64)
    ws = ms.Workspace(pop.n, dtype=mode)
    t = dev(arrs, mode)
    ms.grid_build(ws, *t)
    gt = [torch.from_numpy(np.ascontiguousarray(g[:, k])).to(ws.out_dtype).cuda() for k in range(3)]
    gx, gy, gz, gd, gkg = ms.mech_step_backward(ws, prm, *gt)
    ms.device_status(ws)
    gp = np.stack([a.cpu().numpy().astype(np.float64) for a in (gx, gy, gz)], axis=1)
    worst = check_gradients(gp, gd.cpu().numpy(), gkg.cpu().numpy(), o, prm, g, mode,
                            f"backward {mode} clamp={clamp}")
    print(f"backward {mode} clamp={clamp}: worst err/bound {worst:.3g}")
    if clamp:
        F, _ = oracle.step(*o, prm)
        assert np.sum(prm["dt"] * np.linalg.norm(F, axis=1) > prm["max_disp"]) > 50
    # bitwise repeatable
    again = ms.mech_step_backward(ws, prm, *gt)
    for a, b in zip((gx, gy, gz, gd, gkg), again):
        assert torch.equal(a, b)


def test_single_step_autograd_f64():
    prm = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)
    pop = smooth_pop(500, 15.0, 50, prm)
    t = [a.requires_grad_(True) for a in dev(pop.arrays(), "f64")]
    kap = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    gam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    ws = ms.Workspace(pop.n, dtype="f64")
    rest = dict(dt=0.01, max_disp=3.0, adherence=0.0)
    D = msa.mech_step_fn(*t, kap, gam, ws, rest)
    w = torch.linspace(-1, 1, pop.n, dtype=torch.float64, device="cuda")
    L = (D[0] * w).sum() + (D[1] * w * w).sum() - D[2].sum()
    L.backward()
    g = np.stack([w.cpu().numpy(), (w * w).cpu().numpy(), -np.ones(pop.n)], axis=1)
    gp = np.stack([t[k].grad.cpu().numpy() for k in range(3)], axis=1)
    check_gradients(gp, t[3].grad.cpu().numpy(), [kap.grad.item(), gam.grad.item()], pop.arrays(),
                    prm, g, "f64", "autograd step")


def test_two_autograd_steps_on_one_workspace_f64():
    """Two differentiable steps on one workspace (x1 = x0 + D0 out of place,
    loss on D1): the first step's backward finds the workspace rebuilt for
    x1 and builds the grid of x0 again.  Checked against the oracle's adjoint
    chained through both steps."""
    prm = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)
    rest = dict(dt=0.01, max_disp=3.0, adherence=0.0)
    pop = smooth_pop(600, 15.0, 55, prm, steps=2)
    arrs = pop.arrays()
    x0 = [a.requires_grad_(True) for a in dev(arrs, "f64")]
    kap = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    gam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    ws = ms.Workspace(pop.n, dtype="f64")
    D0 = msa.mech_step_fn(*x0, kap, gam, ws, rest)
    x1 = [a + b for a, b in zip(x0[:3], D0)]
    D1 = msa.mech_step_fn(*x1, x0[3], kap, gam, ws, rest)
    w = torch.linspace(-1, 1, pop.n, dtype=torch.float64, device="cuda")
    L = (D1[0] * w).sum() + (D1[1] * w * w).sum() - D1[2].sum()
    L.backward()
    # oracle: dL/dx1 = J1^T g1; dL/dx0 = dL/dx1 + J0^T dL/dx1; d and kappa, gamma from both
    g1 = np.stack([w.cpu().numpy(), (w * w).cpu().numpy(), -np.ones(pop.n)], axis=1)
    _, D0o = oracle.step(*arrs, prm)
    a1 = (arrs[0] + D0o[:, 0], arrs[1] + D0o[:, 1], arrs[2] + D0o[:, 2], arrs[3])
    gp1, gd1, kg1 = oracle.step_adjoint(*a1, prm, g1)
    gp0, gd0, kg0 = oracle.step_adjoint(*arrs, prm, gp1)
    Sp1, Ap1, Sd1, Ad1, sk1 = oracle.adjoint_scales(*a1, prm, g1, UNIT["f64"])
    Sp0, Ap0, Sd0, Ad0, sk0 = oracle.adjoint_scales(*arrs, prm, gp1, UNIT["f64"])
    tau = TAU_G["f64"]
    gp = np.stack([x0[k].grad.cpu().numpy() for k in range(3)], axis=1)
    check_vectors(gp, gp1 + gp0, tau * (Sp0 + Sp1 + np.linalg.norm(gp1, axis=1)) + Ap0 + Ap1,
                  "two steps dL/dx0")
    check_vectors(x0[3].grad.cpu().numpy()[:, None], (gd0 + gd1)[:, None],
                  tau * (Sd0 + Sd1) + Ad0 + Ad1, "two steps dL/dd")
    assert abs(kap.grad.item() - (kg0[0] + kg1[0])) <= tau * (sk0[0] + sk1[0]) + sk0[1] + sk1[1]
    assert abs(gam.grad.item() - (kg0[1] + kg1[1])) <= tau * (sk0[2] + sk1[2]) + sk0[3] + sk1[3]
    assert np.abs(gp0).max() > 1e-3                      # the first step does contribute


@pytest.mark.parametrize("mode", ["f64", "f32", "f32_pos64"])
def test_backward_accumulate_is_backward_plus_sum(mode):
    """ms_mech_step_backward_accumulate equals ms_mech_step_backward followed
    by the rollout sums done elementwise (each term converted to the
    positions' type, then added), bit for bit; plain and batched."""
    prm = dict(kappa=2.0, gamma=1.0, dt=0.05, max_disp=0.02, adherence=0.0)
    pop = workloads.uniform(9001, mean_neighbors=15.0, seed=12)
    rng = np.random.default_rng(12)
    ws = ms.Workspace(pop.n, dtype=mode)
    t = dev(pop.arrays(), mode)
    ms.grid_build(ws, *t)
    pin = [torch.from_numpy(rng.normal(size=pop.n)).to(ws.in_dtype).cuda() for _ in range(3)]
    d0 = torch.from_numpy(rng.normal(size=pop.n)).to(ws.in_dtype).cuda()
    k0 = torch.tensor([0.25, -0.5], dtype=torch.float64, device="cuda")
    ox, oy, oz, od, gkg = ms.mech_step_backward(ws, prm, *[a.to(ws.out_dtype) for a in pin])
    want_p = [a + o.to(ws.in_dtype) for a, o in zip(pin, (ox, oy, oz))]
    want_d = d0 + od.to(ws.in_dtype)
    want_k = k0 + gkg
    pb, db, kb = [a.clone() for a in pin], d0.clone(), k0.clone()
    ms.mech_step_backward_accumulate(ws, prm, pb, db, kb)
    ms.device_status(ws)
    for a, b in zip(pb + [db, kb], want_p + [want_d, want_k]):
        assert torch.equal(a, b)
    # batched: three simulations with their own parameters
    b = workloads.batched(n_sims=3, log10_min=3.0, log10_max=3.6, seed=12)
    Pd = ms.params_tensor([dict(prm, kappa=float(k), gamma=float(gm)) for k, gm in zip(b.kappa, b.gamma)],
                          "cuda")
    spec = ms.BatchSpec(b.offsets)
    wsb = ms.Workspace(b.n, max_sims=b.n_sims, dtype=mode)
    ms.grid_build_batched(wsb, *dev(b.arrays(), mode), spec)
    pin = [torch.from_numpy(rng.normal(size=b.n)).to(wsb.in_dtype).cuda() for _ in range(3)]
    d0 = torch.zeros(b.n, dtype=wsb.in_dtype, device="cuda")
    k0 = torch.ones(2 * b.n_sims, dtype=torch.float64, device="cuda")
    ox, oy, oz, od, gkg = ms.mech_step_backward_batched(wsb, Pd, *[a.to(wsb.out_dtype) for a in pin])
    want_p = [a + o.to(wsb.in_dtype) for a, o in zip(pin, (ox, oy, oz))]
    pb, db, kb = [a.clone() for a in pin], d0.clone(), k0.clone()
    ms.mech_step_backward_batched_accumulate(wsb, Pd, pb, db, kb)
    ms.device_status(wsb)
    for a, w_ in zip(pb, want_p):
        assert torch.equal(a, w_)
    assert torch.equal(db, d0 + od.to(wsb.in_dtype))
    assert torch.equal(kb, k0 + gkg.reshape(-1))


def _rollout_loss(mode, pop, tgt, steps, K, rest, kap=2.0, gam=1.0, ws=None):
    t = [a.requires_grad_(True) for a in dev(pop.arrays(), mode)]
    k = torch.tensor(kap, dtype=torch.float64, requires_grad=True)
    g = torch.tensor(gam, dtype=torch.float64, requires_grad=True)
    ws = ws or ms.Workspace(pop.n, dtype=mode)
    px, py, pz = msa.rollout(*t, k, g, ws, rest, steps, K)
    tx, ty, tz = (torch.from_numpy(np.asarray(a).astype(NP_IN[mode])).cuda() for a in tgt)
    L = ((px - tx) ** 2 + (py - ty) ** 2 + (pz - tz) ** 2).mean()
    L.backward()
    return L.item(), [a.grad.clone() for a in t], k.grad.item(), g.grad.item()


@pytest.mark.parametrize("mode", ["f64", "f32", "f32_pos64"])
def test_rollout_checkpoint_interval_invariance(mode):
    rest = dict(dt=0.05, max_disp=3.0, adherence=0.0)
    pop = workloads.uniform(3000, mean_neighbors=12.0, seed=3)
    tgt = workloads.targets(pop, seed=3)
    r1 = _rollout_loss(mode, pop, tgt, 20, 1, rest)
    r10 = _rollout_loss(mode, pop, tgt, 20, 10, rest)
    assert r1[0] == r10[0]
    for a, b in zip(r1[1], r10[1]):
        assert torch.equal(a, b)
    assert r1[2] == r10[2] and r1[3] == r10[3]


def test_rollout_gradient_matches_oracle_f64():
    prm = dict(kappa=2.0, gamma=1.0, dt=0.05, max_disp=3.0, adherence=0.0)
    rest = dict(dt=0.05, max_disp=3.0, adherence=0.0)
    pop = smooth_pop(800, 12.0, 70, prm, gap=1e-2, steps=6)
    tgt = workloads.targets(pop, seed=1)
    steps = 6
    L, gp, gk, gg = _rollout_loss("f64", pop, tgt, steps, 4, rest)
    Lo = oracle.rollout_loss(*pop.arrays(), prm, steps, tgt)
    gp_o, gd_o, kg_o = oracle.rollout_grad(*pop.arrays(), prm, steps, tgt)
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    gpo = np.stack([a.cpu().numpy() for a in gp[:3]], axis=1)
    assert np.abs(gpo - gp_o).max() <= 1e-10 * np.abs(gp_o).max()
    assert np.abs(gp[3].cpu().numpy() - gd_o).max() <= 1e-10 * np.abs(gd_o).max()
    np.testing.assert_allclose([gk, gg], kg_o, rtol=1e-9)
    # agent by agent: the per-step scales of the oracle's adjoint summed over
    # the trajectory, plus the carried gradient itself
    arrs = pop.arrays()
    traj = oracle.rollout(*arrs, prm, steps)
    t_ = np.stack([np.asarray(a) for a in tgt], axis=1)
    pbar = 2.0 * (traj[-1] - t_) / pop.n
    sp_sum = np.linalg.norm(pbar, axis=1)
    sd_sum = np.zeros(pop.n)
    for s in range(steps - 1, -1, -1):
        q = (traj[s][:, 0], traj[s][:, 1], traj[s][:, 2], arrs[3])
        Sp, Ap, Sd, Ad, _ = oracle.adjoint_scales(*q, prm, pbar, UNIT["f64"])
        pbar = pbar + oracle.step_adjoint(*q, prm, pbar)[0]
        sp_sum += Sp + Ap / TAU_G["f64"] + np.linalg.norm(pbar, axis=1)
        sd_sum += Sd + Ad / TAU_G["f64"]
    check_vectors(gpo, gp_o, 1e-11 * sp_sum, "rollout dL/dp0")
    check_vectors(gp[3].cpu().numpy()[:, None], gd_o[:, None], 1e-11 * sd_sum, "rollout dL/dd")


def test_rollout_gradient_central_differences_gpu_f64():
    """Central finite differences of the GPU FP64 rollout loss itself."""
    prm = dict(kappa=2.0, gamma=1.0, dt=0.05, max_disp=3.0, adherence=0.0)
    rest = dict(dt=0.05, max_disp=3.0, adherence=0.0)
    pop = smooth_pop(300, 12.0, 90, prm, gap=1e-2, steps=5)
    tgt = workloads.targets(pop, seed=2)
    steps, K = 5, 2
    L, gp, gk, gg = _rollout_loss("f64", pop, tgt, steps, K, rest)
    ws = ms.Workspace(pop.n, dtype="f64")

    def loss(arrs, kap=2.0, gam=1.0):
        t = dev(arrs, "f64")
        with torch.no_grad():
            px, py, pz = msa.rollout(*t, kap, gam, ws, rest, steps, K)
            tx, ty, tz = (torch.from_numpy(np.asarray(a)).cuda() for a in tgt)
            return ((px - tx) ** 2 + (py - ty) ** 2 + (pz - tz) ** 2).mean().item()

    h = 1e-6
    arrs = [np.array(a) for a in pop.arrays()]
    scale = max(float(torch.cat(gp[:3]).abs().max()), 1e-6)
    for i in range(0, pop.n, 37):
        for k in range(4):
            ap = [a.copy() for a in arrs]; ap[k][i] += h
            am = [a.copy() for a in arrs]; am[k][i] -= h
            fd = (loss(ap) - loss(am)) / (2 * h)
            got = gp[k][i].item()
            ref = scale if k < 3 else max(float(gp[3].abs().max()), 1e-6)
            assert abs(fd - got) <= 1e-6 * ref + 1e-9, (i, k, fd, got)
    fdk = (loss(arrs, kap=2.0 + h) - loss(arrs, kap=2.0 - h)) / (2 * h)
    fdg = (loss(arrs, gam=1.0 + h) - loss(arrs, gam=1.0 - h)) / (2 * h)
    assert abs(fdk - gk) <= 1e-6 * abs(gk) + 1e-9
    assert abs(fdg - gg) <= 1e-6 * abs(gg) + 1e-9


@pytest.mark.parametrize("mode", ["f64", "f32", "f32_pos64"])
@pytest.mark.parametrize("case", ["uniform_n12", "dense_clusters"])
def test_kept_forces_give_identical_results(mode, case):
    """A forward step that keeps its forces lets the backward skip the force
    recompute only for the same build and parameters; forward and backward
    results are identical bit for bit to the recomputing path, and a new build
    or other parameters fall back to the recompute.  The dense case has
    clamped agents, whose displacement arithmetic must round the same way in
    the keeping and the plain force kernel."""
    pop = workloads.uniform(20000, mean_neighbors=12.0, seed=8) if case == "uniform_n12" else \
        workloads.clusters(20000, n_clusters=3, side=250.0, seed=42)
    n = pop.n
    rng = np.random.default_rng(8)
    g = dev(rng.normal(size=(3, n)), "f64" if mode == "f64" else "f32")
    pa = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)
    pb = dict(pa, kappa=2.5)
    t = dev(pop.arrays(), mode)
    t2 = [a + 0.3 for a in t[:3]] + [t[3]]
    ws0 = ms.Workspace(n, dtype=mode)
    ws1 = ms.Workspace(n, dtype=mode, keep_forces=True)

    def same(u, v):
        for a, b in zip(u, v):
            assert torch.equal(a, b)

    ms.grid_build(ws0, *t)
    ms.grid_build(ws1, *t)
    same(ms.mech_step(ws0, pa), ms.mech_step(ws1, pa))
    same(ms.mech_step_backward(ws0, pa, *g), ms.mech_step_backward(ws1, pa, *g))   # kept
    same(ms.mech_step_backward(ws0, pb, *g), ms.mech_step_backward(ws1, pb, *g))   # other params
    ms.grid_build(ws0, *t2)
    ms.grid_build(ws1, *t2)                                                        # new build
    same(ms.mech_step_backward(ws0, pa, *g), ms.mech_step_backward(ws1, pa, *g))
    ms.device_status(ws1)

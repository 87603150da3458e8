"""Pins of the oracle's reverse-mode derivative against central finite
differences of the oracle's forward step (Eq. 1 and the displacement rule of
Section III).  Finite differences use only the forward pass, so they check the
hand-derived adjoint independently.

The forward map has kinks (contact onset delta = 0, the length bound |v| = m,
the adherence test); s'(delta) is unbounded as delta -> 0+.  Configurations are
drawn until every pair within the interaction radius has |delta| > 1e-2 and
every agent has ||v| - m| > 1e-3 m, so the probes stay on smooth pieces.
"""
import numpy as np
import pytest

import oracle
from paper_2105_00039_amd import workloads


def smooth_config(n, nbrs, seed, params, min_gap=1e-2):
    for s in range(seed, seed + 500):
        pop = workloads.uniform(n, mean_neighbors=nbrs, seed=s)
        pos = np.stack([pop.x, pop.y, pop.z], axis=1)
        diff = pos[:, None, :] - pos[None, :, :]
        l = np.sqrt((diff ** 2).sum(-1))
        r = pop.d / 2
        delta = r[:, None] + r[None, :] - l
        np.fill_diagonal(delta, 10.0)
        near = l < pop.d.max()
        if np.any(np.abs(delta[near]) < min_gap):
            continue
        F, _ = oracle.step(pop.x, pop.y, pop.z, pop.d, params)
        v = params["dt"] * np.linalg.norm(F, axis=1)
        if np.any(np.abs(v - params["max_disp"]) < 1e-3 * params["max_disp"]):
            continue
        return pop
    raise RuntimeError("no smooth configuration found")


def loss_of(pos, d, params, c):
    _, D = oracle.step(pos[:, 0], pos[:, 1], pos[:, 2], d, params)
    return float(np.sum(c * D))


@pytest.mark.parametrize("clamp", [False, True])
def test_step_adjoint_matches_central_differences(clamp):
    params = dict(kappa=2.0, gamma=1.0, dt=0.05 if clamp else 0.01,
                  max_disp=0.02 if clamp else 3.0, adherence=0.0)
    pop = smooth_config(60, 20.0, 20 if clamp else 40, params)
    rng = np.random.default_rng(3)
    c = rng.normal(size=(pop.n, 3))
    pos = np.stack([pop.x, pop.y, pop.z], axis=1)
    gp, gd, gkg = oracle.step_adjoint(pop.x, pop.y, pop.z, pop.d, params, c)
    F, _ = oracle.step(pop.x, pop.y, pop.z, pop.d, params)
    nclamped = int(np.sum(params["dt"] * np.linalg.norm(F, axis=1) > params["max_disp"]))
    if clamp:
        assert nclamped > 10
    else:
        assert nclamped == 0
    h = 1e-5
    scale = max(np.abs(gp).max(), 1e-3)
    for i in range(0, pop.n, 3):
        for k in range(3):
            pp = pos.copy(); pp[i, k] += h
            pm = pos.copy(); pm[i, k] -= h
            fd = (loss_of(pp, pop.d, params, c) - loss_of(pm, pop.d, params, c)) / (2 * h)
            assert abs(fd - gp[i, k]) <= 1e-6 * scale, (i, k, fd, gp[i, k])
        dp = pop.d.copy(); dp[i] += h
        dm = pop.d.copy(); dm[i] -= h
        fd = (loss_of(pos, dp, params, c) - loss_of(pos, dm, params, c)) / (2 * h)
        assert abs(fd - gd[i]) <= 1e-6 * max(np.abs(gd).max(), 1e-3), (i, fd, gd[i])
    for k, key in enumerate(("kappa", "gamma")):
        fd = (loss_of(pos, pop.d, dict(params, **{key: params[key] + h}), c)
              - loss_of(pos, pop.d, dict(params, **{key: params[key] - h}), c)) / (2 * h)
        assert abs(fd - gkg[k]) <= 1e-6 * max(abs(fd), 1e-3), (key, fd, gkg[k])


def test_adherence_blocks_gradient():
    params = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=1e9)
    pop = workloads.uniform(200, mean_neighbors=12.0, seed=2)
    c = np.ones((pop.n, 3))
    gp, gd, gkg = oracle.step_adjoint(pop.x, pop.y, pop.z, pop.d, params, c)
    assert np.all(gp == 0) and np.all(gd == 0) and np.all(gkg == 0)


def test_rollout_gradient_matches_central_differences():
    params = dict(kappa=2.0, gamma=1.0, dt=0.05, max_disp=3.0, adherence=0.0)
    pop = smooth_config(40, 15.0, 60, params, min_gap=3e-2)
    tx, ty, tz = workloads.targets(pop, sigma=1.0, seed=0)
    steps = 4
    gp, gd, gkg = oracle.rollout_grad(pop.x, pop.y, pop.z, pop.d, params, steps, (tx, ty, tz))
    pos = np.stack([pop.x, pop.y, pop.z], axis=1)

    def L(p, d, prm):
        return oracle.rollout_loss(p[:, 0], p[:, 1], p[:, 2], d, prm, steps, (tx, ty, tz))

    h = 1e-6
    for i in range(0, pop.n, 4):
        for k in range(3):
            pp = pos.copy(); pp[i, k] += h
            pm = pos.copy(); pm[i, k] -= h
            fd = (L(pp, pop.d, params) - L(pm, pop.d, params)) / (2 * h)
            assert abs(fd - gp[i, k]) <= 1e-6 * np.abs(gp).max() + 1e-9, (i, k, fd, gp[i, k])
        dp = pop.d.copy(); dp[i] += h
        dm = pop.d.copy(); dm[i] -= h
        fd = (L(pos, dp, params) - L(pos, dm, params)) / (2 * h)
        assert abs(fd - gd[i]) <= 1e-6 * np.abs(gd).max() + 1e-9, (i, fd, gd[i])
    for k, key in enumerate(("kappa", "gamma")):
        fd = (L(pos, pop.d, dict(params, **{key: params[key] + h}))
              - L(pos, pop.d, dict(params, **{key: params[key] - h}))) / (2 * h)
        assert abs(fd - gkg[k]) <= 1e-6 * abs(gkg[k]) + 1e-9, (key, fd, gkg[k])

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


# ------------------------------------------------ gradient acceptance scales ---
#
# oracle.adjoint_scales gives the per-agent scales that GPU gradients are
# compared with.  Pinned to closed forms on the W1 pair (d = 10, 10, 9 apart:
# delta = 1, rho = 2.5, l = 9) and to an all-pairs numpy recomputation; the
# oracle's own gradient must respect them (the scales bound each term).

U24 = 2.0 ** -24
P = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)


def test_adjoint_scales_closed_forms():
    x = np.array([0.0, 9.0])
    z0 = np.zeros(2)
    d = np.array([10.0, 10.0])
    g = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])     # unclamped: Fbar = dt g
    Sp, Ap, Sd, Ad, skg = oracle.adjoint_scales(x, z0, z0, d, P, g, U24)
    W = 0.01                                            # |Fbar_1| + |Fbar_2|
    s = 2.0 - np.sqrt(2.5)
    s_delta = 2.0 - np.sqrt(2.5) / 2.0                  # kappa - gamma rho / (2 sqrt(rho delta))
    s_rho = -1.0 / (2.0 * np.sqrt(2.5))                 # -gamma delta / (2 sqrt(rho delta))
    s_dd = 2.5 ** 2 / (4.0 * 2.5 ** 1.5)                # gamma rho^2 / (4 (rho delta)^1.5)
    c2 = 0.25                                           # r_j^2 / (r_i + r_j)^2
    eta = 4 * U24 * 19.0
    np.testing.assert_allclose(Sp, W * (2 * s / 9.0 + s_delta), rtol=1e-14)
    np.testing.assert_allclose(Sd, 0.5 * W * (s_delta + abs(s_rho) * c2), rtol=1e-14)
    np.testing.assert_allclose(Ap, eta * W * (2 * s_delta / 9.0 + s_dd), rtol=1e-13)
    np.testing.assert_allclose(Ad, 0.5 * eta * W * (s_dd + 1.0 / (4 * np.sqrt(2.5)) * c2), rtol=1e-13)
    # parameter scales: only the ordered pair (1, 2) carries |Fbar_1| = 0.01
    np.testing.assert_allclose(skg, [0.01, eta * 0.01, np.sqrt(2.5) * 0.01,
                                     eta * 2.5 / (2 * np.sqrt(2.5)) * 0.01], rtol=1e-13)
    # apart: nothing
    Sp, Ap, Sd, Ad, skg = oracle.adjoint_scales(np.array([0.0, 10.5]), z0, z0, d, P, g, U24)
    assert np.all(Sp == 0) and np.all(Ap == 0) and np.all(Sd == 0) and np.all(skg == 0)


def test_adjoint_scales_bound_the_gradient_and_match_all_pairs():
    pop = workloads.uniform(400, mean_neighbors=20.0, seed=41)
    x, y, z, d = pop.arrays()
    F0, _ = oracle.step(x, y, z, d, dict(P, dt=0.05, max_disp=1e9))
    # the length bound at the median step: half the agents clamped
    params = dict(P, dt=0.05, max_disp=float(np.median(0.05 * np.linalg.norm(F0, axis=1))))
    g = np.random.default_rng(41).normal(size=(pop.n, 3))
    Sp, Ap, Sd, Ad, skg = oracle.adjoint_scales(x, y, z, d, params, g, 2.0 ** -53)
    gp, gd, gkg = oracle.step_adjoint(x, y, z, d, params, g)
    # each term is bounded by its scale (triangle inequality)
    assert np.all(np.linalg.norm(gp, axis=1) <= Sp * (1 + 1e-12))
    assert np.all(np.abs(gd) <= Sd * (1 + 1e-12))
    assert abs(gkg[0]) <= skg[0] and abs(gkg[1]) <= skg[2]
    # all-pairs recomputation; Fbar from the displacement rule on the oracle's force
    F, _ = oracle.step(x, y, z, d, params)
    v = params["dt"] * F
    vn = np.linalg.norm(v, axis=1)
    clamped = vn > params["max_disp"]
    assert clamped.sum() > 20 and (~clamped).sum() > 20
    vh = v / np.maximum(vn, 1e-300)[:, None]
    Fb = params["dt"] * g
    proj = g - vh * np.sum(vh * g, axis=1, keepdims=True)
    Fb[clamped] = (params["dt"] * params["max_disp"] / vn[clamped])[:, None] * proj[clamped]
    fn = np.linalg.norm(Fb, axis=1)
    p = np.stack([x, y, z], axis=1)
    r = d / 2
    l = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    rs = r[:, None] + r[None, :]
    delta = rs - l
    contact = (delta > 0) & ~np.eye(pop.n, dtype=bool)
    dl = np.where(contact, delta, 1.0)
    rho = r[:, None] * r[None, :] / rs
    sq = np.sqrt(rho * dl)
    s = 2.0 * dl - sq
    s_delta = 2.0 - rho / (2 * sq)
    s_rho = -dl / (2 * sq)
    W = fn[:, None] + fn[None, :]
    c2 = (r[None, :] / rs) ** 2
    Spn = np.where(contact, W * (2 * np.abs(s) / np.where(contact, l, 1.0) + np.abs(s_delta)), 0).sum(1)
    Sdn = np.where(contact, 0.5 * W * (np.abs(s_delta) + np.abs(s_rho) * c2), 0).sum(1)
    np.testing.assert_allclose(Sp, Spn, rtol=1e-11)
    np.testing.assert_allclose(Sd, Sdn, rtol=1e-11)
    np.testing.assert_allclose(skg[0], np.where(contact, dl * fn[:, None], 0).sum(), rtol=1e-11)
    np.testing.assert_allclose(skg[2], np.where(contact, sq * fn[:, None], 0).sum(), rtol=1e-11)

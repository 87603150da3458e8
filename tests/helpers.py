"""Shared helpers of the GPU parity tests (no test functions here)."""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
TAU = {"f32": 1e-4, "f64": 1e-12, "f32_pos64": 1e-4}
UNIT = {"f32": U32, "f64": U64, "f32_pos64": U32}
NP_IN = {"f32": np.float32, "f64": np.float64, "f32_pos64": np.float64}


def oracle_inputs(pop_arrays, mode):
    """What the oracle is fed for a precision mode: the exact values the GPU
    path computes with, widened to FP64: both FP32 modes see the inputs rounded
    to nearest FP32 (the mixed mode rounds its FP64 master positions)."""
    if mode in ("f32", "f32_pos64"):
        return tuple(np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
                     for a in pop_arrays)
    return tuple(np.asarray(a).astype(np.float64) for a in pop_arrays)


def force_bound(S, A, mode):
    """Per-agent acceptance radius for a force: tau * S + A."""
    return TAU[mode] * S + A


def check_vectors(got, want, bound, what):
    """|got_i - want_i| <= bound_i for every agent; exact zero where bound is 0."""
    err = np.linalg.norm(np.asarray(got, dtype=np.float64) - want, axis=1)
    bad = np.nonzero(err > bound)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{what}: {bad.size} agents out of tolerance; first {i}: "
                             f"got {got[i]}, want {want[i]}, err {err[i]:.3e} > bound {bound[i]:.3e}")
    return float(np.max(err / np.maximum(bound, 1e-300), initial=0.0))


# Gradients: per-agent acceptance |g_i - g_oracle_i| <= tau_g * S_i + A_i with
# the scales of oracle.adjoint_scales.  tau_g as for the forces on the FP64
# path; on the FP32 paths 1e-3, which also covers the FP32 force error that the
# length bound passes on to Fbar (the direction of F, up to about 1e-4 S/|F|).
TAU_G = {"f32": 1e-3, "f64": 1e-12, "f32_pos64": 1e-3}


def check_gradients(gp, gd, gkg, arrs_o, params, gD, mode, what, edge=0.0):
    """Compare one backward step's (gp (n,3), gd (n,), gkg (2,)) with the
    oracle's adjoint of the same step, agent by agent.  arrs_o: the inputs as
    the oracle sees them (oracle_inputs)."""
    import oracle
    gp_o, gd_o, kg_o = oracle.step_adjoint(*arrs_o, params, gD, edge)
    Sp, Ap, Sd, Ad, skg = oracle.adjoint_scales(*arrs_o, params, gD, UNIT[mode], edge)
    tau = TAU_G[mode]
    w1 = check_vectors(np.asarray(gp, dtype=np.float64), gp_o, tau * Sp + Ap, f"{what} dL/dp")
    w2 = check_vectors(np.asarray(gd, dtype=np.float64)[:, None], gd_o[:, None], tau * Sd + Ad,
                       f"{what} dL/dd")
    ek = abs(float(gkg[0]) - kg_o[0])
    eg = abs(float(gkg[1]) - kg_o[1])
    assert ek <= tau * skg[0] + skg[1], (what, "kappa", float(gkg[0]), kg_o[0], skg[:2])
    assert eg <= tau * skg[2] + skg[3], (what, "gamma", float(gkg[1]), kg_o[1], skg[2:])
    nz = Sp > 0
    assert np.all(np.asarray(gp)[~nz] == 0), f"{what}: agents without contacts must get 0"
    return max(w1, w2)

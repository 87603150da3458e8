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

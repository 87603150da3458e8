"""FP64 CPU oracle for the mechanical-interaction step (arXiv 2105.00039).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU product path.  It shares no code
with that path.  The arithmetic lives in ``mech_oracle.c`` (plain C99, FP64,
no FMA contraction); this module compiles it on demand with gcc and exposes it
on numpy arrays.

Functions and the passages they follow:

* ``geometry``, ``grid``           uniform grid, Section IV-A.
* ``neighbors``                    27-box neighbourhood within the radius,
                                   Sections III and IV-A.
* ``brute_neighbors``              O(N^2) enumeration of the same sets.
* ``step``                         Eq. 1 summed per agent, then the
                                   displacement rule of Section III.
* ``brute_forces``                 Eq. 1 over all pairs, no grid.
* ``tolerance_scales``             per-agent scales of the acceptance test.
* ``sample``                       ``step`` and ``tolerance_scales`` for a
                                   sample of agents of a large population.
* ``step_adjoint``                 reverse-mode derivative of ``step``.
* ``adjoint_scales``               per-agent scales of the acceptance test
                                   for gradients.
* ``rollout``, ``rollout_grad``    repeated steps with the grid rebuilt each
                                   step (Section IV-A) and their gradient.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mech_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
# The timing copy for the CPU baseline: same source, -O3 for the host it is
# built on.  It is compiled where it runs, never shipped prebuilt.
_LIB_FAST = os.path.join(_HERE, "liborc_native.so")
# A test may point the wrapper at another build of the oracle (the mutation
# tests load deliberately broken copies to show the pins catch them).
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")
_CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]
_CFLAGS_FAST = ["-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                "-fno-fast-math", "-fopenmp"]
_lock = threading.Lock()
_lib = None

OK, EINVAL, ECAPACITY, EINPUT = 0, 1, 2, 4


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False, native: bool = False) -> str:
    """Compile liborc.so with gcc (portable x86-64, OpenMP), or with
    native=True the timing copy liborc_native.so (-O3 -march=native, OpenMP;
    always recompiled, for the host it runs on)."""
    out, flags = (_LIB_FAST, _CFLAGS_FAST) if native else (_LIB, _CFLAGS)
    if native or force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *flags, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def use_native():
    """Load the -O3 -march=native timing copy in place of the test build
    (before the first call; the CPU baseline of the benchmark uses it)."""
    global _lib
    with _lock:
        if _lib is not None:
            raise RuntimeError("oracle already loaded")
        _lib = _bind(ctypes.CDLL(build(native=True)))


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                L = ctypes.CDLL(_LIB_OVERRIDE)
            else:
                build()
                L = ctypes.CDLL(_LIB)
            _lib = _bind(L)
    return _lib


def _bind(L):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    sig = {
        "orc_geometry": [I64, P, P, P, P, D, P, P, P, P],
        "orc_grid": [I64, P, P, P, P, D, P, P, P],
        "orc_neighbors": [I64, P, P, P, P, D, P, P, P, I64],
        "orc_brute_neighbors": [I64, P, P, P, D, P, P, P, I64],
        "orc_step": [I64, P, P, P, P, D, P, P, P, P, P, P, P],
        "orc_brute_forces": [I64, P, P, P, P, D, D, P, P, P],
        "orc_tolerance_scales": [I64, P, P, P, P, D, D, D, D, P, P, P],
        "orc_step_adjoint": [I64, P, P, P, P, D, P, P, P, P, P, P, P, P, P],
        "orc_integrate": [I64, P, P, P, P, P, P],
        "orc_sample": [I64, P, P, P, P, D, P, D, I64, P, P, P, P, P, P, P, P, P, P],
        "orc_adjoint_scales": [I64, P, P, P, P, D, P, P, P, P, D, P, P, P, P, P],
        "orc_set_threads": [ctypes.c_int],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    return L


def set_threads(t: int) -> int:
    """Threads for the following calls (t <= 0 leaves it); returns the count.
    Results do not depend on it."""
    return int(lib().orc_set_threads(int(t)))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


def _params(params):
    keys = ("kappa", "gamma", "dt", "max_disp", "adherence")
    if isinstance(params, dict):
        return np.array([float(params[k]) for k in keys], dtype=np.float64)
    return _f64(params)


def geometry(x, y, z, d, edge=0.0):
    """(origin[3], edge, dims[3], n_boxes) of the grid."""
    x, y, z, d = map(_f64, (x, y, z, d))
    o = np.zeros(3)
    e = np.zeros(1)
    dims = np.zeros(3, dtype=np.int64)
    nb = np.zeros(1, dtype=np.int64)
    _check(lib().orc_geometry(x.size, _p(x), _p(y), _p(z), _p(d), float(edge), _p(o), _p(e),
                              _p(dims), _p(nb)), "geometry")
    return o, float(e[0]), dims, int(nb[0])


def grid(x, y, z, d, edge=0.0):
    """Box index per agent, box start offsets [n_boxes+1] and stable box order."""
    x, y, z, d = map(_f64, (x, y, z, d))
    _, _, _, nb = geometry(x, y, z, d, edge)
    n = x.size
    box = np.zeros(n, dtype=np.int32)
    start = np.zeros(nb + 1, dtype=np.int32)
    perm = np.zeros(n, dtype=np.int32)
    _check(lib().orc_grid(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(box), _p(start), _p(perm)),
           "grid")
    return box, start, perm


def neighbors(x, y, z, d, edge=0.0):
    """(counts[n], offsets[n+1], list) of the canonical neighbour sets."""
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    counts = np.zeros(n, dtype=np.int32)
    offsets = np.zeros(n + 1, dtype=np.int64)
    _check(lib().orc_neighbors(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(counts), _p(offsets),
                               None, 0), "neighbors")
    lst = np.zeros(max(int(offsets[-1]), 1), dtype=np.int32)
    _check(lib().orc_neighbors(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(counts), _p(offsets),
                               _p(lst), lst.size), "neighbors")
    return counts, offsets, lst[: int(offsets[-1])]


def brute_neighbors(x, y, z, radius):
    x, y, z = map(_f64, (x, y, z))
    n = x.size
    counts = np.zeros(n, dtype=np.int32)
    offsets = np.zeros(n + 1, dtype=np.int64)
    _check(lib().orc_brute_neighbors(n, _p(x), _p(y), _p(z), float(radius), _p(counts), _p(offsets),
                                     None, 0), "brute_neighbors")
    lst = np.zeros(max(int(offsets[-1]), 1), dtype=np.int32)
    _check(lib().orc_brute_neighbors(n, _p(x), _p(y), _p(z), float(radius), _p(counts), _p(offsets),
                                     _p(lst), lst.size), "brute_neighbors")
    return counts, offsets, lst[: int(offsets[-1])]


def step(x, y, z, d, params, edge=0.0):
    """Total force F (n,3) and displacement D (n,3) of one step."""
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    F = [np.zeros(n) for _ in range(3)]
    D = [np.zeros(n) for _ in range(3)]
    _check(lib().orc_step(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(_params(params)),
                          *map(_p, F), *map(_p, D)), "step")
    return np.stack(F, axis=1), np.stack(D, axis=1)


def brute_forces(x, y, z, d, kappa, gamma):
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    F = [np.zeros(n) for _ in range(3)]
    _check(lib().orc_brute_forces(n, _p(x), _p(y), _p(z), _p(d), float(kappa), float(gamma),
                                  *map(_p, F)), "brute_forces")
    return np.stack(F, axis=1)


def tolerance_scales(x, y, z, d, kappa, gamma, unit_roundoff, edge=0.0):
    """Per-agent (S, A, contacts) of the acceptance test (see mech_oracle.c)."""
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    S = np.zeros(n)
    A = np.zeros(n)
    C = np.zeros(n, dtype=np.int32)
    _check(lib().orc_tolerance_scales(n, _p(x), _p(y), _p(z), _p(d), float(edge), float(kappa),
                                      float(gamma), float(unit_roundoff), _p(S), _p(A), _p(C)),
           "tolerance_scales")
    return S, A, C


def sample(x, y, z, d, params, idx, unit_roundoff=0.0, edge=0.0):
    """For the agents ``idx`` only: force F (m,3), displacement D (m,3) and the
    acceptance scales S, A, contacts C (m,) -- the rows ``idx`` of ``step`` and
    ``tolerance_scales`` bit for bit, with the grid built over all agents."""
    x, y, z, d = map(_f64, (x, y, z, d))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.size
    F = [np.zeros(m) for _ in range(3)]
    D = [np.zeros(m) for _ in range(3)]
    S = np.zeros(m)
    A = np.zeros(m)
    C = np.zeros(m, dtype=np.int32)
    _check(lib().orc_sample(x.size, _p(x), _p(y), _p(z), _p(d), float(edge), _p(_params(params)),
                            float(unit_roundoff), m, _p(idx), *map(_p, F), *map(_p, D), _p(S), _p(A),
                            _p(C)), "sample")
    return np.stack(F, axis=1), np.stack(D, axis=1), S, A, C


def step_adjoint(x, y, z, d, params, gD, edge=0.0):
    """Given gD = dL/dDelta (n,3): (gp (n,3), gd (n,), [dL/dkappa, dL/dgamma])."""
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    gD = np.asarray(gD, dtype=np.float64)
    g = [np.ascontiguousarray(gD[:, k]) for k in range(3)]
    gp = [np.zeros(n) for _ in range(3)]
    gd = np.zeros(n)
    gkg = np.zeros(2)
    _check(lib().orc_step_adjoint(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(_params(params)),
                                  *map(_p, g), *map(_p, gp), _p(gd), _p(gkg)), "step_adjoint")
    return np.stack(gp, axis=1), gd, gkg


def adjoint_scales(x, y, z, d, params, gD, unit_roundoff, edge=0.0):
    """Per-agent scales of the gradient acceptance test for gD = dL/dDelta:
    (Sp, Ap) for the position gradient, (Sd, Ad) for the diameter gradient,
    and [S_kappa, A_kappa, S_gamma, A_gamma] for the parameter gradients (see
    mech_oracle.c).  A gradient g of the same step computed in another
    precision or order is accepted when |g_i - g_oracle_i| <= tau S_i + A_i."""
    x, y, z, d = map(_f64, (x, y, z, d))
    n = x.size
    gD = np.asarray(gD, dtype=np.float64)
    g = [np.ascontiguousarray(gD[:, k]) for k in range(3)]
    out = [np.zeros(n) for _ in range(4)]
    skg = np.zeros(4)
    _check(lib().orc_adjoint_scales(n, _p(x), _p(y), _p(z), _p(d), float(edge), _p(_params(params)),
                                    *map(_p, g), float(unit_roundoff), *map(_p, out), _p(skg)),
           "adjoint_scales")
    return out[0], out[1], out[2], out[3], skg


def rollout(x, y, z, d, params, steps, edge=0.0):
    """Positions after ``steps`` Jacobi steps, grid rebuilt every step.
    Returns the list of positions p_0 .. p_steps, each (n,3)."""
    p = np.stack([_f64(x), _f64(y), _f64(z)], axis=1).copy()
    out = [p.copy()]
    for _ in range(steps):
        _, D = step(p[:, 0], p[:, 1], p[:, 2], d, params, edge)
        p = p + D
        out.append(p.copy())
    return out


def rollout_loss(x, y, z, d, params, steps, target, edge=0.0):
    """L = mean over agents of |p_T - t|^2."""
    pT = rollout(x, y, z, d, params, steps, edge)[-1]
    t = np.stack([_f64(a) for a in target], axis=1)
    return float(np.mean(np.sum((pT - t) ** 2, axis=1)))


def rollout_grad(x, y, z, d, params, steps, target, edge=0.0):
    """Gradient of ``rollout_loss`` wrt (p_0 (n,3), d (n,), kappa, gamma),
    by reverse accumulation over the stored trajectory: p_{t+1} = p_t + D(p_t),
    so pbar_t = pbar_{t+1} + J_D(p_t)^T pbar_{t+1}."""
    traj = rollout(x, y, z, d, params, steps, edge)
    n = traj[0].shape[0]
    t = np.stack([_f64(a) for a in target], axis=1)
    pbar = 2.0 * (traj[-1] - t) / n
    dbar = np.zeros(n)
    kg = np.zeros(2)
    for s in range(steps - 1, -1, -1):
        p = traj[s]
        gp, gd, gkg = step_adjoint(p[:, 0], p[:, 1], p[:, 2], d, params, pbar, edge)
        pbar = pbar + gp
        dbar += gd
        kg += gkg
    return pbar, dbar, kg

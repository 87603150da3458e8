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


def tiled_boxes(box, dims, shift):
    """Box ids in the exported numbering from the oracle's row-major ids
    (ix + nx*(iy + ny*iz)): x stays fastest and the x-rows (iy, iz) go to
    2^shift x 2^shift tiles, tiles row-major with ceil(ny / 2^shift) along y
    and rows row-major inside a tile (the library's ms_box_order).  Also
    returns the box count of that numbering."""
    box = np.asarray(box, dtype=np.int64)
    nx, ny, nz = (int(v) for v in dims)
    if shift == 0:
        return box, nx * ny * nz
    t = 1 << shift
    ty = -(-ny // t)

    def row(iy, iz):
        return ((iz // t) * ty + iy // t) * t * t + (iz % t) * t + iy % t

    ix, r = box % nx, box // nx
    iy, iz = r % ny, r // ny
    return ix + nx * row(iy, iz), nx * (int(row(ty * t - 1, nz - 1)) + 1)


def grid_in_order(box, dims, shift):
    """The oracle's grid (row-major box ids) renumbered to the exported
    order: box ids, box starts (exclusive scan of the per-box counts, n_boxes
    + 1 entries) and the canonical order (ascending box, then ascending agent
    index), plus the box count."""
    key, nb = tiled_boxes(box, dims, shift)
    cnt = np.bincount(key, minlength=nb) if key.size else np.zeros(nb, dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    perm = np.argsort(key, kind="stable")
    return key, start, perm, nb


def expect_grid(g, box, start, perm, dims, nb, sim=0):
    """The exported grid g (ms.grid_get) equals the oracle's (box ids, box
    starts, canonical order, box count nb), renumbered to the row order the
    build reports (tile_shift)."""
    info = g["info"][sim]
    shift = int(info["tile_shift"])
    if shift:
        box, start, perm, nb = grid_in_order(box, dims, shift)
    assert info["n_boxes"] == nb, (info["n_boxes"], nb, shift)
    assert np.array_equal(g["box_id"].cpu().numpy(), box)
    assert np.array_equal(g["start"].cpu().numpy(), start)
    assert np.array_equal(g["perm"].cpu().numpy(), perm)
    return shift

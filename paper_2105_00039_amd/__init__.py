"""Mechanical-interaction step for 3D agent-based simulations on MI355X.

Python binding of libmechstep.so (include/mechstep.h).  Every step of the
computation runs in the library's HIP kernels; this module only checks and
marshals torch device tensors and passes torch's current HIP stream.

    import torch, paper_2105_00039_amd as ms
    ws = ms.Workspace(n, dtype="f32")
    ms.grid_build(ws, x, y, z, d)             # uniform grid (Section IV-A)
    dx, dy, dz = ms.mech_step(ws, params)     # Eq. 1 + displacement (Section III)
    ms.integrate(x, y, z, dx, dy, dz)

``params`` is a dict with kappa, gamma, dt, max_disp, adherence.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MechStepError, MS_F32, MS_F64, MS_F32_POS64  # noqa: F401

__all__ = [
    "Workspace", "BatchSpec", "grid_build", "mech_step", "mech_step_backward",
    "grid_build_batched", "mech_step_batched", "mech_step_backward_batched", "integrate",
    "mech_step_backward_accumulate", "mech_step_backward_batched_accumulate", "MAX_BOXES",
    "mech_step_integrate_sorted", "mech_step_batched_integrate_sorted",
    "mech_step_integrate", "mech_step_batched_integrate",
    "reorder", "grid_info", "grid_get", "neighbors", "device_status", "copy_probe", "MechStepError",
    "params_tensor", "mech_step_noalloc",
]

_DTYPES = {
    "f32": (MS_F32, torch.float32, torch.float32),
    "f64": (MS_F64, torch.float64, torch.float64),
    "f32_pos64": (MS_F32_POS64, torch.float64, torch.float32),
}
PARAM_KEYS = ("kappa", "gamma", "dt", "max_disp", "adherence")
MAX_BOXES = 1 << 25   # boxes a build can hold over all its simulations


def _stream(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _params(p) -> _lib.ms_params:
    if isinstance(p, _lib.ms_params):
        return p
    return _lib.ms_params(*(float(p[k]) for k in PARAM_KEYS))


def params_tensor(plist, device) -> torch.Tensor:
    """Per-simulation parameters as a device float64 tensor [B, 5] (ms_params layout)."""
    rows = [[float(p[k]) for k in PARAM_KEYS] for p in plist]
    return torch.tensor(rows, dtype=torch.float64, device=device).contiguous()


class Workspace:
    """Device workspace of one grid (or one batch of grids).

    max_boxes defaults to 4 boxes per agent plus 4096 (at most MAX_BOXES =
    2^25, the most a build can hold), enough for the uniform and clustered
    populations of the benchmarks; a build that needs more reports
    MS_ECAPACITY through :func:`device_status`.
    """

    def __init__(self, max_agents: int, max_boxes: int | None = None, max_sims: int = 1,
                 dtype: str = "f32", device=None, keep_forces: bool = False,
                 gather_list: int = 0, gather_block: int = 0, box_order: str = "auto",
                 gather_walk: str = "lanes"):
        self.lib = _lib.load()
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be one of {list(_DTYPES)}")
        self.dtype_name = dtype
        self.code, self.in_dtype, self.out_dtype = _DTYPES[dtype]
        if max_boxes is None:
            max_boxes = min(4 * max(int(max_agents), 1) + 4096, MAX_BOXES)
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = self.lib.ms_workspace_bytes(int(max_agents), int(max_boxes), int(max_sims), self.code)
        if nbytes == 0:
            raise ValueError("invalid workspace capacities")
        self.buffer = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.c = _lib.ms_workspace()
        _lib.check(self.lib.ms_workspace_init(ctypes.byref(self.c), _ptr(self.buffer), int(nbytes),
                                              int(max_agents), int(max_boxes), int(max_sims),
                                              self.code, _stream(self.device)))
        self.keep_forces = keep_forces
        self.gather_list = gather_list
        self.gather_block = gather_block
        self.box_order = box_order
        self.gather_walk = gather_walk
        self.builds = 0   # grid builds issued on this workspace (the autograd layer checks it)

    @property
    def gather_list(self) -> int:
        """Contact-list length of the forward gather (0 = default 32, or 32 or
        40); results do not depend on it, speed does (see autotune)."""
        return int(self.c.gather_list)

    @gather_list.setter
    def gather_list(self, v: int):
        self.c.gather_list = int(v)

    @property
    def gather_block(self) -> int:
        """Threads per block of the forward gather (0 = default 64, or 64 or
        256); results do not depend on it, speed does (see autotune)."""
        return int(self.c.gather_block)

    @gather_block.setter
    def gather_block(self, v: int):
        self.c.gather_block = int(v)

    @property
    def sorted_input(self) -> bool:
        """Whether the next build takes its inputs as nearly box-sorted (set by
        the sorted-state step and reorder, cleared by every build; speed only)."""
        return bool(self.c.sorted_input)

    @sorted_input.setter
    def sorted_input(self, on: bool):
        self.c.sorted_input = 1 if on else 0

    _WALKS = {"lanes": 0, "planes": 1}

    @property
    def gather_walk(self) -> str:
        """How the gathers' lanes walk their 9 stencil runs: "lanes" (default;
        each lane all of its runs in turn) or "planes" (the z-planes
        together); results do not depend on it, speed does (see autotune)."""
        return {v: k for k, v in self._WALKS.items()}.get(int(self.c.gather_walk),
                                                          str(self.c.gather_walk))

    @gather_walk.setter
    def gather_walk(self, v: str):
        if v not in self._WALKS:
            raise ValueError(f"gather_walk must be one of {sorted(self._WALKS)}, not {v!r}")
        self.c.gather_walk = self._WALKS[v]

    _BOX_ORDERS = {"auto": 0, "rows": 1, "tiles": 2}

    @property
    def box_order(self) -> str:
        """Row order of the boxes of the single-simulation builds: "auto"
        (default; 16 x 16 tiles of rows once a z-plane holds many agents),
        "rows" (row-major) or "tiles".  Box ids, box starts and the slot
        order follow it; forces and displacements do not."""
        return {v: k for k, v in self._BOX_ORDERS.items()}.get(int(self.c.box_order),
                                                               str(self.c.box_order))

    @box_order.setter
    def box_order(self, v: str):
        if v not in self._BOX_ORDERS:
            raise ValueError(f"box_order must be one of {sorted(self._BOX_ORDERS)}, not {v!r}")
        self.c.box_order = self._BOX_ORDERS[v]

    @property
    def keep_forces(self) -> bool:
        """Whether mech_step keeps the forces for the next mech_step_backward
        on the same build and parameters (which then skips recomputing them)."""
        return bool(self.c.keep_forces)

    @keep_forces.setter
    def keep_forces(self, on: bool):
        self.c.keep_forces = 1 if on else 0

    @property
    def n_agents(self) -> int:
        return int(self.c.n_agents)

    @property
    def n_sims(self) -> int:
        return int(self.c.n_sims)

    @property
    def nbytes(self) -> int:
        return int(self.c.bytes)


class BatchSpec:
    """Simulation offsets of a batch: host copy (sizes) and device copy (kernels)."""

    def __init__(self, offsets, device=None, edges=None):
        off = torch.as_tensor(offsets, dtype=torch.int64).cpu().contiguous()
        self.offsets_host = off
        self.n_sims = int(off.numel() - 1)
        self.n_total = int(off[-1])
        dev = torch.device(device if device is not None else "cuda")
        self.offsets = off.to(dev)
        self.edges = None if edges is None else torch.as_tensor(edges, dtype=torch.float64).to(dev).contiguous()


def _check_in(ws: Workspace, *ts, n=None, dtype=None):
    dtype = dtype or ws.in_dtype
    for t in ts:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError("expected CUDA (HIP) tensors")
        if t.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {t.dtype}")
        if not t.is_contiguous() or t.dim() != 1:
            raise ValueError("expected contiguous 1-D tensors")
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} elements, got {t.numel()}")


def grid_build(ws: Workspace, x, y, z, d, edge: float = 0.0):
    """Uniform grid of the agents (Section IV-A); edge <= 0 uses the largest diameter."""
    n = x.numel()
    _check_in(ws, x, y, z, d, n=n)
    _lib.check(ws.lib.ms_grid_build(ctypes.byref(ws.c), _ptr(x), _ptr(y), _ptr(z), _ptr(d), n,
                                    float(edge), _stream(x.device)))
    ws.builds += 1


def _outs(ws, n, out, device):
    if out is None:
        return tuple(torch.empty(n, dtype=ws.out_dtype, device=device) for _ in range(3))
    _check_in(ws, *out, n=n, dtype=ws.out_dtype)
    return out


def mech_step(ws: Workspace, params, out=None):
    """Displacements (dx, dy, dz) of one step on the last plain build."""
    n = ws.n_agents
    dx, dy, dz = _outs(ws, n, out, ws.device)
    p = _params(params)
    _lib.check(ws.lib.ms_mech_step(ctypes.byref(ws.c), ctypes.byref(p), _ptr(dx), _ptr(dy), _ptr(dz),
                                   _stream(ws.device)))
    return dx, dy, dz


def mech_step_integrate(ws: Workspace, params, x, y, z, out=None):
    """One rollout step on the last plain build: the displacements are added
    to the positions x, y, z in place (bitwise as mech_step then integrate);
    out, when given, also receives (dx, dy, dz)."""
    n = ws.n_agents
    _check_in(ws, x, y, z, n=n)
    d = (None, None, None) if out is None else _outs(ws, n, out, ws.device)
    p = _params(params)
    _lib.check(ws.lib.ms_mech_step_integrate(ctypes.byref(ws.c), ctypes.byref(p), _ptr(x), _ptr(y),
                                             _ptr(z), *(_ptr(a) for a in d), _stream(ws.device)))
    return out


def _sorted_outs(ws, n, state_out, disp_out):
    if state_out is None:
        state_out = tuple(torch.empty(n, dtype=ws.in_dtype, device=ws.device) for _ in range(4))
    else:
        _check_in(ws, *state_out, n=n)
    d = (None, None, None) if disp_out is None else _outs(ws, n, disp_out, ws.device)
    return state_out, d


def mech_step_integrate_sorted(ws: Workspace, params, x, y, z, d, state_out=None, disp_out=None):
    """One rollout step on the box-sorted state: returns (x', y', z', d'), the
    positions after the step and the diameters in the slot order of the last
    plain build (renumbered as :func:`reorder` renumbers).  x, y, z, d are the
    build's inputs (read only in the mixed mode).  state_out / disp_out: optional
    preallocated outputs; disp_out receives the displacements in slot order."""
    n = ws.n_agents
    _check_in(ws, x, y, z, d, n=n)
    so, dd = _sorted_outs(ws, n, state_out, disp_out)
    p = _params(params)
    _lib.check(ws.lib.ms_mech_step_integrate_sorted(
        ctypes.byref(ws.c), ctypes.byref(p), *(_ptr(a) for a in (x, y, z, d)), *(_ptr(a) for a in so),
        *(_ptr(a) for a in dd), _stream(ws.device)))
    return so


def mech_step_batched_integrate_sorted(ws: Workspace, params_dev, x, y, z, d, state_out=None,
                                       disp_out=None):
    """mech_step_integrate_sorted for every simulation of the last batched build."""
    n = ws.n_agents
    if params_dev.shape != (ws.n_sims, 5) or params_dev.dtype != torch.float64:
        raise ValueError(f"params must be float64 [{ws.n_sims}, 5]")
    _check_in(ws, x, y, z, d, n=n)
    so, dd = _sorted_outs(ws, n, state_out, disp_out)
    _lib.check(ws.lib.ms_mech_step_batched_integrate_sorted(
        ctypes.byref(ws.c), _ptr(params_dev), *(_ptr(a) for a in (x, y, z, d)),
        *(_ptr(a) for a in so), *(_ptr(a) for a in dd), _stream(ws.device)))
    return so


def mech_step_backward(ws: Workspace, params, gdx, gdy, gdz, out=None, g_params=None):
    """(gx, gy, gz, gd, g_params[2]) = pullback of dL/dDelta through one step."""
    n = ws.n_agents
    _check_in(ws, gdx, gdy, gdz, n=n, dtype=ws.out_dtype)
    if out is None:
        out = tuple(torch.empty(n, dtype=ws.out_dtype, device=ws.device) for _ in range(4))
    if g_params is None:
        g_params = torch.empty(2, dtype=torch.float64, device=ws.device)
    gx, gy, gz, gd = out
    p = _params(params)
    _lib.check(ws.lib.ms_mech_step_backward(ctypes.byref(ws.c), ctypes.byref(p), _ptr(gdx), _ptr(gdy),
                                            _ptr(gdz), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gd),
                                            _ptr(g_params), _stream(ws.device)))
    return gx, gy, gz, gd, g_params


def mech_step_backward_accumulate(ws: Workspace, params, pbar, dbar, g_params):
    """One backward step of a rollout on the last plain build (of p_t):
    pbar = (pbx, pby, pbz) holds dL/dp_{t+1} and becomes dL/dp_t in place;
    dbar (dL/dd) and g_params (device float64 [2], dL/dkappa, dL/dgamma) are
    added to.  pbar and dbar have the positions' dtype."""
    n = ws.n_agents
    _check_in(ws, *pbar, dbar, n=n)
    _check_gp(g_params, 2)
    p = _params(params)
    _lib.check(ws.lib.ms_mech_step_backward_accumulate(ctypes.byref(ws.c), ctypes.byref(p),
                                                       *(_ptr(a) for a in pbar), _ptr(dbar),
                                                       _ptr(g_params), _stream(ws.device)))


def mech_step_backward_batched_accumulate(ws: Workspace, params_dev, pbar, dbar, g_params):
    """mech_step_backward_accumulate for every simulation of the last batched
    build; g_params: device float64 [B, 2] (or [2B]) added to."""
    n = ws.n_agents
    _check_in(ws, *pbar, dbar, n=n)
    if params_dev.shape != (ws.n_sims, 5) or params_dev.dtype != torch.float64:
        raise ValueError(f"params must be float64 [{ws.n_sims}, 5]")
    _check_gp(g_params, 2 * ws.n_sims)
    _lib.check(ws.lib.ms_mech_step_backward_batched_accumulate(
        ctypes.byref(ws.c), _ptr(params_dev), *(_ptr(a) for a in pbar), _ptr(dbar), _ptr(g_params),
        _stream(ws.device)))


def _check_gp(g, numel):
    if (not isinstance(g, torch.Tensor) or g.device.type != "cuda" or g.dtype != torch.float64
            or not g.is_contiguous() or g.numel() != numel):
        raise ValueError(f"g_params must be a contiguous float64 device tensor of {numel} elements")


def grid_build_batched(ws: Workspace, x, y, z, d, spec: BatchSpec):
    n = spec.n_total
    _check_in(ws, x, y, z, d, n=n)
    _lib.check(ws.lib.ms_grid_build_batched(ctypes.byref(ws.c), _ptr(x), _ptr(y), _ptr(z), _ptr(d),
                                            _ptr(spec.offsets), spec.n_sims, n, _ptr(spec.edges),
                                            _stream(x.device)))
    ws.builds += 1


def mech_step_batched(ws: Workspace, params_dev: torch.Tensor, out=None):
    """params_dev: float64 device tensor [B, 5] (see :func:`params_tensor`)."""
    n = ws.n_agents
    if params_dev.dtype != torch.float64 or params_dev.device.type != "cuda" or not params_dev.is_contiguous():
        raise TypeError("params must be a contiguous float64 device tensor [B, 5]")
    if params_dev.shape != (ws.n_sims, 5):
        raise ValueError(f"params must have shape ({ws.n_sims}, 5)")
    dx, dy, dz = _outs(ws, n, out, ws.device)
    _lib.check(ws.lib.ms_mech_step_batched(ctypes.byref(ws.c), _ptr(params_dev), _ptr(dx), _ptr(dy),
                                           _ptr(dz), _stream(ws.device)))
    return dx, dy, dz


def mech_step_batched_integrate(ws: Workspace, params_dev: torch.Tensor, x, y, z, out=None):
    """mech_step_integrate for every simulation of the last batched build."""
    n = ws.n_agents
    if params_dev.dtype != torch.float64 or params_dev.device.type != "cuda" or not params_dev.is_contiguous():
        raise TypeError("params must be a contiguous float64 device tensor [B, 5]")
    if params_dev.shape != (ws.n_sims, 5):
        raise ValueError(f"params must have shape ({ws.n_sims}, 5)")
    _check_in(ws, x, y, z, n=n)
    d = (None, None, None) if out is None else _outs(ws, n, out, ws.device)
    _lib.check(ws.lib.ms_mech_step_batched_integrate(
        ctypes.byref(ws.c), _ptr(params_dev), _ptr(x), _ptr(y), _ptr(z), *(_ptr(a) for a in d),
        _stream(ws.device)))
    return out


def mech_step_backward_batched(ws: Workspace, params_dev, gdx, gdy, gdz, out=None, g_params=None):
    n = ws.n_agents
    _check_in(ws, gdx, gdy, gdz, n=n, dtype=ws.out_dtype)
    if params_dev.shape != (ws.n_sims, 5) or params_dev.dtype != torch.float64:
        raise ValueError(f"params must be float64 [{ws.n_sims}, 5]")
    if out is None:
        out = tuple(torch.empty(n, dtype=ws.out_dtype, device=ws.device) for _ in range(4))
    if g_params is None:
        g_params = torch.empty(2 * ws.n_sims, dtype=torch.float64, device=ws.device)
    gx, gy, gz, gd = out
    _lib.check(ws.lib.ms_mech_step_backward_batched(ctypes.byref(ws.c), _ptr(params_dev), _ptr(gdx),
                                                    _ptr(gdy), _ptr(gdz), _ptr(gx), _ptr(gy), _ptr(gz),
                                                    _ptr(gd), _ptr(g_params), _stream(ws.device)))
    return gx, gy, gz, gd, g_params.view(ws.n_sims, 2)


def integrate(x, y, z, dx, dy, dz):
    """p <- p + Delta in place (FP64 positions with FP32 displacements allowed)."""
    n = x.numel()
    if x.dtype == torch.float32:
        code = MS_F32
    elif dx.dtype == torch.float64:
        code = MS_F64
    else:
        code = MS_F32_POS64
    lib = _lib.load()
    for t in (x, y, z, dx, dy, dz):
        if t.numel() != n or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError("integrate: contiguous device tensors of equal length required")
    _lib.check(lib.ms_integrate(_ptr(x), _ptr(y), _ptr(z), _ptr(dx), _ptr(dy), _ptr(dz), n, code,
                                _stream(x.device)))


def reorder(ws: Workspace, src, out=None):
    """out[k] = src[perm[k]]: a per-agent device tensor (1, 2, 4, 8 or
    16-byte elements) into the slot order of the last build (ascending box,
    x-quarter inside the box, input index).  Applied to every per-agent array
    it keeps a rollout's state box-sorted (ms_reorder)."""
    n = ws.n_agents
    if ws.c.built and (src.numel() != n or not src.is_contiguous() or src.device.type != "cuda"):
        raise ValueError("reorder: a contiguous device tensor of n_agents elements is required")
    if out is None:
        out = torch.empty_like(src)
    elif out.numel() != src.numel() or out.dtype != src.dtype or not out.is_contiguous():
        raise ValueError("reorder: out must match src")
    _lib.check(ws.lib.ms_reorder(ctypes.byref(ws.c), _ptr(src), _ptr(out), src.element_size(),
                                 _stream(ws.device)))
    return out


def grid_info(ws: Workspace):
    """Synchronising per-simulation geometry of the last build (origin, edge,
    dims, box count, box base, agent count, row tile shift), without copying
    any array."""
    B = max(ws.n_sims, 1)
    info = (_lib.ms_grid_info * B)()
    st = ws.lib.ms_grid_get(ctypes.byref(ws.c), info, None, None, None, _stream(ws.device))
    geo = [dict(origin=tuple(i.origin), edge=i.edge, dims=tuple(i.dims), error=i.error,
                n_boxes=i.n_boxes, box_base=i.box_base, n_agents=i.n_agents,
                tile_shift=i.tile_shift) for i in info]
    _lib.check(st)
    return geo


def grid_get(ws: Workspace):
    """Synchronising export of the last build: per-simulation geometry and the
    box index, box start and box-sorted order arrays (device int32 tensors)."""
    geo = grid_info(ws)
    n = ws.n_agents
    total = sum(g["n_boxes"] for g in geo)
    box = torch.empty(n, dtype=torch.int32, device=ws.device)
    start = torch.empty(total + 1, dtype=torch.int32, device=ws.device)
    perm = torch.empty(n, dtype=torch.int32, device=ws.device)
    _lib.check(ws.lib.ms_grid_get(ctypes.byref(ws.c), None, _ptr(box), _ptr(start), _ptr(perm),
                                  _stream(ws.device)))
    return dict(info=geo, box_id=box, start=start, perm=perm)


def neighbors(ws: Workspace):
    """(counts int32 [n], offsets int64 [n+1], list int32 [total]) of the last build."""
    n = ws.n_agents
    counts = torch.empty(max(n, 1), dtype=torch.int32, device=ws.device)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=ws.device)
    total = ctypes.c_int64(0)
    _lib.check(ws.lib.ms_neighbors(ctypes.byref(ws.c), _ptr(counts), _ptr(offsets), None, 0,
                                   ctypes.byref(total), _stream(ws.device)))
    lst = torch.empty(max(total.value, 1), dtype=torch.int32, device=ws.device)
    _lib.check(ws.lib.ms_neighbors(ctypes.byref(ws.c), _ptr(counts), _ptr(offsets), _ptr(lst),
                                   lst.numel(), ctypes.byref(total), _stream(ws.device)))
    return counts[:n], offsets, lst[: total.value]


def mech_step_noalloc(x, y, z, d, params, dtype: str = "f32", edge: float = 0.0, out=None,
                      dev_error=None):
    """Grid build + one step on the library's static workspace (no allocation
    inside the library; at most NOALLOC_MAX_AGENTS agents).  out: (dx, dy, dz)
    to fill, else allocated here; dev_error: None or a device int32 tensor of
    one element that receives the build's device error bits."""
    lib = _lib.load()
    if dtype not in _DTYPES:
        raise ValueError(f"dtype must be one of {list(_DTYPES)}")
    code, in_dtype, out_dtype = _DTYPES[dtype]
    n = int(x.numel())
    for t in (x, y, z, d):
        if t.dtype != in_dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"inputs must be contiguous {in_dtype} device tensors of equal length")
    if out is None:
        out = tuple(torch.empty(n, dtype=out_dtype, device=x.device) for _ in range(3))
    for t in out:
        if t.dtype != out_dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"outputs must be contiguous {out_dtype} device tensors of length n")
    if dev_error is not None and (dev_error.dtype != torch.int32 or not dev_error.is_cuda):
        raise ValueError("dev_error must be an int32 device tensor")
    p = _params(params)
    _lib.check(lib.ms_mech_step_noalloc(_ptr(x), _ptr(y), _ptr(z), _ptr(d), n, code, float(edge),
                                        ctypes.byref(p), *(_ptr(t) for t in out), _ptr(dev_error),
                                        _stream(x.device)))
    return out


def device_status(ws: Workspace):
    """Synchronise and raise MechStepError if the last build failed on the device."""
    _lib.check(ws.lib.ms_device_status(ctypes.byref(ws.c), _stream(ws.device)))


def copy_probe(dst: torch.Tensor, src: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    _lib.check(_lib.load().ms_copy_probe(_ptr(dst), _ptr(src), nbytes, _stream(src.device)))

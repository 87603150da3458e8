"""Seeded synthetic populations of spherical agents.

This module only draws inputs: agent positions, diameters, per-simulation force
coefficients and rollout targets. It holds none of the method's arithmetic (no
binning, no neighbour test, no force), so both the GPU path and the CPU oracle
can be fed from it without sharing any of the computation.

The paper measures on populations it generates itself (Section V): a cell
lattice that proliferates (benchmark A) and about two million agents at random
positions in a cube whose side is varied to set the mean number of neighbours
per agent (benchmark B, with the neighbour counts on the x-axis of the runtime
figure). The recipes below reproduce those shapes synthetically:

* ``lattice``   16^3 cubic lattice, spacing 9, coordinate jitter U(-0.5, 0.5),
                diameters U[9.5, 10.5] (the small deterministic analogue of the
                equal-volume cell grid of benchmark A).
* ``uniform``   N agents uniform in a cube [0, L]^3, diameters U[8, 12]; L is
                set so that the expected number of other agents within the
                interaction radius R = 12 equals ``mean_neighbors``
                (benchmark B's density sweep).
* ``clusters``  N agents from isotropic Gaussian clusters (sigma = 5% of the
                cube side) for highly uneven box occupancy.
* ``batched``   many independent uniform populations with log-uniform sizes,
                per-simulation densities and force coefficients.
* ``targets``   initial positions plus Gaussian noise, used as the regression
                target of a differentiable rollout.
* ``grow_and_divide``  a synthetic proliferation rule for variable
                populations (benchmark A's population grows by cell
                division; the simulator's own rules are not part of the
                paper): every diameter grows by a factor, agents above a
                threshold split into two daughters of half the volume placed
                symmetrically along a random direction.

Draw order with ``numpy.random.default_rng(seed)`` (PCG64): positions, then
diameters, then per-simulation parameters, then targets. FP32 inputs are the
FP64 draws rounded to nearest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Interaction radius used to define densities: the largest diameter drawn.
DENSITY_RADIUS = 12.0


def cube_side(n_agents: int, mean_neighbors: float, radius: float = DENSITY_RADIUS) -> float:
    """Side L of a cube holding ``n_agents`` uniformly so that a sphere of
    ``radius`` around an agent holds ``mean_neighbors`` others on average."""
    return (n_agents * (4.0 / 3.0) * math.pi * radius ** 3 / mean_neighbors) ** (1.0 / 3.0)


@dataclass
class Population:
    """One population in structure-of-arrays form (FP64 master copy)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    d: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self, dtype=np.float64):
        """(x, y, z, d) as contiguous arrays of ``dtype`` (RN rounding)."""
        return tuple(np.ascontiguousarray(a.astype(dtype)) for a in (self.x, self.y, self.z, self.d))


def lattice(side: int = 16, spacing: float = 9.0, jitter: float = 0.5,
            dmin: float = 9.5, dmax: float = 10.5, seed: int = 0) -> Population:
    rng = np.random.default_rng(seed)
    g = np.arange(side, dtype=np.float64) * spacing
    # x fastest, then y, then z
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    if jitter > 0:
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    d = rng.uniform(dmin, dmax, size=pos.shape[0])
    return Population(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), d,
                      name=f"lattice{side}^3", meta=dict(spacing=spacing, jitter=jitter))


def uniform(n: int, mean_neighbors: float | None = None, side: float | None = None,
            dmin: float = 8.0, dmax: float = 12.0, seed: int = 0) -> Population:
    if side is None:
        side = cube_side(n, mean_neighbors)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, size=(n, 3))
    d = rng.uniform(dmin, dmax, size=n)
    return Population(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), d,
                      name=f"uniform{n}", meta=dict(side=side, mean_neighbors=mean_neighbors))


def clusters(n: int, n_clusters: int = 64, side: float | None = None, sigma_frac: float = 0.05,
             dmin: float = 8.0, dmax: float = 12.0, seed: int = 0) -> Population:
    """Isotropic Gaussian clusters; centres U[0.15L, 0.85L]^3, sigma = sigma_frac * L.
    The default side is the uniform cube with 12 mean neighbours at this N."""
    if side is None:
        side = cube_side(n, 12.0)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15 * side, 0.85 * side, size=(n_clusters, 3))
    per = np.full(n_clusters, n // n_clusters)
    per[: n - per.sum()] += 1
    owner = np.repeat(np.arange(n_clusters), per)
    pos = centres[owner] + rng.normal(0.0, sigma_frac * side, size=(n, 3))
    d = rng.uniform(dmin, dmax, size=n)
    return Population(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), d,
                      name=f"clusters{n}", meta=dict(side=side, n_clusters=n_clusters))


@dataclass
class Batch:
    """Concatenated populations with ``offsets[b]:offsets[b+1]`` per simulation."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    d: np.ndarray
    offsets: np.ndarray          # int64 [B+1]
    kappa: np.ndarray            # [B]
    gamma: np.ndarray            # [B]
    meta: dict = field(default_factory=dict)

    @property
    def n_sims(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    def arrays(self, dtype=np.float64):
        return tuple(np.ascontiguousarray(a.astype(dtype)) for a in (self.x, self.y, self.z, self.d))

    def sim(self, b: int) -> Population:
        s, e = int(self.offsets[b]), int(self.offsets[b + 1])
        return Population(self.x[s:e].copy(), self.y[s:e].copy(), self.z[s:e].copy(), self.d[s:e].copy(),
                          name=f"sim{b}")


def batched(n_sims: int = 256, log10_min: float = 3.0, log10_max: float = 5.0,
            nbr_min: float = 4.0, nbr_max: float = 30.0, kappa_range=(1.0, 4.0),
            gamma_range=(0.5, 2.0), dmin: float = 8.0, dmax: float = 12.0, seed: int = 0) -> Batch:
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(log10_min, log10_max, size=n_sims)).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    nbrs = rng.uniform(nbr_min, nbr_max, size=n_sims)
    offsets = np.zeros(n_sims + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    pos = np.empty((n, 3))
    for b in range(n_sims):
        L = cube_side(int(sizes[b]), float(nbrs[b]))
        pos[offsets[b]:offsets[b + 1]] = rng.uniform(0.0, L, size=(int(sizes[b]), 3))
    d = rng.uniform(dmin, dmax, size=n)
    kappa = rng.uniform(*kappa_range, size=n_sims)
    gamma = rng.uniform(*gamma_range, size=n_sims)
    return Batch(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), d, offsets, kappa, gamma,
                 meta=dict(sizes=sizes, mean_neighbors=nbrs))


def targets(pop: Population, sigma: float = 1.0, seed: int = 0):
    """Rollout regression target: the initial positions plus N(0, sigma^2) noise.
    Uses its own stream (seed + 1000003) so the population draws are unchanged."""
    rng = np.random.default_rng(seed + 1000003)
    noise = rng.normal(0.0, sigma, size=(pop.n, 3))
    return pop.x + noise[:, 0], pop.y + noise[:, 1], pop.z + noise[:, 2]


def grow_and_divide(x, y, z, d, rng, growth: float = 1.02, d_max: float = 12.0):
    """One step of the synthetic proliferation rule on FP64 arrays: d *= growth;
    every agent with d > d_max divides.  The mother keeps its index and becomes
    daughter 1 at p + (d/4)u, daughter 2 is appended (in order of the mothers'
    indices) at p - (d/4)u, both with diameter d / 2^(1/3) (half the volume).
    u is a unit vector drawn from ``rng`` per dividing agent (normalised
    Gaussian triple)."""
    d = d * growth
    div = np.nonzero(d > d_max)[0]
    if div.size == 0:
        return x.copy(), y.copy(), z.copy(), d
    u = rng.normal(size=(div.size, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    off = (d[div] / 4.0)[:, None] * u
    dd = d[div] / 2.0 ** (1.0 / 3.0)
    x, y, z, d = x.copy(), y.copy(), z.copy(), d.copy()
    px, py, pz = x[div].copy(), y[div].copy(), z[div].copy()
    x[div], y[div], z[div], d[div] = px + off[:, 0], py + off[:, 1], pz + off[:, 2], dd
    return (np.concatenate([x, px - off[:, 0]]), np.concatenate([y, py - off[:, 1]]),
            np.concatenate([z, pz - off[:, 2]]), np.concatenate([d, dd]))


# Named workloads: the paper's benchmark shapes at the sizes measured here
# (2M uniform agents at several densities, 16.8M clustered, 256 simulations,
# 262,144 agents for the differentiated rollout).
DEFAULT_PARAMS = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)
FULL_N = 2_097_152


def workload(name: str, seed: int = 0):
    if name == "lattice4096":
        return lattice(seed=seed)
    if name.startswith("uniform2M_n"):
        nb = float(name.split("_n")[1])
        return uniform(FULL_N, mean_neighbors=nb, seed=seed)
    if name == "clusters16M":
        return clusters(16_777_216, seed=seed)
    if name == "batched256":
        return batched(seed=seed)
    if name == "adjoint262k":
        return uniform(262_144, mean_neighbors=12.0, seed=seed)
    raise KeyError(name)

"""Seeded synthetic inputs for the hybridized Q1-RT0-P0 poromechanics step.

This module is shared *as data* by the FP64 CPU oracle (``oracle/``) and the
HIP library (``paper_2002_09603_amd``).  It draws random fields and builds
node coordinates and problem descriptions; it holds none of the method's
arithmetic (no element integrals, no assembly, no solver).

Workload recipe (the paper's test problems are a unit cube cantilever and the
SPE10 reservoir; the SPE10 permeability data is not available, so seeded
log-normal and layered fields of the same size class stand in for it):

* ``unit8``      8x8x8 unit cube, isotropic log-normal kappa (ln 1e-3, sigma 1)
* ``cube64``     64^3, log-normal kappa sigma 2, nu 0.3, S_eps in {0, 1e-4}
* ``layered128`` 128^3, kxx=kyy=1e-2, kzz=1e-6 in even 8-cell layers,
                 isotropic 1e-6 in odd layers, times exp(N(0,1))
* ``perturbed96`` 96^3, nodes displaced by U(-0.2h, 0.2h) per component
                 (boundary-normal components kept), kappa sigma 1
* ``spe192``     192x192x96 on [0,2]x[0,2]x[0,1], kappa sigma 3,
                 E = 1e4 exp(0.5 N(0,1)), 20 geometric time steps 1e-3..1

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
Cell arrays are cell-lexicographic (i fastest, then j, then k); node arrays are
node-lexicographic with the same ordering.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

__all__ = [
    "Problem", "uniform_coords", "perturbed_coords", "lognormal_kappa",
    "layered_kappa", "lognormal_E", "observation_cells", "dt_schedule",
    "make_config", "CONFIG_NAMES",
]


@dataclass
class Problem:
    """Complete description of one backward-Euler step problem (data only).

    Boundary conditions, ``bc == "column"`` (all workloads): bottom face
    (z = z_min) displacement fixed; top face (z = z_max) loaded by ``traction``
    and drained (face pressure ``p_top``); all other boundary parts
    traction-free and no-flow.  ``rollers`` additionally fixes the normal
    displacement on the four lateral faces (one-dimensional consolidation).
    ``bc == "cantilever"``: face x = x_min fixed, top face loaded, no-flow
    everywhere (the paper's cantilever test).
    """
    name: str
    nx: int
    ny: int
    nz: int
    coords: np.ndarray                # (n_nodes, 3) float64
    E: np.ndarray                     # (n_cells,) float64, Young's modulus
    kappa: np.ndarray                 # (n_cells, 3) float64, diagonal permeability
    nu: float = 0.25
    biot: float = 1.0
    S_eps: float = 0.0
    mu: float = 1.0
    dt: float = 1e-2
    traction: tuple = (0.0, 0.0, -1.0)
    p_top: float = 0.0
    rollers: bool = False
    bc: str = "column"                # "column" or "cantilever"
    stabilize: bool = True
    dts: Optional[np.ndarray] = None  # multi-step schedule (None: one step)
    obs_cells: Optional[np.ndarray] = None
    fd_cells: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_faces(self) -> int:
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)

    @property
    def n_total(self) -> int:
        return 3 * self.n_nodes + self.n_cells + self.n_faces

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def uniform_coords(nx: int, ny: int, nz: int, Lx: float = 1.0, Ly: float = 1.0,
                   Lz: float = 1.0) -> np.ndarray:
    """Node coordinates of the uniform box [0,Lx]x[0,Ly]x[0,Lz]."""
    x = np.linspace(0.0, Lx, nx + 1)
    y = np.linspace(0.0, Ly, ny + 1)
    z = np.linspace(0.0, Lz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)


def perturbed_coords(nx: int, ny: int, nz: int, seed: int, amp: float = 0.2,
                     Lx: float = 1.0, Ly: float = 1.0, Lz: float = 1.0) -> np.ndarray:
    """Uniform box nodes displaced by U(-amp*h, amp*h) per component.

    The component normal to a boundary plane is left unperturbed on nodes of
    that plane, so the six sides stay planar.  Draw order: one
    ``uniform(size=(n_nodes, 3))`` call, node-lexicographic.
    """
    X = uniform_coords(nx, ny, nz, Lx, Ly, Lz)
    h = np.array([Lx / nx, Ly / ny, Lz / nz])
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, size=X.shape) * (amp * h)[None, :]
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    d[(i == 0) | (i == nx), 0] = 0.0
    d[(j == 0) | (j == ny), 1] = 0.0
    d[(k == 0) | (k == nz), 2] = 0.0
    return X + d


def lognormal_kappa(n_cells: int, sigma: float, seed: int, base: float = 1e-3) -> np.ndarray:
    """Isotropic per-cell permeability base*exp(sigma*xi), xi ~ N(0,1)."""
    xi = np.random.default_rng(seed).standard_normal(n_cells)
    k = base * np.exp(sigma * xi)
    return np.repeat(k[:, None], 3, axis=1)


def layered_kappa(nx: int, ny: int, nz: int, sigma: float, seed: int,
                  layer: int = 8) -> np.ndarray:
    """Alternating layers of ``layer`` cells in z: even layers
    diag(1e-2, 1e-2, 1e-6), odd layers isotropic 1e-6; every component of a
    cell is multiplied by the same exp(sigma*xi), xi ~ N(0,1)."""
    n = nx * ny * nz
    xi = np.random.default_rng(seed).standard_normal(n)
    kcell = np.repeat(np.arange(nz), nx * ny)
    even = (kcell // layer) % 2 == 0
    K = np.empty((n, 3))
    K[even] = (1e-2, 1e-2, 1e-6)
    K[~even] = (1e-6, 1e-6, 1e-6)
    return K * np.exp(sigma * xi)[:, None]


def lognormal_E(n_cells: int, sigma: float, seed: int, base: float = 1e4) -> np.ndarray:
    xi = np.random.default_rng(seed).standard_normal(n_cells)
    return base * np.exp(sigma * xi)


def observation_cells(n_cells: int, count: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(n_cells, count, replace=False)).astype(np.int64)


def dt_schedule(n_steps: int = 20, first: float = 1e-3, last: float = 1.0) -> np.ndarray:
    """Geometric time-step sizes from ``first`` to ``last`` inclusive."""
    if n_steps == 1:
        return np.array([first])
    return first * (last / first) ** (np.arange(n_steps) / (n_steps - 1))


CONFIG_NAMES = ("unit8", "cube64", "layered128", "perturbed96", "spe192")

# Fixed seeds of the workloads (one per random field).
SEEDS = {"unit8": 8, "cube64": 64, "layered128": 128, "perturbed96": 96, "spe192": 192}


def make_config(name: str, n: Optional[int] = None, S_eps: float = 0.0,
                seed: Optional[int] = None) -> Problem:
    """Build one named workload.  ``n`` overrides the cells per axis (the
    shape rules of the workload are kept), for reduced-size parity cases."""
    s = SEEDS[name] if seed is None else seed
    if name == "unit8":
        m = 8 if n is None else n
        nc = m ** 3
        return Problem(name, m, m, m, uniform_coords(m, m, m), np.full(nc, 1e4),
                       lognormal_kappa(nc, 1.0, s), nu=0.25, S_eps=0.0, dt=1e-2)
    if name == "cube64":
        m = 64 if n is None else n
        nc = m ** 3
        return Problem(name, m, m, m, uniform_coords(m, m, m), np.full(nc, 1e4),
                       lognormal_kappa(nc, 2.0, s), nu=0.3, S_eps=S_eps, dt=1e-2)
    if name == "layered128":
        m = 128 if n is None else n
        nc = m ** 3
        return Problem(name, m, m, m, uniform_coords(m, m, m), np.full(nc, 1e4),
                       layered_kappa(m, m, m, 1.0, s), nu=0.25, S_eps=0.0, dt=1e-2)
    if name == "perturbed96":
        m = 96 if n is None else n
        nc = m ** 3
        return Problem(name, m, m, m, perturbed_coords(m, m, m, s), np.full(nc, 1e4),
                       lognormal_kappa(nc, 1.0, s + 1), nu=0.25, S_eps=0.0, dt=1e-2,
                       obs_cells=observation_cells(nc, min(64, nc), s + 2),
                       fd_cells=observation_cells(nc, min(16, nc), s + 3))
    if name == "spe192":
        if n is None:
            nx, ny, nz = 192, 192, 96
        else:
            nx, ny, nz = 2 * n, 2 * n, n
        nc = nx * ny * nz
        return Problem(name, nx, ny, nz, uniform_coords(nx, ny, nz, 2.0, 2.0, 1.0),
                       lognormal_E(nc, 0.5, s + 1), lognormal_kappa(nc, 3.0, s),
                       nu=0.25, S_eps=0.0, dt=1e-3, dts=dt_schedule(20),
                       obs_cells=observation_cells(nc, min(64, nc), s + 2))
    raise KeyError(name)


def cantilever(n: int, dt: float, stabilize: bool = True) -> Problem:
    """The paper's 3D cantilever (Sec. 5.2): unit cube, E = 1e5, nu = 0.4,
    b = 1, S_eps = 0, kappa = 1e-7, mu = 1e-3, face x=0 fixed, no-flow
    everywhere, unit load on the top face."""
    nc = n ** 3
    return Problem("cantilever", n, n, n, uniform_coords(n, n, n), np.full(nc, 1e5),
                   np.full((nc, 3), 1e-7), nu=0.4, biot=1.0, S_eps=0.0, mu=1e-3,
                   dt=dt, bc="cantilever", stabilize=stabilize)

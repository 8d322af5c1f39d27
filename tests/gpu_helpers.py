"""Shared helpers of the GPU parity tests (oracle side on the CPU, HIP side
through the C ABI binding)."""
import numpy as np

from synth import Problem, uniform_coords, perturbed_coords


def graded_coords(nx, ny, nz, ratio=1.15):
    """Axis-aligned box on [0,1]^3 whose x spacing grows geometrically by
    ``ratio`` (cells are boxes but not translates of one another)."""
    X = uniform_coords(nx, ny, nz)
    xs = (ratio ** np.arange(nx + 1) - 1.0) / (ratio ** nx - 1.0)
    X[:, 0] = xs[np.rint(X[:, 0] * nx).astype(int)]
    return X


def box_problem(nx, ny, nz, seed=0, perturb=False, S_eps=0.0, nu=0.25, dt=1e-2, sigma_k=1.0,
                sigma_E=0.3, p_top=0.0, rollers=False, stabilize=True, bc="column", graded=False):
    """Seeded non-cubic box with log-normal E and anisotropic diagonal kappa
    (bc "column": bottom fixed, top drained; "cantilever": face x = 0 fixed,
    no-flow everywhere; graded: geometric spacing in x)."""
    rng = np.random.default_rng(seed)
    nc = nx * ny * nz
    coords = (perturbed_coords(nx, ny, nz, seed + 1) if perturb else
              (graded_coords(nx, ny, nz) if graded else uniform_coords(nx, ny, nz)))
    E = 1e4 * np.exp(sigma_E * rng.standard_normal(nc))
    kappa = 1e-3 * np.exp(sigma_k * rng.standard_normal((nc, 3)))
    return Problem("box", nx, ny, nz, coords, E, kappa, nu=nu, S_eps=S_eps, dt=dt, p_top=p_top,
                   rollers=rollers, stabilize=stabilize, bc=bc)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)

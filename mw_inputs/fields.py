"""Seeded permittivity maps on the tetrahedra (piecewise constant, one value
per tetrahedron) and seeded source points.

Time convention e^{+i omega t}: lossy media have Im eps_r < 0 (the gel of the
paper is 44 - 20i).
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh, tet_centroids


def homogeneous(mesh: Mesh, eps: complex) -> np.ndarray:
    return np.full(mesh.nt, complex(eps), dtype=np.complex128)


def gaussian_field(points: np.ndarray, corr_len: float, seed: int, n_modes: int = 256) -> np.ndarray:
    """Unit-variance smooth random field by random Fourier features:
    g(x) = sqrt(2/M) sum_m cos(w_m . x + b_m), w_m ~ N(0, corr_len^-2 I),
    b_m ~ U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, 1.0 / corr_len, size=(n_modes, 3))
    b = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return np.sqrt(2.0 / n_modes) * np.cos(points @ w.T + b).sum(axis=1)


def chamber_phantom(mesh: Mesh, eps_gel: complex = 44 - 20j, eps_obj: complex = 45 - 25j,
                    centre=(0.0, 0.0, 0.14), semi_axes=(0.09, 0.07, 0.10),
                    sigma: float = 0.05, corr_len: float = 0.02, seed: int = 2) -> np.ndarray:
    """Gel background with a centred ellipsoid whose permittivity carries a
    multiplicative smooth random perturbation (1 + sigma g)."""
    c = tet_centroids(mesh)
    eps = homogeneous(mesh, eps_gel)
    q = (((c - np.asarray(centre)) / np.asarray(semi_axes)) ** 2).sum(axis=1)
    inside = q <= 1.0
    g = gaussian_field(c[inside], corr_len, seed)
    eps[inside] = complex(eps_obj) * (1.0 + sigma * g)
    return eps


def add_inclusion(mesh: Mesh, eps: np.ndarray, centre=(0.03, 0.0, 0.14), radius: float = 0.01,
                  real_factor: float = 1.2) -> np.ndarray:
    """Spherical inclusion: Re eps scaled by ``real_factor``, Im eps unchanged."""
    c = tet_centroids(mesh)
    inside = ((c - np.asarray(centre)) ** 2).sum(axis=1) <= radius * radius
    out = eps.copy()
    out[inside] = out[inside].real * real_factor + 1j * out[inside].imag
    return out


def tets_near(mesh: Mesh, centre, radius: float) -> np.ndarray:
    c = tet_centroids(mesh)
    return np.nonzero(((c - np.asarray(centre)) ** 2).sum(axis=1) <= radius * radius)[0]


def dipole_points(n: int, seed: int = 0, lo: float = 0.125, hi: float = 0.875) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, (n, 3))

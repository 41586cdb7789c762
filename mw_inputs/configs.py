"""Named synthetic workloads.

cube8      : unit cube, 8^3 cells (3072 tets, 4184 edges), eps_r = 1 - 0.1i,
             k0 = 4 pi, impedance on every face, 4 unit z-dipoles at seeded
             interior points, 8 subdomains, overlap 1, GMRES(30), tol 1e-10.
chamber05  : imaging chamber r = 0.15 m, H = 0.28 m at 0.5 GHz, 10 points per
             gel wavelength (~214k edges); gel 44 - 20i with a centred
             ellipsoid 45 - 25i carrying a 5 % smooth random perturbation;
             32 ports on the ring z = 0.14 m; 64 subdomains; FP64.
chamber10  : same chamber at 1 GHz (~1.64M edges), 160 ports on 5 rings,
             1600 subdomains (at most ~4k local unknowns each); mixed vs FP64.
inversion05: chamber05 mesh, 'measured' S from the map plus a 1 cm spherical
             inclusion (Re eps x 1.2), forward + adjoint on 32 ports.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields, mesh as meshmod, partition

C0 = meshmod.C0


@dataclass
class Workload:
    name: str
    mesh: meshmod.Mesh
    eps: np.ndarray           # complex128 [nt]
    k0: float
    beta_imp: complex         # impedance coefficient on TAG_IMPEDANCE faces
    ports: list               # PortSpec list (port k <-> btag k+1)
    n_sub: int
    part: np.ndarray          # int32 [nt]
    overlap: int = 1
    restart: int = 30
    tol: float = 1e-8
    dipoles: np.ndarray | None = None      # [np, 3] points (z-directed)
    tx: np.ndarray | None = None           # transmitting port indices
    rx: np.ndarray | None = None           # receiving port indices
    extra: dict = field(default_factory=dict)

    @property
    def nrhs(self) -> int:
        if self.dipoles is not None:
            return int(self.dipoles.shape[0])
        return int(len(self.tx))


def k0_of(freq_hz: float) -> float:
    return 2.0 * np.pi * freq_hz / C0


def cube(n: int = 8, eps: complex = 1 - 0.1j, k0: float = 4 * np.pi, n_sub: int = 8,
         ndip: int = 4, seed: int = 0, tol: float = 1e-10, restart: int = 30) -> Workload:
    m = meshmod.cube_mesh(n)
    e = fields.homogeneous(m, eps)
    beta = k0 * np.sqrt(complex(eps))
    part = partition.rcb(m, n_sub)
    dip = fields.dipole_points(ndip, seed)
    return Workload(name=f"cube{n}", mesh=m, eps=e, k0=k0, beta_imp=beta, ports=[], n_sub=n_sub,
                    part=part, tol=tol, restart=restart, dipoles=dip)


def chamber(freq_hz: float, rings=(0.14,), n_per_ring: int = 32, n_sub: int = 64,
            eps_gel: complex = 44 - 20j, phantom: bool = True, tol: float = 1e-8,
            restart: int = 30, port_size: float = 0.026, radius: float = 0.15,
            height: float = 0.28, ppw: float = 10.0, name: str | None = None) -> Workload:
    k0 = k0_of(freq_hz)
    beta = k0 * np.sqrt(complex(eps_gel))
    ports = meshmod.chamber_ports(n_per_ring, rings, port_size, port_size, radius, beta)
    m = meshmod.cylinder_mesh(freq_hz, radius, height, eps_gel, ppw, ports)
    e = fields.chamber_phantom(m, eps_gel) if phantom else fields.homogeneous(m, eps_gel)
    part = partition.rcb(m, n_sub)
    allp = np.arange(len(ports), dtype=np.int32)
    return Workload(name=name or f"chamber{freq_hz / 1e9:g}GHz", mesh=m, eps=e, k0=k0,
                    beta_imp=beta, ports=ports, n_sub=n_sub, part=part, tol=tol,
                    restart=restart, tx=allp.copy(), rx=allp.copy())


def cube8() -> Workload:
    return cube(8)


def chamber05(n_sub: int = 64) -> Workload:
    return chamber(0.5e9, rings=(0.14,), n_sub=n_sub, name="chamber05")


def chamber10(n_sub: int = 1600) -> Workload:
    return chamber(1.0e9, rings=(0.06, 0.10, 0.14, 0.18, 0.22), n_sub=n_sub, name="chamber10")


def inversion05(n_sub: int = 64) -> Workload:
    w = chamber05(n_sub)
    true_eps = fields.add_inclusion(w.mesh, w.eps)
    near = fields.tets_near(w.mesh, (0.03, 0.0, 0.14), 0.03)
    fd = np.sort(np.random.default_rng(4).choice(near, size=20, replace=False))
    w.name = "inversion05"
    w.extra = {"eps_true": true_eps, "fd_tets": fd}
    return w


def small_chamber(freq_hz: float = 0.25e9, n_per_ring: int = 8, n_sub: int = 8, rings=(0.14,),
                  tol: float = 1e-10) -> Workload:
    """Coarse chamber used where the oracle must run a sparse direct solve in
    seconds (same geometry and labels, fewer cells)."""
    return chamber(freq_hz, rings=rings, n_per_ring=n_per_ring, n_sub=n_sub, tol=tol,
                   name=f"chamber{freq_hz / 1e9:g}GHz_small")

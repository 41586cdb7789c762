"""Seeded inputs of the serving workload: a menu of chamber problems and a
Poisson stream of requests against it.

Menu: the imaging chamber meshed at 0.3125, 0.5, 0.75 and 1 GHz (10 points
per gel wavelength; about 50k, 214k, 690k and 1.64M edges), 160 ports on 5
rings, two permittivity versions per mesh (the phantom map, and the map with
a 1 cm inclusion), ceil(edges / 1000) subdomains.

Requests: arrival times of a Poisson process (rate 4 per second), 400
requests, 75 % field solves and 25 % misfit-gradient evaluations; the number
of right-hand sides is a log-uniform integer in [1, 160] for solves and in
[1, 32] for gradients; the transmitting ports are a uniform random subset;
the mesh and the permittivity version are uniform random choices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import configs, fields, partition

SERVE_FREQS = (0.3125e9, 0.5e9, 0.75e9, 1.0e9)
RINGS5 = (0.06, 0.10, 0.14, 0.18, 0.22)


def count_edges(tet: np.ndarray) -> int:
    """Distinct vertex pairs of the tetrahedra (mesh size in edges)."""
    t = np.sort(np.asarray(tet, dtype=np.int64), axis=1)
    pairs = np.concatenate([t[:, [a, b]] for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))])
    key = pairs[:, 0] * (int(t.max()) + 1) + pairs[:, 1]
    return int(np.unique(key).size)


@dataclass
class MenuEntry:
    name: str
    workload: configs.Workload      # mesh, ports, partition, version-0 permittivity
    eps_versions: list              # complex128 [nt] per version
    n_edges: int


def serving_menu(freqs=SERVE_FREQS, rings=RINGS5, n_per_ring: int = 32, edges_per_sub: int = 1000,
                 tol: float = 1e-8) -> list[MenuEntry]:
    menu = []
    for f in freqs:
        w = configs.chamber(f, rings=rings, n_per_ring=n_per_ring, n_sub=1, tol=tol, name=f"serve{f / 1e9:g}GHz")
        ne = count_edges(w.mesh.tet)
        w.n_sub = int(np.ceil(ne / edges_per_sub))
        w.part = partition.rcb(w.mesh, w.n_sub)
        menu.append(MenuEntry(w.name, w, [w.eps, fields.add_inclusion(w.mesh, w.eps)], ne))
    return menu


@dataclass
class Request:
    rid: int
    t_arrive: float        # seconds after the start of the stream
    mesh: int              # menu index
    version: int           # permittivity version
    kind: str              # "solve" | "gradient"
    tx: np.ndarray         # int32 transmitting ports (one right-hand side each)
    rx: np.ndarray         # int32 receiving ports (gradient: S rows)
    s_meas: np.ndarray | None = None   # complex128 [len(rx), len(tx)] (gradient)

    @property
    def ncols(self) -> int:
        return int(self.tx.size)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, size: int) -> np.ndarray:
    u = rng.uniform(np.log(lo), np.log(hi + 1), size)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def serving_requests(n_req: int = 400, rate: float = 4.0, seed: int = 5, n_meshes: int = 4,
                     n_versions: int = 2, nports: int = 160, max_solve: int = 160, max_grad: int = 32,
                     p_grad: float = 0.25) -> list[Request]:
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_req))
    is_grad = rng.random(n_req) < p_grad
    mesh = rng.integers(0, n_meshes, n_req)
    ver = rng.integers(0, n_versions, n_req)
    ns = log_uniform_int(rng, 1, max_solve, n_req)
    ng = log_uniform_int(rng, 1, max_grad, n_req)
    out = []
    allp = np.arange(nports, dtype=np.int32)
    for k in range(n_req):
        nc = int(ng[k] if is_grad[k] else ns[k])
        tx = np.sort(rng.choice(nports, size=nc, replace=False)).astype(np.int32)
        if is_grad[k]:
            sm = 0.01 * (rng.standard_normal((nports, nc)) + 1j * rng.standard_normal((nports, nc)))
            out.append(Request(k, float(t[k]), int(mesh[k]), int(ver[k]), "gradient", tx, allp.copy(), sm))
        else:
            out.append(Request(k, float(t[k]), int(mesh[k]), int(ver[k]), "solve", tx, allp.copy()))
    return out

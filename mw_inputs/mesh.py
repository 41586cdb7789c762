"""Seeded synthetic tetrahedral meshes of the paper's geometries.

The imaging chamber of the paper (a metallic cylinder filled with a matching
gel, antennas on its lateral wall, metallic bottom, impedance condition on the
top; Section 2 and the description of the EMTensor chamber) and a unit cube
used for the small checks.

Every mesh is a Kuhn (Freudenthal) split of a structured grid: each cube cell
with lower corner c is cut into the 6 tetrahedra
(c, c+e_p0, c+e_p0+e_p1, c+(1,1,1)) for the 6 axis permutations p, which is a
conforming triangulation.  Tetrahedra list their vertices in ascending global
order.  This module only builds geometry and boundary labels; it holds none of
the finite-element arithmetic.

Boundary labels (``btag``):
  * ``TAG_PEC`` (-1): perfectly conducting wall,
  * ``TAG_IMPEDANCE`` (0): first-order impedance (absorbing) boundary,
  * ``k >= 1``: aperture of antenna port ``k - 1``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TAG_PEC = -1
TAG_IMPEDANCE = 0

C0 = 299792458.0

# the six axis permutations of the Kuhn split
_PERMS = np.array([[0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]])


@dataclass
class Mesh:
    xyz: np.ndarray          # float64 [nv, 3]
    tet: np.ndarray          # int32 [nt, 4], ascending vertex ids
    bface: np.ndarray        # int32 [nbf, 3], ascending vertex ids
    btag: np.ndarray         # int32 [nbf]
    cell_of_tet: np.ndarray  # int32 [nt], structured cell index (for partitioning)
    cell_ijk: np.ndarray     # int32 [ncell, 3], integer cell coordinates
    info: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tet.shape[0])


def _kuhn_tets(cells: np.ndarray, vid) -> np.ndarray:
    """cells: int [nc, 3] lower corners; vid(i, j, k) -> vertex id arrays."""
    out = np.empty((cells.shape[0], 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        c = cells.copy()
        out[:, p, 0] = vid(c)
        c = c.copy()
        c[:, perm[0]] += 1
        out[:, p, 1] = vid(c)
        c = c.copy()
        c[:, perm[1]] += 1
        out[:, p, 2] = vid(c)
        out[:, p, 3] = vid(cells + 1)
    return out.reshape(-1, 4)


def _boundary_faces(tet: np.ndarray) -> np.ndarray:
    """Faces (ascending triples) that belong to exactly one tetrahedron."""
    f = np.concatenate([tet[:, [0, 1, 2]], tet[:, [0, 1, 3]],
                        tet[:, [0, 2, 3]], tet[:, [1, 2, 3]]])
    f = np.sort(f, axis=1)
    uniq, cnt = np.unique(f, axis=0, return_counts=True)
    return uniq[cnt == 1].astype(np.int32)


def cube_mesh(n: int, length: float = 1.0) -> Mesh:
    """Unit cube [0, length]^3 cut into n^3 cells, 6 tets each.

    Every boundary face is an impedance face.
    """
    npt = n + 1
    g = np.arange(npt) * (length / n)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(c):
        return (c[:, 0] * npt + c[:, 1]) * npt + c[:, 2]

    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    tet = np.sort(_kuhn_tets(cells, vid), axis=1).astype(np.int32)
    bface = _boundary_faces(tet)
    btag = np.full(bface.shape[0], TAG_IMPEDANCE, dtype=np.int32)
    cell_of_tet = np.repeat(np.arange(cells.shape[0]), 6).astype(np.int32)
    return Mesh(xyz=xyz, tet=tet, bface=bface, btag=btag, cell_of_tet=cell_of_tet,
                cell_ijk=cells.astype(np.int32), info={"kind": "cube", "n": n, "length": length})


@dataclass
class PortSpec:
    """Rectangular antenna aperture on the lateral wall of the chamber.

    The incident field is the TE10-like profile  pol * cos(pi * s / width),
    s = radius * wrap(atan2(y, x) - theta), on faces tagged with this port.
    """
    theta: float
    z: float
    width: float
    height: float
    radius: float
    beta: complex
    pol: tuple = (0.0, 0.0, 1.0)


def chamber_ports(n_per_ring: int, ring_z, width: float, height: float,
                  radius: float, beta: complex):
    ports = []
    for z in ring_z:
        for i in range(n_per_ring):
            ports.append(PortSpec(theta=2.0 * np.pi * i / n_per_ring, z=float(z), width=width,
                                  height=height, radius=radius, beta=complex(beta)))
    return ports


def gel_wavelength(freq_hz: float, eps_gel: complex) -> float:
    return C0 / (freq_hz * np.sqrt(complex(eps_gel)).real)


def cylinder_mesh(freq_hz: float, radius: float = 0.15, height: float = 0.28,
                  eps_gel: complex = 44 - 20j, ppw: float = 10.0, ports=None) -> Mesh:
    """Staircase cylinder of the imaging chamber at about ``ppw`` points per
    wavelength of the gel.

    Cells of a (nxy x nxy x nz) grid over [-r, r]^2 x [0, H] are kept when the
    (x, y) centre of the cell lies inside the circle of radius r.  The bottom
    is PEC, the top an impedance face, the lateral wall PEC except on port
    apertures (a face belongs to port k when its centroid lies within the
    port's (arc, z) rectangle).
    """
    hmesh = gel_wavelength(freq_hz, eps_gel) / ppw
    nxy = int(np.ceil(2.0 * radius / hmesh))
    nz = int(round(height / hmesh))
    dx = 2.0 * radius / nxy
    dz = height / nz
    ii, jj, kk = np.meshgrid(np.arange(nxy), np.arange(nxy), np.arange(nz), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    cx = -radius + (cells[:, 0] + 0.5) * dx
    cy = -radius + (cells[:, 1] + 0.5) * dx
    keep = cx * cx + cy * cy < radius * radius
    cells = cells[keep]
    npt_xy = nxy + 1
    npt_z = nz + 1

    def vid_full(c):
        return (c[:, 0] * npt_xy + c[:, 1]) * npt_z + c[:, 2]

    tet_full = _kuhn_tets(cells, vid_full)
    used, tet_c = np.unique(tet_full.ravel(), return_inverse=True)
    tet = np.sort(tet_c.reshape(-1, 4), axis=1).astype(np.int32)
    vi = used // (npt_xy * npt_z)
    vj = (used // npt_z) % npt_xy
    vk = used % npt_z
    xyz = np.stack([-radius + vi * dx, -radius + vj * dx, vk * dz], axis=1)

    bface = _boundary_faces(tet)
    p = xyz[bface]                     # [nbf, 3, 3]
    cen = p.mean(axis=1)
    zmin = p[:, :, 2].min(axis=1)
    zmax = p[:, :, 2].max(axis=1)
    btag = np.full(bface.shape[0], TAG_PEC, dtype=np.int32)
    flat = zmax - zmin < 1e-12 * height
    top = flat & (np.abs(zmin - height) < 1e-9 * height)
    btag[top] = TAG_IMPEDANCE
    lateral = ~flat
    if ports:
        phi = np.arctan2(cen[:, 1], cen[:, 0])
        for k, pt in enumerate(ports):
            d = np.angle(np.exp(1j * (phi - pt.theta)))
            s = pt.radius * d
            inside = lateral & (np.abs(s) <= 0.5 * pt.width) & (np.abs(cen[:, 2] - pt.z) <= 0.5 * pt.height)
            btag[inside] = k + 1
    cell_of_tet = np.repeat(np.arange(cells.shape[0]), 6).astype(np.int32)
    info = {"kind": "cylinder", "freq_hz": freq_hz, "radius": radius, "height": height,
            "h": hmesh, "nxy": nxy, "nz": nz, "eps_gel": complex(eps_gel)}
    return Mesh(xyz=xyz, tet=tet, bface=bface, btag=btag, cell_of_tet=cell_of_tet,
                cell_ijk=cells.astype(np.int32), info=info)


def tet_centroids(mesh: Mesh) -> np.ndarray:
    return mesh.xyz[mesh.tet].mean(axis=1)

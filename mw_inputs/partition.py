"""Non-overlapping partition of the tetrahedra into subdomains.

The paper partitions with a graph partitioner (SCOTCH or METIS); the method
only needs some non-overlapping partition.  This stand-in is recursive
coordinate bisection on the structured cells (the 6 tetrahedra of a cell stay
together): split the current set of cells along the axis of largest integer
extent, at the count that matches the requested part ratio.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


def rcb_cells(ijk: np.ndarray, nparts: int) -> np.ndarray:
    part = np.zeros(ijk.shape[0], dtype=np.int32)

    def rec(idx: np.ndarray, p0: int, np_: int):
        if np_ == 1:
            part[idx] = p0
            return
        pts = ijk[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        ax = int(np.argmax(ext))          # ties -> lowest axis
        nl = np_ // 2
        order = np.lexsort((pts[:, (ax + 2) % 3], pts[:, (ax + 1) % 3], pts[:, ax]))
        cut = int(round(idx.size * nl / np_))
        rec(idx[order[:cut]], p0, nl)
        rec(idx[order[cut:]], p0 + nl, np_ - nl)

    rec(np.arange(ijk.shape[0]), 0, nparts)
    return part


def rcb(mesh: Mesh, nparts: int) -> np.ndarray:
    """int32 [nt] subdomain id of every tetrahedron."""
    cpart = rcb_cells(mesh.cell_ijk, nparts)
    return cpart[mesh.cell_of_tet].astype(np.int32)

"""Oracle: one-level Optimized Restricted Additive Schwarz (ORAS), plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Follows Section 3 of the paper:
  * overlapping decomposition: T_i^d = T_i^{d-1} plus the tetrahedra adjacent
    to it; "adjacent" is read as "sharing a vertex" (the only reading under
    which the support of the P1 function chi~_i stays inside T_i^d);
  * R_i: Boolean restriction to the non-PEC edges of T_i^d (ascending ids);
  * partition of unity, equations (algebPartUnity) and (chi): chi~_i = 1 at
    the nodes of T_i^0 and 0 at the other nodes of T_i^d,
    chi_i = chi~_i / sum_j chi~_j, and D_i[e] = chi_i at the midpoint of e,
    i.e. the mean of the values at its two end nodes;
  * B_i: the Maxwell operator assembled from the tetrahedra of T_i^d only,
    with the physical boundary terms of faces owned by those tetrahedra and
    an impedance transmission term i k int (E x n).(v x n) on the faces of
    T_i^d that are neither shared by two of its tetrahedra nor on the
    physical boundary; k = k0 sqrt(Re eps_r) of the tetrahedron owning the
    face (the paper's k = omega sqrt(mu0 eps) with the real permittivity);
  * M^-1 = sum_i R_i^T D_i B_i^-1 R_i, equation (ORAS), each B_i^-1 by a
    sparse direct LU (scipy SuperLU).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


@dataclass
class Subdomain:
    tets: np.ndarray      # tetrahedra of T_i^delta
    gdof: np.ndarray      # local -> global free dof (R_i)
    D: np.ndarray         # partition-of-unity weights on the local dofs
    B: sp.csc_matrix      # local matrix with transmission conditions
    lu: object = None


def grow(tet: np.ndarray, nv: int, mask: np.ndarray, delta: int) -> np.ndarray:
    for _ in range(delta):
        nodes = np.zeros(nv, dtype=bool)
        nodes[tet[mask].ravel()] = True
        mask = mask | nodes[tet].any(axis=1)
    return mask


def _all_faces(tet: np.ndarray):
    loc = [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]
    f = np.concatenate([tet[:, l] for l in loc])
    own = np.tile(np.arange(tet.shape[0]), 4)
    return f, own


def node_counts(tet: np.ndarray, part: np.ndarray, nv: int) -> np.ndarray:
    """Number of subdomains whose T_j^0 holds each node: the denominator of
    equation (chi)."""
    cnt = np.zeros(nv)
    for i in range(int(part.max()) + 1):
        nodes = np.zeros(nv, dtype=bool)
        nodes[tet[part == i].ravel()] = True
        cnt += nodes
    return cnt


def decompose(fp: fem.FEProblem, part: np.ndarray, delta: int = 1, factor: bool = True, subset=None, cnt=None):
    """All subdomains, or only those listed in ``subset`` (cnt: node_counts,
    if already known)."""
    nsub = int(part.max()) + 1
    nv = fp.nv
    if cnt is None:
        cnt = node_counts(fp.tet, part, nv)
    # boundary-face lookup: key -> (beta, face index)
    key_b = _face_keys(fp.bface, nv)
    order_b = np.argsort(key_b)
    k0sq = fp.k0 * fp.k0
    subs = []
    for i in (range(nsub) if subset is None else subset):
        t0 = part == i
        td = grow(fp.tet, nv, t0, delta)
        tets = np.nonzero(td)[0]
        ledges = np.unique(fp.t2e[tets].ravel())
        ledges = ledges[~fp.pec[ledges]]
        gdof = fp.dof[ledges]
        nodes0 = np.zeros(nv, dtype=bool)
        nodes0[fp.tet[t0].ravel()] = True
        chi = np.where(nodes0, 1.0, 0.0) / np.maximum(cnt, 1.0)
        D = 0.5 * (chi[fp.edges[ledges, 0]] + chi[fp.edges[ledges, 1]])
        # local numbering of global edges
        lmap = np.full(fp.edges.shape[0], -1, dtype=np.int64)
        lmap[ledges] = np.arange(ledges.size)
        n_i = ledges.size
        # volume terms of the tetrahedra of T_i^delta
        Et = fp.K[tets] - k0sq * fp.eps[tets, None, None] * fp.M[tets]
        d = lmap[fp.t2e[tets]]
        r = np.repeat(d[:, :, None], 6, axis=2)
        c = np.repeat(d[:, None, :], 6, axis=1)
        keep = (r >= 0) & (c >= 0)
        B = sp.coo_matrix((Et[keep], (r[keep], c[keep])), shape=(n_i, n_i)).tocsr()
        # faces of T_i^delta that appear once among its tetrahedra
        f, own = _all_faces(fp.tet[tets])
        fk = _face_keys(f, nv)
        uk, first, counts = np.unique(fk, return_index=True, return_counts=True)
        single = first[counts == 1]
        fsingle = np.sort(f[single], axis=1)
        fown = tets[own[single]]
        fkey = uk[counts == 1]
        pos = np.searchsorted(key_b[order_b], fkey)
        pos = np.minimum(pos, key_b.size - 1)
        is_phys = key_b[order_b][pos] == fkey
        phys_idx = order_b[pos[is_phys]]
        beta_f = np.concatenate([fp.bf_beta[phys_idx],
                                 fp.k0 * np.sqrt(fp.eps[fown[~is_phys]].real).astype(np.complex128)])
        faces = np.concatenate([fp.bface[phys_idx], fsingle[~is_phys]])
        nz = beta_f != 0
        faces, beta_f = faces[nz], beta_f[nz]
        if faces.shape[0]:
            MF = fem.face_mass(fp.xyz, faces)
            fe = fem.face_edges(faces, fp.edges, nv)
            d = lmap[fe]
            r = np.repeat(d[:, :, None], 3, axis=2)
            c = np.repeat(d[:, None, :], 3, axis=1)
            keep = (r >= 0) & (c >= 0)
            vals = (1j * beta_f[:, None, None] * MF)[keep]
            B = B + sp.coo_matrix((vals, (r[keep], c[keep])), shape=(n_i, n_i)).tocsr()
        B = B.tocsc()
        sd = Subdomain(tets=tets, gdof=gdof, D=D, B=B)
        if factor:
            sd.lu = spla.splu(B)
        subs.append(sd)
    return subs


def _face_keys(f: np.ndarray, nv: int) -> np.ndarray:
    f = np.sort(f, axis=1).astype(np.int64)
    return (f[:, 0] * nv + f[:, 1]) * nv + f[:, 2]


def oras_apply(subs, V: np.ndarray) -> np.ndarray:
    """z = sum_i R_i^T D_i B_i^-1 R_i v for every column of V."""
    Z = np.zeros_like(V, dtype=np.complex128)
    for s in subs:
        y = s.lu.solve(np.ascontiguousarray(V[s.gdof]))
        Z[s.gdof] += s.D[:, None] * y
    return Z


def oras_dense(subs, n: int) -> np.ndarray:
    """Explicit M^-1 (tiny meshes only): sum_i R_i^T D_i B_i^-1 R_i."""
    Mi = np.zeros((n, n), dtype=np.complex128)
    for s in subs:
        Binv = np.linalg.inv(s.B.toarray())
        Mi[np.ix_(s.gdof, s.gdof)] += s.D[:, None] * Binv
    return Mi


def partition_identity(subs, n: int) -> np.ndarray:
    """sum_i R_i^T D_i R_i as a diagonal (should be all ones)."""
    d = np.zeros(n)
    for s in subs:
        np.add.at(d, s.gdof, s.D)
    return d

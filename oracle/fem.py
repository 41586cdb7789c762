"""Oracle: lowest-order Nedelec (Whitney) edge-element discretisation of the
time-harmonic Maxwell problem, plain FP64 numpy/scipy.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything under
``oracle/``.  It shares no code with the GPU library.

What it computes (paper Section 2, equations (pbdirect) and (pbdirectvarf),
Section 2.1, equation (linsys)):

    find E in V:  int_Omega curl E . curl v - kappa E . v
                  + sum_ports/impedance  i beta int_Gamma (E x n).(v x n)
                  = int_{Gamma_j} g_j . v                      for all v in V,

with kappa = k0^2 eps_r (time factor e^{+i omega t}, so Im eps_r <= 0 for a
lossy medium), E x n = 0 on the metallic (PEC) walls.  The form is bilinear
(no conjugation), hence A is complex symmetric.  Degrees of freedom are the
circulations of the field along the oriented mesh edges (lo -> hi global
vertex id).

Element matrices use the closed forms of the Whitney functions
N_ab = l_a grad l_b - l_b grad l_a (l = barycentric coordinates):
    curl N_ab = 2 grad l_a x grad l_b,
    int l_x l_y = vol (1 + delta_xy) / 20  on a tetrahedron,
    int l_x l_y = area (1 + delta_xy) / 12 on a triangle,
and (E x n).(v x n) = E_t . v_t on a boundary face, whose tangential traces are
the 2-D Whitney functions built from the surface gradients of the face.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

TAG_PEC = -1
TAG_IMPEDANCE = 0

# local edges of a tetrahedron with ascending vertices, and of a triangle
TET_EDGES = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]])
TRI_EDGES = np.array([[0, 1], [0, 2], [1, 2]])


# ---------------------------------------------------------------- topology
def mesh_edges(tet: np.ndarray, nv: int):
    """Canonical oriented edges (lexicographic (lo, hi)) and the tet -> edge map."""
    pairs = tet[:, TET_EDGES].reshape(-1, 2).astype(np.int64)
    key = pairs[:, 0] * nv + pairs[:, 1]
    uniq, inv = np.unique(key, return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], axis=1)
    return edges, inv.reshape(-1, 6)


def edge_ids(edges: np.ndarray, nv: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    key = edges[:, 0] * nv + edges[:, 1]
    q = np.minimum(a, b).astype(np.int64) * nv + np.maximum(a, b)
    idx = np.searchsorted(key, q)
    assert np.all(key[np.minimum(idx, key.size - 1)] == q), "edge not in mesh"
    return idx


def face_edges(bface: np.ndarray, edges: np.ndarray, nv: int) -> np.ndarray:
    f = np.sort(bface, axis=1)
    return np.stack([edge_ids(edges, nv, f[:, i], f[:, j]) for i, j in TRI_EDGES], axis=1)


def face_owner(tet: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """Index of a tetrahedron containing each (boundary) face."""
    nv = int(tet.max()) + 1
    loc = [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]
    tf = np.concatenate([tet[:, l] for l in loc]).astype(np.int64)
    key = (tf[:, 0] * nv + tf[:, 1]) * nv + tf[:, 2]
    own = np.tile(np.arange(tet.shape[0]), 4)
    order = np.argsort(key, kind="stable")
    f = np.sort(faces, axis=1).astype(np.int64)
    q = (f[:, 0] * nv + f[:, 1]) * nv + f[:, 2]
    pos = np.searchsorted(key[order], q)
    assert np.all(key[order][pos] == q)
    return own[order][pos]


# ---------------------------------------------------------------- geometry
def tet_geometry(xyz: np.ndarray, tet: np.ndarray):
    """Barycentric coefficients: l_a(x) = c0[a] + g[a] . x, and volumes."""
    P = np.ones((tet.shape[0], 4, 4))
    P[:, :, 1:] = xyz[tet]
    C = np.linalg.inv(P)                     # P C = I: column a holds l_a's coefficients
    g = np.transpose(C[:, 1:, :], (0, 2, 1))  # [nt, 4 (vertex), 3]
    c0 = C[:, 0, :]
    vol = np.abs(np.linalg.det(P)) / 6.0
    return c0, g, vol


def element_matrices(xyz: np.ndarray, tet: np.ndarray):
    """Curl-curl K_t and mass M_t (6 x 6, real) of every tetrahedron."""
    _, g, vol = tet_geometry(xyz, tet)
    a, b = TET_EDGES[:, 0], TET_EDGES[:, 1]
    curl = 2.0 * np.cross(g[:, a, :], g[:, b, :])               # [nt, 6, 3]
    K = vol[:, None, None] * np.einsum("tpk,tqk->tpq", curl, curl)
    gg = np.einsum("tik,tjk->tij", g, g)                          # g_i . g_j
    mm = (np.ones((4, 4)) + np.eye(4)) / 20.0                     # int l_x l_y / vol
    M = np.zeros_like(K)
    for p in range(6):
        pa, pb = a[p], b[p]
        for q in range(6):
            qc, qd = a[q], b[q]
            M[:, p, q] = (mm[pa, qc] * gg[:, pb, qd] - mm[pa, qd] * gg[:, pb, qc]
                          - mm[pb, qc] * gg[:, pa, qd] + mm[pb, qd] * gg[:, pa, qc])
    M *= vol[:, None, None]
    return K, M


def cubic_bary_weights() -> np.ndarray:
    """W3[v, x, y] = int_T l_v l_x l_y / vol: 3! prod(m_i!) / 6! over the
    multiplicities m_i of the indices (1/120 all different, 1/60 two equal,
    1/20 all equal)."""
    W = np.zeros((4, 4, 4))
    for v in range(4):
        for x in range(4):
            for y in range(4):
                m = np.bincount([v, x, y], minlength=4)
                W[v, x, y] = 6.0 * np.prod([math.factorial(int(k)) for k in m]) / 720.0
    return W


def element_mass_p1(xyz: np.ndarray, tet: np.ndarray) -> np.ndarray:
    """M1[t, v] = int_t l_v N_p . N_q (6 x 6 per vertex v): the mass matrix of a
    coefficient that is linear on the tetrahedron, sum_v kappa_v M1[t, v]
    (Section 6 discretises kappa with P1 elements).  Sum over v = M_t."""
    _, g, vol = tet_geometry(xyz, tet)
    a, b = TET_EDGES[:, 0], TET_EDGES[:, 1]
    gg = np.einsum("tik,tjk->tij", g, g)
    W = cubic_bary_weights()
    M1 = np.zeros((tet.shape[0], 4, 6, 6))
    for v in range(4):
        for p in range(6):
            pa, pb = a[p], b[p]
            for q in range(6):
                qc, qd = a[q], b[q]
                M1[:, v, p, q] = (W[v, pa, qc] * gg[:, pb, qd] - W[v, pa, qd] * gg[:, pb, qc]
                                  - W[v, pb, qc] * gg[:, pa, qd] + W[v, pb, qd] * gg[:, pa, qc])
    return M1 * vol[:, None, None, None]


def face_geometry(xyz: np.ndarray, faces: np.ndarray):
    """Surface gradients s[f, 3 (vertex), 3], areas and unit normals."""
    f = np.sort(faces, axis=1)
    p0, p1, p2 = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
    e1, e2 = p1 - p0, p2 - p0
    n = np.cross(e1, e2)
    n2 = (n * n).sum(axis=1)
    s1 = np.cross(e2, n) / n2[:, None]
    s2 = np.cross(n, e1) / n2[:, None]
    s0 = -s1 - s2
    area = 0.5 * np.sqrt(n2)
    return np.stack([s0, s1, s2], axis=1), area, n / np.sqrt(n2)[:, None]


def face_mass(xyz: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """int_F (N_p x n).(N_q x n) for the 3 edges of each face (3 x 3, real)."""
    s, area, _ = face_geometry(xyz, faces)
    a, b = TRI_EDGES[:, 0], TRI_EDGES[:, 1]
    ss = np.einsum("fik,fjk->fij", s, s)
    mm = (np.ones((3, 3)) + np.eye(3)) / 12.0
    M = np.zeros((faces.shape[0], 3, 3))
    for p in range(3):
        for q in range(3):
            M[:, p, q] = (mm[a[p], a[q]] * ss[:, b[p], b[q]] - mm[a[p], b[q]] * ss[:, b[p], a[q]]
                          - mm[b[p], a[q]] * ss[:, a[p], b[q]] + mm[b[p], b[q]] * ss[:, a[p], a[q]])
    return M * area[:, None, None]


# ---------------------------------------------------------------- problem
@dataclass
class FEProblem:
    nv: int
    xyz: np.ndarray
    tet: np.ndarray
    edges: np.ndarray          # [ne, 2]
    t2e: np.ndarray            # [nt, 6]
    pec: np.ndarray            # bool [ne]
    dof: np.ndarray            # [ne] -> free dof index or -1
    free: np.ndarray           # free edge ids, ascending (dof k <-> edge free[k])
    K: np.ndarray              # [nt, 6, 6]
    M: np.ndarray              # [nt, 6, 6]
    bface: np.ndarray          # [nbf, 3] ascending
    btag: np.ndarray
    bf2e: np.ndarray           # [nbf, 3]
    bf_beta: np.ndarray        # complex beta per boundary face (0 on PEC)
    MF: np.ndarray             # [nbf, 3, 3]
    k0: float
    eps: np.ndarray
    A: sp.csr_matrix           # free x free, complex128

    @property
    def n(self) -> int:
        return int(self.free.size)


def _scatter(rows, cols, vals, n):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def assemble_matrix(tet, t2e, K, M, eps, k0, bf2e, bf_beta, MF, dof, n):
    """A = sum_t (K_t - k0^2 eps_t M_t) + sum_F i beta_F M_F, PEC dofs removed."""
    Et = K - (k0 * k0) * eps[:, None, None] * M
    d = dof[t2e]                                              # [nt, 6]
    r = np.repeat(d[:, :, None], 6, axis=2)
    c = np.repeat(d[:, None, :], 6, axis=1)
    keep = (r >= 0) & (c >= 0)
    A = _scatter(r[keep], c[keep], Et[keep], n)
    imp = bf_beta != 0
    if imp.any():
        Ef = 1j * bf_beta[imp, None, None] * MF[imp]
        dfc = dof[bf2e[imp]]
        r = np.repeat(dfc[:, :, None], 3, axis=2)
        c = np.repeat(dfc[:, None, :], 3, axis=1)
        keep = (r >= 0) & (c >= 0)
        A = A + _scatter(r[keep], c[keep], Ef[keep], n)
    A.sum_duplicates()
    return A.tocsr()


def build(mesh, eps, k0: float, beta_imp: complex, ports) -> FEProblem:
    """Discretise problem (pbdirect) on ``mesh`` (Section 2.1)."""
    tet = np.sort(mesh.tet, axis=1).astype(np.int64)
    nv = mesh.xyz.shape[0]
    edges, t2e = mesh_edges(tet, nv)
    bface = np.sort(mesh.bface, axis=1).astype(np.int64)
    btag = np.asarray(mesh.btag)
    bf2e = face_edges(bface, edges, nv)
    pec = np.zeros(edges.shape[0], dtype=bool)
    pec[bf2e[btag == TAG_PEC].ravel()] = True
    free = np.nonzero(~pec)[0]
    dof = np.full(edges.shape[0], -1, dtype=np.int64)
    dof[free] = np.arange(free.size)
    K, M = element_matrices(mesh.xyz, tet)
    MF = face_mass(mesh.xyz, bface)
    beta = np.zeros(bface.shape[0], dtype=np.complex128)
    beta[btag == TAG_IMPEDANCE] = beta_imp
    for k, pt in enumerate(ports):
        beta[btag == k + 1] = pt.beta
    eps = np.asarray(eps, dtype=np.complex128)
    A = assemble_matrix(tet, t2e, K, M, eps, k0, bf2e, beta, MF, dof, free.size)
    return FEProblem(nv=nv, xyz=mesh.xyz, tet=tet, edges=edges, t2e=t2e, pec=pec, dof=dof,
                     free=free, K=K, M=M, bface=bface, btag=btag, bf2e=bf2e, bf_beta=beta,
                     MF=MF, k0=k0, eps=eps, A=A)


def with_eps(fp: FEProblem, eps) -> FEProblem:
    eps = np.asarray(eps, dtype=np.complex128)
    A = assemble_matrix(fp.tet, fp.t2e, fp.K, fp.M, eps, fp.k0, fp.bf2e, fp.bf_beta, fp.MF,
                        fp.dof, fp.n)
    return FEProblem(**{**fp.__dict__, "eps": eps, "A": A})


def with_eps_vertex(fp: FEProblem, eps_v, M1: np.ndarray | None = None) -> FEProblem:
    """The operator with eps_r linear on every tetrahedron, given at the
    vertices: sum_t K_t - k0^2 sum_v eps_v M1[t, v] + boundary terms.  The
    problem's eps becomes the tetrahedron means (used by the transmission
    wavenumber of the preconditioner)."""
    eps_v = np.asarray(eps_v, dtype=np.complex128)
    if M1 is None:
        M1 = element_mass_p1(fp.xyz, fp.tet)
    Meps = np.einsum("tv,tvpq->tpq", eps_v[fp.tet], M1)
    A = assemble_matrix(fp.tet, fp.t2e, fp.K, Meps, np.ones(fp.tet.shape[0], dtype=np.complex128), fp.k0,
                        fp.bf2e, fp.bf_beta, fp.MF, fp.dof, fp.n)
    return FEProblem(**{**fp.__dict__, "eps": eps_v[fp.tet].mean(axis=1), "A": A})


# ---------------------------------------------------------------- sources
def locate(fp: FEProblem, x: np.ndarray):
    """Lowest-index tetrahedron whose barycentrics at x are all >= -1e-12."""
    c0, g, _ = tet_geometry(fp.xyz, fp.tet)
    lam = c0 + np.einsum("tak,k->ta", g, x)
    ok = np.nonzero((lam >= -1e-12).all(axis=1))[0]
    t = int(ok[0])
    return t, lam[t], g[t]


def rhs_dipoles(fp: FEProblem, points: np.ndarray, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    """b[e] = dir . N_e(x0): a unit point dipole at x0 (free dofs x npoints)."""
    B = np.zeros((fp.n, points.shape[0]), dtype=np.complex128)
    d = np.asarray(direction, dtype=float)
    for j, x in enumerate(points):
        t, lam, g = locate(fp, x)
        for p, (a, b) in enumerate(TET_EDGES):
            k = fp.dof[fp.t2e[t, p]]
            if k >= 0:
                B[k, j] += d @ (lam[a] * g[b] - lam[b] * g[a])
    return B


def port_mode(pt, x: np.ndarray) -> np.ndarray:
    """Incident TE10-like profile of a port: pol * cos(pi s / width)."""
    phi = np.arctan2(x[..., 1], x[..., 0])
    s = pt.radius * np.angle(np.exp(1j * (phi - pt.theta)))
    return np.cos(np.pi * s / pt.width)[..., None] * np.asarray(pt.pol, dtype=float)


def port_vectors(fp: FEProblem, ports):
    """p_k[e] = int_{Gamma_k} E0_k . N_e and nu_k = int_{Gamma_k} |E0_k|^2 with the
    edge-midpoint rule (weights area/3) on every face of port k; Section 3,
    equation (sij)."""
    s, area, nrm = face_geometry(fp.xyz, fp.bface)
    P = np.zeros((fp.n, len(ports)))
    nu = np.zeros(len(ports))
    for k, pt in enumerate(ports):
        fs = np.nonzero(fp.btag == k + 1)[0]
        for f in fs:
            v = fp.xyz[fp.bface[f]]
            for (u, w) in TRI_EDGES:          # quadrature point: midpoint of face edge (u, w)
                lam = np.zeros(3)
                lam[u] = lam[w] = 0.5
                xm = 0.5 * (v[u] + v[w])
                e0 = port_mode(pt, xm)
                e0 = e0 - (e0 @ nrm[f]) * nrm[f]
                wq = area[f] / 3.0
                nu[k] += wq * (e0 @ e0)
                for q, (a, b) in enumerate(TRI_EDGES):
                    dof = fp.dof[fp.bf2e[f, q]]
                    if dof >= 0:
                        Nq = lam[a] * s[f, b] - lam[b] * s[f, a]
                        P[dof, k] += wq * (e0 @ Nq)
    return P, nu


def rhs_ports(fp: FEProblem, ports, tx) -> np.ndarray:
    """b_j = int_{Gamma_j} g_j . v with g_j = 2 i beta_j E0_j (incoming mode)."""
    P, _ = port_vectors(fp, ports)
    beta = np.array([ports[j].beta for j in tx])
    return P[:, tx] * (2j * beta)[None, :]

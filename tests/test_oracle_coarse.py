"""Pins of the oracle's two-level ORAS (oracle/coarse.py) against special
cases and invariants that any correct deflated coarse correction satisfies,
and of its coarse fields against independently built Whitney functions and
line integrals.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import coarse, dd, fem, gmres

RNG = np.random.default_rng(77)


@pytest.fixture(scope="module")
def cube4():
    w = mi.configs.cube(4, n_sub=4, ndip=3)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    return w, fp


def _rand(n, k):
    return RNG.normal(size=(n, k)) + 1j * RNG.normal(size=(n, k))


def test_full_coarse_space_gives_the_inverse(cube4):
    """Z spanning every unknown: Q = A^-1, so M2^-1 = A^-1 whatever the
    subdomain solves are, and GMRES stops after one iteration."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1)
    M2 = coarse.TwoLevel(fp, subs, Z=sp.identity(fp.n, format="csc"))
    V = _rand(fp.n, 3)
    np.testing.assert_allclose(M2.apply(V), spla.splu(fp.A.tocsc()).solve(V), rtol=0,
                               atol=1e-10 * np.abs(spla.splu(fp.A.tocsc()).solve(V)).max())
    B = fem.rhs_dipoles(fp, w.dipoles)
    _, it, rr = gmres.gmres(fp.A, B, M2, tol=1e-10)
    assert (it == 1).all() and (rr <= 1e-10).all()


def test_one_subdomain_stays_exact(cube4):
    """N_S = 1: M^-1 = A^-1 and the correction changes nothing."""
    w, fp = cube4
    part = np.zeros(w.mesh.nt, dtype=np.int32)
    M2 = coarse.TwoLevel(fp, dd.decompose(fp, part, 1))
    B = fem.rhs_dipoles(fp, w.dipoles)
    _, it, rr = gmres.gmres(fp.A, B, M2, tol=1e-10)
    assert (it == 1).all() and (rr <= 1e-10).all()


@pytest.mark.parametrize("kind", ["const", "wave"])
def test_deflation_invariants(cube4, kind):
    """M2^-1 A is the identity on span(Z), the residual handed to the
    one-level preconditioner is Z-orthogonal, E is complex symmetric, and
    the columns of Z are supported on their own subdomain with weight D_i."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1)
    M2 = coarse.TwoLevel(fp, subs, kind, k=fp.k0)
    Z = M2.Z.toarray()
    np.testing.assert_allclose(M2.apply(fp.A @ Z), Z, rtol=0, atol=1e-10 * np.abs(Z).max())
    V = _rand(fp.n, 4)
    R = V - fp.A @ M2.coarse(V)
    assert np.abs(M2.Z.T @ R).max() <= 1e-11 * np.abs(V).max() * np.abs(Z).sum(axis=0).max()
    assert np.abs(M2.E - M2.E.T).max() <= 1e-13 * np.abs(M2.E).max()
    nk = M2.size // len(subs)
    for i, s in enumerate(subs):
        blk = Z[:, i * nk:(i + 1) * nk]
        outside = np.ones(fp.n, dtype=bool)
        outside[s.gdof] = False
        assert not blk[outside].any()
        zero_w = s.gdof[s.D == 0]
        assert not blk[zero_w].any()


def test_constant_fields_are_exact_interpolants():
    """Phi[:, a] (kind 'const') are the circulations of the constant field
    e_a, so the Whitney interpolant built from them (barycentric gradients by
    a 4 x 4 solve, independent of fem) equals e_a everywhere in every
    tetrahedron whose six edges are unknowns of the subdomain."""
    w = mi.configs.cube(3, n_sub=2, ndip=1)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    s = dd.decompose(fp, w.part, 1, factor=False)[0]
    Phi = coarse.local_fields(fp, s, "const")
    pos = {int(g): k for k, g in enumerate(s.gdof)}
    checked = 0
    for t in s.tets:
        dofs = [int(fp.dof[fp.t2e[t, q]]) for q in range(6)]
        if any(d < 0 or d not in pos for d in dofs):
            continue
        X = fp.xyz[fp.tet[t]]
        G = np.linalg.solve(np.c_[np.ones(4), X], np.eye(4))[1:, :].T     # G[a] = grad l_a
        cir = np.array([Phi[pos[d]] for d in dofs])                      # [6 edges, 3 fields]
        for lam in ([0.25] * 4, [0.7, 0.1, 0.1, 0.1], [0.1, 0.2, 0.3, 0.4]):
            N = np.array([lam[a] * G[b] - lam[b] * G[a] for a, b in fem.TET_EDGES])
            np.testing.assert_allclose(cir.T @ N, np.eye(3), atol=1e-12)
        checked += 1
    assert checked >= 20


def test_wave_fields_are_edge_circulations():
    """Phi (kind 'wave', after the three constants) against a 6-point
    Gauss-Legendre line integral of Re/Im(p exp(-i k d.x)) . t along each
    edge: the midpoint rule's error is below (k h)^2 / 24 of the value's
    scale."""
    w = mi.configs.cube(3, n_sub=2, ndip=1)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    s = dd.decompose(fp, w.part, 1, factor=False)[1]
    k = 2.5
    Phi = coarse.local_fields(fp, s, "wave", k)
    gx, gw = np.polynomial.legendre.leggauss(6)
    e = fp.edges[fp.free[s.gdof]]
    xa, xb = fp.xyz[e[:, 0]], fp.xyz[e[:, 1]]
    h = np.linalg.norm(xb - xa, axis=1).max()
    col = 3
    for kd, p in coarse.wave_fields(k):
        ref = np.zeros(s.gdof.size, dtype=complex)
        for x, wq in zip(gx, gw):
            pts = xa + 0.5 * (x + 1) * (xb - xa)
            ref += 0.5 * wq * np.exp(-1j * (pts @ kd)) * ((xb - xa) @ p)
        for part, got in ((ref.real, Phi[:, col]), (ref.imag, Phi[:, col + 1])):
            assert np.abs(got - part).max() <= (k * h) ** 2 / 24 * h + 1e-14
        col += 2
    assert col == Phi.shape[1] == 15

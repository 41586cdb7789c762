"""Pins of the oracle's ORAS preconditioner, GMRES and adjoint gradient
against special cases, invariants and brute force.  CPU only."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import dd, fem, gmres, inverse

RNG = np.random.default_rng(99)


@pytest.fixture(scope="module")
def cube4():
    w = mi.configs.cube(4, n_sub=4, ndip=3)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    return w, fp


def test_partition_of_unity_identity(cube4):
    w, fp = cube4
    for nsub in (2, 4, 7):
        part = mi.partition.rcb(w.mesh, nsub)
        subs = dd.decompose(fp, part, 1, factor=False)
        np.testing.assert_allclose(dd.partition_identity(subs, fp.n), 1.0, atol=1e-15)
        assert all((s.D >= 0).all() and (s.D <= 1).all() for s in subs)


def test_one_subdomain_is_exact(cube4):
    """N_S = 1: B_1 = A, D_1 = I, so right-preconditioned GMRES stops after
    one iteration."""
    w, fp = cube4
    part = np.zeros(w.mesh.nt, dtype=np.int32)
    subs = dd.decompose(fp, part, 1)
    assert abs(subs[0].B - fp.A).max() < 1e-14 * abs(fp.A).max()
    np.testing.assert_array_equal(subs[0].D, 1.0)
    B = fem.rhs_dipoles(fp, w.dipoles)
    X, it, rr = gmres.gmres(fp.A, B, lambda V: dd.oras_apply(subs, V), tol=1e-10)
    assert (it == 1).all() and (rr < 1e-10).all()


def test_large_overlap_gives_exact_inverse(cube4):
    """When every T_i^delta is the whole mesh, B_i = A and M^-1 = A^-1."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, delta=10)
    assert all(s.gdof.size == fp.n for s in subs)
    Ainv = np.linalg.inv(fp.A.toarray())
    np.testing.assert_allclose(dd.oras_dense(subs, fp.n), Ainv, atol=1e-10 * np.abs(Ainv).max())


def test_oras_apply_equals_dense_sum(cube4):
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1)
    Md = dd.oras_dense(subs, fp.n)
    V = RNG.normal(size=(fp.n, 3)) + 1j * RNG.normal(size=(fp.n, 3))
    np.testing.assert_allclose(dd.oras_apply(subs, V), Md @ V, rtol=1e-9, atol=1e-11 * np.abs(Md @ V).max())


def test_local_matrix_matches_global_away_from_interface(cube4):
    """B_i = R_i A R_i^T on rows whose edge touches only tetrahedra of T_i^delta
    and lies on no interface face (the transmission term acts on the
    subdomain boundary only); B_i is complex symmetric."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1, factor=False)
    for s in subs:
        Bd = s.B.toarray()
        assert np.abs(Bd - Bd.T).max() < 1e-14 * np.abs(Bd).max()
        inside = np.zeros(fp.edges.shape[0], dtype=bool)
        inside_t = np.zeros(fp.tet.shape[0], dtype=bool)
        inside_t[s.tets] = True
        # an edge is interior when all tetrahedra around it are in T_i^delta
        cnt_all = np.bincount(fp.t2e.ravel(), minlength=fp.edges.shape[0])
        cnt_in = np.bincount(fp.t2e[inside_t].ravel(), minlength=fp.edges.shape[0])
        inside = (cnt_all == cnt_in) & (cnt_in > 0)
        ledge = fp.free[s.gdof]
        rows = np.nonzero(inside[ledge])[0]
        RA = fp.A[s.gdof][:, s.gdof].toarray()
        np.testing.assert_allclose(Bd[rows], RA[rows], atol=1e-13 * np.abs(RA).max())


def test_givens_rotation_zeroes():
    for a, b in [(1 + 2j, 3.0), (0j, 2.0), (-1e-3 + 4j, 0.0)]:
        c, s, r = gmres.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        v = G @ np.array([a, b])
        assert abs(v[1]) < 1e-14 * max(abs(a), b, 1e-300) + 1e-300
        assert abs(v[0] - r) < 1e-14 * abs(r) + 1e-300
        assert abs(abs(c) ** 2 + abs(s) ** 2 - 1) < 1e-14


def test_gmres_minimal_residual_property(cube4):
    """Without restart, after k steps GMRES attains the minimum of
    ||b - A M^-1 y|| over the Krylov space K_k(A M^-1, b): compare with a
    least-squares solve over an explicitly built (QR-orthonormalised) basis."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1)
    prec = lambda V: dd.oras_apply(subs, V)  # noqa: E731
    b = fem.rhs_dipoles(fp, w.dipoles[:1])
    for k in (1, 3, 5):
        X, it, rr = gmres.gmres(fp.A, b, prec, tol=1e-30, restart=50, maxit=k)
        Kb = [b[:, 0]]
        for _ in range(k - 1):
            Kb.append(fp.A @ prec(Kb[-1][:, None])[:, 0])
        Q, _ = np.linalg.qr(np.stack(Kb, axis=1))
        AMQ = np.stack([fp.A @ prec(Q[:, [i]])[:, 0] for i in range(k)], axis=1)
        y = np.linalg.lstsq(AMQ, b[:, 0], rcond=None)[0]
        best = np.linalg.norm(b[:, 0] - AMQ @ y) / np.linalg.norm(b)
        assert it[0] == k
        assert abs(rr[0] - best) <= 1e-8 * best + 1e-14


def test_gmres_matches_direct_and_restarts(cube4):
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1)
    B = fem.rhs_dipoles(fp, w.dipoles)
    U = spla.splu(fp.A.tocsc()).solve(B)
    for m in (30, 4):          # m = 4 forces several restart cycles
        X, it, rr = gmres.gmres(fp.A, B, lambda V: dd.oras_apply(subs, V), tol=1e-11, restart=m)
        assert (rr <= 1e-11).all()
        err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
        assert (err < 1e-8).all(), err


def test_woodbury_perturbed_solve_matches_refactorisation():
    """The FD machinery: an exact Woodbury update equals a fresh sparse LU of
    the perturbed matrix."""
    w = mi.configs.small_chamber(0.25e9, n_per_ring=4)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    lu, U = inverse.forward(fp, w.ports, w.tx)
    B = fem.rhs_ports(fp, w.ports, w.tx)
    P, nu = fem.port_vectors(fp, w.ports)
    Smes = inverse.s_matrix(P, nu, U, w.rx) * 0.9
    t = int(np.argmax(np.abs(fp.eps)))
    h = 1e-3
    e1 = fp.eps.copy()
    e1[t] += h
    e2 = fp.eps.copy()
    e2[t] -= h
    J1 = inverse.misfit(inverse.s_matrix(P, nu, spla.splu(fem.with_eps(fp, e1).A.tocsc()).solve(B), w.rx), Smes)
    J2 = inverse.misfit(inverse.s_matrix(P, nu, spla.splu(fem.with_eps(fp, e2).A.tocsc()).solve(B), w.rx), Smes)
    fd_direct = (J1 - J2) / (2 * h)
    fd_wb = inverse.woodbury_fd(fp, lu, U, B, P, nu, w.rx, Smes, t, h)
    assert abs(fd_wb - fd_direct) <= 1e-8 * abs(fd_direct) + 1e-15


def test_adjoint_gradient_matches_finite_differences():
    """Section 5: the adjoint gradient equals central differences of J (done
    exactly by Woodbury) in the Re and Im directions of eps_t."""
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    lu, U = inverse.forward(fp, w.ports, w.tx)
    B = fem.rhs_ports(fp, w.ports, w.tx)
    P, nu = fem.port_vectors(fp, w.ports)
    # 'measured' data from a perturbed permittivity
    eps_true = fp.eps * (1 + 0.05 * RNG.normal(size=fp.eps.size))
    Smes = inverse.s_matrix(P, nu, spla.splu(fem.with_eps(fp, eps_true).A.tocsc()).solve(B), w.rx)
    J, S, grad = inverse.adjoint_gradient(fp, lu, P, nu, U, w.tx, w.rx, Smes)
    tets = RNG.choice(fp.tet.shape[0], size=6, replace=False)
    for t in tets:
        h = 1e-4 * abs(fp.eps[t])
        dre = inverse.woodbury_fd(fp, lu, U, B, P, nu, w.rx, Smes, t, h)
        dim = inverse.woodbury_fd(fp, lu, U, B, P, nu, w.rx, Smes, t, 1j * h)
        fd = dre + 1j * dim
        assert abs(grad[t] - fd) <= 1e-5 * abs(fd) + 1e-12 * np.abs(grad).max(), (t, grad[t], fd)


def test_local_matrices_have_positive_definite_imaginary_part(cube4):
    """With every tetrahedron lossy (Im eps_r < 0, e^{+i omega t}), the
    imaginary part of each local matrix B_i (mass term -k0^2 Im(eps) M,
    impedance and transmission terms beta M_F, k M_F) is positive definite;
    so x^H B_i x never vanishes, every leading block of B_i is nonsingular and
    a symmetric factorisation without interchanges cannot break down -- the
    reading behind the GPU's L D L^T subdomain factors."""
    w, fp = cube4
    subs = dd.decompose(fp, w.part, 1, factor=False)
    for s in subs:
        Bd = s.B.toarray()
        ev = np.linalg.eigvalsh(Bd.imag)
        assert ev.min() > 1e-8 * ev.max(), ev.min()
        # unpivoted Gaussian elimination runs through with no small pivot
        A = Bd.copy()
        piv = []
        for k in range(A.shape[0]):
            piv.append(abs(A[k, k]))
            A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:]) / A[k, k]
        assert min(piv) > 1e-6 * np.abs(Bd).max()


def test_pooled_oras_equals_serial_sum(cube4):
    """The process-pool form of the preconditioner (one share of the
    subdomains per worker, partial sums added in worker order) equals the
    serial sum over subdomains to rounding, for more columns than one pass
    takes."""
    from oracle import pool
    w, fp = cube4
    part = mi.partition.rcb(w.mesh, 7)
    subs = dd.decompose(fp, part, 1)
    V = RNG.normal(size=(fp.n, 5)) + 1j * RNG.normal(size=(fp.n, 5))
    Zs = dd.oras_apply(subs, V)
    with pool.PooledORAS(fp, part, 1, nproc=3, max_cols=2) as M:
        Zp = M.apply(V)
    np.testing.assert_allclose(Zp, Zs, rtol=0, atol=1e-13 * np.abs(Zs).max())

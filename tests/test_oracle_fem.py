"""Pins of the oracle's edge-element discretisation against facts fixed by the
mathematics (closed forms, quadrature, invariants, brute force), independent
of the oracle's own closed-form formulas.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import fem

RNG = np.random.default_rng(1234)

# degree-2 rule on the tetrahedron (4 points, equal weights)
_A, _B = 0.5854101966249685, 0.1381966011250105
TET_Q2 = np.array([[_A, _B, _B, _B], [_B, _A, _B, _B], [_B, _B, _A, _B], [_B, _B, _B, _A]])
# degree-3 rule (5 points, Keast/Stroud): centroid -4/5, four points 9/20
TET_Q3_PTS = np.array([[0.25] * 4, [0.5, 1 / 6, 1 / 6, 1 / 6], [1 / 6, 0.5, 1 / 6, 1 / 6],
                       [1 / 6, 1 / 6, 0.5, 1 / 6], [1 / 6, 1 / 6, 1 / 6, 0.5]])
TET_Q3_W = np.array([-0.8, 0.45, 0.45, 0.45, 0.45])
# degree-2 interior rule on the triangle
TRI_Q2 = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
# degree-4 rule on the triangle (Dunavant, 6 points)
_a1, _b1, _w1 = 0.108103018168070, 0.445948490915965, 0.223381589678011
_a2, _b2, _w2 = 0.816847572980459, 0.091576213509771, 0.109951743655322
TRI_Q4 = np.array([[_a1, _b1, _b1], [_b1, _a1, _b1], [_b1, _b1, _a1],
                   [_a2, _b2, _b2], [_b2, _a2, _b2], [_b2, _b2, _a2]])
TRI_Q4_W = np.array([_w1] * 3 + [_w2] * 3)


def random_tet():
    while True:
        P = RNG.normal(size=(4, 3))
        if abs(np.linalg.det(np.c_[np.ones(4), P])) > 0.3:
            return P


def whitney_at(P, lam):
    """Whitney functions N_ab = l_a grad l_b - l_b grad l_a at barycentric point lam,
    with barycentric gradients from solving the 4x4 system (not fem's formulas)."""
    T = np.c_[np.ones(4), P]
    g = np.linalg.solve(T, np.eye(4))[1:, :].T    # g[a] = grad l_a
    return np.array([lam[a] * g[b] - lam[b] * g[a] for a, b in fem.TET_EDGES])


def test_mass_matrix_matches_quadrature():
    for _ in range(5):
        P = random_tet()
        vol = abs(np.linalg.det(np.c_[np.ones(4), P])) / 6
        Mq = np.zeros((6, 6))
        for lam in TET_Q2:
            N = whitney_at(P, lam)
            Mq += vol / 4 * N @ N.T
        K, M = fem.element_matrices(P, np.array([[0, 1, 2, 3]]))
        np.testing.assert_allclose(M[0], Mq, rtol=1e-12, atol=1e-12 * np.abs(Mq).max())


def test_p1_coefficient_mass_matches_cubic_quadrature():
    """int_t l_v N_p . N_q (degree 3) by the 5-point degree-3 rule with
    independently built Whitney functions; and sum_v over the four vertex
    matrices gives the plain mass matrix (the l_v sum to one)."""
    for _ in range(5):
        P = random_tet()
        vol = abs(np.linalg.det(np.c_[np.ones(4), P])) / 6
        Mq = np.zeros((4, 6, 6))
        for lam, wq in zip(TET_Q3_PTS, TET_Q3_W):
            N = whitney_at(P, lam)
            for v in range(4):
                Mq[v] += vol * wq * lam[v] * (N @ N.T)
        M1 = fem.element_mass_p1(P, np.array([[0, 1, 2, 3]]))[0]
        np.testing.assert_allclose(M1, Mq, rtol=1e-11, atol=1e-12 * np.abs(Mq).max())
        _, M = fem.element_matrices(P, np.array([[0, 1, 2, 3]]))
        np.testing.assert_allclose(M1.sum(axis=0), M[0], rtol=1e-13, atol=1e-14 * np.abs(M).max())


def test_p1_operator_with_constant_field_is_the_p0_operator():
    w = mi.configs.cube(2)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    c = 2.5 - 0.7j
    A1 = fem.with_eps_vertex(fp, np.full(fp.nv, c)).A
    A0 = fem.with_eps(fp, np.full(fp.tet.shape[0], c)).A
    assert abs(A1 - A0).max() <= 1e-13 * abs(A0).max()


def test_curl_matrix_matches_numerical_curl():
    for _ in range(5):
        P = random_tet()
        vol = abs(np.linalg.det(np.c_[np.ones(4), P])) / 6
        T = np.c_[np.ones(4), P]
        C = np.linalg.inv(T)
        x0 = P.mean(axis=0)
        hstep = 1e-3

        def N_at(x):
            lam = C.T @ np.r_[1.0, x]
            return whitney_at(P, lam)

        J = np.zeros((6, 3, 3))            # J[p, i, j] = d N_p,i / d x_j (exact: N is affine)
        for j in range(3):
            e = np.zeros(3)
            e[j] = hstep
            J[:, :, j] = (N_at(x0 + e) - N_at(x0 - e)) / (2 * hstep)
        curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)
        Kq = vol * curl @ curl.T
        K, _ = fem.element_matrices(P, np.array([[0, 1, 2, 3]]))
        np.testing.assert_allclose(K[0], Kq, rtol=1e-9, atol=1e-9 * np.abs(Kq).max())


def test_constant_field_reproduction():
    """u_e = c . (x_b - x_a) interpolates the constant field c exactly:
    sum_e u_e N_e = c, u^T M u = |c|^2 vol, K u = 0."""
    for _ in range(5):
        P = random_tet()
        vol = abs(np.linalg.det(np.c_[np.ones(4), P])) / 6
        c = RNG.normal(size=3)
        u = np.array([c @ (P[b] - P[a]) for a, b in fem.TET_EDGES])
        for lam in RNG.dirichlet(np.ones(4), size=4):
            np.testing.assert_allclose(whitney_at(P, lam).T @ u, c, rtol=1e-12, atol=1e-12)
        K, M = fem.element_matrices(P, np.array([[0, 1, 2, 3]]))
        assert abs(u @ M[0] @ u - (c @ c) * vol) < 1e-12 * (c @ c) * vol
        assert np.abs(K[0] @ u).max() < 1e-11 * np.abs(K[0]).max() * np.abs(u).max()


def test_element_matrices_symmetric_and_mass_spd():
    P = random_tet()
    K, M = fem.element_matrices(P, np.array([[0, 1, 2, 3]]))
    np.testing.assert_allclose(K[0], K[0].T, atol=1e-13 * np.abs(K).max())
    np.testing.assert_allclose(M[0], M[0].T, atol=1e-13 * np.abs(M).max())
    assert np.linalg.eigvalsh(M[0]).min() > 0


def test_face_mass_matches_tangential_trace_quadrature():
    """int_F (N_p x n).(N_q x n) with the 3-D Whitney functions of the tet that
    owns the face, projected on the face plane, integrated by a degree-2
    triangle rule."""
    for _ in range(5):
        P = random_tet()
        face = [0, 1, 3]
        Q = P[face]
        nrm = np.cross(Q[1] - Q[0], Q[2] - Q[0])
        area = 0.5 * np.linalg.norm(nrm)
        nrm /= np.linalg.norm(nrm)
        # face edges (0,1), (0,3), (1,3) are tet edges 0, 2, 4
        tet_edge_of_face_edge = [0, 2, 4]
        Mq = np.zeros((3, 3))
        for mu in TRI_Q2:
            lam = np.zeros(4)
            lam[face] = mu
            N = whitney_at(P, lam)[tet_edge_of_face_edge]
            Nt = N - np.outer(N @ nrm, nrm)
            Mq += area / 3 * Nt @ Nt.T
        MF = fem.face_mass(P, np.array([face]))[0]
        np.testing.assert_allclose(MF, Mq, rtol=1e-12, atol=1e-12 * np.abs(Mq).max())


def test_kuhn_cube_edge_count_closed_form():
    """Edges of the Kuhn split of an N^3 grid: 3N(N+1)^2 axis edges,
    3N^2(N+1) face diagonals, N^3 body diagonals."""
    for n in (1, 2, 3, 8):
        m = mi.mesh.cube_mesh(n)
        edges, _ = fem.mesh_edges(m.tet, m.nv)
        assert edges.shape[0] == 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3


def _global_curl_matrix(fp):
    d = fp.t2e
    r = np.repeat(d[:, :, None], 6, axis=2)
    c = np.repeat(d[:, None, :], 6, axis=1)
    ne = fp.edges.shape[0]
    return sp.coo_matrix((fp.K.ravel(), (r.ravel(), c.ravel())), shape=(ne, ne)).tocsr()


def test_curl_of_gradient_vanishes():
    w = mi.configs.cube(4, n_sub=2)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    ne, nv = fp.edges.shape[0], fp.nv
    G = sp.coo_matrix((np.r_[-np.ones(ne), np.ones(ne)],
                       (np.r_[np.arange(ne), np.arange(ne)], np.r_[fp.edges[:, 0], fp.edges[:, 1]])),
                      shape=(ne, nv)).tocsr()
    Kg = _global_curl_matrix(fp)
    phi = RNG.normal(size=nv)
    assert np.abs(Kg @ (G @ phi)).max() < 1e-12 * np.abs(Kg).max() * np.abs(phi).max()
    # integer face-edge incidence C satisfies C G = 0 exactly; the boundary of
    # the face a<b<c traversed a->b->c->a is +e(a,b) + e(b,c) - e(a,c)
    fe = fp.bf2e                        # columns: e(a,b), e(a,c), e(b,c)
    nf = fe.shape[0]
    Cm = sp.coo_matrix((np.tile([1.0, -1.0, 1.0], nf), (np.repeat(np.arange(nf), 3), fe.ravel())),
                       shape=(nf, ne)).tocsr()
    assert np.abs((Cm @ G).toarray()).max() == 0
    # the full operator on a gradient field reduces to its mass and boundary parts
    gphi = (G @ phi)[fp.free]
    lhs = fp.A @ gphi
    rhs = (fem.assemble_matrix(fp.tet, fp.t2e, 0 * fp.K, fp.M, fp.eps, fp.k0, fp.bf2e, fp.bf_beta,
                               fp.MF, fp.dof, fp.n)) @ gphi
    np.testing.assert_allclose(lhs, rhs, atol=1e-10 * np.abs(lhs).max())


def test_matrix_complex_symmetric():
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    d = fp.A - fp.A.T
    assert abs(d).max() <= 1e-15 * abs(fp.A).max()
    assert fp.A.dtype == np.complex128


@pytest.mark.parametrize("n,ne,nnz", [(1, 19, 163), (2, 98, 1106)])
def test_dense_bruteforce_tiny_cubes(n, ne, nnz):
    """On 1- and 2-cell cubes the sparse direct solve equals a dense solve of
    the matrix assembled entry by entry from the element matrices."""
    m = mi.mesh.cube_mesh(n)
    eps = np.full(m.nt, 1 - 0.1j)
    k0 = 3.0
    fp = fem.build(m, eps, k0, k0 * np.sqrt(1 - 0.1j), [])
    assert fp.n == ne and fp.A.nnz == nnz
    Ad = np.zeros((ne, ne), dtype=complex)
    for t in range(m.nt):
        for p in range(6):
            for q in range(6):
                Ad[fp.t2e[t, p], fp.t2e[t, q]] += fp.K[t, p, q] - k0 ** 2 * eps[t] * fp.M[t, p, q]
    for f in range(fp.bface.shape[0]):
        for p in range(3):
            for q in range(3):
                Ad[fp.bf2e[f, p], fp.bf2e[f, q]] += 1j * fp.bf_beta[f] * fp.MF[f, p, q]
    np.testing.assert_allclose(fp.A.toarray(), Ad, atol=1e-14 * np.abs(Ad).max())
    b = RNG.normal(size=(ne, 3)) + 1j * RNG.normal(size=(ne, 3))
    x1 = np.linalg.solve(Ad, b)
    x2 = spla.splu(fp.A.tocsc()).solve(b)
    np.testing.assert_allclose(x2, x1, rtol=1e-10, atol=1e-12 * np.abs(x1).max())


def test_dipole_reciprocity():
    w = mi.configs.cube8()
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    B = fem.rhs_dipoles(fp, w.dipoles)
    U = spla.splu(fp.A.tocsc()).solve(B)
    G = B.T @ U
    assert np.abs(G - G.T).max() < 1e-12 * np.abs(G).max()
    # the dipole at x0 only touches the 6 edges of its tetrahedron
    assert ((np.abs(B) > 0).sum(axis=0) <= 6).all()


def test_port_reciprocity_and_projection():
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P, nu = fem.port_vectors(fp, w.ports)
    assert (nu > 0).all()
    B = fem.rhs_ports(fp, w.ports, w.tx)
    U = spla.splu(fp.A.tocsc()).solve(B)
    S = np.conj(P.T @ U) / nu[:, None]
    W = nu[:, None] * S
    assert np.abs(W - W.T).max() < 1e-10 * np.abs(W).max()
    # every port vector is supported on the edges of its own faces (the
    # values of p_k and nu_k are pinned on a flat aperture below)
    for k in range(len(w.ports)):
        e = set(fp.dof[fp.bf2e[fp.btag == k + 1].ravel()]) - {-1}
        assert set(np.nonzero(P[:, k])[0]) <= e


def _plane_wave_error(n, k0=2 * np.pi, eps=1 - 0.1j, d=(1.0, 2.0, 2.0), p=(2.0, -1.0, 0.0), pec_z=False):
    """L2 and curl errors of the discrete solution for the plane wave
    E = p exp(-i k d.x) on the cube with N = n cells per side.  Every face
    carries the exact impedance data g = (curl E) x n + i k E_t, except with
    pec_z the faces z = 0 and z = 1, which are metallic (E x n = 0 there
    requires p parallel to z: the TEM wave between two parallel plates)."""
    m = mi.mesh.cube_mesh(n)
    k = k0 * np.sqrt(eps)
    d = np.asarray(d, dtype=float) / np.linalg.norm(d)
    p = np.asarray(p, dtype=float) / np.linalg.norm(p)
    if pec_z:
        zf = m.xyz[m.bface][:, :, 2]
        on_plate = (np.abs(zf).max(axis=1) < 1e-12) | (np.abs(zf - 1.0).max(axis=1) < 1e-12)
        m.btag = np.where(on_plate, fem.TAG_PEC, m.btag).astype(np.int32)
    fp = fem.build(m, np.full(m.nt, eps), k0, k, [])

    def E(x):
        return p * np.exp(-1j * k * (x @ d))[..., None]

    # boundary data g = (curl E) x n + i k E_t on every non-PEC face (outward normals)
    s, area, nrm = fem.face_geometry(fp.xyz, fp.bface)
    cen = fp.xyz[fp.bface].mean(axis=1)
    out = np.sign(((cen - 0.5) * nrm).sum(axis=1))
    nrm = nrm * out[:, None]
    b = np.zeros(fp.n, dtype=complex)
    for f in range(fp.bface.shape[0]):
        if fp.btag[f] == fem.TAG_PEC:
            continue
        X = fp.xyz[fp.bface[f]]
        nn = nrm[f]
        for mu, wq in zip(TRI_Q4, TRI_Q4_W):
            x = mu @ X
            Ex = E(x)
            g = 1j * k * (Ex - nn * (nn @ Ex) - (d @ nn) * Ex + (Ex @ nn) * d)
            for q, (a, bb) in enumerate(fem.TRI_EDGES):
                dof = fp.dof[fp.bf2e[f, q]]
                if dof >= 0:
                    Nq = mu[a] * s[f, bb] - mu[bb] * s[f, a]
                    b[dof] += area[f] * wq * (g @ Nq)
    u = spla.splu(fp.A.tocsc()).solve(b)
    # L2 and curl errors by a degree-3 rule on every tetrahedron; eliminated
    # (PEC) edges carry a zero circulation
    c0, gr, vol = fem.tet_geometry(fp.xyz, fp.tet)
    dt = fp.dof[fp.t2e]
    ut = np.where(dt >= 0, u[np.maximum(dt, 0)], 0.0)
    e2 = c2 = 0.0
    a, bb = fem.TET_EDGES[:, 0], fem.TET_EDGES[:, 1]
    curlN = 2 * np.cross(gr[:, a, :], gr[:, bb, :])
    curl_h = np.einsum("tp,tpk->tk", ut, curlN)
    for lam, wq in zip(TET_Q3_PTS, TET_Q3_W):
        x = np.einsum("a,tak->tk", lam, fp.xyz[fp.tet])
        N = lam[a][None, :, None] * gr[:, bb, :] - lam[bb][None, :, None] * gr[:, a, :]
        Eh = np.einsum("tp,tpk->tk", ut, N)
        Ex = E(x)
        cE = -1j * k * np.cross(d, Ex)
        e2 += (wq * vol * (np.abs(Ex - Eh) ** 2).sum(axis=1)).sum()
        c2 += (wq * vol * (np.abs(cE - curl_h) ** 2).sum(axis=1)).sum()
    return np.sqrt(e2), np.sqrt(c2)


def test_plane_wave_first_order_convergence():
    """Homogeneous plane wave with exact impedance data: lowest-order Nedelec
    converges at O(h) in L2 and in the curl (Monk 2003)."""
    errs = [_plane_wave_error(n) for n in (4, 8, 16)]
    e = np.array(errs)
    rates = np.log2(e[:-1] / e[1:])
    assert (rates[-1] >= 0.9).all(), (e, rates)
    assert e[-1, 0] < 0.15 and e[-1, 1] < 0.8 * 2 * np.pi


def test_parallel_plate_wave_with_pec_walls_converges():
    """E = z exp(-i k x) between metallic plates z = 0 and z = 1 (equation
    (eqmetal): E x n = 0 holds there exactly), exact impedance data on the
    four other faces: with the PEC edges eliminated the discrete solution
    converges at O(h) in L2 and in the curl.  Treating the plates as natural
    (curl E x n = 0) or impedance faces, or eliminating the wrong edges,
    leaves an O(1) error."""
    e = np.array([_plane_wave_error(n, d=(1.0, 0.0, 0.0), p=(0.0, 0.0, 1.0), pec_z=True) for n in (4, 8)])
    rates = np.log2(e[0] / e[1])
    assert (rates >= 0.9).all(), (e, rates)
    assert e[1, 0] < 0.25 and e[1, 1] < 0.25 * 2 * np.pi


def _flat_port(n):
    """Box [2, 3] x [-0.5, 0.5] x [0, 1] with n^3 cells; the face x = 3 is
    the aperture of one port (arc coordinate s = 3 atan2(y, x), width 1,
    polarisation with a normal component), every other face impedance (no
    PEC edge is eliminated, so every edge of the aperture is an unknown)."""
    m = mi.mesh.cube_mesh(n)
    m.xyz = m.xyz + np.array([2.0, -0.5, 0.0])
    xf = m.xyz[m.bface][:, :, 0]
    m.btag = np.where(np.abs(xf - 3.0).max(axis=1) < 1e-12, 1, fem.TAG_IMPEDANCE).astype(np.int32)
    pt = mi.mesh.PortSpec(theta=0.0, z=0.5, width=1.0, height=1.0, radius=3.0, beta=5.0 - 0.5j,
                          pol=(0.5, 0.6, 0.8))
    fp = fem.build(m, np.full(m.nt, 1 - 0.1j), 3.0, 3.0, [pt])
    return fp, pt


def test_port_projection_and_norm_against_exact_integrals():
    """Section 4, equation (sij): p_k[e] = int E0 . N_e and
    nu_k = int |E0_t|^2 over the aperture.  Whitney functions reproduce
    every field c(x) = a + b x x of the lowest-order edge-element space
    exactly from its circulations int_e c . t (= c(midpoint) . t_e, the
    integrand being linear), so sum_e (int_e c . t) p_k[e] = int_Gamma E0 . c_t;
    on the flat aperture x = 3 this and nu_k are integrals of
    cos(pi s / width) times polynomials, computed here by adaptive
    quadrature.  The edge-midpoint rule is exact for quadratics, so the
    discrepancies must fall at least as h^2 under refinement."""
    from scipy.integrate import dblquad, quad

    prof = lambda y: np.cos(np.pi * 3.0 * np.arctan2(y, 3.0))   # noqa: E731
    I2 = quad(lambda y: prof(y) ** 2, -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)[0]
    pol = np.array([0.5, 0.6, 0.8])
    pol_t = pol * np.array([0.0, 1.0, 1.0])                    # tangential part on x = 3
    fields = [(np.array([0.3, -1.2, 0.7]), np.zeros(3)), (np.array([1.0, 0.0, 0.0]), np.zeros(3)),
              (np.array([-0.4, 0.9, 1.1]), np.array([0.5, -0.8, 1.3])),
              (np.zeros(3), np.array([-1.1, 0.4, 0.6]))]
    exact = []
    for a, b in fields:
        f = lambda z, y: prof(y) * (pol_t @ (a + np.cross(b, [3.0, y, z])))   # noqa: E731
        exact.append(dblquad(f, -0.5, 0.5, 0.0, 1.0, epsabs=1e-13, epsrel=1e-13)[0])
    exact = np.array(exact)
    errs_p, errs_nu = [], []
    for n in (4, 8, 16):
        fp, pt = _flat_port(n)
        P, nu = fem.port_vectors(fp, [pt])
        xa, xb = fp.xyz[fp.edges[fp.free, 0]], fp.xyz[fp.edges[fp.free, 1]]
        mid, t = 0.5 * (xa + xb), xb - xa
        lhs = np.array([((a + np.cross(b, mid)) * t).sum(axis=1) @ P[:, 0] for a, b in fields])
        errs_p.append(np.abs(lhs - exact).max() / np.abs(exact).max())
        errs_nu.append(abs(nu[0] - I2 * (pol_t @ pol_t)) / (I2 * (pol_t @ pol_t)))
    errs_p, errs_nu = np.array(errs_p), np.array(errs_nu)
    assert errs_p[-1] < 1e-3 and errs_nu[-1] < 1e-3, (errs_p, errs_nu)
    # entry by entry on the coarsest mesh: the same edge-midpoint rule applied
    # to the tangential traces of the 3-D Whitney functions of the
    # tetrahedron owning each aperture face (barycentric gradients from a
    # 4 x 4 solve, not fem's surface gradients)
    fp, pt = _flat_port(4)
    P, _ = fem.port_vectors(fp, [pt])
    own = fem.face_owner(fp.tet, fp.bface)
    pref = np.zeros(fp.n)
    for f in np.nonzero(fp.btag == 1)[0]:
        tv = fp.tet[own[f]]
        X = fp.xyz[tv]
        fv = fp.bface[f]
        nrm = np.cross(fp.xyz[fv[1]] - fp.xyz[fv[0]], fp.xyz[fv[2]] - fp.xyz[fv[0]])
        area = 0.5 * np.linalg.norm(nrm)
        nrm /= 2 * area
        for u, v in ((0, 1), (0, 2), (1, 2)):
            lam = np.zeros(4)
            lam[np.searchsorted(tv, fv[u])] = lam[np.searchsorted(tv, fv[v])] = 0.5
            x = lam @ X
            e0 = fem.port_mode(pt, x)
            e0t = e0 - (e0 @ nrm) * nrm
            N = whitney_at(X, lam)
            for q, (a, b) in enumerate(fem.TET_EDGES):
                if tv[a] in fv and tv[b] in fv:
                    e = fem.edge_ids(fp.edges, fp.nv, np.array([tv[a]]), np.array([tv[b]]))[0]
                    pref[fp.dof[e]] += area / 3.0 * (e0t @ N[q])
    assert np.abs(P[:, 0] - pref).max() <= 1e-13 * np.abs(pref).max()
    assert (np.log2(errs_p[:-1] / errs_p[1:]) >= 1.9).all(), errs_p
    assert (np.log2(errs_nu[:-1] / errs_nu[1:]) >= 1.9).all(), errs_nu

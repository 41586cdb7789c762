"""Pins of the oracle's outer inversion loop (Section 5: L-BFGS on the
normalised, regularised misfit (defJ2) over a P1 permittivity): adjoint
identities, exact P1 integrals, finite differences of J, the minimiser at
the true parameter, and L-BFGS on a quadratic.  CPU only."""
import numpy as np
import pytest

import mw_inputs as mi
from oracle import fem, inverse, inversion

RNG = np.random.default_rng(17)


@pytest.fixture(scope="module")
def small():
    # 0.15 GHz: 6,146 unknowns, so that every evaluation of J (a sparse LU and
    # 16 solves) takes about a second
    w = mi.configs.small_chamber(0.15e9, n_per_ring=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    return w, fp


def test_vertex_mean_and_its_transpose(small):
    w, fp = small
    nv = fp.xyz.shape[0]
    c = 44 - 20j
    np.testing.assert_allclose(inversion.vertex_mean(fp.tet, np.full(nv, c)), c)
    a = RNG.normal(size=nv) + 1j * RNG.normal(size=nv)
    b = RNG.normal(size=fp.tet.shape[0]) + 1j * RNG.normal(size=fp.tet.shape[0])
    lhs = np.sum(inversion.vertex_mean(fp.tet, a) * b)
    rhs = np.sum(a * inversion.vertex_mean_adjoint(fp.tet, nv, b))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_p1_stiffness_exact_on_linear_fields(small):
    """K1 annihilates constants and integrates |grad(c.x)|^2 = |c|^2 exactly."""
    w, fp = small
    K1 = inversion.stiffness_p1(fp.xyz, fp.tet)
    assert np.abs(K1 @ np.ones(fp.xyz.shape[0])).max() <= 1e-10 * abs(K1).max()
    _, _, vol = fem.tet_geometry(fp.xyz, fp.tet)
    used = np.zeros(fp.xyz.shape[0], dtype=bool)
    used[fp.tet.ravel()] = True
    c = np.array([0.3, -1.2, 2.0])
    e = fp.xyz @ c
    assert abs(e @ (K1 @ e) - (c @ c) * vol.sum()) <= 1e-10 * (c @ c) * vol.sum()


def _objective(w, fp, alpha, seed=5, p1=False):
    """Data from a perturbed vertex permittivity; the empty chamber is the
    homogeneous gel; returns the objective and the true vertex field."""
    nv = fp.xyz.shape[0]
    rng = np.random.default_rng(seed)
    e_gel = np.full(nv, 44 - 20j)
    e_true = e_gel * (1 + 0.05 * rng.normal(size=nv))
    P, nu = fem.port_vectors(fp, w.ports)
    # on this coarse mesh two apertures have all their edges on the PEC wall
    # (P_i = 0, S_ij = 0): use the others
    w.tx = w.rx = np.nonzero(np.abs(P).sum(axis=0) > 0)[0].astype(np.int32)
    B = fem.rhs_ports(fp, w.ports, w.tx)

    def S_of(ev):
        f = fem.with_eps_vertex(fp, ev) if p1 else fem.with_eps(fp, inversion.vertex_mean(fp.tet, ev))
        import scipy.sparse.linalg as spla
        return inverse.s_matrix(P, nu, spla.splu(f.A.tocsc()).solve(B), w.rx)

    return inversion.Objective(fp, w.ports, w.tx, w.rx, S_of(e_true), S_of(e_gel), alpha, p1=p1), e_gel, e_true


@pytest.mark.parametrize("alpha,p1", [(0.0, False), (1e-3, False), (0.0, True), (1e-3, True)])
def test_objective_gradient_matches_finite_differences(small, alpha, p1):
    w, fp = small
    obj, e_gel, _ = _objective(w, fp, alpha, p1=p1)
    J, g, _ = obj(e_gel)
    nv = fp.xyz.shape[0]
    for k in range(3):
        d = RNG.normal(size=nv) + 1j * RNG.normal(size=nv)
        h = 1e-4
        Jp, _, _ = obj(e_gel + h * d)
        Jm, _, _ = obj(e_gel - h * d)
        fd = (Jp - Jm) / (2 * h)
        an = float(np.sum((np.conj(g) * d).real))
        assert abs(an - fd) <= 1e-5 * abs(fd), (k, an, fd)


@pytest.mark.parametrize("p1", [False, True])
def test_true_parameter_is_a_minimiser(small, p1):
    """Without regularisation J = 0 and grad J = 0 at the parameter that made the data."""
    w, fp = small
    obj, _, e_true = _objective(w, fp, 0.0, p1=p1)
    J, g, _ = obj(e_true)
    J0, g0, _ = obj(np.full(fp.xyz.shape[0], 44 - 20j))
    assert J <= 1e-20 * J0
    assert np.abs(g).max() <= 1e-9 * np.abs(g0).max()


def test_lbfgs_minimises_a_quadratic():
    """J(e) = 1/2 x^T Q x - b^T x over x = [Re e; Im e] (Q SPD): the iterates
    decrease J monotonically and reach Q^-1 b."""
    n = 12
    rng = np.random.default_rng(3)
    M = rng.normal(size=(2 * n, 2 * n))
    Q = M @ M.T + 2 * n * np.eye(2 * n)
    b = rng.normal(size=2 * n)
    xs = np.linalg.solve(Q, b)

    def fun(e):
        x = np.concatenate([e.real, e.imag])
        gx = Q @ x - b
        return 0.5 * x @ Q @ x - b @ x, gx[:n] + 1j * gx[n:], None

    es, Js, nev = inversion.lbfgs(fun, np.zeros(n, dtype=complex), iters=60, mem=5, step0=0.1)
    assert all(Js[k + 1] <= Js[k] for k in range(len(Js) - 1))
    x = np.concatenate([es[-1].real, es[-1].imag])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_lbfgs_reduces_the_chamber_misfit(small):
    w, fp = small
    obj, e_gel, e_true = _objective(w, fp, 1e-4)
    es, Js, nev = inversion.lbfgs(obj, e_gel, iters=3, step0=0.5)
    assert len(Js) == 4 and all(Js[k + 1] < Js[k] for k in range(3))
    assert Js[-1] < 0.5 * Js[0]

"""Pins of the oracle's block GMRES (the block Krylov method of the paper's
conclusion, textbook form) against finite termination, brute-force minimal
residuals over the block Krylov space, direct solves and its breakdown rules.
CPU only."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import dd, fem, gmres


@pytest.fixture(scope="module")
def cube4():
    w = mi.configs.cube(4, n_sub=4, ndip=3)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    subs = dd.decompose(fp, w.part, 1)
    B = fem.rhs_dipoles(fp, w.dipoles)
    return fp, subs, B


def _cplx(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_block_krylov_space_fills_in_n_over_p_steps():
    """n = 12, p = 4, no preconditioner: after 3 block steps the block Krylov
    space is all of C^12 (generically), so the solution is exact."""
    rng = np.random.default_rng(1)
    A = _cplx(rng, 12, 12)
    B = _cplx(rng, 12, 4)
    X, it, rr = gmres.block_gmres(A, B, lambda V: V, tol=1e-13, p=4)
    assert (it == 3).all()
    np.testing.assert_allclose(X, np.linalg.solve(A, B), atol=1e-12 * np.abs(np.linalg.solve(A, B)).max())


def test_block_minimal_residual_property(cube4):
    """Without restart, k block steps attain, for every column c, the minimum
    of ||b_c - A M^-1 y|| over the block Krylov space
    span{R0, (A M^-1) R0, ..., (A M^-1)^(k-1) R0}: compare with a least-squares
    solve over an explicitly built basis.  That space contains column c's own
    Krylov space, so the residual is also no larger than ordinary GMRES's
    after k steps."""
    fp, subs, B = cube4
    prec = lambda V: dd.oras_apply(subs, V)  # noqa: E731
    for k in (1, 2, 3):
        X, it, rr = gmres.block_gmres(fp.A, B, prec, tol=1e-30, restart=50, maxit=k, p=3)
        blocks = [B]
        for _ in range(k - 1):
            blocks.append(fp.A @ prec(blocks[-1]))
        Q, _ = np.linalg.qr(np.concatenate(blocks, axis=1))
        AMQ = fp.A @ prec(Q)
        assert (it == k).all()
        _, it1, rr1 = gmres.gmres(fp.A, B, prec, tol=1e-30, restart=50, maxit=k)
        for c in range(B.shape[1]):
            y = np.linalg.lstsq(AMQ, B[:, c], rcond=None)[0]
            best = np.linalg.norm(B[:, c] - AMQ @ y) / np.linalg.norm(B[:, c])
            assert abs(rr[c] - best) <= 1e-8 * best + 1e-14
            assert rr[c] <= rr1[c] * (1 + 1e-8)


def test_block_gmres_matches_direct_with_restarts(cube4):
    fp, subs, B = cube4
    U = spla.splu(fp.A.tocsc()).solve(B)
    prec = lambda V: dd.oras_apply(subs, V)  # noqa: E731
    for m, p in ((30, 3), (2, 2), (3, 1)):    # short m forces restarts; p = 2 leaves a ragged block
        X, it, rr = gmres.block_gmres(fp.A, B, prec, tol=1e-11, restart=m, p=p)
        assert (rr <= 1e-11).all()
        err = np.linalg.norm(X - U, axis=0) / np.linalg.norm(U, axis=0)
        assert (err < 1e-8).all(), (m, p, err)


def test_block_size_one_is_ordinary_gmres(cube4):
    fp, subs, B = cube4
    prec = lambda V: dd.oras_apply(subs, V)  # noqa: E731
    X1, it1, _ = gmres.block_gmres(fp.A, B, prec, tol=1e-10, p=1)
    X0, it0, _ = gmres.gmres(fp.A, B, prec, tol=1e-10)
    np.testing.assert_array_equal(it1, it0)
    np.testing.assert_allclose(X1, X0, atol=1e-9 * np.abs(X0).max())


def test_rank_deficient_start_falls_back_to_ordinary_gmres(cube4):
    """A repeated right-hand side makes the starting block rank deficient;
    its block leaves block mode and still converges."""
    fp, subs, B = cube4
    B2 = np.concatenate([B, B[:, :1]], axis=1)
    U = spla.splu(fp.A.tocsc()).solve(B2)
    prec = lambda V: dd.oras_apply(subs, V)  # noqa: E731
    X, it, rr = gmres.block_gmres(fp.A, B2, prec, tol=1e-11, p=4)
    _, it0, _ = gmres.gmres(fp.A, B2, prec, tol=1e-11)
    np.testing.assert_array_equal(it, it0)
    assert (rr <= 1e-11).all()
    np.testing.assert_allclose(X, U, atol=1e-8 * np.abs(U).max())


def test_lucky_breakdown_ends_the_cycle_exactly():
    """When A M^-1 = I the first new block is zero: step 0 alone solves the
    system and the cycle ends there."""
    rng = np.random.default_rng(2)
    A = _cplx(rng, 20, 20) + 8 * np.eye(20)
    B = _cplx(rng, 20, 3)
    Ainv = np.linalg.inv(A)
    X, it, rr = gmres.block_gmres(A, B, lambda V: Ainv @ V, tol=1e-13, p=3)
    assert (it == 1).all() and (rr <= 1e-13).all()

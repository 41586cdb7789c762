"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances:
  * assembly, sources, port projections: 1e-13 relative (same formulas, FP64,
    different summation order);
  * FP64 preconditioner apply: 1e-11 relative (dense LU vs sparse LU of the
    same B_i, well conditioned local problems);
  * fields: relative L2 <= 1e-6 per column against a sparse direct solve,
    GMRES run to 1e-10 (forward error <= cond * residual);
  * mixed precision (complex FP32 factors): preconditioner 1e-5, fields 1e-6
    (the outer FP64 GMRES with iterative refinement reaches the same
    tolerance).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import dd, fem, gmres, inverse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def ctx():
    from paper_1607_02573_amd import solver
    c = solver.Context(0)
    yield c


@pytest.fixture(scope="module")
def cube(ctx):
    from paper_1607_02573_amd import solver
    w = mi.configs.cube8()
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P = solver.problem_from_workload(ctx, w)
    yield w, fp, P
    P.close()


@pytest.fixture(scope="module")
def chamber_small(ctx):
    from paper_1607_02573_amd import solver
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P = solver.problem_from_workload(ctx, w)
    yield w, fp, P
    P.close()


def _gpu_csr(P):
    rp, col, val = P.matrix()
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(P.n, P.n))


@pytest.mark.parametrize("which", ["cube", "chamber_small"])
def test_matrix_matches_oracle(which, request):
    w, fp, P = request.getfixturevalue(which)
    A = _gpu_csr(P)
    Ao = fp.A.tocsr()
    Ao.sort_indices()
    assert np.array_equal(A.indptr, Ao.indptr) and np.array_equal(A.indices, Ao.indices)
    assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max()
    eod, _ = P.dof_edges()
    assert np.array_equal(eod, fp.free)


def test_dipole_rhs(cube):
    w, fp, P = cube
    Bg = P.rhs_dipoles(w.dipoles).cpu().numpy()
    Bo = fem.rhs_dipoles(fp, w.dipoles)
    assert np.abs(Bg - Bo).max() <= 1e-13 * np.abs(Bo).max()


def test_port_rhs_and_norms(chamber_small):
    w, fp, P = chamber_small
    Po, nuo = fem.port_vectors(fp, w.ports)
    np.testing.assert_allclose(P.port_norms(), nuo, rtol=1e-13)
    Bg = P.rhs_ports(w.tx).cpu().numpy()
    Bo = fem.rhs_ports(fp, w.ports, w.tx)
    assert np.abs(Bg - Bo).max() <= 1e-13 * np.abs(Bo).max()


@pytest.fixture(params=["recursive", "rows"])
def form(request):
    """Both forms of the subdomain triangular solves (the automatic choice
    takes the recursive one at these sizes); back to automatic afterwards."""
    return request.param


def _factor(P, w, prec, form):
    P.set_solve_form(form)
    try:
        P.factor(w.part, w.n_sub, 1, prec)
    finally:
        P.set_solve_form("auto")


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-5)])
@pytest.mark.parametrize("which", ["cube", "chamber_small"])
def test_preconditioner_matches_oracle(which, prec, tol, form, request):
    w, fp, P = request.getfixturevalue(which)
    _factor(P, w, prec, form)
    subs = dd.decompose(fp, w.part, 1)
    rng = np.random.default_rng(11)
    V = rng.normal(size=(P.n, 5)) + 1j * rng.normal(size=(P.n, 5))
    Zg = P.apply_preconditioner(torch.from_numpy(V).cuda()).cpu().numpy()
    Zo = dd.oras_apply(subs, V)
    assert _rel(Zg, Zo) <= tol


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_cube_solve_matches_direct(cube, prec, form):
    w, fp, P = cube
    _factor(P, w, prec, form)
    Bo = fem.rhs_dipoles(fp, w.dipoles)
    X, info = P.solve(torch.from_numpy(Bo).cuda(), tol=1e-10, restart=30)
    U = spla.splu(fp.A.tocsc()).solve(Bo)
    err = np.linalg.norm(X.cpu().numpy() - U, axis=0) / np.linalg.norm(U, axis=0)
    assert (err <= 1e-6).all(), err
    assert (info.relres <= 1e-10).all()
    if prec == "c128":
        # same preconditioner, same Krylov process: same iteration counts as the oracle
        subs = dd.decompose(fp, w.part, 1)
        _, it_o, _ = gmres.gmres(fp.A, Bo, lambda V: dd.oras_apply(subs, V), tol=1e-10, restart=30)
        assert np.abs(info.iters - it_o).max() <= 1, (info.iters, it_o)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_chamber_solve_and_s_matrix(chamber_small, prec, form):
    w, fp, P = chamber_small
    _factor(P, w, prec, form)
    Bg = P.rhs_ports(w.tx)
    X, info = P.solve(Bg, tol=1e-10, restart=30)
    lu = spla.splu(fp.A.tocsc())
    U = lu.solve(fem.rhs_ports(fp, w.ports, w.tx))
    Xc = X.cpu().numpy()
    err = np.linalg.norm(Xc - U, axis=0) / np.linalg.norm(U, axis=0)
    assert (err <= 1e-6).all(), err
    Po, nuo = fem.port_vectors(fp, w.ports)
    So = inverse.s_matrix(Po, nuo, U, w.rx)
    Sg = P.s_matrix(X, w.rx).cpu().numpy()
    assert _rel(Sg, So) <= 1e-6
    # reciprocity of the GPU S-matrix: nu_i S_ij = nu_j S_ji
    W = nuo[:, None] * Sg
    assert np.abs(W - W.T).max() <= 1e-6 * np.abs(W).max()


@pytest.mark.parametrize("n", [1, 2])
def test_tiny_cubes_dense_bruteforce(ctx, n):
    from paper_1607_02573_amd import solver
    m = mi.mesh.cube_mesh(n)
    eps = np.full(m.nt, 1 - 0.1j)
    k0 = 3.0
    P = solver.Problem(ctx, m.xyz, m.tet, m.bface, m.btag, eps, k0, k0 * np.sqrt(1 - 0.1j), [])
    fp = fem.build(m, eps, k0, k0 * np.sqrt(1 - 0.1j), [])
    part = mi.partition.rcb(m, 2 if n == 2 else 1)
    P.factor(part, int(part.max()) + 1, 1, "c128")
    rng = np.random.default_rng(n)
    b = rng.normal(size=(P.n, 3)) + 1j * rng.normal(size=(P.n, 3))
    X, info = P.solve(torch.from_numpy(b).cuda(), tol=1e-12, restart=50)
    xd = np.linalg.solve(fp.A.toarray(), b)
    assert _rel(X.cpu().numpy(), xd) <= 1e-9
    P.close()


def test_batch_invariance_and_reproducibility(chamber_small):
    """Pseudo-block columns are independent: a column solved alone equals the
    same column solved among others, bit for bit; a rerun is bitwise equal."""
    w, fp, P = chamber_small
    for prec in ("c128", "c64"):
        P.factor(w.part, w.n_sub, 1, prec)
        Bg = P.rhs_ports(w.tx)
        Xall, _ = P.solve(Bg, tol=1e-9)
        Xall2, _ = P.solve(Bg, tol=1e-9)
        assert torch.equal(Xall, Xall2)
        for j in (0, 3, 7):
            Xj, _ = P.solve(Bg[:, j:j + 1].contiguous(), tol=1e-9)
            assert torch.equal(Xj[:, 0], Xall[:, j]), (prec, j)
        Xs, _ = P.solve(Bg[:, 2:5].contiguous(), tol=1e-9)
        assert torch.equal(Xs, Xall[:, 2:5])


def test_adjoint_gradient_matches_oracle_and_fd(chamber_small):
    """Section 5: the GPU adjoint gradient (factors reused) against the oracle's
    adjoint gradient and exact (Woodbury) central differences."""
    w, fp, P = chamber_small
    P.factor(w.part, w.n_sub, 1, "c128")
    rng = np.random.default_rng(21)
    eps_true = w.eps * (1 + 0.05 * rng.normal(size=w.eps.size))
    lu = spla.splu(fp.A.tocsc())
    Bo = fem.rhs_ports(fp, w.ports, w.tx)
    U = lu.solve(Bo)
    Po, nuo = fem.port_vectors(fp, w.ports)
    Smes = inverse.s_matrix(Po, nuo, spla.splu(fem.with_eps(fp, eps_true).A.tocsc()).solve(Bo), w.rx)
    J_o, S_o, g_o = inverse.adjoint_gradient(fp, lu, Po, nuo, U, w.tx, w.rx, Smes)
    J, S, g = P.misfit_gradient(w.tx, w.rx, torch.from_numpy(Smes).cuda(), tol=1e-11)
    g = g.cpu().numpy()
    assert abs(J - J_o) <= 1e-7 * J_o
    assert _rel(S.cpu().numpy(), S_o) <= 1e-7
    assert _rel(g, g_o) <= 1e-6
    for t in np.argsort(-np.abs(g_o))[:4]:
        h = 1e-4 * abs(fp.eps[t])
        fd = (inverse.woodbury_fd(fp, lu, U, Bo, Po, nuo, w.rx, Smes, t, h)
              + 1j * inverse.woodbury_fd(fp, lu, U, Bo, Po, nuo, w.rx, Smes, t, 1j * h))
        assert abs(g[t] - fd) <= 1e-5 * abs(fd), (t, g[t], fd)


def test_autograd_function(chamber_small):
    from paper_1607_02573_amd.autograd import s_of_eps
    w, fp, P = chamber_small
    eps = torch.from_numpy(w.eps.copy()).cuda().requires_grad_(True)
    S = s_of_eps(eps, P, w.part, w.n_sub, w.tx, w.rx, tol=1e-11)
    Smes = S.detach() * 0.97
    J = 0.5 * (S - Smes).abs().pow(2).sum()
    J.backward()
    lu = spla.splu(fp.A.tocsc())
    Po, nuo = fem.port_vectors(fp, w.ports)
    U = lu.solve(fem.rhs_ports(fp, w.ports, w.tx))
    _, _, g_o = inverse.adjoint_gradient(fp, lu, Po, nuo, U, w.tx, w.rx, Smes.cpu().numpy())
    assert _rel(eps.grad.cpu().numpy(), g_o) <= 1e-6


def test_error_paths(ctx):
    from paper_1607_02573_amd import binding, solver
    m = mi.mesh.cube_mesh(4)
    # singular local problems: kappa = 0 and PEC everywhere (curl-curl kernel)
    btag = np.full(m.btag.shape, -1, dtype=np.int32)
    P = solver.Problem(ctx, m.xyz, m.tet, m.bface, btag, np.zeros(m.nt, complex), 3.0, 0.0, [])
    part = mi.partition.rcb(m, 2)
    with pytest.raises(binding.MwError) as e:
        P.factor(part, 2, 1, "c128")
    assert e.value.code == binding.MW_ESINGULAR
    with pytest.raises(binding.MwError) as e:
        P.factor(np.full(m.nt, 5, dtype=np.int32), 2, 1, "c128")
    assert e.value.code == binding.MW_EINVAL
    P.close()
    # a budget far too small for the factors: MW_ENOMEM, nothing left allocated
    small = solver.Context(0, budget_bytes=8 << 20)
    w = mi.configs.cube8()
    P2 = solver.problem_from_workload(small, w)
    with pytest.raises(binding.MwError) as e:
        P2.factor(w.part, w.n_sub, 1, "c128")
    assert e.value.code == binding.MW_ENOMEM
    P2.close()
    small.close()
    # solving before factoring
    P3 = solver.problem_from_workload(ctx, w)
    with pytest.raises(binding.MwError) as e:
        P3.solve(P3.rhs_dipoles(w.dipoles))
    assert e.value.code == binding.MW_EINVAL
    # no convergence within maxit: MW_ENOCONV, X holds the last iterate
    P3.factor(w.part, w.n_sub, 1, "c128")
    X, info = P3.solve(P3.rhs_dipoles(w.dipoles), tol=1e-12, maxit=3, raise_noconv=False)
    assert (info.iters == 3).all() and (info.relres > 1e-12).all()
    with pytest.raises(binding.MwError) as e:
        P3.solve(P3.rhs_dipoles(w.dipoles), tol=1e-12, maxit=3)
    assert e.value.code == binding.MW_ENOCONV
    P3.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_preconditioner_column_counts(chamber_small, prec, tol, form):
    """Every tile width of the batched triangular solves (1 .. >160 columns)."""
    w, fp, P = chamber_small
    _factor(P, w, prec, form)
    subs = dd.decompose(fp, w.part, 1)
    rng = np.random.default_rng(5)
    for nc in (1, 3, 33, 65, 97, 130, 170):
        V = rng.normal(size=(P.n, nc)) + 1j * rng.normal(size=(P.n, nc))
        Zg = P.apply_preconditioner(torch.from_numpy(V).cuda()).cpu().numpy()
        Zo = dd.oras_apply(subs, V)
        # per column
        err = np.linalg.norm(Zg - Zo, axis=0) / np.linalg.norm(Zo, axis=0)
        assert err.max() <= tol, (nc, err.max())
        # each column is independent of the others (bitwise)
        Z1 = P.apply_preconditioner(torch.from_numpy(np.ascontiguousarray(V[:, :1])).cuda()).cpu().numpy()
        assert np.array_equal(Z1[:, 0], Zg[:, 0]), nc


def test_fp32_krylov_basis_reaches_the_same_solution(chamber_small):
    """Mixed precision keeps the Arnoldi basis in complex FP32 by default; the
    stopping test stays on the true FP64 residual, so every basis kind (FP64,
    FP32 with the preconditioned candidates kept, FP32 lean) reaches the
    tolerance and the same fields (within what the tolerance allows), with
    at most a few more iterations for the rounded basis."""
    w, fp, P = chamber_small
    P.factor(w.part, w.n_sub, 1, "c64")
    Bg = P.rhs_ports(w.tx)
    out = {}
    for kind in ("fp64", "auto", "fp32-lean"):
        P.set_krylov_basis(kind)
        try:
            out[kind] = P.solve(Bg, tol=1e-10, restart=30)
        finally:
            P.set_krylov_basis("auto")
    (X64, i64), (X32, i32), (XL, iL) = out["fp64"], out["auto"], out["fp32-lean"]
    assert (i64.relres <= 1e-10).all() and (i32.relres <= 1e-10).all() and (iL.relres <= 1e-10).all()
    U = spla.splu(fp.A.tocsc()).solve(fem.rhs_ports(fp, w.ports, w.tx))
    for X in (X64, X32, XL):
        err = np.linalg.norm(X.cpu().numpy() - U, axis=0) / np.linalg.norm(U, axis=0)
        assert (err <= 1e-6).all(), err.max()
    assert (i32.iters <= i64.iters + 3).all(), (i32.iters, i64.iters)
    assert (iL.iters <= i64.iters + 3).all(), (iL.iters, i64.iters)

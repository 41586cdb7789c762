"""Both subdomain factorisations (LU with partial pivoting, L D L^T without
interchanges) on the GPU: the same preconditioner to rounding, the same
solutions against the oracle's direct solve, and the automatic choice."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import dd, fem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def chamber():
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P = solver.problem_from_workload(ctx, w)
    yield w, fp, P
    P.set_factorization("auto")
    P.close()
    ctx.close()


@pytest.mark.parametrize("form", ["recursive", "rows"])
@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 2e-5)])
def test_ldlt_and_lu_give_the_same_preconditioner(chamber, prec, tol, form):
    """M^-1 V with either factorisation, and either form of the triangular
    solves, equals the oracle's ORAS apply (sparse LU of every B_i) to the
    factor precision."""
    w, fp, P = chamber
    P.set_solve_form(form)
    subs = dd.decompose(fp, w.part, 1)
    rng = np.random.default_rng(11)
    V = rng.normal(size=(fp.n, 40)) + 1j * rng.normal(size=(fp.n, 40))
    Zo = dd.oras_apply(subs, V)
    Vg = torch.from_numpy(V).cuda()
    out = {}
    for kind in ("lu", "ldlt"):
        P.set_factorization(kind)
        P.factor(w.part, w.n_sub, 1, prec)
        assert P.info().factorization == {"lu": 1, "ldlt": 2}[kind]
        out[kind] = P.apply_preconditioner(Vg).cpu().numpy()
        err = np.linalg.norm(out[kind] - Zo) / np.linalg.norm(Zo)
        assert err <= tol, (kind, err)
    P.set_factorization("auto")
    P.set_solve_form("auto")


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ldlt_solutions_match_direct(chamber, prec):
    w, fp, P = chamber
    P.set_factorization("ldlt")
    P.factor(w.part, w.n_sub, 1, prec)
    Bo = np.ascontiguousarray(fem.rhs_ports(fp, w.ports, w.tx))
    X, info = P.solve(torch.from_numpy(Bo).cuda(), tol=1e-10)
    U = spla.splu(fp.A.tocsc()).solve(Bo)
    err = np.linalg.norm(X.cpu().numpy() - U, axis=0) / np.linalg.norm(U, axis=0)
    assert (info.relres <= 1e-10).all() and (err <= 1e-7).all(), err.max()
    P.set_factorization("lu")
    P.factor(w.part, w.n_sub, 1, prec)
    _, info_lu = P.solve(torch.from_numpy(Bo).cuda(), tol=1e-10)
    assert np.abs(info.iters - info_lu.iters).max() <= (0 if prec == "c128" else 2)
    P.set_factorization("auto")


def test_automatic_choice():
    """Lossy everywhere: L D L^T; one lossless tetrahedron: LU."""
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.cube(4, n_sub=2, ndip=2)
    P = solver.problem_from_workload(ctx, w)
    P.factor(w.part, w.n_sub, 1, "c128")
    assert P.info().factorization == 2
    eps = w.eps.copy()
    eps[7] = eps[7].real + 0j
    P.update_eps(torch.from_numpy(eps).cuda())
    P.factor(w.part, w.n_sub, 1, "c128")
    assert P.info().factorization == 1
    P.close()
    ctx.close()


def test_refused_factorisation_kind(chamber):
    from paper_1607_02573_amd import binding
    w, fp, P = chamber
    with pytest.raises(binding.MwError) as e:
        binding.check(binding.lib().mw_set_factorization(P.h, 7))
    assert e.value.code == binding.MW_EINVAL


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 2e-5)])
def test_refactoring_after_new_permittivity_and_kind(chamber, prec, tol):
    """A refill after a factorisation without interchanges clears only the
    band of every B_i (the rest is still zero); after LU with interchanges it
    clears everything.  Factor a sequence of permittivities and kinds and
    check every preconditioner against the oracle's for that permittivity."""
    w, fp, P = chamber
    rng = np.random.default_rng(12)
    V = rng.normal(size=(fp.n, 8)) + 1j * rng.normal(size=(fp.n, 8))
    Vg = torch.from_numpy(V).cuda()
    for step, kind in enumerate(("ldlt", "ldlt", "lu", "ldlt", "ldlt")):
        eps = w.eps * (1.0 + 0.05 * step)
        P.update_eps(torch.from_numpy(np.ascontiguousarray(eps)).cuda())
        P.set_factorization(kind)
        P.factor(w.part, w.n_sub, 1, prec)
        Zo = dd.oras_apply(dd.decompose(fem.with_eps(fp, eps), w.part, 1), V)
        Z = P.apply_preconditioner(Vg).cpu().numpy()
        err = np.linalg.norm(Z - Zo) / np.linalg.norm(Zo)
        assert err <= tol, (step, kind, err)
    P.update_eps(torch.from_numpy(np.ascontiguousarray(w.eps)).cuda())
    P.set_factorization("auto")

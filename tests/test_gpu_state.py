"""GPU checks of the library's state handling through the C ABI, each
against the FP64 oracle:

* the internal partition (tet_part = NULL) gives the same preconditioner as
  the oracle's ORAS on the partition mw_host_partition reports;
* overlap delta = 2 (Section 3's recursion taken twice) against the oracle;
* a failed L D L^T factorisation (singular local matrices) leaves nothing
  behind: refactoring with a valid permittivity gives the oracle's
  preconditioner again;
* non-finite data end in MW_ENUMERIC (permittivity: at factorisation;
  right-hand side: in the solve);
* the autograd backward uses the operator of its own forward pass even when
  another forward pass changed the problem in between (Section 5: the adjoint
  problem has the state problem's operator).
Per-column relative bounds: 1e-11 (FP64 factors), 1e-5 (FP32 factors), as
in the other parity tests.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import dd, fem, inverse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _colerr(Zg, Zo):
    return (np.linalg.norm(Zg - Zo, axis=0) / np.linalg.norm(Zo, axis=0)).max()


@pytest.fixture(scope="module")
def small():
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P = solver.problem_from_workload(ctx, w)
    yield w, fp, P
    P.close()
    ctx.close()


def _apply_both(P, subs, nc, seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(P.n, nc)) + 1j * rng.normal(size=(P.n, nc))
    Zg = P.apply_preconditioner(torch.from_numpy(V).cuda()).cpu().numpy()
    return Zg, dd.oras_apply(subs, V)


def test_internal_partition_matches_oracle(small):
    from paper_1607_02573_amd import binding
    w, fp, P = small
    m = w.mesh
    print("[state] internal partition, 11 parts", flush=True)
    part = binding.host_partition(m.xyz, m.tet, m.bface, m.btag, 11)
    P.factor(None, 11, 1, "c128")
    assert P.info().n_sub == 11
    assert P.factor_bytes(None, 11, 1, "c128") == P.info().factor_bytes
    Zg, Zo = _apply_both(P, dd.decompose(fp, part, 1), 5, 1)
    assert _colerr(Zg, Zo) <= 1e-11


def test_overlap_two_matches_oracle(small):
    w, fp, P = small
    print("[state] overlap 2", flush=True)
    subs = dd.decompose(fp, w.part, 2)
    for prec, tol in (("c128", 1e-11), ("c64", 1e-5)):
        P.factor(w.part, w.n_sub, 2, prec)
        Zg, Zo = _apply_both(P, subs, 7, 2)
        assert _colerr(Zg, Zo) <= tol, prec
    X, info = P.solve(P.rhs_ports(w.tx[:4]), tol=1e-10)
    U = spla.splu(fp.A.tocsc()).solve(fem.rhs_ports(fp, w.ports, w.tx[:4]))
    assert _colerr(X.cpu().numpy(), U) <= 1e-6


def test_failed_ldlt_leaves_no_stale_factors(small):
    """A successful L D L^T first (so that a refill would clear the band
    only), then a forced L D L^T of singular local matrices (eps = 0: the
    curl-curl kernel), then the valid permittivity again."""
    from paper_1607_02573_amd import binding
    w, fp, P = small
    subs = dd.decompose(fp, w.part, 1)
    eps = torch.from_numpy(w.eps).cuda()
    P.set_factorization("ldlt")
    try:
        for prec, tol in (("c64", 1e-5), ("c128", 1e-11)):
            print(f"[state] failed L D L^T then refactor, {prec}", flush=True)
            P.update_eps(eps)
            P.factor(w.part, w.n_sub, 1, prec)
            P.update_eps(torch.zeros_like(eps))
            with pytest.raises(binding.MwError) as e:
                P.factor(w.part, w.n_sub, 1, prec)
            assert e.value.code == binding.MW_ESINGULAR
            assert P.info().factorization == 0
            with pytest.raises(binding.MwError):
                P.apply_preconditioner(torch.ones((P.n, 1), dtype=torch.complex128, device="cuda"))
            P.update_eps(eps)
            P.factor(w.part, w.n_sub, 1, prec)
            assert P.info().factorization == binding.MW_FACTOR_LDLT
            Zg, Zo = _apply_both(P, subs, 3, 3)
            assert _colerr(Zg, Zo) <= tol, prec
    finally:
        P.set_factorization("auto")


def test_non_finite_inputs_raise_enumeric(small):
    from paper_1607_02573_amd import binding
    w, fp, P = small
    print("[state] non-finite permittivity and right-hand side", flush=True)
    e = w.eps.copy()
    e[17] = np.nan
    P.update_eps(torch.from_numpy(e).cuda())
    with pytest.raises(binding.MwError) as err:
        P.factor(w.part, w.n_sub, 1, "c64")
    assert err.value.code == binding.MW_ENUMERIC
    e[17] = complex(np.inf, -1.0)
    P.update_eps(torch.from_numpy(e).cuda())
    with pytest.raises(binding.MwError) as err:
        P.factor(w.part, w.n_sub, 1, "c64")
    assert err.value.code == binding.MW_ENUMERIC
    P.update_eps(torch.from_numpy(w.eps).cuda())
    P.factor(w.part, w.n_sub, 1, "c64")
    Bm = P.rhs_ports(w.tx[:3])
    Bm[5, 1] = complex(np.nan, 0.0)
    with pytest.raises(binding.MwError) as err:
        P.solve(Bm, tol=1e-8)
    assert err.value.code == binding.MW_ENUMERIC


def test_backward_after_another_forward_uses_its_own_operator(small):
    from paper_1607_02573_amd.autograd import s_of_eps
    w, fp, P = small
    print("[state] autograd: two forward passes, backward on the first", flush=True)
    rng = np.random.default_rng(8)
    e1 = w.eps.copy()
    e2 = w.eps * (1 + 0.1 * rng.normal(size=w.eps.size))
    eps1 = torch.from_numpy(e1).cuda().requires_grad_(True)
    eps2 = torch.from_numpy(e2).cuda().requires_grad_(True)
    S1 = s_of_eps(eps1, P, w.part, w.n_sub, w.tx, w.rx, tol=1e-11)
    S2 = s_of_eps(eps2, P, w.part, w.n_sub, w.tx, w.rx, tol=1e-11)
    Smes = (S1.detach() * 0.97).cpu().numpy()
    J = 0.5 * (S1 - torch.from_numpy(Smes).cuda()).abs().pow(2).sum()
    J.backward()
    lu = spla.splu(fp.A.tocsc())
    Po, nuo = fem.port_vectors(fp, w.ports)
    U = lu.solve(fem.rhs_ports(fp, w.ports, w.tx))
    _, _, g_o = inverse.adjoint_gradient(fp, lu, Po, nuo, U, w.tx, w.rx, Smes)
    g = eps1.grad.cpu().numpy()
    assert np.linalg.norm(g - g_o) <= 1e-6 * np.linalg.norm(g_o)
    assert S2.shape == S1.shape

"""GPU parity of the two-level preconditioner (mw_set_coarse_space, the
coarse space of three weighted constant fields per subdomain) against the
oracle's two-level ORAS (oracle/coarse.py) on the same partition:

* the apply Z = M2^-1 V, per column, 1e-11 (FP64 factors) and 1e-5 (FP32);
* GMRES iteration counts of the oracle's two-level GMRES (+-1) and fields
  within 1e-6 of a sparse direct solve;
* a column solved alone or among others gives the same bits;
* the coarse size is reported, mw_apply_preconditioner_noalloc refuses the
  two-level form, and switching the coarse space off gives the one-level
  preconditioner again.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import coarse, dd, fem, gmres

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _colerr(Zg, Zo):
    return (np.linalg.norm(Zg - Zo, axis=0) / np.linalg.norm(Zo, axis=0)).max()


@pytest.fixture(scope="module", params=["cube8", "small_chamber"])
def case(request):
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.cube8() if request.param == "cube8" else mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    subs = dd.decompose(fp, w.part, 1)
    M2 = coarse.TwoLevel(fp, subs, "const")
    P = solver.problem_from_workload(ctx, w)
    yield request.param, w, fp, subs, M2, P
    P.close()
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_two_level_apply_matches_oracle(case, prec, tol):
    name, w, fp, subs, M2, P = case
    print(f"[coarse] {name} {prec}: two-level apply", flush=True)
    P.set_coarse_space("const")
    P.factor(w.part, w.n_sub, 1, prec)
    assert P.info().coarse_size == 3 * w.n_sub == M2.size
    rng = np.random.default_rng(12)
    for nc in (1, 5, 33):
        V = rng.normal(size=(P.n, nc)) + 1j * rng.normal(size=(P.n, nc))
        Zg = P.apply_preconditioner(torch.from_numpy(V).cuda()).cpu().numpy()
        assert _colerr(Zg, M2.apply(V)) <= tol, nc


def test_two_level_gmres_matches_oracle(case):
    name, w, fp, subs, M2, P = case
    print(f"[coarse] {name}: two-level GMRES vs oracle", flush=True)
    B = np.ascontiguousarray(fem.rhs_dipoles(fp, w.dipoles) if w.dipoles is not None
                             else fem.rhs_ports(fp, w.ports, w.tx[:4]))
    _, it_o, _ = gmres.gmres(fp.A, B, M2, tol=1e-10)
    _, it_1, _ = gmres.gmres(fp.A, B, lambda V: dd.oras_apply(subs, V), tol=1e-10)
    U = spla.splu(fp.A.tocsc()).solve(B)
    P.set_coarse_space("const")
    for prec in ("c128", "c64"):
        P.factor(w.part, w.n_sub, 1, prec)
        X, info = P.solve(torch.from_numpy(B).cuda(), tol=1e-10)
        assert _colerr(X.cpu().numpy(), U) <= 1e-6, prec
        if prec == "c128":
            assert np.abs(info.iters - it_o).max() <= 1, (info.iters, it_o)
    print(f"[coarse] {name}: iterations one-level {it_1.tolist()}, two-level {it_o.tolist()}", flush=True)


def test_two_level_columns_are_independent(case):
    name, w, fp, subs, M2, P = case
    P.set_coarse_space("const")
    P.factor(w.part, w.n_sub, 1, "c64")
    B = P.rhs_dipoles(w.dipoles) if w.dipoles is not None else P.rhs_ports(w.tx)
    Xall, _ = P.solve(B, tol=1e-9)
    for j in (0, B.shape[1] - 1):
        Xj, _ = P.solve(B[:, j:j + 1].contiguous(), tol=1e-9)
        assert torch.equal(Xj[:, 0], Xall[:, j]), j


def test_two_level_switches(case):
    from paper_1607_02573_amd import binding
    name, w, fp, subs, M2, P = case
    P.set_coarse_space("const")
    P.factor(w.part, w.n_sub, 1, "c128")
    V = torch.ones((P.n, 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.MwError) as e:
        P.apply_preconditioner_noalloc(V, torch.empty_like(V))
    assert e.value.code == binding.MW_EINVAL
    P.set_coarse_space("none")
    with pytest.raises(binding.MwError):      # factors invalid until refactored
        P.apply_preconditioner(V)
    P.factor(w.part, w.n_sub, 1, "c128")
    assert P.info().coarse_size == 0
    Zg = P.apply_preconditioner(V).cpu().numpy()
    assert _colerr(Zg, dd.oras_apply(subs, V.cpu().numpy())) <= 1e-11

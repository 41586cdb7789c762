"""GPU checks at the full sizes of the benchmark workloads, in the launch
configuration bench.py times, on outputs the FP64 oracle can check one by
one or through properties that hold at any size (a global sparse direct
solve of the 1 GHz chamber does not fit a CPU test):

* the assembled operator equals the oracle's, entry by entry (1e-13);
* every column converges, and sampled columns have a relative residual
  <= 1.2e-8 against the oracle's own matrix and sources (the solve's 1e-8
  is measured on the GPU's matrix, equal to the oracle's to roundoff);
* the S-matrix equals the oracle's port projections of the same fields,
  and is reciprocal (nu_i S_ij = nu_j S_ji) to the solver tolerance;
* mixed-precision fields agree with the FP64 path to the tolerance level;
* the adjoint gradient of the 0.5 GHz inversion step agrees with a central
  difference of J along a random direction on the 20 seeded tetrahedra.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import mw_inputs as mi
from oracle import fem, inverse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _csr(P):
    rp, col, val = P.matrix()
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(P.n, P.n))


# runs first: the 1 GHz fixture below holds most of the device memory until the
# end of the module
def test_inversion05_gradient_directional_difference():
    from paper_1607_02573_amd import solver
    print("[fullsize] 0.5 GHz inversion step: forward + adjoint on 32 ports", flush=True)
    w = mi.configs.inversion05()
    ctx = solver.Context(0)
    P = solver.problem_from_workload(ctx, w)
    dev = torch.device("cuda")
    eps_true = torch.from_numpy(w.extra["eps_true"]).to(dev)
    P.update_eps(eps_true)
    P.factor(w.part, w.n_sub, 1, "c128")
    U, _ = P.solve(P.rhs_ports(w.tx), tol=1e-11)
    S_meas = P.s_matrix(U, w.rx)
    eps0 = torch.from_numpy(w.eps).to(dev)
    P.update_eps(eps0)
    P.factor(w.part, w.n_sub, 1, "c128")
    J, S, g = P.misfit_gradient(w.tx, w.rx, S_meas, tol=1e-11)
    assert J > 0
    rng = np.random.default_rng(7)
    d = np.zeros(w.mesh.nt, dtype=np.complex128)
    d[w.extra["fd_tets"]] = rng.normal(size=20) + 1j * rng.normal(size=20)
    d *= 1e-4 * np.abs(w.eps).max() / np.abs(d).max()
    dd = torch.from_numpy(d).to(dev)

    def J_at(e):
        P.update_eps(e)
        P.factor(w.part, w.n_sub, 1, "c128")
        Ue, _ = P.solve(P.rhs_ports(w.tx), tol=1e-11)
        return 0.5 * float((P.s_matrix(Ue, w.rx) - S_meas).abs().pow(2).sum())

    fd = (J_at(eps0 + dd) - J_at(eps0 - dd)) / 2
    lin = float(torch.sum(torch.conj(g) * dd).real)
    print(f"[fullsize] directional derivative: adjoint {lin:.6e}, central difference {fd:.6e}", flush=True)
    assert abs(lin - fd) <= 1e-5 * abs(fd)
    P.close()
    ctx.close()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def chamber10():
    from paper_1607_02573_amd import solver
    print("[fullsize] building the 1 GHz chamber workload and the oracle operator", flush=True)
    w = mi.configs.chamber10()
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    total = torch.cuda.mem_get_info()[1]
    ctx = solver.Context(0, budget_bytes=int(total - (24 << 30)))
    P = solver.problem_from_workload(ctx, w)
    yield w, fp, P
    P.close()
    ctx.close()


def test_chamber10_operator_equals_oracle(chamber10):
    w, fp, P = chamber10
    A = _csr(P)
    Ao = fp.A.tocsr()
    Ao.sort_indices()
    assert A.shape == Ao.shape and A.nnz == Ao.nnz
    assert np.array_equal(A.indptr, Ao.indptr) and np.array_equal(A.indices, Ao.indices)
    assert np.abs(A.data - Ao.data).max() <= 1e-13 * np.abs(Ao.data).max()


def test_chamber10_mixed_160_rhs(chamber10):
    w, fp, P = chamber10
    print("[fullsize] mixed precision: factor 1600 subdomains, solve 160 port RHS", flush=True)
    P.factor(w.part, w.n_sub, 1, "c64")
    Bg = P.rhs_ports(w.tx)
    X, info = P.solve(Bg, tol=1e-8, restart=30)
    assert (info.relres <= 1e-8).all() and info.iters.max() < 100
    Bo = fem.rhs_ports(fp, w.ports, w.tx[[0, 37, 81, 159]])
    Xs = X[:, [0, 37, 81, 159]].cpu().numpy()
    res = np.linalg.norm(Bo - fp.A @ Xs, axis=0) / np.linalg.norm(Bo, axis=0)
    assert (res <= 1.2e-8).all(), res
    # S from the oracle's port vectors applied to the same fields, and reciprocity
    Po, nuo = fem.port_vectors(fp, w.ports)
    S = P.s_matrix(X, w.rx).cpu().numpy()
    So = inverse.s_matrix(Po, nuo, X.cpu().numpy(), w.rx)
    assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()
    Wm = nuo[:, None] * S
    assert np.abs(Wm - Wm.T).max() <= 1e-6 * np.abs(Wm).max()
    test_chamber10_mixed_160_rhs.fields = X[:, :32].cpu()


def test_chamber10_mixed_160_rhs_block(chamber10):
    """Block GMRES (five blocks of 32) on the same factors: every column
    converges, sampled residuals against the oracle's matrix, fewer
    iterations than pseudo-block, and the same fields to the tolerance level."""
    w, fp, P = chamber10
    print("[fullsize] mixed precision, block GMRES: solve 160 port RHS", flush=True)
    Bg = P.rhs_ports(w.tx)
    X, info = P.solve(Bg, tol=1e-8, restart=30, block=32)
    assert (info.relres <= 1e-8).all()
    Bo = fem.rhs_ports(fp, w.ports, w.tx[[3, 64, 127, 158]])
    Xs = X[:, [3, 64, 127, 158]].cpu().numpy()
    res = np.linalg.norm(Bo - fp.A @ Xs, axis=0) / np.linalg.norm(Bo, axis=0)
    assert (res <= 1.2e-8).all(), res
    Xp = getattr(test_chamber10_mixed_160_rhs, "fields", None)
    print(f"[fullsize] block iterations max {info.iters.max()} mean {info.iters.mean():.1f}", flush=True)
    if Xp is not None:
        err = (torch.linalg.norm(X[:, :32].cpu() - Xp, dim=0) / torch.linalg.norm(Xp, dim=0)).max().item()
        print(f"[fullsize] block vs pseudo-block fields: max relative L2 {err:.2e}", flush=True)
        assert err <= 1e-6


def test_chamber10_fp64_chunk_and_mixed_error(chamber10):
    w, fp, P = chamber10
    print("[fullsize] FP64: factor, solve 32 RHS", flush=True)
    P.factor(w.part, w.n_sub, 1, "c128")
    X, info = P.solve(P.rhs_ports(w.tx[:32]), tol=1e-8, restart=30)
    assert (info.relres <= 1e-8).all()
    Bo = fem.rhs_ports(fp, w.ports, w.tx[[0, 31]])
    Xs = X[:, [0, 31]].cpu().numpy()
    res = np.linalg.norm(Bo - fp.A @ Xs, axis=0) / np.linalg.norm(Bo, axis=0)
    assert (res <= 1.2e-8).all(), res
    Xm = getattr(test_chamber10_mixed_160_rhs, "fields", None)
    if Xm is not None:
        err = (torch.linalg.norm(Xm - X.cpu(), dim=0) / torch.linalg.norm(X.cpu(), dim=0)).max().item()
        print(f"[fullsize] mixed vs FP64 fields: max relative L2 {err:.2e}", flush=True)
        assert err <= 1e-6

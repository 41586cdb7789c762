"""The outer inversion loop (Section 5: L-BFGS over a vertex permittivity on
the normalised, regularised misfit (defJ2)) driven by the GPU solver,
against the same loop in the FP64 oracle (sparse LU for every solve), on the
same data: misfit values and iterates after three L-BFGS steps."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mw_inputs as mi
from oracle import fem, inverse, inversion as oinv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    w = mi.configs.small_chamber(0.15e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P, nu = fem.port_vectors(fp, w.ports)
    ports = np.nonzero(np.abs(P).sum(axis=0) > 0)[0].astype(np.int32)
    nv = fp.xyz.shape[0]
    rng = np.random.default_rng(5)
    e_gel = np.full(nv, 44 - 20j)
    e_true = e_gel * (1 + 0.05 * rng.normal(size=nv))
    B = fem.rhs_ports(fp, w.ports, ports)

    def S_of(ev):
        f = fem.with_eps(fp, oinv.vertex_mean(fp.tet, ev))
        return inverse.s_matrix(P, nu, spla.splu(f.A.tocsc()).solve(B), ports)

    S_mes, S_empty = S_of(e_true), S_of(e_gel)
    obj = oinv.Objective(fp, w.ports, ports, ports, S_mes, S_empty, 1e-4)
    es, Js, nev = oinv.lbfgs(obj, e_gel, iters=3, step0=0.5)
    return w, ports, S_mes, S_empty, e_gel, es, Js, nev


@pytest.mark.parametrize("recycle", ["none", "warm", "project"])
@pytest.mark.parametrize("prec,tol,rtol", [("c128", 1e-11, 1e-7), ("c64", 1e-10, 1e-6)])
def test_lbfgs_on_gpu_matches_oracle(setup, prec, tol, rtol, recycle):
    from paper_1607_02573_amd import inversion, solver
    w, ports, S_mes, S_empty, e_gel, es, Js, nev = setup
    ctx = solver.Context(0)
    Pg = solver.problem_from_workload(ctx, w)
    inv = inversion.Inversion(Pg, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, ports, ports, S_mes, S_empty, 1e-4,
                              precision=prec, tol=tol, recycle=recycle)
    h = inv.run(e_gel, iters=3, step0=0.5)
    if recycle != "none":
        # later evaluations start from the previous fields: fewer iterations
        assert sum(f + a for f, a in h.iters[1:]) < sum(f + a for f, a in h.iters[:1]) * (len(h.iters) - 1)
    assert h.evaluations == nev
    assert len(h.J) == len(Js) == 4
    np.testing.assert_allclose(h.J, Js, rtol=rtol)
    for eg, eo in zip(h.eps, es):
        assert np.linalg.norm(eg - eo) <= rtol * np.linalg.norm(eo)
    assert h.J[-1] < 0.5 * h.J[0]
    inv.close()
    Pg.close()
    ctx.close()


def test_projected_start_needs_no_more_iterations(setup):
    """The projected start X0 = U Y (Y the least-squares combination of all
    previous fields) has a starting residual no larger than the warm start's
    (Y = I is one of the choices), column by column: over the same accepted
    iterates, its GMRES iteration total is at most the warm start's (2 %
    slack: a smaller starting residual need not save an iteration in every
    column, since GMRES stops at a tolerance relative to ||b||)."""
    from paper_1607_02573_amd import inversion, solver
    w, ports, S_mes, S_empty, e_gel, es, Js, nev = setup
    ctx = solver.Context(0)
    Pg = solver.problem_from_workload(ctx, w)
    tot = {}
    for mode in ("warm", "project"):
        inv = inversion.Inversion(Pg, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, ports, ports, S_mes, S_empty, 1e-4,
                                  precision="c128", tol=1e-11, recycle=mode)
        h = inv.run(e_gel, iters=3, step0=0.5)
        np.testing.assert_allclose(h.J, Js, rtol=1e-7)
        tot[mode] = sum(f + a for f, a in h.iters[1:])
        inv.close()
    assert tot["project"] <= 1.02 * tot["warm"], tot
    Pg.close()
    ctx.close()


def test_block_mode_inversion_matches(setup):
    """The same loop with block GMRES for the forward and adjoint solves."""
    from paper_1607_02573_amd import inversion, solver
    w, ports, S_mes, S_empty, e_gel, es, Js, nev = setup
    ctx = solver.Context(0)
    Pg = solver.problem_from_workload(ctx, w)
    inv = inversion.Inversion(Pg, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, ports, ports, S_mes, S_empty, 1e-4,
                              precision="c128", tol=1e-11, block=32)
    h = inv.run(e_gel, iters=3, step0=0.5)
    np.testing.assert_allclose(h.J, Js, rtol=1e-7)
    inv.close()
    Pg.close()
    ctx.close()


@pytest.fixture(scope="module")
def setup_p1():
    w = mi.configs.small_chamber(0.15e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P, nu = fem.port_vectors(fp, w.ports)
    ports = np.nonzero(np.abs(P).sum(axis=0) > 0)[0].astype(np.int32)
    nv = fp.xyz.shape[0]
    rng = np.random.default_rng(6)
    e_gel = np.full(nv, 44 - 20j)
    e_true = e_gel * (1 + 0.05 * rng.normal(size=nv))
    B = fem.rhs_ports(fp, w.ports, ports)

    def S_of(ev):
        f = fem.with_eps_vertex(fp, ev)
        return inverse.s_matrix(P, nu, spla.splu(f.A.tocsc()).solve(B), ports)

    S_mes, S_empty = S_of(e_true), S_of(e_gel)
    obj = oinv.Objective(fp, w.ports, ports, ports, S_mes, S_empty, 1e-4, p1=True)
    es, Js, nev = oinv.lbfgs(obj, e_gel, iters=3, step0=0.5)
    return w, fp, ports, S_mes, S_empty, e_gel, e_true, es, Js, nev


def test_vertex_permittivity_operator_and_gradient_match_oracle(setup_p1):
    """The operator with a vertex permittivity (exact P1 mass term) equals the
    oracle's entry by entry, and the vertex gradient of a misfit equals the
    oracle's adjoint gradient of the same data."""
    from paper_1607_02573_amd import solver
    w, fp, ports, S_mes, S_empty, e_gel, e_true, es, Js, nev = setup_p1
    ctx = solver.Context(0)
    Pg = solver.problem_from_workload(ctx, w)
    Pg.update_eps_vertex(torch.from_numpy(e_true).cuda())
    rp, col, val = Pg.matrix()
    import scipy.sparse as sp
    A = sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(Pg.n, Pg.n))
    Ao = fem.with_eps_vertex(fp, e_true).A.tocsr()
    assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max()
    obj = oinv.Objective(fp, w.ports, ports, ports, S_mes, S_empty, 0.0, p1=True)
    J, g_o, _ = obj(e_gel)
    from paper_1607_02573_amd import inversion
    inv = inversion.Inversion(Pg, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, ports, ports, S_mes, S_empty, 0.0,
                              precision="c128", tol=1e-12, p1=True)
    Jg, g_g = inv.objective(e_gel)
    assert abs(Jg - J) <= 1e-9 * abs(J)
    assert np.abs(g_g - g_o).max() <= 1e-7 * np.abs(g_o).max()
    inv.close()
    Pg.close()
    ctx.close()


def test_lbfgs_with_vertex_permittivity_matches_oracle(setup_p1):
    from paper_1607_02573_amd import inversion, solver
    w, fp, ports, S_mes, S_empty, e_gel, e_true, es, Js, nev = setup_p1
    ctx = solver.Context(0)
    Pg = solver.problem_from_workload(ctx, w)
    inv = inversion.Inversion(Pg, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, ports, ports, S_mes, S_empty, 1e-4,
                              precision="c128", tol=1e-11, p1=True)
    h = inv.run(e_gel, iters=3, step0=0.5)
    assert h.evaluations == nev
    np.testing.assert_allclose(h.J, Js, rtol=1e-7)
    for eg, eo in zip(h.eps, es):
        assert np.linalg.norm(eg - eo) <= 1e-7 * np.linalg.norm(eo)
    inv.close()
    Pg.close()
    ctx.close()

"""GPU tests of the serving pieces: continuous batching (columns joining and
leaving at restart boundaries) against mw_solve, its error paths, and the
serving loop (admission, eviction of idle factors, gradients through the
batch) against direct calls of the same library on the same factors."""
import numpy as np
import pytest

import mw_inputs as mi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def small(request):
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    P = solver.problem_from_workload(ctx, w)
    yield ctx, w, P
    P.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_batch_columns_equal_single_solves(small, prec):
    """Columns that join a running batch at different restarts give exactly
    the iterates of a solve of that column alone (x0 = 0, same restart)."""
    from paper_1607_02573_amd import solver
    ctx, w, P = small
    P.factor(w.part, w.n_sub, 1, prec)
    tol, m = 1e-9, 8
    B = P.rhs_ports(np.arange(8))
    b = solver.Batch(P, 6, tol=tol, restart=m)
    b.join(10, B[:, 0:3].contiguous())
    na, nf = b.cycle()
    assert na == 3 and nf == 0
    b.join(11, B[:, 5:7].contiguous())
    assert b.info().free_cols == 1
    b.cycle()
    b.join(12, B[:, 7:8].contiguous())
    done = {}
    for _ in range(200):
        b.cycle()
        while True:
            tag, nc = b.poll()
            if tag < 0:
                break
            done[tag] = b.take(tag, nc)
        if len(done) == 3:
            break
    assert set(done) == {10, 11, 12}
    assert b.info().active_cols == 0 and b.info().free_cols == 6 and b.info().work_bytes == 0
    cols = {10: [0, 1, 2], 11: [5, 6], 12: [7]}
    for tag, js in cols.items():
        X, it, rr = done[tag]
        for k, j in enumerate(js):
            Xj, inf = P.solve(B[:, j:j + 1].contiguous(), tol=tol, restart=m)
            assert torch.equal(X[:, k], Xj[:, 0]), (prec, tag, j)
            assert it[k] == inf.iters[0] and rr[k] == inf.relres[0]
            assert rr[k] <= tol
    b.close()


def test_batch_errors(small):
    from paper_1607_02573_amd import binding, solver
    ctx, w, P = small
    P.factor(w.part, w.n_sub, 1, "c64")
    B = P.rhs_ports(np.arange(4))
    b = solver.Batch(P, 3, tol=1e-8)
    with pytest.raises(binding.MwError) as e:
        b.join(0, B)                       # 4 columns, 3 slots
    assert e.value.code == binding.MW_ENOMEM
    b.join(0, B[:, :2].contiguous())
    with pytest.raises(binding.MwError):
        b.join(0, B[:, 2:3].contiguous())  # tag in use
    with pytest.raises(binding.MwError):
        b.take(0, 2)                       # not finished
    with pytest.raises(binding.MwError) as e:
        P.close()                          # a batch still refers to the problem
    assert e.value.code == binding.MW_EINVAL
    # a zero right-hand side finishes at once with x = 0
    b.join(1, torch.zeros((P.n, 1), dtype=torch.complex128, device="cuda"))
    assert b.poll() == (1, 1)
    X, it, rr = b.take(1, 1)
    assert it[0] == 0 and float(X.abs().max()) == 0.0
    b.close()
    # released factors: cycles refuse, refactoring restores
    b = solver.Batch(P, 2)
    P.release_factors()
    b.join(0, B[:, :1].contiguous())
    with pytest.raises(binding.MwError):
        b.cycle()
    P.factor(w.part, w.n_sub, 1, "c64")
    for _ in range(100):
        b.cycle()
        if b.poll()[0] == 0:
            break
    X, it, rr = b.take(0, 1)
    assert rr[0] <= 1e-8
    b.close()


def test_serving_loop_matches_direct_calls():
    """A small menu served with an admission budget that cannot hold every
    factor at once: all requests finish, idle factors get evicted and
    rebuilt, and every result equals the direct library call."""
    from paper_1607_02573_amd import serve, solver
    ctx = solver.Context(0)
    menu = mi.serving.serving_menu(freqs=(0.2e9, 0.25e9), rings=(0.14,), n_per_ring=8, edges_per_sub=800)
    reqs = mi.serving.serving_requests(n_req=14, rate=20.0, seed=5, n_meshes=2, nports=8, max_solve=8, max_grad=4,
                                       p_grad=0.35)
    logs = []
    srv = serve.Server(ctx, menu, tol=1e-9, restart=10, max_cols=8, log=logs.append)
    # room for the base, the two largest factor sets and a little workspace
    f = sorted((q["factor"] + q["slots"] for q in srv.adm.p.values()), reverse=True)
    per = max(q["per_col"] for q in srv.adm.p.values())
    srv.adm.budget = srv.adm.base + f[0] + f[1] + 8 * per
    out = srv.run(reqs, progress_s=5.0)
    assert all(o.error is None for o in out), [o.error for o in out if o.error]
    assert all(o.t_done >= o.t_admit >= o.t_arrive for o in out)
    assert srv.evictions >= 1
    summ = serve.summarize(out, max(o.t_done for o in out))
    assert summ["p99_s"] >= summ["p50_s"] > 0
    for r, o in zip(sorted(reqs, key=lambda r: r.t_arrive), out):
        P = srv.slots[(r.mesh, r.version)].problem
        if srv.slots[(r.mesh, r.version)].batch is not None:
            srv.slots[(r.mesh, r.version)].batch.close()
            srv.slots[(r.mesh, r.version)].batch = None
        P.factor(srv.slots[(r.mesh, r.version)].part, srv.slots[(r.mesh, r.version)].n_sub, 1, "c64")
        if r.kind == "solve":
            X, inf = P.solve(P.rhs_ports(r.tx), tol=1e-9, restart=10)
            S = P.s_matrix(X, r.rx).cpu()
            Sg = torch.cat([o.S[k] for k in sorted(o.S)], dim=1)
            assert torch.allclose(Sg, S, rtol=0, atol=1e-12 * float(S.abs().max())), r.rid
        else:
            Sm = torch.from_numpy(r.s_meas).cuda()
            J, S, g = P.misfit_gradient(r.tx, r.rx, Sm, tol=1e-9, restart=10)
            assert abs(o.J - J) <= 1e-12 * abs(J), r.rid
            assert float((o.grad - g).abs().max()) <= 1e-10 * float(g.abs().max()), r.rid
    srv.close()
    ctx.close()

"""CPU checks of the GPU inversion driver's host side: its vertex averaging and
P1 stiffness equal the oracle's, and its L-BFGS takes the oracle's steps on a
quadratic (no device needed)."""
import numpy as np

import mw_inputs as mi
from oracle import fem, inversion as oinv


def test_vertex_maps_and_stiffness_equal_oracle():
    from paper_1607_02573_amd import inversion
    w = mi.configs.small_chamber(0.15e9, n_per_ring=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    nv = w.mesh.xyz.shape[0]
    rng = np.random.default_rng(1)
    ev = rng.normal(size=nv) + 1j * rng.normal(size=nv)
    A = inversion.vertex_average_matrix(w.mesh.tet, nv)
    np.testing.assert_allclose(A @ ev, oinv.vertex_mean(w.mesh.tet, ev), rtol=1e-14)
    K = inversion.p1_stiffness(w.mesh.xyz, w.mesh.tet)
    Ko = oinv.stiffness_p1(fp.xyz, fp.tet)
    assert abs(K - Ko).max() <= 1e-12 * abs(Ko).max()


def test_lbfgs_steps_equal_oracle_on_a_quadratic():
    from paper_1607_02573_amd import inversion
    n = 9
    rng = np.random.default_rng(2)
    M = rng.normal(size=(2 * n, 2 * n))
    Q = M @ M.T + 0.5 * np.eye(2 * n)
    b = rng.normal(size=2 * n)

    def fun(e):
        x = np.concatenate([e.real, e.imag])
        g = Q @ x - b
        return 0.5 * x @ Q @ x - b @ x, g[:n] + 1j * g[n:]

    class Quad(inversion.Inversion):
        def __init__(self):
            self.nv = n
            self.history = inversion.History()

        def objective(self, e):
            self.history.evaluations += 1
            return fun(e)

    h = Quad().run(np.zeros(n, dtype=complex), iters=25, mem=4, step0=0.3)
    es, Js, nev = oinv.lbfgs(lambda e: (*fun(e), None), np.zeros(n, dtype=complex), iters=25, mem=4, step0=0.3)
    assert h.evaluations == nev
    np.testing.assert_allclose(h.J, Js, rtol=1e-10, atol=1e-12 * abs(Js[0]))
    assert np.abs(h.eps[-1] - es[-1]).max() <= 1e-9 * np.abs(es[-1]).max()

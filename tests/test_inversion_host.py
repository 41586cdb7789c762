"""CPU checks of the library's host side of the inversion loop: its L-BFGS
(mw_lbfgs, driven through a Python objective) takes the oracle's steps on a
quadratic and minimises it; bad options are refused (no device needed)."""
import numpy as np
import pytest

from oracle import inversion as oinv


def _quadratic(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(2 * n, 2 * n))
    Q = M @ M.T + 0.5 * np.eye(2 * n)
    b = rng.normal(size=2 * n)
    return Q, b


def test_lbfgs_steps_equal_oracle_on_a_quadratic():
    from paper_1607_02573_amd import binding
    n = 9
    Q, b = _quadratic(n, 2)

    def real_fun(x):
        return 0.5 * x @ Q @ x - b @ x, Q @ x - b

    def cplx_fun(e):
        x = np.concatenate([e.real, e.imag])
        J, g = real_fun(x)
        return J, g[:n] + 1j * g[n:], None

    x, Jh, Xh, nev = binding.lbfgs(real_fun, np.zeros(2 * n), iters=25, mem=4, step0=0.3)
    es, Js, nev_o = oinv.lbfgs(cplx_fun, np.zeros(n, dtype=complex), iters=25, mem=4, step0=0.3)
    assert nev == nev_o
    np.testing.assert_allclose(Jh, Js, rtol=1e-10, atol=1e-12 * abs(Js[0]))
    xo = np.concatenate([es[-1].real, es[-1].imag])
    assert np.abs(x - xo).max() <= 1e-9 * np.abs(xo).max()
    for k in range(len(es)):
        np.testing.assert_allclose(Xh[k], np.concatenate([es[k].real, es[k].imag]), rtol=1e-9, atol=1e-12)
    # J decreases at every accepted step, towards the minimiser of the quadratic
    assert (np.diff(Jh) < 0).all()
    xs = np.linalg.solve(Q, b)
    assert np.linalg.norm(x - xs) <= 1e-2 * np.linalg.norm(xs)


def test_lbfgs_refuses_bad_options_and_reports_objective_errors():
    from paper_1607_02573_amd import binding
    with pytest.raises(binding.MwError):
        binding.lbfgs(lambda x: (float(x @ x), 2 * x), np.ones(3), iters=2, mem=0)
    with pytest.raises(ZeroDivisionError):
        binding.lbfgs(lambda x: (1 / 0, x), np.ones(3), iters=2)

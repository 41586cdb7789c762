#!/usr/bin/env python3
"""Writes the stored oracle results that the full-size GPU tests compare with.

Calls only oracle/ (and the seeded input generators of mw_inputs/); nothing
here reads a GPU result.  A global sparse direct solve of the 0.5 GHz and
1 GHz chambers does not fit a test, so the reference fields come from the
oracle's own ORAS-GMRES (oracle/dd.py via oracle/pool.py, oracle/gmres.py)
on the same partition, at a tighter tolerance than the GPU tests use:

  chamber05_oracle.npz    0.5 GHz chamber, 64 subdomains: ports 0, 8, 16, 24
                          at relative residual 1e-10;
  chamber10_oracle.npz    1 GHz chamber, 1600 subdomains: ports 5 (ring
                          z = 0.06 m) and 90 (ring z = 0.14 m) at 1e-10;
  inversion05_oracle.npz  0.5 GHz inversion step: 'measured' S at the
                          phantom with inclusion, S, J and the adjoint
                          gradient (Section 5) at the phantom, on the 20
                          seeded tetrahedra, every solve at 1e-11.

Each file holds the S entries, per-column norms of the fields over all
unknowns, the fields at a seeded sample of unknowns (the indices are stored
beside them), GMRES iteration counts and true relative residuals, and a
fingerprint of the inputs (n, nnz, sum of eps) that the tests check first.

    python tests/golden/make_oracle_fixtures.py [chamber05] [chamber10] [inversion05]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mw_inputs as mi  # noqa: E402
from oracle import fem, gmres, inverse, pool  # noqa: E402

NSAMPLE = 4000


def _fingerprint(w, fp):
    return np.array([fp.n, fp.A.nnz, w.eps.sum().real, w.eps.sum().imag, w.n_sub])


def _solve(fp, w, M, B, tol):
    t0 = time.perf_counter()
    X, it, rr = gmres.gmres(fp.A, B, M.apply, tol=tol, restart=w.restart, maxit=1000)
    print(f"  gmres: {B.shape[1]} columns, iterations {it.tolist()}, relres max {rr.max():.2e}, "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    assert (rr <= tol).all()
    return X, it, rr


def forward_fixture(name, w, tx, tol, nproc):
    t0 = time.perf_counter()
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    P, nu = fem.port_vectors(fp, w.ports)
    B = fem.rhs_ports(fp, w.ports, tx)
    print(f"{name}: n={fp.n}, assembly {time.perf_counter() - t0:.1f} s", flush=True)
    with pool.PooledORAS(fp, w.part, w.overlap, nproc=nproc, max_cols=len(tx)) as M:
        print(f"  {w.n_sub} subdomains factored on {M.nproc} processes in {M.t_setup:.1f} s", flush=True)
        X, it, rr = _solve(fp, w, M, B, tol)
    idx = np.sort(np.random.default_rng(21).choice(fp.n, size=NSAMPLE, replace=False))
    S = inverse.s_matrix(P, nu, X, w.rx)
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), tx=np.asarray(tx), rx=w.rx, tol=tol,
                        S=S, norms=np.linalg.norm(X, axis=0), idx=idx, U_sample=X[idx], iters=it, relres=rr,
                        fingerprint=_fingerprint(w, fp))


def inversion_fixture(nproc):
    name = "inversion05"
    w = mi.configs.inversion05()
    tol = 1e-11
    fd = w.extra["fd_tets"]
    t0 = time.perf_counter()
    fpt = fem.build(w.mesh, w.extra["eps_true"], w.k0, w.beta_imp, w.ports)
    P, nu = fem.port_vectors(fpt, w.ports)
    B = fem.rhs_ports(fpt, w.ports, w.tx)
    print(f"{name}: n={fpt.n}, assembly {time.perf_counter() - t0:.1f} s", flush=True)
    with pool.PooledORAS(fpt, w.part, w.overlap, nproc=nproc, max_cols=len(w.tx)) as M:
        Ut, _, _ = _solve(fpt, w, M, B, tol)
    S_meas = inverse.s_matrix(P, nu, Ut, w.rx)
    del Ut, M
    fp = fem.with_eps(fpt, w.eps)
    with pool.PooledORAS(fp, w.part, w.overlap, nproc=nproc, max_cols=len(w.tx)) as M:
        U, it_f, rr_f = _solve(fp, w, M, B, tol)
        S = inverse.s_matrix(P, nu, U, w.rx)
        r = S - S_meas
        J = inverse.misfit(S, S_meas)
        # adjoint data (Section 5, problem (pbadj)): lambda_j = sum_i r_ij p_i / nu_i
        Lam = (P[:, w.rx] / nu[w.rx][None, :]) @ r
        F, it_a, rr_a = _solve(fp, w, M, Lam, tol)
    ut = inverse.local_values(fp, U)[fd]
    ft = inverse.local_values(fp, F)[fd]
    G = (fp.k0 ** 2) * np.einsum("tpj,tpq,tqj->t", ft, fp.M[fd], ut)
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), tx=w.tx, rx=w.rx, tol=tol, S_meas=S_meas,
                        S=S, J=J, fd_tets=fd, grad_fd=np.conj(G), iters_forward=it_f, iters_adjoint=it_a,
                        relres_forward=rr_f, relres_adjoint=rr_a, fingerprint=_fingerprint(w, fp))


def main():
    which = sys.argv[1:] or ["chamber05", "chamber10", "inversion05"]
    nproc = int(os.environ.get("ORACLE_PROCS", os.cpu_count() or 1))
    for name in which:
        t0 = time.perf_counter()
        if name == "chamber05":
            forward_fixture(name, mi.configs.chamber05(), np.array([0, 8, 16, 24]), 1e-10, nproc)
        elif name == "chamber10":
            forward_fixture(name, mi.configs.chamber10(), np.array([5, 90]), 1e-10, nproc)
        elif name == "inversion05":
            inversion_fixture(nproc)
        else:
            raise SystemExit(f"unknown fixture {name}")
        print(f"{name}: written in {time.perf_counter() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()

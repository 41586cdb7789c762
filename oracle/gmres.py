"""Oracle: right-preconditioned restarted GMRES(m), pseudo-block over many
right-hand sides, plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Section 6 of the paper: every linear system is solved by GMRES right-
preconditioned with ORAS and stopped when the unpreconditioned relative
residual ||b - A x|| / ||b|| falls below the tolerance (1e-8 there); several
right-hand sides are solved together by a pseudo-block method, in which each
right-hand side keeps its own Krylov space and only the arithmetic of the
different right-hand sides is fused.

Textbook right-preconditioned GMRES (Saad, Iterative Methods for Sparse
Linear Systems, 2nd ed., Algorithm 9.5) with the Hermitian inner product,
classical Gram-Schmidt applied twice (CGS2) and complex Givens rotations.
x0 = 0.  At the end of each cycle the true residual b - A x is recomputed and
decides convergence (and restarts the next cycle).
"""
from __future__ import annotations

import numpy as np


def givens(a: complex, b: float):
    """c (real), s (complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    rho = np.hypot(abs(a), b)
    if rho == 0.0:
        return 1.0, 0.0 + 0.0j, 0.0 + 0.0j
    if abs(a) == 0.0:
        return 0.0, 1.0 + 0.0j, complex(b)
    ph = a / abs(a)
    return abs(a) / rho, ph * b / rho, ph * rho


def gmres(A, B: np.ndarray, prec, tol: float = 1e-8, restart: int = 30, maxit: int = 1000):
    """Solve A X = B column by column (pseudo-block).

    prec(V) applies M^-1 to the columns of V.  Returns X and per-column
    (iterations, true relative residual).
    """
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), dtype=np.complex128)
    bnorm = np.linalg.norm(B, axis=0)
    iters = np.zeros(nrhs, dtype=np.int64)
    relres = np.ones(nrhs)
    todo = np.nonzero(bnorm > 0)[0]
    relres[bnorm == 0] = 0.0
    while todo.size:
        R = B[:, todo] - A @ X[:, todo]
        rn = np.linalg.norm(R, axis=0)
        relres[todo] = rn / bnorm[todo]
        still = relres[todo] > tol
        still &= iters[todo] < maxit
        todo = todo[still]
        if not todo.size:
            break
        R, rn = R[:, still], rn[still]
        q = todo.size
        m = restart
        V = np.zeros((m + 1, n, q), dtype=np.complex128)
        H = np.zeros((m + 1, m, q), dtype=np.complex128)
        cs = np.zeros((m, q))
        sn = np.zeros((m, q), dtype=np.complex128)
        g = np.zeros((m + 1, q), dtype=np.complex128)
        V[0] = R / rn
        g[0] = rn
        k = np.zeros(q, dtype=np.int64)      # Krylov dimension reached per column
        active = np.ones(q, dtype=bool)
        for j in range(m):
            act = np.nonzero(active)[0]
            if not act.size:
                break
            Z = prec(V[j][:, act])
            W = A @ Z
            Vj = V[: j + 1][:, :, act]                  # [j+1, n, a]
            h = np.einsum("knc,nc->kc", Vj.conj(), W)   # first Gram-Schmidt pass
            W = W - np.einsum("knc,kc->nc", Vj, h)
            h2 = np.einsum("knc,nc->kc", Vj.conj(), W)  # second pass
            W = W - np.einsum("knc,kc->nc", Vj, h2)
            h = h + h2
            hn = np.linalg.norm(W, axis=0)
            for c_, col in enumerate(act):
                hc = np.zeros(j + 2, dtype=np.complex128)
                hc[: j + 1] = h[:, c_]
                hc[j + 1] = hn[c_]
                for i in range(j):                     # previous rotations
                    t = cs[i, col] * hc[i] + sn[i, col] * hc[i + 1]
                    hc[i + 1] = -np.conj(sn[i, col]) * hc[i] + cs[i, col] * hc[i + 1]
                    hc[i] = t
                c, s, r = givens(hc[j], hn[c_])
                cs[j, col], sn[j, col] = c, s
                hc[j], hc[j + 1] = r, 0.0
                H[: j + 2, j, col] = hc
                g[j + 1, col] = -np.conj(s) * g[j, col]
                g[j, col] = c * g[j, col]
                k[col] = j + 1
                iters[todo[col]] += 1
                if hn[c_] > 0:
                    V[j + 1][:, col] = W[:, c_] / hn[c_]
                if (abs(g[j + 1, col]) / bnorm[todo[col]] <= tol or hn[c_] == 0.0
                        or iters[todo[col]] >= maxit):
                    active[col] = False
        # x += M^-1 (V y),  H y = g on the Krylov dimension of each column
        U = np.zeros((n, q), dtype=np.complex128)
        for col in range(q):
            kk = k[col]
            if kk == 0:
                continue
            y = np.linalg.solve(np.triu(H[:kk, :kk, col]), g[:kk, col])
            U[:, col] = np.einsum("knc,k->n", V[:kk][:, :, [col]], y)
        X[:, todo] += prec(U)
    return X, iters, relres

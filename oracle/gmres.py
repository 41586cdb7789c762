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


def block_gmres(A, B: np.ndarray, prec, tol: float = 1e-8, restart: int = 30, maxit: int = 1000,
                p: int = 32, delta: float = 1e-7):
    """Solve A X = B by restarted block GMRES(m) with blocks of p columns.

    The block Krylov method the paper's conclusion names as a way to share one
    Krylov space among many right-hand sides (Section 7), in the textbook form
    (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Section 6.12,
    block Arnoldi and block GMRES), right-preconditioned with prec = M^-1 and
    stopped on the unpreconditioned relative residual of every column
    (Section 6):

      * R0 = B_blk - A X_blk = V_0 S0 (thin QR);
      * step j: W = A M^-1 V_j, block classical Gram-Schmidt applied twice
        (H_ij = V_i^H W accumulated over both passes), W = V_{j+1} H_{j+1,j}
        (thin QR);
      * after step j, Y_j = argmin ||E_1 S0 - Hbar_j Y|| column by column
        (least squares over the (j+2)p x (j+1)p block Hessenberg matrix) and
        the residual estimate of column c is the norm of column c of
        E_1 S0 - Hbar_j Y_j;
      * the block stops when every column's estimate is <= tol ||b_c||, after
        m steps, or when a column would pass maxit; then
        X_blk += M^-1 [V_0 .. V_{j}] Y_j.

    Restarts recompute the true residual; columns below tol leave, and the
    remaining ones are regrouped, in column order, into blocks of p.
    Breakdown: the new block W is numerically rank deficient when some
    diagonal entry of H_{j+1,j} is <= delta times the largest column norm of
    A M^-1 V_j; step j still enters the least-squares problem (only
    H_{j+1,j}^H H_{j+1,j} matters there, so the deficient directions need no
    basis vector) and the block's cycle ends after it.  A block whose
    starting residual block is rank deficient in the same sense leaves block
    mode: those columns are finished by ordinary GMRES (gmres above) from the
    current iterate.  delta = 1e-7 sits above the square root of the FP64
    unit roundoff, the smallest relative pivot a Cholesky-based QR (the GPU
    solver's) still resolves, so both sides see the same breakdowns.

    Returns X and per-column (iterations, true relative residual).
    """
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), dtype=np.complex128)
    bnorm = np.linalg.norm(B, axis=0)
    iters = np.zeros(nrhs, dtype=np.int64)
    relres = np.ones(nrhs)
    relres[bnorm == 0] = 0.0
    single = np.zeros(nrhs, dtype=bool)     # columns handed to ordinary GMRES
    todo = np.nonzero(bnorm > 0)[0]
    while todo.size:
        R = B[:, todo] - A @ X[:, todo]
        relres[todo] = np.linalg.norm(R, axis=0) / bnorm[todo]
        keep = (relres[todo] > tol) & (iters[todo] < maxit) & ~single[todo]
        todo, R = todo[keep], R[:, keep]
        for b0 in range(0, todo.size, p):
            cols = todo[b0:b0 + p]
            steps = min(restart, maxit - int(iters[cols].max()))
            dX, done = _block_cycle(A, prec, R[:, b0:b0 + p], steps, tol * bnorm[cols], delta)
            if done == 0:
                single[cols] = True
                continue
            X[:, cols] += dX
            iters[cols] += done
    rest = np.nonzero(single)[0]
    if rest.size:
        # ordinary GMRES on the correction, to the same absolute tolerance
        R = B[:, rest] - A @ X[:, rest]
        for c, col in enumerate(rest):
            rn = np.linalg.norm(R[:, c])
            if rn <= tol * bnorm[col]:
                relres[col] = rn / bnorm[col]
                continue
            D, it, _ = gmres(A, R[:, [c]], prec, tol=tol * bnorm[col] / rn, restart=restart,
                             maxit=maxit - int(iters[col]))
            X[:, col] += D[:, 0]
            iters[col] += it[0]
            relres[col] = np.linalg.norm(B[:, col] - A @ X[:, col]) / bnorm[col]
    return X, iters, relres


def _block_cycle(A, prec, R0: np.ndarray, m: int, atol: np.ndarray, delta: float):
    """One cycle of block GMRES on the residual block R0 (n x q).  Returns the
    correction M^-1 V Y and the number of steps taken (0: rank-deficient
    start)."""
    n, q = R0.shape
    V0, S0 = np.linalg.qr(R0)
    if np.abs(np.diag(S0)).min() <= delta * np.linalg.norm(R0, axis=0).max():
        return None, 0
    V = [V0]
    H = np.zeros(((m + 1) * q, m * q), dtype=np.complex128)
    E = np.zeros(((m + 1) * q, q), dtype=np.complex128)
    E[:q] = S0
    Y, steps = None, 0
    for j in range(m):
        W = A @ prec(V[j])
        scale = np.linalg.norm(W, axis=0).max()
        Vs = np.concatenate(V, axis=1)
        h = Vs.conj().T @ W
        W = W - Vs @ h
        h2 = Vs.conj().T @ W
        W = W - Vs @ h2
        Vn, Rn = np.linalg.qr(W)
        H[: (j + 1) * q, j * q:(j + 1) * q] = h + h2
        H[(j + 1) * q:(j + 2) * q, j * q:(j + 1) * q] = Rn
        V.append(Vn)
        Hj = H[: (j + 2) * q, : (j + 1) * q]
        Ej = E[: (j + 2) * q]
        Y = np.linalg.lstsq(Hj, Ej, rcond=None)[0]
        steps = j + 1
        if (np.linalg.norm(Ej - Hj @ Y, axis=0) <= atol).all():
            break
        if np.abs(np.diag(Rn)).min() <= delta * scale:
            break
    return prec(np.concatenate(V[:steps], axis=1) @ Y), steps

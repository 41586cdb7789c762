"""Outer inversion loop on the GPU solver (Section 5 of the paper).

The unknown is the relative permittivity at the mesh vertices; the Maxwell
operator takes on each tetrahedron the mean of its four vertex values, or with
`p1` the linear coefficient integrated exactly in the mass term
(mw_update_eps_vertex, gradient by mw_gradient_vertex).  The
misfit is equation (defJ2): every pair (i, j) divided by |S_ij^empty|^2 (the
S-matrix of the chamber filled with the matching medium only), plus a
Tikhonov term alpha/2 int |grad eps_r|^2, exact for the piecewise-linear field
through the P1 stiffness matrix.  The optimiser is L-BFGS (limited-memory BFGS,
two-loop recursion, Nocedal & Wright Alg. 7.4/7.5) over [Re eps; Im eps] with
a backtracking Armijo line search (c1 = 1e-4, halving); its first step moves
the largest entry by `step0`.

Every evaluation of J and its gradient runs on the device through the C ABI:
the permittivity update and subdomain factorisation (mw_update_eps,
mw_factor_subdomains), the forward solves of all transmitting ports and the
S-matrix (mw_solve, mw_s_matrix), and one adjoint solve with the same factors
plus the per-tetrahedron gradient (mw_adjoint_rhs, mw_solve, mw_gradient).
With `recycle`, the forward and adjoint fields of the previous evaluation are
the initial guesses of the next one (the permittivity moves little between
evaluations, so GMRES starts from a small residual; the stopping test stays
relative to ||b||) -- the simplest form of the Krylov-information reuse
across inversion iterations that the paper's conclusion proposes.  The optimiser's
vector algebra, the vertex/tetrahedron maps and the Tikhonov product (one
sparse product over the vertices) run on the host, between evaluations.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import torch


def vertex_average_matrix(tet: np.ndarray, nv: int) -> sp.csr_matrix:
    """nt x nv matrix of the tetrahedron means of vertex values (entries 1/4)."""
    nt = tet.shape[0]
    rows = np.repeat(np.arange(nt), 4)
    return sp.csr_matrix((np.full(4 * nt, 0.25), (rows, tet.ravel())), shape=(nt, nv))


def p1_stiffness(xyz: np.ndarray, tet: np.ndarray) -> sp.csr_matrix:
    """Matrix of int grad(phi_a) . grad(phi_b) over the P1 hat functions:
    each tetrahedron contributes vol * G G^T with G the 4 x 3 gradients of its
    barycentric coordinates (rows of the inverse of the 4 x 4 matrix [1 x])."""
    nt = tet.shape[0]
    X = np.empty((nt, 4, 4))
    X[:, :, 0] = 1.0
    X[:, :, 1:] = xyz[tet]
    Ginv = np.linalg.inv(X)                     # column a: coefficients of lambda_a
    G = np.swapaxes(Ginv[:, 1:, :], 1, 2)       # [nt, 4, 3]
    vol = np.abs(np.linalg.det(X)) / 6.0
    Ke = vol[:, None, None] * (G @ np.swapaxes(G, 1, 2))
    r = np.broadcast_to(tet[:, :, None], (nt, 4, 4)).ravel()
    c = np.broadcast_to(tet[:, None, :], (nt, 4, 4)).ravel()
    nv = xyz.shape[0]
    return sp.coo_matrix((Ke.ravel(), (r, c)), shape=(nv, nv)).tocsr()


@dataclass
class History:
    eps: list = field(default_factory=list)      # accepted vertex fields (host, complex)
    J: list = field(default_factory=list)        # their misfits
    evaluations: int = 0
    seconds: float = 0.0
    solve_columns: int = 0                       # forward + adjoint right-hand sides solved
    iters: list = field(default_factory=list)    # (forward, adjoint) mean GMRES iterations per evaluation


class Inversion:
    def __init__(self, problem, xyz, tet, part, n_sub: int, tx, rx, S_mes: np.ndarray, S_empty: np.ndarray,
                 alpha: float, precision: str = "c64", tol: float = 1e-8, restart: int = 30, block: int = 0,
                 overlap: int = 1, recycle: bool = True, p1: bool = False):
        self.P = problem
        self.tet = np.ascontiguousarray(tet)
        self.nv = xyz.shape[0]
        self.part, self.n_sub, self.overlap = part, n_sub, overlap
        self.tx = np.ascontiguousarray(tx, dtype=np.int32)
        self.rx = np.ascontiguousarray(rx, dtype=np.int32)
        self.S_mes = np.asarray(S_mes, dtype=np.complex128)
        self.weight = 1.0 / np.abs(np.asarray(S_empty)) ** 2
        if not np.isfinite(self.weight).all():
            raise ValueError("S_empty has zero entries: the normalised misfit is undefined")
        self.alpha = float(alpha)
        self.precision, self.tol, self.restart, self.block = precision, tol, restart, block
        self.avg = vertex_average_matrix(self.tet, self.nv)
        self.K1 = p1_stiffness(np.asarray(xyz, dtype=np.float64), self.tet)
        self.dev = problem.ctx.device
        self.recycle = recycle
        self.p1 = p1
        self._U = self._F = None
        self.history = History()

    def objective(self, eps_v: np.ndarray):
        """J and dJ/dRe eps_v + i dJ/dIm eps_v at the vertex field eps_v."""
        P = self.P
        if self.p1:
            P.update_eps_vertex(torch.from_numpy(np.ascontiguousarray(eps_v, dtype=np.complex128)).to(self.dev))
        else:
            P.update_eps(torch.from_numpy(np.ascontiguousarray(self.avg @ eps_v)).to(self.dev))
        P.factor(self.part, self.n_sub, self.overlap, self.precision)
        U, info = P.solve(P.rhs_ports(self.tx), tol=self.tol, restart=self.restart, block=self.block,
                          x0=self._U if self.recycle else None)
        S = P.s_matrix(U, self.rx).cpu().numpy()
        r = S - self.S_mes
        J_data = 0.5 * float(np.sum(self.weight * np.abs(r) ** 2))
        gS = torch.from_numpy(np.ascontiguousarray(self.weight * r)).to(self.dev)
        F, info_a = P.solve(P.adjoint_rhs(gS, self.rx), tol=self.tol, restart=self.restart, block=self.block,
                            x0=self._F if self.recycle else None)
        g_d = (P.gradient_vertex(U, F).cpu().numpy() if self.p1
               else self.avg.T @ P.gradient(U, F).cpu().numpy())
        if self.recycle:
            self._U, self._F = U, F
        self.history.iters.append((float(info.iters.mean()), float(info_a.iters.mean())))
        kr, ki = self.K1 @ eps_v.real, self.K1 @ eps_v.imag
        J = J_data + 0.5 * self.alpha * float(eps_v.real @ kr + eps_v.imag @ ki)
        g = g_d + self.alpha * (kr + 1j * ki)
        self.history.evaluations += 1
        self.history.solve_columns += 2 * len(self.tx)
        return J, g

    def run(self, eps0: np.ndarray, iters: int, mem: int = 5, step0: float = 0.5, c1: float = 1e-4,
            max_backtrack: int = 20) -> History:
        """L-BFGS from the vertex field eps0 for `iters` accepted steps (fewer if
        a line search fails); returns the accepted iterates and misfits."""
        h = self.history
        t_start = time.perf_counter()
        nv = self.nv
        as_real = lambda z: np.concatenate([z.real, z.imag])  # noqa: E731
        as_cplx = lambda v: v[:nv] + 1j * v[nv:]              # noqa: E731
        x = as_real(np.asarray(eps0, dtype=np.complex128))
        J, g = self.objective(as_cplx(x))
        g = as_real(g)
        h.eps.append(as_cplx(x))
        h.J.append(J)
        pairs: deque = deque(maxlen=mem)      # (s, y, 1 / y.s), oldest first
        for _ in range(iters):
            d = -g
            coef = []
            for s, y, rho in reversed(pairs):
                a = rho * float(s @ d)
                d = d - a * y
                coef.append(a)
            if pairs:
                s, y, _ = pairs[-1]
                d = d * (float(s @ y) / float(y @ y))
                step = 1.0
            else:
                step = step0 / np.abs(d).max()
            for (s, y, rho), a in zip(pairs, reversed(coef)):
                d = d + (a - rho * float(y @ d)) * s
            slope = float(g @ d)
            accepted = False
            for _ in range(max_backtrack):
                x_new = x + step * d
                J_new, g_new = self.objective(as_cplx(x_new))
                if J_new <= J + c1 * step * slope:
                    accepted = True
                    break
                step *= 0.5
            if not accepted:
                break
            g_new = as_real(g_new)
            s, y = x_new - x, g_new - g
            sy = float(s @ y)
            if sy > 1e-12 * np.sqrt(float(s @ s) * float(y @ y)):
                pairs.append((s, y, 1.0 / sy))
            x, J, g = x_new, J_new, g_new
            h.eps.append(as_cplx(x))
            h.J.append(J)
        h.seconds += time.perf_counter() - t_start
        return h

"""Oracle: the outer inversion loop (Section 5), plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

  * Unknown: the relative permittivity at the mesh vertices (P1), as the
    paper's kappa = k0^2 eps_r is discretised with P1 elements in its
    reconstructions (Section 6).  The Maxwell operator takes either, on every
    tetrahedron, the mean of its four vertex values (one-point quadrature of
    the coefficient in the mass term), or with `p1` the linear coefficient
    integrated exactly: sum_v eps_v int_t l_v N_p . N_q (fem.element_mass_p1).
  * Misfit, equation (defJ2): each pair (i, j) normalised by the empty-chamber
    coefficient, plus a Tikhonov term on the gradient of the parameter,
        J = 1/2 sum_ij |S_ij - Smes_ij|^2 / |Sempty_ij|^2
            + alpha/2 int |grad eps_r|^2,
    the integral exact for P1 fields: alpha/2 (Re e^T K1 Re e + Im e^T K1 Im e)
    with K1 the P1 stiffness matrix (kappa = k0^2 eps_r: the factor k0^4 of
    the paper's form is absorbed in alpha).
  * Gradient (dJ/dRe + i dJ/dIm at each vertex): the adjoint gradient per
    tetrahedron of the data term (Section 5, the adjoint problem (pbadj) with
    data weighted by 1/|Sempty_ij|^2), mapped to the vertices by the transpose
    of the averaging, plus alpha K1 e; with `p1`, vertex v collects
    conj(k0^2 sum_j f_j|_t^T M1[t, v] u_j|_t) over its tetrahedra.
  * Optimiser: L-BFGS, the two-loop recursion (Nocedal and Wright, Numerical
    Optimization, 2nd ed., Algorithms 7.4 and 7.5) on x = [Re e; Im e] with
    memory `mem`, H0 = (s^T y / y^T y) I from the latest pair, and a
    backtracking line search on the Armijo condition (c1 = 1e-4, step halved);
    the first step is scaled so that it moves the largest entry by `step0`.
    The paper names L-BFGS without its parameters; these are the reading.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, inverse


def vertex_mean(tet: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Per-tetrahedron mean of the vertex values."""
    return ev[tet].mean(axis=1)


def vertex_mean_adjoint(tet: np.ndarray, nv: int, gt: np.ndarray) -> np.ndarray:
    """Transpose of vertex_mean: g_v = sum over the tetrahedra t at v of g_t / 4."""
    out = np.zeros(nv, dtype=np.result_type(gt, np.complex128))
    np.add.at(out, tet.ravel(), np.repeat(gt / 4.0, 4))
    return out


def stiffness_p1(xyz: np.ndarray, tet: np.ndarray) -> sp.csr_matrix:
    """K1[a, b] = int grad(phi_a) . grad(phi_b) over P1 hat functions."""
    _, g, vol = fem.tet_geometry(xyz, tet)            # barycentric gradients [nt, 4, 3], volumes
    Kt = vol[:, None, None] * np.einsum("tad,tbd->tab", g, g)
    rows = np.repeat(tet, 4, axis=1).ravel()
    cols = np.tile(tet, (1, 4)).ravel()
    nv = xyz.shape[0]
    return sp.csr_matrix((Kt.ravel(), (rows, cols)), shape=(nv, nv))


class Objective:
    """J (equation defJ2) and its vertex gradient, every solve by sparse LU."""

    def __init__(self, fp: fem.FEProblem, ports, tx, rx, Smes, Sempty, alpha: float, p1: bool = False):
        self.fp, self.ports = fp, ports
        self.M1 = fem.element_mass_p1(fp.xyz, fp.tet) if p1 else None
        self.tx, self.rx = np.asarray(tx), np.asarray(rx)
        self.Smes = Smes
        self.w = 1.0 / np.abs(Sempty) ** 2
        self.alpha = alpha
        self.K1 = stiffness_p1(fp.xyz, fp.tet)
        self.P, self.nu = fem.port_vectors(fp, ports)
        self.B = fem.rhs_ports(fp, ports, self.tx)
        self.evals = 0

    def __call__(self, ev: np.ndarray):
        nv = self.fp.xyz.shape[0]
        if self.M1 is not None:
            fp = fem.with_eps_vertex(self.fp, ev, self.M1)
        else:
            fp = fem.with_eps(self.fp, vertex_mean(self.fp.tet, ev))
        lu = spla.splu(fp.A.tocsc())
        U = lu.solve(self.B)
        S = inverse.s_matrix(self.P, self.nu, U, self.rx)
        r = S - self.Smes
        Jd = 0.5 * float(np.sum(self.w * np.abs(r) ** 2))
        # adjoint with the weighted residual: d(Jd) = Re sum conj(w r) dS
        if self.M1 is not None:
            Lam = (self.P[:, self.rx] / self.nu[self.rx][None, :]) @ (self.w * r)
            F = lu.solve(Lam)
            ut, ft = inverse.local_values(fp, U), inverse.local_values(fp, F)
            G = (fp.k0 ** 2) * np.einsum("tpj,tvpq,tqj->tv", ft, self.M1, ut)
            gd = np.zeros(nv, dtype=np.complex128)
            np.add.at(gd, self.fp.tet.ravel(), G.ravel())
            gd = np.conj(gd)
        else:
            _, _, gt = inverse.adjoint_gradient(fp, lu, self.P, self.nu, U, self.tx, self.rx,
                                                S - self.w * r)
            gd = vertex_mean_adjoint(self.fp.tet, nv, gt)
        Kr, Ki = self.K1 @ ev.real, self.K1 @ ev.imag
        Jr = 0.5 * self.alpha * float(ev.real @ Kr + ev.imag @ Ki)
        g = gd + self.alpha * (Kr + 1j * Ki)
        self.evals += 1
        return Jd + Jr, g, S


def lbfgs(fun, e0: np.ndarray, iters: int, mem: int = 5, step0: float = 0.5, c1: float = 1e-4,
          max_backtrack: int = 20):
    """L-BFGS on the complex vertex vector e (real variables [Re e; Im e]).
    fun(e) -> (J, grad, extra) with grad = dJ/dRe + i dJ/dIm.  Returns the
    iterates, their J values and the number of evaluations of fun."""
    def split(z):
        return np.concatenate([z.real, z.imag])

    def join(x):
        h = x.size // 2
        return x[:h] + 1j * x[h:]

    x = split(e0)
    J, g, _ = fun(join(x))
    g = split(g)
    S, Y = [], []
    xs, Js = [join(x)], [J]
    nev = 1
    for k in range(iters):
        # two-loop recursion: d = -H g
        q = g.copy()
        a = []
        for s, y in reversed(list(zip(S, Y))):
            rho = 1.0 / (y @ s)
            ai = rho * (s @ q)
            q -= ai * y
            a.append((rho, ai, s, y))
        if S:
            q *= (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
            t = 1.0
        else:
            t = step0 / np.abs(q).max()
        for rho, ai, s, y in reversed(a):
            b = rho * (y @ q)
            q += (ai - b) * s
        d = -q
        slope = g @ d
        for _ in range(max_backtrack):
            xn = x + t * d
            Jn, gn, _ = fun(join(xn))
            nev += 1
            if Jn <= J + c1 * t * slope:
                break
            t *= 0.5
        else:
            break
        gn = split(gn)
        s, y = xn - x, gn - g
        if y @ s > 1e-12 * np.sqrt((y @ y) * (s @ s)):
            S.append(s)
            Y.append(y)
            if len(S) > mem:
                S.pop(0)
                Y.pop(0)
        x, J, g = xn, Jn, gn
        xs.append(join(x))
        Js.append(J)
    return xs, Js, nev

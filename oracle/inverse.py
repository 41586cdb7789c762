"""Oracle: scattering parameters, misfit and its adjoint gradient, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Section 4 of the paper:
  * equation (sij): S_ij = int_{Gamma_i} conj(E_j) . E0_i / int_{Gamma_i} |E0_i|^2,
    discretely S_ij = conj(p_i^T u_j) / nu_i (E0 is real here);
  * equation (defJ): J = 1/2 sum_ij |S_ij - Smes_ij|^2;
  * Section 5, problems (pblin) and (pbadj): the adjoint field F_j solves the
    same (complex-symmetric) operator with port data
    (S_ij - Smes_ij) / nu_i * conj(E0_i), and
    DJ(kappa, dkappa) = Re int conj(dkappa) sum_j conj(E_j . F_j).
Discretely, with eps_r piecewise constant per tetrahedron and
A(eps) = sum_t K_t - k0^2 eps_t M_t + (boundary terms independent of eps):
    lambda_j = sum_i r_ij p_i / nu_i,   f_j = A^-1 lambda_j,
    dJ = Re[ sum_t G_t d eps_t ],       G_t = k0^2 sum_j f_j|_t^T M_t u_j|_t,
and the gradient in PyTorch's convention (dJ/dRe + i dJ/dIm) is conj(G_t).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def s_matrix(P: np.ndarray, nu: np.ndarray, U: np.ndarray, rx) -> np.ndarray:
    rx = np.asarray(rx)
    return np.conj(P[:, rx].T @ U) / nu[rx, None]


def misfit(S: np.ndarray, Smes: np.ndarray) -> float:
    return 0.5 * float(np.sum(np.abs(S - Smes) ** 2))


def local_values(fp: fem.FEProblem, U: np.ndarray) -> np.ndarray:
    """u restricted to the 6 edges of every tetrahedron (0 on PEC edges)."""
    d = fp.dof[fp.t2e]                       # [nt, 6]
    out = np.zeros(d.shape + (U.shape[1],), dtype=np.complex128)
    ok = d >= 0
    out[ok] = U[d[ok]]
    return out


def adjoint_gradient(fp: fem.FEProblem, lu, P, nu, U, tx, rx, Smes):
    """J, S and grad_eps (complex, per tetrahedron) from the forward fields U."""
    S = s_matrix(P, nu, U, rx)
    r = S - Smes
    rx = np.asarray(rx)
    Lam = (P[:, rx] / nu[rx][None, :]) @ r            # [n, ntx]
    F = lu.solve(Lam)
    ut = local_values(fp, U)
    ft = local_values(fp, F)
    G = (fp.k0 ** 2) * np.einsum("tpj,tpq,tqj->t", ft, fp.M, ut)
    return misfit(S, Smes), S, np.conj(G)


def forward(fp: fem.FEProblem, ports, tx):
    lu = spla.splu(fp.A.tocsc())
    B = fem.rhs_ports(fp, ports, tx)
    return lu, lu.solve(B)


def woodbury_fd(fp: fem.FEProblem, lu, U, B, P, nu, rx, Smes, t: int, h: complex):
    """Central difference of J along eps_t -> eps_t +/- h, each perturbed
    solve done exactly by the Sherman-Morrison-Woodbury identity on the
    rank <= 6 update  A(eps + h e_t) = A - k0^2 h Q M_t Q^T  (Q: the free edges
    of tetrahedron t)."""
    d = fp.dof[fp.t2e[t]]
    keep = d >= 0
    idx = d[keep]
    Mt = fp.M[t][np.ix_(keep, keep)]
    Q = np.zeros((fp.n, idx.size), dtype=np.complex128)
    Q[idx, np.arange(idx.size)] = 1.0
    AiQ = lu.solve(Q)                                  # A^-1 Q
    QtAiQ = AiQ[idx, :]
    Up = []
    for sgn in (+1.0, -1.0):
        C = -(fp.k0 ** 2) * (sgn * h) * Mt
        # (A + Q C Q^T)^-1 u-form:  u' = u - A^-1 Q (I + C Q^T A^-1 Q)^-1 C Q^T u
        Up.append(np.linalg.solve(np.eye(idx.size) + C @ QtAiQ, C @ U[idx, :]))
    # J+ - J- = 1/2 sum Re[(S+ - S-) conj(S+ + S- - 2 Smes)], with S+ - S- formed
    # from U+ - U- = -A^-1 Q (c+ - c-) so that no large terms cancel
    Sp = s_matrix(P, nu, U - AiQ @ Up[0], rx)
    Sm = s_matrix(P, nu, U - AiQ @ Up[1], rx)
    dS = s_matrix(P, nu, -(AiQ @ (Up[0] - Up[1])), rx)
    dJ = 0.5 * float(np.sum((dS * np.conj(Sp + Sm - 2.0 * Smes)).real))
    return dJ / (2.0 * abs(h))

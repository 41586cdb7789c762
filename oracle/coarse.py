"""Oracle: two-level ORAS, the one-level preconditioner of oracle/dd.py plus a
coarse correction, plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

The paper's conclusion (Section 7) names a two-level method, a coarse space
added to ORAS so that the iteration count stops growing with the number of
subdomains (Section 6.1, Table tabscaling: 43 -> 81 iterations from 256 to
2048 subdomains); it gives no construction.  The reading taken here:

  * coarse space: every subdomain i contributes k real fields Phi_i (n_i x k)
    on its own unknowns, weighted by its partition of unity:
        Z_i = R_i^T D_i Phi_i,     Z = [Z_1 ... Z_N]  (n x kN);
    the fields are edge interpolants (circulations int_e f . t) of global
    vector fields f: 'const' takes the three constant fields x, y, z
    (Phi[e, a] = t_e[a], t_e = x_hi - x_lo: a field of the lowest-order space
    reproduced exactly by it), 'wave' adds the real and imaginary parts of
    plane waves p exp(-i k d.x) of the background medium (k = k0 sqrt(Re
    eps_gel)), directions x, y, z, two polarisations each, evaluated at the
    edge midpoint times p . t_e;
  * coarse operator E = Z^T A Z (kN x kN, complex symmetric, Z real);
  * correction in the deflated ("balanced") form
        M2^-1 v = M^-1 (v - A Q v) + Q v,   Q = Z E^-1 Z^T,
    so that M2^-1 A is the identity on span(Z) and the residual handed to
    M^-1 is Z-orthogonal: Z^T (v - A Q v) = 0.
E^-1 is applied by a dense LU (numpy), which is exact to rounding for the
coarse sizes used here.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import dd


def edge_geometry(fp):
    """Edge vectors t_e = x_hi - x_lo and midpoints of the free unknowns."""
    e = fp.edges[fp.free]
    xa, xb = fp.xyz[e[:, 0]], fp.xyz[e[:, 1]]
    return xb - xa, 0.5 * (xa + xb)


def wave_fields(k: float):
    """(k d, polarisation p) pairs: d = x, y, z, each with the two unit
    polarisations perpendicular to it (the real and imaginary parts of a wave
    along -d are those along d, up to sign, so they would repeat)."""
    out = []
    for ax in range(3):
        d = np.zeros(3)
        d[ax] = 1.0
        for q in (1, 2):
            p = np.zeros(3)
            p[(ax + q) % 3] = 1.0
            out.append((k * d, p))
    return out


def local_fields(fp, sub: dd.Subdomain, kind: str = "const", k: float = 0.0) -> np.ndarray:
    """Phi_i (n_i x k) for one subdomain: circulations of the chosen global
    fields along its edges (not yet weighted by D_i)."""
    t, mid = edge_geometry(fp)
    ti, mi = t[sub.gdof], mid[sub.gdof]
    cols = [ti[:, a] for a in range(3)]
    if kind == "wave":
        for kd, p in wave_fields(k):
            ph = np.exp(-1j * (mi @ kd)) * (ti @ p)
            cols += [ph.real, ph.imag]
    elif kind != "const":
        raise ValueError(kind)
    return np.stack(cols, axis=1)


class TwoLevel:
    """M2^-1 of the deflated two-level ORAS for the subdomains `subs`.  Z is
    kept sparse (each column lives on one subdomain); E is formed densely."""

    def __init__(self, fp, subs, kind: str = "const", k: float = 0.0, Z=None):
        self.fp, self.subs = fp, subs
        n = fp.n
        if Z is None:
            rows, cols, vals, off = [], [], [], 0
            for s in subs:
                Phi = s.D[:, None] * local_fields(fp, s, kind, k)
                nk = Phi.shape[1]
                rows.append(np.repeat(s.gdof, nk))
                cols.append(np.tile(off + np.arange(nk), s.gdof.size))
                vals.append(Phi.ravel())
                off += nk
            Z = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, off))
        self.Z = sp.csc_matrix(Z)
        self.E = np.asarray((self.Z.T @ (fp.A @ self.Z)).todense())
        self.lu = sla.lu_factor(self.E)

    @property
    def size(self) -> int:
        return self.Z.shape[1]

    def coarse(self, V: np.ndarray) -> np.ndarray:
        """Q V = Z E^-1 Z^T V."""
        return self.Z @ sla.lu_solve(self.lu, self.Z.T @ V)

    def apply(self, V: np.ndarray) -> np.ndarray:
        Qv = self.coarse(V)
        return dd.oras_apply(self.subs, V - self.fp.A @ Qv) + Qv

    def __call__(self, V: np.ndarray) -> np.ndarray:
        return self.apply(V)

"""The outer inversion loop (Section 5 of the paper) behind the C ABI.

mw_inversion_* runs every part of an evaluation in the library (permittivity
update and factors, forward and adjoint solves, the normalised misfit of
equation (defJ2), the vertex gradient and the Tikhonov term) and the L-BFGS
iteration itself (mw_lbfgs, host code of the library); this module only
marshals arguments: host arrays to device tensors, options to the C
structures, and the library's history back to Python.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .binding import check, lib, ptr


@dataclass
class History:
    eps: list = field(default_factory=list)      # accepted vertex fields (host, complex)
    J: list = field(default_factory=list)        # their misfits
    evaluations: int = 0
    seconds: float = 0.0
    solve_columns: int = 0                       # forward + adjoint right-hand sides solved
    iters: list = field(default_factory=list)    # (forward, adjoint) mean GMRES iterations per evaluation


class Inversion:
    """L-BFGS over the vertex permittivity on the library's device objective.

    recycle: how each evaluation's solves reuse the previous evaluation's
    fields: 'none' (zero start), 'warm' (each column from its own previous
    field) or 'project' (all columns from the least-squares combination of
    all previous fields).

    part: the non-overlapping partition (int32 [nt]) or None for the
    library's own; S_mes, S_empty: nrx x ntx complex (host or device)."""

    def __init__(self, problem, xyz, tet, part, n_sub: int, tx, rx, S_mes, S_empty, alpha: float,
                 precision: str = "c64", tol: float = 1e-8, restart: int = 30, block: int = 0, overlap: int = 1,
                 recycle="warm", p1: bool = False, maxit: int = 1000):
        self.P = problem
        self.nv = int(np.asarray(xyz).shape[0])
        modes = {"none": 0, "warm": 1, "project": 2, False: 0, True: 1, 0: 0, 1: 1, 2: 2}
        if recycle not in modes:
            raise ValueError("recycle must be 'none', 'warm' or 'project'")
        self.recycle, self.p1 = ("none", "warm", "project")[modes[recycle]], p1
        dev = problem.ctx.device
        self._mesh, self._keep = B.make_mesh(xyz, tet, np.zeros((0, 3), np.int32), np.zeros(0, np.int32))
        self._tx = np.ascontiguousarray(tx, dtype=np.int32)
        self._rx = np.ascontiguousarray(rx, dtype=np.int32)
        self._part = None if part is None else np.ascontiguousarray(part, dtype=np.int32)
        Sm = torch.as_tensor(np.asarray(S_mes, dtype=np.complex128)).to(dev).contiguous()
        Se = torch.as_tensor(np.asarray(S_empty, dtype=np.complex128)).to(dev).contiguous()
        assert Sm.shape == Se.shape == (self._rx.size, self._tx.size)
        o = B.mw_inversion_opts(alpha=float(alpha), p1=int(p1), recycle=modes[recycle], n_sub=int(n_sub),
                                overlap=int(overlap), precision={"c128": B.MW_C128, "c64": B.MW_C64}[precision],
                                solve=B.mw_solve_opts(tol=float(tol), restart=int(restart), maxit=int(maxit),
                                                      use_x0=0, block=int(block)))
        h = C.c_void_p()
        check(lib().mw_inversion_create(problem.h, C.byref(self._mesh),
                                        None if self._part is None else ptr(self._part), C.byref(o),
                                        self._tx.size, ptr(self._tx), self._rx.size, ptr(self._rx), ptr(Sm), ptr(Se),
                                        C.byref(h)))
        self.h = h
        self.history = History()

    def _info(self):
        inf = B.mw_inversion_info()
        check(lib().mw_inversion_get_info(self.h, 0, None, None, C.byref(inf)))
        ne = inf.evaluations
        f, a = np.zeros(max(ne, 1)), np.zeros(max(ne, 1))
        check(lib().mw_inversion_get_info(self.h, ne, ptr(f), ptr(a), C.byref(inf)))
        h = self.history
        h.evaluations, h.seconds, h.solve_columns = inf.evaluations, inf.seconds, inf.solve_columns
        h.iters = [(float(f[k]), float(a[k])) for k in range(ne)]

    def objective(self, eps_v: np.ndarray):
        """J and dJ/dRe eps_v + i dJ/dIm eps_v at the vertex field eps_v."""
        dev = self.P.ctx.device
        e = torch.from_numpy(np.ascontiguousarray(eps_v, dtype=np.complex128)).to(dev)
        g = torch.empty_like(e)
        J = C.c_double()
        check(lib().mw_inversion_objective(self.h, ptr(e), C.addressof(J), ptr(g)))
        self._info()
        return J.value, g.cpu().numpy()

    def run(self, eps0: np.ndarray, iters: int, mem: int = 5, step0: float = 0.5, c1: float = 1e-4,
            max_backtrack: int = 20) -> History:
        """L-BFGS from the vertex field eps0 for `iters` accepted steps (fewer if
        a line search fails); returns the accepted iterates and misfits."""
        dev = self.P.ctx.device
        e = torch.from_numpy(np.ascontiguousarray(eps0, dtype=np.complex128)).to(dev)
        Jh = np.zeros(iters + 1)
        Eh = np.zeros((iters + 1, self.nv), dtype=np.complex128)
        acc, nev = C.c_int32(), C.c_int32()
        lo = B.mw_lbfgs_opts(mem=mem, step0=step0, c1=c1, max_backtrack=max_backtrack)
        check(lib().mw_inversion_run(self.h, C.byref(lo), int(iters), ptr(e), ptr(Jh), ptr(Eh), C.addressof(acc),
                                     C.addressof(nev)))
        h = self.history
        h.J += Jh[: acc.value + 1].tolist()
        h.eps += [Eh[k].copy() for k in range(acc.value + 1)]
        self._info()
        return h

    def close(self):
        """Frees the library's inversion state (before the problem is closed)."""
        if self.h:
            check(lib().mw_inversion_destroy(self.h))
            self.h = None

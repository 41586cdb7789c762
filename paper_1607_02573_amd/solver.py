"""Torch-facing wrappers of the C ABI: device tensors in, device tensors out.

PyTorch provides device memory and the stream; every computation is a call
into libmw.so.  Multi-vectors are (n, nrhs) contiguous complex128 tensors on
the context's device.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from .binding import check, lib, ptr


@dataclass
class SolveInfo:
    iters: np.ndarray
    relres: np.ndarray
    max_iters: int
    cycles: int
    chunks: int
    t_solve: float


def _opts(tol, restart, maxit, use_x0, block=0):
    return B.mw_solve_opts(tol=float(tol), restart=int(restart), maxit=int(maxit), use_x0=int(use_x0),
                           block=int(block))


def _dev_tensor(t: torch.Tensor, dtype, device, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    return t


class Context:
    """A device, its stream and an HBM byte budget for the library."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream: torch.cuda.Stream | None = None):
        L = lib()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        check(L.mw_create(C.byref(h), device, int(budget_bytes)))
        self.h = h
        self.stream = stream or torch.cuda.current_stream(self.device)
        check(L.mw_set_stream(self.h, C.c_void_p(self.stream.cuda_stream)))

    def info(self) -> tuple[int, int]:
        """(budget, bytes held) of the context."""
        b, u = C.c_int64(), C.c_int64()
        check(lib().mw_ctx_get_info(self.h, C.addressof(b), C.addressof(u)))
        return b.value, u.value

    def close(self):
        if self.h:
            check(lib().mw_destroy(self.h))
            self.h = None


class Problem:
    """One mesh + permittivity + boundary data, its operator and factors."""

    def __init__(self, ctx: Context, xyz, tet, bface, btag, eps, k0: float, beta_imp: complex, ports=()):
        self.ctx = ctx
        L = lib()
        m, self._mesh_keep = B.make_mesh(xyz, tet, bface, btag)
        self.nv = int(m.nv)
        eps = np.ascontiguousarray(np.asarray(eps, dtype=np.complex128))
        assert eps.shape == (m.nt,)
        nports = len(ports)
        parr = (B.mw_port * max(nports, 1))()
        for k, pt in enumerate(ports):
            b = complex(pt.beta)
            parr[k].beta = B.mw_complex(b.real, b.imag)
            parr[k].radius, parr[k].theta, parr[k].width = pt.radius, pt.theta, pt.width
            for a in range(3):
                parr[k].pol[a] = float(pt.pol[a])
        h = C.c_void_p()
        b = complex(beta_imp)
        check(L.mw_assemble(ctx.h, C.byref(m), ptr(eps), float(k0), B.mw_complex(b.real, b.imag),
                            C.addressof(parr), nports, C.byref(h)))
        self.h = h
        self.k0 = float(k0)
        self.nports = nports
        inf = self.info()
        self.n, self.nnz, self.nt = inf.n, inf.nnz, inf.nt

    # ------------------------------------------------------------------ info
    def info(self) -> B.mw_problem_info:
        i = B.mw_problem_info()
        check(lib().mw_problem_get_info(self.h, C.byref(i)))
        return i

    def dof_edges(self):
        i = self.info()
        eod = np.empty(i.n, dtype=np.int32)
        ev = np.empty(i.n_edges * 2, dtype=np.int32)
        check(lib().mw_dof_edges(self.h, ptr(eod), ptr(ev)))
        return eod, ev.reshape(-1, 2)

    def matrix(self):
        dev = self.ctx.device
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(self.nnz, dtype=torch.complex128, device=dev)
        check(lib().mw_get_matrix(self.h, ptr(rp), ptr(col), ptr(val)))
        return rp, col, val

    def close(self):
        if self.h:
            check(lib().mw_destroy_problem(self.h))
            self.h = None

    # ------------------------------------------------------------------ data
    def update_eps(self, eps: torch.Tensor):
        _dev_tensor(eps, torch.complex128, self.ctx.device, "eps")
        check(lib().mw_update_eps(self.h, ptr(eps)))

    def update_eps_vertex(self, eps_v: torch.Tensor):
        """eps_r linear on every tetrahedron, given at the mesh vertices."""
        _dev_tensor(eps_v, torch.complex128, self.ctx.device, "eps_v")
        if eps_v.numel() != self.nv:
            raise ValueError(f"eps_v must have {self.nv} entries (one per vertex)")
        check(lib().mw_update_eps_vertex(self.h, ptr(eps_v)))

    def rhs_ports(self, tx) -> torch.Tensor:
        tx = np.ascontiguousarray(tx, dtype=np.int32)
        Bm = torch.empty((self.n, tx.size), dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_rhs_ports(self.h, tx.size, ptr(tx), ptr(Bm)))
        return Bm

    def rhs_dipoles(self, points, dirs=None) -> torch.Tensor:
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        if dirs is None:
            dirs = np.tile([0.0, 0.0, 1.0], (pts.shape[0], 1))
        dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        Bm = torch.empty((self.n, pts.shape[0]), dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_rhs_dipoles(self.h, pts.shape[0], ptr(pts), ptr(dirs), ptr(Bm)))
        return Bm

    def port_norms(self) -> np.ndarray:
        nu = np.empty(max(self.nports, 1))
        check(lib().mw_port_norms(self.h, ptr(nu)))
        return nu[: self.nports]

    # ------------------------------------------------------------------ preconditioner
    def set_coarse_space(self, kind: str):
        """'none' (one-level ORAS) or 'const' (two-level: three weighted
        constant fields per subdomain); takes effect at the next factor()."""
        k = {"none": B.MW_COARSE_NONE, "const": B.MW_COARSE_CONST}[kind]
        check(lib().mw_set_coarse_space(self.h, k))

    def set_factorization(self, kind: str):
        """'auto' (L D L^T when every tetrahedron is lossy, else LU), 'lu' or 'ldlt'."""
        k = {"auto": B.MW_FACTOR_AUTO, "lu": B.MW_FACTOR_LU, "ldlt": B.MW_FACTOR_LDLT}[kind]
        check(lib().mw_set_factorization(self.h, k))

    def set_solve_form(self, form: str):
        """'auto' (block rows for 512 subdomains or more), 'recursive' or 'rows';
        used by the next factor()."""
        f = {"auto": B.MW_SOLVE_AUTO, "recursive": B.MW_SOLVE_RECURSIVE, "rows": B.MW_SOLVE_ROWS}[form]
        check(lib().mw_set_solve_form(self.h, f))

    def set_krylov_basis(self, kind: str):
        """'auto' (complex FP32 with FP32 factors, the preconditioned candidates
        kept), 'fp32-lean' (FP32 without them: less memory per column) or
        'fp64'; used by later solves."""
        kinds = {"auto": B.MW_BASIS_AUTO, "fp64": B.MW_BASIS_FP64, "fp32-lean": B.MW_BASIS_FP32_LEAN}
        check(lib().mw_set_krylov_basis(self.h, kinds[kind]))

    def factor(self, part, n_sub: int, overlap: int = 1, precision: str = "c128"):
        """Fill and factor the B_i; part = None takes the library's own
        partition (recursive coordinate bisection of the centroids)."""
        prec = {"c128": B.MW_C128, "c64": B.MW_C64}[precision]
        if part is None:
            check(lib().mw_factor_subdomains(self.h, int(n_sub), int(overlap), prec, None))
            return
        part = np.ascontiguousarray(part, dtype=np.int32)
        check(lib().mw_factor_subdomains(self.h, int(n_sub), int(overlap), prec, ptr(part)))

    def factor_bytes(self, part, n_sub: int, overlap: int = 1, precision: str = "c64") -> int:
        """Device bytes of the factors of this partition (decomposition built once before)."""
        prec = {"c128": B.MW_C128, "c64": B.MW_C64}[precision]
        out = C.c_int64()
        if part is None:
            check(lib().mw_factor_bytes(self.h, int(n_sub), int(overlap), prec, None, C.addressof(out)))
            return out.value
        part = np.ascontiguousarray(part, dtype=np.int32)
        check(lib().mw_factor_bytes(self.h, int(n_sub), int(overlap), prec, ptr(part), C.addressof(out)))
        return out.value

    def state(self) -> int:
        """Counter that changes whenever the operator or the factors change."""
        return int(self.info().state)

    def release_factors(self):
        check(lib().mw_release_factors(self.h))

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        check(lib().mw_problem_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def apply_preconditioner(self, V: torch.Tensor) -> torch.Tensor:
        _dev_tensor(V, torch.complex128, self.ctx.device, "V")
        Z = torch.empty_like(V)
        check(lib().mw_apply_preconditioner(self.h, V.shape[1], ptr(V), ptr(Z)))
        return Z

    def apply_preconditioner_noalloc(self, V: torch.Tensor, Z: torch.Tensor) -> torch.Tensor:
        """Z = M^-1 V into the caller's Z, through the entry point that
        allocates nothing (local vectors in the library's fixed buffer)."""
        _dev_tensor(V, torch.complex128, self.ctx.device, "V")
        _dev_tensor(Z, torch.complex128, self.ctx.device, "Z")
        if Z.shape != V.shape:
            raise ValueError("Z must have the shape of V")
        check(lib().mw_apply_preconditioner_noalloc(self.h, V.shape[1], ptr(V), ptr(Z)))
        return Z

    # ------------------------------------------------------------------ solve
    def solve(self, Bm: torch.Tensor, tol=1e-8, restart=30, maxit=1000, x0: torch.Tensor | None = None,
              raise_noconv: bool = True, block: int = 0):
        """GMRES solve of A X = Bm; block = 32 groups the columns into blocks
        of 32 sharing one block Krylov space, block = 0 keeps one Krylov space
        per column (pseudo-block)."""
        _dev_tensor(Bm, torch.complex128, self.ctx.device, "B")
        nrhs = Bm.shape[1]
        if x0 is not None:
            if (not isinstance(x0, torch.Tensor) or x0.dtype != torch.complex128 or x0.device != self.ctx.device
                    or x0.shape != Bm.shape):
                raise ValueError(f"x0 must be a complex128 tensor of shape {tuple(Bm.shape)} on {self.ctx.device}")
            X = x0.clone(memory_format=torch.contiguous_format)
        else:
            X = torch.empty_like(Bm)
        it = np.zeros(nrhs, dtype=np.int32)
        rr = np.zeros(nrhs)
        info = B.mw_solve_info(iters=ptr(it) if nrhs else None, relres=ptr(rr) if nrhs else None)
        o = _opts(tol, restart, maxit, x0 is not None, block)
        code = lib().mw_solve(self.h, nrhs, ptr(Bm), ptr(X), C.byref(o), C.byref(info))
        if code != B.MW_OK and not (code == B.MW_ENOCONV and not raise_noconv):
            check(code)
        return X, SolveInfo(it, rr, info.max_iters, info.cycles, info.chunks, info.t_solve)

    # ------------------------------------------------------------------ S, J, gradient
    def s_matrix(self, U: torch.Tensor, rx) -> torch.Tensor:
        rx = np.ascontiguousarray(rx, dtype=np.int32)
        _dev_tensor(U, torch.complex128, self.ctx.device, "U")
        S = torch.empty((rx.size, U.shape[1]), dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_s_matrix(self.h, rx.size, ptr(rx), U.shape[1], ptr(U), ptr(S)))
        return S

    def adjoint_gradient(self, U: torch.Tensor, gS: torch.Tensor, tx, rx, tol=1e-8, restart=30, maxit=1000,
                         block: int = 0):
        tx = np.ascontiguousarray(tx, dtype=np.int32)
        rx = np.ascontiguousarray(rx, dtype=np.int32)
        _dev_tensor(U, torch.complex128, self.ctx.device, "U")
        _dev_tensor(gS, torch.complex128, self.ctx.device, "gS")
        g = torch.empty(self.nt, dtype=torch.complex128, device=self.ctx.device)
        o = _opts(tol, restart, maxit, 0, block)
        check(lib().mw_adjoint_gradient(self.h, tx.size, ptr(tx), rx.size, ptr(rx), ptr(U), ptr(gS), ptr(g),
                                        C.byref(o), None))
        return g

    def misfit_gradient(self, tx, rx, S_meas: torch.Tensor, tol=1e-8, restart=30, maxit=1000, block: int = 0):
        tx = np.ascontiguousarray(tx, dtype=np.int32)
        rx = np.ascontiguousarray(rx, dtype=np.int32)
        _dev_tensor(S_meas, torch.complex128, self.ctx.device, "S_meas")
        S = torch.empty((rx.size, tx.size), dtype=torch.complex128, device=self.ctx.device)
        g = torch.empty(self.nt, dtype=torch.complex128, device=self.ctx.device)
        J = C.c_double()
        o = _opts(tol, restart, maxit, 0, block)
        check(lib().mw_misfit_gradient(self.h, tx.size, ptr(tx), rx.size, ptr(rx), ptr(S_meas), C.addressof(J),
                                       ptr(S), ptr(g), C.byref(o)))
        return J.value, S, g


    def adjoint_rhs(self, gS: torch.Tensor, rx) -> torch.Tensor:
        rx = np.ascontiguousarray(rx, dtype=np.int32)
        _dev_tensor(gS, torch.complex128, self.ctx.device, "gS")
        lam = torch.empty((self.n, gS.shape[1]), dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_adjoint_rhs(self.h, rx.size, ptr(rx), gS.shape[1], ptr(gS), ptr(lam)))
        return lam

    def gradient(self, U: torch.Tensor, F: torch.Tensor) -> torch.Tensor:
        _dev_tensor(U, torch.complex128, self.ctx.device, "U")
        _dev_tensor(F, torch.complex128, self.ctx.device, "F")
        assert U.shape == F.shape
        g = torch.empty(self.nt, dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_gradient(self.h, U.shape[1], ptr(U), ptr(F), ptr(g)))
        return g

    def gradient_vertex(self, U: torch.Tensor, F: torch.Tensor) -> torch.Tensor:
        """Vertex gradient (dL/dRe + i dL/dIm of eps_v) with eps_r given at the vertices."""
        _dev_tensor(U, torch.complex128, self.ctx.device, "U")
        _dev_tensor(F, torch.complex128, self.ctx.device, "F")
        assert U.shape == F.shape
        g = torch.empty(self.nv, dtype=torch.complex128, device=self.ctx.device)
        check(lib().mw_gradient_vertex(self.h, U.shape[1], ptr(U), ptr(F), ptr(g)))
        return g

    def misfit(self, S: torch.Tensor, S_meas: torch.Tensor, weights: torch.Tensor | None = None):
        """J = 1/2 sum w |S - S_meas|^2 and gS = w (S - S_meas) (w = 1 if None)."""
        _dev_tensor(S, torch.complex128, self.ctx.device, "S")
        _dev_tensor(S_meas, torch.complex128, self.ctx.device, "S_meas")
        assert S.shape == S_meas.shape
        if weights is not None:
            _dev_tensor(weights, torch.float64, self.ctx.device, "weights")
            assert weights.shape == S.shape
        gS = torch.empty_like(S)
        J = C.c_double()
        check(lib().mw_misfit_weighted(self.h, S.numel(), ptr(S), ptr(S_meas),
                                       None if weights is None else ptr(weights), ptr(gS), C.addressof(J)))
        return J.value, gS


class Batch:
    """Continuous batching of GMRES columns over one problem's factors: requests
    join between restart cycles and leave when all their columns converged."""

    def __init__(self, problem: Problem, max_cols: int, tol=1e-8, restart=30, maxit=1000):
        self.problem = problem
        h = C.c_void_p()
        o = _opts(tol, restart, maxit, 0)
        check(lib().mw_batch_create(problem.h, int(max_cols), C.byref(o), C.byref(h)))
        self.h = h

    def join(self, tag: int, Bm: torch.Tensor):
        _dev_tensor(Bm, torch.complex128, self.problem.ctx.device, "B")
        check(lib().mw_batch_join(self.h, int(tag), Bm.shape[1], ptr(Bm)))

    def cycle(self) -> tuple[int, int]:
        """One restart cycle; returns (columns that ran, requests finished)."""
        na, nf = C.c_int32(), C.c_int32()
        check(lib().mw_batch_cycle(self.h, C.addressof(na), C.addressof(nf)))
        return na.value, nf.value

    def poll(self) -> tuple[int, int]:
        """(tag, ncols) of the oldest finished request, or (-1, 0)."""
        t, nc = C.c_int64(), C.c_int32()
        check(lib().mw_batch_poll(self.h, C.addressof(t), C.addressof(nc)))
        return t.value, nc.value

    def take(self, tag: int, ncols: int, raise_noconv: bool = True):
        X = torch.empty((self.problem.n, ncols), dtype=torch.complex128, device=self.problem.ctx.device)
        it = np.zeros(ncols, dtype=np.int32)
        rr = np.zeros(ncols)
        code = lib().mw_batch_take(self.h, int(tag), ptr(X), ptr(it), ptr(rr))
        if code != B.MW_OK and not (code == B.MW_ENOCONV and not raise_noconv):
            check(code)
        return X, it, rr

    def info(self) -> B.mw_batch_info:
        i = B.mw_batch_info()
        check(lib().mw_batch_get_info(self.h, C.byref(i)))
        return i

    def close(self):
        if self.h:
            check(lib().mw_batch_destroy(self.h))
            self.h = None


def problem_from_workload(ctx: Context, w) -> Problem:
    """Problem for a seeded synthetic workload (see mw_inputs.configs)."""
    m = w.mesh
    return Problem(ctx, m.xyz, m.tet, m.bface, m.btag, w.eps, w.k0, w.beta_imp, w.ports)

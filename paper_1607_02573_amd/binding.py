"""ctypes binding of libmw.so (include/mw.h): argument marshalling only.

Every step of the solve path runs inside the library's HIP kernels; this
module checks tensor shapes/dtypes/devices, passes raw pointers and turns
non-zero status codes into exceptions.  There is no CPU fallback: a missing
library raises ``MwLibraryMissing``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmw.so")

MW_OK, MW_EINVAL, MW_ENOMEM, MW_ESINGULAR, MW_ENOCONV, MW_ENUMERIC, MW_EDEVICE = 0, -1, -2, -3, -4, -5, -6
MW_C128, MW_C64 = 0, 1
MW_FACTOR_AUTO, MW_FACTOR_LU, MW_FACTOR_LDLT = 0, 1, 2
MW_SOLVE_AUTO, MW_SOLVE_RECURSIVE, MW_SOLVE_ROWS = 0, 1, 2
MW_BASIS_AUTO, MW_BASIS_FP64, MW_BASIS_FP32_LEAN = 0, 1, 2
MW_COARSE_NONE, MW_COARSE_CONST = 0, 1
STATUS_NAMES = {0: "MW_OK", -1: "MW_EINVAL", -2: "MW_ENOMEM", -3: "MW_ESINGULAR", -4: "MW_ENOCONV",
                -5: "MW_ENUMERIC", -6: "MW_EDEVICE"}


class MwLibraryMissing(RuntimeError):
    pass


class MwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class mw_complex(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class mw_mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("xyz", C.c_void_p), ("nt", C.c_int32), ("tet", C.c_void_p),
                ("nbf", C.c_int32), ("bface", C.c_void_p), ("btag", C.c_void_p)]


class mw_port(C.Structure):
    _fields_ = [("beta", mw_complex), ("radius", C.c_double), ("theta", C.c_double), ("width", C.c_double),
                ("pol", C.c_double * 3)]


class mw_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("maxit", C.c_int32), ("use_x0", C.c_int32),
                ("block", C.c_int32)]


class mw_solve_info(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("relres", C.c_void_p), ("max_iters", C.c_int32), ("cycles", C.c_int32),
                ("chunks", C.c_int32), ("t_solve", C.c_double)]


NOALLOC_SCRATCH_BYTES = 64 << 20   # MW_NOALLOC_SCRATCH_BYTES


class mw_problem_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_edges", C.c_int64), ("nt", C.c_int32),
                ("nports", C.c_int32), ("n_sub", C.c_int32), ("sum_ni", C.c_int64), ("max_ni", C.c_int32),
                ("precision", C.c_int32), ("factor_bytes", C.c_int64), ("t_assemble", C.c_double),
                ("t_decompose", C.c_double), ("t_factor", C.c_double), ("factorization", C.c_int32),
                ("state", C.c_int64), ("coarse_size", C.c_int32)]


class mw_lbfgs_opts(C.Structure):
    _fields_ = [("mem", C.c_int32), ("step0", C.c_double), ("c1", C.c_double), ("max_backtrack", C.c_int32)]


class mw_inversion_opts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("p1", C.c_int32), ("recycle", C.c_int32), ("n_sub", C.c_int32),
                ("overlap", C.c_int32), ("precision", C.c_int32), ("solve", mw_solve_opts)]


class mw_inversion_info(C.Structure):
    _fields_ = [("evaluations", C.c_int32), ("solve_columns", C.c_int64), ("seconds", C.c_double)]


# mw_objective_fn: (user, x, J, g) -> mw_status
OBJECTIVE_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                           C.POINTER(C.c_double))


class mw_batch_info(C.Structure):
    _fields_ = [("max_cols", C.c_int32), ("free_cols", C.c_int32), ("active_cols", C.c_int32),
                ("requests", C.c_int32), ("finished", C.c_int32), ("cycles", C.c_int64), ("slot_bytes", C.c_int64),
                ("work_bytes", C.c_int64), ("bytes_per_col", C.c_int64)]


_P = C.c_void_p
_I = C.c_int32
_SIGS = {
    "mw_create": [C.POINTER(_P), C.c_int, C.c_int64],
    "mw_set_stream": [_P, _P],
    "mw_destroy": [_P],
    "mw_assemble": [_P, C.POINTER(mw_mesh), _P, C.c_double, mw_complex, _P, _I, C.POINTER(_P)],
    "mw_update_eps": [_P, _P],
    "mw_problem_get_info": [_P, C.POINTER(mw_problem_info)],
    "mw_dof_edges": [_P, _P, _P],
    "mw_destroy_problem": [_P],
    "mw_get_matrix": [_P, _P, _P, _P],
    "mw_rhs_ports": [_P, _I, _P, _P],
    "mw_rhs_dipoles": [_P, _I, _P, _P, _P],
    "mw_factor_subdomains": [_P, _I, _I, C.c_int, _P],
    "mw_apply_preconditioner": [_P, _I, _P, _P],
    "mw_apply_preconditioner_noalloc": [_P, _I, _P, _P],
    "mw_solve": [_P, _I, _P, _P, C.POINTER(mw_solve_opts), C.POINTER(mw_solve_info)],
    "mw_s_matrix": [_P, _I, _P, _I, _P, _P],
    "mw_port_norms": [_P, _P],
    "mw_adjoint_gradient": [_P, _I, _P, _I, _P, _P, _P, _P, C.POINTER(mw_solve_opts), C.POINTER(mw_solve_info)],
    "mw_misfit_gradient": [_P, _I, _P, _I, _P, _P, _P, _P, _P, C.POINTER(mw_solve_opts)],
    "mw_adjoint_rhs": [_P, _I, _P, _I, _P, _P],
    "mw_gradient": [_P, _I, _P, _P, _P],
    "mw_misfit": [_P, C.c_int64, _P, _P, _P, _P],
    "mw_ctx_get_info": [_P, _P, _P],
    "mw_problem_set_stream": [_P, _P],
    "mw_release_factors": [_P],
    "mw_factor_bytes": [_P, _I, _I, C.c_int, _P, _P],
    "mw_batch_create": [_P, _I, C.POINTER(mw_solve_opts), C.POINTER(_P)],
    "mw_batch_join": [_P, C.c_int64, _I, _P],
    "mw_batch_cycle": [_P, _P, _P],
    "mw_batch_poll": [_P, _P, _P],
    "mw_batch_take": [_P, C.c_int64, _P, _P, _P],
    "mw_batch_get_info": [_P, C.POINTER(mw_batch_info)],
    "mw_batch_destroy": [_P],
    "mw_host_topology": [C.POINTER(mw_mesh), _P, _P, _P, _P, _P, _P],
    "mw_host_decomposition": [C.POINTER(mw_mesh), _P, _I, _I, _P, _P, _P, _P],
    "mw_host_block_lstsq": [_I, _I, _P, _P, C.c_double, _P, _P],
    "mw_host_partition": [C.POINTER(mw_mesh), _I, _P],
    "mw_host_factor_storage": [C.POINTER(mw_mesh), _P, _I, _I, _I, _P, _P, _P, _P],
    "mw_set_factorization": [_P, _I],
    "mw_set_solve_form": [_P, _I],
    "mw_set_krylov_basis": [_P, _I],
    "mw_update_eps_vertex": [_P, _P],
    "mw_gradient_vertex": [_P, _I, _P, _P, _P],
    "mw_set_coarse_space": [_P, _I],
    "mw_misfit_weighted": [_P, C.c_int64, _P, _P, _P, _P, _P],
    "mw_lbfgs": [C.c_int64, _P, _I, C.POINTER(mw_lbfgs_opts), OBJECTIVE_FN, _P, _P, _P, _P, _P],
    "mw_inversion_create": [_P, C.POINTER(mw_mesh), _P, C.POINTER(mw_inversion_opts), _I, _P, _I, _P, _P, _P,
                            C.POINTER(_P)],
    "mw_inversion_objective": [_P, _P, _P, _P],
    "mw_inversion_run": [_P, C.POINTER(mw_lbfgs_opts), _I, _P, _P, _P, _P, _P],
    "mw_inversion_get_info": [_P, _I, _P, _P, C.POINTER(mw_inversion_info)],
    "mw_inversion_destroy": [_P],
}
EXPORTED = list(_SIGS) + ["mw_last_error", "mw_host_last_error", "mw_timer_families", "mw_timer_name",
                          "mw_timer_enable", "mw_timer_reset"]

_lib = None


def lib():
    """Load libmw.so (built in-tree); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MwLibraryMissing(f"{LIB_PATH} not found: build it with `python -m paper_1607_02573_amd.build`")
    L = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.mw_last_error.restype = C.c_char_p
    L.mw_last_error.argtypes = []
    L.mw_host_last_error.restype = C.c_char_p
    L.mw_host_last_error.argtypes = []
    L.mw_timer_families.restype = C.c_int32
    L.mw_timer_families.argtypes = []
    L.mw_timer_name.restype = C.c_char_p
    L.mw_timer_name.argtypes = [C.c_int32]
    L.mw_timer_enable.restype = None
    L.mw_timer_enable.argtypes = [C.c_int32]
    L.mw_timer_reset.restype = None
    L.mw_timer_reset.argtypes = []
    L.mw_timer_read.restype = C.c_int
    L.mw_timer_read.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    _lib = L
    return L


def check(code: int, host: bool = False):
    if code != MW_OK:
        L = lib()
        msg = (L.mw_host_last_error() if host else L.mw_last_error()).decode(errors="replace")
        raise MwError(code, msg)


def ptr(a) -> int:
    """Raw address of a contiguous numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return a.data_ptr()


def make_mesh(xyz: np.ndarray, tet: np.ndarray, bface: np.ndarray, btag: np.ndarray):
    """mw_mesh over host arrays (the arrays are returned to keep them alive)."""
    keep = (np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tet, dtype=np.int32),
            np.ascontiguousarray(bface, dtype=np.int32), np.ascontiguousarray(btag, dtype=np.int32))
    m = mw_mesh(nv=keep[0].shape[0], xyz=ptr(keep[0]), nt=keep[1].shape[0], tet=ptr(keep[1]),
                nbf=keep[2].shape[0], bface=ptr(keep[2]) if keep[2].size else None,
                btag=ptr(keep[3]) if keep[3].size else None)
    return m, keep


def host_topology(xyz, tet, bface, btag):
    """Edge numbering and CSR pattern from the library's host code (no GPU)."""
    L = lib()
    m, keep = make_mesh(xyz, tet, bface, btag)
    n, nnz, ne = C.c_int64(), C.c_int64(), C.c_int64()
    check(L.mw_host_topology(C.byref(m), C.addressof(n), C.addressof(nnz), C.addressof(ne), None, None, None), True)
    eod = np.empty(n.value, dtype=np.int32)
    rp = np.empty(n.value + 1, dtype=np.int64)
    col = np.empty(nnz.value, dtype=np.int32)
    check(L.mw_host_topology(C.byref(m), C.addressof(n), C.addressof(nnz), C.addressof(ne), ptr(eod), ptr(rp),
                             ptr(col)), True)
    return {"n": n.value, "nnz": nnz.value, "n_edges": ne.value, "edge_of_dof": eod, "row_ptr": rp, "col": col}


def host_decomposition(xyz, tet, bface, btag, part, n_sub: int, overlap: int = 1):
    """Local unknowns and partition-of-unity weights from the library's host code."""
    L = lib()
    m, keep = make_mesh(xyz, tet, bface, btag)
    part = np.ascontiguousarray(part, dtype=np.int32)
    n_loc = np.zeros(n_sub, dtype=np.int32)
    nf = np.zeros(n_sub, dtype=np.int64)
    check(L.mw_host_decomposition(C.byref(m), ptr(part), n_sub, overlap, ptr(n_loc), ptr(nf), None, None), True)
    tot = int(n_loc.sum())
    sub_dof = np.empty(tot, dtype=np.int32)
    D = np.empty(tot)
    check(L.mw_host_decomposition(C.byref(m), ptr(part), n_sub, overlap, ptr(n_loc), ptr(nf), ptr(sub_dof),
                                  ptr(D)), True)
    off = np.r_[0, np.cumsum(n_loc)]
    return {"n_loc": n_loc, "n_faces": nf, "sub_dof": [sub_dof[off[i]:off[i + 1]] for i in range(n_sub)],
            "D": [D[off[i]:off[i + 1]] for i in range(n_sub)]}


def host_partition(xyz, tet, bface, btag, n_sub: int) -> np.ndarray:
    """The library's own partition (tet_part = NULL): int32 [nt]."""
    m, keep = make_mesh(xyz, tet, bface, btag)
    part = np.empty(m.nt, dtype=np.int32)
    check(lib().mw_host_partition(C.byref(m), int(n_sub), ptr(part)), host=True)
    del keep
    return part


def lbfgs(fun, x0: np.ndarray, iters: int, mem: int = 5, step0: float = 0.5, c1: float = 1e-4,
          max_backtrack: int = 20):
    """The library's host L-BFGS (mw_lbfgs) on a Python objective
    fun(x) -> (J, g) over real vectors; returns the last accepted x, the
    accepted J values and iterates, and the number of evaluations."""
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    n = x.size
    err = []

    def cb(user, xp, Jp, gp):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            J, g = fun(xv)
            Jp[0] = float(J)
            np.ctypeslib.as_array(gp, shape=(n,))[:] = np.asarray(g, dtype=np.float64)
            return MW_OK
        except Exception as e:  # pragma: no cover - surfaced below
            err.append(e)
            return MW_EINVAL

    f = OBJECTIVE_FN(cb)
    Jh = np.zeros(iters + 1)
    Xh = np.zeros((iters + 1, n))
    acc, nev = C.c_int32(), C.c_int32()
    o = mw_lbfgs_opts(mem=mem, step0=step0, c1=c1, max_backtrack=max_backtrack)
    code = lib().mw_lbfgs(n, ptr(x), iters, C.byref(o), f, None, ptr(Jh), ptr(Xh), C.addressof(acc),
                          C.addressof(nev))
    if err:
        raise err[0]
    check(code)
    return x, Jh[: acc.value + 1], Xh[: acc.value + 1], nev.value


def host_factor_storage(xyz, tet, bface, btag, part, n_sub: int, overlap: int = 1, sub: int = 0):
    """Factor storage of the decomposition: (dense elements, banded elements,
    stored column range [lo, hi) of every 64-row block of subdomain `sub`)."""
    m, keep = make_mesh(xyz, tet, bface, btag)
    part = np.ascontiguousarray(part, dtype=np.int32)
    dense, band = C.c_int64(), C.c_int64()
    lo = np.zeros(8192 // 64, dtype=np.int32)
    hi = np.zeros(8192 // 64, dtype=np.int32)
    check(lib().mw_host_factor_storage(C.byref(m), ptr(part), int(n_sub), int(overlap), int(sub), ptr(lo), ptr(hi),
                                       C.addressof(dense), C.addressof(band)), host=True)
    del keep
    nb = int((hi > 0).sum())
    return dense.value, band.value, lo[:nb], hi[:nb]


def timer_enable(on: bool = True):
    lib().mw_timer_enable(1 if on else 0)


def timer_reset():
    lib().mw_timer_reset()


def timer_read() -> dict:
    """{family: {launches, ms, flops, bytes}} since the last reset."""
    L = lib()
    out = {}
    for f in range(L.mw_timer_families()):
        n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        check(L.mw_timer_read(f, C.addressof(n), C.addressof(ms), C.addressof(fl), C.addressof(by)))
        out[L.mw_timer_name(f).decode()] = {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    return out


def host_block_lstsq(S0: np.ndarray, H: np.ndarray, width: int = 32):
    """Run the library's host least-squares update of block GMRES over the
    block columns of H ((steps+1)*32 x steps*32); returns the per-step
    residual norms [steps, 32] and the final Y [steps*32, 32]."""
    L = lib()
    steps = H.shape[1] // 32
    S0 = np.ascontiguousarray(S0, dtype=np.complex128)
    H = np.ascontiguousarray(H, dtype=np.complex128)
    res = np.zeros((steps, 32))
    Y = np.zeros((steps * 32, 32), dtype=np.complex128)
    check(L.mw_host_block_lstsq(steps, width, ptr(S0), ptr(H), 0.0, ptr(res), ptr(Y)), True)
    return res, Y


def host_block_cholesky(G: np.ndarray, thr: float):
    """The library's Cholesky factor of a 32 x 32 block Gram matrix and its
    count of pivots <= thr relative to the largest diagonal entry."""
    L = lib()
    G = np.ascontiguousarray(G, dtype=np.complex128)
    nd = np.zeros(1)
    R = np.zeros((32, 32), dtype=np.complex128)
    check(L.mw_host_block_lstsq(0, 32, None, ptr(G), float(thr), ptr(nd), ptr(R)), True)
    return R, int(nd[0])

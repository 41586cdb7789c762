"""MI355X-native ORAS-preconditioned GMRES for the edge-element Maxwell
systems of microwave tomography (Tournier et al., Parallel Computing).

The work happens in libmw.so (HIP kernels for gfx950 behind the C ABI of
include/mw.h); this package only binds it.  Build it with
``python -m paper_1607_02573_amd.build``.
"""
from .binding import LIB_PATH, MwError, MwLibraryMissing, lib  # noqa: F401


def __getattr__(name):
    # torch-dependent parts are imported lazily
    if name in ("Context", "Problem", "problem_from_workload", "SolveInfo"):
        from . import solver
        return getattr(solver, name)
    if name in ("MaxwellS", "s_of_eps"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)

"""Oracle: the ORAS preconditioner of oracle/dd.py spread over worker
processes, so that the large chamber meshes are factored and solved on all
host cores.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Nothing here is new arithmetic.  Each worker process (forked from the caller,
so it shares the assembled problem) builds and factors one contiguous share
of the subdomains with dd.decompose, then applies
    z_w = sum_{i in share w} R_i^T D_i B_i^-1 R_i v
(dd.oras_apply restricted to its share) to the vectors the caller places in
shared memory; the caller adds the partial sums z_w in worker order.  This is
equation (ORAS) of Section 3 with the sum over subdomains grouped by worker.
SuperLU factors cannot be pickled, which is why they stay inside the worker
that made them.

Fork only from a process that has not initialised a GPU runtime: the
workers use numpy and scipy alone, single-threaded.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from . import dd


def _worker(fp, part, delta, share, n, max_cols, vbuf, zbuf, slot, conn):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        # built a few at a time, keeping only what the apply needs (R_i, D_i
        # and the factors), so that the workers' memory stays near the
        # factors' own size
        subs = []
        cnt = dd.node_counts(fp.tet, part, fp.nv)
        for k in range(0, len(share), 32):
            for s in dd.decompose(fp, part, delta, factor=True, subset=list(share[k:k + 32]), cnt=cnt):
                s.B = s.tets = None
                subs.append(s)
        lu_bytes = sum(16 * s.lu.nnz for s in subs)   # (s.lu.L would copy the factors)
        conn.send(("ready", time.perf_counter() - t0, lu_bytes))
        V_all = np.frombuffer(vbuf, dtype=np.complex128)
        Z_all = np.frombuffer(zbuf, dtype=np.complex128).reshape(-1, n * max_cols)
        while True:
            msg = conn.recv()
            if msg is None:
                break
            nc = int(msg)
            V = V_all[: n * nc].reshape(n, nc)
            Z = Z_all[slot, : n * nc].reshape(n, nc)
            Z[:] = 0.0
            for s in subs:
                Z[s.gdof] += s.D[:, None] * s.lu.solve(np.ascontiguousarray(V[s.gdof]))
            conn.send("done")
    conn.close()


class PooledORAS:
    """M^-1 of equation (ORAS) over `nproc` forked workers (all host CPUs by
    default); apply() takes up to `max_cols` columns at a time."""

    def __init__(self, fp, part: np.ndarray, delta: int = 1, nproc: int | None = None, max_cols: int = 8):
        nsub = int(part.max()) + 1
        nproc = max(1, min(nproc or os.cpu_count() or 1, nsub))
        self.n, self.max_cols, self.nproc = fp.n, max_cols, nproc
        ctx = mp.get_context("fork")
        self._v = ctx.RawArray("d", 2 * fp.n * max_cols)
        self._z = ctx.RawArray("d", 2 * fp.n * max_cols * nproc)
        shares = np.array_split(np.arange(nsub), nproc)
        self._conns, self._procs = [], []
        t0 = time.perf_counter()
        for w, share in enumerate(shares):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(fp, part, delta, share, fp.n, max_cols, self._v, self._z, w, b),
                            daemon=True)
            p.start()
            self._conns.append(a)
            self._procs.append(p)
        ready = [c.recv() for c in self._conns]
        self.t_setup = time.perf_counter() - t0
        self.worker_setup_s = [r[1] for r in ready]
        self.lu_bytes = sum(r[2] for r in ready)
        self._V = np.frombuffer(self._v, dtype=np.complex128)
        self._Z = np.frombuffer(self._z, dtype=np.complex128).reshape(nproc, -1)

    def __call__(self, V: np.ndarray) -> np.ndarray:
        return self.apply(V)

    def apply(self, V: np.ndarray) -> np.ndarray:
        n, nc = V.shape
        out = np.empty((n, nc), dtype=np.complex128)
        for c0 in range(0, nc, self.max_cols):
            c1 = min(nc, c0 + self.max_cols)
            k = c1 - c0
            self._V[: n * k].reshape(n, k)[:] = V[:, c0:c1]
            for c in self._conns:
                c.send(k)
            for c in self._conns:
                assert c.recv() == "done"
            Z = self._Z[0, : n * k].reshape(n, k).copy()
            for w in range(1, self.nproc):
                Z += self._Z[w, : n * k].reshape(n, k)
            out[:, c0:c1] = Z
        return out

    def close(self):
        for c in self._conns:
            try:
                c.send(None)
            except (BrokenPipeError, OSError):
                pass
        for p in self._procs:
            p.join(timeout=30)
            if p.is_alive():
                p.kill()
        self._conns, self._procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

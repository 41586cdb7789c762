"""Serving loop: solve and misfit-gradient requests over a menu of problems
on one GPU.

The library supplies the mechanisms: the context's byte budget (a hard
limit), factors that can be released and rebuilt without redoing the
decomposition (the factor cache), continuous batching of GMRES columns
(mw_batch_*: columns join and leave at restart boundaries) and one HIP stream
per problem.  This module adds the policy: an arrival queue, admission by
bytes with least-recently-used eviction of idle factors, and one worker
thread per problem that joins admitted requests into its batch, runs restart
cycles and finishes requests (S matrix; for gradients the misfit, the adjoint
sources, a second pass through the batch and the gradient).

Admission counts, per problem: its factors and column slots while they are
resident, plus the GMRES workspace of the widest set of open columns since
the batch last idled (the library frees that workspace when a batch idles).
A request wider than what fits beside its factors is split into column
groups that are admitted separately.  The PyTorch tensors a group passes
through (sources, fields, adjoint sources: at most four n-vectors per
column at a time) are counted per column too, and each worker returns its
stream's cached blocks to the device when a group finishes, so that the
library's own allocations, which fail rather than wait, always find room.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .solver import Batch, Context, Problem


@dataclass(eq=False)
class Group:
    """Columns of one request admitted together."""
    req: object
    cols: np.ndarray          # indices into req.tx
    phase: int = 0            # gradient: 0 forward, 1 adjoint
    U: torch.Tensor | None = None


@dataclass
class Outcome:
    rid: int
    kind: str
    mesh: int
    version: int
    ncols: int
    t_arrive: float
    t_admit: float = -1.0
    t_done: float = -1.0
    iters_max: int = 0
    relres_max: float = 0.0
    J: float | None = None
    error: str | None = None
    groups_left: int = 0
    S: dict = field(default_factory=dict)     # group start column -> S block (host)
    grad: torch.Tensor | None = None


class Admission:
    """Byte accounting of the serving loop (host only).  Each problem key has
    (factor_bytes + slot_bytes) while its factors are wanted resident, and
    bytes_per_col * peak_cols of GMRES workspace."""

    def __init__(self, budget: int, base: int):
        self.budget, self.base = int(budget), int(base)
        self.p = {}

    def add_problem(self, key, factor_bytes: int, slot_bytes: int, bytes_per_col: int, max_cols: int):
        self.p[key] = dict(factor=int(factor_bytes), slots=int(slot_bytes), per_col=int(bytes_per_col),
                           max_cols=int(max_cols), resident=False, open=0, peak=0, last=0.0, evicting=False)

    def reserved(self, key) -> int:
        q = self.p[key]
        return (q["factor"] + q["slots"] if q["resident"] else 0) + q["per_col"] * q["peak"]

    def total(self) -> int:
        return self.base + sum(self.reserved(k) for k in self.p)

    def delta(self, key, ncols: int) -> int:
        q = self.p[key]
        d = 0 if q["resident"] else q["factor"] + q["slots"]
        return d + q["per_col"] * (max(q["peak"], q["open"] + ncols) - q["peak"])

    def fits(self, key, ncols: int) -> bool:
        q = self.p[key]
        return q["open"] + ncols <= q["max_cols"] and self.total() + self.delta(key, ncols) <= self.budget

    def group_cols(self, key) -> int:
        """Widest column group that fits beside this problem's factors alone."""
        q = self.p[key]
        room = self.budget - self.base - q["factor"] - q["slots"]
        return int(max(0, min(q["max_cols"], room // max(q["per_col"], 1))))

    def admit(self, key, ncols: int, now: float):
        q = self.p[key]
        q["resident"] = True
        q["evicting"] = False
        q["open"] += ncols
        q["peak"] = max(q["peak"], q["open"])
        q["last"] = now

    def finish(self, key, ncols: int):
        q = self.p[key]
        q["open"] -= ncols
        assert q["open"] >= 0
        if q["open"] == 0:
            q["peak"] = 0

    def victims(self, key, need: int, busy) -> list:
        """Idle resident problems (least recently used first) whose eviction frees `need` bytes."""
        cand = sorted((k for k, q in self.p.items() if k != key and q["resident"] and q["open"] == 0
                       and not q["evicting"] and k not in busy), key=lambda k: self.p[k]["last"])
        out, freed = [], 0
        for k in cand:
            if freed >= need:
                break
            out.append(k)
            freed += self.p[k]["factor"] + self.p[k]["slots"]
        return out if freed >= need else []

    def evicted(self, key):
        q = self.p[key]
        q["resident"] = False
        q["evicting"] = False
        q["peak"] = 0


class _Slot:
    def __init__(self, key, problem: Problem, part, n_sub: int, stream):
        self.key = key
        self.problem = problem
        self.part = part
        self.n_sub = n_sub
        self.stream = stream
        self.inbox = deque()
        self.batch: Batch | None = None
        self.factored = False
        self.evict = False
        self.tags = {}
        self.next_tag = 0
        self.thread = None
        self.factorisations = 0


class Server:
    """menu: list of mw_inputs.serving.MenuEntry.  Builds every (mesh, version)
    problem, its decomposition and its byte figures before serving."""

    TORCH_VECTORS_PER_COL = 4

    def __init__(self, ctx: Context, menu, tol=1e-8, restart=30, maxit=1000, max_cols=160, log=print,
                 budget_bytes: int | None = None, basis: str = "fp32-lean"):
        self.ctx, self.tol, self.restart, self.maxit, self.log = ctx, tol, restart, maxit, log
        self.cond = threading.Condition()
        self.slots = {}
        self.stop = False
        self.evictions = 0
        t0 = time.perf_counter()
        figures = {}
        for mi, entry in enumerate(menu):
            w = entry.workload
            for v, eps in enumerate(entry.eps_versions):
                stream = torch.cuda.Stream(device=ctx.device)
                m = w.mesh
                with torch.cuda.stream(stream):
                    P = Problem(ctx, m.xyz, m.tet, m.bface, m.btag, eps, w.k0, w.beta_imp, w.ports)
                    P.set_stream(stream)
                    # batches are bounded by memory: the lean FP32 basis costs
                    # m n 8 bytes less per column than keeping the
                    # preconditioned candidates, so more columns share a batch
                    # (400-request run with 1 GHz meshes: p99 49.8 against
                    # 90.7 s, 88 against 68 columns/s)
                    P.set_krylov_basis(basis)
                    P.factor(w.part, w.n_sub, 1, "c64")       # builds the decomposition once
                    fb = P.factor_bytes(w.part, w.n_sub, 1, "c64")
                    b = Batch(P, max_cols, tol, restart, maxit)
                    inf = b.info()
                    b.close()
                    P.release_factors()
                key = (mi, v)
                self.slots[key] = _Slot(key, P, w.part, w.n_sub, stream)
                figures[key] = (fb, inf.slot_bytes, inf.bytes_per_col + self.TORCH_VECTORS_PER_COL * P.n * 16,
                                max_cols)
                self.log(f"[serve] problem {entry.name} v{v}: n={P.n}, {w.n_sub} subdomains, factors "
                         f"{fb / 2**30:.1f} GiB, {inf.bytes_per_col / 2**20:.0f} MiB per column")
        budget, used = ctx.info()
        self.adm = Admission(min(budget, budget_bytes) if budget_bytes else budget, used)
        for key, f in figures.items():
            self.adm.add_problem(key, *f)
        self.t_setup = time.perf_counter() - t0

    # -------------------------------------------------------------- workers
    def _worker(self, s: _Slot):
        while True:
            with self.cond:
                while not (s.inbox or s.tags or s.evict or self.stop):
                    self.cond.wait()
                if self.stop and not s.inbox and not s.tags:
                    return
                evict = s.evict and not s.inbox and not s.tags
                jobs = list(s.inbox)
                s.inbox.clear()
            try:
                with torch.cuda.stream(s.stream):
                    if evict:
                        self._evict(s)
                        continue
                    self._step(s, jobs)
            except Exception as e:  # a failed library call fails the requests it touched
                self.log(f"[serve] problem {s.key}: {e}")
                with self.cond:
                    failed = {id(g): g for g in jobs + list(s.tags.values())}
                    for g in failed.values():
                        self._finish(s, g, error=str(e))
                    s.tags.clear()
                if s.batch is not None:   # its slots may hold the failed columns
                    try:
                        s.batch.close()
                    finally:
                        s.batch = None

    def _evict(self, s: _Slot):
        if s.batch is not None:
            s.batch.close()
            s.batch = None
        s.problem.release_factors()
        s.factored = False
        with self.cond:
            s.evict = False
            self.adm.evicted(s.key)
            self.evictions += 1
            self.cond.notify_all()

    def _step(self, s: _Slot, jobs):
        P = s.problem
        if jobs and not s.factored:
            P.factor(s.part, s.n_sub, 1, "c64")
            s.factored = True
            s.factorisations += 1
        if jobs and s.batch is None:
            s.batch = Batch(P, self.adm.p[s.key]["max_cols"], self.tol, self.restart, self.maxit)
        for g in jobs:
            r = g.req
            Bm = P.rhs_ports(r.tx[g.cols])
            self._join(s, g, Bm)
        if s.tags:
            s.batch.cycle()
        while True:
            tag, nc = s.batch.poll()
            if tag < 0:
                break
            X, it, rr = s.batch.take(tag, nc, raise_noconv=False)
            g = s.tags.pop(tag)
            out = self.outcomes[g.req.rid]
            out.iters_max = max(out.iters_max, int(it.max()))
            out.relres_max = max(out.relres_max, float(rr.max()))
            r = g.req
            if r.kind == "solve":
                out.S[int(g.cols[0])] = P.s_matrix(X, r.rx).cpu()
                del X
                torch.cuda.empty_cache()
                with self.cond:
                    self._finish(s, g)
            elif g.phase == 0:
                S = P.s_matrix(X, r.rx)
                Sm = torch.from_numpy(np.ascontiguousarray(r.s_meas[:, g.cols])).to(S.device)
                J, gS = P.misfit(S, Sm)
                out.J = J
                out.S[int(g.cols[0])] = S.cpu()
                lam = P.adjoint_rhs(gS, r.rx)
                g.phase, g.U = 1, X
                self._join(s, g, lam)
            else:
                out.grad = P.gradient(g.U, X)
                g.U = None
                del X
                torch.cuda.empty_cache()
                with self.cond:
                    self._finish(s, g)

    def _join(self, s: _Slot, g: Group, Bm):
        tag = s.next_tag
        s.next_tag += 1
        s.batch.join(tag, Bm)
        s.tags[tag] = g

    def _finish(self, s: _Slot, g: Group, error: str | None = None):
        """Called with the lock held."""
        out = self.outcomes[g.req.rid]
        if error:
            out.error = error
        self.adm.finish(s.key, len(g.cols))
        out.groups_left -= 1
        if out.groups_left == 0:
            out.t_done = time.perf_counter() - self.t0
            self.n_done += 1
        self.cond.notify_all()

    # -------------------------------------------------------------- dispatcher
    def run(self, requests, progress_s: float = 10.0):
        """Serves `requests` (mw_inputs.serving.Request, sorted by arrival) in
        real time; returns one Outcome per request."""
        reqs = sorted(requests, key=lambda r: r.t_arrive)
        self.outcomes = {r.rid: Outcome(r.rid, r.kind, r.mesh, r.version, r.ncols, r.t_arrive) for r in reqs}
        self.n_done = 0
        self.stop = False
        self.t0 = time.perf_counter()
        for s in self.slots.values():
            s.thread = threading.Thread(target=self._worker, args=(s,), daemon=True)
            s.thread.start()
        pending = deque()
        i = 0
        last_log = 0.0
        with self.cond:
            while self.n_done < len(reqs):
                now = time.perf_counter() - self.t0
                while i < len(reqs) and reqs[i].t_arrive <= now:
                    r = reqs[i]
                    key = (r.mesh, r.version)
                    gc = self.adm.group_cols(key)
                    if gc < 1:
                        raise RuntimeError(f"problem {key} does not fit the budget even alone")
                    groups = [Group(r, np.arange(a, min(a + gc, r.ncols))) for a in range(0, r.ncols, gc)]
                    self.outcomes[r.rid].groups_left = len(groups)
                    pending.extend(groups)
                    i += 1
                self._admit(pending, now)
                if now - last_log >= progress_s:
                    last_log = now
                    self.log(f"[serve] t={now:6.1f}s arrived {i}/{len(reqs)} done {self.n_done} queued groups "
                             f"{len(pending)} reserved {self.adm.total() / 2**30:.0f}/{self.adm.budget / 2**30:.0f} GiB "
                             f"resident {sum(q['resident'] for q in self.adm.p.values())}")
                wait = (reqs[i].t_arrive - now) if i < len(reqs) else progress_s
                self.cond.wait(timeout=max(0.001, min(wait, 1.0)))
            self.stop = True
            self.cond.notify_all()
        for s in self.slots.values():
            s.thread.join()
        return [self.outcomes[r.rid] for r in reqs]

    def _admit(self, pending: deque, now: float):
        """First fit in arrival order; the oldest group that does not fit may
        evict idle factors (lock held)."""
        blocked = False
        busy = {key for key, s in self.slots.items() if s.inbox or s.tags}
        waiting = list(pending)
        pending.clear()
        for g in waiting:
            key = (g.req.mesh, g.req.version)
            nc = len(g.cols)
            s = self.slots[key]
            if self.adm.fits(key, nc) and not s.evict:
                self.adm.admit(key, nc, now)
                out = self.outcomes[g.req.rid]
                if out.t_admit < 0:
                    out.t_admit = now
                s.inbox.append(g)
                busy.add(key)
                self.cond.notify_all()
                continue
            pending.append(g)
            if not blocked:
                blocked = True
                q = self.adm.p[key]
                if q["open"] + nc > q["max_cols"]:
                    continue
                need = self.adm.total() + self.adm.delta(key, nc) - self.adm.budget
                for v in self.adm.victims(key, need, busy):
                    self.adm.p[v]["evicting"] = True
                    self.slots[v].evict = True
                self.cond.notify_all()

    def close(self):
        for s in self.slots.values():
            if s.batch is not None:
                s.batch.close()
                s.batch = None
            s.problem.close()


def summarize(outcomes, t_wall: float) -> dict:
    lat = np.array([o.t_done - o.t_arrive for o in outcomes if o.error is None])
    cols = sum(o.ncols * (2 if o.kind == "gradient" else 1) for o in outcomes if o.error is None)
    by_kind = {}
    for kind in ("solve", "gradient"):
        lk = np.array([o.t_done - o.t_arrive for o in outcomes if o.kind == kind and o.error is None])
        if lk.size:
            by_kind[kind] = {"n": int(lk.size), "p50_s": float(np.percentile(lk, 50)),
                             "p99_s": float(np.percentile(lk, 99))}
    return {"requests": len(outcomes), "failed": sum(o.error is not None for o in outcomes),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "rhs_columns": int(cols), "rhs_per_s": cols / t_wall if t_wall > 0 else None,
            "makespan_s": t_wall, "by_kind": by_kind,
            "max_relres": max((o.relres_max for o in outcomes), default=0.0)}

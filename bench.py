#!/usr/bin/env python3
"""Benchmark: repeated ORAS-GMRES solves of the edge-element Maxwell system
for many antenna right-hand sides on one MI355X.

One step is one pass of the whole solve path over one batch, as every
iteration of the inversion repeats it after eps changes:
  eps (resident on the device) -> assembly of A's values, dense subdomain
  matrices and their LU factors, port sources, ORAS-preconditioned
  pseudo-block GMRES to FP64 relative residual tol, S-matrix.
The mesh topology and the overlapping decomposition (index lists) do not
change between inversion iterations; they are built once before timing.

Default workload: imaging chamber at 1 GHz (1,375,920 tetrahedra,
1,597,629 unknowns), 160 ports on 5 rings, 1600 subdomains, overlap 1,
GMRES(30), tol 1e-8, mixed precision (complex FP32 subdomain factors and
triangular solves, FP64 GMRES with iterative refinement); the FP64 path
(complex FP64 factors) is timed beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6}
MFMA_FAMILIES = ("trsm_gemm", "lu_gemm")
# block Gram-Schmidt of block GMRES: complex FP64 products on the matrix cores
FP64_MFMA_FAMILIES = ("bgs_dots", "bgs_update")

# HBM bytes per launch of the dominant kernel family, from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE) over this benchmark at its
# defaults, each scaled by what the same counter reads for a plain copy of
# known size (--copy-probe-mib).  Valid only for the kernel source it was
# taken on: a different hash of that file reports null.
PMC_TRAFFIC = {"family": "trsm_gemm", "source": "paper_1607_02573_amd/csrc/dense.hip",
               "sha256": "bea924fae70f20f8c33e40644df2ef35a9e5f4525516ed97ffd74958c3d89e38",
               "bytes_per_launch": 1.0437e11}   # FETCH 9.194e10 + WRITE 1.243e10 (pmc_row_sweep_chamber10_mixed)


def measured_traffic(family: str):
    import hashlib
    t = PMC_TRAFFIC
    if t is None or t["family"] != family:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return t["bytes_per_launch"]


MIXED_DTYPE = "c64 factors/TRSM (FP32 MFMA), c64 Krylov basis, f64 GMRES arithmetic and residuals"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    import mw_inputs as mi
    if name == "chamber10":
        return mi.configs.chamber10()
    if name == "chamber05":
        return mi.configs.chamber05()
    if name == "inversion05":
        return mi.configs.inversion05()
    if name == "cube8":
        return mi.configs.cube8()
    raise SystemExit(f"unknown workload {name}")


def run_steps(P, w, eps_dev, prec, nsteps, tol, restart, maxit, tx, rx, block=0):
    import torch
    stats = []
    for _ in range(nsteps):
        t0 = time.perf_counter()
        P.update_eps(eps_dev)                       # A(eps) values on the device
        P.factor(w.part, w.n_sub, 1, prec)          # B_i fill + batched LU
        t1 = time.perf_counter()
        Bm = P.rhs_ports(tx) if w.dipoles is None else P.rhs_dipoles(w.dipoles)
        X, info = P.solve(Bm, tol=tol, restart=restart, maxit=maxit, raise_noconv=False, block=block)
        S = P.s_matrix(X, rx) if w.dipoles is None and len(rx) else None
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stats.append({"t_setup": t1 - t0, "t_solve": t2 - t1, "iters": info.iters.copy(),
                      "relres": info.relres.copy(), "chunks": info.chunks, "cycles": info.cycles})
        last = (X, S)
    return stats, last


def family_table(fam: dict, mfma_peak_tflops: float, wall_s: float):
    """Per kernel family: time, rates, the roofline that bounds it and the
    fraction of it reached.  The roofline time of a family is the larger of
    its algorithmic flops at the compute peak (MFMA at `mfma_peak_tflops` for
    the dense factor/solve families, FP64 vector for the Krylov kernels) and
    its algorithmic bytes at 8 TB/s.  Also the whole run's roofline time (the
    sum over families) over its wall time."""
    out, roof_s = {}, 0.0
    for k, v in fam.items():
        s = max(v["ms"], 1e-9) * 1e-3
        dense = k in MFMA_FAMILIES or k in ("trsm_leaf", "lu_panel", "lu_other") or k in FP64_MFMA_FAMILIES
        peak = PEAK["fp64_TFLOPs"] if (k in FP64_MFMA_FAMILIES or not dense) else mfma_peak_tflops
        t_flop = v["flops"] / (peak * 1e12)
        t_byte = v["bytes"] / (PEAK["hbm_GBs"] * 1e9)
        t_roof, bound = (t_flop, "mfma" if dense else "alu") if t_flop >= t_byte else (t_byte, "hbm")
        roof_s += t_roof
        out[k] = {"ms": round(v["ms"], 2), "launches": v["launches"], "TFLOPs": round(v["flops"] / s / 1e12, 2),
                  "GBs": round(v["bytes"] / s / 1e9, 1), "bound": bound, "frac": round(t_roof / s, 3)}
    return out, {"roofline_s": roof_s, "wall_s": wall_s, "frac": roof_s / wall_s if wall_s > 0 else None}


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(w, tx, tol: float, restart: int, ncols: int = 2):
    """The oracle (plain FP64 numpy/scipy, SuperLU subdomain factors) timed on
    this host's cores, on the same workload: re-assembly of A for the
    permittivity and the port sources of all columns, then every subdomain
    built and factored on a process pool of all cores (oracle/pool.py), then
    its pseudo-block ORAS-GMRES on `ncols` of the port columns to the same
    tolerance.  Columns are independent in pseudo-block GMRES, so the whole
    job's time is t_assembly + t_factor + (nrhs / ncols) * t_solve.  Runs
    before the GPU is touched (the pool forks).  Returns the baseline record
    and the oracle's problem (matrix and sources), which the per-result
    error check reuses."""
    from oracle import fem, gmres, pool
    nproc = host_cores()
    nrhs = len(tx)
    t0 = time.perf_counter()
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    fp = fem.with_eps(fp, w.eps)
    B = fem.rhs_ports(fp, w.ports, tx) if w.dipoles is None else fem.rhs_dipoles(fp, w.dipoles)
    t_asm = time.perf_counter() - t0
    cols = np.unique(np.linspace(0, nrhs - 1, ncols).round().astype(int))
    with pool.PooledORAS(fp, w.part, w.overlap, nproc=nproc, max_cols=len(cols)) as M:
        t_fac = M.t_setup
        t0 = time.perf_counter()
        _, it, rr = gmres.gmres(fp.A, B[:, cols], M.apply, tol=tol, restart=restart)
        t_solve = time.perf_counter() - t0
    total = t_asm + t_fac + (nrhs / len(cols)) * t_solve
    rec = {"value": nrhs / total, "unit": "RHS/s", "cores": nproc, "kind": "oracle",
           "host_cpus": os.cpu_count(),
           "sample": (f"oracle on {w.name} ({fp.n} unknowns) on {nproc} host cores, measured: re-assembly of A "
                      f"and the {nrhs} sources {t_asm:.1f} s; all {w.n_sub} subdomains built and SuperLU-factored "
                      f"on a {nproc}-process pool {t_fac:.1f} s; pseudo-block ORAS-GMRES of columns "
                      f"{cols.tolist()} to {tol:g}: {t_solve:.1f} s, iterations {it.tolist()}, relres max "
                      f"{rr.max():.1e}; RHS/s = {nrhs} / (assembly + factor + {nrhs}/{len(cols)} x solve) "
                      f"(columns are independent); topology {t_build:.1f} s not counted")}
    return rec, fp, B


def oracle_errors(w, fp, B, X, tx, label: str):
    """Error of GPU fields X (device, n x nrhs, columns = ports tx) against
    the oracle: the relative residual ||b - A x|| / ||b|| with the oracle's
    own matrix and sources on 16 evenly spaced columns, and, where stored
    oracle fields exist for this workload (tests/golden, written by the
    oracle's ORAS-GMRES at 1e-10), the field error on their ports."""
    import torch
    nrhs = X.shape[1]
    cols = np.unique(np.linspace(0, nrhs - 1, min(16, nrhs)).round().astype(int))
    Xc = X[:, cols].cpu().numpy()
    res = np.linalg.norm(B[:, cols] - fp.A @ Xc, axis=0) / np.linalg.norm(B[:, cols], axis=0)
    out = {"relres_oracle_A_max": float(res.max()), "relres_columns": len(cols)}
    path = os.path.join(ROOT, "tests", "golden", f"{w.name}_oracle.npz")
    if os.path.exists(path) and w.dipoles is None:
        z = np.load(path)
        pos = {int(t): k for k, t in enumerate(tx)}
        if int(z["fingerprint"][0]) == fp.n and all(int(t) in pos for t in z["tx"]):
            c = [pos[int(t)] for t in z["tx"]]
            Xs = X[torch.from_numpy(z["idx"]).to(X.device)][:, c].cpu().numpy()
            e_s = np.linalg.norm(Xs - z["U_sample"], axis=0) / np.linalg.norm(z["U_sample"], axis=0)
            e_n = np.abs(torch.linalg.norm(X[:, c], dim=0).cpu().numpy() - z["norms"]) / z["norms"]
            out["fields_vs_oracle"] = {"ports": [int(t) for t in z["tx"]], "oracle_tol": float(z["tol"]),
                                       "sample_relL2_max": float(e_s.max()), "norm_rel_max": float(e_n.max()),
                                       "sample_size": int(z["idx"].size)}
    log(f"[bench] {label} vs oracle: relres (oracle A) max {out['relres_oracle_A_max']:.2e}"
        + (f", fields {out['fields_vs_oracle']['sample_relL2_max']:.2e}" if "fields_vs_oracle" in out else ""))
    return out


def serving_leg(args, freqs, n_req: int, rate: float):
    """Continuous-batching service over a menu of chamber problems (seeded
    Poisson arrivals of solve and gradient requests); returns the summary."""
    import torch

    import mw_inputs as mi
    from paper_1607_02573_amd import serve, solver
    menu = mi.serving.serving_menu(freqs=freqs)
    reqs = mi.serving.serving_requests(n_req=n_req, rate=rate, n_meshes=len(menu))
    total = torch.cuda.mem_get_info()[1]
    ctx = solver.Context(0, budget_bytes=int(total - (8 << 30)))
    srv = serve.Server(ctx, menu, tol=args.tol, restart=args.restart, maxit=args.maxit, log=log,
                       budget_bytes=int(total - (20 << 30)))
    t0 = time.perf_counter()
    out = srv.run(reqs)
    t_wall = time.perf_counter() - t0
    summ = serve.summarize(out, t_wall)
    summ["evictions"] = srv.evictions
    summ["setup_s"] = srv.t_setup
    summ["factorisations"] = {f"{menu[k[0]].name}/v{k[1]}": sl.factorisations for k, sl in srv.slots.items()}
    summ["budget_bytes"] = srv.adm.budget
    summ["menu"] = [f"{e.name}: {e.n_edges} edges, {e.workload.n_sub} subdomains" for e in menu]
    srv.close()
    ctx.close()
    return summ


def serve_main(args):
    """Continuous-batching service over a menu of problems: Poisson arrivals,
    admission by bytes, factor cache with LRU eviction, one stream per problem."""
    import torch

    import mw_inputs as mi
    from paper_1607_02573_amd import serve, solver
    log("[serve] generating the menu (4 chamber meshes, 2 permittivity versions each)")
    t0 = time.perf_counter()
    menu = mi.serving.serving_menu()
    log(f"[serve] menu ready in {time.perf_counter() - t0:.1f} s: " +
        ", ".join(f"{e.name} {e.n_edges} edges / {e.workload.n_sub} subdomains" for e in menu))
    reqs = mi.serving.serving_requests(n_req=args.serve_requests, rate=args.serve_rate)
    total = torch.cuda.mem_get_info()[1]
    # library hard cap 8 GiB below the device; admission (library + PyTorch
    # temporaries) 20 GiB below it
    ctx = solver.Context(0, budget_bytes=int(total - (8 << 30)))
    srv = serve.Server(ctx, menu, tol=args.tol, restart=args.restart, maxit=args.maxit, log=log,
                       budget_bytes=int(total - (20 << 30)))
    log(f"[serve] {len(srv.slots)} problems set up in {srv.t_setup:.1f} s; serving {len(reqs)} requests "
        f"at {args.serve_rate}/s")
    t0 = time.perf_counter()
    out = srv.run(reqs)
    t_wall = time.perf_counter() - t0
    summ = serve.summarize(out, t_wall)
    facts = {f"{menu[k[0]].name}/v{k[1]}": s.factorisations for k, s in srv.slots.items()}
    line = {
        "metric": "serving request latency p50 (p99 beside it), mixed precision, rel-res tol",
        "value": summ["p50_s"], "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "p99_s": summ["p99_s"], "mean_s": summ["mean_s"], "by_kind": summ["by_kind"],
        "rhs_columns": summ["rhs_columns"], "rhs_per_s": summ["rhs_per_s"], "makespan_s": t_wall,
        "failed": summ["failed"], "max_relres": summ["max_relres"],
        "factorisations": facts, "evictions": srv.evictions, "setup_s": srv.t_setup,
        "dtype": MIXED_DTYPE, "data": "synthetic",
        "config": {"workload": "chamber serving menu: 0.3125/0.5/0.75/1 GHz meshes x 2 permittivity versions, "
                               "160 ports, ceil(edges/1000) subdomains; Poisson arrivals",
                   "requests": len(reqs), "rate_per_s": args.serve_rate, "tol": args.tol,
                   "restart": args.restart, "budget_bytes": srv.adm.budget},
    }
    print(json.dumps(line), flush=True)
    srv.close()
    ctx.close()


def invert_main(args):
    """The outer inversion loop (L-BFGS on the normalised, regularised misfit
    over a vertex permittivity) on the workload: synthetic data from the
    per-tetrahedron phantom with a 1 cm inclusion, S_empty from the
    homogeneous gel, start from the gel; prints one JSON line."""
    import torch

    import mw_inputs as mi
    from paper_1607_02573_amd import inversion, solver
    w = make_workload(args.workload)
    tx = w.tx if args.nrhs == 0 else w.tx[: args.nrhs]
    rx = w.rx
    eps_true = w.extra.get("eps_true") if w.extra else None
    if eps_true is None:
        eps_true = mi.fields.add_inclusion(w.mesh, w.eps)
    total = torch.cuda.mem_get_info()[1]
    ctx = solver.Context(0, budget_bytes=int(total - (24 << 30)))
    P = solver.problem_from_workload(ctx, w)

    def s_of(eps_t):
        P.update_eps(torch.from_numpy(np.ascontiguousarray(eps_t)).cuda())
        P.factor(w.part, w.n_sub, 1, "c64")
        U, _ = P.solve(P.rhs_ports(tx), tol=1e-10, restart=args.restart, maxit=args.maxit)
        S = P.s_matrix(U, rx).cpu().numpy()
        del U
        return S

    log(f"[invert] {w.name}: data at the phantom with inclusion, S_empty at the homogeneous gel")
    gel = 44 - 20j    # the matching medium that fills the empty chamber
    S_mes = s_of(eps_true)
    S_empty = s_of(np.full(w.mesh.nt, gel))
    inv = inversion.Inversion(P, w.mesh.xyz, w.mesh.tet, w.part, w.n_sub, tx, rx, S_mes, S_empty, args.alpha,
                              precision="c64", tol=args.tol, restart=args.restart, block=args.block,
                              recycle=args.recycle, p1=args.p1)
    e0 = np.full(w.mesh.xyz.shape[0], gel)
    log(f"[invert] L-BFGS x{args.invert} from the gel")
    torch.cuda.synchronize()
    h = inv.run(e0, iters=args.invert, step0=args.step0)
    line = {
        "metric": "inversion: seconds per L-BFGS evaluation (factor + forward + adjoint solves), mixed precision",
        "value": h.seconds / h.evaluations, "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "iterations": len(h.J) - 1, "evaluations": h.evaluations, "J": h.J, "seconds": h.seconds,
        "rhs_solves_per_s": h.solve_columns / h.seconds,
        "gmres_iters_per_evaluation": h.iters, "recycle": inv.recycle,
        "dtype": MIXED_DTYPE, "data": "synthetic",
        "config": {"workload": f"{w.name}: {P.n} unknowns, {len(tx)} ports, {w.n_sub} subdomains; vertex "
                               f"permittivity ({w.mesh.xyz.shape[0]} vertices, "
                               f"{'exact P1 mass term' if args.p1 else 'tetrahedron means'}), defJ2 misfit, "
                               f"alpha {args.alpha:g}",
                   "tol": args.tol, "restart": args.restart, "gmres": "block" if args.block else "pseudo-block"},
    }
    print(json.dumps(line), flush=True)
    inv.close()
    P.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chamber10")
    ap.add_argument("--nrhs", type=int, default=0, help="0 = all ports of the workload")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--maxit", type=int, default=600)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--block", type=int, default=0, choices=(0, 32),
                    help="0: pseudo-block GMRES; 32: block GMRES with blocks of 32 right-hand sides")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--basis", choices=("auto", "fp64", "fp32-lean"), default="auto",
                    help="Krylov basis of the mixed-precision solves: complex FP32 with the preconditioned "
                         "candidates kept (auto), complex FP32 without them (fp32-lean) or complex FP64")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain elementwise copy (torch.neg) of this many MiB, the known-size "
                         "kernel that calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--serve", action="store_true",
                    help="serve the seeded request stream over the 4-mesh x 2-permittivity chamber menu and print "
                         "its latency line instead of the batch benchmark")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-short", type=int, default=40,
                    help="requests of the short serving leg of the default line (0: none)")
    ap.add_argument("--two-level-steps", type=int, default=2,
                    help="timed mixed steps with the two-level preconditioner beside the one-level line (0: none)")
    ap.add_argument("--cpu-cols", type=int, default=2,
                    help="port columns the oracle baseline solves (the rest scaled by column count)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--invert", type=int, default=0,
                    help="run this many L-BFGS iterations of the outer inversion loop on the workload and print "
                         "its line instead of the batch benchmark")
    ap.add_argument("--alpha", type=float, default=1e-4, help="Tikhonov weight of the inversion loop")
    ap.add_argument("--step0", type=float, default=0.5, help="largest vertex change of the first L-BFGS step")
    ap.add_argument("--recycle", choices=("none", "warm", "project"), default="warm",
                    help="inversion loop: start every solve from zero, from its own previous field, or from the "
                         "least-squares combination of all previous fields")
    ap.add_argument("--p1", action="store_true",
                    help="inversion loop: the permittivity linear on every tetrahedron, integrated exactly "
                         "(instead of the tetrahedron mean of the vertex values)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this library solves all subdomains "
              "of a problem on a single MI355X and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    # the oracle baseline forks a process pool: it runs before the GPU is touched
    w = None
    cpu = fp_oracle = B_oracle = None
    if not (args.serve or args.invert):
        log(f"[bench] generating workload {args.workload}")
        w = make_workload(args.workload)
        tx = w.tx if w.dipoles is None else np.arange(w.nrhs)
        if args.nrhs and w.dipoles is None:
            tx = w.tx[: args.nrhs]
        tol = args.tol if args.workload != "cube8" else w.tol
        if not args.no_cpu:
            log(f"[bench] cpu_baseline: the oracle on {host_cores()} host cores")
            cpu, fp_oracle, B_oracle = cpu_baseline(w, tx, tol, args.restart, args.cpu_cols)
            log(f"[bench] cpu_baseline: {cpu['value']:.4f} RHS/s ({cpu['sample']})")

    import torch

    from paper_1607_02573_amd import binding, solver
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    binding.lib()   # fails loudly if the HIP library is not built
    if args.serve:
        serve_main(args)
        return
    if args.invert:
        invert_main(args)
        return
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read, {args.copy_probe_mib} MiB written")
        del src, dst

    rx = w.rx if w.rx is not None else np.zeros(0, dtype=np.int32)
    nrhs = len(tx) if w.dipoles is None else w.nrhs

    total = torch.cuda.mem_get_info()[1]
    ctx = solver.Context(0, budget_bytes=int(total - (24 << 30)))
    t0 = time.perf_counter()
    P = solver.problem_from_workload(ctx, w)
    torch.cuda.synchronize()
    t_topo = time.perf_counter() - t0
    eps_dev = torch.from_numpy(np.ascontiguousarray(w.eps)).cuda()
    log(f"[bench] n={P.n} nnz={P.nnz} topology+assembly {t_topo:.2f} s; first factorisation (decomposition)")
    P.set_krylov_basis(args.basis)
    P.factor(w.part, w.n_sub, 1, "c64")
    inf = P.info()
    log(f"[bench] decomposition {inf.t_decompose:.2f} s, n_sub={inf.n_sub}, sum n_i={inf.sum_ni}, max n_i={inf.max_ni}")

    # ---------------- mixed precision (the measured configuration)
    if args.warmup:
        log(f"[bench] warmup x{args.warmup}")
        run_steps(P, w, eps_dev, "c64", args.warmup, tol, args.restart, args.maxit, tx, rx, args.block)
    binding.timer_enable(True)
    binding.timer_reset()
    log(f"[bench] timed mixed steps x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, (Xm, Sm) = run_steps(P, w, eps_dev, "c64", args.steps, tol, args.restart, args.maxit, tx, rx,
                             args.block)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    fam = binding.timer_read()
    binding.timer_enable(False)
    ok = int(sum((s["relres"] <= tol).sum() for s in st))
    value = ok / T
    solve_rate = sum(len(s["relres"]) for s in st) / sum(s["t_solve"] for s in st)
    it_mixed = np.concatenate([s["iters"] for s in st])
    log(f"[bench] mixed: {T / args.steps:.2f} s/step, {value:.2f} RHS/s e2e, iters {it_mixed.min()}-{it_mixed.max()}")

    # dominant kernel family and its roofline
    famt = {k: v for k, v in fam.items() if v["launches"] > 0}
    dom = max(famt, key=lambda k: famt[k]["ms"])
    d = famt[dom]
    if dom in MFMA_FAMILIES:
        ach = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK["fp32_TFLOPs"], "unit": "TFLOP/s"}
    else:
        ach = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBs"], "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    roof["launches"] = d["launches"]
    roof["avg_launch_us"] = d["ms"] * 1e3 / d["launches"]
    kernel_table, solve_roof = family_table(famt, PEAK["fp32_TFLOPs"], T)

    err_mixed = err_fp64 = None
    if fp_oracle is not None:
        err_mixed = oracle_errors(w, fp_oracle, B_oracle, Xm, tx, "mixed")

    # ---------------- two-level preconditioner (coarse space), same mixed step
    two_level = None
    if args.two_level_steps > 0 and args.block == 0:
        del Xm, Sm
        Xm = Sm = None
        torch.cuda.empty_cache()
        P.set_coarse_space("const")
        log(f"[bench] two-level: warm-up step, then {args.two_level_steps} timed mixed steps")
        run_steps(P, w, eps_dev, "c64", 1, tol, args.restart, args.maxit, tx, rx)
        binding.timer_enable(True)
        binding.timer_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2, (X2, S2) = run_steps(P, w, eps_dev, "c64", args.two_level_steps, tol, args.restart, args.maxit, tx, rx)
        torch.cuda.synchronize()
        T2 = time.perf_counter() - t0
        fam2 = binding.timer_read()
        binding.timer_enable(False)
        ok2 = int(sum((s["relres"] <= tol).sum() for s in st2))
        it2 = np.concatenate([s["iters"] for s in st2])
        two_level = {"value": ok2 / T2, "unit": "RHS/s", "ms_per_step": 1e3 * T2 / args.two_level_steps,
                     "steps": args.two_level_steps, "iters_mean": float(it2.mean()), "iters_max": int(it2.max()),
                     "converged": ok2, "coarse_size": int(P.info().coarse_size),
                     "solve_rhs_per_s": sum(len(s["relres"]) for s in st2) / sum(s["t_solve"] for s in st2),
                     "setup_s": st2[-1]["t_setup"], "chunks": st2[-1]["chunks"],
                     "coarse_ms_per_step": fam2["coarse"]["ms"] / args.two_level_steps,
                     "one_level": {"value": value, "iters_mean": float(it_mixed.mean()),
                                   "ms_per_step": 1e3 * T / args.steps},
                     "coarse_space": "three partition-of-unity-weighted constant fields per subdomain, "
                                     "deflated correction M^-1 (v - A q) + q, q = Z E^-1 Z^T v",
                     "error_vs_oracle": oracle_errors(w, fp_oracle, B_oracle, X2, tx, "two-level")
                     if fp_oracle is not None else None}
        log(f"[bench] two-level: {T2 / args.two_level_steps:.2f} s/step, {two_level['value']:.2f} RHS/s, iters "
            f"{it2.min()}-{it2.max()} (one-level {it_mixed.min()}-{it_mixed.max()})")
        del X2, S2
        P.set_coarse_space("none")
        P.factor(w.part, w.n_sub, 1, "c64")

    # ---------------- FP64 path, same workload
    fp64 = None
    if Xm is None and args.fp64_steps > 0 and args.workload != "cube8":
        # the mixed fields for the comparison below: the last mixed step again
        _, (Xm, Sm) = run_steps(P, w, eps_dev, "c64", 1, tol, args.restart, args.maxit, tx, rx, args.block)
    if args.fp64_steps > 0 and args.workload != "cube8":
        Xm_host = Xm[:, : min(8, Xm.shape[1])].cpu()
        Sm_host = Sm.cpu() if Sm is not None else None
        del Xm, Sm
        torch.cuda.empty_cache()
        log("[bench] FP64 warm-up step (allocates the complex-FP64 factors and the solve workspace)")
        run_steps(P, w, eps_dev, "c128", 1, tol, args.restart, args.maxit, tx, rx, args.block)
        torch.cuda.synchronize()
        log(f"[bench] FP64 steps x{args.fp64_steps}")
        binding.timer_enable(True)
        binding.timer_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st64, (X64, S64) = run_steps(P, w, eps_dev, "c128", args.fp64_steps, tol, args.restart, args.maxit, tx, rx,
                                     args.block)
        torch.cuda.synchronize()
        T64 = time.perf_counter() - t0
        fam64 = binding.timer_read()
        binding.timer_enable(False)
        ok64 = int(sum((s["relres"] <= tol).sum() for s in st64))
        it64 = np.concatenate([s["iters"] for s in st64])
        if fp_oracle is not None:
            err_fp64 = oracle_errors(w, fp_oracle, B_oracle, X64, tx, "FP64")
        x64 = X64[:, : Xm_host.shape[1]].cpu()
        dx = (torch.linalg.norm(Xm_host - x64, dim=0) / torch.linalg.norm(x64, dim=0)).max().item()
        dS = ((Sm_host - S64.cpu()).abs().max() / S64.cpu().abs().max()).item() if Sm_host is not None else None
        fp64 = {"value": ok64 / T64, "ms_per_step": 1e3 * T64 / args.fp64_steps, "iters_mean": float(it64.mean()),
                "chunks": st64[-1]["chunks"], "solve_rhs_per_s": sum(len(s["relres"]) for s in st64)
                / sum(s["t_solve"] for s in st64), "setup_s": st64[-1]["t_setup"],
                "mixed_vs_fp64_field_relL2_max": dx, "mixed_vs_fp64_S_rel_max": dS, "error_vs_oracle": err_fp64,
                "kernels": family_table({k: v for k, v in fam64.items() if v["launches"] > 0},
                                        PEAK["fp64_TFLOPs"], T64)[0]}
        log(f"[bench] FP64: {T64 / args.fp64_steps:.2f} s/step, {fp64['value']:.2f} RHS/s; mixed-vs-fp64 field {dx:.2e}")
        del X64, S64
    else:
        del Xm, Sm

    del fp_oracle, B_oracle, eps_dev
    P.close()
    ctx.close()
    torch.cuda.empty_cache()
    latency = None
    if args.serve_short > 0:
        log(f"[bench] serving leg: {args.serve_short} requests at {args.serve_rate}/s on the 0.3125 and 0.5 GHz "
            "chambers")
        summ = serving_leg(args, (0.3125e9, 0.5e9), args.serve_short, args.serve_rate)
        log(f"[bench] serving: p50 {summ['p50_s']:.2f} s, p99 {summ['p99_s']:.2f} s, {summ['rhs_per_s']:.1f} "
            f"columns/s, failed {summ['failed']}")
        latency = {"p50_s": summ["p50_s"], "p99_s": summ["p99_s"], "mean_s": summ["mean_s"],
                   "by_kind": summ["by_kind"], "requests": summ["requests"], "failed": summ["failed"],
                   "rhs_columns": summ["rhs_columns"], "rhs_per_s": summ["rhs_per_s"],
                   "makespan_s": summ["makespan_s"], "max_relres": summ["max_relres"],
                   "evictions": summ["evictions"], "factorisations": summ["factorisations"],
                   "config": {"workload": "continuous-batching service, chamber menu " + "; ".join(summ["menu"]) +
                              f"; 2 permittivity versions each; seeded Poisson arrivals at {args.serve_rate}/s, "
                              f"{args.serve_short} requests, 75 % solves (1-160 columns) / 25 % gradients (1-32)",
                              "precision": "c64 factors + f64 GMRES", "tol": args.tol,
                              "budget_bytes": summ["budget_bytes"]}}
    out = {
        "metric": "RHS solves/s at rel-res 1e-8, mixed vs FP64 ORAS-GMRES; p50/p99 latency",
        "value": value,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": MIXED_DTYPE if args.basis == "auto" else MIXED_DTYPE.replace("c64 Krylov", "f64 Krylov"),
        "data": "synthetic",
        "config": {"workload": f"{w.name}: n={P.n} unknowns, {w.mesh.nt} tets, {nrhs} port RHS, "
                               f"{w.n_sub} subdomains overlap 1, "
                               f"{'block ' if args.block else ''}GMRES({args.restart}), tol {tol:g}, mixed precision",
                   "nrhs": nrhs, "n_sub": w.n_sub, "n": P.n, "restart": args.restart, "tol": tol,
                   "gmres": f"block GMRES, blocks of {args.block}" if args.block else "pseudo-block GMRES"},
        "solve_rhs_per_s": solve_rate,
        "setup_s": st[-1]["t_setup"],
        "iters_mean": float(it_mixed.mean()),
        "iters_max": int(it_mixed.max()),
        "converged": ok,
        "error_vs_oracle": err_mixed,
        "two_level": two_level,
        "latency": latency,
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "roofline": roof,
        "kernels": kernel_table,
        "whole_run_roofline": solve_roof,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

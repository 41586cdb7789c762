#!/usr/bin/env python3
"""Iteration counts of one-level and two-level ORAS-GMRES with the oracle:
the study behind the choice of coarse space for the two-level
preconditioner (Section 7, first avenue; Section 6.1, Table tabscaling, for
the growth of the one-level count with the number of subdomains).

    python tests/coarse_study.py [--freq 0.5e9] [--n-sub 214] [--ports 0,8,16,24]

builds the seeded chamber, decomposes it (overlap 1), and runs the oracle's
pseudo-block GMRES(30) to 1e-8 on the chosen port sources with
  * the one-level ORAS M^-1,
  * the deflated two-level ORAS with the three constant fields per subdomain,
  * the same with plane waves of the background medium added (15 fields),
printing the coarse size and the mean / max iteration count of each.
Only oracle/ and the seeded input generators are used.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import mw_inputs as mi  # noqa: E402
from oracle import coarse, dd, fem, gmres  # noqa: E402


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--freq", type=float, default=0.5e9)
    ap.add_argument("--n-sub", type=int, default=214)
    ap.add_argument("--ports", default="0,8,16,24")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--eps-gel", type=complex, default=44 - 20j, help="background (gel) permittivity")
    a = ap.parse_args(argv)

    w = mi.configs.chamber(a.freq, rings=(0.14,), n_sub=a.n_sub, eps_gel=a.eps_gel)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    tx = np.array([int(p) for p in a.ports.split(",")])
    B = fem.rhs_ports(fp, w.ports, tx)
    t0 = time.perf_counter()
    subs = dd.decompose(fp, w.part, 1)
    print(f"chamber {a.freq / 1e9:g} GHz: n = {fp.n}, {a.n_sub} subdomains, ports {tx.tolist()} "
          f"(decomposition and local factors {time.perf_counter() - t0:.1f} s)", flush=True)
    k = w.k0 * np.sqrt(a.eps_gel.real)

    def one_level(V):
        return dd.oras_apply(subs, V)

    cases = [("one-level", None, one_level)]
    for kind in ("const", "wave"):
        M2 = coarse.TwoLevel(fp, subs, kind, k)
        cases.append((f"two-level {kind}", M2.size, M2))
    for name, size, prec in cases:
        t0 = time.perf_counter()
        _, it, rr = gmres.gmres(fp.A, B, prec, tol=a.tol, restart=30)
        extra = f", coarse size {size}" if size else ""
        print(f"{name}{extra}: iterations mean {it.mean():.1f} max {it.max()}, "
              f"largest final relative residual {rr.max():.1e} ({time.perf_counter() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    main()

"""Writes the stored optima of tests/golden/ with the FP64 oracle alone.

Every value here comes from ``oracle`` run on inputs drawn by ``synth``; the
GPU library is not involved.

optima_256.json
    F_eps* of the 256^2 tree-group workload (8 ellipses, 20% variable-density
    mask, sigma 0.01, 4-level Haar, quadtree-pair groups, lambda 0.035,
    eps 1e-10) for seeds 0-15 and for the fresh seeds 20000-20015 (disjoint
    from the seeds the warm-start network was trained and validated on).
    F_eps is strictly convex (Section 3.3 with eps > 0), so its minimiser and
    F_eps* are unique; the oracle approaches it by 300 outer iterations of
    Algorithm 2 with 20 PCG iterations each (eq. 15 with the
    preconditioner of eq. 17), and records its last relative decrease
    (F_eps^{k-1} - F_eps^k) / F_eps^k as the certificate of convergence.

tv_lex_32.json
    F_eps* of a 32^2 TV problem (isotropic, periodic differences, 15% radial
    mask, lambda 0.01) reached with the preconditioner in the paper's own
    lexicographic order (the triangular factors of eqs. 41-43 applied by
    forward and backward Gauss-Seidel sweeps), Algorithm 3 run until the
    relative decrease is at most 1e-13 (at most 2000 outer iterations of 20
    PCG iterations).

Usage: python tests/golden/make_golden.py [optima|tv|all] [--jobs J]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SEEDS_256 = list(range(16)) + list(range(20000, 20016))
OUTER_256, PCG_256 = 300, 20


def optimum_256(seed: int) -> dict:
    import synth
    from oracle.firls import Operators, firls
    ops = Operators.from_problem(synth.cfg1(seed))
    t0 = time.perf_counter()
    rep = firls(ops, OUTER_256, PCG_256, tau=0.0)
    h = rep.history
    return {"seed": seed, "F_eps": rep.F_eps, "F": rep.F, "outer_iters": rep.outer_iters,
            "last_rel_decrease": (h[-2] - h[-1]) / h[-1], "seconds": round(time.perf_counter() - t0, 1)}


def tv_problem_32():
    import synth
    return synth.make_problem(32, 7, psi="tv", levels=0, groups="tv_iso", lam=0.01, sigma=0.005,
                              n_ellipses=6, mask_kind="radial", frac=0.15, ramp=True)


def tv_lex_32() -> dict:
    from oracle.firls import Operators, firls
    ops = Operators.from_problem(tv_problem_32())
    t0 = time.perf_counter()
    rep = firls(ops, 2000, 20, tau=1e-13, precond="sgs_lex")
    h = rep.history
    return {"n": 32, "seed": 7, "F_eps": rep.F_eps, "F": rep.F, "outer_iters": rep.outer_iters,
            "converged": rep.converged, "last_rel_decrease": (h[-2] - h[-1]) / h[-1],
            "precond": "sgs_lex", "pcg_iters": 20, "tau": 1e-13, "seconds": round(time.perf_counter() - t0, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="?", default="all", choices=("optima", "tv", "all"))
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    if a.what in ("tv", "all"):
        rec = tv_lex_32()
        with open(os.path.join(HERE, "tv_lex_32.json"), "w") as f:
            json.dump({"source": "tests/golden/make_golden.py (oracle only)", "workload":
                       "32x32, 6 ellipses + ramp, 15% radial mask, sigma 0.005, periodic isotropic TV, "
                       "lambda 0.01, eps 1e-10", **rec}, f, indent=1)
        print("tv", rec, flush=True)
    if a.what in ("optima", "all"):
        with ProcessPoolExecutor(a.jobs) as ex:
            recs = list(ex.map(optimum_256, SEEDS_256))
        with open(os.path.join(HERE, "optima_256.json"), "w") as f:
            json.dump({"source": "tests/golden/make_golden.py (oracle only)",
                       "workload": "256x256 tree-group FIRLS_OG: 8 ellipses, 20% VD mask, sigma 0.01, 4-level "
                                   "Haar, quadtree-pair groups, lambda 0.035, eps 1e-10",
                       "method": f"oracle FIRLS, {OUTER_256} outer x {PCG_256} PCG iterations, tau 0",
                       "optima": recs}, f, indent=1)
        print("optima", [(r["seed"], r["F_eps"], r["last_rel_decrease"]) for r in recs], flush=True)


if __name__ == "__main__":
    main()

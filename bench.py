"""Benchmark: batched FIRLS_OG solves at 256^2 on one MI355X.

One step = one batched solve of B slices of the tree-group CS-MRI workload
(256 x 256 ellipse phantoms, 20% variable-density k-space mask, sigma 0.01,
4-level Haar, each coefficient grouped with its quadtree parent, lambda
0.035, eps 1e-10, FP32 vectors with FP64 scalars, 4 PCG iterations per
outer iteration) through the whole hot path: the learned warm start (network
on A^H b, measured samples put back, A^H b kept where it has the lower
objective), then FIRLS on every slice until its relative objective decrease
falls below tau (calibrated so that the final objective is within 1e-4 of
the optimum) or 50 outer iterations.  Inputs are generated and uploaded
before the timed region; the sub-batch size is autotuned before it.

Prints one JSON line: solves/s, the roofline of the dominant kernel
(HIP-event durations of every launch, measured on one more step of the same
call right after the timed steps), the achieved
algorithmic HBM rate of the whole path, the gap to the optimum of every
slice, the same solves from the zero-filled start (the ablation), and the
FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at 256² CS-MRI to 1e-4 rel. objective, learned vs plain; HBM GB/s"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per pixel per launch of each PCG kernel class for a
# Haar slice in FP32 (c64 = 8 B, r32 = 4 B, u8 mask = 1 B), the minimum each
# kernel must stream:
#   rowfwd : read r, d, p; write p, t         (p not read at k = 0)
#   col    : read t, mask bits; write t
#   rowinv : read t, p, d; write q            (the last iteration: read p, d)
#   update : the fused step, read x, p, q, r, d; write x, r, p, t; or the
#            paired pass, read t, p, d, x, r; write x, r, p, t
def bytes_per_px(cls: str, K: int, fused: bool = True, last_rowinv_only: bool = False) -> float:
    """Algorithmic HBM bytes per pixel of one launch of a kernel class.
    ``fused``: the paper's preconditioner, whose residual passes also carry
    the last PCG step's x update and the first one's z0, p0 and row FFT.
    The paired pass (the row inverse of iteration k - 1 in the launch of
    step k: "update", read t, p, x, r, d; write x, r, p, t, also 68 B)
    leaves no row-inverse launch for K >= 2: the last iteration's sum
    lambda sum d |Phi p|^2 rides in its own launch as well, except in
    launches across shapes, which keep that iteration's row inverse
    (``last_rowinv_only``: read p and d, 12 B)."""
    if not fused and cls in ("r0_rowfwd", "r0_rowinv"):
        return {"r0_rowfwd": 20.0, "r0_rowinv": 28.0}[cls]
    if fused and cls == "rowinv":
        # K launches per solve, the last reading only p and d (12 B)
        return 12.0 if last_rowinv_only else 28.0 - 16.0 / K
    return {
        "rowfwd": 28.0,        # first iteration: read r, d; write p, t
        "col": 16.125,         # read t, mask bits; write t
        "rowinv": 28.0,        # read t, p, d; write q
        "update": 68.0,        # read x, p, q, r, d; write x, r, p, t
        "last_x": 24.0,        # read x, p; write x
        "psi_sq": 12.0,        # read x; write |Phi x|^2 (TV only)
        "group_w": 10.0,       # read |z|^2 of members (~2 per group), write W
        "group_d": 12.0,       # read W of the groups of each coefficient (~2), write d
        "r0_rowfwd": 36.0,     # read x, p; write x, t, d (x += alpha p of the last PCG step folded in;
                               # the first evaluation of a slice skips p and the x write: 20)
        "r0_col": 25.0,        # read t, mask, b; write t
        "r0_rowinv": 44.0,     # read t, x, d; write r, p0 and t (z0, p0 and its row FFT folded in)
        "r0_update": 12.0,     # read r, d (TV only)
        "adjoint": 33.0,       # read b, mask; write t; read t; write x
    }.get(cls, 0.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--slices", type=int, default=None,
                    help="slices per step (default: 500 for mri, 32 for tv512, 1024 for fp64_64, 64 for uneven)")
    ap.add_argument("--seed0", type=int, default=None,
                    help="first seed of the batch (mri default: the 500 fresh evaluation seeds 20000-20499 of "
                         "the learned-start workload, disjoint from the network's training seeds; else 0)")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--pcg", type=int, default=None, help="PCG iterations per outer iteration (workload default)")
    ap.add_argument("--max-outer", type=int, default=None)
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--prec", choices=("fp32", "fp64"), default=None,
                    help="working precision (tv512: fp32 by default, with the FP64 run of the same slices "
                         "reported beside it)")
    ap.add_argument("--no-fp64-ref", action="store_true", help="tv512: skip the FP64 comparison run")
    ap.add_argument("--ref-outer", type=int, default=300,
                    help="outer iterations of the reference solve that estimates the optimum")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gap", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1411_5057_amd", "weights", "warmstart_256.f32"),
                    help="warm-start network parameters (float32, ABI order); skipped if missing")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--precond", choices=("paper", "jacobi", "none"), default="paper",
                    help="inner preconditioner: the paper's (eq. 17), Jacobi (diag S) or none (plain CG)")
    ap.add_argument("--no-tune", action="store_true", help="skip the sub-batch autotuner")
    ap.add_argument("--sub-batch", type=int, default=-1,
                    help="slices per sub-batch instead of the autotuner's choice (0: all at once); "
                         "profiler runs pin the unprofiled choice, since the profiler skews the trials")
    ap.add_argument("--launch", choices=("graphs", "direct"), default=None,
                    help="launch mode instead of the autotuner's choice (with --sub-batch)")
    ap.add_argument("--schedule", choices=("per_shape", "across", "largest_first"), default=None,
                    help="launches of a mixed-shape batch (with --sub-batch; default: the autotuner's choice)")
    ap.add_argument("--no-pair", action="store_true",
                    help="run the PCG row-inverse pass and the step as two launches (A/B of the paired pass)")
    ap.add_argument("--workload", choices=("mri", "dense", "tv512", "fp64_64", "uneven"), default="mri",
                    help="mri: the 256^2 tree-group CS-MRI benchmark (default); tv512: FIRLS_TV at 512^2; "
                         "fp64_64: plain l1 FIRLS in FP64 at 64^2; uneven: 64 slices of mixed sizes and "
                         "regularisers in one call; dense: 64^2 images measured by one shared dense random "
                         "projection (30%% of N rows), the MFMA path")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    a = ap.parse_args()
    d = WORKLOAD_DEFAULTS[a.workload]
    for k in ("slices", "pcg", "max_outer", "tau", "prec", "seed0"):
        if getattr(a, k) is None:
            setattr(a, k, d[k])
    return a


# Per workload: slices per step, PCG iterations per outer iteration, outer
# cap, stop tolerance tau (relative F_eps decrease) and precision.  tau is
# calibrated so that every slice ends within 1e-4 of its optimum.
WORKLOAD_DEFAULTS = {
    "mri": dict(seed0=20000, slices=500, pcg=4, max_outer=50, tau=8e-6, prec="fp32"),
    "dense": dict(seed0=0, slices=256, pcg=10, max_outer=50, tau=1e-5, prec="fp32"),
    # TV: the paper's run length for FIRLS_TV (29 outer iterations, Section
    # 5.5.2); its MM iteration approaches the optimum slowly on
    # piecewise-constant images with eps = 1e-10, so the gap is reported
    "tv512": dict(seed0=0, slices=32, pcg=10, max_outer=30, tau=0.0, prec="fp32"),
    "fp64_64": dict(seed0=0, slices=1024, pcg=20, max_outer=30, tau=0.0, prec="fp64"),
    "uneven": dict(seed0=0, slices=64, pcg=4, max_outer=100, tau=8e-6, prec="fp32"),
}


def make_inputs(seeds, n, torch):
    import synth
    bs, ms, lams = [], [], []
    for s in seeds:
        p = synth.cfg1(s, n=n)
        bs.append(p.b)
        ms.append(p.mask)
        lams.append(p.lam)
    b = torch.from_numpy(np.stack(bs)).to(torch.complex64).cuda().contiguous()
    m = torch.from_numpy(np.stack(ms)).cuda().contiguous()
    return p, b, m, lams


def oracle_optima():
    """F_eps* per seed written by tests/golden/make_golden.py (FP64 oracle,
    300 outer x 20 PCG iterations), or {} if absent."""
    path = os.path.join(ROOT, "tests", "golden", "optima_256.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {int(r["seed"]): float(r["F_eps"]) for r in json.load(f)["optima"]}


def _oracle_share(job):
    """One worker of the CPU baseline: the FP64 oracle, untouched, on its
    share of the sampled slices, in a fresh interpreter (numpy and the
    oracle only, one thread).  Returns per slice its solving time and the
    errors of the GPU's result for it against the oracle's."""
    n, tau, max_outer, K, share = job
    import synth
    from oracle.firls import Operators, firls
    out = []
    for seed, x, fe_gpu, outer_gpu in share:
        ops = Operators.from_problem(synth.cfg1(seed, n=n))
        t0 = time.perf_counter()
        rep = firls(ops, max_outer, K, tau=tau)
        dt = time.perf_counter() - t0
        xd = x.astype(np.complex128)
        fe = ops.objective(xd)[0]
        out.append({"seed": seed, "seconds": dt, "pcg_oracle": rep.pcg_iters,
                    "outer_gpu": int(outer_gpu), "outer_oracle": rep.outer_iters,
                    "F_eps_rel_diff": abs(fe - rep.F_eps) / rep.F_eps,
                    "F_eps_reported_vs_fp64": abs(fe_gpu - fe) / fe,
                    "x_rel_l2": float(np.linalg.norm(xd - rep.x) / np.linalg.norm(rep.x)),
                    "x_max_rel": float(np.max(np.abs(xd - rep.x)) / np.max(np.abs(rep.x)))})
    return out


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, tau, max_outer, K, seeds, gpu_x, gpu_fe, per_worker=5, workers=None):
    """The FP64 oracle, untouched, on the first slices of the same workload
    (the first seeds of the timed batch) in a pool of worker processes, one
    per host core (at most 16, the host share of one GPU), each solving
    ``per_worker`` slices one after another.  Pool throughput = slices over
    the slowest worker's solving time (the workers run at once); the
    single-core time per solve is the mean.  Each oracle result is also the
    reference of the GPU's result for the same slice (plain start, same K,
    tau and cap): the per-result error against the FP64 oracle."""
    import multiprocessing as mp
    P = workers or max(1, min(os.cpu_count() or 1, 16))
    ns = min(len(seeds), P * per_worker)
    P = min(P, ns)
    shares = [[] for _ in range(P)]
    for i in range(ns):
        shares[i % P].append((seeds[i], gpu_x[i], gpu_fe[i][0], gpu_fe[i][1]))
    # the workers start as fresh interpreters (nothing of this process's
    # GPU state), single-threaded
    keep = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in keep:
        os.environ[v] = "1"
    jobs = [(n, tau, max_outer, K, sh) for sh in shares]
    try:
        with mp.get_context("spawn").Pool(P) as pool:
            # bounded: a pool whose workers cannot start would wait forever
            parts = pool.map_async(_oracle_share, jobs).get(timeout=600)
    except Exception as e:   # no pool on this host: the same slices in this process
        print(f"cpu baseline: worker pool unavailable ({e!r}); one process", file=sys.stderr)
        P = 1
        parts = [_oracle_share((n, tau, max_outer, K, [it for sh in shares for it in sh]))]
    finally:
        for v, old in keep.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    errs = sorted((e for part in parts for e in part), key=lambda e: e["seed"])
    wall = max(sum(e["seconds"] for e in part) for part in parts)
    solve_s = float(np.mean([e["seconds"] for e in errs]))
    outer = float(np.mean([e["outer_oracle"] for e in errs]))
    pcg_s = sum(e["pcg_oracle"] for e in errs) / wall
    same = [e for e in errs if e["outer_gpu"] == e["outer_oracle"]]
    per_result = {
        "slices": len(errs), "same_outer_count": len(same),
        "F_eps_rel_diff_max": max(e["F_eps_rel_diff"] for e in errs),
        "F_eps_rel_diff_max_same_count": max([e["F_eps_rel_diff"] for e in same], default=None),
        "x_rel_l2_max_same_count": max([e["x_rel_l2"] for e in same], default=None),
        "x_max_rel_max_same_count": max([e["x_max_rel"] for e in same], default=None),
        "reported_F_eps_vs_fp64_max": max(e["F_eps_reported_vs_fp64"] for e in errs),
        "note": "GPU plain-start results against the FP64 oracle run from the same start with the same K, tau and "
                "cap; x compared where both took the same number of outer iterations",
        "per_slice": [{k: v for k, v in e.items() if k not in ("seconds", "pcg_oracle")} for e in errs]}
    return {"value": len(errs) / wall, "unit": "solves/s", "cores": P, "kind": "oracle",
            "single_core_s_per_solve": solve_s, "pcg_iters_per_s": pcg_s, "outer_iters_mean": outer,
            "host": f"{host_cpu_model()}, nproc {os.cpu_count()}",
            "sample": f"{len(errs)} slices (seeds {seeds[0]}-{seeds[len(errs) - 1]}) of the same workload, "
                      f"{outer:.1f} outer x {K} PCG on average, numpy FP64, {P} single-threaded worker "
                      f"processes of {per_worker} slices at most each; slowest worker {wall:.1f} s of solving"}, \
        per_result


def timed(solver, run, steps, warmup, profile, torch):
    """Warm up, then time ``steps`` calls of run() (HIP events per launch
    when ``profile``).  Returns (seconds, last reports, profile dict).
    Python's cyclic garbage collector is paused over the timed calls, as
    timeit does: a full collection of the input generator's objects takes
    tens of milliseconds and would otherwise land inside a step now and
    then."""
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    if profile:
        solver.profile(True)
    gc.collect()
    gc_on = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        for _ in range(steps):
            out = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        if gc_on:
            gc.enable()
    prof = solver.profile_read() if profile else {}
    solver.profile(False)
    return dt, out, prof


def roofline_of(prof, n, K, dt, slices, fused=True):
    """Dominant PCG kernel by measured time: algorithmic bytes per launch
    over its average HIP-event duration; plus the whole path's rate.
    ``slices`` solves of the instrumented step each start with one residual
    pass that has no x update to fold in."""
    npx = n * n
    lro = last_rowinv_only(prof)
    tot_bytes = sum(bytes_per_px(c, K, fused, lro) * v["slice_launches"] * npx for c, v in prof.items())
    if prof.get("r0_rowfwd", {}).get("launches", 0) and not prof.get("last_x", {}).get("launches", 0):
        tot_bytes -= 16.0 * npx * slices
    pcg_cls = {c: v for c, v in prof.items() if c in ("rowfwd", "col", "rowinv", "update", "last_x")}
    dom = max(pcg_cls, key=lambda c: pcg_cls[c]["ms"])
    v = prof[dom]
    per_launch_bytes = bytes_per_px(dom, K, fused, lro) * npx * v["slice_launches"] / v["launches"]
    avg_s = v["ms"] / v["launches"] / 1e3
    ach = per_launch_bytes / avg_s / 1e9
    tr = traffic_record()
    traffic = None
    if tr is not None and tr.get("n") == n and dom in tr["traffic_bytes_per_px"]:
        traffic = tr["traffic_bytes_per_px"][dom] * npx * v["slice_launches"] / v["launches"]
    roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": per_launch_bytes}
    return roof, tot_bytes / dt / 1e9, {c: round(v["ms"], 3) for c, v in prof.items() if v["launches"]}


def traffic_record():
    """Measured HBM bytes per pixel of each PCG kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel
    sources (else None)."""
    path = os.path.join(ROOT, "profiles", "firls_pcg_256_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic_record:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None
    return rec if pcg_source_sha() == rec["kernel_source_sha"] else None


def pcg_source_sha():
    """Hash of the sources the FIRLS kernels and their launches are built
    from (every file under csrc/ except the network's cnn_* and the dense
    GEMM's)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1411_5057_amd", "csrc", "*"))):
        b = os.path.basename(f)
        if b.startswith("cnn") or b.startswith("gemm_dense"):
            continue
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def gap_stats(fe, fstar):
    g = (fe - fstar) / fstar
    return {"max": float(g.max()), "p99": float(np.quantile(g, 0.99)), "median": float(np.median(g)),
            "frac_le_1e-4": float(np.mean(g <= 1e-4))}


FP32_MFMA_PEAK_TFLOPS = 157.3


def run_dense(a, torch, F):
    """Random-projection compressive sensing (Section 5.2): B images of
    64 x 64, one dense Gaussian sensing matrix with M = 0.3 N rows shared by
    all of them, tree-group Haar.  The products with A are batched MFMA
    GEMMs; their roofline is MFMA-bound."""
    import synth
    n, B, K = 64, a.slices, a.pcg
    base = synth.make_dense_problem(n, 0, m_frac=0.3, psi="haar", levels=4, groups="quadtree", lam=0.03, sigma=0.01)
    Am = base.Amat
    M = Am.shape[0]
    rs = np.random.default_rng(1)
    bs = []
    for s in range(B):
        img = synth.phantom(n, 8, 5000 + s)
        bs.append(Am @ img.ravel() + 0.01 * (rs.standard_normal(M) + 1j * rs.standard_normal(M)))
    b = torch.from_numpy(np.stack(bs)).to(torch.complex64).cuda().contiguous()
    shape = F.Shape(n, "haar", 4, base.group_ptr, base.group_idx, A=Am)
    solver = F.Solver([shape], prec="fp32", max_slices=B, max_outer=a.max_outer, pcg_iters=K,
                      outer_tol=a.tau, eps=1e-10)
    x = torch.zeros((B, n, n), dtype=torch.complex64, device="cuda")
    batch = solver.prepare([dict(b=b[i], mask=None, x=x[i], lam=base.lam) for i in range(B)])
    run = lambda: (solver.solve_batched(batch), None)
    dt, (reps, _), _ = timed(solver, run, a.steps, a.warmup, False, torch)
    _, _, prof = timed(solver, run, 1, 0, True, torch)
    v = prof["col"]                       # the two GEMMs of every PCG iteration
    flops = 2.0 * 2.0 * M * n * n * v["slice_launches"] / v["launches"]   # 2 real columns per slice
    avg_s = v["ms"] / v["launches"] / 1e3
    ach = flops / avg_s / 1e12
    outer = np.array([r["outer_iters"] for r in reps])
    out = {"metric": "solves/s, 64^2 random-projection CS (M = 0.3 N), tree-group Haar", "value": B * a.steps / dt,
           "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded ellipse phantoms, one Gaussian N(0, 1/M) sensing matrix)",
           "config": {"workload": f"{B} slices of 64x64, dense A {M}x{n * n}, 4-level Haar, quadtree groups, "
                                  f"lambda 0.03, {K} PCG per outer, tau {a.tau:g} (max {a.max_outer})",
                      "n": n, "m": M, "slices": B, "pcg_iters": K},
           "outer_iters_mean": float(outer.mean()), "outer_iters_max": int(outer.max()),
           "converged_frac": float(np.mean([r["converged"] for r in reps])),
           "roofline": {"bound": "mfma", "kernel": "gemm (A p and A^T y)", "achieved": ach,
                        "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_MFMA_PEAK_TFLOPS,
                        "traffic": None, "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops},
           "kernel_ms": {c: round(u["ms"], 3) for c, u in prof.items() if u["launches"]}}
    if not a.no_gap:
        ref = F.Solver([shape], prec="fp32", max_slices=B, max_outer=a.ref_outer, pcg_iters=K, outer_tol=0.0,
                       eps=1e-10)
        xr = torch.zeros_like(x)
        rr = ref.solve_batched([dict(b=b[i], mask=None, x=xr[i], lam=base.lam) for i in range(B)])
        out["gap_to_optimum"] = gap_stats(np.array([r["F_eps"] for r in reps]), np.array([r["F_eps"] for r in rr]))
        ref.close()
    print(json.dumps(out))
    solver.close()


def last_rowinv_only(ps: dict) -> bool:
    """Whether a profile's row-inverse launches are only those of the last
    PCG iterations (one per solve: the paired pass across shapes) rather
    than one per iteration, from the slice counts of the two classes."""
    ri, co = ps.get("rowinv", {}).get("slice_launches", 0), ps.get("col", {}).get("slice_launches", 0)
    return 0 < ri < 0.75 * co


def psi_bytes_per_px(cls: str, psi: str, K: int, prec: str, last_only: bool = False) -> float:
    """Algorithmic HBM bytes per pixel of one launch of a kernel class for
    one shape kind (the paper's preconditioner).  FP64 doubles every vector
    and real array (the mask bits stay 1 bit per pixel).  TV, per PCG
    iteration: rowfwd reads z and p, writes p and t (32; 24 at k = 0); col
    reads t and the mask bits, writes t; rowinv reads t, p, both weights,
    writes q (32); update reads x, p, q, r, both weights, writes x, r, z
    (64).  Per outer iteration: |D x|^2 (read x, write 2 reals: 16), W (read
    2 reals, write 1: 12), d (16), the residual passes (16, 25, 32) and z0
    (read r and both weights, write z: 24)."""
    sc = 2.0 if prec == "fp64" else 1.0
    if psi == "haar":
        b = bytes_per_px(cls, K, True, last_only)
        return (b - 0.125) * sc + 0.125 if cls == "col" else b * sc
    tv = {"rowfwd": 32.0 - 8.0 / K, "col": 16.125, "rowinv": 32.0, "update": 64.0, "psi_sq": 16.0,
          "group_w": 12.0, "group_d": 16.0, "r0_rowfwd": 16.0, "r0_col": 25.0, "r0_rowinv": 32.0,
          "r0_update": 24.0, "adjoint": 33.0}.get(cls, 0.0)
    return (tv - 0.125) * sc + 0.125 if cls == "col" else tv * sc


def workload_problems(a):
    import synth
    if a.workload == "tv512":
        return [synth.cfg2(s) for s in range(a.seed0, a.seed0 + a.slices)], "FIRLS_TV, 512x512, 40 ellipses + ramp, " \
            "15% radial mask, sigma 0.005, periodic isotropic TV, lambda 0.01, eps 1e-10"
    if a.workload == "fp64_64":
        return [synth.cfg0(s) for s in range(a.seed0, a.seed0 + a.slices)], "plain l1 FIRLS_OG, 64x64, 25% VD mask, " \
            "sigma 0.01, 3-level Haar, singleton groups, lambda 0.035, eps 1e-10"
    return synth.cfg3_set(a.seed0, count=a.slices), \
        "uneven batch: sizes from {128,192,256,384,512}^2, 15-30% VD masks, sigma and lambda U[0.005,0.05], " \
        "tree-group Haar (L=4) and isotropic TV mixed 50/50, one call"


def run_workload(a, torch, F):
    """TV 512^2, FP64 64^2 and the uneven batch: one step = one batched
    solve of the workload's slices."""
    probs, desc = workload_problems(a)
    prec, K, B = a.prec, a.pcg, len(probs)
    keys = []
    for p in probs:
        k = (p.n, p.psi, p.levels)
        if k not in keys:
            keys.append(k)
    shapes = []
    for (n, psi, L) in keys:
        ref = next(p for p in probs if (p.n, p.psi, p.levels) == (n, psi, L))
        shapes.append(F.Shape(n, psi, L, ref.group_ptr, ref.group_idx))
    sid = [keys.index((p.n, p.psi, p.levels)) for p in probs]
    cdt = torch.complex64 if prec == "fp32" else torch.complex128

    def items_for(dt):
        out = []
        for p, k in zip(probs, sid):
            b = torch.from_numpy(p.b).to(dt).cuda()
            out.append(dict(b=b, mask=torch.from_numpy(p.mask).cuda(), x=torch.zeros_like(b), lam=p.lam, shape_id=k))
        return out

    solver = F.Solver(shapes, prec=prec, max_slices=B, max_outer=a.max_outer, pcg_iters=K, outer_tol=a.tau,
                      eps=1e-10)
    items = items_for(cdt)
    solver.set_paired(not a.no_pair)
    if a.sub_batch >= 0:
        solver.set_chunk(a.sub_batch)
        solver.set_graphs(a.launch != "direct")
        if a.schedule:
            solver.set_schedule({"per_shape": F.FIRLS_SCHED_PER_SHAPE, "across": F.FIRLS_SCHED_ACROSS,
                                 "largest_first": F.FIRLS_SCHED_ACROSS_LARGEST_FIRST}[a.schedule])
        chunk = a.sub_batch
    else:
        chunk = solver.autotune(items) if not a.no_tune else 0
        if a.no_pair:
            solver.set_paired(False)
    batch = solver.prepare(items)
    run = lambda: (solver.solve_batched(batch), None)
    dt, (reps, _), _ = timed(solver, run, a.steps, a.warmup, False, torch)
    prof = {}
    if not a.no_profile:
        _, _, prof = timed(solver, run, 1, 0, True, torch)
        per_shape = [solver.profile_read(i) for i in range(len(shapes))]
    outer = np.array([r["outer_iters"] for r in reps])
    pcg = np.array([r["pcg_iters"] for r in reps])
    fe = np.array([r["F_eps"] for r in reps])
    out = {"metric": f"solves/s ({a.workload})", "value": B * a.steps / dt, "unit": "solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == "fp32" else "f64",
           "data": "synthetic (seeded ellipse phantoms, VD or radial masks, complex Gaussian noise)",
           "config": {"workload": f"{desc}; {B} slices per step, {K} PCG per outer, stop at rel. F_eps decrease "
                                  f"{a.tau:g} (max {a.max_outer})", "slices": B, "pcg_iters": K, "tau": a.tau,
                      "max_outer": a.max_outer, "prec": prec, "sub_batch": chunk,
                      "launch": "graphs" if solver.graphs else "direct",
                      "schedule": ["per_shape", "across", "largest_first"][solver.schedule],
                      "paired": solver.paired,
                      "shapes": [f"{n}x{n} {psi}" for (n, psi, _) in keys]},
           "outer_iters_mean": float(outer.mean()), "outer_iters_max": int(outer.max()),
           "pcg_iters_per_s": float(pcg.sum() * a.steps / dt),
           "converged_frac": float(np.mean([r["converged"] for r in reps]))}
    if prof:
        pcg_cls = ("rowfwd", "col", "rowinv", "update", "last_x")
        tot_bytes, cls_bytes = 0.0, {}
        for i, (n, psi, _) in enumerate(keys):
            ps = per_shape[i]
            for c, v in ps.items():
                bb = psi_bytes_per_px(c, "haar" if psi == "haar" else "tv", K, prec,
                                      last_rowinv_only(ps)) * n * n * v["slice_launches"]
                tot_bytes += bb
                cls_bytes[c] = cls_bytes.get(c, 0.0) + bb
        dom = max((c for c in prof if c in pcg_cls and prof[c]["launches"]), key=lambda c: prof[c]["ms"])
        v = prof[dom]
        ach = cls_bytes[dom] / (v["ms"] / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": None,
                           "avg_launch_us": v["ms"] / v["launches"] * 1e3,
                           "bytes_per_launch": cls_bytes[dom] / v["launches"]}
        out["hbm_gbs_algorithmic"] = tot_bytes / (dt / a.steps) / 1e9
        out["kernel_ms"] = {c: round(u["ms"], 3) for c, u in prof.items() if u["launches"]}
        out["launches_per_step"] = int(sum(u["launches"] for u in prof.values()))
    if not a.no_gap:
        ref = F.Solver(shapes, prec=prec, max_slices=B, max_outer=a.ref_outer, pcg_iters=K, outer_tol=0.0, eps=1e-10)
        rit = items_for(cdt)
        rr = ref.solve_batched(rit)
        out["gap_to_optimum"] = gap_stats(fe, np.array([r["F_eps"] for r in rr]))
        out["gap_to_optimum"]["reference"] = f"same slices, {a.ref_outer} outer iterations, tau = 0"
        by = {}
        for (n, psi, _), r, f0 in zip([keys[k] for k in sid], rr, fe):
            by.setdefault(psi, []).append((f0 - r["F_eps"]) / r["F_eps"])
        out["gap_to_optimum"]["max_by_kind"] = {k: float(np.max(v)) for k, v in by.items()}
        ref.close()
    if a.workload == "tv512" and prec == "fp32" and not a.no_fp64_ref:
        # the same slices in FP64 with the same K, tau and cap
        s64 = F.Solver(shapes, prec="fp64", max_slices=B, max_outer=a.max_outer, pcg_iters=K, outer_tol=a.tau,
                       eps=1e-10)
        it64 = items_for(torch.complex128)
        r64 = s64.solve_batched(it64)
        dx = [float(torch.linalg.vector_norm(u["x"].to(torch.complex128) - w["x"]) / torch.linalg.vector_norm(w["x"]))
              for u, w in zip(items, it64)]
        f64 = np.array([r["F_eps"] for r in r64])
        o64 = np.array([r["outer_iters"] for r in r64])
        out["fp32_vs_fp64"] = {"F_eps_rel_diff_max": float(np.max(np.abs(fe - f64) / f64)),
                               "x_rel_l2_max": max(dx), "same_outer_count_frac": float(np.mean(o64 == outer)),
                               "fp64_outer_iters_mean": float(o64.mean())}
        s64.close()
    print(json.dumps(out))
    solver.close()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(slices are independent, so several GPUs would each run their own batch)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1411_5057_amd import firls as F

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "dense":
        return run_dense(a, torch, F)
    if a.workload in ("tv512", "fp64_64", "uneven"):
        return run_workload(a, torch, F)
    B, n, K = a.slices, a.n, a.pcg
    if a.copy_calib_mb:
        src = torch.ones(a.copy_calib_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    seeds = list(range(a.seed0, a.seed0 + B))
    p0, b, m, lams = make_inputs(seeds, n, torch)
    shape = F.Shape(n, "haar", 4, p0.group_ptr, p0.group_idx)
    pc = {"paper": F.FIRLS_PC_PAPER, "jacobi": F.FIRLS_PC_JACOBI, "none": F.FIRLS_PC_NONE}[a.precond]
    solver = F.Solver([shape], prec="fp32", max_slices=B, max_outer=a.max_outer, pcg_iters=K,
                      outer_tol=a.tau, eps=1e-10, precond=pc)
    x = torch.zeros_like(b)
    items = [dict(b=b[i], mask=m[i], x=x[i], lam=lams[i]) for i in range(B)]
    solver.set_paired(not a.no_pair)
    if a.sub_batch >= 0:
        chunk = a.sub_batch
        solver.set_chunk(chunk)
        solver.set_graphs(a.launch != "direct")
    else:
        chunk = solver.autotune(items) if not a.no_tune else 0
        if a.no_pair:
            solver.set_paired(False)
    use_learned = not a.no_learned and os.path.exists(a.weights) and n == 256
    net = F.Net(n, min(B, 64), np.fromfile(a.weights, dtype="<f4")) if use_learned else None

    # the same buffers every step: marshalled once
    batch_plain = solver.prepare(items)
    batch_learned = solver.prepare(items, learned=True)

    def run_plain():
        return solver.solve_batched(batch_plain), None

    def run_learned():
        return solver.solve_batched_learned(net, batch_learned)

    main_run = run_learned if use_learned else run_plain
    dt, (reps, used), _ = timed(solver, main_run, a.steps, a.warmup, False, torch)
    # kernel durations: one more step of the same call with HIP events around
    # every launch (events turn graph replay off, so this step is not timed)
    prof, dt_prof = {}, None
    if not a.no_profile:
        dt_prof, _, prof = timed(solver, main_run, 1, 0, True, torch)
    value = B * a.steps / dt
    outer = np.array([r["outer_iters"] for r in reps])
    pcg = np.array([r["pcg_iters"] for r in reps])
    fe = np.array([r["F_eps"] for r in reps])
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ellipse phantoms, VD masks, complex Gaussian noise)",
        "config": {"workload": f"tree-group FIRLS_OG, {n}x{n}, 20% VD mask, sigma 0.01, 4-level Haar, "
                               f"quadtree-pair groups, lambda 0.035, eps 1e-10, {B} slices per step "
                               f"(seeds {seeds[0]}-{seeds[-1]}), "
                               f"{K} PCG per outer, stop at rel. F_eps decrease {a.tau:g} (max {a.max_outer}), "
                               f"start: {'learned warm start (network + data consistency, A^H b fallback)' if use_learned else 'A^H b'}",
                   "n": n, "slices": B, "pcg_iters": K, "tau": a.tau, "max_outer": a.max_outer,
                   "start": "learned" if use_learned else "zero-filled", "sub_batch": chunk,
                   "launch": "graphs" if solver.graphs else "direct",
                   "paired": solver.paired, "precond": a.precond},
        "outer_iters_mean": float(outer.mean()), "outer_iters_max": int(outer.max()),
        "pcg_iters_per_s": float(pcg.sum() * a.steps / dt),
        "converged_frac": float(np.mean([r["converged"] for r in reps])),
    }
    if used is not None:
        out["learned_start_kept_frac"] = float(np.mean(used))
        out["weights"] = os.path.relpath(a.weights, ROOT)
    if prof:
        # the instrumented step does 1/steps of the timed work
        out["roofline"], out["hbm_gbs_algorithmic"], out["kernel_ms"] = roofline_of(prof, n, K, dt / a.steps, B, a.precond == "paper")
        out["kernel_time_frac_of_instrumented_step"] = sum(v["ms"] for v in prof.values()) / 1e3 / dt_prof
    plain = None
    if use_learned:
        dtp, (reps_p, _), _ = timed(solver, run_plain, a.steps, a.warmup, False, torch)
        op = np.array([r["outer_iters"] for r in reps_p])
        plain = {"value": B * a.steps / dtp, "unit": "solves/s", "ms_per_step": 1e3 * dtp / a.steps,
                 "outer_iters_mean": float(op.mean()), "outer_iters_max": int(op.max()),
                 "fe": np.array([r["F_eps"] for r in reps_p])}
    if not a.no_gap:
        # optimum estimate: the same slices, tau = 0, ref_outer outer iterations
        ref = F.Solver([shape], prec="fp32", max_slices=B, max_outer=a.ref_outer, pcg_iters=K,
                       outer_tol=0.0, eps=1e-10)
        xr = torch.zeros_like(b)
        rr = ref.solve_batched([dict(b=b[i], mask=m[i], x=xr[i], lam=lams[i]) for i in range(B)])
        fstar = np.array([r["F_eps"] for r in rr])
        out["gap_to_optimum"] = gap_stats(fe, fstar)
        out["gap_to_optimum"]["reference"] = f"same slices, {a.ref_outer} outer iterations, tau = 0"
        if plain is not None:
            plain["gap_to_optimum"] = gap_stats(plain["fe"], fstar)
        ref.close()
    # the oracle's optima where they are stored (golden seeds of this batch)
    fstar_or = oracle_optima()
    gold = [(i, sd) for i, sd in enumerate(seeds) if sd in fstar_or]
    if gold and n == 256:
        fs = np.array([fstar_or[sd] for _, sd in gold])
        g = {"seeds": f"{len(gold)} slices with a stored oracle optimum "
                      f"(tests/golden/optima_256.json: FP64 oracle, 300 outer x 20 PCG)",
             "gap": gap_stats(np.array([fe[i] for i, _ in gold]), fs)}
        if plain is not None:
            g["gap_plain"] = gap_stats(np.array([plain["fe"][i] for i, _ in gold]), fs)
        out["gap_to_oracle_optimum"] = g
    if plain is not None:
        out["outer_iters_saved"] = {"mean": plain["outer_iters_mean"] - out["outer_iters_mean"],
                                    "frac": 1.0 - out["outer_iters_mean"] / plain["outer_iters_mean"]}
        plain.pop("fe")
        out["plain"] = plain
        out["learned_speedup_vs_plain"] = value / plain["value"]
    if not a.no_cpu:
        # the x buffers hold the last timed call's results, which are from
        # the plain start (A^H b) whether or not the learned leg ran first
        xs = x.cpu().numpy()
        last = reps_p if use_learned else reps
        cb, per = cpu_baseline(n, a.tau, a.max_outer, K, seeds, xs,
                               [(r["F_eps"], r["outer_iters"]) for r in last])
        out["cpu_baseline"] = cb
        out["error_vs_fp64_oracle"] = per
    print(json.dumps(out))
    if net is not None:
        net.close()
    solver.close()


if __name__ == "__main__":
    main()

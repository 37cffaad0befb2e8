"""Full-size workloads on the GPU.

TV at 512^2 (40 ellipses + ramp, 15% radial mask, periodic differences,
isotropic TV): FP32 and FP64 runs against the FP64 oracle, and the FP32 vs
FP64 gap.  The 64-slice uneven batch (sizes 128..512, tree-group Haar and TV
mixed): one batched call; sampled slices are compared with the oracle one by
one, every slice is checked for the properties that hold at any size.
"""
import numpy as np
import pytest

import synth
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, dev_mask, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def gpu_solve(p, prec, T, K, tau=0.0):
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    s = F.Solver([shape_of(p)], prec=prec, max_outer=T, pcg_iters=K, outer_tol=tau)
    b = dev_complex(p.b, prec)
    x = torch.zeros_like(b)
    rep = s.solve(b, dev_mask(p.mask), x, p.lam)
    return to_np(x), rep


def test_tv_512_fp32_fp64():
    p = synth.cfg2(0)
    T, K = 6, 20
    ops = Operators.from_problem(p)
    ref = firls(ops, T, K)
    x32, r32 = gpu_solve(p, "fp32", T, K)
    x64, r64 = gpu_solve(p, "fp64", T, K)
    f32, f64 = ops.objective(x32)[0], ops.objective(x64)[0]
    assert abs(f64 - ref.F_eps) <= 1e-10 * ref.F_eps
    assert abs(f32 - ref.F_eps) <= 1e-5 * ref.F_eps
    err = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    print(f"TV 512^2: F_eps rel err fp32 {abs(f32 - ref.F_eps) / ref.F_eps:.2e}, "
          f"fp64 {abs(f64 - ref.F_eps) / ref.F_eps:.2e}; ||x32 - x64|| / ||x64|| = {err:.2e}")
    assert err < 1e-4


def test_uneven_batch_64():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = synth.cfg3_set(0)
    keys = sorted({(p.n, p.psi) for p in probs})
    shapes, sid = [], {}
    for k in keys:
        first = next(p for p in probs if (p.n, p.psi) == k)
        sid[k] = len(shapes)
        shapes.append(shape_of(first))
    T, K = 4, 20
    s = F.Solver(shapes, prec="fp32", max_slices=len(probs), max_outer=T, pcg_iters=K)
    items = []
    for p in probs:
        b = dev_complex(p.b, "fp32")
        items.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam, shape_id=sid[(p.n, p.psi)]))
    reps = s.solve_batched(items)
    for rep in reps:
        assert rep["status"] == 0 and rep["outer_iters"] == T and np.isfinite(rep["F_eps"])
    # every slice: the objective of the result is below the zero-filled
    # start's (Theorem 2) and matches what the library reports
    for p, it, rep in zip(probs, items, reps):
        b, m = it["b"], it["mask"]
        z = torch.empty_like(b)
        s.adjoint(b, m, z, shape_id=it["shape_id"])
        f0 = s.objective(b, m, p.lam, z, shape_id=it["shape_id"])[0]
        f1 = s.objective(b, m, p.lam, it["x"], shape_id=it["shape_id"])[0]
        assert f1 < f0
        assert abs(f1 - rep["F_eps"]) <= 1e-6 * f1
    # sampled slices against the oracle: the largest of each regulariser and one small one
    pick = {max((i for i, p in enumerate(probs) if p.psi == "haar"), key=lambda i: probs[i].n),
            max((i for i, p in enumerate(probs) if p.psi == "tv"), key=lambda i: probs[i].n),
            min(range(len(probs)), key=lambda i: probs[i].n)}
    for i in sorted(pick):
        ops = Operators.from_problem(probs[i])
        ref = firls(ops, T, K)
        fe = ops.objective(to_np(items[i]["x"]))[0]
        assert abs(fe - ref.F_eps) <= 1e-5 * ref.F_eps, (i, probs[i].n, probs[i].psi)

"""GPU parity on degenerate inputs against the oracle: zero measurements,
full sampling, a single (DC) sample, the smallest image (one Haar tile),
and batches that are empty or fill the handle exactly.

Bars as in test_gpu_solve: 1e-10 (FP64) and 1e-5 (FP32) relative objective
against the FP64 oracle, evaluated by the oracle on the GPU's result.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, dev_mask, rel, shape_of, to_np, torch_cuda
from tests.test_gpu_solve import OBJ_TOL, check

pytestmark = pytest.mark.gpu


def base(n=64, seed=3, psi="haar"):
    if psi == "haar":
        return synth.make_problem(n, seed, psi="haar", levels=3 if n >= 64 else 4, groups="quadtree", lam=0.03,
                                  sigma=0.01, frac=0.25)
    return synth.make_problem(n, seed, psi="tv", levels=0, groups="tv_iso", lam=0.02, sigma=0.01, frac=0.3)


@pytest.mark.parametrize("psi", ["haar", "tv"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_zero_measurements(psi, prec):
    """b = 0: x* = 0. The zero-filled start is already optimal, every PCG
    step has a zero residual (alpha and beta guarded to 0), F_eps is
    lambda * (number of groups) * sqrt(eps), and the stop rule fires at the
    second evaluation, as in the oracle."""
    p = dataclasses.replace(base(psi=psi), b=np.zeros((64, 64), dtype=np.complex128))
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    s = F.Solver([shape_of(p)], prec=prec, max_outer=10, pcg_iters=5, outer_tol=1e-6, eps=p.eps)
    b = dev_complex(p.b, prec)
    x = torch.zeros_like(b)
    rep = s.solve(b, dev_mask(p.mask), x, p.lam)
    ops = Operators.from_problem(p)
    ref = firls(ops, 10, 5, tau=1e-6)
    assert np.all(to_np(x) == 0.0)
    assert rep["status"] >= 0 and rep["converged"] == 1
    assert rep["outer_iters"] == ref.outer_iters
    expect = p.lam * (len(p.group_ptr) - 1) * np.sqrt(p.eps)
    assert abs(ref.F_eps - expect) <= 1e-12 * expect
    assert abs(rep["F_eps"] - expect) <= OBJ_TOL[prec] * expect


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_sampling(prec):
    """Every k-space entry sampled: A^H A = I, so for Haar the paper's
    preconditioner is S itself and one PCG iteration solves each
    reweighted system."""
    p0 = base()
    m = np.ones((64, 64), dtype=np.uint8)
    p = dataclasses.replace(p0, mask=m, b=synth.measure(p0.truth, m, synth.noise(64, 0.01, p0.seed)))
    x, rep, ref = check(p, prec, 6, 1)
    if prec == "fp64":
        assert rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_dc_sample(prec):
    """Only the DC entry sampled (rho = 1/N): the data fix one number and
    the penalty does the rest."""
    p0 = base()
    m = np.zeros((64, 64), dtype=np.uint8)
    m[0, 0] = 1
    p = dataclasses.replace(p0, mask=m, b=synth.measure(p0.truth, m, synth.noise(64, 0.01, p0.seed)))
    x, rep, ref = check(p, prec, 5, 10)
    if prec == "fp64":
        assert rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_smallest_image_one_tile(prec):
    """16 x 16 with 4 Haar levels: the whole image is one tile and one row
    band."""
    p = base(n=16, seed=4)
    x, rep, ref = check(p, prec, 8, 10)
    if prec == "fp64":
        assert rel(x, ref.x) < 1e-8


def test_empty_batch_is_rejected():
    torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = base()
    s = F.Solver([shape_of(p)], prec="fp32", max_slices=2, max_outer=2, pcg_iters=2)
    with pytest.raises(F.FirlsError):
        s.solve_batched([])


def test_batch_at_capacity_and_beyond():
    """max_slices slices run; one more is rejected before any work."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = [base(seed=10 + i) for i in range(3)]
    s = F.Solver([shape_of(probs[0])], prec="fp64", max_slices=3, max_outer=4, pcg_iters=8, eps=probs[0].eps)
    items = [dict(b=dev_complex(q.b, "fp64"), mask=dev_mask(q.mask), x=torch.zeros((64, 64), dtype=torch.complex128,
                                                                                    device="cuda"), lam=q.lam)
             for q in probs]
    reps = s.solve_batched(items)
    for q, it, r in zip(probs, items, reps):
        ref = firls(Operators.from_problem(q), 4, 8)
        assert r["status"] >= 0 and r["outer_iters"] == 4
        assert rel(to_np(it["x"]), ref.x) < 1e-8
    with pytest.raises(F.FirlsError):
        s.solve_batched(items + items[:1])

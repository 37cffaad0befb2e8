"""GPU parity of multi-contrast reconstruction (Section 5.6: FIRLS_MT with
wavelet joint sparsity, FIRLS_JTV with joint TV) against the oracle's
stacked problem.  Each slice carries C contrasts as C contiguous images;
groups run across contrasts, one PCG solves each reweighted system.

Bars as for single images: operators 1e-5 (FP32) / 1e-12 (FP64) relative;
whole solves 1e-5 / 1e-10 relative objective, evaluated by the oracle on
the GPU's own result.
"""
import numpy as np
import pytest

import synth
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, dev_mask, rel, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}
OBJ_TOL = {"fp32": 1e-5, "fp64": 1e-10}
CASES = [("haar", "joint", 3), ("tv", "jtv", 2), ("tvp", "jtv", 2), ("haar", "quadtree", 2)]


def problem(n, psi, groups, C, seed=1):
    return synth.make_mc_problem(n, seed, C=C, psi=psi, levels=3 if psi == "haar" else 0, groups=groups,
                                 lam=0.03, sigma=0.01, frac=0.25)


def crandn(seed, shape):
    rs = np.random.default_rng(seed)
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi,groups,C", CASES)
@pytest.mark.parametrize("n", [32, 128])
def test_mc_operators(n, psi, groups, C, prec):
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = problem(n, psi, groups, C)
    ops = Operators.from_problem(p)
    s = F.Solver([shape_of(p)], prec=prec)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    xw, v = crandn(3, (C, n, n)), crandn(4, (C, n, n))
    m = dev_mask(p.mask)
    # weights d(x)
    _, d_ref = ops.weights(xw)
    d = torch.empty(ops.n_coef, dtype=torch.float32 if prec == "fp32" else torch.float64, device="cuda")
    s.weights(dev_complex(xw, prec), d)
    np.testing.assert_allclose(d.cpu().numpy(), d_ref, rtol=TOL[prec] * 10, atol=0)
    # S p and P^{-1} r
    out = torch.empty((C, n, n), dtype=dt, device="cuda")
    s.system(m, p.lam, dev_complex(xw, prec), dev_complex(v, prec), out)
    assert rel(to_np(out), ops.S(v, d_ref)) < TOL[prec]
    s.precond(m, p.lam, dev_complex(xw, prec), dev_complex(v, prec), out)
    assert rel(to_np(out), ops.precond(d_ref)(v)) < TOL[prec]
    # objective and A^H b
    x = ops.AHb() + 0.05 * xw
    got = s.objective(dev_complex(p.b, prec), m, p.lam, dev_complex(x, prec))
    ref = ops.objective(to_np(dev_complex(x, prec)))
    for g, r in zip(got, ref):
        assert abs(g - r) <= TOL[prec] * abs(r)
    s.adjoint(dev_complex(p.b, prec), m, out)
    assert rel(to_np(out), ops.AHb()) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi,groups,C", CASES)
def test_mc_solve(psi, groups, C, prec):
    """8 outer x 20 PCG iterations from A^H b."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = problem(64, psi, groups, C, seed=5)
    ops = Operators.from_problem(p)
    s = F.Solver([shape_of(p)], prec=prec, max_outer=8, pcg_iters=20, eps=p.eps)
    b = dev_complex(p.b, prec)
    x = torch.zeros_like(b)
    rep = s.solve(b, dev_mask(p.mask), x, p.lam)
    ref = firls(ops, 8, 20)
    fe = ops.objective(to_np(x))[0]
    assert rep["status"] >= 0 and rep["outer_iters"] == 8
    assert abs(fe - ref.F_eps) <= OBJ_TOL[prec] * ref.F_eps, (fe, ref.F_eps)
    assert abs(rep["F_eps"] - fe) <= OBJ_TOL[prec] * fe
    if prec == "fp64":
        assert rel(to_np(x), ref.x) < 1e-8


def test_mc_batched_with_single_contrast_and_stop_rule():
    """One batch mixing a single image, an FIRLS_MT slice and an FIRLS_JTV
    slice, each run to the relative-decrease stop rule."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = [synth.make_problem(64, 7, psi="haar", levels=3, groups="quadtree", lam=0.03, sigma=0.01, frac=0.25),
             problem(64, "haar", "joint", 3, seed=8), problem(64, "tv", "jtv", 2, seed=9)]
    s = F.Solver([shape_of(q) for q in probs], prec="fp64", max_slices=3, max_outer=40, pcg_iters=20,
                 outer_tol=1e-5)
    items = []
    for i, q in enumerate(probs):
        b = dev_complex(q.b, "fp64")
        items.append(dict(b=b, mask=dev_mask(q.mask), x=torch.zeros_like(b), lam=q.lam, shape_id=i))
    reps = s.solve_batched(items)
    for q, it, rep in zip(probs, items, reps):
        ops = Operators.from_problem(q)
        ref = firls(ops, 40, 20, tau=1e-5)
        assert rep["converged"] == 1 and rep["outer_iters"] == ref.outer_iters
        assert abs(ops.objective(to_np(it["x"]))[0] - ref.F_eps) <= 1e-10 * ref.F_eps


def test_mc_rejects_shapes_beyond_the_partial_sum_slots():
    from paper_1411_5057_amd import firls as F
    p = problem(512, "tv", "jtv", 2)
    with pytest.raises(F.FirlsError):
        F.Solver([shape_of(p)], prec="fp32")       # 2 x 512 TV tiles exceed the partial-sum slots

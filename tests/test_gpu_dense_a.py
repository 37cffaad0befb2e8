"""GPU parity of FIRLS with a dense random-projection sensing matrix
(Section 5.2) against the oracle.  The products A v and A^T y run as
batched MFMA GEMMs over the slices of a launch; everything else is the
image-domain machinery of the masked-FFT path.

Bars: operators 1e-5 (FP32; K-long FP32 dot products) / 1e-12 (FP64)
relative; whole solves 1e-5 / 1e-10 relative objective.
"""
import numpy as np
import pytest

import synth
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, rel, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}
OBJ_TOL = {"fp32": 1e-5, "fp64": 1e-10}


def problem(n, psi, seed=1, m_frac=0.4):
    return synth.make_dense_problem(n, seed, m_frac=m_frac, psi=psi, levels=3 if psi == "haar" else 0,
                                    groups="quadtree" if psi == "haar" else "tv_iso", lam=0.03, sigma=0.01)


def crandn(seed, shape):
    rs = np.random.default_rng(seed)
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv"])
@pytest.mark.parametrize("n,m_frac", [(32, 0.4), (64, 0.3)])
def test_dense_operators(n, m_frac, psi, prec):
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = problem(n, psi, m_frac=m_frac)
    ops = Operators.from_problem(p)
    s = F.Solver([shape_of(p)], prec=prec)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    b = dev_complex(p.b, prec)
    out = torch.empty((n, n), dtype=dt, device="cuda")
    s.adjoint(b, None, out)
    assert rel(to_np(out), ops.AHb()) < TOL[prec]
    xw, v = crandn(3, (n, n)), crandn(4, (n, n))
    _, d = ops.weights(xw)
    s.system(None, p.lam, dev_complex(xw, prec), dev_complex(v, prec), out)
    assert rel(to_np(out), ops.S(v, d)) < TOL[prec]
    s.precond(None, p.lam, dev_complex(xw, prec), dev_complex(v, prec), out)
    assert rel(to_np(out), ops.precond(d)(v)) < TOL[prec]
    x = ops.AHb() + 0.05 * xw
    got = s.objective(b, None, p.lam, dev_complex(x, prec))
    ref = ops.objective(to_np(dev_complex(x, prec)))
    for g, r in zip(got, ref):
        assert abs(g - r) <= 10 * TOL[prec] * abs(r)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv"])
def test_dense_solve(psi, prec):
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = problem(64, psi, seed=5, m_frac=0.35)
    ops = Operators.from_problem(p)
    s = F.Solver([shape_of(p)], prec=prec, max_outer=8, pcg_iters=20, eps=p.eps)
    b = dev_complex(p.b, prec)
    x = torch.zeros((64, 64), dtype=b.dtype, device="cuda")
    rep = s.solve(b, None, x, p.lam)
    ref = firls(ops, 8, 20)
    fe = ops.objective(to_np(x))[0]
    assert rep["status"] >= 0 and rep["outer_iters"] == 8
    assert abs(fe - ref.F_eps) <= OBJ_TOL[prec] * ref.F_eps, (fe, ref.F_eps)
    assert abs(rep["F_eps"] - fe) <= OBJ_TOL[prec] * fe
    if prec == "fp64":
        assert rel(to_np(x), ref.x) < 1e-8


def test_dense_batch_spans_column_tiles_and_mixes_with_fft_shapes():
    """70 slices sharing one sensing matrix (three 32-slice column tiles of
    the GEMMs, the last one partial) plus two masked-FFT slices, one call,
    stop rule on; every slice against its own oracle run."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    base = problem(32, "haar", seed=11, m_frac=0.45)
    rs = np.random.default_rng(12)
    dense = []
    for i in range(70):
        q = problem(32, "haar", seed=11, m_frac=0.45)
        img = synth.phantom(32, 6, 100 + i)
        q.b = q.Amat @ img.ravel() + 0.01 * (rs.standard_normal(q.Amat.shape[0]) + 1j * rs.standard_normal(q.Amat.shape[0]))
        dense.append(q)
    fft = [synth.make_problem(32, 200 + i, psi="haar", levels=3, groups="quadtree", lam=0.03, sigma=0.01, frac=0.3)
           for i in range(2)]
    s = F.Solver([shape_of(base), shape_of(fft[0])], prec="fp64", max_slices=72, max_outer=12, pcg_iters=15,
                 outer_tol=1e-6)
    items = []
    for q in dense:
        b = dev_complex(q.b, "fp64")
        items.append(dict(b=b, mask=None, x=torch.zeros((32, 32), dtype=b.dtype, device="cuda"), lam=q.lam, shape_id=0))
    for q in fft:
        b = dev_complex(q.b, "fp64")
        items.append(dict(b=b, mask=torch.from_numpy(q.mask).cuda(), x=torch.zeros_like(b), lam=q.lam, shape_id=1))
    reps = s.solve_batched(items)
    for q, it, rep in zip(dense + fft, items, reps):
        ops = Operators.from_problem(q)
        ref = firls(ops, 12, 15, tau=1e-6)
        assert rep["outer_iters"] == ref.outer_iters
        assert abs(ops.objective(to_np(it["x"]))[0] - ref.F_eps) <= 1e-10 * ref.F_eps

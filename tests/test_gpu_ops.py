"""GPU parity of each step of the hot path against the FP64 oracle.

Each operator entry point of the C ABI (A^H, the weights d, S, P^{-1}, the
objective) is compared element by element with the oracle on the same
seeded inputs, at every built image size in both precisions: in norm and at
every element (|g - r| against max |r|).  FP64 must agree to rounding
(1e-12 relative); FP32 to 1e-5 relative (the FP32 tolerance the whole solve
is held to), which bounds a few ulps of the FFT / Haar / difference
arithmetic.
"""
import numpy as np
import pytest

import synth
from oracle import fourier
from oracle.firls import Operators
from tests.gpu_util import dev_complex, dev_mask, max_err, rel, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 48, 64, 96, 128, 192, 256, 384, 512]
TOL = {"fp32": 1e-5, "fp64": 1e-12}


def problem(n, psi, seed=1, groups=None, L=None):
    if psi == "haar":
        L = L if L is not None else (4 if n % 16 == 0 else 3)
        return synth.make_problem(n, seed, psi="haar", levels=L, groups=groups or "quadtree",
                                  lam=0.035, sigma=0.01, frac=0.25)
    return synth.make_problem(n, seed, psi=psi, levels=0, groups=groups or "tv_iso",
                              lam=0.02, sigma=0.01, frac=0.25)


def solver(prob, prec, **kw):
    from paper_1411_5057_amd import firls as F
    return F.Solver([shape_of(prob)], prec=prec, **kw)


def crandn(seed, n):
    rs = np.random.default_rng(seed)
    return rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", SIZES)
def test_adjoint(n, prec):
    torch = torch_cuda()
    p = problem(n, "haar", L=3)
    s = solver(p, prec)
    b, m = dev_complex(p.b, prec), dev_mask(p.mask)
    x = torch.empty_like(b)
    s.adjoint(b, m, x)
    ref = fourier.AH(p.b * p.mask, p.mask)
    assert rel(to_np(x), ref) < TOL[prec]
    assert max_err(to_np(x), ref) < TOL[prec]


@pytest.mark.parametrize("prec,psi,L,groups", [
    ("fp32", "haar", 4, "quadtree"), ("fp32", "haar", 3, "singletons"), ("fp32", "haar", 2, "quadtree"),
    ("fp64", "haar", 3, "quadtree"), ("fp64", "haar", 1, "singletons"),
    ("fp32", "tv", 0, "tv_iso"), ("fp32", "tv", 0, "tv_aniso"), ("fp64", "tv", 0, "tv_iso"),
    ("fp32", "tvp", 0, "tv_iso"), ("fp32", "tvp", 0, "tv_aniso"), ("fp64", "tvp", 0, "tv_iso")])
@pytest.mark.parametrize("n", [32, 96, 256])
def test_weights(n, prec, psi, L, groups):
    torch = torch_cuda()
    p = problem(n, psi, groups=groups, L=L)
    s = solver(p, prec)
    x = crandn(3, n)
    ops = Operators.from_problem(p)
    _, d_ref = ops.weights(x)
    d = torch.empty(ops.n_coef, dtype=torch.float32 if prec == "fp32" else torch.float64, device="cuda")
    s.weights(dev_complex(x, prec), d)
    np.testing.assert_allclose(d.cpu().numpy(), d_ref, rtol=TOL[prec] * 10, atol=0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv", "tvp"])
@pytest.mark.parametrize("n", [32, 64, 96, 192, 256, 512])
def test_system(n, psi, prec):
    torch = torch_cuda()
    p = problem(n, psi, L=3)
    s = solver(p, prec)
    ops = Operators.from_problem(p)
    xw, pv = crandn(4, n), crandn(5, n)
    _, d = ops.weights(xw)
    ref = ops.S(pv, d)
    q = torch.empty((n, n), dtype=torch.complex64 if prec == "fp32" else torch.complex128, device="cuda")
    s.system(dev_mask(p.mask), p.lam, dev_complex(xw, prec), dev_complex(pv, prec), q)
    assert rel(to_np(q), ref) < TOL[prec]
    assert max_err(to_np(q), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv", "tvp"])
@pytest.mark.parametrize("n", [32, 64, 192, 256])
def test_precond(n, psi, prec):
    torch = torch_cuda()
    p = problem(n, psi, L=3)
    s = solver(p, prec)
    ops = Operators.from_problem(p)
    xw, r = crandn(6, n), crandn(7, n)
    _, d = ops.weights(xw)
    ref = ops.precond(d)(r)
    z = torch.empty((n, n), dtype=torch.complex64 if prec == "fp32" else torch.complex128, device="cuda")
    s.precond(dev_mask(p.mask), p.lam, dev_complex(xw, prec), dev_complex(r, prec), z)
    assert rel(to_np(z), ref) < TOL[prec]
    assert max_err(to_np(z), ref) < TOL[prec]


@pytest.mark.parametrize("kind", ["jacobi", "none"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv", "tvp"])
@pytest.mark.parametrize("n", [32, 256])
def test_precond_ablation_variants(n, psi, prec, kind):
    """Jacobi (diag S) and identity preconditioners against the oracle's."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = problem(n, psi, L=3 if psi == "haar" else None)
    s = solver(p, prec, precond={"jacobi": F.FIRLS_PC_JACOBI, "none": F.FIRLS_PC_NONE}[kind])
    ops = Operators.from_problem(p)
    xw, r = crandn(16, n), crandn(17, n)
    _, d = ops.weights(xw)
    ref = ops.precond(d, kind)(r)
    z = torch.empty((n, n), dtype=torch.complex64 if prec == "fp32" else torch.complex128, device="cuda")
    s.precond(dev_mask(p.mask), p.lam, dev_complex(xw, prec), dev_complex(r, prec), z)
    assert rel(to_np(z), ref) < TOL[prec]
    assert max_err(to_np(z), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("psi", ["haar", "tv", "tvp"])
@pytest.mark.parametrize("n", [32, 128, 256])
def test_objective(n, psi, prec):
    p = problem(n, psi, L=3)
    s = solver(p, prec)
    ops = Operators.from_problem(p)
    x = ops.AHb() + 0.05 * crandn(8, n)
    got = s.objective(dev_complex(p.b, prec), dev_mask(p.mask), p.lam, dev_complex(x, prec))
    xr = to_np(dev_complex(x, prec))        # the values the GPU saw
    ref = ops.objective(xr)
    for g, r in zip(got, ref):
        assert abs(g - r) <= TOL[prec] * abs(r)


def test_invalid_arguments_raise():
    from paper_1411_5057_amd import firls as F
    p = problem(64, "haar")
    with pytest.raises(F.FirlsError):
        F.Solver([F.Shape(100, "haar", 2)])          # size not built
    with pytest.raises(F.FirlsError):
        F.Solver([F.Shape(64, "haar", 5)])           # too many levels
    with pytest.raises(F.FirlsError):
        F.Solver([shape_of(p)], pcg_iters=0)
    bad = shape_of(p)
    bad.group_idx = bad.group_idx.copy()
    bad.group_idx[3] = 64 * 64
    with pytest.raises(F.FirlsError):
        F.Solver([bad])

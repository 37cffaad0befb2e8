"""Pins of the dense random-projection operator (Section 5.2 and the
comparison with FOCUSS: A is a dense M x N matrix instead of R F).

Checks: adjoint and dense system; rho = mean diag(A^T A); PCG against a
Cholesky solve; an orthogonal A (A^T A = I) reduces FIRLS to closed-form
group shrinkage; an independent minimiser (L-BFGS) reaches the same
optimum; and the preconditioner ranking of Section 5.2 (eq. 17 against
Jacobi and plain CG) on this operator.
"""
import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import dense, haar
from oracle.firls import Operators, firls, pcg


def crandn(rs, *shape):
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


def prob(n=8, m_frac=0.5, psi="haar", L=2, groups="quadtree", lam=0.05, seed=2):
    return synth.make_dense_problem(n, seed, m_frac=m_frac, psi=psi, levels=L if psi == "haar" else 0,
                                    groups=groups, lam=lam, sigma=0.01)


def test_adjoint_rho_and_dense_system():
    p = prob()
    ops = Operators.from_problem(p)
    rs = np.random.default_rng(1)
    x, y = crandn(rs, 8, 8), crandn(rs, p.Amat.shape[0])
    assert abs(np.vdot(ops.A(x), y) - np.vdot(x.ravel(), ops.AH(y).ravel())) < 1e-11
    assert abs(ops.rho - np.mean(np.diag(p.Amat.T @ p.Amat))) < 1e-14
    d = rs.uniform(0.5, 3.0, ops.n_coef)
    P = dense.Psi(8, "haar", 2)
    S = p.Amat.T @ p.Amat + ops.lam * P.T @ (d[:, None] * P)
    np.testing.assert_allclose(ops.S(x, d).ravel(), S @ x.ravel(), atol=1e-12)
    xs, _ = pcg(ops, d, ops.AHb(), 300)
    np.testing.assert_allclose(xs.ravel(), np.linalg.solve(S, ops.AHb().ravel()), atol=1e-9)


def test_orthogonal_sensing_gives_group_shrinkage():
    """A orthogonal (M = N): A^T A = I, rho = 1, P = S, so one PCG
    iteration solves each reweighted system and the limit is the group
    shrinkage of beta = Phi A^T b (disjoint groups)."""
    n, L, lam, eps = 8, 2, 0.2, 1e-10
    p = prob(n=n, m_frac=1.0, L=L, groups="singletons", lam=lam)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n * n, n * n)))
    p.Amat = Q
    p.b = Q @ p.truth.ravel() + 0.01 * np.random.default_rng(4).standard_normal(n * n)
    ops = Operators.from_problem(p, eps=eps)
    assert abs(ops.rho - 1.0) < 1e-12
    beta = haar.fwd(ops.AHb(), L).ravel()
    x = ops.AHb()
    for _ in range(3):
        _, d = ops.weights(x)
        x, _ = pcg(ops, d, x, 1)
        np.testing.assert_allclose(haar.fwd(x, L).ravel(), beta / (1.0 + lam * d), atol=1e-11)
    rep = firls(ops, 3000, 1)     # coefficients at the threshold converge slowly
    star = dense.group_shrinkage(beta, p.group_ptr, p.group_idx, lam, eps)
    np.testing.assert_allclose(haar.fwd(rep.x, L).ravel(), star, atol=1e-7)


@pytest.mark.parametrize("psi", ["haar", "tv"])
def test_lbfgs_reaches_same_optimum(psi):
    p = prob(n=8, psi=psi, groups="quadtree" if psi == "haar" else "tv_iso", lam=0.05)
    ops = Operators.from_problem(p, eps=1e-4)
    n = ops.n

    def f_and_g(v):
        x = (v[: n * n] + 1j * v[n * n:]).reshape(n, n)
        _, d = ops.weights(x)
        g = ops.S(x, d) - ops.AHb()
        return ops.objective(x)[0], np.concatenate([g.real.ravel(), g.imag.ravel()])

    x0 = ops.AHb()
    res = scipy.optimize.minimize(f_and_g, np.concatenate([x0.real.ravel(), x0.imag.ravel()]), jac=True,
                                  method="L-BFGS-B", options={"maxiter": 20000, "ftol": 1e-15, "gtol": 1e-12})
    rep = firls(ops, 400, 40)
    assert abs(rep.F_eps - res.fun) <= 1e-9 * abs(res.fun)


def test_preconditioner_ranking_on_random_projections():
    """Section 5.2 (Fig. 2): with a random projection and a wavelet basis,
    a few PCG iterations with eq. 17 beat many more of Jacobi or plain CG
    (error of the reweighted subproblem against its exact solution, at the
    weights of the fifth outer iteration)."""
    p = prob(n=16, m_frac=0.4, L=3, groups="singletons", lam=0.05, seed=6)
    ops = Operators.from_problem(p)
    x0 = firls(ops, 5, 20).x
    _, d = ops.weights(x0)
    P = dense.Psi(16, "haar", 3)
    S = p.Amat.T @ p.Amat + ops.lam * P.T @ (d[:, None] * P)
    xs = np.linalg.solve(S, ops.AHb().ravel()).reshape(16, 16)
    err = {}
    for pc, k in (("pseudo", 15), ("jacobi", 60), ("none", 60)):
        x, _ = pcg(ops, d, x0, k, precond=pc)
        err[pc] = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err["pseudo"] < err["jacobi"] and err["pseudo"] < err["none"]

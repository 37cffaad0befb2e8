"""Pins of the oracle's preconditioners, PCG and outer loop.

Closed forms: P = S when the mask is full (PCG then converges in one
iteration), exact inverses against dense matrices, the SGS factors of the
TV preconditioner against their dense product, PCG against a Cholesky
solve, the group-shrinkage solution of A = F with disjoint groups and its
per-iteration IRLS update, and the theorems as invariants (monotone F_eps,
majoriser, stationarity), plus an independent L-BFGS minimisation.
"""
import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import dense, haar
from oracle.firls import Operators, firls, inner, pcg, stationarity


def crandn(rs, *shape):
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


def haar_problem(n=8, L=2, groups="quadtree", frac=0.3, seed=3, lam=0.05, mask="vd"):
    return Operators.from_problem(synth.make_problem(
        n, seed, psi="haar", levels=L, groups=groups, lam=lam, sigma=0.01,
        frac=frac, mask_kind=mask))


def tv_problem(n=8, frac=0.3, seed=3, lam=0.05, psi="tv"):
    return Operators.from_problem(synth.make_problem(
        n, seed, psi=psi, levels=0, groups="tv_iso", lam=lam, sigma=0.01, frac=frac))


def dense_P(ops, d):
    P = dense.Psi(ops.n, ops.psi, ops.levels)
    return ops.rho * np.eye(ops.n ** 2) + ops.lam * P.T @ (d[:, None] * P)


# -- preconditioners (eq. 17, eqs. 40-43) ---------------------------------------

def test_pseudo_diagonal_inverse_is_exact():
    ops = haar_problem()
    rs = np.random.default_rng(1)
    d = rs.uniform(0.5, 5.0, ops.n_coef)
    r = crandn(rs, ops.n, ops.n)
    z = ops.precond(d, "pseudo")(r)
    np.testing.assert_allclose(dense_P(ops, d) @ z.ravel(), r.ravel(), atol=1e-12)


def test_full_mask_makes_P_equal_S_one_iteration():
    """With every k-space sample kept, A^H A = I and rho = 1, so P = S and
    PCG solves the system in one iteration."""
    ops = haar_problem(n=16, L=3, mask="full")
    assert ops.rho == 1.0
    rs = np.random.default_rng(2)
    d = rs.uniform(0.1, 50.0, ops.n_coef)
    x, _ = pcg(ops, d, np.zeros((16, 16), complex), 1)
    res = ops.S(x, d) - ops.AHb()
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(ops.AHb())


def sgs_dense(Pm, order):
    """(D+L) D^{-1} (D+U) of P permuted to ``order`` then permuted back."""
    Pp = Pm[np.ix_(order, order)]
    D = np.diag(np.diag(Pp))
    Lo = np.tril(Pp, -1)
    Up = np.triu(Pp, 1)
    M = (D + Lo) @ np.linalg.inv(D) @ (D + Up)
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    return M[np.ix_(inv, inv)]


@pytest.mark.parametrize("psi", ["tv", "tvp"])
@pytest.mark.parametrize("n", [4, 8])
def test_tv_sgs_matches_dense_factors(n, psi):
    ops = tv_problem(n=n, psi=psi)
    rs = np.random.default_rng(n)
    d = np.repeat(rs.uniform(0.2, 4.0, n * n), 1)
    d = np.concatenate([d, d])                      # isotropic: same W for D1, D2 rows
    Pm = dense_P(ops, d)
    r = crandn(rs, n, n)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    lin = np.arange(n * n)
    rb = np.concatenate([lin[((ii + jj) % 2 == 0).ravel()], lin[((ii + jj) % 2 == 1).ravel()]])
    for kind, order in (("sgs_lex", lin), ("sgs_rb", rb)):
        M = sgs_dense(Pm, order)
        np.testing.assert_allclose(M, M.T, atol=1e-12)
        assert np.min(np.linalg.eigvalsh(M)) > 0
        z = ops.precond(d, kind)(r)
        np.testing.assert_allclose(M @ z.ravel(), r.ravel(), atol=1e-11)


def test_tv_sgs_general_weights_and_small_lambda():
    """Distinct D1 / D2 weights (anisotropic groups) and lambda -> 0, where
    the factors collapse to rho I."""
    n = 8
    ops = tv_problem(n=n)
    rs = np.random.default_rng(9)
    d = rs.uniform(0.2, 4.0, 2 * n * n)
    r = crandn(rs, n, n)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    lin = np.arange(n * n)
    rb = np.concatenate([lin[((ii + jj) % 2 == 0).ravel()], lin[((ii + jj) % 2 == 1).ravel()]])
    M = sgs_dense(dense_P(ops, d), rb)
    np.testing.assert_allclose(M @ ops.precond(d, "sgs_rb")(r).ravel(), r.ravel(), atol=1e-11)
    ops.lam = 1e-12
    np.testing.assert_allclose(ops.precond(d, "sgs_rb")(r), r / ops.rho, rtol=1e-9)


# -- PCG (Section 3.2) -------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["haar", "tv", "tvp"])
def test_pcg_converges_to_cholesky_solution(kind):
    ops = haar_problem() if kind == "haar" else tv_problem(psi=kind)
    rs = np.random.default_rng(4)
    d = rs.uniform(0.5, 20.0, ops.n_coef)
    if kind != "haar":
        d[ops.n ** 2:] = d[:ops.n ** 2]
    xs = dense.solve_S(ops, d)
    x, _ = pcg(ops, d, ops.AHb(), 200)
    np.testing.assert_allclose(x, xs, atol=1e-10 * np.abs(xs).max())
    for pc in ("none", "jacobi"):
        x2, _ = pcg(ops, d, ops.AHb(), 300, precond=pc)
        np.testing.assert_allclose(x2, xs, atol=1e-8 * np.abs(xs).max())


def test_pcg_preconditioner_beats_cg_and_jacobi():
    """Section 5.2: a few iterations with the proposed preconditioner beat
    many more of plain CG and Jacobi PCG (subproblem error against the exact
    Cholesky solve, at the weights of the fifth outer iteration)."""
    ops = haar_problem(n=16, L=3, frac=0.3, lam=0.035)
    x0 = firls(ops, 5, 20).x
    _, d = ops.weights(x0)
    xs = dense.solve_S(ops, d)
    err = {}
    for pc, k in (("pseudo", 10), ("jacobi", 50), ("none", 50)):
        x, _ = pcg(ops, d, x0, k, precond=pc)
        err[pc] = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err["pseudo"] < err["jacobi"] and err["pseudo"] < err["none"]


def test_tv_sgs_beats_jacobi_and_cg():
    """Section 5.3: the TV preconditioner of eq. (40) needs fewer PCG
    iterations than Jacobi, and far fewer than plain CG (residual reduction
    1e-2 at the weights of the third outer iteration, 32^2 radial mask)."""
    p = synth.make_problem(32, 4, psi="tv", levels=0, groups="tv_iso", lam=0.01, sigma=0.005,
                           mask_kind="radial", frac=0.15, ramp=True)
    ops = Operators.from_problem(p)
    x0 = firls(ops, 3, 20).x
    _, d = ops.weights(x0)
    b = ops.AHb()
    r0 = np.linalg.norm(b - ops.S(x0, d))
    need = {}
    for pc in ("sgs_rb", "jacobi", "none"):
        rec = []
        pcg(ops, d, x0, 150, precond=pc, record=rec)
        res = [np.linalg.norm(b - ops.S(xk, d)) / r0 for xk in rec]
        need[pc] = next((k for k, v in enumerate(res) if v <= 1e-2), 10 ** 9)
    assert need["sgs_rb"] < need["jacobi"] < need["none"]
    assert need["none"] > 2 * need["sgs_rb"]


def test_Q_majorises_and_decreases_along_pcg():
    """F_eps <= Q(., W^k) with equality at x^k (eqs. 20-21), and Q(., W^k)
    decreases along PCG started at x^k (eq. 24)."""
    ops = haar_problem(n=16, L=3)
    rs = np.random.default_rng(5)
    xk = ops.AHb()
    W, d = ops.weights(xk)
    assert abs(ops.Q(xk, W) - ops.objective(xk)[0]) < 1e-12 * ops.objective(xk)[0]
    for _ in range(5):
        y = xk + 0.3 * crandn(rs, 16, 16)
        assert ops.objective(y)[0] <= ops.Q(y, W) + 1e-12
    rec = []
    pcg(ops, d, xk, 15, record=rec)
    q = [ops.Q(xk, W)] + [ops.Q(x, W) for x in rec]
    assert all(q[i + 1] <= q[i] + 1e-12 * abs(q[i]) for i in range(len(q) - 1))


# -- outer loop (Algorithms 2, 3; Theorems 2, 3) ----------------------------------

@pytest.mark.parametrize("kind,K", [("haar", 3), ("haar", 20), ("tv", 3), ("tv", 20), ("tvp", 3), ("tvp", 20)])
def test_objective_monotone_any_pcg_count(kind, K):
    """Theorem 2 holds whatever the number of inner iterations."""
    ops = haar_problem(n=16, L=3, lam=0.035) if kind == "haar" else tv_problem(n=16, lam=0.02, psi=kind)
    rep = firls(ops, 15, K)
    h = np.asarray(rep.history)
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])


@pytest.mark.parametrize("kind,bound", [("haar", 2e-4), ("tv", 1e-5), ("tvp", 1e-5)])
def test_stationarity_at_convergence(kind, bound):
    """Theorem 3: the iterates approach a point where S(W(x)) x = A^H b,
    the gradient of F_eps (eps = 1e-6 keeps the run short)."""
    if kind == "haar":
        ops = haar_problem(n=16, L=3, lam=0.035)
    else:
        ops = tv_problem(n=16, lam=0.02, psi=kind)
    ops.eps = 1e-6
    s = [stationarity(ops, firls(ops, T, 30).x) for T in (20, 50, 100)]
    assert s[0] > s[1] > s[2] and s[2] < bound


def test_full_mask_disjoint_groups_closed_form():
    """A = F with every sample kept and disjoint groups: each IRLS step is
    alpha <- beta / (1 + lambda d) in Haar coefficients (P = S, one PCG
    iteration is exact), and the limit is the group shrinkage of beta."""
    n, L, lam, eps = 16, 3, 0.2, 1e-10
    p = synth.make_problem(n, 8, psi="haar", levels=L, groups="singletons",
                           lam=lam, sigma=0.01, mask_kind="full")
    # disjoint 2-coefficient groups: pair Mallat index 2i with 2i+1
    ptr = np.arange(0, n * n + 1, 2, dtype=np.int32)
    idx = np.arange(n * n, dtype=np.int32)
    p.group_ptr, p.group_idx = ptr, idx
    ops = Operators.from_problem(p, eps=eps)
    beta = haar.fwd(ops.AHb(), L).ravel()
    x = ops.AHb()
    for _ in range(4):
        _, d = ops.weights(x)
        alpha = beta / (1.0 + lam * d)
        x, _ = pcg(ops, d, x, 1)
        np.testing.assert_allclose(haar.fwd(x, L).ravel(), alpha, atol=1e-12)
    rep = firls(ops, 300, 1)
    star = dense.group_shrinkage(beta, ptr, idx, lam, eps)
    np.testing.assert_allclose(haar.fwd(rep.x, L).ravel(), star, atol=1e-7)


def test_lbfgs_reaches_same_optimum():
    """An independent minimiser of F_eps (scipy L-BFGS on the real and
    imaginary parts) agrees with FIRLS on the optimal value (F_eps is
    strictly convex, so the optimum is unique)."""
    ops = haar_problem(n=8, L=2, lam=0.05)
    ops.eps = 1e-4
    n = ops.n

    def f_and_g(v):
        x = (v[: n * n] + 1j * v[n * n:]).reshape(n, n)
        Fe = ops.objective(x)[0]
        _, d = ops.weights(x)
        g = ops.S(x, d) - ops.AHb()       # gradient of F_eps (complex)
        return Fe, np.concatenate([g.real.ravel(), g.imag.ravel()])

    x0 = ops.AHb()
    v0 = np.concatenate([x0.real.ravel(), x0.imag.ravel()])
    res = scipy.optimize.minimize(f_and_g, v0, jac=True, method="L-BFGS-B",
                                  options={"maxiter": 20000, "ftol": 1e-15, "gtol": 1e-12})
    rep = firls(ops, 300, 40)
    assert abs(rep.F_eps - res.fun) <= 1e-9 * abs(res.fun)


def test_gradient_identity_used_by_lbfgs():
    """The gradient of F_eps is S(W(x)) x - A^H b (eq. 15 at the current
    weights), checked by central differences."""
    ops = haar_problem(n=8, L=2, lam=0.05)
    ops.eps = 1e-3
    rs = np.random.default_rng(6)
    x = ops.AHb() + 0.1 * crandn(rs, 8, 8)
    _, d = ops.weights(x)
    g = ops.S(x, d) - ops.AHb()
    v = crandn(rs, 8, 8)
    h = 1e-6
    fd = (ops.objective(x + h * v)[0] - ops.objective(x - h * v)[0]) / (2 * h)
    assert abs(fd - inner(g, v)) < 1e-6 * max(1.0, abs(fd))


# -- reconstruction quality (Section 5.4) -----------------------------------------

def test_snr_db_closed_forms():
    """SNR = 10 log10(var(truth) / MSE) on the magnitude image, pinned by
    cases whose MSE is known in closed form: a constant offset c gives
    MSE = c^2; scaling by 2 gives MSE = mean(truth^2); a pure phase or sign
    change leaves the magnitude, so the SNR is infinite."""
    from oracle.firls import snr_db
    rs = np.random.default_rng(7)
    truth = rs.uniform(0.0, 1.0, (16, 16))
    var = float(np.mean((truth - truth.mean()) ** 2))
    for c in (0.01, 0.25):
        assert snr_db(truth + c, truth) == pytest.approx(10 * np.log10(var / c ** 2), rel=1e-12)
    assert snr_db(2.0 * truth, truth) == pytest.approx(10 * np.log10(var / np.mean(truth ** 2)), rel=1e-12)
    assert snr_db(truth * np.exp(0.7j), truth) > 250.0
    assert snr_db(-truth.astype(np.complex128), truth) == np.inf

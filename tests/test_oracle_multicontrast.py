"""Pins of the multi-contrast oracle (Section 5.6: FIRLS_MT with wavelet
joint sparsity, FIRLS_JTV with joint TV).

The C contrasts are one problem on the stacked vector x = [x_0; ...; x_{C-1}]:
A and Psi are block diagonal, the groups run across contrasts, and one PCG
(one set of scalars) solves each reweighted system.  These tests check the
stacked operators against dense block matrices, the joint group shrinkage in
closed form, and that contrast-separable groups give the single-contrast
optima.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import dense, fourier, haar
from oracle.firls import Operators, firls, pcg, stationarity


def crandn(rs, *shape):
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


def mc(n=8, C=2, psi="haar", groups="joint", L=2, lam=0.05, seed=3, mask="vd", frac=0.3):
    return Operators.from_problem(synth.make_mc_problem(
        n, seed, C=C, psi=psi, levels=L, groups=groups, lam=lam, sigma=0.01, frac=frac,
        mask_kind=mask))


def dense_psi(ops):
    """Stacked Psi with the block row order of the oracle (Haar blocks by
    contrast; TV: all D1 blocks, then all D2 blocks)."""
    n, C = ops.n, ops.C
    if ops.psi == "haar":
        return scipy.linalg.block_diag(*[dense.Phi(n, ops.levels)] * C)
    D = dense.Psi(n, ops.psi)
    N = n * n
    return np.vstack([scipy.linalg.block_diag(*[D[:N]] * C), scipy.linalg.block_diag(*[D[N:]] * C)])


def dense_S(ops, d):
    n, C = ops.n, ops.C
    F = dense.F2(n)
    AHA = scipy.linalg.block_diag(*[F.conj().T @ (ops.mask[c].ravel()[:, None] * F) for c in range(C)])
    P = dense_psi(ops)
    return AHA + ops.lam * P.T @ (d[:, None] * P)


@pytest.mark.parametrize("psi,groups", [("haar", "joint"), ("tv", "jtv"), ("tvp", "jtv"), ("haar", "quadtree")])
def test_stacked_system_matches_dense(psi, groups):
    ops = mc(psi=psi, groups=groups, L=2 if psi == "haar" else 0)
    rs = np.random.default_rng(1)
    d = rs.uniform(0.5, 3.0, ops.n_coef)
    x = crandn(rs, ops.C, ops.n, ops.n)
    np.testing.assert_allclose(ops.S(x, d).ravel(), dense_S(ops, d) @ x.ravel(), atol=1e-12)
    z = crandn(rs, ops.n_coef)
    # Psi^T is the adjoint of Psi
    assert abs(np.vdot(ops.psi_fwd(x), z) - np.vdot(x.ravel(), ops.psi_adj(z).ravel())) < 1e-10
    # rho is the mean diagonal of the stacked A^H A
    assert abs(ops.rho - ops.mask.mean()) < 1e-15


@pytest.mark.parametrize("psi,kind", [("haar", "pseudo"), ("haar", "jacobi"), ("tv", "sgs_rb"),
                                      ("tv", "sgs_lex"), ("tvp", "sgs_rb"), ("tv", "jacobi")])
def test_stacked_preconditioners_match_dense(psi, kind):
    ops = mc(psi=psi, groups="joint" if psi == "haar" else "jtv", L=2 if psi == "haar" else 0)
    rs = np.random.default_rng(2)
    d = rs.uniform(0.5, 3.0, ops.n_coef)
    r = crandn(rs, ops.C, ops.n, ops.n)
    Pd = dense_psi(ops)
    Pm = ops.rho * np.eye(ops.C * ops.n ** 2) + ops.lam * Pd.T @ (d[:, None] * Pd)
    z = ops.precond(d, kind)(r)
    if kind == "pseudo":
        np.testing.assert_allclose(Pm @ z.ravel(), r.ravel(), atol=1e-11)
    elif kind == "jacobi":
        np.testing.assert_allclose(np.diag(Pm) * z.ravel(), r.ravel(), atol=1e-11)
    else:
        # block diagonal SGS: each contrast's block in the single-contrast order
        n, N = ops.n, ops.n ** 2
        ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        lin = np.arange(N)
        order = lin if kind == "sgs_lex" else np.concatenate(
            [lin[((ii + jj) % 2 == 0).ravel()], lin[((ii + jj) % 2 == 1).ravel()]])
        for c in range(ops.C):
            blk = Pm[c * N:(c + 1) * N, c * N:(c + 1) * N][np.ix_(order, order)]
            D = np.diag(np.diag(blk))
            M = (D + np.tril(blk, -1)) @ np.linalg.inv(D) @ (D + np.triu(blk, 1))
            inv = np.empty_like(order)
            inv[order] = np.arange(N)
            M = M[np.ix_(inv, inv)]
            np.testing.assert_allclose(M @ z[c].ravel(), r[c].ravel(), atol=1e-10)


def test_joint_group_shrinkage_closed_form():
    """Full masks (A = F per contrast, rho = 1, P = S) and joint groups: each
    IRLS step is alpha = beta / (1 + lambda d) in Haar coefficients, and the
    limit shrinks each group's C-vector of coefficients by the group
    soft-threshold (with eps) jointly across contrasts."""
    n, L, C, lam, eps = 16, 3, 3, 0.2, 1e-10
    p = synth.make_mc_problem(n, 8, C=C, psi="haar", levels=L, groups="joint", lam=lam, sigma=0.01,
                              mask_kind="full")
    ops = Operators.from_problem(p, eps=eps)
    beta = ops.psi_fwd(ops.AHb())
    x = ops.AHb()
    for _ in range(4):
        _, d = ops.weights(x)
        x, _ = pcg(ops, d, x, 1)
        np.testing.assert_allclose(ops.psi_fwd(x), beta / (1.0 + lam * d), atol=1e-12)
    rep = firls(ops, 300, 1)
    star = dense.group_shrinkage(beta, p.group_ptr, p.group_idx, lam, eps)
    np.testing.assert_allclose(ops.psi_fwd(rep.x), star, atol=1e-7)
    # groups really couple the contrasts: a shared weight per group
    _, d = ops.weights(rep.x)
    N = n * n
    np.testing.assert_allclose(d[:N], d[N:2 * N])


@pytest.mark.parametrize("psi,groups,L", [("haar", "quadtree", 2), ("tv", "tv_iso", 0)])
def test_separable_groups_give_single_contrast_optima(psi, groups, L):
    """Groups that do not cross contrasts make F_eps a sum over contrasts,
    so the stacked optimum is the tuple of single-contrast optima (the
    shared PCG scalars change the path, not the limit)."""
    n, C = 8, 2
    p = synth.make_mc_problem(n, 5, C=C, psi=psi, levels=L, groups=groups, lam=0.05, sigma=0.01, frac=0.4)
    ops = Operators.from_problem(p, eps=1e-6)
    rep = firls(ops, 400, 30, tau=1e-14)
    for c in range(C):
        q = synth.make_problem(n, 5, psi=psi, levels=L, groups=groups, lam=0.05, sigma=0.01, frac=0.4)
        q.mask, q.b = p.mask[c], p.b[c]
        one = Operators.from_problem(q, eps=1e-6)
        ref = firls(one, 400, 30, tau=1e-14)
        assert abs(one.objective(rep.x[c])[0] - ref.F_eps) <= 1e-9 * ref.F_eps
        np.testing.assert_allclose(rep.x[c], ref.x, atol=1e-5 * np.abs(ref.x).max())


@pytest.mark.parametrize("psi,groups", [("haar", "joint"), ("tv", "jtv")])
def test_monotone_and_stationary(psi, groups):
    """Theorems 2 and 3 on the stacked problem."""
    ops = mc(n=16, C=2, psi=psi, groups=groups, L=3 if psi == "haar" else 0, lam=0.03)
    h = np.asarray(firls(ops, 15, 5).history)
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])
    ops.eps = 1e-6
    st = [stationarity(ops, firls(ops, T, 30).x) for T in (10, 40, 120)]
    assert st[0] > st[1] > st[2] and st[2] < 1e-3

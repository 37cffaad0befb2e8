"""Pins of the oracle's linear operators against definitions written out.

Each check compares the fast oracle operator with something other than
itself: the DFT by its sum, the Haar transform by Kronecker products of the
1D Haar matrix, differences by shift matrices, the group rule by an explicit
replication matrix G (Fig. 1), adjoints by dot-product identities.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dense, fourier, groups, haar, tv
from oracle.firls import Operators

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crandn(rs, *shape):
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


# -- Fourier (Section 5.4) ----------------------------------------------------

@pytest.mark.parametrize("n", [4, 6, 8, 12, 16])
def test_fft_matches_dft_definition(n):
    rs = np.random.default_rng(n)
    x = crandn(rs, n, n)
    np.testing.assert_allclose(fourier.fft2u(x), fourier.dft2_naive(x), atol=1e-12)
    np.testing.assert_allclose(fourier.ifft2u(fourier.dft2_naive(x)), x, atol=1e-12)


def test_dft_unitary_and_parseval():
    F = dense.F2(6)
    np.testing.assert_allclose(F.conj().T @ F, np.eye(36), atol=1e-12)
    x = crandn(np.random.default_rng(1), 16, 16)
    assert abs(np.linalg.norm(fourier.fft2u(x)) - np.linalg.norm(x)) < 1e-12


def test_A_adjoint_identity():
    rs = np.random.default_rng(2)
    m = (rs.random((16, 16)) < 0.3).astype(np.float64)
    x, y = crandn(rs, 16, 16), crandn(rs, 16, 16)
    lhs = np.vdot(fourier.A(x, m), y)
    rhs = np.vdot(x, fourier.AH(y, m))
    assert abs(lhs - rhs) < 1e-11


def test_rho_is_every_diagonal_entry_of_AHA():
    """Section 5.4: the mean diagonal of A^T A is the sampling ratio; for the
    unitary F every diagonal entry equals M / N."""
    m = synth.vd_mask(8, 0.25, 3).astype(np.float64)
    F = dense.F2(8)
    AHA = F.conj().T @ (m.ravel()[:, None] * F)
    np.testing.assert_allclose(np.diag(AHA).real, fourier.rho(m), atol=1e-13)
    np.testing.assert_allclose(np.diag(AHA).imag, 0.0, atol=1e-13)


# -- Haar (Section 3.1) ------------------------------------------------------------

@pytest.mark.parametrize("n,L", [(4, 1), (8, 1), (8, 2), (8, 3), (16, 2), (16, 4)])
def test_haar_matches_kronecker_matrix(n, L):
    rs = np.random.default_rng(10 * n + L)
    x = crandn(rs, n, n)
    P = dense.Phi(n, L)
    np.testing.assert_allclose(haar.fwd(x, L).ravel(), P @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(haar.adj(x, L).ravel(), P.T @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(P.T @ P, np.eye(n * n), atol=1e-12)


def test_haar_inverse_and_constant_image():
    rs = np.random.default_rng(5)
    x = crandn(rs, 32, 32)
    np.testing.assert_allclose(haar.adj(haar.fwd(x, 4), 4), x, atol=1e-12)
    c = 0.37
    z = haar.fwd(np.full((32, 32), c), 4)
    h = 32 >> 4
    np.testing.assert_allclose(z[:h, :h], c * 2 ** 4, atol=1e-12)
    z[:h, :h] = 0.0
    assert np.max(np.abs(z)) < 1e-12


def test_haar_single_level_hand_values():
    """One level on a 2x2 image: [[a, b], [c, d]] -> averages and
    differences with factor 1/2 in 2D."""
    a, b, c, d = 1.0, 2.0, 3.0, 5.0
    z = haar.fwd(np.array([[a, b], [c, d]]), 1)
    np.testing.assert_allclose(z, [[(a + b + c + d) / 2, (a - b + c - d) / 2],
                                   [(a + b - c - d) / 2, (a - b - c + d) / 2]], atol=1e-15)


# -- TV differences (Section 4.1) ---------------------------------------------------

def test_tv_matches_shift_matrices_and_adjoint():
    n = 6
    rs = np.random.default_rng(7)
    x = crandn(rs, n, n)
    np.testing.assert_allclose(tv.d1(x).ravel(), dense.D1(n) @ x.ravel(), atol=1e-13)
    np.testing.assert_allclose(tv.d2(x).ravel(), dense.D2(n) @ x.ravel(), atol=1e-13)
    y = crandn(rs, 2 * n * n)
    assert abs(np.vdot(tv.fwd(x), y) - np.vdot(x.ravel(), tv.adj(y, n).ravel())) < 1e-11
    np.testing.assert_allclose(tv.fwd(np.full((n, n), 2.5)), 0.0, atol=1e-14)


def test_tv_hand_values():
    x = np.arange(9, dtype=np.float64).reshape(3, 3)
    assert tv.d1(x)[0, 0] == x[1, 0] - x[0, 0]
    assert tv.d1(x)[2, 1] == x[0, 1] - x[2, 1]       # periodic wrap
    assert tv.d2(x)[1, 2] == x[1, 0] - x[1, 2]


def test_paper_tv_matches_printed_matrices_and_adjoint():
    """The paper's D1, D2 (Section 4.1): ones on the diagonal, minus ones one
    pixel above (D1) or one pixel to the left (D2), no wrap; built here as
    Kronecker products of the printed bidiagonal with the identity."""
    n = 6
    rs = np.random.default_rng(8)
    x = crandn(rs, n, n)
    np.testing.assert_allclose(tv.d1p(x).ravel(), dense.D1p(n) @ x.ravel(), atol=1e-13)
    np.testing.assert_allclose(tv.d2p(x).ravel(), dense.D2p(n) @ x.ravel(), atol=1e-13)
    y = crandn(rs, 2 * n * n)
    assert abs(np.vdot(tv.fwd_p(x), y) - np.vdot(x.ravel(), tv.adj_p(y, n).ravel())) < 1e-11
    # injective: the first row of each difference keeps the pixel itself
    P = dense.Psi(n, "tvp")
    assert np.linalg.matrix_rank(P) == n * n


def test_paper_tv_hand_values():
    x = np.arange(9, dtype=np.float64).reshape(3, 3) + 1.0
    assert tv.d1p(x)[0, 2] == x[0, 2]                # first row: identity
    assert tv.d1p(x)[2, 1] == x[2, 1] - x[1, 1]
    assert tv.d2p(x)[1, 0] == x[1, 0]                # first column: identity
    assert tv.d2p(x)[1, 2] == x[1, 2] - x[1, 1]
    # a constant image leaves only the boundary identity rows
    z = tv.fwd_p(np.full((3, 3), 2.0))
    assert np.count_nonzero(z) == 3 + 3 and np.all(z[z != 0] == 2.0)


# -- Group replication G (Section 3.1, Fig. 1) ----------------------------------

def dense_G(ptr, idx, count):
    G = np.zeros((len(idx), count))
    G[np.arange(len(idx)), idx] = 1.0
    return G


def test_fig1_group_matrices():
    spec = json.load(open(os.path.join(GOLDEN, "fig1_groups.json")))
    n = spec["signal_length"]
    rs = np.random.default_rng(11)
    for key, grp in spec["cases"].items():
        ptr = np.concatenate([[0], np.cumsum([len(g) for g in grp])]).astype(np.int32)
        idx = np.asarray([i - 1 for g in grp for i in g], dtype=np.int32)
        G = dense_G(ptr, idx, n)
        assert G.shape[0] == spec["G_rows"][key]
        np.testing.assert_array_equal(G.sum(axis=0), spec["membership_count"][key])
        z = crandn(rs, n)
        W = groups.weights(z, ptr, idx, 1e-10)
        # W repeats each group weight |g_i| times (eq. 13)
        Wfull = np.repeat(W, np.diff(ptr))
        Gz = G @ z
        for gi in range(len(grp)):
            seg = slice(ptr[gi], ptr[gi + 1])
            np.testing.assert_allclose(W[gi], 1 / np.sqrt(np.sum(np.abs(Gz[seg]) ** 2) + 1e-10))
        d = groups.replicated_diag(W, ptr, idx, n)
        np.testing.assert_allclose(np.diag(G.T @ np.diag(Wfull) @ G), d, atol=1e-12)
        off = G.T @ np.diag(Wfull) @ G - np.diag(d)
        assert np.max(np.abs(off)) == 0.0   # G^T W G is diagonal


def test_singleton_weights_are_standard_irls():
    """Section 3.1: with one element per group the weights are those of
    standard IRLS, W_i = (|z_i|^2 + eps)^{-1/2}."""
    rs = np.random.default_rng(12)
    z = crandn(rs, 50)
    ptr, idx = synth.groups_singletons(50)
    np.testing.assert_allclose(groups.weights(z, ptr, idx, 1e-6), 1 / np.sqrt(np.abs(z) ** 2 + 1e-6))


def test_quadtree_groups_membership():
    n, L = 16, 3
    ptr, idx = synth.groups_quadtree_pairs(n, L)
    G = dense_G(ptr, idx, n * n)
    assert G.shape == (2 * n * n - n * n // 4 ** (L - 1), n * n)
    cnt = G.sum(axis=0).reshape(n, n)
    assert cnt[0, 0] == 1 and cnt[1, 1] == 1       # coarsest approximation
    assert cnt[n - 1, n - 1] == 1                  # finest detail: a leaf
    assert cnt[1, 3] == 5                          # level-L detail: self + 4 children
    assert cnt[n // 4 - 1, n // 2 - 1] == 5        # level-2 detail: self + 4 children


# -- System S (eq. 15, eq. 39) and its dense form ------------------------------------

@pytest.mark.parametrize("psi", ["haar", "tv", "tvp"])
def test_S_matches_dense(psi):
    n = 8
    p = synth.make_problem(n, 4, psi=psi, levels=2 if psi == "haar" else 0,
                           groups="quadtree" if psi == "haar" else "tv_iso",
                           lam=0.05, sigma=0.01, frac=0.3)
    ops = Operators.from_problem(p)
    rs = np.random.default_rng(13)
    d = rs.uniform(0.5, 3.0, ops.n_coef)
    x = crandn(rs, n, n)
    S = dense.S_matrix(ops, d)
    np.testing.assert_allclose(ops.S(x, d).ravel(), S @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(S, S.conj().T, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(S)) > 0


def test_psi_diag_matches_dense():
    rs = np.random.default_rng(14)
    for psi, L in (("haar", 2), ("haar", 3), ("tv", 0), ("tvp", 0)):
        p = synth.make_problem(8, 1, psi=psi, levels=L,
                               groups="singletons" if psi == "haar" else "tv_iso",
                               lam=0.05, sigma=0.01)
        ops = Operators.from_problem(p)
        d = rs.uniform(0.5, 3.0, ops.n_coef)
        P = dense.Psi(8, psi, L)
        np.testing.assert_allclose(ops.psi_diag(d).ravel(), np.diag(P.T @ (d[:, None] * P)), atol=1e-12)

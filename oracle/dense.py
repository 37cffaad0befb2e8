"""Dense matrices of every operator, for images of a few hundred pixels.

These are built from the definitions (Kronecker products of the 1D DFT and
1D Haar matrices, shift matrices for the differences), independently of the
fast operators, and serve to pin them: exact S, exact IRLS steps by
Cholesky, and the closed-form group shrinkage when A is the full unitary
Fourier transform (mask of ones) and groups are disjoint.

Vectors are images flattened row-major.
"""
import numpy as np

from . import fourier


def F2(n):
    """Unitary 2D DFT acting on row-major vec(X): kron(F_n, F_n)."""
    Fn = fourier.dft_matrix(n)
    return np.kron(Fn, Fn)


def haar_1d(m):
    """One level of the orthonormal 1D Haar step on length m: averages in the
    first m/2 outputs, differences in the last m/2."""
    H = np.zeros((m, m))
    s = 1.0 / np.sqrt(2.0)
    for i in range(m // 2):
        H[i, 2 * i] = s
        H[i, 2 * i + 1] = s
        H[m // 2 + i, 2 * i] = s
        H[m // 2 + i, 2 * i + 1] = -s
    return H


def Phi(n, L):
    """L-level 2D Haar as an n^2 x n^2 matrix: level l applies
    kron(H_h, H_h) to the top-left h x h block (h = n / 2^(l-1)) and the
    identity to every other entry."""
    N = n * n
    M = np.eye(N)
    for lev in range(L):
        h = n >> lev
        blk = np.array([r * n + c for r in range(h) for c in range(h)])
        step = np.eye(N)
        step[np.ix_(blk, blk)] = np.kron(haar_1d(h), haar_1d(h))
        M = step @ M
    return M


def shift(n, dr, dc):
    """Permutation matrix with (S x)[r, c] = x[(r + dr) mod n, (c + dc) mod n]."""
    N = n * n
    S = np.zeros((N, N))
    for r in range(n):
        for c in range(n):
            S[r * n + c, ((r + dr) % n) * n + (c + dc) % n] = 1.0
    return S


def D1(n):
    return shift(n, 1, 0) - np.eye(n * n)


def D2(n):
    return shift(n, 0, 1) - np.eye(n * n)


def bidiag(n):
    """n x n: ones on the diagonal, minus ones just below (the paper's
    difference matrix of Section 4.1 on one image column or row)."""
    return np.eye(n) - np.eye(n, k=-1)


def D1p(n):
    """The paper's vertical differences on the row-major vector: B on the row index."""
    return np.kron(bidiag(n), np.eye(n))


def D2p(n):
    return np.kron(np.eye(n), bidiag(n))


def Psi(n, psi, L=0):
    if psi == "haar":
        return Phi(n, L)
    if psi == "tvp":
        return np.vstack([D1p(n), D2p(n)])
    return np.vstack([D1(n), D2(n)])


def S_matrix(ops, d):
    """Dense S = F^H diag(m) F + lambda Psi^T diag(d) Psi."""
    n = ops.n
    F = F2(n)
    P = Psi(n, ops.psi, ops.levels)
    m = ops.mask.ravel()
    return F.conj().T @ (m[:, None] * F) + ops.lam * P.T @ (d[:, None] * P)


def solve_S(ops, d):
    """Exact minimiser of Q(., W) (eq. 14) by Cholesky of the dense S."""
    S = S_matrix(ops, d)
    Lc = np.linalg.cholesky(S)
    rhs = ops.AHb().ravel()
    y = np.linalg.solve(Lc, rhs)
    return np.linalg.solve(Lc.conj().T, y).reshape(ops.n, ops.n)


def shrink_norm(beta_norm, lam, eps, iters=200):
    """t >= 0 solving t + lam t / sqrt(t^2 + eps) = beta_norm (bisection).

    The stationarity condition of 1/2 (t - ||beta||)^2 + lam sqrt(t^2 + eps)
    along the direction of beta."""
    lo, hi = 0.0, float(beta_norm)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid + lam * mid / np.sqrt(mid * mid + eps) > beta_norm:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def group_shrinkage(beta, ptr, idx, lam, eps):
    """Minimiser of 1/2 ||alpha - beta||^2 + lam sum_g sqrt(||alpha_g||^2 + eps)
    for disjoint groups covering every coefficient."""
    alpha = np.zeros_like(beta)
    for g in range(len(ptr) - 1):
        mem = idx[ptr[g]:ptr[g + 1]]
        nb = float(np.linalg.norm(beta[mem]))
        if nb == 0.0:
            continue
        alpha[mem] = shrink_norm(nb, lam, eps) * beta[mem] / nb
    return alpha

"""Group weights of the reweighted problem (Section 3.1, eqs. 12-13).

Psi = G Phi with G made of rows of the identity, so the rows of G Phi x are
coefficients of Phi x, some of them replicated.  A group map is given as
CSR lists over the coefficient indices: group i holds the coefficients
``idx[ptr[i]:ptr[i+1]]``.

W_i = (||(G Phi x)_{g_i}||^2 + eps)^{-1/2}                   (eq. 12)
W (N' x N') repeats W_i |g_i| times on its diagonal             (eq. 13)
G^T W G is diagonal; its entry j is d_j = sum over groups containing j of W_i.
For TV the coefficients are the 2N rows of [D1 x; D2 x] and eq. (37)
is the pixel-pair case of the same rule.
"""
import numpy as np


def group_sq(z, ptr, idx):
    """s_i = sum_{j in g_i} |z_j|^2, float64 per group."""
    a = np.abs(z.ravel()[idx]) ** 2
    sizes = np.diff(ptr)
    out = np.zeros(len(sizes), dtype=np.float64)
    nz = sizes > 0
    out[nz] = np.add.reduceat(a, ptr[:-1][nz])
    return out


def weights(z, ptr, idx, eps):
    """Per-group W_i."""
    return 1.0 / np.sqrt(group_sq(z, ptr, idx) + eps)


def replicated_diag(W, ptr, idx, count):
    """d = diag(G^T W G): d_j = sum_{i: j in g_i} W_i."""
    d = np.zeros(count, dtype=np.float64)
    np.add.at(d, idx, np.repeat(W, np.diff(ptr)))
    return d


def penalty(z, ptr, idx, eps):
    """sum_i sqrt(||z_{g_i}||^2 + eps), and the unsmoothed sum_i ||z_{g_i}||."""
    s = group_sq(z, ptr, idx)
    return float(np.sum(np.sqrt(s + eps))), float(np.sum(np.sqrt(s)))

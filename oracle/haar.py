"""Orthonormal 2D Haar wavelet Phi (Section 3.1: an orthogonal sparse basis).

One level: along every row, pairs (x[2i], x[2i+1]) become the average
(x[2i] + x[2i+1]) / sqrt(2) stored at column i and the difference
(x[2i] - x[2i+1]) / sqrt(2) stored at column h + i; then the same along
every column.  Level l repeats this on the top-left approximation block of
side n / 2^(l-1).  Coefficients are kept in this Mallat layout over the
whole n x n image.  Phi is real and orthogonal, so Phi^T = Phi^{-1}; on
complex images it acts on real and imaginary parts alike.
"""
import numpy as np

_S = 1.0 / np.sqrt(2.0)


def _fwd_1d(blk, axis):
    if axis == 1:
        a = (blk[:, 0::2] + blk[:, 1::2]) * _S
        d = (blk[:, 0::2] - blk[:, 1::2]) * _S
        return np.concatenate([a, d], axis=1)
    a = (blk[0::2, :] + blk[1::2, :]) * _S
    d = (blk[0::2, :] - blk[1::2, :]) * _S
    return np.concatenate([a, d], axis=0)


def _inv_1d(blk, axis):
    h = blk.shape[axis] // 2
    out = np.empty_like(blk)
    if axis == 1:
        a, d = blk[:, :h], blk[:, h:]
        out[:, 0::2] = (a + d) * _S
        out[:, 1::2] = (a - d) * _S
    else:
        a, d = blk[:h, :], blk[h:, :]
        out[0::2, :] = (a + d) * _S
        out[1::2, :] = (a - d) * _S
    return out


def fwd(x, L):
    """z = Phi x (Mallat layout)."""
    z = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    h = z.shape[0]
    for _ in range(L):
        blk = _fwd_1d(z[:h, :h], axis=1)
        z[:h, :h] = _fwd_1d(blk, axis=0)
        h //= 2
    return z


def adj(z, L):
    """x = Phi^T z (= Phi^{-1} z)."""
    x = np.array(z, dtype=np.result_type(z, np.float64), copy=True)
    n = x.shape[0]
    for lev in range(L - 1, -1, -1):
        h = n >> lev
        blk = _inv_1d(x[:h, :h], axis=0)
        x[:h, :h] = _inv_1d(blk, axis=1)
    return x

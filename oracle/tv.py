"""First-order finite differences for TV (Section 4.1).

Two boundaries:

periodic ("tv"):
  (D1 x)[r, c] = x[r+1, c] - x[r, c]  (vertical),
  (D2 x)[r, c] = x[r, c+1] - x[r, c]  (horizontal), indices mod n;
  the adjoints are (D1^T y)[r, c] = y[r-1, c] - y[r, c], likewise for D2.

the paper's matrices ("tvp"): lower bidiagonal, ones on the diagonal and
minus ones one row (D1) or one image column (D2) below it, acting on each
image column / row, so the first entry of each difference is the pixel
itself:
  (D1 x)[r, c] = x[r, c] - x[r-1, c] for r >= 1,   x[0, c] for r = 0,
  (D2 x)[r, c] = x[r, c] - x[r, c-1] for c >= 1,   x[r, 0] for c = 0;
  D = I - S with S the shift by one; D^T = I - S^T:
  (D1^T y)[r, c] = y[r, c] - y[r+1, c] for r <= n-2, y[n-1, c] for r = n-1.
"""
import numpy as np


def d1(x):
    return np.roll(x, -1, axis=0) - x


def d2(x):
    return np.roll(x, -1, axis=1) - x


def d1t(y):
    return np.roll(y, 1, axis=0) - y


def d2t(y):
    return np.roll(y, 1, axis=1) - y


def fwd(x):
    """Psi x = [D1 x; D2 x] as one vector of length 2N (D1 rows first)."""
    return np.concatenate([d1(x).ravel(), d2(x).ravel()])


def adj(z, n):
    """Psi^T z for z = [z1; z2]."""
    N = n * n
    return d1t(z[:N].reshape(n, n)) + d2t(z[N:].reshape(n, n))


# -- the paper's non-periodic differences ------------------------------------

def d1p(x):
    y = x.copy()
    y[1:, :] -= x[:-1, :]
    return y


def d2p(x):
    y = x.copy()
    y[:, 1:] -= x[:, :-1]
    return y


def d1pt(y):
    x = y.copy()
    x[:-1, :] -= y[1:, :]
    return x


def d2pt(y):
    x = y.copy()
    x[:, :-1] -= y[:, 1:]
    return x


def fwd_p(x):
    """[D1 x; D2 x] with the paper's matrices (length 2N, D1 rows first)."""
    return np.concatenate([d1p(x).ravel(), d2p(x).ravel()])


def adj_p(z, n):
    N = n * n
    return d1pt(z[:N].reshape(n, n)) + d2pt(z[N:].reshape(n, n))

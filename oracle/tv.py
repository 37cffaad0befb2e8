"""First-order finite differences for TV (Section 4.1), periodic boundary.

(D1 x)[r, c] = x[r+1, c] - x[r, c]  (vertical),
(D2 x)[r, c] = x[r, c+1] - x[r, c]  (horizontal), indices mod n.
The adjoints are (D1^T y)[r, c] = y[r-1, c] - y[r, c] and likewise for D2.
The paper's printed matrices use a non-periodic first row; the periodic
reading is the one the TV workload here fixes.
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

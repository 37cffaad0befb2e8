"""Undersampled Fourier operator of CS-MRI (Section 5.4): A = R F.

F is the unitary 2D DFT (1/n normalisation both ways, DC at [0, 0]), R keeps
the sampled rows of the identity.  Measurements live on the full n x n grid
and are zero off the mask, so R^T R = diag(mask) and A^H A = F^H diag(m) F.
The FFT is numpy's, used as a library primitive; ``dft_matrix`` is the
definition written out, for pins on tiny sizes.
"""
import numpy as np


def fft2u(x):
    return np.fft.fft2(x, norm="ortho")


def ifft2u(y):
    return np.fft.ifft2(y, norm="ortho")


def A(x, mask):
    """A x = m * F x."""
    return mask * fft2u(x)


def AH(y, mask):
    """A^H y = F^H (m * y)."""
    return ifft2u(mask * y)


def AHA(x, mask):
    return AH(A(x, mask), mask)


def dft_matrix(n):
    """Unitary 1D DFT matrix, entry (k, j) = exp(-2 pi i k j / n) / sqrt(n)."""
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def dft2_naive(x):
    """2D unitary DFT by the definition: F_n X F_n^T (F_n symmetric)."""
    Fn = dft_matrix(x.shape[0])
    return Fn @ x @ Fn.T


def rho(mask):
    """Mean of diag(A^H A): every diagonal entry equals M / N for unitary F
    (Section 5.4: the mean diagonal is the sampling ratio)."""
    return float(np.count_nonzero(mask)) / mask.size

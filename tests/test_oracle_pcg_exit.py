"""The oracle's early PCG exit (eta > 0) against brute force.

The PCG stopping criterion of Algorithms 2 and 3 is left open by the paper;
it is read as a relative preconditioned-residual test: stop after the first
iteration j with <r_j, P^{-1} r_j> <= eta^2 <r_0, P^{-1} r_0>.  On a 16 x 16
problem S and P^{-1} are formed as dense matrices by applying the operators
to every unit vector, and the residual of each returned iterate is computed
from scratch (A^H b - S x), independent of the recurrence r -= alpha q the
solver runs: the returned iterate must satisfy the test, the iterate one
step before must not, and the result must be the plain K = j run.
"""
import numpy as np
import pytest

import synth
from oracle.firls import Operators, pcg


def dense(f, n):
    cols = []
    for i in range(n * n):
        e = np.zeros(n * n, dtype=np.complex128)
        e[i] = 1.0
        cols.append(f(e.reshape(n, n)).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("psi,groups,levels", [("haar", "quadtree", 2), ("tv", "tv_iso", 0)])
def test_exit_at_first_small_preconditioned_residual(psi, groups, levels):
    n = 16
    p = synth.make_problem(n, 4, psi=psi, levels=levels, groups=groups, lam=0.05, sigma=0.01, frac=0.3)
    ops = Operators.from_problem(p)
    rs = np.random.default_rng(9)
    xw = rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n))
    _, d = ops.weights(xw)
    S = dense(lambda v: ops.S(v, d), n)
    Pinv = dense(ops.precond(d), n)
    assert np.allclose(S, S.conj().T, atol=1e-12)          # Hermitian
    assert np.allclose(Pinv, Pinv.conj().T, atol=1e-12)
    rhs = ops.AHb().ravel()
    x0 = ops.AHb()

    def rz(x):
        r = rhs - S @ x.ravel()
        return float(np.real(np.vdot(r, Pinv @ r)))

    K = 60
    seen = set()
    for eta in (0.5, 0.1, 1e-2, 1e-3):
        x, it = pcg(ops, d, x0, K, eta=eta)
        assert 1 <= it < K
        seen.add(it)
        assert rz(x) <= eta * eta * rz(x0) * (1 + 1e-9)
        xp, _ = pcg(ops, d, x0, it - 1)
        assert rz(xp) > eta * eta * rz(x0) * (1 - 1e-9)
        xk, itk = pcg(ops, d, x0, it)
        assert itk == it
        np.testing.assert_allclose(x, xk, rtol=0, atol=1e-12 * np.abs(xk).max())
    assert len(seen) >= 3                                    # the thresholds stop at different j


def test_eta_zero_runs_every_iteration():
    p = synth.make_problem(16, 5, psi="haar", levels=2, groups="quadtree", lam=0.05, sigma=0.01, frac=0.3)
    ops = Operators.from_problem(p)
    _, d = ops.weights(ops.AHb())
    _, it = pcg(ops, d, ops.AHb(), 7)
    assert it == 7

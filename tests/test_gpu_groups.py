"""GPU parity of band-local group maps of every padded-list width.

The residual row pass of the Haar path computes the group weights and d of
each row band on chip when every group lies inside one band, reading
padded member and membership lists of width 1, 2, 4 or 8, or the CSR lists
when a group or a coefficient's membership is wider than 8.  Runs of
level-1 horizontal-detail coefficients along one Mallat row all sit in one
pixel row of the in-place layout, so groups made of such runs (everything
else singletons) are band-local for any run length; overlapping runs give
coefficients more than one group.

Bars as in test_gpu_solve: 1e-10 (FP64) and 1e-5 (FP32) relative objective
against the FP64 oracle.
"""
import dataclasses

import numpy as np
import pytest

import synth
from tests.gpu_util import rel
from tests.test_gpu_solve import check

pytestmark = pytest.mark.gpu


def row_run_groups(n, L, width, stride):
    level, band = synth.mallat_level_band(n, L)
    idx = np.arange(n * n).reshape(n, n)
    cols = np.arange(n // 2, n)                       # level 1, band 1: rows [0, n/2), cols [n/2, n)
    assert np.all(level[: n // 2, n // 2:] == 1) and np.all(band[: n // 2, n // 2:] == 1)
    groups, covered = [], np.zeros(n * n, dtype=bool)
    for i in range(n // 2):
        for s in range(0, len(cols) - width + 1, stride):
            g = idx[i, cols[s:s + width]]
            groups.append(g)
            covered[g] = True
    groups += [[j] for j in np.flatnonzero(~covered)]
    ptr = np.zeros(len(groups) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(g) for g in groups])
    return ptr, np.concatenate([np.asarray(g) for g in groups]).astype(np.int32)


@pytest.mark.parametrize("width,stride,prec", [
    (4, 4, "fp32"),     # members 4, memberships 1
    (4, 2, "fp32"),     # members 4, memberships 2
    (8, 2, "fp64"),     # members 8, memberships 4
    (16, 16, "fp32"),   # members 16: CSR lists
    (16, 4, "fp64"),    # members 16, memberships 4: CSR lists
])
def test_band_local_runs(width, stride, prec):
    base = synth.make_problem(64, 6, psi="haar", levels=3, groups="singletons", lam=0.03, sigma=0.01, frac=0.25)
    ptr, idx = row_run_groups(64, 3, width, stride)
    p = dataclasses.replace(base, group_ptr=ptr, group_idx=idx)
    x, rep, ref = check(p, prec, 5, 10)
    assert rep["outer_iters"] == 5
    if prec == "fp64":
        assert rel(x, ref.x) < 1e-8

"""Helpers shared by the GPU tests: tensors from numpy and a solver set-up
from a synthetic problem.  The GPU side is reached only through the C ABI
binding; the oracle only through ``oracle``."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch


def dev_complex(a, prec):
    torch = torch_cuda()
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda().contiguous()


def dev_mask(m):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(m.astype(np.uint8))).cuda().contiguous()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def shape_of(prob):
    from paper_1411_5057_amd import firls as F
    return F.Shape(prob.n, prob.psi, prob.levels, prob.group_ptr, prob.group_idx, getattr(prob, "C", 1),
                   getattr(prob, "Amat", None))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def max_err(a, b):
    """max |a - b| over elements, relative to max |b| (every element is held
    to the bar, not only the norm)."""
    a, b = np.ravel(a), np.ravel(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))

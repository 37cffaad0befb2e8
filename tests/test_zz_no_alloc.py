"""The allocation-free batched solve (firls_solve_batched_noalloc) against
firls_solve_batched: same kernels on the library's fixed per-GPU scratch
instead of allocated workspace, so reports and x must agree bitwise.  Two
calls in a row, the second with a smaller batch (the scratch keeps the
first call's contents, which the second must not depend on), and a batch
too large for the scratch, rejected before any work."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_complex, dev_mask, torch_cuda

pytestmark = pytest.mark.gpu


def _problems():
    haar = [synth.make_problem(128, 400 + i, psi="haar", levels=4, groups="quadtree", lam=0.035 * (1 + i % 2),
                               sigma=0.01, frac=0.2) for i in range(4)]
    tv = [synth.make_problem(64, 410 + i, psi="tv", levels=0, groups="tv_iso", lam=0.02, sigma=0.01, frac=0.3)
          for i in range(2)]
    return haar, tv


def _items(torch, probs_and_ids):
    """(problem, shape id, given start) -> batch items; a given start is the
    zero image (x_is_init), the others start from A^H b."""
    out = []
    for p, sid, init in probs_and_ids:
        b = dev_complex(p.b, "fp32")
        out.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam, shape_id=sid,
                        x_is_init=init))
    return out


def test_noalloc_matches_batched_on_two_calls():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    haar, tv = _problems()
    shapes = [F.Shape(128, "haar", 4, haar[0].group_ptr, haar[0].group_idx), F.Shape(64, "tv", 0)]
    s = F.Solver(shapes, prec="fp32", max_slices=8, max_outer=30, pcg_iters=4, outer_tol=2e-5, eps=haar[0].eps)
    calls = [[(p, 0, False) for p in haar] + [(p, 1, False) for p in tv],   # 6 slices, both shapes
             [(haar[3], 0, False), (tv[1], 1, True), (haar[0], 0, False)]]  # then 3, in another order
    for k, probs in enumerate(calls):
        ref_items = _items(torch, probs)
        ref = s.solve_batched(ref_items)
        got_items = _items(torch, probs)
        got = s.solve_batched_noalloc(got_items)
        assert len({r["outer_iters"] for r in ref}) > 1
        for r, q in zip(got, ref):
            assert r == q, k
            assert r["status"] >= 0
        for a, b in zip(got_items, ref_items):
            assert torch.equal(a["x"], b["x"]), k


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    """20 slices of 256^2 need about 71 MB, more than the 64 MiB scratch:
    the call fails before any work and leaves x untouched; the handle then
    solves normally."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = synth.make_problem(256, 430, psi="haar", levels=4, groups="quadtree", lam=0.035, sigma=0.01, frac=0.2)
    s = F.Solver([F.Shape(256, "haar", 4, p.group_ptr, p.group_idx)], prec="fp32", max_slices=20, max_outer=2,
                 pcg_iters=2, eps=p.eps)
    b = dev_complex(p.b, "fp32")
    m = dev_mask(p.mask)
    xs = [torch.full_like(b, 0.25) for _ in range(20)]
    with pytest.raises(F.FirlsError) as e:
        s.solve_batched_noalloc([dict(b=b, mask=m, x=x, lam=p.lam) for x in xs])
    assert e.value.code == F.FIRLS_E_INVALID and "scratch" in str(e.value)
    assert all(torch.all(x == 0.25) for x in xs)
    few = [dict(b=b, mask=m, x=torch.zeros_like(b), lam=p.lam) for _ in range(2)]
    ref = [dict(b=b, mask=m, x=torch.zeros_like(b), lam=p.lam) for _ in range(2)]
    assert s.solve_batched_noalloc(few) == s.solve_batched(ref)
    assert all(torch.equal(a["x"], c["x"]) for a, c in zip(few, ref))

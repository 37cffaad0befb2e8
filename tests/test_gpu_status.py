"""Per-slice statuses of the solve entry points, each forced from the host
so that every kernel still exits normally:

- FIRLS_E_BREAKDOWN: PCG meets <p, S p> <= 0 with a nonzero residual, which
  cannot happen for the Hermitian positive definite S of eq. (15) / eq. (39)
  (Section 3.2) in exact arithmetic; a test hook makes every <p, S p>
  negative.
- FIRLS_W_NONMONOTONE: F_eps rose between outer iterations, against
  Theorem 2 (Section 3.3); a test hook removes the rounding slack of the
  check, so the warning is raised without changing the arithmetic.
- FIRLS_E_INVALID per slice: a TV slice whose mask leaves out DC (the
  difference operators annihilate constants, so the minimiser would not be
  unique); the other slices of the call are solved as usual.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_complex, dev_mask, shape_of, torch_cuda

pytestmark = pytest.mark.gpu


def _probs(psi, count, seed0):
    if psi == "haar":
        return [synth.make_problem(64, seed0 + i, psi="haar", levels=4, groups="quadtree", lam=0.035,
                                   sigma=0.01, frac=0.2) for i in range(count)]
    return [synth.make_problem(64, seed0 + i, psi="tv", levels=0, groups="tv_iso", lam=0.02, sigma=0.01,
                               frac=0.3) for i in range(count)]


def _items(torch, probs, prec="fp32"):
    out = []
    for p in probs:
        b = dev_complex(p.b, prec)
        out.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam))
    return out


@pytest.mark.parametrize("paired", [True, False])
@pytest.mark.parametrize("psi", ["haar", "tv"])
def test_breakdown_is_reported(psi, paired):
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = _probs(psi, 3, 300)
    s = F.Solver([shape_of(probs[0])], prec="fp32", max_slices=3, max_outer=4, pcg_iters=4, outer_tol=1e-6,
                 eps=probs[0].eps)
    s.set_paired(paired)
    ref = s.solve_batched(_items(torch, probs))
    assert all(r["status"] >= 0 for r in ref)
    s.test_hooks(F.FIRLS_TEST_BREAKDOWN)
    batch = s.prepare(_items(torch, probs))
    with pytest.raises(F.FirlsError) as e:
        s.solve_batched(batch)
    assert e.value.code == F.FIRLS_E_BREAKDOWN
    assert "breakdown" in str(e.value)
    # every slice stops at the outer check after its first PCG run
    assert list(batch.reports["status"]) == [F.FIRLS_E_BREAKDOWN] * 3
    assert list(batch.reports["outer_iters"]) == [1] * 3
    s.test_hooks(0)
    assert s.solve_batched(_items(torch, probs)) == ref


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_nonmonotone_warning_leaves_the_results(prec):
    """The hook only changes the check's verdict: reports carry the warning,
    the call returns it (a warning, not an error), and x is bitwise the same
    as without the hook."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = _probs("haar", 2, 320)
    s = F.Solver([shape_of(probs[0])], prec=prec, max_slices=2, max_outer=5, pcg_iters=4, eps=probs[0].eps)
    a = _items(torch, probs, prec)
    ref = s.solve_batched(a)
    assert all(r["status"] == F.FIRLS_OK for r in ref)
    s.test_hooks(F.FIRLS_TEST_NONMONOTONE)
    b = _items(torch, probs, prec)
    got = s.solve_batched(b)
    for r, q in zip(got, ref):
        assert r["status"] == F.FIRLS_W_NONMONOTONE
        assert {k: v for k, v in r.items() if k != "status"} == {k: v for k, v in q.items() if k != "status"}
    for u, v in zip(a, b):
        assert torch.equal(u["x"], v["x"])


@pytest.mark.parametrize("chunk,bad", [(0, 1), (2, 1), (2, 3)])
def test_tv_mask_without_dc_is_rejected_per_slice(chunk, bad):
    """One slice of 4 has its DC sample removed: it reports FIRLS_E_INVALID
    and keeps its x, the call returns the error, and the other slices'
    reports and x are bitwise those of a batch without it (also with two
    streamed slots, the bad slice starting at once or entering a slot
    later)."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = _probs("tv", 4, 340)
    s = F.Solver([shape_of(probs[0])], prec="fp32", max_slices=4, max_outer=20, pcg_iters=4, outer_tol=1e-3,
                 eps=probs[0].eps)
    s.set_chunk(chunk)
    good = [i for i in range(4) if i != bad]
    ref_items = _items(torch, [probs[i] for i in good])
    ref = s.solve_batched(ref_items)
    items = _items(torch, probs)
    items[bad]["mask"][0, 0] = 0
    items[bad]["x"].fill_(0.5)
    batch = s.prepare(items)
    with pytest.raises(F.FirlsError) as e:
        s.solve_batched(batch)
    assert e.value.code == F.FIRLS_E_INVALID
    assert "DC" in str(e.value)
    reps = F.report_dicts(batch.reports)
    assert reps[bad]["status"] == F.FIRLS_E_INVALID and reps[bad]["outer_iters"] == 0
    assert torch.all(items[bad]["x"] == 0.5)
    for j, i in enumerate(good):
        assert reps[i] == ref[j]
        assert torch.equal(items[i]["x"], ref_items[j]["x"])


def test_haar_mask_without_dc_is_solved():
    """Haar penalises every coefficient, the coarsest approximation
    included, so the minimiser is unique without DC: such a slice is
    solved."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = _probs("haar", 1, 360)[0]
    s = F.Solver([shape_of(p)], prec="fp32", max_slices=1, max_outer=3, pcg_iters=4, eps=p.eps)
    m = p.mask.copy()
    m[0, 0] = 0
    b = dev_complex(p.b * m, "fp32")
    x = torch.zeros_like(b)
    rep = s.solve(b, dev_mask(m), x, p.lam)
    assert rep["status"] == F.FIRLS_OK and rep["outer_iters"] == 3
    assert np.isfinite(rep["F_eps"])

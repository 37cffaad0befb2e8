"""Launches across shapes (FIRLS_SCHED_ACROSS, _LARGEST_FIRST) against
per-shape launches and the FP64 oracle.

A batch mixing image sides and regularisers runs each position of the outer
iteration as one launch per kernel class and mode over all shapes; each
workgroup finds its slice, block and parameters in a work table.  The
per-shape kernel bodies are the same code, so results must match the
per-shape schedule: reports and x compared element by element (to FP32
rounding, MATCH_TOL of max |x|, since the compiler may fuse multiply-adds
differently in the merged kernels), outer iteration counts exactly, and
sampled slices against the oracle at the usual bar.
"""
import numpy as np
import pytest

import synth
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, dev_mask, max_err, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu

MATCH_TOL = {"fp32": 1e-5, "fp64": 1e-12}


def mixed(prec):
    """Haar (tree groups) at sides 64, 96, 128, 192, 256 and 384 (in FP32
    the paired pass with two tile columns per thread, its own kernel across
    shapes; in FP64 the two-launch form) and TV at 64 and 128, two slices
    of some."""
    probs = []
    for i, n in enumerate((64, 96, 128, 192, 256, 384, 64, 128)):
        probs.append(synth.make_problem(n, 600 + i, psi="haar", levels=4, groups="quadtree",
                                        lam=0.02 + 0.005 * i, sigma=0.01, frac=0.22))
    for i, n in enumerate((64, 128, 64)):
        probs.append(synth.make_problem(n, 620 + i, psi="tv", levels=0, groups="tv_iso", lam=0.02,
                                        sigma=0.01, frac=0.3))
    return probs


def setup(prec, T=40, K=4, tau=1e-5):
    from paper_1411_5057_amd import firls as F
    probs = mixed(prec)
    keys, shapes = [], []
    for p in probs:
        k = (p.n, p.psi)
        if k not in keys:
            keys.append(k)
            shapes.append(shape_of(p))
    sid = [keys.index((p.n, p.psi)) for p in probs]
    s = F.Solver(shapes, prec=prec, max_slices=len(probs), max_outer=T, pcg_iters=K, outer_tol=tau,
                 eps=probs[0].eps)
    return s, probs, sid


def items(torch, probs, sid, prec):
    out = []
    for p, k in zip(probs, sid):
        b = dev_complex(p.b, prec)
        out.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam, shape_id=k))
    return out


@pytest.mark.parametrize("paired", [True, False])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_schedules_agree(prec, paired):
    """Every schedule, with graph replay and direct launches, with the
    paired PCG pass on and off, gives the per-shape results."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    s, probs, sid = setup(prec)
    s.set_paired(paired)
    runs = {}
    for sched in (F.FIRLS_SCHED_PER_SHAPE, F.FIRLS_SCHED_ACROSS, F.FIRLS_SCHED_ACROSS_LARGEST_FIRST):
        for graphs in (False, True):
            s.set_schedule(sched)
            s.set_graphs(graphs)
            it = items(torch, probs, sid, prec)
            runs[(sched, graphs)] = (s.solve_batched(it), [to_np(u["x"]) for u in it])
    ref_r, ref_x = runs[(F.FIRLS_SCHED_PER_SHAPE, False)]
    assert len({r["outer_iters"] for r in ref_r}) > 1
    for key, (r, x) in runs.items():
        for a, b, xa, xb in zip(r, ref_r, x, ref_x):
            assert a["status"] == b["status"] and a["outer_iters"] == b["outer_iters"], key
            assert abs(a["F_eps"] - b["F_eps"]) <= MATCH_TOL[prec] * b["F_eps"], key
            assert max_err(xa, xb) <= MATCH_TOL[prec], (key, max_err(xa, xb))
    # the schedules' own replays are bitwise stable
    for sched in (F.FIRLS_SCHED_ACROSS, F.FIRLS_SCHED_ACROSS_LARGEST_FIRST):
        (r1, x1), (r2, x2) = runs[(sched, False)], runs[(sched, True)]
        assert r1 == r2
        assert all(np.array_equal(a, b) for a, b in zip(x1, x2))


def test_across_shapes_against_the_oracle():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    T, K = 6, 10
    s, probs, sid = setup("fp32", T=T, K=K, tau=0.0)
    s.set_schedule(F.FIRLS_SCHED_ACROSS_LARGEST_FIRST)
    it = items(torch, probs, sid, "fp32")
    reps = s.solve_batched(it)
    for i in (2, 5, 9):          # Haar 128 (paired), Haar 384 (paired, two tile columns per thread), TV 128
        ops = Operators.from_problem(probs[i])
        ref = firls(ops, T, K)
        fe = ops.objective(to_np(it[i]["x"]))[0]
        assert reps[i]["outer_iters"] == T
        assert abs(fe - ref.F_eps) <= 1e-5 * ref.F_eps, (i, fe, ref.F_eps)


def test_autotune_considers_the_schedules():
    """The autotuner times the schedules of a mixed batch and keeps one;
    the solve after it matches the per-shape reference."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    s, probs, sid = setup("fp32")
    ref = s.solve_batched(items(torch, probs, sid, "fp32"))
    s.autotune(items(torch, probs, sid, "fp32"))
    assert s.schedule in (F.FIRLS_SCHED_PER_SHAPE, F.FIRLS_SCHED_ACROSS, F.FIRLS_SCHED_ACROSS_LARGEST_FIRST)
    got = s.solve_batched(items(torch, probs, sid, "fp32"))
    for a, b in zip(got, ref):
        assert a["outer_iters"] == b["outer_iters"]
        assert abs(a["F_eps"] - b["F_eps"]) <= 1e-5 * b["F_eps"]

"""A caller-owned workspace (firls_config.workspace, sized by
firls_workspace_bytes(cfg)): the same kernels on the caller's buffer give
bitwise the results of the library's own workspace (also streamed through
fewer slots); a buffer below the size, or misaligned, is refused at
create."""
import pytest

import synth
from tests.gpu_util import dev_complex, dev_mask, shape_of, torch_cuda

pytestmark = pytest.mark.gpu


def _items(torch, probs):
    out = []
    for p in probs:
        b = dev_complex(p.b, "fp32")
        out.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam))
    return out


def test_caller_workspace_matches_library_workspace():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    probs = [synth.make_problem(128, 500 + i, psi="haar", levels=4, groups="quadtree", lam=0.035, sigma=0.01,
                                frac=0.2) for i in range(5)]
    kw = dict(prec="fp32", max_slices=5, max_outer=20, pcg_iters=4, outer_tol=1e-5, eps=probs[0].eps)
    own = F.Solver([shape_of(probs[0])], **kw)
    theirs = F.Solver([shape_of(probs[0])], workspace=True, **kw)
    assert theirs.workspace.numel() == F.firls_workspace_bytes(theirs.cfg)
    a, b = _items(torch, probs), _items(torch, probs)
    assert own.solve_batched(a) == theirs.solve_batched(b)
    assert all(torch.equal(u["x"], v["x"]) for u, v in zip(a, b))
    # streamed through 2 slots: fits the same buffer
    theirs.set_chunk(2)
    c = _items(torch, probs)
    assert theirs.solve_batched(c) == own.solve_batched(_items(torch, probs))


def test_caller_workspace_too_small_is_refused():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    p = synth.make_problem(64, 510, psi="haar", levels=4, groups="quadtree", lam=0.035, sigma=0.01, frac=0.2)
    probe = F.Solver([shape_of(p)], prec="fp32", max_slices=2)
    need = F.firls_workspace_bytes(probe.cfg)
    probe.close()
    with pytest.raises(F.FirlsError) as e:
        F.Solver([shape_of(p)], prec="fp32", max_slices=2,
                 workspace=torch.empty(need - 256, dtype=torch.uint8, device="cuda"))
    assert e.value.code == F.FIRLS_E_INVALID and "workspace" in str(e.value)
    with pytest.raises(F.FirlsError):         # not 256-byte aligned
        buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        F.Solver([shape_of(p)], prec="fp32", max_slices=2, workspace=buf[16:16 + need])

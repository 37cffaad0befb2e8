"""The C-ABI library loads and exports every entry point that
include/firls.h declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "firls.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|int|size_t|const char\*)\s+(firls_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("firls_create", "firls_solve", "firls_solve_batched", "firls_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1411_5057_amd import firls as F
    if not os.path.exists(F.LIB_PATH):
        pytest.fail("libfirls.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(F.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(declared()) == sorted(F.EXPORTED)


def test_binding_has_no_cpu_fallback():
    """The binding never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_1411_5057_amd", "firls.py")).read()
    assert "oracle" not in src


def test_batch_records_match_the_abi_structures():
    """The column-wise batch marshalling writes the same bytes as filling
    the ctypes structures one by one, and report records read back the same
    fields (host memory only: the data pointers are of CPU tensors)."""
    import numpy as np
    import torch
    from paper_1411_5057_amd import firls as F
    b = torch.zeros(3, 16, 16, dtype=torch.complex64)
    m = torch.zeros(3, 16, 16, dtype=torch.uint8)
    x = torch.zeros_like(b)
    items = [dict(b=b[i], mask=m[i] if i != 1 else None, x=x[i], lam=0.01 * (i + 1), shape_id=i % 2,
                  x_is_init=(i == 2)) for i in range(3)]
    want = (F.firls_slice * 3)()
    for i, it in enumerate(items):
        want[i] = F.firls_slice(i % 2, int(i == 2), 0.01 * (i + 1), b[i].data_ptr(),
                                0 if i == 1 else m[i].data_ptr(), x[i].data_ptr())
    got = F.slice_array(items)
    assert got.tobytes() == bytes(want)
    forced = F.slice_array(items, True)
    assert list(forced["x_is_init"]) == [1, 1, 1]
    reps = (F.firls_report * 2)()
    reps[0] = F.firls_report(0, 7, 28, 1, 1.5, 1.25, 0.5, 1e-6)
    reps[1] = F.firls_report(-5, 3, 12, 0, 2.5, 2.25, 1.5, 0.0)
    arr = np.frombuffer(bytes(reps), dtype=F.REPORT_DTYPE)
    assert F.report_dicts(arr) == [r.as_dict() for r in reps]
    batch = F.Batch(items)
    assert len(batch) == 3 and batch.slices.tobytes() == bytes(want)


def test_binding_rejects_buffers_the_kernels_would_misread():
    """Host-side checks of the binding (no GPU needed): wrong dtype, a
    strided view, a wrong element count and a tensor in host memory are
    refused before any pointer reaches the library."""
    import numpy as np
    import torch
    from paper_1411_5057_amd import firls as F
    n = 16
    shapes = [F.Shape(n, "haar", 2), F.Shape(n, "tv", 0, channels=2)]
    ok = dict(b=torch.zeros(n, n, dtype=torch.complex64), mask=torch.ones(n, n, dtype=torch.uint8),
              x=torch.zeros(n, n, dtype=torch.complex64), lam=0.01)

    def bad(**kw):
        it = dict(ok, **kw)
        with pytest.raises((ValueError, TypeError)) as e:
            F.slice_array([it], shapes=shapes, prec="fp32")
        return str(e.value)

    assert "complex64" in bad(b=torch.zeros(n, n, dtype=torch.complex128))
    assert "uint8" in bad(mask=torch.ones(n, n, dtype=torch.bool))
    assert "contiguous" in bad(x=torch.zeros(n, 2 * n, dtype=torch.complex64)[:, ::2])
    assert "elements" in bad(x=torch.zeros(n, n - 1, dtype=torch.complex64))
    assert "elements" in bad(shape_id=1)          # two contrasts need 2 n^2 values
    assert "out of range" in bad(shape_id=2)
    assert "required" in bad(mask=None)           # only a dense sensing matrix may omit it
    assert "torch tensor" in bad(b=np.zeros((n, n), np.complex64))
    assert "GPU" in bad()                          # everything else right, but in host memory
    with pytest.raises(ValueError, match="complex128"):
        F.check_tensor(torch.zeros(4, dtype=torch.complex64), "x", torch.complex128, 4)
    # without shapes the marshalling alone runs (host pointers are fine there)
    assert len(F.slice_array([ok])) == 1


def test_workspace_bytes_from_the_configuration():
    """firls_workspace_bytes(cfg) needs no device: max_slices times the
    largest per-slice workspace.  For a 256^2 FP32 Haar slice with 65536
    groups: r, p, q, t (4 x 512 KiB), d and |Psi x|^2 (2 x 256 KiB), W
    (256 KiB), the packed mask (8 KiB) and 197 x 512 FP64 partial sums."""
    from paper_1411_5057_amd import firls as F
    import synth
    p = synth.make_problem(256, 0, psi="haar", levels=4, groups="quadtree", lam=0.035, sigma=0.01, frac=0.2)
    shapes = [F.Shape(64, "tv", 0), F.Shape(256, "haar", 4, p.group_ptr, p.group_idx)]
    cs = (F.firls_shape * 2)(*[s.c() for s in shapes])
    cfg = F.firls_config()
    cfg.n_shapes, cfg.shapes, cfg.max_slices, cfg.prec = 2, cs, 3, F.FIRLS_FP32
    per = 4 * 524288 + 2 * 262144 + 4 * 65536 + 8192 + 197 * 512 * 8
    assert len(p.group_ptr) - 1 == 65536
    assert F.firls_workspace_bytes(cfg) == 3 * per
    cfg.prec = F.FIRLS_FP64
    assert F.firls_workspace_bytes(cfg) == 3 * (4 * 2 * 524288 + 2 * 524288 + 8 * 65536 + 8192 + 197 * 512 * 8)
    cfg.max_slices = 0
    assert F.firls_workspace_bytes(cfg) == 0


def test_create_validates_the_configuration_before_any_device_call():
    """Out-of-range settings are rejected by firls_create itself with
    FIRLS_E_INVALID and a message, before it touches a device (so this runs
    without one): pcg_rtol must lie in [0, 1), pcg_iters in 1..64, eps > 0."""
    import ctypes
    from paper_1411_5057_amd import firls as F
    shapes = (F.firls_shape * 1)(F.Shape(64, "haar", 3).c())

    def create(**kw):
        cfg = F.firls_config()
        cfg.n_shapes, cfg.shapes, cfg.max_slices, cfg.prec = 1, shapes, 1, F.FIRLS_FP32
        cfg.eps, cfg.max_outer, cfg.pcg_iters = 1e-10, 5, 10
        for k, v in kw.items():
            setattr(cfg, k, v)
        h = ctypes.c_void_p()
        rc = F.load().firls_create(ctypes.byref(cfg), ctypes.byref(h))
        assert not h.value
        return rc, F.load().firls_last_error().decode()

    for bad in (-0.1, 1.0, 2.0, float("nan")):
        rc, msg = create(pcg_rtol=bad)
        assert rc == F.FIRLS_E_INVALID and "pcg_rtol" in msg, (bad, rc, msg)
    rc, msg = create(pcg_iters=65)
    assert rc == F.FIRLS_E_INVALID and "pcg_iters" in msg
    rc, msg = create(eps=0.0)
    assert rc == F.FIRLS_E_INVALID and "eps" in msg

"""GPU parity at the 256^2 benchmark workload, in the configuration the
benchmark times, against the FP64 oracle and the oracle-written optima in
tests/golden/optima_256.json (tests/golden/make_golden.py):

- the operating point: 4 PCG iterations per outer iteration, stop at a
  relative F_eps decrease of 8e-6 (at most 50), 64 streamed slots with
  slices entering slots as others stop, the paired PCG pass, direct
  launches;
- the learned warm start with the shipped network parameters: network
  output against the oracle's bfloat16-emulating network, then the whole
  learned solve against the oracle run from the same start;
- network gradients at 256^2.

The stop rule is a floating-point decision on an integer (how many outer
iterations), taken in FP32 vectors with FP64 sums on the GPU and in FP64 in
the oracle; when the two counts agree the objectives must agree to 1e-5
(the FP32 bar) and x to X_TOL of its largest entry at every pixel, and
either way each result must be within 1e-4 of the optimum.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import cnn, fourier
from oracle.firls import Operators, firls
from tests.gpu_util import dev_complex, dev_mask, rel, shape_of, to_np, torch_cuda

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(os.path.dirname(HERE), "paper_1411_5057_amd", "weights", "warmstart_256.f32")
K, TAU, TMAX, SLOTS = 4, 8e-6, 50, 64
X_TOL = 2e-4     # per pixel, of max |x|: FP32 vectors after ~100 PCG steps


def optima():
    with open(os.path.join(HERE, "golden", "optima_256.json")) as f:
        return {r["seed"]: r["F_eps"] for r in json.load(f)["optima"]}


def compare(ops, seed, x_gpu, rep, start=None, obj_tol=1e-5, x_tol=X_TOL):
    """One GPU result against the oracle run from the same start with the
    same K, tau and cap, and against the stored optimum."""
    ref = firls(ops, TMAX, K, tau=TAU, x1=start)
    fe = ops.objective(x_gpu)[0]
    fstar = optima()[seed]
    xerr = float(np.max(np.abs(x_gpu - ref.x)) / np.max(np.abs(ref.x)))
    print(f"seed {seed}: outer gpu {rep['outer_iters']} oracle {ref.outer_iters}; F_eps rel. diff "
          f"{abs(fe - ref.F_eps) / ref.F_eps:.2e}; gaps to optimum gpu {(fe - fstar) / fstar:.2e} oracle "
          f"{(ref.F_eps - fstar) / fstar:.2e}; max |dx| / max |x| {xerr:.2e}")
    assert abs(rep["F_eps"] - fe) <= 1e-5 * fe           # the GPU's own objective of its x
    assert fe >= fstar * (1 - 1e-9), (seed, fe, fstar)    # nothing beats the optimum
    assert (fe - fstar) / fstar <= 1e-4, (seed, fe, fstar)
    assert (ref.F_eps - fstar) / fstar <= 1e-4
    if rep["outer_iters"] == ref.outer_iters:
        assert abs(fe - ref.F_eps) <= obj_tol * ref.F_eps, (seed, fe, ref.F_eps)
        if x_tol is not None:
            assert xerr <= x_tol, (seed, xerr)
    else:
        assert abs(rep["outer_iters"] - ref.outer_iters) <= 1, (rep["outer_iters"], ref.outer_iters)
    return ref


def test_operating_point_streamed_slots():
    """72 slices through 64 slots: seeds 16-71 and 0-7 start at once, seeds
    8-15 enter slots as others stop.  Sampled: two of each kind."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    order = list(range(16, 72)) + list(range(16))
    probs = {s: synth.cfg1(s) for s in order}
    p0 = probs[0]
    s = F.Solver([shape_of(p0)], prec="fp32", max_slices=len(order), max_outer=TMAX, pcg_iters=K, outer_tol=TAU,
                 eps=p0.eps)
    s.set_chunk(SLOTS)
    s.set_graphs(False)
    s.set_paired(True)
    items = []
    for sd in order:
        b = dev_complex(probs[sd].b, "fp32")
        items.append(dict(b=b, mask=dev_mask(probs[sd].mask), x=torch.zeros_like(b), lam=probs[sd].lam))
    reps = s.solve_batched(items)
    assert all(r["status"] >= 0 and r["converged"] == 1 for r in reps)
    for sd in (0, 1, 14, 15):
        i = order.index(sd)
        compare(Operators.from_problem(probs[sd]), sd, to_np(items[i]["x"]), reps[i])


def test_network_output_with_shipped_weights():
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    flat = np.fromfile(WEIGHTS, dtype="<f4")
    params = F.unflatten_params(flat)
    zf = np.stack([Operators.from_problem(synth.cfg1(sd)).AHb() for sd in (20000, 20001)])
    zt = dev_complex(zf, "fp32")
    net = F.Net(256, 2, flat)
    x0 = torch.empty_like(zt)
    net.forward(zt, x0)
    zfr = to_np(zt)
    ref, _ = cnn.forward(params, zfr, bf16_mode=True)
    got = to_np(x0) - zfr
    assert rel(got, ref - zfr) < 1e-3
    assert np.max(np.abs(got - (ref - zfr))) < 2e-2 * np.max(np.abs(ref - zfr))


def test_learned_solve_with_shipped_weights():
    """The learned start (network, measured samples put back, the better of
    it and A^H b by F_eps) and FIRLS from there, on two fresh seeds."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    flat = np.fromfile(WEIGHTS, dtype="<f4")
    params = F.unflatten_params(flat)
    seeds = (20000, 20001)
    probs = [synth.cfg1(sd) for sd in seeds]
    s = F.Solver([shape_of(probs[0])], prec="fp32", max_slices=2, max_outer=TMAX, pcg_iters=K, outer_tol=TAU,
                 eps=probs[0].eps)
    s.set_graphs(False)
    net = F.Net(256, 2, flat)
    items = []
    for p in probs:
        b = dev_complex(p.b, "fp32")
        items.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam))
    reps, used = s.solve_batched_learned(net, items)
    for sd, p, it, rep, u in zip(seeds, probs, items, reps, used):
        ops = Operators.from_problem(p)
        zf = ops.AHb()
        zfr = to_np(dev_complex(zf, "fp32"))
        x0, _ = cnn.forward(params, zfr[None], bf16_mode=True)
        x0 = fourier.ifft2u(ops.b + (1.0 - ops.mask) * fourier.fft2u(x0[0]))
        keep = ops.objective(x0)[0] <= ops.objective(zf)[0]
        assert u == int(keep)
        # the GPU forms A^H b in FP32 and rounds it to bfloat16 for the
        # network, so its start differs from the oracle's by bfloat16
        # roundings: x is compared through the objective only
        compare(ops, sd, to_np(it["x"]), rep, start=x0 if keep else zf, obj_tol=2e-5, x_tol=None)


def test_network_gradients_256():
    """Loss and weight gradients of the network at 256^2, batch 2, against
    the oracle's backward pass (bfloat16 emulation)."""
    from paper_1411_5057_amd import firls as F
    flat = np.fromfile(WEIGHTS, dtype="<f4")
    params = F.unflatten_params(flat)
    ops = [Operators.from_problem(synth.cfg1(sd)) for sd in (20002, 20003)]
    zf = np.stack([o.AHb() for o in ops])
    rs = np.random.default_rng(21)
    label = zf + 0.05 * (rs.standard_normal(zf.shape) + 1j * rs.standard_normal(zf.shape))
    net = F.Net(256, 2, flat)
    zt, lt = dev_complex(zf, "fp32"), dev_complex(label, "fp32")
    g, loss = net.gradients(zt, lt)
    zfr, lr_ = to_np(zt), to_np(lt)
    x0, cache = cnn.forward(params, zfr, bf16_mode=True)
    ref_loss = cnn.loss(x0, lr_)
    grads = cnn.backward(cache, cnn.loss_grad(x0, lr_))
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    gg = F.unflatten_params(g)
    for layer in range(5):
        assert rel(gg[layer][0], grads[layer][0]) < 1e-2, layer
        assert rel(gg[layer][1], grads[layer][1]) < 1e-2, layer


def test_trained_network_saves_outer_iterations():
    """What the trained network gains over the method without it: 32 fresh
    seeds (20000-20031, disjoint from the training and validation seeds
    30000-34255) solved at the benchmark setting from the learned start and
    from A^H b.  Every result is within 1e-4 of the optimum where it is
    stored (seeds 20000-20015), and the learned start needs fewer outer
    iterations on average."""
    torch = torch_cuda()
    from paper_1411_5057_amd import firls as F
    seeds = list(range(20000, 20032))
    probs = [synth.cfg1(sd) for sd in seeds]
    s = F.Solver([shape_of(probs[0])], prec="fp32", max_slices=len(seeds), max_outer=TMAX, pcg_iters=K,
                 outer_tol=TAU, eps=probs[0].eps)
    net = F.Net(256, len(seeds), np.fromfile(WEIGHTS, dtype="<f4"))

    def items():
        out = []
        for p in probs:
            b = dev_complex(p.b, "fp32")
            out.append(dict(b=b, mask=dev_mask(p.mask), x=torch.zeros_like(b), lam=p.lam))
        return out

    plain = s.solve_batched(items())
    learned, used = s.solve_batched_learned(net, items())
    fstar = optima()
    for sd, a, b in zip(seeds, plain, learned):
        if sd in fstar:
            assert (a["F_eps"] - fstar[sd]) / fstar[sd] <= 1e-4
            assert (b["F_eps"] - fstar[sd]) / fstar[sd] <= 1e-4
    op = np.mean([r["outer_iters"] for r in plain])
    ol = np.mean([r["outer_iters"] for r in learned])
    print(f"mean outer iterations: plain {op:.2f}, learned {ol:.2f} (kept {np.mean(used):.2f})")
    assert ol < op

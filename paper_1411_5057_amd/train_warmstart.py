"""Train the warm-start network on FIRLS solutions computed by this library.

Data: tree-group 256^2 problems (20% VD mask, sigma 0.01, 4-level Haar,
quadtree-pair groups, lambda 0.035) on seeds [seed0, seed0 + n_train) plus a
validation set; inputs are the zero-filled images A^H b, labels the FIRLS
solutions run to a tight tolerance.  The default loss is the squared error
on the k-space entries the solve-time data-consistency step keeps from the
network (the unsampled ones).  Training runs the library's own
forward, backward and Adam kernels (firls_cnn_train_step).  Writes the
float32 parameters (firls ABI order) and a JSON record next to them.

    python -m paper_1411_5057_amd.train_warmstart --out paper_1411_5057_amd/weights/warmstart_256
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, last layer scaled by 0.1 (the start is
    then close to A^H b); float32 in the ABI's parameter order."""
    rs = np.random.default_rng(np.random.SeedSequence([int(seed), 29]))
    ch = (2, 32, 32, 32, 32, 2)
    parts = []
    for i in range(5):
        W = rs.standard_normal((3, 3, ch[i], ch[i + 1])) * math.sqrt(2.0 / (9 * ch[i]))
        if i == 4:
            W *= 0.1
        parts += [W.ravel(), np.zeros(ch[i + 1])]
    return np.concatenate(parts).astype(np.float32)


def _gen(seed: int):
    import synth
    p = synth.cfg1(seed)
    return p.b.astype(np.complex64), p.mask, p.lam


def generate(seeds, workers: int):
    with ProcessPoolExecutor(workers) as ex:
        out = list(ex.map(_gen, seeds, chunksize=16))
    b = np.stack([o[0] for o in out])
    m = np.stack([o[1] for o in out])
    lam = [o[2] for o in out]
    return b, m, lam


def solve_all(F, torch, shape, b, m, lam, *, max_outer, tau, chunk=256):
    """x = FIRLS solutions (max_outer = 0 gives A^H b)."""
    x = torch.zeros_like(b)
    s = F.Solver([shape], prec="fp32", max_slices=chunk, max_outer=max_outer, pcg_iters=20,
                 outer_tol=tau, eps=1e-10)
    reps = []
    for c in range(0, b.shape[0], chunk):
        items = [dict(b=b[i], mask=m[i], x=x[i], lam=lam[i]) for i in range(c, min(c + chunk, b.shape[0]))]
        reps += s.solve_batched(items)
    s.close()
    return x, reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4000)
    ap.add_argument("--val", type=int, default=256)
    ap.add_argument("--seed0", type=int, default=30000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--label-tau", type=float, default=1e-7)
    ap.add_argument("--label-outer", type=int, default=200)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 4))
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "warmstart_256"))
    ap.add_argument("--loss", choices=("image", "dc"), default="dc",
                    help="image: squared error to the FIRLS solution; dc: the same on the k-space entries the "
                         "data-consistency step keeps from the network (the unsampled ones)")
    a = ap.parse_args()

    import torch
    import synth
    from paper_1411_5057_amd import firls as F

    t0 = time.time()
    seeds = list(range(a.seed0, a.seed0 + a.train + a.val))
    b_np, m_np, lam = generate(seeds, a.workers)
    print(f"generated {len(seeds)} problems in {time.time() - t0:.1f} s", flush=True)
    b = torch.from_numpy(b_np).cuda()
    m = torch.from_numpy(m_np).cuda()
    p0 = synth.cfg1(a.seed0)
    shape = F.Shape(256, "haar", 4, p0.group_ptr, p0.group_idx)
    t1 = time.time()
    zf, _ = solve_all(F, torch, shape, b, m, lam, max_outer=0, tau=0.0)
    label, reps = solve_all(F, torch, shape, b, m, lam, max_outer=a.label_outer, tau=a.label_tau)
    torch.cuda.synchronize()
    outer = np.array([r["outer_iters"] for r in reps])
    print(f"labels: {len(reps)} FIRLS solves in {time.time() - t1:.1f} s, outer mean {outer.mean():.1f} "
          f"max {outer.max()}", flush=True)
    del b

    net = F.Net(256, a.batch, he_init(a.init_seed))
    # With the data-consistency loss the target of a batch is
    # x* + A^H A (x0 - x*), x0 the network's current output: the squared
    # error to it is ||(I - A^H A)(x0 - x*)||^2 = ||(1 - m) F (x0 - x*)||^2 / N,
    # the error on the unsampled entries only (A^H A by the library's
    # operator with a vanishing regulariser weight).
    op = F.Solver([shape], prec="fp32", max_slices=1, eps=1e-10) if a.loss == "dc" else None
    zero = torch.zeros(256, 256, dtype=torch.complex64, device="cuda")
    x0b = torch.empty(a.batch, 256, 256, dtype=torch.complex64, device="cuda")
    qb = torch.empty_like(x0b)

    def target(idx_or_slice, zfb, lab):
        if op is None:
            return lab
        nb = zfb.shape[0]
        net.forward(zfb, x0b[:nb])
        r = (x0b[:nb] - lab).contiguous()
        mb = m[idx_or_slice]
        for i in range(nb):
            op.system(mb[i], 1e-30, zero, r[i], qb[i])
        return (lab + qb[:nb]).contiguous()
    rs = np.random.default_rng(a.init_seed)
    ntr = a.train
    steps_per_epoch = ntr // a.batch
    total = steps_per_epoch * a.epochs
    history = []
    step = 0
    t2 = time.time()

    def val_loss():
        losses = []
        for c in range(ntr, ntr + a.val, a.batch):
            e = min(c + a.batch, ntr + a.val)
            _, l = net.gradients(zf[c:e], target(slice(c, e), zf[c:e], label[c:e]))
            losses.append(l * (e - c))
        return float(np.sum(losses) / a.val)

    base = val_loss()
    print(f"initial validation loss {base:.4e}", flush=True)
    for ep in range(a.epochs):
        perm = rs.permutation(ntr)
        tot = 0.0
        for k in range(steps_per_epoch):
            idx = torch.from_numpy(np.sort(perm[k * a.batch:(k + 1) * a.batch])).cuda()
            lr = a.lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            zfb = zf.index_select(0, idx).contiguous()
            tot += net.train_step(zfb, target(idx, zfb, label.index_select(0, idx).contiguous()), lr)
            step += 1
        vl = val_loss()
        history.append({"epoch": ep + 1, "train_loss": tot / steps_per_epoch, "val_loss": vl})
        print(f"epoch {ep + 1}: train {tot / steps_per_epoch:.4e} val {vl:.4e} ({time.time() - t2:.1f} s)", flush=True)
    params = net.get_params()
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    params.astype("<f4").tofile(a.out + ".f32")
    rec = {"image": 256, "workload": "tree-group 256^2, 20% VD, sigma 0.01, L=4, lambda 0.035",
           "train_seeds": [a.seed0, a.seed0 + a.train], "val_seeds": [a.seed0 + a.train, a.seed0 + a.train + a.val],
           "labels": {"pcg_iters": 20, "outer_tol": a.label_tau, "max_outer": a.label_outer},
           "batch": a.batch, "epochs": a.epochs, "lr": a.lr, "schedule": "cosine", "loss": a.loss,
           "initial_val_loss": base, "history": history, "seconds": time.time() - t0}
    with open(a.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"final_val_loss": history[-1]["val_loss"], "initial_val_loss": base}), flush=True)


if __name__ == "__main__":
    main()

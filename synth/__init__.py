"""Seeded synthetic inputs for the FIRLS CS-MRI problems.

This module draws the problem inputs that both the CPU oracle and the GPU
library consume: phantom images, k-space sampling masks, measurement noise,
the measured k-space data b, and group maps G given as CSR lists over the
rows of the sparsifying transform.  It holds none of the reconstruction
method: no wavelet, no finite difference, no reweighting, no solver.

The measurement b is simulated as a scanner would record it, by a library
FFT (numpy, unitary, DC at index [0, 0]) of the phantom plus complex noise on
the sampled entries.  Any b is a valid input of the reconstruction problem,
so nothing in a parity check depends on how b was produced.

Random streams: numpy ``default_rng(SeedSequence([seed, stream]))`` with
stream 0 = phantom, 1 = mask, 2 = noise, 3 = per-slice parameters.

Problem statement followed (Sections 5.4 and 5.5.1, CS-MRI): A = R F with F the 2D
Fourier transform and R a selection of M rows of the identity; more samples
are drawn at low frequency than at high frequency; the sampling ratio is
M / N.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "rng", "phantom", "vd_mask", "radial_mask", "noise", "measure",
    "mallat_level_band", "groups_singletons", "groups_quadtree_pairs",
    "groups_tv_iso", "groups_tv_aniso", "groups_joint", "groups_jtv",
    "Problem", "make_problem", "make_mc_problem", "make_dense_problem", "cfg0", "cfg1", "cfg2",
    "cfg3_set", "CFG3_SIZES",
]

PHANTOM, MASK, NOISE, PARAMS, CONTRAST, SENSING = 0, 1, 2, 3, 4, 5


def rng(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    """Stream ``stream`` of ``seed``; ``sub`` > 0 selects one of several
    independent sub-streams (the channels of a multi-contrast problem)."""
    key = [int(seed), int(stream)] if sub == 0 else [int(seed), int(stream), int(sub)]
    return np.random.default_rng(np.random.SeedSequence(key))


def phantom(n: int, n_ellipses: int, seed: int, ramp: bool = False, contrasts: int = 0) -> np.ndarray:
    """Sum of random filled ellipses on an n x n grid (float64, real).

    Pixel centres lie in (-1, 1)^2; ellipse centres U[-0.7, 0.7]^2, semi-axes
    U[0.05, 0.45], rotation U[0, pi), intensity U[0, 1].  With ``ramp`` a
    seeded linear ramp alpha*u + beta*v, alpha, beta ~ U[-0.25, 0.25], is added.
    With ``contrasts`` = C > 0 the result is C images of the same anatomy
    (the same ellipses) in C contrasts: ellipse e has intensity U[0, 1] drawn
    per contrast from that contrast's own stream (shape (C, n, n)).
    """
    g = rng(seed, PHANTOM)
    c = -1.0 + (2.0 * np.arange(n) + 1.0) / n
    v, u = np.meshgrid(c, c, indexing="ij")      # v: row coordinate, u: column
    C = max(contrasts, 1)
    img = np.zeros((C, n, n), dtype=np.float64)
    amps = [rng(seed, CONTRAST, ch + 1) for ch in range(C)] if contrasts else None
    for _ in range(n_ellipses):
        cx, cy = g.uniform(-0.7, 0.7, size=2)
        a, b = g.uniform(0.05, 0.45, size=2)
        th = g.uniform(0.0, math.pi)
        amp = g.uniform(0.0, 1.0)
        du, dv = u - cx, v - cy
        up = du * math.cos(th) + dv * math.sin(th)
        vp = -du * math.sin(th) + dv * math.cos(th)
        inside = (up / a) ** 2 + (vp / b) ** 2 <= 1.0
        for ch in range(C):
            img[ch] += (amps[ch].uniform(0.0, 1.0) if contrasts else amp) * inside
    if ramp:
        al, be = g.uniform(-0.25, 0.25, size=2)
        img += al * u + be * v
    return img if contrasts else img[0]


def _centred_k(n: int) -> Tuple[np.ndarray, np.ndarray]:
    k = np.arange(n) - n // 2
    return np.meshgrid(k, k, indexing="ij")


def vd_mask(n: int, frac: float, seed: int, sub: int = 0) -> np.ndarray:
    """Variable-density random k-space mask (uint8, unshifted: DC at [0, 0]).

    Exactly M = round(frac * n^2) entries are drawn without replacement with
    probability proportional to (1 - |k| / kmax)^2, kmax = n / sqrt(2), on
    centred integer frequencies k in [-n/2, n/2)^2.  DC is always kept.
    ``sub`` > 0 draws an independent mask (one per contrast).
    """
    g = rng(seed, MASK, sub)
    ky, kx = _centred_k(n)
    rad = np.sqrt(kx.astype(np.float64) ** 2 + ky.astype(np.float64) ** 2)
    w = (1.0 - rad / (n / math.sqrt(2.0))) ** 2
    N = n * n
    M = int(round(frac * N))
    flat_w = w.ravel().copy()
    dc = (n // 2) * n + (n // 2)
    flat_w[dc] = 0.0
    pick = g.choice(N, size=M - 1, replace=False, p=flat_w / flat_w.sum())
    m = np.zeros(N, dtype=np.uint8)
    m[pick] = 1
    m[dc] = 1
    return np.ascontiguousarray(np.fft.ifftshift(m.reshape(n, n)))


def radial_mask(n: int, coverage: float, seed: int) -> np.ndarray:
    """Radial-like random mask: spokes through DC at angles U[0, pi).

    Each spoke is rasterised at step 0.5 by nearest centred integer frequency;
    spokes are added until at least ``coverage`` of the grid is sampled.
    Returned unshifted (DC at [0, 0]).
    """
    g = rng(seed, MASK)
    m = np.zeros((n, n), dtype=np.uint8)
    N = n * n
    t = np.arange(-n, n + 0.5, 0.5)
    while m.sum() < coverage * N:
        th = g.uniform(0.0, math.pi)
        kx = np.rint(t * math.cos(th)).astype(np.int64)
        ky = np.rint(t * math.sin(th)).astype(np.int64)
        ok = (kx >= -n // 2) & (kx < n // 2) & (ky >= -n // 2) & (ky < n // 2)
        m[ky[ok] + n // 2, kx[ok] + n // 2] = 1
    m[n // 2, n // 2] = 1
    return np.ascontiguousarray(np.fft.ifftshift(m))


def noise(n: int, sigma: float, seed: int, sub: int = 0) -> np.ndarray:
    """Complex Gaussian noise sigma * (g1 + i g2), g ~ N(0, 1) (complex128)."""
    g = rng(seed, NOISE, sub)
    return sigma * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))


def measure(img: np.ndarray, mask: np.ndarray, nz: np.ndarray) -> np.ndarray:
    """Simulated acquisition: mask * (unitary FFT(img) + noise), complex128."""
    k = np.fft.fft2(img, norm="ortho")
    return (mask.astype(np.float64) * (k + nz)).astype(np.complex128)


# ---------------------------------------------------------------------------
# Group maps (G as CSR lists of transform-row indices; Section 3.1, Fig. 1)
# ---------------------------------------------------------------------------

def mallat_level_band(n: int, L: int):
    """Per Mallat position (row-major, n x n): (level, band) arrays.

    level 1..L for detail coefficients, band 1 = [0,h)x[h,2h), 2 = [h,2h)x[0,h),
    3 = [h,2h)^2 with h = n / 2^level; the coarsest approximation has level L
    and band 0.  Pure index bookkeeping of the coefficient layout.
    """
    r = np.arange(n)[:, None] * np.ones((1, n), dtype=np.int64)
    c = np.ones((n, 1), dtype=np.int64) * np.arange(n)[None, :]
    level = np.zeros((n, n), dtype=np.int64)
    band = np.zeros((n, n), dtype=np.int64)
    for lev in range(1, L + 1):
        h = n >> lev
        sel = (np.maximum(r, c) >= h) & (np.maximum(r, c) < 2 * h)
        level[sel] = lev
        band[sel & (r < h)] = 1
        band[sel & (r >= h) & (c < h)] = 2
        band[sel & (r >= h) & (c >= h)] = 3
    h = n >> L
    ll = (r < h) & (c < h)
    level[ll] = L
    band[ll] = 0
    return level, band


def groups_singletons(count: int):
    """Standard sparsity: G = I (Fig. 1(a))."""
    return np.arange(count + 1, dtype=np.int32), np.arange(count, dtype=np.int32)


def groups_quadtree_pairs(n: int, L: int):
    """Wavelet tree groups: each coefficient c owns the group {c, parent(c)}.

    A detail coefficient at level < L is paired with its quadtree parent at
    Mallat position (floor(r/2), floor(c/2)); the coarsest approximation and
    the level-L details form singleton groups.  Groups overlap: a parent is
    replicated into its children's groups through G (Section 3.1).
    """
    level, band = mallat_level_band(n, L)
    N = n * n
    j = np.arange(N, dtype=np.int64)
    has_parent = (band.ravel() != 0) & (level.ravel() < L)
    r, c = j // n, j % n
    parent = (r // 2) * n + (c // 2)
    ptr = np.zeros(N + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(1 + has_parent)
    idx = np.empty(int(ptr[-1]), dtype=np.int64)
    idx[ptr[:-1]] = j
    idx[ptr[:-1][has_parent] + 1] = parent[has_parent]
    return ptr.astype(np.int32), idx.astype(np.int32)


def groups_tv_iso(n: int):
    """Isotropic TV: group p = {row p of D1, row p of D2} (rows N + p)."""
    N = n * n
    ptr = np.arange(0, 2 * N + 1, 2, dtype=np.int32)
    idx = np.empty(2 * N, dtype=np.int32)
    idx[0::2] = np.arange(N)
    idx[1::2] = N + np.arange(N)
    return ptr, idx


def groups_tv_aniso(n: int):
    """Anisotropic TV: every difference is its own group."""
    return groups_singletons(2 * n * n)


def groups_joint(n: int, C: int):
    """Joint sparsity across C contrasts (non-overlapping, FIRLS_MT): group j
    holds coefficient j of every contrast, indices c * N + j."""
    N = n * n
    ptr = np.arange(0, C * N + 1, C, dtype=np.int64)
    idx = (np.arange(C)[None, :] * N + np.arange(N)[:, None]).ravel()
    return ptr.astype(np.int32), idx.astype(np.int32)


def groups_jtv(n: int, C: int):
    """Joint TV across C contrasts (FIRLS_JTV): group p holds row p of D1 and
    of D2 of every contrast; rows are numbered D1 of contrast c at c*N + p,
    D2 of contrast c at C*N + c*N + p."""
    N = n * n
    ptr = np.arange(0, 2 * C * N + 1, 2 * C, dtype=np.int64)
    ch = np.arange(C)[None, :] * N + np.arange(N)[:, None]
    idx = np.concatenate([ch, C * N + ch], axis=1).ravel()
    return ptr.astype(np.int32), idx.astype(np.int32)


# ---------------------------------------------------------------------------
# Problem bundles for the workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One reconstruction problem.  With C > 1 contrasts, mask, b and truth
    are (C, n, n) and the transform rows of contrast c come in blocks (Haar:
    c*N + j; TV: D1 rows of all contrasts, then D2 rows)."""
    n: int
    psi: str                     # "haar", "tv" (periodic) or "tvp" (the paper's D)
    levels: int                  # Haar levels (0 for TV)
    lam: float
    eps: float
    mask: np.ndarray             # uint8 n x n, unshifted
    b: np.ndarray                # complex128 n x n, zero off-mask
    truth: np.ndarray            # float64 n x n phantom
    group_ptr: np.ndarray        # int32 [s+1]
    group_idx: np.ndarray        # int32 [N']
    seed: int
    name: str = ""
    C: int = 1
    Amat: Optional[np.ndarray] = None   # dense sensing matrix (M x N); b then has M entries

    @property
    def rho(self) -> float:
        return float(self.mask.sum()) / float(self.mask.size)


_GROUP_CACHE: dict = {}


def _groups(kind: str, n: int, L: int):
    key = (kind, n, L)
    if key not in _GROUP_CACHE:
        if kind == "singletons":
            _GROUP_CACHE[key] = groups_singletons(n * n)
        elif kind == "quadtree":
            _GROUP_CACHE[key] = groups_quadtree_pairs(n, L)
        elif kind == "tv_iso":
            _GROUP_CACHE[key] = groups_tv_iso(n)
        elif kind == "tv_aniso":
            _GROUP_CACHE[key] = groups_tv_aniso(n)
        else:
            raise ValueError(kind)
    return _GROUP_CACHE[key]


def make_problem(n: int, seed: int, *, psi: str, levels: int, groups: str,
                 lam: float, sigma: float, n_ellipses: int = 8,
                 mask_kind: str = "vd", frac: float = 0.25, ramp: bool = False,
                 eps: float = 1e-10, name: str = "") -> Problem:
    img = phantom(n, n_ellipses, seed, ramp=ramp)
    if mask_kind == "vd":
        m = vd_mask(n, frac, seed)
    elif mask_kind == "radial":
        m = radial_mask(n, frac, seed)
    elif mask_kind == "full":
        m = np.ones((n, n), dtype=np.uint8)
    else:
        raise ValueError(mask_kind)
    b = measure(img, m, noise(n, sigma, seed))
    ptr, idx = _groups(groups, n, levels)
    return Problem(n=n, psi=psi, levels=levels, lam=lam, eps=eps, mask=m, b=b,
                   truth=img, group_ptr=ptr, group_idx=idx, seed=seed, name=name)


def make_mc_problem(n: int, seed: int, *, C: int, psi: str, levels: int, groups: str,
                    lam: float, sigma: float, n_ellipses: int = 8, frac: float = 0.25,
                    mask_kind: str = "vd", eps: float = 1e-10, name: str = "") -> Problem:
    """Multi-contrast problem (Section 5.6): C images of one anatomy, each
    with its own variable-density mask (same sampling ratio) and noise.
    groups: "joint" (Haar, FIRLS_MT), "jtv" (TV, FIRLS_JTV), or a
    single-contrast map kind applied to every contrast separately."""
    img = phantom(n, n_ellipses, seed, contrasts=C)
    masks, bs = [], []
    for ch in range(C):
        if mask_kind == "vd":
            m = vd_mask(n, frac, seed, sub=ch + 1)
        elif mask_kind == "full":
            m = np.ones((n, n), dtype=np.uint8)
        else:
            raise ValueError(mask_kind)
        masks.append(m)
        bs.append(measure(img[ch], m, noise(n, sigma, seed, sub=ch + 1)))
    if groups == "joint":
        ptr, idx = groups_joint(n, C)
    elif groups == "jtv":
        ptr, idx = groups_jtv(n, C)
    else:
        p1, i1 = _groups(groups, n, levels)
        N, cnt = n * n, (1 if psi == "haar" else 2) * n * n
        ptrs, idxs = [], []
        for ch in range(C):
            ptrs.append(p1[:-1] + ch * len(i1))
            # a contrast's rows: Haar block ch; TV D1 block ch and D2 block ch
            m_idx = i1.astype(np.int64) + ch * N if psi == "haar" else \
                np.where(i1 < N, i1 + ch * N, i1 - N + C * N + ch * N)
            idxs.append(m_idx)
        ptr = np.concatenate(ptrs + [[C * len(i1)]]).astype(np.int32)
        idx = np.concatenate(idxs).astype(np.int32)
        assert cnt * C >= idx.max() + 1
    return Problem(n=n, psi=psi, levels=levels, lam=lam, eps=eps, mask=np.stack(masks),
                   b=np.stack(bs), truth=img, group_ptr=ptr, group_idx=idx, seed=seed,
                   name=name, C=C)


def make_dense_problem(n: int, seed: int, *, m_frac: float, psi: str, levels: int, groups: str,
                       lam: float, sigma: float, n_ellipses: int = 8, eps: float = 1e-10,
                       name: str = "") -> Problem:
    """Random-projection compressive sensing of an n x n image (Section 5.2:
    a 64 x 64 patch measured by a random projection): A is M x N with
    M = round(m_frac N) and i.i.d. N(0, 1/M) entries, b = A x + complex
    noise (sigma per component)."""
    img = phantom(n, n_ellipses, seed)
    N = n * n
    M = int(round(m_frac * N))
    Am = rng(seed, SENSING).standard_normal((M, N)) / math.sqrt(M)
    g = rng(seed, NOISE)
    b = Am @ img.ravel() + sigma * (g.standard_normal(M) + 1j * g.standard_normal(M))
    ptr, idx = _groups(groups, n, levels)
    return Problem(n=n, psi=psi, levels=levels, lam=lam, eps=eps, mask=np.ones((n, n), dtype=np.uint8),
                   b=b.astype(np.complex128), truth=img, group_ptr=ptr, group_idx=idx, seed=seed,
                   name=name, Amat=Am)


def cfg0(seed: int, n: int = 64) -> Problem:
    """Plain FIRLS_L1, FP64: 64^2, 8 ellipses, 25% VD mask, sigma 0.01,
    3-level Haar, singleton groups, lambda 0.035."""
    return make_problem(n, seed, psi="haar", levels=3, groups="singletons",
                        lam=0.035, sigma=0.01, frac=0.25, name="cfg0")


def cfg1(seed: int, n: int = 256) -> Problem:
    """Overlapping-group (tree) FIRLS_OG: 256^2, 8 ellipses, 20% VD mask,
    sigma 0.01, 4-level Haar, quadtree-pair groups, lambda 0.035."""
    return make_problem(n, seed, psi="haar", levels=4, groups="quadtree",
                        lam=0.035, sigma=0.01, frac=0.20, name="cfg1")


def cfg2(seed: int, n: int = 512) -> Problem:
    """FIRLS_TV: 512^2, 40 ellipses plus ramp, 15% radial mask, sigma 0.005,
    periodic forward differences, isotropic TV, lambda 0.01."""
    return make_problem(n, seed, psi="tv", levels=0, groups="tv_iso",
                        lam=0.01, sigma=0.005, n_ellipses=40, mask_kind="radial",
                        frac=0.15, ramp=True, name="cfg2")


CFG3_SIZES = (128, 192, 256, 384, 512)


def cfg3_set(seed: int = 0, count: int = 64, sizes=CFG3_SIZES,
             size_cap: Optional[int] = None) -> List[Problem]:
    """Batched uneven solves: sizes drawn from ``sizes``, masks 15-30% VD,
    sigma and lambda U[0.005, 0.05]; half tree-group Haar (L=4), half
    isotropic TV, assigned by a seeded permutation.  ``size_cap`` shrinks
    every size to at most that value (for quick checks), keeping the mix."""
    g = rng(seed, PARAMS)
    ns = g.choice(np.asarray(sizes), size=count)
    kinds = g.permutation(np.arange(count) % 2)
    fr = g.uniform(0.15, 0.30, size=count)
    sg = g.uniform(0.005, 0.05, size=count)
    lm = g.uniform(0.005, 0.05, size=count)
    out = []
    for i in range(count):
        n = int(ns[i]) if size_cap is None else min(int(ns[i]), size_cap)
        s = 1000 * (seed + 1) + i
        if kinds[i] == 0:
            out.append(make_problem(n, s, psi="haar", levels=4, groups="quadtree",
                                    lam=float(lm[i]), sigma=float(sg[i]),
                                    frac=float(fr[i]), name="cfg3-haar"))
        else:
            out.append(make_problem(n, s, psi="tv", levels=0, groups="tv_iso",
                                    lam=float(lm[i]), sigma=float(sg[i]),
                                    frac=float(fr[i]), name="cfg3-tv"))
    return out

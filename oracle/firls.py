"""FIRLS in plain FP64 NumPy (test infrastructure only).

Problem (Section 1, eq. 3; Section 3.1, eq. 8; Section 4.1, eq. 35):

    min_x  F(x) = 1/2 ||A x - b||^2 + lambda ||Psi x||_{2,1},

with A = R F (Section 5.4), Psi = G Phi (orthonormal Haar, overlapping groups
through G) or Psi = [D1; D2] (isotropic TV).  x is complex: A^T reads A^H and
Psi, being real, acts on real and imaginary parts alike; ||.|| is the complex
modulus.

The smoothing eps of the weights (eq. 12, eq. 37) makes the method an exact
majorise-minimise scheme for the smoothed objective

    F_eps(x) = 1/2 ||A x - b||^2 + lambda sum_i sqrt(||(Psi x)_{g_i}||^2 + eps),

which is what ``objective`` returns first (the unsmoothed F second).

Algorithm 2 (FIRLS_OG) / Algorithm 3 (FIRLS_TV), one outer iteration k:
  1. W^k from x^k (eq. 12 / eq. 37), d = diag(G^T W^k G) (eq. 13 / eq. 38);
  2. S = A^H A + lambda Psi^T diag(d) Psi   (eq. 15 / eq. 39);
  3. P = rho I + lambda Psi^T diag(d) Psi with rho the mean of diag(A^H A)
     (eq. 17 / eq. 40); for Haar P^{-1} = Phi^T (rho I + lambda d)^{-1} Phi
     exactly; for TV P is approximated by triangular factors (eqs. 41-43);
  4. PCG on S x = A^H b started from x^k gives x^{k+1}.
The outer stopping rule is not fixed by the paper; here the loop stops when
the relative decrease of F_eps falls to tau or after T_max solves.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

from . import fourier, groups, haar, tv


def inner(u, v) -> float:
    """Real part of the Hermitian inner product sum conj(u) v.

    For the Hermitian positive definite S and the real symmetric P^{-1} the
    PCG scalars are real, so this is the complex PCG of the normal equations.
    """
    return float(np.real(np.vdot(u.ravel(), v.ravel())))


@dataclasses.dataclass
class Operators:
    n: int
    psi: str
    levels: int
    lam: float
    eps: float
    mask: np.ndarray
    b: np.ndarray
    group_ptr: np.ndarray
    group_idx: np.ndarray
    C: int = 1          # contrasts (Section 5.6); x, mask, b are (C, n, n) when C > 1
    Amat: Optional[np.ndarray] = None   # dense sensing matrix (M x N, real) instead of R F

    @classmethod
    def from_problem(cls, p, eps: Optional[float] = None, lam: Optional[float] = None):
        Am = getattr(p, "Amat", None)
        return cls(n=p.n, psi=p.psi, levels=p.levels,
                   lam=p.lam if lam is None else lam,
                   eps=p.eps if eps is None else eps,
                   mask=None if Am is not None else p.mask.astype(np.float64),
                   b=p.b.copy() if Am is not None else p.mask * p.b,
                   group_ptr=p.group_ptr, group_idx=p.group_idx, C=getattr(p, "C", 1), Amat=Am)

    # -- the measurement operator ---------------------------------------------
    # CS-MRI: A = R F (Section 5.4).  Dense: A is an M x N matrix acting on the
    # row-major image vector (the random projections of Section 5.2 and of the
    # comparison with FOCUSS, Table 1).
    def A(self, x):
        if self.Amat is not None:     # real A: act on real and imaginary parts
            v = np.asarray(x).ravel()
            return self.Amat @ v.real + 1j * (self.Amat @ v.imag)
        return fourier.A(x, self.mask)

    def AH(self, y):
        if self.Amat is not None:
            y = np.asarray(y)
            return (self.Amat.T @ y.real + 1j * (self.Amat.T @ y.imag)).reshape(self.n, self.n)
        return fourier.AH(y, self.mask)

    # -- Psi and its adjoint ------------------------------------------------
    # With C contrasts Psi is block diagonal: Psi x = [Psi x_0; ...; Psi x_{C-1}]
    # for Haar; for TV the D1 rows of all contrasts come first, then the D2
    # rows (so a joint TV group lists 2C rows).
    def _psi_fwd1(self, x):
        if self.psi == "haar":
            return haar.fwd(x, self.levels).ravel()
        if self.psi == "tvp":
            return tv.fwd_p(x)
        return tv.fwd(x)

    def _psi_adj1(self, z):
        if self.psi == "haar":
            return haar.adj(z.reshape(self.n, self.n), self.levels)
        if self.psi == "tvp":
            return tv.adj_p(z, self.n)
        return tv.adj(z, self.n)

    def psi_fwd(self, x):
        if self.C == 1:
            return self._psi_fwd1(x)
        zs = [self._psi_fwd1(x[c]) for c in range(self.C)]
        if self.psi == "haar":
            return np.concatenate(zs)
        N = self.n * self.n
        return np.concatenate([z[:N] for z in zs] + [z[N:] for z in zs])

    def psi_adj(self, z):
        if self.C == 1:
            return self._psi_adj1(z)
        N, C = self.n * self.n, self.C
        if self.psi == "haar":
            return np.stack([self._psi_adj1(z[c * N:(c + 1) * N]) for c in range(C)])
        return np.stack([self._psi_adj1(np.concatenate([z[c * N:(c + 1) * N], z[(C + c) * N:(C + c + 1) * N]]))
                         for c in range(C)])

    def _coef_blocks(self, d):
        """Per-contrast views of a coefficient vector in the single-contrast
        order (the inverse of the block layout above)."""
        N, C = self.n * self.n, self.C
        if self.psi == "haar":
            return [d[c * N:(c + 1) * N] for c in range(C)]
        return [np.concatenate([d[c * N:(c + 1) * N], d[(C + c) * N:(C + c + 1) * N]]) for c in range(C)]

    @property
    def n_coef(self) -> int:
        return self.C * self.n * self.n * (1 if self.psi == "haar" else 2)

    @property
    def rho(self) -> float:
        if self.Amat is not None:        # mean of diag(A^T A)
            return float(np.sum(self.Amat * self.Amat)) / self.Amat.shape[1]
        return fourier.rho(self.mask)

    def AHb(self):
        return self.AH(self.b)

    # -- reweighting ----------------------------------------------------------
    def weights(self, x):
        """(W per group, d = diag(G^T W G) per coefficient)."""
        z = self.psi_fwd(x)
        W = groups.weights(z, self.group_ptr, self.group_idx, self.eps)
        d = groups.replicated_diag(W, self.group_ptr, self.group_idx, self.n_coef)
        return W, d

    # -- objective -----------------------------------------------------------
    def data_term(self, x) -> float:
        r = self.A(x) - self.b
        return 0.5 * float(np.real(np.vdot(r, r)))

    def objective(self, x):
        """(F_eps, F, data term)."""
        data = self.data_term(x)
        pe, p0 = groups.penalty(self.psi_fwd(x), self.group_ptr, self.group_idx, self.eps)
        return data + self.lam * pe, data + self.lam * p0, data

    def Q(self, x, W) -> float:
        """Majoriser of F_eps at the point W came from (eqs. 9-11 with eps):
        sqrt(s + eps) <= ((s + eps) W + 1 / W) / 2, equality at that point."""
        s = groups.group_sq(self.psi_fwd(x), self.group_ptr, self.group_idx)
        return self.data_term(x) + 0.5 * self.lam * float(np.sum((s + self.eps) * W + 1.0 / W))

    # -- system and preconditioners -----------------------------------------
    def S(self, x, d):
        """S x = A^H A x + lambda Psi^T diag(d) Psi x (eq. 15 / eq. 39)."""
        return self.AH(self.A(x)) + self.lam * self.psi_adj(d * self.psi_fwd(x))

    def _tv_bands(self, d):
        """(diagonal a of P = rho I + lambda (D1^T W1 D1 + D2^T W2 D2), W1, W2);
        (C, n, n) arrays for C contrasts."""
        n, C = self.n, self.C
        shp = (n, n) if C == 1 else (C, n, n)
        d1 = d[: C * n * n].reshape(shp)
        d2 = d[C * n * n:].reshape(shp)
        return self.rho + self.lam * self.psi_diag(d), d1, d2

    def _tv_offdiag(self, v, d1, d2):
        """sum_{q != p} P[p, q] v[q] for P of eq. (40).
        Periodic: P[p, p+e1] = -lam d1[p], P[p, p-e1] = -lam d1[p-e1].
        Paper's D: P[p, p-e1] = -lam d1[p] (r >= 1), P[p, p+e1] = -lam d1[p+e1]
        (r <= n-2), the same along columns with d2."""
        lam = self.lam
        if self.psi == "tvp":
            out = np.zeros_like(v)
            out[..., 1:, :] += d1[..., 1:, :] * v[..., :-1, :]
            out[..., :-1, :] += d1[..., 1:, :] * v[..., 1:, :]
            out[..., :, 1:] += d2[..., :, 1:] * v[..., :, :-1]
            out[..., :, :-1] += d2[..., :, 1:] * v[..., :, 1:]
            return -lam * out
        return -lam * (d1 * np.roll(v, -1, axis=-2) + np.roll(d1 * v, 1, axis=-2)
                       + d2 * np.roll(v, -1, axis=-1) + np.roll(d2 * v, 1, axis=-1))

    def precond(self, d, kind: str = "auto") -> Callable:
        """Return r -> P^{-1} r.

        kinds: 'pseudo' (Haar, eq. 17: Phi^T (rho + lambda d)^{-1} Phi),
        'sgs_rb' / 'sgs_lex' (TV: (D+L) D^{-1} (D+U) of eq. 40 in red-black or
        row-major order, the triangular factors of eqs. 42-43), 'jacobi'
        (diag(S)^{-1}), 'none' (plain CG).
        """
        if kind == "auto":
            kind = "pseudo" if self.psi == "haar" else "sgs_rb"
        n, rho, lam = self.n, self.rho, self.lam
        if kind == "none":
            return lambda r: r.copy()
        if kind == "pseudo":
            assert self.psi == "haar"
            if self.C > 1:
                invs = [1.0 / (rho + lam * dc.reshape(n, n)) for dc in self._coef_blocks(d)]
                return lambda r: np.stack([haar.adj(invs[c] * haar.fwd(r[c], self.levels), self.levels)
                                           for c in range(self.C)])
            inv = 1.0 / (rho + lam * d.reshape(n, n))
            return lambda r: haar.adj(inv * haar.fwd(r, self.levels), self.levels)
        if kind == "jacobi":
            dg = rho + lam * self.psi_diag(d)
            return lambda r: r / dg
        assert self.psi in ("tv", "tvp")
        a, d1, d2 = self._tv_bands(d)
        if kind == "sgs_rb":
            ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
            red = ((ii + jj) % 2) == 0
            black = ~red

            def apply(r):
                y = np.where(red, r / a, 0.0)
                y = np.where(black, (r - self._tv_offdiag(y, d1, d2)) / a, y)
                zb = np.where(black, y, 0.0)
                return np.where(red, y - self._tv_offdiag(zb, d1, d2) / a, zb)
            return apply
        if kind == "sgs_lex":
            if self.C > 1:     # P is block diagonal over contrasts
                return lambda r: np.stack([self._sgs_lex(r[c], a[c], d1[c], d2[c]) for c in range(self.C)])
            return lambda r: self._sgs_lex(r, a, d1, d2)
        raise ValueError(kind)

    def tv_neighbours(self, p, d1, d2):
        """[(q, P[p, q])] for the neighbours of pixel p (four periodic ones,
        or those inside the image for the paper's D)."""
        n, lam = self.n, self.lam
        r, c = divmod(p, n)
        if self.psi == "tvp":
            out = []
            if r >= 1:
                out.append(((r - 1) * n + c, -lam * d1[r, c]))
            if r <= n - 2:
                out.append(((r + 1) * n + c, -lam * d1[r + 1, c]))
            if c >= 1:
                out.append((r * n + c - 1, -lam * d2[r, c]))
            if c <= n - 2:
                out.append((r * n + c + 1, -lam * d2[r, c + 1]))
            return out
        return [(((r + 1) % n) * n + c, -lam * d1[r, c]),
                (((r - 1) % n) * n + c, -lam * d1[(r - 1) % n, c]),
                (r * n + (c + 1) % n, -lam * d2[r, c]),
                (r * n + (c - 1) % n, -lam * d2[r, (c - 1) % n])]

    def _sgs_lex(self, rvec, a, d1, d2):
        """Forward then backward Gauss-Seidel sweep in row-major order
        (pure Python loops; small images only)."""
        N = self.n * self.n
        r = rvec.ravel()
        av = a.ravel()
        y = np.zeros(N, dtype=np.complex128)
        for p in range(N):
            acc = r[p]
            for q, v in self.tv_neighbours(p, d1, d2):
                if q < p:
                    acc -= v * y[q]
            y[p] = acc / av[p]
        z = np.zeros(N, dtype=np.complex128)
        for p in range(N - 1, -1, -1):
            acc = av[p] * y[p]
            for q, v in self.tv_neighbours(p, d1, d2):
                if q > p:
                    acc -= v * z[q]
            z[p] = acc / av[p]
        return z.reshape(self.n, self.n)

    def psi_diag(self, d):
        """diag(Psi^T diag(d) Psi) as an n x n array."""
        n = self.n
        if self.C > 1:
            one = dataclasses.replace(self, C=1)
            return np.stack([one.psi_diag(dc) for dc in self._coef_blocks(d)])
        if self.psi in ("tv", "tvp"):
            d1 = d[: n * n].reshape(n, n)
            d2 = d[n * n:].reshape(n, n)
            if self.psi == "tv":
                return d1 + np.roll(d1, 1, axis=0) + d2 + np.roll(d2, 1, axis=1)
            # column j of D1 has +1 at row j and -1 at row j + e1 (if inside)
            out = d1 + d2
            out[:-1, :] += d1[1:, :]
            out[:, :-1] += d2[:, 1:]
            return out
        # Haar: every coefficient reaches a pixel through one chain of 1D
        # steps whose entries are +-1/sqrt(2), so Phi[j, p]^2 is a product of
        # 1/2 factors: apply the inverse transform with (a + d) / 2 to both
        # children.
        x = d.reshape(n, n).astype(np.float64).copy()
        for lev in range(self.levels - 1, -1, -1):
            h = n >> lev
            blk = x[:h, :h]
            t = np.empty_like(blk)
            t[0::2, :] = (blk[: h // 2, :] + blk[h // 2:, :]) / 2.0
            t[1::2, :] = t[0::2, :]
            u = np.empty_like(t)
            u[:, 0::2] = (t[:, : h // 2] + t[:, h // 2:]) / 2.0
            u[:, 1::2] = u[:, 0::2]
            x[:h, :h] = u
        return x


def pcg(ops: Operators, d, x0, K: int, precond: str = "auto", eta: float = 0.0,
        record: Optional[List] = None):
    """Preconditioned CG for S x = A^H b from x0 (Section 3.2; Saad's PCG).

    Runs exactly K iterations, or stops early once <r, z> <= eta^2 <r0, z0>
    when eta > 0.  ``record`` (a list) receives every iterate.
    Returns (x, iterations done).
    """
    Pinv = ops.precond(d, precond)
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = ops.AHb() - ops.S(x, d)
    z = Pinv(r)
    p = z.copy()
    rz = inner(r, z)
    rz0 = rz
    it = 0
    for it in range(1, K + 1):
        q = ops.S(p, d)
        pq = inner(p, q)
        # For HPD S a zero <p, Sp> or <r, z> only occurs once the residual
        # is exactly zero; the step is then zero.
        alpha = rz / pq if pq > 0.0 else 0.0
        x = x + alpha * p
        r = r - alpha * q
        z = Pinv(r)
        rz_new = inner(r, z)
        if record is not None:
            record.append(x.copy())
        if eta > 0.0 and rz_new <= eta * eta * rz0:
            break
        beta = rz_new / rz if rz > 0.0 else 0.0
        rz = rz_new
        p = z + beta * p
    return x, it


@dataclasses.dataclass
class Report:
    x: np.ndarray
    outer_iters: int
    pcg_iters: int
    F_eps: float
    F: float
    history: List[float]
    converged: bool


def firls(ops: Operators, T_max: int, K: int, tau: float = 0.0, x1=None,
          precond: str = "auto", eta: float = 0.0) -> Report:
    """FIRLS_OG (Algorithm 2) or FIRLS_TV (Algorithm 3).

    x^1 = A^H b unless given (Section 3.3 recommends this start).  At each
    outer iteration the objective of x^k is evaluated, the stop rule
    (F_eps^{k-1} - F_eps^k) <= tau F_eps^k is tested (k > 1, tau > 0), and
    otherwise W, d are refreshed and K PCG iterations give x^{k+1}.
    """
    x = ops.AHb() if x1 is None else np.array(x1, dtype=np.complex128, copy=True)
    hist: List[float] = []
    pcg_total = 0
    outer = 0
    converged = False
    while True:
        Fe, F, _ = ops.objective(x)
        hist.append(Fe)
        if len(hist) > 1 and tau > 0.0 and (hist[-2] - Fe) <= tau * Fe:
            converged = True
            break
        if outer >= T_max:
            break
        _, d = ops.weights(x)
        x, it = pcg(ops, d, x, K, precond=precond, eta=eta)
        pcg_total += it
        outer += 1
    return Report(x=x, outer_iters=outer, pcg_iters=pcg_total, F_eps=Fe, F=F,
                  history=hist, converged=converged)


def stationarity(ops: Operators, x) -> float:
    """||S(W(x)) x - A^H b|| / ||A^H b|| (the fixed-point condition of
    Theorem 3, eq. 27)."""
    _, d = ops.weights(x)
    g = ops.S(x, d) - ops.AHb()
    return float(np.linalg.norm(g) / np.linalg.norm(ops.AHb()))


def snr_db(x, truth) -> float:
    """SNR = 10 log10(var(x0) / MSE) (Section 5.4), magnitude image."""
    mse = np.mean((np.abs(x) - truth) ** 2)
    with np.errstate(divide="ignore"):
        return float(10.0 * np.log10(np.var(truth) / mse))   # +inf for an exact magnitude

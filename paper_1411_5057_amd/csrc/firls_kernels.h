// FIRLS kernels (templated; instantiated per precision and image size).
//
// One PCG iteration on a batch of slices of one shape (TV) is four launches:
//   k_rowfwd  : read z, p = z + beta p, then row FFTs of p -> t
//   k_col     : column FFT, times mask / n^2, column inverse FFT (t in place)
//   k_rowinv  : row inverse FFTs of t plus lambda Psi^T diag(d) Psi p -> q,
//               and the partials of <p, q>
//   k_update  : alpha = <r,z>/<p,q>, x += alpha p, r -= alpha q, and
//               z = M^{-1} r in red-black order (eqs. 40-43) with <r, z>
// so q = S p with S of eq. (15) / eq. (39).  With Haar (pseudo-diagonal
// preconditioner Phi^T (rho + lambda d)^{-1} Phi, eq. 17) the update of one
// iteration and the row pass of the next are one launch (RF_STEP_HAAR):
// it needs beta_k = <r_{k+1}, z_{k+1}> / <r_k, z_k> before the global sum of
// <r_{k+1}, z_{k+1}> exists, and takes it from the recurrence
//   <r_{k+1}, z_{k+1}> = alpha_k^2 <q_k, P^{-1} q_k> - <r_k, z_k>,
// which follows from r_{k+1} = r_k - alpha_k q_k and <q_k, z_k> = <p_k, q_k>
// (S-conjugacy of p_k and p_{k-1}); the row-inverse pass sums
// <q_k, P^{-1} q_k> alongside <p_k, q_k>.  alpha_{k+1} uses the directly
// summed <r_{k+1}, z_{k+1}>, so the recurrence only enters beta and never
// accumulates.  After the last iteration only x += alpha p is needed (r is
// recomputed from x at the next outer iteration).
// The FP64 partial sums of each inner product are written one per workgroup
// and summed, in index order,
// by every workgroup that needs the scalar.
//
// Row passes work on bands of band_rows(n) full rows; the Haar parts run in
// registers on 16-row tile columns (haar_col), the FFT parts through LDS.
#pragma once
#include <type_traits>

#include "firls_dev.h"

namespace firls {

template <typename T, int N> struct Geo {
  static constexpr int COLS = strip_cols(sizeof(T) == 8, N);   // strip width of column passes
};

// The twiddle table exp(-2 pi i k / N), k < N, copied into LDS behind the
// LINES lines of the FFT buffer.  The first stage of an FFT uses no
// twiddles and ends with a barrier, so the copy is visible before any use.
template <typename T, int N, int LINES>
__device__ __forceinline__ const cplx<T>* lds_twiddles(cplx<T>* lds, const void* tw) {
  cplx<T>* t = lds + LINES * LdsLayout<N>::LS;
  const cplx<T>* g = static_cast<const cplx<T>*>(tw);
  for (int i = threadIdx.x; i < N; i += NT) t[i] = g[i];
  return t;
}

// The spectrum scratch t between the three FFT passes is stored strip-major:
// column strip j (COLS columns) of contrast c is one contiguous block of n
// rows x COLS values.  The column pass then streams whole blocks, and a row
// band still meets it as runs of COLS values per row.  ``row`` counts the
// rows of all contrasts (row = c n + local row).
template <typename T, int N>
__device__ __forceinline__ size_t t_index(int row, int col) {
  constexpr int TS = Geo<T, N>::COLS;
  const int ch = row / N, lr = row - ch * N;
  return (size_t)ch * N * N + (size_t)(col / TS) * (N * TS) + (size_t)lr * TS + (col % TS);
}

// The workgroup's place: slice (index into the desc and state arrays) and
// its block within the slice (row band, column strip or tile).  A kernel
// launched per shape takes them from its grid and the slice list; a launch
// across shapes reads them from its work table.
struct Blk {
  int x;   // block within the slice
  int s;   // slice
};

#define FIRLS_SLICE_PROLOGUE_S(sidx)              \
  const int s_ = (sidx);                         \
  if (!P.state[s_].active) return;               \
  const SliceDesc& D = P.desc[s_];

// The preconditioner on one tile column (16 rows of column ``col``; v in the
// pixel domain, dg points at the weight d of the first row, row stride N):
// acc += <v, P^{-1} v>, and with NEED_Z v becomes P^{-1} v.
//   PC_PAPER : Phi^T ((Phi v) / (rho + lambda d))                 (eq. 17)
//   PC_JACOBI: v / (rho + lambda diag(Phi^T diag(d) Phi))         (diag of S)
//   PC_NONE  : v                                                  (plain CG)
// The paper's preconditioner with the 16 weights d already in registers.
template <bool NEED_Z, typename T>
__device__ __forceinline__ void precond_tile_paper(cplx<T> (&v)[16], const T (&dv)[16], int L, int col, T rho,
                                                   T lam, double& acc) {
  haar_col<false>(v, L, col);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const T iv = pc_inv(rho, lam, dv[s]);
    acc += (double)(cabs2t(v[s]) * iv);
    if (NEED_Z) v[s] = v[s] * iv;
  }
  if (NEED_Z) haar_col<true>(v, L, col);
}

template <bool NEED_Z, int N, int PC, typename T>
__device__ __forceinline__ void precond_tile_k(cplx<T> (&v)[16], const T* dg, int L, int col, T rho, T lam,
                                               double& acc) {
  if constexpr (PC == PC_PAPER) {
    haar_col<false>(v, L, col);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const T iv = pc_inv(rho, lam, dg[s * N]);
      acc += (double)(cabs2t(v[s]) * iv);
      if (NEED_Z) v[s] = v[s] * iv;
    }
    if (NEED_Z) haar_col<true>(v, L, col);
  } else if constexpr (PC == PC_JACOBI) {
    T e[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) e[s] = dg[s * N];
    haar_diag_col(e, L, col);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const T iv = pc_inv(rho, lam, e[s]);
      acc += (double)(cabs2t(v[s]) * iv);
      if (NEED_Z) v[s] = v[s] * iv;
    }
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) acc += (double)cabs2t(v[s]);
  }
}

// The same with the kind chosen at run time (uniform per launch).
template <bool NEED_Z, int N, typename T>
__device__ __forceinline__ void precond_tile(cplx<T> (&v)[16], const T* dg, int L, int col, T rho, T lam,
                                             int pc, double& acc) {
  if (pc == PC_PAPER) precond_tile_k<NEED_Z, N, PC_PAPER>(v, dg, L, col, rho, lam, acc);
  else if (pc == PC_JACOBI) precond_tile_k<NEED_Z, N, PC_JACOBI>(v, dg, L, col, rho, lam, acc);
  else precond_tile_k<NEED_Z, N, PC_NONE>(v, dg, L, col, rho, lam, acc);
}

// Early exit of the PCG solve (the PCG stopping criterion of Algorithms 2
// and 3, which the paper leaves open, read as a relative preconditioned-
// residual test): the first iteration j >= 1 whose <r_j, z_j> is at most
// eta^2 <r_0, z_0>, or 0.  Every kernel that forms a step decides from
// the same <r_j, z_j> partials (written by earlier launches of the solve),
// so all workgroups agree without communicating.
__device__ __forceinline__ int pcg_stop_at(const Params& P, const SliceDesc& D, int k) {
  if (!(P.eta2 > 0.0)) return 0;
  const double lim = P.eta2 * slot_sum(slot_ptr(D, SLOT_RZ0), P.nrz);
  for (int j = 1; j <= k; ++j)
    if (slot_sum(slot_ptr(D, SLOT_RZ0 + j), P.nrz) <= lim) return j;
  return 0;
}

// alpha = <r_k, z_k> / <p_k, S p_k> of PCG step k of slice s.  For HPD S,
// <p, S p> is positive whenever the residual is not zero (then <r, z> > 0
// and p != 0), so a non-positive (or NaN) <p, S p> with <r, z> > 0 is a
// breakdown: the first workgroup records FIRLS_E_BREAKDOWN, which stops the
// slice at its next outer check, and the step is taken as zero.  A zero
// residual (both zero) is the ordinary end of the iteration: a zero step.
// After the early exit every later step is zero (x and r stay at the
// iterate of the exit), and the first workgroup records how many
// iterations the solve took.  The test hook TEST_BREAKDOWN turns <p, S p>
// negative.
__device__ __forceinline__ double pcg_alpha(const Params& P, Blk B, int k, double rz, double pq) {
  const int stop = pcg_stop_at(P, P.desc[B.s], k);
  if (stop) {
    if (B.x == 0 && threadIdx.x == 0) P.state[B.s].pcg_stop = stop;
    return 0.0;
  }
  if (P.test_flags & TEST_BREAKDOWN) pq = -fabs(pq);
  if (pq > 0.0) return rz / pq;
  if (rz > 0.0 && B.x == 0 && threadIdx.x == 0 && P.state[B.s].status >= 0) P.state[B.s].status = ST_E_BREAKDOWN;
  return 0.0;
}

// A PCG launch whose work belongs to step k (it computes alpha_k, or feeds
// only <p_k, S p_k>) does nothing once the early exit has removed that
// step: every later step is zero, and nothing after the solve reads what
// these launches would write (the next residual pass recomputes r, z, p
// from x).  The first workgroup records the exit, as pcg_alpha would.
// Uniform over the workgroup, so it may return before any barrier.
__device__ __forceinline__ bool pcg_skip(const Params& P, const SliceDesc& D, int s, int bx, int k) {
  if (!(P.eta2 > 0.0) || k < 1) return false;
  const int stop = pcg_stop_at(P, D, k);
  if (stop && bx == 0 && threadIdx.x == 0) P.state[s].pcg_stop = stop;
  return stop != 0;
}

// Objective of the current x and the outer stopping rule of slice s (one
// workgroup; every thread takes part in the sums).  F_eps = data + lambda
// sum sqrt(s_g + eps); stop when (F_eps^{prev} - F_eps) <= tau F_eps after
// the first evaluation, or once Tmax solves are done; otherwise count the
// solve that follows.
__device__ __forceinline__ void outer_check_wg(const Params& P, int s) {
  SliceState& S = P.state[s];
  const SliceDesc& D = P.desc[s];
  const double data = P.no_data ? 0.0 : slot_sum(slot_ptr(D, SLOT_DATA), P.ndata);
  const double re = slot_sum(slot_ptr(D, SLOT_REG_EPS), P.nreg);
  const double r0 = slot_sum(slot_ptr(D, SLOT_REG0), P.nreg);
  if (threadIdx.x != 0) return;
  const double Fe = data + D.lambda * re;
  const double F = data + D.lambda * r0;
  const bool first = S.evals == 0;
  const double prev = S.Fe;
  // the solve before this check (counted as K iterations when it started)
  // may have stopped early
  if (!first && S.pcg_stop > 0) S.pcg -= P.K - S.pcg_stop;
  S.pcg_stop = 0;
  S.Fe_prev = first ? Fe : prev;
  S.rel = first ? 0.0 : (prev - Fe) / Fe;
  S.Fe = Fe;
  S.F = F;
  S.data = data;
  S.evals += 1;
  // Theorem 2: with x^{k+1} from PCG started at x^k (any number of
  // iterations, each lowering the majoriser) F_eps never rises; beyond the
  // rounding slack a rise is reported (the stop rule then ends the slice
  // when tau > 0)
  if (!first && S.status == ST_OK && isfinite(Fe) && Fe > prev * (1.0 + P.mono_slack)) S.status = ST_W_NONMONOTONE;
  if (S.status < 0) {
    S.active = 0;   // a PCG pass recorded an error (sync time-out, breakdown): stop, keep it
  } else if (!isfinite(Fe)) {
    S.status = ST_E_NONFINITE;
    S.active = 0;
  } else if (!first && P.tau > 0.0 && (prev - Fe) <= P.tau * Fe) {
    S.converged = 1;
    S.active = 0;
  } else if (S.outer >= P.Tmax) {
    if (P.tau > 0.0 && S.status == ST_OK) S.status = ST_W_MAXITER;
    S.active = 0;
  } else {
    S.outer += 1;
    S.pcg += P.K;
  }
  // a slice that goes on runs K PCG iterations, whose last x += alpha p the
  // next residual pass applies
  if (P.fold_x) S.pend = S.active;
  // the host polls this word to learn when the test ran and its outcome: a
  // system-scope store goes straight to host memory
  if (P.stop_flags)
    __hip_atomic_store(P.stop_flags + s, (S.evals << 1) | S.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// TV coefficients are stored in forward slots: slot (r, c) of D1 holds
// v[r+1, c] - s1(r) v[r, c] and slot (r, c) of D2 holds v[r, c+1] - s2(c) v[r, c]
// (indices mod n).  Periodic differences have s = 1 everywhere.  The paper's
// non-periodic D (backward differences whose first row is the pixel itself,
// Section 4.1) is the same with s1(n-1) = s2(n-1) = 0: its coefficient for
// pixel (r, c) sits in slot (r-1, c) of D1 / (r, c-1) of D2, and the slots
// that wrap hold the identity rows.  The host maps the caller's coefficient
// order to these slots.
__device__ __forceinline__ bool tv_cut(int tvb, int i, int n) { return tvb && i == n - 1; }

// (D1^T W1 D1 + D2^T W2 D2) v at pixel (r, c), lambda left out:
//   s1(r) W1[r] (v[r] - v[r+1]) + W1[r-1] (v[r] - s1(r-1) v[r-1]) + (same along c)
// tv_gather loads what one pixel needs (so a caller can issue the loads of
// several pixels before using any), tv_combine forms the value.
template <typename T>
struct TvNb {
  cplx<T> v0, vrp, vrm, vcp, vcm;
  T a, b, e, f;
};
template <typename T>
__device__ __forceinline__ TvNb<T> tv_gather(const cplx<T>* v, const T* w1, const T* w2, int n, int r, int c, int tvb) {
  const int rp = r + 1 == n ? 0 : r + 1, rm = r == 0 ? n - 1 : r - 1;
  const int cp = c + 1 == n ? 0 : c + 1, cm = c == 0 ? n - 1 : c - 1;
  TvNb<T> g;
  g.v0 = v[r * n + c];
  g.vrp = v[rp * n + c];
  g.vcp = v[r * n + cp];
  g.a = tv_cut(tvb, r, n) ? (T)0 : w1[r * n + c];
  g.b = w1[rm * n + c];
  g.e = tv_cut(tvb, c, n) ? (T)0 : w2[r * n + c];
  g.f = w2[r * n + cm];
  g.vrm = tv_cut(tvb, rm, n) ? cplx<T>{(T)0, (T)0} : v[rm * n + c];
  g.vcm = tv_cut(tvb, cm, n) ? cplx<T>{(T)0, (T)0} : v[r * n + cm];
  return g;
}
template <typename T>
__device__ __forceinline__ cplx<T> tv_combine(const TvNb<T>& g) {
  return (g.v0 - g.vrp) * g.a + (g.v0 - g.vrm) * g.b + (g.v0 - g.vcp) * g.e + (g.v0 - g.vcm) * g.f;
}

// ---------------------------------------------------------------------------
// Weights of the groups g0 .. g1-1 of one row band from |Phi x|^2 in LDS
// (lists of width W, member offsets within the band): W_g into WL and the
// penalty partials.  Each thread takes groups g0 + tid + k NT, eight at a
// time, their list loads first.
template <int W, typename T>
__device__ __forceinline__ void band_group_weights(const uint16_t* gell, int g0, int g1, const T* sqL, T* WL, T eps,
                                                   double& ae, double& a0) {
  for (int gb = g0 + (int)threadIdx.x; gb < g1; gb += 8 * NT) {
    uint16_t e[8][W];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int g = gb + u * NT;
      if (g < g1) ell_row_w<W>(gell + (size_t)g * W, e[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int g = gb + u * NT;
      if (g < g1) {
        T w, ve, v0;
        group_weight(ell_gather<W>(e[u], sqL), eps, w, ve, v0);
        WL[g - g0] = w;
        ae += (double)ve;
        a0 += (double)v0;
      }
    }
  }
}

// d of the band's PIX coefficients: sum of W over the groups in each
// coefficient's list (width W, group offsets from the band's first group).
template <int W, int PIX, typename T>
__device__ __forceinline__ void band_d(const uint16_t* tell, const T* WL, T* d) {
  static_assert(PIX % NT == 0, "band not a multiple of the workgroup");
  constexpr int E = PIX / NT;
  constexpr int CH = E % 8 == 0 ? 8 : (E % 4 == 0 ? 4 : (E % 3 == 0 ? 3 : 1));
#pragma unroll
  for (int c = 0; c < E; c += CH) {
    uint16_t e[CH][W];
#pragma unroll
    for (int u = 0; u < CH; ++u) ell_row_w<W>(tell + (size_t)(threadIdx.x + (c + u) * NT) * W, e[u]);
#pragma unroll
    for (int u = 0; u < CH; ++u) d[threadIdx.x + (c + u) * NT] = ell_gather<W>(e[u], WL);
  }
}

template <typename T, int N, int MODE>
__device__ __forceinline__ void rowfwd_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  using Lay = LdsLayout<N>;
  using U = Units<N, ROWS>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  __shared__ double red[2 * NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if constexpr (MODE == RF_STEP_HAAR || MODE == RF_PCG_HAAR || MODE == RF_PCG_Z) {
    if (pcg_skip(P, D, s_, B.x, MODE == RF_STEP_HAAR ? P.k - 1 : P.k)) return;
  }
  const size_t off = (size_t)B.x * ROWS * N;
  const C* tw = lds_twiddles<T, N, ROWS>(lds, P.tw);
  C* t = static_cast<C*>(D.t);
  const int row0 = B.x * ROWS;
  auto gdst = [&](int l, int q, C v) { t[t_index<T, N>(row0 + l, q)] = v; };
  if constexpr (MODE == RF_PLAIN) {
    const C* x = static_cast<const C*>(D.x) + off;
    fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, [&](int l, int q) { return x[l * N + q]; }, gdst);
  } else if constexpr (MODE == RF_SQW_HAAR || MODE == RF_PEN_HAAR) {
    // RF_PEN_HAAR: only the penalty partials of x (no x update, d or FFT).
    constexpr bool PEN = MODE == RF_PEN_HAAR;
    // Every group lies inside one row band (tree groups do: parent and child
    // share a Haar tile), so the weights need nothing outside this band:
    // |Phi x|^2 into LDS, W_g of the band's groups (eq. 12) and the penalty
    // partials, then d = diag(G^T W G) of the band's coefficients (eq. 13),
    // all on chip; x stays in registers meanwhile and then goes through the
    // same LDS for the row FFTs.
    // With fold_x a pending x += alpha p of the last PCG iteration (alpha
    // from its <r,z> and <p,q> sums) is applied first and x written back.
    C* x = static_cast<C*>(D.x) + off;
    const bool pend = !PEN && P.fold_x && P.state[s_].pend;
    T al = (T)0;
    if (pend) {
      const double rz = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k), P.nrz);
      const double pq = slot_sum(slot_ptr(D, SLOT_PQ0 + P.k), P.npq);
      al = (T)pcg_alpha(P, Blk{B.x, s_}, P.k, rz, pq);
    }
    const C* p = static_cast<const C*>(D.p) + off;
    T* sqL = reinterpret_cast<T*>(smem);           // ROWS * N values
    T* WL = sqL + ROWS * N;                         // the band's groups
    C xv[U::PER][16];
#pragma unroll
    for (int k = 0; k < U::PER; ++k) {
      if (!U::valid(k)) continue;
      const int col = U::col(k), row = U::row(k);
#pragma unroll
      for (int s = 0; s < 16; ++s) xv[k][s] = x[(row + s) * N + col];
      if (pend) {
        C pv[16];   // all loads before the first store (see the update step)
#pragma unroll
        for (int s = 0; s < 16; ++s) pv[s] = p[(row + s) * N + col];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          xv[k][s] = xv[k][s] + pv[s] * al;
          x[(row + s) * N + col] = xv[k][s];
        }
      }
      C v[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) v[s] = xv[k][s];
      haar_col<false>(v, P.L, col);
#pragma unroll
      for (int s = 0; s < 16; ++s) sqL[(row + s) * N + col] = (T)cabs2(v[s]);
    }
    __syncthreads();
    const int g0 = P.shape.bgptr[B.x], g1 = P.shape.bgptr[B.x + 1];
    const ShapeDev& G = P.shape;
    double ae = 0.0, a0 = 0.0;
    T* d = static_cast<T*>(D.d) + off;
    if (G.gell) {
      // padded lists of compile-time width: each thread's list loads are
      // issued together, ahead of the LDS gathers that use them
      auto groups = [&](auto wtag) {
        constexpr int W = decltype(wtag)::value;
        band_group_weights<W>(G.gell, g0, g1, sqL, WL, (T)P.eps, ae, a0);
      };
      switch (G.gw) {
        case 1: groups(std::integral_constant<int, 1>{}); break;
        case 2: groups(std::integral_constant<int, 2>{}); break;
        case 4: groups(std::integral_constant<int, 4>{}); break;
        default: groups(std::integral_constant<int, 8>{}); break;
      }
      if constexpr (!PEN) {
        __syncthreads();
        auto members = [&](auto wtag) {
          constexpr int W = decltype(wtag)::value;
          band_d<W, ROWS * N>(G.tell + off * W, WL, d);
        };
        switch (G.tw) {
          case 1: members(std::integral_constant<int, 1>{}); break;
          case 2: members(std::integral_constant<int, 2>{}); break;
          case 4: members(std::integral_constant<int, 4>{}); break;
          default: members(std::integral_constant<int, 8>{}); break;
        }
      }
    } else {
      for (int g = g0 + (int)threadIdx.x; g < g1; g += NT) {
        T s2 = (T)0;
        for (int j = G.gptr[g]; j < G.gptr[g + 1]; ++j) s2 += sqL[G.gidx[j] - (int)off];
        T w, ve, v0;
        group_weight(s2, (T)P.eps, w, ve, v0);
        WL[g - g0] = w;
        ae += (double)ve;
        a0 += (double)v0;
      }
      if constexpr (!PEN) {
        __syncthreads();
        for (int j = threadIdx.x; j < ROWS * N; j += NT) {
          T s2 = (T)0;
          for (int t = G.tptr[off + j]; t < G.tptr[off + j + 1]; ++t) s2 += WL[G.tidx[t] - g0];
          d[j] = s2;
        }
      }
    }
    block_sum2(ae, a0, red);       // also orders the LDS reads above before the FFT
    if (threadIdx.x == 0) {
      slot_wptr(D, SLOT_REG_EPS)[B.x] = ae;
      slot_wptr(D, SLOT_REG0)[B.x] = a0;
    }
    if constexpr (!PEN) {
#pragma unroll
      for (int k = 0; k < U::PER; ++k) {
        if (!U::valid(k)) continue;
        const int col = U::col(k), row = U::row(k);
#pragma unroll
        for (int s = 0; s < 16; ++s) lds[Lay::at(row + s, col)] = xv[k][s];
      }
      __syncthreads();
      fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, LdsIO<T, N>{lds}, gdst);
    }
  } else if constexpr (MODE == RF_SQ_HAAR) {
    // row FFTs of x and, from the same read, |Phi x|^2 per coefficient
    const C* x = static_cast<const C*>(D.x) + off;
    T* sq = static_cast<T*>(D.sq) + off;
#pragma unroll
    for (int k = 0; k < U::PER; ++k) {
      if (!U::valid(k)) continue;
      const int col = U::col(k), row = U::row(k);
      C v[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        v[s] = x[(row + s) * N + col];
        lds[Lay::at(row + s, col)] = v[s];
      }
      haar_col<false>(v, P.L, col);
#pragma unroll
      for (int s = 0; s < 16; ++s) sq[(row + s) * N + col] = (T)cabs2(v[s]);
    }
    if (!P.nofft) {   // a dense sensing matrix takes p itself, not its row FFT
      __syncthreads();
      fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, LdsIO<T, N>{lds}, gdst);
    }
  } else {
    double beta = 0.0;
    if (MODE != RF_STEP_HAAR && P.k > 0) {
      const double rz = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k), P.nrz);
      const double rzo = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k - 1), P.nrz);
      beta = rzo > 0.0 ? rz / rzo : 0.0;
    }
    const T bt = (T)beta;
    C* p = static_cast<C*>(D.p) + off;
    if constexpr (MODE == RF_STEP_HAAR) {
      // end of iteration k - 1 (alpha, x, r, <r_k, z_k>) and start of
      // iteration k (z_k, p_k = z_k + beta p_{k-1}) in one pass
      const double rzo = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k - 1), P.nrz);
      const double pqo = slot_sum(slot_ptr(D, SLOT_PQ0 + P.k - 1), P.npq);
      const double qqo = slot_sum(slot_ptr(D, SLOT_QQ0 + P.k - 1), P.nrz);
      const double ald = pcg_alpha(P, Blk{B.x, s_}, P.k - 1, rzo, pqo);
      const double rzn = ald * ald * qqo - rzo;
      const T al = (T)ald;
      const T bs = (T)(rzo > 0.0 && rzn > 0.0 ? rzn / rzo : 0.0);
      C* x = static_cast<C*>(D.x) + off;
      C* r = static_cast<C*>(D.r[0]) + off;
      const C* q = static_cast<const C*>(D.q) + off;
      const T* d = static_cast<const T*>(D.d) + off;
      const T rhot = (T)P.state[s_].rho, lam = (T)D.lambda;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < U::PER; ++k) {
        if (!U::valid(k)) continue;
        const int col = U::col(k), row = U::row(k);
        C v[16];
        // p_{k-1} waits in this thread's own LDS cells until beta p is added.
        // Loads go ahead of the stores in chunks: the compiler cannot prove
        // that x, r, p and q do not overlap, so it keeps every load after
        // the stores before it.
        constexpr int CH = 8;
#pragma unroll
        for (int s0 = 0; s0 < 16; s0 += CH) {
          C po[CH], xo[CH], qo[CH];
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int g = (row + s0 + u) * N + col;
            po[u] = p[g];
            xo[u] = x[g];
            v[s0 + u] = r[g];
            qo[u] = q[g];
          }
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int g = (row + s0 + u) * N + col;
            lds[Lay::at(row + s0 + u, col)] = po[u];
            x[g] = xo[u] + po[u] * al;
            v[s0 + u] = v[s0 + u] - qo[u] * al;
            r[g] = v[s0 + u];
          }
        }
        precond_tile_k<true, N, PC_PAPER>(v, d + row * N + col, P.L, col, rhot, lam, acc);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const int a = Lay::at(row + s, col);
          const C pn = v[s] + lds[a] * bs;
          p[(row + s) * N + col] = pn;
          lds[a] = pn;
        }
      }
      const double tot = block_sum(acc, red);
      if (threadIdx.x == 0) slot_wptr(D, SLOT_RZ0 + P.k)[B.x] = tot;
    } else if constexpr (MODE == RF_PCG_HAAR) {
      // z = P^{-1} r in registers (precond_tile), p = z + beta p
      const C* r = static_cast<const C*>(D.r[0]) + off;
      const T* d = static_cast<const T*>(D.d) + off;
      const T rho = (T)P.state[s_].rho, lam = (T)D.lambda;
#pragma unroll
      for (int k = 0; k < U::PER; ++k) {
        if (!U::valid(k)) continue;
        const int col = U::col(k), row = U::row(k);
        C v[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = r[(row + s) * N + col];
        double unused = 0.0;
        precond_tile<true, N>(v, d + row * N + col, P.L, col, rho, lam, P.precond, unused);
        C po[16];   // p is not read at k = 0; its loads go before the stores
#pragma unroll
        for (int s = 0; s < 16; ++s) po[s] = P.k > 0 ? p[(row + s) * N + col] : C{(T)0, (T)0};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const C pn = P.k > 0 ? v[s] + po[s] * bt : v[s];
          p[(row + s) * N + col] = pn;
          lds[Lay::at(row + s, col)] = pn;
        }
      }
    } else {
      // p = z + beta p over the band, eight pixels per thread at a time with
      // their loads ahead of the stores (the compiler cannot prove that p
      // and z do not overlap, and would otherwise wait for every load)
      const C* z = static_cast<const C*>(D.z) + off;
      constexpr int PER = ROWS * N / NT, CH = 8;
      static_assert(PER * NT == ROWS * N, "whole band per workgroup");
#pragma unroll
      for (int e0 = 0; e0 < PER; e0 += CH) {
        C zv[CH], pv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int i = threadIdx.x + (e0 + u) * NT;
          if (e0 + u < PER) {
            zv[u] = z[i];
            pv[u] = P.k > 0 ? p[i] : C{(T)0, (T)0};
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int i = threadIdx.x + (e0 + u) * NT;
          if (e0 + u < PER) {
            const C pn = P.k > 0 ? zv[u] + pv[u] * bt : zv[u];
            p[i] = pn;
            lds[Lay::at(i / N, i % N)] = pn;
          }
        }
      }
    }
    if (!P.nofft) {   // a dense sensing matrix takes p itself, not its row FFT
      __syncthreads();
      fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, LdsIO<T, N>{lds}, gdst);
    }
  }
}
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_rowfwd(Params P) {
  rowfwd_body<T, N, MODE>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__device__ __forceinline__ void col_body(const Params& P, const Blk B) {
  constexpr int COLS = Geo<T, N>::COLS;
  using C = cplx<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  __shared__ double red[NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if constexpr (MODE == COL_SP || MODE == COL_SP_PQ) {
    if (pcg_skip(P, D, s_, B.x, P.k)) return;
  }
  // workgroup = (contrast ch, strip): strips of all contrasts in turn
  constexpr int STRIPS = N / COLS;
  const int ch = B.x / STRIPS, strip = B.x - ch * STRIPS;
  const int col0 = strip * COLS;
  const C* tw = lds_twiddles<T, N, COLS>(lds, P.tw);
  C* t = static_cast<C*>(D.t) + (size_t)ch * N * N + (size_t)strip * N * COLS;   // this strip's block
  // sampled(c, row): bit of column col0 + c in the packed mask word of its
  // 16 columns and the row
  const uint16_t* mw = D.mbits + (size_t)ch * N;
  auto sampled = [&](int c, int row) {
    const int gc = col0 + c;
    return (mw[(size_t)(gc >> 4) * N * P.C + row] >> (gc & 15)) & 1u;
  };
  auto gsrc = [&](int c, int row) { return t[row * COLS + c]; };
  auto gdst = [&](int c, int row, C v) { t[row * COLS + c] = v; };
  const T sn = (T)1 / (T)N;
  // the spectrum passes from the forward to the inverse column FFT in
  // registers (fft_lines_fwd_inv); the mask bits of the positions this
  // thread will hold are fetched first, so no load waits between the
  // transforms; the partial sums of a mode are complete once the inverse
  // has started, and are summed after it
  using Map = FwdInvMap<T, N, COLS, COLMAP>;
  uint32_t mine[Map::ITER];   // bit r: position r of butterfly i sampled
#pragma unroll
  for (int i = 0; i < Map::ITER; ++i) {
    int c, j;
    mine[i] = 0u;
    if (!Map::at(i, c, j)) continue;
#pragma unroll
    for (int r = 0; r < Map::RL; ++r) mine[i] |= (uint32_t)sampled(c, j + r * Map::NBL) << r;
  }
  auto smp = [&](int i, int r) { return (mine[i] >> r) & 1u; };
  if constexpr (MODE == COL_SP) {
    const T sc = sn * sn;
    fft_lines_fwd_inv<T, N, COLS, COLMAP>(lds, tw, gsrc, [&](int i, int r, int c, int row, C v) {
      return smp(i, r) ? v * sc : C{(T)0, (T)0};
    }, gdst);
  } else if constexpr (MODE == COL_SP_PQ) {
    // as COL_SP, and the partials of <p, A^H A p> = ||m F p||^2 / n^2 go to
    // the <p, S p> slot after the row pass's partials
    const T sc = sn * sn;
    double acc = 0.0;
    fft_lines_fwd_inv<T, N, COLS, COLMAP>(lds, tw, gsrc, [&](int i, int r, int c, int row, C v) {
      C u{(T)0, (T)0};
      if (smp(i, r)) {
        acc += (double)(cabs2t(v) * sc);
        u = v * sc;
      }
      return u;
    }, gdst);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) slot_wptr(D, SLOT_PQ0 + P.k)[P.C * (N / band_rows(N)) + B.x] = tot;
  } else if constexpr (MODE == COL_R0) {
    // k = (F x) at the sampled entries; keep m (b - k) / n for the inverse
    // and accumulate 1/2 ||m F x - b||^2.
    const C* b = static_cast<const C*>(D.b);
    double acc = 0.0;
    fft_lines_fwd_inv<T, N, COLS, COLMAP>(lds, tw, gsrc, [&](int i, int r, int c, int row, C v) {
      const size_t g = (size_t)(ch * N + row) * N + col0 + c;
      C u{(T)0, (T)0};
      if (smp(i, r)) {
        u = b[g] - v * sn;
        acc += cabs2(u);
        u = u * sn;
      }
      return u;
    }, gdst);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) slot_wptr(D, SLOT_DATA)[B.x] = 0.5 * tot;
  } else if constexpr (MODE == COL_DC) {
    // data consistency: keep F x where unsampled, put b where sampled
    // (k = m b + (1 - m) F x), then the column inverse with 1/n
    const C* b = static_cast<const C*>(D.b);
    fft_lines_fwd_inv<T, N, COLS, COLMAP>(lds, tw, gsrc, [&](int i, int r, int c, int row, C v) {
      const size_t g = (size_t)(ch * N + row) * N + col0 + c;
      return (smp(i, r) ? b[g] : v * sn) * sn;
    }, gdst);
  } else {
    const C* b = static_cast<const C*>(D.b);
    fft_lines<T, N, COLS, COLMAP, true>(lds, tw, [&](int c, int row) {
      const size_t g = (size_t)(ch * N + row) * N + col0 + c;
      return sampled(c, row) ? b[g] * sn : C{(T)0, (T)0};
    }, gdst);
  }
}
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_col(Params P) {
  col_body<T, N, MODE>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__device__ __forceinline__ void rowinv_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  using Lay = LdsLayout<N>;
  using U = Units<N, ROWS>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  __shared__ double red[NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if constexpr (MODE == RI_SP_HAAR || MODE == RI_SP_TV) {
    if (pcg_skip(P, D, s_, B.x, P.k)) return;
  }
  const int row0 = B.x * ROWS;
  const size_t off = (size_t)row0 * N;
  const C* tw = lds_twiddles<T, N, ROWS>(lds, P.tw);
  const C* tin = static_cast<const C*>(D.t);
  auto gsrc = [&](int l, int q) { return tin[t_index<T, N>(row0 + l, q)]; };
  if constexpr (MODE == RI_PLAIN) {
    C* x = static_cast<C*>(D.x) + off;
    fft_lines<T, N, ROWS, ROWMAP, true>(lds, tw, gsrc, [&](int l, int q, C v) { x[l * N + q] = v; });
  } else {
    constexpr bool SP = (MODE == RI_SP_HAAR || MODE == RI_SP_TV);
    constexpr bool HAAR = (MODE == RI_SP_HAAR || MODE == RI_R0_HAAR || MODE == RI_R0_HAAR_P0);
    // v: the vector the regulariser acts on; out: q (S p) or r (A^H b - S x)
    const C* vfull = static_cast<const C*>(SP ? D.p : D.x);
    const C* v = vfull + off;
    C* out = static_cast<C*>(SP ? D.q : D.r[0]) + off;
    const T lam = (T)D.lambda;
    const T sgn = SP ? (T)1 : (T)-1;
    double acc = 0.0;
    // the objective and stop test of this outer iteration (every partial it
    // needs is complete before this pass): the slice's first workgroup runs
    // it; a stopped slice's workgroups that start later just exit
    if (!SP && P.check_r0 && B.x == 0) outer_check_wg(P, s_);
    if constexpr (HAAR) {
      // A^H A part into LDS (row inverse FFT, or with a dense sensing matrix
      // the product A^T A v in t, row-major), then lambda Phi^T (d * Phi v)
      // in registers
      // q of the fused step's last iteration is never read (the next
      // residual pass needs only alpha and p): that launch forms only
      // lambda sum d |Phi p|^2, with no transform of t
      const bool q_dead = SP && P.q_dead;
      if (q_dead) {
      } else if (P.nofft) {
        const C* av = static_cast<const C*>(D.t) + off;
        for (int i = threadIdx.x; i < ROWS * N; i += NT) lds[Lay::at(i / N, i % N)] = av[i];
        __syncthreads();
      } else {
        fft_lines<T, N, ROWS, ROWMAP, true>(lds, tw, gsrc, LdsIO<T, N>{lds});
      }
      const T* d = static_cast<const T*>(D.d) + off;
      const T rho = (T)P.state[s_].rho;
      double acc2 = 0.0;
#pragma unroll
      for (int k = 0; k < U::PER; ++k) {
        if (!U::valid(k)) continue;
        const int col = U::col(k), row = U::row(k);
        C w[16];
        T dv[16];   // read once: the regulariser and the preconditioner both use it
        // <p, S p> = ||A p||^2 + lambda sum d |Phi p|^2: the first part
        // comes from the column pass, the second is summed here
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          w[s] = v[(row + s) * N + col];
          dv[s] = d[(row + s) * N + col];
        }
        haar_col<false>(w, P.L, col);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const T ld = lam * dv[s];
          if (SP) acc += (double)(ld * cabs2t(w[s]));
          w[s] = w[s] * (ld * sgn);
        }
        if (q_dead) continue;
        haar_col<true>(w, P.L, col);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const C o = lds[Lay::at(row + s, col)] + w[s];
          out[(row + s) * N + col] = o;
          w[s] = o;
        }
        // <o, P^{-1} o>: <q, P^{-1} q> for the beta recurrence, or <r0, z0>
        if constexpr (SP) {
          // only the fused step (paper's preconditioner) uses <q, P^{-1} q>,
          // and not after the last iteration
          if (P.precond == PC_PAPER) precond_tile_paper<false>(w, dv, P.L, col, rho, lam, acc2);
        } else if constexpr (MODE == RI_R0_HAAR_P0) {
          // the first PCG iteration's start: z0 = P^{-1} r0, p0 = z0, whose
          // row FFTs follow from this thread's own LDS cells (already read)
          precond_tile_paper<true>(w, dv, P.L, col, rho, lam, acc2);
          C* p = static_cast<C*>(D.p) + off;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            p[(row + s) * N + col] = w[s];
            lds[Lay::at(row + s, col)] = w[s];
          }
        } else {
          precond_tile<false, N>(w, d + row * N + col, P.L, col, rho, lam, P.precond, acc2);
        }
      }
      if (!q_dead) {
        const double t2 = block_sum(acc2, red);
        if (threadIdx.x == 0) slot_wptr(D, SP ? SLOT_QQ0 + P.k : SLOT_RZ0)[B.x] = t2;
      }
      if constexpr (MODE == RI_R0_HAAR_P0) {
        __syncthreads();
        C* tout = static_cast<C*>(D.t);
        fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, LdsIO<T, N>{lds},
                                             [&](int l, int q, C val) { tout[t_index<T, N>(row0 + l, q)] = val; });
      }
    } else {
      // this band's contrast: its image, its D1 weights and its D2 weights
      const int ch = row0 / N, lrow0 = row0 - ch * N;
      const size_t NN = (size_t)N * N;
      const C* vch = vfull + ch * NN;
      const T* w1 = static_cast<const T*>(D.d) + ch * NN;
      const T* w2 = static_cast<const T*>(D.d) + (P.C + ch) * NN;
      auto emit = [&](int l, int q, C val) {
        const int i = l * N + q;
        const C o = val + tv_combine(tv_gather<T>(vch, w1, w2, N, lrow0 + l, q, P.tvb)) * (lam * sgn);
        out[i] = o;
        if (SP) acc += cdot(v[i], o);
      };
      if (P.nofft) {
        const C* av = static_cast<const C*>(D.t) + off;
        for (int i = threadIdx.x; i < ROWS * N; i += NT) emit(i / N, i % N, av[i]);
      } else {
        fft_lines<T, N, ROWS, ROWMAP, true>(lds, tw, gsrc, emit);
      }
    }
    if constexpr (SP) {
      const double tot = block_sum(acc, red);
      if (threadIdx.x == 0) slot_wptr(D, SLOT_PQ0 + P.k)[B.x] = tot;
    }
  }
}
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_rowinv(Params P) {
  rowinv_body<T, N, MODE>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// ---------------------------------------------------------------------------
// The row-inverse pass of PCG iteration k - 1 and the fused step of
// iteration k in one launch (Haar, the paper's preconditioner, FFT
// operator; one row band per workgroup, one tile column per thread):
//   A: q = S p_{k-1} (row inverse FFT of the column pass's output plus
//      lambda Phi^T (d * Phi p)), the partials of <p, S p> and
//      <q, P^{-1} q>;
//   a barrier among the workgroups of the slice (their partials complete
//      alpha and the beta recurrence);
//   B: x += alpha p, r -= alpha q, z = P^{-1} r, <r, z>, p_k = z + beta p,
//      and the row FFT of p_k; with LAST_SUM, in the last iteration
//      (k = K - 1) also the partials of lambda sum d |Phi p_k|^2, so that
//      no row-inverse launch follows (the column pass adds ||A p_k||^2).
//      The launch across shapes leaves LAST_SUM out (its register budget
//      is tighter) and keeps that iteration's row-inverse launch.
// q waits in the thread's own LDS cells across the barrier (where A^H A p
// was), so it never goes through memory, and d in registers; B reads p
// again (keeping it in registers as well would spill).  The barrier counts arrivals in the
// slice's counter k, which grows by one band count per outer iteration
// (zeroed when the slice starts); the partials it publishes are the only
// data that crosses workgroups, written and read device-coherently, so no
// cache write-back or invalidation is needed.  Workgroups start in index
// order and a slice's bands are consecutive, so the workgroups that wait
// never hold back one that a slice still needs.  The wait is bounded: past
// the limit the slice is marked FIRLS_E_SYNC and the workgroup goes on.
// Four workgroups per CU in FP32, as the other row passes (without the
// bound the compiler takes registers for only two); two in FP64, as the
// FP64 fused step.  The closing row FFT is laid out
// from a thread index the compiler cannot see through, so its addresses
// are recomputed there rather than kept live from phase A, which would
// not fit the 128 registers of that occupancy and spill.
template <typename T, int N, bool LAST_SUM>
__device__ __forceinline__ void pcg_pair_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  using Lay = LdsLayout<N>;
  using U = Units<N, ROWS>;
  static_assert(U::PER <= 2, "one or two tile columns per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  __shared__ double red[NT / 64];
  __shared__ int timed_out;
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if (pcg_skip(P, D, s_, B.x, P.k - 1)) {
    // still counted at the slice's barrier, so later launches' targets hold
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(slot_wptr(D, SLOT_SYNC)) + P.k, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int row0 = B.x * ROWS;
  const size_t off = (size_t)row0 * N;
  const C* tw = lds_twiddles<T, N, ROWS>(lds, P.tw);
  const int k = P.k;
  const T* d = static_cast<const T*>(D.d) + off;
  const T rho = (T)P.state[s_].rho, lam = (T)D.lambda;
  C* p = static_cast<C*>(D.p) + off;
  // d of the thread's tile columns stays in registers from A to B
  T dv[U::PER][16];
  // A: the row inverse of iteration k - 1
  {
    const C* tin = static_cast<const C*>(D.t);
    fft_lines<T, N, ROWS, ROWMAP, true>(lds, tw, [&](int l, int q) { return tin[t_index<T, N>(row0 + l, q)]; },
                                        LdsIO<T, N>{lds});
    double acc = 0.0, acc2 = 0.0;
#pragma unroll
    for (int ku = 0; ku < U::PER; ++ku) {
      if (!U::valid(ku)) continue;
      const int col = U::col(ku), row = U::row(ku);
      C w[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        w[s] = p[(row + s) * N + col];
        dv[ku][s] = d[(row + s) * N + col];
      }
      haar_col<false>(w, P.L, col);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const T ld = lam * dv[ku][s];
        acc += (double)(ld * cabs2t(w[s]));
        w[s] = w[s] * ld;
      }
      haar_col<true>(w, P.L, col);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int a = Lay::at(row + s, col);
        w[s] = lds[a] + w[s];
        lds[a] = w[s];
      }
      precond_tile_paper<false>(w, dv[ku], P.L, col, rho, lam, acc2);
    }
    // the partials other workgroups read in B go out as device-coherent
    // stores; nothing else crosses workgroups, so the barrier needs no
    // cache write-back or invalidation
    const double t2 = block_sum(acc2, red);
    if (threadIdx.x == 0)
      __hip_atomic_store(slot_wptr(D, SLOT_QQ0 + k - 1) + B.x, t2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0)
      __hip_atomic_store(slot_wptr(D, SLOT_PQ0 + k - 1) + B.x, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // barrier among the slice's workgroups: the partial stores complete, the
  // arrival is counted, then the wait for the rest
  if (threadIdx.x == 0) {
    uint32_t* cnt = reinterpret_cast<uint32_t*>(slot_wptr(D, SLOT_SYNC)) + k;
    // (the test hook asks for one arrival more than can come and gives up
    // after a few polls, so the time-out path runs without a long wait)
    const bool hook = (P.test_flags & TEST_SYNC_TIMEOUT) != 0;
    const uint32_t bands = (uint32_t)(P.C * (N / ROWS));   // the slice's workgroups
    const uint32_t target = bands * (uint32_t)P.state[s_].outer + (hook ? 1u : 0u);
    const uint32_t limit = hook ? 64u : (1u << 20);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int late = 0;
    for (uint32_t spin = 0; __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++spin) {
      if (spin >= limit) {
        late = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    timed_out = late;
  }
  __syncthreads();
  if (timed_out && threadIdx.x == 0) P.state[s_].status = ST_E_SYNC;
  // B: the step of iteration k (this launch's partials read device-coherently)
  const double rzo = slot_sum(slot_ptr(D, SLOT_RZ0 + k - 1), P.nrz);
  const double pqo = slot_sum_coherent(slot_ptr(D, SLOT_PQ0 + k - 1), P.npq);
  const double qqo = slot_sum_coherent(slot_ptr(D, SLOT_QQ0 + k - 1), P.nrz);
  const double ald = pcg_alpha(P, Blk{B.x, s_}, k - 1, rzo, pqo);
  const double rzn = ald * ald * qqo - rzo;
  const T al = (T)ald;
  const T bs = (T)(rzo > 0.0 && rzn > 0.0 ? rzn / rzo : 0.0);
  // in the last iteration no launch inverts p_k's rows (its q is never
  // read): this one also sums lambda d |Phi p_k|^2, the regulariser's part
  // of <p_k, S p_k>, in the row-inverse pass's order, from the thread's
  // own LDS cells of p_k and d read again (keeping d and p_k in registers
  // through the p stores would spill), before the closing row FFT
  const bool last = LAST_SUM && k == P.K - 1;
  double acc = 0.0, accq = 0.0;
#pragma unroll
  for (int ku = 0; ku < U::PER; ++ku) {
    if (!U::valid(ku)) continue;
    // the tile column's indices again, opaque to the compiler, so the
    // addresses of A are not kept alive through the barrier for reuse here
    int cb = U::col(ku), rb = U::row(ku);
    asm volatile("" : "+v"(cb), "+v"(rb));
    C* x = static_cast<C*>(D.x) + off;
    C* r = static_cast<C*>(D.r[0]) + off;
    C v[16];
    // loads ahead of the stores, in chunks (the compiler cannot prove that
    // x and r do not overlap)
    constexpr int CH = 4;
#pragma unroll
    for (int s0 = 0; s0 < 16; s0 += CH) {
      C xo[CH], po[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int g = (rb + s0 + u) * N + cb;
        po[u] = p[g];
        xo[u] = x[g];
        v[s0 + u] = r[g];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int g = (rb + s0 + u) * N + cb;
        const int a = Lay::at(rb + s0 + u, cb);
        const C qo = lds[a];
        lds[a] = po[u];   // p_{k-1} waits in the cell of q until beta p is added
        x[g] = xo[u] + po[u] * al;
        v[s0 + u] = v[s0 + u] - qo * al;
        r[g] = v[s0 + u];
      }
    }
    precond_tile_paper<true>(v, dv[ku], P.L, cb, rho, lam, acc);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int a = Lay::at(rb + s, cb);
      const C pn = v[s] + lds[a] * bs;
      p[(rb + s) * N + cb] = pn;
      lds[a] = pn;
    }
    if (last) {
      // the tile column once more from an opaque index, so no address of
      // the loops above stays live into this one
      int u = threadIdx.x + ku * NT;
      asm volatile("" : "+v"(u));
      const int c2 = u % N, r2 = (u / N) * 16;
      const T* dk = static_cast<const T*>(D.d) + off;
      C w[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) w[s] = lds[Lay::at(r2 + s, c2)];
      haar_col<false>(w, P.L, c2);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const T ld = lam * dk[(r2 + s) * N + c2];
        accq += (double)(ld * cabs2t(w[s]));
      }
    }
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) slot_wptr(D, SLOT_RZ0 + k)[B.x] = tot;
  C* t = static_cast<C*>(D.t);
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  fft_lines<T, N, ROWS, ROWMAP, false>(lds, tw, LdsIO<T, N>{lds},
                                       [&](int l, int q, C val) { t[t_index<T, N>(row0 + l, q)] = val; }, tid);
  if (last) {
    const double tq = block_sum(accq, red);
    if (threadIdx.x == 0) slot_wptr(D, SLOT_PQ0 + k)[B.x] = tq;
  }
}
// Workgroups per CU of the paired pass: four in FP32 with one tile column
// per thread, two in FP64 or with two tile columns per thread (sides 384
// and 512, whose row passes hold two workgroups per CU anyway).
template <typename T, int N>
constexpr int pair_wgs_per_cu() {
  return sizeof(T) == 4 && Units<N, band_rows(N)>::PER == 1 ? 4 : 2;
}
template <typename T, int N>
__global__ __launch_bounds__(NT, (pair_wgs_per_cu<T, N>())) void k_pcg_pair(Params P) {
  pcg_pair_body<T, N, true>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// ---------------------------------------------------------------------------
// |Phi x|^2 per coefficient (Haar, in-place coefficient layout).
template <typename T, int N>
__device__ __forceinline__ void psi_sq_haar_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  using U = Units<N, ROWS>;
  FIRLS_SLICE_PROLOGUE_S(B.s)
  const size_t off = (size_t)B.x * ROWS * N;
  const C* x = static_cast<const C*>(D.x) + off;
  T* sq = static_cast<T*>(D.sq) + off;
#pragma unroll
  for (int k = 0; k < U::PER; ++k) {
    if (!U::valid(k)) continue;
    const int col = U::col(k), row = U::row(k);
    C v[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = x[(row + s) * N + col];
    haar_col<false>(v, P.L, col);
#pragma unroll
    for (int s = 0; s < 16; ++s) sq[(row + s) * N + col] = (T)cabs2(v[s]);
  }
}
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_psi_sq_haar(Params P) {
  psi_sq_haar_body<T, N>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// Haar PCG update in the textbook order, for the Jacobi and identity
// preconditioners (whose slower inner convergence makes the beta
// recurrence of the fused step less accurate in single precision):
// alpha = <r,z>/<p,q>, x += alpha p, r -= alpha q, and the partials of the
// new <r, P^{-1} r>.  The next k_rowfwd (mode 1) forms z, beta and p.
template <typename T, int N>
__device__ __forceinline__ void update_haar_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  using U = Units<N, ROWS>;
  __shared__ double red[NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if (pcg_skip(P, D, s_, B.x, P.k)) return;
  const size_t off = (size_t)B.x * ROWS * N;
  const double rz = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k), P.nrz);
  const double pq = slot_sum(slot_ptr(D, SLOT_PQ0 + P.k), P.npq);
  const T al = (T)pcg_alpha(P, Blk{B.x, s_}, P.k, rz, pq);
  C* x = static_cast<C*>(D.x) + off;
  C* r = static_cast<C*>(D.r[0]) + off;
  const C* p = static_cast<const C*>(D.p) + off;
  const C* q = static_cast<const C*>(D.q) + off;
  const T* d = static_cast<const T*>(D.d) + off;
  const T rho = (T)P.state[s_].rho, lam = (T)D.lambda;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < U::PER; ++k) {
    if (!U::valid(k)) continue;
    const int col = U::col(k), row = U::row(k);
    C v[16];
    constexpr int CH = 8;   // loads ahead of stores, as in the fused step
#pragma unroll
    for (int s0 = 0; s0 < 16; s0 += CH) {
      C xo[CH], po[CH], qo[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int g = (row + s0 + u) * N + col;
        xo[u] = x[g];
        po[u] = p[g];
        v[s0 + u] = r[g];
        qo[u] = q[g];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int g = (row + s0 + u) * N + col;
        x[g] = xo[u] + po[u] * al;
        v[s0 + u] = v[s0 + u] - qo[u] * al;
        r[g] = v[s0 + u];
      }
    }
    precond_tile<false, N>(v, d + row * N + col, P.L, col, rho, lam, P.precond, acc);
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) slot_wptr(D, SLOT_RZ0 + P.k + 1)[B.x] = tot;
}
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_update_haar(Params P) {
  update_haar_body<T, N>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// After the last PCG iteration (Haar): alpha = <r, z> / <p, q>, x += alpha p.
template <typename T, int N>
__device__ __forceinline__ void last_x_body(const Params& P, const Blk B) {
  constexpr int ROWS = band_rows(N);
  using C = cplx<T>;
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if (pcg_skip(P, D, s_, B.x, P.k)) return;
  const size_t off = (size_t)B.x * ROWS * N;
  const double rz = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k), P.nrz);
  const double pq = slot_sum(slot_ptr(D, SLOT_PQ0 + P.k), P.npq);
  const T al = (T)pcg_alpha(P, Blk{B.x, s_}, P.k, rz, pq);
  C* x = static_cast<C*>(D.x) + off;
  const C* p = static_cast<const C*>(D.p) + off;
  // E elements per thread, CH at a time with their loads ahead of their
  // stores (a band always holds a multiple of NT pixels)
  constexpr int TOT = ROWS * N, E = TOT / NT;
  static_assert(TOT % NT == 0, "band not a multiple of the workgroup");
  constexpr int CH = E % 8 == 0 ? 8 : (E % 4 == 0 ? 4 : (E % 3 == 0 ? 3 : 1));
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += CH) {
    C xv[CH], pv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = threadIdx.x + (e0 + u) * NT;
      xv[u] = x[i];
      pv[u] = p[i];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) x[threadIdx.x + (e0 + u) * NT] = xv[u] + pv[u] * al;
  }
}
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_last_x(Params P) {
  last_x_body<T, N>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// ---------------------------------------------------------------------------
// Precision-only kernels (no FFT size).
// ---------------------------------------------------------------------------

// |D1 x|^2 and |D2 x|^2 per pixel (TV).
template <typename T>
__device__ __forceinline__ void psi_sq_tv_body(const Params& P, const Blk B) {
  using C = cplx<T>;
  FIRLS_SLICE_PROLOGUE_S(B.s)
  const int n = P.n;
  const C* x = static_cast<const C*>(D.x);
  T* sq = static_cast<T*>(D.sq);
  const int total = P.C * n * n;        // D1 rows of every contrast, then D2 rows
  for (int i = B.x * NT * 4 + threadIdx.x, e = 0; e < 4 && i < total; ++e, i += NT) {
    const int r = i / n, c = i - r * n;          // r counts rows of all contrasts
    const int lr = r % n;                         // row within the contrast
    const int rp = lr + 1 == n ? r - lr : r + 1, cp = c + 1 == n ? 0 : c + 1;
    const C v = x[i], z{(T)0, (T)0};
    sq[i] = (T)cabs2(x[rp * n + c] - (tv_cut(P.tvb, lr, n) ? z : v));
    sq[total + i] = (T)cabs2(x[r * n + cp] - (tv_cut(P.tvb, c, n) ? z : v));
  }
}
template <typename T>
__global__ __launch_bounds__(NT) void k_psi_sq_tv(Params P) {
  psi_sq_tv_body<T>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// W_g = (sum_{j in g} |z_j|^2 + eps)^{-1/2} (eq. 12 / eq. 37) and the
// penalty partials sum sqrt(s_g + eps), sum sqrt(s_g).
template <typename T>
__device__ __forceinline__ void group_w_body(const Params& P, const Blk B) {
  __shared__ double red[2 * NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  const T* sq = static_cast<const T*>(D.sq);
  T* W = static_cast<T*>(D.W);
  const int ng = P.shape.n_groups;
  double ae = 0.0, a0 = 0.0;
#pragma unroll
  for (int e = 0; e < GROUPS_PER_WG / NT; ++e) {
    const int g = B.x * GROUPS_PER_WG + e * NT + threadIdx.x;
    if (g < ng) {
      double s = 0.0;
      for (int j = P.shape.gptr[g]; j < P.shape.gptr[g + 1]; ++j) s += (double)sq[P.shape.gidx[j]];
      const double v = sqrt(s + P.eps);
      W[g] = (T)(1.0 / v);
      ae += v;
      a0 += sqrt(s);
    }
  }
  block_sum2(ae, a0, red);
  if (threadIdx.x == 0) {
    slot_wptr(D, SLOT_REG_EPS)[B.x] = ae;
    slot_wptr(D, SLOT_REG0)[B.x] = a0;
  }
}
template <typename T>
__global__ __launch_bounds__(NT) void k_group_w(Params P) {
  group_w_body<T>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// d_j = sum over groups containing j of W_g (diag(G^T W G), eq. 13).
template <typename T>
__device__ __forceinline__ void group_d_body(const Params& P, const Blk B) {
  FIRLS_SLICE_PROLOGUE_S(B.s)
  const T* W = static_cast<const T*>(D.W);
  T* d = static_cast<T*>(D.d);
  const int nc = P.shape.n_coef;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int j = B.x * NT * 4 + e * NT + threadIdx.x;
    if (j < nc) {
      double s = 0.0;
      for (int t = P.shape.tptr[j]; t < P.shape.tptr[j + 1]; ++t) s += (double)W[P.shape.tidx[t]];
      d[j] = (T)s;
    }
  }
}
template <typename T>
__global__ __launch_bounds__(NT) void k_group_d(Params P) {
  group_d_body<T>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


// TV preconditioner z = M^{-1} r with M = (D + L) D^{-1} (D + U) the
// symmetric Gauss-Seidel factors of P = rho I + lambda (D1^T W1 D1 +
// D2^T W2 D2) (eq. 40; the L and U of eqs. 42-43) in red-black order:
//   y_red = r / a;  y_black = (r - sum P_pq y_q) / a;
//   z_black = y_black;  z_red = y_red - (sum P_pq z_q) / a.
// With PC_JACOBI z = r / a (a = diag P = diag S) and with PC_NONE z = r.
// Each workgroup owns a TV_TR x TV_TC tile and recomputes a two-pixel halo
// of r (and a three-pixel halo of the weights) in LDS.  In UP_STEP mode
// the residual is read from r[k & 1] and written to r[(k + 1) & 1], so a
// halo never sees a neighbour's update; x and p of the thread's own pixels
// are loaded first, so their latency overlaps the preconditioner.
template <typename T, int MODE>
__device__ __forceinline__ void update_tv_body(const Params& P, const Blk B) {
  using C = cplx<T>;
  constexpr int H = 2, RR = TV_TR + 2 * H, RC = TV_TC + 2 * H, WR = RR + 1, WC = RC + 1;
  constexpr int OUT = TV_TR * TV_TC / NT;   // pixels per thread
  static_assert(OUT * NT == TV_TR * TV_TC, "whole tile per workgroup");
  static_assert((RC - 2) % 2 == 0, "as many black as red cells in an interior row");
  __shared__ C rn[RR * RC];
  __shared__ C y[RR * RC];
  __shared__ T av[RR * RC];
  __shared__ T w1[WR * WC];
  __shared__ T w2[WR * WC];
  __shared__ double red[NT / 64];
  FIRLS_SLICE_PROLOGUE_S(B.s)
  if constexpr (MODE == UP_STEP) {
    if (pcg_skip(P, D, s_, B.x, P.k)) return;
  }
  const int n = P.n;
  const int tiles_x = n / TV_TC;
  // Workgroup i runs on XCD i mod 8, each XCD with its own L2: the tiles
  // are dealt out so each XCD gets a contiguous run of them (whole tile
  // rows), and neighbouring tiles, whose halos overlap, share an L2.
  const int tiles = P.nrz;
  const int tile = (tiles & 7) ? B.x : (B.x & 7) * (tiles >> 3) + (B.x >> 3);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  // tiles run over the rows of all contrasts; a tile lies in one contrast,
  // whose image (and D1, D2 weights) the pointers below select
  const int ch = (ty * TV_TR) / n;
  const int r0 = ty * TV_TR - ch * n, c0 = tx * TV_TC;
  const size_t cb = (size_t)ch * n * n;
  const int par = (MODE == UP_STEP) ? (P.k & 1) : 0;
  const C* rin = static_cast<const C*>(D.r[par]) + cb;
  const T* d1 = static_cast<const T*>(D.d) + cb;
  const T* d2 = static_cast<const T*>(D.d) + (size_t)P.C * n * n + cb;
  C* x = static_cast<C*>(D.x) + cb;
  const C* p = static_cast<const C*>(D.p) + cb;
  // region cell (lr, lc) is red when (par0 + lr + lc) is even
  const int par0 = (r0 + c0) & 1;
  C xv[OUT], pv[OUT];
  if constexpr (MODE == UP_STEP) {
#pragma unroll
    for (int e = 0; e < OUT; ++e) {
      const int i = threadIdx.x + e * NT;
      const size_t g = (size_t)(r0 + i / TV_TC) * n + (c0 + i % TV_TC);
      xv[e] = x[g];
      pv[e] = p[g];
    }
  }
  T al = (T)0;
  if constexpr (MODE != UP_INIT) {
    const double rz = slot_sum(slot_ptr(D, SLOT_RZ0 + P.k), P.nrz);
    const double pq = slot_sum(slot_ptr(D, SLOT_PQ0 + P.k), P.npq);
    al = (T)pcg_alpha(P, Blk{B.x, s_}, P.k, rz, pq);
  }
  const C* q = static_cast<const C*>(D.q) + cb;
  // coupling weights: slots that hold identity rows (tvb) couple nothing
  for (int i = threadIdx.x; i < WR * WC; i += NT) {
    const int lr = i / WC, lc = i - lr * WC;
    const int gr = wrapi(r0 - H - 1 + lr, n), gc = wrapi(c0 - H - 1 + lc, n);
    const size_t g = (size_t)gr * n + gc;
    w1[i] = tv_cut(P.tvb, gr, n) ? (T)0 : d1[g];
    w2[i] = tv_cut(P.tvb, gc, n) ? (T)0 : d2[g];
  }
  for (int i = threadIdx.x; i < RR * RC; i += NT) {
    const int lr = i / RC, lc = i - lr * RC;
    const size_t g = (size_t)wrapi(r0 - H + lr, n) * n + wrapi(c0 - H + lc, n);
    C v = rin[g];
    if (MODE == UP_STEP) v = v - q[g] * al;
    rn[i] = v;
  }
  __syncthreads();
  const T rho = (T)P.state[s_].rho, lam = (T)D.lambda;
  // weights around region cell (lr, lc): W1(p) at w(lr+1, lc+1), W1(p-e1) at
  // w(lr, lc+1), W2(p) at w(lr+1, lc+1), W2(p-e2) at w(lr+1, lc).
#define W1P(lr, lc) w1[((lr) + 1) * WC + (lc) + 1]
#define W1M(lr, lc) w1[(lr) * WC + (lc) + 1]
#define W2P(lr, lc) w2[((lr) + 1) * WC + (lc) + 1]
#define W2M(lr, lc) w2[((lr) + 1) * WC + (lc)]
  for (int i = threadIdx.x; i < RR * RC; i += NT) {
    const int lr = i / RC, lc = i - lr * RC;
    T a = rho + lam * (W1P(lr, lc) + W1M(lr, lc) + W2P(lr, lc) + W2M(lr, lc));
    if (P.tvb) {
      // the identity-row slot of pixel row 0 / column 0 adds its weight to
      // the diagonal only
      const int gr = wrapi(r0 - H + lr, n), gc = wrapi(c0 - H + lc, n);
      if (gr == 0) a += lam * d1[(size_t)(n - 1) * n + gc];
      if (gc == 0) a += lam * d2[(size_t)gr * n + n - 1];
    }
    av[i] = a;
    const bool red_cell = ((r0 - H + lr + c0 - H + lc) & 1) == 0;
    if (red_cell) y[i] = rn[i] * ((T)1 / a);
  }
  __syncthreads();
  const int pc = P.precond;
  // the black cells of the interior only (half of each row), so no lane
  // idles on a red one
  constexpr int BPR = (RC - 2) / 2;   // black cells per interior row
  for (int i = threadIdx.x; pc == PC_PAPER && i < (RR - 2) * BPR; i += NT) {
    const int row = i / BPR;
    const int lr = 1 + row;
    const int lc = 1 + ((par0 + lr) & 1) + 2 * (i - row * BPR);
    const int o = lr * RC + lc;
    const C s = y[o + RC] * W1P(lr, lc) + y[o - RC] * W1M(lr, lc) + y[o + 1] * W2P(lr, lc) + y[o - 1] * W2M(lr, lc);
    y[o] = (rn[o] + s * lam) * ((T)1 / av[o]);
  }
  __syncthreads();
  C* z = static_cast<C*>(D.z) + cb;
  C* rout = static_cast<C*>(D.r[par ^ 1]) + cb;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < OUT; ++e) {
    const int i = threadIdx.x + e * NT;
    const int lr = H + i / TV_TC, lc = H + i % TV_TC;
    const int o = lr * RC + lc;
    const bool red_cell = ((par0 + lr + lc) & 1) == 0;
    C zz = pc == PC_PAPER ? y[o] : (pc == PC_JACOBI ? rn[o] * ((T)1 / av[o]) : rn[o]);
    if (pc == PC_PAPER && red_cell) {
      const C s = y[o + RC] * W1P(lr, lc) + y[o - RC] * W1M(lr, lc) + y[o + 1] * W2P(lr, lc) + y[o - 1] * W2M(lr, lc);
      zz = zz + s * (lam / av[o]);
    }
    const size_t g = (size_t)(r0 + lr - H) * n + (c0 + lc - H);
    z[g] = zz;
    acc += cdot(rn[o], zz);
    if (MODE == UP_STEP) {
      rout[g] = rn[o];
      x[g] = xv[e] + pv[e] * al;
    }
  }
#undef W1P
#undef W1M
#undef W2P
#undef W2M
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) slot_wptr(D, SLOT_RZ0 + (MODE == UP_STEP ? P.k + 1 : 0))[tile] = tot;
}
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_update_tv(Params P) {
  update_tv_body<T, MODE>(P, Blk{(int)blockIdx.x, P.list[blockIdx.y]});
}


}  // namespace firls

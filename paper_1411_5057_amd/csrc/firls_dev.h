// Device building blocks: complex arithmetic, small DFTs, the LDS-staged
// mixed-radix FFT used by the row and column passes, tile-local Haar in
// LDS, and deterministic FP64 workgroup reductions.
#pragma once
#include <hip/hip_runtime.h>
#include "firls_types.h"

namespace firls {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> operator*(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// Sums of two products are written as one explicit fused multiply-add and
// one product.  Left to contraction, the compiler picks which product to
// fuse per kernel, so the same formula could round differently in two
// kernels that must agree bitwise (the FFT passes of the paired and the
// separate PCG launches, say).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {fmat(a.x, b.x, -(a.y * b.y)), fmat(a.x, b.y, a.y * b.x)};
}
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
  return {fmat(a.x, b.x, a.y * b.y), fmat(a.y, b.x, -(a.x * b.y))};
}
template <typename T> __device__ __forceinline__ double cabs2(cplx<T> a) {
  return fmat((double)a.x, (double)a.x, (double)a.y * (double)a.y);
}
template <typename T> __device__ __forceinline__ double cdot(cplx<T> a, cplx<T> b) {  // Re(conj(a) b)
  return fmat((double)a.x, (double)b.x, (double)a.y * (double)b.y);
}
template <typename T> __device__ __forceinline__ T cabs2t(cplx<T> a) { return fmat(a.x, a.x, a.y * a.y); }

// 1 / (rho + lambda d) of the pseudo-diagonal preconditioner (eq. 17).  Every
// kernel that applies P^{-1} or sums <v, P^{-1} v> takes it from here, so
// all of them use the same operator (single precision: the hardware
// reciprocal, within 1 ulp; the preconditioner need not be exact, only
// symmetric positive definite and the same everywhere).
__device__ __forceinline__ float pc_inv(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double pc_inv(double v) { return 1.0 / v; }
// 1 / (rho + lambda d) with the denominator as one fused multiply-add, so
// it rounds the same wherever it is formed (a separate lambda d product,
// shared with the regulariser, would round it differently).
__device__ __forceinline__ float pc_inv(float rho, float lam, float d) { return pc_inv(__builtin_fmaf(lam, d, rho)); }
__device__ __forceinline__ double pc_inv(double rho, double lam, double d) { return pc_inv(__builtin_fma(lam, d, rho)); }

// cos(2 pi e / 16) and sin(2 pi e / 16), e = 0..15.
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};

// exp(-+ 2 pi i e / R) for R dividing 16 (forward: minus sign).
template <typename T, int R, bool INV>
__device__ __forceinline__ cplx<T> unit_root(int e) {
  const int k = (e * (16 / R)) & 15;
  const T c = (T)kC16[k];
  const T s = (T)kS16[k];
  return INV ? cplx<T>{c, s} : cplx<T>{c, -s};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: X[k] = sum_r v[r] exp(-+2 pi i r k / R).
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV> struct SmallDFT;

template <typename T, bool INV> struct SmallDFT<T, 2, INV> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, bool INV> struct SmallDFT<T, 3, INV> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    const T h = (T)0.86602540378443865;  // sqrt(3) / 2
    cplx<T> a = v[0], s = v[1] + v[2], d = v[1] - v[2];
    cplx<T> m = a - s * (T)0.5;
    // forward: X1 = m - i h d, X2 = m + i h d; inverse swaps the signs
    cplx<T> ihd = INV ? cplx<T>{-h * d.y, h * d.x} : cplx<T>{h * d.y, -h * d.x};
    v[0] = a + s;
    v[1] = m + ihd;
    v[2] = m - ihd;
  }
};

template <typename T, bool INV> struct SmallDFT<T, 4, INV> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> s0 = v[0] + v[2], d0 = v[0] - v[2];
    cplx<T> s1 = v[1] + v[3], d1 = v[1] - v[3];
    // forward multiplies d1 by -i, inverse by +i
    cplx<T> jd1 = INV ? cplx<T>{-d1.y, d1.x} : cplx<T>{d1.y, -d1.x};
    v[0] = s0 + s1;
    v[2] = s0 - s1;
    v[1] = d0 + jd1;
    v[3] = d0 - jd1;
  }
};

// R = A * B: input n = m + A s, output k = k1 + B k2;
// X[k1 + B k2] = sum_m w_A^{m k2} ( w_R^{m k1} sum_s v[m + A s] w_B^{s k1} ).
template <typename T, int A, int B, bool INV>
__device__ __forceinline__ void dft_composite(cplx<T>* v) {
  constexpr int R = A * B;
  cplx<T> y[A][B];
#pragma unroll
  for (int m = 0; m < A; ++m) {
    cplx<T> tmp[B];
#pragma unroll
    for (int s = 0; s < B; ++s) tmp[s] = v[m + A * s];
    SmallDFT<T, B, INV>::run(tmp);
#pragma unroll
    for (int k1 = 0; k1 < B; ++k1) y[m][k1] = (m * k1 == 0) ? tmp[k1] : cmul(tmp[k1], unit_root<T, R, INV>(m * k1));
  }
#pragma unroll
  for (int k1 = 0; k1 < B; ++k1) {
    cplx<T> tmp[A];
#pragma unroll
    for (int m = 0; m < A; ++m) tmp[m] = y[m][k1];
    SmallDFT<T, A, INV>::run(tmp);
#pragma unroll
    for (int k2 = 0; k2 < A; ++k2) v[k1 + B * k2] = tmp[k2];
  }
}

template <typename T, bool INV> struct SmallDFT<T, 8, INV> {
  __device__ __forceinline__ static void run(cplx<T>* v) { dft_composite<T, 2, 4, INV>(v); }
};
template <typename T, bool INV> struct SmallDFT<T, 16, INV> {
  __device__ __forceinline__ static void run(cplx<T>* v) { dft_composite<T, 4, 4, INV>(v); }
};

// ---------------------------------------------------------------------------
// Radix plans.  Forward stages use R0, R1, R2 in order; the inverse uses the
// reverse order (a Stockham pass accepts any order of the factors).
// ---------------------------------------------------------------------------
template <int N> struct Plan;
template <> struct Plan<16>  { static constexpr int S = 1, R0 = 16, R1 = 1,  R2 = 1; };
template <> struct Plan<32>  { static constexpr int S = 2, R0 = 8,  R1 = 4,  R2 = 1; };
template <> struct Plan<48>  { static constexpr int S = 2, R0 = 16, R1 = 3,  R2 = 1; };
template <> struct Plan<64>  { static constexpr int S = 2, R0 = 16, R1 = 4,  R2 = 1; };
template <> struct Plan<96>  { static constexpr int S = 3, R0 = 16, R1 = 2,  R2 = 3; };
template <> struct Plan<128> { static constexpr int S = 2, R0 = 16, R1 = 8,  R2 = 1; };
template <> struct Plan<192> { static constexpr int S = 3, R0 = 16, R1 = 4,  R2 = 3; };
template <> struct Plan<256> { static constexpr int S = 2, R0 = 16, R1 = 16, R2 = 1; };
template <> struct Plan<384> { static constexpr int S = 3, R0 = 16, R1 = 8,  R2 = 3; };
template <> struct Plan<512> { static constexpr int S = 3, R0 = 16, R1 = 16, R2 = 2; };

// LDS layout of LINES lines of N complex values: one pad slot every 16
// values and an odd line stride keep both line-major and position-major
// lane orders free of heavy bank conflicts.
template <int N> struct LdsLayout {
  static constexpr int LS = N + N / 16 + 1;
  __device__ __forceinline__ static int at(int line, int pos) { return line * LS + pos + (pos >> 4); }
};

enum Map : int { ROWMAP = 0, COLMAP = 1 };

// One Stockham stage (Govindaraju et al. formulation): butterfly j of a
// line reads v[r] = in[j + r N/R], applies twiddles w_{NS R}^{(j mod NS) r},
// takes a radix-R DFT and writes out[(j / NS) NS R + j mod NS + r NS].
template <typename T, int N, int R, int NS, int LINES, int MAP, bool INV>
struct Stage {
  static constexpr int NB = N / R;
  static constexpr int TOT = LINES * NB;
  static constexpr int ITER = (TOT + NT - 1) / NT;

  __device__ __forceinline__ static void decode(int b, int& line, int& j) {
    if (MAP == ROWMAP) { line = b / NB; j = b - line * NB; }
    else { j = b / LINES; line = b - j * LINES; }
  }

  template <class Src>
  __device__ __forceinline__ static void load(cplx<T> (&v)[ITER][R], Src& src, const cplx<T>* tw,
                                              int tid = threadIdx.x) {
#pragma unroll
    for (int i = 0; i < ITER; ++i) {
      const int b = tid + i * NT;
      if (TOT % NT != 0 && b >= TOT) continue;
      int line, j;
      decode(b, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src(line, j + r * NB);
      if (NS > 1) {
        const int step = (j % NS) * (N / (NS * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[r * step];
          if (INV) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      SmallDFT<T, R, INV>::run(v[i]);
    }
  }

  template <class Dst>
  __device__ __forceinline__ static void store(cplx<T> (&v)[ITER][R], Dst& dst, int tid = threadIdx.x) {
#pragma unroll
    for (int i = 0; i < ITER; ++i) {
      const int b = tid + i * NT;
      if (TOT % NT != 0 && b >= TOT) continue;
      int line, j;
      decode(b, line, j);
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst(line, base + r * NS, v[i][r]);
    }
  }
};

template <typename T, int N>
struct LdsIO {
  cplx<T>* buf;
  __device__ __forceinline__ cplx<T> operator()(int line, int pos) const { return buf[LdsLayout<N>::at(line, pos)]; }
  __device__ __forceinline__ void operator()(int line, int pos, cplx<T> v) const { buf[LdsLayout<N>::at(line, pos)] = v; }
};

// FFT (INV = false: exp(-...), unnormalised) of LINES lines of length N.
// The first stage reads src(line, pos), the last writes dst(line, pos, v);
// intermediate stages go through ``lds`` (LINES x LdsLayout<N>::LS).
// Barriers bracket every LDS phase, so src / dst may themselves be LDS.
// ``tid`` is the work-item index the butterflies are assigned by; a kernel
// with two FFTs far apart passes a copy the compiler cannot see through, so
// the second one's addresses are recomputed instead of being kept live (and
// spilled) from the first.
template <typename T, int N, int LINES, int MAP, bool INV, class Src, class Dst>
__device__ __forceinline__ void fft_lines(cplx<T>* lds, const cplx<T>* tw, Src src, Dst dst, int tid = threadIdx.x) {
  using P = Plan<N>;
  constexpr int A0 = INV ? (P::S == 3 ? P::R2 : (P::S == 2 ? P::R1 : P::R0)) : P::R0;
  constexpr int A1 = INV ? (P::S == 3 ? P::R1 : P::R0) : P::R1;
  constexpr int A2 = INV ? P::R0 : P::R2;
  LdsIO<T, N> io{lds};
  using S0 = Stage<T, N, A0, 1, LINES, MAP, INV>;
  cplx<T> v0[S0::ITER][A0];
  S0::load(v0, src, tw, tid);
  __syncthreads();
  if constexpr (P::S == 1) {
    S0::store(v0, dst, tid);
    __syncthreads();
  } else {
    S0::store(v0, io, tid);
    __syncthreads();
    using S1 = Stage<T, N, A1, A0, LINES, MAP, INV>;
    cplx<T> v1[S1::ITER][A1];
    S1::load(v1, io, tw, tid);
    __syncthreads();
    if constexpr (P::S == 2) {
      S1::store(v1, dst, tid);
      __syncthreads();
    } else {
      S1::store(v1, io, tid);
      __syncthreads();
      using S2 = Stage<T, N, A2, A0 * A1, LINES, MAP, INV>;
      cplx<T> v2[S2::ITER][A2];
      S2::load(v2, io, tw, tid);
      __syncthreads();
      S2::store(v2, dst, tid);
      __syncthreads();
    }
  }
}

// Forward FFT of LINES lines, a pointwise map of the spectrum, inverse FFT:
// dst(line, pos, IFFT(mid(line, k, FFT(src))[k])).  In the Stockham order the
// last forward stage (radix RL) leaves butterfly j of a line holding the
// spectrum at positions j + r N / RL, exactly the inputs of butterfly j of
// the first inverse stage (same radix, no twiddles), so the spectrum stays
// in registers between the two transforms: one LDS round trip and two
// barriers fewer than two fft_lines calls.
// Which spectrum positions this thread holds between the two transforms:
// its i-th butterfly (i < ITER) is (line, j) and holds positions
// j + r NBL, r < RL.
template <typename T, int N, int LINES, int MAP>
struct FwdInvMap {
  using P = Plan<N>;
  static constexpr int RL = P::S == 3 ? P::R2 : (P::S == 2 ? P::R1 : P::R0);
  static constexpr int NBL = N / RL;
  using L = Stage<T, N, RL, NBL, LINES, MAP, false>;
  static constexpr int ITER = L::ITER;
  __device__ __forceinline__ static bool at(int i, int& line, int& j) {
    const int b = threadIdx.x + i * NT;
    if (L::TOT % NT != 0 && b >= L::TOT) return false;
    L::decode(b, line, j);
    return true;
  }
};

// ``mid(i, r, line, pos, v)`` gets the spectrum value v at (line, pos), the
// r-th value of this thread's i-th butterfly (FwdInvMap).
template <typename T, int N, int LINES, int MAP, class Src, class Mid, class Dst>
__device__ __forceinline__ void fft_lines_fwd_inv(cplx<T>* lds, const cplx<T>* tw, Src src, Mid mid, Dst dst) {
  using P = Plan<N>;
  using Map = FwdInvMap<T, N, LINES, MAP>;
  constexpr int RL = Map::RL;
  constexpr int NBL = Map::NBL;
  LdsIO<T, N> io{lds};
  using L = Stage<T, N, RL, NBL, LINES, MAP, false>;    // last forward stage
  using I0 = Stage<T, N, RL, 1, LINES, MAP, true>;      // first inverse stage
  cplx<T> v[L::ITER][RL];
  if constexpr (P::S == 1) {
    L::load(v, src, tw);
  } else {
    using S0 = Stage<T, N, P::R0, 1, LINES, MAP, false>;
    {
      cplx<T> v0[S0::ITER][P::R0];
      S0::load(v0, src, tw);
      __syncthreads();
      S0::store(v0, io);
      __syncthreads();
    }
    if constexpr (P::S == 3) {
      using S1 = Stage<T, N, P::R1, P::R0, LINES, MAP, false>;
      cplx<T> v1[S1::ITER][P::R1];
      S1::load(v1, io, tw);
      __syncthreads();
      S1::store(v1, io);
      __syncthreads();
    }
    L::load(v, io, tw);
  }
#pragma unroll
  for (int i = 0; i < L::ITER; ++i) {
    int line, j;
    if (!Map::at(i, line, j)) continue;
#pragma unroll
    for (int r = 0; r < RL; ++r) v[i][r] = mid(i, r, line, j + r * NBL, v[i][r]);
    SmallDFT<T, RL, true>::run(v[i]);
  }
  if constexpr (P::S == 1) {
    I0::store(v, dst);
    __syncthreads();
  } else {
    __syncthreads();   // the last forward stage's LDS reads are done
    I0::store(v, io);
    __syncthreads();
    if constexpr (P::S == 2) {
      using I1 = Stage<T, N, P::R0, RL, LINES, MAP, true>;
      cplx<T> u[I1::ITER][P::R0];
      I1::load(u, io, tw);
      __syncthreads();
      I1::store(u, dst);
      __syncthreads();
    } else {
      using I1 = Stage<T, N, P::R1, RL, LINES, MAP, true>;
      {
        cplx<T> u[I1::ITER][P::R1];
        I1::load(u, io, tw);
        __syncthreads();
        I1::store(u, io);
        __syncthreads();
      }
      using I2 = Stage<T, N, P::R0, RL * P::R1, LINES, MAP, true>;
      cplx<T> u[I2::ITER][P::R0];
      I2::load(u, io, tw);
      __syncthreads();
      I2::store(u, dst);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Register-resident tile-local orthonormal Haar.
//
// An L-level Haar of the whole image only mixes pixels inside aligned
// tiles of side 2^L, so every tile is transformed on its own.  A thread
// holds v[s], s < 16, the 16 rows of one image column inside a 16-row
// group; neighbouring columns sit in neighbouring lanes.  One level with
// stride st = 2^(lev-1) maps each 2x2 block [a b; c d] of the current
// approximation (rows s, s+st; columns c, c+st, s and c multiples of 2st) to
//   left column : (a+b+c+d)/2 at row s, (a+b-c-d)/2 at row s+st
//   right column: (a-b+c-d)/2 at row s, (a-b-c+d)/2 at row s+st,
// keeping every coefficient on the pixel position it is computed on (the
// in-place, interleaved layout).  This 2x2 map is symmetric and its own
// inverse, so the inverse transform applies the same level step with the
// levels in reverse order.  Rows pair inside the thread; columns pair with
// lane ^ st through cross-lane shuffles.  The library's coefficient layout
// (weights d, |Psi x|^2) is this in-place layout.
// ---------------------------------------------------------------------------
// The value of lane ^ ST (ST = 1, 2, 4 or 8: inside a row of 16 lanes)
// through DPP moves instead of an LDS permute: quad_perm [1,0,3,2] and
// [2,3,0,1] for 1 and 2, row_ror:8 for 8, and for 4 the lane takes
// row_ror:12 (lane + 4) or row_ror:4 (lane - 4) by its bit 2.
template <int ST>
__device__ __forceinline__ int xor_lane_i(int x) {
  static_assert(ST == 1 || ST == 2 || ST == 4 || ST == 8, "stride inside a DPP row");
  if constexpr (ST == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
  else if constexpr (ST == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
  else if constexpr (ST == 8) return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
  else {
    const int up = __builtin_amdgcn_update_dpp(0, x, 0x12C, 0xF, 0xF, false);
    const int dn = __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);
    return (threadIdx.x & 4) ? dn : up;
  }
}
template <int ST>
__device__ __forceinline__ float xor_lane(float v) { return __int_as_float(xor_lane_i<ST>(__float_as_int(v))); }
template <int ST>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane_i<ST>((int)(b & 0xFFFFFFFFll)), hi = xor_lane_i<ST>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <int ST, typename T>
__device__ __forceinline__ cplx<T> xor_lane_c(cplx<T> v) {
  return cplx<T>{xor_lane<ST>(v.x), xor_lane<ST>(v.y)};
}

template <int ST, typename T>
__device__ __forceinline__ void haar_level(cplx<T> (&v)[16], int col) {
  const bool active = (col & (ST - 1)) == 0;
  const bool right = (col & ST) != 0;
  const T h = (T)0.5;
#pragma unroll
  for (int s = 0; s < 16; s += 2 * ST) {
    const cplx<T> S = v[s] + v[s + ST];
    const cplx<T> D = v[s] - v[s + ST];
    const cplx<T> So = xor_lane_c<ST>(S);
    const cplx<T> Do = xor_lane_c<ST>(D);
    if (active) {
      v[s] = (right ? So - S : S + So) * h;
      v[s + ST] = (right ? Do - D : D + Do) * h;
    }
  }
}

template <bool INV, typename T>
__device__ __forceinline__ void haar_col(cplx<T> (&v)[16], int L, int col) {
  if (!INV) {
    if (L >= 1) haar_level<1>(v, col);
    if (L >= 2) haar_level<2>(v, col);
    if (L >= 3) haar_level<4>(v, col);
    if (L >= 4) haar_level<8>(v, col);
  } else {
    if (L >= 4) haar_level<8>(v, col);
    if (L >= 3) haar_level<4>(v, col);
    if (L >= 2) haar_level<2>(v, col);
    if (L >= 1) haar_level<1>(v, col);
  }
}

// diag(Phi^T diag(d) Phi) from d (both in the in-place layout), in
// registers: every coefficient reaches a pixel through one chain of level
// steps with entries +-1/2, so the squared entries form the same tree with
// every entry 1/4.  The transpose therefore replaces each 2x2 block by the
// mean of its four values, levels from the coarsest down.
template <int ST, typename T>
__device__ __forceinline__ void haar_diag_level(T (&v)[16], int col) {
  const bool active = (col & (ST - 1)) == 0;
#pragma unroll
  for (int s = 0; s < 16; s += 2 * ST) {
    const T S = v[s] + v[s + ST];
    const T So = xor_lane<ST>(S);
    if (active) v[s] = v[s + ST] = (S + So) * (T)0.25;
  }
}

template <typename T>
__device__ __forceinline__ void haar_diag_col(T (&v)[16], int L, int col) {
  if (L >= 4) haar_diag_level<8>(v, col);
  if (L >= 3) haar_diag_level<4>(v, col);
  if (L >= 2) haar_diag_level<2>(v, col);
  if (L >= 1) haar_diag_level<1>(v, col);
}

// Work units of a band of ROWS rows and N columns: unit u covers column
// u % N of the 16-row group u / N.  Thread t owns units t, t + NT, ...
template <int N, int ROWS>
struct Units {
  static constexpr int COUNT = (ROWS / 16) * N;
  static constexpr int PER = (COUNT + NT - 1) / NT;
  __device__ __forceinline__ static bool valid(int k) { return COUNT % NT == 0 || (int)threadIdx.x + k * NT < COUNT; }
  __device__ __forceinline__ static int col(int k) { return ((int)threadIdx.x + k * NT) % N; }
  __device__ __forceinline__ static int row(int k) { return (((int)threadIdx.x + k * NT) / N) * 16; }
};

// ---------------------------------------------------------------------------
// Group weights.
// ---------------------------------------------------------------------------
// A padded list of compile-time width W (1, 2, 4 or 8 entries) in one load.
template <int W>
__device__ __forceinline__ void ell_row_w(const uint16_t* p, uint16_t (&e)[W]) {
  static_assert(W == 1 || W == 2 || W == 4 || W == 8, "list width");
  if constexpr (W == 1) {
    e[0] = p[0];
  } else if constexpr (W == 2) {
    const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
    e[0] = (uint16_t)v; e[1] = (uint16_t)(v >> 16);
  } else if constexpr (W == 4) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    e[0] = (uint16_t)v.x; e[1] = (uint16_t)(v.x >> 16); e[2] = (uint16_t)v.y; e[3] = (uint16_t)(v.y >> 16);
  } else {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    e[0] = (uint16_t)v.x; e[1] = (uint16_t)(v.x >> 16); e[2] = (uint16_t)v.y; e[3] = (uint16_t)(v.y >> 16);
    e[4] = (uint16_t)v.z; e[5] = (uint16_t)(v.z >> 16); e[6] = (uint16_t)v.w; e[7] = (uint16_t)(v.w >> 16);
  }
}

// Sum over a list of the LDS values it names (0xFFFF pads), in list order.
template <int W, typename T>
__device__ __forceinline__ T ell_gather(const uint16_t (&e)[W], const T* vals) {
  T s = (T)0;
#pragma unroll
  for (int m = 0; m < W; ++m)
    if (e[m] != 0xFFFFu) s += vals[e[m]];
  return s;
}

// W = (s2 + eps)^(-1/2) (eq. 12), ve = sqrt(s2 + eps) and v0 = sqrt(s2) (the
// smoothed and plain penalty terms) in the working precision: FP32 uses the
// hardware square root and reciprocal square root (about 1 ulp), FP64 the
// correctly rounded operations.
__device__ __forceinline__ void group_weight(float s2, float eps, float& w, float& ve, float& v0) {
  const float q = s2 + eps;
  w = __builtin_amdgcn_rsqf(q);
  ve = __builtin_amdgcn_sqrtf(q);
  v0 = __builtin_amdgcn_sqrtf(s2);
}
__device__ __forceinline__ void group_weight(double s2, double eps, double& w, double& ve, double& v0) {
  ve = sqrt(s2 + eps);
  w = 1.0 / ve;
  v0 = sqrt(s2);
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions.
// ---------------------------------------------------------------------------
// Sum over the 64 lanes; every lane gets the same bits: pairs inside rows
// of 16 lanes through DPP (lane ^ 1, 2, 4, 8), then lane ^ 16 through a
// swizzle, then lane 0's and lane 32's halves read as scalars and added in
// one order.
__device__ __forceinline__ double swizzle_xor16(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xFFFFFFFFll), (16 << 10) | 0x1F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), (16 << 10) | 0x1F);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += xor_lane<1>(v);
  v += xor_lane<2>(v);
  v += xor_lane<4>(v);
  v += xor_lane<8>(v);
  v += swizzle_xor16(v);
  return read_lane(v, 0) + read_lane(v, 32);
}

// Sum over the workgroup; every thread gets the result.  ``red`` is a
// __shared__ double[NT / 64] scratch.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// Two sums over the workgroup with one pair of barriers; ``red`` holds
// 2 NT / 64 doubles.  Each result is bitwise what block_sum gives.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[wid] = a;
    red[NT / 64 + wid] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    sa += red[w];
    sb += red[NT / 64 + w];
  }
  a = sa;
  b = sb;
}

// Sum of ``count`` partials of a slot, in a fixed order, formed by every
// wave on its own (lane l adds partials l, l + 64, ..., then a butterfly):
// no barrier, and every wave of every workgroup gets the same bits.
__device__ __forceinline__ double slot_sum(const double* slot, int count) {
  double v = 0.0;
  for (int i = threadIdx.x & 63; i < count; i += 64) v += slot[i];
  return wave_sum(v);
}

// The same over partials that other workgroups of the running launch wrote
// with device-coherent stores (loads that bypass non-coherent caches).
__device__ __forceinline__ double slot_sum_coherent(const double* slot, int count) {
  double v = 0.0;
  for (int i = threadIdx.x & 63; i < count; i += 64)
    v += __hip_atomic_load(slot + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return wave_sum(v);
}

__device__ __forceinline__ const double* slot_ptr(const SliceDesc& D, int s) { return D.parts + (size_t)s * PMAX; }
__device__ __forceinline__ double* slot_wptr(const SliceDesc& D, int s) { return D.parts + (size_t)s * PMAX; }

}  // namespace firls

// Products with a dense sensing matrix A (random projections of Section
// 5.2), batched over the slices of one launch.
//
// The real matrix A (Mp x N, row-major, N = n^2, rows >= M zero) multiplies
// the complex vectors of up to GEMM_BS slices at a time: the real and
// imaginary parts of slice j are columns 2j and 2j+1 of the right operand,
// read in place from the slice's own vector (x, p, y or b).  Tiles of
// GEMM_BM rows x 64 columns run on MFMA (FP32: v_mfma_f32_16x16x4f32, FP64:
// v_mfma_f64_16x16x4f64), four waves of GEMM_BM/2 x 32, with 32-deep slices of both
// operands staged in LDS and the next slices fetched meanwhile.  Per-slice
// partial sums (data term, ||A p||^2) are reduced in a fixed order: one
// partial per row tile.
#include "firls_inst.h"

namespace firls {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using V = f32x4;
  __device__ __forceinline__ static V mac(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element (row, col) of a 16 x 16 tile held by lane, register r
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
  using V = f64x4;
  __device__ __forceinline__ static V mac(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int BK = GEMM_BK;     // depth of one LDS stage
constexpr int BN = 2 * GEMM_BS; // real columns per tile
constexpr int MI = GEMM_BM / 32;   // 16-row MFMA tiles per wave (two waves share the rows)
constexpr int WR = GEMM_BM / 2;    // rows per wave
constexpr int NI = BN / 32;        // 16-column MFMA tiles per wave (two waves share the columns)
constexpr int WC = BN / 2;         // columns per wave
// LDS row padding: a stride of 16 banks (mod 32) puts the four k rows one
// MFMA operand read touches on disjoint banks
constexpr int PAD = 16;

}  // namespace

// Epilogue of one GEMM_BM x 64 output tile: thread (wave, lane) owns the MFMA
// output positions (mi, ni, r); ``val(mi, ni, r)`` gives the finished sum.
// Scatters to the slices' vectors and, for G_AX_R0 / G_AP, writes one
// per-slice partial of the squares (fixed reduction order).
template <typename T, int MODE, class Val>
__device__ __forceinline__ void gemm_epilogue(const Params& P, int row0, int j0, Val val,
                                              double (&colpart)[2][BN]) {
  using M = Mfma<T>;
  constexpr bool PARTIAL = (MODE == G_AX_R0 || MODE == G_AP);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * WR, wc = (wave & 1) * WC;
  const int Mv = P.shape.M;
  double csq[NI];
#pragma unroll
  for (int ni = 0; ni < NI; ++ni) csq[ni] = 0.0;
#pragma unroll
  for (int ni = 0; ni < NI; ++ni) {
    const int col = wc + 16 * ni + (lane & 15);
    const int j = j0 + (col >> 1), c = col & 1;
    const bool live = j < P.count && P.state[P.list[j]].active;
    T* dst = nullptr;
    const T* bv = nullptr;
    if (live) {
      const SliceDesc& D = P.desc[P.list[j]];
      dst = static_cast<T*>(MODE == G_ATB ? D.x : (MODE == G_ATY ? D.t : D.y));
      bv = static_cast<const T*>(D.b);
    }
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + 16 * mi + M::row(lane, r);
        T v = val(mi, ni, r);
        if (MODE == G_AX_R0) v = (live && gr < Mv) ? bv[2 * (size_t)gr + c] - v : (T)0;
        if (live) dst[2 * (size_t)gr + c] = v;
        if (PARTIAL) csq[ni] += live ? (double)v * (double)v : 0.0;
      }
  }
  if constexpr (PARTIAL) {
    // lanes l, l+16, l+32, l+48 hold the same column: fold them, then the
    // two waves sharing a column block, always in the same order
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      csq[ni] += __shfl_xor(csq[ni], 16, 64);
      csq[ni] += __shfl_xor(csq[ni], 32, 64);
      if (lane < 16) colpart[wave >> 1][wc + 16 * ni + lane] = csq[ni];
    }
    __syncthreads();
    if (tid < GEMM_BS) {
      const int j = j0 + tid;
      if (j < P.count) {
        const int sid = P.list[j];
        const SliceDesc& D = P.desc[sid];
        if (P.state[sid].active) {
          const double tot = (colpart[0][2 * tid] + colpart[1][2 * tid]) + (colpart[0][2 * tid + 1] + colpart[1][2 * tid + 1]);
          const int Mp = P.shape.Mp;
          if (MODE == G_AX_R0) slot_wptr(D, SLOT_DATA)[blockIdx.x] = 0.5 * tot;
          else if (P.pq_gemm) slot_wptr(D, SLOT_PQ0 + P.k)[P.npq - Mp / GEMM_BM + blockIdx.x] = tot;
        }
      }
    }
  }
}

// Scratch index of output (row, real column) of split s: [s][row][col] with
// gridDim.y * BN columns.
__device__ __forceinline__ size_t gemm_scr(int s, int row, int rows, int col) {
  return ((size_t)s * rows + row) * (size_t)(gridDim.y * BN) + col;
}

// One GEMM_BM x 64 output tile per workgroup (split s = blockIdx.z of P.gsplit
// takes K range [s K / S, (s+1) K / S)); the next BK-deep slices of both
// operands are fetched into registers while the current ones (in LDS) feed
// the MFMAs, so global latency overlaps the arithmetic.  With a split the
// raw sums go to scratch and k_gemm_reduce finishes them.
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_gemm(Params P) {
  using M = Mfma<T>;
  constexpr bool TRANS = (MODE == G_ATB || MODE == G_ATY);   // A^T v
  __shared__ T As[BK][GEMM_BM + PAD];       // As[k][row]
  __shared__ T Bs[BK][BN + PAD];            // Bs[k][col]
  __shared__ double colpart[2][BN];
  const int N = P.n * P.n;
  const int Mp = P.shape.Mp, Mv = P.shape.M;
  const int K = TRANS ? Mp : N;
  const int KS = K / P.gsplit;              // a multiple of BK (host-checked)
  const int kbeg = blockIdx.z * KS, kend = kbeg + KS;
  const int row0 = blockIdx.x * GEMM_BM;
  const int j0 = blockIdx.y * GEMM_BS;
  const T* A = static_cast<const T*>(P.shape.A);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // operand fetch roles (fixed for the whole K loop)
  //   A, not transposed: row ar, k offsets ak .. ak+AE-1 (contiguous)
  //   A, transposed:     k row ak, rows ar .. ar+AE-1 (contiguous)
  //   B: slice jl, reals BE part .. BE part + BE-1 of its 2 BK-long run
  constexpr int AE = GEMM_BM * BK / NT;            // A values per thread and stage
  const int ar = TRANS ? (tid % (GEMM_BM / AE)) * AE : tid / (BK / AE);
  const int ak = TRANS ? tid / (GEMM_BM / AE) : (tid % (BK / AE)) * AE;
  constexpr int BE = 2 * BK * GEMM_BS / NT;          // B reals per thread and stage
  const int jl = tid / (2 * BK / BE), part = tid % (2 * BK / BE);
  const T* bsrc = nullptr;
  if (j0 + jl < P.count) {
    const SliceDesc& D = P.desc[P.list[j0 + jl]];
    const void* v = MODE == G_ATB ? D.b : (MODE == G_AX_R0 ? D.x : (MODE == G_AP ? D.p : D.y));
    bsrc = static_cast<const T*>(v);
  }
  const int kmax_b = MODE == G_ATB ? Mv : K;   // b has only M rows
  T ra[AE], rb[BE];
  auto fetch = [&](int k0) {
    const T* src = TRANS ? A + (size_t)(k0 + ak) * N + row0 + ar : A + (size_t)(row0 + ar) * N + k0 + ak;
#pragma unroll
    for (int e = 0; e < AE; ++e) ra[e] = src[e];
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int k = k0 + ((part * BE + e) >> 1);
      rb[e] = (bsrc && k < kmax_b) ? bsrc[2 * (size_t)k + (e & 1)] : (T)0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      if (TRANS) As[ak][ar + e] = ra[e];
      else As[ak + e][ar] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) Bs[(part * BE + e) >> 1][2 * jl + (e & 1)] = rb[e];
  };

  const int wr = (wave >> 1) * WR, wc = (wave & 1) * WC;
  typename M::V acc[MI][NI];
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b) acc[a][b] = typename M::V{0, 0, 0, 0};

  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    stash();
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
      T a[MI], b[NI];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) a[mi] = As[k][wr + 16 * mi + (lane & 15)];
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) b[ni] = Bs[k][wc + 16 * ni + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = M::mac(a[mi], b[ni], acc[mi][ni]);
    }
    __syncthreads();
  }

  if (P.gsplit > 1) {
    T* scr = static_cast<T*>(P.gscr);
    const int rows = TRANS ? N : Mp;
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + wr + 16 * mi + M::row(lane, r);
          const int col = blockIdx.y * BN + wc + 16 * ni + (lane & 15);
          scr[gemm_scr(blockIdx.z, row, rows, col)] = acc[mi][ni][r];
        }
    return;
  }
  gemm_epilogue<T, MODE>(P, row0, j0, [&](int mi, int ni, int r) { return acc[mi][ni][r]; }, colpart);
}

// Sum of the P.gsplit partial tiles (split order fixed), then the epilogue.
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_gemm_reduce(Params P) {
  using M = Mfma<T>;
  constexpr bool TRANS = (MODE == G_ATB || MODE == G_ATY);
  __shared__ double colpart[2][BN];
  const int rows = TRANS ? P.n * P.n : P.shape.Mp;
  const int row0 = blockIdx.x * GEMM_BM, j0 = blockIdx.y * GEMM_BS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * WR, wc = (wave & 1) * WC;
  const T* scr = static_cast<const T*>(P.gscr);
  // every partial of this thread's 16 outputs is loaded before the
  // epilogue's first store (which the compiler would otherwise keep every
  // later load behind); splits are added in their fixed order
  T sum[MI][NI][4];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[mi][ni][r] = (T)0;
  for (int sp = 0; sp < P.gsplit; ++sp)
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + wr + 16 * mi + M::row(lane, r);
          const int col = blockIdx.y * BN + wc + 16 * ni + (lane & 15);
          sum[mi][ni][r] += scr[gemm_scr(sp, row, rows, col)];
        }
  gemm_epilogue<T, MODE>(P, row0, j0, [&](int mi, int ni, int r) { return sum[mi][ni][r]; }, colpart);
}

template <typename T, int MODE>
hipError_t L_gemm(const Params& P, dim3 g, hipStream_t st) {
  // with split-K the timed interval runs from the product's start to the
  // reduction's end
  const LaunchTiming& t = launch_timing();
  const bool split = P.gsplit > 1;
  launch_kernel(k_gemm<T, MODE>, dim3(g.x, g.y, P.gsplit), dim3(NT), 0, st, t.start, split ? nullptr : t.stop, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !split) return e;
  launch_kernel(k_gemm_reduce<T, MODE>, g, dim3(NT), 0, st, nullptr, t.stop, P);
  return hipGetLastError();
}

template <typename T>
GemmKernels make_gemm() {
  GemmKernels k{};
  k.g[G_ATB] = L_gemm<T, G_ATB>;
  k.g[G_AX_R0] = L_gemm<T, G_AX_R0>;
  k.g[G_AP] = L_gemm<T, G_AP>;
  k.g[G_ATY] = L_gemm<T, G_ATY>;
  return k;
}

const GemmKernels* gemm_kernels(bool fp64) {
  static const GemmKernels k32 = make_gemm<float>();
  static const GemmKernels k64 = make_gemm<double>();
  return fp64 ? &k64 : &k32;
}

}  // namespace firls

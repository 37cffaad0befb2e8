// Products with a dense sensing matrix A (random projections of Section
// 5.2), batched over the slices of one launch.
//
// The real matrix A (Mp x N, row-major, N = n^2, rows >= M zero) multiplies
// the complex vectors of up to GEMM_BS slices at a time: the real and
// imaginary parts of slice j are columns 2j and 2j+1 of the right operand,
// read in place from the slice's own vector (x, p, y or b).  Tiles of
// GEMM_BM rows x 64 columns run on MFMA (FP32: v_mfma_f32_16x16x4f32, FP64:
// v_mfma_f64_16x16x4f64), four waves of 32 x 32, with 16-deep slices of both
// operands staged in LDS.  Per-slice partial sums (data term, ||A p||^2)
// are reduced in a fixed order: one partial per row tile.
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

constexpr int BK = 16;          // depth of one LDS stage
constexpr int BN = 2 * GEMM_BS; // real columns per tile
constexpr int PAD = 4;

}  // namespace

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_gemm(Params P) {
  using C = cplx<T>;
  using M = Mfma<T>;
  constexpr bool TRANS = (MODE == G_ATB || MODE == G_ATY);   // A^T v
  __shared__ T As[BK][GEMM_BM + PAD];       // As[k][row]
  __shared__ T Bs[BK][BN + PAD];            // Bs[k][col]
  __shared__ double sq[GEMM_BM][BN + 1];    // squares for the per-slice partials
  __shared__ double colsum[BN];
  const int N = P.n * P.n;
  const int Mp = P.shape.Mp, Mv = P.shape.M;
  const int K = TRANS ? Mp : N;
  const int row0 = blockIdx.x * GEMM_BM;
  const int j0 = blockIdx.y * GEMM_BS;
  const T* A = static_cast<const T*>(P.shape.A);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // the slice whose operand column pair this thread loads (fixed for the loop)
  const int jl = tid >> 3, part = tid & 7;
  const int jg = j0 + jl;
  const T* bsrc = nullptr;
  if (jg < P.count) {
    const SliceDesc& D = P.desc[P.list[jg]];
    const void* v = MODE == G_ATB ? D.b : (MODE == G_AX_R0 ? D.x : (MODE == G_AP ? D.p : D.y));
    bsrc = static_cast<const T*>(v);
  }
  const int kmax_b = MODE == G_ATB ? Mv : K;   // b has only M rows

  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  typename M::V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename M::V{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile: GEMM_BM rows x BK, stored As[k][row]
    if (!TRANS) {
      const int r = tid >> 2, k4 = (tid & 3) * 4;
      const T* src = A + (size_t)(row0 + r) * N + k0 + k4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[k4 + e][r] = src[e];
    } else {
      const int k = tid >> 4, r4 = (tid & 15) * 4;
      const T* src = A + (size_t)(k0 + k) * N + row0 + r4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[k][r4 + e] = src[e];
    }
    // B tile: BK rows x BN columns; slice jl supplies 2 BK consecutive reals
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = part * 4 + e, kk = idx >> 1, c = idx & 1;
      const int k = k0 + kk;
      Bs[kk][2 * jl + c] = (bsrc && k < kmax_b) ? bsrc[2 * (size_t)k + c] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const T a = As[k][wr + 16 * mi + (lane & 15)];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = M::mac(a, Bs[k][wc + 16 * ni + (lane & 15)], acc[mi][ni]);
      }
    }
    __syncthreads();
  }

  // epilogue: scatter to the slices' vectors, squares into LDS
  constexpr bool PARTIAL = (MODE == G_AX_R0 || MODE == G_AP);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * mi + M::row(lane, r);
        const int col = wc + 16 * ni + (lane & 15);
        const int gr = row0 + row, j = j0 + (col >> 1), c = col & 1;
        T v = acc[mi][ni][r];
        double s2 = 0.0;
        if (j < P.count) {
          const int sid = P.list[j];
          const SliceDesc& D = P.desc[sid];
          if (P.state[sid].active) {
            if (MODE == G_ATB) {
              static_cast<T*>(D.x)[2 * (size_t)gr + c] = v;
            } else if (MODE == G_ATY) {
              static_cast<T*>(D.t)[2 * (size_t)gr + c] = v;
            } else {
              if (MODE == G_AX_R0) v = gr < Mv ? static_cast<const T*>(D.b)[2 * (size_t)gr + c] - v : (T)0;
              static_cast<T*>(D.y)[2 * (size_t)gr + c] = v;
              s2 = (double)v * (double)v;
            }
          }
        }
        if (PARTIAL) sq[row][col] = s2;
      }
  if constexpr (PARTIAL) {
    __syncthreads();
    if (tid < BN) {
      double t = 0.0;
      for (int r = 0; r < GEMM_BM; ++r) t += sq[r][tid];
      colsum[tid] = t;
    }
    __syncthreads();
    if (tid < GEMM_BS) {
      const int j = j0 + tid;
      if (j < P.count) {
        const int sid = P.list[j];
        const SliceDesc& D = P.desc[sid];
        if (P.state[sid].active) {
          const double tot = colsum[2 * tid] + colsum[2 * tid + 1];
          if (MODE == G_AX_R0) slot_wptr(D, SLOT_DATA)[blockIdx.x] = 0.5 * tot;
          else if (P.pq_gemm) slot_wptr(D, SLOT_PQ0 + P.k)[P.npq - Mp / GEMM_BM + blockIdx.x] = tot;
        }
      }
    }
  }
}

template <typename T, int MODE>
hipError_t L_gemm(const Params& P, dim3 g, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm<T, MODE>), g, dim3(NT), 0, st, P);
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

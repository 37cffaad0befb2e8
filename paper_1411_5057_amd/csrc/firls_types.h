// Shared host/device structures of the FIRLS library (internal).
#pragma once
#include <stdint.h>

namespace firls {

constexpr int NT = 256;          // threads per workgroup (4 wave64)
constexpr int KMAX = 64;         // largest PCG iteration count per outer iteration
constexpr int PMAX = 512;        // partial sums per slot per slice
constexpr int GROUPS_PER_WG = 1024;
constexpr int TV_TR = 16;        // TV preconditioner tile rows
constexpr int TV_TC = 32;        // TV preconditioner tile columns

// Rows per workgroup of the row passes for an n x n image: a multiple of 16
// (one Haar tile row of side 16) chosen so a band holds about 4096 pixels.
__host__ __device__ constexpr int band_rows(int n) {
  return n >= 192 ? 16 : ((n == 128 || n == 96) ? 32 : n);
}
// Columns per workgroup of the column pass.
// Enough columns that the first FFT stage's butterflies fill the workgroup
// at small sides (the whole image up to 64), 16 from 192 up (8 in FP64 above
// 256), with a strip of at most about 70 KB of LDS.
__host__ __device__ constexpr int strip_cols(bool fp64, int n) {
  return n <= 64 ? n : (n <= 128 ? 32 : (fp64 && n > 256 ? 8 : 16));
}

// Slots of the per-slice FP64 partial-sum area.  Every slot holds up to
// PMAX partials, each written by exactly one workgroup, and every consumer
// sums them in index order, so all reductions are deterministic.
enum Slot : int {
  SLOT_DATA = 0,      // 1/2 ||m F x - b||^2 partials (column pass)
  SLOT_REG_EPS = 1,   // sum sqrt(s_g + eps)        (group pass)
  SLOT_REG0 = 2,      // sum sqrt(s_g)              (group pass)
  SLOT_PQ0 = 3,       // <p_k, S p_k>, k = 0..KMAX-1 (Haar: row-pass partials,
                      // then ||A p_k||^2 partials of the column pass)
  SLOT_RZ0 = 3 + KMAX,  // <r_k, z_k>, k = 0..KMAX
  SLOT_QQ0 = 4 + 2 * KMAX,  // <q_k, P^{-1} q_k>, k = 0..KMAX-1 (Haar)
  SLOT_SYNC = 4 + 3 * KMAX,  // uint32 barrier counters k = 0..KMAX-1 of the paired PCG pass
  SLOT_COUNT = 5 + 3 * KMAX
};

enum Psi : int { PSI_HAAR = 0, PSI_TV = 1 };

// Per-slice status codes written on the device (the ABI's FIRLS_* values).
enum SliceStatus : int { ST_OK = 0, ST_W_MAXITER = 1, ST_W_NONMONOTONE = 2, ST_E_INVALID = -1, ST_E_NONFINITE = -5,
                         ST_E_SYNC = -6, ST_E_BREAKDOWN = -7 };
// Test hooks (Params::test_flags), set only through firls_test_hooks.
enum TestFlag : int { TEST_SYNC_TIMEOUT = 1, TEST_BREAKDOWN = 2, TEST_NONMONOTONE = 4 };
enum Precond : int { PC_PAPER = 0, PC_JACOBI = 1, PC_NONE = 2 };

// Kernel variants (template modes).
enum RowFwdMode : int { RF_PLAIN = 0, RF_PCG_HAAR = 1, RF_PCG_Z = 2, RF_STEP_HAAR = 3, RF_SQ_HAAR = 4,
                        RF_SQW_HAAR = 5, RF_PEN_HAAR = 6 };
enum ColMode : int { COL_SP = 0, COL_R0 = 1, COL_AHB = 2, COL_DC = 3, COL_SP_PQ = 4 };
// RI_R0_HAAR_P0: the Haar residual pass that also forms z0 = P^{-1} r0 with
// the paper's preconditioner, p0 and its row FFT (its own instantiation,
// so it carries no registers for the other preconditioners).
enum RowInvMode : int { RI_PLAIN = 0, RI_SP_HAAR = 1, RI_SP_TV = 2, RI_R0_HAAR = 3, RI_R0_TV = 4, RI_R0_HAAR_P0 = 5 };
enum UpdMode : int { UP_INIT = 0, UP_STEP = 1 };
// Dense sensing matrix products (batched over the slices of a launch):
//   G_ATB   x = A^T b            (zero-filled start)
//   G_AX_R0 y = b - A x          (+ partials of 1/2 ||A x - b||^2)
//   G_AP    y = A p              (+ partials of ||A p||^2 = <p, A^T A p>)
//   G_ATY   t = A^T y
enum GemmMode : int { G_ATB = 0, G_AX_R0 = 1, G_AP = 2, G_ATY = 3 };
constexpr int GEMM_BM = 128;     // rows per workgroup tile
constexpr int GEMM_BS = 32;      // slices (64 real columns) per workgroup tile
constexpr int GEMM_BK = 32;      // depth of one LDS stage of the GEMM

// Per-slice device pointers.  Caller-owned: b, mask, x.  The rest is
// library workspace.  Complex vectors are n x n interleaved (re, im) of the
// working precision; d / sq are real arrays of the transform's size (n^2
// for Haar in the tile-major coefficient layout, 2 n^2 for TV); W is per
// group.
struct SliceDesc {
  const void* b;
  const uint8_t* mask;
  void* x;
  void* r[2];
  void* p;
  void* q;
  void* t;
  void* z;
  void* d;
  void* sq;
  void* W;
  uint16_t* mbits;   // mask bits: word [c16][row] = mask[row][16 c16 .. 16 c16 + 15]
  void* y;           // dense sensing matrix only: A v (Mp complex)
  double* parts;
  double rho_fixed;  // > 0: rho of a dense sensing matrix (mean diag A^T A); else from the mask
  double lambda;
  int32_t n;
  int32_t shape;
  int32_t C;         // contrasts stacked as C blocks of n rows
  int32_t need_dc;   // a solve of a TV slice: every contrast's mask must sample DC
};

// Per-slice device state of the outer loop (FP64 scalars on the device).
struct SliceState {
  double rho;        // mean diag(A^H A) = sampled fraction
  double Fe;         // F_eps at the last evaluation
  double F;          // F (eps = 0) at the last evaluation
  double data;       // 1/2 ||A x - b||^2 at the last evaluation
  double Fe_prev;    // F_eps at the evaluation before
  double rel;        // (Fe_prev - Fe) / Fe
  int32_t active;    // 1 while the slice still iterates
  int32_t outer;     // reweighted solves done
  int32_t pcg;       // PCG iterations done
  int32_t status;    // SliceStatus
  int32_t converged;
  int32_t evals;     // objective evaluations done
  int32_t pend;      // x += alpha p of the last PCG iteration not yet applied
                     // (folded into the next residual row pass)
  int32_t pcg_stop;  // PCG iterations the current solve took when its early
                     // exit fired (0: none yet); the outer check books it
};

// One slot refill of a streamed batch (a sub-batch whose slots take the
// next queued slice as soon as theirs stops): the stopped slice ``old``
// (>= 0) has its final state saved at state[final_base + old], and the slot
// takes the inputs of the new slice.
struct RefillRec {
  const void* b;
  const uint8_t* mask;
  void* x;
  double lambda;
  int32_t slot;
  int32_t old;
};
struct RefillArgs {
  const RefillRec* rec;   // host-mapped, ``count`` records
  int32_t count;
  int32_t final_base;
  SliceDesc* desc;
  SliceState* state;
  int32_t* list;          // out: the refilled slots, in record order
  int32_t* stop_flags;    // host-mapped stop word per slot (a slice rejected at its start writes 0)
};

// Group map of one shape on the device (internal coefficient indices).
constexpr int ELL_MAX = 8;        // widest padded group / membership list

struct ShapeDev {
  const int32_t* gptr;   // [n_groups + 1]
  const int32_t* gidx;   // members
  const int32_t* tptr;   // [n_coef + 1] coefficient -> groups (transpose)
  const int32_t* tidx;
  const int32_t* perm;   // user coefficient index -> internal index
  int32_t n_groups;
  int32_t n_coef;
  const int32_t* bgptr;  // band-local group maps: groups of row band b are bgptr[b] .. bgptr[b+1]-1
  // band-local maps with small groups, padded (ELLPACK) lists:
  // gell[g * gw + m] = m-th member of group g, tell[j * tw + m] = m-th group
  // holding coefficient j, both relative to the row band (member offset in
  // the band, group offset from bgptr[b]); 0xFFFF pads
  const uint16_t* gell;
  const uint16_t* tell;
  int32_t gw, tw;        // list widths: 1, 2, 4 or 8 (ELL_MAX)
  const void* A;         // dense sensing matrix, Mp x n^2 row-major (rows >= M zero), or null
  int32_t M;             // measurements of the dense matrix
  int32_t Mp;            // M rounded up to the GEMM row tile
};

// Launches across shapes: one workgroup per item; the item names the slice,
// the block within it and the parameters (an entry of a device table of
// Params, one per shape and launch position) its shape's kernel runs with.
struct MultiItem {
  int32_t s;   // slice
  int32_t x;   // block within the slice
  int32_t p;   // Params entry
};
struct MultiArgs;   // below Params

// Kernel classes of launches across shapes (the mode is the kernel's
// template mode where it has one).
enum MultiClass : int { MC_ROWFWD = 0, MC_COL, MC_ROWINV, MC_PAIR, MC_PSI_SQ_HAAR, MC_UPDATE_HAAR, MC_LAST_X,
                        MC_PSI_SQ_TV, MC_GROUP_W, MC_GROUP_D, MC_UPDATE_TV, MC_OUTER_CHECK, MC_COUNT };
constexpr int MC_MODES = 7;

#define FIRLS_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

// Kernel parameters (passed by value).
struct Params {
  const SliceDesc* desc;
  SliceState* state;
  const int32_t* list;   // slice ids; blockIdx.y indexes it
  const void* tw;        // twiddles exp(-2 pi i k / n), k < n
  ShapeDev shape;
  int32_t n;
  int32_t L;             // Haar levels
  int32_t k;             // PCG iteration index
  int32_t fold_x;        // the last PCG step's x += alpha p rides in the next residual row pass
  int32_t q_dead;        // PCG row inverse: nothing reads this q or <q, P^-1 q> (last iteration of the fused step)
  int32_t test_flags;    // test hooks (TEST_*): conditions forced from the host so the error paths run
  int32_t p0_prep;       // the residual's row-inverse pass also forms z0, p0 = z0 and its row FFTs (host: picks RI_R0_HAAR_P0)
  int32_t check_r0;      // ... and its first workgroup runs the outer check (Haar)
  int32_t K;             // PCG iterations per outer iteration
  int32_t Tmax;
  int32_t precond;
  int32_t nrz;           // partial counts of the <r,z>, <p,q>, data and penalty slots
  int32_t npq;
  int32_t ndata;
  int32_t nreg;
  int32_t no_data;       // objective check: take the data term as 0
  int32_t tvb;           // TV boundary: 0 periodic, 1 the paper's non-periodic D
  int32_t C;             // contrasts: the image is C blocks of n rows (one per contrast)
  int32_t nofft;         // dense sensing matrix: row passes skip / replace the FFT
  int32_t count;         // slices in ``list`` (GEMM column tiles)
  int32_t pq_gemm;       // the A p product adds ||A p||^2 partials to <p, S p> (Haar)
  int32_t gsplit;        // GEMM split-K factor (1: no split)
  void* gscr;            // GEMM split-K partial tiles
  double eps;
  double tau;
  double mono_slack;     // outer check: F_eps may exceed its previous value by this fraction (rounding)
  double eta2;           // PCG early exit: stop once <r_j, z_j> <= eta2 <r_0, z_0> (0: run all K)
  void* out;             // op entry points: extra output
  int32_t* stop_flags;   // host-mapped word per slice, (evaluations << 1) | active,
                         // written by the outer check (null: not written)
};

struct MultiArgs {
  const Params* __restrict__ table;
  const MultiItem* __restrict__ items;
};

}  // namespace firls

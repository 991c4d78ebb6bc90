// Internal declarations of librecip: the factor handle, device helpers and the
// host-side launchers each translation unit exports to the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "recip.h"

namespace rcp {

// Storage tile edge and Gauss-Jordan panel width.  A Schur-complement block of
// size ny is padded to np = ceil(ny / TB) * TB (identity in the padding) and
// stored as its lower-triangular TB x TB tiles, packed row by row:
// tile (I, J), I >= J, sits at index I (I + 1) / 2 + J, row-major inside.
constexpr int TB = 32;
constexpr int NVEC = 8;          // complex128 work vectors of nx*ny in the buffer
constexpr int MAX_BATCH = 8;     // geometries factored side by side (two chains each)

// Work-vector roles.
enum { V_Z = 0, V_Y = 1, V_RHS = 2, V_LAM = 3, V_ARHS = 4, V_RES = 5, V_DU = 6, V_TMP = 7 };

struct Layout {
  size_t off_X, off_eps, off_sxc, off_sxf, off_syc, off_syf;
  size_t off_dco, off_eco, off_cco;
  size_t off_L, off_Q, off_P;     // GJ panel workspace, 4 slots for each of 2 chains
  size_t off_health, off_vec, off_red, off_fft;
  size_t off_part;                // per-tile partial sums of the vector sweep, 2 chains
  size_t off_status;              // pivot check of the last factorisation (int32)
  size_t total;
};

}  // namespace rcp

struct rcp_factors {
  int nx, ny, npml;
  double h, k0, pml_R;
  int pml_m;
  int precision;
  int np, nt;                 // padded block size, tiles per edge
  size_t tiles;               // packed tiles per block = nt (nt + 1) / 2
  size_t block_elems;         // complex elements per block = tiles * TB * TB
  size_t elem_bytes;          // 16 (complex128) or 8 (complex64)
  int m;                      // middle block of the twisted elimination
  size_t fft_cap;             // complex128 capacity of each FFT buffer
  char* base;
  rcp::Layout lay;
  void* X;
  double* eps;
  double2 *sxc, *sxf, *syc, *syf;
  double2 *dco, *eco, *cco;
  void* wsL[8];                // panel buffers: chain c, panel p at slot 4c + (p mod 4)
  void* wsQ[8];
  double2* wsP[8];
  double* health;
  int32_t* status;            // 0: every pivot passed; else 1 + first failing panel (device)
  double2* vec[rcp::NVEC];
  double* red;
  double2* fft[4];            // symbol spectrum, work, temp, W v
  double2* part[2];           // vector-sweep partial sums of chain c: tiles x (row, column) x TB
  // statistics of the last refined solve
  int last_iters;
  double last_residual;
  // 3D vector operator (maxwell3d.hip): blocks are x-slices of n = 3 gy gz
  // edge unknowns (component c, then j, k); ny holds n.  The couplings between
  // slices are sparse, not diagonal: per slice row the entries of the
  // diagonal block (column in the slice) and of the couplings to the next
  // slice (by row of slice i) and from the previous one (by column of slice
  // i+1), each a fixed number of (index, value) slots, index -1 when unused.
  int dim3 = 0;
  int gy = 0, gz = 0;
  int32_t* d_idx = nullptr;
  double2* d_val = nullptr;
  int32_t* cr_idx = nullptr;   // A_{i,i+1}(a, .) for row a of slice i
  double2* cr_val = nullptr;
  int32_t* cl_idx = nullptr;   // A_{i,i+1}(., b) for column b of slice i+1
  double2* cl_val = nullptr;
};

namespace rcp {

// ---------------------------------------------------------------------------
// error plumbing
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_check(hipError_t e, const char* what);

#define RCP_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return rcp::hip_check(_e, #call); \
  } while (0)

Layout compute_layout(int nx, int ny, int precision);
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

inline void* block_ptr(const rcp_factors* f, int i) {
  return static_cast<char*>(f->X) + size_t(i) * f->block_elems * f->elem_bytes;
}

// ---------------------------------------------------------------------------
// Optional launch timing for benchmarks: when enabled, every sample_every-th
// launch of a kernel class is bracketed by two HIP events on its stream, and
// the algorithmic work of that launch (flops or bytes) is recorded with it.
enum KClass {
  K_GJ_PANEL = 0,
  K_GJ_UPDATE = 1,
  K_SCHUR = 2,
  K_GEMV = 3,
  K_GEMM = 4,
  K_GJ_LAST = 5,
  K_ZGEMM = 6,
  K_ENGINE = 7,   // launches of the factorisation engine (mixed geometries)
  K_NCLASS = 8
};
void ktimer_begin(int cls, hipStream_t s, double work, void** token);
void ktimer_end(void* token, hipStream_t s);
struct KTimer {
  void* tok = nullptr;
  hipStream_t s;
  KTimer(int cls, hipStream_t st, double work) : s(st) { ktimer_begin(cls, st, work, &tok); }
  ~KTimer() {
    if (tok) ktimer_end(tok, s);
  }
};
// A launch of one kernel that is timed when sampled: the two events are handed
// to the launch itself (hipExtLaunchKernel), so they take the kernel's own
// start and end and not the dispatch around it.  Launches of several kernels
// timed as one sample keep the events bracketing them (KTimer).
struct KSample {
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
KSample ktimer_sample(int cls, double work);
template <typename... P, typename... A>
hipError_t klaunch(int cls, double work, void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t s,
                   A... args) {
  const KSample t = ktimer_sample(cls, work);
  if (t.e0) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.e0, t.e1, 0, static_cast<P>(args)...);
  } else {
    kernel<<<grid, block, 0, s>>>(static_cast<P>(args)...);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers (assembly.hip)
int launch_eps_from_widths(const rcp_grid* g, const rcp_pillars* p, double* eps, hipStream_t s);
int launch_assemble(rcp_factors* f, const double* eps_src, hipStream_t s);
int launch_width_grad(const rcp_grid* g, const rcp_pillars* p, const double* grad_eps,
                      double* grad_w, hipStream_t s);

// Field fld of job q (uniform) of a kernel-argument job table, selected one
// field at a time so that the table stays in kernel-argument registers.
#define RCP_SEL4(js, q, o, fld)                                                    \
  ((q) < (o) + 2 ? ((q) == (o) ? js.j[(o)].fld : js.j[(o) + 1].fld)                \
                 : ((q) == (o) + 2 ? js.j[(o) + 2].fld : js.j[(o) + 3].fld))
#define RCP_SEL16(js, q, fld)                                                      \
  ((q) < 8 ? ((q) < 4 ? RCP_SEL4(js, q, 0, fld) : RCP_SEL4(js, q, 4, fld))         \
           : ((q) < 12 ? RCP_SEL4(js, q, 8, fld) : RCP_SEL4(js, q, 12, fld)))

// factor.hip
// Factor B (1..MAX_BATCH) geometries of identical shape in the same launches.
int factor_blocks(rcp_factors* const* fs, int B, hipStream_t s);
// The same without waiting: the factorisation and the pivot check on the
// device (each set's status word), enqueued on s.
int factor_blocks_async(rcp_factors* const* fs, int B, hipStream_t s);
// Enqueues the pivot check of B finished factor sets into their status words.
int enqueue_pivot_check(rcp_factors* const* fs, int B, hipStream_t s);
// Waits for s and turns set f's status word into RCP_OK or RCP_ESINGULAR
// (the message names the panel, its block and its pivot modulus); prefix
// starts the message.
int read_pivot_check(const rcp_factors* f, hipStream_t s, const std::string& prefix);
// The factorisation engine (geometries of any size in shared launches, admitted
// between rounds); see include/recip.h.
int engine_create(int precision, rcp_engine** out);
void engine_destroy(rcp_engine* e);
int engine_active(const rcp_engine* e);
int engine_precision(const rcp_engine* e);
int engine_add(rcp_engine* e, rcp_factors* f);
int engine_step(rcp_engine* e, int rounds, hipStream_t s, rcp_factors** done, int* status,
                int cap, int* ndone);

// solve.hip
// Workspace of the many-right-hand-side sweep's k-split tiles (optional): up
// to GEMM_SPLIT_TILES partial 64 x 64 complex128 tiles.
constexpr int GEMM_SPLIT_TILES = 1024;
constexpr size_t GEMM_SPLIT_BYTES = size_t(GEMM_SPLIT_TILES) * 64 * 64 * 16;
// u = A^{-1} f (conjop = 0) or conj(A)^{-1} f = A^{-dag} f (conjop = 1), one
// right-hand side, f and u complex128 nx*ny, f != u.  Blocks outside
// [nz_lo, nz_hi] of f are known to be zero.
// out[q] = base[q] + X_{blocks[q]} g[q] (block size f->ny; base may be null),
// for one or two blocks in one launch, by the single-RHS sweep's kernels
// (part_area[q]: which of the two partial-sum areas a job uses).  FP64.
int block_products(rcp_factors* f, int count, const int* blocks, const double2* const* g,
                   const double2* const* base, double2* const* out, const int* part_area,
                   int conjop, hipStream_t s);
int solve_vec(rcp_factors* f, const double2* rhs, double2* u, int conjop, int nz_lo, int nz_hi,
              hipStream_t s);
// The same for B (1..MAX_BATCH) factor sets of identical shape and precision,
// their sweeps advancing in the same launches: u[g] = A_g^{-1} rhs[g].
int solve_vec_batch(rcp_factors* const* fs, int B, const double2* const* rhs, double2* const* u,
                    int conjop, const int* nz_lo, const int* nz_hi, hipStream_t s);
// Refined (FP32 factors) or plain (FP64) single-RHS solve with statistics.
int solve_vec_refined(rcp_factors* f, const double2* rhs, double2* u, int conjop, int nz_lo,
                      int nz_hi, double tol, int max_refine, hipStream_t s, rcp_solve_stats* st);
// nrhs right-hand sides in (R, nx, ny) layout, FP64 factors.  If fline != null
// the right-hand sides are line sources: fline[r * nx + i] on row jline.
int solve_multi_fp64(rcp_factors* f, int nrhs, const double2* B, const double2* fline, int jline,
                     double2* X, int conjop, hipStream_t s,
                     double2* split_ws = nullptr);
int residual_norms(rcp_factors* f, const double2* b, const double2* x, double2* r, int conjop,
                   hipStream_t s, double* rnorm, double* bnorm);

// maxwell3d.hip -- Schur complements of 3D blocks for the engine (chains
// whose geometry is 3D form them here before their pivot work).  Slots per
// slice row: in-slice entries, and entries of a coupling to a neighbour slice.
constexpr int K3D_DW = 12;
constexpr int K3D_CW = 4;
struct Schur3dJob {
  void* dst;
  const void* src1;     // X of the previous block (left chain or middle), or null
  const void* src2;     // X of the next block (right chain or middle), or null
  const int32_t* d_idx;  // rows of this block's diagonal block
  const double2* d_val;
  const int32_t* c1_idx; // couplings to src1's slice, by row of this slice
  const double2* c1_val;
  const int32_t* c2_idx; // couplings to src2's slice
  const double2* c2_val;
  int n, tiles;
};
int schur3d(const Schur3dJob* jobs, int count, hipStream_t s);

// form.hip
int objective_rhs(rcp_factors* f, const rcp_objective* o, double2* w, int* nz_lo, int* nz_hi,
                  hipStream_t s);
int toeplitz_form(rcp_factors* f, const rcp_light* L, const double2* z, double* F_dev,
                  double2* v_out, double2* Tv_out, hipStream_t s);
int grad_eps(rcp_factors* f, const double2* lam, const double2* z, double* grad, hipStream_t s);
int scatter_line(rcp_factors* f, const rcp_light* L, const double2* Tv, double2* rhs,
                 hipStream_t s);
int bf_per_angle_at(rcp_factors* f, const rcp_objective* o, const double2* U, int R,
                    double* per_angle, int r0, hipStream_t s);
int gl_nodes(const rcp_light* L, int n, double* theta, double* wts, hipStream_t s);
int planewave_lines(rcp_factors* f, const rcp_light* L, const double* theta, int R,
                    double2* fline, hipStream_t s);
int bf_sum(const double* weights, const double* per_angle, int n, double* F_dev, hipStream_t s);
int fill_zero(void* p, size_t bytes, hipStream_t s);
// out[q] = sum_g w[g] x_g[q] over n values, and F[count] = sum_g w[g] F[g]
// (fixed order; count <= MAX_BATCH)
int weighted_sum(int count, const double* w, double* const* x, size_t n, double* F, double* out,
                 hipStream_t s);

// dense.hip -- complex FP64 products out[n][m] = sum_l A[m][l] opB(B[n][l]) on
// MFMA, split over l into S parts of Ls values (partial products at
// out + z * split_stride), and what the dense form and the ensemble
// correlation build from them.
struct ZSplit {
  int S, Ls;
};
ZSplit zgemm_split(int Md, int Nd, int L);
// Nd_used (> 0): rows of B that carry data (the timer's flop count); the rest
// are zero padding.
int zgemm_nt(const double2* A, int lda, const double2* B, int ldb, bool conjb, double2* out,
             int ldo, size_t split_stride, int Md, int Nd, int L, ZSplit sp, hipStream_t s,
             int Nd_used = 0);
// Work of the dense-form calls for K outputs on an M-cell line: objective
// right-hand sides (K fields, also the adjoint fields), reciprocal fields (K),
// the line values V^T and W V (Kp = K rounded up to 16 rows), the split
// partial products, per-block sums and the adjoint line sources.
struct DenseLayout {
  int Kp, nmb;
  ZSplit sp;
  size_t off_B, off_Z, off_Vt, off_Y, off_part, off_red, off_fline, total;
};
DenseLayout dense_layout(int nx, int ny, int K, int M);
int gather_lines(const double2* Z, size_t N, int ny, int js, int i0, int M, int K, int Kp,
                 double2* Vt, hipStream_t s);
// Y = W V (Kp x M, row k = output k), F[k] = Re v_k^dag y_k, F[K] = sum_k F[k]
int dense_form(const double2* W, int M, const double2* Vt, int K, const DenseLayout& D,
               double2* part, double2* Y, double* red, double* F, hipStream_t s);
int scatter_lines(const double2* Y, int M, int K, int nx, int i0, double2* fline, hipStream_t s);
int grad_eps_many(rcp_factors* f, int K, const double2* lam, const double2* z, double* grad,
                  hipStream_t s);
struct CorrLayout {
  size_t off_G, off_S, off_part, total;
};
CorrLayout corr_layout(int M, int N);
int correlation_matrix(int M, int N, int i0, int npml, double h, double n_s, double k0,
                       const double* theta, const double2* Cq, double2* W, char* work,
                       hipStream_t s);

}  // namespace rcp

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
__device__ __forceinline__ double2 cinv(double2 a) {
  double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

template <typename T> struct cplx;
template <> struct cplx<double> { using t = double2; };
template <> struct cplx<float> { using t = float2; };

// Loads and stores of data that streams through a kernel once (the factor
// tiles of a pass or of a block product), with the nontemporal hint, so that
// they do not push data the kernel reads again (panel rows, vectors) out of L2.
__device__ __forceinline__ double2 load_stream(const double2* p) {
  using v2 = double __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 load_stream(const float2* p) {
  using v2 = float __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void store_stream(double2* p, double2 a) {
  using v2 = double __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2{a.x, a.y}, reinterpret_cast<v2*>(p));
}
__device__ __forceinline__ void store_stream(float2* p, float2 a) {
  using v2 = float __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2{a.x, a.y}, reinterpret_cast<v2*>(p));
}

__device__ __forceinline__ double2 to_c128(double2 a) { return a; }
__device__ __forceinline__ double2 to_c128(float2 a) { return make_double2(a.x, a.y); }
template <typename T2> __device__ __forceinline__ T2 from_c128(double2 a);
template <> __device__ __forceinline__ double2 from_c128<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_c128<float2>(double2 a) {
  return make_float2(static_cast<float>(a.x), static_cast<float>(a.y));
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
template <typename T> struct v4of;
template <> struct v4of<double> { using t = v4d; };
template <> struct v4of<float> { using t = v4f; };

// One 16x16x4 matrix-core product D = A B + C per wave.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; D column l % 16 lands in lane l, and
// register r of that lane holds D row mfma_row<T>(l / 16, r): 4 (l / 16) + r
// for the f32 instruction, l / 16 + 4 r for the f64 one (both checked on gfx950).
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int mfma_row(int lk, int r);
template <> __device__ __forceinline__ int mfma_row<double>(int lk, int r) { return lk + 4 * r; }
template <> __device__ __forceinline__ int mfma_row<float>(int lk, int r) { return 4 * lk + r; }

// packed lower-tile index helpers
__host__ __device__ __forceinline__ size_t tile_index(int I, int J) {
  return size_t(I) * (I + 1) / 2 + J;
}
__device__ __forceinline__ void tile_coords(int t, int* I, int* J) {
  int i = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *I = i;
  *J = t - i * (i + 1) / 2;
}

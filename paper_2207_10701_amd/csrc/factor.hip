// Block factorisation of the FDFD operator A (Sec. "Reciprocal approach":
// the single solve u = A^{-1} b the method needs, here by a direct method).
//
// A is block tridiagonal along x with diagonal blocks D_i (tridiagonal, size
// ny) and diagonal couplings C_i between columns i and i+1.  Two-ended
// (twisted) elimination, middle block m = nx / 2:
//   left  chain  S_0 = D_0,        S_i = D_i - C_{i-1} X_{i-1} C_{i-1},  X_i = S_i^{-1}, i < m
//   right chain  T_{nx-1} = D_{nx-1}, T_i = D_i - C_i X_{i+1} C_i,     X_i = T_i^{-1}, i > m
//   middle       Z = D_m - C_{m-1} X_{m-1} C_{m-1} - C_m X_{m+1} C_m,  X_m = Z^{-1}
// Both chains advance in the same launches.  Every block is complex symmetric
// (A = A^T), so each inverse is computed by the symmetric blocked Gauss-Jordan
// sweep on its lower TB x TB tiles only.  Sweeping panel K of a symmetric S:
//   P = S_KK^{-1},  L = S(:, K),  Q = L P,
//   S_IJ <- S_IJ - Q_I L_J^T (I, J != K),  S_IK <- Q_I,  S_KK <- -P,
// and after all panels the tiles hold -S^{-1}; the last panel negates.
//
// One geometry, one panel per launch with look-ahead: launch k applies update
// k to every tile outside tile column k+1, while a few workgroups compute the
// update-k values of column k+1 directly in the layout the next panel needs,
// invert the next pivot block and form Q for panel k+1 into the other half of
// double-buffered panel buffers.  Column k+1 values never go back to the
// factor tiles: update k+1 overwrites that column anyway.  No dependencies
// between the workgroups of a launch.
//
// Batches (2 to 8 geometries side by side): two panels per pass, each tile
// read and written once per pair; one workgroup per chain does the next
// pair's pivot work inside the pass and a short launch forms the next pair's
// row tiles (the two-panel section below).  The pivot work that opens a block
// rides in the launch that forms the block's Schur complement.
//
// The TB x TB pivot blocks are inverted without pivoting, in FP64 for both
// storage precisions, and the smallest pivot modulus of every panel is
// recorded for the health check.
#include <cmath>
#include <vector>

#include "rcp_internal.h"

namespace {
using namespace rcp;

// Placement of a launch's jobs on the 8 XCDs.  Workgroups are dealt to the
// XCDs round robin (workgroup b runs on XCD b mod 8); each XCD's share is split
// into two interleaved half-slots h = 2 x + (s mod 2), s = b / 8.  Half-slot h
// serves job q[h]: its workgroups w = off[h], off[h] + stride[h], ... (a job on
// u half-slots has offsets 0 .. u-1 and stride u; q[h] = -1: unused).  Keeping
// a chain's workgroups on few XCDs keeps the panel buffers they all read in
// those XCDs' L2; a job's share of half-slots follows its share of the work.
constexpr int NHALF = 16;
struct XMap {
  int q[NHALF];
  int off[NHALF];
  int stride[NHALF];
};
#define RCP_SELA4(a, h, o) \
  ((h) < (o) + 2 ? ((h) == (o) ? a[(o)] : a[(o) + 1]) : ((h) == (o) + 2 ? a[(o) + 2] : a[(o) + 3]))
#define RCP_SELA16(a, h)                                                            \
  ((h) < 8 ? ((h) < 4 ? RCP_SELA4(a, h, 0) : RCP_SELA4(a, h, 4))                    \
           : ((h) < 12 ? RCP_SELA4(a, h, 8) : RCP_SELA4(a, h, 12)))

__device__ __forceinline__ bool xjob(const XMap& m, int* q, int* w) {
  const int b = blockIdx.x;
  const int x = b & 7, s = b >> 3;
  const int h = 2 * x + (s & 1);
  *q = RCP_SELA16(m.q, h);
  *w = RCP_SELA16(m.off, h) + (s >> 1) * RCP_SELA16(m.stride, h);
  return *q >= 0;
}

struct GJJob {
  int k;         // panel index
  int last;      // update: final panel, negate the result
  int wgs;       // workgroups of this job (update part + look-ahead part)
  int wgs_upd;   // of which the trailing-update part
  void* X;       // packed tiles of the block
  void* L;       // panel k: TB-row tiles of L = S(:, k)
  void* Q;       // panel k: Q = L P
  double2* P;    // panel k: TB x TB pivot-block inverse
  void* Ln;      // panel k+1 buffers (look-ahead output)
  void* Qn;
  double2* Pn;
  double* health;   // min |pivot| slot of the panel this job inverts
  int tiles;        // packed tiles of the block (per job: chains may differ in size)
};
constexpr int MAXJ = 2 * MAX_BATCH;   // chains per launch: two per geometry
struct GJJobs {
  GJJob j[MAXJ];
  int n;
  XMap x;
};

// Job q of a launch; fields are selected one at a time so that the table stays
// in kernel-argument registers.
__device__ __forceinline__ GJJob pick(const GJJobs& js, int q) {
#define RCP_SEL(fld) RCP_SEL16(js, q, fld)
  GJJob jb;
  jb.k = RCP_SEL(k);
  jb.last = RCP_SEL(last);
  jb.wgs = RCP_SEL(wgs);
  jb.wgs_upd = RCP_SEL(wgs_upd);
  jb.X = RCP_SEL(X);
  jb.L = RCP_SEL(L);
  jb.Q = RCP_SEL(Q);
  jb.P = RCP_SEL(P);
  jb.Ln = RCP_SEL(Ln);
  jb.Qn = RCP_SEL(Qn);
  jb.Pn = RCP_SEL(Pn);
  jb.health = RCP_SEL(health);
  jb.tiles = RCP_SEL(tiles);
#undef RCP_SEL
  return jb;
}

// 1 / d for d > 0: hardware reciprocal estimate refined by two steps of
// Newton's method r <- r (2 - d r).
__device__ __forceinline__ double recip_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// k index carried by MFMA operand slot (k-step s, lane group lk) when the left
// operand comes straight from an accumulator of the transposed block (see
// lookahead_work): 4 s + lk for the f64 layout, 16 (s / 4) + 4 lk + s % 4 for f32.
template <typename T> __device__ __forceinline__ int acc_k(int s, int lk);
template <> __device__ __forceinline__ int acc_k<double>(int s, int lk) { return 4 * s + lk; }
template <> __device__ __forceinline__ int acc_k<float>(int s, int lk) {
  return 16 * (s >> 2) + 4 * lk + (s & 3);
}

__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }

// Gauss-Jordan inversion of the TB x TB block in A (FP64), result back in A,
// eliminating two columns per step with the 2 x 2 diagonal block B of rows and
// columns p, p+1 as pivot (inverted in closed form; no row exchanges):
//   pivot rows      R <- B^{-1} R,       their pivot columns <- B^{-1}
//   other rows r    m_r <- m_r - F_r B^{-1} R,   their pivot columns <- -F_r B^{-1}
// with F_r = (m_rp, m_r,p+1).  256 threads; thread owns row r, columns
// c0..c0+3, kept in registers.  The block lives in A and W in turn: a step
// reads everything it needs from one (the pivot block, its row's pivot
// columns, its columns of the pivot rows, all at once), writes its four
// values to the other, then one barrier; sixteen steps end in A (a loop, not
// unrolled: the steps would hold registers the update path of the same
// kernels needs).  Returns min |det B|^(1/2).
__device__ __forceinline__ void pivot_step(int P, double2 (&m)[4], const double2 (*S)[TB + 1],
                                           double2 (*D)[TB + 1], int r, int c0, double& mindet2) {
  const double2 a = S[P][P], bb = S[P][P + 1], cc = S[P + 1][P], d = S[P + 1][P + 1];
  const double2 f0 = S[r][P], f1 = S[r][P + 1];
  double2 q0[4], q1[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    q0[c] = S[P][c0 + c];
    q1[c] = S[P + 1][c0 + c];
  }
  const double2 det = csub(cmul(a, d), cmul(bb, cc));
  const double dd = det.x * det.x + det.y * det.y;
  mindet2 = (dd < mindet2 || dd != dd) ? dd : mindet2;
  const double rd = recip_pos(dd);
  const double2 idet = make_double2(det.x * rd, -det.y * rd);
  const double2 i00 = cmul(d, idet), i01 = cneg(cmul(bb, idet)), i10 = cneg(cmul(cc, idet)),
                i11 = cmul(a, idet);
  const bool r0 = (r == P), r1 = (r == P + 1);
  const double2 g0 = cadd(cmul(f0, i00), cmul(f1, i10));
  const double2 g1 = cadd(cmul(f0, i01), cmul(f1, i11));
  const double2 b0 = r0 ? cneg(i00) : r1 ? cneg(i10) : g0;
  const double2 b1 = r0 ? cneg(i01) : r1 ? cneg(i11) : g1;
  const bool keep = !(r0 || r1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = c0 + c;
    double2 v = keep ? m[c] : make_double2(0.0, 0.0);
    v = csub(v, cmul(b0, q0[c]));
    v = csub(v, cmul(b1, q1[c]));
    m[c] = (col == P) ? cneg(b0) : (col == P + 1) ? cneg(b1) : v;
    D[r][col] = m[c];
  }
  __syncthreads();
}

__device__ double invert_pivot_block(double2 (*A)[TB + 1], double2 (*W)[TB + 1]) {
  static_assert((TB / 2) % 2 == 0, "an even number of steps ends in A");
  const int tid = threadIdx.x;
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  double2 m[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) m[c] = A[r][c0 + c];
  double mindet2 = INFINITY;
  double2 (*S)[TB + 1] = A;
  double2 (*D)[TB + 1] = W;
#pragma unroll 1
  for (int P = 0; P < TB; P += 2) {
    pivot_step(P, m, S, D, r, c0, mindet2);
    double2 (*t)[TB + 1] = S;
    S = D;
    D = t;
  }
  return sqrt(sqrt(mindet2));   // |det B|^(1/2): same scale as a scalar pivot
}

// The same inversion in single precision, for single-precision factors (their
// tile products are single precision too, and their solves are refined in
// double): the block is read from A, the steps run on two float2 views of W
// (W holds two single-precision blocks), and the inverse is written back to
// A.  The chain of dependent operations per step is shorter in single
// precision (hardware reciprocal and one Newton step), about 6.9 against
// 11.5 us per inversion.
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void pivot_step_f(int P, float2 (&m)[4], const float2 (*S)[TB + 1],
                                             float2 (*D)[TB + 1], int r, int c0, float& mindet2) {
  const float2 a = S[P][P], bb = S[P][P + 1], cc = S[P + 1][P], d = S[P + 1][P + 1];
  const float2 f0 = S[r][P], f1 = S[r][P + 1];
  float2 q0[4], q1[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    q0[c] = S[P][c0 + c];
    q1[c] = S[P + 1][c0 + c];
  }
  const float2 ad = cmulf(a, d), bc = cmulf(bb, cc);
  const float2 det = make_float2(ad.x - bc.x, ad.y - bc.y);
  const float dd = det.x * det.x + det.y * det.y;
  mindet2 = (dd < mindet2 || dd != dd) ? dd : mindet2;
  float rd = __builtin_amdgcn_rcpf(dd);
  rd = fmaf(rd, fmaf(-dd, rd, 1.0f), rd);
  const float2 idet = make_float2(det.x * rd, -det.y * rd);
  const float2 i00 = cmulf(d, idet), i11 = cmulf(a, idet);
  const float2 t01 = cmulf(bb, idet), t10 = cmulf(cc, idet);
  const float2 i01 = make_float2(-t01.x, -t01.y), i10 = make_float2(-t10.x, -t10.y);
  const bool r0 = (r == P), r1 = (r == P + 1);
  const float2 u0 = cmulf(f0, i00), u1 = cmulf(f1, i10), w0 = cmulf(f0, i01), w1 = cmulf(f1, i11);
  const float2 g0 = make_float2(u0.x + u1.x, u0.y + u1.y), g1 = make_float2(w0.x + w1.x, w0.y + w1.y);
  const float2 b0 = r0 ? make_float2(-i00.x, -i00.y) : r1 ? make_float2(-i10.x, -i10.y) : g0;
  const float2 b1 = r0 ? make_float2(-i01.x, -i01.y) : r1 ? make_float2(-i11.x, -i11.y) : g1;
  const bool keep = !(r0 || r1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = c0 + c;
    float2 v = keep ? m[c] : make_float2(0.0f, 0.0f);
    const float2 x0 = cmulf(b0, q0[c]), x1 = cmulf(b1, q1[c]);
    v = make_float2(v.x - x0.x - x1.x, v.y - x0.y - x1.y);
    m[c] = (col == P) ? make_float2(-b0.x, -b0.y) : (col == P + 1) ? make_float2(-b1.x, -b1.y) : v;
    D[r][col] = m[c];
  }
  __syncthreads();
}

__device__ double invert_pivot_block_f(double2 (*A)[TB + 1], double2 (*W)[TB + 1]) {
  static_assert(2 * sizeof(float2) == sizeof(double2), "W holds two single-precision blocks");
  const int tid = threadIdx.x;
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  float2 (*S)[TB + 1] = reinterpret_cast<float2 (*)[TB + 1]>(&W[0][0]);
  float2 (*D)[TB + 1] = S + TB;
  float2 m[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double2 v = A[r][c0 + c];
    m[c] = make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
    S[r][c0 + c] = m[c];
  }
  __syncthreads();
  float mindet2 = INFINITY;
#pragma unroll 1
  for (int P = 0; P < TB; P += 2) {
    pivot_step_f(P, m, S, D, r, c0, mindet2);
    float2 (*t)[TB + 1] = S;
    S = D;
    D = t;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) A[r][c0 + c] = make_double2(m[c].x, m[c].y);
  __syncthreads();
  return sqrt(sqrt(static_cast<double>(mindet2)));
}

// The pivot-block inverse in the precision of the factors
template <typename T>
__device__ __forceinline__ double invert_pivot(double2 (*A)[TB + 1], double2 (*W)[TB + 1]) {
  if constexpr (sizeof(T) == sizeof(float))
    return invert_pivot_block_f(A, W);
  else
    return invert_pivot_block(A, W);
}

// Complex products on the matrix cores take three real products each (Gauss):
// a b accumulates as t1 += ar br, t2 -= ai bi, t3 += (ar + ai)(br + bi), and
// the complex sum is (t1 + t2, t3 - t1 + t2).  A product to subtract passes
// -a.  A quarter fewer MFMAs than the four-product form; the rounding error of
// the imaginary part is bounded by the magnitudes of the operands rather than
// of the parts, which is the normwise accuracy the elimination relies on.
template <typename V4, typename T>
__device__ __forceinline__ void cmac3(V4& t1, V4& t2, V4& t3, T ar, T ai, T br, T bi) {
  t1 = mfma16(ar, br, t1);
  t2 = mfma16(-ai, bi, t2);
  t3 = mfma16(ar + ai, br + bi, t3);
}

template <typename V4>
__device__ __forceinline__ void zero3(V4& t1, V4& t2, V4& t3) {
  t1 = V4{0, 0, 0, 0};
  t2 = V4{0, 0, 0, 0};
  t3 = V4{0, 0, 0, 0};
}

// element q of the complex sum held by t1, t2, t3
template <typename V4>
__device__ __forceinline__ auto re3(const V4& t1, const V4& t2, int q) { return t1[q] + t2[q]; }
template <typename V4>
__device__ __forceinline__ auto im3(const V4& t1, const V4& t2, const V4& t3, int q) {
  return t3[q] - t1[q] + t2[q];
}

// (re, im) blocks (a, b), a in [a0, a1), b in [b0, b1), += the sums in t1, t2, t3
template <typename T>
__device__ __forceinline__ void fold3_blocks(typename v4of<T>::t (*re)[2], typename v4of<T>::t (*im)[2],
                                             const typename v4of<T>::t (*t1)[2],
                                             const typename v4of<T>::t (*t2)[2],
                                             const typename v4of<T>::t (*t3)[2], int a0, int a1, int b0,
                                             int b1) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (a < a0 || a >= a1 || b < b0 || b >= b1) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        re[a][b][q] += re3(t1[a][b], t2[a][b], q);
        im[a][b][q] += im3(t1[a][b], t2[a][b], t3[a][b], q);
      }
    }
}

// acc (one 32 x 32 tile in MFMA accumulator layout) -= A B^T, with A and B
// 32 x 32 row-major tiles; blocks (a, b) with a in [a0, a1), b in [b0, b1).
template <typename T>
__device__ __forceinline__ void tile_nt_update(typename v4of<T>::t (*cre)[2],
                                               typename v4of<T>::t (*cim)[2],
                                               const typename cplx<T>::t* A,
                                               const typename cplx<T>::t* B, int lr, int lk,
                                               int a0, int a1, int b0, int b1) {
  using T2 = typename cplx<T>::t;
  T2 av[2][8], bv[2][8];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      if (x >= a0 && x < a1) av[x][s] = A[(16 * x + lr) * TB + 4 * s + lk];
      if (x >= b0 && x < b1) bv[x][s] = B[(16 * x + lr) * TB + 4 * s + lk];
    }
  using V4 = typename v4of<T>::t;
  V4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) zero3(t1[a][b], t2[a][b], t3[a][b]);
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (a < a0 || a >= a1) continue;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b < b0 || b >= b1) continue;
        cmac3(t1[a][b], t2[a][b], t3[a][b], -av[a][s].x, -av[a][s].y, bv[b][s].x, bv[b][s].y);
      }
    }
  fold3_blocks<T>(cre, cim, t1, t2, t3, a0, a1, b0, b1);
}

// Trailing-update product of one tile, pipelined: acc = S - A B^T with the
// loads of S issued first (they arrive while the products run) and the
// operands A, B (32 x 32 row-major) fetched in four chunks of two k-steps,
// chunk c+1 in flight while chunk c multiplies into zeroed accumulators.
template <typename T2>
__device__ __forceinline__ void load_ksteps(T2 (&av)[2][2], T2 (&bv)[2][2], const T2* A,
                                            const T2* B, int ch, int lr, int lk) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      av[x][s] = A[(16 * x + lr) * TB + 8 * ch + 4 * s + lk];
      bv[x][s] = B[(16 * x + lr) * TB + 8 * ch + 4 * s + lk];
    }
}

// The same chunk from k-major panel tiles (element (r, k) at k TB + r).
template <typename T2>
__device__ __forceinline__ void load_ksteps_t(T2 (&av)[2][2], T2 (&bv)[2][2], const T2* A,
                                              const T2* B, int ch, int lr, int lk) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      av[x][s] = A[(8 * ch + 4 * s + lk) * TB + 16 * x + lr];
      bv[x][s] = B[(8 * ch + 4 * s + lk) * TB + 16 * x + lr];
    }
}

template <typename T>
__device__ __forceinline__ void mma_ksteps(typename v4of<T>::t (*t1)[2],
                                           typename v4of<T>::t (*t2)[2],
                                           typename v4of<T>::t (*t3)[2],
                                           const typename cplx<T>::t (&av)[2][2],
                                           const typename cplx<T>::t (&bv)[2][2]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        cmac3(t1[a][b], t2[a][b], t3[a][b], -av[a][s].x, -av[a][s].y, bv[b][s].x, bv[b][s].y);
}

template <typename T>
__device__ __forceinline__ void tile_update_pipelined(typename cplx<T>::t* dst,
                                                      const typename cplx<T>::t* A,
                                                      const typename cplx<T>::t* B, T sg,
                                                      int lr, int lk) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  T2 sv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[a][b][q] = load_stream(&dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr]);
  V4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) zero3(t1[a][b], t2[a][b], t3[a][b]);
  T2 a0[2][2], b0[2][2], a1[2][2], b1[2][2];
  load_ksteps(a0, b0, A, B, 0, lr, lk);
  load_ksteps(a1, b1, A, B, 1, lr, lk);
  mma_ksteps<T>(t1, t2, t3, a0, b0);
  load_ksteps(a0, b0, A, B, 2, lr, lk);
  mma_ksteps<T>(t1, t2, t3, a1, b1);
  load_ksteps(a1, b1, A, B, 3, lr, lk);
  mma_ksteps<T>(t1, t2, t3, a0, b0);
  mma_ksteps<T>(t1, t2, t3, a1, b1);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = (sv[a][b][q].x + re3(t1[a][b], t2[a][b], q)) * sg;
        v.y = (sv[a][b][q].y + im3(t1[a][b], t2[a][b], t3[a][b], q)) * sg;
        store_stream(&dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr], v);
      }
}

template <typename T>
__device__ __forceinline__ void tile_store_acc(typename v4of<T>::t (*cre)[2],
                                               typename v4of<T>::t (*cim)[2],
                                               typename cplx<T>::t* D, T sg, int lr, int lk) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        typename cplx<T>::t v;
        v.x = cre[a][b][q] * sg;
        v.y = cim[a][b][q] * sg;
        D[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr] = v;
      }
}

// Q tile = L tile * P with L given row-major in memory (panel kernel) ...
template <typename T>
__device__ __forceinline__ void q_from_rows(typename v4of<T>::t (*cre)[2],
                                            typename v4of<T>::t (*cim)[2],
                                            const typename cplx<T>::t (*af)[8],
                                            double2 (*Ps)[TB + 1], int lr, int lk, bool acc_kmap) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int kk = acc_kmap ? acc_k<T>(s, lk) : 4 * s + lk;
    T bre[2], bim[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      double2 pv = Ps[kk][16 * b + lr];
      bre[b] = static_cast<T>(pv.x);
      bim[b] = static_cast<T>(pv.y);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T are = af[a][s].x, aim = af[a][s].y, naim = -aim;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(are, bre[b], cre[a][b]);
        cim[a][b] = mfma16(are, bim[b], cim[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(naim, bim[b], cre[a][b]);
        cim[a][b] = mfma16(aim, bre[b], cim[a][b]);
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void zero_acc(typename v4of<T>::t (*cre)[2],
                                         typename v4of<T>::t (*cim)[2]) {
  using V4 = typename v4of<T>::t;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = V4{0, 0, 0, 0};
      cim[a][b] = V4{0, 0, 0, 0};
    }
}

// Panel 0 of a block: every workgroup inverts the pivot block, then each wave
// forms one row tile I of L (copied out) and Q = L P.
template <typename T>
__device__ void panel_work(const GJJob& jb, int wg, int nt, double2 (*Ps)[TB + 1],
                           double2 (*Ws)[TB + 1]) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  T2* X = static_cast<T2*>(jb.X);
  const int K = jb.k;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int I = wg * 4 + wave;
  const bool active = I < nt && I != K;
  {
    const T2* D = X + tile_index(K, K) * TB * TB;
    for (int e = tid; e < TB * TB; e += 256) Ps[e / TB][e % TB] = to_c128(D[e]);
  }
  T2 af[2][8];
  if (active) {
    const T2* src = (I >= K) ? X + tile_index(I, K) * TB * TB : X + tile_index(K, I) * TB * TB;
    const bool trans = I < K;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        int rr = 16 * a + lr, kk = 4 * s + lk;
        af[a][s] = trans ? src[kk * TB + rr] : src[rr * TB + kk];
      }
  }
  __syncthreads();
  const double minpiv = invert_pivot<T>(Ps, Ws);
  if (wg == 0) {
    for (int e = tid; e < TB * TB; e += 256) jb.Pn[e] = Ps[e / TB][e % TB];
    if (tid == 0) *jb.health = minpiv;
  }
  if (!active) return;
  T2* Lb = static_cast<T2*>(jb.Ln) + size_t(I) * TB * TB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int s = 0; s < 8; ++s) Lb[(16 * a + lr) * TB + 4 * s + lk] = af[a][s];
  V4 cre[2][2], cim[2][2];
  zero_acc<T>(cre, cim);
  q_from_rows<T>(cre, cim, af, Ps, lr, lk, false);
  tile_store_acc<T>(cre, cim, static_cast<T2*>(jb.Qn) + size_t(I) * TB * TB, T(1), lr, lk);
}

// Trailing update k: one wave per packed tile, skipping tile column `skip`.
template <typename T>
__device__ void update_work(const GJJob& jb, int wg, size_t tiles, int skip) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const size_t t = size_t(wg) * 4 + wave;
  if (t >= tiles) return;
  int I, J;
  tile_coords(static_cast<int>(t), &I, &J);
  if (I == skip || J == skip) return;
  const int K = jb.k;
  T2* dst = static_cast<T2*>(jb.X) + t * TB * TB;
  const T sg = jb.last ? T(-1) : T(1);
  const T2* Q = static_cast<const T2*>(jb.Q);
  const T2* L = static_cast<const T2*>(jb.L);
  if (I == K && J == K) {
    for (int e = lane; e < TB * TB; e += 64) {
      double2 p = jb.P[e];
      T2 v;
      v.x = static_cast<T>(-p.x) * sg;
      v.y = static_cast<T>(-p.y) * sg;
      dst[e] = v;
    }
    return;
  }
  if (J == K || I == K) {
    const T2* q = Q + size_t(J == K ? I : J) * TB * TB;
    for (int e = lane; e < TB * TB; e += 64) {
      int rr = e / TB, cc = e % TB;
      T2 v = (J == K) ? q[e] : q[cc * TB + rr];
      v.x *= sg;
      v.y *= sg;
      dst[e] = v;
    }
    return;
  }
  const int lr = lane & 15, lk = lane >> 4;
  tile_update_pipelined<T>(dst, Q + size_t(I) * TB * TB, L + size_t(J) * TB * TB, sg, lr, lk);
}

// Look-ahead for panel Kn = k + 1.  Workgroup g handles the R row tiles
// I = g R .. g R + R - 1, one wave per 16 x 16 quadrant (qa, qb):
//  1. the two 16 x 16 blocks (a', qa), a' = 0, 1, of L_{Kn}[I]^T
//     after update k, in accumulator layout:
//       I >  Kn: S(I,Kn)^T - L_k[Kn] Q_k[I]^T
//       I <  Kn, I != k: S(Kn,I) - Q_k[Kn] L_k[I]^T
//       I == k: Q_k[Kn]                  (tile (Kn, k) lies in pivot column k)
//     these registers are rows 16 qa .. 16 qa + 15 of L_{Kn}[I], i.e. the left
//     operand of Q = L P, without a transpose;
//  2. quadrant (qa, qb) of the updated pivot block S(Kn,Kn) - Q_k[Kn] L_k[Kn]^T
//     into LDS; 3. invert it (all waves); 4. per row tile, quadrant (qa, qb) of
//     Q_{Kn}[I] = L_{Kn}[I] P.
// Every look-ahead workgroup of a chain inverts the same pivot block: R = 2
// halves those redundant inversions when sixteen chains share the GPU.
template <typename T>
__device__ __forceinline__ void lt_row(const GJJob& jb, int I, typename v4of<T>::t (*cre)[2],
                                       typename v4of<T>::t (*cim)[2], int lr, int lk, int qa,
                                       int qb) {
  using T2 = typename cplx<T>::t;
  const T2* X = static_cast<const T2*>(jb.X);
  const T2* Q = static_cast<const T2*>(jb.Q);
  const T2* L = static_cast<const T2*>(jb.L);
  const int k = jb.k, Kn = k + 1;
  // accumulator init: element (i, j) of block (a', qa) of L^T
  const T2* src;
  bool tr;
  if (I == k) {
    src = Q + size_t(Kn) * TB * TB;
    tr = false;
  } else if (I > Kn) {
    src = X + tile_index(I, Kn) * TB * TB;
    tr = true;
  } else {
    src = X + tile_index(Kn, I) * TB * TB;
    tr = false;
  }
#pragma unroll
  for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * a2 + mfma_row<T>(lk, q), j = 16 * qa + lr;
      T2 v = tr ? src[j * TB + i] : src[i * TB + j];
      cre[a2][0][q] = v.x;
      cim[a2][0][q] = v.y;
    }
  if (I > Kn)
    tile_nt_update<T>(cre, cim, L + size_t(Kn) * TB * TB, Q + size_t(I) * TB * TB + 16 * qa * TB,
                      lr, lk, 0, 2, 0, 1);
  else if (I != k)
    tile_nt_update<T>(cre, cim, Q + size_t(Kn) * TB * TB, L + size_t(I) * TB * TB + 16 * qa * TB,
                      lr, lk, 0, 2, 0, 1);
  if (qb == 0) {   // rows 16 qa .. of L_{Kn}[I] for the update of panel Kn
    T2* Lb = static_cast<T2*>(jb.Ln) + size_t(I) * TB * TB;
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = cre[a2][0][q];
        v.y = cim[a2][0][q];
        Lb[(16 * qa + lr) * TB + 16 * a2 + mfma_row<T>(lk, q)] = v;
      }
  }
}

// Quadrant (qa, qb) of Q_{Kn}[I]: A fragments (row 16 qa + lr, k-step 4 a' + q)
// come from the L^T accumulators, B fragments from P with the matching k index.
template <typename T>
__device__ __forceinline__ void q_row(const GJJob& jb, int I, const typename v4of<T>::t (*cre)[2],
                                      const typename v4of<T>::t (*cim)[2], double2 (*Ps)[TB + 1],
                                      int lr, int lk, int qa, int qb) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  V4 t1, t2, t3;
  zero3(t1, t2, t3);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const double2 pv = Ps[acc_k<T>(s, lk)][16 * qb + lr];
    cmac3(t1, t2, t3, cre[s >> 2][0][s & 3], cim[s >> 2][0][s & 3], static_cast<T>(pv.x),
          static_cast<T>(pv.y));
  }
  T2* Qb = static_cast<T2*>(jb.Qn) + size_t(I) * TB * TB + (16 * qa) * TB + 16 * qb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T2 v;
    v.x = re3(t1, t2, q);
    v.y = im3(t1, t2, t3, q);
    Qb[mfma_row<T>(lk, q) * TB + lr] = v;
  }
}

template <typename T, int R>
__device__ void lookahead_work(const GJJob& jb, int g, int nt, double2 (*Ps)[TB + 1],
                               double2 (*Ws)[TB + 1]) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const T2* X = static_cast<const T2*>(jb.X);
  const T2* Q = static_cast<const T2*>(jb.Q);
  const T2* L = static_cast<const T2*>(jb.L);
  const int Kn = jb.k + 1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int qa = wave >> 1, qb = wave & 1;
  V4 cre[R][2][2], cim[R][2][2];   // per row tile: [a'][0] used
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int I = g * R + r;
    if (I < nt && I != Kn) lt_row<T>(jb, I, cre[r], cim[r], lr, lk, qa, qb);
  }
  {  // quadrant (qa, qb) of the updated pivot block
    V4 dre[2][2], dim[2][2];
    const T2* S = X + tile_index(Kn, Kn) * TB * TB + (16 * qa) * TB + 16 * qb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T2 v = S[mfma_row<T>(lk, q) * TB + lr];
      dre[0][0][q] = v.x;
      dim[0][0][q] = v.y;
    }
    tile_nt_update<T>(dre, dim, Q + size_t(Kn) * TB * TB + (16 * qa) * TB,
                      L + size_t(Kn) * TB * TB + (16 * qb) * TB, lr, lk, 0, 1, 0, 1);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      Ps[16 * qa + mfma_row<T>(lk, q)][16 * qb + lr] =
          make_double2(static_cast<double>(dre[0][0][q]), static_cast<double>(dim[0][0][q]));
  }
  __syncthreads();
  const double minpiv = invert_pivot<T>(Ps, Ws);
  if (g == 0) {
    for (int e = tid; e < TB * TB; e += 256) jb.Pn[e] = Ps[e / TB][e % TB];
    if (tid == 0) *jb.health = minpiv;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int I = g * R + r;
    if (I < nt && I != Kn) q_row<T>(jb, I, cre[r], cim[r], Ps, lr, lk, qa, qb);
  }
}

// ---------------------------------------------------------------------------
// Two panels per pass.  Launch j applies panels K = k and K2 = k+1 to every
// tile (a rank-64 update, each tile read and written once for two panels)
// while the look-ahead workgroups form panels K3 = k+2 and K4 = k+3 from the
// tiles as they were before the pass.  With S the tiles before, S' after
// panel K and S'' after both, on the full symmetric matrix (L0, Q0, P0 of
// panel K; L1, Q1, P1 of panel K2, whose L1 = S'(:, K2)):
//   S''_IJ = S_IJ - Q0_I L0_J^T - Q1_I L1_J^T              I, J not in {K, K2}
//   S''_IK = Q0_I - Q1_I Q0_K2                              I != K, K2
//   S''_KK = -P0 - Q1_K Q0_K2
//   S''_I,K2 = Q1_I,   S''_K2,K2 = -P1
// since S'_K,K2 = (Q0_K2)^T.  The look-ahead takes L3 = S''(:, K3), P3, Q3 and
// then L4_I = S''_I,K4 - Q3_I (L3_K4)^T = S''_I,K4 - S''_I,K3 (Q3_K4)^T (P3 is
// symmetric), P4 = (S''_K4,K4 - Q3_K4 L3_K4^T)^{-1}, Q4 = L4 P4.  Panel p lives
// in slot p mod 4 of its chain's four panel buffers, each 32 x 32 panel tile
// stored k-major (element (r, k) at k TB + r): the sixteen lanes that supply
// one MFMA operand column then read 256 contiguous bytes instead of sixteen
// rows.  A block opens with pass K = -2, which applies nothing and forms
// panels 0 and 1 by the same pivot work and row launch.
struct GJ2Job {
  int k;         // first panel of the pair this launch applies
  int nlook;     // panels formed ahead: 0, 1 (k+2) or 2 (k+2, k+3)
  int last;      // final pass: negate the result
  int wgs;       // workgroups of this job (update part + look-ahead part)
  int wgs_upd;   // of which the trailing-update part
  void* X;       // packed tiles of the block
  void* Lb;      // slot 0 of the chain's L panel buffers (np x TB each)
  void* Qb;
  double2* Pb;   // slot 0 of the chain's pivot-block inverses (TB x TB each)
  double* health;   // min |pivot| slots of this block, one per panel
  int nt;        // tiles per block edge (per job: chains may differ in size)
  int tiles;     // packed tiles per block
  int open;      // k_gj2_step: 1 = this job opens its block (Schur complement
                 // formed beside the pivot work of panels 0 and 1)
};
struct GJ2Jobs {
  GJ2Job j[MAXJ];
  int n;
  XMap x;
};

__device__ __forceinline__ GJ2Job pick2(const GJ2Jobs& js, int q) {
#define RCP_SEL(fld) RCP_SEL16(js, q, fld)
  GJ2Job jb;
  jb.k = RCP_SEL(k);
  jb.nlook = RCP_SEL(nlook);
  jb.last = RCP_SEL(last);
  jb.wgs = RCP_SEL(wgs);
  jb.wgs_upd = RCP_SEL(wgs_upd);
  jb.X = RCP_SEL(X);
  jb.Lb = RCP_SEL(Lb);
  jb.Qb = RCP_SEL(Qb);
  jb.Pb = RCP_SEL(Pb);
  jb.health = RCP_SEL(health);
  jb.nt = RCP_SEL(nt);
  jb.tiles = RCP_SEL(tiles);
  jb.open = RCP_SEL(open);
#undef RCP_SEL
  return jb;
}

// Panel buffers of panel p (slot p mod 4); a buffer holds nt row tiles.
template <typename T2>
__device__ __forceinline__ T2* slot_ptr(void* base, int p, int nt) {
  return static_cast<T2*>(base) + size_t(p & 3) * nt * TB * TB;
}

// acc (MFMA accumulator layout) -= A B with A, B k-major TB x TB panel tiles
// (element (r, k) at k TB + r; B not transposed); blocks (a, b) with a in
// [a0, a1), b in [b0, b1).
template <typename T>
__device__ __forceinline__ void tile_nn_update(typename v4of<T>::t (*cre)[2],
                                               typename v4of<T>::t (*cim)[2],
                                               const typename cplx<T>::t* A,
                                               const typename cplx<T>::t* B, int lr, int lk,
                                               int a0, int a1, int b0, int b1) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  V4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) zero3(t1[a][b], t2[a][b], t3[a][b]);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int kk = 4 * s + lk;
    T2 av[2], bv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      if (x >= a0 && x < a1) av[x] = A[kk * TB + 16 * x + lr];
      if (x >= b0 && x < b1) bv[x] = B[(16 * x + lr) * TB + kk];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (a < a0 || a >= a1) continue;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b < b0 || b >= b1) continue;
        cmac3(t1[a][b], t2[a][b], t3[a][b], -av[a].x, -av[a].y, bv[b].x, bv[b].y);
      }
    }
  }
  fold3_blocks<T>(cre, cim, t1, t2, t3, a0, a1, b0, b1);
}

// dst = sg (S - A0 B0^T - A1 B1^T) with k-major panel tiles A0, B0, A1, B1:
// eight chunks of two k-steps into zeroed accumulators, each chunk requested
// two chunks ahead of its products (a chunk's products take less than a round
// trip to L2 in single precision); S is added at the end.  Vector loads retire
// in issue order, so the tile S (from HBM) is requested after the first three
// chunks (from L2): the first products wait only for L2, and S arrives while
// they run.
template <typename T>
__device__ __forceinline__ void tile_update2_pipelined(typename cplx<T>::t* dst,
                                                       const typename cplx<T>::t* A0,
                                                       const typename cplx<T>::t* B0,
                                                       const typename cplx<T>::t* A1,
                                                       const typename cplx<T>::t* B1, T sg,
                                                       int lr, int lk) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  V4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) zero3(t1[a][b], t2[a][b], t3[a][b]);
  // eight chunks of two k-steps (four from panel k, four from panel k + 1),
  // each requested two chunks ahead of its products
  T2 av[3][2][2], bv[3][2][2];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) load_ksteps_t(av[ch], bv[ch], A0, B0, ch, lr, lk);
  T2 sv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[a][b][q] = load_stream(&dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr]);
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    mma_ksteps<T>(t1, t2, t3, av[ch % 3], bv[ch % 3]);
    const int nx = ch + 3;
    if (nx < 8) load_ksteps_t(av[ch % 3], bv[ch % 3], nx < 4 ? A0 : A1, nx < 4 ? B0 : B1, nx & 3, lr, lk);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = (sv[a][b][q].x + re3(t1[a][b], t2[a][b], q)) * sg;
        v.y = (sv[a][b][q].y + im3(t1[a][b], t2[a][b], t3[a][b], q)) * sg;
        store_stream(&dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr], v);
      }
}

// Pass with panels K, K2 = K + 1 on one packed tile per wave.
template <typename T>
__device__ void update2_work(const GJ2Job& jb, int wg, int nt, size_t tiles) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const size_t t = size_t(wg) * 4 + wave;
  if (t >= tiles) return;
  int I, J;
  tile_coords(static_cast<int>(t), &I, &J);
  const int K = jb.k, K2 = K + 1;
  // the pivot tiles of the next pair belong to its pivot work (which reads
  // them as they were before this pass); every other tile is updated, so the
  // next pair's columns hold S'' for its row panels
  if (jb.nlook >= 1 && I == K + 2 && J == K + 2) return;
  if (jb.nlook >= 2 && I == K + 3 && (J == K + 2 || J == K + 3)) return;
  T2* dst = static_cast<T2*>(jb.X) + t * TB * TB;
  const T sg = jb.last ? T(-1) : T(1);
  const T2* L0 = slot_ptr<T2>(jb.Lb, K, nt);
  const T2* Q0 = slot_ptr<T2>(jb.Qb, K, nt);
  const T2* L1 = slot_ptr<T2>(jb.Lb, K2, nt);
  const T2* Q1 = slot_ptr<T2>(jb.Qb, K2, nt);
  const double2* P0 = jb.Pb + size_t(K & 3) * TB * TB;
  const double2* P1 = jb.Pb + size_t(K2 & 3) * TB * TB;
  const size_t TT = size_t(TB) * TB;
  if (I == K2 && J == K2) {
    for (int e = lane; e < TB * TB; e += 64) {
      T2 v;
      v.x = static_cast<T>(-P1[e].x) * sg;
      v.y = static_cast<T>(-P1[e].y) * sg;
      dst[e] = v;
    }
    return;
  }
  if (J == K2 || I == K2) {
    const T2* q = Q1 + (J == K2 ? I : J) * TT;
    for (int e = lane; e < TB * TB; e += 64) {
      const int rr = e / TB, cc = e % TB;
      T2 v = (J == K2) ? q[cc * TB + rr] : q[e];
      v.x *= sg;
      v.y *= sg;
      dst[e] = v;
    }
    return;
  }
  const int lr = lane & 15, lk = lane >> 4;
  if (I == K || J == K) {
    // column K: Q0_R - Q1_R Q0_K2 for row R (R = I below the pivot, R = J in
    // row K, stored transposed); the pivot tile: -P0 - Q1_K Q0_K2
    const int R = (J == K) ? I : J;
    V4 cre[2][2], cim[2][2];
    zero_acc<T>(cre, cim);
    tile_nn_update<T>(cre, cim, Q1 + R * TT, Q0 + K2 * TT, lr, lk, 0, 2, 0, 2);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = 16 * a + mfma_row<T>(lk, q), cc = 16 * b + lr;
          double2 base;
          if (I == K && J == K) {
            base = cneg(P0[rr * TB + cc]);
          } else {
            base = to_c128(Q0[R * TT + cc * TB + rr]);
          }
          T2 v;
          v.x = (static_cast<T>(base.x) + cre[a][b][q]) * sg;
          v.y = (static_cast<T>(base.y) + cim[a][b][q]) * sg;
          if (J == K)
            dst[rr * TB + cc] = v;
          else
            dst[cc * TB + rr] = v;
        }
    return;
  }
  tile_update2_pipelined<T>(dst, Q0 + I * TT, L0 + J * TT, Q1 + I * TT, L1 + J * TT, sg, lr, lk);
}

// acc (one 16 x 16 block) -= A B^T over the 32 k of k-major panel tiles, A and
// B offset to the block's first row (element (r, k) at k TB + r).
template <typename T>
__device__ __forceinline__ void quad_nt_update_t(typename v4of<T>::t& cre, typename v4of<T>::t& cim,
                                                 const typename cplx<T>::t* A,
                                                 const typename cplx<T>::t* B, int lr, int lk) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  T2 av[8], bv[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    av[s] = A[(4 * s + lk) * TB + lr];
    bv[s] = B[(4 * s + lk) * TB + lr];
  }
  V4 t1, t2, t3;
  zero3(t1, t2, t3);
#pragma unroll
  for (int s = 0; s < 8; ++s) cmac3(t1, t2, t3, -av[s].x, -av[s].y, bv[s].x, bv[s].y);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cre[q] += re3(t1, t2, q);
    cim[q] += im3(t1, t2, t3, q);
  }
}

// Quadrant (qa, qb) of S''_{R,C} for R >= C, R, C not in {K, K2}.
template <typename T>
__device__ __forceinline__ void quad2(const GJ2Job& jb, int nt, int R, int C,
                                      typename v4of<T>::t (*dre)[2],
                                      typename v4of<T>::t (*dim)[2], int lr, int lk, int qa,
                                      int qb) {
  using T2 = typename cplx<T>::t;
  const T2* X = static_cast<const T2*>(jb.X);
  const int K = jb.k, K2 = K + 1;
  const size_t TT = size_t(TB) * TB;
  const T2* S = X + tile_index(R, C) * TT + (16 * qa) * TB + 16 * qb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T2 v = S[mfma_row<T>(lk, q) * TB + lr];
    dre[0][0][q] = v.x;
    dim[0][0][q] = v.y;
  }
  if (K < 0) return;   // the start of a block: no panels applied yet
  quad_nt_update_t<T>(dre[0][0], dim[0][0], slot_ptr<T2>(jb.Qb, K, nt) + R * TT + 16 * qa,
                      slot_ptr<T2>(jb.Lb, K, nt) + C * TT + 16 * qb, lr, lk);
  quad_nt_update_t<T>(dre[0][0], dim[0][0], slot_ptr<T2>(jb.Qb, K2, nt) + R * TT + 16 * qa,
                      slot_ptr<T2>(jb.Lb, K2, nt) + C * TT + 16 * qb, lr, lk);
}

template <typename T>
__device__ __forceinline__ void quad_to_lds(const typename v4of<T>::t (*dre)[2],
                                            const typename v4of<T>::t (*dim)[2],
                                            double2 (*D)[TB + 1], int lr, int lk, int qa, int qb) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    D[16 * qa + mfma_row<T>(lk, q)][16 * qb + lr] =
        make_double2(static_cast<double>(dre[0][0][q]), static_cast<double>(dim[0][0][q]));
}

// L^T accumulator blocks (a', qa) -> rows 16 qa .. of the L panel tile.
template <typename T>
__device__ __forceinline__ void store_lt(const typename v4of<T>::t (*cre)[2],
                                         const typename v4of<T>::t (*cim)[2],
                                         typename cplx<T>::t* Lt, int lr, int lk, int qa) {
  using T2 = typename cplx<T>::t;
#pragma unroll
  for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T2 v;
      v.x = cre[a2][0][q];
      v.y = cim[a2][0][q];
      Lt[(16 * a2 + mfma_row<T>(lk, q)) * TB + 16 * qa + lr] = v;
    }
}

// Quadrant (qa, qb) of Q = L P from L^T accumulator blocks and the P fragment
// pf[s] = P[acc_k(s)][16 qb + lr] (loaded beforehand).
template <typename T>
__device__ __forceinline__ void q_quad_f(const typename v4of<T>::t (*cre)[2],
                                         const typename v4of<T>::t (*cim)[2], const double2 (&pf)[8],
                                         typename cplx<T>::t* Qt, int lr, int lk, int qa, int qb) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  V4 t1, t2, t3;
  zero3(t1, t2, t3);
#pragma unroll
  for (int s = 0; s < 8; ++s)
    cmac3(t1, t2, t3, cre[s >> 2][0][s & 3], cim[s >> 2][0][s & 3], static_cast<T>(pf[s].x),
          static_cast<T>(pf[s].y));
  T2* Qb = Qt + (16 * qb) * TB + 16 * qa;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T2 v;
    v.x = re3(t1, t2, q);
    v.y = im3(t1, t2, t3, q);
    Qb[lr * TB + mfma_row<T>(lk, q)] = v;
  }
}

// Pivot work of the next pair, once per chain (the last workgroup-sized job of
// a pass): P3 = S''_{K3,K3}^{-1}; with K4: E = L3_K4 = S''_{K4,K3} and
// Q3_K4 = E P3 (their rows of the K3 panel buffers), P4 = (S''_{K4,K4} -
// Q3_K4 E^T)^{-1}.  Columns K3 and K4 are not touched by the pass, so this
// reads the tiles as they were before it.  The exchange rows of each
// inversion live in a buffer that is idle at the time.
template <typename T>
__device__ void pivot2_work(const GJ2Job& jb, int nt, double2 (*B1)[TB + 1],
                            double2 (*B2)[TB + 1], double2 (*B3)[TB + 1]) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const int K = jb.k, K3 = K + 2, K4 = K + 3;
  const bool two = jb.nlook == 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int qa = wave >> 1, qb = wave & 1;
  const size_t TT = size_t(TB) * TB;
  // The three quadrants of the pivot area (K3 K3, K4 K3, K4 K4) are formed
  // before the first inversion, so that their loads overlap one another and
  // the inversion, not the chain of pivot work; E waits in B2, D4 in registers.
  V4 dre[1][2], dim[1][2], ere[1][2], eim[1][2], fre[1][2], fim[1][2];
  quad2<T>(jb, nt, K3, K3, dre, dim, lr, lk, qa, qb);
  if (two) {
    quad2<T>(jb, nt, K4, K3, ere, eim, lr, lk, qa, qb);
    quad2<T>(jb, nt, K4, K4, fre, fim, lr, lk, qa, qb);
  }
  quad_to_lds<T>(dre, dim, B1, lr, lk, qa, qb);
  if (two) {
    quad_to_lds<T>(ere, eim, B2, lr, lk, qa, qb);
    // E is row K4 of the K3 panel's L buffer
    T2* Lt = slot_ptr<T2>(jb.Lb, K3, nt) + K4 * TT + (16 * qb) * TB + 16 * qa;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T2 v;
      v.x = ere[0][0][q];
      v.y = eim[0][0][q];
      Lt[lr * TB + mfma_row<T>(lk, q)] = v;
    }
  }
  __syncthreads();
  const double min3 = invert_pivot<T>(B1, B3);   // P3
  double2* P3 = jb.Pb + size_t(K3 & 3) * TT;
  for (int e = tid; e < TB * TB; e += 256) P3[e] = B1[e / TB][e % TB];
  if (tid == 0) jb.health[K3] = min3;
  if (!two) return;
  V4 qre, qim;   // Q3_K4 = E P3, quadrant (qa, qb)
  {
    V4 t1, t2, t3;
    zero3(t1, t2, t3);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int kk = 4 * s + lk;
      const double2 av = B2[16 * qa + lr][kk], pv = B1[kk][16 * qb + lr];
      cmac3(t1, t2, t3, static_cast<T>(av.x), static_cast<T>(av.y), static_cast<T>(pv.x),
            static_cast<T>(pv.y));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      qre[q] = re3(t1, t2, q);
      qim[q] = im3(t1, t2, t3, q);
    }
  }
  {
    T2* Qt = slot_ptr<T2>(jb.Qb, K3, nt) + K4 * TT + (16 * qb) * TB + 16 * qa;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      B3[16 * qa + mfma_row<T>(lk, q)][16 * qb + lr] =
          make_double2(static_cast<double>(qre[q]), static_cast<double>(qim[q]));
      T2 v;
      v.x = qre[q];
      v.y = qim[q];
      Qt[lr * TB + mfma_row<T>(lk, q)] = v;
    }
  }
  __syncthreads();
  {   // D4' = D4 - Q3_K4 E^T
    V4 t1, t2, t3;
    zero3(t1, t2, t3);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int kk = 4 * s + lk;
      const double2 av = B3[16 * qa + lr][kk], bv = B2[16 * qb + lr][kk];
      cmac3(t1, t2, t3, static_cast<T>(-av.x), static_cast<T>(-av.y), static_cast<T>(bv.x),
            static_cast<T>(bv.y));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      fre[0][0][q] += re3(t1, t2, q);
      fim[0][0][q] += im3(t1, t2, t3, q);
    }
  }
  __syncthreads();
  quad_to_lds<T>(fre, fim, B2, lr, lk, qa, qb);
  __syncthreads();
  const double min4 = invert_pivot<T>(B2, B1);   // P4
  double2* P4 = jb.Pb + size_t(K4 & 3) * TT;
  for (int e = tid; e < TB * TB; e += 256) P4[e] = B2[e / TB][e % TB];
  if (tid == 0) jb.health[K4] = min4;
  // Row tile K3 of panel K4, from what is at hand: L4_K3 = (Q3_K4)^T (B3)
  // and Q4_K3 = L4_K3 P4 (B2), so that the row launch takes only the rows
  // outside the pivot pair
  {
    V4 cre[2][2], cim[2][2];
    double2 pf[8];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 v = B3[16 * a2 + mfma_row<T>(lk, q)][16 * qa + lr];
        cre[a2][0][q] = static_cast<T>(v.x);
        cim[a2][0][q] = static_cast<T>(v.y);
      }
#pragma unroll
    for (int s = 0; s < 8; ++s) pf[s] = B2[acc_k<T>(s, lk)][16 * qb + lr];
    if (qb == 0) store_lt<T>(cre, cim, slot_ptr<T2>(jb.Lb, K4, nt) + K3 * TT, lr, lk, qa);
    q_quad_f<T>(cre, cim, pf, slot_ptr<T2>(jb.Qb, K4, nt) + K3 * TT, lr, lk, qa, qb);
  }
}

// Rows 16 qa .. 16 qa + 15 of tile (I, C) of the full symmetric matrix as the
// accumulator blocks (a', qa), a' = 0, 1, of its transpose, from the packed
// tiles (tile (I, C) for I > C, tile (C, I) transposed for I < C), staged in
// LDS first.
// Staging: the stored tile (max(I, C), min(I, C)) copied row-major into LDS by
// the workgroup with contiguous loads.
template <typename T>
__device__ __forceinline__ void stage_tile(const GJ2Job& jb, int I, int C,
                                           typename cplx<T>::t (*lds)[TB + 1]) {
  using T2 = typename cplx<T>::t;
  const T2* src = static_cast<const T2*>(jb.X) +
                  (I > C ? tile_index(I, C) : tile_index(C, I)) * size_t(TB) * TB;
  for (int e = threadIdx.x; e < TB * TB; e += 256) lds[e / TB][e % TB] = src[e];
}

// Reading the rows from the staged tile (below: the stored tile is (I, C)).
template <typename T>
__device__ __forceinline__ void load_lt_lds(const typename cplx<T>::t (*lds)[TB + 1], bool below,
                                            typename v4of<T>::t (*cre)[2],
                                            typename v4of<T>::t (*cim)[2], int lr, int lk, int qa) {
#pragma unroll
  for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * a2 + mfma_row<T>(lk, q), j = 16 * qa + lr;
      const typename cplx<T>::t v = below ? lds[j][i] : lds[i][j];
      cre[a2][0][q] = v.x;
      cim[a2][0][q] = v.y;
    }
}

// Row tile I (outside the pivot pair K3, K4) of the next pair's panels after
// the pass, whose tiles of columns K3, K4 now hold S'': L3_I = S''_{I,K3},
// Q3_I = L3_I P3; with K4: L4_I = S''_{I,K4} - L3_I (Q3_K4)^T, Q4_I = L4_I P4.
// Rows K3 and K4 of the panels and the pivots come from the pivot work.  The
// operands of the first two products are loaded before the first store, so
// one memory latency covers them.
template <typename T>
__device__ void rows2_work(const GJ2Job& jb, int I, int nt, typename cplx<T>::t (*lt)[TB][TB + 1],
                           typename cplx<T>::t (*xch)[4][64]) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const int K = jb.k, K3 = K + 2, K4 = K + 3;
  const bool two = jb.nlook == 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int qa = wave >> 1, qb = wave & 1;
  const size_t TT = size_t(TB) * TB;
  const double2* P3 = jb.Pb + size_t(K3 & 3) * TT;
  const double2* P4 = jb.Pb + size_t(K4 & 3) * TT;
  const T2* Qk = slot_ptr<T2>(jb.Qb, K3, nt) + K4 * TT;
  V4 c3re[2][2], c3im[2][2], c4re[2][2], c4im[2][2];
  double2 p3[8], p4[8];
  T2 qk[8];   // row block qb of Q3_K4, the part of the L4 update this wave does
  // S''_{I,K3} (and S''_{I,K4}) through LDS: half of them are stored
  // transposed, and a direct read in the accumulator layout would take
  // sixteen rows per quarter-wave
  stage_tile<T>(jb, I, K3, lt[0]);
  if (two) stage_tile<T>(jb, I, K4, lt[1]);
#pragma unroll
  for (int s = 0; s < 8; ++s) p3[s] = P3[acc_k<T>(s, lk) * TB + 16 * qb + lr];
  if (two) {
#pragma unroll
    for (int s = 0; s < 8; ++s) qk[s] = Qk[acc_k<T>(s, lk) * TB + 16 * qb + lr];
  }
  __syncthreads();
  load_lt_lds<T>(lt[0], I > K3, c3re, c3im, lr, lk, qa);
  if (two) load_lt_lds<T>(lt[1], I > K4, c4re, c4im, lr, lk, qa);
  if (qb == 0) store_lt<T>(c3re, c3im, slot_ptr<T2>(jb.Lb, K3, nt) + I * TT, lr, lk, qa);
  q_quad_f<T>(c3re, c3im, p3, slot_ptr<T2>(jb.Qb, K3, nt) + I * TT, lr, lk, qa, qb);
  if (!two) return;
  // P4 is needed only by the last product: loaded here, it arrives during the
  // L4 update and exchange, and its registers are free during Q3
#pragma unroll
  for (int s = 0; s < 8; ++s) p4[s] = P4[acc_k<T>(s, lk) * TB + 16 * qb + lr];
  // L4_I^T -= Q3_K4 L3_I^T, right operand from the L3 blocks: block (qb, qa)
  // here, block (1 - qb, qa) in the wave of the same qa, exchanged in LDS
  V4 hre = qb ? c4re[1][0] : c4re[0][0];
  V4 him = qb ? c4im[1][0] : c4im[0][0];
  {
    V4 t1, t2, t3;
    zero3(t1, t2, t3);
#pragma unroll
    for (int s = 0; s < 8; ++s)
      cmac3(t1, t2, t3, -qk[s].x, -qk[s].y, c3re[s >> 2][0][s & 3], c3im[s >> 2][0][s & 3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hre[q] += re3(t1, t2, q);
      him[q] += im3(t1, t2, t3, q);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T2 v;
    v.x = hre[q];
    v.y = him[q];
    xch[wave][q][lane] = v;
  }
  __syncthreads();
  V4 ore, oim;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T2 v = xch[wave ^ 1][q][lane];
    ore[q] = v.x;
    oim[q] = v.y;
  }
  c4re[0][0] = qb ? ore : hre;
  c4im[0][0] = qb ? oim : him;
  c4re[1][0] = qb ? hre : ore;
  c4im[1][0] = qb ? him : oim;
  if (qb == 0) store_lt<T>(c4re, c4im, slot_ptr<T2>(jb.Lb, K4, nt) + I * TT, lr, lk, qa);
  q_quad_f<T>(c4re, c4im, p4, slot_ptr<T2>(jb.Qb, K4, nt) + I * TT, lr, lk, qa, qb);
}

// Host: the placement of n jobs whose workgroup counts are wgs[q] (a job's
// share of the 16 half-slots follows its share of the workgroups, at least
// one each; a job with an even share takes whole XCDs, the odd remainders are
// paired largest with smallest), and the grid that covers it.
int build_xmap(const int* wgs, int n, XMap* m) {
  long long total = 0;
  for (int q = 0; q < n; ++q) total += wgs[q] > 0 ? wgs[q] : 0;
  int u[MAXJ] = {};
  int used = 0;
  double frac[MAXJ] = {};
  for (int q = 0; q < n; ++q) {
    const double ideal = total > 0 ? double(NHALF) * (wgs[q] > 0 ? wgs[q] : 0) / double(total) : 0.0;
    u[q] = static_cast<int>(ideal);
    if (u[q] < 1) u[q] = 1;
    frac[q] = ideal - u[q];
    used += u[q];
  }
  while (used > NHALF) {   // minimum shares overshot: take from the largest
    int big = 0;
    for (int q = 1; q < n; ++q) if (u[q] > u[big]) big = q;
    --u[big];
    --used;
  }
  while (used < NHALF) {   // largest remainders first
    int best = 0;
    for (int q = 1; q < n; ++q) if (frac[q] > frac[best]) best = q;
    ++u[best];
    frac[best] -= 1.0;
    ++used;
  }
  int hq[NHALF], hoff[NHALF], hstr[NHALF];
  int h = 0;
  int single[MAXJ], ns = 0;
  for (int q = 0; q < n; ++q) {   // whole XCDs
    for (int i = 0; i + 1 < u[q]; i += 2) {
      hq[h] = q; hoff[h] = i; hstr[h] = u[q]; ++h;
      hq[h] = q; hoff[h] = i + 1; hstr[h] = u[q]; ++h;
    }
    if (u[q] & 1) single[ns++] = q;
  }
  // odd remainders: sort by load per half-slot, pair largest with smallest
  for (int a = 1; a < ns; ++a)
    for (int b = a; b > 0; --b) {
      const int x = single[b], y = single[b - 1];
      if (double(wgs[x]) / u[x] > double(wgs[y]) / u[y]) {
        single[b] = y;
        single[b - 1] = x;
      } else {
        break;
      }
    }
  for (int a = 0, b = ns - 1; a <= b; ++a, --b) {
    const int qa = single[a];
    hq[h] = qa; hoff[h] = u[qa] - 1; hstr[h] = u[qa]; ++h;
    if (a != b) {
      const int qb = single[b];
      hq[h] = qb; hoff[h] = u[qb] - 1; hstr[h] = u[qb]; ++h;
    } else {
      hq[h] = -1; hoff[h] = 0; hstr[h] = 1; ++h;
    }
  }
  int slots = 0;   // per half-slot
  for (int i = 0; i < NHALF; ++i) {
    m->q[i] = i < h ? hq[i] : -1;
    m->off[i] = i < h ? hoff[i] : 0;
    m->stride[i] = i < h ? hstr[i] : 1;
    if (m->q[i] >= 0) {
      const int r = ceil_div(wgs[m->q[i]] - m->off[i], m->stride[i]);
      if (r > slots) slots = r;
    }
  }
  return 8 * 2 * slots;
}

// Places a job table's jobs (by their workgroup counts) and returns the grid.
template <typename Jobs>
int map_jobs(Jobs& js) {
  int wgs[MAXJ];
  for (int q = 0; q < js.n; ++q) wgs[q] = js.j[q].wgs;
  return build_xmap(wgs, js.n, &js.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gj_panel(GJJobs jobs, int nt) {
  __shared__ double2 Ps[TB][TB + 1];
  __shared__ double2 Ws[TB][TB + 1];
  int q, w;
  if (!xjob(jobs.x, &q, &w)) return;
  GJJob jb = pick(jobs, q);
  if (w >= jb.wgs) return;
  panel_work<T>(jb, w, nt, Ps, Ws);
}

// Update k (all tiles; negated when last) -- the final panel of a block.  The
// jobs may differ in tile count (the grid covers the largest).
template <typename T>
__global__ __launch_bounds__(256) void k_gj_update(GJJobs jobs) {
  int q, w;
  if (!xjob(jobs.x, &q, &w)) return;
  GJJob jb = pick(jobs, q);
  if (w >= jb.wgs) return;
  update_work<T>(jb, w, size_t(jb.tiles), -1);
}

// Update k outside column k+1, plus the look-ahead panel k+1 (R row tiles per
// look-ahead workgroup).  Within each job the look-ahead workgroups come first,
// so that they are dispatched first: they carry the launch's critical path.
template <typename T, int R>
__global__ __launch_bounds__(256, 2) void k_gj_fused(GJJobs jobs, int nt, size_t tiles) {
  __shared__ double2 Ps[TB][TB + 1];
  __shared__ double2 Ws[TB][TB + 1];
  const int look = jobs.j[0].wgs - jobs.j[0].wgs_upd;   // look-ahead workgroups per job
  int q, w;
  if (!xjob(jobs.x, &q, &w)) return;
  GJJob jb = pick(jobs, q);
  if (w >= jb.wgs) return;
  if (w < look)
    lookahead_work<T, R>(jb, w, nt, Ps, Ws);
  else
    update_work<T>(jb, w - look, tiles, jb.k + 1);
}

// Panels k and k+1 applied to all tiles outside the look-ahead columns, plus
// the pivot work of panels k+2 (and k+3): one workgroup per job, first.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gj2_fused(GJ2Jobs jobs) {
  __shared__ double2 B1[TB][TB + 1];
  __shared__ double2 B2[TB][TB + 1];
  __shared__ double2 B3[TB][TB + 1];
  int q, w;
  if (!xjob(jobs.x, &q, &w)) return;
  const GJ2Job jb = pick2(jobs, q);
  if (w >= jb.wgs) return;
  if (w < jb.wgs - jb.wgs_upd)
    pivot2_work<T>(jb, jb.nt, B1, B2, B3);
  else
    update2_work<T>(jb, w - (jb.wgs - jb.wgs_upd), jb.nt, size_t(jb.tiles));
}

// The row tiles of panels k+2 (and k+3) outside the pivot rows, one per
// workgroup (jb.wgs = nt - nlook of them).
template <typename T>
__global__ __launch_bounds__(256) void k_gj2_rows(GJ2Jobs jobs) {
  __shared__ typename cplx<T>::t lt[2][TB][TB + 1];
  __shared__ typename cplx<T>::t xch[4][4][64];
  int q, w;
  if (!xjob(jobs.x, &q, &w)) return;
  const GJ2Job jb = pick2(jobs, q);
  if (w >= jb.wgs) return;
  const int K3 = jb.k + 2;   // rows K3 (and K4) come from the pivot work
  rows2_work<T>(jb, w < K3 ? w : w + jb.nlook, jb.nt, lt, xch);
}

// The tiles of panel p (slot p mod 4) of each job's L and Q buffers
// transposed in place, one tile per workgroup: the one-panel kernels write
// row-major tiles, the two-panel passes read and write k-major ones.  The grid
// has 2 * maxnt workgroups per job; jobs may differ in nt.
struct PanelTr {
  void* L;
  void* Q;
  int nt;
  int p;
};
struct PanelTrs {
  PanelTr j[MAXJ];
  int n;
  int maxnt;
};

template <typename T>
__global__ __launch_bounds__(256) void k_panel_transpose(PanelTrs js) {
  using T2 = typename cplx<T>::t;
  __shared__ T2 buf[TB][TB + 1];
  const int per = 2 * js.maxnt;
  const int q = blockIdx.x / per;
  int r = blockIdx.x - q * per;
  const int which = r / js.maxnt;
  const int I = r - which * js.maxnt;
  const int nt = RCP_SEL16(js, q, nt);
  if (I >= nt) return;
  const int p = RCP_SEL16(js, q, p);
  void* const base = which ? RCP_SEL16(js, q, Q) : RCP_SEL16(js, q, L);
  T2* const t = slot_ptr<T2>(base, p, nt) + size_t(I) * TB * TB;
  for (int e = threadIdx.x; e < TB * TB; e += 256) buf[e / TB][e % TB] = t[e];
  __syncthreads();
  for (int e = threadIdx.x; e < TB * TB; e += 256) t[e] = buf[e % TB][e / TB];
}

// dst = D - C1 src1 C1 - C2 src2 C2 on packed tiles (src may be null), with
// identity in the padding.  D is the tridiagonal diagonal block of column i.
struct SchurJob {
  void* dst;
  const void* src1;
  const void* src2;
  const double2* dco;   // diagonal of D (ny)
  const double2* eco;   // coupling j -> j+1 (ny)
  const double2* c1;    // x-couplings (ny) or null
  const double2* c2;
  int ny;               // block size of this job's geometry
  int tiles;            // its packed tiles per block
};
struct SchurJobs {
  SchurJob j[MAXJ];
  int n;
  int maxtiles;   // k_schur: workgroups per job
};

template <typename T>
__device__ __forceinline__ SchurJob schur_job_of(const SchurJobs& jobs, int ji) {
  SchurJob jb;
  jb.dst = RCP_SEL16(jobs, ji, dst);
  jb.src1 = RCP_SEL16(jobs, ji, src1);
  jb.src2 = RCP_SEL16(jobs, ji, src2);
  jb.dco = RCP_SEL16(jobs, ji, dco);
  jb.eco = RCP_SEL16(jobs, ji, eco);
  jb.c1 = RCP_SEL16(jobs, ji, c1);
  jb.c2 = RCP_SEL16(jobs, ji, c2);
  jb.ny = RCP_SEL16(jobs, ji, ny);
  jb.tiles = RCP_SEL16(jobs, ji, tiles);
  return jb;
}

// Packed tiles t0 .. t0 + NTL - 1 (those below tiles) of dst, by the 256
// threads of a workgroup: each thread forms its elements in registers before
// it stores any, so that all of its loads are in flight together (a store
// might alias a later load otherwise).
template <typename T, int NTL>
__device__ __forceinline__ void schur_tiles(const SchurJob& jb, size_t t0, size_t tiles) {
  using T2 = typename cplx<T>::t;
  const int ny = jb.ny;
  constexpr int EPT = TB * TB / 256;
  double2 v[NTL][EPT];
#pragma unroll
  for (int k = 0; k < NTL; ++k) {
    const size_t t = t0 + k;
    if (t >= tiles) break;
    int I, J;
    tile_coords(static_cast<int>(t), &I, &J);
    const T2* s1 = jb.src1 ? static_cast<const T2*>(jb.src1) + t * TB * TB : nullptr;
    const T2* s2 = jb.src2 ? static_cast<const T2*>(jb.src2) + t * TB * TB : nullptr;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int a = I * TB + e / TB, b = J * TB + e % TB;
      double2 x = make_double2(0.0, 0.0);
      if (a == b) {
        x = (a < ny) ? jb.dco[a] : make_double2(1.0, 0.0);
      } else if (a == b + 1 && a < ny) {
        x = jb.eco[b];
      } else if (b == a + 1 && b < ny) {
        x = jb.eco[a];
      }
      if (a < ny && b < ny) {
        if (s1) x = csub(x, cmul(cmul(jb.c1[a], jb.c1[b]), to_c128(s1[e])));
        if (s2) x = csub(x, cmul(cmul(jb.c2[a], jb.c2[b]), to_c128(s2[e])));
      }
      v[k][u] = x;
    }
  }
#pragma unroll
  for (int k = 0; k < NTL; ++k) {
    const size_t t = t0 + k;
    if (t >= tiles) break;
    T2* dst = static_cast<T2*>(jb.dst) + t * TB * TB;
#pragma unroll
    for (int u = 0; u < EPT; ++u) dst[threadIdx.x + 256 * u] = from_c128<T2>(v[k][u]);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_schur(SchurJobs jobs) {
  const size_t t = blockIdx.x % jobs.maxtiles;
  const int ji = static_cast<int>(blockIdx.x / jobs.maxtiles);
  const SchurJob jb = schur_job_of<T>(jobs, ji);
  schur_tiles<T, 1>(jb, t, size_t(jb.tiles));
}

// The Schur complements that start the next blocks of a two-panel sweep, and
// the pivot work of their panels 0 and 1 beside them (the pass K = -2): per
// chain, workgroup 0 forms the three tiles of that pivot area, (0, 0), (1, 0)
// and (1, 1), and inverts the pivots, while the other workgroups form the
// remaining tiles, OPEN_TILES each.  The pivot inversions, latency-bound, run while
// the rest of the block streams through HBM.  sj.j[q] and gj.j[q] describe
// the same block; gj.j[q].wgs = 1 + ceil((tiles - 3) / OPEN_TILES).
constexpr int OPEN_TILES = 2;
template <typename T>
__device__ __forceinline__ void open_work(const GJ2Jobs& gj, const SchurJobs& sj, int q, int w,
                                          double2 (*B1)[TB + 1], double2 (*B2)[TB + 1],
                                          double2 (*B3)[TB + 1]) {
  const SchurJob sjob = schur_job_of<T>(sj, q);
  if (w == 0) {
    schur_tiles<T, 3>(sjob, 0, 3);
    __syncthreads();   // the tiles are read back by every wave of this workgroup
    const GJ2Job jb = pick2(gj, q);
    pivot2_work<T>(jb, jb.nt, B1, B2, B3);
  } else {
    schur_tiles<T, OPEN_TILES>(sjob, 3 + size_t(w - 1) * OPEN_TILES, size_t(sjob.tiles));
  }
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_gj2_open(GJ2Jobs gj, SchurJobs sj) {
  __shared__ double2 B1[TB][TB + 1];
  __shared__ double2 B2[TB][TB + 1];
  __shared__ double2 B3[TB][TB + 1];
  int q, w;
  if (!xjob(gj.x, &q, &w)) return;
  if (w >= RCP_SEL16(gj, q, wgs)) return;
  open_work<T>(gj, sj, q, w, B1, B2, B3);
}

// One step of every chain of a mixed launch (chains of different geometries,
// each at its own place in its own sweep): a job either opens its block
// (jb.open: the Schur complement beside the pivot work of panels 0 and 1, as
// k_gj2_open) or applies its next pair of panels with the pivot work of the
// pair after (as k_gj2_fused).
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gj2_step(GJ2Jobs gj, SchurJobs sj) {
  __shared__ double2 B1[TB][TB + 1];
  __shared__ double2 B2[TB][TB + 1];
  __shared__ double2 B3[TB][TB + 1];
  int q, w;
  if (!xjob(gj.x, &q, &w)) return;
  const GJ2Job jb = pick2(gj, q);
  if (w >= jb.wgs) return;
  if (jb.open) {
    open_work<T>(gj, sj, q, w, B1, B2, B3);
  } else if (w < jb.wgs - jb.wgs_upd) {
    pivot2_work<T>(jb, jb.nt, B1, B2, B3);
  } else {
    update2_work<T>(jb, w - (jb.wgs - jb.wgs_upd), jb.nt, size_t(jb.tiles));
  }
}

// Factor B same-shape geometries in lockstep: every launch carries the chains
// of all of them (two per geometry).
template <typename T>
int run_factor(rcp_factors* const* fs, int B, hipStream_t s, bool pairs) {
  const rcp_factors* f0 = fs[0];
  const int N = f0->nx, ny = f0->ny, nt = f0->nt, m = f0->m;
  const size_t tiles = f0->tiles;
  const int lenL = m, lenR = N - 1 - m;
  auto D = [&](int g, int i) { return fs[g]->dco + size_t(i) * ny; };
  auto E = [&](int g, int i) { return fs[g]->eco + size_t(i) * ny; };
  auto C = [&](int g, int i) { return fs[g]->cco + size_t(i) * ny; };

  struct Chain {
    int g, c, block;
  };
  // chains whose block-opening pivot work (pass K = -2) already ran beside
  // their Schur complements
  Chain opened[MAXJ];
  int nopened = 0;
  // Schur complements js.j[q] = the next block of chain ch[q]; with two-panel
  // sweeps the opening pivot work of those blocks rides in the same launch
  auto schur = [&](SchurJobs js, const Chain* ch) -> int {
    nopened = 0;
    if (js.n == 0) return RCP_OK;
    int nsrc = 0;
    for (int q = 0; q < js.n; ++q) nsrc += 1 + (js.j[q].src1 != nullptr) + (js.j[q].src2 != nullptr);
    const double sbytes = double(nsrc) * tiles * TB * TB * f0->elem_bytes;
    for (int q = 0; q < js.n; ++q) {
      js.j[q].ny = ny;
      js.j[q].tiles = static_cast<int>(tiles);
    }
    js.maxtiles = static_cast<int>(tiles);
    if (!pairs || nt < 2) {
      RCP_HIP(klaunch(K_SCHUR, sbytes, k_schur<T>, dim3(static_cast<int>(tiles * js.n)), dim3(256), s,
                      js));
      return RCP_OK;
    }
    GJ2Jobs gj{};
    const int per = 1 + ceil_div(static_cast<int>(tiles) - 3, OPEN_TILES);
    for (int q = 0; q < js.n; ++q) {
      const rcp_factors* f = fs[ch[q].g];
      if (block_ptr(f, ch[q].block) != js.j[q].dst) return fail(RCP_EINVAL, "internal: opener job order");
      GJ2Job b{};
      b.k = -2;
      b.nlook = 2;
      b.wgs = per;
      b.X = js.j[q].dst;
      b.Lb = f->wsL[4 * ch[q].c];
      b.Qb = f->wsQ[4 * ch[q].c];
      b.Pb = f->wsP[4 * ch[q].c];
      b.health = f->health + size_t(ch[q].block) * nt;
      b.nt = nt;
      b.tiles = static_cast<int>(tiles);
      b.open = 1;
      gj.j[gj.n++] = b;
      opened[q] = ch[q];
    }
    const int grid = map_jobs(gj);
    RCP_HIP(klaunch(K_SCHUR, sbytes, k_gj2_open<T>, dim3(grid), dim3(256), s, gj, js));
    nopened = js.n;
    return RCP_OK;
  };
  const int upd_wgs = static_cast<int>((tiles + 3) / 4);
  const int pan_wgs = ceil_div(nt, 4);   // first panel: four row tiles per workgroup
  const double cmac = 8.0 * TB * TB * TB;   // flops of one TB^3 complex product
  // Sweep the given blocks (chain c of geometry g) through all panels; the
  // panel buffers of chain c alternate between halves 2c and 2c+1.
  auto sweep = [&](int nch, const Chain* ch) -> int {
    bool open_done = nopened == nch;
    for (int q = 0; q < nch && open_done; ++q)
      open_done = opened[q].g == ch[q].g && opened[q].c == ch[q].c && opened[q].block == ch[q].block;
    nopened = 0;
    // single-panel job k: panel k in slot k mod 4, panel k+1 in the next slot
    auto job = [&](const Chain& x, int k) {
      const rcp_factors* f = fs[x.g];
      GJJob b{};
      b.k = k;
      b.X = block_ptr(f, x.block);
      const int cur = 4 * x.c + (k & 3), nxt = 4 * x.c + ((k + 1) & 3);
      b.L = f->wsL[cur];
      b.Q = f->wsQ[cur];
      b.P = f->wsP[cur];
      b.Ln = f->wsL[nxt];
      b.Qn = f->wsQ[nxt];
      b.Pn = f->wsP[nxt];
      b.health = f->health + size_t(x.block) * nt + (k + 1 < nt ? k + 1 : k);
      b.tiles = static_cast<int>(tiles);
      return b;
    };
    if (!pairs || nt < 2) {   // panel 0 (the "next" slot of k = -1, i.e. slot 0)
      GJJobs js{};
      for (int q = 0; q < nch; ++q) {
        GJJob b = job(ch[q], -1);
        b.k = 0;
        b.health = fs[ch[q].g]->health + size_t(ch[q].block) * nt;
        b.wgs = pan_wgs;
        js.j[js.n++] = b;
      }
      const int grid = map_jobs(js);
      RCP_HIP(klaunch(K_GJ_PANEL, nch * cmac * nt, k_gj_panel<T>, dim3(grid), dim3(256), s, js, nt));
    }
    if (!pairs) {
      // one panel per launch: update k of every tile outside column k+1 fused
      // with the look-ahead of panel k+1; two look-ahead row tiles per
      // workgroup when sixteen chains share the GPU, otherwise one
      const int R = nch >= 16 ? 2 : 1;
      const int look_wgs = ceil_div(nt, R);
      for (int k = 0; k + 1 < nt; ++k) {
        GJJobs js{};
        for (int q = 0; q < nch; ++q) {
          GJJob b = job(ch[q], k);
          b.wgs_upd = upd_wgs;
          b.wgs = upd_wgs + look_wgs;
          js.j[js.n++] = b;
        }
        const int grid = map_jobs(js);
        const double w = nch * cmac * double(tiles);
        if (R == 1)
          RCP_HIP(klaunch(K_GJ_UPDATE, w, k_gj_fused<T, 1>, dim3(grid), dim3(256), s, js, nt, tiles));
        else
          RCP_HIP(klaunch(K_GJ_UPDATE, w, k_gj_fused<T, 2>, dim3(grid), dim3(256), s, js, nt, tiles));
      }
      GJJobs js{};   // final update, negated
      for (int q = 0; q < nch; ++q) {
        GJJob b = job(ch[q], nt - 1);
        b.last = 1;
        b.wgs = upd_wgs;
        b.wgs_upd = upd_wgs;
        js.j[js.n++] = b;
      }
      const int grid = map_jobs(js);
      RCP_HIP(klaunch(K_GJ_LAST, nch * cmac * double(tiles - nt), k_gj_update<T>, dim3(grid), dim3(256),
                      s, js));
      return RCP_OK;
    }
    PanelTrs tr{};
    for (int q = 0; q < nch; ++q)
      tr.j[tr.n++] = PanelTr{fs[ch[q].g]->wsL[4 * ch[q].c], fs[ch[q].g]->wsQ[4 * ch[q].c], nt, nt - 1};
    tr.maxnt = nt;
    // pairs (K, K+1); the look-ahead forms the next pair (or the last panel).
    // K = -2 opens the block: no panels to apply, only the pivot work and row
    // tiles of panels 0 and 1 on the untouched tiles
    for (int K = -2; K + 1 < nt; K += 2) {
      const int nlook = nt - (K + 2) >= 2 ? 2 : nt - (K + 2);
      const int last = nlook == 0 ? 1 : 0;
      const int look_wgs = nlook > 0 ? 1 : 0;   // the pivot work of the next pair
      const int upd = K < 0 ? 0 : upd_wgs;
      GJ2Jobs js{};
      for (int q = 0; q < nch; ++q) {
        const rcp_factors* f = fs[ch[q].g];
        GJ2Job b{};
        b.k = K;
        b.nlook = nlook;
        b.last = last;
        b.wgs_upd = upd;
        b.wgs = upd + look_wgs;
        b.X = block_ptr(f, ch[q].block);
        b.Lb = f->wsL[4 * ch[q].c];
        b.Qb = f->wsQ[4 * ch[q].c];
        b.Pb = f->wsP[4 * ch[q].c];
        b.health = f->health + size_t(ch[q].block) * nt;
        b.nt = nt;
        b.tiles = static_cast<int>(tiles);
        js.j[js.n++] = b;
      }
      if (K >= 0 || !open_done) {
        const int grid = map_jobs(js);
        RCP_HIP(klaunch(K < 0 ? K_GJ_PANEL : (last ? K_GJ_LAST : K_GJ_UPDATE),
                        K < 0 ? nch * 6.0 * cmac : nch * 2.0 * cmac * double(tiles), k_gj2_fused<T>,
                        dim3(grid), dim3(256), s, js));
      }
      // row tiles of the next pair's panels; the pivot rows come from the
      // pivot work, and with two tiles per edge nothing else is left
      const int rows = nt - nlook;
      if (nlook > 0 && rows > 0) {
        for (int q = 0; q < js.n; ++q) js.j[q].wgs = rows;
        const int grid = map_jobs(js);
        RCP_HIP(klaunch(K_GJ_PANEL, nch * cmac * nlook * rows, k_gj2_rows<T>, dim3(grid), dim3(256), s,
                        js));
      }
    }
    if (nt & 1) {   // odd panel count: the last panel alone, negated
      if (nt >= 3) {   // formed by the last pass: back to row-major
        k_panel_transpose<T><<<nch * 2 * nt, 256, 0, s>>>(tr);
        RCP_HIP(hipGetLastError());
      }
      GJJobs js{};
      for (int q = 0; q < nch; ++q) {
        GJJob b = job(ch[q], nt - 1);
        b.last = 1;
        b.wgs = upd_wgs;
        b.wgs_upd = upd_wgs;
        js.j[js.n++] = b;
      }
      const int grid = map_jobs(js);
      RCP_HIP(klaunch(K_GJ_LAST, nch * cmac * double(tiles - nt), k_gj_update<T>, dim3(grid), dim3(256),
                      s, js));
    }
    return RCP_OK;
  };

  {   // chain heads
    SchurJobs js{};
    Chain nxt[MAXJ];
    for (int g = 0; g < B; ++g) {
      if (lenL > 0) {
        nxt[js.n] = Chain{g, 0, 0};
        js.j[js.n++] = SchurJob{block_ptr(fs[g], 0), nullptr, nullptr, D(g, 0), E(g, 0), nullptr, nullptr,
                                ny, static_cast<int>(tiles)};
      }
      if (lenR > 0) {
        nxt[js.n] = Chain{g, 1, N - 1};
        js.j[js.n++] = SchurJob{block_ptr(fs[g], N - 1), nullptr, nullptr, D(g, N - 1), E(g, N - 1),
                                nullptr, nullptr, ny, static_cast<int>(tiles)};
      }
    }
    int rc = schur(js, nxt);
    if (rc) return rc;
  }
  const int steps = lenL > lenR ? lenL : lenR;
  for (int st = 0; st < steps; ++st) {
    Chain ch[MAXJ];
    int nch = 0;
    const int bL = st < lenL ? st : -1, bR = st < lenR ? N - 1 - st : -1;
    for (int g = 0; g < B; ++g) {
      if (bL >= 0) ch[nch++] = Chain{g, 0, bL};
      if (bR >= 0) ch[nch++] = Chain{g, 1, bR};
    }
    int rc = sweep(nch, ch);
    if (rc) return rc;
    SchurJobs js{};
    Chain nxt[MAXJ];
    for (int g = 0; g < B; ++g) {
      if (bL >= 0 && bL + 1 < m) {
        nxt[js.n] = Chain{g, 0, bL + 1};
        js.j[js.n++] = SchurJob{block_ptr(fs[g], bL + 1), block_ptr(fs[g], bL), nullptr,
                                D(g, bL + 1), E(g, bL + 1), C(g, bL), nullptr, ny,
                                static_cast<int>(tiles)};
      }
      if (bR >= 0 && bR - 1 > m) {
        nxt[js.n] = Chain{g, 1, bR - 1};
        js.j[js.n++] = SchurJob{block_ptr(fs[g], bR - 1), block_ptr(fs[g], bR), nullptr,
                                D(g, bR - 1), E(g, bR - 1), C(g, bR - 1), nullptr, ny,
                                static_cast<int>(tiles)};
      }
    }
    rc = schur(js, nxt);
    if (rc) return rc;
  }
  {   // middle blocks
    SchurJobs js{};
    Chain ch[MAXJ];
    int nch = 0;
    for (int g = 0; g < B; ++g) {
      SchurJob z{block_ptr(fs[g], m), nullptr, nullptr, D(g, m), E(g, m), nullptr, nullptr, ny,
                 static_cast<int>(tiles)};
      if (m - 1 >= 0) {
        z.src1 = block_ptr(fs[g], m - 1);
        z.c1 = C(g, m - 1);
      }
      if (m + 1 < N) {
        z.src2 = block_ptr(fs[g], m + 1);
        z.c2 = C(g, m);
      }
      js.j[js.n++] = z;
      ch[nch++] = Chain{g, 0, m};
    }
    int rc = schur(js, ch);
    if (rc) return rc;
    rc = sweep(nch, ch);
    if (rc) return rc;
  }
  return RCP_OK;
}

// The pivot check of a finished factorisation on the device: status = 0 when
// every panel's smallest pivot modulus is finite and above tiny, else 1 + the
// first panel (block-major) that is not.  One workgroup per factor set.
struct PivotCheck {
  const double* health;
  int count;
  double tiny;
  int32_t* status;
};
struct PivotChecks {
  PivotCheck j[MAX_BATCH];
  int n;
};
__global__ __launch_bounds__(256) void k_pivot_check(PivotChecks pc) {
  __shared__ int first[256];
  PivotCheck c = pc.j[0];
  for (int q = 1; q < MAX_BATCH; ++q)
    if (q == static_cast<int>(blockIdx.x)) c = pc.j[q];
  int f = 0x7fffffff;
  for (int q = threadIdx.x; q < c.count; q += 256) {
    const double h = c.health[q];
    if (!(h > c.tiny) || !isfinite(h)) {
      f = q;
      break;
    }
  }
  first[threadIdx.x] = f;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) first[threadIdx.x] = min(first[threadIdx.x], first[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *c.status = first[0] == 0x7fffffff ? 0 : first[0] + 1;
}

// ---------------------------------------------------------------------------
// Factorisation engine: geometries of any size share launches.  Each chain
// (left, right, then the middle block) advances one step per round: a round
// is one k_gj2_step launch (every chain opens its next block or applies its
// next pair of panels), the row tiles of the panels it formed, and for chains
// that end a block with an odd panel the transpose and final update.  A new
// geometry joins at the next round; a finished one leaves.  Every chain does
// exactly what the batched two-panel sweep does to it, so the factors of a
// geometry are the same bits whatever else shares the launches.
struct EChain {
  int g;       // geometry slot
  int c;       // panel buffers of chain c (0: left and middle, 1: right)
  int dir;     // +1 left, -1 right, 0 middle
  int block;
  int K;       // next pass; -2 opens the block
};

struct EGeom {
  rcp_factors* f = nullptr;
  int chains_left = 0;   // side chains still running (0..2); then the middle block
  bool middle = false;
};

constexpr int kOpenTilesPerWg = OPEN_TILES;

template <typename T>
int engine_round(std::vector<EGeom>& geoms, std::vector<EChain>& chains, hipStream_t s,
                 std::vector<int>* finished) {
  const int nch = static_cast<int>(chains.size());
  if (nch == 0) return RCP_OK;
  if (nch > MAXJ) return fail(RCP_EINVAL, "internal: too many chains in a round");
  const double cmac = 8.0 * TB * TB * TB;
  GJ2Jobs gj{};
  SchurJobs sj{};
  int nlook_of[MAXJ];
  double work = 0.0;
  // 3D geometries open their blocks here: the Schur complement with the sparse
  // slice couplings, then a step that only does the pivot work of panels 0, 1
  Schur3dJob s3[MAXJ];
  int n3 = 0;
  for (int q = 0; q < nch; ++q) {
    const EChain& x = chains[q];
    const rcp_factors* f = geoms[x.g].f;
    if (!f->dim3 || x.K != -2) continue;
    const int n = f->ny, N = f->nx;
    Schur3dJob z{};
    z.dst = block_ptr(f, x.block);
    z.d_idx = f->d_idx + size_t(x.block) * n * K3D_DW;
    z.d_val = f->d_val + size_t(x.block) * n * K3D_DW;
    z.n = n;
    z.tiles = static_cast<int>(f->tiles);
    if ((x.dir > 0 || x.dir == 0) && x.block > 0) {   // from block - 1: column lists of boundary block - 1
      z.src1 = block_ptr(f, x.block - 1);
      z.c1_idx = f->cl_idx + size_t(x.block - 1) * n * K3D_CW;
      z.c1_val = f->cl_val + size_t(x.block - 1) * n * K3D_CW;
    }
    if ((x.dir < 0 || x.dir == 0) && x.block < N - 1) {   // from block + 1: row lists of boundary block
      z.src2 = block_ptr(f, x.block + 1);
      z.c2_idx = f->cr_idx + size_t(x.block) * n * K3D_CW;
      z.c2_val = f->cr_val + size_t(x.block) * n * K3D_CW;
    }
    s3[n3++] = z;
  }
  if (n3 > 0) {
    int rc = schur3d(s3, n3, s);
    if (rc) return rc;
  }
  for (int q = 0; q < nch; ++q) {
    const EChain& x = chains[q];
    const rcp_factors* f = geoms[x.g].f;
    const int nt = f->nt, N = f->nx, ny = f->ny;
    const int tiles = static_cast<int>(f->tiles);
    GJ2Job b{};
    b.k = x.K;
    b.nt = nt;
    b.tiles = tiles;
    b.X = block_ptr(f, x.block);
    b.Lb = f->wsL[4 * x.c];
    b.Qb = f->wsQ[4 * x.c];
    b.Pb = f->wsP[4 * x.c];
    b.health = f->health + size_t(x.block) * nt;
    SchurJob z{};
    z.dst = b.X;
    z.ny = ny;
    z.tiles = tiles;
    if (x.K == -2 && f->dim3) {   // Schur complement formed above: pivot work only
      b.nlook = 2;
      b.wgs_upd = 0;
      b.wgs = 1;
      work += 6.0 * cmac;
    } else if (x.K == -2) {   // open: Schur complement of this block + pivot work of panels 0, 1
      b.open = 1;
      b.nlook = 2;
      b.wgs = 1 + ceil_div(tiles - 3, kOpenTilesPerWg);
      z.dco = f->dco + size_t(x.block) * ny;
      z.eco = f->eco + size_t(x.block) * ny;
      if (x.dir > 0 && x.block > 0) {
        z.src1 = block_ptr(f, x.block - 1);
        z.c1 = f->cco + size_t(x.block - 1) * ny;
      } else if (x.dir < 0 && x.block < N - 1) {
        z.src1 = block_ptr(f, x.block + 1);
        z.c1 = f->cco + size_t(x.block) * ny;
      } else if (x.dir == 0) {
        if (x.block - 1 >= 0) {
          z.src1 = block_ptr(f, x.block - 1);
          z.c1 = f->cco + size_t(x.block - 1) * ny;
        }
        if (x.block + 1 < N) {
          z.src2 = block_ptr(f, x.block + 1);
          z.c2 = f->cco + size_t(x.block) * ny;
        }
      }
      work += 6.0 * cmac;
    } else {
      b.nlook = nt - (x.K + 2) >= 2 ? 2 : nt - (x.K + 2);
      b.last = b.nlook == 0 ? 1 : 0;
      b.wgs_upd = ceil_div(tiles, 4);
      b.wgs = b.wgs_upd + (b.nlook > 0 ? 1 : 0);
      work += 2.0 * cmac * tiles;
    }
    nlook_of[q] = b.nlook;
    gj.j[gj.n++] = b;
    sj.j[sj.n++] = z;
  }
  {
    const int grid = map_jobs(gj);
    RCP_HIP(klaunch(K_ENGINE, work, k_gj2_step<T>, dim3(grid), dim3(256), s, gj, sj));
  }
  // row tiles of the panels the step formed (outside its pivot rows)
  {
    GJ2Jobs rj{};
    double rw = 0.0;
    for (int q = 0; q < nch; ++q) {
      const int rows = gj.j[q].nt - nlook_of[q];
      if (nlook_of[q] > 0 && rows > 0) {
        GJ2Job b = gj.j[q];
        b.open = 0;
        b.wgs = rows;
        rj.j[rj.n++] = b;
        rw += cmac * nlook_of[q] * rows;
      }
    }
    if (rj.n > 0) {
      const int grid = map_jobs(rj);
      RCP_HIP(klaunch(K_ENGINE, rw, k_gj2_rows<T>, dim3(grid), dim3(256), s, rj));
    }
  }
  // odd panel counts: the last panel alone, negated, after its rows
  {
    PanelTrs tr{};
    GJJobs uj{};
    double uw = 0.0;
    for (int q = 0; q < nch; ++q) {
      if (chains[q].K == -2 || nlook_of[q] != 1) continue;
      const EChain& x = chains[q];
      const rcp_factors* f = geoms[x.g].f;
      const int nt = f->nt, k = nt - 1;
      tr.j[tr.n++] = PanelTr{f->wsL[4 * x.c], f->wsQ[4 * x.c], nt, k};
      if (nt > tr.maxnt) tr.maxnt = nt;
      GJJob b{};
      b.k = k;
      b.last = 1;
      b.X = block_ptr(f, x.block);
      const int cur = 4 * x.c + (k & 3), nxt = 4 * x.c + ((k + 1) & 3);
      b.L = f->wsL[cur];
      b.Q = f->wsQ[cur];
      b.P = f->wsP[cur];
      b.Ln = f->wsL[nxt];
      b.Qn = f->wsQ[nxt];
      b.Pn = f->wsP[nxt];
      b.health = f->health + size_t(x.block) * nt + k;
      b.tiles = static_cast<int>(f->tiles);
      b.wgs = ceil_div(b.tiles, 4);
      b.wgs_upd = b.wgs;
      uj.j[uj.n++] = b;
      uw += cmac * double(f->tiles - nt);
    }
    if (uj.n > 0) {
      k_panel_transpose<T><<<uj.n * 2 * tr.maxnt, 256, 0, s>>>(tr);
      RCP_HIP(hipGetLastError());
      const int grid = map_jobs(uj);
      RCP_HIP(klaunch(K_ENGINE, uw, k_gj_update<T>, dim3(grid), dim3(256), s, uj));
    }
  }
  // advance
  std::vector<EChain> next;
  next.reserve(chains.size() + 2);
  for (int q = 0; q < nch; ++q) {
    EChain x = chains[q];
    const GJ2Job& b = gj.j[q];
    const bool opening = x.K == -2;
    const bool block_done = !opening && (b.last || nlook_of[q] == 1);
    if (!block_done) {
      x.K = opening ? 0 : x.K + 2;
      next.push_back(x);
      continue;
    }
    EGeom& G = geoms[x.g];
    const rcp_factors* f = G.f;
    if (x.dir == 0) {   // middle block done: the geometry is factored
      finished->push_back(x.g);
      continue;
    }
    const int nb = x.block + x.dir;
    const bool more = x.dir > 0 ? nb < f->m : nb > f->m;
    if (more) {
      x.block = nb;
      x.K = -2;
      next.push_back(x);
      continue;
    }
    if (--G.chains_left == 0) {
      G.middle = true;
      next.push_back(EChain{x.g, 0, 0, f->m, -2});
    }
  }
  chains.swap(next);
  return RCP_OK;
}

}  // namespace

struct rcp_engine {
  int precision = 0;
  std::vector<EGeom> geoms;     // slots; f == nullptr when free
  std::vector<EChain> chains;
  int active = 0;
};

namespace rcp {

int engine_create(int precision, rcp_engine** out) {
  rcp_engine* e = new (std::nothrow) rcp_engine();
  if (!e) return fail(RCP_ENOMEM, "host allocation failed");
  e->precision = precision;
  e->geoms.resize(MAX_BATCH);
  *out = e;
  return RCP_OK;
}

void engine_destroy(rcp_engine* e) { delete e; }

int engine_active(const rcp_engine* e) { return e->active; }

int engine_precision(const rcp_engine* e) { return e->precision; }

int engine_add(rcp_engine* e, rcp_factors* f) {
  if (f->precision != e->precision) return fail(RCP_EINVAL, "precision differs from the engine's");
  if (f->nt < 2) return fail(RCP_EINVAL, "the engine needs blocks of more than 32 rows");
  int slot = -1;
  for (int g = 0; g < MAX_BATCH; ++g)
    if (!e->geoms[g].f) {
      slot = g;
      break;
    }
  if (slot < 0) return fail(RCP_EINVAL, "engine full: 8 geometries in flight");
  EGeom& G = e->geoms[slot];
  G.f = f;
  G.middle = false;
  G.chains_left = 0;
  const int N = f->nx, m = f->m;
  if (m > 0) {   // left chain: blocks 0 .. m-1
    e->chains.push_back(EChain{slot, 0, +1, 0, -2});
    ++G.chains_left;
  }
  if (N - 1 - m > 0) {   // right chain: blocks N-1 .. m+1
    e->chains.push_back(EChain{slot, 1, -1, N - 1, -2});
    ++G.chains_left;
  }
  if (G.chains_left == 0) {
    G.middle = true;
    e->chains.push_back(EChain{slot, 0, 0, m, -2});
  }
  ++e->active;
  return RCP_OK;
}

// Health of a finished geometry: the device pivot check, then one wait.
static int check_health(rcp_factors* f, hipStream_t s) {
  rcp_factors* one[1] = {f};
  int rc = enqueue_pivot_check(one, 1, s);
  return rc ? rc : read_pivot_check(f, s, "");
}

int engine_step(rcp_engine* e, int rounds, hipStream_t s, rcp_factors** done, int* status,
                int cap, int* ndone) {
  *ndone = 0;
  std::vector<int> fin;
  for (int r = 0; r < rounds && !e->chains.empty() && fin.empty(); ++r) {
    int rc = e->precision == RCP_FP64 ? engine_round<double>(e->geoms, e->chains, s, &fin)
                                      : engine_round<float>(e->geoms, e->chains, s, &fin);
    if (rc) return rc;
  }
  for (int g : fin) {
    rcp_factors* f = e->geoms[g].f;
    e->geoms[g].f = nullptr;
    --e->active;
    if (*ndone < cap) {
      done[*ndone] = f;
      status[*ndone] = check_health(f, s);
      ++*ndone;
    }
  }
  return RCP_OK;
}

int factor_blocks_async(rcp_factors* const* fs, int B, hipStream_t s) {
  if (B < 1 || B > MAXJ / 2) return fail(RCP_EINVAL, "batch of 1 to 8 geometries");
  const int prec = fs[0]->precision;
  // Batches take two panels per pass (each tile read and written once per two
  // panels; the pivot work of the next pair rides in the pass); one geometry
  // alone is bound by the chain of pivot inversions, which one panel per
  // launch keeps shortest.
  const bool pairs = B >= 2;
  int rc = (prec == RCP_FP64) ? run_factor<double>(fs, B, s, pairs) : run_factor<float>(fs, B, s, pairs);
  if (rc) return rc;
  return enqueue_pivot_check(fs, B, s);
}

int factor_blocks(rcp_factors* const* fs, int B, hipStream_t s) {
  int rc = factor_blocks_async(fs, B, s);
  for (int g = 0; g < B && !rc; ++g)
    rc = read_pivot_check(fs[g], s, B > 1 ? "geometry " + std::to_string(g) + ": " : "");
  return rc;
}

int enqueue_pivot_check(rcp_factors* const* fs, int B, hipStream_t s) {
  if (B < 1 || B > MAX_BATCH) return fail(RCP_EINVAL, "internal: pivot check of 1 to 8 sets");
  PivotChecks pc{};
  for (int g = 0; g < B; ++g) {
    const rcp_factors* f = fs[g];
    // diagonal entries are O(4/h^2); a pivot below 1e-13 of that scale is
    // treated as singular
    pc.j[pc.n++] = PivotCheck{f->health, f->nx * f->nt, 1e-13 * 4.0 / (f->h * f->h), f->status};
  }
  k_pivot_check<<<pc.n, 256, 0, s>>>(pc);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int read_pivot_check(const rcp_factors* f, hipStream_t s, const std::string& prefix) {
  int32_t st = 0;
  RCP_HIP(hipMemcpyAsync(&st, f->status, sizeof(st), hipMemcpyDeviceToHost, s));
  RCP_HIP(hipStreamSynchronize(s));
  if (st == 0) return RCP_OK;
  const int q = st - 1;
  double h = 0.0;
  RCP_HIP(hipMemcpy(&h, f->health + q, sizeof(h), hipMemcpyDeviceToHost));
  return fail(RCP_ESINGULAR, prefix + "pivot block " + std::to_string(q % f->nt) + " of column block " +
                                 std::to_string(q / f->nt) + " has pivot modulus " + std::to_string(h));
}

}  // namespace rcp

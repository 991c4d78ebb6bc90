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
// Look-ahead: launch k applies update k to every tile outside tile column
// k+1, while a few workgroups compute the update-k values of column k+1
// directly in the layout the next panel needs, invert the next pivot block
// and form Q for panel k+1 into the other half of double-buffered panel
// buffers.  Column k+1 values never go back to the factor tiles: update k+1
// overwrites that column anyway.  One launch per panel, no dependencies
// between the workgroups of a launch.
//
// The TB x TB pivot blocks are inverted without pivoting, in FP64 for both
// storage precisions, and the smallest pivot modulus of every panel is
// recorded for the health check.
#include <cmath>
#include <vector>

#include "rcp_internal.h"

namespace {
using namespace rcp;

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
};
constexpr int MAXJ = 2 * MAX_BATCH;   // chains per launch: two per geometry
struct GJJobs {
  GJJob j[MAXJ];
  int n;
};

// Job of this workgroup: every job of a launch has the same workgroup count;
// fields are selected one at a time so that the table stays in kernel-argument
// registers.
__device__ __forceinline__ GJJob pick(const GJJobs& js, int* wg) {
  const int per = js.j[0].wgs;
  const int q = *wg / per;
  *wg -= q * per;
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

// Gauss-Jordan inversion of the TB x TB block in Ps (FP64), result back in Ps,
// eliminating two columns per step with the 2 x 2 diagonal block B of rows and
// columns p, p+1 as pivot (inverted in closed form; no row exchanges):
//   pivot rows      R <- B^{-1} R,       their pivot columns <- B^{-1}
//   other rows r    m_r <- m_r - F_r B^{-1} R,   their pivot columns <- -F_r B^{-1}
// with F_r = (m_rp, m_r,p+1).  256 threads; thread owns row r, columns
// c0..c0+3 in registers; pivot rows/columns are exchanged through
// double-buffered LDS, one barrier per step.  Returns min |det B|^(1/2).
__device__ double invert_pivot_block(double2 (*Ps)[TB + 1], double2 (*xr)[TB],
                                     double2 (*xc)[TB]) {
  const int tid = threadIdx.x;
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  double2 m[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) m[c] = Ps[r][c0 + c];
  double mindet2 = INFINITY;
  for (int p = 0; p < TB; p += 2) {
    const int b = (p >> 1) & 1;
    if (r == p) {
#pragma unroll
      for (int c = 0; c < 4; ++c) xr[2 * b][c0 + c] = m[c];
    }
    if (r == p + 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) xr[2 * b + 1][c0 + c] = m[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c0 + c == p) xc[2 * b][r] = m[c];
      if (c0 + c == p + 1) xc[2 * b + 1][r] = m[c];
    }
    __syncthreads();
    const double2 a = xr[2 * b][p], bb = xr[2 * b][p + 1], cc = xr[2 * b + 1][p],
                  d = xr[2 * b + 1][p + 1];
    const double2 det = csub(cmul(a, d), cmul(bb, cc));
    const double dd = det.x * det.x + det.y * det.y;
    mindet2 = (dd < mindet2 || dd != dd) ? dd : mindet2;
    const double rd = recip_pos(dd);
    const double2 idet = make_double2(det.x * rd, -det.y * rd);
    const double2 i00 = cmul(d, idet), i01 = cneg(cmul(bb, idet)), i10 = cneg(cmul(cc, idet)),
                  i11 = cmul(a, idet);
    const bool r0 = (r == p), r1 = (r == p + 1);
    const double2 f0 = xc[2 * b][r], f1 = xc[2 * b + 1][r];
    const double2 g0 = cadd(cmul(f0, i00), cmul(f1, i10));
    const double2 g1 = cadd(cmul(f0, i01), cmul(f1, i11));
    const double2 b0 = r0 ? cneg(i00) : r1 ? cneg(i10) : g0;
    const double2 b1 = r0 ? cneg(i01) : r1 ? cneg(i11) : g1;
    const bool keep = !(r0 || r1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = c0 + c;
      double2 v = keep ? m[c] : make_double2(0.0, 0.0);
      v = csub(v, cmul(b0, xr[2 * b][col]));
      v = csub(v, cmul(b1, xr[2 * b + 1][col]));
      m[c] = (col == p) ? cneg(b0) : (col == p + 1) ? cneg(b1) : v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c) Ps[r][c0 + c] = m[c];
  __syncthreads();
  return sqrt(sqrt(mindet2));   // |det B|^(1/2): same scale as a scalar pivot
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
#pragma unroll
  for (int s = 0; s < 8; ++s) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (a < a0 || a >= a1) continue;
      const T nare = -av[a][s].x, aim = av[a][s].y, naim = -av[a][s].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b < b0 || b >= b1) continue;
        cre[a][b] = mfma16(nare, bv[b][s].x, cre[a][b]);
        cim[a][b] = mfma16(nare, bv[b][s].y, cim[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b < b0 || b >= b1) continue;
        cre[a][b] = mfma16(aim, bv[b][s].y, cre[a][b]);
        cim[a][b] = mfma16(naim, bv[b][s].x, cim[a][b]);
      }
    }
  }
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

template <typename T>
__device__ __forceinline__ void mma_ksteps(typename v4of<T>::t (*cre)[2],
                                           typename v4of<T>::t (*cim)[2],
                                           const typename cplx<T>::t (&av)[2][2],
                                           const typename cplx<T>::t (&bv)[2][2]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T nare = -av[a][s].x, aim = av[a][s].y, naim = -av[a][s].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(nare, bv[b][s].x, cre[a][b]);
        cim[a][b] = mfma16(nare, bv[b][s].y, cim[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(aim, bv[b][s].y, cre[a][b]);
        cim[a][b] = mfma16(naim, bv[b][s].x, cim[a][b]);
      }
    }
  }
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
      for (int q = 0; q < 4; ++q) sv[a][b][q] = dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr];
  V4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = V4{0, 0, 0, 0};
      cim[a][b] = V4{0, 0, 0, 0};
    }
  T2 a0[2][2], b0[2][2], a1[2][2], b1[2][2];
  load_ksteps(a0, b0, A, B, 0, lr, lk);
  load_ksteps(a1, b1, A, B, 1, lr, lk);
  mma_ksteps<T>(cre, cim, a0, b0);
  load_ksteps(a0, b0, A, B, 2, lr, lk);
  mma_ksteps<T>(cre, cim, a1, b1);
  load_ksteps(a1, b1, A, B, 3, lr, lk);
  mma_ksteps<T>(cre, cim, a0, b0);
  mma_ksteps<T>(cre, cim, a1, b1);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = (sv[a][b][q].x + cre[a][b][q]) * sg;
        v.y = (sv[a][b][q].y + cim[a][b][q]) * sg;
        dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr] = v;
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
                           double2 (*xrow)[TB], double2 (*xcol)[TB]) {
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
  const double minpiv = invert_pivot_block(Ps, xrow, xcol);
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
  V4 qre = V4{0, 0, 0, 0}, qim = V4{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int kk = acc_k<T>(s, lk);
    const double2 pv = Ps[kk][16 * qb + lr];
    const T bre = static_cast<T>(pv.x), bim = static_cast<T>(pv.y);
    const T are = cre[s >> 2][0][s & 3], aim = cim[s >> 2][0][s & 3];
    qre = mfma16(are, bre, qre);
    qim = mfma16(are, bim, qim);
    qre = mfma16(-aim, bim, qre);
    qim = mfma16(aim, bre, qim);
  }
  T2* Qb = static_cast<T2*>(jb.Qn) + size_t(I) * TB * TB + (16 * qa) * TB + 16 * qb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T2 v;
    v.x = qre[q];
    v.y = qim[q];
    Qb[mfma_row<T>(lk, q) * TB + lr] = v;
  }
}

template <typename T, int R>
__device__ void lookahead_work(const GJJob& jb, int g, int nt, double2 (*Ps)[TB + 1],
                               double2 (*xrow)[TB], double2 (*xcol)[TB]) {
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
  const double minpiv = invert_pivot_block(Ps, xrow, xcol);
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

// Workgroup -> (job q, index w within the job).  Workgroups are dealt to the 8
// XCDs round robin.  When the job count n divides 8, job q gets the XCDs x with
// x % n == q; when 8 divides n, XCD x serves jobs x, x + 8, ...; either way
// the panel buffers a chain's workgroups all read stay in the L2 of its own
// XCDs.  For n dividing 8 the grid is padded to a multiple of 8 (grid_size) and
// the surplus workgroups return false.
__device__ __forceinline__ bool job_of(int n, int per, int* q, int* w) {
  const int b = blockIdx.x;
  const int x = b & 7, slot = b >> 3;
  if (8 % n == 0) {
    *q = x % n;
    *w = slot * (8 / n) + x / n;
  } else if (n % 8 == 0) {
    const int m = n / 8;
    *q = x + 8 * (slot % m);
    *w = slot / m;
  } else {
    *q = b / per;
    *w = b - *q * per;
  }
  return *w < per;
}

int grid_size(int n, int per) { return 8 % n == 0 ? 8 * ceil_div(n * per, 8) : n * per; }

template <typename T>
__global__ __launch_bounds__(256) void k_gj_panel(GJJobs jobs, int nt) {
  __shared__ double2 Ps[TB][TB + 1];
  __shared__ double2 xrow[4][TB], xcol[4][TB];
  int q, w;
  if (!job_of(jobs.n, jobs.j[0].wgs, &q, &w)) return;
  int wg = q * jobs.j[0].wgs + w;
  GJJob jb = pick(jobs, &wg);
  panel_work<T>(jb, wg, nt, Ps, xrow, xcol);
}

// Update k (all tiles; negated when last) -- the final panel of a block.
template <typename T>
__global__ __launch_bounds__(256) void k_gj_update(GJJobs jobs, size_t tiles) {
  int q, w;
  if (!job_of(jobs.n, jobs.j[0].wgs, &q, &w)) return;
  int wg = q * jobs.j[0].wgs + w;
  GJJob jb = pick(jobs, &wg);
  update_work<T>(jb, wg, tiles, -1);
}

// Update k outside column k+1, plus the look-ahead panel k+1 (R row tiles per
// look-ahead workgroup).  Within each job the look-ahead workgroups come first,
// so that they are dispatched first: they carry the launch's critical path.
template <typename T, int R>
__global__ __launch_bounds__(256, 2) void k_gj_fused(GJJobs jobs, int nt, size_t tiles) {
  __shared__ double2 Ps[TB][TB + 1];
  __shared__ double2 xrow[4][TB], xcol[4][TB];
  const int look = jobs.j[0].wgs - jobs.j[0].wgs_upd;   // look-ahead workgroups per job
  int q, w;
  if (!job_of(jobs.n, jobs.j[0].wgs, &q, &w)) return;
  int tmp = q * jobs.j[0].wgs + w;
  GJJob jb = pick(jobs, &tmp);
  if (w < look)
    lookahead_work<T, R>(jb, w, nt, Ps, xrow, xcol);
  else
    update_work<T>(jb, w - look, tiles, jb.k + 1);
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
};
struct SchurJobs {
  SchurJob j[MAXJ];
  int n;
};

template <typename T>
__global__ __launch_bounds__(256) void k_schur(SchurJobs jobs, int ny, size_t tiles) {
  using T2 = typename cplx<T>::t;
  const size_t t = blockIdx.x % tiles;
  const int ji = static_cast<int>(blockIdx.x / tiles);
  void* const jdst = RCP_SEL16(jobs, ji, dst);
  const void* const jsrc1 = RCP_SEL16(jobs, ji, src1);
  const void* const jsrc2 = RCP_SEL16(jobs, ji, src2);
  const double2* const dco = RCP_SEL16(jobs, ji, dco);
  const double2* const eco = RCP_SEL16(jobs, ji, eco);
  const double2* const c1 = RCP_SEL16(jobs, ji, c1);
  const double2* const c2 = RCP_SEL16(jobs, ji, c2);
  int I, J;
  tile_coords(static_cast<int>(t), &I, &J);
  T2* dst = static_cast<T2*>(jdst) + t * TB * TB;
  const T2* s1 = jsrc1 ? static_cast<const T2*>(jsrc1) + t * TB * TB : nullptr;
  const T2* s2 = jsrc2 ? static_cast<const T2*>(jsrc2) + t * TB * TB : nullptr;
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    int a = I * TB + e / TB, b = J * TB + e % TB;
    double2 v = make_double2(0.0, 0.0);
    if (a == b) {
      v = (a < ny) ? dco[a] : make_double2(1.0, 0.0);
    } else if (a == b + 1 && a < ny) {
      v = eco[b];
    } else if (b == a + 1 && b < ny) {
      v = eco[a];
    }
    if (a < ny && b < ny) {
      if (s1) v = csub(v, cmul(cmul(c1[a], c1[b]), to_c128(s1[e])));
      if (s2) v = csub(v, cmul(cmul(c2[a], c2[b]), to_c128(s2[e])));
    }
    dst[e] = from_c128<T2>(v);
  }
}

// Factor B same-shape geometries in lockstep: every launch carries the chains
// of all of them (two per geometry).
template <typename T>
int run_factor(rcp_factors* const* fs, int B, hipStream_t s) {
  const rcp_factors* f0 = fs[0];
  const int N = f0->nx, ny = f0->ny, nt = f0->nt, m = f0->m;
  const size_t tiles = f0->tiles;
  const int lenL = m, lenR = N - 1 - m;
  auto D = [&](int g, int i) { return fs[g]->dco + size_t(i) * ny; };
  auto E = [&](int g, int i) { return fs[g]->eco + size_t(i) * ny; };
  auto C = [&](int g, int i) { return fs[g]->cco + size_t(i) * ny; };

  auto schur = [&](SchurJobs js) -> int {
    if (js.n == 0) return RCP_OK;
    int nsrc = 0;
    for (int q = 0; q < js.n; ++q) nsrc += 1 + (js.j[q].src1 != nullptr) + (js.j[q].src2 != nullptr);
    KTimer kt(K_SCHUR, s, double(nsrc) * tiles * TB * TB * f0->elem_bytes);
    k_schur<T><<<static_cast<int>(tiles * js.n), 256, 0, s>>>(js, ny, tiles);
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  };
  const int upd_wgs = static_cast<int>((tiles + 3) / 4);
  const int pan_wgs = ceil_div(nt, 4);   // first panel: four row tiles per workgroup
  const double cmac = 8.0 * TB * TB * TB;   // flops of one TB^3 complex product
  // Sweep the given blocks (chain c of geometry g) through all panels; the
  // panel buffers of chain c alternate between halves 2c and 2c+1.
  struct Chain {
    int g, c, block;
  };
  auto sweep = [&](int nch, const Chain* ch) -> int {
    auto job = [&](const Chain& x, int k) {
      const rcp_factors* f = fs[x.g];
      GJJob b{};
      b.k = k;
      b.X = block_ptr(f, x.block);
      const int cur = 2 * x.c + (k & 1), nxt = 2 * x.c + ((k + 1) & 1);
      b.L = f->wsL[cur];
      b.Q = f->wsQ[cur];
      b.P = f->wsP[cur];
      b.Ln = f->wsL[nxt];
      b.Qn = f->wsQ[nxt];
      b.Pn = f->wsP[nxt];
      b.health = f->health + size_t(x.block) * nt + (k + 1 < nt ? k + 1 : k);
      return b;
    };
    {   // panel 0 (writes the "next" buffers of k = -1, i.e. half 2c)
      GJJobs js{};
      for (int q = 0; q < nch; ++q) {
        GJJob b = job(ch[q], -1);
        b.k = 0;
        b.health = fs[ch[q].g]->health + size_t(ch[q].block) * nt;
        b.wgs = pan_wgs;
        js.j[js.n++] = b;
      }
      KTimer kt(K_GJ_PANEL, s, nch * cmac * nt);
      k_gj_panel<T><<<grid_size(nch, pan_wgs), 256, 0, s>>>(js, nt);
      RCP_HIP(hipGetLastError());
    }
    // look-ahead row tiles per workgroup: two when sixteen chains share the GPU
    // (84 -> 76 us per launch on 1080-row blocks), otherwise one (shortest chain)
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
      KTimer kt(K_GJ_UPDATE, s, nch * cmac * double(tiles));
      const int grid = grid_size(nch, upd_wgs + look_wgs);
      if (R == 1)
        k_gj_fused<T, 1><<<grid, 256, 0, s>>>(js, nt, tiles);
      else
        k_gj_fused<T, 2><<<grid, 256, 0, s>>>(js, nt, tiles);
      RCP_HIP(hipGetLastError());
    }
    {   // final update, negated
      GJJobs js{};
      for (int q = 0; q < nch; ++q) {
        GJJob b = job(ch[q], nt - 1);
        b.last = 1;
        b.wgs = upd_wgs;
        b.wgs_upd = upd_wgs;
        js.j[js.n++] = b;
      }
      KTimer kt(K_GJ_LAST, s, nch * cmac * double(tiles - nt));
      k_gj_update<T><<<grid_size(nch, upd_wgs), 256, 0, s>>>(js, tiles);
      RCP_HIP(hipGetLastError());
    }
    return RCP_OK;
  };

  {   // chain heads
    SchurJobs js{};
    for (int g = 0; g < B; ++g) {
      if (lenL > 0)
        js.j[js.n++] = SchurJob{block_ptr(fs[g], 0), nullptr, nullptr, D(g, 0), E(g, 0), nullptr, nullptr};
      if (lenR > 0)
        js.j[js.n++] = SchurJob{block_ptr(fs[g], N - 1), nullptr, nullptr, D(g, N - 1), E(g, N - 1),
                                nullptr, nullptr};
    }
    int rc = schur(js);
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
    for (int g = 0; g < B; ++g) {
      if (bL >= 0 && bL + 1 < m)
        js.j[js.n++] = SchurJob{block_ptr(fs[g], bL + 1), block_ptr(fs[g], bL), nullptr,
                                D(g, bL + 1), E(g, bL + 1), C(g, bL), nullptr};
      if (bR >= 0 && bR - 1 > m)
        js.j[js.n++] = SchurJob{block_ptr(fs[g], bR - 1), block_ptr(fs[g], bR), nullptr,
                                D(g, bR - 1), E(g, bR - 1), C(g, bR - 1), nullptr};
    }
    rc = schur(js);
    if (rc) return rc;
  }
  {   // middle blocks
    SchurJobs js{};
    Chain ch[MAXJ];
    int nch = 0;
    for (int g = 0; g < B; ++g) {
      SchurJob z{block_ptr(fs[g], m), nullptr, nullptr, D(g, m), E(g, m), nullptr, nullptr};
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
    int rc = schur(js);
    if (rc) return rc;
    rc = sweep(nch, ch);
    if (rc) return rc;
  }
  return RCP_OK;
}

}  // namespace

namespace rcp {

int factor_blocks(rcp_factors* const* fs, int B, hipStream_t s) {
  if (B < 1 || B > MAXJ / 2) return fail(RCP_EINVAL, "batch of 1 to 8 geometries");
  const int prec = fs[0]->precision;
  int rc = (prec == RCP_FP64) ? run_factor<double>(fs, B, s) : run_factor<float>(fs, B, s);
  if (rc) return rc;
  // pivot health: one wait, then scan the smallest pivot modulus of every panel
  RCP_HIP(hipStreamSynchronize(s));
  for (int g = 0; g < B; ++g) {
    const rcp_factors* f = fs[g];
    const size_t nh = size_t(f->nx) * f->nt;
    std::vector<double> h(nh);
    RCP_HIP(hipMemcpy(h.data(), f->health, nh * sizeof(double), hipMemcpyDeviceToHost));
    // diagonal entries are O(4/h^2); a pivot below 1e-13 of that scale is treated as singular
    const double tiny = 1e-13 * 4.0 / (f->h * f->h);
    for (size_t q = 0; q < nh; ++q) {
      if (!(h[q] > tiny) || !std::isfinite(h[q])) {
        return fail(RCP_ESINGULAR, "geometry " + std::to_string(g) + ": pivot block " +
                                       std::to_string(q % f->nt) + " of column block " +
                                       std::to_string(q / f->nt) + " has pivot modulus " +
                                       std::to_string(h[q]));
      }
    }
  }
  return RCP_OK;
}

}  // namespace rcp

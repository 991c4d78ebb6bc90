// Forward / back substitution with the block inverses of the twisted
// elimination (the single reciprocal solve of Sec. "Reciprocal approach", and
// the many forward solves of the brute-force average, Eq. 6).
//
// With X_i the stored block inverses and middle block m:
//   forward left   g_i = X_i (f_i - C_{i-1} g_{i-1}),   i = 0 .. m-1
//   forward right  g_i = X_i (f_i - C_i g_{i+1}),       i = nx-1 .. m+1
//   middle         u_m = X_m (f_m - C_{m-1} g_{m-1} - C_m g_{m+1})
//   back left      u_i = g_i - X_i (C_i u_{i+1}),       i = m-1 .. 0
//   back right     u_i = g_i - X_i (C_{i-1} u_{i-1}),   i = m+1 .. nx-1
// conj(A)^{-1} (= A^{-dag}, since A = A^T) uses conj(X_i) and conj(C_i).
// One right-hand side: a symmetric matrix-vector product per block.  Blocks
// of more than GEMV_NT_MAX tiles per edge read each packed lower tile once (row
// and column shares of every tile, then a fixed-order sum per row; bound by
// HBM); smaller blocks use one launch per step, which reads the tiles above
// the diagonal again as transposes (bound by latency).  Many right-hand sides:
// an MFMA GEMM per block.
#include <cmath>
#include <vector>

#include <limits>
#include <mutex>

#include <rocblas/rocblas.h>

#include "rcp_internal.h"

namespace {
using namespace rcp;

// Blocks of at most GEMV_NT_MAX tiles per edge use the one-launch product
// k_gemv (it reads the tiles above the diagonal a second time, as transposes,
// but saves the second launch, which dominates for small blocks).
constexpr int GEMV_NT_MAX = 20;
constexpr int GEMV_NPMAX = GEMV_NT_MAX * TB;

struct SvJob {
  const void* X;
  double2* out;
  const double2* base;   // out = base + X g (base may be null)
  const double2* f;      // g = f - C1 v1 - C2 v2 (each term optional)
  const double2* v1;
  const double2* c1;
  const double2* v2;
  const double2* c2;
  double2* part;         // partial sums of this chain (tiles x 2 x TB)
};
// Job table of a launch: the left and right chain step of each factor set; two
// entries for one set, 2 MAX_BATCH for batches (the table is a kernel argument,
// so a single solve does not carry the batch-sized one).
template <int NJ>
struct SvJobs {
  SvJob j[NJ];
  int n;
};

__device__ __forceinline__ double2 maybe_conj(double2 a, int c) {
  return c ? make_double2(a.x, -a.y) : a;
}

template <int NJ>
__device__ __forceinline__ SvJob job_of(const SvJobs<NJ>& jobs, int ji) {
  SvJob jb;
  if constexpr (NJ == 2) {
    jb = jobs.j[0];
    if (ji == 1) jb = jobs.j[1];
  } else {
    static_assert(NJ == 16, "job tables of 2 or 16 entries");
    jb.X = RCP_SEL16(jobs, ji, X);
    jb.out = RCP_SEL16(jobs, ji, out);
    jb.base = RCP_SEL16(jobs, ji, base);
    jb.f = RCP_SEL16(jobs, ji, f);
    jb.v1 = RCP_SEL16(jobs, ji, v1);
    jb.c1 = RCP_SEL16(jobs, ji, c1);
    jb.v2 = RCP_SEL16(jobs, ji, v2);
    jb.c2 = RCP_SEL16(jobs, ji, c2);
    jb.part = RCP_SEL16(jobs, ji, part);
  }
  return jb;
}

// One 512-thread workgroup per (job, 8-row quarter of a 32-row strip), so a
// block is spread over 4 * nt workgroups.  Wave w takes the tiles J = w + 8u
// of the strip.  Every load instruction of a wave reads whole cache lines:
//   stored tile (I, J <= I): its rows r0 .. r0+7 are 4 KB contiguous; lane l
//     of load c holds row 2c + l/32, column l%32, and keeps a partial sum per
//     c (reduced over the 32 lanes of equal l/32 at the end);
//   tile (J > I, I), used transposed: columns r0 .. r0+7 of each of its 32
//     rows (128 B each); lane l of load c holds row 8c + l/8, column r0 + l%8,
//     and keeps one partial sum for output row l%8 (reduced over l/8).
// All tile loads are issued before the input vector is formed in LDS, so one
// memory latency covers the step.  Partial sums are combined in a fixed
// order: the result does not depend on scheduling.
// MT = tiles per wave = ceil(nt / 8).  Used for small blocks (nt <= GEMV_NT_MAX),
// where one launch per step beats the two of the tile-once product below.
template <typename T, int MT, int NJ>
__global__ __launch_bounds__(512) void k_gemv(SvJobs<NJ> jobs, int nt, int ny, int conjop) {
  using T2 = typename cplx<T>::t;
  __shared__ double2 g[GEMV_NPMAX];
  __shared__ double2 redd[8][8];
  __shared__ double2 redt[8][8];
  const int per_job = 4 * nt;
  const int ji = blockIdx.x / per_job, rem = blockIdx.x % per_job;
  const int I = rem >> 2, r0 = (rem & 3) * 8;
  const SvJob jb = job_of(jobs, ji);
  const int tid = threadIdx.x;
  const T2* X = static_cast<const T2*>(jb.X);
  const int wave = tid >> 6, lane = tid & 63;
  T2 x[MT][4];
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int J = wave + 8 * u;
    if (J < nt) {
      if (J <= I) {
        const T2* t = X + tile_index(I, J) * TB * TB + r0 * TB + lane;
#pragma unroll
        for (int c = 0; c < 4; ++c) x[u][c] = t[c * 64];
      } else {
        const T2* t = X + tile_index(J, I) * TB * TB + (lane >> 3) * TB + r0 + (lane & 7);
#pragma unroll
        for (int c = 0; c < 4; ++c) x[u][c] = t[c * 8 * TB];
      }
    }
  }
  const int np = nt * TB;
  for (int k = tid; k < np; k += 512) {
    double2 v = make_double2(0.0, 0.0);
    if (k < ny) {
      if (jb.f) v = jb.f[k];
      if (jb.v1) v = csub(v, cmul(maybe_conj(jb.c1[k], conjop), jb.v1[k]));
      if (jb.v2) v = csub(v, cmul(maybe_conj(jb.c2[k], conjop), jb.v2[k]));
    }
    g[k] = v;
  }
  __syncthreads();
  const double cs_im = conjop ? -1.0 : 1.0;
  double2 accd[4], acct = make_double2(0.0, 0.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) accd[c] = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int J = wave + 8 * u;
    if (J < nt) {
      if (J <= I) {
        const double2 gv = g[J * TB + (lane & 31)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double2 xv = to_c128(x[u][c]);
          xv.y *= cs_im;
          accd[c] = cadd(accd[c], cmul(xv, gv));
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double2 xv = to_c128(x[u][c]);
          xv.y *= cs_im;
          acct = cadd(acct, cmul(xv, g[J * TB + 8 * c + (lane >> 3)]));
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      accd[c].x += __shfl_xor(accd[c].x, d, 64);
      accd[c].y += __shfl_xor(accd[c].y, d, 64);
    }
  }
#pragma unroll
  for (int d = 8; d < 64; d <<= 1) {
    acct.x += __shfl_xor(acct.x, d, 64);
    acct.y += __shfl_xor(acct.y, d, 64);
  }
  if ((lane & 31) == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) redd[wave][2 * c + (lane >> 5)] = accd[c];
  }
  if (lane < 8) redt[wave][lane] = acct;
  __syncthreads();
  if (tid < 8) {
    double2 sum = make_double2(0.0, 0.0);
    for (int w = 0; w < 8; ++w) sum = cadd(sum, cadd(redd[w][tid], redt[w][tid]));
    const int row = I * TB + r0 + tid;
    if (row < ny) {
      double2 b = jb.base ? jb.base[row] : make_double2(0.0, 0.0);
      jb.out[row] = cadd(b, sum);
    }
  }
}

// y = op(X) g for a symmetric block X stored as its packed lower tiles, every
// stored tile read once.  One wave per stored tile (I, J), J <= I, packed
// index t; it writes two 32-vectors of partial sums:
//   part[t][0] = op(X_IJ) g_J     (a share of the rows of strip I)
//   part[t][1] = op(X_IJ)^T g_I   (a share of the rows of strip J; J < I only)
// and k_symv_reduce adds the shares of each row in a fixed order.
// g = f - op(C1) v1 - op(C2) v2 (each term optional), zero in the padding.
// In registers, load c (0..15) of lane l holds row 2c + l/32, column l%32 of
// the tile, so each load instruction reads 1 KB (complex128) contiguous.  The
// column shares are summed in-lane over the 16 loads, then across the two
// half-waves; the row shares across the 32 lanes of a half-wave by recursive
// halving (each exchange halves the values a lane holds).
template <typename T, int NJ>
__global__ __launch_bounds__(256) void k_symv_tiles(SvJobs<NJ> jobs, int ny, int tiles,
                                                    int conjop) {
  using T2 = typename cplx<T>::t;
  __shared__ double2 gs[4][64];
  const int per_job = (tiles + 3) >> 2;
  const int ji = blockIdx.x / per_job;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = (blockIdx.x - ji * per_job) * 4 + wave;
  const SvJob jb = job_of(jobs, ji);
  const int tt = t < tiles ? t : tiles - 1;
  int I = static_cast<int>((sqrtf(8.0f * tt + 1.0f) - 1.0f) * 0.5f);
  if ((I + 1) * (I + 2) / 2 <= tt) ++I;
  if (I * (I + 1) / 2 > tt) --I;
  const int J = tt - I * (I + 1) / 2;
  const T2* X = static_cast<const T2*>(jb.X) + size_t(tt) * TB * TB + lane;
  T2 x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = load_stream(&X[c * 64]);
  {
    const int k = (lane < 32 ? J : I) * TB + (lane & 31);
    double2 v = make_double2(0.0, 0.0);
    if (k < ny) {
      if (jb.f) v = jb.f[k];
      if (jb.v1) v = csub(v, cmul(maybe_conj(jb.c1[k], conjop), jb.v1[k]));
      if (jb.v2) v = csub(v, cmul(maybe_conj(jb.c2[k], conjop), jb.v2[k]));
    }
    gs[wave][lane] = v;
  }
  __syncthreads();
  if (t >= tiles) return;
  const double cs_im = conjop ? -1.0 : 1.0;
  const int h = lane >> 5;
  const double2 gj = gs[wave][lane & 31];
  double2 rp[16];
  double2 cp = make_double2(0.0, 0.0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double2 xv = to_c128(x[c]);
    xv.y *= cs_im;
    rp[c] = cmul(xv, gj);
    cp = cadd(cp, cmul(xv, gs[wave][32 + 2 * c + h]));
  }
  // 16 row values -> 8 (lane bit 4) -> 4 (bit 3) -> 2 (bit 2) -> 1 (bit 1);
  // lane l then holds row 2 ((l >> 1) & 15) + h summed over bits 4..1
#pragma unroll
  for (int w = 8, b = 16; w >= 1; w >>= 1, b >>= 1) {
    const bool up = (lane & b) != 0;
#pragma unroll
    for (int i = 0; i < w; ++i) {
      const double2 send = up ? rp[i] : rp[i + w];
      const double2 keep = up ? rp[i + w] : rp[i];
      rp[i] = make_double2(keep.x + __shfl_xor(send.x, b, 64), keep.y + __shfl_xor(send.y, b, 64));
    }
  }
  rp[0].x += __shfl_xor(rp[0].x, 1, 64);
  rp[0].y += __shfl_xor(rp[0].y, 1, 64);
  cp.x += __shfl_xor(cp.x, 32, 64);
  cp.y += __shfl_xor(cp.y, 32, 64);
  double2* P = jb.part + size_t(t) * 2 * TB;
  if ((lane & 1) == 0) P[2 * ((lane >> 1) & 15) + h] = rp[0];
  if (J < I && lane < 32) P[TB + lane] = cp;
}

// out[k] = base[k] + the shares of row k of strip I = k / TB: part[(I, J)][0]
// for J <= I, part[(J, I)][1] for J > I.  One workgroup per (job, strip):
// thread (q, r) sums the shares of row r with J = q mod 8 in ascending J, then
// the eight sums of each row are added in q order.
template <int NJ>
__global__ __launch_bounds__(256) void k_symv_reduce(SvJobs<NJ> jobs, int nt, int ny) {
  __shared__ double2 red[8][TB];
  const int ji = blockIdx.x / nt;
  const int I = blockIdx.x - ji * nt;
  const int q = threadIdx.x >> 5, r = threadIdx.x & 31;
  const SvJob jb = job_of(jobs, ji);
  const double2* P = jb.part;
  double2 sum = make_double2(0.0, 0.0);
  for (int J = q; J < nt; J += 8) {
    const size_t at = J <= I ? tile_index(I, J) * 2 * TB + r : tile_index(J, I) * 2 * TB + TB + r;
    sum = cadd(sum, P[at]);
  }
  red[q][r] = sum;
  __syncthreads();
  const int k = I * TB + threadIdx.x;
  if (threadIdx.x < TB && k < ny) {
    double2 s = red[0][threadIdx.x];
#pragma unroll
    for (int u = 1; u < 8; ++u) s = cadd(s, red[u][threadIdx.x]);
    jb.out[k] = jb.base ? cadd(jb.base[k], s) : s;
  }
}

// ---------------------------------------------------------------------------
// Many right-hand sides: out[r, :] = base[r, :] + (in[r, :] X)  (X symmetric),
// in[r, k] = f[r, k] (+ line source) - C1 v1[r, k] - C2 v2[r, k].
// Rows r of one block sit rstride apart (layout R x nx x ny).
struct MmJob {
  const double2* X;
  double2* out;
  const double2* base;
  const double2* f;
  const double2* fline;   // R x nx line-source values on row jline, or null
  const double2* v1;
  const double2* c1;
  const double2* v2;
  const double2* c2;
  int block;
};
struct MmJobs {
  MmJob j[2];
  int n;
};

constexpr int MT = 64;   // workgroup tile (rows r) x (columns j)
constexpr int KC = 16;   // k chunk staged in LDS
static_assert(GEMM_SPLIT_TILES * MT * MT * 16 == GEMM_SPLIT_BYTES, "split workspace size");

// Staging of one k chunk: every thread fetches 4 elements of the right-hand
// side tile (formed on the fly: f + line source - C1 v1 - C2 v2) and 4 of the
// block tile into registers; they are stored to LDS after the previous chunk's
// products, so the global loads of chunk c+1 overlap the MFMA work of chunk c.
struct MmStage {
  double2 a[4], b[4];
};

__device__ __forceinline__ void mm_fetch(const MmJob& jb, MmStage& st, int kc, int r0, int j0,
                                         int R, int nx, int ny, int nt, size_t rstride,
                                         size_t boff, int jline, int conjop) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {   // A: 64 rows x 16 k, contiguous along k
    const int e = tid + 256 * u, rr = e >> 4, kk = e & 15;
    const int r = r0 + rr, k = kc * KC + kk;
    double2 v = make_double2(0.0, 0.0);
    if (r < R && k < ny) {
      const size_t q = size_t(r) * rstride + boff + k;
      if (jb.f) v = jb.f[q];
      if (jb.fline && k == jline) v = cadd(v, jb.fline[size_t(r) * nx + jb.block]);
      if (jb.v1) v = csub(v, cmul(maybe_conj(jb.c1[k], conjop), jb.v1[q]));
      if (jb.v2) v = csub(v, cmul(maybe_conj(jb.c2[k], conjop), jb.v2[q]));
    }
    st.a[u] = v;
  }
  const int K = (kc * KC) / TB, koff = (kc * KC) % TB;
#pragma unroll
  for (int u = 0; u < 4; ++u) {   // B: 16 k x 64 j as two 16 x 32 halves of storage tiles
    const int e = tid + 256 * u, half = e >> 9, idx = e & 511;
    const int J = j0 / TB + half;
    double2 x = make_double2(0.0, 0.0);
    if (J < nt) {
      if (K >= J) {   // rows koff.. of tile (K, J): contiguous along j
        x = jb.X[tile_index(K, J) * TB * TB + (koff + (idx >> 5)) * TB + (idx & 31)];
      } else {        // X(k, j) = X(j, k): columns koff.. of tile (J, K), contiguous along k
        x = jb.X[tile_index(J, K) * TB * TB + (idx >> 4) * TB + koff + (idx & 15)];
      }
    }
    if (conjop) x.y = -x.y;
    st.b[u] = x;
  }
}

__device__ __forceinline__ void mm_store(const MmStage& st, double2 (*As)[KC + 1],
                                         double2 (*Bs)[MT + 1], int kc, int j0, int nt) {
  const int tid = threadIdx.x;
  const int K = (kc * KC) / TB;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;
    As[e >> 4][e & 15] = st.a[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, half = e >> 9, idx = e & 511;
    const int J = j0 / TB + half;
    int kk, jj;
    if (J >= nt || K >= J) {
      kk = idx >> 5;
      jj = idx & 31;
    } else {
      jj = idx >> 4;
      kk = idx & 15;
    }
    Bs[kk][half * TB + jj] = st.b[u];
  }
}

// Tile t of a sweep step: its job, row tile and column tile.  Tiles with all
// MT right-hand-side rows come first (for all jobs), the partial row tiles
// (R mod MT rows) last.
__device__ __forceinline__ void gemm_tile_of(int t, int njobs, int R, int ntile_j, int* ji, int* rt,
                                             int* jt) {
  const int nfull = R / MT;
  const int nfb = njobs * nfull * ntile_j;
  if (t < nfb) {
    *ji = t / (nfull * ntile_j);
    const int w = t - *ji * nfull * ntile_j;
    *rt = w / ntile_j;
    *jt = w - *rt * ntile_j;
  } else {
    *ji = (t - nfb) / ntile_j;
    *rt = nfull;
    *jt = (t - nfb) - *ji * ntile_j;
  }
}

// One sweep step of the many-right-hand-side solve: out = base + RHS X_i for
// every (job, 64-row, 64-column) tile, RHS formed on the fly, X_i read from
// its packed symmetric tiles; four waves, each a 32 x 32 quarter.
// Workgroups b < nwhole take tile b whole.  The tiles after them (the ones that
// would leave a few CUs a tile more than the rest) are split along k into
// nsplit parts, workgroup nwhole + s taking part s % nsplit of tile
// nwhole + s / nsplit; a part writes its 64 x 64 partial sum to ws[s] and
// k_gemm_fixup adds the parts in order.
__global__ __launch_bounds__(256, 3) void k_gemm_sweep(MmJobs jobs, int R, int nx, int ny, int nt,
                                                        size_t rstride, int jline, int conjop,
                                                        int nwhole, int nsplit, double2* ws) {
  __shared__ double2 As[MT][KC + 1];
  __shared__ double2 Bs[KC][MT + 1];
  const int ntile_j = ceil_div(nt * TB, MT);
  const int b = blockIdx.x;
  const int nk = nt * TB / KC;
  int tile = b, kc0 = 0, kc1 = nk;
  if (b >= nwhole) {
    const int sp = b - nwhole, part = sp % nsplit;
    tile = nwhole + sp / nsplit;
    kc0 = part * nk / nsplit;
    kc1 = (part + 1) * nk / nsplit;
  }
  int ji, rt, jt;
  gemm_tile_of(tile, jobs.n, R, ntile_j, &ji, &rt, &jt);
  MmJob jb = jobs.j[0];
  if (ji == 1) jb = jobs.j[1];
  const int r0 = rt * MT, j0 = jt * MT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const size_t boff = size_t(jb.block) * ny;
  v4d cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = v4d{0, 0, 0, 0};
      cim[a][b] = v4d{0, 0, 0, 0};
    }
  MmStage st;
  mm_fetch(jb, st, kc0, r0, j0, R, nx, ny, nt, rstride, boff, jline, conjop);
  for (int kc = kc0; kc < kc1; ++kc) {
    __syncthreads();
    mm_store(st, As, Bs, kc, j0, nt);
    __syncthreads();
    if (kc + 1 < kc1) mm_fetch(jb, st, kc + 1, r0, j0, R, nx, ny, nt, rstride, boff, jline, conjop);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      double2 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[32 * wr + 16 * a + lr][4 * s + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[4 * s + lk][32 * wc + 16 * b + lr];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double naim = -av[a].y;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cre[a][b] = mfma16(av[a].x, bv[b].x, cre[a][b]);
          cre[a][b] = mfma16(naim, bv[b].y, cre[a][b]);
          cim[a][b] = mfma16(av[a].x, bv[b].y, cim[a][b]);
          cim[a][b] = mfma16(av[a].y, bv[b].x, cim[a][b]);
        }
      }
    }
  }
  if (b >= nwhole) {   // a k part: the whole 64 x 64 partial sum, row-major
    double2* P = ws + size_t(b - nwhole) * MT * MT;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = 32 * wr + 16 * a + mfma_row<double>(lk, q), cc = 32 * wc + 16 * bb + lr;
          P[rr * MT + cc] = make_double2(cre[a][bb][q], cim[a][bb][q]);
        }
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r = r0 + 32 * wr + 16 * a + mfma_row<double>(lk, q);
        int j = j0 + 32 * wc + 16 * b + lr;
        if (r < R && j < ny) {
          size_t o = size_t(r) * rstride + boff + j;
          double2 v = make_double2(cre[a][b][q], cim[a][b][q]);
          if (jb.base) v = cadd(v, jb.base[o]);
          jb.out[o] = v;
        }
      }
}

// out = base + the nsplit partial sums of split tile nwhole + blockIdx.x, added
// in part order.
__global__ __launch_bounds__(256) void k_gemm_fixup(MmJobs jobs, int R, int ny, int nt,
                                                     size_t rstride, int nwhole, int nsplit,
                                                     const double2* __restrict__ ws) {
  const int ntile_j = ceil_div(nt * TB, MT);
  int ji, rt, jt;
  gemm_tile_of(nwhole + blockIdx.x, jobs.n, R, ntile_j, &ji, &rt, &jt);
  MmJob jb = jobs.j[0];
  if (ji == 1) jb = jobs.j[1];
  const size_t boff = size_t(jb.block) * ny;
  const double2* P = ws + size_t(blockIdx.x) * nsplit * MT * MT;
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int r = rt * MT + e / MT, j = jt * MT + e % MT;
    if (r >= R || j >= ny) continue;
    double2 v = P[e];
    for (int q = 1; q < nsplit; ++q) v = cadd(v, P[size_t(q) * MT * MT + e]);
    const size_t o = size_t(r) * rstride + boff + j;
    if (jb.base) v = cadd(v, jb.base[o]);
    jb.out[o] = v;
  }
}

// A few right-hand sides (R < 64): the 64 x 64 tiles above would leave most of
// the GPU idle (17 workgroups per block on 1080-row blocks), so one workgroup
// takes a 16 (RHS) x 16 (column) output tile and its MW_WAVES waves take
// interleaved 16-wide k chunks (a few each, so that the chain of dependent
// loads per wave stays short), reduced through LDS in wave order.  Within a
// chunk lane group lk supplies k = 4 lk + s at MFMA step s, so that every lane
// reads four consecutive values of the right-hand side row and of the stored
// tile row (direct rows for tiles (K >= J), contiguous columns of tile (J, K)
// used transposed otherwise); no LDS staging.
constexpr int MW_WAVES = 16;
__global__ __launch_bounds__(64 * MW_WAVES) void k_mm_narrow(MmJobs jobs, int R, int nx, int ny,
                                                             int nt, size_t rstride, int jline,
                                                             int conjop) {
  __shared__ double2 red[MW_WAVES][16][16];
  const int ntile_r = ceil_div(R, 16), ntile_j = 2 * nt;
  const int per_job = ntile_r * ntile_j;
  const int ji = blockIdx.x / per_job;
  const int w = blockIdx.x % per_job;
  const int rt = w / ntile_j, jt = w % ntile_j;
  MmJob jb = jobs.j[0];
  if (ji == 1) jb = jobs.j[1];
  const int r0 = rt * 16, j0 = jt * 16;
  const int J = j0 / TB, jj = (j0 % TB) + (threadIdx.x & 15);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int r = r0 + lr;
  const bool rok = r < R;
  const size_t boff = size_t(jb.block) * ny;
  const size_t rbase = size_t(rok ? r : 0) * rstride + boff;
  v4d cre = v4d{0, 0, 0, 0}, cim = v4d{0, 0, 0, 0};
  const int nk = 2 * nt;
  for (int kc = wave; kc < nk; kc += MW_WAVES) {
    const int kb = kc * 16 + 4 * lk;   // this lane's k: kb .. kb + 3, one storage tile row K
    double2 a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = kb + s;
      double2 v = make_double2(0.0, 0.0);
      if (rok && k < ny) {
        const size_t q = rbase + k;
        if (jb.f) v = jb.f[q];
        if (jb.fline && k == jline) v = cadd(v, jb.fline[size_t(r) * nx + jb.block]);
        if (jb.v1) v = csub(v, cmul(maybe_conj(jb.c1[k], conjop), jb.v1[q]));
        if (jb.v2) v = csub(v, cmul(maybe_conj(jb.c2[k], conjop), jb.v2[q]));
      }
      a[s] = v;
    }
    const int K = kb / TB, kk = kb % TB;
    if (K >= J) {
      const double2* t = jb.X + tile_index(K, J) * TB * TB + kk * TB + jj;
#pragma unroll
      for (int s = 0; s < 4; ++s) b[s] = t[s * TB];
    } else {
      const double2* t = jb.X + tile_index(J, K) * TB * TB + jj * TB + kk;
#pragma unroll
      for (int s = 0; s < 4; ++s) b[s] = t[s];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double by = conjop ? -b[s].y : b[s].y;
      cre = mfma16(a[s].x, b[s].x, cre);
      cre = mfma16(-a[s].y, by, cre);
      cim = mfma16(a[s].x, by, cim);
      cim = mfma16(a[s].y, b[s].x, cim);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[wave][mfma_row<double>(lk, q)][lr] = make_double2(cre[q], cim[q]);
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = mfma_row<double>(lk, q);
      double2 v = red[0][i][lr];
      for (int u = 1; u < MW_WAVES; ++u) v = cadd(v, red[u][i][lr]);
      const int rr = r0 + i, j = j0 + lr;
      if (rr < R && j < ny) {
        const size_t o = size_t(rr) * rstride + boff + j;
        if (jb.base) v = cadd(v, jb.base[o]);
        jb.out[o] = v;
      }
    }
  }
}

// r = b - A x  (conj(A) if conjop) and per-workgroup partial sums of |r|^2, |b|^2
__global__ __launch_bounds__(256) void k_residual(int nx, int ny, const double2* __restrict__ dco,
                                                   const double2* __restrict__ eco,
                                                   const double2* __restrict__ cco,
                                                   const double2* __restrict__ b,
                                                   const double2* __restrict__ x,
                                                   double2* __restrict__ r, int conjop,
                                                   double* __restrict__ part) {
  __shared__ double sr[256], sb[256];
  size_t q = size_t(blockIdx.x) * 256 + threadIdx.x;
  double rr = 0.0, bb = 0.0;
  if (q < size_t(nx) * ny) {
    int i = static_cast<int>(q / ny), j = static_cast<int>(q % ny);
    double2 ax = cmul(maybe_conj(dco[q], conjop), x[q]);
    if (i > 0) ax = cadd(ax, cmul(maybe_conj(cco[q - ny], conjop), x[q - ny]));
    if (i + 1 < nx) ax = cadd(ax, cmul(maybe_conj(cco[q], conjop), x[q + ny]));
    if (j > 0) ax = cadd(ax, cmul(maybe_conj(eco[q - 1], conjop), x[q - 1]));
    if (j + 1 < ny) ax = cadd(ax, cmul(maybe_conj(eco[q], conjop), x[q + 1]));
    double2 bv = b[q];
    double2 rv = csub(bv, ax);
    if (r) r[q] = rv;
    rr = cabs2(rv);
    bb = cabs2(bv);
  }
  sr[threadIdx.x] = rr;
  sb[threadIdx.x] = bb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = sb[0];
  }
}

// fixed-order final sum of n pairs -> out[0], out[1]
__global__ void k_sum_pairs(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

__global__ void k_axpy(size_t n, const double2* __restrict__ dx, double2* __restrict__ x) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) x[q] = cadd(x[q], dx[q]);
}

// Forward and back sweeps of B factor sets of identical shape in lockstep:
// every launch carries the left and right chain step of each set.
template <typename T, int NJ>
int run_solve_vec(rcp_factors* const* fs, int B, const double2* const* rhs, double2* const* u,
                  int conjop, const int* nz_lo, const int* nz_hi, hipStream_t s) {
  using SvJobs = ::SvJobs<NJ>;
  const rcp_factors* f0 = fs[0];
  const int N = f0->nx, ny = f0->ny, nt = f0->nt, m = f0->m;
  const int lenL = m, lenR = N - 1 - m;
  auto U = [&](int g, int i) { return u[g] + size_t(i) * ny; };
  auto Fb = [&](int g, int i) { return rhs[g] + size_t(i) * ny; };
  auto C = [&](int g, int i) { return fs[g]->cco + size_t(i) * ny; };
  auto launch = [&](SvJobs& js) -> int {
    if (js.n == 0) return RCP_OK;
    KTimer kt(K_GEMV, s, double(js.n) * f0->tiles * TB * TB * sizeof(typename cplx<T>::t));
    if (nt <= GEMV_NT_MAX) {
      const dim3 grid(4 * nt * js.n);
      switch ((nt + 7) / 8) {
        case 1: k_gemv<T, 1, NJ><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
        case 2: k_gemv<T, 2, NJ><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
        default: k_gemv<T, 3, NJ><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
      }
      RCP_HIP(hipGetLastError());
      return RCP_OK;
    }
    const int tiles = static_cast<int>(f0->tiles);
    k_symv_tiles<T, NJ><<<((tiles + 3) / 4) * js.n, 256, 0, s>>>(js, ny, tiles, conjop);
    RCP_HIP(hipGetLastError());
    k_symv_reduce<NJ><<<nt * js.n, 256, 0, s>>>(js, nt, ny);
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  };
  // the left chain's steps (and the middle block) use set g's partial-sum
  // area 0, the right chain's area 1
  auto P = [&](int g, int c) { return fs[g]->part[c]; };
  // forward sweeps; g_i is known zero while no source block has been passed
  std::vector<std::vector<char>> zero(B, std::vector<char>(N, 0));
  const int steps = lenL > lenR ? lenL : lenR;
  for (int st = 0; st < steps; ++st) {
    SvJobs js{};
    for (int g = 0; g < B; ++g) {
      std::vector<char>& z = zero[g];
      if (st < lenL) {
        int i = st;
        bool prevz = (i == 0) || z[i - 1];
        if (i < nz_lo[g] && prevz) {
          z[i] = 1;
        } else {
          js.j[js.n++] = SvJob{block_ptr(fs[g], i), U(g, i), nullptr, Fb(g, i),
                               prevz ? nullptr : U(g, i - 1), i > 0 ? C(g, i - 1) : nullptr,
                               nullptr, nullptr, P(g, 0)};
        }
      }
      if (st < lenR) {
        int i = N - 1 - st;
        bool prevz = (i == N - 1) || z[i + 1];
        if (i > nz_hi[g] && prevz) {
          z[i] = 1;
        } else {
          js.j[js.n++] = SvJob{block_ptr(fs[g], i), U(g, i), nullptr, Fb(g, i),
                               prevz ? nullptr : U(g, i + 1), i < N - 1 ? C(g, i) : nullptr,
                               nullptr, nullptr, P(g, 1)};
        }
      }
    }
    int rc = launch(js);
    if (rc) return rc;
  }
  {
    SvJobs js{};
    for (int g = 0; g < B; ++g) {
      SvJob z{block_ptr(fs[g], m), U(g, m), nullptr, Fb(g, m), nullptr, nullptr, nullptr, nullptr,
              P(g, 0)};
      if (m - 1 >= 0 && !zero[g][m - 1]) {
        z.v1 = U(g, m - 1);
        z.c1 = C(g, m - 1);
      }
      if (m + 1 < N && !zero[g][m + 1]) {
        z.v2 = U(g, m + 1);
        z.c2 = C(g, m);
      }
      js.j[js.n++] = z;
    }
    int rc = launch(js);
    if (rc) return rc;
  }
  for (int st = 0; st < steps; ++st) {
    SvJobs js{};
    for (int g = 0; g < B; ++g) {
      if (st < lenL) {
        int i = m - 1 - st;
        js.j[js.n++] = SvJob{block_ptr(fs[g], i), U(g, i), zero[g][i] ? nullptr : U(g, i), nullptr,
                             U(g, i + 1), C(g, i), nullptr, nullptr, P(g, 0)};
      }
      if (st < lenR) {
        int i = m + 1 + st;
        js.j[js.n++] = SvJob{block_ptr(fs[g], i), U(g, i), zero[g][i] ? nullptr : U(g, i), nullptr,
                             U(g, i - 1), C(g, i - 1), nullptr, nullptr, P(g, 1)};
      }
    }
    int rc = launch(js);
    if (rc) return rc;
  }
  return RCP_OK;
}

}  // namespace

namespace rcp {

int solve_vec_batch(rcp_factors* const* fs, int B, const double2* const* rhs, double2* const* u,
                    int conjop, const int* nz_lo, const int* nz_hi, hipStream_t s) {
  if (B < 1 || B > MAX_BATCH) return fail(RCP_EINVAL, "batch of 1 to 8 factor sets");
  const bool fp64 = fs[0]->precision == RCP_FP64;
  if (B == 1)
    return fp64 ? run_solve_vec<double, 2>(fs, B, rhs, u, conjop, nz_lo, nz_hi, s)
                : run_solve_vec<float, 2>(fs, B, rhs, u, conjop, nz_lo, nz_hi, s);
  return fp64 ? run_solve_vec<double, 2 * MAX_BATCH>(fs, B, rhs, u, conjop, nz_lo, nz_hi, s)
              : run_solve_vec<float, 2 * MAX_BATCH>(fs, B, rhs, u, conjop, nz_lo, nz_hi, s);
}

int solve_vec(rcp_factors* f, const double2* rhs, double2* u, int conjop, int nz_lo, int nz_hi,
              hipStream_t s) {
  return solve_vec_batch(&f, 1, &rhs, &u, conjop, &nz_lo, &nz_hi, s);
}

int block_products(rcp_factors* f, int count, const int* blocks, const double2* const* g,
                   const double2* const* base, double2* const* out, const int* part_area,
                   int conjop, hipStream_t s) {
  if (count < 1 || count > 2) return fail(RCP_EINVAL, "internal: one or two block products");
  if (f->precision != RCP_FP64) return fail(RCP_EINVAL, "internal: FP64 factors only");
  SvJobs<2> js{};
  for (int q = 0; q < count; ++q)
    js.j[js.n++] = SvJob{block_ptr(f, blocks[q]), out[q], base[q], g[q], nullptr, nullptr,
                         nullptr, nullptr, f->part[part_area[q]]};
  const int nt = f->nt, ny = f->ny;
  KTimer kt(K_GEMV, s, double(js.n) * f->tiles * TB * TB * sizeof(double2));
  if (nt <= GEMV_NT_MAX) {
    const dim3 grid(4 * nt * js.n);
    switch ((nt + 7) / 8) {
      case 1: k_gemv<double, 1, 2><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
      case 2: k_gemv<double, 2, 2><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
      default: k_gemv<double, 3, 2><<<grid, 512, 0, s>>>(js, nt, ny, conjop); break;
    }
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  }
  const int tiles = static_cast<int>(f->tiles);
  k_symv_tiles<double, 2><<<((tiles + 3) / 4) * js.n, 256, 0, s>>>(js, ny, tiles, conjop);
  RCP_HIP(hipGetLastError());
  k_symv_reduce<2><<<nt * js.n, 256, 0, s>>>(js, nt, ny);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int residual_norms(rcp_factors* f, const double2* b, const double2* x, double2* r, int conjop,
                   hipStream_t s, double* rnorm, double* bnorm) {
  size_t N = size_t(f->nx) * f->ny;
  int blocks = static_cast<int>((N + 255) / 256);
  // partial sums live in the reduction scratch after a 2-double result slot
  double* part = f->red + 2;
  k_residual<<<blocks, 256, 0, s>>>(f->nx, f->ny, f->dco, f->eco, f->cco, b, x, r, conjop, part);
  RCP_HIP(hipGetLastError());
  k_sum_pairs<<<1, 256, 0, s>>>(part, blocks, f->red);
  RCP_HIP(hipGetLastError());
  double h[2];
  RCP_HIP(hipMemcpyAsync(h, f->red, sizeof(h), hipMemcpyDeviceToHost, s));
  RCP_HIP(hipStreamSynchronize(s));
  *rnorm = std::sqrt(h[0]);
  *bnorm = std::sqrt(h[1]);
  return RCP_OK;
}

int solve_vec_refined(rcp_factors* f, const double2* rhs, double2* u, int conjop, int nz_lo,
                      int nz_hi, double tol, int max_refine, hipStream_t s, rcp_solve_stats* st) {
  int rc = solve_vec(f, rhs, u, conjop, nz_lo, nz_hi, s);
  if (rc) return rc;
  if (f->precision == RCP_FP64) {
    if (st) {
      double rn, bn;
      rc = residual_norms(f, rhs, u, nullptr, conjop, s, &rn, &bn);
      if (rc) return rc;
      st->iters = 0;
      st->rel_residual = bn > 0 ? rn / bn : 0.0;
    }
    return RCP_OK;
  }
  double2* r = f->vec[V_RES];
  double2* du = f->vec[V_DU];
  size_t N = size_t(f->nx) * f->ny;
  int it = 0;
  double rel = 0.0;
  for (;;) {
    double rn, bn;
    rc = residual_norms(f, rhs, u, r, conjop, s, &rn, &bn);
    if (rc) return rc;
    rel = bn > 0 ? rn / bn : 0.0;
    if (rel <= tol) break;
    if (it >= max_refine) {
      f->last_iters = it;
      f->last_residual = rel;
      if (st) {
        st->iters = it;
        st->rel_residual = rel;
      }
      return fail(RCP_ENOCONV, "refinement stopped after " + std::to_string(it) +
                                   " steps at relative residual " + std::to_string(rel));
    }
    rc = solve_vec(f, r, du, conjop, 0, f->nx - 1, s);
    if (rc) return rc;
    k_axpy<<<static_cast<int>((N + 255) / 256), 256, 0, s>>>(N, du, u);
    RCP_HIP(hipGetLastError());
    ++it;
  }
  f->last_iters = it;
  f->last_residual = rel;
  if (st) {
    st->iters = it;
    st->rel_residual = rel;
  }
  return RCP_OK;
}

// The brute force's sweep step as a library GEMM: the right-hand sides of job
// jb formed once (g = f + line source - C1 v1 - C2 v2, n x R column-major,
// leading dimension ny) and X_i unpacked from its packed symmetric tiles into a
// dense matrix (element (k, j) at k ny + j, as the tiled sweep reads it), then
// out = base + X^T g by rocBLAS ZGEMM (base = out or none).
__global__ __launch_bounds__(256) void k_form_rhs(MmJob jb, int R, int nx, int ny, size_t rstride,
                                                   int jline, int conjop, double2* __restrict__ G) {
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= size_t(R) * ny) return;
  const int r = static_cast<int>(t / ny), k = static_cast<int>(t % ny);
  const size_t q = size_t(r) * rstride + size_t(jb.block) * ny + k;
  double2 v = make_double2(0.0, 0.0);
  if (jb.f) v = jb.f[q];
  if (jb.fline && k == jline) v = cadd(v, jb.fline[size_t(r) * nx + jb.block]);
  if (jb.v1) v = csub(v, cmul(maybe_conj(jb.c1[k], conjop), jb.v1[q]));
  if (jb.v2) v = csub(v, cmul(maybe_conj(jb.c2[k], conjop), jb.v2[q]));
  G[t] = v;
}

__global__ __launch_bounds__(256) void k_unpack_sym(const double2* __restrict__ X, int ny, int conjop,
                                                     double2* __restrict__ Xd) {
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= size_t(ny) * ny) return;
  const int k = static_cast<int>(t / ny), j = static_cast<int>(t % ny);
  const int K = k / TB, J = j / TB;
  double2 x = K >= J ? X[tile_index(K, J) * TB * TB + (k % TB) * TB + (j % TB)]
                     : X[tile_index(J, K) * TB * TB + (j % TB) * TB + (k % TB)];
  if (conjop) x.y = -x.y;
  Xd[t] = x;
}

// One rocBLAS handle per device, made on first use (the library is not
// thread-safe per handle: calls take the lock).
constexpr int kMaxDevices = 64;
rocblas_handle g_blas[kMaxDevices] = {};
std::mutex g_blas_mu;

int library_step(const MmJobs& js, int R, int nx, int ny, size_t rstride, int jline, int conjop,
                 double2* ws, hipStream_t s) {
  int dev = 0;
  RCP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RCP_EINVAL, "device index out of range");
  double2* G = ws;
  double2* Xd = ws + align256(size_t(R) * ny * 16) / 16;
  std::lock_guard<std::mutex> lk(g_blas_mu);
  if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success)
    return fail(RCP_EHIP, "rocblas_create_handle failed");
  rocblas_handle h = g_blas[dev];
  if (rocblas_set_stream(h, s) != rocblas_status_success) return fail(RCP_EHIP, "rocblas_set_stream failed");
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  for (int q = 0; q < js.n; ++q) {
    const MmJob& jb = js.j[q];
    k_form_rhs<<<static_cast<int>((size_t(R) * ny + 255) / 256), 256, 0, s>>>(jb, R, nx, ny, rstride, jline,
                                                                             conjop, G);
    RCP_HIP(hipGetLastError());
    k_unpack_sym<<<static_cast<int>((size_t(ny) * ny + 255) / 256), 256, 0, s>>>(jb.X, ny, conjop, Xd);
    RCP_HIP(hipGetLastError());
    if (jb.base && jb.base != jb.out) return fail(RCP_EINVAL, "internal: a sweep base other than its output");
    rocblas_double_complex* C = reinterpret_cast<rocblas_double_complex*>(jb.out + size_t(jb.block) * ny);
    if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, ny, R, ny, &one,
                      reinterpret_cast<const rocblas_double_complex*>(Xd), ny,
                      reinterpret_cast<const rocblas_double_complex*>(G), ny, jb.base ? &one : &zero, C,
                      static_cast<rocblas_int>(rstride)) != rocblas_status_success)
      return fail(RCP_EHIP, "rocblas_zgemm failed");
  }
  return RCP_OK;
}

// How a sweep step's tiles are split (see k_gemm_sweep): the tiles beyond the
// last whole round over the CUs are cut into the number of k parts (at most
// 8, at most GEMM_SPLIT_TILES partial tiles in all) that gives the busiest CU
// the least work, ceil(rem * parts / cus) / parts tiles.
struct GemmSplit {
  int nwhole, nsplit;
};
// Workspace of library_step: the right-hand sides and the dense block.
size_t library_ws(int R, int ny) { return align256(size_t(R) * ny * 16) + size_t(ny) * ny * 16; }
GemmSplit gemm_split(int tiles, int nk, bool have_ws) {
  GemmSplit g{tiles, 1};
  if (!have_ws) return g;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return g;
  const int rem = tiles % cus;
  if (rem == 0) return g;
  int best = 1;
  double best_load = 1.0;
  for (int P = 2; P <= 8 && P <= nk && rem * P <= GEMM_SPLIT_TILES; ++P) {
    const double load = double(ceil_div(rem * P, cus)) / P;
    if (load < best_load - 1e-12) {
      best_load = load;
      best = P;
    }
  }
  if (best > 1) {
    g.nwhole = tiles - rem;
    g.nsplit = best;
  }
  return g;
}

int solve_multi_fp64(rcp_factors* f, int R, const double2* B, const double2* fline, int jline,
                     double2* Xo, int conjop, hipStream_t s, double2* split_ws) {
  const int N = f->nx, ny = f->ny, nt = f->nt, m = f->m;
  const size_t rs = size_t(N) * ny;
  const int lenL = m, lenR = N - 1 - m;
  auto O = [&](int i) { return Xo + size_t(i) * ny; };
  auto Bb = [&](int i) { return B ? B + size_t(i) * ny : nullptr; };
  auto C = [&](int i) { return f->cco + size_t(i) * ny; };
  const bool narrow = R < MT;   // 16 x 16 output tiles (k_mm_narrow)
  const int per_job = narrow ? ceil_div(R, 16) * 2 * nt : ceil_div(R, MT) * ceil_div(nt * TB, MT);
  auto launch = [&](MmJobs& js) -> int {
    if (js.n == 0) return RCP_OK;
    const double w = 8.0 * js.n * double(R) * ny * ny;
    if (narrow)
      RCP_HIP(klaunch(K_GEMM, w, k_mm_narrow, dim3(per_job * js.n), dim3(64 * MW_WAVES), s, js, R, N,
                      ny, nt, rs, jline, conjop));
    else if (split_ws && library_ws(R, ny) <= GEMM_SPLIT_BYTES &&
             rs <= size_t(std::numeric_limits<rocblas_int>::max())) {
      KTimer kt(K_GEMM, s, w);
      return library_step(js, R, N, ny, rs, jline, conjop, split_ws, s);
    } else {
      const int tiles = per_job * js.n;
      const GemmSplit g = gemm_split(tiles, nt * TB / KC, split_ws != nullptr);
      const int grid = g.nwhole + (tiles - g.nwhole) * g.nsplit;
      RCP_HIP(klaunch(K_GEMM, w, k_gemm_sweep, dim3(grid), dim3(256), s, js, R, N, ny, nt, rs, jline,
                      conjop, g.nwhole, g.nsplit, split_ws));
      if (g.nwhole < tiles) {
        k_gemm_fixup<<<tiles - g.nwhole, 256, 0, s>>>(js, R, ny, nt, rs, g.nwhole, g.nsplit, split_ws);
        RCP_HIP(hipGetLastError());
      }
    }
    return RCP_OK;
  };
  // job pointers address block i inside row 0; the kernel adds r * rstride
  auto job = [&](int i, double2* out, const double2* base, const double2* fb, const double2* v1,
                 const double2* c1, const double2* v2, const double2* c2) {
    MmJob j{};
    j.X = static_cast<const double2*>(block_ptr(f, i));
    j.out = out - size_t(i) * ny;       // kernel adds block offset
    j.base = base ? base - size_t(i) * ny : nullptr;
    j.f = fb ? fb - size_t(i) * ny : nullptr;
    j.fline = fline;
    j.v1 = v1 ? v1 - size_t(i) * ny : nullptr;
    j.c1 = c1;
    j.v2 = v2 ? v2 - size_t(i) * ny : nullptr;
    j.c2 = c2;
    j.block = i;
    return j;
  };
  const int steps = lenL > lenR ? lenL : lenR;
  for (int st = 0; st < steps; ++st) {
    MmJobs js{};
    if (st < lenL) {
      int i = st;
      js.j[js.n++] = job(i, O(i), nullptr, Bb(i), i > 0 ? O(i - 1) : nullptr,
                         i > 0 ? C(i - 1) : nullptr, nullptr, nullptr);
    }
    if (st < lenR) {
      int i = N - 1 - st;
      js.j[js.n++] = job(i, O(i), nullptr, Bb(i), i < N - 1 ? O(i + 1) : nullptr,
                         i < N - 1 ? C(i) : nullptr, nullptr, nullptr);
    }
    int rc = launch(js);
    if (rc) return rc;
  }
  {
    MmJobs js{};
    js.j[js.n++] = job(m, O(m), nullptr, Bb(m), m > 0 ? O(m - 1) : nullptr,
                       m > 0 ? C(m - 1) : nullptr, m + 1 < N ? O(m + 1) : nullptr,
                       m + 1 < N ? C(m) : nullptr);
    int rc = launch(js);
    if (rc) return rc;
  }
  for (int st = 0; st < steps; ++st) {
    MmJobs js{};
    if (st < lenL) {
      int i = m - 1 - st;
      MmJob j = job(i, O(i), O(i), nullptr, O(i + 1), C(i), nullptr, nullptr);
      j.fline = nullptr;
      js.j[js.n++] = j;
    }
    if (st < lenR) {
      int i = m + 1 + st;
      MmJob j = job(i, O(i), O(i), nullptr, O(i - 1), C(i - 1), nullptr, nullptr);
      j.fline = nullptr;
      js.j[js.n++] = j;
    }
    int rc = launch(js);
    if (rc) return rc;
  }
  return RCP_OK;
}

}  // namespace rcp

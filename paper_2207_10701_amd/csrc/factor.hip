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
// The nb x nb pivot blocks are inverted without pivoting (in FP64 for both
// storage precisions) and the smallest pivot modulus of every panel is
// recorded for the health check.
#include <cmath>
#include <vector>

#include "rcp_internal.h"

namespace {
using namespace rcp;

struct GJJob {
  int kind;      // 0: panel (P, L, Q), 1: trailing update
  int k;         // panel index
  int last;      // update: final panel, negate
  int wgs;       // workgroups of this job
  void* X;       // packed tiles of the block
  void* L;       // np x TB panel copy
  void* Q;       // np x TB  L P
  double2* P;    // TB x TB pivot-block inverse
  double* health;
};
struct GJJobs {
  GJJob j[4];
  int n;
};

__device__ __forceinline__ GJJob pick(const GJJobs& js, int* wg) {
  GJJob jb = js.j[0];
  int w = *wg;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q + 1 < js.n && w >= jb.wgs) {
      w -= jb.wgs;
      jb = js.j[q + 1];
    }
  }
  *wg = w;
  return jb;
}

// Panel step: every workgroup inverts the pivot block (FP64, in LDS), then each
// wave forms one row tile I of L (copied) and Q = L P.
template <typename T>
__device__ void panel_work(const GJJob& jb, int wg, int nt, double2 (*Ps)[TB + 1]) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  T2* X = static_cast<T2*>(jb.X);
  const int K = jb.k;
  const int tid = threadIdx.x;
  const T2* D = X + tile_index(K, K) * TB * TB;
  for (int e = tid; e < TB * TB; e += 256) Ps[e / TB][e % TB] = to_c128(D[e]);
  __syncthreads();

  // Gauss-Jordan inversion without pivoting; thread owns row r, columns c0..c0+3.
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  double minpiv = INFINITY;
  for (int p = 0; p < TB; ++p) {
    double2 piv = Ps[p][p];
    double2 ip = cinv(piv);
    double2 fr = Ps[r][p];
    double2 prow[4], mine[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      prow[c] = Ps[p][c0 + c];
      mine[c] = Ps[r][c0 + c];
    }
    double a = sqrt(cabs2(piv));
    minpiv = (a < minpiv || a != a) ? a : minpiv;
    __syncthreads();
    if (r == p) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Ps[p][c0 + c] = (c0 + c == p) ? ip : cmul(prow[c], ip);
    } else {
      double2 fi = cmul(fr, ip);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        Ps[r][c0 + c] = (c0 + c == p) ? make_double2(-fi.x, -fi.y) : csub(mine[c], cmul(fi, prow[c]));
    }
    __syncthreads();
  }
  if (wg == 0) {
    for (int e = tid; e < TB * TB; e += 256) jb.P[e] = Ps[e / TB][e % TB];
    if (tid == 0) *jb.health = minpiv;
  }

  const int wave = tid >> 6, lane = tid & 63;
  const int I = wg * 4 + wave;
  if (I >= nt || I == K) return;
  const int lr = lane & 15, lk = lane >> 4;
  const T2* src = (I >= K) ? X + tile_index(I, K) * TB * TB : X + tile_index(K, I) * TB * TB;
  const bool trans = I < K;
  T2 af[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int rr = 16 * a + lr, kk = 4 * s + lk;
      af[a][s] = trans ? src[kk * TB + rr] : src[rr * TB + kk];
    }
  T2* Lb = static_cast<T2*>(jb.L) + size_t(I) * TB * TB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int s = 0; s < 8; ++s) Lb[(16 * a + lr) * TB + 4 * s + lk] = af[a][s];

  V4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = V4{0, 0, 0, 0};
      cim[a][b] = V4{0, 0, 0, 0};
    }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    T bre[2], bim[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      double2 pv = Ps[4 * s + lk][16 * b + lr];
      bre[b] = static_cast<T>(pv.x);
      bim[b] = static_cast<T>(pv.y);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      T are = af[a][s].x, aim = af[a][s].y, naim = -aim;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(are, bre[b], cre[a][b]);
        cre[a][b] = mfma16(naim, bim[b], cre[a][b]);
        cim[a][b] = mfma16(are, bim[b], cim[a][b]);
        cim[a][b] = mfma16(aim, bre[b], cim[a][b]);
      }
    }
  }
  T2* Qb = static_cast<T2*>(jb.Q) + size_t(I) * TB * TB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = cre[a][b][q];
        v.y = cim[a][b][q];
        Qb[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr] = v;
      }
}

// Trailing update: one wave per packed tile.
template <typename T>
__device__ void update_work(const GJJob& jb, int wg, size_t tiles) {
  using T2 = typename cplx<T>::t;
  using V4 = typename v4of<T>::t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const size_t t = size_t(wg) * 4 + wave;
  if (t >= tiles) return;
  int I, J;
  tile_coords(static_cast<int>(t), &I, &J);
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
  V4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v = dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr];
        cre[a][b][q] = v.x;
        cim[a][b][q] = v.y;
      }
  const T2* QI = Q + size_t(I) * TB * TB;
  const T2* LJ = L + size_t(J) * TB * TB;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    T2 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = QI[(16 * a + lr) * TB + 4 * s + lk];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = LJ[(16 * b + lr) * TB + 4 * s + lk];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      T nare = -av[a].x, aim = av[a].y, naim = -av[a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cre[a][b] = mfma16(nare, bv[b].x, cre[a][b]);
        cre[a][b] = mfma16(aim, bv[b].y, cre[a][b]);
        cim[a][b] = mfma16(nare, bv[b].y, cim[a][b]);
        cim[a][b] = mfma16(naim, bv[b].x, cim[a][b]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T2 v;
        v.x = cre[a][b][q] * sg;
        v.y = cim[a][b][q] * sg;
        dst[(16 * a + mfma_row<T>(lk, q)) * TB + 16 * b + lr] = v;
      }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gj(GJJobs jobs, int nt, size_t tiles) {
  __shared__ double2 Ps[TB][TB + 1];
  int wg = blockIdx.x;
  GJJob jb = pick(jobs, &wg);
  if (jb.kind == 0)
    panel_work<T>(jb, wg, nt, Ps);
  else
    update_work<T>(jb, wg, tiles);
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
  SchurJob j[2];
  int n;
};

template <typename T>
__global__ __launch_bounds__(256) void k_schur(SchurJobs jobs, int ny, size_t tiles) {
  using T2 = typename cplx<T>::t;
  const size_t t = blockIdx.x % tiles;
  const int ji = static_cast<int>(blockIdx.x / tiles);
  SchurJob jb = jobs.j[0];
  if (ji == 1) jb = jobs.j[1];
  int I, J;
  tile_coords(static_cast<int>(t), &I, &J);
  T2* dst = static_cast<T2*>(jb.dst) + t * TB * TB;
  const T2* s1 = jb.src1 ? static_cast<const T2*>(jb.src1) + t * TB * TB : nullptr;
  const T2* s2 = jb.src2 ? static_cast<const T2*>(jb.src2) + t * TB * TB : nullptr;
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    int a = I * TB + e / TB, b = J * TB + e % TB;
    double2 v = make_double2(0.0, 0.0);
    if (a == b) {
      v = (a < ny) ? jb.dco[a] : make_double2(1.0, 0.0);
    } else if (a == b + 1 && a < ny) {
      v = jb.eco[b];
    } else if (b == a + 1 && b < ny) {
      v = jb.eco[a];
    }
    if (a < ny && b < ny) {
      if (s1) v = csub(v, cmul(cmul(jb.c1[a], jb.c1[b]), to_c128(s1[e])));
      if (s2) v = csub(v, cmul(cmul(jb.c2[a], jb.c2[b]), to_c128(s2[e])));
    }
    dst[e] = from_c128<T2>(v);
  }
}

template <typename T>
int run_factor(rcp_factors* f, hipStream_t s) {
  const int N = f->nx, ny = f->ny, nt = f->nt, m = f->m;
  const size_t tiles = f->tiles;
  const int lenL = m, lenR = N - 1 - m;
  auto D = [&](int i) { return f->dco + size_t(i) * ny; };
  auto E = [&](int i) { return f->eco + size_t(i) * ny; };
  auto C = [&](int i) { return f->cco + size_t(i) * ny; };

  auto schur = [&](SchurJobs js) -> int {
    if (js.n == 0) return RCP_OK;
    k_schur<T><<<static_cast<int>(tiles * js.n), 256, 0, s>>>(js, ny, tiles);
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  };
  const int upd_wgs = static_cast<int>((tiles + 3) / 4);
  const int pan_wgs = ceil_div(nt, 4);
  // sweep the blocks of up to two chains through all panels
  auto sweep = [&](int nb, const int* blocks) -> int {
    for (int k = 0; k < nt; ++k) {
      GJJobs pj{}, uj{};
      int gp = 0, gu = 0;
      for (int c = 0; c < nb; ++c) {
        GJJob b{};
        b.kind = 0;
        b.k = k;
        b.wgs = pan_wgs;
        b.X = block_ptr(f, blocks[c]);
        b.L = f->wsL[c];
        b.Q = f->wsQ[c];
        b.P = f->wsP[c];
        b.health = f->health + size_t(blocks[c]) * nt + k;
        pj.j[pj.n++] = b;
        gp += pan_wgs;
        GJJob u = b;
        u.kind = 1;
        u.last = (k == nt - 1);
        u.wgs = upd_wgs;
        uj.j[uj.n++] = u;
        gu += upd_wgs;
      }
      k_gj<T><<<gp, 256, 0, s>>>(pj, nt, tiles);
      RCP_HIP(hipGetLastError());
      k_gj<T><<<gu, 256, 0, s>>>(uj, nt, tiles);
      RCP_HIP(hipGetLastError());
    }
    return RCP_OK;
  };

  // chain heads
  {
    SchurJobs js{};
    if (lenL > 0) js.j[js.n++] = SchurJob{block_ptr(f, 0), nullptr, nullptr, D(0), E(0), nullptr, nullptr};
    if (lenR > 0)
      js.j[js.n++] = SchurJob{block_ptr(f, N - 1), nullptr, nullptr, D(N - 1), E(N - 1), nullptr, nullptr};
    int rc = schur(js);
    if (rc) return rc;
  }
  const int steps = lenL > lenR ? lenL : lenR;
  for (int st = 0; st < steps; ++st) {
    int blocks[2], nb = 0;
    int bL = st < lenL ? st : -1, bR = st < lenR ? N - 1 - st : -1;
    if (bL >= 0) blocks[nb++] = bL;
    if (bR >= 0) blocks[nb++] = bR;
    int rc = sweep(nb, blocks);
    if (rc) return rc;
    SchurJobs js{};
    if (bL >= 0 && bL + 1 < m)
      js.j[js.n++] = SchurJob{block_ptr(f, bL + 1), block_ptr(f, bL), nullptr, D(bL + 1), E(bL + 1),
                              C(bL), nullptr};
    if (bR >= 0 && bR - 1 > m)
      js.j[js.n++] = SchurJob{block_ptr(f, bR - 1), block_ptr(f, bR), nullptr, D(bR - 1), E(bR - 1),
                              C(bR - 1), nullptr};
    rc = schur(js);
    if (rc) return rc;
  }
  // middle block
  {
    SchurJobs js{};
    SchurJob z{block_ptr(f, m), nullptr, nullptr, D(m), E(m), nullptr, nullptr};
    if (m - 1 >= 0) {
      z.src1 = block_ptr(f, m - 1);
      z.c1 = C(m - 1);
    }
    if (m + 1 < N) {
      z.src2 = block_ptr(f, m + 1);
      z.c2 = C(m);
    }
    js.j[js.n++] = z;
    int rc = schur(js);
    if (rc) return rc;
    int blocks[1] = {m};
    rc = sweep(1, blocks);
    if (rc) return rc;
  }
  return RCP_OK;
}

}  // namespace

namespace rcp {

int factor_blocks(rcp_factors* f, hipStream_t s) {
  int rc = (f->precision == RCP_FP64) ? run_factor<double>(f, s) : run_factor<float>(f, s);
  if (rc) return rc;
  // pivot health: one wait, then scan the smallest pivot modulus of every panel
  const size_t nh = size_t(f->nx) * f->nt;
  std::vector<double> h(nh);
  RCP_HIP(hipMemcpyAsync(h.data(), f->health, nh * sizeof(double), hipMemcpyDeviceToHost, s));
  RCP_HIP(hipStreamSynchronize(s));
  // diagonal entries are O(4/h^2); a pivot below 1e-13 of that scale is treated as singular
  const double tiny = 1e-13 * 4.0 / (f->h * f->h);
  for (size_t q = 0; q < nh; ++q) {
    if (!(h[q] > tiny) || !std::isfinite(h[q])) {
      return fail(RCP_ESINGULAR, "pivot block " + std::to_string(q % f->nt) + " of column block " +
                                     std::to_string(q / f->nt) + " has pivot modulus " +
                                     std::to_string(h[q]));
    }
  }
  return RCP_OK;
}

}  // namespace rcp

// Eq. 7 for any current correlation W and for several outputs on the same
// factors, and the correlation of a finite ensemble of correlated planewaves.
//
// Sec. "Incoherent light" notes that the reciprocal technique holds for
// arbitrarily correlated light: then W is a dense Hermitian M x M matrix on the
// incidence line and v^dag W v needs the product W v.  With K outputs w_k
// (focal spots or output modes; Sec. "Concluding remarks" on averages over
// many spots or modes) the K reciprocal fields v_k share the factors and the
// products are one complex matrix product Y = W V (M x M by M x K) on the
// matrix cores.  The ensemble correlation of Eq. 1 and 3, written as sums over
// a finite set of planewaves b0(theta_q) with amplitude correlation
// C_qq' = <a_q conj(a_q')>, is W = G C G^dag with G_jq = b0(theta_q)(x_j): two
// more products of the same kind.
//
// All three products have the form out[n][m] = sum_l A[m][l] opB(B[n][l])
// with both operands contiguous along the contraction index l, so each lane
// loads four consecutive complex values of one row per step.
#include <cmath>

#include "rcp_internal.h"

namespace {
using namespace rcp;

constexpr int ZG_ROWS = 64;   // rows m per workgroup: four waves of 16
constexpr int ZG_TARGET_WGS = 1024;

// Complex FP64 product on MFMA 16x16x4: one wave owns 16 rows m and 16 * NCB
// columns n.  Lane (c16 = lane % 16, g = lane / 16) supplies, at step s of a
// 16-wide chunk of l, A[m0 + c16][l0 + 4 g + s] as MFMA operand A[c16][g] and
// B[n + c16][l0 + 4 g + s] as operand B[g][c16]: the same l for the same
// k-index g, so the sum over g and s covers the chunk.  Real and imaginary parts
// take four real products.  Workgroup z sums l in [z Ls, (z + 1) Ls) and writes
// its partial product to out + z * split_stride.
template <int NCB, bool CONJB>
__global__ __launch_bounds__(256) void k_zgemm_nt(const double2* __restrict__ A, int lda,
                                                  const double2* __restrict__ B, int ldb,
                                                  double2* __restrict__ out, int ldo,
                                                  size_t split_stride, int Md, int Nd, int L,
                                                  int Ls) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.x * ZG_ROWS + wave * 16;
  const int n0 = blockIdx.y * (16 * NCB);
  const int lb = blockIdx.z * Ls;
  const int le = min(L, lb + Ls);
  const int am = m0 + c16;
  const bool aok = am < Md;
  const double2* Ap = A + size_t(aok ? am : 0) * lda;
  const double2* Bp[NCB];
  bool bok[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int bn = n0 + cb * 16 + c16;
    bok[cb] = bn < Nd;
    Bp[cb] = B + size_t(bok[cb] ? bn : 0) * ldb;
  }
  v4d ar[NCB], ai[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) ar[cb][r] = ai[cb][r] = 0.0;
  const double2 zero = make_double2(0.0, 0.0);
  for (int l0 = lb; l0 < le; l0 += 16) {
    const int l = l0 + 4 * g;
    // loads from in-range addresses only (index clamped), values outside
    // the matrix replaced by zero afterwards
    double2 a[4], b[NCB][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool lok = l + s < le;
      const int lc = lok ? l + s : le - 1;
      const double2 t = Ap[lc];
      a[s] = (aok && lok) ? t : zero;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const double2 u = Bp[cb][lc];
        b[cb][s] = (bok[cb] && lok) ? u : zero;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const double bx = b[cb][s].x, by = CONJB ? -b[cb][s].y : b[cb][s].y;
        ar[cb] = mfma16(a[s].x, bx, ar[cb]);
        ar[cb] = mfma16(-a[s].y, by, ar[cb]);
        ai[cb] = mfma16(a[s].x, by, ai[cb]);
        ai[cb] = mfma16(a[s].y, bx, ai[cb]);
      }
    }
  }
  double2* o = out + size_t(blockIdx.z) * split_stride;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int n = n0 + cb * 16 + c16;
    if (n >= Nd) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + mfma_row<double>(g, r);
      if (m < Md) o[size_t(n) * ldo + m] = make_double2(ar[cb][r], ai[cb][r]);
    }
  }
}

// out[q] = sum over splits of part[s * stride + q], in split order
__global__ void k_split_sum(const double2* __restrict__ part, size_t stride, int S, size_t n,
                            double2* __restrict__ out) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double2 acc = part[q];
  for (int s = 1; s < S; ++s) acc = cadd(acc, part[size_t(s) * stride + q]);
  out[q] = acc;
}

// G[j][q] = b0(theta_q) at line cell j: (2 i k0 sqrt(n cos th) / h) e^{i n k0 sin th x_j}
__global__ void k_source_matrix(const double* __restrict__ theta, int N, int M, int i0, int npml,
                                double h, double n, double k0, double2* __restrict__ G) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(M) * N) return;
  const int j = static_cast<int>(q / N), a = static_cast<int>(q % N);
  const double th = theta[a];
  const double amp = 2.0 * k0 * sqrt(n * cos(th)) / h;
  const double x = (i0 + j - npml + 0.5) * h;
  double sn, cs;
  sincos(n * k0 * sin(th) * x, &sn, &cs);
  G[q] = make_double2(-amp * sn, amp * cs);
}

// Vt[k][j] = z_k on the incidence line; rows K..Kp-1 zero
__global__ void k_gather_lines(const double2* __restrict__ Z, size_t N, int ny, int js, int i0,
                               int M, int K, int Kp, double2* __restrict__ Vt) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(Kp) * M) return;
  const int k = static_cast<int>(q / M), j = static_cast<int>(q % M);
  Vt[q] = k < K ? Z[size_t(k) * N + size_t(i0 + j) * ny + js] : make_double2(0.0, 0.0);
}

// Y[k][m] = sum of the split partial products; red[k][mb] = Re sum_m conj(v) y
// over the 256 rows of block mb (fixed-order tree)
__global__ __launch_bounds__(256) void k_dense_reduce(const double2* __restrict__ part,
                                                      size_t stride, int S,
                                                      const double2* __restrict__ Vt,
                                                      double2* __restrict__ Y, int M,
                                                      double* __restrict__ red, int nmb) {
  __shared__ double sh[256];
  const int k = blockIdx.y, m = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (m < M) {
    const size_t q = size_t(k) * M + m;
    double2 y = part[q];
    for (int s = 1; s < S; ++s) y = cadd(y, part[size_t(s) * stride + q]);
    Y[q] = y;
    const double2 v = Vt[q];
    acc = v.x * y.x + v.y * y.y;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[size_t(k) * nmb + blockIdx.x] = sh[0];
}

// F[k] = sum_mb red[k][mb]; F[K] = sum_k F[k] (fixed order)
__global__ __launch_bounds__(256) void k_dense_final(const double* __restrict__ red, int nmb,
                                                     int K, double* __restrict__ F) {
  __shared__ double sh[256];
  double tot = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) {
    double a = 0.0;
    for (int b = 0; b < nmb; ++b) a += red[size_t(k) * nmb + b];
    F[k] = a;
    tot += a;
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) F[K] = sh[0];
}

// line sources of the adjoint solves: fline[k][i] = Y[k][i - i0] on [i0, i0 + M)
__global__ void k_scatter_lines(const double2* __restrict__ Y, int M, int K, int nx, int i0,
                                double2* __restrict__ fline) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(K) * nx) return;
  const int k = static_cast<int>(q / nx), i = static_cast<int>(q % nx);
  fline[q] = (i >= i0 && i < i0 + M) ? Y[size_t(k) * M + (i - i0)] : make_double2(0.0, 0.0);
}

// dF/deps_q = -2 k0^2 Re(conj(sx sy)_q sum_k conj(lambda_kq) z_kq)
__global__ void k_grad_eps_many(int nx, int ny, int K, double k0, const double2* __restrict__ sxc,
                                const double2* __restrict__ syc, const double2* __restrict__ lam,
                                const double2* __restrict__ z, double* __restrict__ g) {
  const size_t N = size_t(nx) * ny;
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const int i = static_cast<int>(q / ny), j = static_cast<int>(q % ny);
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < K; ++k) acc = cadd(acc, cmul(cconj(lam[size_t(k) * N + q]), z[size_t(k) * N + q]));
  const double2 t = cmul(cconj(cmul(sxc[i], syc[j])), acc);
  g[q] = -2.0 * k0 * k0 * t.x;
}

int blocks_of(size_t n) { return static_cast<int>((n + 255) / 256); }

}  // namespace

namespace rcp {

int zgemm_cols_per_wave(int Nd) { return Nd <= 16 ? 1 : (Nd <= 32 ? 2 : 4); }

ZSplit zgemm_split(int Md, int Nd, int L) {
  const int tiles = ceil_div(Md, ZG_ROWS) * ceil_div(Nd, 16 * zgemm_cols_per_wave(Nd));
  int S = ceil_div(ZG_TARGET_WGS, tiles);
  const int maxS = ceil_div(L, 64);   // at least 64 values of l per split
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  ZSplit sp;
  sp.Ls = ceil_div(ceil_div(L, S), 16) * 16;
  sp.S = ceil_div(L, sp.Ls);
  return sp;
}

int zgemm_nt(const double2* A, int lda, const double2* B, int ldb, bool conjb, double2* out,
             int ldo, size_t split_stride, int Md, int Nd, int L, ZSplit sp, hipStream_t s,
             int Nd_used) {
  const int ncb = zgemm_cols_per_wave(Nd);
  dim3 grid(ceil_div(Md, ZG_ROWS), ceil_div(Nd, 16 * ncb), sp.S);
  if (grid.y > 65535 || grid.z > 65535) return fail(RCP_EINVAL, "matrix product too large");
  KTimer kt(K_ZGEMM, s, 8.0 * double(Md) * (Nd_used > 0 ? Nd_used : Nd) * L);
#define RCP_ZG(NC, CJ)                                                                      \
  k_zgemm_nt<NC, CJ><<<grid, 256, 0, s>>>(A, lda, B, ldb, out, ldo, split_stride, Md, Nd, L, \
                                          sp.Ls)
  if (ncb == 1)
    conjb ? RCP_ZG(1, true) : RCP_ZG(1, false);
  else if (ncb == 2)
    conjb ? RCP_ZG(2, true) : RCP_ZG(2, false);
  else
    conjb ? RCP_ZG(4, true) : RCP_ZG(4, false);
#undef RCP_ZG
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

// out (Nd x Md, row stride Md) = sum_l A[m][l] opB(B[n][l]); part holds
// sp.S * Nd * Md partial products when sp.S > 1.
static int zgemm_full(const double2* A, const double2* B, bool conjb, double2* out, double2* part,
                      int Md, int Nd, int L, hipStream_t s) {
  ZSplit sp = zgemm_split(Md, Nd, L);
  const size_t n = size_t(Nd) * Md;
  if (sp.S == 1) return zgemm_nt(A, L, B, L, conjb, out, Md, 0, Md, Nd, L, sp, s);
  int rc = zgemm_nt(A, L, B, L, conjb, part, Md, n, Md, Nd, L, sp, s);
  if (rc) return rc;
  k_split_sum<<<blocks_of(n), 256, 0, s>>>(part, n, sp.S, n, out);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

DenseLayout dense_layout(int nx, int ny, int K, int M) {
  DenseLayout D{};
  D.Kp = ceil_div(K, 16) * 16;
  D.sp = zgemm_split(M, D.Kp, M);
  D.nmb = ceil_div(M, 256);
  const size_t N = size_t(nx) * ny;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  D.off_B = take(size_t(K) * N * 16);
  D.off_Z = take(size_t(K) * N * 16);
  D.off_Vt = take(size_t(D.Kp) * M * 16);
  D.off_Y = take(size_t(D.Kp) * M * 16);
  D.off_part = take(size_t(D.sp.S) * D.Kp * M * 16);
  D.off_red = take(size_t(K) * D.nmb * 8);
  D.off_fline = take(size_t(K) * nx * 16);
  D.total = o;
  return D;
}

int gather_lines(const double2* Z, size_t N, int ny, int js, int i0, int M, int K, int Kp,
                 double2* Vt, hipStream_t s) {
  k_gather_lines<<<blocks_of(size_t(Kp) * M), 256, 0, s>>>(Z, N, ny, js, i0, M, K, Kp, Vt);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int dense_form(const double2* W, int M, const double2* Vt, int K, const DenseLayout& D,
               double2* part, double2* Y, double* red, double* F, hipStream_t s) {
  const size_t stride = size_t(D.Kp) * M;
  int rc = zgemm_nt(W, M, Vt, M, false, part, M, stride, M, D.Kp, M, D.sp, s, K);
  if (rc) return rc;
  dim3 grid(D.nmb, K);
  k_dense_reduce<<<grid, 256, 0, s>>>(part, stride, D.sp.S, Vt, Y, M, red, D.nmb);
  RCP_HIP(hipGetLastError());
  k_dense_final<<<1, 256, 0, s>>>(red, D.nmb, K, F);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int scatter_lines(const double2* Y, int M, int K, int nx, int i0, double2* fline, hipStream_t s) {
  k_scatter_lines<<<blocks_of(size_t(K) * nx), 256, 0, s>>>(Y, M, K, nx, i0, fline);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int grad_eps_many(rcp_factors* f, int K, const double2* lam, const double2* z, double* grad,
                  hipStream_t s) {
  k_grad_eps_many<<<blocks_of(size_t(f->nx) * f->ny), 256, 0, s>>>(f->nx, f->ny, K, f->k0, f->sxc,
                                                                   f->syc, lam, z, grad);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

CorrLayout corr_layout(int M, int N) {
  CorrLayout Lc{};
  const ZSplit s1 = zgemm_split(N, M, N), s2 = zgemm_split(M, M, N);
  size_t part = 0;
  if (s1.S > 1) part = size_t(s1.S) * M * N * 16;
  if (s2.S > 1 && size_t(s2.S) * M * M * 16 > part) part = size_t(s2.S) * M * M * 16;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  Lc.off_G = take(size_t(M) * N * 16);
  Lc.off_S = take(size_t(M) * N * 16);
  Lc.off_part = take(part);
  Lc.total = o;
  return Lc;
}

// W = G C G^dag: S[l][q] = sum_q' C[q][q'] conj(G[l][q']), W[j][l] = sum_q G[j][q] S[l][q]
int correlation_matrix(int M, int N, int i0, int npml, double h, double n_s, double k0,
                       const double* theta, const double2* Cq, double2* W, char* work,
                       hipStream_t s) {
  CorrLayout Lc = corr_layout(M, N);
  double2* G = reinterpret_cast<double2*>(work + Lc.off_G);
  double2* S = reinterpret_cast<double2*>(work + Lc.off_S);
  double2* part = reinterpret_cast<double2*>(work + Lc.off_part);
  k_source_matrix<<<blocks_of(size_t(M) * N), 256, 0, s>>>(theta, N, M, i0, npml, h, n_s, k0, G);
  RCP_HIP(hipGetLastError());
  int rc = zgemm_full(Cq, G, true, S, part, N, M, N, s);
  if (rc) return rc;
  return zgemm_full(S, G, false, W, part, M, M, N, s);
}

}  // namespace rcp

// The quadratic form of Eq. 7 on the incidence line, its gradient, and the
// sources and reductions of the brute-force average of Eq. 6.
//
// Sec. "Reciprocal approach": with translation-invariant correlations
// W(x1, x2) = C(x1 - x2), so v^dag W v is a Toeplitz quadratic form; W v is a
// convolution, computed here by embedding the Toeplitz matrix in a circulant
// of power-of-two size P >= 2M - 1 and applying it with FFTs.
//
// Correlation of the unit-power equivalent currents (Sec. "Incoherent light",
// Eq. 3-4 and the annulus formula of Sec. "Designs"; the current of a
// unit-power planewave is J = -2 i k0 sqrt(n cos theta) over one cell height,
// and sigma = sin(theta) turns the cos(theta) weight into the Jacobian):
//   cone     C(d) = (4 k0^2 n / h^2) (sin c / c) sinc(K d sin c)
//   annulus  C(d) = (4 k0^2 n / h^2) [sin th2 sinc(K d sin th2)
//                                    - sin th1 sinc(K d sin th1)] / (th2 - th1)
// with K = n k0 and sinc z = sin z / z.
#include <cmath>

#include "rcp_internal.h"

namespace {
using namespace rcp;

__device__ double sinc_(double z) {
  double a = fabs(z);
  if (a < 1e-4) return 1.0 - z * z / 6.0 + z * z * z * z / 120.0;
  return sin(z) / z;
}

__device__ double2 symbol_value(int kind, double c, double th1, double th2, double n, double k0,
                                double h, const double2* table, int M, int m) {
  if (kind == RCP_SYMBOL_TABLE) return table[m + M - 1];
  double d = m * h;
  double K = n * k0;
  double pref = 4.0 * k0 * k0 * n / (h * h);
  if (kind == RCP_CONE) return make_double2(pref * (sin(c) / c) * sinc_(K * d * sin(c)), 0.0);
  double s1 = sin(th1), s2 = sin(th2);
  return make_double2(pref * (s2 * sinc_(K * d * s2) - s1 * sinc_(K * d * s1)) / (th2 - th1), 0.0);
}

__global__ void k_fill_zero(double2* p, size_t n) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) p[q] = make_double2(0.0, 0.0);
}

__global__ void k_set(double2* p, size_t idx, double2 v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[idx] = v;
}

// collimator objective on row jm: w_i = (h / L) exp(i k0 n_m sin(phi) x_i)
__global__ void k_mode_row(double2* w, int ny, int jm, int i0, int M, int npml, double h,
                           double kx) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int i = i0 + m;
  double x = (i - npml + 0.5) * h;
  double L = M * h;
  double sn, cs;
  sincos(kx * x, &sn, &cs);
  w[size_t(i) * ny + jm] = make_double2(cs * h / L, sn * h / L);
}

// circulant embedding of the Toeplitz symbol
__global__ void k_symbol_circ(double2* circ, int P, int M, int kind, double c, double th1,
                              double th2, double n, double k0, double h, const double2* table) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double2 v = make_double2(0.0, 0.0);
  if (p < M)
    v = symbol_value(kind, c, th1, th2, n, k0, h, table, M, p);
  else if (p > P - M)
    v = symbol_value(kind, c, th1, th2, n, k0, h, table, M, p - P);
  circ[p] = v;
}

// v = z on the incidence line, zero-padded to P
__global__ void k_gather_pad(const double2* z, int ny, int js, int i0, int M, int P, double2* buf,
                             double2* v_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double2 v = make_double2(0.0, 0.0);
  if (p < M) {
    v = z[size_t(i0 + p) * ny + js];
    if (v_out) v_out[p] = v;
  }
  buf[p] = v;
}

__device__ __forceinline__ unsigned bitrev(unsigned x, int bits) {
  return __brev(x) >> (32 - bits);
}

// whole transform in LDS, P <= 4096: bit-reversed load, radix-2 DIT stages
__global__ __launch_bounds__(1024) void k_fft_lds(double2* buf, int P, int logP, double sign) {
  __shared__ double2 a[4096];
  for (int p = threadIdx.x; p < P; p += 1024) a[bitrev(p, logP)] = buf[p];
  __syncthreads();
  for (int half = 1; half < P; half <<= 1) {
    for (int b = threadIdx.x; b < P / 2; b += 1024) {
      int pos = b & (half - 1);
      int i = ((b - pos) << 1) + pos;
      int j = i + half;
      double sn, cs;
      sincospi(sign * static_cast<double>(pos) / half, &sn, &cs);
      double2 w = make_double2(cs, sn);
      double2 t = cmul(w, a[j]);
      double2 u = a[i];
      a[i] = cadd(u, t);
      a[j] = csub(u, t);
    }
    __syncthreads();
  }
  for (int p = threadIdx.x; p < P; p += 1024) buf[p] = a[p];
}

__global__ void k_bitrev_copy(const double2* in, double2* out, int P, int logP) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) out[bitrev(p, logP)] = in[p];
}

__global__ void k_fft_stage(double2* a, int P, int half, double sign) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= P / 2) return;
  int pos = b & (half - 1);
  int i = ((b - pos) << 1) + pos;
  int j = i + half;
  double sn, cs;
  sincospi(sign * static_cast<double>(pos) / half, &sn, &cs);
  double2 t = cmul(make_double2(cs, sn), a[j]);
  double2 u = a[i];
  a[i] = cadd(u, t);
  a[j] = csub(u, t);
}

__global__ void k_pointwise(double2* a, const double2* b, int P) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) a[p] = cmul(a[p], b[p]);
}

// Tv = buf[0..M) / P, F = Re sum conj(v) Tv (fixed-order reduction, one block)
__global__ __launch_bounds__(1024) void k_form_dot(const double2* buf, const double2* vpad, int M,
                                                   int P, double2* Tv, double* F) {
  __shared__ double s[1024];
  double acc = 0.0;
  double ip = 1.0 / P;
  for (int p = threadIdx.x; p < M; p += 1024) {
    double2 t = cscale(buf[p], ip);
    if (Tv) Tv[p] = t;
    double2 v = vpad[p];
    acc += v.x * t.x + v.y * t.y;   // Re(conj(v) t)
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *F = s[0];
}

__global__ void k_scatter_line(const double2* Tv, int ny, int js, int i0, int M, double2* rhs) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < M) rhs[size_t(i0 + p) * ny + js] = Tv[p];
}

// dF/deps_q = -2 k0^2 Re(conj(lambda_q) conj(sx sy)_q z_q)
__global__ void k_grad_eps(int nx, int ny, double k0, const double2* __restrict__ sxc,
                           const double2* __restrict__ syc, const double2* __restrict__ lam,
                           const double2* __restrict__ z, double* __restrict__ g) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(nx) * ny) return;
  int i = static_cast<int>(q / ny), j = static_cast<int>(q % ny);
  double2 s = cconj(cmul(sxc[i], syc[j]));
  double2 t = cmul(cmul(cconj(lam[q]), s), z[q]);
  g[q] = -2.0 * k0 * k0 * t.x;
}

// line sources of the brute force: b0(theta) = (2 i k0 sqrt(n cos th) / h) e^{i K sin th x}
__global__ void k_planewave_lines(const double* __restrict__ theta, int R, int nx, int i0, int i1,
                                  int npml, double h, double n, double k0,
                                  double2* __restrict__ fline) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(R) * nx) return;
  int r = static_cast<int>(q / nx), i = static_cast<int>(q % nx);
  double2 v = make_double2(0.0, 0.0);
  if (i >= i0 && i < i1) {
    double th = theta[r];
    double amp = 2.0 * k0 * sqrt(n * cos(th)) / h;
    double x = (i - npml + 0.5) * h;
    double sn, cs;
    sincos(n * k0 * sin(th) * x, &sn, &cs);
    v = cmul(make_double2(0.0, amp), make_double2(cs, sn));
  }
  fline[q] = v;
}

// |w^dag u_r|^2 per right-hand side r (one workgroup each)
__global__ __launch_bounds__(256) void k_bf_amp(const double2* __restrict__ U, size_t rstride,
                                                int ny, int kind, int fi, int fj, int jm, int i0,
                                                int M, int npml, double h, double kx,
                                                double* __restrict__ pa, int r0) {
  __shared__ double sre[256], sim[256];
  int r = blockIdx.x;
  const double2* u = U + size_t(r) * rstride;
  double2 acc = make_double2(0.0, 0.0);
  if (kind == RCP_CONCENTRATOR) {
    if (threadIdx.x == 0) acc = u[size_t(fi) * ny + fj];
  } else {
    double L = M * h;
    for (int m = threadIdx.x; m < M; m += 256) {
      int i = i0 + m;
      double x = (i - npml + 0.5) * h;
      double sn, cs;
      sincos(kx * x, &sn, &cs);
      double2 wc = make_double2(cs * h / L, -sn * h / L);   // conj(w)
      acc = cadd(acc, cmul(wc, u[size_t(i) * ny + jm]));
    }
  }
  sre[threadIdx.x] = acc.x;
  sim[threadIdx.x] = acc.y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) pa[r0 + r] = sre[0] * sre[0] + sim[0] * sim[0];
}

__global__ __launch_bounds__(256) void k_weighted_sum(const double* __restrict__ w,
                                                      const double* __restrict__ pa, int n,
                                                      double* __restrict__ F) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) acc += w[q] * pa[q];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *F = s[0];
}

// Legendre P_n and its derivative at x by the three-term recurrence
__device__ void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x;
  for (int j = 1; j < n; ++j) {
    double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

// node k (ascending) of each interval: Newton iteration on P_n from the
// asymptotic first guess cos(pi (root + 3/4) / (n + 1/2)) of the descending root
__global__ void k_gl_nodes(int n, int nint, double lo0, double hi0, double lo1, double hi1,
                           double alpha, double* theta, double* wts) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * nint) return;
  int seg = q / n, k = q % n;
  int root = n - 1 - k;
  double x = cos(3.14159265358979323846 * (root + 0.75) / (n + 0.5));
  double pn, dpn;
  for (int it = 0; it < 60; ++it) {
    legendre(n, x, &pn, &dpn);
    double dx = pn / dpn;
    x -= dx;
    if (fabs(dx) < 1e-15) break;
  }
  legendre(n, x, &pn, &dpn);
  double w = 2.0 / ((1.0 - x * x) * dpn * dpn);
  double lo = seg ? lo1 : lo0, hi = seg ? hi1 : hi0;
  theta[q] = 0.5 * (hi - lo) * x + 0.5 * (hi + lo);
  wts[q] = 0.5 * (hi - lo) * w * alpha;
}

// out[q] = sum_g w_g x_g[q] (g in order); thread 0 of block 0 also sets
// F[count] = sum_g w_g F[g]
struct WSum {
  const double* x[MAX_BATCH];
  double w[MAX_BATCH];
};
__global__ void k_weighted_fields(WSum a, int count, size_t n, double* __restrict__ F,
                               double* __restrict__ out) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q == 0) {
    double t = 0.0;
    for (int g = 0; g < count; ++g) t += a.w[g] * F[g];
    F[count] = t;
  }
  if (q >= n) return;
  double acc = 0.0;
  for (int g = 0; g < count; ++g) acc += a.w[g] * a.x[g][q];
  out[q] = acc;
}

int fft_inplace(rcp_factors* f, double2* buf, int P, double sign, hipStream_t s) {
  int logP = 0;
  while ((1 << logP) < P) ++logP;
  if (P <= 4096) {
    k_fft_lds<<<1, 1024, 0, s>>>(buf, P, logP, sign);
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  }
  double2* tmp = f->fft[2];
  k_bitrev_copy<<<ceil_div(P, 256), 256, 0, s>>>(buf, tmp, P, logP);
  RCP_HIP(hipGetLastError());
  for (int half = 1; half < P; half <<= 1) {
    k_fft_stage<<<ceil_div(P / 2, 256), 256, 0, s>>>(tmp, P, half, sign);
    RCP_HIP(hipGetLastError());
  }
  RCP_HIP(hipMemcpyAsync(buf, tmp, size_t(P) * sizeof(double2), hipMemcpyDeviceToDevice, s));
  return RCP_OK;
}

}  // namespace

namespace rcp {

int fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / sizeof(double2);
  if (n == 0) return RCP_OK;
  k_fill_zero<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(static_cast<double2*>(p), n);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int objective_rhs(rcp_factors* f, const rcp_objective* o, double2* w, int* nz_lo, int* nz_hi,
                  hipStream_t s) {
  int rc = fill_zero(w, size_t(f->nx) * f->ny * sizeof(double2), s);
  if (rc) return rc;
  if (o->kind == RCP_CONCENTRATOR) {
    k_set<<<1, 64, 0, s>>>(w, size_t(o->i_f) * f->ny + o->j_f, make_double2(1.0, 0.0));
    RCP_HIP(hipGetLastError());
    *nz_lo = *nz_hi = o->i_f;
  } else {
    int M = o->i1 - o->i0;
    k_mode_row<<<ceil_div(M, 256), 256, 0, s>>>(w, f->ny, o->j_m, o->i0, M, f->npml, f->h,
                                                 f->k0 * o->n_m * std::sin(o->phi));
    RCP_HIP(hipGetLastError());
    *nz_lo = o->i0;
    *nz_hi = o->i1 - 1;
  }
  return RCP_OK;
}

static int fft_size(int M) {
  int P = 2;
  while (P < 2 * M - 1) P <<= 1;
  return P;
}

int toeplitz_form(rcp_factors* f, const rcp_light* L, const double2* z, double* F_dev,
                  double2* v_out, double2* Tv_out, hipStream_t s) {
  const int M = L->i1 - L->i0;
  const int P = fft_size(M);
  if (size_t(P) > f->fft_cap) return fail(RCP_EINVAL, "aperture too long for the FFT buffers");
  double2* chat = f->fft[0];
  double2* buf = f->fft[1];
  k_symbol_circ<<<ceil_div(P, 256), 256, 0, s>>>(chat, P, M, L->kind, L->c, L->th1, L->th2, L->n_s,
                                                  f->k0, f->h,
                                                  reinterpret_cast<const double2*>(L->symbol_dev));
  RCP_HIP(hipGetLastError());
  int rc = fft_inplace(f, chat, P, -1.0, s);
  if (rc) return rc;
  // keep the zero-padded v in the temp buffer's upper half? use v_out or a work vector
  double2* vpad = f->vec[V_TMP];
  k_gather_pad<<<ceil_div(P, 256), 256, 0, s>>>(z, f->ny, L->j_s, L->i0, M, P, buf, v_out);
  RCP_HIP(hipGetLastError());
  RCP_HIP(hipMemcpyAsync(vpad, buf, size_t(M) * sizeof(double2), hipMemcpyDeviceToDevice, s));
  rc = fft_inplace(f, buf, P, -1.0, s);
  if (rc) return rc;
  k_pointwise<<<ceil_div(P, 256), 256, 0, s>>>(buf, chat, P);
  RCP_HIP(hipGetLastError());
  rc = fft_inplace(f, buf, P, 1.0, s);
  if (rc) return rc;
  k_form_dot<<<1, 1024, 0, s>>>(buf, vpad, M, P, Tv_out, F_dev);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int grad_eps(rcp_factors* f, const double2* lam, const double2* z, double* grad, hipStream_t s) {
  size_t N = size_t(f->nx) * f->ny;
  k_grad_eps<<<static_cast<int>((N + 255) / 256), 256, 0, s>>>(f->nx, f->ny, f->k0, f->sxc, f->syc,
                                                                lam, z, grad);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int scatter_line(rcp_factors* f, const rcp_light* L, const double2* Tv, double2* rhs,
                 hipStream_t s) {
  int rc = fill_zero(rhs, size_t(f->nx) * f->ny * sizeof(double2), s);
  if (rc) return rc;
  int M = L->i1 - L->i0;
  k_scatter_line<<<ceil_div(M, 256), 256, 0, s>>>(Tv, f->ny, L->j_s, L->i0, M, rhs);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int planewave_lines(rcp_factors* f, const rcp_light* L, const double* theta, int R, double2* fline,
                    hipStream_t s) {
  size_t n = size_t(R) * f->nx;
  k_planewave_lines<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(
      theta, R, f->nx, L->i0, L->i1, f->npml, f->h, L->n_s, f->k0, fline);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int bf_per_angle_at(rcp_factors* f, const rcp_objective* o, const double2* U, int R,
                    double* per_angle, int r0, hipStream_t s) {
  k_bf_amp<<<R, 256, 0, s>>>(U, size_t(f->nx) * f->ny, f->ny, o->kind, o->i_f, o->j_f, o->j_m,
                             o->i0, o->i1 - o->i0, f->npml, f->h,
                             f->k0 * o->n_m * std::sin(o->phi), per_angle, r0);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

// Gauss-Legendre nodes in theta (Sec. "Brute-force quadrature"), ascending, split
// evenly over the intervals of the light; wts = node weight times <|a(theta)|^2>.
int gl_nodes(const rcp_light* L, int n, double* theta, double* wts, hipStream_t s) {
  int nint = L->kind == RCP_ANNULUS ? 2 : 1;
  int per = n / nint;
  double lo0, hi0, lo1 = 0, hi1 = 0, alpha;
  if (nint == 1) {
    lo0 = -L->c;
    hi0 = L->c;
    alpha = 1.0 / (2.0 * L->c);
  } else {
    lo0 = -L->th2;
    hi0 = -L->th1;
    lo1 = L->th1;
    hi1 = L->th2;
    alpha = 1.0 / (2.0 * (L->th2 - L->th1));
  }
  k_gl_nodes<<<ceil_div(n, 64), 64, 0, s>>>(per, nint, lo0, hi0, lo1, hi1, alpha, theta, wts);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int weighted_sum(int count, const double* w, double* const* x, size_t n, double* F, double* out,
                 hipStream_t s) {
  WSum a{};
  for (int g = 0; g < count; ++g) {
    a.x[g] = x[g];
    a.w[g] = w[g];
  }
  k_weighted_fields<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(a, count, n, F, out);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int bf_sum(const double* weights, const double* per_angle, int n, double* F_dev, hipStream_t s) {
  k_weighted_sum<<<1, 256, 0, s>>>(weights, per_angle, n, F_dev);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

}  // namespace rcp

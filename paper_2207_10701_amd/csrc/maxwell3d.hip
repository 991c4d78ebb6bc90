// The 3D vector problem (Sec. "Concluding remarks": in 3D the reciprocal
// average needs one solve per field component the figure of merit reads --
// three for a focal spot, two for an output mode -- and the incident light
// varies over two angles and two polarisations).
//
// curl curl E - k^2 eps E = i k J on a Yee grid (E_x at ((i+1/2)h, jh, kh),
// E_y at (ih, (j+1/2)h, kh), E_z at (ih, jh, (k+1/2)h), tangential E zero
// beyond the grid), with the uniaxial form of the stretched-coordinate PML,
//   A = C^T D_mu^{-1} C - k^2 D_eps eps,  D = diag(s_a s_b / s_c),
// which is complex symmetric.  Ordered by x-slices i (unknowns of slice i:
// component c, then j, then k; n = 3 ny nz per slice), A is block tridiagonal
// with diagonal blocks of the in-slice curl-curl and couplings between
// neighbouring slices that are sparse but not diagonal (E_x of slice i meets
// E_y, E_z of slice i+1 through the faces normal to y and z).  The blocks are
// eliminated by the same two-ended elimination and symmetric Gauss-Jordan
// sweep on packed tiles as the 2D operator (the factorisation engine); only
// the Schur complements S = D - C^T X C and the coupling products of the
// solves differ, and live here.
#include <cmath>
#include <string>
#include <vector>

#include "rcp_internal.h"

namespace {
using namespace rcp;

constexpr int DW = K3D_DW;   // in-slice entries per row (the curl-curl has at most 9)
constexpr int CW = K3D_CW;   // entries per row of a coupling to a neighbouring slice (<= 4)

struct Grid3 {
  int nx, ny, nz, npml;
  double h, k0, sigma;   // sigma of the stretch profile
  int pml_m;
};

__device__ __forceinline__ double2 stretch(const Grid3& g, int n_axis, double xi) {
  // s(xi) = 1 + i sigma (d / L)^m, d the depth into the PML (cell units xi)
  if (g.npml == 0) return make_double2(1.0, 0.0);
  double d = fmax(fmax(g.npml - xi, xi - (n_axis - g.npml)), 0.0) / g.npml;
  double p = 1.0;
  for (int q = 0; q < g.pml_m; ++q) p *= d;
  return make_double2(1.0, g.sigma * p);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// s_a s_b / s_c at position (x, y, z) (cell units) for axis c.
__device__ __forceinline__ double2 uniaxial(const Grid3& g, double x, double y, double z, int c) {
  const double2 s[3] = {stretch(g, g.nx, x), stretch(g, g.ny, y), stretch(g, g.nz, z)};
  const int a = c == 0 ? 1 : 0, b = c == 2 ? 1 : 2;
  return cdiv(cmul(s[a], s[b]), s[c]);
}

// Face-edge incidence of the forward-difference curl: the face normal to cf at
// cell f carries H_cf = sum over its four edges of sgn / h * E_comp(f + off):
//   H_x = dE_z/dy - dE_y/dz, H_y = dE_x/dz - dE_z/dx, H_z = dE_y/dx - dE_x/dy.
__constant__ int kComp[3][4] = {{2, 2, 1, 1}, {0, 0, 2, 2}, {1, 1, 0, 0}};
__constant__ int kSgn[3][4] = {{1, -1, -1, 1}, {1, -1, -1, 1}, {1, -1, -1, 1}};
__constant__ int kOff[3][4][3] = {{{0, 1, 0}, {0, 0, 0}, {0, 0, 1}, {0, 0, 0}},
                                  {{0, 0, 1}, {0, 0, 0}, {1, 0, 0}, {0, 0, 0}},
                                  {{1, 0, 0}, {0, 0, 0}, {0, 1, 0}, {0, 0, 0}}};

__device__ __forceinline__ int slice_index(const Grid3& g, int c, int j, int k) {
  return (c * g.ny + j) * g.nz + k;
}

// Adds v at column col of a short (index, value) list.
template <int W>
__device__ __forceinline__ void list_add(int* idx, double2* val, int col, double2 v) {
#pragma unroll
  for (int q = 0; q < W; ++q) {
    if (idx[q] == col) {
      val[q] = cadd(val[q], v);
      return;
    }
    if (idx[q] < 0) {
      idx[q] = col;
      val[q] = v;
      return;
    }
  }
}

// One row of A per thread (edge (c, i, j, k)): the products over the four faces
// that hold the edge, sorted into the diagonal block of its slice and the
// couplings to the next and the previous slice.
__global__ void k_assemble3d(Grid3 g, const double* __restrict__ eps, int32_t* d_idx,
                             double2* d_val, int32_t* cr_idx, double2* cr_val, int32_t* cl_idx,
                             double2* cl_val) {
  const int n = 3 * g.ny * g.nz;
  const long long tot = (long long)g.nx * n;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = static_cast<int>(t / n), a = static_cast<int>(t % n);
  const int c = a / (g.ny * g.nz), j = (a / g.nz) % g.ny, k = a % g.nz;
  int di[DW], ri[CW], li[CW];
  double2 dv[DW], rv[CW], lv[CW];
#pragma unroll
  for (int q = 0; q < DW; ++q) {
    di[q] = -1;
    dv[q] = make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    ri[q] = li[q] = -1;
    rv[q] = lv[q] = make_double2(0.0, 0.0);
  }
  const int e0[3] = {i, j, k};
  const int nn[3] = {g.nx, g.ny, g.nz};
  const double h2 = g.h * g.h;
  for (int cf = 0; cf < 3; ++cf) {
    for (int s0 = 0; s0 < 4; ++s0) {
      if (kComp[cf][s0] != c) continue;
      int f[3];
      bool in = true;
      for (int d = 0; d < 3; ++d) {
        f[d] = e0[d] - kOff[cf][s0][d];
        in = in && f[d] >= 0 && f[d] < nn[d];
      }
      if (!in) continue;
      // 1 / D_mu at the face centre: H_cf at (f + 1/2) except f along cf
      double pos[3] = {f[0] + 0.5, f[1] + 0.5, f[2] + 0.5};
      pos[cf] -= 0.5;
      const double2 dmu = uniaxial(g, pos[0], pos[1], pos[2], cf);
      const double2 w = cdiv(make_double2(double(kSgn[cf][s0]) / h2, 0.0), dmu);
      for (int s1 = 0; s1 < 4; ++s1) {
        int e[3];
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
          e[d] = f[d] + kOff[cf][s1][d];
          ok = ok && e[d] < nn[d];
        }
        if (!ok) continue;
        const double2 v = make_double2(w.x * kSgn[cf][s1], w.y * kSgn[cf][s1]);
        const int col = slice_index(g, kComp[cf][s1], e[1], e[2]);
        if (e[0] == i)
          list_add<DW>(di, dv, col, v);
        else if (e[0] == i + 1)
          list_add<CW>(ri, rv, col, v);
        else
          list_add<CW>(li, lv, col, v);
      }
    }
  }
  // - k^2 D_eps eps on the diagonal, at the edge's own position
  double pe[3] = {double(i), double(j), double(k)};
  pe[c] += 0.5;
  const double2 de = uniaxial(g, pe[0], pe[1], pe[2], c);
  const double e_ = eps[(size_t)i * n + a];
  list_add<DW>(di, dv, a, make_double2(-g.k0 * g.k0 * e_ * de.x, -g.k0 * g.k0 * e_ * de.y));
  const size_t row = (size_t)i * n + a;
#pragma unroll
  for (int q = 0; q < DW; ++q) {
    d_idx[row * DW + q] = di[q];
    d_val[row * DW + q] = dv[q];
  }
  if (i + 1 < g.nx) {   // A_{i,i+1}(a, .): row a of boundary i
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      cr_idx[row * CW + q] = ri[q];
      cr_val[row * CW + q] = rv[q];
    }
  }
  if (i > 0) {   // A_{i,i-1}(a, .) = A_{i-1,i}(., a): column a of boundary i-1
    const size_t r2 = (size_t)(i - 1) * n + a;
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      cl_idx[r2 * CW + q] = li[q];
      cl_val[r2 * CW + q] = lv[q];
    }
  }
}

// Permittivity at the three E positions of every cell, from square pillars of
// side w centred at (x_p, y_p) in the layers [k0, k0 + layers) above a substrate
// of sub_layers (the mean of eps over the h x h square around the component's
// (x, y)).  Output in the slice order (i, c, j, k).
__global__ void k_eps3d(int nx, int ny, int nz, int npml, double h, int npil,
                        const double* __restrict__ centers, const double* __restrict__ widths,
                        double eps_bg, double eps_sub, double eps_pil, int sub_layers, int pk0,
                        int players, double* __restrict__ eps) {
  const int n = 3 * ny * nz;
  const long long tot = (long long)nx * n;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = static_cast<int>(t / n), a = static_cast<int>(t % n);
  const int c = a / (ny * nz), j = (a / nz) % ny, k = a % nz;
  const double x = (i + (c == 0 ? 0.5 : 0.0) - npml) * h;
  const double y = (j + (c == 1 ? 0.5 : 0.0) - npml) * h;
  const double z = k + (c == 2 ? 0.5 : 0.0);
  double v = eps_bg;
  if (z < sub_layers) {
    v = eps_sub;
  } else if (z >= pk0 && z < pk0 + players) {
    double frac = 0.0;
    for (int p = 0; p < npil; ++p) {
      const double xc = centers[2 * p], yc = centers[2 * p + 1], hw = 0.5 * widths[p];
      const double fx = fmax(fmin(x + 0.5 * h, xc + hw) - fmax(x - 0.5 * h, xc - hw), 0.0) / h;
      const double fy = fmax(fmin(y + 0.5 * h, yc + hw) - fmax(y - 0.5 * h, yc - hw), 0.0) / h;
      frac += fx * fy;
    }
    v = eps_bg + (eps_pil - eps_bg) * frac;
  }
  eps[t] = v;
}

// Element (a, b) of the symmetric part of a block stored as packed lower
// tiles.  The Gauss-Jordan sweep keeps its diagonal tiles whole, and their two
// halves agree only to rounding; the mean of (a, b) and (b, a) there makes
// x_at(a, b) == x_at(b, a) bit for bit.  (Reading one half as it stands would
// hand the next Schur complement an antisymmetric part, which the symmetric
// sweep of the next block cannot represent; along a chain of 3D blocks that
// error grew about a hundredfold per block.)
__device__ __forceinline__ double2 x_at(const double2* X, int a, int b) {
  if (a < b) {
    const int t = a;
    a = b;
    b = t;
  }
  const int I = a / TB, J = b / TB;
  const double2* T = X + tile_index(I, J) * TB * TB;
  const double2 u = T[(a % TB) * TB + (b % TB)];
  if (I != J) return u;
  const double2 w = T[(b % TB) * TB + (a % TB)];
  return make_double2(0.5 * (u.x + w.x), 0.5 * (u.y + w.y));
}

struct Schur3dJobs {
  Schur3dJob j[2 * MAX_BATCH];
  int n;
  int maxtiles;
};

// dst = D - C1 src1 C1^T - C2 src2 C2^T on packed tiles, identity in the padding;
// one thread per element of the lower tiles.  Both halves of a diagonal tile
// are computed as the element (max, min) in one order of terms, so dst is
// symmetric bit for bit.
__global__ __launch_bounds__(256) void k_schur3d(Schur3dJobs js) {
  const int per = js.maxtiles * 4;   // 256 threads x 4 workgroups per tile
  const int q = blockIdx.x / per;
  const int r = blockIdx.x - q * per;
  const Schur3dJob jb = js.j[q];
  const int t = r / 4;
  if (t >= jb.tiles) return;
  int I, J;
  tile_coords(t, &I, &J);
  const int e = (r % 4) * 256 + threadIdx.x;
  const int ea = I * TB + e / TB, eb = J * TB + e % TB;
  const int a = ea > eb ? ea : eb, b = ea > eb ? eb : ea;
  double2 v = make_double2(0.0, 0.0);
  if (a >= jb.n || b >= jb.n) {
    if (a == b) v = make_double2(1.0, 0.0);
  } else {
    const size_t ra = (size_t)a * DW;
#pragma unroll
    for (int u = 0; u < DW; ++u)
      if (jb.d_idx[ra + u] == b) v = jb.d_val[ra + u];
    const void* srcs[2] = {jb.src1, jb.src2};
    const int32_t* ci[2] = {jb.c1_idx, jb.c2_idx};
    const double2* cv[2] = {jb.c1_val, jb.c2_val};
    for (int sidx = 0; sidx < 2; ++sidx) {
      if (!srcs[sidx]) continue;
      const double2* X = static_cast<const double2*>(srcs[sidx]);
      const int32_t* ii = ci[sidx];
      const double2* vv = cv[sidx];
      for (int p = 0; p < CW; ++p) {
        const int pa = ii[(size_t)a * CW + p];
        if (pa < 0) continue;
        double2 acc = make_double2(0.0, 0.0);
        for (int p2 = 0; p2 < CW; ++p2) {
          const int pb = ii[(size_t)b * CW + p2];
          if (pb < 0) continue;
          acc = cadd(acc, cmul(x_at(X, pa, pb), vv[(size_t)b * CW + p2]));
        }
        v = csub(v, cmul(vv[(size_t)a * CW + p], acc));
      }
    }
  }
  static_cast<double2*>(jb.dst)[(size_t)t * TB * TB + e] = v;
}

// g = f - sum of the coupling products of up to two neighbouring fields
// (conj of the coupling values for the conjugate operator).
struct Couple {
  const double2* f;
  const int32_t* idx[2];
  const double2* val[2];
  const double2* v[2];
  double2* g;
};
__global__ void k_couple3d(Couple cp, int n, int conjop) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double2 s = cp.f ? cp.f[a] : make_double2(0.0, 0.0);
  for (int q = 0; q < 2; ++q) {
    if (!cp.v[q]) continue;
    for (int p = 0; p < CW; ++p) {
      const int b = cp.idx[q][(size_t)a * CW + p];
      if (b < 0) continue;
      double2 c = cp.val[q][(size_t)a * CW + p];
      if (conjop) c.y = -c.y;
      s = csub(s, cmul(c, cp.v[q][b]));
    }
  }
  cp.g[a] = s;
}

// Right-hand sides of the objective (columns of w as full fields): the three
// components at the focus cell, or the two polarisations of the output mode
// (h^2 / area) e_pol exp(i k_par . r) on the tangential components of plane km.
__global__ void k_objective3d(int nx, int ny, int nz, int npml, double h, double k0,
                              rcp_objective3d o, double2* __restrict__ W, size_t N) {
  const int m = o.kind == RCP_CONCENTRATOR ? 3 : 2;
  const size_t tot = N * m;
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int col = static_cast<int>(t / N);
  const size_t q = t - size_t(col) * N;
  const int n = 3 * ny * nz;
  const int i = static_cast<int>(q / n), a = static_cast<int>(q % n);
  const int c = a / (ny * nz), j = (a / nz) % ny, k = a % nz;
  double2 v = make_double2(0.0, 0.0);
  if (o.kind == RCP_CONCENTRATOR) {
    if (c == col && i == o.i_f && j == o.j_f && k == o.k_f) v = make_double2(1.0, 0.0);
  } else if (k == o.k_m && c < 2 && i >= npml && i < nx - npml && j >= npml && j < ny - npml) {
    const double area = (nx - 2 * npml) * h * (ny - 2 * npml) * h;
    const double ca = cos(o.azimuth), sa = sin(o.azimuth);
    // s: normal to the plane of incidence; p: along the tangential wavevector
    const double e = col == 0 ? (c == 0 ? -sa : ca) : (c == 0 ? ca : sa);
    const double x = (i + (c == 0 ? 0.5 : 0.0) - npml) * h;
    const double y = (j + (c == 1 ? 0.5 : 0.0) - npml) * h;
    const double kk = k0 * o.n_m * sin(o.theta);
    const double ph = kk * (ca * x + sa * y);
    const double amp = h * h / area * e;
    v = make_double2(amp * cos(ph), amp * sin(ph));
  }
  W[t] = v;
}

// Unit-power sheet current of direction d (theta, azimuth) and polarisation
// pol (0 = s, 1 = p) on the physical cells of plane ks, as b = i k J / h:
// |J_s| = 2 sqrt(n cos theta), |J_p| = 2 sqrt(n / cos theta), phase
// exp(i K sin theta (cos az x + sin az y)), K = n k, x and y of each component.
__device__ __forceinline__ double2 sheet_value(int i, int j, int c, int npml, double h, double k0,
                                               double n_s, double th, double az, int pol) {
  const double ca = cos(az), sa = sin(az), ct = cos(th);
  const double amp = pol == 0 ? 2.0 * sqrt(n_s * ct) : 2.0 * sqrt(n_s / ct);
  const double e = pol == 0 ? (c == 0 ? -sa : ca) : (c == 0 ? ca : sa);
  const double x = (i + (c == 0 ? 0.5 : 0.0) - npml) * h;
  const double y = (j + (c == 1 ? 0.5 : 0.0) - npml) * h;
  const double K = n_s * k0 * sin(th);
  const double ph = K * (ca * x + sa * y);
  const double s = k0 * amp * e / h;   // b = i k J / h
  return make_double2(-s * sin(ph), s * cos(ph));
}

__global__ void k_source3d(int nx, int ny, int nz, int npml, double h, double k0, int ks,
                           double n_s, double th, double az, int pol, double2* __restrict__ b,
                           size_t N) {
  const size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const int n = 3 * ny * nz;
  const int i = static_cast<int>(q / n), a = static_cast<int>(q % n);
  const int c = a / (ny * nz), j = (a / nz) % ny, k = a % nz;
  double2 v = make_double2(0.0, 0.0);
  if (k == ks && c < 2 && i >= npml && i < nx - npml && j >= npml && j < ny - npml)
    v = sheet_value(i, j, c, npml, h, k0, n_s, th, az, pol);
  b[q] = v;
}

// out[(col, d, pol)] = |b_(d,pol)^dag z_col|^2 over the incidence plane: one
// workgroup per (col, d, pol), a fixed-order reduction.
__global__ __launch_bounds__(256) void k_plane_proj3d(int nx, int ny, int nz, int npml, double h,
                                                      double k0, int ks, double n_s,
                                                      const double* __restrict__ dirs, int ndir,
                                                      const double2* __restrict__ Z, size_t N,
                                                      double* __restrict__ out) {
  __shared__ double sr[256], si[256];
  const int g = blockIdx.x;
  const int col = g / (2 * ndir), d = (g / 2) % ndir, pol = g % 2;
  const double th = dirs[3 * d], az = dirs[3 * d + 1];
  const int mx = nx - 2 * npml, my = ny - 2 * npml;
  const int n = 3 * ny * nz;
  double2 acc = make_double2(0.0, 0.0);
  for (int e = threadIdx.x; e < 2 * mx * my; e += 256) {
    const int c = e / (mx * my), r = e % (mx * my);
    const int i = npml + r / my, j = npml + r % my;
    const double2 b = sheet_value(i, j, c, npml, h, k0, n_s, th, az, pol);
    const double2 z = Z[size_t(col) * N + size_t(i) * n + (c * ny + j) * nz + ks];
    acc = cadd(acc, make_double2(b.x * z.x + b.y * z.y, b.x * z.y - b.y * z.x));   // conj(b) z
  }
  sr[threadIdx.x] = acc.x;
  si[threadIdx.x] = acc.y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = sr[0] * sr[0] + si[0] * si[0];
}

// out[r] = sum over the m objective columns of |w_col^dag u_r|^2, one workgroup
// per forward field u_r, fixed-order reduction.
__global__ __launch_bounds__(256) void k_obj_amp3d(const double2* __restrict__ W, int m,
                                                   const double2* __restrict__ U, size_t N,
                                                   double* __restrict__ out) {
  __shared__ double sr[256], si[256];
  double tot = 0.0;
  for (int col = 0; col < m; ++col) {
    double2 acc = make_double2(0.0, 0.0);
    for (size_t q = threadIdx.x; q < N; q += 256) {
      const double2 w = W[size_t(col) * N + q];
      if (w.x == 0.0 && w.y == 0.0) continue;
      const double2 u = U[size_t(blockIdx.x) * N + q];
      acc = cadd(acc, make_double2(w.x * u.x + w.y * u.y, w.x * u.y - w.y * u.x));
    }
    sr[threadIdx.x] = acc.x;
    si[threadIdx.x] = acc.y;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        sr[threadIdx.x] += sr[threadIdx.x + s];
        si[threadIdx.x] += si[threadIdx.x + s];
      }
      __syncthreads();
    }
    tot += sr[0] * sr[0] + si[0] * si[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// F = sum_d weight_d sum_(k < per) vals[d * per + k] (and, with cols > 1, over
// the columns first: vals[(col, d, k)]), in a fixed order by one thread.
__global__ void k_weighted3d(const double* __restrict__ dirs, int ndir, const double* __restrict__ vals,
                             int cols, int per, double* __restrict__ F) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int d = 0; d < ndir; ++d) {
    double v = 0.0;
    for (int col = 0; col < cols; ++col)
      for (int k = 0; k < per; ++k) v += vals[(size_t(col) * ndir + d) * per + k];
    s += dirs[3 * d + 2] * v;
  }
  *F = s;
}

}  // namespace

namespace rcp {

int schur3d(const Schur3dJob* jobs, int count, hipStream_t s) {
  if (count < 1) return RCP_OK;
  if (count > 2 * MAX_BATCH) return fail(RCP_EINVAL, "internal: too many 3D Schur jobs");
  Schur3dJobs js{};
  for (int q = 0; q < count; ++q) {
    js.j[js.n++] = jobs[q];
    if (jobs[q].tiles > js.maxtiles) js.maxtiles = jobs[q].tiles;
  }
  k_schur3d<<<js.n * js.maxtiles * 4, 256, 0, s>>>(js);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

}  // namespace rcp

using namespace rcp;

namespace {

struct Layout3 {
  size_t off_X, off_eps, off_didx, off_dval, off_cridx, off_crval, off_clidx, off_clval;
  size_t off_L, off_Q, off_P, off_health, off_vec, off_part, off_status, total;
};

Layout3 layout3(const rcp_grid3d* g) {
  Layout3 L{};
  const int n = 3 * g->ny * g->nz;
  const int np = ceil_div(n, TB) * TB, nt = np / TB;
  const size_t tiles = size_t(nt) * (nt + 1) / 2;
  const size_t N = size_t(g->nx) * n;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.off_X = take(size_t(g->nx) * tiles * TB * TB * 16);
  L.off_eps = take(N * 8);
  L.off_didx = take(N * DW * 4);
  L.off_dval = take(N * DW * 16);
  L.off_cridx = take(N * CW * 4);
  L.off_crval = take(N * CW * 16);
  L.off_clidx = take(N * CW * 4);
  L.off_clval = take(N * CW * 16);
  L.off_L = take(8 * size_t(np) * TB * 16);
  L.off_Q = take(8 * size_t(np) * TB * 16);
  L.off_P = take(8 * size_t(TB) * TB * 16);
  L.off_health = take(size_t(g->nx) * nt * 8);
  L.off_vec = take(4 * N * 16);
  L.off_part = take(2 * 2 * tiles * TB * 16);
  L.off_status = take(4);
  L.total = o;
  return L;
}

int check_grid3d(const rcp_grid3d* g) {
  if (!g) return fail(RCP_EINVAL, "grid is NULL");
  if (g->nx < 3 || g->ny < 1 || g->nz < 1) return fail(RCP_EINVAL, "grid too small");
  if (g->npml < 0 || 2 * g->npml >= g->nx || 2 * g->npml >= g->ny || 2 * g->npml >= g->nz)
    return fail(RCP_EINVAL, "PML layers overlap or leave no physical region");
  if (!(g->h > 0) || !(g->k0 > 0)) return fail(RCP_EINVAL, "h and k0 must be positive");
  if (g->npml > 0 && (!(g->pml_R > 0 && g->pml_R < 1) || g->pml_m < 0))
    return fail(RCP_EINVAL, "PML reflection must be in (0, 1)");
  const long long n = 3LL * g->ny * g->nz;
  if (n <= TB || n > (1 << 16)) return fail(RCP_EINVAL, "3 ny nz must be 33 to 65536");
  return RCP_OK;
}

Grid3 grid3(const rcp_factors* f) {
  Grid3 g{f->nx, f->gy, f->gz, f->npml, f->h, f->k0, 0.0, f->pml_m};
  if (f->npml > 0) {
    const double L = f->npml * f->h;
    g.sigma = (f->pml_m + 1) * std::log(1.0 / f->pml_R) / (2.0 * f->k0 * L);
  }
  return g;
}

int check_obj3d(const rcp_factors* f, const rcp_objective3d* o) {
  if (!o) return fail(RCP_EINVAL, "objective is NULL");
  const int p = f->npml;
  if (o->kind == RCP_CONCENTRATOR) {
    if (o->i_f < p || o->i_f >= f->nx - p || o->j_f < p || o->j_f >= f->gy - p || o->k_f < p ||
        o->k_f >= f->gz - p)
      return fail(RCP_EINVAL, "focus cell outside the physical region");
  } else if (o->kind == RCP_COLLIMATOR) {
    if (o->k_m < p || o->k_m >= f->gz - p) return fail(RCP_EINVAL, "monitor plane outside");
    if (!(o->n_m > 0)) return fail(RCP_EINVAL, "monitor index must be positive");
  } else {
    return fail(RCP_EINVAL, "unknown objective kind");
  }
  return RCP_OK;
}

int check_light3d(const rcp_factors* f, const rcp_light3d* L) {
  if (!L) return fail(RCP_EINVAL, "light is NULL");
  if (L->k_s < f->npml || L->k_s >= f->gz - f->npml) return fail(RCP_EINVAL, "incidence plane outside");
  if (!(L->n_s > 0)) return fail(RCP_EINVAL, "source index must be positive");
  if (L->ndir < 1 || L->ndir > (1 << 16) || !L->dirs_dev) return fail(RCP_EINVAL, "bad direction rule");
  return RCP_OK;
}

// u = A^{-1} b (conjop = 0) or conj(A)^{-1} b = A^{-dag} b (conjop = 1): the
// twisted block sweeps with the sparse slice couplings applied by k_couple3d.
int solve3d(rcp_factors* f, const double2* b, double2* u, int conjop, hipStream_t s) {
  const int N = f->nx, n = f->ny, m = f->m;
  const int lenL = m, lenR = N - 1 - m;
  double2* g0 = f->vec[2];
  double2* g1 = f->vec[3];
  auto U = [&](int i) { return u + size_t(i) * n; };
  auto B = [&](int i) { return b + size_t(i) * n; };
  auto CR = [&](int i) { return f->cr_idx + size_t(i) * n * CW; };
  auto CRv = [&](int i) { return f->cr_val + size_t(i) * n * CW; };
  auto CL = [&](int i) { return f->cl_idx + size_t(i) * n * CW; };
  auto CLv = [&](int i) { return f->cl_val + size_t(i) * n * CW; };
  const int cgrid = ceil_div(n, 256);
  auto couple = [&](const double2* fb, int nsrc, const int32_t* i0, const double2* v0,
                    const double2* x0, const int32_t* i1, const double2* v1, const double2* x1,
                    double2* g) -> int {
    Couple cp{fb, {i0, i1}, {v0, v1}, {nsrc > 0 ? x0 : nullptr, nsrc > 1 ? x1 : nullptr}, g};
    k_couple3d<<<cgrid, 256, 0, s>>>(cp, n, conjop);
    RCP_HIP(hipGetLastError());
    return RCP_OK;
  };
  const int steps = lenL > lenR ? lenL : lenR;
  for (int st = 0; st < steps; ++st) {   // forward: y_i = X_i (b_i - A_{i,i-+1} y_{i-+1})
    int blocks[2], areas[2], cnt = 0;
    const double2* gs[2];
    const double2* bases[2] = {nullptr, nullptr};
    double2* outs[2];
    if (st < lenL) {
      const int i = st;
      int rc = couple(B(i), i > 0 ? 1 : 0, i > 0 ? CL(i - 1) : nullptr,
                      i > 0 ? CLv(i - 1) : nullptr, i > 0 ? U(i - 1) : nullptr, nullptr, nullptr,
                      nullptr, g0);
      if (rc) return rc;
      blocks[cnt] = i;
      gs[cnt] = g0;
      outs[cnt] = U(i);
      areas[cnt++] = 0;
    }
    if (st < lenR) {
      const int i = N - 1 - st;
      int rc = couple(B(i), i < N - 1 ? 1 : 0, i < N - 1 ? CR(i) : nullptr,
                      i < N - 1 ? CRv(i) : nullptr, i < N - 1 ? U(i + 1) : nullptr, nullptr,
                      nullptr, nullptr, g1);
      if (rc) return rc;
      blocks[cnt] = i;
      gs[cnt] = g1;
      outs[cnt] = U(i);
      areas[cnt++] = 1;
    }
    int rc = block_products(f, cnt, blocks, gs, bases, outs, areas, conjop, s);
    if (rc) return rc;
  }
  {   // middle
    int rc = couple(B(m), 2, m > 0 ? CL(m - 1) : nullptr, m > 0 ? CLv(m - 1) : nullptr,
                    m > 0 ? U(m - 1) : nullptr, m + 1 < N ? CR(m) : nullptr,
                    m + 1 < N ? CRv(m) : nullptr, m + 1 < N ? U(m + 1) : nullptr, g0);
    if (rc) return rc;
    const int blocks[1] = {m}, areas[1] = {0};
    const double2* gs[1] = {g0};
    const double2* bases[1] = {nullptr};
    double2* outs[1] = {U(m)};
    rc = block_products(f, 1, blocks, gs, bases, outs, areas, conjop, s);
    if (rc) return rc;
  }
  for (int st = 0; st < steps; ++st) {   // back: u_i = y_i - X_i A_{i,i+-1} u_{i+-1}
    int blocks[2], areas[2], cnt = 0;
    const double2* gs[2];
    const double2* bases[2];
    double2* outs[2];
    if (st < lenL) {
      const int i = m - 1 - st;
      int rc = couple(nullptr, 1, CR(i), CRv(i), U(i + 1), nullptr, nullptr, nullptr, g0);
      if (rc) return rc;
      blocks[cnt] = i;
      gs[cnt] = g0;
      bases[cnt] = U(i);
      outs[cnt] = U(i);
      areas[cnt++] = 0;
    }
    if (st < lenR) {
      const int i = m + 1 + st;
      int rc = couple(nullptr, 1, CL(i - 1), CLv(i - 1), U(i - 1), nullptr, nullptr, nullptr, g1);
      if (rc) return rc;
      blocks[cnt] = i;
      gs[cnt] = g1;
      bases[cnt] = U(i);
      outs[cnt] = U(i);
      areas[cnt++] = 1;
    }
    int rc = block_products(f, cnt, blocks, gs, bases, outs, areas, conjop, s);
    if (rc) return rc;
  }
  return RCP_OK;
}

}  // namespace

extern "C" {

size_t rcp_factor3d_bytes(const rcp_grid3d* grid) {
  if (check_grid3d(grid) != RCP_OK) return 0;
  return layout3(grid).total;
}

int rcp_eps3d_from_pillars(const rcp_grid3d* grid, const rcp_pillars3d* p, double* eps_out_dev,
                           rcp_stream stream) {
  int rc = check_grid3d(grid);
  if (rc) return rc;
  if (!p || p->n < 0 || (p->n > 0 && (!p->centers_dev || !p->widths_dev)))
    return fail(RCP_EINVAL, "bad pillar description");
  if (!eps_out_dev) return fail(RCP_EINVAL, "eps_out_dev is NULL");
  const long long tot = 3LL * grid->nx * grid->ny * grid->nz;
  k_eps3d<<<static_cast<int>((tot + 255) / 256), 256, 0, stream>>>(
      grid->nx, grid->ny, grid->nz, grid->npml, grid->h, p->n, p->centers_dev, p->widths_dev,
      p->eps_bg, p->eps_sub, p->eps_pillar, p->sub_layers, p->pillar_k0, p->pillar_layers,
      eps_out_dev);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int rcp_factor3d(const rcp_grid3d* grid, void* buf_dev, size_t buf_bytes, rcp_stream stream,
                 rcp_factors** out) {
  if (!out) return fail(RCP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_grid3d(grid);
  if (rc) return rc;
  if (!grid->eps_dev) return fail(RCP_EINVAL, "eps_dev is NULL");
  const Layout3 L = layout3(grid);
  if (!buf_dev || buf_bytes < L.total)
    return fail(RCP_ENOMEM, "factor buffer needs " + std::to_string(L.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(buf_dev) % 256 != 0)
    return fail(RCP_EINVAL, "factor buffer must be 256-byte aligned");
  rcp_factors* f = new (std::nothrow) rcp_factors();
  if (!f) return fail(RCP_ENOMEM, "host allocation failed");
  const int n = 3 * grid->ny * grid->nz;
  f->dim3 = 1;
  f->gy = grid->ny;
  f->gz = grid->nz;
  f->nx = grid->nx;
  f->ny = n;
  f->npml = grid->npml;
  f->h = grid->h;
  f->k0 = grid->k0;
  f->pml_R = grid->pml_R;
  f->pml_m = grid->pml_m;
  f->precision = RCP_FP64;
  f->np = ceil_div(n, TB) * TB;
  f->nt = f->np / TB;
  f->tiles = size_t(f->nt) * (f->nt + 1) / 2;
  f->block_elems = f->tiles * TB * TB;
  f->elem_bytes = 16;
  f->m = grid->nx / 2;
  char* b = static_cast<char*>(buf_dev);
  f->base = b;
  f->X = b + L.off_X;
  f->eps = reinterpret_cast<double*>(b + L.off_eps);
  f->d_idx = reinterpret_cast<int32_t*>(b + L.off_didx);
  f->d_val = reinterpret_cast<double2*>(b + L.off_dval);
  f->cr_idx = reinterpret_cast<int32_t*>(b + L.off_cridx);
  f->cr_val = reinterpret_cast<double2*>(b + L.off_crval);
  f->cl_idx = reinterpret_cast<int32_t*>(b + L.off_clidx);
  f->cl_val = reinterpret_cast<double2*>(b + L.off_clval);
  const size_t panel = size_t(f->np) * TB * 16;
  for (int c = 0; c < 8; ++c) {
    f->wsL[c] = b + L.off_L + c * panel;
    f->wsQ[c] = b + L.off_Q + c * panel;
    f->wsP[c] = reinterpret_cast<double2*>(b + L.off_P) + c * TB * TB;
  }
  f->health = reinterpret_cast<double*>(b + L.off_health);
  f->status = reinterpret_cast<int32_t*>(b + L.off_status);
  const size_t N = size_t(f->nx) * n;
  for (int v = 0; v < NVEC; ++v) f->vec[v] = nullptr;
  for (int v = 0; v < 4; ++v) f->vec[v] = reinterpret_cast<double2*>(b + L.off_vec) + v * N;
  for (int c = 0; c < 2; ++c)
    f->part[c] = reinterpret_cast<double2*>(b + L.off_part) + c * 2 * f->tiles * TB;
  rc = RCP_OK;
  {
    hipError_t he = hipMemcpyAsync(f->eps, grid->eps_dev, N * 8, hipMemcpyDeviceToDevice, stream);
    if (he == hipSuccess) {
      k_assemble3d<<<static_cast<int>((N + 255) / 256), 256, 0, stream>>>(
          grid3(f), f->eps, f->d_idx, f->d_val, f->cr_idx, f->cr_val, f->cl_idx, f->cl_val);
      he = hipGetLastError();
    }
    if (he != hipSuccess) rc = hip_check(he, "3D assembly");
  }
  // the block elimination: the factorisation engine with this one geometry
  rcp_engine* e = nullptr;
  if (!rc) rc = engine_create(RCP_FP64, &e);
  if (!rc) rc = engine_add(e, f);
  while (!rc && engine_active(e) > 0) {
    rcp_factors* done[MAX_BATCH];
    int status[MAX_BATCH], nd = 0;
    rc = engine_step(e, 1 << 20, stream, done, status, MAX_BATCH, &nd);
    for (int q = 0; q < nd && !rc; ++q) rc = status[q];
  }
  if (e) engine_destroy(e);
  if (rc) {
    delete f;
    return rc;
  }
  *out = f;
  return RCP_OK;
}

int rcp_solve3d(const rcp_factors* fc, const void* b_dev, void* x_dev, int32_t conj_transpose,
                rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f || !f->dim3) return fail(RCP_EINVAL, "factors of a 3D grid expected");
  if (!b_dev || !x_dev || b_dev == x_dev) return fail(RCP_EINVAL, "NULL or aliased vectors");
  return solve3d(f, static_cast<const double2*>(b_dev), static_cast<double2*>(x_dev),
                 conj_transpose ? 1 : 0, stream);
}

size_t rcp_average3d_work_bytes(const rcp_factors* f, const rcp_objective3d* o,
                                const rcp_light3d* L) {
  if (!f || !f->dim3 || !o || !L || L->ndir < 1) return 0;
  const size_t N = size_t(f->nx) * f->ny;
  const int m = o->kind == RCP_CONCENTRATOR ? 3 : 2;
  const size_t vals = size_t(m > 2 ? m : 2) * 2 * L->ndir;
  return align256(2 * m * N * 16) + align256(2 * N * 16) + align256(vals * 8);
}

int rcp_reciprocal_average3d(const rcp_factors* fc, const rcp_objective3d* o,
                             const rcp_light3d* L, double* F_dev, void* work_dev,
                             size_t work_bytes, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f || !f->dim3) return fail(RCP_EINVAL, "factors of a 3D grid expected");
  int rc = check_obj3d(f, o);
  if (!rc) rc = check_light3d(f, L);
  if (rc) return rc;
  if (!F_dev) return fail(RCP_EINVAL, "F_dev is NULL");
  const size_t need = rcp_average3d_work_bytes(f, o, L);
  if (!work_dev || work_bytes < need) return fail(RCP_ENOMEM, "3D workspace needs " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(work_dev) % 256 != 0)
    return fail(RCP_EINVAL, "workspace must be 256-byte aligned");
  const size_t N = size_t(f->nx) * f->ny;
  const int m = o->kind == RCP_CONCENTRATOR ? 3 : 2;
  char* w = static_cast<char*>(work_dev);
  double2* Wc = reinterpret_cast<double2*>(w);
  double2* Z = Wc + size_t(m) * N;
  double* vals = reinterpret_cast<double*>(w + align256(2 * m * N * 16) + align256(2 * N * 16));
  k_objective3d<<<static_cast<int>((N * m + 255) / 256), 256, 0, stream>>>(
      f->nx, f->gy, f->gz, f->npml, f->h, f->k0, *o, Wc, N);
  RCP_HIP(hipGetLastError());
  for (int c = 0; c < m; ++c) {   // one reciprocal solve per component: z = A^{-dag} w
    rc = solve3d(f, Wc + size_t(c) * N, Z + size_t(c) * N, 1, stream);
    if (rc) return rc;
  }
  k_plane_proj3d<<<m * 2 * L->ndir, 256, 0, stream>>>(f->nx, f->gy, f->gz, f->npml, f->h, f->k0,
                                                       L->k_s, L->n_s, L->dirs_dev, L->ndir, Z, N,
                                                       vals);
  RCP_HIP(hipGetLastError());
  k_weighted3d<<<1, 64, 0, stream>>>(L->dirs_dev, L->ndir, vals, m, 2, F_dev);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int rcp_brute_force_average3d(const rcp_factors* fc, const rcp_objective3d* o,
                              const rcp_light3d* L, double* F_dev, double* per_dev,
                              void* work_dev, size_t work_bytes, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f || !f->dim3) return fail(RCP_EINVAL, "factors of a 3D grid expected");
  int rc = check_obj3d(f, o);
  if (!rc) rc = check_light3d(f, L);
  if (rc) return rc;
  if (!F_dev) return fail(RCP_EINVAL, "F_dev is NULL");
  const size_t need = rcp_average3d_work_bytes(f, o, L);
  if (!work_dev || work_bytes < need) return fail(RCP_ENOMEM, "3D workspace needs " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(work_dev) % 256 != 0)
    return fail(RCP_EINVAL, "workspace must be 256-byte aligned");
  const size_t N = size_t(f->nx) * f->ny;
  const int m = o->kind == RCP_CONCENTRATOR ? 3 : 2;
  char* w = static_cast<char*>(work_dev);
  double2* Wc = reinterpret_cast<double2*>(w);
  double2* src = reinterpret_cast<double2*>(w + align256(2 * m * N * 16));
  double2* u = src + N;
  double* vals = per_dev ? per_dev
                         : reinterpret_cast<double*>(w + align256(2 * m * N * 16) + align256(2 * N * 16));
  k_objective3d<<<static_cast<int>((N * m + 255) / 256), 256, 0, stream>>>(
      f->nx, f->gy, f->gz, f->npml, f->h, f->k0, *o, Wc, N);
  RCP_HIP(hipGetLastError());
  std::vector<double> dirs(3 * size_t(L->ndir));
  RCP_HIP(hipMemcpyAsync(dirs.data(), L->dirs_dev, dirs.size() * 8, hipMemcpyDeviceToHost, stream));
  RCP_HIP(hipStreamSynchronize(stream));
  for (int d = 0; d < L->ndir; ++d) {   // one forward solve per direction and polarisation
    for (int pol = 0; pol < 2; ++pol) {
      k_source3d<<<static_cast<int>((N + 255) / 256), 256, 0, stream>>>(
          f->nx, f->gy, f->gz, f->npml, f->h, f->k0, L->k_s, L->n_s, dirs[3 * d], dirs[3 * d + 1],
          pol, src, N);
      RCP_HIP(hipGetLastError());
      rc = solve3d(f, src, u, 0, stream);
      if (rc) return rc;
      k_obj_amp3d<<<1, 256, 0, stream>>>(Wc, m, u, N, vals + 2 * d + pol);
      RCP_HIP(hipGetLastError());
    }
  }
  k_weighted3d<<<1, 64, 0, stream>>>(L->dirs_dev, L->ndir, vals, 1, 2, F_dev);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

}  // extern "C"

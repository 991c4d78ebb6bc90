// Permittivity map, PML stretches and the coefficients of the FDFD operator.
//
// The operator is the finite-difference form of the scalar (TM) Helmholtz
// problem u = A^{-1} b of Sec. "Reciprocal approach", with a stretched-
// coordinate PML, multiplied through by s_x s_y so that A = A^T:
//   coupling (i,j)-(i+1,j) = s_y(j) / (s_x(face i+1) h^2)
//   coupling (i,j)-(i,j+1) = s_x(i) / (s_y(face j+1) h^2)
//   diagonal              = -(sum of the four couplings, grid-boundary faces
//                             included) + k0^2 eps s_x(i) s_y(j)
// Neighbours outside the grid are dropped (u = 0 beyond the PML).
#include "rcp_internal.h"

namespace {

__device__ double2 pml_stretch(double xi, int n_axis, int npml, double h, double k0, double R,
                               int m) {
  double depth = fmax(fmax(npml - xi, xi - (n_axis - npml)), 0.0) * h;
  if (depth <= 0.0 || npml == 0) return make_double2(1.0, 0.0);
  double L = npml * h;
  double sigma = (m + 1) * log(1.0 / R) / (2.0 * k0 * L);
  double r = depth / L, p = 1.0;
  for (int e = 0; e < m; ++e) p *= r;
  return make_double2(1.0, sigma * p);
}

__global__ void k_stretch(int nx, int ny, int npml, double h, double k0, double R, int m,
                          double2* sxc, double2* sxf, double2* syc, double2* syf) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nx) sxc[t] = pml_stretch(t + 0.5, nx, npml, h, k0, R, m);
  if (t <= nx) sxf[t] = pml_stretch(static_cast<double>(t), nx, npml, h, k0, R, m);
  if (t < ny) syc[t] = pml_stretch(t + 0.5, ny, npml, h, k0, R, m);
  if (t <= ny) syf[t] = pml_stretch(static_cast<double>(t), ny, npml, h, k0, R, m);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) { return cmul(a, cinv(b)); }

__global__ void k_coefs(int nx, int ny, double h, double k0, const double* __restrict__ eps,
                        const double2* __restrict__ sxc, const double2* __restrict__ sxf,
                        const double2* __restrict__ syc, const double2* __restrict__ syf,
                        double* __restrict__ eps_copy, double2* __restrict__ dco,
                        double2* __restrict__ eco, double2* __restrict__ cco) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(nx) * ny) return;
  int i = static_cast<int>(q / ny), j = static_cast<int>(q % ny);
  double ih2 = 1.0 / (h * h);
  double2 cxm = cscale(cdiv(syc[j], sxf[i]), ih2);
  double2 cxp = cscale(cdiv(syc[j], sxf[i + 1]), ih2);
  double2 cym = cscale(cdiv(sxc[i], syf[j]), ih2);
  double2 cyp = cscale(cdiv(sxc[i], syf[j + 1]), ih2);
  double e = eps[q];
  eps_copy[q] = e;
  double2 kk = cscale(cmul(sxc[i], syc[j]), k0 * k0 * e);
  double2 s = cadd(cadd(cxm, cxp), cadd(cym, cyp));
  dco[q] = csub(kk, s);
  eco[q] = (j + 1 < ny) ? cyp : make_double2(0.0, 0.0);
  cco[q] = (i + 1 < nx) ? cxp : make_double2(0.0, 0.0);
}

__device__ double overlap(double x_lo, double x_hi, double c, double w) {
  double lo = fmax(x_lo, c - 0.5 * w), hi = fmin(x_hi, c + 0.5 * w);
  return fmax(hi - lo, 0.0);
}

__global__ void k_eps(int nx, int ny, int npml, double h, int npil,
                      const double* __restrict__ centers, const double* __restrict__ widths,
                      double eps_bg, double eps_sub, double eps_pil, int sub_rows, int row0,
                      int rows, double* __restrict__ eps) {
  size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= size_t(nx) * ny) return;
  int i = static_cast<int>(q / ny), j = static_cast<int>(q % ny);
  double e = eps_bg;
  if (j < sub_rows) e = eps_sub;
  if (j >= row0 && j < row0 + rows) {
    double xc = (i - npml + 0.5) * h;
    double frac = 0.0;
    for (int p = 0; p < npil; ++p) frac += overlap(xc - 0.5 * h, xc + 0.5 * h, centers[p], widths[p]);
    e = eps_bg + (eps_pil - eps_bg) * (frac / h);
  }
  eps[q] = e;
}

// One wave per pillar: sums dF/deps over the pillar rows of the two cells that
// hold its edges (half-open cells: an edge on a face belongs to the right cell).
__global__ void k_width_grad(int nx, int ny, int npml, double h, int npil,
                             const double* __restrict__ centers, const double* __restrict__ widths,
                             double eps_bg, double eps_pil, int row0, int rows,
                             const double* __restrict__ g, double* __restrict__ gw) {
  int p = blockIdx.x;
  int lane = threadIdx.x;
  if (p >= npil) return;
  double x0 = -npml * h;
  double c = centers[p], w = widths[p];
  int il = static_cast<int>(floor((c - 0.5 * w - x0) / h));
  int ir = static_cast<int>(floor((c + 0.5 * w - x0) / h));
  double s = 0.0;
  for (int r = lane; r < rows; r += 64) {
    int j = row0 + r;
    if (il >= 0 && il < nx) s += g[size_t(il) * ny + j];
    if (ir >= 0 && ir < nx) s += g[size_t(ir) * ny + j];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) gw[p] = s * (eps_pil - eps_bg) / (2.0 * h);
}

}  // namespace

namespace rcp {

int launch_eps_from_widths(const rcp_grid* g, const rcp_pillars* p, double* eps, hipStream_t s) {
  size_t N = size_t(g->nx) * g->ny;
  int blocks = static_cast<int>((N + 255) / 256);
  k_eps<<<blocks, 256, 0, s>>>(g->nx, g->ny, g->npml, g->h, p->n, p->centers_dev, p->widths_dev,
                               p->eps_bg, p->eps_sub, p->eps_pillar, p->sub_rows, p->row0, p->rows,
                               eps);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int launch_assemble(rcp_factors* f, const double* eps_src, hipStream_t s) {
  int n = (f->nx > f->ny ? f->nx : f->ny) + 1;
  k_stretch<<<ceil_div(n, 256), 256, 0, s>>>(f->nx, f->ny, f->npml, f->h, f->k0, f->pml_R,
                                              f->pml_m, f->sxc, f->sxf, f->syc, f->syf);
  RCP_HIP(hipGetLastError());
  size_t N = size_t(f->nx) * f->ny;
  k_coefs<<<static_cast<int>((N + 255) / 256), 256, 0, s>>>(f->nx, f->ny, f->h, f->k0, eps_src,
                                                            f->sxc, f->sxf, f->syc, f->syf, f->eps,
                                                            f->dco, f->eco, f->cco);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

int launch_width_grad(const rcp_grid* g, const rcp_pillars* p, const double* grad_eps,
                      double* grad_w, hipStream_t s) {
  if (p->n <= 0) return RCP_OK;
  k_width_grad<<<p->n, 64, 0, s>>>(g->nx, g->ny, g->npml, g->h, p->n, p->centers_dev,
                                   p->widths_dev, p->eps_bg, p->eps_pillar, p->row0, p->rows,
                                   grad_eps, grad_w);
  RCP_HIP(hipGetLastError());
  return RCP_OK;
}

}  // namespace rcp

/*
 * recip.h -- C ABI of librecip: the reciprocal angle average of incoherent light
 * through a 2D metasurface, on one AMD Instinct MI355X (gfx950).
 *
 * Method (Pestourie, Yao, Kante, Johnson, "Efficient inverse design of
 * large-area metasurfaces for incoherent light"):
 *   - Sec. "Reciprocal approach", Eq. 7: the angle-averaged figure of merit
 *     <|w^dag u|^2> equals v^dag W v, with v = A^{-dag} w the field of ONE
 *     "reciprocal" solve (the objective w used as the source), restricted to
 *     the incidence line, and W the cross-correlation of the equivalent source
 *     currents there.
 *   - Sec. "Incoherent light", Eq. 3-4 and the annulus formula of Sec.
 *     "Designs": for angle-uncorrelated light W(x1, x2) = C(x1 - x2) is
 *     Toeplitz, so W v is a convolution evaluated by FFT.
 *   - Eq. 6: the brute-force average it replaces integrates |w^dag u(theta)|^2
 *     over incident angles, one forward solve per quadrature node
 *     (Sec. "Brute-force quadrature": Gauss-Legendre in theta).
 *   - Sec. "Reciprocal approach": gradient 2 Re(v^dag W grad v) by one adjoint
 *     solve.
 *
 * The operator A is the symmetric stretched-coordinate PML finite-difference
 * form of (laplacian + k0^2 eps) u = -f, multiplied through by s_x s_y, on an
 * nx x ny cell grid.  It is block tridiagonal along x (block i = grid column i,
 * block size ny) and is factored by a two-ended (twisted) block elimination
 * whose dense Schur-complement blocks are inverted by a symmetric blocked
 * Gauss-Jordan sweep on MFMA.
 *
 * Conventions
 *   - Complex arrays are interleaved (re, im): double[2] per element
 *     (torch.complex128) unless stated otherwise.
 *   - Grid fields are x-major: cell (i, j) is element q = i * ny + j.
 *   - Cell (i, j) has its centre at x = (i - npml + 1/2) h,
 *     y = (j - npml + 1/2) h; the physical region is
 *     npml <= i < nx - npml, npml <= j < ny - npml.
 *   - All pointers named *_dev are device pointers owned by the caller; the
 *     library never frees caller memory.  The library owns only the small host
 *     handle returned by rcp_factor.
 *   - Every call enqueues on `stream` and returns without waiting, except
 *     where stated (rcp_factor and rcp_factor_batch wait once to read the
 *     pivot check, which rcp_factor_batch_async leaves on the device;
 *     refined solves wait once per refinement step to test convergence).
 *   - Calls that use the same rcp_factors must be ordered on one stream: they
 *     share work vectors inside the factor buffer.
 *   - Return value: 0 on success, or a negative RCP_E* code; the message of
 *     the last failure on the calling thread is returned by rcp_last_error().
 *     No C++ exception crosses this interface.
 */
#ifndef RECIP_H
#define RECIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rcp_stream; /* a hipStream_t; NULL = default stream */

enum {
  RCP_OK = 0,
  RCP_EINVAL = -1,     /* bad shape, index outside the physical region, bad light, ... */
  RCP_ENOMEM = -2,     /* caller buffer smaller than required                          */
  RCP_ESINGULAR = -3,  /* non-finite or vanishing pivot; message names the block       */
  RCP_ENOCONV = -4,    /* refinement did not reach tol; message gives the residual      */
  RCP_EHIP = -5        /* HIP runtime error                                             */
};

enum { RCP_FP64 = 0, RCP_FP32_REFINED = 1 };
enum { RCP_CONCENTRATOR = 0, RCP_COLLIMATOR = 1 };
enum { RCP_CONE = 0, RCP_ANNULUS = 1, RCP_SYMBOL_TABLE = 2 };

/* Grid and PML.  PML stretch s(xi) = 1 + i sigma (d/L)^m with d the depth into
 * the layer, L = npml h, sigma = (m+1) ln(1/pml_R) / (2 k0 L).  k0 = 2 pi /
 * vacuum wavelength.  eps_dev: nx*ny float64 cell permittivities (device);
 * copied into the factor buffer by rcp_factor. */
typedef struct {
  int32_t nx, ny, npml;
  double h, k0;
  double pml_R;
  int32_t pml_m;
  const double* eps_dev;
} rcp_grid;

/* Pillar layer (Sec. "Designs": a single layer of dielectric pillars on a
 * substrate).  Rows j < sub_rows hold eps_sub; rows [row0, row0 + rows) hold
 * pillars of permittivity eps_pillar centred at centers_dev[p] (physical x)
 * with widths widths_dev[p]; each cell takes the arithmetic mean of eps over
 * its x extent.  Everything else is eps_bg.  Arrays are device float64. */
typedef struct {
  int32_t n;
  const double* centers_dev;
  const double* widths_dev;
  double eps_bg, eps_sub, eps_pillar;
  int32_t sub_rows, row0, rows;
} rcp_pillars;

/* Objective w (Sec. "Reciprocal approach": FOM |w^dag u|^2).
 *   CONCENTRATOR: w = e_q at the focus cell (i_f, j_f): w^dag u = u(focus).
 *   COLLIMATOR:   w = (h / L) exp(i k0 n_m sin(phi) x) on row j_m over columns
 *                 [i0, i1), L = (i1 - i0) h: w^dag u is the amplitude of the
 *                 planewave output mode at angle phi. */
typedef struct {
  int32_t kind;
  int32_t i_f, j_f;
  int32_t j_m, i0, i1;
  double phi, n_m;
} rcp_objective;

/* Incoherent light on the incidence line: row j_s, columns [i0, i1) (M cells),
 * medium index n_s; angles theta are measured in that medium.
 *   CONE:    <|a|^2> = 1/(2c) on [-c, c]
 *   ANNULUS: <|a|^2> = 1/(2(th2 - th1)) on [-th2, -th1] u [th1, th2]
 *   SYMBOL_TABLE: symbol_dev holds 2M-1 complex128 values C(m h),
 *                 m = -(M-1) .. M-1 (index m + M - 1); C(-d) = conj C(d).
 * The equivalent source of a unit-power planewave is the line current
 * J(theta) = -2 i k0 sqrt(n_s cos theta) spread over one cell height, so
 * C(d) = int <|a|^2> |J|^2 / h^2 exp(i K d sin theta) dtheta, K = n_s k0. */
typedef struct {
  int32_t j_s, i0, i1;
  double n_s;
  int32_t kind;
  double c, th1, th2;
  const double* symbol_dev;
} rcp_light;

typedef struct rcp_factors rcp_factors;

typedef struct {
  int32_t iters;         /* refinement steps taken (0 for plain FP64)        */
  double rel_residual;   /* ||b - A x|| / ||b|| after the last step (refined) */
} rcp_solve_stats;

/* a1 -- permittivity map from pillar widths (Sec. "Designs"; widths are the
 * design parameters p of Sec. "Reciprocal approach").  eps_out_dev: nx*ny
 * float64.  grid->eps_dev is ignored. */
int rcp_eps_from_widths(const rcp_grid* grid, const rcp_pillars* pillars,
                        double* eps_out_dev, rcp_stream stream);

/* Bytes of device memory rcp_factor needs for this grid and precision
 * (factor blocks, operator coefficients, work vectors and scratch of the
 * solves).  Exact; serving
 * admits requests by this number.  Returns 0 for an invalid grid. */
size_t rcp_factor_bytes(const rcp_grid* grid, int32_t precision);

/* a2 + a3 -- assemble A (Sec. "Reciprocal approach": u = A^{-1} b) and factor
 * it: twisted block elimination along x, every Schur-complement block
 * inverted on the GPU (complex128 for RCP_FP64, complex64 for
 * RCP_FP32_REFINED).  buf_dev: caller buffer of at least
 * rcp_factor_bytes(grid, precision) bytes, 256-byte aligned; it must stay
 * alive and untouched while *out is used.  Waits for the stream once at the
 * end to read the device pivot check (RCP_ESINGULAR names the first bad
 * block); rcp_factor_batch_async does not wait. */
int rcp_factor(const rcp_grid* grid, int32_t precision, void* buf_dev, size_t buf_bytes,
               rcp_stream stream, rcp_factors** out);

/* a2 + a3 for `count` (1..16) geometries of identical grid shape (eps and k0
 * may differ: several wavelengths of one geometry factor side by side),
 * factored in the same kernel launches (their elimination chains run side by
 * side, two Gauss-Jordan panels per pass over the tiles; a lone geometry takes
 * one panel per launch, so its factors agree with a batch's to rounding).
 * Above 8 the geometries form two groups ([0, ceil(count/2)) and the rest),
 * each factored in its own launches on one of two streams that the library
 * creates per device (default priority, kept until the process ends), forked
 * from and joined back into `stream`; one call enqueues the second group from
 * a host thread of its own.  A geometry's factors are the same in any batch of
 * two or more, so they do not depend on the grouping.
 * grids[g], bufs[g] (each buf_bytes >= rcp_factor_bytes, 256-byte aligned,
 * non-overlapping) and out[g] as for rcp_factor.  On failure no
 * handle is returned and the message names the geometry. */
int rcp_factor_batch(int32_t count, const rcp_grid* grids, int32_t precision, void* const* bufs,
                     size_t buf_bytes, rcp_stream stream, rcp_factors** out);

/* a2 + a3 as rcp_factor_batch, enqueued only: returns the handles at once and
 * never waits.  The pivot check runs on the device after the factorisation
 * and leaves each set's status word (0 when every pivot passed, else 1 + the
 * first failing panel, block-major); until it has been read the results of
 * calls on the set are those of a factorisation that may have failed (a
 * singular block gives infinite or NaN fields).  Argument checks and errors
 * as rcp_factor_batch. */
int rcp_factor_batch_async(int32_t count, const rcp_grid* grids, int32_t precision,
                           void* const* bufs, size_t buf_bytes, rcp_stream stream,
                           rcp_factors** out);
/* The pivot check of set f: waits for `stream` (on which its factorisation was
 * enqueued), then RCP_OK or RCP_ESINGULAR (naming the panel and its block). */
int rcp_factors_status(const rcp_factors* f, rcp_stream stream);
/* Device address of f's status word (int32, inside the factor buffer), for
 * callers that read it on their own stream or in their own kernels; valid
 * after the factorisation's launches on its stream.  NULL for NULL f. */
const int32_t* rcp_factors_status_dev(const rcp_factors* f);

/* a3 + a11 -- the factorisation engine: geometries of any grid size factored
 * in shared kernel launches, admitted while others are in progress
 * (continuous batching of the factorisation).  Every geometry's chains
 * (twisted block elimination, two Gauss-Jordan panels per pass) advance one
 * pass per round; a round carries every chain of every geometry in flight, so
 * small and large requests fill the GPU together.  The factors of a geometry
 * are bit-identical to rcp_factor_batch's for the same grid (batch of two or
 * more) whatever else shares the launches.  One precision per engine; at
 * most 8 geometries in flight; blocks of more than 32 rows (ny > 32).  The
 * engine is not thread-safe: one host thread drives it. */
typedef struct rcp_engine rcp_engine;
int rcp_engine_create(int32_t precision, rcp_engine** out);
/* Frees the engine.  Handles of geometries still in flight stay the caller's
 * (release them); their factors are incomplete. */
void rcp_engine_destroy(rcp_engine* e);
/* Admit a geometry: checks as rcp_factor, assembles the operator on stream and
 * returns its handle in *out; its factorisation advances from the engine's
 * next round.  The handle must not be used or released before a step reports
 * it done.  RCP_EINVAL when 8 geometries are in flight.  buf_dev as for
 * rcp_factor (caller-owned, rcp_factor_bytes, 256-byte aligned). */
int rcp_engine_add(rcp_engine* e, const rcp_grid* grid, void* buf_dev, size_t buf_bytes,
                   rcp_stream stream, rcp_factors** out);
/* Enqueue up to `rounds` rounds on stream, returning after the first round in
 * which some geometry completes.  done[0 .. *n_done - 1] get the completed
 * handles and status[] their pivot check (RCP_OK or RCP_ESINGULAR, checked
 * with one wait for the stream per step that completes geometries); cap >= 8.
 * *n_active (may be NULL): geometries still in flight.  Work enqueued on
 * stream; a completed handle is usable in stream order. */
int rcp_engine_step(rcp_engine* e, int32_t rounds, rcp_stream stream, rcp_factors** done,
                    int32_t* status, int32_t cap, int32_t* n_done, int32_t* n_active);

/* Solve A X = B for nrhs right-hand sides (or A^dag X = B when
 * conj_transpose != 0, using A = A^T).  B_dev, X_dev: nrhs x nx x ny
 * complex128 (row r is one grid field); B_dev and X_dev must not overlap
 * (RCP_EINVAL).  RCP_FP32_REFINED factors: iterative refinement with FP64 residuals
 * until ||r|| / ||b|| <= tol or max_refine steps (RCP_ENOCONV); each step
 * waits for the stream.  tol and max_refine are ignored for RCP_FP64.
 * stats may be NULL. */
int rcp_solve_multi_rhs(const rcp_factors* f, int32_t nrhs, const void* B_dev, void* X_dev,
                        int32_t conj_transpose, double tol, int32_t max_refine,
                        rcp_stream stream, rcp_solve_stats* stats);

/* a4-a7 -- Eq. 7: F = v^dag W v with v = A^{-dag} w on the incidence line, W v
 * by circulant embedding and FFT.  F_dev: one float64.  Optional outputs
 * (NULL to skip): v_dev (M complex128), z_dev (nx*ny complex128, the whole
 * reciprocal field A^{-dag} w). */
int rcp_reciprocal_average(const rcp_factors* f, const rcp_objective* obj,
                           const rcp_light* light, double* F_dev, void* v_dev, void* z_dev,
                           rcp_stream stream);

/* Device workspace rcp_brute_force_average needs for nangles nodes solved
 * rhs_chunk at a time (node tables, line sources, one chunk of fields and,
 * for rhs_chunk >= 64, 64 MiB of partial sums that balance each block
 * product's tiles over the compute units). */
size_t rcp_brute_force_work_bytes(const rcp_factors* f, int32_t nangles, int32_t rhs_chunk);

/* a8 -- Eq. 6 by nangles-point Gauss-Legendre quadrature in theta (split evenly
 * over the two intervals of an annulus): one forward solve per node, in
 * chunks of rhs_chunk right-hand sides on the same factors.  F_dev: one
 * float64; per_angle_dev (optional, nangles float64): |w^dag u(theta_q)|^2 in
 * node order (ascending theta).  RCP_FP64 factors and CONE / ANNULUS light only. */
int rcp_brute_force_average(const rcp_factors* f, const rcp_objective* obj,
                            const rcp_light* light, int32_t nangles, int32_t rhs_chunk,
                            void* work_dev, size_t work_bytes, double* F_dev,
                            double* per_angle_dev, rcp_stream stream);

/* a9 -- gradient of F (Sec. "Reciprocal approach"): lambda = A^{-1} P^T (W v),
 * dF/deps_q = -2 k0^2 Re(conj(lambda_q) conj(s_x s_y)_q z_q), from one extra
 * solve.  F_dev: one float64 (same value as rcp_reciprocal_average);
 * grad_eps_dev: nx*ny float64. */
int rcp_adjoint_grad(const rcp_factors* f, const rcp_objective* obj, const rcp_light* light,
                     double* F_dev, double* grad_eps_dev, rcp_stream stream);

/* a9 for `count` (1..8) factor sets of identical grid and precision, e.g.
 * from one rcp_factor_batch call: the same computation as rcp_adjoint_grad
 * for each set g with objs[g] and lights[g], results bit-identical to it.
 * With RCP_FP64 factors the two solves of all sets advance in the same
 * kernel launches.  F_dev: count float64 (device); grad_eps_dev: count
 * device pointers (host array), each nx*ny float64.  A set may appear once. */
int rcp_adjoint_grad_batch(int32_t count, rcp_factors* const* factors,
                           const rcp_objective* objs, const rcp_light* lights, double* F_dev,
                           double* const* grad_eps_dev, rcp_stream stream);

/* a11 -- several evaluations on one cached factor set (requests for the same
 * geometry with their own objectives and lights, Eq. 7 each): F_k = v_k^dag
 * T_k v_k with v_k = (A^{-dag} w_k) on the incidence line of lights[k] and
 * T_k its Toeplitz correlation.  RCP_FP64 factors with count >= 2 solve all
 * objectives in one multi-RHS sweep (every factor block read once for all of
 * them); otherwise one (refined) solve per objective.  Each F_k equals
 * rcp_reciprocal_average with objs[k] and lights[k] to rounding.  F_dev:
 * count float64 (device).  work_dev: at least
 * rcp_reciprocal_many_work_bytes(f, count) bytes, 256-byte aligned, scratch
 * (RCP_EINVAL when misaligned).  count 1..64; RCP_ENOMEM when work_bytes is
 * short. */
size_t rcp_reciprocal_many_work_bytes(const rcp_factors* f, int32_t count);
int rcp_reciprocal_average_many(const rcp_factors* f, int32_t count, const rcp_objective* objs,
                                const rcp_light* lights, double* F_dev, void* work_dev,
                                size_t work_bytes, rcp_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluations as rcp_reciprocal_average_many (same checks, same kernels, the
 * same F to the bit) with the workspace taken from a static device array of
 * RCP_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends, instead of work_dev.  Allocates nothing.  Its
 * address on a device is looked up on the first call with that device
 * current.  RCP_ENOMEM when rcp_reciprocal_many_work_bytes(f, count) exceeds
 * the array (2 count nx ny complex128 values: e.g. count <= 3 on a 2040 x 1080
 * grid).  All calls on one GPU share its array: calls that overlap in time on
 * one GPU (other streams, other host threads) race and give wrong results;
 * order them on one stream.  The workspace is written before it is read, so
 * nothing carries over from the previous call. */
#define RCP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int rcp_reciprocal_average_many_noalloc(const rcp_factors* f, int32_t count,
                                        const rcp_objective* objs, const rcp_light* lights,
                                        double* F_dev, rcp_stream stream);

/* ---- any correlation W and many outputs --------------------------------
 * Sec. "Incoherent light": the reciprocal identity of Eq. 7 holds for
 * arbitrarily correlated light, where W is a dense Hermitian M x M matrix on
 * the incidence line rather than a Toeplitz one.  Sec. "Concluding remarks":
 * averages over many focal spots or output modes w_k add up to the trace form
 * sum_k v_k^dag W v_k, one reciprocal solve per output on the same factors.
 * Only j_s, i0, i1 and n_s of `line` are used here (M = i1 - i0 cells); its
 * kind and angles are ignored.  W_dev: M x M complex128, row-major,
 * W[j][l] = W(x_j, x_l) with x_j the centre of column i0 + j; W is taken as
 * Hermitian (the real part of each form is returned).  work_dev: at least the
 * bytes reported by the *_work_bytes call, 256-byte aligned, not overlapping
 * any other argument; its contents are scratch. */

/* Device workspace of the two dense-form calls for nout (1..4096) outputs on an
 * m-cell line (0 for invalid arguments). */
size_t rcp_dense_work_bytes(const rcp_factors* f, int32_t nout, int32_t m);

/* F_k = v_k^dag W v_k with v_k = (A^{-dag} w_k) on the line, for the nout
 * outputs objs[k] (W V on the matrix cores).  F_dev: nout + 1 float64, F_k
 * then the sum over k.  V_dev (optional, NULL to skip): nout x M complex128,
 * row k = v_k.  RCP_FP64 factors with nout >= 2 solve all outputs in one
 * multi-RHS sweep; otherwise one (refined) solve per output. */
int rcp_reciprocal_average_dense(const rcp_factors* f, int32_t nout, const rcp_objective* objs,
                                 const rcp_light* line, const void* W_dev, double* F_dev,
                                 void* V_dev, void* work_dev, size_t work_bytes,
                                 rcp_stream stream);

/* Gradient of sum_k F_k (Sec. "Reciprocal approach", one adjoint solve per
 * output): lambda_k = A^{-1} P^T (W v_k),
 * d(sum F)/deps_q = -2 k0^2 Re(conj(s_x s_y)_q sum_k conj(lambda_kq) z_kq).
 * F_dev: nout + 1 float64 as above; grad_eps_dev: nx*ny float64. */
int rcp_adjoint_grad_dense(const rcp_factors* f, int32_t nout, const rcp_objective* objs,
                           const rcp_light* line, const void* W_dev, double* F_dev,
                           double* grad_eps_dev, void* work_dev, size_t work_bytes,
                           rcp_stream stream);

/* Device workspace of rcp_correlation_matrix (0 for invalid arguments). */
size_t rcp_correlation_work_bytes(int32_t m, int32_t nangles);

/* Eq. 1 and 3 for a finite ensemble: light made of nangles planewaves at
 * angles theta_dev[q] (float64, radians in the source medium, |theta| < pi/2)
 * whose random amplitudes have correlation C_dev[q][q'] = <a_q conj(a_q')>
 * (nangles x nangles complex128, row-major) has the line correlation
 * W = G C G^dag, G[j][q] = b0(theta_q) at column i0 + j, b0 the unit-power
 * equivalent source above.  W_dev: M x M complex128, row-major.  Uses nx,
 * npml, h and k0 of grid (eps_dev is ignored). */
int rcp_correlation_matrix(const rcp_grid* grid, const rcp_light* line, int32_t nangles,
                           const double* theta_dev, const void* C_dev, void* W_dev,
                           void* work_dev, size_t work_bytes, rcp_stream stream);

/* Broadband (Sec. "Method": the single-wavelength calculation repeated at
 * several wavelengths; Sec. "Concluding remarks": the frequency integral as a
 * weighted quadrature over the spectrum).  count (1..8) factor sets of one
 * grid shape and precision, typically one rcp_factor_batch call whose grids
 * differ in k0 (the wavelengths of the rule; eps too if the material is
 * dispersive), with objs[g] and lights[g] at that wavelength and host weights
 * weights[g]: F_dev (count + 1 float64) receives F_g then sum_g weights[g] F_g;
 * grad_eps_dev (nx*ny float64) receives sum_g weights[g] dF_g/deps.  Uses each
 * set's work vectors as scratch (calls on a set must be ordered on one
 * stream). */
int rcp_broadband_grad(int32_t count, rcp_factors* const* factors, const rcp_objective* objs,
                       const rcp_light* lights, const double* weights, double* F_dev,
                       double* grad_eps_dev, rcp_stream stream);

/* a1 backward -- chain rule from dF/deps to dF/dwidth_p: each pillar edge moves
 * by dw/2 and changes the fill of the cell holding it by dw/(2h) in every
 * pillar row.  grad_w_dev: pillars->n float64. */
int rcp_width_grad(const rcp_grid* grid, const rcp_pillars* pillars, const double* grad_eps_dev,
                   double* grad_w_dev, rcp_stream stream);

/* ---- 3D (Sec. "Concluding remarks") -------------------------------------
 * curl curl E - k0^2 eps E = i k0 J on a Yee grid of nx x ny x nz cells
 * (E_x at ((i+1/2)h, jh, kh), E_y at (ih, (j+1/2)h, kh), E_z at (ih, jh,
 * (k+1/2)h), tangential E zero beyond the grid) with the uniaxial form of the
 * stretched-coordinate PML (same profile as the 2D operator on every axis);
 * A is complex symmetric.  Fields and eps are in slice order: index
 * i n + (c ny + j) nz + k with n = 3 ny nz (x-slice i, component c).  The
 * factorisation is the same two-ended block elimination over the x-slices
 * (blocks of n unknowns, 33 <= n <= 65536) with sparse couplings between
 * slices.  FP64 only.  In 3D the reciprocal average takes one solve per field
 * component the objective reads: three for the intensity |E|^2 at a focal
 * spot, two for the power in an output planewave mode. */
typedef struct {
  int32_t nx, ny, nz, npml;
  double h, k0, pml_R;
  int32_t pml_m;
  const double* eps_dev;   /* 3 nx ny nz float64, slice order (device) */
} rcp_grid3d;

/* Square pillars of side widths_dev[p] centred at (centers_dev[2p],
 * centers_dev[2p+1]) (physical coordinates, origin at the lower corner of the
 * physical region) in the z-layers [pillar_k0, pillar_k0 + pillar_layers) (cell
 * units, grid index), substrate below sub_layers; each E component takes the
 * mean of eps over the h x h square around its (x, y). */
typedef struct {
  int32_t n;
  const double* centers_dev;
  const double* widths_dev;
  double eps_bg, eps_sub, eps_pillar;
  int32_t sub_layers, pillar_k0, pillar_layers;
} rcp_pillars3d;

/* CONCENTRATOR: F reads the three components on the edges of cell (i_f, j_f,
 * k_f): |E|^2 there.  COLLIMATOR: the two polarisations (s, p) of the output
 * planewave in direction (theta, azimuth) (medium index n_m) on plane k_m,
 * w = (h^2 / area) e_pol exp(i k0 n_m sin theta (cos az x + sin az y)) on the
 * tangential components of the physical cells. */
typedef struct {
  int32_t kind;
  int32_t i_f, j_f, k_f;
  int32_t k_m;
  double theta, azimuth, n_m;
} rcp_objective3d;

/* Incoherent light on plane k_s (medium index n_s): ndir directions with
 * dirs_dev[3d .. 3d+2] = (theta, azimuth, weight), the weight including the
 * mean-square amplitude <|a|^2> of the direction; both polarisations carry
 * the same weight and are uncorrelated.  The unit-power sheet currents are
 * |J_s| = 2 sqrt(n_s cos theta) (normal to the plane of incidence) and
 * |J_p| = 2 sqrt(n_s / cos theta) (along the tangential wavevector), with the
 * phase exp(i k0 n_s sin theta (cos az x + sin az y)); b = i k0 J / h. */
typedef struct {
  int32_t k_s;
  double n_s;
  int32_t ndir;
  const double* dirs_dev;
} rcp_light3d;

/* 3D permittivity from pillars (eps_out_dev: 3 nx ny nz float64, slice order). */
int rcp_eps3d_from_pillars(const rcp_grid3d* grid, const rcp_pillars3d* pillars,
                           double* eps_out_dev, rcp_stream stream);
/* Bytes of the caller buffer rcp_factor3d needs (0 for an invalid grid). */
size_t rcp_factor3d_bytes(const rcp_grid3d* grid);
/* Assemble and factor; waits for the stream once (pivot check, RCP_ESINGULAR). */
int rcp_factor3d(const rcp_grid3d* grid, void* buf_dev, size_t buf_bytes, rcp_stream stream,
                 rcp_factors** out);
/* x = A^{-1} b, or A^{-dag} b = conj(A)^{-1} b when conj_transpose != 0 (nx n
 * complex128 each, slice order, not aliased). */
int rcp_solve3d(const rcp_factors* f, const void* b_dev, void* x_dev, int32_t conj_transpose,
                rcp_stream stream);
/* Workspace of the two 3D averages (256-byte aligned). */
size_t rcp_average3d_work_bytes(const rcp_factors* f, const rcp_objective3d* obj,
                                const rcp_light3d* light);
/* Eq. 7 in 3D: one reciprocal solve z_c = A^{-dag} w_c per component the
 * objective reads, then F = sum_c v_c^dag W v_c on the incidence plane with
 * W = sum_d weight_d (b_s b_s^dag + b_p b_p^dag), evaluated as
 * sum_c sum_d weight_d (|b_s^dag v_c|^2 + |b_p^dag v_c|^2).  F_dev: one float64. */
int rcp_reciprocal_average3d(const rcp_factors* f, const rcp_objective3d* obj,
                             const rcp_light3d* light, double* F_dev, void* work_dev,
                             size_t work_bytes, rcp_stream stream);
/* Eq. 6 in 3D: one forward solve per direction and polarisation (2 ndir),
 * F = sum_d weight_d sum_pol sum_c |w_c^dag E_(d,pol)|^2.  per_dev (optional,
 * 2 ndir float64): the value of each (direction, polarisation).  Waits for the
 * stream once to read the directions. */
int rcp_brute_force_average3d(const rcp_factors* f, const rcp_objective3d* obj,
                              const rcp_light3d* light, double* F_dev, double* per_dev,
                              void* work_dev, size_t work_bytes, rcp_stream stream);

/* Releases the host handle only; buf_dev stays with the caller. */
void rcp_factors_release(rcp_factors* f);

/* Message of the last failing call on this thread ("" if none). */
const char* rcp_last_error(void);

/* Iteration count and final relative residual of the last refined solve made
 * by rcp_reciprocal_average / rcp_adjoint_grad on these factors. */
int rcp_last_solve_stats(const rcp_factors* f, rcp_solve_stats* stats);

/* Launch timing for benchmarks (not thread-safe across concurrent timing
 * sessions).  rcp_timing_start(k) brackets every k-th launch of each kernel
 * class with HIP events on the launching stream (k = 0 turns timing off);
 * rcp_timing_stop waits for those events and fills stats[c] for the classes
 *   0 Gauss-Jordan panels formed apart from a tile update (first panel of a
 *     block; for batches the row tiles of each next pair of panels, and the
 *     pass that opens a block with the pivot work of panels 0 and 1 when the
 *     Schur-complement launch did not carry it)     work = algorithmic flops
 *   1 Gauss-Jordan tile update: for batches panels k, k+1 in one pass with
 *     the pivot work of panels k+2, k+3; for one geometry update k fused
 *     with panel k+1                                  work = algorithmic flops
 *   2 Schur-complement formation (for batches with the pivot work that opens
 *     the next block)               work = bytes of factor blocks read + written
 *   3 single-RHS block product     work = bytes of factor blocks read
 *   4 multi-RHS block GEMM         work = algorithmic flops (8 per complex MAC)
 *   5 Gauss-Jordan last pass of a block (negated)    work = algorithmic flops
 *   6 dense complex product (W V, ensemble W)        work = algorithmic flops
 *   7 launches of the factorisation engine (steps, row tiles, final
 *     updates of mixed geometries)                   work = algorithmic flops
 * launches counts every launch, samples / ms / work only the timed ones. */
#define RCP_NKCLASS 8
typedef struct {
  int64_t launches, samples;
  double ms, work;
} rcp_kernel_stat;
int rcp_timing_start(int32_t sample_every);
int rcp_timing_stop(rcp_kernel_stat* stats, int32_t n);

/* Introspection for tests and benchmarks. */
int rcp_factors_info(const rcp_factors* f, int32_t* nx, int32_t* ny, int32_t* precision,
                     int32_t* padded_n, int32_t* tile);

#ifdef __cplusplus
}
#endif
#endif /* RECIP_H */

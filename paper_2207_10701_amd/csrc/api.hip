// C ABI of librecip (declared in include/recip.h): argument checks, buffer
// layout, and the host-side order of the steps of each call.
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "rcp_internal.h"

namespace rcp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return RCP_EHIP;
}

Layout compute_layout(int nx, int ny, int precision) {
  Layout L{};
  const int np = ceil_div(ny, TB) * TB, nt = np / TB;
  const size_t tiles = size_t(nt) * (nt + 1) / 2;
  const size_t eb = precision == RCP_FP64 ? 16 : 8;
  const size_t N = size_t(nx) * ny;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.off_X = take(size_t(nx) * tiles * TB * TB * eb);
  L.off_eps = take(N * 8);
  L.off_sxc = take(size_t(nx) * 16);
  L.off_sxf = take(size_t(nx + 1) * 16);
  L.off_syc = take(size_t(ny) * 16);
  L.off_syf = take(size_t(ny + 1) * 16);
  L.off_dco = take(N * 16);
  L.off_eco = take(N * 16);
  L.off_cco = take(N * 16);
  L.off_L = take(8 * size_t(np) * TB * eb);
  L.off_Q = take(8 * size_t(np) * TB * eb);
  L.off_P = take(8 * size_t(TB) * TB * 16);
  L.off_health = take(size_t(nx) * nt * 8);
  L.off_vec = take(NVEC * N * 16);
  L.off_red = take((2 + 2 * ((N + 255) / 256)) * 8);
  size_t cap = 2;
  while (cap < 2 * size_t(nx)) cap <<= 1;
  L.off_fft = take(4 * cap * 16);
  L.off_part = take(2 * 2 * tiles * TB * 16);
  L.off_status = take(4);
  L.total = o;
  return L;
}

// ---- launch timing ---------------------------------------------------------
namespace {
struct TimerSample {
  int cls;
  hipEvent_t e0, e1;
  double work;
};
struct TimerState {
  std::mutex mu;
  int every = 0;
  long long launches[K_NCLASS] = {};
  std::vector<TimerSample*> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
TimerState g_timer;
}  // namespace

void ktimer_begin(int cls, hipStream_t s, double work, void** token) {
  *token = nullptr;
  if (g_timer.every <= 0) return;
  std::lock_guard<std::mutex> lk(g_timer.mu);
  long long n = g_timer.launches[cls]++;
  if (n % g_timer.every) return;
  TimerSample* ts = new TimerSample{cls, g_timer.get(), g_timer.get(), work};
  if (!ts->e0 || !ts->e1 || hipEventRecord(ts->e0, s) != hipSuccess) {
    delete ts;
    return;
  }
  g_timer.pending.push_back(ts);
  *token = ts;
}

void ktimer_end(void* token, hipStream_t s) {
  (void)hipEventRecord(static_cast<TimerSample*>(token)->e1, s);
}

KSample ktimer_sample(int cls, double work) {
  KSample out;
  if (g_timer.every <= 0) return out;
  std::lock_guard<std::mutex> lk(g_timer.mu);
  long long n = g_timer.launches[cls]++;
  if (n % g_timer.every) return out;
  TimerSample* ts = new TimerSample{cls, g_timer.get(), g_timer.get(), work};
  if (!ts->e0 || !ts->e1) {
    delete ts;
    return out;
  }
  g_timer.pending.push_back(ts);
  out.e0 = ts->e0;
  out.e1 = ts->e1;
  return out;
}

static size_t fft_capacity(int nx) {
  size_t cap = 2;
  while (cap < 2 * size_t(nx)) cap <<= 1;
  return cap;
}


}  // namespace rcp

using namespace rcp;

namespace {

constexpr double kRefineTol = 1e-12;
constexpr int kRefineMax = 10;

int check_grid(const rcp_grid* g) {
  if (!g) return fail(RCP_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1) return fail(RCP_EINVAL, "nx and ny must be positive");
  if (g->npml < 0 || 2 * g->npml >= g->nx || 2 * g->npml >= g->ny)
    return fail(RCP_EINVAL, "PML layers overlap or leave no physical region");
  if (!(g->h > 0) || !(g->k0 > 0)) return fail(RCP_EINVAL, "h and k0 must be positive");
  if (g->npml > 0 && (!(g->pml_R > 0 && g->pml_R < 1) || g->pml_m < 0))
    return fail(RCP_EINVAL, "pml_R must lie in (0, 1) and pml_m >= 0");
  if (ceil_div(g->ny, TB) * TB > 2048) return fail(RCP_EINVAL, "ny above 2048 is not supported");
  return RCP_OK;
}

bool in_phys_x(const rcp_factors* f, int i) { return i >= f->npml && i < f->nx - f->npml; }
bool in_phys_y(const rcp_factors* f, int j) { return j >= f->npml && j < f->ny - f->npml; }

int check_objective(const rcp_factors* f, const rcp_objective* o) {
  if (f->dim3) return fail(RCP_EINVAL, "factors of a 3D grid: use the rcp_*3d calls");
  if (!o) return fail(RCP_EINVAL, "objective is NULL");
  if (o->kind == RCP_CONCENTRATOR) {
    if (!in_phys_x(f, o->i_f) || !in_phys_y(f, o->j_f))
      return fail(RCP_EINVAL, "focus cell outside the physical region");
  } else if (o->kind == RCP_COLLIMATOR) {
    if (!in_phys_y(f, o->j_m)) return fail(RCP_EINVAL, "monitor row outside the physical region");
    if (o->i0 >= o->i1 || !in_phys_x(f, o->i0) || !in_phys_x(f, o->i1 - 1))
      return fail(RCP_EINVAL, "monitor columns empty or outside the physical region");
    if (!(o->n_m > 0)) return fail(RCP_EINVAL, "monitor index must be positive");
  } else {
    return fail(RCP_EINVAL, "unknown objective kind");
  }
  return RCP_OK;
}

int check_line(const rcp_factors* f, const rcp_light* L) {
  if (!L) return fail(RCP_EINVAL, "light is NULL");
  if (!in_phys_y(f, L->j_s)) return fail(RCP_EINVAL, "incidence row outside the physical region");
  if (L->i0 >= L->i1 || !in_phys_x(f, L->i0) || !in_phys_x(f, L->i1 - 1))
    return fail(RCP_EINVAL, "incidence columns empty or outside the physical region");
  if (!(L->n_s > 0)) return fail(RCP_EINVAL, "source medium index must be positive");
  return RCP_OK;
}

int check_light(const rcp_factors* f, const rcp_light* L, bool need_alpha) {
  int rc = check_line(f, L);
  if (rc) return rc;
  const double half_pi = 1.5707963267948966;
  if (L->kind == RCP_CONE) {
    if (!(L->c > 0 && L->c < half_pi)) return fail(RCP_EINVAL, "cone half-angle must lie in (0, pi/2)");
  } else if (L->kind == RCP_ANNULUS) {
    if (!(L->th1 >= 0 && L->th1 < L->th2 && L->th2 < half_pi))
      return fail(RCP_EINVAL, "annulus needs 0 <= th1 < th2 < pi/2");
  } else if (L->kind == RCP_SYMBOL_TABLE) {
    if (need_alpha) return fail(RCP_EINVAL, "brute force needs a cone or annulus distribution");
    if (!L->symbol_dev) return fail(RCP_EINVAL, "symbol table is NULL");
  } else {
    return fail(RCP_EINVAL, "unknown light kind");
  }
  return RCP_OK;
}

constexpr int kMaxOutputs = 4096;

// Arguments shared by the dense-form calls; on success *D is the work layout.
int check_dense(const rcp_factors* f, int32_t nout, const rcp_objective* objs,
                const rcp_light* line, const void* W_dev, const double* F_dev, const void* work,
                size_t work_bytes, DenseLayout* D) {
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  if (nout < 1 || nout > kMaxOutputs) return fail(RCP_EINVAL, "nout must be 1 to 4096");
  if (!objs) return fail(RCP_EINVAL, "objectives are NULL");
  for (int k = 0; k < nout; ++k) {
    int rc = check_objective(f, &objs[k]);
    if (rc) return fail(rc, "output " + std::to_string(k) + ": " + g_err);
  }
  int rc = check_line(f, line);
  if (rc) return rc;
  if (!W_dev || !F_dev) return fail(RCP_EINVAL, "NULL W or F");
  *D = dense_layout(f->nx, f->ny, nout, line->i1 - line->i0);
  if (!work || work_bytes < D->total)
    return fail(RCP_ENOMEM, "dense-form workspace needs " + std::to_string(D->total) + " bytes");
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(RCP_EINVAL, "workspace must be 256-byte aligned");
  return RCP_OK;
}

// z_k = A^{-dag} w_k for every output, into the Z rows of the workspace
int dense_fields(rcp_factors* f, int K, const rcp_objective* objs, const DenseLayout& D, char* w,
                 hipStream_t s) {
  const size_t N = size_t(f->nx) * f->ny;
  double2* Bf = reinterpret_cast<double2*>(w + D.off_B);
  double2* Z = reinterpret_cast<double2*>(w + D.off_Z);
  int lo, hi;
  if (f->precision == RCP_FP64 && K >= 2) {   // all outputs in one multi-RHS sweep
    for (int k = 0; k < K; ++k) {
      int rc = objective_rhs(f, &objs[k], Bf + k * N, &lo, &hi, s);
      if (rc) return rc;
    }
    return solve_multi_fp64(f, K, Bf, nullptr, 0, Z, 1, s);
  }
  for (int k = 0; k < K; ++k) {
    int rc = objective_rhs(f, &objs[k], f->vec[V_RHS], &lo, &hi, s);
    if (!rc)
      rc = solve_vec_refined(f, f->vec[V_RHS], Z + k * N, 1, lo, hi, kRefineTol, kRefineMax, s,
                             nullptr);
    if (rc) return rc;
  }
  return RCP_OK;
}

// reciprocal fields, their line values and the dense form: F[0..K-1], F[K]
int dense_average(rcp_factors* f, int K, const rcp_objective* objs, const rcp_light* line,
                  const double2* W, double* F, const DenseLayout& D, char* w, hipStream_t s) {
  const int M = line->i1 - line->i0;
  int rc = dense_fields(f, K, objs, D, w, s);
  if (rc) return rc;
  double2* Vt = reinterpret_cast<double2*>(w + D.off_Vt);
  rc = gather_lines(reinterpret_cast<double2*>(w + D.off_Z), size_t(f->nx) * f->ny, f->ny,
                    line->j_s, line->i0, M, K, D.Kp, Vt, s);
  if (rc) return rc;
  return dense_form(W, M, Vt, K, D, reinterpret_cast<double2*>(w + D.off_part),
                    reinterpret_cast<double2*>(w + D.off_Y), reinterpret_cast<double*>(w + D.off_red),
                    F, s);
}

int reciprocal_field(rcp_factors* f, const rcp_objective* obj, double2* z, hipStream_t s) {
  int lo, hi;
  double2* w = f->vec[V_RHS];
  int rc = objective_rhs(f, obj, w, &lo, &hi, s);
  if (rc) return rc;
  // z = A^{-dag} w = conj(A)^{-1} w  (A = A^T)
  return solve_vec_refined(f, w, z, 1, lo, hi, kRefineTol, kRefineMax, s, nullptr);
}

// One factor set in a caller buffer (layout L): the handle, its views of the
// buffer, and the operator assembled on the stream.
int init_factors(const rcp_grid* grid, int32_t precision, const Layout& L, void* buf,
                 rcp_stream stream, rcp_factors** out) {
  *out = nullptr;
  rcp_factors* f = new (std::nothrow) rcp_factors();
  if (!f) return fail(RCP_ENOMEM, "host allocation failed");
  *out = f;
  f->nx = grid->nx;
  f->ny = grid->ny;
  f->npml = grid->npml;
  f->h = grid->h;
  f->k0 = grid->k0;
  f->pml_R = grid->pml_R;
  f->pml_m = grid->pml_m;
  f->precision = precision;
  f->np = ceil_div(grid->ny, TB) * TB;
  f->nt = f->np / TB;
  f->tiles = size_t(f->nt) * (f->nt + 1) / 2;
  f->block_elems = f->tiles * TB * TB;
  f->elem_bytes = precision == RCP_FP64 ? 16 : 8;
  f->m = grid->nx / 2;
  f->fft_cap = fft_capacity(grid->nx);
  f->lay = L;
  char* b = static_cast<char*>(buf);
  f->base = b;
  f->X = b + L.off_X;
  f->eps = reinterpret_cast<double*>(b + L.off_eps);
  f->sxc = reinterpret_cast<double2*>(b + L.off_sxc);
  f->sxf = reinterpret_cast<double2*>(b + L.off_sxf);
  f->syc = reinterpret_cast<double2*>(b + L.off_syc);
  f->syf = reinterpret_cast<double2*>(b + L.off_syf);
  f->dco = reinterpret_cast<double2*>(b + L.off_dco);
  f->eco = reinterpret_cast<double2*>(b + L.off_eco);
  f->cco = reinterpret_cast<double2*>(b + L.off_cco);
  const size_t panel = size_t(f->np) * TB * f->elem_bytes;
  for (int c = 0; c < 8; ++c) {
    f->wsL[c] = b + L.off_L + c * panel;
    f->wsQ[c] = b + L.off_Q + c * panel;
    f->wsP[c] = reinterpret_cast<double2*>(b + L.off_P) + c * TB * TB;
  }
  f->health = reinterpret_cast<double*>(b + L.off_health);
  f->status = reinterpret_cast<int32_t*>(b + L.off_status);
  const size_t N = size_t(f->nx) * f->ny;
  for (int v = 0; v < NVEC; ++v) f->vec[v] = reinterpret_cast<double2*>(b + L.off_vec) + v * N;
  f->red = reinterpret_cast<double*>(b + L.off_red);
  for (int q = 0; q < 4; ++q)
    f->fft[q] = reinterpret_cast<double2*>(b + L.off_fft) + q * f->fft_cap;
  for (int c = 0; c < 2; ++c)
    f->part[c] = reinterpret_cast<double2*>(b + L.off_part) + c * 2 * f->tiles * TB;
  f->last_iters = 0;
  f->last_residual = 0.0;
  int rc = launch_assemble(f, grid->eps_dev, stream);
  if (rc) {
    delete f;
    *out = nullptr;
  }
  return rc;
}

}  // namespace

extern "C" {

const char* rcp_last_error(void) { return g_err.c_str(); }

int rcp_timing_start(int32_t sample_every) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  for (TimerSample* t : g_timer.pending) {
    g_timer.pool.push_back(t->e0);
    g_timer.pool.push_back(t->e1);
    delete t;
  }
  g_timer.pending.clear();
  for (auto& c : g_timer.launches) c = 0;
  g_timer.every = sample_every > 0 ? sample_every : 0;
  return RCP_OK;
}

int rcp_timing_stop(rcp_kernel_stat* out, int32_t n) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  g_timer.every = 0;
  for (int c = 0; c < n && c < K_NCLASS; ++c) {
    out[c].launches = g_timer.launches[c];
    out[c].samples = 0;
    out[c].ms = 0.0;
    out[c].work = 0.0;
  }
  int rc = RCP_OK;
  for (TimerSample* t : g_timer.pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t->e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t->e0, t->e1);
    if (e != hipSuccess) {
      rc = hip_check(e, "rcp_timing_stop");
    } else if (t->cls < n) {
      out[t->cls].samples += 1;
      out[t->cls].ms += ms;
      out[t->cls].work += t->work;
    }
    g_timer.pool.push_back(t->e0);
    g_timer.pool.push_back(t->e1);
    delete t;
  }
  g_timer.pending.clear();
  return rc;
}

int rcp_eps_from_widths(const rcp_grid* grid, const rcp_pillars* pillars, double* eps_out_dev,
                        rcp_stream stream) {
  if (!grid || grid->nx < 1 || grid->ny < 1) return fail(RCP_EINVAL, "bad grid");
  if (!pillars || pillars->n < 0 || (pillars->n > 0 && (!pillars->centers_dev || !pillars->widths_dev)))
    return fail(RCP_EINVAL, "bad pillar description");
  if (!eps_out_dev) return fail(RCP_EINVAL, "eps_out_dev is NULL");
  return launch_eps_from_widths(grid, pillars, eps_out_dev, stream);
}

size_t rcp_factor_bytes(const rcp_grid* grid, int32_t precision) {
  if (check_grid(grid) != RCP_OK) return 0;
  if (precision != RCP_FP64 && precision != RCP_FP32_REFINED) return 0;
  return compute_layout(grid->nx, grid->ny, precision).total;
}

}  // extern "C"

namespace {
// rcp_factor_batch takes up to two groups of MAX_BATCH geometries: above
// MAX_BATCH the groups run on two streams of the library, side by side: the
// matrix cores idle by one group's passes (while its tile loads and its pivot
// chains are in flight) run the other's (single-precision factors, half the
// bytes, fit sixteen geometries of 2040 x 1080 cells in HBM).
constexpr int MAX_FACTOR_BATCH = 2 * MAX_BATCH;
constexpr int MAX_DEVICES = 64;

// The two streams of a device (default priority), created on first use and
// kept until the process ends.
std::mutex g_side_mu;
hipStream_t g_side[MAX_DEVICES][2] = {};

int side_streams(int dev, hipStream_t* out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RCP_EINVAL, "device index above 63");
  std::lock_guard<std::mutex> lk(g_side_mu);
  for (int i = 0; i < 2; ++i) {
    if (!g_side[dev][i]) RCP_HIP(hipStreamCreateWithFlags(&g_side[dev][i], hipStreamNonBlocking));
    out[i] = g_side[dev][i];
  }
  return RCP_OK;
}

struct Events {
  hipEvent_t e[3] = {};
  ~Events() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);   // released once the recorded work is done
  }
};

// Geometries [0, h) and [h, count) (h = ceil(count / 2)) assembled and factored
// on the two side streams, both forked from and joined back into s.  The
// second group is enqueued by a thread of its own: enqueuing blocks once a
// stream's launch queue is full, and one thread would then run the groups one
// after the other.  Each group has at least two geometries when count > 8, so
// every geometry's factors are those of any batch of two or more.
int factor_two_groups(int32_t count, const rcp_grid* grids, int32_t precision, const Layout& L,
                      void* const* bufs, hipStream_t s, rcp_factors** fs) {
  int dev = 0;
  RCP_HIP(hipGetDevice(&dev));
  hipStream_t side[2];
  int rc = side_streams(dev, side);
  if (rc) return rc;
  Events ev;
  for (hipEvent_t& x : ev.e) RCP_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  RCP_HIP(hipEventRecord(ev.e[0], s));
  for (hipStream_t x : side) RCP_HIP(hipStreamWaitEvent(x, ev.e[0], 0));
  const int h = (count + 1) / 2;
  const int first[2] = {0, h}, n[2] = {h, count - h};
  int grc[2] = {RCP_OK, RCP_OK};
  std::string gerr[2];
  auto group = [&](int i) {
    int r = i ? (hipSetDevice(dev) == hipSuccess ? RCP_OK : fail(RCP_EHIP, "hipSetDevice failed"))
              : RCP_OK;
    for (int g = first[i]; g < first[i] + n[i] && !r; ++g)
      r = init_factors(&grids[g], precision, L, bufs[g], side[i], &fs[g]);
    if (!r) r = factor_blocks_async(fs + first[i], n[i], side[i]);
    grc[i] = r;
    if (r) gerr[i] = g_err;
  };
  bool threaded = true;
  std::thread t1;
  try {
    t1 = std::thread(group, 1);
  } catch (const std::system_error&) {
    threaded = false;   // no thread: the groups are enqueued one after the other
  }
  group(0);
  if (threaded)
    t1.join();
  else
    group(1);
  for (int i = 0; i < 2; ++i) {
    RCP_HIP(hipEventRecord(ev.e[1 + i], side[i]));
    RCP_HIP(hipStreamWaitEvent(s, ev.e[1 + i], 0));
  }
  for (int i = 0; i < 2; ++i)
    if (grc[i])
      return fail(grc[i], "geometries " + std::to_string(first[i]) + ".." +
                              std::to_string(first[i] + n[i] - 1) + ": " + gerr[i]);
  return RCP_OK;
}

int factor_batch(int32_t count, const rcp_grid* grids, int32_t precision, void* const* bufs,
                 size_t buf_bytes, rcp_stream stream, rcp_factors** out, bool wait) {
  if (!out || !grids || !bufs) return fail(RCP_EINVAL, "NULL argument");
  if (count < 1 || count > MAX_FACTOR_BATCH) return fail(RCP_EINVAL, "count must be 1 to 16");
  for (int g = 0; g < count; ++g) out[g] = nullptr;
  if (precision != RCP_FP64 && precision != RCP_FP32_REFINED)
    return fail(RCP_EINVAL, "unknown precision");
  for (int g = 0; g < count; ++g) {
    int rc = check_grid(&grids[g]);
    if (rc) return rc;
    if (!grids[g].eps_dev) return fail(RCP_EINVAL, "eps_dev is NULL");
    const rcp_grid& a = grids[0];
    const rcp_grid& c = grids[g];
    if (c.nx != a.nx || c.ny != a.ny || c.npml != a.npml || c.h != a.h || c.pml_R != a.pml_R ||
        c.pml_m != a.pml_m)
      return fail(RCP_EINVAL, "a batch needs identical grids (only eps and k0 may differ)");
  }
  Layout L = compute_layout(grids[0].nx, grids[0].ny, precision);
  if (buf_bytes < L.total)
    return fail(RCP_ENOMEM, "factor buffer holds " + std::to_string(buf_bytes) + " bytes, needs " +
                                std::to_string(L.total));
  for (int g = 0; g < count; ++g) {
    if (!bufs[g]) return fail(RCP_ENOMEM, "factor buffer is NULL");
    if (reinterpret_cast<uintptr_t>(bufs[g]) % 256 != 0)
      return fail(RCP_EINVAL, "factor buffer must be 256-byte aligned");
    for (int h2 = 0; h2 < g; ++h2) {
      const char* x0 = static_cast<const char*>(bufs[g]);
      const char* y0 = static_cast<const char*>(bufs[h2]);
      if (x0 < y0 + L.total && y0 < x0 + L.total) return fail(RCP_EINVAL, "factor buffers overlap");
    }
  }
  rcp_factors* fs[MAX_FACTOR_BATCH] = {};   // count <= MAX_FACTOR_BATCH checked above
  int rc = RCP_OK;
  if (count <= MAX_BATCH) {
    for (int g = 0; g < count && !rc; ++g) rc = init_factors(&grids[g], precision, L, bufs[g], stream, &fs[g]);
    if (!rc) rc = wait ? factor_blocks(fs, count, stream) : factor_blocks_async(fs, count, stream);
  } else {
    rc = factor_two_groups(count, grids, precision, L, bufs, stream, fs);
    for (int g = 0; g < count && !rc && wait; ++g)
      rc = read_pivot_check(fs[g], stream, "geometry " + std::to_string(g) + ": ");
  }
  if (rc) {
    for (int g = 0; g < count; ++g) delete fs[g];
    return rc;
  }
  for (int g = 0; g < count; ++g) out[g] = fs[g];
  return RCP_OK;
}
}  // namespace

extern "C" {

int rcp_factor_batch(int32_t count, const rcp_grid* grids, int32_t precision, void* const* bufs,
                     size_t buf_bytes, rcp_stream stream, rcp_factors** out) {
  return factor_batch(count, grids, precision, bufs, buf_bytes, stream, out, true);
}

int rcp_factor_batch_async(int32_t count, const rcp_grid* grids, int32_t precision,
                           void* const* bufs, size_t buf_bytes, rcp_stream stream,
                           rcp_factors** out) {
  return factor_batch(count, grids, precision, bufs, buf_bytes, stream, out, false);
}

int rcp_factors_status(const rcp_factors* f, rcp_stream stream) {
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  return read_pivot_check(f, stream, "");
}

const int32_t* rcp_factors_status_dev(const rcp_factors* f) { return f ? f->status : nullptr; }

int rcp_factor(const rcp_grid* grid, int32_t precision, void* buf_dev, size_t buf_bytes,
               rcp_stream stream, rcp_factors** out) {
  if (!out) return fail(RCP_EINVAL, "out is NULL");
  if (!grid) return fail(RCP_EINVAL, "grid is NULL");
  void* bufs[1] = {buf_dev};
  return rcp_factor_batch(1, grid, precision, bufs, buf_bytes, stream, out);
}

int rcp_engine_create(int32_t precision, rcp_engine** out) {
  if (!out) return fail(RCP_EINVAL, "out is NULL");
  *out = nullptr;
  if (precision != RCP_FP64 && precision != RCP_FP32_REFINED)
    return fail(RCP_EINVAL, "unknown precision");
  return engine_create(precision, out);
}

void rcp_engine_destroy(rcp_engine* e) {
  if (e) engine_destroy(e);
}

int rcp_engine_add(rcp_engine* e, const rcp_grid* grid, void* buf_dev, size_t buf_bytes,
                   rcp_stream stream, rcp_factors** out) {
  if (!out) return fail(RCP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!e) return fail(RCP_EINVAL, "engine is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!grid->eps_dev) return fail(RCP_EINVAL, "eps_dev is NULL");
  if (ceil_div(grid->ny, TB) < 2) return fail(RCP_EINVAL, "the engine needs ny > 32");
  if (engine_active(e) >= MAX_BATCH) return fail(RCP_EINVAL, "engine full: 8 geometries in flight");
  const int prec = engine_precision(e);
  Layout L = compute_layout(grid->nx, grid->ny, prec);
  if (!buf_dev) return fail(RCP_ENOMEM, "factor buffer is NULL");
  if (buf_bytes < L.total)
    return fail(RCP_ENOMEM, "factor buffer holds " + std::to_string(buf_bytes) + " bytes, needs " +
                                std::to_string(L.total));
  if (reinterpret_cast<uintptr_t>(buf_dev) % 256 != 0)
    return fail(RCP_EINVAL, "factor buffer must be 256-byte aligned");
  rcp_factors* f = nullptr;
  rc = init_factors(grid, prec, L, buf_dev, stream, &f);
  if (!rc) rc = engine_add(e, f);
  if (rc) {
    delete f;
    return rc;
  }
  *out = f;
  return RCP_OK;
}

int rcp_engine_step(rcp_engine* e, int32_t rounds, rcp_stream stream, rcp_factors** done,
                    int32_t* status, int32_t cap, int32_t* n_done, int32_t* n_active) {
  if (!e || !n_done) return fail(RCP_EINVAL, "NULL argument");
  *n_done = 0;
  if (rounds < 1) return fail(RCP_EINVAL, "rounds must be >= 1");
  if (cap < MAX_BATCH || !done || !status)
    return fail(RCP_EINVAL, "done and status must hold 8 entries");
  int nd = 0;
  int rc = engine_step(e, rounds, stream, done, status, cap, &nd);
  *n_done = nd;
  if (n_active) *n_active = engine_active(e);
  return rc;
}

void rcp_factors_release(rcp_factors* f) { delete f; }

int rcp_factors_info(const rcp_factors* f, int32_t* nx, int32_t* ny, int32_t* precision,
                     int32_t* padded_n, int32_t* tile) {
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  if (nx) *nx = f->nx;
  if (ny) *ny = f->ny;
  if (precision) *precision = f->precision;
  if (padded_n) *padded_n = f->np;
  if (tile) *tile = TB;
  return RCP_OK;
}

int rcp_last_solve_stats(const rcp_factors* f, rcp_solve_stats* st) {
  if (!f || !st) return fail(RCP_EINVAL, "NULL argument");
  st->iters = f->last_iters;
  st->rel_residual = f->last_residual;
  return RCP_OK;
}

int rcp_solve_multi_rhs(const rcp_factors* fc, int32_t nrhs, const void* B_dev, void* X_dev,
                        int32_t conj_transpose, double tol, int32_t max_refine, rcp_stream stream,
                        rcp_solve_stats* stats) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  if (f->dim3) return fail(RCP_EINVAL, "factors of a 3D grid: use rcp_solve3d");
  if (nrhs < 1) return fail(RCP_EINVAL, "nrhs must be >= 1");
  if (!B_dev || !X_dev) return fail(RCP_EINVAL, "NULL right-hand side or solution");
  const size_t N = size_t(f->nx) * f->ny;
  const char* b0 = static_cast<const char*>(B_dev);
  const char* x0 = static_cast<const char*>(X_dev);
  const size_t bytes = size_t(nrhs) * N * 16;
  if (b0 < x0 + bytes && x0 < b0 + bytes) return fail(RCP_EINVAL, "B and X must not overlap");
  const double2* B = static_cast<const double2*>(B_dev);
  double2* X = static_cast<double2*>(X_dev);
  const int conjop = conj_transpose ? 1 : 0;
  if (f->precision == RCP_FP64 && nrhs >= 2) {
    int rc = solve_multi_fp64(f, nrhs, B, nullptr, 0, X, conjop, stream);
    if (rc) return rc;
    if (stats) {
      stats->iters = 0;
      stats->rel_residual = 0.0;
    }
    return RCP_OK;
  }
  double worst = 0.0;
  int iters = 0;
  for (int r = 0; r < nrhs; ++r) {
    rcp_solve_stats st{};
    int rc = solve_vec_refined(f, B + r * N, X + r * N, conjop, 0, f->nx - 1, tol, max_refine, stream,
                               (stats || f->precision != RCP_FP64) ? &st : nullptr);
    if (rc) return rc;
    if (st.rel_residual > worst) worst = st.rel_residual;
    if (st.iters > iters) iters = st.iters;
  }
  if (stats) {
    stats->iters = iters;
    stats->rel_residual = worst;
  }
  return RCP_OK;
}

int rcp_reciprocal_average(const rcp_factors* fc, const rcp_objective* obj, const rcp_light* light,
                           double* F_dev, void* v_dev, void* z_dev, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  int rc = check_objective(f, obj);
  if (!rc) rc = check_light(f, light, false);
  if (rc) return rc;
  if (!F_dev) return fail(RCP_EINVAL, "F_dev is NULL");
  double2* z = z_dev ? static_cast<double2*>(z_dev) : f->vec[V_Z];
  rc = reciprocal_field(f, obj, z, stream);
  if (rc) return rc;
  return toeplitz_form(f, light, z, F_dev, static_cast<double2*>(v_dev), nullptr, stream);
}

size_t rcp_reciprocal_many_work_bytes(const rcp_factors* f, int32_t count) {
  if (!f || count < 1 || count > 64) return 0;
  return align256(2 * size_t(count) * f->nx * f->ny * sizeof(double2));
}

}  // extern "C"

namespace {

// Checks shared by rcp_reciprocal_average_many and its allocation-free variant.
int check_many(const rcp_factors* f, int32_t count, const rcp_objective* objs,
               const rcp_light* lights, const double* F_dev) {
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  if (count < 1 || count > 64) return fail(RCP_EINVAL, "count must be 1 to 64");
  if (!objs || !lights || !F_dev) return fail(RCP_EINVAL, "NULL argument");
  for (int k = 0; k < count; ++k) {
    int rc = check_objective(f, &objs[k]);
    if (!rc) rc = check_light(f, &lights[k], false);
    if (rc) return rc;
  }
  return RCP_OK;
}

// The evaluations of rcp_reciprocal_average_many on a workspace of at least
// rcp_reciprocal_many_work_bytes(f, count) bytes (every byte of it is written
// before it is read).
int reciprocal_many(rcp_factors* f, int32_t count, const rcp_objective* objs,
                    const rcp_light* lights, double* F_dev, void* work, hipStream_t stream) {
  const size_t N = size_t(f->nx) * f->ny;
  double2* B = static_cast<double2*>(work);
  double2* Z = B + size_t(count) * N;
  int lo, hi, rc = RCP_OK;
  if (f->precision == RCP_FP64 && count >= 2) {   // all objectives in one multi-RHS sweep
    for (int k = 0; k < count && !rc; ++k) rc = objective_rhs(f, &objs[k], B + k * N, &lo, &hi, stream);
    if (!rc) rc = solve_multi_fp64(f, count, B, nullptr, 0, Z, 1, stream);
  } else {
    for (int k = 0; k < count && !rc; ++k) {
      rc = objective_rhs(f, &objs[k], f->vec[V_RHS], &lo, &hi, stream);
      if (!rc)
        rc = solve_vec_refined(f, f->vec[V_RHS], Z + k * N, 1, lo, hi, kRefineTol, kRefineMax,
                               stream, nullptr);
    }
  }
  for (int k = 0; k < count && !rc; ++k)
    rc = toeplitz_form(f, &lights[k], Z + k * N, F_dev + k, nullptr, nullptr, stream);
  return rc;
}

}  // namespace

// Workspace of the allocation-free entry point: one array per GPU, held until
// the process ends.  In host code `scratch` only names the array (a host-side
// stand-in, not a device address); its address on each device comes from
// hipGetSymbolAddress with that device current and is kept per device.
static __device__ __align__(256) unsigned char scratch[RCP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = -1;
  RCP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RCP_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    RCP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RCP_EHIP, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return RCP_OK;
}
}  // namespace

extern "C" {

int rcp_reciprocal_average_many(const rcp_factors* fc, int32_t count, const rcp_objective* objs,
                                const rcp_light* lights, double* F_dev, void* work_dev,
                                size_t work_bytes, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (reinterpret_cast<uintptr_t>(work_dev) % 256 != 0)
    return fail(RCP_EINVAL, "workspace must be 256-byte aligned");
  int rc = check_many(f, count, objs, lights, F_dev);
  if (rc) return rc;
  if (!work_dev) return fail(RCP_EINVAL, "NULL argument");
  const size_t need = rcp_reciprocal_many_work_bytes(f, count);
  if (work_bytes < need) return fail(RCP_ENOMEM, "work buffer: need " + std::to_string(need) + " bytes");
  return reciprocal_many(f, count, objs, lights, F_dev, work_dev, stream);
}

int rcp_reciprocal_average_many_noalloc(const rcp_factors* fc, int32_t count,
                                        const rcp_objective* objs, const rcp_light* lights,
                                        double* F_dev, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  int rc = check_many(f, count, objs, lights, F_dev);
  if (rc) return rc;
  const size_t need = rcp_reciprocal_many_work_bytes(f, count);
  if (need > RCP_NOALLOC_SCRATCH_BYTES)
    return fail(RCP_ENOMEM, std::to_string(count) + " evaluations on this grid need " +
                                std::to_string(need) + " bytes of workspace; the scratch array holds " +
                                std::to_string(size_t(RCP_NOALLOC_SCRATCH_BYTES)));
  void* work = nullptr;
  rc = scratch_address(&work);
  if (rc) return rc;
  return reciprocal_many(f, count, objs, lights, F_dev, work, stream);
}

int rcp_adjoint_grad(const rcp_factors* fc, const rcp_objective* obj, const rcp_light* light,
                     double* F_dev, double* grad_eps_dev, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  int rc = check_objective(f, obj);
  if (!rc) rc = check_light(f, light, false);
  if (rc) return rc;
  if (!F_dev || !grad_eps_dev) return fail(RCP_EINVAL, "NULL output");
  double2* z = f->vec[V_Z];
  rc = reciprocal_field(f, obj, z, stream);
  if (rc) return rc;
  double2* Tv = f->fft[3];
  rc = toeplitz_form(f, light, z, F_dev, nullptr, Tv, stream);
  if (rc) return rc;
  double2* arhs = f->vec[V_ARHS];
  rc = scatter_line(f, light, Tv, arhs, stream);
  if (rc) return rc;
  double2* lam = f->vec[V_LAM];
  rc = solve_vec_refined(f, arhs, lam, 0, light->i0, light->i1 - 1, kRefineTol, kRefineMax, stream,
                         nullptr);
  if (rc) return rc;
  return grad_eps(f, lam, z, grad_eps_dev, stream);
}

int rcp_adjoint_grad_batch(int32_t count, rcp_factors* const* factors, const rcp_objective* objs,
                           const rcp_light* lights, double* F_dev, double* const* grad_eps_dev,
                           rcp_stream stream) {
  if (count < 1 || count > MAX_BATCH) return fail(RCP_EINVAL, "count must be 1 to 8");
  if (!factors || !objs || !lights || !F_dev || !grad_eps_dev)
    return fail(RCP_EINVAL, "NULL argument");
  rcp_factors* fs[MAX_BATCH] = {};
  for (int g = 0; g < count; ++g) {
    fs[g] = factors[g];
    if (!fs[g]) return fail(RCP_EINVAL, "factors " + std::to_string(g) + " is NULL");
    const rcp_factors& a = *fs[0];
    const rcp_factors& c = *fs[g];
    if (c.nx != a.nx || c.ny != a.ny || c.precision != a.precision)
      return fail(RCP_EINVAL, "a batch needs factors of identical grid and precision");
    for (int h = 0; h < g; ++h)
      if (fs[h] == fs[g]) return fail(RCP_EINVAL, "the same factors appear twice in a batch");
    int rc = check_objective(fs[g], &objs[g]);
    if (!rc) rc = check_light(fs[g], &lights[g], false);
    if (rc) return rc;
    if (!grad_eps_dev[g]) return fail(RCP_EINVAL, "NULL output");
  }
  if (fs[0]->precision != RCP_FP64) {   // refinement runs per factor set
    for (int g = 0; g < count; ++g) {
      int rc = rcp_adjoint_grad(fs[g], &objs[g], &lights[g], F_dev + g, grad_eps_dev[g], stream);
      if (rc) return rc;
    }
    return RCP_OK;
  }
  // the same steps as rcp_adjoint_grad, the two solves of all sets in lockstep
  const double2* rhs[MAX_BATCH];
  double2* sol[MAX_BATCH];
  int lo[MAX_BATCH], hi[MAX_BATCH];
  for (int g = 0; g < count; ++g) {
    double2* w = fs[g]->vec[V_RHS];
    int rc = objective_rhs(fs[g], &objs[g], w, &lo[g], &hi[g], stream);
    if (rc) return rc;
    rhs[g] = w;
    sol[g] = fs[g]->vec[V_Z];
  }
  int rc = solve_vec_batch(fs, count, rhs, sol, 1, lo, hi, stream);
  if (rc) return rc;
  for (int g = 0; g < count; ++g) {
    rcp_factors* f = fs[g];
    double2* Tv = f->fft[3];
    rc = toeplitz_form(f, &lights[g], f->vec[V_Z], F_dev + g, nullptr, Tv, stream);
    if (!rc) rc = scatter_line(f, &lights[g], Tv, f->vec[V_ARHS], stream);
    if (rc) return rc;
    rhs[g] = f->vec[V_ARHS];
    sol[g] = f->vec[V_LAM];
    lo[g] = lights[g].i0;
    hi[g] = lights[g].i1 - 1;
  }
  rc = solve_vec_batch(fs, count, rhs, sol, 0, lo, hi, stream);
  if (rc) return rc;
  for (int g = 0; g < count; ++g) {
    rc = grad_eps(fs[g], fs[g]->vec[V_LAM], fs[g]->vec[V_Z], grad_eps_dev[g], stream);
    if (rc) return rc;
  }
  return RCP_OK;
}

int rcp_broadband_grad(int32_t count, rcp_factors* const* factors, const rcp_objective* objs,
                       const rcp_light* lights, const double* weights, double* F_dev,
                       double* grad_eps_dev, rcp_stream stream) {
  if (count < 1 || count > MAX_BATCH) return fail(RCP_EINVAL, "count must be 1 to 8");
  if (!factors || !weights || !F_dev || !grad_eps_dev) return fail(RCP_EINVAL, "NULL argument");
  for (int g = 0; g < count; ++g)
    if (!std::isfinite(weights[g])) return fail(RCP_EINVAL, "weights must be finite");
  // each set's gradient goes to its own scratch vector, then the weighted sum
  double* grads[MAX_BATCH];
  for (int g = 0; g < count; ++g) {
    if (!factors[g]) return fail(RCP_EINVAL, "factors " + std::to_string(g) + " is NULL");
    grads[g] = reinterpret_cast<double*>(factors[g]->vec[V_TMP]);
  }
  int rc = rcp_adjoint_grad_batch(count, factors, objs, lights, F_dev, grads, stream);
  if (rc) return rc;
  return weighted_sum(count, weights, grads, size_t(factors[0]->nx) * factors[0]->ny, F_dev,
                      grad_eps_dev, stream);
}

int rcp_width_grad(const rcp_grid* grid, const rcp_pillars* pillars, const double* grad_eps_dev,
                   double* grad_w_dev, rcp_stream stream) {
  if (!grid || grid->nx < 1 || grid->ny < 1) return fail(RCP_EINVAL, "bad grid");
  if (!pillars || pillars->n < 0) return fail(RCP_EINVAL, "bad pillar description");
  if (!grad_eps_dev || (pillars->n > 0 && !grad_w_dev)) return fail(RCP_EINVAL, "NULL argument");
  if (pillars->row0 < 0 || pillars->row0 + pillars->rows > grid->ny)
    return fail(RCP_EINVAL, "pillar rows outside the grid");
  return launch_width_grad(grid, pillars, grad_eps_dev, grad_w_dev, stream);
}

size_t rcp_brute_force_work_bytes(const rcp_factors* f, int32_t nangles, int32_t rhs_chunk) {
  if (!f || nangles < 1 || rhs_chunk < 1) return 0;
  const size_t N = size_t(f->nx) * f->ny;
  size_t o = 0;
  o = align256(o + 3 * size_t(nangles) * 8);
  o = align256(o + size_t(rhs_chunk) * f->nx * 16);
  o = align256(o + size_t(rhs_chunk) * N * 16);
  if (rhs_chunk >= 64) o = align256(o + GEMM_SPLIT_BYTES);   // k-split partial tiles of the sweep
  return o;
}

int rcp_brute_force_average(const rcp_factors* fc, const rcp_objective* obj, const rcp_light* light,
                            int32_t nangles, int32_t rhs_chunk, void* work_dev, size_t work_bytes,
                            double* F_dev, double* per_angle_dev, rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  if (!f) return fail(RCP_EINVAL, "factors is NULL");
  if (f->precision != RCP_FP64)
    return fail(RCP_EINVAL, "the brute-force baseline runs on RCP_FP64 factors");
  int rc = check_objective(f, obj);
  if (!rc) rc = check_light(f, light, true);
  if (rc) return rc;
  if (nangles < 1 || rhs_chunk < 1) return fail(RCP_EINVAL, "nangles and rhs_chunk must be >= 1");
  if (light->kind == RCP_ANNULUS && nangles % 2)
    return fail(RCP_EINVAL, "annulus needs an even node count");
  if (!F_dev) return fail(RCP_EINVAL, "F_dev is NULL");
  size_t need = rcp_brute_force_work_bytes(f, nangles, rhs_chunk);
  if (!work_dev || work_bytes < need)
    return fail(RCP_ENOMEM, "brute-force workspace needs " + std::to_string(need) + " bytes");
  char* w = static_cast<char*>(work_dev);
  double* theta = reinterpret_cast<double*>(w);
  double* wts = theta + nangles;
  double* pa = per_angle_dev ? per_angle_dev : wts + nangles;
  size_t o = align256(3 * size_t(nangles) * 8);
  double2* fline = reinterpret_cast<double2*>(w + o);
  o = align256(o + size_t(rhs_chunk) * f->nx * 16);
  double2* U = reinterpret_cast<double2*>(w + o);
  o = align256(o + size_t(rhs_chunk) * size_t(f->nx) * f->ny * 16);
  double2* split = rhs_chunk >= 64 ? reinterpret_cast<double2*>(w + o) : nullptr;
  rc = gl_nodes(light, nangles, theta, wts, stream);
  if (rc) return rc;
  for (int r0 = 0; r0 < nangles; r0 += rhs_chunk) {
    int R = nangles - r0 < rhs_chunk ? nangles - r0 : rhs_chunk;
    rc = planewave_lines(f, light, theta + r0, R, fline, stream);
    if (rc) return rc;
    rc = solve_multi_fp64(f, R, nullptr, fline, light->j_s, U, 0, stream, split);
    if (rc) return rc;
    rc = bf_per_angle_at(f, obj, U, R, pa, r0, stream);
    if (rc) return rc;
  }
  return bf_sum(wts, pa, nangles, F_dev, stream);
}

size_t rcp_dense_work_bytes(const rcp_factors* f, int32_t nout, int32_t m) {
  if (!f || nout < 1 || nout > kMaxOutputs || m < 1 || m > f->nx) return 0;
  return dense_layout(f->nx, f->ny, nout, m).total;
}

int rcp_reciprocal_average_dense(const rcp_factors* fc, int32_t nout, const rcp_objective* objs,
                                 const rcp_light* line, const void* W_dev, double* F_dev,
                                 void* V_dev, void* work_dev, size_t work_bytes,
                                 rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  DenseLayout D;
  int rc = check_dense(f, nout, objs, line, W_dev, F_dev, work_dev, work_bytes, &D);
  if (rc) return rc;
  char* w = static_cast<char*>(work_dev);
  rc = dense_average(f, nout, objs, line, static_cast<const double2*>(W_dev), F_dev, D, w, stream);
  if (rc || !V_dev) return rc;
  const int M = line->i1 - line->i0;
  RCP_HIP(hipMemcpyAsync(V_dev, w + D.off_Vt, size_t(nout) * M * sizeof(double2),
                         hipMemcpyDeviceToDevice, stream));
  return RCP_OK;
}

int rcp_adjoint_grad_dense(const rcp_factors* fc, int32_t nout, const rcp_objective* objs,
                           const rcp_light* line, const void* W_dev, double* F_dev,
                           double* grad_eps_dev, void* work_dev, size_t work_bytes,
                           rcp_stream stream) {
  rcp_factors* f = const_cast<rcp_factors*>(fc);
  DenseLayout D;
  int rc = check_dense(f, nout, objs, line, W_dev, F_dev, work_dev, work_bytes, &D);
  if (rc) return rc;
  if (!grad_eps_dev) return fail(RCP_EINVAL, "grad_eps_dev is NULL");
  char* w = static_cast<char*>(work_dev);
  rc = dense_average(f, nout, objs, line, static_cast<const double2*>(W_dev), F_dev, D, w, stream);
  if (rc) return rc;
  const int K = nout, M = line->i1 - line->i0;
  const size_t N = size_t(f->nx) * f->ny;
  double2* Y = reinterpret_cast<double2*>(w + D.off_Y);
  double2* Lam = reinterpret_cast<double2*>(w + D.off_B);   // the right-hand sides are spent
  if (f->precision == RCP_FP64 && K >= 2) {
    double2* fline = reinterpret_cast<double2*>(w + D.off_fline);
    rc = scatter_lines(Y, M, K, f->nx, line->i0, fline, stream);
    if (!rc) rc = solve_multi_fp64(f, K, nullptr, fline, line->j_s, Lam, 0, stream);
    if (rc) return rc;
  } else {
    for (int k = 0; k < K; ++k) {
      rc = scatter_line(f, line, Y + size_t(k) * M, f->vec[V_ARHS], stream);
      if (!rc)
        rc = solve_vec_refined(f, f->vec[V_ARHS], Lam + k * N, 0, line->i0, line->i1 - 1,
                               kRefineTol, kRefineMax, stream, nullptr);
      if (rc) return rc;
    }
  }
  return grad_eps_many(f, K, Lam, reinterpret_cast<double2*>(w + D.off_Z), grad_eps_dev, stream);
}

size_t rcp_correlation_work_bytes(int32_t m, int32_t nangles) {
  if (m < 1 || nangles < 1 || m > (1 << 16) || nangles > (1 << 16)) return 0;
  return corr_layout(m, nangles).total;
}

int rcp_correlation_matrix(const rcp_grid* grid, const rcp_light* line, int32_t nangles,
                           const double* theta_dev, const void* C_dev, void* W_dev,
                           void* work_dev, size_t work_bytes, rcp_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!line) return fail(RCP_EINVAL, "light is NULL");
  const int npml = grid->npml;
  if (line->i0 >= line->i1 || line->i0 < npml || line->i1 > grid->nx - npml)
    return fail(RCP_EINVAL, "incidence columns empty or outside the physical region");
  if (!(line->n_s > 0)) return fail(RCP_EINVAL, "source medium index must be positive");
  const int M = line->i1 - line->i0;
  if (nangles < 1 || nangles > (1 << 16)) return fail(RCP_EINVAL, "nangles must be 1 to 65536");
  if (!theta_dev || !C_dev || !W_dev) return fail(RCP_EINVAL, "NULL argument");
  const size_t need = rcp_correlation_work_bytes(M, nangles);
  if (!work_dev || work_bytes < need)
    return fail(RCP_ENOMEM, "correlation workspace needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(work_dev) % 256 != 0)
    return fail(RCP_EINVAL, "workspace must be 256-byte aligned");
  return correlation_matrix(M, nangles, line->i0, npml, grid->h, line->n_s, grid->k0, theta_dev,
                            static_cast<const double2*>(C_dev), static_cast<double2*>(W_dev),
                            static_cast<char*>(work_dev), stream);
}

}  // extern "C"

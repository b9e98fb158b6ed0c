// C-ABI of libdgp: plans, parameters, and the host-side orchestration of the
// field solve (Sec. III B/C), the PM step (Sec. III A), the adjoints and the
// binned power spectrum.  Every array step runs in the HIP kernels of
// passes.hip, relax.hip, adjoint.hip and pm.hip; this file only sequences
// launches, owns the workspace and reads the few convergence scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dgp.h"
#include "dgp_internal.h"


using namespace dgp;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(DGP_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

#define LAUNCHCHK()                                                                            \
  do {                                                                                         \
    hipError_t e_ = hipGetLastError();                                                         \
    if (e_ != hipSuccess) return fail(DGP_E_HIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

extern "C" const char* dgp_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ twiddle tables (per device, per N)
namespace dgp {
constexpr int kMaxDev = 64;
constexpr int kLogMin = 3, kLogMax = 9;
static void* g_tw[kMaxDev][kLogMax + 1][2];   // [dev][log2 n][0 = double, 1 = float]
static std::mutex g_tw_mu;

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

template <typename T>
const cx<T>* twiddles(int n) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return static_cast<const cx<T>*>(g_tw[dev][ilog2(n)][sizeof(T) == 4 ? 1 : 0]);
}
template const cx<double>* twiddles<double>(int);
template const cx<float>* twiddles<float>(int);
}  // namespace dgp

// exp(-2 pi i m / n) in double: long-double cos/sin of 2 pi m / n, exact values at the quarter points
static void twiddle_values(int n, std::vector<double>& re, std::vector<double>& im) {
  re.resize(n);
  im.resize(n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int m = 0; m < n; ++m) {
    const long double ang = two_pi * (long double)m / (long double)n;
    re[m] = (double)cosl(ang);
    im[m] = (double)-sinl(ang);
  }
  // exact values at the quarter points
  for (int m = 0; m < n; m += n / 4) {
    const int qd = m / (n / 4);
    re[m] = (qd == 0) ? 1.0 : (qd == 2) ? -1.0 : 0.0;
    im[m] = (qd == 1) ? -1.0 : (qd == 3) ? 1.0 : 0.0;
  }
}

static int ensure_twiddles(int n) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev >= kMaxDev) return fail(DGP_E_UNSUPPORTED, "device index %d too large", dev);
  std::lock_guard<std::mutex> lk(g_tw_mu);
  for (int l = kLogMin; l <= ilog2(n); ++l) {
    const int nn = 1 << l;
    if (g_tw[dev][l][0] != nullptr) continue;
    std::vector<double> re, im;
    twiddle_values(nn, re, im);
    std::vector<double> hd(2 * nn);
    std::vector<float> hf(2 * nn);
    for (int m = 0; m < nn; ++m) {
      hd[2 * m] = re[m];
      hd[2 * m + 1] = im[m];
      hf[2 * m] = (float)re[m];
      hf[2 * m + 1] = (float)im[m];
    }
    void* dd = nullptr;
    void* df = nullptr;
    HIPCHK(hipMalloc(&dd, sizeof(double) * 2 * nn));
    HIPCHK(hipMalloc(&df, sizeof(float) * 2 * nn));
    HIPCHK(hipMemcpy(dd, hd.data(), sizeof(double) * 2 * nn, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(df, hf.data(), sizeof(float) * 2 * nn, hipMemcpyHostToDevice));
    g_tw[dev][l][0] = dd;
    g_tw[dev][l][1] = df;
  }
  return DGP_OK;
}

// ------------------------------------------------------------------ background (Sec. II)
static double hubble_E(double om0, double a) {
  const double b = 1.0 - om0;
  return 0.5 * (b + std::sqrt(b * b + 4.0 * om0 / (a * a * a)));
}
static constexpr double kCOverH0 = 2997.92458;
// flat LCDM with the same Omega_m0: the background of the standard-gravity (GR) runs
static double hubble_E_lcdm(double om0, double a) { return std::sqrt(om0 / (a * a * a) + (1.0 - om0)); }

extern "C" int dgp_params_init(dgp_params* p, double omega_m0, double a) {
  if (!p) return fail(DGP_E_INVALID, "params is NULL");
  if (!(omega_m0 > 0.0 && omega_m0 < 1.0) || !(a > 0.0) || !std::isfinite(a))
    return fail(DGP_E_INVALID, "omega_m0 must be in (0,1) and a > 0");
  std::memset(p, 0, sizeof *p);
  p->omega_m0 = omega_m0;
  p->a = a;
  const double E = hubble_E(omega_m0, a);
  const double eta = E / (1.0 - omega_m0);
  const double den = eta * (2.0 * eta - 1.0);
  p->E = E;
  p->eta = eta;
  p->beta = (2.0 * eta * eta - 2.0 * eta - 1.0) / den;
  p->alpha = 3.0 * (2.0 * eta * eta - 2.0 * eta + 1.0) / den;
  p->A = 3.0 * (eta - 1.0) / eta;
  p->gamma = 3.0 * p->beta * (eta - 1.0) / (2.0 * eta - 1.0);
  p->c2 = (3.0 * eta * eta - 5.0 * eta + 1.0) / (2.0 * eta * eta * (2.0 * eta - 1.0));
  p->kappa = kCOverH0 / (a * E);
  p->lambda = 1.0;
  p->w = 1.0 / 3.0;
  p->omega_relax = 1.0;
  p->tol = 1e-2;
  p->max_iter = 100;
  p->init = DGP_INIT_LINEAR;
  p->nonlocal = 1;
  p->force_mode = DGP_FORCE_NLDGP;
  p->check_every = 4;
  return DGP_OK;
}

static int check_params(const dgp_params* p) {
  if (!p) return fail(DGP_E_INVALID, "params is NULL");
  const double v[] = {p->a, p->E, p->eta, p->alpha, p->beta, p->A, p->gamma, p->c2, p->kappa, p->lambda, p->w,
                      p->omega_relax, p->tol};
  for (double x : v)
    if (!std::isfinite(x)) return fail(DGP_E_INVALID, "non-finite parameter");
  if (!(p->lambda > 0.0)) return fail(DGP_E_INVALID, "lambda must be > 0");
  if (!(p->w >= 0.0 && p->w < 1.0)) return fail(DGP_E_INVALID, "w must be in [0, 1)");
  if (!(p->omega_relax > 0.0 && p->omega_relax <= 1.0)) return fail(DGP_E_INVALID, "omega_relax must be in (0, 1]");
  if (p->max_iter < 0 || p->max_iter >= kMaxHist - 1) return fail(DGP_E_INVALID, "max_iter must be in [0, %d)", kMaxHist - 1);
  if (p->init < 0 || p->init > 2) return fail(DGP_E_INVALID, "bad init");
  if (p->force_mode < 0 || p->force_mode > 3) return fail(DGP_E_INVALID, "bad force_mode");
  if (!(p->alpha > 0.0) || !(p->kappa > 0.0) || !(p->eta > 0.0)) return fail(DGP_E_INVALID, "alpha, kappa, eta must be > 0");
  return DGP_OK;
}

// ------------------------------------------------------------------ plan
struct dgp_plan {
  int n = 0, batch = 0, precision = 0, device = 0;
  double box = 0.0;
  size_t n3 = 0, hs = 0;   // real and half-spectrum element counts per field per batch element
  // float64 solve workspace
  double* U = nullptr;               // [3][B][n3]
  double* S = nullptr;               // [B][n3]
  cx<double>* spec_u = nullptr;      // [B][hs]
  cx<double>* spec6 = nullptr;       // [8][B][hs]; fields 6, 7: axis-0/1 spectra of delta (kept) and u
  double* partial = nullptr;         // [B][groups][2]
  int groups64 = 0;
  // float32 solve workspace (precision form)
  float* U32 = nullptr;
  float* S32 = nullptr;
  cx<float>* spec_u32 = nullptr;
  cx<float>* spec6_32 = nullptr;
  double* partial32 = nullptr;
  int groups32 = 0;
  // control
  SolveCtl* ctl = nullptr;           // device [B]
  SolveCtl* ctl_host = nullptr;      // pinned [B]
  int* n_active = nullptr;
  int* n_active_host = nullptr;
  double* mean_u = nullptr;          // [B]
  double* means_host = nullptr;      // pinned [B]: <u> of the returned iterates
  int hint32 = 0, hint64 = 0;        // passes of the last solve (float32 phase, float64 solve or phase)
  double* vec = nullptr;             // [4][B] scratch scalars (eps, means)
  double* red = nullptr;             // reduction scratch
  // PM (batch 1)
  long long* grid = nullptr;         // [n3]
  double* delta = nullptr;           // [n3]
  double* mesh3 = nullptr;           // [3][n3] force mesh (float64 plans)
  float* mesh3_32 = nullptr;         // [3][n3] force mesh (precision-form plans)
  // power spectrum
  double* bin_tab = nullptr;         // thresholds + coefficients
  double* bin_partial = nullptr;
  double* bin_host = nullptr;        // pinned
  // adjoint (allocated on first use)
  double* adj = nullptr;             // [9][B][n3]
  double* adj_red = nullptr;
  double* adj_vec = nullptr;         // [B] <h22 mu> of the current multipliers
  SolveCtl* adj_ctl = nullptr;       // device [B]
  SolveCtl* adj_ctl_host = nullptr;  // pinned [B]
  // non-finite particle flag (device, one 8-byte slot) and its pinned host copy; fixed-point
  // scale state of the interpolation adjoint
  int* flag = nullptr;
  int* flag_host = nullptr;
  unsigned long long* fx_state = nullptr;
  std::vector<void*> dev_allocs;
  // caller-owned device workspace (dgp_plan_create_ws): buffers are carved from it, 256-byte aligned
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  bool dry = false;   // size query (dgp_workspace_bytes): count the bytes, allocate nothing
  std::vector<void*> host_allocs;
  size_t bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // live per-kernel timing (HIP events around launches on the caller's stream)
  bool timing = false;
  unsigned int t_mask = 0xffffffffu;   // classes timed while timing is on
  struct Pend { hipEvent_t a, b; int cls; };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pend> pend;
  double t_ms[DGP_T_NCLASS] = {};
  long long t_cnt[DGP_T_NCLASS] = {};
};

static hipEvent_t ev_get(dgp_plan* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scope that brackets the launches it encloses with two events when timing is on.
struct Timed {
  dgp_plan* pl;
  hipStream_t s;
  int cls;
  hipEvent_t a = nullptr;
  Timed(dgp_plan* p, hipStream_t st, int c) : pl(p), s(st), cls(c) {
    if (pl->timing && ((pl->t_mask >> cls) & 1u) && (a = ev_get(pl)) != nullptr) (void)hipEventRecord(a, s);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = ev_get(pl);
    if (!b) return;
    (void)hipEventRecord(b, s);
    pl->pend.push_back({a, b, cls});
  }
};

// A timed class of one kernel launch: the two events are handed to the launch, which records
// them as part of its dispatch (no marker packets between this kernel and its neighbours).
struct TimedLaunch {
  dgp_plan* pl;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(dgp_plan* p, int c) : pl(p), cls(c) {
    if (!pl->timing || !((pl->t_mask >> cls) & 1u)) return;
    a = ev_get(pl);
    b = a ? ev_get(pl) : nullptr;
    if (a && !b) {
      pl->ev_pool.push_back(a);
      a = nullptr;
    }
  }
  ~TimedLaunch() {
    if (a && b) pl->pend.push_back({a, b, cls});
  }
};

// accumulate completed event pairs (call after the stream has been synchronised)
static void timing_flush(dgp_plan* pl) {
  for (auto& q : pl->pend) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      pl->t_ms[q.cls] += ms;
      pl->t_cnt[q.cls] += 1;
    } else {
      (void)hipGetLastError();
    }
    pl->ev_pool.push_back(q.a);
    pl->ev_pool.push_back(q.b);
  }
  pl->pend.clear();
}

template <typename T>
static constexpr int tcls(int base) { return base + (sizeof(T) == 4 ? DGP_T_FP32_OFFSET : 0); }

// Device buffer of `count` elements, accounted in 256-byte units: from the caller's workspace when
// the plan has one, counted only in a size query, else hipMalloc.
template <typename T>
static int dalloc(dgp_plan* pl, T** ptr, size_t count) {
  const size_t bytes = (sizeof(T) * (count ? count : 1) + 255) & ~size_t(255);
  if (pl->dry) {
    pl->bytes += bytes;
    *ptr = nullptr;
    return DGP_OK;
  }
  if (pl->ws) {
    if (bytes > pl->ws_bytes - pl->ws_used)
      return fail(DGP_E_INVALID, "caller workspace of %zu bytes is too small (%zu more needed at this point)",
                  pl->ws_bytes, pl->ws_used + bytes - pl->ws_bytes);
    *ptr = reinterpret_cast<T*>(pl->ws + pl->ws_used);
    pl->ws_used += bytes;
    pl->bytes += bytes;
    return DGP_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGP_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  pl->dev_allocs.push_back(p);
  pl->bytes += bytes;
  *ptr = static_cast<T*>(p);
  return DGP_OK;
}

template <typename T>
static int halloc(dgp_plan* pl, T** ptr, size_t count) {
  if (pl->dry) {
    *ptr = nullptr;
    return DGP_OK;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, sizeof(T) * (count ? count : 1), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGP_E_NOMEM, "hipHostMalloc failed");
  }
  pl->host_allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return DGP_OK;
}

static void plan_free(dgp_plan* pl) {
  for (auto& q : pl->pend) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
  for (void* p : pl->dev_allocs) (void)hipFree(p);
  for (void* p : pl->host_allocs) (void)hipHostFree(p);
  if (pl->ev0) (void)hipEventDestroy(pl->ev0);
  if (pl->ev1) (void)hipEventDestroy(pl->ev1);
  delete pl;
}

#define TRY(expr)               \
  do {                          \
    int r_ = (expr);            \
    if (r_ < 0) return r_;      \
  } while (0)

static int plan_alloc(dgp_plan* pl) {
  const size_t B = pl->batch, n3 = pl->n3, hs = pl->hs;
  TRY(dalloc(pl, &pl->U, 3 * B * n3));
  TRY(dalloc(pl, &pl->S, B * n3));
  TRY(dalloc(pl, &pl->spec_u, B * hs));
  TRY(dalloc(pl, &pl->spec6, 8 * B * hs));   // 6 pass spectra + the delta and u spectra of the PM step
  pl->groups64 = relax_groups(pl->n, 8);
  TRY(dalloc(pl, &pl->partial, B * pl->groups64 * 2));
  if (pl->precision == DGP_FP32) {
    TRY(dalloc(pl, &pl->U32, 3 * B * n3));
    TRY(dalloc(pl, &pl->S32, B * n3));
    TRY(dalloc(pl, &pl->spec_u32, B * hs));
    TRY(dalloc(pl, &pl->spec6_32, 8 * B * hs));   // as spec6: fields 6, 7 for the PM step's force mesh
    pl->groups32 = relax_groups(pl->n, 4);
    TRY(dalloc(pl, &pl->partial32, B * pl->groups32 * 2));
  }
  TRY(dalloc(pl, &pl->ctl, B));
  TRY(halloc(pl, &pl->ctl_host, B));
  TRY(dalloc(pl, &pl->n_active, 1));
  TRY(halloc(pl, &pl->n_active_host, 1));
  TRY(dalloc(pl, &pl->mean_u, B));
  TRY(halloc(pl, &pl->means_host, B));
  TRY(dalloc(pl, &pl->vec, 4 * B));
  TRY(dalloc(pl, &pl->red, absmean_scratch_doubles(n3, (int)B) + 16));
  if (B == 1) {
    TRY(dalloc(pl, &pl->grid, n3));
    TRY(dalloc(pl, &pl->delta, n3));
    if (pl->precision == DGP_FP32)
      TRY(dalloc(pl, &pl->mesh3_32, 3 * n3));
    else
      TRY(dalloc(pl, &pl->mesh3, 3 * n3));
  }
  TRY(dalloc(pl, &pl->flag, 2));
  TRY(halloc(pl, &pl->flag_host, 2));
  TRY(dalloc(pl, &pl->fx_state, 4));
  TRY(dalloc(pl, &pl->bin_tab, 129 + 128 * B));
  TRY(dalloc(pl, &pl->bin_partial, (size_t)p3_row_groups(pl->n) * B * 2 * 128));
  TRY(halloc(pl, &pl->bin_host, (size_t)p3_row_groups(pl->n) * B * 2 * 128));
  return DGP_OK;
}

static int check_plan_sizes(int n, int batch, double box, int precision) {
  if (n < 8 || n > 512 || (n & (n - 1)) != 0) return fail(DGP_E_INVALID, "N must be a power of two in [8, 512], got %d", n);
  if (batch < 1 || batch > 4096) return fail(DGP_E_INVALID, "batch must be in [1, 4096]");
  if (!(box > 0.0) || !std::isfinite(box)) return fail(DGP_E_INVALID, "box must be > 0");
  if (precision != DGP_FP64 && precision != DGP_FP32) return fail(DGP_E_INVALID, "bad precision");
  return DGP_OK;
}

static void plan_init(dgp_plan* pl, int n, int batch, double box, int precision) {
  pl->n = n;
  pl->batch = batch;
  pl->box = box;
  pl->precision = precision;
  pl->n3 = (size_t)n * n * n;
  pl->hs = (size_t)(n / 2 + 1) * n * n;
}

static int adj_alloc(dgp_plan* pl);

static int plan_create(dgp_plan** out, int n, int batch, double box, int precision, void* ws, size_t ws_bytes) {
  if (!out) return fail(DGP_E_INVALID, "plan pointer is NULL");
  *out = nullptr;
  TRY(check_plan_sizes(n, batch, box, precision));
  dgp_plan* pl = new dgp_plan;
  plan_init(pl, n, batch, box, precision);
  pl->ws = static_cast<char*>(ws);
  pl->ws_bytes = ws ? ws_bytes : 0;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    delete pl;
    return fail(DGP_E_HIP, "hipGetDevice failed");
  }
  int r = ensure_twiddles(n);
  if (r == DGP_OK) r = plan_alloc(pl);
  if (r == DGP_OK && (hipEventCreate(&pl->ev0) != hipSuccess || hipEventCreate(&pl->ev1) != hipSuccess))
    r = fail(DGP_E_HIP, "hipEventCreate failed");
  if (r != DGP_OK) {
    plan_free(pl);
    return r;
  }
  *out = pl;
  return DGP_OK;
}

extern "C" int dgp_plan_create(dgp_plan** out, int n, int batch, double box, int precision) {
  return plan_create(out, n, batch, box, precision, nullptr, 0);
}

extern "C" size_t dgp_workspace_bytes(int n, int batch, int precision, int with_adjoint) {
  if (check_plan_sizes(n, batch, 1.0, precision) != DGP_OK) return 0;
  dgp_plan dry;
  dry.dry = true;
  plan_init(&dry, n, batch, 1.0, precision);
  if (plan_alloc(&dry) != DGP_OK) return 0;
  if (with_adjoint && adj_alloc(&dry) != DGP_OK) return 0;
  return dry.bytes;
}

extern "C" int dgp_plan_create_ws(dgp_plan** out, int n, int batch, double box, int precision, void* workspace,
                                  size_t workspace_bytes) {
  if (!out) return fail(DGP_E_INVALID, "plan pointer is NULL");
  *out = nullptr;
  TRY(check_plan_sizes(n, batch, box, precision));
  if (!workspace) return fail(DGP_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(DGP_E_INVALID, "workspace must be 256-byte aligned");
  const size_t need = dgp_workspace_bytes(n, batch, precision, 0);
  if (workspace_bytes < need)
    return fail(DGP_E_INVALID, "workspace of %zu bytes is smaller than the %zu bytes this plan needs", workspace_bytes,
                need);
  return plan_create(out, n, batch, box, precision, workspace, workspace_bytes);
}

extern "C" int dgp_plan_destroy(dgp_plan* pl) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  plan_free(pl);
  return DGP_OK;
}

extern "C" size_t dgp_plan_device_bytes(const dgp_plan* pl) { return pl ? pl->bytes : 0; }

// ------------------------------------------------------------------ helpers
static SpecCoef spec_coef(const dgp_plan* pl, const dgp_params* p) {
  SpecCoef c{};
  const bool nl = p->nonlocal != 0;
  c.kf = 2.0 * M_PI / pl->box;
  c.kappa = p->kappa;
  c.A = p->A;
  c.beta = nl ? p->beta : 0.0;
  c.alpha = p->alpha;
  c.gamma = nl ? p->gamma : 0.0;
  c.om15 = 1.5 * (p->eta - 1.0) / p->eta;
  c.inv2eta = 1.0 / (2.0 * p->eta);
  c.c2 = nl ? p->c2 : 0.0;
  c.inv_eta_nl = nl ? 1.0 / p->eta : 0.0;
  c.force_scale = kCOverH0 * kCOverH0;
  c.inv_n3 = 1.0 / double(pl->n3);
  c.lam2 = 2.0 * p->lambda;
  c.force_mode = p->force_mode;
  c.power_c = 0;
  c.nbins = 64;
  return c;
}

static SolveCfg solve_cfg(const dgp_plan* pl, const dgp_params* p, double tol, int max_iter) {
  SolveCfg c{};
  c.lam = p->lambda;
  c.w = p->w;
  c.alpha = p->alpha;
  c.gamma = p->nonlocal ? p->gamma : 0.0;
  c.omega = p->omega_relax;
  c.tol = tol;
  c.max_iter = max_iter;
  c.fixed = p->tol < 0.0 ? 1 : 0;
  c.n = pl->n;
  c.batch = pl->batch;
  return c;
}

// 3D forward transform of real fields [nb][n3] -> half spectrum [nb][hs] (axis 0 last index order kept)
template <typename T>
static int fwd3(dgp_plan* pl, const T* in, cx<T>* spec, int nb, const SolveCtl* ctl, hipStream_t s) {
  launch_p1_fwd<T>(pl->n, in, spec, nb, ctl, s);
  launch_p2<T>(pl->n, spec, 1, nb, -1, ctl, s);
  LAUNCHCHK();
  return DGP_OK;
}

// ------------------------------------------------------------------ the relaxation (one precision)
template <typename T>
struct Ws {
  T* U;
  T* S;
  cx<T>* spec_u;
  cx<T>* spec6;
  double* partial;
  int groups;
};

static Ws<double> ws64(dgp_plan* pl) { return {pl->U, pl->S, pl->spec_u, pl->spec6, pl->partial, pl->groups64}; }
static Ws<float> ws32(dgp_plan* pl) { return {pl->U32, pl->S32, pl->spec_u32, pl->spec6_32, pl->partial32, pl->groups32}; }

// S and the linear guess from delta (float64; S32 / U32 receive their float32 roundings when
// given).  The axis-0/1 spectrum of delta stays in spectral field 6, where the PM step's
// force computation picks it up.
static int setup_source(dgp_plan* pl, const dgp_params* p, const double* delta, Ws<double>& w, bool want_linear,
                        hipStream_t s, float* S32 = nullptr, float* U32 = nullptr) {
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  const SpecCoef cf = spec_coef(pl, p);
  Timed tm(pl, s, DGP_T_SETUP);
  cx<double>* dspec = w.spec6 + 6 * fs;
  TRY(fwd3<double>(pl, delta, dspec, B, nullptr, s));
  launch_p3<double>(n, SPEC_SOURCE, dspec, fs, 1, w.spec6, fs, 2, B, cf, nullptr, nullptr, nullptr, nullptr, s);
  launch_p2<double>(n, w.spec6, 2, B, +1, nullptr, s);
  launch_p1_inv<double>(n, w.spec6, w.S, B, nullptr, s, S32);
  if (want_linear) launch_p1_inv<double>(n, w.spec6 + fs, w.U, B, nullptr, s, U32);
  LAUNCHCHK();
  return DGP_OK;
}

// enqueue one relaxation pass on the iterate whose axis-0..1 spectrum is in spec_u
template <typename T>
static int enqueue_pass(dgp_plan* pl, const dgp_params* p, Ws<T>& w, const SolveCfg& cfg, hipStream_t s) {
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  const SpecCoef cf = spec_coef(pl, p);
  {
    Timed t(pl, s, tcls<T>(DGP_T_AXIS1_FWD));
    launch_p2<T>(n, w.spec_u, 1, B, -1, pl->ctl, s);
  }
  {
    Timed t(pl, s, tcls<T>(DGP_T_FANOUT));
    launch_p3<T>(n, SPEC_HSPLIT, w.spec_u, fs, 1, w.spec6, fs, 3, B, cf, nullptr, nullptr, pl->mean_u, pl->ctl, s);
  }
  {
    Timed t(pl, s, tcls<T>(DGP_T_AXIS1_INV));
    launch_p2_split<T>(n, w.spec6, fs, B, pl->ctl, s);
  }
  {
    TimedLaunch t(pl, tcls<T>(DGP_T_RELAX));
    launch_relax<T>(n, w.spec6, w.U, w.S, w.spec_u, w.partial, pl->mean_u, B, cfg, pl->ctl, s, t.a, t.b);
  }
  {
    Timed t(pl, s, tcls<T>(DGP_T_FINALIZE));
    launch_finalize(w.partial, w.groups, pl->ctl, cfg, pl->n_active, s);
  }
  LAUNCHCHK();
  return DGP_OK;
}

// Run passes until every batch element is done.  The host reads the control
// blocks between chunks and sizes the next chunk from the observed linear
// convergence rate, so few passes are launched after the last element has
// stopped (such launches exit at once but still cost a launch).  `first` sets
// the first chunk (0: two passes); with check = false the first chunk is only
// enqueued (no host round trip) and the loop returns.
template <typename T>
static int run_loop(dgp_plan* pl, const dgp_params* p, Ws<T>& w, const SolveCfg& cfg, hipStream_t s, int first,
                    bool check) {
  const int B = pl->batch;
  const int cap = p->check_every > 0 ? p->check_every : 4;
  int k = 0;
  int chunk = std::min(first > 0 ? first : 2, cfg.max_iter + 1);
  if (cfg.fixed && cfg.tol < 0.0) chunk = cfg.max_iter + 1;   // every pass is known in advance
  for (;;) {
    for (int i = 0; i < chunk && k <= cfg.max_iter; ++i, ++k) TRY(enqueue_pass<T>(pl, p, w, cfg, s));
    if (!check) return DGP_OK;
    HIPCHK(hipMemcpyAsync(pl->ctl_host, pl->ctl, sizeof(SolveCtl) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    timing_flush(pl);
    int active = 0, next = cap;
    for (int b = 0; b < B; ++b) {
      const SolveCtl& C = pl->ctl_host[b];
      if (C.done) continue;
      ++active;
      int m = 1;
      const int n = C.iters;   // the next pass evaluates iterate n; hist[n-1], hist[n-2] are known
      if (n >= 2 && n - 1 < kMaxHist) {
        const double r1 = C.hist[n - 1], r0 = C.hist[n - 2];
        if (r1 > 0.0 && r0 > r1 && cfg.tol > 0.0) {
          const double need = std::log(cfg.tol / r1) / std::log(r1 / r0);
          m = need <= 1.0 ? 1 : int(std::ceil(need));
        }
      }
      next = std::min(next, std::max(1, m));
    }
    if (active == 0 || k > cfg.max_iter) break;
    chunk = next;
  }
  return DGP_OK;
}

// passes the slowest element needed (control blocks already on the host)
static int max_passes(const dgp_plan* pl) {
  int m = 0;
  for (int b = 0; b < pl->batch; ++b) m = std::max(m, pl->ctl_host[b].passes);
  return m;
}

static int status_rank(int st) { return st == DGP_OK ? 0 : (st == DGP_NOT_CONVERGED ? 2 : 1); }

// Enqueue the copy of the decided iterates into u_state (the device picks each
// element's buffer), their means, and the copies of the control blocks and means to
// pinned host memory.  collect_finish reads them once the stream has been synchronised.
template <typename T>
static int collect_enqueue(dgp_plan* pl, Ws<T>& w, double* u_state, hipStream_t s) {
  const int B = pl->batch;
  launch_take_result<T>(pl->ctl, w.U, B, pl->n3, u_state, pl->red, pl->vec + B, s);
  HIPCHK(hipMemcpyAsync(pl->means_host, pl->vec + B, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(pl->ctl_host, pl->ctl, sizeof(SolveCtl) * B, hipMemcpyDeviceToHost, s));
  LAUNCHCHK();
  return DGP_OK;
}

// After the stream is synchronised: fill info and return the worst status.
static int collect_finish(dgp_plan* pl, dgp_info* info, float ms) {
  int worst = DGP_OK, invalid = -1;
  for (int b = 0; b < pl->batch; ++b) {
    const SolveCtl& C = pl->ctl_host[b];
    if (C.status == kStatusInvalid) {
      if (invalid < 0) invalid = b;
    } else if (status_rank(C.status) > status_rank(worst)) {
      worst = C.status;
    }
    if (!info) continue;
    info[b].status = C.status == kStatusInvalid ? DGP_E_INVALID : C.status;
    info[b].iters = C.iters1 + C.iters;
    info[b].passes = C.passes1 + C.passes;
    info[b].passes_fp64 = C.passes;
    info[b].resid = C.resid;
    info[b].resid_min = C.resid_min;
    info[b].eps = C.eps;
    info[b].bad_fraction = C.bad_frac;
    info[b].mean_u = pl->means_host[b];
    info[b].ms_total = ms;
  }
  if (invalid >= 0)
    return fail(DGP_E_INVALID, "batch element %d: non-finite input or iterate (delta, particle positions or the "
                "warm-start field); no output is valid", invalid);
  return worst;
}

// C = lapbar^{-1} u for [B] fields
static int c_field(dgp_plan* pl, const dgp_params* p, const double* u, double* c_out, hipStream_t s) {
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  const SpecCoef cf = spec_coef(pl, p);
  TRY(fwd3<double>(pl, u, pl->spec_u, B, nullptr, s));
  launch_p3<double>(n, SPEC_CFIELD, pl->spec_u, fs, 1, pl->spec6, fs, 1, B, cf, nullptr, nullptr, nullptr, nullptr, s);
  launch_p2<double>(n, pl->spec6, 1, B, +1, nullptr, s);
  launch_p1_inv<double>(n, pl->spec6, c_out, B, nullptr, s);
  LAUNCHCHK();
  return DGP_OK;
}

// plain float64 solve from the chosen initial iterate
static int solve64(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s) {
  Ws<double> w = ws64(pl);
  const int B = pl->batch;
  TRY(setup_source(pl, p, delta, w, p->init == DGP_INIT_LINEAR, s));
  if (p->init == DGP_INIT_WARM) {
    HIPCHK(hipMemcpyAsync(w.U, u_state, sizeof(double) * B * pl->n3, hipMemcpyDeviceToDevice, s));
  } else if (p->init == DGP_INIT_ZERO) {
    launch_fill_zero(w.U, (size_t)B * pl->n3, s);
  }
  launch_absmean<double>(pl->n3, w.S, B, pl->red, pl->vec, nullptr, s);
  launch_ctl_init(pl->ctl, pl->vec, B, s);
  // a pass starts from the axis-0 spectrum of its iterate (what the fused pass writes)
  launch_p1_fwd<double>(pl->n, w.U, w.spec_u, B, nullptr, s);
  const SolveCfg cfg = solve_cfg(pl, p, p->tol, p->max_iter);
  TRY(run_loop<double>(pl, p, w, cfg, s, pl->hint64, true));
  pl->hint64 = max_passes(pl);
  return collect_enqueue<double>(pl, w, u_state, s);
}

int solve32_polish(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s);

// Enqueue a solve in the plan's form; ends with collect_enqueue (no final synchronisation).
static int solve_spherical(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s);

static int solve_enqueue(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s) {
  if (p->spherical) return solve_spherical(pl, p, delta, u_state, s);
  return pl->precision == DGP_FP32 ? solve32_polish(pl, p, delta, u_state, s) : solve64(pl, p, delta, u_state, s);
}

// Spherical approximation (Eqs. FullDGP2sph, SphPoi): the source in float64, then the first
// w = 1/3 update from u = 0, which at u = 0 is a pointwise function of S (the nonlocal linear
// terms enter through S, as in the paper's spherical runs).
static int solve_spherical(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s) {
  Ws<double> w = ws64(pl);
  const int B = pl->batch;
  TRY(setup_source(pl, p, delta, w, false, s));
  launch_absmean<double>(pl->n3, w.S, B, pl->red, pl->vec, nullptr, s);
  launch_spherical(pl->n3, B, w.S, w.U, p->alpha, p->lambda, pl->partial, pl->ctl, pl->vec, s);
  return collect_enqueue<double>(pl, w, u_state, s);
}

extern "C" int dgp_solve_field(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, double* c_out,
                               dgp_info* info, void* stream) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  TRY(check_params(p));
  if (!delta || !u_state) return fail(DGP_E_INVALID, "delta and u_state are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipEventRecord(pl->ev0, s));
  TRY(solve_enqueue(pl, p, delta, u_state, s));
  if (c_out) TRY(c_field(pl, p, u_state, c_out, s));
  HIPCHK(hipEventRecord(pl->ev1, s));
  HIPCHK(hipEventSynchronize(pl->ev1));
  timing_flush(pl);
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
  return collect_finish(pl, info, ms);
}

// ------------------------------------------------------------------ precision form: float32 passes + float64 polish
#ifndef DGP_SWITCH_TOL
#define DGP_SWITCH_TOL 1e-6
#endif

// Phase 1 runs float32 relaxation passes (float64 pointwise arithmetic and
// reductions) from the initial guess until the float32 residual reaches
// max(tol, switch_tol) (or phase 1 ends on max_iter or bad points); phase 2
// continues with float64 passes, from the update that the last float32 pass
// computed, until the float64 residual meets tol.  The returned residual is always
// a float64 evaluation.
int solve32_polish(dgp_plan* pl, const dgp_params* p, const double* delta, double* u_state, hipStream_t s) {
  const int B = pl->batch;
  const size_t n3 = pl->n3;
  Ws<float> w32 = ws32(pl);
  Ws<double> w = ws64(pl);
  // the source (and the linear guess) are formed once in float64: phase 2 needs them
  // exact, and phase 1 takes their rounding, which is closer than a float32 evaluation
  // the float64 initial guess stays in the float64 phase's first buffer (the warm start of
  // phase 2 if phase 1 accepts the initial guess as it is)
  TRY(setup_source(pl, p, delta, w, p->init == DGP_INIT_LINEAR, s, w32.S, w32.U));
  if (p->init == DGP_INIT_WARM) {
    HIPCHK(hipMemcpyAsync(w.U, u_state, sizeof(double) * B * n3, hipMemcpyDeviceToDevice, s));
    launch_convert<float>(B * n3, u_state, 0, w32.U, s);
  } else if (p->init == DGP_INIT_ZERO) {
    launch_fill_zero(w.U, (size_t)B * n3, s);
    launch_fill_zero(w32.U, (size_t)B * n3 / 2, s);   // n3 is even
  }
  // eps = <|S|> of the float64 source; it stays in the control blocks for both phases
  launch_absmean<double>(n3, w.S, B, pl->red, pl->vec, nullptr, s);
  launch_ctl_init(pl->ctl, pl->vec, B, s);
  launch_p1_fwd<float>(pl->n, w32.U, w32.spec_u, B, nullptr, s);
  const double switch_tol = std::max(p->tol, double(DGP_SWITCH_TOL));
  const SolveCfg cfg32 = solve_cfg(pl, p, switch_tol, p->max_iter);
  // phase 1: after the plan's first solve, one pass more than the last solve's phase 1
  // took, enqueued without a host round trip (passes after an element stops exit at once;
  // an element still running at the end continues in phase 2)
  if (pl->hint32 > 0)
    TRY(run_loop<float>(pl, p, w32, cfg32, s, pl->hint32 + 1, false));
  else
    TRY(run_loop<float>(pl, p, w32, cfg32, s, 0, true));
  launch_handoff(pl->ctl, w32.U, B, n3, w.U, s);
  launch_p1_fwd<double>(pl->n, w.U, w.spec_u, B, nullptr, s);
  const SolveCfg cfg = solve_cfg(pl, p, p->tol, p->max_iter);
  TRY(run_loop<double>(pl, p, w, cfg, s, pl->hint64, true));
  // learn the pass counts for the next solve on this plan
  int p1 = 0;
  bool cut = false;
  for (int b = 0; b < B; ++b) {
    p1 = std::max(p1, pl->ctl_host[b].passes1);
    cut = cut || !pl->ctl_host[b].phase1_done;
  }
  pl->hint32 = cut ? p1 + 2 : p1;
  pl->hint64 = max_passes(pl);
  return collect_enqueue<double>(pl, w, u_state, s);
}

// ------------------------------------------------------------------ PM
static int require_batch1(const dgp_plan* pl) {
  if (pl->batch != 1) return fail(DGP_E_UNSUPPORTED, "particle entry points need a batch-1 plan");
  return DGP_OK;
}

// (a non-finite position raises the plan's flag and turns delta into NaN, which the solve's
// source then reports as invalid input)
static int deposit_impl(dgp_plan* pl, const void* pos, int fp32, long long np, long long* grid, double* delta,
                        bool remove_mean, hipStream_t s) {
  Timed tm(pl, s, DGP_T_DEPOSIT);
  launch_fill_zero(grid, pl->n3, s);
  launch_zero_flag(pl->flag, s);
  launch_deposit(pl->n, pl->box, pos, fp32, np, grid, pl->flag, s);
  if (delta) {
    if (remove_mean) {   // the mean of the counts (deterministic reduction), removed in the same pass
      launch_absmean<long long>(pl->n3, grid, 1, pl->red, nullptr, pl->vec, s);
      launch_counts_to_delta(pl->n, grid, np, delta, pl->flag, s, pl->vec);
    } else {
      launch_counts_to_delta(pl->n, grid, np, delta, pl->flag, s);
    }
  }
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_deposit(dgp_plan* pl, const void* pos, int pos_is_fp32, long long np, long long* grid_fixed,
                           double* delta, void* stream) {
  if (!pl || !pos || np < 1) return fail(DGP_E_INVALID, "plan, pos and np >= 1 are required");
  TRY(require_batch1(pl));
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(deposit_impl(pl, pos, pos_is_fp32, np, grid_fixed ? grid_fixed : pl->grid, delta, true, s));
  if (!grid_fixed && !delta) return DGP_OK;
  return DGP_OK;
}

// force mesh g = -(c/H0)^2 grad phi, [3][n3] (and phi into phi_n when given).  A float64
// plan forms it in float64 into mesh3; a precision-form plan forms it with float32 transforms
// into mesh3_32 (the field solve itself stays polished to the float64 tolerance).
// delta_ready: spectral field 6 already holds the float64 axis-0/1 spectrum of delta (left
// there by the solve's setup on the same delta).
static int force_mesh(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u, double* phi_n,
                      bool delta_ready, hipStream_t s) {
  Timed tm(pl, s, DGP_T_FORCES);
  const int n = pl->n;
  const size_t fs = pl->hs, n3 = pl->n3;
  SpecCoef cf = spec_coef(pl, p);
  if (p->force_mode == DGP_FORCE_GR) {   // Eq. GRPoisson in the LCDM background: kbar = c k/(a H), (3/2) Omega_m(a)
    const double e = hubble_E_lcdm(p->omega_m0, p->a);
    cf.kappa = kCOverH0 / (p->a * e);
    cf.om15 = 1.5 * p->omega_m0 / (p->a * p->a * p->a * e * e);
  }
  const bool use_u = p->force_mode == DGP_FORCE_NLDGP;
  if (pl->precision == DGP_FP32) {
    cx<float>* fin = pl->spec6_32 + 6 * fs;   // delta, then u
    float* tmp = pl->U32;                     // the solve's float32 iterates are free here
    if (delta_ready)
      launch_convert<float>(2 * fs, pl->spec6 + 6 * fs, 0, reinterpret_cast<float*>(fin), s);
    else
      launch_p1_fwd_from64(n, delta, fin, 1, nullptr, s);
    if (use_u) launch_p1_fwd_from64(n, u, fin + fs, 1, nullptr, s);
    if (!delta_ready)
      launch_p2<float>(n, fin, use_u ? 2 : 1, 1, -1, nullptr, s);
    else if (use_u)
      launch_p2<float>(n, fin + fs, 1, 1, -1, nullptr, s);
    launch_p3<float>(n, SPEC_FORCES, fin, fs, use_u ? 2 : 1, pl->spec6_32, fs, 2, 1, cf, nullptr, nullptr, nullptr,
                     nullptr, s);
    launch_p2_force_split<float>(n, pl->spec6_32, fs, 1, phi_n ? 1 : 0, cf.force_scale * cf.kf, s);
    launch_p1_inv<float>(n, pl->spec6_32, pl->mesh3_32, 3, nullptr, s);
    if (phi_n) {
      launch_p1_inv<float>(n, pl->spec6_32 + 3 * fs, tmp, 1, nullptr, s);
      launch_convert<double>(n3, tmp, 1, phi_n, s);
    }
    LAUNCHCHK();
    return DGP_OK;
  }
  cx<double>* fin = pl->spec6 + 6 * fs;   // delta, then u
  if (!delta_ready) launch_p1_fwd<double>(n, delta, fin, 1, nullptr, s);
  if (use_u) launch_p1_fwd<double>(n, u, fin + fs, 1, nullptr, s);
  if (!delta_ready)
    launch_p2<double>(n, fin, use_u ? 2 : 1, 1, -1, nullptr, s);
  else if (use_u)
    launch_p2<double>(n, fin + fs, 1, 1, -1, nullptr, s);
  launch_p3<double>(n, SPEC_FORCES, fin, fs, use_u ? 2 : 1, pl->spec6, fs, 2, 1, cf, nullptr, nullptr, nullptr,
                    nullptr, s);
  launch_p2_force_split<double>(n, pl->spec6, fs, 1, phi_n ? 1 : 0, cf.force_scale * cf.kf, s);
  launch_p1_inv<double>(n, pl->spec6, pl->mesh3, 3, nullptr, s);
  if (phi_n) launch_p1_inv<double>(n, pl->spec6 + 3 * fs, phi_n, 1, nullptr, s);
  LAUNCHCHK();
  return DGP_OK;
}

// the plan's force mesh and its element type
static const void* mesh_of(const dgp_plan* pl, int* fp32) {
  *fp32 = pl->precision == DGP_FP32 ? 1 : 0;
  return *fp32 ? static_cast<const void*>(pl->mesh3_32) : static_cast<const void*>(pl->mesh3);
}

extern "C" int dgp_pm_forces(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u_state,
                             const void* pos, int pos_is_fp32, long long np, double* force, double* phi_n,
                             void* stream) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  TRY(check_params(p));
  TRY(require_batch1(pl));
  if (!delta || !pos || !force || np < 1) return fail(DGP_E_INVALID, "delta, pos, force and np >= 1 are required");
  if (p->force_mode == DGP_FORCE_NLDGP && !u_state) return fail(DGP_E_INVALID, "u_state is required for nlDGP forces");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(force_mesh(pl, p, delta, u_state, phi_n, false, s));
  int mfp32 = 0;
  const void* mesh = mesh_of(pl, &mfp32);
  launch_interp(pl->n, pl->box, mesh, mfp32, 3, pos, pos_is_fp32, np, force, s);
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_step(dgp_plan* pl, const dgp_params* p, void* pos, void* vel, int is_fp32, long long np, double dlna,
                        double* u_state, dgp_info* info, void* stream) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  TRY(check_params(p));
  TRY(require_batch1(pl));
  if (!pos || !vel || !u_state || np < 1) return fail(DGP_E_INVALID, "pos, vel, u_state and np >= 1 are required");
  if (!std::isfinite(dlna)) return fail(DGP_E_INVALID, "dlna must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(deposit_impl(pl, pos, is_fp32, np, pl->grid, pl->delta, false, s));
  const bool solve = p->force_mode == DGP_FORCE_NLDGP;
  if (solve) {
    HIPCHK(hipEventRecord(pl->ev0, s));
    TRY(solve_enqueue(pl, p, pl->delta, u_state, s));
    HIPCHK(hipEventRecord(pl->ev1, s));
  }
  TRY(force_mesh(pl, p, pl->delta, u_state, nullptr, solve, s));
  const double a = p->a;
  double (*const hub)(double, double) = p->force_mode == DGP_FORCE_GR ? hubble_E_lcdm : hubble_E;
  const double e_n = hub(p->omega_m0, a);
  const double a_h = a * std::exp(0.5 * dlna);
  const double e_h = hub(p->omega_m0, a_h);
  const double kick = dlna / e_n;
  const double drift = dlna / (a_h * a_h * e_h);
  {
    Timed tm(pl, s, DGP_T_INTERP_KICK);
    int mfp32 = 0;
    const void* mesh = mesh_of(pl, &mfp32);
    launch_interp_kick_drift(pl->n, pl->box, mesh, mfp32, pos, vel, is_fp32, np, kick, drift, s);
  }
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(pl->flag_host, pl->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  timing_flush(pl);
  if (*pl->flag_host)
    return fail(DGP_E_INVALID, "non-finite particle position: the step's outputs are not valid");
  if (!solve) return DGP_OK;
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
  return collect_finish(pl, info, ms);
}

extern "C" int dgp_deposit_noalloc(int n, double box, const void* pos, int pos_is_fp32, long long np,
                                   long long* grid_fixed, double* delta, void* stream) {
  if (!pos || !grid_fixed || !delta || np < 1) return fail(DGP_E_INVALID, "pos, grid_fixed, delta and np >= 1 are required");
  if (n < 8 || n > 512 || (n & (n - 1)) != 0) return fail(DGP_E_INVALID, "N must be a power of two in [8, 512], got %d", n);
  if (!(box > 0.0) || !std::isfinite(box)) return fail(DGP_E_INVALID, "box must be > 0");
  double* sc = nullptr;
  size_t cap = 0;
  const int r = noalloc_scratch(&sc, &cap);
  if (r != 0) return fail(r == -2 ? DGP_E_UNSUPPORTED : DGP_E_HIP, "device scratch of the allocation-free deposit unavailable");
  const size_t n3 = (size_t)n * n * n;
  const size_t parts = absmean_scratch_doubles(n3, 1);
  if (parts + 4 > cap)
    return fail(DGP_E_INVALID, "N = %d needs %zu scratch doubles, the allocation-free deposit has %zu", n, parts + 4, cap);
  double* mean = sc + parts;
  int* flag = reinterpret_cast<int*>(sc + parts + 2);
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_fill_zero(grid_fixed, n3, s);
  launch_zero_flag(flag, s);
  launch_deposit(n, box, pos, pos_is_fp32, np, grid_fixed, flag, s);
  launch_absmean<long long>(n3, grid_fixed, 1, sc, nullptr, mean, s);
  launch_counts_to_delta(n, grid_fixed, np, delta, flag, s, mean);
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_interp(dgp_plan* pl, const double* mesh, int ncomp, const void* pos, int pos_is_fp32, long long np,
                          double* out, void* stream) {
  if (!pl || !mesh || !pos || !out || np < 1) return fail(DGP_E_INVALID, "plan, mesh, pos, out and np >= 1 are required");
  if (ncomp < 1 || ncomp > 3) return fail(DGP_E_INVALID, "ncomp must be in [1, 3]");
  TRY(require_batch1(pl));
  launch_interp(pl->n, pl->box, mesh, 0, ncomp, pos, pos_is_fp32, np, out, static_cast<hipStream_t>(stream));
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_interp_backward(dgp_plan* pl, const double* mesh, int ncomp, const void* pos, int pos_is_fp32,
                                   long long np, const double* grad_out, double* grad_pos, double* grad_mesh,
                                   void* stream) {
  if (!pl || !pos || !grad_out || np < 1) return fail(DGP_E_INVALID, "plan, pos, grad_out and np >= 1 are required");
  if (ncomp < 1 || ncomp > 3) return fail(DGP_E_INVALID, "ncomp must be in [1, 3]");
  if (!grad_pos && !grad_mesh) return fail(DGP_E_INVALID, "nothing to compute: grad_pos and grad_mesh are both NULL");
  if (grad_pos && !mesh) return fail(DGP_E_INVALID, "grad_pos needs the mesh");
  TRY(require_batch1(pl));
  launch_interp_backward(pl->n, pl->box, mesh, ncomp, pos, pos_is_fp32, np, grad_out, grad_pos, grad_mesh, pl->grid,
                         pl->fx_state, pl->flag, static_cast<hipStream_t>(stream));
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_deposit_backward(dgp_plan* pl, const void* pos, int pos_is_fp32, long long np,
                                    const double* grad_delta, double* grad_pos, void* stream) {
  if (!pl || !pos || !grad_delta || !grad_pos || np < 1) return fail(DGP_E_INVALID, "missing argument");
  TRY(require_batch1(pl));
  launch_deposit_backward(pl->n, pl->box, pos, pos_is_fp32, np, grad_delta, grad_pos, static_cast<hipStream_t>(stream));
  LAUNCHCHK();
  return DGP_OK;
}

// ------------------------------------------------------------------ power spectrum
static void bin_thresholds(int n, int nbins, std::vector<double>& t) {
  t.resize(nbins + 1);
  const double half = n / 2;
  for (int b = 0; b <= nbins; ++b) t[b] = std::ceil(std::pow(half, 2.0 * b / nbins));
  t[nbins] = half * half + 1.0;
}

static int power_impl(dgp_plan* pl, const dgp_params* p, const double* field, int of_c, int nbins,
                      std::vector<double>& sums, std::vector<double>& cnts, hipStream_t s) {
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  std::vector<double> thr;
  bin_thresholds(n, nbins, thr);
  HIPCHK(hipMemcpyAsync(pl->bin_tab, thr.data(), sizeof(double) * thr.size(), hipMemcpyHostToDevice, s));
  SpecCoef cf = spec_coef(pl, p);
  cf.nbins = nbins;
  cf.power_c = of_c ? 1 : 0;
  TRY(fwd3<double>(pl, field, pl->spec_u, B, nullptr, s));
  launch_p3<double>(n, SPEC_POWER, pl->spec_u, fs, 1, nullptr, 0, 0, B, cf, pl->bin_tab, pl->bin_partial, nullptr,
                    nullptr, s);
  LAUNCHCHK();
  const int g = p3_row_groups(n);
  const size_t cnt = (size_t)B * g * 2 * nbins;
  HIPCHK(hipMemcpyAsync(pl->bin_host, pl->bin_partial, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  sums.assign((size_t)B * nbins, 0.0);
  cnts.assign((size_t)B * nbins, 0.0);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < g; ++k) {
      const double* row = pl->bin_host + ((size_t)b * g + k) * 2 * nbins;
      for (int i = 0; i < nbins; ++i) {
        sums[(size_t)b * nbins + i] += row[i];
        cnts[(size_t)b * nbins + i] += row[nbins + i];
      }
    }
  return DGP_OK;
}

extern "C" int dgp_power_spectrum(dgp_plan* pl, const dgp_params* p, const double* field, int of_c, int nbins,
                                  double* pk, double* counts, void* stream) {
  if (!pl || !field || !pk) return fail(DGP_E_INVALID, "missing argument");
  TRY(check_params(p));
  if (nbins < 1 || nbins > 128) return fail(DGP_E_INVALID, "nbins must be in [1, 128]");
  std::vector<double> sums, cnts;
  TRY(power_impl(pl, p, field, of_c, nbins, sums, cnts, static_cast<hipStream_t>(stream)));
  const double norm = std::pow(pl->box, 3) / (double(pl->n3) * double(pl->n3));
  for (int b = 0; b < pl->batch; ++b)
    for (int i = 0; i < nbins; ++i) {
      const double c = cnts[(size_t)b * nbins + i];
      pk[(size_t)b * nbins + i] = c > 0 ? sums[(size_t)b * nbins + i] / c * norm : 0.0;
    }
  if (counts)
    for (int i = 0; i < nbins; ++i) counts[i] = cnts[i];
  return DGP_OK;
}

extern "C" int dgp_power_spectrum_backward(dgp_plan* pl, const dgp_params* p, const double* field, int of_c,
                                           int nbins, const double* grad_pk, double* grad_field, void* stream) {
  if (!pl || !field || !grad_pk || !grad_field) return fail(DGP_E_INVALID, "missing argument");
  TRY(check_params(p));
  if (nbins < 1 || nbins > 128) return fail(DGP_E_INVALID, "nbins must be in [1, 128]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<double> sums, cnts;
  TRY(power_impl(pl, p, field, of_c, nbins, sums, cnts, s));
  const int n = pl->n, B = pl->batch;
  std::vector<double> tab;
  bin_thresholds(n, nbins, tab);
  const double norm = std::pow(pl->box, 3) / (double(pl->n3) * double(pl->n3));
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < nbins; ++i) {
      const double c = cnts[(size_t)b * nbins + i];
      tab.push_back(c > 0 ? grad_pk[(size_t)b * nbins + i] * norm / c * 2.0 * double(pl->n3) : 0.0);
    }
  HIPCHK(hipMemcpyAsync(pl->bin_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s));
  SpecCoef cf = spec_coef(pl, p);
  cf.nbins = nbins;
  cf.power_c = of_c ? 1 : 0;
  const size_t fs = (size_t)B * pl->hs;
  TRY(fwd3<double>(pl, field, pl->spec_u, B, nullptr, s));
  launch_p3<double>(n, SPEC_POWER_GRAD, pl->spec_u, fs, 1, pl->spec6, fs, 1, B, cf, pl->bin_tab, nullptr, nullptr,
                    nullptr, s);
  launch_p2<double>(n, pl->spec6, 1, B, +1, nullptr, s);
  launch_p1_inv<double>(n, pl->spec6, grad_field, B, nullptr, s);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return DGP_OK;
}

// ------------------------------------------------------------------ raw transforms (tests of the FFT itself)
extern "C" int dgp_fft_forward(dgp_plan* pl, const double* field, double* spectrum, void* stream) {
  if (!pl || !field || !spectrum) return fail(DGP_E_INVALID, "missing argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  dgp_params p;
  dgp_params_init(&p, 0.27, 1.0);
  const SpecCoef cf = spec_coef(pl, &p);
  if (pl->precision == DGP_FP64) {
    TRY(fwd3<double>(pl, field, pl->spec_u, B, nullptr, s));
    launch_p3<double>(n, SPEC_FWD_ONLY, pl->spec_u, fs, 1, reinterpret_cast<cx<double>*>(spectrum), fs, 1, B, cf,
                      nullptr, nullptr, nullptr, nullptr, s);
  } else {
    launch_convert<float>(B * pl->n3, field, 0, pl->U32, s);
    TRY(fwd3<float>(pl, pl->U32, pl->spec_u32, B, nullptr, s));
    launch_p3<float>(n, SPEC_FWD_ONLY, pl->spec_u32, fs, 1, pl->spec6_32, fs, 1, B, cf, nullptr, nullptr, nullptr,
                     nullptr, s);
    launch_convert<double>(2 * fs, pl->spec6_32, 1, spectrum, s);
  }
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_fft_inverse(dgp_plan* pl, const double* spectrum, double* field, void* stream) {
  if (!pl || !field || !spectrum) return fail(DGP_E_INVALID, "missing argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs;
  dgp_params p;
  dgp_params_init(&p, 0.27, 1.0);
  const SpecCoef cf = spec_coef(pl, &p);
  if (pl->precision == DGP_FP64) {
    launch_p3<double>(n, SPEC_INV_ONLY, reinterpret_cast<const cx<double>*>(spectrum), fs, 1, pl->spec_u, fs, 1, B, cf,
                      nullptr, nullptr, nullptr, nullptr, s);
    launch_p2<double>(n, pl->spec_u, 1, B, +1, nullptr, s);
    launch_p1_inv<double>(n, pl->spec_u, field, B, nullptr, s);
  } else {
    launch_convert<float>(2 * fs, spectrum, 0, reinterpret_cast<float*>(pl->spec6_32), s);
    launch_p3<float>(n, SPEC_INV_ONLY, pl->spec6_32, fs, 1, pl->spec_u32, fs, 1, B, cf, nullptr, nullptr, nullptr,
                     nullptr, s);
    launch_p2<float>(n, pl->spec_u32, 1, B, +1, nullptr, s);
    launch_p1_inv<float>(n, pl->spec_u32, pl->U32, B, nullptr, s);
    launch_convert<double>(B * pl->n3, pl->U32, 1, field, s);
  }
  LAUNCHCHK();
  return DGP_OK;
}

int adjoint_solve(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u_star, const double* grad_u,
                  double* grad_delta, dgp_info* info, hipStream_t s);

// float64 work fields of the adjoint and the diagnostics, allocated on first use: [9][B][n3]
// (five Hessians, three multiplier buffers, the returned multipliers), reduction scratch and
// the adjoint's own control blocks (the forward solve's stay as its last solve left them)
// the adjoint's device buffers (Hessians of u*, multipliers, reductions, control blocks)
static int adj_alloc(dgp_plan* pl) {
  const size_t bn = (size_t)pl->batch * pl->n3;
  TRY(dalloc(pl, &pl->adj, 9 * bn));
  const size_t red = std::max((size_t)adjoint_groups(pl->n3) * 2, (size_t)adj_step_groups(pl->n) * 3);
  TRY(dalloc(pl, &pl->adj_red, red * pl->batch));
  TRY(dalloc(pl, &pl->adj_vec, pl->batch));
  TRY(dalloc(pl, &pl->adj_ctl, pl->batch));
  TRY(halloc(pl, &pl->adj_ctl_host, pl->batch));
  return DGP_OK;
}

static int ensure_adj(dgp_plan* pl) {
  if (pl->adj_ctl_host) return DGP_OK;
  return adj_alloc(pl);
}

// h00, h11, h01, h02, h12 of u (H5: [5][B][n3]; h22 follows from the trace identity) and <u>
// into pl->mean_u, float64
static int hessians(dgp_plan* pl, const dgp_params* p, const double* u, double* H5, hipStream_t s) {
  const int n = pl->n, B = pl->batch;
  const size_t fs = (size_t)B * pl->hs, bn = (size_t)B * pl->n3;
  const SpecCoef cf = spec_coef(pl, p);
  TRY(fwd3<double>(pl, u, pl->spec_u, B, nullptr, s));
  launch_p3<double>(n, SPEC_HSPLIT, pl->spec_u, fs, 1, pl->spec6, fs, 3, B, cf, nullptr, nullptr, pl->mean_u, nullptr,
                    s);
  launch_p2_split<double>(n, pl->spec6, fs, B, nullptr, s);
  for (int f = 0; f < 5; ++f) launch_p1_inv<double>(n, pl->spec6 + f * fs, H5 + f * bn, B, nullptr, s);
  LAUNCHCHK();
  return DGP_OK;
}

extern "C" int dgp_solve_field_backward(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u_star,
                                        const double* grad_u, double* grad_delta, dgp_info* info, void* stream) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  TRY(check_params(p));
  if (!delta || !u_star || !grad_u || !grad_delta) return fail(DGP_E_INVALID, "missing argument");
  return adjoint_solve(pl, p, delta, u_star, grad_u, grad_delta, info, static_cast<hipStream_t>(stream));
}

// Transposed relaxation mu <- D^{-1} (g + M^T mu) (see adjoint.hip), then dL/ddelta = S mu.
int adjoint_solve(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u_star, const double* grad_u,
                  double* grad_delta, dgp_info* info, hipStream_t s) {
  (void)delta;   // S does not depend on delta; the solve's delta only fixed u*
  const int n = pl->n, B = pl->batch;
  const size_t n3 = pl->n3, fs = (size_t)B * pl->hs, bn = (size_t)B * n3;
  TRY(ensure_adj(pl));
  double* H5 = pl->adj;
  double* MU = pl->adj + 5 * bn;    // three multiplier buffers, bn apart
  double* RES = pl->adj + 8 * bn;   // the returned multipliers, gathered per element
  const SpecCoef cf = spec_coef(pl, p);
  const double lam = p->lambda, w = p->w, alpha = p->alpha;
  const AdjCoef ak{2.0 * lam, w, alpha, 2.0 * (1.0 - w) * lam};
  const int G = adjoint_groups(n3), GS = adj_step_groups(n);
  // Hessians of u* (h00, h11, h01, h02, h12) and <u*>
  TRY(hessians(pl, p, u_star, H5, s));
  // mu_0 = g / D into buffer 0, with the checks that D stays away from 0 and g is finite
  launch_adj_init(n3, B, grad_u, u_star, MU, ak.dscale, alpha, pl->adj_red, s);
  launch_pair_means(pl->adj_red, G, n3, B, pl->vec, pl->vec + B, s);
  LAUNCHCHK();
  std::vector<double> host(2 * B);
  HIPCHK(hipMemcpyAsync(host.data(), pl->vec, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b) {
    if (host[b] > 0.0)
      return fail(DGP_E_INVALID, "batch element %d: u* has points where 2 (1-w) lam u + alpha <= 1e-12 alpha "
                  "(bad-point vertices of an unconverged solve) or non-finite values; the implicit adjoint does not "
                  "exist there", b);
    if (host[B + b] > 0.0) return fail(DGP_E_INVALID, "batch element %d: grad_u is not finite", b);
  }
  // device control: element b's multiplier k lives in MU + buf * bn + b * n3 (buffers rotate)
  for (int b = 0; b < B; ++b) {
    SolveCtl& C = pl->adj_ctl_host[b];
    std::memset(&C, 0, sizeof(SolveCtl));
    C.cur = 0;
    C.out = 1;
    C.best = 0;
    C.resid_min = std::numeric_limits<double>::infinity();
  }
  HIPCHK(hipMemcpyAsync(pl->adj_ctl, pl->adj_ctl_host, sizeof(SolveCtl) * B, hipMemcpyHostToDevice, s));
  // products of mu_0 and their axis-0 transforms, <h22 mu_0>
  launch_adj_step(n, false, nullptr, MU, bn, u_star, H5, grad_u, pl->mean_u, pl->adj_vec, pl->spec6, fs, pl->adj_red,
                  ak, pl->adj_ctl, B, s);
  launch_adj_finalize(false, pl->adj_red, GS, pl->adj_ctl, pl->adj_vec, n3, p->tol, p->max_iter, B, s);
  LAUNCHCHK();
  // iterations in chunks; the host only reads the control blocks between chunks (iterations of
  // an element that has decided exit at once)
  const int limit = std::max(p->max_iter, 0) + 1;   // evaluations an element can take
  int enqueued = 0;
  int chunk = 4;
  while (enqueued < limit) {
    const int m = std::min(chunk, limit - enqueued);
    for (int j = 0; j < m; ++j) {
      launch_p2_adj_split(n, pl->spec6, fs, B, cf.lam2, pl->adj_ctl, s);
      launch_p3<double>(n, SPEC_ADJ_COMBINE3, pl->spec6, fs, 3, pl->spec_u, fs, 1, B, cf, nullptr, nullptr, nullptr,
                        pl->adj_ctl, s);
      launch_p2<double>(n, pl->spec_u, 1, B, +1, pl->adj_ctl, s);
      launch_adj_step(n, true, pl->spec_u, MU, bn, u_star, H5, grad_u, pl->mean_u, pl->adj_vec, pl->spec6, fs,
                      pl->adj_red, ak, pl->adj_ctl, B, s);
      launch_adj_finalize(true, pl->adj_red, GS, pl->adj_ctl, pl->adj_vec, n3, p->tol, p->max_iter, B, s);
    }
    LAUNCHCHK();
    enqueued += m;
    HIPCHK(hipMemcpyAsync(pl->adj_ctl_host, pl->adj_ctl, sizeof(SolveCtl) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    for (int b = 0; b < B; ++b) all = all && pl->adj_ctl_host[b].done;
    if (all) break;
    chunk = std::min(2 * chunk, 16);
  }
  // gather each element's returned multipliers, then dL/ddelta = S mu (multiplier A (1 - beta/kbar), k = 0 -> 0)
  for (int b = 0; b < B; ++b) {
    const SolveCtl& C = pl->adj_ctl_host[b];
    if (!C.done) return fail(DGP_E_HIP, "adjoint control block %d undecided after max_iter", b);
    HIPCHK(hipMemcpyAsync(RES + (size_t)b * n3, MU + (size_t)C.result * bn + (size_t)b * n3, sizeof(double) * n3,
                          hipMemcpyDeviceToDevice, s));
  }
  TRY(fwd3<double>(pl, RES, pl->spec_u, B, nullptr, s));
  launch_p3<double>(n, SPEC_SOURCE, pl->spec_u, fs, 1, pl->spec6, fs, 2, B, cf, nullptr, nullptr, nullptr, nullptr, s);
  launch_p2<double>(n, pl->spec6, 1, B, +1, nullptr, s);
  launch_p1_inv<double>(n, pl->spec6, grad_delta, B, nullptr, s);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  int worst = DGP_OK;
  for (int b = 0; b < B; ++b) {
    const SolveCtl& C = pl->adj_ctl_host[b];
    const int st = C.status == 0 ? DGP_OK : DGP_NOT_CONVERGED;
    if (st != DGP_OK) worst = st;
    if (info) {
      std::memset(&info[b], 0, sizeof(dgp_info));
      info[b].status = st;
      info[b].iters = C.iters;
      info[b].passes = C.passes;
      info[b].passes_fp64 = C.passes;
      info[b].resid = C.resid;
      info[b].resid_min = C.resid_min;
    }
  }
  return worst;
}

// ------------------------------------------------------------------ live kernel timing
extern "C" int dgp_diagnostics(dgp_plan* pl, const dgp_params* p, const double* delta, const double* u_state,
                               double* nonelliptic, double* pc_over_pm, double* delta_gradc, int nbins, void* stream) {
  if (!pl || !u_state) return fail(DGP_E_INVALID, "plan and u_state are required");
  TRY(check_params(p));
  if ((pc_over_pm || delta_gradc) && (nbins < 1 || nbins > 128)) return fail(DGP_E_INVALID, "nbins must be in [1, 128]");
  if (pc_over_pm && !delta) return fail(DGP_E_INVALID, "P_c/P_m needs delta");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = pl->batch;
  if (nonelliptic) {
    TRY(ensure_adj(pl));
    TRY(hessians(pl, p, u_state, pl->adj, s));
    launch_nonelliptic(pl->n3, B, u_state, pl->adj, pl->mean_u, p->lambda, p->alpha, pl->adj_red, s);
    launch_pair_means(pl->adj_red, adjoint_groups(pl->n3), pl->n3, B, pl->vec, nullptr, s);
    HIPCHK(hipMemcpyAsync(pl->means_host, pl->vec, sizeof(double) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b) nonelliptic[b] = pl->means_host[b];
  }
  if (pc_over_pm) {   // Eq. cdef: c = alpha eta / (3 (eta - 1)) u
    std::vector<double> su, cu, sd, cd;
    TRY(power_impl(pl, p, u_state, 0, nbins, su, cu, s));
    TRY(power_impl(pl, p, delta, 0, nbins, sd, cd, s));
    const double coef = p->alpha * p->eta / (3.0 * (p->eta - 1.0));
    for (size_t i = 0; i < (size_t)B * nbins; ++i) {
      const double pu = cu[i] > 0 ? su[i] / cu[i] : 0.0, pd = cd[i] > 0 ? sd[i] / cd[i] : 0.0;
      pc_over_pm[i] = pd > 0 ? coef * coef * pu / pd : 0.0;
    }
  }
  if (delta_gradc) {   // Eq. DGradC: 4 pi k^5 P_C(k) at the bin centres kf (N/2)^((b + 1/2) / nbins)
    std::vector<double> sc, cc;
    TRY(power_impl(pl, p, u_state, 1, nbins, sc, cc, s));
    const double norm = std::pow(pl->box, 3) / (double(pl->n3) * double(pl->n3));
    const double kf = 2.0 * M_PI / pl->box;
    for (int b = 0; b < B; ++b)
      for (int i = 0; i < nbins; ++i) {
        const size_t j = (size_t)b * nbins + i;
        const double kc = kf * std::pow(pl->n / 2.0, (i + 0.5) / nbins);
        const double pk = cc[j] > 0 ? sc[j] / cc[j] * norm : 0.0;
        delta_gradc[j] = 4.0 * M_PI * std::pow(kc, 5) * pk;
      }
  }
  return DGP_OK;
}

extern "C" int dgp_solve_history(dgp_plan* pl, int b, double* resid, double* bad, int cap) {
  if (!pl || b < 0 || b >= pl->batch || cap < 0) return fail(DGP_E_INVALID, "bad plan, batch index or capacity");
  const SolveCtl& C = pl->ctl_host[b];   // as left by the last solve's final synchronisation
  int m = std::min(std::min(C.passes, kMaxHist), cap);
  for (int i = 0; i < m; ++i) {
    if (resid) resid[i] = C.hist[i];
    if (bad) bad[i] = C.hist_bad[i];
  }
  return m;
}

extern "C" int dgp_run(dgp_plan* pl, const dgp_params* p, void* pos, void* vel, int is_fp32, long long np,
                       double a_start, double dlna, int n_steps, double a_switch, double* u_state, dgp_info* info,
                       void* stream) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  TRY(check_params(p));
  if (n_steps < 0 || !(a_start > 0.0) || !std::isfinite(a_start) || !std::isfinite(dlna) || !std::isfinite(a_switch))
    return fail(DGP_E_INVALID, "need n_steps >= 0, a_start > 0 and finite dlna, a_switch");
  int worst = DGP_OK;
  bool solved = false;
  for (int k = 0; k < n_steps; ++k) {
    const double a = a_start * std::exp(k * dlna);
    dgp_params q;
    TRY(dgp_params_init(&q, p->omega_m0, a));
    q.lambda = p->lambda;
    q.w = p->w;
    q.omega_relax = p->omega_relax;
    q.tol = p->tol;
    q.max_iter = p->max_iter;
    q.nonlocal = p->nonlocal;
    q.check_every = p->check_every;
    q.spherical = p->spherical;
    const bool early = p->force_mode == DGP_FORCE_NLDGP && a < a_switch;
    q.force_mode = early ? DGP_FORCE_LDGP : p->force_mode;
    q.init = (q.force_mode == DGP_FORCE_NLDGP && solved) ? DGP_INIT_WARM : p->init;
    dgp_info one{};
    const int st = dgp_step(pl, &q, pos, vel, is_fp32, np, dlna, u_state, &one, stream);
    if (st < 0) return st;
    if (q.force_mode == DGP_FORCE_NLDGP) solved = true;
    if (info) info[k] = one;
    if (status_rank(st) > status_rank(worst)) worst = st;
  }
  return worst;
}

extern "C" int dgp_timing_enable(dgp_plan* pl, int on) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  timing_flush(pl);
  pl->timing = on != 0;
  for (int i = 0; i < DGP_T_NCLASS; ++i) {
    pl->t_ms[i] = 0.0;
    pl->t_cnt[i] = 0;
  }
  return DGP_OK;
}

extern "C" int dgp_timing_classes(dgp_plan* pl, unsigned int class_mask) {
  if (!pl) return fail(DGP_E_INVALID, "plan is NULL");
  pl->t_mask = class_mask;
  return DGP_OK;
}

extern "C" int dgp_timing_read(dgp_plan* pl, int cls, double* total_ms, long long* launches) {
  if (!pl || cls < 0 || cls >= DGP_T_NCLASS) return fail(DGP_E_INVALID, "bad timing class");
  timing_flush(pl);
  if (total_ms) *total_ms = pl->t_ms[cls];
  if (launches) *launches = pl->t_cnt[cls];
  return DGP_OK;
}

// Internal declarations shared by the libdgp translation units (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "fft_engine.h"

namespace dgp {

// Spectral multiplier modes of the axis-2 pass (forward FFT of each input row,
// per-mode combination, inverse FFT of each output row).
enum SpecMode : int {
  SPEC_SOURCE = 1,    // delta(k) -> S(k) = A(1 - beta/kbar) delta, u_lin(k) = S/(alpha - gamma/kbar)
  SPEC_CFIELD = 2,    // u(k) -> C(k) = -u/kbar^2
  SPEC_FORCES = 3,    // delta(k)[, u(k)] -> phi(k) (slot 0) and g_2 = -(c/H0)^2 i k_2 phi(k) (slot 2)
  SPEC_POWER = 4,     // f(k) -> per-bin sums of |f|^2 (no outputs); optional 1/kbar^2 weight
  SPEC_POWER_GRAD = 5,// f(k) -> per-bin coefficient * f(k) [* 1/kbar^4]
  SPEC_ADJ_COMBINE3 = 6,// the three group sums of launch_p2_adj_split -> one combined spectrum
  SPEC_COPY = 7,      // identity (plain forward+inverse round trip, for tests)
  SPEC_FWD_ONLY = 8,  // forward axis-2 transform only (spectrum export)
  SPEC_INV_ONLY = 9,  // inverse axis-2 transform only, times 1/N^3 (spectrum import)
  SPEC_HSPLIT = 10,   // u(k) -> C' = u/|n|^2, i n2 C' and -u/kbar into slots 0, 3 and 5 of the six
                      // relaxation fields (h00, h11, h01, h02, h12 and the nonlocal term after the
                      // axis-1 pass launch_p2_split, which applies the axis-1 and axis-0 factors)
};

enum ForceMode : int { FORCE_NLDGP = 0, FORCE_LDGP = 1, FORCE_GRH = 2, FORCE_GR = 3 };

// Coefficients consumed by the spectral kernels (all double; fp32 kernels round at use).
struct SpecCoef {
  double kf;        // 2 pi / L
  double kappa;     // c/(aH) [Mpc/h]
  double A, beta, alpha, gamma;   // effective (nonlocal terms zeroed when disabled)
  double om15;      // (3/2)(eta-1)/eta
  double inv2eta;   // 1/(2 eta)
  double c2;        // coefficient of sqrt(-lap) C in the modified Poisson equation (0 if nonlocal off)
  double inv_eta_nl;// 1/eta in the sqrt(-lap) phi term (0 if nonlocal off)
  double force_scale;  // (c/H0)^2
  double inv_n3;    // 1/N^3 (inverse-transform normalisation, folded into the multiplier)
  double lam2;      // 2 lam (adjoint combine)
  int force_mode;   // ForceMode
  int power_c;      // POWER/POWER_GRAD: weight |f|^2 by 1/kbar^4 (spectrum of C from u)
  int nbins;        // POWER: number of bins
};

// Per-batch-element control block of the relaxation (device memory).
constexpr int kMaxHist = 256;
constexpr int kStatusInvalid = 3;
struct SolveCtl {
  int done;         // 1 once the returned iterate is decided
  int status;       // 0 ok, 1 not converged (max_iter), 2 stopped at min residual with bad points,
                    // kStatusInvalid: non-finite input or iterate (no valid output)
  int iters;        // updates applied to the current iterate
  int cur;          // buffer index holding u^(iters)
  int out;          // buffer the next update writes
  int best;         // buffer index of the minimum-residual iterate
  int result;       // buffer index of the returned iterate
  int bad_seen;
  int passes;       // residual evaluations executed
  int last_bad;     // bad points of the last update
  int final_bad;    // bad points of the update computed by the pass that met tol (-1: none)
  int iters1;       // precision form: updates and passes of the float32 phase (0 otherwise)
  int passes1;
  int phase1_done;  // the float32 phase had decided before the float64 phase started
  double eps;       // <|S|>
  double resid;     // r of the returned iterate
  double resid_min;
  double bad_frac;
  double mean_u;    // <u> of the current iterate (from its k = 0 mode)
  double hist[kMaxHist];       // r of the iterate evaluated by pass n
  double hist_bad[kMaxHist];   // bad-point fraction of the update computed by pass n
};

struct SolveCfg {
  double lam, w, alpha, gamma, omega, tol;
  int max_iter;
  int fixed;        // 1: exactly max_iter updates, the last iterate returned (no minimum-residual stop)
  int n;            // mesh size
  int batch;
};

// Real-FFT tile geometry: complex "pair columns" per workgroup for the axis-0 passes.
template <typename T, int N, int R>
struct AxisTile {
  static constexpr int kT = N / R;                                       // threads per transform
  static constexpr int kBase = 128 / (2 * int(sizeof(T)) * 2);           // pairs for 128-B complex rows
  static constexpr int kWant = (64 / kT > kBase) ? 64 / kT : kBase;
  static constexpr int kTP = (kWant > N / 2) ? N / 2 : kWant;            // pairs per workgroup
  static constexpr int kThreads = kTP * kT;
};

// Column tile of the axis-1 pass.
template <typename T, int N, int R>
struct ColTile {
  static constexpr int kT = N / R;
  static constexpr int kBase = 128 / int(sizeof(cx<T>));
  static constexpr int kWant0 = (64 / kT > kBase) ? 64 / kT : kBase;
  // up to 512 threads, or 1024 when that is what a 128-byte row segment takes (64-byte segments
  // would split cache lines between workgroups on different XCDs)
  static constexpr int kMaxThreads = (kBase * kT > 512 && kBase * kT <= 1024) ? kBase * kT : 512;
  static constexpr int kCap = (kMaxThreads / kT > 1) ? kMaxThreads / kT : 1;
  static constexpr int kWant = (kWant0 > kCap) ? kCap : kWant0;
  static constexpr int kTY = (kWant > N) ? N : kWant;
  static constexpr int kThreads = kTY * kT;
};

// Row tile of the axis-2 pass.
template <int N, int R>
struct RowTile {
  static constexpr int kT = N / R;
  static constexpr int kRW = (256 / kT > 1) ? 256 / kT : 1;
  static constexpr int kThreads = kRW * kT;
};

// XCD-aware workgroup order.  Workgroups are dispatched round-robin over the 8 XCDs of an
// MI355X by their linear index, and each XCD has its own L2.  Logical tiles are assigned so
// that one XCD works through a contiguous range of them, so neighbouring tiles that share
// 128-byte lines are fetched through the same L2.  The map is a bijection of the grid, so the
// result does not depend on how the hardware actually dispatches.
// 1D form for particle chunks: consecutive chunks (neighbouring Lagrangian blocks, whose
// mesh boxes overlap) run on the same XCD and share its L2.
__device__ __forceinline__ long long xcd_chunk() {
  const long long g = gridDim.x, i = blockIdx.x;
  return ((g & 7) == 0) ? (i & 7) * (g >> 3) + (i >> 3) : i;
}

__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int gx = gridDim.x, g = gridDim.x * gridDim.y;
  const int i = blockIdx.y * gx + blockIdx.x;
  const int l = ((g & 7) == 0) ? (i & 7) * (g >> 3) + (i >> 3) : i;
  bx = l % gx;
  by = l / gx;
}

// ------------------------------------------------------------------ launchers
// All launchers are asynchronous on `stream`; `done` (may be null) is a per-batch
// flag array: work for a batch element whose flag is set is skipped.

template <typename T>
void launch_p1_fwd(int n, const T* in, cx<T>* out, int batch, const SolveCtl* ctl, hipStream_t s);
// float32 axis-0 forward pass of a float64 real field (rounded on load)
void launch_p1_fwd_from64(int n, const double* in, cx<float>* out, int batch, const SolveCtl* ctl, hipStream_t s);
template <typename T>
void launch_p1_inv(int n, const cx<T>* in, T* out, int batch, const SolveCtl* ctl, hipStream_t s,
                   float* out32 = nullptr);   // out32: optional float32 copy of out
// nf fields, each [batch][H][N][N]; DIR -1 forward, +1 inverse
template <typename T>
void launch_p2(int n, cx<T>* data, int nf, int batch, int dir, const SolveCtl* ctl, hipStream_t s);
// axis-1 inverse pass of the split Hessian: slots 0, 3, 5 of the six fields (fstride apart, each
// [batch][H][N][N]) -> all six, with the axis-1 and axis-0 factors (slot 0 -> 0: n0^2, 1: n1^2,
// 2: n0 n1; slot 3 -> 3: -i n0, 4: -i n1; slot 5 -> 5: 1; a factor odd in n_d is 0 at the Nyquist
// index of d)
template <typename T>
void launch_p2_split(int n, cx<T>* data, size_t fstride, int batch, const SolveCtl* ctl, hipStream_t s);
// forward axis-1 pass of the adjoint's combine: six product spectra (axis-0 transformed) -> the
// three group sums in slots 0, 3, 5, with the axis-1 and axis-0 factors and the 2 lam weights
void launch_p2_adj_split(int n, cx<double>* data, size_t fstride, int batch, double lam2, const SolveCtl* ctl,
                         hipStream_t s);
// axis-1 inverse pass of the force mesh: phi (slot 0) and g2 (slot 2) from the axis-2 pass ->
// g0, g1, g2 in slots 0..2 and phi in slot 3 when with_phi; fk = (c/H0)^2 kf
template <typename T>
void launch_p2_force_split(int n, cx<T>* data, size_t fstride, int batch, int with_phi, double fk, hipStream_t s);
// axis-2 pass: nin input arrays (each [batch][H][N][N]) -> nout output arrays
template <typename T>
void launch_p3(int n, SpecMode mode, const cx<T>* in, size_t in_stride, int nin, cx<T>* out,
               size_t out_stride, int nout, int batch, const SpecCoef& coef, const double* bin_coef,
               double* bin_partial, double* mean_out, const SolveCtl* ctl, hipStream_t s);
int p3_row_groups(int n);   // workgroups per batch element of the axis-2 pass (for POWER partials)

// fused relaxation pass (inverse axis-0 of 6 spectra + pointwise update + forward axis-0);
// ev0/ev1 (may be null): timing events recorded by the kernel's dispatch at its start and end
template <typename T>
void launch_relax(int n, const cx<T>* spec6, T* ubuf, const T* s_field, cx<T>* spec_u, double* partial,
                  const double* mean_u, int batch, const SolveCfg& cfg, const SolveCtl* ctl, hipStream_t s,
                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int relax_groups(int n, int elem_bytes);   // workgroups per batch element of the fused pass

void launch_finalize(const double* partial, int groups, SolveCtl* ctl, const SolveCfg& cfg,
                     int* n_active, hipStream_t s);

// reductions: per-batch mean of |x| and mean of x (double results)
template <typename T>
void launch_absmean(size_t n3, const T* x, int batch, double* scratch, double* abs_mean, double* mean,
                    hipStream_t s);
size_t absmean_scratch_doubles(size_t n3, int batch);
// control blocks: eps from abs_mean[b], buffer roles reset
void launch_ctl_init(SolveCtl* ctl, const double* eps, int batch, hipStream_t s);
// spherical approximation (Eqs. FullDGP2sph, SphPoi): u = the first w = 1/3 update from u = 0,
// u = 2 S / (alpha + sqrt(alpha^2 + (8/3) lam S)) (vertex where the discriminant is negative),
// for [batch][n3] S into u; then the control blocks record a decided one-update solve
// (per-workgroup bad counts go through `partial`, which must hold batch x 4096 x 2 doubles)
void launch_spherical(size_t n3, int batch, const double* S, double* u, double alpha, double lam, double* partial,
                      SolveCtl* ctl, const double* eps, hipStream_t s);
// end of the float32 phase: per element, the warm start for float64 (the update of the
// pass that met the switch tolerance unless it met bad points, else the checked iterate;
// the latest iterate if the phase was still running) converted into dst[B][n3], then the
// control re-initialised for the float64 phase with the float32 counts kept
void launch_handoff(SolveCtl* ctl, const float* U32, int batch, size_t n3, double* dst, hipStream_t s);
// the returned iterate of every element, as float64, into dst[B][n3], and its mean into
// mean[B] (scratch: absmean_scratch_doubles(n3, batch) doubles)
template <typename T>
void launch_take_result(const SolveCtl* ctl, const T* U, int batch, size_t n3, double* dst, double* scratch,
                        double* mean, hipStream_t s);

// per-batch means of the two columns of [batch][groups][2] partial sums
void launch_pair_means(const double* part, int groups, size_t n3, int batch, double* out0, double* out1,
                       hipStream_t s);

// adjoint (transposed relaxation) pointwise kernels
int adjoint_groups(size_t n3);
// mu = g / D, with per-workgroup counts of points where D <= 0 (or not finite) and of non-finite g
// in part (adjoint_groups(n3) x batch x 2 doubles)
void launch_adj_init(size_t n3, int batch, const double* g, const double* u, double* mu, double dscale, double alpha,
                     double* part, hipStream_t s);
// coefficients of the transposed update: 2 lam, w, alpha and D's slope 2 (1-w) lam
struct AdjCoef {
  double lam2, w, alpha, dscale;
};
// workgroups per batch element of launch_adj_step (its partial sums: [batch][groups][3])
int adj_step_groups(int n);
// one fused adjoint iteration step (see adjoint.hip); mubuf holds three multiplier buffers
// mu_stride apart, indexed by ctl[b].cur / ctl[b].out; spec6: six half spectra spec_stride apart
void launch_adj_step(int n, bool update, const cx<double>* qspec, double* mubuf, size_t mu_stride, const double* u,
                     const double* h5, const double* g, const double* mean_u, const double* mean_h22mu,
                     cx<double>* spec6, size_t spec_stride, double* part, const AdjCoef& k, const SolveCtl* ctl,
                     int batch, hipStream_t s);
// <h22 mu'> per element and, with eval, the convergence decision of the step just run
void launch_adj_finalize(bool eval, const double* part, int groups, SolveCtl* ctl, double* mean_h22mu, size_t n3,
                         double tol, int max_iter, int batch, hipStream_t s);

// counts of points where Eq. FullDGP2 is not elliptic (Appendix), per workgroup into part
// (adjoint_groups(n3) x batch x 2 doubles); launch_pair_means turns them into fractions
void launch_nonelliptic(size_t n3, int batch, const double* u, const double* h5, const double* mean_u, double lam,
                        double alpha, double* part, hipStream_t s);

// PM kernels.  `bad` (device int) is raised when a particle coordinate is not finite.
void launch_deposit(int n, double box, const void* pos, int pos_fp32, long long np, long long* grid, int* bad,
                    hipStream_t s);
// delta = Q 2^-40 N^3/np - 1 (NaN everywhere when *bad is set)
// delta from the fixed-point counts; mean_q (optional, device): the mean of the counts, whose delta
// value is subtracted in the same pass (mean removal)
void launch_counts_to_delta(int n, const long long* grid, long long np, double* delta, const int* bad, hipStream_t s,
                            const double* mean_q = nullptr);
// zero `words` 8-byte words (a fill kernel: no memset node in captured streams)
void launch_fill_zero(void* p, size_t words, hipStream_t s);
void launch_zero_flag(int* bad, hipStream_t s);
// out[k][p] = CIC interpolation of component k of mesh [nc][n3] (nc in 1..3), float64 (mesh_fp32 = 0)
// or float32 (1) mesh
void launch_interp(int n, double box, const void* mesh, int mesh_fp32, int nc, const void* pos, int pos_fp32,
                   long long np, double* out, hipStream_t s);
void launch_interp_kick_drift(int n, double box, const void* mesh3, int mesh_fp32, void* pos, void* vel, int fp32,
                              long long np, double kick, double drift, hipStream_t s);
void launch_deposit_backward(int n, double box, const void* pos, int pos_fp32, long long np,
                             const double* grad_delta, double* grad_pos, hipStream_t s);
// adjoint of launch_interp for dL/dout = g [nc][np]: grad_pos [3][np] (optional) and grad_mesh [nc][n3]
// (optional, deterministic fixed-point sums); grid: n3 int64 scratch, st: 3 words of scratch
void launch_interp_backward(int n, double box, const double* mesh, int nc, const void* pos, int pos_fp32, long long np,
                            const double* g, double* grad_pos, double* grad_mesh, long long* grid,
                            unsigned long long* st, int* bad, hipStream_t s);
template <typename T>
void launch_convert(size_t count, const void* in, int in_fp32, T* out, hipStream_t s);

// per-device address and size (doubles) of the allocation-free deposit's static scratch;
// 0 on success, -1 when the HIP runtime fails, -2 for a device index beyond the table
int noalloc_scratch(double** ptr, size_t* capacity);

}  // namespace dgp

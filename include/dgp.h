/*
 * libdgp -- MI355X (gfx950) field solve of the DGP brane-bending mode inside a
 * particle-mesh step.  C ABI: plain pointers and sizes only.
 *
 * Method: Chan & Scoccimarro, "Large-Scale Structure in Brane-Induced Gravity II.
 * Numerical Simulations".  The field equations are Eq. FullDGP1 (modified Poisson
 * equation for the Newtonian potential phi) and Eq. FullDGP2 (fully nonlinear
 * equation for the brane-bending mode C); the solver is the FFT-relaxation of
 * Sec. III B with the w-split of Sec. III C; the PM step is Sec. III A.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers.  Every array argument is a pointer to device memory of
 *    the current HIP device (the device the plan was created on), except the
 *    `dgp_params` / `dgp_info` structs, which live in host memory.  All arrays
 *    belong to the caller; the library never frees them.
 *  - Layouts.  A mesh field is float64 in C order, [batch][N][N][N], the last
 *    index fastest; mesh axis d is particle coordinate d.  Particles are SoA,
 *    [3][np] (x of all particles, then y, then z), float32 or float64 as flagged.
 *    Mesh node j sits at x = j * L / N; positions lie in [0, L).
 *  - Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued asynchronously; entry points that iterate (solve, step, backward)
 *    synchronise the stream to read the convergence scalars and return when their
 *    outputs are complete.  One plan must not be used by two streams at once.
 *  - Errors.  Functions return a dgp_status.  Negative values are errors: no
 *    output is valid and dgp_last_error() (per calling thread) describes it.
 *    Positive values are warnings: outputs are valid.  Nothing aborts or exits.
 */
#ifndef DGP_H
#define DGP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGP_API_VERSION 1

typedef struct dgp_plan dgp_plan;

typedef enum {
  DGP_OK = 0,
  DGP_NOT_CONVERGED = 1,   /* max_iter reached; the minimum-residual iterate is returned */
  DGP_BAD_POINTS = 2,      /* bad points occurred and the residual stopped decreasing; the
                              minimum-residual iterate is returned (Sec. III C, Fig. 4 text) */
  DGP_E_INVALID = -1,      /* bad argument: null pointer, unsupported N, non-finite or out-of-range parameter */
  DGP_E_NOMEM = -2,        /* device allocation failed */
  DGP_E_HIP = -3,          /* a HIP runtime call failed */
  DGP_E_UNSUPPORTED = -4   /* valid request this plan cannot serve (e.g. batch > 1 for a PM step) */
} dgp_status;

typedef enum { DGP_FP64 = 0, DGP_FP32 = 1 } dgp_precision;
/* DGP_FP32: FFTs, spectral multipliers and stored fields in float32; residual,
 * discriminant, root selection, k = 0 / mean handling and reductions in float64;
 * the solve finishes with float64 passes (polish) so the returned iterate meets
 * the same float64 normalised-residual tolerance as DGP_FP64. */

typedef enum { DGP_INIT_LINEAR = 0, DGP_INIT_ZERO = 1, DGP_INIT_WARM = 2 } dgp_init;
/* Force laws (Sec. IV): the full DGP equations (nlDGP), their linearised form (lDGP, Eq. LinearDGP), GR
 * with the DGP expansion history (GRH, Eq. GRPoisson) and standard gravity with its own expansion
 * history (GR: flat LCDM with the same Omega_m0 in the Poisson coefficient and in the kick-drift). */
typedef enum { DGP_FORCE_NLDGP = 0, DGP_FORCE_LDGP = 1, DGP_FORCE_GRH = 2, DGP_FORCE_GR = 3 } dgp_force_mode;

/* Parameters of one field solve / PM step.  dgp_params_init fills every field
 * from (Omega_m0, a); callers may then override any of them. */
typedef struct {
  double omega_m0;     /* present matter density; the paper uses 0.27 (Sec. III A) */
  double a;            /* scale factor */
  /* background and coefficients of Eqs. FullDGP1/FullDGP2 (Sec. II) */
  double E;            /* H/H0 from Eq. DGPFriedmann with r_c H0 = 1/(1 - Omega_m0) */
  double eta;          /* r_c H */
  double alpha;        /* 3 (2 eta^2 - 2 eta + 1) / (eta (2 eta - 1)) */
  double beta;         /* (2 eta^2 - 2 eta - 1) / (eta (2 eta - 1)) */
  double A;            /* 3 (eta - 1) / eta, source coefficient of Eq. FullDGP2 */
  double gamma;        /* 3 beta (eta - 1) / (2 eta - 1), sqrt(-lap) C coefficient of Eq. FullDGP2 */
  double c2;           /* (3 eta^2 - 5 eta + 1) / (2 eta^2 (2 eta - 1)), sqrt(-lap) C coefficient of Eq. FullDGP1 */
  double kappa;        /* c / (a H) in Mpc/h: kbar = kappa |k| */
  /* solver */
  double lambda;       /* coefficient of the two quadratic terms of Eq. FullDGP2 (1 = paper); > 0 */
  double w;            /* split of Eq. FullDGP2wpara, in [0, 1); paper: 1/3 */
  double omega_relax;  /* damping u <- (1-omega) u + omega u_new, in (0, 1]; paper: 1 */
  double tol;          /* stop when <|R|>/eps <= tol (Eq. normres); paper: 0.01.  tol < 0: no stopping
                          test, exactly max_iter updates and the last iterate returned with DGP_OK
                          (reproducible update counts, e.g. for finite differences); the adjoint
                          takes tol < 0 as "run max_iter iterations" (DGP_NOT_CONVERGED) */
  int max_iter;        /* maximum number of relaxation updates (>= 0) */
  int init;            /* dgp_init: starting iterate */
  int nonlocal;        /* 1 keeps the sqrt(-lap) and lap^{-1/2} terms (paper), 0 drops them */
  int force_mode;      /* dgp_force_mode used by dgp_pm_forces / dgp_step */
  int check_every;     /* passes between host reads of the convergence flags (>= 1; default 4) */
  int spherical;       /* 1: spherical approximation (Eqs. FullDGP2sph, SphPoi) instead of the full
                          solve: u is the first w = 1/3 update from u = 0, a local function of the
                          source (info: iters 1, passes 0, resid -1 = not evaluated); 0: full solve */
} dgp_params;

/* Per-batch-element report of a solve (host memory, one per batch element). */
typedef struct {
  int status;          /* dgp_status of this element */
  int iters;           /* relaxation updates applied to the returned iterate */
  int passes;          /* residual evaluations executed (float64 + float32) */
  int passes_fp64;     /* of which in float64 */
  double resid;        /* <|R|>/eps of the returned iterate (float64 evaluation) */
  double resid_min;    /* smallest residual seen */
  double eps;          /* <|S|>, S = A (1 - beta lap^{-1/2}) delta (Eq. normres) */
  double bad_fraction; /* fraction of bad points in the last update (Sec. III C) */
  double mean_u;       /* <u> of the returned iterate (diagnostic) */
  double ms_total;     /* wall time of the call on the stream, ms */
} dgp_info;

/* Fill *p from (omega_m0, a): background (Eq. DGPFriedmann), coefficients (Sec. II),
 * lambda = 1, w = 1/3, omega_relax = 1, tol = 0.01, max_iter = 100,
 * init = DGP_INIT_LINEAR, nonlocal = 1, force_mode = DGP_FORCE_NLDGP, check_every = 4.
 * Host only.  DGP_E_INVALID if p is NULL, omega_m0 not in (0, 1) or a <= 0. */
int dgp_params_init(dgp_params* p, double omega_m0, double a);

/* Create a plan for an N^3 periodic mesh of side `box` [Mpc/h], `batch` independent
 * fields, precision dgp_precision.  N is a power of two in [8, 512].  The plan
 * allocates its device workspace on the current device (hipMalloc) and frees it
 * in dgp_plan_destroy.  DGP_E_INVALID on bad sizes, DGP_E_NOMEM on allocation failure. */
int dgp_plan_create(dgp_plan** plan, int n, int batch, double box, int precision);
/* Device bytes a plan of these sizes uses: its buffers, each rounded up to 256 bytes, as
 * dgp_plan_create allocates them (with_adjoint = 0), plus the buffers of the implicit adjoint
 * that the first dgp_solve_field_backward or dgp_diagnostics call adds (with_adjoint != 0).
 * A host-side computation (no device call).  Returns 0 for invalid sizes.  The per-device
 * twiddle tables (shared by every plan, a few tens of KB) are not included. */
size_t dgp_workspace_bytes(int n, int batch, int precision, int with_adjoint);
/* dgp_plan_create on a caller-owned device workspace: every device buffer of the plan is carved
 * from `workspace` (device memory on the current device, 256-byte aligned, at least
 * dgp_workspace_bytes(n, batch, precision, 0) bytes; the caller keeps ownership and must keep
 * it alive until dgp_plan_destroy).  With at least dgp_workspace_bytes(..., 1) bytes the
 * adjoint's buffers come from it too; otherwise the first call that needs them returns
 * DGP_E_INVALID.  The plan still allocates its small pinned host buffers and its events.
 * DGP_E_INVALID on bad sizes, a NULL or misaligned workspace, or one that is too small. */
int dgp_plan_create_ws(dgp_plan** plan, int n, int batch, double box, int precision, void* workspace,
                       size_t workspace_bytes);
int dgp_plan_destroy(dgp_plan* plan);
/* Device bytes held by the plan (256-byte units; equal to dgp_workspace_bytes for the same
 * sizes, with_adjoint once the adjoint's buffers exist). */
size_t dgp_plan_device_bytes(const dgp_plan* plan);

/* CIC mass assignment (Sec. III A, Eq. CIC), deterministic.
 * pos [3][np] (float32 if pos_is_fp32 else float64), np >= 1, batch-1 plans only.
 * grid_fixed [N^3] int64 (optional, may be NULL): sum over particles of
 *   rint(W * 2^40) with W = (w_x w_y) w_z, per-axis weights (1 - f, f) in float64;
 *   identical bits for any particle order.
 * delta [N^3] float64 (optional): Q 2^-40 N^3/np - 1 with its mean removed.
 * Positions must be finite; the call does not synchronise, so a non-finite coordinate is not
 * reported here: it makes every cell of delta NaN (grid_fixed is then unspecified), which a
 * following dgp_solve_field rejects with DGP_E_INVALID. */
int dgp_deposit(dgp_plan* plan, const void* pos, int pos_is_fp32, long long np, long long* grid_fixed,
                double* delta, void* stream);

/* dgp_deposit without a plan and without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arithmetic and outputs (the same bits) as dgp_deposit on an N^3 mesh of side `box`;
 * grid_fixed [N^3] int64 and delta [N^3] float64 are both required, N a power of two in [8, 512].
 * The mean removal's partial sums, the mean and the non-finite flag live in a 32 KiB static
 * device array that each GPU holds until the process ends; all calls on one device share it, so
 * calls that overlap on one device race.  Enqueues fill kernels (no memset nodes) and allocates
 * nothing.  Asynchronous; a non-finite position makes delta NaN, as for dgp_deposit. */
int dgp_deposit_noalloc(int n, double box, const void* pos, int pos_is_fp32, long long np, long long* grid_fixed,
                        double* delta, void* stream);

/* Field solve of Eq. FullDGP2 by FFT-relaxation (Sec. III B, Eq. FFTrelax; w-split of
 * Sec. III C, Eqs. nabla^2Cwpara and Bwpara).
 * delta   [batch][N^3] float64 density contrast (its mean is ignored: k = 0 multipliers are 0).
 *         A uniform delta has S = 0 and eps = 0: its solution u = 0 is returned with r = 0.
 * u_state [batch][N^3] float64, u = lapbar C.  Read as the starting iterate when
 *         p->init == DGP_INIT_WARM (warm start from the previous step, Sec. III B);
 *         always overwritten with the returned iterate.
 * c_out   [batch][N^3] float64, optional: C = lapbar^{-1} u (C(k) = -u(k)/kbar^2).
 * info    host array of batch dgp_info, optional.
 * Returns the worst status over the batch.  DGP_E_INVALID (no output valid) when an element's
 * delta or warm-start field is not finite (its info status is DGP_E_INVALID too). */
int dgp_solve_field(dgp_plan* plan, const dgp_params* p, const double* delta, double* u_state, double* c_out,
                    dgp_info* info, void* stream);

/* Forces on particles from the modified Poisson equation (Eq. FullDGP1; lDGP: its linear
 * form; GRH: Eq. GRPoisson with the same background; GR: Eq. GRPoisson with the flat LCDM
 * background, kbar = c k/(a H_LCDM)) and the spectral gradient i k phi
 * (Sec. III A), interpolated with the CIC weights.
 * delta [N^3], u_state [N^3] (the solved u; unused for lDGP/GRH), pos [3][np].
 * force [3][np] float64 output: g = -(c/H0)^2 grad phi at each particle (H0 = 1, Mpc/h).
 * phi_n [N^3] float64, optional: phi on the mesh (units of c^2).  Batch-1 plans only. */
int dgp_pm_forces(dgp_plan* plan, const dgp_params* p, const double* delta, const double* u_state, const void* pos,
                  int pos_is_fp32, long long np, double* force, double* phi_n, void* stream);

/* One PM step at scale factor p->a: deposit, field solve (u_state in/out, started as
 * p->init says), forces, CIC interpolation and a leapfrog step in ln a:
 *   vel += dlna * g / E(a);  pos += dlna * vel / (a_h^2 E(a_h)), a_h = a e^{dlna/2}
 * (E of the DGP background, or of flat LCDM for DGP_FORCE_GR);
 * positions wrapped into [0, L).  vel holds p = a^2 dx/dt at half steps.
 * pos, vel [3][np] (float32 if is_fp32), updated in place.
 * DGP_E_INVALID (outputs not valid) when a position is not finite. */
int dgp_step(dgp_plan* plan, const dgp_params* p, void* pos, void* vel, int is_fp32, long long np, double dlna,
             double* u_state, dgp_info* info, void* stream);

/* Implicit adjoint of the converged solve: given g = dL/du at u* (the output of
 * dgp_solve_field with the same delta and params), solves J^T mu = g by the transposed
 * relaxation and returns dL/ddelta = S^T mu, S = A (1 - beta/kbar) (k = 0 -> 0).
 * delta, u_star, grad_u, grad_delta: [batch][N^3] float64.  Uses p->tol as the relative
 * tolerance on <|J^T mu - g|>/<|g|> and p->max_iter; at max_iter the minimum-residual mu is
 * used and DGP_NOT_CONVERGED returned.  DGP_E_INVALID when u_star has points with
 * D = 2 (1-w) lam u + alpha <= 1e-12 alpha (the vertex value of a bad point, up to rounding: the
 * solve did not converge there and the transposed relaxation would divide by about zero) or
 * non-finite values, or when
 * grad_u is not finite.  Convergence is decided on the device; the call synchronises the stream
 * between chunks of 4, 8, then 16 transposed-relaxation iterations and returns when grad_delta
 * is complete. */
int dgp_solve_field_backward(dgp_plan* plan, const dgp_params* p, const double* delta, const double* u_star,
                             const double* grad_u, double* grad_delta, dgp_info* info, void* stream);

/* Adjoint of the CIC deposit with respect to positions (unquantised weights):
 * grad_pos [3][np] = (N^3/np) sum_c grad_delta[c] dW_c/dx.  Batch-1 plans only. */
int dgp_deposit_backward(dgp_plan* plan, const void* pos, int pos_is_fp32, long long np, const double* grad_delta,
                         double* grad_pos, void* stream);

/* CIC interpolation of a caller mesh to particles (Sec. III A: the force is interpolated with
 * the assignment function of the deposit, Eq. CIC): out[m][p] = sum_c W_c(x_p) mesh[m][c],
 * W_c = w_x w_y w_z with per-axis weights (1 - f, f).  mesh [ncomp][N^3] float64, ncomp in [1, 3];
 * pos [3][np] (float32 if pos_is_fp32); out [ncomp][np] float64.  Batch-1 plans; asynchronous. */
int dgp_interp(dgp_plan* plan, const double* mesh, int ncomp, const void* pos, int pos_is_fp32, long long np,
               double* out, void* stream);

/* Adjoint of dgp_interp for grad_out = dL/dout [ncomp][np] (float64):
 * grad_pos [3][np] (optional): dL/dx_p = sum_m grad_out[m][p] sum_c mesh[m][c] dW_c/dx_p, with
 *   dw/dx = -N/L for the lower node and +N/L for the upper one (mesh is required for it);
 * grad_mesh [ncomp][N^3] (optional): dL/dmesh[m][c] = sum_p grad_out[m][p] W_c(x_p), the transposed
 *   scatter, summed in 64-bit fixed point (terms rounded to a multiple of 2^-e, e set per call from
 *   max|grad_out| and the largest cell mass so no sum overflows): the same bits in any particle order.
 * Uses the plan's deposit workspace (its int64 grid is overwritten).  Asynchronous; a non-finite
 * position or grad_out value makes grad_mesh NaN.  DGP_E_INVALID when both outputs are NULL or
 * grad_pos is requested without mesh. */
int dgp_interp_backward(dgp_plan* plan, const double* mesh, int ncomp, const void* pos, int pos_is_fp32,
                        long long np, const double* grad_out, double* grad_pos, double* grad_mesh, void* stream);

/* Binned power spectrum of a mesh field ([batch][N^3]), or, with of_c = 1, of
 * C = lapbar^{-1} u for a field u.  nbins logarithmic bins between 2 pi/L and the
 * Nyquist pi N/L (mode m in bin b when T_b <= |m|^2 < T_{b+1}, T_b = ceil((N/2)^(2b/nbins))),
 * P_b = (L^3/N^6) <|F(k)|^2>.  pk [batch][nbins] and counts [nbins] (optional, mode
 * multiplicities) are HOST arrays; the call synchronises the stream.  nbins in [1, 128]. */
int dgp_power_spectrum(dgp_plan* plan, const dgp_params* p, const double* field, int of_c, int nbins, double* pk,
                       double* counts, void* stream);

/* Gradient of sum_b grad_pk[b] P_b with respect to the field.  grad_pk: HOST array
 * [batch][nbins]; field, grad_field: device [batch][N^3]. */
int dgp_power_spectrum_backward(dgp_plan* plan, const dgp_params* p, const double* field, int of_c, int nbins,
                                const double* grad_pk, double* grad_field, void* stream);

/* 3D real FFT of [batch][N^3] float64 (forward, unnormalised) into the plan's half
 * spectrum layout [batch][N/2+1][N][N] complex (interleaved re, im; half axis = axis 0),
 * and its inverse (carries 1/N^3).  For tests of the transform itself. */
int dgp_fft_forward(dgp_plan* plan, const double* field, double* spectrum, void* stream);
int dgp_fft_inverse(dgp_plan* plan, const double* spectrum, double* field, void* stream);

/* Live kernel timing.  When enabled, the plan brackets the launches of each class
 * below with HIP events on the caller's stream and accumulates their elapsed times
 * once the stream has been synchronised (every solve / step synchronises before
 * returning).  Enabling resets the counters.  Classes with the DGP_T_FP32_OFFSET
 * added are the float32 launches of the precision form. */
enum {
  DGP_T_AXIS1_FWD = 0,   /* forward axis-1 pass of the iterate's spectrum, per relaxation pass */
  DGP_T_FANOUT = 1,      /* axis-2 pass: forward FFT, 3 spectral multipliers, 3 inverse FFTs */
  DGP_T_AXIS1_INV = 2,   /* inverse axis-1 pass: 3 spectra in, 6 out (axis-1 factors) */
  DGP_T_RELAX = 3,       /* fused axis-0 inverse of 6 spectra + pointwise update + axis-0 forward */
  DGP_T_FINALIZE = 4,    /* residual reduction and stopping rules */
  DGP_T_SETUP = 5,       /* source S, eps and linear guess from delta */
  DGP_T_DEPOSIT = 6,     /* CIC deposit and density contrast */
  DGP_T_FORCES = 7,      /* modified Poisson + gradient: force mesh */
  DGP_T_INTERP_KICK = 8, /* CIC interpolation fused with the leapfrog update */
  DGP_T_FP32_OFFSET = 16,
  DGP_T_NCLASS = 32
};
int dgp_timing_enable(dgp_plan* plan, int on);
/* Restrict timing to the classes whose bits are set in class_mask (bit c for class c;
 * all classes by default).  Each timed launch adds two event records to the stream, so a
 * run that reports whole-step throughput times only the class it needs. */
int dgp_timing_classes(dgp_plan* plan, unsigned int class_mask);
/* total_ms / launches (either may be NULL) of one class since the last enable. */
int dgp_timing_read(dgp_plan* plan, int cls, double* total_ms, long long* launches);

/* Multi-step PM run (Sec. III A time stepping, Sec. III D): n_steps leapfrog steps of dlna
 * starting at scale factor a_start.  Step k runs at a_k = a_start exp(k dlna) with the
 * background coefficients of params recomputed for a_k (the other fields of params are used
 * as given).  For params->force_mode = DGP_FORCE_NLDGP: while a_k < a_switch the force law is
 * the linearised DGP one (DGP_FORCE_LDGP, no field solve, as the paper does at early times); from
 * the first step with a_k >= a_switch on it is the full one, and every nonlinear solve after the
 * first starts from the previous step's field (warm start).  The other force modes (the lDGP,
 * GRH and GR comparison runs) use their law at every step and ignore a_switch.  pos, vel, u_state as for dgp_step; info: n_steps entries (or
 * NULL).  Returns the worst step status, or a negative error (the run stops at the first). */
int dgp_run(dgp_plan* plan, const dgp_params* params, void* pos, void* vel, int is_fp32, long long np,
            double a_start, double dlna, int n_steps, double a_switch, double* u_state, dgp_info* info,
            void* stream);

/* Diagnostics of a solved field u = lap C (host outputs; any output may be NULL):
 * nonelliptic[B]: fraction of mesh points where Eq. FullDGP2 is not elliptic, i.e. where the
 *   matrix of dF/d(h_ij), (2 lam u + alpha) I - 2 lam h, is not definite (Appendix, Eq.
 *   EllipticMatrix; Hessians spectral, float64);
 * pc_over_pm[B][nbins]: P_c / P_m with c = alpha eta / (3 (eta - 1)) u (Eq. cdef, Sec. IV) and
 *   P_m the power of delta (needs delta), same binning as dgp_power_spectrum (0 in empty bins);
 * delta_gradc[B][nbins]: Delta_gradC = 4 pi k^5 P_C(k) (Eq. DGradC) at the bin centres
 *   kf (N/2)^((b + 1/2) / nbins), kf = 2 pi / L.
 * Synchronises the stream.  Errors: DGP_E_INVALID for NULL plan / u_state, nbins outside
 * [1, 128] when a spectrum is requested, or pc_over_pm without delta. */
int dgp_diagnostics(dgp_plan* plan, const dgp_params* params, const double* delta, const double* u_state,
                    double* nonelliptic, double* pc_over_pm, double* delta_gradc, int nbins, void* stream);

/* Convergence history of the last solve of batch element b: resid[i] = <|R|>/eps of the
 * iterate evaluated by pass i and bad[i] = bad-point fraction of the update that pass computed
 * (Sec. III C, Fig. 3).  For the precision form this is the float64 phase.  Either array may
 * be NULL; returns the number of entries written (at most cap), or a negative error. */
int dgp_solve_history(dgp_plan* plan, int b, double* resid, double* bad, int cap);

/* Message of the last error on the calling thread ("" if none). */
const char* dgp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGP_H */

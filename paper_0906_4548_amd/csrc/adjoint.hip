// Implicit adjoint of the converged field solve.
//
// The solve returns u* with G(u*, delta) = 0 for the discrete Eq. FullDGP2,
//   G(u) = lam [u^2 - sum_ij h_ij^2] + alpha u + gamma N u - S(delta).
// For a loss L(u*) the implicit-function theorem gives dL/ddelta = S^T mu with
// J^T mu = dL/du, J = dG/du.  The spectral operators H_ij (Hessian multipliers)
// and N (-1/kbar) are real and even, hence self-adjoint, so
//   J^T mu = D mu - M^T mu,   D = 2 (1-w) lam u + alpha,
//   M^T mu = 2 lam [ sum_ij H_ij (h_ij mu) - w u mu ] - gamma N mu,
// and the transposed relaxation mu <- D^{-1} (g + M^T mu) has the iteration
// spectrum of the forward relaxation linearised at u*, so it converges when the
// forward does.  With H_22 = I - <.> - H_00 - H_11 the six products collapse to
// five spectral ones plus a local term:
//   sum_ij H_ij(h_ij mu) = H_00((h00-h22) mu) + H_11((h11-h22) mu)
//                        + 2 [H_01(h01 mu) + H_02(h02 mu) + H_12(h12 mu)] + (h22 mu - <h22 mu>).
// One iteration runs four kernels: the axis-1 forward pass of the six product
// spectra, the axis-2 "combine" pass (six forward transforms in, the multipliers,
// one inverse out), the axis-1 inverse pass, and k_adj_step here, which takes the
// axis-0 inverse of the combined spectrum, applies the transposed update pointwise,
// forms the six products of the new multiplier and forward-transforms them along
// axis 0 for the next iteration.  k_adj_finalize decides convergence on the device
// (three multiplier buffers rotated like the forward solve's iterates), so the host
// only looks at the control blocks between chunks of iterations.
#include "dgp_internal.h"

namespace dgp {

template <typename T>
const cx<T>* twiddles(int n);   // device table exp(-2 pi i m / n), defined with the plan code

#define DGP_DISPATCH_N(n, CALL) \
  switch (n) {                  \
    case 8: CALL(8); break;     \
    case 16: CALL(16); break;   \
    case 32: CALL(32); break;   \
    case 64: CALL(64); break;   \
    case 128: CALL(128); break; \
    case 256: CALL(256); break; \
    case 512: CALL(512); break; \
    default: break;             \
  }

// mu = g / D; per workgroup, the number of points where D = 2 (1-w) lam u + alpha is at most
// dmin = 1e-12 alpha (the vertex value of a bad point gives D = 0 up to rounding: there the
// implicit adjoint does not exist) or not finite, and the number of non-finite g
// (part[b][group][0..1])
__global__ void __launch_bounds__(256)
k_adj_init(size_t n3, const double* __restrict__ g, const double* __restrict__ u, double* __restrict__ mu,
           double dscale, double alpha, double* __restrict__ part) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n3;
  double nd = 0.0, ng = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double d = dscale * u[off + i] + alpha;
    const double gg = g[off + i];
    nd += (d > 1e-12 * alpha && isfinite(d)) ? 0.0 : 1.0;
    ng += isfinite(gg) ? 0.0 : 1.0;
    mu[off + i] = gg / d;
  }
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = nd;
  r1[threadIdx.x] = ng;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      r0[threadIdx.x] += r0[threadIdx.x + st];
      r1[threadIdx.x] += r1[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = r0[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
  }
}

// Geometry of k_adj_step: radix-4 axis-0 transforms (the update holds five fields per element,
// the products two), column pairs for 128-byte rows; registers planned for two waves per SIMD.
template <int N>
struct AdjGeo {
  using P = typename PlanPick<N, 2>::type;
  static constexpr int R = P::R;
  using G = AxisTile<double, N, R>;
  static constexpr int kTP = G::kTP, kT = G::kT, kThreads = G::kThreads;
};

// One transposed relaxation step fused with the axis-0 transforms around it, for a tile of
// axis-0 column pairs of batch element b (multiplier buffers indexed by the control block):
//   UPDATE: q = axis-0 inverse of the combined spectrum (the spectral part of M^T mu), then per
//     point M^T mu = q + 2 lam (h22 mu - <h22 mu>) - 2 lam w u mu, the residual
//     |D mu - M^T mu - g| and mu' = (g + M^T mu) / D, written to the next buffer;
//   !UPDATE: mu' = mu (the first products of an adjoint solve).
// Then the six products (h00-h22) mu', (h11-h22) mu', h01 mu', h02 mu', h12 mu', mu' are
// forward-transformed along axis 0 and written as half spectra [6][batch][N/2+1][N][N].
// Per workgroup: sum |res|, sum |g| and sum h22 mu' into part[b][group][0..2].
template <int N, bool UPDATE>
__global__ void __launch_bounds__(AdjGeo<N>::kThreads, 2)
k_adj_step(const cx<double>* __restrict__ qspec, double* __restrict__ mubuf, size_t mu_stride,
           const double* __restrict__ u, const double* __restrict__ h5, const double* __restrict__ g,
           const double* __restrict__ mean_u, const double* __restrict__ mean_h22mu,
           cx<double>* __restrict__ spec6, size_t spec_stride, double* __restrict__ part, AdjCoef k,
           const SolveCtl* __restrict__ ctl, const cx<double>* __restrict__ tw, int batch) {
  using T = double;
  using AG = AdjGeo<N>;
  using P = typename AG::P;
  constexpr int R = AG::R, TP = AG::kTP, TT = AG::kT, NT = AG::kThreads, H = N / 2 + 1;
  constexpr size_t NN = (size_t)N * N, N3 = NN * N;
  constexpr int LSZ = (H * 2 * TP > N * TP) ? H * 2 * TP : N * TP;
  const int b = blockIdx.z;
  if (ctl[b].done) return;
  int tile, i1;
  xcd_tile(tile, i1);
  const int c = threadIdx.x % TP, t = threadIdx.x / TP;
  const int i2 = (tile * TP + c) * 2;
  __shared__ cx<T> lds[LSZ];
  __shared__ double red[3][NT];
  LdsCol<T, TP> L{lds, c};
  const size_t fs = (size_t)batch * N3;
  const size_t off = (size_t)b * N3 + (size_t)i1 * N + i2;   // point (0, i1, i2) of a real field
  auto ld = [&](const double* f, int e) { return *reinterpret_cast<const cx<T>*>(f + off + (size_t)e * NN); };
  const double ub = mean_u[b];
  const double* mu = mubuf + (size_t)ctl[b].cur * mu_stride;
  double sr = 0.0, sg = 0.0, sh = 0.0;
  cx<T> m[R], hz[R], v[R];
  if constexpr (UPDATE) {
    const cx<T>* src = qspec + (size_t)b * H * NN + (size_t)i1 * N + i2;
    for (int kk = t; kk < H; kk += TT) {
      lds[kk * 2 * TP + 2 * c] = src[(size_t)kk * NN];
      lds[kk * 2 * TP + 2 * c + 1] = src[(size_t)kk * NN + 1];
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      cx<T> xa, xb;
      if (e <= N / 2) {
        xa = lds[e * 2 * TP + 2 * c];
        xb = lds[e * 2 * TP + 2 * c + 1];
        if (e == 0 || e == N / 2) { xa.y = T(0); xb.y = T(0); }
      } else {
        xa = conjg(lds[(N - e) * 2 * TP + 2 * c]);
        xb = conjg(lds[(N - e) * 2 * TP + 2 * c + 1]);
      }
      v[q] = mk(xa.x - xb.y, xa.y + xb.x);   // columns i2 (real part) and i2 + 1 (imaginary part)
    }
    fft<T, N, P, +1>(v, tw, L, t);
    const double mh = mean_h22mu[b];
    double* mo = mubuf + (size_t)ctl[b].out * mu_stride;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      const cx<T> mm = ld(mu, e), uu = ld(u, e), a0 = ld(h5, e), a1 = ld(h5 + fs, e), gg = ld(g, e);
      double mn[2], hh[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double mj = j ? mm.y : mm.x, uj = j ? uu.y : uu.x, gj = j ? gg.y : gg.x;
        const double h22 = (uj - ub) - (j ? a0.y : a0.x) - (j ? a1.y : a1.x);
        const double mt = (j ? v[q].y : v[q].x) + k.lam2 * (h22 * mj - mh) - k.lam2 * k.w * uj * mj;
        const double d = k.dscale * uj + k.alpha;
        sr += fabs(d * mj - mt - gj);
        sg += fabs(gj);
        mn[j] = (gj + mt) / d;
        hh[j] = h22;
      }
      m[q] = mk(mn[0], mn[1]);
      hz[q] = mk(hh[0], hh[1]);
      *reinterpret_cast<cx<T>*>(mo + off + (size_t)e * NN) = m[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      const cx<T> uu = ld(u, e), a0 = ld(h5, e), a1 = ld(h5 + fs, e);
      m[q] = ld(mu, e);
      hz[q] = mk((uu.x - ub) - a0.x - a1.x, (uu.y - ub) - a0.y - a1.y);
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) sh += hz[q].x * m[q].x + hz[q].y * m[q].y;
  cx<T>* dst0 = spec6 + (size_t)b * H * NN + (size_t)i1 * N + i2;
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      if (f < 2) {
        const cx<T> a = ld(h5 + f * fs, e);
        v[q] = mk((a.x - hz[q].x) * m[q].x, (a.y - hz[q].y) * m[q].y);
      } else if (f < 5) {
        const cx<T> a = ld(h5 + f * fs, e);
        v[q] = mk(a.x * m[q].x, a.y * m[q].y);
      } else {
        v[q] = m[q];
      }
    }
    // (the first stage of the transform orders its LDS stores after every thread's previous reads)
    fft<T, N, P, -1>(v, tw, L, t);
    lds_barrier();
#pragma unroll
    for (int q = 0; q < R; ++q) lds[(t + q * TT) * TP + c] = v[q];
    lds_barrier();
    cx<T>* dst = dst0 + f * spec_stride;
    for (int kk = t; kk < H; kk += TT) {
      const cx<T> zk = lds[kk * TP + c];
      const cx<T> zn = lds[((N - kk) & (N - 1)) * TP + c];
      store_stream(&dst[(size_t)kk * NN], mk(T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y)));
      store_stream(&dst[(size_t)kk * NN + 1], mk(T(0.5) * (zk.y + zn.y), T(0.5) * (zn.x - zk.x)));
    }
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sg;
  red[2][threadIdx.x] = sh;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const size_t gi = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const size_t groups = (size_t)gridDim.x * gridDim.y;
    for (int j = 0; j < 3; ++j) part[((size_t)b * groups + gi) * 3 + j] = red[j][0];
  }
}

// Convergence control of the adjoint iteration (one workgroup of 1024 threads).  Per active
// element: <h22 mu'> for the next update; with EVAL, r = sum |res| / sum |g| of the multiplier
// that the step's update started from, and the rules of the host loop it replaces: r <= tol
// returns it; otherwise the minimum-residual multiplier is kept (buffer `best`), and at
// max_iter updates (or a non-finite r) that one is returned; else the buffers rotate.
template <bool EVAL>
__global__ void __launch_bounds__(1024)
k_adj_finalize(const double* __restrict__ part, int groups, SolveCtl* __restrict__ ctl, double* __restrict__ mean_h22mu,
               double inv_n3, double tol, int max_iter, int batch) {
  __shared__ double red[3][1024];
  for (int b = 0; b < batch; ++b) {
    __syncthreads();
    if (ctl[b].done) continue;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const double* pb = part + (size_t)b * groups * 3;
    for (int gi = threadIdx.x; gi < groups; gi += 1024) {
      a0 += pb[(size_t)gi * 3];
      a1 += pb[(size_t)gi * 3 + 1];
      a2 += pb[(size_t)gi * 3 + 2];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st)
        for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      SolveCtl& C = ctl[b];
      mean_h22mu[b] = red[2][0] * inv_n3;
      if (EVAL) {
        const double r = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
        const int n = C.iters;
        if (n < kMaxHist) C.hist[n] = r;
        C.passes += 1;
        bool done = false;
        if (r <= tol) {
          C.status = 0;
          C.result = C.cur;
          C.resid = r;
          done = true;
        } else if (r < C.resid_min) {
          C.resid_min = r;
          C.best = C.cur;
        }
        if (!done && (n >= max_iter || r != r)) {
          C.status = 1;
          C.result = C.best;
          C.resid = C.resid_min;
          done = true;
        }
        if (r < C.resid_min) C.resid_min = r;
        if (!done) {
          C.iters = n + 1;
          const int nc = C.out;
          C.cur = nc;
          C.out = 3 - nc - C.best;
        }
        C.done = done ? 1 : 0;
      }
    }
  }
}

// Ellipticity test (Appendix, Eq. EllipticMatrix): at every point the matrix of dF/d(h_ij),
// (2 lam u + alpha) I - 2 lam h, is definite (all eigenvalues of one sign) or not.  Sylvester's
// criterion on the leading principal minors decides definiteness; per-workgroup counts of the
// points that are not elliptic go to part[b][g][2] (second slot 0) for the mean reduction.
__global__ void __launch_bounds__(256)
k_nonelliptic(size_t n3, int batch, const double* __restrict__ u, const double* __restrict__ h5,
              const double* __restrict__ mean_u, double lam, double alpha, double* __restrict__ part) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n3, fs = (size_t)batch * n3;
  const double ub = mean_u[b];
  double cnt = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const size_t k = off + i;
    const double uu = u[k];
    const double h00 = h5[k], h11 = h5[fs + k], h01 = h5[2 * fs + k], h02 = h5[3 * fs + k], h12 = h5[4 * fs + k];
    const double h22 = (uu - ub) - h00 - h11;
    const double d = 2.0 * lam * uu + alpha, c = -2.0 * lam;
    const double m00 = d + c * h00, m11 = d + c * h11, m22 = d + c * h22;
    const double m01 = c * h01, m02 = c * h02, m12 = c * h12;
    const double d1 = m00;
    const double d2 = m00 * m11 - m01 * m01;
    const double d3 = m00 * (m11 * m22 - m12 * m12) - m01 * (m01 * m22 - m12 * m02) + m02 * (m01 * m12 - m11 * m02);
    const bool elliptic = (d1 > 0.0 && d2 > 0.0 && d3 > 0.0) || (d1 < 0.0 && d2 > 0.0 && d3 < 0.0);
    cnt += elliptic ? 0.0 : 1.0;
  }
  __shared__ double r[256];
  r[threadIdx.x] = cnt;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) r[threadIdx.x] += r[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = r[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
  }
}

static int adj_groups(size_t n3) {
  size_t g = (n3 + 255) / 256;
  return int(g > 1024 ? 1024 : g);
}

int adjoint_groups(size_t n3) { return adj_groups(n3); }

void launch_nonelliptic(size_t n3, int batch, const double* u, const double* h5, const double* mean_u, double lam,
                        double alpha, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_nonelliptic, dim3(adj_groups(n3), batch), dim3(256), 0, s, n3, batch, u, h5, mean_u, lam, alpha,
                     part);
}

void launch_adj_init(size_t n3, int batch, const double* g, const double* u, double* mu, double dscale, double alpha,
                     double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_init, dim3(adj_groups(n3), batch), dim3(256), 0, s, n3, g, u, mu, dscale, alpha, part);
}

int adj_step_groups(int n) {
  int g = 0;
#define C(NN) g = (NN / (2 * AdjGeo<NN>::kTP)) * NN;
  DGP_DISPATCH_N(n, C)
#undef C
  return g;
}

void launch_adj_step(int n, bool update, const cx<double>* qspec, double* mubuf, size_t mu_stride, const double* u,
                     const double* h5, const double* g, const double* mean_u, const double* mean_h22mu,
                     cx<double>* spec6, size_t spec_stride, double* part, const AdjCoef& k, const SolveCtl* ctl,
                     int batch, hipStream_t s) {
  const cx<double>* tw = twiddles<double>(n);
#define C(NN)                                                                                                   \
  {                                                                                                             \
    dim3 grid(NN / (2 * AdjGeo<NN>::kTP), NN, batch);                                                           \
    if (update)                                                                                                 \
      hipLaunchKernelGGL((k_adj_step<NN, true>), grid, dim3(AdjGeo<NN>::kThreads), 0, s, qspec, mubuf,         \
                         mu_stride, u, h5, g, mean_u, mean_h22mu, spec6, spec_stride, part, k, ctl, tw, batch); \
    else                                                                                                        \
      hipLaunchKernelGGL((k_adj_step<NN, false>), grid, dim3(AdjGeo<NN>::kThreads), 0, s, qspec, mubuf,        \
                         mu_stride, u, h5, g, mean_u, mean_h22mu, spec6, spec_stride, part, k, ctl, tw, batch); \
  }
  DGP_DISPATCH_N(n, C)
#undef C
}

void launch_adj_finalize(bool eval, const double* part, int groups, SolveCtl* ctl, double* mean_h22mu, size_t n3,
                         double tol, int max_iter, int batch, hipStream_t s) {
  if (eval)
    hipLaunchKernelGGL(k_adj_finalize<true>, dim3(1), dim3(1024), 0, s, part, groups, ctl, mean_h22mu, 1.0 / double(n3),
                       tol, max_iter, batch);
  else
    hipLaunchKernelGGL(k_adj_finalize<false>, dim3(1), dim3(1024), 0, s, part, groups, ctl, mean_h22mu,
                       1.0 / double(n3), tol, max_iter, batch);
}

}  // namespace dgp

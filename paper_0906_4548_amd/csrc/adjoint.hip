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
// The spectral part is formed by the axis-2 "combine" pass (six forward
// transforms in, one inverse out); the kernels here are the pointwise steps.
#include "dgp_internal.h"

namespace dgp {

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

// products p_f = (h00-h22) mu, (h11-h22) mu, h01 mu, h02 mu, h12 mu, mu; partial sums of h22 mu
__global__ void __launch_bounds__(256)
k_adj_products(size_t n3, int batch, const double* __restrict__ mu, const double* __restrict__ u,
               const double* __restrict__ h5, const double* __restrict__ mean_u, double* __restrict__ p6,
               double* __restrict__ part) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n3;
  const size_t fs = (size_t)batch * n3;
  const double ub = mean_u[b];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const size_t k = off + i;
    const double m = mu[k];
    const double h00 = h5[k], h11 = h5[fs + k];
    const double h22 = (u[k] - ub) - h00 - h11;
    p6[k] = (h00 - h22) * m;
    p6[fs + k] = (h11 - h22) * m;
    p6[2 * fs + k] = h5[2 * fs + k] * m;
    p6[3 * fs + k] = h5[3 * fs + k] * m;
    p6[4 * fs + k] = h5[4 * fs + k] * m;
    p6[5 * fs + k] = m;
    acc += h22 * m;
  }
  __shared__ double r[256];
  r[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) r[threadIdx.x] += r[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = r[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
  }
}

// M^T mu = q + 2 lam (h22 mu - <h22 mu>) - 2 lam w u mu;  res = D mu - M^T mu - g;  mu <- (g + M^T mu) / D
__global__ void __launch_bounds__(256)
k_adj_update(size_t n3, const double* __restrict__ q, const double* __restrict__ mu, double* __restrict__ mu_new,
             const double* __restrict__ u,
             const double* __restrict__ h5, const double* __restrict__ mean_u, const double* __restrict__ mean_h22mu,
             const double* __restrict__ g, double lam, double w, double alpha, double* __restrict__ part,
             int batch) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * n3;
  const size_t fs = (size_t)batch * n3;
  const double ub = mean_u[b], mh = mean_h22mu[b];
  double sr = 0.0, sg = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const size_t k = off + i;
    const double m = mu[k], uu = u[k];
    const double h22 = (uu - ub) - h5[k] - h5[fs + k];
    const double mt = q[k] + 2.0 * lam * (h22 * m - mh) - 2.0 * lam * w * uu * m;
    const double d = 2.0 * (1.0 - w) * lam * uu + alpha;
    const double gg = g[k];
    sr += fabs(d * m - mt - gg);
    sg += fabs(gg);
    mu_new[k] = (gg + mt) / d;
  }
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = sr;
  r1[threadIdx.x] = sg;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = r0[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
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

void launch_adj_products(size_t n3, int batch, const double* mu, const double* u, const double* h5,
                         const double* mean_u, double* p6, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_products, dim3(adj_groups(n3), batch), dim3(256), 0, s, n3, batch, mu, u, h5, mean_u, p6,
                     part);
}

void launch_adj_update(size_t n3, int batch, const double* q, const double* mu, double* mu_new, const double* u,
                       const double* h5, const double* mean_u, const double* mean_h22mu, const double* g, double lam,
                       double w, double alpha, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_update, dim3(adj_groups(n3), batch), dim3(256), 0, s, n3, q, mu, mu_new, u, h5, mean_u,
                     mean_h22mu, g, lam, w, alpha, part, batch);
}

}  // namespace dgp

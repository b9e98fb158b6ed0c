// Particle-mesh kernels: deterministic CIC deposit, density contrast, CIC
// interpolation fused with the leapfrog kick-drift, and the CIC adjoint.
//
// CIC (Sec. III A, Eq. CIC): tent window W(x) = 1 - |x|/h per axis, 3D weight the
// product of the three; the same weights interpolate the force back (no
// self-force).  Mesh node j sits at x = j h.  The deposit is made bit-exact and
// order independent: per-axis weights (1 - f, f) in FP64 with no fused
// multiply-add, the 3D weight as (w_x w_y) w_z, quantised to Q = rint(W 2^40)
// and summed with 64-bit integer atomics.
#include "dgp_internal.h"

namespace dgp {

constexpr double kQScale = 1099511627776.0;  // 2^40

struct Cic {
  int i0[3], i1[3];
  double w0[3], w1[3];
};

template <typename P>
__device__ __forceinline__ Cic cic_of(const P* __restrict__ pos, long long np, long long p, int n, double scale) {
#pragma clang fp contract(off)
  Cic c;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double s = double(pos[(size_t)d * np + p]) * scale;
    const double fl = floor(s);
    const double f = s - fl;
    long long i = (long long)fl % n;
    if (i < 0) i += n;
    c.i0[d] = int(i);
    c.i1[d] = int((i + 1) % n);
    c.w0[d] = 1.0 - f;
    c.w1[d] = f;
  }
  return c;
}

#ifndef DGP_DEPOSIT_GROUP
#define DGP_DEPOSIT_GROUP 64
#endif
// Lane -> particle map of the deposit: groups of G consecutive particles per lane group, the
// 64/G groups of one wavefront taken from distant parts of the array, so one atomic
// instruction spreads over 64/G cache lines instead of a few (a bijection of [0, 64 W)).
template <int G>
__device__ __forceinline__ long long deposit_index(long long np) {
  const long long w = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  const long long waves = (np + 63) >> 6;
  if (G >= 64) return ((long long)blockIdx.x * 256 + threadIdx.x);
  if (w >= waves) return np;  // surplus wavefronts of the last block
  return (long long)(l % G) + (long long)G * (w + waves * (long long)(l / G));
}

template <typename P>
__global__ void __launch_bounds__(256)
k_deposit(const P* __restrict__ pos, long long np, int n, double scale, unsigned long long* __restrict__ grid) {
#pragma clang fp contract(off)
  const long long p = deposit_index<DGP_DEPOSIT_GROUP>(np);
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
    const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
      const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
        const size_t iz = (size_t)(cc ? c.i1[2] : c.i0[2]);
        const unsigned long long q = (unsigned long long)(long long)rint(wgt * kQScale);
        atomicAdd(&grid[(ix * n + iy) * n + iz], q);
      }
    }
  }
}

// XCD id of the executing wave (hardware register XCC_ID, bits [3:0]); clamped to 8 copies.
__device__ __forceinline__ int xcc_id() {
  return int(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20)) & 7;
}

// Deposit into the private grid copy of the executing XCD with workgroup-scope atomics: every
// workgroup of one XCD shares that XCD's L2, where the integer atomics are performed.
template <typename P>
__global__ void __launch_bounds__(256)
k_deposit_xcd(const P* __restrict__ pos, long long np, int n, double scale, unsigned long long* __restrict__ copies) {
#pragma clang fp contract(off)
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const size_t n3 = (size_t)n * n * n;
  unsigned long long* grid = copies + (size_t)xcc_id() * n3;
  const Cic c = cic_of(pos, np, p, n, scale);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
    const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
      const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
        const size_t iz = (size_t)(cc ? c.i1[2] : c.i0[2]);
        const unsigned long long q = (unsigned long long)(long long)rint(wgt * kQScale);
        __hip_atomic_fetch_add(&grid[(ix * n + iy) * n + iz], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

// grid = sum of the 8 copies (then the copies are cleared for the next deposit)
__global__ void __launch_bounds__(256)
k_sum_copies(unsigned long long* __restrict__ copies, size_t n3, long long* __restrict__ grid) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    unsigned long long s = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      s += copies[x * n3 + i];
      copies[x * n3 + i] = 0ull;
    }
    grid[i] = (long long)s;
  }
}

__global__ void __launch_bounds__(256)
k_counts_to_delta(const long long* __restrict__ grid, size_t n3, double qscale, double* __restrict__ delta) {
#pragma clang fp contract(off)
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double d = double(grid[i]) * qscale;
    delta[i] = d - 1.0;
  }
}

__global__ void __launch_bounds__(256)
k_sub_mean(double* __restrict__ x, size_t n3, const double* __restrict__ mean) {
  const int b = blockIdx.y;
  const double m = mean[b];
  double* xb = x + (size_t)b * n3;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) xb[i] -= m;
}

// interpolate a 3-component mesh [3][N^3] to particles
template <typename P>
__device__ __forceinline__ void gather3(const double* __restrict__ mesh3, size_t n3, int n, const Cic& c,
                                        double (&f)[3]) {
  f[0] = f[1] = f[2] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
    const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
      const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
        const size_t idx = (ix * n + iy) * n + (size_t)(cc ? c.i1[2] : c.i0[2]);
        f[0] += wgt * mesh3[idx];
        f[1] += wgt * mesh3[n3 + idx];
        f[2] += wgt * mesh3[2 * n3 + idx];
      }
    }
  }
}

template <typename P>
__global__ void __launch_bounds__(256)
k_interp(const double* __restrict__ mesh3, const P* __restrict__ pos, long long np, int n, double scale,
         double* __restrict__ force) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
  double f[3];
  gather3<P>(mesh3, (size_t)n * n * n, n, c, f);
  force[p] = f[0];
  force[np + p] = f[1];
  force[2 * np + p] = f[2];
}

// leapfrog with momenta at half steps: p += kick * g(x_n); x += drift * p; wrap into [0, L)
template <typename P>
__global__ void __launch_bounds__(256)
k_interp_kick_drift(const double* __restrict__ mesh3, P* __restrict__ pos, P* __restrict__ vel, long long np,
                    int n, double scale, double box, double kick, double drift) {
#pragma clang fp contract(off)
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
  double f[3];
  gather3<P>(mesh3, (size_t)n * n * n, n, c, f);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * np + p;
    const double v = double(vel[k]) + kick * f[d];
    double x = double(pos[k]) + drift * v;
    x = x - box * floor(x / box);
    P xo = P(x);
    if (xo >= P(box)) xo = xo - P(box);
    vel[k] = P(v);
    pos[k] = xo;
  }
}

// dL/dx_p = (N^3/Np) sum_c g_c dW_c/dx_p  (derivative of the unquantised weights)
template <typename P>
__global__ void __launch_bounds__(256)
k_deposit_backward(const P* __restrict__ pos, long long np, int n, double scale, const double* __restrict__ g,
                   double mass, double* __restrict__ grad) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
    const double dx = a ? scale : -scale;
    const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wy = b ? c.w1[1] : c.w0[1];
      const double dy = b ? scale : -scale;
      const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wz = cc ? c.w1[2] : c.w0[2];
        const double dz = cc ? scale : -scale;
        const double gc = g[(ix * n + iy) * n + (size_t)(cc ? c.i1[2] : c.i0[2])];
        gx += gc * dx * wy * wz;
        gy += gc * wx * dy * wz;
        gz += gc * wx * wy * dz;
      }
    }
  }
  grad[p] = gx * mass;
  grad[np + p] = gy * mass;
  grad[2 * np + p] = gz * mass;
}

template <typename T>
__global__ void __launch_bounds__(256) k_convert(size_t count, const void* __restrict__ in, int in_fp32, T* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
    out[i] = in_fp32 ? T(static_cast<const float*>(in)[i]) : T(static_cast<const double*>(in)[i]);
}

static unsigned grid_for(long long count) {
  long long g = (count + 255) / 256;
  return unsigned(g < 1 ? 1 : g);
}
static unsigned grid_strided(size_t count) {
  size_t g = (count + 255) / 256;
  return unsigned(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

void launch_deposit(int n, double box, const void* pos, int pos_fp32, long long np, long long* grid, hipStream_t s) {
  const double scale = double(n) / box;
  if (pos_fp32)
    hipLaunchKernelGGL((k_deposit<float>), dim3(grid_for(np)), dim3(256), 0, s, static_cast<const float*>(pos), np, n,
                       scale, reinterpret_cast<unsigned long long*>(grid));
  else
    hipLaunchKernelGGL((k_deposit<double>), dim3(grid_for(np)), dim3(256), 0, s, static_cast<const double*>(pos), np,
                       n, scale, reinterpret_cast<unsigned long long*>(grid));
}

void launch_deposit_xcd(int n, double box, const void* pos, int pos_fp32, long long np, unsigned long long* copies,
                        long long* grid, hipStream_t s) {
  const double scale = double(n) / box;
  if (pos_fp32)
    hipLaunchKernelGGL((k_deposit_xcd<float>), dim3(grid_for(np)), dim3(256), 0, s, static_cast<const float*>(pos),
                       np, n, scale, copies);
  else
    hipLaunchKernelGGL((k_deposit_xcd<double>), dim3(grid_for(np)), dim3(256), 0, s, static_cast<const double*>(pos),
                       np, n, scale, copies);
  const size_t n3 = (size_t)n * n * n;
  hipLaunchKernelGGL(k_sum_copies, dim3(grid_strided(n3)), dim3(256), 0, s, copies, n3, grid);
}

void launch_counts_to_delta(int n, const long long* grid, long long np, double* delta, hipStream_t s) {
  const size_t n3 = (size_t)n * n * n;
  const double qscale = ldexp(double(n3) / double(np), -40);
  hipLaunchKernelGGL(k_counts_to_delta, dim3(grid_strided(n3)), dim3(256), 0, s, grid, n3, qscale, delta);
}

void launch_sub_mean(size_t n3, double* x, int batch, const double* mean, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_strided(n3), batch), dim3(256), 0, s, x, n3, mean);
}

void launch_interp(int n, double box, const double* mesh3, const void* pos, int pos_fp32, long long np, double* force,
                   hipStream_t s) {
  const double scale = double(n) / box;
  if (pos_fp32)
    hipLaunchKernelGGL((k_interp<float>), dim3(grid_for(np)), dim3(256), 0, s, mesh3, static_cast<const float*>(pos),
                       np, n, scale, force);
  else
    hipLaunchKernelGGL((k_interp<double>), dim3(grid_for(np)), dim3(256), 0, s, mesh3,
                       static_cast<const double*>(pos), np, n, scale, force);
}

void launch_interp_kick_drift(int n, double box, const double* mesh3, void* pos, void* vel, int fp32, long long np,
                              double kick, double drift, hipStream_t s) {
  const double scale = double(n) / box;
  if (fp32)
    hipLaunchKernelGGL((k_interp_kick_drift<float>), dim3(grid_for(np)), dim3(256), 0, s, mesh3,
                       static_cast<float*>(pos), static_cast<float*>(vel), np, n, scale, box, kick, drift);
  else
    hipLaunchKernelGGL((k_interp_kick_drift<double>), dim3(grid_for(np)), dim3(256), 0, s, mesh3,
                       static_cast<double*>(pos), static_cast<double*>(vel), np, n, scale, box, kick, drift);
}

void launch_deposit_backward(int n, double box, const void* pos, int pos_fp32, long long np, const double* grad_delta,
                             double* grad_pos, hipStream_t s) {
  const double scale = double(n) / box;
  const double mass = double(n) * n * n / double(np);
  if (pos_fp32)
    hipLaunchKernelGGL((k_deposit_backward<float>), dim3(grid_for(np)), dim3(256), 0, s,
                       static_cast<const float*>(pos), np, n, scale, grad_delta, mass, grad_pos);
  else
    hipLaunchKernelGGL((k_deposit_backward<double>), dim3(grid_for(np)), dim3(256), 0, s,
                       static_cast<const double*>(pos), np, n, scale, grad_delta, mass, grad_pos);
}

template <typename T>
void launch_convert(size_t count, const void* in, int in_fp32, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<T>), dim3(grid_strided(count)), dim3(256), 0, s, count, in, in_fp32, out);
}
template void launch_convert<double>(size_t, const void*, int, double*, hipStream_t);
template void launch_convert<float>(size_t, const void*, int, float*, hipStream_t);

}  // namespace dgp

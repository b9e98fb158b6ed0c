// Particle-mesh kernels: deterministic CIC deposit, density contrast, CIC
// interpolation fused with the leapfrog kick-drift, and the CIC adjoint.
//
// CIC (Sec. III A, Eq. CIC): tent window W(x) = 1 - |x|/h per axis, 3D weight the
// product of the three; the same weights interpolate the force back (no
// self-force).  Mesh node j sits at x = j h.  The deposit is made bit-exact and
// order independent: per-axis weights (1 - f, f) in FP64 with no fused
// multiply-add, the 3D weight as (w_x w_y) w_z, quantised to Q = rint(W 2^40)
// and summed with 64-bit integer atomics.
#include <mutex>

#include "dgp_internal.h"

namespace dgp {

constexpr double kQScale = 1099511627776.0;  // 2^40

struct Cic {
  int i0[3], i1[3];
  double w0[3], w1[3];
};

// cell and weights of a particle at x (already in mesh units: x = pos * N / L)
__device__ __forceinline__ Cic cic_at(const double (&s3)[3], int n) {
#pragma clang fp contract(off)
  Cic c;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double s = s3[d];
    const double fl = floor(s);
    const double f = s - fl;
    const int i = int((long long)fl & (n - 1));   // periodic wrap (n is a power of two)
    c.i0[d] = i;
    c.i1[d] = (i + 1) & (n - 1);
    c.w0[d] = 1.0 - f;
    c.w1[d] = f;
  }
  return c;
}

template <typename P>
__device__ __forceinline__ Cic cic_of(const P* __restrict__ pos, long long np, long long p, int n, double scale) {
#pragma clang fp contract(off)
  double s3[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) s3[d] = double(pos[(size_t)d * np + p]) * scale;
  return cic_at(s3, n);
}

// Binned deposit.  A workgroup takes a chunk of consecutive particles, finds the
// periodic bounding box of their CIC cells and, when the box fits the LDS histogram,
// sums the chunk's quantised weights there with LDS atomics and then adds each
// non-zero box cell to the mesh with one global atomic.  Integer sums make the result
// identical to the direct deposit in any order; the gain needs spatially coherent
// chunks (particles stored in compact Lagrangian blocks).  A chunk whose box is too
// large takes the direct per-particle atomics.  Larger chunks mean fewer global atomics per
// particle (a box's surface grows slower than its volume) but more registers and LDS: the
// geometry is chosen by mesh size, from the measured deposit times of the Zel'dovich loads
// (256^3 float64 particles: 512 / 1024 / 2048 particles per chunk 357 / 299 / 322 us; 512^3
// float32 particles: 2.84 / 2.84 / 2.45 ms).  The 2048-particle chunk recomputes each
// particle's cell and weights after the box instead of holding them across its barriers, and
// sizes its histogram at three cells per particle: occupancy 2 -> 3 waves per SIMD, 512^3
// 2.43 -> 2.12 ms (the 1024-particle chunk, LDS-bound at four, gains nothing from either).
template <int CH>
struct DepGeo {
  static constexpr int kChunk = CH;                         // particles per workgroup
  static constexpr int kPPT = CH / 256;                     // particles per thread
  static constexpr bool kRecompute = CH >= 2048;
  static constexpr int kCap = (kRecompute ? 3 : 4) * CH;    // cells of the LDS histogram (8 bytes each)
  static_assert(CH % 256 == 0, "chunk must be a multiple of the workgroup size");
};
// the interpolation adjoint's scatter (up to three components per cell in LDS) keeps its own
constexpr int kIgChunk = 512, kIgPPT = kIgChunk / 256, kIgCap = 2048;

// offset of cell i from the reference cell r on a periodic axis of n cells, in [-n/2, n/2)
__device__ __forceinline__ int periodic_offset(int i, int r, int n) {
  int o = i - r;
  if (o < -n / 2) o += n;
  if (o >= n / 2) o -= n;
  return o;
}

// Periodic bounding box of a chunk's CIC base cells, relative to the base cell cr of its
// first particle: offsets in [-n/2, n/2) per axis, box lo[d] .. lo[d] + ext[d] - 1 (the
// +1 corners included).  xs holds the positions of the thread's particles (p0 + threadIdx.x
// + 256 k), loaded by the caller.  Returns true when the box volume is at most `cap`.
// Every thread of the (256-thread) workgroup must call it.
template <int PPT, typename P>
__device__ __forceinline__ bool chunk_box(const P* __restrict__ pos, const P (&xs)[PPT][3], long long np, int n,
                                          double scale, long long p0, int cap, Cic& cr, Cic (&cs)[PPT],
                                          int (&off)[PPT][3], int (&bx)[6]) {
  __shared__ int wlo[4][3], whi[4][3];
  __shared__ int sbox[7];
  cr = cic_of(pos, np, p0, n, scale);
  int lo[3] = {n, n, n}, hi[3] = {-n, -n, -n};
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const long long p = p0 + threadIdx.x + k * 256;
    if (p < np) {
      const double s3[3] = {double(xs[k][0]) * scale, double(xs[k][1]) * scale, double(xs[k][2]) * scale};
      cs[k] = cic_at(s3, n);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        off[k][d] = periodic_offset(cs[k].i0[d], cr.i0[d], n);
        lo[d] = min(lo[d], off[k][d]);
        hi[d] = max(hi[d], off[k][d] + 1);
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wlo[threadIdx.x >> 6][d] = lo[d];
      whi[threadIdx.x >> 6][d] = hi[d];
    }
  }
  lds_barrier();
  if (threadIdx.x == 0) {
    long long vol = 1;
    for (int d = 0; d < 3; ++d) {
      int l = wlo[0][d], h = whi[0][d];
      for (int w = 1; w < 4; ++w) {
        l = min(l, wlo[w][d]);
        h = max(h, whi[w][d]);
      }
      sbox[d] = l;
      sbox[3 + d] = h - l + 1;
      vol *= h - l + 1;
    }
    sbox[6] = vol <= cap ? 1 : 0;
  }
  lds_barrier();
#pragma unroll
  for (int d = 0; d < 6; ++d) bx[d] = sbox[d];
  return sbox[6] != 0;
}

// the positions of the thread's particles in a chunk (unused slots past np left at 0); streaming
// loads: a kernel reads each particle once
template <int PPT, typename P>
__device__ __forceinline__ void load_chunk(const P* __restrict__ a, long long np, long long p0, P (&xs)[PPT][3]) {
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const long long p = p0 + threadIdx.x + k * 256;
#pragma unroll
    for (int d = 0; d < 3; ++d) xs[k][d] = p < np ? __builtin_nontemporal_load(&a[(size_t)d * np + p]) : P(0);
  }
}

// raise *bad when one of the thread's particles has a non-finite coordinate (the cell index of
// such a particle is still reduced into the mesh, so no access leaves it; the caller reports it)
template <int PPT, typename P>
__device__ __forceinline__ void flag_nonfinite(const P (&xs)[PPT][3], int* __restrict__ bad) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < PPT; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = ok && isfinite(double(xs[k][d]));
  if (!ok) atomicOr(bad, 1);
}

// mesh index of box cell i (row-major over the box extents), wrapped onto the periodic mesh
__device__ __forceinline__ size_t box_cell(int i, const Cic& cr, const int (&bx)[6], int n) {
  const int plane = bx[4] * bx[5];
  const int x = i / plane, r = i - x * plane;
  const int y = r / bx[5], z = r - y * bx[5];
  const size_t gx = (size_t)((cr.i0[0] + bx[0] + x) & (n - 1));   // periodic wrap (n is a power of two)
  const size_t gy = (size_t)((cr.i0[1] + bx[1] + y) & (n - 1));
  const size_t gz = (size_t)((cr.i0[2] + bx[2] + z) & (n - 1));
  return (gx * n + gy) * n + gz;
}

template <typename P, int CH>
__global__ void __launch_bounds__(256)
k_deposit_bin(const P* __restrict__ pos, long long np, int n, double scale, unsigned long long* __restrict__ grid,
              int* __restrict__ bad) {
#pragma clang fp contract(off)
  using G = DepGeo<CH>;
  constexpr int kDepPPT = G::kPPT;
  __shared__ unsigned long long hist[G::kCap];
  const long long p0 = xcd_chunk() * G::kChunk;
  P xs[kDepPPT][3];
  load_chunk<kDepPPT>(pos, np, p0, xs);
  flag_nonfinite<kDepPPT>(xs, bad);
  Cic cr, cs[kDepPPT];
  int off[kDepPPT][3], bx[6];
  const bool binned = chunk_box<kDepPPT>(pos, xs, np, n, scale, p0, G::kCap, cr, cs, off, bx);
  const int vol = bx[3] * bx[4] * bx[5];
  if (binned)
    for (int i = threadIdx.x; i < vol; i += 256) hist[i] = 0ull;
  lds_barrier();
#pragma unroll
  for (int k = 0; k < kDepPPT; ++k) {
    const long long p = p0 + threadIdx.x + k * 256;
    if (p >= np) continue;
    // with kRecompute the cell and weights again from the position (the chunk box's arithmetic)
    const double s3[3] = {double(xs[k][0]) * scale, double(xs[k][1]) * scale, double(xs[k][2]) * scale};
    const Cic c = G::kRecompute ? cic_at(s3, n) : cs[k];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double wx = a ? c.w1[0] : c.w0[0];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
          const unsigned long long q = (unsigned long long)(long long)rint(wgt * kQScale);
          if (binned) {
            const int li = ((off[k][0] + a - bx[0]) * bx[4] + (off[k][1] + b - bx[1])) * bx[5] + (off[k][2] + cc - bx[2]);
            atomicAdd(&hist[li], q);
          } else {
            const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
            const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
            const size_t iz = (size_t)(cc ? c.i1[2] : c.i0[2]);
            atomicAdd(&grid[(ix * n + iy) * n + iz], q);
          }
        }
      }
    }
  }
  if (!binned) return;
  lds_barrier();
  for (int i = threadIdx.x; i < vol; i += 256) {
    const unsigned long long v = hist[i];
    if (v != 0ull) atomicAdd(&grid[box_cell(i, cr, bx, n)], v);
  }
}

// delta = counts * qscale - 1; with mean_q (the mean of the fixed-point counts, a deterministic
// reduction of the grid), minus the mean of delta, qscale <q> - 1, in the same pass
__global__ void __launch_bounds__(256)
k_counts_to_delta(const long long* __restrict__ grid, size_t n3, double qscale, double* __restrict__ delta,
                  const int* __restrict__ bad, const double* __restrict__ mean_q) {
#pragma clang fp contract(off)
  const bool nan_out = *bad != 0;   // a non-finite position: delta is undefined, mark it so
  const double m = mean_q ? *mean_q * qscale - 1.0 : 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double d = double(grid[i]) * qscale;
    delta[i] = nan_out ? __builtin_nan("") : (d - 1.0) - m;
  }
}

// CIC interpolation of an NC-component field: f[k] = sum over the 8 corners of
// (w_x w_y) w_z times the corner value of component k; `at(a, b, c, k)` reads the value.
template <int NC, class At>
__device__ __forceinline__ void gather_corners(const Cic& c, const At& at, double (&f)[NC]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < NC; ++k) f[k] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
#pragma unroll
        for (int k = 0; k < NC; ++k) f[k] += wgt * at(a, b, cc, k);
      }
    }
  }
}

// flat mesh index of corner (a, b, cc) of a particle's CIC cell
__device__ __forceinline__ size_t corner_index(const Cic& c, int a, int b, int cc, int n) {
  const size_t ix = (size_t)(a ? c.i1[0] : c.i0[0]);
  const size_t iy = (size_t)(b ? c.i1[1] : c.i0[1]);
  const size_t iz = (size_t)(cc ? c.i1[2] : c.i0[2]);
  return (ix * n + iy) * n + iz;
}

// interpolate an NC-component mesh [NC][N^3] to particles
template <int NC, typename M>
__device__ __forceinline__ void gather_mesh(const M* __restrict__ mesh, size_t n3, int n, const Cic& c,
                                            double (&f)[NC]) {
  gather_corners<NC>(
      c, [&](int a, int b, int cc, int k) { return double(mesh[(size_t)k * n3 + corner_index(c, a, b, cc, n)]); }, f);
}

// out[k][p] = sum_c W_c(x_p) mesh[k][c]
template <typename P, typename M, int NC>
__global__ void __launch_bounds__(256)
k_interp(const M* __restrict__ mesh, const P* __restrict__ pos, long long np, int n, double scale,
         double* __restrict__ out) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
  double f[NC];
  gather_mesh<NC, M>(mesh, (size_t)n * n * n, n, c, f);
#pragma unroll
  for (int k = 0; k < NC; ++k) out[(size_t)k * np + p] = f[k];
}

// Leapfrog with momenta at half steps: p += kick * g(x_n); x += drift * p; wrap into [0, L).
// The force mesh of the chunk's box is staged in LDS (coalesced rows), with the chunking of the
// binned deposit (smaller chunks: three components per cell in LDS); chunks with larger boxes
// gather from the mesh.
#ifndef DGP_GATHER_CHUNK
#define DGP_GATHER_CHUNK 256
#endif
#ifndef DGP_GATHER_BIN_CAP
#define DGP_GATHER_BIN_CAP 1024
#endif
constexpr int kGatherChunk = DGP_GATHER_CHUNK;
constexpr int kGatherPPT = kGatherChunk / 256;
constexpr int kGatherCap = DGP_GATHER_BIN_CAP;
static_assert(kGatherChunk % 256 == 0, "chunk must be a multiple of the workgroup size");

template <typename P, typename M>
__global__ void __launch_bounds__(256)
k_interp_kick_drift_bin(const M* __restrict__ mesh3, P* __restrict__ pos, P* __restrict__ vel, long long np,
                        int n, double scale, double box, double kick, double drift) {
#pragma clang fp contract(off)
  __shared__ M fl[3 * kGatherCap];
  const size_t n3 = (size_t)n * n * n;
  const long long p0 = xcd_chunk() * kGatherChunk;
  // positions and velocities are loaded together up front and kept in registers
  P xs[kGatherPPT][3], vs[kGatherPPT][3];
  load_chunk<kGatherPPT>(pos, np, p0, xs);
  load_chunk<kGatherPPT>(vel, np, p0, vs);
  Cic cr, cs[kGatherPPT];
  int off[kGatherPPT][3], bx[6];
  const bool binned = chunk_box<kGatherPPT>(pos, xs, np, n, scale, p0, kGatherCap, cr, cs, off, bx);
  if (binned) {
    const int vol = bx[3] * bx[4] * bx[5];
    for (int i = threadIdx.x; i < vol; i += 256) {
      const size_t g = box_cell(i, cr, bx, n);
      fl[i] = mesh3[g];
      fl[kGatherCap + i] = mesh3[n3 + g];
      fl[2 * kGatherCap + i] = mesh3[2 * n3 + g];
    }
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < kGatherPPT; ++k) {
    const long long p = p0 + threadIdx.x + k * 256;
    if (p >= np) continue;
    double f[3];
    // the cell and weights again from the position (the chunk box's arithmetic): not holding
    // them across the staging loop and its barrier leaves 65 instead of 75 VGPRs (occupancy
    // 6 -> 7-8; 512^3 float32 particles 2.71 -> 2.30 ms, 256^3 unchanged)
    const double s3[3] = {double(xs[k][0]) * scale, double(xs[k][1]) * scale, double(xs[k][2]) * scale};
    const Cic ck = cic_at(s3, n);
    if (binned) {
      gather_corners<3>(
          ck,
          [&](int a, int b, int cc, int q) {
            const int li = ((off[k][0] + a - bx[0]) * bx[4] + (off[k][1] + b - bx[1])) * bx[5] + (off[k][2] + cc - bx[2]);
            return double(fl[q * kGatherCap + li]);
          },
          f);
    } else {
      gather_mesh<3, M>(mesh3, n3, n, ck, f);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const size_t i = (size_t)d * np + p;
      const double v = double(vs[k][d]) + kick * f[d];
      double x = double(xs[k][d]) + drift * v;
      x = x - box * floor(x / box);
      P xo = P(x);
      if (xo >= P(box)) xo = xo - P(box);
      __builtin_nontemporal_store(P(v), &vel[i]);   // streaming: read again only by the next step
      __builtin_nontemporal_store(xo, &pos[i]);
    }
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

// ------------------------------------------------------------------ CIC interpolation adjoint
// The interpolation out[m][p] = sum_c W_c(x_p) mesh[m][c] (Sec. III A: forces are interpolated
// with the deposit's assignment function, Eq. CIC; unquantised weights W_c = w_x w_y w_z) has,
// for g = dL/dout,
//   dL/dx_p        = sum_m g[m][p] sum_c mesh[m][c] dW_c/dx_p     (gather, k_interp_grad_pos)
//   dL/dmesh[m][c] = sum_p g[m][p] W_c(x_p)                       (scatter, k_interp_grad_mesh_bin)
// The scatter sums in 64-bit fixed point, so the result has the same bits in any particle order:
// every term is rounded to an integer multiple of 2^-e, e chosen per call so that no sum can
// reach 2^62 (a cell's sum is at most max|g| times its mass sum_p W_c, which the deposit of the
// same positions bounds).

// dL/dx_p: per particle, the 8 corners of its cell
template <typename P, int NC>
__global__ void __launch_bounds__(256)
k_interp_grad_pos(const double* __restrict__ mesh, const P* __restrict__ pos, long long np, int n, double scale,
                  const double* __restrict__ g, double* __restrict__ grad) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cic c = cic_of(pos, np, p, n, scale);
  const size_t n3 = (size_t)n * n * n;
  double gm[NC];
#pragma unroll
  for (int m = 0; m < NC; ++m) gm[m] = g[(size_t)m * np + p];
  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? c.w1[0] : c.w0[0];
    const double dx = a ? scale : -scale;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wy = b ? c.w1[1] : c.w0[1];
      const double dy = b ? scale : -scale;
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const double wz = cc ? c.w1[2] : c.w0[2];
        const double dz = cc ? scale : -scale;
        const size_t idx = corner_index(c, a, b, cc, n);
        double proj = 0.0;
#pragma unroll
        for (int m = 0; m < NC; ++m) proj += gm[m] * mesh[(size_t)m * n3 + idx];
        gx += proj * dx * wy * wz;
        gy += proj * wx * dy * wz;
        gz += proj * wx * wy * dz;
      }
    }
  }
  grad[p] = gx;
  grad[np + p] = gy;
  grad[2 * np + p] = gz;
}

__global__ void k_zero_scale_state(unsigned long long* __restrict__ st, int* __restrict__ bad) {
  if (threadIdx.x < 3) st[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) *bad = 0;
}

// st[0]: bit pattern of max |g| (non-negative doubles order like their bit patterns), st[1]: the
// largest fixed-point mass of the grid; *bad raised for a non-finite g
__global__ void __launch_bounds__(256)
k_max_abs_and_mass(const double* __restrict__ g, size_t count, const long long* __restrict__ grid, size_t n3,
                   unsigned long long* __restrict__ st, int* __restrict__ bad) {
  double m = 0.0;
  long long mm = 0;
  bool ok = true;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
    const double v = g[i];
    ok = ok && isfinite(v);
    m = fmax(m, fabs(v));
  }
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) mm = max(mm, grid[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o, 64));
    mm = max(mm, __shfl_xor(mm, o, 64));
  }
  if (!ok) atomicOr(bad, 1);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&st[0], (unsigned long long)__double_as_longlong(m));
    atomicMax(&st[1], (unsigned long long)mm);
  }
}

// st[2] = e with (max|g|) (mass bound) 2^e < 2^62
__global__ void k_interp_scale(unsigned long long* __restrict__ st) {
  if (threadIdx.x != 0) return;
  const double gmax = __longlong_as_double((long long)st[0]);
  const double mass = double((long long)st[1]) * 0x1p-40 * (1.0 + 0x1p-20) + 0x1p-20;
  const double bound = gmax * mass;
  int e = 0;
  if (bound > 0.0 && isfinite(bound)) {
    int ex = 0;
    (void)frexp(bound, &ex);   // bound < 2^ex
    e = 62 - ex;
    e = e > 960 ? 960 : (e < -960 ? -960 : e);
  }
  st[2] = (unsigned long long)(long long)e;
}

template <typename P, int NC>
__global__ void __launch_bounds__(256)
k_interp_grad_mesh_bin(const P* __restrict__ pos, long long np, int n, double scale, const double* __restrict__ g,
                       const unsigned long long* __restrict__ st, unsigned long long* __restrict__ acc) {
#pragma clang fp contract(off)
  __shared__ unsigned long long hist[NC * kIgCap];
  const size_t n3 = (size_t)n * n * n;
  const int e = (int)(long long)st[2];
  const long long p0 = xcd_chunk() * kIgChunk;
  P xs[kIgPPT][3];
  load_chunk<kIgPPT>(pos, np, p0, xs);
  Cic cr, cs[kIgPPT];
  int off[kIgPPT][3], bx[6];
  const bool binned = chunk_box<kIgPPT>(pos, xs, np, n, scale, p0, kIgCap, cr, cs, off, bx);
  const int vol = bx[3] * bx[4] * bx[5];
  if (binned)
    for (int i = threadIdx.x; i < vol; i += 256)
#pragma unroll
      for (int m = 0; m < NC; ++m) hist[m * kIgCap + i] = 0ull;
  lds_barrier();
#pragma unroll
  for (int k = 0; k < kIgPPT; ++k) {
    const long long p = p0 + threadIdx.x + k * 256;
    if (p >= np) continue;
    const Cic& c = cs[k];
    double gm[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) gm[m] = g[(size_t)m * np + p];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double wx = a ? c.w1[0] : c.w0[0];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double wxy = wx * (b ? c.w1[1] : c.w0[1]);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          const double wgt = wxy * (cc ? c.w1[2] : c.w0[2]);
          const int li = ((off[k][0] + a - bx[0]) * bx[4] + (off[k][1] + b - bx[1])) * bx[5] + (off[k][2] + cc - bx[2]);
          const size_t gi = corner_index(c, a, b, cc, n);
#pragma unroll
          for (int m = 0; m < NC; ++m) {
            const unsigned long long q = (unsigned long long)(long long)rint(ldexp(gm[m] * wgt, e));
            if (binned) atomicAdd(&hist[m * kIgCap + li], q);
            else atomicAdd(&acc[(size_t)m * n3 + gi], q);
          }
        }
      }
    }
  }
  if (!binned) return;
  lds_barrier();
  for (int i = threadIdx.x; i < vol; i += 256) {
    const size_t gi = box_cell(i, cr, bx, n);
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const unsigned long long v = hist[m * kIgCap + i];
      if (v != 0ull) atomicAdd(&acc[(size_t)m * n3 + gi], v);
    }
  }
}

// in place: the fixed-point sums (int64 bit patterns) become doubles q 2^-e (NaN when *bad)
__global__ void __launch_bounds__(256)
k_fixed_to_double(unsigned long long* __restrict__ x, size_t count, const unsigned long long* __restrict__ st,
                  const int* __restrict__ bad) {
  const int e = (int)(long long)st[2];
  const bool nan_out = *bad != 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
    const double v = nan_out ? __builtin_nan("") : ldexp(double((long long)x[i]), -e);
    x[i] = (unsigned long long)__double_as_longlong(v);
  }
}

__global__ void __launch_bounds__(256) k_fill_zero(unsigned long long* __restrict__ x, size_t count) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) x[i] = 0ull;
}

__global__ void k_zero_flag(int* __restrict__ bad) {
  if (threadIdx.x == 0) *bad = 0;
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

void launch_deposit(int n, double box, const void* pos, int pos_fp32, long long np, long long* grid, int* bad,
                    hipStream_t s) {
  const double scale = double(n) / box;
  auto* out = reinterpret_cast<unsigned long long*>(grid);
  const bool big = n >= 512;   // chunk by mesh size (DepGeo)
  const int ch = big ? 2048 : 1024;
  const unsigned g = unsigned((np + ch - 1) / ch);
  const float* p32 = static_cast<const float*>(pos);
  const double* p64 = static_cast<const double*>(pos);
  if (pos_fp32 && big)
    hipLaunchKernelGGL((k_deposit_bin<float, 2048>), dim3(g), dim3(256), 0, s, p32, np, n, scale, out, bad);
  else if (pos_fp32)
    hipLaunchKernelGGL((k_deposit_bin<float, 1024>), dim3(g), dim3(256), 0, s, p32, np, n, scale, out, bad);
  else if (big)
    hipLaunchKernelGGL((k_deposit_bin<double, 2048>), dim3(g), dim3(256), 0, s, p64, np, n, scale, out, bad);
  else
    hipLaunchKernelGGL((k_deposit_bin<double, 1024>), dim3(g), dim3(256), 0, s, p64, np, n, scale, out, bad);
}

void launch_counts_to_delta(int n, const long long* grid, long long np, double* delta, const int* bad, hipStream_t s,
                            const double* mean_q) {
  const size_t n3 = (size_t)n * n * n;
  const double qscale = ldexp(double(n3) / double(np), -40);
  hipLaunchKernelGGL(k_counts_to_delta, dim3(grid_strided(n3)), dim3(256), 0, s, grid, n3, qscale, delta, bad, mean_q);
}

void launch_fill_zero(void* p, size_t words, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_strided(words)), dim3(256), 0, s, static_cast<unsigned long long*>(p),
                     words);
}


template <typename M, int NC>
static void interp_m(int n, double box, const M* mesh, const void* pos, int pos_fp32, long long np, double* out,
                     hipStream_t s) {
  const double scale = double(n) / box;
  if (pos_fp32)
    hipLaunchKernelGGL((k_interp<float, M, NC>), dim3(grid_for(np)), dim3(256), 0, s, mesh,
                       static_cast<const float*>(pos), np, n, scale, out);
  else
    hipLaunchKernelGGL((k_interp<double, M, NC>), dim3(grid_for(np)), dim3(256), 0, s, mesh,
                       static_cast<const double*>(pos), np, n, scale, out);
}

void launch_interp(int n, double box, const void* mesh, int mesh_fp32, int nc, const void* pos, int pos_fp32,
                   long long np, double* out, hipStream_t s) {
#define DGP_INTERP(NC)                                                                                        \
  if (mesh_fp32) interp_m<float, NC>(n, box, static_cast<const float*>(mesh), pos, pos_fp32, np, out, s);     \
  else interp_m<double, NC>(n, box, static_cast<const double*>(mesh), pos, pos_fp32, np, out, s);
  switch (nc) {
    case 1: DGP_INTERP(1) break;
    case 2: DGP_INTERP(2) break;
    default: DGP_INTERP(3) break;
  }
#undef DGP_INTERP
}

template <typename M>
static void kick_m(int n, double box, const M* mesh3, void* pos, void* vel, int fp32, long long np, double kick,
                   double drift, hipStream_t s) {
  const double scale = double(n) / box;
  const unsigned g = unsigned((np + kGatherChunk - 1) / kGatherChunk);
  if (fp32)
    hipLaunchKernelGGL((k_interp_kick_drift_bin<float, M>), dim3(g), dim3(256), 0, s, mesh3, static_cast<float*>(pos),
                       static_cast<float*>(vel), np, n, scale, box, kick, drift);
  else
    hipLaunchKernelGGL((k_interp_kick_drift_bin<double, M>), dim3(g), dim3(256), 0, s, mesh3,
                       static_cast<double*>(pos), static_cast<double*>(vel), np, n, scale, box, kick, drift);
}

void launch_interp_kick_drift(int n, double box, const void* mesh3, int mesh_fp32, void* pos, void* vel, int fp32,
                              long long np, double kick, double drift, hipStream_t s) {
  if (mesh_fp32)
    kick_m(n, box, static_cast<const float*>(mesh3), pos, vel, fp32, np, kick, drift, s);
  else
    kick_m(n, box, static_cast<const double*>(mesh3), pos, vel, fp32, np, kick, drift, s);
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

void launch_zero_flag(int* bad, hipStream_t s) { hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, s, bad); }

template <typename P, int NC>
static void interp_bwd_t(int n, double box, const double* mesh, const P* pos, long long np, const double* g,
                         double* grad_pos, double* grad_mesh, long long* grid, unsigned long long* st, int* bad,
                         hipStream_t s) {
  const double scale = double(n) / box;
  const size_t n3 = (size_t)n * n * n;
  if (grad_pos)
    hipLaunchKernelGGL((k_interp_grad_pos<P, NC>), dim3(grid_for(np)), dim3(256), 0, s, mesh, pos, np, n, scale, g,
                       grad_pos);
  if (!grad_mesh) return;
  auto* acc = reinterpret_cast<unsigned long long*>(grad_mesh);
  launch_fill_zero(acc, NC * n3, s);
  launch_fill_zero(grid, n3, s);
  hipLaunchKernelGGL(k_zero_scale_state, dim3(1), dim3(64), 0, s, st, bad);
  launch_deposit(n, box, pos, sizeof(P) == 4, np, grid, bad, s);
  hipLaunchKernelGGL(k_max_abs_and_mass, dim3(grid_strided(n3)), dim3(256), 0, s, g, (size_t)NC * np, grid, n3, st,
                     bad);
  hipLaunchKernelGGL(k_interp_scale, dim3(1), dim3(64), 0, s, st);
  const unsigned gch = unsigned((np + kIgChunk - 1) / kIgChunk);
  hipLaunchKernelGGL((k_interp_grad_mesh_bin<P, NC>), dim3(gch), dim3(256), 0, s, pos, np, n, scale, g, st, acc);
  hipLaunchKernelGGL(k_fixed_to_double, dim3(grid_strided(NC * n3)), dim3(256), 0, s, acc, NC * n3, st, bad);
}

void launch_interp_backward(int n, double box, const double* mesh, int nc, const void* pos, int pos_fp32, long long np,
                            const double* g, double* grad_pos, double* grad_mesh, long long* grid,
                            unsigned long long* st, int* bad, hipStream_t s) {
#define DGP_IB(P, NC) \
  interp_bwd_t<P, NC>(n, box, mesh, static_cast<const P*>(pos), np, g, grad_pos, grad_mesh, grid, st, bad, s)
  if (pos_fp32) {
    if (nc == 1) DGP_IB(float, 1);
    else if (nc == 2) DGP_IB(float, 2);
    else DGP_IB(float, 3);
  } else {
    if (nc == 1) DGP_IB(double, 1);
    else if (nc == 2) DGP_IB(double, 2);
    else DGP_IB(double, 3);
  }
#undef DGP_IB
}

// ------------------------------------------------------------------ allocation-free deposit scratch
// Device scratch of the allocation-free deposit entry point: the per-workgroup partial sums of the
// mean removal, the mean and the non-finite flag.  One copy per device, held until the process
// ends; every call on a device shares it, so calls that overlap on one device race.  Host code
// uses the per-device address from hipGetSymbolAddress, never the array's name.
constexpr size_t kNoallocScratchDoubles = 4096;   // 32 KiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

static void* g_noalloc_ptr[64];
static std::mutex g_noalloc_mu;

int noalloc_scratch(double** ptr, size_t* capacity) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (dev < 0 || dev >= 64) return -2;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {   // once per device, with that device current
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return -1;
    g_noalloc_ptr[dev] = p;
  }
  *ptr = static_cast<double*>(g_noalloc_ptr[dev]);
  *capacity = kNoallocScratchDoubles;
  return 0;
}

template <typename T>
void launch_convert(size_t count, const void* in, int in_fp32, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<T>), dim3(grid_strided(count)), dim3(256), 0, s, count, in, in_fp32, out);
}
template void launch_convert<double>(size_t, const void*, int, double*, hipStream_t);
template void launch_convert<float>(size_t, const void*, int, float*, hipStream_t);

}  // namespace dgp

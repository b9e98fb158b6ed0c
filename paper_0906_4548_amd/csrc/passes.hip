// Axis passes of the 3D real FFT on the periodic mesh, and the spectral multipliers.
//
// Layouts (C order, last index fastest):
//   real field      [batch][N][N][N]          index (i0, i1, i2)
//   spectrum        [batch][N/2+1][N][N]      complex, index (k0, k1, k2)
// The real-to-complex step runs along axis 0 (the slowest), so the half axis is
// k0 and every pass moves whole N x N planes: no odd-sized inner dimension.
//   axis-0 pass (p1): strided columns, two real columns packed as one complex
//                     transform (x_a + i x_b), separated with Hermitian symmetry;
//   axis-1 pass (p2): strided complex columns, tiles of 128-byte row segments;
//   axis-2 pass (p3): contiguous complex rows; forward transform, spectral
//                     multipliers, inverse transforms of every output.
// Forward transforms are unnormalised; the 1/N^3 of the inverse is folded into
// the spectral multipliers (numpy convention).
//
// Spectral conventions (the Fourier-space operators of Sec. II and III B):
//   k_d = kf * n_d with signed mode numbers n_d in [-N/2, N/2); kbar = kappa |k|;
//   k = 0 multipliers of 1/kbar, 1/k^2, k_i k_j / k^2 are 0; a multiplier odd in
//   component d (mixed Hessian terms, the gradient) is 0 at the Nyquist index of d.
#include "dgp_internal.h"

namespace dgp {

// radix plan and workgroup shapes of each pass, per element type and mesh size
#ifndef DGP_P3_WAVE_SYNC
#define DGP_P3_WAVE_SYNC 1
#endif
// Plan choice per pass and element type (0: 8 elements per thread, 1: up to 16,
// 2: 4), picked from measured pass times at 256^3 on gfx950.
#ifndef DGP_PLAN_P1
#define DGP_PLAN_P1 0
#endif
#ifndef DGP_PLAN_P2_F64
#define DGP_PLAN_P2_F64 1
#endif
#ifndef DGP_PLAN_P2_F32
#define DGP_PLAN_P2_F32 1
#endif
// Axis 2: radix 8 in both precisions, two LDS exchanges per transform instead of radix 4's three
// (the split Hessian pass, four transforms per row, is bound by them: 256^3 float32 66 -> 53 us,
// float64 95 -> 90 us); a row's transform stays inside one wavefront up to N = 512
#ifndef DGP_PLAN_P3_F64
#define DGP_PLAN_P3_F64 0
#endif
#ifndef DGP_PLAN_P3_F32
#define DGP_PLAN_P3_F32 0
#endif
// Column tile of the axis-0 passes: AxisTile, widened from N = 256 on, where the planes are
// 0.5-4 MB apart and the narrow tile's row segments per plane stream poorly (at 256^3 the
// float64 set-up, which also writes float32 copies, 465 -> 432 us; the float32 force mesh
// 347 -> 331 us; a float64-form step -70 us).
#ifndef DGP_P1_WIDE_MIN
#define DGP_P1_WIDE_MIN 256
#endif
template <typename T, int N, int R>
struct P1Tile {
  using A = AxisTile<T, N, R>;
  static constexpr int kTP =
      (N >= DGP_P1_WIDE_MIN && 2 * A::kTP * A::kT <= 1024 && 2 * A::kTP <= N / 2) ? 2 * A::kTP : A::kTP;
  static constexpr int kT = A::kT, kThreads = kTP * kT;
};

template <typename T, int N>
struct Geo {
  static constexpr bool kF32 = sizeof(T) == 4;
  using P = typename PlanPick<N, DGP_PLAN_P1>::type;
  using P2 = typename PlanPick<N, kF32 ? DGP_PLAN_P2_F32 : DGP_PLAN_P2_F64>::type;
  using P3 = typename PlanPick<N, kF32 ? DGP_PLAN_P3_F32 : DGP_PLAN_P3_F64>::type;
  static constexpr int R = P::R;
  static constexpr int kP1 = P1Tile<T, N, R>::kThreads;
  static constexpr int kP2 = ColTile<T, N, P2::R>::kThreads;
  static constexpr int kP3 = RowTile<N, P3::R>::kThreads;
};

__device__ __forceinline__ bool batch_done(const SolveCtl* ctl, int b) {
  return ctl != nullptr && ctl[b].done != 0;
}

// ------------------------------------------------------------------ axis 0, forward (real -> complex)
// I: element type of the real input (float64 input to a float32 transform is rounded on load)
template <typename T, int N, typename I = T>
__global__ void __launch_bounds__((Geo<T, N>::kP1))
k_p1_fwd(const I* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
         const SolveCtl* __restrict__ ctl) {
  using P = typename Geo<T, N>::P;
  constexpr int R = P::R;
  using G = P1Tile<T, N, R>;
  constexpr int TP = G::kTP, TT = G::kT, H = N / 2 + 1;
  const int b = blockIdx.z;
  if (batch_done(ctl, b)) return;
  int tile, i1;
  xcd_tile(tile, i1);
  const int c = threadIdx.x % TP, t = threadIdx.x / TP;
  const int i2 = (tile * TP + c) * 2;
  __shared__ cx<T> lds[N * TP];
  const I* src = in + (size_t)b * N * N * N + (size_t)i1 * N + i2;
  cx<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const cx<I> x = *reinterpret_cast<const cx<I>*>(src + (size_t)(t + q * TT) * N * N);
    v[q] = mk(T(x.x), T(x.y));
  }
  LdsCol<T, TP> L{lds, c};
  fft<T, N, P, -1>(v, tw, L, t);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) lds[(t + q * TT) * TP + c] = v[q];
  __syncthreads();
  cx<T>* dst = out + (size_t)b * H * N * N + (size_t)i1 * N + i2;
  for (int k = t; k < H; k += TT) {
    const cx<T> zk = lds[k * TP + c];
    const cx<T> zn = lds[((N - k) & (N - 1)) * TP + c];
    // x_a(k) = (Z(k) + conj Z(N-k)) / 2,  x_b(k) = (Z(k) - conj Z(N-k)) / (2i)
    const cx<T> xa = mk(T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y));
    const cx<T> xb = mk(T(0.5) * (zk.y + zn.y), T(0.5) * (zn.x - zk.x));
    store_stream(&dst[(size_t)k * N * N], xa);   // read by the next pass
    store_stream(&dst[(size_t)k * N * N + 1], xb);
  }
}

// ------------------------------------------------------------------ axis 0, inverse (complex -> real)
template <typename T, int N>
__global__ void __launch_bounds__((Geo<T, N>::kP1))
k_p1_inv(const cx<T>* __restrict__ in, T* __restrict__ out, const cx<T>* __restrict__ tw,
         const SolveCtl* __restrict__ ctl, float* __restrict__ out32) {
  using P = typename Geo<T, N>::P;
  constexpr int R = P::R;
  using G = P1Tile<T, N, R>;
  constexpr int TP = G::kTP, TT = G::kT, H = N / 2 + 1;
  constexpr int LSZ = (H * 2 * TP > N * TP) ? H * 2 * TP : N * TP;
  const int b = blockIdx.z;
  if (batch_done(ctl, b)) return;
  int tile, i1;
  xcd_tile(tile, i1);
  const int c = threadIdx.x % TP, t = threadIdx.x / TP;
  const int i2 = (tile * TP + c) * 2;
  __shared__ cx<T> lds[LSZ];
  const cx<T>* src = in + (size_t)b * H * N * N + (size_t)i1 * N + i2;
  for (int k = t; k < H; k += TT) {
    lds[k * 2 * TP + 2 * c] = src[(size_t)k * N * N];
    lds[k * 2 * TP + 2 * c + 1] = src[(size_t)k * N * N + 1];
  }
  __syncthreads();
  cx<T> v[R];
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
    v[q] = mk(xa.x - xb.y, xa.y + xb.x);   // x_a + i x_b
  }
  LdsCol<T, TP> L{lds, c};
  fft<T, N, P, +1>(v, tw, L, t);
  T* dst = out + (size_t)b * N * N * N + (size_t)i1 * N + i2;
#pragma unroll
  for (int q = 0; q < R; ++q) store_stream(reinterpret_cast<cx<T>*>(dst + (size_t)(t + q * TT) * N * N), v[q]);
  if (out32) {   // optional float32 rounding of the same output
    float* d32 = out32 + (size_t)b * N * N * N + (size_t)i1 * N + i2;
#pragma unroll
    for (int q = 0; q < R; ++q)
      *reinterpret_cast<float2*>(d32 + (size_t)(t + q * TT) * N * N) = make_float2(float(v[q].x), float(v[q].y));
  }
}

// ------------------------------------------------------------------ axis 1 (strided complex columns, in place)
template <typename T, int N, int DIR>
__global__ void __launch_bounds__((Geo<T, N>::kP2))
k_p2(cx<T>* __restrict__ data, int batch, const cx<T>* __restrict__ tw, const SolveCtl* __restrict__ ctl) {
  using P = typename Geo<T, N>::P2;
  constexpr int R = P::R;
  using G = ColTile<T, N, R>;
  constexpr int TY = G::kTY, TT = G::kT, H = N / 2 + 1;
  const int fb = blockIdx.z;
  if (batch_done(ctl, fb % batch)) return;
  const int k0 = blockIdx.y;
  const int c = threadIdx.x % TY, t = threadIdx.x / TY;
  __shared__ cx<T> lds[N * TY];
  cx<T>* base = data + ((size_t)fb * H + k0) * N * N + blockIdx.x * TY + c;
  cx<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = base[(size_t)(t + q * TT) * N];
  LdsCol<T, TY> L{lds, c};
  fft<T, N, P, DIR>(v, tw, L, t);
#pragma unroll
  for (int q = 0; q < R; ++q) base[(size_t)(t + q * TT) * N] = v[q];
}

// Axis-1 inverse pass of the split Hessian.  The axis-2 pass wrote C' = u/|n|^2 to slot 0, i n2 C'
// to slot 3 and the nonlocal term to slot 5; k0 is fixed per workgroup here, so this pass applies
// both remaining factors (axis 1 and axis 0) of each Hessian multiplier n_i n_j / |n|^2:
//   slot 0 -> 0 (h00: n0^2), 1 (h11: n1^2), 2 (h01: n0 n1);
//   slot 3 -> 3 (h02: -i n0), 4 (h12: -i n1);  slot 5 -> 5 (1);
// a factor odd in n_d is 0 at the Nyquist index of d.
// Plans of the split pass: the input tile is held in registers across the outputs, so the float64
// pass takes radix 8 (fewer registers per thread than the axis-1 pass's radix 16; measured at
// 256^3 on gfx950: 229 vs 246 us per launch, float32 keeps radix 16: 116 vs 129 us)
#ifndef DGP_PLAN_P2S_F64
#define DGP_PLAN_P2S_F64 0
#endif
#ifndef DGP_PLAN_P2S_F32
#define DGP_PLAN_P2S_F32 DGP_PLAN_P2_F32
#endif
// Cache policy of the split Hessian passes (1: nontemporal), per element type, from measured
// pass times at 256^3 and 512^3 on gfx950.  Float32: the axis-2 pass's three outputs (203 MB at
// 256^3) are stored through the 256 MB last-level cache, where the axis-1 split pass, which reads
// each of them once (streaming), finds part of them; float64 (405 MB) streams both ways.  The
// split pass streams its six outputs, which only the relaxation kernel reads.
#ifndef DGP_HSPLIT_STREAM_STORE_F32
#define DGP_HSPLIT_STREAM_STORE_F32 0
#endif
#ifndef DGP_HSPLIT_STREAM_STORE_F64
#define DGP_HSPLIT_STREAM_STORE_F64 1
#endif
#ifndef DGP_P2S_STREAM_LOAD_F32
#define DGP_P2S_STREAM_LOAD_F32 1
#endif
#ifndef DGP_P2S_STREAM_LOAD_F64
#define DGP_P2S_STREAM_LOAD_F64 0
#endif
#ifndef DGP_P2S_STREAM_STORE
#define DGP_P2S_STREAM_STORE 1
#endif
template <typename T, int N>
struct P2SGeo {
  using P = typename PlanPick<N, sizeof(T) == 4 ? DGP_PLAN_P2S_F32 : DGP_PLAN_P2S_F64>::type;
  using G = ColTile<T, N, P::R>;
};

// factor of output o (0..2 - role) of input slot role (0, 1, 2) at axis-1 index k1
template <typename T, int N>
__device__ __forceinline__ cx<T> p2s_factor(int role, int o, T n0, bool q0, int k1, cx<T> x) {
  const T n1 = T(k1 < N / 2 ? k1 : k1 - N);
  const bool q1 = k1 == N / 2;
  if (role == 0) {   // real factors
    const T m = o == 0 ? n0 * n0 : o == 1 ? n1 * n1 : (q0 || q1) ? T(0) : n0 * n1;
    return scale(x, m);
  } else if (role == 1) {   // -i n0, -i n1
    const T m = o == 0 ? (q0 ? T(0) : n0) : (q1 ? T(0) : n1);
    return mk(m * x.y, -m * x.x);
  }
  return x;
}

// A workgroup takes one column tile of one input slot, holds it in registers and writes every
// output that derives from it (blockIdx.z = role * batch + element, so the three-output tiles are
// dispatched first); the tile is read whole before the first store, so output slot + 0 can
// overwrite it (no other workgroup touches its columns).  The twiddle pointer and the lane index are made opaque per output, so that twiddles, row addresses
// and factors are not held across the output loop.  (Re-reading the tile from cache for each output
// instead of holding it measured 470 vs 229 us per float64 launch at 256^3.)
template <typename T, int N>
__global__ void __launch_bounds__((P2SGeo<T, N>::G::kThreads))
k_p2_split(cx<T>* __restrict__ data, size_t fstride, int batch, const cx<T>* __restrict__ tw,
           const SolveCtl* __restrict__ ctl) {
  using P = typename P2SGeo<T, N>::P;
  constexpr int R = P::R;
  using G = typename P2SGeo<T, N>::G;
  constexpr int TY = G::kTY, TT = G::kT, H = N / 2 + 1;
  const int role = blockIdx.z / batch, b = blockIdx.z % batch;
  if (batch_done(ctl, b)) return;
  const int k0 = blockIdx.y;
  const int c = threadIdx.x % TY;
  int t = threadIdx.x / TY;
  __shared__ cx<T> lds[N * TY];
  const int slot = role == 0 ? 0 : role == 1 ? 3 : 5;
  const size_t off = ((size_t)b * H + k0) * N * N + blockIdx.x * TY + c;
  const cx<T>* src = data + slot * fstride + off;
  const T n0 = T(k0);
  const bool q0 = k0 == N / 2;
  LdsCol<T, TY> L{lds, c};
  cx<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if constexpr (sizeof(T) == 4 ? DGP_P2S_STREAM_LOAD_F32 : DGP_P2S_STREAM_LOAD_F64)
      v[q] = load_stream(&src[(size_t)(t + q * TT) * N]);
    else v[q] = src[(size_t)(t + q * TT) * N];
  }
#pragma unroll 1
  for (int o = 2 - role; o >= 0; --o) {
    const cx<T>* twq = tw;
    asm volatile("" : "+s"(twq), "+v"(t));
    cx<T> w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      w[q] = p2s_factor<T, N>(role, o, n0, q0, t + q * TT, v[q]);
    }
    fft<T, N, P, +1>(w, twq, L, t);
    cx<T>* dst = data + (slot + o) * fstride + off;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if constexpr (DGP_P2S_STREAM_STORE) store_stream(&dst[(size_t)(t + q * TT) * N], w[q]);
      else dst[(size_t)(t + q * TT) * N] = w[q];
    }
  }
}

// Transposed split for the implicit adjoint's combine (float64): forward axis-1 transform of the
// six product spectra (axis-0 transformed by the adjoint step), each times the axis-1 and axis-0
// factors of its Hessian multiplier and its weight (2 lam on the diagonal terms, 4 lam on the
// off-diagonal ones: the pair ij and ji), summed per group into slots 0, 3 and 5:
//   0 <- 2 lam (n0^2 f0 + n1^2 f1 + 2 n0 n1 f2);  3 <- 4 lam (n0 f3 + n1 f4);  5 <- f5;
// a factor odd in n_d is 0 at the Nyquist index of d.  SPEC_ADJ_COMBINE3 applies the rest
// (1/|n|^2, n2/|n|^2, gamma/kbar).  A workgroup takes one column tile of one group; the sum is
// stored over the group's first input after every input tile has been read.
template <int N>
__global__ void __launch_bounds__((P2SGeo<double, N>::G::kThreads))
k_p2_adj_split(cx<double>* __restrict__ data, size_t fstride, int batch, double lam2,
               const cx<double>* __restrict__ tw, const SolveCtl* __restrict__ ctl) {
  using T = double;
  using P = typename P2SGeo<T, N>::P;
  constexpr int R = P::R;
  using G = typename P2SGeo<T, N>::G;
  constexpr int TY = G::kTY, TT = G::kT, H = N / 2 + 1;
  const int role = blockIdx.z / batch, b = blockIdx.z % batch;
  if (batch_done(ctl, b)) return;
  const int k0 = blockIdx.y;
  const int c = threadIdx.x % TY;
  int t = threadIdx.x / TY;
  __shared__ cx<T> lds[N * TY];
  const int slot = role == 0 ? 0 : role == 1 ? 3 : 5;
  const size_t off = ((size_t)b * H + k0) * N * N + blockIdx.x * TY + c;
  const T n0 = T(k0);
  const bool q0 = k0 == N / 2;
  LdsCol<T, TY> L{lds, c};
  cx<T> acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = mk(T(0), T(0));
#pragma unroll 1
  for (int i = 0; i < 3 - role; ++i) {
    const cx<T>* twq = tw;
    asm volatile("" : "+s"(twq), "+v"(t));
    const int f = slot + i;
    const cx<T>* src = data + f * fstride + off;
    cx<T> v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[(size_t)(t + q * TT) * N];
    fft<T, N, P, -1>(v, twq, L, t);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k1 = t + q * TT;
      const T n1 = T(k1 < N / 2 ? k1 : k1 - N);
      const bool q1 = k1 == N / 2;
      T m;
      if (f == 0) m = lam2 * n0 * n0;
      else if (f == 1) m = lam2 * n1 * n1;
      else if (f == 2) m = (q0 || q1) ? T(0) : T(2) * lam2 * n0 * n1;
      else if (f == 3) m = q0 ? T(0) : T(2) * lam2 * n0;
      else if (f == 4) m = q1 ? T(0) : T(2) * lam2 * n1;
      else m = T(1);
      acc[q] = acc[q] + scale(v[q], m);
    }
  }
  cx<T>* dst = data + slot * fstride + off;
#pragma unroll
  for (int q = 0; q < R; ++q) dst[(size_t)(t + q * TT) * N] = acc[q];
}

// Axis-1 inverse pass of the force mesh: the axis-2 pass wrote phi to slot 0 and g2 to slot 2;
// k0 is fixed per workgroup, so this pass forms g0 = -(c/H0)^2 (i k0) phi into slot 0 and
// g1 = -(c/H0)^2 (i k1) phi into slot 1 (k_d = 0 at the Nyquist index of d), phi itself into slot 3
// when asked for, and inverts g2 in place.  Role 0 holds its phi tile in registers across its
// outputs (written in descending slots, the in-place one last); role 1 is a plain inverse.
template <typename T, int N>
__global__ void __launch_bounds__((P2SGeo<T, N>::G::kThreads))
k_p2_force_split(cx<T>* __restrict__ data, size_t fstride, int batch, int with_phi, double fk,
                 const cx<T>* __restrict__ tw) {
  using P = typename P2SGeo<T, N>::P;
  constexpr int R = P::R;
  using G = typename P2SGeo<T, N>::G;
  constexpr int TY = G::kTY, TT = G::kT, H = N / 2 + 1;
  const int role = blockIdx.z / batch, b = blockIdx.z % batch;
  const int k0 = blockIdx.y;
  const int c = threadIdx.x % TY;
  int t = threadIdx.x / TY;
  __shared__ cx<T> lds[N * TY];
  const int slot = role == 0 ? 0 : 2;
  const size_t off = ((size_t)b * H + k0) * N * N + blockIdx.x * TY + c;
  const cx<T>* src = data + slot * fstride + off;
  const T f0 = k0 == N / 2 ? T(0) : T(fk * double(k0));   // (c/H0)^2 k0
  LdsCol<T, TY> L{lds, c};
  cx<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = src[(size_t)(t + q * TT) * N];
  // outputs of role 0: o = 2 phi (slot 3, when asked for), 1 g1 (slot 1), 0 g0 (slot 0)
#pragma unroll 1
  for (int o = role == 0 ? (with_phi ? 2 : 1) : 0; o >= 0; --o) {
    const cx<T>* twq = tw;
    asm volatile("" : "+s"(twq), "+v"(t));
    cx<T> w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k1 = t + q * TT;
      T f = T(0);
      if (role == 0 && o == 0) f = f0;
      else if (role == 0 && o == 1) f = k1 == N / 2 ? T(0) : T(fk * double(k1 < N / 2 ? k1 : k1 - N));
      w[q] = (role == 1 || o == 2) ? v[q] : mk(f * v[q].y, -f * v[q].x);
    }
    fft<T, N, P, +1>(w, twq, L, t);
    cx<T>* dst = data + (role == 1 ? 2 : o == 2 ? 3 : o) * fstride + off;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[(size_t)(t + q * TT) * N] = w[q];
  }
}

// ------------------------------------------------------------------ axis 2 with spectral multipliers
struct Mode3 {
  int n0, n1, n2;        // signed mode numbers (n0 >= 0 on the half axis)
  bool q0, q1, q2;       // Nyquist flags
  long long msq;         // |n|^2
};

__device__ __forceinline__ Mode3 mode_of(int N, int k0, int k1, int k2) {
  Mode3 m;
  m.n0 = k0;
  m.n1 = (k1 < N / 2) ? k1 : k1 - N;
  m.n2 = (k2 < N / 2) ? k2 : k2 - N;
  m.q0 = (k0 == N / 2);
  m.q1 = (k1 == N / 2);
  m.q2 = (k2 == N / 2);
  m.msq = (long long)m.n0 * m.n0 + (long long)m.n1 * m.n1 + (long long)m.n2 * m.n2;
  return m;
}

template <typename T, int N, SpecMode MODE>
__global__ void __launch_bounds__((Geo<T, N>::kP3))
k_p3(const cx<T>* __restrict__ in, size_t in_stride, cx<T>* __restrict__ out, size_t out_stride,
     const cx<T>* __restrict__ tw, SpecCoef cf, const double* __restrict__ bin_coef,
     double* __restrict__ bin_partial, double* __restrict__ mean_out, const SolveCtl* __restrict__ ctl) {
  using P = typename Geo<T, N>::P3;
  constexpr int R = P::R;
  using G = RowTile<N, R>;
  constexpr int RW = G::kRW, TT = G::kT, H = N / 2 + 1;
  constexpr int ROWS = H * N;
  const int b = blockIdx.y;
  if (batch_done(ctl, b)) return;
  const int t = threadIdx.x % TT, c = threadIdx.x / TT;
  const int row = blockIdx.x * RW + c;
  const bool valid = row < ROWS;
  const int rr = valid ? row : 0;
  const int k0 = rr / N, k1 = rr % N;
  __shared__ cx<T> lds[RW * LdsRow<T, N>::kStride];
  // a row's N/R threads are consecutive lanes; when they fit in one wavefront its exchanges are wave-local
  LdsRow<T, N, (TT <= 64 && 64 % TT == 0 && DGP_P3_WAVE_SYNC)> L{lds, c};
  const size_t roff = (size_t)b * ROWS * N + (size_t)rr * N;

  cx<T> v[R];
  auto load_row = [&](const cx<T>* src) {
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = valid ? src[roff + t + q * TT] : mk(T(0), T(0));
  };
  auto store_row = [&](cx<T>* dst, cx<T> (&w)[R]) {
    if (valid) {
#pragma unroll
      for (int q = 0; q < R; ++q) store_stream(&dst[roff + t + q * TT], w[q]);   // read by the next pass
    }
  };
  const double kf = cf.kf;

  if constexpr (MODE == SPEC_FWD_ONLY || MODE == SPEC_INV_ONLY) {
    load_row(in);
    if constexpr (MODE == SPEC_FWD_ONLY) {
      fft<T, N, P, -1>(v, tw, L, t);
    } else {
      fft<T, N, P, +1>(v, tw, L, t);
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = scale(v[q], T(cf.inv_n3));
    }
    store_row(out, v);
    return;
  } else if constexpr (MODE == SPEC_POWER) {
    // deterministic binning: every mode's (bin, weighted |f|^2) goes to LDS, then thread b sums
    // bin b over the workgroup's modes in a fixed order
    constexpr int NE = G::kThreads * R;
    __shared__ double pval[NE];
    __shared__ short pbin[NE];
    load_row(in);
    fft<T, N, P, -1>(v, tw, L, t);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int slot = (c * R + q) * TT + t;
      short bin = -1;
      double val = 0.0;
      if (valid) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        const double ms = double(m.msq);
        if (ms >= bin_coef[0] && ms < bin_coef[cf.nbins]) {
          int lo = 0, hi = cf.nbins;   // largest lo with thr[lo] <= ms
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bin_coef[mid] <= ms) lo = mid; else hi = mid;
          }
          const double mult = (m.n0 == 0 || m.q0) ? 1.0 : 2.0;
          double p2 = double(v[q].x) * double(v[q].x) + double(v[q].y) * double(v[q].y);
          if (cf.power_c) {
            const double kb2 = cf.kappa * cf.kappa * kf * kf * ms;
            p2 /= kb2 * kb2;
          }
          bin = short(lo);
          val = mult * p2;
        }
      }
      pval[slot] = val;
      pbin[slot] = bin;
    }
    __syncthreads();
    double* dstp = bin_partial + ((size_t)b * gridDim.x + blockIdx.x) * 2 * cf.nbins;
    for (int bb = threadIdx.x; bb < cf.nbins; bb += blockDim.x) {
      double sum = 0.0, cnt = 0.0;
      for (int i = 0; i < NE; ++i) {
        if (pbin[i] == bb) {
          sum += pval[i];
          const int kk0 = (blockIdx.x * RW + i / (TT * R)) / N;   // plane of the mode's row
          cnt += (kk0 == 0 || kk0 == N / 2) ? 1.0 : 2.0;
        }
      }
      dstp[bb] = sum;
      dstp[cf.nbins + bb] = cnt;
    }
    return;
  } else if constexpr (MODE == SPEC_ADJ_COMBINE3) {
    // the three group sums of k_p2_adj_split (slots 0, 3, 5: the axis-1 and axis-0 factors and
    // the 2 lam weights applied) times the rest of each multiplier: 1/|n|^2, n2/|n|^2 (0 at the
    // Nyquist index of axis 2) and gamma/kbar
    cx<T> acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = mk(T(0), T(0));
#pragma unroll 1
    for (int g = 0; g < 3; ++g) {
      load_row(in + (g == 0 ? 0 : g == 1 ? 3 : 5) * in_stride);
      fft<T, N, P, -1>(v, tw, L, t);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        if (m.msq == 0) continue;
        const double ik2 = 1.0 / double(m.msq);
        double mult;
        if (g == 0) mult = ik2;
        else if (g == 1) mult = m.q2 ? 0.0 : double(m.n2) * ik2;
        else mult = cf.gamma / (cf.kappa * kf * sqrt(double(m.msq)));
        const T mm = T(mult * cf.inv_n3);
        acc[q] = acc[q] + scale(v[q], mm);
      }
    }
    fft<T, N, P, +1>(acc, tw, L, t);
    store_row(out, acc);
    return;
  } else {
    // single-input or two-input modes
    load_row(in);
    fft<T, N, P, -1>(v, tw, L, t);
    cx<T> v2[(MODE == SPEC_FORCES) ? R : 1];
    if constexpr (MODE == SPEC_FORCES) {
      if (cf.force_mode == FORCE_NLDGP) {
        cx<T> keep[R];
#pragma unroll
        for (int q = 0; q < R; ++q) keep[q] = v[q];
        load_row(in + in_stride);
        fft<T, N, P, -1>(v, tw, L, t);
#pragma unroll
        for (int q = 0; q < R; ++q) { v2[q] = v[q]; v[q] = keep[q]; }
      }
    }
    if constexpr (MODE == SPEC_HSPLIT) {
      if (valid && k0 == 0 && k1 == 0 && t == 0 && mean_out != nullptr) mean_out[b] = double(v[0].x) * cf.inv_n3;
    }
    if constexpr (MODE == SPEC_HSPLIT) {
      // The Hessian multipliers n_i n_j / |n|^2 factor as (1/|n|^2) times one factor per axis:
      // this pass applies 1/|n|^2 and the axis-2 factor i n2 (0 at the Nyquist index), the axis-1
      // pass (k_p2_split) the axis-1 and axis-0 factors.  Per mode: ic = 1/(N^3 |n|^2) and
      // ib = -1/(N^3 kappa kf |n|), both 0 at n = 0; float32 fields form them in float32
      // (reciprocal and reciprocal-sqrt estimates, the reciprocal refined by one Newton step).
      T ic[R], ib[R], a2[R];
      const float in3f = float(cf.inv_n3), ikbs = float(cf.inv_n3 / (cf.kappa * kf));
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        const bool nz = m.msq != 0;
        if constexpr (sizeof(T) == 4) {
          const float ms = float(m.msq);
          float r = __builtin_amdgcn_rcpf(ms);
          r = r * (2.0f - ms * r);
          ic[q] = nz ? r * in3f : 0.0f;
          ib[q] = nz ? -__builtin_amdgcn_rsqf(ms) * ikbs : 0.0f;
        } else {
          const double ms = double(m.msq);
          ic[q] = nz ? cf.inv_n3 / ms : 0.0;
          ib[q] = nz ? -cf.inv_n3 / (cf.kappa * kf * sqrt(ms)) : 0.0;
        }
        a2[q] = m.q2 ? T(0) : T(m.n2);
      }
#pragma unroll 1
      for (int o = 0; o < 3; ++o) {
        cx<T> w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (o == 0) {
            w[q] = scale(v[q], ic[q]);
          } else if (o == 1) {   // i n2 C'
            const T mq = a2[q] * ic[q];
            w[q] = mk(-mq * v[q].y, mq * v[q].x);
          } else {
            w[q] = scale(v[q], ib[q]);
          }
        }
        fft<T, N, P, +1>(w, tw, L, t);
        cx<T>* dsto = out + (o == 0 ? 0 : o == 1 ? 3 : 5) * out_stride;
        if constexpr (sizeof(T) == 4 ? DGP_HSPLIT_STREAM_STORE_F32 : DGP_HSPLIT_STREAM_STORE_F64) {
          store_row(dsto, w);
        } else if (valid) {
#pragma unroll
          for (int q = 0; q < R; ++q) dsto[roff + t + q * TT] = w[q];
        }
      }
      return;
    }
    if constexpr (MODE == SPEC_FORCES) {
      // phi(k) once per mode, times 1/N^3 (0 at k = 0); the force g_d = -(c/H0)^2 (i k_d) phi with
      // k_d = 0 at the Nyquist index of d
      cx<T> ph[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        ph[q] = mk(T(0), T(0));
        if (m.msq != 0) {
          const double ms = double(m.msq);
          const double kb = cf.kappa * kf * sqrt(ms);
          const double ikb = 1.0 / kb;
          // phi(k) from the modified Poisson equation (or its linear / GR forms)
          const double dr = double(v[q].x), di = double(v[q].y);
          double nr, ni, den;
          if (cf.force_mode == FORCE_GRH || cf.force_mode == FORCE_GR) {   // Eq. GRPoisson (kappa, om15 of the run's background)
            nr = cf.om15 * dr; ni = cf.om15 * di; den = kb * kb;
          } else {
            double ur, ui;
            if (cf.force_mode == FORCE_NLDGP) {
              ur = double(v2[q].x); ui = double(v2[q].y);
            } else {   // linear solution from delta
              const double sl = cf.A * (1.0 - cf.beta * ikb) / (cf.alpha - cf.gamma * ikb);
              ur = sl * dr; ui = sl * di;
            }
            const double cu = -cf.inv2eta + cf.c2 * ikb;
            nr = cf.om15 * dr + cu * ur;
            ni = cf.om15 * di + cu * ui;
            den = kb * kb + kb * cf.inv_eta_nl;
          }
          ph[q] = mk(T(-nr / den * cf.inv_n3), T(-ni / den * cf.inv_n3));
        }
      }
      // two outputs: phi (slot 0; the axis-1 pass k_p2_force_split forms g0, g1 and phi from it)
      // and g2 (slot 2), the gradient factor being a product of per-axis factors
#pragma unroll 1
      for (int o = 0; o < 2; ++o) {
        cx<T> w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (o == 0) {
            w[q] = ph[q];
          } else {
            const Mode3 m = mode_of(N, k0, k1, t + q * TT);
            const T f = m.q2 ? T(0) : T(cf.force_scale * kf * double(m.n2));   // (c/H0)^2 k_2
            w[q] = mk(f * ph[q].y, -f * ph[q].x);
          }
        }
        fft<T, N, P, +1>(w, tw, L, t);
        store_row(out + 2 * o * out_stride, w);
      }
      return;
    }
    if constexpr (MODE == SPEC_SOURCE) {
      // the two multipliers once per mode, times 1/N^3 (0 at k = 0): S = A (1 - beta/kbar) delta
      // and the linear solution S / (alpha - gamma/kbar)
      T m0[R], m1[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        m0[q] = T(0);
        m1[q] = T(0);
        if (m.msq != 0) {
          const double ikb = 1.0 / (cf.kappa * kf * sqrt(double(m.msq)));
          const double sv = cf.A * (1.0 - cf.beta * ikb);
          m0[q] = T(sv * cf.inv_n3);
          m1[q] = T(sv / (cf.alpha - cf.gamma * ikb) * cf.inv_n3);
        }
      }
#pragma unroll 1
      for (int o = 0; o < 2; ++o) {
        cx<T> w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) w[q] = scale(v[q], o ? m1[q] : m0[q]);
        fft<T, N, P, +1>(w, tw, L, t);
        store_row(out + o * out_stride, w);
      }
      return;
    }
    constexpr int NOUT = 1;
#pragma unroll 1
    for (int o = 0; o < NOUT; ++o) {
      cx<T> w[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Mode3 m = mode_of(N, k0, k1, t + q * TT);
        const double ms = double(m.msq);
        cx<T> res = mk(T(0), T(0));
        if (m.msq != 0) {
          const double ik2 = 1.0 / ms;
          const double kb = cf.kappa * kf * sqrt(ms);
          const double ikb = 1.0 / kb;
          if constexpr (MODE == SPEC_CFIELD) {
            res = scale(v[q], T(-ikb * ikb * cf.inv_n3));
          } else if constexpr (MODE == SPEC_COPY) {
            res = scale(v[q], T(cf.inv_n3));
          } else if constexpr (MODE == SPEC_POWER_GRAD) {
            double coef = 0.0;
            const double* thr = bin_coef;
            if (ms >= thr[0] && ms < thr[cf.nbins]) {
              int lo = 0, hi = cf.nbins;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (thr[mid] <= ms) lo = mid; else hi = mid;
              }
              coef = thr[cf.nbins + 1 + (size_t)b * cf.nbins + lo];
              if (cf.power_c) coef *= (ikb * ikb) * (ikb * ikb);
            }
            res = scale(v[q], T(coef * cf.inv_n3));
          }
        }
        w[q] = res;
      }
      fft<T, N, P, +1>(w, tw, L, t);
      store_row(out + o * out_stride, w);
    }
  }
}

// ------------------------------------------------------------------ launchers
template <typename T, int N, typename I = T>
static void p1_fwd_n(const I* in, cx<T>* out, int batch, const SolveCtl* ctl, const cx<T>* tw, hipStream_t s) {
  using G = P1Tile<T, N, Geo<T, N>::R>;
  dim3 grid(N / (2 * G::kTP), N, batch);
  hipLaunchKernelGGL((k_p1_fwd<T, N, I>), grid, dim3(G::kThreads), 0, s, in, out, tw, ctl);
}
template <typename T, int N>
static void p1_inv_n(const cx<T>* in, T* out, int batch, const SolveCtl* ctl, const cx<T>* tw, float* out32,
                     hipStream_t s) {
  using G = P1Tile<T, N, Geo<T, N>::R>;
  dim3 grid(N / (2 * G::kTP), N, batch);
  hipLaunchKernelGGL((k_p1_inv<T, N>), grid, dim3(G::kThreads), 0, s, in, out, tw, ctl, out32);
}
template <typename T, int N>
static void p2_n(cx<T>* data, int nf, int batch, int dir, const SolveCtl* ctl, const cx<T>* tw, hipStream_t s) {
  using G = ColTile<T, N, Geo<T, N>::P2::R>;
  dim3 grid(N / G::kTY, N / 2 + 1, nf * batch);
  if (dir < 0) hipLaunchKernelGGL((k_p2<T, N, -1>), grid, dim3(G::kThreads), 0, s, data, batch, tw, ctl);
  else hipLaunchKernelGGL((k_p2<T, N, +1>), grid, dim3(G::kThreads), 0, s, data, batch, tw, ctl);
}
template <typename T, int N>
static void p2_split_n(cx<T>* data, size_t fstride, int batch, const SolveCtl* ctl, const cx<T>* tw, hipStream_t s) {
  using G = typename P2SGeo<T, N>::G;
  dim3 grid(N / G::kTY, N / 2 + 1, 3 * batch);
  hipLaunchKernelGGL((k_p2_split<T, N>), grid, dim3(G::kThreads), 0, s, data, fstride, batch, tw, ctl);
}
template <int N>
static void p2_adj_split_n(cx<double>* data, size_t fstride, int batch, double lam2, const SolveCtl* ctl,
                           const cx<double>* tw, hipStream_t s) {
  using G = typename P2SGeo<double, N>::G;
  dim3 grid(N / G::kTY, N / 2 + 1, 3 * batch);
  hipLaunchKernelGGL((k_p2_adj_split<N>), grid, dim3(G::kThreads), 0, s, data, fstride, batch, lam2, tw, ctl);
}
template <typename T, int N>
static void p2_force_split_n(cx<T>* data, size_t fstride, int batch, int with_phi, double fk, const cx<T>* tw,
                             hipStream_t s) {
  using G = typename P2SGeo<T, N>::G;
  dim3 grid(N / G::kTY, N / 2 + 1, 2 * batch);
  hipLaunchKernelGGL((k_p2_force_split<T, N>), grid, dim3(G::kThreads), 0, s, data, fstride, batch, with_phi, fk, tw);
}
template <typename T, int N>
static void p3_n(SpecMode mode, const cx<T>* in, size_t is, cx<T>* out, size_t os, int batch, const SpecCoef& cf,
                 const double* bc, double* bp, double* mean, const SolveCtl* ctl, const cx<T>* tw, hipStream_t s) {
  using G = RowTile<N, Geo<T, N>::P3::R>;
  constexpr int ROWS = (N / 2 + 1) * N;
  dim3 grid((ROWS + G::kRW - 1) / G::kRW, batch);
  dim3 blk(G::kThreads);
#define DGP_P3(M) hipLaunchKernelGGL((k_p3<T, N, M>), grid, blk, 0, s, in, is, out, os, tw, cf, bc, bp, mean, ctl)
  switch (mode) {
    case SPEC_SOURCE: DGP_P3(SPEC_SOURCE); break;
    case SPEC_CFIELD: DGP_P3(SPEC_CFIELD); break;
    case SPEC_FORCES: DGP_P3(SPEC_FORCES); break;
    case SPEC_POWER: DGP_P3(SPEC_POWER); break;
    case SPEC_POWER_GRAD: DGP_P3(SPEC_POWER_GRAD); break;
    case SPEC_ADJ_COMBINE3: DGP_P3(SPEC_ADJ_COMBINE3); break;
    case SPEC_COPY: DGP_P3(SPEC_COPY); break;
    case SPEC_FWD_ONLY: DGP_P3(SPEC_FWD_ONLY); break;
    case SPEC_INV_ONLY: DGP_P3(SPEC_INV_ONLY); break;
    case SPEC_HSPLIT: DGP_P3(SPEC_HSPLIT); break;
  }
#undef DGP_P3
}

template <typename T>
const cx<T>* twiddles(int n);   // defined in api.cpp: device table exp(-2 pi i m / n)

#define DGP_DISPATCH_N(n, CALL)        \
  switch (n) {                         \
    case 8: CALL(8); break;            \
    case 16: CALL(16); break;          \
    case 32: CALL(32); break;          \
    case 64: CALL(64); break;          \
    case 128: CALL(128); break;        \
    case 256: CALL(256); break;        \
    case 512: CALL(512); break;        \
    default: break;                    \
  }

template <typename T>
void launch_p1_fwd(int n, const T* in, cx<T>* out, int batch, const SolveCtl* ctl, hipStream_t s) {
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p1_fwd_n<T, NN>(in, out, batch, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
void launch_p1_fwd_from64(int n, const double* in, cx<float>* out, int batch, const SolveCtl* ctl, hipStream_t s) {
  const cx<float>* tw = twiddles<float>(n);
#define C(NN) p1_fwd_n<float, NN, double>(in, out, batch, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
template <typename T>
void launch_p1_inv(int n, const cx<T>* in, T* out, int batch, const SolveCtl* ctl, hipStream_t s, float* out32) {
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p1_inv_n<T, NN>(in, out, batch, ctl, tw, out32, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
template <typename T>
void launch_p2(int n, cx<T>* data, int nf, int batch, int dir, const SolveCtl* ctl, hipStream_t s) {
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p2_n<T, NN>(data, nf, batch, dir, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
template <typename T>
void launch_p2_split(int n, cx<T>* data, size_t fstride, int batch, const SolveCtl* ctl, hipStream_t s) {
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p2_split_n<T, NN>(data, fstride, batch, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
void launch_p2_adj_split(int n, cx<double>* data, size_t fstride, int batch, double lam2, const SolveCtl* ctl,
                         hipStream_t s) {
  const cx<double>* tw = twiddles<double>(n);
#define C(NN) p2_adj_split_n<NN>(data, fstride, batch, lam2, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
template <typename T>
void launch_p2_force_split(int n, cx<T>* data, size_t fstride, int batch, int with_phi, double fk, hipStream_t s) {
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p2_force_split_n<T, NN>(data, fstride, batch, with_phi, fk, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}
template <typename T>
void launch_p3(int n, SpecMode mode, const cx<T>* in, size_t in_stride, int nin, cx<T>* out, size_t out_stride,
               int nout, int batch, const SpecCoef& coef, const double* bin_coef, double* bin_partial,
               double* mean_out, const SolveCtl* ctl, hipStream_t s) {
  (void)nin;
  (void)nout;
  const cx<T>* tw = twiddles<T>(n);
#define C(NN) p3_n<T, NN>(mode, in, in_stride, out, out_stride, batch, coef, bin_coef, bin_partial, mean_out, ctl, tw, s)
  DGP_DISPATCH_N(n, C)
#undef C
}

int p3_row_groups(int n) {   // row groups of the float64 axis-2 pass (the P(k) binning uses it)
  int r = 0;
#define C(NN)                                                          \
  {                                                                    \
    using G = RowTile<NN, Geo<double, NN>::P3::R>;                     \
    r = ((NN / 2 + 1) * NN + G::kRW - 1) / G::kRW;                     \
  }
  DGP_DISPATCH_N(n, C)
#undef C
  return r;
}

template void launch_p1_fwd<double>(int, const double*, cx<double>*, int, const SolveCtl*, hipStream_t);
template void launch_p1_fwd<float>(int, const float*, cx<float>*, int, const SolveCtl*, hipStream_t);
template void launch_p1_inv<double>(int, const cx<double>*, double*, int, const SolveCtl*, hipStream_t, float*);
template void launch_p1_inv<float>(int, const cx<float>*, float*, int, const SolveCtl*, hipStream_t, float*);
template void launch_p2<double>(int, cx<double>*, int, int, int, const SolveCtl*, hipStream_t);
template void launch_p2<float>(int, cx<float>*, int, int, int, const SolveCtl*, hipStream_t);
template void launch_p2_split<double>(int, cx<double>*, size_t, int, const SolveCtl*, hipStream_t);
template void launch_p2_split<float>(int, cx<float>*, size_t, int, const SolveCtl*, hipStream_t);
template void launch_p2_force_split<double>(int, cx<double>*, size_t, int, int, double, hipStream_t);
template void launch_p2_force_split<float>(int, cx<float>*, size_t, int, int, double, hipStream_t);
template void launch_p3<double>(int, SpecMode, const cx<double>*, size_t, int, cx<double>*, size_t, int, int,
                                const SpecCoef&, const double*, double*, double*, const SolveCtl*, hipStream_t);
template void launch_p3<float>(int, SpecMode, const cx<float>*, size_t, int, cx<float>*, size_t, int, int,
                               const SpecCoef&, const double*, double*, double*, const SolveCtl*, hipStream_t);

}  // namespace dgp

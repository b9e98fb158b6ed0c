// Fused FFT-relaxation pass and its device-side convergence control.
//
// One relaxation pass (Sec. III B, Eq. FFTrelax with the w-split of Sec. III C)
// evaluates the residual of the current iterate u^(n) and produces u^(n+1).  The
// kernel here is its last stage: for a tile of axis-0 columns it
//   1. inverse-transforms along axis 0 the five Hessian spectra h00, h11, h01,
//      h02, h12 and the nonlocal spectrum Nf = -u(k)/kbar (the other two axes
//      were inverted by the preceding passes), accumulating in registers (float64;
//      float32 in the float32 form) sum_ij h_ij^2 and h22 = (u - <u>) - h00 - h11 (the trace identity:
//      h00 + h11 + h22 = u - <u>, exact on the mesh, saves a sixth transform);
//   2. evaluates, per point, the residual R of Eq. FullDGP2, B' of Eq. Bwpara,
//      the discriminant of Eq. nabla^2Cwpara and its + root in the stable form
//      2 B'/(alpha + sqrt(Delta)); a negative discriminant is a bad point and
//      takes the vertex -alpha/(2 (1-w) lam) (Sec. III C);
//   3. writes u^(n+1) and immediately forward-transforms it along axis 0, so
//      the next pass starts from its axis-0 spectrum;
//   4. reduces sum |R| (FP64) and the bad-point count per workgroup.
// A single-workgroup kernel then forms r = <|R|>/eps (Eq. normres) per batch
// element and runs the stopping rules; kernels of later passes read the
// per-element `done` flag and exit at once.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include "dgp_internal.h"

namespace dgp {

template <typename T>
const cx<T>* twiddles(int n);

// FFT plans of the axis-0 transforms in the relaxation pass (0: radix 8, 1: radix 16, 2: radix 4)
#ifndef DGP_PLAN_RELAX
#define DGP_PLAN_RELAX 2
#endif
#ifndef DGP_PLAN_RELAX_F32
#define DGP_PLAN_RELAX_F32 0
#endif
#ifndef DGP_RELAX_F32ACC
#define DGP_RELAX_F32ACC 1
#endif
#ifndef DGP_RELAX_TP_F32
#define DGP_RELAX_TP_F32 8
#endif
#ifndef DGP_RELAX_MINW_F32
#define DGP_RELAX_MINW_F32 1
#endif
// column pairs of the float32 kernel from N = 512 on
#ifndef DGP_RELAX_TP_WIDE_F32
#define DGP_RELAX_TP_WIDE_F32 16
#endif
// smallest N whose float32 relaxation kernel pairs its lanes: the two threads whose transform
// elements e and N - e share a spectral row sit in one wavefront and load that row in the same
// instruction (one request instead of two)
#ifndef DGP_RELAX_PAIRED_MIN
#define DGP_RELAX_PAIRED_MIN 256
#endif
// smallest N whose float32 relaxation kernel re-derives its lane indices at every field, so that
// the per-lane addresses built from them are not held across the field loop (at N = 512 the
// 1024-thread workgroup leaves 128 VGPRs per lane)
#ifndef DGP_RELAX_REMAT_MIN
#define DGP_RELAX_REMAT_MIN 256
#endif
// padding rows of the float32 kernel's transform exchanges (one after every DGP_RELAX_LDSPAD rows)
#ifndef DGP_RELAX_LDSPAD
#define DGP_RELAX_LDSPAD 8
#endif
// smallest N whose float32 relaxation kernel keeps the running h22 = -(h00 + h11) in LDS (each
// thread its own slots) instead of registers across the field loop
#ifndef DGP_RELAX_PARK_MIN
#define DGP_RELAX_PARK_MIN 256
#endif

// axis-0 tile of the relaxation kernel: AxisTile with an optional number of column pairs
template <typename T, int N, int R, int TPSET>
struct RelaxTile {
  static constexpr int kT = AxisTile<T, N, R>::kT;
  static constexpr int kTP = TPSET > 0 ? (TPSET < N / 2 ? TPSET : N / 2) : AxisTile<T, N, R>::kTP;
  static constexpr int kThreads = kTP * kT;
};

// geometry of the float32 relaxation kernel
template <typename T, int N>
struct RelaxGeo {
  static_assert(sizeof(T) == 4, "the block-synchronous relaxation kernel is the float32 one");
  // at N >= 512 the spectral planes are 2 MB apart and a 128-byte row segment per plane streams
  // poorly: radix 8 and 16 column pairs (256-byte segments)
  static constexpr bool kWide = N >= 512;
  using P = typename PlanPick<N, (kWide ? 0 : DGP_PLAN_RELAX_F32)>::type;
  static constexpr int R = P::R;
  using G = RelaxTile<T, N, R, (kWide ? DGP_RELAX_TP_WIDE_F32 : DGP_RELAX_TP_F32)>;
  // minimum wavefronts per SIMD the register allocation plans for (second launch bound)
  static constexpr int kMinWaves = DGP_RELAX_MINW_F32;
  // accumulators of the float32 form (sum h^2 and -(h00 + h11)): float32 or float64; the
  // residual, discriminant and root are float64 either way
  using Acc = typename std::conditional<DGP_RELAX_F32ACC, float, double>::type;
  // lane order of the paired loads (needs an even number of transform positions per wavefront)
  static constexpr bool kPaired = N >= DGP_RELAX_PAIRED_MIN && (64 / G::kTP) % 2 == 0;
  static constexpr bool kRemat = N >= DGP_RELAX_REMAT_MIN;
  static constexpr bool kPark = N >= DGP_RELAX_PARK_MIN;
};

// sum over the W lanes of a wavefront segment (butterfly order, deterministic)
template <int W>
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}
template <int W>
__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}

// Per-point residual and update in float64 (Eqs. FullDGP2, Bwpara, nabla^2Cwpara).  The + root
// 2 B' / (alpha + sqrt(Delta)) is formed without branches: the hardware estimates of
// 1/sqrt(Delta) and of the reciprocal of the denominator (float64 instructions) are refined by
// one Newton step each, sqrt(Delta) = Delta / sqrt(Delta) gets one Heron correction and the
// quotient one residual correction (each correction squares the relative error).  Delta = 0 takes sqrt = 0, and a
// negative Delta (a bad point) takes the vertex -alpha / (2 (1-w) lam).  Straight-line code
// lets the compiler interleave the points of a thread.
struct PointCoef {
  double lam, w, alpha, gamma, omega, mu, vertex, c4;
};

__device__ __forceinline__ PointCoef point_coef(const SolveCfg& cfg, double mu) {
  PointCoef k;
  k.lam = cfg.lam;
  k.w = cfg.w;
  k.alpha = cfg.alpha;
  k.gamma = cfg.gamma;
  k.omega = cfg.omega;
  k.mu = mu;
  k.vertex = -cfg.alpha / (2.0 * (1.0 - cfg.w) * cfg.lam);
  k.c4 = 4.0 * (1.0 - cfg.w) * cfg.lam;
  return k;
}

// u: iterate, s: source, nf: nonlocal term, s2: sum of the squared Hessian entries other than
// h22, h22m: -(h00 + h11) (h22 = h22m + u - <u> by the trace identity)
__device__ __forceinline__ double relax_point(const PointCoef& k, double u, double s, double nf, double s2,
                                              double h22m, double& abs_r, int& nbad) {
  const double hz = h22m + (u - k.mu);
  const double sh2 = s2 + hz * hz;
  const double res = k.lam * (u * u - sh2) + k.alpha * u + k.gamma * nf - s;
  abs_r += fabs(res);
  const double bp = k.lam * (sh2 - k.w * u * u) - k.gamma * nf + s;
  const double disc = k.alpha * k.alpha + k.c4 * bp;
  nbad += disc < 0.0 ? 1 : 0;
  double y = __builtin_amdgcn_rsq(disc);
  y = y * (1.5 - (0.5 * disc) * (y * y));
  double sq = disc * y;
  sq = fma(0.5 * y, fma(-sq, sq, disc), sq);   // Heron correction of sqrt(Delta)
  sq = disc > 0.0 ? sq : 0.0;
  const double den = k.alpha + sq;
  double r = __builtin_amdgcn_rcp(den);
  r = r * (2.0 - den * r);
  const double num = 2.0 * bp;
  double x = num * r;
  x = fma(r, fma(-den, x, num), x);
  x = disc < 0.0 ? k.vertex : x;
  if (k.omega != 1.0) x = (1.0 - k.omega) * u + k.omega * x;
  return x;
}

template <int R, typename V, typename A>
__device__ __forceinline__ void relax_points(const PointCoef& k, const V (&up)[R], const V (&spv)[R], const V (&nfv)[R],
                                             const A (&s2)[R][2], const A (&h22)[R][2], double (&un)[R][2],
                                             double& abs_r, int& nbad) {
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      un[q][j] = relax_point(k, double(j ? up[q].y : up[q].x), double(j ? spv[q].y : spv[q].x),
                             double(j ? nfv[q].y : nfv[q].x), double(s2[q][j]), double(h22[q][j]), abs_r, nbad);
}

// float32 kernel: block-synchronous transforms; each thread loads, one field ahead, exactly the
// spectral rows its transform elements need (row e, or row N - e conjugated), so the tile is not
// staged in LDS
template <typename T, int N>
__global__ void __launch_bounds__((RelaxGeo<T, N>::G::kThreads), (RelaxGeo<T, N>::kMinWaves))
k_relax(const cx<T>* __restrict__ spec6, size_t fstride, T* __restrict__ ubuf, const T* __restrict__ sfield,
        cx<T>* __restrict__ spec_u, double* __restrict__ partial, const double* __restrict__ mean_u, SolveCfg cfg,
        const SolveCtl* __restrict__ ctl, const cx<T>* __restrict__ tw) {
  using RG = RelaxGeo<T, N>;
  using P = typename RG::P;
  using Acc = typename RG::Acc;
  constexpr int R = P::R;
  using G = typename RG::G;
  constexpr int TP = G::kTP, TT = G::kT, H = N / 2 + 1;
  constexpr size_t N3 = (size_t)N * N * N;
  const int b = blockIdx.z;
  if (ctl[b].done) return;
  const int cur = ctl[b].cur, nxt = ctl[b].out;
  int tile, i1;
  xcd_tile(tile, i1);
  int c = threadIdx.x % TP;
  // transform element index t of this thread.  Paired order: positions g = 0, 1 take t = 0 and
  // TT/2 (their own partners), then g = 2k, 2k + 1 take t = k and TT - k, so a wavefront (64/TP
  // consecutive positions, an even count) holds both threads of every pair; elements e = t + q TT
  // and N - e = (TT - t) + (R - 1 - q) TT read the same spectral row
  const int g = threadIdx.x / TP;
  constexpr bool PAIRED = RG::kPaired;
  int t = !PAIRED ? g : g < 2 ? g * (TT / 2) : (g & 1) ? TT - (g >> 1) : (g >> 1);
  const int i2 = (tile * TP + c) * 2;
  // transform exchanges, then (kPark) R slots per thread for the running h22
  constexpr int PG = DGP_RELAX_LDSPAD, LROWS = PG > 0 ? N + N / PG : N;
  __shared__ cx<T> lds[LROWS * TP + (RG::kPark ? R * G::kThreads : 0)];
  cx<T>* const park = lds + LROWS * TP + threadIdx.x;   // slot q at park[q * kThreads]
  __shared__ double red[(G::kThreads + 63) / 64];
  __shared__ int redi[(G::kThreads + 63) / 64];
  // the twiddle table is read from LDS: the seven transforms of a pass would otherwise wait on
  // cached global loads at every stage
  __shared__ cx<T> twl[N];
  for (int i = threadIdx.x; i < N; i += G::kThreads) twl[i] = tw[i];

  const size_t col = (size_t)b * H * N * N + (size_t)i1 * N + i2;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const size_t col0 = (size_t)b * H * N * N + (size_t)i1 * N + (size_t)tile * TP * 2;
  // element q of thread t is row e = t + q TT of the Hermitian-extended column pair; rows e > N/2
  // come from row N - e (conjugated when used); streaming loads (the last use of these spectra in
  // the pass).  With paired lanes, threads t > TT/2 load their elements in reverse slot order, so
  // that slot q of both threads of a pair addresses the same row.
  cx<T> pd[R][2];
  // (a workgroup-uniform base plus a 32-bit lane offset: one register per address)
  static_assert((size_t)(N / 2 + 1) * N * N * sizeof(cx<T>) < (size_t(1) << 32), "32-bit row offsets");
  auto fetch_direct = [&](int f) {
    const char* src = reinterpret_cast<const char*>(spec6 + f * fstride + col0);
#pragma unroll
    for (int q = 0; q < R; ++q) {   // slot q holds element R - 1 - q when rev
      const bool rev = PAIRED && t > TT / 2;
      const int e = t + (rev ? R - 1 - q : q) * TT;
      const unsigned r = e <= N / 2 ? e : N - e;
      const f4* a = reinterpret_cast<const f4*>(src + (r * unsigned(N * N) + 2u * c) * unsigned(sizeof(cx<T>)));
      const f4 x = __builtin_nontemporal_load(a);
      pd[q][0] = mk(T(x.x), T(x.y));
      pd[q][1] = mk(T(x.z), T(x.w));
    }
  };
  fetch_direct(0);

  Acc s2[R][2], h22[R][2];
  cx<T> v[R];
  cx<T> up[R], spv[R];
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    if constexpr (RG::kRemat) asm volatile("" : "+v"(t), "+v"(c));   // opaque: recomputed per field
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      const bool rev = PAIRED && t > TT / 2;
      cx<T> xa = rev ? pd[R - 1 - q][0] : pd[q][0], xb = rev ? pd[R - 1 - q][1] : pd[q][1];
      if (e > N / 2) {
        xa = conjg(xa);
        xb = conjg(xb);
      }
      if (e == 0 || e == N / 2) { xa.y = T(0); xb.y = T(0); }
      v[q] = mk(xa.x - xb.y, xa.y + xb.x);   // x_a + i x_b
    }
    if (f < 5) fetch_direct(f + 1);
    {
      LdsCol<T, TP, PG> L{lds, c};
      fft<T, N, P, +1>(v, twl, L, t);
    }
    if (f < 5) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const Acc hx = Acc(v[q].x), hy = Acc(v[q].y);
        if (f == 0) {
          s2[q][0] = hx * hx;
          s2[q][1] = hy * hy;
          if constexpr (RG::kPark) {
            park[q * G::kThreads] = mk(T(-hx), T(-hy));
          } else {
            h22[q][0] = -hx;
            h22[q][1] = -hy;
          }
        } else if (f == 1) {
          s2[q][0] += hx * hx;
          s2[q][1] += hy * hy;
          if constexpr (RG::kPark) {
            const cx<T> hz = park[q * G::kThreads];
            park[q * G::kThreads] = mk(hz.x - T(hx), hz.y - T(hy));
          } else {
            h22[q][0] -= hx;
            h22[q][1] -= hy;
          }
        } else {
          s2[q][0] += Acc(2) * hx * hx;
          s2[q][1] += Acc(2) * hy * hy;
        }
      }
    }
  }
  // pointwise residual and update; v holds Nf (field addresses formed after the field loop)
  const T* uin = ubuf + ((size_t)cur * cfg.batch + b) * N3 + (size_t)i1 * N + i2;
  const T* sp = sfield + (size_t)b * N3 + (size_t)i1 * N + i2;
  const PointCoef pc = point_coef(cfg, mean_u[b]);
  T* uout = ubuf + ((size_t)nxt * cfg.batch + b) * N3 + (size_t)i1 * N + i2;
  double abs_r = 0.0;
  int nbad = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const size_t off = (size_t)(t + q * TT) * N * N;
    up[q] = *reinterpret_cast<const cx<T>*>(uin + off);
    spv[q] = *reinterpret_cast<const cx<T>*>(sp + off);
  }
  if constexpr (RG::kPark) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const cx<T> hz = park[q * G::kThreads];
      h22[q][0] = Acc(hz.x);
      h22[q][1] = Acc(hz.y);
    }
  }
  double un[R][2];
  relax_points(pc, up, spv, v, s2, h22, un, abs_r, nbad);
  if constexpr (RG::kRemat) asm volatile("" : "+v"(t), "+v"(c));   // the epilogue's addresses from here
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const size_t off = (size_t)(t + q * TT) * N * N;
    const cx<T> o = mk(T(un[q][0]), T(un[q][1]));
    store_stream(reinterpret_cast<cx<T>*>(uout + off), o);   // read again next pass only
    v[q] = o;
  }
  // forward axis-0 transform of u^(n+1)
  {
    LdsCol<T, TP, PG> L{lds, c};
    fft<T, N, P, -1>(v, twl, L, t);
  }
  lds_barrier();
#pragma unroll
  for (int q = 0; q < R; ++q) lds[(t + q * TT) * TP + c] = v[q];
  constexpr int WW = G::kThreads < 64 ? G::kThreads : 64;   // lanes of a (possibly partial) wavefront
  abs_r = wave_sum<WW>(abs_r);
  nbad = wave_sum<WW>(nbad);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = abs_r;
    redi[threadIdx.x >> 6] = nbad;
  }
  lds_barrier();
  cx<T>* dst = spec_u + col;
  for (int k = t; k < H; k += TT) {
    const cx<T> zk = lds[k * TP + c];
    const cx<T> zn = lds[((N - k) & (N - 1)) * TP + c];
    dst[(size_t)k * N * N] = mk(T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y));
    dst[(size_t)k * N * N + 1] = mk(T(0.5) * (zk.y + zn.y), T(0.5) * (zn.x - zk.x));
  }
  // per-wavefront sums added in wavefront order (deterministic)
  if (threadIdx.x == 0) {
    double sr = 0.0;
    int sb = 0;
#pragma unroll
    for (int i = 0; i < (G::kThreads + 63) / 64; ++i) {
      sr += red[i];
      sb += redi[i];
    }
    const size_t g = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const size_t groups = (size_t)gridDim.x * gridDim.y;
    partial[((size_t)b * groups + g) * 2] = sr;
    partial[((size_t)b * groups + g) * 2 + 1] = double(sb);
  }
}


// ------------------------------------------------------------------ float64 kernel (wave-local)
// Same pass as k_relax, restructured so that each axis-0 transform is carried by the
// lanes of one wavefront: its Stockham exchanges then need wavefront ordering only,
// and the workgroup barriers drop from one pair per stage to one per field.  Global
// traffic stays coalesced: spectral tiles are fetched row-wise into a double-buffered,
// padded LDS tile; a transform reads its own two columns of the tile and reuses the
// same slots (only its wavefront touches them) for the exchanges.  Below N = 512, u and S are
// read row-wise too and redistributed to the transforms through the two tiles once the field
// loop is done.
#ifndef DGP_RELAXW_TP_F64
#define DGP_RELAXW_TP_F64 0
#endif
#ifndef DGP_RELAXW_MINW_F64
#define DGP_RELAXW_MINW_F64 3
#endif
// column pairs of the float64 kernel from N = 512 on
#ifndef DGP_RELAXW_TP_WIDE_F64
#define DGP_RELAXW_TP_WIDE_F64 8
#endif
// smallest N whose float64 relaxation kernel reads its twiddles from LDS
#ifndef DGP_RELAXW_TWLDS_MIN
#define DGP_RELAXW_TWLDS_MIN 512
#endif

// float64 kernel: u and S read row-wise (consecutive lanes on one row) and redistributed through
// LDS (1), instead of each lane reading its own transform's elements, 64 rows per instruction (0)
// (256^3 on gfx950: 345 vs 363 us per launch)
#ifndef DGP_RELAXW_US_LDS
#define DGP_RELAXW_US_LDS 1
#endif

template <typename T, int N>
struct RelaxWGeo {
  static_assert(sizeof(T) == 8, "the wave-local relaxation kernel is the float64 one");
  // at N >= 512: radix 8 (one 512-point transform per wavefront) and 8 column pairs
  static constexpr bool kWide = N >= 512;
  using P = typename PlanPick<N, (kWide ? 0 : DGP_PLAN_RELAX)>::type;
  static constexpr int R = P::R;
  using G = AxisTile<T, N, R>;
  static constexpr int kTPSet = kWide ? DGP_RELAXW_TP_WIDE_F64 : DGP_RELAXW_TP_F64;
  static constexpr int kTP = kTPSet > 0 ? (kTPSet < N / 2 ? kTPSet : N / 2) : G::kTP;
  static constexpr int kT = G::kT, kThreads = kTP * kT, H = N / 2 + 1;
  static constexpr int kMinWaves = kWide ? 2 : DGP_RELAXW_MINW_F64;   // the LDS tile allows one workgroup per CU from N = 512
  // twiddles from an LDS copy: held in registers, the loop-invariant twiddles of the six
  // inverse transforms would need 56 VGPRs across the field loop at N = 512, where the kernel
  // already uses all 256 of a two-waves-per-SIMD allocation
  static constexpr bool kTwLds = N >= DGP_RELAXW_TWLDS_MIN;
  // u and S read row-wise and redistributed through LDS (below N = 512: the staging registers
  // would not fit the wide geometry's allocation)
  static constexpr bool kUsLds = DGP_RELAXW_US_LDS && !kWide;
  static_assert(kT <= 64 && 64 % kT == 0, "a transform must stay inside one wavefront");
  static constexpr int kSP = 2 * kTP + 1;                            // padded tile row, complex
  static constexpr int kTile = H * kSP;
  static constexpr int kNPF = (H * kTP + kThreads - 1) / kThreads;   // column pairs fetched per thread
  static constexpr int kWaves = (kThreads + 63) / 64;
  static constexpr int kWidth = kThreads < 64 ? kThreads : 64;       // lanes of a (possibly partial) wavefront
};

// Exchange slots of transform c inside its own two tile columns (2c, 2c+1).
template <typename T, int SP>
struct LdsPair {
  cx<T>* base;
  int c;
  __device__ __forceinline__ cx<T> load(int e) const { return base[(e >> 1) * SP + 2 * c + (e & 1)]; }
  __device__ __forceinline__ void store(int e, cx<T> v) const { base[(e >> 1) * SP + 2 * c + (e & 1)] = v; }
  __device__ __forceinline__ void sync() const { wave_sync(); }
};


// (the second launch bound is the minimum number of wavefronts per SIMD to plan registers for)
template <typename T, int N>
__global__ void __launch_bounds__((RelaxWGeo<T, N>::kThreads), (RelaxWGeo<T, N>::kMinWaves))
k_relax_w(const cx<T>* __restrict__ spec6, size_t fstride, T* __restrict__ ubuf, const T* __restrict__ sfield,
          cx<T>* __restrict__ spec_u, double* __restrict__ partial, const double* __restrict__ mean_u, SolveCfg cfg,
          const SolveCtl* __restrict__ ctl, const cx<T>* __restrict__ tw) {
  using W = RelaxWGeo<T, N>;
  using P = typename W::P;
  constexpr int R = W::R, TP = W::kTP, TT = W::kT, NT = W::kThreads, H = N / 2 + 1, SP = W::kSP;
  constexpr int NPF = W::kNPF;
  constexpr size_t N3 = (size_t)N * N * N, NN = (size_t)N * N;
  const int b = blockIdx.z;
  if (ctl[b].done) return;
  const int cur = ctl[b].cur, nxt = ctl[b].out;
  int tile, i1;
  xcd_tile(tile, i1);
  const int i2 = tile * 2 * TP;
  const int c = threadIdx.x / TT, t = threadIdx.x % TT;   // transform mapping
  __shared__ cx<T> lds[2 * W::kTile];
  __shared__ double redd[W::kWaves];
  __shared__ int redi[W::kWaves];
  __shared__ cx<T> twl[W::kTwLds ? N : 1];
  const cx<T>* twp = tw;
  if constexpr (W::kTwLds) {
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = tw[i];   // ordered by the first field's barrier
    twp = twl;
  }

  const size_t col0 = (size_t)b * H * NN + (size_t)i1 * N + i2;
  cx<T> pf[NPF][2];
  // every thread loads NPF pairs, indices past the tile clamped to its last pair, so the
  // staging registers are assigned unconditionally and stay in registers
  auto fetch = [&](int f) {
    const cx<T>* src = spec6 + f * fstride + col0;
#pragma unroll
    for (int r = 0; r < NPF; ++r) {
      const int idx = min(int(threadIdx.x) + r * NT, H * TP - 1);
      const int k = idx / TP, p = idx % TP;
      const cx<T>* q = src + (size_t)k * NN + 2 * p;
      pf[r][0] = mk(q[0].x, q[0].y);   // member-wise: a 16-byte struct copy would stay in private memory
      pf[r][1] = mk(q[1].x, q[1].y);
    }
  };
  // (a clamped index rewrites the last pair with the value it already holds)
  auto stash = [&](cx<T>* buf) {
#pragma unroll
    for (int r = 0; r < NPF; ++r) {
      const int idx = min(int(threadIdx.x) + r * NT, H * TP - 1);
      const int k = idx / TP, p = idx % TP;
      buf[k * SP + 2 * p].x = pf[r][0].x;
      buf[k * SP + 2 * p].y = pf[r][0].y;
      buf[k * SP + 2 * p + 1].x = pf[r][1].x;
      buf[k * SP + 2 * p + 1].y = pf[r][1].y;
    }
  };
  fetch(0);

  double s2[R][2], h22[R][2];
  cx<T> v[R], up[R], spv[R];
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    cx<T>* buf = lds + (f & 1) * W::kTile;
    stash(buf);
    lds_barrier();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      cx<T> xa, xb;
      if (e <= N / 2) {
        xa = buf[e * SP + 2 * c];
        xb = buf[e * SP + 2 * c + 1];
        if (e == 0 || e == N / 2) { xa.y = T(0); xb.y = T(0); }
      } else {
        xa = conjg(buf[(N - e) * SP + 2 * c]);
        xb = conjg(buf[(N - e) * SP + 2 * c + 1]);
      }
      v[q] = mk(xa.x - xb.y, xa.y + xb.x);
    }
    if (f < 5) fetch(f + 1);
    LdsPair<T, SP> X{buf, c};
    fft<T, N, P, +1>(v, twp, X, t);
    if (f < 5) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double hx = v[q].x, hy = v[q].y;
        if (f == 0) {
          s2[q][0] = hx * hx;
          s2[q][1] = hy * hy;
          h22[q][0] = -hx;
          h22[q][1] = -hy;
        } else if (f == 1) {
          s2[q][0] += hx * hx;
          s2[q][1] += hy * hy;
          h22[q][0] -= hx;
          h22[q][1] -= hy;
        } else {
          s2[q][0] += 2.0 * hx * hx;
          s2[q][1] += 2.0 * hy * hy;
        }
      }
    }
  }
  // pointwise residual and update (v holds Nf); u^(n+1) is staged in tile 0 (free since the last barrier).
  // The field addresses are formed here, after the field loop, so that they are not held in
  // registers across it.
  const PointCoef pc = point_coef(cfg, mean_u[b]);
  T* ust = reinterpret_cast<T*>(lds);
  double abs_r = 0.0;
  int nbad = 0;
  if constexpr (W::kUsLds) {
    // row-wise reads (TP lanes per row, one column pair each) into tile 0 (u) and tile 1 (S),
    // rows 2 TP + 1 values apart; tile 1 is free once every wavefront has finished its last
    // inverse transform (first barrier); the second barrier orders the reads before the forward
    // transform's exchanges in tile 1
    constexpr int NU = (N * TP + NT - 1) / NT;
    const T* ur = ubuf + ((size_t)cur * cfg.batch + b) * N3 + (size_t)i1 * N + i2;
    const T* sr = sfield + (size_t)b * N3 + (size_t)i1 * N + i2;
    cx<T> lu[NU], ls[NU];
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      const int idx = min(int(threadIdx.x) + r * NT, N * TP - 1);
      const int e = idx / TP, p = idx % TP;
      lu[r] = *reinterpret_cast<const cx<T>*>(ur + (size_t)e * NN + 2 * p);
      ls[r] = *reinterpret_cast<const cx<T>*>(sr + (size_t)e * NN + 2 * p);
    }
    T* sst = reinterpret_cast<T*>(lds + W::kTile);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      const int idx = min(int(threadIdx.x) + r * NT, N * TP - 1);
      const int e = idx / TP, p = idx % TP;
      ust[e * (2 * TP + 1) + 2 * p] = lu[r].x;
      ust[e * (2 * TP + 1) + 2 * p + 1] = lu[r].y;
      sst[e * (2 * TP + 1) + 2 * p] = ls[r].x;
      sst[e * (2 * TP + 1) + 2 * p + 1] = ls[r].y;
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      up[q] = mk(ust[e * (2 * TP + 1) + 2 * c], ust[e * (2 * TP + 1) + 2 * c + 1]);
      spv[q] = mk(sst[e * (2 * TP + 1) + 2 * c], sst[e * (2 * TP + 1) + 2 * c + 1]);
    }
    lds_barrier();
  } else {
    const T* uin = ubuf + ((size_t)cur * cfg.batch + b) * N3 + (size_t)i1 * N + i2 + 2 * c;
    const T* sp = sfield + (size_t)b * N3 + (size_t)i1 * N + i2 + 2 * c;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = t + q * TT;
      up[q] = *reinterpret_cast<const cx<T>*>(uin + (size_t)e * NN);
      spv[q] = *reinterpret_cast<const cx<T>*>(sp + (size_t)e * NN);
    }
  }
  double un[R][2];
  relax_points(pc, up, spv, v, s2, h22, un, abs_r, nbad);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int e = t + q * TT;
    const cx<T> o = mk(T(un[q][0]), T(un[q][1]));
    ust[e * (2 * TP + 1) + 2 * c] = o.x;
    ust[e * (2 * TP + 1) + 2 * c + 1] = o.y;
    v[q] = o;
  }
  // forward axis-0 transform of u^(n+1), exchanges in the transform's own columns of tile 1
  {
    LdsPair<T, SP> X{lds + W::kTile, c};
    fft<T, N, P, -1>(v, twp, X, t);
  }
  abs_r = wave_sum<W::kWidth>(abs_r);
  nbad = wave_sum<W::kWidth>(nbad);
  if ((threadIdx.x & 63) == 0) {
    redd[threadIdx.x >> 6] = abs_r;
    redi[threadIdx.x >> 6] = nbad;
  }
  lds_barrier();
  // u^(n+1) out of tile 0 (coalesced); the spectrum into tile 1, column-major with one pad
  T* uout = ubuf + ((size_t)nxt * cfg.batch + b) * N3 + (size_t)i1 * N + i2;
  for (int idx = threadIdx.x; idx < N * TP; idx += NT) {
    const int e = idx / TP, p = idx % TP;
    const cx<T> o = mk(ust[e * (2 * TP + 1) + 2 * p], ust[e * (2 * TP + 1) + 2 * p + 1]);
    *reinterpret_cast<cx<T>*>(uout + (size_t)e * NN + 2 * p) = o;
  }
  cx<T>* zt = lds + W::kTile;
#pragma unroll
  for (int q = 0; q < R; ++q) zt[c * (N + 1) + t + q * TT] = v[q];
  lds_barrier();
  cx<T>* dst = spec_u + col0;
  for (int idx = threadIdx.x; idx < H * TP; idx += NT) {
    const int k = idx / TP, p = idx % TP;
    const cx<T> zk = zt[p * (N + 1) + k];
    const cx<T> zn = zt[p * (N + 1) + ((N - k) & (N - 1))];
    dst[(size_t)k * NN + 2 * p] = mk(T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y));
    dst[(size_t)k * NN + 2 * p + 1] = mk(T(0.5) * (zk.y + zn.y), T(0.5) * (zn.x - zk.x));
  }
  if (threadIdx.x == 0) {
    double sr = 0.0;
    int sb = 0;
    for (int i = 0; i < W::kWaves; ++i) {
      sr += redd[i];
      sb += redi[i];
    }
    const size_t g = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const size_t groups = (size_t)gridDim.x * gridDim.y;
    partial[((size_t)b * groups + g) * 2] = sr;
    partial[((size_t)b * groups + g) * 2 + 1] = double(sb);
  }
}

// Convergence control: one workgroup of 1024 threads walks the batch (per element: strided
// partial sums, wavefront shuffles, a fixed-order sum over the 16 wavefronts).
__global__ void __launch_bounds__(1024)
k_finalize(const double* __restrict__ partial, int groups, SolveCtl* __restrict__ ctl, SolveCfg cfg,
           int* __restrict__ n_active) {
  __shared__ double sr[16], sb[16];
  __shared__ int active;
  if (threadIdx.x == 0) active = 0;
  const double n3 = double(cfg.n) * cfg.n * cfg.n;
  for (int b = 0; b < cfg.batch; ++b) {
    __syncthreads();
    if (ctl[b].done) continue;
    double ar = 0.0, ab = 0.0;
    const double2* pb = reinterpret_cast<const double2*>(partial) + (size_t)b * groups;
    for (int g = threadIdx.x; g < groups; g += 1024) {
      const double2 v = pb[g];
      ar += v.x;
      ab += v.y;
    }
    ar = wave_sum<64>(ar);
    ab = wave_sum<64>(ab);
    if ((threadIdx.x & 63) == 0) {
      sr[threadIdx.x >> 6] = ar;
      sb[threadIdx.x >> 6] = ab;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 1; i < 16; ++i) {
        sr[0] += sr[i];
        sb[0] += sb[i];
      }
      SolveCtl& C = ctl[b];
      // eps = 0 only for a uniform delta (S = 0), whose exact solution u = 0 has R = 0
      const double r = C.eps > 0.0 ? sr[0] / (n3 * C.eps) : (sr[0] == 0.0 ? 0.0 : __builtin_huge_val());
      const int nbad = int(sb[0]);
      const int n = C.iters;
      if (n < kMaxHist) {
        C.hist[n] = r;
        C.hist_bad[n] = double(nbad) / n3;
      }
      C.passes += 1;
      bool done = false;
      if (r != r) {   // a non-finite iterate (non-finite warm start, or divergence): nothing to return
        C.status = kStatusInvalid;
        C.result = C.cur;
        C.resid = r;
        done = true;
      } else if (r <= cfg.tol) {
        C.status = 0;
        C.result = C.cur;
        C.resid = r;
        C.final_bad = nbad;   // that pass's update sits in buffer C.out
        done = true;
      } else if (r < C.resid_min) {
        C.resid_min = r;
        C.best = C.cur;
      } else if (C.bad_seen && !cfg.fixed) {
        C.status = 2;
        C.result = C.best;
        C.resid = C.resid_min;
        done = true;
      }
      if (r < C.resid_min) C.resid_min = r;
      if (!done && n + C.iters1 >= cfg.max_iter) {
        if (cfg.fixed) {   // the requested number of updates: the last iterate
          C.status = 0;
          C.result = C.cur;
          C.resid = r;
        } else {
          C.status = 1;
          C.result = C.best;
          C.resid = C.resid_min;
        }
        done = true;
      }
      if (!done) {
        C.last_bad = nbad;
        C.bad_frac = double(nbad) / n3;
        if (nbad > 0) C.bad_seen = 1;
        C.iters = n + 1;
        const int nc = C.out;
        C.cur = nc;
        C.out = 3 - nc - C.best;
        ++active;
      }
      C.done = done ? 1 : 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *n_active = active;
}

// Per-batch mean of |x| and of x, deterministic two-level reduction.
template <typename T>
__global__ void __launch_bounds__(256)
k_absmean_partial(const T* __restrict__ x, size_t n3, double* __restrict__ part) {
  const int b = blockIdx.y;
  const T* xb = x + (size_t)b * n3;
  double sa = 0.0, sm = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double v = double(xb[i]);
    sa += fabs(v);
    sm += v;
  }
  __shared__ double ra[256], rm[256];
  ra[threadIdx.x] = sa;
  rm[threadIdx.x] = sm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      ra[threadIdx.x] += ra[threadIdx.x + s];
      rm[threadIdx.x] += rm[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = ra[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = rm[0];
  }
}

__global__ void __launch_bounds__(256)
k_absmean_final(const double* __restrict__ part, int groups, size_t n3, double* __restrict__ abs_mean,
                double* __restrict__ mean) {
  const int b = blockIdx.x;
  __shared__ double ra[256], rm[256];
  double sa = 0.0, sm = 0.0;
  for (int g = threadIdx.x; g < groups; g += 256) {
    sa += part[((size_t)b * groups + g) * 2];
    sm += part[((size_t)b * groups + g) * 2 + 1];
  }
  ra[threadIdx.x] = sa;
  rm[threadIdx.x] = sm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      ra[threadIdx.x] += ra[threadIdx.x + s];
      rm[threadIdx.x] += rm[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (abs_mean) abs_mean[b] = ra[0] / double(n3);
    if (mean) mean[b] = rm[0] / double(n3);
  }
}

// ------------------------------------------------------------------ launchers
// (ev0, ev1: optional timing events recorded by the dispatch itself, at the kernel's start and
// end, without separate marker packets in the stream)
template <typename T, int N>
static void relax_n(const cx<T>* spec6, T* ubuf, const T* sfield, cx<T>* spec_u, double* partial,
                    const double* mean_u, int batch, const SolveCfg& cfg, const SolveCtl* ctl, hipStream_t s,
                    hipEvent_t ev0, hipEvent_t ev1) {
  constexpr size_t fstride = (size_t)(N / 2 + 1) * N * N;
  if constexpr (sizeof(T) == 8) {
    using W = RelaxWGeo<T, N>;
    dim3 grid(N / (2 * W::kTP), N, batch);
    hipExtLaunchKernelGGL((k_relax_w<T, N>), grid, dim3(W::kThreads), 0, s, ev0, ev1, 0, spec6, fstride * batch,
                          ubuf, sfield, spec_u, partial, mean_u, cfg, ctl, twiddles<T>(N));
  } else {
    using G = typename RelaxGeo<T, N>::G;
    dim3 grid(N / (2 * G::kTP), N, batch);
    hipExtLaunchKernelGGL((k_relax<T, N>), grid, dim3(G::kThreads), 0, s, ev0, ev1, 0, spec6, fstride * batch,
                          ubuf, sfield, spec_u, partial, mean_u, cfg, ctl, twiddles<T>(N));
  }
}

template <typename T>
void launch_relax(int n, const cx<T>* spec6, T* ubuf, const T* sfield, cx<T>* spec_u, double* partial,
                  const double* mean_u, int batch, const SolveCfg& cfg, const SolveCtl* ctl, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1) {
#define C(NN) relax_n<T, NN>(spec6, ubuf, sfield, spec_u, partial, mean_u, batch, cfg, ctl, s, ev0, ev1)
  switch (n) {
    case 8: C(8); break;
    case 16: C(16); break;
    case 32: C(32); break;
    case 64: C(64); break;
    case 128: C(128); break;
    case 256: C(256); break;
    case 512: C(512); break;
    default: break;
  }
#undef C
}

// column pairs per workgroup of the relaxation kernel that launches for (T, N)
template <typename T, int N>
static constexpr int relax_tp() {
  if constexpr (sizeof(T) == 8) return RelaxWGeo<T, N>::kTP;
  else return RelaxGeo<T, N>::G::kTP;
}

int relax_groups(int n, int elem_bytes) {
  int tp = 0;
#define C(NN)                                                                       \
  case NN:                                                                          \
    tp = (elem_bytes == 8) ? relax_tp<double, NN>() : relax_tp<float, NN>();       \
    break;
  switch (n) { C(8) C(16) C(32) C(64) C(128) C(256) C(512) default: return 0; }
#undef C
  return (n / (2 * tp)) * n;
}

void launch_finalize(const double* partial, int groups, SolveCtl* ctl, const SolveCfg& cfg, int* n_active,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, partial, groups, ctl, cfg, n_active);
}

__device__ void ctl_reset(SolveCtl& C) {
  C.done = 0;
  C.status = 0;
  C.iters = 0;
  C.cur = 0;
  C.out = 1;
  C.best = 2;
  C.result = 0;
  C.bad_seen = 0;
  C.passes = 0;
  C.last_bad = 0;
  C.final_bad = -1;
  C.resid = 0.0;
  C.resid_min = __builtin_huge_val();
  C.bad_frac = 0.0;
  C.mean_u = 0.0;
  for (int i = 0; i < kMaxHist; ++i) {
    C.hist[i] = -1.0;
    C.hist_bad[i] = -1.0;
  }
}

// a non-finite eps means a non-finite delta (or position): the element is decided at once as invalid
__device__ __forceinline__ void mark_invalid_input(SolveCtl& C) {
  if (!isfinite(C.eps)) {
    C.done = 1;
    C.status = kStatusInvalid;
  }
}

__global__ void k_ctl_init(SolveCtl* __restrict__ ctl, const double* __restrict__ eps, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  SolveCtl& C = ctl[b];
  ctl_reset(C);
  C.eps = eps[b];
  C.iters1 = 0;
  C.passes1 = 0;
  C.phase1_done = 1;
  mark_invalid_input(C);
}

// -1: the float32 phase met its tolerance on the initial guess itself, whose float64 form
// already sits in the float64 phase's first buffer
__device__ __forceinline__ int handoff_buffer(const SolveCtl& C) {
  if (!C.done) return C.cur;
  if (C.status == 0 && C.iters == 0) return -1;
  return (C.status == 0 && C.final_bad == 0) ? C.out : C.result;
}

// copies the selected buffer; with part != nullptr it also leaves per-workgroup sums of |x|
// and x (the layout k_absmean_final reads)
template <typename T>
__global__ void __launch_bounds__(256)
k_take_buffer(const SolveCtl* __restrict__ ctl, const T* __restrict__ U, int batch, size_t n3, double* __restrict__ dst,
              int handoff, double* __restrict__ part) {
  const int b = blockIdx.y;
  const int src = handoff ? handoff_buffer(ctl[b]) : ctl[b].result;
  if (src < 0) return;   // (handoff only: no reduction is requested there)
  const T* in = U + ((size_t)src * batch + b) * n3;
  double* out = dst + (size_t)b * n3;
  double sa = 0.0, sm = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double v = double(in[i]);
    out[i] = v;
    sa += fabs(v);
    sm += v;
  }
  if (!part) return;
  sa = wave_sum<64>(sa);
  sm = wave_sum<64>(sm);
  __shared__ double ra[4], rm[4];
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = sa;
    rm[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = ((ra[0] + ra[1]) + ra[2]) + ra[3];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = ((rm[0] + rm[1]) + rm[2]) + rm[3];
  }
}

// keeps eps (the float64 source's) and records the float32 phase's counts
__global__ void k_ctl_phase2(SolveCtl* __restrict__ ctl, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  SolveCtl& C = ctl[b];
  const int src = handoff_buffer(C);
  const bool invalid = C.status == kStatusInvalid;
  C.iters1 = C.iters + ((C.done && src == C.out) ? 1 : 0);
  C.passes1 = C.passes;
  C.phase1_done = C.done;
  ctl_reset(C);
  if (invalid) {
    C.done = 1;
    C.status = kStatusInvalid;
  }
}

static int absmean_groups(size_t n3) {
  size_t g = (n3 + 255) / 256;
  return int(g > 1024 ? 1024 : g);
}

static unsigned copy_groups(size_t n3) {
  const size_t g = (n3 + 255) / 256;
  return unsigned(g > 4096 ? 4096 : g);
}

void launch_handoff(SolveCtl* ctl, const float* U32, int batch, size_t n3, double* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_take_buffer<float>), dim3(copy_groups(n3), batch), dim3(256), 0, s, ctl, U32, batch, n3, dst,
                     1, nullptr);
  hipLaunchKernelGGL(k_ctl_phase2, dim3((batch + 63) / 64), dim3(64), 0, s, ctl, batch);
}

// ------------------------------------------------------------------ spherical approximation
__global__ void __launch_bounds__(256)
k_spherical(size_t n3, const double* __restrict__ S, double* __restrict__ u, double alpha, double lam,
            double* __restrict__ partial) {
  const int b = blockIdx.y;
  const double c4 = 4.0 * (1.0 - 1.0 / 3.0) * lam;
  const double vertex = -alpha / (2.0 * (1.0 - 1.0 / 3.0) * lam);
  const double* sb = S + (size_t)b * n3;
  double* ub = u + (size_t)b * n3;
  int nbad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
    const double bp = sb[i];   // B' = S at u = 0 (Hessian and nonlocal terms vanish)
    const double disc = alpha * alpha + c4 * bp;
    if (disc < 0.0) {
      ub[i] = vertex;
      ++nbad;
    } else {
      ub[i] = 2.0 * bp / (alpha + sqrt(disc));
    }
  }
  nbad = wave_sum<64>(nbad);
  __shared__ int rb[4];
  if ((threadIdx.x & 63) == 0) rb[threadIdx.x >> 6] = nbad;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[(size_t)b * gridDim.x + blockIdx.x] = double(((rb[0] + rb[1]) + rb[2]) + rb[3]);
}

__global__ void __launch_bounds__(256)
k_ctl_spherical(SolveCtl* __restrict__ ctl, const double* __restrict__ eps, const double* __restrict__ partial,
                int groups, size_t n3) {
  const int b = blockIdx.x;
  double nb = 0.0;
  for (int g = threadIdx.x; g < groups; g += 256) nb += partial[(size_t)b * groups + g];
  nb = wave_sum<64>(nb);
  __shared__ double rb[4];
  if ((threadIdx.x & 63) == 0) rb[threadIdx.x >> 6] = nb;
  __syncthreads();
  if (threadIdx.x != 0) return;
  SolveCtl& C = ctl[b];
  ctl_reset(C);
  C.eps = eps[b];
  C.iters1 = 0;
  C.passes1 = 0;
  C.phase1_done = 1;
  C.done = 1;
  C.status = 0;
  C.iters = 1;
  C.result = 0;
  C.resid = -1.0;       // not evaluated: the approximation is not a root of Eq. FullDGP2
  C.resid_min = -1.0;
  C.bad_frac = (((rb[0] + rb[1]) + rb[2]) + rb[3]) / double(n3);
  C.hist_bad[0] = C.bad_frac;
  mark_invalid_input(C);
}

void launch_spherical(size_t n3, int batch, const double* S, double* u, double alpha, double lam, double* partial,
                      SolveCtl* ctl, const double* eps, hipStream_t s) {
  const int g = int(std::min<size_t>(4096, (n3 + 255) / 256));
  hipLaunchKernelGGL(k_spherical, dim3(g, batch), dim3(256), 0, s, n3, S, u, alpha, lam, partial);
  hipLaunchKernelGGL(k_ctl_spherical, dim3(batch), dim3(256), 0, s, ctl, eps, partial, g, n3);
}

template <typename T>
void launch_take_result(const SolveCtl* ctl, const T* U, int batch, size_t n3, double* dst, double* scratch,
                        double* mean, hipStream_t s) {
  const int g = absmean_groups(n3);
  hipLaunchKernelGGL((k_take_buffer<T>), dim3(g, batch), dim3(256), 0, s, ctl, U, batch, n3, dst, 0, scratch);
  hipLaunchKernelGGL(k_absmean_final, dim3(batch), dim3(256), 0, s, scratch, g, n3, nullptr, mean);
}

template void launch_take_result<double>(const SolveCtl*, const double*, int, size_t, double*, double*, double*,
                                         hipStream_t);
template void launch_take_result<float>(const SolveCtl*, const float*, int, size_t, double*, double*, double*,
                                        hipStream_t);

void launch_ctl_init(SolveCtl* ctl, const double* eps, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3((batch + 63) / 64), dim3(64), 0, s, ctl, eps, batch);
}


size_t absmean_scratch_doubles(size_t n3, int batch) { return (size_t)absmean_groups(n3) * batch * 2; }

template <typename T>
void launch_absmean(size_t n3, const T* x, int batch, double* scratch, double* abs_mean, double* mean,
                    hipStream_t s) {
  const int g = absmean_groups(n3);
  hipLaunchKernelGGL((k_absmean_partial<T>), dim3(g, batch), dim3(256), 0, s, x, n3, scratch);
  hipLaunchKernelGGL(k_absmean_final, dim3(batch), dim3(256), 0, s, scratch, g, n3, abs_mean, mean);
}

void launch_pair_means(const double* part, int groups, size_t n3, int batch, double* out0, double* out1,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_absmean_final, dim3(batch), dim3(256), 0, s, part, groups, n3, out0, out1);
}

template void launch_relax<double>(int, const cx<double>*, double*, const double*, cx<double>*, double*,
                                   const double*, int, const SolveCfg&, const SolveCtl*, hipStream_t, hipEvent_t,
                                   hipEvent_t);
template void launch_relax<float>(int, const cx<float>*, float*, const float*, cx<float>*, double*,
                                  const double*, int, const SolveCfg&, const SolveCtl*, hipStream_t, hipEvent_t,
                                  hipEvent_t);
template void launch_absmean<double>(size_t, const double*, int, double*, double*, double*, hipStream_t);
template void launch_absmean<float>(size_t, const float*, int, double*, double*, double*, hipStream_t);
template void launch_absmean<long long>(size_t, const long long*, int, double*, double*, double*, hipStream_t);

}  // namespace dgp

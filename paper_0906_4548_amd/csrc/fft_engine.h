// Register-resident Stockham FFT for gfx950 (64-wide wavefronts, LDS exchanges).
//
// One N-point complex transform is carried by T = N / R threads.  Thread t of a
// transform holds R elements in registers; on entry and on exit element q of
// thread t is x[t + q*T] (natural order in both), so global loads and stores of
// a transform are coalesced whichever way the caller lays columns across lanes.
// Between radix stages the data goes through LDS through a caller-supplied
// accessor, so the same engine serves strided columns (one lane per column)
// and contiguous rows (consecutive lanes along the row).
//
// Stages follow the Stockham autosort formulation: a stage of radix r after a
// span Ns reads in[j + q*N/r], multiplies by W_{Ns*r}^{q*(j mod Ns)}, applies an
// r-point DFT and writes out[(j div Ns)*Ns*r + (j mod Ns) + q*Ns].  Twiddles
// come from a table tw[m] = exp(-2 pi i m / N) computed on the host in double
// precision.  DIR = -1 is the forward (e^{-i...}) transform, +1 the inverse
// (unnormalised).
#pragma once
#include <hip/hip_runtime.h>

namespace dgp {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }

// Streaming (nontemporal) global accesses for data that the same kernel will not touch again:
// on gfx950 they keep the last-level cache from filling with lines that would only be written
// back (stores) or evicted (loads) later, while the following pass reads its inputs.
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk(T(x.x), T(x.y));
}
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 x;
  x.x = v.x;
  x.y = v.y;
  __builtin_nontemporal_store(x, reinterpret_cast<v2*>(p));
}

// multiply by exp(DIR * i * pi/2 * m) for m = 1 (DIR=-1: -i), exact.
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  if constexpr (DIR < 0) return mk(a.y, -a.x);   // * (-i)
  else return mk(-a.y, a.x);                     // * (+i)
}

// Constants of the 16th roots of unity: cos(2 pi m / 16) for m = 0..4.
constexpr double kC16_1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kS16_1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kSqrtHalf = 0.70710678118654752440;

// multiply by W_16^m (DIR=-1: exp(-2 pi i m/16)), m compile-time.
template <int M, int DIR, typename T>
__device__ __forceinline__ cx<T> w16(cx<T> a) {
  constexpr int m = ((M % 16) + 16) % 16;
  const T c1 = T(kC16_1), s1 = T(kS16_1), h = T(kSqrtHalf);
  // angle theta = DIR * 2 pi m / 16; result = a * (cos theta + i sin theta)
  T cr, ci;
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return rot90<DIR>(a);
  else if constexpr (m == 8) return mk(-a.x, -a.y);
  else if constexpr (m == 12) return rot90<-DIR>(a);
  else {
    if constexpr (m == 1) { cr = c1; ci = s1; }
    else if constexpr (m == 2) { cr = h; ci = h; }
    else if constexpr (m == 3) { cr = s1; ci = c1; }
    else if constexpr (m == 5) { cr = -s1; ci = c1; }
    else if constexpr (m == 6) { cr = -h; ci = h; }
    else if constexpr (m == 7) { cr = -c1; ci = s1; }
    else if constexpr (m == 9) { cr = -c1; ci = -s1; }
    else if constexpr (m == 10) { cr = -h; ci = -h; }
    else if constexpr (m == 11) { cr = -s1; ci = -c1; }
    else if constexpr (m == 13) { cr = s1; ci = -c1; }
    else if constexpr (m == 14) { cr = h; ci = -h; }
    else { cr = c1; ci = -s1; }  // m == 15
    // sin(theta) carries the sign of DIR
    const T sn = (DIR < 0) ? -ci : ci;
    return mk(a.x * cr - a.y * sn, a.x * sn + a.y * cr);
  }
}

// In-register small DFTs, X[k] = sum_n x[n] exp(DIR 2 pi i n k / r), natural order in and out.
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a - b;
  a = a + b;
  b = t;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cx<T> t2 = v[1] + v[3], t3 = rot90<DIR>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // radix-2 x 4: even/odd 4-point DFTs, then twiddle W_8^k and combine
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  o[1] = w16<2, DIR>(o[1]);
  o[2] = w16<4, DIR>(o[2]);
  o[3] = w16<6, DIR>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = e[k] + o[k];
    v[k + 4] = e[k] - o[k];
  }
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // 4 x 4: columns n1 (stride 4 inputs), twiddle W_16^{n1 k2}, then rows
  cx<T> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = v[n1 + 4 * n2];
    dft4<DIR>(a[n1]);
  }
  a[1][1] = w16<1, DIR>(a[1][1]);
  a[1][2] = w16<2, DIR>(a[1][2]);
  a[1][3] = w16<3, DIR>(a[1][3]);
  a[2][1] = w16<2, DIR>(a[2][1]);
  a[2][2] = w16<4, DIR>(a[2][2]);
  a[2][3] = w16<6, DIR>(a[2][3]);
  a[3][1] = w16<3, DIR>(a[3][1]);
  a[3][2] = w16<6, DIR>(a[3][2]);
  a[3][3] = w16<9, DIR>(a[3][3]);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cx<T> b[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
    dft4<DIR>(b);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = b[k1];
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 16) dft16<DIR>(v);
  else static_assert(R == 2, "unsupported radix");
}

// Radix plans: R elements per thread, stage radices (first == R, others divide R).
template <int N> struct Plan;
template <> struct Plan<8>   { static constexpr int R = 8;  static constexpr int S = 1; static constexpr int r[5] = {8, 0, 0, 0, 0}; };
template <> struct Plan<16>  { static constexpr int R = 16; static constexpr int S = 1; static constexpr int r[5] = {16, 0, 0, 0, 0}; };
template <> struct Plan<32>  { static constexpr int R = 8;  static constexpr int S = 2; static constexpr int r[5] = {8, 4, 0, 0, 0}; };
template <> struct Plan<64>  { static constexpr int R = 8;  static constexpr int S = 2; static constexpr int r[5] = {8, 8, 0, 0, 0}; };
template <> struct Plan<128> { static constexpr int R = 16; static constexpr int S = 2; static constexpr int r[5] = {16, 8, 0, 0, 0}; };
template <> struct Plan<256> { static constexpr int R = 16; static constexpr int S = 2; static constexpr int r[5] = {16, 16, 0, 0, 0}; };
template <> struct Plan<512> { static constexpr int R = 8;  static constexpr int S = 3; static constexpr int r[5] = {8, 8, 8, 0, 0}; };

// Plans with at most 8 elements per thread (for kernels that keep extra per-element state).
template <int N> struct Plan8;
template <> struct Plan8<8>   { static constexpr int R = 8; static constexpr int S = 1; static constexpr int r[5] = {8, 0, 0, 0, 0}; };
template <> struct Plan8<16>  { static constexpr int R = 8; static constexpr int S = 2; static constexpr int r[5] = {8, 2, 0, 0, 0}; };
template <> struct Plan8<32>  { static constexpr int R = 8; static constexpr int S = 2; static constexpr int r[5] = {8, 4, 0, 0, 0}; };
template <> struct Plan8<64>  { static constexpr int R = 8; static constexpr int S = 2; static constexpr int r[5] = {8, 8, 0, 0, 0}; };
template <> struct Plan8<128> { static constexpr int R = 8; static constexpr int S = 3; static constexpr int r[5] = {8, 8, 2, 0, 0}; };
template <> struct Plan8<256> { static constexpr int R = 8; static constexpr int S = 3; static constexpr int r[5] = {8, 8, 4, 0, 0}; };
template <> struct Plan8<512> { static constexpr int R = 8; static constexpr int S = 3; static constexpr int r[5] = {8, 8, 8, 0, 0}; };

// Plans with 4 elements per thread (twice the threads per transform, more LDS exchanges).
template <int N> struct Plan4;
template <> struct Plan4<8>   { static constexpr int R = 4; static constexpr int S = 2; static constexpr int r[5] = {4, 2, 0, 0, 0}; };
template <> struct Plan4<16>  { static constexpr int R = 4; static constexpr int S = 2; static constexpr int r[5] = {4, 4, 0, 0, 0}; };
template <> struct Plan4<32>  { static constexpr int R = 4; static constexpr int S = 3; static constexpr int r[5] = {4, 4, 2, 0, 0}; };
template <> struct Plan4<64>  { static constexpr int R = 4; static constexpr int S = 3; static constexpr int r[5] = {4, 4, 4, 0, 0}; };
template <> struct Plan4<128> { static constexpr int R = 4; static constexpr int S = 4; static constexpr int r[5] = {4, 4, 4, 2, 0}; };
template <> struct Plan4<256> { static constexpr int R = 4; static constexpr int S = 4; static constexpr int r[5] = {4, 4, 4, 4, 0}; };
template <> struct Plan4<512> { static constexpr int R = 4; static constexpr int S = 5; static constexpr int r[5] = {4, 4, 4, 4, 2}; };

// Plan selection: 0 = at most 8 elements per thread (Plan8), 1 = up to 16 (Plan).
template <int N, int SEL> struct PlanPick { using type = Plan8<N>; };
template <int N> struct PlanPick<N, 1> { using type = Plan<N>; };
template <int N> struct PlanPick<N, 2> { using type = Plan4<N>; };

// One Stockham stage.  v: the thread's R registers.  lds: accessor with
// load(e), store(e, value) for element e of this thread's transform.  The
// caller guarantees a barrier-safe LDS region per transform.
template <typename T, int N, int R, int r, int Ns, bool FIRST, bool LAST, int DIR, class Lds>
__device__ __forceinline__ void fft_stage(cx<T> (&v)[R], const cx<T>* __restrict__ tw, Lds& lds, int t) {
  constexpr int TT = N / R;   // threads per transform
  constexpr int B = R / r;    // butterflies per thread in this stage
  static_assert(R % r == 0, "stage radix must divide R");
  static_assert(!FIRST || r == R, "first stage radix must be R");
  cx<T> x[R];
  if constexpr (FIRST) {
#pragma unroll
    for (int q = 0; q < R; ++q) x[q] = v[q];
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * TT;
#pragma unroll
      for (int q = 0; q < r; ++q) x[b * r + q] = lds.load(j + q * (N / r));
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * TT;
    if constexpr (Ns > 1) {
      const int k = j % Ns;
#pragma unroll
      for (int q = 1; q < r; ++q) {
        const cx<T> w = tw[(q * k * (N / (Ns * r))) & (N - 1)];
        x[b * r + q] = (DIR < 0) ? cmul(x[b * r + q], w) : cmulc(x[b * r + q], w);
      }
    }
    dft_small<r, DIR>(&x[b * r]);
  }
  if constexpr (!LAST) {
    lds.sync();
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * TT;
      const int base = (j / Ns) * Ns * r + (j % Ns);
#pragma unroll
      for (int q = 0; q < r; ++q) lds.store(base + q * Ns, x[b * r + q]);
    }
    lds.sync();
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int q = 0; q < r; ++q) v[b + q * B] = x[b * r + q];
  }
}

// Stages I..S-1 of plan P; NS is the span before stage I.
template <typename T, int N, class P, int DIR, int I, int NS, class Lds>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[P::R], const cx<T>* __restrict__ tw, Lds& lds, int t) {
  if constexpr (I < P::S) {
    fft_stage<T, N, P::R, P::r[I], NS, I == 0, I == P::S - 1, DIR>(v, tw, lds, t);
    fft_stages<T, N, P, DIR, I + 1, NS * P::r[I]>(v, tw, lds, t);
  }
}

// Full N-point transform with plan P.
template <typename T, int N, class P, int DIR, class Lds>
__device__ __forceinline__ void fft(cx<T> (&v)[P::R], const cx<T>* __restrict__ tw, Lds& lds, int t) {
  fft_stages<T, N, P, DIR, 0, 1>(v, tw, lds, t);
}

// Workgroup barrier that orders LDS traffic only.  __syncthreads() fences every address
// space, and on this architecture the load counter it must drain also counts outstanding
// global loads, so a barrier inside a transform would wait for the next tile's prefetch;
// with the fence restricted to LDS the prefetch stays in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS accessor for strided columns: element e of column c at base[e * C + c], with one padding
// row after every PG rows when PG > 0 (a first radix-r stage stores rows r apart; PG = r
// spreads them over the banks).  The region holds (N + N / PG) * C elements.
template <typename T, int C, int PG = 0>
struct LdsCol {
  cx<T>* base;
  int c;
  __device__ __forceinline__ int at(int e) const {
    const unsigned u = unsigned(e);
    return int(PG > 0 ? u + u / PG : u) * C + c;
  }
  __device__ __forceinline__ cx<T> load(int e) const { return base[at(e)]; }
  __device__ __forceinline__ void store(int e, cx<T> v) const { base[at(e)] = v; }
  __device__ __forceinline__ void sync() const { lds_barrier(); }
};

// padding of the axis-2 pass's LDS rows (measured: 4, 8, 16 and 32 within noise of each other)
#ifndef DGP_ROW_PAD
#define DGP_ROW_PAD 16
#endif
// LDS accessor for contiguous rows: element e of row c at base[c * (N + N/P) + e + e/P], P = kPad.
// WAVE: every row is carried by lanes of a single wavefront (N/R <= 64), so the row's LDS
// exchanges only need ordering within the wavefront, not a workgroup barrier.
template <typename T, int N, bool WAVE = false>
struct LdsRow {
  cx<T>* base;
  int c;
  static constexpr int kPad = DGP_ROW_PAD;   // one padding element after every kPad elements
  static constexpr int kStride = N + N / kPad;
  __device__ __forceinline__ int at(int e) const { return c * kStride + e + unsigned(e) / kPad; }
  __device__ __forceinline__ cx<T> load(int e) const { return base[at(e)]; }
  __device__ __forceinline__ void store(int e, cx<T> v) const { base[at(e)] = v; }
  __device__ __forceinline__ void sync() const {
    if constexpr (WAVE) wave_sync();
    else lds_barrier();
  }
};

}  // namespace dgp

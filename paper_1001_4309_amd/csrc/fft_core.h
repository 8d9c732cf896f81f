// Register/LDS Stockham FFT for rows held by TPR threads (gfx950).
//
// Layout: a length-L row is held by TPR threads, R = L / TPR values each;
// thread t holds element t + TPR * i in register slot i.  Every stage of the
// Stockham autosort (decimation in time) formulation reads its butterfly
// inputs x[j + k L/r] from exactly these slots, so the first stage runs
// straight from the values loaded from memory, the last stage leaves the
// output in natural order in the same slots, and an inverse transform can
// start from a forward transform's output with no exchange in between.
// Between stages the values go through LDS once (written in the stage's
// output order, read back as t + TPR * i), or, where they only move between
// lanes 16 or 32 apart, through lane swaps in registers.
//
// When TPR <= 64 a row lives inside one wavefront, so an exchange needs only
// wave-level ordering of the LDS accesses, no workgroup barrier.
//
// Published formulation restated here: Stockham autosort FFT as in
// C. Van Loan, "Computational Frameworks for the Fast Fourier Transform"
// (1992), in the per-butterfly form used for GPUs by Govindaraju et al.,
// "High performance discrete Fourier transforms on graphics processors" (2008):
// butterfly j of a radix-r stage with Ns outputs already combined takes
// x[j + k L/r], multiplies input k by exp(-+2 pi i k (j mod Ns) / (Ns r)),
// applies a length-r DFT and writes output k to (j / Ns) Ns r + (j mod Ns) + k Ns.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace sfd {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex products with the fused multiply-adds written out, so that every
// call site rounds the same way whatever the compiler's contraction choices
// around it (kernels that hold a transform differently then still agree
// bit for bit).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}

// cos and sin of 2 pi k / n as compile-time constants (double, rounded to
// float where used).  The angle is reduced exactly with integers to the
// nearest quarter turn q/4 plus a remainder f in [-1/8, 1/8] turn; sin and
// cos of 2 pi f come from their Taylor series (|2 pi f| <= pi/4: 14 terms
// reach double precision), then rotate by q quarter turns.
constexpr double kPi = 3.14159265358979323846264338327950288;
struct SinCos {
  double s, c;
};
constexpr SinCos sincos_turn(long k, long n) {
  const long m = ((k % n) + n) % n;         // angle 2 pi m / n, m in [0, n)
  const long q = (4 * m + n / 2) / n;       // nearest quarter turn (0..4)
  const double f = (double)(4 * m - q * n) / (double)(4 * n);  // remainder in turns
  const double t = 2.0 * kPi * f, t2 = t * t;
  double sn = t, cs = 1.0, ts = t, tc = 1.0;
  for (int i = 1; i < 14; ++i) {
    ts *= -t2 / (double)((2 * i) * (2 * i + 1));
    tc *= -t2 / (double)((2 * i - 1) * (2 * i));
    sn += ts;
    cs += tc;
  }
  switch (q % 4) {
    case 0: return {sn, cs};
    case 1: return {cs, -sn};
    case 2: return {-sn, -cs};
    default: return {-cs, sn};
  }
}

// a * exp(sgn 2 pi i K / N), sgn = -1 forward, +1 inverse.  Multiples of a
// quarter turn are exact sign/swap operations, odd multiples of an eighth
// turn use the common factor 1/sqrt(2).
template <int N, int K, bool INV>
__device__ __forceinline__ float2 mul_w(float2 a) {
  constexpr int k = ((K % N) + N) % N;
  constexpr SinCos w = sincos_turn(k, N);
  constexpr float c = static_cast<float>(w.c);
  constexpr float s = static_cast<float>(INV ? w.s : -w.s);
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == N) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * k == N || 4 * k == 3 * N) {
    if constexpr (s > 0) return make_float2(-a.y, a.x);
    else return make_float2(a.y, -a.x);
  } else if constexpr ((8 * k) % N == 0) {
    constexpr float h = 0.70710678118654752440f;
    constexpr float sc = c > 0 ? 1.f : -1.f;
    constexpr float ss = s > 0 ? 1.f : -1.f;
    return make_float2((sc * a.x - ss * a.y) * h, (ss * a.x + sc * a.y) * h);
  } else {
    return make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.x, s, a.y * c));
  }
}

template <int N, bool INV, int K = 0>
__device__ __forceinline__ void combine(float2 (&out)[N], const float2 (&e)[N / 2], const float2 (&o)[N / 2]) {
  if constexpr (K < N / 2) {
    const float2 w = mul_w<N, K, INV>(o[K]);
    out[K] = cadd(e[K], w);
    out[K + N / 2] = csub(e[K], w);
    combine<N, INV, K + 1>(out, e, o);
  }
}

// Length-N DFT for odd N from its symmetric pairs: with s_k = a_k + a_{N-k}
// and d_k = a_k - a_{N-k} (k = 1 .. (N-1)/2),
//   X_0 = a_0 + sum s_k,
//   X_m, X_{N-m} = a_0 + sum_k cos(2 pi k m / N) s_k  -/+ i sgn sum_k sin(2 pi k m / N) d_k,
// sgn = +1 forward, -1 inverse (the direct definition, regrouped).
template <int N, int M, int K = 0>
__device__ __forceinline__ void odd_sums(float2& re, float2& im, const float2 (&sp)[(N - 1) / 2],
                                         const float2 (&dp)[(N - 1) / 2]) {
  if constexpr (K < (N - 1) / 2) {
    constexpr SinCos w = sincos_turn((K + 1) * M, N);
    constexpr float c = static_cast<float>(w.c), s = static_cast<float>(w.s);
    re = make_float2(fmaf(c, sp[K].x, re.x), fmaf(c, sp[K].y, re.y));
    im = make_float2(fmaf(s, dp[K].x, im.x), fmaf(s, dp[K].y, im.y));
    odd_sums<N, M, K + 1>(re, im, sp, dp);
  }
}
template <int N, bool INV, int M = 1>
__device__ __forceinline__ void odd_outputs(float2 (&out)[N], float2 a0, const float2 (&sp)[(N - 1) / 2],
                                            const float2 (&dp)[(N - 1) / 2]) {
  if constexpr (M <= (N - 1) / 2) {
    float2 re = a0, im = make_float2(0.f, 0.f);
    odd_sums<N, M>(re, im, sp, dp);
    // Forward: X_m = re - i im, X_{N-m} = re + i im; inverse the other way.
    const float2 mi = INV ? make_float2(-im.y, im.x) : make_float2(im.y, -im.x);
    out[M] = cadd(re, mi);
    out[N - M] = csub(re, mi);
    odd_outputs<N, INV, M + 1>(out, a0, sp, dp);
  }
}

// Length-N DFT for odd N from its symmetric pairs: with s_k = a_k + a_{N-k}
// and d_k = a_k - a_{N-k} (k = 1 .. (N-1)/2) and t = 2 pi k m / N,
//   X_0 = a_0 + sum s_k,
//   X_m, X_{N-m} = (a_0 + sum_k cos(t) s_k) -/+ i sgn sum_k sin(t) d_k,
// sgn = +1 forward, -1 inverse (the definition with the terms k and N - k
// taken together).
template <int N, bool INV>
__device__ __forceinline__ void dft_odd(float2 (&a)[N]) {
  constexpr int H = (N - 1) / 2;
  float2 sp[H], dp[H];
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    sp[k - 1] = cadd(a[k], a[N - k]);
    dp[k - 1] = csub(a[k], a[N - k]);
  }
  float2 out[N];
  float2 x0 = a[0];
#pragma unroll
  for (int k = 0; k < H; ++k) x0 = cadd(x0, sp[k]);
  out[0] = x0;
  odd_outputs<N, INV>(out, a[0], sp, dp);
#pragma unroll
  for (int i = 0; i < N; ++i) a[i] = out[i];
}

// Split-radix combination (Duhamel and Hollmann, 1984): with E the DFT of
// the even samples, O1 and O3 those of the samples 1 and 3 mod 4, w the
// N-th root of unity of the transform's sign, and for k < N/4
//   s = w^k O1[k] + w^{3k} O3[k],  d = w^k O1[k] - w^{3k} O3[k],
// X[k] = E[k] + s, X[k + N/2] = E[k] - s, and X[k + N/4], X[k + 3N/4] =
// E[k + N/4] -/+ i d (forward; the signs swap for the inverse), since
// w^{N/4} = -i (forward) and w^{3N/4} = +i.
template <int N, bool INV, int K = 0>
__device__ __forceinline__ void split_combine(float2 (&out)[N], const float2 (&e)[N / 2], const float2 (&o1)[N / 4],
                                              const float2 (&o3)[N / 4]) {
  if constexpr (K < N / 4) {
    const float2 p = mul_w<N, K, INV>(o1[K]);
    const float2 q = mul_w<N, 3 * K, INV>(o3[K]);
    const float2 sm = cadd(p, q), df = csub(p, q);
    const float2 jd = INV ? make_float2(-df.y, df.x) : make_float2(df.y, -df.x);
    out[K] = cadd(e[K], sm);
    out[K + N / 2] = csub(e[K], sm);
    out[K + N / 4] = cadd(e[K + N / 4], jd);
    out[K + 3 * N / 4] = csub(e[K + N / 4], jd);
    split_combine<N, INV, K + 1>(out, e, o1, o3);
  }
}

// In-place length-N DFT of a register array (natural order in and out):
// split-radix decimation in time for N divisible by 4 (except 8), radix 2
// for other even N, down to a length-4 kernel, or to an odd length (3, 5, 7)
// evaluated from its symmetric pairs.
template <int N, bool INV>
__device__ __forceinline__ void dft(float2 (&a)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N % 2 == 1) {
    dft_odd<N, INV>(a);
  } else if constexpr (N == 2) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (N == 4) {
    const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const float2 t2 = cadd(a[1], a[3]);
    const float2 t3 = mul_w<4, 1, INV>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (N % 4 != 0 || N == 8) {
    // Radix 2 (for N = 8 it takes fewer instructions than the split form).
    float2 e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    dft<N / 2, INV>(e);
    dft<N / 2, INV>(o);
    combine<N, INV>(a, e, o);
  } else {
    // Split radix: the even samples as one half-length DFT, the samples
    // 1 mod 4 and 3 mod 4 as two quarter-length DFTs (see split_combine).
    float2 e[N / 2], o1[N / 4], o3[N / 4];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) e[i] = a[2 * i];
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      o1[i] = a[4 * i + 1];
      o3[i] = a[4 * i + 3];
    }
    dft<N / 2, INV>(e);
    dft<N / 4, INV>(o1);
    dft<N / 4, INV>(o3);
    split_combine<N, INV>(a, e, o1, o3);
  }
}

// Length-N DFT whose inputs N/2..N-1 are zero (they are not read).  Powers
// of two from 16: split radix, whose three parts have zero upper halves of
// their own.  Otherwise split by output parity, X[2m] = DFT_{N/2}(a)[m] and
// X[2m+1] = DFT_{N/2}(a w^j)[m], which drops the first level of additions.
template <int N, bool INV, int J = 0>
__device__ __forceinline__ void twist_half(float2 (&hi)[N / 2], const float2 (&a)[N]) {
  if constexpr (J < N / 2) {
    hi[J] = mul_w<N, J, INV>(a[J]);
    twist_half<N, INV, J + 1>(hi, a);
  }
}
template <int N, bool INV>
__device__ __forceinline__ void dft_half_in(float2 (&a)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N >= 16 && (N & (N - 1)) == 0) {
    // Split radix with each part's own zero upper half.
    float2 e[N / 2], o1[N / 4], o3[N / 4];
#pragma unroll
    for (int i = 0; i < N / 4; ++i) e[i] = a[2 * i];
#pragma unroll
    for (int i = 0; i < N / 8; ++i) {
      o1[i] = a[4 * i + 1];
      o3[i] = a[4 * i + 3];
    }
    dft_half_in<N / 2, INV>(e);
    dft_half_in<N / 4, INV>(o1);
    dft_half_in<N / 4, INV>(o3);
    split_combine<N, INV>(a, e, o1, o3);
  } else {
    float2 lo[N / 2], hi[N / 2];
#pragma unroll
    for (int j = 0; j < N / 2; ++j) lo[j] = a[j];
    twist_half<N, INV>(hi, a);
    dft<N / 2, INV>(lo);
    dft<N / 2, INV>(hi);
#pragma unroll
    for (int m = 0; m < N / 2; ++m) {
      a[2 * m] = lo[m];
      a[2 * m + 1] = hi[m];
    }
  }
}

// Outputs 0..N/2-1 of a length-N DFT (the others are left unspecified): the
// last decimation-in-time level without its subtractions.
template <int N, bool INV, int K = 0>
__device__ __forceinline__ void combine_low(float2 (&out)[N], const float2 (&e)[N / 2], const float2 (&o)[N / 2]) {
  if constexpr (K < N / 2) {
    out[K] = cadd(e[K], mul_w<N, K, INV>(o[K]));
    combine_low<N, INV, K + 1>(out, e, o);
  }
}
template <int N, bool INV>
__device__ __forceinline__ void dft_low_out(float2 (&a)[N]) {
  if constexpr (N == 1) {
    return;
  } else {
    float2 e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    dft<N / 2, INV>(e);
    dft<N / 2, INV>(o);
    combine_low<N, INV>(a, e, o);
  }
}

// ---------------------------------------------------------------------------
// Plans and twiddle tables.

template <int a, int... rest>
struct FirstOf {
  static constexpr int value = a;
};

template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
  static constexpr int product = (Rs * ...);
  static constexpr int first = FirstOf<Rs...>::value;
};

// A transform shape: length L held by TPR threads (R = L / TPR values each)
// and the radix order of its stages.  TPR <= 64 keeps a row inside one
// wavefront.
template <int L_, int TPR_, typename Rad_>
struct FftShape {
  static constexpr int L = L_;
  static constexpr int TPR = TPR_;
  static constexpr int R = L_ / TPR_;
  using Rad = Rad_;
  static_assert(Rad_::product == L_, "radices must multiply to L");
};

// Shapes of the row/column passes (one row per wavefront up to L = 2048).
template <int L>
struct PassPlan;
template <> struct PassPlan<64> : FftShape<64, 4, Radices<16, 4>> {};
template <> struct PassPlan<128> : FftShape<128, 8, Radices<16, 8>> {};
template <> struct PassPlan<256> : FftShape<256, 16, Radices<16, 16>> {};
template <> struct PassPlan<512> : FftShape<512, 32, Radices<16, 8, 4>> {};
template <> struct PassPlan<1024> : FftShape<1024, 64, Radices<16, 8, 8>> {};
template <> struct PassPlan<2048> : FftShape<2048, 64, Radices<32, 8, 8>> {};
// Smooth lengths between 1024 and 2048 (a hologram of 1024 samples with a
// view of 256, 512 or 768 needs L >= 1279, 1535, 1791): power-of-two stages
// first, the stage with the odd factor last (see stage_compute).
template <> struct PassPlan<1280> : FftShape<1280, 64, Radices<4, 4, 4, 20>> {};
template <> struct PassPlan<1536> : FftShape<1536, 64, Radices<8, 8, 24>> {};
template <> struct PassPlan<1792> : FftShape<1792, 64, Radices<4, 4, 4, 28>> {};
template <> struct PassPlan<4096> : FftShape<4096, 128, Radices<32, 16, 8>> {};
template <> struct PassPlan<8192> : FftShape<8192, 256, Radices<32, 16, 16>> {};

// Shapes of the single kernel-spectrum transforms: spread over a whole
// 256-thread workgroup so that one transform finishes quickly.
template <int L>
struct SpecPlan;
template <> struct SpecPlan<64> : FftShape<64, 8, Radices<8, 8>> {};
template <> struct SpecPlan<128> : FftShape<128, 16, Radices<8, 8, 2>> {};
template <> struct SpecPlan<256> : FftShape<256, 32, Radices<8, 8, 4>> {};
template <> struct SpecPlan<512> : FftShape<512, 64, Radices<8, 8, 8>> {};
template <> struct SpecPlan<1024> : FftShape<1024, 128, Radices<8, 8, 8, 2>> {};
template <> struct SpecPlan<2048> : FftShape<2048, 256, Radices<8, 8, 8, 4>> {};
template <> struct SpecPlan<1280> : PassPlan<1280> {};
template <> struct SpecPlan<1536> : PassPlan<1536> {};
template <> struct SpecPlan<1792> : PassPlan<1792> {};
template <> struct SpecPlan<4096> : FftShape<4096, 256, Radices<16, 16, 16>> {};
template <> struct SpecPlan<8192> : FftShape<8192, 256, Radices<32, 16, 16>> {};

// Twiddle table of a shape: for every stage after the first (Ns > 1), the
// entries exp(-2 pi i k jm / (Ns r)) stored as [k - 1][jm], k in [1, r),
// jm in [0, Ns), so that consecutive butterflies read consecutive entries.
template <typename Rad>
struct TwInfo;
template <int... Rs>
struct TwInfo<Radices<Rs...>> {
  static constexpr int S = sizeof...(Rs);
  static constexpr int r[S] = {Rs...};
  static constexpr int ns(int s) {
    int n = 1;
    for (int i = 0; i < s; ++i) n *= r[i];
    return n;
  }
  static constexpr int off(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += (r[i] - 1) * ns(i);
    return o;
  }
  static constexpr int total = off(S);
};

template <class P>
constexpr int twiddle_entries() {
  return TwInfo<typename P::Rad>::total;
}

// Global-memory access through address space 1, so that the compiler emits
// global (not flat) instructions with a scalar base and 32-bit offsets.
// (The host compilation pass only parses these; it never runs them.)
template <typename T>
__device__ __forceinline__ T gld(const T* p, unsigned i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((__attribute__((address_space(1))) const T*)p)[i];
#else
  return p[i];
#endif
}
template <typename T>
__device__ __forceinline__ void gst(T* p, unsigned i, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(1))) T*)p)[i] = v;
#else
  p[i] = v;
#endif
}

// Scheduling fence: the compiler may not move instructions across it.  Used
// to bound how far loads are hoisted, which otherwise inflates register use
// and costs occupancy.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// ---------------------------------------------------------------------------
// Exchanges.

template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    // LDS accesses of one wavefront are performed in order; this keeps the
    // compiler from moving them across the exchange.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
  // Stages are separate scheduling regions: no load of a later stage is
  // hoisted across the exchange (that would hold its registers meanwhile).
  __builtin_amdgcn_sched_barrier(0);
}

// LDS row padding: one spare 4-byte slot after every 32 (the LDS has 32
// banks and serves half a wavefront per cycle; with this padding the stride-r
// writes of a radix-32 first stage and the unit-stride reads both hit 32
// distinct banks).  Linear, so unrolled accesses keep immediate offsets.
__host__ __device__ constexpr int lds_pad(int p) { return p + (p >> 5); }
__host__ __device__ constexpr int lds_row_len(int L) { return L + L / 32; }

// Bytes of LDS one row needs for its exchanges.
template <int L, bool SPLIT>
constexpr int row_lds_bytes() {
  return lds_row_len(L) * (SPLIT ? 4 : 8);
}

// Padded LDS index of stage output k of a butterfly, split as a runtime base
// (per butterfly) plus a compile-time offset: pad(A + jm + k Ns) = wbase +
// woff(k) with A = (j - jm) r, a multiple of Ns r.  Exact for power-of-two
// Ns and r:
// - Ns a multiple of 32: k Ns is a multiple of 32, so its padding separates;
// - Ns r a multiple of 32 (Ns < 32): A is a multiple of 32, and jm plus
//   k Ns mod 32 stays below 32 (jm < Ns, and Ns divides 32), so the padding
//   of A + jm + k Ns is A/32 + floor(k Ns / 32);
// - Ns r below 32: A mod 32 + jm + k Ns < A mod 32 + Ns r <= 32, so the
//   padding is A/32 alone.
template <int r, int Ns>
__device__ __forceinline__ int lds_wbase(int j) {
  const int jm = j & (Ns - 1);
  const int A = (j - jm) * r;
  if constexpr (Ns % 32 == 0) return A + jm + ((A + jm) >> 5);
  else return A + (A >> 5) + jm;
}
template <int r, int Ns>
__device__ __forceinline__ constexpr int lds_woff(int k) {
  return (Ns % 32 == 0 || (Ns * r) % 32 == 0) ? k * Ns + ((k * Ns) >> 5) : k * Ns;
}
// Padded LDS index of element t + TPR i (exact when TPR is a multiple of 32;
// otherwise computed directly).
template <int TPR>
__device__ __forceinline__ int lds_ridx(int t, int i) {
  if constexpr (TPR % 32 == 0) return t + (t >> 5) + TPR * i + ((TPR * i) >> 5);
  else return lds_pad(t + TPR * i);
}

// Twiddles of one stage held in registers: for butterfly q of the thread
// (j = t + TPR q) and input k >= 1, exp(-2 pi i k (j mod Ns) / (Ns r)) from
// the stage's part of the table.  Loaded one stage ahead (before the previous
// stage's exchange) so that their latency overlaps the LDS round trip.
// Where a transform's twiddles come from: the table in global memory, a copy
// of it in LDS (same layout), computed on the fly (FP32 sincospi of the exact
// argument k jm / (Ns r)), or computed from one sincospi per butterfly with
// the powers w^k formed by squarings and products (at most 2 log2 r complex
// multiplications deep, so a few FP32 ulps).  The computed forms serve single
// transforms that run alone, where waiting for table reads would dominate.
enum TwSrc { kTwGlobal = 0, kTwShared = 1, kTwCompute = 2, kTwPower = 3 };

// When Ns divides TPR every butterfly of a thread has the same j mod Ns, so
// one set of twiddles serves them all (SAME): loaded once, held once.
template <int TPR, int R, int r, int Ns, int TWS = kTwGlobal>
struct StageTw {
  static constexpr int nb = R / r;
  static constexpr bool any = Ns > 1;
  static constexpr bool SAME = any && TPR % Ns == 0 && TWS != kTwPower;
  static constexpr int nq = SAME ? 1 : nb;
  float2 w[any ? nq : 1][any ? r - 1 : 1];
  __device__ __forceinline__ float2 get(int q, int k) const { return w[SAME ? 0 : q][k]; }
  __device__ __forceinline__ void begin(int) {}
  __device__ __forceinline__ void end(int) {}
  __device__ __forceinline__ void load(int t, const float2* __restrict__ tw) {
    if constexpr (any && TWS == kTwPower) {
#pragma unroll
      for (int q = 0; q < nb; ++q) {
        const unsigned jm = (unsigned)(t + TPR * q) & (unsigned)(Ns - 1);
        float sn, cs;
        sincospif(-2.0f * (float)jm / (float)(Ns * r), &sn, &cs);
        float2 p2[5];  // w^(2^b)
        p2[0] = make_float2(cs, sn);
#pragma unroll
        for (int b = 1; b < 5; ++b) p2[b] = cmul(p2[b - 1], p2[b - 1]);
#pragma unroll
        for (int k = 1; k < r; ++k) {
          float2 acc = make_float2(1.f, 0.f);
          bool first = true;
#pragma unroll
          for (int b = 0; b < 5; ++b)
            if ((k >> b) & 1) {
              acc = first ? p2[b] : cmul(acc, p2[b]);
              first = false;
            }
          w[q][k - 1] = acc;
        }
      }
    } else if constexpr (any) {
#pragma unroll
      for (int q = 0; q < nq; ++q) {
        const unsigned jm = (unsigned)(t + TPR * q) & (unsigned)(Ns - 1);
#pragma unroll
        for (int k = 1; k < r; ++k) {
          if constexpr (TWS == kTwCompute) {
            float sn, cs;
            sincospif(-2.0f * (float)(k * (int)jm) / (float)(Ns * r), &sn, &cs);
            w[q][k - 1] = make_float2(cs, sn);
          } else if constexpr (TWS == kTwShared) {
            w[q][k - 1] = tw[(k - 1) * Ns + (int)jm];
          } else {
            w[q][k - 1] = gld(tw, (unsigned)((k - 1) * Ns) + jm);
          }
        }
      }
    }
  }
};

// Twiddles of one stage fetched per butterfly, one butterfly ahead, so that
// two butterflies' worth are held at a time instead of the whole stage's.
// Used after a lane-swap exchange, which leaves no LDS round trip to hide a
// whole stage's twiddle loads behind and so gains nothing from loading them
// early.
template <int TPR, int R, int r, int Ns, int TWS>
struct StageTwStream {
  static_assert(TWS == kTwGlobal || TWS == kTwShared, "streamed twiddles come from a table");
  static constexpr int nb = R / r;
  float2 cur[r - 1], nxt[r - 1];
  const float2* tw;
  int t;
  __device__ __forceinline__ void fetch(float2 (&w)[r - 1], int q) const {
    const unsigned jm = (unsigned)(t + TPR * q) & (unsigned)(Ns - 1);
#pragma unroll
    for (int k = 1; k < r; ++k)
      w[k - 1] = TWS == kTwShared ? tw[(k - 1) * Ns + (int)jm] : gld(tw, (unsigned)((k - 1) * Ns) + jm);
  }
  __device__ __forceinline__ void load(int t_, const float2* tw_) {
    t = t_;
    tw = tw_;
    fetch(cur, 0);
  }
  __device__ __forceinline__ void begin(int q) {
    if (q + 1 < nb) fetch(nxt, q + 1);
  }
  __device__ __forceinline__ float2 get(int, int k) const { return cur[k]; }
  __device__ __forceinline__ void end(int q) {
    if (q + 1 < nb) {
#pragma unroll
      for (int k = 0; k < r - 1; ++k) cur[k] = nxt[k];
    }
  }
};

// Butterflies of one Stockham stage.  v[i] holds element t + TPR * i of the
// stage input.  The outputs stay in v (butterfly q's output k in slot
// q + k nb, which for the last stage is natural order) unless the exchange
// is complex (not SPLIT), in which case they go straight to the LDS buffer.
// PRUNE: 1 = the upper half of every butterfly's inputs is zero (the padded
// half of a forward transform's first stage); 2 = only the lower half of
// every butterfly's outputs is needed (the cropped half of an inverse
// transform's last stage; the slots of the upper half are left as they are).
template <int L, int TPR, int r, int Ns, bool INV, bool LAST, bool SPLIT, int PRUNE, class TWH>
__device__ __forceinline__ void stage_compute(float2 (&v)[L / TPR], void* __restrict__ buf, int t, TWH& W) {
  constexpr int R = L / TPR;
  constexpr int nb = R / r;
  static_assert(R % r == 0, "radix must divide the values per thread");
  // A radix that is not a power of two may only close a transform: the last
  // stage writes no exchange, and its twiddle index j mod Ns needs Ns a power
  // of two.
  static_assert((r <= 32 && (32 % r) == 0) || (LAST && (Ns & (Ns - 1)) == 0),
                "radices are powers of two up to 32, except in the last stage");
  float2* cbuf = static_cast<float2*>(buf);
#pragma unroll
  for (int q = 0; q < nb; ++q) {
    const int j = t + TPR * q;
    W.begin(q);
    float2 b[r];
    constexpr int kin = PRUNE == 1 ? r / 2 : r;
#pragma unroll
    for (int k = 0; k < kin; ++k) b[k] = v[q + k * nb];
#pragma unroll
    for (int k = kin; k < r; ++k) b[k] = make_float2(0.f, 0.f);  // not read by dft_half_in
    if constexpr (Ns > 1) {
#pragma unroll
      for (int k = 1; k < kin; ++k) b[k] = INV ? cmulc(b[k], W.get(q, k - 1)) : cmul(b[k], W.get(q, k - 1));
    }
    if constexpr (PRUNE == 1) dft_half_in<r, INV>(b);
    else if constexpr (PRUNE == 2) dft_low_out<r, INV>(b);
    else dft<r, INV>(b);
    W.end(q);
    if constexpr (nb > 1) sched_fence();
    if constexpr (LAST || SPLIT) {
      constexpr int kout = PRUNE == 2 ? r / 2 : r;
#pragma unroll
      for (int k = 0; k < kout; ++k) v[q + k * nb] = b[k];
    } else {
      const int wb = lds_wbase<r, Ns>(j);
#pragma unroll
      for (int k = 0; k < r; ++k) cbuf[wb + lds_woff<r, Ns>(k)] = b[k];
    }
  }
}

// Exchange after a stage: outputs (in LDS, or in v for SPLIT) are reloaded as
// element t + TPR * i of the next stage's input.
// An inactive row (active false) only meets the exchange's barriers.
template <int L, int TPR, int r, int Ns, bool SPLIT>
__device__ __forceinline__ void stage_exchange(float2 (&v)[L / TPR], void* __restrict__ buf, int t, bool active) {
  constexpr int R = L / TPR;
  constexpr int nb = R / r;
  constexpr bool WAVE = TPR <= 64;
  float2* cbuf = static_cast<float2*>(buf);
  float* fbuf = static_cast<float*>(buf);
  if constexpr (!SPLIT) {
    lds_sync<WAVE>();
    if (active) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cbuf[lds_ridx<TPR>(t, i)];
    }
    lds_sync<WAVE>();
  } else {
    // Real parts, then imaginary parts, through a float buffer of L slots.
    if (active) {
#pragma unroll
      for (int q = 0; q < nb; ++q) {
        const int wb = lds_wbase<r, Ns>(t + TPR * q);
#pragma unroll
        for (int k = 0; k < r; ++k) fbuf[wb + lds_woff<r, Ns>(k)] = v[q + k * nb].x;
      }
    }
    lds_sync<WAVE>();
    // In place: every old real part is already in LDS.
    if (active) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[i].x = fbuf[lds_ridx<TPR>(t, i)];
    }
    lds_sync<WAVE>();
    if (active) {
#pragma unroll
      for (int q = 0; q < nb; ++q) {
        const int wb = lds_wbase<r, Ns>(t + TPR * q);
#pragma unroll
        for (int k = 0; k < r; ++k) fbuf[wb + lds_woff<r, Ns>(k)] = v[q + k * nb].y;
      }
    }
    lds_sync<WAVE>();
    if (active) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[i].y = fbuf[lds_ridx<TPR>(t, i)];
    }
    lds_sync<WAVE>();
  }
}

// Lane swaps.  v_permlane32_swap exchanges the upper 32 lanes of its first
// operand with the lower 32 lanes of its second; v_permlane16_swap exchanges
// the odd 16-lane rows of its first operand with the even rows of its second.
// Either way, with a value bound for the lower lanes (lane bit clear) first
// and one bound for the upper lanes second, every lane is left holding the
// value that came from a lower lane first and the one from an upper lane
// second.
template <int D>
__device__ __forceinline__ void swap_lanes(float2& x, float2& y) {
  static_assert(D == 16 || D == 32, "lane swaps exist at distance 16 and 32");
  const uint32_t ax = __float_as_uint(x.x), ay = __float_as_uint(x.y);
  const uint32_t bx = __float_as_uint(y.x), by = __float_as_uint(y.y);
  if constexpr (D == 32) {
    const auto re = __builtin_amdgcn_permlane32_swap(ax, bx, false, false);
    const auto im = __builtin_amdgcn_permlane32_swap(ay, by, false, false);
    x = make_float2(__uint_as_float(re[0]), __uint_as_float(im[0]));
    y = make_float2(__uint_as_float(re[1]), __uint_as_float(im[1]));
  } else {
    const auto re = __builtin_amdgcn_permlane16_swap(ax, bx, false, false);
    const auto im = __builtin_amdgcn_permlane16_swap(ay, by, false, false);
    x = make_float2(__uint_as_float(re[0]), __uint_as_float(im[0]));
    y = make_float2(__uint_as_float(re[1]), __uint_as_float(im[1]));
  }
}

// Exchange after stage (Ns, r) of a row of TPR <= 64 threads when Ns >= 16
// and m = TPR / Ns divides r.  Butterfly q of thread t (j = t + TPR q) writes
// output k to element (t - t mod Ns + TPR q) r + t mod Ns + Ns k, which is
// lane t mod Ns + Ns (k mod m) of the row, slot (t / Ns)(r / m) + q r + k / m:
// only the lane bits above Ns change, from the source group g = t / Ns to the
// destination group k mod m.  One round of lane swaps per such bit (distance
// Ns, and 2 Ns when m = 4) moves every value to its lane in registers, with
// no LDS round trip and no wait; the values then sit by source group g.
template <int TPR, int r, int Ns, bool SPLIT>
constexpr bool kLaneSwap = SPLIT && TPR <= 64 && Ns >= 16 && Ns < TPR && TPR % Ns == 0 &&
                           r % (TPR / Ns) == 0 && (r & (r - 1)) == 0;

template <int TPR, int R, int r, int Ns>
__device__ __forceinline__ void lane_swap_exchange(float2 (&v)[R]) {
  constexpr int nb = R / r;
  constexpr int m = TPR / Ns;
  static_assert(m == 2 || m == 4, "one or two rounds of lane swaps");
  float2 w[R];
#pragma unroll
  for (int q = 0; q < nb; ++q) {
#pragma unroll
    for (int kk = 0; kk < r / m; ++kk) {
      float2 e[m];  // indexed by destination group, then by source group
#pragma unroll
      for (int c = 0; c < m; ++c) e[c] = v[q + (kk * m + c) * nb];
#pragma unroll
      for (int c = 0; c < m; c += 2) swap_lanes<Ns>(e[c], e[c + 1]);
      if constexpr (m == 4) {
        swap_lanes<2 * Ns>(e[0], e[2]);
        swap_lanes<2 * Ns>(e[1], e[3]);
      }
#pragma unroll
      for (int g = 0; g < m; ++g) w[g * (r / m) + q * r + kk] = e[g];
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = w[i];
}

// Stage (Ns, r) with its twiddles W already loaded (or, streamed, their
// first butterfly's); loads the next stage's before this stage's exchange.
template <int L, int TPR, bool INV, bool SPLIT, int TWS, bool HALF, int Ns, int OFF, int r, int... rest, class TWH>
__device__ __forceinline__ void fft_stages(float2 (&v)[L / TPR], void* buf, int t, const float2* tw, TWH& W,
                                           bool active) {
  constexpr bool last = sizeof...(rest) == 0;
  constexpr int prune = !HALF ? 0 : (!INV && Ns == 1) ? 1 : (INV && last) ? 2 : 0;
  if (active) stage_compute<L, TPR, r, Ns, INV, last, SPLIT, prune>(v, buf, t, W);
  if constexpr (!last) {
    constexpr int next_off = OFF + (Ns > 1 ? (r - 1) * Ns : 0);
    constexpr int rn = Radices<rest...>::first;
    if constexpr (kLaneSwap<TPR, r, Ns, SPLIT>) {
      using Full = StageTw<TPR, L / TPR, rn, Ns * r, TWS>;
      using Stream = StageTwStream<TPR, L / TPR, rn, Ns * r, TWS>;
      constexpr bool stream = !Full::SAME && Full::nq > 1 && (TWS == kTwGlobal || TWS == kTwShared);
      std::conditional_t<stream, Stream, Full> Wn{};
      if (active) {
        Wn.load(t, tw + next_off);
        lane_swap_exchange<TPR, L / TPR, r, Ns>(v);
      }
      __builtin_amdgcn_sched_barrier(0);
      fft_stages<L, TPR, INV, SPLIT, TWS, HALF, Ns * r, next_off, rest...>(v, buf, t, tw, Wn, active);
    } else {
      StageTw<TPR, L / TPR, rn, Ns * r, TWS> Wn{};
      if (active) Wn.load(t, tw + next_off);
      stage_exchange<L, TPR, r, Ns, SPLIT>(v, buf, t, active);
      fft_stages<L, TPR, INV, SPLIT, TWS, HALF, Ns * r, next_off, rest...>(v, buf, t, tw, Wn, active);
    }
  }
}

template <class P, bool INV, bool SPLIT, int TWS, bool HALF, int r0, int... Rs>
__device__ __forceinline__ void fft_run(Radices<r0, Rs...>, float2 (&v)[P::R], void* buf, int t, const float2* tw,
                                        bool active) {
  StageTw<P::TPR, P::R, r0, 1, TWS> W0{};  // the first stage has no twiddles
  fft_stages<P::L, P::TPR, INV, SPLIT, TWS, HALF, 1, 0, r0, Rs...>(v, buf, t, tw, W0, active);
}

// Forward (INV = false) or unnormalised inverse (INV = true) FFT of one row
// of shape P.  ``buf`` is the row's LDS exchange buffer
// (row_lds_bytes<P::L, SPLIT>() bytes); ``tw`` is the twiddle table of P in
// global memory (kTwGlobal) or LDS (kTwShared), unused with kTwCompute.
// HALF: a forward transform whose input's upper half (elements L/2..L-1) is
// zero, or an inverse transform of which only the lower half of the output
// is used; the first (forward) or last (inverse) stage skips that half.
// active false: the row computes nothing and only meets the barriers of a
// transform whose row spans several wavefronts (v is left as it was).
template <class P, bool INV, bool SPLIT, int TWS = kTwGlobal, bool HALF = false>
__device__ __forceinline__ void fft_row(float2 (&v)[P::R], void* buf, int t, const float2* tw, bool active = true) {
  fft_run<P, INV, SPLIT, TWS, HALF>(typename P::Rad{}, v, buf, t, tw, active);
}

// Twiddle table entry e of a shape's table (layout of TwInfo), evaluated in FP64
// and rounded once.  Returns false past the end of the table.
template <int Ns, int OFF, int r, int... rest>
__device__ __forceinline__ bool twiddle_find(int e, float2* out) {
  if constexpr (Ns > 1) {
    constexpr int cnt = (r - 1) * Ns;
    if (e >= OFF && e < OFF + cnt) {
      const int rel = e - OFF;
      const int k = rel / Ns + 1;
      const int jm = rel - (k - 1) * Ns;
      double sn, cs;
      sincospi(-2.0 * (double)(k * jm) / (double)(Ns * r), &sn, &cs);
      *out = make_float2((float)cs, (float)sn);
      return true;
    }
  }
  if constexpr (sizeof...(rest) > 0) {
    return twiddle_find<Ns * r, OFF + (Ns > 1 ? (r - 1) * Ns : 0), rest...>(e, out);
  } else {
    return false;
  }
}

template <int... Rs>
__device__ __forceinline__ bool twiddle_entry_r(Radices<Rs...>, int e, float2* out) {
  return twiddle_find<1, 0, Rs...>(e, out);
}

template <class P>
__device__ __forceinline__ bool twiddle_entry(int e, float2* out) {
  return twiddle_entry_r(typename P::Rad{}, e, out);
}

}  // namespace sfd

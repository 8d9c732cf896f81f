// Register/LDS Stockham FFT for one row per group of TPR threads (gfx950).
//
// Layout: a length-L row is held by TPR threads, R = L / TPR values each;
// thread t holds element t + TPR * i in register slot i.  Every stage of the
// Stockham autosort (decimation in time) formulation reads its butterfly
// inputs x[j + k L/r] from exactly these slots, so the first stage runs
// straight from the values loaded from HBM, the last stage leaves the output
// in natural order in the same slots, and an inverse transform can start
// from a forward transform's output with no exchange in between.  Between
// stages the values go through LDS once (write in the stage's output order,
// read back as t + TPR * i).
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

namespace sfd {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// cos(2 pi k / 32) for k = 0..8; other angles follow by symmetry.
constexpr double kCos32[9] = {1.0,
                              0.98078528040323044912618223613424,
                              0.92387953251128675612818318939679,
                              0.83146961230254523707878837761791,
                              0.70710678118654752440084436210485,
                              0.55557023301960222474283081394853,
                              0.38268343236508977172845998403040,
                              0.19509032201612826784828486847702,
                              0.0};

constexpr double cos32(int k) {
  k = ((k % 32) + 32) % 32;
  return k <= 8 ? kCos32[k] : k <= 16 ? -kCos32[16 - k] : k <= 24 ? -kCos32[k - 16] : kCos32[32 - k];
}
constexpr double sin32(int k) { return cos32(k - 8); }

// a * exp(sgn 2 pi i K / N), sgn = -1 forward, +1 inverse; N divides 32.
template <int N, int K, bool INV>
__device__ __forceinline__ float2 mul_w(float2 a) {
  constexpr int k32 = ((K * (32 / N)) % 32 + 32) % 32;
  constexpr float c = static_cast<float>(cos32(k32));
  constexpr float s = static_cast<float>(INV ? sin32(k32) : -sin32(k32));
  if constexpr (k32 == 0) {
    return a;
  } else if constexpr (k32 == 16) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (k32 == 8 || k32 == 24) {
    // multiply by i * s with s = +-1
    if constexpr (s > 0) return make_float2(-a.y, a.x);
    else return make_float2(a.y, -a.x);
  } else if constexpr (k32 % 8 == 4) {
    constexpr float h = 0.70710678118654752440f;
    constexpr float sc = c > 0 ? 1.f : -1.f;
    constexpr float ss = s > 0 ? 1.f : -1.f;
    return make_float2((sc * a.x - ss * a.y) * h, (ss * a.x + sc * a.y) * h);
  } else {
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
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

// In-place length-N DFT of a register array (natural order in and out),
// radix-2 decimation in time down to a length-4 kernel.
template <int N, bool INV>
__device__ __forceinline__ void dft(float2 (&a)[N]) {
  if constexpr (N == 1) {
    return;
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
  } else {
    float2 e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    dft<N / 2, INV>(e);
    dft<N / 2, INV>(o);
    combine<N, INV>(a, e, o);
  }
}

// LDS row padding: one spare slot after every 16 elements.
__host__ __device__ constexpr int lds_pad(int p) { return p + (p >> 4); }
__host__ __device__ constexpr int lds_row_len(int L) { return L + L / 16; }

// One Stockham stage.  v[i] holds element t + TPR * i of the stage input.
// If LAST, the stage output replaces v in natural order; otherwise it goes
// through the row's LDS buffer and v is reloaded in the same t + TPR * i
// layout.  ``tw`` is exp(-2 pi i e / L), e in [0, L).
template <int L, int TPR, int r, int Ns, bool INV, bool LAST>
__device__ __forceinline__ void fft_stage(float2 (&v)[L / TPR], float2* __restrict__ buf, int t,
                                          const float2* __restrict__ tw) {
  constexpr int R = L / TPR;
  constexpr int nb = R / r;
  static_assert(R % r == 0, "radix must divide the values per thread");
#pragma unroll
  for (int q = 0; q < nb; ++q) {
    const int j = t + TPR * q;
    float2 b[r];
#pragma unroll
    for (int k = 0; k < r; ++k) b[k] = v[q + k * nb];
    if constexpr (Ns > 1) {
      const int jm = j & (Ns - 1);
      constexpr int step = L / (Ns * r);
#pragma unroll
      for (int k = 1; k < r; ++k) {
        const float2 w = tw[k * jm * step];
        b[k] = INV ? cmulc(b[k], w) : cmul(b[k], w);
      }
    }
    dft<r, INV>(b);
    if constexpr (LAST) {
#pragma unroll
      for (int k = 0; k < r; ++k) v[q + k * nb] = b[k];
    } else {
      const int jm = j & (Ns - 1);
      const int base = (j - jm) * r + jm;
#pragma unroll
      for (int k = 0; k < r; ++k) buf[lds_pad(base + k * Ns)] = b[k];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = buf[lds_pad(t + TPR * i)];
    __syncthreads();
  }
}

template <int L, int TPR, bool INV, int Ns, int r, int... rest>
__device__ __forceinline__ void fft_stages(float2 (&v)[L / TPR], float2* __restrict__ buf, int t,
                                           const float2* __restrict__ tw) {
  constexpr bool last = sizeof...(rest) == 0;
  fft_stage<L, TPR, r, Ns, INV, last>(v, buf, t, tw);
  if constexpr (!last) fft_stages<L, TPR, INV, Ns * r, rest...>(v, buf, t, tw);
}

template <int... Rs>
struct Radices {
  static constexpr int product = (Rs * ...);
};

// Transform plan per length: threads per row, values per thread, radix order.
template <int L>
struct FftPlan;
template <> struct FftPlan<64> { static constexpr int TPR = 4; using Rad = Radices<16, 4>; };
template <> struct FftPlan<128> { static constexpr int TPR = 8; using Rad = Radices<16, 8>; };
template <> struct FftPlan<256> { static constexpr int TPR = 16; using Rad = Radices<16, 16>; };
template <> struct FftPlan<512> { static constexpr int TPR = 32; using Rad = Radices<16, 8, 4>; };
template <> struct FftPlan<1024> { static constexpr int TPR = 64; using Rad = Radices<16, 8, 8>; };
template <> struct FftPlan<2048> { static constexpr int TPR = 128; using Rad = Radices<16, 16, 8>; };
template <> struct FftPlan<4096> { static constexpr int TPR = 256; using Rad = Radices<16, 16, 16>; };
template <> struct FftPlan<8192> { static constexpr int TPR = 256; using Rad = Radices<32, 16, 16>; };

template <int L, bool INV, int... Rs>
__device__ __forceinline__ void fft_run(Radices<Rs...>, float2 (&v)[L / FftPlan<L>::TPR], float2* buf, int t,
                                        const float2* tw) {
  static_assert(Radices<Rs...>::product == L, "radices must multiply to L");
  fft_stages<L, FftPlan<L>::TPR, INV, 1, Rs...>(v, buf, t, tw);
}

// Forward (INV = false) or unnormalised inverse (INV = true) FFT of one row.
template <int L, bool INV>
__device__ __forceinline__ void fft_row(float2 (&v)[L / FftPlan<L>::TPR], float2* buf, int t, const float2* tw) {
  fft_run<L, INV>(typename FftPlan<L>::Rad{}, v, buf, t, tw);
}

}  // namespace sfd

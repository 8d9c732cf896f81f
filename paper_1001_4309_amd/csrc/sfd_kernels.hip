// HIP kernels for batched Shifted-Fresnel reconstruction on gfx950.
//
//  tables_kernel   chirp tables of Eqs. (2)-(4) per view and axis, phases in
//                  FP64 reduced to [-1, 1] half-turns before sin/cos, plus the
//                  FFT twiddle tables.
//  spectrum_kernel FFT_L(h) / L per view and axis (steps 5-6 of Section 2.2,
//                  done per axis because h of Eq. (4) is separable).
//  pass_kernel     one padded 1D chirp convolution per row, fused:
//                  load row, multiply by the pre-chirp (step 3), zero-pad
//                  (step 2), FFT (step 4), multiply by the kernel spectrum
//                  (step 7), inverse FFT (step 8), crop (step 9), and either
//                  the post-chirp or |.|^2 (step 10, Eq. 5); the row's
//                  outputs are stored transposed so the next axis again
//                  reads contiguous rows.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "sfd_internal.h"

namespace sfd {

// exp(i pi v) with v reduced to [-1, 1] in FP64 first, then evaluated in FP64
// and rounded once to complex64.
__device__ __forceinline__ float2 cispi_f64(double v) {
  const double r = v - 2.0 * rint(0.5 * v);
  double s, c;
  sincospi(r, &s, &c);
  return make_float2(static_cast<float>(c), static_cast<float>(s));
}

// The same phase carried entirely in FP32 (comparison variant).
__device__ __forceinline__ float2 cispi_f32(float v) {
  const float r = v - 2.0f * rintf(0.5f * v);
  float s, c;
  sincospif(r, &s, &c);
  return make_float2(c, s);
}

__device__ __forceinline__ float2 pre_value(const AxisJob& J, int m) {
  if (J.flags & kPhaseFp32) {
    const float p0 = (float)J.p0, a0 = (float)J.a0, il = (float)J.inv_lz, S = (float)J.S, c1 = (float)J.c1;
    const float fm = (float)m;
    const float x0 = fm * p0 + a0;
    float2 v = cispi_f32(x0 * x0 * il - 2.0f * fm * S * c1 - S * fm * fm);
    if (J.flags & kMomentX0) {
      const float w = x0 * (float)J.wscale;
      v = make_float2(v.x * w, v.y * w);
    }
    return v;
  }
  const double dm = (double)m;
  const double x0 = dm * J.p0 + J.a0;
  float2 v = cispi_f64(x0 * x0 * J.inv_lz - 2.0 * dm * J.S * J.c1 - J.S * (double)((int64_t)m * m));
  if (J.flags & kMomentX0) {
    const float w = (float)(x0 * J.wscale);
    v = make_float2(v.x * w, v.y * w);
  }
  return v;
}

__device__ __forceinline__ float2 post_value(const AxisJob& J, int m) {
  if (J.flags & kPhaseFp32) {
    const float p1 = (float)J.p1, a1 = (float)J.a1, a0 = (float)J.a0, il = (float)J.inv_lz, S = (float)J.S;
    const float fm = (float)m;
    const float x1 = fm * p1 + a1;
    return cispi_f32(x1 * x1 * il - 2.0f * a0 * x1 * il - S * fm * fm);
  }
  const double dm = (double)m;
  const double x1 = dm * J.p1 + J.a1;
  return cispi_f64(x1 * x1 * J.inv_lz - 2.0 * J.a0 * x1 * J.inv_lz - J.S * (double)((int64_t)m * m));
}

// h of Eq. (4) at storage index i in [0, L): lag k = i for i < n1, k = i - L
// otherwise; zero outside k in [-(n0-1), n1-1].
__device__ __forceinline__ float2 kernel_value(const AxisJob& J, int i) {
  const int k = i < J.n1 ? i : i - J.L;
  if (k < -(J.n0 - 1)) return make_float2(0.f, 0.f);
  if (J.flags & kPhaseFp32) {
    const float fk = (float)k;
    return cispi_f32((float)J.S * fk * fk);
  }
  return cispi_f64(J.S * (double)((int64_t)k * k));
}

// grid: x covers max(n0 + n1 + L) entries per job, y = jobs then twiddle tables.
__global__ void __launch_bounds__(256) tables_kernel(const AxisJob* __restrict__ jobs, int njobs,
                                                     const TwiddleJob* __restrict__ tws, int ntw) {
  const int y = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (y < njobs) {
    const AxisJob J = jobs[y];
    if (i < J.n0) {
      J.pre[i] = pre_value(J, i);
    } else if (i < J.n0 + J.n1) {
      if (J.post) J.post[i - J.n0] = post_value(J, i - J.n0);
    } else if (i < J.n0 + J.n1 + J.L) {
      const int e = i - J.n0 - J.n1;
      J.H[e] = kernel_value(J, e);
    }
  } else if (y - njobs < ntw) {
    const TwiddleJob T = tws[y - njobs];
    if (i < T.L) {
      double s, c;
      sincospi(-2.0 * (double)i / (double)T.L, &s, &c);
      T.tw[i] = make_float2((float)c, (float)s);
    }
  }
}

// One workgroup per (view, axis) job of length L: H <- FFT(h) / L in place.
template <int L>
__global__ void __launch_bounds__(FftPlan<L>::TPR) spectrum_kernel(const AxisJob* __restrict__ jobs, int first,
                                                                   const float2* __restrict__ tw) {
  constexpr int TPR = FftPlan<L>::TPR;
  constexpr int R = L / TPR;
  __shared__ float2 lds[lds_row_len(L)];
  const AxisJob& J = jobs[first + blockIdx.x];
  float2* H = J.H;
  const int t = threadIdx.x;
  float2 v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = H[t + TPR * i];
  fft_row<L, false>(v, lds, t, tw);
  const float inv = 1.0f / (float)L;
#pragma unroll
  for (int i = 0; i < R; ++i) H[t + TPR * i] = make_float2(v[i].x * inv, v[i].y * inv);
}

template <int L>
struct PassShape {
  static constexpr int TPR = FftPlan<L>::TPR;
  static constexpr int R = L / TPR;
  static constexpr int G = (8192 / L) * TPR <= 512 ? 8192 / L : 512 / TPR;  // rows per workgroup
  static constexpr int THREADS = G * TPR;
};

// Map a workgroup to a tile so that consecutive tiles (which write adjacent
// pieces of the same cache lines in the transposed store) run on the same
// XCD: workgroups are dispatched round-robin over the 8 XCDs.
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int per = total >> 3;
  if ((total & 7) != 0 || per == 0) return b;
  return (b & 7) * per + (b >> 3);
}

template <int L>
__global__ void __launch_bounds__(PassShape<L>::THREADS) pass_kernel(const PassArgs args,
                                                                     const float2* __restrict__ tw) {
  constexpr int TPR = PassShape<L>::TPR;
  constexpr int R = PassShape<L>::R;
  constexpr int G = PassShape<L>::G;
  constexpr int ROWLEN = lds_row_len(L);
  __shared__ float2 lds[G * ROWLEN];

  const int tile = xcd_tile(blockIdx.x, args.total_tiles);
  // Job containing this tile (binary search over the prefix in kernel arguments).
  int lo = 0, hi = args.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args.tile_prefix[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const RowJob J = args.jobs[lo];
  const int row0 = (tile - args.tile_prefix[lo]) * G;
  const int g = threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  const int row = row0 + g;
  const bool valid = row < J.n_rows;
  float2* buf = lds + g * ROWLEN;

  // Steps 2-3: load the row times the pre-chirp, zero beyond n_in.
  float2 v[R];
  if (J.mode & kInReal) {
    const float* in = static_cast<const float*>(J.in) + (int64_t)(valid ? row : 0) * J.in_ld;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      if (valid && m < J.n_in) {
        const float a = in[m];
        const float2 p = J.pre[m];
        v[i] = make_float2(a * p.x, a * p.y);
      } else {
        v[i] = make_float2(0.f, 0.f);
      }
    }
  } else {
    const float2* in = static_cast<const float2*>(J.in) + (int64_t)(valid ? row : 0) * J.in_ld;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      v[i] = (valid && m < J.n_in) ? cmul(in[m], J.pre[m]) : make_float2(0.f, 0.f);
    }
  }

  // Step 4: forward FFT; step 7: multiply by FFT(h)/L; step 8: inverse FFT.
  fft_row<L, false>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = cmul(v[i], J.H[t + TPR * i]);
  fft_row<L, true>(v, buf, t, tw);

  // Steps 9-10: crop to n_out, post-chirp and/or |.|^2, transposed store
  // staged through LDS so that G consecutive rows are written together.
  const int n_out = J.n_out;
  const int SP = n_out + 1;  // staging stride per row (odd, against bank conflicts)
  if (J.mode & kUsePost) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      if (m < n_out) v[i] = cmul(v[i], J.post[m]);
    }
  }
  if (J.mode & kUseScale) {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = cmul(v[i], J.scale);
  }
  if (J.mode & kOutField) {
    __syncthreads();
    float2* st = lds + g * SP;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      if (m < n_out) st[m] = v[i];
    }
    __syncthreads();
    float2* out = static_cast<float2*>(J.out);
    for (int e = threadIdx.x; e < G * n_out; e += G * TPR) {
      const int m = e / G;
      const int gg = e - m * G;
      if (row0 + gg < J.n_rows) out[(int64_t)m * J.out_ld + row0 + gg] = lds[gg * SP + m];
    }
  }
  if (J.mode & kOutIntensity) {
    __syncthreads();
    float* st = reinterpret_cast<float*>(lds) + g * SP;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      if (m < n_out) st[m] = (v[i].x * v[i].x + v[i].y * v[i].y) * J.iscale;
    }
    __syncthreads();
    const float* sb = reinterpret_cast<const float*>(lds);
    float* out = (J.mode & kOutField) ? J.out2 : static_cast<float*>(J.out);
    for (int e = threadIdx.x; e < G * n_out; e += G * TPR) {
      const int m = e / G;
      const int gg = e - m * G;
      if (row0 + gg < J.n_rows) out[(int64_t)m * J.out_ld + row0 + gg] = sb[gg * SP + m];
    }
  }
}

bool supported_length(int L) {
  switch (L) {
    case 64: case 128: case 256: case 512: case 1024: case 2048: case 4096: case 8192: return true;
    default: return false;
  }
}

int rows_per_tile(int L) {
  switch (L) {
    case 64: return PassShape<64>::G;
    case 128: return PassShape<128>::G;
    case 256: return PassShape<256>::G;
    case 512: return PassShape<512>::G;
    case 1024: return PassShape<1024>::G;
    case 2048: return PassShape<2048>::G;
    case 4096: return PassShape<4096>::G;
    case 8192: return PassShape<8192>::G;
    default: return 0;
  }
}

hipError_t launch_tables(const AxisJob* d_jobs, int njobs, int max_len, const TwiddleJob* d_tw, int ntw,
                         int max_L, hipStream_t s) {
  const int span = max_len > max_L ? max_len : max_L;
  dim3 grid((span + 255) / 256, njobs + ntw);
  hipLaunchKernelGGL(tables_kernel, grid, dim3(256), 0, s, d_jobs, njobs, d_tw, ntw);
  return hipGetLastError();
}

template <int L>
static hipError_t spectra_l(const AxisJob* d_jobs, int first, int count, const float2* tw, hipStream_t s) {
  hipLaunchKernelGGL(spectrum_kernel<L>, dim3(count), dim3(FftPlan<L>::TPR), 0, s, d_jobs, first, tw);
  return hipGetLastError();
}

hipError_t launch_spectra(int L, const AxisJob* d_jobs, int first, int count, const float2* tw, hipStream_t s) {
  switch (L) {
    case 64: return spectra_l<64>(d_jobs, first, count, tw, s);
    case 128: return spectra_l<128>(d_jobs, first, count, tw, s);
    case 256: return spectra_l<256>(d_jobs, first, count, tw, s);
    case 512: return spectra_l<512>(d_jobs, first, count, tw, s);
    case 1024: return spectra_l<1024>(d_jobs, first, count, tw, s);
    case 2048: return spectra_l<2048>(d_jobs, first, count, tw, s);
    case 4096: return spectra_l<4096>(d_jobs, first, count, tw, s);
    case 8192: return spectra_l<8192>(d_jobs, first, count, tw, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L>
static hipError_t pass_l(const PassArgs& a, const float2* tw, hipStream_t s) {
  hipLaunchKernelGGL(pass_kernel<L>, dim3(a.total_tiles), dim3(PassShape<L>::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

hipError_t launch_pass(int L, const PassArgs& a, const float2* tw, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
  switch (L) {
    case 64: return pass_l<64>(a, tw, s);
    case 128: return pass_l<128>(a, tw, s);
    case 256: return pass_l<256>(a, tw, s);
    case 512: return pass_l<512>(a, tw, s);
    case 1024: return pass_l<1024>(a, tw, s);
    case 2048: return pass_l<2048>(a, tw, s);
    case 4096: return pass_l<4096>(a, tw, s);
    case 8192: return pass_l<8192>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sfd

// HIP kernels for batched Shifted-Fresnel reconstruction on gfx950.
//
// A view separates into a y transform of every hologram column followed by
// an x transform of every row of the result (every factor of Eqs. 2-4 is an
// x-only term times a y-only term).  Each transform is one padded 1D chirp
// convolution: multiply by the pre-chirp (step 3 of Section 2.2), zero-pad
// (step 2), FFT (step 4), multiply by the kernel spectrum (step 7), inverse
// FFT (step 8), crop (step 9), then the post-chirp or |.|^2 (step 10, Eq. 5).
//
// This file holds the kernels around the passes; the pass bodies are in
// sfd_device.h, instantiated as col_kernel (sfd_cols.hip), row_kernel
// (sfd_rows.hip) and inside persist_kernel (sfd_persist.hip).
//
//  setup_kernel    everything a batch needs before the passes, by role:
//                  kernel spectra FFT_L(h)/L per view and axis (steps 5-6,
//                  per axis since h of Eq. 4 is separable), the pre/post
//                  chirp tables of Eqs. (2)-(3) (phases reduced in FP64),
//                  the FFT twiddle tables, and the column-major hologram
//                  copies the column pass reads.
//  gradz_kernel    dL/dz of each view from its five FP64 sums.
//  sums_kernel     the first two of those sums from the caller's forward
//                  field and dL/dI.
//  gather_kernel   per-hologram sums of the per-view adjoints.
//  blit_kernel     descriptor images written from kernel arguments (the
//                  no-allocation entry point).
#include "sfd_device.h"

namespace sfd {
template <int L>
static int twiddle_len_l(bool spec) {
  return spec ? twiddle_entries<SpecPlan<L>>() : twiddle_entries<PassPlan<L>>();
}
int twiddle_len(int L, bool spec) {
  switch (L) {
    case 64: return twiddle_len_l<64>(spec);
    case 128: return twiddle_len_l<128>(spec);
    case 256: return twiddle_len_l<256>(spec);
    case 512: return twiddle_len_l<512>(spec);
    case 1024: return twiddle_len_l<1024>(spec);
    case 1280: return twiddle_len_l<1280>(spec);
    case 1536: return twiddle_len_l<1536>(spec);
    case 1792: return twiddle_len_l<1792>(spec);
    case 2048: return twiddle_len_l<2048>(spec);
    case 4096: return twiddle_len_l<4096>(spec);
    case 8192: return twiddle_len_l<8192>(spec);
    default: return -1;
  }
}

// One kernel for all setup roles; MAXL bounds the spectrum lengths of the
// launch so that LDS (and with it occupancy) follows the plan's lengths.
template <int MAXL>
__global__ void __launch_bounds__(kSetupThreads) setup_kernel(const SetupArgs A) {
  __shared__ __align__(16) unsigned char lds[setup_lds_bytes<MAXL>()];
  int r = 0;
  while (r + 1 < A.nroles && (int)blockIdx.x >= A.roles[r + 1].first_block) ++r;
  const SetupRole& Ro = A.roles[r];
  const int rb = blockIdx.x - Ro.first_block;
  switch (Ro.kind) {
    case kRoleSpectrum:
      switch (Ro.a) {
        case 64: setup_spectrum<64>(A, Ro, rb, lds); break;
        case 128: setup_spectrum<128>(A, Ro, rb, lds); break;
        case 256: setup_spectrum<256>(A, Ro, rb, lds); break;
        case 512: setup_spectrum<512>(A, Ro, rb, lds); break;
        case 1024: setup_spectrum<1024>(A, Ro, rb, lds); break;
        case 1280: setup_spectrum<1280>(A, Ro, rb, lds); break;
        case 1536: setup_spectrum<1536>(A, Ro, rb, lds); break;
        case 1792: setup_spectrum<1792>(A, Ro, rb, lds); break;
        case 2048: setup_spectrum<2048>(A, Ro, rb, lds); break;
        case 4096:
          if constexpr (MAXL >= 4096) setup_spectrum<4096>(A, Ro, rb, lds);
          break;
        case 8192:
          if constexpr (MAXL >= 8192) setup_spectrum<8192>(A, Ro, rb, lds);
          break;
        default: break;
      }
      break;
    case kRoleTables: {
      const int job = Ro.b + rb / Ro.a;
      const int i = (rb % Ro.a) * kSetupThreads + threadIdx.x;
      const AxisJob& J = A.axis[job];
      if (i < J.n0) gst(J.pre, (unsigned)i, pre_value(J, i));
      else if (J.post && i < J.n0 + J.n1) gst(J.post, (unsigned)(i - J.n0), post_value(J, i - J.n0));
      break;
    }
    case kRoleTwiddles: {
      const TwiddleJob& T = A.tw[Ro.a];
      const int i = rb * kSetupThreads + threadIdx.x;
      float2 w;
      if (i < T.count && twiddle_any(T.L, T.spec != 0, i, &w)) gst(T.tw, (unsigned)i, w);
      break;
    }
    case kRoleTiles: {
      const TileJob& T = A.tiles[Ro.a];
      const int c0 = (rb % Ro.b) * kTrBlock;
      const int r0 = (rb / Ro.b) * kTrBlock;
      if (T.complex_in) transpose_block<float2>(T, r0, c0, reinterpret_cast<float2*>(lds));
      else transpose_block<float>(T, r0, c0, reinterpret_cast<float*>(lds));
      break;
    }
    default: break;
  }
}

bool supported_length(int L) { return twiddle_len(L, false) >= 0; }

template <int L>
static int fast_input_l() {
  return FastIn<L>::RIN * FastIn<L>::TPR;
}
int fast_input(int L) {
  switch (L) {
    case 64: return fast_input_l<64>();
    case 128: return fast_input_l<128>();
    case 256: return fast_input_l<256>();
    case 512: return fast_input_l<512>();
    case 1024: return fast_input_l<1024>();
    case 1280: return fast_input_l<1280>();
    case 1536: return fast_input_l<1536>();
    case 1792: return fast_input_l<1792>();
    case 2048: return fast_input_l<2048>();
    case 4096: return fast_input_l<4096>();
    case 8192: return fast_input_l<8192>();
    default: return -1;
  }
}

int pass_tile_widths(int L, bool col, int* widths, int cap, int* per_slot) {
  int n = 0;
#define SFD_PUSH(l, g, p)          \
  if (l == L) {                    \
    if (n < cap) {                 \
      widths[n] = g;               \
      if (per_slot) per_slot[n] = p; \
    }                              \
    ++n;                           \
  }
  if (col) {
    SFD_COL_SHAPES(SFD_PUSH)
  } else {
    SFD_ROW_SHAPES(SFD_PUSH)
  }
#undef SFD_PUSH
  return n;
}

int rows_per_tile(int L, bool col) {
  int g = 0;
  return pass_tile_widths(L, col, &g, 1) > 0 ? g : 0;
}

// Sum of a tile-partial array (acc index k) in a fixed order.
__device__ __forceinline__ void sum_partials(const double* p, int n, int k, double* re, double* im, double* sh) {
  double r = 0.0, i = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) {
    r += p[t * 4 + 2 * k];
    i += p[t * 4 + 2 * k + 1];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    r += __shfl_xor(r, off, 64);
    i += __shfl_xor(i, off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[(threadIdx.x >> 6) * 2] = r;
    sh[(threadIdx.x >> 6) * 2 + 1] = i;
  }
  __syncthreads();
  *re = sh[0] + sh[2] + sh[4] + sh[6];
  *im = sh[1] + sh[3] + sh[5] + sh[7];
}

__global__ void __launch_bounds__(256) gradz_kernel(const GradZJob* __restrict__ jobs) {
  __shared__ double sh[8];
  const GradZJob& J = jobs[blockIdx.x];
  double s1r, s1i, s2r, s2i, s3r, s3i, s4r, s4i, s5r, s5i;
  sum_partials(J.p12, J.n12, 0, &s1r, &s1i, sh);
  sum_partials(J.p12, J.n12, 1, &s2r, &s2i, sh);
  sum_partials(J.p3, J.n3, 0, &s3r, &s3i, sh);
  sum_partials(J.p4, J.n4, 0, &s4r, &s4i, sh);
  sum_partials(J.p5, J.n5, 0, &s5r, &s5i, sh);
  if (threadIdx.x == 0) {
    // Re[(i k - 1/z) S1] = -k Im S1 - Re S1 / z;  Re[-i a X] = a Im X.
    const double xi = s2i - 2.0 * s3i - 2.0 * s4i + s5i;
    const double a = M_PI / (J.lam * J.z * J.z);
    *J.out = -J.k * s1i - s1r / J.z + a * xi;
  }
}

// grid: x = block of the job (blocks past its nblocks return), y = jobs.
// FP64 per thread, then across the block in a fixed order.
__global__ void __launch_bounds__(256) sums_kernel(const SumJob* __restrict__ jobs) {
  __shared__ double sh[16];
  const SumJob& J = jobs[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= J.nblocks) return;
  const int r0 = (int)((int64_t)b * J.ny / J.nblocks), r1 = (int)((int64_t)(b + 1) * J.ny / J.nblocks);
  double s1 = 0.0, s2 = 0.0;
  const int n = (r1 - r0) * J.nx;
  for (int e = threadIdx.x; e < n; e += 256) {
    const int row = r0 + e / J.nx, m = e - (row - r0) * J.nx;
    const int64_t at = (int64_t)row * J.ld + m;
    const float2 u = J.u[at];
    const double p = 2.0 * (double)J.gi[at] * ((double)u.x * u.x + (double)u.y * u.y);
    const double X = m * J.xp + J.xa, Y = row * J.yp + J.ya;
    s1 += p;
    s2 += p * (X * X + Y * Y);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[(threadIdx.x >> 6) * 2] = s1;
    sh[(threadIdx.x >> 6) * 2 + 1] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* p = J.partial + (size_t)b * 4;
    p[0] = sh[0] + sh[2] + sh[4] + sh[6];
    p[1] = 0.0;
    p[2] = sh[1] + sh[3] + sh[5] + sh[7];
    p[3] = 0.0;
  }
}

// grid: x covers the largest gradient, y = jobs.
__global__ void __launch_bounds__(256) gather_kernel(const GatherJob* __restrict__ jobs) {
  const GatherJob& J = jobs[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= J.n) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int k = 0; k < J.nsrc; ++k) {
    const float2 x = gld(J.src[k], (unsigned)i);
    acc = cadd(acc, x);
  }
  if (J.real_out) gst(reinterpret_cast<float*>(J.dst), (unsigned)i, acc.x);
  else gst(J.dst, (unsigned)i, acc);
}

hipError_t launch_gradz(const GradZJob* d_jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gradz_kernel, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_sums(const SumJob* d_jobs, int njobs, int max_blocks, hipStream_t s) {
  if (njobs <= 0 || max_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(sums_kernel, dim3(max_blocks, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherJob* d_jobs, int njobs, int max_n, hipStream_t s) {
  if (njobs <= 0 || max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((max_n + 255) / 256, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_setup(const SetupArgs& a, hipStream_t s) {
  if (a.total_blocks <= 0) return hipSuccess;
  if (a.max_l > 8192) return hipErrorInvalidValue;
  if (a.max_l <= 2048)
    hipLaunchKernelGGL(setup_kernel<2048>, dim3(a.total_blocks), dim3(kSetupThreads), 0, s, a);
  else
    hipLaunchKernelGGL(setup_kernel<8192>, dim3(a.total_blocks), dim3(kSetupThreads), 0, s, a);
  return hipGetLastError();
}

int spectra_per_block(int L) {
  switch (L) {
    case 64: return SpecShape<64>::GS;
    case 128: return SpecShape<128>::GS;
    case 256: return SpecShape<256>::GS;
    case 512: return SpecShape<512>::GS;
    case 1024: return SpecShape<1024>::GS;
    case 1280: return SpecShape<1280>::GS;
    case 1536: return SpecShape<1536>::GS;
    case 1792: return SpecShape<1792>::GS;
    case 2048: return SpecShape<2048>::GS;
    case 4096: return SpecShape<4096>::GS;
    case 8192: return SpecShape<8192>::GS;
    default: return 0;
  }
}


// Host-to-device copy through kernel arguments: each launch carries
// kBlitWords words of the image in its argument block and stores them.  No
// host staging buffer and no allocation are involved (the runtime's own
// argument buffers carry the data).
constexpr int kBlitWords = 512;
struct BlitArgs {
  uint32_t w[kBlitWords];
};
__global__ void __launch_bounds__(256) blit_kernel(uint32_t* dst, int n, const BlitArgs a) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = a.w[i];
}

hipError_t launch_blit(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes % 4) return hipErrorInvalidValue;
  const size_t words = bytes / 4;
  const uint32_t* sw = static_cast<const uint32_t*>(src);
  uint32_t* dw = static_cast<uint32_t*>(dst);
  for (size_t off = 0; off < words; off += kBlitWords) {
    const int n = (int)(words - off < (size_t)kBlitWords ? words - off : (size_t)kBlitWords);
    BlitArgs a;
    for (int i = 0; i < n; ++i) a.w[i] = sw[off + i];
    hipLaunchKernelGGL(blit_kernel, dim3(1), dim3(256), 0, s, dw + off, n, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pass(int L, bool col, int G, int var, const PassArgs& a, const float2* tw, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
  return col ? launch_col_pass(L, G, var, a, tw, s) : launch_row_pass(L, G, var, a, tw, s);
}

}  // namespace sfd

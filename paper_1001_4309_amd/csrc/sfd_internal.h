// Internal descriptors shared by the host planner and the HIP kernels.
//
// One view of the Shifted-Fresnel map (Section 2.1, Eqs. 1-4) separates into
// an x transform applied to every hologram row and a y transform applied to
// every column of the result, because every factor of Eqs. (2)-(4) is an
// x-only term times a y-only term.  Each 1D transform is
//
//   out[m1] = post[m1] * sum_{m0} h[m1 - m0] * pre[m0] * in[m0]
//
// evaluated as IFFT_L(H * FFT_L(pad(pre * in))) on a padded length
// L >= N0 + N1 - 1, with H = FFT_L(h) / L.  With x0 = m0 p0 + a0 and
// x1 = m1 p1 + a1 the three factors are (phases in units of pi):
//   pre  (Eq. 3): x0^2/(lambda z) - 2 m0 S a1/p1 - S m0^2
//   h    (Eq. 4): S k^2,  k = m1 - m0 in [-(N0-1), N1-1]
//   post (Eq. 2): x1^2/(lambda z) - 2 a0 x1/(lambda z) - S m1^2
// with S = p0 p1 / (lambda z).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sfd {

// Table-building job for one axis of one view (Eqs. 2-4).
struct AxisJob {
  double a0, a1;   // x0[m] = m p0 + a0, x1[m] = m p1 + a1 (metres)
  double p0, p1;   // pitches (metres)
  double inv_lz;   // 1 / (lambda z)
  double S;        // p0 p1 / (lambda z)
  double c1;       // a1 / p1: output-grid offset in output pixels
  double wscale;   // moment weight scale (pre *= x0 * wscale when kMomentX0)
  float2* pre;     // [n0]
  float2* post;    // [n1] or nullptr
  float2* H;       // [L]: h on input, FFT(h)/L after the spectrum kernel
  int32_t n0, n1, L;
  int32_t flags;   // kPhaseFp32, kMomentX0
};

enum : int32_t { kPhaseFp32 = 1, kMomentX0 = 2 };

// One batched 1D transform over rows (one view, one axis).  Row r of the input
// is in + r * in_ld (n_in elements, float32 or complex64); output element m of
// row r goes to out[m * out_ld + r] (a transposed store, so that the next
// axis again reads contiguous rows).
struct RowJob {
  const void* in;
  void* out;           // complex64, or float32 when only the intensity is written
  float* out2;         // float32 intensity when both outputs are written, else nullptr
  const float2* pre;   // [n_in]
  const float2* H;     // [L]
  const float2* post;  // [n_out] or nullptr
  float2 scale;        // complex factor on the output (field mode)
  float iscale;        // intensity scale
  int32_t n_rows, n_in, n_out;
  int64_t in_ld, out_ld;
  int32_t mode;        // kInReal | kOutIntensity | kOutField | kUsePost | kUseScale
  int32_t pad_;
};

enum : int32_t { kInReal = 1, kOutIntensity = 2, kUsePost = 4, kUseScale = 8, kOutField = 16 };

constexpr int kMaxJobsPerLaunch = 256;

struct PassArgs {
  const RowJob* jobs;
  int32_t njobs;
  int32_t total_tiles;
  int32_t tile_prefix[kMaxJobsPerLaunch + 1];
};

struct TwiddleJob {
  float2* tw;  // [L]: exp(-2 pi i e / L)
  int32_t L;
};

// Host-side launchers (defined in sfd_kernels.hip).
hipError_t launch_tables(const AxisJob* d_jobs, int njobs, int max_len, const TwiddleJob* d_tw,
                         int ntw, int max_L, hipStream_t s);
hipError_t launch_spectra(int L, const AxisJob* d_jobs, int first, int count, const float2* tw,
                          hipStream_t s);
hipError_t launch_pass(int L, const PassArgs& args, const float2* tw, hipStream_t s);

// Rows per workgroup for a transform length (the tile height of a pass).
int rows_per_tile(int L);
bool supported_length(int L);

}  // namespace sfd

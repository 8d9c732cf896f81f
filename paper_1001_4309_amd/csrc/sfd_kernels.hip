// HIP kernels for batched Shifted-Fresnel reconstruction on gfx950.
//
// A view separates into a y transform of every hologram column followed by
// an x transform of every row of the result (every factor of Eqs. 2-4 is an
// x-only term times a y-only term).  Each transform is one padded 1D chirp
// convolution: multiply by the pre-chirp (step 3 of Section 2.2), zero-pad
// (step 2), FFT (step 4), multiply by the kernel spectrum (step 7), inverse
// FFT (step 8), crop (step 9), then the post-chirp or |.|^2 (step 10, Eq. 5).
//
//  setup_kernel    everything a batch needs before the passes, by role:
//                  kernel spectra FFT_L(h)/L per view and axis (steps 5-6,
//                  per axis since h of Eq. 4 is separable), the pre/post
//                  chirp tables of Eqs. (2)-(3) (phases reduced in FP64),
//                  the FFT twiddle tables, and the column-major hologram
//                  copies the column pass reads.
//  col_kernel      the y transforms: G columns per workgroup, stores
//                  leaving through LDS staging so that global accesses are
//                  G elements wide; writes the N1y x N0x intermediate.
//  row_kernel      the x transforms: one row per TPR threads, contiguous
//                  loads and stores straight from registers.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_core.h"
#include "sfd_internal.h"

namespace sfd {

// exp(i pi v) for a large phase v (in half-turns).  The reduction to
// [-1, 1] is done in FP64, exact enough for phases of 10^5 half-turns and
// more.  The reduced argument r is split as r_hi + r_lo with r_hi its FP32
// rounding; FP32 sin/cos of pi r_hi and the first-order correction for
// pi r_lo (|pi r_lo| < 1e-7, so the dropped second-order term is ~1e-14)
// give the FP32 result at FP32 sin/cos accuracy without FP64 trigonometry.
__device__ __forceinline__ float2 cispi_f64(double v) {
  const double r = v - 2.0 * rint(0.5 * v);
  const float rh = static_cast<float>(r);
  const float rl = static_cast<float>((r - static_cast<double>(rh)) * M_PI);
  float s, c;
  sincospif(rh, &s, &c);
  return make_float2(fmaf(-s, rl, c), fmaf(c, rl, s));
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
  float2 v;
  if (J.flags & kPhaseFp32) {
    const float p1 = (float)J.p1, a1 = (float)J.a1, a0 = (float)J.a0, il = (float)J.inv_lz, S = (float)J.S;
    const float fm = (float)m;
    const float x1 = fm * p1 + a1;
    v = cispi_f32(x1 * x1 * il - 2.0f * a0 * x1 * il - S * fm * fm);
  } else {
    const double dm = (double)m;
    const double x1 = dm * J.p1 + J.a1;
    v = cispi_f64(x1 * x1 * J.inv_lz - 2.0 * J.a0 * x1 * J.inv_lz - J.S * (double)((int64_t)m * m));
  }
  return cmul(v, J.post_scale);
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

template <int L>
__device__ __forceinline__ bool twiddle_l(bool spec, int e, float2* out) {
  return spec ? twiddle_entry<SpecPlan<L>>(e, out) : twiddle_entry<PassPlan<L>>(e, out);
}
__device__ __forceinline__ bool twiddle_any(int L, bool spec, int e, float2* out) {
  switch (L) {
    case 64: return twiddle_l<64>(spec, e, out);
    case 128: return twiddle_l<128>(spec, e, out);
    case 256: return twiddle_l<256>(spec, e, out);
    case 512: return twiddle_l<512>(spec, e, out);
    case 1024: return twiddle_l<1024>(spec, e, out);
    case 2048: return twiddle_l<2048>(spec, e, out);
    case 4096: return twiddle_l<4096>(spec, e, out);
    case 8192: return twiddle_l<8192>(spec, e, out);
    default: return false;
  }
}

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
    case 2048: return twiddle_len_l<2048>(spec);
    case 4096: return twiddle_len_l<4096>(spec);
    case 8192: return twiddle_len_l<8192>(spec);
    default: return -1;
  }
}

// Split (real/imaginary in turn) LDS exchanges halve the LDS a row needs.
constexpr bool kSplit = true;

// Setup roles ---------------------------------------------------------------

// Spectrum: H = FFT_L(h) / L for GS axis jobs of length L per workgroup (one,
// or as many as fill the workgroup when a transform needs 128+ threads).  All
// threads first evaluate h of Eq. (4) (FP64 phase) into LDS, then the
// transform threads run the FFT with computed twiddles (a lone transform
// would otherwise wait on table reads at every stage); this role depends on
// no other.
template <int L>
struct SpecShape {
  using P = SpecPlan<L>;
  static constexpr int GS = kSetupThreads / P::TPR;  // spectra per workgroup
  static constexpr int BYTES = GS * row_lds_bytes<L, kSplit>();  // exchange rows
};

template <int L>
__device__ __forceinline__ void setup_spectrum(const SetupArgs& A, const SetupRole& Ro, int rb, void* lds) {
  using P = SpecPlan<L>;
  constexpr int TPR = P::TPR;
  constexpr int R = P::R;
  constexpr int GS = SpecShape<L>::GS;
  // Each thread evaluates h straight into its FFT input slots (element
  // t + TPR i).  The job is the same for every thread of a transform: its
  // fields are read once (scalar loads when a transform spans whole
  // wavefronts), and its output pointer is kept for the end.
  const int g = TPR >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  const int k = rb * GS + g;
  float2* Hg = nullptr;
  float2 v[R];
  if (k < Ro.c) {
    const AxisJob J = A.axis[Ro.b + k];
    Hg = J.H;
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = kernel_value(J, t + TPR * i);
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = make_float2(0.f, 0.f);
  }
  // Twiddles from the spectrum-shape table (built once per workspace),
  // fetched a stage ahead.
  fft_row<P, false, kSplit, kTwGlobal>(v, static_cast<char*>(lds) + g * row_lds_bytes<L, kSplit>(), t, Ro.tw);
  if (!Hg) return;
  const float inv = 1.0f / (float)L;
#pragma unroll
  for (int i = 0; i < R; ++i) gst(Hg, (unsigned)(t + TPR * i), make_float2(v[i].x * inv, v[i].y * inv));
}

// Stores through a buffer resource of a given extent in bytes: the hardware
// drops a store whose offset lies at or past the extent (range checking of
// raw buffer addressing).  A store that only some lanes make is then still
// one unconditional instruction, so the number of memory operations in
// flight does not depend on the predicate, and a later wait for an earlier
// load does not have to wait for the stores too.  kDrop lies past every
// extent used here: an extent covers at most one grid of complex entries
// with sides below 8192 + padding, far below 2^31 bytes.
constexpr uint32_t kDrop = 0x80000000u;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t store_rsrc(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
// AUX: the store's cache-policy bits.  kWriteThrough (sc0 sc1: system
// scope) sends the data on to memory as it is stored, so that it leaves no
// dirty lines behind for the cache write-back at the end of the kernel, which
// the next kernel waits for.
constexpr int kWriteThrough = 1 | 16;
template <int AUX = 0>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)off, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 x) {
  const u32x2_t w = {__builtin_bit_cast(uint32_t, x.x), __builtin_bit_cast(uint32_t, x.y)};
  __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, AUX);
}

// Column-major copy (see TileJob) of one kTrBlock x kTrBlock block: rows of
// the block are read with consecutive threads on consecutive columns, and
// written back as columns with consecutive threads on consecutive rows.
// Camera samples of type S resized along x (see TileJob): for column c of
// the grid, the two neighbours of its source position in rows r0 + hi + STEP k,
// blended.
template <typename S, int K, int STEP>
__device__ __forceinline__ void resample_loads(const TileJob& J, int r0, int hi, int c, float (&v)[K]) {
  const S* in = static_cast<const S*>(J.in);
  const int ns = J.nx_src;
  double sx = ((double)c + 0.5) * (double)ns / (double)J.nx - 0.5;
  sx = fmin(fmax(sx, 0.0), (double)(ns - 1));
  const int i0 = (int)sx;
  const int i1 = i0 + 1 < ns ? i0 + 1 : ns - 1;
  const float wt = (float)(sx - (double)i0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int n = r0 + hi + STEP * k < J.ny ? r0 + hi + STEP * k : J.ny - 1;
    const float a = (float)gld(in, (unsigned)(n * ns + i0)), b = (float)gld(in, (unsigned)(n * ns + i1));
    v[k] = fmaf(wt, b - a, a);
  }
}

template <typename T>
__device__ __forceinline__ void transpose_block(const TileJob& J, int r0, int c0, T* buf) {
  constexpr int B = kTrBlock, SP = B + 1, STEP = kSetupThreads / B, K = B / STEP;
  const T* in = static_cast<const T*>(J.in);
  const int lo = threadIdx.x % B, hi = threadIdx.x / B;
  // All loads first (clamped to the grid, so they are unconditional), then
  // the LDS writes: the loads' latencies overlap.
  T v[K];
  const int c = c0 + lo < J.nx ? c0 + lo : J.nx - 1;
  if constexpr (sizeof(T) == 4) {
    if (J.nx_src > 0) {
      if (J.src_bits == 8) resample_loads<unsigned char, K, STEP>(J, r0, hi, c, v);
      else if (J.src_bits == 16) resample_loads<unsigned short, K, STEP>(J, r0, hi, c, v);
      else resample_loads<float, K, STEP>(J, r0, hi, c, v);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int n = r0 + hi + STEP * k < J.ny ? r0 + hi + STEP * k : J.ny - 1;
        v[k] = gld(in, (unsigned)(n * J.nx + c));
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int n = r0 + hi + STEP * k < J.ny ? r0 + hi + STEP * k : J.ny - 1;
      v[k] = gld(in, (unsigned)(n * J.nx + c));
    }
  }
  if constexpr (sizeof(T) == 8) {
    if (J.in2) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int n = r0 + hi + STEP * k < J.ny ? r0 + hi + STEP * k : J.ny - 1;
        const float a = 2.0f * gld(J.in2, (unsigned)(n * J.nx + c));
        v[k] = make_float2(a * v[k].x, a * v[k].y);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) buf[(hi + STEP * k) * SP + lo] = v[k];
  __syncthreads();
  // Column cc of the block becomes row c0 + cc of the copy; entries outside
  // the grid fall past the store resource's extent (rows) or are sent past
  // it (columns).
  const auto rs = store_rsrc(J.out, (uint32_t)J.nx * (uint32_t)J.ld * (uint32_t)sizeof(T));
  const int n = r0 + lo;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int cc = hi + STEP * k;
    const bool ok = n < J.ny && c0 + cc < J.nx;
    bst(rs, ok ? (uint32_t)((c0 + cc) * J.ld + n) * (uint32_t)sizeof(T) : kDrop, buf[lo * SP + cc]);
  }
}

template <int L>
constexpr int spectrum_lds_bytes() {
  return SpecShape<L>::BYTES;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS of a setup launch whose spectra have lengths <= MAXL.
template <int MAXL>
constexpr int setup_lds_bytes() {
  int b = kTrBlock * (kTrBlock + 1) * 8;
  if (MAXL >= 64) b = cmax(b, spectrum_lds_bytes<64>());
  if (MAXL >= 128) b = cmax(b, spectrum_lds_bytes<128>());
  if (MAXL >= 256) b = cmax(b, spectrum_lds_bytes<256>());
  if (MAXL >= 512) b = cmax(b, spectrum_lds_bytes<512>());
  if (MAXL >= 1024) b = cmax(b, spectrum_lds_bytes<1024>());
  if (MAXL >= 2048) b = cmax(b, spectrum_lds_bytes<2048>());
  if (MAXL >= 4096) b = cmax(b, spectrum_lds_bytes<4096>());
  if (MAXL >= 8192) b = cmax(b, spectrum_lds_bytes<8192>());
  return b;
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

// Occupancy targets (wavefronts per SIMD) handed to the register allocator.
#ifndef SFD_ROW_WPE
#define SFD_ROW_WPE 1
#endif
#ifndef SFD_COL_WPE
#define SFD_COL_WPE 1
#endif

// Workgroup shape of a pass: G transforms (rows or columns) per workgroup,
// held by NS = G / P slots of TPR threads each; a slot runs P transforms in
// turn.
template <int L, int G_, int P_ = 1>
struct PassShape {
  static constexpr int TPR = PassPlan<L>::TPR;
  static constexpr int G = G_;
  static constexpr int P = P_;
  static constexpr int NS = G_ / P_;
  static constexpr int THREADS = NS * TPR;
  static constexpr int NW = THREADS / 64;
  static_assert(G_ % P_ == 0, "a slot runs a whole number of transforms");
  static_assert(THREADS % 64 == 0 && THREADS <= 1024, "a pass workgroup is 1 to 16 whole wavefronts");
};


// Map a workgroup to a tile so that consecutive tiles (which touch adjacent
// pieces of the same cache lines) run on the same XCD: workgroups are
// dispatched round-robin over the 8 XCDs.
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int per = total >> 3;
  if ((total & 7) != 0 || per == 0) return b;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int find_job(const PassArgs& args, int tile) {
  int lo = 0, hi = args.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args.tile_prefix[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Wave-uniform value (the compiler then keeps it, and addresses built from
// it, in scalar registers).
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The same value, opaque to the compiler: addresses derived from it inside
// a loop are then formed in each iteration rather than hoisted out of the
// loop and held in registers across it.
__device__ __forceinline__ int opaque(int x) {
  int y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// The padded, pre-chirped row (n >= 1).  The common case n = L/2 (the
// paper's doubled grid) is straight-line code; otherwise loads go to a
// clamped index (so they still issue back to back) and the padding is
// selected to zero.
template <bool REAL, bool PRE>
__device__ __forceinline__ float2 pre_times_in(const void* in, const float2* pre, unsigned m) {
  float2 x;
  if constexpr (REAL) x = make_float2(gld(static_cast<const float*>(in), m), 0.f);
  else x = gld(static_cast<const float2*>(in), m);
  if constexpr (!PRE) return x;
  const float2 p = gld(pre, m);
  if constexpr (REAL) return make_float2(x.x * p.x, x.x * p.y);
  else return cmul(x, p);
}
template <int TPR, int R, bool REAL, bool PRE>
__device__ __forceinline__ void load_row_t(float2 (&v)[R], const void* in, const float2* pre, int n, int t) {
  if (n == TPR * R / 2) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) v[i] = pre_times_in<REAL, PRE>(in, pre, (unsigned)(t + TPR * i));
#pragma unroll
    for (int i = R / 2; i < R; ++i) v[i] = make_float2(0.f, 0.f);
    return;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int m = t + TPR * i;
    const float2 x = pre_times_in<REAL, PRE>(in, pre, (unsigned)(m < n ? m : n - 1));
    v[i] = m < n ? x : make_float2(0.f, 0.f);
    if ((i & 7) == 7) sched_fence();
  }
}
// The common case only (n = L/2): the first half loaded, the padding zero.
template <int TPR, int R, bool REAL>
__device__ __forceinline__ void load_half(float2 (&v)[R], const void* in, const float2* pre, int t) {
  if (pre) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) v[i] = pre_times_in<REAL, true>(in, pre, (unsigned)(t + TPR * i));
  } else {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) v[i] = pre_times_in<REAL, false>(in, pre, (unsigned)(t + TPR * i));
  }
#pragma unroll
  for (int i = R / 2; i < R; ++i) v[i] = make_float2(0.f, 0.f);
}

// v[i] = in[t + TPR i] (times pre[t + TPR i] unless pre is null) for
// t + TPR i < n, zero beyond.
template <int TPR, int R, bool REAL>
__device__ __forceinline__ void load_row(float2 (&v)[R], const void* in, const float2* pre, int n, int t) {
  if (pre) load_row_t<TPR, R, REAL, true>(v, in, pre, n, t);
  else load_row_t<TPR, R, REAL, false>(v, in, pre, n, t);
}

// Epilogue reduction of the row kernel (see RowJob): FP64 per thread over
// the rows it holds (row_accumulate), then across the wavefront and the
// workgroup in a fixed order, one complex pair per tile into J.partial
// (reduce_tile).
template <int TPR, int R>
__device__ __forceinline__ void row_accumulate(const RowJob& J, const float2 (&v)[R], int row, bool valid, int t,
                                               double (&a)[4]) {
  if (valid) {
    const int n_out = J.n_out;
    const int mode = J.mode;
    const double Y = row * J.yp + J.ya;
    const int64_t base = (int64_t)row * J.red_ld;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int m = t + TPR * i;
      if (m < n_out) {
        float2 G, V;
        if (mode & kRedSwap) {
          G = v[i];
          V = gld(J.uref + base, (unsigned)m);
        } else if (mode & kRedIntensity) {
          const float gi = 2.0f * gld(J.giref + base, (unsigned)m);
          G = make_float2(gi * v[i].x, gi * v[i].y);
          V = v[i];
        } else if (J.giref) {
          const float gi = 2.0f * gld(J.giref + base, (unsigned)m);
          const float2 u = gld(J.uref + base, (unsigned)m);
          G = make_float2(gi * u.x, gi * u.y);
          V = v[i];
        } else {
          G = gld(J.gref + base, (unsigned)m);
          V = v[i];
        }
        double pr, pi;
        if (mode & kRedIntensity) {
          // conj(2 gi V) V = 2 gi |V|^2: real by construction.
          pr = (double)G.x * V.x + (double)G.y * V.y;
          pi = 0.0;
        } else {
          pr = (double)G.x * V.x + (double)G.y * V.y;
          pi = (double)G.x * V.y - (double)G.y * V.x;
        }
        const double X = m * J.xp + J.xa;
        const double r2 = X * X + Y * Y;
        const double w0 = J.wc[0][0] * X + J.wc[0][1] * Y + J.wc[0][2] * r2 + J.wc[0][3];
        const double w1 = J.wc[1][0] * X + J.wc[1][1] * Y + J.wc[1][2] * r2 + J.wc[1][3];
        a[0] += w0 * pr;
        a[1] += w0 * pi;
        a[2] += w1 * pr;
        a[3] += w1 * pi;
      }
    }
  }
}
template <int NW>
__device__ __forceinline__ void reduce_tile(const RowJob& J, double (&a)[4], int tile, double* sbuf) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a[k] += __shfl_xor(a[k], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sbuf[wave * 4 + k] = a[k];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sbuf[w * 4 + threadIdx.x];
    gst(J.partial, (unsigned)(tile * 4 + threadIdx.x), s);
  }
}

// Per-workgroup LDS copies of the transform's twiddle table and of the job's
// kernel spectrum H (for lengths up to 2048, where both fit beside the
// exchange buffers): one cooperative load at the start of the workgroup,
// overlapped with the rows' own loads, replaces the per-stage table reads and
// the H reads of every row.
template <int L>
struct SharedTables {
  static constexpr bool on = L <= 2048;
  static constexpr int tw_n = twiddle_entries<PassPlan<L>>();
  static constexpr int bytes = on ? (tw_n + L) * 8 : 0;
  static constexpr int src = on ? kTwShared : kTwGlobal;
};

// Cooperative copies into LDS at the start of a workgroup: the twiddle
// table, the job's H and, for slots that run several transforms of the job
// (PRE), the first L/2 entries of its pre-chirp when it has one.  Every
// thread issues all of its loads before its first LDS write, so that their
// latencies overlap; a thread past the end of a table reloads its last
// entry instead of skipping the load, which keeps the loads branch-free.
template <int N, int THREADS>
struct CopyShare {
  static constexpr int K = N > 0 ? (N + THREADS - 1) / THREADS : 0;
  static constexpr int KA = K > 0 ? K : 1;  // register array size
};
template <int N, int THREADS, int KA>
__device__ __forceinline__ void copy_load(float4 (&r)[KA], const float2* src) {
  const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int k = 0; k < CopyShare<N, THREADS>::K; ++k) {
    const int e = threadIdx.x + k * THREADS;
    r[k] = gld(s4, (unsigned)(e < N ? e : N - 1));
  }
}
template <int N, int THREADS, int KA>
__device__ __forceinline__ void copy_store(float2* dst, const float4 (&r)[KA]) {
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int k = 0; k < CopyShare<N, THREADS>::K; ++k) {
    const int e = threadIdx.x + k * THREADS;
    if (N % THREADS == 0 || e < N) d4[e] = r[k];
  }
}
template <int L, int THREADS, bool PRE>
__device__ __forceinline__ void stage_tables(float2* tws, float2* hs, float2* ps, const float2* __restrict__ tw,
                                             const float2* __restrict__ H, const float2* __restrict__ pre) {
  static_assert(SharedTables<L>::tw_n % 2 == 0, "tables are copied two entries at a time");
  constexpr int NT = SharedTables<L>::tw_n / 2;
  constexpr int NH = L / 2;
  constexpr int NP = PRE ? L / 4 : 0;
  float4 a[CopyShare<NT, THREADS>::KA];
  float4 b[CopyShare<NH, THREADS>::KA];
  float4 c[CopyShare<NP, THREADS>::KA];
  copy_load<NT, THREADS>(a, tw);
  copy_load<NH, THREADS>(b, H);
  if constexpr (PRE) {
    if (pre) copy_load<NP, THREADS>(c, pre);
  }
  copy_store<NT, THREADS>(tws, a);
  copy_store<NH, THREADS>(hs, b);
  if constexpr (PRE) {
    if (pre) copy_store<NP, THREADS>(ps, c);
  }
}

// The common case (input of L/2 samples) in two steps, so that the loads of
// the next transform can be issued before the current one is computed:
// fetch_half loads the raw first half (a real input only into .x),
// apply_half forms the padded, pre-chirped row from it (pre from LDS, or
// none when ps is null).
template <int TPR, bool REAL, int H>
__device__ __forceinline__ void fetch_half(float2 (&x)[H], const void* in, int64_t off, int t) {
  if constexpr (REAL) {
    const float* p = static_cast<const float*>(in) + off;
#pragma unroll
    for (int i = 0; i < H; ++i) x[i].x = gld(p, (unsigned)(t + TPR * i));
  } else {
    const float2* p = static_cast<const float2*>(in) + off;
#pragma unroll
    for (int i = 0; i < H; ++i) x[i] = gld(p, (unsigned)(t + TPR * i));
  }
}
template <int TPR, int R, bool REAL>
__device__ __forceinline__ void apply_half(float2 (&v)[R], const float2 (&x)[R / 2], const float2* ps, int t) {
  if (!ps) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) v[i] = REAL ? make_float2(x[i].x, 0.f) : x[i];
  } else {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const float2 p = ps[t + TPR * i];
      v[i] = REAL ? make_float2(x[i].x * p.x, x[i].x * p.y) : cmul(x[i], p);
    }
  }
#pragma unroll
  for (int i = R / 2; i < R; ++i) v[i] = make_float2(0.f, 0.f);
}

// x transforms: row r of the job reads in + r * in_ld and writes
// out + r * out_ld (contiguous), both straight from registers.
// VAR selects a specialisation, which keeps the code of the common cases
// small: 0 = any job; 1 = every job of the launch has an input of L/2
// samples, a complex input, an output of at most L/2 and no reduction (half
// loads, pruned transforms, no reduction epilogue); 2 = as 1, and the jobs
// write only intensities.  P > 1: each slot runs several rows in turn.  In
// the specialisations a slot (one wavefront) takes the rows of its tile one
// at a time from a counter in LDS, so that a wavefront that gets more of its
// SIMD takes more rows and the wavefronts of the workgroup finish together;
// the next row's input is fetched while the current row is transformed, and
// the pre-chirp is read from an LDS copy.  The general kernel runs rows
// row0 + p NS, p < P, of its tile.
template <int L, int GR, int VAR, int P>
__global__ void __launch_bounds__((PassShape<L, GR, P>::THREADS)) __attribute__((amdgpu_waves_per_eu(SFD_ROW_WPE))) row_kernel(const PassArgs args, const float2* __restrict__ tw) {
  using S = PassShape<L, GR, P>;
  constexpr int TPR = S::TPR;
  constexpr int R = L / TPR;
  constexpr int NS = S::NS;
  constexpr int RB = row_lds_bytes<L, kSplit>();
  constexpr bool FAST = VAR >= 1;
  constexpr bool INT_ONLY = VAR == 2;
  constexpr bool PF = FAST && P > 1;
  using T = SharedTables<L>;
  static_assert(P == 1 || (T::on && TPR <= 64), "slots of several transforms are single wavefronts with LDS tables");
  static_assert(!PF || TPR == 64, "a queue slot is one whole wavefront");
  constexpr int PRE_BYTES = PF ? (L / 2) * 8 : 0;
  // Shared tables, the pre-chirp copy, exchange buffers, then room for the
  // epilogue reduction (4 doubles per wavefront).
  __shared__ __align__(16) unsigned char lds[T::bytes + PRE_BYTES + NS * RB + S::NW * 32 + (PF ? 16 : 0)];
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  float2* ps = reinterpret_cast<float2*>(lds + T::bytes);
  unsigned char* xbuf = lds + T::bytes + PRE_BYTES;

  const int tile = xcd_tile(blockIdx.x, args.total_tiles);
  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  // With TPR >= 64 a row is a whole number of wavefronts: g is wave-uniform.
  const int g = TPR >= 64 ? uniform(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  // Slot g runs rows row0 + p NS, p < P.  A row past the end of the job
  // computes on row 0 and stores nothing.
  const int row0 = (tile - args.tile_prefix[jid]) * GR + g;
  // The job's fields, read once here (before any store, so that they can be
  // scalar loads) rather than at their uses inside the row loop.
  const int n_rows = J.n_rows;
  const int n_in = J.n_in;
  const int n_out = J.n_out;
  const int mode = J.mode;
  // Row jobs of the specialisations read complex inputs (the launcher
  // checks); the general kernel takes either.
  const bool real_in = !FAST && (mode & kInReal) != 0;
  const void* in = J.in;
  const int64_t in_ld = J.in_ld;
  const int64_t out_ld = J.out_ld;
  const float2* __restrict__ pre = J.pre;
  const float2* __restrict__ H = J.H;
  const float2* __restrict__ post = J.post;
  void* const out1 = J.out;
  float* const out2 = J.out2;
  const float sc = J.iscale;

  // Row counter of the tile (PF), after the reduction scratch.  A wavefront
  // takes one row per LDS atomic, made by its first lane; the row is valid in
  // that lane only until passed through uniform().
  int* const counter = reinterpret_cast<int*>(xbuf + NS * RB + S::NW * 32);
  const int tile_row0 = (tile - args.tile_prefix[jid]) * GR;
  const int tile_rows = n_rows - tile_row0 < GR ? n_rows - tile_row0 : GR;
  if constexpr (PF) {
    if (threadIdx.x == 0) *counter = 0;
    __syncthreads();
  }
  const bool lane0 = (threadIdx.x & 63) == 0;
  auto grab = [&]() -> int {
    int r = 0;
    if (lane0) r = atomicAdd(counter, 1);
    return r;
  };
  float2 v[R];
  float2 x[PF ? R / 2 : 1];
  auto load = [&](int row, int t) {
    const int64_t off = (int64_t)(row < n_rows ? row : 0) * in_ld;
    if constexpr (PF) {
      fetch_half<TPR, false>(x, in, off, t);
    } else if constexpr (FAST) {
      load_half<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, t);
    } else {
      if (real_in) load_row<TPR, R, true>(v, static_cast<const float*>(in) + off, pre, n_in, t);
      else load_row<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, n_in, t);
    }
  };
  // PF: rows of the tile by their index in it (valid below tile_rows).
  int r_cur = row0, r_next = 0;
  if constexpr (PF) {
    r_cur = uniform(grab());
    if (r_cur < tile_rows) load(tile_row0 + r_cur, t);
    r_next = r_cur < tile_rows ? uniform(grab()) : tile_rows;
  } else {
    load(row0, t);
  }

  if constexpr (T::on) {
    stage_tables<L, S::THREADS, PF>(tws, hs, ps, tw, H, pre);
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // HALF: the common case (input of L/2 samples, output of at most L/2),
  // where the first forward and the last inverse stage skip the padded and
  // the cropped half.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? R / 2 : R;
    // HALF with a row per wavefront: a row's outputs (field of, intensity
    // oi) leave through one store resource per row, of n_out entries (none
    // for a row past the job's end).  With several rows per slot, a row's
    // outputs are stored only once the next row's input has arrived (the
    // wait for that input then finds no store of this row in flight), and
    // written through (measured: the next kernel starts sooner, as with the
    // column kernel's intermediate).
    constexpr bool BUF = HALF && TPR >= 64;
    float2 of[BUF && !INT_ONLY ? RL : 1];
    float oi[BUF ? RL : 1];
    auto flush = [&](int r, int lane) {
      if constexpr (BUF) {
        const uint32_t lim = r < n_rows ? (uint32_t)n_out : 0u;
        if (!INT_ONLY && (mode & kOutField)) {
          const auto rs = store_rsrc(static_cast<float2*>(out1) + (int64_t)r * out_ld, lim * 8u);
#pragma unroll
          for (int i = 0; i < RL; ++i) bst<PF ? kWriteThrough : 0>(rs, (uint32_t)(lane + TPR * i) * 8u, of[i]);
        }
        if (mode & kOutIntensity) {
          float* o = ((!INT_ONLY && (mode & kOutField)) ? out2 : static_cast<float*>(out1)) + (int64_t)r * out_ld;
          const auto rs = store_rsrc(o, lim * 4u);
#pragma unroll
          for (int i = 0; i < RL; ++i) bst<PF ? kWriteThrough : 0>(rs, (uint32_t)(lane + TPR * i) * 4u, oi[i]);
        }
      }
    };
    int prev = -1;  // PF: the row whose outputs wait in of / oi
    int pend = 0;   // PF: the row after next (index in the tile), in the first lane
#pragma unroll 1
    for (int p = 0; PF ? r_cur < tile_rows : p < P; ++p) {
      const int tl = P > 1 ? opaque(t) : t;
      const int row = PF ? tile_row0 + r_cur : row0 + p * NS;
      const bool valid = row < n_rows;
      if constexpr (PF) {
        apply_half<TPR, R, false>(v, x, pre ? ps : nullptr, tl);
        sched_fence();
        if (prev >= 0) flush(prev, tl);
        sched_fence();
        if (r_next < tile_rows) load(tile_row0 + r_next, tl);
        // The row after next: taken now, read after this row's transforms.
        pend = r_next < tile_rows ? grab() : tile_rows;
      } else if (p > 0) {
        load(row, tl);
      }
      fft_row<PassPlan<L>, false, kSplit, T::src, HALF>(v, buf, tl, twx);
      sched_fence();
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[tl + TPR * i] : gld(H, (unsigned)(tl + TPR * i)));
      sched_fence();
      fft_row<PassPlan<L>, true, kSplit, T::src, HALF>(v, buf, tl, twx);

      if (!INT_ONLY && (mode & kUsePost)) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          const int m = tl + TPR * i;
          // HALF: a clamped (branch-free) load; entries past n_out are never stored.
          if (HALF) v[i] = cmul(v[i], gld(post, (unsigned)(m < n_out ? m : n_out - 1)));
          else if (TPR * (i + 1) <= n_out || m < n_out) v[i] = cmul(v[i], gld(post, (unsigned)m));
        }
      }
      if constexpr (BUF) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          if constexpr (!INT_ONLY) of[i] = v[i];
          oi[i] = fmaf(v[i].x, v[i].x, v[i].y * v[i].y) * sc;
        }
        if constexpr (!PF) flush(row, tl);
      } else {
        if (!INT_ONLY && valid && (mode & kOutField)) {
          float2* out = static_cast<float2*>(out1) + (int64_t)row * out_ld;
#pragma unroll
          for (int i = 0; i < RL; ++i) {
            const int m = tl + TPR * i;
            if (TPR * (i + 1) <= n_out || m < n_out) gst(out, (unsigned)m, v[i]);
          }
        }
        if (valid && (mode & kOutIntensity)) {
          float* out = ((!INT_ONLY && (mode & kOutField)) ? out2 : static_cast<float*>(out1)) + (int64_t)row * out_ld;
#pragma unroll
          for (int i = 0; i < RL; ++i) {
            const int m = tl + TPR * i;
            if (TPR * (i + 1) <= n_out || m < n_out) gst(out, (unsigned)m, fmaf(v[i].x, v[i].x, v[i].y * v[i].y) * sc);
          }
        }
      }
      if constexpr (!HALF) {
        if (mode & kReduce) row_accumulate<TPR, R>(J, v, row, valid, tl, acc);
      }
      if constexpr (PF) {
        prev = row;
        r_cur = r_next;
        r_next = uniform(pend);
      }
    }
    if constexpr (PF) {
      if (prev >= 0) flush(prev, t);
    }
    if constexpr (!HALF) {
      if (mode & kReduce)
        reduce_tile<S::NW>(J, acc, tile - args.tile_prefix[jid], reinterpret_cast<double*>(xbuf + NS * RB));
    }
  };
  if constexpr (FAST) body(std::true_type{});
  else body(std::false_type{});
}

// y transforms: column c of the job reads in[c * in_ld + n] for n < n_in
// (the column-major copy of its grid, see TileJob) and writes
// out[m * out_ld + c] for m < n_out (complex).  The NS columns that the
// slots of a workgroup hold at once leave through LDS staging in chunks of
// L/2 rows, so that each global store covers NS consecutive columns.  P > 1
// as in the row kernel.
template <int L, int GC, int VAR, int P>
__global__ void __launch_bounds__((PassShape<L, GC, P>::THREADS)) __attribute__((amdgpu_waves_per_eu(SFD_COL_WPE))) col_kernel(const PassArgs args, const float2* __restrict__ tw) {
  using S = PassShape<L, GC, P>;
  constexpr int TPR = S::TPR;
  constexpr int R = L / TPR;
  constexpr int NS = S::NS;
  constexpr int THREADS = S::THREADS;
  // VAR: 0 = any job; 1 = the jobs' inputs are L/2 samples, complex, their
  // outputs at most L/2; 2 = as 1 with real inputs and no post-chirp (the
  // hologram of an intensity-only plan); 3 = as 1 with real inputs.
  constexpr bool FAST = VAR >= 1;
  constexpr bool REAL = VAR >= 2;
  constexpr bool NO_POST = VAR == 2;
  constexpr bool PF = FAST && P > 1;
  constexpr int RB = row_lds_bytes<L, kSplit>();
  constexpr int C = L / 2;    // staging chunk along the transform
  constexpr int SST = C + 9;  // staging stride per column (elements)
  constexpr int STAGE_BYTES = NS * SST * 8;
  constexpr int XCH_BYTES = NS * RB > STAGE_BYTES ? NS * RB : STAGE_BYTES;
  using T = SharedTables<L>;
  static_assert((NS & (NS - 1)) == 0, "slots per workgroup must be a power of two");
  static_assert(P == 1 || (T::on && TPR <= 64), "slots of several transforms are single wavefronts with LDS tables");
  constexpr int PRE_BYTES = PF ? (L / 2) * 8 : 0;
  // Shared tables, the pre-chirp copy, then the exchange buffers (reused as
  // the store staging).
  __shared__ __align__(16) unsigned char lds[T::bytes + PRE_BYTES + XCH_BYTES];
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  float2* ps = reinterpret_cast<float2*>(lds + T::bytes);
  unsigned char* xbuf = lds + T::bytes + PRE_BYTES;
  float2* st = reinterpret_cast<float2*>(xbuf);

  const int tile = xcd_tile(blockIdx.x, args.total_tiles);
  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  const int c0 = (tile - args.tile_prefix[jid]) * GC;
  const int g = TPR >= 64 ? uniform(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  // The job's fields, read once here (before any store, so that they can be
  // scalar loads) rather than at their uses inside the column loop.
  const int ncols = J.n_rows;
  const int n_in = J.n_in;
  const int n_out = J.n_out;
  const int mode = J.mode;
  const int in_ld = (int)J.in_ld;
  const int out_ld = (int)J.out_ld;
  const void* in = J.in;
  float2* const out0 = static_cast<float2*>(J.out);
  const float2* __restrict__ pre = J.pre;
  const float2* __restrict__ H = J.H;
  const float2* __restrict__ post = J.post;
  const float2* __restrict__ colscale = J.colscale;
  const bool real_in = FAST ? REAL : (mode & kInReal) != 0;

  // Slot g runs columns c0 + p NS + g, p < P, each loaded like a row from the
  // column-major input copy (a column past the grid's edge computes on the
  // last one and stores nothing), with its colscale factor.
  float2 v[R];
  float2 x[PF ? R / 2 : 1];
  float2 csn = make_float2(1.f, 0.f);
  auto load = [&](int p, int t) {
    const int c = c0 + p * NS + g;
    const int cl = c < ncols ? c : ncols - 1;
    const int64_t off = (int64_t)cl * in_ld;
    if constexpr (PF) {
      fetch_half<TPR, REAL>(x, in, off, t);
    } else if constexpr (FAST) {
      if constexpr (REAL) load_half<TPR, R, true>(v, static_cast<const float*>(in) + off, pre, t);
      else load_half<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, t);
    } else {
      if (real_in) load_row<TPR, R, true>(v, static_cast<const float*>(in) + off, pre, n_in, t);
      else load_row<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, n_in, t);
    }
    if (colscale) csn = gld(colscale, (unsigned)cl);
  };
  load(0, t);

  if constexpr (T::on) {
    stage_tables<L, THREADS, PF>(tws, hs, ps, tw, H, pre);
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  // HALF as in the row kernel; then only the first staging chunk exists.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? R / 2 : R;
    constexpr int NC = HALF ? 1 : 2;
    // HALF: a round's staged values (R / 2 per thread) leave through a
    // store resource of n_out rows from the round's first column cb: rows
    // m >= n_out fall past its extent, columns past the grid's edge are sent
    // past it.  With several rounds, a round's values stay staged until the
    // next round's input has arrived, and are stored then (as in the row
    // kernel).
    auto flush = [&](int cb, int tid) {
      if constexpr (HALF) {
        const int gs = tid & (NS - 1);
        const bool col_ok = cb + gs < ncols;
        const auto rs = store_rsrc(out0 + cb, (uint32_t)(n_out * out_ld) * 8u);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
          const int m = (tid + k * THREADS) / NS;
          // Write-through in the kernels whose slots run several transforms
          // (measured: the row pass then starts sooner); the single-transform
          // kernels measured faster with the default policy.
          bst<PF ? kWriteThrough : 0>(rs, col_ok ? (uint32_t)(m * out_ld + gs) * 8u : kDrop, st[gs * SST + m]);
        }
      }
    };
#pragma unroll 1
    for (int p = 0; p < P; ++p) {
      const int tl = P > 1 ? opaque(t) : t;
      const int tid = P > 1 ? opaque((int)threadIdx.x) : (int)threadIdx.x;
      // Column of the store staging loop for this thread (fixed: THREADS is a multiple of NS).
      const int gs = tid & (NS - 1);
      const int cb = c0 + p * NS;  // first column of this round
      const bool col_ok = cb + gs < ncols;
      float2* out = out0 + cb + gs;
      float2 cs;
      if constexpr (PF) {
        cs = csn;
        apply_half<TPR, R, REAL>(v, x, pre ? ps : nullptr, tl);
        sched_fence();
        if (p > 0) {
          flush(cb - NS, tid);
          // The exchanges below reuse the staging memory.
          __syncthreads();
        }
        if (p + 1 < P) load(p + 1, tl);
      } else {
        if (p > 0) load(p, tl);
        cs = csn;
      }
      fft_row<PassPlan<L>, false, kSplit, T::src, HALF>(v, buf, tl, twx);
      sched_fence();
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[tl + TPR * i] : gld(H, (unsigned)(tl + TPR * i)));
      sched_fence();
      fft_row<PassPlan<L>, true, kSplit, T::src, HALF>(v, buf, tl, twx);

      if (!NO_POST && (mode & kUsePost)) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          const int m = tl + TPR * i;
          // HALF: a clamped (branch-free) load; entries past n_out are never stored.
          if (HALF) v[i] = cmul(v[i], gld(post, (unsigned)(m < n_out ? m : n_out - 1)));
          else if (TPR * (i + 1) <= n_out || m < n_out) v[i] = cmul(v[i], gld(post, (unsigned)m));
        }
      }
      if (colscale) {
#pragma unroll
        for (int i = 0; i < RL; ++i) v[i] = cmul(v[i], cs);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int m_lo = c * C;
        if (m_lo >= n_out) break;
        __syncthreads();
#pragma unroll
        for (int i = c * (R / 2); i < (c + 1) * (R / 2); ++i) {
          const int m = tl + TPR * i;
          if (TPR * (i + 1) <= n_out || m < n_out) st[g * SST + (m - m_lo)] = v[i];
        }
        __syncthreads();
        if constexpr (HALF) {
          if constexpr (!PF) flush(cb, tid);
        } else {
          const int cnt = (n_out - m_lo < C ? n_out - m_lo : C) * NS;
          for (int e = tid; e < cnt; e += THREADS) {
            const int m = m_lo + e / NS;
            if (col_ok) gst(out, (unsigned)(m * out_ld), st[gs * SST + (m - m_lo)]);
          }
        }
      }
      // The next round's exchanges reuse the staging memory (PF: after its flush).
      if (!PF && p + 1 < P) __syncthreads();
    }
    if constexpr (PF) flush(c0 + (P - 1) * NS, threadIdx.x);
  };
  if constexpr (FAST) body(std::true_type{});
  else body(std::false_type{});
}

bool supported_length(int L) { return twiddle_len(L, false) >= 0; }

// Shapes a pass can be launched with at each length: X(L, G, P), G the tile
// width (transforms per workgroup), P the transforms each slot runs in turn.
// The workgroup is G / P slots of TPR threads, and their exchange rows must
// fit in LDS; the first entry per length is the default.
#define SFD_ROW_SHAPES(X) \
  X(64, 32, 1) X(64, 16, 1) X(64, 64, 1) X(128, 16, 1) X(128, 8, 1) X(128, 32, 1) X(256, 8, 1) X(256, 4, 1) \
  X(256, 16, 1) X(512, 4, 1) X(512, 2, 1) X(512, 8, 1) X(1024, 2, 1) X(1024, 1, 1) X(1024, 4, 1) X(1024, 8, 2) \
  X(1024, 16, 2) X(2048, 2, 1) X(2048, 1, 1) X(2048, 4, 1) X(2048, 8, 2) X(2048, 16, 2) X(4096, 1, 1) X(8192, 1, 1)
#define SFD_COL_SHAPES(X) \
  X(64, 32, 1) X(64, 16, 1) X(128, 16, 1) X(128, 8, 1) X(256, 8, 1) X(256, 4, 1) X(512, 8, 1) X(512, 4, 1) \
  X(1024, 8, 1) X(1024, 4, 1) X(1024, 16, 1) X(1024, 32, 2) X(2048, 8, 1) X(2048, 4, 1) X(2048, 2, 1) \
  X(2048, 16, 2) X(4096, 2, 1) X(4096, 4, 1) X(8192, 1, 1) X(8192, 2, 1)

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
  gst(J.dst, (unsigned)i, acc);
}

hipError_t launch_gradz(const GradZJob* d_jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gradz_kernel, dim3(njobs), dim3(256), 0, s, d_jobs);
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
    case 2048: return SpecShape<2048>::GS;
    case 4096: return SpecShape<4096>::GS;
    case 8192: return SpecShape<8192>::GS;
    default: return 0;
  }
}

hipError_t launch_pass(int L, bool col, int G, int var, const PassArgs& a, const float2* tw, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
#define SFD_LAUNCH_V(kern, l, g, p, v) \
  hipLaunchKernelGGL((kern<l, g, v, p>), dim3(a.total_tiles), dim3(PassShape<l, g, p>::THREADS), 0, s, a, tw)
#define SFD_LAUNCH_ROW(l, g, p)                             \
  if (!col && L == l && G == g) {                           \
    if (var == 2) SFD_LAUNCH_V(row_kernel, l, g, p, 2);     \
    else if (var == 1) SFD_LAUNCH_V(row_kernel, l, g, p, 1); \
    else SFD_LAUNCH_V(row_kernel, l, g, p, 0);              \
    return hipGetLastError();                               \
  }
#define SFD_LAUNCH_COL(l, g, p)                             \
  if (col && L == l && G == g) {                            \
    if (var == 3) SFD_LAUNCH_V(col_kernel, l, g, p, 3);     \
    else if (var == 2) SFD_LAUNCH_V(col_kernel, l, g, p, 2); \
    else if (var == 1) SFD_LAUNCH_V(col_kernel, l, g, p, 1); \
    else SFD_LAUNCH_V(col_kernel, l, g, p, 0);              \
    return hipGetLastError();                               \
  }
  SFD_ROW_SHAPES(SFD_LAUNCH_ROW)
  SFD_COL_SHAPES(SFD_LAUNCH_COL)
#undef SFD_LAUNCH_ROW
#undef SFD_LAUNCH_COL
#undef SFD_LAUNCH_V
  return hipErrorInvalidValue;
}

}  // namespace sfd

// HIP kernels for batched Shifted-Fresnel reconstruction on gfx950.
//
// A view separates into a y transform of every hologram column followed by
// an x transform of every row of the result (every factor of Eqs. 2-4 is an
// x-only term times a y-only term).  Each transform is one padded 1D chirp
// convolution: multiply by the pre-chirp (step 3 of Section 2.2), zero-pad
// (step 2), FFT (step 4), multiply by the kernel spectrum (step 7), inverse
// FFT (step 8), crop (step 9), then the post-chirp or |.|^2 (step 10, Eq. 5).
//
//  tables_kernel   chirp tables of Eqs. (2)-(4) per view and axis, phases in
//                  FP64 reduced to [-1, 1] half-turns before sin/cos, plus the
//                  FFT twiddle tables.
//  spectrum_kernel FFT_L(h) / L per view and axis (steps 5-6, per axis since
//                  h of Eq. 4 is separable).
//  col_kernel      the y transforms: G columns per workgroup, loaded and
//                  stored through LDS staging so that global accesses are
//                  G elements wide; writes the N1y x N0x intermediate.
//  row_kernel      the x transforms: one row per TPR threads, contiguous
//                  loads and stores straight from registers.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_core.h"
#include "sfd_internal.h"

namespace sfd {

// exp(i pi v) with v reduced to [-1, 1] in FP64 first, then evaluated in FP64
// and rounded once to complex64.
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
  static constexpr int STAGE = GS * L * 8;
  static constexpr int EXCH = GS * row_lds_bytes<L, kSplit>();
  static constexpr int BYTES = STAGE > EXCH ? STAGE : EXCH;
};

template <int L>
__device__ __forceinline__ void setup_spectrum(const SetupArgs& A, const SetupRole& Ro, int rb, void* lds) {
  using P = SpecPlan<L>;
  constexpr int TPR = P::TPR;
  constexpr int R = P::R;
  constexpr int GS = SpecShape<L>::GS;
  float2* hs = static_cast<float2*>(lds);
  // The job is the same for every thread of a transform: its fields are read
  // once (scalar loads) before the loop rather than per element, and its
  // output pointer is kept for the end.
  float2* Hout[GS];
#pragma unroll
  for (int gj = 0; gj < GS; ++gj) {
    const int k = rb * GS + gj;
    Hout[gj] = nullptr;
    if (k < Ro.c) {
      const AxisJob J = A.axis[Ro.b + k];
      Hout[gj] = J.H;
      for (int i = threadIdx.x; i < L; i += kSetupThreads) hs[gj * L + i] = kernel_value(J, i);
    } else {
      for (int i = threadIdx.x; i < L; i += kSetupThreads) hs[gj * L + i] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  const int g = threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  float2 v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = hs[g * L + t + TPR * i];
  __syncthreads();
  fft_row<P, false, kSplit, kTwCompute>(v, static_cast<char*>(lds) + g * row_lds_bytes<L, kSplit>(), t, nullptr);
  float2* Hg = Hout[0];
#pragma unroll
  for (int gj = 1; gj < GS; ++gj)
    if (g == gj) Hg = Hout[gj];
  if (!Hg) return;
  const float inv = 1.0f / (float)L;
#pragma unroll
  for (int i = 0; i < R; ++i) gst(Hg, (unsigned)(t + TPR * i), make_float2(v[i].x * inv, v[i].y * inv));
}

// Column-major copy (see TileJob) of one kTrBlock x kTrBlock block: rows of
// the block are read with consecutive threads on consecutive columns, and
// written back as columns with consecutive threads on consecutive rows.
template <typename T>
__device__ __forceinline__ void transpose_block(const TileJob& J, int r0, int c0, T* buf) {
  constexpr int B = kTrBlock, SP = B + 1, STEP = kSetupThreads / B;
  const T* in = static_cast<const T*>(J.in);
  T* out = static_cast<T*>(J.out);
  const int lo = threadIdx.x % B, hi = threadIdx.x / B;
#pragma unroll
  for (int k = 0; k < B / STEP; ++k) {
    const int rr = hi + STEP * k;
    const int n = r0 + rr, c = c0 + lo;
    T v{};
    if (n < J.ny && c < J.nx) {
      v = gld(in, (unsigned)(n * J.nx + c));
      if constexpr (sizeof(T) == 8) {
        if (J.in2) {
          const float a = 2.0f * gld(J.in2, (unsigned)(n * J.nx + c));
          v = make_float2(a * v.x, a * v.y);
        }
      }
    }
    buf[rr * SP + lo] = v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < B / STEP; ++k) {
    const int cc = hi + STEP * k;
    const int n = r0 + lo, c = c0 + cc;
    if (n < J.ny && c < J.nx) gst(out, (unsigned)(c * J.ld + n), buf[lo * SP + cc]);
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

// Workgroup shape of a pass: G rows (or columns) of TPR threads each.
template <int L, int G_>
struct PassShape {
  static constexpr int TPR = PassPlan<L>::TPR;
  static constexpr int G = G_;
  static constexpr int THREADS = G * TPR;
  static constexpr int NW = THREADS / 64;
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

// Epilogue reduction of the row kernel (see RowJob): FP64 per thread, then
// across the wavefront and the workgroup in a fixed order, one complex pair
// per tile into J.partial.
template <int TPR, int R, int NW>
__device__ __forceinline__ void row_reduce(const RowJob& J, const float2 (&v)[R], int row, bool valid, int t, int tile,
                                           double* sbuf) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
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

template <int L, int THREADS>
__device__ __forceinline__ void stage_tables(float2* tws, float2* hs, const float2* __restrict__ tw,
                                             const float2* __restrict__ H) {
  static_assert(SharedTables<L>::tw_n % 2 == 0, "tables are copied two entries at a time");
  float4* t4 = reinterpret_cast<float4*>(tws);
  float4* h4 = reinterpret_cast<float4*>(hs);
  const float4* tg = reinterpret_cast<const float4*>(tw);
  const float4* hg = reinterpret_cast<const float4*>(H);
#pragma unroll 4
  for (int e = threadIdx.x; e < SharedTables<L>::tw_n / 2; e += THREADS) t4[e] = gld(tg, (unsigned)e);
#pragma unroll 4
  for (int e = threadIdx.x; e < L / 2; e += THREADS) h4[e] = gld(hg, (unsigned)e);
}

// x transforms: row r of the job reads in + r * in_ld and writes
// out + r * out_ld (contiguous), both straight from registers.
// VAR selects a specialisation, which keeps the code of the common cases
// small: 0 = any job; 1 = every job of the launch has an input of L/2
// samples, an output of at most L/2 and no reduction (half loads, pruned
// transforms, no reduction epilogue); 2 = as 1, and the jobs write only
// intensities.
template <int L, int GR, int VAR>
__global__ void __launch_bounds__((PassShape<L, GR>::THREADS)) __attribute__((amdgpu_waves_per_eu(SFD_ROW_WPE))) row_kernel(const PassArgs args, const float2* __restrict__ tw) {
  using S = PassShape<L, GR>;
  constexpr int TPR = S::TPR;
  constexpr int R = L / TPR;
  constexpr int G = S::G;
  constexpr int RB = row_lds_bytes<L, kSplit>();
  constexpr bool FAST = VAR >= 1;
  constexpr bool INT_ONLY = VAR == 2;
  using T = SharedTables<L>;
  // Shared tables, exchange buffers, then room for the epilogue reduction (4
  // doubles per wavefront).
  __shared__ __align__(16) unsigned char lds[T::bytes + G * RB + S::NW * 32];
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  unsigned char* xbuf = lds + T::bytes;

  const int tile = xcd_tile(blockIdx.x, args.total_tiles);
  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  // With TPR >= 64 a row is a whole number of wavefronts: g is wave-uniform.
  const int g = TPR >= 64 ? uniform(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  const int row = (tile - args.tile_prefix[jid]) * G + g;
  const bool valid = row < J.n_rows;
  const int vrow = valid ? row : 0;
  const int n_in = J.n_in;

  // A row past the end of the job computes on row 0 and stores nothing.
  float2 v[R];
  if constexpr (FAST) {
    if (J.mode & kInReal)
      load_half<TPR, R, true>(v, static_cast<const float*>(J.in) + (int64_t)vrow * J.in_ld, J.pre, t);
    else
      load_half<TPR, R, false>(v, static_cast<const float2*>(J.in) + (int64_t)vrow * J.in_ld, J.pre, t);
  } else {
    if (J.mode & kInReal)
      load_row<TPR, R, true>(v, static_cast<const float*>(J.in) + (int64_t)vrow * J.in_ld, J.pre, n_in, t);
    else
      load_row<TPR, R, false>(v, static_cast<const float2*>(J.in) + (int64_t)vrow * J.in_ld, J.pre, n_in, t);
  }

  const float2* __restrict__ H = J.H;
  if constexpr (T::on) {
    stage_tables<L, S::THREADS>(tws, hs, tw, H);
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  const int n_out = J.n_out;
  const int mode = J.mode;
  // HALF: the common case (input of L/2 samples, output of at most L/2),
  // where the first forward and the last inverse stage skip the padded and
  // the cropped half.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? R / 2 : R;
    fft_row<PassPlan<L>, false, kSplit, T::src, HALF>(v, buf, t, twx);
    sched_fence();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[t + TPR * i] : gld(H, (unsigned)(t + TPR * i)));
    sched_fence();
    fft_row<PassPlan<L>, true, kSplit, T::src, HALF>(v, buf, t, twx);

    if (!INT_ONLY && (mode & kUsePost)) {
      const float2* post = J.post;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const int m = t + TPR * i;
        if (TPR * (i + 1) <= n_out || m < n_out) v[i] = cmul(v[i], gld(post, (unsigned)m));
      }
    }
    if (!INT_ONLY && valid && (mode & kOutField)) {
      float2* out = static_cast<float2*>(J.out) + (int64_t)row * J.out_ld;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const int m = t + TPR * i;
        if (TPR * (i + 1) <= n_out || m < n_out) gst(out, (unsigned)m, v[i]);
      }
    }
    if (valid && (mode & kOutIntensity)) {
      float* out = ((!INT_ONLY && (mode & kOutField)) ? J.out2 : static_cast<float*>(J.out)) + (int64_t)row * J.out_ld;
      const float sc = J.iscale;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const int m = t + TPR * i;
        if (TPR * (i + 1) <= n_out || m < n_out) gst(out, (unsigned)m, (v[i].x * v[i].x + v[i].y * v[i].y) * sc);
      }
    }
    if constexpr (!HALF) {
      if (mode & kReduce) row_reduce<TPR, R, S::NW>(J, v, row, valid, t, tile - args.tile_prefix[jid],
                                                             reinterpret_cast<double*>(xbuf + G * RB));
    }
  };
  if constexpr (FAST) body(std::true_type{});
  else body(std::false_type{});
}

// y transforms: column c of the job reads in[c * in_ld + n] for n < n_in
// (the column-major copy of its grid, see TileJob) and writes
// out[m * out_ld + c] for m < n_out (complex).  The G columns of a workgroup
// leave through LDS staging in chunks of L/2 rows, so that each global store
// covers G consecutive columns.
template <int L, int GC, int VAR>
__global__ void __launch_bounds__((PassShape<L, GC>::THREADS)) __attribute__((amdgpu_waves_per_eu(SFD_COL_WPE))) col_kernel(const PassArgs args, const float2* __restrict__ tw) {
  using S = PassShape<L, GC>;
  constexpr int TPR = S::TPR;
  constexpr int R = L / TPR;
  constexpr int G = S::G;
  constexpr int THREADS = S::THREADS;
  // As in row_kernel; column passes write fields, so VAR 2 here means no
  // post-chirp (intensity-only plans).
  constexpr bool FAST = VAR >= 1;
  constexpr bool NO_POST = VAR == 2;
  constexpr int RB = row_lds_bytes<L, kSplit>();
  constexpr int C = L / 2;    // staging chunk along the transform
  constexpr int SST = C + 9;  // staging stride per column (elements)
  constexpr int STAGE_BYTES = G * SST * 8;
  constexpr int XCH_BYTES = G * RB > STAGE_BYTES ? G * RB : STAGE_BYTES;
  using T = SharedTables<L>;
  static_assert((G & (G - 1)) == 0, "columns per workgroup must be a power of two");
  // Shared tables, then the exchange buffers (reused as the store staging).
  __shared__ __align__(16) unsigned char lds[T::bytes + XCH_BYTES];
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  unsigned char* xbuf = lds + T::bytes;
  float2* st = reinterpret_cast<float2*>(xbuf);

  const int tile = xcd_tile(blockIdx.x, args.total_tiles);
  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  const int c0 = (tile - args.tile_prefix[jid]) * G;
  const int g = TPR >= 64 ? uniform(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  const int ncols = J.n_rows;
  const int n_in = J.n_in;
  const int in_ld = (int)J.in_ld;
  const float2* __restrict__ pre = J.pre;
  const bool real_in = (J.mode & kInReal) != 0;
  // Column of the store staging loop for this thread (fixed: THREADS is a multiple of G).
  const int gs = threadIdx.x & (G - 1);
  const bool col_ok = c0 + gs < ncols;

  // Column c0 + g of the column-major input copy, loaded like a row (a
  // column past the grid's edge computes on the last one and stores nothing).
  const int cl = c0 + g < ncols ? c0 + g : ncols - 1;
  float2 v[R];
  if constexpr (FAST) {
    if (real_in) load_half<TPR, R, true>(v, static_cast<const float*>(J.in) + (int64_t)cl * in_ld, pre, t);
    else load_half<TPR, R, false>(v, static_cast<const float2*>(J.in) + (int64_t)cl * in_ld, pre, t);
  } else {
    if (real_in)
      load_row<TPR, R, true>(v, static_cast<const float*>(J.in) + (int64_t)cl * in_ld, pre, n_in, t);
    else
      load_row<TPR, R, false>(v, static_cast<const float2*>(J.in) + (int64_t)cl * in_ld, pre, n_in, t);
  }

  const float2* __restrict__ H = J.H;
  if constexpr (T::on) {
    stage_tables<L, THREADS>(tws, hs, tw, H);
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  const int n_out = J.n_out;
  float2* out = static_cast<float2*>(J.out) + c0 + gs;
  const int out_ld = (int)J.out_ld;
  // HALF as in the row kernel; then only the first staging chunk exists.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? R / 2 : R;
    constexpr int NC = HALF ? 1 : 2;
    fft_row<PassPlan<L>, false, kSplit, T::src, HALF>(v, buf, t, twx);
    sched_fence();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[t + TPR * i] : gld(H, (unsigned)(t + TPR * i)));
    sched_fence();
    fft_row<PassPlan<L>, true, kSplit, T::src, HALF>(v, buf, t, twx);

    if (!NO_POST && (J.mode & kUsePost)) {
      const float2* post = J.post;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const int m = t + TPR * i;
        if (TPR * (i + 1) <= n_out || m < n_out) v[i] = cmul(v[i], gld(post, (unsigned)m));
      }
    }
    if (J.colscale) {
      const float2 cs = gld(J.colscale, (unsigned)cl);
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
        const int m = t + TPR * i;
        if (TPR * (i + 1) <= n_out || m < n_out) st[g * SST + (m - m_lo)] = v[i];
      }
      __syncthreads();
      const int cnt = (n_out - m_lo < C ? n_out - m_lo : C) * G;
      for (int e = threadIdx.x; e < cnt; e += THREADS) {
        const int m = m_lo + e / G;
        if (col_ok) gst(out, (unsigned)(m * out_ld), st[gs * SST + (m - m_lo)]);
      }
    }
  };
  if constexpr (FAST) body(std::true_type{});
  else body(std::false_type{});
}

bool supported_length(int L) { return twiddle_len(L, false) >= 0; }

// Tile widths a pass can be launched with at each length (the workgroup is
// G * TPR threads and G exchange rows must fit in LDS); the first entry is
// the default.
#define SFD_ROW_SHAPES(X) \
  X(64, 32) X(64, 16) X(64, 64) X(128, 16) X(128, 8) X(128, 32) X(256, 8) X(256, 4) X(256, 16) \
  X(512, 4) X(512, 2) X(512, 8) X(1024, 2) X(1024, 1) X(1024, 4) X(2048, 2) X(2048, 1) X(2048, 4) \
  X(4096, 1) X(8192, 1)
#define SFD_COL_SHAPES(X) \
  X(64, 32) X(64, 16) X(128, 16) X(128, 8) X(256, 8) X(256, 4) X(512, 8) X(512, 4) \
  X(1024, 8) X(1024, 4) X(1024, 16) X(2048, 8) X(2048, 4) X(2048, 2) X(4096, 2) X(4096, 4) \
  X(8192, 1) X(8192, 2)

int pass_tile_widths(int L, bool col, int* widths, int cap) {
  int n = 0;
#define SFD_PUSH(l, g) \
  if (l == L) {        \
    if (n < cap) widths[n] = g; \
    ++n;               \
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
#define SFD_LAUNCH_V(kern, l, g, v) \
  hipLaunchKernelGGL((kern<l, g, v>), dim3(a.total_tiles), dim3(PassShape<l, g>::THREADS), 0, s, a, tw)
#define SFD_LAUNCH_ROW(l, g)                          \
  if (!col && L == l && G == g) {                     \
    if (var == 2) SFD_LAUNCH_V(row_kernel, l, g, 2);  \
    else if (var == 1) SFD_LAUNCH_V(row_kernel, l, g, 1); \
    else SFD_LAUNCH_V(row_kernel, l, g, 0);           \
    return hipGetLastError();                         \
  }
#define SFD_LAUNCH_COL(l, g)                          \
  if (col && L == l && G == g) {                      \
    if (var == 2) SFD_LAUNCH_V(col_kernel, l, g, 2);  \
    else if (var == 1) SFD_LAUNCH_V(col_kernel, l, g, 1); \
    else SFD_LAUNCH_V(col_kernel, l, g, 0);           \
    return hipGetLastError();                         \
  }
  SFD_ROW_SHAPES(SFD_LAUNCH_ROW)
  SFD_COL_SHAPES(SFD_LAUNCH_COL)
#undef SFD_LAUNCH_ROW
#undef SFD_LAUNCH_COL
#undef SFD_LAUNCH_V
  return hipErrorInvalidValue;
}

}  // namespace sfd

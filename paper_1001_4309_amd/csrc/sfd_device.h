// Device code shared by the kernel translation units: chirp values of
// Eqs. (2)-(4), the setup roles, and the bodies of the column and row passes
// (templates instantiated by sfd_cols.hip, sfd_rows.hip and
// sfd_persist.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_core.h"
#include "sfd_internal.h"

namespace sfd {

// Global (address space 1) integer views used by the coherent loads and
// write-through stores below.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(1))) const uint32_t g_u32;
typedef __attribute__((address_space(1))) const uint64_t g_u64;
typedef __attribute__((address_space(1))) uint64_t g_u64w;
#else
typedef const uint32_t g_u32;
typedef const uint64_t g_u64;
typedef uint64_t g_u64w;
#endif

// Global loads that are coherent across the XCDs (device-scope relaxed
// atomic loads: they bypass the per-XCD caches' possibly stale lines).  The
// persistent launch reads what other items of the same launch wrote, on any
// XCD, through these; COH = false gives ordinary loads.
template <bool COH>
__device__ __forceinline__ float gld_c(const float* p, unsigned i) {
  if constexpr (COH) {
    return __builtin_bit_cast(float, __hip_atomic_load((g_u32*)p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  } else {
    return gld(p, i);
  }
}
template <bool COH>
__device__ __forceinline__ float2 gld_c(const float2* p, unsigned i) {
  if constexpr (COH) {
    return __builtin_bit_cast(float2, __hip_atomic_load((g_u64*)p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  } else {
    return gld(p, i);
  }
}
template <bool COH>
__device__ __forceinline__ float4 gld_c(const float4* p, unsigned i) {
  if constexpr (COH) {
    const float2 a = gld_c<true>(reinterpret_cast<const float2*>(p), 2 * i);
    const float2 b = gld_c<true>(reinterpret_cast<const float2*>(p), 2 * i + 1);
    return make_float4(a.x, a.y, b.x, b.y);
  } else {
    return gld(p, i);
  }
}

// A descriptor that no kernel writes (the call's descriptor image), read
// into scalar registers: the pointer (the same in every lane of the
// wavefront) is made wave-uniform and read through the constant address
// space, which the compiler serves with scalar loads.  For descriptors
// reached through pointers that it cannot otherwise prove global, uniform
// or unwritten.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  // (readfirstlane returns a signed int: each half goes through uint32_t so
  // that the low half is not sign-extended into the high one.)
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint64_t u = (hi << 32) | lo;
  return *reinterpret_cast<const __attribute__((address_space(4))) T*>(u);
#else
  return *p;
#endif
}

// Cooperative copies of N float4 from global memory into LDS by THREADS
// threads.  Every thread issues all of its loads before its first LDS
// write, so that their latencies overlap; a thread past the end of a table
// reloads its last entry instead of skipping the load, which keeps the loads
// branch-free.
template <int N, int THREADS>
struct CopyShare {
  static constexpr int K = N > 0 ? (N + THREADS - 1) / THREADS : 0;
  static constexpr int KA = K > 0 ? K : 1;  // register array size
};
template <int N, int THREADS, int KA, bool COH = false>
__device__ __forceinline__ void copy_load(float4 (&r)[KA], const float2* src, int tid) {
  const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int k = 0; k < CopyShare<N, THREADS>::K; ++k) {
    const int e = tid + k * THREADS;
    r[k] = gld_c<COH>(s4, (unsigned)(e < N ? e : N - 1));
  }
}
template <int N, int THREADS, int KA>
__device__ __forceinline__ void copy_store(float2* dst, const float4 (&r)[KA], int tid) {
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int k = 0; k < CopyShare<N, THREADS>::K; ++k) {
    const int e = tid + k * THREADS;
    if (N % THREADS == 0 || e < N) d4[e] = r[k];
  }
}
// exp(i pi v) for a large phase v (in half-turns).  The reduction to
// [-1, 1] is done in FP64, exact enough for phases of 10^5 half-turns and
// more.  The reduced argument r is split as r_hi + r_lo with r_hi its FP32
// rounding; FP32 sin/cos of pi r_hi and the first-order correction for
// pi r_lo (|pi r_lo| < 1e-7, so the dropped second-order term is ~1e-14)
// give the FP32 result at FP32 sin/cos accuracy without FP64 trigonometry.
__device__ __forceinline__ float2 cispi_f64(double v) {
#pragma clang fp contract(off)
  const double r = v - 2.0 * rint(0.5 * v);
  const float rh = static_cast<float>(r);
  const float rl = static_cast<float>((r - static_cast<double>(rh)) * M_PI);
  float s, c;
  sincospif(rh, &s, &c);
  return make_float2(fmaf(-s, rl, c), fmaf(c, rl, s));
}

// The same phase carried entirely in FP32 (comparison variant).
__device__ __forceinline__ float2 cispi_f32(float v) {
#pragma clang fp contract(off)
  const float r = v - 2.0f * rintf(0.5f * v);
  float s, c;
  sincospif(r, &s, &c);
  return make_float2(c, s);
}

// The chirp values below are written with explicit fused multiply-adds and
// no contraction left to the compiler, so that every kernel that evaluates
// one (the setup kernel, the persistent launch's setup items and its column
// tiles) rounds it identically.
__device__ __forceinline__ float2 pre_value(const AxisJob& J, int m) {
#pragma clang fp contract(off)
  if (J.flags & kPhaseFp32) {
    const float p0 = (float)J.p0, a0 = (float)J.a0, il = (float)J.inv_lz, S = (float)J.S, c1 = (float)J.c1;
    const float fm = (float)m;
    const float x0 = fmaf(fm, p0, a0);
    float2 v = cispi_f32(fmaf(-S * fm, fm, fmaf(x0 * x0, il, -(2.0f * fm * S * c1))));
    if (J.flags & kMomentX0) {
      const float w = x0 * (float)J.wscale;
      v = make_float2(v.x * w, v.y * w);
    }
    return v;
  }
  const double dm = (double)m;
  const double x0 = fma(dm, J.p0, J.a0);
  float2 v = cispi_f64(fma(-J.S, (double)((int64_t)m * m), fma(x0 * x0, J.inv_lz, -(2.0 * dm * J.S * J.c1))));
  if (J.flags & kMomentX0) {
    const float w = (float)(x0 * J.wscale);
    v = make_float2(v.x * w, v.y * w);
  }
  return v;
}

__device__ __forceinline__ float2 post_value(const AxisJob& J, int m) {
#pragma clang fp contract(off)
  float2 v;
  if (J.flags & kPhaseFp32) {
    const float p1 = (float)J.p1, a1 = (float)J.a1, a0 = (float)J.a0, il = (float)J.inv_lz, S = (float)J.S;
    const float fm = (float)m;
    const float x1 = fmaf(fm, p1, a1);
    v = cispi_f32(fmaf(-S * fm, fm, fmaf(x1 * x1, il, -(2.0f * a0 * x1 * il))));
  } else {
    const double dm = (double)m;
    const double x1 = fma(dm, J.p1, J.a1);
    v = cispi_f64(fma(-J.S, (double)((int64_t)m * m), fma(x1 * x1, J.inv_lz, -(2.0 * J.a0 * x1 * J.inv_lz))));
  }
  return cmul(v, J.post_scale);
}

// h of Eq. (4) at storage index i in [0, L): lag k = i for i < n1, k = i - L
// otherwise; zero outside k in [-(n0-1), n1-1].
// h at lag k (without the window), which depends on k^2 only.
__device__ __forceinline__ float2 kernel_lag(const AxisJob& J, int k) {
#pragma clang fp contract(off)
  if (J.flags & kPhaseFp32) {
    const float fk = (float)k;
    return cispi_f32((float)J.S * fk * fk);
  }
  return cispi_f64(J.S * (double)((int64_t)k * k));
}
__device__ __forceinline__ float2 kernel_value(const AxisJob& J, int i) {
  const int k = i < J.n1 ? i : i - J.L;
  if (k < -(J.n0 - 1)) return make_float2(0.f, 0.f);
  return kernel_lag(J, k);
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
    case 1280: return twiddle_l<1280>(spec, e, out);
    case 1536: return twiddle_l<1536>(spec, e, out);
    case 1792: return twiddle_l<1792>(spec, e, out);
    case 2048: return twiddle_l<2048>(spec, e, out);
    case 4096: return twiddle_l<4096>(spec, e, out);
    case 8192: return twiddle_l<8192>(spec, e, out);
    default: return false;
  }
}


// Split (real/imaginary in turn) LDS exchanges halve the LDS a row needs.
constexpr bool kSplit = true;
// The lone kernel-spectrum transforms exchange complex values (one LDS round
// trip and two barriers per exchange instead of two and four): their
// latency, not their LDS footprint, is what matters.
constexpr bool kSpecSplit = false;

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
  // Up to L = 2048 the shape's twiddle table is staged in LDS (its loads are
  // issued first and overlap the evaluation of h; the stages then read LDS);
  // longer spectra read theirs from global memory, a stage ahead.
  static constexpr bool TW_LDS = L <= 2048;
  static constexpr int TW_N = twiddle_entries<P>();
  static constexpr int TW_BYTES = TW_LDS ? TW_N * 8 : 0;
  static constexpr int BYTES = GS * row_lds_bytes<L, kSpecSplit>() + TW_BYTES;  // exchange rows, table
};

// One kernel spectrum H = FFT_L(h) / L by the TPR threads of row g of a
// spectrum workgroup (t = thread in the row, r = thread in the group of
// kSetupThreads that shares the LDS area lds); J null: the row computes and
// stores nothing (it still takes part in the barriers and the table copy).  Each
// thread evaluates h straight into its FFT input slots (element t + TPR i).
// The twiddles come from the spectrum-shape table (built once per
// workspace): staged in LDS (SpecShape::TW_LDS, loads issued before h is
// evaluated) or read from global memory a stage ahead.
// Store of a complex value; WT: written through to memory at system scope
// (a relaxed atomic store), so that no dirty copy stays in the writer's
// XCD cache when other XCDs read it in the same launch.
template <bool WT>
__device__ __forceinline__ void gst_c(float2* p, unsigned i, float2 v) {
  if constexpr (WT) {
    __hip_atomic_store((g_u64w*)p + i, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    gst(p, i, v);
  }
}

// LAGS: the group's h values are already in its exchange row (evaluated by
// the caller with more threads; kSetupThreads-wide transforms only).
template <int L, bool WT = false, bool LAGS = false>
__device__ __forceinline__ void spectrum_row(const AxisJob* J, const float2* tw, void* lds, int g, int t, int r) {
  using P = SpecPlan<L>;
  using Sh = SpecShape<L>;
  constexpr int TPR = P::TPR;
  constexpr int R = P::R;
  constexpr int NT = Sh::TW_N / 2;  // table entries as float4 pairs
  static_assert(!Sh::TW_LDS || Sh::TW_N % 2 == 0, "tables are copied two entries at a time");
  float2* const tws = reinterpret_cast<float2*>(static_cast<char*>(lds) + Sh::GS * row_lds_bytes<L, kSpecSplit>());
  float4 twr[Sh::TW_LDS ? CopyShare<NT, kSetupThreads>::KA : 1];
  if constexpr (Sh::TW_LDS) copy_load<NT, kSetupThreads, CopyShare<NT, kSetupThreads>::KA>(twr, tw, r);
  float2* Hg = nullptr;
  float2 v[R];
  // The job's fields are read once (into scalar registers when a transform
  // spans whole wavefronts, so that every lane of one works on the same job),
  // and its output pointer is kept for the end.
  AxisJob Jv{};
  if (J) {
    if constexpr (TPR >= 64) Jv = load_uniform(J);
    else Jv = *J;
    Hg = Jv.H;
  }
  if constexpr (TPR == kSetupThreads) {
    // One transform per group: h depends on the lag's square only, so the
    // group evaluates it once per |lag| < max(n0, n1) into the exchange row
    // (not in use yet) and every thread picks its entries from there.
    float2* const e = static_cast<float2*>(lds);
    const int M = Jv.n0 > Jv.n1 ? Jv.n0 : Jv.n1;
    if (J && !LAGS)
      for (int m = r; m < M; m += kSetupThreads) e[m] = kernel_lag(Jv, m);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int idx = t + TPR * i;
      const int k = idx < Jv.n1 ? idx : idx - L;
      v[i] = (J && k >= -(Jv.n0 - 1)) ? e[k < 0 ? -k : k] : make_float2(0.f, 0.f);
    }
  } else if (J) {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = kernel_value(Jv, t + TPR * i);
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = make_float2(0.f, 0.f);
  }
  if constexpr (Sh::TW_LDS) {
    copy_store<NT, kSetupThreads>(tws, twr, r);
    __syncthreads();
    fft_row<P, false, kSpecSplit, kTwShared>(v, static_cast<char*>(lds) + g * row_lds_bytes<L, kSpecSplit>(), t, tws,
                                             J != nullptr);
  } else {
    if constexpr (TPR == kSetupThreads) __syncthreads();  // every lag read before the exchanges write
    fft_row<P, false, kSpecSplit, kTwGlobal>(v, static_cast<char*>(lds) + g * row_lds_bytes<L, kSpecSplit>(), t, tw,
                                             J != nullptr);
  }
  if (!Hg) return;
  const float inv = 1.0f / (float)L;
#pragma unroll
  for (int i = 0; i < R; ++i) gst_c<WT>(Hg, (unsigned)(t + TPR * i), make_float2(v[i].x * inv, v[i].y * inv));
}

// Spectrum role of the setup kernel: GS spectra of length L per workgroup.
template <int L>
__device__ __forceinline__ void setup_spectrum(const SetupArgs& A, const SetupRole& Ro, int rb, void* lds) {
  constexpr int TPR = SpecPlan<L>::TPR;
  constexpr int GS = SpecShape<L>::GS;
  const int g = TPR >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / TPR) : threadIdx.x / TPR;
  const int t = threadIdx.x - g * TPR;
  const int k = rb * GS + g;
  spectrum_row<L>(k < Ro.c ? &A.axis[Ro.b + k] : nullptr, Ro.tw, lds, g, t, (int)threadIdx.x);
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
  if (MAXL >= 2048) b = cmax(cmax(b, spectrum_lds_bytes<2048>()), spectrum_lds_bytes<1280>());
  if (MAXL >= 2048) b = cmax(cmax(b, spectrum_lds_bytes<1536>()), spectrum_lds_bytes<1792>());
  if (MAXL >= 4096) b = cmax(b, spectrum_lds_bytes<4096>());
  if (MAXL >= 8192) b = cmax(b, spectrum_lds_bytes<8192>());
  return b;
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

// Input slots of the specialised (fast) pass kernels: the input fills the
// first RIN x TPR samples of the padded row (half of it at power-of-two
// lengths, the paper's doubled grid; 1024 samples at the smooth lengths,
// where a 1024-sample hologram meets a smaller view), and the output is at
// most as long.  PRUNE: the input is exactly half the row, so the first
// forward and last inverse stage skip the zero and the cropped half.
template <int L>
struct FastIn {
  static constexpr int TPR = PassPlan<L>::TPR;
  static constexpr int R = PassPlan<L>::R;
  static constexpr bool pow2 = (L & (L - 1)) == 0;
  static constexpr int RIN = pow2 ? R / 2 : 1024 / TPR;
  static constexpr bool PRUNE = 2 * RIN == R;
  static_assert(RIN * TPR <= L, "the input fits the padded row");
};

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
// The common case only (n = RIN TPR, see FastIn): the first RIN slots
// loaded, the padding zero.
template <int TPR, int R, int RIN, bool REAL>
__device__ __forceinline__ void load_half(float2 (&v)[R], const void* in, const float2* pre, int t) {
  if (pre) {
#pragma unroll
    for (int i = 0; i < RIN; ++i) v[i] = pre_times_in<REAL, true>(in, pre, (unsigned)(t + TPR * i));
  } else {
#pragma unroll
    for (int i = 0; i < RIN; ++i) v[i] = pre_times_in<REAL, false>(in, pre, (unsigned)(t + TPR * i));
  }
#pragma unroll
  for (int i = RIN; i < R; ++i) v[i] = make_float2(0.f, 0.f);
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
// N: the slots that can hold outputs (the first N of the R).
template <int TPR, int N, int R>
__device__ __forceinline__ void row_accumulate(const RowJob& J, const float2 (&v)[R], int row, bool valid, int t,
                                               double (&a)[4]) {
  static_assert(N <= R, "output slots are among the row's slots");
  if (valid) {
    const int n_out = J.n_out;
    const int mode = J.mode;
    const double Y = row * J.yp + J.ya;
    const int64_t base = (int64_t)row * J.red_ld;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int m = t + TPR * i;
      if (m < n_out) {
        float2 G, V;
        if (mode & kRedSwap) {
          G = v[i];
          V = (mode & kRedRealRef)
                  ? make_float2(gld(reinterpret_cast<const float*>(J.uref) + base, (unsigned)m), 0.f)
                  : gld(J.uref + base, (unsigned)m);
        } else if (J.giref) {
          const float gi = 2.0f * gld(J.giref + base, (unsigned)m);
          const float2 u = gld(J.uref + base, (unsigned)m);
          G = make_float2(gi * u.x, gi * u.y);
          V = v[i];
        } else {
          G = gld(J.gref + base, (unsigned)m);
          V = v[i];
        }
        const double pr = (double)G.x * V.x + (double)G.y * V.y;
        const double pi = (double)G.x * V.y - (double)G.y * V.x;
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

// row_accumulate for the fast kernels' N = RIN output slots: every reference
// load of the row is issued first (branch-free: entries past n_out read the
// last one and are not accumulated), so that one wait covers them all; then
// the same products and sums in the same order.
template <int TPR, int N, int R>
__device__ __forceinline__ void row_accumulate_batched(const RowJob& J, const float2 (&v)[R], int row, bool valid,
                                                       int t, double (&a)[4]) {
  static_assert(N <= R, "output slots are among the row's slots");
  if (!valid) return;
  const int n_out = J.n_out;
  const int mode = J.mode;
  const bool gi = J.giref != nullptr;
  const int64_t base = (int64_t)row * J.red_ld;
  float2 A[N];
  float B[N];
  if (mode & kRedSwap) {
    if (mode & kRedRealRef) {
      const float* u = reinterpret_cast<const float*>(J.uref) + base;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int m = t + TPR * i;
        A[i] = make_float2(gld(u, (unsigned)(m < n_out ? m : n_out - 1)), 0.f);
      }
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int m = t + TPR * i;
        A[i] = gld(J.uref + base, (unsigned)(m < n_out ? m : n_out - 1));
      }
    }
  } else if (gi) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int m = t + TPR * i;
      const unsigned mc = (unsigned)(m < n_out ? m : n_out - 1);
      A[i] = gld(J.uref + base, mc);
      B[i] = gld(J.giref + base, mc);
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int m = t + TPR * i;
      A[i] = gld(J.gref + base, (unsigned)(m < n_out ? m : n_out - 1));
    }
  }
  const double Y = row * J.yp + J.ya;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int m = t + TPR * i;
    if (m < n_out) {
      float2 G, V;
      if (mode & kRedSwap) {
        G = v[i];
        V = A[i];
      } else if (gi) {
        const float g2 = 2.0f * B[i];
        G = make_float2(g2 * A[i].x, g2 * A[i].y);
        V = v[i];
      } else {
        G = A[i];
        V = v[i];
      }
      const double pr = (double)G.x * V.x + (double)G.y * V.y;
      const double pi = (double)G.x * V.y - (double)G.y * V.x;
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

// Cooperative copies into LDS at the start of a workgroup (see CopyShare):
// the twiddle table, the job's H and, for slots that run several transforms
// of the job (PRE), the first L/2 entries of its pre-chirp when it has one.
template <int L, int THREADS, bool PRE, int NPRE = L / 2, bool COH = false, bool HCOPY = true, bool TWCOPY = true>
__device__ __forceinline__ void stage_tables(float2* tws, float2* hs, float2* ps, const float2* __restrict__ tw,
                                             const float2* __restrict__ H, const float2* __restrict__ pre, int tid) {
  static_assert(SharedTables<L>::tw_n % 2 == 0, "tables are copied two entries at a time");
  constexpr int NT = TWCOPY ? SharedTables<L>::tw_n / 2 : 0;
  constexpr int NH = HCOPY ? L / 2 : 0;
  constexpr int NP = PRE ? NPRE / 2 : 0;
  float4 a[CopyShare<NT, THREADS>::KA];
  float4 b[CopyShare<NH, THREADS>::KA];
  float4 c[CopyShare<NP, THREADS>::KA];
  copy_load<NT, THREADS>(a, tw, tid);
  copy_load<NH, THREADS, CopyShare<NH, THREADS>::KA, COH>(b, H, tid);
  if constexpr (PRE) {
    if (pre) copy_load<NP, THREADS, CopyShare<NP, THREADS>::KA, COH>(c, pre, tid);
  }
  copy_store<NT, THREADS>(tws, a, tid);
  copy_store<NH, THREADS>(hs, b, tid);
  if constexpr (PRE) {
    if (pre) copy_store<NP, THREADS>(ps, c, tid);
  }
}
// The kernel spectrum H alone into LDS (its copy deferred by stage_tables).
template <int L, int THREADS, bool COH>
__device__ __forceinline__ void stage_spectrum(float2* hs, const float2* __restrict__ H, int tid) {
  constexpr int NH = L / 2;
  float4 b[CopyShare<NH, THREADS>::KA];
  copy_load<NH, THREADS, CopyShare<NH, THREADS>::KA, COH>(b, H, tid);
  copy_store<NH, THREADS>(hs, b, tid);
}

// A camera sample resized along x (see TileJob): row n of a frame of ns
// samples per row, read at column c of a grid nx wide.
template <typename S>
__device__ __forceinline__ float resample_at(const S* in, int ns, int nx, int n, int c) {
  double sx = ((double)c + 0.5) * (double)ns / (double)nx - 0.5;
  sx = fmin(fmax(sx, 0.0), (double)(ns - 1));
  const int i0 = (int)sx;
  const int i1 = i0 + 1 < ns ? i0 + 1 : ns - 1;
  const float wt = (float)(sx - (double)i0);
  const float a = (float)gld(in, (unsigned)(n * ns + i0)), b = (float)gld(in, (unsigned)(n * ns + i1));
  return fmaf(wt, b - a, a);
}

// Row-major real input of a column tile's round (RowJob::in_fmt != 0): the
// round's NS columns from cb on, every one of the K x THREADS / NS rows, by
// the whole workgroup (element f = tid + THREADS k is row f / NS, column
// cb + f % NS; columns past the grid repeat its last).  Rows of NS
// consecutive samples; the format is decided once, outside the loads.
template <int K, int THREADS, int NS>
__device__ __forceinline__ void fetch_rowmajor(float2 (&x)[K], const void* in, int fmt, int ld, int ncols, int cb,
                                               int tid) {
  auto run = [&](auto sample) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int f = tid + THREADS * k;
      const int c = cb + f % NS;
      x[k].x = sample(f / NS, c < ncols ? c : ncols - 1);
    }
  };
  if (fmt == 32) run([&](int n, int c) { return gld(static_cast<const float*>(in), (unsigned)(n * ld + c)); });
  else if (fmt == 8)
    run([&](int n, int c) { return resample_at(static_cast<const unsigned char*>(in), ld, ncols, n, c); });
  else if (fmt == 16)
    run([&](int n, int c) { return resample_at(static_cast<const unsigned short*>(in), ld, ncols, n, c); });
  else run([&](int n, int c) { return resample_at(static_cast<const float*>(in), ld, ncols, n, c); });
}

// The common case (input of L/2 samples) in two steps, so that the loads of
// the next transform can be issued before the current one is computed:
// fetch_half loads the raw first half (a real input only into .x),
// apply_half forms the padded, pre-chirped row from it (pre from LDS, or
// none when ps is null).
template <int TPR, bool REAL, int H, bool COH = false>
__device__ __forceinline__ void fetch_half(float2 (&x)[H], const void* in, int64_t off, int t) {
  if constexpr (REAL) {
    const float* p = static_cast<const float*>(in) + off;
#pragma unroll
    for (int i = 0; i < H; ++i) x[i].x = gld_c<COH>(p, (unsigned)(t + TPR * i));
  } else {
    const float2* p = static_cast<const float2*>(in) + off;
#pragma unroll
    for (int i = 0; i < H; ++i) x[i] = gld_c<COH>(p, (unsigned)(t + TPR * i));
  }
}
template <int TPR, int R, int RIN, bool REAL>
__device__ __forceinline__ void apply_half(float2 (&v)[R], const float2 (&x)[RIN], const float2* ps, int t) {
  if (!ps) {
#pragma unroll
    for (int i = 0; i < RIN; ++i) v[i] = REAL ? make_float2(x[i].x, 0.f) : x[i];
  } else {
#pragma unroll
    for (int i = 0; i < RIN; ++i) {
      const float2 p = ps[t + TPR * i];
      v[i] = REAL ? make_float2(x[i].x * p.x, x[i].x * p.y) : cmul(x[i], p);
    }
  }
#pragma unroll
  for (int i = RIN; i < R; ++i) v[i] = make_float2(0.f, 0.f);
}

// x transforms: row r of the job reads in + r * in_ld and writes
// out + r * out_ld (contiguous), both straight from registers.
// VAR selects a specialisation, which keeps the code of the common cases
// small: 0 = any job; 1 = every job of the launch has an input of L/2
// samples, a complex input, an output of at most L/2 and no reduction (half
// loads, pruned transforms, no reduction epilogue); 2 = as 1, and the jobs
// write only intensities; 3 = as 1 with the reduction epilogue (over the
// outputs of the first half).  P > 1: each slot runs several rows in turn.  In
// the specialisations a slot (one wavefront) takes the rows of its tile one
// at a time from a counter in LDS, so that a wavefront that gets more of its
// SIMD takes more rows and the wavefronts of the workgroup finish together;
// the next row's input is fetched while the current row is transformed, and
// the pre-chirp is read from an LDS copy.  The general kernel runs rows
// row0 + p NS, p < P, of its tile.
// LDS bytes of one row tile: shared tables, the pre-chirp copy, exchange
// buffers, then room for the epilogue reduction (4 doubles per wavefront)
// and the tile's row counter.
template <int L, int GR, int VAR, int P>
struct RowLds {
  using S = PassShape<L, GR, P>;
  static constexpr bool PF = VAR >= 1 && P > 1;
  static constexpr int PRE_BYTES = PF ? FastIn<L>::RIN * FastIn<L>::TPR * 8 : 0;
  static constexpr int bytes =
      SharedTables<L>::bytes + PRE_BYTES + S::NS * row_lds_bytes<L, kSplit>() + S::NW * 32 + (PF ? 16 : 0);
};

// A call made once the body's last transform is computed, before its last
// stores leave (the persistent launch takes its next ticket there, so that
// the ticket's latency overlaps the stores).  NoTail does nothing.
struct NoTail {
  __device__ __forceinline__ void operator()() const {}
};

// tid: the thread's index in the workgroup (threadIdx.x; the persistent
// launch passes it through an opaque move, so that nothing derived from it
// is hoisted out of its item loop).  The same holds for col_body.
// COH: read what other items of a persistent launch wrote (the input, H,
// the pre- and post-chirps) with loads coherent across XCDs (gld_c).
// TW_STAGED: the caller has already put the twiddle table into the tile's
// LDS tables (a persistent launch fetches it while it waits for the view's
// column tiles).
template <int L, int GR, int VAR, int P, bool COH = false, bool TW_STAGED = false, typename TAIL = NoTail>
__device__ __forceinline__ void row_body(const PassArgs& args, const float2* __restrict__ tw, const int tile,
                                         unsigned char* __restrict__ lds, const int tid, const TAIL& tail = TAIL{}) {
  using S = PassShape<L, GR, P>;
  constexpr int TPR = S::TPR;
  constexpr int R = L / TPR;
  constexpr int NS = S::NS;
  constexpr int RB = row_lds_bytes<L, kSplit>();
  constexpr bool FAST = VAR >= 1;
  constexpr bool INT_ONLY = VAR == 2;
  constexpr bool RED = VAR == 3;
  constexpr bool PF = FAST && P > 1;
  using T = SharedTables<L>;
  static_assert(P == 1 || (T::on && TPR <= 64), "slots of several transforms are single wavefronts with LDS tables");
  static_assert(!PF || TPR == 64, "a queue slot is one whole wavefront");
  constexpr int PRE_BYTES = RowLds<L, GR, VAR, P>::PRE_BYTES;
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  float2* ps = reinterpret_cast<float2*>(lds + T::bytes);
  unsigned char* xbuf = lds + T::bytes + PRE_BYTES;

  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  // With TPR >= 64 a row is a whole number of wavefronts: g is wave-uniform.
  const int g = TPR >= 64 ? uniform(tid / TPR) : tid / TPR;
  const int t = tid - g * TPR;
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
    if (tid == 0) *counter = 0;
    __syncthreads();
  }
  const bool lane0 = (tid & 63) == 0;
  auto grab = [&]() -> int {
    int r = 0;
    if (lane0) r = atomicAdd(counter, 1);
    return r;
  };
  constexpr int RIN = FastIn<L>::RIN;
  constexpr bool PRUNE = FastIn<L>::PRUNE;
  float2 v[R];
  float2 x[PF ? RIN : 1];
  auto load = [&](int row, int t) {
    const int64_t off = (int64_t)(row < n_rows ? row : 0) * in_ld;
    if constexpr (PF) {
      fetch_half<TPR, false, RIN, COH>(x, in, off, t);
    } else if constexpr (FAST) {
      load_half<TPR, R, RIN, false>(v, static_cast<const float2*>(in) + off, pre, t);
    } else {
      if (real_in) load_row<TPR, R, true>(v, static_cast<const float*>(in) + off, pre, n_in, t);
      else load_row<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, n_in, t);
    }
  };
  static_assert(!TW_STAGED || T::on, "staged twiddles go with LDS tables");
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
    stage_tables<L, S::THREADS, PF, RIN * TPR, COH, true, !TW_STAGED>(tws, hs, ps, tw, H, pre, tid);
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // HALF: the common case (input of RIN TPR samples, output of at most as
  // many, see FastIn), where with PRUNE the first forward and the last
  // inverse stage skip the padded and the cropped half.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? RIN : R;
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
        apply_half<TPR, R, RIN, false>(v, x, pre ? ps : nullptr, tl);
        sched_fence();
        if (prev >= 0) flush(prev, tl);
        sched_fence();
        if (r_next < tile_rows) load(tile_row0 + r_next, tl);
        // The row after next: taken now, read after this row's transforms.
        pend = r_next < tile_rows ? grab() : tile_rows;
      } else if (p > 0) {
        load(row, tl);
      }
      fft_row<PassPlan<L>, false, kSplit, T::src, HALF && PRUNE>(v, buf, tl, twx);
      sched_fence();
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[tl + TPR * i] : gld(H, (unsigned)(tl + TPR * i)));
      sched_fence();
      fft_row<PassPlan<L>, true, kSplit, T::src, HALF && PRUNE>(v, buf, tl, twx);

      if (!INT_ONLY && (mode & kUsePost)) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          const int m = tl + TPR * i;
          // HALF: a clamped (branch-free) load; entries past n_out are never stored.
          if (HALF) v[i] = cmul(v[i], gld_c<COH>(post, (unsigned)(m < n_out ? m : n_out - 1)));
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
      if constexpr (RED && HALF) {
        if (mode & kReduce) row_accumulate_batched<TPR, RL>(J, v, row, valid, tl, acc);
      } else if constexpr (!HALF) {
        if (mode & kReduce) row_accumulate<TPR, RL>(J, v, row, valid, tl, acc);
      }
      if constexpr (PF) {
        prev = row;
        r_cur = r_next;
        r_next = uniform(pend);
      }
    }
    if constexpr (PF) {
      tail();
      if (prev >= 0) flush(prev, t);
    }
    if constexpr (!HALF || RED) {
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
// LDS bytes of one column tile: shared tables, the pre-chirp copy, then the
// exchange buffers (reused as the store staging).
template <int L, int GC, int VAR, int P>
struct ColLds {
  using S = PassShape<L, GC, P>;
  static constexpr bool PF = VAR >= 1 && P > 1;
  static constexpr int CIN = FastIn<L>::RIN * FastIn<L>::TPR;  // rows of the fast kernels' one staging chunk
  // The pre-chirp copy, then (kernels that evaluate it themselves) the
  // colscale factors of the tile's GC columns and a flag word.
  static constexpr int PRE_BYTES = PF ? CIN * 8 + GC * 8 + 16 : 0;
  static constexpr int STAGE_BYTES = S::NS * ((CIN > L / 2 ? CIN : L / 2) + 9) * 8;
  static constexpr int XCH_BYTES =
      S::NS * row_lds_bytes<L, kSplit>() > STAGE_BYTES ? S::NS * row_lds_bytes<L, kSplit>() : STAGE_BYTES;
  static constexpr int bytes = SharedTables<L>::bytes + PRE_BYTES + XCH_BYTES;
};

// RM: a persistent launch's real-hologram column tiles read the hologram
// itself, row-major (RowJob::in_fmt), and turn each round's columns around
// in an LDS area after the tile's own (kColRmBytes); no column-major copy.
// SELF (slots of several columns only): the tile evaluates the pre-chirp of
// its columns and their colscale factors itself from the view's axis jobs
// (RowJob::ax_pre, ax_scale) instead of reading the chirp tables, so that a
// persistent launch's column tiles wait for nothing but the kernel spectrum.
// DEFER: the first thread asks dep.ready() at the start whether the spectrum
// is in; if so it is copied with the other tables, otherwise the tile waits
// for it (dep(), a call every thread makes) only once its first columns'
// forward transforms are done, and copies it then.
template <int L>
constexpr int col_rm_bytes() {
  return 8 * (FastIn<L>::RIN * FastIn<L>::TPR + 4) * 4;
}
template <int L, int GC, int VAR, int P, bool COH = false, bool RM = false, bool SELF = false,
          bool DEFER = false, typename TAIL = NoTail, typename DEP = NoTail>
__device__ __forceinline__ void col_body(const PassArgs& args, const float2* __restrict__ tw, const int tile,
                                         unsigned char* __restrict__ lds, const int tid0, const TAIL& tail = TAIL{},
                                         const DEP& dep = DEP{}) {
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
  constexpr int RIN = FastIn<L>::RIN;
  constexpr bool PRUNE = FastIn<L>::PRUNE;
  // Staging chunk along the transform: the fast kernels' outputs (at most
  // RIN TPR rows) in one chunk, the general kernel's in two of L/2 rows.
  constexpr int C = FAST ? RIN * TPR : L / 2;
  constexpr int SST = ColLds<L, GC, VAR, P>::CIN > L / 2 ? ColLds<L, GC, VAR, P>::CIN + 9 : L / 2 + 9;
  using T = SharedTables<L>;
  static_assert((NS & (NS - 1)) == 0, "slots per workgroup must be a power of two");
  static_assert(P == 1 || (T::on && TPR <= 64), "slots of several transforms are single wavefronts with LDS tables");
  constexpr int PRE_BYTES = ColLds<L, GC, VAR, P>::PRE_BYTES;
  float2* tws = reinterpret_cast<float2*>(lds);
  float2* hs = tws + T::tw_n;
  float2* ps = reinterpret_cast<float2*>(lds + T::bytes);
  unsigned char* xbuf = lds + T::bytes + PRE_BYTES;
  float2* st = reinterpret_cast<float2*>(xbuf);
  float2* const csl = ps + ColLds<L, GC, VAR, P>::CIN;  // SELF: colscale of the tile's columns
  static_assert(!SELF || (PF && (RIN * TPR) % THREADS == 0), "self-evaluated chirps: slots of several columns");
  static_assert(!DEFER || SELF, "a deferred spectrum goes with self-evaluated chirps");

  const int jid = find_job(args, tile);
  const RowJob& J = args.jobs[jid];
  const int c0 = (tile - args.tile_prefix[jid]) * GC;
  const int g = TPR >= 64 ? uniform(tid0 / TPR) : tid0 / TPR;
  const int t = tid0 - g * TPR;
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
  float2 x[PF ? RIN : 1];
  float2 csn = make_float2(1.f, 0.f);
  static_assert(!RM || (PF && REAL && NS == 8), "row-major input: real, several columns per slot, 8 slots");
  constexpr int RS = RIN * TPR + 4;  // LDS stride of a column of the round (RM)
  float* const rmb = reinterpret_cast<float*>(lds + ColLds<L, GC, VAR, P>::bytes);
  const int in_fmt = RM ? J.in_fmt : 0;
  auto load = [&](int p, int t, int tw_) {
    const int c = c0 + p * NS + g;
    const int cl = c < ncols ? c : ncols - 1;
    const int64_t off = (int64_t)cl * in_ld;
    if constexpr (RM) {
      fetch_rowmajor<RIN, THREADS, NS>(x, in, in_fmt, in_ld, ncols, c0 + p * NS, tw_);
    } else if constexpr (PF) {
      fetch_half<TPR, REAL, RIN, COH>(x, in, off, t);
    } else if constexpr (FAST) {
      if constexpr (REAL) load_half<TPR, R, RIN, true>(v, static_cast<const float*>(in) + off, pre, t);
      else load_half<TPR, R, RIN, false>(v, static_cast<const float2*>(in) + off, pre, t);
    } else {
      if (real_in) load_row<TPR, R, true>(v, static_cast<const float*>(in) + off, pre, n_in, t);
      else load_row<TPR, R, false>(v, static_cast<const float2*>(in) + off, pre, n_in, t);
    }
    if constexpr (!SELF) {
      if (colscale) csn = gld_c<COH>(colscale, (unsigned)cl);
    }
  };
  bool r0 = false;
  if constexpr (DEFER) {
    if (tid0 == 0) r0 = dep.ready();
  }
  // SELF: the twiddle table's loads (and the spectrum's, when it is not
  // deferred) and the first columns' loads are issued before the chirps are
  // evaluated, so that their latency overlaps that evaluation.
  constexpr int NTW = T::tw_n / 2, NH = L / 2;
  float4 twr[SELF ? CopyShare<NTW, THREADS>::KA : 1];
  float4 hr[SELF && !DEFER ? CopyShare<NH, THREADS>::KA : 1];
  if constexpr (SELF) {
    // Both axis jobs first: their loads (a chain behind the row job's) then
    // overlap each other and the loads below.
    const AxisJob ay = load_uniform(args.axis + J.ax_pre);
    const AxisJob ax = load_uniform(args.axis + J.ax_scale);
    copy_load<NTW, THREADS>(twr, tw, tid0);
    if constexpr (!DEFER) copy_load<NH, THREADS, CopyShare<NH, THREADS>::KA, COH>(hr, H, tid0);
    load(0, t, tid0);
    if (pre) {
#pragma unroll
      for (int k = 0; k < RIN * TPR / THREADS; ++k) ps[tid0 + k * THREADS] = pre_value(ay, tid0 + k * THREADS);
    }
    if (colscale && tid0 < GC) {
      const int c = c0 + tid0;
      csl[tid0] = pre_value(ax, c < ncols ? c : ncols - 1);
    }
    sched_fence();
  } else {
    load(0, t, tid0);
  }

  bool ready = true;  // the spectrum is copied with the other tables
  if constexpr (DEFER) {
    int* const rdy = reinterpret_cast<int*>(csl + GC);
    if (tid0 == 0) *rdy = r0 ? 1 : 0;
    __syncthreads();
    ready = uniform(*rdy) != 0;
  }
  if constexpr (T::on) {
    if constexpr (SELF) {
      copy_store<NTW, THREADS>(tws, twr, tid0);
      if constexpr (!DEFER) copy_store<NH, THREADS>(hs, hr, tid0);
    } else {
      stage_tables<L, THREADS, PF, RIN * TPR, COH, !DEFER>(tws, hs, ps, tw, H, pre, tid0);
    }
    if constexpr (DEFER) {
      if (ready) stage_spectrum<L, THREADS, COH>(hs, H, tid0);
    }
    __syncthreads();
  }
  const float2* twx = T::on ? tws : tw;
  void* buf = xbuf + g * RB;
  // HALF as in the row kernel; then only the first staging chunk exists.
  auto body = [&](auto half_c) {
    constexpr bool HALF = decltype(half_c)::value;
    constexpr int RL = HALF ? RIN : R;
    constexpr int NC = HALF ? 1 : 2;
    // HALF: a round's staged values (RIN per thread) leave through a
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
        for (int k = 0; k < RIN; ++k) {
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
      const int tid = P > 1 ? opaque(tid0) : tid0;
      // Column of the store staging loop for this thread (fixed: THREADS is a multiple of NS).
      const int gs = tid & (NS - 1);
      const int cb = c0 + p * NS;  // first column of this round
      const bool col_ok = cb + gs < ncols;
      float2* out = out0 + cb + gs;
      float2 cs;
      if constexpr (PF) {
        if constexpr (SELF) cs = csl[p * NS + g];
        else cs = csn;
        if constexpr (RM) {
          // The round's columns turned around: slot g takes column g.
#pragma unroll
          for (int k = 0; k < RIN; ++k) {
            const int f = tid + THREADS * k;
            rmb[(f % NS) * RS + f / NS] = x[k].x;
          }
          __syncthreads();
#pragma unroll
          for (int i = 0; i < RIN; ++i) x[i].x = rmb[g * RS + tl + TPR * i];
        }
        apply_half<TPR, R, RIN, REAL>(v, x, pre ? ps : nullptr, tl);
        sched_fence();
        if (p > 0) {
          flush(cb - NS, tid);
          // The exchanges below reuse the staging memory.
          __syncthreads();
        }
        if (p + 1 < P) load(p + 1, tl, tid);
      } else {
        if (p > 0) load(p, tl, tid);
        cs = csn;
      }
      fft_row<PassPlan<L>, false, kSplit, T::src, HALF && PRUNE>(v, buf, tl, twx);
      sched_fence();
      if constexpr (DEFER) {
        if (p == 0 && !ready) {
          dep();
          stage_spectrum<L, THREADS, COH>(hs, H, tid);
          __syncthreads();
        }
      }
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cmul(v[i], T::on ? hs[tl + TPR * i] : gld(H, (unsigned)(tl + TPR * i)));
      sched_fence();
      fft_row<PassPlan<L>, true, kSplit, T::src, HALF && PRUNE>(v, buf, tl, twx);

      if (!NO_POST && (mode & kUsePost)) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          const int m = tl + TPR * i;
          // HALF: a clamped (branch-free) load; entries past n_out are never stored.
          if (HALF) v[i] = cmul(v[i], gld_c<COH>(post, (unsigned)(m < n_out ? m : n_out - 1)));
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
        for (int i = c * (RL / NC); i < (c + 1) * (RL / NC); ++i) {
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
    if constexpr (PF) {
      tail();
      flush(c0 + (P - 1) * NS, tid0);
    }
  };
  if constexpr (FAST) body(std::true_type{});
  else body(std::false_type{});
}



// Shapes a pass can be launched with at each length: X(L, G, P), G the tile
// width (transforms per workgroup), P the transforms each slot runs in turn.
// The workgroup is G / P slots of TPR threads, and their exchange rows must
// fit in LDS; the first entry per length is the default.
#define SFD_ROW_SHAPES(X) \
  X(64, 32, 1) X(64, 16, 1) X(64, 64, 1) X(128, 16, 1) X(128, 8, 1) X(128, 32, 1) X(256, 8, 1) X(256, 4, 1) \
  X(256, 16, 1) X(512, 4, 1) X(512, 2, 1) X(512, 8, 1) X(1024, 2, 1) X(1024, 1, 1) X(1024, 4, 1) X(1024, 8, 2) \
  X(1024, 16, 2) X(1280, 8, 2) X(1280, 16, 2) X(1280, 2, 1) X(1536, 8, 2) X(1536, 16, 2) X(1536, 2, 1) \
  X(1792, 8, 2) X(1792, 16, 2) X(1792, 2, 1) X(2048, 2, 1) X(2048, 1, 1) X(2048, 4, 1) X(2048, 8, 2) \
  X(2048, 16, 2) X(4096, 1, 1) X(8192, 1, 1)
#define SFD_COL_SHAPES(X) \
  X(64, 32, 1) X(64, 16, 1) X(128, 16, 1) X(128, 8, 1) X(256, 8, 1) X(256, 4, 1) X(512, 8, 1) X(512, 4, 1) \
  X(1024, 8, 1) X(1024, 4, 1) X(1024, 16, 1) X(1024, 32, 2) X(1280, 16, 2) X(1280, 8, 1) X(1536, 16, 2) \
  X(1536, 8, 1) X(1792, 16, 2) X(1792, 8, 1) X(2048, 8, 1) X(2048, 4, 1) X(2048, 2, 1) X(2048, 16, 2) \
  X(4096, 2, 1) X(4096, 4, 1) X(8192, 1, 1) X(8192, 2, 1)

// Launchers of the pass kernels (sfd_rows.hip, sfd_cols.hip).
hipError_t launch_row_pass(int L, int G, int var, const PassArgs& a, const float2* tw, hipStream_t s);
hipError_t launch_col_pass(int L, int G, int var, const PassArgs& a, const float2* tw, hipStream_t s);

}  // namespace sfd

// The persistent launch: every step of a batched forward in one kernel.
#include "sfd_device.h"

namespace sfd {

// ---------------------------------------------------------------------------
// Persistent launch (see PersistArgs): one kernel runs every item of a batch
// (setup, hologram strips, column tiles, row tiles), taking items in ticket
// order and waiting on completion counters for the items it depends on.

// Both passes of a persistent launch: kPG transforms per workgroup in
// kPG / kPP slots of one wavefront, each running kPP transforms in turn.
constexpr int kPG = 16, kPP = 2;
static_assert(PassShape<2048, kPG, kPP>::THREADS == kPersistThreads, "persistent workgroup shape");
static_assert(PassShape<1792, kPG, kPP>::THREADS == kPersistThreads, "persistent workgroup shape");
static_assert(PassShape<1536, kPG, kPP>::THREADS == kPersistThreads, "persistent workgroup shape");
static_assert(PassShape<1280, kPG, kPP>::THREADS == kPersistThreads, "persistent workgroup shape");
static_assert(PassShape<1024, kPG, kPP>::THREADS == kPersistThreads, "persistent workgroup shape");
static_assert(kStripW == kPG, "a column tile reads exactly one strip");

bool persist_length(int L) { return L == 1024 || L == 1280 || L == 1536 || L == 1792 || L == 2048; }

template <int L>
struct PersistPassLds {
  static constexpr int col = cmax(cmax(ColLds<L, kPG, 1, kPP>::bytes, ColLds<L, kPG, 2, kPP>::bytes),
                                  ColLds<L, kPG, 3, kPP>::bytes);
  static constexpr int row = cmax(RowLds<L, kPG, 1, kPP>::bytes, RowLds<L, kPG, 2, kPP>::bytes);
  static constexpr int bytes = cmax(col, row);
};
// Strip items stage a chunk of kStripW columns: 1024 rows of float32 or 512
// of complex64, with a column stride of CH + 4 elements.
constexpr int kStripLdsBytes = cmax(kStripW * (1024 + 4) * 4, kStripW * (512 + 4) * 8);
constexpr int kSetupItemLdsBytes =
    2 * cmax(cmax(cmax(SpecShape<1024>::BYTES, SpecShape<1280>::BYTES), cmax(SpecShape<1536>::BYTES,
                                                                            SpecShape<1792>::BYTES)),
             SpecShape<2048>::BYTES);
constexpr int kPersistPassLds =
    cmax(cmax(cmax(PersistPassLds<1024>::bytes, PersistPassLds<1280>::bytes),
              cmax(PersistPassLds<1536>::bytes, PersistPassLds<1792>::bytes)),
         PersistPassLds<2048>::bytes);
constexpr int kPersistLds = cmax(kPersistPassLds, cmax(kStripLdsBytes, kSetupItemLdsBytes));
// The real-hologram instance's column tiles turn their rows around in LDS
// after the tile's own area (col_rm_bytes; 1024-sample columns at every
// persistent length).
constexpr int kRmLdsBytes = cmax(cmax(ColLds<2048, kPG, 2, kPP>::bytes, ColLds<1792, kPG, 2, kPP>::bytes),
                                 cmax(cmax(ColLds<1536, kPG, 2, kPP>::bytes, ColLds<1280, kPG, 2, kPP>::bytes),
                                      ColLds<1024, kPG, 2, kPP>::bytes)) +
                            col_rm_bytes<2048>();
static_assert(col_rm_bytes<2048>() == col_rm_bytes<1280>() && col_rm_bytes<1024>() <= col_rm_bytes<2048>(),
              "one row-major staging size");

// Counters are read and advanced at device scope: the workgroups of a launch
// run on every XCD, and each XCD has its own L2.
__device__ __forceinline__ uint32_t sync_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t sync_add(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin limit of a dependency wait (each round is a device-scope load and a
// short sleep, about a microsecond): far beyond any real wait, so that a
// broken counter ends the launch with wrong results and a raised error word
// instead of hanging the device.
constexpr uint32_t kSpinLimit = 1u << 21;

// Memory ordering between items.  Everything an item writes for later items
// (spectra, chirp tables, strips of the hologram copy, the intermediate) is
// stored written-through at system scope, and everything an item reads from
// earlier items is loaded with device-coherent loads (gld_c), so no item
// ever finds a stale line in its XCD's cache and no cache-wide flush or
// invalidation is needed between items: a counter advances once every
// store of the item has completed (the barrier waits for them), and an item
// starts once its counters have reached their targets.

// Wait until counters a and b (b may be null) reach their targets: the
// first thread polls (with a backoff that grows to about a microsecond), the
// others wait at the barrier.
__device__ __forceinline__ void wait_counts(uint32_t* sync, const uint32_t* a, uint32_t ta, const uint32_t* b,
                                            uint32_t tb) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while ((sync_load(a) < ta || (b && sync_load(b) < tb)) && spins < kSpinLimit) {
      if (spins < 4) __builtin_amdgcn_s_sleep(4);
      else if (spins < 16) __builtin_amdgcn_s_sleep(16);
      else __builtin_amdgcn_s_sleep(40);
      ++spins;
    }
    if (spins >= kSpinLimit)
      __hip_atomic_store(&sync[kSyncErr * kSyncStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// Publish the workgroup's results: every thread's stores have completed
// (the barrier waits for them), then the first thread advances the counter.
__device__ __forceinline__ void signal_count(uint32_t* p) {
  __syncthreads();
  if (threadIdx.x == 0) sync_add(p, 1u);
}

// Spectrum item: one kernel spectrum (one axis of one view) with the setup
// kernel's transform shape (the two launch modes then give bit-identical
// results), written through (later items read it on other XCDs).  The
// first half of the workgroup runs the transform; the second half helps
// evaluate h where the shape evaluates it once per lag, and then only meets
// the transform's barriers, so each SIMD runs one transform's wavefront.
template <int L>
__device__ __forceinline__ void spectrum_item(const AxisJob* J, const float2* tw, unsigned char* lds, int tid) {
  constexpr int TPR = SpecPlan<L>::TPR;
  const int half = tid / kSetupThreads, r = tid - half * kSetupThreads;
  const int g = TPR >= 64 ? uniform(r / TPR) : r / TPR;
  const int t = r - g * TPR;
  if constexpr (TPR == kSetupThreads) {
    const AxisJob Jv = load_uniform(J);
    const int M = Jv.n0 > Jv.n1 ? Jv.n0 : Jv.n1;
    float2* const e = reinterpret_cast<float2*>(lds);  // the first half's exchange row
    for (int m = tid; m < M; m += kPersistThreads) e[m] = kernel_lag(Jv, m);
    spectrum_row<L, true, true>(half == 0 ? J : nullptr, tw, lds + half * SpecShape<L>::BYTES, g, t, r);
  } else {
    spectrum_row<L, true>(half == 0 && g == 0 ? J : nullptr, tw, lds + half * SpecShape<L>::BYTES, g, t, r);
  }
}

// Setup items of view v, three per view so that they run side by side:
// part 0 its y spectrum (what its column tiles wait for), part 1 its x
// spectrum, part 2 the chirp tables of both axes (each axis's fields read
// once).
__device__ __forceinline__ void persist_setup(const PersistArgs& A, int v, int part, unsigned char* lds, int tid) {
  const AxisJob* X = &A.axis[2 * v];
  const AxisJob* Y = &A.axis[2 * v + 1];
  if (part < 2) {
    const AxisJob* J = part == 0 ? Y : X;
    const float2* tw = A.tw_view[2 * v + (part == 0 ? 1 : 0)];
    switch (J->L) {
      case 2048: spectrum_item<2048>(J, tw, lds, tid); break;
      case 1792: spectrum_item<1792>(J, tw, lds, tid); break;
      case 1536: spectrum_item<1536>(J, tw, lds, tid); break;
      case 1280: spectrum_item<1280>(J, tw, lds, tid); break;
      default: spectrum_item<1024>(J, tw, lds, tid); break;
    }
    return;
  }
  const AxisJob jx = *X, jy = *Y;
  const int nx = jx.n0 + (jx.post ? jx.n1 : 0);
  const int total = nx + jy.n0 + (jy.post ? jy.n1 : 0);
  for (int i = tid; i < total; i += kPersistThreads) {
    if (i < jx.n0) gst_c<true>(jx.pre, (unsigned)i, pre_value(jx, i));
    else if (i < nx) gst_c<true>(jx.post, (unsigned)(i - jx.n0), post_value(jx, i - jx.n0));
    else if (i - nx < jy.n0) gst_c<true>(jy.pre, (unsigned)(i - nx), pre_value(jy, i - nx));
    else gst_c<true>(jy.post, (unsigned)(i - nx - jy.n0), post_value(jy, i - nx - jy.n0));
  }
}

// Strip item: columns [c0, c0 + kStripW) of a hologram, every row, into its
// column-major copy (see TileJob).  Rows go in chunks of CH: every load of a
// chunk is issued before the first is used (rows of kStripW consecutive
// samples; the sample format is decided once, outside the loads), the chunk
// is turned around in LDS, and each column leaves as a contiguous run of CH
// samples, written through (later items read it on other XCDs).
// FMT: 0 float32 (or complex64 for T = float2), 8 / 16 / 32 camera samples
// resized along x (real input only).
template <typename T, int CH, int FMT>
__device__ __forceinline__ void strip_chunks(const TileJob J, int c0, T* buf, int tid) {
  constexpr int W = kStripW, K = CH * W / kPersistThreads, ST = CH + 4;
  const int nx = J.nx, ny = J.ny, ld = J.ld, ns = J.nx_src;
  const auto rs = store_rsrc(J.out, (uint32_t)nx * (uint32_t)ld * (uint32_t)sizeof(T));
  for (int r0 = 0; r0 < ny; r0 += CH) {
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int f = tid + kPersistThreads * k;
      const int n0 = r0 + f / W, cc = c0 + f % W;
      const int n = n0 < ny ? n0 : ny - 1, c = cc < nx ? cc : nx - 1;
      if constexpr (FMT == 0) v[k] = gld(static_cast<const T*>(J.in), (unsigned)(n * nx + c));
      else if constexpr (FMT == 8) v[k] = resample_at(static_cast<const unsigned char*>(J.in), ns, nx, n, c);
      else if constexpr (FMT == 16) v[k] = resample_at(static_cast<const unsigned short*>(J.in), ns, nx, n, c);
      else v[k] = resample_at(static_cast<const float*>(J.in), ns, nx, n, c);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int f = tid + kPersistThreads * k;
      buf[(f % W) * ST + f / W] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int f = tid + kPersistThreads * k;
      const int c = f / CH, n = f % CH;
      const bool ok = r0 + n < ny && c0 + c < nx;
      bst<kWriteThrough>(rs, ok ? (uint32_t)((c0 + c) * ld + r0 + n) * (uint32_t)sizeof(T) : kDrop,
                         buf[c * ST + n]);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void persist_strip(const TileJob* Jp, int c0, unsigned char* lds, int tid) {
  const TileJob J = *Jp;  // fields read once
  if (J.complex_in) strip_chunks<float2, 512, 0>(J, c0, reinterpret_cast<float2*>(lds), tid);
  else if (J.nx_src <= 0) strip_chunks<float, 1024, 0>(J, c0, reinterpret_cast<float*>(lds), tid);
  else if (J.src_bits == 8) strip_chunks<float, 1024, 8>(J, c0, reinterpret_cast<float*>(lds), tid);
  else if (J.src_bits == 16) strip_chunks<float, 1024, 16>(J, c0, reinterpret_cast<float*>(lds), tid);
  else strip_chunks<float, 1024, 32>(J, c0, reinterpret_cast<float*>(lds), tid);
}

// CPLX: the kernel instance for complex holograms (column specialisation 1);
// the real-hologram instance holds specialisations 2 and 3.  Keeping them
// apart keeps each instance's register need that of its largest body.
// A column tile's dependency on its view's y-spectrum item (col_body's DEFER):
// ready() asks without waiting, the call waits (spec null: nothing to wait
// for, the tables are kept from an earlier call).
struct SpecDep {
  uint32_t* sync;
  const uint32_t* spec;
  __device__ bool ready() const { return !spec || sync_load(spec) >= 1u; }
  __device__ void operator()() const {
    if (spec) wait_counts(sync, spec, 1u, nullptr, 0u);
  }
};

// Column tiles evaluate their pre-chirp and colscale factors themselves
// (col_body's SELF), so they depend only on their view's y-spectrum item, and
// real-hologram tiles wait for it (dep) only before their first spectrum
// multiply (DEFER).
template <int L, bool CPLX, typename TAIL, typename DEP>
__device__ __forceinline__ void persist_col(const Segment& sg, int tile, unsigned char* lds, int tid, const TAIL& tail,
                                            const DEP& dep) {
  if constexpr (CPLX) {
    col_body<L, kPG, 1, kPP, true, false, true>(*sg.args, sg.tw, tile, lds, tid, tail);
  } else {
    if (sg.var == 2) col_body<L, kPG, 2, kPP, true, true, true, true>(*sg.args, sg.tw, tile, lds, tid, tail, dep);
    else col_body<L, kPG, 3, kPP, true, true, true, true>(*sg.args, sg.tw, tile, lds, tid, tail, dep);
  }
}
// A row tile's twiddle table (pairs of entries, at most kTwStageK per
// thread), fetched by the persistent kernel while it waits for the view's
// column tiles: loads, then (after the wait) LDS stores.
constexpr int kTwStageK = (SharedTables<2048>::tw_n / 2 + kPersistThreads - 1) / kPersistThreads;
__device__ __forceinline__ int twiddle_pairs(int L) {
  switch (L) {
    case 2048: return SharedTables<2048>::tw_n / 2;
    case 1792: return SharedTables<1792>::tw_n / 2;
    case 1536: return SharedTables<1536>::tw_n / 2;
    case 1280: return SharedTables<1280>::tw_n / 2;
    default: return SharedTables<1024>::tw_n / 2;
  }
}
static_assert(SharedTables<1792>::tw_n <= SharedTables<2048>::tw_n && SharedTables<1536>::tw_n <= SharedTables<2048>::tw_n &&
                  SharedTables<1280>::tw_n <= SharedTables<2048>::tw_n && SharedTables<1024>::tw_n <= SharedTables<2048>::tw_n,
              "the 2048 table is the longest");
__device__ __forceinline__ void stage_load(float4 (&a)[kTwStageK], const float2* tw, int n, int tid) {
  const float4* s4 = reinterpret_cast<const float4*>(tw);
#pragma unroll
  for (int k = 0; k < kTwStageK; ++k) {
    const int e = tid + k * kPersistThreads;
    a[k] = gld(s4, (unsigned)(e < n ? e : n - 1));
  }
}
__device__ __forceinline__ void stage_store(float2* tws, const float4 (&a)[kTwStageK], int n, int tid) {
  float4* d4 = reinterpret_cast<float4*>(tws);
#pragma unroll
  for (int k = 0; k < kTwStageK; ++k) {
    const int e = tid + k * kPersistThreads;
    if (e < n) d4[e] = a[k];
  }
}

// Row tiles find their twiddle table already in LDS.
template <int L, typename TAIL>
__device__ __forceinline__ void persist_row(const Segment& sg, int tile, unsigned char* lds, int tid, const TAIL& tail) {
  if (sg.var == 2) row_body<L, kPG, 2, kPP, true, true>(*sg.args, sg.tw, tile, lds, tid, tail);
  else row_body<L, kPG, 1, kPP, true, true>(*sg.args, sg.tw, tile, lds, tid, tail);
}

template <bool CPLX>
__global__ void __launch_bounds__(kPersistThreads) persist_kernel(const PersistArgs* __restrict__ pa) {
  __shared__ __align__(16) unsigned char lds[CPLX ? kPersistLds : cmax(kPersistLds, kRmLdsBytes)];
  __shared__ int s_ticket;
  const PersistArgs& A = *pa;
  uint32_t* const sync = A.sync;
  const int total = A.total;
  const int nview = A.nview;
  // Counter c is sync[c * kSyncStride].
  uint32_t* const spec_done = sync + kSyncHead * kSyncStride;
  uint32_t* const tab_done = spec_done + nview * kSyncStride;
  uint32_t* const col_done = tab_done + nview * kSyncStride;
  uint32_t* const strip_done = col_done + nview * kSyncStride;
  if (threadIdx.x == 0) s_ticket = (int)sync_add(&sync[kSyncTicket * kSyncStride], 1u);
  for (;;) {
    __syncthreads();
    const int t = s_ticket;
    if (t >= total) break;
    // The thread index enters each item through an opaque move: nothing
    // derived from it is hoisted out of the item loop (and held in registers
    // across every item).
    const int tid = opaque((int)threadIdx.x);
    int k = 0;
    while (k + 1 < A.nseg && t >= A.seg[k + 1].first) ++k;
    const Segment& sg = A.seg[k];
    const int local = t - sg.first;
    // Column and row tiles take the next ticket once their last transform is
    // computed (its latency then overlaps their last stores); the short setup
    // and strip items take it when they are done.
    uint32_t next = 0;
    bool took = false;
    const auto tail = [&]() {
      if (threadIdx.x == 0) next = sync_add(&sync[kSyncTicket * kSyncStride], 1u);
      took = true;
    };
    switch (sg.kind) {
      case kItemSetup: {
        // Items 0 .. nview-1: y spectrum of view i (its column tiles wait
        // for spec_done); nview .. 2 nview - 1: x spectrum, then the chirp
        // tables (its row tiles wait for both on tab_done).
        const int part = local / nview, v = local - part * nview;
        persist_setup(A, v, part, lds, tid);
        signal_count(part == 0 ? &spec_done[v * kSyncStride] : &tab_done[v * kSyncStride]);
        break;
      }
      case kItemStrip: {
        // Only complex holograms have strips (real ones are read in place).
        if constexpr (CPLX) {
          const int nsp = (A.tiles[0].nx + kStripW - 1) / kStripW;
          persist_strip(&A.tiles[local / nsp], (local % nsp) * kStripW, lds, tid);
        }
        signal_count(&strip_done[local * kSyncStride]);
        break;
      }
      case kItemCol: {
        const PassArgs& PA = *sg.args;
        const int jid = find_job(PA, local);
        const RowJob& J = PA.jobs[jid];
        const int view = J.view;
        const int nsp = (A.tiles[0].nx + kStripW - 1) / kStripW;
        const int strip = J.copy * nsp + (local - PA.tile_prefix[jid]);
        // Complex holograms: the strip and the spectra before the tile
        // starts.  Real holograms are read in place (no strips), and the
        // spectra are waited for inside the tile (dep).
        if (A.nstrips > 0)
          wait_counts(sync, &strip_done[strip * kSyncStride], 1u,
                      A.wait_setup ? &spec_done[view * kSyncStride] : nullptr, 1u);
        const SpecDep dep{sync, A.wait_setup ? &spec_done[view * kSyncStride] : nullptr};
        switch (sg.L) {
          case 2048: persist_col<2048, CPLX>(sg, local, lds, tid, tail, dep); break;
          case 1792: persist_col<1792, CPLX>(sg, local, lds, tid, tail, dep); break;
          case 1536: persist_col<1536, CPLX>(sg, local, lds, tid, tail, dep); break;
          case 1280: persist_col<1280, CPLX>(sg, local, lds, tid, tail, dep); break;
          default: persist_col<1024, CPLX>(sg, local, lds, tid, tail, dep); break;
        }
        signal_count(&col_done[view * kSyncStride]);
        break;
      }
      default: {
        const PassArgs& PA = *sg.args;
        const int view = PA.jobs[find_job(PA, local)].view;
        // The view's column tiles (and with them its spectra, which they
        // waited for) and, for the post-chirp, its tables item: waited for
        // inside the tile, once its twiddle loads are in flight.
        // The twiddle loads are in flight while the first thread polls.
        float4 twa[kTwStageK];
        const int ntw = twiddle_pairs(sg.L);
        stage_load(twa, sg.tw, ntw, tid);
        wait_counts(sync, &col_done[view * kSyncStride], (uint32_t)A.col_tiles[view],
                    A.wait_setup ? &tab_done[view * kSyncStride] : nullptr, 2u);
        stage_store(reinterpret_cast<float2*>(lds), twa, ntw, tid);
        switch (sg.L) {
          case 2048: persist_row<2048>(sg, local, lds, tid, tail); break;
          case 1792: persist_row<1792>(sg, local, lds, tid, tail); break;
          case 1536: persist_row<1536>(sg, local, lds, tid, tail); break;
          case 1280: persist_row<1280>(sg, local, lds, tid, tail); break;
          default: persist_row<1024>(sg, local, lds, tid, tail); break;
        }
        __syncthreads();
        break;
      }
    }
    // (A ticket taken early in an item would hold its item back behind this
    // one while other workgroups idle.)
    if (threadIdx.x == 0) s_ticket = took ? (int)next : (int)sync_add(&sync[kSyncTicket * kSyncStride], 1u);
  }
  // Leaving: the last workgroup out resets the counters for the next launch
  // (every item is done once every workgroup has taken a ticket past the end).
  __shared__ int s_last;
  if (threadIdx.x == 0) s_last = sync_add(&sync[kSyncExit * kSyncStride], 1u) == gridDim.x - 1;
  __syncthreads();
  if (s_last) {
    const int n = persist_sync_counters(nview, A.nstrips);
    for (int i = threadIdx.x; i < n; i += kPersistThreads)
      if (i != kSyncErr) __hip_atomic_store(&sync[i * kSyncStride], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void zero_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_persist(const PersistArgs* pa, int grid, bool complex_in, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (complex_in) hipLaunchKernelGGL(persist_kernel<true>, dim3(grid), dim3(kPersistThreads), 0, s, pa);
  else hipLaunchKernelGGL(persist_kernel<false>, dim3(grid), dim3(kPersistThreads), 0, s, pa);
  return hipGetLastError();
}

hipError_t launch_zero(uint32_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

int persist_resident_blocks() {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int per_cu2 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<false>, kPersistThreads, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, persist_kernel<true>, kPersistThreads, 0) != hipSuccess)
    return 0;
  per_cu = per_cu < per_cu2 ? per_cu : per_cu2;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

}  // namespace sfd

// Internal descriptors shared by the host planner and the HIP kernels.
//
// One view of the Shifted-Fresnel map (Section 2.1, Eqs. 1-4) separates into
// a y transform applied to every hologram column and an x transform applied
// to every row of the result, because every factor of Eqs. (2)-(4) is an
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

#include "sfd.h"

namespace sfd {

// Table-building job for one axis of one view (Eqs. 2-4).
struct AxisJob {
  double a0, a1;   // x0[m] = m p0 + a0, x1[m] = m p1 + a1 (metres)
  double p0, p1;   // pitches (metres)
  double inv_lz;   // 1 / (lambda z)
  double S;        // p0 p1 / (lambda z)
  double c1;       // a1 / p1: output-grid offset in output pixels
  double wscale;   // moment weight scale (pre *= x0 * wscale when kMomentX0)
  float2 post_scale;  // complex factor folded into post (the prefactor c on one axis)
  float2* pre;     // [n0]
  float2* post;    // [n1] or nullptr
  float2* H;       // [L]: h on input, FFT(h)/L after the spectrum kernel
  int32_t n0, n1, L;
  int32_t flags;   // kPhaseFp32, kMomentX0
};

enum : int32_t { kPhaseFp32 = 1, kMomentX0 = 2 };

// One batched set of 1D transforms (one view, one axis).
// Row kernel: transform r reads in + r * in_ld (n_in elements) and writes
// out + r * out_ld (n_out elements).  Column kernel: transform c reads
// in[n * in_ld + c] and writes out[m * out_ld + c].  n_rows counts the
// transforms in both cases.
struct RowJob {
  const void* in;      // float32 (kInReal) or complex64
  void* out;           // complex64, or float32 when only the intensity is written
  float* out2;         // float32 intensity when both outputs are written, else nullptr
  const float2* pre;   // [n_in], or nullptr when the input already carries it
  const float2* H;     // [L]
  const float2* post;  // [n_out] or nullptr
  // Column pass only, or nullptr: output column c is multiplied by colscale[c]
  // (the next pass's pre-chirp, which is constant along a column).
  const float2* colscale;
  float iscale;        // intensity scale
  int32_t n_rows, n_in, n_out;
  int64_t in_ld, out_ld;
  int32_t mode;        // kInReal | kOutIntensity | kOutField | kUsePost | kReduce ...
  int32_t view;        // the view the job belongs to (persistent launches)
  int32_t copy;        // column pass: the hologram copy it reads (persistent launches)
  // Column pass of a persistent launch over real holograms: 0 when ``in`` is
  // the column-major copy; otherwise ``in`` is the hologram itself, row-major
  // with in_ld samples per row, and in_fmt gives their format (32: float32
  // at the grid's width; 8, 16: camera samples, 33: float32 camera samples,
  // resized from in_ld samples per row as in TileJob).
  int32_t in_fmt;
  // Column pass: the batch's axis jobs (PassArgs::axis) of the view's y axis
  // (its pre-chirp) and x axis (colscale), for kernels that evaluate those
  // chirps themselves instead of reading the tables (persistent launches).
  int32_t ax_pre, ax_scale;
  int32_t pad_;

  // Epilogue reductions (row kernel, kReduce): over the row's outputs V(m),
  //   acc_k += conj(G) * w_k * V,  w_k = wc[k][0] X + wc[k][1] Y + wc[k][2] (X^2 + Y^2) + wc[k][3],
  // X = m xp + xa, Y = row yp + ya (coordinates of the output grid), with
  // G = gref[row][m] or, when giref is set, G = 2 giref[row][m] uref[row][m].
  // kRedSwap instead takes G = V and V = uref[row][m].  Each tile writes its
  // two complex FP64 sums to partial[tile * 4 .. + 4].
  const float2* gref;
  const float* giref;
  const float2* uref;
  double* partial;
  int64_t red_ld;
  double xp, xa, yp, ya;
  double wc[2][4];
};

enum : int32_t {
  kInReal = 1,
  kOutIntensity = 2,
  kUsePost = 4,
  kOutField = 16,
  kReduce = 32,
  kRedSwap = 64,
  kRedRealRef = 256,  // kRedSwap with a real reference: uref points to float32 values
};

constexpr int kMaxJobsPerLaunch = 256;

struct PassArgs {
  const RowJob* jobs;
  const AxisJob* axis;  // the batch's axis jobs (see RowJob::ax_pre), or nullptr
  int32_t njobs;
  int32_t total_tiles;
  int32_t tile_prefix[kMaxJobsPerLaunch + 1];
};

struct TwiddleJob {
  float2* tw;     // stage-major twiddle table of one transform shape (see fft_core.h)
  int32_t L;
  int32_t count;  // entries
  int32_t spec;   // 0: the passes' shape of L, 1: the kernel-spectrum shape of L
  int32_t pad_;
};

// A grid rewritten column-major for the column pass: out[c * ld + n] =
// in[n * nx + c] (n < ny, c < nx), so that each column is contiguous and the
// column pass loads it like a row.
struct TileJob {
  const void* in;   // [ny][nx] float32 or complex64 ([ny][nx_src] camera samples when nx_src > 0)
  const float* in2; // complex input only: if set, the copy holds 2 in2 * in (a gradient
                    // with respect to the field formed from dL/dI and the field)
  void* out;
  int32_t nx, ny;
  int32_t ld;       // elements between consecutive columns of the copy (>= ny)
  int32_t complex_in;
  // Real input only: > 0 when the input rows hold nx_src camera samples of
  // src_bits bits each (32: float32; 8, 16: unsigned integers, taken at their
  // value), resized to nx along x as they are copied (bilinear, half-pixel
  // centres: sample c is read at s = (c + 1/2) nx_src / nx - 1/2, clamped to
  // the row; the identity when nx_src == nx).
  int32_t nx_src;
  int32_t src_bits;
};
constexpr int kTrBlock = 64;  // square block one setup workgroup transposes (16 loads in flight per thread)

// z-derivative of one view from the reduction partials (see sfd_backward):
//   dL/dz = Re[(i k - 1/z) S1 - (i pi / (lambda z^2)) (S2 - 2 S3 - 2 S4 + S5)]
// with S1, S2 from the first accumulators of p12 (acc 0 and 1), S3, S4, S5
// from acc 0 of p3, p4, p5.
struct GradZJob {
  const double* p12;
  const double* p3;
  const double* p4;
  const double* p5;
  int32_t n12, n3, n4, n5;  // tiles
  double k, z, lam;
  double* out;
};

// The first two z-derivative sums of a view straight from its forward field
// u and dL/dI (gi), when the caller passes the field: with G = 2 gi u,
// conj(G) u = 2 gi |u|^2 summed with weight 1 (S1) and X^2 + Y^2 (S2) over
// the view grid (X = m xp + xa, Y = row yp + ya).  Block b of nblocks takes
// rows [b ny / nblocks, (b + 1) ny / nblocks) and writes its two sums to
// partial[b * 4 .. + 4] in the layout of the row kernel's tile partials.
struct SumJob {
  const float* gi;
  const float2* u;
  double* partial;
  int32_t nx, ny, ld, nblocks;
  double xp, xa, yp, ya;
};

// Sum of per-view adjoint results into a hologram's gradient (its real part
// only when real_out: dst is then float32).
struct GatherJob {
  const float2* const* src;  // device array of nsrc pointers
  float2* dst;
  int32_t nsrc;
  int32_t n;
  int32_t real_out;
  int32_t pad_;
};

// One launch builds everything a batch needs before the passes.  Workgroups
// take roles by index range: kernel spectra (FFT(h)/L, h evaluated in
// registers), pre/post chirp tables, FFT twiddle tables, hologram column
// tiles.  The roles are independent of each other.
enum : int32_t { kRoleSpectrum = 0, kRoleTables = 1, kRoleTwiddles = 2, kRoleTiles = 3 };
constexpr int kMaxSetupRoles = 64;  // SetupArgs stays well inside the 4 KiB kernel-argument space
struct SetupRole {
  int32_t kind;
  int32_t first_block, nblocks;
  int32_t a, b, c;  // spectrum: L, first axis job, count; tables: chunks per job, first job, count;
                    // twiddles: job; tiles: job, column blocks
  const float2* tw;  // spectrum: twiddle table of the spectrum shape of L
};
struct SetupArgs {
  const AxisJob* axis;
  const TwiddleJob* tw;
  const TileJob* tiles;
  int32_t nroles;
  int32_t total_blocks;
  int32_t max_l;  // longest spectrum of the launch (0 if none)
  SetupRole roles[kMaxSetupRoles];
};
static_assert(sizeof(SetupArgs) <= 4096, "setup arguments are passed by value as kernel arguments");
constexpr int kSetupThreads = 256;

// Persistent launch: every stage of a batch in one launch.  Workgroups take
// items from a ticket counter in the order of the segments below (each item
// depends only on items with smaller tickets, so the launch cannot deadlock
// whatever number of its workgroups are resident):
//   kItemSetup  three per view: its kernel spectrum Hy, its kernel
//               spectrum Hx, and its pre/post chirp tables;
//   kItemStrip  kStripW columns of a hologram rewritten column-major (the
//               copy the column pass reads, see TileJob);
//   kItemCol    a column-pass tile; waits for its view's Hy and the strip
//               holding its columns;
//   kItemRow    a row-pass tile; waits for every column tile of its view,
//               its Hx and its chirp tables.
// Completion counters live in the workspace (PersistSync).  The last
// workgroup to leave resets them to zero, so every launch, and every replay
// of a graph holding it, starts from zero without a memset.
enum : int32_t { kItemSetup = 0, kItemStrip = 1, kItemCol = 2, kItemRow = 3 };
constexpr int kMaxSegments = 16;
constexpr int kStripW = 16;           // columns per strip item: one column tile of the persistent shapes
constexpr int kPersistThreads = 512;  // workgroup size of the persistent launch
struct Segment {
  int32_t kind;
  int32_t first;         // first ticket of the segment
  int32_t count;         // items
  int32_t L;             // col/row: transform length
  int32_t var;           // col/row: kernel specialisation (as launch_pass)
  int32_t pad_;
  const PassArgs* args;  // col/row: the pass arguments of the segment's jobs
  const float2* tw;      // col/row: twiddle table of the passes' shape of L
};
struct PersistArgs {
  Segment seg[kMaxSegments];
  int32_t nseg;
  int32_t total;          // items over all segments
  int32_t grid;           // workgroups of the launch
  int32_t nview;
  int32_t wait_setup;     // tiles wait for their view's setup items (0 when tables are kept)
  int32_t ncopy;
  int32_t nstrips;        // strip items (all copies)
  int32_t pad_;
  const AxisJob* axis;    // 2 per view: x, then y
  const TileJob* tiles;   // per hologram copy
  const int32_t* col_tiles;    // per view: column tiles (the row tiles' target)
  const float2* const* tw_view;  // per view: twiddle tables of the kernel-spectrum shape of Lx, Ly
  uint32_t* sync;         // counters, see persist_sync_words
};
// Counter layout, one counter per kSyncStride words (its own 256-byte line:
// a counter that workgroups poll shares no line with one they advance):
// [0] ticket, [1] workgroups that left, [2] error word (set when a
// dependency wait gave up; never reset by the kernel), then per view its
// Hy counter (target 1), its Hx and chirp-table counter (target 2) and its
// column-tile counter, then one counter per strip item.
constexpr int kSyncStride = 64;
constexpr int kSyncTicket = 0, kSyncExit = 1, kSyncErr = 2, kSyncHead = 3;
__host__ __device__ inline int persist_sync_counters(int nview, int nstrips) { return kSyncHead + 3 * nview + nstrips; }
__host__ __device__ inline int persist_sync_words(int nview, int nstrips) {
  return kSyncStride * persist_sync_counters(nview, nstrips);
}

// Host-side launchers (defined in sfd_kernels.hip).
hipError_t launch_setup(const SetupArgs& args, hipStream_t s);
// Axis jobs one spectrum workgroup handles at a transform length.
int spectra_per_block(int L);

// col = true: the y transforms (column kernel); false: the x transforms.
// G is the tile width (transforms per workgroup): one of
// pass_tile_widths(L, col).  var selects a specialised kernel; with
// F = fast_input(L):  row pass: 1 when every job has n_in == F, n_out <= F,
// a complex input and no kReduce; 2 when, in addition, no job applies a
// post-chirp and every job writes intensities only.  Column pass: 1 when
// every job has n_in == F, n_out <= F and a complex input; 2 when every job
// has n_in == F, n_out <= F, a real input and no post-chirp; 3 as 2 with
// post-chirps allowed.  0 otherwise.
hipError_t launch_pass(int L, bool col, int G, int var, const PassArgs& args, const float2* tw, hipStream_t s);

// Persistent launch (see PersistArgs): pa is a device copy; grid workgroups;
// complex_in selects the instance for complex holograms.
hipError_t launch_persist(const PersistArgs* pa, int grid, bool complex_in, hipStream_t s);
// Zero n counters (the first launch on a workspace).
hipError_t launch_zero(uint32_t* p, int n, hipStream_t s);
// Lengths the persistent launch supports (the passes' shape of a row in one
// wavefront, with two transforms per slot).
bool persist_length(int L);
// Workgroups of the persistent launch resident at once on this device.
int persist_resident_blocks();

// Copy ``bytes`` (a multiple of 4) from host memory to device memory on
// stream s through kernel arguments (no staging buffer, no allocation).
hipError_t launch_blit(void* dst, const void* src, size_t bytes, hipStream_t s);

hipError_t launch_gradz(const GradZJob* d_jobs, int njobs, hipStream_t s);
hipError_t launch_sums(const SumJob* d_jobs, int njobs, int max_blocks, hipStream_t s);
hipError_t launch_gather(const GatherJob* d_jobs, int njobs, int max_n, hipStream_t s);

// Tile widths (transforms per workgroup) a pass supports at length L, the
// default first; returns how many there are (writes at most cap of them,
// and, when per_slot is set, the transforms each slot runs in turn).
int pass_tile_widths(int L, bool col, int* widths, int cap, int* per_slot = nullptr);
// The default tile width of a pass at length L (0 if L is unsupported).
int rows_per_tile(int L, bool col);
bool supported_length(int L);
// Input length of the specialised pass kernels at length L: L / 2 at powers
// of two, 1024 at the smooth lengths 1280, 1536 and 1792 (see FastIn).
int fast_input(int L);
// Entries of the twiddle table of the passes' (spec = false) or the kernel
// spectrum's (spec = true) transform shape of length L.
int twiddle_len(int L, bool spec);

// The reconstruction behind sfd_reconstruct (no_alloc = false) and
// sfd_reconstruct_noalloc (no_alloc = true: the workspace is the library's
// static scratch array; descriptors go up through kernel arguments, kernels
// are launched directly, and the plan's cached workspace state is rebuilt
// whenever another plan used the scratch last).
sfd_status reconstruct_impl(sfd_plan_s* plan, const void* holo, const double* z_or_null, void* const* out,
                            void* workspace, size_t ws_bytes, hipStream_t stream, bool no_alloc);
// Set the calling thread's error message (see sfd_last_error) and return s.
sfd_status set_error(sfd_status s, const char* msg);

}  // namespace sfd

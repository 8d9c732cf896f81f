/*
 * sfd.h - batched Shifted-Fresnel reconstruction on AMD Instinct MI355X (gfx950).
 *
 * The operation (Shimobaba, Masuda, Ichihashi, Ito, "Real-time digital
 * holographic microscopy observable in multi-view and multi-resolution",
 * Section 2.1, Eqs. 1-5): a hologram u0 sampled at pitch (px0, py0) on a
 * grid shifted by (Ox0, Oy0) is propagated over a signed distance z onto a
 * reconstruction grid with its own size, pitch (px1, py1) and shift
 * (Ox1, Oy1), and the intensity I = |u1|^2 is returned (Eq. 5).  A view is one
 * such (grid, z) pair; many views of one or more holograms are computed in one
 * call (the multi-view scheme of Section 2.2, steps 2-10, for every view).
 *
 * Discrete definition implemented (Eqs. 1-4 are its chirp factorisation):
 *
 *   u1[n1][m1] = c(z) * sum_{n0,m0} u0[n0][m0]
 *                 * exp(i pi ((x1[m1]-x0[m0])^2 + (y1[n1]-y0[n0])^2) / (lambda z))
 *   c(z)       = exp(i k z) * px0 * py0 / (i lambda z),   k = 2 pi / lambda
 *   x[m]       = (m - floor(nx/2)) * px + ox,   y[n] = (n - floor(ny/2)) * py + oy
 *
 * i.e. centred grids with shifts in metres, the hologram's area element in
 * c(z), and any zero padding L >= N0 + N1 - 1 per axis (the paper doubles the
 * grid).  The intensity keeps |c|^2 = (px0 py0 / (lambda z))^2.
 *
 * Memory: every array argument marked "device" is device memory owned by the
 * caller.  Images are row-major [ny][nx] (y = rows, x = columns); complex
 * values are interleaved (re, im) float32 pairs ("complex64").  The library
 * never allocates device memory and never synchronises the device; it
 * enqueues work on the caller's stream.
 *
 * Errors: every call returns an sfd_status.  Arguments are validated on the
 * host before any HIP call; on error nothing is enqueued and
 * sfd_last_error() (thread-local) describes the failure.  NaN or Inf inside
 * the data propagates, as in BLAS.
 */
#ifndef SFD_H
#define SFD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SFD_OK = 0,
  SFD_ERR_INVALID_ARG = 1, /* bad value, null or misaligned pointer */
  SFD_ERR_UNSUPPORTED = 2, /* valid request this library does not implement (e.g. L too large) */
  SFD_ERR_WORKSPACE = 3,   /* workspace smaller than sfd_workspace_size() */
  SFD_ERR_HIP = 4,         /* a HIP runtime call failed; message names it */
  SFD_ERR_INTERNAL = 5
} sfd_status;

/* A sampled plane (Section 2.1 symbol list).  nx, ny >= 1 samples along x
 * (columns) and y (rows); pitches px, py > 0 in metres; shifts ox, oy in
 * metres.  Sample m sits at x = (m - floor(nx/2)) * px + ox. */
typedef struct {
  int32_t nx, ny;
  double px, py;
  double ox, oy;
} sfd_grid;

/* One reconstruction view: its grid, the signed distance z != 0 from the
 * hologram plane (metres; z < 0 back-propagates), and the index of the
 * hologram it reads (0 <= holo < n_holo). */
typedef struct {
  sfd_grid out;
  double z;
  int32_t holo;
} sfd_view;

typedef struct sfd_plan_s* sfd_plan_t;

/* Plan flags.  Exactly one input kind and at least one output kind must be
 * set; with both output kinds, each call writes the intensities and the
 * fields. */
enum {
  SFD_IN_REAL_F32 = 1u << 0,   /* holograms are float32 [n_holo][ny][nx] */
  SFD_IN_C64 = 1u << 1,        /* holograms are complex64 fields [n_holo][ny][nx] */
  SFD_OUT_INTENSITY = 1u << 2, /* outputs are float32 I = |u1|^2 (Eq. 5) */
  SFD_OUT_FIELD = 1u << 3,     /* outputs are the complex64 field u1 (Eq. 1 with C1) */
  SFD_PHASE_FP32 = 1u << 4,    /* evaluate chirp phases in FP32 instead of FP64 (comparison only) */
  SFD_PER_VIEW_LAUNCH = 1u << 5, /* launch the kernels one view at a time (baseline for batching) */
  SFD_EAGER = 1u << 6,           /* batched calls launch their kernels directly instead of replaying
                                    the plan's HIP graph */
  SFD_REUSE_TABLES = 1u << 7,    /* streaming (the repeated steps 1-11 of Section 2.2): the chirp
                                    tables and kernel spectra of a call are kept for the next call on
                                    the same workspace when its distances are the same, so that call
                                    runs only the hologram copy and the two passes */
  SFD_WITH_BACKWARD = 1u << 8    /* real-hologram plans: lay out the workspace for sfd_backward too
                                    (complex-input plans always have it) */
};

/*
 * Create a plan for n_views views of n_holo holograms that share one grid.
 * Host only: no HIP call is made.  Chooses the padded FFT length per view and
 * axis (smallest supported L >= N0 + N1 - 1), lays out the workspace, and
 * precomputes the FP64 per-view scalars of Eqs. (2)-(4).
 *   plan       [out] receives the plan handle (set to NULL on error)
 *   wavelength lambda in metres, finite and > 0
 *   holo_grid  grid shared by all holograms (shifts allowed)
 *   n_holo     >= 1
 *   views      host array of n_views >= 1 views (copied; the caller keeps ownership)
 *   flags      SFD_IN_* | SFD_OUT_* | optional SFD_PHASE_FP32, SFD_PER_VIEW_LAUNCH,
 *              SFD_EAGER
 * Errors: SFD_ERR_INVALID_ARG for non-finite or non-positive lambda or
 * pitches, z == 0 or non-finite, sizes < 1, holo index out of range, missing
 * or conflicting flags; SFD_ERR_UNSUPPORTED when a padded length would exceed
 * 8192, i.e. N0 + N1 - 1 > 8192 on an axis.  The cap is deliberate: a row of
 * 8192 complex values is the longest transform one workgroup holds in
 * registers and LDS (256 threads x 32 values, a 66 KiB exchange row), which
 * covers the paper's grids (L = 2048) and 4096^2 holograms; L = 16384 would
 * need a transform split over workgroups (a four-step FFT through HBM) and is
 * not built.
 */
sfd_status sfd_plan(sfd_plan_t* plan, double wavelength, const sfd_grid* holo_grid,
                    int32_t n_holo, const sfd_view* views, int32_t n_views, uint32_t flags);

/* Bytes of device workspace the plan needs for sfd_reconstruct and
 * sfd_backward.  The workspace must stay dedicated to this plan while the plan
 * lives (device-side descriptors are cached in it between calls). */
sfd_status sfd_workspace_size(sfd_plan_t plan, size_t* bytes);

/* Padded transform lengths chosen for view v: lx, ly (host query, for tests
 * and benchmarks). */
sfd_status sfd_view_lengths(sfd_plan_t plan, int32_t v, int32_t* lx, int32_t* ly);

/*
 * Reconstruct every view (Section 2.2, steps 2-10).
 *   holo        device, n_holo x [ny][nx] float32 or complex64 (per the plan
 *               flags), 16-byte aligned
 *   z_or_null   host array of n_views distances overriding the plan's z (each
 *               finite, != 0), or NULL to keep them
 *   out         host array of n_views device pointers, each [ny][nx] of the
 *               view's grid, float32 (intensity) or complex64 (field),
 *               16-byte aligned; with both output flags it holds 2 n_views
 *               pointers, the intensities first and then the fields.
 *               Outputs must not overlap each other, the holograms or the
 *               workspace.
 *   workspace   device, >= sfd_workspace_size bytes, 256-byte aligned
 *   ws_bytes    size of workspace in bytes
 *   stream      HIP stream the work is enqueued on (0 = null stream)
 * The persistent schedule (see sfd_set_launch) is one kernel launched
 * directly.  The pass schedule of batched plans (no SFD_PER_VIEW_LAUNCH, no
 * SFD_EAGER) records its kernel sequence once per workspace into a HIP graph
 * owned by the plan and replays it on every later call; the kernels read the call's pointers and distances
 * from descriptors that each call copies into the workspace first (on
 * ``stream``, only when they changed), so one graph serves every call.  When
 * ``stream`` is being captured by the caller, or kernel timing is on, the
 * kernels are launched directly instead; a caller's captured graph then reads
 * the descriptors from the workspace when it is replayed, so make one
 * uncaptured call with the same arguments first (which writes them), and no
 * call with other pointers or distances on that workspace between replays.
 * With SFD_REUSE_TABLES, a call whose distances equal those of the previous
 * call on the same workspace reuses that call's tables and spectra (the
 * workspace keeps them); sfd_backward on the workspace invalidates them.
 */
sfd_status sfd_reconstruct(sfd_plan_t plan, const void* holo, const double* z_or_null,
                           void* const* out, void* workspace, size_t ws_bytes,
                           hipStream_t stream);

/*
 * Gradients of a real loss through reconstruct: the adjoint (conjugate chirps
 * and the transposed scaled convolution, A(z)^H = (px0 py0)/(px1 py1) A(-z)
 * with the two planes swapped) and the derivative with respect to each
 * view's z.  Requires a plan made with SFD_IN_C64, or with SFD_IN_REAL_F32
 * and SFD_WITH_BACKWARD (not with sfd_set_raw_input frames).
 *   grad_out    host array of n_views device pointers.  If field_out is NULL
 *               each is complex64 [ny][nx]: g = dL/dRe(u1) + i dL/dIm(u1).
 *               Otherwise each is float32 dL/dI and g = 2 (dL/dI) u1 is formed
 *               on the device.
 *   field_out   NULL, or host array of n_views device pointers to the complex64
 *               fields u1 of the forward call (SFD_OUT_FIELD plan or saved) at
 *               the same distances; the first two sums of dL/dz are then taken
 *               from them directly (no forward pass is recomputed), so they
 *               must be that call's fields
 *   holo        device, the forward's inputs (complex64, or float32 for a real
 *               plan; needed for dL/dz)
 *   z_or_null   as in sfd_reconstruct
 *   grad_in     device, n_holo x [ny][nx]: sum over the views of each hologram
 *               of A^H g, complex64 (PyTorch's convention for complex inputs);
 *               for a real plan float32, its real part (the gradient with
 *               respect to a real input)
 *   grad_z      device, n_views doubles receiving dL/dz, or NULL to skip the
 *               z-derivative work
 */
sfd_status sfd_backward(sfd_plan_t plan, void* const* grad_out, void* const* field_out,
                        const void* holo, const double* z_or_null, void* grad_in,
                        double* grad_z, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Schedule autotuner.  Times every tile width (transforms per workgroup) the
 * column (y) and row (x) passes support at each of the plan's transform
 * lengths, one pass and length at a time with the others fixed (two sweeps),
 * by running the plan's whole forward ``reps`` times per candidate on the
 * caller's data, launched as the plan's calls are (graph replays for batched
 * plans); keeps the fastest in the plan and in a process-wide table
 * that later plans with the same hologram grid, view sizes and flags start
 * from.  Arguments as in sfd_reconstruct; outputs are overwritten.
 * Synchronises ``stream``.  The workspace layout does not change, so the same
 * workspace stays valid.  When the environment variable SFD_TUNE_CACHE names
 * a file, the result is also written there (JSON, keyed by the target
 * architecture, the schedule version, the hologram grid and count, the flags
 * and the view sizes: the things the padded lengths follow from), and
 * sfd_plan starts new plans of the same key from it in later processes; a
 * file that does not parse is ignored (and replaced by the next autotune).
 *   reps   timed forwards per candidate, 1..1000
 */
sfd_status sfd_autotune(sfd_plan_t plan, const void* holo, void* const* out, void* workspace,
                        size_t ws_bytes, int32_t reps, hipStream_t stream);

/* Tile width the plan uses for the column (col != 0) or row (col == 0) pass
 * at transform length L (host query). */
sfd_status sfd_schedule(sfd_plan_t plan, int32_t L, int32_t col, int32_t* tile_width);

/* Set that tile width by hand (host only).  Errors: SFD_ERR_INVALID_ARG if
 * the plan has no transforms of length L or the pass has no kernel of that
 * tile width at L.  Results do not depend on the tile width: every transform
 * is computed the same way whatever workgroup holds it. */
sfd_status sfd_set_schedule(sfd_plan_t plan, int32_t L, int32_t col, int32_t tile_width);

/*
 * One frame of the real-time loop (Section 2.2: steps 1-11 repeated for every
 * captured hologram).  Copies the frame from host memory into the next of
 * two device buffers on the plan's own copy stream, then enqueues
 * sfd_reconstruct of that buffer (with the plan's distances) on ``stream``,
 * after the copy.  The call returns at once: the copy of frame k + 1 runs
 * while frame k is reconstructed.  A frame's copy waits for the
 * reconstruction that last read its buffer (frame k - 2), and so does the
 * call itself (on the host): at most two frames are in flight.
 *   host_frame  host, n_holo x [ny][nx] float32 or complex64 per the plan
 *               flags; pinned (hipHostMalloc) for the copy to overlap, and
 *               left unchanged until the copy is done
 *   dev_holo    host array of two distinct device buffers of that size,
 *               16-byte aligned, the same two on every call of the plan
 *   out, workspace, ws_bytes, stream: as in sfd_reconstruct.  The outputs of
 *               frame k may be overwritten by a later frame given the same
 *               pointers: read them (in stream order) before that.
 * With SFD_REUSE_TABLES the tables and spectra are computed for the first
 * frame only.  Errors: SFD_ERR_INVALID_ARG for NULL or equal buffers or a
 * per-view plan; the sfd_reconstruct errors.
 */
sfd_status sfd_stream_frame(sfd_plan_t plan, const void* host_frame, void* const* dev_holo, void* const* out,
                            void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Raw camera frames (the paper resizes its 1360 x 1024 CCD frames to the
 * hologram grid before reconstructing, Section 3).  After this call the
 * plan's holograms arrive as n_holo x [ny][nx_raw] camera samples of
 * sample_bits bits: 32 for float32, 8 or 16 for unsigned integers (taken at
 * their value).  They are converted and resized along x to the plan's
 * hologram grid (nx samples of pitch px) as they are copied for the column
 * pass: bilinear interpolation with half-pixel centres, sample c read at
 * s = (c + 1/2) nx_raw / nx - 1/2, clamped to [0, nx_raw - 1] (the identity
 * when nx_raw == nx).  nx_raw = 0 turns it off.  The pitch of the plan's
 * grid stays the caller's (nx_raw / nx times the camera's).  Real-input plans
 * only; affects sfd_reconstruct, sfd_autotune and sfd_stream_frame (whose
 * copies then move the camera samples).  Errors: SFD_ERR_INVALID_ARG
 * (complex plan, nx_raw outside [0, 65536], sample_bits not 8, 16 or 32),
 * SFD_ERR_UNSUPPORTED (frame above 2^28 samples).
 */
sfd_status sfd_set_raw_input(sfd_plan_t plan, int32_t nx_raw, int32_t sample_bits);

/* Tile widths (transforms per workgroup) the column (col != 0) or row
 * (col == 0) pass has kernels for at transform length L, the default first
 * (host query, no plan needed).  Writes up to cap widths to ``widths`` and,
 * when ``per_slot`` is not NULL, for each the number of transforms that one
 * slot of TPR threads of that workgroup runs in turn (1, or more when the
 * kernel fetches the next transform's input while it computes the current
 * one).  Returns how many widths there are (0 when L is not a supported
 * length), or -1 if cap < 0 or cap > 0 with widths NULL. */
int32_t sfd_tile_widths(int32_t L, int32_t col, int32_t* widths, int32_t* per_slot, int32_t cap);

/*
 * sfd_reconstruct without a caller workspace and without any allocation,
 * for callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * static device array of the library, sfd_noalloc_capacity() bytes (64 MiB:
 * enough for a 1024^2 hologram with four 1024^2 views at padded length 2048),
 * held on every GPU the library runs on until the process ends.  The call
 * allocates nothing: descriptors reach the device through kernel
 * arguments, the kernels are launched directly on ``stream`` (no graph is
 * recorded), and no host staging buffer is used.
 *   plan, holo, z_or_null, out, stream: as in sfd_reconstruct.
 * Every call on a GPU shares that GPU's array, and the array keeps the last
 * call's contents: a call of another plan than the previous one rebuilds the
 * plan's tables and zeroes its counters first.  Calls that overlap in time on
 * one GPU (several streams or threads) race on the array and must not be
 * made.  Errors: SFD_ERR_WORKSPACE when sfd_workspace_size of the plan
 * exceeds the array (checked before any HIP call), and the sfd_reconstruct
 * errors.
 */
sfd_status sfd_reconstruct_noalloc(sfd_plan_t plan, const void* holo, const double* z_or_null,
                                   void* const* out, hipStream_t stream);
size_t sfd_noalloc_capacity(void);

/* Kernel kinds reported by sfd_profile_report. */
enum {
  SFD_KERNEL_TABLES = 0,   /* chirp and twiddle tables (Eqs. 2-4) */
  SFD_KERNEL_SPECTRA = 1,  /* FFT of the chirp kernel h per axis (steps 5-6) */
  SFD_KERNEL_PASS_X = 2,   /* fused x transforms of the rows, crop, post-chirp or |.|^2 (steps 2-4, 7-10) */
  SFD_KERNEL_PASS_Y = 3,   /* fused y transforms of the hologram columns (steps 2-4, 7-9) */
  SFD_KERNEL_OTHER = 4,    /* backward-only reductions and gathers */
  SFD_KERNEL_PERSIST = 5,  /* the persistent launch: every step of a batched forward in one kernel */
  SFD_KERNEL_KINDS = 6
};

/*
 * Launch schedule of a batched forward (Section 2.2, steps 2-10 for every
 * view of every hologram).
 *   SFD_LAUNCH_PASSES      three launches per call: setup (tables, spectra,
 *                          hologram copies), every column pass, every row
 *                          pass, with the tile widths of sfd_set_schedule.
 *   SFD_LAUNCH_PERSISTENT  one launch per call.  Its workgroups take work
 *                          items in a fixed order from a ticket counter: per
 *                          view three setup items (its y kernel spectrum, its
 *                          x kernel spectrum, its chirp tables), the
 *                          hologram copies in strips of 16 columns, the
 *                          column tiles, the row tiles.  An item waits on
 *                          completion counters for the items it reads (a
 *                          column tile for its view's y spectrum and its
 *                          strip, a row tile for every column tile of its
 *                          view, its x spectrum and its tables), and
 *                          those always hold smaller tickets, so the launch
 *                          completes however many of its workgroups are
 *                          resident.  The counters live in the workspace; the
 *                          first call on a workspace zeroes them and the last
 *                          workgroup of every launch resets them, so graph
 *                          replays need no memset.  Two calls on one
 *                          workspace must not run concurrently (they would
 *                          share the counters, as they share the tables).
 *                          Available for batched plans where every view's
 *                          padded lengths are 1024, 1280, 1536, 1792 or 2048
 *                          with the hologram filling half of each at 1024
 *                          and 2048 (the paper's doubled grid), 1024 samples
 *                          at the smooth lengths, and the view no larger.
 * Plans start persistent where it is available; sfd_autotune keeps the
 * faster of the two.  Errors: SFD_ERR_INVALID_ARG (unknown mode),
 * SFD_ERR_UNSUPPORTED (persistent mode not available for the plan).
 */
enum { SFD_LAUNCH_PASSES = 0, SFD_LAUNCH_PERSISTENT = 1 };
sfd_status sfd_set_launch(sfd_plan_t plan, int32_t mode);
sfd_status sfd_launch_mode(sfd_plan_t plan, int32_t* mode, int32_t* persistent_available);

/*
 * Length policy (the radix choice of the schedule).  Any padded length
 * L >= N0 + N1 - 1 evaluates the same linear convolution (Section 2.2,
 * steps 2 and 9).  Each axis takes the smallest supported length that the
 * policy allows: powers of two always, and the smooth lengths named by the
 * mask smooth: SFD_SMOOTH_1280 = 2^8 5, SFD_SMOOTH_1536 = 2^9 3,
 * SFD_SMOOTH_1792 = 2^8 7 (transforms closing with a radix-20, -24 or -28
 * stage).  0 is the paper's doubled grid (powers of two only).  Default:
 * SFD_SMOOTH_1280 (the one smooth length measured faster than 2048 on
 * gfx950).  The workspace is sized for every policy, so the same workspace
 * stays valid.  sfd_autotune switches each smooth length that changes some
 * view's length on or off and keeps the faster setting.  Errors:
 * SFD_ERR_INVALID_ARG (bits other than the three).
 */
enum { SFD_SMOOTH_1280 = 1, SFD_SMOOTH_1536 = 2, SFD_SMOOTH_1792 = 4, SFD_SMOOTH_ALL = 7 };
sfd_status sfd_set_length_policy(sfd_plan_t plan, int32_t smooth);
sfd_status sfd_length_policy(sfd_plan_t plan, int32_t* smooth);

/*
 * Dependency faults of persistent launches on a workspace: a wait that gave
 * up after about two seconds (a counter that never reached its target, which
 * would otherwise hang the device) sets an error word in the workspace; the
 * call's results are then undefined.  Copies the word to *faults
 * (synchronises ``stream``) and clears it when ``clear`` is set.  Diagnostic
 * and test use.
 */
sfd_status sfd_sync_faults(sfd_plan_t plan, void* workspace, size_t ws_bytes, int32_t clear, uint32_t* faults,
                           hipStream_t stream);

/* Benchmark timing.  While enabled, each kernel the plan launches is
 * bracketed by two HIP events recorded on the launch stream.  Enabling (or
 * re-enabling) clears the record.  Host only apart from the event records. */
sfd_status sfd_profile_enable(sfd_plan_t plan, int32_t enable);

/* Launch count and summed event-measured duration (milliseconds) of one
 * kernel kind since profiling was enabled.  Waits for the recorded events. */
sfd_status sfd_profile_report(sfd_plan_t plan, int32_t kind, int64_t* launches, double* total_ms);

/* Release the plan's host resources.  Passing NULL is allowed. */
sfd_status sfd_destroy(sfd_plan_t plan);

/* Message describing the last error on the calling thread ("" if none). */
const char* sfd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SFD_H */

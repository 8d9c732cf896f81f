// C-ABI of the batched Shifted-Fresnel library: validation, planning,
// workspace layout and launch sequencing.  See include/sfd.h for the
// contract of every entry point.
#include "sfd.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "sfd_internal.h"

namespace {

thread_local std::string g_err;

sfd_status fail(sfd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define SFD_HIP_TRY(expr)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(SFD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

bool grid_ok(const sfd_grid& g, std::string* why, const char* what) {
  char buf[256];
  if (g.nx < 1 || g.ny < 1) {
    std::snprintf(buf, sizeof buf, "%s: sizes must be >= 1 (got %d x %d)", what, g.nx, g.ny);
    *why = buf;
    return false;
  }
  if (!finite_pos(g.px) || !finite_pos(g.py)) {
    std::snprintf(buf, sizeof buf, "%s: pitches must be finite and > 0", what);
    *why = buf;
    return false;
  }
  if (!std::isfinite(g.ox) || !std::isfinite(g.oy)) {
    std::snprintf(buf, sizeof buf, "%s: shifts must be finite", what);
    *why = buf;
    return false;
  }
  return true;
}

// Padded lengths the transforms support, ascending: powers of two and the
// smooth lengths 1280 = 2^8 5, 1536 = 2^9 3, 1792 = 2^8 7.
constexpr int kLengths[] = {64, 128, 256, 512, 1024, 1280, 1536, 1792, 2048, 4096, 8192};

// Length policy: a mask of the smooth lengths a plan may use (bit 0: 1280,
// bit 1: 1536, bit 2: 1792); 0 keeps to powers of two (the paper's
// doubling).  The default allows 1280 only: measured per view at the paper's
// 1024-sample holograms, 1280 (radices 4, 4, 4, 20) beats 2048 while 1536
// (8, 8, 24) only matches it and 1792 (4, 4, 4, 28) loses to it.
constexpr int kSmoothAll = 7, kSmoothDefault = 1;
bool smooth_allowed(int L, int mask) {
  return (L & (L - 1)) == 0 || (L == 1280 && (mask & 1)) || (L == 1536 && (mask & 2)) || (L == 1792 && (mask & 4));
}

// Smallest supported padded length for a linear convolution of n0 inputs
// onto n1 outputs (reading of steps 2 and 9: any L >= n0 + n1 - 1 is exact)
// among those the mask allows.
int choose_length(int n0, int n1, int mask = kSmoothDefault) {
  const long need = (long)n0 + (long)n1 - 1;
  for (int L : kLengths)
    if (L >= need && smooth_allowed(L, mask)) return L;
  return -1;
}

// Per-axis FP64 scalars of Eqs. (2)-(4) (see sfd_internal.h).
struct AxisScalars {
  double a0, a1, p0, p1, inv_lz, S, c1;
};

AxisScalars axis_scalars(int n0, double p0, double o0, int n1, double p1, double o1, double lam, double z) {
  AxisScalars a;
  a.p0 = p0;
  a.p1 = p1;
  a.a0 = -(double)(n0 / 2) * p0 + o0;
  a.a1 = -(double)(n1 / 2) * p1 + o1;
  a.inv_lz = 1.0 / (lam * z);
  a.S = p0 * p1 / (lam * z);
  a.c1 = a.a1 / p1;
  return a;
}

// c(z) = exp(i k z) px0 py0 / (i lambda z) = (px0 py0 / (lambda z)) exp(i pi (2 z / lambda - 1/2)),
// with the half-turn count reduced in FP64 before sin/cos.
void prefactor(double lam, double z, double px0, double py0, double* re, double* im) {
  const double turns = 2.0 * z / lam - 0.5;  // in units of pi
  const double r = turns - 2.0 * std::nearbyint(0.5 * turns);
  const double mag = px0 * py0 / (lam * z);
  *re = mag * std::cos(M_PI * r);
  *im = mag * std::sin(M_PI * r);
}

struct ViewLayout {
  int lx = 0, ly = 0;
  int tile = -1;  // index of the hologram's column-major copy the column pass reads
  size_t prex = 0, prey = 0, postx = 0, posty = 0, hx = 0, hy = 0, inter = 0;
};

// Column-major copy of a hologram for the column passes (see sfd::TileJob).
struct TileLayout {
  int holo;
  size_t off;
};

// Column stride (elements) of a column-major copy of a grid with ny rows:
// padded off a power of two so that the transposing writes spread over the
// memory channels.
int col_ld(int ny) { return (ny + 63) / 64 * 64 + 64; }

// Narrowest tile width of a pass at length L (the most tiles).
int min_tile_width(int L, bool col) {
  int w[16];
  const int n = std::min(sfd::pass_tile_widths(L, col, w, 16), 16);
  int m = 1 << 30;
  for (int i = 0; i < n; ++i) m = std::min(m, w[i]);
  return m;
}

// Row stride of the N1y x N0x intermediate: padded off a power of two so the
// column pass's strided writes spread over the cache channels.
int inter_ld(int n0x) { return (n0x + 15) / 16 * 16 + 16; }

}  // namespace

namespace {
// Tuned schedules, keyed by the plan's shapes: (col, L, shape signature) ->
// tile width; (2, 0, signature) -> persistent launch; (3, 0, signature) ->
// smooth lengths.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, std::string>, int> g_tuned;

// ---- Persisted schedule cache (environment variable SFD_TUNE_CACHE) ------
// A JSON file {"format": "sfd-schedule-cache", "entries": {KEY: {"col":
// {"L": width, ...}, "row": {...}, "persist": 0|1, "smooth": mask}, ...}}
// with KEY = "<arch>|v<schedule version>|<hologram grid, hologram count,
// flags, view sizes>".  sfd_autotune writes it, sfd_plan reads it; a file
// that does not parse (or another format) is ignored, and rewritten by the
// next autotune.
constexpr int kScheduleVersion = 2;
constexpr const char* kArch = "gfx950";

// Minimal JSON reader for that file: objects, strings without escapes,
// integers.  Returns false on anything else.
struct JVal {
  enum Kind { kObj, kStr, kInt } kind = kInt;
  long long i = 0;
  std::string s;
  std::map<std::string, JVal> o;
};
struct JReader {
  const std::string& t;
  size_t p = 0;
  void ws() {
    while (p < t.size() && (t[p] == ' ' || t[p] == '\n' || t[p] == '\t' || t[p] == '\r')) ++p;
  }
  bool str(std::string* out) {
    ws();
    if (p >= t.size() || t[p] != '"') return false;
    const size_t e = t.find('"', p + 1);
    if (e == std::string::npos) return false;
    *out = t.substr(p + 1, e - p - 1);
    if (out->find('\\') != std::string::npos) return false;
    p = e + 1;
    return true;
  }
  bool val(JVal* v, int depth) {
    ws();
    if (p >= t.size() || depth > 8) return false;
    if (t[p] == '{') {
      v->kind = JVal::kObj;
      ++p;
      ws();
      if (p < t.size() && t[p] == '}') return ++p, true;
      for (;;) {
        std::string k;
        if (!str(&k)) return false;
        ws();
        if (p >= t.size() || t[p] != ':') return false;
        ++p;
        if (!val(&v->o[k], depth + 1)) return false;
        ws();
        if (p < t.size() && t[p] == ',') { ++p; continue; }
        if (p < t.size() && t[p] == '}') return ++p, true;
        return false;
      }
    }
    if (t[p] == '"') {
      v->kind = JVal::kStr;
      return str(&v->s);
    }
    size_t e = p;
    if (e < t.size() && t[e] == '-') ++e;
    while (e < t.size() && t[e] >= '0' && t[e] <= '9') ++e;
    if (e == p) return false;
    v->kind = JVal::kInt;
    v->i = std::stoll(t.substr(p, e - p));
    p = e;
    return true;
  }
};

bool read_cache(const std::string& path, JVal* root) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  JReader r{text};
  if (!r.val(root, 0)) return false;
  r.ws();
  if (r.p != text.size() || root->kind != JVal::kObj) return false;
  const auto fm = root->o.find("format");
  if (fm == root->o.end() || fm->second.kind != JVal::kStr || fm->second.s != "sfd-schedule-cache") return false;
  const auto en = root->o.find("entries");
  return en != root->o.end() && en->second.kind == JVal::kObj;
}

std::string cache_key(const std::string& sig) {
  return std::string(kArch) + "|v" + std::to_string(kScheduleVersion) + "|" + sig;
}

// Entries of the cache file for ``sig`` into the in-process table (caller
// holds g_tune_mu).
void load_cached(const std::string& sig) {
  const char* path = std::getenv("SFD_TUNE_CACHE");
  if (!path || !*path) return;
  JVal root;
  if (!read_cache(path, &root)) return;
  const auto& entries = root.o["entries"].o;
  const auto it = entries.find(cache_key(sig));
  if (it == entries.end() || it->second.kind != JVal::kObj) return;
  const JVal& e = it->second;
  for (int col = 0; col < 2; ++col) {
    const auto pc = e.o.find(col ? "col" : "row");
    if (pc == e.o.end() || pc->second.kind != JVal::kObj) continue;
    for (const auto& kv : pc->second.o)
      if (kv.second.kind == JVal::kInt && kv.second.i > 0)
        g_tuned[std::make_tuple(col, std::atoi(kv.first.c_str()), sig)] = (int)kv.second.i;
  }
  for (const char* k : {"persist", "smooth"}) {
    const auto pk = e.o.find(k);
    if (pk != e.o.end() && pk->second.kind == JVal::kInt && pk->second.i >= 0 && pk->second.i <= kSmoothAll)
      g_tuned[std::make_tuple(k[0] == 'p' ? 2 : 3, 0, sig)] = k[0] == 'p' ? pk->second.i != 0 : (int)pk->second.i;
  }
}

// Write the plan's schedule into the cache file (other entries kept when
// the file parses; an unparsable file is replaced).
void store_cached(const std::string& sig, const std::map<int, int>& gcol, const std::map<int, int>& grow,
                  bool persist, int smooth) {
  const char* path = std::getenv("SFD_TUNE_CACHE");
  if (!path || !*path) return;
  JVal root;
  std::map<std::string, std::string> kept;  // key -> serialised entry
  auto ser = [](const JVal& v, auto& self) -> std::string {
    if (v.kind == JVal::kInt) return std::to_string(v.i);
    if (v.kind == JVal::kStr) return "\"" + v.s + "\"";
    std::string out = "{";
    bool first = true;
    for (const auto& kv : v.o) {
      out += (first ? "" : ", ") + std::string("\"") + kv.first + "\": " + self(kv.second, self);
      first = false;
    }
    return out + "}";
  };
  if (read_cache(path, &root))
    for (const auto& kv : root.o["entries"].o) kept[kv.first] = ser(kv.second, ser);
  auto widths = [](const std::map<int, int>& m) {
    std::string out = "{";
    bool first = true;
    for (const auto& kv : m) {
      out += (first ? "" : ", ") + std::string("\"") + std::to_string(kv.first) + "\": " + std::to_string(kv.second);
      first = false;
    }
    return out + "}";
  };
  kept[cache_key(sig)] = "{\"col\": " + widths(gcol) + ", \"row\": " + widths(grow) +
                         ", \"persist\": " + (persist ? "1" : "0") + ", \"smooth\": " + std::to_string(smooth) + "}";
  std::string text = "{\"format\": \"sfd-schedule-cache\", \"version\": " + std::to_string(kScheduleVersion) +
                     ", \"entries\": {\n";
  bool first = true;
  for (const auto& kv : kept) {
    text += (first ? "  \"" : ",\n  \"") + kv.first + "\": " + kv.second;
    first = false;
  }
  text += "\n}}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  std::fclose(f);
  if (ok) std::rename(tmp.c_str(), path);
  else std::remove(tmp.c_str());
}
}  // namespace

namespace {
std::atomic<uint64_t> g_plan_serial{0};
// Which plan used a no-allocation scratch array (per device address) last.
std::mutex g_scratch_mu;
std::map<void*, uint64_t> g_scratch_owner;
}  // namespace

struct sfd_plan_s {
  const uint64_t serial = ++g_plan_serial;
  double lam = 0;
  sfd_grid holo{};
  int n_holo = 0;
  std::vector<sfd_view> views;
  uint32_t flags = 0;

  std::vector<ViewLayout> lay;
  std::vector<TileLayout> tiles;
  std::vector<int> lengths;           // distinct L values used
  std::map<int, size_t> tw_off;       // twiddle table of the passes' shape per L
  std::map<int, size_t> tws_off;      // twiddle table of the kernel-spectrum shape per L
  int raw_nx = 0;                     // sfd_set_raw_input: camera samples per hologram row (0: none)
  int raw_bits = 32;                  // and their size
  void* tw_ready_ws = nullptr;        // workspace whose twiddle tables are current
  // Two forward descriptor slots (desc_off, desc_off2) of desc_bytes each: a
  // caller that alternates between two inputs (the streaming loop's two
  // hologram buffers) finds both images resident and uploads nothing.
  size_t desc_off = 0, desc_off2 = 0, desc_bytes = 0;
  int fwd_slot = 0;  // the forward slot of the last call
  size_t ws_bytes = 0;

  // Descriptor upload state.
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t upload_event = nullptr;
  std::vector<unsigned char> last_desc[3];  // forward, backward, second forward descriptor images
  void* last_ws[3] = {nullptr, nullptr, nullptr};
  void forget_descs() {
    for (auto& d : last_desc) d.clear();
  }

  // Backward (adjoint and z-derivative) workspace layout, SFD_IN_C64 plans.
  struct BwdLayout {
    size_t prexf, preyf, postxf, postyf, prexm, preym, prexa, preya, postxa, postya;
    size_t hxf, hyf, hxa, hya;
    size_t gtile;  // column-major copy of the view's gradient (ld col_ld(view ny))
    size_t wf, wm, wa, vbuf;  // vbuf = 0: adjoint written straight into grad_in
    size_t p12, p3, p4, p5;
    int nt_r, nt_a;           // tiles of the row passes on the view grid / hologram grid
  };
  std::vector<BwdLayout> blay;
  std::vector<int> holo_views;  // views per hologram
  size_t bwd_desc_off = 0, bwd_desc_bytes = 0;

  // Benchmark timing (sfd_profile_enable).
  bool profiling = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;

  // Persistent launch (batched plans whose passes all have persistent
  // shapes): counters in the workspace, zeroed once per workspace.
  int smooth = kSmoothDefault;  // length policy: smooth lengths allowed (see choose_length)
  bool persist_ok = false;   // the plan's shapes allow it
  bool persist = false;      // the schedule uses it
  size_t sync_off = 0;
  int sync_words = 0;
  int nstrips = 0;
  int col_tiles = 0;         // column tiles per view
  void* sync_ready_ws = nullptr;
  int persist_grid = 0;

  // Schedule: tile width per transform length of the column (y) and row (x)
  // passes; lengths not listed use the default.
  std::map<int, int> gcol, grow;
  std::string shape_sig;  // hologram grid, view sizes and flags, for the tuning table
  int tile_g(int L, bool col) const {
    const auto& m = col ? gcol : grow;
    const auto it = m.find(L);
    return it != m.end() ? it->second : sfd::rows_per_tile(L, col);
  }

  // Recorded forward launch sequence (batched plans), per forward
  // descriptor slot, with [0] and without [1] the tables and spectra
  // (SFD_REUSE_TABLES): valid for graph_ws.
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* graph_ws = nullptr;

  // SFD_REUSE_TABLES: the workspace whose tables and spectra hold the
  // distances tables_z.
  void* tables_ws = nullptr;
  std::vector<double> tables_z;

  void drop_graph() {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        if (gexec[a][b]) (void)hipGraphExecDestroy(gexec[a][b]);
        if (graph[a][b]) (void)hipGraphDestroy(graph[a][b]);
        gexec[a][b] = nullptr;
        graph[a][b] = nullptr;
      }
    graph_ws = nullptr;
  }

  // sfd_stream_frame: the copy stream and, per device buffer, the events
  // that order a frame's copy after the reconstruction that last read the
  // buffer, and that reconstruction after the copy.
  hipStream_t copy_stream = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t consumed[2] = {nullptr, nullptr};
  bool consumed_set[2] = {false, false};
  int64_t frames = 0;

  ~sfd_plan_s() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    for (int b = 0; b < 2; ++b) {
      if (copied[b]) (void)hipEventDestroy(copied[b]);
      if (consumed[b]) (void)hipEventDestroy(consumed[b]);
    }
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
    if (upload_event) (void)hipEventDestroy(upload_event);
    if (pinned) (void)hipHostFree(pinned);
  }
};

namespace {

hipError_t take_event(sfd_plan_s* P, hipEvent_t* e) {
  if (!P->event_pool.empty()) {
    *e = P->event_pool.back();
    P->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Brackets one kernel launch with events when profiling is on.
struct KernelTimer {
  sfd_plan_s* P;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t begin() {
    if (!P->profiling) return hipSuccess;
    hipError_t e = take_event(P, &a);
    if (e == hipSuccess) e = take_event(P, &b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    return e;
  }
  hipError_t end() {
    if (!P->profiling || !a) return hipSuccess;
    hipError_t e = hipEventRecord(b, s);
    if (e == hipSuccess) P->recs.push_back({kind, a, b});
    return e;
  }
};

#define SFD_TIMED(plan, kind, stream, launch)                 \
  do {                                                        \
    KernelTimer kt_{(plan), (kind), (stream)};                \
    SFD_HIP_TRY(kt_.begin());                                 \
    SFD_HIP_TRY(launch);                                      \
    SFD_HIP_TRY(kt_.end());                                   \
  } while (0)

// Host images of the device descriptors for one forward call, in the order
// they are laid out in the workspace descriptor area.
struct CallDescs {
  std::vector<sfd::AxisJob> axis;      // sorted by L
  std::vector<sfd::TwiddleJob> tw;
  std::vector<sfd::TileJob> tiles;
  std::vector<sfd::RowJob> rows;       // column-pass jobs, then row-pass jobs
  std::vector<int> axis_L;             // L of each axis job
  std::vector<int> row_L;              // L of each row job
  int n_pass_x = 0;
  // Persistent launch: device address of its arguments and its item count.
  const sfd::PersistArgs* d_pa = nullptr;
  int persist_total = 0;
};

size_t bwd_desc_capacity(int n_views, int n_holo, int n_lengths, int n_tiles) {
  return align_up(sizeof(sfd::AxisJob) * 6 * n_views) + align_up(sizeof(sfd::TwiddleJob) * 2 * n_lengths) +
         align_up(sizeof(sfd::TileJob) * (n_tiles + n_views)) + align_up(sizeof(sfd::RowJob) * 7 * n_views) +
         align_up(sizeof(sfd::GradZJob) * n_views) + align_up(sizeof(sfd::GatherJob) * n_holo) +
         align_up(sizeof(void*) * n_views) + align_up(sizeof(sfd::SumJob) * n_views);
}

// Persistent launch descriptors after the row jobs: the launch arguments,
// one PassArgs per pass segment, column tiles per view, twiddle tables per
// view and axis.
size_t persist_desc_bytes(int n_views) {
  return align_up(sizeof(sfd::PersistArgs)) + align_up(sizeof(sfd::PassArgs) * sfd::kMaxSegments) +
         align_up(sizeof(int32_t) * n_views) + align_up(sizeof(void*) * 2 * n_views);
}

size_t desc_capacity(int n_views, int n_lengths, int n_tiles) {
  return align_up(sizeof(sfd::AxisJob) * 2 * n_views) + align_up(sizeof(sfd::TwiddleJob) * 2 * n_lengths) +
         align_up(sizeof(sfd::TileJob) * n_tiles) + align_up(sizeof(sfd::RowJob) * 2 * n_views) +
         persist_desc_bytes(n_views);
}

// The twiddle tables of length L, both shapes: the passes' and the kernel
// spectra's (built once per workspace).
void add_twiddle_jobs(const sfd_plan_s* P, char* ws, int L, std::vector<sfd::TwiddleJob>* out) {
  for (int spec = 0; spec < 2; ++spec) {
    sfd::TwiddleJob t{};
    t.tw = reinterpret_cast<float2*>(ws + (spec ? P->tws_off.at(L) : P->tw_off.at(L)));
    t.L = L;
    t.count = sfd::twiddle_len(L, spec != 0);
    t.spec = spec;
    out->push_back(t);
  }
}


sfd_status build_descs(sfd_plan_s* P, const void* holo, const double* z, void* const* out, char* ws,
                       CallDescs* D) {
  const int V = (int)P->views.size();
  const bool field = (P->flags & SFD_OUT_FIELD) != 0;
  const bool in_real = (P->flags & SFD_IN_REAL_F32) != 0;
  const int32_t pflags = (P->flags & SFD_PHASE_FP32) ? sfd::kPhaseFp32 : 0;
  const sfd_grid& h = P->holo;
  const size_t in_elem = in_real ? sizeof(float) : sizeof(float2);
  const size_t holo_stride =
      P->raw_nx > 0 ? (size_t)P->raw_nx * h.ny * (P->raw_bits / 8) : (size_t)h.nx * h.ny * in_elem;

  struct AxisTmp {
    sfd::AxisJob j;
    int L;
    int key;  // 2 v + axis
  };
  std::vector<AxisTmp> ax;
  ax.reserve(2 * V);
  for (int v = 0; v < V; ++v) {
    const sfd_view& w = P->views[v];
    const ViewLayout& L = P->lay[v];
    const double zz = z ? z[v] : w.z;
    double c_re, c_im;
    prefactor(P->lam, zz, h.px, h.py, &c_re, &c_im);
    AxisScalars sx = axis_scalars(h.nx, h.px, h.ox, w.out.nx, w.out.px, w.out.ox, P->lam, zz);
    AxisScalars sy = axis_scalars(h.ny, h.py, h.oy, w.out.ny, w.out.py, w.out.oy, P->lam, zz);
    for (int a = 0; a < 2; ++a) {
      const AxisScalars& s = a == 0 ? sx : sy;
      sfd::AxisJob j{};
      j.a0 = s.a0;
      j.a1 = s.a1;
      j.p0 = s.p0;
      j.p1 = s.p1;
      j.inv_lz = s.inv_lz;
      j.S = s.S;
      j.c1 = s.c1;
      j.wscale = 0.0;
      // The prefactor c(z) rides on the x post-chirp (field output only).
      j.post_scale = a == 0 ? make_float2((float)c_re, (float)c_im) : make_float2(1.f, 0.f);
      j.pre = reinterpret_cast<float2*>(ws + (a == 0 ? L.prex : L.prey));
      j.post = field ? reinterpret_cast<float2*>(ws + (a == 0 ? L.postx : L.posty)) : nullptr;
      j.H = reinterpret_cast<float2*>(ws + (a == 0 ? L.hx : L.hy));
      j.n0 = a == 0 ? h.nx : h.ny;
      j.n1 = a == 0 ? w.out.nx : w.out.ny;
      j.L = a == 0 ? L.lx : L.ly;
      j.flags = pflags;
      ax.push_back({j, j.L, 2 * v + a});
    }
  }
  // The setup launch groups the spectra by length; the persistent launch's
  // setup items find a view's two axis jobs at 2v (x) and 2v + 1 (y).
  if (!(P->flags & SFD_PER_VIEW_LAUNCH) && !P->persist)
    std::stable_sort(ax.begin(), ax.end(), [](const AxisTmp& a, const AxisTmp& b) { return a.L < b.L; });
  D->axis.clear();
  D->axis_L.clear();
  std::vector<int> axis_pos(2 * V);
  for (auto& a : ax) {
    axis_pos[a.key] = (int)D->axis.size();
    D->axis.push_back(a.j);
    D->axis_L.push_back(a.L);
  }
  D->tw.clear();
  for (int L : P->lengths) add_twiddle_jobs(P, ws, L, &D->tw);
  D->tiles.clear();
  for (const TileLayout& T : P->tiles) {
    sfd::TileJob j{};
    j.in = static_cast<const char*>(holo) + (size_t)T.holo * holo_stride;
    j.out = ws + T.off;
    j.nx = h.nx;
    j.ny = h.ny;
    j.ld = col_ld(h.ny);
    j.complex_in = in_real ? 0 : 1;
    j.nx_src = P->raw_nx;
    j.src_bits = P->raw_bits;
    D->tiles.push_back(j);
  }

  // Column pass (y transforms of the hologram columns) then row pass (x
  // transforms of the rows of the N1y x N0x intermediate), one job per view,
  // stable-sorted by L within each pass.
  D->rows.clear();
  D->row_L.clear();
  const bool inten = (P->flags & SFD_OUT_INTENSITY) != 0;
  std::vector<std::pair<int, sfd::RowJob>> px, py;
  for (int v = 0; v < V; ++v) {
    const sfd_view& w = P->views[v];
    const ViewLayout& L = P->lay[v];
    const double zz = z ? z[v] : w.z;
    double c_re, c_im;
    prefactor(P->lam, zz, h.px, h.py, &c_re, &c_im);

    const int ldw = inter_ld(h.nx);
    sfd::RowJob jc{};
    jc.out = ws + L.inter;
    jc.pre = reinterpret_cast<const float2*>(ws + L.prey);
    jc.H = reinterpret_cast<const float2*>(ws + L.hy);
    jc.post = field ? reinterpret_cast<const float2*>(ws + L.posty) : nullptr;
    jc.iscale = 1.f;
    jc.n_rows = h.nx;
    jc.n_in = h.ny;
    jc.n_out = w.out.ny;
    jc.out_ld = ldw;
    jc.mode = (in_real ? sfd::kInReal : 0) | (field ? sfd::kUsePost : 0) | sfd::kOutField;
    jc.in = ws + P->tiles[L.tile].off;
    jc.in_ld = col_ld(h.ny);
    jc.colscale = reinterpret_cast<const float2*>(ws + L.prex);
    jc.view = v;
    jc.copy = L.tile;
    jc.ax_pre = axis_pos[2 * v + 1];
    jc.ax_scale = axis_pos[2 * v];
    if (P->persist && in_real) {
      // The persistent launch reads real holograms in place, row-major.
      jc.in = static_cast<const char*>(holo) + (size_t)w.holo * holo_stride;
      jc.in_ld = P->raw_nx > 0 ? P->raw_nx : h.nx;
      jc.in_fmt = P->raw_nx > 0 ? (P->raw_bits == 32 ? 33 : P->raw_bits) : 32;
    }
    py.push_back({L.ly, jc});

    sfd::RowJob jr{};
    jr.in = ws + L.inter;
    jr.out = field ? out[inten ? V + v : v] : out[v];
    jr.out2 = (field && inten) ? static_cast<float*>(out[v]) : nullptr;
    jr.pre = nullptr;  // the column pass applied pre_x (constant along each column)
    jr.H = reinterpret_cast<const float2*>(ws + L.hx);
    jr.post = field ? reinterpret_cast<const float2*>(ws + L.postx) : nullptr;
    // With the field written, |c|^2 is already inside it (c rides on post).
    jr.iscale = field ? 1.f : (float)(c_re * c_re + c_im * c_im);
    jr.n_rows = w.out.ny;
    jr.n_in = h.nx;
    jr.n_out = w.out.nx;
    jr.in_ld = ldw;
    jr.out_ld = w.out.nx;
    jr.mode = (field ? (sfd::kUsePost | sfd::kOutField) : 0) | (inten ? sfd::kOutIntensity : 0);
    jr.view = v;
    jr.copy = L.tile;
    px.push_back({L.lx, jr});
  }
  auto by_len = [](const std::pair<int, sfd::RowJob>& a, const std::pair<int, sfd::RowJob>& b) {
    return a.first < b.first;
  };
  if (!(P->flags & SFD_PER_VIEW_LAUNCH)) {
    std::stable_sort(px.begin(), px.end(), by_len);
    std::stable_sort(py.begin(), py.end(), by_len);
  }
  for (auto& p : py) {
    D->rows.push_back(p.second);
    D->row_L.push_back(p.first);
  }
  for (auto& p : px) {
    D->rows.push_back(p.second);
    D->row_L.push_back(p.first);
  }
  D->n_pass_x = (int)py.size();  // jobs of the first (column) pass
  return SFD_OK;
}

// Kernel specialisation of a pass over row jobs [i, j) of length L (the
// rule of launch_pass, see sfd_internal.h).
int pass_var(const CallDescs& D, int i, int j, int L, bool col) {
  bool fast = true, no_post = true, int_only = true, all_real = true, all_complex = true, reduce = false;
  for (int k = i; k < j; ++k) {
    const sfd::RowJob& r = D.rows[k];
    const int F = sfd::fast_input(L);
    // The reduction epilogue has a specialised row kernel (3), not a column one.
    fast = fast && r.n_in == F && r.n_out <= F && (!col || !(r.mode & sfd::kReduce));
    reduce = reduce || (r.mode & sfd::kReduce);
    no_post = no_post && !(r.mode & sfd::kUsePost);
    int_only = int_only && (r.mode & sfd::kOutIntensity) && !(r.mode & sfd::kOutField);
    all_real = all_real && (r.mode & sfd::kInReal);
    all_complex = all_complex && !(r.mode & sfd::kInReal);
  }
  if (fast && col) return all_complex ? 1 : !all_real ? 0 : no_post ? 2 : 3;
  if (fast && all_complex) return reduce ? 3 : no_post && int_only ? 2 : 1;
  return 0;
}

// Serialise descriptors into the workspace layout; returns the byte image.
void pack_descs(const sfd_plan_s* P, const CallDescs& D, std::vector<unsigned char>* img, size_t* off_axis,
                size_t* off_tw, size_t* off_rows, size_t* off_tiles_out = nullptr) {
  const int V = (int)P->views.size();
  *off_axis = 0;
  *off_tw = align_up(sizeof(sfd::AxisJob) * 2 * V);
  const size_t off_tiles = *off_tw + align_up(sizeof(sfd::TwiddleJob) * 2 * P->lengths.size());
  if (off_tiles_out) *off_tiles_out = off_tiles;
  *off_rows = off_tiles + align_up(sizeof(sfd::TileJob) * P->tiles.size());
  const size_t total = *off_rows + sizeof(sfd::RowJob) * D.rows.size();
  img->assign(total, 0);
  std::memcpy(img->data() + *off_axis, D.axis.data(), sizeof(sfd::AxisJob) * D.axis.size());
  std::memcpy(img->data() + *off_tw, D.tw.data(), sizeof(sfd::TwiddleJob) * D.tw.size());
  std::memcpy(img->data() + off_tiles, D.tiles.data(), sizeof(sfd::TileJob) * D.tiles.size());
  std::memcpy(img->data() + *off_rows, D.rows.data(), sizeof(sfd::RowJob) * D.rows.size());
}

// Runs of jobs [first, end) with equal L and at most kMaxJobsPerLaunch jobs.
template <typename F>
void for_length_runs(const CallDescs& D, int first, int end, F f) {
  int i = first;
  while (i < end) {
    const int L = D.row_L[i];
    int j = i;
    while (j < end && D.row_L[j] == L && j - i < sfd::kMaxJobsPerLaunch) ++j;
    f(i, j, L);
    i = j;
  }
}

// Segments of a persistent launch for the plan's shapes (setup when
// ``tables``, strips, then a column and a row segment per length run).
int persist_segments(const sfd_plan_s* P, const CallDescs& D, bool tables) {
  int n = (tables ? 1 : 0) + 1;
  for_length_runs(D, 0, D.n_pass_x, [&](int, int, int) { ++n; });
  for_length_runs(D, D.n_pass_x, (int)D.rows.size(), [&](int, int, int) { ++n; });
  (void)P;
  return n;
}

// Append the persistent launch's descriptors to the image (after the row
// jobs) and set D->d_pa and D->persist_total.  Every pointer they hold is a
// workspace address, so the image only changes with the plan's schedule,
// the call's tables flag and the call's pointers.
void pack_persist(const sfd_plan_s* P, CallDescs* D, char* ws, bool tables, std::vector<unsigned char>* img,
                  size_t off_axis, size_t off_tiles, size_t off_rows, size_t base_off) {
  const int V = (int)P->views.size();
  char* dbase = ws + base_off;
  const size_t off_pa = align_up(off_rows + sizeof(sfd::RowJob) * D->rows.size());
  const size_t off_pass = off_pa + align_up(sizeof(sfd::PersistArgs));
  const size_t off_ct = off_pass + align_up(sizeof(sfd::PassArgs) * sfd::kMaxSegments);
  const size_t off_twv = off_ct + align_up(sizeof(int32_t) * V);
  const size_t end = off_twv + align_up(sizeof(void*) * 2 * V);
  img->resize(end, 0);
  sfd::PersistArgs pa{};
  std::vector<sfd::PassArgs> pass;
  int t = 0;
  auto add = [&](int kind, int count, int L, int var, const sfd::PassArgs* args, const float2* tw) {
    sfd::Segment& g = pa.seg[pa.nseg++];
    g.kind = kind;
    g.first = t;
    g.count = count;
    g.L = L;
    g.var = var;
    g.args = args;
    g.tw = tw;
    t += count;
  };
  if (tables) add(sfd::kItemSetup, 3 * V, 0, 0, nullptr, nullptr);  // y spectra, x spectra, tables, per view
  if (P->nstrips > 0) add(sfd::kItemStrip, P->nstrips, 0, 0, nullptr, nullptr);
  const auto* d_rows = reinterpret_cast<const sfd::RowJob*>(dbase + off_rows);
  const auto* d_pass = reinterpret_cast<const sfd::PassArgs*>(dbase + off_pass);
  for (int col = 1; col >= 0; --col) {
    const int first = col ? 0 : D->n_pass_x, last = col ? D->n_pass_x : (int)D->rows.size();
    for_length_runs(*D, first, last, [&](int i, int j, int L) {
      sfd::PassArgs a{};
      a.jobs = d_rows + i;
      a.axis = reinterpret_cast<const sfd::AxisJob*>(dbase + off_axis);
      a.njobs = j - i;
      int acc = 0;
      for (int k = i; k < j; ++k) {
        a.tile_prefix[k - i] = acc;
        acc += (D->rows[k].n_rows + sfd::kStripW - 1) / sfd::kStripW;
      }
      a.tile_prefix[j - i] = acc;
      a.total_tiles = acc;
      add(col ? sfd::kItemCol : sfd::kItemRow, acc, L, pass_var(*D, i, j, L, col != 0), d_pass + pass.size(),
          reinterpret_cast<const float2*>(ws + P->tw_off.at(L)));
      pass.push_back(a);
    });
  }
  pa.total = t;
  pa.grid = std::max(1, std::min(t, P->persist_grid));
  pa.nview = V;
  pa.wait_setup = tables ? 1 : 0;
  pa.ncopy = (int)P->tiles.size();
  pa.nstrips = P->nstrips;
  pa.axis = reinterpret_cast<const sfd::AxisJob*>(dbase + off_axis);
  pa.tiles = reinterpret_cast<const sfd::TileJob*>(dbase + off_tiles);
  pa.col_tiles = reinterpret_cast<const int32_t*>(dbase + off_ct);
  pa.tw_view = reinterpret_cast<const float2* const*>(dbase + off_twv);
  pa.sync = reinterpret_cast<uint32_t*>(ws + P->sync_off);
  std::vector<int32_t> ct(V, P->col_tiles);
  std::vector<const float2*> twv(2 * V);
  for (int v = 0; v < V; ++v) {
    twv[2 * v] = reinterpret_cast<const float2*>(ws + P->tws_off.at(P->lay[v].lx));
    twv[2 * v + 1] = reinterpret_cast<const float2*>(ws + P->tws_off.at(P->lay[v].ly));
  }
  std::memcpy(img->data() + off_pa, &pa, sizeof pa);
  std::memcpy(img->data() + off_pass, pass.data(), sizeof(sfd::PassArgs) * pass.size());
  std::memcpy(img->data() + off_ct, ct.data(), sizeof(int32_t) * V);
  std::memcpy(img->data() + off_twv, twv.data(), sizeof(void*) * 2 * V);
  D->d_pa = reinterpret_cast<const sfd::PersistArgs*>(dbase + off_pa);
  D->persist_total = t;
}

// Copy a descriptor image into the workspace at ``dst_off`` (slot 0:
// forward, 1: backward), unless the same image already sits there.
sfd_status upload(sfd_plan_s* P, int slot, const std::vector<unsigned char>& img, char* ws, size_t dst_off,
                  hipStream_t stream) {
  if (P->last_ws[slot] == ws && P->last_desc[slot] == img) return SFD_OK;
  if (!P->upload_event) SFD_HIP_TRY(hipEventCreateWithFlags(&P->upload_event, hipEventDisableTiming));
  if (P->pinned_bytes < img.size()) {
    if (P->pinned) {
      SFD_HIP_TRY(hipEventSynchronize(P->upload_event));
      SFD_HIP_TRY(hipHostFree(P->pinned));
      P->pinned = nullptr;
    }
    SFD_HIP_TRY(hipHostMalloc(&P->pinned, img.size(), hipHostMallocDefault));
    P->pinned_bytes = img.size();
  } else {
    // The previous upload may still be reading the staging buffer.
    SFD_HIP_TRY(hipEventSynchronize(P->upload_event));
  }
  std::memcpy(P->pinned, img.data(), img.size());
  SFD_HIP_TRY(hipMemcpyAsync(ws + dst_off, P->pinned, img.size(), hipMemcpyHostToDevice, stream));
  SFD_HIP_TRY(hipEventRecord(P->upload_event, stream));
  P->last_desc[slot] = img;
  P->last_ws[slot] = ws;
  return SFD_OK;
}

// Setup launch(es) for axis jobs [a0, a0 + na), all twiddle tables if
// ``twiddles``, and tile jobs [t0, t0 + nt).
sfd_status launch_setup_for(sfd_plan_s* P, const CallDescs& D, char* ws, const sfd::AxisJob* d_axis,
                            const sfd::TwiddleJob* d_tw, const sfd::TileJob* d_tiles, int a0, int na,
                            bool twiddles, int t0, int nt, hipStream_t stream, int spec_count = -1) {
  // Spectra for axis jobs [a0, a0 + spec_count) (default: all na), tables for [a0, a0 + na).
  const int ns = spec_count < 0 ? na : spec_count;
  sfd::SetupArgs A{};
  A.axis = d_axis;
  A.tw = d_tw;
  A.tiles = d_tiles;
  auto flush = [&]() -> sfd_status {
    if (A.nroles == 0) return SFD_OK;
    SFD_TIMED(P, SFD_KERNEL_TABLES, stream, sfd::launch_setup(A, stream));
    A.nroles = 0;
    A.total_blocks = 0;
    A.max_l = 0;
    return SFD_OK;
  };
  auto add = [&](sfd::SetupRole r) -> sfd_status {
    if (r.nblocks <= 0) return SFD_OK;
    if (A.nroles == sfd::kMaxSetupRoles) {
      sfd_status st = flush();
      if (st != SFD_OK) return st;
    }
    r.first_block = A.total_blocks;
    if (r.kind == sfd::kRoleSpectrum) A.max_l = std::max(A.max_l, r.a);
    A.roles[A.nroles++] = r;
    A.total_blocks += r.nblocks;
    return SFD_OK;
  };
  sfd_status st;
  // Kernel spectra: runs of equal L.
  for (int i = a0; i < a0 + ns;) {
    int j = i;
    while (j < a0 + ns && D.axis_L[j] == D.axis_L[i]) ++j;
    const int L = D.axis_L[i];
    const int per = sfd::spectra_per_block(L);
    if ((st = add({sfd::kRoleSpectrum, 0, (j - i + per - 1) / per, L, i, j - i,
                   reinterpret_cast<const float2*>(ws + P->tws_off.at(L))})) != SFD_OK)
      return st;
    i = j;
  }
  // Pre/post chirp tables.
  int span = 0;
  for (int i = a0; i < a0 + na; ++i) span = std::max(span, D.axis[i].n0 + (D.axis[i].post ? D.axis[i].n1 : 0));
  const int chunks = (span + sfd::kSetupThreads - 1) / sfd::kSetupThreads;
  if (na > 0 && (st = add({sfd::kRoleTables, 0, na * chunks, chunks, a0, na, nullptr})) != SFD_OK) return st;
  if (twiddles)
    for (int k = 0; k < (int)D.tw.size(); ++k)
      if ((st = add({sfd::kRoleTwiddles, 0, (D.tw[k].count + sfd::kSetupThreads - 1) / sfd::kSetupThreads, k, 0,
                     0, nullptr})) != SFD_OK)
        return st;
  for (int k = t0; k < t0 + nt; ++k) {
    const int cb = (D.tiles[k].nx + sfd::kTrBlock - 1) / sfd::kTrBlock;
    const int rb = (D.tiles[k].ny + sfd::kTrBlock - 1) / sfd::kTrBlock;
    if ((st = add({sfd::kRoleTiles, 0, cb * rb, k, cb, 0, nullptr})) != SFD_OK) return st;
  }
  return flush();
}

// Launch the passes of row jobs [first, first + count) grouped by L.
sfd_status launch_rows(const CallDescs& D, const sfd::RowJob* d_rows, int first, int count,
                       sfd_plan_s* P, char* ws, hipStream_t stream, int kind) {
  const bool col = kind == SFD_KERNEL_PASS_Y;
  int i = first;
  const int end = first + count;
  while (i < end) {
    const int L = D.row_L[i];
    int j = i;
    while (j < end && D.row_L[j] == L && j - i < sfd::kMaxJobsPerLaunch) ++j;
    sfd::PassArgs a{};
    a.jobs = d_rows + i;
    a.njobs = j - i;
    const int G = P->tile_g(L, col);
    int acc = 0;
    for (int k = i; k < j; ++k) {
      a.tile_prefix[k - i] = acc;
      acc += (D.rows[k].n_rows + G - 1) / G;
    }
    a.tile_prefix[j - i] = acc;
    a.total_tiles = acc;
    const int var = pass_var(D, i, j, L, col);
    const float2* tw = reinterpret_cast<const float2*>(ws + P->tw_off.at(L));
    SFD_TIMED(P, kind, stream, sfd::launch_pass(L, col, G, var, a, tw, stream));
    i = j;
  }
  return SFD_OK;
}

// Tile counts that follow the schedule (the allocations were sized for every
// tile width, so offsets never move).
void apply_schedule(sfd_plan_s* P) {
  for (size_t v = 0; v < P->blay.size(); ++v) {
    sfd_plan_s::BwdLayout& B = P->blay[v];
    const sfd_grid& o = P->views[v].out;
    const int gr = P->tile_g(P->lay[v].lx, false);
    B.nt_r = (o.ny + gr - 1) / gr;
    B.nt_a = (P->holo.ny + gr - 1) / gr;
  }
  P->drop_graph();
}

// Whether the persistent launch serves the plan's current lengths: a batched
// plan whose passes all run the persistent shapes (fast inputs, see
// fast_input, at a persistent length) in few enough segments.
bool persist_eligible(const sfd_plan_s* P) {
  if (P->flags & SFD_PER_VIEW_LAUNCH) return false;
  const sfd_grid& h = P->holo;
  std::map<int, int> per_len;
  for (size_t v = 0; v < P->views.size(); ++v) {
    const sfd_grid& o = P->views[v].out;
    const int lx = P->lay[v].lx, ly = P->lay[v].ly;
    if (!(sfd::persist_length(lx) && sfd::persist_length(ly) && h.nx == sfd::fast_input(lx) &&
          o.nx <= sfd::fast_input(lx) && h.ny == sfd::fast_input(ly) && o.ny <= sfd::fast_input(ly)))
      return false;
    per_len[ly]++;
    per_len[-lx]++;
  }
  int segs = 2;
  for (const auto& kv : per_len) segs += (kv.second + sfd::kMaxJobsPerLaunch - 1) / sfd::kMaxJobsPerLaunch;
  return segs <= sfd::kMaxSegments;
}

// Length policy (see choose_length).  Per-view arrays are sized for the
// longest choice (powers of two).
void set_lengths(sfd_plan_s* P, int smooth) {
  P->smooth = smooth;
  for (size_t v = 0; v < P->views.size(); ++v) {
    P->lay[v].lx = choose_length(P->holo.nx, P->views[v].out.nx, smooth);
    P->lay[v].ly = choose_length(P->holo.ny, P->views[v].out.ny, smooth);
  }
}

// The batched forward sequence: every view's tables, spectra and hologram
// tiles (tables = false: the tiles only), then all column passes, then all
// row passes.
sfd_status launch_forward(sfd_plan_s* P, const CallDescs& D, char* ws, const sfd::AxisJob* d_axis,
                          const sfd::TwiddleJob* d_tw, const sfd::TileJob* d_tiles, const sfd::RowJob* d_rows,
                          hipStream_t stream, bool tables = true) {
  sfd_status st;
  if (P->persist) {
    SFD_TIMED(P, SFD_KERNEL_PERSIST, stream,
              sfd::launch_persist(D.d_pa, std::max(1, std::min(D.persist_total, P->persist_grid)),
                                  (P->flags & SFD_IN_C64) != 0, stream));
    return SFD_OK;
  }
  if ((st = launch_setup_for(P, D, ws, d_axis, d_tw, d_tiles, 0, tables ? (int)D.axis.size() : 0, false, 0,
                             (int)D.tiles.size(), stream)) != SFD_OK)
    return st;
  if ((st = launch_rows(D, d_rows, 0, D.n_pass_x, P, ws, stream, SFD_KERNEL_PASS_Y)) != SFD_OK) return st;
  return launch_rows(D, d_rows, D.n_pass_x, (int)D.rows.size() - D.n_pass_x, P, ws, stream, SFD_KERNEL_PASS_X);
}

sfd_status check_common(sfd_plan_t plan, void* workspace, size_t ws_bytes) {
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  if (!workspace) return fail(SFD_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(SFD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < plan->ws_bytes)
    return fail(SFD_ERR_WORKSPACE, "workspace is " + std::to_string(ws_bytes) + " bytes, plan needs " +
                                       std::to_string(plan->ws_bytes));
  return SFD_OK;
}

sfd_status check_z(const sfd_plan_s* P, const double* z) {
  if (!z) return SFD_OK;
  for (size_t v = 0; v < P->views.size(); ++v)
    if (!std::isfinite(z[v]) || z[v] == 0.0)
      return fail(SFD_ERR_INVALID_ARG, "z[" + std::to_string(v) + "] must be finite and non-zero");
  return SFD_OK;
}

// Backward pass (see include/sfd.h).  Per view v with u1 = A u0 and
// g = dL/dRe(u1) + i dL/dIm(u1):
//   grad_in[holo(v)] += A^H g, with A^H = conj(c) Ay^H (x) Ax^H: the same two
//     passes on g with the planes swapped and z -> -z;
//   dL/dz = Re sum conj(g) du1/dz, du1/dz = A (i k - 1/z - i pi r^2/(lambda z^2)) u0 with
//     r^2 = x1^2 - 2 x1 x0 + x0^2 (+ y terms), i.e. (separability)
//     dL/dz = Re[(i k - 1/z) S1 - (i pi/(lambda z^2)) (S2 - 2 S3 - 2 S4 + S5)],
//     S1 = sum conj(g) u1, S2 = sum conj(g) (x1^2 + y1^2) u1,
//     S3 = sum conj(g) x1 A(x0 u0), S4 = sum conj(g) y1 A(y0 u0),
//     S5 = sum conj(A^H g) (x0^2 + y0^2) u0.
// A(x0 u0) reuses the y pass of u0; A(y0 u0) takes one more y pass.  The
// sums are fused into the row-pass epilogues (FP64) and finished per view.
sfd_status run_backward(sfd_plan_s* P, void* const* grad_out, void* const* field_out, const void* holo,
                        const double* z_or_null, void* grad_in, double* grad_z, char* ws, hipStream_t stream) {
  const int V = (int)P->views.size();
  const sfd_grid& h = P->holo;
  const bool want_z = grad_z != nullptr;
  const bool from_i = field_out != nullptr;  // grad_out holds dL/dI
  const bool real_in = (P->flags & SFD_IN_C64) == 0;  // a real hologram: its gradient is Re(A^H g)
  const size_t holo_stride = (size_t)h.nx * h.ny * (real_in ? sizeof(float) : sizeof(float2));
  const double k = 2.0 * M_PI / P->lam;
  CallDescs D;

  // Axis jobs: spectrum-bearing ones (fx, fy, ax, ay per view) first, sorted
  // by L, then the moment tables (mx, my), which reuse fx/fy spectra.
  struct AxisTmp {
    sfd::AxisJob j;
    int L;
  };
  std::vector<AxisTmp> spec, mom;
  auto fill = [&](const AxisScalars& sc, int n0, int n1, int L, size_t pre, size_t post, size_t H, float2 ps,
                  int32_t flags) {
    sfd::AxisJob j{};
    j.a0 = sc.a0;
    j.a1 = sc.a1;
    j.p0 = sc.p0;
    j.p1 = sc.p1;
    j.inv_lz = sc.inv_lz;
    j.S = sc.S;
    j.c1 = sc.c1;
    j.wscale = 1.0;
    j.post_scale = ps;
    j.pre = reinterpret_cast<float2*>(ws + pre);
    j.post = post ? reinterpret_cast<float2*>(ws + post) : nullptr;
    j.H = reinterpret_cast<float2*>(ws + H);
    j.n0 = n0;
    j.n1 = n1;
    j.L = L;
    j.flags = flags;
    return j;
  };
  const int32_t pflags = (P->flags & SFD_PHASE_FP32) ? sfd::kPhaseFp32 : 0;
  for (int v = 0; v < V; ++v) {
    const sfd_view& w = P->views[v];
    const sfd_plan_s::BwdLayout& B = P->blay[v];
    const ViewLayout& L = P->lay[v];
    const double z = z_or_null ? z_or_null[v] : w.z;
    double c_re, c_im, ca_re, ca_im;
    prefactor(P->lam, z, h.px, h.py, &c_re, &c_im);
    prefactor(P->lam, -z, h.px, h.py, &ca_re, &ca_im);  // conj(c(z))
    const AxisScalars fx = axis_scalars(h.nx, h.px, h.ox, w.out.nx, w.out.px, w.out.ox, P->lam, z);
    const AxisScalars fy = axis_scalars(h.ny, h.py, h.oy, w.out.ny, w.out.py, w.out.oy, P->lam, z);
    const AxisScalars ax = axis_scalars(w.out.nx, w.out.px, w.out.ox, h.nx, h.px, h.ox, P->lam, -z);
    const AxisScalars ay = axis_scalars(w.out.ny, w.out.py, w.out.oy, h.ny, h.py, h.oy, P->lam, -z);
    const float2 one = make_float2(1.f, 0.f);
    spec.push_back({fill(ax, w.out.nx, h.nx, L.lx, B.prexa, B.postxa, B.hxa, make_float2((float)ca_re, (float)ca_im),
                         pflags),
                    L.lx});
    spec.push_back({fill(ay, w.out.ny, h.ny, L.ly, B.preya, B.postya, B.hya, one, pflags), L.ly});
    if (want_z) {
      spec.push_back({fill(fx, h.nx, w.out.nx, L.lx, B.prexf, B.postxf, B.hxf, make_float2((float)c_re, (float)c_im),
                           pflags),
                      L.lx});
      spec.push_back({fill(fy, h.ny, w.out.ny, L.ly, B.preyf, B.postyf, B.hyf, one, pflags), L.ly});
      mom.push_back({fill(fx, h.nx, w.out.nx, L.lx, B.prexm, 0, B.hxf, one, pflags | sfd::kMomentX0), L.lx});
      mom.push_back({fill(fy, h.ny, w.out.ny, L.ly, B.preym, 0, B.hyf, one, pflags | sfd::kMomentX0), L.ly});
    }
  }
  std::stable_sort(spec.begin(), spec.end(), [](const AxisTmp& a, const AxisTmp& b) { return a.L < b.L; });
  for (auto& a : spec) {
    D.axis.push_back(a.j);
    D.axis_L.push_back(a.L);
  }
  const int n_spec = (int)D.axis.size();
  for (auto& a : mom) {
    D.axis.push_back(a.j);
    D.axis_L.push_back(a.L);
  }
  for (int L : P->lengths) add_twiddle_jobs(P, ws, L, &D.tw);

  // Tiles: the hologram's (for the z-moment passes) and each view's gradient.
  if (want_z)
    for (const TileLayout& T : P->tiles) {
      sfd::TileJob j{};
      j.in = static_cast<const char*>(holo) + (size_t)T.holo * holo_stride;
      j.out = ws + T.off;
      j.nx = h.nx;
      j.ny = h.ny;
      j.ld = col_ld(h.ny);
      j.complex_in = real_in ? 0 : 1;
      D.tiles.push_back(j);
    }
  const int gtile0 = (int)D.tiles.size();
  for (int v = 0; v < V; ++v) {
    const sfd_plan_s::BwdLayout& B = P->blay[v];
    sfd::TileJob j{};
    j.in = from_i ? field_out[v] : grad_out[v];
    j.in2 = from_i ? static_cast<const float*>(grad_out[v]) : nullptr;
    j.out = ws + B.gtile;
    j.nx = P->views[v].out.nx;
    j.ny = P->views[v].out.ny;
    j.ld = col_ld(P->views[v].out.ny);
    j.complex_in = 1;
    D.tiles.push_back(j);
  }

  // Passes.  Column jobs: the adjoint's y pass of g (C3) and, for dL/dz, the
  // forward (C1) and y-moment (C2) y passes of u0.  Row jobs: the adjoint's
  // x pass (R4, stores A^H g, reduces S5) and, for dL/dz, R1 (S1, S2),
  // R2 (S3), R3 (S4).
  std::vector<std::pair<int, sfd::RowJob>> cols, rows;
  std::vector<sfd::SumJob> sums;
  for (int v = 0; v < V; ++v) {
    const sfd_view& w = P->views[v];
    const sfd_plan_s::BwdLayout& B = P->blay[v];
    const ViewLayout& L = P->lay[v];
    const int ldh = inter_ld(h.nx), ldo = inter_ld(w.out.nx);
    const double z = z_or_null ? z_or_null[v] : w.z;
    const AxisScalars fx = axis_scalars(h.nx, h.px, h.ox, w.out.nx, w.out.px, w.out.ox, P->lam, z);
    const AxisScalars fy = axis_scalars(h.ny, h.py, h.oy, w.out.ny, w.out.py, w.out.oy, P->lam, z);
    const char* u0 = static_cast<const char*>(holo) + (size_t)w.holo * holo_stride;
    auto col = [&](const void* in, int in_ld, size_t out, int out_ld, size_t pre, size_t H, size_t post, int n_rows,
                   int n_in, int n_out) {
      sfd::RowJob j{};
      j.in = in;
      j.out = ws + out;
      j.pre = reinterpret_cast<const float2*>(ws + pre);
      j.H = reinterpret_cast<const float2*>(ws + H);
      j.post = reinterpret_cast<const float2*>(ws + post);
      j.iscale = 1.f;
      j.n_rows = n_rows;
      j.n_in = n_in;
      j.n_out = n_out;
      j.in_ld = in_ld;
      j.out_ld = out_ld;
      j.mode = sfd::kUsePost | sfd::kOutField;
      return j;
    };
    cols.push_back({L.ly, col(ws + B.gtile, col_ld(w.out.ny), B.wa, ldo, B.preya, B.hya, B.postya, w.out.nx, w.out.ny,
                             h.ny)});
    if (want_z) {
      const TileLayout& T = P->tiles[L.tile];
      cols.push_back({L.ly, col(ws + T.off, col_ld(h.ny), B.wf, ldh, B.preyf, B.hyf, B.postyf, h.nx, h.ny,
                                w.out.ny)});
      cols.push_back({L.ly, col(ws + T.off, col_ld(h.ny), B.wm, ldh, B.preym, B.hyf, B.postyf, h.nx, h.ny,
                                w.out.ny)});
      if (real_in) {
        cols[cols.size() - 1].second.mode |= sfd::kInReal;
        cols[cols.size() - 2].second.mode |= sfd::kInReal;
      }
    }
    auto row = [&](size_t in, int in_ld, size_t pre, size_t H, size_t post, int n_rows, int n_in, int n_out,
                   int32_t mode, size_t partial) {
      sfd::RowJob j{};
      j.in = ws + in;
      j.pre = reinterpret_cast<const float2*>(ws + pre);
      j.H = reinterpret_cast<const float2*>(ws + H);
      j.post = reinterpret_cast<const float2*>(ws + post);
      j.iscale = 1.f;
      j.n_rows = n_rows;
      j.n_in = n_in;
      j.n_out = n_out;
      j.in_ld = in_ld;
      j.mode = sfd::kUsePost | mode;
      j.partial = reinterpret_cast<double*>(ws + partial);
      return j;
    };
    // R4: A^H g onto the hologram grid; S5 = sum conj(v) (x0^2 + y0^2) u0.
    sfd::RowJob r4 = row(B.wa, ldo, B.prexa, B.hxa, B.postxa, h.ny, w.out.nx, h.nx, sfd::kOutField, B.p5);
    r4.out = B.vbuf ? static_cast<void*>(ws + B.vbuf)
                    : static_cast<void*>(static_cast<char*>(grad_in) + (size_t)w.holo * holo_stride);
    r4.out_ld = h.nx;
    if (want_z) {
      r4.mode |= sfd::kReduce | sfd::kRedSwap | (real_in ? sfd::kRedRealRef : 0);
      r4.uref = reinterpret_cast<const float2*>(u0);
      r4.red_ld = h.nx;
      r4.xp = fx.p0;
      r4.xa = fx.a0;
      r4.yp = fy.p0;
      r4.ya = fy.a0;
      r4.wc[0][2] = 1.0;
    }
    rows.push_back({L.lx, r4});
    if (want_z) {
      auto gset = [&](sfd::RowJob& j) {
        j.red_ld = w.out.nx;
        j.xp = fx.p1;
        j.xa = fx.a1;
        j.yp = fy.p1;
        j.ya = fy.a1;
        if (from_i) {
          j.giref = static_cast<const float*>(grad_out[v]);
          j.uref = static_cast<const float2*>(field_out[v]);
        } else {
          j.gref = static_cast<const float2*>(grad_out[v]);
        }
      };
      // S1 (weight 1) and S2 (weight x1^2 + y1^2): from the caller's field
      // u1 when it is given (no transform), else from R1, u1 recomputed.
      if (from_i) {
        sfd::SumJob sj{};
        sj.gi = static_cast<const float*>(grad_out[v]);
        sj.u = static_cast<const float2*>(field_out[v]);
        sj.partial = reinterpret_cast<double*>(ws + B.p12);
        sj.nx = w.out.nx;
        sj.ny = w.out.ny;
        sj.ld = w.out.nx;
        sj.nblocks = std::min(64, B.nt_r);
        sj.xp = fx.p1;
        sj.xa = fx.a1;
        sj.yp = fy.p1;
        sj.ya = fy.a1;
        sums.push_back(sj);
      } else {
        sfd::RowJob r1 = row(B.wf, ldh, B.prexf, B.hxf, B.postxf, w.out.ny, h.nx, w.out.nx, sfd::kReduce, B.p12);
        gset(r1);
        r1.wc[0][3] = 1.0;
        r1.wc[1][2] = 1.0;
        rows.push_back({L.lx, r1});
      }
      // R2: A(x0 u0); S3 (weight x1).
      sfd::RowJob r2 = row(B.wf, ldh, B.prexm, B.hxf, B.postxf, w.out.ny, h.nx, w.out.nx, sfd::kReduce, B.p3);
      gset(r2);
      r2.wc[0][0] = 1.0;
      rows.push_back({L.lx, r2});
      // R3: A(y0 u0); S4 (weight y1).
      sfd::RowJob r3 = row(B.wm, ldh, B.prexf, B.hxf, B.postxf, w.out.ny, h.nx, w.out.nx, sfd::kReduce, B.p4);
      gset(r3);
      r3.wc[0][1] = 1.0;
      rows.push_back({L.lx, r3});
    }
  }
  auto by_len = [](const std::pair<int, sfd::RowJob>& a, const std::pair<int, sfd::RowJob>& b) {
    return a.first < b.first;
  };
  std::stable_sort(cols.begin(), cols.end(), by_len);
  std::stable_sort(rows.begin(), rows.end(), by_len);
  for (auto& c : cols) {
    D.rows.push_back(c.second);
    D.row_L.push_back(c.first);
  }
  D.n_pass_x = (int)cols.size();
  for (auto& r : rows) {
    D.rows.push_back(r.second);
    D.row_L.push_back(r.first);
  }

  // z-derivative and gather jobs, and the gather source lists.
  std::vector<sfd::GradZJob> gz;
  if (want_z)
    for (int v = 0; v < V; ++v) {
      const sfd_plan_s::BwdLayout& B = P->blay[v];
      sfd::GradZJob j{};
      j.p12 = reinterpret_cast<const double*>(ws + B.p12);
      j.p3 = reinterpret_cast<const double*>(ws + B.p3);
      j.p4 = reinterpret_cast<const double*>(ws + B.p4);
      j.p5 = reinterpret_cast<const double*>(ws + B.p5);
      j.n12 = j.n3 = j.n4 = B.nt_r;
      if (from_i) j.n12 = std::min(64, B.nt_r);
      j.n5 = B.nt_a;
      j.k = k;
      j.z = z_or_null ? z_or_null[v] : P->views[v].z;
      j.lam = P->lam;
      j.out = grad_z + v;
      gz.push_back(j);
    }

  // Image: axis | twiddles | tiles | rows | gradz | gather | gather sources.
  std::vector<unsigned char> img;
  size_t o_axis = 0, o_tw = align_up(sizeof(sfd::AxisJob) * 6 * V);
  size_t o_tiles = o_tw + align_up(sizeof(sfd::TwiddleJob) * 2 * P->lengths.size());
  size_t o_rows = o_tiles + align_up(sizeof(sfd::TileJob) * (P->tiles.size() + V));
  size_t o_gz = o_rows + align_up(sizeof(sfd::RowJob) * 7 * V);
  size_t o_ga = o_gz + align_up(sizeof(sfd::GradZJob) * V);
  size_t o_src = o_ga + align_up(sizeof(sfd::GatherJob) * P->n_holo);
  size_t o_sum = o_src + align_up(sizeof(void*) * V);
  const size_t total = o_sum + sizeof(sfd::SumJob) * sums.size();
  if (total > P->bwd_desc_bytes) return fail(SFD_ERR_INTERNAL, "backward descriptor area too small");
  char* dbase = ws + P->bwd_desc_off;
  std::vector<sfd::GatherJob> ga;
  std::vector<const float2*> srcs;
  for (int hh = 0; hh < P->n_holo; ++hh) {
    if (P->holo_views[hh] == 1 && !real_in) continue;  // written directly by its view's adjoint pass
    sfd::GatherJob j{};
    j.real_out = real_in ? 1 : 0;
    j.src = reinterpret_cast<const float2* const*>(dbase + o_src) + srcs.size();
    j.dst = reinterpret_cast<float2*>(static_cast<char*>(grad_in) + (size_t)hh * holo_stride);
    j.n = h.nx * h.ny;
    for (int v = 0; v < V; ++v)
      if (P->views[v].holo == hh) srcs.push_back(reinterpret_cast<const float2*>(ws + P->blay[v].vbuf));
    j.nsrc = (int)srcs.size() - (int)(j.src - reinterpret_cast<const float2* const*>(dbase + o_src));
    ga.push_back(j);
  }
  img.assign(total, 0);
  std::memcpy(img.data() + o_axis, D.axis.data(), sizeof(sfd::AxisJob) * D.axis.size());
  std::memcpy(img.data() + o_tw, D.tw.data(), sizeof(sfd::TwiddleJob) * D.tw.size());
  std::memcpy(img.data() + o_tiles, D.tiles.data(), sizeof(sfd::TileJob) * D.tiles.size());
  std::memcpy(img.data() + o_rows, D.rows.data(), sizeof(sfd::RowJob) * D.rows.size());
  if (!gz.empty()) std::memcpy(img.data() + o_gz, gz.data(), sizeof(sfd::GradZJob) * gz.size());
  if (!ga.empty()) std::memcpy(img.data() + o_ga, ga.data(), sizeof(sfd::GatherJob) * ga.size());
  if (!srcs.empty()) std::memcpy(img.data() + o_src, srcs.data(), sizeof(void*) * srcs.size());
  if (!sums.empty()) std::memcpy(img.data() + o_sum, sums.data(), sizeof(sfd::SumJob) * sums.size());
  sfd_status st = upload(P, 1, img, ws, P->bwd_desc_off, stream);
  if (st != SFD_OK) return st;
  const auto* d_axis = reinterpret_cast<const sfd::AxisJob*>(dbase + o_axis);
  const auto* d_tw = reinterpret_cast<const sfd::TwiddleJob*>(dbase + o_tw);
  const auto* d_tiles = reinterpret_cast<const sfd::TileJob*>(dbase + o_tiles);
  const auto* d_rows = reinterpret_cast<const sfd::RowJob*>(dbase + o_rows);

  if (P->tw_ready_ws != ws) {
    if ((st = launch_setup_for(P, D, ws, d_axis, d_tw, d_tiles, 0, 0, true, 0, 0, stream)) != SFD_OK) return st;
    P->tw_ready_ws = ws;
  }
  if ((st = launch_setup_for(P, D, ws, d_axis, d_tw, d_tiles, 0, (int)D.axis.size(), false, 0, (int)D.tiles.size(),
                             stream, n_spec)) != SFD_OK)
    return st;
  (void)gtile0;
  if ((st = launch_rows(D, d_rows, 0, D.n_pass_x, P, ws, stream, SFD_KERNEL_PASS_Y)) != SFD_OK) return st;
  if ((st = launch_rows(D, d_rows, D.n_pass_x, (int)D.rows.size() - D.n_pass_x, P, ws, stream,
                        SFD_KERNEL_PASS_X)) != SFD_OK)
    return st;
  if (!sums.empty())
    SFD_TIMED(P, SFD_KERNEL_OTHER, stream,
              sfd::launch_sums(reinterpret_cast<const sfd::SumJob*>(dbase + o_sum), (int)sums.size(), 64, stream));
  if (want_z)
    SFD_TIMED(P, SFD_KERNEL_OTHER, stream,
              sfd::launch_gradz(reinterpret_cast<const sfd::GradZJob*>(dbase + o_gz), V, stream));
  if (!ga.empty())
    SFD_TIMED(P, SFD_KERNEL_OTHER, stream,
              sfd::launch_gather(reinterpret_cast<const sfd::GatherJob*>(dbase + o_ga), (int)ga.size(),
                                 h.nx * h.ny, stream));
  return SFD_OK;
}

}  // namespace

extern "C" {

const char* sfd_last_error(void) { return g_err.c_str(); }

sfd_status sfd_plan(sfd_plan_t* plan, double wavelength, const sfd_grid* holo_grid, int32_t n_holo,
                    const sfd_view* views, int32_t n_views, uint32_t flags) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan output pointer is NULL");
  *plan = nullptr;
  if (!finite_pos(wavelength)) return fail(SFD_ERR_INVALID_ARG, "wavelength must be finite and > 0");
  if (!holo_grid) return fail(SFD_ERR_INVALID_ARG, "holo_grid is NULL");
  std::string why;
  if (!grid_ok(*holo_grid, &why, "holo_grid")) return fail(SFD_ERR_INVALID_ARG, why);
  if (n_holo < 1) return fail(SFD_ERR_INVALID_ARG, "n_holo must be >= 1");
  if (!views) return fail(SFD_ERR_INVALID_ARG, "views is NULL");
  if (n_views < 1) return fail(SFD_ERR_INVALID_ARG, "n_views must be >= 1");
  if (n_views > 65536) return fail(SFD_ERR_UNSUPPORTED, "at most 65536 views per plan");
  const uint32_t known = SFD_IN_REAL_F32 | SFD_IN_C64 | SFD_OUT_INTENSITY | SFD_OUT_FIELD | SFD_PHASE_FP32 |
                         SFD_PER_VIEW_LAUNCH | SFD_EAGER | SFD_REUSE_TABLES | SFD_WITH_BACKWARD;
  if (flags & ~known) return fail(SFD_ERR_INVALID_ARG, "unknown flag bits");
  if (((flags & SFD_IN_REAL_F32) != 0) == ((flags & SFD_IN_C64) != 0))
    return fail(SFD_ERR_INVALID_ARG, "exactly one of SFD_IN_REAL_F32 and SFD_IN_C64 must be set");
  if ((flags & (SFD_OUT_INTENSITY | SFD_OUT_FIELD)) == 0)
    return fail(SFD_ERR_INVALID_ARG, "at least one of SFD_OUT_INTENSITY and SFD_OUT_FIELD must be set");
  const sfd_grid& h = *holo_grid;
  if ((long)h.nx * h.ny > (1L << 28)) return fail(SFD_ERR_UNSUPPORTED, "hologram larger than 2^28 samples");
  for (int v = 0; v < n_views; ++v) {
    const sfd_view& w = views[v];
    const std::string name = "views[" + std::to_string(v) + "]";
    if (!grid_ok(w.out, &why, name.c_str())) return fail(SFD_ERR_INVALID_ARG, why);
    if (!std::isfinite(w.z) || w.z == 0.0) return fail(SFD_ERR_INVALID_ARG, name + ".z must be finite and non-zero");
    if (w.holo < 0 || w.holo >= n_holo) return fail(SFD_ERR_INVALID_ARG, name + ".holo out of range");
    if (choose_length(h.nx, w.out.nx) < 0 || choose_length(h.ny, w.out.ny) < 0)
      return fail(SFD_ERR_UNSUPPORTED, name + ": N0 + N1 - 1 exceeds 8192 on an axis");
  }

  auto* P = new (std::nothrow) sfd_plan_s;
  if (!P) return fail(SFD_ERR_INTERNAL, "out of host memory");
  P->lam = wavelength;
  P->holo = h;
  P->n_holo = n_holo;
  P->views.assign(views, views + n_views);
  P->flags = flags;
  const bool field = (flags & SFD_OUT_FIELD) != 0;

  // Padded lengths of both length policies (smooth lengths where they are
  // shorter, or powers of two only): the workspace holds the twiddle tables
  // of both, and every per-view array is sized for the longer choice, so the
  // schedule can switch policies on the same workspace.
  std::vector<int> ls;
  for (int v = 0; v < n_views; ++v)
    for (int smooth : {0, kSmoothAll}) {
      ls.push_back(choose_length(h.nx, views[v].out.nx, smooth));
      ls.push_back(choose_length(h.ny, views[v].out.ny, smooth));
    }
  std::sort(ls.begin(), ls.end());
  ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
  P->lengths = ls;

  // Column-major copies: one per hologram a view reads.
  const size_t in_elem = (flags & SFD_IN_REAL_F32) ? sizeof(float) : sizeof(float2);
  P->lay.resize(n_views);
  std::vector<int> copy_of(n_holo, -1);
  for (int v = 0; v < n_views; ++v) {
    const int hv = views[v].holo;
    if (copy_of[hv] < 0) {
      copy_of[hv] = (int)P->tiles.size();
      P->tiles.push_back(TileLayout{hv, 0});
    }
    P->lay[v].tile = copy_of[hv];
  }

  size_t off = 0;
  P->desc_off = off;
  P->desc_bytes = desc_capacity(n_views, (int)ls.size(), (int)P->tiles.size());
  off += P->desc_bytes;
  P->desc_off2 = off;
  off += P->desc_bytes;
  for (TileLayout& T : P->tiles) {
    T.off = off;
    off += align_up((size_t)h.nx * col_ld(h.ny) * in_elem);
  }
  for (int L : ls) {
    P->tw_off[L] = off;
    off += align_up(sizeof(float2) * std::max(1, sfd::twiddle_len(L, false)));
    P->tws_off[L] = off;
    off += align_up(sizeof(float2) * std::max(1, sfd::twiddle_len(L, true)));
  }
  for (int v = 0; v < n_views; ++v) {
    ViewLayout& L = P->lay[v];
    const sfd_grid& o = views[v].out;
    L.lx = choose_length(h.nx, o.nx);
    L.ly = choose_length(h.ny, o.ny);
    const int lx2 = choose_length(h.nx, o.nx, false), ly2 = choose_length(h.ny, o.ny, false);
    auto take = [&](size_t bytes) {
      const size_t at = off;
      off += align_up(bytes);
      return at;
    };
    L.prex = take(sizeof(float2) * h.nx);
    L.prey = take(sizeof(float2) * h.ny);
    if (field) {
      L.postx = take(sizeof(float2) * o.nx);
      L.posty = take(sizeof(float2) * o.ny);
    }
    L.hx = take(sizeof(float2) * lx2);
    L.hy = take(sizeof(float2) * ly2);
    L.inter = take(sizeof(float2) * (size_t)o.ny * inter_ld(h.nx));  // N1y x N0x after the y transforms
  }
  // Persistent launch: its counters, when any length policy allows it.
  {
    bool ok_any = false;
    for (int mask = 0; mask <= kSmoothAll; ++mask) {
      set_lengths(P, mask);
      ok_any = ok_any || persist_eligible(P);
    }
    set_lengths(P, kSmoothDefault);
    P->persist_ok = persist_eligible(P);
    P->persist = P->persist_ok;
    if (ok_any) {
      // Strips of the column-major copy for complex holograms only: the
      // column tiles read real holograms in place.
      P->nstrips = (flags & SFD_IN_C64) ? (int)P->tiles.size() * ((h.nx + sfd::kStripW - 1) / sfd::kStripW) : 0;
      P->col_tiles = (h.nx + sfd::kStripW - 1) / sfd::kStripW;
      P->sync_words = sfd::persist_sync_words(n_views, P->nstrips);
      P->sync_off = off;
      off += align_up(sizeof(uint32_t) * P->sync_words);
    }
  }
  if (flags & (SFD_IN_C64 | SFD_WITH_BACKWARD)) {
    // Backward: per view its own forward, moment and adjoint tables, the
    // gradient's column tiles, three intermediates, an adjoint buffer when
    // the hologram has several views, and the reduction partials.
    auto take = [&](size_t bytes) {
      const size_t at = off;
      off += align_up(bytes);
      return at;
    };
    P->holo_views.assign(n_holo, 0);
    for (int v = 0; v < n_views; ++v) P->holo_views[views[v].holo]++;
    P->bwd_desc_off = off;
    P->bwd_desc_bytes = bwd_desc_capacity(n_views, n_holo, (int)ls.size(), (int)P->tiles.size());
    off += P->bwd_desc_bytes;
    P->blay.resize(n_views);
    const size_t c8 = sizeof(float2);
    for (int v = 0; v < n_views; ++v) {
      sfd_plan_s::BwdLayout& B = P->blay[v];
      const sfd_grid& o = views[v].out;
      // Sized for the longer (power-of-two) length choice.
      const int lx = choose_length(h.nx, o.nx, false), ly = choose_length(h.ny, o.ny, false);
      B.prexf = take(c8 * h.nx);
      B.preyf = take(c8 * h.ny);
      B.postxf = take(c8 * o.nx);
      B.postyf = take(c8 * o.ny);
      B.prexm = take(c8 * h.nx);
      B.preym = take(c8 * h.ny);
      B.prexa = take(c8 * o.nx);
      B.preya = take(c8 * o.ny);
      B.postxa = take(c8 * h.nx);
      B.postya = take(c8 * h.ny);
      B.hxf = take(c8 * lx);
      B.hyf = take(c8 * ly);
      B.hxa = take(c8 * lx);
      B.hya = take(c8 * ly);
      B.gtile = take(c8 * (size_t)o.nx * col_ld(o.ny));
      B.wf = take(c8 * (size_t)o.ny * inter_ld(h.nx));
      B.wm = take(c8 * (size_t)o.ny * inter_ld(h.nx));
      B.wa = take(c8 * (size_t)h.ny * inter_ld(o.nx));
      // Adjoint buffer: several views sum into a hologram's gradient, and a
      // real hologram's gradient is the real part of the complex adjoint.
      B.vbuf = (P->holo_views[views[v].holo] > 1 || !(flags & SFD_IN_C64)) ? take(c8 * (size_t)h.nx * h.ny) : 0;
      // Partials: room for the most row-pass tiles any schedule launches.
      const int gmin = std::min(min_tile_width(lx, false), min_tile_width(choose_length(h.nx, o.nx), false));
      B.nt_r = (o.ny + gmin - 1) / gmin;
      B.nt_a = (h.ny + gmin - 1) / gmin;
      B.p12 = take(4 * sizeof(double) * B.nt_r);
      B.p3 = take(4 * sizeof(double) * B.nt_r);
      B.p4 = take(4 * sizeof(double) * B.nt_r);
      B.p5 = take(4 * sizeof(double) * B.nt_a);
    }
  }
  P->ws_bytes = off;
  // Start from the tuning table for these shapes, if an earlier autotune filled it.
  {
    std::string sig = std::to_string(h.nx) + "x" + std::to_string(h.ny) + "/" + std::to_string(n_holo) + "/" +
                      std::to_string(flags & ~(uint32_t)SFD_EAGER);
    for (int v = 0; v < n_views; ++v)
      sig += ";" + std::to_string(views[v].out.nx) + "x" + std::to_string(views[v].out.ny) + "@" +
             std::to_string(views[v].holo);
    P->shape_sig = sig;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tuned.find(std::make_tuple(2, 0, sig)) == g_tuned.end()) load_cached(sig);
    for (int L : ls)
      for (int col = 0; col < 2; ++col) {
        const auto it = g_tuned.find(std::make_tuple(col, L, sig));
        if (it != g_tuned.end()) (col ? P->gcol : P->grow)[L] = it->second;
      }
    const auto il = g_tuned.find(std::make_tuple(3, 0, sig));
    if (il != g_tuned.end() && il->second != P->smooth) {
      set_lengths(P, il->second);
      P->persist_ok = persist_eligible(P);
      P->persist = P->persist_ok;
    }
    const auto it = g_tuned.find(std::make_tuple(2, 0, sig));
    if (it != g_tuned.end()) P->persist = P->persist_ok && it->second != 0;
  }
  apply_schedule(P);
  *plan = P;
  return SFD_OK;
}

sfd_status sfd_workspace_size(sfd_plan_t plan, size_t* bytes) {
  g_err.clear();
  if (!plan || !bytes) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->ws_bytes;
  return SFD_OK;
}

sfd_status sfd_view_lengths(sfd_plan_t plan, int32_t v, int32_t* lx, int32_t* ly) {
  g_err.clear();
  if (!plan || !lx || !ly) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  if (v < 0 || v >= (int)plan->views.size()) return fail(SFD_ERR_INVALID_ARG, "view index out of range");
  *lx = plan->lay[v].lx;
  *ly = plan->lay[v].ly;
  return SFD_OK;
}

}  // extern "C"

sfd_status sfd::set_error(sfd_status s, const char* msg) { return fail(s, msg); }

sfd_status sfd::reconstruct_impl(sfd_plan_s* plan, const void* holo, const double* z_or_null, void* const* out,
                                 void* workspace, size_t ws_bytes, hipStream_t stream, bool no_alloc) {
  sfd_status st = check_common(plan, workspace, ws_bytes);
  if (st != SFD_OK) return st;
  if (!holo) return fail(SFD_ERR_INVALID_ARG, "holo is NULL");
  if (reinterpret_cast<uintptr_t>(holo) % 16) return fail(SFD_ERR_INVALID_ARG, "holo must be 16-byte aligned");
  if (!out) return fail(SFD_ERR_INVALID_ARG, "out is NULL");
  const int V = (int)plan->views.size();
  const int n_out = ((plan->flags & SFD_OUT_FIELD) && (plan->flags & SFD_OUT_INTENSITY)) ? 2 * V : V;
  for (int v = 0; v < n_out; ++v) {
    if (!out[v]) return fail(SFD_ERR_INVALID_ARG, "out[" + std::to_string(v) + "] is NULL");
    if (reinterpret_cast<uintptr_t>(out[v]) % 16)
      return fail(SFD_ERR_INVALID_ARG, "out[" + std::to_string(v) + "] must be 16-byte aligned");
  }
  if ((st = check_z(plan, z_or_null)) != SFD_OK) return st;

  char* ws = static_cast<char*>(workspace);
  if (no_alloc) {
    // The scratch array is shared by every plan: state cached for it (twiddle
    // tables, zeroed counters, descriptors, kept tables) is valid only if this
    // plan used it last.
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    uint64_t& owner = g_scratch_owner[workspace];
    if (owner != plan->serial) {
      if (plan->tw_ready_ws == ws) plan->tw_ready_ws = nullptr;
      if (plan->sync_ready_ws == ws) plan->sync_ready_ws = nullptr;
      if (plan->tables_ws == ws) plan->tables_ws = nullptr;
      for (auto& lw : plan->last_ws)
        if (lw == ws) lw = nullptr;
      owner = plan->serial;
    }
  }
  // SFD_REUSE_TABLES: this call needs no tables or spectra when the
  // workspace holds those of the same distances.
  bool tables = true;
  if ((plan->flags & SFD_REUSE_TABLES) && !(plan->flags & SFD_PER_VIEW_LAUNCH)) {
    std::vector<double> zz(V);
    for (int v = 0; v < V; ++v) zz[v] = z_or_null ? z_or_null[v] : plan->views[v].z;
    tables = !(plan->tables_ws == ws && plan->tables_z == zz);
    plan->tables_ws = nullptr;  // set again once this call's launches are enqueued
    plan->tables_z = std::move(zz);
  }
  CallDescs D;
  if ((st = build_descs(plan, holo, z_or_null, out, ws, &D)) != SFD_OK) return st;
  std::vector<unsigned char> img0, img;
  size_t off_axis, off_tw, off_rows, off_tiles;
  pack_descs(plan, D, &img0, &off_axis, &off_tw, &off_rows, &off_tiles);
  if (plan->persist && plan->persist_grid <= 0) {
    plan->persist_grid = sfd::persist_resident_blocks();
    if (plan->persist_grid <= 0) return fail(SFD_ERR_HIP, "occupancy query of the persistent kernel failed");
  }
  // Forward descriptor slot s (0, 1) at its offset, remembered as image idx.
  auto slot_off = [&](int s) { return s == 0 ? plan->desc_off : plan->desc_off2; };
  auto slot_idx = [](int s) { return s == 0 ? 0 : 2; };
  auto make = [&](int s) {
    img = img0;
    if (plan->persist) pack_persist(plan, &D, ws, tables, &img, off_axis, off_tiles, off_rows, slot_off(s));
  };
  int slot = 0;
  if (no_alloc) {
    // Slot 0, written by kernel-argument copies instead of the pinned staging
    // buffer (which the first upload would allocate).
    make(0);
    if (!(plan->last_ws[0] == ws && plan->last_desc[0] == img)) {
      img.resize((img.size() + 3) / 4 * 4, 0);
      SFD_HIP_TRY(sfd::launch_blit(ws + plan->desc_off, img.data(), img.size(), stream));
      plan->last_desc[0] = img;
      plan->last_ws[0] = ws;
    }
  } else {
    // The last call's slot if its image is still there, else the other slot
    // if its image is, else the other slot gets this image (so that two
    // alternating images both stay resident).
    const int cand[2] = {plan->fwd_slot, 1 - plan->fwd_slot};
    bool found = false;
    for (int c : cand) {
      make(c);
      slot = c;
      if (plan->last_ws[slot_idx(c)] == ws && plan->last_desc[slot_idx(c)] == img) {
        found = true;
        break;
      }
    }
    if (!found && (st = upload(plan, slot_idx(slot), img, ws, slot_off(slot), stream)) != SFD_OK) return st;
    plan->fwd_slot = slot;
  }
  const size_t sb = slot_off(slot);
  const auto* d_axis = reinterpret_cast<const sfd::AxisJob*>(ws + sb + off_axis);
  const auto* d_tw = reinterpret_cast<const sfd::TwiddleJob*>(ws + sb + off_tw);
  const auto* d_rows = reinterpret_cast<const sfd::RowJob*>(ws + sb + off_rows);
  const auto* d_tiles = reinterpret_cast<const sfd::TileJob*>(ws + sb + off_tiles);

  // The twiddle tables depend only on the transform shapes: built once per
  // workspace (which stays dedicated to the plan).  The persistent launch's
  // counters are zeroed once per workspace; every launch leaves them zero.
  if (plan->tw_ready_ws != ws) {
    if ((st = launch_setup_for(plan, D, ws, d_axis, d_tw, d_tiles, 0, 0, true, 0, 0, stream)) != SFD_OK) return st;
    plan->tw_ready_ws = ws;
  }
  if (plan->persist_ok && plan->sync_ready_ws != ws) {
    SFD_HIP_TRY(sfd::launch_zero(reinterpret_cast<uint32_t*>(ws + plan->sync_off), plan->sync_words, stream));
    plan->sync_ready_ws = ws;
  }
  if (plan->flags & SFD_PER_VIEW_LAUNCH) {
    // Baseline: every stage launched for one view at a time (axis jobs stay
    // in view order: 2v = x, 2v + 1 = y).
    for (int v = 0; v < V; ++v) {
      if ((st = launch_setup_for(plan, D, ws, d_axis, d_tw, d_tiles, 2 * v, 2, false, plan->lay[v].tile, 1,
                                 stream)) !=
          SFD_OK)
        return st;
      if ((st = launch_rows(D, d_rows, v, 1, plan, ws, stream, SFD_KERNEL_PASS_Y)) != SFD_OK) return st;
      if ((st = launch_rows(D, d_rows, D.n_pass_x + v, 1, plan, ws, stream, SFD_KERNEL_PASS_X)) != SFD_OK)
        return st;
    }
    return SFD_OK;
  }
  // The persistent schedule is one kernel: it is launched directly (a graph
  // replay of that one node measured about 10 us slower per call than the
  // launch itself).  The pass schedule replays its recorded launches.
  const bool use_graph = !(plan->flags & SFD_EAGER) && !plan->profiling && !no_alloc && !plan->persist;
  if (use_graph) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SFD_HIP_TRY(hipStreamIsCapturing(stream, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      if (plan->graph_ws != ws) plan->drop_graph();
      hipGraph_t& graph = plan->graph[tables ? 0 : 1][slot];
      hipGraphExec_t& gexec = plan->gexec[tables ? 0 : 1][slot];
      if (!gexec) {
        // Record on a private stream: the caller's stream is never put in
        // capture mode.
        if (!plan->cap_stream) SFD_HIP_TRY(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
        SFD_HIP_TRY(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
        st = launch_forward(plan, D, ws, d_axis, d_tw, d_tiles, d_rows, plan->cap_stream, tables);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(plan->cap_stream, &g);
        if (st != SFD_OK || e != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return st != SFD_OK ? st : fail(SFD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        graph = g;
        SFD_HIP_TRY(hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0));
        plan->graph_ws = ws;
      }
      SFD_HIP_TRY(hipGraphLaunch(gexec, stream));
      if (plan->flags & SFD_REUSE_TABLES) plan->tables_ws = ws;
      return SFD_OK;
    }
  }
  st = launch_forward(plan, D, ws, d_axis, d_tw, d_tiles, d_rows, stream, tables);
  if (st == SFD_OK && (plan->flags & SFD_REUSE_TABLES)) plan->tables_ws = ws;
  return st;
}

extern "C" {

sfd_status sfd_reconstruct(sfd_plan_t plan, const void* holo, const double* z_or_null, void* const* out,
                           void* workspace, size_t ws_bytes, hipStream_t stream) {
  g_err.clear();
  return sfd::reconstruct_impl(plan, holo, z_or_null, out, workspace, ws_bytes, stream, false);
}

sfd_status sfd_backward(sfd_plan_t plan, void* const* grad_out, void* const* field_out, const void* holo,
                        const double* z_or_null, void* grad_in, double* grad_z, void* workspace,
                        size_t ws_bytes, hipStream_t stream) {
  g_err.clear();
  sfd_status st = check_common(plan, workspace, ws_bytes);
  if (st != SFD_OK) return st;
  if (!(plan->flags & (SFD_IN_C64 | SFD_WITH_BACKWARD)))
    return fail(SFD_ERR_INVALID_ARG, "sfd_backward needs a plan made with SFD_IN_C64 or SFD_WITH_BACKWARD");
  if (plan->raw_nx > 0) return fail(SFD_ERR_INVALID_ARG, "sfd_backward does not take raw camera frames");
  if (!grad_out) return fail(SFD_ERR_INVALID_ARG, "grad_out is NULL");
  if (!holo || reinterpret_cast<uintptr_t>(holo) % 16)
    return fail(SFD_ERR_INVALID_ARG, "holo must be a non-NULL 16-byte aligned device pointer");
  if (!grad_in || reinterpret_cast<uintptr_t>(grad_in) % 16)
    return fail(SFD_ERR_INVALID_ARG, "grad_in must be a non-NULL 16-byte aligned device pointer");
  if (grad_z && reinterpret_cast<uintptr_t>(grad_z) % 8)
    return fail(SFD_ERR_INVALID_ARG, "grad_z must be 8-byte aligned");
  const int V = (int)plan->views.size();
  for (int v = 0; v < V; ++v) {
    if (!grad_out[v] || reinterpret_cast<uintptr_t>(grad_out[v]) % 16)
      return fail(SFD_ERR_INVALID_ARG, "grad_out[" + std::to_string(v) + "] must be non-NULL and 16-byte aligned");
    if (field_out && (!field_out[v] || reinterpret_cast<uintptr_t>(field_out[v]) % 16))
      return fail(SFD_ERR_INVALID_ARG, "field_out[" + std::to_string(v) + "] must be non-NULL and 16-byte aligned");
  }
  if ((st = check_z(plan, z_or_null)) != SFD_OK) return st;
  plan->tables_ws = nullptr;  // the backward rewrites the workspace's tables
  return run_backward(plan, grad_out, field_out, holo, z_or_null, grad_in, grad_z, static_cast<char*>(workspace),
                      stream);
}

sfd_status sfd_autotune(sfd_plan_t plan, const void* holo, void* const* out, void* workspace, size_t ws_bytes,
                        int32_t reps, hipStream_t stream) {
  g_err.clear();
  sfd_status st = check_common(plan, workspace, ws_bytes);
  if (st != SFD_OK) return st;
  if (reps < 1 || reps > 1000) return fail(SFD_ERR_INVALID_ARG, "reps must be in [1, 1000]");
  if (plan->profiling) return fail(SFD_ERR_INVALID_ARG, "turn kernel timing off before autotuning");
  // Candidates run the way the plan runs its calls (graph replays unless
  // the plan is eager or launches per view): the launch gaps between the
  // kernels are part of what a tile width changes.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct EventGuard {
    hipEvent_t* a;
    hipEvent_t* b;
    ~EventGuard() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } eguard{&e0, &e1};
  SFD_HIP_TRY(hipEventCreate(&e0));
  SFD_HIP_TRY(hipEventCreate(&e1));
  auto timed = [&](float* ms) -> sfd_status {
    sfd_status s2 = sfd_reconstruct(plan, holo, nullptr, out, workspace, ws_bytes, stream);  // warm-up
    if (s2 != SFD_OK) return s2;
    SFD_HIP_TRY(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r)
      if ((s2 = sfd_reconstruct(plan, holo, nullptr, out, workspace, ws_bytes, stream)) != SFD_OK) return s2;
    SFD_HIP_TRY(hipEventRecord(e1, stream));
    SFD_HIP_TRY(hipEventSynchronize(e1));
    SFD_HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    return SFD_OK;
  };
  // Tile widths are tuned on the passes' schedule.
  const bool was_persist = plan->persist;
  if (was_persist && (st = sfd_set_launch(plan, SFD_LAUNCH_PASSES)) != SFD_OK) return st;
  std::vector<std::pair<int, int>> passes;  // (col, L)
  for (const ViewLayout& v : plan->lay) {
    passes.push_back({1, v.ly});
    passes.push_back({0, v.lx});
  }
  std::sort(passes.begin(), passes.end());
  passes.erase(std::unique(passes.begin(), passes.end()), passes.end());
  // Two sweeps over the passes: a pass's best width can depend on the
  // others'.
  const size_t n_passes = passes.size();
  for (size_t k = 0; k < n_passes; ++k) passes.push_back(passes[k]);
  for (const auto& pl : passes) {
    const int col = pl.first, L = pl.second;
    int widths[16];
    const int n = std::min(sfd::pass_tile_widths(L, col != 0, widths, 16), 16);
    auto& m = col ? plan->gcol : plan->grow;
    int best = plan->tile_g(L, col != 0);
    float best_ms = 0.f;
    for (int i = 0; i < n; ++i) {
      m[L] = widths[i];
      apply_schedule(plan);
      float ms = 0.f;
      if ((st = timed(&ms)) != SFD_OK) {
        m[L] = best;
        apply_schedule(plan);
        return st;
      }
      if (i == 0 || ms < best_ms) {
        best_ms = ms;
        best = widths[i];
      }
    }
    m[L] = best;
    apply_schedule(plan);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(col, L, plan->shape_sig)] = best;
  }
  if (was_persist || plan->persist_ok) {
    // The passes' schedule is tuned; keep the faster of it and the
    // persistent launch.
    float t_pass = 0.f, t_persist = 0.f;
    if ((st = timed(&t_pass)) != SFD_OK) return st;
    if ((st = sfd_set_launch(plan, SFD_LAUNCH_PERSISTENT)) != SFD_OK) return st;
    if ((st = timed(&t_persist)) != SFD_OK) return st;
    const bool keep = t_persist <= t_pass;
    if (!keep && (st = sfd_set_launch(plan, SFD_LAUNCH_PASSES)) != SFD_OK) return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(2, 0, plan->shape_sig)] = keep ? 1 : 0;
  }
  // Radix choice: each smooth length (1280, 1536, 1792 with their radix-5,
  // -3 and -7 closing stages) is switched on or off in turn where that
  // changes some view's padded length, timed on its default tile widths and,
  // where available, the persistent launch; the faster setting is kept.
  bool tried = false;
  for (int bit = 1; bit <= 4; bit <<= 1) {
    const int other = plan->smooth ^ bit;
    bool differ = false;
    for (size_t v = 0; v < plan->views.size(); ++v) {
      const sfd_grid& o = plan->views[v].out;
      differ = differ || choose_length(plan->holo.nx, o.nx, plan->smooth) != choose_length(plan->holo.nx, o.nx, other) ||
               choose_length(plan->holo.ny, o.ny, plan->smooth) != choose_length(plan->holo.ny, o.ny, other);
    }
    if (!differ) continue;
    tried = true;
    float t_cur = 0.f, t_other = 0.f;
    if ((st = timed(&t_cur)) != SFD_OK) return st;
    const int cur_mask = plan->smooth;
    const bool cur_persist = plan->persist;
    if ((st = sfd_set_length_policy(plan, other)) != SFD_OK) return st;
    if (plan->persist_ok && (st = sfd_set_launch(plan, SFD_LAUNCH_PERSISTENT)) != SFD_OK) return st;
    if ((st = timed(&t_other)) != SFD_OK) return st;
    if (t_cur <= t_other) {
      if ((st = sfd_set_length_policy(plan, cur_mask)) != SFD_OK) return st;
      if ((st = sfd_set_launch(plan, cur_persist ? SFD_LAUNCH_PERSISTENT : SFD_LAUNCH_PASSES)) != SFD_OK) return st;
    }
  }
  if (tried) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(3, 0, plan->shape_sig)] = plan->smooth;
    g_tuned[std::make_tuple(2, 0, plan->shape_sig)] = plan->persist ? 1 : 0;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(2, 0, plan->shape_sig)] = plan->persist ? 1 : 0;
    store_cached(plan->shape_sig, plan->gcol, plan->grow, plan->persist, plan->smooth);
  }
  return SFD_OK;
}

sfd_status sfd_schedule(sfd_plan_t plan, int32_t L, int32_t col, int32_t* tile_width) {
  g_err.clear();
  if (!plan || !tile_width) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  if (std::find(plan->lengths.begin(), plan->lengths.end(), (int)L) == plan->lengths.end())
    return fail(SFD_ERR_INVALID_ARG, "the plan has no transforms of length " + std::to_string(L));
  *tile_width = plan->tile_g(L, col != 0);
  return SFD_OK;
}

int32_t sfd_tile_widths(int32_t L, int32_t col, int32_t* widths, int32_t* per_slot, int32_t cap) {
  g_err.clear();
  if (cap < 0 || (cap > 0 && !widths)) {
    fail(SFD_ERR_INVALID_ARG, "sfd_tile_widths: cap < 0, or widths is NULL");
    return -1;
  }
  int w[64], p[64];
  const int n = sfd::pass_tile_widths(L, col != 0, w, 64, p);
  for (int k = 0; k < std::min(n, (int)cap); ++k) {
    widths[k] = w[k];
    if (per_slot) per_slot[k] = p[k];
  }
  return n;
}

sfd_status sfd_set_schedule(sfd_plan_t plan, int32_t L, int32_t col, int32_t tile_width) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  if (std::find(plan->lengths.begin(), plan->lengths.end(), (int)L) == plan->lengths.end())
    return fail(SFD_ERR_INVALID_ARG, "the plan has no transforms of length " + std::to_string(L));
  int widths[16];
  const int n = std::min(sfd::pass_tile_widths(L, col != 0, widths, 16), 16);
  if (std::find(widths, widths + n, (int)tile_width) == widths + n)
    return fail(SFD_ERR_INVALID_ARG, "no " + std::string(col ? "column" : "row") + " pass kernel of tile width " +
                                         std::to_string(tile_width) + " at length " + std::to_string(L));
  (col ? plan->gcol : plan->grow)[L] = tile_width;
  apply_schedule(plan);
  return SFD_OK;
}

sfd_status sfd_set_launch(sfd_plan_t plan, int32_t mode) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  if (mode != SFD_LAUNCH_PASSES && mode != SFD_LAUNCH_PERSISTENT)
    return fail(SFD_ERR_INVALID_ARG, "unknown launch mode " + std::to_string(mode));
  if (mode == SFD_LAUNCH_PERSISTENT && !plan->persist_ok)
    return fail(SFD_ERR_UNSUPPORTED, "the persistent launch is not available for this plan's shapes");
  const bool want = mode == SFD_LAUNCH_PERSISTENT;
  if (want != plan->persist) {
    plan->persist = want;
    plan->drop_graph();
    plan->forget_descs();  // the descriptor layout differs: upload on the next call
  }
  return SFD_OK;
}

sfd_status sfd_set_length_policy(sfd_plan_t plan, int32_t smooth) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  if (smooth < 0 || smooth > kSmoothAll) return fail(SFD_ERR_INVALID_ARG, "length policy must be a mask of bits 0..2");
  if (smooth == plan->smooth) return SFD_OK;
  const bool was_persist = plan->persist;
  set_lengths(plan, smooth);
  plan->persist_ok = persist_eligible(plan);
  plan->persist = was_persist && plan->persist_ok;
  plan->tables_ws = nullptr;     // spectra of other lengths
  plan->forget_descs();
  apply_schedule(plan);          // also drops the recorded graphs
  return SFD_OK;
}

sfd_status sfd_length_policy(sfd_plan_t plan, int32_t* smooth) {
  g_err.clear();
  if (!plan || !smooth) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  *smooth = plan->smooth;
  return SFD_OK;
}

sfd_status sfd_launch_mode(sfd_plan_t plan, int32_t* mode, int32_t* persistent_available) {
  g_err.clear();
  if (!plan || !mode) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  *mode = plan->persist ? SFD_LAUNCH_PERSISTENT : SFD_LAUNCH_PASSES;
  if (persistent_available) *persistent_available = plan->persist_ok ? 1 : 0;
  return SFD_OK;
}

sfd_status sfd_sync_faults(sfd_plan_t plan, void* workspace, size_t ws_bytes, int32_t clear, uint32_t* faults,
                           hipStream_t stream) {
  g_err.clear();
  sfd_status st = check_common(plan, workspace, ws_bytes);
  if (st != SFD_OK) return st;
  if (!faults) return fail(SFD_ERR_INVALID_ARG, "faults is NULL");
  *faults = 0;
  if (!plan->persist_ok || plan->sync_ready_ws != workspace) return SFD_OK;
  uint32_t* w = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + plan->sync_off) +
                sfd::kSyncErr * sfd::kSyncStride;
  SFD_HIP_TRY(hipMemcpyAsync(faults, w, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  SFD_HIP_TRY(hipStreamSynchronize(stream));
  if (clear && *faults) SFD_HIP_TRY(sfd::launch_zero(w, 1, stream));
  return SFD_OK;
}

sfd_status sfd_profile_enable(sfd_plan_t plan, int32_t enable) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  for (auto& r : plan->recs) {
    SFD_HIP_TRY(hipEventSynchronize(r.b));
    plan->event_pool.push_back(r.a);
    plan->event_pool.push_back(r.b);
  }
  plan->recs.clear();
  plan->profiling = enable != 0;
  return SFD_OK;
}

sfd_status sfd_profile_report(sfd_plan_t plan, int32_t kind, int64_t* launches, double* total_ms) {
  g_err.clear();
  if (!plan || !launches || !total_ms) return fail(SFD_ERR_INVALID_ARG, "NULL argument");
  if (kind < 0 || kind >= SFD_KERNEL_KINDS) return fail(SFD_ERR_INVALID_ARG, "unknown kernel kind");
  int64_t n = 0;
  double ms = 0.0;
  for (auto& r : plan->recs) {
    if (r.kind != kind) continue;
    SFD_HIP_TRY(hipEventSynchronize(r.b));
    float t = 0.f;
    SFD_HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return SFD_OK;
}

sfd_status sfd_stream_frame(sfd_plan_t plan, const void* host_frame, void* const* dev_holo, void* const* out,
                            void* workspace, size_t ws_bytes, hipStream_t stream) {
  g_err.clear();
  sfd_status st = check_common(plan, workspace, ws_bytes);
  if (st != SFD_OK) return st;
  if (!host_frame) return fail(SFD_ERR_INVALID_ARG, "host_frame is NULL");
  if (!dev_holo || !dev_holo[0] || !dev_holo[1] || dev_holo[0] == dev_holo[1])
    return fail(SFD_ERR_INVALID_ARG, "dev_holo must hold two distinct device buffers");
  if (plan->flags & SFD_PER_VIEW_LAUNCH)
    return fail(SFD_ERR_INVALID_ARG, "sfd_stream_frame needs a batched plan (no SFD_PER_VIEW_LAUNCH)");
  const sfd_grid& h = plan->holo;
  const size_t bytes = plan->raw_nx > 0 ? (size_t)plan->n_holo * plan->raw_nx * h.ny * (plan->raw_bits / 8)
                                        : (size_t)plan->n_holo * h.nx * h.ny * ((plan->flags & SFD_IN_REAL_F32) ? 4 : 8);
  if (!plan->copy_stream) {
    SFD_HIP_TRY(hipStreamCreateWithFlags(&plan->copy_stream, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      SFD_HIP_TRY(hipEventCreateWithFlags(&plan->copied[b], hipEventDisableTiming));
      SFD_HIP_TRY(hipEventCreateWithFlags(&plan->consumed[b], hipEventDisableTiming));
    }
  }
  const int b = (int)(plan->frames & 1);
  // The copy waits for the reconstruction that last read this buffer (frame
  // k - 2).  The host waits for it too: at most two frames are in flight.
  // Measured: letting the host run further ahead (queues of many frames with
  // their cross-stream waits) made the loop several times slower.
  if (plan->consumed_set[b]) {
    SFD_HIP_TRY(hipEventSynchronize(plan->consumed[b]));
    SFD_HIP_TRY(hipStreamWaitEvent(plan->copy_stream, plan->consumed[b], 0));
  }
  SFD_HIP_TRY(hipMemcpyAsync(dev_holo[b], host_frame, bytes, hipMemcpyHostToDevice, plan->copy_stream));
  SFD_HIP_TRY(hipEventRecord(plan->copied[b], plan->copy_stream));
  SFD_HIP_TRY(hipStreamWaitEvent(stream, plan->copied[b], 0));
  if ((st = sfd_reconstruct(plan, dev_holo[b], nullptr, out, workspace, ws_bytes, stream)) != SFD_OK) return st;
  SFD_HIP_TRY(hipEventRecord(plan->consumed[b], stream));
  plan->consumed_set[b] = true;
  ++plan->frames;
  return SFD_OK;
}

sfd_status sfd_set_raw_input(sfd_plan_t plan, int32_t nx_raw, int32_t sample_bits) {
  g_err.clear();
  if (!plan) return fail(SFD_ERR_INVALID_ARG, "plan is NULL");
  if (!(plan->flags & SFD_IN_REAL_F32)) return fail(SFD_ERR_INVALID_ARG, "raw camera input needs a real-input plan");
  if (nx_raw < 0 || nx_raw > 65536) return fail(SFD_ERR_INVALID_ARG, "nx_raw must be in [0, 65536]");
  if (sample_bits != 8 && sample_bits != 16 && sample_bits != 32)
    return fail(SFD_ERR_INVALID_ARG, "sample_bits must be 8, 16 or 32");
  if ((long)nx_raw * plan->holo.ny > (1L << 28)) return fail(SFD_ERR_UNSUPPORTED, "raw frame larger than 2^28 samples");
  plan->raw_nx = nx_raw;
  plan->raw_bits = nx_raw > 0 ? sample_bits : 32;
  // Camera input has its own tuned schedule (it reads other data).
  const size_t cut = plan->shape_sig.find(";raw");
  if (cut != std::string::npos) plan->shape_sig.erase(cut);
  if (nx_raw > 0) plan->shape_sig += ";raw" + std::to_string(nx_raw) + "/" + std::to_string(plan->raw_bits);
  plan->drop_graph();
  plan->forget_descs();
  return SFD_OK;
}

sfd_status sfd_destroy(sfd_plan_t plan) {
  g_err.clear();
  delete plan;
  return SFD_OK;
}

}  // extern "C"

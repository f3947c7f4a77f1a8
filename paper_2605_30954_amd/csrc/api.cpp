// C ABI entry points: argument checks, launch planning, workspace layout,
// hipGraph capture/replay and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "errors.h"
#include "gpgomea_eval.h"
#include "kernels.h"

namespace gg {
namespace {

constexpr int kMaxSpans = 256;    // forward partial sums per individual (upper bound)
constexpr int kMaxAdjSpans = 256;  // gradient partials per (individual, constant) (upper bound)
constexpr int64_t kAdjPartEntries = int64_t(1) << 26;  // cap on M x C_max x spans (512 MB)
constexpr int kPlainMaxBlocks = 1024;
constexpr int kPlainAdjSpans = 1024;  // spans (blocks) of one plain-form adjoint launch
constexpr size_t kRedoPoolBytes = size_t(4) << 20;  // bad-tile masks (slots of tile_words words)
constexpr uint32_t kKnownFlags =
    GPGOMEA_LINEAR_SCALING | GPGOMEA_FP64_NODES | GPGOMEA_PLAIN | GPGOMEA_NO_GRAPH;

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Shape {
  int M, L_max, C_max, F;
  int64_t N, ldx;
  uint32_t flags;
};

int check_shape(const Shape& s) {
  if (s.flags & ~kKnownFlags) return fail(GPGOMEA_E_ARG, "unknown flag bits 0x%x", s.flags & ~kKnownFlags);
  if (s.M < 1) return fail(GPGOMEA_E_SHAPE, "M=%d must be >= 1", s.M);
  if (s.L_max < 1 || s.L_max > GPGOMEA_MAX_LEN)
    return fail(GPGOMEA_E_SHAPE, "L_max=%d outside [1, %d]", s.L_max, GPGOMEA_MAX_LEN);
  if (s.C_max < 0 || s.C_max > GPGOMEA_MAX_CONSTS)
    return fail(GPGOMEA_E_SHAPE, "C_max=%d outside [0, %d]", s.C_max, GPGOMEA_MAX_CONSTS);
  if (s.F < 1 || s.F > GPGOMEA_MAX_FEATURES)
    return fail(GPGOMEA_E_SHAPE, "F=%d outside [1, %d]", s.F, GPGOMEA_MAX_FEATURES);
  if (s.N < 1 || s.N > (int64_t(1) << 40)) return fail(GPGOMEA_E_SHAPE, "N=%lld out of range", (long long)s.N);
  if (s.ldx < s.N) return fail(GPGOMEA_E_SHAPE, "ldx=%lld < N=%lld", (long long)s.ldx, (long long)s.N);
  if (int64_t(s.M) * (kMaxSpans + 1) > (int64_t(1) << 31) || int64_t(s.M) * kAdjChunks * 8 > (int64_t(1) << 31))
    return fail(GPGOMEA_E_SHAPE, "M=%d too large", s.M);
  return GPGOMEA_OK;
}

// stack slots needed by the deepest program that fits in L_max tokens:
// floor(log2((L_max + 1) / 2)) binary levels (an upper bound)
int slots_for(int L_max) {
  int leaves = (L_max + 1) / 2, d = 0;
  while ((1 << (d + 1)) <= leaves) ++d;
  return std::max(d, 1);
}

// Gradient spans: at most kMaxAdjSpans, and few enough that the partial
// buffer [M][C_max][spans] stays within kAdjPartEntries doubles.
int adj_span_cap(const Shape& s) {
  const int64_t per = int64_t(s.M) * std::max(s.C_max, 1);
  return int(std::max<int64_t>(1, std::min<int64_t>(kMaxAdjSpans, kAdjPartEntries / per)));
}
int plain_adj_spans(int64_t N, int R) {
  return int(std::max<int64_t>(1, std::min<int64_t>(kPlainAdjSpans, (N + R - 1) / R)));
}

struct Layout {
  size_t stats, yscr, meta, uops, events, ab, part, plain_part, ticket, gpart, lists, counts, redo,
      redo_span, rpool, plist, pcount, pfb, pfbc, pgpart, pspan, tune, total;
  int U_stride, ET, lstride, fbstride, adj_spans;
};

Layout layout_of(const Shape& s) {
  Layout l{};
  l.U_stride = s.L_max + 2;
  l.ET = std::max(1, s.L_max);  // flush events per program: at most L_max - 1
  l.lstride = s.M * kAdjChunks;
  l.fbstride = l.lstride * kAdjParts;  // a binary64 list: up to 4 parts per entry
  l.adj_spans = adj_span_cap(s);
  const size_t M = size_t(s.M), Cm = size_t(std::max(s.C_max, 1));
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  l.stats = take(ST_COUNT * sizeof(double));
  l.yscr = take(3 * kStatBlocks * sizeof(double));
  l.meta = take(M * sizeof(ProgMeta));
  l.uops = take(M * l.U_stride * sizeof(uint2));
  l.events = take(M * l.ET * sizeof(uint2));
  l.ab = take(M * AB_WORDS * sizeof(double));
  l.part = take(M * kMaxSpans * 4 * sizeof(double));
  l.plain_part = take(size_t(kPlainMaxBlocks) * 4 * sizeof(double));
  l.ticket = take(64);
  l.gpart = take(M * Cm * l.adj_spans * sizeof(double));
  // the class lists, then the two binary64 lists (shallow, deep)
  l.lists = take((size_t(kAdjClasses) * l.lstride + 2 * size_t(l.fbstride)) * sizeof(int32_t));
  l.counts = take(16 * sizeof(int32_t));
  l.redo = take(M * kAdjChunks * sizeof(int32_t));
  l.redo_span = take(M * kAdjChunks * l.adj_spans * sizeof(int32_t));
  l.rpool = take(kRedoPoolBytes);  // bad-tile masks of the binary64 fallback
  l.plist = take(M * kAdjChunks * sizeof(int32_t));  // plain form: per-individual entries
  l.pcount = take(M * kAdjClasses * sizeof(int32_t));  // per individual and work class
  l.pfb = take(M * 2 * kAdjChunks * kAdjParts * sizeof(int32_t));
  l.pfbc = take(M * 2 * sizeof(int32_t));
  l.pgpart = take(Cm * kPlainAdjSpans * sizeof(double));  // one individual's partials
  l.pspan = take(size_t(kAdjChunks) * kPlainAdjSpans * sizeof(int32_t));
  l.tune = take(M * (Cm + 2) * sizeof(double));  // outputs of the autotuner's trial calls
  l.total = o;
  return l;
}

// ---------------------------------------------------------------- planning
struct TuneKey {
  int fp64, Lcls, F, Ncls, Mcls, grad;
  bool operator<(const TuneKey& o) const {
    return std::tie(fp64, Lcls, F, Ncls, Mcls, grad) < std::tie(o.fp64, o.Lcls, o.F, o.Ncls, o.Mcls, o.grad);
  }
};
int log2cls(int64_t v) {
  int c = 0;
  while ((int64_t(1) << (c + 1)) <= v) ++c;
  return c;
}
TuneKey tune_key(const Shape& s, bool grad) {
  return {int((s.flags & GPGOMEA_FP64_NODES) != 0), log2cls(s.L_max + 1), s.F, log2cls(s.N),
          log2cls(s.M), int(grad)};
}
// Forward: K rows per lane, R rows per tile, G individuals per group.
// Adjoint: R, G common to the path classes; K = bit mask of the classes 0-2
// that run 2 rows per lane instead of 4 (classes 3 and 4 always run 2).
struct Tuned {
  int K, R, G;
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tuned;  // forward choices
std::map<TuneKey, Tuned> g_tuned_adj;

void finish_spans(TileCfg& c, int M, int64_t N, int max_spans) {
  const int64_t tiles = (N + c.R - 1) / c.R;
  c.n_groups = (M + c.G - 1) / c.G;
  c.tiles_per_span = int((tiles + max_spans - 1) / max_spans);
  if (c.tiles_per_span < 1) c.tiles_per_span = 1;
  c.n_spans = int((tiles + c.tiles_per_span - 1) / c.tiles_per_span);
}

// untuned forward tiles: at most 31 KB of LDS, so that five blocks (five waves
// per SIMD, what the eight-rows-per-lane forward is compiled for) share a CU
int forward_lds_cap() { return std::min(lds_limit_bytes(), 31 * 1024); }

// Row tile of the one-program-per-launch form: the largest of 2048, 1024, ...
// rows (a multiple of its batch) whose LDS stays within 64 KB.  It does not
// follow the fused kernel's tuned tile, which is sized for five blocks per CU.
int plain_tile_rows(const Shape& s, int K) {
  const int BR = 64 * K;
  int R = 2048;
  while (R > BR && size_t(s.F) * R * 4 + size_t(R) * 8 > size_t(64 * 1024)) R /= 2;
  const int64_t Nr = (s.N + BR - 1) / BR * BR;
  if (Nr < R) R = int(Nr);
  return std::max(R, BR);
}

TileCfg plan_forward(const Shape& s, const Tuned* t) {
  TileCfg c;
  const bool fp64 = (s.flags & GPGOMEA_FP64_NODES) != 0;
  c.K = fp64 ? 4 : 8;
  c.D = slots_for(s.L_max) <= 4 ? 4 : 8;  // plain form's stack slots
  c.W = 4;
  const int BR = 64 * c.K;
  const int64_t Nr = (s.N + BR - 1) / BR * BR;
  if (t) {
    c.K = fp64 ? 4 : t->K;
    c.R = t->R;
    c.G = t->G;
    const int64_t Nt = (s.N + 64 * c.K - 1) / (64 * c.K) * (64 * c.K);
    if (Nt < c.R) c.R = int(Nt);
  } else {
    c.R = 2048;
    while (c.R > BR && forward_lds_bytes(s.F, c.R, 64) > size_t(forward_lds_cap())) c.R /= 2;
    if (Nr < c.R) c.R = int(Nr);
    const int64_t tiles = (s.N + c.R - 1) / c.R;
    const int64_t target = 2048;
    int64_t G = (int64_t(s.M) * tiles + target - 1) / target;
    G = std::max<int64_t>(G, std::min(s.M, c.W));
    c.G = int(std::min<int64_t>(G, 64));
  }
  c.R = std::max(c.R, 64 * c.K);
  c.R = c.R / (64 * c.K) * (64 * c.K);
  // at most kFwdMaxG programs per group: the forward kernel keeps a group's
  // metadata in an LDS table of that size
  c.G = std::max(1, std::min({c.G, s.M, kFwdMaxG}));
  finish_spans(c, s.M, s.N, kMaxSpans);
  return c;
}

// Adjoint plan: the path classes share the row tile R (a multiple of 256,
// every class's batch), the group size G and the spans; class c's grid holds
// n_groups[c] group slots per span (blocks loop over the groups of their
// slot).  The fallback pass uses small groups, so that the flagged spans of
// different entries run in parallel blocks.
struct AdjPlan {
  int R = 512, G = 32;
  int Kmask = 0;  // classes 0-2 with bit c set run 2 rows per lane, else 4
  int n_spans = 1, tiles_per_span = 1;
  int64_t span_rows = 0;
  bool on[kAdjClasses] = {false, false, false, false, false};
  int n_groups[kAdjClasses] = {1, 1, 1, 1, 1};
  int fb_G = 4, fb_groups = 1;
  int plain_spans = 1;
  int64_t plain_span_rows = 0;
};

AdjPlan plan_adjoint(const Shape& s, const Tuned* t, int span_cap) {
  AdjPlan a;
  if (t) {
    a.R = t->R;
    a.G = t->G;
    a.Kmask = t->K & 7;
  }
  const int cap = lds_limit_bytes() - int(kAdjStaticLds);  // static LDS of the path kernels
  a.R = std::max(256, a.R / 256 * 256);
  while (a.R > 256 && adjoint_path_lds_bytes(s.F, a.R, 64, kAdjChunkNC, 4, true) > size_t(cap)) a.R /= 2;
  const int64_t Nr = (s.N + 255) / 256 * 256;
  if (Nr < a.R) a.R = int(Nr);
  a.G = std::max(1, std::min({a.G, s.M, 64}));  // the group list is lane-held
  const int Cm = s.C_max;
  a.on[0] = Cm >= 1;
  a.on[1] = Cm > 4;
  a.on[2] = Cm > 8;
  a.on[3] = Cm > 16;
  a.on[4] = Cm >= 1 && s.L_max >= 127;  // five or more stack slots need 64 leaves
  const int groups = (s.M + a.G - 1) / a.G;
  for (int c = 0; c < kAdjClasses; ++c) a.n_groups[c] = groups;
  // spans: enough work items (span, group) to fill the chip many times over
  // (about 16K); each span costs one partial per (individual, constant)
  const int64_t tiles = (s.N + a.R - 1) / a.R;
  int64_t want = (16384 + groups - 1) / groups;
  want = std::max<int64_t>(1, std::min<int64_t>({want, tiles, int64_t(span_cap)}));
  a.tiles_per_span = int((tiles + want - 1) / want);
  a.span_rows = int64_t(a.tiles_per_span) * a.R;
  a.n_spans = int((s.N + a.span_rows - 1) / a.span_rows);
  a.fb_G = std::min(4, s.M * kAdjChunks);
  a.fb_groups = std::min(64, (s.M * kAdjChunks + a.fb_G - 1) / a.fb_G);
  a.plain_spans = plain_adj_spans(s.N, a.R);
  const int64_t ptiles = (tiles + a.plain_spans - 1) / a.plain_spans;
  a.plain_span_rows = ptiles * a.R;
  a.plain_spans = int((s.N + a.plain_span_rows - 1) / a.plain_span_rows);
  return a;
}

bool adjoint_plan_fits(const Shape& s, const AdjPlan& a) {
  const int cap = lds_limit_bytes() - int(kAdjStaticLds);
  return adjoint_path_lds_bytes(s.F, a.R, a.G, kAdjChunkNC, 4, false) <= size_t(cap) &&
         adjoint_path_lds_bytes(s.F, a.R, 8, kAdjChunkNC, 4, true) <= size_t(cap);
}

// ------------------------------------------------------------ graph cache
// A call on a non-default stream is captured and launched as one hipGraph.
// The executable graph is cached per (shapes, flags, launch plan), not per
// pointer or batch size: every call captures its launch sequence again (host
// work only) and updates the cached executable graph in place
// (hipGraphExecUpdate: same kernels in the same order, new arguments and grid
// sizes), so calls with new output buffers or another batch size M reuse it.
// When the update is refused the graph is instantiated anew.  The cache holds
// at most kGraphCacheMax executables; the least recently used one is
// destroyed once its last launch has completed.
constexpr size_t kGraphCacheMax = 16;
struct GraphKey {
  std::vector<int64_t> v;
  bool operator<(const GraphKey& o) const { return v < o.v; }
};
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;   // recorded after the last launch
  uint64_t used = 0;
  std::vector<uintptr_t> sig;  // pointers and M the executable holds
};
std::mutex g_graph_mu;
std::map<GraphKey, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;

#define GG_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(GPGOMEA_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void destroy_entry(GraphEntry& e) {
  if (e.done) {
    (void)hipEventSynchronize(e.done);
    (void)hipEventDestroy(e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  e = GraphEntry{};
}

// ------------------------------------------------------- kernel timing hook
// With profiling on, every launch of a call is bracketed by hipEvents on the
// call's stream (graphs are bypassed: events cannot be read inside a replay).
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;
std::map<std::string, long> g_prof_counts;  // work counters of profiled calls
thread_local bool t_no_alloc = false;  // the no-allocation entry point is enqueuing

struct ProfScope {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (g_prof && !t_no_alloc && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(b, s);
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof_recs.push_back({name, a, b});
    }
  }
};
#define GG_TIMED(name, call)        \
  do {                              \
    ProfScope ps_(name, c.stream);  \
    GG_HIP(call);                   \
  } while (0)

struct Call {
  Shape s;
  const int8_t* ops;
  const float* consts;
  const float* X;
  const float* y;
  double* fitness;
  double* aux;
  double* grad;
  int8_t* status;
  char* ws;
  hipStream_t stream;
  bool with_grad;
};

const char* const kClassName[kAdjClasses] = {"adjoint_c4", "adjoint_c8", "adjoint_c16", "adjoint_c32",
                                             "adjoint_deep"};

// Profiled calls outside graph capture only: how much of the gradient fell
// back to binary64 (entries, row tiles, spans redone whole).  Synchronises the
// stream; counted into the profile report.
void count_fallback(const Call& c, const int* counts, const uint64_t* pool, int tile_words, int pool_cap) {
  if (!g_prof || t_no_alloc) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  int32_t h[kAdjClasses + 3] = {};
  if (hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
      hipStreamSynchronize(c.stream) != hipSuccess)
    return;
  long tiles = 0;
  const int slots = std::min(h[kAdjClasses + 2], pool_cap);
  if (slots > 0 && tile_words > 0) {
    std::vector<uint64_t> m(size_t(slots) * tile_words);
    if (hipMemcpyAsync(m.data(), pool, m.size() * 8, hipMemcpyDeviceToHost, c.stream) == hipSuccess &&
        hipStreamSynchronize(c.stream) == hipSuccess)
      for (uint64_t w : m) tiles += __builtin_popcountll(w);
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_counts["fallback_entries"] += h[kAdjClasses] + h[kAdjClasses + 1];
  g_prof_counts["fallback_entry_spans"] += h[kAdjClasses + 2];
  g_prof_counts["fallback_tiles"] += tiles;
  g_prof_counts["fallback_pool_overflow"] += std::max(0, h[kAdjClasses + 2] - pool_cap);
}

// Enqueue the whole pipeline on c.stream.
int enqueue_fused(const Call& c, const TileCfg& fc, const AdjPlan& ac) {
  const Layout l = layout_of(c.s);
  const bool fp64 = (c.s.flags & GPGOMEA_FP64_NODES) != 0;
  char* ws = c.ws;
  double* stats = reinterpret_cast<double*>(ws + l.stats);
  double* yscr = reinterpret_cast<double*>(ws + l.yscr);
  ProgMeta* meta = reinterpret_cast<ProgMeta*>(ws + l.meta);
  uint2* uops = reinterpret_cast<uint2*>(ws + l.uops);
  uint2* events = reinterpret_cast<uint2*>(ws + l.events);
  double* ab = reinterpret_cast<double*>(ws + l.ab);
  double* part = reinterpret_cast<double*>(ws + l.part);
  double* gpart = reinterpret_cast<double*>(ws + l.gpart);
  int* lists = reinterpret_cast<int*>(ws + l.lists);
  int* counts = reinterpret_cast<int*>(ws + l.counts);
  int* redo = reinterpret_cast<int*>(ws + l.redo);
  int32_t* redo_span = reinterpret_cast<int32_t*>(ws + l.redo_span);
  uint64_t* rpool = reinterpret_cast<uint64_t*>(ws + l.rpool);
  // tile-granular fallback: one mask bit per row tile of a span
  const int tile_words = ac.tiles_per_span <= 64 * kTileWords ? (ac.tiles_per_span + 63) / 64 : 0;
  const int pool_cap = tile_words ? int(kRedoPoolBytes / (size_t(tile_words) * 8)) : 0;
  const DataArgs d{c.X, c.s.ldx, c.s.F, c.s.N, c.y};
  const int M = c.s.M;
  const bool grad_work = c.with_grad && c.s.C_max > 0;
  GG_TIMED("ystats", launch_ystats(c.y, c.s.N, stats, yscr, c.stream));
  GG_TIMED("compile", launch_compile(c.ops, M, c.s.L_max, c.consts, c.s.C_max, c.s.F, 8, l.U_stride,
                                     uops, meta, events, l.ET, c.stream));
  GG_TIMED("probe", launch_probe(fp64, uops, l.U_stride, meta, M, d, c.stream));
  const bool sse = c.aux != nullptr || !(c.s.flags & GPGOMEA_LINEAR_SCALING);

  // one launch of an adjoint class over `list`
  auto adj = [&](int cls, int K, const int* list, const int* count, int G, int n_groups, int n_spans,
                 int64_t span_rows, double* gp, int gstride, int gi0, int32_t* rspan, int rstride, int ebase,
                 int* fbl, int* fbc, int fbs, bool split) {
    AdjLaunch L{cls, K, uops, l.U_stride, meta, d, stats, ab, gp, c.s.C_max, gstride, gi0, list, count,
                ac.R, G, n_groups, n_spans, span_rows, events, l.ET, redo, rspan, rstride, ebase, fbl, fbc,
                fbs, split, rpool, counts + kAdjClasses + 2, pool_cap, tile_words};
    return launch_adjoint_class(L, c.stream);
  };

  if (c.s.flags & GPGOMEA_PLAIN) {
    // one launch per individual: forward (last block finalizes), then its
    // gradient: the path kernel with the block's waves sharing the
    // individual, its binary64 fallback, and its gradient finalize
    unsigned* ticket = reinterpret_cast<unsigned*>(ws + l.ticket);
    double* pp = reinterpret_cast<double*>(ws + l.plain_part);
    GG_HIP(launch_fill_u32(ticket, 1, 0u, c.stream));
    TileCfg pc = fc;
    pc.R = plain_tile_rows(c.s, fc.K);
    for (int i = 0; i < M; ++i)
      GG_TIMED("plain_forward", launch_plain_forward(fp64, pc, i, uops, l.U_stride, meta, d, stats, pp, ticket,
                                                     c.s.flags, c.fitness, c.aux, c.status, ab, c.stream));
    if (grad_work) {
      int* plist = reinterpret_cast<int*>(ws + l.plist);
      int* pcount = reinterpret_cast<int*>(ws + l.pcount);
      int* pfb = reinterpret_cast<int*>(ws + l.pfb);
      int* pfbc = reinterpret_cast<int*>(ws + l.pfbc);
      double* pg = reinterpret_cast<double*>(ws + l.pgpart);
      int32_t* pspan = reinterpret_cast<int32_t*>(ws + l.pspan);
      GG_TIMED("plain_lists", launch_adjoint_plain_lists(meta, ab, M, plist, pcount, pfbc, redo, c.stream));
      const int P = ac.plain_spans;
      for (int i = 0; i < M; ++i) {
        const int e0 = i * kAdjChunks;
        // this individual's two binary64 lists (32 parts each) and their counts
        constexpr int kFb = kAdjChunks * kAdjParts;
        int* fb = pfb + 2 * kFb * i;
        int* fbc = pfbc + 2 * i;
        // the individual's work class as in the fused form (the other four
        // class launches find an empty list and return at once)
        for (int cls = 0; cls < kAdjClasses; ++cls) {
          if (!ac.on[cls]) continue;
          const int K = cls >= 3 || ((ac.Kmask >> cls) & 1) ? 2 : 4;
          GG_TIMED("plain_adjoint", adj(cls, K, plist + e0, pcount + size_t(i) * kAdjClasses + cls, kAdjChunks, 1,
                                        P, ac.plain_span_rows, pg, P, i, pspan, P, e0, fb, fbc, kFb, true));
        }
        GG_TIMED("plain_fallback", adj(kAdjFallback, 2, fb, fbc, kAdjChunks, 1, P, ac.plain_span_rows, pg, P, i,
                                       pspan, P, e0, nullptr, nullptr, 0, true));
        GG_TIMED("plain_fallback", adj(kAdjFallbackWide, 2, fb + kFb, fbc + 1, kAdjChunks, 1, P,
                                       ac.plain_span_rows, pg, P, i, pspan, P, e0, nullptr, nullptr, 0, true));
        GG_TIMED("plain_grad_finalize",
                 launch_grad_finalize(meta, i, 1, c.s.C_max, pg, P, P, stats, ab, c.grad, c.stream));
      }
    } else if (c.with_grad) {  // no constants: nothing to differentiate (grad has no entries)
    }
    return GPGOMEA_OK;
  }
  GG_TIMED("fused_forward", launch_fused_forward(fp64, fc, uops, l.U_stride, meta, M, d, stats, part, sse,
                                                 c.stream));
  GG_TIMED("finalize", launch_finalize(meta, M, part, fc.n_spans, stats, c.s.flags, c.fitness, c.aux,
                                       c.status, ab, c.stream));
  if (grad_work) {
    int* fbl = lists + size_t(kAdjClasses) * l.lstride;  // two binary64 lists, fbstride apart
    int* fbc = counts + kAdjClasses;
    const int S = ac.n_spans, gs = l.adj_spans;
    GG_TIMED("adjoint_partition",
             launch_adjoint_partition(meta, ab, M, l.lstride, lists, counts, redo, c.stream));
    for (int cls = 0; cls < kAdjClasses; ++cls) {
      if (!ac.on[cls]) continue;
      const int K = cls >= 3 || ((ac.Kmask >> cls) & 1) ? 2 : 4;
      // the chunked classes (32 constants per entry) work in groups of at
      // most 32, so that their blocks' binary64 accumulators leave room for
      // four blocks per CU (the waves they are compiled for)
      const int G = cls >= 3 ? std::min(ac.G, 32) : ac.G;
      GG_TIMED(kClassName[cls], adj(cls, K, lists + size_t(cls) * l.lstride, counts + cls, G, ac.n_groups[cls],
                                    S, ac.span_rows, gpart, gs, 0, redo_span, gs, 0, fbl, fbc, l.fbstride, false));
    }
    GG_TIMED("adjoint_fallback", adj(kAdjFallback, 2, fbl, fbc, ac.fb_G, ac.fb_groups, S, ac.span_rows, gpart, gs,
                                     0, redo_span, gs, 0, nullptr, nullptr, 0, false));
    GG_TIMED("adjoint_fallback", adj(kAdjFallbackWide, 2, fbl + l.fbstride, fbc + 1, ac.fb_G, ac.fb_groups, S,
                                     ac.span_rows, gpart, gs, 0, redo_span, gs, 0, nullptr, nullptr, 0, false));
    GG_TIMED("grad_finalize",
             launch_grad_finalize(meta, 0, M, c.s.C_max, gpart, gs, S, stats, ab, c.grad, c.stream));
    count_fallback(c, counts, rpool, tile_words, pool_cap);
  }
  return GPGOMEA_OK;
}

void plans_for(const Shape& s, TileCfg& fc, AdjPlan& ac) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(tune_key(s, false));
  fc = plan_forward(s, it == g_tuned.end() ? nullptr : &it->second);
  auto ia = g_tuned_adj.find(tune_key(s, true));
  ac = plan_adjoint(s, ia == g_tuned_adj.end() ? nullptr : &ia->second, adj_span_cap(s));
}

int run_call(const Call& c) {
  (void)hipGetLastError();  // launches below report their own errors only
  TileCfg fc;
  AdjPlan ac;
  plans_for(c.s, fc, ac);
  if (c.with_grad && !adjoint_plan_fits(c.s, ac))
    return fail(GPGOMEA_E_UNSUPPORTED, "no adjoint block fits LDS for F=%d", c.s.F);
  if (fc.G > kFwdMaxG || ac.G > 64)
    return fail(GPGOMEA_E_UNSUPPORTED, "group too large (forward %d of at most %d, adjoint %d of at most 64)",
                fc.G, kFwdMaxG, ac.G);
  const bool graph =
      !(c.s.flags & (GPGOMEA_NO_GRAPH | GPGOMEA_PLAIN)) && c.stream != nullptr && !g_prof;
  if (!graph) return enqueue_fused(c, fc, ac);

  // the launch sequence depends on these (not on pointers or M)
  GraphKey key;
  key.v = {int64_t(c.with_grad), int64_t(c.aux != nullptr), int64_t(c.s.L_max), int64_t(c.s.C_max),
           int64_t(c.s.F), c.s.N, c.s.ldx, int64_t(c.s.flags), int64_t(fc.K), int64_t(fc.R),
           int64_t(ac.R), int64_t(ac.Kmask), int64_t(reinterpret_cast<uintptr_t>(c.stream))};
  const std::vector<uintptr_t> sig = {uintptr_t(c.ops),    uintptr_t(c.consts), uintptr_t(c.X),
                                      uintptr_t(c.y),      uintptr_t(c.fitness), uintptr_t(c.aux),
                                      uintptr_t(c.grad),   uintptr_t(c.status), uintptr_t(c.ws),
                                      uintptr_t(c.s.M)};
  std::lock_guard<std::mutex> lk(g_graph_mu);
  GraphEntry& e = g_graphs[key];
  if (!(e.exec && e.sig == sig)) {  // new arguments: capture, then update or instantiate
    hipGraph_t g = nullptr;
    GG_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_fused(c, fc, ac);
    const hipError_t ec = hipStreamEndCapture(c.stream, &g);
    if (rc != GPGOMEA_OK || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (!e.exec) g_graphs.erase(key);
      return rc != GPGOMEA_OK ? rc : fail(GPGOMEA_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    }
    if (e.exec) {
      // the executable's previous launch must have completed before its
      // arguments change
      GG_HIP(hipEventSynchronize(e.done));
      hipGraphNode_t bad_node = nullptr;
      hipGraphExecUpdateResult res = hipGraphExecUpdateError;
      const hipError_t eu = hipGraphExecUpdate(e.exec, g, &bad_node, &res);
      if (eu != hipSuccess || res != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();
        destroy_entry(e);
      }
    }
    if (!e.exec) {
      const hipError_t ei = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        e.exec = nullptr;
        g_graphs.erase(key);
        return fail(GPGOMEA_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
      }
    }
    (void)hipGraphDestroy(g);
    e.sig = sig;
  }
  if (!e.done) GG_HIP(hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
  GG_HIP(hipGraphLaunch(e.exec, c.stream));
  GG_HIP(hipEventRecord(e.done, c.stream));
  e.used = ++g_graph_clock;
  while (g_graphs.size() > kGraphCacheMax) {  // evict the least recently used
    auto lru = g_graphs.begin();
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
      if (it->second.used < lru->second.used) lru = it;
    destroy_entry(lru->second);
    g_graphs.erase(lru);
  }
  return GPGOMEA_OK;
}

int check_call(const Shape& s, const void* ops, const void* consts, const void* X, const void* y,
               const void* fitness, void* ws, size_t ws_bytes) {
  if (!ops || !X || !y || !fitness || !ws) return fail(GPGOMEA_E_ARG, "NULL required pointer");
  if (s.C_max > 0 && !consts) return fail(GPGOMEA_E_ARG, "consts is NULL but C_max > 0");
  const int rc = check_shape(s);
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GPGOMEA_E_WORKSPACE, "workspace not 256-byte aligned");
  const size_t need = layout_of(s).total;
  if (ws_bytes < need)
    return fail(GPGOMEA_E_WORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  return GPGOMEA_OK;
}

}  // namespace
}  // namespace gg

using namespace gg;

extern "C" int gpgomea_version(void) { return 10000; }

extern "C" const char* gpgomea_last_error(void) { return last_error().c_str(); }

extern "C" size_t gpgomea_workspace_bytes(int32_t M, int32_t L_max, int32_t C_max, int32_t F,
                                          int64_t N, uint32_t flags) {
  const Shape s{M, L_max, C_max, F, N, N, flags};
  if (check_shape(s) != GPGOMEA_OK) return 0;
  return layout_of(s).total;
}

extern "C" int gpgomea_eval_batch(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                  int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                                  const float* y, uint32_t flags, double* fitness, double* aux,
                                  int8_t* status, void* workspace, size_t workspace_bytes,
                                  void* stream) {
  const Shape s{M, L_max, C_max, F, N, ldx, flags};
  int rc = check_call(s, ops, consts, X, y, fitness, workspace, workspace_bytes);
  if (rc) return rc;
  Call c{s, ops, consts, X, y, fitness, aux, nullptr, status, static_cast<char*>(workspace),
         static_cast<hipStream_t>(stream), false};
  return run_call(c);
}

// ------------------------------------------------------ no-allocation entry
// Fitness scratch for callers that cannot allocate: a file-scope device array
// (each GPU holds its own copy until the process ends).  Host code reaches it
// only through the address hipGetSymbolAddress gives on each device, taken
// once per device with that device current; the array's name itself is not a
// device address on the host.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace gg {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (resolved on the
// first call there); E_HIP on failure.
int scratch_address(void** out) {
  int dev = 0;
  GG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GPGOMEA_E_HIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GPGOMEA_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GPGOMEA_OK;
}
}  // namespace
}  // namespace gg

extern "C" size_t gpgomea_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int gpgomea_eval_batch_noalloc(const int8_t* ops, int32_t M, int32_t L_max,
                                          const float* consts, int32_t C_max, const float* X,
                                          int32_t F, int64_t N, int64_t ldx, const float* y,
                                          uint32_t flags, double* fitness, double* aux,
                                          int8_t* status, void* stream) {
  const Shape s{M, L_max, C_max, F, N, ldx, flags};
  if (!ops || !X || !y || !fitness) return fail(GPGOMEA_E_ARG, "NULL required pointer");
  if (C_max > 0 && !consts) return fail(GPGOMEA_E_ARG, "consts is NULL but C_max > 0");
  int rc = check_shape(s);
  if (rc) return rc;
  // the fitness path uses the leading regions of the workspace layout only
  // (statistics, programs, flush events, fit, forward partials, plain ticket)
  const size_t need = layout_of(s).gpart;
  if (need > kScratchBytes)
    return fail(GPGOMEA_E_WORKSPACE,
                "shape needs %zu bytes of scratch; the no-allocation entry point holds %zu "
                "(use gpgomea_eval_batch with a workspace)",
                need, kScratchBytes);
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  (void)hipGetLastError();
  Call c{s, ops, consts, X, y, fitness, aux, nullptr, status, static_cast<char*>(ws),
         static_cast<hipStream_t>(stream), false};
  TileCfg fc;
  AdjPlan ac;
  plans_for(s, fc, ac);
  if (fc.G > kFwdMaxG)
    return fail(GPGOMEA_E_UNSUPPORTED, "group of more than %d programs (forward %d)", kFwdMaxG, fc.G);
  // direct launches only: no graph instantiation, no timing events
  t_no_alloc = true;
  rc = enqueue_fused(c, fc, ac);
  t_no_alloc = false;
  return rc;
}

extern "C" int gpgomea_grad_consts(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                   int32_t C_max, const float* X, int32_t F, int64_t N,
                                   int64_t ldx, const float* y, uint32_t flags, double* fitness,
                                   double* aux, double* grad, int8_t* status, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  const Shape s{M, L_max, C_max, F, N, ldx, flags};
  int rc = check_call(s, ops, consts, X, y, fitness, workspace, workspace_bytes);
  if (rc) return rc;
  if (!grad && C_max > 0) return fail(GPGOMEA_E_ARG, "grad is NULL but C_max > 0");
  if (flags & GPGOMEA_FP64_NODES)
    return fail(GPGOMEA_E_UNSUPPORTED, "the adjoint runs in binary32 nodes only");
  Call c{s, ops, consts, X, y, fitness, aux, grad, status, static_cast<char*>(workspace),
         static_cast<hipStream_t>(stream), true};
  return run_call(c);
}

namespace gg {
namespace {
int check_design(const int8_t* ops, int32_t M, int32_t L_max, const float* consts, int32_t C_max,
                 const float* X, int32_t F, int64_t N, int64_t ldx, const float* y, int32_t block,
                 double* fitness) {
  if (M < 0 || L_max < 1 || L_max > GPGOMEA_MAX_LEN || C_max < 0 || C_max > GPGOMEA_MAX_CONSTS ||
      F < 1 || F > GPGOMEA_MAX_FEATURES || N < 1 || ldx < N)
    return fail(GPGOMEA_E_SHAPE, "M=%d L_max=%d C_max=%d F=%d N=%lld ldx=%lld outside the limits", M, L_max,
                C_max, F, (long long)N, (long long)ldx);
  if (block < 64 || block > 1024 || (block & (block - 1)))
    return fail(GPGOMEA_E_ARG, "block=%d must be a power of two in [64, 1024]", block);
  if (M > 0 && (!ops || !X || !y || !fitness || (C_max > 0 && !consts)))
    return fail(GPGOMEA_E_ARG, "NULL required pointer");
  return GPGOMEA_OK;
}
}  // namespace
}  // namespace gg

extern "C" int gpgomea_eval_design1(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                    int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                                    const float* y, int32_t block, double* fitness, int8_t* status,
                                    void* stream) {
  using namespace gg;
  int rc = check_design(ops, M, L_max, consts, C_max, X, F, N, ldx, y, block, fitness);
  if (rc) return rc;
  (void)hipGetLastError();
  const DesignArgs a{ops, M, L_max, consts, C_max, F, X, ldx, N, y, block, fitness, status};
  GG_HIP(launch_design1(a, static_cast<hipStream_t>(stream)));
  return GPGOMEA_OK;
}

extern "C" int gpgomea_eval_design2(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                    int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                                    const float* y, int32_t block, int32_t blocks_per_program,
                                    double* partial, double* fitness, int8_t* status, void* stream) {
  using namespace gg;
  int rc = check_design(ops, M, L_max, consts, C_max, X, F, N, ldx, y, block, fitness);
  if (rc) return rc;
  if (blocks_per_program < 1 || int64_t(blocks_per_program) * M > (int64_t(1) << 31) - 1)
    return fail(GPGOMEA_E_ARG, "blocks_per_program=%d (M=%d) out of range", blocks_per_program, M);
  if (M > 0 && !partial) return fail(GPGOMEA_E_ARG, "NULL partial");
  (void)hipGetLastError();
  const DesignArgs a{ops, M, L_max, consts, C_max, F, X, ldx, N, y, block, fitness, status};
  GG_HIP(launch_design2(a, blocks_per_program, partial, static_cast<hipStream_t>(stream)));
  return GPGOMEA_OK;
}

extern "C" int gpgomea_adam_consts(float* consts, int32_t M, int32_t C_max, const double* grad,
                                   const double* fitness, float* moments, float* best_consts,
                                   double* best_fitness, int32_t t, double lr, double beta1,
                                   double beta2, double eps, void* stream) {
  using namespace gg;
  if (M < 0 || C_max < 0 || C_max > GPGOMEA_MAX_CONSTS)
    return fail(GPGOMEA_E_SHAPE, "M=%d, C_max=%d outside [0, %d]", M, C_max, GPGOMEA_MAX_CONSTS);
  if (t < 1) return fail(GPGOMEA_E_ARG, "step number t=%d must be >= 1", t);
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return fail(GPGOMEA_E_ARG, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0");
  if (M == 0) return GPGOMEA_OK;
  if (!fitness || !best_fitness) return fail(GPGOMEA_E_ARG, "NULL fitness or best_fitness");
  if (C_max > 0 && (!consts || !grad || !moments || !best_consts))
    return fail(GPGOMEA_E_ARG, "NULL consts, grad, moments or best_consts with C_max > 0");
  // 1 - beta and the bias corrections in binary64 (in binary32 they cancel:
  // 1 - float(0.999) is 1.3e-5 away from 0.001, relatively)
  const AdamParams p{float(lr), float(beta1), float(beta2), float(eps), float(1.0 - beta1),
                     float(1.0 - beta2), float(1.0 - std::pow(beta1, t)), float(1.0 - std::pow(beta2, t))};
  if (!(p.bias1 > 0.0f) || !(p.bias2 > 0.0f)) return fail(GPGOMEA_E_ARG, "bias correction is zero");
  const size_t mc = size_t(M) * size_t(C_max);
  (void)hipGetLastError();
  GG_HIP(launch_adam_consts(consts, M, C_max, grad, fitness, moments, moments + mc, best_consts,
                            best_fitness, p, static_cast<hipStream_t>(stream)));
  return GPGOMEA_OK;
}

extern "C" int gpgomea_clear_graphs(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& kv : g_graphs) destroy_entry(kv.second);
  g_graphs.clear();
  return GPGOMEA_OK;
}

extern "C" int gpgomea_graph_count(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  return int(g_graphs.size());
}

// --------------------------------------------------------------- profiling
extern "C" int gpgomea_profile(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof = enable != 0;
  return GPGOMEA_OK;
}

extern "C" int gpgomea_profile_report(char* buf, int32_t len) {
  // the text is built once per report; a size query (buf == NULL) keeps it for
  // the call that fetches it
  thread_local std::string pending;
  thread_local bool have = false;
  if (!have) {
    std::vector<ProfRec> recs;
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      recs.swap(g_prof_recs);
    }
    std::map<std::string, std::pair<long, double>> acc;
    for (auto& r : recs) {
      float ms = 0.0f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        auto& e = acc[r.name];
        e.first += 1;
        e.second += ms;
      }
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    pending.clear();
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      for (auto& kv : g_prof_counts) acc[kv.first] = {kv.second, 0.0};
      g_prof_counts.clear();
    }
    for (auto& kv : acc) {
      char line[160];
      std::snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first,
                    kv.second.second);
      pending += line;
    }
    have = true;
  }
  if (!buf || len <= 0) return int(pending.size()) + 1;
  std::strncpy(buf, pending.c_str(), size_t(len) - 1);
  buf[len - 1] = 0;
  const int n = int(std::min<size_t>(pending.size(), size_t(len) - 1));
  have = false;
  pending.clear();
  return n;
}

extern "C" int gpgomea_op_costs(double* out, int32_t n, int32_t iters, float* dev_scratch,
                                void* stream) {
  if (!out || !dev_scratch) return fail(GPGOMEA_E_ARG, "NULL pointer");
  if (n < int(UOP_NUM) + 1 || iters < 16) return fail(GPGOMEA_E_SHAPE, "need n >= %d, iters >= 16", int(UOP_NUM) + 1);
  (void)hipGetLastError();
  if (measure_op_costs(out, n, iters, static_cast<hipStream_t>(stream), dev_scratch) != 0)
    return fail(GPGOMEA_E_ARG, "bad arguments");
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GPGOMEA_E_HIP, "op cost kernels: %s", hipGetErrorString(e));
  return GPGOMEA_OK;
}

// ------------------------------------------------------------------ tuning
// ------------------------------------------------------------------ autotune
namespace {

constexpr int64_t kTuneRows = int64_t(1) << 20;  // rows the trial calls use at most

// Fastest of `trials` timed runs of the whole pipeline under the given plans
// (after one untimed run), in ms; negative on a HIP error.
float time_plans(const Call& c, const TileCfg& fc, const AdjPlan& ac, int trials) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
  float best = -1.0f;
  if (enqueue_fused(c, fc, ac) == GPGOMEA_OK) {
    best = 1e30f;
    for (int t = 0; t < trials; ++t) {
      float ms = 0.0f;
      if (hipEventRecord(e0, c.stream) != hipSuccess || enqueue_fused(c, fc, ac) != GPGOMEA_OK ||
          hipEventRecord(e1, c.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        best = -1.0f;
        break;
      }
      best = std::min(best, ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

std::string tune_line(const char* table, const TuneKey& k, const Tuned& t) {
  char b[256];
  std::snprintf(b, sizeof(b),
                "  {\"table\": \"%s\", \"fp64\": %d, \"Lcls\": %d, \"F\": %d, \"Ncls\": %d, "
                "\"Mcls\": %d, \"grad\": %d, \"K\": %d, \"R\": %d, \"G\": %d}",
                table, k.fp64, k.Lcls, k.F, k.Ncls, k.Mcls, k.grad, t.K, t.R, t.G);
  return b;
}

bool json_int(const std::string& line, const char* key, int* out) {
  const std::string pat = std::string("\"") + key + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  char* end = nullptr;
  const long v = std::strtol(line.c_str() + at + pat.size(), &end, 10);
  if (end == line.c_str() + at + pat.size()) return false;
  *out = int(v);
  return true;
}

// Read a tuning file (one entry per line) into the tables; false if unreadable.
bool read_tuning(const char* path, int* n_read) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  int n = 0;
  while (std::getline(f, line)) {
    const bool fwd = line.find("\"table\": \"fwd\"") != std::string::npos;
    const bool adj = line.find("\"table\": \"adj\"") != std::string::npos;
    if (!fwd && !adj) continue;
    TuneKey k{};
    Tuned t{};
    if (!(json_int(line, "fp64", &k.fp64) && json_int(line, "Lcls", &k.Lcls) &&
          json_int(line, "F", &k.F) && json_int(line, "Ncls", &k.Ncls) &&
          json_int(line, "Mcls", &k.Mcls) && json_int(line, "grad", &k.grad) &&
          json_int(line, "K", &t.K) && json_int(line, "R", &t.R) && json_int(line, "G", &t.G)))
      continue;
    if (t.K < 0 || t.R < 64 || t.G < 1 || (fwd && t.K < 1)) continue;
    (fwd ? g_tuned : g_tuned_adj)[k] = t;
    ++n;
  }
  if (n_read) *n_read = n;
  return true;
}

bool write_tuning(const char* path) {
  std::ostringstream o;
  o << "{\"gpgomea_tuning\": 2, \"entries\": [\n";
  bool first = true;
  for (const auto& e : g_tuned) {
    o << (first ? "" : ",\n") << tune_line("fwd", e.first, e.second);
    first = false;
  }
  for (const auto& e : g_tuned_adj) {
    o << (first ? "" : ",\n") << tune_line("adj", e.first, e.second);
    first = false;
  }
  o << "\n]}\n";
  std::ofstream f(path, std::ios::trunc);
  if (!f) return false;
  f << o.str();
  return bool(f);
}

}  // namespace

extern "C" int gpgomea_autotune(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                                const float* y, uint32_t flags, int32_t with_grad, void* workspace,
                                size_t workspace_bytes, const char* cache_path, int32_t trials,
                                char* out_desc, int32_t desc_len, void* stream) {
  const Shape s{M, L_max, C_max, F, N, ldx, flags};
  if (flags & GPGOMEA_PLAIN) return fail(GPGOMEA_E_ARG, "autotune tunes the fused form (PLAIN set)");
  if (with_grad && (flags & GPGOMEA_FP64_NODES))
    return fail(GPGOMEA_E_UNSUPPORTED, "the adjoint runs in binary32 nodes only");
  if (trials < 1) return fail(GPGOMEA_E_ARG, "trials=%d must be >= 1", trials);
  const Layout l = layout_of(s);
  char* ws = static_cast<char*>(workspace);
  double* fit = reinterpret_cast<double*>(ws + l.tune);
  int rc = check_call(s, ops, consts, X, y, fit, workspace, workspace_bytes);
  if (rc) return rc;
  (void)hipGetLastError();
  // trial calls run on a prefix of the rows; the choice is stored for the
  // full shape's class
  Shape st = s;
  st.N = std::min<int64_t>(s.N, kTuneRows);
  st.flags = (flags & ~GPGOMEA_NO_GRAPH) | GPGOMEA_NO_GRAPH;
  const bool fp64 = (flags & GPGOMEA_FP64_NODES) != 0;
  double* grad = fit + M;
  int8_t* status = reinterpret_cast<int8_t*>(grad + size_t(M) * std::max(C_max, 1));
  Call c{st, ops, consts, X, y, fit, nullptr, nullptr, status, ws, static_cast<hipStream_t>(stream),
         false};

  // forward: rows per lane K, rows per LDS tile R, individuals per group G
  const int Ks_f[2] = {8, 4};
  const int Rs_f[4] = {256, 512, 1024, 2048};
  const int Gs_f[4] = {16, 32, 64, 128};
  const int lds = lds_limit_bytes();
  Tuned best_f{0, 0, 0};
  float best_f_ms = 1e30f;
  TileCfg fc_best;
  for (int k : Ks_f) {
    if (fp64 && k != 4) continue;
    for (int r : Rs_f) {
      if (r < 64 * k) continue;
      for (int g : Gs_f) {
        if (forward_lds_bytes(F, r, g) > size_t(lds)) continue;
        const Tuned t{k, r, g};
        const TileCfg fc = plan_forward(st, &t);
        const AdjPlan ac = plan_adjoint(st, nullptr, adj_span_cap(s));
        const float ms = time_plans(c, fc, ac, trials);
        if (ms < 0.0f) {
          const std::string why = last_error();
          return fail(GPGOMEA_E_HIP, "autotune trial failed: %s", why.c_str());
        }
        if (ms < best_f_ms) {
          best_f_ms = ms;
          best_f = t;
          fc_best = fc;
        }
      }
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[tune_key(s, false)] = best_f;
  char desc[512];
  int len = std::snprintf(desc, sizeof(desc), "forward K=%d R=%d G=%d (%.3f ms on %lld rows)", best_f.K,
                          best_f.R, best_f.G, double(best_f_ms), (long long)st.N);

  if (with_grad && C_max > 0) {
    c.with_grad = true;
    c.grad = grad;
    // the path classes' tile R and group G, and which of classes 0-2 run two
    // rows per lane (K mask; only the classes the shape can populate vary)
    const int Rs_a[3] = {256, 512, 1024};
    const int Gs_a[4] = {8, 16, 32, 64};
    const int kmasks[4] = {0, 4, 6, 7};  // class 2 first: its register array is the largest
    Tuned best_a{-1, 0, 0};
    float best_a_ms = 1e30f;
    for (int km : kmasks) {
      if ((km & 2) && C_max <= 4) continue;
      if ((km & 4) && C_max <= 8) continue;
      for (int r : Rs_a) {
        for (int g : Gs_a) {
          const Tuned t{km, r, g};
          const AdjPlan ac = plan_adjoint(st, &t, adj_span_cap(s));
          if (ac.R != r || !adjoint_plan_fits(st, ac)) continue;  // clamped: same as another
          const float ms = time_plans(c, fc_best, ac, trials);
          if (ms < 0.0f) {
            const std::string why = last_error();
            return fail(GPGOMEA_E_HIP, "autotune trial failed: %s", why.c_str());
          }
          if (ms < best_a_ms) {
            best_a_ms = ms;
            best_a = t;
          }
        }
      }
    }
    if (best_a.K >= 0) {
      g_tuned_adj[tune_key(s, true)] = best_a;
      len += std::snprintf(desc + len, sizeof(desc) - size_t(len),
                           "; fitness+gradient with adjoint Kmask=%d R=%d G=%d (%.3f ms)", best_a.K, best_a.R,
                           best_a.G, double(best_a_ms));
    }
  }
  if (cache_path) {
    int n = 0;
    std::map<TuneKey, Tuned> keep_f = g_tuned, keep_a = g_tuned_adj;
    (void)read_tuning(cache_path, &n);  // merge: entries of this process win
    for (const auto& e : keep_f) g_tuned[e.first] = e.second;
    for (const auto& e : keep_a) g_tuned_adj[e.first] = e.second;
    if (!write_tuning(cache_path)) return fail(GPGOMEA_E_ARG, "cannot write %s", cache_path);
  }
  if (out_desc && desc_len > 0) {
    std::strncpy(out_desc, desc, size_t(desc_len) - 1);
    out_desc[desc_len - 1] = '\0';
  }
  return GPGOMEA_OK;
}

extern "C" int gpgomea_load_tuning(const char* cache_path) {
  if (!cache_path) return fail(GPGOMEA_E_ARG, "cache_path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int n = 0;
  if (!read_tuning(cache_path, &n)) return fail(GPGOMEA_E_ARG, "cannot read %s", cache_path);
  return n;
}

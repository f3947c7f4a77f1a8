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
constexpr int kMaxAdjSpans = 256;  // gradient partials per individual (upper bound)
constexpr int64_t kAdjPartEntries = int64_t(1) << 24;  // cap on M x spans x C_max (128 MB)
constexpr int kPlainMaxBlocks = 1024;
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
  if (int64_t(s.M) * (kMaxSpans + 1) > (int64_t(1) << 31))
    return fail(GPGOMEA_E_SHAPE, "M=%d too large", s.M);
  return GPGOMEA_OK;
}

// stack slots needed by the deepest program that fits in L_max tokens:
// floor(log2((L_max + 1) / 2)) binary levels
int slots_for(int L_max) {
  int leaves = (L_max + 1) / 2, d = 0;
  while ((1 << (d + 1)) <= leaves) ++d;
  return std::max(d, 1);
}

// Gradient partials per individual: at most kMaxAdjSpans, and few enough that
// the partial buffer stays within kAdjPartEntries doubles.
int adj_span_cap(const Shape& s) {
  const int64_t per = int64_t(s.M) * std::max(s.C_max, 1);
  return int(std::max<int64_t>(1, std::min<int64_t>(kMaxAdjSpans, kAdjPartEntries / per)));
}

struct Layout {
  size_t stats, yscr, meta, uops, merges, ab, part, plain_part, ticket, gpart, adjl, redo_span, tune,
      total;
  int U_stride;
  int MT;  // merge descriptors per program
};

Layout layout_of(const Shape& s) {
  Layout l{};
  l.U_stride = s.L_max + 2;
  size_t o = 0;
  l.stats = o;
  o = align256(o + ST_COUNT * sizeof(double));
  l.yscr = o;
  o = align256(o + 3 * kStatBlocks * sizeof(double));
  l.meta = o;
  o = align256(o + size_t(s.M) * sizeof(ProgMeta));
  l.uops = o;
  o = align256(o + size_t(s.M) * l.U_stride * sizeof(uint2));
  l.MT = std::max(1, s.C_max);
  l.merges = o;
  o = align256(o + size_t(s.M) * l.MT * sizeof(uint32_t));
  l.ab = o;
  o = align256(o + size_t(s.M) * 2 * sizeof(double));
  l.part = o;
  o = align256(o + size_t(s.M) * kMaxSpans * 4 * sizeof(double));
  l.plain_part = o;
  o = align256(o + size_t(kPlainMaxBlocks) * 4 * sizeof(double));
  l.ticket = o;
  o = align256(o + 64);
  l.gpart = o;
  o = align256(o + size_t(s.M) * adj_span_cap(s) * std::max(s.C_max, 1) * sizeof(double));
  l.adjl = o;  // adjoint tier lists [4][M], counts [4], then the path redo flags [M], or
               // per-individual counts [M][4] + a list
  o = align256(o + size_t(s.M) * 8 * sizeof(int32_t) + 64);
  l.redo_span = o;  // path tier fallback: [M][n_spans] bytes
  o = align256(o + size_t(s.M) * kMaxAdjSpans);
  l.tune = o;  // outputs of the autotuner's trial calls: fitness, grad, status
  o = align256(o + size_t(s.M) * (std::max(s.C_max, 1) + 2) * sizeof(double));
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
struct Tuned {
  int K, R, G;
  int TC;  // adjoint: tier A tape entries when F = 0 (0 for the forward)
  int F;   // adjoint: path tier constants NC (K, R, G are then the path tier's); 0 = no path tier
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

int forward_lds_cap() { return std::min(lds_limit_bytes(), 64 * 1024); }

TileCfg plan_forward(const Shape& s, const Tuned* t) {
  TileCfg c;
  const bool fp64 = (s.flags & GPGOMEA_FP64_NODES) != 0;
  c.K = fp64 ? 4 : 8;
  c.D = fp64 ? 8 : (slots_for(s.L_max) <= 4 ? 4 : 8);
  c.NP = uop_pairs(s.L_max);
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
  // at most 64 programs per group: the forward kernel keeps a group's
  // metadata in a 64-entry LDS table
  c.G = std::max(1, std::min({c.G, s.M, 64}));
  finish_spans(c, s.M, s.N, kMaxSpans);
  return c;
}

// Adjoint plan.  Path tier: programs with at most NC constants in path
// forward mode, (K, NC) = (4, 12) unless tuned to (4, 16), (4, 8), (8, 8),
// (2, 16) or (2, 32).
// Tier A: K rows per lane with a TC-entry register tape, (K, TC) = (4, 16)
// unless tuned (without a path tier) to (2, 16) or (2, 32).  W = 4 waves; a
// row tile of at most 32 KB untuned, so that several blocks share a CU.
// Tier B: (2, 32) for the tapes between tier A's and 32 entries.  Tier C: the
// largest LDS-tape block that fits the worst-case tape (L_max - 1 entries per
// wave).  All tiers use the same spans, set by the path tier (tier A without
// one); the other tiers' tiles divide the span.
bool reg_variant(int K, int TC) { return (K == 4 && TC == 16) || (K == 2 && (TC == 16 || TC == 32)); }
bool path_variant(int K, int NC) {
  return (K == 4 && (NC == 16 || NC == 12 || NC == 8)) || (K == 8 && NC == 8) ||
         (K == 2 && (NC == 32 || NC == 16));
}

AdjPlan plan_adjoint(const Shape& s, int D, const Tuned* t, int span_cap) {
  AdjPlan a;
  const int Cm = std::max(1, s.C_max);
  const int cap = lds_limit_bytes() - 64;  // static LDS of the kernels
  TileCfg& pt = a.path;
  TileCfg& r = a.reg;
  pt.D = r.D = D;
  pt.NP = r.NP = uop_pairs(s.L_max);
  pt.W = r.W = 4;
  pt.K = 4;
  a.nc_p = 12;  // (4, 12) is the largest variant that keeps three waves per SIMD
  pt.G = 16;
  pt.R = 1024;
  r.K = 4;
  a.tc_a = 16;
  a.tc_b = 32;
  a.lane_consts = std::min(Cm, 32);
  r.G = 16;
  r.R = 1024;
  if (t) {
    if (t->F > 0 && path_variant(t->K, t->F)) {
      pt.K = t->K;
      a.nc_p = t->F;
      pt.R = t->R;
      pt.G = t->G;
    } else if (t->F == 0) {
      a.nc_p = 0;
      if (reg_variant(t->K, t->TC)) {
        r.K = t->K;
        a.tc_a = t->TC;
      }
      r.R = t->R;
      r.G = t->G;
    }
  }
  const bool path = a.nc_p > 0;
  TileCfg& lead = path ? pt : r;
  const size_t tile_cap = t ? size_t(cap) : size_t(32 * 1024);
  auto lead_lds = [&](int R) {
    return path ? adjoint_path_lds_bytes(s.F, R, lead.G, Cm, lead.W, a.nc_p)
                : adjoint_reg_lds_bytes(s.F, R, lead.G, Cm, lead.W, a.lane_consts, 1);
  };
  while (lead.R > 64 * lead.K &&
         (size_t(s.F) * lead.R * 4 + size_t(lead.R) * 8 > tile_cap || lead_lds(lead.R) > size_t(cap)))
    lead.R /= 2;
  const int64_t Nr = (s.N + 255) / 256 * 256;  // a multiple of every tier's batch
  if (Nr < lead.R) lead.R = int(Nr);
  lead.R = std::max(256, lead.R / 256 * 256);
  // at most 64 programs per group: the path kernel holds a group's list one
  // entry per lane
  lead.G = std::max(1, std::min({lead.G, s.M, 64}));
  lead.n_groups = (s.M + lead.G - 1) / lead.G;
  // spans: enough blocks to fill the chip many times over (about 16K work
  // items, down to one row tile each).  The adjoint's cost per (program, tile)
  // varies with the program, so small items keep the waves of the last rounds
  // busy; each span costs one partial per (program, constant) in HBM.
  const int64_t tiles = (s.N + lead.R - 1) / lead.R;
  int64_t want = (16384 + lead.n_groups - 1) / lead.n_groups;
  want = std::max<int64_t>(1, std::min<int64_t>({want, tiles, int64_t(span_cap)}));
  lead.tiles_per_span = int((tiles + want - 1) / want);
  a.span_rows = int64_t(lead.tiles_per_span) * lead.R;
  a.n_spans = int((s.N + a.span_rows - 1) / a.span_rows);
  lead.n_spans = a.n_spans;
  if (path) {  // tier A: the path tile or a power-of-two fraction of it
    r.R = pt.R;
    while (r.R > 64 * r.K && adjoint_reg_lds_bytes(s.F, r.R, r.G, Cm, r.W, a.lane_consts, 1) > size_t(cap))
      r.R /= 2;
    r.G = std::max(1, std::min(r.G, s.M));
    r.n_groups = (s.M + r.G - 1) / r.G;
    r.n_spans = a.n_spans;
    r.tiles_per_span = int(a.span_rows / r.R);
  }

  // A program of L tokens has at most L - 1 tape entries (one per tree edge)
  // and at most C_max constants, so small shapes never reach tiers A, B or C.
  a.tape_cap = std::max(1, s.L_max - 1);
  // with a path tier, individuals whose partials overflow fall back to tier B
  // (or C for tapes longer than tier B's)
  const bool beyond_path = !path || Cm > a.nc_p;
  a.need_a = beyond_path;
  a.need_b = (beyond_path && a.tape_cap > a.tc_a && a.tc_b > a.tc_a) || path;
  // tier B: few individuals, each shared by the block's waves; G_b of them
  // per group, a bounded number of group slots per span (blocks loop)
  TileCfg& b = a.reg_b;
  b = r;
  b.K = 2;
  // with a path tier, tier B holds only the path tier's few fallen-back
  // programs: one per group, so that their flagged spans run in parallel
  // blocks rather than one after another in one block
  b.G = path ? 1 : std::max(1, std::min(4, s.M));
  while (b.G > 1 && adjoint_reg_lds_bytes(s.F, b.R, b.G, Cm, b.W, a.lane_consts, b.W) > size_t(cap)) --b.G;
  b.n_groups = std::min((s.M + b.G - 1) / b.G, 32);
  a.need_wide = (beyond_path &&
                 (a.tape_cap > std::max(a.tc_a, a.need_b ? a.tc_b : 0) || Cm > a.lane_consts)) ||
                (path && a.tape_cap > a.tc_b);

  // tier C: its tile must divide span_rows (powers of two <= r.R)
  TileCfg& w = a.wide;
  w.D = 8;
  bool ok = false;
  const int Ks[2] = {2, 1};
  const int Ws[3] = {4, 2, 1};
  const int Gs[3] = {16, 8, 4};
  for (int k : Ks) {
    for (int wv : Ws) {
      for (int rr = r.R; rr >= 64 * k && !ok; rr /= 2) {
        if (rr % (64 * k)) continue;
        for (int g : Gs) {
          if (adjoint_lds_bytes(s.F, rr, g, Cm, wv, k, a.tape_cap) <= size_t(cap)) {
            w.K = k;
            w.W = wv;
            w.R = rr;
            w.G = g;
            ok = true;
            break;
          }
        }
      }
      if (ok) break;
    }
    if (ok) break;
  }
  if (!ok) {  // smallest block; the caller reports the shape as unsupported
    w.K = 1;
    w.W = 1;
    w.R = 64;
    w.G = 1;
  }
  w.G = std::max(1, std::min(w.G, s.M));
  w.n_groups = std::min((s.M + w.G - 1) / w.G, 16);  // group slots per span; blocks loop
  w.n_spans = a.n_spans;
  w.tiles_per_span = int(a.span_rows / w.R);
  return a;
}

bool adjoint_plan_fits(const Shape& s, const AdjPlan& a) {
  const int cap = lds_limit_bytes() - 64;
  const int Cm = std::max(1, s.C_max);
  if (a.nc_p > 0 && adjoint_path_lds_bytes(s.F, a.path.R, a.path.G, Cm, a.path.W, a.nc_p) > size_t(cap))
    return false;
  if (a.need_a && adjoint_reg_lds_bytes(s.F, a.reg.R, a.reg.G, Cm, a.reg.W, a.lane_consts, 1) > size_t(cap))
    return false;
  if (a.need_b &&
      adjoint_reg_lds_bytes(s.F, a.reg_b.R, a.reg_b.G, Cm, a.reg_b.W, a.lane_consts, a.reg_b.W) > size_t(cap))
    return false;
  if (!a.need_wide) return true;
  return adjoint_lds_bytes(s.F, a.wide.R, a.wide.G, std::max(1, s.C_max), a.wide.W, a.wide.K,
                           a.tape_cap) <= size_t(cap) &&
         a.span_rows % a.wide.R == 0;
}

// ------------------------------------------------------------ graph cache
struct GraphKey {
  std::vector<uintptr_t> v;
  bool operator<(const GraphKey& o) const { return v < o.v; }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;

#define GG_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(GPGOMEA_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

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

struct ProfScope {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (g_prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
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

// Enqueue the whole fused pipeline on c.stream.
int enqueue_fused(const Call& c, const TileCfg& fc, const AdjPlan& ac) {
  const Layout l = layout_of(c.s);
  const bool fp64 = (c.s.flags & GPGOMEA_FP64_NODES) != 0;
  double* stats = reinterpret_cast<double*>(c.ws + l.stats);
  double* yscr = reinterpret_cast<double*>(c.ws + l.yscr);
  ProgMeta* meta = reinterpret_cast<ProgMeta*>(c.ws + l.meta);
  uint2* uops = reinterpret_cast<uint2*>(c.ws + l.uops);
  uint32_t* merges = reinterpret_cast<uint32_t*>(c.ws + l.merges);
  double* ab = reinterpret_cast<double*>(c.ws + l.ab);
  double* part = reinterpret_cast<double*>(c.ws + l.part);
  double* gpart = reinterpret_cast<double*>(c.ws + l.gpart);
  const DataArgs d{c.X, c.s.ldx, c.s.F, c.s.N, c.y};
  const int D = fp64 ? 8 : fc.D;
  GG_TIMED("ystats", launch_ystats(c.y, c.s.N, stats, yscr, c.stream));
  GG_TIMED("compile", launch_compile(c.ops, c.s.M, c.s.L_max, c.consts, c.s.C_max, c.s.F, D, l.U_stride,
                                     uops, meta, merges, l.MT, c.stream));
  GG_TIMED("probe", launch_probe(fp64, fc.K, D, uops, l.U_stride, meta, c.s.M, d, c.stream));
  const bool sse = c.aux != nullptr || !(c.s.flags & GPGOMEA_LINEAR_SCALING);
  if (c.s.flags & GPGOMEA_PLAIN) {
    unsigned* ticket = reinterpret_cast<unsigned*>(c.ws + l.ticket);
    double* pp = reinterpret_cast<double*>(c.ws + l.plain_part);
    GG_HIP(launch_fill_u32(ticket, 1, 0u, c.stream));
    for (int i = 0; i < c.s.M; ++i)
      GG_TIMED("plain_forward", launch_plain_forward(fp64, fc, i, uops, l.U_stride, meta, d, stats, pp, ticket,
                                                     c.s.flags, c.fitness, c.aux, c.status, ab, c.stream));
    if (c.with_grad) {
      // the plain form differentiates with the tape tiers only
      const Tuned tape_only{4, 1024, 16, 16, 0};
      const AdjPlan one = plan_adjoint(Shape{1, c.s.L_max, c.s.C_max, c.s.F, c.s.N, c.s.ldx, c.s.flags}, D,
                                       &tape_only, adj_span_cap(c.s));
      int* pcounts = reinterpret_cast<int*>(c.ws + l.adjl);
      int* list0 = pcounts + 4 * size_t(c.s.M);
      GG_TIMED("plain_tiers", launch_adjoint_tier_flags(one, meta, ab, c.s.M, pcounts, list0, c.stream));
      for (int i = 0; i < c.s.M; ++i) {
        const uint2* ui = uops + size_t(i) * l.U_stride;
        double* gi = gpart + size_t(i) * one.n_spans * c.s.C_max;
        const double* abi = ab + 2 * size_t(i);
        const int* ci = pcounts + 4 * size_t(i);
        if (one.need_a)
          GG_TIMED("plain_adjoint", launch_adjoint_reg(one, 0, ui, l.U_stride, meta + i, 1, c.s.C_max, d,
                                                       stats, abi, gi, list0, ci + 0, nullptr, nullptr,
                                                       c.stream));
        if (one.need_b)
          GG_TIMED("plain_adjoint", launch_adjoint_reg(one, 1, ui, l.U_stride, meta + i, 1, c.s.C_max, d,
                                                       stats, abi, gi, list0, ci + 1, nullptr, nullptr,
                                                       c.stream));
        if (one.need_wide)
          GG_TIMED("plain_adjoint", launch_adjoint_lds(one, ui, l.U_stride, meta + i, 1, c.s.C_max, d, stats,
                                                       abi, gi, list0, ci + 2, nullptr, nullptr, c.stream));
      }
      GG_TIMED("grad_finalize", launch_grad_finalize(meta, c.s.M, c.s.C_max, gpart, one.n_spans, stats, ab,
                                                     c.s.flags, c.status, c.grad, c.stream));
    }
    return GPGOMEA_OK;
  }
  GG_TIMED("fused_forward", launch_fused_forward(fp64, fc, uops, l.U_stride, meta, c.s.M, d, stats, part, sse,
                                                 c.stream));
  GG_TIMED("finalize", launch_finalize(meta, c.s.M, part, fc.n_spans, stats, c.s.flags, c.fitness, c.aux,
                                       c.status, ab, c.stream));
  if (c.with_grad) {
    int* lists = reinterpret_cast<int*>(c.ws + l.adjl);
    int* counts = lists + 4 * size_t(c.s.M);
    const size_t M = size_t(c.s.M);
    int* redo = counts + 4;  // path fallback flags [M], right after the four counts
    uint8_t* redo_span = reinterpret_cast<uint8_t*>(c.ws + l.redo_span);
    int* rd = ac.nc_p > 0 ? redo : nullptr;  // the tape tiers' fallback flags
    uint8_t* rs = ac.nc_p > 0 ? redo_span : nullptr;
    GG_TIMED("adjoint_partition", launch_adjoint_partition(ac, meta, ab, c.s.M, lists, counts, rd, c.stream));
    if (ac.nc_p > 0) {
      GG_TIMED("adjoint_path", launch_adjoint_path(ac, uops, l.U_stride, meta, c.s.M, c.s.C_max, d, stats, ab,
                                                   gpart, merges, l.MT, redo, redo_span, lists, counts,
                                                   c.stream));
    }
    if (ac.need_a)
      GG_TIMED("adjoint_reg", launch_adjoint_reg(ac, 0, uops, l.U_stride, meta, c.s.M, c.s.C_max, d, stats,
                                                 ab, gpart, lists, counts + 0, nullptr, nullptr, c.stream));
    if (ac.need_b)
      GG_TIMED("adjoint_reg_b", launch_adjoint_reg(ac, 1, uops, l.U_stride, meta, c.s.M, c.s.C_max, d, stats,
                                                   ab, gpart, lists + M, counts + 1, rd, rs, c.stream));
    if (ac.need_wide)
      GG_TIMED("adjoint_lds", launch_adjoint_lds(ac, uops, l.U_stride, meta, c.s.M, c.s.C_max, d, stats, ab,
                                                 gpart, lists + 2 * M, counts + 2, rd, rs, c.stream));
    GG_TIMED("grad_finalize", launch_grad_finalize(meta, c.s.M, c.s.C_max, gpart, ac.n_spans, stats, ab,
                                                   c.s.flags, c.status, c.grad, c.stream));
  }
  return GPGOMEA_OK;
}

int run_call(const Call& c) {
  (void)hipGetLastError();  // launches below report their own errors only
  TileCfg fc;
  AdjPlan ac;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(c.s, false));
    fc = plan_forward(c.s, it == g_tuned.end() ? nullptr : &it->second);
    auto ia = g_tuned_adj.find(tune_key(c.s, true));
    ac = plan_adjoint(c.s, fc.D, ia == g_tuned_adj.end() ? nullptr : &ia->second, adj_span_cap(c.s));
  }
  if (c.with_grad && !adjoint_plan_fits(c.s, ac))
    return fail(GPGOMEA_E_UNSUPPORTED, "no adjoint block fits LDS for L_max=%d, F=%d", c.s.L_max, c.s.F);
  // the forward kernel's per-group metadata table and the path kernel's
  // lane-held group list have 64 entries
  if (fc.G > 64 || (c.with_grad && ac.nc_p > 0 && ac.path.G > 64))
    return fail(GPGOMEA_E_UNSUPPORTED, "group of more than 64 programs (forward %d, path %d)", fc.G,
                ac.path.G);
  const bool graph =
      !(c.s.flags & (GPGOMEA_NO_GRAPH | GPGOMEA_PLAIN)) && c.stream != nullptr && !g_prof;
  if (!graph) return enqueue_fused(c, fc, ac);

  GraphKey key;
  key.v = {uintptr_t(c.with_grad), uintptr_t(c.ops), uintptr_t(c.consts), uintptr_t(c.X),
           uintptr_t(c.y), uintptr_t(c.fitness), uintptr_t(c.aux), uintptr_t(c.grad),
           uintptr_t(c.status), uintptr_t(c.ws), uintptr_t(c.s.M), uintptr_t(c.s.L_max),
           uintptr_t(c.s.C_max), uintptr_t(c.s.F), uintptr_t(c.s.N), uintptr_t(c.s.ldx),
           uintptr_t(c.s.flags), uintptr_t(fc.K), uintptr_t(fc.R), uintptr_t(fc.G),
           uintptr_t(ac.reg.R), uintptr_t(ac.reg.G), uintptr_t(ac.reg.K), uintptr_t(ac.tc_a),
           uintptr_t(ac.n_spans), uintptr_t(ac.nc_p), uintptr_t(ac.path.K), uintptr_t(ac.path.R),
           uintptr_t(ac.path.G)};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) exec = it->second;
  }
  if (!exec) {
    GG_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_fused(c, fc, ac);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c.stream, &g);
    if (rc != GPGOMEA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(GPGOMEA_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(GPGOMEA_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graphs[key] = exec;
  }
  GG_HIP(hipGraphLaunch(exec, c.stream));
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

extern "C" int gpgomea_grad_consts(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                                   int32_t C_max, const float* X, int32_t F, int64_t N,
                                   int64_t ldx, const float* y, uint32_t flags, double* fitness,
                                   double* aux, double* grad, int8_t* status, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  const Shape s{M, L_max, C_max, F, N, ldx, flags};
  int rc = check_call(s, ops, consts, X, y, fitness, workspace, workspace_bytes);
  if (rc) return rc;
  if (!grad) return fail(GPGOMEA_E_ARG, "grad is NULL");
  if (flags & GPGOMEA_FP64_NODES)
    return fail(GPGOMEA_E_UNSUPPORTED, "the adjoint runs in binary32 nodes only");
  Call c{s, ops, consts, X, y, fitness, aux, grad, status, static_cast<char*>(workspace),
         static_cast<hipStream_t>(stream), true};
  return run_call(c);
}

extern "C" int gpgomea_clear_graphs(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
  g_graphs.clear();
  return GPGOMEA_OK;
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
                "\"Mcls\": %d, \"grad\": %d, \"K\": %d, \"R\": %d, \"G\": %d, \"TC\": %d, "
                "\"TF\": %d}",
                table, k.fp64, k.Lcls, k.F, k.Ncls, k.Mcls, k.grad, t.K, t.R, t.G, t.TC, t.F);
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
    if (!json_int(line, "TC", &t.TC)) t.TC = 0;
    if (!json_int(line, "TF", &t.F)) t.F = 0;
    if (t.K < 1 || t.R < 64 || t.G < 1) continue;
    (fwd ? g_tuned : g_tuned_adj)[k] = t;
    ++n;
  }
  if (n_read) *n_read = n;
  return true;
}

bool write_tuning(const char* path) {
  std::ostringstream o;
  o << "{\"gpgomea_tuning\": 1, \"entries\": [\n";
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

  // forward: rows per lane K, rows per LDS tile R, individuals per block G
  const int Ks_f[2] = {8, 4};
  const int Rs_f[5] = {256, 512, 1024, 2048, 4096};
  const int Gs_f[5] = {4, 8, 16, 32, 64};
  const int lds = lds_limit_bytes();
  Tuned best_f{0, 0, 0, 0, 0};
  float best_f_ms = 1e30f;
  TileCfg fc_best;
  for (int k : Ks_f) {
    if (fp64 && k != 4) continue;
    for (int r : Rs_f) {
      if (r < 64 * k) continue;
      for (int g : Gs_f) {
        if (forward_lds_bytes(F, r, g) > size_t(lds)) continue;
        const Tuned t{k, r, g, 0, 0};
        const TileCfg fc = plan_forward(st, &t);
        const AdjPlan ac = plan_adjoint(st, fc.D, nullptr, adj_span_cap(s));
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

  if (with_grad) {
    c.with_grad = true;
    c.grad = grad;
    // (K, NC) of the path tier, or (K, TC) of tier A without one (F = 0)
    struct Cand {
      int K, TC, F;
    };
    const Cand cands[9] = {{4, 0, 16}, {4, 0, 12}, {4, 0, 8}, {8, 0, 8}, {2, 0, 16},
                           {2, 0, 32}, {4, 16, 0}, {2, 16, 0}, {2, 32, 0}};
    const int Rs_a[5] = {256, 512, 768, 1024, 2048};
    const int Gs_a[4] = {4, 8, 16, 32};
    Tuned best_a{0, 0, 0, 0, 0};
    float best_a_ms = 1e30f;
    for (const Cand& cd : cands) {
      if (cd.F > 0 && C_max == 0) continue;
      for (int r : Rs_a) {
        for (int g : Gs_a) {
          const Tuned t{cd.K, r, g, cd.TC, cd.F};
          const AdjPlan ac = plan_adjoint(st, fc_best.D, &t, adj_span_cap(s));
          const int lead_r = ac.nc_p > 0 ? ac.path.R : ac.reg.R;
          if (lead_r != r || !adjoint_plan_fits(st, ac)) continue;  // clamped: same as another
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
    if (best_a.K) {
      g_tuned_adj[tune_key(s, true)] = best_a;
      len += std::snprintf(desc + len, sizeof(desc) - size_t(len),
                           "; fitness+gradient with adjoint K=%d TC=%d NC=%d R=%d G=%d (%.3f ms)",
                           best_a.K, best_a.TC, best_a.F, best_a.R, best_a.G, double(best_a_ms));
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

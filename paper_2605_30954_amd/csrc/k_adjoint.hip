// Reverse-mode gradient of the fitness with respect to every constant.
//
// With linear scaling the optimal (a, b) have zero partials (envelope
// theorem), so  d LS-MSE / d c_j = (2b/N) sum_r (a + b p_r - y_r) dp_r/dc_j;
// without it  d MSE / d c_j = (2/N) sum_r (p_r - y_r) dp_r/dc_j.  Both are
// written  (2 s1/N) sum_r (s0 + s1 p_r - y_r) dp_r/dc_j  with (s0, s1) = (a, b)
// or (0, 1), taken from the forward pass (which must run first).
//
// Per row tile and individual a wave runs the program forward over K rows per
// lane, storing every local partial the reverse sweep will need on a tape
// (the tree's values are recomputed per tile rather than kept from the
// forward pass), seeds the output adjoint with the residual, and walks the
// uops backwards.  A tree node has exactly one parent, so adjoints never
// accumulate except at constants.
//
// The individuals are split into tiers by the size of their tape (the
// partials the reverse sweep needs) and their constant count; a partition
// kernel writes one list per tier after the forward pass, and one kernel per
// tier walks its own list:
//  * k_adj_reg, tier A and tier B: the tape is a register array of TC entries
//    per row addressed by a wave-uniform index (indirect VGPR addressing, no
//    LDS); tier A uses a small tape (most programs), tier B TC = 32.  Every
//    lane sums its own rows' constant adjoints in an LDS column (binary32 over
//    the R/64 rows of one tile); once per (tile, individual) the wave adds the
//    64 columns in binary64.  LDS holds little more than the row tile, so
//    several blocks share a CU.
//  * k_adj_lds, tier C (longer tapes, or more constants than columns): the
//    tape lives in wave-private LDS; all waves of a block share one individual
//    and reduce its constant adjoints across the wave (binary64) per batch.
// Every kernel cuts the rows into the same spans, so every (individual, span)
// partial is written exactly once.
#include <hip/hip_runtime.h>

#include "interp.h"
#include "kernels.h"

namespace gg {

struct AdjParams {
  const uint2* uops;
  int U_stride;
  const ProgMeta* meta;
  int M, C_max;
  const float* X;
  int64_t ldx;
  int F;
  int64_t N;
  const float* y;
  const double* stats;
  const double* ab;
  double* gpart;      // [M][n_spans][C_max]
  const int* list;    // this tier's individuals, in batch order
  const int* count;   // their number
  int R, G, n_groups, n_spans;
  int64_t span_rows;  // rows per span (common to every tier)
  int tape_cap;       // LDS tape entries per wave (tier C)
  int lane_consts;    // CC: constant columns per wave (register tiers)
  const uint32_t* merges;  // [M][MT] flush events (path tier)
  int MT;
  int* redo;               // [M] path tier: set when an individual's partials are not finite
  uint8_t* redo_span;      // [M][n_spans] ... and for which spans; the tape tiers then
                           // redo only those spans of a flagged individual
  int* fb_lists;           // path tier: the tier lists [4][M] and counts [4], to which
  int* fb_counts;          // a flagged individual is appended (tier B, or C)
  int tc_b;                // tier B's tape entries
};

// A tape tier skips span s of individual i when i fell back from the path
// tier and the path tier's partials of span s are finite (they are kept).
__device__ inline bool keep_path_span(const AdjParams& p, int i, int span) {
  return p.redo != nullptr && p.redo[i] != 0 && p.redo_span[size_t(i) * p.n_spans + span] == 0;
}

// A tape tier has nothing to do on span s for a group whose individuals all
// keep the path tier's partials of s (the fallback tier holds only fallen-back
// individuals, flagged on few spans): the block skips the span, staging
// included.  Block-uniform (global data only).
__device__ inline bool group_keeps_span(const AdjParams& p, int base, int Gn, int span) {
  if (p.redo == nullptr) return false;
  for (int jj = 0; jj < Gn; ++jj)
    if (!keep_path_span(p, p.list[base + jj], span)) return false;
  return true;
}

// Tier of an individual: -1 no gradient work (bad program, non-finite, b = 0
// or no constant), 3 path forward mode (at most ncP constants), 0 register
// tape A, 1 register tape B, 2 LDS tape.
constexpr int kTiers = 4;
constexpr int kTierPath = 3;
__device__ inline int adj_tier(const ProgMeta& pm, double s1, int tcA, int tcB, int CC, int ncP) {
  if (pm.status != 0 || s1 == 0.0 || pm.n_const <= 0) return -1;
  if (pm.n_const <= ncP) return kTierPath;
  if (pm.n_const <= CC && pm.n_tape <= tcA) return 0;
  if (pm.n_const <= CC && pm.n_tape <= tcB) return 1;
  return 2;
}

// One block: thread t classifies a contiguous chunk of individuals; a
// block-wide scan of the per-thread counts gives each chunk its offsets, so
// the lists keep batch order (deterministic).
constexpr int kPartThreads = 1024;
__global__ __launch_bounds__(kPartThreads) void k_adj_partition(
    const ProgMeta* __restrict__ meta, const double* __restrict__ ab, int M, int tcA, int tcB,
    int CC, int ncP, int* __restrict__ lists, int* __restrict__ counts, int* __restrict__ redo) {
  __shared__ int sc[kTiers][kPartThreads];
  const int t = threadIdx.x;
  const int chunk = (M + kPartThreads - 1) / kPartThreads;
  const int lo = min(M, t * chunk), hi = min(M, lo + chunk);
  int n[kTiers] = {0, 0, 0, 0};
  for (int i = lo; i < hi; ++i) {
    if (redo) redo[i] = 0;  // the path tier's fallback flags start clear
    const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ncP);
#pragma unroll
    for (int q = 0; q < kTiers; ++q) n[q] += k == q;
  }
#pragma unroll
  for (int q = 0; q < kTiers; ++q) sc[q][t] = n[q];
  __syncthreads();
  for (int o = 1; o < kPartThreads; o <<= 1) {  // inclusive Hillis-Steele scan
    int a[kTiers] = {0, 0, 0, 0};
    if (t >= o) {
#pragma unroll
      for (int q = 0; q < kTiers; ++q) a[q] = sc[q][t - o];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTiers; ++q) sc[q][t] += a[q];
    __syncthreads();
  }
  int w[kTiers];
#pragma unroll
  for (int q = 0; q < kTiers; ++q) w[q] = sc[q][t] - n[q];  // exclusive offsets
  for (int i = lo; i < hi; ++i) {
    const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ncP);
#pragma unroll
    for (int q = 0; q < kTiers; ++q)
      if (k == q) lists[size_t(q) * M + w[q]++] = i;
  }
  if (t == kPartThreads - 1) {
#pragma unroll
    for (int q = 0; q < kTiers; ++q) counts[q] = sc[q][t];
  }
}

// Wave-private tape in LDS: entry e, lane l at base[(e*64 + l)*K].
template <int K>
struct LdsTape {
  using V = typename VecT<float, K>::type;
  float* base;
  int lane;
  __device__ inline float* at(int e) const { return base + (size_t(e) * 64 + lane) * K; }
  __device__ inline void put(int e, const V& v) {
    float* q = at(e);
    if constexpr (K == 4) {
      *reinterpret_cast<float4*>(q) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (K == 2) {
      *reinterpret_cast<float2*>(q) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) q[j] = v[j];
    }
  }
  __device__ inline V get(int e) const {
    const float* q = at(e);
    V v;
    if constexpr (K == 4) {
      const float4 t = *reinterpret_cast<const float4*>(q);
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (K == 2) {
      const float2 t = *reinterpret_cast<const float2*>(q);
      v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = q[j];
    }
    return v;
  }
};

// Tape of TC entries in VGPRs: one TC-float vector per row of the lane (a
// vector register tuple holds at most 32 floats, and only a vector that fits
// one tuple is addressed in registers).  The entry index is wave-uniform (it
// follows the uop stream), so the compiler reads and writes the tuples with
// s_set_gpr_idx moves instead of scratch memory.  The path tier's array T is
// a RegTape indexed only by compile-time entries (fixed registers).
template <int K, int TC>
struct RegTape {
  static_assert(TC <= 32, "a tape row must fit one VGPR tuple");
  using V = typename VecT<float, K>::type;
  typedef float A __attribute__((ext_vector_type(TC)));
  A a[K];
  __device__ inline void put(int e, const V& v) {
#pragma unroll
    for (int j = 0; j < K; ++j) a[j][e] = v[j];
  }
  __device__ inline V get(int e) const {
    V v;
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = a[j][e];
    return v;
  }
};

// Value and local partials of a non-cheap operator on K rows: fa = d result /
// d acc operand, fs = d result / d src operand (unary operators leave fs
// untouched).  NOP leaves acc and the partials as they are.
template <int K>
__device__ inline void op_partials(uint32_t op, typename VecT<float, K>::type& acc,
                                   const typename VecT<float, K>::type& t,
                                   typename VecT<float, K>::type& fa,
                                   typename VecT<float, K>::type& fs) {
  using P = Prot<float>;
  using Dv = Deriv<float>;
  switch (op) {
    case UOP_DIV:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::div(acc[j], t[j]);
        float da, ds;
        Dv::ddiv(acc[j], t[j], v, da, ds);
        acc[j] = v; fa[j] = da; fs[j] = ds;
      }
      GG_BRANCH();
      break;
    case UOP_RDIV:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::div(t[j], acc[j]);
        float da, ds;
        Dv::ddiv(t[j], acc[j], v, ds, da);
        acc[j] = v; fa[j] = da; fs[j] = ds;
      }
      GG_BRANCH();
      break;
    case UOP_POW:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::pow_(acc[j], t[j]);
        float da, ds;
        Dv::dpow(acc[j], t[j], v, da, ds);
        acc[j] = v; fa[j] = da; fs[j] = ds;
      }
      GG_BRANCH();
      break;
    case UOP_RPOW:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::pow_(t[j], acc[j]);
        float da, ds;
        Dv::dpow(t[j], acc[j], v, ds, da);
        acc[j] = v; fa[j] = da; fs[j] = ds;
      }
      GG_BRANCH();
      break;
    case UOP_SIN:
#pragma unroll
      for (int j = 0; j < K; ++j) { fa[j] = Dv::dsin(acc[j]); acc[j] = P::sin_(acc[j]); }
      GG_BRANCH();
      break;
    case UOP_COS:
#pragma unroll
      for (int j = 0; j < K; ++j) { fa[j] = Dv::dcos(acc[j]); acc[j] = P::cos_(acc[j]); }
      GG_BRANCH();
      break;
    case UOP_SQ:
#pragma unroll
      for (int j = 0; j < K; ++j) { fa[j] = 2.0f * acc[j]; acc[j] = acc[j] * acc[j]; }
      GG_BRANCH();
      break;
    case UOP_SQRT:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::sqrt_(acc[j]);
        fa[j] = Dv::dsqrt(acc[j], v);
        acc[j] = v;
      }
      GG_BRANCH();
      break;
    case UOP_EXP:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = P::exp_(acc[j]);
        fa[j] = Dv::dexp(acc[j], v);
        acc[j] = v;
      }
      GG_BRANCH();
      break;
    case UOP_LOG:
#pragma unroll
      for (int j = 0; j < K; ++j) { fa[j] = Dv::dlog(acc[j]); acc[j] = P::log_(acc[j]); }
      GG_BRANCH();
      break;
    default:
      GG_BRANCH();
      break;
  }
}

// Forward sweep with the tape (float nodes).  Same values as run_program; in
// addition each uop stores d(result)/d(acc operand) and d(result)/d(src
// operand) when the reverse sweep needs them (tape_acc / tape_src), acc's
// entry first.
template <int K, int D, class Src, class Tape>
__device__ inline typename VecT<float, K>::type run_forward_taped(
    const Src& prog, const float* __restrict__ xt, int rstride, int lrow, Tape& tape) {
  using V = typename VecT<float, K>::type;
  Slots<V, D> st;
  V acc = 0.0f, t = 0.0f, pre = 0.0f;
  const float* __restrict__ xl = xt + lrow;
  uint2 cur = prog.at(0);
  prefetch_operand<float, K>(cur.x, xl, rstride, pre);
  int pc = 0, tp = 0;
#pragma unroll 1
  while (cur.x != UOP_END_HDR) {
    const uint2 nxt = prog.at(pc + 1);
    const uint32_t h = cur.x;
    operand_stage<float, K, D>(h, f32_of(cur.y), xl, rstride, acc, t, pre, st);
    prefetch_operand<float, K>(nxt.x, xl, rstride, pre);  // next uop's first variable
    if (h & U_CHEAP) {  // ADD 1, SUB 2, RSUB 3, MUL 4
      if (h & 4u) {
        // d(acc*t)/d acc = t (a constant src needs no tape), d/d t = acc
        if ((h & (HDR_ADJ_ACC | U_SC)) == HDR_ADJ_ACC) { tape.put(tp, t); ++tp; GG_BRANCH(); }
        if (h & HDR_ADJ_SRC) { tape.put(tp, acc); ++tp; GG_BRANCH(); }
        acc = acc * t;
        GG_BRANCH();
      } else if (h & 2u) {
        if (h & 1u) { acc = t - acc; GG_BRANCH(); }
        else { acc = acc - t; GG_BRANCH(); }
        GG_BRANCH();
      } else {
        acc = acc + t;
        GG_BRANCH();
      }
      GG_BRANCH();
    } else if (h & (HDR_ADJ_ACC | HDR_ADJ_SRC)) {  // a constant below: value and partials
      V fa = 1.0f, fs = 1.0f;
      op_partials<K>(uop_op(h), acc, t, fa, fs);
      if ((h & HDR_ADJ_ACC) && uop_op(h) != UOP_NOP) { tape.put(tp, fa); ++tp; GG_BRANCH(); }
      if (h & HDR_ADJ_SRC) { tape.put(tp, fs); ++tp; GG_BRANCH(); }
      GG_BRANCH();
    } else {
      op_value<float, K>(uop_op(h), acc, t);
      GG_BRANCH();
    }
    cur = nxt;
    ++pc;
  }
  return acc;
}

// Sum over the wave of this lane's values on valid rows, in binary64.  kv is
// the number of the tile's valid rows from the lane's first row on, so element
// j is valid iff row_off(j) < kv (padding rows are excluded: their adjoints may
// be NaN after multiplying a zero by an infinite partial).
template <int K>
__device__ inline double wave_total(const typename VecT<float, K>::type& v, int kv) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) s += row_off<K>(j) < kv ? double(v[j]) : 0.0;
  return wave_sum(s);
}

// Where constant adjoints go.  WaveSink: reduced across the wave at once and
// added to the individual's binary64 accumulator (same value on every lane).
// LaneSink: this lane's rows summed into its own LDS column (entry c at
// col[c * kColStride]); the wave reduces the columns later.
constexpr int kColStride = 65;  // 64 lanes + 1: column reads are bank-conflict free

struct WaveSink {
  double* gacc;
  template <class V, int K>
  __device__ inline void add(uint32_t c, const V& v, int kv) {
    const double s = wave_total<K>(v, kv);
    gacc[c] += s;
  }
};
struct LaneSink {
  float* col;
  // FULL: every row of the batch is valid (no per-element test)
  template <class V, int K, bool FULL = false>
  __device__ inline void add(uint32_t c, const V& v, int kv) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) s += (FULL || row_off<K>(j) < kv) ? v[j] : 0.0f;
    // read-modify-write inside the LDS unit (ds_add_f32, no return value, so
    // nothing waits on it); only this lane writes this word, in program order
    (void)atomicAdd(&col[c * kColStride], s);
  }
};

// Path tier sink: g * T[e] of this lane's valid rows added into the LDS column
// of constant e, for e < nc (wave-uniform), expanded over the compile-time
// entry index so T is read from fixed registers.
template <int E, int K, int NC, bool FULL>
__device__ inline void sink_path(LaneSink& sink, const RegTape<K, NC>& T,
                                 const typename VecT<float, K>::type& g, int nc, int kv) {
  if constexpr (E < NC) {
    if (E >= nc) return;
    sink.template add<typename VecT<float, K>::type, K, FULL>(uint32_t(E), g * T.get(E), kv);
    sink_path<E + 1, K, NC, FULL>(sink, T, g, nc, kv);
  }
}

// Reverse sweep.  g = adjoint of the program output per row (zero on padding
// rows); kv = valid rows of the tile from this lane's first row on (element j
// is valid iff row_off(j) < kv).  Uops with no constant below them and
// no push are skipped with one test.
template <int K, int D, class Src, class Tape, class Sink>
__device__ inline void run_reverse(const Src& prog, int n_uops, int n_tape,
                                   typename VecT<float, K>::type g, const Tape& tape, Sink& sink,
                                   int kv) {
  using V = typename VecT<float, K>::type;
  Slots<V, D> gs;  // adjoints of pushed subtrees
  V gsrc = 0.0f;
  int tp = n_tape;
  uint2 nxt = prog.at(n_uops >= 2 ? n_uops - 2 : 0);
#pragma unroll 1
  for (int pc = n_uops - 2; pc >= 0; --pc) {
    const uint2 u = nxt;
    nxt = prog.at(pc > 0 ? pc - 1 : 0);
    const uint32_t h = u.x;
    if (h & (HDR_ADJ_ACC | HDR_ADJ_SRC | HDR_PUSH)) {
      if (h & HDR_ADJ_SRC) {  // d result / d src
        if (h & U_CHEAP) {
          if (h & 4u) { --tp; gsrc = g * tape.get(tp); GG_BRANCH(); }       // MUL
          else if ((h & 3u) == 2u) { gsrc = -g; GG_BRANCH(); }              // SUB
          else { gsrc = g; GG_BRANCH(); }                                   // ADD, RSUB
          GG_BRANCH();
        } else {
          --tp;
          gsrc = g * tape.get(tp);  // DIV, RDIV, POW, RPOW
          GG_BRANCH();
        }
        if (h & U_SC) { sink.template add<V, K>(uop_arg2(h), gsrc, kv); GG_BRANCH(); }
        else if (h & U_SP) { gs.put(uop_arg2(h), gsrc); GG_BRANCH(); }
        GG_BRANCH();
      }
      if (h & HDR_ADJ_ACC) {  // d result / d acc operand
        if (h & U_CHEAP) {
          if (h & 4u) {  // MUL: the src factor (a constant src is the payload)
            if (h & U_SC) { g = g * f32_of(u.y); GG_BRANCH(); }
            else { --tp; g = g * tape.get(tp); GG_BRANCH(); }
            GG_BRANCH();
          } else if ((h & 3u) == 3u) {
            g = -g;  // RSUB
            GG_BRANCH();
          }
          GG_BRANCH();
        } else if (uop_op(h) != UOP_NOP) {
          --tp;
          g = g * tape.get(tp);
          GG_BRANCH();
        }
        if (h & U_LDC) { sink.template add<V, K>(uop_arg2(h), g, kv); GG_BRANCH(); }
        GG_BRANCH();
      }
      if (h & HDR_PUSH) { gs.get(uop_push_slot(h), g); GG_BRANCH(); }
      GG_BRANCH();
    }
  }
}

// ------------------------------------------------------- path forward mode
// Forward accumulation for a tree without a tape.  d p / d c_j is the product
// of the local partials on the path from constant j to the root.  The
// constants of any subtree are contiguous in postfix order, so every value
// carries one "pending" factor per row, the product of the partials since its
// constants were last folded into a register array T (entry j: the product
// from constant j up to that point).  A uop with a constant in one operand
// only multiplies that operand's pending factor by its partial.  The pending
// factor is folded into T over the operand's constant range at a merge (a uop
// whose two operands both hold constants; each operand with its own partial)
// and at the push of a value that holds constants, after which the factor
// restarts at 1; a single constant's entry is assigned the first time.  At
// the root, d p / d c_j = pending * T[j].
// The compile step lists the flush events in uop order (lane m of `mt` holds
// event m): each side is lo | n << 7 | assign << 14, a merge's src side in
// bits 15..29.
// Chain-rule product f * p in which a factor f of exactly 0 gives 0 whatever
// p holds.  A local partial of 0 (an operator's protected region, the clamp
// of exp) ends every derivative path through it; forming the product from the
// leaves up can first overflow p to infinity (a huge inner partial), and the
// plain product 0 * inf would be NaN where the derivative is 0.
template <int K>
__device__ inline typename VecT<float, K>::type zmul(const typename VecT<float, K>::type& f,
                                                     const typename VecT<float, K>::type& p) {
  typename VecT<float, K>::type r;
#pragma unroll
  for (int j = 0; j < K; ++j) r[j] = f[j] == 0.0f ? 0.0f : f[j] * p[j];
  return r;
}

// T[e] *= f for e in [lo, hi), expanded over the compile-time entry index E
// (direct register operands, no relative addressing): two uniform compares per
// entry up to the range's end.
template <int E, int K, int NC>
__device__ inline void scale_range(RegTape<K, NC>& T, uint32_t lo, uint32_t hi,
                                   const typename VecT<float, K>::type& f) {
  if constexpr (E < NC) {
    if (uint32_t(E) >= hi) return;
    if (uint32_t(E) >= lo) {
      T.put(E, zmul<K>(f, T.get(E)));
      GG_BRANCH();
    }
    scale_range<E + 1, K, NC>(T, lo, hi, f);
  }
}
// T[e] = f for e = lo (no entry when lo >= NC), expanded like scale_range.
template <int E, int K, int NC>
__device__ inline void assign_at(RegTape<K, NC>& T, uint32_t lo,
                                 const typename VecT<float, K>::type& f) {
  if constexpr (E < NC) {
    if (uint32_t(E) == lo) {
      T.put(E, f);
      GG_BRANCH();
      return;
    }
    assign_at<E + 1, K, NC>(T, lo, f);
  }
}

template <int K, int NC>
__device__ inline void path_flush(RegTape<K, NC>& T, uint32_t side,
                                  const typename VecT<float, K>::type& f) {
  const uint32_t lo = side & 127u, n = (side >> 7) & 127u;
  if (side & (1u << 14)) {
    assign_at<0, K, NC>(T, lo, f);
    GG_BRANCH();
  } else {
    scale_range<0, K, NC>(T, lo, lo + n, f);
    GG_BRANCH();
  }
}

template <int K, int D, int NC, class Src>
__device__ inline typename VecT<float, K>::type run_forward_path(
    const Src& prog, uint32_t mt, const float* __restrict__ xt, int rstride, int lrow,
    RegTape<K, NC>& T, typename VecT<float, K>::type& p) {
  using V = typename VecT<float, K>::type;
  Slots<V, D> st;
  V acc = 0.0f, t = 0.0f, pre = 0.0f;
  p = 1.0f;
  // a lone constant whose value is never pushed is never flushed: its entry
  // stays 1 (with two or more constants every entry is written by a merge)
  T.put(0, V(1.0f));
  int mi = 0;
  const float* __restrict__ xl = xt + lrow;
  uint2 cur = prog.at(0);
  prefetch_operand<float, K>(cur.x, xl, rstride, pre);
  int pc = 0;
#pragma unroll 1
  while (cur.x != UOP_END_HDR) {
    const uint2 nxt = prog.at(pc + 1);
    const uint32_t h = cur.x;
    const float c = f32_of(cur.y);
    // operands (a constant and a popped value start with pending factor 1)
    if (h & (U_LDV | U_LDC)) {
      if (h & HDR_PUSH) {
        st.put(uop_push_slot(h), acc);
        if (h & U_PUSHC) {
          const uint32_t ev = uint32_t(__builtin_amdgcn_readlane(int(mt), mi));
          ++mi;
          path_flush<K, NC>(T, ev, p);
          GG_BRANCH();
        }
        GG_BRANCH();
      }
      if (h & U_LDV) {
        acc = pre;
        GG_BRANCH();
      } else {
        acc = bcast<float, K>(c);
        p = 1.0f;
        GG_BRANCH();
      }
      GG_BRANCH();
    }
    if (h & U_TPRE) {
      t = pre;
      GG_BRANCH();
    } else if (h & U_SC) {
      t = bcast<float, K>(c);
      GG_BRANCH();
    } else if (h & U_TX2) {
      t = lds_rows<float, K>(xl + uop_arg2(h) * rstride);
      GG_BRANCH();
    } else if (h & U_SP) {
      st.get(uop_arg2(h), t);
      GG_BRANCH();
    }
    prefetch_operand<float, K>(nxt.x, xl, rstride, pre);
    if ((h & (U_CHEAP | HDR_ADJ_SRC)) == U_CHEAP) {
      // ADD 1, SUB 2, RSUB 3, MUL 4 with no constant in the src operand: the
      // pending factor follows the acc operand (d/d acc is 1, -1 or t).  When
      // the acc operand holds no constant either, p is dead: it is reset
      // before it is next read (a constant load, or a src operand that holds
      // a constant)
      if (h & 4u) {
        p = t * p;
        acc = acc * t;
        GG_BRANCH();
      } else if (h & 2u) {
        if (h & 1u) { p = -p; acc = t - acc; GG_BRANCH(); }
        else { acc = acc - t; GG_BRANCH(); }
        GG_BRANCH();
      } else {
        acc = acc + t;
        GG_BRANCH();
      }
      GG_BRANCH();
    } else if (h & (HDR_ADJ_ACC | HDR_ADJ_SRC)) {
      V fa = 1.0f, fs = 1.0f;  // d result / d acc operand, / d src operand
      if (h & U_CHEAP) {
        if (h & 4u) {
          fa = t;
          fs = acc;
          acc = acc * t;
          GG_BRANCH();
        } else if (h & 2u) {
          if (h & 1u) { fa = -1.0f; acc = t - acc; GG_BRANCH(); }
          else { fs = -1.0f; acc = acc - t; GG_BRANCH(); }
          GG_BRANCH();
        } else {
          acc = acc + t;
          GG_BRANCH();
        }
        GG_BRANCH();
      } else {
        op_partials<K>(uop_op(h), acc, t, fa, fs);
        GG_BRANCH();
      }
      if (h & HDR_ADJ_ACC) {
        if (h & HDR_ADJ_SRC) {  // merge
          const uint32_t ev = uint32_t(__builtin_amdgcn_readlane(int(mt), mi));
          ++mi;
          path_flush<K, NC>(T, ev & 0x7fffu, zmul<K>(fa, p));
          path_flush<K, NC>(T, ev >> 15, fs);
          p = 1.0f;
          GG_BRANCH();
        } else {
          p = zmul<K>(fa, p);
          GG_BRANCH();
        }
        GG_BRANCH();
      } else {
        p = fs;  // the src operand holds a constant; its pending factor is 1
        GG_BRANCH();
      }
      GG_BRANCH();
    } else {
      op_value<float, K>(uop_op(h), acc, t);
      GG_BRANCH();
    }
    cur = nxt;
    ++pc;
  }
  return acc;
}

// Block prologue shared by the tier kernels: the (span, group slot) of this
// block with the same XCD-aware numbering as the forward kernel (consecutive
// items, which share a span and so the same rows of X, land on one XCD and
// its L2).  A block takes groups slot, slot + n_groups, ... of its tier's list.
struct AdjItem {
  int span, slot;
};
__device__ inline AdjItem adj_item(const AdjParams& p) {
  const int total = p.n_spans * p.n_groups;
  const int b0 = blockIdx.x;
  const int x = b0 & 7, kk = b0 >> 3, q = total >> 3, r8 = total & 7;
  const int item = x * q + (x < r8 ? x : r8) + kk;
  const int span = item / p.n_groups;
  return {span, item - span * p.n_groups};
}

// Stage one row tile of X (feature-major; rows past the last valid one hold
// a copy of a valid row and are masked by adj_seed and the sinks) and the
// centred targets (zero past the last row) into LDS.  The caller barriers.
template <int W>
__device__ inline void adj_stage(const AdjParams& p, float* xs, double* yts, int64_t r0, int nvalid,
                                 double ybar) {
  stage_x_async<W>(xs, p.X, p.ldx, p.F, p.R, r0, p.N);
  stage_y(yts, p.y, p.R, r0, nvalid, ybar);
  __builtin_amdgcn_s_waitcnt(0);  // the tile's direct loads have landed
}

// Per-row output adjoint: the residual (s0 - ybar) + s1 p - (y - ybar) in
// binary64, zero on padding rows (FULL: the batch has none).
template <int K, bool FULL = false>
__device__ inline typename VecT<float, K>::type adj_seed(const typename VecT<float, K>::type& v,
                                                         double s0m, double s1,
                                                         const double* yts, int lrow, int nvalid) {
  typename VecT<float, K>::type g;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool ok = FULL || lrow + row_off<K>(j) < nvalid;
    const double res = (s0m + s1 * double(v[j])) - yts[lrow + row_off<K>(j)];
    g[j] = ok ? float(res) : 0.0f;
  }
  return g;
}

// Write the partials of this group (individuals list[base .. base+Gn)).
// A tape tier (FALLBACK = true) leaves alone the spans of a fallen-back
// individual that the path tier got right; the path tier writes every span.
template <bool FALLBACK = true>
__device__ inline void adj_write(const AdjParams& p, int span, int base, int Gn, const double* gacc) {
  for (int j = threadIdx.x; j < Gn * p.C_max; j += blockDim.x) {
    const int jj = j / p.C_max, c = j - jj * p.C_max;
    const int i = p.list[base + jj];
    if (FALLBACK && keep_path_span(p, i, span)) continue;
    p.gpart[(size_t(i) * p.n_spans + span) * p.C_max + c] = gacc[j];
  }
}

// Per-wave column sums of the constant adjoints (binary64), added to acc[c].
// Lane l converts its own entry of column c (consecutive words across the
// lanes: conflict-free) and a fixed DPP tree sums the wave; one column at a
// time, so the cost follows the program's constant count.
template <int W>
__device__ inline void reduce_columns(const float* lacc, int nc, int lane, double* acc) {
  // the wave's column writes must land before lane l reads entry l
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int c = 0; c < nc; ++c) {  // wave-uniform
    const double s = wave_sum(double(lacc[c * kColStride + lane]));
    // every lane holds the same total and stores the same value (no divergent
    // branch between the cross-lane sums of consecutive columns)
    acc[c] += s;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SPLIT = false (tier A): the waves claim whole individuals from the tile's
// queue.  SPLIT = true (tier B, few individuals): all W waves share each
// individual, wave w taking batches w, w+W, ... with its own copy of the
// accumulators, summed in wave order at the end (bitwise repeatable).
template <int K, int D, int W, int TC, int NP, bool SPLIT>
__global__ __launch_bounds__(W * 64) void k_adj_reg(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int COPIES = SPLIT ? W : 1;
  const int R = p.R;
  const int CC = p.lane_consts;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;  // COPIES * G * C_max
  float* lacc_all = reinterpret_cast<float*>(gacc + size_t(COPIES) * p.G * p.C_max);  // W * CC * 65

  const AdjItem it = adj_item(p);
  const int cnt = __builtin_amdgcn_readfirstlane(*p.count);
  if (it.slot * p.G >= cnt) return;  // whole block: nothing of this tier here
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  float* lacc = lacc_all + size_t(wv) * CC * kColStride;
  LaneSink sink{lacc + lane};
  const int GC = p.G * p.C_max;
  double* gmine = gacc + (SPLIT ? size_t(wv) * GC : 0);
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);

  __shared__ int queue;
  for (int grp = it.slot; grp * p.G < cnt; grp += p.n_groups) {  // block-uniform
    const int base = grp * p.G;
    const int Gn = min(p.G, cnt - base);
    if (group_keeps_span(p, base, Gn, it.span)) continue;
    __syncthreads();  // previous group's partials written
    for (int j = threadIdx.x; j < COPIES * GC; j += blockDim.x) gacc[j] = 0.0;
    for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
      const int nvalid = int(min<int64_t>(R, s_end - r0));
      __syncthreads();
      if (threadIdx.x == 0) queue = 0;
      adj_stage<W>(p, xs, yts, r0, nvalid, ybar);
      __syncthreads();
      const int nbatch = (nvalid + BR - 1) / BR;
      // the next individual (claimed from the queue, or simply the next one
      // when the waves share each individual) has its program loaded into
      // registers while this one runs
      UopRegs<NP> prog, prog_next;
      int jj = SPLIT ? 0 : claim_next(&queue);
      if (jj < Gn) prog.load(p.uops + size_t(p.list[base + jj]) * p.U_stride, p.U_stride);
      while (jj < Gn) {  // wave-uniform
        const int i = __builtin_amdgcn_readfirstlane(p.list[base + jj]);
        const int jn = SPLIT ? jj + 1 : claim_next(&queue);
        if (jn < Gn) prog_next.load(p.uops + size_t(p.list[base + jn]) * p.U_stride, p.U_stride);
        const ProgMeta pm = p.meta[i];
        const int nc = __builtin_amdgcn_readfirstlane(pm.n_const);
        const double s1 = p.ab[size_t(i) * 2 + 1];
        const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;
        for (int c = 0; c < nc; ++c) lacc[c * kColStride + lane] = 0.0f;
        const int nb = keep_path_span(p, i, it.span) ? 0 : nbatch;
        for (int b = SPLIT ? wv : 0; b < nb; b += SPLIT ? W : 1) {
          const int lrow = b * BR + lane_row<K>(lane);
          RegTape<K, TC> tape;
          const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
          const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
          const int kv = nvalid - lrow;
          run_reverse<K, D>(prog, pm.n_uops, pm.n_tape, g, tape, sink, kv);
        }
        reduce_columns<W>(lacc, nc, lane, gmine + size_t(jj) * p.C_max);
        prog = prog_next;
        jj = jn;
      }
    }
    __syncthreads();
    if constexpr (SPLIT) {
      for (int j = threadIdx.x; j < GC; j += blockDim.x) {
#pragma unroll
        for (int w = 1; w < W; ++w) gacc[j] += gacc[size_t(w) * GC + j];
      }
    }
    adj_write(p, it.span, base, Gn, gacc);  // each thread reads what it summed
  }
}

// Path tier: programs with at most NC constants, differentiated in path
// forward mode (one sweep, no tape).  Waves claim whole individuals from the
// tile's queue; each lane sums its rows' constant adjoints in an LDS column.
template <int K, int D, int W, int NC, int NP>
__global__ __launch_bounds__(W * 64) void k_adj_path(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;  // G * C_max
  float* lacc_all = reinterpret_cast<float*>(gacc + size_t(p.G) * p.C_max);  // W * NC * 65

  const AdjItem it = adj_item(p);
  const int cnt = __builtin_amdgcn_readfirstlane(*p.count);
  if (it.slot * p.G >= cnt) return;  // whole block: nothing of this tier here
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  float* lacc = lacc_all + size_t(wv) * NC * kColStride;
  LaneSink sink{lacc + lane};
  const int GC = p.G * p.C_max;
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);
  const uint32_t* meta_w = reinterpret_cast<const uint32_t*>(p.meta);
  const uint32_t* ab_w = reinterpret_cast<const uint32_t*>(p.ab);

  __shared__ int queue;
  for (int grp = it.slot; grp * p.G < cnt; grp += p.n_groups) {  // block-uniform
    const int base = grp * p.G;
    const int Gn = min(p.G, cnt - base);
    // lane j holds the group's j-th individual (G <= 64)
    const int lst = lane < Gn ? p.list[base + lane] : 0;
    __syncthreads();  // previous group's partials written
    for (int j = threadIdx.x; j < GC; j += blockDim.x) gacc[j] = 0.0;
    for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
      const int nvalid = int(min<int64_t>(R, s_end - r0));
      __syncthreads();
      if (threadIdx.x == 0) queue = 0;
      adj_stage<W>(p, xs, yts, r0, nvalid, ybar);
      __syncthreads();
      const int nbatch = (nvalid + BR - 1) / BR;
      // the next claimed individual has its program, merge ranges, constant
      // count and fit coefficients loaded into registers while this one runs
      UopRegs<NP> prog, prog_next;
      uint32_t mt = 0, mt_next = 0;
      LaneWords iw, iw_next;  // n_const, then a and b as four words
      int jj = claim_next(&queue);
      if (jj < Gn) {
        const int i0 = __builtin_amdgcn_readlane(lst, jj);
        prog.load(p.uops + size_t(i0) * p.U_stride, p.U_stride);
        mt = lane < p.MT ? p.merges[size_t(i0) * p.MT + lane] : 0u;
        iw.load(meta_w + size_t(i0) * kMetaWords + kMetaNConst, 1, ab_w + size_t(i0) * 4, 4);
      }
      while (jj < Gn) {  // wave-uniform
        const int nc = int(iw.get(0));
        const double s0m = words_double(iw.get(1), iw.get(2)) - ybar;
        const double s1 = words_double(iw.get(3), iw.get(4));
        const int jn = claim_next(&queue);
        if (jn < Gn) {
          const int i1 = __builtin_amdgcn_readlane(lst, jn);
          prog_next.load(p.uops + size_t(i1) * p.U_stride, p.U_stride);
          mt_next = lane < p.MT ? p.merges[size_t(i1) * p.MT + lane] : 0u;
          iw_next.load(meta_w + size_t(i1) * kMetaWords + kMetaNConst, 1, ab_w + size_t(i1) * 4, 4);
        }
        for (int c = 0; c < nc; ++c) lacc[c * kColStride + lane] = 0.0f;
        for (int b = 0; b < nbatch; ++b) {
          const int lrow = b * BR + lane_row<K>(lane);
          RegTape<K, NC> T;
          typename VecT<float, K>::type pf;
          const auto v = run_forward_path<K, D, NC>(prog, mt, xs, R, lrow, T, pf);
          const int kv = nvalid - lrow;
          if ((b + 1) * BR <= nvalid) {  // a full batch (wave-uniform): no row tests
            const auto g = adj_seed<K, true>(v, s0m, s1, yts, lrow, nvalid) * pf;
            sink_path<0, K, NC, true>(sink, T, g, nc, kv);
          } else {
            const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid) * pf;
            sink_path<0, K, NC, false>(sink, T, g, nc, kv);
          }
        }
        reduce_columns<W>(lacc, nc, lane, gacc + size_t(jj) * p.C_max);
        prog = prog_next;
        mt = mt_next;
        iw = iw_next;
        jj = jn;
      }
    }
    __syncthreads();
    adj_write<false>(p, it.span, base, Gn, gacc);
    // a partial that is not finite may be an overflow of an intermediate
    // product that the reverse sweep does not form: that span of the
    // individual is differentiated again by the tape tiers.  The first span
    // of an individual to fall back appends it to tier B's list (tier C's for
    // a longer tape or more constants); the tape tiers' results do not depend
    // on the order of their lists.
    for (int jj = threadIdx.x; jj < Gn; jj += blockDim.x) {
      bool bad = false;
      for (int c = 0; c < p.C_max; ++c) bad = bad || !isfinite(gacc[size_t(jj) * p.C_max + c]);
      const int i = p.list[base + jj];
      p.redo_span[size_t(i) * p.n_spans + it.span] = bad ? 1 : 0;
      if (bad && atomicExch(&p.redo[i], 1) == 0) {
        const ProgMeta& pm = p.meta[i];
        const int tier = (pm.n_const <= p.lane_consts && pm.n_tape <= p.tc_b) ? 1 : 2;
        const int slot = atomicAdd(&p.fb_counts[tier], 1);
        p.fb_lists[size_t(tier) * p.M + slot] = i;
      }
    }
  }
}

// Tier C: all W waves share each individual (wave w takes batches w, w+W, ...
// of a tile and adds to its own copy of the accumulators; the copies are
// summed in wave order: bitwise repeatable).
template <int K, int D, int W>
__global__ __launch_bounds__(W * 64) void k_adj_lds(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  const AdjItem it = adj_item(p);
  const int cnt = __builtin_amdgcn_readfirstlane(*p.count);
  if (it.slot * p.G >= cnt) return;

  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;  // W copies of G * C_max
  const size_t off_tape =
      (size_t(p.F) * R * 4 + size_t(R) * 8 + size_t(W) * p.G * p.C_max * 8 + 15) & ~size_t(15);
  float* tape_all = reinterpret_cast<float*>(smem_raw + off_tape);

  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  LdsTape<K> tape{tape_all + size_t(wv) * p.tape_cap * 64 * K, lane};
  const int GC = p.G * p.C_max;
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);

  for (int grp = it.slot; grp * p.G < cnt; grp += p.n_groups) {
    const int base = grp * p.G;
    const int Gn = min(p.G, cnt - base);
    if (group_keeps_span(p, base, Gn, it.span)) continue;
    __syncthreads();
    for (int j = threadIdx.x; j < W * GC; j += blockDim.x) gacc[j] = 0.0;
    for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
      const int nvalid = int(min<int64_t>(R, s_end - r0));
      __syncthreads();
      adj_stage<W>(p, xs, yts, r0, nvalid, ybar);
      __syncthreads();
      const int nbatch = (nvalid + BR - 1) / BR;
      for (int jj = 0; jj < Gn; ++jj) {  // uniform over the block
        const int i = __builtin_amdgcn_readfirstlane(p.list[base + jj]);
        if (keep_path_span(p, i, it.span)) continue;
        const ProgMeta pm = p.meta[i];
        if (__builtin_amdgcn_readfirstlane(pm.n_tape) > p.tape_cap) continue;  // cannot happen
        const double s1 = p.ab[size_t(i) * 2 + 1];
        const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;
        const UopMem prog{p.uops + size_t(i) * p.U_stride};
        WaveSink sink{gacc + size_t(wv) * GC + size_t(jj) * p.C_max};
        for (int b = wv; b < nbatch; b += W) {
          const int lrow = b * BR + lane_row<K>(lane);
          const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
          const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
          const int kv = nvalid - lrow;
          run_reverse<K, D>(prog, pm.n_uops, pm.n_tape, g, tape, sink, kv);
        }
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < GC; j += blockDim.x) {
#pragma unroll
      for (int w = 1; w < W; ++w) gacc[j] += gacc[size_t(w) * GC + j];
    }
    adj_write(p, it.span, base, Gn, gacc);  // each thread reads what it summed
  }
}

template <int K, int D, int W, int TC, int NP>
static hipError_t reg_impl1(const TileCfg& c, int CC, bool split, const AdjParams& ap,
                            hipStream_t s) {
  const size_t sh = adjoint_reg_lds_bytes(ap.F, c.R, c.G, ap.C_max, W, CC, split ? W : 1);
  const dim3 grid(ap.n_spans * ap.n_groups), block(W * 64);
  if (split)
    hipLaunchKernelGGL((k_adj_reg<K, D, W, TC, NP, true>), grid, block, sh, s, ap);
  else
    hipLaunchKernelGGL((k_adj_reg<K, D, W, TC, NP, false>), grid, block, sh, s, ap);
  return hipGetLastError();
}

// programs of up to 63 tokens use D = 4 (one register pair); longer ones D = 8
template <int K, int D, int W, int TC>
static hipError_t reg_impl(const TileCfg& c, int CC, bool split, const AdjParams& ap,
                           hipStream_t s) {
  if constexpr (D == 4) {
    if (c.NP != 1) return hipErrorInvalidValue;
    return reg_impl1<K, 4, W, TC, 1>(c, CC, split, ap, s);
  } else {
    switch (c.NP) {
      case 1: return reg_impl1<K, 8, W, TC, 1>(c, CC, split, ap, s);
      case 2: return reg_impl1<K, 8, W, TC, 2>(c, CC, split, ap, s);
      case 4: return reg_impl1<K, 8, W, TC, 4>(c, CC, split, ap, s);
      case 8: return reg_impl1<K, 8, W, TC, 8>(c, CC, split, ap, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <int K, int D, int W, int NC, int NP>
static hipError_t path_impl1(const TileCfg& c, const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_path_lds_bytes(ap.F, c.R, c.G, ap.C_max, W, NC);
  hipLaunchKernelGGL((k_adj_path<K, D, W, NC, NP>), dim3(ap.n_spans * ap.n_groups), dim3(W * 64),
                     sh, s, ap);
  return hipGetLastError();
}

template <int K, int D, int W, int NC>
static hipError_t path_impl(const TileCfg& c, const AdjParams& ap, hipStream_t s) {
  if constexpr (D == 4) {
    if (c.NP != 1) return hipErrorInvalidValue;
    return path_impl1<K, 4, W, NC, 1>(c, ap, s);
  } else {
    switch (c.NP) {
      case 1: return path_impl1<K, 8, W, NC, 1>(c, ap, s);
      case 2: return path_impl1<K, 8, W, NC, 2>(c, ap, s);
      case 4: return path_impl1<K, 8, W, NC, 4>(c, ap, s);
      case 8: return path_impl1<K, 8, W, NC, 8>(c, ap, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <int K, int D, int W>
static hipError_t lds_impl(const TileCfg& c, const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_lds_bytes(ap.F, c.R, c.G, ap.C_max, W, K, ap.tape_cap);
  hipLaunchKernelGGL((k_adj_lds<K, D, W>), dim3(ap.n_spans * ap.n_groups), dim3(W * 64), sh, s, ap);
  return hipGetLastError();
}

static AdjParams adj_params(const AdjPlan& a, const TileCfg& c, int n_groups, const uint2* uops,
                            int U_stride, const ProgMeta* meta, int M, int C_max,
                            const DataArgs& d, const double* stats, const double* ab,
                            double* gpart, const int* list, const int* count,
                            const uint32_t* merges = nullptr, int MT = 0, int* redo = nullptr,
                            uint8_t* redo_span = nullptr, int* fb_lists = nullptr,
                            int* fb_counts = nullptr) {
  return AdjParams{uops, U_stride, meta, M, C_max, d.X, d.ldx, d.F, d.N, d.y, stats, ab, gpart,
                   list, count, c.R, c.G, n_groups, a.n_spans, a.span_rows, a.tape_cap,
                   a.lane_consts, merges, MT, redo, redo_span, fb_lists, fb_counts,
                   a.need_b ? a.tc_b : a.tc_a};
}

hipError_t launch_adjoint_partition(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                    int* lists, int* counts, int* redo, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_partition, dim3(1), dim3(kPartThreads), 0, s, meta, ab, M, a.tc_a,
                     a.need_b ? a.tc_b : a.tc_a, a.lane_consts, a.nc_p, lists, counts, redo);
  return hipGetLastError();
}

// Plain form: per individual i, counts[kTiers*i + k] = 1 if it is in tier k,
// else 0, and list0[0] = 0 (each per-individual launch lists its one individual).
__global__ __launch_bounds__(256) void k_adj_tier_flags(const ProgMeta* __restrict__ meta,
                                                        const double* __restrict__ ab, int M,
                                                        int tcA, int tcB, int CC, int ncP,
                                                        int* __restrict__ counts,
                                                        int* __restrict__ list0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) list0[0] = 0;
  if (i >= M) return;
  const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ncP);
#pragma unroll
  for (int q = 0; q < kTiers; ++q) counts[kTiers * i + q] = k == q;
}

hipError_t launch_adjoint_tier_flags(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                     int* counts, int* list0, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_tier_flags, dim3((M + 255) / 256), dim3(256), 0, s, meta, ab, M, a.tc_a,
                     a.need_b ? a.tc_b : a.tc_a, a.lane_consts, a.nc_p, counts, list0);
  return hipGetLastError();
}

hipError_t launch_adjoint_reg(const AdjPlan& a, int tier, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, int* redo,
                              uint8_t* redo_span, hipStream_t s) {
  const TileCfg& c = tier == 0 ? a.reg : a.reg_b;
  const int TC = tier == 0 ? a.tc_a : a.tc_b;
  const AdjParams ap = adj_params(a, c, c.n_groups, uops, U_stride, meta, M, C_max, d, stats, ab,
                                  gpart, list, count, nullptr, 0, redo, redo_span);
  const int CC = a.lane_consts;
  const bool split = tier == 1;  // tier B: few individuals, the waves share each one
  if (c.W != 4) return hipErrorInvalidValue;
  if (c.K == 4 && TC == 16 && c.D == 4) return reg_impl<4, 4, 4, 16>(c, CC, split, ap, s);
  if (c.K == 4 && TC == 16 && c.D == 8) return reg_impl<4, 8, 4, 16>(c, CC, split, ap, s);
  if (c.K == 2 && TC == 16 && c.D == 4) return reg_impl<2, 4, 4, 16>(c, CC, split, ap, s);
  if (c.K == 2 && TC == 16 && c.D == 8) return reg_impl<2, 8, 4, 16>(c, CC, split, ap, s);
  if (c.K == 2 && TC == 32 && c.D == 4) return reg_impl<2, 4, 4, 32>(c, CC, split, ap, s);
  if (c.K == 2 && TC == 32 && c.D == 8) return reg_impl<2, 8, 4, 32>(c, CC, split, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

hipError_t launch_adjoint_path(const AdjPlan& a, const uint2* uops, int U_stride,
                               const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                               const double* stats, const double* ab, double* gpart,
                               const uint32_t* merges, int MT, int* redo, uint8_t* redo_span,
                               int* lists, int* counts, hipStream_t s) {
  const TileCfg& c = a.path;
  const AdjParams ap = adj_params(a, c, c.n_groups, uops, U_stride, meta, M, C_max, d, stats, ab,
                                  gpart, lists + size_t(kTierPath) * M, counts + kTierPath, merges, MT,
                                  redo, redo_span, lists, counts);
  if (c.W != 4 || MT < 1 || !redo || !redo_span) return hipErrorInvalidValue;
  if (c.K == 4 && a.nc_p == 16 && c.D == 4) return path_impl<4, 4, 4, 16>(c, ap, s);
  if (c.K == 4 && a.nc_p == 16 && c.D == 8) return path_impl<4, 8, 4, 16>(c, ap, s);
  if (c.K == 8 && a.nc_p == 8 && c.D == 4) return path_impl<8, 4, 4, 8>(c, ap, s);
  if (c.K == 8 && a.nc_p == 8 && c.D == 8) return path_impl<8, 8, 4, 8>(c, ap, s);
  if (c.K == 2 && a.nc_p == 32 && c.D == 4) return path_impl<2, 4, 4, 32>(c, ap, s);
  if (c.K == 2 && a.nc_p == 32 && c.D == 8) return path_impl<2, 8, 4, 32>(c, ap, s);
  if (c.K == 4 && a.nc_p == 8 && c.D == 4) return path_impl<4, 4, 4, 8>(c, ap, s);
  if (c.K == 4 && a.nc_p == 8 && c.D == 8) return path_impl<4, 8, 4, 8>(c, ap, s);
  if (c.K == 4 && a.nc_p == 12 && c.D == 4) return path_impl<4, 4, 4, 12>(c, ap, s);
  if (c.K == 4 && a.nc_p == 12 && c.D == 8) return path_impl<4, 8, 4, 12>(c, ap, s);
  if (c.K == 2 && a.nc_p == 16 && c.D == 4) return path_impl<2, 4, 4, 16>(c, ap, s);
  if (c.K == 2 && a.nc_p == 16 && c.D == 8) return path_impl<2, 8, 4, 16>(c, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

hipError_t launch_adjoint_lds(const AdjPlan& a, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, int* redo, uint8_t* redo_span,
                              hipStream_t s) {
  const TileCfg& w = a.wide;
  const AdjParams ap = adj_params(a, w, w.n_groups, uops, U_stride, meta, M, C_max, d, stats, ab,
                                  gpart, list, count, nullptr, 0, redo, redo_span);
  if (w.D != 8) return hipErrorInvalidValue;
  if (w.K == 2 && w.W == 4) return lds_impl<2, 8, 4>(w, ap, s);
  if (w.K == 2 && w.W == 2) return lds_impl<2, 8, 2>(w, ap, s);
  if (w.K == 2 && w.W == 1) return lds_impl<2, 8, 1>(w, ap, s);
  if (w.K == 1 && w.W == 4) return lds_impl<1, 8, 4>(w, ap, s);
  if (w.K == 1 && w.W == 2) return lds_impl<1, 8, 2>(w, ap, s);
  if (w.K == 1 && w.W == 1) return lds_impl<1, 8, 1>(w, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

// One wave per (individual, constant): lane l sums spans l, l+64, ... in
// order, then a fixed xor-tree over the wave.
__global__ __launch_bounds__(256) void k_grad_finalize(const ProgMeta* __restrict__ meta, int M,
                                                       int C_max, const double* __restrict__ gpart,
                                                       int n_spans, const double* __restrict__ stats,
                                                       const double* __restrict__ ab,
                                                       double* __restrict__ grad) {
  const int64_t idx = __builtin_amdgcn_readfirstlane(
      int(int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (idx >= int64_t(M) * C_max) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const int i = int(idx / C_max), j = int(idx - int64_t(i) * C_max);
  const ProgMeta pm = meta[i];
  const double s1 = ab[size_t(i) * 2 + 1];
  const bool live = pm.status == 0 && j < pm.n_const && s1 != 0.0;
  double g = 0.0;
  if (live) {
    const double* q = gpart + size_t(i) * n_spans * C_max + j;
    for (int s = lane; s < n_spans; s += 64) g += q[size_t(s) * C_max];
  }
  g = wave_sum(g);
  if (lane == 0) grad[idx] = live ? g * (2.0 * s1 / stats[ST_N]) : 0.0;
}

hipError_t launch_grad_finalize(const ProgMeta* meta, int M, int C_max, const double* gpart,
                                int n_spans, const double* stats, const double* ab,
                                uint32_t flags, const int8_t* status, double* grad,
                                hipStream_t s) {
  (void)flags;
  (void)status;
  const int64_t n = int64_t(M) * C_max;  // one wave each, 4 per block
  hipLaunchKernelGGL(k_grad_finalize, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, meta, M,
                     C_max, gpart, n_spans, stats, ab, grad);
  return hipGetLastError();
}

}  // namespace gg

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
};

// Tier of an individual: -1 no gradient work (bad program, non-finite, b = 0
// or no constant), 0 tier A (register tape, or forward mode for at most ntF
// constants: one tangent per constant, no tape), 1 register tape B, 2 LDS
// tape.  (Slot 3 of the lists is unused.)
constexpr int kTiers = 4;
__device__ inline int adj_tier(const ProgMeta& pm, double s1, int tcA, int tcB, int CC, int ntF) {
  if (pm.status != 0 || s1 == 0.0 || pm.n_const <= 0) return -1;
  if (pm.n_const <= ntF) return 0;  // forward mode inside the tier A kernel
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
    int CC, int ntF, int* __restrict__ lists, int* __restrict__ counts) {
  __shared__ int sc[kTiers][kPartThreads];
  const int t = threadIdx.x;
  const int chunk = (M + kPartThreads - 1) / kPartThreads;
  const int lo = min(M, t * chunk), hi = min(M, lo + chunk);
  int n[kTiers] = {0, 0, 0, 0};
  for (int i = lo; i < hi; ++i) {
    const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ntF);
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
    const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ntF);
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
// s_set_gpr_idx moves instead of scratch memory.
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
  while (!(cur.x & U_END)) {
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

// Sum over the wave of this lane's first `kv` values (padding rows excluded:
// their adjoints may be NaN after multiplying a zero by an infinite partial),
// in binary64.
template <int K>
__device__ inline double wave_total(const typename VecT<float, K>::type& v, int kv) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) s += j < kv ? double(v[j]) : 0.0;
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
  template <class V, int K>
  __device__ inline void add(uint32_t c, const V& v, int kv) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) s += j < kv ? v[j] : 0.0f;
    // read-modify-write inside the LDS unit (ds_add_f32, no return value, so
    // nothing waits on it); only this lane writes this word, in program order
    (void)atomicAdd(&col[c * kColStride], s);
  }
};

// Reverse sweep.  g = adjoint of the program output per row (zero on padding
// rows); kv = valid rows of this lane.  Uops with no constant below them and
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

// ----------------------------------------------------------- forward mode
// Tier F: programs with at most NT constants.  Every value carries NT
// tangents (d value / d c_q for its program's constants q < NT), propagated
// with the same local partials as the reverse sweep: one interpreter sweep,
// no tape and no reverse pass.  A subtree without a constant has zero
// tangents (the uop's adjoint flags say which operands hold constants), so
// the tangent work is done only on constant paths.
template <int K, int NT>
struct Tangents {
  typename VecT<float, K>::type q[NT];
};

template <int K, int D, int NT, class Src>
__device__ inline typename VecT<float, K>::type run_forward_tangent(
    const Src& prog, const float* __restrict__ xt, int rstride, int lrow, Tangents<K, NT>& ad) {
  using V = typename VecT<float, K>::type;
  Slots<V, D> st;
  Slots<V, D> sd[NT];  // tangents of the pushed values
  V acc = 0.0f, t = 0.0f, pre = 0.0f;
  Tangents<K, NT> td;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    ad.q[q] = 0.0f;
    td.q[q] = 0.0f;
  }
  const float* __restrict__ xl = xt + lrow;
  uint2 cur = prog.at(0);
  prefetch_operand<float, K>(cur.x, xl, rstride, pre);
  int pc = 0;
#pragma unroll 1
  while (!(cur.x & U_END)) {
    const uint2 nxt = prog.at(pc + 1);
    const uint32_t h = cur.x;
    const float c = f32_of(cur.y);
    // operands and their tangents (a constant: unit tangent for its own index)
    if (h & (U_LDV | U_LDC)) {
      if (h & HDR_PUSH) {
        st.put(uop_push_slot(h), acc);
#pragma unroll
        for (int q = 0; q < NT; ++q) sd[q].put(uop_push_slot(h), ad.q[q]);
        GG_BRANCH();
      }
      if (h & U_LDV) {
        acc = pre;
#pragma unroll
        for (int q = 0; q < NT; ++q) ad.q[q] = 0.0f;
        GG_BRANCH();
      } else {
        acc = bcast<float, K>(c);
        const uint32_t k = uop_arg2(h);
#pragma unroll
        for (int q = 0; q < NT; ++q) ad.q[q] = uint32_t(q) == k ? 1.0f : 0.0f;
        GG_BRANCH();
      }
      GG_BRANCH();
    }
    if (h & U_TPRE) {
      t = pre;
#pragma unroll
      for (int q = 0; q < NT; ++q) td.q[q] = 0.0f;
      GG_BRANCH();
    } else if (h & U_SC) {
      t = bcast<float, K>(c);
      const uint32_t k = uop_arg2(h);
#pragma unroll
      for (int q = 0; q < NT; ++q) td.q[q] = uint32_t(q) == k ? 1.0f : 0.0f;
      GG_BRANCH();
    } else if (h & U_TX2) {
      t = lds_rows<float, K>(xl + uop_arg2(h) * rstride);
#pragma unroll
      for (int q = 0; q < NT; ++q) td.q[q] = 0.0f;
      GG_BRANCH();
    } else if (h & U_SP) {
      st.get(uop_arg2(h), t);
#pragma unroll
      for (int q = 0; q < NT; ++q) sd[q].get(uop_arg2(h), td.q[q]);
      GG_BRANCH();
    }
    prefetch_operand<float, K>(nxt.x, xl, rstride, pre);
    if (h & U_CHEAP) {  // ADD 1, SUB 2, RSUB 3, MUL 4
      if (h & (HDR_ADJ_ACC | HDR_ADJ_SRC)) {
        if (h & 4u) {
#pragma unroll
          for (int q = 0; q < NT; ++q) ad.q[q] = t * ad.q[q] + acc * td.q[q];
          acc = acc * t;
          GG_BRANCH();
        } else if (h & 2u) {
          if (h & 1u) {
            acc = t - acc;
#pragma unroll
            for (int q = 0; q < NT; ++q) ad.q[q] = td.q[q] - ad.q[q];
            GG_BRANCH();
          } else {
            acc = acc - t;
#pragma unroll
            for (int q = 0; q < NT; ++q) ad.q[q] = ad.q[q] - td.q[q];
            GG_BRANCH();
          }
          GG_BRANCH();
        } else {
          acc = acc + t;
#pragma unroll
          for (int q = 0; q < NT; ++q) ad.q[q] = ad.q[q] + td.q[q];
          GG_BRANCH();
        }
        GG_BRANCH();
      } else {  // no constant below: value only
        if (h & 4u) { acc = acc * t; GG_BRANCH(); }
        else if (h & 2u) {
          if (h & 1u) { acc = t - acc; GG_BRANCH(); }
          else { acc = acc - t; GG_BRANCH(); }
          GG_BRANCH();
        } else { acc = acc + t; GG_BRANCH(); }
        GG_BRANCH();
      }
      GG_BRANCH();
    } else if (h & (HDR_ADJ_ACC | HDR_ADJ_SRC)) {  // value, local partials, tangents
      V fa = 1.0f, fs = 0.0f;
      op_partials<K>(uop_op(h), acc, t, fa, fs);
      // a unary operator has no src operand: fs stays 0 and td is not used
      if (h & (U_TPRE | U_SC | U_TX2 | U_SP)) {
#pragma unroll
        for (int q = 0; q < NT; ++q) ad.q[q] = fa * ad.q[q] + fs * td.q[q];
        GG_BRANCH();
      } else {
#pragma unroll
        for (int q = 0; q < NT; ++q) ad.q[q] = fa * ad.q[q];
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
#pragma unroll 4
  for (int r = threadIdx.x; r < p.R; r += blockDim.x)
    yts[r] = r < nvalid ? double(p.y[r0 + r]) - ybar : 0.0;
  __builtin_amdgcn_s_waitcnt(0);  // the tile's direct loads have landed
}

// Per-row output adjoint: the residual (s0 - ybar) + s1 p - (y - ybar) in
// binary64, zero on padding rows.
template <int K>
__device__ inline typename VecT<float, K>::type adj_seed(const typename VecT<float, K>::type& v,
                                                         double s0m, double s1,
                                                         const double* yts, int lrow, int nvalid) {
  typename VecT<float, K>::type g;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool ok = lrow + j < nvalid;
    const double res = (s0m + s1 * double(v[j])) - yts[lrow + j];
    g[j] = ok ? float(res) : 0.0f;
  }
  return g;
}

// Write the partials of this group (individuals list[base .. base+Gn)).
__device__ inline void adj_write(const AdjParams& p, int span, int base, int Gn, const double* gacc) {
  for (int j = threadIdx.x; j < Gn * p.C_max; j += blockDim.x) {
    const int jj = j / p.C_max, c = j - jj * p.C_max;
    const int i = p.list[base + jj];
    p.gpart[(size_t(i) * p.n_spans + span) * p.C_max + c] = gacc[j];
  }
}

// Per-wave column sums of the constant adjoints (binary64), added to acc[c].
template <int W>
__device__ inline void reduce_columns(const float* lacc, int nc, int lane, double* acc) {
  // the wave's column writes must land before lane c reads column c
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < nc) {
    const float* colc = lacc + lane * kColStride;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
    for (int k = 0; k < 64; k += 4) {
      a0 += double(colc[k]);
      a1 += double(colc[k + 1]);
      a2 += double(colc[k + 2]);
      a3 += double(colc[k + 3]);
    }
    acc[lane] += (a0 + a1) + (a2 + a3);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SPLIT = false (tier A): the waves claim whole individuals from the tile's
// queue.  SPLIT = true (tier B, few individuals): all W waves share each
// individual, wave w taking batches w, w+W, ... with its own copy of the
// accumulators, summed in wave order at the end (bitwise repeatable).
// NT > 0: an individual with at most NT constants is differentiated in
// forward mode (one sweep, tangents instead of a tape); the others in reverse
// mode.  One launch serves both kinds, so the queue balances them.
template <int K, int D, int W, int TC, int NP, bool SPLIT, int NT>
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
        if (NT > 0 && nc <= NT) {  // forward mode (wave-uniform)
          for (int b = SPLIT ? wv : 0; b < nbatch; b += SPLIT ? W : 1) {
            const int lrow = b * BR + lane * K;
            Tangents<K, (NT > 0 ? NT : 1)> ad;
            const auto v = run_forward_tangent<K, D, (NT > 0 ? NT : 1)>(prog, xs, R, lrow, ad);
            const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
            const int kv = max(0, min(K, nvalid - lrow));
#pragma unroll
            for (int q = 0; q < (NT > 0 ? NT : 1); ++q) {
              if (q < nc) {  // wave-uniform
                const typename VecT<float, K>::type gq = g * ad.q[q];
                sink.template add<typename VecT<float, K>::type, K>(uint32_t(q), gq, kv);
              }
            }
          }
        } else {
          for (int b = SPLIT ? wv : 0; b < nbatch; b += SPLIT ? W : 1) {
            const int lrow = b * BR + lane * K;
            RegTape<K, TC> tape;
            const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
            const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
            const int kv = max(0, min(K, nvalid - lrow));
            run_reverse<K, D>(prog, pm.n_uops, pm.n_tape, g, tape, sink, kv);
          }
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
        const ProgMeta pm = p.meta[i];
        if (__builtin_amdgcn_readfirstlane(pm.n_tape) > p.tape_cap) continue;  // cannot happen
        const double s1 = p.ab[size_t(i) * 2 + 1];
        const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;
        const UopMem prog{p.uops + size_t(i) * p.U_stride};
        WaveSink sink{gacc + size_t(wv) * GC + size_t(jj) * p.C_max};
        for (int b = wv; b < nbatch; b += W) {
          const int lrow = b * BR + lane * K;
          const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
          const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
          const int kv = max(0, min(K, nvalid - lrow));
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
static hipError_t reg_impl1(const TileCfg& c, int CC, bool split, int nt, const AdjParams& ap,
                            hipStream_t s) {
  const size_t sh = adjoint_reg_lds_bytes(ap.F, c.R, c.G, ap.C_max, W, CC, split ? W : 1);
  const dim3 grid(ap.n_spans * ap.n_groups), block(W * 64);
  if (split)
    hipLaunchKernelGGL((k_adj_reg<K, D, W, TC, NP, true, 0>), grid, block, sh, s, ap);
  else if (nt == 2)
    hipLaunchKernelGGL((k_adj_reg<K, D, W, TC, NP, false, 2>), grid, block, sh, s, ap);
  else if (nt == 0)
    hipLaunchKernelGGL((k_adj_reg<K, D, W, TC, NP, false, 0>), grid, block, sh, s, ap);
  else
    return hipErrorInvalidValue;  // no kernel instantiated for this tangent count
  return hipGetLastError();
}

// programs of up to 63 tokens use D = 4 (one register pair); longer ones D = 8
template <int K, int D, int W, int TC>
static hipError_t reg_impl(const TileCfg& c, int CC, bool split, int nt, const AdjParams& ap,
                           hipStream_t s) {
  if constexpr (D == 4) {
    if (c.NP != 1) return hipErrorInvalidValue;
    return reg_impl1<K, 4, W, TC, 1>(c, CC, split, nt, ap, s);
  } else {
    switch (c.NP) {
      case 1: return reg_impl1<K, 8, W, TC, 1>(c, CC, split, nt, ap, s);
      case 2: return reg_impl1<K, 8, W, TC, 2>(c, CC, split, nt, ap, s);
      case 4: return reg_impl1<K, 8, W, TC, 4>(c, CC, split, nt, ap, s);
      case 8: return reg_impl1<K, 8, W, TC, 8>(c, CC, split, nt, ap, s);
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
                            double* gpart, const int* list, const int* count) {
  return AdjParams{uops, U_stride, meta, M, C_max, d.X, d.ldx, d.F, d.N, d.y, stats, ab, gpart,
                   list, count, c.R, c.G, n_groups, a.n_spans, a.span_rows, a.tape_cap,
                   a.lane_consts};
}

hipError_t launch_adjoint_partition(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                    int* lists, int* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_partition, dim3(1), dim3(kPartThreads), 0, s, meta, ab, M, a.tc_a,
                     a.need_b ? a.tc_b : a.tc_a, a.lane_consts, a.need_f ? a.nt_f : 0, lists, counts);
  return hipGetLastError();
}

// Plain form: per individual i, counts[kTiers*i + k] = 1 if it is in tier k,
// else 0, and list0[0] = 0 (each per-individual launch lists its one individual).
__global__ __launch_bounds__(256) void k_adj_tier_flags(const ProgMeta* __restrict__ meta,
                                                        const double* __restrict__ ab, int M,
                                                        int tcA, int tcB, int CC, int ntF,
                                                        int* __restrict__ counts,
                                                        int* __restrict__ list0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) list0[0] = 0;
  if (i >= M) return;
  const int k = adj_tier(meta[i], ab[size_t(i) * 2 + 1], tcA, tcB, CC, ntF);
#pragma unroll
  for (int q = 0; q < kTiers; ++q) counts[kTiers * i + q] = k == q;
}

hipError_t launch_adjoint_tier_flags(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                     int* counts, int* list0, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_tier_flags, dim3((M + 255) / 256), dim3(256), 0, s, meta, ab, M, a.tc_a,
                     a.need_b ? a.tc_b : a.tc_a, a.lane_consts, a.need_f ? a.nt_f : 0, counts, list0);
  return hipGetLastError();
}

hipError_t launch_adjoint_reg(const AdjPlan& a, int tier, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, hipStream_t s) {
  const TileCfg& c = tier == 0 ? a.reg : a.reg_b;
  const int TC = tier == 0 ? a.tc_a : a.tc_b;
  const AdjParams ap = adj_params(a, c, c.n_groups, uops, U_stride, meta, M, C_max, d, stats, ab,
                                  gpart, list, count);
  const int CC = a.lane_consts;
  const bool split = tier == 1;  // tier B: few individuals, the waves share each one
  const int nt = tier == 0 && a.need_f ? a.nt_f : 0;  // forward mode in tier A
  if (c.W != 4) return hipErrorInvalidValue;
  if (c.K == 4 && TC == 16 && c.D == 4) return reg_impl<4, 4, 4, 16>(c, CC, split, nt, ap, s);
  if (c.K == 4 && TC == 16 && c.D == 8) return reg_impl<4, 8, 4, 16>(c, CC, split, nt, ap, s);
  if (c.K == 2 && TC == 16 && c.D == 4) return reg_impl<2, 4, 4, 16>(c, CC, split, nt, ap, s);
  if (c.K == 2 && TC == 16 && c.D == 8) return reg_impl<2, 8, 4, 16>(c, CC, split, nt, ap, s);
  if (c.K == 2 && TC == 32 && c.D == 4) return reg_impl<2, 4, 4, 32>(c, CC, split, nt, ap, s);
  if (c.K == 2 && TC == 32 && c.D == 8) return reg_impl<2, 8, 4, 32>(c, CC, split, nt, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

hipError_t launch_adjoint_lds(const AdjPlan& a, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, hipStream_t s) {
  const TileCfg& w = a.wide;
  const AdjParams ap = adj_params(a, w, w.n_groups, uops, U_stride, meta, M, C_max, d, stats, ab,
                                  gpart, list, count);
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

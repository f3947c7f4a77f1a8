// Gradient of the fitness with respect to every constant of every individual.
//
// With linear scaling the optimal (a, b) have zero partials (envelope
// theorem), so  d LS-MSE / d c_j = (2b/N) sum_r (a + b p_r - y_r) dp_r/dc_j;
// without it  d MSE / d c_j = (2/N) sum_r (p_r - y_r) dp_r/dc_j.  Both are
// written  (2 s1/N) sum_r (s0 + s1 p_r - y_r) dp_r/dc_j  with (s0, s1) = (a, b)
// or (0, 1), taken from the forward pass (which must run first).
//
// Path forward mode.  In a tree every node has one parent, so dp/dc_j is the
// product of the local partials on the path from constant j to the root.  The
// constants of any subtree are contiguous in postfix order, so one forward
// sweep computes every dp/dc_j with no tape and no reverse pass: each value
// carries a "pending" factor per row (the product of the partials since its
// constants were last folded into T), and a register array T holds, per
// constant, the product from the constant up to its last fold.  A uop whose
// constants sit in one operand multiplies that operand's pending factor by its
// partial; at a merge (both operands hold constants) and at the push of a
// value holding constants, the pending factors are folded into T over the
// operands' constant ranges (the compile step lists these flush events per
// program, in uop order).  At the root dp/dc_j = pending * T[j].  The tree's
// values are recomputed per row tile rather than kept from the forward pass.
//
// Work classes.  T costs K * NC registers per lane, so a program is sent to
// the kernel whose NC fits its constant count: NC = 4, 8, 16 or 32 (more
// constants are cut into chunks of 32, each chunk a separate entry that
// tracks only its own constants).  Programs needing more than four stack
// slots (127 tokens or more) go to an eight-slot class.  A partition kernel
// writes one list of entries (individual * 8 + chunk) per class, in batch
// order, and one kernel per class walks its list.
//
// Binary64 fallback.  The chain-rule products are binary32; a product taken
// from the leaves up can leave the binary32 range while the true partial does
// not (or the true partial itself can exceed it).  The row tiles of an entry
// whose sums are not finite are recomputed by the same kernel in binary64
// chain-rule arithmetic (node values stay binary32, identical to the forward
// pass), in parts of 8 constants, by one of two fallback classes: 4 stack
// slots (4 rows per lane; 2 in the one-program form), or 8 slots (2 rows per
// lane).
//
// Every (entry, span) partial has exactly one writer (two in order for a
// fallen-back span), so results are bitwise repeatable for a fixed plan.
#include <hip/hip_runtime.h>

#include "interp.h"
#include "kernels.h"


namespace gg {

struct AdjParams {
  const uint2* uops;
  int U_stride;
  const ProgMeta* meta;
  const float* X;
  int64_t ldx;
  int F;
  int64_t N;
  const float* y;
  const double* stats;
  const double* ab;
  double* gpart;       // partial sums: gpart[((i - gi0) * C_max + j) * gstride + span]
  int C_max, gstride, gi0;
  const int* list;     // entries of this launch: individual * 8 + chunk
  const int* count;    // their number (device)
  int R, G, n_groups, n_spans;
  int64_t span_rows;   // rows per span (common to every class)
  const uint2* events; // flush events [M][ET]
  int ET;
  int* redo;           // [M * 8] per entry: some span fell back (cleared by the partition)
  int32_t* redo_span;  // [(e - ebase) * rstride + span]: 0 the span's binary32 sums are whole,
                       // -1 every tile of it is redone in binary64, k > 0 the tiles set in
                       // pool slot k - 1 are
  int rstride, ebase;
  int* fb_list;        // parts (entry * 4 + q: constants 8q .. 8q + 7 of the entry's chunk)
  int* fb_count;       // of the fallen-back entries, appended by the binary32 kernels: at most
  int fb_stride;       // 4 stack slots at fb_list[0 ..] (count fb_count[0]), the others at
                       // fb_list[fb_stride ..] (count fb_count[1])
  uint64_t* pool;      // bad-tile masks, tile_words words per slot
  int* pool_count;     // slots taken (cleared by the partition)
  int pool_cap;
  int tile_words;      // words per mask; 0: spans are redone whole (plain form, long spans)
};

constexpr int kChunk = 32;       // constants per entry of the chunked classes
constexpr int kMaxChunks = 8;    // GPGOMEA_MAX_CONSTS / kChunk
constexpr int kShallow = 4;      // stack slots of the shallow classes
constexpr int kPathWaves = 4;
constexpr int kAdjItems = 2048;  // work items a short class list is spread over
constexpr int kSub = 8;          // constants per item of the binary64 lists
constexpr int kSubs = kChunk / kSub;

// A list item: the class lists hold entries (individual * 8 + chunk of 32);
// the binary64 lists hold entry * 4 + part, each part 8 constants of its
// entry's chunk.  e: the entry, c_lo: the item's first constant ordinal.
struct Item {
  int e, c_lo;
};
template <bool SUB>
__device__ inline Item item_of(int v) {
  if constexpr (SUB) return {v / kSubs, ((v / kSubs) & (kMaxChunks - 1)) * kChunk + (v % kSubs) * kSub};
  return {v, (v & (kMaxChunks - 1)) * kChunk};
}

template <typename C, int K>
using CVec = typename VecT<C, K>::type;

// ---------------------------------------------------------------- partition
// Class of an individual: -1 no gradient work (bad program, non-finite, b = 0
// or no constant); 0..3 shallow with at most 4, 8, 16 or any number of
// constants (chunks of 32 for class 3); 4 deep (more than four stack slots,
// chunks of 32).
__device__ inline int adj_class(const ProgMeta& pm, double s1) {
  if (pm.status != 0 || s1 == 0.0 || pm.n_const <= 0) return -1;
  if (pm.slots > kShallow) return 4;
  if (pm.n_const <= 4) return 0;
  if (pm.n_const <= 8) return 1;
  if (pm.n_const <= 16) return 2;
  return 3;
}
__device__ inline int adj_chunks(int cls, int nc) {
  return cls < 0 ? 0 : (cls >= 3 ? (nc + kChunk - 1) / kChunk : 1);
}

// One block: thread t classifies a contiguous chunk of individuals; a
// block-wide scan of the per-thread entry counts gives each thread its
// offsets, so every list keeps batch order (deterministic).  Also clears the
// per-entry fallback flags and the fallback count.
constexpr int kPartThreads = 1024;
__global__ __launch_bounds__(kPartThreads) void k_adj_partition(
    const ProgMeta* __restrict__ meta, const double* __restrict__ ab, int M, int lstride,
    int* __restrict__ lists, int* __restrict__ counts, int* __restrict__ redo) {
  __shared__ int sc[kAdjClasses][kPartThreads];
  const int t = threadIdx.x;
  const int chunk = (M + kPartThreads - 1) / kPartThreads;
  const int lo = min(M, t * chunk), hi = min(M, lo + chunk);
  int n[kAdjClasses] = {0, 0, 0, 0, 0};
  for (int i = lo; i < hi; ++i) {
#pragma unroll
    for (int k = 0; k < kMaxChunks; ++k) redo[size_t(i) * kMaxChunks + k] = 0;
    const ProgMeta pm = meta[i];
    const int c = adj_class(pm, ab[size_t(i) * AB_WORDS + AB_S1]);
    const int ne = adj_chunks(c, pm.n_const);
#pragma unroll
    for (int q = 0; q < kAdjClasses; ++q) n[q] += c == q ? ne : 0;
  }
#pragma unroll
  for (int q = 0; q < kAdjClasses; ++q) sc[q][t] = n[q];
  __syncthreads();
  for (int o = 1; o < kPartThreads; o <<= 1) {  // inclusive Hillis-Steele scan
    int a[kAdjClasses] = {0, 0, 0, 0, 0};
    if (t >= o) {
#pragma unroll
      for (int q = 0; q < kAdjClasses; ++q) a[q] = sc[q][t - o];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kAdjClasses; ++q) sc[q][t] += a[q];
    __syncthreads();
  }
  int w[kAdjClasses];
#pragma unroll
  for (int q = 0; q < kAdjClasses; ++q) w[q] = sc[q][t] - n[q];  // exclusive offsets
  for (int i = lo; i < hi; ++i) {
    const ProgMeta pm = meta[i];
    const int c = adj_class(pm, ab[size_t(i) * AB_WORDS + AB_S1]);
    const int ne = adj_chunks(c, pm.n_const);
#pragma unroll
    for (int q = 0; q < kAdjClasses; ++q)
      if (c == q)
        for (int k = 0; k < ne; ++k) lists[size_t(q) * lstride + w[q]++] = i * kMaxChunks + k;
  }
  if (t == kPartThreads - 1) {
#pragma unroll
    for (int q = 0; q < kAdjClasses; ++q) counts[q] = sc[q][t];
    counts[kAdjClasses] = 0;  // fallback lists
    counts[kAdjClasses + 1] = 0;
    counts[kAdjClasses + 2] = 0;  // bad-tile mask pool
  }
}

// Plain form: per individual i, its entries at plist[8i ..] and their number
// in its work class, pcount[5i + class] (the other four counts 0, all five 0
// without gradient work); its two fallback counts pfb_count[2i],
// pfb_count[2i + 1] cleared; its per-entry fallback flags cleared.
__global__ __launch_bounds__(256) void k_adj_plain_lists(const ProgMeta* __restrict__ meta,
                                                         const double* __restrict__ ab, int M,
                                                         int* __restrict__ plist, int* __restrict__ pcount,
                                                         int* __restrict__ pfb_count, int* __restrict__ redo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const ProgMeta pm = meta[i];
  const int c = adj_class(pm, ab[size_t(i) * AB_WORDS + AB_S1]);
  const int ne = adj_chunks(c, pm.n_const);
  for (int k = 0; k < kMaxChunks; ++k) {
    plist[size_t(i) * kMaxChunks + k] = i * kMaxChunks + k;
    redo[size_t(i) * kMaxChunks + k] = 0;
  }
  // the work class the fused form gives the individual: its entries in that
  // class's count, none in the others
#pragma unroll
  for (int q = 0; q < kAdjClasses; ++q) pcount[size_t(i) * kAdjClasses + q] = c == q ? ne : 0;
  pfb_count[2 * i] = 0;
  pfb_count[2 * i + 1] = 0;
}

// ------------------------------------------------------------- arithmetic
// Chain-rule product f * p in which a factor of exactly 0 gives 0 whatever
// the other holds: a local partial of 0 (an operator's protected region, the
// clamp of exp) ends every derivative path through it, while a product taken
// from the leaves up may already have overflowed, or a node value may be
// infinite and absorbed above (0 * inf would be NaN where the derivative is
// 0).  Binary32: one v_mul_legacy_f32 (0 times anything is 0, either side).
template <int K, typename C>
__device__ inline CVec<C, K> zmul(const CVec<C, K>& f, const CVec<C, K>& p) {
  CVec<C, K> r;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if constexpr (sizeof(C) == 4) {
      float m;
      asm("v_mul_legacy_f32 %0, %1, %2" : "=v"(m) : "v"(f[j]), "v"(p[j]));
      r[j] = m;
    } else {
      r[j] = (f[j] == 0.0 || p[j] == 0.0) ? 0.0 : f[j] * p[j];
    }
  }
  return r;
}

template <int K, typename C>
__device__ inline CVec<C, K> widen(const CVec<float, K>& v) {
  if constexpr (sizeof(C) == 4) {
    return v;
  } else {
    CVec<C, K> r;
#pragma unroll
    for (int j = 0; j < K; ++j) r[j] = C(v[j]);
    return r;
  }
}

// Value and local partials of a non-cheap operator on K rows: fa = d result /
// d acc operand, fs = d result / d src operand (unary operators leave fs
// untouched; NOP leaves everything as it is).  The value is always the
// binary32 operator (bitwise the forward pass's); the partials are formed in
// the chain type C.  Every discrete decision (guard, clamp) is the binary32
// one the value took.
template <int K, typename C>
__device__ inline void op_partials(uint32_t op, CVec<float, K>& acc, const CVec<float, K>& t,
                                   CVec<C, K>& fa, CVec<C, K>& fs) {
  using P = Prot<float>;
  constexpr float G = P::G, CL = P::CL;
  switch (op) {
    case UOP_DIV:
    case UOP_RDIV:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const bool rev = op == UOP_RDIV;
        const float a = rev ? t[j] : acc[j], b = rev ? acc[j] : t[j];
        const float v = P::div(a, b);
        const bool g = fabsf(b) < G;
        const C r = C(1) / C(b);
        const C da = g ? C(0) : r, db = g ? C(0) : -C(v) * r;
        acc[j] = v;
        fa[j] = rev ? db : da;
        fs[j] = rev ? da : db;
      }
      GG_BRANCH();
      break;
    case UOP_POW:
    case UOP_RPOW:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const bool rev = op == UOP_RPOW;
        const float a = rev ? t[j] : acc[j], b = rev ? acc[j] : t[j];
        const float l = logf(fabsf(a));
        const float e = b * l;
        const bool live = !(fabsf(a) < G) && e >= -CL && e <= CL;
        const float v = P::pow_(a, b);
        C da, db;
        if constexpr (sizeof(C) == 4) {
          da = live ? v * b / a : 0.0f;
          db = live ? v * l : 0.0f;
        } else {
          da = live ? C(v) * C(b) / C(a) : C(0);
          db = live ? C(v) * log(fabs(C(a))) : C(0);
        }
        acc[j] = v;
        fa[j] = rev ? db : da;
        fs[j] = rev ? da : db;
      }
      GG_BRANCH();
      break;
    case UOP_SIN:
    case UOP_COS:
      // value and partial share one argument reduction
#pragma unroll
      for (int j = 0; j < K; ++j) {
        float sv, cv;
        sincosf(acc[j], &sv, &cv);  // |partial| <= 1: binary32 has the range
        fa[j] = C(op == UOP_SIN ? cv : -sv);
        acc[j] = op == UOP_SIN ? sv : cv;
      }
      GG_BRANCH();
      break;
    case UOP_SQ:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        fa[j] = C(2) * C(acc[j]);
        acc[j] = acc[j] * acc[j];
      }
      GG_BRANCH();
      break;
    case UOP_SQRT:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float a = acc[j];
        const float v = P::sqrt_(a);
        fa[j] = a == 0.0f ? C(0) : (a > 0.0f ? C(0.5) : C(-0.5)) / C(v);
        acc[j] = v;
      }
      GG_BRANCH();
      break;
    case UOP_EXP:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float a = acc[j];
        const float v = P::exp_(a);
        fa[j] = (a >= -CL && a <= CL) ? C(v) : C(0);
        acc[j] = v;
      }
      GG_BRANCH();
      break;
    case UOP_LOG:
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float a = acc[j];
        fa[j] = fabsf(a) < G ? C(0) : C(1) / C(a);
        acc[j] = P::log_(a);
      }
      GG_BRANCH();
      break;
    default:
      GG_BRANCH();
      break;
  }
}

// ------------------------------------------------------------- path state
// T: NC K-vectors, indexed only by compile-time entries (fixed registers, no
// relative addressing, no scratch).
template <int K, int NC, typename C>
struct TArr {
  CVec<C, K> v[NC];
};

// T[e] *= f for e in [lo, hi) (local entries; lo may be negative, hi may
// exceed NC).  A switch on the first entry (a binary search of uniform
// compares) enters one unrolled chain over the compile-time entry index, which
// then costs one uniform compare per entry up to the range's end.
#define GG_SCALE_CASE(E)                       \
  case E:                                      \
    if constexpr (E < NC) {                    \
      if (E >= hi) break;                      \
      T.v[E] = zmul<K, C>(f, T.v[E]);          \
    }                                          \
    [[fallthrough]];
template <int K, int NC, typename C>
__device__ inline void scale_range(TArr<K, NC, C>& T, int lo, int hi, const CVec<C, K>& f) {
  static_assert(NC <= 32, "the chain below has 32 entries");
  switch (lo < 0 ? 0 : lo) {
    GG_SCALE_CASE(0) GG_SCALE_CASE(1) GG_SCALE_CASE(2) GG_SCALE_CASE(3)
    GG_SCALE_CASE(4) GG_SCALE_CASE(5) GG_SCALE_CASE(6) GG_SCALE_CASE(7)
    GG_SCALE_CASE(8) GG_SCALE_CASE(9) GG_SCALE_CASE(10) GG_SCALE_CASE(11)
    GG_SCALE_CASE(12) GG_SCALE_CASE(13) GG_SCALE_CASE(14) GG_SCALE_CASE(15)
    GG_SCALE_CASE(16) GG_SCALE_CASE(17) GG_SCALE_CASE(18) GG_SCALE_CASE(19)
    GG_SCALE_CASE(20) GG_SCALE_CASE(21) GG_SCALE_CASE(22) GG_SCALE_CASE(23)
    GG_SCALE_CASE(24) GG_SCALE_CASE(25) GG_SCALE_CASE(26) GG_SCALE_CASE(27)
    GG_SCALE_CASE(28) GG_SCALE_CASE(29) GG_SCALE_CASE(30) GG_SCALE_CASE(31)
    default:
      break;
  }
}
#undef GG_SCALE_CASE
// T[lo] = f (no entry when lo lies outside [0, NC)).
template <int E, int K, int NC, typename C>
__device__ inline void assign_at(TArr<K, NC, C>& T, int lo, const CVec<C, K>& f) {
  if constexpr (E < NC) {
    if (E == lo) {
      T.v[E] = f;
      GG_BRANCH();
      return;
    }
    assign_at<E + 1, K, NC, C>(T, lo, f);
  }
}
// One side of a flush event (lo | n << 9 | assign << 18, absolute constant
// ordinals) applied to the chunk whose first constant is c_lo.
template <int K, int NC, typename C>
__device__ inline void path_flush(TArr<K, NC, C>& T, uint32_t side, int c_lo, const CVec<C, K>& f) {
  const int lo = int(side & 511u) - c_lo, n = int((side >> 9) & 511u);
  if (side & (1u << 18)) {
    assign_at<0, K, NC, C>(T, lo, f);
    GG_BRANCH();
  } else {
    scale_range<K, NC, C>(T, lo, lo + n, f);
    GG_BRANCH();
  }
}

// Forward sweep of one program over K rows per lane with path forward mode.
// Returns the predictions; T and p (the root's pending factor) give
// dp/dc_{c_lo + e} = p * T[e].  Same values as run_program (the binary32
// operators in the same order).
template <int K, int D, int NC, typename C, bool ROLL>
__device__ inline CVec<float, K> run_forward_path(UopWin<ROLL>& prog, EventWin& ev,
                                                  const float* __restrict__ xt, int rstride, int lrow,
                                                  int c_lo, TArr<K, NC, C>& T, CVec<C, K>& p) {
  using V = CVec<float, K>;
  using CV = CVec<C, K>;
  Slots<V, D> st;
  V acc = 0.0f, t = 0.0f, pre = 0.0f;
  p = C(1);
  // a lone constant whose value is never pushed is never flushed: its entry
  // stays 1 (with two or more constants every entry is written by a flush)
  T.v[0] = CV(C(1));
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
          const uint2 e = ev.at(mi);
          ++mi;
          path_flush<K, NC, C>(T, e.x, c_lo, p);
          GG_BRANCH();
        }
        GG_BRANCH();
      }
      if (h & U_LDV) {
        acc = pre;
        GG_BRANCH();
      } else {
        acc = bcast<float, K>(c);
        p = C(1);
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
        p = zmul<K, C>(widen<K, C>(t), p);
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
      CV fa = C(1), fs = C(1);  // d result / d acc operand, / d src operand
      if (h & U_CHEAP) {
        if (h & 4u) {
          fa = widen<K, C>(t);
          fs = widen<K, C>(acc);
          acc = acc * t;
          GG_BRANCH();
        } else if (h & 2u) {
          if (h & 1u) { fa = C(-1); acc = t - acc; GG_BRANCH(); }
          else { fs = C(-1); acc = acc - t; GG_BRANCH(); }
          GG_BRANCH();
        } else {
          acc = acc + t;
          GG_BRANCH();
        }
        GG_BRANCH();
      } else {
        op_partials<K, C>(uop_op(h), acc, t, fa, fs);
        GG_BRANCH();
      }
      if (h & HDR_ADJ_ACC) {
        if (h & HDR_ADJ_SRC) {  // merge
          const uint2 e = ev.at(mi);
          ++mi;
          path_flush<K, NC, C>(T, e.x, c_lo, zmul<K, C>(fa, p));
          path_flush<K, NC, C>(T, e.y, c_lo, fs);
          p = C(1);
          GG_BRANCH();
        } else {
          p = zmul<K, C>(fa, p);
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

// Per-row output adjoint: the residual (s0 - ybar) + s1 p - (y - ybar) in
// binary64 times the individual's power-of-two inverse scale (exact), rounded
// to the chain type, zero on padding rows (FULL: the batch has none).
template <int K, typename C, bool FULL>
__device__ inline CVec<C, K> adj_seed(const CVec<float, K>& v, double s0m, double s1, double isc,
                                      const double* yts, int lrow, int nvalid) {
  CVec<C, K> g;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool ok = FULL || lrow + row_off<K>(j) < nvalid;
    const double res = ((s0m + s1 * double(v[j])) - yts[lrow + row_off<K>(j)]) * isc;
    g[j] = ok ? C(res) : C(0);
  }
  return g;
}

// Column sums: cols[e] += sum over this lane's valid rows of g * T[e], for
// e < ncl (wave-uniform), expanded over the compile-time entry index, with g
// the residual times the root's pending factor.  Both products absorb zeros
// (a pending factor of 0 ends the path even where T[e] overflowed).  A lane's
// column accumulates the rows of one tile (binary32 in the main classes, as
// many terms as the tile has rows per lane).
template <int E, int K, int NC, typename C, bool FULL>
__device__ inline void sink_cols(C* cols, const TArr<K, NC, C>& T, const CVec<C, K>& g, int ncl, int kv) {
  if constexpr (E < NC) {
    if (E >= ncl) return;
    const CVec<C, K> d = zmul<K, C>(g, T.v[E]);
    C s = cols[E];
#pragma unroll
    for (int j = 0; j < K; ++j) s += (FULL || row_off<K>(j) < kv) ? d[j] : C(0);
    cols[E] = s;
    sink_cols<E + 1, K, NC, C, FULL>(cols, T, g, ncl, kv);
  }
}
// acc[e] += the wave's sum of column e (binary64, fixed DPP tree), e < ncl.
// Every lane holds the same total and stores the same value (no divergent
// branch between the cross-lane sums of consecutive columns).
template <int E, int NC, typename C>
__device__ inline void flush_cols(const C* cols, int ncl, double* acc) {
  if constexpr (E < NC) {
    if (E >= ncl) return;
    acc[E] += wave_sum(double(cols[E]));
    flush_cols<E + 1, NC, C>(cols, ncl, acc);
  }
}

// Block prologue: the (span, group slot) of this block with the same XCD-aware
// numbering as the forward kernel (consecutive items, which share a span and so
// the same rows of X, land on one XCD and its L2).  A block takes groups slot,
// slot + n_groups, ... of its class list.
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

// The binary64 pass redoes span s of entry e only where the binary32 pass
// flagged it.
__device__ inline bool span_flagged(const AdjParams& p, int e, int span) {
  return p.redo_span[size_t(e - p.ebase) * p.rstride + span] != 0;
}

// One class kernel.  K rows per lane, D stack slots, NC constants per entry,
// ROLL: programs longer than one 64-uop window, C: chain-rule type (float for
// the class lists, double for the fallback pass).  SPLIT = false: the waves
// claim whole entries from the tile's queue.  SPLIT = true (plain form, one
// individual per launch): all W waves share each entry, wave w taking batches
// w, w+W, ... with its own copy of the accumulators, summed in wave order at
// the end (bitwise repeatable).
// Waves per SIMD a class kernel is compiled for, trading registers for
// occupancy where it measured faster on MI355X (full size, 512-row tiles, so
// that a block needs under 40 KB of LDS and four share a CU):
// - the binary32 classes ask for four (128 VGPRs, some values and part of the
//   register array T then kept in scratch): on the large-template workload
//   the <= 4 and <= 8 classes ran 12% and 5% faster than at three waves, the
//   <= 16 class 634 -> 513 -> 486 ms from two to three to four waves, the
//   chunks of 32 (in groups of at most 32, whose blocks then fit four to a
//   CU) 199 -> 191 -> 134 ms from two to three to four; 7-12% on the
//   height-5 and mixed-height workloads.  With 1024-row tiles of 9 features
//   only three blocks fit the LDS and the request costs 2-4%;
// - the <= 8 class at four rows per lane asks for five (96 VGPRs): 2% faster
//   than at four;
// - the binary64 redo asks for three (168 VGPRs instead of 224): about 20%
//   faster than at two.
template <int K, int NC, typename C>
constexpr int adj_min_waves() {
  if constexpr (sizeof(C) != 4) return 3;
  return (K == 4 && NC == 8) ? 5 : 4;
}
template <int K, int D, int W, int NC, bool ROLL, typename C, bool SPLIT>
__global__ __launch_bounds__(W * 64, (adj_min_waves<K, NC, C>())) void k_adj_path(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr bool F64 = sizeof(C) == 8;
  constexpr bool SUB = F64;  // the binary64 pass works on parts of 8 constants
  static_assert(!SUB || NC == kSub, "binary64 items hold 8 constants");
  constexpr int COPIES = SPLIT ? W : 1;
  const int R = p.R;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;  // COPIES * G * NC

  const AdjItem it = adj_item(p);
  const int cnt = __builtin_amdgcn_readfirstlane(*p.count);
  // group size: G, or smaller for a short list so that its (span, group) work
  // items still number about kAdjItems; at least two entries per wave, so the
  // waves' shares of a group stay balanced
  const int G = max(min(2 * W, p.G), min(p.G, int(int64_t(cnt) * p.n_spans / kAdjItems)));
  if (it.slot * G >= cnt) return;  // whole block: nothing of this list here
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  const int GC = p.G * NC;
  double* gmine = gacc + (SPLIT ? size_t(wv) * GC : 0);
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);
  const uint32_t* meta_w = reinterpret_cast<const uint32_t*>(p.meta);
  const uint32_t* ab_w = reinterpret_cast<const uint32_t*>(p.ab);
  const uint2 endu = make_uint2(UOP_END_HDR, 0u), zero2 = make_uint2(0u, 0u);

  __shared__ int queue;
  // one bit per row tile of the span and group entry: binary32 pass, the
  // tiles whose sums were not finite (left out of the partials); binary64
  // pass, the tiles to redo.  rstate: the entries' redo states.
  __shared__ uint64_t tmask[64][kTileWords];
  __shared__ int rstate[64];
  const bool tiled = !SPLIT && p.tile_words > 0;
  for (int grp = it.slot; grp * G < cnt; grp += p.n_groups) {  // block-uniform
    const int base = grp * G;
    const int Gn = min(G, cnt - base);
    // lane j holds the group's j-th entry (G <= 64)
    const int lst = lane < Gn ? p.list[base + lane] : 0;
    if constexpr (F64) {  // nothing flagged on this span: skip it, staging included
      bool any = false;
      for (int jj = 0; jj < Gn; ++jj) any = any || span_flagged(p, item_of<SUB>(p.list[base + jj]).e, it.span);
      if (!any) continue;
    }
    __syncthreads();  // previous group's partials written
    for (int j = threadIdx.x; j < COPIES * GC; j += blockDim.x) gacc[j] = 0.0;
    if (tiled) {
      for (int j = threadIdx.x; j < 64 * kTileWords; j += blockDim.x) {
        const int jj = j / kTileWords, w = j - jj * kTileWords;
        uint64_t m = 0;
        if (F64 && jj < Gn && w < p.tile_words) {
          const int st = p.redo_span[size_t(item_of<SUB>(p.list[base + jj]).e - p.ebase) * p.rstride + it.span];
          m = st < 0 ? ~uint64_t(0) : st > 0 ? p.pool[size_t(st - 1) * p.tile_words + w] : 0;
        }
        tmask[jj][w] = m;
      }
    }
    for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
      const int nvalid = int(min<int64_t>(R, s_end - r0));
      const int tile = int((r0 - s_begin) / R);
      __syncthreads();
      if (F64 && tiled) {  // no entry of the group redoes this tile: skip it (block-uniform)
        bool need = false;
        for (int jj = 0; jj < Gn; ++jj) need = need || ((tmask[jj][tile >> 6] >> (tile & 63)) & 1);
        if (!need) continue;
      }
      if (threadIdx.x == 0) queue = 0;
      stage_x_async<W>(xs, p.X, p.ldx, p.F, R, r0, p.N);
      stage_y(yts, p.y, R, r0, nvalid, ybar);
      __builtin_amdgcn_s_waitcnt(0);  // the tile's direct loads have landed
      __syncthreads();
      const int nbatch = (nvalid + BR - 1) / BR;
      // the next entry has its first program window, first event window,
      // constant count and fit coefficients loaded while this one runs
      uint32_t u0lo = 0, u0hi = 0, u1lo = 0, u1hi = 0, e0lo = 0, e0hi = 0, e1lo = 0, e1hi = 0;
      LaneWords iw, iw_next;  // n_const, then s0, s1 and the inverse scale as six words
      int jj = SPLIT ? 0 : claim_next(&queue);
      if (jj < Gn) {
        const int i0 = item_of<SUB>(__builtin_amdgcn_readlane(lst, jj)).e >> 3;
        load_window(p.uops + size_t(i0) * p.U_stride, 0, p.U_stride, endu, u0lo, u0hi);
        load_window(p.events + size_t(i0) * p.ET, 0, p.ET, zero2, e0lo, e0hi);
        iw.load(meta_w + size_t(i0) * kMetaWords + kMetaNConst, 1, ab_w + size_t(i0) * 2 * AB_WORDS, 6);
      }
      while (jj < Gn) {  // wave-uniform
        const Item itm = item_of<SUB>(__builtin_amdgcn_readlane(lst, jj));
        const int e = itm.e;
        const int i = e >> 3;
        const int c_lo = itm.c_lo;
        const int nc = int(iw.get(0));
        const double s0m = words_double(iw.get(1), iw.get(2)) - ybar;
        const double s1 = words_double(iw.get(3), iw.get(4));
        const double isc = words_double(iw.get(5), iw.get(6));
        const int jn = SPLIT ? jj + 1 : claim_next(&queue);
        if (jn < Gn) {
          const int i1 = item_of<SUB>(__builtin_amdgcn_readlane(lst, jn)).e >> 3;
          load_window(p.uops + size_t(i1) * p.U_stride, 0, p.U_stride, endu, u1lo, u1hi);
          load_window(p.events + size_t(i1) * p.ET, 0, p.ET, zero2, e1lo, e1hi);
          iw_next.load(meta_w + size_t(i1) * kMetaWords + kMetaNConst, 1, ab_w + size_t(i1) * 2 * AB_WORDS, 6);
        }
        const int ncl = min(NC, nc - c_lo);  // constants this entry tracks
        bool run = true;
        if constexpr (F64)
          run = tiled ? ((tmask[jj][tile >> 6] >> (tile & 63)) & 1) != 0 : span_flagged(p, e, it.span);
        if (run) {
          C cols[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) cols[k] = C(0);
          const uint2* prow = p.uops + size_t(i) * p.U_stride;
          const uint2* erow = p.events + size_t(i) * p.ET;
          for (int b = SPLIT ? wv : 0; b < nbatch; b += SPLIT ? W : 1) {
            const int lrow = b * BR + lane_row<K>(lane);
            UopWin<ROLL> prog;
            prog.begin(prow, p.U_stride, u0lo, u0hi);
            EventWin ev;
            ev.begin(erow, p.ET, e0lo, e0hi);
            TArr<K, NC, C> T;
            CVec<C, K> pf;
            const auto v = run_forward_path<K, D, NC, C, ROLL>(prog, ev, xs, R, lrow, c_lo, T, pf);
            const int kv = nvalid - lrow;
            if ((b + 1) * BR <= nvalid) {  // a full batch (wave-uniform): no row tests
              const CVec<C, K> g = zmul<K, C>(adj_seed<K, C, true>(v, s0m, s1, isc, yts, lrow, nvalid), pf);
              sink_cols<0, K, NC, C, true>(cols, T, g, ncl, kv);
            } else {
              const CVec<C, K> g = zmul<K, C>(adj_seed<K, C, false>(v, s0m, s1, isc, yts, lrow, nvalid), pf);
              sink_cols<0, K, NC, C, false>(cols, T, g, ncl, kv);
            }
          }
          if (!F64 && tiled) {
            // a column sum that is not finite: this tile of the entry is left
            // out and redone in binary64 (wave-uniform decision)
            bool lbad = false;
#pragma unroll
            for (int k = 0; k < NC; ++k) lbad = lbad || (k < ncl && !isfinite(cols[k]));
            if (__ballot(lbad) != 0) {
              if (lane == 0) tmask[jj][tile >> 6] |= uint64_t(1) << (tile & 63);
            } else {
              flush_cols<0, NC, C>(cols, ncl, gmine + size_t(jj) * NC);
            }
          } else {
            flush_cols<0, NC, C>(cols, ncl, gmine + size_t(jj) * NC);
          }
        }
        u0lo = u1lo;
        u0hi = u1hi;
        e0lo = e1lo;
        e0hi = e1hi;
        iw = iw_next;
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
    if constexpr (!F64) {
      // the entries' redo states on this span: tiled, the tiles left out (their
      // mask goes to a pool slot; a full pool redoes the whole span); untiled,
      // sums that are not finite redo the whole span.  The first span of an
      // entry to fall back appends it to the fallback list (whose order does
      // not change any result)
      for (int jj = threadIdx.x; jj < Gn; jj += blockDim.x) {
        const int e = p.list[base + jj];
        const int ncl = min(NC, p.meta[e >> 3].n_const - (e & (kMaxChunks - 1)) * kChunk);
        int st = 0;
        if (tiled) {
          bool any = false;
          for (int w = 0; w < p.tile_words; ++w) any = any || tmask[jj][w] != 0;
          if (any) {
            const int slot = atomicAdd(p.pool_count, 1);
            if (slot < p.pool_cap) {
              for (int w = 0; w < p.tile_words; ++w) p.pool[size_t(slot) * p.tile_words + w] = tmask[jj][w];
              st = slot + 1;
            } else {
              st = -1;
            }
          }
        } else {
          bool bad = false;
          for (int k = 0; k < ncl; ++k) bad = bad || !isfinite(gacc[size_t(jj) * NC + k]);
          st = bad ? -1 : 0;
        }
        rstate[jj] = st;
        p.redo_span[size_t(e - p.ebase) * p.rstride + it.span] = st;
        if (st != 0 && atomicExch(&p.redo[e], 1) == 0) {
          // its parts of 8 constants go to the binary64 list of its depth
          const int deep = p.meta[e >> 3].slots > kShallow ? 1 : 0;
          const int parts = (ncl + kSub - 1) / kSub;
          const int slot = atomicAdd(p.fb_count + deep, parts);
          for (int q = 0; q < parts; ++q) p.fb_list[size_t(deep) * p.fb_stride + slot + q] = e * kSubs + q;
        }
      }
      __syncthreads();
    }
    // each thread writes what it summed.  Binary32: the sums of the tiles kept
    // (0 where the whole span is redone); binary64: adds the redone tiles
    for (int j = threadIdx.x; j < GC; j += blockDim.x) {
      const int jj = j / NC, k = j - jj * NC;
      if (jj >= Gn) continue;
      const Item itm = item_of<SUB>(p.list[base + jj]);
      const int e = itm.e;
      const int i = e >> 3, cj = itm.c_lo + k;
      if (cj >= p.meta[i].n_const) continue;
      double* dst = p.gpart + (size_t(i - p.gi0) * p.C_max + cj) * p.gstride + it.span;
      if constexpr (F64) {
        if (span_flagged(p, e, it.span)) *dst += gacc[j];
      } else {
        *dst = rstate[jj] < 0 ? 0.0 : gacc[j];
      }
    }
  }
}

// -------------------------------------------------------------- launchers
size_t adjoint_path_lds_bytes(int F, int R, int G, int NC, int W, bool split) {
  return size_t(F) * R * 4 + size_t(R) * 8 + size_t(split ? W : 1) * G * NC * 8;
}

template <int K, int D, int NC, bool ROLL, typename C, bool SPLIT>
static hipError_t path_launch(const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_path_lds_bytes(ap.F, ap.R, ap.G, NC, kPathWaves, SPLIT);
  hipLaunchKernelGGL((k_adj_path<K, D, kPathWaves, NC, ROLL, C, SPLIT>), dim3(ap.n_spans * ap.n_groups),
                     dim3(kPathWaves * 64), sh, s, ap);
  return hipGetLastError();
}

template <bool ROLL, bool SPLIT>
static hipError_t class_launch(int cls, int K, const AdjParams& ap, hipStream_t s) {
  switch (cls) {
    case 0:
      return K == 4 ? path_launch<4, kShallow, 4, ROLL, float, SPLIT>(ap, s)
                    : path_launch<2, kShallow, 4, ROLL, float, SPLIT>(ap, s);
    case 1:
      return K == 4 ? path_launch<4, kShallow, 8, ROLL, float, SPLIT>(ap, s)
                    : path_launch<2, kShallow, 8, ROLL, float, SPLIT>(ap, s);
    case 2:
      return K == 4 ? path_launch<4, kShallow, 16, ROLL, float, SPLIT>(ap, s)
                    : path_launch<2, kShallow, 16, ROLL, float, SPLIT>(ap, s);
    case 3: return path_launch<2, kShallow, kChunk, ROLL, float, SPLIT>(ap, s);
    case 4: return path_launch<2, 8, kChunk, ROLL, float, SPLIT>(ap, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_partition(const ProgMeta* meta, const double* ab, int M, int lstride,
                                    int* lists, int* counts, int* redo, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_partition, dim3(1), dim3(kPartThreads), 0, s, meta, ab, M, lstride, lists,
                     counts, redo);
  return hipGetLastError();
}

hipError_t launch_adjoint_plain_lists(const ProgMeta* meta, const double* ab, int M, int* plist,
                                      int* pcount, int* pfb_count, int* redo, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_plain_lists, dim3((M + 255) / 256), dim3(256), 0, s, meta, ab, M, plist,
                     pcount, pfb_count, redo);
  return hipGetLastError();
}

hipError_t launch_adjoint_class(const AdjLaunch& L, hipStream_t s) {
  const AdjParams ap{L.uops, L.U_stride, L.meta, L.d.X, L.d.ldx, L.d.F, L.d.N, L.d.y, L.stats, L.ab,
                     L.gpart, L.C_max, L.gstride, L.gi0, L.list, L.count, L.R, L.G, L.n_groups,
                     L.n_spans, L.span_rows, L.events, L.ET, L.redo, L.redo_span, L.rstride,
                     L.ebase, L.fb_list, L.fb_count, L.fb_stride, L.pool, L.pool_count, L.pool_cap,
                     L.split ? 0 : L.tile_words};
  if (L.G < 1 || L.G > 64) return hipErrorInvalidValue;  // the group list is lane-held
  const bool roll = L.U_stride > 64;
  if (L.cls == kAdjFallback) {  // binary64 chain rule: parts of 8 constants, 4 slots
    if (L.split) return roll ? path_launch<2, kShallow, kSub, true, double, true>(ap, s)
                             : path_launch<2, kShallow, kSub, false, double, true>(ap, s);
    return roll ? path_launch<4, kShallow, kSub, true, double, false>(ap, s)
                : path_launch<4, kShallow, kSub, false, double, false>(ap, s);
  }
  if (L.cls == kAdjFallbackWide) {  // binary64 chain rule: parts of 8 constants, 8 slots
    if (L.split) return roll ? path_launch<2, 8, kSub, true, double, true>(ap, s)
                             : path_launch<2, 8, kSub, false, double, true>(ap, s);
    return roll ? path_launch<2, 8, kSub, true, double, false>(ap, s)
                : path_launch<2, 8, kSub, false, double, false>(ap, s);
  }
  // a class kernel; in the plain form (split) the block's waves share each entry
  if (L.split)
    return roll ? class_launch<true, true>(L.cls, L.K, ap, s) : class_launch<false, true>(L.cls, L.K, ap, s);
  return roll ? class_launch<true, false>(L.cls, L.K, ap, s) : class_launch<false, false>(L.cls, L.K, ap, s);
}

// ------------------------------------------------------------ grad finalize
// One wave per (individual, constant): lane l sums spans l, l+64, ... in
// order, then a fixed DPP tree over the wave.  grad = 2 s1 scale / N * sum
// (zero past the individual's constants and without gradient work).
__global__ __launch_bounds__(256) void k_grad_finalize(const ProgMeta* __restrict__ meta, int i0, int M,
                                                       int C_max, const double* __restrict__ gpart,
                                                       int gstride, int n_spans,
                                                       const double* __restrict__ stats,
                                                       const double* __restrict__ ab,
                                                       double* __restrict__ grad) {
  const int64_t idx = __builtin_amdgcn_readfirstlane(
      int(int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (idx >= int64_t(M) * C_max) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const int ii = int(idx / C_max), j = int(idx - int64_t(ii) * C_max);
  const int i = i0 + ii;
  const ProgMeta pm = meta[i];
  const double s1 = ab[size_t(i) * AB_WORDS + AB_S1];
  const double sc = ab[size_t(i) * AB_WORDS + AB_SCALE];
  const bool live = pm.status == 0 && j < pm.n_const && s1 != 0.0;
  double g = 0.0;
  if (live) {
    const double* q = gpart + size_t(idx) * gstride;
    for (int sp = lane; sp < n_spans; sp += 64) g += q[sp];
  }
  g = wave_sum(g);
  if (lane == 0) grad[size_t(i) * C_max + j] = live ? g * (2.0 * s1 * sc / stats[ST_N]) : 0.0;
}

hipError_t launch_grad_finalize(const ProgMeta* meta, int i0, int M, int C_max, const double* gpart,
                                int gstride, int n_spans, const double* stats, const double* ab,
                                double* grad, hipStream_t s) {
  const int64_t n = int64_t(M) * C_max;  // one wave each, 4 per block
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_finalize, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, meta, i0, M, C_max,
                     gpart, gstride, n_spans, stats, ab, grad);
  return hipGetLastError();
}

}  // namespace gg

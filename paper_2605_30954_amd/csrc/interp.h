// Register-stack interpreter for one uop program over K rows per lane.
//
// The paper evaluates an individual's postfix program with a stack, one
// forward pass per data point, all threads of a block running the same
// program so control flow never diverges (Section 3.2, "Evaluation on the
// GPU").  Here a whole wave (64 lanes) runs one program: the uop stream is
// wave-uniform, read with scalar loads one uop ahead, and every lane evaluates
// K rows at once so each decoded uop is amortised over K*64 rows.
//
// Code-shape rules this file follows (checked in the gfx950 ISA):
//  * the accumulator and the D stack slots are separate vector-typed values
//    (never an indexed array), so they live in VGPRs and are never spilled to
//    scratch by dynamic indexing;
//  * dispatch is a chain of independent uniform `if` blocks, each ending in an
//    empty volatile asm statement: the block stays a branch (no if-conversion
//    into per-element selects) and updates its registers in place (no
//    structurizer copies at the joins).
//
// Variables are read from the block's row tile in LDS (feature-major,
// `rstride` floats per feature); lane l of a batch owns rows
// [row0 + l*K, row0 + l*K + K).
#pragma once
#include <hip/hip_runtime.h>

#include "devmath.h"
#include "uop.h"

#define GG_BRANCH() asm volatile("")

namespace gg {

template <typename T, int K>
struct VecT {
  typedef T type __attribute__((ext_vector_type(K)));
};

// Rows of a batch.  A batch covers 64*K consecutive rows of the tile.  For
// K >= 4, lane l holds rows 4l + 256q + {0, 1, 2, 3} for q < K/4: each float4
// LDS read takes a 16-byte run per lane with consecutive lanes on consecutive
// runs (no bank conflict), where K consecutive rows per lane would put lanes
// l and l + 8 on the same banks.  For K < 4, lane l holds rows lK + j.
// Element j of a lane is row lane_row(l) + row_off(j) of the batch.
template <int K>
__host__ __device__ constexpr int lane_row(int lane) {
  return K >= 4 ? 4 * lane : K * lane;
}
template <int K>
__host__ __device__ constexpr int row_off(int j) {
  return K >= 4 ? (j >> 2) * 256 + (j & 3) : j;
}

template <typename T, int K>
__device__ inline typename VecT<T, K>::type lds_rows(const float* __restrict__ p) {
  typename VecT<T, K>::type v;
  static_assert(K % 4 == 0 || K < 4, "K must be 1, 2 or a multiple of 4");
  if constexpr (K >= 4) {
#pragma unroll
    for (int j = 0; j < K; j += 4) {
      const float4 q = *reinterpret_cast<const float4*>(p + row_off<K>(j));
      v[j] = T(q.x);
      v[j + 1] = T(q.y);
      v[j + 2] = T(q.z);
      v[j + 3] = T(q.w);
    }
  } else if constexpr (K == 2) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    v[0] = T(q.x);
    v[1] = T(q.y);
  } else {
    v[0] = T(p[0]);
  }
  return v;
}

// A wave-uniform binary32 value (in an SGPR) copied to every element of a
// K-vector with one VALU move per element (the compiler would otherwise pair
// the elements into 64-bit moves fed by a chain of scalar copies).
template <typename T, int K>
__device__ inline typename VecT<T, K>::type bcast(float c) {
  typename VecT<T, K>::type v;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      float x;
      asm("v_mov_b32 %0, %1" : "=v"(x) : "s"(c));
      v[j] = x;
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = T(c);
  }
  return v;
}

// D register slots, addressed by a wave-uniform slot number.
template <typename V, int D>
struct Slots {
  static_assert(D >= 1 && D <= 8, "1..8 stack slots");
  V s0, s1, s2, s3, s4, s5, s6, s7;

  __device__ inline void put(uint32_t k, const V& a) {
    if (k == 0) { s0 = a; GG_BRANCH(); }
    if constexpr (D > 1) if (k == 1) { s1 = a; GG_BRANCH(); }
    if constexpr (D > 2) if (k == 2) { s2 = a; GG_BRANCH(); }
    if constexpr (D > 3) if (k == 3) { s3 = a; GG_BRANCH(); }
    if constexpr (D > 4) if (k == 4) { s4 = a; GG_BRANCH(); }
    if constexpr (D > 5) if (k == 5) { s5 = a; GG_BRANCH(); }
    if constexpr (D > 6) if (k == 6) { s6 = a; GG_BRANCH(); }
    if constexpr (D > 7) if (k == 7) { s7 = a; GG_BRANCH(); }
  }
  __device__ inline void get(uint32_t k, V& a) const {
    if (k == 0) { a = s0; GG_BRANCH(); }
    if constexpr (D > 1) if (k == 1) { a = s1; GG_BRANCH(); }
    if constexpr (D > 2) if (k == 2) { a = s2; GG_BRANCH(); }
    if constexpr (D > 3) if (k == 3) { a = s3; GG_BRANCH(); }
    if constexpr (D > 4) if (k == 4) { a = s4; GG_BRANCH(); }
    if constexpr (D > 5) if (k == 5) { a = s5; GG_BRANCH(); }
    if constexpr (D > 6) if (k == 6) { a = s6; GG_BRANCH(); }
    if constexpr (D > 7) if (k == 7) { a = s7; GG_BRANCH(); }
  }
};

__device__ inline float f32_of(uint32_t bits) { return __uint_as_float(bits); }

// Read-only data that every lane of a wave reads at the same address (uop
// streams, per-individual metadata): accessed through the constant address
// space so the compiler emits scalar loads into SGPRs.
template <typename T>
using const_as_ptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ inline T load_uniform(const T* p, int i) {
  return ((const_as_ptr<T>)p)[i];
}

// Wave-uniform scalar load of a uop.
__device__ inline uint2 load_uop(const uint2* __restrict__ prog, int pc) {
  const unsigned long long v = load_uniform(reinterpret_cast<const unsigned long long*>(prog), pc);
  return make_uint2(uint32_t(v), uint32_t(v >> 32));
}

// Where the interpreter reads its uops from.  Both give the same uop for a
// wave-uniform pc.
//
// UopMem: scalar loads from the uop array (one uop ahead).  Simple, but a
// scalar load's wait (lgkmcnt) is shared with the LDS row reads and scalar
// loads return out of order, so every wait for a row also waits for the next
// uop; used by the kernels where that does not matter.
struct UopMem {
  const uint2* __restrict__ p;
  __device__ inline uint2 at(int pc) const { return load_uop(p, pc); }
};

// Lane-held window of a stream of 64-bit words (uops, flush events): lane l
// holds word base + l.  One coalesced vector load (vmcnt, not lgkmcnt).  Words
// at or past `n` read as `fill`.
__device__ inline void load_window(const uint2* __restrict__ p, int base, int n, uint2 fill,
                                   uint32_t& lo, uint32_t& hi) {
  const int idx = base + int(threadIdx.x & 63);
  uint2 u = fill;
  if (idx < n) u = p[idx];
  lo = u.x;
  hi = u.y;
}
__device__ inline uint2 read_window(uint32_t lo, uint32_t hi, int l) {
  return make_uint2(uint32_t(__builtin_amdgcn_readlane(int(lo), l)),
                    uint32_t(__builtin_amdgcn_readlane(int(hi), l)));
}

// UopWin<ROLL>: the program held in VGPRs 64 uops at a time (lane l of the
// current window holds uop 64w + l); at() copies a uop into SGPRs with
// v_readlane, so the interpreter loop issues no memory access for its
// instruction stream.  The first window is loaded one individual ahead by the
// caller (load_window) and handed to begin().  ROLL (programs of more than 64
// uops): entering a window loads the next one, which becomes current when the
// program counter crosses into it 64 uops later, so its load latency is
// hidden by the uops in between.  at() must be called with pc = 0, 1, 2, ...
// in order (a forward sweep).
template <bool ROLL>
struct UopWin {
  uint32_t lo = 0, hi = 0, nlo = 0, nhi = 0;
  const uint2* __restrict__ p = nullptr;
  int n = 0;  // words of the program's uop row that may be read
  __device__ inline void begin(const uint2* __restrict__ prog, int n_words, uint32_t lo0, uint32_t hi0) {
    lo = lo0;
    hi = hi0;
    if constexpr (ROLL) {
      p = prog;
      n = n_words;
      if (n_words > 64) load_window(prog, 64, n_words, make_uint2(UOP_END_HDR, 0u), nlo, nhi);
    }
  }
  __device__ inline uint2 at(int pc) {
    const int l = pc & 63;
    if constexpr (ROLL) {
      if (l == 0 && pc != 0) {  // wave-uniform: crossing into the next window
        lo = nlo;
        hi = nhi;
        if (pc + 64 < n) load_window(p, pc + 64, n, make_uint2(UOP_END_HDR, 0u), nlo, nhi);
        GG_BRANCH();
      }
    }
    return read_window(lo, hi, l);
  }
};

// Flush events of path forward mode (one uint2 each), consumed in order: the
// first 64 are lane-held (loaded one individual ahead, like a program's first
// window); later windows are loaded when reached (few programs have more than
// 64 events).
struct EventWin {
  uint32_t lo = 0, hi = 0;
  const uint2* __restrict__ p = nullptr;
  int n = 0;
  __device__ inline void begin(const uint2* __restrict__ ev, int n_ev, uint32_t lo0, uint32_t hi0) {
    lo = lo0;
    hi = hi0;
    p = ev;
    n = n_ev;
  }
  __device__ inline uint2 at(int m) {
    const int l = m & 63;
    if (l == 0 && m != 0) {  // wave-uniform
      load_window(p, m, n, make_uint2(0u, 0u), lo, hi);
      GG_BRANCH();
    }
    return read_window(lo, hi, l);
  }
};

// Sum of a binary64 value over the 64 lanes of a wave, returned to every lane
// (wave-uniform).  Data-parallel-primitive moves only, no LDS traffic: an
// inclusive scan inside each row of 16 lanes (row_shr 1, 2, 4, 8), then the
// row totals are carried across rows (row_bcast 15 into rows 1 and 3,
// row_bcast 31 into rows 2 and 3), so lane 63 holds the total.  A lane with no
// source reads 0.  Fixed pattern: bitwise repeatable.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double((long long)uint32_t(lo) | ((long long)hi << 32));
}
__device__ inline double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b), 63);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
  return __longlong_as_double((long long)uint32_t(lo) | ((long long)hi << 32));
}

// Row-tile staging with direct global-to-LDS loads (global_load_lds_dword):
// the W waves of the block issue the tile's 64-row chunks of every feature
// back to back, with no register round trip and no wait per load; the caller
// waits once (s_waitcnt 0) and barriers before reading.  Rows past the last
// valid one read a clamped valid row: padding rows are masked by every
// consumer.  R is a multiple of 64.
template <int W>
__device__ inline void stage_x_async(float* xs, const float* __restrict__ X, int64_t ldx, int F,
                                     int R, int64_t r0, int64_t N) {
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int per = R >> 6;  // chunks per feature
  const int nq = F * per;
  for (int q = wv; q < nq; q += W) {  // wave-uniform
    const int f = q / per, r = (q - f * per) << 6;
    const int64_t row = min<int64_t>(r0 + r + lane, N - 1);
    __builtin_amdgcn_global_load_lds(X + size_t(f) * ldx + row, xs + size_t(f) * R + r, 4, 0, 0);
  }
}

// Centred targets of a row tile in binary64 (zero past the last valid row;
// nvalid >= 1).  Every load reads a clamped valid row unconditionally, so a
// thread's loads are in flight together instead of one wait per branch.
__device__ inline void stage_y(double* yts, const float* __restrict__ y, int R, int64_t r0,
                               int nvalid, double ybar) {
  constexpr int U = 4;
  const int bd = blockDim.x;
  for (int r = threadIdx.x; r < R; r += U * bd) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = y[r0 + min(r + u * bd, nvalid - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ru = r + u * bd;
      if (ru < R) yts[ru] = ru < nvalid ? double(v[u]) - ybar : 0.0;
    }
  }
}

// Per-individual words (metadata, fit coefficients) fetched one individual
// ahead, like a program's first window: lane w holds word w, a coalesced vector load.  Reading
// a word back (v_readlane) waits only for loads issued one individual ago,
// where a scalar or vector load of the current individual's words, issued
// after the next program's prefetch, would wait for that prefetch as well.
struct LaneWords {
  uint32_t v = 0;
  // words [0, n0) from a, then [n0, n0 + n1) from b
  __device__ inline void load(const uint32_t* __restrict__ a, int n0,
                              const uint32_t* __restrict__ b = nullptr, int n1 = 0) {
    const int lane = threadIdx.x & 63;
    v = 0u;
    if (lane < n0) v = a[lane];
    else if (lane < n0 + n1) v = b[lane - n0];
  }
  __device__ inline uint32_t get(int w) const { return __builtin_amdgcn_readlane(v, w); }
};
// binary64 from its low and high words
__device__ inline double words_double(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(uint64_t(hi) << 32 | lo));
}

// Dynamic work queue of one block and one row tile: every wave claims the
// next index from an LDS counter (one atomic by lane 0; the value is made
// wave-uniform with readfirstlane, so loops on it exit with a scalar branch),
// which keeps the waves of a block busy until the tile's barrier however
// unequal the programs are.  The counter must be reset before the tile.
__device__ inline int claim_next(int* ctr) {
  int t = 0;
  if ((threadIdx.x & 63) == 0) t = atomicAdd(ctr, 1);
  return __builtin_amdgcn_readfirstlane(t);
}

// Per-element application of the protected operators to K-vectors.
template <typename T, int K>
struct VOps {
  using V = typename VecT<T, K>::type;
  using P = Prot<T>;
#define GG_MAP1(name, expr)                              \
  __device__ static inline V name(V a) {                 \
    V r;                                                 \
    _Pragma("unroll") for (int j = 0; j < K; ++j) {      \
      const T x = a[j];                                  \
      r[j] = (expr);                                     \
    }                                                    \
    return r;                                            \
  }
#define GG_MAP2(name, expr)                              \
  __device__ static inline V name(V a, V b) {            \
    V r;                                                 \
    _Pragma("unroll") for (int j = 0; j < K; ++j) {      \
      const T x = a[j], z = b[j];                        \
      r[j] = (expr);                                     \
    }                                                    \
    return r;                                            \
  }
  GG_MAP1(sin, P::sin_(x))
  GG_MAP1(cos, P::cos_(x))
  GG_MAP1(sqrt, P::sqrt_(x))
  GG_MAP1(exp, P::exp_(x))
  GG_MAP1(log, P::log_(x))
  GG_MAP2(div, P::div(x, z))
  GG_MAP2(pow, P::pow_(x, z))
#undef GG_MAP1
#undef GG_MAP2
};

// Operand prefetch: the first variable operand of uop header h (field var1)
// is read from the row tile into `pre`, so that the LDS latency overlaps the
// work of the uop before it.
template <typename T, int K>
__device__ inline void prefetch_operand(uint32_t h, const float* __restrict__ xl, int rstride,
                                        typename VecT<T, K>::type& pre) {
  if (h & U_V1) {
    pre = lds_rows<T, K>(xl + uop_var1(h) * rstride);
    GG_BRANCH();
  }
}

// Operand stage shared by the interpreters: push, load prefix and the src
// operand of uop h.  Every header bit is tested once (a condition the compiler
// could share between blocks would be kept as a lane mask and cost extra
// instructions per test).  On return acc holds the acc operand and t the src
// operand; `pre` holds the uop's first variable operand (read one uop ahead).
template <typename T, int K, int D>
__device__ inline void operand_stage(uint32_t h, float c, const float* __restrict__ xl,
                                     int rstride, typename VecT<T, K>::type& acc,
                                     typename VecT<T, K>::type& t,
                                     const typename VecT<T, K>::type& pre,
                                     Slots<typename VecT<T, K>::type, D>& st) {
  if (h & (U_LDV | U_LDC)) {  // first leaf of a subtree (after pushing the pending value)
    if (h & HDR_PUSH) {
      st.put(uop_push_slot(h), acc);
      GG_BRANCH();
    }
    if (h & U_LDV) {
      acc = pre;
      GG_BRANCH();
    } else {
      acc = bcast<T, K>(c);
      GG_BRANCH();
    }
    GG_BRANCH();
  }
  if (h & U_TPRE) {
    t = pre;
    GG_BRANCH();
  } else if (h & U_SC) {
    t = bcast<T, K>(c);
    GG_BRANCH();
  } else if (h & U_TX2) {
    t = lds_rows<T, K>(xl + uop_arg2(h) * rstride);
    GG_BRANCH();
  } else if (h & U_SP) {
    st.get(uop_arg2(h), t);
    GG_BRANCH();
  }
}

// Value of a non-cheap operator on K rows (NOP leaves acc unchanged).
template <typename T, int K>
__device__ inline void op_value(uint32_t op, typename VecT<T, K>::type& acc,
                                const typename VecT<T, K>::type& t) {
  using O = VOps<T, K>;
  switch (op) {
    case UOP_DIV: acc = O::div(acc, t); GG_BRANCH(); break;
    case UOP_RDIV: acc = O::div(t, acc); GG_BRANCH(); break;
    case UOP_POW: acc = O::pow(acc, t); GG_BRANCH(); break;
    case UOP_RPOW: acc = O::pow(t, acc); GG_BRANCH(); break;
    case UOP_SIN: acc = O::sin(acc); GG_BRANCH(); break;
    case UOP_COS: acc = O::cos(acc); GG_BRANCH(); break;
    case UOP_SQ: acc = acc * acc; GG_BRANCH(); break;
    case UOP_SQRT: acc = O::sqrt(acc); GG_BRANCH(); break;
    case UOP_EXP: acc = O::exp(acc); GG_BRANCH(); break;
    case UOP_LOG: acc = O::log(acc); GG_BRANCH(); break;
    default: GG_BRANCH(); break;  // NOP
  }
}

// Evaluate the program on K rows per lane; returns the predictions.
//   prog    uop source of this individual (UopMem or UopWin)
//   xt      LDS row tile: feature k, row r at xt[k*rstride + r]
//   lrow    this lane's first row within the tile (batch start + lane_row)
//
// The scalar unit is shared by the four SIMDs of a compute unit and its
// instructions (field tests, branches) bound the interpreter's rate, so every
// decision is a single-bit test of the header, the tests are nested (a uop
// pays only for the path it takes) and the END test sits at the loop latch.
template <typename T, int K, int D, class Src>
__device__ inline typename VecT<T, K>::type run_program(Src& prog,
                                                        const float* __restrict__ xt, int rstride,
                                                        int lrow) {
  using V = typename VecT<T, K>::type;
  using O = VOps<T, K>;
  Slots<V, D> st;
  V acc = T(0), t = T(0), pre = T(0);
  const float* __restrict__ xl = xt + lrow;
  uint2 cur = prog.at(0);
  prefetch_operand<T, K>(cur.x, xl, rstride, pre);
  int pc = 0;
#pragma unroll 1
  while (cur.x != UOP_END_HDR) {
    const uint2 nxt = prog.at(pc + 1);
    const uint32_t h = cur.x;
    const float c = f32_of(cur.y);
    operand_stage<T, K, D>(h, c, xl, rstride, acc, t, pre, st);
    // `pre` is consumed: start reading the next uop's first variable operand
    prefetch_operand<T, K>(nxt.x, xl, rstride, pre);
    if (h & U_CHEAP) {  // ADD 1, SUB 2, RSUB 3, MUL 4: bit 2 = MUL, else bits 0-1
      if (h & 4u) {
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
    } else {
      switch (uop_op(h)) {
        case UOP_DIV: acc = O::div(acc, t); GG_BRANCH(); break;
        case UOP_RDIV: acc = O::div(t, acc); GG_BRANCH(); break;
        case UOP_POW: acc = O::pow(acc, t); GG_BRANCH(); break;
        case UOP_RPOW: acc = O::pow(t, acc); GG_BRANCH(); break;
        case UOP_SIN: acc = O::sin(acc); GG_BRANCH(); break;
        case UOP_COS: acc = O::cos(acc); GG_BRANCH(); break;
        case UOP_SQ: acc = acc * acc; GG_BRANCH(); break;
        case UOP_SQRT: acc = O::sqrt(acc); GG_BRANCH(); break;
        case UOP_EXP: acc = O::exp(acc); GG_BRANCH(); break;
        case UOP_LOG: acc = O::log(acc); GG_BRANCH(); break;
        default: GG_BRANCH(); break;  // NOP
      }
      GG_BRANCH();
    }
    cur = nxt;
    ++pc;
  }
  return acc;
}

}  // namespace gg

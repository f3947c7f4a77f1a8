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
// Two kernels share this code and split the individuals between them:
//  * k_adj_reg (most individuals): the tape is a register array of TC entries
//    addressed by a wave-uniform index (indirect VGPR addressing, no LDS), and
//    every lane sums its own rows' constant adjoints in an LDS column (binary32
//    over the R/64 rows of one tile); once per (tile, individual) the wave
//    adds the 64 columns in binary64.  LDS then holds only the row tile, so
//    several blocks share a CU.
//  * k_adj_lds (individuals whose tape exceeds TC entries or whose constants
//    exceed the column count): the tape lives in wave-private LDS and every
//    constant adjoint is reduced across the wave (binary64) per batch.
// A block writes the partials of the individuals it processed; both kernels
// cut the rows into the same spans, so every (individual, span) partial is
// written by exactly one of them.
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
  int R, G, n_groups, n_spans;
  int64_t span_rows;  // rows per span (common to both kernels)
  int tape_cap;       // LDS tape entries per wave (k_adj_lds)
  int reg_tape;       // TC: register tape entries (k_adj_reg)
  int lane_consts;    // CC: constant columns per wave (k_adj_reg)
};

// Which kernel owns individual i (both evaluate the same predicate).
__device__ inline bool adj_active(const ProgMeta& pm, double s1) {
  return pm.status == 0 && s1 != 0.0 && pm.n_const > 0;
}
__device__ inline bool adj_fits_reg(const ProgMeta& pm, int TC, int CC) {
  return pm.n_tape <= TC && pm.n_const <= CC;
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

// Forward sweep with the tape (float nodes).  Same values as run_program; in
// addition each uop stores d(result)/d(acc operand) and d(result)/d(src
// operand) when the reverse sweep needs them (tape_acc / tape_src).
template <int K, int D, class Tape>
__device__ inline typename VecT<float, K>::type run_forward_taped(
    const uint2* __restrict__ prog, const float* __restrict__ xt, int rstride, int lrow,
    Tape& tape) {
  using V = typename VecT<float, K>::type;
  using P = Prot<float>;
  using Dv = Deriv<float>;
  Slots<V, D> st;
  V acc = 0.0f, t = 0.0f, fa = 1.0f, fs = 1.0f;
  const float* __restrict__ xl = xt + lrow;
  uint2 cur = load_uop(prog, 0);
  int pc = 0, tp = 0;
#pragma unroll 1
  for (;;) {
    const uint2 nxt = load_uop(prog, pc + 1);
    const uint32_t h = cur.x;
    const uint32_t op = uop_op(h);
    if (op == UOP_END) break;
    const uint32_t ld = uop_load(h);
    const float c = f32_of(cur.y);
    if (ld != LD_NONE) {
      if (h & HDR_PUSH) { st.put(uop_push_slot(h), acc); GG_BRANCH(); }
      if (ld == LD_VAR) { acc = lds_rows<float, K>(xl + uop_load_arg(h) * rstride); GG_BRANCH(); }
      if (ld == LD_CONST) { acc = c; GG_BRANCH(); }
      GG_BRANCH();
    }
    const uint32_t sk = uop_src(h);
    if (sk == SRC_VAR) { t = lds_rows<float, K>(xl + uop_src_arg(h) * rstride); GG_BRANCH(); }
    if (sk == SRC_POP) { st.get(uop_src_arg(h), t); GG_BRANCH(); }
    if (sk == SRC_CONST) { t = c; GG_BRANCH(); }
    if (op == UOP_ADD) { acc = acc + t; GG_BRANCH(); }
    if (op == UOP_SUB) { acc = acc - t; GG_BRANCH(); }
    if (op == UOP_RSUB) { acc = t - acc; GG_BRANCH(); }
    if (op == UOP_MUL) { fa = t; fs = acc; acc = acc * t; GG_BRANCH(); }
    if (op >= UOP_DIV) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float a = acc[j], b = t[j];
        float v = a, da = 1.0f, ds = 1.0f;
        if (op == UOP_DIV) { v = P::div(a, b); Dv::ddiv(a, b, v, da, ds); }
        if (op == UOP_RDIV) { v = P::div(b, a); Dv::ddiv(b, a, v, ds, da); }
        if (op == UOP_POW) { v = P::pow_(a, b); Dv::dpow(a, b, v, da, ds); }
        if (op == UOP_RPOW) { v = P::pow_(b, a); Dv::dpow(b, a, v, ds, da); }
        if (op == UOP_SIN) { v = P::sin_(a); da = Dv::dsin(a); }
        if (op == UOP_COS) { v = P::cos_(a); da = Dv::dcos(a); }
        if (op == UOP_SQ) { v = a * a; da = 2.0f * a; }
        if (op == UOP_SQRT) { v = P::sqrt_(a); da = Dv::dsqrt(a, v); }
        if (op == UOP_EXP) { v = P::exp_(a); da = Dv::dexp(a, v); }
        if (op == UOP_LOG) { v = P::log_(a); da = Dv::dlog(a); }
        acc[j] = v;
        fa[j] = da;
        fs[j] = ds;
      }
      GG_BRANCH();
    }
    if (tape_acc(h)) { tape.put(tp, fa); ++tp; GG_BRANCH(); }
    if (tape_src(h)) { tape.put(tp, fs); ++tp; GG_BRANCH(); }
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
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
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
    col[c * kColStride] += s;
  }
};

// Reverse sweep.  g = adjoint of the program output per row (zero on padding
// rows); kv = valid rows of this lane.
template <int K, int D, class Tape, class Sink>
__device__ inline void run_reverse(const uint2* __restrict__ prog, int n_uops, int n_tape,
                                   typename VecT<float, K>::type g, const Tape& tape, Sink& sink,
                                   int kv) {
  using V = typename VecT<float, K>::type;
  Slots<V, D> gs;  // adjoints of pushed subtrees
  V gsrc = 0.0f;
  int tp = n_tape;
  uint2 nxt = load_uop(prog, n_uops >= 2 ? n_uops - 2 : 0);
#pragma unroll 1
  for (int pc = n_uops - 2; pc >= 0; --pc) {
    const uint2 u = nxt;
    nxt = load_uop(prog, pc > 0 ? pc - 1 : 0);
    const uint32_t h = u.x;
    const uint32_t op = uop_op(h);
    const uint32_t sk = uop_src(h);
    const int ts = tape_src(h), ta = tape_acc(h);
    if (h & HDR_ADJ_SRC) {  // d result / d src
      if (ts) { --tp; gsrc = g * tape.get(tp); GG_BRANCH(); }
      if (!ts && op == UOP_SUB) { gsrc = -g; GG_BRANCH(); }
      if (!ts && op != UOP_SUB) { gsrc = g; GG_BRANCH(); }  // ADD, RSUB: +1
      if (sk == SRC_CONST) { sink.template add<V, K>(uop_src_arg(h), gsrc, kv); GG_BRANCH(); }
      if (sk == SRC_POP) { gs.put(uop_src_arg(h), gsrc); GG_BRANCH(); }
      GG_BRANCH();
    }
    if (h & HDR_ADJ_ACC) {  // d result / d acc operand
      if (ta) { --tp; g = g * tape.get(tp); GG_BRANCH(); }
      if (!ta && op == UOP_RSUB) { g = -g; GG_BRANCH(); }
      if (!ta && op == UOP_MUL) { g = g * f32_of(u.y); GG_BRANCH(); }  // constant factor
      if (uop_load(h) == LD_CONST) { sink.template add<V, K>(uop_load_arg(h), g, kv); GG_BRANCH(); }
      GG_BRANCH();
    }
    if (h & HDR_PUSH) { gs.get(uop_push_slot(h), g); GG_BRANCH(); }
  }
}

// Block prologue shared by both kernels: the (span, group) of this block with
// the same XCD-aware numbering as the forward kernel (consecutive items, which
// share a span and so the same rows of X, land on one XCD and its L2).
struct AdjItem {
  int span, ind0, Gn;
};
__device__ inline AdjItem adj_item(const AdjParams& p) {
  const int total = p.n_spans * p.n_groups;
  const int b0 = blockIdx.x;
  const int x = b0 & 7, kk = b0 >> 3, q = total >> 3, r8 = total & 7;
  const int item = x * q + (x < r8 ? x : r8) + kk;
  const int span = item / p.n_groups, grp = item - span * p.n_groups;
  const int ind0 = grp * p.G;
  return {span, ind0, min(p.G, p.M - ind0)};
}

// Stage one row tile of X (feature-major, zero past the last row) and the
// centred targets into LDS.
__device__ inline void adj_stage(const AdjParams& p, float* xs, double* yts, int64_t r0, int nvalid,
                                 double ybar) {
  for (int f = 0; f < p.F; ++f) {
    const float* __restrict__ src = p.X + size_t(f) * p.ldx + r0;
    for (int r = threadIdx.x; r < p.R; r += blockDim.x) xs[size_t(f) * p.R + r] = r < nvalid ? src[r] : 0.0f;
  }
  for (int r = threadIdx.x; r < p.R; r += blockDim.x)
    yts[r] = r < nvalid ? double(p.y[r0 + r]) - ybar : 0.0;
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

// Write this block's partials of the individuals `mine` selects.
template <class Pred>
__device__ inline void adj_write(const AdjParams& p, const AdjItem& it, const double* gacc, Pred mine) {
  for (int j = threadIdx.x; j < it.Gn * p.C_max; j += blockDim.x) {
    const int jj = j / p.C_max, c = j - jj * p.C_max;
    const int i = it.ind0 + jj;
    if (mine(i)) p.gpart[(size_t(i) * p.n_spans + it.span) * p.C_max + c] = gacc[j];
  }
}

template <int K, int D, int W, int TC>
__global__ __launch_bounds__(W * 64) void k_adj_reg(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  const int CC = p.lane_consts;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;                                    // G * C_max
  float* lacc_all = reinterpret_cast<float*>(gacc + size_t(p.G) * p.C_max);  // W * CC * 65

  const AdjItem it = adj_item(p);
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  float* lacc = lacc_all + size_t(wv) * CC * kColStride;
  LaneSink sink{lacc + lane};

  for (int j = threadIdx.x; j < it.Gn * p.C_max; j += blockDim.x) gacc[j] = 0.0;
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);
  for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
    const int nvalid = int(min<int64_t>(R, s_end - r0));
    __syncthreads();
    adj_stage(p, xs, yts, r0, nvalid, ybar);
    __syncthreads();
    const int nbatch = (nvalid + BR - 1) / BR;
    for (int jj = wv; jj < it.Gn; jj += W) {  // wave-uniform trip count
      const int i = it.ind0 + jj;
      const ProgMeta pm = p.meta[i];
      const double s1 = p.ab[size_t(i) * 2 + 1];
      const int skip = !adj_active(pm, s1) || !adj_fits_reg(pm, TC, CC);
      if (__builtin_amdgcn_readfirstlane(skip)) continue;
      const int nc = __builtin_amdgcn_readfirstlane(pm.n_const);
      const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;
      const uint2* prog = p.uops + size_t(i) * p.U_stride;
      for (int c = 0; c < nc; ++c) lacc[c * kColStride + lane] = 0.0f;
      for (int b = 0; b < nbatch; ++b) {
        const int lrow = b * BR + lane * K;
        RegTape<K, TC> tape;
        const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
        const auto g = adj_seed<K>(v, s0m, s1, yts, lrow, nvalid);
        const int kv = max(0, min(K, nvalid - lrow));
        run_reverse<K, D>(prog, pm.n_uops, pm.n_tape, g, tape, sink, kv);
      }
      // the wave's column writes must land before lane c reads column c
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < nc) {
        const float* colc = lacc + lane * kColStride;
        double s0 = 0.0, s1r = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
        for (int k = 0; k < 64; k += 4) {
          s0 += double(colc[k]);
          s1r += double(colc[k + 1]);
          s2 += double(colc[k + 2]);
          s3 += double(colc[k + 3]);
        }
        gacc[size_t(jj) * p.C_max + lane] += (s0 + s1r) + (s2 + s3);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  adj_write(p, it, gacc, [&](int i) {
    const ProgMeta pm = p.meta[i];
    return adj_active(pm, p.ab[size_t(i) * 2 + 1]) && adj_fits_reg(pm, TC, CC);
  });
}

// LDS-tape kernel: only the individuals the register kernel cannot take.
// They are rare, so all W waves share each one: wave w takes batches w, w+W,
// ... of a tile and adds its constant adjoints to its own copy of the
// accumulators; the copies are summed in wave order at the end (bitwise
// repeatable).  A block whose group holds none of them exits at once.
template <int K, int D, int W>
__global__ __launch_bounds__(W * 64) void k_adj_lds(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  const int TC = p.reg_tape, CC = p.lane_consts;
  __shared__ int any;
  const AdjItem it = adj_item(p);
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (int(threadIdx.x) < it.Gn) {
    const int i = it.ind0 + threadIdx.x;
    const ProgMeta pm = p.meta[i];
    if (adj_active(pm, p.ab[size_t(i) * 2 + 1]) && !adj_fits_reg(pm, TC, CC)) any = 1;
  }
  __syncthreads();
  if (any == 0) return;

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

  for (int j = threadIdx.x; j < W * GC; j += blockDim.x) gacc[j] = 0.0;
  const int64_t s_begin = int64_t(it.span) * p.span_rows;
  const int64_t s_end = min<int64_t>(p.N, s_begin + p.span_rows);
  for (int64_t r0 = s_begin; r0 < s_end; r0 += R) {
    const int nvalid = int(min<int64_t>(R, s_end - r0));
    __syncthreads();
    adj_stage(p, xs, yts, r0, nvalid, ybar);
    __syncthreads();
    const int nbatch = (nvalid + BR - 1) / BR;
    for (int jj = 0; jj < it.Gn; ++jj) {  // uniform over the block
      const int i = it.ind0 + jj;
      const ProgMeta pm = p.meta[i];
      const double s1 = p.ab[size_t(i) * 2 + 1];
      const int skip = !adj_active(pm, s1) || adj_fits_reg(pm, TC, CC) || pm.n_tape > p.tape_cap;
      if (__builtin_amdgcn_readfirstlane(skip)) continue;
      const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;
      const uint2* prog = p.uops + size_t(i) * p.U_stride;
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
  adj_write(p, it, gacc, [&](int i) {
    const ProgMeta pm = p.meta[i];
    return adj_active(pm, p.ab[size_t(i) * 2 + 1]) && !adj_fits_reg(pm, TC, CC);
  });
}

template <int K, int D, int W, int TC>
static hipError_t reg_impl(const AdjPlan& a, const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_reg_lds_bytes(ap.F, a.reg.R, a.reg.G, ap.C_max, W, a.lane_consts);
  const int nb = a.n_spans * a.reg.n_groups;
  hipLaunchKernelGGL((k_adj_reg<K, D, W, TC>), dim3(nb), dim3(W * 64), sh, s, ap);
  return hipGetLastError();
}

template <int K, int D, int W>
static hipError_t lds_impl(const AdjPlan& a, const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_lds_bytes(ap.F, a.wide.R, a.wide.G, ap.C_max, W, K, ap.tape_cap);
  const int nb = a.n_spans * a.wide.n_groups;
  hipLaunchKernelGGL((k_adj_lds<K, D, W>), dim3(nb), dim3(W * 64), sh, s, ap);
  return hipGetLastError();
}

static AdjParams adj_params(const AdjPlan& a, const TileCfg& c, const uint2* uops, int U_stride,
                            const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                            const double* stats, const double* ab, double* gpart) {
  return AdjParams{uops, U_stride, meta, M, C_max, d.X, d.ldx, d.F, d.N, d.y, stats, ab, gpart,
                   c.R, c.G, c.n_groups, a.n_spans, a.span_rows, a.tape_cap, a.reg_tape,
                   a.lane_consts};
}

hipError_t launch_adjoint_reg(const AdjPlan& a, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart, hipStream_t s) {
  const AdjParams ap = adj_params(a, a.reg, uops, U_stride, meta, M, C_max, d, stats, ab, gpart);
  const TileCfg& r = a.reg;
  if (r.W != 4) return hipErrorInvalidValue;
  if (r.K == 4 && a.reg_tape == 16 && r.D == 4) return reg_impl<4, 4, 4, 16>(a, ap, s);
  if (r.K == 4 && a.reg_tape == 16 && r.D == 8) return reg_impl<4, 8, 4, 16>(a, ap, s);
  if (r.K == 2 && a.reg_tape == 32 && r.D == 4) return reg_impl<2, 4, 4, 32>(a, ap, s);
  if (r.K == 2 && a.reg_tape == 32 && r.D == 8) return reg_impl<2, 8, 4, 32>(a, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

hipError_t launch_adjoint_lds(const AdjPlan& a, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart, hipStream_t s) {
  const AdjParams ap = adj_params(a, a.wide, uops, U_stride, meta, M, C_max, d, stats, ab, gpart);
  const TileCfg& w = a.wide;
  if (w.D != 8) return hipErrorInvalidValue;
  if (w.K == 2 && w.W == 4) return lds_impl<2, 8, 4>(a, ap, s);
  if (w.K == 2 && w.W == 2) return lds_impl<2, 8, 2>(a, ap, s);
  if (w.K == 2 && w.W == 1) return lds_impl<2, 8, 1>(a, ap, s);
  if (w.K == 1 && w.W == 4) return lds_impl<1, 8, 4>(a, ap, s);
  if (w.K == 1 && w.W == 2) return lds_impl<1, 8, 2>(a, ap, s);
  if (w.K == 1 && w.W == 1) return lds_impl<1, 8, 1>(a, ap, s);
  return hipErrorInvalidValue;  // no kernel instantiated for this launch shape
}

__global__ __launch_bounds__(256) void k_grad_finalize(const ProgMeta* __restrict__ meta, int M,
                                                       int C_max, const double* __restrict__ gpart,
                                                       int n_spans, const double* __restrict__ stats,
                                                       const double* __restrict__ ab,
                                                       double* __restrict__ grad) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(M) * C_max) return;
  const int i = int(idx / C_max), j = int(idx - int64_t(i) * C_max);
  const ProgMeta pm = meta[i];
  double g = 0.0;
  const double s1 = ab[size_t(i) * 2 + 1];
  if (pm.status == 0 && j < pm.n_const && s1 != 0.0) {
    const double* q = gpart + size_t(i) * n_spans * C_max + j;
    for (int s = 0; s < n_spans; ++s) g += q[size_t(s) * C_max];
    g *= 2.0 * s1 / stats[ST_N];
  }
  grad[idx] = g;
}

hipError_t launch_grad_finalize(const ProgMeta* meta, int M, int C_max, const double* gpart,
                                int n_spans, const double* stats, const double* ab,
                                uint32_t flags, const int8_t* status, double* grad,
                                hipStream_t s) {
  (void)flags;
  (void)status;
  const int64_t n = int64_t(M) * C_max;
  hipLaunchKernelGGL(k_grad_finalize, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, meta, M,
                     C_max, gpart, n_spans, stats, ab, grad);
  return hipGetLastError();
}

}  // namespace gg

// Reverse-mode gradient of the fitness with respect to every constant.
//
// With linear scaling the optimal (a, b) have zero partials (envelope
// theorem), so  d LS-MSE / d c_j = (2b/N) sum_r (a + b p_r - y_r) dp_r/dc_j;
// without it  d MSE / d c_j = (2/N) sum_r (p_r - y_r) dp_r/dc_j.  Both are
// written  (2 s1/N) sum_r (s0 + s1 p_r - y_r) dp_r/dc_j  with (s0, s1) = (a, b)
// or (0, 1), taken from the forward pass (which must run first).
//
// Per row tile and individual a wave runs the program forward over K rows per
// lane, storing every local partial the reverse sweep will need on a
// wave-private LDS tape (the tree's values are recomputed per tile rather than
// kept from the forward pass), seeds the output adjoint with the residual, and
// walks the uops backwards.  A tree node has exactly one parent, so adjoints
// never accumulate except at constants: each constant's adjoint is summed over
// the wave's rows and added (binary64) to the block's per-(individual,
// constant) accumulator in LDS; a block writes one partial per span.
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
  double* gpart;  // [M][n_spans][C_max]
  int R, G, n_groups, n_spans, tiles_per_span, tape_cap;
};

template <int K>
struct TapeRef {
  using V = typename VecT<float, K>::type;
  float* base;  // this wave's tape: entry e, lane l at base[(e*64 + l)*K]
  int lane;
  __device__ inline float* at(int e) const { return base + (size_t(e) * 64 + lane) * K; }
  __device__ inline void put(int e, const V& v) const {
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

// Forward sweep with the tape (float nodes).  Same values as run_program; in
// addition each uop stores d(result)/d(acc operand) and d(result)/d(src
// operand) when the reverse sweep needs them (tape_acc / tape_src).
template <int K, int D>
__device__ inline typename VecT<float, K>::type run_forward_taped(
    const uint2* __restrict__ prog, const float* __restrict__ xt, int rstride, int lrow,
    const TapeRef<K>& tape) {
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
    if (tape_acc(h)) { tape.put(tp++, fa); GG_BRANCH(); }
    if (tape_src(h)) { tape.put(tp++, fs); GG_BRANCH(); }
    cur = nxt;
    ++pc;
  }
  return acc;
}

// Sum over the wave of this lane's first `kv` values (padding rows excluded:
// their adjoints may be NaN after multiplying a zero by an infinite partial).
// Summed in binary64: a constant whose gradient is a cancelling sum (one the
// linear fit absorbs has an exactly zero gradient) keeps its float32 per-row
// terms but loses nothing more in the reduction.
template <int K>
__device__ inline double wave_total(const typename VecT<float, K>::type& v, int kv) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) s += j < kv ? double(v[j]) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

// Reverse sweep.  g = adjoint of the program output per row (zero on padding
// rows); gacc = this individual's constant accumulators in LDS (binary64).
template <int K, int D>
__device__ inline void run_reverse(const uint2* __restrict__ prog, int n_uops, int n_tape,
                                   typename VecT<float, K>::type g, const TapeRef<K>& tape,
                                   double* gacc, int lane, int kv) {
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
      if (ts) { gsrc = g * tape.get(--tp); GG_BRANCH(); }
      if (!ts && op == UOP_SUB) { gsrc = -g; GG_BRANCH(); }
      if (!ts && op != UOP_SUB) { gsrc = g; GG_BRANCH(); }  // ADD, RSUB: +1
      if (sk == SRC_CONST) {
        const double s = wave_total<K>(gsrc, kv);  // same value on every lane
        gacc[uop_src_arg(h)] += s;
        GG_BRANCH();
      }
      if (sk == SRC_POP) { gs.put(uop_src_arg(h), gsrc); GG_BRANCH(); }
      GG_BRANCH();
    }
    if (h & HDR_ADJ_ACC) {  // d result / d acc operand
      if (ta) { g = g * tape.get(--tp); GG_BRANCH(); }
      if (!ta && op == UOP_RSUB) { g = -g; GG_BRANCH(); }
      if (!ta && op == UOP_MUL) { g = g * f32_of(u.y); GG_BRANCH(); }  // constant factor
      if (uop_load(h) == LD_CONST) {
        const double s = wave_total<K>(g, kv);
        gacc[uop_load_arg(h)] += s;
        GG_BRANCH();
      }
      GG_BRANCH();
    }
    if (h & HDR_PUSH) { gs.get(uop_push_slot(h), g); GG_BRANCH(); }
  }
}

template <int K, int D, int W>
__global__ __launch_bounds__(W * 64) void k_fused_adj(AdjParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* gacc = yts + R;  // G * C_max
  const size_t off_ctr = (size_t(p.F) * R * 4 + size_t(R) * 8 + size_t(p.G) * p.C_max * 8 + 15) & ~size_t(15);
  float* tape_all = reinterpret_cast<float*>(smem_raw + off_ctr + 16);

  const int total = p.n_spans * p.n_groups;
  const int b0 = blockIdx.x;
  const int x = b0 & 7, kk = b0 >> 3, q = total >> 3, r8 = total & 7;
  const int item = x * q + (x < r8 ? x : r8) + kk;
  const int span = item / p.n_groups, grp = item - span * p.n_groups;
  const int ind0 = grp * p.G;
  const int Gn = min(p.G, p.M - ind0);
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;
  TapeRef<K> tape{tape_all + size_t(wv) * p.tape_cap * 64 * K, lane};

  for (int j = threadIdx.x; j < Gn * p.C_max; j += blockDim.x) gacc[j] = 0.0;
  const int64_t span_r0 = int64_t(span) * p.tiles_per_span * R;
  for (int tile = 0; tile < p.tiles_per_span; ++tile) {
    const int64_t r0 = span_r0 + int64_t(tile) * R;
    if (r0 >= p.N) break;
    const int nvalid = int(min<int64_t>(R, p.N - r0));
    __syncthreads();
    for (int f = 0; f < p.F; ++f) {
      const float* __restrict__ src = p.X + size_t(f) * p.ldx + r0;
      for (int r = threadIdx.x; r < R; r += blockDim.x) xs[size_t(f) * R + r] = r < nvalid ? src[r] : 0.0f;
    }
    for (int r = threadIdx.x; r < R; r += blockDim.x)
      yts[r] = r < nvalid ? double(p.y[r0 + r]) - ybar : 0.0;
    __syncthreads();
    const int nbatch = (nvalid + BR - 1) / BR;
    for (int jj = wv; jj < Gn; jj += W) {  // wave-uniform, see the forward kernel
      const int i = ind0 + jj;
      const ProgMeta pm = p.meta[i];
      const double s1 = p.ab[size_t(i) * 2 + 1];
      const int skip = pm.status != 0 || s1 == 0.0 || pm.n_const == 0 || pm.n_tape > p.tape_cap;
      if (__builtin_amdgcn_readfirstlane(skip)) continue;
      const double s0m = p.ab[size_t(i) * 2 + 0] - ybar;  // residual = (s0 - ybar) + s1 p - yt
      const uint2* prog = p.uops + size_t(i) * p.U_stride;
      double* ga = gacc + size_t(jj) * p.C_max;
      for (int b = 0; b < nbatch; ++b) {
        const int lrow = b * BR + lane * K;
        typename VecT<float, K>::type g;
        const auto v = run_forward_taped<K, D>(prog, xs, R, lrow, tape);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const bool ok = lrow + j < nvalid;
          const double res = (s0m + s1 * double(v[j])) - yts[lrow + j];
          g[j] = ok ? float(res) : 0.0f;
        }
        const int kv = max(0, min(K, nvalid - lrow));
        run_reverse<K, D>(prog, pm.n_uops, pm.n_tape, g, tape, ga, lane, kv);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < Gn * p.C_max; j += blockDim.x) {
    const int jj = j / p.C_max, c = j - jj * p.C_max;
    p.gpart[(size_t(ind0 + jj) * p.n_spans + span) * p.C_max + c] = gacc[j];
  }
}

template <int K, int D, int W>
static hipError_t adj_impl(const TileCfg& c, const AdjParams& ap, hipStream_t s) {
  const size_t sh = adjoint_lds_bytes(ap.F, ap.R, ap.G, ap.C_max, W, K, ap.tape_cap);
  const int nb = c.n_spans * c.n_groups;
  hipLaunchKernelGGL((k_fused_adj<K, D, W>), dim3(nb), dim3(W * 64), sh, s, ap);
  return hipGetLastError();
}

hipError_t launch_fused_adjoint(const TileCfg& c, const uint2* uops, int U_stride,
                                const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                                const double* stats, const double* ab, double* gpart,
                                float* tape_spill, int tape_lds, hipStream_t s) {
  (void)tape_spill;
  AdjParams ap{uops, U_stride, meta, M, C_max, d.X, d.ldx, d.F, d.N, d.y, stats, ab, gpart,
               c.R, c.G, c.n_groups, c.n_spans, c.tiles_per_span, tape_lds};
  if (c.D != 8) return hipErrorInvalidValue;
  if (c.K == 2 && c.W == 4) return adj_impl<2, 8, 4>(c, ap, s);
  if (c.K == 2 && c.W == 2) return adj_impl<2, 8, 2>(c, ap, s);
  if (c.K == 2 && c.W == 1) return adj_impl<2, 8, 1>(c, ap, s);
  if (c.K == 1 && c.W == 4) return adj_impl<1, 8, 4>(c, ap, s);
  if (c.K == 1 && c.W == 2) return adj_impl<1, 8, 2>(c, ap, s);
  if (c.K == 1 && c.W == 1) return adj_impl<1, 8, 1>(c, ap, s);
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

// Per-call preparation kernels:
//   * dataset statistics of y (mean, population variance), two passes in
//     binary64 with fixed-order reductions (deterministic);
//   * the device compile step that turns each postfix program into the uop
//     stream of the register-stack interpreter and validates it;
//   * the probe that evaluates each program on the first rows to get the
//     shift used by the moment sums.
#include <hip/hip_runtime.h>

#include "gpgomea_ops.h"
#include "interp.h"
#include "kernels.h"

namespace gg {

// ---------------------------------------------------------------- statistics
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kStatBlocks) void k_ysum(const float* __restrict__ y, int64_t N,
                                                      double* __restrict__ part) {
  __shared__ double sh[kStatBlocks];
  double acc = 0.0;
  for (int64_t r = int64_t(blockIdx.x) * kStatBlocks + threadIdx.x; r < N;
       r += int64_t(gridDim.x) * kStatBlocks)
    acc += double(y[r]);
  const double s = block_sum<kStatBlocks>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of the kStatBlocks partials, one per thread, in a fixed tree order.
__device__ inline double sum_partials(const double* __restrict__ part, double* sh) {
  return block_sum<kStatBlocks>(part[threadIdx.x], sh);
}

__global__ __launch_bounds__(kStatBlocks) void k_ydev(const float* __restrict__ y, int64_t N,
                                                      const double* __restrict__ psum,
                                                      double* __restrict__ pdev,
                                                      double* __restrict__ pss) {
  __shared__ double sh[kStatBlocks];
  const double ybar = sum_partials(psum, sh) / double(N);
  double a = 0.0, b = 0.0;
  for (int64_t r = int64_t(blockIdx.x) * kStatBlocks + threadIdx.x; r < N;
       r += int64_t(gridDim.x) * kStatBlocks) {
    const double d = double(y[r]) - ybar;
    a += d;
    b = fma(d, d, b);
  }
  const double sa = block_sum<kStatBlocks>(a, sh);
  const double sb = block_sum<kStatBlocks>(b, sh);
  if (threadIdx.x == 0) {
    pdev[blockIdx.x] = sa;
    pss[blockIdx.x] = sb;
  }
}

// ybar, Var(y) = mean of (y - ybar)^2 minus the square of the mean deviation
// (a rounding-level correction), and sum (y - ybar).
__global__ __launch_bounds__(kStatBlocks) void k_yfinal(const double* __restrict__ scratch, int64_t N,
                                                        double* __restrict__ stats) {
  __shared__ double sh[kStatBlocks];
  const double ybar = sum_partials(scratch, sh) / double(N);
  const double sd = sum_partials(scratch + kStatBlocks, sh);
  const double ss = sum_partials(scratch + 2 * kStatBlocks, sh);
  if (threadIdx.x != 0) return;
  const double md = sd / double(N);
  const double vy = ss / double(N) - md * md;
  stats[ST_YBAR] = ybar;
  stats[ST_VY] = vy > 0.0 ? vy : 0.0;
  stats[ST_YT] = sd;
  stats[ST_N] = double(N);
}

hipError_t launch_ystats(const float* y, int64_t N, double* stats, double* scratch, hipStream_t s) {
  const int nb = kStatBlocks;  // blocks of the passes = threads of the partial sums
  hipLaunchKernelGGL(k_ysum, dim3(nb), dim3(kStatBlocks), 0, s, y, N, scratch);
  hipLaunchKernelGGL(k_ydev, dim3(nb), dim3(kStatBlocks), 0, s, y, N, scratch, scratch + nb,
                     scratch + 2 * nb);
  hipLaunchKernelGGL(k_yfinal, dim3(1), dim3(kStatBlocks), 0, s, scratch, N, stats);
  return hipGetLastError();
}

// ------------------------------------------------------------------ compile
constexpr int kLMax = 512;

struct CompileLds {
  int16_t kl[kLMax], kr[kLMax], ci[kLMax], stk[kLMax];
  int16_t clo[kLMax], cnum[kLMax];  // constants of the subtree: ordinals [clo, clo + cnum)
  int8_t sym[kLMax];
  uint8_t need[kLMax], hasc[kLMax], stt[kLMax];
  uint8_t written[kLMax];  // path mode: the subtree's constant entries have been written
};

__device__ inline int arity_of(int s) {
  if ((s >= GPGOMEA_SYM_ADD && s <= GPGOMEA_SYM_DIV) || s == GPGOMEA_SYM_POW) return 2;
  if (s >= GPGOMEA_SYM_SIN && s <= GPGOMEA_SYM_LOG) return 1;
  return 0;
}
__device__ inline bool is_term(int s) { return s == GPGOMEA_SYM_CONST || s >= GPGOMEA_SYM_VAR0; }

__device__ inline uint32_t bin_uop(int s, bool reversed) {
  switch (s) {
    case GPGOMEA_SYM_ADD: return UOP_ADD;
    case GPGOMEA_SYM_SUB: return reversed ? UOP_RSUB : UOP_SUB;
    case GPGOMEA_SYM_MUL: return UOP_MUL;
    case GPGOMEA_SYM_DIV: return reversed ? UOP_RDIV : UOP_DIV;
    default: return reversed ? UOP_RPOW : UOP_POW;
  }
}
__device__ inline uint32_t un_uop(int s) {
  switch (s) {
    case GPGOMEA_SYM_SIN: return UOP_SIN;
    case GPGOMEA_SYM_COS: return UOP_COS;
    case GPGOMEA_SYM_SQ: return UOP_SQ;
    case GPGOMEA_SYM_SQRT: return UOP_SQRT;
    case GPGOMEA_SYM_EXP: return UOP_EXP;
    default: return UOP_LOG;
  }
}
__device__ inline int uop_cost(uint32_t op) {
  switch (op) {
    case UOP_DIV: case UOP_RDIV: return 10;
    case UOP_POW: case UOP_RPOW: return 40;
    case UOP_SIN: case UOP_COS: return 30;
    case UOP_SQRT: return 8;
    case UOP_EXP: return 12;
    case UOP_LOG: return 16;
    case UOP_END: case UOP_NOP: return 0;
    default: return 1;
  }
}

// Path forward mode keeps, per constant j, an entry T[j]: the product of the
// local partials from constant j up to the last point where its subtree was
// folded into T ("flushed": at a merge, a uop whose two operands both hold
// constants, and at the push of a value that holds constants).  The compile
// step lists these flush events in uop order, one uint2 each (x: the acc side
// of a merge or the pushed value, y: a merge's src side, 0 for a push); a
// side is
//   lo (9 bits) | n (9 bits) << 9 | assign << 18
// where [lo, lo + n) is the operand's constant range (contiguous in postfix
// order) and `assign` says the entry has never been written (a single
// constant): T[lo] = f instead of T[e] *= f.  A program of L tokens has at most
// L - 1 events (one merge and one push per binary operator), so a row of
// L_max events never overflows.
__device__ inline uint32_t flush_side(int lo, int n, bool assign) {
  return uint32_t(lo & 511) | (uint32_t(n & 511) << 9) | (assign ? 1u << 18 : 0u);
}

// Emits uops of one program; state lives in LDS, one active lane.
struct Emitter {
  uint2* out;
  const float* cs;
  CompileLds* L;
  uint2* events;  // flush events, in uop order
  int event_cap = 0, n_event = 0;
  int n = 0, cap = 0, tape = 0, cost = 0;
  bool push_pending = false;
  uint32_t push_slot = 0;
  int push_node = -1;  // the subtree pushed by the next uop
  bool bad = false;

  __device__ inline void event(uint32_t a, uint32_t s) {
    if (n_event < event_cap) events[n_event] = make_uint2(a, s);
    else bad = true;  // cannot happen (event_cap >= L_max - 1); never drop one silently
    ++n_event;
  }
  __device__ inline void emit(uint32_t hdr, uint32_t payload) {
    if (push_pending) {
      if (uop_load(hdr) == LD_NONE) bad = true;  // a pushed subtree starts with a load
      const int pn = push_node;
      const bool hc = L->hasc[pn] != 0;
      hdr = with_push(hdr, push_slot, hc);
      if (hc) {  // the pushed value's pending factor is folded into T
        event(flush_side(L->clo[pn], L->cnum[pn], !L->written[pn]), 0u);
        L->written[pn] = 1;
      }
      push_pending = false;
    }
    if (n >= cap) {
      bad = true;
      return;
    }
    out[n++] = make_uint2(hdr, payload);
    tape += tape_acc(hdr) + tape_src(hdr);
    cost += uop_cost(uop_op(hdr));
  }
  // the uop just emitted merges operand subtree a (acc) and b (src), both
  // holding constants; the result's entries are all written
  __device__ inline void merge(int a, int b) {
    event(flush_side(L->clo[a], L->cnum[a], !L->written[a]),
          flush_side(L->clo[b], L->cnum[b], !L->written[b]));
  }
};

// terminal operand descriptor: (src kind, arg, payload, has-constant)
__device__ inline void term_operand(const CompileLds& L, int t, const float* cs, uint32_t& kind,
                                    uint32_t& arg, uint32_t& pay, bool& hc) {
  const int s = L.sym[t];
  if (s == GPGOMEA_SYM_CONST) {
    kind = SRC_CONST;
    arg = uint32_t(L.ci[t]);
    pay = __float_as_uint(cs[L.ci[t]]);
    hc = true;
  } else {
    kind = SRC_VAR;
    arg = uint32_t(s - GPGOMEA_SYM_VAR0);
    pay = 0;
    hc = false;
  }
}

__global__ __launch_bounds__(256) void k_compile(const int8_t* __restrict__ ops, int M, int L_max,
                                                 const float* __restrict__ consts, int C_max, int F,
                                                 int Dmax, int U_stride, uint2* __restrict__ uops,
                                                 ProgMeta* __restrict__ meta,
                                                 uint2* __restrict__ events, int ET) {
  __shared__ CompileLds smem[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  CompileLds& L = smem[w];
  if (i < M)
    for (int t = lane; t < L_max; t += 64) L.sym[t] = ops[size_t(i) * L_max + t];
  __syncthreads();
  if (i >= M || lane != 0) return;

  const float* cs = consts + size_t(i) * C_max;
  uint2* out = uops + size_t(i) * U_stride;
  ProgMeta pm{};
  pm.status = 0;
  // ---- parse, validate, Sethi-Ullman need, constant ordinals
  int Ln = 0;
  while (Ln < L_max && L.sym[Ln] != GPGOMEA_SYM_END) ++Ln;
  bool bad = (Ln == 0);
  int sp = 0, nc = 0;
  for (int t = 0; t < Ln && !bad; ++t) {
    const int s = L.sym[t];
    const int ar = arity_of(s);
    L.kl[t] = L.kr[t] = -1;
    L.ci[t] = -1;
    L.clo[t] = int16_t(nc);
    L.cnum[t] = 0;
    L.written[t] = 0;
    if (ar == 0) {
      if (s == GPGOMEA_SYM_CONST) {
        if (nc >= C_max) bad = true;
        L.ci[t] = int16_t(nc++);
        L.hasc[t] = 1;
        L.cnum[t] = 1;
      } else if (s >= GPGOMEA_SYM_VAR0 && s - GPGOMEA_SYM_VAR0 < F) {
        L.hasc[t] = 0;
      } else {
        bad = true;
      }
      L.need[t] = 0;
    } else {
      if (sp < ar) {
        bad = true;
        break;
      }
      if (ar == 2) {
        const int b = L.stk[--sp], a = L.stk[--sp];
        L.kl[t] = int16_t(a);
        L.kr[t] = int16_t(b);
        const bool ta = is_term(L.sym[a]), tb = is_term(L.sym[b]);
        int nd;
        if (ta && tb) nd = 0;
        else if (ta) nd = L.need[b];
        else if (tb) nd = L.need[a];
        else {
          const int na = L.need[a], nb = L.need[b];
          nd = (na >= nb) ? max(na, 1 + nb) : max(nb, 1 + na);
        }
        L.need[t] = uint8_t(nd > 255 ? 255 : nd);
        L.hasc[t] = L.hasc[a] | L.hasc[b];
        L.clo[t] = L.clo[a];  // the left operand's constants come first in postfix
        L.cnum[t] = int16_t(L.cnum[a] + L.cnum[b]);
      } else {
        const int a = L.stk[--sp];
        L.kl[t] = int16_t(a);
        L.need[t] = L.need[a];
        L.hasc[t] = L.hasc[a];
        L.clo[t] = L.clo[a];
        L.cnum[t] = L.cnum[a];
      }
    }
    L.stk[sp++] = int16_t(t);
  }
  if (!bad && sp != 1) bad = true;
  Emitter E;
  E.out = out;
  E.cs = cs;
  E.L = &L;
  E.events = events + size_t(i) * ET;
  E.event_cap = ET;
  E.cap = U_stride - 2;
  int maxsp = 0;
  if (!bad) {
    const int root = L.stk[0];
    if (L.need[root] > Dmax) bad = true;
    // ---- emission: explicit post-order traversal, Sethi-Ullman child order
    int top = 0;
    L.stk[0] = int16_t(root);
    L.stt[0] = 0;
    int dsp = 0;
    while (top >= 0 && !bad && !E.bad) {
      const int n = L.stk[top];
      const int st = L.stt[top];
      const int s = L.sym[n];
      const int ar = arity_of(s);
      if (ar == 0) {  // a lone terminal program
        uint32_t k, a, pay;
        bool hc;
        term_operand(L, n, cs, k, a, pay, hc);
        const uint32_t ld = (k == SRC_CONST) ? LD_CONST : LD_VAR;
        E.emit(make_hdr(UOP_NOP, SRC_NONE, 0, ld, a) | (hc ? HDR_ADJ_ACC : 0), pay);
        --top;
        continue;
      }
      if (ar == 1) {
        const int c = L.kl[n];
        if (!is_term(L.sym[c])) {
          if (st == 0) {
            L.stt[top] = 1;
            ++top;
            L.stk[top] = int16_t(c);
            L.stt[top] = 0;
            continue;
          }
          E.emit(make_hdr(un_uop(s), SRC_NONE, 0, LD_NONE, 0) | (L.hasc[c] ? HDR_ADJ_ACC : 0), 0);
          L.written[n] = L.written[c];
        } else {
          uint32_t k, a, pay;
          bool hc;
          term_operand(L, c, cs, k, a, pay, hc);
          const uint32_t ld = (k == SRC_CONST) ? LD_CONST : LD_VAR;
          E.emit(make_hdr(un_uop(s), SRC_NONE, 0, ld, a) | (hc ? HDR_ADJ_ACC : 0), pay);
        }
        --top;
        continue;
      }
      const int a = L.kl[n], b = L.kr[n];
      const bool ta = is_term(L.sym[a]), tb = is_term(L.sym[b]);
      if (ta && tb) {
        uint32_t ka, aa, pa, kb, ab, pb;
        bool ha, hb;
        term_operand(L, a, cs, ka, aa, pa, ha);
        term_operand(L, b, cs, kb, ab, pb, hb);
        if (ka == SRC_CONST && kb == SRC_CONST) {
          E.emit(make_hdr(UOP_NOP, SRC_NONE, 0, LD_CONST, aa) | HDR_ADJ_ACC, pa);
          E.emit(make_hdr(bin_uop(s, false), SRC_CONST, ab, LD_NONE, 0) | HDR_ADJ_ACC | HDR_ADJ_SRC, pb);
          E.merge(a, b);
          L.written[n] = 1;
        } else if (ka == SRC_CONST) {  // load the variable b, constant a is the src: a op b
          E.emit(make_hdr(bin_uop(s, true), SRC_CONST, aa, LD_VAR, ab) | HDR_ADJ_SRC, pa);
        } else {  // load variable a; b is a variable or a constant
          E.emit(make_hdr(bin_uop(s, false), kb, ab, LD_VAR, aa) | (hb ? HDR_ADJ_SRC : 0), pb);
        }
        --top;
        continue;
      }
      if (ta || tb) {
        const int nt = ta ? b : a;  // the non-terminal operand, evaluated into acc
        const int tt = ta ? a : b;
        if (st == 0) {
          L.stt[top] = 1;
          ++top;
          L.stk[top] = int16_t(nt);
          L.stt[top] = 0;
          continue;
        }
        uint32_t k, ar2, pay;
        bool hc;
        term_operand(L, tt, cs, k, ar2, pay, hc);
        E.emit(make_hdr(bin_uop(s, ta), k, ar2, LD_NONE, 0) | (L.hasc[nt] ? HDR_ADJ_ACC : 0) |
                   (hc ? HDR_ADJ_SRC : 0),
               pay);
        if (L.hasc[nt] && hc) {
          E.merge(nt, tt);
          L.written[n] = 1;
        } else {
          L.written[n] = L.written[nt];  // the terminal holds no entry
        }
        --top;
        continue;
      }
      // both operands are subtrees: the one needing more slots goes first
      const bool b_first = L.need[b] > L.need[a];
      const int first = b_first ? b : a, second = b_first ? a : b;
      if (st == 0) {
        L.stt[top] = 1;
        ++top;
        L.stk[top] = int16_t(first);
        L.stt[top] = 0;
        continue;
      }
      if (st == 1) {
        L.stt[top] = 2;
        E.push_pending = true;
        E.push_node = first;
        E.push_slot = uint32_t(dsp);
        ++dsp;
        if (dsp > maxsp) maxsp = dsp;
        if (dsp > Dmax) bad = true;
        ++top;
        L.stk[top] = int16_t(second);
        L.stt[top] = 0;
        continue;
      }
      --dsp;
      // acc = second, S[dsp] = first.  first == a: a op b = S op acc (reversed)
      E.emit(make_hdr(bin_uop(s, !b_first), SRC_POP, uint32_t(dsp), LD_NONE, 0) |
                 (L.hasc[second] ? HDR_ADJ_ACC : 0) | (L.hasc[first] ? HDR_ADJ_SRC : 0),
             0);
      if (L.hasc[second] && L.hasc[first]) {
        E.merge(second, first);
        L.written[n] = 1;
      } else {
        L.written[n] = L.written[second] | L.written[first];
      }
      --top;
    }
  }
  bad = bad || E.bad;
  if (bad) {
    out[0] = make_uint2(UOP_END_HDR, 0);
    out[1] = make_uint2(UOP_END_HDR, 0);
    pm.status = 2;
    pm.n_uops = 1;
  } else {
    out[E.n] = make_uint2(UOP_END_HDR, 0);
    out[E.n + 1] = make_uint2(UOP_END_HDR, 0);
    pm.n_uops = E.n + 1;
    pm.slots = maxsp;
    pm.n_tape = E.tape;
    pm.n_const = nc;
    pm.cost = E.cost;
    pm.n_merge = E.n_event;
  }
  pm.mu = 0.0f;
  meta[i] = pm;
}

hipError_t launch_compile(const int8_t* ops, int M, int L_max, const float* consts, int C_max,
                          int F, int Dmax, int U_stride, uint2* uops, ProgMeta* meta,
                          uint2* events, int ET, hipStream_t s) {
  const int nb = (M + 3) / 4;
  hipLaunchKernelGGL(k_compile, dim3(nb), dim3(256), 0, s, ops, M, L_max, consts, C_max, F, Dmax,
                     U_stride, uops, meta, events, ET);
  return hipGetLastError();
}

// -------------------------------------------------------------------- probe
// One wave per individual; the block stages the first 64*K rows of X in LDS.
// The program is read into registers 64 uops at a time (coalesced loads), so
// the uop stream costs no memory round trip per uop.  Eight stack slots: the
// probe evaluates every program, whatever its depth.
template <typename T, int K, int D, bool ROLL>
__global__ __launch_bounds__(256) void k_probe(const uint2* __restrict__ uops, int U_stride,
                                               ProgMeta* __restrict__ meta, int M,
                                               const float* __restrict__ X, int64_t ldx, int F,
                                               int64_t N) {
  extern __shared__ float xs[];  // F * 64*K
  constexpr int R = 64 * K;
  const int nval = int(N < R ? N : R);
  for (int idx = threadIdx.x; idx < F * R; idx += blockDim.x) {
    const int f = idx / R, r = idx - f * R;
    xs[idx] = r < nval ? X[size_t(f) * ldx + r] : 0.0f;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
  if (i >= M) return;
  if (meta[i].status != 0) return;
  const uint2* prow = uops + size_t(i) * U_stride;
  uint32_t lo, hi;
  load_window(prow, 0, U_stride, make_uint2(UOP_END_HDR, 0u), lo, hi);
  UopWin<ROLL> prog;
  prog.begin(prow, U_stride, lo, hi);
  const auto p = run_program<T, K, D>(prog, xs, R, lane_row<K>(lane));
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool v = lane_row<K>(lane) + row_off<K>(j) < nval;
    s += v ? float(p[j]) : 0.0f;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const float mu = s / float(nval);
  if (lane == 0) meta[i].mu = isfinite(mu) ? mu : 0.0f;
}

template <typename T, int K, int D, bool ROLL>
static hipError_t probe_impl(const uint2* uops, int U_stride, ProgMeta* meta, int M,
                             const DataArgs& d, hipStream_t s) {
  const size_t sh = size_t(d.F) * 64 * K * sizeof(float);
  hipLaunchKernelGGL((k_probe<T, K, D, ROLL>), dim3((M + 3) / 4), dim3(256), sh, s, uops, U_stride,
                     meta, M, d.X, d.ldx, d.F, d.N);
  return hipGetLastError();
}

hipError_t launch_probe(bool fp64, const uint2* uops, int U_stride, ProgMeta* meta, int M,
                        const DataArgs& d, hipStream_t s) {
  const bool roll = U_stride > 64;  // programs of more than 64 uops possible
  if (fp64) return roll ? probe_impl<double, 4, 8, true>(uops, U_stride, meta, M, d, s)
                        : probe_impl<double, 4, 8, false>(uops, U_stride, meta, M, d, s);
  return roll ? probe_impl<float, 4, 8, true>(uops, U_stride, meta, M, d, s)
              : probe_impl<float, 4, 8, false>(uops, U_stride, meta, M, d, s);
}

int lds_limit_bytes() {
  static int v = [] {
    int dev = 0, val = 65536;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    return val;
  }();
  return v;
}

}  // namespace gg

namespace gg {

__global__ void k_fill_u32(unsigned* __restrict__ p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace gg

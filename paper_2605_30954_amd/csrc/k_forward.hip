// Forward fitness kernels.
//
// Both forms accumulate, per individual and in binary64, the additive
// moments of its predictions p over the rows:
//   A = sum (p - mu),  B = sum (p - mu)^2,  C = sum (p - mu) * (y - ybar),
//   E = sum (p - y)^2                                  (raw squared error)
// with mu a per-individual shift (mean prediction on the first rows) that keeps
// B - A^2/N free of cancellation.  Every one of them is a sum over rows, so the
// rows can be split over lanes, waves and blocks (the data parallelism of
// Section 3.2 needs an additive loss; the linear-scaling fit only needs these
// additive moments).  The finalize turns them into the least-squares fit and
// the MSE / LS-MSE / NMSE of Eq. 1-2.
//
// Fused form: a block stages a tile of rows (feature-major X and y - ybar) in
// LDS once and every wave of the block evaluates the group's individuals on
// it (wave w takes individuals w, w+W, ...); a block sweeps `tiles_per_span`
// tiles before it writes the group's partial sums.
// Plain form: one launch per individual over all rows; its last block to
// finish sums the per-block partials and finalizes (the per-individual launch
// pattern the paper contrasts with its batched design).
#include <hip/hip_runtime.h>

#include "gpgomea_eval.h"
#include "interp.h"
#include "kernels.h"

namespace gg {

struct FwdParams {
  const uint2* uops;
  int U_stride;
  const ProgMeta* meta;
  int M;
  const float* X;
  int64_t ldx;
  int F;
  int64_t N;
  const float* y;
  const double* stats;
  double* part;
  int R, G, n_groups, n_spans, tiles_per_span;
};

template <bool SSE>
struct Moments {
  double a = 0.0, b = 0.0, c = 0.0, e = 0.0;
  __device__ inline void add(double d, double yt, double emu) {
    a += d;
    b = fma(d, d, b);
    c = fma(d, yt, c);
    if (SSE) {
      const double r = (d + emu) - yt;  // p - y = (p - mu) + (mu - ybar) - (y - ybar)
      e = fma(r, r, e);
    }
  }
};

// Accumulate K predictions of this lane into the moments.
template <typename T, int K, bool SSE>
__device__ inline void accumulate(Moments<SSE>& m, const typename VecT<T, K>::type& p,
                                  const double* __restrict__ yt, int lrow, int nvalid, double mu,
                                  double emu) {
  if (lrow + row_off<K>(K - 1) < nvalid) {
#pragma unroll
    for (int j = 0; j < K; ++j) m.add(double(p[j]) - mu, yt[lrow + row_off<K>(j)], emu);
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const bool v = lrow + row_off<K>(j) < nvalid;
      const double d = double(p[j]) - mu;
      m.add(v ? d : 0.0, v ? yt[lrow + row_off<K>(j)] : 0.0, v ? emu : 0.0);
    }
  }
}

// Copy rows [r0, r0+nvalid) of every feature into the LDS tile (zero beyond).
__device__ inline void stage_tile(float* __restrict__ xs, const float* __restrict__ X, int64_t ldx,
                                  int F, int R, int64_t r0, int nvalid) {
  for (int f = 0; f < F; ++f) {
    const float* __restrict__ src = X + size_t(f) * ldx + r0;
    float* __restrict__ dst = xs + size_t(f) * R;
    for (int r = threadIdx.x; r < R; r += blockDim.x) dst[r] = r < nvalid ? src[r] : 0.0f;
  }
}

// XCD-aware work mapping: the hardware hands consecutive blocks to the 8
// XCDs in turn; give each XCD a contiguous run of work items so the items
// that share a row span also share an L2.
__device__ inline int xcd_item(int b, int total) {
  const int x = b & 7, k = b >> 3;
  const int q = total >> 3, r = total & 7;
  return x * q + (x < r ? x : r) + k;
}

// Stack depth passes.  Most programs need at most 4 register stack slots
// (a program needing s slots has at least 2^(s+1) leaves, so 5 or more occur
// only from 127 tokens on).  A batch that may hold deeper programs runs two
// launches: pass 1 with 4 slots skips the deep programs, pass 2 with 8 slots
// evaluates only them (a block whose group has none exits before staging).
enum : int { PASS_ALL = 0, PASS_SHALLOW = 1, PASS_DEEP = 2 };
constexpr int kShallowSlots = 4;

__device__ inline bool in_pass(int pass, int slots) {
  return pass == PASS_ALL || (pass == PASS_SHALLOW ? slots <= kShallowSlots : slots > kShallowSlots);
}

// The binary32 forward at eight rows per lane is compiled for five waves per
// SIMD (at most 96 VGPRs; part of the register stack then lives in scratch
// memory, touched only by programs that need those slots): with a row tile of
// at most 32 KB of LDS, five blocks of four waves share a CU.  Measured on
// MI355X at full size on the large-template workload: 608, 539, 514 and
// 557 ms at three, four, five and six waves per SIMD; five waves were also
// 2-6% faster than four on the other workloads.
template <typename T, int K>
constexpr int fwd_min_waves() {
  return (sizeof(T) == 4 && K == 8) ? 5 : 1;
}
template <typename T, int K, int D, int W, bool SSE, bool ROLL, int PASS>
__global__ __launch_bounds__(W * 64, (fwd_min_waves<T, K>())) void k_fused_fwd(FwdParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  double* accs = yts + R;  // G * 4

  const int total = p.n_spans * p.n_groups;
  const int item = xcd_item(blockIdx.x, total);
  const int span = item / p.n_groups, grp = item - span * p.n_groups;
  const int ind0 = grp * p.G;
  const int Gn = min(p.G, p.M - ind0);
  const int lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  constexpr int BR = 64 * K;

  if constexpr (PASS == PASS_DEEP) {  // block-uniform: nothing of this pass in the group
    bool any = false;
    for (int j = 0; j < Gn; ++j) any = any || p.meta[ind0 + j].slots > kShallowSlots;
    if (!any) return;
  }
  __shared__ int queue;
  // status (0 evaluate, else skip) and mu of the group's individuals
  // (G <= kFwdMaxG), read with the queue claim: one LDS round trip per
  // individual, no global load
  __shared__ uint2 gmeta[kFwdMaxG];
  for (int j = threadIdx.x; j < Gn * 4; j += blockDim.x) accs[j] = 0.0;
  for (int j = threadIdx.x; j < Gn; j += blockDim.x) {
    const ProgMeta& m = p.meta[ind0 + j];
    const bool run = m.status == 0 && in_pass(PASS, m.slots);
    gmeta[j] = make_uint2(run ? 0u : 1u, __float_as_uint(m.mu));
  }

  const int64_t span_r0 = int64_t(span) * p.tiles_per_span * R;
  for (int tile = 0; tile < p.tiles_per_span; ++tile) {
    const int64_t r0 = span_r0 + int64_t(tile) * R;
    if (r0 >= p.N) break;
    const int nvalid = int(min<int64_t>(R, p.N - r0));
    __syncthreads();  // previous tile fully consumed
    if (threadIdx.x == 0) queue = 0;
    stage_x_async<W>(xs, p.X, p.ldx, p.F, R, r0, p.N);
    stage_y(yts, p.y, R, r0, nvalid, ybar);
    __builtin_amdgcn_s_waitcnt(0);  // the tile's direct loads have landed
    __syncthreads();
    const int nbatch = (nvalid + BR - 1) / BR;
    // the waves claim the group's individuals from the tile's queue (a
    // wave-uniform loop, no cross-lane traffic under divergent control); the
    // next individual is claimed and its first program window loaded while
    // this one runs
    uint32_t w0lo = 0, w0hi = 0, w1lo = 0, w1hi = 0;
    const uint2 endu = make_uint2(UOP_END_HDR, 0u);
    int jj = claim_next(&queue);
    if (jj < Gn) load_window(p.uops + size_t(ind0 + jj) * p.U_stride, 0, p.U_stride, endu, w0lo, w0hi);
    while (jj < Gn) {
      const uint2 gm = gmeta[jj];
      const int jn = claim_next(&queue);
      const int skip = __builtin_amdgcn_readfirstlane(int(gm.x));
      const float mu_f = __uint_as_float(__builtin_amdgcn_readfirstlane(int(gm.y)));
      if (jn < Gn) load_window(p.uops + size_t(ind0 + jn) * p.U_stride, 0, p.U_stride, endu, w1lo, w1hi);
      if (skip == 0) {
        const double mu = double(mu_f);
        const double emu = mu - ybar;
        const uint2* prow = p.uops + size_t(ind0 + jj) * p.U_stride;
        Moments<SSE> m;
        for (int b = 0; b < nbatch; ++b) {
          const int lrow = b * BR + lane_row<K>(lane);
          UopWin<ROLL> prog;
          prog.begin(prow, p.U_stride, w0lo, w0hi);
          const auto v = run_program<T, K, D>(prog, xs, R, lrow);
          accumulate<T, K, SSE>(m, v, yts, lrow, nvalid, mu, emu);
        }
        const double sa = wave_sum(m.a), sb = wave_sum(m.b), sc = wave_sum(m.c);
        const double se = SSE ? wave_sum(m.e) : 0.0;
        // every lane holds the same totals: all lanes store the same value (no
        // divergent branch between the cross-lane sums of consecutive individuals)
        accs[jj * 4 + 0] += sa;
        accs[jj * 4 + 1] += sb;
        accs[jj * 4 + 2] += sc;
        accs[jj * 4 + 3] += se;
      }
      w0lo = w1lo;
      w0hi = w1hi;
      jj = jn;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < Gn * 4; j += blockDim.x) {
    const int jj = j >> 2, q = j & 3;
    if (gmeta[jj].x == 0u || PASS == PASS_ALL)
      p.part[(size_t(ind0 + jj) * p.n_spans + span) * 4 + q] = accs[j];
  }
}

template <typename T, int K, int D, int W, bool ROLL, int PASS>
static hipError_t fused_impl(const TileCfg& c, const FwdParams& fp, bool sse, hipStream_t s) {
  const size_t sh = forward_lds_bytes(fp.F, fp.R, fp.G);
  const int nb = c.n_spans * c.n_groups;
  if (sse)
    hipLaunchKernelGGL((k_fused_fwd<T, K, D, W, true, ROLL, PASS>), dim3(nb), dim3(W * 64), sh, s, fp);
  else
    hipLaunchKernelGGL((k_fused_fwd<T, K, D, W, false, ROLL, PASS>), dim3(nb), dim3(W * 64), sh, s, fp);
  return hipGetLastError();
}

// Programs of up to 63 tokens (at most 64 uops with END) are held in one
// window; longer ones roll.  A batch that may hold programs needing more than
// four stack slots (127 tokens or more) runs the shallow and the deep pass.
template <typename T, int K>
static hipError_t fused_k(const TileCfg& c, const FwdParams& fp, bool sse, bool roll, bool deep_possible,
                          hipStream_t s) {
  hipError_t e;
  if (!roll) return fused_impl<T, K, kShallowSlots, 4, false, PASS_ALL>(c, fp, sse, s);
  if (!deep_possible) return fused_impl<T, K, kShallowSlots, 4, true, PASS_ALL>(c, fp, sse, s);
  e = fused_impl<T, K, kShallowSlots, 4, true, PASS_SHALLOW>(c, fp, sse, s);
  if (e != hipSuccess) return e;
  return fused_impl<T, K, 8, 4, true, PASS_DEEP>(c, fp, sse, s);
}

hipError_t launch_fused_forward(bool fp64, const TileCfg& c, const uint2* uops, int U_stride,
                                const ProgMeta* meta, int M, const DataArgs& d,
                                const double* stats, double* part, bool want_sse, hipStream_t s) {
  FwdParams fp{uops, U_stride, meta, M, d.X, d.ldx, d.F, d.N, d.y, stats, part,
               c.R, c.G, c.n_groups, c.n_spans, c.tiles_per_span};
  const bool roll = U_stride > 64;               // L_max + 1 > 64 uops possible
  const bool deep = U_stride - 2 >= 127;         // L_max >= 127: 5+ slots possible
  if (fp64) return fused_k<double, 4>(c, fp, want_sse, roll, deep, s);
  if (c.K == 4) return fused_k<float, 4>(c, fp, want_sse, roll, deep, s);
  if (c.K == 8) return fused_k<float, 8>(c, fp, want_sse, roll, deep, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ finalize
// Fit and fitness of one individual from its summed moments (binary64):
//   pbar = mu + A/N,  Spp = B - A^2/N,  Spy = C - (A/N) * sum(y - ybar)
//   degenerate if Spp/N <= 1e-12 * max(pbar^2, 1e-300): b = 0, a = mean(y)
//   else b = Spy/Spp, a = mean(y) - b*pbar, LS-MSE = max(Var(y) - Spy^2/(N Spp), 0)
//   MSE = E/N (Eq. 1), NMSE = fitness / Var(y) (Eq. 2)
__device__ inline void finalize_one(double A, double B, double C, double E, double mu,
                                    const double* __restrict__ st, uint32_t flags, int pstatus,
                                    double* fit, double* aux4, int8_t* status, double* ab2) {
  const double N = st[ST_N], ybar = st[ST_YBAR], vy = st[ST_VY], ytsum = st[ST_YT];
  const double ymean = ybar + ytsum / N;
  int sts = pstatus != 0 ? 2 : 0;
  if (sts == 0 && !(isfinite(A) && isfinite(B) && isfinite(C))) sts = 1;
  double f, a, b, mse, nmse;
  if (sts != 0) {
    f = mse = nmse = INFINITY;
    a = ymean;
    b = 0.0;
  } else {
    const double pbar = mu + A / N;
    double spp = B - A * (A / N);
    if (spp < 0.0) spp = 0.0;
    const double spy = C - (A / N) * ytsum;
    mse = E / N;
    double ls;
    if (spp / N <= 1e-12 * fmax(pbar * pbar, 1e-300)) {
      b = 0.0;
      a = ymean;
      ls = vy;
    } else {
      b = spy / spp;
      a = ymean - b * pbar;
      ls = vy - spy * (spy / spp) / N;
      if (ls < 0.0) ls = 0.0;
    }
    f = (flags & GPGOMEA_LINEAR_SCALING) ? ls : mse;
    nmse = vy > 0.0 ? f / vy : (f == 0.0 ? 0.0 : INFINITY);
  }
  *fit = f;
  if (status) *status = int8_t(sts);
  if (aux4) {
    aux4[0] = a;
    aux4[1] = b;
    aux4[2] = mse;
    aux4[3] = nmse;
  }
  if (ab2) {  // seed of the adjoint: residual ab2[S0] + ab2[S1] p - y, scaled
    const bool ls = (flags & GPGOMEA_LINEAR_SCALING) != 0;
    ab2[AB_S0] = ls ? a : 0.0;
    ab2[AB_S1] = sts != 0 ? 0.0 : (ls ? b : 1.0);
    // 2^e with e the exponent of the RMS residual sqrt(f) (1 when f is 0 or
    // not finite): the residuals divided by it are O(1) on average
    int e = 0;
    if (sts == 0 && f > 0.0 && isfinite(f)) (void)frexp(sqrt(f), &e);
    ab2[AB_INV_SCALE] = ldexp(1.0, -e);
    ab2[AB_SCALE] = ldexp(1.0, e);
  }
}

// One wave per individual: lane l sums spans l, l+64, ... in order, then a
// fixed xor-tree over the wave (bitwise repeatable for a given span count).
__global__ __launch_bounds__(256) void k_finalize(const ProgMeta* __restrict__ meta, int M,
                                                  const double* __restrict__ part, int n_spans,
                                                  const double* __restrict__ stats, uint32_t flags,
                                                  double* __restrict__ fitness,
                                                  double* __restrict__ aux,
                                                  int8_t* __restrict__ status,
                                                  double* __restrict__ ab) {
  const int i = __builtin_amdgcn_readfirstlane(int(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (i >= M) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const ProgMeta pm = meta[i];
  double A = 0, B = 0, C = 0, E = 0;
  if (pm.status == 0) {
    const double* q = part + size_t(i) * n_spans * 4;
    for (int s = lane; s < n_spans; s += 64) {
      A += q[4 * s + 0];
      B += q[4 * s + 1];
      C += q[4 * s + 2];
      E += q[4 * s + 3];
    }
  }
  A = wave_sum(A);
  B = wave_sum(B);
  C = wave_sum(C);
  E = wave_sum(E);
  if (lane == 0)
    finalize_one(A, B, C, E, double(pm.mu), stats, flags, pm.status, fitness + i,
                 aux ? aux + size_t(i) * 4 : nullptr, status ? status + i : nullptr,
                 ab ? ab + size_t(i) * AB_WORDS : nullptr);
}

hipError_t launch_finalize(const ProgMeta* meta, int M, const double* part, int n_spans,
                           const double* stats, uint32_t flags, double* fitness, double* aux,
                           int8_t* status, double* ab, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((M + 3) / 4), dim3(256), 0, s, meta, M, part, n_spans,
                     stats, flags, fitness, aux, status, ab);
  return hipGetLastError();
}

// -------------------------------------------------------------------- plain
struct PlainParams {
  const uint2* prog;
  const ProgMeta* meta;  // this individual's
  const float* X;
  int64_t ldx;
  int F;
  int64_t N;
  const float* y;
  const double* stats;
  double* part;  // [gridDim.x][4]
  unsigned* ticket;
  uint32_t flags;
  double* fitness;
  double* aux;
  int8_t* status;
  double* ab;
  int R;
};

template <typename T, int K, int D, int W, bool SSE>
__global__ __launch_bounds__(W * 64) void k_plain_fwd(PlainParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = p.R;
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* yts = reinterpret_cast<double*>(smem_raw + size_t(p.F) * R * sizeof(float));
  __shared__ double red[W][4];
  __shared__ bool is_last;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double ybar = p.stats[ST_YBAR];
  const ProgMeta pm = *p.meta;
  const double mu = double(pm.mu), emu = mu - ybar;
  constexpr int BR = 64 * K;
  Moments<SSE> m;
  if (pm.status == 0) {
    for (int64_t r0 = int64_t(blockIdx.x) * R; r0 < p.N; r0 += int64_t(gridDim.x) * R) {
      const int nvalid = int(min<int64_t>(R, p.N - r0));
      __syncthreads();
      stage_tile(xs, p.X, p.ldx, p.F, R, r0, nvalid);
      for (int r = threadIdx.x; r < R; r += blockDim.x)
        yts[r] = r < nvalid ? double(p.y[r0 + r]) - ybar : 0.0;
      __syncthreads();
      const int nbatch = (nvalid + BR - 1) / BR;
      for (int b = w; b < nbatch; b += W) {
        const int lrow = b * BR + lane_row<K>(lane);
        UopMem prog{p.prog};
        const auto v = run_program<T, K, D>(prog, xs, R, lrow);
        accumulate<T, K, SSE>(m, v, yts, lrow, nvalid, mu, emu);
      }
    }
  }
  const double sa = wave_sum(m.a), sb = wave_sum(m.b), sc = wave_sum(m.c);
  const double se = SSE ? wave_sum(m.e) : 0.0;
  if (lane == 0) {
    red[w][0] = sa;
    red[w][1] = sb;
    red[w][2] = sc;
    red[w][3] = se;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double q[4] = {0, 0, 0, 0};
    for (int k = 0; k < W; ++k)
      for (int t = 0; t < 4; ++t) q[t] += red[k][t];
    for (int t = 0; t < 4; ++t) p.part[size_t(blockIdx.x) * 4 + t] = q[t];
    __threadfence();
    const unsigned done = atomicAdd(p.ticket, 1u);
    is_last = (done == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    double A = 0, B = 0, C = 0, E = 0;
    const volatile double* q = p.part;
    for (unsigned b = 0; b < gridDim.x; ++b) {
      A += q[4 * b + 0];
      B += q[4 * b + 1];
      C += q[4 * b + 2];
      E += q[4 * b + 3];
    }
    finalize_one(A, B, C, E, mu, p.stats, p.flags, pm.status, p.fitness, p.aux, p.status, p.ab);
    *p.ticket = 0u;  // ready for the next launch on this stream
  }
}

int plain_blocks(const TileCfg& c, int64_t N) {
  const int64_t t = (N + c.R - 1) / c.R;
  return int(t < 1024 ? t : 1024);
}

template <typename T, int K, int D, int W>
static hipError_t plain_impl(const TileCfg& c, const PlainParams& pp, bool sse, hipStream_t s) {
  const size_t sh = size_t(pp.F) * pp.R * sizeof(float) + size_t(pp.R) * sizeof(double);
  const int nb = plain_blocks(c, pp.N);
  if (sse)
    hipLaunchKernelGGL((k_plain_fwd<T, K, D, W, true>), dim3(nb), dim3(W * 64), sh, s, pp);
  else
    hipLaunchKernelGGL((k_plain_fwd<T, K, D, W, false>), dim3(nb), dim3(W * 64), sh, s, pp);
  return hipGetLastError();
}

hipError_t launch_plain_forward(bool fp64, const TileCfg& c, int i, const uint2* uops,
                                int U_stride, const ProgMeta* meta, const DataArgs& d,
                                const double* stats, double* part, unsigned* ticket,
                                uint32_t flags, double* fitness, double* aux, int8_t* status,
                                double* ab, hipStream_t s) {
  PlainParams pp{uops + size_t(i) * U_stride,
                 meta + i,
                 d.X,
                 d.ldx,
                 d.F,
                 d.N,
                 d.y,
                 stats,
                 part,
                 ticket,
                 flags,
                 fitness + i,
                 aux ? aux + size_t(i) * 4 : nullptr,
                 status ? status + i : nullptr,
                 ab ? ab + size_t(i) * AB_WORDS : nullptr,
                 c.R};
  const bool sse = aux != nullptr || !(flags & GPGOMEA_LINEAR_SCALING);
  if (fp64) return plain_impl<double, 4, 8, 4>(c, pp, sse, s);
  if (c.K == 4) {
    if (c.D <= 4) return plain_impl<float, 4, 4, 4>(c, pp, sse, s);
    return plain_impl<float, 4, 8, 4>(c, pp, sse, s);
  }
  if (c.D <= 4) return plain_impl<float, 8, 4, 4>(c, pp, sse, s);
  return plain_impl<float, 8, 8, 4>(c, pp, sse, s);
}

}  // namespace gg

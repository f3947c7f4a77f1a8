// The paper's two GPU evaluation designs (Section 3.2, "Evaluation on the
// GPU", and Fig. 2), kept as comparators of the fused batch path:
//
//   design 1: one workgroup per program.  The program's tokens and constants
//             are staged in LDS; thread t interprets the program for rows t,
//             t + B, t + 2B, ... with an operand stack in private memory,
//             accumulating its squared errors in a register; a tree reduction
//             in LDS gives the program's sum, and the MSE is written out.
//   design 2: several workgroups per program, each over one contiguous block
//             of rows, writing its partial sum to global memory; a second
//             kernel adds a program's partial sums.
//
// Both compute the raw MSE of Eq. 1, as the paper's designs do (linear
// scaling is not part of them).  They read the library's postfix programs
// (one byte per token; the paper's two arrays of node type and node value hold
// the same information).  The paper does not state the precision of the
// reduction: squared errors are accumulated in binary64 here, so that the
// comparators meet the same 1e-5 bar as the fused path at 1e7 rows.
// The operators are the library's protected ones (devmath.h).
#include <hip/hip_runtime.h>

#include "devmath.h"
#include "gpgomea_ops.h"
#include "kernels.h"

namespace gg {
namespace {

constexpr int kDesignStack = 16;  // operand stack entries per thread

// Run one program on row r.  err: 0 ok, 2 bad program (unknown token,
// variable >= F, more constants than C, stack under/overflow, not exactly
// one result).  The error is the same for every row, so it is uniform.
__device__ inline float rpn_eval(const int8_t* tok, const float* cval, int L, int C, int F,
                                 const float* __restrict__ X, int64_t ldx, int64_t r, int& err) {
  using P = Prot<float>;
  float st[kDesignStack];
  int sp = 0, ci = 0;
  for (int k = 0; k < L; ++k) {
    const int t = tok[k];
    if (t == GPGOMEA_SYM_END) break;
    if (t >= GPGOMEA_SYM_VAR0) {
      const int v = t - GPGOMEA_SYM_VAR0;
      if (v >= F || sp >= kDesignStack) {
        err = 2;
        return 0.0f;
      }
      st[sp++] = X[int64_t(v) * ldx + r];
    } else if (t == GPGOMEA_SYM_CONST) {
      if (ci >= C || sp >= kDesignStack) {
        err = 2;
        return 0.0f;
      }
      st[sp++] = cval[ci++];
    } else if (t >= 0 && t < GPGOMEA_NUM_OPS) {
      const bool unary = t == GPGOMEA_SYM_SIN || t == GPGOMEA_SYM_COS || t == GPGOMEA_SYM_SQ ||
                         t == GPGOMEA_SYM_SQRT || t == GPGOMEA_SYM_EXP || t == GPGOMEA_SYM_LOG;
      if (sp < (unary ? 1 : 2)) {
        err = 2;
        return 0.0f;
      }
      const float a = unary ? st[sp - 1] : st[sp - 2];
      const float b = st[sp - 1];
      float v;
      switch (t) {
        case GPGOMEA_SYM_ADD: v = a + b; break;
        case GPGOMEA_SYM_SUB: v = a - b; break;
        case GPGOMEA_SYM_MUL: v = a * b; break;
        case GPGOMEA_SYM_DIV: v = P::div(a, b); break;
        case GPGOMEA_SYM_SIN: v = P::sin_(a); break;
        case GPGOMEA_SYM_COS: v = P::cos_(a); break;
        case GPGOMEA_SYM_SQ: v = a * a; break;
        case GPGOMEA_SYM_SQRT: v = P::sqrt_(a); break;
        case GPGOMEA_SYM_EXP: v = P::exp_(a); break;
        case GPGOMEA_SYM_LOG: v = P::log_(a); break;
        default: v = P::pow_(a, b); break;
      }
      if (!unary) --sp;
      st[sp - 1] = v;
    } else {
      err = 2;
      return 0.0f;
    }
  }
  if (sp != 1) err = 2;
  return st[0];
}

// Stage program i in LDS: tokens (L bytes, padded to 4) then constants.
__device__ inline void stage_program(const int8_t* __restrict__ ops, const float* __restrict__ consts,
                                     int i, int L, int C, int8_t* tok, float* cval) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) tok[k] = ops[int64_t(i) * L + k];
  for (int k = threadIdx.x; k < C; k += blockDim.x) cval[k] = consts[int64_t(i) * C + k];
  __syncthreads();
}

// Block-wide sum of one double per thread (LDS tree); every thread gets it.
__device__ inline double block_tree_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Rows [r0, r1) of program i with thread stride: squared errors (binary64),
// and whether a prediction was not finite.
__device__ inline double rows_sse(const int8_t* tok, const float* cval, int L, int C, int F,
                                  const float* __restrict__ X, int64_t ldx, const float* __restrict__ y,
                                  int64_t r0, int64_t r1, int& err, int& nonfinite) {
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const float p = rpn_eval(tok, cval, L, C, F, X, ldx, r, err);
    if (err) break;
    if (!isfinite(p)) nonfinite = 1;
    const double d = double(p) - double(y[r]);
    acc += d * d;
  }
  return acc;
}

__global__ __launch_bounds__(1024) void k_design1(const int8_t* __restrict__ ops, int L,
                                                  const float* __restrict__ consts, int C, int F,
                                                  const float* __restrict__ X, int64_t ldx, int64_t N,
                                                  const float* __restrict__ y, double* __restrict__ fitness,
                                                  int8_t* __restrict__ status) {
  extern __shared__ double lds_d[];
  double* red = lds_d;                                       // blockDim doubles
  float* cval = reinterpret_cast<float*>(red + blockDim.x);  // C floats
  int8_t* tok = reinterpret_cast<int8_t*>(cval + C);         // L bytes
  const int i = blockIdx.x;
  stage_program(ops, consts, i, L, C, tok, cval);
  int err = 0, nonfinite = 0;
  const double part = rows_sse(tok, cval, L, C, F, X, ldx, y, 0, N, err, nonfinite);
  const int any_err = __syncthreads_or(err);
  const int any_nf = __syncthreads_or(nonfinite);
  const double sse = block_tree_sum(part, red);
  if (threadIdx.x == 0) {
    const int st = any_err ? 2 : (any_nf || !isfinite(sse)) ? 1 : 0;
    fitness[i] = st ? __builtin_inf() : sse / double(N);
    if (status) status[i] = int8_t(st);
  }
}

__global__ __launch_bounds__(1024) void k_design2_part(const int8_t* __restrict__ ops, int L,
                                                       const float* __restrict__ consts, int C, int F,
                                                       const float* __restrict__ X, int64_t ldx, int64_t N,
                                                       const float* __restrict__ y, int nb,
                                                       double* __restrict__ part) {
  extern __shared__ double lds_d[];
  double* red = lds_d;
  float* cval = reinterpret_cast<float*>(red + blockDim.x);
  int8_t* tok = reinterpret_cast<int8_t*>(cval + C);
  const int i = int(blockIdx.x / unsigned(nb)), b = int(blockIdx.x % unsigned(nb));
  stage_program(ops, consts, i, L, C, tok, cval);
  const int64_t chunk = (N + nb - 1) / nb;
  const int64_t r0 = int64_t(b) * chunk;
  const int64_t r1 = r0 + chunk < N ? r0 + chunk : N;
  int err = 0, nonfinite = 0;
  const double p = rows_sse(tok, cval, L, C, F, X, ldx, y, r0, r1, err, nonfinite);
  const int any_err = __syncthreads_or(err);
  const int any_nf = __syncthreads_or(nonfinite);
  const double s = block_tree_sum(p, red);
  // a block's flags travel in its partial: NaN = bad program, +inf = a
  // prediction that was not finite
  if (threadIdx.x == 0)
    part[int64_t(i) * nb + b] = any_err ? __builtin_nan("") : any_nf ? __builtin_inf() : s;
}

// One wave per program: add its nb partial sums.
__global__ __launch_bounds__(256) void k_design2_reduce(const double* __restrict__ part, int M, int nb,
                                                        int64_t N, double* __restrict__ fitness,
                                                        int8_t* __restrict__ status) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= M) return;
  double s = 0.0;
  int bad = 0, nf = 0;
  for (int b = lane; b < nb; b += 64) {
    const double v = part[int64_t(i) * nb + b];
    bad |= isnan(v);
    nf |= isinf(v);
    s += v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    bad |= __shfl_xor(bad, off, 64);
    nf |= __shfl_xor(nf, off, 64);
  }
  if (lane == 0) {
    const int st = bad ? 2 : (nf || !isfinite(s)) ? 1 : 0;
    fitness[i] = st ? __builtin_inf() : s / double(N);
    if (status) status[i] = int8_t(st);
  }
}

size_t design_lds_bytes(int L, int C, int block) {
  return size_t(block) * 8 + size_t(C) * 4 + ((size_t(L) + 3) & ~size_t(3));
}

}  // namespace

hipError_t launch_design1(const DesignArgs& a, hipStream_t s) {
  if (a.M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_design1, dim3(unsigned(a.M)), dim3(unsigned(a.block)),
                     design_lds_bytes(a.L, a.C, a.block), s, a.ops, a.L, a.consts, a.C, a.F, a.X, a.ldx,
                     a.N, a.y, a.fitness, a.status);
  return hipGetLastError();
}

hipError_t launch_design2(const DesignArgs& a, int nb, double* part, hipStream_t s) {
  if (a.M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_design2_part, dim3(unsigned(int64_t(nb) * a.M)), dim3(unsigned(a.block)),
                     design_lds_bytes(a.L, a.C, a.block), s, a.ops, a.L, a.consts, a.C, a.F, a.X, a.ldx,
                     a.N, a.y, nb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_design2_reduce, dim3(unsigned((a.M + 3) / 4)), dim3(256), 0, s, part, a.M, nb, a.N,
                     a.fitness, a.status);
  return hipGetLastError();
}

}  // namespace gg

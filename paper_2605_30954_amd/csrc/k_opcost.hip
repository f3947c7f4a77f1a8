// Operator cost microbenchmark.
//
// The interpreter's work per row is a sequence of protected operators; the
// time the vector ALU alone would need for them is the reference the
// interpreter's efficiency is measured against.  Each kernel below applies
// one operator (the same device routine the interpreter calls) `iters` times
// to 8 independent values per lane, with enough waves to fill every SIMD, so
// its duration is pure ALU throughput of that routine:
//     c(op) = duration * peak_lane_op_rate / (lanes * iters * 8)
// in "lane-ops" (1 = one non-packed VALU instruction per lane).
#include <hip/hip_runtime.h>

#include "interp.h"
#include "kernels.h"

namespace gg {

constexpr int kCostLanes = 8;

template <int OP>
__device__ inline float cost_apply(float a, float b) {
  using P = Prot<float>;
  if constexpr (OP == UOP_ADD) return a + b;
  if constexpr (OP == UOP_SUB) return a - b;
  if constexpr (OP == UOP_MUL) return a * b;
  if constexpr (OP == UOP_DIV) return P::div(a, b);
  if constexpr (OP == UOP_POW) return P::pow_(a, b);
  if constexpr (OP == UOP_SIN) return P::sin_(a);
  if constexpr (OP == UOP_COS) return P::cos_(a);
  if constexpr (OP == UOP_SQ) return a * a;
  if constexpr (OP == UOP_SQRT) return P::sqrt_(a);
  if constexpr (OP == UOP_EXP) return P::exp_(a);
  if constexpr (OP == UOP_LOG) return P::log_(a);
  return a;
}

// Keeps values in a range where no operator takes a rare slow path, without
// letting the compiler fold the chain: v <- op(v, b) * s + t mixes back.
template <int OP>
__global__ __launch_bounds__(256) void k_opcost(float* __restrict__ out, int iters, float seed) {
  float v[kCostLanes];
  const float b = 1.0009765625f + 1e-7f * float(threadIdx.x & 7);
#pragma unroll
  for (int j = 0; j < kCostLanes; ++j) v[j] = 1.25f + 0.01f * float(j) + seed * float(threadIdx.x & 15);
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kCostLanes; ++j) v[j] = cost_apply<OP>(v[j], b);
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
                 "+v"(v[6]), "+v"(v[7]));
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kCostLanes; ++j) s += v[j];
  if (s == 12345.678f) out[blockIdx.x] = s;  // never true; keeps the work alive
}

// Binary64 accumulate step of the moment sums (cvt + 4 FMA/ADD per row).
__global__ __launch_bounds__(256) void k_opcost_moments(float* __restrict__ out, int iters, float seed) {
  double a = 0, b = 0, c = 0;
  float p = 1.5f + seed * float(threadIdx.x);
  const double yt = 0.25, mu = 1.0;
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kCostLanes; ++j) {
      const double d = double(p) - mu;
      a += d;
      b = fma(d, d, b);
      c = fma(d, yt, c);
      p = p * 1.0000001f;
    }
    asm volatile("" : "+v"(p));
  }
  if (a + b + c == 12345.678) out[blockIdx.x] = float(a);
}

template <int OP>
static float time_one(int iters, hipStream_t s, float* out) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int blocks = 256 * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
  hipLaunchKernelGGL(k_opcost<OP>, dim3(blocks), dim3(256), 0, s, out, 4, 0.001f);  // warm
  (void)hipEventRecord(e0, s);
  hipLaunchKernelGGL(k_opcost<OP>, dim3(blocks), dim3(256), 0, s, out, iters, 0.001f);
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

static float time_moments(int iters, hipStream_t s, float* out) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int blocks = 256 * 8;
  hipLaunchKernelGGL(k_opcost_moments, dim3(blocks), dim3(256), 0, s, out, 4, 0.001f);
  (void)hipEventRecord(e0, s);
  hipLaunchKernelGGL(k_opcost_moments, dim3(blocks), dim3(256), 0, s, out, iters, 0.001f);
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// out[op] for op in UOP numbering (ADD..LOG; RSUB/RDIV/RPOW copy their
// forward twins), out[UOP_NUM] = binary64 moment step per row.  Units: seconds
// per lane-application; the caller converts with its peak rate.
int measure_op_costs(double* out, int n, int iters, hipStream_t s, float* scratch) {
  if (n < UOP_NUM + 1) return -1;
  const double lanes = 256.0 * 8 * 256;
  const double apps = lanes * double(iters) * kCostLanes;
  auto put = [&](int op, float ms) { out[op] = double(ms) * 1e-3 / apps; };
  for (int i = 0; i < n; ++i) out[i] = 0.0;
  put(UOP_ADD, time_one<UOP_ADD>(iters, s, scratch));
  put(UOP_SUB, time_one<UOP_SUB>(iters, s, scratch));
  put(UOP_MUL, time_one<UOP_MUL>(iters, s, scratch));
  put(UOP_DIV, time_one<UOP_DIV>(iters, s, scratch));
  put(UOP_POW, time_one<UOP_POW>(iters / 4, s, scratch) * 4.0f);
  put(UOP_SIN, time_one<UOP_SIN>(iters / 4, s, scratch) * 4.0f);
  put(UOP_COS, time_one<UOP_COS>(iters / 4, s, scratch) * 4.0f);
  put(UOP_SQ, time_one<UOP_SQ>(iters, s, scratch));
  put(UOP_SQRT, time_one<UOP_SQRT>(iters, s, scratch));
  put(UOP_EXP, time_one<UOP_EXP>(iters, s, scratch));
  put(UOP_LOG, time_one<UOP_LOG>(iters, s, scratch));
  out[UOP_RSUB] = out[UOP_SUB];
  out[UOP_RDIV] = out[UOP_DIV];
  out[UOP_RPOW] = out[UOP_POW];
  out[UOP_NUM] = double(time_moments(iters, s, scratch)) * 1e-3 / apps;
  return 0;
}

}  // namespace gg

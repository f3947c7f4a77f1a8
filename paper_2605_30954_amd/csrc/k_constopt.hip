// Constant optimisation driven by the fitness gradient: one Adam step
// (Kingma & Ba, "Adam: A Method for Stochastic Optimization", 2015, Alg. 1)
// on every program's constants, with the best constants seen so far kept per
// program.  The paper names real-valued constant optimisation as the next
// thing to integrate with the GPU evaluation (Section 5); the gradient comes
// from the fused fitness + gradient call.
//
// One wave per program (constants strided over its 64 lanes): the program's
// fitness and best fitness are wave-uniform, so the "better" decision and the
// best-fitness update need no synchronisation.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace gg {
namespace {

__global__ __launch_bounds__(64) void k_adam_consts(float* __restrict__ consts, int C,
                                                    const double* __restrict__ grad,
                                                    const double* __restrict__ fitness,
                                                    float* __restrict__ mom1, float* __restrict__ mom2,
                                                    float* __restrict__ best_c,
                                                    double* __restrict__ best_f, AdamParams p) {
  const int i = blockIdx.x;
  const double f = fitness[i];
  const bool better = f < best_f[i];  // a NaN or +inf fitness is never better
  const bool finite = isfinite(f);
  const size_t row = size_t(i) * size_t(C);
  for (int j = threadIdx.x; j < C; j += 64) {
    const size_t k = row + size_t(j);
    const float c = consts[k];
    if (better) best_c[k] = c;
    if (!finite) {  // the step left the finite region: back to the best point
      consts[k] = better ? c : best_c[k];
      mom1[k] = 0.0f;
      mom2[k] = 0.0f;
      continue;
    }
    const float g = float(grad[k]);
    if (!isfinite(g)) continue;
    const float m = p.beta1 * mom1[k] + p.omb1 * g;
    const float v = p.beta2 * mom2[k] + p.omb2 * (g * g);
    if (!isfinite(v)) continue;  // g^2 beyond binary32: this constant keeps its state
    mom1[k] = m;
    mom2[k] = v;
    const float mhat = m / p.bias1;
    const float vhat = v / p.bias2;
    consts[k] = c - p.lr * mhat / (sqrtf(vhat) + p.eps);
  }
  if (threadIdx.x == 0 && better) best_f[i] = f;
}

}  // namespace

hipError_t launch_adam_consts(float* consts, int M, int C, const double* grad, const double* fitness,
                              float* mom1, float* mom2, float* best_c, double* best_f,
                              const AdamParams& p, hipStream_t s) {
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam_consts, dim3(unsigned(M)), dim3(64), 0, s, consts, C, grad, fitness, mom1,
                     mom2, best_c, best_f, p);
  return hipGetLastError();
}

}  // namespace gg

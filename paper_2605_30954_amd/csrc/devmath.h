// Protected operators in node precision (float or double), device side.
//
// Semantics (the paper lists the operators of Tab. 2 without saying how they
// are protected; this is the reading the whole library implements):
//   div_p(a,b)  = 1 if |b| < G else a/b
//   sqrt_p(a)   = sqrt(|a|)
//   exp_c(a)    = exp(clamp(a, -80, 80)), NaN passed through the clamp
//   log_p(a)    = 0 if |a| < G else log|a|
//   pow_p(a,b)  = 0 if |a| < G else exp(clamp(b * log|a|, -80, 80))
// with G the binary32 value nearest to 1e-6 in both precisions.
// Division and square root are correctly rounded (hipcc's default); sin, cos,
// exp and log are the ROCm device library's (ocml) routines.
#pragma once
#include <hip/hip_runtime.h>

#include "gpgomea_ops.h"

namespace gg {

template <typename T>
struct Prot;

template <>
struct Prot<float> {
  static constexpr float G = float(GPGOMEA_GUARD);
  static constexpr float CL = float(GPGOMEA_CLAMP);
  __device__ static inline float clamp(float t) { return t < -CL ? -CL : (t > CL ? CL : t); }
  __device__ static inline float div(float a, float b) { return fabsf(b) < G ? 1.0f : a / b; }
  __device__ static inline float sqrt_(float a) { return sqrtf(fabsf(a)); }
  __device__ static inline float exp_(float a) { return expf(clamp(a)); }
  __device__ static inline float log_(float a) { return fabsf(a) < G ? 0.0f : logf(fabsf(a)); }
  __device__ static inline float pow_(float a, float b) {
    const float l = logf(fabsf(a));
    return fabsf(a) < G ? 0.0f : expf(clamp(b * l));
  }
  __device__ static inline float sin_(float a) { return sinf(a); }
  __device__ static inline float cos_(float a) { return cosf(a); }
};

template <>
struct Prot<double> {
  static constexpr double G = double(float(GPGOMEA_GUARD));
  static constexpr double CL = GPGOMEA_CLAMP;
  __device__ static inline double clamp(double t) { return t < -CL ? -CL : (t > CL ? CL : t); }
  __device__ static inline double div(double a, double b) { return fabs(b) < G ? 1.0 : a / b; }
  __device__ static inline double sqrt_(double a) { return sqrt(fabs(a)); }
  __device__ static inline double exp_(double a) { return exp(clamp(a)); }
  __device__ static inline double log_(double a) { return fabs(a) < G ? 0.0 : log(fabs(a)); }
  __device__ static inline double pow_(double a, double b) {
    const double l = log(fabs(a));
    return fabs(a) < G ? 0.0 : exp(clamp(b * l));
  }
  __device__ static inline double sin_(double a) { return sin(a); }
  __device__ static inline double cos_(double a) { return cos(a); }
};

// Local partial derivatives used by the adjoint (same conventions as the
// semantics: a guarded branch or a saturated clamp has derivative 0, and
// sqrt|a| has derivative 0 at a = 0).
template <typename T>
struct Deriv {
  using P = Prot<T>;
  // d div_p(a,b)/da, d/db given the value v = a/b
  __device__ static inline void ddiv(T a, T b, T v, T& da, T& db) {
    const bool g = fabs(b) < P::G;
    const T r = T(1) / b;
    da = g ? T(0) : r;
    db = g ? T(0) : -v * r;
  }
  __device__ static inline void dpow(T a, T b, T v, T& da, T& db) {
    const bool g = fabs(a) < P::G;
    const T l = ::log(fabs(a));
    const T t = b * l;
    const bool live = !g && t >= -P::CL && t <= P::CL;
    da = live ? v * b / a : T(0);
    db = live ? v * l : T(0);
  }
  __device__ static inline T dsin(T a) { return ::cos(a); }
  __device__ static inline T dcos(T a) { return -::sin(a); }
  __device__ static inline T dsqrt(T a, T v) { return a == T(0) ? T(0) : (a > T(0) ? T(0.5) : T(-0.5)) / v; }
  __device__ static inline T dexp(T a, T v) { return (a >= -P::CL && a <= P::CL) ? v : T(0); }
  __device__ static inline T dlog(T a) { return fabs(a) < P::G ? T(0) : T(1) / a; }
};

}  // namespace gg

// Wright omega function omega(z) = W_0(e^z), the solution w > 0 of
// w + log(w) = z, for real z.  Table 1 (squared-error datafit), Table 2 and
// Appendix A (squared-l2 / elastic-net weight steps) need W_0(c e^z), which is
// omega(z + log c) without the overflow of e^z.
//
// Method: a region-wise starting value followed by the fourth-order iteration
// of Fritsch, Shafer & Crowley (Comm. ACM 16(2), 1973), in the form used by
// Lawrence, Corless & Jeffrey (ACM TOMS 38(3), Algorithm 917, 2012):
//   r = z - w - log w,
//   w <- w * (1 + r/(1+w) * ((1+w)(1+w+2r/3) - r/2) / ((1+w)(1+w+2r/3) - r)).
// For z << 0 the fixed point w = exp(z - w) converges quadratically from e^z;
// for very large z, w = z - log z to working precision.
#pragma once
#include <hip/hip_runtime.h>

template <typename T> struct omega_consts;
template <> struct omega_consts<float>  { static constexpr float  big = 1.0e8f;  static constexpr int iters = 2; };
template <> struct omega_consts<double> { static constexpr double big = 1.0e150; static constexpr int iters = 3; };

template <typename T>
__device__ __forceinline__ T wright_omega(T z) {
  if (!(z == z)) return z;                      // NaN propagates
  if (z < T(-18)) {                              // w ~ e^z; one fixed-point pass w = e^{z-w}
    T w = exp(z);
    return exp(z - w);
  }
  if (z > omega_consts<T>::big) {
    if (z == T(INFINITY)) return z;
    T lz = log(z);
    return z - lz + lz / z;
  }
  T w;
  if (z < T(-2))      w = exp(z - exp(z));
  else if (z < T(1))  w = T(0.82) * log1p(exp(z));
  else                w = z - log(z);
#pragma unroll
  for (int it = 0; it < omega_consts<T>::iters; ++it) {
    T r = z - w - log(w);
    T a = (T(1) + w) * (T(1) + w + T(2) / T(3) * r);
    w = w * (T(1) + r / (T(1) + w) * (a - T(0.5) * r) / (a - r));
  }
  return w;
}

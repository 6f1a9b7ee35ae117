// Small device helpers: complex loads/stores with storage conversion.
#pragma once
#include <hip/hip_runtime.h>

namespace gwr {

__device__ __forceinline__ void ldc(const double2* p, double& re, double& im) {
  double2 v = *p;
  re = v.x;
  im = v.y;
}
__device__ __forceinline__ void ldc(const float2* p, double& re, double& im) {
  float2 v = *p;
  re = (double)v.x;
  im = (double)v.y;
}
__device__ __forceinline__ void stc(double2* p, double re, double im) { *p = make_double2(re, im); }
__device__ __forceinline__ void stc(float2* p, double re, double im) {
  *p = make_float2((float)re, (float)im);
}

// exp(i * 2 pi * frac) for a phase given as a fraction of a full turn
__device__ __forceinline__ void turn(double frac, double& c, double& s) { sincospi(2.0 * frac, &s, &c); }

}  // namespace gwr

namespace gwr {

// Prefetch helpers.  A prefetch loads unconditionally (from `p` when ok, else from the
// always-valid `base`) and keeps the value in its storage type; the validity mask is
// applied only when the value is consumed (keep()).  Neither a conversion nor a zero
// fill touches the destination register at the load, so the compiler never has to wait
// for the load (or, memory counters completing in order, for older stores) there.
template <class T>
__device__ __forceinline__ T ldraw(const T* p, const T* base, bool ok) {
  return *(ok ? p : base);
}
template <class T>
__device__ __forceinline__ T keep(const T& v, bool ok) {
  T z;
  z.x = ok ? v.x : 0;
  z.y = ok ? v.y : 0;
  return z;
}

}  // namespace gwr

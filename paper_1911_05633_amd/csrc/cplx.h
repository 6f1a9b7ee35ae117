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

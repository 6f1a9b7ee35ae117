// Electron count for the chemical-potential update (Sec. 4):
//   n = -g sum_a Re G^{R=0}_aa(beta^-)  or, from k space,  -(g / N_k) sum_k sum_a Re G_aa(k, beta^-),
// one FP64 reduction over the diagonal entries of the last tau slice (n_slices = 1 or N_k).
#include "cplx.h"
#include "internal.h"

namespace gwr {
namespace {

template <class TI>
__global__ __launch_bounds__(256) void density_kernel(const TI* __restrict__ GR, long long slice_off, int n_orb,
                                                      int n_slices, double g, double* __restrict__ n_dev) {
  __shared__ double part[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n_slices * n_orb; i += 256) {
    const int k = i / n_orb, a = i - k * n_orb;
    double re, im;
    ldc(GR + slice_off + ((long long)k * n_orb + a) * n_orb + a, re, im);
    s += re;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_dev = -g * part[0];
}

}  // namespace

gw_status launch_density(const gw_cell* c, const void* G, gw_dtype t, int space, double g, double* n_dev,
                         hipStream_t s) {
  // last tau slice; R = 0 only, or every k (averaged)
  const long long off = (long long)(c->n_tau - 1) * c->N_R * c->N_orb * c->N_orb;
  const int ns = space == 0 ? 1 : c->N_R;
  const double gs = space == 0 ? g : g / c->N_R;
  if (t == GW_C128)
    hipLaunchKernelGGL(density_kernel<double2>, dim3(1), dim3(256), 0, s, (const double2*)G, off, c->N_orb, ns, gs,
                       n_dev);
  else
    hipLaunchKernelGGL(density_kernel<float2>, dim3(1), dim3(256), 0, s, (const float2*)G, off, c->N_orb, ns, gs,
                       n_dev);
  return check_launch("density");
}

}  // namespace gwr

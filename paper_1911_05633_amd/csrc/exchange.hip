// Static (exchange) part of the self-energy.  Sec. 2 evaluates it with the MT-MT expression of
// Eq. (8) after replacing the screening interaction by the bare one, W~(tau) -> V, and the Green's
// function by -G(beta):
//   Sigma_x^R_ab = -sum C^I_aa' (-G^R_a'b'(beta)) V^R_IJ C^J_bb'.
// The self-energy kernels run on the single time slice tau = beta^- (one time point from the
// pointer to that slice) with V^R in place of W; the result is then negated, which applies the
// -G(beta).
#include "internal.h"

namespace gwr {
namespace {

__global__ __launch_bounds__(256) void negate_c128(double2* __restrict__ S, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double2 v = S[i];
    S[i] = make_double2(-v.x, -v.y);
  }
}

bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
  auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return !(x < y + nb && y < x + na);
}

}  // namespace
}  // namespace gwr

using namespace gwr;

extern "C" gw_status gw_exchange(const gw_cell* c, const void* GR, const void* VR, void* Sx, gw_precision prec,
                                 void* stream) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!GR || !VR || !Sx) return fail(GW_ERR_ARG, "NULL tensor");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const size_t slice = (size_t)c->N_R * c->N_orb * c->N_orb;
  const size_t ng = (size_t)c->n_tau * slice, nv = (size_t)c->N_R * c->N_pb * c->N_pb;
  if (!disjoint(GR, ng * es, Sx, slice * 16) || !disjoint(VR, nv * es, Sx, slice * 16))
    return fail(GW_ERR_ARG, "Sigma_x overlaps an input");
  const char* g_beta = static_cast<const char*>(GR) + (size_t)(c->n_tau - 1) * slice * es;
  hipStream_t s = (hipStream_t)stream;
  gw_status st = launch_self_energy(c, g_beta, VR, Sx, prec, s, 1);
  if (st != GW_OK) return st;
  const long long n = (long long)slice;
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(negate_c128, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s,
                     (double2*)Sx, n);
  return check_launch("gw_exchange");
}

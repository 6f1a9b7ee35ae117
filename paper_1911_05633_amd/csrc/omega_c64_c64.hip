// Matsubara transforms with c64 input and c64 output storage.
#include "omega_kernels.h"

namespace gwr {

gw_status tau2omega_c64_c64(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, void* out,
                          long long cols, hipStream_t s) {
  return tau2omega_typed(c, (const double2*)T, n_omega, parity, (const float2*)in, (float2*)out, cols, s);
}

gw_status drain_c64_c64(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, void* out, int n,
                      hipStream_t s) {
  return drain_typed(c, (const double2*)T, n_omega, parity, (const float2*)in, (float2*)out, n, GW_C64, s);
}

}  // namespace gwr

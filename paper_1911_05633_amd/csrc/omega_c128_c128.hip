// Matsubara transforms with c128 input and c128 output storage.
#include "omega_kernels.h"

namespace gwr {

gw_status tau2omega_c128_c128(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, void* out,
                          long long cols, hipStream_t s) {
  return tau2omega_typed(c, (const double2*)T, n_omega, parity, (const double2*)in, (double2*)out, cols, s);
}

gw_status drain_c128_c128(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, void* out, int n,
                      hipStream_t s) {
  return drain_typed(c, (const double2*)T, n_omega, parity, (const double2*)in, (double2*)out, n, GW_C128, s);
}

}  // namespace gwr

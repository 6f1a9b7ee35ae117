// Dispatch of the Matsubara transforms on the storage types of their operands.
#include "internal.h"

namespace gwr {

#define GWR_OMEGA_DECL(ti, to)                                                                            \
  gw_status tau2omega_##ti##_##to(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, \
                                  void* out, long long cols, hipStream_t s);                              \
  gw_status drain_##ti##_##to(const gw_cell* c, const void* T, int n_omega, int parity, const void* in,     \
                              void* out, int n, hipStream_t s);
GWR_OMEGA_DECL(c128, c128)
GWR_OMEGA_DECL(c128, c64)
GWR_OMEGA_DECL(c64, c128)
GWR_OMEGA_DECL(c64, c64)
#undef GWR_OMEGA_DECL

gw_status launch_tau2omega(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                           void* out, gw_dtype ot, long long cols, hipStream_t s) {
  if (it == GW_C128 && ot == GW_C128) return tau2omega_c128_c128(c, T, n_omega, parity, in, out, cols, s);
  if (it == GW_C128 && ot == GW_C64) return tau2omega_c128_c64(c, T, n_omega, parity, in, out, cols, s);
  if (it == GW_C64 && ot == GW_C128) return tau2omega_c64_c128(c, T, n_omega, parity, in, out, cols, s);
  return tau2omega_c64_c64(c, T, n_omega, parity, in, out, cols, s);
}

gw_status launch_drain(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                       void* out, gw_dtype ot, int n, hipStream_t s) {
  if (it == GW_C128 && ot == GW_C128) return drain_c128_c128(c, T, n_omega, parity, in, out, n, s);
  if (it == GW_C128 && ot == GW_C64) return drain_c128_c64(c, T, n_omega, parity, in, out, n, s);
  if (it == GW_C64 && ot == GW_C128) return drain_c64_c128(c, T, n_omega, parity, in, out, n, s);
  return drain_c64_c64(c, T, n_omega, parity, in, out, n, s);
}

}  // namespace gwr

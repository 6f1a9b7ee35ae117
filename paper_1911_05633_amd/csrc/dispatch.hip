// Kernel selection for the P and Sigma contractions.
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace gwr {

gw_status launch_p_generic(const gw_cell* c, const void* GR, void* P, double g, gw_precision p, hipStream_t s);
gw_status launch_s_generic(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision p,
                           hipStream_t s);

// GWR_KERNELS=generic selects the plain VALU kernels for every block shape (used by the
// tests to check the MFMA kernels against them on the device).
static bool force_generic() {
  const char* v = std::getenv("GWR_KERNELS");
  return v && std::strcmp(v, "generic") == 0;
}

gw_status launch_polarizability(const gw_cell* c, const void* GR, void* P, double g, gw_precision p,
                                hipStream_t s) {
  if (p == GW_BF16X3) return fail(GW_ERR_UNSUPPORTED, "BF16x3 polarizability not built yet");
  (void)force_generic();
  return launch_p_generic(c, GR, P, g, p, s);
}

gw_status launch_self_energy(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision p,
                             hipStream_t s) {
  if (p == GW_BF16X3) return fail(GW_ERR_UNSUPPORTED, "BF16x3 self-energy not built yet");
  (void)force_generic();
  return launch_s_generic(c, GR, WR, S, p, s);
}

}  // namespace gwr

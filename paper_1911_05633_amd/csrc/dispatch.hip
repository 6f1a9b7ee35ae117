// Kernel selection for the P and Sigma contractions, one launch per species pair.
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace gwr {

void launch_p_generic_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                           double g, gw_precision p, hipStream_t s);
void launch_s_generic_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR,
                           const void* WR, void* S, gw_precision p, hipStream_t s, int nt);
bool mfma_pair_ok(const SpeciesDev& A, const SpeciesDev& B);
void launch_p_mfma_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                        double g, gw_precision p, hipStream_t s);
void launch_s_mfma_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR,
                        const void* WR, void* S, gw_precision p, hipStream_t s, int nt);
void launch_p_mfma_gen(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                       double g, gw_precision p, hipStream_t s);
void launch_s_mfma_gen(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, const void* WR,
                       void* S, gw_precision p, hipStream_t s, int nt);

// GWR_KERNELS=generic selects the plain VALU kernels for every block shape; the tests
// use it to check the matrix-core kernels against them on the device.
static bool force_generic() {
  const char* v = std::getenv("GWR_KERNELS");
  return v && std::strcmp(v, "generic") == 0;
}

gw_status launch_polarizability(const gw_cell* c, const void* GR, void* P, double g, gw_precision p,
                                hipStream_t s) {
  // GW_BF16X3: split-precision BF16 kernel for the 9-orbital / 49..64-function species
  // pairs, the FP32 kernels for every other shape.  Pairs beyond the compact kernels' tiles
  // (more than 9 orbitals or 64 product functions on either atom) run the general
  // matrix-core kernels.
  const bool gen = force_generic();
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const SpeciesDev &A = c->sp[sa], &B = c->sp[sb];
      if (A.atoms.empty() || B.atoms.empty()) continue;
      if (gen)
        launch_p_generic_pair(c, A, B, GR, P, g, p, s);
      else if (mfma_pair_ok(A, B) && mfma_pair_ok(B, A))
        launch_p_mfma_pair(c, A, B, GR, P, g, p, s);
      else
        launch_p_mfma_gen(c, A, B, GR, P, g, p, s);
    }
  return check_launch("polarizability");
}

gw_status launch_self_energy(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision p,
                             hipStream_t s, int n_tau) {
  const int nt = n_tau < 0 ? c->n_tau : n_tau;
  // GW_BF16X3: split-precision BF16 kernel for the 9-orbital / 49..64-function species
  // pairs, the FP32 kernels for every other shape
  const bool gen = force_generic();
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const SpeciesDev &A = c->sp[sa], &B = c->sp[sb];
      if (A.atoms.empty() || B.atoms.empty()) continue;
      if (gen)
        launch_s_generic_pair(c, A, B, GR, WR, S, p, s, nt);
      else if (mfma_pair_ok(A, B))
        launch_s_mfma_pair(c, A, B, GR, WR, S, p, s, nt);
      else
        launch_s_mfma_gen(c, A, B, GR, WR, S, p, s, nt);
    }
  return check_launch("self-energy");
}

}  // namespace gwr

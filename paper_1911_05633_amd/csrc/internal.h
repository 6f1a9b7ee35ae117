// Internal declarations of libgwr (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gwr.h"

namespace gwr {

constexpr int kMaxOrb = 16;
constexpr int kMaxPb = 128;
constexpr int kMaxR = 64;
constexpr double kTauTol = 1e-12;  // relative to beta: end points and mirror symmetry of the tau grid
constexpr int kMaxPairs = kMaxOrb * (kMaxOrb + 1) / 2;  // 136

// Per-species device constants.
struct SpeciesDev {
  int n = 0, m = 0;     // orbitals, product functions
  int np = 0;           // unordered orbital pairs n(n+1)/2
  int np_pad = 0;       // np rounded up to a multiple of 16
  int m_pad = 0;        // m rounded up to a multiple of 16
  double* C = nullptr;          // [m][n][n] FP64 (plain layout)
  float* C32 = nullptr;         // [m][n][n] FP32
  double* Cpair = nullptr;      // [m_pad][np_pad] FP64, C^I_{ab} at pair p = {a <= b}, zero padded
  float* Cpair32 = nullptr;     // same, FP32
  std::vector<int> atoms;       // atoms of this species (host)
  int* atoms_dev = nullptr;     // same on device
  int2* offs_dev = nullptr;     // per atom of this species: (first product function, first orbital)
};

struct PairTables {
  // unordered pair p -> (a, b), a <= b, row-major over a then b >= a, per orbital count n
  unsigned char a[kMaxPairs];
  unsigned char b[kMaxPairs];
};

}  // namespace gwr

struct gw_cell {
  int device = 0;
  int n_cu = 256;                      // compute units of the device (sizes persistent grids)
  int n_atoms = 0, n_species = 0;
  std::vector<int> species;            // per atom
  std::vector<int> n_orb, n_pb;        // per species
  std::vector<int> orb_off, pb_off;    // per atom, size n_atoms + 1
  int N_orb = 0, N_pb = 0;
  int mesh[3] = {1, 1, 1};
  int N_R = 1;
  int n_tau = 0;
  double beta = 0;
  std::vector<double> tau;             // host, the grid given at creation
  double* tau_dev = nullptr;           // the same on the device
  std::vector<int> minusR;             // host
  int* minusR_dev = nullptr;
  int* orb_off_dev = nullptr;
  int* pb_off_dev = nullptr;
  int* species_dev = nullptr;
  std::vector<gwr::SpeciesDev> sp;
  std::vector<void*> owned;            // every device allocation, freed at destroy
  // real-space cutoff (gw_cell_set_pairs): kept blocks (R, A, B, mA, mB) on the host, and per
  // species pair (sa * n_species + sb) on the device as (R, index of A in its species, index
  // of B in its species, mA | mB << 16)
  bool pairs_set = false;
  std::vector<int> pair_list;
  std::vector<int4*> pair_dev;
  std::vector<int4*> pair_dev_mfma;    // same blocks as two int4 each (see launch_p_mfma_list)
  std::vector<int> pair_cnt;
  // packed layout of the kept blocks (gw_*_packed): elements per tau slice; per kept block
  // (R, mA | mB << 16, pA, pB), (offset, 0, 0, 0); per (A, B) pair (CSR over A * n_atoms + B) the
  // kept blocks (R, mA | mB << 16, offset, 0)
  long long packed_per_tau = 0;
  int4* packed_blocks_dev = nullptr;
  int4* packed_ab_items_dev = nullptr;
  int* packed_ab_ptr_dev = nullptr;
  double2* kr_phase_dev = nullptr;     // [N_k][N_R]: exp(+i k.R)
};

namespace gwr {

// thread-local error detail
void set_error(const std::string& msg);
gw_status fail(gw_status s, const std::string& msg);
gw_status check_launch(const char* what);

inline size_t csize(gw_dtype t) { return t == GW_C128 ? 16 : 8; }

// launchers (defined in the kernel sources); all validation is done by the caller
gw_status launch_fourier(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot,
                         int n, int sign, hipStream_t s);
gw_status launch_tau2omega(const gw_cell* c, const void* T, int n_omega, int parity, const void* in,
                           gw_dtype it, void* out, gw_dtype ot, long long cols, hipStream_t s);
gw_status launch_drain(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                       void* out, gw_dtype ot, int n, hipStream_t s);
gw_status launch_polarizability(const gw_cell* c, const void* GR, void* P, double g, gw_precision p,
                                hipStream_t s);
// plain kernels over a list of (R, iA, iB, mA | mB << 16) blocks of one species pair
void launch_p_generic_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                           const void* GR, void* P, double g, gw_precision p, hipStream_t s);
void launch_s_generic_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                           const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s);
// matrix-core kernels over a list of (R, mA | mB << 16, pb A, orb A), (pb B, orb B, 0, 0)
// entries; false when the shape / precision has no list kernel
bool mfma_pair_ok(const SpeciesDev& A, const SpeciesDev& B);
bool launch_p_mfma_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                        const void* GR, void* P, double g, gw_precision p, hipStream_t s);
bool launch_s_mfma_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                        const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s);
// n_tau < 0: the cell's time points; otherwise that many slices of GR and WR from the pointers given
gw_status launch_self_energy(const gw_cell* c, const void* GR, const void* WR, void* S,
                             gw_precision p, hipStream_t s, int n_tau = -1);
gw_status launch_density(const gw_cell* c, const void* G, gw_dtype t, int space, double g, double* n_dev,
                         hipStream_t s);

}  // namespace gwr

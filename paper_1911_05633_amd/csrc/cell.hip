// Cell description, validation and the C-ABI entry points of libgwr.
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "internal.h"

namespace gwr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

gw_status fail(gw_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

gw_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GW_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GW_OK;
}

template <class T>
static gw_status upload(gw_cell* c, T** dst, const T* src, size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(T) + 16) != hipSuccess) return fail(GW_ERR_NOMEM, "hipMalloc failed");
  c->owned.push_back(p);
  if (hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(GW_ERR_HIP, "hipMemcpy failed");
  *dst = static_cast<T*>(p);
  return GW_OK;
}

static int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace gwr

using namespace gwr;

extern "C" {

const char* gw_status_string(gw_status s) {
  switch (s) {
    case GW_OK: return "ok";
    case GW_ERR_ARG: return "invalid argument";
    case GW_ERR_SHAPE: return "inconsistent or unsupported shape";
    case GW_ERR_NOMEM: return "device allocation failed";
    case GW_ERR_HIP: return "HIP runtime error";
    case GW_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char* gw_last_error(void) { return g_last_error.c_str(); }

void gw_cell_destroy(gw_cell* cell) {
  if (!cell) return;
  int cur = 0;
  bool have = hipGetDevice(&cur) == hipSuccess;
  if (have && cur != cell->device) (void)hipSetDevice(cell->device);
  for (void* p : cell->owned) (void)hipFree(p);
  if (have && cur != cell->device) (void)hipSetDevice(cur);
  delete cell;
}

gw_status gw_cell_create(gw_cell** out, int n_atoms, const int* species_of_atom, int n_species,
                         const int* n_orb, const int* n_pb, const double* C, const int* mesh,
                         int n_tau, double beta, const double* tau) {
  if (!out) return fail(GW_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!species_of_atom || !n_orb || !n_pb || !C || !mesh) return fail(GW_ERR_ARG, "NULL input array");
  if (!tau) return fail(GW_ERR_ARG, "tau grid is NULL");
  if (n_atoms < 1 || n_species < 1) return fail(GW_ERR_SHAPE, "need n_atoms >= 1 and n_species >= 1");
  if (n_tau < 2 || n_tau > 256) return fail(GW_ERR_SHAPE, "need 2 <= n_tau <= 256");
  if (!(beta > 0) || !std::isfinite(beta)) return fail(GW_ERR_ARG, "beta must be positive and finite");
  // the grid runs from 0+ to beta- and is symmetric about beta / 2: the polarizability's mirror,
  // the drains' parity pairing and the beta- slice of the density and the exchange rely on it
  const double ttol = kTauTol * beta;
  for (int i = 0; i < n_tau; ++i)
    if (!std::isfinite(tau[i])) return fail(GW_ERR_ARG, "tau has a non-finite entry");
  if (std::fabs(tau[0]) > ttol || std::fabs(tau[n_tau - 1] - beta) > ttol)
    return fail(GW_ERR_ARG, "tau must start at 0 and end at beta");
  for (int i = 0; i + 1 < n_tau; ++i)
    if (!(tau[i + 1] > tau[i])) return fail(GW_ERR_ARG, "tau must be strictly increasing");
  for (int i = 0; i < n_tau; ++i)
    if (std::fabs(tau[i] + tau[n_tau - 1 - i] - beta) > ttol)
      return fail(GW_ERR_ARG, "tau grid is not symmetric about beta / 2");
  for (int i = 0; i < 3; ++i)
    if (mesh[i] < 1) return fail(GW_ERR_SHAPE, "mesh entries must be >= 1");
  const int NR = mesh[0] * mesh[1] * mesh[2];
  if (NR > kMaxR) return fail(GW_ERR_SHAPE, "N_R above the supported maximum of 64");
  for (int s = 0; s < n_species; ++s) {
    if (n_orb[s] < 1 || n_orb[s] > kMaxOrb) return fail(GW_ERR_SHAPE, "n_orb must be in [1, 16]");
    if (n_pb[s] < 1 || n_pb[s] > kMaxPb) return fail(GW_ERR_SHAPE, "n_pb must be in [1, 128]");
  }
  for (int a = 0; a < n_atoms; ++a)
    if (species_of_atom[a] < 0 || species_of_atom[a] >= n_species)
      return fail(GW_ERR_ARG, "species_of_atom out of range");

  gw_cell* c = new gw_cell();
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(GW_ERR_HIP, "hipGetDevice failed");
  }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      c->n_cu < 1)
    c->n_cu = 256;
  c->n_atoms = n_atoms;
  c->n_species = n_species;
  c->species.assign(species_of_atom, species_of_atom + n_atoms);
  c->n_orb.assign(n_orb, n_orb + n_species);
  c->n_pb.assign(n_pb, n_pb + n_species);
  c->orb_off.resize(n_atoms + 1);
  c->pb_off.resize(n_atoms + 1);
  c->orb_off[0] = c->pb_off[0] = 0;
  for (int a = 0; a < n_atoms; ++a) {
    c->orb_off[a + 1] = c->orb_off[a] + n_orb[species_of_atom[a]];
    c->pb_off[a + 1] = c->pb_off[a] + n_pb[species_of_atom[a]];
  }
  c->N_orb = c->orb_off[n_atoms];
  c->N_pb = c->pb_off[n_atoms];
  for (int i = 0; i < 3; ++i) c->mesh[i] = mesh[i];
  c->N_R = NR;
  c->n_tau = n_tau;
  c->beta = beta;
  c->tau.assign(tau, tau + n_tau);
  c->minusR.resize(NR);
  for (int n1 = 0; n1 < mesh[0]; ++n1)
    for (int n2 = 0; n2 < mesh[1]; ++n2)
      for (int n3 = 0; n3 < mesh[2]; ++n3) {
        int r = (n1 * mesh[1] + n2) * mesh[2] + n3;
        int m1 = (mesh[0] - n1) % mesh[0], m2 = (mesh[1] - n2) % mesh[1], m3 = (mesh[2] - n3) % mesh[2];
        c->minusR[r] = (m1 * mesh[1] + m2) * mesh[2] + m3;
      }

  // symmetric coefficients, then device layouts
  c->sp.resize(n_species);
  size_t off = 0;
  gw_status st = GW_OK;
  for (int s = 0; s < n_species && st == GW_OK; ++s) {
    SpeciesDev& d = c->sp[s];
    const int n = n_orb[s], m = n_pb[s];
    d.n = n;
    d.m = m;
    d.np = n * (n + 1) / 2;
    d.np_pad = round_up(d.np, 16);
    d.m_pad = round_up(m, 16);
    const double* Cs = C + off;
    off += (size_t)m * n * n;
    double cmax = 0;
    for (int i = 0; i < m * n * n; ++i) {
      if (!std::isfinite(Cs[i])) {
        gw_cell_destroy(c);
        return fail(GW_ERR_ARG, "C has a non-finite entry");
      }
      cmax = std::fmax(cmax, std::fabs(Cs[i]));
    }
    for (int I = 0; I < m; ++I)
      for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
          if (std::fabs(Cs[(I * n + a) * n + b] - Cs[(I * n + b) * n + a]) > 1e-12 * cmax) {
            gw_cell_destroy(c);
            return fail(GW_ERR_ARG, "C must be symmetric in its two orbital indices");
          }
    std::vector<float> c32(Cs, Cs + (size_t)m * n * n);
    std::vector<double> cp((size_t)d.m_pad * d.np_pad, 0.0);
    std::vector<float> cp32((size_t)d.m_pad * d.np_pad, 0.0f);
    for (int I = 0; I < m; ++I) {
      int p = 0;
      for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b, ++p) {
          cp[(size_t)I * d.np_pad + p] = Cs[(I * n + a) * n + b];
          cp32[(size_t)I * d.np_pad + p] = (float)Cs[(I * n + a) * n + b];
        }
    }
    for (int a = 0; a < n_atoms; ++a)
      if (species_of_atom[a] == s) d.atoms.push_back(a);
    if (d.atoms.empty()) d.atoms.push_back(-1);  // placeholder, never launched
    if ((st = upload(c, &d.C, Cs, (size_t)m * n * n)) != GW_OK) break;
    if ((st = upload(c, &d.C32, c32.data(), c32.size())) != GW_OK) break;
    if ((st = upload(c, &d.Cpair, cp.data(), cp.size())) != GW_OK) break;
    if ((st = upload(c, &d.Cpair32, cp32.data(), cp32.size())) != GW_OK) break;
    if ((st = upload(c, &d.atoms_dev, d.atoms.data(), d.atoms.size())) != GW_OK) break;
    std::vector<int2> offs(d.atoms.size(), make_int2(0, 0));
    for (size_t i = 0; i < d.atoms.size(); ++i)
      if (d.atoms[i] >= 0) offs[i] = make_int2(c->pb_off[d.atoms[i]], c->orb_off[d.atoms[i]]);
    if ((st = upload(c, &d.offs_dev, offs.data(), offs.size())) != GW_OK) break;
    if (d.atoms[0] < 0) d.atoms.clear();
  }
  if (st == GW_OK) st = upload(c, &c->minusR_dev, c->minusR.data(), c->minusR.size());
  if (st == GW_OK) st = upload(c, &c->orb_off_dev, c->orb_off.data(), c->orb_off.size());
  if (st == GW_OK) st = upload(c, &c->pb_off_dev, c->pb_off.data(), c->pb_off.size());
  if (st == GW_OK) st = upload(c, &c->species_dev, c->species.data(), c->species.size());
  if (st == GW_OK) st = upload(c, &c->tau_dev, c->tau.data(), c->tau.size());
  if (st == GW_OK) {
    // exp(+i k.R) for every (k, R) of the mesh, k.R = 2 pi sum_i j_i n_i / N_i taken modulo one turn
    std::vector<double2> ph((size_t)NR * NR);
    for (int kq = 0; kq < NR; ++kq)
      for (int r = 0; r < NR; ++r) {
        const int j[3] = {kq / (mesh[1] * mesh[2]), (kq / mesh[2]) % mesh[1], kq % mesh[2]};
        const int n[3] = {r / (mesh[1] * mesh[2]), (r / mesh[2]) % mesh[1], r % mesh[2]};
        double frac = 0;
        for (int i = 0; i < 3; ++i) frac += (double)((j[i] * n[i]) % mesh[i]) / mesh[i];
        frac -= std::floor(frac);
        ph[(size_t)kq * NR + r] = make_double2(std::cos(2.0 * M_PI * frac), std::sin(2.0 * M_PI * frac));
      }
    st = upload(c, &c->kr_phase_dev, ph.data(), ph.size());
  }
  if (st != GW_OK) {
    std::string msg = g_last_error;
    gw_cell_destroy(c);
    return fail(st, msg);
  }
  *out = c;
  return GW_OK;
}

size_t gw_workspace_bytes(const gw_cell* c, gw_precision prec) {
  // the hot-path calls keep every temporary in registers and LDS; prec is accepted for the
  // signature's sake (no precision needs scratch either)
  (void)c;
  (void)prec;
  return 0;
}

gw_status gw_cell_tau(const gw_cell* c, double* tau) {
  if (!c || !tau) return fail(GW_ERR_ARG, "NULL pointer");
  std::memcpy(tau, c->tau.data(), c->tau.size() * sizeof(double));
  return GW_OK;
}

int gw_cell_n_orb_total(const gw_cell* c) { return c ? c->N_orb : 0; }
int gw_cell_n_pb_total(const gw_cell* c) { return c ? c->N_pb : 0; }
int gw_cell_n_R(const gw_cell* c) { return c ? c->N_R : 0; }

}  // extern "C"

// ---------------------------------------------------------------------------
// argument checks shared by the entry points
// ---------------------------------------------------------------------------
namespace {

gw_status check_cell(const gw_cell* c) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  return GW_OK;
}

bool valid_dtype(gw_dtype t) { return t == GW_C128 || t == GW_C64; }
bool valid_prec(gw_precision p) { return p == GW_FP64 || p == GW_FP32 || p == GW_BF16X3; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// in/out aliasing rule of the transforms: identical pointers with identical type, or disjoint
gw_status check_alias(const void* in, size_t nin, gw_dtype it, const void* out, size_t nout, gw_dtype ot) {
  if (in == out) {
    if (it != ot) return fail(GW_ERR_ARG, "in-place transform needs in_type == out_type");
    return GW_OK;
  }
  if (overlap(in, nin, out, nout)) return fail(GW_ERR_ARG, "in and out overlap without being identical");
  return GW_OK;
}

}  // namespace

extern "C" {

static gw_status fourier_common(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot,
                                int basis, void* stream, int sign) {
  gw_status st = check_cell(c);
  if (st != GW_OK) return st;
  if (!in || !out) return fail(GW_ERR_ARG, "NULL tensor");
  if (!valid_dtype(it) || !valid_dtype(ot)) return fail(GW_ERR_ARG, "bad dtype");
  if (basis != 0 && basis != 1) return fail(GW_ERR_ARG, "basis must be 0 (orbital) or 1 (product)");
  const long long n = basis == 0 ? c->N_orb : c->N_pb;
  const long long elems = (long long)c->n_tau * c->N_R * n * n;
  st = check_alias(in, elems * csize(it), it, out, elems * csize(ot), ot);
  if (st != GW_OK) return st;
  return launch_fourier(c, in, it, out, ot, (int)n, sign, (hipStream_t)stream);
}

gw_status gw_fourier_k2r(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot, int basis,
                         void* stream) {
  return fourier_common(c, in, it, out, ot, basis, stream, +1);
}

gw_status gw_fourier_r2k(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot, int basis,
                         void* stream) {
  return fourier_common(c, in, it, out, ot, basis, stream, -1);
}

static gw_status omega_common(const gw_cell* c, const void* T, int n_omega, int parity, const void* in,
                              gw_dtype it, void* out, gw_dtype ot, int basis, long long* n_out) {
  gw_status st = check_cell(c);
  if (st != GW_OK) return st;
  if (!T || !in || !out) return fail(GW_ERR_ARG, "NULL tensor");
  if (parity < -1 || parity > 1) return fail(GW_ERR_ARG, "parity must be -1, 0 or +1");
  if (!valid_dtype(it) || !valid_dtype(ot)) return fail(GW_ERR_ARG, "bad dtype");
  if (basis != 0 && basis != 1) return fail(GW_ERR_ARG, "basis must be 0 (orbital) or 1 (product)");
  if (n_omega < 1 || n_omega > 256) return fail(GW_ERR_SHAPE, "n_omega must be in [1, 256]");
  const long long n = basis == 0 ? c->N_orb : c->N_pb;
  const long long cols = (long long)c->N_R * n * n;
  if (in == out) {
    if (it != ot) return fail(GW_ERR_ARG, "in-place transform needs in_type == out_type");
  } else if (overlap(in, c->n_tau * cols * csize(it), out, n_omega * cols * csize(ot))) {
    return fail(GW_ERR_ARG, "in and out overlap without being identical");
  }
  *n_out = n;
  return GW_OK;
}

gw_status gw_tau2omega(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                       void* out, gw_dtype ot, int basis, void* stream) {
  long long n = 0;
  gw_status st = omega_common(c, T, n_omega, parity, in, it, out, ot, basis, &n);
  if (st != GW_OK) return st;
  return launch_tau2omega(c, T, n_omega, parity, in, it, out, ot, (long long)c->N_R * n * n,
                          (hipStream_t)stream);
}

gw_status gw_drain(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                   void* out, gw_dtype ot, int basis, void* stream) {
  long long n = 0;
  gw_status st = omega_common(c, T, n_omega, parity, in, it, out, ot, basis, &n);
  if (st != GW_OK) return st;
  return launch_drain(c, T, n_omega, parity, in, it, out, ot, (int)n, (hipStream_t)stream);
}

gw_status gw_polarizability(const gw_cell* c, const void* GR, void* P, double g, gw_precision prec,
                            void* stream) {
  gw_status st = check_cell(c);
  if (st != GW_OK) return st;
  if (!GR || !P) return fail(GW_ERR_ARG, "NULL tensor");
  if (!valid_prec(prec)) return fail(GW_ERR_ARG, "bad precision");
  if (!std::isfinite(g)) return fail(GW_ERR_ARG, "spin factor must be finite");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  if (overlap(GR, (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb * es, P,
              (size_t)c->n_tau * c->N_R * c->N_pb * c->N_pb * es))
    return fail(GW_ERR_ARG, "GR and P overlap");
  return launch_polarizability(c, GR, P, g, prec, (hipStream_t)stream);
}

gw_status gw_self_energy(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision prec,
                         void* stream) {
  gw_status st = check_cell(c);
  if (st != GW_OK) return st;
  if (!GR || !WR || !S) return fail(GW_ERR_ARG, "NULL tensor");
  if (!valid_prec(prec)) return fail(GW_ERR_ARG, "bad precision");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const size_t ng = (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb;
  const size_t nw = (size_t)c->n_tau * c->N_R * c->N_pb * c->N_pb;
  if (overlap(GR, ng * es, S, ng * 16) || overlap(WR, nw * es, S, ng * 16))
    return fail(GW_ERR_ARG, "Sigma overlaps an input");
  return launch_self_energy(c, GR, WR, S, prec, (hipStream_t)stream);
}

gw_status gw_density(const gw_cell* c, const void* G, gw_dtype t, int space, double g, double* n_dev,
                     void* stream) {
  gw_status st = check_cell(c);
  if (st != GW_OK) return st;
  if (!G || !n_dev) return fail(GW_ERR_ARG, "NULL pointer");
  if (!valid_dtype(t)) return fail(GW_ERR_ARG, "bad dtype");
  if (space != 0 && space != 1) return fail(GW_ERR_ARG, "space must be 0 (R) or 1 (k)");
  if (!std::isfinite(g)) return fail(GW_ERR_ARG, "spin factor must be finite");
  return launch_density(c, G, t, space, g, n_dev, (hipStream_t)stream);
}

// T[m][j] for exact integration of the piecewise-linear interpolant against exp(i w tau).
// Interval [t_j, t_j + h]: left weight h * phi1(i w h), right weight h * phi2(i w h) with
// phi1(z) = (e^z - 1 - z) / z^2 = sum_k z^k / (k+2)!,  phi2(z) = (e^z (z - 1) + 1) / z^2
// = sum_k (k+1) z^k / (k+2)!; the series is used for |z| < 1/2 to avoid cancellation.
gw_status gw_tau2omega_matrix(int n_tau, const double* tau, int n_omega, const double* omega, double* T) {
  if (!tau || !omega || !T) return fail(GW_ERR_ARG, "NULL pointer");
  if (n_tau < 2 || n_omega < 1) return fail(GW_ERR_SHAPE, "need n_tau >= 2 and n_omega >= 1");
  for (int j = 0; j + 1 < n_tau; ++j)
    if (!(tau[j + 1] > tau[j])) return fail(GW_ERR_ARG, "tau must be strictly increasing");
  using cd = std::complex<double>;
  std::vector<cd> out((size_t)n_omega * n_tau, cd(0, 0));
  for (int m = 0; m < n_omega; ++m) {
    const double w = omega[m];
    for (int j = 0; j + 1 < n_tau; ++j) {
      const double h = tau[j + 1] - tau[j];
      const cd z(0.0, w * h);
      cd p1, p2;
      if (std::abs(z) < 0.5) {
        cd zk(1.0, 0.0);
        double fact = 2.0;  // (k+2)!
        p1 = p2 = cd(0, 0);
        for (int k = 0; k < 24; ++k) {
          p1 += zk / fact;
          p2 += zk * (double)(k + 1) / fact;
          zk *= z;
          fact *= (double)(k + 3);
        }
      } else {
        const cd ez = std::exp(z);
        p1 = (ez - 1.0 - z) / (z * z);
        p2 = (ez * (z - 1.0) + 1.0) / (z * z);
      }
      const cd ph = std::exp(cd(0.0, w * tau[j]));
      out[(size_t)m * n_tau + j] += ph * h * p1;
      out[(size_t)m * n_tau + j + 1] += ph * h * p2;
    }
  }
  std::memcpy(T, out.data(), out.size() * sizeof(cd));
  return GW_OK;
}

}  // extern "C"

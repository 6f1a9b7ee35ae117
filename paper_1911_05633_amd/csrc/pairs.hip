// Real-space cutoff and distance tiers of the product basis (Sec. 2, Figs. 1 and 2):
// the planner of the kept (R, A, B) blocks and the contractions over them.
//
// A block (R, A, B) couples atom A in cell R with atom B in cell 0.  The distance between
// the two centres is d = |R' a + r_A - r_B| for the lattice vector R' of R (R' equal to R
// modulo the mesh) that minimises it; the block is kept when d <= r_c and is zero
// otherwise.  The mesh must be fine enough that no second image of a pair lies inside the
// sphere.  A kept block uses all product functions of both atoms when A = B in the same
// cell, the first m_B of each atom when 0 < d <= r_b and the first m_C when r_b < d <= r_c.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace gwr;

namespace {

template <class T>
gw_status upload_owned(gw_cell* c, T** dst, const T* src, size_t n) {
  *dst = nullptr;
  if (n == 0) return GW_OK;
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return fail(GW_ERR_NOMEM, "hipMalloc failed for the pair list");
  c->owned.push_back(p);
  if (hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(GW_ERR_HIP, "hipMemcpy failed for the pair list");
  *dst = static_cast<T*>(p);
  return GW_OK;
}

gw_status cell_on_device(const gw_cell* c) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  return GW_OK;
}

// GWR_KERNELS=generic selects the plain kernels, as for the dense entry points
bool force_generic() {
  const char* v = std::getenv("GWR_KERNELS");
  return v && std::strcmp(v, "generic") == 0;
}

double norm3(const double* v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace

extern "C" {

gw_status gw_cell_set_pairs(gw_cell* c, const double* lattice, const double* positions, double r_b, double r_c,
                            const int* m_tier) {
  gw_status st = cell_on_device(c);
  if (st != GW_OK) return st;
  if (!lattice || !positions || !m_tier) return fail(GW_ERR_ARG, "NULL input array");
  if (!std::isfinite(r_b) || !std::isfinite(r_c) || r_b < 0 || r_c < r_b)
    return fail(GW_ERR_ARG, "need 0 <= r_b <= r_c, both finite");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(lattice[i])) return fail(GW_ERR_ARG, "lattice has a non-finite entry");
  for (int i = 0; i < 3 * c->n_atoms; ++i)
    if (!std::isfinite(positions[i])) return fail(GW_ERR_ARG, "positions have a non-finite entry");
  for (int s = 0; s < c->n_species; ++s)
    for (int t = 0; t < 2; ++t)
      if (m_tier[2 * s + t] < 1 || m_tier[2 * s + t] > c->n_pb[s] || m_tier[2 * s + t] > 0xffff)
        return fail(GW_ERR_ARG, "m_tier entries must be in [1, n_pb of the species]");
  const double* a = lattice;
  double vol;
  {
    double x[3];
    cross3(a + 3, a + 6, x);
    vol = std::fabs(a[0] * x[0] + a[1] * x[1] + a[2] * x[2]);
  }
  if (!(vol > 0)) return fail(GW_ERR_ARG, "lattice vectors are linearly dependent");
  // image search range: the Born-von Karman supercell has plane spacings N_i h_i, with h_i
  // the spacing of the lattice planes spanned by the other two vectors; images of a pair
  // within r_c differ from the nearest one by at most 2 r_c + the cell diameter
  double diam = 0;
  for (int A = 0; A < c->n_atoms; ++A)
    for (int B = 0; B < c->n_atoms; ++B) {
      double v[3];
      for (int i = 0; i < 3; ++i) v[i] = positions[3 * A + i] - positions[3 * B + i];
      diam = std::fmax(diam, norm3(v));
    }
  int K[3];
  for (int i = 0; i < 3; ++i) {
    double x[3];
    cross3(a + 3 * ((i + 1) % 3), a + 3 * ((i + 2) % 3), x);
    const double h = vol / norm3(x);
    K[i] = (int)std::ceil((r_c + diam) / (c->mesh[i] * h)) + 1;
  }
  std::vector<int> host;
  std::vector<std::vector<int4>> groups((size_t)c->n_species * c->n_species);
  std::vector<std::vector<int4>> groups2((size_t)c->n_species * c->n_species);
  std::vector<int> index_in_species(c->n_atoms, 0);
  for (int s = 0; s < c->n_species; ++s)
    for (size_t i = 0; i < c->sp[s].atoms.size(); ++i) index_in_species[c->sp[s].atoms[i]] = (int)i;
  for (int n1 = 0; n1 < c->mesh[0]; ++n1)
    for (int n2 = 0; n2 < c->mesh[1]; ++n2)
      for (int n3 = 0; n3 < c->mesh[2]; ++n3) {
        const int R = (n1 * c->mesh[1] + n2) * c->mesh[2] + n3;
        for (int A = 0; A < c->n_atoms; ++A)
          for (int B = 0; B < c->n_atoms; ++B) {
            double best = INFINITY;
            int inside = 0;
            for (int k1 = -K[0]; k1 <= K[0]; ++k1)
              for (int k2 = -K[1]; k2 <= K[1]; ++k2)
                for (int k3 = -K[2]; k3 <= K[2]; ++k3) {
                  const double l1 = n1 + (double)k1 * c->mesh[0], l2 = n2 + (double)k2 * c->mesh[1],
                               l3 = n3 + (double)k3 * c->mesh[2];
                  double v[3];
                  for (int i = 0; i < 3; ++i)
                    v[i] = l1 * a[i] + l2 * a[3 + i] + l3 * a[6 + i] + positions[3 * A + i] - positions[3 * B + i];
                  const double d = norm3(v);
                  if (d <= r_c) ++inside;
                  best = std::fmin(best, d);
                }
            if (inside > 1)
              return fail(GW_ERR_ARG,
                          "the mesh is too coarse for r_c: a pair has two periodic images inside the sphere");
            if (!(best <= r_c)) continue;
            const int sA = c->species[A], sB = c->species[B];
            int mA, mB;
            if (A == B && R == 0) {
              mA = c->n_pb[sA];
              mB = c->n_pb[sB];
            } else if (best <= r_b) {
              mA = m_tier[2 * sA];
              mB = m_tier[2 * sB];
            } else {
              mA = m_tier[2 * sA + 1];
              mB = m_tier[2 * sB + 1];
            }
            host.insert(host.end(), {R, A, B, mA, mB});
          }
      }
  // Packed layout of the kept blocks, in list order: block b at offset off[b] of a tau slice,
  // its mA x mB functions row-major.  The mirror (-R, B, A) of every kept block is kept.
  const long long nkept = (long long)host.size() / 5;
  std::vector<long long> off(nkept + 1, 0);
  std::vector<int> where((size_t)c->N_R * c->n_atoms * c->n_atoms, -1);
  for (long long b = 0; b < nkept; ++b) {
    const int* e = &host[(size_t)5 * b];
    off[b + 1] = off[b] + (long long)e[3] * e[4];
    where[((size_t)e[0] * c->n_atoms + e[1]) * c->n_atoms + e[2]] = (int)b;
  }
  if (off[nkept] > 0x7fffffffLL) return fail(GW_ERR_SHAPE, "packed slice above 2^31 elements");
  std::vector<int4> blocks;                       // per kept block: (R, mA | mB << 16, pA, pB), (off, 0, 0, 0)
  std::vector<int> ab_ptr((size_t)c->n_atoms * c->n_atoms + 1, 0);
  std::vector<int4> ab_items;                     // per (A, B), its kept blocks: (R, mA | mB << 16, off, 0)
  for (long long b = 0; b < nkept; ++b) {
    const int* e = &host[(size_t)5 * b];
    const int R = e[0], A = e[1], B = e[2], mA = e[3], mB = e[4];
    const int sA = c->species[A], sB = c->species[B];
    const int mirror = where[((size_t)c->minusR[R] * c->n_atoms + B) * c->n_atoms + A];
    if (mirror < 0) return fail(GW_ERR_HIP, "pair list is not closed under (R, A, B) -> (-R, B, A)");
    groups[(size_t)sA * c->n_species + sB].push_back(
        make_int4(R, index_in_species[A], index_in_species[B], mA | (mB << 16)));
    auto& g2 = groups2[(size_t)sA * c->n_species + sB];
    g2.push_back(make_int4(R, mA | (mB << 16), c->pb_off[A], c->orb_off[A]));
    g2.push_back(make_int4(c->pb_off[B], c->orb_off[B], (int)off[b], (int)off[mirror]));
    blocks.push_back(make_int4(R, mA | (mB << 16), c->pb_off[A], c->pb_off[B]));
    blocks.push_back(make_int4((int)off[b], 0, 0, 0));
    ++ab_ptr[(size_t)A * c->n_atoms + B + 1];
  }
  for (size_t i = 1; i < ab_ptr.size(); ++i) ab_ptr[i] += ab_ptr[i - 1];
  ab_items.resize(nkept > 0 ? nkept : 0);
  {
    std::vector<int> fill(ab_ptr.begin(), ab_ptr.end() - 1);
    for (long long b = 0; b < nkept; ++b) {
      const int* e = &host[(size_t)5 * b];
      ab_items[fill[(size_t)e[1] * c->n_atoms + e[2]]++] = make_int4(e[0], e[3] | (e[4] << 16), (int)off[b], 0);
    }
  }
  std::vector<int4*> dev(groups.size(), nullptr), dev2(groups.size(), nullptr);
  std::vector<int> cnt(groups.size(), 0);
  for (size_t g = 0; g < groups.size(); ++g) {
    cnt[g] = (int)groups[g].size();
    st = upload_owned(c, &dev[g], groups[g].data(), groups[g].size());
    if (st != GW_OK) return st;
    st = upload_owned(c, &dev2[g], groups2[g].data(), groups2[g].size());
    if (st != GW_OK) return st;
  }
  int4 *blocks_dev = nullptr, *items_dev = nullptr;
  int* ptr_dev = nullptr;
  if ((st = upload_owned(c, &blocks_dev, blocks.data(), blocks.size())) != GW_OK) return st;
  if ((st = upload_owned(c, &items_dev, ab_items.data(), ab_items.size())) != GW_OK) return st;
  if ((st = upload_owned(c, &ptr_dev, ab_ptr.data(), ab_ptr.size())) != GW_OK) return st;
  c->pair_list.swap(host);
  c->pair_dev.swap(dev);
  c->pair_dev_mfma.swap(dev2);
  c->pair_cnt.swap(cnt);
  c->packed_per_tau = off[nkept];
  c->packed_blocks_dev = blocks_dev;
  c->packed_ab_items_dev = items_dev;
  c->packed_ab_ptr_dev = ptr_dev;
  c->pairs_set = true;
  return GW_OK;
}

gw_status gw_cell_pairs(const gw_cell* c, long long* n_pairs, int* pairs, long long capacity) {
  if (!c || !n_pairs) return fail(GW_ERR_ARG, "NULL argument");
  if (!c->pairs_set) return fail(GW_ERR_ARG, "no pair list: call gw_cell_set_pairs first");
  const long long n = (long long)c->pair_list.size() / 5;
  *n_pairs = n;
  if (pairs) {
    if (capacity < 0) return fail(GW_ERR_ARG, "capacity must be >= 0");
    const long long k = n < capacity ? n : capacity;
    for (long long i = 0; i < 5 * k; ++i) pairs[i] = c->pair_list[(size_t)i];
  }
  return GW_OK;
}

static gw_status pairs_common(const gw_cell* c, gw_precision prec) {
  gw_status st = cell_on_device(c);
  if (st != GW_OK) return st;
  if (!c->pairs_set) return fail(GW_ERR_ARG, "no pair list: call gw_cell_set_pairs first");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  return GW_OK;
}

gw_status gw_polarizability_pairs(const gw_cell* c, const void* GR, void* P, double g, gw_precision prec,
                                  void* stream) {
  gw_status st = pairs_common(c, prec);
  if (st != GW_OK) return st;
  if (!GR || !P) return fail(GW_ERR_ARG, "NULL tensor");
  if (!std::isfinite(g)) return fail(GW_ERR_ARG, "spin factor must be finite");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const size_t ng = (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb, np = (size_t)c->n_tau * c->N_R * c->N_pb * c->N_pb;
  const auto x = reinterpret_cast<uintptr_t>(GR), y = reinterpret_cast<uintptr_t>(P);
  if (x < y + np * es && y < x + ng * es) return fail(GW_ERR_ARG, "GR and P overlap");
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const size_t gi = (size_t)sa * c->n_species + sb;
      const SpeciesDev &A = c->sp[sa], &B = c->sp[sb];
      if (c->pair_cnt[gi] == 0) continue;
      if (!force_generic() && mfma_pair_ok(A, B) && mfma_pair_ok(B, A))
        launch_p_mfma_list(c, A, B, c->pair_dev_mfma[gi], c->pair_cnt[gi], GR, P, g, prec, (hipStream_t)stream);
      else
        launch_p_generic_list(c, A, B, c->pair_dev[gi], c->pair_cnt[gi], GR, P, g, prec, (hipStream_t)stream);
    }
  return check_launch("polarizability over the pair list");
}

gw_status gw_self_energy_pairs(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision prec,
                               void* stream) {
  gw_status st = pairs_common(c, prec);
  if (st != GW_OK) return st;
  if (!GR || !WR || !S) return fail(GW_ERR_ARG, "NULL tensor");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const size_t ng = (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb, nw = (size_t)c->n_tau * c->N_R * c->N_pb * c->N_pb;
  const auto s0 = reinterpret_cast<uintptr_t>(S), g0 = reinterpret_cast<uintptr_t>(GR),
             w0 = reinterpret_cast<uintptr_t>(WR);
  if ((g0 < s0 + ng * 16 && s0 < g0 + ng * es) || (w0 < s0 + ng * 16 && s0 < w0 + nw * es))
    return fail(GW_ERR_ARG, "Sigma overlaps an input");
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const size_t gi = (size_t)sa * c->n_species + sb;
      const SpeciesDev &A = c->sp[sa], &B = c->sp[sb];
      if (c->pair_cnt[gi] == 0) continue;
      if (force_generic() || !mfma_pair_ok(A, B) ||
          !launch_s_mfma_list(c, A, B, c->pair_dev_mfma[gi], c->pair_cnt[gi], GR, WR, S, prec, (hipStream_t)stream))
        launch_s_generic_list(c, A, B, c->pair_dev[gi], c->pair_cnt[gi], GR, WR, S, prec, (hipStream_t)stream);
    }
  return check_launch("self-energy over the pair list");
}

}  // extern "C"

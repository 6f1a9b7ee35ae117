// Packed storage of the real-space cutoff path (Sec. 2, Figs. 1 and 2: two-point functions kept
// only for pairs within R_max, each in the product basis of its distance tier).
//
// A tau slice of a packed tensor holds the kept (R, A, B) blocks one after the other, in the
// order of the cell's list, each as its mA x mB kept functions row-major: sum_b mA_b mB_b
// elements per slice instead of N_R N_pb^2.  The contractions write P and read W in this layout
// (the general matrix-core kernels with the packed offsets in their block list); the lattice sums
// go between it and the dense k-space layout that the Dyson steps need:
//   r2k: out[t][q][pA + I][pB + J] = sum over kept (R, A, B) of exp(-i q.R) F_(R,A,B)(t)[I][J]
//        (zero where no kept block has the function pair);
//   k2r: F_(R,A,B)(t)[I][J] = N_k^-1 sum_q exp(+i q.R) in[t][q][pA + I][pB + J].
#include <cmath>

#include "cplx.h"
#include "internal.h"

namespace gwr {

void launch_p_mfma_packed(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                          long long ptot, const void* GR, void* P, double g, gw_precision p, hipStream_t s);
void launch_s_mfma_packed(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                          long long ptot, const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s);

namespace {

constexpr int kQC = 16;  // k points per pass of a thread

// one thread per function pair (I, J) of the (A, B) block at one tau, every k
template <class TI, class TO>
__global__ __launch_bounds__(256) void r2k_packed(const TI* __restrict__ in, TO* __restrict__ out,
                                                  const int* __restrict__ ab_ptr, const int4* __restrict__ items,
                                                  const double2* __restrict__ ph, const int* __restrict__ pb_off,
                                                  int n_atoms, int NR, int Np, long long ptot) {
  const int A = blockIdx.y / n_atoms, B = blockIdx.y - A * n_atoms, t = blockIdx.z;
  const int pA = pb_off[A], pB = pb_off[B], mAf = pb_off[A + 1] - pA, mBf = pb_off[B + 1] - pB;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= mAf * mBf) return;
  const int I = e / mBf, J = e - I * mBf;
  const int i0 = ab_ptr[blockIdx.y], i1 = ab_ptr[blockIdx.y + 1];
  const TI* src = in + (long long)t * ptot;
  for (int q0 = 0; q0 < NR; q0 += kQC) {
    double ar[kQC], ai[kQC];
#pragma unroll
    for (int u = 0; u < kQC; ++u) ar[u] = ai[u] = 0.0;
    for (int it = i0; it < i1; ++it) {
      const int4 b = items[it];
      const int mA = b.y & 0xffff, mB = b.y >> 16;
      if (I >= mA || J >= mB) continue;
      double vr, vi;
      ldc(src + b.z + (long long)I * mB + J, vr, vi);
#pragma unroll
      for (int u = 0; u < kQC; ++u)
        if (q0 + u < NR) {
          const double2 p = ph[(long long)(q0 + u) * NR + b.x];  // exp(+i q.R); the sum takes its conjugate
          ar[u] += p.x * vr + p.y * vi;
          ai[u] += p.x * vi - p.y * vr;
        }
    }
#pragma unroll
    for (int u = 0; u < kQC; ++u)
      if (q0 + u < NR) stc(out + (((long long)t * NR + q0 + u) * Np + pA + I) * Np + pB + J, ar[u], ai[u]);
  }
}

// one thread per kept function pair (I, J) of a kept block at one tau
template <class TI, class TO>
__global__ __launch_bounds__(256) void k2r_packed(const TI* __restrict__ in, TO* __restrict__ out,
                                                  const int4* __restrict__ blocks, const double2* __restrict__ ph,
                                                  int NR, int Np, long long ptot) {
  const int4 b = blocks[2 * blockIdx.y];
  const int off = blocks[2 * blockIdx.y + 1].x, t = blockIdx.z;
  const int mA = b.y & 0xffff, mB = b.y >> 16;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= mA * mB) return;
  const int I = e / mB, J = e - I * mB;
  double ar = 0.0, ai = 0.0;
  for (int q = 0; q < NR; ++q) {
    double vr, vi;
    ldc(in + (((long long)t * NR + q) * Np + b.z + I) * Np + b.w + J, vr, vi);
    const double2 p = ph[(long long)q * NR + b.x];
    ar += p.x * vr - p.y * vi;
    ai += p.x * vi + p.y * vr;
  }
  stc(out + (long long)t * ptot + off + e, ar / NR, ai / NR);
}

gw_status packed_common(const gw_cell* c) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!c->pairs_set) return fail(GW_ERR_ARG, "no pair list: call gw_cell_set_pairs first");
  return GW_OK;
}

bool overlapping(const void* a, size_t na, const void* b, size_t nb) {
  auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

int max_pb(const gw_cell* c) {
  int m = 0;
  for (int s = 0; s < c->n_species; ++s) m = m > c->n_pb[s] ? m : c->n_pb[s];
  return m;
}

template <class TI, class TO>
void r2k_launch(const gw_cell* c, const void* in, void* out, hipStream_t s) {
  const int mm = max_pb(c);
  const dim3 grid((unsigned)((mm * mm + 255) / 256), (unsigned)(c->n_atoms * c->n_atoms), (unsigned)c->n_tau);
  hipLaunchKernelGGL((r2k_packed<TI, TO>), grid, dim3(256), 0, s, (const TI*)in, (TO*)out, c->packed_ab_ptr_dev,
                     c->packed_ab_items_dev, c->kr_phase_dev, c->pb_off_dev, c->n_atoms, c->N_R, c->N_pb,
                     c->packed_per_tau);
}

template <class TI, class TO>
void k2r_launch(const gw_cell* c, const void* in, void* out, hipStream_t s) {
  const int mm = max_pb(c);
  const long long nk = (long long)c->pair_list.size() / 5;
  if (nk == 0) return;  // no kept block: nothing to write
  const dim3 grid((unsigned)((mm * mm + 255) / 256), (unsigned)nk, (unsigned)c->n_tau);
  hipLaunchKernelGGL((k2r_packed<TI, TO>), grid, dim3(256), 0, s, (const TI*)in, (TO*)out, c->packed_blocks_dev,
                     c->kr_phase_dev, c->N_R, c->N_pb, c->packed_per_tau);
}

gw_status lattice_packed(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot, bool to_k,
                         hipStream_t s) {
  if (!in || !out) return fail(GW_ERR_ARG, "NULL tensor");
  if ((it != GW_C128 && it != GW_C64) || (ot != GW_C128 && ot != GW_C64)) return fail(GW_ERR_ARG, "bad dtype");
  const long long nk = (long long)c->pair_list.size() / 5;
  if (c->n_tau > 65535 || (long long)c->n_atoms * c->n_atoms > 65535 || nk > 65535)
    return fail(GW_ERR_SHAPE, "more than 65535 atom pairs, kept blocks or time points");
  const size_t npk = (size_t)c->n_tau * c->packed_per_tau, nd = (size_t)c->n_tau * c->N_R * c->N_pb * c->N_pb;
  if (overlapping(in, (to_k ? npk : nd) * csize(it), out, (to_k ? nd : npk) * csize(ot)))
    return fail(GW_ERR_ARG, "in and out overlap");
#define GWR_PK(TI, TO)                 \
  do {                                 \
    if (to_k)                          \
      r2k_launch<TI, TO>(c, in, out, s); \
    else                               \
      k2r_launch<TI, TO>(c, in, out, s); \
  } while (0)
  if (it == GW_C128 && ot == GW_C128)
    GWR_PK(double2, double2);
  else if (it == GW_C128)
    GWR_PK(double2, float2);
  else if (ot == GW_C128)
    GWR_PK(float2, double2);
  else
    GWR_PK(float2, float2);
#undef GWR_PK
  return check_launch(to_k ? "R -> k of a packed tensor" : "k -> R into a packed tensor");
}

}  // namespace
}  // namespace gwr

using namespace gwr;

extern "C" {

gw_status gw_cell_packed_size(const gw_cell* c, long long* per_tau) {
  if (!c || !per_tau) return fail(GW_ERR_ARG, "NULL argument");
  if (!c->pairs_set) return fail(GW_ERR_ARG, "no pair list: call gw_cell_set_pairs first");
  *per_tau = c->packed_per_tau;
  return GW_OK;
}

gw_status gw_polarizability_packed(const gw_cell* c, const void* GR, void* P, double g, gw_precision prec,
                                   void* stream) {
  gw_status st = packed_common(c);
  if (st != GW_OK) return st;
  if (!GR || !P) return fail(GW_ERR_ARG, "NULL tensor");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  if (!std::isfinite(g)) return fail(GW_ERR_ARG, "spin factor must be finite");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  if (overlapping(GR, (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb * es, P,
                  (size_t)c->n_tau * c->packed_per_tau * es))
    return fail(GW_ERR_ARG, "GR and P overlap");
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const size_t gi = (size_t)sa * c->n_species + sb;
      if (c->pair_cnt[gi] == 0) continue;
      launch_p_mfma_packed(c, c->sp[sa], c->sp[sb], c->pair_dev_mfma[gi], c->pair_cnt[gi], c->packed_per_tau, GR,
                           P, g, prec, (hipStream_t)stream);
    }
  return check_launch("polarizability, packed");
}

gw_status gw_self_energy_packed(const gw_cell* c, const void* GR, const void* WR, void* S, gw_precision prec,
                                void* stream) {
  gw_status st = packed_common(c);
  if (st != GW_OK) return st;
  if (!GR || !WR || !S) return fail(GW_ERR_ARG, "NULL tensor");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const size_t ng = (size_t)c->n_tau * c->N_R * c->N_orb * c->N_orb, nw = (size_t)c->n_tau * c->packed_per_tau;
  if (overlapping(S, ng * 16, GR, ng * es) || overlapping(S, ng * 16, WR, nw * es))
    return fail(GW_ERR_ARG, "Sigma overlaps an input");
  for (int sa = 0; sa < c->n_species; ++sa)
    for (int sb = 0; sb < c->n_species; ++sb) {
      const size_t gi = (size_t)sa * c->n_species + sb;
      if (c->pair_cnt[gi] == 0) continue;
      launch_s_mfma_packed(c, c->sp[sa], c->sp[sb], c->pair_dev_mfma[gi], c->pair_cnt[gi], c->packed_per_tau, GR,
                           WR, S, prec, (hipStream_t)stream);
    }
  return check_launch("self-energy, packed");
}

gw_status gw_fourier_r2k_packed(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot,
                                void* stream) {
  gw_status st = packed_common(c);
  if (st != GW_OK) return st;
  return lattice_packed(c, in, it, out, ot, true, (hipStream_t)stream);
}

gw_status gw_fourier_k2r_packed(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot,
                                void* stream) {
  gw_status st = packed_common(c);
  if (st != GW_OK) return st;
  return lattice_packed(c, in, it, out, ot, false, (hipStream_t)stream);
}

gw_status gw_drain_packed(const gw_cell* c, const void* T, int n_omega, int parity, const void* in, gw_dtype it,
                          void* out, gw_dtype ot, void* stream) {
  gw_status st = packed_common(c);
  if (st != GW_OK) return st;
  if (!T) return fail(GW_ERR_ARG, "NULL tensor");
  if (parity < -1 || parity > 1) return fail(GW_ERR_ARG, "parity must be -1, 0 or +1");
  if (n_omega < 1 || n_omega > 256) return fail(GW_ERR_SHAPE, "n_omega must be in [1, 256]");
  st = lattice_packed(c, in, it, out, ot, true, (hipStream_t)stream);
  if (st != GW_OK) return st;
  return launch_tau2omega(c, T, n_omega, parity, out, ot, out, ot, (long long)c->N_R * c->N_pb * c->N_pb,
                          (hipStream_t)stream);
}

}  // extern "C"

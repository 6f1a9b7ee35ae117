// Plain LDS-tiled VALU kernels for Eqs. (5) and (8), any block shape within the
// cell limits (n <= 16, m <= 128).  One workgroup per (tau, R, A, B) block.
// They serve shapes the MFMA kernels do not cover and are the reference the
// MFMA kernels are checked against on the GPU.
//
//   P:      V^I_ad = sum_b C^I_ab Y_db,  U^I_cd = sum_a X_ac V^I_ad,
//           P_IJ = -g sum_cd U^I_cd C^J_cd
//           (X = G^R(tau)[A, B], Y = G^{-R}(beta - tau)[B, A])
//   Sigma:  Z^I_bb' = sum_J W_IJ C^J_bb',  T^I_a'b = sum_b' X_a'b' Z^I_bb',
//           Sigma_ab = -sum_{I, a'} C^I_aa' T^I_a'b
//           (X = G^R(tau)[A, B], W = W^R(tau)[A, B])
#include "cplx.h"
#include "internal.h"

namespace gwr {
namespace {

constexpr int kIch = 4;  // product functions per LDS chunk

struct BlockIdx {
  int t, R, A, B;
  int mA, mB;  // product functions kept on each side (all of them without a block list)
};

// Block b of the launch: every (t, R, iA, iB) in order, or, with a block list, (t, list
// entry) with the entry (R, iA, iB, mA | mB << 16) of the real-space cutoff.
__device__ __forceinline__ BlockIdx decode(long long b, int NR, int nA, int nB, const int* atomsA,
                                           const int* atomsB, const int4* list, int nlist, int mA, int mB) {
  BlockIdx o;
  if (list) {
    const int4 e = list[b % nlist];
    o.t = (int)(b / nlist);
    o.R = e.x;
    o.A = atomsA[e.y];
    o.B = atomsB[e.z];
    o.mA = e.w & 0xffff;
    o.mB = e.w >> 16;
    return o;
  }
  const int iB = (int)(b % nB);
  b /= nB;
  const int iA = (int)(b % nA);
  b /= nA;
  o.R = (int)(b % NR);
  o.t = (int)(b / NR);
  o.A = atomsA[iA];
  o.B = atomsB[iB];
  o.mA = mA;
  o.mB = mB;
  return o;
}

template <class CT, class RT>
__global__ __launch_bounds__(256) void p_generic(const CT* __restrict__ GR, CT* __restrict__ P,
                                                 const RT* __restrict__ CA, const RT* __restrict__ CB, int nA,
                                                 int mA, int nB, int mB, const int* atomsA, int cntA,
                                                 const int* atomsB, int cntB, const int* orb_off,
                                                 const int* pb_off, const int* minusR, int NR, int n_tau, int No,
                                                 int Np, double g, const int4* list, int nlist) {
  __shared__ double2 X[kMaxOrb * kMaxOrb], Y[kMaxOrb * kMaxOrb];
  __shared__ double2 V[kIch * kMaxOrb * kMaxOrb], U[kIch * kMaxOrb * kMaxOrb];
  const BlockIdx bi = decode(blockIdx.x, NR, cntA, cntB, atomsA, atomsB, list, nlist, mA, mB);
  const int tm = n_tau - 1 - bi.t, mR = minusR[bi.R];
  const int oA = orb_off[bi.A], oB = orb_off[bi.B], pA = pb_off[bi.A], pB = pb_off[bi.B];
  const long long sl = (long long)No * No;
  const CT* Gt = GR + ((long long)bi.t * NR + bi.R) * sl;
  const CT* Gm = GR + ((long long)tm * NR + mR) * sl;
  for (int i = threadIdx.x; i < nA * nB; i += 256) {
    const int a = i / nB, c = i % nB;
    double re, im;
    ldc(Gt + (long long)(oA + a) * No + oB + c, re, im);
    X[a * nB + c] = make_double2(re, im);
  }
  for (int i = threadIdx.x; i < nB * nA; i += 256) {
    const int d = i / nA, b = i % nA;
    double re, im;
    ldc(Gm + (long long)(oB + d) * No + oA + b, re, im);
    Y[d * nA + b] = make_double2(re, im);
  }
  __syncthreads();
  CT* Pblk = P + ((long long)bi.t * NR + bi.R) * Np * Np;
  for (int I0 = 0; I0 < mA; I0 += kIch) {
    const int ni = min(kIch, mA - I0);
    const int nc = max(0, min(ni, bi.mA - I0));  // rows of this chunk inside the block's basis
    // V^I_ad
    for (int i = threadIdx.x; i < nc * nA * nB; i += 256) {
      const int il = i / (nA * nB), r = i % (nA * nB), a = r / nB, d = r % nB;
      const RT* Ci = CA + (long long)(I0 + il) * nA * nA + a * nA;
      double sr = 0, si = 0;
      for (int b = 0; b < nA; ++b) {
        const double2 y = Y[d * nA + b];
        sr += (double)Ci[b] * y.x;
        si += (double)Ci[b] * y.y;
      }
      V[il * nA * nB + a * nB + d] = make_double2(sr, si);
    }
    __syncthreads();
    // U^I_cd
    for (int i = threadIdx.x; i < nc * nB * nB; i += 256) {
      const int il = i / (nB * nB), r = i % (nB * nB), c = r / nB, d = r % nB;
      double sr = 0, si = 0;
      for (int a = 0; a < nA; ++a) {
        const double2 x = X[a * nB + c], v = V[il * nA * nB + a * nB + d];
        sr += x.x * v.x - x.y * v.y;
        si += x.x * v.y + x.y * v.x;
      }
      U[il * nB * nB + c * nB + d] = make_double2(sr, si);
    }
    __syncthreads();
    // P_IJ; zero outside the block's basis
    for (int i = threadIdx.x; i < ni * mB; i += 256) {
      const int il = i / mB, J = i % mB;
      double sr = 0, si = 0;
      if (il < nc && J < bi.mB) {
        const RT* Cj = CB + (long long)J * nB * nB;
        for (int cd = 0; cd < nB * nB; ++cd) {
          const double2 u = U[il * nB * nB + cd];
          sr += u.x * (double)Cj[cd];
          si += u.y * (double)Cj[cd];
        }
      }
      stc(Pblk + (long long)(pA + I0 + il) * Np + pB + J, -g * sr, -g * si);
    }
    __syncthreads();
  }
}

template <class CT, class RT>
__global__ __launch_bounds__(256) void s_generic(const CT* __restrict__ GR, const CT* __restrict__ WR,
                                                 double2* __restrict__ S, const RT* __restrict__ CA,
                                                 const RT* __restrict__ CB, int nA, int mA, int nB, int mB,
                                                 const int* atomsA, int cntA, const int* atomsB, int cntB,
                                                 const int* orb_off, const int* pb_off, int NR, int No, int Np,
                                                 const int4* list, int nlist) {
  __shared__ double2 X[kMaxOrb * kMaxOrb];
  __shared__ double2 Z[kIch * kMaxOrb * kMaxOrb], Tt[kIch * kMaxOrb * kMaxOrb];
  const BlockIdx bi = decode(blockIdx.x, NR, cntA, cntB, atomsA, atomsB, list, nlist, mA, mB);
  const int oA = orb_off[bi.A], oB = orb_off[bi.B], pA = pb_off[bi.A], pB = pb_off[bi.B];
  const long long slG = (long long)No * No, slW = (long long)Np * Np;
  const CT* Gt = GR + ((long long)bi.t * NR + bi.R) * slG;
  const CT* Wt = WR + ((long long)bi.t * NR + bi.R) * slW;
  for (int i = threadIdx.x; i < nA * nB; i += 256) {
    const int a = i / nB, c = i % nB;
    double re, im;
    ldc(Gt + (long long)(oA + a) * No + oB + c, re, im);
    X[a * nB + c] = make_double2(re, im);
  }
  double accr = 0, acci = 0;  // Sigma_ab for (a, b) = threadIdx.x
  const int my_a = threadIdx.x / nB, my_b = threadIdx.x % nB;
  const bool owner = (int)threadIdx.x < nA * nB;
  __syncthreads();
  // W entries outside the block's basis (I >= mA, J >= mB of the cutoff tier) do not enter
  for (int I0 = 0; I0 < bi.mA; I0 += kIch) {
    const int ni = min(kIch, bi.mA - I0);
    for (int i = threadIdx.x; i < ni * nB * nB; i += 256) {
      const int il = i / (nB * nB), r = i % (nB * nB);
      const CT* Wrow = Wt + (long long)(pA + I0 + il) * Np + pB;
      double sr = 0, si = 0;
      for (int J = 0; J < bi.mB; ++J) {
        double wr, wi;
        ldc(Wrow + J, wr, wi);
        const double cj = (double)CB[(long long)J * nB * nB + r];
        sr += wr * cj;
        si += wi * cj;
      }
      Z[il * nB * nB + r] = make_double2(sr, si);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ni * nA * nB; i += 256) {
      const int il = i / (nA * nB), r = i % (nA * nB), ap = r / nB, b = r % nB;
      double sr = 0, si = 0;
      for (int bp = 0; bp < nB; ++bp) {
        const double2 x = X[ap * nB + bp], z = Z[il * nB * nB + b * nB + bp];
        sr += x.x * z.x - x.y * z.y;
        si += x.x * z.y + x.y * z.x;
      }
      Tt[il * nA * nB + ap * nB + b] = make_double2(sr, si);
    }
    __syncthreads();
    if (owner) {
      for (int il = 0; il < ni; ++il) {
        const RT* Ci = CA + (long long)(I0 + il) * nA * nA + my_a * nA;
        for (int ap = 0; ap < nA; ++ap) {
          const double2 tv = Tt[il * nA * nB + ap * nB + my_b];
          accr += (double)Ci[ap] * tv.x;
          acci += (double)Ci[ap] * tv.y;
        }
      }
    }
    __syncthreads();
  }
  if (owner) {
    double2* Sblk = S + ((long long)bi.t * NR + bi.R) * slG;
    Sblk[(long long)(oA + my_a) * No + oB + my_b] = make_double2(-accr, -acci);
  }
}

}  // namespace

// Launch the generic kernels for one species pair, over every block or over a block list
// (list != nullptr: n entries, n_tau blocks each).
static void p_generic_launch(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                             const void* GR, void* P, double g, gw_precision p, hipStream_t s) {
  const long long blocks = list ? (long long)c->n_tau * n
                                : (long long)c->n_tau * c->N_R * A.atoms.size() * B.atoms.size();
  if (blocks == 0) return;
  if (p == GW_FP64)
    hipLaunchKernelGGL((p_generic<double2, double>), dim3((unsigned)blocks), dim3(256), 0, s, (const double2*)GR,
                       (double2*)P, A.C, B.C, A.n, A.m, B.n, B.m, A.atoms_dev, (int)A.atoms.size(), B.atoms_dev,
                       (int)B.atoms.size(), c->orb_off_dev, c->pb_off_dev, c->minusR_dev, c->N_R, c->n_tau,
                       c->N_orb, c->N_pb, g, list, n);
  else
    hipLaunchKernelGGL((p_generic<float2, float>), dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)GR,
                       (float2*)P, A.C32, B.C32, A.n, A.m, B.n, B.m, A.atoms_dev, (int)A.atoms.size(), B.atoms_dev,
                       (int)B.atoms.size(), c->orb_off_dev, c->pb_off_dev, c->minusR_dev, c->N_R, c->n_tau,
                       c->N_orb, c->N_pb, g, list, n);
}

static void s_generic_launch(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                             const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s, int nt) {
  const long long blocks = list ? (long long)nt * n : (long long)nt * c->N_R * A.atoms.size() * B.atoms.size();
  if (blocks == 0) return;
  if (p == GW_FP64)
    hipLaunchKernelGGL((s_generic<double2, double>), dim3((unsigned)blocks), dim3(256), 0, s, (const double2*)GR,
                       (const double2*)WR, (double2*)S, A.C, B.C, A.n, A.m, B.n, B.m, A.atoms_dev,
                       (int)A.atoms.size(), B.atoms_dev, (int)B.atoms.size(), c->orb_off_dev, c->pb_off_dev,
                       c->N_R, c->N_orb, c->N_pb, list, n);
  else
    hipLaunchKernelGGL((s_generic<float2, float>), dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.C32, B.C32, A.n, A.m, B.n, B.m, A.atoms_dev,
                       (int)A.atoms.size(), B.atoms_dev, (int)B.atoms.size(), c->orb_off_dev, c->pb_off_dev,
                       c->N_R, c->N_orb, c->N_pb, list, n);
}

void launch_p_generic_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                           double g, gw_precision p, hipStream_t s) {
  p_generic_launch(c, A, B, nullptr, 0, GR, P, g, p, s);
}

void launch_s_generic_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR,
                           const void* WR, void* S, gw_precision p, hipStream_t s, int nt) {
  s_generic_launch(c, A, B, nullptr, 0, GR, WR, S, p, s, nt);
}

void launch_p_generic_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                           const void* GR, void* P, double g, gw_precision p, hipStream_t s) {
  if (n > 0) p_generic_launch(c, A, B, list, n, GR, P, g, p, s);
}

void launch_s_generic_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                           const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s) {
  if (n > 0) s_generic_launch(c, A, B, list, n, GR, WR, S, p, s, c->n_tau);
}

}  // namespace gwr

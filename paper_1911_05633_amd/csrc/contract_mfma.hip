// Eqs. (5) and (8) on the matrix cores (FP64 16x16x4 and FP32 16x16x4 MFMA).
//
// Both contractions are rewritten over UNORDERED orbital pairs, using that every
// product-basis vertex C^I_ab is symmetric in (a, b): with p = {a, b} (45 pairs
// for 9 orbitals) and C~^I_p = C^I_ab,
//
//   P_IJ     = -g sum_{p, p'} C~^I_p Q_{p p'} C~^J_p'
//              Q_{{a,b},{c,d}} = sum over the distinct orderings (a1,b1) of {a,b}
//                                and (c1,d1) of {c,d} of X_{a1 c1} Y_{d1 b1},
//              X = G^R(tau)[A, B],  Y = G^{-R}(beta - tau)[B, A];
//   Sigma_ab = -sum_{a', b'} X_{a'b'} K_{{a,a'},{b,b'}},
//              K_{p, p'} = sum_I C~^I_p Z^I_p',  Z^I_p' = sum_J W_IJ C~^J_p',
//              X = G^R(tau)[A, B],  W = W^R(tau)[A, B].
//
// Each becomes two chained real GEMMs with K = 48 (P: H = C~_A Q, then H C~_B^T;
// Sigma: Z = W C~_B^T, then C~_A^T Z).  The D fragment of the first MFMA is
// used in place as the B operand of the second: register j of an FP64
// 16x16x4 D fragment holds rows g + 4j (g = lane / 16), exactly the k = g rows of
// a 4-deep K step, so the first product's M rows are permuted such that the four
// rows of a register share one (re | im) part and four consecutive pair indices.
//
// P additionally uses P^R_IJ(beta - tau) = P^{-R}_JI(tau) (symmetric C): only
// tau_i with i <= n_tau - 1 - i is evaluated and every block is written twice.
// Workgroups are persistent over (tau, R, A, B) blocks of one species pair and keep
// the C~ operands they reuse in registers.
#include "cplx.h"
#include "internal.h"

namespace gwr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class RT>
struct Mma;
template <>
struct Mma<double> {
  typedef d4 acc;
  typedef double2 cplx;
  static __device__ __forceinline__ d4 op(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // D fragment: register j of lane group g (= lane / 16) holds row g + 4 j
  static __device__ __forceinline__ int drow(int g, int j) { return g + 4 * j; }
  static __device__ __forceinline__ void split(int r, int& g, int& j) {
    g = r & 3;
    j = r >> 2;
  }
};
template <>
struct Mma<float> {
  typedef f4 acc;
  typedef float2 cplx;
  static __device__ __forceinline__ f4 op(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // D fragment: register j of lane group g holds row 4 g + j
  static __device__ __forceinline__ int drow(int g, int j) { return 4 * g + j; }
  static __device__ __forceinline__ void split(int r, int& g, int& j) {
    g = r >> 2;
    j = r & 3;
  }
};

constexpr int kPL = 48;       // padded pair count handled here (n <= 9)
constexpr int kKA = kPL / 4;  // K steps over pairs
constexpr int kMP = 64;       // padded product functions handled here (m <= 64)
constexpr int kJT = kMP / 16;
constexpr int kTS = 33;       // complex row stride of a wavefront's P output staging tile
constexpr int kKJ = kMP / 4;

template <class RT>
__device__ __forceinline__ typename Mma<RT>::cplx mk(double re, double im) {
  typename Mma<RT>::cplx v;
  v.x = (RT)re;
  v.y = (RT)im;
  return v;
}

__device__ __forceinline__ void pair_of(int p, int n, unsigned char& a, unsigned char& b) {
  int x = 0;
  while (p >= n - x) {
    p -= n - x;
    ++x;
  }
  a = (unsigned char)x;
  b = (unsigned char)(x + p);
}

__device__ __forceinline__ int pair_index(int a, int b, int n) {
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  return a * n - a * (a - 1) / 2 + (b - a);
}

struct PairArgs {
  int nA, nB, mA, mB, npA, npB, nppA, nppB, mpA, mpB;
  const int* atomsA;
  int cntA;
  const int* atomsB;
  int cntB;
  const int2* offsA;  // per atom of species A (B): (first product function, first orbital)
  const int2* offsB;
  const int* orb_off;
  const int* pb_off;
  const int* minusR;
  int NR, n_tau, n_half, No, Np;
  long long nblocks;
  // block list of the real-space cutoff (nullptr: every block): entry i is
  // list[2 i] = (R, mA | mB << 16, first product function of A, first orbital of A),
  // list[2 i + 1] = (first product function of B, first orbital of B, 0, 0)
  const int4* list;
  int nlist;
  long long ptot;  // packed layout: elements per tau slice (sum of mA mB over the kept blocks)
};

// Block walk shared by the kernels below.  Dense: every (tau, R, iA, iB) in counting order
// (iB fastest), atom offsets from the per-species tables.  LIST: every (tau, list entry),
// the entry index held in iA; R, the offsets and the kept product functions come from it.
struct Blk {
  int t, R, iA, iB;
  int2 oa, ob;  // (first product function, first orbital) of atoms A and B
  int mt;       // product functions kept on A and B, mA | mB << 16 (all of them when dense)
};

template <bool LIST>
__device__ __forceinline__ void blk_start(Blk& k, long long b, const PairArgs& q) {
  if constexpr (LIST) {
    k.t = (int)(b / q.nlist);
    k.iA = (int)(b - (long long)k.t * q.nlist);
    k.iB = 0;
    k.R = 0;
  } else {
    k.iB = (int)(b % q.cntB);
    b /= q.cntB;
    k.iA = (int)(b % q.cntA);
    b /= q.cntA;
    k.R = (int)(b % q.NR);
    k.t = (int)(b / q.NR);
  }
}

template <bool LIST>
__device__ __forceinline__ void blk_step(Blk& k, const PairArgs& q) {
  if constexpr (LIST) {
    if (++k.iA == q.nlist) {
      k.iA = 0;
      ++k.t;
    }
  } else {
    if (++k.iB == q.cntB) {
      k.iB = 0;
      if (++k.iA == q.cntA) {
        k.iA = 0;
        if (++k.R == q.NR) {
          k.R = 0;
          ++k.t;
        }
      }
    }
  }
}

template <bool LIST>
__device__ __forceinline__ void blk_fill(Blk& k, const PairArgs& q) {
  if constexpr (LIST) {
    const int4 e0 = q.list[2 * k.iA], e1 = q.list[2 * k.iA + 1];
    k.R = e0.x;
    k.mt = e0.y;
    k.oa = make_int2(e0.z, e0.w);
    k.ob = make_int2(e1.x, e1.y);
  } else {
    k.oa = q.offsA[k.iA < q.cntA ? k.iA : 0];
    k.ob = q.offsB[k.iB < q.cntB ? k.iB : 0];
    k.mt = q.mA | (q.mB << 16);
  }
}

// Dense walk of the polarizability kernels in bands: kPBand consecutive atoms of A for each
// atom of B, the A atom fastest, (tau, R) slowest.  Consecutive blocks of a band write the
// two halves of the 128-byte lines that their mirror-block rows share, a block apart, so that
// they mostly meet in L2 and reach HBM as whole lines (partial-line writes reach it far more
// slowly); in counting order (B fastest) those halves are written 72 blocks apart.
constexpr int kPBand = 4;
__device__ __forceinline__ int band_size(int iA, const PairArgs& q) {
  const int b0 = iA - iA % kPBand;
  return q.cntA - b0 < kPBand ? q.cntA - b0 : kPBand;
}
template <class BK>  // Blk or GBlk (their t, R, iA, iB)
__device__ __forceinline__ void bblk_start(BK& k, long long b, const PairArgs& q) {
  const long long per = (long long)q.cntA * q.cntB;
  const long long tr = b / per;
  const int r = (int)(b - tr * per);
  k.R = (int)(tr % q.NR);
  k.t = (int)(tr / q.NR);
  const int full = q.cntA / kPBand, rem = q.cntA - kPBand * full;
  if (r < full * kPBand * q.cntB) {
    const int band = r / (kPBand * q.cntB), r2 = r - band * kPBand * q.cntB;
    k.iB = r2 / kPBand;
    k.iA = kPBand * band + (r2 - kPBand * k.iB);
  } else {
    const int r2 = r - full * kPBand * q.cntB;
    k.iB = r2 / rem;
    k.iA = kPBand * full + (r2 - rem * k.iB);
  }
}
template <class BK>
__device__ __forceinline__ void bblk_step(BK& k, const PairArgs& q) {
  const int bs = band_size(k.iA, q), a = k.iA % kPBand;
  if (a + 1 < bs) {
    ++k.iA;
    return;
  }
  k.iA -= a;
  if (++k.iB == q.cntB) {
    k.iB = 0;
    k.iA += bs;
    if (k.iA == q.cntA) {
      k.iA = 0;
      if (++k.R == q.NR) {
        k.R = 0;
        ++k.t;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// polarizability
// ---------------------------------------------------------------------------
constexpr int kQS = 56;      // LDS row stride of Q (complex): 4 consecutive rows land 32 banks apart
constexpr int kQE = (kPL * kPL + 255) / 256;  // Q entries per thread
constexpr int kCS = kPL + 1; // LDS row stride of C~_B (real): 16 consecutive rows hit distinct banks

// SH selects compile-time tile counts (no per-MFMA guards): 1 = np_pad 48 / m_pad 64 on both
// atoms (9 orbitals, 49..64 product functions), 2 = np_pad 16 / m_pad 16; 0 = read from q.
template <class RT, class CT, int SH, bool LIST = false>
__global__ __launch_bounds__(256, 2) void p_mfma(const CT* __restrict__ GR, CT* __restrict__ P,
                                                 const RT* __restrict__ CpA, const RT* __restrict__ CpB,
                                                 const PairArgs q, double g) {
  using M = Mma<RT>;
  typedef typename M::cplx CR;
  __shared__ CR Xs[kMaxOrb * kMaxOrb], Ys[kMaxOrb * kMaxOrb];
  __shared__ CR Qs[kPL * kQS];
  __shared__ RT Cb[kMP * kCS];
  __shared__ __align__(16) float2 Ts[sizeof(RT) == 4 ? 4 * 16 * kTS : 1];  // FP32: [wavefront][I][J half]
  __shared__ unsigned char ta[kPL], tb[kPL], tc[kPL], td[kPL];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  if (tid < q.npA) pair_of(tid, q.nA, ta[tid], tb[tid]);
  if (tid < q.npB) pair_of(tid, q.nB, tc[tid], td[tid]);
  for (int i = tid; i < q.mpB * q.nppB; i += 256) {
    const int J = i / q.nppB, pp = i - J * q.nppB;
    Cb[J * kCS + pp] = CpB[i];
  }
  const int nKA = SH == 1 ? 12 : SH == 2 ? 4 : q.nppA / 4;
  const int nTB = SH == 1 ? 6 : SH == 2 ? 2 : q.nppB / 8;
  const int nJT = SH == 1 ? 4 : SH == 2 ? 1 : (q.mB + 15) / 16;
  const int nIT = SH == 1 ? 4 : SH == 2 ? 1 : q.mpA / 16;
  __syncthreads();  // pair tables staged
  // per-thread Q entries: packed (a, b, c, d) of p = {a, b} and p' = {c, d}, or all ones
  // outside the live pairs, and the LDS offset of the entry
  unsigned qpk[kQE];
  int qoff[kQE];
#pragma unroll
  for (int e = 0; e < kQE; ++e) {
    const int i = tid + 256 * e;
    const int p = i / q.nppB, pp = i - p * q.nppB;
    qoff[e] = p * kQS + pp;
    qpk[e] = (i < q.nppA * q.nppB && p < q.npA && pp < q.npB)
                 ? (unsigned)ta[p] | ((unsigned)tb[p] << 8) | ((unsigned)tc[pp] << 16) | ((unsigned)td[pp] << 24)
                 : 0xffffffffu;
  }
  // each wavefront owns at most one I tile (m_pad <= 64): its C~_A operands are loaded once
  RT b1[kKA];
#pragma unroll
  for (int ks = 0; ks < kKA; ++ks) b1[ks] = (w < nIT && ks < nKA) ? CpA[(16 * w + li) * q.nppA + 4 * ks + lk] : RT(0);
  int rg, rj;
  M::split(li, rg, rj);
  const int row_pp = 4 * (rj >> 1) + rg, row_part = rj & 1;
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  const RT* Qd = reinterpret_cast<const RT*>(Qs);
  // Blocks are walked in one contiguous range per workgroup; (tau, R, iA, iB) advance by
  // counting (B fastest) and the atom offsets come from the per-species (pb, orb) tables,
  // the entries of block b + 2 being loaded while block b is multiplied.
  __shared__ int mRs[kMaxR];
  for (int i = tid; i < q.NR; i += 256) mRs[i] = q.minusR[i];
  // the X and Y tiles of the next block are loaded into registers (one element per thread,
  // n_A n_B <= 81 < 256) while the current block is on the matrix cores
  CT xr, yr;  // kept in the storage type until stored to LDS (no wait at the load)
  const bool xok = tid < q.nA * q.nB;
  auto fetch = [&](const Blk& k) {
    const int a = tid / q.nB, c = tid - a * q.nB;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR, xok);
    const int d = tid / q.nA, bb = tid - d * q.nA;
    yr = ldraw(GR + ((long long)(q.n_tau - 1 - k.t) * q.NR + mRs[k.R]) * sl + (long long)(k.ob.y + d) * q.No +
                   k.oa.y + bb,
               GR, xok);
  };
  auto stage = [&]() {
    if (tid < q.nA * q.nB) {
      Xs[tid] = mk<RT>((double)xr.x, (double)xr.y);
      Ys[tid] = mk<RT>((double)yr.x, (double)yr.y);
    }
  };
  // Order per block: issue the G loads of the next block; form Q from this block's tiles;
  // barrier; matrix phase and stores; stage the next tiles into LDS (their loads were
  // issued a whole block earlier); barrier.
  const long long per = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per;
  const long long bend = bbeg + per < q.nblocks ? bbeg + per : q.nblocks;
  Blk cur;
  // dense: band walk; block list: its contiguous range
  auto adv = [&](Blk& x) {
    if constexpr (LIST)
      blk_step<true>(x, q);
    else
      bblk_step(x, q);
  };
  if constexpr (LIST)
    blk_start<true>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  else
    bblk_start(cur, bbeg < q.nblocks ? bbeg : 0, q);
  blk_fill<LIST>(cur, q);
  Blk nxt = cur, nn = cur;
  adv(nxt);
  blk_fill<LIST>(nxt, q);
  adv(nn);
  adv(nn);
  __syncthreads();  // minus-R table staged
  if (bbeg < bend) {
    fetch(cur);
    stage();
  }
  __syncthreads();

  for (long long blk = bbeg; blk < bend; ++blk) {
    const Blk k = cur;
    const int t = k.t, R = k.R;
    const int tm = q.n_tau - 1 - t, mR = mRs[R];
    const int pA = k.oa.x, pB = k.ob.x;
    const bool more = blk + 1 < bend;
    if (more) fetch(nxt);
    Blk nf = nn;
    blk_fill<LIST>(nf, q);
    // Q over unordered pairs (zero outside the live pairs); the pair tables of this
    // thread's entries are held in registers
#pragma unroll
    for (int e = 0; e < kQE; ++e) {
      const int i = tid + 256 * e;
      if (i < q.nppA * q.nppB) {
        RT qr = 0, qi = 0;
        const unsigned pk = qpk[e];
        if (pk != 0xffffffffu) {
          const int a = pk & 0xff, bq = (pk >> 8) & 0xff, c = (pk >> 16) & 0xff, d = pk >> 24;
          const int nB = q.nB, nA = q.nA;
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int c1 = s2 ? d : c, d1 = s2 ? c : d;
            if (s2 == 1 && c == d) break;
            CR x = Xs[a * nB + c1], y = Ys[d1 * nA + bq];
            qr += x.x * y.x - x.y * y.y;
            qi += x.x * y.y + x.y * y.x;
            if (a != bq) {
              x = Xs[bq * nB + c1];
              y = Ys[d1 * nA + a];
              qr += x.x * y.x - x.y * y.y;
              qi += x.x * y.y + x.y * y.x;
            }
          }
        }
        Qs[qoff[e]] = mk<RT>(qr, qi);
      }
    }
    __syncthreads();

    CT* Pd = P + ((long long)t * q.NR + R) * slp;
    CT* Pm = P + ((long long)tm * q.NR + mR) * slp;
    if (w < nIT) {
      const int it = w;
      typename M::acc acc2[kJT][2];
#pragma unroll
      for (int Jt = 0; Jt < kJT; ++Jt) acc2[Jt][0] = acc2[Jt][1] = typename M::acc{0, 0, 0, 0};
      // first product for tile tt: rows (p', part) of Q^T against C~_A^T
      // FP32: all A operands of the tile are read from LDS first, then two independent
      // accumulation chains (even and odd K steps) keep the matrix pipe fed.  FP64 keeps
      // one chain with the reads interleaved (its register budget is already full).
      auto gemm1 = [&](int tt) {
        const int pp = 8 * tt + row_pp;
        if constexpr (sizeof(RT) == 8) {
          typename M::acc a1 = {0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < kKA; ++ks)
            if (ks < nKA) a1 = M::op(Qd[((4 * ks + lk) * kQS + pp) * 2 + row_part], b1[ks], a1);
          return a1;
        }
        RT av[kKA];
#pragma unroll
        for (int ks = 0; ks < kKA; ++ks) av[ks] = ks < nKA ? Qd[((4 * ks + lk) * kQS + pp) * 2 + row_part] : RT(0);
        __builtin_amdgcn_sched_barrier(0);  // keep every read ahead of the products
        typename M::acc e = {0, 0, 0, 0}, o = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < kKA; ks += 2) {
          if (ks < nKA) e = M::op(av[ks], b1[ks], e);
          if (ks + 1 < nKA) o = M::op(av[ks + 1], b1[ks + 1], o);
        }
        return e + o;
      };
      typename M::acc acc1 = gemm1(0);
#pragma unroll 1
      for (int tt = 0; tt < nTB; ++tt) {
        typename M::acc nxt = {0, 0, 0, 0};
        if (tt + 1 < nTB) nxt = gemm1(tt + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int Jt = 0; Jt < kJT; ++Jt)
            if (Jt < nJT) {
              const RT a = Cb[(16 * Jt + li) * kCS + 8 * tt + 4 * h + lk];
              acc2[Jt][0] = M::op(a, acc1[2 * h], acc2[Jt][0]);
              acc2[Jt][1] = M::op(a, acc1[2 * h + 1], acc2[Jt][1]);
            }
        acc1 = nxt;
      }
      const int I = 16 * it + li;
      if constexpr (sizeof(RT) == 4) {
        // FP32 (lane rows J = 16 Jt + 4 lk + j): the mirror block takes 128-byte runs directly,
        // the direct block goes through a per-wavefront LDS tile and leaves as 16-byte stores
        // along J, as in p_bf16x3
        const float gf = (float)(-g);
        float2* Tw = Ts + w * 16 * kTS;
        const bool ev = ((q.Np | pB) & 1) == 0;
#pragma unroll
        for (int hf = 0; hf < (kJT + 1) / 2; ++hf) {
#pragma unroll
          for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int Jt = 2 * hf + jt, Jl = 16 * jt + M::drow(lk, j), J = 32 * hf + Jl;
              if (Jt < kJT) {
                const bool kp = Jt < nJT && (!LIST || (I < (k.mt & 0xffff) && J < (k.mt >> 16)));
                Tw[li * kTS + Jl] = kp ? make_float2(gf * (float)acc2[Jt][0][j], gf * (float)acc2[Jt][1][j])
                                       : make_float2(0.f, 0.f);
              }
            }
#pragma unroll
          for (int i4 = 0; i4 < 4; ++i4) {
            const int rr = (lane >> 4) + 4 * i4, Jl = 2 * (lane & 15), J = 32 * hf + Jl, Ir = 16 * it + rr;
            if (Ir < q.mA && J < q.mB) {
              const float2 v0 = Tw[rr * kTS + Jl];
              float2* dst = reinterpret_cast<float2*>(Pd) + (long long)(pA + Ir) * q.Np + pB + J;
              if (J + 1 < q.mB) {
                const float2 v1 = Tw[rr * kTS + Jl + 1];
                if (ev) {
                  *reinterpret_cast<float4*>(dst) = make_float4(v0.x, v0.y, v1.x, v1.y);
                } else {
                  dst[0] = v0;
                  dst[1] = v1;
                }
              } else {
                dst[0] = v0;
              }
            }
          }
        }
        if (t != tm && I < q.mA) {
#pragma unroll
          for (int Jt = 0; Jt < kJT; ++Jt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int J = 16 * Jt + M::drow(lk, j);
              if (Jt < nJT && J < q.mB) {
                const bool kp = !LIST || (I < (k.mt & 0xffff) && J < (k.mt >> 16));
                reinterpret_cast<float2*>(Pm)[(long long)(pB + J) * q.Np + pA + I] =
                    kp ? make_float2(gf * (float)acc2[Jt][0][j], gf * (float)acc2[Jt][1][j]) : make_float2(0.f, 0.f);
              }
            }
        }
      } else if (I < q.mA) {
#pragma unroll
        for (int Jt = 0; Jt < kJT; ++Jt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int J = 16 * Jt + M::drow(lk, j);
            if (Jt < nJT && J < q.mB) {
              // a listed block keeps I < mA, J < mB of its tier and is zero elsewhere
              const bool kp = !LIST || (I < (k.mt & 0xffff) && J < (k.mt >> 16));
              const double re = kp ? -g * (double)acc2[Jt][0][j] : 0.0, im = kp ? -g * (double)acc2[Jt][1][j] : 0.0;
              stc(Pd + (long long)(pA + I) * q.Np + pB + J, re, im);
              if (t != tm) stc(Pm + (long long)(pB + J) * q.Np + pA + I, re, im);
            }
          }
      }
    }
    if (more) stage();  // Xs, Ys were last read before the barrier above
    cur = nxt;
    nxt = nf;
    adv(nn);
    __syncthreads();
  }
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int kWBS = 72;                    // bf16 row stride of a W plane
constexpr int kWBP = kMP * kWBS;            // bf16 elements per W plane
constexpr int kCBS = 40;                    // bf16 per (plane, step, p) row of C~_A: 4 groups of 8 + pad

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// bf16(x) in the low half, bf16(y) in the high half (round to nearest even)
__device__ __forceinline__ unsigned pack_bf16x2(float x, float y) {
  const bf2 h = {(__bf16)x, (__bf16)y};
  return __builtin_bit_cast(unsigned, h);
}
typedef unsigned u4 __attribute__((ext_vector_type(4)));
// split_bf16 of x and y at once: hi and lo packed as (x, y)
// (x's bf16 is moved to the high half with one byte permute: v_perm_b32 with selector
// 0x01000c0c puts bytes 0, 1 of hi in bytes 2, 3 and zeros below, so that the compiler does
// not convert x a second time to form it)
__device__ __forceinline__ void split_bf16x2(float x, float y, unsigned& hi, unsigned& lo) {
  hi = pack_bf16x2(x, y);
  lo = pack_bf16x2(x - __uint_as_float(__builtin_amdgcn_perm(0u, hi, 0x01000c0cu)),
                   y - __uint_as_float(hi & 0xffff0000u));
}
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// ---------------------------------------------------------------------------
// polarizability on the BF16 matrix cores with split-precision products (GW_BF16X3),
// for 9-orbital species with 49..64 product functions on both atoms.  Same blocks, band walk,
// G-tile prefetch and tau mirror as p_mfma.  Q is formed in FP32 and written split into bf16
// hi / lo planes stored transposed, Q^T[p'][p] (row stride 72: the 16-byte A-operand reads of
// eight lanes hit distinct banks).  GEMM1 (wavefront w, I tile w):
// D1[p'][I] = sum_p Q[p][p'] C~_A[I][p] per part and per 16-row block pb of p', K = p in
// two 32-deep steps (p >= 48 zero).  GEMM2: acc[J][I] += sum_p' C~_B[J][p'] D1[p'][I], its
// K = p' taken in steps of two D1 blocks split in registers, K slot 8 g + e <->
// p' = 32 s + 16 (e / 4) + 4 g + e % 4; C~_B sits in LDS in that slot order.
// ---------------------------------------------------------------------------
constexpr int kQBS = 72;              // bf16 row stride of a Q^T plane
constexpr int kQBP = kPL * kQBS;      // bf16 elements per plane
constexpr int kCBB = 40;              // bf16 per (plane, step, J) row of C~_B

template <bool LIST = false>
__global__ __launch_bounds__(256, 2) void p_bf16x3(const float2* __restrict__ GR, float2* __restrict__ P,
                                                   const float* __restrict__ CpA, const float* __restrict__ CpB,
                                                   const PairArgs q, double g) {
  __shared__ float2 Xs[kMaxOrb * kMaxOrb], Ys[kMaxOrb * kMaxOrb];
  __shared__ __align__(16) __bf16 Qb[4 * kQBP];                // [part][hi|lo][p'][p]
  __shared__ __align__(16) __bf16 Cbb[2 * 2 * kMP * kCBB];     // [hi|lo][step][J][slot]
  __shared__ __align__(16) float2 Ts[4 * 16 * kTS];            // [wavefront][I][J half]
  __shared__ unsigned char ta[kPL], tb[kPL], tc[kPL], td[kPL];
  __shared__ int mRs[kMaxR];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  if (tid < q.npA) pair_of(tid, q.nA, ta[tid], tb[tid]);
  if (tid < q.npB) pair_of(tid, q.nB, tc[tid], td[tid]);
  for (int i = tid; i < q.NR; i += 256) mRs[i] = q.minusR[i];
  for (int i = tid; i < 4 * kQBP; i += 256) Qb[i] = (__bf16)0.f;  // p >= 48 stays zero
  for (int i = tid; i < 2 * kMP * 32; i += 256) {
    const int st = i / (kMP * 32), r = i - st * kMP * 32, J = r / 32, slot = r - J * 32;
    const int gg = slot >> 3, e = slot & 7;
    const int pp = 32 * st + 16 * (e >> 2) + 4 * gg + (e & 3);
    const float v = (J < q.mpB && pp < q.nppB) ? CpB[J * q.nppB + pp] : 0.f;
    __bf16 h, l;
    split_bf16(v, h, l);
    Cbb[((0 * 2 + st) * kMP + J) * kCBB + 8 * gg + e] = h;
    Cbb[((1 * 2 + st) * kMP + J) * kCBB + 8 * gg + e] = l;
  }
  // GEMM1 B operand: lane (I = 16 w + li, g) holds p = 32 s + 8 g + e
  bf8 cah[2], cal[2];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int pp = 32 * st + 8 * lk + e;
      const float v = pp < q.nppA ? CpA[(16 * w + li) * q.nppA + pp] : 0.f;
      __bf16 h, l;
      split_bf16(v, h, l);
      cah[st][e] = h;
      cal[st][e] = l;
    }
  __syncthreads();  // pair tables, minus-R table, Q zero padding staged
  // per-thread Q entries (p fastest): packed (a, b, c, d) of p = {a, b}, p' = {c, d}
  unsigned qpk[kQE];
  int qoff[kQE];
#pragma unroll
  for (int e = 0; e < kQE; ++e) {
    const int i = tid + 256 * e;
    const int pp = i / q.nppA, p = i - pp * q.nppA;
    qoff[e] = pp * kQBS + p;
    qpk[e] = (i < q.nppA * q.nppB && p < q.npA && pp < q.npB)
                 ? (unsigned)ta[p] | ((unsigned)tb[p] << 8) | ((unsigned)tc[pp] << 16) | ((unsigned)td[pp] << 24)
                 : 0xffffffffu;
  }
  __builtin_amdgcn_s_waitcnt(0);
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  float2 xr, yr;
  const bool xok = tid < q.nA * q.nB;
  auto fetch = [&](const Blk& k) {
    const int a = tid / q.nB, c = tid - a * q.nB;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR, xok);
    const int d = tid / q.nA, bb = tid - d * q.nA;
    yr = ldraw(GR + ((long long)(q.n_tau - 1 - k.t) * q.NR + mRs[k.R]) * sl + (long long)(k.ob.y + d) * q.No +
                   k.oa.y + bb,
               GR, xok);
  };
  auto stage = [&]() {
    if (xok) {
      Xs[tid] = xr;
      Ys[tid] = yr;
    }
  };
  const long long per = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per;
  const long long bend = bbeg + per < q.nblocks ? bbeg + per : q.nblocks;
  Blk cur;
  // dense: band walk; block list: its contiguous range
  auto adv = [&](Blk& x) {
    if constexpr (LIST)
      blk_step<true>(x, q);
    else
      bblk_step(x, q);
  };
  if constexpr (LIST)
    blk_start<true>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  else
    bblk_start(cur, bbeg < q.nblocks ? bbeg : 0, q);
  blk_fill<LIST>(cur, q);
  Blk nxt = cur, nn = cur;
  adv(nxt);
  blk_fill<LIST>(nxt, q);
  adv(nn);
  adv(nn);
  if (bbeg < bend) {
    fetch(cur);
    stage();
  }
  __syncthreads();
  // GEMM1 for part pt and p' block pb
  auto gemm1 = [&](int pt, int pb) {
    f4 d = {0, 0, 0, 0};
    const int row = (16 * pb + li) * kQBS + 8 * lk;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const bf8 ah = *reinterpret_cast<const bf8*>(&Qb[(2 * pt + 0) * kQBP + row + 32 * st]);
      const bf8 al = *reinterpret_cast<const bf8*>(&Qb[(2 * pt + 1) * kQBP + row + 32 * st]);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, cah[st], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, cal[st], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, cah[st], d, 0, 0, 0);
    }
    return d;
  };
  for (long long blk = bbeg; blk < bend; ++blk) {
    const Blk k = cur;
    const int t = k.t, R = k.R;
    const int tm = q.n_tau - 1 - t, mR = mRs[R];
    const int pA = k.oa.x, pB = k.ob.x;
    const bool more = blk + 1 < bend;
    if (more) fetch(nxt);
    Blk nf = nn;
    blk_fill<LIST>(nf, q);
    // Q over unordered pairs, written split and transposed
#pragma unroll
    for (int e = 0; e < kQE; ++e) {
      const int i = tid + 256 * e;
      if (i < q.nppA * q.nppB) {
        float qr = 0, qi = 0;
        const unsigned pk = qpk[e];
        if (pk != 0xffffffffu) {
          const int a = pk & 0xff, bq = (pk >> 8) & 0xff, c = (pk >> 16) & 0xff, d = pk >> 24;
          const int nB = q.nB, nA = q.nA;
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int c1 = s2 ? d : c, d1 = s2 ? c : d;
            if (s2 == 1 && c == d) break;
            float2 x = Xs[a * nB + c1], y = Ys[d1 * nA + bq];
            qr += x.x * y.x - x.y * y.y;
            qi += x.x * y.y + x.y * y.x;
            if (a != bq) {
              x = Xs[bq * nB + c1];
              y = Ys[d1 * nA + a];
              qr += x.x * y.x - x.y * y.y;
              qi += x.x * y.y + x.y * y.x;
            }
          }
        }
        __bf16 h, l;
        split_bf16(qr, h, l);
        Qb[0 * kQBP + qoff[e]] = h;
        Qb[1 * kQBP + qoff[e]] = l;
        split_bf16(qi, h, l);
        Qb[2 * kQBP + qoff[e]] = h;
        Qb[3 * kQBP + qoff[e]] = l;
      }
    }
    __syncthreads();

    float2* Pd = P + ((long long)t * q.NR + R) * slp;
    float2* Pm = P + ((long long)tm * q.NR + mR) * slp;
    {
      f4 acc2[4][2];  // step 0 starts them from an inline zero operand
#pragma unroll
      for (int st = 0; st < 2; ++st) {
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
          const f4 d0 = gemm1(pt, 2 * st);
          const f4 d1 = st == 0 ? gemm1(pt, 1) : f4{0, 0, 0, 0};
          unsigned hw[4], lw[4];  // dword d: K slots 2 d, 2 d + 1
          split_bf16x2(d0[0], d0[1], hw[0], lw[0]);
          split_bf16x2(d0[2], d0[3], hw[1], lw[1]);
          split_bf16x2(d1[0], d1[1], hw[2], lw[2]);
          split_bf16x2(d1[2], d1[3], hw[3], lw[3]);
          const bf8 bh = __builtin_bit_cast(bf8, u4{hw[0], hw[1], hw[2], hw[3]});
          const bf8 bl = __builtin_bit_cast(bf8, u4{lw[0], lw[1], lw[2], lw[3]});
#pragma unroll
          for (int Jt = 0; Jt < 4; ++Jt) {
            const bf8 ah = *reinterpret_cast<const bf8*>(&Cbb[((0 * 2 + st) * kMP + 16 * Jt + li) * kCBB + 8 * lk]);
            const bf8 al = *reinterpret_cast<const bf8*>(&Cbb[((1 * 2 + st) * kMP + 16 * Jt + li) * kCBB + 8 * lk]);
            acc2[Jt][pt] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, st == 0 ? f4{0, 0, 0, 0} : acc2[Jt][pt], 0, 0, 0);
            acc2[Jt][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc2[Jt][pt], 0, 0, 0);
            acc2[Jt][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc2[Jt][pt], 0, 0, 0);
          }
        }
      }
      // Lane (li, lk) holds J = 16 Jt + 4 lk + j of row I.  The mirror block's rows (J) take
      // these as 128-byte runs directly.  The direct block's rows (I) go through a per-wave LDS
      // tile, one 32-column half at a time, and leave as 16-byte stores along J.
      const int I = 16 * w + li;
      const float gf = (float)(-g);
      float2* Tw = Ts + w * 16 * kTS;
      const bool ev = ((q.Np | pB) & 1) == 0;
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
        for (int jt = 0; jt < 2; ++jt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int Jl = 16 * jt + 4 * lk + j, J = 32 * hf + Jl;
            const bool kp = !LIST || (I < (k.mt & 0xffff) && J < (k.mt >> 16));
            const f4& ar = acc2[2 * hf + jt][0];
            const f4& ai = acc2[2 * hf + jt][1];
            Tw[li * kTS + Jl] = kp ? make_float2(gf * ar[j], gf * ai[j]) : make_float2(0.f, 0.f);
          }
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int rr = (lane >> 4) + 4 * it, Jl = 2 * (lane & 15), J = 32 * hf + Jl, Ir = 16 * w + rr;
          if (Ir < q.mA && J < q.mB) {
            const float2 v0 = Tw[rr * kTS + Jl];
            float2* dst = Pd + (long long)(pA + Ir) * q.Np + pB + J;
            if (J + 1 < q.mB) {
              const float2 v1 = Tw[rr * kTS + Jl + 1];
              if (ev) {
                *reinterpret_cast<float4*>(dst) = make_float4(v0.x, v0.y, v1.x, v1.y);
              } else {
                dst[0] = v0;
                dst[1] = v1;
              }
            } else {
              dst[0] = v0;
            }
          }
        }
      }
      if (t != tm && I < q.mA) {
#pragma unroll
        for (int Jt = 0; Jt < 4; ++Jt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int J = 16 * Jt + 4 * lk + j;
            if (J < q.mB) {
              const bool kp = !LIST || (I < (k.mt & 0xffff) && J < (k.mt >> 16));
              Pm[(long long)(pB + J) * q.Np + pA + I] =
                  kp ? make_float2(gf * acc2[Jt][0][j], gf * acc2[Jt][1][j]) : make_float2(0.f, 0.f);
            }
          }
      }
    }
    if (more) stage();
    cur = nxt;
    nxt = nf;
    adv(nn);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// self-energy.  192 threads: wavefront w owns the 16 pairs p' = 16 w .. 16 w + 15 of
// atom B (idle in the matrix phase if 16 w >= np_pad(B)).  W^R(tau)[A, B] streams
// through an LDS tile of 16 rows (I) with coalesced loads; the next tile is
// fetched into registers while the current one is multiplied.  The first product
// runs separately on Re W and Im W (rows I), so every 16-byte W element read from
// LDS feeds two MFMAs.  The W tile and the K block share one LDS region, which
// keeps a workgroup under 40 KB so that four of them (three wavefronts per SIMD)
// fit on a compute unit.
// ---------------------------------------------------------------------------
constexpr int kWS = kMP + 1;                     // W tile row stride (complex)
constexpr int kKS = kPL + 1;                     // K row stride (complex)
constexpr int kSThreads = 192;
constexpr int kWPT = (16 * kMP + kSThreads - 1) / kSThreads;

template <class RT, class CT, bool LIST = false>
__global__ __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(3))) void s_mfma(const CT* __restrict__ GR, const CT* __restrict__ WR,
                                                 double2* __restrict__ S, const RT* __restrict__ CpA,
                                                 const RT* __restrict__ CpB, const PairArgs q) {
  using M = Mma<RT>;
  typedef typename M::cplx CR;
  constexpr size_t kWbytes = 16 * kWS * sizeof(CR);
  constexpr size_t kKbytes = kPL * kKS * sizeof(CR);
  __shared__ __align__(16) unsigned char U[kWbytes > kKbytes ? kWbytes : kKbytes];
  __shared__ CR Xs[90];  // X as a zero-padded 10 x 9 tile: fixed trip counts in the unfold
  __shared__ unsigned char pidA[81], pidB[81];
  CR* Wb = reinterpret_cast<CR*>(U);
  CR* Ks = reinterpret_cast<CR*>(U);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int nIT = q.mpA / 16, nKJ = q.mpB / 4, nMT = q.nppA / 16;
  const bool mm = 16 * w < q.nppB;  // this wavefront has pairs of B
  for (int i = tid; i < q.nA * q.nA; i += kSThreads) pidA[i] = (unsigned char)pair_index(i / q.nA, i % q.nA, q.nA);
  for (int i = tid; i < q.nB * q.nB; i += kSThreads) pidB[i] = (unsigned char)pair_index(i / q.nB, i % q.nB, q.nB);
  RT b1[kKJ];
#pragma unroll
  for (int ks = 0; ks < kKJ; ++ks) b1[ks] = (mm && ks < nKJ) ? CpB[(4 * ks + lk) * q.nppB + 16 * w + li] : RT(0);
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  // unfold: thread (o, half) sums rows a' = 5 half .. 5 half + 4 (rows >= n_A are zero in X)
  const int uo = tid >> 1, uh = tid & 1;

  // block b: (tau, R, atoms) in counting order, or (tau, list entry) with LIST.  Dense: pA, pB
  // hold the atoms (offsets looked up at use, as few live registers as possible); LIST: the
  // offsets themselves and the kept product functions mt = mA | mB << 16.
  struct SBlk {
    int t, R, pA, oA, pB, oB, mt;
  };
  auto decode = [&](long long b) {
    SBlk o;
    if constexpr (LIST) {
      o.t = (int)(b / q.nlist);
      const int i = (int)(b - (long long)o.t * q.nlist);
      const int4 e0 = q.list[2 * i], e1 = q.list[2 * i + 1];
      o.R = e0.x;
      o.mt = e0.y;
      o.pA = e0.z;
      o.oA = e0.w;
      o.pB = e1.x;
      o.oB = e1.y;
    } else {
      const int iB = (int)(b % q.cntB);
      b /= q.cntB;
      const int iA = (int)(b % q.cntA);
      b /= q.cntA;
      o.R = (int)(b % q.NR);
      o.t = (int)(b / q.NR);
      o.pA = q.atomsA[iA];
      o.pB = q.atomsB[iB];
      o.oA = o.oB = o.mt = 0;
    }
    return o;
  };
  CT wreg[kWPT];  // prefetched W tile and X element, in the storage type
  CT xr;
  int wtile = 0;  // I tile of the W values in wreg (their validity is applied at stash())
  int wmt = 0;    // product functions kept by the block of those W values
  auto fetch = [&](const SBlk& k, int it) {
    const int pa = LIST ? k.pA : q.pb_off[k.pA], pb = LIST ? k.pB : q.pb_off[k.pB];
    const CT* Wt = WR + ((long long)k.t * q.NR + k.R) * slp + (long long)pa * q.Np + pb;
#pragma unroll
    for (int u = 0; u < kWPT; ++u) {
      const int i = tid + kSThreads * u, r = i / kMP, c = i - r * kMP, I = 16 * it + r;
      const bool ok = r < 16 && I < q.mA && c < q.mB;
      wreg[u] = ldraw(Wt + (long long)I * q.Np + c, WR, ok);
    }
    wtile = it;
    if constexpr (LIST) wmt = k.mt;
  };
  const bool xok = tid < 90, xin = tid / 9 < q.nA && tid % 9 < q.nB;
  auto fetch_x = [&](const SBlk& k) {
    const int a = tid / 9, c = tid - 9 * a;
    const int oa = LIST ? k.oA : q.orb_off[k.pA], ob = LIST ? k.oB : q.orb_off[k.pB];
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(oa + a) * q.No + ob + c, GR, xok && xin);
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < kWPT; ++u) {
      const int i = tid + kSThreads * u, r = i / kMP, c = i - r * kMP, I = 16 * wtile + r;
      if (r < 16) {
        const bool tier = !LIST || (I < (wmt & 0xffff) && c < (wmt >> 16));
        const CT v = keep(wreg[u], I < q.mA && c < q.mB && tier);
        Wb[r * kWS + c] = mk<RT>((double)v.x, (double)v.y);
      }
    }
  };

  // The first W tile and the X tile of the next block are staged after the unfold has
  // finished with K (same LDS) and before this block's Sigma stores, so waiting for
  // those loads never waits for fresh stores.
  if (blockIdx.x < q.nblocks) {
    fetch(decode(blockIdx.x), 0);
    fetch_x(decode(blockIdx.x));
    if (xok) {
      const CT xv = keep(xr, xin);
      Xs[tid] = mk<RT>((double)xv.x, (double)xv.y);
    }
    stash();
  }
  __syncthreads();
  for (long long blk = blockIdx.x; blk < q.nblocks; blk += gridDim.x) {
    const SBlk k = decode(blk);
    const int oA = LIST ? k.oA : q.orb_off[k.pA], oB = LIST ? k.oB : q.orb_off[k.pB];
    const bool more = blk + gridDim.x < q.nblocks;
    typename M::acc acc2[3][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) acc2[m][0] = acc2[m][1] = typename M::acc{0, 0, 0, 0};
    for (int it = 0; it < nIT; ++it) {
      if (it + 1 < nIT) fetch(k, it + 1);
      if (mm) {
        typename M::acc zr = {0, 0, 0, 0}, zi = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < kKJ; ++ks)
          if (ks < nKJ) {
            const CR wv = Wb[li * kWS + 4 * ks + lk];
            zr = M::op(wv.x, b1[ks], zr);
            zi = M::op(wv.y, b1[ks], zi);
          }
        // K_part[p][p'] += C~_A[I][p] Z_part[I][p'], K steps I = 16 it + drow(lk, j)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int Ik = 16 * it + M::drow(lk, j);
#pragma unroll
          for (int m = 0; m < 3; ++m)
            if (m < nMT) {
              const RT a = CpA[Ik * q.nppA + 16 * m + li];
              acc2[m][0] = M::op(a, zr[j], acc2[m][0]);
              acc2[m][1] = M::op(a, zi[j], acc2[m][1]);
            }
        }
      }
      __syncthreads();
      if (it + 1 < nIT) {
        stash();
        __syncthreads();
      }
    }
    if (more) {
      const SBlk kn = decode(blk + gridDim.x);
      fetch(kn, 0);
      fetch_x(kn);
    }
    if (mm) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m < nMT)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            Ks[(16 * m + M::drow(lk, j)) * kKS + 16 * w + li] = mk<RT>((double)acc2[m][0][j], (double)acc2[m][1][j]);
    }
    __syncthreads();
    // Sigma_ab = -sum_{a', b'} K[{a,a'}][{b,b'}] X_{a'b'} in FP64; the two halves of the
    // a' range sit in neighbouring lanes and are combined with one exchange
    {
      double sr = 0, si = 0;
      const bool live = uo < q.nA * q.nB;
      if (live) {
        const int a = uo / q.nB, bb = uo - a * q.nB;
#pragma unroll 1
        for (int i = 0; i < 5; ++i) {
          const int ap = 5 * uh + i;
          const CR* Kr = Ks + pidA[a * q.nA + (ap < q.nA ? ap : q.nA - 1)] * kKS;
          const int bq = bb * q.nB;
#pragma unroll
          for (int bp = 0; bp < 9; ++bp) {
            const CR kv = Kr[pidB[bq + (bp < q.nB ? bp : q.nB - 1)]], x = Xs[9 * ap + bp];
            sr += (double)kv.x * x.x - (double)kv.y * x.y;
            si += (double)kv.x * x.y + (double)kv.y * x.x;
          }
        }
      }
      sr += __shfl_xor(sr, 1);
      si += __shfl_xor(si, 1);
      __syncthreads();  // K and X no longer read
      if (more) {
        if (xok) {
          const CT xv = keep(xr, xin);
          Xs[tid] = mk<RT>((double)xv.x, (double)xv.y);
        }
        stash();
      }
      if (live && uh == 0) {
        const int a = uo / q.nB, bb = uo - a * q.nB;
        S[((long long)k.t * q.NR + k.R) * sl + (long long)(oA + a) * q.No + oB + bb] = make_double2(-sr, -si);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// self-energy, FP32 storage.  Same contraction as s_mfma, restructured so that no wave
// waits for HBM inside a block: the whole W^R(tau)[A, B] block (<= 64 x 64) sits in LDS
// (row stride 66 complex: the 64 lanes of an A-operand read hit distinct bank pairs)
// and the next block's W is loaded into registers while this one is multiplied, a whole
// block ahead.  C~_A is kept in LDS (row stride 52 floats: conflict-free GEMM2 reads),
// C~_B in registers; the first product of I tile it+1 is issued before the second
// product of tile it.  The FP64 unfold forms the unordered-pair indices arithmetically.
// ---------------------------------------------------------------------------
constexpr int kS32Threads = 192;
constexpr int kW32S = 66;                                            // W row stride (complex)
constexpr int kW32PF = (kMP * kMP + kS32Threads - 1) / kS32Threads;  // prefetched W values per thread
constexpr int kCA32S = 52;                                           // C~_A row stride (floats)
constexpr int kIT32 = kMP / 16;

// NIT = m_pad(A) / 16, NKJ = m_pad(B) / 4, NMT = np_pad(A) / 16 are compile-time so that
// every operand array stays in registers.
template <int NIT, int NKJ, int NMT, bool LIST = false>
__global__ __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(3))) void s_mfma32(
    const float2* __restrict__ GR, const float2* __restrict__ WR, double2* __restrict__ S,
    const float* __restrict__ CpA, const float* __restrict__ CpB, const PairArgs q) {
  __shared__ __align__(16) float2 Ub[kMP * kW32S];  // W block, then the K block
  __shared__ float Ca[kMP * kCA32S];
  // X as a zero-padded tile of 2 HR rows of nine (HR = rows a' per unfold half), so that
  // the unfold loops have fixed trip counts
  constexpr int HR = NMT >= 3 ? 5 : (NMT == 2 ? 4 : 3);
  __shared__ float2 Xs[2 * HR * 9];
  float2* Wb = Ub;
  float2* Ks = Ub;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  constexpr int nIT = NIT, nKJ = NKJ, nMT = NMT;
  const bool mm = 16 * w < q.nppB;  // this wavefront has pairs of B
  for (int i = tid; i < kMP * kCA32S; i += kS32Threads) {
    const int I = i / kCA32S, p = i - I * kCA32S;
    Ca[i] = (I < q.mpA && p < q.nppA) ? CpA[I * q.nppA + p] : 0.f;
  }
  float b1[kKJ];
#pragma unroll
  for (int ks = 0; ks < kKJ; ++ks) b1[ks] = (mm && ks < nKJ) ? CpB[(4 * ks + lk) * q.nppB + 16 * w + li] : 0.f;
  // Settle these loads here, on every path: otherwise the wait inserted before the first
  // use of b1 inside the block loop is a full vmcnt(0), which would also wait for the
  // next block's W prefetch and serialise it with the matrix work.
  __builtin_amdgcn_s_waitcnt(0);
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  const int uo = tid >> 1, uh = tid & 1;
  // Blocks are walked in a contiguous range, so their (tau, R, iA, iB) indices advance by
  // counting (B fastest) and the atom offsets come from the per-species (pb, orb) tables;
  // the table entries of block b + 2 are loaded while block b is multiplied.
  // W rows r = w + 3 u (64 consecutive elements of a row per wavefront), column = lane
  float2 wreg[kW32PF];
  float2 xr;
  const bool lane_ok = lane < q.mB;
  auto fetch = [&](const Blk& k) {
    const float2* p = WR + ((long long)k.t * q.NR + k.R) * slp + (long long)(k.oa.x + w) * q.Np + k.ob.x + lane;
    const long long step = 3LL * q.Np;
#pragma unroll
    for (int u = 0; u < kW32PF; ++u) {
      wreg[u] = ldraw(p, WR, lane_ok && w + 3 * u < q.mA);
      p += step;
    }
  };
  const bool xok = tid < 2 * HR * 9, xin = tid / 9 < q.nA && tid % 9 < q.nB;
  auto fetch_x = [&](const Blk& k) {
    const int a = tid / 9, c = tid - 9 * a;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR,
               xok && xin);
  };
  // mt: product functions kept by the block whose W is staged (W outside them is zero)
  auto stash = [&](int mt) {
#pragma unroll
    for (int u = 0; u < kW32PF; ++u) {
      const int r = w + 3 * u;
      const bool tier = !LIST || (r < (mt & 0xffff) && lane < (mt >> 16));
      if (r < kMP) Wb[r * kW32S + lane] = keep(wreg[u], r < q.mA && lane_ok && tier);
    }
    if (xok) Xs[tid] = keep(xr, xin);
  };
  auto load_ca = [&](int it, float (&ca)[4][3]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < 3; ++m) ca[j][m] = Ca[(16 * it + 4 * lk + j) * kCA32S + 16 * m + li];
  };
  auto gemm1 = [&](int it, f4& zr, f4& zi) {
    zr = f4{0, 0, 0, 0};
    zi = f4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < kKJ; ++ks)
      if (ks < nKJ) {
        const float2 wv = Wb[(16 * it + li) * kW32S + 4 * ks + lk];
        zr = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, b1[ks], zr, 0, 0, 0);
        zi = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, b1[ks], zi, 0, 0, 0);
      }
  };

  // Each workgroup walks one contiguous range of blocks (B fastest): consecutive blocks
  // read neighbouring column ranges of the same W rows, so the cache lines they share
  // are still in this XCD's L2 when the next block is fetched.
  const long long per = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per;
  const long long bend = bbeg + per < q.nblocks ? bbeg + per : q.nblocks;
  Blk cur;
  blk_start<LIST>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  blk_fill<LIST>(cur, q);
  Blk nxt = cur, nn = cur;
  blk_step<LIST>(nxt, q);
  blk_fill<LIST>(nxt, q);
  blk_step<LIST>(nn, q);
  blk_step<LIST>(nn, q);
  if (bbeg < bend) {
    fetch(cur);
    fetch_x(cur);
    stash(cur.mt);
  }
  __syncthreads();
  for (long long blk = bbeg; blk < bend; ++blk) {
    const Blk k = cur;
    const int oA = k.oa.y, oB = k.ob.y;
    const bool more = blk + 1 < bend;
    if (more) {
      fetch(nxt);
      fetch_x(nxt);
    }
    // offsets of block blk + 2 (always loaded, from in-range indices, so that nothing
    // copies the registers before the end of this block), consumed by the next fetch
    Blk nf = nn;
    blk_fill<LIST>(nf, q);
    f4 acc2[3][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) acc2[m][0] = acc2[m][1] = f4{0, 0, 0, 0};
    if (mm) {
      f4 zr0, zi0, zr1, zi1;
      float ca[4][3];
      gemm1(0, zr0, zi0);
#pragma unroll
      for (int it = 0; it < kIT32; ++it) {
        if (it < nIT) {
          load_ca(it, ca);
          if (it + 1 < nIT) gemm1(it + 1, zr1, zi1);
          // K_part[p][p'] += C~_A[I][p] Z_part[I][p'], K steps I = 16 it + 4 lk + j
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = 0; m < 3; ++m)
              if (m < nMT) {
                acc2[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[j][m], zr0[j], acc2[m][0], 0, 0, 0);
                acc2[m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[j][m], zi0[j], acc2[m][1], 0, 0, 0);
              }
          zr0 = zr1;
          zi0 = zi1;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    __syncthreads();  // every wavefront is done with W
    if (mm) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m < nMT)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            Ks[(16 * m + 4 * lk + j) * kKS + 16 * w + li] = make_float2(acc2[m][0][j], acc2[m][1][j]);
    }
    __syncthreads();
    // Sigma_ab = -sum_{a', b'} K[{a,a'}][{b,b'}] X_{a'b'}; lane half uh takes rows
    // a' = HR uh .. HR uh + HR - 1, and the halves meet in one exchange.  Rows a' >= n_A and
    // columns b' >= n_B meet zeros of X; their K indices are clamped to a valid entry.  Each
    // row (nine products) is summed in FP32 with two interleaved partial sums, the rows in
    // FP64: K itself comes from FP32 products of 64-term sums, whose rounding is far above
    // that of a nine-term FP32 row.
    double sr = 0, si = 0;
    const bool live = uo < q.nA * q.nB;
    if (live) {
      const int a = uo / q.nB, bb = uo - a * q.nB;
      int pb[9];
#pragma unroll
      for (int bp = 0; bp < 9; ++bp) pb[bp] = pair_index(bb, bp < q.nB ? bp : q.nB - 1, q.nB);
#pragma unroll 1
      for (int i = 0; i < HR; ++i) {
        const int ap = HR * uh + i;
        const float2* Kr = Ks + pair_index(a, ap < q.nA ? ap : q.nA - 1, q.nA) * kKS;
        const float2* Xr = Xs + 9 * ap;
        float pr[2] = {0.f, 0.f}, pi[2] = {0.f, 0.f};
#pragma unroll
        for (int bp = 0; bp < 9; ++bp) {
          const float2 kv = Kr[pb[bp]], x = Xr[bp];
          pr[bp & 1] = fmaf(kv.x, x.x, fmaf(-kv.y, x.y, pr[bp & 1]));
          pi[bp & 1] = fmaf(kv.x, x.y, fmaf(kv.y, x.x, pi[bp & 1]));
        }
        sr += (double)(pr[0] + pr[1]);
        si += (double)(pi[0] + pi[1]);
      }
    }
    sr += __shfl_xor(sr, 1);
    si += __shfl_xor(si, 1);
    __syncthreads();  // K and X no longer read
    if (more) stash(nxt.mt);
    if (live && uh == 0) {
      const int a = uo / q.nB, bb = uo - a * q.nB;
      S[((long long)k.t * q.NR + k.R) * sl + (long long)(oA + a) * q.No + oB + bb] = make_double2(-sr, -si);
    }
    cur = nxt;
    nxt = nf;
    blk_step<LIST>(nn, q);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// self-energy on the BF16 matrix cores with split-precision products (GW_BF16X3).
// Every FP32 operand x is split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi),
// and a product a b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo lo term, of
// relative size 2^-16, is dropped), accumulated in FP32 by v_mfma_f32_16x16x32_bf16.
// Same blocks and walk as s_mfma32, with four wavefronts: waves 0-2 own the 16-column pair
// tiles of B in the products, all four load and stage W (the next block's W is prefetched in
// two halves, the second after this block's products) and share the orbital unfold (three
// lanes per output, three of the nine rows a' each: X is staged as a zero-padded 9 x 9 tile,
// so the unfold's 27 K and X reads per lane carry no branches and issue together).  The W
// block is split once when it is staged and sits in LDS as four bf16 planes (re hi, re lo,
// im hi, im lo; row stride 72: the 16-byte A-operand reads of eight lanes hit distinct banks).
// GEMM1 (Z = W C~_B) takes K = 64 in two 32-deep steps.  GEMM2 (K = C~_A^T Z) takes
// its K = 64 product functions I in two steps of two I tiles: the D fragments of GEMM1
// for tiles 2s and 2s + 1 (rows 4 g + j in register j of lane group g) are split in
// registers and form the B operand with K slot 8 g + e <-> I = 16 (2 s + e / 4) + 4 g + e % 4;
// C~_A is stored in LDS in that slot order.  Shapes: 9-orbital species with
// 49..64 product functions on both atoms.
// ---------------------------------------------------------------------------

constexpr int kSBWaves = 4;                                   // wavefronts of the BF16-split Sigma kernel
constexpr int kSBThreads = 64 * kSBWaves;
constexpr int kWBU = kMP / (2 * kSBWaves);                    // W row steps per thread (two columns each)

// W16: W rows start on 16-byte boundaries at every block column offset (every species has an
// even number of product functions and W is 16-byte aligned), so a lane loads its column pair as
// one 16-byte access
template <bool LIST, bool W16>
__device__ __forceinline__ void s_bf16x3_body(const float2* __restrict__ GR, const float2* __restrict__ WR,
                                              double2* __restrict__ S, const float* __restrict__ CpA,
                                              const float* __restrict__ CpB, const PairArgs q) {
  __shared__ __align__(16) __bf16 Wp[4 * kWBP];           // W planes, then the K block (FP32)
  __shared__ __align__(16) __bf16 Cap[2 * 2 * kPL * kCBS];  // C~_A [hi|lo][step][p][slot]
  __shared__ float2 Xs[81];
  float2* Ks = reinterpret_cast<float2*>(Wp);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const bool mm = 16 * w < q.nppB;
  // C~_A in GEMM2 slot order, split
  for (int i = tid; i < 2 * kPL * 32; i += kSBThreads) {
    const int st = i / (kPL * 32), r = i - st * kPL * 32, p = r / 32, slot = r - p * 32;
    const int g = slot >> 3, e = slot & 7;
    const int I = 16 * (2 * st + (e >> 2)) + 4 * g + (e & 3);
    const float v = (I < q.mpA && p < q.nppA) ? CpA[I * q.nppA + p] : 0.f;
    __bf16 h, l;
    split_bf16(v, h, l);
    Cap[((0 * 2 + st) * kPL + p) * kCBS + 8 * g + e] = h;
    Cap[((1 * 2 + st) * kPL + p) * kCBS + 8 * g + e] = l;
  }
  // C~_B operands of GEMM1: lane (p' = 16 w + li, g) holds J = 32 s + 8 g + e
  bf8 cbh[2], cbl[2];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int J = 32 * st + 8 * lk + e;
      const float v = mm ? CpB[J * q.nppB + 16 * w + li] : 0.f;
      __bf16 h, l;
      split_bf16(v, h, l);
      cbh[st][e] = h;
      cbl[st][e] = l;
    }
  __builtin_amdgcn_s_waitcnt(0);
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  // orbital unfold: lanes 3 j .. 3 j + 2 of wavefront w (j < 21) share output 21 w + j, each
  // summing three of the nine (padded) rows a'
  const int uo = 21 * w + lane / 3, uh = lane - 3 * (lane / 3);
  // W staging: lane = 32 ro + c holds columns 2 c, 2 c + 1 of rows 8 u + 2 w + ro, so that each
  // split plane takes one 4-byte write per lane and column pair
  float2 wreg[kWBU][2];
  float2 xr;
  const int wro = lane >> 5, wc = 2 * (lane & 31);
  const bool c0_ok = wc < q.mB, c1_ok = wc + 1 < q.mB;
  // rows of steps u in [u0, u1)
  auto fetch = [&](const Blk& k, int u0, int u1) {
    const float2* p = WR + ((long long)k.t * q.NR + k.R) * slp + (long long)(k.oa.x + 2 * w + wro) * q.Np +
                      k.ob.x + wc;
    const long long step = 8LL * q.Np;
#pragma unroll
    for (int u = 0; u < kWBU; ++u)
      if (u >= u0 && u < u1) {
        const bool row_ok = 8 * u + 2 * w + wro < q.mA;
        if (W16) {
          // m_B even: both columns of the pair are valid or neither is
          const float4 v = ldraw(reinterpret_cast<const float4*>(p + u * step),
                                 reinterpret_cast<const float4*>(WR), row_ok && c1_ok);
          wreg[u][0] = make_float2(v.x, v.y);
          wreg[u][1] = make_float2(v.z, v.w);
        } else {
          wreg[u][0] = ldraw(p + u * step, WR, row_ok && c0_ok);
          wreg[u][1] = ldraw(p + u * step + 1, WR, row_ok && c1_ok);
        }
      }
  };
  // X sits in LDS as a 9 x 9 tile, zero outside its n_A x n_B corner, so that the unfold runs
  // the same nine-by-nine loop (no branches) for every species of up to nine orbitals
  const bool xok = tid < 81, xin = tid / 9 < q.nA && tid % 9 < q.nB;
  auto fetch_x = [&](const Blk& k) {
    const int a = tid / 9, c = tid - 9 * a;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR,
               xok && xin);
  };
  // mt: product functions kept by the block whose W is staged (W outside them is zero)
  auto stash = [&](int mt) {
#pragma unroll
    for (int u = 0; u < kWBU; ++u) {
      const int r = 8 * u + 2 * w + wro;
      const bool row_ok = r < q.mA && (!LIST || r < (mt & 0xffff));
      const float2 v0 = keep(wreg[u][0], row_ok && c0_ok && (!LIST || wc < (mt >> 16)));
      const float2 v1 = keep(wreg[u][1], row_ok && c1_ok && (!LIST || wc + 1 < (mt >> 16)));
      unsigned rh, rl, ih, il;
      split_bf16x2(v0.x, v1.x, rh, rl);
      split_bf16x2(v0.y, v1.y, ih, il);
      const int o = r * kWBS + wc;
      *reinterpret_cast<unsigned*>(&Wp[0 * kWBP + o]) = rh;
      *reinterpret_cast<unsigned*>(&Wp[1 * kWBP + o]) = rl;
      *reinterpret_cast<unsigned*>(&Wp[2 * kWBP + o]) = ih;
      *reinterpret_cast<unsigned*>(&Wp[3 * kWBP + o]) = il;
    }
    if (xok) Xs[tid] = keep(xr, xin);
  };
  // GEMM1 for I tile it: zr / zi = rows 16 it .. 16 it + 15 of Re / Im (W C~_B)
  auto gemm1 = [&](int it, f4& zr, f4& zi) {
    zr = f4{0, 0, 0, 0};
    zi = f4{0, 0, 0, 0};
    const int row = (16 * it + li) * kWBS + 8 * lk;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      bf8 a[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const bf8*>(&Wp[pl * kWBP + row + 32 * st]);
      zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], cbh[st], zr, 0, 0, 0);
      zi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], cbh[st], zi, 0, 0, 0);
      zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], cbl[st], zr, 0, 0, 0);
      zi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], cbl[st], zi, 0, 0, 0);
      zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], cbh[st], zr, 0, 0, 0);
      zi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3], cbh[st], zi, 0, 0, 0);
    }
  };
  // GEMM2 step st: acc2[m][part] += C~_A^T Z over I tiles 2 st, 2 st + 1
  auto gemm2 = [&](int st, const f4& zr0, const f4& zi0, const f4& zr1, const f4& zi1, f4 (&acc2)[3][2]) {
    // split two K slots per conversion: dword d of the operand holds slots 2 d, 2 d + 1
    unsigned rh[4], rl[4], ih[4], il[4];
    split_bf16x2(zr0[0], zr0[1], rh[0], rl[0]);
    split_bf16x2(zr0[2], zr0[3], rh[1], rl[1]);
    split_bf16x2(zr1[0], zr1[1], rh[2], rl[2]);
    split_bf16x2(zr1[2], zr1[3], rh[3], rl[3]);
    split_bf16x2(zi0[0], zi0[1], ih[0], il[0]);
    split_bf16x2(zi0[2], zi0[3], ih[1], il[1]);
    split_bf16x2(zi1[0], zi1[1], ih[2], il[2]);
    split_bf16x2(zi1[2], zi1[3], ih[3], il[3]);
    const bf8 brh = __builtin_bit_cast(bf8, u4{rh[0], rh[1], rh[2], rh[3]});
    const bf8 brl = __builtin_bit_cast(bf8, u4{rl[0], rl[1], rl[2], rl[3]});
    const bf8 bih = __builtin_bit_cast(bf8, u4{ih[0], ih[1], ih[2], ih[3]});
    const bf8 bil = __builtin_bit_cast(bf8, u4{il[0], il[1], il[2], il[3]});
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const bf8 ah = *reinterpret_cast<const bf8*>(&Cap[((0 * 2 + st) * kPL + 16 * m + li) * kCBS + 8 * lk]);
      const bf8 al = *reinterpret_cast<const bf8*>(&Cap[((1 * 2 + st) * kPL + 16 * m + li) * kCBS + 8 * lk]);
      // step 0 starts the accumulators from zero (an inline zero operand, no register fill)
      acc2[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brh, st == 0 ? f4{0, 0, 0, 0} : acc2[m][0], 0, 0, 0);
      acc2[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bih, st == 0 ? f4{0, 0, 0, 0} : acc2[m][1], 0, 0, 0);
      acc2[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brl, acc2[m][0], 0, 0, 0);
      acc2[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bil, acc2[m][1], 0, 0, 0);
      acc2[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, brh, acc2[m][0], 0, 0, 0);
      acc2[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bih, acc2[m][1], 0, 0, 0);
    }
  };

  const long long per = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per;
  const long long bend = bbeg + per < q.nblocks ? bbeg + per : q.nblocks;
  Blk cur;
  blk_start<LIST>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  blk_fill<LIST>(cur, q);
  Blk nxt = cur, nn = cur;
  blk_step<LIST>(nxt, q);
  blk_fill<LIST>(nxt, q);
  blk_step<LIST>(nn, q);
  blk_step<LIST>(nn, q);
  if (bbeg < bend) {
    fetch(cur, 0, kWBU);
    fetch_x(cur);
    stash(cur.mt);
  }
  __syncthreads();
  for (long long blk = bbeg; blk < bend; ++blk) {
    const Blk k = cur;
    const int oA = k.oa.y, oB = k.ob.y;
    const bool more = blk + 1 < bend;
    // the next block's W: the first half of its rows now, the second half once this block's
    // products are done (so that they do not hold registers through the products)
    if (more) {
      fetch(nxt, 0, kWBU / 2);
      fetch_x(nxt);
    }
    Blk nf = nn;
    blk_fill<LIST>(nf, q);
    f4 acc2[3][2];  // set by the products (product wavefronts only)
    if (mm) {
      // the product wavefronts issue ahead of staging and unfold work on their SIMD
      __builtin_amdgcn_s_setprio(1);
      f4 zr0, zi0, zr1, zi1;
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        gemm1(2 * st, zr0, zi0);
        gemm1(2 * st + 1, zr1, zi1);
        gemm2(st, zr0, zi0, zr1, zi1, acc2);
        __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    if (more) fetch(nxt, kWBU / 2, kWBU);
    __syncthreads();  // every wavefront is done with W
    if (mm) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          Ks[(16 * m + 4 * lk + j) * kKS + 16 * w + li] = make_float2(acc2[m][0][j], acc2[m][1][j]);
    }
    __syncthreads();
    double sr = 0, si = 0;
    const bool live = lane < 63 && uo < q.nA * q.nB;
    if (live) {
      const int a = uo / q.nB, bb = uo - a * q.nB;
      // columns b' >= n_B and rows a' >= n_A meet zeros of X; their K indices are clamped
      // to a valid entry
      int pb[9];
#pragma unroll
      for (int bp = 0; bp < 9; ++bp) pb[bp] = pair_index(bb, bp < q.nB ? bp : q.nB - 1, q.nB);
      // lane third uh sums rows a' = 3 uh .. 3 uh + 2 (27 products) in FP32, two interleaved
      // partial sums each for re and im, and the thirds meet in FP64: the split products carry
      // about 2^-16 relative error, far above the FP32 rounding of a 27-term sum
      float pr[2] = {0.f, 0.f}, pi[2] = {0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int ap = 3 * uh + i;
        const float2* Kr = Ks + pair_index(a, ap < q.nA ? ap : q.nA - 1, q.nA) * kKS;
        const float2* Xr = Xs + 9 * ap;
#pragma unroll
        for (int bp = 0; bp < 9; ++bp) {
          const float2 kv = Kr[pb[bp]], x = Xr[bp];
          pr[bp & 1] = fmaf(kv.x, x.x, fmaf(-kv.y, x.y, pr[bp & 1]));
          pi[bp & 1] = fmaf(kv.x, x.y, fmaf(kv.y, x.x, pi[bp & 1]));
        }
      }
      sr = (double)pr[0] + (double)pr[1];
      si = (double)pi[0] + (double)pi[1];
    }
    // the three thirds meet in the first lane of the triple
    sr += __shfl_down(sr, 1) + __shfl_down(sr, 2);
    si += __shfl_down(si, 1) + __shfl_down(si, 2);
    __syncthreads();  // K and X no longer read
    if (more) stash(nxt.mt);
    if (live && uh == 0) {
      const int a = uo / q.nB, bb = uo - a * q.nB;
      S[((long long)k.t * q.NR + k.R) * sl + (long long)(oA + a) * q.No + oB + bb] = make_double2(-sr, -si);
    }
    cur = nxt;
    nxt = nf;
    blk_step<LIST>(nn, q);
    __syncthreads();
  }
}

// Both walks ask for three wavefronts per SIMD (three workgroups per CU, 52.9 KB of LDS each):
// the allocator fits them in 168 registers without spilling.
template <bool W16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void s_bf16x3(
    const float2* __restrict__ GR, const float2* __restrict__ WR, double2* __restrict__ S,
    const float* __restrict__ CpA, const float* __restrict__ CpB, const PairArgs q) {
  s_bf16x3_body<false, W16>(GR, WR, S, CpA, CpB, q);
}
template <bool W16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void s_bf16x3_list(
    const float2* __restrict__ GR, const float2* __restrict__ WR, double2* __restrict__ S,
    const float* __restrict__ CpA, const float* __restrict__ CpB, const PairArgs q) {
  s_bf16x3_body<true, W16>(GR, WR, S, CpA, CpB, q);
}

// ---------------------------------------------------------------------------
// General block shapes (up to 16 orbitals and 128 product functions on either atom), on the
// FP32 or FP64 matrix cores.  One workgroup of 8 wavefronts per compute unit walks a
// contiguous range of blocks.
//
// Polarizability: the pair-folded form of p_mfma, P = -g C~_A Q C~_B^T, with Q (up to 144 x 144
// pairs) formed and consumed 16 columns p' at a time so that it never has to sit in LDS whole:
// per column chunk, Q[:, chunk] is formed from the G tiles, GEMM1 gives
// D1[p'][I] = sum_p Q[p][p'] C~_A[I][p] (wavefront w: I tile w, K = np_pad(A)), and GEMM2
// accumulates acc[J][I] += sum_{p' in chunk} C~_B[J][p'] D1[p'][I] from D1 in registers.
// The tau mirror and the two stores are those of p_mfma; the direct block goes through a
// per-wavefront LDS tile so that its rows leave as contiguous runs.
// ---------------------------------------------------------------------------
// Block walk of the general kernels: dense (every (tau, R, iA, iB), B fastest) or, with PACK,
// (tau, kept block of the cutoff list) with the block's packed offsets: list entry i is
// (R, mA | mB << 16, first product function of A, first orbital of A),
// (first product function of B, first orbital of B, packed offset of (R, A, B), packed offset
// of its mirror (-R, B, A)) -- offsets within one tau slice of the packed layout, where a kept
// block is stored as its mA x mB functions, row-major.
struct GBlk {
  int t, R, iA, iB;
  int2 oa, ob;
  int mt, od, om;
};

template <bool PACK>
__device__ __forceinline__ void gblk_start(GBlk& k, long long b, const PairArgs& q) {
  if constexpr (PACK) {
    k.t = (int)(b / q.nlist);
    k.iA = (int)(b - (long long)k.t * q.nlist);
    k.iB = 0;
    k.R = 0;
  } else {
    k.iB = (int)(b % q.cntB);
    b /= q.cntB;
    k.iA = (int)(b % q.cntA);
    b /= q.cntA;
    k.R = (int)(b % q.NR);
    k.t = (int)(b / q.NR);
  }
}

template <bool PACK>
__device__ __forceinline__ void gblk_step(GBlk& k, const PairArgs& q) {
  if constexpr (PACK) {
    if (++k.iA == q.nlist) {
      k.iA = 0;
      ++k.t;
    }
  } else {
    if (++k.iB == q.cntB) {
      k.iB = 0;
      if (++k.iA == q.cntA) {
        k.iA = 0;
        if (++k.R == q.NR) {
          k.R = 0;
          ++k.t;
        }
      }
    }
  }
}

template <bool PACK>
__device__ __forceinline__ void gblk_fill(GBlk& k, const PairArgs& q) {
  if constexpr (PACK) {
    const int4 e0 = q.list[2 * k.iA], e1 = q.list[2 * k.iA + 1];
    k.R = e0.x;
    k.mt = e0.y;
    k.oa = make_int2(e0.z, e0.w);
    k.ob = make_int2(e1.x, e1.y);
    k.od = e1.z;
    k.om = e1.w;
  } else {
    k.oa = q.offsA[k.iA < q.cntA ? k.iA : 0];
    k.ob = q.offsB[k.iB < q.cntB ? k.iB : 0];
    k.mt = q.mA | (q.mB << 16);
    k.od = k.om = 0;
  }
}

constexpr int kGPL = 144;           // padded pair count bound (16 orbitals: 136 pairs)
constexpr int kGKA = kGPL / 4;      // GEMM1 K steps at most
constexpr int kGMP = 128;           // padded product-function bound
constexpr int kGJT = kGMP / 16;     // J tiles at most
constexpr int kGS = 17;             // row stride (elements) of the 16-wide LDS chunks
constexpr int kGThreads = 512;

template <class RT, class CT, bool PACK = false>
__global__ __launch_bounds__(512) void p_mfma_gen(const CT* __restrict__ GR, CT* __restrict__ P,
                                                  const RT* __restrict__ CpA, const RT* __restrict__ CpB,
                                                  const PairArgs q, double g) {
  using M = Mma<RT>;
  typedef typename M::cplx CR;
  __shared__ CR Xs[kMaxOrb * kMaxOrb], Ys[kMaxOrb * kMaxOrb];
  __shared__ CR Qc[kGPL * kGS];           // Q[p][p' - 16 c]
  __shared__ RT Cb[kGMP * kGS];           // C~_B[J][p' - 16 c]
  __shared__ CR Tt[8 * 16 * kGS];         // per wavefront: the direct block's 16 x 16 tile
  __shared__ unsigned char ta[kMaxPairs], tb[kMaxPairs], tc[kMaxPairs], td[kMaxPairs];
  __shared__ int mRs[kMaxR];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  for (int i = tid; i < q.npA; i += kGThreads) pair_of(i, q.nA, ta[i], tb[i]);
  for (int i = tid; i < q.npB; i += kGThreads) pair_of(i, q.nB, tc[i], td[i]);
  for (int i = tid; i < q.NR; i += kGThreads) mRs[i] = q.minusR[i];
  const int nKA = q.nppA / 4, nCh = q.nppB / 16, nJT = (q.mB + 15) / 16;
  const bool act = 16 * w < q.mA;  // this wavefront owns I tile w
  // GEMM1 B operand: lane (k = lk, n = li) holds C~_A[I = 16 w + li][p = 4 ks + lk]; kept in
  // registers for FP32, read from the (cache-resident) table at each use for FP64, whose
  // accumulators leave no room for it
  constexpr bool kRegB = sizeof(RT) == 4;
  RT b1[kRegB ? kGKA : 1];
  const RT* CpArow = CpA + (act ? (16 * w + li) * q.nppA : 0) + lk;
  if constexpr (kRegB) {
#pragma unroll
    for (int ks = 0; ks < kGKA; ++ks) b1[ks] = (act && ks < nKA) ? CpArow[4 * ks] : RT(0);
  }
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  CT xr, yr;
  const bool xok = tid < q.nA * q.nB;
  auto fetch = [&](const GBlk& k) {
    const int a = tid / q.nB, c = tid - a * q.nB;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR, xok);
    const int d = tid / q.nA, bb = tid - d * q.nA;
    yr = ldraw(GR + ((long long)(q.n_tau - 1 - k.t) * q.NR + mRs[k.R]) * sl + (long long)(k.ob.y + d) * q.No +
                   k.oa.y + bb,
               GR, xok);
  };
  auto stage = [&]() {
    if (xok) {
      Xs[tid] = mk<RT>((double)xr.x, (double)xr.y);
      Ys[tid] = mk<RT>((double)yr.x, (double)yr.y);
    }
  };
  const long long per = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per;
  const long long bend = bbeg + per < q.nblocks ? bbeg + per : q.nblocks;
  // dense: band walk; packed block list: its contiguous range
  auto adv = [&](GBlk& x) {
    if constexpr (PACK)
      gblk_step<true>(x, q);
    else
      bblk_step(x, q);
  };
  GBlk cur;
  if constexpr (PACK)
    gblk_start<true>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  else
    bblk_start(cur, bbeg < q.nblocks ? bbeg : 0, q);
  gblk_fill<PACK>(cur, q);
  GBlk nxt = cur;
  adv(nxt);
  __syncthreads();  // pair tables and the minus-R table staged
  if (bbeg < bend) {
    fetch(cur);
    stage();
  }
  __syncthreads();
  for (long long blk = bbeg; blk < bend; ++blk) {
    const GBlk k = cur;
    const int t = k.t, tm = q.n_tau - 1 - t, mR = mRs[k.R];
    const int pA = k.oa.x, pB = k.ob.x;
    // functions kept on A and B (all of them when dense): I tiles and J tiles of the block
    const int kA = k.mt & 0xffff, kB = k.mt >> 16;
    const bool actk = act && 16 * w < kA;
    const int nJTk = PACK ? (kB + 15) / 16 : nJT;
    const bool more = blk + 1 < bend;
    if (more) {
      gblk_fill<PACK>(nxt, q);
      fetch(nxt);
    }
    typename M::acc acc[kGJT][2];
#pragma unroll
    for (int Jt = 0; Jt < kGJT; ++Jt) acc[Jt][0] = acc[Jt][1] = typename M::acc{0, 0, 0, 0};
    for (int ch = 0; ch < nCh; ++ch) {
      // Q[p][16 ch + pc] (zero outside the live pairs) and the matching columns of C~_B
      for (int i = tid; i < q.nppA * 16; i += kGThreads) {
        const int p = i >> 4, pc = i & 15, pp = 16 * ch + pc;
        RT qr = 0, qi = 0;
        if (p < q.npA && pp < q.npB) {
          const int a = ta[p], bq = tb[p], c = tc[pp], d = td[pp];
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int c1 = s2 ? d : c, d1 = s2 ? c : d;
            if (s2 == 1 && c == d) break;
            CR x = Xs[a * q.nB + c1], y = Ys[d1 * q.nA + bq];
            qr += x.x * y.x - x.y * y.y;
            qi += x.x * y.y + x.y * y.x;
            if (a != bq) {
              x = Xs[bq * q.nB + c1];
              y = Ys[d1 * q.nA + a];
              qr += x.x * y.x - x.y * y.y;
              qi += x.x * y.y + x.y * y.x;
            }
          }
        }
        Qc[p * kGS + pc] = mk<RT>(qr, qi);
      }
      for (int i = tid; i < q.mpB * 16; i += kGThreads) {
        const int J = i >> 4, pc = i & 15;
        Cb[J * kGS + pc] = CpB[J * q.nppB + 16 * ch + pc];
      }
      __syncthreads();
      if (actk) {
        // GEMM1: A = Q^T (row p' = li, k = p), two chains (Re Q, Im Q)
        typename M::acc d1r = {0, 0, 0, 0}, d1i = {0, 0, 0, 0};
        // four K steps per uniform branch, their reads issued together (n_KA is a multiple of 4)
#pragma unroll
        for (int g = 0; g < kGKA / 4; ++g)
          if (4 * g < nKA) {
            CR qv[4];
            RT bv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int ks = 4 * g + e;
              qv[e] = Qc[(4 * ks + lk) * kGS + li];
              if constexpr (kRegB)
                bv[e] = b1[ks];
              else
                bv[e] = CpArow[4 * ks];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              d1r = M::op(qv[e].x, bv[e], d1r);
              d1i = M::op(qv[e].y, bv[e], d1i);
            }
          }
        // GEMM2: K = p' of the chunk, step j takes row drow(lk, j) of D1 (register j); one
        // branch per J tile, its four C~_B reads issued together
#pragma unroll
        for (int Jt = 0; Jt < kGJT; ++Jt)
          if (Jt < nJTk) {
            RT a[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = Cb[(16 * Jt + li) * kGS + M::drow(lk, j)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              acc[Jt][0] = M::op(a[j], d1r[j], acc[Jt][0]);
              acc[Jt][1] = M::op(a[j], d1i[j], acc[Jt][1]);
            }
          }
      }
      __syncthreads();  // Qc and Cb are rewritten by the next chunk
    }
    // acc[Jt][part][j]: row J = 16 Jt + drow(lk, j), column I = 16 w + li; P_IJ = -g acc.
    // Dense: P[t][R][pA + I][pB + J] and the mirror P[tm][-R][pB + J][pA + I].  Packed: the
    // block's kA x kB functions at its offset in slice t, and the mirror block's kB x kA at its
    // offset in slice tm.
    if (actk) {
      CT* Pd = PACK ? P + (long long)t * q.ptot + k.od : P + ((long long)t * q.NR + k.R) * slp;
      CT* Pm = PACK ? P + (long long)tm * q.ptot + k.om : P + ((long long)tm * q.NR + mR) * slp;
      const long long sd = PACK ? kB : q.Np, sm = PACK ? kA : q.Np;  // row strides
      const int cd = PACK ? 0 : pB, rd = PACK ? 0 : pA;               // column / row origins
      const int I = 16 * w + li;
      CR* Tw = Tt + w * 16 * kGS;
#pragma unroll
      for (int Jt = 0; Jt < kGJT; ++Jt)
        if (Jt < nJTk) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int Jl = M::drow(lk, j), J = 16 * Jt + Jl;
            const double re = -g * (double)acc[Jt][0][j], im = -g * (double)acc[Jt][1][j];
            Tw[li * kGS + Jl] = mk<RT>(re, im);
            if (t != tm && I < kA && J < kB) stc(Pm + (long long)(cd + J) * sm + rd + I, re, im);
          }
          // the wavefront's own tile: lanes 16 r .. 16 r + 15 store row 4 e + r, 16 consecutive J
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 4 * e + lk, J = 16 * Jt + li, Ir = 16 * w + r;
            const CR v = Tw[r * kGS + li];
            if (Ir < kA && J < kB) stc(Pd + (long long)(rd + Ir) * sd + cd + J, (double)v.x, (double)v.y);
          }
        }
    }
    if (more) stage();  // Xs, Ys were last read before the chunk loop's final barrier
    cur = nxt;
    adv(nxt);
    __syncthreads();
  }
}

// Self-energy for the same general shapes, without the pair folding and its vector-ALU
// unfold: the sum runs as three chained matrix products per chunk of 16 product functions J
// of atom B,
//   M[a'][J][b]  = sum_{b'} X[a'][b'] C^J_{b'b}                      (K = b')
//   L^T[J][a]    = sum_I W[I][J] C^I_{a a'}          for each a'      (K = I)
//   S^T[b][a]   += sum_J M[a'][J][b] L^T[J][a]       for each a'      (K = J, complex x complex)
// (Eq. (8) with C symmetric in its orbital pair).  M goes through LDS, L^T stays in registers
// (the D fragment of its product is the B operand of the next), the chunk of W is staged in
// LDS with row loads.  Wavefront w owns the orbitals a' = w and a' = w + 8 of atom A and keeps
// one accumulator per a'; the sum over a' and over the wavefronts is taken in FP64.  With nine
// orbitals on A the ninth a' would fall to wavefront 0 alone, doubling its products: the second
// slot then takes a' = 8 for the chunks ch with ch mod 8 = w on every wavefront instead (an
// accumulator may mix a', whose contributions are summed anyway).
// ---------------------------------------------------------------------------
template <class RT, class CT, bool PACK = false>
__global__ __launch_bounds__(512) void s_mfma_gen(const CT* __restrict__ GR, const CT* __restrict__ WR,
                                                  double2* __restrict__ S, const RT* __restrict__ CA,
                                                  const RT* __restrict__ CB, const PairArgs q) {
  using M = Mma<RT>;
  typedef typename M::cplx CR;
  constexpr int kGKI = kGMP / 4;           // K steps over I at most
  constexpr int kWU = kGMP * 16 / kGThreads;  // W values of a chunk per thread
  // FP32 keeps two slots of M and of the W chunk (chunk ch in slot ch & 1), so that one barrier
  // per chunk separates its writes from its reads; FP64 (twice the bytes) keeps one slot and
  // three barriers per chunk
  constexpr bool kDB = sizeof(RT) == 4;
  constexpr int kNB = kDB ? 2 : 1;
  __shared__ CR Xs[kMaxOrb * kMaxOrb];     // X[a'][b'], 16 x 16 zero padded
  __shared__ CR Ms[kNB][16 * 16 * kGS];    // M[a'][J - 16 c][b] (row stride kGS)
  __shared__ CR Wc[kNB][kGMP * kGS];       // W[I][J - 16 c]
  __shared__ double2 Spart[kGThreads / 64][kMaxOrb * kMaxOrb];  // per-wavefront partial sums of S
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int nA = q.nA, nB = q.nB, mA = q.mA, mB = q.mB;
  const int nKI = q.mpA / 4, nCh = (mB + 15) / 16;
  const long long sl = (long long)q.No * q.No, slp = (long long)q.Np * q.Np;
  // L's B operand, the same for every block: lane (k = lk, n = a = li) holds C^I_{a a'} for
  // I = 4 ks + lk and the two orbitals a' = w, w + 8 this wavefront owns.  Kept in registers for
  // FP32; FP64 reads it from the (cache-resident) table at each use, its registers being full.
  constexpr bool kRegC = sizeof(RT) == 4;
  // second slot's a' (nine orbitals: a' = 8 on every wavefront, for its share of the chunks)
  const bool rot9 = nA == 9;
  const int ap2 = rot9 ? 8 : w + 8;
  auto ca = [&](int ks, int u) -> RT {
    const int I = 4 * ks + lk, ap = u == 0 ? w : ap2;
    return (ks < nKI && I < mA && li < nA && ap < nA) ? CA[((long long)I * nA + li) * nA + ap] : RT(0);
  };
  RT cav[2][kRegC ? kGKI : 1];
  if constexpr (kRegC) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int ks = 0; ks < kGKI; ++ks) cav[u][ks] = ca(ks, u);
  }
  const long long per_blk = (q.nblocks + gridDim.x - 1) / gridDim.x;
  const long long bbeg = (long long)blockIdx.x * per_blk;
  const long long bend = bbeg + per_blk < q.nblocks ? bbeg + per_blk : q.nblocks;
  // The W chunk (and, with the first chunk, the X tile) that is staged next is loaded into
  // registers a whole chunk ahead; a block's first chunk is loaded during the previous block's last.
  CT wreg[kWU], xr;
  auto wsrc = [&](const GBlk& k, long long& ws) -> const CT* {
    ws = PACK ? (k.mt >> 16) : q.Np;
    return PACK ? WR + (long long)k.t * q.ptot + k.od
                : WR + ((long long)k.t * q.NR + k.R) * slp + (long long)k.oa.x * q.Np + k.ob.x;
  };
  auto load_w = [&](const GBlk& k, int ch) {
    long long ws;
    const CT* Wt = wsrc(k, ws);
    const int kA = k.mt & 0xffff, kB = k.mt >> 16, J0 = 16 * ch;
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      const int i = tid + kGThreads * u, I = i >> 4, Jl = i & 15;
      wreg[u] = ldraw(Wt + (long long)I * ws + J0 + Jl, WR, I < kA && J0 + Jl < kB);
    }
  };
  auto load_x = [&](const GBlk& k) {
    const int a = (tid & 255) >> 4, c = tid & 15;
    xr = ldraw(GR + ((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + c, GR,
               tid < 256 && a < nA && c < nB);
  };
  auto store_w = [&](const GBlk& k, int ch, int sb) {
    const int kA = k.mt & 0xffff, kB = k.mt >> 16, J0 = 16 * ch;
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      const int i = tid + kGThreads * u, I = i >> 4, Jl = i & 15;
      const CT v = keep(wreg[u], I < kA && J0 + Jl < kB);
      Wc[sb][I * kGS + Jl] = mk<RT>((double)v.x, (double)v.y);
    }
  };
  auto store_x = [&](const GBlk& k) {
    if (tid < 256) {
      const int a = tid >> 4, c = tid & 15;
      const CT v = keep(xr, a < nA && c < nB);
      Xs[tid] = mk<RT>((double)v.x, (double)v.y);
    }
  };
  // C^J operands of the M products (lane: J = 16 ch + 2 w + h, b' = 4 ks + lk, b = li); the same
  // for every block, loaded one chunk ahead
  RT cbr[2][4], cbn[2][4];
  auto load_cb = [&](int ch, RT (&dst)[2][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int J = 16 * ch + 2 * w + h, bp = 4 * ks + lk;
        dst[h][ks] = (J < mB && bp < nB && li < nB) ? CB[((long long)J * nB + bp) * nB + li] : RT(0);
      }
  };
  load_cb(0, cbr);
  GBlk cur;
  gblk_start<PACK>(cur, bbeg < q.nblocks ? bbeg : 0, q);
  gblk_fill<PACK>(cur, q);
  GBlk nxt = cur;
  gblk_step<PACK>(nxt, q);
  if (bbeg < bend) {
    load_w(cur, 0);
    load_x(cur);
  }
  if constexpr (kDB) {  // the first block's X; later blocks' are staged at the previous block's end
    if (bbeg < bend) store_x(cur);
    __syncthreads();
  }
  for (long long blk = bbeg; blk < bend; ++blk) {
    const GBlk k = cur;
    const bool more = blk + 1 < bend;
    if (more) gblk_fill<PACK>(nxt, q);
    const int kA = k.mt & 0xffff, kB = k.mt >> 16;
    typename M::acc sr[2], si[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) sr[u] = si[u] = typename M::acc{0, 0, 0, 0};
    // W is zero beyond the block's functions: fewer chunks of J and K steps over I
    const int nChk = PACK ? (kB + 15) / 16 : nCh, nKIk = PACK ? (kA + 3) / 4 : nKI;
    for (int ch = 0; ch < nChk; ++ch) {
      const int J0 = 16 * ch, sb = kDB ? (ch & 1) : 0;
      // Two slots: slot sb was last read by chunk ch - 2, before every wavefront passed chunk
      // ch - 1's barrier (or, at ch < 2, before the previous block's closing barriers)
      store_w(k, ch, sb);
      if constexpr (!kDB) {
        if (ch == 0) store_x(k);
        __syncthreads();  // Xs (first chunk) and Wc staged; Ms free
      }
      if (ch + 1 < nChk) {
        load_w(k, ch + 1);
      } else if (more) {
        load_w(nxt, 0);
        load_x(nxt);
      }
      load_cb(ch + 1 < nChk ? ch + 1 : 0, cbn);
      // M[a'][J][b] for J = J0 + 2 w, J0 + 2 w + 1: A = X (row a' = li, k = b'),
      // B = C^J (k = b', n = b = li)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int Jl = 2 * w + h, J = J0 + Jl;
        typename M::acc mr = {0, 0, 0, 0}, mi = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const CR x = Xs[li * 16 + 4 * ks + lk];
          mr = M::op(x.x, cbr[h][ks], mr);
          mi = M::op(x.y, cbr[h][ks], mi);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          Ms[sb][(M::drow(lk, j) * 16 + Jl) * kGS + li] = mk<RT>((double)mr[j], (double)mi[j]);
      }
      __syncthreads();  // Ms and Wc of this chunk staged
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ap = u == 0 ? w : ap2;
        if (ap < nA && (u == 0 || !rot9 || (ch & 7) == w)) {
          // L^T[J][a] = sum_I W[I][J] C^I_{a a'}: A = W^T (row J = li, k = I), two chains
          typename M::acc lr = {0, 0, 0, 0}, lim = {0, 0, 0, 0};
          if constexpr (kRegC) {
            // four K steps per uniform branch, their W reads issued together (one LDS wait per
            // group instead of one per step); rows past the block's functions are zero in Wc
#pragma unroll
            for (int g = 0; g < kGKI / 4; ++g)
              if (4 * g < nKIk) {
                CR wv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) wv[e] = Wc[sb][(4 * (4 * g + e) + lk) * kGS + li];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  lr = M::op(wv[e].x, cav[u][4 * g + e], lr);
                  lim = M::op(wv[e].y, cav[u][4 * g + e], lim);
                }
              }
          } else {
            // the same groups of four, with C read from the table (zero past its rows)
            for (int g = 0; 4 * g < nKIk; ++g) {
              CR wv[4];
              RT cv[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                wv[e] = Wc[sb][(4 * (4 * g + e) + lk) * kGS + li];
                cv[e] = ca(4 * g + e, u);
              }
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                lr = M::op(wv[e].x, cv[e], lr);
                lim = M::op(wv[e].y, cv[e], lim);
              }
            }
          }
          // S^T[b][a] += sum_J M[a'][J][b] L^T[J][a]; step j: J = J0 + drow(lk, j)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const CR mv = Ms[sb][(ap * 16 + M::drow(lk, j)) * kGS + li];
            sr[u] = M::op(mv.x, lr[j], sr[u]);
            sr[u] = M::op(-mv.y, lim[j], sr[u]);
            si[u] = M::op(mv.x, lim[j], si[u]);
            si[u] = M::op(mv.y, lr[j], si[u]);
          }
        }
      }
      if constexpr (!kDB) __syncthreads();  // Wc and Ms are rewritten by the next chunk
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) cbr[h][ks] = cbn[h][ks];
    }
    // S_ab = -sum over a' of the accumulators (row b = drow(lk, j), column a = li), in FP64: each
    // wavefront adds its two a' and leaves one partial per element, then 256 threads add the 8
    // partials
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {  // a slot that took no a' holds zeros
        vr += (double)sr[u][j];
        vi += (double)si[u][j];
      }
      Spart[w][li * 16 + M::drow(lk, j)] = make_double2(vr, vi);
    }
    // two slots: the next block's X, loaded with this block's last chunk (every wavefront is
    // past that chunk's barrier, so no one reads Xs any more)
    if constexpr (kDB) {
      if (more) store_x(nxt);
    }
    __syncthreads();
    if (tid < 256) {
      const int a = tid >> 4, b = tid & 15;
      if (a < nA && b < nB) {
        double vr = 0.0, vi = 0.0;
#pragma unroll
        for (int r = 0; r < kGThreads / 64; ++r) {
          vr += Spart[r][tid].x;
          vi += Spart[r][tid].y;
        }
        S[((long long)k.t * q.NR + k.R) * sl + (long long)(k.oa.y + a) * q.No + k.ob.y + b] = make_double2(-vr, -vi);
      }
    }
    cur = nxt;
    gblk_step<PACK>(nxt, q);
    __syncthreads();  // Xs and Spart are rewritten by the next block
  }
}

PairArgs make_args(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, int n_half) {
  PairArgs q;
  q.nA = A.n;
  q.nB = B.n;
  q.mA = A.m;
  q.mB = B.m;
  q.npA = A.np;
  q.npB = B.np;
  q.nppA = A.np_pad;
  q.nppB = B.np_pad;
  q.mpA = A.m_pad;
  q.mpB = B.m_pad;
  q.atomsA = A.atoms_dev;
  q.offsA = A.offs_dev;
  q.offsB = B.offs_dev;
  q.cntA = (int)A.atoms.size();
  q.atomsB = B.atoms_dev;
  q.cntB = (int)B.atoms.size();
  q.orb_off = c->orb_off_dev;
  q.pb_off = c->pb_off_dev;
  q.minusR = c->minusR_dev;
  q.NR = c->N_R;
  q.n_tau = c->n_tau;
  q.n_half = n_half;
  q.No = c->N_orb;
  q.Np = c->N_pb;
  q.nblocks = (long long)n_half * c->N_R * q.cntA * q.cntB;
  q.list = nullptr;
  q.nlist = 0;
  q.ptot = 0;
  return q;
}

// Whether the BF16 self-energy may load W column pairs as 16-byte accesses (its W16)
bool w_rows16(const gw_cell* c, const void* WR) {
  if (reinterpret_cast<uintptr_t>(WR) & 15) return false;
  for (const SpeciesDev& s : c->sp)
    if (s.m & 1) return false;
  return true;
}

unsigned grid_for(long long nblocks) { return (unsigned)(nblocks < 2048 ? nblocks : 2048); }

}  // namespace

bool mfma_pair_ok(const SpeciesDev& A, const SpeciesDev& B) {
  return A.np_pad <= kPL && B.np_pad <= kPL && A.m_pad <= kMP && B.m_pad <= kMP;
}

void launch_p_mfma_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                        double g, gw_precision p, hipStream_t s) {
  const PairArgs q = make_args(c, A, B, (c->n_tau + 1) / 2);
  if (q.nblocks == 0) return;
  const int sh = (A.np_pad == 48 && B.np_pad == 48 && A.m_pad == 64 && (B.m + 15) / 16 == 4)   ? 1
                 : (A.np_pad == 16 && B.np_pad == 16 && A.m_pad == 16 && (B.m + 15) / 16 == 1) ? 2
                                                                                              : 0;
  const dim3 grid(grid_for(q.nblocks)), block(256);
#define GWR_P(RT, CT, SHV, CA, CB)                                                                  \
  hipLaunchKernelGGL((p_mfma<RT, CT, SHV>), grid, block, 0, s, (const CT*)GR, (CT*)P, CA, CB, q, g)
  if (p == GW_BF16X3 && sh == 1) {
    hipLaunchKernelGGL(p_bf16x3, grid, block, 0, s, (const float2*)GR, (float2*)P, A.Cpair32, B.Cpair32, q, g);
  } else if (p == GW_FP64) {
    if (sh == 1)
      GWR_P(double, double2, 1, A.Cpair, B.Cpair);
    else if (sh == 2)
      GWR_P(double, double2, 2, A.Cpair, B.Cpair);
    else
      GWR_P(double, double2, 0, A.Cpair, B.Cpair);
  } else {
    if (sh == 1)
      GWR_P(float, float2, 1, A.Cpair32, B.Cpair32);
    else if (sh == 2)
      GWR_P(float, float2, 2, A.Cpair32, B.Cpair32);
    else
      GWR_P(float, float2, 0, A.Cpair32, B.Cpair32);
  }
#undef GWR_P
}

void launch_s_mfma_pair(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR,
                        const void* WR, void* S, gw_precision p, hipStream_t s, int nt) {
  const PairArgs q = make_args(c, A, B, nt);
  if (q.nblocks == 0) return;
  const unsigned threads = kSThreads;
  // s_mfma32 holds three workgroups per compute unit: two full rounds of them
  const long long g32 = 6LL * c->n_cu;
  const unsigned grid32 = (unsigned)(q.nblocks < g32 ? q.nblocks : g32);
  if (p == GW_FP64)
    hipLaunchKernelGGL((s_mfma<double, double2>), dim3(grid_for(q.nblocks)), dim3(threads), 0, s,
                       (const double2*)GR, (const double2*)WR, (double2*)S, A.Cpair, B.Cpair, q);
  else if (p == GW_BF16X3 && A.m_pad == 64 && B.m_pad == 64 && A.np_pad == 48)
    hipLaunchKernelGGL(w_rows16(c, WR) ? s_bf16x3<true> : s_bf16x3<false>, dim3(grid32), dim3(kSBThreads), 0, s,
                       (const float2*)GR, (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  else if (A.m_pad == 64 && B.m_pad == 64 && A.np_pad == 48)  // n = 9 with m in (48, 64]: the Si-like species
    hipLaunchKernelGGL((s_mfma32<4, 16, 3>), dim3(grid32), dim3(kS32Threads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  else if (A.m_pad == 16 && B.m_pad == 16 && A.np_pad == 16)  // up to 5 orbitals and 16 product functions
    hipLaunchKernelGGL((s_mfma32<1, 4, 1>), dim3(grid32), dim3(kS32Threads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  else
    hipLaunchKernelGGL((s_mfma<float, float2>), dim3(grid_for(q.nblocks)), dim3(threads), 0, s,
                       (const float2*)GR, (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
}

// The same kernels over a block list of the real-space cutoff (entries as in PairArgs::list),
// for every shape and precision the dense launchers handle (the caller uses the plain
// kernels for shapes outside mfma_pair_ok).
bool launch_p_mfma_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                        const void* GR, void* P, double g, gw_precision p, hipStream_t s) {
  PairArgs q = make_args(c, A, B, (c->n_tau + 1) / 2);
  q.list = list;
  q.nlist = n;
  q.nblocks = (long long)q.n_half * n;
  if (q.nblocks == 0) return true;
  const int sh = (A.np_pad == 48 && B.np_pad == 48 && A.m_pad == 64 && (B.m + 15) / 16 == 4)   ? 1
                 : (A.np_pad == 16 && B.np_pad == 16 && A.m_pad == 16 && (B.m + 15) / 16 == 1) ? 2
                                                                                              : 0;
  const dim3 grid(grid_for(q.nblocks)), block(256);
#define GWR_P(RT, CT, SHV, CA, CB)                                                                  \
  hipLaunchKernelGGL((p_mfma<RT, CT, SHV, true>), grid, block, 0, s, (const CT*)GR, (CT*)P, CA, CB, q, g)
  if (p == GW_BF16X3 && sh == 1) {
    hipLaunchKernelGGL(p_bf16x3<true>, grid, block, 0, s, (const float2*)GR, (float2*)P, A.Cpair32, B.Cpair32, q,
                       g);
  } else if (p == GW_FP64) {
    if (sh == 1)
      GWR_P(double, double2, 1, A.Cpair, B.Cpair);
    else if (sh == 2)
      GWR_P(double, double2, 2, A.Cpair, B.Cpair);
    else
      GWR_P(double, double2, 0, A.Cpair, B.Cpair);
  } else {
    if (sh == 1)
      GWR_P(float, float2, 1, A.Cpair32, B.Cpair32);
    else if (sh == 2)
      GWR_P(float, float2, 2, A.Cpair32, B.Cpair32);
    else
      GWR_P(float, float2, 0, A.Cpair32, B.Cpair32);
  }
#undef GWR_P
  return true;
}

bool launch_s_mfma_list(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                        const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s) {
  const bool si = A.m_pad == 64 && B.m_pad == 64 && A.np_pad == 48;
  const bool small = A.m_pad == 16 && B.m_pad == 16 && A.np_pad == 16;
  PairArgs q = make_args(c, A, B, c->n_tau);
  q.list = list;
  q.nlist = n;
  q.nblocks = (long long)c->n_tau * n;
  if (q.nblocks == 0) return true;
  const long long g32 = 6LL * c->n_cu;
  const unsigned grid32 = (unsigned)(q.nblocks < g32 ? q.nblocks : g32);
  if (p == GW_FP64)
    hipLaunchKernelGGL((s_mfma<double, double2, true>), dim3(grid_for(q.nblocks)), dim3(kSThreads), 0, s,
                       (const double2*)GR, (const double2*)WR, (double2*)S, A.Cpair, B.Cpair, q);
  else if (!si && !small)
    hipLaunchKernelGGL((s_mfma<float, float2, true>), dim3(grid_for(q.nblocks)), dim3(kSThreads), 0, s,
                       (const float2*)GR, (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  else if (p == GW_BF16X3 && si)
    hipLaunchKernelGGL(w_rows16(c, WR) ? s_bf16x3_list<true> : s_bf16x3_list<false>, dim3(grid32),
                       dim3(kSBThreads), 0, s, (const float2*)GR, (const float2*)WR, (double2*)S, A.Cpair32,
                       B.Cpair32, q);
  else if (si)
    hipLaunchKernelGGL((s_mfma32<4, 16, 3, true>), dim3(grid32), dim3(kS32Threads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  else
    hipLaunchKernelGGL((s_mfma32<1, 4, 1, true>), dim3(grid32), dim3(kS32Threads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.Cpair32, B.Cpair32, q);
  return true;
}

// The general kernels over the kept blocks of the cutoff list, packed layout (list entries with
// the packed offsets; ptot elements per tau slice).
void launch_p_mfma_packed(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                          long long ptot, const void* GR, void* P, double g, gw_precision p, hipStream_t s) {
  PairArgs q = make_args(c, A, B, (c->n_tau + 1) / 2);
  q.list = list;
  q.nlist = n;
  q.ptot = ptot;
  q.nblocks = (long long)q.n_half * n;
  if (q.nblocks == 0) return;
  const unsigned grid = (unsigned)(q.nblocks < c->n_cu ? q.nblocks : c->n_cu);
  if (p == GW_FP64)
    hipLaunchKernelGGL((p_mfma_gen<double, double2, true>), dim3(grid), dim3(kGThreads), 0, s, (const double2*)GR,
                       (double2*)P, A.Cpair, B.Cpair, q, g);
  else
    hipLaunchKernelGGL((p_mfma_gen<float, float2, true>), dim3(grid), dim3(kGThreads), 0, s, (const float2*)GR,
                       (float2*)P, A.Cpair32, B.Cpair32, q, g);
}

void launch_s_mfma_packed(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const int4* list, int n,
                          long long ptot, const void* GR, const void* WR, void* S, gw_precision p, hipStream_t s) {
  PairArgs q = make_args(c, A, B, c->n_tau);
  q.list = list;
  q.nlist = n;
  q.ptot = ptot;
  q.nblocks = (long long)c->n_tau * n;
  if (q.nblocks == 0) return;
  const long long cap = c->n_cu;
  const unsigned grid = (unsigned)(q.nblocks < cap ? q.nblocks : cap);
  if (p == GW_FP64)
    hipLaunchKernelGGL((s_mfma_gen<double, double2, true>), dim3(grid), dim3(kGThreads), 0, s, (const double2*)GR,
                       (const double2*)WR, (double2*)S, A.C, B.C, q);
  else
    hipLaunchKernelGGL((s_mfma_gen<float, float2, true>), dim3(grid), dim3(kGThreads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.C32, B.C32, q);
}

// General shapes on the matrix cores (one workgroup of 8 wavefronts per compute unit).
void launch_p_mfma_gen(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, void* P,
                       double g, gw_precision p, hipStream_t s) {
  const PairArgs q = make_args(c, A, B, (c->n_tau + 1) / 2);
  if (q.nblocks == 0) return;
  const unsigned grid = (unsigned)(q.nblocks < c->n_cu ? q.nblocks : c->n_cu);
  if (p == GW_FP64)
    hipLaunchKernelGGL((p_mfma_gen<double, double2>), dim3(grid), dim3(kGThreads), 0, s, (const double2*)GR,
                       (double2*)P, A.Cpair, B.Cpair, q, g);
  else
    hipLaunchKernelGGL((p_mfma_gen<float, float2>), dim3(grid), dim3(kGThreads), 0, s, (const float2*)GR,
                       (float2*)P, A.Cpair32, B.Cpair32, q, g);
}

void launch_s_mfma_gen(const gw_cell* c, const SpeciesDev& A, const SpeciesDev& B, const void* GR, const void* WR,
                       void* S, gw_precision p, hipStream_t s, int nt) {
  const PairArgs q = make_args(c, A, B, nt);
  if (q.nblocks == 0) return;
  // one workgroup of 8 wavefronts fills a compute unit's registers
  const long long cap = c->n_cu;
  const unsigned grid = (unsigned)(q.nblocks < cap ? q.nblocks : cap);
  if (p == GW_FP64)
    hipLaunchKernelGGL((s_mfma_gen<double, double2>), dim3(grid), dim3(kGThreads), 0, s, (const double2*)GR,
                       (const double2*)WR, (double2*)S, A.C, B.C, q);
  else
    hipLaunchKernelGGL((s_mfma_gen<float, float2>), dim3(grid), dim3(kGThreads), 0, s, (const float2*)GR,
                       (const float2*)WR, (double2*)S, A.C32, B.C32, q);
}

}  // namespace gwr


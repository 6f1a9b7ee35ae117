// Interstitial-grid blocks of P and Sigma, Eqs. (6), (7), (9), (10).  With one space argument on
// an interstitial grid point the MT contraction keeps only the coefficients of the muffin-tin
// side; with both on grid points it becomes an elementwise product.  Blocks per (tau, R):
//   G_og [N_orb][n_g] = G^R_{tL; r'},  G_go [n_g][N_orb] = G^R_{r; tL},  G_gg [n_g][n_g]
//   P_pg [N_pb][n_g], P_gp [n_g][N_pb], P_gg [n_g][n_g];  W likewise;  Sigma like G.
// All of it is memory-bound: the mixed blocks read one column (or row) of G per atom and grid
// point and run an m n^2 contraction on it in registers, the INT-INT blocks are Hadamard
// products (P's with the mirrored, transposed G through an LDS tile).  FP64 arithmetic.
#include "internal.h"

namespace gwr {
namespace {

constexpr int kGT = 32;    // LDS transpose tile of the INT-INT polarizability
constexpr int kCS = 4096;  // doubles of coefficients staged in LDS per pass (whole rows C^K)
constexpr int kMxN = 9, kMxLd = 109;  // p_mixed_mx: orbitals; LDS row stride of C (9 x 12 + 1)
// atoms whose P blocks with the grid run on the matrix cores (p_mixed_mx); the others on p_mixed
__device__ __forceinline__ bool mx_species(int n, int m) { return n <= kMxN && m <= 64; }

__device__ __forceinline__ double2 ld(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct IntArgs {
  int NR, n_tau, No, Np, ng;
  const int* minusR;
  const int* orb_off;   // per atom, n_atoms + 1
  const int* pb_off;
  const int* species;
  const double* C[8];   // per species, [m][n][n]
  int n[8], m[8];
};

// MT-INT and INT-MT blocks of P (Eq. (6) and its mirror partner).  Thread: grid point r;
// block: (256-point chunk, atom t, tau * NR + R); the atom's coefficients pass through LDS a
// few whole C^K at a time (every lane reads the same one: broadcast).
//   MODE 0: P_pg[t K][r] = -g sum_ab C^K_ab G_og[tau][R][t a][r] G_go[tau'][-R][r][t b]
//   MODE 1: P_gp[r][t K] = -g sum_cd G_go[tau][R][r][t c] G_og[tau'][-R][t d][r] C^K_cd
template <class T, int MODE>
__global__ __launch_bounds__(256) void p_mixed(const T* __restrict__ Gog, const T* __restrict__ Ggo, T* __restrict__ P,
                                               double g, const IntArgs q) {
  __shared__ double Cs[kCS];
  const int r = blockIdx.x * 256 + threadIdx.x, t = blockIdx.y;
  const int tau = blockIdx.z / q.NR, R = blockIdx.z - tau * q.NR;
  const bool on = r < q.ng;
  const int tm = q.n_tau - 1 - tau, mR = q.minusR[R];
  const int s = q.species[t], n = q.n[s], m = q.m[s], o = q.orb_off[t], pb = q.pb_off[t];
  if (mx_species(n, m)) return;  // p_mixed_mx covers this atom
  const double* C = q.C[s];
  const long long sl = (long long)q.No * q.ng;  // elements of one (tau, R) block of G_og or G_go
  double2 x[kMaxOrb], y[kMaxOrb];
#pragma unroll
  for (int a = 0; a < kMaxOrb; ++a) {
    if (on && a < n) {
      if (MODE == 0) {
        x[a] = ld(Gog + ((long long)tau * q.NR + R) * sl + (long long)(o + a) * q.ng + r);
        y[a] = ld(Ggo + ((long long)tm * q.NR + mR) * sl + (long long)r * q.No + o + a);
      } else {
        x[a] = ld(Ggo + ((long long)tau * q.NR + R) * sl + (long long)r * q.No + o + a);
        y[a] = ld(Gog + ((long long)tm * q.NR + mR) * sl + (long long)(o + a) * q.ng + r);
      }
    }
  }
  const long long pl = (long long)q.Np * q.ng;
  T* Pb = P + ((long long)tau * q.NR + R) * pl;
  const int nn = n * n, rows = kCS / nn;
  for (int K0 = 0; K0 < m; K0 += rows) {
    const int nk = m - K0 < rows ? m - K0 : rows;
    __syncthreads();
    for (int i = threadIdx.x; i < nk * nn; i += 256) Cs[i] = C[(long long)K0 * nn + i];
    __syncthreads();
    if (!on) continue;
    for (int k = 0; k < nk; ++k) {
      const double* CK = Cs + k * nn;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < kMaxOrb; ++a) {
        if (a < n) {
          double2 row = make_double2(0.0, 0.0);
#pragma unroll
          for (int b = 0; b < kMaxOrb; ++b) {
            if (b < n) {
              const double c = CK[a * n + b];
              row.x += c * y[b].x;
              row.y += c * y[b].y;
            }
          }
          const double2 v = cm(x[a], row);
          acc.x += v.x;
          acc.y += v.y;
        }
      }
      const double2 out = make_double2(-g * acc.x, -g * acc.y);
      const int K = K0 + k;
      if (MODE == 0)
        st(Pb + (long long)(pb + K) * q.ng + r, out);
      else
        st(Pb + (long long)r * q.Np + pb + K, out);
    }
  }
}

// The same blocks on the FP64 matrix cores for atoms with n <= 9 orbitals and m <= 64 product
// functions.  Per atom and (tau, R) block, P[K][r] = -g sum_ab C^K_ab z_ab(r) with
// z_ab(r) = x_a(r) y_b(r) is a real (m x n^2) by complex (n^2 x n_g) product: A = C^K_ab (K rows,
// inner index 12 a + b, zero-padded to 64 x 108 in LDS), B = z (its real and imaginary parts as
// two accumulations).  Wavefront w takes 16 grid points; lane (li, lk) takes the point r0 + li
// and, in column group j, b = 4 j + lk, so it forms z from its own x_a and y_b in registers.
// A workgroup stages C once and walks several (tau, R) blocks (grid.z stride).
typedef double mxd4 __attribute__((ext_vector_type(4)));

template <class T, int MODE>
__global__ __launch_bounds__(256) void p_mixed_mx(const T* __restrict__ Gog, const T* __restrict__ Ggo,
                                                  T* __restrict__ P, double g, const IntArgs q) {
  __shared__ double Cs[64 * kMxLd];
  __shared__ double2 Xs[4 * kMxN * 16];
  const int t = blockIdx.y, tid = threadIdx.x;
  const int s = q.species[t], n = q.n[s], m = q.m[s], o = q.orb_off[t], pb = q.pb_off[t];
  if (!mx_species(n, m)) return;  // p_mixed covers this atom
  const double* C = q.C[s];
  for (int i = tid; i < 64 * kMxLd; i += 256) {
    const int K = i / kMxLd, ab = i - K * kMxLd, a = ab / 12, b = ab - a * 12;
    Cs[i] = (K < m && a < n && b < n) ? C[((long long)K * n + a) * n + b] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int r = blockIdx.x * 64 + 16 * w + li;
  const bool on = r < q.ng;
  const long long sl = (long long)q.No * q.ng, pl = (long long)q.Np * q.ng;
  const int nblk = q.n_tau * q.NR;
  for (int z = blockIdx.z; z < nblk; z += gridDim.z) {
    const int tau = z / q.NR, R = z - tau * q.NR;
    const int tm = q.n_tau - 1 - tau, mR = q.minusR[R];
    double2 x[kMxN], y[kMxN];
#pragma unroll
    for (int a = 0; a < kMxN; ++a) {
      x[a] = y[a] = make_double2(0.0, 0.0);
      if (on && a < n) {
        if (MODE == 0) {
          x[a] = ld(Gog + ((long long)tau * q.NR + R) * sl + (long long)(o + a) * q.ng + r);
          y[a] = ld(Ggo + ((long long)tm * q.NR + mR) * sl + (long long)r * q.No + o + a);
        } else {
          x[a] = ld(Ggo + ((long long)tau * q.NR + R) * sl + (long long)r * q.No + o + a);
          y[a] = ld(Gog + ((long long)tm * q.NR + mR) * sl + (long long)(o + a) * q.ng + r);
        }
      }
    }
    // K index 12 a + b' with b' = 4 j + lk: this lane's y for the three column groups j
    double2 ys[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ys[j] = y[4 * j];
#pragma unroll
      for (int l = 1; l < 4; ++l)
        if (lk == l) ys[j] = 4 * j + l < kMxN ? y[4 * j + l] : make_double2(0.0, 0.0);
    }
    mxd4 ar[4], ai[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ar[i] = ai[i] = mxd4{0, 0, 0, 0};
    double2* Xw = Xs + w * kMxN * 16;  // this wavefront's x_a(r), [a][li]; read back by the same lanes
#pragma unroll
    for (int a = 0; a < kMxN; ++a) Xw[a * 16 + li] = x[a];  // the four lane groups write equal values
#pragma unroll 1
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double2 xa = Xw[a * 16 + li];
        const double zr = xa.x * ys[j].x - xa.y * ys[j].y, zi = xa.x * ys[j].y + xa.y * ys[j].x;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const double c = Cs[(16 * mt + li) * kMxLd + 12 * a + 4 * j + lk];
          ar[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, zr, ar[mt], 0, 0, 0);
          ai[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, zi, ai[mt], 0, 0, 0);
        }
      }
    if (on) {
      T* Pb = P + ((long long)tau * q.NR + R) * pl;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int K = 16 * mt + lk + 4 * j;  // FP64 MFMA output: register j of lane group lk is row lk + 4 j
          if (K < m) {
            const double2 out = make_double2(-g * ar[mt][j], -g * ai[mt][j]);
            if (MODE == 0)
              st(Pb + (long long)(pb + K) * q.ng + r, out);
            else
              st(Pb + (long long)r * q.Np + pb + K, out);
          }
        }
    }
  }
}

// MT-INT and INT-MT blocks of Sigma (Eq. (9) and its partner), W at the same tau as G.
//   MODE 0: S_og[t L][r] = -sum_{I, a'} C^I_{L a'} G_og[t a'][r] W_pg[t I][r]
//   MODE 1: S_go[r][t L] = -sum_{J, b'} G_go[r][t b'] W_gp[r][t J] C^J_{L b'}
template <class T, int MODE>
__global__ __launch_bounds__(256) void s_mixed(const T* __restrict__ Gx, const T* __restrict__ Wx,
                                               double2* __restrict__ S, const IntArgs q) {
  __shared__ double Cs[kCS];
  const int r = blockIdx.x * 256 + threadIdx.x, t = blockIdx.y;
  const int tau = blockIdx.z / q.NR, R = blockIdx.z - tau * q.NR;
  const bool on = r < q.ng;
  const int s = q.species[t], n = q.n[s], m = q.m[s], o = q.orb_off[t], pb = q.pb_off[t];
  const double* C = q.C[s];
  const long long blk = (long long)tau * q.NR + R;
  const long long gl = (long long)q.No * q.ng, wl = (long long)q.Np * q.ng;
  double2 x[kMaxOrb], acc[kMaxOrb];
#pragma unroll
  for (int a = 0; a < kMaxOrb; ++a) {
    acc[a] = make_double2(0.0, 0.0);
    if (on && a < n)
      x[a] = MODE == 0 ? ld(Gx + blk * gl + (long long)(o + a) * q.ng + r) : ld(Gx + blk * gl + (long long)r * q.No + o + a);
  }
  const int nn = n * n, rows = kCS / nn;
  for (int I0 = 0; I0 < m; I0 += rows) {
    const int nk = m - I0 < rows ? m - I0 : rows;
    __syncthreads();
    for (int i = threadIdx.x; i < nk * nn; i += 256) Cs[i] = C[(long long)I0 * nn + i];
    __syncthreads();
    if (!on) continue;
    for (int k = 0; k < nk; ++k) {
      const int I = I0 + k;
      const double2 w = MODE == 0 ? ld(Wx + blk * wl + (long long)(pb + I) * q.ng + r) : ld(Wx + blk * wl + (long long)r * q.Np + pb + I);
      const double* CI = Cs + k * nn;
#pragma unroll
      for (int L = 0; L < kMaxOrb; ++L) {
        if (L < n) {
          double2 cx = make_double2(0.0, 0.0);
#pragma unroll
          for (int a = 0; a < kMaxOrb; ++a) {
            if (a < n) {
              const double c = CI[L * n + a];
              cx.x += c * x[a].x;
              cx.y += c * x[a].y;
            }
          }
          const double2 v = cm(cx, w);
          acc[L].x += v.x;
          acc[L].y += v.y;
        }
      }
    }
  }
  if (!on) return;
  double2* Sb = S + blk * gl;
#pragma unroll
  for (int L = 0; L < kMaxOrb; ++L) {
    if (L < n) {
      const double2 v = make_double2(-acc[L].x, -acc[L].y);
      if (MODE == 0)
        Sb[(long long)(o + L) * q.ng + r] = v;
      else
        Sb[(long long)r * q.No + o + L] = v;
    }
  }
}

// P_gg[tau][R][r][r'] = -g G_gg[tau][R][r][r'] G_gg[tau'][-R][r'][r]  (Eq. (7)); 32 x 32 tiles,
// the mirrored block read coalesced and transposed through LDS.
template <class T>
__global__ __launch_bounds__(256) void p_gg(const T* __restrict__ G, T* __restrict__ P, double g, const IntArgs q) {
  __shared__ double2 tile[kGT][kGT + 1];
  const int tau = blockIdx.z / q.NR, R = blockIdx.z - tau * q.NR;
  const int tm = q.n_tau - 1 - tau, mR = q.minusR[R];
  const int r0 = blockIdx.y * kGT, c0 = blockIdx.x * kGT;  // tile rows r, columns r'
  const long long gl = (long long)q.ng * q.ng;
  const T* Gm = G + ((long long)tm * q.NR + mR) * gl;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // mirrored block, rows r' = c0 + i, columns r = r0 + tx
  for (int i = ty; i < kGT; i += 8) {
    const int rr = c0 + i, cc = r0 + tx;
    tile[i][tx] = (rr < q.ng && cc < q.ng) ? ld(Gm + (long long)rr * q.ng + cc) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const T* Gd = G + ((long long)tau * q.NR + R) * gl;
  T* Pd = P + ((long long)tau * q.NR + R) * gl;
  for (int i = ty; i < kGT; i += 8) {
    const int rr = r0 + i, cc = c0 + tx;
    if (rr < q.ng && cc < q.ng) {
      const double2 v = cm(ld(Gd + (long long)rr * q.ng + cc), tile[tx][i]);
      st(Pd + (long long)rr * q.ng + cc, make_double2(-g * v.x, -g * v.y));
    }
  }
}

// S_gg = -G_gg o W_gg  (Eq. (10)), all tau and R
template <class T>
__global__ __launch_bounds__(256) void s_gg(const T* __restrict__ G, const T* __restrict__ W, double2* __restrict__ S,
                                            long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double2 v = cm(ld(G + i), ld(W + i));
    S[i] = make_double2(-v.x, -v.y);
  }
}

gw_status make_int_args(const gw_cell* c, int ng, IntArgs& q) {
  if (c->n_species > 8) return fail(GW_ERR_UNSUPPORTED, "interstitial blocks support up to 8 species");
  q.NR = c->N_R;
  q.n_tau = c->n_tau;
  q.No = c->N_orb;
  q.Np = c->N_pb;
  q.ng = ng;
  q.minusR = c->minusR_dev;
  q.orb_off = c->orb_off_dev;
  q.pb_off = c->pb_off_dev;
  q.species = c->species_dev;
  for (int s = 0; s < 8; ++s) {
    q.C[s] = s < c->n_species ? c->sp[s].C : nullptr;
    q.n[s] = s < c->n_species ? c->sp[s].n : 0;
    q.m[s] = s < c->n_species ? c->sp[s].m : 0;
  }
  return GW_OK;
}

bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
  auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return !(x < y + nb && y < x + na);
}

gw_status check_common(const gw_cell* c, int ng, gw_dtype t) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (ng < 1) return fail(GW_ERR_SHAPE, "n_grid must be >= 1");
  if (t != GW_C128 && t != GW_C64) return fail(GW_ERR_ARG, "bad dtype");
  if ((long long)c->n_tau * c->N_R > 65535) return fail(GW_ERR_SHAPE, "n_tau * N_R above 65535");
  return GW_OK;
}

}  // namespace
}  // namespace gwr

using namespace gwr;

extern "C" {

gw_status gw_polarizability_int(const gw_cell* c, int ng, const void* Gog, const void* Ggo, const void* Ggg, void* Ppg,
                                void* Pgp, void* Pgg, double g, gw_dtype t, void* stream) {
  gw_status st = check_common(c, ng, t);
  if (st != GW_OK) return st;
  if (!Gog || !Ggo || !Ggg || !Ppg || !Pgp || !Pgg) return fail(GW_ERR_ARG, "NULL tensor");
  if (!std::isfinite(g)) return fail(GW_ERR_ARG, "spin factor must be finite");
  const size_t es = csize(t), bl = (size_t)c->n_tau * c->N_R;
  const size_t nog = bl * c->N_orb * ng * es, ngg = bl * ng * ng * es, npg = bl * c->N_pb * ng * es;
  const void* in[3] = {Gog, Ggo, Ggg};
  const size_t ni[3] = {nog, nog, ngg};
  void* out[3] = {Ppg, Pgp, Pgg};
  const size_t no[3] = {npg, npg, ngg};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      if (!disjoint(in[i], ni[i], out[j], no[j])) return fail(GW_ERR_ARG, "an output overlaps an input");
      if (i < j && !disjoint(out[i], no[i], out[j], no[j])) return fail(GW_ERR_ARG, "outputs overlap");
    }
  IntArgs q;
  st = make_int_args(c, ng, q);
  if (st != GW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const dim3 gm((ng + 255) / 256, c->n_atoms, (unsigned)bl), gt((ng + kGT - 1) / kGT, (ng + kGT - 1) / kGT, (unsigned)bl);
  const dim3 gx((ng + 63) / 64, c->n_atoms, (unsigned)(bl < 48 ? bl : 48));  // 48 WGs share C over the blocks
  if (t == GW_C128) {
    hipLaunchKernelGGL((p_mixed_mx<double2, 0>), gx, dim3(256), 0, s, (const double2*)Gog, (const double2*)Ggo, (double2*)Ppg, g, q);
    hipLaunchKernelGGL((p_mixed_mx<double2, 1>), gx, dim3(256), 0, s, (const double2*)Gog, (const double2*)Ggo, (double2*)Pgp, g, q);
    hipLaunchKernelGGL((p_mixed<double2, 0>), gm, dim3(256), 0, s, (const double2*)Gog, (const double2*)Ggo, (double2*)Ppg, g, q);
    hipLaunchKernelGGL((p_mixed<double2, 1>), gm, dim3(256), 0, s, (const double2*)Gog, (const double2*)Ggo, (double2*)Pgp, g, q);
    hipLaunchKernelGGL(p_gg<double2>, gt, dim3(256), 0, s, (const double2*)Ggg, (double2*)Pgg, g, q);
  } else {
    hipLaunchKernelGGL((p_mixed_mx<float2, 0>), gx, dim3(256), 0, s, (const float2*)Gog, (const float2*)Ggo, (float2*)Ppg, g, q);
    hipLaunchKernelGGL((p_mixed_mx<float2, 1>), gx, dim3(256), 0, s, (const float2*)Gog, (const float2*)Ggo, (float2*)Pgp, g, q);
    hipLaunchKernelGGL((p_mixed<float2, 0>), gm, dim3(256), 0, s, (const float2*)Gog, (const float2*)Ggo, (float2*)Ppg, g, q);
    hipLaunchKernelGGL((p_mixed<float2, 1>), gm, dim3(256), 0, s, (const float2*)Gog, (const float2*)Ggo, (float2*)Pgp, g, q);
    hipLaunchKernelGGL(p_gg<float2>, gt, dim3(256), 0, s, (const float2*)Ggg, (float2*)Pgg, g, q);
  }
  return check_launch("gw_polarizability_int");
}

gw_status gw_self_energy_int(const gw_cell* c, int ng, const void* Gog, const void* Ggo, const void* Ggg,
                             const void* Wpg, const void* Wgp, const void* Wgg, void* Sog, void* Sgo, void* Sgg,
                             gw_dtype t, void* stream) {
  gw_status st = check_common(c, ng, t);
  if (st != GW_OK) return st;
  if (!Gog || !Ggo || !Ggg || !Wpg || !Wgp || !Wgg || !Sog || !Sgo || !Sgg) return fail(GW_ERR_ARG, "NULL tensor");
  const size_t es = csize(t), bl = (size_t)c->n_tau * c->N_R;
  const size_t nog = bl * c->N_orb * ng, ngg = bl * ng * ng, npg = bl * c->N_pb * ng;
  const void* in[6] = {Gog, Ggo, Ggg, Wpg, Wgp, Wgg};
  const size_t ni[6] = {nog * es, nog * es, ngg * es, npg * es, npg * es, ngg * es};
  void* out[3] = {Sog, Sgo, Sgg};
  const size_t no[3] = {nog * 16, nog * 16, ngg * 16};
  for (int j = 0; j < 3; ++j) {
    for (int i = 0; i < 6; ++i)
      if (!disjoint(in[i], ni[i], out[j], no[j])) return fail(GW_ERR_ARG, "an output overlaps an input");
    for (int i = 0; i < j; ++i)
      if (!disjoint(out[i], no[i], out[j], no[j])) return fail(GW_ERR_ARG, "outputs overlap");
  }
  IntArgs q;
  st = make_int_args(c, ng, q);
  if (st != GW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const dim3 gm((ng + 255) / 256, c->n_atoms, (unsigned)bl);
  const long long ne = (long long)ngg;
  const unsigned ge = (unsigned)((ne + 255) / 256 < 4096 ? (ne + 255) / 256 : 4096);
  if (t == GW_C128) {
    hipLaunchKernelGGL((s_mixed<double2, 0>), gm, dim3(256), 0, s, (const double2*)Gog, (const double2*)Wpg, (double2*)Sog, q);
    hipLaunchKernelGGL((s_mixed<double2, 1>), gm, dim3(256), 0, s, (const double2*)Ggo, (const double2*)Wgp, (double2*)Sgo, q);
    hipLaunchKernelGGL(s_gg<double2>, dim3(ge), dim3(256), 0, s, (const double2*)Ggg, (const double2*)Wgg, (double2*)Sgg, ne);
  } else {
    hipLaunchKernelGGL((s_mixed<float2, 0>), gm, dim3(256), 0, s, (const float2*)Gog, (const float2*)Wpg, (double2*)Sog, q);
    hipLaunchKernelGGL((s_mixed<float2, 1>), gm, dim3(256), 0, s, (const float2*)Ggo, (const float2*)Wgp, (double2*)Sgo, q);
    hipLaunchKernelGGL(s_gg<float2>, dim3(ge), dim3(256), 0, s, (const float2*)Ggg, (const float2*)Wgg, (double2*)Sgg, ne);
  }
  return check_launch("gw_self_energy_int");
}

}  // extern "C"

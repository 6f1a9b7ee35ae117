// Screened interaction, Eq. (2): W = V + V P W at every (q, nu), returned as its screening
// part W~ = W - V (the part Eq. (8) consumes; Sec. 2 splits W = V + W~).
//
// With V Hermitian positive definite and the Hermitian part of P(q, nu) negative semidefinite
// (bosonic Matsubara frequencies), W = (I - V P)^-1 V = (V^-1 - P)^-1 and V^-1 - P has a
// positive definite Hermitian part, as do all its Schur complements: every pivot has a
// positive real part, so both inverses are taken by Gauss-Jordan elimination without
// pivoting, in FP64, blocked by 64:
//   per block step k (K = the 64 indices of block k), on M in place:
//     D = M[K,K]^-1                     (one workgroup per matrix, LDS)
//     M[K,J] = D M[K,J]          J != K (row panel)
//     M[I,J] -= M[I,K] M[K,J]    I, J != K (rank-64 update, the bulk of the work)
//     M[I,K] = -M[I,K] D         I != K (column panel);  M[K,K] = D
// Matrices are padded to a multiple of 64 with the identity, whose inverse is itself.  The three
// tile products run on the matrix cores (dy_update_mfma).
// Work: 8 n^3 real flops per inversion (n^3 complex multiply-adds).
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace gwr {
namespace {

constexpr int kDB = 64;   // block size of the elimination
constexpr int kKC = 16;   // depth of one LDS stage of a 64 x 64 tile product
constexpr int kDS = 65;   // complex row stride of the diagonal block in LDS

__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

__global__ void dy_zero_info(int* info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *info = 0;
}

// mode 0: M[c] = V[q0 + c];  mode 1: M[c] = Vinv[q] - P[g] with g = g0 + c, q = g mod N_k.
// Indices beyond n hold the identity.  MT: complex type the elimination runs in.
template <class PT, class MT>
__global__ __launch_bounds__(256) void dy_load(MT* __restrict__ M, long long per, int np, int n, int mode,
                                               const double2* __restrict__ V, const MT* __restrict__ Vinv,
                                               const PT* __restrict__ P, long long g0, int n_k) {
  const int c = blockIdx.y;
  const long long g = g0 + c;
  const int q = mode == 0 ? (int)g : (int)(g % n_k);
  MT* Mc = M + (long long)c * per;
  const long long nn = (long long)np * np;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / np), j = (int)(e - (long long)i * np);
    double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    if (i < n && j < n) {
      if (mode == 0) {
        v = V[((long long)q * n + i) * n + j];
      } else {
        const double2 a = ld2(Vinv + (long long)q * per + e);
        const double2 p = ld2(P + (g * n + i) * n + j);
        v = make_double2(a.x - p.x, a.y - p.y);
      }
    }
    st2(Mc + e, v);
  }
}

// W[g] = M[c] - V[q] on the n x n corner (the subtraction in FP64)
template <class WT, class MT>
__global__ __launch_bounds__(256) void dy_store(const MT* __restrict__ M, long long per, int np, int n,
                                                const double2* __restrict__ V, WT* __restrict__ W, long long g0,
                                                int n_k) {
  const int c = blockIdx.y;
  const long long g = g0 + c;
  const int q = (int)(g % n_k);
  const long long nn = (long long)n * n;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e - (long long)i * n);
    const double2 a = ld2(M + (long long)c * per + (long long)i * np + j);
    const double2 v = V[(long long)q * nn + e];
    st2(W + g * nn + e, make_double2(a.x - v.x, a.y - v.y));
  }
}

// Green's function, Eq. (4): M[c] = -i A with A = (i w_m + mu) I - H(k) - Sigma_x(k) - Sigma(m, k),
// g = g0 + c = m N_k + k, w_m = (2 m + 1) pi / beta; identity beyond n.  -i A has the Hermitian
// part w_m I - (Sigma - Sigma^H) / 2i, positive definite for w_m > 0 and a causal Sigma.
__global__ __launch_bounds__(256) void dy_load_green(double2* __restrict__ M, long long per, int np, int n,
                                                     const double2* __restrict__ H, const double2* __restrict__ Sx,
                                                     const double2* __restrict__ S, double mu, double beta,
                                                     long long g0, int n_k) {
  const int c = blockIdx.y;
  const long long g = g0 + c;
  const int k = (int)(g % n_k), m = (int)(g / n_k);
  const double w = (2.0 * m + 1.0) * M_PI / beta;
  double2* Mc = M + (long long)c * per;
  const long long nn = (long long)np * np;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / np), j = (int)(e - (long long)i * np);
    double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    if (i < n && j < n) {
      const long long o = (long long)i * n + j;
      double2 a = H[(long long)k * n * n + o];
      a = make_double2(-a.x, -a.y);
      if (i == j) {
        a.x += mu;
        a.y += w;
      }
      if (Sx) {
        const double2 x = Sx[(long long)k * n * n + o];
        a.x -= x.x;
        a.y -= x.y;
      }
      if (S) {
        const double2 x = S[g * n * n + o];
        a.x -= x.x;
        a.y -= x.y;
      }
      v = make_double2(a.y, -a.x);  // -i a
    }
    Mc[e] = v;
  }
}

// G[g] = A^-1 = -i M^-1 on the n x n corner
__global__ __launch_bounds__(256) void dy_store_green(const double2* __restrict__ M, long long per, int np, int n,
                                                      double2* __restrict__ G, long long g0) {
  const int c = blockIdx.y;
  const long long g = g0 + c;
  const long long nn = (long long)n * n;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e - (long long)i * n);
    const double2 a = M[(long long)c * per + (long long)i * np + j];
    G[g * nn + e] = make_double2(a.y, -a.x);
  }
}

// Electron count from G at the first n_om fermionic frequencies (one workgroup):
// n = (g / N_k) [N_k N_orb / 2 + (2 / beta) (sum Re Tr G(k, i w_m) - S sum_k c2(k))],
// c2(k) = Re Tr (H(k) + Sigma_x(k)) - mu N_orb, S = sum_{m >= n_om} 1 / w_m^2 (host, closed form).
__global__ __launch_bounds__(256) void dy_count(const double2* __restrict__ G, const double2* __restrict__ H,
                                                const double2* __restrict__ Sx, int n_om, int n_k, int n, double mu,
                                                double beta, double tail, double g, double* __restrict__ n_dev) {
  __shared__ double part[256];
  double a = 0.0, b = 0.0;
  const long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < (long long)n_om * n_k * n; i += 256) {
    const long long mk = i / n;
    const int d = (int)(i - mk * n);
    a += G[mk * nn + (long long)d * n + d].x;
  }
  for (long long i = threadIdx.x; i < (long long)n_k * n; i += 256) {
    const long long k = i / n;
    const int d = (int)(i - k * n);
    b += H[k * nn + (long long)d * n + d].x - mu + (Sx ? Sx[k * nn + (long long)d * n + d].x : 0.0);
  }
  part[threadIdx.x] = a - tail * b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_dev = g / n_k * (0.5 * (double)n_k * n + 2.0 / beta * part[0]);
}

// G(k, tau) from G(k, i w_m) at the first n_om fermionic frequencies w_m = (2 m + 1) pi / beta:
//   G(tau) = (1 / beta) sum over all n of exp(-i w_n tau) G(i w_n), the negative frequencies
//   taken as G(-i w) = G(i w)^H, and the tails 1 / (i w), c2 / (i w)^2 of G, c2 = H - mu + Sigma_x,
//   summed in closed form (their transforms on 0 < tau < beta are -1/2 and (2 tau - beta) / 4):
//   G(tau) = -I / 2 + c2 (2 tau - beta) / 4
//            + (1 / beta) sum_{m < n_om} [exp(-i w_m tau) R_m + exp(+i w_m tau) R_m^H],
//   R_m = G(i w_m) - I / (i w_m) - c2 / (i w_m)^2 = G(i w_m) + i I / w_m + c2 / w_m^2.
// A workgroup takes 256 matrix elements (k, a, b) and a chunk of 16 time points; the phases
// of the chunk are tabulated in LDS first.
constexpr int kGT = 16;  // time points per chunk
__global__ __launch_bounds__(256) void dy_green_tau(const double2* __restrict__ G, const double2* __restrict__ H,
                                                    const double2* __restrict__ Sx, double mu, int n_om, int n_k,
                                                    int n, double beta, const double* __restrict__ tau, int n_tau,
                                                    double mix, double2* __restrict__ out) {
  extern __shared__ double2 ph[];  // [kGT][n_om]: exp(-i w_m tau_i) / beta
  const int i0 = blockIdx.y * kGT, nt = n_tau - i0 < kGT ? n_tau - i0 : kGT;
  for (int e = threadIdx.x; e < nt * n_om; e += 256) {
    const int i = e / n_om, m = e - i * n_om;
    double sn, cs;
    sincospi((2.0 * m + 1.0) * (tau[i0 + i] / beta), &sn, &cs);
    ph[e] = make_double2(cs / beta, -sn / beta);
  }
  __syncthreads();
  const long long nn = (long long)n * n, total = (long long)n_k * nn;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const long long k = e / nn;
  const int a = (int)((e - k * nn) / n), b = (int)(e - k * nn - (long long)a * n);
  const long long eab = e, eba = k * nn + (long long)b * n + a;
  // c2 of (a, b) and of (b, a)
  double2 c2 = H[eab], c2t = H[eba];
  if (Sx) {
    const double2 x = Sx[eab], y = Sx[eba];
    c2.x += x.x;
    c2.y += x.y;
    c2t.x += y.x;
    c2t.y += y.y;
  }
  if (a == b) {
    c2.x -= mu;
    c2t.x -= mu;
  }
  double accr[kGT], acci[kGT];
#pragma unroll
  for (int i = 0; i < kGT; ++i) {
    const double t = i < nt ? tau[i0 + i] : 0.0;
    accr[i] = (a == b ? -0.5 : 0.0) + c2.x * (2.0 * t - beta) * 0.25;
    acci[i] = c2.y * (2.0 * t - beta) * 0.25;
  }
  for (int m = 0; m < n_om; ++m) {
    const double w = (2.0 * m + 1.0) * M_PI / beta, iw2 = 1.0 / (w * w);
    const double2 g = G[(long long)m * total + eab], gt = G[(long long)m * total + eba];
    // R_m(a, b) and conj(R_m(b, a))
    double rr = g.x + c2.x * iw2, ri = g.y + c2.y * iw2 + (a == b ? 1.0 / w : 0.0);
    double hr = gt.x + c2t.x * iw2, hi = -(gt.y + c2t.y * iw2 + (a == b ? 1.0 / w : 0.0));
#pragma unroll
    for (int i = 0; i < kGT; ++i) {
      const double2 p = ph[i * n_om + m];  // exp(-i w tau) / beta; its conjugate for the R^H term
      accr[i] += p.x * rr - p.y * ri + p.x * hr + p.y * hi;
      acci[i] += p.x * ri + p.y * rr + p.x * hi - p.y * hr;
    }
  }
#pragma unroll
  for (int i = 0; i < kGT; ++i)
    if (i < nt) {
      double2* o = out + (long long)(i0 + i) * total + eab;
      if (mix == 1.0) {
        *o = make_double2(accr[i], acci[i]);
      } else {
        const double2 old = *o;
        *o = make_double2(mix * accr[i] + (1.0 - mix) * old.x, mix * acci[i] + (1.0 - mix) * old.y);
      }
    }
}

template <class MT> struct Cx;
template <> struct Cx<double2> {
  typedef double R;
  static __device__ __forceinline__ double2 mk(double x, double y) { return make_double2(x, y); }
};
template <> struct Cx<float2> {
  typedef float R;
  static __device__ __forceinline__ float2 mk(float x, float y) { return make_float2(x, y); }
};

// Inverse of the diagonal block of step k by in-place Gauss-Jordan; written to Dinv[c] and to
// M[c][K,K].  A pivot whose real part is not positive flags the matrix in *info.
template <class MT>
__global__ __launch_bounds__(256) void dy_diag(MT* __restrict__ M, MT* __restrict__ Dinv, long long per, int np,
                                               int k, int* info, int code0, int sign) {
  typedef typename Cx<MT>::R R;
  __shared__ MT D[kDB * kDS];
  __shared__ MT Rw[kDB], Fc[kDB];
  const int c = blockIdx.x, tid = threadIdx.x;
  MT* Mk = M + (long long)c * per + (long long)k * kDB * np + (long long)k * kDB;
  for (int e = tid; e < kDB * kDB; e += 256) {
    const int i = e >> 6, j = e & 63;
    D[i * kDS + j] = Mk[(long long)i * np + j];
  }
  __syncthreads();
  const int i = tid >> 2, j0 = tid & 3;
  for (int p = 0; p < kDB; ++p) {
    const MT piv = D[p * kDS + p];
    const R den = piv.x * piv.x + piv.y * piv.y;
    const MT inv = Cx<MT>::mk(piv.x / den, -piv.y / den);
    if (tid == 0 && info && !(piv.x > R(0) && std::isfinite(piv.x) && std::isfinite(piv.y)))
      atomicCAS(info, 0, sign * (code0 + c + 1));
    if (tid < kDB) {
      const MT a = D[p * kDS + tid];
      Rw[tid] = tid == p ? inv : Cx<MT>::mk(a.x * inv.x - a.y * inv.y, a.x * inv.y + a.y * inv.x);
    } else if (tid < 2 * kDB) {
      const int r = tid - kDB;
      Fc[r] = r == p ? Cx<MT>::mk(R(0), R(0)) : D[r * kDS + p];
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < kDB / 4; ++jj) {
      const int j = j0 + 4 * jj;
      if (i == p) {
        D[p * kDS + j] = Rw[j];
      } else {
        const MT b = j == p ? Cx<MT>::mk(R(0), R(0)) : D[i * kDS + j];
        const MT f = Fc[i], r = Rw[j];
        D[i * kDS + j] = Cx<MT>::mk(b.x - (f.x * r.x - f.y * r.y), b.y - (f.x * r.y + f.y * r.x));
      }
    }
    __syncthreads();
  }
  MT* Dc = Dinv + (long long)c * kDB * kDB;
  for (int e = tid; e < kDB * kDB; e += 256) {
    const int r = e >> 6, s = e & 63;
    const MT v = D[r * kDS + s];
    Dc[e] = v;
    Mk[(long long)r * np + s] = v;
  }
}

// The 64 x 64 tile products of one block step on the matrix cores (grid.z = matrix):
//   OP 0: M[K,J] = D M[K,J]        (grid.x = J tile; row panel)
//   OP 1: M[I,J] -= M[I,K] M[K,J]  (grid.x = J tile, grid.y = I tile; rank-64 update)
//   OP 2: M[I,K] = -M[I,K] D       (grid.x = I tile; column panel)
// 16x16x4 real MFMAs in the element type; a complex product is four of them. Wavefront w owns
// the 32 x 32 quadrant (w / 2, w % 2) of the tile as 2 x 2 MFMA tiles with separate real and
// imaginary accumulators. K is staged through LDS in steps of kKC, and the next stage is loaded
// into registers while the current one is multiplied; for OP 1 the C tile is read into
// registers before the K loop. A tile that is both read and written (OP 0, OP 2) belongs to one
// workgroup, which has read all of it before the barrier that ends the K loop and writes after
// it. WPE caps the wavefronts per SIMD so that everything stays in registers (2 for
// complex128, 4 for complex64).
typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));
template <class MT> struct Mx;
template <> struct Mx<double2> {
  typedef dv4 V;
  static __device__ __forceinline__ dv4 op(double a, double b, dv4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output register j of lane group g (= lane / 16) holds row g + 4 j of the 16 x 16 tile
  static __device__ __forceinline__ int row(int g, int j) { return g + 4 * j; }
};
template <> struct Mx<float2> {
  typedef fv4 V;
  static __device__ __forceinline__ fv4 op(float a, float b, fv4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int j) { return 4 * g + j; }
};

template <int OP, class MT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, WPE))) void dy_update_mfma(
    MT* __restrict__ M, const MT* __restrict__ Dinv, long long per, int np, int k) {
  typedef Mx<MT> X;
  typedef typename X::V V;
  __shared__ MT As[kDB * (kKC + 1)];
  __shared__ MT Bs[kKC * kDB];
  const int c = blockIdx.z, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  MT* Mc = M + (long long)c * per;
  const MT* Dc = Dinv + (long long)c * kDB * kDB;
  const long long K0 = (long long)k * kDB;
  const MT *A, *B;
  long long lda, ldb;
  MT* C;
  if (OP == 0) {  // row panel: M[K,J] = D M[K,J]
    const int J = blockIdx.x;
    if (J == k) return;
    A = Dc;
    lda = kDB;
    B = Mc + K0 * np + (long long)J * kDB;
    ldb = np;
    C = Mc + K0 * np + (long long)J * kDB;
  } else if (OP == 1) {  // rank-64 update: M[I,J] -= M[I,K] M[K,J]
    const int J = blockIdx.x, I = blockIdx.y;
    if (I == k || J == k) return;
    A = Mc + (long long)I * kDB * np + K0;
    lda = np;
    B = Mc + K0 * np + (long long)J * kDB;
    ldb = np;
    C = Mc + (long long)I * kDB * np + (long long)J * kDB;
  } else {  // column panel: M[I,K] = -M[I,K] D
    const int I = blockIdx.x;
    if (I == k) return;
    A = Mc + (long long)I * kDB * np + K0;
    lda = np;
    B = Dc;
    ldb = kDB;
    C = Mc + (long long)I * kDB * np + K0;
  }
  V re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = V{0, 0, 0, 0};
  typedef typename Cx<MT>::R R;
  R cr[2][2][4], ci[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cr[a][b][j] = ci[a][b][j] = R(0);
        if (OP == 1) {
          const MT v = C[(long long)(r0 + 16 * a + X::row(lk, j)) * np + c0 + 16 * b + li];
          cr[a][b][j] = v.x;
          ci[a][b][j] = v.y;
        }
      }
  R par[4], pai[4], pbr[4], pbi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = tid + 256 * r;
    const MT a = A[(long long)(e >> 4) * lda + (e & 15)], b = B[(long long)(e >> 6) * ldb + (e & 63)];
    par[r] = a.x;
    pai[r] = a.y;
    pbr[r] = b.x;
    pbi[r] = b.y;
  }
#pragma unroll
  for (int k0 = 0; k0 < kDB; k0 += kKC) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      As[(e >> 4) * (kKC + 1) + (e & 15)] = Cx<MT>::mk(par[r], pai[r]);
      Bs[(e >> 6) * kDB + (e & 63)] = Cx<MT>::mk(pbr[r], pbi[r]);
    }
    __syncthreads();
    if (k0 + kKC < kDB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = tid + 256 * r;
        const MT a = A[(long long)(e >> 4) * lda + k0 + kKC + (e & 15)];
        const MT b = B[(long long)(k0 + kKC + (e >> 6)) * ldb + (e & 63)];
        par[r] = a.x;
        pai[r] = a.y;
        pbr[r] = b.x;
        pbi[r] = b.y;
      }
    }
#pragma unroll
    for (int ks = 0; ks < kKC / 4; ++ks) {
      const int kk = 4 * ks + lk;
      MT av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[(r0 + 16 * a + li) * (kKC + 1) + kk];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk * kDB + c0 + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          re[a][b] = X::op(av[a].x, bv[b].x, re[a][b]);
          re[a][b] = X::op(-av[a].y, bv[b].y, re[a][b]);
          im[a][b] = X::op(av[a].x, bv[b].y, im[a][b]);
          im[a][b] = X::op(av[a].y, bv[b].x, im[a][b]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        MT* d = C + (long long)(r0 + 16 * a + X::row(lk, j)) * np + c0 + 16 * b + li;
        if (OP == 0)
          *d = Cx<MT>::mk(re[a][b][j], im[a][b][j]);
        else  // OP 1: C - A B (C read before the K loop); OP 2: -A B
          *d = Cx<MT>::mk(cr[a][b][j] - re[a][b][j], ci[a][b][j] - im[a][b][j]);
      }
}

unsigned grid_elems(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

// in-place inverse of `count` padded matrices M[c] (stride per); info codes sign * (code0 + c + 1)
template <class MT>
gw_status gj_invert(MT* M, MT* Dinv, int count, int np, int* info, int code0, int sign, hipStream_t s) {
  const long long per = (long long)np * np;
  const int nt = np / kDB;
  for (int k = 0; k < nt; ++k) {
    hipLaunchKernelGGL(dy_diag<MT>, dim3(count), dim3(256), 0, s, M, Dinv, per, np, k, info, code0, sign);
    if (nt > 1) {
      constexpr int wpe = sizeof(MT) == 16 ? 2 : 4;
      hipLaunchKernelGGL((dy_update_mfma<0, MT, wpe>), dim3(nt, 1, count), dim3(256), 0, s, M, Dinv, per, np, k);
      hipLaunchKernelGGL((dy_update_mfma<1, MT, wpe>), dim3(nt, nt, count), dim3(256), 0, s, M, Dinv, per, np, k);
      hipLaunchKernelGGL((dy_update_mfma<2, MT, wpe>), dim3(nt, 1, count), dim3(256), 0, s, M, Dinv, per, np, k);
    }
  }
  return check_launch("screened interaction: elimination");
}

int padded(int n) { return (n + kDB - 1) / kDB * kDB; }

// es: bytes per complex element of the elimination (16 for FP64, 8 for FP32)
size_t work_bytes(int n_k, int np, long long chunk, size_t es) {
  const long long nd = chunk > n_k ? chunk : n_k;
  return es * ((size_t)np * np * (size_t)(n_k + chunk) + (size_t)kDB * kDB * (size_t)nd);
}

size_t green_bytes(int np, long long chunk) {
  return 16 * ((size_t)np * np * (size_t)chunk + (size_t)kDB * kDB * (size_t)chunk);
}

bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
  auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return !(x < y + nb && y < x + na);
}

}  // namespace
}  // namespace gwr

using namespace gwr;

extern "C" {

gw_status gw_screened_interaction_workspace(const gw_cell* c, int chunk, gw_precision prec, size_t* bytes) {
  if (!c || !bytes) return fail(GW_ERR_ARG, "NULL pointer");
  if (chunk < 1) return fail(GW_ERR_ARG, "chunk must be >= 1");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  *bytes = work_bytes(c->N_R, padded(c->N_pb), chunk, prec == GW_FP64 ? 16 : 8);
  return GW_OK;
}

}  // extern "C"

namespace gwr {
namespace {

// the elimination of gw_screened_interaction in the complex type MT (double2 or float2)
template <class MT>
gw_status screened_run(const gw_cell* c, const void* V, const void* P, gw_dtype pt, void* W, gw_dtype wt,
                       long long total, long long chunk, void* work, int* info, hipStream_t s) {
  const int n_k = c->N_R, n = c->N_pb, np = padded(n);
  const long long per = (long long)np * np;
  MT* Vinv = static_cast<MT*>(work);
  MT* Mw = Vinv + (long long)n_k * per;
  MT* Dinv = Mw + chunk * per;
  if (info) hipLaunchKernelGGL(dy_zero_info, dim3(1), dim3(64), 0, s, info);
  // V^-1 for every q (flag -(q + 1) on a non-positive pivot)
  hipLaunchKernelGGL((dy_load<double2, MT>), dim3(grid_elems(per), n_k), dim3(256), 0, s, Vinv, per, np, n, 0,
                     (const double2*)V, (const MT*)nullptr, (const double2*)nullptr, 0LL, n_k);
  gw_status st = gj_invert(Vinv, Dinv, n_k, np, info, 0, -1, s);
  if (st != GW_OK) return st;
  for (long long g0 = 0; g0 < total; g0 += chunk) {
    const int cnt = (int)(total - g0 < chunk ? total - g0 : chunk);
    if (pt == GW_C128)
      hipLaunchKernelGGL((dy_load<double2, MT>), dim3(grid_elems(per), cnt), dim3(256), 0, s, Mw, per, np, n, 1,
                         (const double2*)nullptr, (const MT*)Vinv, (const double2*)P, g0, n_k);
    else
      hipLaunchKernelGGL((dy_load<float2, MT>), dim3(grid_elems(per), cnt), dim3(256), 0, s, Mw, per, np, n, 1,
                         (const double2*)nullptr, (const MT*)Vinv, (const float2*)P, g0, n_k);
    st = gj_invert(Mw, Dinv, cnt, np, info, (int)g0, 1, s);
    if (st != GW_OK) return st;
    if (wt == GW_C128)
      hipLaunchKernelGGL((dy_store<double2, MT>), dim3(grid_elems((long long)n * n), cnt), dim3(256), 0, s,
                         (const MT*)Mw, per, np, n, (const double2*)V, (double2*)W, g0, n_k);
    else
      hipLaunchKernelGGL((dy_store<float2, MT>), dim3(grid_elems((long long)n * n), cnt), dim3(256), 0, s,
                         (const MT*)Mw, per, np, n, (const double2*)V, (float2*)W, g0, n_k);
  }
  return check_launch("gw_screened_interaction");
}

}  // namespace
}  // namespace gwr

extern "C" {

gw_status gw_screened_interaction(const gw_cell* c, const void* V, const void* P, gw_dtype pt, void* W, gw_dtype wt,
                                  int n_omega, gw_precision prec, void* work, size_t work_size, int* info,
                                  void* stream) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!V || !P || !W || !work) return fail(GW_ERR_ARG, "NULL pointer");
  if ((pt != GW_C128 && pt != GW_C64) || (wt != GW_C128 && wt != GW_C64)) return fail(GW_ERR_ARG, "bad dtype");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(GW_ERR_ARG, "bad precision");
  if (n_omega < 1) return fail(GW_ERR_SHAPE, "n_omega must be >= 1");
  const size_t es = prec == GW_FP64 ? 16 : 8;
  const int n_k = c->N_R, n = c->N_pb, np = padded(n);
  const long long total = (long long)n_omega * n_k;
  long long chunk = 0;
  if (work_size >= work_bytes(n_k, np, 1, es)) {
    long long lo = 1, hi = total;
    while (lo < hi) {
      const long long mid = (lo + hi + 1) / 2;
      if (work_bytes(n_k, np, mid, es) <= work_size) lo = mid; else hi = mid - 1;
    }
    chunk = lo;
  }
  if (chunk < 1) return fail(GW_ERR_SHAPE, "workspace smaller than gw_screened_interaction_workspace(cell, 1, prec)");
  if (chunk > 65535) chunk = 65535;
  const size_t nv = (size_t)n_k * n * n * 16, npw = (size_t)total * n * n;
  const size_t bp = npw * csize(pt), bw = npw * csize(wt), bwork = work_bytes(n_k, np, chunk, es);
  if (!disjoint(V, nv, W, bw) || !disjoint(work, bwork, V, nv) || !disjoint(work, bwork, P, bp) ||
      !disjoint(work, bwork, W, bw))
    return fail(GW_ERR_ARG, "the workspace or V overlaps another operand");
  if (P == W ? pt != wt : !disjoint(P, bp, W, bw))
    return fail(GW_ERR_ARG, "P and W must be the same tensor of one dtype, or disjoint");
  if (info && (!disjoint(info, 4, work, bwork) || !disjoint(info, 4, W, bw)))
    return fail(GW_ERR_ARG, "info overlaps an operand");
  if (prec == GW_FP64)
    return screened_run<double2>(c, V, P, pt, W, wt, total, chunk, work, info, (hipStream_t)stream);
  return screened_run<float2>(c, V, P, pt, W, wt, total, chunk, work, info, (hipStream_t)stream);
}

gw_status gw_green_dyson_workspace(const gw_cell* c, int chunk, size_t* bytes) {
  if (!c || !bytes) return fail(GW_ERR_ARG, "NULL pointer");
  if (chunk < 1) return fail(GW_ERR_ARG, "chunk must be >= 1");
  *bytes = green_bytes(padded(c->N_orb), chunk);
  return GW_OK;
}

}  // extern "C"

namespace gwr {
namespace {

// Checks shared by the two G Dyson entry points: cell on the current device, pointers, sizes.
gw_status green_common(const gw_cell* c, const void* Hk, const void* G, int n_omega, double mu) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!Hk || !G) return fail(GW_ERR_ARG, "NULL pointer");
  if (n_omega < 1) return fail(GW_ERR_SHAPE, "n_omega must be >= 1");
  if (!std::isfinite(mu)) return fail(GW_ERR_ARG, "mu must be finite");
  return GW_OK;
}

// Operand overlaps against G and a workspace of bwork bytes, then the solve in chunks of
// `chunk` matrices through that workspace.
gw_status green_run(const gw_cell* c, const void* Hk, double mu, int n_omega, const void* Sigma,
                    const void* Sigma_x, void* G, void* work, long long chunk, int* info, hipStream_t s) {
  const int n_k = c->N_R, n = c->N_orb, np = padded(n);
  const long long total = (long long)n_omega * n_k;
  if (chunk > total) chunk = total;
  if (chunk > 65535) chunk = 65535;
  const size_t nh = (size_t)n_k * n * n * 16, ng = (size_t)total * n * n * 16, bwork = green_bytes(np, chunk);
  if (!disjoint(Hk, nh, G, ng) || (Sigma_x && !disjoint(Sigma_x, nh, G, ng)) || !disjoint(work, bwork, G, ng) ||
      !disjoint(work, bwork, Hk, nh) || (Sigma && !disjoint(work, bwork, Sigma, ng)) ||
      (Sigma_x && !disjoint(work, bwork, Sigma_x, nh)))
    return fail(GW_ERR_ARG, "an operand overlaps G or the workspace");
  if (Sigma && Sigma != G && !disjoint(Sigma, ng, G, ng))
    return fail(GW_ERR_ARG, "Sigma and G must be the same tensor or disjoint");
  if (info && (!disjoint(info, 4, work, bwork) || !disjoint(info, 4, G, ng)))
    return fail(GW_ERR_ARG, "info overlaps an operand");
  const long long per = (long long)np * np;
  double2* Mw = static_cast<double2*>(work);
  double2* Dinv = Mw + chunk * per;
  if (info) hipLaunchKernelGGL(dy_zero_info, dim3(1), dim3(64), 0, s, info);
  for (long long g0 = 0; g0 < total; g0 += chunk) {
    const int cnt = (int)(total - g0 < chunk ? total - g0 : chunk);
    // every element of the chunk's matrices (padding included) is written here, and the
    // diagonal-block inverses by the elimination: the workspace needs no clearing
    hipLaunchKernelGGL(dy_load_green, dim3(grid_elems(per), cnt), dim3(256), 0, s, Mw, per, np, n,
                       (const double2*)Hk, (const double2*)Sigma_x, (const double2*)Sigma, mu, c->beta, g0, n_k);
    gw_status st = gj_invert(Mw, Dinv, cnt, np, info, (int)g0, 1, s);
    if (st != GW_OK) return st;
    hipLaunchKernelGGL(dy_store_green, dim3(grid_elems((long long)n * n), cnt), dim3(256), 0, s, Mw, per, np, n,
                       (double2*)G, g0);
  }
  return check_launch("gw_green_dyson");
}

// Device scratch of gw_green_dyson_noalloc: one array per device, for callers that cannot
// allocate.  In host code `scratch` only names the symbol; its device address on each GPU is
// looked up once (hipGetSymbolAddress with that GPU current) and kept in scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex scratch_mu;
std::vector<void*> scratch_ptr;  // per device ordinal, nullptr until looked up

gw_status scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (dev >= (int)scratch_ptr.size()) scratch_ptr.resize(dev + 1, nullptr);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GW_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return GW_OK;
}

}  // namespace
}  // namespace gwr

extern "C" {

gw_status gw_green_dyson(const gw_cell* c, const void* Hk, double mu, int n_omega, const void* Sigma,
                         const void* Sigma_x, void* G, void* work, size_t work_size, int* info, void* stream) {
  gw_status st = green_common(c, Hk, G, n_omega, mu);
  if (st != GW_OK) return st;
  if (!work) return fail(GW_ERR_ARG, "NULL pointer");
  const long long chunk = (long long)(work_size / green_bytes(padded(c->N_orb), 1));
  if (chunk < 1) return fail(GW_ERR_SHAPE, "workspace smaller than gw_green_dyson_workspace(cell, 1)");
  return green_run(c, Hk, mu, n_omega, Sigma, Sigma_x, G, work, chunk, info, (hipStream_t)stream);
}

gw_status gw_green_dyson_noalloc(const gw_cell* c, const void* Hk, double mu, int n_omega, const void* Sigma,
                                 const void* Sigma_x, void* G, int* info, void* stream) {
  gw_status st = green_common(c, Hk, G, n_omega, mu);
  if (st != GW_OK) return st;
  const size_t one = green_bytes(padded(c->N_orb), 1);
  if (one > kStaticScratchBytes)
    return fail(GW_ERR_SHAPE, "one matrix of this cell needs " + std::to_string(one) +
                                  " bytes of scratch, above the 64 MiB static scratch of gw_green_dyson_noalloc");
  void* work = nullptr;
  st = scratch_address(c->device, &work);
  if (st != GW_OK) return st;
  return green_run(c, Hk, mu, n_omega, Sigma, Sigma_x, G, work, (long long)(kStaticScratchBytes / one), info,
                   (hipStream_t)stream);
}

static double tail_sum(int n_om, double beta) {
  // sum over m >= n_om of 1 / w_m^2 = (beta / pi)^2 (pi^2 / 8 - sum_{m < n_om} 1 / (2m + 1)^2)
  double head = 0.0;
  for (int m = n_om - 1; m >= 0; --m) head += 1.0 / ((2.0 * m + 1.0) * (2.0 * m + 1.0));
  return (beta / M_PI) * (beta / M_PI) * (M_PI * M_PI / 8.0 - head);
}

gw_status gw_density_omega(const gw_cell* c, const void* G, int n_omega, const void* Hk, const void* Sigma_x,
                           double mu, double spin_factor, double* n_dev, void* stream) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!G || !Hk || !n_dev) return fail(GW_ERR_ARG, "NULL pointer");
  if (n_omega < 1) return fail(GW_ERR_SHAPE, "n_omega must be >= 1");
  if (!std::isfinite(mu) || !std::isfinite(spin_factor)) return fail(GW_ERR_ARG, "mu and spin factor must be finite");
  hipLaunchKernelGGL(dy_count, dim3(1), dim3(256), 0, (hipStream_t)stream, (const double2*)G, (const double2*)Hk,
                     (const double2*)Sigma_x, n_omega, c->N_R, c->N_orb, mu, c->beta, tail_sum(n_omega, c->beta),
                     spin_factor, n_dev);
  return check_launch("gw_density_omega");
}

gw_status gw_update_mu(const gw_cell* c, const void* Hk, const void* Sigma, const void* Sigma_x, int n_omega,
                       double spin_factor, double n_target, double mu_lo, double mu_hi, double tol, int max_iter,
                       void* G, void* work, size_t work_size, double* n_dev, double* mu_out, double* n_out,
                       void* stream) {
  if (!c || !mu_out || !n_out || !n_dev) return fail(GW_ERR_ARG, "NULL pointer");
  if (!(mu_lo < mu_hi) || !std::isfinite(mu_lo) || !std::isfinite(mu_hi) || !(tol > 0) || max_iter < 1 ||
      !std::isfinite(n_target))
    return fail(GW_ERR_ARG, "need finite mu_lo < mu_hi, tol > 0, max_iter >= 1");
  if (Sigma && Sigma == G) return fail(GW_ERR_ARG, "G must not be Sigma: every step reads Sigma again");
  hipStream_t s = (hipStream_t)stream;
  auto count = [&](double mu, double* out) -> gw_status {
    gw_status st = gw_green_dyson(c, Hk, mu, n_omega, Sigma, Sigma_x, G, work, work_size, nullptr, stream);
    if (st != GW_OK) return st;
    st = gw_density_omega(c, G, n_omega, Hk, Sigma_x, mu, spin_factor, n_dev, stream);
    if (st != GW_OK) return st;
    if (hipMemcpyAsync(out, n_dev, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(GW_ERR_HIP, "reading the electron count failed");
    return GW_OK;
  };
  // Illinois regula falsi on f(mu) = count(mu) - n_target: the next mu interpolates the bracket
  // ends linearly; an end kept twice in a row has its residual halved (superlinear, bracketed)
  double lo = mu_lo, hi = mu_hi, n_lo = 0, n_hi = 0;
  gw_status st = count(lo, &n_lo);
  if (st != GW_OK) return st;
  st = count(hi, &n_hi);
  if (st != GW_OK) return st;
  double f_lo = n_lo - n_target, f_hi = n_hi - n_target;
  if (!(f_lo <= 0.0 && 0.0 <= f_hi)) return fail(GW_ERR_ARG, "the bracket does not hold the target count");
  double x = lo, fx = f_lo;
  int side = 0;
  for (int it = 0; it < max_iter; ++it) {
    x = (lo * f_hi - hi * f_lo) / (f_hi - f_lo);
    double nx = 0;
    st = count(x, &nx);
    if (st != GW_OK) return st;
    fx = nx - n_target;
    if (std::fabs(fx) <= tol) break;
    if (fx > 0.0) {
      hi = x;
      f_hi = fx;
      if (side == -1) f_lo *= 0.5;
      side = -1;
    } else {
      lo = x;
      f_lo = fx;
      if (side == 1) f_hi *= 0.5;
      side = 1;
    }
  }
  *mu_out = x;
  *n_out = fx + n_target;
  return GW_OK;
}

gw_status gw_green_tau(const gw_cell* c, const void* G, int n_omega, const void* Hk, const void* Sigma_x, double mu,
                       double mix, void* G_tau, void* stream) {
  if (!c) return fail(GW_ERR_ARG, "cell is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(GW_ERR_HIP, "hipGetDevice failed");
  if (cur != c->device) return fail(GW_ERR_ARG, "current device differs from the cell's device");
  if (!G || !Hk || !G_tau) return fail(GW_ERR_ARG, "NULL pointer");
  if (n_omega < 1 || n_omega > 512) return fail(GW_ERR_SHAPE, "n_omega must be in [1, 512]");
  if (!std::isfinite(mu)) return fail(GW_ERR_ARG, "mu must be finite");
  if (!(mix > 0.0 && mix <= 1.0)) return fail(GW_ERR_ARG, "mix must be in (0, 1]");
  const long long total = (long long)c->N_R * c->N_orb * c->N_orb;
  const size_t ng = (size_t)n_omega * total * 16, no = (size_t)c->n_tau * total * 16, nh = (size_t)total * 16;
  if (!disjoint(G_tau, no, G, ng) || !disjoint(G_tau, no, Hk, nh) || (Sigma_x && !disjoint(G_tau, no, Sigma_x, nh)))
    return fail(GW_ERR_ARG, "G_tau overlaps an input");
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)((c->n_tau + kGT - 1) / kGT));
  const size_t lds = (size_t)kGT * n_omega * sizeof(double2);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)dy_green_tau, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(dy_green_tau, grid, dim3(256), lds, (hipStream_t)stream, (const double2*)G,
                     (const double2*)Hk, (const double2*)Sigma_x, mu, n_omega, c->N_R, c->N_orb, c->beta,
                     c->tau_dev, c->n_tau, mix, (double2*)G_tau);
  return check_launch("gw_green_tau");
}

gw_status gw_omega2tau_matrix(int n_tau, const double* tau, int n_omega, const double* omega, double* Ti) {
  if (!tau || !omega || !Ti) return fail(GW_ERR_ARG, "NULL pointer");
  if (n_omega != n_tau) return fail(GW_ERR_SHAPE, "the inverse needs n_omega == n_tau");
  using cd = std::complex<double>;
  const int n = n_tau;
  std::vector<cd> a((size_t)n * n), x((size_t)n * n, cd(0, 0));
  gw_status st = gw_tau2omega_matrix(n_tau, tau, n_omega, omega, reinterpret_cast<double*>(a.data()));
  if (st != GW_OK) return st;
  for (int i = 0; i < n; ++i) x[(size_t)i * n + i] = 1.0;
  // Gauss-Jordan with partial pivoting on [a | x]
  for (int p = 0; p < n; ++p) {
    int best = p;
    for (int r = p + 1; r < n; ++r)
      if (std::abs(a[(size_t)r * n + p]) > std::abs(a[(size_t)best * n + p])) best = r;
    if (!(std::abs(a[(size_t)best * n + p]) > 0.0)) return fail(GW_ERR_ARG, "tau -> omega matrix is singular");
    if (best != p)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)p * n + j], a[(size_t)best * n + j]);
        std::swap(x[(size_t)p * n + j], x[(size_t)best * n + j]);
      }
    const cd inv = 1.0 / a[(size_t)p * n + p];
    for (int j = 0; j < n; ++j) {
      a[(size_t)p * n + j] *= inv;
      x[(size_t)p * n + j] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == p) continue;
      const cd f = a[(size_t)r * n + p];
      if (f == cd(0, 0)) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)p * n + j];
        x[(size_t)r * n + j] -= f * x[(size_t)p * n + j];
      }
    }
  }
  std::memcpy(Ti, x.data(), x.size() * sizeof(cd));
  return GW_OK;
}

}  // extern "C"

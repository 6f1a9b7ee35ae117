// Imaginary time -> Matsubara frequency transform, alone and fused with R -> k:
// kernels and their launchers, included by one translation unit per storage-type pair
// (omega_<in>_<out>.hip) so that the instantiations compile in parallel.
//
//   out[m][q][e] = sum_tau T[m][tau] sum_R exp(-i q.R) in[tau][R][e]        (gw_drain)
//   out[m][c]    = sum_tau T[m][tau] in[tau][c]                             (gw_tau2omega)
//
// The tau contraction is a real GEMM with the 2x2 block form of the complex
// matrix T, [[Tr, -Ti], [Ti, Tr]] (2 n_omega x 2 n_tau), applied to columns of
// interleaved (re, im) data; it runs on the FP64 MFMA (16x16x4).  A workgroup
// owns up to 64 output columns (CB matrix elements times N_R lattice vectors):
// it stages every tau and R of those elements in LDS with contiguous loads, does
// the separable R -> k sum in registers, then each of its 4 wavefronts computes
// one 16-column tile over all frequencies and writes it back.  Each column is
// read and written exactly once, so in == out (in-place) is safe.
#pragma once

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "cplx.h"
#include "internal.h"

namespace gwr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// GWR_DRAIN=pingpong keeps the paired complex64 drain on the ping-pong kernel; the tests use it to
// check the wide-chunk kernel against it on the device.
inline bool wide_disabled() {
  const char* v = std::getenv("GWR_DRAIN");
  return v && std::strcmp(v, "pingpong") == 0;
}

constexpr int kDrainMaxTau = 96;
constexpr int kDrainMaxOmega = 96;
constexpr int kDrainCols = 64;

// One 1-D pass of the R -> k sum (exp(-i 2 pi j l / L)) of length L along an axis with
// inner stride S over O outer groups; L = 2 and 4 are written as exact butterflies.
template <int O, int L, int S>
__device__ __forceinline__ void dft_pass_minus(double* re, double* im) {
  if constexpr (L == 1) {
    return;
  } else {
#pragma unroll
    for (int o = 0; o < O; ++o) {
#pragma unroll
      for (int i = 0; i < S; ++i) {
        double xr[L], xi[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
          xr[l] = re[(o * L + l) * S + i];
          xi[l] = im[(o * L + l) * S + i];
        }
        double yr[L], yi[L];
        if constexpr (L == 2) {
          yr[0] = xr[0] + xr[1];
          yi[0] = xi[0] + xi[1];
          yr[1] = xr[0] - xr[1];
          yi[1] = xi[0] - xi[1];
        } else if constexpr (L == 4) {
          // w = exp(-i pi / 2) = -i:  y1 = (x0 - x2) - i (x1 - x3),  y3 = (x0 - x2) + i (x1 - x3)
          const double ar = xr[0] + xr[2], ai = xi[0] + xi[2], br = xr[1] + xr[3], bi = xi[1] + xi[3];
          const double cr = xr[0] - xr[2], ci = xi[0] - xi[2], dr = xr[1] - xr[3], di = xi[1] - xi[3];
          yr[0] = ar + br;
          yi[0] = ai + bi;
          yr[2] = ar - br;
          yi[2] = ai - bi;
          yr[1] = cr + di;
          yi[1] = ci - dr;
          yr[3] = cr - di;
          yi[3] = ci + dr;
        } else {
          double cw[L], sw[L];
#pragma unroll
          for (int m = 0; m < L; ++m) turn(-(double)m / (double)L, cw[m], sw[m]);
#pragma unroll
          for (int j = 0; j < L; ++j) {
            double ar = 0, ai = 0;
#pragma unroll
            for (int l = 0; l < L; ++l) {
              const int m = (j * l) % L;
              ar += cw[m] * xr[l] - sw[m] * xi[l];
              ai += cw[m] * xi[l] + sw[m] * xr[l];
            }
            yr[j] = ar;
            yi[j] = ai;
          }
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
          re[(o * L + j) * S + i] = yr[j];
          im[(o * L + j) * S + i] = yi[j];
        }
      }
    }
  }
}

template <int N1, int N2, int N3>
__device__ __forceinline__ void r2k_regs(double* re, double* im) {
  dft_pass_minus<N1 * N2, N3, 1>(re, im);
  dft_pass_minus<N1, N2, N3>(re, im);
  dft_pass_minus<1, N1, N2 * N3>(re, im);
}

// grid: one block per CB-element chunk; 256 threads = 4 wavefronts, one 16-column tile each.
template <int N1, int N2, int N3, class TI, class TO>
__global__ __launch_bounds__(256) void drain_mfma(const double2* __restrict__ T, int n_omega, int n_tau,
                                                  const TI* in, TO* out, long long n2, int CB) {
  constexpr int NR = N1 * N2 * N3;
  extern __shared__ double2 ysh[];  // [n_tau rounded up to even][kDrainCols]
  auto y = reinterpret_cast<double2(*)[kDrainCols]>(ysh);
  const int tid = threadIdx.x;
  const long long e0 = (long long)blockIdx.x * CB;
  const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);  // live elements in this chunk
  const int ncol = NR * CB;

  // phase 1: stage in[tau][R][e0 .. e0+cb) as y[tau][R*CB + c]
  for (int idx = tid; idx < n_tau * ncol; idx += 256) {
    const int t = idx / ncol, rc = idx - t * ncol, R = rc / CB, c = rc - R * CB;
    double a = 0, b = 0;
    if (c < cb) ldc(in + ((long long)t * NR + R) * n2 + e0 + c, a, b);
    y[t][rc] = make_double2(a, b);
  }
  for (int idx = tid; idx < n_tau * (kDrainCols - ncol); idx += 256) {  // zero the padding columns
    const int t = idx / (kDrainCols - ncol), rc = ncol + idx % (kDrainCols - ncol);
    y[t][rc] = make_double2(0.0, 0.0);
  }
  if (n_tau & 1)
    for (int rc = tid; rc < kDrainCols; rc += 256) y[n_tau][rc] = make_double2(0.0, 0.0);
  __syncthreads();

  // phase 2: R -> k for every (tau, c), separable passes in registers, back into LDS
  if constexpr (NR > 1) {
    for (int idx = tid; idx < n_tau * CB; idx += 256) {
      const int t = idx / CB, c = idx - t * CB;
      double re[NR], im[NR];
#pragma unroll
      for (int R = 0; R < NR; ++R) {
        const double2 v = y[t][R * CB + c];
        re[R] = v.x;
        im[R] = v.y;
      }
      dft_pass_minus<N1 * N2, N3, 1>(re, im);
      dft_pass_minus<N1, N2, N3>(re, im);
      dft_pass_minus<1, N1, N2 * N3>(re, im);
#pragma unroll
      for (int q = 0; q < NR; ++q) y[t][q * CB + c] = make_double2(re[q], im[q]);
    }
    __syncthreads();
  }

  // phase 3: FP64 MFMA over tau.  Row r of an M tile (16 rows) is (m, part) with
  // m = 8*mt + 4*(r/8) + r%4 and part = (r/4)%2, so the D fragment of a lane holds the
  // (re, im) pairs of two frequencies; k = 4*ks + l/16 is (tau = 2*ks + k%4/2, part' = k%2).
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt_count = (2 * n_omega + 15) / 16;
  const int ks_count = (n_tau + 1) / 2;
  const int r = li;
  const int m_off = 4 * (r >> 3) + (r & 3), part = (r >> 2) & 1;
  const int tau_off = lk >> 1, partp = lk & 1;
  const double sgn = (part == 0 && partp == 1) ? -1.0 : 1.0;
  const bool use_im = part != partp;
  const int col = 16 * w + li;
  for (int mt0 = 0; mt0 < mt_count; mt0 += 6) {
    d4 acc[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = d4{0, 0, 0, 0};
    for (int ks = 0; ks < ks_count; ++ks) {
      const int tau = 2 * ks + tau_off;
      const double2 yv = y[tau][col];
      const double b = partp ? yv.y : yv.x;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const int m = 8 * (mt0 + i) + m_off;
        double a = 0.0;
        if (m < n_omega && tau < n_tau) {
          const double2 tv = T[(long long)m * n_tau + tau];
          a = sgn * (use_im ? tv.y : tv.x);
        }
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
      }
    }
    // phase 4: lane holds rows lk + 4j: (re, im) of m = 8*mt + lk and of m = 8*mt + 4 + lk
    const int q = col / CB, c = col - q * CB;
    if (col < ncol && c < cb) {
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const int mA = 8 * (mt0 + i) + lk, mB = mA + 4;
        if (mt0 + i < mt_count) {
          if (mA < n_omega) stc(out + ((long long)mA * NR + q) * n2 + e0 + c, acc[i][0], acc[i][1]);
          if (mB < n_omega) stc(out + ((long long)mB * NR + q) * n2 + e0 + c, acc[i][2], acc[i][3]);
        }
      }
    }
  }
}

// Persistent variant with T resident in LDS and the complex product done as three
// real GEMMs (t1 = Tr yr, t2 = Ti yi, t3 = (Tr + Ti)(yr + yi); re = t1 - t2,
// im = t3 - t1 - t2), 3/4 of the MFMA work of the 2x2 block form.  M is the
// frequency (MT tiles of 16), K = tau (steps of 4), N = 16 columns per wavefront.
// A chunk is CB consecutive matrix elements (CB * 16 bytes contiguous per (tau, R)
// row, 256 bytes for complex128 when CB = 16) times the N_R lattice vectors; the
// next chunk is loaded into registers while the current one is on the matrix cores.
// LDS: T [16 MT][nt4 + 1] complex and y [nt4][16 * waves] complex, nt4 = n_tau
// rounded up to 4.
constexpr int kPF = 16;  // prefetched complex values per thread (upper bound)

// REG: each thread owns whole (tau, element) columns of N_R values, so the R -> k sum
// runs in registers between the load and the LDS store; otherwise it runs in LDS.
template <int N1, int N2, int N3, int MT, bool REG, class TI, class TO>
__global__ __launch_bounds__(512, 1) void drain_3m(const double2* __restrict__ T, int n_omega, int n_tau,
                                                   const TI* in, TO* out, long long n2, int CB,
                                                   long long nchunks) {
  constexpr int NR = N1 * N2 * N3;
  constexpr int PU = REG ? (NR <= kPF ? kPF / NR : 1) : kPF;  // columns per thread, or values per thread
  extern __shared__ double2 lds[];
  const int tid = threadIdx.x, nthr = blockDim.x, waves = nthr >> 6;
  const int nt4 = (n_tau + 3) & ~3, ld_t = nt4 + 1, ncp = 16 * waves;
  double2* Ts = lds;                      // [16 MT][ld_t]
  double2* y = lds + 16 * MT * ld_t;      // [nt4][ncp]
  for (int i = tid; i < 16 * MT * ld_t; i += nthr) {
    const int m = i / ld_t, t = i - m * ld_t;
    Ts[i] = (m < n_omega && t < n_tau) ? T[(long long)m * n_tau + t] : make_double2(0.0, 0.0);
  }
  const int ncol = NR * CB;
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int col = 16 * w + li;
  const int ksn = nt4 / 4;
  const int items = nt4 * ncp;
  // prefetch buffer in the storage type: no conversion (and so no wait) at the load
  TI raw[REG ? PU * NR : PU];
  auto fetch = [&](long long ch) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
    if constexpr (REG) {
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int p = tid + nthr * u, t = p / CB, c = p - t * CB;
        const bool live = t < n_tau && c < cb;
#pragma unroll
        for (int R = 0; R < NR; ++R) raw[u * NR + R] = ldraw(in + ((long long)t * NR + R) * n2 + e0 + c, in, live);
      }
    } else {
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int idx = tid + nthr * u;
        const int t = idx / ncp, rc = idx - t * ncp, R = rc / CB, c = rc - R * CB;
        const bool live = idx < items && t < n_tau && rc < ncol && c < cb;
        raw[u] = ldraw(in + ((long long)t * NR + R) * n2 + e0 + c, in, live);
      }
    }
  };
  // zero the padding rows / columns of y once (never written below)
  for (int idx = tid; idx < items; idx += nthr) {
    const int t = idx / ncp, rc = idx - t * ncp;
    if (t >= n_tau || rc >= ncol) y[idx] = make_double2(0.0, 0.0);
  }
  // fill y from the prefetch registers (R -> k in registers, or in LDS)
  auto fill = [&](long long ch) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
    if constexpr (REG) {
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int p = tid + nthr * u, t = p / CB, c = p - t * CB;
        if (t < n_tau) {
          const bool live = c < cb;
          double pr[NR], pi[NR];
#pragma unroll
          for (int R = 0; R < NR; ++R) {
            const TI v = keep(raw[u * NR + R], live);
            pr[R] = (double)v.x;
            pi[R] = (double)v.y;
          }
          r2k_regs<N1, N2, N3>(pr, pi);
#pragma unroll
          for (int q = 0; q < NR; ++q) y[t * ncp + q * CB + c] = make_double2(pr[q], pi[q]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int idx = tid + nthr * u;
        if (idx < items) {
          const int t = idx / ncp, rc = idx - t * ncp;
          if (t < n_tau && rc < ncol) {
            const TI v = keep(raw[u], rc - (rc / CB) * CB < cb);
            y[idx] = make_double2((double)v.x, (double)v.y);
          }
        }
      }
      if constexpr (NR > 1) {
        __syncthreads();
        for (int idx = tid; idx < n_tau * CB; idx += nthr) {
          const int t = idx / CB, c = idx - t * CB;
          double re[NR], im[NR];
#pragma unroll
          for (int R = 0; R < NR; ++R) {
            const double2 v = y[t * ncp + R * CB + c];
            re[R] = v.x;
            im[R] = v.y;
          }
          r2k_regs<N1, N2, N3>(re, im);
#pragma unroll
          for (int q = 0; q < NR; ++q) y[t * ncp + q * CB + c] = make_double2(re[q], im[q]);
        }
      }
    }
  };
  // Order per chunk: matrix phase on y; barrier; y <- next chunk (its loads were issued a
  // whole matrix phase earlier); store this chunk's results; issue the loads of the chunk
  // after next; barrier.  Waiting for the prefetched data never waits for fresh stores.
  if (blockIdx.x < nchunks) {
    fetch(blockIdx.x);
    __syncthreads();  // T and the zero padding staged
    fill(blockIdx.x);
    if (blockIdx.x + gridDim.x < nchunks) fetch(blockIdx.x + gridDim.x);
    __syncthreads();
  }
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
    d4 t1[MT], t2[MT], t3[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) t1[i] = t2[i] = t3[i] = d4{0, 0, 0, 0};
    for (int ks = 0; ks < ksn; ++ks) {
      const int tau = 4 * ks + lk;
      const double2 yv = y[tau * ncp + col];
      const double ys = yv.x + yv.y;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const double2 tv = Ts[(16 * i + li) * ld_t + tau];
        t1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.x, yv.x, t1[i], 0, 0, 0);
        t2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.y, yv.y, t2[i], 0, 0, 0);
        t3[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.x + tv.y, ys, t3[i], 0, 0, 0);
      }
    }
    __syncthreads();  // every wavefront is done reading y
    const long long nxt = ch + gridDim.x;
    if (nxt < nchunks) fill(nxt);
    // D fragment: register j of lane group lk is frequency 16 i + lk + 4 j, column `col`
    if (col < ncol) {
      const int q = col / CB, c = col - q * CB;
      if (c < cb) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int m = 16 * i + lk + 4 * j;
            if (m < n_omega)
              stc(out + ((long long)m * NR + q) * n2 + e0 + c, t1[i][j] - t2[i][j], t3[i][j] - t1[i][j] - t2[i][j]);
          }
      }
    }
    if (nxt + gridDim.x < nchunks) fetch(nxt + gridDim.x);
    __syncthreads();
  }
}

// Ping-pong variant: two streams of four wavefronts share the transform matrix in LDS
// and own one y buffer each (64 columns).  Between two barriers one stream runs its
// matrix phase while the other stores its previous results, refills its y from the
// prefetch registers and issues the loads of its chunk after next, so HBM traffic and
// MFMA overlap inside one workgroup.  Stream s handles chunks 2 blockIdx + s + 2 k gridDim.
//
// SYM = false: general complex T as three real GEMMs (t1 = Tr yr, t2 = Ti yi,
// t3 = (Tr + Ti)(yr + yi)).
// SYM = true: T[m][N-1-i] = s conj(T[m][i]) (s = +1 for bosonic, -1 for fermionic
// frequencies on a grid symmetric about beta/2).  Pairing tau_i with its mirror,
//   sum_i T_mi y_i = sum_{i < N/2} [Tr_mi u_i + i Ti_mi v_i] (+ the middle point),
//   u_i = y_i + s y_{N-1-i},  v_i = y_i - s y_{N-1-i},
// so Re = A [u_r ; -v_i] and Im = A [u_i ; v_r] with one real matrix A whose K rows are
// Tr_mi (row i, i <= (N-1)/2) and Ti_mi (row N-1-i, i < N/2; row N for the middle
// point of an odd N): two real GEMMs instead of three.  A thread loads a row and its
// mirror, forms u and v in registers (they commute with the R -> k sum) and writes
// (u_r, u_i) to row i and (-v_i, v_r) to row N-1-i of y.
template <int N1, int N2, int N3, int MT, bool SYM, class TI, class TO>
__global__ __launch_bounds__(512, 1) void drain_pp(const double2* __restrict__ T, int n_omega, int n_tau,
                                                   double sgn, const TI* in, TO* out, long long n2, int CB,
                                                   long long nchunks) {
  constexpr int NR = N1 * N2 * N3;
  constexpr int NCP = 64;                              // columns per stream chunk
  constexpr int PU = NR <= kPF ? kPF / NR : 1;          // (tau, element) columns per thread
  constexpr int PV = SYM ? PU / 2 : PU;                 // loaded units (a row pair when SYM)
  extern __shared__ double2 lds[];
  const int tid = threadIdx.x;
  const int nt4 = (n_tau + 7) & ~7, ld_t = nt4 + 1;  // K rounded to 8: an even number of K steps
  const int half = (n_tau + 1) / 2;                    // rows i <= mirror(i)
  double2* Ts = lds;                                   // [16 MT][ld_t] complex, or real when SYM
  double* As = reinterpret_cast<double*>(lds);
  const int tsz = SYM ? (16 * MT * ld_t + 1) / 2 : 16 * MT * ld_t;
  const int stream = tid >> 8, stid = tid & 255;       // 256 threads per stream
  double2* y = lds + tsz + stream * nt4 * NCP;
  for (int i = tid; i < 16 * MT * ld_t; i += 512) {
    const int m = i / ld_t, t = i - m * ld_t;
    if constexpr (SYM) {
      double a = 0.0;
      if (m < n_omega) {
        if (t < half) a = T[(long long)m * n_tau + t].x;
        else if (t < n_tau) a = T[(long long)m * n_tau + (n_tau - 1 - t)].y;
        else if (t == n_tau && (n_tau & 1)) a = T[(long long)m * n_tau + (half - 1)].y;
      }
      As[i] = a;
    } else {
      Ts[i] = (m < n_omega && t < n_tau) ? T[(long long)m * n_tau + t] : make_double2(0.0, 0.0);
    }
  }
  const int ncol = NR * CB;
  const int rows = (SYM && (n_tau & 1)) ? n_tau + 1 : n_tau;  // rows of y that fill() writes
  for (int idx = stid; idx < nt4 * NCP; idx += 256) {  // padding rows / columns stay zero
    const int t = idx / NCP, rc = idx - t * NCP;
    if (t >= rows || rc >= ncol) y[idx] = make_double2(0.0, 0.0);
  }
  const int lane = tid & 63, w = (tid >> 6) & 3, li = lane & 15, lk = lane >> 4;
  const int col = 16 * w + li;
  const int ksn = nt4 / 4;
  const long long stride = 2LL * gridDim.x;
  const long long first = 2LL * blockIdx.x + stream;
  const int trows = SYM ? half : n_tau;  // leading rows of the units a thread loads
  TI raw[PU * NR];
  auto fetch = [&](long long ch) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int p = stid + 256 * u, t = p / CB, c = p - t * CB;
      const bool live = ch < nchunks && t < trows && c < cb;
#pragma unroll
      for (int R = 0; R < NR; ++R) {
        if constexpr (SYM) {
          raw[(2 * u) * NR + R] = ldraw(in + ((long long)t * NR + R) * n2 + e0 + c, in, live);
          raw[(2 * u + 1) * NR + R] = ldraw(in + ((long long)(n_tau - 1 - t) * NR + R) * n2 + e0 + c, in, live);
        } else {
          raw[u * NR + R] = ldraw(in + ((long long)t * NR + R) * n2 + e0 + c, in, live);
        }
      }
    }
  };
  auto fill = [&](long long ch) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int p = stid + 256 * u, t = p / CB, c = p - t * CB;
      if (t < trows) {
        const bool live = c < cb;
        if constexpr (SYM) {
          const bool mid = t == n_tau - 1 - t;
          double ur[NR], ui[NR], vr[NR], vi[NR];
#pragma unroll
          for (int R = 0; R < NR; ++R) {
            const TI a = keep(raw[(2 * u) * NR + R], live), b = keep(raw[(2 * u + 1) * NR + R], live);
            const double br = mid ? 0.0 : sgn * (double)b.x, bi = mid ? 0.0 : sgn * (double)b.y;
            ur[R] = (double)a.x + br;
            ui[R] = (double)a.y + bi;
            vr[R] = (double)a.x - br;
            vi[R] = (double)a.y - bi;
          }
          r2k_regs<N1, N2, N3>(ur, ui);
          r2k_regs<N1, N2, N3>(vr, vi);
          const int t2 = mid ? n_tau : n_tau - 1 - t;
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            y[t * NCP + q * CB + c] = make_double2(ur[q], ui[q]);
            y[t2 * NCP + q * CB + c] = make_double2(-vi[q], vr[q]);
          }
        } else {
          double pr[NR], pi[NR];
#pragma unroll
          for (int R = 0; R < NR; ++R) {
            const TI v = keep(raw[u * NR + R], live);
            pr[R] = (double)v.x;
            pi[R] = (double)v.y;
          }
          r2k_regs<N1, N2, N3>(pr, pi);
#pragma unroll
          for (int q = 0; q < NR; ++q) y[t * NCP + q * CB + c] = make_double2(pr[q], pi[q]);
        }
      }
    }
  };
  d4 t1[MT], t2[MT], t3[MT];
  // Two named operand sets: the LDS reads of one K step are issued before the MFMAs of
  // the other, so a single wavefront keeps its SIMD's matrix pipe busy.
  typedef typename std::conditional<SYM, double, double2>::type AT;
  auto matrix = [&]() {
#pragma unroll
    for (int i = 0; i < MT; ++i) t1[i] = t2[i] = t3[i] = d4{0, 0, 0, 0};
    double2 ya, yb;
    AT ta[MT], tb[MT];
    auto load = [&](int ks, double2& yv, AT* tv) {
      const int tau = 4 * ks + lk;
      yv = y[tau * NCP + col];
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        if constexpr (SYM)
          tv[i] = As[(16 * i + li) * ld_t + tau];
        else
          tv[i] = Ts[(16 * i + li) * ld_t + tau];
      }
    };
    auto mma = [&](const double2& yv, const AT* tv) {
      if constexpr (SYM) {
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          t1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[i], yv.x, t1[i], 0, 0, 0);
          t2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[i], yv.y, t2[i], 0, 0, 0);
        }
      } else {
        const double ys = yv.x + yv.y;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          t1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[i].x, yv.x, t1[i], 0, 0, 0);
          t2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[i].y, yv.y, t2[i], 0, 0, 0);
          t3[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[i].x + tv[i].y, ys, t3[i], 0, 0, 0);
        }
      }
    };
    constexpr int NM = SYM ? 2 * MT : 3 * MT;  // MFMAs per K step
    load(0, ya, ta);
    for (int ks = 0; ks < ksn; ks += 2) {  // ksn is even; the last read of ya is a spare one
      load(ks + 1, yb, tb);
      mma(ya, ta);
      load(ks + 2 < ksn ? ks + 2 : ks, ya, ta);
      mma(yb, tb);
      // keep this order: reads of one set, MFMAs of the other, reads, MFMAs
      __builtin_amdgcn_sched_group_barrier(0x100, MT + 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, NM, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, MT + 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, NM, 0);
    }
  };
  auto store = [&](long long ch) {
    const long long e0 = ch * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
    if (col < ncol) {
      const int q = col / CB, c = col - q * CB;
      if (c < cb) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int m = 16 * i + lk + 4 * j;
            if (m < n_omega) {
              if constexpr (SYM)
                stc(out + ((long long)m * NR + q) * n2 + e0 + c, t1[i][j], t2[i][j]);
              else
                stc(out + ((long long)m * NR + q) * n2 + e0 + c, t1[i][j] - t2[i][j],
                    t3[i][j] - t1[i][j] - t2[i][j]);
            }
          }
      }
    }
  };
  // prologue: y <- chunk 0 of each stream, prefetch registers <- chunk 1
  fetch(first);
  __syncthreads();
  if (first < nchunks) fill(first);
  fetch(first + stride);
  __syncthreads();
  // half step h: stream h % 2 multiplies its chunk k = h / 2; the other stream stores
  // its chunk k' = (h - 1) / 2, refills y with k' + 1 and prefetches k' + 2
  const long long kmax = (nchunks - first + stride - 1) / stride;  // chunks of this stream
  const long long kmax0 = (nchunks - 2LL * blockIdx.x + stride - 1) / stride;
  const long long nhalf = 2 * kmax0 + 2;
  for (long long h = 0; h < nhalf; ++h) {
    if ((h & 1) == stream) {
      const long long k = h >> 1;
      if (k < kmax) matrix();
    } else if (h >= 1) {
      const long long k = (h - 1) >> 1;
      if (k < kmax) {
        store(first + k * stride);
        if (k + 1 < kmax) fill(first + (k + 1) * stride);
        fetch(first + (k + 2) * stride);
      }
    }
    __syncthreads();
  }
}

// Wide-chunk variant of the paired (SYM) drain for complex64 storage.  The ping-pong kernel
// moves 64 columns (CB = 64 / N_R elements per row of in and out, 64 bytes at N_R = 8) per
// step, and at that segment size the scattered in-place read and write of 2 x n_tau x N_R rows
// runs at about 2.5 TB/s; 256-byte row segments run near 3.8 TB/s.  So a workgroup here owns
// 256 columns (CB = 256 / N_R elements of every row) per chunk.  To fit LDS, the staged y
// (u / v paired rows after the R -> k butterflies, computed in FP64) is held in complex64,
// the storage precision of the input and the output; the tau contraction stays FP64 MFMA.
// One chunk per iteration, all eight wavefronts in both phases:
//   fill(k)   -- every thread pairs and transforms its units (tau row pair, element) of chunk k
//                from registers into y;
//   barrier;
//   matrix(k)  -- wavefront w multiplies the 32 columns 32 w .. 32 w + 31 by A, one m tile at a
//                time, and stores each tile (two 16-element runs of one q row: 256 bytes at
//                N_R = 8); the loads of chunk k + 1 go out one unit per m tile, so that loads
//                and stores spread over the product phase and land before the next fill;
//   barrier (y is free again).
// Shapes: N_R in {2, 4, 8}, n_tau <= 64, n_omega <= 16 MT <= 64.  A rows are padded by one
// entry (the 16 rows of an A operand read then fall in distinct banks); where that does not fit
// LDS (n_tau > 56 with four m tiles) they are stored unpadded with their columns XOR-swizzled by
// m % 16 instead, and at n_tau = n_omega = 64 y and A fill the 160 KiB of LDS exactly.
constexpr int kWideThreads = 512;
constexpr int kWideCols = 256;
constexpr int kWideMaxTau = 64;

template <int N1, int N2, int N3, int MT, bool SWZ>
__global__ __launch_bounds__(512, 1) void drain_wide(const double2* __restrict__ T, int n_omega, int n_tau,
                                                     double sgn, const float2* in, float2* out, long long n2,
                                                     long long nchunks) {
  constexpr int NR = N1 * N2 * N3;
  constexpr int NCP = kWideCols;
  constexpr int CB = NCP / NR;  // elements per chunk; N_R divides 256
  static_assert(NR * CB == NCP, "the mesh size must divide 256");
  constexpr int UPL = ((kWideMaxTau / 2) * CB + kWideThreads - 1) / kWideThreads;  // units per thread
  extern __shared__ double2 lds[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int nt8 = (n_tau + 7) & ~7;
  // A rows: padded to nt8 + 1, or (SWZ) of length n_tau rounded up to 16 with entry t of row m
  // at t ^ (m % 16)
  constexpr int swz = SWZ ? 15 : 0;
  const int ld_t = SWZ ? (n_tau + 15) & ~15 : nt8 + 1;
  const int half = (n_tau + 1) / 2;
  const int rows = (n_tau & 1) ? n_tau + 1 : n_tau;  // rows of y that fill() writes
  float2* Y = reinterpret_cast<float2*>(lds);         // [nt8][NCP]
  double* As = reinterpret_cast<double*>(Y + nt8 * NCP);  // [16 MT][ld_t], columns swizzled
  // K row t of the paired form: Re T[m][t] for t < half, Im T[m][n_tau - 1 - t] for half <= t <
  // n_tau, Im T[m][half - 1] at t = n_tau for odd n_tau; zero beyond
  for (int i = tid; i < 16 * MT * ld_t; i += kWideThreads) {
    const int m = i / ld_t, t = (i - m * ld_t) ^ (m & swz);
    double a = 0.0;
    if (m < n_omega) {
      if (t < half) a = T[(long long)m * n_tau + t].x;
      else if (t < n_tau) a = T[(long long)m * n_tau + (n_tau - 1 - t)].y;
      else if (t == n_tau && (n_tau & 1)) a = T[(long long)m * n_tau + (half - 1)].y;
    }
    As[i] = a;
  }
  for (int i = tid; i < (nt8 - rows) * NCP; i += kWideThreads) Y[rows * NCP + i] = make_float2(0.f, 0.f);
  const long long stride = gridDim.x;
  const long long first = blockIdx.x;
  const long long kmax = first < nchunks ? (nchunks - first + stride - 1) / stride : 0;
  const int ksn = nt8 / 4;

  float2 raw[UPL][2 * NR];
  auto fetch = [&](long long k, int vsel) {  // the loads of unit vsel of every thread, or all (-1)
    const long long e0 = (first + k * stride) * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
#pragma unroll
    for (int v = 0; v < UPL; ++v) {
      if (vsel >= 0 && v != vsel) continue;
      const int u = tid + kWideThreads * v, ut = u / CB, uc = u - ut * CB;
      const bool live = ut < half && uc < cb;
      const float2* pa = in + (long long)ut * NR * n2 + e0 + uc;
      const float2* pb = in + (long long)(n_tau - 1 - ut) * NR * n2 + e0 + uc;
#pragma unroll
      for (int R = 0; R < NR; ++R) {
        raw[v][R] = ldraw(pa + R * n2, in, live);
        raw[v][NR + R] = ldraw(pb + R * n2, in, live);
      }
    }
  };
  auto fill = [&](long long k) {
    const long long e0 = (first + k * stride) * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
#pragma unroll
    for (int v = 0; v < UPL; ++v) {
      const int u = tid + kWideThreads * v, ut = u / CB, uc = u - ut * CB;
      if (ut >= half) continue;
      const bool live = uc < cb;
      const bool mid = ut == n_tau - 1 - ut;
      const int t2 = mid ? n_tau : n_tau - 1 - ut;
      const double sb = mid ? 0.0 : sgn;  // weight of the mirror row
      // u = y + s y' to row ut, then v = y - s y' as (-v_i, v_r) to row t2
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double wgt = h == 0 ? sb : -sb;
        double xr[NR], xi[NR];
#pragma unroll
        for (int R = 0; R < NR; ++R) {
          const float2 a = keep(raw[v][R], live), b = keep(raw[v][NR + R], live);
          xr[R] = fma(wgt, (double)b.x, (double)a.x);
          xi[R] = fma(wgt, (double)b.y, (double)a.y);
        }
        r2k_regs<N1, N2, N3>(xr, xi);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          if (h == 0)
            Y[ut * NCP + q * CB + uc] = make_float2((float)xr[q], (float)xi[q]);
          else
            Y[t2 * NCP + q * CB + uc] = make_float2((float)-xi[q], (float)xr[q]);
        }
      }
    }
  };
  // output column of tile h of this wavefront: q row and element within the chunk
  int oq[2], oe[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = 32 * w + 16 * h + li;
    oq[h] = col / CB;
    oe[h] = col - oq[h] * CB;
  }
  // one m tile at a time: the loads of one unit of the next chunk, the tile's products, then its
  // stores, so that loads and stores spread over the product phase instead of arriving in bursts
  auto matrix_store = [&](long long k) {
    const long long e0 = (first + k * stride) * CB;
    const int cb = (int)((n2 - e0) < CB ? (n2 - e0) : CB);
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      if (i < UPL && k + 1 < kmax) fetch(k + 1, i);
      d4 acc[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h][0] = acc[h][1] = d4{0, 0, 0, 0};
      for (int ks = 0; ks < ksn; ++ks) {
        const int t = 4 * ks + lk;
        const float2 y0 = Y[t * NCP + 32 * w + li], y1 = Y[t * NCP + 32 * w + 16 + li];
        const double a = As[(16 * i + li) * ld_t + (t ^ (li & swz))];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)y0.x, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)y0.y, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)y1.x, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)y1.y, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (oe[h] >= cb) continue;
        float2* p = out + (long long)oq[h] * n2 + e0 + oe[h];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = 16 * i + lk + 4 * j;
          if (m < n_omega) p[(long long)m * NR * n2] = make_float2((float)acc[h][0][j], (float)acc[h][1][j]);
        }
      }
    }
  };
  if (kmax > 0) fetch(0, -1);
  for (long long k = 0; k < kmax; ++k) {
    fill(k);
    __syncthreads();  // y of chunk k complete (and, at k = 0, A and the zero rows)
    if (k + 1 < kmax)
      for (int v = MT; v < UPL; ++v) fetch(k + 1, v);  // units beyond the m tiles' share
    matrix_store(k);
    __syncthreads();  // every wavefront done reading y
  }
}

// Plain FP64 VALU transform for sizes outside the MFMA kernel's range (tau <= 256).
template <class TI, class TO>
__global__ __launch_bounds__(256) void tau2omega_valu(const double2* __restrict__ T, int n_omega, int n_tau,
                                                      const TI* in, TO* out, long long cols, int CB) {
  extern __shared__ double2 xs[];  // [n_tau][CB]
  const long long c0 = (long long)blockIdx.x * CB;
  for (int idx = threadIdx.x; idx < n_tau * CB; idx += 256) {
    const int t = idx / CB, c = idx - t * CB;
    double a = 0, b = 0;
    if (c0 + c < cols) ldc(in + (long long)t * cols + c0 + c, a, b);
    xs[idx] = make_double2(a, b);
  }
  __syncthreads();
  const int c = threadIdx.x % CB, g = threadIdx.x / CB, G = 256 / CB;
  if (c0 + c >= cols) return;
  for (int m = g; m < n_omega; m += G) {
    double ar = 0, ai = 0;
    for (int t = 0; t < n_tau; ++t) {
      const double2 tv = T[(long long)m * n_tau + t];
      const double2 v = xs[t * CB + c];
      ar += tv.x * v.x - tv.y * v.y;
      ai += tv.x * v.y + tv.y * v.x;
    }
    stc(out + (long long)m * cols + c0 + c, ar, ai);
  }
}

template <int N1, int N2, int N3, int MT, class TI, class TO>
void run_drain_3m(const double2* T, int n_omega, int n_tau, const TI* in, TO* out, long long n2, size_t lds,
                  int waves, int CB, hipStream_t s) {
  constexpr int NR = N1 * N2 * N3;
  const long long nchunks = (n2 + CB - 1) / CB;
  const long long grid = nchunks < 256 ? nchunks : 256;
  const bool reg = NR <= kPF && (long long)n_tau * CB <= (long long)(kPF / NR) * 64 * waves;
  if constexpr (NR <= kPF) {
    if (reg) {
      if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)drain_3m<N1, N2, N3, MT, true, TI, TO>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((drain_3m<N1, N2, N3, MT, true, TI, TO>), dim3((unsigned)grid), dim3(64 * waves), lds,
                         s, T, n_omega, n_tau, in, out, n2, CB, nchunks);
      return;
    }
  }
  {
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)drain_3m<N1, N2, N3, MT, false, TI, TO>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((drain_3m<N1, N2, N3, MT, false, TI, TO>), dim3((unsigned)grid), dim3(64 * waves), lds,
                       s, T, n_omega, n_tau, in, out, n2, CB, nchunks);
  }
}

template <int N1, int N2, int N3, class TI, class TO>
void run_drain(const double2* T, int n_omega, int n_tau, int parity, const TI* in, TO* out, long long n2,
               hipStream_t s) {
  constexpr int NR = N1 * N2 * N3;
  const int MT = (n_omega + 15) / 16;
  const int nt4 = (n_tau + 3) & ~3;
  // wide-chunk kernel for the paired drain in complex64 storage (the mixed path's P drain)
  if constexpr (NR >= 2 && NR <= 8 && kWideCols % NR == 0 && std::is_same<TI, float2>::value &&
                std::is_same<TO, float2>::value) {
    if (parity != 0 && n_tau <= kWideMaxTau && n_omega <= 64 && !wide_disabled()) {
      constexpr int CBW = kWideCols / NR;
      const long long nchunks = (n2 + CBW - 1) / CBW;
      const int nt8 = (n_tau + 7) & ~7;
      int dev = 0, n_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        n_cu = 256;
      const long long grid = nchunks < n_cu ? nchunks : n_cu;
      const size_t ly = (size_t)nt8 * kWideCols * sizeof(float2);
      auto go = [&](auto kern, int mt, bool swz) {
        const size_t lds = ly + (size_t)16 * mt * (swz ? (n_tau + 15) & ~15 : nt8 + 1) * sizeof(double);
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kWideThreads), lds, s, T, n_omega, n_tau,
                           parity < 0 ? -1.0 : 1.0, (const float2*)in, (float2*)out, n2, nchunks);
      };
      if (MT == 1) go(drain_wide<N1, N2, N3, 1, false>, 1, false);
      else if (MT == 2) go(drain_wide<N1, N2, N3, 2, false>, 2, false);
      else if (MT == 3) go(drain_wide<N1, N2, N3, 3, false>, 3, false);
      else if (ly + (size_t)64 * (nt8 + 1) * sizeof(double) <= 160 * 1024) go(drain_wide<N1, N2, N3, 4, false>, 4, false);
      else go(drain_wide<N1, N2, N3, 4, true>, 4, true);
      return;
    }
  }
  // ping-pong kernel: two 64-column streams; needs whole (tau, element) columns per thread
  if constexpr (NR <= kPF) {
    const bool sym = parity != 0 && kPF / NR >= 2;
    const int CB = NR >= 64 ? 1 : 64 / NR;
    const int nt8 = (n_tau + 7) & ~7;
    const size_t tsz = sym ? (size_t)(16 * MT * (nt8 + 1) + 1) / 2 : (size_t)16 * MT * (nt8 + 1);
    const size_t lds = (tsz + 2 * (size_t)nt8 * 64) * sizeof(double2);
    const int units = kPF / NR / (sym ? 2 : 1);                 // loads per thread
    const long long need = (long long)(sym ? (n_tau + 1) / 2 : n_tau) * CB;
    if (MT <= 4 && NR * CB <= 64 && lds <= 160 * 1024 && need <= (long long)units * 256) {
      const long long nchunks = (n2 + CB - 1) / CB;
      const long long grid = (nchunks + 1) / 2 < 256 ? (nchunks + 1) / 2 : 256;
      const double sgn = parity < 0 ? -1.0 : 1.0;
#define GWR_PP(mt, sy)                                                                                       \
  if (MT == mt && sym == sy) {                                                                               \
    (void)hipFuncSetAttribute((const void*)drain_pp<N1, N2, N3, mt, sy, TI, TO>,                             \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                         \
    hipLaunchKernelGGL((drain_pp<N1, N2, N3, mt, sy, TI, TO>), dim3((unsigned)grid), dim3(512), lds, s, T,   \
                       n_omega, n_tau, sgn, in, out, n2, CB, nchunks);                                       \
    return;                                                                                                  \
  }
      GWR_PP(1, false)
      GWR_PP(2, false)
      GWR_PP(3, false)
      GWR_PP(4, false)
      if constexpr (kPF / NR >= 2) {
        GWR_PP(1, true)
        GWR_PP(2, true)
        GWR_PP(3, true)
        GWR_PP(4, true)
      }
#undef GWR_PP
    }
  }
  // persistent 3M kernel: the widest chunk (<= 128 columns) whose T + y fit in LDS and
  // whose prefetch fits the per-thread register budget
  for (int cols = 128; cols >= 16 && MT <= 4; cols /= 2) {
    const int CB = NR >= cols ? 1 : cols / NR;
    const int waves = (NR * CB + 15) / 16;
    if (waves > 8) continue;
    const size_t lds = (size_t)(16 * MT * (nt4 + 1) + nt4 * 16 * waves) * sizeof(double2);
    if (lds > 160 * 1024 || nt4 * 16 * waves > kPF * 64 * waves) continue;
    switch (MT) {
      case 1: run_drain_3m<N1, N2, N3, 1>(T, n_omega, n_tau, in, out, n2, lds, waves, CB, s); return;
      case 2: run_drain_3m<N1, N2, N3, 2>(T, n_omega, n_tau, in, out, n2, lds, waves, CB, s); return;
      case 3: run_drain_3m<N1, N2, N3, 3>(T, n_omega, n_tau, in, out, n2, lds, waves, CB, s); return;
      case 4: run_drain_3m<N1, N2, N3, 4>(T, n_omega, n_tau, in, out, n2, lds, waves, CB, s); return;
      default: break;
    }
  }
  const int CB = kDrainCols / NR;
  const unsigned blocks = (unsigned)((n2 + CB - 1) / CB);
  const size_t lds = (size_t)((n_tau + 1) / 2 * 2) * kDrainCols * sizeof(double2);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)drain_mfma<N1, N2, N3, TI, TO>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((drain_mfma<N1, N2, N3, TI, TO>), dim3(blocks), dim3(256), lds, s, T, n_omega, n_tau, in,
                     out, n2, CB);
}

template <class TI, class TO>
void run_valu(const double2* T, int n_omega, int n_tau, const TI* in, TO* out, long long cols, hipStream_t s) {
  const int CB = n_tau <= 64 ? 64 : (n_tau <= 128 ? 32 : 16);
  const unsigned blocks = (unsigned)((cols + CB - 1) / CB);
  hipLaunchKernelGGL((tau2omega_valu<TI, TO>), dim3(blocks), dim3(256), (size_t)n_tau * CB * sizeof(double2), s,
                     T, n_omega, n_tau, in, out, cols, CB);
}

bool mfma_ok(int n_tau, int n_omega) { return n_tau <= kDrainMaxTau && n_omega <= kDrainMaxOmega; }

// dispatch on the mesh; returns false if the mesh has no fused kernel
template <class TI, class TO>
bool drain_dispatch(const gw_cell* c, const double2* T, int n_omega, int parity, const TI* in, TO* out,
                    long long n2, hipStream_t s) {
  const int a = c->mesh[0], b = c->mesh[1], d = c->mesh[2];
#define GWR_DRAIN(x, y, z)                                                \
  if (a == x && b == y && d == z) {                                       \
    run_drain<x, y, z>(T, n_omega, c->n_tau, parity, in, out, n2, s);     \
    return true;                                                          \
  }
  GWR_DRAIN(1, 1, 1)
  GWR_DRAIN(2, 2, 2)
  GWR_DRAIN(2, 2, 1)
  GWR_DRAIN(3, 2, 1)
  GWR_DRAIN(4, 4, 4)
  GWR_DRAIN(4, 4, 2)
  GWR_DRAIN(2, 1, 1)
#undef GWR_DRAIN
  return false;
}

template <class TI, class TO>
gw_status tau2omega_typed(const gw_cell* c, const double2* T, int n_omega, int parity, const TI* in, TO* out,
                          long long cols, hipStream_t s) {
  if (mfma_ok(c->n_tau, n_omega))
    run_drain<1, 1, 1>(T, n_omega, c->n_tau, parity, in, out, cols, s);
  else
    run_valu(T, n_omega, c->n_tau, in, out, cols, s);
  return check_launch("tau2omega");
}

template <class TI, class TO>
gw_status drain_typed(const gw_cell* c, const double2* T, int n_omega, int parity, const TI* in, TO* out, int n,
                      gw_dtype ot, hipStream_t s) {
  const long long n2 = (long long)n * n;
  // two passes through `out` (R -> k, then tau -> omega over N_R n^2 columns) need room for
  // n_tau rows there: in place, or n_omega >= n_tau
  const bool two_pass_ok = (const void*)in == (const void*)out || n_omega >= c->n_tau;
  // A fused pass keeps whole (tau, element) columns of N_R values per thread only up to N_R = 16;
  // beyond that its chunks hold a few elements per (tau, R) row, short scattered accesses, and
  // the two coalesced passes are the faster route.
  const bool fused_pref = c->N_R <= kPF || !two_pass_ok;
  if (fused_pref && mfma_ok(c->n_tau, n_omega) && drain_dispatch(c, T, n_omega, parity, in, out, n2, s))
    return check_launch("drain");
  if (!two_pass_ok)
    return fail(GW_ERR_UNSUPPORTED, "this mesh / grid needs n_omega >= n_tau or an in-place drain");
  gw_status st = launch_fourier(c, in, sizeof(TI) == 16 ? GW_C128 : GW_C64, out, ot, n, -1, s);
  if (st != GW_OK) return st;
  return tau2omega_typed(c, T, n_omega, parity, out, out, (long long)c->N_R * n2, s);
}

}  // namespace
}  // namespace gwr

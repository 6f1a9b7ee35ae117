// Lattice sums between k and R (Sec. 2: the F^R storage and the R <-> k transforms).
//
//   out^R = scale * sum_k exp(sign * i k.R) in(k)   per tau and per matrix element.
//
// HBM-bound: every element is read once and written once.  One thread owns one
// (tau, element) column of N_R values held in registers; consecutive threads own
// consecutive elements, so each of the N_R loads and stores of a wavefront is a
// contiguous 1 KiB (complex128) run.  The 3-D transform is done as three 1-D
// passes (separable), fully unrolled for the meshes in the table below; other
// meshes use a dense N_R x N_R sum staged through LDS.
#include "cplx.h"
#include "internal.h"

namespace gwr {
namespace {

// One 1-D DFT pass of length L along an axis with inner stride S, over O outer groups,
// acting on the register arrays re/im of size O*L*S.
template <int O, int L, int S, int SIGN>
__device__ __forceinline__ void dft_pass(double* re, double* im) {
  if constexpr (L == 1) {
    return;
  } else {
    double cw[L], sw[L];
#pragma unroll
    for (int m = 0; m < L; ++m) turn((double)(SIGN * m) / (double)L, cw[m], sw[m]);
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
#pragma unroll
        for (int j = 0; j < L; ++j) {
          double ar = 0, ai = 0;
#pragma unroll
          for (int l = 0; l < L; ++l) {
            const int m = (j * l) % L;
            ar += cw[m] * xr[l] - sw[m] * xi[l];
            ai += cw[m] * xi[l] + sw[m] * xr[l];
          }
          re[(o * L + j) * S + i] = ar;
          im[(o * L + j) * S + i] = ai;
        }
      }
    }
  }
}

template <int N1, int N2, int N3, int SIGN, class TI, class TO>
__global__ __launch_bounds__(256) void fourier_sep(const TI* __restrict__ in, TO* __restrict__ out,
                                                   long long ncols, long long n2, double scale) {
  constexpr int NR = N1 * N2 * N3;
  const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncols) return;
  const long long t = col / n2, e = col - t * n2;
  const long long base = t * NR * n2 + e;
  double re[NR], im[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) ldc(in + base + r * n2, re[r], im[r]);
  dft_pass<N1 * N2, N3, 1, SIGN>(re, im);
  dft_pass<N1, N2, N3, SIGN>(re, im);
  dft_pass<1, N1, N2 * N3, SIGN>(re, im);
#pragma unroll
  for (int r = 0; r < NR; ++r) stc(out + base + r * n2, scale * re[r], scale * im[r]);
}

// Dense fallback for any mesh up to 64 points: 64 columns per block staged in LDS.
template <class TI, class TO>
__global__ __launch_bounds__(64) void fourier_dense(const TI* __restrict__ in, TO* __restrict__ out,
                                                    long long ncols, long long n2, int N1, int N2, int N3,
                                                    int sign, double scale) {
  __shared__ double2 x[kMaxR][64];
  const int NR = N1 * N2 * N3;
  const long long col = (long long)blockIdx.x * 64 + threadIdx.x;
  const bool live = col < ncols;
  const long long t = live ? col / n2 : 0, e = live ? col - t * n2 : 0;
  const long long base = t * NR * n2 + e;
  if (live)
    for (int r = 0; r < NR; ++r) {
      double a, b;
      ldc(in + base + r * n2, a, b);
      x[r][threadIdx.x] = make_double2(a, b);
    }
  __syncthreads();
  if (!live) return;
  for (int ro = 0; ro < NR; ++ro) {
    const int j1 = ro / (N2 * N3), j2 = (ro / N3) % N2, j3 = ro % N3;
    double ar = 0, ai = 0;
    for (int r = 0; r < NR; ++r) {
      const int n1 = r / (N2 * N3), m2 = (r / N3) % N2, n3 = r % N3;
      const double frac = (double)((j1 * n1) % N1) / N1 + (double)((j2 * m2) % N2) / N2 +
                          (double)((j3 * n3) % N3) / N3;
      double c, s;
      turn(sign * frac, c, s);
      const double2 v = x[r][threadIdx.x];
      ar += c * v.x - s * v.y;
      ai += c * v.y + s * v.x;
    }
    stc(out + base + ro * n2, scale * ar, scale * ai);
  }
}

template <int N1, int N2, int N3, class TI, class TO>
void run_sep(const TI* in, TO* out, long long ncols, long long n2, int sign, double scale, hipStream_t s) {
  const unsigned blocks = (unsigned)((ncols + 255) / 256);
  if (sign > 0)
    hipLaunchKernelGGL((fourier_sep<N1, N2, N3, 1, TI, TO>), dim3(blocks), dim3(256), 0, s, in, out, ncols, n2,
                       scale);
  else
    hipLaunchKernelGGL((fourier_sep<N1, N2, N3, -1, TI, TO>), dim3(blocks), dim3(256), 0, s, in, out, ncols,
                       n2, scale);
}

template <class TI, class TO>
void dispatch(const gw_cell* c, const TI* in, TO* out, long long ncols, long long n2, int sign, double scale,
              hipStream_t s) {
  const int a = c->mesh[0], b = c->mesh[1], d = c->mesh[2];
#define GWR_MESH(x, y, z)                                            \
  if (a == x && b == y && d == z) {                                  \
    run_sep<x, y, z>(in, out, ncols, n2, sign, scale, s);            \
    return;                                                          \
  }
  GWR_MESH(1, 1, 1)
  GWR_MESH(2, 2, 2)
  GWR_MESH(2, 2, 1)
  GWR_MESH(3, 2, 1)
  GWR_MESH(4, 4, 4)
  GWR_MESH(3, 3, 3)
  GWR_MESH(4, 4, 2)
  GWR_MESH(2, 1, 1)
#undef GWR_MESH
  const unsigned blocks = (unsigned)((ncols + 63) / 64);
  hipLaunchKernelGGL((fourier_dense<TI, TO>), dim3(blocks), dim3(64), 0, s, in, out, ncols, n2, a, b, d, sign,
                     scale);
}

}  // namespace

gw_status launch_fourier(const gw_cell* c, const void* in, gw_dtype it, void* out, gw_dtype ot, int n, int sign,
                         hipStream_t s) {
  const long long n2 = (long long)n * n;
  const long long ncols = (long long)c->n_tau * n2;
  const double scale = sign > 0 ? 1.0 / c->N_R : 1.0;
  if (ncols == 0) return GW_OK;
  if (it == GW_C128 && ot == GW_C128)
    dispatch(c, (const double2*)in, (double2*)out, ncols, n2, sign, scale, s);
  else if (it == GW_C128 && ot == GW_C64)
    dispatch(c, (const double2*)in, (float2*)out, ncols, n2, sign, scale, s);
  else if (it == GW_C64 && ot == GW_C128)
    dispatch(c, (const float2*)in, (double2*)out, ncols, n2, sign, scale, s);
  else
    dispatch(c, (const float2*)in, (float2*)out, ncols, n2, sign, scale, s);
  return check_launch("fourier");
}

}  // namespace gwr

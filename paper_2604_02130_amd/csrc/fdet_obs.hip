// Observables from the Green's functions on gfx950.
//
// Sec. 4, shortcut for simple operators: the expectation value of an operator
// A is a trace of A against the Green's function; at the slice where the
// partial products are empty that is tr((1 - G) A) = tr A - sum_ij G_ij A_ji.
// A = nullptr stands for A = 1 / V, the fermion number n = 1 - tr G / V
// (eq. fermion_number).
//
// The work is two reads of N^2 complex numbers (HBM-bound).  One workgroup
// per 32 x 32 tile reads its tile of G along rows and the transposed tile of
// A along rows too (both coalesced), meeting through LDS; a second one-
// workgroup kernel adds the per-tile partials in a fixed order, so the result
// does not depend on scheduling.
//
// The same shortcut summed over every slice, for a diagonal operator, is read
// off the force sweep's output instead (k_diag_response below).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int TB = 32;       // tile edge
constexpr int TWG = 256;     // threads per workgroup
constexpr int TWAVE = TWG / 64;

__device__ __forceinline__ double obs_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of the workgroup's four values, valid in thread 0.
__device__ __forceinline__ void obs_block_sum4(double (&v)[4], double (*red)[TWAVE]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = obs_wave_sum(v[q]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = 0.0;
      for (int w = 0; w < TWAVE; ++w) s += red[q][w];
      v[q] = s;
    }
  }
}

// Tile (bi, bj) = rows i0 .. i0 + 31 of G, columns j0 .. j0 + 31.  Writes
// part[4 t .. 4 t + 3] = (Re, Im) of sum G_ij A_ji over the tile and of
// sum A_ii over its diagonal (diagonal tiles only), t = bj * nb + bi.  With
// A == nullptr the first pair is sum G_ii over the diagonal.
__global__ __launch_bounds__(TWG) void k_trace_tiles(int N, const double* __restrict__ G,
                                                     const double* __restrict__ A,
                                                     double* __restrict__ part) {
  __shared__ double atr[TB][TB + 1], ati[TB][TB + 1];   // atr[jj][ii] = Re A(j0 + jj, i0 + ii)
  __shared__ double red[4][TWAVE];
  const int nb = gridDim.x;
  const int bi = blockIdx.x, bj = blockIdx.y;
  const int i0 = bi * TB, j0 = bj * TB;
  const int tid = threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (A) {
    for (int e = tid; e < TB * TB; e += TWG) {
      const int jj = e >> 5, ii = e & (TB - 1);
      const int j = j0 + jj, i = i0 + ii;
      double ar = 0.0, ai = 0.0;
      if (i < N && j < N) {
        const size_t o = 2 * ((size_t)j * N + i);
        ar = A[o];
        ai = A[o + 1];
      }
      atr[jj][ii] = ar;
      ati[jj][ii] = ai;
    }
    __syncthreads();
    for (int e = tid; e < TB * TB; e += TWG) {
      const int ii = e >> 5, jj = e & (TB - 1);
      const int i = i0 + ii, j = j0 + jj;
      if (i < N && j < N) {
        const size_t o = 2 * ((size_t)i * N + j);
        const double gr = G[o], gi = G[o + 1];
        const double ar = atr[jj][ii], ai = ati[jj][ii];
        v[0] = fma(gr, ar, v[0]);
        v[0] = fma(-gi, ai, v[0]);
        v[1] = fma(gr, ai, v[1]);
        v[1] = fma(gi, ar, v[1]);
        if (i == j) {
          v[2] += ar;
          v[3] += ai;
        }
      }
    }
  } else if (bi == bj) {
    for (int ii = tid; ii < TB; ii += TWG) {
      const int i = i0 + ii;
      if (i < N) {
        const size_t o = 2 * ((size_t)i * N + i);
        v[0] += G[o];
        v[1] += G[o + 1];
      }
    }
  }
  obs_block_sum4(v, red);
  if (tid == 0) {
    const size_t t = (size_t)bj * nb + bi;
#pragma unroll
    for (int q = 0; q < 4; ++q) part[4 * t + q] = v[q];
  }
}

// out = tr A - sum G_ij A_ji, or 1 - tr G / N without A.
__global__ __launch_bounds__(TWG) void k_trace_final(int N, int ntile, int has_a,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ out) {
  __shared__ double red[4][TWAVE];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < ntile; t += TWG) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += part[4 * (size_t)t + q];
  }
  obs_block_sum4(v, red);
  if (threadIdx.x == 0) {
    if (has_a) {
      out[0] = v[2] - v[0];
      out[1] = v[3] - v[1];
    } else {
      out[0] = 1.0 - v[0] / N;
      out[1] = -v[1] / N;
    }
  }
}

// Average over the slices of the response to diag(a):
//   out = (1 / N_t) sum_t sum_x a_x (1 - G~_t)_xx,  (1 - G~_t)_xx = Im F - i Re F,
// from the force sweep's output (F_{t,x} = i (1 - G~_t)_xx); a == nullptr
// stands for a_x = 1 / N.  One workgroup, rows of the force read along x
// (coalesced), partial sums in a fixed order.
__global__ __launch_bounds__(TWG) void k_diag_response(int Nt, int N,
                                                       const double* __restrict__ fre,
                                                       const double* __restrict__ fim,
                                                       const double* __restrict__ a,
                                                       double* __restrict__ out) {
  __shared__ double red[4][TWAVE];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const double inv_n = 1.0 / N;
  const int64_t total = (int64_t)Nt * N;
  for (int64_t k = threadIdx.x; k < total; k += TWG) {
    const int x = (int)(k % N);
    const double w = a ? a[x] : inv_n;
    v[0] = fma(w, fim[k], v[0]);
    v[1] = fma(-w, fre[k], v[1]);
  }
  obs_block_sum4(v, red);
  if (threadIdx.x == 0) {
    out[0] = v[0] / Nt;
    out[1] = v[1] / Nt;
  }
}

}  // namespace

extern "C" hipError_t fdet_launch_diag_response(int Nt, int N, const double* fre, const double* fim,
                                                const double* a, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_response, dim3(1), dim3(TWG), 0, st, Nt, N, fre, fim, a, out);
  return hipGetLastError();
}

// part: 4 * nb * nb doubles, nb = ceil(N / 32); the host checks N and the sizes.
extern "C" hipError_t fdet_launch_trace(int N, const double* G, const double* A, double* part,
                                        double* out, hipStream_t st) {
  const int nb = (N + TB - 1) / TB;
  hipLaunchKernelGGL(k_trace_tiles, dim3(nb, nb), dim3(TWG), 0, st, N, G, A, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trace_final, dim3(1), dim3(TWG), 0, st, N, nb * nb, A ? 1 : 0, part, out);
  return hipGetLastError();
}

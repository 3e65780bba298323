// Device building blocks for the stabilised fermion determinant on gfx950.
//
// Every routine here is executed by one whole workgroup (WG threads, NWAVE
// 64-wide waves).  Complex matrices are
// planar (separate real and imaginary blocks) and column-major with leading
// dimension ld = Np, the size rounded up to the 16-row MFMA tile; loaders mask
// everything outside N x N, so padding is never read as data.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fdet {

constexpr int WG = 512;
constexpr int NWAVE = WG / 64;

typedef double v4d __attribute__((ext_vector_type(4)));

struct CMat {
  double* re;
  double* im;
  int ld;
  __device__ __forceinline__ double& r(int i, int j) const { return re[(size_t)j * ld + i]; }
  __device__ __forceinline__ double& m(int i, int j) const { return im[(size_t)j * ld + i]; }
};

__host__ __device__ __forceinline__ size_t cmat_doubles(int Np) { return (size_t)2 * Np * Np; }

__device__ __forceinline__ CMat cmat_at(double* base, int Np) {
  CMat c;
  c.re = base;
  c.im = base + (size_t)Np * Np;
  c.ld = Np;
  return c;
}

// Per-workgroup shared state; MAXN bounds the problem size handled.
template <int MAXN>
struct Smem {
  double norms[MAXN];   // partial column norms / scratch values by position
  int tmp0[MAXN];       // scratch index maps of the pivot refresh
  int tmp1[MAXN];
  double csp[MAXN];     // column scale key of the column at each position
  int piv[MAXN];        // original column index at each position
  int pinv[MAXN];       // inverse of piv
  double u0r[MAXN];     // first component of each reflector
  double u0i[MAXN];
  double beta[MAXN];    // reflector scale: H = I - beta u u^H
  double v1[MAXN];      // general per-row vectors
  double v2[MAXN];
  double v3[MAXN];
  double phr[MAXN];     // cos / sin of the field on one slice
  double phi_[MAXN];
  double red[4 * NWAVE];
  double rdr[MAXN];     // diagonal of R by position (register QR)
  double rdi[MAXN];
  int nref;
  int flag;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// f(i, j) over 0 <= i, j < N: columns by wave, rows by lane (coalesced on
// column-major data, no integer division).
template <class F>
__device__ __forceinline__ void for_each_ij(int N, F&& f) {
  for (int j = threadIdx.x >> 6; j < N; j += NWAVE)
    for (int i = threadIdx.x & 63; i < N; i += 64) f(i, j);
}

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace fdet

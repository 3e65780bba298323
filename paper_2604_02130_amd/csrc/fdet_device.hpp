// Device building blocks for the stabilised fermion determinant on gfx950.
//
// Every routine here is executed by one whole workgroup (WG threads, NWAVE
// 64-wide waves) and works on matrices in device memory.  Complex matrices are
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
  double candk[NWAVE];  // per-wave pivot candidates: key, norm, index
  double candn[NWAVE];
  int candi[NWAVE];
  double red[4 * NWAVE];
  double gck[32];       // per-lane-group pivot candidates (register QR)
  double gcn[32];
  int gcc[32];
  double ubr[MAXN];     // reflector broadcast buffer (register QR)
  double ubi[MAXN];
  double rdr[MAXN];     // diagonal of R by position (register QR)
  double rdi[MAXN];
  double a0r, a0i;
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

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Tiled products on the FP64 matrix cores.  A wave owns 16 x 16 output tiles
// round-robin.  For v_mfma_f64_16x16x4f64 lane l supplies A(i0 + l%16,
// k0 + l/16) and B(k0 + l/16, j0 + l%16) and receives C(i0 + l/16 + 4 r,
// j0 + l%16) in accumulator element r (checked on gfx950).
// ---------------------------------------------------------------------------

// real A x real B -> real C.  la(i,k) -> double, lb(k,j) -> double, st(i,j,c)
template <class LA, class LB, class ST>
__device__ void gemm_rr(int Np, LA la, LB lb, ST st) {
  const int lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int nt = Np >> 4, ntiles = nt * nt;
  for (int tile = wave; tile < ntiles; tile += NWAVE) {
    const int ti = tile % nt, tj = tile / nt;
    const int i = (ti << 4) + li, j = (tj << 4) + li;
    v4d c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < Np; k0 += 4) {
      const int k = k0 + lk;
      c = mfma4(la(i, k), lb(k, j), c);
    }
    const int r0 = (ti << 4) + lk, c0 = (tj << 4) + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) st(r0 + 4 * r, c0, c[r]);
  }
}

// real A x complex B -> complex C.  lb(k,j,br,bi); st(i,j,cr,ci)
template <class LA, class LB, class ST>
__device__ void gemm_rc(int Np, LA la, LB lb, ST st) {
  const int lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int nt = Np >> 4, ntiles = nt * nt;
  for (int tile = wave; tile < ntiles; tile += NWAVE) {
    const int ti = tile % nt, tj = tile / nt;
    const int i = (ti << 4) + li, j = (tj << 4) + li;
    v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < Np; k0 += 4) {
      const int k = k0 + lk;
      const double a = la(i, k);
      double br, bi;
      lb(k, j, br, bi);
      cr = mfma4(a, br, cr);
      ci = mfma4(a, bi, ci);
    }
    const int r0 = (ti << 4) + lk, c0 = (tj << 4) + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) st(r0 + 4 * r, c0, cr[r], ci[r]);
  }
}

// complex A x complex B -> complex C.  la(i,k,ar,ai); lb(k,j,br,bi)
template <class LA, class LB, class ST>
__device__ void gemm_cc(int Np, LA la, LB lb, ST st) {
  const int lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int nt = Np >> 4, ntiles = nt * nt;
  for (int tile = wave; tile < ntiles; tile += NWAVE) {
    const int ti = tile % nt, tj = tile / nt;
    const int i = (ti << 4) + li, j = (tj << 4) + li;
    v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int k0 = 0; k0 < Np; k0 += 4) {
      const int k = k0 + lk;
      double ar, ai, br, bi;
      la(i, k, ar, ai);
      lb(k, j, br, bi);
      cr = mfma4(ar, br, cr);
      cr = mfma4(-ai, bi, cr);
      ci = mfma4(ar, bi, ci);
      ci = mfma4(ai, br, ci);
    }
    const int r0 = (ti << 4) + lk, c0 = (tj << 4) + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) st(r0 + 4 * r, c0, cr[r], ci[r]);
  }
}

// complex A x real B -> complex C.  la(i,k,ar,ai); lb(k,j) -> double
template <class LA, class LB, class ST>
__device__ void gemm_cr(int Np, LA la, LB lb, ST st) {
  const int lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int nt = Np >> 4, ntiles = nt * nt;
  for (int tile = wave; tile < ntiles; tile += NWAVE) {
    const int ti = tile % nt, tj = tile / nt;
    const int i = (ti << 4) + li, j = (tj << 4) + li;
    v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < Np; k0 += 4) {
      const int k = k0 + lk;
      double ar, ai;
      la(i, k, ar, ai);
      const double b = lb(k, j);
      cr = mfma4(ar, b, cr);
      ci = mfma4(ai, b, ci);
    }
    const int r0 = (ti << 4) + lk, c0 = (tj << 4) + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) st(r0 + 4 * r, c0, cr[r], ci[r]);
  }
}

// ---------------------------------------------------------------------------
// Householder QR with column pivoting (Sec. 7: D sorted by magnitude).
//
// Reflector H = I - beta u u^H (Hermitian, unitary, det H = -1) maps the
// active column a to -e^{i arg a_0} |a| e_1; u = a + e^{i arg a_0} |a| e_1,
// beta = 1 / (|a| (|a| + |a_0|)).  A zero column gets no reflector
// (beta = 0, det 1).  nref counts the reflectors, so det Q = (-1)^nref.
//
// The pivot key of a column is its remaining norm times keys[column]
// (keys == nullptr: 1).  Householder QR treats every column independently of
// its scale, so this reproduces the pivoted QR of W diag(keys) exactly while
// all arithmetic stays on W; the caller applies diag(keys) to R afterwards.
// Partial norms are recomputed from the updated column each step (no
// downdating).  Ties go to the lowest position.
//
// Output: R in the upper triangle of W, reflector tails below it, S.u0r/u0i,
// S.beta, S.piv (original column at each position), S.csp (key at each
// position), S.nref.  Two workgroup barriers per column.
// ---------------------------------------------------------------------------
template <int MAXN>
__device__ void wg_qrp(CMat W, int N, const double* keys, Smem<MAXN>& S) {
  constexpr int MR = (MAXN + 63) / 64;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();

  for (int k = tid; k < N; k += WG) {
    S.piv[k] = k;
    S.csp[k] = keys ? keys[k] : 1.0;
  }
  {
    double bk = -1.0, bn = 0.0;
    int bi = -1;
    for (int k = wave; k < N; k += NWAVE) {
      double acc = 0.0;
      for (int i = lane; i < N; i += 64) {
        const double a = W.r(i, k), b = W.m(i, k);
        acc += a * a + b * b;
      }
      acc = sqrt(wave_sum(acc));
      const double key = acc * (keys ? keys[k] : 1.0);
      if (lane == 0) S.norms[k] = acc;
      if (key > bk) { bk = key; bn = acc; bi = k; }
    }
    if (lane == 0) { S.candk[wave] = bk; S.candn[wave] = bn; S.candi[wave] = bi; }
  }
  if (tid == 0) S.nref = 0;
  __syncthreads();

  for (int j = 0; j < N; ++j) {
    // ---- phase 1: choose the pivot, swap it into position j
    double bk = -1.0, alpha = 0.0;
    int p = j;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
      const int ci = S.candi[w];
      const double ck = S.candk[w];
      if (ci >= 0 && (ck > bk || (ck == bk && ci < p))) { bk = ck; p = ci; alpha = S.candn[w]; }
    }
    if (bk < 0.0) { p = j; alpha = S.norms[j]; }
    for (int i = tid; i < N; i += WG) {
      if (p != j) {
        const double xr = W.r(i, j), xi = W.m(i, j);
        const double yr = W.r(i, p), yi = W.m(i, p);
        W.r(i, j) = yr; W.m(i, j) = yi;
        W.r(i, p) = xr; W.m(i, p) = xi;
        if (i == j) { S.a0r = yr; S.a0i = yi; }
      } else if (i == j) {
        S.a0r = W.r(i, j); S.a0i = W.m(i, j);
      }
    }
    if (tid == 0 && p != j) {
      double t = S.norms[j]; S.norms[j] = S.norms[p]; S.norms[p] = t;
      t = S.csp[j]; S.csp[j] = S.csp[p]; S.csp[p] = t;
      int q = S.piv[j]; S.piv[j] = S.piv[p]; S.piv[p] = q;
    }
    __syncthreads();

    // ---- phase 2: reflector for column j, applied to the trailing columns
    const double a0r = S.a0r, a0i = S.a0i;
    const double aa0 = hypot(a0r, a0i);
    double er = 1.0, ei = 0.0;
    if (aa0 > 0.0) { er = a0r / aa0; ei = a0i / aa0; }
    const bool refl = alpha > 0.0;
    const double beta = refl ? 1.0 / (alpha * (alpha + aa0)) : 0.0;
    const double u0r = a0r + er * alpha, u0i = a0i + ei * alpha;

    double ur[MR], ui[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int i = j + lane + 64 * m;
      ur[m] = 0.0; ui[m] = 0.0;
      if (i < N) {
        if (i == j) { ur[m] = u0r; ui[m] = u0i; }
        else { ur[m] = W.r(i, j); ui[m] = W.m(i, j); }
      }
    }
    double wbk = -1.0, wbn = 0.0;
    int wbi = -1;
    for (int k = j + 1 + wave; k < N; k += NWAVE) {
      double ar[MR], ai[MR];
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int i = j + lane + 64 * m;
        ar[m] = 0.0; ai[m] = 0.0;
        if (i < N) { ar[m] = W.r(i, k); ai[m] = W.m(i, k); }
        sr += ur[m] * ar[m] + ui[m] * ai[m];
        si += ur[m] * ai[m] - ui[m] * ar[m];
      }
      double pn = 0.0;
      if (refl) {
        const double wr = beta * wave_sum(sr), wi = beta * wave_sum(si);
#pragma unroll
        for (int m = 0; m < MR; ++m) {
          const int i = j + lane + 64 * m;
          if (i < N) {
            ar[m] -= ur[m] * wr - ui[m] * wi;
            ai[m] -= ur[m] * wi + ui[m] * wr;
            W.r(i, k) = ar[m];
            W.m(i, k) = ai[m];
          }
        }
      }
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int i = j + lane + 64 * m;
        if (i > j && i < N) pn += ar[m] * ar[m] + ai[m] * ai[m];
      }
      pn = sqrt(wave_sum(pn));
      const double key = pn * S.csp[k];
      if (lane == 0) S.norms[k] = pn;
      if (key > wbk) { wbk = key; wbn = pn; wbi = k; }
    }
    if (lane == 0) { S.candk[wave] = wbk; S.candn[wave] = wbn; S.candi[wave] = wbi; }
    if (tid == 0) {
      W.r(j, j) = refl ? -er * alpha : 0.0;
      W.m(j, j) = refl ? -ei * alpha : 0.0;
      S.u0r[j] = refl ? u0r : 0.0;
      S.u0i[j] = refl ? u0i : 0.0;
      S.beta[j] = beta;
      if (refl) S.nref += 1;
    }
    __syncthreads();
  }
}

// Load the reflector u_j (rows j..N-1) into lane registers.
template <int MR>
__device__ __forceinline__ void load_reflector(CMat W, int N, int j, double u0r, double u0i,
                                               double* ur, double* ui) {
  const int lane = lane_id();
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int i = j + lane + 64 * m;
    ur[m] = 0.0; ui[m] = 0.0;
    if (i < N) {
      if (i == j) { ur[m] = u0r; ui[m] = u0i; }
      else { ur[m] = W.r(i, j); ui[m] = W.m(i, j); }
    }
  }
}

// Apply H = I - beta u u^H (rows j..N-1) to column c of Y, in place.
template <int MR>
__device__ __forceinline__ void apply_reflector_col(CMat Y, int N, int j, int c, double beta,
                                                    const double* ur, const double* ui) {
  const int lane = lane_id();
  double ar[MR], ai[MR];
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int i = j + lane + 64 * m;
    ar[m] = 0.0; ai[m] = 0.0;
    if (i < N) { ar[m] = Y.r(i, c); ai[m] = Y.m(i, c); }
    sr += ur[m] * ar[m] + ui[m] * ai[m];
    si += ur[m] * ai[m] - ui[m] * ar[m];
  }
  const double wr = beta * wave_sum(sr), wi = beta * wave_sum(si);
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int i = j + lane + 64 * m;
    if (i < N) {
      Y.r(i, c) = ar[m] - (ur[m] * wr - ui[m] * wi);
      Y.m(i, c) = ai[m] - (ur[m] * wi + ui[m] * wr);
    }
  }
}

// Q = H_0 H_1 ... H_{N-1} written explicitly into Q (backward accumulation).
template <int MAXN>
__device__ void wg_form_q(CMat W, int N, CMat Q, Smem<MAXN>& S) {
  constexpr int MR = (MAXN + 63) / 64;
  const int tid = threadIdx.x, wave = wave_id();
  for (int idx = tid; idx < N * N; idx += WG) {
    const int i = idx % N, c = idx / N;
    Q.r(i, c) = (i == c) ? 1.0 : 0.0;
    Q.m(i, c) = 0.0;
  }
  __syncthreads();
  for (int j = N - 1; j >= 0; --j) {
    const double beta = S.beta[j];
    if (beta != 0.0) {
      double ur[MR], ui[MR];
      load_reflector<MR>(W, N, j, S.u0r[j], S.u0i[j], ur, ui);
      for (int c = j + wave; c < N; c += NWAVE) apply_reflector_col<MR>(Q, N, j, c, beta, ur, ui);
    }
    __syncthreads();
  }
}

// Y <- Q^H Y = H_{N-1} ... H_0 Y.  Each wave owns whole columns of Y, so no
// barrier is needed inside; the caller synchronises before and after.
template <int MAXN>
__device__ void wg_apply_qh(CMat W, int N, CMat Y, Smem<MAXN>& S) {
  constexpr int MR = (MAXN + 63) / 64;
  const int wave = wave_id();
  for (int j = 0; j < N; ++j) {
    const double beta = S.beta[j];
    if (beta == 0.0) continue;
    double ur[MR], ui[MR];
    load_reflector<MR>(W, N, j, S.u0r[j], S.u0i[j], ur, ui);
    for (int c = wave; c < N; c += NWAVE) apply_reflector_col<MR>(Y, N, j, c, beta, ur, ui);
  }
}

// Y <- R^{-1} Y for the upper-triangular R stored in W (back substitution).
// Each wave owns whole columns of Y; rows are spread over the lanes.
template <int MAXN>
__device__ void wg_backsolve(CMat W, int N, CMat Y) {
  constexpr int MR = (MAXN + 63) / 64;
  const int lane = lane_id(), wave = wave_id();
  for (int c = wave; c < N; c += NWAVE) {
    double yr[MR], yi[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int i = lane + 64 * m;
      yr[m] = 0.0; yi[m] = 0.0;
      if (i < N) { yr[m] = Y.r(i, c); yi[m] = Y.m(i, c); }
    }
    for (int i = N - 1; i >= 0; --i) {
      const int mi = i >> 6, li = i & 63;
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int m = 0; m < MR; ++m) if (m == mi) { vr = yr[m]; vi = yi[m]; }
      vr = __shfl(vr, li, 64);
      vi = __shfl(vi, li, 64);
      const double dr = W.r(i, i), di = W.m(i, i);
      const double den = dr * dr + di * di;
      const double zr = (vr * dr + vi * di) / den;
      const double zi = (vi * dr - vr * di) / den;
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int k = lane + 64 * m;
        if (k < i) {
          const double rr = W.r(k, i), ri = W.m(k, i);
          yr[m] -= rr * zr - ri * zi;
          yi[m] -= rr * zi + ri * zr;
        } else if (k == i) {
          yr[m] = zr; yi[m] = zi;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int i = lane + 64 * m;
      if (i < N) { Y.r(i, c) = yr[m]; Y.m(i, c) = yi[m]; }
    }
  }
}

}  // namespace fdet

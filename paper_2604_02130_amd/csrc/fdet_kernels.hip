// gfx950 kernels for the stabilised fermion determinant.
//
// One workgroup executes one work item (see fdet_plan.h):
//   IK_EXPM     E = exp(+-dk K) by a scaled Taylor polynomial and squaring
//               (Sec. 8 notes a truncated polynomial may stand for the
//               exponential; Sec. 6 diagonalises instead).
//   IK_CHAIN    product of a range of slices B_t = E diag(e^{i phi_t}) as
//               X diag(D) T (eq. def_matrix_as_product), re-decomposed by a
//               pivoted QR every s slices (Sec. 7 steps 2-3, Sec. 9).
//   IK_COMBINE  stabilised product of two UDV triples
//               (eqs. prod_2_mat_stab .. res_2_mat_stab).
//   IK_CLOSE    log det(1 + X D T) and (1 + X D T)^{-1} (Sec. 7 steps 4-6).
//   IK_FORCE    G~ at a checkpoint from the two stabilised factors of its
//               cyclic product (Sec. 5, stabilised pre- and suffix
//               products), then G~_{t+1} = B_t G~_t B_t^{-1} across the
//               checkpoint interval; F_{t,x} = i (1 - G~_t)_{xx}.
//   IK_EXPORT   copy a UDV triple out in the caller's layout.
#include "fdet_device.hpp"
#include "fdet_plan.h"
#include "fdet_regqr.hpp"
#include "fdet_large.hpp"

namespace fdet {

constexpr double kPi = 3.14159265358979323846;

// 1 / k!, k = 0..16 (each quotient rounded once at compile time)
__constant__ double kInvFact[17] = {
    1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
    1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
    1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0};

// Size classes: N <= NC.  Classes up to 128 keep the matrix being factorised
// in registers and stage products through LDS (fdet_regqr.hpp); the 512
// class works on device memory with blocked, MFMA-based factorisations
// (fdet_large.hpp).  F is a free complex matrix and tst the per-item store of
// the panels' T factors, both used by the 512 class only.
template <int NC>
__device__ __forceinline__ void qr_factor(CMat W, int N, const double* keys, CMat F, double* tst,
                                          SmemC<NC>& S) {
  if constexpr (NC <= 128) rq_qrp<NC>(W, N, keys, S);
  else lg_qrp<NC>(W, N, keys, F, tst, S);
}

template <int NC>
__device__ __forceinline__ void qr_form_q(CMat W, int N, CMat Q, CMat F, const double* tst,
                                          SmemC<NC>& S) {
  if constexpr (NC <= 128) rq_form_q<NC>(N, Q, S);
  else lg_form_q<NC>(W, N, Q, F, tst, S);
  __syncthreads();
}

// C = A B with A, B real or complex (AC, BC)
template <int NC, bool AC, bool BC, class LA, class LB, class ST>
__device__ __forceinline__ void mm(int Np, LA la, LB lb, ST st, SmemC<NC>& S) {
  if constexpr (NC <= 128) gemm_lds<NC, AC, BC>(Np, la, lb, st, S.big);
  else lg_gemm<128, 128, AC, BC>(Np, Np, Np, la, lb, st, S.big);
}

// Y <- R^{-1} Q^H Y for the factor in W
template <int NC>
__device__ __forceinline__ void qr_solve(CMat W, int N, CMat Y, CMat F, const double* tst,
                                         SmemC<NC>& S) {
  if constexpr (NC <= 128) {
    rq_solve<NC>(W, N, Y, S);
  } else {
    lg_apply_qh<NC>(W, N, Y, F, tst, S);
    __syncthreads();
    lg_backsolve<NC>(W, N, Y, S);
  }
  __syncthreads();
}

// per-item store of T factors: after the 4 matrices and 2 Np doubles of the
// item's scratch
__device__ __forceinline__ double* tstore(double* scr, int Np) {
  return scr + 4 * cmat_doubles(Np) + 2 * (size_t)Np;
}

__device__ void status_merge(int32_t* st, int32_t code) {
  if (code == 0 || st == nullptr) return;
  int32_t old = *((volatile int32_t*)st);
  while (true) {
    int32_t worse = (old < 0 || code < 0) ? (old < code ? old : code) : (old > code ? old : code);
    if (worse == old) return;
    int32_t prev = atomicCAS(st, old, worse);
    if (prev == old) return;
    old = prev;
  }
}

template <int NC>
__device__ void load_phases(const Prob& P, int t, SmemC<NC>& S) {
  const int row = t % P.Nt;   // chains of the displaced Green's function wrap around
  for (int x = threadIdx.x; x < P.N; x += WG) {
    double sv, cv;
    sincos(P.phi[(size_t)row * P.N + x], &sv, &cv);
    S.phr[x] = cv;
    S.phi_[x] = sv;
  }
}

__device__ void set_identity(CMat A, int N) {
  for_each_ij(N, [&](int i, int j) {
    A.r(i, j) = (i == j) ? 1.0 : 0.0;
    A.m(i, j) = 0.0;
  });
}

__device__ void copy_cmat(CMat dst, CMat src, int N) {
  for_each_ij(N, [&](int i, int j) {
    dst.r(i, j) = src.r(i, j);
    dst.m(i, j) = src.m(i, j);
  });
}

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) t += red[w];
  __syncthreads();
  return t;
}

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int w = 1; w < NWAVE; ++w) t = fmax(t, red[w]);
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// slice products
// ---------------------------------------------------------------------------

// One slice of the chain: out = B_t in = E diag(e^{i phi_t}) in, one real x
// complex product with the phases applied while the operand is staged (E is
// exp(dk K), or exp(-dk K) for the chains of B_t^{-H}).
template <int NC>
__device__ void slice_apply(const Prob& P, const double* E, CMat in, CMat out, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  mm<NC, false, true>(
      Np, [&](int i, int k) { return (i < N && k < N) ? E[(size_t)k * Np + i] : 0.0; },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) {
          const double xr = in.r(k, j), xi = in.m(k, j);
          const double c = S.phr[k], s = S.phi_[k];
          br = c * xr - s * xi;
          bi = s * xr + c * xi;
        } else {
          br = 0.0; bi = 0.0;
        }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) { out.r(i, j) = cr; out.m(i, j) = ci; }
      }, S);
}

// After the pivoted QR of W with keys: D_new (S.v2) = |R_ii| keys_i and the row scale
// S.v3 = 1 / D_new used to build T' = D_new^{-1} R diag(keys) (unit-modulus
// diagonal).  Returns nothing; flags a zero or non-finite scale in S.flag.
template <int NC>
__device__ void udv_scales(CMat W, int N, SmemC<NC>& S) {
  for (int i = threadIdx.x; i < N; i += WG) {
    const double a = hypot(W.r(i, i), W.m(i, i));
    const double d = a * S.csp[i];
    S.v2[i] = d;
    S.v3[i] = (d > 0.0 && isfinite(d)) ? 1.0 / d : 0.0;
    if (!(d > 0.0) || !isfinite(d)) S.flag = 1;
  }
}

// To = T' Pi^T T2op with T'(i,k) = R(i,k) keys_k / D_new_i for k >= i.
template <int NC, class LT2>
__device__ void udv_new_t(CMat W, int N, int Np, LT2 t2, CMat To, SmemC<NC>& S) {
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N && k >= i) {
          const double sc = S.csp[k] * S.v3[i];
          ar = W.r(i, k) * sc;
          ai = W.m(i, k) * sc;
        } else {
          ar = 0.0; ai = 0.0;
        }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) t2(S.piv[k], j, br, bi);
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) { To.r(i, j) = cr; To.m(i, j) = ci; }
      }, S);
}

// ---------------------------------------------------------------------------
// IK_CHAIN
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_chain(const Prob& P, const Item& it, SmemC<NC>& S);

template <int NC>
__device__ __forceinline__ void do_close(const Prob& P, Udv U, CMat W, CMat Yb, CMat Gint, bool want_g,
                         bool user_out, bool ld_out, double* tst, SmemC<NC>& S);

// The ns slices of a chunk without forming B~_t (Sec. 8 product form, used
// by the sporadic stabilisation of Sec. 9): W = prod over the chunk of
// [prod_k (1 + gamma_k dk K)] diag(e^{i phi_t}) applied to X.  Columns are
// independent, so X goes through LDS in panels of w columns (w a power of
// two, four N x w planes: two buffers, re and im): each panel gets all ns
// slices there, i.e. ns (n + 1) passes of N w elements, each step
// x_i <- x_i + gamma_k dk sum_j K_{i,col_ij} x_{col_ij} a stencil over the
// row's q nonzeros, then it is written to W.  The field phases of the chunk
// are computed once into Ph (re: cos, im: sin, slice-major; ns N <= Np^2).
template <int NC>
__device__ void sparse_slices(const Prob& P, CMat X, CMat W, CMat Ph, int tfirst, int ns,
                              SmemC<NC>& S) {
  const int N = P.N, q = P.sp->q, n = P.sp->n;
  const int32_t* __restrict__ col = P.sp->col;
  const double* __restrict__ val = P.sp->val;
  for (int e = threadIdx.x; e < ns * N; e += WG) {
    const int k = e / N, i = e - k * N;
    const int row = (tfirst + k) % P.Nt;
    double sv, cv;
    sincos(P.phi[(size_t)row * N + i], &sv, &cv);
    Ph.re[e] = cv;
    Ph.im[e] = sv;
  }
  constexpr int LD = NC <= 128 ? BigLds<NC>::N : LG_BIG;
  int lw = 0;
  while ((2 << lw) * 4 * N <= LD && (2 << lw) <= N) ++lw;
  const int w = 1 << lw, ne = N * w;
  double* ar = S.big;
  double* ai = ar + ne;
  double* br = ai + ne;
  double* bi = br + ne;
  __syncthreads();
  for (int c0 = 0; c0 < N; c0 += w) {
    const int wc = min(w, N - c0);
    for (int e = threadIdx.x; e < ne; e += WG) {
      const int i = e >> lw, c = e & (w - 1);
      ar[e] = c < wc ? X.r(i, c0 + c) : 0.0;
      ai[e] = c < wc ? X.m(i, c0 + c) : 0.0;
    }
    __syncthreads();
    double *xr = ar, *xi = ai, *yr = br, *yi = bi;
    for (int k = 0; k < ns; ++k) {
      for (int e = threadIdx.x; e < ne; e += WG) {
        const int i = e >> lw;
        const double cv = Ph.re[k * N + i], sv = Ph.im[k * N + i];
        const double r = xr[e], m = xi[e];
        xr[e] = cv * r - sv * m;
        xi[e] = sv * r + cv * m;
      }
      __syncthreads();
      for (int f = 0; f < n; ++f) {
        const double gr = P.sp->gr[f], gi = P.sp->gi[f];
        for (int e = threadIdx.x; e < ne; e += WG) {
          const int i = e >> lw, c = e & (w - 1);
          double sr = 0.0, si = 0.0;
          for (int j = 0; j < q; ++j) {
            const double v = val[(size_t)i * q + j];
            const int cj = min(max(col[(size_t)i * q + j], 0), N - 1);
            sr = fma(v, xr[(cj << lw) + c], sr);
            si = fma(v, xi[(cj << lw) + c], si);
          }
          yr[e] = xr[e] + (gr * sr - gi * si);
          yi[e] = xi[e] + (gr * si + gi * sr);
        }
        __syncthreads();
        double* t = xr; xr = yr; yr = t;
        t = xi; xi = yi; yi = t;
      }
    }
    for (int e = threadIdx.x; e < ne; e += WG) {
      const int i = e >> lw, c = e & (w - 1);
      if (c < wc) {
        W.r(i, c0 + c) = xr[e];
        W.m(i, c0 + c) = xi[e];
      }
    }
    __syncthreads();
  }
}

template <int NC>
__device__ void chain_chunk(const Prob& P, const Item& it, CMat X, CMat& Tc, CMat& Tt, double* D,
                            CMat W, CMat Y2, int tfirst, int ns, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  if (P.sp) {
    sparse_slices<NC>(P, X, W, Y2, tfirst, ns, S);
  } else {
    CMat src = X;
    CMat dst = (ns & 1) ? W : Y2;
    for (int q = 0; q < ns; ++q) {
      load_phases<NC>(P, tfirst + q, S);
      __syncthreads();
      slice_apply<NC>(P, (it.flags & IF_EINV) ? P.Einv : P.E, src, dst, S);
      __syncthreads();
      src = dst;
      dst = (dst.re == W.re) ? Y2 : W;
    }
  }
  double* tst = tstore(it.scr, Np);
  qr_factor<NC>(W, N, D, Y2, tst, S);
  udv_scales<NC>(W, N, S);
  __syncthreads();
  qr_form_q<NC>(W, N, X, Y2, tst, S);
  udv_new_t<NC>(W, N, Np,
                  [&](int r, int j, double& br, double& bi) { br = Tc.r(r, j); bi = Tc.m(r, j); },
                  Tt, S);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += WG) D[i] = S.v2[i];
  CMat tmp = Tc; Tc = Tt; Tt = tmp;
  __syncthreads();
}

template <int NC>
__device__ __forceinline__ void do_chain(const Prob& P, const Item& it, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  const size_t cd = cmat_doubles(Np);
  CMat X = cmat_at(it.a.X, Np), T = cmat_at(it.a.T, Np);
  double* D = it.a.D;
  CMat W = cmat_at(it.scr, Np), Y2 = cmat_at(it.scr + cd, Np), Tn = cmat_at(it.scr + 2 * cd, Np);
  if (threadIdx.x == 0) S.flag = 0;
  if (it.flags & IF_IDENTITY) {
    set_identity(X, N);
    set_identity(T, N);
    for (int i = threadIdx.x; i < N; i += WG) D[i] = 1.0;
  }
  __syncthreads();
  CMat Tc = T, Tt = Tn;
  const int s = it.s;
  // chunks of at most s slices upward from t0
  for (int tfirst = it.t0; tfirst < it.t1; tfirst += s)
    chain_chunk<NC>(P, it, X, Tc, Tt, D, W, Y2, tfirst, min(s, it.t1 - tfirst), S);
  if (Tc.re != T.re) {
    copy_cmat(T, Tc, N);
    __syncthreads();
  }
  if (threadIdx.x == 0 && S.flag) status_merge(P.status, -4);
}

// ---------------------------------------------------------------------------
// IK_COMBINE and the shared stabilised product
// result = A1 A2 with A1 = (X1, D1, T1) and A2 = (X2, D2, T2): the bracket
// D1 (T1 X2) D2 keeps a unitary factor in the middle product.
// ---------------------------------------------------------------------------
template <int NC, bool RIGHT_Q = false>
__device__ void combine_core(const Prob& P, Udv A1, Udv A2, CMat W, CMat Qb, CMat Xo, CMat To,
                             double* Do, double* tst, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  CMat X1 = cmat_at(A1.X, Np), T1 = cmat_at(A1.T, Np);
  CMat X2 = cmat_at(A2.X, Np), T2 = cmat_at(A2.T, Np);
  const double* D1 = A1.D;
  for (int i = threadIdx.x; i < N; i += WG) S.v1[i] = D1[i];
  __syncthreads();
  // bracket D1 (T1 X2): its column scale D2 is left to the pivoted QR keys
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = T1.r(i, k); ai = T1.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { br = X2.r(k, j); bi = X2.m(k, j); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) { W.r(i, j) = S.v1[i] * cr; W.m(i, j) = S.v1[i] * ci; }
      }, S);
  __syncthreads();
  // To is written last, so it serves as the free matrix until then
  qr_factor<NC>(W, N, A2.D, To, tst, S);
  udv_scales<NC>(W, N, S);
  __syncthreads();
  if constexpr (NC > 128 && RIGHT_Q) {
    if (lg_block_fits(Np)) {
      // X = X1 Q by applying the reflector blocks to a copy of X1 from the
      // right (Q is never formed; Qb is the free matrix)
      copy_cmat(Xo, X1, N);
      __syncthreads();
      lg_right_apply_q<NC>(W, N, Xo, N, Qb, S);
      __syncthreads();
      udv_new_t<NC>(W, N, Np,
                    [&](int r, int j, double& br, double& bi) { br = T2.r(r, j); bi = T2.m(r, j); },
                    To, S);
      __syncthreads();
      for (int i = threadIdx.x; i < N; i += WG) Do[i] = S.v2[i];
      __syncthreads();
      return;
    }
  }
  qr_form_q<NC>(W, N, Qb, To, tst, S);
  // X = X1 Q
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = X1.r(i, k); ai = X1.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { br = Qb.r(k, j); bi = Qb.m(k, j); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) { Xo.r(i, j) = cr; Xo.m(i, j) = ci; }
      }, S);
  // T = T' Pi^T T2
  udv_new_t<NC>(W, N, Np,
                  [&](int r, int j, double& br, double& bi) { br = T2.r(r, j); bi = T2.m(r, j); },
                  To, S);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += WG) Do[i] = S.v2[i];
  __syncthreads();
}

template <int NC>
__device__ __forceinline__ void do_combine(const Prob& P, const Item& it, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  const size_t cd = cmat_doubles(Np);
  CMat W = cmat_at(it.scr, Np), Qb = cmat_at(it.scr + cd, Np);
  CMat Xs = cmat_at(it.scr + 2 * cd, Np), Ts = cmat_at(it.scr + 3 * cd, Np);
  double* Ds = it.scr + 4 * cd;
  if (threadIdx.x == 0) S.flag = 0;
  // Left factor b (the later slices), right factor a; result into o, or a.
  // combine_core reads X_b until the last-but-one product, T_a in the last,
  // and X_a, T_b and the scales only before its QR: a result slot that is
  // neither operand is written directly, one that is an operand takes the
  // parts that operand no longer needs, and the rest goes through scratch.
  const Udv& R = it.o.X ? it.o : it.a;
  const bool is_a = R.X == it.a.X, is_b = R.X == it.b.X;
  CMat Xo = is_b ? Xs : cmat_at(R.X, Np);
  CMat To = is_a ? Ts : cmat_at(R.T, Np);
  double* Do = R.D;
  combine_core<NC, true>(P, it.b, it.a, W, Qb, Xo, To, Do, tstore(it.scr, Np), S);
  if (is_b) copy_cmat(cmat_at(R.X, Np), Xs, N);
  if (is_a) copy_cmat(cmat_at(R.T, Np), Ts, N);
  if (threadIdx.x == 0 && S.flag) status_merge(P.status, -4);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// IK_CLOSE: log det(1 + X D T) and G = (1 + X D T)^{-1}.
// With D_b = max(D, 1) and D_s = min(D, 1):
//   1 + X D T = X (1 + D T X) X^H = X D_b A X^H,  A = D_b^{-1} + D_s T X,
// A has O(1) rows, and its pivoted QR A Pi = Q R gives
//   log det = sum log R_ii + sum log D_b + i pi (nref + parity(Pi)),
//   G = X Pi R^{-1} Q^H D_b^{-1} X^H.
// This is Sec. 7 steps 4-6 with the rows of 1 + D T X divided by D_b first.
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_close(const Prob& P, Udv U, CMat W, CMat Yb, CMat Gint, bool want_g,
                         bool user_out, bool ld_out, double* tst, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  CMat X = cmat_at(U.X, Np), T = cmat_at(U.T, Np);
  bool bad = false;
  for (int i = threadIdx.x; i < N; i += WG) {
    const double d = U.D[i];
    if (!isfinite(d)) bad = true;
    S.v1[i] = d > 1.0 ? d : 1.0;
    S.v2[i] = d < 1.0 ? d : 1.0;
  }
  __syncthreads();
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = T.r(i, k); ai = T.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { br = X.r(k, j); bi = X.m(k, j); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) {
          W.r(i, j) = S.v2[i] * cr + (i == j ? 1.0 / S.v1[i] : 0.0);
          W.m(i, j) = S.v2[i] * ci;
        }
      }, S);
  __syncthreads();
  // T of the UDV is not read again: it serves as the free matrix
  qr_factor<NC>(W, N, nullptr, T, tst, S);
  // log det
  double lr = 0.0, li = 0.0, amin = INFINITY, amax = 0.0;
  for (int i = threadIdx.x; i < N; i += WG) {
    const double rr = W.r(i, i), ri = W.m(i, i);
    const double a = hypot(rr, ri);
    lr += log(a) + log(S.v1[i]);
    li += atan2(ri, rr);
    amin = fmin(amin, a);
    amax = fmax(amax, a);
    if (!isfinite(a)) bad = true;
  }
  lr = block_sum(lr, S.red);
  li = block_sum(li, S.red);
  amax = block_max(amax, S.red);
  amin = -block_max(-amin, S.red);
  const double nbad = block_sum(bad ? 1.0 : 0.0, S.red);
  if (threadIdx.x == 0) {
    // parity of the pivot permutation by cycle counting
    int par = 0;
    for (int i = 0; i < N; ++i) S.pinv[i] = 0;
    for (int i = 0; i < N; ++i) {
      if (S.pinv[i]) continue;
      int j = i, len = 0;
      while (!S.pinv[j]) { S.pinv[j] = 1; j = S.piv[j]; ++len; }
      par ^= (len - 1) & 1;
    }
    double im = li + kPi * (double)((S.nref + par) & 1);
    im = remainder(im, 2.0 * kPi);
    if (im <= -kPi) im += 2.0 * kPi;
    if (ld_out && P.logdet) { P.logdet[0] = lr; P.logdet[1] = im; }
    int32_t code = 0;
    if (nbad > 0.0) code = -4;
    else if (!(amin > 0.0)) code = -3;
    else if (amin < 1e3 * N * 2.220446049250313e-16 * fmax(1.0, amax)) code = 1;
    status_merge(P.status, code);
  }
  __syncthreads();
  if (!want_g) return;
  // Yb = D_b^{-1} X^H
  for_each_ij(N, [&](int i, int j) {
    const double sc = 1.0 / S.v1[i];
    Yb.r(i, j) = X.r(j, i) * sc;
    Yb.m(i, j) = -X.m(j, i) * sc;
  });
  for (int r = threadIdx.x; r < N; r += WG) S.pinv[S.piv[r]] = r;
  __syncthreads();
  qr_solve<NC>(W, N, Yb, T, tst, S);
  // G = X Pi Z: row a of (Pi Z) is row pinv[a] of Z
  double* Gu = P.G;
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = X.r(i, k); ai = X.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { const int r = S.pinv[k]; br = Yb.r(r, j); bi = Yb.m(r, j); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) {
          if (user_out) {
            Gu[2 * ((size_t)i * N + j)] = cr;
            Gu[2 * ((size_t)i * N + j) + 1] = ci;
          } else {
            Gint.r(i, j) = cr;
            Gint.m(i, j) = ci;
          }
        }
      }, S);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// IK_FORCE
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_force(const Prob& P, const Item& it, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  const size_t cd = cmat_doubles(Np);
  CMat W = cmat_at(it.scr, Np), Qb = cmat_at(it.scr + cd, Np);
  CMat Xc = cmat_at(it.scr + 2 * cd, Np), Tc = cmat_at(it.scr + 3 * cd, Np);
  double* Dc = it.scr + 4 * cd;
  if (threadIdx.x == 0) S.flag = 0;
  // G~ at the checkpoint row: (1 + C)^{-1} for its cyclic product C = a b
  combine_core<NC>(P, it.a, it.b, W, Qb, Xc, Tc, Dc, tstore(it.scr, Np), S);
  Udv U;
  U.X = Xc.re; U.T = Tc.re; U.D = Dc;
  do_close<NC>(P, U, W, Qb, W, true, false, (it.flags & IF_OUT_LOGDET) != 0, tstore(it.scr, Np), S);
  // the checkpoint at row 0 holds G~_1 = G = M^{-1} itself (and C_0 = M - 1:
  // the close above gave log det M)
  if ((it.flags & IF_OUT_G) && P.G) {
    for (int idx = threadIdx.x; idx < N * N; idx += WG) {
      const int i = idx / N, j = idx % N;
      P.G[2 * (size_t)idx] = W.r(i, j);
      P.G[2 * (size_t)idx + 1] = W.m(i, j);
    }
  }
  // keep G~ of the checkpoint for the backward direction
  if (it.nb > 0) copy_cmat(Tc, W, N);
  const double* E = P.E;
  const double* Ei = P.Einv;
  auto write_row = [&](CMat G, int t) {
    for (int x = threadIdx.x; x < N; x += WG) {
      P.force[(size_t)t * N + x] = G.m(x, x);
      if (P.force_im) P.force_im[(size_t)t * N + x] = 1.0 - G.r(x, x);
    }
    // (register and LDS classes only: the host rejects the operator trace
    // for N > 128)
    if constexpr (NC <= 128) if (P.op_trace) {
      // tr((1 - G) A) = sum over (x, y) of (delta_xy - G_xy) A_yx; x runs
      // fastest so that both G (column-major) and A (row-major) are read
      // contiguously
      double sr = 0.0, si = 0.0;
      for (int idx = threadIdx.x; idx < N * N; idx += WG) {
        const int y = idx / N, x = idx - y * N;
        const double gr = (x == y ? 1.0 : 0.0) - G.r(x, y), gi = -G.m(x, y);
        const double ar = P.op[2 * (size_t)idx], ai = P.op[2 * (size_t)idx + 1];
        sr += gr * ar - gi * ai;
        si += gr * ai + gi * ar;
      }
      sr = block_sum(sr, S.red);
      si = block_sum(si, S.red);
      if (threadIdx.x == 0) {
        P.op_trace[2 * (size_t)t] = sr;
        P.op_trace[2 * (size_t)t + 1] = si;
      }
    }
  };
  // forward: G~ of row t+1 = B_t G~ B_t^{-1}, B_t = E diag(e^{i phi_t})
  CMat G = W, Y = Qb;
  for (int t = it.t0; t < it.t1; ++t) {
    write_row(G, t);
    if (t + 1 >= it.t1) break;
    load_phases<NC>(P, t, S);
    __syncthreads();
    // Y = E diag(e^{i phi}) G diag(e^{-i phi})
    mm<NC, false, true>(
        Np, [&](int i, int k) { return (i < N && k < N) ? E[(size_t)k * Np + i] : 0.0; },
        [&](int k, int j, double& br, double& bi) {
          if (k < N && j < N) {
            const double gr = G.r(k, j), gi = G.m(k, j);
            // e^{i(phi_k - phi_j)}
            const double c = S.phr[k] * S.phr[j] + S.phi_[k] * S.phi_[j];
            const double s = S.phi_[k] * S.phr[j] - S.phr[k] * S.phi_[j];
            br = c * gr - s * gi;
            bi = s * gr + c * gi;
          } else {
            br = 0.0; bi = 0.0;
          }
        },
        [&](int i, int j, double cr, double ci) {
          if (i < N && j < N) { Y.r(i, j) = cr; Y.m(i, j) = ci; }
        }, S);
    __syncthreads();
    // G = Y E^{-1}
    mm<NC, true, false>(
        Np,
        [&](int i, int k, double& ar, double& ai) {
          if (i < N && k < N) { ar = Y.r(i, k); ai = Y.m(i, k); }
          else { ar = 0.0; ai = 0.0; }
        },
        [&](int k, int j) { return (k < N && j < N) ? Ei[(size_t)j * Np + k] : 0.0; },
        [&](int i, int j, double cr, double ci) {
          if (i < N && j < N) { G.r(i, j) = cr; G.m(i, j) = ci; }
        }, S);
    __syncthreads();
  }
  // backward: G~ of row t = B_t^{-1} G~ of row t+1 B_t (rows mod N_t)
  G = Tc;
  Y = Xc;
  for (int b = 1; b <= it.nb; ++b) {
    int t = it.t0 - b;
    if (t < 0) t += P.Nt;
    load_phases<NC>(P, t, S);
    __syncthreads();
    // Y = E^{-1} G
    mm<NC, false, true>(
        Np, [&](int i, int k) { return (i < N && k < N) ? Ei[(size_t)k * Np + i] : 0.0; },
        [&](int k, int j, double& br, double& bi) {
          if (k < N && j < N) { br = G.r(k, j); bi = G.m(k, j); }
          else { br = 0.0; bi = 0.0; }
        },
        [&](int i, int j, double cr, double ci) {
          if (i < N && j < N) { Y.r(i, j) = cr; Y.m(i, j) = ci; }
        }, S);
    __syncthreads();
    // G = diag(e^{-i phi}) (Y E) diag(e^{i phi})
    mm<NC, true, false>(
        Np,
        [&](int i, int k, double& ar, double& ai) {
          if (i < N && k < N) { ar = Y.r(i, k); ai = Y.m(i, k); }
          else { ar = 0.0; ai = 0.0; }
        },
        [&](int k, int j) { return (k < N && j < N) ? E[(size_t)j * Np + k] : 0.0; },
        [&](int i, int j, double cr, double ci) {
          if (i < N && j < N) {
            // e^{i(phi_j - phi_i)}
            const double c = S.phr[j] * S.phr[i] + S.phi_[j] * S.phi_[i];
            const double s = S.phi_[j] * S.phr[i] - S.phr[j] * S.phi_[i];
            G.r(i, j) = c * cr - s * ci;
            G.m(i, j) = s * cr + c * ci;
          }
        }, S);
    __syncthreads();
    write_row(G, t);
  }
  if (threadIdx.x == 0 && S.flag) status_merge(P.status, -4);
}

// ---------------------------------------------------------------------------
// IK_DISPLACED: G(t, t0) = sign (P + Q^{-1})^{-1} (eq.
// sausage_all_in_denominator; Sec. 7 steps 7-9) with P = Xp Dp Tp (slot a)
// and Q^{-H} = Xq Dq Tq (slot b, the chain of exp(-dk K) diag(e^{i phi_t})),
// so that Q^{-1} = Tq^H Dq Xq^H and
//   P + Q^{-1} = Xp [Dp (Tp Xq) + (Xp^H Tq^H) Dq] Xq^H.
// With Dp = Dp_b Dp_s and Dq = Dq_s Dq_b (big / small parts, each at most 1
// on one side) the bracket is Dp_b W Dq_b with
//   W = Dp_s (Tp Xq) Dq_b^{-1} + Dp_b^{-1} (Xp^H Tq^H) Dq_s,
// whose entries are O(1); one pivoted QR of W then gives
//   G(t, t0) = sign Xq Dq_b^{-1} Pi R^{-1} Q^H Dp_b^{-1} Xp^H.
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_displaced(const Prob& P, const Item& it, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  const size_t cd = cmat_doubles(Np);
  CMat W = cmat_at(it.scr, Np), Yb = cmat_at(it.scr + cd, Np), F = cmat_at(it.scr + 2 * cd, Np);
  CMat Xp = cmat_at(it.a.X, Np), Tp = cmat_at(it.a.T, Np);
  CMat Xq = cmat_at(it.b.X, Np), Tq = cmat_at(it.b.T, Np);
  double* tst = tstore(it.scr, Np);
  bool bad = false;
  // v1 = 1 / Dp_b (kept through the QR, as in the close), v2 = Dp_s,
  // v3 = 1 / Dq_b, norms = Dq_s (both only before the QR)
  for (int i = threadIdx.x; i < N; i += WG) {
    const double dp = it.a.D[i], dq = it.b.D[i];
    if (!isfinite(dp) || !isfinite(dq)) bad = true;
    S.v1[i] = 1.0 / (dp > 1.0 ? dp : 1.0);
    S.v2[i] = dp < 1.0 ? dp : 1.0;
    S.v3[i] = 1.0 / (dq > 1.0 ? dq : 1.0);
    S.norms[i] = dq < 1.0 ? dq : 1.0;
  }
  __syncthreads();
  // W = Dp_s (Tp Xq) Dq_b^{-1}
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = Tp.r(i, k); ai = Tp.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { br = Xq.r(k, j); bi = Xq.m(k, j); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) {
          const double sc = S.v2[i] * S.v3[j];
          W.r(i, j) = sc * cr;
          W.m(i, j) = sc * ci;
        }
      }, S);
  __syncthreads();
  // W += Dp_b^{-1} (Xp^H Tq^H) Dq_s
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = Xp.r(k, i); ai = -Xp.m(k, i); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) { br = Tq.r(j, k); bi = -Tq.m(j, k); }
        else { br = 0.0; bi = 0.0; }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) {
          const double sc = S.v1[i] * S.norms[j];
          W.r(i, j) += sc * cr;
          W.m(i, j) += sc * ci;
        }
      }, S);
  __syncthreads();
  qr_factor<NC>(W, N, nullptr, F, tst, S);
  double amin = INFINITY, amax = 0.0;
  for (int i = threadIdx.x; i < N; i += WG) {
    const double a = hypot(W.r(i, i), W.m(i, i));
    if (!isfinite(a)) bad = true;
    amin = fmin(amin, a);
    amax = fmax(amax, a);
  }
  amax = block_max(amax, S.red);
  amin = -block_max(-amin, S.red);
  const double nbad = block_sum(bad ? 1.0 : 0.0, S.red);
  if (threadIdx.x == 0) {
    int32_t code = 0;
    if (nbad > 0.0) code = -4;
    else if (!(amin > 0.0)) code = -3;
    else if (amin < 1e3 * N * 2.220446049250313e-16 * fmax(1.0, amax)) code = 1;
    status_merge(P.status, code);
  }
  // Yb = Dp_b^{-1} Xp^H
  for_each_ij(N, [&](int i, int j) {
    const double sc = S.v1[i];
    Yb.r(i, j) = Xp.r(j, i) * sc;
    Yb.m(i, j) = -Xp.m(j, i) * sc;
  });
  for (int r = threadIdx.x; r < N; r += WG) S.pinv[S.piv[r]] = r;
  __syncthreads();
  qr_solve<NC>(W, N, Yb, F, tst, S);
  // G = sign Xq Dq_b^{-1} Pi Z: row a of Pi Z is row pinv[a] of Z
  double* Gu = it.out;
  const double sg = (double)it.sign;
  mm<NC, true, true>(
      Np,
      [&](int i, int k, double& ar, double& ai) {
        if (i < N && k < N) { ar = Xq.r(i, k); ai = Xq.m(i, k); }
        else { ar = 0.0; ai = 0.0; }
      },
      [&](int k, int j, double& br, double& bi) {
        if (k < N && j < N) {
          // Dq_b^{-1} from the slot (the QR reused S.v3 for its pivot keys)
          const int r = S.pinv[k];
          const double dq = it.b.D[k];
          const double sc = 1.0 / (dq > 1.0 ? dq : 1.0);
          br = Yb.r(r, j) * sc;
          bi = Yb.m(r, j) * sc;
        } else {
          br = 0.0; bi = 0.0;
        }
      },
      [&](int i, int j, double cr, double ci) {
        if (i < N && j < N) {
          Gu[2 * ((size_t)i * N + j)] = sg * cr;
          Gu[2 * ((size_t)i * N + j) + 1] = sg * ci;
        }
      }, S);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// IK_EXPM: exp(sign dk K) = (Taylor_16(A / 2^q))^(2^q), A = sign dk K,
// q chosen so that |A / 2^q|_1 <= 1/2 (truncation below 1e-19).
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_expm(const Prob& P, const Item& it, SmemC<NC>& S) {
  const int N = P.N, Np = P.Np;
  const double* K = P.K;
  double* out = (it.sign > 0) ? P.E : P.Einv;
  // 1-norm of dk K
  double cm = 0.0;
  for (int j = threadIdx.x; j < N; j += WG) {
    double acc = 0.0;
    for (int i = 0; i < N; ++i) acc += fabs(K[(size_t)i * N + j]);
    cm = fmax(cm, acc);
  }
  const double nrm = fabs(P.dk) * block_max(cm, S.red);
  int q = 0;
  double scaled = nrm;
  while (scaled > 0.5 && q < 1000) { scaled *= 0.5; ++q; }
  const double a = (double)it.sign * P.dk * ldexp(1.0, -q);
  // Degree-16 Taylor polynomial of A = a K by Paterson-Stockmeyer with block
  // 4: A^2, A^3, A^4, then Horner in A^4 over C_j = sum_i A^i / (4j + i)!,
  // i = 0..3 (C_4 = I / 16!): six products instead of sixteen.
  const size_t n2 = (size_t)Np * Np;
  double* Ab = it.scr;
  double* A2 = Ab + n2;
  double* A3 = Ab + 2 * n2;
  double* A4 = Ab + 3 * n2;
  double* R0 = Ab + 4 * n2;
  double* R1 = Ab + 5 * n2;
  for_each_ij(N, [&](int i, int j) { Ab[(size_t)j * Np + i] = a * K[(size_t)i * N + j]; });
  __syncthreads();
  auto ld = [&](const double* M) {
    return [=](int i, int k) { return (i < N && k < N) ? M[(size_t)k * Np + i] : 0.0; };
  };
  auto put = [&](double* M) {
    return [=](int i, int j, double c) {
      if (i < N && j < N) M[(size_t)j * Np + i] = c;
    };
  };
  mm<NC, false, false>(Np, ld(Ab), ld(Ab), put(A2), S);
  __syncthreads();
  mm<NC, false, false>(Np, ld(A2), ld(Ab), put(A3), S);
  __syncthreads();
  mm<NC, false, false>(Np, ld(A2), ld(A2), put(A4), S);
  __syncthreads();
  // C_j(i, j') at one element
  auto cj = [&](int jb, int i, int jj) {
    const size_t o = (size_t)jj * Np + i;
    return ((i == jj) ? kInvFact[4 * jb] : 0.0) + Ab[o] * kInvFact[4 * jb + 1] +
           A2[o] * kInvFact[4 * jb + 2] + A3[o] * kInvFact[4 * jb + 3];
  };
  for_each_ij(N, [&](int i, int j) {
    R0[(size_t)j * Np + i] = A4[(size_t)j * Np + i] * kInvFact[16] + cj(3, i, j);
  });
  __syncthreads();
  double* cur = R0;
  double* nxt = R1;
  for (int jb = 2; jb >= 0; --jb) {
    mm<NC, false, false>(
        Np, ld(cur), ld(A4),
        [&](int i, int j, double c) {
          if (i < N && j < N) nxt[(size_t)j * Np + i] = c + cj(jb, i, j);
        }, S);
    __syncthreads();
    double* t = cur; cur = nxt; nxt = t;
  }
  for (int r = 0; r < q; ++r) {
    mm<NC, false, false>(
        Np, [&](int i, int kk) { return (i < N && kk < N) ? cur[(size_t)kk * Np + i] : 0.0; },
        [&](int kk, int j) { return (kk < N && j < N) ? cur[(size_t)j * Np + kk] : 0.0; },
        [&](int i, int j, double c) {
          if (i < N && j < N) nxt[(size_t)j * Np + i] = c;
        }, S);
    __syncthreads();
    double* t = cur; cur = nxt; nxt = t;
  }
  bool bad = false;
  for_each_ij(N, [&](int i, int j) {
    const double v = cur[(size_t)j * Np + i];
    if (!isfinite(v)) bad = true;
    out[(size_t)j * Np + i] = v;
    if (it.sign > 0 && P.outE) P.outE[(size_t)i * N + j] = v;
  });
  if (bad) status_merge(P.status, -4);
}

// ---------------------------------------------------------------------------
// IK_EXPORT: X, D, T of slot a in the caller's layout.
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void do_export(const Prob& P, const Item& it, SmemC<NC>&) {
  const int N = P.N, Np = P.Np;
  CMat X = cmat_at(it.a.X, Np), T = cmat_at(it.a.T, Np);
  for (int idx = threadIdx.x; idx < N * N; idx += WG) {
    const int i = idx / N, j = idx % N;
    if (P.outX) { P.outX[2 * (size_t)idx] = X.r(i, j); P.outX[2 * (size_t)idx + 1] = X.m(i, j); }
    if (P.outT) { P.outT[2 * (size_t)idx] = T.r(i, j); P.outT[2 * (size_t)idx + 1] = T.m(i, j); }
  }
  for (int i = threadIdx.x; i < N; i += WG)
    if (P.outD) P.outD[i] = it.a.D[i];
}

// Size class of one item inside a launch of class NC: an item with N <= C
// for a smaller class C runs that class's code on the same shared memory
// (SmemC<C> is a prefix-compatible, smaller layout), so a batch of mixed
// sizes pays for each item's own size, not for the largest one.
template <int NC, class F>
__device__ __forceinline__ void by_class(int n, F&& f) {
  if constexpr (NC > 128) {
    f(IC<NC>{});
  } else {
    if constexpr (NC > 32) if (n <= 32) { f(IC<32>{}); return; }
    if constexpr (NC > 64) if (n <= 64) { f(IC<64>{}); return; }
    if constexpr (NC > 80) if (n <= 80) { f(IC<80>{}); return; }
    if constexpr (NC > 96) if (n <= 96) { f(IC<96>{}); return; }
    f(IC<NC>{});
  }
}

// One kernel per work-item kind, so that profiles and timings name the phase.
#define FDET_KERNEL(NAME, BODY)                                                        \
  template <int NC>                                                                  \
  __global__ __launch_bounds__(WG) void NAME(const Prob* __restrict__ probs,           \
                                             const Item* __restrict__ items) {         \
    __shared__ SmemC<NC> S_;                                                          \
    const Item& it = items[blockIdx.x];                                                \
    const Prob& P = probs[it.prob];                                                    \
    by_class<NC>(P.N, [&](auto cls) {                                                  \
      constexpr int C = decltype(cls)::value;                                          \
      static_assert(sizeof(SmemC<C>) <= sizeof(SmemC<NC>), "class layout");           \
      SmemC<C>& S = *reinterpret_cast<SmemC<C>*>(&S_);                                 \
      BODY;                                                                            \
    });                                                                                \
  }

FDET_KERNEL(k_expm, do_expm<C>(P, it, S))
FDET_KERNEL(k_chain, do_chain<C>(P, it, S))
FDET_KERNEL(k_combine, do_combine<C>(P, it, S))
FDET_KERNEL(k_close, do_close<C>(P, it.a, cmat_at(it.scr, P.Np),
                                   cmat_at(it.scr + cmat_doubles(P.Np), P.Np),
                                   cmat_at(it.scr, P.Np), (it.flags & IF_WANT_G) != 0, true, true,
                                   tstore(it.scr, P.Np), S))
FDET_KERNEL(k_force, do_force<C>(P, it, S))
FDET_KERNEL(k_export, do_export<C>(P, it, S))
FDET_KERNEL(k_displaced, do_displaced<C>(P, it, S))

// One item of any kind (the single-launch kernel below).
template <int C>
__device__ __forceinline__ void run_item(const Prob& P, const Item& it, SmemC<C>& S) {
  switch (it.kind) {
    case IK_EXPM: do_expm<C>(P, it, S); break;
    case IK_CHAIN: do_chain<C>(P, it, S); break;
    case IK_COMBINE: do_combine<C>(P, it, S); break;
    case IK_CLOSE:
      do_close<C>(P, it.a, cmat_at(it.scr, P.Np), cmat_at(it.scr + cmat_doubles(P.Np), P.Np),
                  cmat_at(it.scr, P.Np), (it.flags & IF_WANT_G) != 0, true, true,
                  tstore(it.scr, P.Np), S);
      break;
    case IK_FORCE: do_force<C>(P, it, S); break;
    case IK_EXPORT: do_export<C>(P, it, S); break;
    case IK_DISPLACED: do_displaced<C>(P, it, S); break;
    default: break;
  }
}

// The whole plan in one launch: each workgroup claims the next item of the
// list (which the host ordered by a simulated critical-path schedule, every
// item after the items it depends on), waits until those items are complete
// in this launch, runs it and marks it complete.  Because claims follow the
// list order, every item an item waits for has been claimed by a running
// workgroup, so the waits end; an item that nonetheless waits longer than
// `spin_ticks` of the constant-rate clock is skipped with FD_ERR_HIP in the
// problem's status (and still marked complete), so the launch always ends.
// Which workgroup runs an item does not change its arithmetic: results are
// bit-identical to one launch per phase.
template <int NC>
__global__ __launch_bounds__(WG) void k_persist(const Prob* __restrict__ probs,
                                                const Item* __restrict__ items, int nitems,
                                                const int32_t* __restrict__ deps, uint32_t* done,
                                                Sched* sched, uint64_t spin_ticks) {
  __shared__ SmemC<NC> S_;
  __shared__ int s_item;
  __shared__ int s_ok;
  const uint32_t epoch = sched->epoch;
  while (true) {
    if (threadIdx.x == 0)
      s_item = (int)__hip_atomic_fetch_add(&sched->next, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int idx = s_item;
    if (idx >= nitems) break;
    const Item it = items[idx];
    if (threadIdx.x == 0) {
      int ok = 1;
      const uint64_t t0 = wall_clock64();
      for (int d = 0; d < it.ndep && ok; ++d) {
        const uint32_t* f = done + deps[it.dep0 + d];
        while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
          __builtin_amdgcn_s_sleep(8);
          if (wall_clock64() - t0 > spin_ticks) { ok = 0; break; }
        }
      }
      s_ok = ok;
    }
    __syncthreads();
    // acquire: what the items waited for wrote is visible to every wave
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const Prob P = probs[it.prob];
    if (s_ok) {
      by_class<NC>(P.N, [&](auto cls) {
        constexpr int C = decltype(cls)::value;
        static_assert(sizeof(SmemC<C>) <= sizeof(SmemC<NC>), "class layout");
        SmemC<C>& S = *reinterpret_cast<SmemC<C>*>(&S_);
        run_item<C>(P, it, S);
      });
    } else if (threadIdx.x == 0) {
      status_merge(P.status, -5);
    }
    // release: every wave's results are visible before the item is marked
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(done + idx, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

#if FDET_NC == 32
// Clears the status words; with a single-launch plan also starts its next
// launch (epoch + 1, claim counter 0).
__global__ void k_init_status(const Prob* __restrict__ probs, int nprob, Sched* sched) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nprob && probs[i].status) *probs[i].status = 0;
  if (i == 0 && sched) {
    sched->epoch = sched->epoch + 1u;
    sched->next = 0u;
  }
}
#endif

}  // namespace fdet

// Launchers used by the host planner.
template <int NC>
static hipError_t launch_kind(int kind, const fdet::Prob* probs, const fdet::Item* items, int n,
                              hipStream_t st) {
  using namespace fdet;
  const dim3 g(n), b(WG);
  switch (kind) {
    case IK_EXPM: hipLaunchKernelGGL(k_expm<NC>, g, b, 0, st, probs, items); break;
    case IK_CHAIN: hipLaunchKernelGGL(k_chain<NC>, g, b, 0, st, probs, items); break;
    case IK_COMBINE: hipLaunchKernelGGL(k_combine<NC>, g, b, 0, st, probs, items); break;
    case IK_CLOSE: hipLaunchKernelGGL(k_close<NC>, g, b, 0, st, probs, items); break;
    case IK_FORCE: hipLaunchKernelGGL(k_force<NC>, g, b, 0, st, probs, items); break;
    case IK_EXPORT: hipLaunchKernelGGL(k_export<NC>, g, b, 0, st, probs, items); break;
    case IK_DISPLACED: hipLaunchKernelGGL(k_displaced<NC>, g, b, 0, st, probs, items); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// This file is compiled once per launch class (-DFDET_NC=32, 64, 80, 96, 128
// or 512) so that the classes build in parallel; the host dispatches on the
// largest N of a launch (fdet_launch_items in fdet_abi.cpp).
#ifndef FDET_NC
#error "compile with -DFDET_NC=<launch class>"
#endif
#define FDET_CAT2(a, b) a##b
#define FDET_CAT(a, b) FDET_CAT2(a, b)

extern "C" hipError_t FDET_CAT(fdet_launch_items_, FDET_NC)(int kind, const fdet::Prob* probs,
                                                          const fdet::Item* items, int nitems,
                                                          hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  return launch_kind<FDET_NC>(kind, probs, items, nitems, st);
}

// Single launch of a whole plan; grid = workgroups that run at once (at
// most one per item).
// The single launch is switched off in the entry points (FD_SINGLE_LAUNCH
// returns FD_ERR_UNSUPPORTED); its kernel is only compiled with
// -DFDET_SINGLE_LAUNCH_KERNEL.
extern "C" hipError_t FDET_CAT(fdet_launch_persist_, FDET_NC)(
    const fdet::Prob* probs, const fdet::Item* items, int nitems, const int32_t* deps,
    uint32_t* done, fdet::Sched* sched, uint64_t spin_ticks, int grid, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#ifdef FDET_SINGLE_LAUNCH_KERNEL
  hipLaunchKernelGGL(fdet::k_persist<FDET_NC>, dim3(grid), dim3(fdet::WG), 0, st, probs, items,
                     nitems, deps, done, sched, spin_ticks);
  return hipGetLastError();
#else
  (void)probs; (void)items; (void)deps; (void)done; (void)sched; (void)spin_ticks; (void)grid;
  (void)st;
  return hipErrorNotSupported;
#endif
}

// Workgroups of the single-launch kernel that fit on one compute unit.
extern "C" int FDET_CAT(fdet_persist_blocks_per_cu_, FDET_NC)(void) {
  int n = 0;
#ifdef FDET_SINGLE_LAUNCH_KERNEL
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fdet::k_persist<FDET_NC>, fdet::WG, 0) !=
          hipSuccess ||
      n < 1)
#endif
    n = 1;
  return n;
}

#if FDET_NC == 32
extern "C" hipError_t fdet_launch_init_status(const fdet::Prob* probs, int nprob,
                                              fdet::Sched* sched, hipStream_t st) {
  hipLaunchKernelGGL(fdet::k_init_status, dim3((nprob + 255) / 256), dim3(256), 0, st, probs, nprob,
                     sched);
  return hipGetLastError();
}
#endif

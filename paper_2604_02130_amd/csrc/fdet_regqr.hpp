// Workgroup primitives for N <= 128 (one workgroup of WG = 512 threads):
// a register-resident column-pivoted Householder QR, the explicit Q, the
// solve with R and Q^H, and an LDS-staged FP64 MFMA product.
//
// QR layout: the workgroup is 32 groups of 16 lanes (4 per wave, one DPP row
// each).  Physical column c of the matrix being factorised lives in group
// c % 32, slot c / 32; lane l16 = lane % 16 holds rows l16 + 16 m.  A column
// reduction is a 16-lane DPP reduction, so the four groups of a wave reduce
// in the same instructions, and no column leaves the registers during the
// factorisation.  Every Householder vector is written once into an LDS
// triangle, which the explicit Q and the Q^H solve then read without any
// device-memory round trip.
//
// After rq_qrp the factor is also written back to W in pivoted order:
// column j holds R(0..j, j); the reflectors stay in the LDS triangle.
#pragma once

#include "fdet_device.hpp"

namespace fdet {

template <int NC>
struct RegClass {
  static constexpr int CPL = (NC + 31) / 32;   // columns per lane group
  static constexpr int RPL = (NC + 15) / 16;   // rows per lane
};

// k-panel depth of the staged product (4 MFMA k-steps); deeper panels would
// double the prefetch registers of every thread
template <int NC>
__host__ __device__ constexpr int kpanel() { return 16; }

// LDS row stride (doubles) of a staged panel.  The four k-rows that one MFMA
// operand read spans then start 2 doubles (4 banks) apart; measured on
// gfx950, strides of n + 1 .. n + 3 beat n + 16 (mod 32) by 15-90 % on these
// products (the 16-row products of the blocked QR gain the most).
__host__ __device__ constexpr int panel_stride(int n) { return n + 2; }

template <int NC>
struct BigLds {
  static constexpr int TRI = NC * (NC + 1) / 2;              // complex triangle
  static constexpr int PANEL = 4 * kpanel<NC>() * panel_stride(NC);   // two complex panels
  static constexpr int N = (2 * TRI > PANEL) ? 2 * TRI : PANEL;
  static constexpr int UB = 16 * ((NC + 15) / 16);           // one padded column
};

// LDS staging of the large class's macro-tiled product: two complex K panels
// of 16 x 144 doubles (fdet_large.hpp)
constexpr int LG_BIG = 2 * 2 * 16 * 144;

// Shared state of size class NC (N <= NC): the scalar arrays of Smem plus a
// large area used as the reflector / R triangle or as the product's panels.
template <int NC>
struct SmemC : Smem<(NC <= 128 ? 128 : 512)> {
  double big[NC <= 128 ? BigLds<NC>::N : LG_BIG];
  // current reflector as a full column (zero above its row), two buffers
  double ubr[2][NC <= 128 ? BigLds<NC>::UB : 1];
  double ubi[2][NC <= 128 ? BigLds<NC>::UB : 1];
  // large class: T and V^H V of a panel (re, im), block-sum partials and
  // sums, row j of a panel; two buffers each where consecutive steps overlap
  double lgt[NC <= 128 ? 1 : 1024];
  double lgred[NC <= 128 ? 1 : 2 * NWAVE * 32];
  double lgsum[NC <= 128 ? 1 : 2 * 32];
  double lgrow[NC <= 128 ? 1 : 2 * 32];
};

// index of (row r, column j) in the lower (reflector) triangle, r >= j
template <int NC>
__device__ __forceinline__ int tri_lo(int r, int j) { return j * NC - (j * (j - 1)) / 2 + (r - j); }
// index of (row r, column i) in the upper (R) triangle, r <= i
__device__ __forceinline__ int tri_up(int r, int i) { return (i * (i + 1)) / 2 + r; }

// 32-bit DPP move applied to both halves of a double.  Every control used
// here permutes lanes inside a row with all rows and banks enabled, so every
// lane reads a valid source and no previous destination value is needed
// (one instruction per half, no zeroing move).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of a DPP row, result in every lane: quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.  Each step adds
// a commuted pair, so all 16 lanes end with the same bits.
__device__ __forceinline__ double red16(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// compile-time loop: f(IC<B>{}), f(IC<B+1>{}), ..., f(IC<E-1>{})
template <int V>
struct IC {
  static constexpr int value = V;
};
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(IC<B>{});
    static_for<B + 1, E>(f);
  }
}

// The same reflector on the column slots q >= QLO of a lane, rows in blocks
// m >= MLO (the reflector is zero on rows < 16 MLO), reductions interleaved.
// Both bounds are template constants: the skipped work is not emitted.
// Written as explicit fused multiply-add chains, four per complex element for
// u^H y and four for the update: the compiler does not contract
// s += a b + c d by itself, and these loops are bound by VALU issue.
template <int CPL, int RPL, int MLO, int QLO>
__device__ __forceinline__ void rq_reflect_all(double beta, const double* ur, const double* ui,
                                               double (*yr)[RPL], double (*yi)[RPL]) {
  double wr[CPL], wi[CPL];
#pragma unroll
  for (int q = QLO; q < CPL; ++q) {
    double sr = ur[MLO] * yr[q][MLO];
    double si = ur[MLO] * yi[q][MLO];
    sr = fma(ui[MLO], yi[q][MLO], sr);
    si = fma(-ui[MLO], yr[q][MLO], si);
#pragma unroll
    for (int m = MLO + 1; m < RPL; ++m) {
      sr = fma(ur[m], yr[q][m], sr);
      si = fma(ur[m], yi[q][m], si);
      sr = fma(ui[m], yi[q][m], sr);
      si = fma(-ui[m], yr[q][m], si);
    }
    wr[q] = sr;
    wi[q] = si;
  }
#pragma unroll
  for (int q = QLO; q < CPL; ++q) {
    wr[q] = beta * red16(wr[q]);
    wi[q] = beta * red16(wi[q]);
  }
#pragma unroll
  for (int q = QLO; q < CPL; ++q) {
#pragma unroll
    for (int m = MLO; m < RPL; ++m) {
      yr[q][m] = fma(-ur[m], wr[q], yr[q][m]);
      yi[q][m] = fma(-ur[m], wi[q], yi[q][m]);
      yr[q][m] = fma(ui[m], wi[q], yr[q][m]);
      yi[q][m] = fma(-ui[m], wr[q], yi[q][m]);
    }
  }
}

// 1 / sqrt(x) and 1 / x for normal x well inside the exponent range: the
// hardware estimates refined by two Newton steps each (each step doubles the
// number of correct bits of the estimate).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

// Householder coefficients of a column with squared norm s2 (rows >= j) and
// leading element a0: alpha = sqrt(s2), e = a0 / |a0| (1 for a0 = 0) and
// beta = 1 / (alpha (alpha + |a0|)), so that H = I - beta u u^H with
// u = x + e alpha e_j maps x to -e alpha e_j.  The arguments are uniform over
// the wave, so the choice between the refined estimates (the formation of a
// reflector is on the critical path of every column) and the library
// functions (tiny or huge norms) is a scalar branch.
__device__ __forceinline__ void hh_coeffs(double s2, double a0r, double a0i, double& alpha,
                                          double& beta, double& er, double& ei) {
  const double q0 = a0r * a0r + a0i * a0i;
  constexpr double lo = 0x1p-700, hi = 0x1p+700;
  er = 1.0;
  ei = 0.0;
  if (s2 > lo && s2 < hi && (q0 == 0.0 || q0 > lo)) {
    alpha = s2 * rsqrt_nr(s2);
    double aa0 = 0.0;
    if (q0 > 0.0) {
      const double y0 = rsqrt_nr(q0);
      aa0 = q0 * y0;
      er = a0r * y0;
      ei = a0i * y0;
    }
    beta = rcp_nr(alpha * (alpha + aa0));
  } else {
    alpha = sqrt(s2);
    const double aa0 = sqrt(q0);
    if (aa0 > 0.0) {
      const double inv = 1.0 / aa0;
      er = a0r * inv;
      ei = a0i * inv;
    }
    beta = alpha > 0.0 ? 1.0 / (alpha * (alpha + aa0)) : 0.0;
  }
}

// Pivot refresh at the start of row phase JB (step j = 16 JB): the columns
// at positions >= j are ordered again by partial norm (rows >= j) x key,
// decreasing, ties to the lower position, and moved to their new slots
// through W.  Positions < j (finished) stay in place.
template <int NC, int JB, int QLO>
__device__ __forceinline__ void rq_repivot(CMat W, int N,
                                           double (&ar)[RegClass<NC>::CPL][RegClass<NC>::RPL],
                                           double (&ai)[RegClass<NC>::CPL][RegClass<NC>::RPL],
                                           SmemC<NC>& S) {
  constexpr int CPL = RegClass<NC>::CPL, RPL = RegClass<NC>::RPL;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int l16 = lane & 15, grp = wave * 4 + (lane >> 4);
  const int j = 16 * JB;
#pragma unroll
  for (int q = QLO; q < CPL; ++q) {
    const int k = grp + 32 * q;
    double s = 0.0;
#pragma unroll
    for (int m = JB; m < RPL; ++m) {
      s = fma(ar[q][m], ar[q][m], s);
      s = fma(ai[q][m], ai[q][m], s);
    }
    s = red16(s);
    if (k >= j && k < N) {
      if (l16 == 0) S.v3[k] = sqrt(s) * S.csp[k];
#pragma unroll
      for (int m = 0; m < RPL; ++m) {
        const int r = l16 + 16 * m;
        if (r < N) { W.r(r, k) = ar[q][m]; W.m(r, k) = ai[q][m]; }
      }
    }
  }
  __syncthreads();
  for (int k = j + tid; k < N; k += WG) {
    const double kk = S.v3[k];
    int pos = j;
    for (int d = j; d < N; ++d) {
      const double kd = S.v3[d];
      pos += (kd > kk || (kd == kk && d < k)) ? 1 : 0;
    }
    S.tmp0[pos] = k;   // new position pos takes old position k
  }
  __syncthreads();
  for (int p = j + tid; p < N; p += WG) {
    const int k = S.tmp0[p];
    S.tmp1[p] = S.piv[k];
    S.norms[p] = S.csp[k];
  }
  __syncthreads();
  for (int p = j + tid; p < N; p += WG) {
    S.piv[p] = S.tmp1[p];
    S.csp[p] = S.norms[p];
  }
#pragma unroll
  for (int q = QLO; q < CPL; ++q) {
    const int p = grp + 32 * q;
    if (p >= j && p < N) {
      const int k = S.tmp0[p];
#pragma unroll
      for (int m = 0; m < RPL; ++m) {
        const int r = l16 + 16 * m;
        ar[q][m] = r < N ? W.r(r, k) : 0.0;
        ai[q][m] = r < N ? W.m(r, k) : 0.0;
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// rq_qrp: column-pivoted Householder QR of the N x N matrix in W, with the
// pivot order refreshed every 16 columns.
//
// The columns are ordered by key = |column| x keys[c] (keys == nullptr: 1),
// decreasing, ties to the lower index; every 16 columns the remaining ones
// are ordered again by their partial norms (rows not yet eliminated) x key.
// Householder QR treats every column independently of its scale, so this is
// the pivot order of W diag(keys) while all arithmetic stays on W.  Ordering
// once at the start is not enough: for (near-)degenerate scales the T
// factors of the UDV products then grow from product to product.
//
// Output: R in the upper triangle of W in pivoted column order, S.u0r/u0i
// and S.beta of every reflector, S.piv (original column at each position),
// S.csp (key at each position), S.nref (reflectors formed), S.rdr/rdi
// (diagonal of R) and reflector j in the LDS triangle (rows >= j, row j
// holding u0).  Below the diagonal W holds no reflector data on this path;
// consumers read the triangle.
//
// The columns enter the registers already in pivot order: slot q of group g
// holds position k = g + 32 q.  Step j runs in row phase JB = j / 16, where
// the reflector is zero on row blocks m < JB and every slot q < JB / 2 holds
// only positions < j (finished: their rows >= j are never read again), so
// both are left out at compile time.
//
// Per column: the wave holding position j forms the reflector (exact norm)
// and publishes it (one barrier); the remaining slots then take the update
// a <- a - beta u (u^H a).
// ---------------------------------------------------------------------------
template <int NC>
__device__ void rq_qrp(CMat W, int N, const double* keys, SmemC<NC>& S) {
  constexpr int CPL = RegClass<NC>::CPL, RPL = RegClass<NC>::RPL;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int l16 = lane & 15, grp = wave * 4 + (lane >> 4);
  double* tr = S.big;
  double* ti = S.big + BigLds<NC>::TRI;

  // ---- pivot keys from memory
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = grp + 32 * q;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      if (c < N && r < N) {
        const double xr = W.r(r, c), xi = W.m(r, c);
        s += xr * xr + xi * xi;
      }
    }
    s = red16(s);
    if (c < N && l16 == 0) S.v3[c] = sqrt(s) * (keys ? keys[c] : 1.0);
  }
  __syncthreads();
  // position of each column: rank by key (decreasing), ties to the lower index
  for (int c = tid; c < N; c += WG) {
    const double kc = S.v3[c];
    int pos = 0;
    for (int d = 0; d < N; ++d) {
      const double kd = S.v3[d];
      pos += (kd > kc || (kd == kc && d < c)) ? 1 : 0;
    }
    S.pinv[c] = pos;
    S.piv[pos] = c;
    S.csp[pos] = keys ? keys[c] : 1.0;
  }
  if (tid == 0) S.nref = 0;
  __syncthreads();

  // ---- registers in pivot order
  double ar[CPL][RPL], ai[CPL][RPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int k = grp + 32 * q;
    const int c = (k < N) ? S.piv[k] : 0;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      const bool in = k < N && r < N;
      ar[q][m] = in ? W.r(r, c) : 0.0;
      ai[q][m] = in ? W.m(r, c) : 0.0;
    }
  }

  static_for<0, RPL>([&](auto jbc) {
    constexpr int JB = decltype(jbc)::value;
    constexpr int QLO = JB / 2;
    if constexpr (JB > 0) {
      if (16 * JB < N - 1) rq_repivot<NC, JB, QLO>(W, N, ar, ai, S);
    }
    const int jend = min(16 * JB + 16, N);
    for (int j = 16 * JB; j < jend; ++j) {
      const int buf = j & 1;
      const int og = j & 31, qp = j >> 5;
      // ---- the wave holding position j forms the reflector and publishes it
      if (wave == (og >> 2)) {
        double xr = 0.0, xi = 0.0, s = 0.0;
#pragma unroll
        for (int q = QLO; q < CPL; ++q) {
          if (q != qp) continue;
          xr = ar[q][JB];
          xi = ai[q][JB];
#pragma unroll
          for (int m = JB; m < RPL; ++m) {
            const int r = l16 + 16 * m;
            const double vr = (r >= j) ? ar[q][m] : 0.0;
            const double vi = (r >= j) ? ai[q][m] : 0.0;
            s = fma(vr, vr, s);
            s = fma(vi, vi, s);
          }
        }
        // every group of the wave reduced its own slot qp; take the owner's
        const double s2 = readlane_d(red16(s), 16 * (og & 3));
        const int src = 16 * (og & 3) + (j & 15);
        const double a0r = readlane_d(xr, src);
        const double a0i = readlane_d(xi, src);
        double alpha, beta, er, ei;
        hh_coeffs(s2, a0r, a0i, alpha, beta, er, ei);
        const bool refl = alpha > 0.0;
        const double u0r = fma(er, alpha, a0r), u0i = fma(ei, alpha, a0i);
        if (grp == og) {
#pragma unroll
          for (int q = QLO; q < CPL; ++q) {
            if (q != qp) continue;
#pragma unroll
            for (int m = JB; m < RPL; ++m) {
              const int r = l16 + 16 * m;
              double vr = (r > j) ? ar[q][m] : 0.0;
              double vi = (r > j) ? ai[q][m] : 0.0;
              if (r == j) { vr = u0r; vi = u0i; }
              S.ubr[buf][r] = vr;
              S.ubi[buf][r] = vi;
              if (r >= j && r < N) {
                tr[tri_lo<NC>(r, j)] = vr;
                ti[tri_lo<NC>(r, j)] = vi;
              }
            }
          }
        }
        if (lane == 0) {
          S.rdr[j] = refl ? -er * alpha : 0.0;
          S.rdi[j] = refl ? -ei * alpha : 0.0;
          S.u0r[j] = refl ? u0r : 0.0;
          S.u0i[j] = refl ? u0i : 0.0;
          S.beta[j] = beta;
          if (refl) S.nref += 1;
        }
      }
      __syncthreads();

      // ---- the open slots take a <- a - beta u (u^H a).  u is zero above
      // row j, so rows above j do not change; positions <= j only change
      // below their diagonal, which no consumer reads.
      const double beta = S.beta[j];
      double ur[RPL], ui[RPL];
#pragma unroll
      for (int m = JB; m < RPL; ++m) {
        ur[m] = S.ubr[buf][l16 + 16 * m];
        ui[m] = S.ubi[buf][l16 + 16 * m];
      }
      rq_reflect_all<CPL, RPL, JB, QLO>(beta, ur, ui, ar, ai);
    }
  });
  __syncthreads();

  // ---- R back to W (position k = grp + 32 q), with the diagonal exactly as
  // formed (the in-register value carries the rounding of the reflector
  // applied to its own column)
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int k = grp + 32 * q;
    if (k >= N) continue;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      if (r == k) { ar[q][m] = S.rdr[k]; ai[q][m] = S.rdi[k]; }
      if (r < N) { W.r(r, k) = ar[q][m]; W.m(r, k) = ai[q][m]; }
    }
  }
  __syncthreads();
}

// reflector j (rows of this lane in blocks >= MLO) from the LDS triangle
template <int NC, int RPL, int MLO>
__device__ __forceinline__ void rq_load_u(const SmemC<NC>& S, int N, int j, int l16, double* ur,
                                          double* ui) {
  const double* tr = S.big;
  const double* ti = S.big + BigLds<NC>::TRI;
#pragma unroll
  for (int m = MLO; m < RPL; ++m) {
    const int r = l16 + 16 * m;
    const bool in = r >= j && r < N;
    ur[m] = in ? tr[tri_lo<NC>(r, j)] : 0.0;
    ui[m] = in ? ti[tri_lo<NC>(r, j)] : 0.0;
  }
}

// Q = H_0 ... H_{N-1} written to Q (backward accumulation).  Groups own
// whole columns and read reflectors from LDS: no barrier inside.  When H_j is
// applied, columns c < j of the partial product are still e_c and every
// column is zero on rows < j, so slots q < JB / 2 and row blocks < JB (JB =
// j / 16) are left out.  The caller synchronises after (Q complete).
template <int NC>
__device__ void rq_form_q(int N, CMat Q, const SmemC<NC>& S) {
  constexpr int CPL = RegClass<NC>::CPL, RPL = RegClass<NC>::RPL;
  const int lane = lane_id(), wave = wave_id();
  const int l16 = lane & 15, grp = wave * 4 + (lane >> 4);
  double qr[CPL][RPL], qi[CPL][RPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = grp + 32 * q;
#pragma unroll
    for (int m = 0; m < RPL; ++m) { qr[q][m] = (l16 + 16 * m == c) ? 1.0 : 0.0; qi[q][m] = 0.0; }
  }
  static_for<0, RPL>([&](auto kc) {
    constexpr int JB = RPL - 1 - decltype(kc)::value;
    constexpr int QLO = JB / 2;
    for (int j = min(16 * JB + 15, N - 1); j >= 16 * JB; --j) {
      const double beta = S.beta[j];
      if (beta == 0.0) continue;
      double ur[RPL], ui[RPL];
      rq_load_u<NC, RPL, JB>(S, N, j, l16, ur, ui);
      rq_reflect_all<CPL, RPL, JB, QLO>(beta, ur, ui, qr, qi);
    }
  });
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = grp + 32 * q;
    if (c >= N) continue;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      if (r < N) { Q.r(r, c) = qr[q][m]; Q.m(r, c) = qi[q][m]; }
    }
  }
}

// Y <- R^{-1} Q^H Y for the factor of rq_qrp; Y is loaded from and stored
// to Yg.  Q^H is applied from the LDS reflectors (H_j leaves rows < j alone);
// then R (from W) replaces them in the LDS triangle for the back
// substitution, which at row i only touches rows <= i.
template <int NC>
__device__ void rq_solve(CMat W, int N, CMat Yg, SmemC<NC>& S) {
  constexpr int CPL = RegClass<NC>::CPL, RPL = RegClass<NC>::RPL;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int l16 = lane & 15, grp = wave * 4 + (lane >> 4);
  const int gbase = lane & ~15;
  double yr[CPL][RPL], yi[CPL][RPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = grp + 32 * q;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      const bool in = c < N && r < N;
      yr[q][m] = in ? Yg.r(r, c) : 0.0;
      yi[q][m] = in ? Yg.m(r, c) : 0.0;
    }
  }
  static_for<0, RPL>([&](auto jbc) {
    constexpr int JB = decltype(jbc)::value;
    const int jend = min(16 * JB + 16, N);
    for (int j = 16 * JB; j < jend; ++j) {
      const double beta = S.beta[j];
      if (beta == 0.0) continue;
      double ur[RPL], ui[RPL];
      rq_load_u<NC, RPL, JB>(S, N, j, l16, ur, ui);
      rq_reflect_all<CPL, RPL, JB, 0>(beta, ur, ui, yr, yi);
    }
  });
  __syncthreads();
  // R into the LDS triangle (column i, rows 0..i)
  double* tr = S.big;
  double* ti = S.big + BigLds<NC>::TRI;
  for_each_ij(N, [&](int r, int i) {
    if (r <= i) { tr[tri_up(r, i)] = W.r(r, i); ti[tri_up(r, i)] = W.m(r, i); }
  });
  __syncthreads();
  static_for<0, RPL>([&](auto kc) {
    constexpr int IB = RPL - 1 - decltype(kc)::value;   // rows i in block IB
    for (int i = min(16 * IB + 15, N - 1); i >= 16 * IB; --i) {
      const double dr = S.rdr[i], di = S.rdi[i];
      const double rden = 1.0 / (dr * dr + di * di);
      const double ir = dr * rden, ii = -di * rden;   // 1 / R_ii
      const int li = i & 15;
      double cr[IB + 1], ci[IB + 1];
#pragma unroll
      for (int m = 0; m <= IB; ++m) {
        const int r = l16 + 16 * m;
        const bool in = r < i;
        cr[m] = in ? tr[tri_up(r, i)] : 0.0;
        ci[m] = in ? ti[tri_up(r, i)] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const double vr = __shfl(yr[q][IB], gbase + li, 64);
        const double vi = __shfl(yi[q][IB], gbase + li, 64);
        const double zr = fma(vr, ir, -vi * ii);
        const double zi = fma(vr, ii, vi * ir);
#pragma unroll
        for (int m = 0; m <= IB; ++m) {
          const int r = l16 + 16 * m;
          if (r == i) { yr[q][m] = zr; yi[q][m] = zi; }
          yr[q][m] = fma(-cr[m], zr, yr[q][m]);
          yi[q][m] = fma(-cr[m], zi, yi[q][m]);
          yr[q][m] = fma(ci[m], zi, yr[q][m]);
          yi[q][m] = fma(-ci[m], zr, yi[q][m]);
        }
      }
    }
  });
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = grp + 32 * q;
    if (c >= N) continue;
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int r = l16 + 16 * m;
      if (r < N) { Yg.r(r, c) = yr[q][m]; Yg.m(r, c) = yi[q][m]; }
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-staged product C = A B on the FP64 matrix cores (Np <= 128).
//
// K is walked in panels of KP = kpanel<NC>() columns: the whole workgroup
// fetches the next A(:, k0:k0+KP) and B(k0:k0+KP, :) into registers while it
// multiplies the current panels from LDS, so device-memory latency is paid
// once.  Each wave keeps the accumulators of its output tiles (16 x 16,
// round-robin) across all panels.  AC / BC: operand is complex.  Loaders:
// la(i,k,re,im) or la(i,k), lb(k,j,re,im) or lb(k,j), called for indices up
// to NC and returning zero outside N x N; store st(i,j,re,im) or st(i,j,v),
// called for i, j < Np.
// ---------------------------------------------------------------------------
template <int NC, bool AC, bool BC, class LA, class LB, class ST>
__device__ void gemm_lds(int Np, LA la, LB lb, ST st, double* lds) {
  constexpr bool CC = AC || BC;   // complex result
  constexpr int KP = kpanel<NC>();
  // tiles per wave: the 128 class keeps all 8 accumulator tiles of a wave
  // live (one pass over K); smaller classes at most 4 per pass
  constexpr int MAXT = ((NC / 16) * (NC / 16) + NWAVE - 1) / NWAVE;
  constexpr int TCAP = NC >= 128 ? 8 : 4;
  constexpr int TP = MAXT < TCAP ? MAXT : TCAP;
  // the k-steps of a panel fully unrolled except in the 128 class, whose
  // hoisted operands would spill
  constexpr int UNR = NC >= 128 ? 1 : KP / 4;
  constexpr int PER = (NC * KP + WG - 1) / WG;   // panel elements per thread
  // Panels are staged with the class size NC as their extent and stride, so
  // all index arithmetic of the staging is compile-time; elements outside
  // Np are fetched as zeros by the (masking) loaders and never multiplied.
  constexpr int SD = panel_stride(NC);
  constexpr int NEL = NC * KP;
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  double* Ar = lds;
  double* Ai = Ar + KP * SD;
  double* Br = Ar + (AC ? 2 : 1) * KP * SD;
  double* Bi = Br + KP * SD;
  const int nt = Np >> 4, ntiles = nt * nt;
  const int npass = (ntiles + NWAVE * TP - 1) / (NWAVE * TP);

  double fa_r[PER], fa_i[PER], fb_r[PER], fb_i[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + WG * x;
      fa_r[x] = 0.0; fa_i[x] = 0.0; fb_r[x] = 0.0; fb_i[x] = 0.0;
      if (e < NEL) {
        const int i = e % NC, kk = e / NC;            // A: rows fastest
        if constexpr (AC) la(i, k0 + kk, fa_r[x], fa_i[x]);
        else fa_r[x] = la(i, k0 + kk);
        const int kb = e % KP, j = e / KP;            // B: k fastest
        if constexpr (BC) lb(k0 + kb, j, fb_r[x], fb_i[x]);
        else fb_r[x] = lb(k0 + kb, j);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + WG * x;
      if (e < NEL) {
        const int i = e % NC, kk = e / NC;
        Ar[kk * SD + i] = fa_r[x];
        if constexpr (AC) Ai[kk * SD + i] = fa_i[x];
        const int kb = e % KP, j = e / KP;
        Br[kb * SD + j] = fb_r[x];
        if constexpr (BC) Bi[kb * SD + j] = fb_i[x];
      }
    }
  };
  for (int pass = 0; pass < npass; ++pass) {
    v4d cr[TP], ci[TP];
#pragma unroll
    for (int t = 0; t < TP; ++t) {
      cr[t] = v4d{0.0, 0.0, 0.0, 0.0};
      ci[t] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    fetch(0);
    for (int k0 = 0; k0 < Np; k0 += KP) {
      __syncthreads();
      stash();
      __syncthreads();
      if (k0 + KP < Np) fetch(k0 + KP);
#pragma unroll UNR
      for (int sk = 0; sk < KP / 4; ++sk) {
        const int kk = 4 * sk + lk;
#pragma unroll
        for (int t = 0; t < TP; ++t) {
          const int tile = wave + NWAVE * (pass * TP + t);
          if (tile >= ntiles) break;
          const int i = ((tile % nt) << 4) + li, j = ((tile / nt) << 4) + li;
          const double a_r = Ar[kk * SD + i];
          const double b_r = Br[kk * SD + j];
          if constexpr (AC && BC) {
            const double a_i = Ai[kk * SD + i], b_i = Bi[kk * SD + j];
            cr[t] = mfma4(a_r, b_r, cr[t]);
            ci[t] = mfma4(a_r, b_i, ci[t]);
            cr[t] = mfma4(-a_i, b_i, cr[t]);
            ci[t] = mfma4(a_i, b_r, ci[t]);
          } else if constexpr (AC) {
            const double a_i = Ai[kk * SD + i];
            cr[t] = mfma4(a_r, b_r, cr[t]);
            ci[t] = mfma4(a_i, b_r, ci[t]);
          } else if constexpr (BC) {
            const double b_i = Bi[kk * SD + j];
            cr[t] = mfma4(a_r, b_r, cr[t]);
            ci[t] = mfma4(a_r, b_i, ci[t]);
          } else {
            cr[t] = mfma4(a_r, b_r, cr[t]);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TP; ++t) {
      const int tile = wave + NWAVE * (pass * TP + t);
      if (tile >= ntiles) break;
      const int r0 = ((tile % nt) << 4) + lk, c0 = ((tile / nt) << 4) + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (CC) st(r0 + 4 * r, c0, cr[t][r], ci[t][r]);
        else st(r0 + 4 * r, c0, cr[t][r]);
      }
    }
  }
  __syncthreads();
}

}  // namespace fdet

// Workgroup primitives for 128 < N <= 512 (one workgroup of WG = 512 threads
// per work item, matrices in device memory):
//   lg_gemm       macro-tiled FP64 MFMA product with LDS-staged K panels,
//   lg_qrp        column-pivoted blocked Householder QR (pivot order refreshed
//                 per panel, compact WY panels of 16 reflectors, trailing
//                 updates as MFMA products),
//   lg_form_q     explicit Q by backward accumulation of blocks of 64
//                 reflectors (compact WY, rank-64 MFMA updates),
//   lg_apply_qh   Y <- Q^H Y, by the same blocks,
//   lg_backsolve  Y <- R^{-1} Y, blocked by 16 rows.
//
// An unblocked QR streams the whole trailing matrix through device memory at
// every column (N^3 / 3 complex loads and stores); here each panel touches it
// twice, and all O(N^3) work runs on the matrix cores.
//
// Householder conventions are those of the in-register routines: reflector
// H_j = I - beta_j u_j u_j^H with u_j = (0, .., 0, u0_j, W(j+1:, j)), the
// tail stored below the diagonal of W, u0_j in S.u0r/u0i, beta_j in S.beta;
// a panel of reflectors j0 .. j0+pw-1 is H_j0 ... H_{j0+pw-1} = I - V T V^H
// with T upper triangular (pw x pw), stored per panel in `tst`.
#pragma once

#include "fdet_device.hpp"
#include "fdet_regqr.hpp"

namespace fdet {

constexpr int LG_PW = 16;                        // panel width
constexpr int LG_TDBL = 2 * LG_PW * LG_PW;       // doubles per stored T (re, im)

__host__ __device__ constexpr int lg_tstore_doubles(int Np) { return (Np / LG_PW) * LG_TDBL; }

// ---------------------------------------------------------------------------
// C (M x Nc) = C0 + A (M x K) B (K x Nc), macro tiles TM x TN, K panels of 16
// staged in LDS.  One flat loop runs over (macro tile, K panel) steps and
// prefetches the next step's operands into registers while the current one
// multiplies, so a new macro tile's loads overlap the previous tile's
// products and stores.  Loaders are only called inside the logical sizes
// (la(i, k) with i < M, k < K; lb(k, j) with k < K, j < Nc); st(i, j, ..) only
// for i < M, j < Nc.  With INIT, in(i, j, ..) gives C0 (loaded into the
// accumulators when a macro tile starts), else C0 = 0.
// ---------------------------------------------------------------------------
template <int TM, int TN, bool AC, bool BC, bool INIT, class LA, class LB, class ST, class IN>
__device__ void lg_gemm_impl(int M, int Nc, int K, LA la, LB lb, ST st, IN in, double* lds) {
  constexpr bool CC = AC || BC;
  constexpr int KP = 16;
  constexpr int SA = panel_stride(TM), SB = panel_stride(TN);
  constexpr int TMT = TM / 16, TNT = TN / 16, NT = TMT * TNT;
  constexpr int TPW = (NT + NWAVE - 1) / NWAVE;
  constexpr int EA = TM * KP, EB = KP * TN;
  constexpr int PA = (EA + WG - 1) / WG, PB = (EB + WG - 1) / WG;
  static_assert((AC ? 2 : 1) * KP * SA + (BC ? 2 : 1) * KP * SB <= LG_BIG, "LDS staging");
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  double* Ar = lds;
  double* Ai = Ar + KP * SA;
  double* Br = Ar + (AC ? 2 : 1) * KP * SA;
  double* Bi = Br + KP * SB;
  const int mtm = (M + TM - 1) / TM, mtn = (Nc + TN - 1) / TN;
  const int npan = (K + KP - 1) / KP;
  const int nsteps = mtm * mtn * npan;

  double fa_r[PA], fa_i[PA], fb_r[PB], fb_i[PB];
  auto fetch = [&](int step) {
    const int mt = step / npan, k0 = (step % npan) * KP;
    const int bm = (mt % mtm) * TM, bn = (mt / mtm) * TN;
#pragma unroll
    for (int x = 0; x < PA; ++x) {
      const int e = tid + WG * x;
      fa_r[x] = 0.0; fa_i[x] = 0.0;
      const int i = e % TM, kk = e / TM;          // A: rows fastest
      if (e < EA && bm + i < M && k0 + kk < K) {
        if constexpr (AC) la(bm + i, k0 + kk, fa_r[x], fa_i[x]);
        else fa_r[x] = la(bm + i, k0 + kk);
      }
    }
#pragma unroll
    for (int x = 0; x < PB; ++x) {
      const int e = tid + WG * x;
      fb_r[x] = 0.0; fb_i[x] = 0.0;
      const int kb = e % KP, j = e / KP;          // B: k fastest
      if (e < EB && k0 + kb < K && bn + j < Nc) {
        if constexpr (BC) lb(k0 + kb, bn + j, fb_r[x], fb_i[x]);
        else fb_r[x] = lb(k0 + kb, bn + j);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int x = 0; x < PA; ++x) {
      const int e = tid + WG * x;
      if (e < EA) {
        const int i = e % TM, kk = e / TM;
        Ar[kk * SA + i] = fa_r[x];
        if constexpr (AC) Ai[kk * SA + i] = fa_i[x];
      }
    }
#pragma unroll
    for (int x = 0; x < PB; ++x) {
      const int e = tid + WG * x;
      if (e < EB) {
        const int kb = e % KP, j = e / KP;
        Br[kb * SB + j] = fb_r[x];
        if constexpr (BC) Bi[kb * SB + j] = fb_i[x];
      }
    }
  };
  v4d cr[TPW], ci[TPW];
  if (nsteps > 0) fetch(0);
  for (int step = 0; step < nsteps; ++step) {
    const int mt = step / npan, kp = step % npan;
    const int bm = (mt % mtm) * TM, bn = (mt / mtm) * TN;
    if (kp == 0) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        cr[t] = v4d{0.0, 0.0, 0.0, 0.0};
        ci[t] = v4d{0.0, 0.0, 0.0, 0.0};
        if constexpr (INIT) {
          const int tile = wave + NWAVE * t;
          if (tile < NT) {
            const int r0 = ((tile % TMT) << 4) + lk, c0 = ((tile / TMT) << 4) + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int gi = bm + r0 + 4 * r, gj = bn + c0;
              if (gi < M && gj < Nc) {
                double vr = 0.0, vi = 0.0;
                if constexpr (CC) in(gi, gj, vr, vi);
                else in(gi, gj, vr);
                cr[t][r] = vr;
                ci[t][r] = vi;
              }
            }
          }
        }
      }
    }
    __syncthreads();
    stash();
    __syncthreads();
    if (step + 1 < nsteps) fetch(step + 1);
    // two k-steps at a time: fully unrolled, the hoisted LDS operands spill
#pragma unroll 2
    for (int sk = 0; sk < KP / 4; ++sk) {
      const int kk = 4 * sk + lk;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wave + NWAVE * t;
        if (tile >= NT) break;
        const int i = ((tile % TMT) << 4) + li, j = ((tile / TMT) << 4) + li;
        const double a_r = Ar[kk * SA + i];
        const double b_r = Br[kk * SB + j];
        if constexpr (AC && BC) {
          const double a_i = Ai[kk * SA + i], b_i = Bi[kk * SB + j];
          cr[t] = mfma4(a_r, b_r, cr[t]);
          ci[t] = mfma4(a_r, b_i, ci[t]);
          cr[t] = mfma4(-a_i, b_i, cr[t]);
          ci[t] = mfma4(a_i, b_r, ci[t]);
        } else if constexpr (AC) {
          const double a_i = Ai[kk * SA + i];
          cr[t] = mfma4(a_r, b_r, cr[t]);
          ci[t] = mfma4(a_i, b_r, ci[t]);
        } else if constexpr (BC) {
          const double b_i = Bi[kk * SB + j];
          cr[t] = mfma4(a_r, b_r, cr[t]);
          ci[t] = mfma4(a_r, b_i, ci[t]);
        } else {
          cr[t] = mfma4(a_r, b_r, cr[t]);
        }
      }
    }
    if (kp == npan - 1) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wave + NWAVE * t;
        if (tile >= NT) break;
        const int r0 = ((tile % TMT) << 4) + lk, c0 = ((tile / TMT) << 4) + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = bm + r0 + 4 * r, gj = bn + c0;
          if (gi < M && gj < Nc) {
            if constexpr (CC) st(gi, gj, cr[t][r], ci[t][r]);
            else st(gi, gj, cr[t][r]);
          }
        }
      }
    }
  }
  __syncthreads();
}

struct LgNoInit {
  __device__ void operator()(int, int, double&, double&) const {}
  __device__ void operator()(int, int, double&) const {}
};

template <int TM, int TN, bool AC, bool BC, class LA, class LB, class ST>
__device__ __forceinline__ void lg_gemm(int M, int Nc, int K, LA la, LB lb, ST st, double* lds) {
  lg_gemm_impl<TM, TN, AC, BC, false>(M, Nc, K, la, lb, st, LgNoInit{}, lds);
}

// C -= A B in place: the accumulators start from -C and the store negates.
template <int TM, int TN, bool AC, bool BC, class LA, class LB, class LC, class SC>
__device__ __forceinline__ void lg_gemm_sub(int M, int Nc, int K, LA la, LB lb, LC lc, SC sc,
                                            double* lds) {
  lg_gemm_impl<TM, TN, AC, BC, true>(
      M, Nc, K, la, lb,
      [&](int i, int j, double cr, double ci) { sc(i, j, -cr, -ci); },
      [&](int i, int j, double& cr, double& ci) {
        lc(i, j, cr, ci);
        cr = -cr;
        ci = -ci;
      }, lds);
}

// Reflector matrix V of the panel at j0 (pw columns): V(r, c) for rows r of
// the whole matrix, zero above row j0 + c, u0 on it, the tail below.  While
// the QR runs, position j lives in column cmap[j] of W (nullptr: column j).
struct LgPanel {
  CMat W;
  const double* u0r;
  const double* u0i;
  int j0, pw;
  const int* cmap;
  __device__ __forceinline__ void v(int r, int c, double& vr, double& vi) const {
    const int j = j0 + c;
    const int col = cmap ? cmap[j] : j;
    if (r > j) { vr = W.r(r, col); vi = W.m(r, col); }
    else if (r == j) { vr = u0r[j]; vi = u0i[j]; }
    else { vr = 0.0; vi = 0.0; }
  }
};

// Y(j0:j0+M, cols) <- (I - V T' V^H) Y for one panel, T' = T (herm false) or
// T^H (herm true); cols are ycol0 .. ycol0+Nc-1, through ymap if given.  F is
// a free complex matrix holding V^H Y, then T' V^H Y.
template <int NC>
__device__ void lg_apply_panel(const LgPanel& pn, const double* tp, CMat Y, int ycol0, int M, int Nc,
                               CMat F, bool herm, const int* ymap, SmemC<NC>& S) {
  auto ycol = [&](int j) { return ymap ? ymap[ycol0 + j] : ycol0 + j; };
  const int j0 = pn.j0, pw = pn.pw;
  // F(0:pw, 0:Nc) = V^H Y
  lg_gemm<16, 256, true, true>(
      pw, Nc, M,
      [&](int i, int k, double& ar, double& ai) {
        double vr, vi;
        pn.v(j0 + k, i, vr, vi);
        ar = vr; ai = -vi;
      },
      [&](int k, int j, double& br, double& bi) {
        const int c = ycol(j);
        br = Y.r(j0 + k, c); bi = Y.m(j0 + k, c);
      },
      [&](int i, int j, double cr, double ci) { F.r(i, j) = cr; F.m(i, j) = ci; }, S.big);
  // F <- T' F, column by column (T' is pw x pw from tp: re then im, T(i, k)
  // at [k * 16 + i])
  double* tr = S.lgt;
  double* ti = S.lgt + 256;
  for (int e = threadIdx.x; e < 256; e += WG) { tr[e] = tp[e]; ti[e] = tp[256 + e]; }
  __syncthreads();
  for (int j = threadIdx.x; j < Nc; j += WG) {
    double xr[LG_PW], xi[LG_PW];
#pragma unroll
    for (int k = 0; k < LG_PW; ++k) {
      xr[k] = k < pw ? F.r(k, j) : 0.0;
      xi[k] = k < pw ? F.m(k, j) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < LG_PW; ++i) {
      if (i >= pw) break;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int k = 0; k < LG_PW; ++k) {
        // T(i, k) (upper: k >= i) or T^H(i, k) = conj(T(k, i)) (k <= i)
        double t_r, t_i;
        if (!herm) { t_r = (k >= i) ? tr[k * 16 + i] : 0.0; t_i = (k >= i) ? ti[k * 16 + i] : 0.0; }
        else { t_r = (k <= i) ? tr[i * 16 + k] : 0.0; t_i = (k <= i) ? -ti[i * 16 + k] : 0.0; }
        sr += t_r * xr[k] - t_i * xi[k];
        si += t_r * xi[k] + t_i * xr[k];
      }
      F.r(i, j) = sr;
      F.m(i, j) = si;
    }
  }
  __syncthreads();
  // Y -= V F
  lg_gemm_sub<128, 128, true, true>(
      M, Nc, pw,
      [&](int i, int k, double& ar, double& ai) { pn.v(j0 + i, k, ar, ai); },
      [&](int k, int j, double& br, double& bi) { br = F.r(k, j); bi = F.m(k, j); },
      [&](int i, int j, double& cr, double& ci) {
        const int c = ycol(j);
        cr = Y.r(j0 + i, c);
        ci = Y.m(j0 + i, c);
      },
      [&](int i, int j, double cr, double ci) {
        const int c = ycol(j);
        Y.r(j0 + i, c) = cr;
        Y.m(j0 + i, c) = ci;
      }, S.big);
}

// Sum over the workgroup of NV values per thread; every thread receives the
// NV sums.  Two LDS buffers alternate with `buf`, so consecutive calls need
// no extra barrier.
template <int NV, int NC>
__device__ __forceinline__ void lg_block_sums(double* v, int buf, SmemC<NC>& S) {
  static_assert(NV <= 32, "at most 32 values");
  const int lane = lane_id(), wave = wave_id();
  double* part = S.lgred + buf * (NWAVE * 32);
  double* sums = S.lgsum + buf * 32;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = red16(v[k]);
    x = readlane_d(x, 0) + readlane_d(x, 16) + readlane_d(x, 32) + readlane_d(x, 48);
    if (lane == 0) part[wave * 32 + k] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) t += part[w * 32 + threadIdx.x];
    sums[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = sums[k];
}

// ---------------------------------------------------------------------------
// lg_qrp: blocked Householder QR of the N x N matrix in W with the pivot
// order (partial norm x key) refreshed at every panel.  Output as rq_qrp's
// (R in the upper triangle of W in pivoted column order, S.u0r/u0i, S.beta,
// S.piv, S.pinv, S.csp, S.rdr/rdi, S.nref) but with the reflector tails
// below the diagonal of W, plus the T factor of every panel in tst.  F is a
// free complex N x N matrix.
// ---------------------------------------------------------------------------
template <int NC>
__device__ void lg_qrp(CMat W, int N, const double* keys, CMat F, double* tst, SmemC<NC>& S) {
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  // ---- pivot order by key = |column| x keys[c], decreasing, ties to the
  // lower index (one wave per column)
  for (int c = wave; c < N; c += NWAVE) {
    double acc = 0.0;
    for (int i = lane; i < N; i += 64) {
      const double a = W.r(i, c), b = W.m(i, c);
      acc += a * a + b * b;
    }
    acc = wave_sum(acc);
    if (lane == 0) S.v3[c] = sqrt(acc) * (keys ? keys[c] : 1.0);
  }
  __syncthreads();
  for (int c = tid; c < N; c += WG) {
    const double kc = S.v3[c];
    int pos = 0;
    for (int d = 0; d < N; ++d) {
      const double kd = S.v3[d];
      pos += (kd > kc || (kd == kc && d < c)) ? 1 : 0;
    }
    S.piv[pos] = c;
    S.tmp1[pos] = c;   // position -> column of W while the QR runs
    S.csp[pos] = keys ? keys[c] : 1.0;
  }
  if (tid == 0) S.nref = 0;
  __syncthreads();
  int* cmap = S.tmp1;

  const int r = tid;   // this thread's row of every panel
  int step = 0;
  for (int j0 = 0; j0 < N; j0 += LG_PW) {
    const int pw = min(LG_PW, N - j0);
    // ---- pivot refresh: positions >= j0 by partial norm (rows >= j0) x key
    if (j0 > 0 && j0 < N - 1) {
      for (int k = j0 + wave; k < N; k += NWAVE) {
        const int c = cmap[k];
        double acc = 0.0;
        for (int i = j0 + lane; i < N; i += 64) {
          const double a = W.r(i, c), b = W.m(i, c);
          acc += a * a + b * b;
        }
        acc = wave_sum(acc);
        if (lane == 0) S.v3[k] = sqrt(acc) * S.csp[k];
      }
      __syncthreads();
      for (int k = j0 + tid; k < N; k += WG) {
        const double kk = S.v3[k];
        int pos = j0;
        for (int d = j0; d < N; ++d) {
          const double kd = S.v3[d];
          pos += (kd > kk || (kd == kk && d < k)) ? 1 : 0;
        }
        S.tmp0[pos] = k;
      }
      __syncthreads();
      for (int p = j0 + tid; p < N; p += WG) {
        const int k = S.tmp0[p];   // only this thread reads entry p
        S.pinv[p] = cmap[k];
        S.norms[p] = S.csp[k];
        S.tmp0[p] = S.piv[k];
      }
      __syncthreads();
      for (int p = j0 + tid; p < N; p += WG) {
        cmap[p] = S.pinv[p];
        S.csp[p] = S.norms[p];
        S.piv[p] = S.tmp0[p];
      }
      __syncthreads();
    }
    // ---- panel factorisation in registers (row r, columns j0 .. j0+pw-1)
    double pr[LG_PW], pi[LG_PW];
#pragma unroll
    for (int c = 0; c < LG_PW; ++c) {
      const bool in = r >= j0 && r < N && c < pw;
      pr[c] = in ? W.r(r, cmap[j0 + min(c, pw - 1)]) : 0.0;
      pi[c] = in ? W.m(r, cmap[j0 + min(c, pw - 1)]) : 0.0;
    }
    static_for<0, LG_PW>([&](auto jc) {
      constexpr int JJ = decltype(jc)::value;
      if (JJ >= pw) return;
      const int j = j0 + JJ;
      const int buf = step & 1;
      ++step;
      // row j of the panel, for the terms of row j in the sums below
      double* rowj = S.lgrow + buf * 32;
      if (r == j) {
#pragma unroll
        for (int c = JJ; c < LG_PW; ++c) { rowj[c] = pr[c]; rowj[16 + c] = pi[c]; }
      }
      // sums over rows below j: |a_jj|^2 and conj(a_jj) a_c for c > JJ
      constexpr int NV = 1 + 2 * (LG_PW - 1 - JJ);
      double v[NV];
      const bool below = r > j && r < N;
      v[0] = below ? pr[JJ] * pr[JJ] + pi[JJ] * pi[JJ] : 0.0;
#pragma unroll
      for (int c = JJ + 1; c < LG_PW; ++c) {
        const int q = 1 + 2 * (c - JJ - 1);
        v[q] = below ? pr[JJ] * pr[c] + pi[JJ] * pi[c] : 0.0;
        v[q + 1] = below ? pr[JJ] * pi[c] - pi[JJ] * pr[c] : 0.0;
      }
      lg_block_sums<NV>(v, buf, S);
      const double a0r = rowj[JJ], a0i = rowj[16 + JJ];
      const double aa0 = sqrt(a0r * a0r + a0i * a0i);
      const double alpha = sqrt(v[0] + aa0 * aa0);
      double er = 1.0, ei = 0.0;
      if (aa0 > 0.0) { const double inv = 1.0 / aa0; er = a0r * inv; ei = a0i * inv; }
      const bool refl = alpha > 0.0;
      const double beta = refl ? 1.0 / (alpha * (alpha + aa0)) : 0.0;
      const double u0r = refl ? a0r + er * alpha : 0.0, u0i = refl ? a0i + ei * alpha : 0.0;
      // apply H_j to the panel columns c > JJ: a_c -= beta u (u^H a_c),
      // u^H a_c = (sum over rows below j) + conj(u0) a_jc
      const double ur = (r == j) ? u0r : ((r > j && r < N) ? pr[JJ] : 0.0);
      const double ui = (r == j) ? u0i : ((r > j && r < N) ? pi[JJ] : 0.0);
#pragma unroll
      for (int c = JJ + 1; c < LG_PW; ++c) {
        const int q = 1 + 2 * (c - JJ - 1);
        const double ajr = rowj[c], aji = rowj[16 + c];
        const double dr = v[q] + u0r * ajr + u0i * aji;
        const double di = v[q + 1] + u0r * aji - u0i * ajr;
        const double wr = beta * dr, wi = beta * di;
        pr[c] -= ur * wr - ui * wi;
        pi[c] -= ur * wi + ui * wr;
      }
      if (r == j) {
        pr[JJ] = refl ? -er * alpha : 0.0;
        pi[JJ] = refl ? -ei * alpha : 0.0;
      }
      if (tid == 0) {
        S.rdr[j] = refl ? -er * alpha : 0.0;
        S.rdi[j] = refl ? -ei * alpha : 0.0;
        S.u0r[j] = u0r;
        S.u0i[j] = u0i;
        S.beta[j] = beta;
        if (refl) S.nref += 1;
      }
    });
    // ---- panel back to W (rows >= j0)
    if (r >= j0 && r < N) {
#pragma unroll
      for (int c = 0; c < LG_PW; ++c) {
        if (c < pw) { W.r(r, cmap[j0 + c]) = pr[c]; W.m(r, cmap[j0 + c]) = pi[c]; }
      }
    }
    __syncthreads();
    const LgPanel pn{W, S.u0r, S.u0i, j0, pw, cmap};
    // ---- T factor: Gm = V^H V on the matrix cores (rows split over the
    // waves), then T(jj, jj) = beta_jj, T(0:jj, jj) = -beta_jj T(0:jj, 0:jj)
    // Gm(0:jj, jj)
    {
      const int li = lane & 15, lk = lane >> 4;
      v4d gr = {0.0, 0.0, 0.0, 0.0}, gi = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = j0 + 4 * wave; k0 < N; k0 += 4 * NWAVE) {
        const int row = k0 + lk;
        double vr = 0.0, vi = 0.0;
        if (row < N && li < pw) pn.v(row, li, vr, vi);
        // A = V^H (i = li, k = row), B = V (k = row, j = li)
        gr = mfma4(vr, vr, gr);
        gr = mfma4(vi, vi, gr);
        gi = mfma4(vr, vi, gi);
        gi = mfma4(-vi, vr, gi);
      }
      double* part = S.big;   // 8 waves x (re 256, im 256)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lk + 4 * q, jcol = li;
        part[wave * 512 + jcol * 16 + i] = gr[q];
        part[wave * 512 + 256 + jcol * 16 + i] = gi[q];
      }
      __syncthreads();
      double* gmr = S.lgt + 512;
      double* gmi = S.lgt + 768;
      if (tid < 256) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int w = 0; w < NWAVE; ++w) { sr += part[w * 512 + tid]; si += part[w * 512 + 256 + tid]; }
        gmr[tid] = sr;
        gmi[tid] = si;
      }
      double* tr = S.lgt;
      double* ti = S.lgt + 256;
      if (tid < 256) { tr[tid] = 0.0; ti[tid] = 0.0; }
      __syncthreads();
      for (int jj = 0; jj < pw; ++jj) {
        const double bj = S.beta[j0 + jj];
        if (tid < jj) {
          // T(i, jj) = -beta sum_{k=i}^{jj-1} T(i, k) Gm(k, jj)
          const int i = tid;
          double sr = 0.0, si = 0.0;
          for (int k = i; k < jj; ++k) {
            const double a_r = tr[k * 16 + i], a_i = ti[k * 16 + i];
            const double b_r = gmr[jj * 16 + k], b_i = gmi[jj * 16 + k];
            sr += a_r * b_r - a_i * b_i;
            si += a_r * b_i + a_i * b_r;
          }
          tr[jj * 16 + i] = -bj * sr;
          ti[jj * 16 + i] = -bj * si;
        }
        if (tid == jj) { tr[jj * 16 + jj] = bj; ti[jj * 16 + jj] = 0.0; }
        __syncthreads();
      }
      double* tp = tst + (size_t)(j0 / LG_PW) * LG_TDBL;
      if (tid < 256) { tp[tid] = tr[tid]; tp[256 + tid] = ti[tid]; }
      __syncthreads();
    }
    // ---- trailing columns: A <- (I - V T^H V^H) A, A = W(j0:N, j0+pw:N)
    const int nt = N - j0 - pw;
    if (nt > 0) {
      const double* tp = tst + (size_t)(j0 / LG_PW) * LG_TDBL;
      lg_apply_panel<NC>(pn, tp, W, j0 + pw, N - j0, nt, F, true, cmap, S);
    }
  }
  // ---- columns into position order (through F)
  for (int idx = tid; idx < N * N; idx += WG) {
    const int i = idx % N, k = idx / N;
    const int c = cmap[k];
    F.r(i, k) = W.r(i, c);
    F.m(i, k) = W.m(i, c);
  }
  __syncthreads();
  for (int idx = tid; idx < N * N; idx += WG) {
    const int i = idx % N, k = idx / N;
    W.r(i, k) = F.r(i, k);
    W.m(i, k) = F.m(i, k);
  }
  for (int c = tid; c < N; c += WG) S.pinv[S.piv[c]] = c;
  __syncthreads();
}

// Reflectors per block of the aggregated applications below (four panels).
constexpr int LG_NB = 64;

// Y(j0:j0+M, ycol0:ycol0+Nc) <- (I - V T' V^H) Y for the block of reflectors
// j0 .. j0+pw-1 (pw <= LG_NB) as one compact WY product, T' = T (herm false)
// or T^H (herm true): rank-pw updates instead of one rank-16 pass per panel,
// so Y is read and written once per 64 reflectors.  T follows from the
// block's Gram matrix G = V^H V column by column, T(j, j) = beta_j and
// T(0:j, j) = -beta_j T(0:j, 0:j) G(0:j, j) (the recurrence of the panel T
// factors, over 64 columns).  Scratch: the raw storage of the free matrix F
// (2 Np^2 doubles, at least 128 Np + 16384 for Np >= 144): V^H Y and then
// T' V^H Y at ld 64, T' and G (64 x 64 each, re then im).
// T' of the block (pw x pw at ld 64, re then im, at F.re + 2 * 64 * Np) from
// the Gram matrix of its M rows of V, as described above.
template <int NC>
__device__ __forceinline__ void lg_block_t(const LgPanel& pn, int M, CMat F, bool herm, SmemC<NC>& S) {
  const int j0 = pn.j0, pw = pn.pw, Np = F.ld;
  double* tgr = F.re + (size_t)2 * LG_NB * Np;
  double* tgi = tgr + LG_NB * LG_NB;
  double* ggr = tgi + LG_NB * LG_NB;
  double* ggi = ggr + LG_NB * LG_NB;
  auto vh = [&](int i, int k, double& ar, double& ai) {   // V^H (i, k) = conj V(j0 + k, i)
    double vr, vi;
    pn.v(j0 + k, i, vr, vi);
    ar = vr;
    ai = -vi;
  };
  // G = V^H V
  lg_gemm<64, 64, true, true>(
      pw, pw, M, vh, [&](int k, int j, double& br, double& bi) { pn.v(j0 + k, j, br, bi); },
      [&](int i, int j, double cr, double ci) {
        ggr[j * LG_NB + i] = cr;
        ggi[j * LG_NB + i] = ci;
      }, S.big);
  // T by columns in LDS (the staging area is free between products)
  double* tr = S.big;
  double* ti = S.big + LG_NB * LG_NB;
  for (int e = threadIdx.x; e < LG_NB * LG_NB; e += WG) { tr[e] = 0.0; ti[e] = 0.0; }
  __syncthreads();
  // column j of G staged in LDS (two buffers, so one barrier per column)
  double* gcol = S.lgt;
  if (threadIdx.x < pw) {
    gcol[threadIdx.x] = ggr[threadIdx.x];
    gcol[LG_NB + threadIdx.x] = ggi[threadIdx.x];
  }
  __syncthreads();
  for (int j = 0; j < pw; ++j) {
    const double bj = S.beta[j0 + j];
    const double* gc = gcol + (j & 1) * 2 * LG_NB;
    double* gn = gcol + ((j + 1) & 1) * 2 * LG_NB;
    if (j + 1 < pw && threadIdx.x >= 256 && threadIdx.x - 256 < pw) {
      const int k = threadIdx.x - 256;
      gn[k] = ggr[(j + 1) * LG_NB + k];
      gn[LG_NB + k] = ggi[(j + 1) * LG_NB + k];
    }
    if (threadIdx.x < j) {
      const int i = threadIdx.x;
      double sr = 0.0, si = 0.0;
      for (int k = i; k < j; ++k) {
        const double a_r = tr[k * LG_NB + i], a_i = ti[k * LG_NB + i];
        const double b_r = gc[k], b_i = gc[LG_NB + k];
        sr += a_r * b_r - a_i * b_i;
        si += a_r * b_i + a_i * b_r;
      }
      tr[j * LG_NB + i] = -bj * sr;
      ti[j * LG_NB + i] = -bj * si;
    }
    if (threadIdx.x == j) { tr[j * LG_NB + j] = bj; ti[j * LG_NB + j] = 0.0; }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < LG_NB * LG_NB; e += WG) {
    const int i = e % LG_NB, k = e / LG_NB;
    if (!herm) { tgr[e] = tr[e]; tgi[e] = ti[e]; }
    else { tgr[e] = tr[i * LG_NB + k]; tgi[e] = -ti[i * LG_NB + k]; }
  }
  __syncthreads();
}

template <int NC>
__device__ void lg_apply_block(const LgPanel& pn, CMat Y, int ycol0, int M, int Nc, CMat F,
                               bool herm, SmemC<NC>& S) {
  const int j0 = pn.j0, pw = pn.pw, Np = F.ld;
  double* f0r = F.re;
  double* f0i = F.re + (size_t)LG_NB * Np;
  const double* tgr = F.re + (size_t)2 * LG_NB * Np;
  const double* tgi = tgr + LG_NB * LG_NB;
  auto vh = [&](int i, int k, double& ar, double& ai) {   // V^H (i, k) = conj V(j0 + k, i)
    double vr, vi;
    pn.v(j0 + k, i, vr, vi);
    ar = vr;
    ai = -vi;
  };
  lg_block_t<NC>(pn, M, F, herm, S);
  // F = V^H Y
  lg_gemm<64, 128, true, true>(
      pw, Nc, M, vh,
      [&](int k, int j, double& br, double& bi) {
        br = Y.r(j0 + k, ycol0 + j);
        bi = Y.m(j0 + k, ycol0 + j);
      },
      [&](int i, int j, double cr, double ci) {
        f0r[(size_t)j * LG_NB + i] = cr;
        f0i[(size_t)j * LG_NB + i] = ci;
      }, S.big);
  // F <- T' F in place: one macro tile holds all pw rows, and each tile's
  // columns of F are in registers before the tile is stored
  lg_gemm<64, 128, true, true>(
      pw, Nc, pw,
      [&](int i, int k, double& ar, double& ai) {
        ar = tgr[k * LG_NB + i];
        ai = tgi[k * LG_NB + i];
      },
      [&](int k, int j, double& br, double& bi) {
        br = f0r[(size_t)j * LG_NB + k];
        bi = f0i[(size_t)j * LG_NB + k];
      },
      [&](int i, int j, double cr, double ci) {
        f0r[(size_t)j * LG_NB + i] = cr;
        f0i[(size_t)j * LG_NB + i] = ci;
      }, S.big);
  // Y -= V F
  lg_gemm_sub<128, 128, true, true>(
      M, Nc, pw, [&](int i, int k, double& ar, double& ai) { pn.v(j0 + i, k, ar, ai); },
      [&](int k, int j, double& br, double& bi) {
        br = f0r[(size_t)j * LG_NB + k];
        bi = f0i[(size_t)j * LG_NB + k];
      },
      [&](int i, int j, double& cr, double& ci) {
        cr = Y.r(j0 + i, ycol0 + j);
        ci = Y.m(j0 + i, ycol0 + j);
      },
      [&](int i, int j, double cr, double ci) {
        Y.r(j0 + i, ycol0 + j) = cr;
        Y.m(j0 + i, ycol0 + j) = ci;
      }, S.big);
}

// Y(0:M, j0:N) <- Y(0:M, j0:N) (I - V T V^H) for the block of reflectors
// j0 .. j0+pw-1: Z = Y V (M x pw at ld Np in the free matrix), Z <- Z T in
// place (one macro tile holds all pw columns of its rows), Y -= Z V^H.  The
// scratch is that of lg_apply_block.
template <int NC>
__device__ void lg_apply_block_right(const LgPanel& pn, CMat Y, int M, int N, CMat F,
                                     SmemC<NC>& S) {
  const int j0 = pn.j0, pw = pn.pw, Np = F.ld;
  double* zr = F.re;
  double* zi = F.re + (size_t)LG_NB * Np;
  const double* tgr = F.re + (size_t)2 * LG_NB * Np;
  const double* tgi = tgr + LG_NB * LG_NB;
  lg_block_t<NC>(pn, N - j0, F, false, S);
  // Z = Y(:, j0:N) V
  lg_gemm<128, 64, true, true>(
      M, pw, N - j0,
      [&](int i, int k, double& ar, double& ai) { ar = Y.r(i, j0 + k); ai = Y.m(i, j0 + k); },
      [&](int k, int j, double& br, double& bi) { pn.v(j0 + k, j, br, bi); },
      [&](int i, int j, double cr, double ci) {
        zr[(size_t)j * Np + i] = cr;
        zi[(size_t)j * Np + i] = ci;
      }, S.big);
  // Z <- Z T
  lg_gemm<128, 64, true, true>(
      M, pw, pw,
      [&](int i, int k, double& ar, double& ai) {
        ar = zr[(size_t)k * Np + i];
        ai = zi[(size_t)k * Np + i];
      },
      [&](int k, int j, double& br, double& bi) {
        br = tgr[j * LG_NB + k];
        bi = tgi[j * LG_NB + k];
      },
      [&](int i, int j, double cr, double ci) {
        zr[(size_t)j * Np + i] = cr;
        zi[(size_t)j * Np + i] = ci;
      }, S.big);
  // Y(:, j0:N) -= Z V^H
  lg_gemm_sub<128, 128, true, true>(
      M, N - j0, pw,
      [&](int i, int k, double& ar, double& ai) {
        ar = zr[(size_t)k * Np + i];
        ai = zi[(size_t)k * Np + i];
      },
      [&](int k, int j, double& br, double& bi) {
        double vr, vi;
        pn.v(j0 + j, k, vr, vi);
        br = vr;
        bi = -vi;
      },
      [&](int i, int j, double& cr, double& ci) {
        cr = Y.r(i, j0 + j);
        ci = Y.m(i, j0 + j);
      },
      [&](int i, int j, double cr, double ci) {
        Y.r(i, j0 + j) = cr;
        Y.m(i, j0 + j) = ci;
      }, S.big);
}

// Whether the free matrix of padded size Np holds lg_apply_block's scratch
// (Np >= 144, i.e. every N > 128; smaller problems that run this class's
// code inside a batch use one rank-16 pass per panel instead).
__device__ __forceinline__ bool lg_block_fits(int Np) {
  return (size_t)2 * LG_NB * Np + (size_t)4 * LG_NB * LG_NB <= (size_t)2 * Np * Np;
}

// Q = H_0 ... H_{N-1} explicitly into Q: backward over blocks of 64
// reflectors (or of 16, see lg_block_fits), each acting on Q(j0:N, j0:N)
// (columns left of j0 are still unit vectors there, on which the block acts
// as the identity).
template <int NC>
__device__ void lg_form_q(CMat W, int N, CMat Q, CMat F, const double* tst, SmemC<NC>& S) {
  for (int idx = threadIdx.x; idx < N * N; idx += WG) {
    const int i = idx % N, c = idx / N;
    Q.r(i, c) = (i == c) ? 1.0 : 0.0;
    Q.m(i, c) = 0.0;
  }
  __syncthreads();
  if (lg_block_fits(F.ld)) {
    const int nb = (N + LG_NB - 1) / LG_NB;
    for (int b = nb - 1; b >= 0; --b) {
      const int j0 = b * LG_NB, pw = min(LG_NB, N - j0);
      const LgPanel pn{W, S.u0r, S.u0i, j0, pw, nullptr};
      lg_apply_block<NC>(pn, Q, j0, N - j0, N - j0, F, false, S);
    }
  } else {
    const int np = (N + LG_PW - 1) / LG_PW;
    for (int p = np - 1; p >= 0; --p) {
      const int j0 = p * LG_PW, pw = min(LG_PW, N - j0);
      const LgPanel pn{W, S.u0r, S.u0i, j0, pw, nullptr};
      lg_apply_panel<NC>(pn, tst + (size_t)p * LG_TDBL, Q, j0, N - j0, N - j0, F, false, nullptr, S);
    }
  }
}

// Y <- Q^H Y (all N columns), forward over the blocks of lg_form_q.
template <int NC>
__device__ void lg_apply_qh(CMat W, int N, CMat Y, CMat F, const double* tst, SmemC<NC>& S) {
  if (lg_block_fits(F.ld)) {
    const int nb = (N + LG_NB - 1) / LG_NB;
    for (int b = 0; b < nb; ++b) {
      const int j0 = b * LG_NB, pw = min(LG_NB, N - j0);
      const LgPanel pn{W, S.u0r, S.u0i, j0, pw, nullptr};
      lg_apply_block<NC>(pn, Y, 0, N - j0, N, F, true, S);
    }
  } else {
    const int np = (N + LG_PW - 1) / LG_PW;
    for (int p = 0; p < np; ++p) {
      const int j0 = p * LG_PW, pw = min(LG_PW, N - j0);
      const LgPanel pn{W, S.u0r, S.u0i, j0, pw, nullptr};
      lg_apply_panel<NC>(pn, tst + (size_t)p * LG_TDBL, Y, 0, N - j0, N, F, true, nullptr, S);
    }
  }
}

// Y <- Y Q (M rows, all N columns; Q = H_0 ... H_{N-1} of the factor in W),
// forward over the blocks of lg_form_q: 8 M N^2 flops instead of forming Q
// (16/3 N^3) and multiplying by it (8 M N^2).  Requires lg_block_fits(F.ld).
template <int NC>
__device__ void lg_right_apply_q(CMat W, int N, CMat Y, int M, CMat F, SmemC<NC>& S) {
  const int nb = (N + LG_NB - 1) / LG_NB;
  for (int b = 0; b < nb; ++b) {
    const int j0 = b * LG_NB, pw = min(LG_NB, N - j0);
    const LgPanel pn{W, S.u0r, S.u0i, j0, pw, nullptr};
    lg_apply_block_right<NC>(pn, Y, M, N, F, S);
  }
}

// Y <- R^{-1} Y for the upper triangle R of W, by blocks of 16 rows from the
// bottom: solve the diagonal block per column, then remove the block's
// contribution from the rows above with one product.
template <int NC>
__device__ void lg_backsolve(CMat W, int N, CMat Y, SmemC<NC>& S) {
  const int tid = threadIdx.x;
  double* rr = S.lgt;          // R block, column-major 16 x 16
  double* ri = S.lgt + 256;
  const int nb = (N + LG_PW - 1) / LG_PW;
  for (int b = nb - 1; b >= 0; --b) {
    const int i0 = b * LG_PW, bw = min(LG_PW, N - i0);
    if (tid < 256) {
      const int i = tid % 16, k = tid / 16;
      const bool in = i < bw && k < bw && i <= k;
      rr[tid] = in ? W.r(i0 + i, i0 + k) : 0.0;
      ri[tid] = in ? W.m(i0 + i, i0 + k) : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < N; c += WG) {
      double yr[LG_PW], yi[LG_PW];
#pragma unroll
      for (int k = 0; k < LG_PW; ++k) {
        yr[k] = k < bw ? Y.r(i0 + k, c) : 0.0;
        yi[k] = k < bw ? Y.m(i0 + k, c) : 0.0;
      }
#pragma unroll
      for (int i = LG_PW - 1; i >= 0; --i) {
        if (i >= bw) continue;
        double sr = yr[i], si = yi[i];
#pragma unroll
        for (int k = i + 1; k < LG_PW; ++k) {
          const double a_r = rr[k * 16 + i], a_i = ri[k * 16 + i];
          sr -= a_r * yr[k] - a_i * yi[k];
          si -= a_r * yi[k] + a_i * yr[k];
        }
        const double dr = rr[i * 16 + i], di = ri[i * 16 + i];
        const double den = dr * dr + di * di;
        yr[i] = (sr * dr + si * di) / den;
        yi[i] = (si * dr - sr * di) / den;
      }
#pragma unroll
      for (int k = 0; k < LG_PW; ++k) {
        if (k < bw) { Y.r(i0 + k, c) = yr[k]; Y.m(i0 + k, c) = yi[k]; }
      }
    }
    __syncthreads();
    if (i0 > 0) {
      lg_gemm_sub<128, 128, true, true>(
          i0, N, bw,
          [&](int i, int k, double& ar, double& ai) { ar = W.r(i, i0 + k); ai = W.m(i, i0 + k); },
          [&](int k, int j, double& br, double& bi) { br = Y.r(i0 + k, j); bi = Y.m(i0 + k, j); },
          [&](int i, int j, double& cr, double& ci) { cr = Y.r(i, j); ci = Y.m(i, j); },
          [&](int i, int j, double cr, double ci) { Y.r(i, j) = cr; Y.m(i, j) = ci; }, S.big);
    }
  }
}

}  // namespace fdet

// Molecular dynamics of HMC (Sec. 3.1) on gfx950: the leapfrog updates of
// the momenta pi and the fields phi, and the Hamiltonian of the accept step,
//   H = 1/2 sum pi^2 + sum phi^2 / (2 dU) - 2 Re log det M(phi)
// (two fermion flavours whose determinants are complex conjugates, and the
// Gaussian weight of the auxiliary field), whose phi-derivative is
//   dH/dphi = phi / dU - 2 Re F,  F = d log det M / d phi.
// Every update is elementwise over the N_t x N field (HBM-bound, coalesced);
// the energy sums are one workgroup per field in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdet_hmc.h"

namespace {

using fdet::HmcProb;

constexpr int HWG = 256;
constexpr int HWAVE = HWG / 64;

// pi <- pi - h (phi / dU - 2 force)
__global__ __launch_bounds__(HWG) void k_hmc_kick(const HmcProb* __restrict__ hp,
                                                  double* __restrict__ pi,
                                                  const double* __restrict__ force, double dU,
                                                  double h) {
  const HmcProb q = hp[blockIdx.y];
  const double r = 1.0 / dU;
  for (int64_t k = (int64_t)blockIdx.x * HWG + threadIdx.x; k < q.n; k += (int64_t)gridDim.x * HWG) {
    const int64_t g = q.off + k;
    pi[g] -= h * (q.phi[k] * r - 2.0 * force[g]);
  }
}

// phi <- phi + eps pi
__global__ __launch_bounds__(HWG) void k_hmc_drift(const HmcProb* __restrict__ hp,
                                                   const double* __restrict__ pi, double eps) {
  const HmcProb q = hp[blockIdx.y];
  for (int64_t k = (int64_t)blockIdx.x * HWG + threadIdx.x; k < q.n; k += (int64_t)gridDim.x * HWG)
    q.phi[k] += eps * pi[q.off + k];
}

// H of field blockIdx.x; mode 0 stores it in H0, mode 1 writes dH = H - H0.
__global__ __launch_bounds__(HWG) void k_hmc_energy(const HmcProb* __restrict__ hp,
                                                    const double* __restrict__ pi,
                                                    const double* __restrict__ logdet, double dU,
                                                    double* __restrict__ H0,
                                                    double* __restrict__ dH, int mode) {
  __shared__ double red[2][HWAVE];
  const int f = blockIdx.x;
  const HmcProb q = hp[f];
  double sp = 0.0, sf = 0.0;
  for (int64_t k = threadIdx.x; k < q.n; k += HWG) {
    const double a = pi[q.off + k], b = q.phi[k];
    sp = fma(a, a, sp);
    sf = fma(b, b, sf);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sp += __shfl_xor(sp, o, 64);
    sf += __shfl_xor(sf, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sp;
    red[1][threadIdx.x >> 6] = sf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < HWAVE; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    const double H = 0.5 * a + 0.5 * b / dU - 2.0 * logdet[2 * f];
    if (mode == 0) H0[f] = H;
    else dH[f] = H - H0[f];
  }
}

// acc <- step (mode 0) or the worse of the two (errors < 0 before warnings > 0)
__global__ __launch_bounds__(HWG) void k_hmc_status(int nprob, const int32_t* __restrict__ step,
                                                    int32_t* __restrict__ acc, int mode) {
  const int i = blockIdx.x * HWG + threadIdx.x;
  if (i >= nprob) return;
  const int32_t s = step[i];
  if (mode == 0) {
    acc[i] = s;
    return;
  }
  const int32_t a = acc[i];
  acc[i] = (a < 0 || s < 0) ? (a < s ? a : s) : (a > s ? a : s);
}

}  // namespace

// op 0: kick, 1: drift, 2: energy (mode 0 / 1), 3: status fold (mode 0 / 1).
// hp holds nprob descriptors in device memory; maxn is the largest n among
// them.  The host checks every size and pointer before the first launch.
extern "C" hipError_t fdet_launch_hmc(int op, const HmcProb* hp, int nprob, int64_t maxn,
                                      double* pi, const double* force, const double* logdet,
                                      double dU, double h, double* H0, double* dH,
                                      const int32_t* st_step, int32_t* st_acc, int mode,
                                      hipStream_t st) {
  const int64_t blocks = (maxn + HWG - 1) / HWG;
  const dim3 grid((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024), (unsigned)nprob);
  switch (op) {
    case 0:
      hipLaunchKernelGGL(k_hmc_kick, grid, dim3(HWG), 0, st, hp, pi, force, dU, h);
      break;
    case 1:
      hipLaunchKernelGGL(k_hmc_drift, grid, dim3(HWG), 0, st, hp, pi, h);
      break;
    case 2:
      hipLaunchKernelGGL(k_hmc_energy, dim3((unsigned)nprob), dim3(HWG), 0, st, hp, pi, logdet, dU,
                         H0, dH, mode);
      break;
    case 3:
      hipLaunchKernelGGL(k_hmc_status, dim3((unsigned)((nprob + HWG - 1) / HWG)), dim3(HWG), 0, st,
                         nprob, st_step, st_acc, mode);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Observables of the paper's two applications (Sec. 3) and their adjoints.
//
// Baryon power spectrum: the half spectrum X of the gas density (forward unnormalised FFT,
// layout spec[(kz n + ky) nh + kx], nh = n/2 + 1) is binned by the rounded integer
// wavenumber |m| (bin b holds |m| in [b + 1/2, b + 3/2)); a mode of the planes kx = 0 and
// kx = n/2 stands for itself (its conjugate is stored too), every other one for itself and its
// conjugate (weight 2).  Block sums are formed per bin in a fixed order (no atomics), so the
// spectrum is reproducible bit for bit.
//
// Field-level inference: observable O = (rho / rho_mean_gas) T, loss
// 1/2 sum (d - O)^2 / N + 1/2 sum w^2 over the cells and white-noise values w.  T follows the
// dual-energy selection of dh_common.h for a state with the entropy (NQ = 6).
#include <cmath>

#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kPkThreads = 256;
constexpr int kPkPer = 8;                       // modes per thread
constexpr int kPkModes = kPkThreads * kPkPer;   // modes per block
constexpr int kObsThreads = 256;
constexpr int kObsPer = 8;

// rounded |m| of the mode (kx, ky, kz) of the half spectrum, exact in integers
__device__ __forceinline__ int mode_radius(int kx, int ky, int kz, int n) {
  const int my = ky <= n / 2 ? ky : ky - n;
  const int mz = kz <= n / 2 ? kz : kz - n;
  const int m2 = kx * kx + my * my + mz * mz;
  int j = static_cast<int>(sqrtf(static_cast<float>(m2)) + 0.5f);
  if (4 * m2 >= (2 * j + 1) * (2 * j + 1)) ++j;
  if (j > 0 && 4 * m2 < (2 * j - 1) * (2 * j - 1)) --j;
  return j;
}

// partial[(s nbins + b) nblk + block] = sum over the block's modes of bin b of w |X|^2
__global__ void __launch_bounds__(kPkThreads) pk_bin_kernel(const float2* __restrict__ spec,
                                                             int n, int nbins, long long nck,
                                                             double* __restrict__ partial) {
  __shared__ short sbin[kPkModes];
  __shared__ double sval[kPkModes];
  const int nh = n / 2 + 1;
  spec += blockIdx.y * nck;
  const long long base = static_cast<long long>(blockIdx.x) * kPkModes;
  for (int r = 0; r < kPkPer; ++r) {
    const int i = r * kPkThreads + threadIdx.x;
    const long long m = base + i;
    short bin = -1;
    double v = 0.0;
    if (m < nck) {
      const int kx = static_cast<int>(m % nh);
      const long long row = m / nh;
      const int ky = static_cast<int>(row % n), kz = static_cast<int>(row / n);
      const int j = mode_radius(kx, ky, kz, n);
      if (j >= 1 && j <= nbins) {
        const float2 x = spec[m];
        const double w = (kx == 0 || kx == n / 2) ? 1.0 : 2.0;
        v = w * (static_cast<double>(x.x) * x.x + static_cast<double>(x.y) * x.y);
        bin = static_cast<short>(j - 1);
      }
    }
    sbin[i] = bin;
    sval[i] = v;
  }
  __syncthreads();
  const long long nblk = gridDim.x;
  for (int b = threadIdx.x; b < nbins; b += kPkThreads) {
    double acc = 0.0;
    for (int i = 0; i < kPkModes; ++i)
      if (sbin[i] == b) acc += sval[i];
    partial[(static_cast<long long>(blockIdx.y) * nbins + b) * nblk + blockIdx.x] = acc;
  }
}

// spec[m] *= g[s][bin(m)] (0 outside the bins): the adjoint's spectral weights
__global__ void __launch_bounds__(256) pk_scale_kernel(float2* __restrict__ spec,
                                                       const float* __restrict__ g, int n,
                                                       int nbins, long long nck) {
  const long long m = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= nck) return;
  spec += blockIdx.y * nck;
  g += static_cast<long long>(blockIdx.y) * nbins;
  const int nh = n / 2 + 1;
  const int kx = static_cast<int>(m % nh);
  const long long row = m / nh;
  const int j = mode_radius(kx, static_cast<int>(row % n), static_cast<int>(row / n), n);
  const float f = (j >= 1 && j <= nbins) ? g[j - 1] : 0.0f;
  const float2 x = spec[m];
  spec[m] = make_float2(x.x * f, x.y * f);
}

// observable O of one cell (FP64) and its partial derivatives in Q
struct ObsCell {
  double o, d[6];
};

template <int NQ = 5>
__device__ __forceinline__ ObsCell obs_cell(const float* q, long long c, long long nc, double a,
                                            double irm, double efloor, double t_per_e,
                                            double gamma = 0.0) {
  const double rho = q[c], ir = 1.0 / rho, ia2 = 1.0 / (a * a);
  const double m0 = q[nc + c], m1 = q[2 * nc + c], m2 = q[3 * nc + c], et = q[4 * nc + c];
  const double msq = m0 * m0 + m1 * m1 + m2 * m2;
  // rho e = Et / a^2 - |m|^2 / (2 a^2 rho)
  const double e = et * ia2 * ir - 0.5 * msq * ia2 * ir * ir;
  ObsCell r;
  r.d[5] = 0.0;
  const double k = irm * t_per_e;
  if (NQ == 6) {
    const float v[5] = {q[c], q[nc + c], q[2 * nc + c], q[3 * nc + c], q[4 * nc + c]};
    if (!dual_total_branch(v)) {
      // rho e = S rho^(gamma-1) / a^2
      const double sv = q[5 * nc + c], rg = pow(rho, gamma - 1.0);
      const double es = sv * ia2 * rg * ir;
      if (es >= efloor) {
        r.o = k * sv * ia2 * rg;
        r.d[0] = k * (gamma - 1.0) * sv * ia2 * rg * ir;
        r.d[1] = r.d[2] = r.d[3] = r.d[4] = 0.0;
        r.d[5] = k * ia2 * rg;
      } else {
        r.o = k * rho * efloor;
        r.d[0] = k * efloor;
        r.d[1] = r.d[2] = r.d[3] = r.d[4] = 0.0;
      }
      return r;
    }
  }
  if (e >= efloor) {
    r.o = k * (et * ia2 - 0.5 * msq * ia2 * ir);
    r.d[0] = k * 0.5 * msq * ia2 * ir * ir;
    r.d[1] = -k * m0 * ia2 * ir;
    r.d[2] = -k * m1 * ia2 * ir;
    r.d[3] = -k * m2 * ia2 * ir;
    r.d[4] = k * ia2;
  } else {
    r.o = k * rho * efloor;
    r.d[0] = k * efloor;
    r.d[1] = r.d[2] = r.d[3] = r.d[4] = 0.0;
  }
  return r;
}

__device__ void obs_block_store(double v, double* out) {
  __shared__ double sh[kObsThreads];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kObsThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// partial[s nblk + block]: sum of 1/2 (d - O)^2 / N + 1/2 w^2 over the block's cells; with
// lam (the adjoint pass) lam[s][5][nc] = dL/dQ of the data term
template <int NQ>
__global__ void __launch_bounds__(kObsThreads) fli_kernel(
    const float* __restrict__ q, const float* __restrict__ data, const float* __restrict__ nvar,
    const float* __restrict__ white, const double* __restrict__ a_cur, double irm, double efloor,
    double t_per_e, double gamma, long long nc, double* __restrict__ partial,
    float* __restrict__ lam) {
  const int smp = blockIdx.y;
  q += smp * NQ * nc;
  data += smp * nc;
  nvar += smp * nc;
  white += smp * nc;
  if (lam) lam += smp * NQ * nc;
  const double a = a_cur[smp];
  double acc = 0.0;
  const long long base = static_cast<long long>(blockIdx.x) * kObsThreads * kObsPer;
  for (int r = 0; r < kObsPer; ++r) {
    const long long c = base + r * kObsThreads + threadIdx.x;
    if (c >= nc) break;
    const ObsCell oc = obs_cell<NQ>(q, c, nc, a, irm, efloor, t_per_e, gamma);
    const double resid = static_cast<double>(data[c]) - oc.o;
    const double inv = 1.0 / static_cast<double>(nvar[c]);
    const double w = white[c];
    acc += 0.5 * resid * resid * inv + 0.5 * w * w;
    if (lam) {
      const double g = -resid * inv;   // dL/dO
#pragma unroll
      for (int k = 0; k < NQ; ++k) lam[k * nc + c] = static_cast<float>(g * oc.d[k]);
    }
  }
  if (partial) obs_block_store(acc, partial + static_cast<long long>(smp) * gridDim.x);
}

template <int NQ>
__global__ void __launch_bounds__(256) fli_obs_kernel(const float* __restrict__ q, double a,
                                                      double irm, double efloor, double t_per_e,
                                                      double gamma, long long nc,
                                                      float* __restrict__ out) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  out[c] = static_cast<float>(obs_cell<NQ>(q, c, nc, a, irm, efloor, t_per_e, gamma).o);
}

}  // namespace

int pk_blocks(int n) {
  const long long nck = static_cast<long long>(n) * n * (n / 2 + 1);
  return static_cast<int>((nck + kPkModes - 1) / kPkModes);
}

void launch_pk_bin(hipStream_t st, const float2* spec, int nbins, double* partial,
                   const Batch& b) {
  const long long nck = static_cast<long long>(b.n) * b.n * (b.n / 2 + 1);
  if (nbins < 1 || nbins > b.n / 2) throw ArgError("power spectrum: 1 <= nbins <= n/2");
  hipLaunchKernelGGL(pk_bin_kernel, dim3(pk_blocks(b.n), b.S), dim3(kPkThreads), 0, st, spec,
                     b.n, nbins, nck, partial);
  DH_LAUNCH_CHECK();
}

void launch_pk_scale(hipStream_t st, float2* spec, const float* g, int nbins, const Batch& b) {
  const long long nck = static_cast<long long>(b.n) * b.n * (b.n / 2 + 1);
  hipLaunchKernelGGL(pk_scale_kernel, dim3(blocks_for(nck, 256), b.S), dim3(256), 0, st, spec, g,
                     b.n, nbins, nck);
  DH_LAUNCH_CHECK();
}

int fli_blocks(long long nc) {
  return static_cast<int>((nc + kObsThreads * kObsPer - 1) / (kObsThreads * kObsPer));
}

void launch_fli(hipStream_t st, const float* q, const float* data, const float* nvar,
                const float* white, const double* a_cur, double irm, double efloor,
                double t_per_e, double gamma, double* partial, float* lam, const Batch& b) {
  const dim3 grid(fli_blocks(b.nc()), b.S);
  if (b.nq == 6)
    hipLaunchKernelGGL(fli_kernel<6>, grid, dim3(kObsThreads), 0, st, q, data, nvar, white, a_cur,
                       irm, efloor, t_per_e, gamma, b.nc(), partial, lam);
  else
    hipLaunchKernelGGL(fli_kernel<5>, grid, dim3(kObsThreads), 0, st, q, data, nvar, white, a_cur,
                       irm, efloor, t_per_e, gamma, b.nc(), partial, lam);
  DH_LAUNCH_CHECK();
}

void launch_fli_obs(hipStream_t st, const float* q, double a, double irm, double efloor,
                    double t_per_e, float* out, long long nc, int nq, double gamma) {
  if (nq == 6)
    hipLaunchKernelGGL(fli_obs_kernel<6>, dim3(blocks_for(nc, 256)), dim3(256), 0, st, q, a, irm,
                       efloor, t_per_e, gamma, nc, out);
  else
    hipLaunchKernelGGL(fli_obs_kernel<5>, dim3(blocks_for(nc, 256)), dim3(256), 0, st, q, a, irm,
                       efloor, t_per_e, gamma, nc, out);
  DH_LAUNCH_CHECK();
}

}  // namespace dh

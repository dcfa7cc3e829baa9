// Learned star-formation closure: weight packing, training-set generation from the plain
// source term, batched inference, input gradients, and training (loss gradient in the
// weights on the matrix cores, deterministic reduction, Adam).  The network and its
// matrix-core layout are described in dh_mlp.h.
#include <algorithm>
#include <cmath>

#include "dh_kernels.h"
#include "dh_mlp.h"

namespace dh {

namespace {

using namespace mlp;

constexpr int kEvalThreads = 256;          // 4 waves, 64 cells each per tile
constexpr int kTrainWaves = 4;             // waves per training block (share the fragments)

// ------------------------------------------------------------------------- packing
// value of lane `lane`, slot j of fragment f (see dh_mlp.h for the fragment list)
__device__ float frag_value(const float* __restrict__ th, int f, int lane, int j) {
  const int g = lane >> 4, c = lane & 15;
  const int s = slot_unit(g, j);
  if (f < kFrW2) {                                   // W1[16 rt + c][s]
    const int row = 16 * f + c;
    return s < kIn ? th[kOffW1 + row * kIn + s] : 0.0f;
  }
  if (f < kFrW4) {                                   // W2 or W3 [16 rt + c][32 kb + s]
    const int base = f < kFrW3 ? kOffW2 : kOffW3;
    const int q = f - (f < kFrW3 ? kFrW2 : kFrW3);
    const int rt = q >> 1, kb = q & 1;
    return th[base + (16 * rt + c) * kHid + 32 * kb + s];
  }
  if (f < kFrG4) {                                   // W4[c][32 kb + s]
    const int kb = f - kFrW4;
    return c < kOut ? th[kOffW4 + c * kHid + 32 * kb + s] : 0.0f;
  }
  if (f < kFrG3) {                                   // W4^T[16 rt + c][s] = W4[s][16 rt + c]
    const int rt = f - kFrG4;
    return s < kOut ? th[kOffW4 + s * kHid + 16 * rt + c] : 0.0f;
  }
  if (f < kFrG1) {                                   // W3^T or W2^T [16 rt + c][32 kb + s]
    const int base = f < kFrG2 ? kOffW3 : kOffW2;
    const int q = f - (f < kFrG2 ? kFrG3 : kFrG2);
    const int rt = q >> 1, kb = q & 1;
    return th[base + (32 * kb + s) * kHid + 16 * rt + c];
  }
  const int kb = f - kFrG1;                          // W1^T[c][32 kb + s] = W1[32 kb + s][c]
  return c < kIn ? th[kOffW1 + (32 * kb + s) * kIn + c] : 0.0f;
}

__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ th,
                                                   uint4* __restrict__ packed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kFrAll * 64) {
    const int f = i >> 6, lane = i & 63;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = static_cast<__bf16>(frag_value(th, f, lane, j));
    packed[i] = __builtin_bit_cast(uint4, v);
  } else if (i < kFrAll * 64 + kBias) {
    const int k = i - kFrAll * 64;
    float b = 0.0f;
    if (k < 64) b = th[kOffB1 + k];
    else if (k < 128) b = th[kOffB2 + k - 64];
    else if (k < 192) b = th[kOffB3 + k - 128];
    else if (k < 192 + kOut) b = th[kOffB4 + k - 192];
    reinterpret_cast<float*>(packed + kFrAll * 64)[k] = b;
  }
}

// ------------------------------------------------------------------------- training set
// Cell states drawn over the range the simulations visit, with half of the densities and
// half of the temperatures concentrated within a factor e^1.5 of the thresholds; targets
// from the plain relaxed source term in FP64.
__global__ void __launch_bounds__(256) sample_kernel(MlpSampleArgs p, float* __restrict__ x,
                                                     float* __restrict__ y, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const unsigned long long id = static_cast<unsigned long long>(p.first + i);
  uint32_t c0[4] = {static_cast<uint32_t>(id), static_cast<uint32_t>(id >> 32), kTagMlpSample, 0u};
  uint32_t c1[4] = {static_cast<uint32_t>(id), static_cast<uint32_t>(id >> 32), kTagMlpSample, 1u};
  philox4x32_10(c0, p.seed_lo, p.seed_hi);
  philox4x32_10(c1, p.seed_lo, p.seed_hi);
  const double u0 = uniform_open_d(c0[0]), u1 = uniform_open_d(c0[1]);
  const double u2 = uniform_open_d(c0[2]), u3 = uniform_open_d(c0[3]);
  const double u4 = uniform_open_d(c1[0]);
  const bool near_d = (c1[1] >> 31) != 0, near_t = (c1[2] >> 31) != 0;
  const double eps = p.eps_lo + (p.eps_hi - p.eps_lo) * u3;
  const double dc = p.dc_lo + (p.dc_hi - p.dc_lo) * u4;
  const double lnd = near_d ? log(dc) + 1.5 * (2.0 * u0 - 1.0)
                            : p.lnd_lo + (p.lnd_hi - p.lnd_lo) * u0;
  const double lnt = near_t ? log(p.t_c) + 1.5 * (2.0 * u1 - 1.0)
                            : p.lnt_lo + (p.lnt_hi - p.lnt_lo) * u1;
  const double lna = p.lna_lo + (p.lna_hi - p.lna_lo) * u2;
  const double delta = exp(lnd), temp = exp(lnt);
  x[i] = static_cast<float>((lnd - 4.6) / 5.0);
  x[count + i] = static_cast<float>((lnt - 10.4) / 5.0);
  x[2 * count + i] = static_cast<float>((lna + 3.0) / 1.5);
  x[3 * count + i] = static_cast<float>(eps / 0.02 - 1.0);
  x[4 * count + i] = static_cast<float>(dc / 100.0 - 1.0);
  double o0, o1;
  closure_targets(delta, temp, lna, eps, dc, p.omega_b, p.t_c, p.w_rho, p.w_t, o0, o1);
  y[i] = static_cast<float>(o0);
  y[count + i] = static_cast<float>(o1);
}

// ------------------------------------------------------------------------- inference
// input operand of cells [base, base + 16 NCT) from a structure-of-arrays x[5][count]
template <int NCT>
__device__ __forceinline__ Act<NCT> load_inputs(const float* __restrict__ x, long long count,
                                                long long base, int lane) {
  const int g = lane >> 4, c = lane & 15;
  Act<NCT> a;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const long long s = base + 16 * ct + c;
    const bool ok = s < count;
    f4 lo = {0.0f, 0.0f, 0.0f, 0.0f};
    if (ok && g == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) lo[r] = x[r * count + s];
    } else if (ok && g == 1) {
      lo[0] = x[4 * count + s];
    }
    set_half(a.v[0][ct], 0, lo);
    set_half(a.v[0][ct], 1, f4{0.0f, 0.0f, 0.0f, 0.0f});
  }
  return a;
}

__global__ void __launch_bounds__(kEvalThreads) eval_kernel(const uint4* __restrict__ packed,
                                                            const float* __restrict__ x,
                                                            float* __restrict__ out,
                                                            long long count) {
  __shared__ uint4 fr[kFrFwd * 64];
  __shared__ __attribute__((aligned(16))) float bias[kBias];
  load_packed(packed, kFrFwd, fr, bias);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const long long tiles = (count + 63) / 64;
  for (long long t = static_cast<long long>(blockIdx.x) * 4 + wave; t < tiles;
       t += static_cast<long long>(gridDim.x) * 4) {
    const long long base = t * 64;
    const Act<4> xin = load_inputs<4>(x, count, base, lane);
    f4 o[4];
    forward<4>(fr, bias, xin, o, nullptr, nullptr, lane);
    if (g == 0) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const long long s = base + 16 * ct + c;
        if (s < count) {
          out[s] = o[ct][0];
          out[count + s] = o[ct][1];
        }
      }
    }
  }
}

// input gradients, 32 cells per wave pass
__global__ void __launch_bounds__(kEvalThreads) vjp_kernel(const uint4* __restrict__ packed,
                                                           const float* __restrict__ x,
                                                           const float* __restrict__ gout,
                                                           float* __restrict__ gx,
                                                           long long count) {
  __shared__ uint4 fr[kFrAll * 64];
  __shared__ __attribute__((aligned(16))) float bias[kBias];
  load_packed(packed, kFrAll, fr, bias);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const long long tiles = (count + 31) / 32;
  for (long long t = static_cast<long long>(blockIdx.x) * 4 + wave; t < tiles;
       t += static_cast<long long>(gridDim.x) * 4) {
    const long long base = t * 32;
    const Act<2> xin = load_inputs<2>(x, count, base, lane);
    f4 o[2], go[2], dx[2];
    Act<2> sd[3];
    forward<2>(fr, bias, xin, o, sd, nullptr, lane);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const long long s = base + 16 * ct + c;
      go[ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      if (g == 0 && s < count) {
        go[ct][0] = gout[s];
        go[ct][1] = gout[count + s];
      }
    }
    backward<2>(fr, sd, go, dx, nullptr, lane);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const long long s = base + 16 * ct + c;
      if (s >= count) continue;
      if (g == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) gx[r * count + s] = dx[ct][r];
      } else if (g == 1) {
        gx[4 * count + s] = dx[ct][0];
      }
    }
  }
}

// ------------------------------------------------------------------------- training
// A wave takes 32 samples per pass.  The weight gradients sum over samples, so they use the
// matrix cores with the samples as the K dimension; their operands come from LDS transposes
// T[unit][sample] (bf16, row stride kTStride32) of the activations and of dL/dz.
constexpr int kTStride32 = 40;   // 80-byte rows: 16-byte aligned, conflict-free b128 reads
constexpr int kTRows = 16 + 3 * 64 + 64 + 16;   // inputs, h1..h3, dz, dnet

__device__ __forceinline__ void store_act_t(const Act<2>& a, __bf16* T, int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        T[(32 * kb + slot_unit(g, j)) * kTStride32 + 16 * ct + c] = a.v[kb][ct][j];
}

// operand of rows [16 t, 16 t + 16) over the 32 samples (K slots 8g + j = sample 8g + j)
__device__ __forceinline__ bf16x8 load_t(const __bf16* T, int t, int lane) {
  const int g = lane >> 4, c = lane & 15;
  return *reinterpret_cast<const bf16x8*>(T + (16 * t + c) * kTStride32 + 8 * g);
}

// sum over the 32 samples of dZ[16 ot + i][s] H[16 it + j][s]; with TH = null, of dZ alone
__device__ __forceinline__ f4 grad_tile(const __bf16* TZ, int ot, const __bf16* TH, int it,
                                        int lane) {
  bf16x8 b;
  if (TH) {
    b = load_t(TH, it, lane);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = static_cast<__bf16>(1.0f);
  }
  return mfma(load_t(TZ, ot, lane), b, f4{0.0f, 0.0f, 0.0f, 0.0f});
}

// weight and bias gradient of a 64 x 64 layer into the wave's partial vector
__device__ __forceinline__ void write_hidden_grads(const __bf16* TZ, const __bf16* TH, int off_w,
                                                   int off_b, float* __restrict__ pg, int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const f4 d = grad_tile(TZ, ot, TH, it, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) pg[off_w + (16 * ot + 4 * g + r) * kHid + 16 * it + c] = d[r];
    }
    const f4 db = grad_tile(TZ, ot, nullptr, 0, lane);
    if (c == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) pg[off_b + 16 * ot + 4 * g + r] = db[r];
    }
  }
}

// One wave per 32 samples of the batch: loss, dL/do, the backward pass and the gradient of
// every parameter of the objective mean_s sum_k (o_k - y_k)^2 over the batch, written as a
// per-wave partial (partial[wave][kParams], loss_part[wave]).  Waves past the end of the
// batch write zeros.
__global__ void __launch_bounds__(64 * kTrainWaves) train_grad_kernel(
    const uint4* __restrict__ packed, const float* __restrict__ x, const float* __restrict__ y,
    long long n_data, long long start, long long batch, float inv_batch, float* __restrict__ partial,
    double* __restrict__ loss_part) {
  __shared__ uint4 fr[kFrAll * 64];
  __shared__ __attribute__((aligned(16))) float bias[kBias];
  __shared__ __attribute__((aligned(16))) __bf16 tbuf[kTrainWaves][kTRows * kTStride32];
  __shared__ double lred[kTrainWaves][64];
  load_packed(packed, kFrAll, fr, bias);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  __bf16* TX = tbuf[wave];                     // inputs     [16][32]
  __bf16* TH = TX + 16 * kTStride32;           // h1, h2, h3 [3][64][32]
  __bf16* TZ = TH + 3 * 64 * kTStride32;       // dL/dz of the current layer [64][32]
  __bf16* TN = TZ + 64 * kTStride32;           // dL/dnet    [16][32]
  for (int i = lane; i < 16 * kTStride32; i += 64) {
    TX[i] = static_cast<__bf16>(0.0f);
    TN[i] = static_cast<__bf16>(0.0f);
  }
  __syncthreads();
  const long long wg = static_cast<long long>(blockIdx.x) * kTrainWaves + wave;
  const long long base = wg * 32;               // position in the batch
  Act<2> xin;
  long long sidx[2];
  bool ok[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const long long b = base + 16 * ct + c;
    ok[ct] = b < batch;
    sidx[ct] = (start + b) % n_data;
    f4 lo = {0.0f, 0.0f, 0.0f, 0.0f};
    if (ok[ct] && g == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) lo[r] = x[r * n_data + sidx[ct]];
    } else if (ok[ct] && g == 1) {
      lo[0] = x[4 * n_data + sidx[ct]];
    }
    set_half(xin.v[0][ct], 0, lo);
    set_half(xin.v[0][ct], 1, f4{0.0f, 0.0f, 0.0f, 0.0f});
  }
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    if (g < 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) TX[(4 * g + r) * kTStride32 + 16 * ct + c] = xin.v[0][ct][r];
    }
  }
  Act<2> sd[3], hs[3], dz[3];
  f4 o[2], go[2], dx[2];
  forward<2>(fr, bias, xin, o, sd, hs, lane);
#pragma unroll
  for (int l = 0; l < 3; ++l) store_act_t(hs[l], TH + l * 64 * kTStride32, lane);
  double lsum = 0.0;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    go[ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if (g == 0 && ok[ct]) {
#pragma unroll
      for (int k = 0; k < kOut; ++k) {
        const float d = o[ct][k] - y[k * n_data + sidx[ct]];
        lsum += static_cast<double>(d) * d;
        go[ct][k] = 2.0f * d * inv_batch;
      }
    }
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < kOut; ++k)
        TN[k * kTStride32 + 16 * ct + c] = static_cast<__bf16>(go[ct][k] * kOutScale);
    }
  }
  backward<2>(fr, sd, go, dx, dz, lane);
  store_act_t(dz[2], TZ, lane);
  __syncthreads();
  float* pg = partial + wg * kParams;
  // output layer: dW4 = dnet h3^T, db4 = sum of dnet
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const f4 d = grad_tile(TN, 0, TH + 2 * 64 * kTStride32, it, lane);
    if (g == 0) {
#pragma unroll
      for (int r = 0; r < kOut; ++r) pg[kOffW4 + r * kHid + 16 * it + c] = d[r];
    }
  }
  {
    const f4 db = grad_tile(TN, 0, nullptr, 0, lane);
    if (g == 0 && c == 0) {
#pragma unroll
      for (int r = 0; r < kOut; ++r) pg[kOffB4 + r] = db[r];
    }
  }
  // hidden layers 3 and 2 (inputs h2, h1), then 1 (inputs x)
  write_hidden_grads(TZ, TH + 1 * 64 * kTStride32, kOffW3, kOffB3, pg, lane);
  __syncthreads();
  store_act_t(dz[1], TZ, lane);
  __syncthreads();
  write_hidden_grads(TZ, TH, kOffW2, kOffB2, pg, lane);
  __syncthreads();
  store_act_t(dz[0], TZ, lane);
  __syncthreads();
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const f4 d = grad_tile(TZ, ot, TX, 0, lane);
    if (c < kIn) {
#pragma unroll
      for (int r = 0; r < 4; ++r) pg[kOffW1 + (16 * ot + 4 * g + r) * kIn + c] = d[r];
    }
    const f4 db = grad_tile(TZ, ot, nullptr, 0, lane);
    if (c == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) pg[kOffB1 + 16 * ot + 4 * g + r] = db[r];
    }
  }
  // loss of the wave, lanes summed in a fixed order
  lred[wave][lane] = lsum;
  __syncthreads();
  if (lane == 0) {
    double s = 0.0;
    for (int i = 0; i < 64; ++i) s += lred[wave][i];
    loss_part[wg] = s;
  }
}

// Sum of the per-wave partial gradients of kRedParams parameters per block: thread
// (stripe, j) adds partials stripe, stripe + kStripes, ... of parameter base + j, then the
// stripes are added in order; the result does not depend on the launch.
constexpr int kRedParams = 16;
constexpr int kStripes = 16;   // kRedParams * kStripes = 256 threads

__device__ __forceinline__ double sum_partials(const float* __restrict__ partial, int nparts,
                                               int p) {
  __shared__ double sh[kStripes][kRedParams];
  const int j = threadIdx.x % kRedParams, stripe = threadIdx.x / kRedParams;
  double acc = 0.0;
  if (p < kParams)
    for (int w = stripe; w < nparts; w += kStripes)
      acc += partial[static_cast<long long>(w) * kParams + p];
  sh[stripe][j] = acc;
  __syncthreads();
  double s = 0.0;
  if (stripe == 0)
    for (int k = 0; k < kStripes; ++k) s += sh[k][j];
  return s;   // valid in stripe 0
}

// Block-wide sum of the loss partials in a fixed order (valid in thread 0); every thread of
// the block calls it.
__device__ __forceinline__ double sum_loss(const double* __restrict__ loss_part, int nparts) {
  __shared__ double sh[256];
  double l = 0.0;
  for (int w = threadIdx.x; w < nparts; w += 256) l += loss_part[w];
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return sh[0];
}

// grad[p] = sum over partials (fixed order, FP64); loss = sum of loss partials * scale
__global__ void __launch_bounds__(256) reduce_grad_kernel(const float* __restrict__ partial,
                                                          int nparts, const double* __restrict__ loss_part,
                                                          double loss_scale, double* __restrict__ grad,
                                                          double* __restrict__ loss_out) {
  const int p = blockIdx.x * kRedParams + threadIdx.x % kRedParams;
  const double s = sum_partials(partial, nparts, p);
  if (threadIdx.x < kRedParams && p < kParams) grad[p] = s;
  if (blockIdx.x == 0) {
    const double l = sum_loss(loss_part, nparts);
    if (threadIdx.x == 0) *loss_out = l * loss_scale;
  }
}

// Adam update of theta from the summed partial gradients; loss_hist[step] = batch loss
__global__ void __launch_bounds__(256) adam_kernel(const float* __restrict__ partial, int nparts,
                                                   const double* __restrict__ loss_part,
                                                   double loss_scale, float* __restrict__ th,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   AdamArgs a, double* __restrict__ loss_hist) {
  const int p = blockIdx.x * kRedParams + threadIdx.x % kRedParams;
  const double s = sum_partials(partial, nparts, p);
  if (threadIdx.x < kRedParams && p < kParams) {
    const float gr = static_cast<float>(s);
    const float mm = a.beta1 * m[p] + (1.0f - a.beta1) * gr;
    const float vv = a.beta2 * v[p] + (1.0f - a.beta2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    th[p] -= a.lr * (mm * a.corr1) / (sqrtf(vv * a.corr2) + a.eps);
  }
  if (loss_hist && blockIdx.x == 0) {
    const double l = sum_loss(loss_part, nparts);
    if (threadIdx.x == 0) loss_hist[a.step] = l * loss_scale;
  }
}

}  // namespace

int mlp_eval_blocks(long long count) {
  const long long tiles = (count + 31) / 32;
  return static_cast<int>(std::max<long long>(1, std::min<long long>((tiles + 3) / 4, 2048)));
}

void launch_mlp_pack(hipStream_t st, const float* theta, uint4* packed) {
  const int total = kFrAll * 64 + kBias;
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, theta, packed);
  DH_LAUNCH_CHECK();
}

void launch_mlp_sample(hipStream_t st, const MlpSampleArgs& p, float* x, float* y, long long count) {
  hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, x, y, count);
  DH_LAUNCH_CHECK();
}

void launch_mlp_eval(hipStream_t st, const uint4* packed, const float* x, float* out,
                     long long count) {
  hipLaunchKernelGGL(eval_kernel, dim3(mlp_eval_blocks(count)), dim3(kEvalThreads), 0, st, packed,
                     x, out, count);
  DH_LAUNCH_CHECK();
}

void launch_mlp_vjp(hipStream_t st, const uint4* packed, const float* x, const float* gout,
                    float* gx, long long count) {
  hipLaunchKernelGGL(vjp_kernel, dim3(mlp_eval_blocks(count)), dim3(kEvalThreads), 0, st, packed,
                     x, gout, gx, count);
  DH_LAUNCH_CHECK();
}

// partial vectors written by one training launch: a whole number of blocks of waves; waves
// past the end of the batch contribute zeros
int mlp_train_parts(long long batch) {
  const long long waves = (batch + 31) / 32;
  return static_cast<int>((waves + kTrainWaves - 1) / kTrainWaves * kTrainWaves);
}

void launch_mlp_train_grad(hipStream_t st, const uint4* packed, const float* x, const float* y,
                           long long n_data, long long start, long long batch, float* partial,
                           double* loss_part) {
  const int blocks = mlp_train_parts(batch) / kTrainWaves;
  hipLaunchKernelGGL(train_grad_kernel, dim3(blocks), dim3(64 * kTrainWaves), 0, st, packed, x, y,
                     n_data, start, batch, static_cast<float>(1.0 / static_cast<double>(batch)),
                     partial, loss_part);
  DH_LAUNCH_CHECK();
}

void launch_mlp_reduce_grad(hipStream_t st, const float* partial, int nparts,
                            const double* loss_part, double loss_scale, double* grad,
                            double* loss_out) {
  hipLaunchKernelGGL(reduce_grad_kernel, dim3(blocks_for(kParams, kRedParams)), dim3(256), 0, st,
                     partial, nparts, loss_part, loss_scale, grad, loss_out);
  DH_LAUNCH_CHECK();
}

void launch_mlp_adam(hipStream_t st, const float* partial, int nparts, const double* loss_part,
                     double loss_scale, float* theta, float* m, float* v, const AdamArgs& a,
                     double* loss_hist) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(kParams, kRedParams)), dim3(256), 0, st, partial,
                     nparts, loss_part, loss_scale, theta, m, v, a, loss_hist);
  DH_LAUNCH_CHECK();
}

}  // namespace dh

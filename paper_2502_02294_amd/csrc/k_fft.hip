// FFTs for the particle-mesh Poisson solve and the initial conditions (Sec. 2.1, 2.2), with
// the spectral operators fused into the z pass.
//
// Half spectrum layout: spec[(kz * n + ky) * nh + kx], nh = n/2 + 1, kx = 0..n/2.
// Forward transforms are unnormalised; every spectral operator carries the 1/N^3 of the
// inverse.  Passes:
//   x_r2c     rows of n reals -> n/2+1 complex
//   pencil<1> y lines (all (z, kx) lines of a sample, tk consecutive ones per block)
//   pencil<2> z lines ((ky, kx) lines): forward, spectral operator, inverse, each optional,
//             and optional accumulation into the output
//   x_c2r     Hermitian extension of each row, inverse FFT, real part times a scale.
//
// Each n-point line transform is the four-step factorisation n = N1 * N2 with both factors
// done in registers and one transpose through LDS:
//   X[k1 + N1 k2] = sum_j2 W_N2^(j2 k2) W_n^(j2 k1) sum_j1 x[j2 + N2 j1] W_N1^(j1 k1).
// Natural order "D_x": N2 threads per line, thread q holds x[q + N2 r], r < N1.
// Spectral order "D_k": N1 threads per line, thread q holds X[q + N1 r], r < N2.
// The forward transform maps D_x to D_k, the inverse D_k to D_x:
//   x[a + N2 b] = sum_k1 W_N1^(-b k1) W_n^(-a k1) sum_k2 X[k1 + N1 k2] W_N2^(-a k2).
#include <cmath>
#include <vector>

#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxR = 16;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// cos and sin of 2 pi e / 16, e = 0..7
__device__ constexpr float kCos16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                                        0.38268343236508977f, 0.0f, -0.38268343236508977f,
                                        -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kSin16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f,
                                        0.92387953251128674f, 1.0f, 0.92387953251128674f,
                                        0.70710678118654752f, 0.38268343236508977f};

// x * W_16^(+-e): forward exp(-2 pi i e / 16), inverse exp(+2 pi i e / 16); e is a constant
template <bool INV>
__device__ __forceinline__ float2 rot16(float2 x, int e) {
  if (e == 0) return x;
  if (e == 4) return INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
  const float c = kCos16[e], s = INV ? kSin16[e] : -kSin16[e];
  return make_float2(x.x * c - x.y * s, x.x * s + x.y * c);
}

constexpr int bit_reverse(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}
constexpr int log2c(int r) { return r <= 1 ? 0 : 1 + log2c(r / 2); }

// In-register R-point DFT (R = 2, 4, 8, 16) of v[0..R-1], natural order in and out: radix-2
// decimation in time after a bit-reversal permutation, twiddles as constants.
template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2 (&v)[kMaxR]) {
  constexpr int bits = log2c(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bit_reverse(i, bits);
    if (j > i) {
      const float2 t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int m = 2; m <= R; m <<= 1) {
#pragma unroll
    for (int k = 0; k < R; k += m)
#pragma unroll
      for (int j = 0; j < m / 2; ++j) {
        const float2 t = rot16<INV>(v[k + j + m / 2], j * (16 / m));
        const float2 u = v[k + j];
        v[k + j] = cadd(u, t);
        v[k + j + m / 2] = csub(u, t);
      }
  }
}

// W_n^m (forward sign) from the half table tw[m] = exp(-2 pi i m / n), m < n/2
__device__ __forceinline__ float2 tw_full(const float2* tw, int m, int n) {
  const int h = n >> 1;
  const float2 w = tw[m & (h - 1)];
  return m < h ? w : make_float2(-w.x, -w.y);
}

// The transpose of a line transform through this line's exchange buffer ex (n floats): the
// writer thread q puts v[i] (i < NW) at [i WS + q], the reader thread q takes v[j] (j < NR)
// from [q RS + j]; real parts first, then imaginary parts, so the buffer is half the size
// of a complex one (more blocks per CU).  A caller that writes ex again needs a barrier first.
template <int NW, int WS, int NR, int RS>
__device__ __forceinline__ void exchange(float2 (&v)[kMaxR], float* ex, int q, bool writer,
                                         bool reader) {
  float re[kMaxR];
  if (writer)
#pragma unroll
    for (int i = 0; i < NW; ++i) ex[i * WS + q] = v[i].x;
  __syncthreads();
  if (reader)
#pragma unroll
    for (int j = 0; j < NR; ++j) re[j] = ex[q * RS + j];
  __syncthreads();
  if (writer)
#pragma unroll
    for (int i = 0; i < NW; ++i) ex[i * WS + q] = v[i].y;
  __syncthreads();
  if (reader)
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = make_float2(re[j], ex[q * RS + j]);
}

// Forward line transform: D_x (thread q < N2 of the line) -> D_k (thread q < N1).
// ex: this line's exchange buffer (n floats), tw: twiddle half table in LDS.
template <int N1, int N2>
__device__ __forceinline__ void line_forward(float2 (&v)[kMaxR], float* ex, const float2* tw,
                                             int q, bool in_x, bool in_k) {
  constexpr int n = N1 * N2;
  if (in_x) {   // q = j2: DFT over j1, then W_n^(j2 k1), to [k1 * N2 + j2]
    dft_reg<N1, false>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmul(v[k1], tw_full(tw, q * k1, n));
  }
  exchange<N1, N2, N2, N2>(v, ex, q, in_x, in_k);
  if (in_k) dft_reg<N2, false>(v);   // q = k1: DFT over j2 gives X[k1 + N1 k2]
}

// Inverse line transform: D_k (thread q < N1) -> D_x (thread q < N2), unnormalised.
template <int N1, int N2>
__device__ __forceinline__ void line_inverse(float2 (&v)[kMaxR], float* ex, const float2* tw,
                                             int q, bool in_x, bool in_k) {
  constexpr int n = N1 * N2;
  if (in_k) {   // q = k1: inverse DFT over k2 gives index a; times W_n^(-a k1); to [a * N1 + k1]
    dft_reg<N2, true>(v);
#pragma unroll
    for (int a = 0; a < N2; ++a) {
      const float2 w = tw_full(tw, a * q, n);
      v[a] = cmul(v[a], make_float2(w.x, -w.y));
    }
  }
  exchange<N2, N1, N1, N1>(v, ex, q, in_k, in_x);
  if (in_x) dft_reg<N1, true>(v);   // q = a: inverse DFT over k1 gives x[a + N2 b]
}

__device__ __forceinline__ void load_tw(float2* sh_tw, const float2* tw, int n) {
  for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) sh_tw[i] = tw[i];
}

template <int N1, int N2>
struct Lines {
  static constexpr int n = N1 * N2;
  static constexpr int R = N1 > N2 ? N1 : N2;
  static constexpr int tk = kFftThreads / R;   // lines per block
  static constexpr int ps = n + 1;             // padded exchange stride
};

// ------------------------------------------------------------------------------- x passes
// Rows of all samples are consecutive (n^2 per sample); a block's rows lie in one sample.
// Thread t: q = t % R, row = t / R (consecutive lanes walk along the row).
template <int N1, int N2>
__global__ void __launch_bounds__(kFftThreads) x_r2c_kernel(const float* __restrict__ in,
                                                            float2* __restrict__ spec,
                                                            const float2* __restrict__ tw,
                                                            const StepScal* __restrict__ tab,
                                                            long long in_stride) {
  using L = Lines<N1, N2>;
  constexpr int n = L::n, nh = n / 2 + 1;
  __shared__ float EX[L::tk * L::ps];
  __shared__ float2 TW[n / 2];
  const long long row0 = static_cast<long long>(blockIdx.x) * L::tk;
  const long long nn = static_cast<long long>(n) * n;
  const int smp = static_cast<int>(row0 / nn);
  if (!sample_active(tab, smp)) return;
  load_tw(TW, tw, n);
  const int q = threadIdx.x % L::R, r = threadIdx.x / L::R;
  const long long row = row0 + r;
  const float* src = in + smp * in_stride + (row - smp * nn) * n;
  float2 v[kMaxR];
  const bool in_x = q < N2, in_k = q < N1;
  if (in_x)
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) v[j1] = make_float2(src[q + N2 * j1], 0.0f);
  __syncthreads();
  line_forward<N1, N2>(v, EX + r * L::ps, TW, q, in_x, in_k);
  if (in_k)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = q + N1 * k2;
      if (k < nh) spec[row * nh + k] = v[k2];
    }
}

template <int N1, int N2>
__global__ void __launch_bounds__(kFftThreads) x_c2r_kernel(const float2* __restrict__ spec,
                                                            float* __restrict__ out,
                                                            const float2* __restrict__ tw,
                                                            float scale,
                                                            const StepScal* __restrict__ tab,
                                                            long long out_stride) {
  using L = Lines<N1, N2>;
  constexpr int n = L::n, nh = n / 2 + 1;
  __shared__ float EX[L::tk * L::ps];
  __shared__ float2 TW[n / 2];
  const long long row0 = static_cast<long long>(blockIdx.x) * L::tk;
  const long long nn = static_cast<long long>(n) * n;
  const int smp = static_cast<int>(row0 / nn);
  if (!sample_active(tab, smp)) return;
  load_tw(TW, tw, n);
  const int q = threadIdx.x % L::R, r = threadIdx.x / L::R;
  const long long row = row0 + r;
  float2 v[kMaxR];
  const bool in_x = q < N2, in_k = q < N1;
  if (in_k)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {   // Hermitian extension X[n - k] = conj(X[k])
      const int k = q + N1 * k2;
      const float2 w = spec[row * nh + (k < nh ? k : n - k)];
      v[k2] = k < nh ? w : make_float2(w.x, -w.y);
    }
  __syncthreads();
  line_inverse<N1, N2>(v, EX + r * L::ps, TW, q, in_x, in_k);
  if (in_x) {
    float* dst = out + smp * out_stride + (row - smp * nn) * n;
#pragma unroll
    for (int b = 0; b < N1; ++b) dst[q + N2 * b] = v[b].x * scale;
  }
}

// ---------------------------------------------------------------------------- line passes
struct OpArgs {
  int op;          // -1 none, kOpGreen, kOpIcDisp, kOpIcDispT, kOpIcHess, kOpZa, kOpZaT
  float green;     // -(3 Om / 2a) / N^3
  int axis, axis2;
  float sqrt_amp;  // sqrt(A D^2 / V_cell)
  float half_ns;   // spectral index / 2
  float om_h;      // Omega_m h
  float kphys;     // n / box: rad/cell -> h/Mpc
  float inv_n3;    // 1/N^3, times the operator's scale for kOpZa / kOpZaT
  int eh;          // transfer function: 0 BBKS, 1 Eisenstein & Hu without wiggles
  float eh_theta2, eh_alpha, eh_ks;
};

// derivative factor k_j (rad/cell) of mode (fx, fy, fz): zero on the Nyquist plane of its own
// axis (an odd derivative of the real Nyquist mode)
__device__ __forceinline__ float deriv_k(int axis, int fx, int fy, int fz, int n) {
  const int f = axis == 0 ? fx : (axis == 1 ? fy : fz);
  if (f == n / 2 || f == -n / 2) return 0.0f;
  return 6.283185307179586f / static_cast<float>(n) * static_cast<float>(f);
}

// sqrt(P(k)) / sqrt(A D^2 / V_cell) at k = kp h/Mpc: k^(n_s/2) T(k)
__device__ __forceinline__ float sqrt_shape(const OpArgs& o, float kp) {
  float t;
  if (o.eh) {
    const float x = kp * o.eh_ks;
    const float x2 = x * x;
    const float gamma = o.om_h * (o.eh_alpha + (1.0f - o.eh_alpha) / (1.0f + x2 * x2));
    const float q = kp * o.eh_theta2 / gamma;
    const float l = logf(2.0f * 2.718281828459045f + 1.8f * q);
    const float c = 14.2f + 731.0f / (1.0f + 62.5f * q);
    t = l / (l + c * q * q);
  } else {
    const float q = kp / o.om_h;
    const float q2 = 16.1f * q, q3 = 5.46f * q, q4 = 6.71f * q;
    t = logf(1.0f + 2.34f * q) / (2.34f * q) *
        powf(1.0f + 3.89f * q + q2 * q2 + q3 * q3 * q3 + (q4 * q4) * (q4 * q4), -0.25f);
  }
  return powf(kp, o.half_ns) * t;
}

__device__ __forceinline__ int signed_freq(int k, int n) { return k <= n / 2 ? k : k - n; }

// OPK: 0 none, 1 Green's function, 2 initial-condition displacement (o.op says which sign)
template <int OPK>
__device__ __forceinline__ float2 apply_op(const OpArgs& o, int kx, int ky, int kz, int n,
                                           float2 v) {
  const int fx = kx, fy = signed_freq(ky, n), fz = signed_freq(kz, n);
  if (OPK == 0) return v;
  if (OPK == 1) {
    const float c = 6.283185307179586f / static_cast<float>(n);
    const float ax = c * fx, ay = c * fy, az = c * fz;
    const float k2 = ax * ax + ay * ay + az * az;
    if (k2 == 0.0f) return make_float2(0.0f, 0.0f);
    const float f = o.green / k2;
    return make_float2(v.x * f, v.y * f);
  }
  // initial-condition operators (derivative factors from deriv_k):
  //   kOpIcDisp  i k_axis sqrt(P(k)) / k^2 / N^3 (kOpIcDispT: its conjugate), the Zel'dovich
  //              displacement of white noise;
  //   kOpIcHess  k_axis k_axis2 sqrt(P(k)) / k^2 / N^3 (real): second derivative of the
  //              linear potential (its own transpose);
  //   kOpZa      i k_axis / k^2 times inv_n3 (kOpZaT: its conjugate), the displacement of a
  //              given density, scaled
  const float c = 6.283185307179586f / static_cast<float>(n);
  const float ax = c * fx, ay = c * fy, az = c * fz;
  const float k2 = ax * ax + ay * ay + az * az;
  if (k2 == 0.0f) return make_float2(0.0f, 0.0f);
  const float kj = deriv_k(o.axis, fx, fy, fz, n);
  if (o.op == kOpZa || o.op == kOpZaT) {
    const float f = kj / k2 * o.inv_n3;
    const float ff = o.op == kOpZa ? f : -f;
    return make_float2(-v.y * ff, v.x * ff);
  }
  const float kp = sqrtf(k2) * o.kphys;
  const float spec = o.sqrt_amp * sqrt_shape(o, kp);
  if (o.op == kOpIcHess) {
    const float f = kj * deriv_k(o.axis2, fx, fy, fz, n) * spec / k2 * o.inv_n3;
    return make_float2(v.x * f, v.y * f);
  }
  const float f = kj * spec / k2 * o.inv_n3;
  const float ff = o.op == kOpIcDisp ? f : -f;
  // multiply by i * ff
  return make_float2(-v.y * ff, v.x * ff);
}

// Workgroups go to the 8 XCDs (each with its own L2) round robin.  Consecutive line groups
// of a pass share cache lines (a spectrum row of nh = n/2 + 1 complex values is not line
// aligned), so each XCD takes one contiguous range of groups: block b -> group
// (b mod 8) nb/8 + b/8 when nb is a multiple of 8 (a bijection), else b.
__device__ __forceinline__ int xcd_group(int b, int nb) {
  return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

// Line pass along AX (1 = y, 2 = z) over tk consecutive lines of sample blockIdx.y.  Line
// l = fixed * nh + kx (fixed = z for AX = 1, ky for AX = 2); thread t: line t % tk, q = t / tk,
// so consecutive lanes take consecutive kx.  flags: 1 forward, 2 operator, 4 inverse, 8
// accumulate into out.  Input in D_x unless the pass starts with the inverse (D_k).  The
// Green's function factor comes from the sample's step table when there is one.
template <int AX, int N1, int N2, int OPK>
// in and out may alias (in-place passes): no __restrict__ on them
__global__ void __launch_bounds__(kFftThreads) pencil_kernel(const float2* in, float2* out,
                                                             const float2* __restrict__ tw,
                                                             int flags, OpArgs op,
                                                             const StepScal* __restrict__ tab) {
  using L = Lines<N1, N2>;
  constexpr int n = L::n, nh = n / 2 + 1;
  __shared__ float EX[L::tk * L::ps];
  __shared__ float2 TW[n / 2];
  if (!sample_active(tab, blockIdx.y)) return;
  if (tab && op.op == kOpGreen) op.green = tab[blockIdx.y].green;
  const long long slab = static_cast<long long>(n) * n * nh;
  in += blockIdx.y * slab;
  out += blockIdx.y * slab;
  load_tw(TW, tw, n);
  const int li = threadIdx.x % L::tk, q = threadIdx.x / L::tk;
  const int line = xcd_group(blockIdx.x, gridDim.x) * L::tk + li;
  const bool valid = line < n * nh;
  const int fixed = line / nh, kx = line - fixed * nh;
  const long long stride = AX == 1 ? nh : static_cast<long long>(n) * nh;
  const long long base = AX == 1 ? static_cast<long long>(fixed) * n * nh + kx
                                 : static_cast<long long>(fixed) * nh + kx;
  float* ex = EX + li * L::ps;
  float2 v[kMaxR];
  const bool in_x = valid && q < N2, in_k = valid && q < N1;
  if (flags & 1) {
    if (in_x)
#pragma unroll
      for (int r = 0; r < N1; ++r) v[r] = in[base + (q + N2 * r) * stride];
    __syncthreads();
    line_forward<N1, N2>(v, ex, TW, q, in_x, in_k);
  } else {
    if (in_k)
#pragma unroll
      for (int r = 0; r < N2; ++r) v[r] = in[base + (q + N1 * r) * stride];
  }
  if ((flags & 2) && in_k) {
#pragma unroll
    for (int r = 0; r < N2; ++r) {
      const int k = q + N1 * r;
      v[r] = apply_op<OPK>(op, kx, AX == 1 ? k : fixed, AX == 1 ? fixed : k, n, v[r]);
    }
  }
  if (flags & 4) {
    __syncthreads();   // the forward pass may still read the exchange buffer
    line_inverse<N1, N2>(v, ex, TW, q, in_x, in_k);
    if (in_x)
#pragma unroll
      for (int r = 0; r < N1; ++r) {
        const long long g = base + (q + N2 * r) * stride;
        float2 w = v[r];
        if (flags & 8) w = cadd(w, out[g]);
        out[g] = w;
      }
  } else if (in_k) {
#pragma unroll
    for (int r = 0; r < N2; ++r) {
      const long long g = base + (q + N1 * r) * stride;
      float2 w = v[r];
      if (flags & 8) w = cadd(w, out[g]);
      out[g] = w;
    }
  }
}

template <int N1, int N2, int OPK>
void pencil_op(hipStream_t st, int ax, const float2* in, float2* out, const float2* tw,
               int flags, const OpArgs& op, const Batch& b) {
  using L = Lines<N1, N2>;
  constexpr int n = L::n, nh = n / 2 + 1;
  const dim3 grid((n * nh + L::tk - 1) / L::tk, b.S);
  if (ax == 1)
    hipLaunchKernelGGL((pencil_kernel<1, N1, N2, OPK>), grid, dim3(kFftThreads), 0, st, in, out,
                       tw, flags, op, b.tab);
  else
    hipLaunchKernelGGL((pencil_kernel<2, N1, N2, OPK>), grid, dim3(kFftThreads), 0, st, in, out,
                       tw, flags, op, b.tab);
}

template <int N1, int N2>
void pencil_n(hipStream_t st, int ax, const float2* in, float2* out, const float2* tw, int flags,
              const OpArgs& op, const Batch& b) {
  if (!(flags & 2) || op.op < 0)
    pencil_op<N1, N2, 0>(st, ax, in, out, tw, flags & ~2, op, b);
  else if (op.op == kOpGreen)
    pencil_op<N1, N2, 1>(st, ax, in, out, tw, flags, op, b);
  else
    pencil_op<N1, N2, 2>(st, ax, in, out, tw, flags, op, b);
}

template <int N1, int N2>
void r2c_n(hipStream_t st, const float* in, float2* spec, const float2* tw, const Batch& b,
           long long in_stride) {
  using L = Lines<N1, N2>;
  const long long rows = static_cast<long long>(L::n) * L::n * b.S;
  hipLaunchKernelGGL((x_r2c_kernel<N1, N2>), dim3(static_cast<unsigned>(rows / L::tk)),
                     dim3(kFftThreads), 0, st, in, spec, tw, b.tab, in_stride);
}

template <int N1, int N2>
void c2r_n(hipStream_t st, const float2* spec, float* out, const float2* tw, float scale,
           const Batch& b, long long out_stride) {
  using L = Lines<N1, N2>;
  const long long rows = static_cast<long long>(L::n) * L::n * b.S;
  hipLaunchKernelGGL((x_c2r_kernel<N1, N2>), dim3(static_cast<unsigned>(rows / L::tk)),
                     dim3(kFftThreads), 0, st, spec, out, tw, scale, b.tab, out_stride);
}

// n = N1 * N2 with N1 >= N2, both at most 16
#define DH_FFT_DISPATCH(n, CALL)                                  \
  switch (n) {                                                    \
    case 16: CALL(4, 4); break;                                   \
    case 32: CALL(8, 4); break;                                   \
    case 64: CALL(8, 8); break;                                   \
    case 128: CALL(16, 8); break;                                 \
    case 256: CALL(16, 16); break;                                \
    default: throw ArgError("fft: n must be a power of two in [16, 256]"); \
  }

void pencil(hipStream_t st, int ax, const float2* in, float2* out, const float2* tw, int flags,
            const OpArgs& op, const Batch& b) {
#define DH_CALL(a, c) pencil_n<a, c>(st, ax, in, out, tw, flags, op, b)
  DH_FFT_DISPATCH(b.n, DH_CALL)
#undef DH_CALL
  DH_LAUNCH_CHECK();
}

}  // namespace

void fft_make_twiddles(int n, std::vector<float2>& tw) {
  tw.resize(n / 2);
  for (int m = 0; m < n / 2; ++m) {
    const double ang = -2.0 * M_PI * m / n;
    tw[m] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
  }
}

void fft_forward_xy(hipStream_t st, const float* in, float2* spec, const float2* tw,
                    const Batch& b, long long in_stride) {
  const long long is = in_stride < 0 ? b.nc() : in_stride;
#define DH_CALL(a, c) r2c_n<a, c>(st, in, spec, tw, b, is)
  DH_FFT_DISPATCH(b.n, DH_CALL)
#undef DH_CALL
  DH_LAUNCH_CHECK();
  OpArgs none{};
  none.op = -1;
  pencil(st, 1, spec, spec, tw, 1, none, b);
}

void fft_inverse_yx(hipStream_t st, float2* spec, float* out, const float2* tw, float scale,
                    const Batch& b, long long out_stride) {
  OpArgs none{};
  none.op = -1;
  pencil(st, 1, spec, spec, tw, 4, none, b);
  const long long os = out_stride < 0 ? b.nc() : out_stride;
#define DH_CALL(a, c) c2r_n<a, c>(st, spec, out, tw, scale, b, os)
  DH_FFT_DISPATCH(b.n, DH_CALL)
#undef DH_CALL
  DH_LAUNCH_CHECK();
}

void fft_zpass_green(hipStream_t st, float2* spec, const float2* tw, const Batch& b) {
  if (!b.tab) throw ArgError("Poisson pass: step table required");
  OpArgs o{};
  o.op = kOpGreen;
  pencil(st, 2, spec, spec, tw, 1 | 2 | 4, o, b);
}

void fft_zpass_forward(hipStream_t st, const float2* in, float2* out, const float2* tw,
                       const Batch& b) {
  OpArgs none{};
  none.op = -1;
  pencil(st, 2, in, out, tw, 1, none, b);
}

void fft_zpass_inverse(hipStream_t st, float2* spec, const float2* tw, const Batch& b) {
  OpArgs none{};
  none.op = -1;
  pencil(st, 2, spec, spec, tw, 4, none, b);
}

// IC operators on the z pass (see apply_op): out = op(in), forward z transform first and
// inverse after as asked
void fft_zpass_ic(hipStream_t st, const float2* in, float2* out, const float2* tw,
                  const IcOp& op, bool forward_first, bool inverse_after, bool accumulate,
                  const Batch& b) {
  const int n = b.n;
  OpArgs o{};
  o.op = op.op;
  o.axis = op.axis;
  o.axis2 = op.axis2;
  o.sqrt_amp = static_cast<float>(std::sqrt(op.amp));
  o.half_ns = static_cast<float>(0.5 * op.n_s);
  o.om_h = static_cast<float>(op.om_h);
  o.kphys = static_cast<float>(op.kphys);
  o.inv_n3 = static_cast<float>(op.scale / (static_cast<double>(n) * n * n));
  o.eh = op.eh ? 1 : 0;
  o.eh_theta2 = static_cast<float>(op.eh_theta2);
  o.eh_alpha = static_cast<float>(op.eh_alpha);
  o.eh_ks = static_cast<float>(op.eh_ks);
  const int flags = (forward_first ? 1 : 0) | 2 | (inverse_after ? 4 : 0) | (accumulate ? 8 : 0);
  pencil(st, 2, in, out, tw, flags, o, b);
}

}  // namespace dh

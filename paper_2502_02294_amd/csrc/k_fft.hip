// Radix-2 Stockham FFTs in LDS for the particle-mesh Poisson solve and the initial
// conditions (Sec. 2.1, 2.2), with the spectral operators fused into the z pass.
//
// Half spectrum layout: spec[(kz * n + ky) * nh + kx], nh = n/2 + 1, kx = 0..n/2.
// Forward transforms are unnormalised; every spectral operator carries the 1/N^3 of the
// inverse.  Passes:
//   x_r2c     rows of n reals -> n/2+1 complex (full complex FFT of the row in LDS)
//   pencil<1> y pencils (one z plane, tk consecutive kx per block)
//   pencil<2> z pencils (one ky line, tk consecutive kx per block): forward, spectral
//             operator, inverse, each optional, and optional accumulation into the output
//   x_c2r     Hermitian extension of each row, inverse FFT, real part times a scale.
// Stockham step for sub-transform size p: for butterfly i < n/2, k = i mod p,
//   u0 = a[i], u1 = a[i + n/2] * exp(-i pi k / p),  b[2i - k] = u0 + u1, b[2i - k + p] = u0 - u1.
#include <cmath>
#include <vector>

#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kFftThreads = 256;
constexpr int kRowTile = 1024;   // complex elements per x-pass block

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <bool INV>
__device__ float2* lds_fft(float2* a, float2* b, int n, int logn, int npen, int ps,
                           const float2* tw) {
  const int half = n >> 1;
  const int total = npen * half;
  for (int p = 1, s = 0; p < n; p <<= 1, ++s) {
    const int tws = n >> (s + 1);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int pen = t >> (logn - 1);
      const int i = t - pen * half;
      const int k = i & (p - 1);
      const float2 u0 = a[pen * ps + i];
      float2 w = tw[k * tws];
      if (INV) w.y = -w.y;
      const float2 v = cmul(a[pen * ps + i + half], w);
      const int j = (i << 1) - k;
      b[pen * ps + j] = make_float2(u0.x + v.x, u0.y + v.y);
      b[pen * ps + j + p] = make_float2(u0.x - v.x, u0.y - v.y);
    }
    __syncthreads();
    float2* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

__device__ __forceinline__ void load_tw(float2* sh_tw, const float2* tw, int n) {
  for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) sh_tw[i] = tw[i];
}

// Rows of all samples are consecutive (n^2 per sample); a block's rows lie in one sample.
__global__ void __launch_bounds__(kFftThreads) x_r2c_kernel(const float* __restrict__ in,
                                                            float2* __restrict__ spec,
                                                            const float2* __restrict__ tw, int n,
                                                            int logn,
                                                            const StepScal* __restrict__ tab,
                                                            long long in_stride) {
  __shared__ float2 A[kRowTile], B[kRowTile];
  __shared__ float2 TW[128];
  const int rows = kRowTile / n;
  const int nh = n / 2 + 1;
  const long long row0 = static_cast<long long>(blockIdx.x) * rows;
  const long long nn = static_cast<long long>(n) * n;
  const int smp = static_cast<int>(row0 / nn);
  if (!sample_active(tab, smp)) return;
  const float* src = in + smp * in_stride + (row0 - smp * nn) * n;
  load_tw(TW, tw, n);
  for (int t = threadIdx.x; t < rows * n; t += blockDim.x) A[t] = make_float2(src[t], 0.0f);
  __syncthreads();
  float2* r = lds_fft<false>(A, B, n, logn, rows, n, TW);
  for (int t = threadIdx.x; t < rows * nh; t += blockDim.x) {
    const int rr = t / nh, k = t - rr * nh;
    spec[(row0 + rr) * nh + k] = r[rr * n + k];
  }
}

__global__ void __launch_bounds__(kFftThreads) x_c2r_kernel(const float2* __restrict__ spec,
                                                            float* __restrict__ out,
                                                            const float2* __restrict__ tw, int n,
                                                            int logn, float scale,
                                                            const StepScal* __restrict__ tab,
                                                            long long out_stride) {
  __shared__ float2 A[kRowTile], B[kRowTile];
  __shared__ float2 TW[128];
  const int rows = kRowTile / n;
  const int nh = n / 2 + 1;
  const long long row0 = static_cast<long long>(blockIdx.x) * rows;
  const long long nn = static_cast<long long>(n) * n;
  const int smp = static_cast<int>(row0 / nn);
  if (!sample_active(tab, smp)) return;
  float* dst = out + smp * out_stride + (row0 - smp * nn) * n;
  load_tw(TW, tw, n);
  for (int t = threadIdx.x; t < rows * nh; t += blockDim.x) {
    const int rr = t / nh, k = t - rr * nh;
    A[rr * n + k] = spec[(row0 + rr) * nh + k];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < rows * (n - nh); t += blockDim.x) {
    const int rr = t / (n - nh), k = nh + (t - rr * (n - nh));
    const float2 v = A[rr * n + (n - k)];
    A[rr * n + k] = make_float2(v.x, -v.y);
  }
  __syncthreads();
  float2* r = lds_fft<true>(A, B, n, logn, rows, n, TW);
  for (int t = threadIdx.x; t < rows * n; t += blockDim.x) dst[t] = r[t].x * scale;
}

struct OpArgs {
  int op;          // -1 none, kOpGreen, kOpIcDisp, kOpIcDispT
  float green;     // -(3 Om / 2a) / N^3
  int axis;
  double amp;      // A D^2 / V_cell
  double om_h, n_s, kphys;   // Omega_m h, spectral index, (n / box): rad/cell -> h/Mpc
  double inv_n3;
};

__device__ __forceinline__ int signed_freq(int k, int n) { return k <= n / 2 ? k : k - n; }

__device__ float2 apply_op(const OpArgs& o, int kx, int ky, int kz, int n, float2 v) {
  const int fx = kx, fy = signed_freq(ky, n), fz = signed_freq(kz, n);
  if (o.op == kOpGreen) {
    const float c = 6.283185307179586f / static_cast<float>(n);
    const float ax = c * fx, ay = c * fy, az = c * fz;
    const float k2 = ax * ax + ay * ay + az * az;
    if (k2 == 0.0f) return make_float2(0.0f, 0.0f);
    const float f = o.green / k2;
    return make_float2(v.x * f, v.y * f);
  }
  // initial-condition displacement operators, evaluated in double precision
  const double c = 6.283185307179586 / n;
  const double ax = c * fx, ay = c * fy, az = c * fz;
  const double k2 = ax * ax + ay * ay + az * az;
  const int f_axis = o.axis == 0 ? fx : (o.axis == 1 ? fy : fz);
  if (k2 == 0.0 || (f_axis == n / 2 || f_axis == -n / 2)) return make_float2(0.0f, 0.0f);
  const double kj = o.axis == 0 ? ax : (o.axis == 1 ? ay : az);
  const double kp = sqrt(k2) * o.kphys;
  const double q = kp / o.om_h;
  const double tq = log(1.0 + 2.34 * q) / (2.34 * q) *
                    pow(1.0 + 3.89 * q + pow(16.1 * q, 2.0) + pow(5.46 * q, 3.0) + pow(6.71 * q, 4.0),
                        -0.25);
  const double pk = o.amp * pow(kp, o.n_s) * tq * tq;
  const double f = kj * sqrt(pk) / k2 * o.inv_n3;
  const float ff = static_cast<float>(o.op == kOpIcDisp ? f : -f);
  // multiply by i * ff
  return make_float2(-v.y * ff, v.x * ff);
}

// Pencil pass along AX (1 = y, 2 = z) over a tile of tk consecutive kx of sample blockIdx.z.
// flags: 1 forward, 2 operator, 4 inverse, 8 accumulate into out.  The Green's function
// factor comes from the sample's step table when there is one.
template <int AX>
// in and out may alias (in-place passes): no __restrict__ on them
__global__ void __launch_bounds__(kFftThreads) pencil_kernel(const float2* in, float2* out,
                                                             const float2* __restrict__ tw, int n,
                                                             int logn, int kTK, int flags,
                                                             OpArgs op,
                                                             const StepScal* __restrict__ tab) {
  extern __shared__ float2 sh[];
  if (!sample_active(tab, blockIdx.z)) return;
  if (tab && op.op == kOpGreen) op.green = tab[blockIdx.z].green;
  const int ps = n + 1;
  float2* A = sh;
  float2* B = sh + kTK * ps;
  float2* TW = sh + 2 * kTK * ps;
  const int nh = n / 2 + 1;
  const long long slab = static_cast<long long>(n) * n * nh;
  in += blockIdx.z * slab;
  out += blockIdx.z * slab;
  const int kx0 = blockIdx.x * kTK;
  const int fixed = blockIdx.y;   // z for AX = 1, ky for AX = 2
  const long long line_stride = AX == 1 ? nh : static_cast<long long>(n) * nh;
  const long long base = AX == 1 ? static_cast<long long>(fixed) * n * nh
                                 : static_cast<long long>(fixed) * nh;
  load_tw(TW, tw, n);
  for (int t = threadIdx.x; t < kTK * n; t += blockDim.x) {
    const int pen = t % kTK, j = t / kTK;
    const int kx = kx0 + pen;
    A[pen * ps + j] = kx < nh ? in[base + j * line_stride + kx] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  float2* cur = A;
  float2* oth = B;
  if (flags & 1) {
    cur = lds_fft<false>(A, B, n, logn, kTK, ps, TW);
    oth = cur == A ? B : A;
  }
  if (flags & 2) {
    for (int t = threadIdx.x; t < kTK * n; t += blockDim.x) {
      const int pen = t / n, j = t - pen * n;
      const int kx = kx0 + pen;
      if (kx < nh) {
        const int ky = AX == 1 ? j : fixed;
        const int kz = AX == 1 ? fixed : j;
        cur[pen * ps + j] = apply_op(op, kx, ky, kz, n, cur[pen * ps + j]);
      }
    }
    __syncthreads();
  }
  if (flags & 4) cur = lds_fft<true>(cur, oth, n, logn, kTK, ps, TW);
  for (int t = threadIdx.x; t < kTK * n; t += blockDim.x) {
    const int pen = t % kTK, j = t / kTK;
    const int kx = kx0 + pen;
    if (kx < nh) {
      const long long g = base + j * line_stride + kx;
      float2 v = cur[pen * ps + j];
      if (flags & 8) {
        const float2 o = out[g];
        v = make_float2(v.x + o.x, v.y + o.y);
      }
      out[g] = v;
    }
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

size_t pencil_smem(int n, int tk) { return (2 * tk * (n + 1) + n / 2) * sizeof(float2); }

// kx columns per pencil block: 16 (128-byte rows) while the tile fits in 64 KB of LDS
int pencil_tile(int n) { return pencil_smem(n, 16) <= 65536 ? 16 : 8; }

void pencil(hipStream_t st, int ax, const float2* in, float2* out, const float2* tw, int flags,
            const OpArgs& op, const Batch& b) {
  const int n = b.n;
  const int nh = n / 2 + 1;
  const int tk = pencil_tile(n);
  dim3 grid((nh + tk - 1) / tk, n, b.S);
  const size_t smem = pencil_smem(n, tk);
  if (ax == 1)
    hipLaunchKernelGGL(pencil_kernel<1>, grid, dim3(kFftThreads), smem, st, in, out, tw, n,
                       ilog2(n), tk, flags, op, b.tab);
  else
    hipLaunchKernelGGL(pencil_kernel<2>, grid, dim3(kFftThreads), smem, st, in, out, tw, n,
                       ilog2(n), tk, flags, op, b.tab);
  DH_LAUNCH_CHECK();
}

unsigned row_blocks(const Batch& b) {
  return static_cast<unsigned>(static_cast<long long>(b.n) * b.n * b.S / (kRowTile / b.n));
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
  hipLaunchKernelGGL(x_r2c_kernel, dim3(row_blocks(b)), dim3(kFftThreads), 0, st, in, spec, tw,
                     b.n, ilog2(b.n), b.tab, in_stride < 0 ? b.nc() : in_stride);
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
  hipLaunchKernelGGL(x_c2r_kernel, dim3(row_blocks(b)), dim3(kFftThreads), 0, st, spec, out, tw,
                     b.n, ilog2(b.n), scale, b.tab, out_stride < 0 ? b.nc() : out_stride);
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

// IC displacement: out = op_axis(in) then inverse along z (in already transformed in x, y, z)
void fft_zpass_ic(hipStream_t st, const float2* in, float2* out, const float2* tw, int axis,
                  bool transpose, double amp, double om_h, double n_s, double kphys,
                  bool forward_first, bool inverse_after, bool accumulate, const Batch& b) {
  const int n = b.n;
  OpArgs o{};
  o.op = transpose ? kOpIcDispT : kOpIcDisp;
  o.axis = axis;
  o.amp = amp;
  o.om_h = om_h;
  o.n_s = n_s;
  o.kphys = kphys;
  o.inv_n3 = 1.0 / (static_cast<double>(n) * n * n);
  const int flags = (forward_first ? 1 : 0) | 2 | (inverse_after ? 4 : 0) | (accumulate ? 8 : 0);
  pencil(st, 2, in, out, tw, flags, o, b);
}

}  // namespace dh

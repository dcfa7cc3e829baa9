// Learned star-formation closure: a 5 -> 64 -> 64 -> 64 -> 2 SiLU network evaluated by one
// wavefront on 64 cells at a time with the gfx950 BF16 matrix cores (16x16x32, FP32
// accumulate).  The network stands in for the deterministic factors of the star-formation
// probability of Sec. 2.4 (the paper's suggestion of learned sub-grid models, Sec. 4):
//   inputs  x = ((ln Delta - 4.6)/5, (ln T - 10.4)/5, (ln a + 3)/1.5, eps_sf/0.02 - 1,
//               Delta_c/100 - 1),
//   outputs o = 10 * (W4 h3 + b4): o0 = ln(eps_sf / t_ff), o1 = clipped log threshold gate,
//   pi0 = (1 - exp(-exp(o0) dt)) exp(min(o1, 0)).
// Parameters: one flat float vector W1[64][5], b1, W2[64][64], b2, W3[64][64], b3, W4[2][64],
// b4 (8834 values, W[out][in]).
//
// Matrix-core data layout (v_mfma_f32_16x16x32_bf16, wave64, lane = 16 g + c):
//   A operand: row c, k slots 8g..8g+7;  B operand: column c, k slots 8g..8g+7;
//   D result:  column c, rows 4g..4g+3.
// Weights are the A operand (rows = output units), activations the B operand (columns =
// cells).  Slot j of lane group g in K block kb stands for unit 32 kb + 4g + j (j < 4) or
// 32 kb + 16 + 4g + j - 4 (j >= 4), so the D tiles of row tiles 2kb and 2kb+1 concatenated
// are, unchanged, the B operand of the next layer: no data moves between layers.  The same
// slot order is baked into the packed weight fragments.
//
// Packed form (device, written by the pack kernel): 44 fragments of 64 lanes x 8 bf16
// (16 bytes per lane), then 208 floats of biases (b1, b2, b3, b4 padded to 16).
#pragma once

#include <hip/hip_runtime.h>

namespace dh {
namespace mlp {

constexpr int kIn = 5, kHid = 64, kOut = 2;
constexpr int kParams = 8834;
constexpr int kOffW1 = 0, kOffB1 = 320, kOffW2 = 384, kOffB2 = 4480, kOffW3 = 4544,
              kOffB3 = 8640, kOffW4 = 8704, kOffB4 = 8832;
constexpr float kOutScale = 10.0f;

// fragment indices
constexpr int kFrW1 = 0;    // [rt 4]         A = W1      (K: input slots, one block)
constexpr int kFrW2 = 4;    // [rt 4][kb 2]   A = W2
constexpr int kFrW3 = 12;   // [rt 4][kb 2]   A = W3
constexpr int kFrW4 = 20;   // [kb 2]         A = W4      (rows 0, 1 valid)
constexpr int kFrFwd = 22;  // forward fragments end here
constexpr int kFrG4 = 22;   // [rt 4]         A = W4^T    (K: output slots, one block)
constexpr int kFrG3 = 26;   // [rt 4][kb 2]   A = W3^T
constexpr int kFrG2 = 34;   // [rt 4][kb 2]   A = W2^T
constexpr int kFrG1 = 42;   // [kb 2]         A = W1^T    (rows 0..4 valid)
constexpr int kFrAll = 44;
constexpr int kBias = 208;  // b1 0, b2 64, b3 128, b4 192 (padded to 16)
constexpr size_t kPackedBytes = static_cast<size_t>(kFrAll) * 64 * 16 + kBias * sizeof(float);
constexpr size_t kFwdBytes = static_cast<size_t>(kFrFwd) * 64 * 16;
constexpr size_t kBwdBytes = static_cast<size_t>(kFrAll - kFrFwd) * 64 * 16;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// unit of K slot j for lane group g inside a 32-wide K block
__host__ __device__ inline int slot_unit(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + j - 4; }

__device__ __forceinline__ f4 mfma(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 frag(const uint4* fr, int f, int lane) {
  return __builtin_bit_cast(bf16x8, fr[f * 64 + lane]);
}

__device__ __forceinline__ f4 bias4(const float* b, int row0) {
  return *reinterpret_cast<const f4*>(b + row0);
}

__device__ __forceinline__ void set_half(bf16x8& v, int half, f4 x) {
#pragma unroll
  for (int r = 0; r < 4; ++r) v[4 * half + r] = static_cast<__bf16>(x[r]);
}

__device__ __forceinline__ float half_at(const bf16x8& v, int half, int r) {
  return static_cast<float>(v[4 * half + r]);
}

__device__ __forceinline__ void silu_d(float z, float& h, float& d) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  h = z * s;
  d = s * (1.0f + z * (1.0f - s));
}

// Activations of one layer for 16*NCT cells: B operands v[kb][ct], ct = 16-cell column tile.
// Forward-only kernels use NCT = 4 (a wave's 64 cells at once); kernels that keep the
// derivatives for a backward pass use NCT = 2 and take a wave's cells in two halves, which
// keeps every value in registers.
template <int NCT>
struct Act {
  bf16x8 v[2][NCT];
};

// z = W h + b for a hidden layer with NKB K blocks; returns silu(z) as the next operand and,
// if sd != nullptr, silu'(z) in the same layout.
template <int NKB, int NCT>
__device__ __forceinline__ void hidden_layer(const uint4* fr, int f0, const float* b,
                                             const Act<NCT>& in, Act<NCT>& out, Act<NCT>* sd,
                                             int lane) {
  const int g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    f4 acc[NCT];
    const f4 b4v = bias4(b, 16 * rt + 4 * g);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = b4v;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const bf16x8 a = frag(fr, f0 + rt * NKB + kb, lane);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[ct] = mfma(a, in.v[kb][ct], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      f4 h, d;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float hr, dr;
        silu_d(acc[ct][r], hr, dr);
        h[r] = hr;
        d[r] = dr;
      }
      set_half(out.v[rt >> 1][ct], rt & 1, h);
      if (sd) set_half(sd->v[rt >> 1][ct], rt & 1, d);
    }
  }
}

// Forward pass.  x: input operands (only K block 0 is used: slots of inputs 0..4, the rest
// zero).  out[ct]: D tiles of the outputs (lanes g = 0, rows r = 0, 1 valid, rows 2, 3 zero).
// sd[3]: silu' of the hidden layers, hs[3]: the activations; either may be null.
template <int NCT>
__device__ __forceinline__ void forward(const uint4* fr, const float* bias, const Act<NCT>& x,
                                        f4 (&out)[NCT], Act<NCT>* sd, Act<NCT>* hs, int lane) {
  Act<NCT> h1, h2, h3;
  hidden_layer<1>(fr, kFrW1, bias, x, h1, sd ? &sd[0] : nullptr, lane);
  if (hs) hs[0] = h1;
  hidden_layer<2>(fr, kFrW2, bias + 64, h1, h2, sd ? &sd[1] : nullptr, lane);
  if (hs) hs[1] = h2;
  hidden_layer<2>(fr, kFrW3, bias + 128, h2, h3, sd ? &sd[2] : nullptr, lane);
  if (hs) hs[2] = h3;
  const int g = lane >> 4;
  const f4 b4v = bias4(bias + 192, 4 * g);
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    f4 acc = b4v;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) acc = mfma(frag(fr, kFrW4 + kb, lane), h3.v[kb][ct], acc);
    out[ct] = acc * kOutScale;
  }
}

// dz = (W^T dz_next) * sd for a hidden layer; dz_next given as B operands (NKB_NEXT blocks).
template <int NKB_NEXT, int NCT>
__device__ __forceinline__ void hidden_layer_vjp(const uint4* fr, int f0, const Act<NCT>& dnext,
                                                 const Act<NCT>& sd, Act<NCT>& dz, int lane) {
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    f4 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < NKB_NEXT; ++kb) {
      const bf16x8 a = frag(fr, f0 + rt * NKB_NEXT + kb, lane);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[ct] = mfma(a, dnext.v[kb][ct], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      f4 d;
#pragma unroll
      for (int r = 0; r < 4; ++r) d[r] = acc[ct][r] * half_at(sd.v[rt >> 1][ct], rt & 1, r);
      set_half(dz.v[rt >> 1][ct], rt & 1, d);
    }
  }
}

// Backward pass.  gout[ct] = dL/do in the layout of forward's out (zero outside rows 0, 1 of
// lane group 0).  dx[ct]: D tiles of dL/dx (rows = inputs: lane group 0 holds inputs 0..3 in
// r = 0..3, lane group 1 input 4 in r = 0).  If dz != nullptr, dz[l] receives dL/dz of hidden
// layer l + 1 (B-operand layout).  The bfloat16 rounding of operands is passed through as
// the identity.
template <int NCT>
__device__ __forceinline__ void backward(const uint4* fr, const Act<NCT> (&sd)[3],
                                         const f4 (&gout)[NCT], f4 (&dx)[NCT], Act<NCT>* dz,
                                         int lane) {
  // dnet = 10 dL/do as the B operand of W4^T (slots 0, 1 of lane group 0)
  Act<NCT> dn, d3, d2, d1;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    set_half(dn.v[0][ct], 0, gout[ct] * kOutScale);
    set_half(dn.v[0][ct], 1, f4{0.0f, 0.0f, 0.0f, 0.0f});
  }
  hidden_layer_vjp<1>(fr, kFrG4, dn, sd[2], d3, lane);
  if (dz) dz[2] = d3;
  hidden_layer_vjp<2>(fr, kFrG3, d3, sd[1], d2, lane);
  if (dz) dz[1] = d2;
  hidden_layer_vjp<2>(fr, kFrG2, d2, sd[0], d1, lane);
  if (dz) dz[0] = d1;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) acc = mfma(frag(fr, kFrG1 + kb, lane), d1.v[kb][ct], acc);
    dx[ct] = acc;
  }
}

// Copies the first nfrag packed fragments and the biases from global memory into LDS.
// Block-wide; the caller synchronises before use.
__device__ __forceinline__ void load_packed(const uint4* __restrict__ packed, int nfrag,
                                            uint4* fr_lds, float* bias_lds) {
  const int nv = nfrag * 64;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) fr_lds[i] = packed[i];
  const float* b = reinterpret_cast<const float*>(packed + kFrAll * 64);
  for (int i = threadIdx.x; i < kBias; i += blockDim.x) bias_lds[i] = b[i];
}

// Training targets of a cell state (FP64): o0 = ln(eps_sf / t_ff) with t_ff H0 =
// (pi/2) sqrt(a^3 / (Omega_b Delta)), o1 = ln of the two relaxed threshold gates of Sec. 2.4,
// sigmoid((Delta - Delta_c) / (w_rho Delta_c)) sigmoid((T_c - T) / (w_T T_c)), clipped at -30.
__host__ __device__ inline void closure_targets(double delta, double temp, double lna,
                                                double eps, double dc, double omega_b,
                                                double t_c, double w_rho, double w_t,
                                                double& o0, double& o1) {
  o0 = log(eps) - log(1.5707963267948966) - 1.5 * lna + 0.5 * log(omega_b * delta);
  const double y1 = (delta - dc) / (w_rho * dc);
  const double y2 = (t_c - temp) / (w_t * t_c);
  const double ls1 = fmin(y1, 0.0) - log1p(exp(-fabs(y1)));
  const double ls2 = fmin(y2, 0.0) - log1p(exp(-fabs(y2)));
  o1 = fmax(ls1 + ls2, -30.0);
}

}  // namespace mlp
}  // namespace dh

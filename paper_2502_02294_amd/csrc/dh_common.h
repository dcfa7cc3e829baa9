// Internal definitions shared by the HIP translation units of libdiffhydro.
// Device math follows the paper's method; see include/diffhydro.h for the conventions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#define DH_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t _e = (call);                                                                 \
    if (_e != hipSuccess)                                                                   \
      throw ::dh::HipError(std::string(#call) + ": " + hipGetErrorString(_e));              \
  } while (0)

#define DH_LAUNCH_CHECK() DH_HIP(hipGetLastError())

namespace dh {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

inline unsigned blocks_for(long long work, int threads) {
  return static_cast<unsigned>((work + threads - 1) / threads);
}

// ---------------------------------------------------------------------------------------
// Hydro: per-cell primitive recovery, flux along D and the relaxation split (Sec. 2.3.1).
// Q = (rho, m_x, m_y, m_z, Et) with m = a rho U and Et = a^2 rho E.
//   U = m/(a rho), e = Et/(a^2 rho) - U^2/2 floored at e_floor only inside the EOS,
//   p = (gamma-1) rho e, c_s = sqrt(gamma (gamma-1) e), freezing speed c = (|U_d| + c_s)/a,
//   F = (rho U_d / a, rho U_d U + p e_d, a U_d (Et/a^2 + p)),
//   F^R = (c Q + F)/2, F^L = (c Q - F)/2.
// Dual energy (NQ = 6): a sixth component S = (a^2 rho e) rho^(1-gamma), the entropy
// variable, with the flux S U_d / a; the EOS takes e = Et/(a^2 rho) - U^2/2 where that
// exceeds eta1 Et/(a^2 rho), else e_S = S rho^(gamma-2) / a^2 (the selection of Bryan et al.
// 1995 with the entropy form of Ryu et al. 1993).
// ---------------------------------------------------------------------------------------
// Reciprocal and square root on the hardware's approximate units (v_rcp_f32, v_sqrt_f32:
// within 1 ulp).  The hydro kernels take these in place of the correctly rounded division
// and square root, which expand to about ten instructions each; every operand here is a
// normal positive number (density, floored energy) or bounded away from zero (limiter
// denominator), and the error stays at the level of one FP32 rounding.
__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_approx(float x) { return __builtin_amdgcn_sqrtf(x); }

// Gravity source of the gas over a half kick h (operator split): m' = m + rho g h,
// Et' = Et + h g . (m + m')/2, so the internal energy is unchanged.  One function for every
// kernel that applies or recomputes it, with every rounding spelled out (explicit FMAs, no
// contraction left to the compiler), so they all round alike wherever it is inlined.
__device__ __forceinline__ void kick_cell(float rho, const float4 g4, float h, float m[3],
                                          float& et) {
  const float g[3] = {g4.x, g4.y, g4.z};
  float de = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float m0 = m[d];
    const float m1 = fmaf(__fmul_rn(rho, g[d]), h, m0);
    m[d] = m1;
    de = fmaf(__fmul_rn(0.5f, __fadd_rn(m0, m1)), g[d], de);
  }
  et = fmaf(de, h, et);
}

// Dual energy: below kDualEta1 of E the internal energy comes from the entropy; at the end of
// a step the entropy is reset from the total energy where e_E >= kDualEta2 E.
constexpr float kDualEta1 = 1e-3f;
constexpr float kDualEta2 = 0.1f;

// The dual-energy tests of one cell state Q (FP32, written on Q so that they need no a:
// a^2 rho e_E = Et - |m|^2 / (2 rho)).  Every kernel outside the sweeps that needs the
// selection takes it from here, so a cell's screening, its source term and its adjoint agree.
//   dual_total_branch: the EOS takes e_E (e_E > kDualEta1 E);
//   dual_sync_branch: the end-of-step reset of S from the total energy (e_E >= kDualEta2 E).
__device__ __forceinline__ float dual_internal(const float* q) {
  return q[4] - 0.5f * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
}
__device__ __forceinline__ bool dual_total_branch(const float* q) {
  return dual_internal(q) > kDualEta1 * q[4];
}
__device__ __forceinline__ bool dual_sync_branch(const float* q) {
  return dual_internal(q) >= kDualEta2 * q[4];
}

struct HydroK {
  float a, ia, ia2;   // scale factor, 1/a, 1/a^2
  float gm1, gg1;     // gamma-1, gamma*(gamma-1)
  float efloor;
  float gm2;          // gamma-2 (the entropy's internal energy, dual energy only)
};

__host__ __device__ inline HydroK make_hydro(float a, float gamma, float efloor) {
  HydroK k;
  k.a = a;
  k.ia = 1.0f / a;
  k.ia2 = k.ia * k.ia;
  k.gm1 = gamma - 1.0f;
  k.gg1 = gamma * (gamma - 1.0f);
  k.efloor = efloor;
  k.gm2 = gamma - 2.0f;
  return k;
}

// x^y for x > 0 on the hardware's base-2 exponential and logarithm (v_exp_f32, v_log_f32:
// about one ulp each, so a relative error of a few ulp times |y log2 x|)
__device__ __forceinline__ float pow_approx(float x, float y) {
  return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}

template <int D, int NQ = 5>
__device__ __forceinline__ void split_flux(const float* q, const HydroK& h, float* fr,
                                           float* fl) {
  const float rho = q[0];
  const float ir = rcp_approx(rho);
  const float u0 = q[1] * h.ia * ir, u1 = q[2] * h.ia * ir, u2 = q[3] * h.ia * ir;
  const float ke = 0.5f * (u0 * u0 + u1 * u1 + u2 * u2);
  float e;
  if (NQ == 6) {
    const float big = q[4] * h.ia2 * ir;
    const float e_tot = big - ke;
    e = e_tot > kDualEta1 * big ? e_tot : q[5] * h.ia2 * pow_approx(rho, h.gm2);
  } else {
    e = q[4] * h.ia2 * ir - ke;
  }
  e = fmaxf(e, h.efloor);
  const float p = h.gm1 * rho * e;
  const float cs = sqrt_approx(h.gg1 * e);
  const float ud = D == 0 ? u0 : (D == 1 ? u1 : u2);
  const float c = (fabsf(ud) + cs) * h.ia;
  float f[5];
  f[0] = rho * ud * h.ia;
  f[1] = rho * ud * u0 + (D == 0 ? p : 0.0f);
  f[2] = rho * ud * u1 + (D == 1 ? p : 0.0f);
  f[3] = rho * ud * u2 + (D == 2 ? p : 0.0f);
  f[4] = h.a * ud * (q[4] * h.ia2 + p);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    fr[k] = 0.5f * (c * q[k] + f[k]);
    fl[k] = 0.5f * (c * q[k] - f[k]);
  }
  if (NQ == 6) {
    const float f5 = q[5] * ud * h.ia;
    fr[5] = 0.5f * (c * q[5] + f5);
    fl[5] = 0.5f * (c * q[5] - f5);
  }
}

// Vector-Jacobian product of the split fluxes at q: given the adjoints gR = dL/dF^R and
// gL = dL/dF^L (NQ each), returns dL/dq = (dF^R/dq)^T gR + (dF^L/dq)^T gL
//   = 1/2 [ c s + (dc/dq)(q . s) + (dF/dq)^T d ],  s = gR + gL, d = gR - gL.
// Derivatives are those of the floored EOS (zero through e where the floor is active), of
// the branch of the dual-energy selection that the state takes, and of |U_d| with
// sign(0) = 0.
template <int D, int NQ = 5>
__device__ __forceinline__ void split_flux_vjp(const float* q, const HydroK& h, const float* s,
                                               const float* dv, float* out) {
  const float rho = q[0];
  const float ir = rcp_approx(rho);
  const float iar = h.ia * ir;
  const float u[3] = {q[1] * iar, q[2] * iar, q[3] * iar};
  const float ke = 0.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  float eraw, tot = 1.0f, rs = 0.0f;   // tot: the total energy's branch; rs = rho^(gamma-2)
  if (NQ == 6) {
    const float big = q[4] * h.ia2 * ir;
    const float e_tot = big - ke;
    tot = e_tot > kDualEta1 * big ? 1.0f : 0.0f;
    rs = pow_approx(rho, h.gm2);
    eraw = tot > 0.0f ? e_tot : q[5] * h.ia2 * rs;
  } else {
    eraw = q[4] * h.ia2 * ir - ke;
  }
  // 0 where the floor is active (its derivative), 1 elsewhere; every term is computed and
  // masked, so the function has no branches
  const float live = eraw < h.efloor ? 0.0f : 1.0f;
  const float e = fmaxf(eraw, h.efloor);
  const float p = h.gm1 * rho * e;
  const float cs = sqrt_approx(h.gg1 * e);
  const float ud = u[D];
  const float md = q[1 + D];
  const float sgn = md > 0.0f ? 1.0f : (md < 0.0f ? -1.0f : 0.0f);
  const float c = (fabsf(ud) + cs) * h.ia;

  // derivatives of e (zero when floored); the entropy's branch: e = S rho^(gamma-2) / a^2
  const float lt = live * tot;
  float er = lt * (ke - e) * ir;
  if (NQ == 6) er += live * (1.0f - tot) * h.gm2 * e * ir;
  const float liar = -lt * iar;
  float em[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) em[k] = liar * u[k];
  const float eE = lt * h.ia2 * ir;
  const float eS = NQ == 6 ? live * (1.0f - tot) * h.ia2 * rs : 0.0f;
  // pressure derivatives
  const float pr = h.gm1 * (e + rho * er);
  float pm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) pm[k] = h.gm1 * rho * em[k];
  const float pE = h.gm1 * rho * eE;
  // freezing-speed derivatives
  const float cse = live > 0.0f ? 0.5f * h.gg1 * rcp_approx(cs) : 0.0f;   // cs may be 0 if floored
  const float cr = h.ia * (-fabsf(ud) * ir + cse * er);
  float cm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) cm[k] = h.ia * ((k == D ? sgn * iar : 0.0f) + cse * em[k]);
  const float cE = h.ia * cse * eE;

  float qs = q[0] * s[0] + q[1] * s[1] + q[2] * s[2] + q[3] * s[3] + q[4] * s[4];
  if (NQ == 6) qs += q[5] * s[5];
  // (dF/dq)^T dv
  const float H = (q[4] * h.ia2 + p) * ir;
  const float vu = dv[1] * u[0] + dv[2] * u[1] + dv[3] * u[2];
  const float W = dv[1 + D] + dv[4] * h.a * ud;
  float jt[5];
  jt[0] = -ud * vu + pr * W - dv[4] * h.a * ud * H;
  float diag = dv[0] * h.ia2 + h.ia * vu + dv[4] * H;
  if (NQ == 6) {
    // F_S = S U_d / a
    const float fs = dv[5] * q[5] * h.ia;
    jt[0] -= fs * ud * ir;
    diag += fs * iar;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) jt[1 + k] = (k == D ? diag : 0.0f) + ud * h.ia * dv[1 + k] + pm[k] * W;
  jt[4] = pE * W + dv[4] * h.a * ud * h.ia2;

  const float dc[5] = {cr, cm[0], cm[1], cm[2], cE};
#pragma unroll
  for (int k = 0; k < 5; ++k) out[k] = 0.5f * (c * s[k] + dc[k] * qs + jt[k]);
  if (NQ == 6) {
    const float pS = h.gm1 * rho * eS;
    const float cS = h.ia * cse * eS;
    out[5] = 0.5f * (c * s[5] + cS * qs + pS * W + dv[5] * ud * h.ia);
  }
}

// van Leer limiter (Sec. 2.3.2): phi(x, y) = (x y + |x y|) / (x + y + eps sgn(x+y)),
// eps = 1e-20, sgn(0) = +1.  The sweeps call it on half differences, phi(a/2, b/2), written
// here on the undivided differences a, b:
//   van_leer_half(a, b) = a b / (a + b + 2 eps sgn(a+b))  where a b > 0,  0 otherwise.
// Where a b > 0, |a + b| >= 2 sqrt(a b) > 0: the guard only moves the value by at most eps/2
// in absolute terms, below any FP32 flux, and is left out.  The selection on a b > 0 is the
// function itself (an FMA-contracted x y + |x y| is not exactly zero for x y < 0); both
// sides are computed and the discarded one is never read.
constexpr float kLimEps = 1e-20f;

__device__ __forceinline__ float van_leer_half(float a, float b) {
  const float ab = a * b;
  const float r = ab * rcp_approx(a + b);
  return ab > 0.0f ? r : 0.0f;
}

// Partial derivatives of van_leer_half: (b/(a+b))^2 and (a/(a+b))^2 where a b > 0; where
// a b == 0 the derivative of |a b| is taken with sign(0) = 0, which gives half the one-sided
// slopes b/(2(a+b)) and a/(2(a+b)) (the guard keeps them finite at a = b = 0); zero where
// a b < 0.
__device__ __forceinline__ void van_leer_half_d(float a, float b, float& da, float& db) {
  const float ab = a * b;
  const float s = a + b;
  const float id = rcp_approx(s + __builtin_copysignf(2.0f * kLimEps, s));
  const float hb = b * id, ha = a * id;
  // da = hb * (hb, 1/2 or 0 as a b > 0, = 0 or < 0), db likewise with ha: one product each
  // (a zero may come out as -0)
  const float k = ab < 0.0f ? 0.0f : 0.5f;
  da = hb * (ab > 0.0f ? hb : k);
  db = ha * (ab > 0.0f ? ha : k);
}

// ---------------------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC'11): counter-based generator for the white noise and the
// star-formation uniforms.  Counter (cell, step, tag, 0), key (seed lo, seed hi).
// ---------------------------------------------------------------------------------------
constexpr uint32_t kTagWhite = 0x574E0000u;
constexpr uint32_t kTagStarform = 0x53460000u;
constexpr uint32_t kTagMlpSample = 0x4D4C0000u;   // training states of the learned closure

__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// 24 random bits plus one half, times 2^-24: u in (0,1), exact in float and double.
__host__ __device__ inline double uniform_open_d(uint32_t bits) {
  return (static_cast<double>(bits >> 8) + 0.5) * (1.0 / 16777216.0);
}
__host__ __device__ inline float uniform_open_f(uint32_t bits) {
  return (static_cast<float>(bits >> 8) + 0.5f) * (1.0f / 16777216.0f);
}

}  // namespace dh

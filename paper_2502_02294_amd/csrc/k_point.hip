// Pointwise kernels and FP64 reductions: gravity source of the gas (operator-split kick),
// stochastic star formation with supernova heating and its Gumbel-softmax relaxation
// (Sec. 2.4), the CFL speed (eq. dt), conservation sums, the flux-field loss, and the
// initial-condition helpers (Sec. 2.1); with the adjoints of the differentiable ones.
// All reductions are two-pass with a fixed order, so results are reproducible bit for bit.
#include <cmath>

#include "dh_kernels.h"
#include "dh_mlp.h"

namespace dh {

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedPer = 8;   // cells per thread in reduction kernels

__device__ __forceinline__ int wrapi(int j, int n) { return j & (n - 1); }

// block reduction of nv doubles per thread into out[v * stride + blockIdx.x], through the
// LDS scratch sh (NV kRedThreads doubles; the caller synchronises before handing in memory
// that other waves may still read)
template <int NV, bool MAX>
__device__ void block_reduce_in(double (*sh)[kRedThreads], double (&v)[NV], double* out,
                                long long stride) {
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        sh[k][threadIdx.x] = MAX ? fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + off])
                                 : sh[k][threadIdx.x] + sh[k][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k * stride + blockIdx.x] = sh[k][0];
  }
}

template <int NV, bool MAX>
__device__ void block_reduce_store(double (&v)[NV], double* out, long long stride) {
  __shared__ double sh[NV][kRedThreads];
  block_reduce_in<NV, MAX>(sh, v, out, stride);
}

// Partials of a batched reduction: value v of block b of sample s at [(v S + s) nb + b]
// (nb = gridDim.x, S = gridDim.y); returns the base for block_reduce_store's stride S nb.
__device__ __forceinline__ double* sample_partials(double* partial) {
  return partial + static_cast<long long>(blockIdx.y) * gridDim.x;
}
__device__ __forceinline__ long long partial_stride() {
  return static_cast<long long>(gridDim.y) * gridDim.x;
}
// zero partials of an inactive sample's block
template <int NV>
__device__ __forceinline__ void zero_partials(double* partial) {
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sample_partials(partial)[k * partial_stride() + blockIdx.x] = 0.0;
}

// ------------------------------------------------------------------------- gas kick
// (kick_cell, the kick of one cell, is shared with the first sweep of a step: dh_common.h)

// adjoint of kick_cell at one cell: l5 (adjoint after the kick) becomes the adjoint before
// it (the energy component is unchanged); lg = adjoint of g
__device__ __forceinline__ void kick_cell_vjp(float rho, const float m[3], const float4 gv,
                                              float h, float l5[5], float lg[3]) {
  const float g[3] = {gv.x, gv.y, gv.z};
  const float le = l5[4];
  float lr = l5[0];
  float g2 = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float lm = l5[1 + d];
    lr += h * lm * g[d];
    g2 += g[d] * g[d];
    l5[1 + d] = lm + le * h * g[d];
    lg[d] = h * rho * lm + le * (h * m[d] + h * h * rho * g[d]);
  }
  l5[0] = lr + le * 0.5f * h * h * g2;
}

__global__ void __launch_bounds__(256) gas_kick_vjp_kernel(const float* __restrict__ q,
                                                           const float4* __restrict__ g4,
                                                           float* __restrict__ lam,
                                                           float* __restrict__ lam_g,
                                                           long long nc, int nq,
                                                           const StepScal* __restrict__ tab) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  if (c >= nc || !sc.active) return;
  // the entropy of a dual-energy state passes the kick unchanged, and so does its adjoint
  q += blockIdx.y * nq * nc;
  lam += blockIdx.y * nq * nc;
  lam_g += blockIdx.y * 3 * nc;
  g4 += blockIdx.y * nc;
  const float m[3] = {q[nc + c], q[2 * nc + c], q[3 * nc + c]};
  float l5[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) l5[k] = lam[k * nc + c];
  float lg[3];
  kick_cell_vjp(q[c], m, g4[c], sc.h, l5, lg);
#pragma unroll
  for (int k = 0; k < 4; ++k) lam[k * nc + c] = l5[k];
#pragma unroll
  for (int d = 0; d < 3; ++d) lam_g[d * nc + c] = lg[d];
}

// ------------------------------------------------------------------------- source term
// Evaluated in FP64 from the FP32 state (the kernel is memory bound, and the relaxed draw
// sigma(x / tau) amplifies rounding of its argument by 1/tau).
struct SrcCell {
  double rho, ir, delta, e, eraw, temp, x, psf, s1, s2, pi0, z, u;   // ir = 1 / rho
  double rs;      // rho^(gamma-2) where e is the dual-energy entropy's (else unset)
  bool floored;
  bool tot;       // e from the total energy (always, with five components)
};

__device__ __forceinline__ double sigmoid_(double y) { return 1.0 / (1.0 + exp(-y)); }

// The uniform of cell c for the draw of the given step.
__device__ __forceinline__ double starform_uniform(long long c, const SourceArgs& a) {
  uint32_t ctr[4] = {static_cast<uint32_t>(c), a.step, kTagStarform, 0u};
  philox4x32_10(ctr, a.seed_lo, a.seed_hi);
  return uniform_open_d(ctr[0]);
}

// Screening of the relaxed draw z = sigmoid((logit pi0 + logit u) / tau): z is certainly
// below e^-109 (zero in float, and no change of the energy in float) when an FP32 estimate of
// its argument is below -110.  logit u of the 24-bit uniforms is at most
// log((1 - 2^-25) / 2^-25) < 17.33, so a cell whose estimate stays below -110 with that
// bound needs no uniform at all.  The estimate uses the hardware exp2/log2/rcp/sqrt (absolute
// error of the logit near 1e-6, against the margin of tau between -110 and -109); it is +inf
// (no screening) where the float32 probability nears underflow.
constexpr float kMaxLogitU = 17.5f;

__device__ __forceinline__ float fast_exp(float x) { return __expf(x); }
__device__ __forceinline__ float fast_log(float x) { return __logf(x); }
// 1 - exp(-x) for x >= 0, relative error below 1e-4
__device__ __forceinline__ float one_minus_exp_neg(float x) {
  return x < 1e-3f ? x * (1.0f - 0.5f * x) : 1.0f - fast_exp(-x);
}
__device__ __forceinline__ float fast_log_sigmoid(float y) {
  return fminf(y, 0.0f) - fast_log(1.0f + fast_exp(-fabsf(y)));
}
// log p - log(1 - p) from log p
__device__ __forceinline__ float fast_logit_of_log(float logp) {
  return logp - fast_log(1.0f - fast_exp(logp));
}

__device__ __forceinline__ bool screened_out(float logit_pi, float logit_u, const SourceArgs& a) {
  return (logit_pi + logit_u) / static_cast<float>(a.tau) < -110.0f;
}
__device__ __forceinline__ float logit_u_of(double u) {
  const float uf = static_cast<float>(u);
  return fast_log(uf) - fast_log(1.0f - uf);
}

// FP32 estimate of log pi0 - log(1 - pi0) of the plain source term (relaxed mode only)
template <int NQ = 5>
__device__ __forceinline__ float draw_logit_estimate(const float* q5, const SourceArgs& a) {
  if (a.mode != 2) return INFINITY;
  const float rho = q5[0];
  const float ir = rcp_approx(rho), ia = static_cast<float>(1.0 / a.a);
  const float iar = ia * ir;
  const float u0 = q5[1] * iar, u1 = q5[2] * iar, u2 = q5[3] * iar;
  float e_raw = q5[4] * ia * iar - 0.5f * (u0 * u0 + u1 * u1 + u2 * u2);
  if (NQ == 6 && !dual_total_branch(q5))
    e_raw = q5[5] * ia * ia * pow_approx(rho, static_cast<float>(a.gamma - 2.0));
  const float e = fmaxf(e_raw, static_cast<float>(a.efloor));
  const float temp = e * static_cast<float>(a.t_per_e);
  const float delta = rho * static_cast<float>(a.inv_rho_mean);
  // x = eps dt / t_ff = c_x sqrt(delta)
  const float psf = one_minus_exp_neg(static_cast<float>(a.c_x) * sqrt_approx(delta));
  if (!(psf > 1e-30f)) return INFINITY;
  const float y1 = (delta - static_cast<float>(a.delta_c)) * static_cast<float>(a.k_rho);
  const float y2 = (static_cast<float>(a.t_c) - temp) * static_cast<float>(a.k_t);
  return fast_logit_of_log(fast_log(psf) + fast_log_sigmoid(y1) + fast_log_sigmoid(y2));
}

// sigmoid(y) and log sigmoid(y) from one exponential: t = exp(-|y|),
// sigmoid = 1 / (1 + t) (y >= 0) or t / (1 + t), log sigmoid = min(y, 0) - log1p(t)
__device__ __forceinline__ void sigmoid_pair(double y, double& sig, double& log_sig) {
  const double t = exp(-fabs(y));
  sig = (y >= 0.0 ? 1.0 : t) / (1.0 + t);
  log_sig = fmin(y, 0.0) - log1p(t);
}

template <int NQ = 5>
__device__ SrcCell source_eval(const float* q5, double u, const SourceArgs& a) {
  SrcCell s;
  s.rho = q5[0];
  s.ir = 1.0 / s.rho;
  const double ir = s.ir;
  const double ia = 1.0 / a.a;
  const double u0 = q5[1] * ia * ir, u1 = q5[2] * ia * ir, u2 = q5[3] * ia * ir;
  s.eraw = q5[4] * ia * ia * ir - 0.5 * (u0 * u0 + u1 * u1 + u2 * u2);
  s.tot = NQ != 6 || dual_total_branch(q5);
  if (!s.tot) {
    s.rs = pow(s.rho, a.gamma - 2.0);
    s.eraw = q5[5] * ia * ia * s.rs;
  }
  s.floored = s.eraw < a.efloor;
  s.e = s.floored ? a.efloor : s.eraw;
  s.temp = s.e * a.t_per_e;
  s.delta = s.rho * a.inv_rho_mean;
  s.u = u;
  if (a.mode == 1) {
    s.x = 0.0;
    s.psf = 0.0;
    const double gate = (s.delta > a.delta_c && s.temp < a.t_c) ? 1.0 : 0.0;
    s.s1 = s.s2 = gate;
    s.pi0 = 0.0;
    s.z = 0.0;
    if (gate > 0.0) {   // the draw matters only where the thresholds are passed
      s.x = a.c_x * sqrt(s.delta);
      s.psf = -expm1(-s.x);
      s.pi0 = s.psf;
      s.z = s.u > 1.0 - s.pi0 ? 1.0 : 0.0;
    }
    return s;
  }
  // x = eps dt / t_ff, t_ff = (pi/2) sqrt(a^3 / (Omega_b delta))
  s.x = a.c_x * sqrt(s.delta);
  s.psf = -expm1(-s.x);
  double ls1, ls2;
  sigmoid_pair((s.delta - a.delta_c) * a.k_rho, s.s1, ls1);
  sigmoid_pair((a.t_c - s.temp) * a.k_t, s.s2, ls2);
  s.pi0 = s.psf * s.s1 * s.s2;
  const double logpi = log(s.psf) + ls1 + ls2;
  const double logit = logpi - log1p(-s.pi0);
  // logit of u: 1 - u is exact for the 24-bit uniforms
  const double noise = log(s.u / (1.0 - s.u));
  s.z = sigmoid_((logit + noise) * a.inv_tau);
  return s;
}

template <int NQ = 5>
__device__ __forceinline__ void load_q(const float* __restrict__ q, long long c, long long nc,
                                       float* q5) {
#pragma unroll
  for (int k = 0; k < NQ; ++k) q5[k] = q[k * nc + c];
}

// CFL speed of one cell, max_d (|U_d| + c_s) / a, for the FP64 block maxima: evaluated in FP32
// on the hardware reciprocal and square root (a few ulp, so the step's dt moves by ~1e-7 of
// itself against an FP64 evaluation; the maxima, their reduction and dt stay FP64); +inf
// flags a broken state.  With the dual-energy entropy (NQ = 6, gm2 = gamma - 2) c_s takes the
// selected internal energy.
template <int NQ = 5>
__device__ __forceinline__ double cell_speed(const float* q5, double a, double gg1,
                                             double efloor, float gm2 = 0.0f) {
  const float rho = q5[0];
  const float ia = static_cast<float>(1.0 / a);
  const float iar = ia * rcp_approx(rho);
  const float u0 = q5[1] * iar, u1 = q5[2] * iar, u2 = q5[3] * iar;
  const float e_raw = q5[4] * ia * iar - 0.5f * (u0 * u0 + u1 * u1 + u2 * u2);
  float e_sel = e_raw;
  if (NQ == 6 && !dual_total_branch(q5)) e_sel = q5[5] * ia * ia * pow_approx(rho, gm2);
  const float cs =
      sqrt_approx(static_cast<float>(gg1) * fmaxf(e_sel, static_cast<float>(efloor)));
  const float sp = (fmaxf(fabsf(u0), fmaxf(fabsf(u1), fabsf(u2))) + cs) * ia;
  // every component of the total energy enters e_raw, so a NaN or infinity anywhere in the
  // cell shows there (fmaxf and the floor would drop a NaN); the entropy is checked by itself
  // (a cell on the total energy's branch does not use it)
  if (!(rho > 0.0f) || !isfinite(e_raw) || !isfinite(sp) || (NQ == 6 && !isfinite(q5[5])))
    return INFINITY;
  return sp;
}

// Dual energy at the end of the closing pass (NQ = 6): the entropy gains the internal energy
// injected into the cell (e_sn, 0 if none), then is reset from the total energy where
// dual_sync_branch holds.  r1g = rho^(1-gamma).
__device__ __forceinline__ void dual_close(float* q, double e_sn, float r1g) {
  if (e_sn != 0.0) q[5] = static_cast<float>(q[5] + e_sn * static_cast<double>(r1g));
  if (dual_sync_branch(q)) q[5] = dual_internal(q) * r1g;
}

// Closing pass of a step over kRedPer cells per thread: gas half kick, optional tape copy,
// source term, CFL block maximum of the result.  !FULL (the reverse pass's recomputation):
// no star field and no CFL maxima, which only the forward run needs.  znew (optional): the
// step's draw z of every cell (0 where no star forms), for the stars' read-out on the
// particles.  sn_out (optional): the supernova energy a^2 rho z E0 of every cell is written
// there (0 where none) instead of being added to the cell, for the smoothed injection; the
// CFL maxima are then left to the injection pass (partial may be null).
// NQ = 6 (dual energy): the entropy also takes the injected energy, then the end-of-step
// reset (dual_close); with the smoothed injection both follow in the injection pass.
template <bool FULL, int NQ>
__global__ void __launch_bounds__(kRedThreads) close_step_kernel(
    const float* q_in, float* q, const float4* __restrict__ g4, float* __restrict__ star,
    float* __restrict__ q_kicked, double gg1, double* partial, long long nc,
    const StepScal* __restrict__ tab, float* __restrict__ znew, float* __restrict__ sn_out) {
  const StepScal& sc = tab[blockIdx.y];
  const bool do_max = FULL && partial != nullptr;
  if (!sc.active) {
    if (do_max) zero_partials<1>(partial);
    return;
  }
  const float h = sc.h;
  const SourceArgs& a = sc.src;
  q_in += blockIdx.y * NQ * nc;
  q += blockIdx.y * NQ * nc;
  if (q_kicked) q_kicked += blockIdx.y * NQ * nc;
  g4 += blockIdx.y * nc;
  if (FULL) star += blockIdx.y * nc;
  if (znew) znew += blockIdx.y * nc;
  if (sn_out) sn_out += blockIdx.y * nc;
  const float gm2 = static_cast<float>(a.gamma - 2.0), g1m = static_cast<float>(1.0 - a.gamma);
  double vmax[1] = {0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    float q5[NQ];
    load_q<NQ>(q_in, c, nc, q5);
    float m[3] = {q5[1], q5[2], q5[3]};
    kick_cell(q5[0], g4[c], h, m, q5[4]);
    q5[1] = m[0];
    q5[2] = m[1];
    q5[3] = m[2];
    if (q_kicked) {
#pragma unroll
      for (int k = 0; k < NQ; ++k) q_kicked[k * nc + c] = q5[k];
    }
    const float lg = a.mode != 0 ? draw_logit_estimate<NQ>(q5, a) : 0.0f;
    float zc = 0.0f, inj = 0.0f;
    double e_add = 0.0;   // energy injected into this cell
    if (a.mode != 0 && !screened_out(lg, kMaxLogitU, a)) {
      const double u = starform_uniform(c, a);
      if (!screened_out(lg, logit_u_of(u), a)) {
        const SrcCell s = source_eval<NQ>(q5, u, a);
        if (s.z != 0.0) {
          const double e_sn = a.a * a.a * s.rho * s.z * a.e0_code;
          if (sn_out) {
            inj = static_cast<float>(e_sn);
          } else {
            q5[4] = static_cast<float>(q5[4] + e_sn);
            e_add = e_sn;
          }
          if (FULL) star[c] = static_cast<float>(star[c] + s.z);
          zc = static_cast<float>(s.z);
        }
      }
    }
    if (NQ == 6 && !sn_out) dual_close(q5, e_add, pow_approx(q5[0], g1m));
    if (znew) znew[c] = zc;
    if (sn_out) sn_out[c] = inj;
#pragma unroll
    for (int k = (q == q_in ? 1 : 0); k < NQ; ++k) q[k * nc + c] = q5[k];
    if (do_max) vmax[0] = fmax(vmax[0], cell_speed<NQ>(q5, a.a, gg1, a.efloor, gm2));
  }
  if (do_max) block_reduce_store<1, true>(vmax, sample_partials(partial), partial_stride());
}

// Weighted sum of the 27 cells around (ix, iy, iz) of one sample's field f with the weights
// w(ox) w(oy) w(oz), w(0) = 1/2, w(+-1) = 1/4 (periodic): the smoothing of the supernova
// energy, and its transpose (the weights are symmetric).
__device__ __forceinline__ float smooth27(const float* __restrict__ f, unsigned ix, unsigned iy,
                                          unsigned iz, unsigned n1, int lgn) {
  const unsigned xm = (ix - 1) & n1, xp = (ix + 1) & n1;
  float acc = 0.0f;
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz) {
    const float wz = oz == 0 ? 0.5f : 0.25f;
    float accy = 0.0f;
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
      const float wy = oy == 0 ? 0.5f : 0.25f;
      const unsigned row = ((((iz + oz) & n1) << lgn) | ((iy + oy) & n1)) << lgn;
      const float r = 0.5f * f[row | ix] + 0.25f * (f[row | xm] + f[row | xp]);
      accy = fmaf(wy, r, accy);
    }
    acc = fmaf(wz, accy, acc);
  }
  return acc;
}

// Smoothed supernova injection of a step: a^2 rho E += smooth27(sn) per cell, then the CFL
// block maximum of the result (partial may be null: none).  NQ = 6: the entropy takes
// smooth27(sn) rho^(1-gamma) and the end-of-step reset (dual_close).
template <int NQ>
__global__ void __launch_bounds__(kRedThreads) sn_inject_kernel(
    const float* __restrict__ sn, float* __restrict__ q, double gg1, double* partial, int n,
    int lgn, const StepScal* __restrict__ tab) {
  const StepScal& sc = tab[blockIdx.y];
  const long long nc = 1LL << (3 * lgn);
  if (!sc.active) {
    if (partial) zero_partials<1>(partial);
    return;
  }
  const SourceArgs& a = sc.src;
  sn += blockIdx.y * nc;
  q += blockIdx.y * NQ * nc;
  const float gm2 = static_cast<float>(a.gamma - 2.0), g1m = static_cast<float>(1.0 - a.gamma);
  const unsigned n1 = static_cast<unsigned>(n - 1);
  double vmax[1] = {0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    const unsigned uc = static_cast<unsigned>(c);
    const float add = smooth27(sn, uc & n1, (uc >> lgn) & n1, uc >> (2 * lgn), n1, lgn);
    if (NQ == 6) {
      float q6[NQ];
      load_q<NQ>(q, c, nc, q6);
      q6[4] = q6[4] + add;
      dual_close(q6, add, pow_approx(q6[0], g1m));
      q[4 * nc + c] = q6[4];
      q[5 * nc + c] = q6[5];
      if (partial) vmax[0] = fmax(vmax[0], cell_speed<NQ>(q6, a.a, gg1, a.efloor, gm2));
      continue;
    }
    const float e4 = q[4 * nc + c] + add;
    q[4 * nc + c] = e4;
    if (partial) {
      float q5[5];
      load_q(q, c, nc, q5);
      q5[4] = e4;
      vmax[0] = fmax(vmax[0], cell_speed(q5, a.a, gg1, a.efloor));
    }
  }
  if (partial) block_reduce_store<1, true>(vmax, sample_partials(partial), partial_stride());
}

// Adjoint of the smoothed injection into a dual-energy state and of the end-of-step reset
// after it (sn_inject_kernel<6>), at the state the injection pass saw: q4 (the state after the
// sweeps) with the closing gas kick (g4, the table's h) applied as the closing pass applied it
// (where the injection is smoothed the source term leaves the cell's state unchanged), plus
// add = smooth27(sn).  lam: in, the adjoint after the reset; out, that after the closing pass's
// source term.  lam_add: the adjoint of each cell's smoothed energy.
__global__ void __launch_bounds__(256) inject_sync_vjp_kernel(
    const float* __restrict__ q4, const float4* __restrict__ g4, const float* __restrict__ sn,
    float* __restrict__ lam, float* __restrict__ lam_add, int n, int lgn,
    const StepScal* __restrict__ tab) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned nc = 1u << (3 * lgn);
  const StepScal& sc = tab[blockIdx.y];
  if (c >= nc || !sc.active) return;
  const SourceArgs& a = sc.src;
  const long long off = static_cast<long long>(blockIdx.y) * nc;
  q4 += 6 * off;
  g4 += off;
  sn += off;
  lam += 6 * off;
  lam_add += off;
  float q[6];
  load_q<6>(q4, c, nc, q);
  float m[3] = {q[1], q[2], q[3]};
  kick_cell(q[0], g4[c], sc.h, m, q[4]);
  q[1] = m[0];
  q[2] = m[1];
  q[3] = m[2];
  const unsigned n1 = static_cast<unsigned>(n - 1);
  const float add = smooth27(sn, c & n1, (c >> lgn) & n1, c >> (2 * lgn), n1, lgn);
  const float r1g = pow_approx(q[0], static_cast<float>(1.0 - a.gamma));
  float qp[6] = {q[0], q[1], q[2], q[3], q[4] + add, q[5]};
  if (add != 0.0f) qp[5] = static_cast<float>(q[5] + static_cast<double>(add) * r1g);
  double l[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) l[k] = lam[k * nc + c];
  if (dual_sync_branch(qp)) {
    // S' = I r1g, I = Et - |m|^2 / (2 rho)
    const double ir = 1.0 / static_cast<double>(qp[0]);
    const double msq = static_cast<double>(qp[1]) * qp[1] + static_cast<double>(qp[2]) * qp[2] +
                       static_cast<double>(qp[3]) * qp[3];
    const double i_tot = qp[4] - 0.5 * msq * ir;
    l[0] += l[5] * r1g * (0.5 * msq * ir * ir + (1.0 - a.gamma) * i_tot * ir);
#pragma unroll
    for (int d = 0; d < 3; ++d) l[1 + d] -= l[5] * r1g * qp[1 + d] * ir;
    l[4] += l[5] * r1g;
    l[5] = 0.0;
  }
  // Et' = Et + add, S' = S + add rho^(1-gamma)
  if (add != 0.0f) l[0] += l[5] * add * (1.0 - a.gamma) * r1g / static_cast<double>(q[0]);
  lam_add[c] = static_cast<float>(l[4] + l[5] * r1g);
#pragma unroll
  for (int k = 0; k < 6; ++k) lam[k * nc + c] = static_cast<float>(l[k]);
}

// out = smooth27(in) per cell (in: a field of stride in_stride per sample, out: n^3 per
// sample): the adjoint of the smoothed injection on the energy adjoint
__global__ void __launch_bounds__(256) smooth27_kernel(const float* __restrict__ in,
                                                       long long in_stride,
                                                       float* __restrict__ out, int n, int lgn,
                                                       const StepScal* __restrict__ tab) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned nc = 1u << (3 * lgn);
  if (c >= nc || !tab[blockIdx.y].active) return;
  in += blockIdx.y * in_stride;
  out += static_cast<long long>(blockIdx.y) * nc;
  const unsigned n1 = static_cast<unsigned>(n - 1);
  out[c] = smooth27(in, c & n1, (c >> lgn) & n1, c >> (2 * lgn), n1, lgn);
}

// Adjoint of the source term at one cell (state q5 before it): l5 from the adjoint after the
// source to the adjoint before; acc += dL/d(eps_sf, delta_c).  z and its derivatives are
// below 1e-47 where the draw is screened out.
// li: the adjoint of the cell's injected energy, l5[4] itself for the injection into the
// cell, that of the smoothed injection otherwise (with the dual-energy entropy: also its
// share through the entropy).  NQ = 6: T follows the selected internal energy.
template <int NQ = 5>
__device__ __forceinline__ void source_cell_vjp(const float* q5, long long c,
                                                const SourceArgs& a, float* l5, double li,
                                                double acc[2]) {
  const float lg = draw_logit_estimate<NQ>(q5, a);
  if (screened_out(lg, kMaxLogitU, a)) return;
  const double u = starform_uniform(c, a);
  if (screened_out(lg, logit_u_of(u), a)) return;
  const SrcCell s = source_eval<NQ>(q5, u, a);
  const double le = l5[4];
  const double K = a.a * a.a * a.e0_code;
  // Et' = Et + K rho z (into this cell, or spread by the smoothing)
  double lr = l5[0] + li * K * s.z;
  if (a.mode != 1 && li != 0.0) {
    const double dz = s.z * (1.0 - s.z) * a.inv_tau / (1.0 - s.pi0);   // dz / dln(pi0)
    const double coef = li * K * s.rho * dz;
    // dln p_sf / dx = 1 / expm1(x) = (1 - p_sf) / p_sf;  x ~ sqrt(rho)
    const double dlp_dx = (1.0 - s.psf) / s.psf;
    const double ir = s.ir, ia = 1.0 / a.a;
    const double dlnpi_drho_sf = dlp_dx * s.x * 0.5 * ir;
    const double dlnpi_drho_s1 = (1.0 - s.s1) * a.inv_rho_mean * a.k_rho;
    // s2 through T(e)
    const double dlnpi_dT = -(1.0 - s.s2) * a.k_t;
    const double dT = s.floored ? 0.0 : a.t_per_e;
    if (NQ == 6 && !s.tot) {
      // e = S rho^(gamma-2) / a^2
      lr += coef * (dlnpi_drho_sf + dlnpi_drho_s1 + dlnpi_dT * dT * (a.gamma - 2.0) * s.eraw * ir);
      l5[5] = static_cast<float>(l5[5] + coef * dlnpi_dT * dT * (ia * ia * s.rs));
      l5[0] = static_cast<float>(lr);
      acc[0] += coef * (dlp_dx * s.x / a.eps_sf);
      acc[1] += coef * ((1.0 - s.s1) * (-s.delta / (a.w_rho * a.delta_c * a.delta_c)));
      return;
    }
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = q5[1 + d] * ia * ir;
    const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double de_drho = (ke - s.eraw) * ir;
    lr += coef * (dlnpi_drho_sf + dlnpi_drho_s1 + dlnpi_dT * dT * de_drho);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      l5[1 + d] = static_cast<float>(l5[1 + d] + coef * dlnpi_dT * dT * (-u[d] * ia * ir));
    l5[4] = static_cast<float>(le + coef * dlnpi_dT * dT * (ia * ia * ir));
    acc[0] += coef * (dlp_dx * s.x / a.eps_sf);
    acc[1] += coef * ((1.0 - s.s1) * (-s.delta / (a.w_rho * a.delta_c * a.delta_c)));
  }
  l5[0] = static_cast<float>(lr);
}

// Adjoint of the source term and the end-of-step entropy update of a dual-energy cell
// (dual_close) at the kicked state q: l from the adjoint after the closing pass to the adjoint
// before the source term.  The draw and the injected energy are recomputed as the closing
// pass made them.
__device__ __forceinline__ void dual_close_vjp(const float* q, long long c, const SourceArgs& a,
                                               float* l, double acc[2]) {
  double e_sn = 0.0;
  if (a.mode != 0) {
    const float lg = draw_logit_estimate<6>(q, a);
    if (!screened_out(lg, kMaxLogitU, a)) {
      const double u = starform_uniform(c, a);
      if (!screened_out(lg, logit_u_of(u), a)) {
        const SrcCell s = source_eval<6>(q, u, a);
        if (s.z != 0.0) e_sn = a.a * a.a * s.rho * s.z * a.e0_code;
      }
    }
  }
  const float r1g = pow_approx(q[0], static_cast<float>(1.0 - a.gamma));
  float qp[6] = {q[0], q[1], q[2], q[3], q[4], q[5]};
  if (e_sn != 0.0) {
    qp[4] = static_cast<float>(q[4] + e_sn);
    qp[5] = static_cast<float>(q[5] + e_sn * static_cast<double>(r1g));
  }
  double ls = l[5];
  double lr = l[0], le = l[4];
  double lm[3] = {l[1], l[2], l[3]};
  if (dual_sync_branch(qp)) {
    // S' = I r1g, I = Et - |m|^2 / (2 rho), r1g = rho^(1-gamma)
    const double ir = 1.0 / static_cast<double>(qp[0]);
    const double msq = static_cast<double>(qp[1]) * qp[1] + static_cast<double>(qp[2]) * qp[2] +
                       static_cast<double>(qp[3]) * qp[3];
    const double i_tot = qp[4] - 0.5 * msq * ir;
    lr += ls * r1g * (0.5 * msq * ir * ir + (1.0 - a.gamma) * i_tot * ir);
#pragma unroll
    for (int d = 0; d < 3; ++d) lm[d] -= ls * r1g * qp[1 + d] * ir;
    le += ls * r1g;
    ls = 0.0;
  }
  l[1] = static_cast<float>(lm[0]);
  l[2] = static_cast<float>(lm[1]);
  l[3] = static_cast<float>(lm[2]);
  l[5] = static_cast<float>(ls);
  l[4] = static_cast<float>(le);
  // the injection: Et' = Et + e_sn, S' = S + e_sn r1g, e_sn = a^2 rho z E0
  if (e_sn != 0.0) lr += ls * e_sn * (1.0 - a.gamma) * r1g / static_cast<double>(q[0]);
  l[0] = static_cast<float>(lr);
  if (a.mode != 0) source_cell_vjp<6>(q, c, a, l, le + ls * r1g, acc);
}

// Adjoint of the closing pass of a step (plain source term): lam (in: adjoint after the
// source, out: before the closing gas kick), with the state q_kick before the kick;
// lam_g = adjoint of the kick's g; partials of dL/d(eps_sf|delta_c).  The kicked state, the
// source term's input, is recomputed in registers exactly as the closing pass made it (same
// operands, same arithmetic), so one pass over the cells serves both operators.
// OPEN: first the adjoint of the following step's opening gas kick (state q_open, factor of
// tab_open, the same g: its phi_n is this step's phi_{n+1}), adjoint of g into lam_g_open;
// every sample moves in both steps.
// lam_inj (optional): the adjoint of the injected energy of each cell when the injection is
// smoothed (the smoothing of the energy adjoint).
template <bool OPEN, int NQ>
__global__ void __launch_bounds__(kRedThreads) source_kick_vjp_kernel(
    const float* __restrict__ q_kick, const float4* __restrict__ g4, float* __restrict__ lam,
    float* __restrict__ lam_g, double* partial, long long nc, const StepScal* __restrict__ tab,
    const float* __restrict__ q_open, float* __restrict__ lam_g_open,
    const StepScal* __restrict__ tab_open, const float* __restrict__ lam_inj) {
  const StepScal& sc = tab[blockIdx.y];
  if (!sc.active) {
    zero_partials<2>(partial);
    return;
  }
  const SourceArgs& a = sc.src;
  const float h = sc.h;
  q_kick += blockIdx.y * NQ * nc;
  g4 += blockIdx.y * nc;
  lam += blockIdx.y * NQ * nc;
  lam_g += blockIdx.y * 3 * nc;
  if (lam_inj) lam_inj += blockIdx.y * nc;
  float h_open = 0.0f;
  if (OPEN) {
    q_open += blockIdx.y * NQ * nc;
    lam_g_open += blockIdx.y * 3 * nc;
    h_open = tab_open[blockIdx.y].h;
  }
  double acc[2] = {0.0, 0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    float q5[NQ], l5[NQ];
    load_q<NQ>(q_kick, c, nc, q5);
    load_q<NQ>(lam, c, nc, l5);
    const float4 gv = g4[c];
    if (OPEN) {
      const float mo[3] = {q_open[nc + c], q_open[2 * nc + c], q_open[3 * nc + c]};
      float lgo[3];
      kick_cell_vjp(q_open[c], mo, gv, h_open, l5, lgo);
#pragma unroll
      for (int d = 0; d < 3; ++d) lam_g_open[d * nc + c] = lgo[d];
    }
    const float m0[3] = {q5[1], q5[2], q5[3]};
    float m[3] = {q5[1], q5[2], q5[3]};
    kick_cell(q5[0], gv, h, m, q5[4]);
    q5[1] = m[0];
    q5[2] = m[1];
    q5[3] = m[2];
    if (NQ == 6 && !lam_inj)
      dual_close_vjp(q5, c, a, l5, acc);
    else if (a.mode != 0)
      source_cell_vjp<NQ>(q5, c, a, l5, lam_inj ? lam_inj[c] : l5[4], acc);
    float lg[3];
    kick_cell_vjp(q5[0], m0, gv, h, l5, lg);
#pragma unroll
    for (int k = 0; k < NQ; ++k) lam[k * nc + c] = l5[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) lam_g[d * nc + c] = lg[d];
  }
  block_reduce_store<2, false>(acc, sample_partials(partial), partial_stride());
}

// ------------------------------------------------------------------------- learned closure
// The closure replaces the star-formation probability of the source term by the network of
// dh_mlp.h: o = net(x(Q)), pi0 = (1 - exp(-exp(o0) dt)) exp(min(o1, 0)); the draw and the
// supernova energy are those of the plain term.  Each wave evaluates the network on its 64
// consecutive cells; the per-cell inputs and outputs pass through LDS.
constexpr int kStage = 8;   // floats per cell in the LDS stage

// network inputs of one cell (FP64 from the FP32 state, then FP32); NQ = 6: T of the
// internal energy the dual-energy selection takes (tot: that of the total energy), as the
// plain source term (source_eval)
template <int NQ = 5>
__device__ __forceinline__ void closure_inputs(const float* q5, const SourceArgs& a, float x[5],
                                               double& e_raw, bool& floored, bool& tot) {
  const double rho = q5[0];
  const double ir = 1.0 / rho, ia = 1.0 / a.a;
  const double u0 = q5[1] * ia * ir, u1 = q5[2] * ia * ir, u2 = q5[3] * ia * ir;
  e_raw = q5[4] * ia * ia * ir - 0.5 * (u0 * u0 + u1 * u1 + u2 * u2);
  tot = NQ != 6 || dual_total_branch(q5);
  if (!tot) e_raw = q5[5] * ia * ia * pow(rho, a.gamma - 2.0);
  floored = e_raw < a.efloor;
  const double e = floored ? a.efloor : e_raw;
  // the logarithms on the hardware's (FP32, ~1e-7 absolute): the network sees its inputs as
  // bfloat16 numbers, whose resolution is 4e-3
  x[0] = (fast_log(static_cast<float>(rho * a.inv_rho_mean)) - 4.6f) * 0.2f;
  x[1] = (fast_log(static_cast<float>(e * a.t_per_e)) - 10.4f) * 0.2f;
  x[2] = static_cast<float>((log(a.a) + 3.0) / 1.5);
  x[3] = static_cast<float>(a.eps_sf / 0.02 - 1.0);
  x[4] = static_cast<float>(a.delta_c / 100.0 - 1.0);
}

// Network inputs x[5][ld] and the plain relaxed term's targets y[2][ld] (mlp::closure_targets)
// of every cell of one sample's state: the closure trained and checked on the states a run
// visits.  NQ = 6: T of the selected internal energy.
template <int NQ>
__global__ void __launch_bounds__(256) closure_state_kernel(const float* __restrict__ q,
                                                            SourceArgs a, float* __restrict__ x,
                                                            float* __restrict__ y, long long nc,
                                                            long long ld) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  float q5[NQ], xin[5];
  load_q<NQ>(q, c, nc, q5);
  double e_raw;
  bool floored, tot;
  closure_inputs<NQ>(q5, a, xin, e_raw, floored, tot);
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k * ld + c] = xin[k];
  const double e = floored ? a.efloor : e_raw;
  double o0, o1;
  mlp::closure_targets(q5[0] * a.inv_rho_mean, e * a.t_per_e, log(a.a), a.eps_sf, a.delta_c,
                       a.omega_b, a.t_c, a.w_rho, a.w_t, o0, o1);
  y[c] = static_cast<float>(o0);
  y[ld + c] = static_cast<float>(o1);
}

// input operands of 16 NCT cells from the stage (slots 0..4 of each cell)
template <int NCT>
__device__ __forceinline__ mlp::Act<NCT> stage_operands(const float (*stage)[kStage], int lane) {
  const int g = lane >> 4, c = lane & 15;
  mlp::Act<NCT> in;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    mlp::f4 lo = {0.0f, 0.0f, 0.0f, 0.0f};
    if (g == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) lo[r] = stage[16 * ct + c][r];
    } else if (g == 1) {
      lo[0] = stage[16 * ct + c][4];
    }
    mlp::set_half(in.v[0][ct], 0, lo);
    mlp::set_half(in.v[0][ct], 1, mlp::f4{0.0f, 0.0f, 0.0f, 0.0f});
  }
  return in;
}

// Each wave of the closure kernels owns its 64 cells' slots of the LDS stage and exchanges
// values only among its own lanes, so the waves synchronise on their own: the fences order
// the wave's LDS writes before its later reads, and the waves of a block run independently
// (one wave's matrix products overlap another's scalar work).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct ClosureDraw {
  double x, psf, pi0, z, lgate;
};

// pi0 from the outputs and the draw with uniform u (FP64, as the plain term)
__device__ __forceinline__ ClosureDraw closure_draw(float o0, float o1, double u,
                                                    const SourceArgs& a) {
  ClosureDraw d;
  d.x = exp(static_cast<double>(o0)) * a.dt;
  d.psf = -expm1(-d.x);
  d.lgate = fmin(static_cast<double>(o1), 0.0);
  d.pi0 = d.psf * exp(d.lgate);
  if (a.mode == 1) {
    d.z = u > 1.0 - d.pi0 ? 1.0 : 0.0;
  } else {
    const double logit = log(d.psf) + d.lgate - log1p(-d.pi0);
    d.z = sigmoid_((logit + log(u) - log1p(-u)) / a.tau);
  }
  return d;
}

// FP32 estimate of log pi0 - log(1 - pi0) of the learned closure (relaxed mode only)
__device__ __forceinline__ float closure_logit_estimate(float o0, float o1, const SourceArgs& a) {
  if (a.mode != 2) return INFINITY;
  const float psf = one_minus_exp_neg(fast_exp(o0) * static_cast<float>(a.dt));
  if (!(psf > 1e-30f)) return INFINITY;
  return fast_logit_of_log(fast_log(psf) + fminf(o1, 0.0f));
}

// Closing pass with the learned closure (same cells per block as close_step_kernel).
// NQ = 6 (dual energy): T from the selected internal energy, the entropy takes the injected
// energy and the end-of-step reset (dual_close; with the smoothed injection, in the injection
// pass).
template <int NQ>
__global__ void __launch_bounds__(kRedThreads) close_step_mlp_kernel(
    const float* q_in, float* q, const float4* __restrict__ g4, float* __restrict__ star,
    float* __restrict__ q_kicked, double gg1, double* partial, long long nc,
    const StepScal* __restrict__ tab, float* __restrict__ znew, float* __restrict__ sn_out) {
  const StepScal& sc = tab[blockIdx.y];
  if (!sc.active) {
    if (partial) zero_partials<1>(partial);
    return;
  }
  const float h = sc.h;
  const SourceArgs& a = sc.src;
  q_in += blockIdx.y * NQ * nc;
  q += blockIdx.y * NQ * nc;
  if (q_kicked) q_kicked += blockIdx.y * NQ * nc;
  const float gm2 = static_cast<float>(a.gamma - 2.0), g1m = static_cast<float>(1.0 - a.gamma);
  g4 += blockIdx.y * nc;
  star += blockIdx.y * nc;
  if (znew) znew += blockIdx.y * nc;
  if (sn_out) sn_out += blockIdx.y * nc;
  __shared__ uint4 fr[mlp::kFrFwd * 64];
  __shared__ __attribute__((aligned(16))) float bias[mlp::kBias];
  __shared__ __attribute__((aligned(16))) float stage[kRedThreads / 64][64][kStage];
  mlp::load_packed(a.mlp, mlp::kFrFwd, fr, bias);
  __syncthreads();   // the weights; from here on every wave works on its own cells
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  double vmax[1] = {0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    const bool valid = c < nc;
    float q5[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) q5[k] = k == 0 || k >= 4 ? 1.0f : 0.0f;
    if (valid) {
      load_q<NQ>(q_in, c, nc, q5);
      float m[3] = {q5[1], q5[2], q5[3]};
      kick_cell(q5[0], g4[c], h, m, q5[4]);
      q5[1] = m[0];
      q5[2] = m[1];
      q5[3] = m[2];
      if (q_kicked) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) q_kicked[k * nc + c] = q5[k];
      }
    }
    float xin[5];
    double e_raw;
    bool floored, tot;
    closure_inputs<NQ>(q5, a, xin, e_raw, floored, tot);
#pragma unroll
    for (int k = 0; k < 5; ++k) stage[wave][lane][k] = valid ? xin[k] : 0.0f;
    wave_sync();
    mlp::f4 o[4];
    mlp::forward<4>(fr, bias, stage_operands<4>(stage[wave], lane), o, nullptr, nullptr, lane);
    if (g == 0) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        stage[wave][16 * ct + cl][5] = o[ct][0];
        stage[wave][16 * ct + cl][6] = o[ct][1];
      }
    }
    wave_sync();
    if (valid) {
      const float o0 = stage[wave][lane][5], o1 = stage[wave][lane][6];
      const float lg = closure_logit_estimate(o0, o1, a);
      const double u = screened_out(lg, kMaxLogitU, a) ? 0.5 : starform_uniform(c, a);
      float zc = 0.0f, inj = 0.0f;
      double e_add = 0.0;   // energy injected into this cell
      if (!screened_out(lg, kMaxLogitU, a) && !screened_out(lg, logit_u_of(u), a)) {
        const ClosureDraw d = closure_draw(o0, o1, u, a);
        if (d.z != 0.0) {
          const double e_sn = a.a * a.a * static_cast<double>(q5[0]) * d.z * a.e0_code;
          if (sn_out) {
            inj = static_cast<float>(e_sn);
          } else {
            q5[4] = static_cast<float>(q5[4] + e_sn);
            e_add = e_sn;
          }
          star[c] = static_cast<float>(star[c] + d.z);
          zc = static_cast<float>(d.z);
        }
      }
      if (NQ == 6 && !sn_out) dual_close(q5, e_add, pow_approx(q5[0], g1m));
      if (znew) znew[c] = zc;
      if (sn_out) sn_out[c] = inj;
#pragma unroll
      for (int k = (q == q_in ? 1 : 0); k < NQ; ++k) q[k * nc + c] = q5[k];
      if (partial) vmax[0] = fmax(vmax[0], cell_speed<NQ>(q5, a.a, gg1, a.efloor, gm2));
    }
    wave_sync();
  }
  if (partial) {
    // the stage, free once every wave is done, holds the reduction (no LDS of its own, so
    // more blocks share a CU)
    __syncthreads();
    block_reduce_in<1, true>(reinterpret_cast<double (*)[kRedThreads]>(&stage[0][0][0]), vmax,
                             sample_partials(partial), partial_stride());
  }
}

// Adjoint of the closure's source update at the kicked state q: lam (in: after, out:
// before); partial[0|1][block] = dL/d(eps_sf | delta_c), which enter through the inputs.
// Two waves per SIMD (256 registers a lane): the compiler keeps a few values in scratch, and
// the kernel still runs ~30% faster at 256^3 than with every value in registers at one wave
// per SIMD (342 registers); a third wave costs more in spills than it gains.
// NQ = 6 (dual energy): first the adjoints of the end-of-step entropy reset and of the
// entropy's share of the injection (as dual_close_vjp), then the closure's; T of the
// internal energy the selection takes.
template <int NQ>
__global__ void __launch_bounds__(kRedThreads, 2) source_vjp_mlp_kernel(
    const float* __restrict__ q, float* __restrict__ lam, double* partial, long long nc,
    const StepScal* __restrict__ tab, const float* __restrict__ lam_inj) {
  const StepScal& sc = tab[blockIdx.y];
  if (!sc.active) {
    zero_partials<2>(partial);
    return;
  }
  const SourceArgs& a = sc.src;
  q += blockIdx.y * NQ * nc;
  lam += blockIdx.y * NQ * nc;
  if (lam_inj) lam_inj += blockIdx.y * nc;
  const float g1m = static_cast<float>(1.0 - a.gamma);
  __shared__ uint4 fr[mlp::kFrAll * 64];
  __shared__ __attribute__((aligned(16))) float bias[mlp::kBias];
  __shared__ __attribute__((aligned(16))) float stage[kRedThreads / 64][64][kStage];
  mlp::load_packed(a.mlp, mlp::kFrAll, fr, bias);
  __syncthreads();   // the weights; from here on every wave works on its own cells
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const double K = a.a * a.a * a.e0_code;
  double acc[2] = {0.0, 0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    const bool valid = c < nc;
    float q5[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) q5[k] = k == 0 || k >= 4 ? 1.0f : 0.0f;
    if (valid) load_q<NQ>(q, c, nc, q5);
    float xin[5];
    double e_raw;
    bool floored, tot;
    closure_inputs<NQ>(q5, a, xin, e_raw, floored, tot);
#pragma unroll
    for (int k = 0; k < 5; ++k) stage[wave][lane][k] = valid ? xin[k] : 0.0f;
    wave_sync();
    // per half of 32 cells: the forward, dL/do of those cells (their lanes), then, if any of
    // them is nonzero, the forward again with its derivatives and the backward.  Where every
    // cell of the half is screened out (dL/do = 0) the backward would return exact zeros and
    // is skipped: its input gradients are set to zero instead.
    double le = 0.0, li = 0.0, z = 0.0;   // adjoints of the energy and of the injection
    bool loaded = false;                   // le and li read
    float l6[6];                           // NQ = 6: the cell's adjoint after the entropy's
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const float (*sh)[kStage] = stage[wave] + 32 * half;
      mlp::f4 oh[2], go[2], dx[2];
      mlp::forward<2>(fr, bias, stage_operands<2>(sh, lane), oh, nullptr, nullptr, lane);
      if (g == 0) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          stage[wave][32 * half + 16 * ct + cl][5] = oh[ct][0];
          stage[wave][32 * half + 16 * ct + cl][6] = oh[ct][1];
        }
      }
      wave_sync();
      if ((lane >> 5) == half) {
        // dL/do of this lane's cell; the lane reads and then overwrites its own slots
        double go0 = 0.0, go1 = 0.0;
        if (valid) {
          const float o0 = stage[wave][lane][5], o1 = stage[wave][lane][6];
          const float lg = closure_logit_estimate(o0, o1, a);
          const double u = screened_out(lg, kMaxLogitU, a) ? 0.5 : starform_uniform(c, a);
          const bool drawn = !screened_out(lg, kMaxLogitU, a) && !screened_out(lg, logit_u_of(u), a);
          ClosureDraw d{};
          if (drawn) {
            d = closure_draw(o0, o1, u, a);
            z = d.z;
          }
          if (NQ == 6 && lam_inj) {
            // smoothed injection: its adjoint and the reset's were taken before
#pragma unroll
            for (int k = 0; k < 6; ++k) l6[k] = lam[k * nc + c];
            le = l6[4];
            li = lam_inj[c];
            loaded = true;
          } else if (NQ == 6) {
            // the reset at the state after the injection, then the entropy's share of it
            const double e_sn = K * q5[0] * z;
            const float r1g = pow_approx(q5[0], g1m);
            float qp[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) qp[k] = q5[k];
            if (e_sn != 0.0) {
              qp[4] = static_cast<float>(q5[4] + e_sn);
              qp[5] = static_cast<float>(q5[5] + e_sn * static_cast<double>(r1g));
            }
            double lc[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) lc[k] = lam[k * nc + c];
            if (dual_sync_branch(qp)) {
              // S' = I r1g, I = Et - |m|^2 / (2 rho)
              const double ir = 1.0 / static_cast<double>(qp[0]);
              const double msq = static_cast<double>(qp[1]) * qp[1] +
                                 static_cast<double>(qp[2]) * qp[2] +
                                 static_cast<double>(qp[3]) * qp[3];
              const double i_tot = qp[4] - 0.5 * msq * ir;
              lc[0] += lc[5] * r1g * (0.5 * msq * ir * ir + (1.0 - a.gamma) * i_tot * ir);
#pragma unroll
              for (int dd = 0; dd < 3; ++dd) lc[1 + dd] -= lc[5] * r1g * qp[1 + dd] * ir;
              lc[4] += lc[5] * r1g;
              lc[5] = 0.0;
            }
            if (e_sn != 0.0) lc[0] += lc[5] * e_sn * (1.0 - a.gamma) * r1g / static_cast<double>(q5[0]);
#pragma unroll
            for (int k = 0; k < 6; ++k) l6[k] = static_cast<float>(lc[k]);
            le = l6[4];
            li = le + static_cast<double>(l6[5]) * r1g;
            loaded = true;
          }
          if (drawn) {
            if (NQ != 6) {
              le = lam[4 * nc + c];
              li = lam_inj ? lam_inj[c] : le;
              loaded = true;
            }
            if (a.mode != 1 && li != 0.0) {
              const double dz = d.z * (1.0 - d.z) / a.tau / (1.0 - d.pi0);   // dz / dln(pi0)
              const double coef = li * K * q5[0] * dz;
              go0 = coef * d.x / expm1(d.x);                // dln p_sf / do0
              go1 = o1 < 0.0f ? coef : 0.0;                  // dln gate / do1
            }
          }
        }
        stage[wave][lane][5] = static_cast<float>(go0);
        stage[wave][lane][6] = static_cast<float>(go1);
      }
      // wave-uniform: does a cell of this half have a nonzero dL/do (as stored, FP32)?
      const bool own = (lane >> 5) == half;
      const bool live = __any(own && (stage[wave][lane][5] != 0.0f || stage[wave][lane][6] != 0.0f));
      wave_sync();
      if (live) {
        mlp::Act<2> sd[3];
        mlp::forward<2>(fr, bias, stage_operands<2>(sh, lane), oh, sd, nullptr, lane);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          go[ct] = mlp::f4{0.0f, 0.0f, 0.0f, 0.0f};
          if (g == 0) {
            go[ct][0] = sh[16 * ct + cl][5];
            go[ct][1] = sh[16 * ct + cl][6];
          }
        }
        mlp::backward<2>(fr, sd, go, dx, nullptr, lane);
        wave_sync();
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          float* cellst = stage[wave][32 * half + 16 * ct + cl];
          if (g == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cellst[k] = dx[ct][k];
          } else if (g == 1) {
            cellst[4] = dx[ct][0];
          }
        }
      } else if (own) {
#pragma unroll
        for (int k = 0; k < 5; ++k) stage[wave][lane][k] = 0.0f;
      }
      wave_sync();
    }
    const double gx0 = stage[wave][lane][0], gx1 = stage[wave][lane][1];
    if (NQ == 6) {
      if (valid) {
        // Et' = Et + K rho z; x0 = (ln Delta - 4.6)/5, x1 = (ln T - 10.4)/5 with T ~ e of the
        // selected branch: e_E (rho, m, Et) or e_S = S rho^(gamma-2) / a^2 (rho, S)
        const double rho = q5[0];
        const double ir = 1.0 / rho, ia = 1.0 / a.a;
        const double ge = floored ? 0.0 : gx1 / (5.0 * e_raw);   // dL/de
        double l[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) l[k] = l6[k];
        l[0] += li * K * z + gx0 / (5.0 * rho);
        if (tot) {
          double u[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) u[d] = q5[1 + d] * ia * ir;
          const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
          l[0] += ge * (ke - e_raw) * ir;
#pragma unroll
          for (int d = 0; d < 3; ++d) l[1 + d] += ge * (-u[d] * ia * ir);
          l[4] += ge * (ia * ia * ir);
        } else {
          l[0] += ge * (a.gamma - 2.0) * e_raw * ir;
          l[5] += ge * ia * ia * pow(rho, a.gamma - 2.0);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) lam[k * nc + c] = static_cast<float>(l[k]);
      }
    } else if (valid && (z != 0.0 || gx0 != 0.0 || gx1 != 0.0)) {
      // a cell with no draw (z = 0, so dL/do = 0) and no input gradient keeps its adjoint
      if (!loaded) {
        le = lam[4 * nc + c];
        li = lam_inj ? lam_inj[c] : le;
      }
      // Et' = Et + K rho z; inputs x0 = (ln Delta - 4.6)/5, x1 = (ln T - 10.4)/5 with T ~ e
      const double rho = q5[0];
      const double ir = 1.0 / rho, ia = 1.0 / a.a;
      double u[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) u[d] = q5[1 + d] * ia * ir;
      const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      const double ge = floored ? 0.0 : gx1 / (5.0 * e_raw);   // dL/de
      lam[c] = static_cast<float>(lam[c] + li * K * z + gx0 / (5.0 * rho) + ge * (ke - e_raw) * ir);
#pragma unroll
      for (int d = 0; d < 3; ++d)
        lam[(1 + d) * nc + c] = static_cast<float>(lam[(1 + d) * nc + c] + ge * (-u[d] * ia * ir));
      lam[4 * nc + c] = static_cast<float>(le + ge * (ia * ia * ir));
    }
    if (valid) {
      acc[0] += stage[wave][lane][3] / 0.02;
      acc[1] += stage[wave][lane][4] / 100.0;
    }
    wave_sync();
  }
  // the stage, free once every wave is done, holds the reduction: 54 KB of LDS per block, so
  // three blocks (three waves per SIMD) share a CU
  static_assert(sizeof(stage) >= 2 * kRedThreads * sizeof(double), "stage too small");
  __syncthreads();
  block_reduce_in<2, false>(reinterpret_cast<double (*)[kRedThreads]>(&stage[0][0][0]), acc,
                            sample_partials(partial), partial_stride());
}

// ------------------------------------------------------------------------- CFL
template <int NQ>
__global__ void __launch_bounds__(kRedThreads) cfl_partial_kernel(const float* __restrict__ q,
                                                                  const double* __restrict__ a_cur,
                                                                  double gg1, double efloor,
                                                                  float gm2, double* partial,
                                                                  long long nc) {
  const double a = a_cur[blockIdx.y];
  q += blockIdx.y * NQ * nc;
  double v[1] = {0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    float q5[NQ];
    load_q<NQ>(q, c, nc, q5);
    v[0] = fmax(v[0], cell_speed<NQ>(q5, a, gg1, efloor, gm2));
  }
  block_reduce_store<1, true>(v, sample_partials(partial), partial_stride());
}

// single block: out[v] = reduce over in[v * stride + 0..count)
__global__ void __launch_bounds__(kRedThreads) reduce_kernel(const double* __restrict__ in,
                                                             int count, int stride, int is_max,
                                                             double* out) {
  __shared__ double sh[kRedThreads];
  const int v = blockIdx.x;
  double acc = is_max ? -INFINITY : 0.0;
  for (int i = threadIdx.x; i < count; i += kRedThreads) {
    const double x = in[static_cast<long long>(v) * stride + i];
    acc = is_max ? fmax(acc, x) : acc + x;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      sh[threadIdx.x] = is_max ? fmax(sh[threadIdx.x], sh[threadIdx.x + off])
                               : sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

// ------------------------------------------------------------------------- sums
__global__ void __launch_bounds__(kRedThreads) conservation_kernel(const float* __restrict__ q,
                                                                   const float* __restrict__ mom,
                                                                   double* partial, long long nc) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] += q[k * nc + c];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[5 + k] += mom[k * nc + c];
  }
  block_reduce_store<8, false>(v, partial, gridDim.x);
}

__global__ void __launch_bounds__(kRedThreads) loss_kernel(const float* __restrict__ rho,
                                                           const float* __restrict__ target,
                                                           double A, double beta, double irm,
                                                           double* partial, long long nc,
                                                           long long qs) {
  rho += blockIdx.y * qs;   // density row of the sample's Q
  target += blockIdx.y * nc;
  double v[1] = {0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    const double f = exp(-A * pow(rho[c] * irm, beta));
    const double d = f - target[c];
    v[0] += d * d;
  }
  block_reduce_store<1, false>(v, sample_partials(partial), partial_stride());
}

// lam_rho = scale * 2 (F - F_t) dF/drho / nc ; partial[0|1] = dL/dA, dL/dbeta
__global__ void __launch_bounds__(kRedThreads) loss_vjp_kernel(const float* __restrict__ rho,
                                                               const float* __restrict__ target,
                                                               double A, double beta, double irm,
                                                               float* __restrict__ lam_rho,
                                                               double* partial, long long nc,
                                                               long long qs) {
  rho += blockIdx.y * qs;
  target += blockIdx.y * nc;
  lam_rho += blockIdx.y * qs;
  double v[2] = {0.0, 0.0};
  const long long base = static_cast<long long>(blockIdx.x) * kRedThreads * kRedPer;
  const double w = 2.0 / static_cast<double>(nc);
  for (int r = 0; r < kRedPer; ++r) {
    const long long c = base + r * kRedThreads + threadIdx.x;
    if (c >= nc) break;
    const double dl = rho[c] * irm;
    const double db = pow(dl, beta);
    const double f = exp(-A * db);
    const double g = w * (f - target[c]) * f;
    lam_rho[c] = static_cast<float>(g * (-A * beta * db / dl) * irm);
    v[0] += g * (-db);
    v[1] += g * (-A * db * log(dl));
  }
  block_reduce_store<2, false>(v, sample_partials(partial), partial_stride());
}

__global__ void flux_kernel(const float* __restrict__ rho, double A, double beta, double irm,
                            float* __restrict__ out, long long nc) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  out[c] = static_cast<float>(exp(-A * pow(rho[c] * irm, beta)));
}

// T of one sample's cells; nq = 6: the dual-energy selection (gm2 = gamma - 2)
__global__ void temperature_kernel(const float* __restrict__ q, float a, float efloor,
                                   float t_per_e, float* __restrict__ out, long long nc, int nq,
                                   float gm2) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const float rho = q[c], ia = 1.0f / a;
  const float u0 = q[nc + c] * ia / rho, u1 = q[2 * nc + c] * ia / rho, u2 = q[3 * nc + c] * ia / rho;
  float e = q[4 * nc + c] * ia * ia / rho - 0.5f * (u0 * u0 + u1 * u1 + u2 * u2);
  if (nq == 6) {
    const float v[5] = {rho, q[nc + c], q[2 * nc + c], q[3 * nc + c], q[4 * nc + c]};
    if (!dual_total_branch(v)) e = q[5 * nc + c] * ia * ia * pow_approx(rho, gm2);
  }
  out[c] = fmaxf(e, efloor) * t_per_e;
}

// ------------------------------------------------------------------------- initial conditions
__global__ void white_noise_kernel(float* __restrict__ out, uint32_t k0, uint32_t k1,
                                   long long nc) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  uint32_t ctr[4] = {static_cast<uint32_t>(c), 0u, kTagWhite, 0u};
  philox4x32_10(ctr, k0, k1);
  const double u1 = uniform_open_d(ctr[0]), u2 = uniform_open_d(ctr[1]);
  out[c] = static_cast<float>(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

// x = q + psi, p = vfac vel (vel = psi with first-order displacements)
__global__ void ic_particles_kernel(const float* __restrict__ psi, const float* __restrict__ vel,
                                    float* __restrict__ pos, float* __restrict__ mom, float vfac,
                                    int n, long long np) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  psi += blockIdx.y * 3 * np;
  vel += blockIdx.y * 3 * np;
  pos += blockIdx.y * 3 * np;
  mom += blockIdx.y * 3 * np;
  const int l[3] = {static_cast<int>(i % n), static_cast<int>((i / n) % n),
                    static_cast<int>(i / (static_cast<long long>(n) * n))};
  const float fn = static_cast<float>(n);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float s = psi[d * np + i];
    float x = static_cast<float>(l[d]) + 0.5f + s;
    x -= fn * floorf(x / fn);
    if (x >= fn) x -= fn;
    pos[d * np + i] = x;
    mom[d * np + i] = vfac * vel[d * np + i];
  }
}

// Second-order LPT source delta2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2) from the six second
// derivatives hess[s][6][nc] in the order xx, yy, zz, xy, xz, yz
__global__ void lpt2_source_kernel(const float* __restrict__ hess, float* __restrict__ d2,
                                   long long nc) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  hess += blockIdx.y * 6 * nc;
  d2 += blockIdx.y * nc;
  const float xx = hess[c], yy = hess[nc + c], zz = hess[2 * nc + c];
  const float xy = hess[3 * nc + c], xz = hess[4 * nc + c], yz = hess[5 * nc + c];
  d2[c] = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz;
}

// adjoint of lpt2_source for one second derivative k (order as above): out = dL/dphi_k
__global__ void lpt2_source_vjp_kernel(const float* __restrict__ hess,
                                       const float* __restrict__ lam_d2, int k,
                                       float* __restrict__ out, long long nc) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  hess += blockIdx.y * 6 * nc;
  lam_d2 += blockIdx.y * nc;
  out += blockIdx.y * nc;
  const float l = lam_d2[c];
  float v;
  if (k < 3) {   // d/dphi_kk of the products: the sum of the other two diagonal entries
    const float a = hess[((k + 1) % 3) * nc + c], b = hess[((k + 2) % 3) * nc + c];
    v = l * (a + b);
  } else {
    v = -2.0f * l * hess[k * nc + c];
  }
  out[c] = v;
}

// second-order LPT: vel = psi + r psi2, psi = psi + psi2 (r = f2 / f1)
__global__ void lpt2_combine_kernel(float* __restrict__ psi, const float* __restrict__ psi2,
                                    float* __restrict__ vel, float r, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float a = psi[i], b = psi2[i];
  vel[i] = fmaf(r, b, a);
  psi[i] = a + b;
}

// nq = 6: also the dual-energy entropy S = a^2 e_init rho^(2-gamma) (g2m = 2 - gamma)
__global__ void ic_gas_kernel(const float* __restrict__ cic, const float* __restrict__ psi,
                              float* __restrict__ q, float f_b, float vfac, float a, float e_init,
                              long long nc, int nq, float g2m) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  cic += blockIdx.y * nc;
  psi += blockIdx.y * 3 * nc;
  q += blockIdx.y * nq * nc;
  const float rho = f_b * cic[c];
  q[c] = rho;
  float u2 = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float p = vfac * psi[d * nc + c];
    q[(1 + d) * nc + c] = rho * p;
    const float u = p / a;
    u2 += u * u;
  }
  q[4 * nc + c] = a * a * rho * (e_init + 0.5f * u2);
  if (nq == 6) q[5 * nc + c] = a * a * e_init * pow_approx(rho, g2m);
}

// adjoint of ic_gas: lam_cic = f_b * lam_rho_total ; lam_psi += contributions
__global__ void ic_gas_vjp_kernel(const float* __restrict__ cic, const float* __restrict__ psi,
                                  const float* __restrict__ lam, float f_b, float vfac, float a,
                                  float e_init, float* __restrict__ lam_cic,
                                  float* __restrict__ lam_psi, long long nc, int nq, float g2m) {
  const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  cic += blockIdx.y * nc;
  psi += blockIdx.y * 3 * nc;
  lam += blockIdx.y * nq * nc;
  lam_cic += blockIdx.y * nc;
  lam_psi += blockIdx.y * 3 * nc;
  const float rho = f_b * cic[c];
  const float le = lam[4 * nc + c];
  float lr = lam[c];
  float p2 = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float p = vfac * psi[d * nc + c];
    const float lm = lam[(1 + d) * nc + c];
    lr += lm * p;
    p2 += p * p;
    // Et = a^2 rho e_init + rho |p|^2 / 2
    lam_psi[d * nc + c] += vfac * (lm * rho + le * rho * p);
  }
  lr += le * (a * a * e_init + 0.5f * p2);
  // S = a^2 e_init rho^(2-gamma): dS/drho = (2-gamma) a^2 e_init rho^(1-gamma)
  if (nq == 6) lr += lam[5 * nc + c] * g2m * a * a * e_init * pow_approx(rho, g2m - 1.0f);
  lam_cic[c] = f_b * lr;
}

__global__ void fill_kernel(float* p, float v, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

}  // namespace

void launch_gas_kick_vjp(hipStream_t st, const float* q_before, const float4* g4, float* lam_q,
                         float* lam_g, const Batch& b) {
  if (!b.tab) throw ArgError("gas kick adjoint: step table required");
  hipLaunchKernelGGL(gas_kick_vjp_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st,
                     q_before, g4, lam_q, lam_g, b.nc(), b.nq, b.tab);
  DH_LAUNCH_CHECK();
}

// The closure kernels are chosen per launch: every sample of a batch has the same closure.
void launch_close_step(hipStream_t st, const float* q_in, float* q, const float4* g4,
                       float* star, float* q_kicked, double gamma, double* block_max,
                       const Batch& b, bool closure, float* znew, float* sn_out) {
  if (!b.tab) throw ArgError("closing pass: step table required");
  if ((star == nullptr && block_max != nullptr) || (closure && !star))
    throw ArgError("closing pass: CFL maxima need the star field (so does the closure)");
  if ((star == nullptr && znew != nullptr) || (block_max != nullptr && sn_out != nullptr))
    throw ArgError("closing pass: new stars need the star field; a smoothed injection takes "
                   "the CFL maxima to the injection pass");
  const dim3 grid(sum_blocks(b.nc()), b.S);
  const double gg1 = gamma * (gamma - 1.0);
#define DH_CLOSE(FULL, NQ)                                                                      \
  hipLaunchKernelGGL((close_step_kernel<FULL, NQ>), grid, dim3(kRedThreads), 0, st, q_in, q, g4, \
                     star, q_kicked, gg1, block_max, b.nc(), b.tab, znew, sn_out)
  if (closure && b.nq == 6)
    hipLaunchKernelGGL(close_step_mlp_kernel<6>, grid, dim3(kRedThreads), 0, st, q_in, q, g4, star,
                       q_kicked, gg1, block_max, b.nc(), b.tab, znew, sn_out);
  else if (closure)
    hipLaunchKernelGGL(close_step_mlp_kernel<5>, grid, dim3(kRedThreads), 0, st, q_in, q, g4, star,
                       q_kicked, gg1, block_max, b.nc(), b.tab, znew, sn_out);
  else if (b.nq == 6) {
    if (star) DH_CLOSE(true, 6);
    else DH_CLOSE(false, 6);
  } else {
    if (star) DH_CLOSE(true, 5);
    else DH_CLOSE(false, 5);
  }
#undef DH_CLOSE
  DH_LAUNCH_CHECK();
}

static int log2_int(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

void launch_sn_inject(hipStream_t st, const float* sn, float* q, double gamma, double* block_max,
                      const Batch& b) {
  if (!b.tab) throw ArgError("supernova injection: step table required");
  if (b.nq == 6)
    hipLaunchKernelGGL(sn_inject_kernel<6>, dim3(sum_blocks(b.nc()), b.S), dim3(kRedThreads), 0,
                       st, sn, q, gamma * (gamma - 1.0), block_max, b.n, log2_int(b.n), b.tab);
  else
    hipLaunchKernelGGL(sn_inject_kernel<5>, dim3(sum_blocks(b.nc()), b.S), dim3(kRedThreads), 0,
                       st, sn, q, gamma * (gamma - 1.0), block_max, b.n, log2_int(b.n), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_inject_sync_vjp(hipStream_t st, const float* q4, const float4* g4, const float* sn,
                            float* lam, float* lam_add, const Batch& b) {
  if (!b.tab) throw ArgError("injection adjoint: step table required");
  if (b.nq != 6) throw ArgError("injection adjoint: dual-energy state only");
  hipLaunchKernelGGL(inject_sync_vjp_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st,
                     q4, g4, sn, lam, lam_add, b.n, log2_int(b.n), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_smooth27(hipStream_t st, const float* in, long long in_stride, float* out,
                     const Batch& b) {
  if (!b.tab) throw ArgError("smoothing: step table required");
  hipLaunchKernelGGL(smooth27_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st, in,
                     in_stride, out, b.n, log2_int(b.n), b.tab);
  DH_LAUNCH_CHECK();
}

int sum_blocks(long long count) {
  return static_cast<int>((count + kRedThreads * kRedPer - 1) / (kRedThreads * kRedPer));
}
int source_vjp_blocks(int n) { return sum_blocks(static_cast<long long>(n) * n * n); }
int cfl_blocks(int n) { return sum_blocks(static_cast<long long>(n) * n * n); }

void launch_source_vjp(hipStream_t st, const float* q_before, float* lam_q, double* partials,
                       const Batch& b, const float* lam_inj) {
  if (!b.tab) throw ArgError("source adjoint: step table required");
  const dim3 grid(source_vjp_blocks(b.n), b.S);
  if (b.nq == 6)
    hipLaunchKernelGGL(source_vjp_mlp_kernel<6>, grid, dim3(kRedThreads), 0, st, q_before, lam_q,
                       partials, b.nc(), b.tab, lam_inj);
  else
    hipLaunchKernelGGL(source_vjp_mlp_kernel<5>, grid, dim3(kRedThreads), 0, st, q_before, lam_q,
                       partials, b.nc(), b.tab, lam_inj);
  DH_LAUNCH_CHECK();
}

void launch_source_kick_vjp(hipStream_t st, const float* q_kick, const float4* g4,
                            float* lam_q, float* lam_g, double* partials, const Batch& b,
                            const float* q_open, float* lam_g_open, const StepScal* tab_open,
                            const float* lam_inj) {
  if (!b.tab) throw ArgError("closing pass adjoint: step table required");
  if (q_open && (!lam_g_open || !tab_open))
    throw ArgError("closing pass adjoint: opening kick operands");
  const dim3 grid(source_vjp_blocks(b.n), b.S);
#define DH_SKV(OPEN, NQ)                                                                      \
  hipLaunchKernelGGL((source_kick_vjp_kernel<OPEN, NQ>), grid, dim3(kRedThreads), 0, st, q_kick, \
                     g4, lam_q, lam_g, partials, b.nc(), b.tab, q_open, lam_g_open, tab_open,    \
                     lam_inj)
  if (b.nq == 6) {
    if (q_open) DH_SKV(true, 6);
    else DH_SKV(false, 6);
  } else {
    if (q_open) DH_SKV(true, 5);
    else DH_SKV(false, 5);
  }
#undef DH_SKV
  DH_LAUNCH_CHECK();
}

void launch_cfl_partial(hipStream_t st, const float* q, const double* a_cur, double gamma,
                        double efloor, double* block_max, const Batch& b) {
  const float gm2 = static_cast<float>(gamma - 2.0);
  if (b.nq == 6)
    hipLaunchKernelGGL(cfl_partial_kernel<6>, dim3(cfl_blocks(b.n), b.S), dim3(kRedThreads), 0, st,
                       q, a_cur, gamma * (gamma - 1.0), efloor, gm2, block_max, b.nc());
  else
    hipLaunchKernelGGL(cfl_partial_kernel<5>, dim3(cfl_blocks(b.n), b.S), dim3(kRedThreads), 0, st,
                       q, a_cur, gamma * (gamma - 1.0), efloor, gm2, block_max, b.nc());
  DH_LAUNCH_CHECK();
}

void launch_reduce_max(hipStream_t st, const double* in, int count, int stride, int nvec,
                       double* out) {
  hipLaunchKernelGGL(reduce_kernel, dim3(nvec), dim3(kRedThreads), 0, st, in, count, stride, 1,
                     out);
  DH_LAUNCH_CHECK();
}

void launch_reduce_sum(hipStream_t st, const double* in, int count, int stride, int nvec,
                       double* out) {
  hipLaunchKernelGGL(reduce_kernel, dim3(nvec), dim3(kRedThreads), 0, st, in, count, stride, 0, out);
  DH_LAUNCH_CHECK();
}

void launch_conservation_partial(hipStream_t st, const float* q, const float* mom,
                                 double* partial, int nblocks, long long nc) {
  hipLaunchKernelGGL(conservation_kernel, dim3(nblocks), dim3(kRedThreads), 0, st, q, mom,
                     partial, nc);
  DH_LAUNCH_CHECK();
}

void launch_loss_partial(hipStream_t st, const float* rho, const float* target, double A,
                         double beta, float inv_rho_mean, double* partial, const Batch& b) {
  hipLaunchKernelGGL(loss_kernel, dim3(sum_blocks(b.nc()), b.S), dim3(kRedThreads), 0, st, rho,
                     target, A, beta, static_cast<double>(inv_rho_mean), partial, b.nc(), b.qs());
  DH_LAUNCH_CHECK();
}

void launch_loss_vjp(hipStream_t st, const float* rho, const float* target, double A, double beta,
                     float inv_rho_mean, float* lam_rho, double* partial, const Batch& b) {
  hipLaunchKernelGGL(loss_vjp_kernel, dim3(sum_blocks(b.nc()), b.S), dim3(kRedThreads), 0, st, rho,
                     target, A, beta, static_cast<double>(inv_rho_mean), lam_rho, partial, b.nc(),
                     b.qs());
  DH_LAUNCH_CHECK();
}

void launch_flux_field(hipStream_t st, const float* rho, double A, double beta, float inv_rho_mean,
                       float* out, long long nc) {
  hipLaunchKernelGGL(flux_kernel, dim3(blocks_for(nc, 256)), dim3(256), 0, st, rho, A, beta,
                     static_cast<double>(inv_rho_mean), out, nc);
  DH_LAUNCH_CHECK();
}

void launch_temperature(hipStream_t st, const float* q, float a, float efloor, float t_per_e,
                        float* out, long long nc, int nq, double gamma) {
  hipLaunchKernelGGL(temperature_kernel, dim3(blocks_for(nc, 256)), dim3(256), 0, st, q, a, efloor,
                     t_per_e, out, nc, nq, static_cast<float>(gamma - 2.0));
  DH_LAUNCH_CHECK();
}

void launch_white_noise(hipStream_t st, float* out, uint32_t seed_lo, uint32_t seed_hi, int n) {
  const long long nc = static_cast<long long>(n) * n * n;
  hipLaunchKernelGGL(white_noise_kernel, dim3(blocks_for(nc, 256)), dim3(256), 0, st, out, seed_lo,
                     seed_hi, nc);
  DH_LAUNCH_CHECK();
}

void launch_ic_particles(hipStream_t st, const float* psi, const float* vel, float* pos,
                         float* mom, float vfac, const Batch& b) {
  hipLaunchKernelGGL(ic_particles_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st, psi,
                     vel, pos, mom, vfac, b.n, b.nc());
  DH_LAUNCH_CHECK();
}

void launch_lpt2_source(hipStream_t st, const float* hess, float* d2, const Batch& b) {
  hipLaunchKernelGGL(lpt2_source_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st,
                     hess, d2, b.nc());
  DH_LAUNCH_CHECK();
}

void launch_lpt2_source_vjp(hipStream_t st, const float* hess, const float* lam_d2, int k,
                            float* out, const Batch& b) {
  hipLaunchKernelGGL(lpt2_source_vjp_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0,
                     st, hess, lam_d2, k, out, b.nc());
  DH_LAUNCH_CHECK();
}

void launch_lpt2_combine(hipStream_t st, float* psi, const float* psi2, float* vel, float r,
                         long long count) {
  hipLaunchKernelGGL(lpt2_combine_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, psi,
                     psi2, vel, r, count);
  DH_LAUNCH_CHECK();
}

void launch_ic_gas(hipStream_t st, const float* cic, const float* psi, float* q, float f_b,
                   float vfac, float a, float e_init, double gamma, const Batch& b) {
  hipLaunchKernelGGL(ic_gas_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st, cic, psi,
                     q, f_b, vfac, a, e_init, b.nc(), b.nq, static_cast<float>(2.0 - gamma));
  DH_LAUNCH_CHECK();
}

void launch_ic_gas_vjp(hipStream_t st, const float* cic, const float* psi, const float* lam_q,
                       float f_b, float vfac, float a, float e_init, double gamma, float* lam_cic,
                       float* lam_psi, const Batch& b) {
  hipLaunchKernelGGL(ic_gas_vjp_kernel, dim3(blocks_for(b.nc(), 256), b.S), dim3(256), 0, st, cic,
                     psi, lam_q, f_b, vfac, a, e_init, lam_cic, lam_psi, b.nc(), b.nq,
                     static_cast<float>(2.0 - gamma));
  DH_LAUNCH_CHECK();
}

void launch_closure_state(hipStream_t st, const float* q, const SourceArgs& a, float* x, float* y,
                          long long nc, long long ld, int nq) {
  if (nq == 6)
    hipLaunchKernelGGL(closure_state_kernel<6>, dim3(blocks_for(nc, 256)), dim3(256), 0, st, q, a,
                       x, y, nc, ld);
  else
    hipLaunchKernelGGL(closure_state_kernel<5>, dim3(blocks_for(nc, 256)), dim3(256), 0, st, q, a,
                       x, y, nc, ld);
  DH_LAUNCH_CHECK();
}

void launch_fill(hipStream_t st, float* p, float v, long long count) {
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, v, count);
  DH_LAUNCH_CHECK();
}

}  // namespace dh

// Host-side launchers of the HIP kernels of libdiffhydro (one stream per call).
#pragma once

#include <vector>

#include "dh_common.h"

namespace dh {

// ---- hydro (k_hydro.hip)
void launch_sweep(hipStream_t st, const float* qin, float* qout, int n, int axis, float dt,
                  const HydroK& h1, const HydroK& h2);
// lam_h_scratch: 5 n^3 floats, used by the y/z adjoints
void launch_sweep_vjp(hipStream_t st, const float* qin, const float* lam_out, float* lam_in,
                      float* lam_h_scratch, int n, int axis, float dt, const HydroK& h1,
                      const HydroK& h2);

// ---- particle mesh (k_pm.hip)
struct Bins {          // counting sort of particles by CIC base cell
  uint32_t* key;       // [np] base cell of each particle
  uint32_t* rank;      // [np] scratch: arrival rank inside its bin
  uint32_t* count;     // [nc]
  uint32_t* start;     // [nc + 1] exclusive prefix sum of count
  uint32_t* sorted;    // [np] particle ids, bins in cell order, ids ascending inside a bin
  uint32_t* block_sums;  // [scan blocks]
  float4* spos;        // [np] positions in bin order
  float4* sval;        // [np] a particle vector field in bin order (adjoint deposits)
};
size_t scan_block_count(long long nc);
void launch_keys(hipStream_t st, const float* pos, uint32_t* key, int n);
// sort by b.key (already computed for pos) and gather pos into bin order
void launch_sort(hipStream_t st, const Bins& b, const float* pos, int n);
// b.sval = v[3][np] in bin order
void launch_gather_sorted(hipStream_t st, const Bins& b, const float* v, int n);
// out = rho_gas + m_dm * CIC(sorted positions) + offset; rho_gas may be null (then 0)
void launch_deposit(hipStream_t st, const Bins& b, const float* rho_gas, float m_dm, float offset,
                    float* out, int n);
// out_accum[3][nc] += scale * CIC deposit of b.sval
void launch_deposit_vec(hipStream_t st, const Bins& b, float scale, float* out_accum, int n);
// g4 = (-grad phi, 0) by two-point central differences
void launch_grad(hipStream_t st, const float* phi, float4* g4, int n);
// g at particles: out[3][np] = CIC read-out of g4
void launch_readout_g(hipStream_t st, const float4* g4, const float* pos, float* out, int n);
// opening kick + drift (+ keys; optional copies of the new momenta and positions), closing kick
void launch_kick_drift(hipStream_t st, const float4* g4, float* pos, float* mom, uint32_t* key,
                       float h_kick, float drift_fac, float* mom_copy, float* pos_copy, int n);
void launch_kick(hipStream_t st, const float4* g4, const float* pos, float* mom, float h_kick,
                 int n);
// adjoint of p' = p + h g(x) with respect to x: lam_x += h sum_c dw/dx (g_c . lam_p')
void launch_kick_vjp_pos(hipStream_t st, const float4* g4, const float* pos,
                         const float* lam_p, float h_kick, float* lam_x, int n);
// adjoint of the deposit wrt positions: lam_x += mass sum_c lam_delta_c dw_c/dx
void launch_deposit_vjp_pos(hipStream_t st, const float* lam_delta, const float* pos,
                            float mass, float* lam_x, int n);
// y += a x, elementwise
void launch_axpy(hipStream_t st, float* y, const float* x, float a, long long count);
// lam_phi = (adjoint of the central-difference gradient) lam_g + lam_phi_in
void launch_grad_vjp(hipStream_t st, const float* lam_g, const float* lam_phi_in, float* lam_phi,
                     int n);

// ---- FFT and spectral operators (k_fft.hip)
enum SpecOp { kOpGreen = 0, kOpIcDisp = 1, kOpIcDispT = 2 };
void fft_make_twiddles(int n, std::vector<float2>& tw);
// real field -> half spectrum transformed along x and y (z pass separate)
void fft_forward_xy(hipStream_t st, const float* in, float2* spec, const float2* tw, int n);
// inverse along y, then c2r along x with a scale
void fft_inverse_yx(hipStream_t st, float2* spec, float* out, const float2* tw, int n, float scale);
// z pass: forward, Green's function (green = -(3 Om/2a)/N^3), inverse
void fft_zpass_green(hipStream_t st, float2* spec, const float2* tw, int n, float green);
void fft_zpass_forward(hipStream_t st, const float2* in, float2* out, const float2* tw, int n);
void fft_zpass_inverse(hipStream_t st, float2* spec, const float2* tw, int n);
// z pass with the initial-condition operator i k_axis T(k)/k^2 / N^3 (or its conjugate)
void fft_zpass_ic(hipStream_t st, const float2* in, float2* out, const float2* tw, int n,
                  int axis, bool transpose, double amp, double om_h, double n_s, double kphys,
                  bool forward_first, bool inverse_after, bool accumulate);

// ---- pointwise / reductions (k_point.hip)
// q_out = q_in after the half kick (q_out may equal q_in)
void launch_gas_kick(hipStream_t st, const float* q_in, float* q_out, const float4* g4, float h,
                     int n);
void launch_gas_kick_vjp(hipStream_t st, const float* q_before, const float4* g4, float h,
                         float* lam_q, float* lam_g, int n);
struct SourceArgs {   // FP64: the source term is evaluated in double precision
  double a, dt, inv_rho_mean, omega_b, efloor, t_per_e, e0_code;
  double eps_sf, delta_c, t_c, w_rho, w_t, tau;
  int mode;
  uint32_t seed_lo, seed_hi, step;
  const uint4* mlp;   // packed closure network (dh_mlp.h): pi0 from the network; null: plain
};
// closing pass of a step, from q_in (may equal q) into q: gas half kick with g4, optional copy of the kicked state to
// q_kicked (tape), source term (if a.mode != 0), FP64 block maxima of the CFL speed of the
// result at scale factor a.a into block_max[cfl_blocks(n)]
void launch_close_step(hipStream_t st, const float* q_in, float* q, const float4* g4, float h,
                       float* star, const SourceArgs& a, float* q_kicked, double gamma,
                       double* block_max, int n);
// adjoint of the source term; accumulates dL/d(eps_sf, delta_c) partials per block
void launch_source_vjp(hipStream_t st, const float* q_before, float* lam_q, const SourceArgs& a,
                       double* partials, int nblocks_out, int n);
int source_vjp_blocks(int n);
// FP64 block maxima of the CFL speed max_d (|U_d| + c_s)/a
int cfl_blocks(int n);
void launch_cfl_partial(hipStream_t st, const float* q, double a, double gamma, double efloor,
                        double* block_max, int n);
void launch_reduce_max(hipStream_t st, const double* in, int count, double* out);
void launch_reduce_sum(hipStream_t st, const double* in, int count, int stride, int nvec,
                       double* out);
int sum_blocks(long long count);
// FP64 block sums of several fields: partial[v * nblocks + b]
void launch_conservation_partial(hipStream_t st, const float* q, const float* mom,
                                 double* partial, int nblocks, long long nc);
void launch_loss_partial(hipStream_t st, const float* rho, const float* target, double A,
                         double beta, float inv_rho_mean, double* partial, int nblocks,
                         long long nc);
void launch_loss_vjp(hipStream_t st, const float* rho, const float* target, double A, double beta,
                     float inv_rho_mean, float* lam_rho, double* partial, int nblocks, long long nc);
void launch_flux_field(hipStream_t st, const float* rho, double A, double beta,
                       float inv_rho_mean, float* out, long long nc);
void launch_temperature(hipStream_t st, const float* q, float a, float efloor, float t_per_e,
                        float* out, long long nc);
void launch_white_noise(hipStream_t st, float* out, uint32_t seed_lo, uint32_t seed_hi, int n);
// IC: particles from displacement and gas from the deposit
void launch_ic_particles(hipStream_t st, const float* psi, float* pos, float* mom, float vfac,
                         int n);
void launch_ic_gas(hipStream_t st, const float* cic, const float* psi, float* q, float f_b,
                   float vfac, float a, float e_init, int n);
void launch_ic_gas_vjp(hipStream_t st, const float* cic, const float* psi, const float* lam_q,
                       float f_b, float vfac, float a, float e_init, float* lam_cic,
                       float* lam_psi, int n);
void launch_fill(hipStream_t st, float* p, float v, long long count);
void launch_check_finite(hipStream_t st, const float* q, long long nc, int* flag);

// ---- learned closure network (k_mlp.hip; layout in dh_mlp.h)
struct MlpSampleArgs {   // ranges of the training states (natural logs where named ln)
  long long first;       // index of the first sample (Philox counter)
  uint32_t seed_lo, seed_hi;
  double lnd_lo, lnd_hi, lnt_lo, lnt_hi, lna_lo, lna_hi, eps_lo, eps_hi, dc_lo, dc_hi;
  double t_c, omega_b, w_rho, w_t;
};
struct AdamArgs {
  float lr, beta1, beta2, eps;
  float corr1, corr2;    // 1 / (1 - beta^t)
  int step;
};
// packed[kFrAll * 64 fragments + biases] from the flat parameter vector
void launch_mlp_pack(hipStream_t st, const float* theta, uint4* packed);
// x[5][count] network inputs and y[2][count] targets of the plain source term
void launch_mlp_sample(hipStream_t st, const MlpSampleArgs& p, float* x, float* y, long long count);
// out[2][count] = network(x[5][count])
void launch_mlp_eval(hipStream_t st, const uint4* packed, const float* x, float* out,
                     long long count);
// gx[5][count] = (d out / d x)^T gout[2][count]
void launch_mlp_vjp(hipStream_t st, const uint4* packed, const float* x, const float* gout,
                    float* gx, long long count);
// per-wave partial gradients partial[mlp_train_parts(batch)][kParams] and loss sums of the
// objective mean_s sum_k (o_k - y_k)^2 over samples (start + i) mod n_data, i < batch
int mlp_train_parts(long long batch);
void launch_mlp_train_grad(hipStream_t st, const uint4* packed, const float* x, const float* y,
                           long long n_data, long long start, long long batch, float* partial,
                           double* loss_part);
void launch_mlp_reduce_grad(hipStream_t st, const float* partial, int nparts,
                            const double* loss_part, double loss_scale, double* grad,
                            double* loss_out);
void launch_mlp_adam(hipStream_t st, const float* partial, int nparts, const double* loss_part,
                     double loss_scale, float* theta, float* m, float* v, const AdamArgs& a,
                     double* loss_hist);

}  // namespace dh

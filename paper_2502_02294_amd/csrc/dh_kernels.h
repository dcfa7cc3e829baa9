// Host-side launchers of the HIP kernels of libdiffhydro (one stream per call).
#pragma once

#include <vector>

#include "dh_common.h"

namespace dh {

// ---- batches
// A handle holds S independent samples of n^3 cells and n^3 particles, stacked: every array
// is S consecutive copies of its single-sample layout.  A launch covers all samples (the
// sample is blockIdx.y, blockIdx.z in the pencil passes).  The per-sample scalars of a step
// come from a device table of S entries; a sample whose entry is not active is left as it
// is (kernels that write a separate output copy their input there, the identity of the
// step).  tab == nullptr: every sample active, no step scalars used.
struct SourceArgs {   // FP64: the source term is evaluated in double precision
  double a, dt, inv_rho_mean, omega_b, efloor, t_per_e, e0_code;
  double gamma;       // adiabatic index (the dual-energy entropy's powers of rho)
  double eps_sf, delta_c, t_c, w_rho, w_t, tau;
  // per-step constants: x = eps_sf dt / t_ff = c_x sqrt(delta) with
  // t_ff = (pi/2) sqrt(a^3 / (omega_b delta)); gate arguments (delta - delta_c) k_rho and
  // (t_c - T) k_t, k_rho = 1 / (w_rho delta_c), k_t = 1 / (w_t t_c); inv_tau = 1 / tau
  double c_x, k_rho, k_t, inv_tau;
  int mode;
  uint32_t seed_lo, seed_hi, step;
  const uint4* mlp;   // packed closure network (dh_mlp.h): pi0 from the network; null: plain
};
struct StepScal {
  SourceArgs src;     // source term at a(t+dt)
  HydroK h1, h2;      // sweep stages at a(t) and a(t+dt/2)
  float dt, h;        // step length, half kick of the gas (dt/2)
  float h_open;       // opening dark-matter kick factor (dt/2, or FastPM's growth-factor one)
  float h_close;      // closing dark-matter kick factor (likewise)
  float drift;        // dark-matter drift factor: dt / a(t+dt/2)^2, or FastPM's
  float green;        // Poisson: -(3 Om / 2 a(t+dt)) / N^3
  float h_dm;         // reverse pass: closing dark-matter kick of this step + opening of the next
  float h_prev;       // closing dark-matter kick of the sample's previous step, when deferred
  int active;
};
struct Batch {
  int n;                 // cells per side of one sample
  int S;                 // samples
  const StepScal* tab;   // device table [S] or null
  int nq = 5;            // gas components per cell: 5, or 6 with the dual-energy entropy
  long long nc() const { return static_cast<long long>(n) * n * n; }
  long long qs() const { return nq * nc(); }   // floats of one sample's gas state
};

__device__ __forceinline__ bool sample_active(const StepScal* tab, int smp) {
  return tab == nullptr || tab[smp].active != 0;
}

// ---- hydro (k_hydro.hip): one sweep with dt, h1, h2 of the table (tab required)
// With g4 (the first sweep of a step): the opening gas half kick (the table's h) is applied
// to each cell as it is loaded.
void launch_sweep(hipStream_t st, const float* qin, float* qout, const Batch& b, int axis,
                  const float4* g4 = nullptr);
// adjoint of one sweep: lam_in = (dU'/dU)^T lam_out at U = qin (not in place); with g4 (the
// first sweep of a step) U is qin after the opening gas half kick, applied again on load
void launch_sweep_vjp(hipStream_t st, const float* qin, const float* lam_out, float* lam_in,
                      const Batch& b, int axis, const float4* g4 = nullptr);

// ---- particle mesh (k_pm.hip)
// Keys are global bins: sample * n^3 + CIC base cell, so one counting sort orders the
// particles of every sample.
struct Bins {          // counting sort of particles by CIC base cell
  uint32_t* key;       // [S np] bin of each particle
  uint32_t* rank;      // [S np] scratch: arrival rank inside its bin
  uint32_t* count;     // [S nc]
  uint32_t* start;     // [S nc + 1] exclusive prefix sum of count
  uint32_t* sorted;    // [S np] particle ids, bins in order, ids ascending inside a bin
  uint32_t* block_sums;  // [scan blocks]
  uint32_t* large;     // [1 + large_bin_capacity(total)]: count, then bins of many particles
  float4* spos;        // [S np] positions in bin order
  float4* sval;        // [S np] a particle vector field in bin order (adjoint deposits)
};
size_t scan_block_count(long long nbins);
// entries of Bins::large for `total` particles (bins of more than 32 particles)
long long large_bin_capacity(long long total);
void launch_keys(hipStream_t st, const float* pos, uint32_t* key, const Batch& b);
// aux[id] += CIC read-out of znew at each particle (bin order: spos, sorted of the positions
// at the end of the step; samples that sit the step out are skipped)
void launch_star_readout(hipStream_t st, const float* znew, const float4* spos,
                         const uint32_t* sorted, float* aux, const Batch& b);
// sort by bins.key (already computed for pos) and gather pos into bin order; counted: the
// histogram was made by launch_kick_drift (count_into)
void launch_sort(hipStream_t st, const Bins& bins, const float* pos, const Batch& b,
                 bool counted = false);
// bins.sval = v[3][np] (per sample) in bin order
void launch_gather_sorted(hipStream_t st, const Bins& bins, const float* v, const Batch& b);
// out = rho_gas + m_dm * CIC(sorted positions) + offset; rho_gas (sample s at
// rho_gas + s * rho_stride: 5 n^3 for the density row of Q) may be null (then 0)
void launch_deposit(hipStream_t st, const Bins& bins, const float* rho_gas,
                    long long rho_stride, float m_dm, float offset, float* out, const Batch& b);
// out_accum[3][nc] += scale * CIC deposit of bins.sval, scale = h_open (merged: h_dm) of the
// table
void launch_deposit_vec(hipStream_t st, const Bins& bins, bool merged, float* out_accum,
                        const Batch& b);
// g4 = (-grad phi, 0) by two-point central differences
void launch_grad(hipStream_t st, const float* phi, float4* g4, const Batch& b);
// g at particles: out[3][np] = CIC read-out of g4
void launch_readout_g(hipStream_t st, const float4* g4, const float* pos, float* out,
                      const Batch& b);
// opening kick (h_open) + drift (drift) + keys: positions read from pos_in and written to pos
// (the same array for an update in place); optional copies of the new momenta and positions.
// prev: first the previous step's closing kick (h_prev of the table), as launch_kick would.
// count_into (optional, key == count_into->key): also the histogram of the following
// launch_sort(..., counted = true) (count zeroed here, arrival ranks)
void launch_kick_drift(hipStream_t st, const float4* g4, const float* pos_in, float* pos,
                       float* mom, uint32_t* key, float* mom_copy, float* pos_copy, bool prev,
                       const Batch& b, const Bins* count_into = nullptr);
// closing kick p += h_close g(x)
void launch_kick(hipStream_t st, const float4* g4, const float* pos, float* mom, const Batch& b);
// adjoint of p' = p + k g(x) with respect to x: lam_x += k sum_c dw/dx (g_c . lam_p'), with
// k = h_open (merged: h_dm) of the table
void launch_kick_vjp_pos(hipStream_t st, const float4* g4, const float* pos,
                         const float* lam_p, bool merged, float* lam_x, const Batch& b);
// adjoint of the deposit wrt positions: lam_x += mass sum_c lam_delta_c dw_c/dx; with lam_p
// (table required), first (with g4) the merged kicks' term of launch_kick_vjp_pos and last
// the drift's adjoint lam_p += drift lam_x
void launch_deposit_vjp_pos(hipStream_t st, const float* lam_delta, const float* pos,
                            float mass, float* lam_x, float* lam_p, const float4* g4,
                            const Batch& b);
// y[s] += a x[s] over `count` values per sample (strides ys, xs); a times the table's drift
// factor if by_drift
void launch_axpy(hipStream_t st, float* y, const float* x, float a, long long count,
                 long long ys, long long xs, bool by_drift, const Batch& b);
// lam_phi = (adjoint of the central-difference gradient) lam_g + lam_phi_in
void launch_grad_vjp(hipStream_t st, const float* lam_g, const float* lam_phi_in, float* lam_phi,
                     const Batch& b);
// lam_phi = the launch above for lam_g0 alone (lam_phi_in null), then for lam_g with that as
// lam_phi_in, in one pass (the same roundings)
void launch_grad_vjp2(hipStream_t st, const float* lam_g0, const float* lam_g, float* lam_phi,
                      const Batch& b);

// ---- FFT and spectral operators (k_fft.hip)
enum SpecOp {
  kOpGreen = 0, kOpIcDisp = 1, kOpIcDispT = 2, kOpIcHess = 3, kOpZa = 4, kOpZaT = 5
};
// An initial-condition operator of the z pass: op, axes, the spectrum (amplitude
// A D^2 / V_cell, n_s, Omega_m h, n / box, transfer function) and a scale for kOpZa(T)
struct IcOp {
  int op = kOpIcDisp, axis = 0, axis2 = 0;
  double amp = 0, n_s = 1, om_h = 1, kphys = 1, scale = 1;
  bool eh = false;
  double eh_theta2 = 1, eh_alpha = 1, eh_ks = 0;
};
void fft_make_twiddles(int n, std::vector<float2>& tw);
// real field -> half spectrum transformed along x and y (z pass separate); sample s of the
// input starts at in + s * in_stride (default n^3)
void fft_forward_xy(hipStream_t st, const float* in, float2* spec, const float2* tw,
                    const Batch& b, long long in_stride = -1);
// inverse along y, then c2r along x with a scale; sample s of the output at out + s out_stride
void fft_inverse_yx(hipStream_t st, float2* spec, float* out, const float2* tw, float scale,
                    const Batch& b, long long out_stride = -1);
// z pass: forward, Green's function (the table's green), inverse
void fft_zpass_green(hipStream_t st, float2* spec, const float2* tw, const Batch& b);
void fft_zpass_forward(hipStream_t st, const float2* in, float2* out, const float2* tw,
                       const Batch& b);
void fft_zpass_inverse(hipStream_t st, float2* spec, const float2* tw, const Batch& b);
// z pass with an initial-condition operator (IcOp; the 1/N^3 of the inverse included)
void fft_zpass_ic(hipStream_t st, const float2* in, float2* out, const float2* tw,
                  const IcOp& op, bool forward_first, bool inverse_after, bool accumulate,
                  const Batch& b);

// ---- observables of Sec. 3 (k_observe.hip)
// per-block sums of w |X|^2 by bin of the rounded |m| (bins 1..nbins) of a half spectrum
// [S][n][n][n/2+1]: partial[(s nbins + b) pk_blocks(n) + block]
int pk_blocks(int n);
void launch_pk_bin(hipStream_t st, const float2* spec, int nbins, double* partial, const Batch& b);
// spec[s][m] *= g[s][bin(m) - 1] (0 outside bins 1..nbins)
void launch_pk_scale(hipStream_t st, float2* spec, const float* g, int nbins, const Batch& b);
// field-level loss 1/2 sum (d - O)^2 / N + 1/2 sum w^2, O = rho irm T(e): per-block partials
// partial[s fli_blocks(nc) + block] (partial may be null) and, with lam, dL/dQ of the data
// term into lam[s][nq][nc]; a_cur[s] the scale factor of each sample (device)
int fli_blocks(long long nc);
void launch_fli(hipStream_t st, const float* q, const float* data, const float* nvar,
                const float* white, const double* a_cur, double irm, double efloor,
                double t_per_e, double gamma, double* partial, float* lam, const Batch& b);
void launch_fli_obs(hipStream_t st, const float* q, double a, double irm, double efloor,
                    double t_per_e, float* out, long long nc, int nq, double gamma);

// ---- pointwise / reductions (k_point.hip)
// (the opening gas half kick is applied inside the first sweep of a step: launch_sweep)
void launch_gas_kick_vjp(hipStream_t st, const float* q_before, const float4* g4, float* lam_q,
                         float* lam_g, const Batch& b);
// closing pass of a step, from q_in (may equal q) into q: gas half kick with g4, optional
// copy of the kicked state to q_kicked (tape), source term (if src.mode != 0; with the
// learned closure if `closure`), FP64 block maxima of the CFL speed of the result at src.a
// into block_max[S][cfl_blocks(n)].  star and block_max both null (plain source only): the
// star field and the CFL maxima are skipped (the reverse pass's recomputation).  znew: the
// step's draw of every cell (0 where none; needs star).  sn_out: the supernova energy of
// every cell goes there instead of into the cell (for launch_sn_inject; block_max null).
void launch_close_step(hipStream_t st, const float* q_in, float* q, const float4* g4,
                       float* star, float* q_kicked, double gamma, double* block_max,
                       const Batch& b, bool closure, float* znew = nullptr,
                       float* sn_out = nullptr);
// smoothed supernova injection: a^2 rho E += the 27-cell smoothing of sn (weights 1/2, 1/4 per
// axis), then the CFL block maxima as launch_close_step (block_max may be null); with the
// dual-energy state the entropy takes its share and the end-of-step reset follows
void launch_sn_inject(hipStream_t st, const float* sn, float* q, double gamma, double* block_max,
                      const Batch& b);
// out[s][n^3] = the same smoothing of in (sample stride in_stride): its adjoint
void launch_smooth27(hipStream_t st, const float* in, long long in_stride, float* out,
                     const Batch& b);
// dual-energy state: adjoint of the smoothed injection and the reset after it, at q4 (the state
// after the sweeps) with the closing gas kick (g4) and the step's injection field sn; lam
// updated in place, lam_add[s][n^3] = adjoint of each cell's smoothed energy
void launch_inject_sync_vjp(hipStream_t st, const float* q4, const float4* g4, const float* sn,
                            float* lam, float* lam_add, const Batch& b);
// adjoint of the source term with the learned closure; dL/d(eps_sf, delta_c) partials per
// block: partials[(v S + s) nb + block], nb = source_vjp_blocks(n).  lam_inj: adjoint of
// each cell's injected energy when the injection is smoothed (null: the energy adjoint).
void launch_source_vjp(hipStream_t st, const float* q_before, float* lam_q, double* partials,
                       const Batch& b, const float* lam_inj = nullptr);
// adjoint of the closing pass with the plain source term (or none, src.mode 0) from the
// state q_kick before the closing gas half kick with g4 (the kicked state is recomputed):
// the source, then the kick (lam_g = adjoint of g), in one pass; partials as
// launch_source_vjp (zeros without source).  With q_open: first the adjoint of the next
// step's opening gas kick (its start state q_open, table tab_open, the same g4; every sample
// active in both steps), its adjoint of g into lam_g_open.
void launch_source_kick_vjp(hipStream_t st, const float* q_kick, const float4* g4,
                            float* lam_q, float* lam_g, double* partials, const Batch& b,
                            const float* q_open = nullptr, float* lam_g_open = nullptr,
                            const StepScal* tab_open = nullptr, const float* lam_inj = nullptr);
int source_vjp_blocks(int n);
// FP64 block maxima of the CFL speed max_d (|U_d| + c_s)/a with a = a_cur[s]:
// block_max[s][cfl_blocks(n)]
int cfl_blocks(int n);
void launch_cfl_partial(hipStream_t st, const float* q, const double* a_cur, double gamma,
                        double efloor, double* block_max, const Batch& b);
// out[v] = max (or sum) of in[v * stride + 0..count), v < nvec
void launch_reduce_max(hipStream_t st, const double* in, int count, int stride, int nvec,
                       double* out);
void launch_reduce_sum(hipStream_t st, const double* in, int count, int stride, int nvec,
                       double* out);
int sum_blocks(long long count);
// FP64 block sums of several fields of one sample: partial[v * nblocks + b]
void launch_conservation_partial(hipStream_t st, const float* q, const float* mom,
                                 double* partial, int nblocks, long long nc);
// flux-field loss: partial[s nb + block], nb = sum_blocks(nc)
void launch_loss_partial(hipStream_t st, const float* rho, const float* target, double A,
                         double beta, float inv_rho_mean, double* partial, const Batch& b);
// lam_rho = dL/drho (per sample, mean over the sample's cells); dL/d(A, beta) partials
// [(v S + s) nb + block]
void launch_loss_vjp(hipStream_t st, const float* rho, const float* target, double A, double beta,
                     float inv_rho_mean, float* lam_rho, double* partial, const Batch& b);
void launch_flux_field(hipStream_t st, const float* rho, double A, double beta,
                       float inv_rho_mean, float* out, long long nc);
// T of one sample's state q (nq components; 6: the dual-energy selection)
void launch_temperature(hipStream_t st, const float* q, float a, float efloor, float t_per_e,
                        float* out, long long nc, int nq, double gamma);
void launch_white_noise(hipStream_t st, float* out, uint32_t seed_lo, uint32_t seed_hi, int n);
// IC: particles from displacement and gas from the deposit
// x = q + psi, p = vfac vel (vel = psi for first-order displacements)
void launch_ic_particles(hipStream_t st, const float* psi, const float* vel, float* pos,
                         float* mom, float vfac, const Batch& b);
// second-order LPT: delta2 from the six second derivatives hess[s][6][nc] (xx, yy, zz, xy, xz,
// yz), its adjoint for derivative k, and vel = psi + r psi2, psi += psi2 over count values
void launch_lpt2_source(hipStream_t st, const float* hess, float* d2, const Batch& b);
void launch_lpt2_source_vjp(hipStream_t st, const float* hess, const float* lam_d2, int k,
                            float* out, const Batch& b);
void launch_lpt2_combine(hipStream_t st, float* psi, const float* psi2, float* vel, float r,
                         long long count);
// (b.nq = 6: also the dual-energy entropy of e_init)
void launch_ic_gas(hipStream_t st, const float* cic, const float* psi, float* q, float f_b,
                   float vfac, float a, float e_init, double gamma, const Batch& b);
void launch_ic_gas_vjp(hipStream_t st, const float* cic, const float* psi, const float* lam_q,
                       float f_b, float vfac, float a, float e_init, double gamma, float* lam_cic,
                       float* lam_psi, const Batch& b);
void launch_fill(hipStream_t st, float* p, float v, long long count);
// network inputs x[5][ld] and plain targets y[2][ld] of the nc cells of one sample's state q
// (nq components), at the scale factor and parameters of a
void launch_closure_state(hipStream_t st, const float* q, const SourceArgs& a, float* x, float* y,
                          long long nc, long long ld, int nq);

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

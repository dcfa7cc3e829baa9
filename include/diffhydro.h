/*
 * diffhydro.h -- C ABI of the MI355X (gfx950) implementation of one time step of
 * differentiable cosmological hydrodynamics (Horowitz & Lukic, arXiv:2502.02294), with its
 * reverse-mode pass.
 *
 * The method (paper Sec. 2): gas obeys the comoving Euler equations in conservation form
 * (eq. cont, eq. momentum, eq. ev, eq. conservation), solved with the relaxing TVD scheme,
 * a two-stage Runge-Kutta step (eq. TVD_halfstep, eq. TVD_fullstep), the van Leer limiter
 * and Strang dimensional splitting (Sec. 2.3.1-2.3.2); dark matter is evolved by a
 * particle-mesh solver with kick-drift-kick leapfrog (Sec. 2.2, eq. dm_hamil); the global
 * time step follows the CFL condition (eq. dt) or a predefined schedule (Sec. 2.3.3); a
 * stochastic star-formation source term injects supernova energy, relaxed by the binary
 * Gumbel-softmax for differentiation (Sec. 2.4, eq. gumbelsoftmax); the initial state is a
 * Gaussian random field with Zel'dovich displacements (Sec. 2.1).
 *
 * Conventions
 *  - Every call returns int: DH_OK (0) or a negative DH_E_* code; dh_last_error() then
 *    holds a message.  No C++ exception crosses this boundary.
 *  - Device pointers ("d_" prefix) are caller-owned, contiguous, on the handle's device,
 *    and are only read or written during the call's stream work; host pointers likewise.
 *    The library owns every internal buffer, the checkpoints and the reverse-mode tape.
 *  - Grid fields are float32 arrays of n^3 values indexed (z*n + y)*n + x (x fastest).
 *    Particle fields are float32 structure-of-arrays [3][n^3] (x, y, z components), in
 *    particle order id = (z*n + y)*n + x of the initial lattice.
 *  - Units: length in cells (comoving), time in 1/H0, velocities in cells*H0, i.e.
 *    100*box/n km/s.  Gas state Q = (rho, a rho U_x, a rho U_y, a rho U_z, a^2 rho E) with
 *    mean gas density Omega_b/Omega_m and mean total matter density 1 per cell.
 *  - Work is enqueued on the handle's stream (dh_set_stream, default the null stream).
 *    Calls that return host scalars synchronise that stream; others are asynchronous.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - Batches: a handle created with cfg.batch = S > 1 holds S independent samples of the
 *    same size and cosmology (the parameter sampler).  Every device array exchanged with
 *    the handle then holds S consecutive single-sample arrays, every per-sample host output
 *    S values (documented per call), and every kernel launch covers all samples at once.
 *    Sample s uses white-noise seed (seed + s) in dh_init_from_seed and star-formation key
 *    (sf_seed + s).  The samples step in lockstep: each has its own dt (its own CFL or
 *    schedule); one that has reached its end sits out the remaining steps unchanged.
 */
#ifndef DIFFHYDRO_H
#define DIFFHYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DH_OK = 0,
    DH_E_INVAL = -1,      /* bad argument (size, null pointer, out-of-range option) */
    DH_E_OOM = -2,        /* device or host allocation failed */
    DH_E_HIP = -3,        /* a HIP runtime call failed */
    DH_E_NONFINITE = -4,  /* non-finite or non-positive density found in the state */
    DH_E_SCHEDULE = -5,   /* a replayed schedule entry is not a positive finite dt, or a
                             replayed step exceeds the Courant number cfg.cfl_forward */
    DH_E_STATE = -6       /* call out of order (e.g. backward before forward) */
};

enum { DH_SUBGRID_OFF = 0, DH_SUBGRID_HARD = 1, DH_SUBGRID_RELAXED = 2 };

/* Star-formation probability of the source term: the plain formula (Sec. 2.4.1) or the
 * learned closure (a small network standing in for it, in the spirit of the learned
 * sub-grid models of Sec. 4; see dh_mlp_* below).  The draw and the supernova energy are
 * the same in both. */
enum { DH_CLOSURE_PLAIN = 0, DH_CLOSURE_MLP = 1 };

/* Kick and drift factors of the dark matter's kick-drift-kick step: the leapfrog in t (kicks
 * dt/2, drift dt / a(t+dt/2)^2), or the growth-factor factors of FastPM that the paper's
 * particle mesh uses (Sec. 2.2), exact for the linear growing mode: with D the growth factor,
 * G = a^2 dD/dt and F = dG/dt = (3 Om / 2a) D, opening kick (G(a_half) - G(a0)) / F(a0),
 * drift (D(a1) - D(a0)) / G(a_half), closing kick (G(a1) - G(a_half)) / F(a1).  The gas
 * kicks are dt/2 in both. */
enum { DH_KDK_PLAIN = 0, DH_KDK_FASTPM = 1 };

/* Matter transfer function of the initial spectrum P(k) = A k^n_s T(k)^2 (Sec. 2.1): BBKS of
 * q = k / (Omega_m h), or the Eisenstein & Hu (1998) fitting formula without the baryon
 * oscillations, which the paper's family of initial conditions uses. */
enum { DH_TRANSFER_BBKS = 0, DH_TRANSFER_EH = 1 };

/* Run configuration.  dh_config_default() fills the values of the paper's workloads. */
typedef struct dh_config {
    int32_t n;           /* cells per side; power of two, 16..256                        */
    double box;          /* comoving box side [Mpc/h]                                     */
    double omega_m, omega_b, h, sigma8, n_s;   /* flat LambdaCDM, BBKS spectrum          */
    double gamma;        /* adiabatic index (5/3)                                         */
    double mu;           /* mean molecular weight used only for T <-> e                   */
    double a_init;       /* initial scale factor                                          */
    double t_init;       /* initial gas temperature [K]                                   */
    double cfl;          /* Courant number C_max of eq. dt                                */
    double dlna_max;     /* cap on dln a per step                                          */
    double t_floor;      /* temperature floor [K] applied only inside the EOS              */
    int32_t subgrid;     /* DH_SUBGRID_*                                                   */
    double tau;          /* Gumbel-softmax temperature (Sec. 2.4.2; 0.1)                   */
    uint64_t sf_seed;    /* key of the per-cell, per-step star-formation uniforms          */
    int32_t ckpt_every;  /* checkpoint interval in steps for dh_forward/dh_backward (>=1)  */
    int32_t closure;     /* DH_CLOSURE_*; MLP needs subgrid != OFF and dh_set_closure()    */
    int32_t batch;       /* samples in the handle (>= 1); n^3 * batch <= 2^31              */
    double cfl_forward;  /* largest Courant number a replayed step may reach on the state it
                            is applied to (C_forward of Sec. 2.3.3; default 1.5 cfl); 0: no
                            check                                                         */
    int32_t kdk;         /* DH_KDK_*: the dark matter's step factors                        */
    int32_t star_dm;     /* 1: the stars formed in each step are read out by CIC at the
                            particles' end-of-step positions and added to the particles'
                            auxiliary field DH_FIELD_STAR_DM (Sec. 2.4.1: new stars are
                            associated with nearby dark matter; a diagnostic without effect on
                            the evolution and without adjoint)                               */
    int32_t sn_smooth;   /* 1: the supernova energy a^2 rho z E0 of a cell is spread over the
                            cell and its 26 neighbours with weights w(ox) w(oy) w(oz),
                            w(0) = 1/2, w(+-1) = 1/4 (periodic; the total is unchanged), the
                            start of the Sedov-Taylor blast of Sec. 2.4.1 on the grid; 0: all
                            of it into the cell.  Differentiated like the rest of the step   */
    int32_t lpt;         /* order of the initial displacements: 1 Zel'dovich, 2 second-order
                            LPT (Psi2 = -(D2/D1^2) IFFT(i k delta2_k / k^2) from
                            delta2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2) of the linear
                            potential, D2/D1^2 = -3/7 Omega_m(a)^(-1/143), velocities with
                            f2 = 2 Omega_m(a)^(6/11)); differentiated by dh_backward          */
    int32_t transfer;    /* DH_TRANSFER_*                                                   */
    int32_t dual_energy; /* 1: the dual-energy formalism, the extension of the single-energy
                            scheme named in Sec. 2.3: a sixth gas component S = (a^2 rho e)
                            rho^(1-gamma), the entropy variable, advected with the flux
                            S U_d / a; the EOS takes e = E - U^2/2 where that exceeds
                            1e-3 E and S rho^(gamma-2) / a^2 elsewhere, and at the end of
                            each step S is reset from the total energy where E - U^2/2 >=
                            0.1 E (Bryan et al. 1995 with the entropy of Ryu et al. 1993).
                            Differentiated by dh_backward, also with closure = MLP (the
                            network's T from the selected internal energy) and sn_smooth = 1
                            (the entropy takes its share of the smoothed energy before the
                            reset; a taped step keeps the injection field, 4 B per cell) */
} dh_config;

/* Model parameters (double).  A, beta: flux observable F = exp(-A Delta^beta) of the loss;
 * eps_sf: star-formation efficiency per free-fall time; delta_c: gas overdensity
 * threshold; t_c: temperature threshold [K]; e0: supernova specific energy
 * [(1000 km/s)^2]; w_rho, w_t: widths of the relaxed thresholds relative to delta_c, t_c. */
typedef struct dh_params {
    double A, beta, eps_sf, delta_c, t_c, e0, w_rho, w_t;
} dh_params;

/* Fields for dh_get_field / dh_set_field.  Sizes in floats: Q = 5 n^3 (6 n^3 with
 * cfg.dual_energy: the entropy S is the sixth component), POS and MOM = 3 n^3, the rest n^3.
 * TEMP (get only) is the gas temperature [K] from the floored energy (the dual-energy
 * selection where cfg.dual_energy).
 * STAR_DM: the particles' auxiliary field of read-out stars, in particle order (needs
 * cfg.star_dm; zeroed by the initial conditions).  OBS_TEMP (get only): the observable of
 * the field-level inference, O = (rho / rho_mean_gas) T [K], the gas-mass-weighted
 * temperature (Sec. 3.2). */
typedef enum dh_field {
    DH_FIELD_Q = 0, DH_FIELD_RHO = 1, DH_FIELD_POS = 2, DH_FIELD_MOM = 3,
    DH_FIELD_STAR = 4, DH_FIELD_PHI = 5, DH_FIELD_TEMP = 6, DH_FIELD_FLUX = 7,
    DH_FIELD_STAR_DM = 8, DH_FIELD_OBS_TEMP = 9
} dh_field;

typedef struct dh_sim dh_sim;

void dh_config_default(dh_config* cfg);
void dh_params_default(dh_params* p);

/* Allocates every device buffer on the current HIP device.  Errors: DH_E_INVAL for an
 * unsupported n or non-physical cosmology, DH_E_OOM, DH_E_HIP. */
int dh_create(const dh_config* cfg, dh_sim** out);
int dh_destroy(dh_sim* sim);
/* hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL. */
int dh_set_stream(dh_sim* sim, void* hip_stream);
int dh_set_params(dh_sim* sim, const dh_params* p);
/* Star-formation parameters of one sample of a batch (eps_sf, delta_c, t_c, e0, w_rho, w_t
 * of p; the loss parameters A, beta stay those of dh_set_params, shared by all samples). */
int dh_set_sample_params(dh_sim* sim, int32_t sample, const dh_params* p);

/* Initial state (Sec. 2.1): white noise -> delta_k = FFT(w) sqrt(P(k) D(a_i)^2 / V_cell)
 * -> Zel'dovich displacement Psi = IFFT(i k delta_k / k^2) -> particles x = q + Psi,
 * p = a^2 E(a) f(a) Psi; gas rho = f_b CIC(x), velocity of the particles on the lattice,
 * T = t_init; the potential of the initial state.  Resets time, step count and schedule.
 * _from_seed draws the noise with the library's Philox-4x32-10 generator (one normal per
 * cell by Box-Muller); _from_noise takes caller noise d_white[n^3] (device). */
int dh_init_from_seed(dh_sim* sim, uint64_t seed);
int dh_init_from_noise(dh_sim* sim, const float* d_white);

/* One step (operator order: CFL dt or next schedule entry; opening half kicks of gas and
 * dark matter with g_n; drift; three sweeps in the Strang order of this step; CIC deposit
 * and Poisson solve; closing half kicks with g_{n+1}; source term).  dt_out, a_out (of
 * sample 0) may be NULL.  Returns DH_E_NONFINITE if the new state has a non-finite or
 * non-positive density. */
int dh_step(dh_sim* sim, double* dt_out, double* a_out);
/* Steps until a >= a_final for every sample (the last step of each is clipped to land on
 * a_final); *nsteps_out = number of lockstep steps taken.  Inside the loop the closing
 * dark-matter half kick of a step is applied together with the next step's opening kick
 * (one pass over the particles, the same roundings as dh_step's separate kicks); the state
 * is complete again when the call returns. */
int dh_run_to(dh_sim* sim, double a_final, int32_t* nsteps_out);
/* nsteps steps as dh_step would take them one by one (same results bit for bit), in one
 * call, with the kick fusion of dh_run_to; *nsteps_out (may be NULL) = steps taken (fewer
 * only on error).  nsteps < 0: DH_E_INVAL; DH_E_NONFINITE as dh_step. */
int dh_run_steps(dh_sim* sim, int32_t nsteps, int32_t* nsteps_out);

/* Predefined schedule (Sec. 2.3.3).  set: the next steps take dts[0..n) in order (then the
 * CFL again); n = 0 clears it.  get: the dt of every step since the last init, at most
 * cap values, total count in *n_out.
 * A replayed entry is clipped, like a CFL step, so as not to pass the end of a dh_run_to or
 * dh_forward.  Accuracy check of a replay (Sec. 2.3.3): a schedule recorded on a fiducial
 * run at Courant number C_fid = cfg.cfl is valid for another run as long as each replayed
 * dt_fid stays within C_forward / C_fid of the step dt_sol = C_fid / v that eq. dt gives on
 * that run's own state (v = max over cells and axes of (|U_d| + c_s)/a), i.e. dt_fid v <=
 * C_forward.  (The paper prints the ratio the other way up, C_fid / C_forward < 1, which a
 * replay of the fiducial run on itself, ratio 1, would already violate.)  The calls that
 * take steps check every replayed step of the call against cfg.cfl_forward and return
 * DH_E_SCHEDULE when one exceeds it; the steps are still taken (the state is that of the
 * whole call), and a dh_forward that fails the check cannot be followed by dh_backward. */
int dh_set_schedule(dh_sim* sim, const double* dts, int32_t n);
int dh_get_schedule(const dh_sim* sim, double* dts, int32_t cap, int32_t* n_out);
/* The same for one sample of a batch (dh_set_schedule sets every sample's; dh_get_schedule
 * returns sample 0's). */
int dh_set_sample_schedule(dh_sim* sim, int32_t sample, const double* dts, int32_t n);
int dh_get_sample_schedule(const dh_sim* sim, int32_t sample, double* dts, int32_t cap,
                           int32_t* n_out);

/* Copy a field to / from caller device memory (see dh_field).  set_field of Q, POS or RHO
 * invalidates the potential; dh_refresh_potential() recomputes it from the current gas and
 * particles at the current scale factor. */
int dh_get_field(dh_sim* sim, dh_field f, float* d_out);
int dh_set_field(dh_sim* sim, dh_field f, const float* d_in);
int dh_refresh_potential(dh_sim* sim);
/* Current time.  set_time sets a (and t = t(a)) and the step counter used for the Strang
 * order and the random-number counters. */
int dh_get_time(const dh_sim* sim, double* a, double* t, int32_t* step);
int dh_set_time(dh_sim* sim, double a, int32_t step);
/* Scale factor and time of every sample (host arrays of batch values; either may be NULL). */
int dh_get_sample_times(const dh_sim* sim, double* a, double* t);

/* Differentiable run: init from d_white, then step to a_final with checkpoints every
 * cfg.ckpt_every steps (replaying each sample's schedule if one was set, else recording
 * it); *nsteps_out = number of lockstep steps. */
int dh_forward(dh_sim* sim, const float* d_white, double a_final, int32_t* nsteps_out);
/* How many steps of a dh_forward keep data for the reverse pass, which then recomputes less
 * (the results are the same bit for bit): first whole checkpoint segments keep their full
 * tape (the reverse pass recomputes nothing there; about 140 bytes per cell and step), then
 * further steps keep their particle sort and end-of-step potential (its recomputation skips
 * the sort, the deposit and the Poisson solve; about 28 bytes per cell and step).
 * max_steps < 0 (the default): as many as device memory allows after the reverse pass's own
 * buffers and a 4 GiB margin; 0: none (every segment is recomputed from its checkpoint).
 * Takes effect at the next dh_forward. */
int dh_set_store_limit(dh_sim* sim, int32_t max_steps);
/* What the last dh_forward kept: *taped = steps on its own tape (the first ones, whole
 * checkpoint segments or all), *sorted = further steps with a kept sort and potential.
 * Either pointer may be NULL. */
int dh_get_store_info(const dh_sim* sim, int32_t* taped, int32_t* sorted);
/* Loss L = mean over cells of (F - F_target)^2 with F = exp(-A (rho/rho_mean)^beta) on the
 * current state; FP64 reduction.  d_target[n^3] device (per sample); loss_out: one value
 * per sample. */
int dh_loss(dh_sim* sim, const float* d_target, double* loss_out);
/* Observables of the paper's applications (Sec. 3) on the current state.
 * Baryon power spectrum (the statistic of the parameter inference): with the overdensity
 * delta_b = rho / rho_mean_gas - 1 and its unnormalised transform X_m over the n^3 integer
 * wavenumber vectors m, P_b = (L^3 / n^6) sum_{m in bin b} |X_m|^2 / W_b [(Mpc/h)^3], where
 * bin b = 0..nbins-1 holds the modes whose |m| rounds to b + 1 (no |m| is a half-integer)
 * and W_b is their number; 1 <= nbins <= n/2.  pk_out[S][nbins] (host); k_out[nbins] the
 * nominal wavenumbers 2 pi (b + 1) / L [h/Mpc] and nmodes_out[nbins] = W_b, either may be
 * NULL.  FP64 sums in a fixed order (reproducible bit for bit). */
int dh_power_spectrum(dh_sim* sim, int32_t nbins, double* pk_out, double* k_out,
                      double* nmodes_out);
/* Gaussian loss of a mock spectrum, L = 1/2 (P - P_obs)^T C^-1 (P - P_obs) with pk_obs
 * [S][nbins] and the inverse covariance cinv [nbins][nbins] (host, row-major, shared by the
 * samples; the paper estimates C from independent boxes); loss_out[S].  A following
 * dh_backward(NULL) differentiates it (dL/dA = dL/dbeta = 0). */
int dh_power_loss(dh_sim* sim, int32_t nbins, const double* pk_obs, const double* cinv,
                  double* loss_out);
/* Negative log-posterior of the field-level inference (Sec. 3.2):
 * L = 1/2 sum_i (d_i - O_i)^2 / N_i + 1/2 sum_i w_i^2 with O of DH_FIELD_OBS_TEMP, the data
 * d_data, pixel noise variances d_noise_var and the white noise d_white of the run (the
 * initial phases, standard-normal prior), all device [S][n^3] (copied).  loss_out[S].  A
 * following dh_backward(NULL) differentiates it, prior included. */
int dh_fli_loss(dh_sim* sim, const float* d_data, const float* d_noise_var,
                const float* d_white, double* loss_out);

/* Reverse pass of the last dh_forward.  d_grad_rho: adjoint of the final gas density
 * (device n^3 per sample) or NULL for the gradient of the last loss call (dh_loss,
 * dh_power_loss or dh_fli_loss; each sample's own loss).  Outputs: d_grad_white[n^3] per
 * sample (device) and grad_params[4] per sample = dL/d(A, beta, eps_sf, delta_c) (host, FP64,
 * summed over steps in a fixed order).  The time schedule is held fixed.  DH_E_STATE if no
 * forward (or no loss, with NULL) precedes it. */
int dh_backward(dh_sim* sim, const float* d_grad_rho, float* d_grad_white, double* grad_params);

/* Kernel timing for measurement.  While a family is set, every launch of that kernel family
 * made by the stepping calls and dh_backward (not the dh_stage_* calls) is bracketed by a
 * pair of HIP events on the handle's stream: DH_KTIME_SWEEP_KICK the first hydro sweep of a
 * step (with the opening gas kick), DH_KTIME_SWEEP the second and third sweeps,
 * DH_KTIME_SWEEP_VJP the sweep adjoints; -1 stops timing.  Setting it discards earlier
 * records.  dh_get_kernel_timing synchronises the stream and returns the number of timed
 * launches since the last set or get and their mean duration [ms], then discards them. */
enum { DH_KTIME_SWEEP_KICK = 0, DH_KTIME_SWEEP = 1, DH_KTIME_SWEEP_VJP = 2 };
int dh_set_kernel_timing(dh_sim* sim, int32_t family);
int dh_get_kernel_timing(dh_sim* sim, int32_t* count, double* mean_ms);

/* FP64 sums over the current state, 8 values per sample: out[0] gas mass, out[1..3] gas
 * momentum a rho U, out[4] total gas energy a^2 rho E, out[5..7] dark-matter momentum (mass
 * times p). */
int dh_conservation(dh_sim* sim, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the sums of dh_conservation over caller
 * buffers, without a handle.  d_q[batch][5][n^3] gas state, d_mom[batch][3][n^3] particle
 * momenta p, m_dm the dark-matter particle mass; d_out[8 * batch] (device, FP64) receives
 * per sample the 8 values of dh_conservation, bit for bit (the same kernels and summation
 * order).  Enqueued on hip_stream (a hipStream_t or NULL); asynchronous: no allocation and
 * no synchronisation, so it may be captured into a HIP graph.  The reduction's block
 * partials live in a library-owned static device array of 512 KiB per device (each device
 * that the library runs on holds it until the process ends), which limits n to 256:
 * larger n, n < 1, batch < 1 or a null pointer return DH_E_INVAL, a failed device lookup
 * DH_E_HIP; dh_last_error(NULL) then holds the message (per thread).  Every call on a device
 * shares that array: calls that overlap on one device (different streams, or threads)
 * race and must be ordered by the caller. */
int dh_conservation_noalloc(const float* d_q, const float* d_mom, int32_t n, int32_t batch,
                            double m_dm, double* d_out, void* hip_stream);

/* Single stages on caller buffers (one sample's size), for verification of each kernel
 * against a reference.  They do not touch the handle's state.  All pointers are device
 * float32.
 *  sweep:    q_out = one relaxing-TVD sweep of q_in along axis (0 x, 1 y, 2 z) over dt,
 *            with scale factors a_stage1, a_stage2 (Sec. 2.3.1-2.3.2); q holds the handle's
 *            gas components (5 n^3 floats, 6 n^3 with cfg.dual_energy).
 *  sweep_vjp: lam_in = (d sweep / d q_in)^T lam_out at q_in.
 *  poisson:  phi = solution of lap(phi) = (3 Om / 2a) delta (Green's function -1/k^2).
 *  deposit:  delta = rho_gas + m_dm CIC(pos) - 1 (cell-sorted, deterministic).
 *  readout:  out[3][np] = CIC interpolation of the central-difference g = -grad(phi).  */
int dh_stage_sweep(dh_sim* sim, const float* d_q_in, float* d_q_out, int32_t axis, double dt,
                   double a_stage1, double a_stage2);
int dh_stage_sweep_vjp(dh_sim* sim, const float* d_q_in, const float* d_lam_out,
                       float* d_lam_in, int32_t axis, double dt, double a_stage1,
                       double a_stage2);
int dh_stage_poisson(dh_sim* sim, const float* d_delta, float* d_phi, double a);
int dh_stage_deposit(dh_sim* sim, const float* d_rho_gas, const float* d_pos, float* d_delta);
int dh_stage_readout(dh_sim* sim, const float* d_phi, const float* d_pos, float* d_g);

/* Message of the last failed call on sim; with sim NULL, of the last failed handle-free
 * call (dh_conservation_noalloc) on this thread. */
const char* dh_last_error(const dh_sim* sim);
const char* dh_strerror(int code);

/* ---------------------------------------------------------------------------------------
 * Learned star-formation closure.
 *
 * Network: inputs x = ((ln Delta - 4.6)/5, (ln T - 10.4)/5, (ln a + 3)/1.5, eps_sf/0.02 - 1,
 * Delta_c/100 - 1) with Delta the gas overdensity and T [K] the temperature; three hidden
 * layers of 64 with SiLU; outputs o = 10 (W4 h3 + b4).  In the simulation the outputs give
 * the star-formation probability of a step, pi0 = (1 - exp(-exp(o0) dt)) exp(min(o1, 0)):
 * o0 stands for ln(eps_sf / t_ff) and o1 for the log of the two threshold gates of the
 * relaxed model (Sec. 2.4), clipped at -30.  Inference and training run on the matrix
 * cores in bfloat16 with float32 accumulation.
 *
 * Parameters: DH_MLP_NPARAMS floats, W1[64][5], b1[64], W2[64][64], b2[64], W3[64][64],
 * b3[64], W4[2][64], b4[2] (W[out][in]), in host memory for set/get.
 * Arrays of samples are device float32 structure-of-arrays: x[5][count], outputs and
 * targets [2][count].
 * ------------------------------------------------------------------------------------- */
#define DH_MLP_NPARAMS 8834

/* Network weights for DH_CLOSURE_MLP runs of this simulation (host h_theta, copied). */
int dh_set_closure(dh_sim* sim, const float* h_theta);

typedef struct dh_mlp dh_mlp;

/* Training options: Adam (beta1, beta2, eps) with a cosine learning-rate decay from lr to
 * lr_final over `steps` steps of `batch` samples; batch k takes samples
 * [(k batch) mod count, ...) cyclically. */
typedef struct dh_mlp_train_opts {
    int64_t batch;
    int32_t steps;
    double lr, lr_final, beta1, beta2, eps;
} dh_mlp_train_opts;

/* Ranges of the training states: ln Delta, ln T [K], ln a uniform over [lo, hi], except
 * that with probability 1/2 each, ln Delta (ln T) is drawn within +-1.5 of ln Delta_c
 * (ln T_c); eps_sf and Delta_c uniform over [lo, hi].  Defaults (dh_mlp_sample_defaults):
 * Delta in [1e-2, 3e4], T in [1, 3e8] K, a in [0.008, 0.32], eps_sf and Delta_c within
 * +-50% of 0.02 and 100. */
typedef struct dh_mlp_sample_opts {
    double lnd_lo, lnd_hi, lnt_lo, lnt_hi, lna_lo, lna_hi;
    double eps_lo, eps_hi, dc_lo, dc_hi;
} dh_mlp_sample_opts;

void dh_mlp_train_defaults(dh_mlp_train_opts* opts);
void dh_mlp_sample_defaults(dh_mlp_sample_opts* opts);

/* A network with its training state on the current HIP device. */
int dh_mlp_create(dh_mlp** out);
int dh_mlp_destroy(dh_mlp* net);
int dh_mlp_set_stream(dh_mlp* net, void* hip_stream);
/* Uniform(+-1/sqrt(fan_in)) weights from the library's Philox generator. */
int dh_mlp_init_weights(dh_mlp* net, uint64_t seed);
int dh_mlp_set_weights(dh_mlp* net, const float* h_theta);
int dh_mlp_get_weights(dh_mlp* net, float* h_theta);
/* Training set of the closure: states drawn over the ranges of opts, samples first ..
 * first + count - 1 of the stream of `seed` (so that sets can be made in pieces); inputs
 * d_x[5][count] and targets d_y[2][count] = (ln(eps_sf/t_ff), clipped log gate) of the plain
 * relaxed source term, computed in FP64; omega_b and p (t_c, w_rho, w_t) as in dh_config and
 * dh_params.  opts NULL: defaults. */
int dh_mlp_sample(dh_mlp* net, const dh_mlp_sample_opts* opts, double omega_b,
                  const dh_params* p, uint64_t seed, int64_t first, int64_t count, float* d_x,
                  float* d_y);
/* Training and checking on the states a run visits: the network inputs d_x[5][S n^3] and
 * the targets d_y[2][S n^3] (as dh_mlp_sample's) of every cell of the handle's current state
 * (sample s at columns s n^3 ..), with its scale factor and parameters.  Caller-owned device
 * buffers; asynchronous.  With the dual-energy state, T is that of the selected internal
 * energy (as the closure and the plain source term take it). */
int dh_closure_states(dh_sim* sim, float* d_x, float* d_y);
/* d_out[2][count] = network(d_x). */
int dh_mlp_eval(dh_mlp* net, const float* d_x, int64_t count, float* d_out);
/* d_gx[5][count] = (d out / d x)^T d_gout[2][count] (BF16 rounding passed as identity). */
int dh_mlp_vjp(dh_mlp* net, const float* d_x, const float* d_gout, int64_t count, float* d_gx);
/* Objective L = mean over samples of sum_k (o_k - y_k)^2 and its gradient in the weights
 * (host h_grad[DH_MLP_NPARAMS], FP64), summed in a fixed order. */
int dh_mlp_grad(dh_mlp* net, const float* d_x, const float* d_y, int64_t count, double* h_grad,
                double* loss_out);
/* Adam on the objective over the set (d_x, d_y); h_loss (host, opts.steps values, or NULL)
 * receives the batch objective before each step.  The optimiser state restarts with each
 * call. */
int dh_mlp_train(dh_mlp* net, const float* d_x, const float* d_y, int64_t count,
                 const dh_mlp_train_opts* opts, double* h_loss);
const char* dh_mlp_last_error(const dh_mlp* net);

#ifdef __cplusplus
}
#endif
#endif

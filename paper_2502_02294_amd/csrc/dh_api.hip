// libdiffhydro: host engine and C ABI (include/diffhydro.h).
//
// One time step (operator order; every arrow is a kernel launch on the handle's stream):
//   dt (CFL in FP64 on the device, or the next schedule entry)
//   -> gas opening half kick with g_n -> DM opening half kick + drift + cell keys
//   -> three sweeps in the Strang order of the step (Sec. 2.3.2)
//   -> counting sort -> CIC deposit of gas + DM -> FFT Poisson at a(t+dt) -> phi_{n+1}
//   -> gas and DM closing half kicks with g_{n+1} -> star-formation source term.
// Reverse mode: the forward keeps a checkpoint of the state every ckpt_every steps; the
// backward re-runs each segment from its checkpoint, keeping every intermediate the
// adjoint kernels need (the tape of that segment), then applies the adjoint of each step
// in reverse order, and finally the adjoint of the initial conditions.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/diffhydro.h"
#include "dh_cosmo.h"
#include "dh_kernels.h"
#include "dh_mlp.h"

namespace {

using dh::ArgError;
using dh::HipError;

constexpr double kBoltzmann = 1.380649e-23;       // J/K
constexpr double kProtonMass = 1.67262192369e-27;  // kg

struct Plan {
  double t0, dt, a0, ah, a1;
  int step;
  int axes[3];
};

const int kStrang[6][3] = {{0, 1, 2}, {2, 1, 0}, {2, 0, 1}, {1, 0, 2}, {1, 2, 0}, {0, 2, 1}};

struct TapeStep {
  float* q[6];      // Q0 start, Q1 after opening kick (sweep-1 input), Q2, Q3 sweep inputs,
                    // Q4 after sweeps, Q5 after closing kick (source input)
  float *x0, *x1;             // particle positions at the start and after the drift
  float *phi0, *phi1;
  Plan plan;
};

struct Ckpt {
  float *q, *pos, *mom, *star, *phi;
  double t, a;
  int step;
};

}  // namespace

struct dh_sim {
  dh_config cfg;
  dh_params prm;
  int n = 0;
  long long nc = 0, np = 0, nck = 0;
  hipStream_t st = nullptr;
  dh::Cosmo cosmo{};
  double amp = 0, f_b = 0, vel_unit = 0, t_per_e = 0, e_init = 0, e_floor = 0, m_dm = 0;

  // state
  float *q = nullptr, *pos = nullptr, *mom = nullptr, *star = nullptr, *phi = nullptr;
  double t = 0, a = 0;
  int step = 0;
  bool phi_valid = false, initialised = false;

  // scratch
  float *q2 = nullptr, *delta = nullptr, *cic = nullptr, *psi = nullptr, *fscratch = nullptr;
  float2 *spec = nullptr, *spec2 = nullptr, *tw = nullptr;
  float4* g4 = nullptr;        // (-grad phi, 0) of the current potential
  float4* g4b = nullptr;       // scratch acceleration field for the reverse pass and stages
  dh::Bins bins{};
  double* cfl_red = nullptr;   // CFL block maxima of the current state (from the closing pass)
  bool cfl_partials = false;   // cfl_red holds the maxima of the current state
  bool speed_known = false;    // speed holds the CFL speed of the current state
  double speed = 0.0;
  double* red = nullptr;       // block partials
  double* red_out = nullptr;   // reduced values
  double* host_out = nullptr;  // pinned
  int red_blocks = 0;

  // adjoint buffers
  float *lq = nullptr, *lq2 = nullptr, *lh = nullptr, *lx = nullptr, *lp = nullptr,
        *lphi = nullptr, *lphi2 = nullptr, *lg = nullptr, *ldelta = nullptr, *lpsi = nullptr,
        *lcic = nullptr;
  double* param_steps = nullptr;   // [2 * cap] per-step dL/d(eps_sf, delta_c)
  int param_cap = 0;

  // learned closure: flat weights and their packed matrix-core form
  float* mlp_theta = nullptr;
  uint4* mlp_packed = nullptr;
  bool mlp_ready = false;

  // schedule
  std::vector<double> recorded;
  std::vector<double> replay;
  size_t replay_pos = 0;

  // reverse mode
  std::vector<Ckpt> ckpts;
  std::vector<TapeStep> tape;
  bool have_forward = false, have_loss = false;
  int fwd_steps = 0;
  float* loss_target = nullptr;

  std::vector<void*> allocs;
  std::string err;

  template <typename T>
  T* alloc(long long count) {
    void* p = nullptr;
    if (hipMalloc(&p, static_cast<size_t>(count) * sizeof(T)) != hipSuccess)
      throw std::bad_alloc();
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) allocs.erase(it);
    (void)hipFree(p);
  }
};

namespace {

int fail(dh_sim* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

template <typename F>
int guarded(dh_sim* s, F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    return fail(s, DH_E_INVAL, e.what());
  } catch (const HipError& e) {
    return fail(s, DH_E_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(s, DH_E_OOM, "device or host allocation failed");
  } catch (const std::exception& e) {
    return fail(s, DH_E_HIP, e.what());
  }
}

void copy_d2d(dh_sim* s, float* dst, const float* src, long long count) {
  DH_HIP(hipMemcpyAsync(dst, src, static_cast<size_t>(count) * sizeof(float),
                        hipMemcpyDeviceToDevice, s->st));
}

dh::HydroK hydro_at(const dh_sim* s, double a) {
  return dh::make_hydro(static_cast<float>(a), static_cast<float>(s->cfg.gamma),
                        static_cast<float>(s->e_floor));
}

void sync(dh_sim* s) { DH_HIP(hipStreamSynchronize(s->st)); }

// bins of the particle positions pos
void sort_particles(dh_sim* s, const float* pos) {
  dh::launch_keys(s->st, pos, s->bins.key, s->n);
  dh::launch_sort(s->st, s->bins, pos, s->n);
}

// phi_out = Poisson solve of delta at scale factor a; uses spec
void poisson(dh_sim* s, const float* delta, float* phi_out, double a) {
  dh::fft_forward_xy(s->st, delta, s->spec, s->tw, s->n);
  const double n3 = static_cast<double>(s->nc);
  dh::fft_zpass_green(s->st, s->spec, s->tw, s->n,
                      static_cast<float>(-(1.5 * s->cfg.omega_m / a) / n3));
  dh::fft_inverse_yx(s->st, s->spec, phi_out, s->tw, s->n, 1.0f);
}

// phi = Poisson(rho_gas + m_dm CIC(pos) - 1) and g4 = -grad(phi), with the bins of the
// particle positions already built
void potential_from_bins(dh_sim* s, const float* rho_gas, float* phi_out, float4* g4_out,
                         double a) {
  dh::launch_deposit(s->st, s->bins, rho_gas, static_cast<float>(s->m_dm), -1.0f, s->delta, s->n);
  poisson(s, s->delta, phi_out, a);
  dh::launch_grad(s->st, phi_out, g4_out, s->n);
}

void state_changed(dh_sim* s) {
  s->cfl_partials = false;
  s->speed_known = false;
}

// CFL speed max over cells and axes of (|U_d| + c_s)/a of the current state (FP64 on the
// device); +inf when the state holds a non-finite value or a non-positive density
double current_speed(dh_sim* s) {
  if (s->speed_known) return s->speed;
  if (!s->cfl_partials)
    dh::launch_cfl_partial(s->st, s->q, s->a, s->cfg.gamma, s->e_floor, s->cfl_red, s->n);
  dh::launch_reduce_max(s->st, s->cfl_red, dh::cfl_blocks(s->n), s->red_out);
  DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, sizeof(double), hipMemcpyDeviceToHost, s->st));
  sync(s);
  s->speed = s->host_out[0];
  s->speed_known = true;
  return s->speed;
}

dh::SourceArgs source_args(const dh_sim* s, const Plan& pl) {
  dh::SourceArgs a{};
  a.a = pl.a1;
  a.dt = pl.dt;
  a.inv_rho_mean = 1.0 / s->f_b;
  a.omega_b = s->cfg.omega_b;
  a.efloor = s->e_floor;
  a.t_per_e = s->t_per_e;
  a.e0_code = s->prm.e0 * 1e6 / (s->vel_unit * s->vel_unit);
  a.eps_sf = s->prm.eps_sf;
  a.delta_c = s->prm.delta_c;
  a.t_c = s->prm.t_c;
  a.w_rho = s->prm.w_rho;
  a.w_t = s->prm.w_t;
  a.tau = s->cfg.tau;
  a.mode = s->cfg.subgrid;
  a.seed_lo = static_cast<uint32_t>(s->cfg.sf_seed & 0xFFFFFFFFull);
  a.seed_hi = static_cast<uint32_t>(s->cfg.sf_seed >> 32);
  a.step = static_cast<uint32_t>(pl.step);
  a.mlp = s->cfg.closure == DH_CLOSURE_MLP ? s->mlp_packed : nullptr;
  return a;
}

Plan make_plan(const dh_sim* s, double dt) {
  Plan p{};
  p.t0 = s->t;
  p.dt = dt;
  p.a0 = s->a;
  p.ah = s->cosmo.a_of_t(s->t + 0.5 * dt);
  p.a1 = s->cosmo.a_of_t(s->t + dt);
  p.step = s->step;
  for (int k = 0; k < 3; ++k) p.axes[k] = kStrang[s->step % 6][k];
  return p;
}

// One step of the method on the handle state.  With a tape entry, keeps its intermediates.
void do_step(dh_sim* s, const Plan& pl, TapeStep* tp) {
  const int n = s->n;
  const long long nc = s->nc, np = s->np;
  const float h = static_cast<float>(0.5 * pl.dt);
  if (tp) {
    tp->plan = pl;
    copy_d2d(s, tp->q[0], s->q, 5 * nc);
    copy_d2d(s, tp->x0, s->pos, 3 * np);
    copy_d2d(s, tp->phi0, s->phi, nc);
  }
  const dh::HydroK h1 = hydro_at(s, pl.a0), h2 = hydro_at(s, pl.ah);
  const float dtf = static_cast<float>(pl.dt);
  const float drift = static_cast<float>(pl.dt / (pl.ah * pl.ah));
  if (tp) {
    // the kick, the sweeps and the closing pass write their results straight into the tape
    dh::launch_gas_kick(s->st, s->q, tp->q[1], s->g4, h, n);
    dh::launch_kick_drift(s->st, s->g4, s->pos, s->mom, s->bins.key, h, drift, nullptr, tp->x1, n);
    for (int k = 0; k < 3; ++k)
      dh::launch_sweep(s->st, tp->q[1 + k], tp->q[2 + k], n, pl.axes[k], dtf, h1, h2);
    dh::launch_sort(s->st, s->bins, s->pos, n);
    potential_from_bins(s, tp->q[4], s->phi, s->g4, pl.a1);
    copy_d2d(s, tp->phi1, s->phi, nc);
    dh::launch_close_step(s->st, tp->q[4], s->q, s->g4, h, s->star, source_args(s, pl), tp->q[5],
                          s->cfg.gamma, s->cfl_red, n);
  } else {
    // opening half kicks with g_n, drift with a(t + dt/2)
    dh::launch_gas_kick(s->st, s->q, s->q, s->g4, h, n);
    dh::launch_kick_drift(s->st, s->g4, s->pos, s->mom, s->bins.key, h, drift, nullptr, nullptr, n);
    // sweeps in the Strang order of the step
    for (int k = 0; k < 3; ++k) {
      dh::launch_sweep(s->st, s->q, s->q2, n, pl.axes[k], dtf, h1, h2);
      std::swap(s->q, s->q2);
    }
    // Poisson at a(t + dt) from gas + DM (keys were written by the drift)
    dh::launch_sort(s->st, s->bins, s->pos, n);
    potential_from_bins(s, s->q, s->phi, s->g4, pl.a1);
    // closing gas half kick with g_{n+1}, source term and the CFL maxima: one pass
    dh::launch_close_step(s->st, s->q, s->q, s->g4, h, s->star, source_args(s, pl), nullptr,
                          s->cfg.gamma, s->cfl_red, n);
  }
  dh::launch_kick(s->st, s->g4, s->pos, s->mom, h, n);
  DH_LAUNCH_CHECK();
  s->t = pl.t0 + pl.dt;
  s->a = pl.a1;
  s->step = pl.step + 1;
  s->speed_known = false;
  s->cfl_partials = true;
}

void refresh_potential(dh_sim* s) {
  sort_particles(s, s->pos);
  potential_from_bins(s, s->q, s->phi, s->g4, s->a);
  s->phi_valid = true;
}

void initial_conditions(dh_sim* s, const float* d_white) {
  const int n = s->n;
  const double ai = s->cfg.a_init;
  const double d = s->cosmo.growth(ai);
  const double vcell = std::pow(s->cfg.box / n, 3.0);
  const double amp = s->amp * d * d / vcell;
  dh::fft_forward_xy(s->st, d_white, s->spec2, s->tw, n);
  dh::fft_zpass_forward(s->st, s->spec2, s->spec2, s->tw, n);
  for (int j = 0; j < 3; ++j) {
    dh::fft_zpass_ic(s->st, s->spec2, s->spec, s->tw, n, j, false, amp, s->cfg.omega_m * s->cfg.h,
                     s->cfg.n_s, n / s->cfg.box, false, true, false);
    dh::fft_inverse_yx(s->st, s->spec, s->psi + j * s->nc, s->tw, n, 1.0f);
  }
  const double vfac = ai * ai * s->cosmo.E(ai) * s->cosmo.growth_rate(ai);
  dh::launch_ic_particles(s->st, s->psi, s->pos, s->mom, static_cast<float>(vfac), n);
  sort_particles(s, s->pos);
  dh::launch_deposit(s->st, s->bins, nullptr, 1.0f, 0.0f, s->cic, n);
  dh::launch_ic_gas(s->st, s->cic, s->psi, s->q, static_cast<float>(s->f_b),
                    static_cast<float>(vfac), static_cast<float>(ai), static_cast<float>(s->e_init),
                    n);
  dh::launch_fill(s->st, s->star, 0.0f, s->nc);
  s->t = s->cosmo.t_of_a(ai);
  s->a = ai;
  s->step = 0;
  potential_from_bins(s, s->q, s->phi, s->g4, ai);
  s->phi_valid = true;
  state_changed(s);
  s->initialised = true;
  s->recorded.clear();
  s->replay_pos = 0;
}

// next dt: schedule entry or CFL (eq. dt) with the dln a cap, clipped to t_end (< 0: none)
int next_dt(dh_sim* s, double t_end, double* dt_out) {
  double dt;
  if (s->replay_pos < s->replay.size()) {
    dt = s->replay[s->replay_pos++];
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(s, DH_E_SCHEDULE, "schedule entry is not a positive finite dt");
  } else {
    const double v = current_speed(s);
    if (!std::isfinite(v) || !(v > 0.0))
      return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
    dt = std::min(s->cfg.cfl / v, s->cfg.dlna_max / s->cosmo.E(s->a));
    if (t_end > 0.0 && s->t + dt > t_end) dt = t_end - s->t;
  }
  *dt_out = dt;
  return DH_OK;
}

int step_once(dh_sim* s, double t_end, TapeStep* tp, double* dt_used) {
  if (!s->initialised) return fail(s, DH_E_STATE, "no initial state");
  if (s->cfg.closure == DH_CLOSURE_MLP && !s->mlp_ready)
    return fail(s, DH_E_STATE, "closure network weights not set (dh_set_closure)");
  if (!s->phi_valid) refresh_potential(s);
  double dt;
  int rc = next_dt(s, t_end, &dt);
  if (rc) return rc;
  do_step(s, make_plan(s, dt), tp);
  s->recorded.push_back(dt);
  if (dt_used) *dt_used = dt;
  return DH_OK;
}

void alloc_tape_entry(dh_sim* s, TapeStep& t) {
  for (int k = 0; k < 6; ++k) t.q[k] = s->alloc<float>(5 * s->nc);
  t.x0 = s->alloc<float>(3 * s->np);
  t.x1 = s->alloc<float>(3 * s->np);
  t.phi0 = s->alloc<float>(s->nc);
  t.phi1 = s->alloc<float>(s->nc);
}

void save_ckpt(dh_sim* s, Ckpt& c) {
  if (!c.q) {
    c.q = s->alloc<float>(5 * s->nc);
    c.pos = s->alloc<float>(3 * s->np);
    c.mom = s->alloc<float>(3 * s->np);
    c.star = s->alloc<float>(s->nc);
    c.phi = s->alloc<float>(s->nc);
  }
  copy_d2d(s, c.q, s->q, 5 * s->nc);
  copy_d2d(s, c.pos, s->pos, 3 * s->np);
  copy_d2d(s, c.mom, s->mom, 3 * s->np);
  copy_d2d(s, c.star, s->star, s->nc);
  copy_d2d(s, c.phi, s->phi, s->nc);
  c.t = s->t;
  c.a = s->a;
  c.step = s->step;
}

void load_ckpt(dh_sim* s, const Ckpt& c) {
  copy_d2d(s, s->q, c.q, 5 * s->nc);
  copy_d2d(s, s->pos, c.pos, 3 * s->np);
  copy_d2d(s, s->mom, c.mom, 3 * s->np);
  copy_d2d(s, s->star, c.star, s->nc);
  copy_d2d(s, s->phi, c.phi, s->nc);
  s->t = c.t;
  s->a = c.a;
  s->step = c.step;
  dh::launch_grad(s->st, s->phi, s->g4, s->n);
  s->phi_valid = true;
  state_changed(s);
}

// Adjoint of one step.  In: lq, lx, lp, lphi = adjoints of the state after the step (lphi is
// the adjoint of phi_{n+1} from the following step).  Out: the same buffers hold the
// adjoints of the state at the start of the step.
// The opening dark-matter kick of the following step acts at the same positions, with the
// same g and the same adjoint momentum as this step's closing kick, so its adjoint is merged
// here with factor h_next (0 for the last step); this step's own opening kick is left to the
// previous step, or to finish_first_kick after the first step.
void step_vjp(dh_sim* s, const TapeStep& T, int param_slot, float h_next) {
  const int n = s->n;
  const long long nc = s->nc, np = s->np;
  const Plan& pl = T.plan;
  const float h = static_cast<float>(0.5 * pl.dt);
  hipStream_t st = s->st;
  // source term
  if (s->cfg.subgrid != DH_SUBGRID_OFF) {
    const int nb = dh::source_vjp_blocks(n);
    dh::launch_source_vjp(st, T.q[5], s->lq, source_args(s, pl), s->red, nb, n);
    dh::launch_reduce_sum(st, s->red, nb, nb, 2, s->param_steps + 2 * param_slot);
  }
  // closing kicks (gas from Q4, DM at x1) -> lambda_g -> lambda_phi_{n+1}
  dh::launch_grad(st, T.phi1, s->g4b, n);
  dh::launch_gas_kick_vjp(st, T.q[4], s->g4b, h, s->lq, s->lg, n);
  sort_particles(s, T.x1);
  dh::launch_gather_sorted(st, s->bins, s->lp, n);
  dh::launch_deposit_vec(st, s->bins, h + h_next, s->lg, n);
  dh::launch_kick_vjp_pos(st, s->g4b, T.x1, s->lp, h + h_next, s->lx, n);
  dh::launch_grad_vjp(st, s->lg, s->lphi, s->lphi2, n);
  // Poisson (symmetric operator) and deposit at x1
  poisson(s, s->lphi2, s->ldelta, pl.a1);
  dh::launch_axpy(st, s->lq, s->ldelta, 1.0f, nc);
  dh::launch_deposit_vjp_pos(st, s->ldelta, T.x1, static_cast<float>(s->m_dm), s->lx, n);
  // sweeps in reverse
  const dh::HydroK h1 = hydro_at(s, pl.a0), h2 = hydro_at(s, pl.ah);
  for (int k = 2; k >= 0; --k) {
    dh::launch_sweep_vjp(st, T.q[1 + k], s->lq, s->lq2, s->lh, n, pl.axes[k],
                         static_cast<float>(pl.dt), h1, h2);
    std::swap(s->lq, s->lq2);
  }
  // drift: x1 = x0 + p_half dt / a_h^2
  dh::launch_axpy(st, s->lp, s->lx, static_cast<float>(pl.dt / (pl.ah * pl.ah)), 3 * np);
  // opening gas kick with phi_n
  dh::launch_grad(st, T.phi0, s->g4b, n);
  dh::launch_gas_kick_vjp(st, T.q[0], s->g4b, h, s->lq, s->lg, n);
  dh::launch_grad_vjp(st, s->lg, nullptr, s->lphi, n);
}

// Adjoint of the opening dark-matter kick of the first step (x0, phi0 of its tape entry)
void finish_first_kick(dh_sim* s, const TapeStep& T) {
  const int n = s->n;
  const float h = static_cast<float>(0.5 * T.plan.dt);
  hipStream_t st = s->st;
  dh::launch_grad(st, T.phi0, s->g4b, n);
  dh::launch_fill(st, s->lg, 0.0f, 3 * s->nc);
  sort_particles(s, T.x0);
  dh::launch_gather_sorted(st, s->bins, s->lp, n);
  dh::launch_deposit_vec(st, s->bins, h, s->lg, n);
  dh::launch_kick_vjp_pos(st, s->g4b, T.x0, s->lp, h, s->lx, n);
  dh::launch_grad_vjp(st, s->lg, s->lphi, s->lphi, n);
}

// Adjoint of the initial conditions: lq, lx, lp, lphi at a_init -> d_grad_white
void ic_vjp(dh_sim* s, float* d_grad_white) {
  const int n = s->n;
  const long long nc = s->nc;
  hipStream_t st = s->st;
  const double ai = s->cfg.a_init;
  // phi_0 = Poisson(rho_gas + m_dm CIC(x) - 1)
  poisson(s, s->lphi, s->ldelta, ai);
  dh::launch_axpy(st, s->lq, s->ldelta, 1.0f, nc);
  // positions of the initial particles are recomputed from psi
  const double vfac = ai * ai * s->cosmo.E(ai) * s->cosmo.growth_rate(ai);
  dh::launch_ic_particles(st, s->psi, s->pos, s->fscratch, static_cast<float>(vfac), n);
  dh::launch_deposit_vjp_pos(st, s->ldelta, s->pos, static_cast<float>(s->m_dm), s->lx, n);
  // gas: rho = f_b CIC(x), m = rho p(q), Et = a^2 rho (e_init + |p/a|^2/2)
  dh::launch_fill(st, s->lpsi, 0.0f, 3 * nc);
  dh::launch_ic_gas_vjp(st, s->cic, s->psi, s->lq, static_cast<float>(s->f_b),
                        static_cast<float>(vfac), static_cast<float>(ai),
                        static_cast<float>(s->e_init), s->lcic, s->lpsi, n);
  dh::launch_deposit_vjp_pos(st, s->lcic, s->pos, 1.0f, s->lx, n);
  // x = q + psi, p = vfac psi
  dh::launch_axpy(st, s->lpsi, s->lx, 1.0f, 3 * nc);
  dh::launch_axpy(st, s->lpsi, s->lp, static_cast<float>(vfac), 3 * nc);
  // psi_j = IFFT(i k_j T(k)/k^2 FFT(w)) -> lambda_w = sum_j IFFT(-i k_j T/k^2 FFT(lambda_psi_j))
  const double d = s->cosmo.growth(ai);
  const double amp = s->amp * d * d / std::pow(s->cfg.box / n, 3.0);
  for (int j = 0; j < 3; ++j) {
    dh::fft_forward_xy(st, s->lpsi + j * nc, s->spec, s->tw, n);
    dh::fft_zpass_ic(st, s->spec, s->spec2, s->tw, n, j, true, amp, s->cfg.omega_m * s->cfg.h,
                     s->cfg.n_s, n / s->cfg.box, true, false, j > 0);
  }
  dh::fft_zpass_inverse(st, s->spec2, s->tw, n);
  dh::fft_inverse_yx(st, s->spec2, d_grad_white, s->tw, n, 1.0f);
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

void dh_config_default(dh_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n = 32;
  c->box = 10.0;
  c->omega_m = 0.3;
  c->omega_b = 0.05;
  c->h = 0.7;
  c->sigma8 = 0.8;
  c->n_s = 0.96;
  c->gamma = 5.0 / 3.0;
  c->mu = 0.6;
  c->a_init = 0.01;
  c->t_init = 100.0;
  c->cfl = 0.4;
  c->dlna_max = 0.04;
  c->t_floor = 1.0;
  c->subgrid = DH_SUBGRID_OFF;
  c->tau = 0.1;
  c->sf_seed = 102;
  c->ckpt_every = 16;
}

void dh_params_default(dh_params* p) {
  if (!p) return;
  p->A = 0.3;
  p->beta = 1.6;
  p->eps_sf = 0.02;
  p->delta_c = 100.0;
  p->t_c = std::pow(10.0, 4.5);
  p->e0 = 0.03;
  p->w_rho = 0.1;
  p->w_t = 0.1;
}

int dh_create(const dh_config* cfg, dh_sim** out) {
  if (!cfg || !out) return DH_E_INVAL;
  *out = nullptr;
  const int n = cfg->n;
  if (!pow2(n) || n < 16 || n > 256) return DH_E_INVAL;
  if (!(cfg->omega_m > 0 && cfg->omega_m < 1 && cfg->omega_b > 0 && cfg->omega_b < cfg->omega_m &&
        cfg->box > 0 && cfg->a_init > 0 && cfg->a_init < 1 && cfg->cfl > 0 && cfg->dlna_max > 0 &&
        cfg->gamma > 1 && cfg->tau > 0 && cfg->ckpt_every >= 1 && cfg->subgrid >= 0 &&
        cfg->subgrid <= 2 && cfg->t_floor > 0 && cfg->t_init > 0 && cfg->sigma8 > 0 &&
        (cfg->closure == DH_CLOSURE_PLAIN ||
         (cfg->closure == DH_CLOSURE_MLP && cfg->subgrid != DH_SUBGRID_OFF))))
    return DH_E_INVAL;
  auto s = std::make_unique<dh_sim>();
  int rc = guarded(s.get(), [&]() -> int {
    s->cfg = *cfg;
    dh_params_default(&s->prm);
    s->n = n;
    s->nc = static_cast<long long>(n) * n * n;
    s->np = s->nc;
    s->nck = static_cast<long long>(n) * n * (n / 2 + 1);
    s->cosmo.om = cfg->omega_m;
    s->cosmo.ol = 1.0 - cfg->omega_m;
    s->amp = dh::spectrum_amplitude(cfg->omega_m, cfg->h, cfg->n_s, cfg->sigma8);
    s->f_b = cfg->omega_b / cfg->omega_m;
    s->m_dm = 1.0 - s->f_b;
    s->vel_unit = 100.0 * cfg->box / n;
    s->t_per_e = (cfg->gamma - 1.0) * cfg->mu * kProtonMass / kBoltzmann *
                 (s->vel_unit * 1e3) * (s->vel_unit * 1e3);
    s->e_init = cfg->t_init / s->t_per_e;
    s->e_floor = cfg->t_floor / s->t_per_e;
    const long long nc = s->nc, np = s->np;
    s->q = s->alloc<float>(5 * nc);
    s->q2 = s->alloc<float>(5 * nc);
    s->pos = s->alloc<float>(3 * np);
    s->mom = s->alloc<float>(3 * np);
    s->star = s->alloc<float>(nc);
    s->phi = s->alloc<float>(nc);
    s->delta = s->alloc<float>(nc);
    s->cic = s->alloc<float>(nc);
    s->psi = s->alloc<float>(3 * nc);
    s->fscratch = s->alloc<float>(3 * np);
    s->spec = s->alloc<float2>(s->nck);
    s->spec2 = s->alloc<float2>(s->nck);
    s->tw = s->alloc<float2>(n / 2);
    s->bins.key = s->alloc<uint32_t>(np);
    s->bins.rank = s->alloc<uint32_t>(np);
    s->bins.count = s->alloc<uint32_t>(nc);
    s->bins.start = s->alloc<uint32_t>(nc + 1);
    s->bins.sorted = s->alloc<uint32_t>(np);
    s->bins.block_sums = s->alloc<uint32_t>(static_cast<long long>(dh::scan_block_count(nc)) + 1);
    s->bins.spos = s->alloc<float4>(np);
    s->bins.sval = s->alloc<float4>(np);
    s->g4 = s->alloc<float4>(nc);
    s->g4b = s->alloc<float4>(nc);
    s->cfl_red = s->alloc<double>(dh::cfl_blocks(n) + 1);
    s->red_blocks = dh::sum_blocks(nc);
    s->red = s->alloc<double>(8LL * s->red_blocks + 8);
    s->red_out = s->alloc<double>(16);
    if (cfg->closure == DH_CLOSURE_MLP) {
      s->mlp_theta = s->alloc<float>(dh::mlp::kParams);
      s->mlp_packed = s->alloc<uint4>(static_cast<long long>(dh::mlp::kPackedBytes / sizeof(uint4)));
    }
    void* hp = nullptr;
    DH_HIP(hipHostMalloc(&hp, 16 * sizeof(double), hipHostMallocDefault));
    s->host_out = static_cast<double*>(hp);
    std::vector<float2> tw;
    dh::fft_make_twiddles(n, tw);
    DH_HIP(hipMemcpy(s->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
    return DH_OK;
  });
  if (rc != DH_OK) {
    dh_destroy(s.release());
    return rc;
  }
  *out = s.release();
  return DH_OK;
}

int dh_destroy(dh_sim* s) {
  if (!s) return DH_OK;
  (void)hipDeviceSynchronize();
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->host_out) (void)hipHostFree(s->host_out);
  delete s;
  return DH_OK;
}

int dh_set_stream(dh_sim* s, void* stream) {
  if (!s) return DH_E_INVAL;
  s->st = static_cast<hipStream_t>(stream);
  return DH_OK;
}

int dh_set_params(dh_sim* s, const dh_params* p) {
  if (!s || !p) return DH_E_INVAL;
  if (!(p->eps_sf >= 0 && p->delta_c > 0 && p->t_c > 0 && p->w_rho > 0 && p->w_t > 0 && p->e0 >= 0))
    return fail(s, DH_E_INVAL, "non-physical parameters");
  s->prm = *p;
  return DH_OK;
}

int dh_set_closure(dh_sim* s, const float* h_theta) {
  if (!s || !h_theta) return DH_E_INVAL;
  if (s->cfg.closure != DH_CLOSURE_MLP)
    return fail(s, DH_E_STATE, "simulation was created without the learned closure");
  return guarded(s, [&]() -> int {
    DH_HIP(hipMemcpyAsync(s->mlp_theta, h_theta, dh::mlp::kParams * sizeof(float),
                          hipMemcpyHostToDevice, s->st));
    dh::launch_mlp_pack(s->st, s->mlp_theta, s->mlp_packed);
    sync(s);
    s->mlp_ready = true;
    return DH_OK;
  });
}

int dh_init_from_seed(dh_sim* s, uint64_t seed) {
  if (!s) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    dh::launch_white_noise(s->st, s->delta, static_cast<uint32_t>(seed & 0xFFFFFFFFull),
                           static_cast<uint32_t>(seed >> 32), s->n);
    copy_d2d(s, s->fscratch, s->delta, s->nc);
    initial_conditions(s, s->fscratch);
    s->have_forward = false;
    return DH_OK;
  });
}

int dh_init_from_noise(dh_sim* s, const float* d_white) {
  if (!s || !d_white) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    initial_conditions(s, d_white);
    s->have_forward = false;
    return DH_OK;
  });
}

int dh_step(dh_sim* s, double* dt_out, double* a_out) {
  if (!s) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    double dt = 0;
    int rc = step_once(s, -1.0, nullptr, &dt);
    if (rc) return rc;
    s->have_forward = false;
    const double v = current_speed(s);   // also validates the new state
    if (!std::isfinite(v)) return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
    if (dt_out) *dt_out = dt;
    if (a_out) *a_out = s->a;
    return DH_OK;
  });
}

int dh_run_to(dh_sim* s, double a_final, int32_t* nsteps_out) {
  if (!s || !(a_final > 0)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const double t_end = s->cosmo.t_of_a(a_final);
    int count = 0;
    while (s->t < t_end * (1.0 - 1e-12)) {
      int rc = step_once(s, t_end, nullptr, nullptr);
      if (rc) return rc;
      ++count;
    }
    s->have_forward = false;
    if (nsteps_out) *nsteps_out = count;
    return DH_OK;
  });
}

int dh_set_schedule(dh_sim* s, const double* dts, int32_t n) {
  if (!s || n < 0 || (n > 0 && !dts)) return DH_E_INVAL;
  s->replay.assign(dts, dts + n);
  s->replay_pos = 0;
  return DH_OK;
}

int dh_get_schedule(const dh_sim* s, double* dts, int32_t cap, int32_t* n_out) {
  if (!s) return DH_E_INVAL;
  const int32_t n = static_cast<int32_t>(s->recorded.size());
  for (int32_t i = 0; i < std::min(n, cap); ++i) dts[i] = s->recorded[i];
  if (n_out) *n_out = n;
  return DH_OK;
}

int dh_get_field(dh_sim* s, dh_field f, float* d_out) {
  if (!s || !d_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    switch (f) {
      case DH_FIELD_Q: copy_d2d(s, d_out, s->q, 5 * s->nc); break;
      case DH_FIELD_RHO: copy_d2d(s, d_out, s->q, s->nc); break;
      case DH_FIELD_POS: copy_d2d(s, d_out, s->pos, 3 * s->np); break;
      case DH_FIELD_MOM: copy_d2d(s, d_out, s->mom, 3 * s->np); break;
      case DH_FIELD_STAR: copy_d2d(s, d_out, s->star, s->nc); break;
      case DH_FIELD_PHI:
        if (!s->phi_valid) refresh_potential(s);
        copy_d2d(s, d_out, s->phi, s->nc);
        break;
      case DH_FIELD_TEMP:
        dh::launch_temperature(s->st, s->q, static_cast<float>(s->a), static_cast<float>(s->e_floor),
                               static_cast<float>(s->t_per_e), d_out, s->nc);
        break;
      case DH_FIELD_FLUX:
        dh::launch_flux_field(s->st, s->q, s->prm.A, s->prm.beta, static_cast<float>(1.0 / s->f_b),
                              d_out, s->nc);
        break;
      default: return fail(s, DH_E_INVAL, "unknown field");
    }
    return DH_OK;
  });
}

int dh_set_field(dh_sim* s, dh_field f, const float* d_in) {
  if (!s || !d_in) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    switch (f) {
      case DH_FIELD_Q: copy_d2d(s, s->q, d_in, 5 * s->nc); s->phi_valid = false; break;
      case DH_FIELD_RHO: copy_d2d(s, s->q, d_in, s->nc); s->phi_valid = false; break;
      case DH_FIELD_POS: copy_d2d(s, s->pos, d_in, 3 * s->np); s->phi_valid = false; break;
      case DH_FIELD_MOM: copy_d2d(s, s->mom, d_in, 3 * s->np); break;
      case DH_FIELD_STAR: copy_d2d(s, s->star, d_in, s->nc); break;
      case DH_FIELD_PHI:
        copy_d2d(s, s->phi, d_in, s->nc);
        dh::launch_grad(s->st, s->phi, s->g4, s->n);
        s->phi_valid = true;
        break;
      default: return fail(s, DH_E_INVAL, "field cannot be set");
    }
    s->initialised = true;
    s->have_forward = false;
    state_changed(s);
    return DH_OK;
  });
}

int dh_refresh_potential(dh_sim* s) {
  if (!s) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    refresh_potential(s);
    return DH_OK;
  });
}

int dh_get_time(const dh_sim* s, double* a, double* t, int32_t* step) {
  if (!s) return DH_E_INVAL;
  if (a) *a = s->a;
  if (t) *t = s->t;
  if (step) *step = s->step;
  return DH_OK;
}

int dh_set_time(dh_sim* s, double a, int32_t step) {
  if (!s || !(a > 0) || step < 0) return DH_E_INVAL;
  s->a = a;
  s->t = s->cosmo.t_of_a(a);
  s->step = step;
  s->phi_valid = false;
  state_changed(s);
  return DH_OK;
}

int dh_forward(dh_sim* s, const float* d_white, double a_final, int32_t* nsteps_out) {
  if (!s || !d_white || !(a_final > s->cfg.a_init)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    initial_conditions(s, d_white);
    s->replay_pos = 0;
    const double t_end = s->cosmo.t_of_a(a_final);
    const int K = s->cfg.ckpt_every;
    size_t nck = 0;
    int count = 0;
    const bool replaying = !s->replay.empty();
    while (s->t < t_end * (1.0 - 1e-12)) {
      if (replaying && s->replay_pos >= s->replay.size()) break;   // schedule fully replayed
      if (count % K == 0) {
        if (nck == s->ckpts.size()) s->ckpts.push_back(Ckpt{});
        save_ckpt(s, s->ckpts[nck++]);
      }
      int rc = step_once(s, t_end, nullptr, nullptr);
      if (rc) return rc;
      ++count;
    }
    const double v = current_speed(s);
    if (!std::isfinite(v)) return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
    s->fwd_steps = count;
    s->have_forward = true;
    s->have_loss = false;
    if (nsteps_out) *nsteps_out = count;
    return DH_OK;
  });
}

int dh_loss(dh_sim* s, const float* d_target, double* loss_out) {
  if (!s || !d_target || !loss_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int nb = s->red_blocks;
    dh::launch_loss_partial(s->st, s->q, d_target, s->prm.A, s->prm.beta,
                            static_cast<float>(1.0 / s->f_b), s->red, nb, s->nc);
    dh::launch_reduce_sum(s->st, s->red, nb, nb, 1, s->red_out);
    DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, sizeof(double), hipMemcpyDeviceToHost, s->st));
    sync(s);
    *loss_out = s->host_out[0] / static_cast<double>(s->nc);
    if (!s->loss_target) s->loss_target = s->alloc<float>(s->nc);
    copy_d2d(s, s->loss_target, d_target, s->nc);
    s->have_loss = s->have_forward;
    return DH_OK;
  });
}

int dh_backward(dh_sim* s, const float* d_grad_rho, float* d_grad_white, double* grad_params) {
  if (!s || !d_grad_white || !grad_params) return DH_E_INVAL;
  if (!s->have_forward) return fail(s, DH_E_STATE, "dh_backward needs a preceding dh_forward");
  if (!d_grad_rho && !s->have_loss) return fail(s, DH_E_STATE, "dh_backward without d_grad_rho needs dh_loss");
  return guarded(s, [&]() -> int {
    const int n = s->n;
    const long long nc = s->nc, np = s->np;
    const int nsteps = s->fwd_steps;
    const int K = s->cfg.ckpt_every;
    if (!s->lq) {
      s->lq = s->alloc<float>(5 * nc);
      s->lq2 = s->alloc<float>(5 * nc);
      s->lh = s->alloc<float>(5 * nc);
      s->lx = s->alloc<float>(3 * np);
      s->lp = s->alloc<float>(3 * np);
      s->lphi = s->alloc<float>(nc);
      s->lphi2 = s->alloc<float>(nc);
      s->lg = s->alloc<float>(3 * nc);
      s->ldelta = s->alloc<float>(nc);
      s->lpsi = s->alloc<float>(3 * nc);
      s->lcic = s->alloc<float>(nc);
    }
    if (s->param_cap < nsteps + 2) {
      if (s->param_steps) s->release(s->param_steps);
      s->param_cap = nsteps + 2;
      s->param_steps = s->alloc<double>(2LL * s->param_cap);
    }
    // final state adjoint
    dh::launch_fill(s->st, s->lq, 0.0f, 5 * nc);
    dh::launch_fill(s->st, s->lx, 0.0f, 3 * np);
    dh::launch_fill(s->st, s->lp, 0.0f, 3 * np);
    dh::launch_fill(s->st, s->lphi, 0.0f, nc);
    double gA = 0.0, gB = 0.0;
    if (d_grad_rho) {
      copy_d2d(s, s->lq, d_grad_rho, nc);
    } else {
      const int nb = s->red_blocks;
      dh::launch_loss_vjp(s->st, s->q, s->loss_target, s->prm.A, s->prm.beta,
                          static_cast<float>(1.0 / s->f_b), s->lq, s->red, nb, nc);
      dh::launch_reduce_sum(s->st, s->red, nb, nb, 2, s->red_out);
      DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s->st));
      sync(s);
      gA = s->host_out[0];
      gB = s->host_out[1];
    }
    // segments in reverse
    const int nseg = (nsteps + K - 1) / K;
    if (s->tape.size() < static_cast<size_t>(std::min(K, nsteps))) {
      const size_t want = static_cast<size_t>(std::min(K, nsteps));
      while (s->tape.size() < want) {
        s->tape.push_back(TapeStep{});
        alloc_tape_entry(s, s->tape.back());
      }
    }
    // keep the forward's final state to restore it afterwards
    Ckpt final_state{};
    save_ckpt(s, final_state);
    const std::vector<double> sched = s->recorded;
    dh::launch_fill(s->st, reinterpret_cast<float*>(s->param_steps), 0.0f, 4LL * s->param_cap);
    float h_next = 0.0f;
    for (int g = nseg - 1; g >= 0; --g) {
      load_ckpt(s, s->ckpts[g]);
      const int s0 = g * K, s1 = std::min(nsteps, s0 + K);
      for (int k = s0; k < s1; ++k) do_step(s, make_plan(s, sched[k]), &s->tape[k - s0]);
      for (int k = s1 - 1; k >= s0; --k) {
        step_vjp(s, s->tape[k - s0], k, h_next);
        h_next = static_cast<float>(0.5 * sched[k]);
      }
    }
    if (nsteps > 0) finish_first_kick(s, s->tape[0]);
    ic_vjp(s, d_grad_white);
    // restore the final state of the forward run
    load_ckpt(s, final_state);
    s->release(final_state.q);
    s->release(final_state.pos);
    s->release(final_state.mom);
    s->release(final_state.star);
    s->release(final_state.phi);
    // parameter gradients: fixed-order host sum of the per-step FP64 partials
    std::vector<double> ps(2 * static_cast<size_t>(nsteps));
    if (nsteps > 0)
      DH_HIP(hipMemcpyAsync(ps.data(), s->param_steps, ps.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s->st));
    sync(s);
    double ge = 0.0, gd = 0.0;
    for (int k = 0; k < nsteps; ++k) {
      ge += ps[2 * k];
      gd += ps[2 * k + 1];
    }
    grad_params[0] = gA;
    grad_params[1] = gB;
    grad_params[2] = ge;
    grad_params[3] = gd;
    return DH_OK;
  });
}

int dh_conservation(dh_sim* s, double* out) {
  if (!s || !out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int nb = s->red_blocks;
    dh::launch_conservation_partial(s->st, s->q, s->mom, s->red, nb, s->nc);
    dh::launch_reduce_sum(s->st, s->red, nb, nb, 8, s->red_out);
    DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s->st));
    sync(s);
    for (int k = 0; k < 8; ++k) out[k] = s->host_out[k];
    for (int k = 5; k < 8; ++k) out[k] *= s->m_dm;
    return DH_OK;
  });
}

int dh_stage_sweep(dh_sim* s, const float* d_q_in, float* d_q_out, int32_t axis, double dt,
                   double a1, double a2) {
  if (!s || !d_q_in || !d_q_out || axis < 0 || axis > 2 || d_q_in == d_q_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    dh::launch_sweep(s->st, d_q_in, d_q_out, s->n, axis, static_cast<float>(dt), hydro_at(s, a1),
                     hydro_at(s, a2));
    return DH_OK;
  });
}

int dh_stage_sweep_vjp(dh_sim* s, const float* d_q_in, const float* d_lam_out, float* d_lam_in,
                       int32_t axis, double dt, double a1, double a2) {
  if (!s || !d_q_in || !d_lam_out || !d_lam_in || axis < 0 || axis > 2) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    if (!s->lh) s->lh = s->alloc<float>(5 * s->nc);
    dh::launch_sweep_vjp(s->st, d_q_in, d_lam_out, d_lam_in, s->lh, s->n, axis,
                         static_cast<float>(dt), hydro_at(s, a1), hydro_at(s, a2));
    return DH_OK;
  });
}

int dh_stage_poisson(dh_sim* s, const float* d_delta, float* d_phi, double a) {
  if (!s || !d_delta || !d_phi || !(a > 0)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    poisson(s, d_delta, d_phi, a);
    return DH_OK;
  });
}

int dh_stage_deposit(dh_sim* s, const float* d_rho_gas, const float* d_pos, float* d_delta) {
  if (!s || !d_rho_gas || !d_pos || !d_delta) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    sort_particles(s, d_pos);
    dh::launch_deposit(s->st, s->bins, d_rho_gas, static_cast<float>(s->m_dm), -1.0f, d_delta, s->n);
    return DH_OK;
  });
}

int dh_stage_readout(dh_sim* s, const float* d_phi, const float* d_pos, float* d_g) {
  if (!s || !d_phi || !d_pos || !d_g) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    dh::launch_grad(s->st, d_phi, s->g4b, s->n);
    dh::launch_readout_g(s->st, s->g4b, d_pos, d_g, s->n);
    return DH_OK;
  });
}

const char* dh_last_error(const dh_sim* s) { return s ? s->err.c_str() : "null handle"; }

const char* dh_strerror(int code) {
  switch (code) {
    case DH_OK: return "ok";
    case DH_E_INVAL: return "invalid argument";
    case DH_E_OOM: return "out of memory";
    case DH_E_HIP: return "HIP runtime error";
    case DH_E_NONFINITE: return "non-finite or non-positive state";
    case DH_E_SCHEDULE: return "schedule error";
    case DH_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

}  // extern "C"

// libdiffhydro: host engine and C ABI (include/diffhydro.h).
//
// One time step (operator order; every arrow is a kernel launch on the handle's stream):
//   dt (CFL in FP64 on the device, or the next schedule entry)
//   -> gas opening half kick with g_n -> DM opening half kick + drift + cell keys
//   -> three sweeps in the Strang order of the step (Sec. 2.3.2)
//   -> counting sort -> CIC deposit of gas + DM -> FFT Poisson at a(t+dt) -> phi_{n+1}
//   -> gas and DM closing half kicks with g_{n+1} -> star-formation source term.
// A handle holds S independent samples (S = 1 for a single simulation): every launch covers
// all of them, each with its own dt, scale factors and parameters from a per-step device
// table; the samples advance in lockstep by global step, and a sample that has reached its
// end (or the end of its replayed schedule) sits out the remaining steps.
// Reverse mode: the forward keeps a checkpoint of the state every ckpt_every steps; the
// backward re-runs each segment from its checkpoint, keeping every intermediate the
// adjoint kernels need (the tape of that segment), then applies the adjoint of each step
// in reverse order, and finally the adjoint of the initial conditions.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/diffhydro.h"
#include "dh_cosmo.h"
#include "dh_kernels.h"
#include "dh_mlp.h"

const char* dh_noalloc_last_error_message();   // noalloc_api.hip

namespace {

using dh::ArgError;
using dh::Batch;
using dh::HipError;
using dh::StepScal;

constexpr double kBoltzmann = 1.380649e-23;       // J/K
constexpr double kProtonMass = 1.67262192369e-27;  // kg

struct Plan {        // one sample's part of a step
  double t0, dt, a0, ah, a1;
  bool active;
  bool replayed;     // dt is an entry of a replayed schedule
};

struct StepPlan {    // one global step of all samples
  int step;          // global step counter (Strang order, random-number counter)
  int slot;          // index of its table in the handle's table store
  int axes[3];
  std::vector<Plan> smp;
};

const int kStrang[6][3] = {{0, 1, 2}, {2, 1, 0}, {2, 0, 1}, {1, 0, 2}, {1, 2, 0}, {0, 2, 1}};

struct TapeStep {
  float* q[6];      // Q0 start, Q1 not stored (the sweep-1 input, Q0 after the opening gas
                    // kick, which the first sweep's adjoint applies again), Q2, Q3 sweep
                    // inputs, Q4 after sweeps, Q5 after closing kick (source input; kept only
                    // for the learned closure, the plain source's adjoint recomputes it)
  float* x0;                  // particle positions at the start
  const float* x1;            // after the drift: not stored (the positions do not change
                              // after the drift, so x1 is the next step's x0, or the state's
                              // positions after a segment's last step); set by the reverse pass
  float* phi0;
  const float* phi1;          // not stored either: the next step's phi0, or the state's phi
                              // after a segment's last step; set by the reverse pass
  uint32_t *start, *sorted;   // the step's sort of x1 (bin starts, ids in bin order)
  float4* spos;               // x1 in that bin order
  float* sn;                  // dual energy with the smoothed injection: the step's per-cell
                              // injected energy before the smoothing (else null)
  // the sort the reverse pass uses: the buffers above, or the forward's stored one
  uint32_t *vstart, *vsorted;
  float4* vspos;
  StepPlan plan;
};

struct Ckpt {
  float *q, *pos, *mom, *star, *phi;
  std::vector<double> t, a;
  int step;
};

// What a forward step computed that its recomputation in the reverse pass would compute
// again, bit for bit: the sort of the post-drift positions (bin starts, ids, positions in
// bin order) and the end-of-step potential.  Kept per step while memory allows.
struct StepStore {
  uint32_t* start = nullptr;
  uint32_t* sorted = nullptr;
  float4* spos = nullptr;
  float* phi = nullptr;
};

}  // namespace

struct dh_sim {
  dh_config cfg;
  dh_params prm;                    // shared parameters (loss: A, beta)
  std::vector<dh_params> sprm;      // per-sample parameters of the source term
  int n = 0, S = 1;
  int nq = 5;   // gas components per cell: 6 with the dual-energy entropy
  long long nc = 0, np = 0, nck = 0;
  hipStream_t st = nullptr;
  dh::Cosmo cosmo{};
  dh::HeathTable heath;            // growth integral for the per-step FastPM factors
  double amp = 0, f_b = 0, vel_unit = 0, t_per_e = 0, e_init = 0, e_floor = 0, m_dm = 0;

  // state (S samples stacked)
  float *q = nullptr, *pos = nullptr, *mom = nullptr, *star = nullptr, *phi = nullptr;
  std::vector<double> t, a;         // per sample
  int step = 0;                     // global step counter
  bool phi_valid = false, initialised = false;

  // stars read out on the particles (cfg.star_dm): auxiliary field [S][np] and the step's
  // draw per cell; smoothed injection (cfg.sn_smooth): the injected energy per cell (and the
  // adjoint of it in the reverse pass)
  float *aux = nullptr, *znew = nullptr, *sn_buf = nullptr;
  float* sn_buf2 = nullptr;   // dual energy with the smoothed injection: the injection's adjoint
  // second-order LPT initial conditions (cfg.lpt == 2): the six second derivatives of the
  // linear potential [S][6][n^3] and the velocity displacement Psi + (f2/f1) Psi2 [S][3][n^3],
  // kept for the adjoint of the initial conditions
  float *hess = nullptr, *lptv = nullptr;

  // scratch
  float *q2 = nullptr, *delta = nullptr, *cic = nullptr, *psi = nullptr, *fscratch = nullptr;
  float2 *spec = nullptr, *spec2 = nullptr, *tw = nullptr;
  float4* g4 = nullptr;        // (-grad phi, 0) of the current potential
  float4* g4b = nullptr;       // scratch acceleration field for the reverse pass and stages
  int g4b_phi0_of = -1;         // g4b holds -grad of this step's phi0 (every sample moved), or -1
  // Closing dark-matter half kicks left to the next step's kick-drift pass (one pass over the
  // particles instead of two): factor per sample, 0 when none.  Only the step loops of
  // run_to / forward / run_steps and the recomputation of the reverse pass defer, and they
  // apply (or, for a discarded state, drop) what is left before returning, so outside them
  // the state is always complete.
  std::vector<float> kick_due;
  bool kick_pending = false;
  dh::Bins bins{};
  double* cfl_red = nullptr;   // CFL block maxima of the current state (from the closing pass)
  bool cfl_partials = false;   // cfl_red holds the maxima of the current state
  bool speed_known = false;    // speed holds the CFL speeds of the current state
  std::vector<double> speed;
  double* red = nullptr;       // block partials
  double* red_out = nullptr;   // reduced values
  double* host_out = nullptr;  // pinned
  double* d_acur = nullptr;    // scale factor of each sample (CFL recomputation)
  int red_blocks = 0;

  // per-step tables: slot k holds the S entries of the k-th step since the last init
  StepScal* tabs = nullptr;
  // replay check (Sec. 2.3.3): CFL speed of the state each replayed step started from
  // (device [tab_cap][S]), which (slot, sample) pairs were replayed, and the first slot not
  // yet checked
  double* speed_log = nullptr;
  std::vector<double> replayed;   // [tab_cap][S]: the replayed dt, 0 for a CFL step
  int checked_slots = 0;
  StepScal* htabs = nullptr;   // pinned mirror
  int tab_cap = 0;
  int nslots = 0;
  StepScal* cur_tab = nullptr;    // state table: every sample active at its current a
  StepScal* stage_tab = nullptr;  // single entry for the stage calls
  StepScal stage_last{};          // what stage_tab holds (valid once uploaded)
  bool stage_valid = false;
  StepScal* hstage = nullptr;     // pinned staging of cur_tab / stage_tab

  // adjoint buffers
  float *lq = nullptr, *lq2 = nullptr, *lx = nullptr, *lp = nullptr,
        *lphi = nullptr, *lphi2 = nullptr, *lg = nullptr, *lg2 = nullptr, *ldelta = nullptr,
        *lpsi = nullptr, *lcic = nullptr;
  // adjoint of a step's opening gas kick left to the closing-pass adjoint of the step before
  // (same cells, same g): the step's start state and table
  bool open_pending = false;
  const float* open_q0 = nullptr;
  const StepScal* open_tab = nullptr;
  double* param_steps = nullptr;   // [cap][2 S] per-step dL/d(eps_sf, delta_c)
  int param_cap = 0;

  // learned closure: flat weights and their packed matrix-core form
  float* mlp_theta = nullptr;
  uint4* mlp_packed = nullptr;
  bool mlp_ready = false;

  // schedules (per sample)
  std::vector<std::vector<double>> recorded, replay;
  std::vector<size_t> replay_pos;

  // reverse mode
  std::vector<Ckpt> ckpts;
  Ckpt keep{};   // the state set aside during the reverse pass
  // per-step results of the last dh_forward: steps [0, store_valid) are held in store;
  // store_limit = how many steps this forward may keep (memory budget)
  std::vector<StepStore> store;
  int store_valid = 0, store_limit = 0;
  int store_max = -1;   // caller's cap on stored steps (< 0: none)
  // the forward's own tape of its first steps [0, taped) (whole checkpoint segments, or the
  // whole run): the reverse pass recomputes nothing there.  tape_limit = the budget of this
  // forward (a multiple of ckpt_every); store entries are then those of steps tape_limit + j.
  std::vector<TapeStep> ftape;
  int taped = 0, tape_limit = 0;
  std::vector<TapeStep> tape;
  std::vector<StepPlan> fwd_plans;   // plans of the last dh_forward, in order
  bool have_forward = false, have_loss = false;
  // which loss dh_backward(NULL) differentiates: the flux MSE (dh_loss), the Gaussian
  // power-spectrum loss (dh_power_loss) or the field-level posterior (dh_fli_loss)
  enum { kLossFlux = 0, kLossPower = 1, kLossFli = 2 };
  int loss_kind = kLossFlux;
  // power spectrum: block partials, bin counts of the last nbins, the loss's adjoint weights
  double* pk_part = nullptr;
  int pk_part_bins = 0;
  std::vector<double> pk_counts;
  int pk_counts_bins = 0;
  std::vector<float> pk_g;       // [S][nbins] spectral weights of the adjoint
  float* d_pk_g = nullptr;
  int pk_loss_bins = 0;
  // field-level posterior: data, noise variance and white noise (copies), [S][n^3] each
  float *fli_data = nullptr, *fli_nvar = nullptr, *fli_white = nullptr;
  double* fli_part = nullptr;
  int fwd_steps = 0;
  float* loss_target = nullptr;

  // kernel timing for measurement (dh_set_kernel_timing): the launches of one kernel family
  // inside steps and reverse passes are bracketed by HIP event pairs on the handle's stream
  int ktime_family = -1;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kt_events;
  size_t kt_used = 0;

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

// Records an event pair around the launches made during its lifetime when the handle times
// kernel family `fam` (see dh_set_kernel_timing); nothing otherwise.
struct KernelTimer {
  dh_sim* s;
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  KernelTimer(dh_sim* sim, int fam) : s(sim) {
    if (s->ktime_family != fam) return;
    if (s->kt_used == s->kt_events.size()) {
      std::pair<hipEvent_t, hipEvent_t> p{};
      DH_HIP(hipEventCreate(&p.first));
      DH_HIP(hipEventCreate(&p.second));
      s->kt_events.push_back(p);
    }
    ev = &s->kt_events[s->kt_used++];
    DH_HIP(hipEventRecord(ev->first, s->st));
  }
  ~KernelTimer() {
    if (ev) (void)hipEventRecord(ev->second, s->st);
  }
};

void copy_d2d(dh_sim* s, float* dst, const float* src, long long count) {
  DH_HIP(hipMemcpyAsync(dst, src, static_cast<size_t>(count) * sizeof(float),
                        hipMemcpyDeviceToDevice, s->st));
}

dh::HydroK hydro_at(const dh_sim* s, double a) {
  return dh::make_hydro(static_cast<float>(a), static_cast<float>(s->cfg.gamma),
                        static_cast<float>(s->e_floor));
}

void sync(dh_sim* s) { DH_HIP(hipStreamSynchronize(s->st)); }

Batch batch(const dh_sim* s, const StepScal* tab) { return Batch{s->n, s->S, tab, s->nq}; }

float green_at(const dh_sim* s, double a) {
  return static_cast<float>(-(1.5 * s->cfg.omega_m / a) / static_cast<double>(s->nc));
}

dh::SourceArgs source_args(const dh_sim* s, int smp, double a1, double dt, int step) {
  const dh_params& p = s->sprm[smp];
  dh::SourceArgs a{};
  a.a = a1;
  a.dt = dt;
  a.inv_rho_mean = 1.0 / s->f_b;
  a.omega_b = s->cfg.omega_b;
  a.efloor = s->e_floor;
  a.gamma = s->cfg.gamma;
  a.t_per_e = s->t_per_e;
  a.e0_code = p.e0 * 1e6 / (s->vel_unit * s->vel_unit);
  a.eps_sf = p.eps_sf;
  a.delta_c = p.delta_c;
  a.t_c = p.t_c;
  a.w_rho = p.w_rho;
  a.w_t = p.w_t;
  a.tau = s->cfg.tau;
  a.c_x = p.eps_sf * dt * std::sqrt(a.omega_b / (a1 * a1 * a1)) / 1.5707963267948966;
  a.k_rho = 1.0 / (p.w_rho * p.delta_c);
  a.k_t = 1.0 / (p.w_t * p.t_c);
  a.inv_tau = 1.0 / a.tau;
  a.mode = s->cfg.subgrid;
  const uint64_t seed = s->cfg.sf_seed + static_cast<uint64_t>(smp);   // sample s: key + s
  a.seed_lo = static_cast<uint32_t>(seed & 0xFFFFFFFFull);
  a.seed_hi = static_cast<uint32_t>(seed >> 32);
  a.step = static_cast<uint32_t>(step);
  a.mlp = s->cfg.closure == DH_CLOSURE_MLP ? s->mlp_packed : nullptr;
  return a;
}

StepScal entry_of(const dh_sim* s, int smp, const Plan& p, int step) {
  StepScal e{};
  e.src = source_args(s, smp, p.active ? p.a1 : p.a0, p.active ? p.dt : 0.0, step);
  e.active = p.active ? 1 : 0;
  if (!p.active) return e;
  e.dt = static_cast<float>(p.dt);
  e.h = static_cast<float>(0.5 * p.dt);
  if (s->cfg.kdk == DH_KDK_FASTPM) {
    double k0, dr, k1;
    dh::fastpm_factors(s->cosmo, s->heath, p.a0, p.ah, p.a1, &k0, &dr, &k1);
    e.h_open = static_cast<float>(k0);
    e.drift = static_cast<float>(dr);
    e.h_close = static_cast<float>(k1);
  } else {
    e.h_open = e.h_close = e.h;
    e.drift = static_cast<float>(p.dt / (p.ah * p.ah));
  }
  e.h1 = hydro_at(s, p.a0);
  e.h2 = hydro_at(s, p.ah);
  e.green = green_at(s, p.a1);
  e.h_dm = e.h_close;
  e.h_prev = s->kick_due[smp];
  return e;
}

// Grows the table store to hold `slots` steps (keeping the tables written so far).
void ensure_tab_slots(dh_sim* s, int slots) {
  if (slots <= s->tab_cap) return;
  const int cap = std::max(slots, 2 * s->tab_cap + 64);
  sync(s);
  StepScal* d = s->alloc<StepScal>(static_cast<long long>(cap) * s->S);
  double* sl = s->alloc<double>(static_cast<long long>(cap) * s->S);
  void* hp = nullptr;
  DH_HIP(hipHostMalloc(&hp, static_cast<size_t>(cap) * s->S * sizeof(StepScal),
                       hipHostMallocDefault));
  StepScal* h = static_cast<StepScal*>(hp);
  if (s->tabs) {
    const size_t bytes = static_cast<size_t>(s->tab_cap) * s->S * sizeof(StepScal);
    DH_HIP(hipMemcpy(d, s->tabs, bytes, hipMemcpyDeviceToDevice));
    DH_HIP(hipMemcpy(sl, s->speed_log, static_cast<size_t>(s->tab_cap) * s->S * sizeof(double),
                     hipMemcpyDeviceToDevice));
    std::memcpy(h, s->htabs, bytes);
    s->release(s->tabs);
    s->release(s->speed_log);
    (void)hipHostFree(s->htabs);
  }
  s->tabs = d;
  s->speed_log = sl;
  s->replayed.resize(static_cast<size_t>(cap) * s->S, 0.0);
  s->htabs = h;
  s->tab_cap = cap;
}

// Writes the table of a planned step into its slot (host mirror and device).  Each slot
// has its own pinned host memory, so no copy in flight is ever overwritten.
void upload_plan(dh_sim* s, const StepPlan& sp) {
  ensure_tab_slots(s, sp.slot + 1);
  StepScal* h = s->htabs + static_cast<size_t>(sp.slot) * s->S;
  for (int i = 0; i < s->S; ++i) h[i] = entry_of(s, i, sp.smp[i], sp.step);
  DH_HIP(hipMemcpyAsync(s->tabs + static_cast<size_t>(sp.slot) * s->S, h,
                        static_cast<size_t>(s->S) * sizeof(StepScal), hipMemcpyHostToDevice,
                        s->st));
}

const StepScal* tab_of(const dh_sim* s, const StepPlan& sp) {
  return s->tabs + static_cast<size_t>(sp.slot) * s->S;
}

// Table of the current state: every sample active at its own scale factor (Poisson green).
// The staging buffer is reused only after the stream has drained.
const StepScal* state_table(dh_sim* s) {
  sync(s);
  for (int i = 0; i < s->S; ++i) {
    StepScal e{};
    e.active = 1;
    e.green = green_at(s, s->a[i]);
    e.h1 = e.h2 = hydro_at(s, s->a[i]);
    e.src = source_args(s, i, s->a[i], 0.0, s->step);
    s->hstage[i] = e;
  }
  DH_HIP(hipMemcpyAsync(s->cur_tab, s->hstage, static_cast<size_t>(s->S) * sizeof(StepScal),
                        hipMemcpyHostToDevice, s->st));
  return s->cur_tab;
}

// Single entry for the stage calls (layout of one sample).  Repeated calls with the same
// entry reuse the device copy: no drain of the stream and no upload between their launches.
const StepScal* stage_table(dh_sim* s, const StepScal& e) {
  if (s->stage_valid && std::memcmp(&s->stage_last, &e, sizeof(StepScal)) == 0)
    return s->stage_tab;
  sync(s);
  s->hstage[0] = e;
  DH_HIP(hipMemcpyAsync(s->stage_tab, s->hstage, sizeof(StepScal), hipMemcpyHostToDevice, s->st));
  s->stage_last = e;
  s->stage_valid = true;
  return s->stage_tab;
}

// Applies the deferred closing kicks (same arithmetic as the kick at the end of a step).
void flush_kick(dh_sim* s) {
  if (!s->kick_pending) return;
  sync(s);
  for (int i = 0; i < s->S; ++i) {
    StepScal e{};
    e.active = s->kick_due[i] != 0.0f ? 1 : 0;
    e.h_close = s->kick_due[i];
    s->hstage[i] = e;
  }
  DH_HIP(hipMemcpyAsync(s->cur_tab, s->hstage, static_cast<size_t>(s->S) * sizeof(StepScal),
                        hipMemcpyHostToDevice, s->st));
  dh::launch_kick(s->st, s->g4, s->pos, s->mom, Batch{s->n, s->S, s->cur_tab, s->nq});
  std::fill(s->kick_due.begin(), s->kick_due.end(), 0.0f);
  s->kick_pending = false;
}

// drops deferred kicks that a new state replaces
void drop_kick(dh_sim* s) {
  std::fill(s->kick_due.begin(), s->kick_due.end(), 0.0f);
  s->kick_pending = false;
}

long long store_step_bytes(const dh_sim* s) {
  const long long S = s->S;
  return (s->nc * S + 1) * 4 + s->np * S * (4 + 16) + s->nc * S * 4;
}

// the dual-energy state with the smoothed injection (its tape keeps the injection field)
bool dual_smooth(const dh_sim* s) {
  return s->nq == 6 && s->cfg.sn_smooth && s->cfg.subgrid != DH_SUBGRID_OFF;
}

long long tape_entry_bytes(const dh_sim* s) {
  const long long S = s->S, nc = s->nc * S, np = s->np * S;
  const bool closure = s->cfg.closure == DH_CLOSURE_MLP && s->cfg.subgrid != DH_SUBGRID_OFF;
  return (closure ? 5 : 4) * s->nq * nc * 4 + 3 * np * 4 + nc * 4 + (nc + 1) * 4 + np * 4 +
         np * 16 + (dual_smooth(s) ? nc * 4 : 0);
}

// Device memory the first reverse pass still has to allocate (tape entries, adjoint buffers,
// the spare state set).
long long reverse_pass_bytes(const dh_sim* s) {
  const long long S = s->S, nc = s->nc * S, np = s->np * S;
  const long long entry = tape_entry_bytes(s);
  long long need = 0;
  const long long k = s->cfg.ckpt_every;
  if (static_cast<long long>(s->tape.size()) < k)
    need += (k - static_cast<long long>(s->tape.size())) * entry;
  if (!s->lq) need += (29 + 2 * (s->nq - 5)) * nc * 4;
  if (!s->keep.q) need += s->nq * nc * 4 + 6 * np * 4 + 2 * nc * 4;
  return need;
}

// What the next forward may keep for the reverse pass, from what the device has free after
// the reverse pass's own buffers and a margin of 4 GiB (entries allocated earlier are
// reused), within the caller's cap: first the full tape of whole checkpoint segments, then
// the sort and potential of further steps.
void plan_storage(dh_sim* s) {
  size_t free_b = 0, total_b = 0;
  long long avail = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
    avail = static_cast<long long>(free_b) - reverse_pass_bytes(s) - (4LL << 30);
  else
    (void)hipGetLastError();
  if (avail < 0) avail = 0;
  const long long K = s->cfg.ckpt_every;
  const long long cap = s->store_max >= 0 ? s->store_max : (1LL << 20);
  const long long entry = tape_entry_bytes(s), sstep = store_step_bytes(s);
  const long long have_t = static_cast<long long>(s->ftape.size());
  long long tl = std::min(cap, have_t + avail / entry);
  tl -= tl % K;
  const long long new_t = std::max(0LL, tl - have_t) * entry;
  const long long sl = std::min(cap - tl, static_cast<long long>(s->store.size()) +
                                              std::max(0LL, avail - new_t) / sstep);
  s->tape_limit = static_cast<int>(tl);
  s->store_limit = static_cast<int>(std::max(0LL, sl));
  s->store_valid = 0;
  s->taped = 0;
}

// Keeps the sort (the bins trade buffers with the store: no copy) and potential of the
// forward step with store index k (step tape_limit + k).  Returns false (and keeps nothing
// more in this forward) when the memory is not there.
bool keep_step(dh_sim* s, int k) {
  if (k >= s->store_limit || k != s->store_valid) return false;
  if (k == static_cast<int>(s->store.size())) {
    const long long S = s->S;
    StepStore e;
    void* p[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t bytes[4] = {static_cast<size_t>(s->nc * S + 1) * 4,
                             static_cast<size_t>(s->np * S) * 4,
                             static_cast<size_t>(s->np * S) * 16,
                             static_cast<size_t>(s->nc * S) * 4};
    for (int i = 0; i < 4; ++i) {
      if (hipMalloc(&p[i], bytes[i]) != hipSuccess) {
        (void)hipGetLastError();
        for (int j = 0; j < i; ++j) s->release(p[j]);
        s->store_limit = k;
        return false;
      }
      s->allocs.push_back(p[i]);
    }
    e.start = static_cast<uint32_t*>(p[0]);
    e.sorted = static_cast<uint32_t*>(p[1]);
    e.spos = static_cast<float4*>(p[2]);
    e.phi = static_cast<float*>(p[3]);
    s->store.push_back(e);
  }
  StepStore& e = s->store[k];
  std::swap(s->bins.start, e.start);
  std::swap(s->bins.sorted, e.sorted);
  std::swap(s->bins.spos, e.spos);
  copy_d2d(s, e.phi, s->phi, s->nc * s->S);
  s->store_valid = k + 1;
  return true;
}

// bins of the particle positions pos (all samples of b)
void sort_particles(dh_sim* s, const float* pos, const Batch& b) {
  dh::launch_keys(s->st, pos, s->bins.key, b);
  dh::launch_sort(s->st, s->bins, pos, b);
}

// phi_out = Poisson solve of delta with the Green's factor of each sample's table entry
void poisson(dh_sim* s, const float* delta, float* phi_out, const Batch& b) {
  dh::fft_forward_xy(s->st, delta, s->spec, s->tw, b);
  dh::fft_zpass_green(s->st, s->spec, s->tw, b);
  dh::fft_inverse_yx(s->st, s->spec, phi_out, s->tw, 1.0f, b);
}

// phi = Poisson(rho_gas + m_dm CIC(pos) - 1) and g4 = -grad(phi), with the bins of the
// particle positions already built
void potential_from_bins(dh_sim* s, const float* rho_gas, float* phi_out, float4* g4_out,
                         const Batch& b) {
  dh::launch_deposit(s->st, s->bins, rho_gas, s->nq * s->nc, static_cast<float>(s->m_dm), -1.0f,
                     s->delta, b);
  poisson(s, s->delta, phi_out, b);
  dh::launch_grad(s->st, phi_out, g4_out, b);
}

void state_changed(dh_sim* s) {
  s->cfl_partials = false;
  s->speed_known = false;
}

// CFL speeds, max over cells and axes of (|U_d| + c_s)/a, of each sample's current state
// (FP64 on the device); +inf when a state holds a non-finite value or a non-positive density
const std::vector<double>& current_speed(dh_sim* s) {
  if (s->speed_known) return s->speed;
  const int nb = dh::cfl_blocks(s->n);
  if (!s->cfl_partials) {
    sync(s);
    std::memcpy(s->host_out, s->a.data(), s->S * sizeof(double));
    DH_HIP(hipMemcpyAsync(s->d_acur, s->host_out, s->S * sizeof(double), hipMemcpyHostToDevice,
                          s->st));
    dh::launch_cfl_partial(s->st, s->q, s->d_acur, s->cfg.gamma, s->e_floor, s->cfl_red,
                           batch(s, nullptr));
  }
  dh::launch_reduce_max(s->st, s->cfl_red, nb, nb, s->S, s->red_out);
  DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, s->S * sizeof(double), hipMemcpyDeviceToHost,
                        s->st));
  sync(s);
  s->speed.assign(s->host_out, s->host_out + s->S);
  s->speed_known = true;
  s->cfl_partials = true;
  return s->speed;
}

bool all_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// Closing pass of a step from q_in (the state after the sweeps) into s->q: gas half kick,
// source term (kicked state to q_kicked if given), star field and CFL maxima if `full`; then
// the smoothed supernova injection (cfg.sn_smooth, with the CFL maxima) and, if `readout`,
// the step's new stars read out on the particles (cfg.star_dm; spos, sorted: the sort of the
// end-of-step positions).
void close_pass(dh_sim* s, const float* q_in, float* q_kicked, bool full, bool readout,
                const float4* spos, const uint32_t* sorted, const Batch& b, bool closure,
                float* sn = nullptr) {
  const bool smooth = s->cfg.sn_smooth && s->cfg.subgrid != DH_SUBGRID_OFF;
  const bool stars = readout && full && s->znew && s->cfg.subgrid != DH_SUBGRID_OFF;
  float* snb = sn ? sn : s->sn_buf;   // a tape keeps the injection field where it has room
  dh::launch_close_step(s->st, q_in, s->q, s->g4, full ? s->star : nullptr, q_kicked,
                        s->cfg.gamma, full && !smooth ? s->cfl_red : nullptr, b, closure,
                        stars ? s->znew : nullptr, smooth ? snb : nullptr);
  if (smooth) dh::launch_sn_inject(s->st, snb, s->q, s->cfg.gamma, full ? s->cfl_red : nullptr, b);
  if (stars) dh::launch_star_readout(s->st, s->znew, spos, sorted, s->aux, b);
}

// One step of the method on the handle state.  With a tape entry, keeps its intermediates.
// defer: leave the closing dark-matter kick to the next step's kick-drift pass.
// store_k >= 0: store index of a forward step (no tape: keep its sort and potential if the
// budget allows; recomputing: take them from the store when it holds them).  recompute: the
// reverse pass's recomputation into a tape (else a tape entry records a forward step).
void do_step(dh_sim* s, const StepPlan& sp, TapeStep* tp, bool defer, int store_k,
             bool recompute) {
  const long long nc = s->nc, np = s->np;
  if (!defer) flush_kick(s);
  const bool prev = s->kick_pending;
  const Batch b = batch(s, tab_of(s, sp));
  const float* pos_in = s->pos;
  if (tp) {
    tp->plan = sp;
    bool all = true;
    for (int i = 0; i < s->S; ++i) all = all && sp.smp[i].active;
    if (all) {
      // every sample moves: the state buffers become the tape's step-start entries and the
      // step writes the new state into the tape's former buffers (every pass below writes
      // all of its output), so nothing is copied
      std::swap(s->q, tp->q[0]);
      std::swap(s->pos, tp->x0);
      std::swap(s->phi, tp->phi0);
      pos_in = tp->x0;
    } else {
      copy_d2d(s, tp->q[0], s->q, s->nq * nc * s->S);
      copy_d2d(s, tp->x0, s->pos, 3 * np * s->S);
      copy_d2d(s, tp->phi0, s->phi, nc * s->S);
    }
  }
  const bool closure = s->cfg.closure == DH_CLOSURE_MLP && s->cfg.subgrid != DH_SUBGRID_OFF;
  if (tp) {
    // the sweeps (the first one also applies the opening gas kick) and the closing pass write
    // their results straight into the tape
    const bool kept = recompute && store_k >= 0 && store_k < s->store_valid;
    dh::launch_kick_drift(s->st, s->g4, pos_in, s->pos, s->mom, s->bins.key, nullptr, nullptr,
                          prev, b, kept ? nullptr : &s->bins);
    {
      KernelTimer kt(s, DH_KTIME_SWEEP_KICK);
      dh::launch_sweep(s->st, tp->q[0], tp->q[2], b, sp.axes[0], s->g4);
    }
    for (int k = 1; k < 3; ++k) {
      KernelTimer kt(s, DH_KTIME_SWEEP);
      dh::launch_sweep(s->st, tp->q[1 + k], tp->q[2 + k], b, sp.axes[k]);
    }
    if (kept) {
      // the forward kept this step's sort and potential: no sort, deposit or Poisson solve
      const StepStore& e = s->store[store_k];
      copy_d2d(s, s->phi, e.phi, nc * s->S);
      dh::launch_grad(s->st, s->phi, s->g4, b);
      tp->vstart = e.start;
      tp->vsorted = e.sorted;
      tp->vspos = e.spos;
    } else {
      dh::launch_sort(s->st, s->bins, s->pos, b, true);
      potential_from_bins(s, tp->q[4], s->phi, s->g4, b);
      // the tape keeps this sort of x1 for the reverse pass; the next sort writes the tape's
      // former buffers
      std::swap(s->bins.start, tp->start);
      std::swap(s->bins.sorted, tp->sorted);
      std::swap(s->bins.spos, tp->spos);
      tp->vstart = tp->start;
      tp->vsorted = tp->sorted;
      tp->vspos = tp->spos;
    }
    // the recomputation needs neither the star field nor the CFL maxima (plain source)
    const bool full = !recompute || closure;
    close_pass(s, tp->q[4], closure ? tp->q[5] : nullptr, full, !recompute, tp->vspos,
               tp->vsorted, b, closure, tp->sn);
  } else {
    // opening half kicks with g_n (the gas one inside the first sweep), drift with
    // a(t + dt/2)
    dh::launch_kick_drift(s->st, s->g4, s->pos, s->pos, s->mom, s->bins.key, nullptr, nullptr,
                          prev, b, &s->bins);
    // sweeps in the Strang order of the step (a sample that sits out is copied along)
    for (int k = 0; k < 3; ++k) {
      KernelTimer kt(s, k == 0 ? DH_KTIME_SWEEP_KICK : DH_KTIME_SWEEP);
      dh::launch_sweep(s->st, s->q, s->q2, b, sp.axes[k], k == 0 ? s->g4 : nullptr);
      std::swap(s->q, s->q2);
    }
    // Poisson at a(t + dt) from gas + DM (keys and their histogram were made by the drift)
    dh::launch_sort(s->st, s->bins, s->pos, b, true);
    potential_from_bins(s, s->q, s->phi, s->g4, b);
    // closing gas half kick with g_{n+1}, source term and the CFL maxima: one pass
    close_pass(s, s->q, nullptr, true, true, s->bins.spos, s->bins.sorted, b, closure);
    if (store_k >= 0) keep_step(s, store_k);
  }
  // closing dark-matter half kick with g_{n+1} (deferred: the factor the table holds)
  if (!defer) dh::launch_kick(s->st, s->g4, s->pos, s->mom, b);
  DH_LAUNCH_CHECK();
  bool all = true;
  for (int i = 0; i < s->S; ++i) {
    const Plan& p = sp.smp[i];
    if (!p.active) {
      all = false;
      continue;
    }
    if (defer) {
      s->kick_due[i] = s->htabs[static_cast<size_t>(sp.slot) * s->S + i].h_close;
      s->kick_pending = true;
    }
    s->t[i] = p.t0 + p.dt;
    s->a[i] = p.a1;
  }
  s->step = sp.step + 1;
  s->speed_known = false;
  // the closing pass left the CFL maxima of every sample that moved (zeros for the others),
  // except in the reverse pass's recomputation
  s->cfl_partials = all && !recompute;
}

void refresh_potential(dh_sim* s) {
  const Batch b = batch(s, state_table(s));
  sort_particles(s, s->pos, b);
  potential_from_bins(s, s->q, s->phi, s->g4, b);
  s->phi_valid = true;
}

void reset_clock(dh_sim* s) {
  const double ai = s->cfg.a_init;
  std::fill(s->t.begin(), s->t.end(), s->cosmo.t_of_a(ai));
  std::fill(s->a.begin(), s->a.end(), ai);
  s->step = 0;
  s->nslots = 0;
  s->checked_slots = 0;
  std::fill(s->replayed.begin(), s->replayed.end(), 0.0);
  for (auto& r : s->recorded) r.clear();
  std::fill(s->replay_pos.begin(), s->replay_pos.end(), 0);
}

// The spectral operator op (kOpIcDisp, kOpIcHess, ...) of the initial conditions with the
// handle's linear spectrum at a_init
dh::IcOp ic_op(const dh_sim* s, int op, int axis, int axis2 = 0, double scale = 1.0) {
  const int n = s->n;
  const double ai = s->cfg.a_init;
  const double d = s->cosmo.growth(ai);
  dh::IcOp o;
  o.op = op;
  o.axis = axis;
  o.axis2 = axis2;
  o.amp = s->amp * d * d / std::pow(s->cfg.box / n, 3.0);
  o.n_s = s->cfg.n_s;
  o.om_h = s->cfg.omega_m * s->cfg.h;
  o.kphys = n / s->cfg.box;
  o.scale = scale;
  o.eh = s->cfg.transfer == DH_TRANSFER_EH;
  const dh::EhShape e = dh::eh_shape(s->cfg.omega_m, s->cfg.omega_b, s->cfg.h);
  o.eh_theta2 = e.theta2;
  o.eh_alpha = e.alpha;
  o.eh_ks = e.ks;
  return o;
}

// second derivative k of the linear potential: (xx, yy, zz, xy, xz, yz)
const int kHessAxes[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};

// second-order LPT at a_init: (-D2 / D1^2, f2 / f1) with D2 = -3/7 D1^2 Omega_m(a)^(-1/143),
// f2 = 2 Omega_m(a)^(6/11) (fits of Bouchet et al. 1995)
void lpt2_factors(const dh_sim* s, double* c2, double* r) {
  const double ai = s->cfg.a_init;
  const double om_a = s->cfg.omega_m / (ai * ai * ai * s->cosmo.E(ai) * s->cosmo.E(ai));
  *c2 = 3.0 / 7.0 * std::pow(om_a, -1.0 / 143.0);
  *r = 2.0 * std::pow(om_a, 6.0 / 11.0) / s->cosmo.growth_rate(ai);
}

void initial_conditions(dh_sim* s, const float* d_white) {
  const int n = s->n;
  const long long nc = s->nc;
  const double ai = s->cfg.a_init;
  const Batch all = batch(s, nullptr);
  dh::fft_forward_xy(s->st, d_white, s->spec2, s->tw, all);
  dh::fft_zpass_forward(s->st, s->spec2, s->spec2, s->tw, all);
  for (int j = 0; j < 3; ++j) {
    dh::fft_zpass_ic(s->st, s->spec2, s->spec, s->tw, ic_op(s, dh::kOpIcDisp, j), false, true,
                     false, all);
    dh::fft_inverse_yx(s->st, s->spec, s->psi + j * nc, s->tw, 1.0f, all, 3 * nc);
  }
  const float* vel = s->psi;
  if (s->cfg.lpt == 2) {
    // second derivatives of the linear potential, the source delta2 and its displacement
    for (int k = 0; k < 6; ++k) {
      dh::fft_zpass_ic(s->st, s->spec2, s->spec, s->tw,
                       ic_op(s, dh::kOpIcHess, kHessAxes[k][0], kHessAxes[k][1]), false, true,
                       false, all);
      dh::fft_inverse_yx(s->st, s->spec, s->hess + k * nc, s->tw, 1.0f, all, 6 * nc);
    }
    dh::launch_lpt2_source(s->st, s->hess, s->delta, all);
    double c2, r;
    lpt2_factors(s, &c2, &r);
    dh::fft_forward_xy(s->st, s->delta, s->spec, s->tw, all);
    for (int j = 0; j < 3; ++j) {
      dh::fft_zpass_ic(s->st, s->spec, s->spec2, s->tw, ic_op(s, dh::kOpZa, j, 0, c2), true, true,
                       false, all);
      dh::fft_inverse_yx(s->st, s->spec2, s->fscratch + j * nc, s->tw, 1.0f, all, 3 * nc);
    }
    dh::launch_lpt2_combine(s->st, s->psi, s->fscratch, s->lptv, static_cast<float>(r),
                            3 * nc * s->S);
    vel = s->lptv;
  }
  const double vfac = ai * ai * s->cosmo.E(ai) * s->cosmo.growth_rate(ai);
  drop_kick(s);
  dh::launch_ic_particles(s->st, s->psi, vel, s->pos, s->mom, static_cast<float>(vfac), all);
  sort_particles(s, s->pos, all);
  dh::launch_deposit(s->st, s->bins, nullptr, 0, 1.0f, 0.0f, s->cic, all);
  dh::launch_ic_gas(s->st, s->cic, vel, s->q, static_cast<float>(s->f_b),
                    static_cast<float>(vfac), static_cast<float>(ai), static_cast<float>(s->e_init),
                    s->cfg.gamma, all);
  dh::launch_fill(s->st, s->star, 0.0f, s->nc * s->S);
  if (s->aux) dh::launch_fill(s->st, s->aux, 0.0f, s->np * s->S);
  reset_clock(s);
  potential_from_bins(s, s->q, s->phi, s->g4, batch(s, state_table(s)));
  s->phi_valid = true;
  state_changed(s);
  s->initialised = true;
}

// Plans the next step of every sample: the next schedule entry, or the CFL dt (eq. dt) with
// the dln a cap, clipped to land on t_end (< 0: none).  A sample at t_end, or whose replayed
// schedule is used up (with stop_at_replay_end), sits out.  *any = whether a sample moves.
// the current scale factor of every sample into d_acur
void upload_scale_factors(dh_sim* s) {
  sync(s);
  std::memcpy(s->host_out, s->a.data(), s->S * sizeof(double));
  DH_HIP(hipMemcpyAsync(s->d_acur, s->host_out, s->S * sizeof(double), hipMemcpyHostToDevice,
                        s->st));
}

// Mode counts W_b (full spectrum) of bins 1..nbins of the rounded |m|: host, exact, cached.
const std::vector<double>& pk_counts(dh_sim* s, int nbins) {
  if (s->pk_counts_bins == nbins) return s->pk_counts;
  const int n = s->n;
  std::vector<double> w(nbins, 0.0);
  for (int kz = 0; kz < n; ++kz) {
    const long long mz = kz <= n / 2 ? kz : kz - n;
    for (int ky = 0; ky < n; ++ky) {
      const long long my = ky <= n / 2 ? ky : ky - n;
      for (int kx = 0; kx <= n / 2; ++kx) {
        const long long m2 = static_cast<long long>(kx) * kx + my * my + mz * mz;
        long long j = static_cast<long long>(std::sqrt(static_cast<double>(m2)) + 0.5);
        if (4 * m2 >= (2 * j + 1) * (2 * j + 1)) ++j;
        if (j > 0 && 4 * m2 < (2 * j - 1) * (2 * j - 1)) --j;
        if (j >= 1 && j <= nbins) w[j - 1] += (kx == 0 || kx == n / 2) ? 1.0 : 2.0;
      }
    }
  }
  s->pk_counts = w;
  s->pk_counts_bins = nbins;
  return s->pk_counts;
}

// half spectrum of each sample's gas density into s->spec (forward, unnormalised)
void density_spectrum(dh_sim* s, const Batch& b) {
  dh::fft_forward_xy(s->st, s->q, s->spec, s->tw, b, s->nq * s->nc);
  dh::fft_zpass_forward(s->st, s->spec, s->spec, s->tw, b);
}

// power spectrum of the current gas overdensity: pk[s][b] (FP64, host)
void power_spectrum(dh_sim* s, int nbins, std::vector<double>& pk) {
  const int S = s->S;
  const int nblk = dh::pk_blocks(s->n);
  if (s->pk_part_bins < nbins) {
    if (s->pk_part) s->release(s->pk_part);
    s->pk_part = nullptr;
    s->pk_part = s->alloc<double>(static_cast<long long>(S) * nbins * nblk);
    s->pk_part_bins = nbins;
  }
  const Batch b = batch(s, nullptr);
  density_spectrum(s, b);
  dh::launch_pk_bin(s->st, s->spec, nbins, s->pk_part, b);
  std::vector<double> sums(static_cast<size_t>(S) * nbins);
  double* d_sums = s->red;   // S nbins <= 8 red_blocks S + 8 doubles
  dh::launch_reduce_sum(s->st, s->pk_part, nblk, nblk, S * nbins, d_sums);
  DH_HIP(hipMemcpyAsync(sums.data(), d_sums, sums.size() * sizeof(double), hipMemcpyDeviceToHost,
                        s->st));
  sync(s);
  const std::vector<double>& w = pk_counts(s, nbins);
  const double n3 = static_cast<double>(s->nc);
  // P_b = (L^3 / n^6) sum |X|^2 / W_b of delta = rho / rho_mean - 1 (X of rho / rho_mean: the
  // mean only enters the mode m = 0, outside every bin)
  const double c = s->cfg.box * s->cfg.box * s->cfg.box / (n3 * n3) / (s->f_b * s->f_b);
  pk.assign(sums.size(), 0.0);
  for (int i = 0; i < S; ++i)
    for (int k = 0; k < nbins; ++k)
      pk[static_cast<size_t>(i) * nbins + k] = c * sums[static_cast<size_t>(i) * nbins + k] / w[k];
}

// adjoint of the power-spectrum loss into lam_rho (component 0 of s->lq): with G_m = g_b c /
// W_b, dL/drho_x = 2 sum_m G_m Re(X_m e^{i k_m x}), i.e. twice the unnormalised inverse
// transform of G X
void power_loss_vjp(dh_sim* s) {
  const Batch b = batch(s, nullptr);
  const int nbins = s->pk_loss_bins;
  if (!s->d_pk_g) s->d_pk_g = s->alloc<float>(static_cast<long long>(s->S) * (s->n / 2));
  DH_HIP(hipMemcpyAsync(s->d_pk_g, s->pk_g.data(), s->pk_g.size() * sizeof(float),
                        hipMemcpyHostToDevice, s->st));
  density_spectrum(s, b);
  dh::launch_pk_scale(s->st, s->spec, s->d_pk_g, nbins, b);
  dh::fft_zpass_inverse(s->st, s->spec, s->tw, b);
  dh::fft_inverse_yx(s->st, s->spec, s->lq, s->tw, 2.0f, b, s->nq * s->nc);
  sync(s);   // pk_g is host memory read by the copy above
}

int plan_step(dh_sim* s, double t_end, bool stop_at_replay_end, StepPlan& sp, bool* any) {
  sp.step = s->step;
  for (int k = 0; k < 3; ++k) sp.axes[k] = kStrang[s->step % 6][k];
  sp.smp.assign(s->S, Plan{});
  *any = false;
  const std::vector<double>* speeds = nullptr;
  for (int i = 0; i < s->S; ++i) {
    Plan& p = sp.smp[i];
    p.t0 = s->t[i];
    p.a0 = s->a[i];
    p.active = false;
    if (t_end > 0.0 && s->t[i] >= t_end * (1.0 - 1e-12)) continue;
    double dt;
    p.replayed = false;
    if (s->replay_pos[i] < s->replay[i].size()) {
      dt = s->replay[i][s->replay_pos[i]];
      if (!(dt > 0.0) || !std::isfinite(dt))
        return fail(s, DH_E_SCHEDULE, "schedule entry is not a positive finite dt");
      if (t_end > 0.0 && s->t[i] + dt > t_end) dt = t_end - s->t[i];
      p.replayed = true;
    } else {
      if (stop_at_replay_end && !s->replay[i].empty()) continue;
      if (!speeds) speeds = &current_speed(s);
      const double v = (*speeds)[i];
      if (!std::isfinite(v) || !(v > 0.0))
        return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
      dt = std::min(s->cfg.cfl / v, s->cfg.dlna_max / s->cosmo.E(s->a[i]));
      if (t_end > 0.0 && s->t[i] + dt > t_end) dt = t_end - s->t[i];
    }
    p.dt = dt;
    p.ah = s->cosmo.a_of_t(p.t0 + 0.5 * dt);
    p.a1 = s->cosmo.a_of_t(p.t0 + dt);
    p.active = true;
    *any = true;
  }
  return DH_OK;
}

void commit_plan(dh_sim* s, const StepPlan& sp) {
  for (int i = 0; i < s->S; ++i) {
    if (!sp.smp[i].active) continue;
    if (s->replay_pos[i] < s->replay[i].size()) ++s->replay_pos[i];
    s->recorded[i].push_back(sp.smp[i].dt);
  }
}

// Checks the handle and plans the next step of all samples (plan_step).
int prepare_step(dh_sim* s, double t_end, bool stop_at_replay_end, StepPlan& sp, bool* any) {
  if (!s->initialised) return fail(s, DH_E_STATE, "no initial state");
  if (s->cfg.closure == DH_CLOSURE_MLP && !s->mlp_ready)
    return fail(s, DH_E_STATE, "closure network weights not set (dh_set_closure)");
  if (!s->phi_valid) refresh_potential(s);
  return plan_step(s, t_end, stop_at_replay_end, sp, any);
}

// CFL speed of the current state of every sample into the speed log of a replayed step's
// slot (device to device: the run does not wait for it; check_replay reads the log).
void log_replay_speed(dh_sim* s, const StepPlan& sp) {
  bool any = false;
  for (int i = 0; i < s->S; ++i) {
    const Plan& p = sp.smp[i];
    s->replayed[static_cast<size_t>(sp.slot) * s->S + i] = p.active && p.replayed ? p.dt : 0.0;
    any = any || (p.active && p.replayed);
  }
  if (!any || !(s->cfg.cfl_forward > 0.0)) return;
  const int nb = dh::cfl_blocks(s->n);
  if (!s->cfl_partials) {
    sync(s);
    std::memcpy(s->host_out, s->a.data(), s->S * sizeof(double));
    DH_HIP(hipMemcpyAsync(s->d_acur, s->host_out, s->S * sizeof(double), hipMemcpyHostToDevice,
                          s->st));
    dh::launch_cfl_partial(s->st, s->q, s->d_acur, s->cfg.gamma, s->e_floor, s->cfl_red,
                           batch(s, nullptr));
    s->cfl_partials = true;
  }
  dh::launch_reduce_max(s->st, s->cfl_red, nb, nb, s->S,
                        s->speed_log + static_cast<size_t>(sp.slot) * s->S);
}

// Accuracy check of the replayed steps taken since the last check (Sec. 2.3.3): each
// replayed dt times the CFL speed of the state it was applied to, its Courant number on
// that state, may not exceed cfg.cfl_forward.
int check_replay(dh_sim* s) {
  const int from = s->checked_slots, to = s->nslots;
  s->checked_slots = to;
  if (!(s->cfg.cfl_forward > 0.0) || to <= from) return DH_OK;
  const size_t S = static_cast<size_t>(s->S);
  bool any = false;
  for (size_t k = from * S; k < to * S; ++k) any = any || s->replayed[k] > 0.0;
  if (!any) return DH_OK;
  std::vector<double> v((to - from) * S);
  DH_HIP(hipMemcpyAsync(v.data(), s->speed_log + from * S, v.size() * sizeof(double),
                        hipMemcpyDeviceToHost, s->st));
  sync(s);
  for (int k = from; k < to; ++k)
    for (size_t i = 0; i < S; ++i) {
      const double dt = s->replayed[k * S + i];
      if (!(dt > 0.0)) continue;
      const double c = dt * v[(k - from) * S + i];
      if (!(c <= s->cfg.cfl_forward * (1.0 + 1e-9)))
        return fail(s, DH_E_SCHEDULE,
                    "replayed step " + std::to_string(k) + " of sample " + std::to_string(i) +
                        " has Courant number " + std::to_string(c) + " > cfl_forward " +
                        std::to_string(s->cfg.cfl_forward) + " on this run's state");
    }
  return DH_OK;
}

// Takes a planned step (at least one sample moves).
void take_step(dh_sim* s, StepPlan& sp, bool defer, int store_k = -1,
               TapeStep* tp = nullptr) {
  sp.slot = s->nslots++;
  upload_plan(s, sp);
  log_replay_speed(s, sp);
  do_step(s, sp, tp, defer, store_k, false);
  commit_plan(s, sp);
}

// Plans and takes one step of all samples; *moved = false when no sample had a step left.
int step_once(dh_sim* s, double t_end, bool stop_at_replay_end, StepPlan* out, bool* moved,
              bool defer) {
  StepPlan sp;
  bool any = false;
  int rc = prepare_step(s, t_end, stop_at_replay_end, sp, &any);
  if (rc) return rc;
  *moved = any;
  if (!any) return DH_OK;
  take_step(s, sp, defer);
  if (out) *out = sp;
  return DH_OK;
}

void alloc_tape_entry(dh_sim* s, TapeStep& t) {
  const long long S = s->S;
  const bool closure = s->cfg.closure == DH_CLOSURE_MLP && s->cfg.subgrid != DH_SUBGRID_OFF;
  for (int k = 0; k < 6; ++k)
    t.q[k] = k != 1 && (k < 5 || closure) ? s->alloc<float>(s->nq * s->nc * S) : nullptr;
  t.x0 = s->alloc<float>(3 * s->np * S);
  t.x1 = nullptr;
  t.phi0 = s->alloc<float>(s->nc * S);
  t.phi1 = nullptr;
  t.start = s->alloc<uint32_t>(s->nc * S + 1);
  t.sorted = s->alloc<uint32_t>(s->np * S);
  t.spos = s->alloc<float4>(s->np * S);
  t.sn = dual_smooth(s) ? s->alloc<float>(s->nc * S) : nullptr;
}

// alloc_tape_entry that gives the memory back and returns false when it is not there
bool try_alloc_tape_entry(dh_sim* s, TapeStep& t) {
  const size_t mark = s->allocs.size();
  try {
    alloc_tape_entry(s, t);
    return true;
  } catch (const std::bad_alloc&) {
    (void)hipGetLastError();
    while (s->allocs.size() > mark) s->release(s->allocs.back());
    t = TapeStep{};
    return false;
  }
}

void save_ckpt(dh_sim* s, Ckpt& c) {
  const long long S = s->S;
  flush_kick(s);
  if (!c.q) {
    c.q = s->alloc<float>(s->nq * s->nc * S);
    c.pos = s->alloc<float>(3 * s->np * S);
    c.mom = s->alloc<float>(3 * s->np * S);
    c.star = s->alloc<float>(s->nc * S);
    c.phi = s->alloc<float>(s->nc * S);
  }
  copy_d2d(s, c.q, s->q, s->nq * s->nc * S);
  copy_d2d(s, c.pos, s->pos, 3 * s->np * S);
  copy_d2d(s, c.mom, s->mom, 3 * s->np * S);
  copy_d2d(s, c.star, s->star, s->nc * S);
  copy_d2d(s, c.phi, s->phi, s->nc * S);
  c.t = s->t;
  c.a = s->a;
  c.step = s->step;
}

void load_ckpt(dh_sim* s, const Ckpt& c) {
  const long long S = s->S;
  drop_kick(s);
  copy_d2d(s, s->q, c.q, s->nq * s->nc * S);
  copy_d2d(s, s->pos, c.pos, 3 * s->np * S);
  copy_d2d(s, s->mom, c.mom, 3 * s->np * S);
  copy_d2d(s, s->star, c.star, s->nc * S);
  copy_d2d(s, s->phi, c.phi, s->nc * S);
  s->t = c.t;
  s->a = c.a;
  s->step = c.step;
  dh::launch_grad(s->st, s->phi, s->g4, batch(s, nullptr));
  s->phi_valid = true;
  state_changed(s);
}

// Moves the state buffers aside without copying (the reverse pass then works in a spare set,
// allocated once) and back again afterwards.
void stash_state(dh_sim* s) {
  flush_kick(s);
  Ckpt& c = s->keep;
  const long long S = s->S;
  if (!c.q) {
    c.q = s->alloc<float>(s->nq * s->nc * S);
    c.pos = s->alloc<float>(3 * s->np * S);
    c.mom = s->alloc<float>(3 * s->np * S);
    c.star = s->alloc<float>(s->nc * S);
    c.phi = s->alloc<float>(s->nc * S);
  }
  std::swap(s->q, c.q);
  std::swap(s->pos, c.pos);
  std::swap(s->mom, c.mom);
  std::swap(s->star, c.star);
  std::swap(s->phi, c.phi);
  c.t = s->t;
  c.a = s->a;
  c.step = s->step;
}

void unstash_state(dh_sim* s) {
  Ckpt& c = s->keep;
  drop_kick(s);
  std::swap(s->q, c.q);
  std::swap(s->pos, c.pos);
  std::swap(s->mom, c.mom);
  std::swap(s->star, c.star);
  std::swap(s->phi, c.phi);
  s->t = c.t;
  s->a = c.a;
  s->step = c.step;
  dh::launch_grad(s->st, s->phi, s->g4, batch(s, nullptr));
  s->phi_valid = true;
  state_changed(s);
}

// Adjoint of one step.  In: lq, lx, lp, lphi = adjoints of the state after the step (lphi is
// the adjoint of phi_{n+1} from the following step).  Out: the same buffers hold the
// adjoints of the state at the start of the step.
// The opening dark-matter kick of the following step acts at the same positions, with the
// same g and the same adjoint momentum as this step's closing kick, so its adjoint is merged
// here (factor h_dm = h of this step + h of the next, the latter 0 after a sample's last
// step); this step's own opening kick is left to the previous step, or to
// finish_first_kick after the first step.  A sample that sat the step out keeps its adjoints.
// defer_open: the step before is the next one to be processed (same tape): the opening gas
// kick's adjoint may be left to its closing-pass adjoint (one pass over the cells).
void opening_kick_vjp(dh_sim* s, const float* q0, const Batch& b) {
  dh::launch_gas_kick_vjp(s->st, q0, s->g4b, s->lq, s->lg, b);
  dh::launch_grad_vjp(s->st, s->lg, nullptr, s->lphi, b);
}

void flush_open_vjp(dh_sim* s) {
  if (!s->open_pending) return;
  opening_kick_vjp(s, s->open_q0, Batch{s->n, s->S, s->open_tab, s->nq});
  s->open_pending = false;
}

void step_vjp(dh_sim* s, const TapeStep& T, bool defer_open) {
  const long long nc = s->nc;
  const StepPlan& sp = T.plan;
  const Batch b = batch(s, tab_of(s, sp));
  hipStream_t st = s->st;
  const bool source = s->cfg.subgrid != DH_SUBGRID_OFF;
  const bool closure = source && s->cfg.closure == DH_CLOSURE_MLP;
  // source term and closing kicks (gas from Q4, DM at x1) -> lambda_g -> lambda_phi_{n+1}.
  // phi1 of this step is phi0 of the next one (bit for bit, also across a checkpoint), whose
  // gradient the previous call left in g4b when every sample moved in both steps
  bool all = true;
  for (int i = 0; i < s->S; ++i) all = all && sp.smp[i].active;
  const bool reuse = all && s->g4b_phi0_of == sp.step + 1;
  // with the dual-energy state and the smoothed injection the reset's adjoint below needs the
  // next step's opening kick taken first: not fused
  const bool fuse_open = s->open_pending && reuse && !closure && !dual_smooth(s);
  if (!fuse_open) flush_open_vjp(s);   // with the next step's g, still in g4b
  if (!reuse) dh::launch_grad(st, T.phi1, s->g4b, b);
  const int nb = dh::source_vjp_blocks(s->n);
  // smoothed injection: the adjoint of each cell's injected energy is the smoothing of the
  // energy adjoint (the weights are symmetric); the next step's opening gas kick leaves the
  // energy adjoint unchanged, so it may be taken before the fused kernel applies that kick
  const float* lam_inj = nullptr;
  if (source && s->cfg.sn_smooth && s->nq == 6) {
    // dual energy: the reset after the injection and the entropy's share of it first
    dh::launch_inject_sync_vjp(st, T.q[4], s->g4b, T.sn, s->lq, s->sn_buf2, b);
    dh::launch_smooth27(st, s->sn_buf2, nc, s->sn_buf, b);
    lam_inj = s->sn_buf;
  } else if (source && s->cfg.sn_smooth) {
    dh::launch_smooth27(st, s->lq + 4 * nc, s->nq * nc, s->sn_buf, b);
    lam_inj = s->sn_buf;
  }
  if (closure) {
    dh::launch_source_vjp(st, T.q[5], s->lq, s->red, b, lam_inj);
    dh::launch_gas_kick_vjp(st, T.q[4], s->g4b, s->lq, s->lg, b);
  } else if (fuse_open) {
    dh::launch_source_kick_vjp(st, T.q[4], s->g4b, s->lq, s->lg, s->red, b, s->open_q0, s->lg2,
                               s->open_tab, lam_inj);
    s->open_pending = false;
  } else {
    dh::launch_source_kick_vjp(st, T.q[4], s->g4b, s->lq, s->lg, s->red, b, nullptr, nullptr,
                               nullptr, lam_inj);
  }
  if (source)
    dh::launch_reduce_sum(st, s->red, nb, nb, 2 * s->S, s->param_steps + 2LL * s->S * sp.slot);
  // x1 in bin order as the recomputed step's sort left it, then lambda_p in the same order
  dh::Bins tb = s->bins;
  tb.start = T.vstart;
  tb.sorted = T.vsorted;
  tb.spos = T.vspos;
  dh::launch_gather_sorted(st, tb, s->lp, b);
  dh::launch_deposit_vec(st, tb, true, s->lg, b);
  // lambda_phi_{n+1}: with the next step's opening kick taken above, its g adjoint (lg2) first
  if (fuse_open)
    dh::launch_grad_vjp2(st, s->lg2, s->lg, s->lphi2, b);
  else
    dh::launch_grad_vjp(st, s->lg, s->lphi, s->lphi2, b);
  // Poisson (symmetric operator) and deposit at x1
  poisson(s, s->lphi2, s->ldelta, b);
  dh::launch_axpy(st, s->lq, s->ldelta, 1.0f, nc, s->nq * nc, nc, false, b);
  // with the kicks' term at x1 (g4b still holds g_{n+1}) and the drift
  // x1 = x0 + p_half dt / a_h^2: lambda_p += (dt / a_h^2) lambda_x
  dh::launch_deposit_vjp_pos(st, s->ldelta, T.x1, static_cast<float>(s->m_dm), s->lx, s->lp,
                             s->g4b, b);
  // g_n from phi_n: the first sweep's input is Q0 after the opening gas kick with it
  dh::launch_grad(st, T.phi0, s->g4b, b);
  s->g4b_phi0_of = all ? sp.step : -1;
  // sweeps in reverse
  for (int k = 2; k >= 0; --k) {
    {
      KernelTimer kt(s, DH_KTIME_SWEEP_VJP);
      if (k > 0)
        dh::launch_sweep_vjp(st, T.q[1 + k], s->lq, s->lq2, b, sp.axes[k]);
      else
        dh::launch_sweep_vjp(st, T.q[0], s->lq, s->lq2, b, sp.axes[0], s->g4b);
    }
    std::swap(s->lq, s->lq2);
  }
  // opening gas kick with g_n
  if (defer_open && all && !closure) {
    s->open_pending = true;
    s->open_q0 = T.q[0];
    s->open_tab = tab_of(s, sp);
  } else {
    opening_kick_vjp(s, T.q[0], b);
  }
}

// Adjoint of the opening dark-matter kick of the first step (x0, phi0 of its tape entry)
void finish_first_kick(dh_sim* s, const TapeStep& T) {
  const Batch b = batch(s, tab_of(s, T.plan));
  hipStream_t st = s->st;
  dh::launch_grad(st, T.phi0, s->g4b, b);
  s->g4b_phi0_of = -1;
  dh::launch_fill(st, s->lg, 0.0f, 3 * s->nc * s->S);
  sort_particles(s, T.x0, b);
  dh::launch_gather_sorted(st, s->bins, s->lp, b);
  dh::launch_deposit_vec(st, s->bins, false, s->lg, b);
  dh::launch_kick_vjp_pos(st, s->g4b, T.x0, s->lp, false, s->lx, b);
  dh::launch_grad_vjp(st, s->lg, s->lphi, s->lphi, b);
}

// Adjoint of the initial conditions: lq, lx, lp, lphi at a_init -> d_grad_white
void ic_vjp(dh_sim* s, float* d_grad_white) {
  const int n = s->n;
  const long long nc = s->nc;
  hipStream_t st = s->st;
  const double ai = s->cfg.a_init;
  const Batch all = batch(s, nullptr);
  std::fill(s->a.begin(), s->a.end(), ai);
  const Batch b0 = batch(s, state_table(s));
  // phi_0 = Poisson(rho_gas + m_dm CIC(x) - 1)
  poisson(s, s->lphi, s->ldelta, b0);
  dh::launch_axpy(st, s->lq, s->ldelta, 1.0f, nc, s->nq * nc, nc, false, all);
  // positions of the initial particles are recomputed from psi (the momenta, written to
  // scratch, are not needed)
  const double vfac = ai * ai * s->cosmo.E(ai) * s->cosmo.growth_rate(ai);
  const bool lpt2 = s->cfg.lpt == 2;
  const float* vel = lpt2 ? s->lptv : s->psi;
  dh::launch_ic_particles(st, s->psi, vel, s->pos, s->fscratch, static_cast<float>(vfac), all);
  dh::launch_deposit_vjp_pos(st, s->ldelta, s->pos, static_cast<float>(s->m_dm), s->lx, nullptr,
                             nullptr, all);
  // gas: rho = f_b CIC(x), m = rho p(q), Et = a^2 rho (e_init + |p/a|^2/2); with first-order
  // displacements the velocity displacement is psi itself and its adjoint goes to lpsi, with
  // second-order ones it has its own adjoint (lvel, in fscratch)
  float* lvel = lpt2 ? s->fscratch : s->lpsi;
  dh::launch_fill(st, s->lpsi, 0.0f, 3 * nc * s->S);
  if (lpt2) dh::launch_fill(st, lvel, 0.0f, 3 * nc * s->S);
  dh::launch_ic_gas_vjp(st, s->cic, vel, s->lq, static_cast<float>(s->f_b),
                        static_cast<float>(vfac), static_cast<float>(ai),
                        static_cast<float>(s->e_init), s->cfg.gamma, s->lcic, lvel, all);
  dh::launch_deposit_vjp_pos(st, s->lcic, s->pos, 1.0f, s->lx, nullptr, nullptr, all);
  // x = q + psi, p = vfac vel
  dh::launch_axpy(st, s->lpsi, s->lx, 1.0f, 3 * nc, 3 * nc, 3 * nc, false, all);
  dh::launch_axpy(st, lvel, s->lp, static_cast<float>(vfac), 3 * nc, 3 * nc, 3 * nc, false, all);
  bool acc = false;   // spec2 accumulates the spectrum of lambda_w
  if (lpt2) {
    // psi = Psi1 + Psi2, vel = Psi1 + r Psi2: lambda_Psi2 = lambda_psi + r lambda_vel (into
    // lx, free now), lambda_Psi1 = lambda_psi + lambda_vel (into lpsi)
    double c2, r;
    lpt2_factors(s, &c2, &r);
    copy_d2d(s, s->lx, s->lpsi, 3 * nc * s->S);
    dh::launch_axpy(st, s->lx, lvel, static_cast<float>(r), 3 * nc, 3 * nc, 3 * nc, false, all);
    dh::launch_axpy(st, s->lpsi, lvel, 1.0f, 3 * nc, 3 * nc, 3 * nc, false, all);
    // Psi2_j = IFFT(i k_j c2 / k^2 FFT(delta2)) -> lambda_delta2 (into ldelta)
    for (int j = 0; j < 3; ++j) {
      dh::fft_forward_xy(st, s->lx + j * nc, s->spec, s->tw, all, 3 * nc);
      dh::fft_zpass_ic(st, s->spec, s->spec2, s->tw, ic_op(s, dh::kOpZaT, j, 0, c2), true, false,
                       j > 0, all);
    }
    dh::fft_zpass_inverse(st, s->spec2, s->tw, all);
    dh::fft_inverse_yx(st, s->spec2, s->ldelta, s->tw, 1.0f, all);
    // delta2 from the second derivatives phi_ab = IFFT(k_a k_b T/k^2 FFT(w)): lambda_w gains
    // IFFT(k_a k_b T/k^2 FFT(lambda_phi_ab)) (a real operator is its own transpose)
    for (int k = 0; k < 6; ++k) {
      dh::launch_lpt2_source_vjp(st, s->hess, s->ldelta, k, s->lcic, all);
      dh::fft_forward_xy(st, s->lcic, s->spec, s->tw, all);
      dh::fft_zpass_ic(st, s->spec, s->spec2, s->tw,
                       ic_op(s, dh::kOpIcHess, kHessAxes[k][0], kHessAxes[k][1]), true, false,
                       acc, all);
      acc = true;
    }
  }
  // psi_j = IFFT(i k_j T(k)/k^2 FFT(w)) -> lambda_w = sum_j IFFT(-i k_j T/k^2 FFT(lambda_psi_j))
  for (int j = 0; j < 3; ++j) {
    dh::fft_forward_xy(st, s->lpsi + j * nc, s->spec, s->tw, all, 3 * nc);
    dh::fft_zpass_ic(st, s->spec, s->spec2, s->tw, ic_op(s, dh::kOpIcDispT, j), true, false,
                     acc || j > 0, all);
  }
  dh::fft_zpass_inverse(st, s->spec2, s->tw, all);
  dh::fft_inverse_yx(st, s->spec2, d_grad_white, s->tw, 1.0f, all);
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool params_ok(const dh_params* p) {
  return p->eps_sf >= 0 && p->delta_c > 0 && p->t_c > 0 && p->w_rho > 0 && p->w_t > 0 &&
         p->e0 >= 0;
}

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
  c->closure = DH_CLOSURE_PLAIN;
  c->batch = 1;
  c->cfl_forward = 1.5 * c->cfl;
  c->kdk = DH_KDK_PLAIN;
  c->star_dm = 0;
  c->sn_smooth = 0;
  c->lpt = 1;
  c->transfer = DH_TRANSFER_BBKS;
  c->dual_energy = 0;
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
  if (!pow2(n) || n < 16 || n > 256 || cfg->batch < 1 || cfg->batch > 4096) return DH_E_INVAL;
  const int S = cfg->batch;
  if (static_cast<long long>(n) * n * n * S > (1LL << 31)) return DH_E_INVAL;
  if (!(cfg->omega_m > 0 && cfg->omega_m < 1 && cfg->omega_b > 0 && cfg->omega_b < cfg->omega_m &&
        cfg->box > 0 && cfg->a_init > 0 && cfg->a_init < 1 && cfg->cfl > 0 && cfg->dlna_max > 0 &&
        cfg->gamma > 1 && cfg->tau > 0 && cfg->ckpt_every >= 1 && cfg->subgrid >= 0 &&
        cfg->cfl_forward >= 0 && (cfg->kdk == DH_KDK_PLAIN || cfg->kdk == DH_KDK_FASTPM) &&
        cfg->subgrid <= 2 && cfg->t_floor > 0 && cfg->t_init > 0 && cfg->sigma8 > 0 &&
        (cfg->star_dm == 0 || cfg->star_dm == 1) && (cfg->sn_smooth == 0 || cfg->sn_smooth == 1) &&
        (cfg->lpt == 1 || cfg->lpt == 2) &&
        (cfg->transfer == DH_TRANSFER_BBKS || cfg->transfer == DH_TRANSFER_EH) &&
        (cfg->dual_energy == 0 ||
         cfg->dual_energy == 1) &&
        (cfg->closure == DH_CLOSURE_PLAIN ||
         (cfg->closure == DH_CLOSURE_MLP && cfg->subgrid != DH_SUBGRID_OFF))))
    return DH_E_INVAL;
  auto s = std::make_unique<dh_sim>();
  int rc = guarded(s.get(), [&]() -> int {
    s->cfg = *cfg;
    dh_params_default(&s->prm);
    s->sprm.assign(S, s->prm);
    s->n = n;
    s->S = S;
    s->nq = cfg->dual_energy ? 6 : 5;
    s->nc = static_cast<long long>(n) * n * n;
    s->np = s->nc;
    s->nck = static_cast<long long>(n) * n * (n / 2 + 1);
    s->cosmo.om = cfg->omega_m;
    s->cosmo.ol = 1.0 - cfg->omega_m;
    if (cfg->kdk == DH_KDK_FASTPM) s->heath.build(s->cosmo, 4.0, 4096);
    s->amp = dh::spectrum_amplitude(cfg->omega_m, cfg->h, cfg->n_s, cfg->sigma8,
                                    cfg->transfer == DH_TRANSFER_EH, cfg->omega_b);
    s->f_b = cfg->omega_b / cfg->omega_m;
    s->m_dm = 1.0 - s->f_b;
    s->vel_unit = 100.0 * cfg->box / n;
    s->t_per_e = (cfg->gamma - 1.0) * cfg->mu * kProtonMass / kBoltzmann *
                 (s->vel_unit * 1e3) * (s->vel_unit * 1e3);
    s->e_init = cfg->t_init / s->t_per_e;
    s->e_floor = cfg->t_floor / s->t_per_e;
    s->t.assign(S, 0.0);
    s->a.assign(S, cfg->a_init);
    s->recorded.assign(S, {});
    s->replay.assign(S, {});
    s->replay_pos.assign(S, 0);
    s->kick_due.assign(S, 0.0f);
    const long long nc = s->nc * S, np = s->np * S;
    s->q = s->alloc<float>(s->nq * nc);
    s->q2 = s->alloc<float>(s->nq * nc);
    s->pos = s->alloc<float>(3 * np);
    s->mom = s->alloc<float>(3 * np);
    s->star = s->alloc<float>(nc);
    if (cfg->star_dm) {
      s->aux = s->alloc<float>(np);
      s->znew = s->alloc<float>(nc);
      DH_HIP(hipMemset(s->aux, 0, static_cast<size_t>(np) * sizeof(float)));
    }
    if (cfg->sn_smooth) s->sn_buf = s->alloc<float>(nc);
    if (cfg->sn_smooth && cfg->dual_energy) s->sn_buf2 = s->alloc<float>(nc);
    if (cfg->lpt == 2) {
      s->hess = s->alloc<float>(6 * nc);
      s->lptv = s->alloc<float>(3 * nc);
    }
    s->phi = s->alloc<float>(nc);
    s->delta = s->alloc<float>(nc);
    s->cic = s->alloc<float>(nc);
    s->psi = s->alloc<float>(3 * nc);
    s->fscratch = s->alloc<float>(3 * np);
    s->spec = s->alloc<float2>(s->nck * S);
    s->spec2 = s->alloc<float2>(s->nck * S);
    s->tw = s->alloc<float2>(n / 2);
    s->bins.key = s->alloc<uint32_t>(np);
    s->bins.rank = s->alloc<uint32_t>(np);
    s->bins.count = s->alloc<uint32_t>(nc);
    s->bins.start = s->alloc<uint32_t>(nc + 1);
    s->bins.sorted = s->alloc<uint32_t>(np);
    s->bins.block_sums = s->alloc<uint32_t>(static_cast<long long>(dh::scan_block_count(nc)) + 1);
    s->bins.large = s->alloc<uint32_t>(1 + dh::large_bin_capacity(np));
    s->bins.spos = s->alloc<float4>(np);
    s->bins.sval = s->alloc<float4>(np);
    s->g4 = s->alloc<float4>(nc);
    s->g4b = s->alloc<float4>(nc);
    s->cfl_red = s->alloc<double>(static_cast<long long>(dh::cfl_blocks(n)) * S + 1);
    s->red_blocks = dh::sum_blocks(s->nc);
    s->red = s->alloc<double>(8LL * s->red_blocks * S + 8);
    s->red_out = s->alloc<double>(8LL * S + 16);
    s->d_acur = s->alloc<double>(S);
    s->cur_tab = s->alloc<StepScal>(S);
    s->stage_tab = s->alloc<StepScal>(1);
    if (cfg->closure == DH_CLOSURE_MLP) {
      s->mlp_theta = s->alloc<float>(dh::mlp::kParams);
      s->mlp_packed = s->alloc<uint4>(static_cast<long long>(dh::mlp::kPackedBytes / sizeof(uint4)));
    }
    void* hp = nullptr;
    DH_HIP(hipHostMalloc(&hp, (8 * S + 16) * sizeof(double), hipHostMallocDefault));
    s->host_out = static_cast<double*>(hp);
    DH_HIP(hipHostMalloc(&hp, S * sizeof(StepScal), hipHostMallocDefault));
    s->hstage = static_cast<StepScal*>(hp);
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
  for (auto& e : s->kt_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->host_out) (void)hipHostFree(s->host_out);
  if (s->hstage) (void)hipHostFree(s->hstage);
  if (s->htabs) (void)hipHostFree(s->htabs);
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
  if (!params_ok(p)) return fail(s, DH_E_INVAL, "non-physical parameters");
  s->prm = *p;
  s->sprm.assign(s->S, *p);
  return DH_OK;
}

int dh_set_sample_params(dh_sim* s, int32_t sample, const dh_params* p) {
  if (!s || !p || sample < 0 || sample >= s->S) return DH_E_INVAL;
  if (!params_ok(p)) return fail(s, DH_E_INVAL, "non-physical parameters");
  s->sprm[sample] = *p;
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
    for (int i = 0; i < s->S; ++i) {
      const uint64_t k = seed + static_cast<uint64_t>(i);
      dh::launch_white_noise(s->st, s->fscratch + s->nc * i,
                             static_cast<uint32_t>(k & 0xFFFFFFFFull),
                             static_cast<uint32_t>(k >> 32), s->n);
    }
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
    StepPlan sp;
    bool moved = false;
    int rc = step_once(s, -1.0, false, &sp, &moved, false);
    if (rc) return rc;
    s->have_forward = false;
    rc = check_replay(s);
    if (rc) return rc;
    if (!all_finite(current_speed(s)))   // also validates the new state
      return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
    if (dt_out) *dt_out = moved ? sp.smp[0].dt : 0.0;
    if (a_out) *a_out = s->a[0];
    return DH_OK;
  });
}

int dh_run_to(dh_sim* s, double a_final, int32_t* nsteps_out) {
  if (!s || !(a_final > 0)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const double t_end = s->cosmo.t_of_a(a_final);
    int count = 0;
    int rc = DH_OK;
    for (;;) {
      bool moved = false;
      rc = step_once(s, t_end, false, nullptr, &moved, true);
      if (rc || !moved) break;
      ++count;
    }
    flush_kick(s);
    s->have_forward = false;
    if (nsteps_out) *nsteps_out = count;
    if (rc) return rc;
    return check_replay(s);
  });
}

int dh_run_steps(dh_sim* s, int32_t nsteps, int32_t* nsteps_out) {
  if (!s || nsteps < 0) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    int count = 0;
    int rc = DH_OK;
    while (count < nsteps) {
      bool moved = false;
      rc = step_once(s, -1.0, false, nullptr, &moved, true);
      if (rc || !moved) break;
      ++count;
    }
    flush_kick(s);
    s->have_forward = false;
    if (nsteps_out) *nsteps_out = count;
    if (rc) return rc;
    rc = check_replay(s);
    if (rc) return rc;
    if (!all_finite(current_speed(s)))   // also validates the new state
      return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
    return DH_OK;
  });
}

int dh_set_schedule(dh_sim* s, const double* dts, int32_t n) {
  if (!s || n < 0 || (n > 0 && !dts)) return DH_E_INVAL;
  for (int i = 0; i < s->S; ++i) {
    s->replay[i].assign(dts, dts + n);
    s->replay_pos[i] = 0;
  }
  return DH_OK;
}

int dh_set_sample_schedule(dh_sim* s, int32_t sample, const double* dts, int32_t n) {
  if (!s || sample < 0 || sample >= s->S || n < 0 || (n > 0 && !dts)) return DH_E_INVAL;
  s->replay[sample].assign(dts, dts + n);
  s->replay_pos[sample] = 0;
  return DH_OK;
}

int dh_get_sample_schedule(const dh_sim* s, int32_t sample, double* dts, int32_t cap,
                           int32_t* n_out) {
  if (!s || sample < 0 || sample >= s->S || cap < 0 || (cap > 0 && !dts)) return DH_E_INVAL;
  const std::vector<double>& r = s->recorded[sample];
  const int32_t n = static_cast<int32_t>(r.size());
  for (int32_t i = 0; i < std::min(n, cap); ++i) dts[i] = r[i];
  if (n_out) *n_out = n;
  return DH_OK;
}

int dh_get_schedule(const dh_sim* s, double* dts, int32_t cap, int32_t* n_out) {
  return dh_get_sample_schedule(s, 0, dts, cap, n_out);
}

int dh_get_field(dh_sim* s, dh_field f, float* d_out) {
  if (!s || !d_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const long long nc = s->nc, S = s->S;
    switch (f) {
      case DH_FIELD_Q: copy_d2d(s, d_out, s->q, s->nq * nc * S); break;
      case DH_FIELD_RHO:
        for (int i = 0; i < S; ++i) copy_d2d(s, d_out + nc * i, s->q + s->nq * nc * i, nc);
        break;
      case DH_FIELD_POS: copy_d2d(s, d_out, s->pos, 3 * s->np * S); break;
      case DH_FIELD_MOM: copy_d2d(s, d_out, s->mom, 3 * s->np * S); break;
      case DH_FIELD_STAR: copy_d2d(s, d_out, s->star, nc * S); break;
      case DH_FIELD_STAR_DM:
        if (!s->aux) return fail(s, DH_E_INVAL, "the star read-out needs cfg.star_dm");
        copy_d2d(s, d_out, s->aux, s->np * S);
        break;
      case DH_FIELD_OBS_TEMP:
        for (int i = 0; i < S; ++i)
          dh::launch_fli_obs(s->st, s->q + s->nq * nc * i, s->a[i], 1.0 / s->f_b, s->e_floor,
                             s->t_per_e, d_out + nc * i, nc, s->nq, s->cfg.gamma);
        break;
      case DH_FIELD_PHI:
        if (!s->phi_valid) refresh_potential(s);
        copy_d2d(s, d_out, s->phi, nc * S);
        break;
      case DH_FIELD_TEMP:
        for (int i = 0; i < S; ++i)
          dh::launch_temperature(s->st, s->q + s->nq * nc * i, static_cast<float>(s->a[i]),
                                 static_cast<float>(s->e_floor), static_cast<float>(s->t_per_e),
                                 d_out + nc * i, nc, s->nq, s->cfg.gamma);
        break;
      case DH_FIELD_FLUX:
        for (int i = 0; i < S; ++i)
          dh::launch_flux_field(s->st, s->q + s->nq * nc * i, s->prm.A, s->prm.beta,
                                static_cast<float>(1.0 / s->f_b), d_out + nc * i, nc);
        break;
      default: return fail(s, DH_E_INVAL, "unknown field");
    }
    return DH_OK;
  });
}

int dh_set_field(dh_sim* s, dh_field f, const float* d_in) {
  if (!s || !d_in) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const long long nc = s->nc, S = s->S;
    switch (f) {
      case DH_FIELD_Q: copy_d2d(s, s->q, d_in, s->nq * nc * S); s->phi_valid = false; break;
      case DH_FIELD_RHO:
        for (int i = 0; i < S; ++i) copy_d2d(s, s->q + s->nq * nc * i, d_in + nc * i, nc);
        s->phi_valid = false;
        break;
      case DH_FIELD_POS: copy_d2d(s, s->pos, d_in, 3 * s->np * S); s->phi_valid = false; break;
      case DH_FIELD_MOM: copy_d2d(s, s->mom, d_in, 3 * s->np * S); break;
      case DH_FIELD_STAR: copy_d2d(s, s->star, d_in, nc * S); break;
      case DH_FIELD_STAR_DM:
        if (!s->aux) return fail(s, DH_E_INVAL, "the star read-out needs cfg.star_dm");
        copy_d2d(s, s->aux, d_in, s->np * S);
        break;
      case DH_FIELD_PHI:
        copy_d2d(s, s->phi, d_in, nc * S);
        dh::launch_grad(s->st, s->phi, s->g4, batch(s, nullptr));
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
  if (a) *a = s->a[0];
  if (t) *t = s->t[0];
  if (step) *step = s->step;
  return DH_OK;
}

int dh_get_sample_times(const dh_sim* s, double* a, double* t) {
  if (!s) return DH_E_INVAL;
  for (int i = 0; i < s->S; ++i) {
    if (a) a[i] = s->a[i];
    if (t) t[i] = s->t[i];
  }
  return DH_OK;
}

int dh_set_time(dh_sim* s, double a, int32_t step) {
  if (!s || !(a > 0) || step < 0) return DH_E_INVAL;
  std::fill(s->a.begin(), s->a.end(), a);
  std::fill(s->t.begin(), s->t.end(), s->cosmo.t_of_a(a));
  s->step = step;
  s->phi_valid = false;
  state_changed(s);
  return DH_OK;
}

int dh_set_store_limit(dh_sim* s, int32_t max_steps) {
  if (!s) return DH_E_INVAL;
  s->store_max = max_steps < 0 ? -1 : max_steps;
  return DH_OK;
}

int dh_get_store_info(const dh_sim* s, int32_t* taped, int32_t* sorted) {
  if (!s) return DH_E_INVAL;
  if (taped) *taped = s->taped;
  if (sorted) *sorted = s->store_valid;
  return DH_OK;
}

int dh_forward(dh_sim* s, const float* d_white, double a_final, int32_t* nsteps_out) {
  if (!s || !d_white || !(a_final > s->cfg.a_init)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    s->have_forward = false;
    initial_conditions(s, d_white);
    const double t_end = s->cosmo.t_of_a(a_final);
    const int K = s->cfg.ckpt_every;
    int count = 0;
    s->fwd_plans.clear();
    plan_storage(s);
    for (;;) {
      StepPlan sp;
      bool any = false;
      int rc = prepare_step(s, t_end, true, sp, &any);
      if (rc) {
        flush_kick(s);
        return rc;
      }
      if (!any) break;
      if (count < s->tape_limit && count % K == 0) {
        // a segment's tape entries at its start; if the memory is not there after all, this
        // segment and the following ones take checkpoints instead
        const int need = std::min(count + K, s->tape_limit);
        while (static_cast<int>(s->ftape.size()) < need) {
          s->ftape.push_back(TapeStep{});
          if (!try_alloc_tape_entry(s, s->ftape.back())) {
            s->ftape.pop_back();
            s->tape_limit = count;
            break;
          }
        }
      }
      if (count < s->tape_limit) {
        // recorded into the forward's own tape (no checkpoint needed for these segments)
        take_step(s, sp, true, -1, &s->ftape[count]);
        s->taped = count + 1;
      } else {
        // a checkpoint at the start of every K-th step (none after the last step)
        if (count % K == 0) {
          const size_t g = static_cast<size_t>(count / K);
          if (s->ckpts.size() <= g) s->ckpts.resize(g + 1);
          save_ckpt(s, s->ckpts[g]);
        }
        take_step(s, sp, true, count - s->tape_limit);
      }
      s->fwd_plans.push_back(sp);
      ++count;
    }
    flush_kick(s);
    if (nsteps_out) *nsteps_out = count;
    int rc = check_replay(s);
    if (rc) return rc;
    if (!all_finite(current_speed(s)))
      return fail(s, DH_E_NONFINITE, "state has a non-finite value or a non-positive density");
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
                            static_cast<float>(1.0 / s->f_b), s->red, batch(s, nullptr));
    dh::launch_reduce_sum(s->st, s->red, nb, nb, s->S, s->red_out);
    DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, s->S * sizeof(double), hipMemcpyDeviceToHost,
                          s->st));
    sync(s);
    for (int i = 0; i < s->S; ++i) loss_out[i] = s->host_out[i] / static_cast<double>(s->nc);
    if (!s->loss_target) s->loss_target = s->alloc<float>(s->nc * s->S);
    copy_d2d(s, s->loss_target, d_target, s->nc * s->S);
    s->have_loss = s->have_forward;
    s->loss_kind = dh_sim::kLossFlux;
    return DH_OK;
  });
}

int dh_backward(dh_sim* s, const float* d_grad_rho, float* d_grad_white, double* grad_params) {
  if (!s || !d_grad_white || !grad_params) return DH_E_INVAL;
  if (!s->have_forward) return fail(s, DH_E_STATE, "dh_backward needs a preceding dh_forward");
  if (!d_grad_rho && !s->have_loss) return fail(s, DH_E_STATE, "dh_backward without d_grad_rho needs dh_loss");
  return guarded(s, [&]() -> int {
    const int S = s->S;
    const long long nc = s->nc, np = s->np;
    const int nsteps = s->fwd_steps;
    s->g4b_phi0_of = -1;
    s->open_pending = false;
    const int K = s->cfg.ckpt_every;
    if (!s->lq) {
      s->lq = s->alloc<float>(s->nq * nc * S);
      s->lq2 = s->alloc<float>(s->nq * nc * S);
      s->lx = s->alloc<float>(3 * np * S);
      s->lp = s->alloc<float>(3 * np * S);
      s->lphi = s->alloc<float>(nc * S);
      s->lphi2 = s->alloc<float>(nc * S);
      s->lg = s->alloc<float>(3 * nc * S);
      s->lg2 = s->alloc<float>(3 * nc * S);
      s->ldelta = s->alloc<float>(nc * S);
      s->lpsi = s->alloc<float>(3 * nc * S);
      s->lcic = s->alloc<float>(nc * S);
    }
    if (s->param_cap < nsteps + 2) {
      if (s->param_steps) s->release(s->param_steps);
      s->param_steps = nullptr;
      s->param_cap = nsteps + 2;
      s->param_steps = s->alloc<double>(2LL * S * s->param_cap);
    }
    // dark-matter kick factors of the reverse pass: the step's closing kick plus the same
    // sample's next opening kick (0 after its last step)
    for (int k = 0; k < nsteps; ++k) {
      const StepPlan& sp = s->fwd_plans[k];
      StepScal* h = s->htabs + static_cast<size_t>(sp.slot) * S;
      for (int i = 0; i < S; ++i) {
        if (!sp.smp[i].active) continue;
        const bool next = k + 1 < nsteps && s->fwd_plans[k + 1].smp[i].active;
        const float hn =
            next ? s->htabs[static_cast<size_t>(s->fwd_plans[k + 1].slot) * S + i].h_open : 0.0f;
        h[i].h_dm = h[i].h_close + hn;
      }
    }
    if (nsteps > 0)
      DH_HIP(hipMemcpyAsync(s->tabs, s->htabs,
                            static_cast<size_t>(s->fwd_plans.back().slot + 1) * S * sizeof(StepScal),
                            hipMemcpyHostToDevice, s->st));
    // final state adjoint
    dh::launch_fill(s->st, s->lq, 0.0f, s->nq * nc * S);
    dh::launch_fill(s->st, s->lx, 0.0f, 3 * np * S);
    dh::launch_fill(s->st, s->lp, 0.0f, 3 * np * S);
    dh::launch_fill(s->st, s->lphi, 0.0f, nc * S);
    std::vector<double> gA(S, 0.0), gB(S, 0.0);
    if (d_grad_rho) {
      for (int i = 0; i < S; ++i) copy_d2d(s, s->lq + s->nq * nc * i, d_grad_rho + nc * i, nc);
    } else if (s->loss_kind == dh_sim::kLossPower) {
      power_loss_vjp(s);
    } else if (s->loss_kind == dh_sim::kLossFli) {
      upload_scale_factors(s);
      dh::launch_fli(s->st, s->q, s->fli_data, s->fli_nvar, s->fli_white, s->d_acur,
                     1.0 / s->f_b, s->e_floor, s->t_per_e, s->cfg.gamma, nullptr, s->lq,
                     batch(s, nullptr));
    } else {
      const int nb = s->red_blocks;
      dh::launch_loss_vjp(s->st, s->q, s->loss_target, s->prm.A, s->prm.beta,
                          static_cast<float>(1.0 / s->f_b), s->lq, s->red, batch(s, nullptr));
      dh::launch_reduce_sum(s->st, s->red, nb, nb, 2 * S, s->red_out);
      DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, 2 * S * sizeof(double),
                            hipMemcpyDeviceToHost, s->st));
      sync(s);
      for (int i = 0; i < S; ++i) {
        gA[i] = s->host_out[i];
        gB[i] = s->host_out[S + i];
      }
    }
    // segments in reverse
    const int nseg = (nsteps + K - 1) / K;
    // the recomputation's tape, if some segment is not on the forward's own tape
    const size_t want = s->taped < nsteps ? static_cast<size_t>(std::min(K, nsteps)) : 0;
    while (s->tape.size() < want) {
      s->tape.push_back(TapeStep{});
      alloc_tape_entry(s, s->tape.back());
    }
    // set the forward's final state aside to restore it afterwards
    stash_state(s);
    dh::launch_fill(s->st, reinterpret_cast<float*>(s->param_steps), 0.0f,
                    4LL * S * s->param_cap);
    for (int g = nseg - 1; g >= 0; --g) {
      const int s0 = g * K, s1 = std::min(nsteps, s0 + K);
      if (s1 <= s->taped) {
        // recorded by the forward: x1 and phi1 of a step are the next step's x0 and phi0,
        // or, after the recorded steps, those of the next checkpoint or the final state
        for (int k = s1 - 1; k >= s0; --k) {
          TapeStep& T = s->ftape[k];
          if (k + 1 < s->taped) {
            T.x1 = s->ftape[k + 1].x0;
            T.phi1 = s->ftape[k + 1].phi0;
          } else if (k + 1 == nsteps) {
            T.x1 = s->keep.pos;
            T.phi1 = s->keep.phi;
          } else {
            T.x1 = s->ckpts[(k + 1) / K].pos;
            T.phi1 = s->ckpts[(k + 1) / K].phi;
          }
          step_vjp(s, T, k > s0);
        }
        continue;
      }
      load_ckpt(s, s->ckpts[g]);
      // the recomputed trajectory is the forward's bit for bit (the forward also deferred
      // its kicks and applied them before each checkpoint); the momenta after the last
      // step of the segment are not needed, so its pending kick is dropped
      for (int k = s0; k < s1; ++k)
        do_step(s, s->fwd_plans[k], &s->tape[k - s0], true,
                k >= s->tape_limit ? k - s->tape_limit : -1, true);
      drop_kick(s);
      for (int k = s1 - 1; k >= s0; --k) {
        TapeStep& T = s->tape[k - s0];
        T.x1 = k + 1 < s1 ? s->tape[k + 1 - s0].x0 : s->pos;
        T.phi1 = k + 1 < s1 ? s->tape[k + 1 - s0].phi0 : s->phi;
        step_vjp(s, T, k > s0);
      }
    }
    if (nsteps > 0) finish_first_kick(s, s->taped > 0 ? s->ftape[0] : s->tape[0]);
    ic_vjp(s, d_grad_white);
    // the field-level posterior's prior 1/2 |w|^2 adds w
    if (!d_grad_rho && s->loss_kind == dh_sim::kLossFli)
      dh::launch_axpy(s->st, d_grad_white, s->fli_white, 1.0f, nc, nc, nc, false,
                      batch(s, nullptr));
    // restore the final state of the forward run
    unstash_state(s);
    // parameter gradients: fixed-order host sum of the per-step FP64 partials
    std::vector<double> ps(2 * static_cast<size_t>(S) * (nsteps > 0 ? nsteps : 1));
    if (nsteps > 0)
      DH_HIP(hipMemcpyAsync(ps.data(), s->param_steps, 2 * static_cast<size_t>(S) * nsteps *
                                                           sizeof(double),
                            hipMemcpyDeviceToHost, s->st));
    sync(s);
    for (int i = 0; i < S; ++i) {
      double ge = 0.0, gd = 0.0;
      for (int k = 0; k < nsteps; ++k) {
        const size_t slot = static_cast<size_t>(s->fwd_plans[k].slot);
        ge += ps[2 * S * slot + i];
        gd += ps[2 * S * slot + S + i];
      }
      grad_params[4 * i + 0] = gA[i];
      grad_params[4 * i + 1] = gB[i];
      grad_params[4 * i + 2] = ge;
      grad_params[4 * i + 3] = gd;
    }
    return DH_OK;
  });
}

int dh_power_spectrum(dh_sim* s, int32_t nbins, double* pk_out, double* k_out,
                      double* nmodes_out) {
  if (!s || !pk_out || nbins < 1 || nbins > s->n / 2) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    std::vector<double> pk;
    power_spectrum(s, nbins, pk);
    std::memcpy(pk_out, pk.data(), pk.size() * sizeof(double));
    const std::vector<double>& w = pk_counts(s, nbins);
    for (int k = 0; k < nbins; ++k) {
      if (k_out) k_out[k] = 2.0 * M_PI * (k + 1) / s->cfg.box;
      if (nmodes_out) nmodes_out[k] = w[k];
    }
    return DH_OK;
  });
}

int dh_power_loss(dh_sim* s, int32_t nbins, const double* pk_obs, const double* cinv,
                  double* loss_out) {
  if (!s || !pk_obs || !cinv || !loss_out || nbins < 1 || nbins > s->n / 2) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int S = s->S;
    std::vector<double> pk;
    power_spectrum(s, nbins, pk);
    const std::vector<double>& w = pk_counts(s, nbins);
    const double n3 = static_cast<double>(s->nc);
    const double c = s->cfg.box * s->cfg.box * s->cfg.box / (n3 * n3) / (s->f_b * s->f_b);
    s->pk_g.assign(static_cast<size_t>(S) * nbins, 0.0f);
    for (int i = 0; i < S; ++i) {
      const double* p = pk.data() + static_cast<size_t>(i) * nbins;
      const double* o = pk_obs + static_cast<size_t>(i) * nbins;
      double L = 0.0;
      for (int a = 0; a < nbins; ++a) {
        double g = 0.0;   // (C^-1 (P - P_obs))_a
        for (int k = 0; k < nbins; ++k) g += cinv[static_cast<size_t>(a) * nbins + k] * (p[k] - o[k]);
        L += 0.5 * (p[a] - o[a]) * g;
        s->pk_g[static_cast<size_t>(i) * nbins + a] = static_cast<float>(g * c / w[a]);
      }
      loss_out[i] = L;
    }
    s->pk_loss_bins = nbins;
    s->have_loss = s->have_forward;
    s->loss_kind = dh_sim::kLossPower;
    return DH_OK;
  });
}

int dh_closure_states(dh_sim* s, float* d_x, float* d_y) {
  if (!s || !d_x || !d_y) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const long long ld = s->nc * s->S;
    for (int i = 0; i < s->S; ++i)
      dh::launch_closure_state(s->st, s->q + s->nq * s->nc * i, source_args(s, i, s->a[i], 0.0, 0),
                               d_x + s->nc * i, d_y + s->nc * i, s->nc, ld, s->nq);
    return DH_OK;
  });
}

int dh_fli_loss(dh_sim* s, const float* d_data, const float* d_noise_var, const float* d_white,
                double* loss_out) {
  if (!s || !d_data || !d_noise_var || !d_white || !loss_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int S = s->S;
    const long long nc = s->nc;
    if (!s->fli_data) {
      s->fli_data = s->alloc<float>(nc * S);
      s->fli_nvar = s->alloc<float>(nc * S);
      s->fli_white = s->alloc<float>(nc * S);
      s->fli_part = s->alloc<double>(static_cast<long long>(dh::fli_blocks(nc)) * S);
    }
    copy_d2d(s, s->fli_data, d_data, nc * S);
    copy_d2d(s, s->fli_nvar, d_noise_var, nc * S);
    copy_d2d(s, s->fli_white, d_white, nc * S);
    upload_scale_factors(s);
    const int nb = dh::fli_blocks(nc);
    dh::launch_fli(s->st, s->q, s->fli_data, s->fli_nvar, s->fli_white, s->d_acur, 1.0 / s->f_b,
                   s->e_floor, s->t_per_e, s->cfg.gamma, s->fli_part, nullptr, batch(s, nullptr));
    dh::launch_reduce_sum(s->st, s->fli_part, nb, nb, S, s->red_out);
    DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, S * sizeof(double), hipMemcpyDeviceToHost,
                          s->st));
    sync(s);
    for (int i = 0; i < S; ++i) loss_out[i] = s->host_out[i];
    s->have_loss = s->have_forward;
    s->loss_kind = dh_sim::kLossFli;
    return DH_OK;
  });
}

int dh_set_kernel_timing(dh_sim* s, int32_t family) {
  if (!s || family < -1 || family > DH_KTIME_SWEEP_VJP) return DH_E_INVAL;
  s->ktime_family = family;
  s->kt_used = 0;
  return DH_OK;
}

int dh_get_kernel_timing(dh_sim* s, int32_t* count, double* mean_ms) {
  if (!s || !count || !mean_ms) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    sync(s);
    double total = 0.0;
    for (size_t i = 0; i < s->kt_used; ++i) {
      float ms = 0.0f;
      DH_HIP(hipEventElapsedTime(&ms, s->kt_events[i].first, s->kt_events[i].second));
      total += ms;
    }
    *count = static_cast<int32_t>(s->kt_used);
    *mean_ms = s->kt_used ? total / static_cast<double>(s->kt_used) : 0.0;
    s->kt_used = 0;
    return DH_OK;
  });
}

int dh_conservation(dh_sim* s, double* out) {
  if (!s || !out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int nb = s->red_blocks;
    for (int i = 0; i < s->S; ++i) {
      dh::launch_conservation_partial(s->st, s->q + s->nq * s->nc * i, s->mom + 3 * s->np * i, s->red,
                                      nb, s->nc);
      dh::launch_reduce_sum(s->st, s->red, nb, nb, 8, s->red_out);
      DH_HIP(hipMemcpyAsync(s->host_out, s->red_out, 8 * sizeof(double), hipMemcpyDeviceToHost,
                            s->st));
      sync(s);
      for (int k = 0; k < 8; ++k) out[8 * i + k] = s->host_out[k];
      for (int k = 5; k < 8; ++k) out[8 * i + k] *= s->m_dm;
    }
    return DH_OK;
  });
}

int dh_stage_sweep(dh_sim* s, const float* d_q_in, float* d_q_out, int32_t axis, double dt,
                   double a1, double a2) {
  if (!s || !d_q_in || !d_q_out || axis < 0 || axis > 2 || d_q_in == d_q_out) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    StepScal e{};
    e.active = 1;
    e.dt = static_cast<float>(dt);
    e.h1 = hydro_at(s, a1);
    e.h2 = hydro_at(s, a2);
    dh::launch_sweep(s->st, d_q_in, d_q_out, Batch{s->n, 1, stage_table(s, e), s->nq}, axis);
    return DH_OK;
  });
}

int dh_stage_sweep_vjp(dh_sim* s, const float* d_q_in, const float* d_lam_out, float* d_lam_in,
                       int32_t axis, double dt, double a1, double a2) {
  if (!s || !d_q_in || !d_lam_out || !d_lam_in || axis < 0 || axis > 2) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    StepScal e{};
    e.active = 1;
    e.dt = static_cast<float>(dt);
    e.h1 = hydro_at(s, a1);
    e.h2 = hydro_at(s, a2);
    dh::launch_sweep_vjp(s->st, d_q_in, d_lam_out, d_lam_in, Batch{s->n, 1, stage_table(s, e), s->nq},
                         axis);
    return DH_OK;
  });
}

int dh_stage_poisson(dh_sim* s, const float* d_delta, float* d_phi, double a) {
  if (!s || !d_delta || !d_phi || !(a > 0)) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    StepScal e{};
    e.active = 1;
    e.green = green_at(s, a);
    poisson(s, d_delta, d_phi, Batch{s->n, 1, stage_table(s, e), s->nq});
    return DH_OK;
  });
}

int dh_stage_deposit(dh_sim* s, const float* d_rho_gas, const float* d_pos, float* d_delta) {
  if (!s || !d_rho_gas || !d_pos || !d_delta) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const Batch one{s->n, 1, nullptr, s->nq};
    sort_particles(s, d_pos, one);
    dh::launch_deposit(s->st, s->bins, d_rho_gas, s->nc, static_cast<float>(s->m_dm), -1.0f,
                       d_delta, one);
    return DH_OK;
  });
}

int dh_stage_readout(dh_sim* s, const float* d_phi, const float* d_pos, float* d_g) {
  if (!s || !d_phi || !d_pos || !d_g) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const Batch one{s->n, 1, nullptr, s->nq};
    dh::launch_grad(s->st, d_phi, s->g4b, one);
    s->g4b_phi0_of = -1;
    dh::launch_readout_g(s->st, s->g4b, d_pos, d_g, one);
    return DH_OK;
  });
}

// handle-free calls (dh_conservation_noalloc) keep their last message per thread
const char* dh_last_error(const dh_sim* s) {
  return s ? s->err.c_str() : dh_noalloc_last_error_message();
}
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

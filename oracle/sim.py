"""Configuration, state and the full time step of the oracle.

One step from t_n to t_n + dt (operator order; the order of the kicks, drift, sweeps and
source is a reading of Sec. 2.2-2.4, which state the operators but not one sequence):
  1. dt from the CFL condition (eq. dt) and a cap on dln a, or the next entry of a given
     schedule (a predefined schedule is what the paper differentiates through, Sec. 2.3.3);
  2. opening half kicks with g_n = -grad(phi_n): gas (source S_g) and dark matter;
  3. dark-matter drift with a(t_n + dt/2) (the dark matter's kick and drift factors are
     those of the leapfrog in t, or FastPM's growth-factor factors: dm_factors);
  4. three relaxing-TVD sweeps in the Strang order of this step;
  5. CIC deposit of gas + dark matter and the FFT Poisson solve at a(t_n+dt) -> phi_{n+1};
  6. closing half kicks with g_{n+1}: gas and dark matter;
  7. the star-formation source term with a(t_n+dt), or the learned closure standing in for
     its probability (oracle.mlp) when the configuration carries network weights; optionally
     with the supernova energy spread over neighbouring cells (subgrid.smooth_injection);
  8. optionally, the stars formed in the step read out by CIC at the particles' positions
     and added to the particles' auxiliary field (Sec. 2.4.1: the new stars are associated
     with nearby dark-matter particles, a diagnostic that does not act on the evolution);
  9. with the dual-energy formalism, the entropy reset from the total energy where the
     internal energy is a large enough part of it (hydro.dual_sync).
The state carries phi so that each step solves Poisson once; phi of the initial state is
solved from the initial particles and gas.
"""

import math
from dataclasses import dataclass, replace

import numpy as np
import torch

from . import cosmology, gravity, hydro, ics, mlp, philox, subgrid


@dataclass
class Config:
    n: int = 32
    box: float = 10.0            # comoving side [Mpc/h]
    omega_m: float = 0.3
    omega_b: float = 0.05
    h: float = 0.7
    sigma8: float = 0.8
    n_s: float = 0.96
    gamma: float = 5.0 / 3.0
    mu: float = 0.6
    a_init: float = 0.01
    t_init: float = 100.0        # K
    cfl: float = 0.4
    dlna_max: float = 0.04
    t_floor: float = 1.0         # K, only inside the equation of state
    subgrid: int = subgrid.MODE_OFF
    tau: float = 0.1
    sf_seed: int = 102
    closure_theta: object = None  # flat network parameters (oracle.mlp), None: plain source
    closure_bf16: bool = True     # round the network's product operands to bfloat16
    kdk: int = 0                  # dark-matter step factors: KDK_PLAIN or KDK_FASTPM
    lpt: int = 1                  # order of the initial displacements (1 Zel'dovich, 2 2LPT)
    transfer: int = 0             # cosmology.TRANSFER_BBKS or TRANSFER_EH
    sn_smooth: bool = False       # supernova energy spread over the neighbouring cells
    star_dm: bool = False         # keep the stars' read-out on the particles (State.aux)
    dual_energy: bool = False     # carry the entropy variable S as a sixth gas component

    # derived quantities (filled by finish())
    amp: float = 0.0
    f_b: float = 0.0
    vel_unit: float = 0.0        # km/s per code velocity unit (cells * H0)
    t_per_e: float = 0.0
    e_init: float = 0.0
    e_floor: float = 0.0

    def finish(self):
        c = replace(self)
        c.amp = cosmology.spectrum_amplitude(c.omega_m, c.h, c.n_s, c.sigma8, c.transfer,
                                             c.omega_b)
        c.f_b = c.omega_b / c.omega_m
        c.vel_unit = 100.0 * c.box / c.n
        c.t_per_e = subgrid.kelvin_per_code_energy(c.gamma, c.mu, c.vel_unit)
        c.e_init = c.t_init / c.t_per_e
        c.e_floor = c.t_floor / c.t_per_e
        return c


KDK_PLAIN, KDK_FASTPM = 0, 1


def dm_factors(cfg, a0, a_half, a1, dt):
    """(opening kick, drift, closing kick) factors of the dark matter over one step: the plain
    leapfrog in t (dt/2, dt / a_half^2, dt/2), or the growth-factor factors of FastPM
    (cosmology.fastpm_factors).  The gas kicks are dt/2 in both."""
    if cfg.kdk == KDK_FASTPM:
        return cosmology.fastpm_factors(a0, a_half, a1, cfg.omega_m)
    return 0.5 * dt, dt / (a_half * a_half), 0.5 * dt


@dataclass
class Params:
    A: float = 0.3               # flux observable F = exp(-A Delta^beta)
    beta: float = 1.6
    eps_sf: float = 0.02         # star-formation efficiency per free-fall time
    delta_c: float = 100.0       # gas overdensity threshold
    t_c: float = 10 ** 4.5       # K, temperature threshold
    e0: float = 0.03             # SN specific energy [(1000 km/s)^2]
    w_rho: float = 0.1           # sigmoid widths, relative to the thresholds
    w_t: float = 0.1


@dataclass
class State:
    q: torch.Tensor      # [5, n, n, n], or [6, n, n, n] with the entropy (dual energy)
    x: torch.Tensor      # [3, n^3]
    p: torch.Tensor      # [3, n^3]
    star: torch.Tensor   # [n, n, n]
    phi: torch.Tensor    # [n, n, n]
    t: float
    a: float
    step: int
    aux: object = None   # [n^3] stars read out on the particles (Config.star_dm), else None


def potential(q, x, a, cfg):
    delta = gravity.total_overdensity(q[0], x, 1.0 - cfg.f_b, cfg.n)
    return gravity.poisson(delta, a, cfg.omega_m)


def initial_state(white, cfg):
    """State at a_init from white noise [n, n, n] (float64 tensor, may require grad)."""
    return state_from_qxp(*ics.initial_state(white, cfg), cfg)


def state_from_qxp(q, x, p, cfg):
    """State at a_init from gas, particle positions and momenta; phi is solved here."""
    a = cfg.a_init
    return State(q=q, x=x, p=p, star=torch.zeros_like(q[0]), phi=potential(q, x, a, cfg),
                 t=cosmology.time_of_a(a, cfg.omega_m), a=a, step=0)


def cfl_dt(state, cfg, t_end=None):
    """dt = min(C a / max(|U_d|+c_s), dlna_max / E(a)), clipped to land on t_end (eq. dt)."""
    with torch.no_grad():
        vmax = hydro.max_signal_speed(state.q, state.a, cfg.gamma, cfg.e_floor)
    dt = min(cfg.cfl / vmax, cfg.dlna_max / cosmology.hubble_e(state.a, cfg.omega_m))
    if t_end is not None and state.t + dt > t_end:
        dt = t_end - state.t
    return dt


def step(state, cfg, prm, dt):
    """Advance one step of length dt (see module docstring).  Returns the new State."""
    n = cfg.n
    om = cfg.omega_m
    a0 = state.a
    a_half = cosmology.a_of_time(state.t + 0.5 * dt, om)
    a1 = cosmology.a_of_time(state.t + dt, om)
    h = 0.5 * dt

    k_open, drift, k_close = dm_factors(cfg, a0, a_half, a1, dt)

    g = gravity.grad_central(state.phi)
    q = gravity.gas_kick(state.q, g, h)
    p = gravity.dm_kick(state.p, state.x, g, k_open)
    x = gravity.dm_drift_by(state.x, p, drift, n)

    for d in hydro.strang_axes(state.step):
        q = hydro.sweep(q, d, dt, a0, a_half, cfg.gamma, cfg.e_floor)

    phi = potential(q, x, a1, cfg)
    g = gravity.grad_central(phi)
    q = gravity.gas_kick(q, g, h)
    p = gravity.dm_kick(p, x, g, k_close)

    star = state.star
    aux = state.aux
    if cfg.star_dm and aux is None:
        aux = torch.zeros(n ** 3, dtype=x.dtype)
    if cfg.subgrid != subgrid.MODE_OFF:
        u = torch.from_numpy(philox.starform_uniform(cfg.sf_seed, state.step, n))
        if cfg.closure_theta is not None:
            theta = torch.as_tensor(cfg.closure_theta, dtype=torch.float64)
            q, star, z = mlp.apply_closure(
                q, star, a1, dt, u, theta, rho_mean_gas=cfg.f_b, gamma=cfg.gamma,
                e_floor=cfg.e_floor, t_per_e=cfg.t_per_e,
                e0_code=prm.e0 * 1e6 / cfg.vel_unit ** 2, eps_sf=prm.eps_sf,
                delta_c=prm.delta_c, tau=cfg.tau, mode=cfg.subgrid, bf16=cfg.closure_bf16,
                with_draw=True, smooth=cfg.sn_smooth)
        else:
            q, star, z = subgrid.apply_source(
                q, star, a1, dt, u, rho_mean_gas=cfg.f_b, omega_b=cfg.omega_b,
                gamma=cfg.gamma, e_floor=cfg.e_floor, t_per_e=cfg.t_per_e,
                e0_code=prm.e0 * 1e6 / cfg.vel_unit ** 2, eps_sf=prm.eps_sf,
                delta_c=prm.delta_c, t_c=prm.t_c, w_rho=prm.w_rho, w_t=prm.w_t, tau=cfg.tau,
                mode=cfg.subgrid, smooth=cfg.sn_smooth, with_draw=True)
        if cfg.star_dm:
            # the step's new stars, read out at the particles' end-of-step positions
            aux = aux + gravity.cic_readout(z, x)
    if cfg.dual_energy:
        q = hydro.dual_sync(q, a1, cfg.gamma)
    return State(q=q, x=x, p=p, star=star, phi=phi, t=state.t + dt, a=a1, step=state.step + 1,
                 aux=aux)


def run(state, cfg, prm, *, a_final=None, nsteps=None, schedule=None):
    """Step until a >= a_final (CFL steps, last one clipped) or for a given schedule / count.
    Returns (state, list of dt)."""
    dts = []
    t_end = cosmology.time_of_a(a_final, cfg.omega_m) if a_final is not None else None
    i = 0
    while True:
        if schedule is not None:
            if i >= len(schedule):
                break
            dt = float(schedule[i])
        else:
            if nsteps is not None and i >= nsteps:
                break
            if t_end is not None and state.t >= t_end * (1 - 1e-12):
                break
            dt = cfl_dt(state, cfg, t_end)
        state = step(state, cfg, prm, dt)
        dts.append(dt)
        i += 1
    return state, dts


def flux_observable(rho, f_b, A, beta):
    """F = exp(-A Delta^beta), Delta = rho / rho_mean_gas."""
    return torch.exp(-A * (rho / f_b) ** beta)


def loss(state, target_flux, cfg, A, beta):
    """Mean squared difference of the final flux field against a target."""
    f = flux_observable(state.q[0], cfg.f_b, A, beta)
    return ((f - target_flux) ** 2).mean()


def conservation(state, cfg):
    """FP64 sums: gas mass, gas momentum (3), total gas energy, DM momentum (3)."""
    q = state.q
    return np.array([float(q[0].sum()), float(q[1].sum()), float(q[2].sum()), float(q[3].sum()),
                     float(q[4].sum()),
                     float(state.p[0].sum()) * (1 - cfg.f_b), float(state.p[1].sum()) * (1 - cfg.f_b),
                     float(state.p[2].sum()) * (1 - cfg.f_b)])


def default_config(**kw):
    return Config(**kw).finish()

"""Stochastic star formation with supernova heating (Sec. 2.4.1) and its relaxed,
differentiable form (Sec. 2.4.2, eq. reparam, eq. gumbelsoftmax).

Per cell and step:
  Delta = rho / rho_mean_gas, T from the specific internal energy;
  star-formation probability over the step  p_sf = 1 - exp(-eps_sf dt / t_ff), with the
  free-fall time of the proper gas density, t_ff = sqrt(3 pi / (32 G rho_prop)); in units
  of 1/H0 this is (pi/2) sqrt(a^3 / (Omega_b Delta));
  hard (discrete) model:  pi0 = p_sf * [Delta > Delta_c] * [T < T_c], z = Bernoulli(pi0);
  relaxed model: the thresholds become sigmoids, pi0 = p_sf s((Delta-Delta_c)/(w_rho Delta_c))
  s((T_c - T)/(w_T T_c)), and the draw the binary Gumbel-softmax
      z = s((log pi0 - log(1-pi0) + g0 - g1) / tau),
  where g0 - g1 of two independent Gumbel(0,1) variables is the logistic variable
  ln u - ln(1-u) of one uniform u.  The hard draw with the same u is z = [u > 1 - pi0],
  the tau -> 0 limit of the relaxed one.
Effect of a formation event: the specific energy E0 is added in the cell,
a^2 rho E += a^2 rho z E0, and the diagnostic star field gains z.  The gas mass is unchanged.
In a dual-energy state the entropy variable gains the same internal energy,
S += a^2 rho z E0 rho^(1-gamma).
E0 is given in (1000 km/s)^2.

Smoothed injection (an option; Sec. 2.4.1 models the supernova heating as the start of a
Sedov-Taylor blast in the surrounding gas, without fixing how the energy is placed): the
energy a^2 rho z E0 of each cell is spread over that cell and its 26 neighbours with the
weights w(ox) w(oy) w(oz), w(0) = 1/2, w(+-1) = 1/4, periodic.  The weights sum to one, so
the total energy injected is that of the local form.
"""

import math

import torch

from . import hydro

K_BOLTZMANN = 1.380649e-23      # J / K
M_PROTON = 1.67262192369e-27    # kg

MODE_OFF, MODE_HARD, MODE_RELAXED = 0, 1, 2


def kelvin_per_code_energy(gamma, mu, vel_unit_kms):
    """T = (gamma-1) mu m_p e / k_B, with e in code units of (vel_unit km/s)^2."""
    return (gamma - 1.0) * mu * M_PROTON / K_BOLTZMANN * (vel_unit_kms * 1e3) ** 2


def temperature(q, a, gamma, e_floor, t_per_e):
    """Gas temperature [K] from the floored specific internal energy (of the total energy,
    or the dual-energy selection: hydro.internal_energy)."""
    e, _ = hydro.internal_energy(q, a, gamma)
    return torch.clamp(e, min=e_floor) * t_per_e


def free_fall_time(delta, a, omega_b):
    """t_ff H0 = (pi/2) sqrt(a^3 / (Omega_b Delta)) for gas overdensity Delta."""
    return 0.5 * math.pi * torch.sqrt(a ** 3 / (omega_b * delta))


def formation_probability(delta, temp, a, dt, omega_b, eps_sf, delta_c, t_c, w_rho, w_t, mode):
    """pi0 for the hard or the relaxed model (see module docstring)."""
    p_sf = -torch.expm1(-eps_sf * dt / free_fall_time(delta, a, omega_b))
    if mode == MODE_HARD:
        gate = ((delta > delta_c) & (temp < t_c)).to(delta.dtype)
        return p_sf * gate
    return (p_sf * torch.sigmoid((delta - delta_c) / (w_rho * delta_c))
            * torch.sigmoid((t_c - temp) / (w_t * t_c)))


def draw(pi0, u, tau, mode):
    """Hard Bernoulli draw or its Gumbel-softmax relaxation, from the same uniform u."""
    if mode == MODE_HARD:
        return (u > 1.0 - pi0).to(pi0.dtype)
    logit = torch.log(pi0) - torch.log1p(-pi0)
    noise = torch.log(u) - torch.log1p(-u)
    return torch.sigmoid((logit + noise) / tau)


def smooth_injection(s):
    """The field s [n, n, n] spread over each cell and its 26 neighbours with the weights
    w(ox) w(oy) w(oz), w(0) = 1/2, w(+-1) = 1/4 (periodic), one axis after the other."""
    for d in range(3):
        s = 0.5 * s + 0.25 * (torch.roll(s, 1, d) + torch.roll(s, -1, d))
    return s


def apply_source(q, star, a, dt, u, *, rho_mean_gas, omega_b, gamma, e_floor, t_per_e,
                 e0_code, eps_sf, delta_c, t_c, w_rho, w_t, tau, mode, smooth=False,
                 with_draw=False):
    """Returns (Q, star) after one step of the source term (and the draw z, with_draw).
    smooth: the supernova energy is spread over the neighbouring cells (module docstring)."""
    rho = q[0]
    delta = rho / rho_mean_gas
    temp = temperature(q, a, gamma, e_floor, t_per_e)
    pi0 = formation_probability(delta, temp, a, dt, omega_b, eps_sf, delta_c, t_c,
                                w_rho, w_t, mode)
    z = draw(pi0, u, tau, mode)
    inj = a * a * rho * z * e0_code
    add = smooth_injection(inj) if smooth else inj
    e_new = q[4] + add
    # a dual-energy state: the entropy variable of the added internal energy, in the cell
    # that receives it
    extra = [q[5] + add * rho ** (1.0 - gamma)] if q.shape[0] > 5 else []
    out = (torch.stack([q[0], q[1], q[2], q[3], e_new] + extra), star + z)
    return out + (z,) if with_draw else out

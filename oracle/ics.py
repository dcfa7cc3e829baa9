"""Initial conditions of the oracle (Sec. 2.1): a Gaussian random field shaped by the linear
power spectrum, Zel'dovich (first-order LPT) displacements of a particle lattice, and a gas
state that tracks the dark matter.

  delta_k  = FFT(w)_k sqrt(P(k) D(a_i)^2 / V_cell)      (FFT unnormalised, inverse 1/N^3)
  Psi_k    = i k delta_k / k^2   (k in rad/cell, so div Psi = -delta; the derivative factor
             is zero on the Nyquist plane of its own axis, k = 0 mode zero)
  x        = q + Psi(q)  with q the cell centres;   p = a u = a_i^2 E(a_i) f(a_i) Psi(q)
  gas      rho = f_b CIC(x), momentum a rho U = rho p(q) on the cells, T = T_init.
The white noise w is an input, so the initial field is differentiable with respect to it.

Second-order LPT (an option; the paper evolves its initial field with LPT, Sec. 2.1): with
the potential phi of the linear field (lap phi = delta) and its second derivatives
phi_ij = IFFT(k_i k_j delta_k / k^2),
  delta2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2),
  Psi2   = -(D2 / D1^2) IFFT(i k delta2_k / k^2),      (D2 / D1^2 = -3/7 Omega_m(a)^(-1/143))
  x = q + Psi + Psi2,   p = a_i^2 E(a_i) (f(a_i) Psi + f2(a_i) Psi2),
every derivative factor k_j zero on the Nyquist plane of its own axis, as for Psi.
"""

import math

import torch

from . import cosmology, gravity


def lattice(n, dtype=torch.float64):
    """Cell-centre positions q [3, n^3] in particle order id = (z n + y) n + x."""
    r = torch.arange(n, dtype=dtype) + 0.5
    z, y, x = torch.meshgrid(r, r, r, indexing="ij")
    return torch.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)])


def linear_density(white, cfg):
    """delta_L at a_init from white noise [n, n, n] (torch float64)."""
    n = cfg.n
    kz, ky, kx = gravity.wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    kphys = torch.sqrt(k2) * (n / cfg.box)          # rad/cell -> h/Mpc
    pos = kphys > 0
    ks = torch.where(pos, kphys, torch.ones_like(kphys))
    tk = cosmology.transfer(ks, cfg.omega_m, cfg.omega_b, cfg.h, cfg.transfer, log=torch.log,
                            sqrt=torch.sqrt)
    pk = cfg.amp * ks ** cfg.n_s * tk ** 2
    pk = torch.where(pos, pk, torch.zeros_like(pk))
    d = cosmology.growth(cfg.a_init, cfg.omega_m)
    v_cell = (cfg.box / n) ** 3
    dk = torch.fft.rfftn(white) * torch.sqrt(pk * d * d / v_cell)
    return dk


def za_displacement(dk, n):
    """Psi [3, z, y, x] from the linear density spectrum (rfftn layout)."""
    kz, ky, kx = gravity.wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    inv_k2 = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)),
                         torch.zeros_like(k2))
    nyq = math.pi
    out = []
    for kj in (kx, ky, kz):
        kj_eff = torch.where(kj.abs() == nyq, torch.zeros_like(kj), kj)
        out.append(torch.fft.irfftn(1j * kj_eff * inv_k2 * dk, s=(n, n, n)))
    return torch.stack(out)


def _derivative_factors(n):
    """k_x, k_y, k_z (rad/cell, rfftn layout), each zero on the Nyquist plane of its axis, and
    1/k^2 (0 at k = 0)."""
    kz, ky, kx = gravity.wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    inv_k2 = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)),
                         torch.zeros_like(k2))
    eff = [torch.where(kj.abs() == math.pi, torch.zeros_like(kj), kj) for kj in (kx, ky, kz)]
    return eff, inv_k2


def second_order_source(dk, n):
    """delta2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2) of the linear spectrum dk (rfftn layout)."""
    eff, inv_k2 = _derivative_factors(n)
    hess = {}
    for i in range(3):
        for j in range(i, 3):
            hess[i, j] = torch.fft.irfftn(eff[i] * eff[j] * inv_k2 * dk, s=(n, n, n))
    return (hess[0, 0] * hess[1, 1] + hess[0, 0] * hess[2, 2] + hess[1, 1] * hess[2, 2]
            - hess[0, 1] ** 2 - hess[0, 2] ** 2 - hess[1, 2] ** 2)


def lpt2_displacement(dk, n, a, om):
    """Second-order displacement Psi2 [3, z, y, x] of the linear spectrum dk at scale factor a
    (module docstring)."""
    d2, _ = cosmology.lpt2_factors(a, om)
    return -d2 * za_displacement(torch.fft.rfftn(second_order_source(dk, n)), n)


def state_from_displacement(psi, cfg, psi2=None):
    """(Q, x, p) at a_init for a Zel'dovich displacement field psi [3, n, n, n] on the lattice
    (and a second-order one psi2, which moves the particles with the velocity factor f2)."""
    n = cfg.n
    a = cfg.a_init
    vfac = a * a * cosmology.hubble_e(a, cfg.omega_m) * cosmology.growth_rate(a, cfg.omega_m)
    vel = vfac * psi
    if psi2 is not None:
        _, f2 = cosmology.lpt2_factors(a, cfg.omega_m)
        vel = vel + a * a * cosmology.hubble_e(a, cfg.omega_m) * f2 * psi2
        psi = psi + psi2
    psi_p = psi.reshape(3, -1)
    x = torch.remainder(lattice(n) + psi_p, float(n))
    p = vel.reshape(3, -1)
    rho = cfg.f_b * gravity.cic_deposit(x, 1.0, n)
    mom = rho * vel
    u = mom / (a * rho)
    etot = a * a * rho * (cfg.e_init + 0.5 * (u * u).sum(0))
    # dual energy: the entropy variable of the initial internal energy, a^2 rho e_init
    # rho^(1-gamma)
    extra = ([(a * a * cfg.e_init * rho ** (2.0 - cfg.gamma))[None]]
             if getattr(cfg, "dual_energy", False) else [])
    q = torch.cat([rho[None], mom, etot[None]] + extra)
    return q, x, p


def initial_state(white, cfg):
    """Returns (Q, x, p) at a_init from white noise [n, n, n] (float64 tensor), with first- or
    second-order LPT (cfg.lpt)."""
    dk = linear_density(white, cfg)
    psi2 = lpt2_displacement(dk, cfg.n, cfg.a_init, cfg.omega_m) if cfg.lpt == 2 else None
    return state_from_displacement(za_displacement(dk, cfg.n), cfg, psi2)

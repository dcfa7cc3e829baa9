"""Particle-mesh gravity of the oracle (Sec. 2.2): cloud-in-cell deposit and read-out, FFT
Poisson solve, central-difference gradient, leapfrog kick and drift.

Equations of motion (eq. dm_hamil): dx/dt = u/a, d(a u)/dt = g with g = -grad(phi).
Particle variables are the comoving position x [cells] and p = a u, so dx/dt = p/a^2 and
dp/dt = g.  The peculiar potential obeys lap(phi) = (3 Om / 2a) delta_m, delta_m the total
(gas + dark matter) overdensity with mean matter density 1 per cell.

Mesh conventions (readings of Sec. 2.2, which names CIC and an FFT Poisson solve only): the
mesh is the gas grid; CIC uses cell centres, i0 = floor(x - 1/2), w1 = x - 1/2 - i0; the
same weights deposit and read out;
the Green's function is -1/k^2 with continuous k = 2 pi n / N, k = 0 set to zero; no CIC
deconvolution; g on the mesh by the two-point central difference.
"""

import math

import torch


def _corners(x, n):
    """Indices and weights of the 8 CIC corners for positions x [3, Np]."""
    s = x - 0.5
    i0 = torch.floor(s)
    w1 = s - i0
    w0 = 1.0 - w1
    i0 = i0.long() % n
    i1 = (i0 + 1) % n
    out = []
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                ix = i1[0] if cx else i0[0]
                iy = i1[1] if cy else i0[1]
                iz = i1[2] if cz else i0[2]
                w = (w1[0] if cx else w0[0]) * (w1[1] if cy else w0[1]) * (w1[2] if cz else w0[2])
                out.append(((iz * n + iy) * n + ix, w))
    return out


def cic_deposit(x, mass, n):
    """Mass per cell [z, y, x] of particles at x [3, Np], each of mass `mass` (scalar or [Np])."""
    rho = torch.zeros(n ** 3, dtype=x.dtype)
    for idx, w in _corners(x, n):
        rho = rho.index_add(0, idx, mass * w)
    return rho.reshape(n, n, n)


def cic_readout(field, x):
    """Field [z, y, x] (or [k, z, y, x]) interpolated to x [3, Np] with the CIC weights."""
    n = field.shape[-1]
    flat = field.reshape(*field.shape[:-3], n ** 3)
    acc = 0.0
    for idx, w in _corners(x, n):
        acc = acc + flat[..., idx] * w
    return acc


def wavenumbers(n, dtype=torch.float64):
    """k_z, k_y, k_x in rad/cell broadcastable to the rfftn layout [n, n, n//2+1]."""
    kz = 2.0 * math.pi * torch.fft.fftfreq(n, dtype=dtype).reshape(n, 1, 1)
    ky = 2.0 * math.pi * torch.fft.fftfreq(n, dtype=dtype).reshape(1, n, 1)
    kx = 2.0 * math.pi * torch.fft.rfftfreq(n, dtype=dtype).reshape(1, 1, n // 2 + 1)
    return kz, ky, kx


def poisson(delta, a, om):
    """phi with lap(phi) = (3 Om/2a) delta: phi_k = -(3 Om / 2a) delta_k / k^2, phi_0 = 0."""
    n = delta.shape[-1]
    kz, ky, kx = wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    green = torch.where(k2 > 0, -1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)),
                        torch.zeros_like(k2))
    dk = torch.fft.rfftn(delta, dim=(-3, -2, -1))
    return torch.fft.irfftn(dk * (1.5 * om / a) * green, s=(n, n, n), dim=(-3, -2, -1))


def grad_central(phi):
    """Acceleration g_d = -(phi_{j+1} - phi_{j-1})/2 along each axis: [3, z, y, x]."""
    dims = {0: 2, 1: 1, 2: 0}
    return torch.stack([-(torch.roll(phi, -1, dims[d]) - torch.roll(phi, 1, dims[d])) / 2.0
                        for d in range(3)])


def total_overdensity(rho_gas, x, dm_mass, n):
    """delta_m = (rho_gas + CIC(dark matter)) / rho_mean - 1 with rho_mean = 1 per cell."""
    return rho_gas + cic_deposit(x, dm_mass, n) - 1.0


def gas_kick(q, g, h):
    """Gravity source S_g of eq. conservation over a time h, in operator-split form:
    m += rho g h;  a^2 rho E += m_bar . g h with m_bar the mean of m before and after,
    which leaves the internal energy a^2 rho e unchanged (and with it the entropy of a
    dual-energy state, passed through)."""
    rho = q[0]
    m_old = q[1:4]
    m_new = m_old + rho * g * h
    e_new = q[4] + (0.5 * (m_old + m_new) * g).sum(0) * h
    return torch.cat([rho[None], m_new, e_new[None], q[5:]])


def dm_kick(p, x, g, h):
    """p += g(x) h with g read out at the particles by CIC."""
    return p + cic_readout(g, x) * h


def dm_drift_by(x, p, factor, n):
    """x += p * factor, wrapped into the periodic box [0, n)."""
    return torch.remainder(x + p * factor, float(n))


def dm_drift(x, p, dt, a_mid, n):
    """x += p dt / a_mid^2 (midpoint rule for dx/dt = p/a^2), periodic wrap to [0, n)."""
    return torch.remainder(x + p * (dt / (a_mid * a_mid)), float(n))

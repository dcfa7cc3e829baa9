"""Pins of the oracle's second-order LPT initial conditions and the Eisenstein & Hu transfer
function (Sec. 2.1): for one plane wave the second-order source vanishes exactly (the
Zel'dovich solution is exact in one dimension); for two crossing waves the second-order
displacement has the closed form derived from the definitions; the growth factors reach
their Einstein-de Sitter values D2 = -3/7 D1^2, f2 = 2 at early times; the transfer function
tends to 1 at small k and to its large-q asymptote ln(1.8 q) / (14.2 q^2)."""

import math

import numpy as np
import torch

import synth_inputs as si
from oracle import cosmology, gravity, ics, sim as osim

torch.set_default_dtype(torch.float64)


def _grid(n):
    i = torch.arange(n, dtype=torch.float64)
    return i[:, None, None], i[None, :, None], i[None, None, :]   # z, y, x


def test_plane_wave_has_no_second_order_displacement():
    n = 16
    z, y, x = _grid(n)
    for kvec in ((0, 0, 3), (0, 2, 0), (1, 1, 2)):
        k = [2 * math.pi * m / n for m in kvec]          # (kz, ky, kx)
        delta = 0.2 * torch.cos(k[0] * z + k[1] * y + k[2] * x).expand(n, n, n)
        dk = torch.fft.rfftn(delta)
        d2 = ics.second_order_source(dk, n)
        assert float(d2.abs().max()) < 1e-15, kvec
        psi2 = ics.lpt2_displacement(dk, n, 0.01, 0.3)
        assert float(psi2.abs().max()) < 1e-15, kvec


def test_two_crossing_waves_match_the_closed_form():
    n, A, B, m1, m2 = 32, 0.3, 0.2, 3, 5
    z, y, x = _grid(n)
    k1, k2 = 2 * math.pi * m1 / n, 2 * math.pi * m2 / n
    delta = (A * torch.cos(k1 * x) + B * torch.cos(k2 * y)).expand(n, n, n)
    dk = torch.fft.rfftn(delta)
    # phi_xx = A cos(k1 x), phi_yy = B cos(k2 y), mixed derivatives zero
    d2 = ics.second_order_source(dk, n)
    expect = (A * B * torch.cos(k1 * x) * torch.cos(k2 * y)).expand(n, n, n)
    assert torch.allclose(d2, expect, rtol=0, atol=1e-14)
    a, om = 0.05, 0.3
    c2 = -cosmology.lpt2_factors(a, om)[0]
    psi2 = ics.lpt2_displacement(dk, n, a, om)
    amp = c2 * A * B / (k1 * k1 + k2 * k2)
    ex = (-amp * k1 * torch.sin(k1 * x) * torch.cos(k2 * y)).expand(n, n, n)
    ey = (-amp * k2 * torch.cos(k1 * x) * torch.sin(k2 * y)).expand(n, n, n)
    assert torch.allclose(psi2[0], ex, rtol=0, atol=1e-14)
    assert torch.allclose(psi2[1], ey, rtol=0, atol=1e-14)
    assert float(psi2[2].abs().max()) < 1e-15


def test_second_order_growth_reaches_einstein_de_sitter():
    d2, f2 = cosmology.lpt2_factors(1e-4, 0.3)
    assert abs(d2 + 3.0 / 7.0) < 1e-9 and abs(f2 - 2.0) < 1e-8
    assert abs(cosmology.omega_m_of_a(1.0, 0.3) - 0.3) < 1e-15
    d2, f2 = cosmology.lpt2_factors(1.0, 0.3)
    assert abs(d2 + 3.0 / 7.0 * 0.3 ** (-1.0 / 143.0)) < 1e-15
    assert abs(f2 - 2.0 * 0.3 ** (6.0 / 11.0)) < 1e-15


def test_lpt2_state_moves_particles_and_velocities_by_both_orders():
    n = 16
    cfg1 = osim.default_config(n=n, box=4.0, a_init=0.05)
    cfg2 = osim.default_config(n=n, box=4.0, a_init=0.05, lpt=2)
    w = torch.from_numpy(si.white_noise(n, 12)).double()
    q1, x1, p1 = ics.initial_state(w, cfg1)
    q2, x2, p2 = ics.initial_state(w, cfg2)
    dk = ics.linear_density(w, cfg2)
    psi2 = ics.lpt2_displacement(dk, n, cfg2.a_init, cfg2.omega_m).reshape(3, -1)
    a = cfg2.a_init
    _, f2 = cosmology.lpt2_factors(a, cfg2.omega_m)
    dx = ((x2 - x1 + n / 2) % n) - n / 2
    assert torch.allclose(dx, psi2, rtol=0, atol=1e-11)
    assert torch.allclose(p2 - p1, a * a * cosmology.hubble_e(a, cfg2.omega_m) * f2 * psi2,
                          rtol=0, atol=1e-13)
    assert abs(float(q2[0].sum()) - cfg2.f_b * n ** 3) < 1e-9
    assert float(psi2.abs().max()) > 1e-4 * float((x1 - ics.lattice(n)).abs().max())
    # Psi2 is a gradient: curl-free and of zero mean
    ps = torch.fft.rfftn(psi2.reshape(3, n, n, n), dim=(-3, -2, -1))
    kz, ky, kx = gravity.wavenumbers(n)
    kx, ky = (torch.where(k.abs() == math.pi, torch.zeros_like(k), k) for k in (kx, ky))
    curl_z = kx * ps[1] - ky * ps[0]
    assert float(curl_z.abs().max()) < 1e-9 * float(ps.abs().max())
    assert float(psi2.mean(1).abs().max()) < 1e-15


def test_eh_transfer_limits_and_normalisation():
    om, ob, h = 0.3, 0.05, 0.7
    assert abs(cosmology.eh_nowiggle_transfer(1e-7, om, ob, h) - 1.0) < 1e-5
    # large q: T q^2 -> ln(1.8 q) / 14.2 (q = k theta^2 / Gamma, Gamma -> alpha Om h)
    theta2 = (2.7255 / 2.7) ** 2
    wm, fb = om * h * h, ob / om
    alpha = 1.0 - 0.328 * math.log(431.0 * wm) * fb + 0.38 * math.log(22.3 * wm) * fb * fb
    for k in (1e4, 1e5):
        q = k * theta2 / (om * h * alpha)
        t = cosmology.eh_nowiggle_transfer(k, om, ob, h)
        assert abs(t * q * q / (math.log(1.8 * q) / 14.2) - 1.0) < 2e-3
    # the baryons suppress Eisenstein & Hu below BBKS of the same Om h, by tens of percent
    for k in (0.05, 0.2, 1.0):
        r = cosmology.eh_nowiggle_transfer(k, om, ob, h) / cosmology.bbks_transfer(k / (om * h))
        assert 0.5 < r < 1.2, (k, r)
    amp = cosmology.spectrum_amplitude(om, h, 0.96, 0.8, cosmology.TRANSFER_EH, ob)
    pk = lambda k: amp * k ** 0.96 * cosmology.eh_nowiggle_transfer(k, om, ob, h) ** 2 if k > 0 else 0.0
    assert abs(cosmology.sigma_r(pk, 8.0) - 0.8) < 1e-9

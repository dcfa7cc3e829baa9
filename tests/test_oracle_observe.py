"""Pins of the oracle's observables (Sec. 3): the baryon power spectrum against closed forms
(a single plane wave puts all its power in one bin with the amplitude fixed by Parseval; the
binning counts every mode of |m| <= nbins + 1/2 once; white noise has the flat spectrum
L^3 sigma^2 / n^3), the Gaussian spectrum loss and the field-level log-posterior on states
whose observable is known in closed form, and their gradients against central differences."""

import math

import numpy as np
import torch

import synth_inputs as si
from oracle import observe, sim as osim, subgrid

torch.set_default_dtype(torch.float64)


def _count_modes(n, j):
    """Brute-force count of integer vectors in the n^3 fft box whose |m| rounds to j."""
    half = n // 2
    c = 0
    rng = range(-half, half)
    for mz in rng:
        for my in rng:
            for mx in rng:
                r = math.sqrt(mx * mx + my * my + mz * mz)
                if j - 0.5 <= r < j + 0.5:
                    c += 1
    return c


def test_wavenumber_bins_round_exactly():
    n = 12
    j = observe.wavenumber_bins(n)
    for jj in range(0, 8):
        assert int((j == jj).sum()) == _count_modes(n, jj), jj


def test_plane_wave_power_is_in_one_bin():
    n, box, amp, f_b = 16, 5.0, 0.3, 0.2
    idx = torch.arange(n, dtype=torch.float64)
    for (mz, my, mx) in ((0, 0, 3), (1, 2, 2), (4, 0, 3)):
        m = math.sqrt(mx * mx + my * my + mz * mz)
        b = int(round(m)) - 1
        delta = amp * torch.cos(2 * math.pi * (mz * idx[:, None, None] + my * idx[None, :, None]
                                               + mx * idx[None, None, :]) / n)
        pk, kb, w = observe.power_spectrum(f_b * (1.0 + delta), f_b, box, 7)
        # two modes +-m, each |X| = amp n^3 / 2
        expect = box ** 3 * 2 * (amp * n ** 3 / 2) ** 2 / n ** 6 / float(w[b])
        assert abs(float(pk[b]) - expect) < 1e-12 * expect
        others = torch.cat([pk[:b], pk[b + 1:]])
        assert float(others.abs().max()) < 1e-20 * expect
        assert abs(float(kb[b]) - 2 * math.pi * (b + 1) / box) < 1e-15


def test_white_noise_spectrum_is_flat():
    n, box, sigma = 64, 20.0, 0.1
    rng = np.random.default_rng(4)
    d = torch.from_numpy(rng.standard_normal((n, n, n))) * sigma
    pk, _, w = observe.power_spectrum(1.0 + d, 1.0, box, 30)
    expect = box ** 3 * sigma ** 2 / n ** 3
    # each bin averages W_b independent chi-square(2)/2 modes (pairs): 5 sigma bound
    for b in range(3, 30):
        assert abs(float(pk[b]) / expect - 1.0) < 5.0 / math.sqrt(float(w[b]) / 2), b


def test_power_loss_closed_form_and_gradient():
    n, box, f_b, nb = 8, 4.0, 0.2, 4
    rng = np.random.default_rng(6)
    rho = torch.from_numpy(f_b * (1 + 0.2 * rng.standard_normal((n, n, n)))).requires_grad_(True)
    pk_obs = torch.from_numpy(rng.uniform(0.0, 0.1, nb))
    a = torch.from_numpy(rng.standard_normal((nb, nb)))
    cinv = a @ a.T + nb * torch.eye(nb)
    pk, _, _ = observe.power_spectrum(rho, f_b, box, nb)
    L = observe.power_loss(pk, pk_obs, cinv)
    r = (pk - pk_obs).detach().numpy()
    assert abs(float(L.detach()) - 0.5 * r @ cinv.numpy() @ r) < 1e-13 * abs(float(L.detach()))
    (g,) = torch.autograd.grad(L, rho)
    for idx in ((0, 0, 0), (3, 5, 1), (7, 2, 6)):
        h = 1e-6
        e = torch.zeros_like(rho)
        e[idx] = h
        with torch.no_grad():
            lp = observe.power_loss(observe.power_spectrum(rho + e, f_b, box, nb)[0], pk_obs, cinv)
            lm = observe.power_loss(observe.power_spectrum(rho - e, f_b, box, nb)[0], pk_obs, cinv)
        fd = float(lp - lm) / (2 * h)
        assert abs(fd - float(g[idx])) < 1e-6 * float(g.abs().max()), idx


def test_fli_observable_and_loss_on_a_uniform_state():
    """Uniform gas at rest: O = T everywhere (rho = rho_mean), the loss is the closed form."""
    n = 8
    cfg = osim.default_config(n=n, box=4.0)
    a, temp = 0.2, 2.5e4
    e = temp / cfg.t_per_e
    rho = cfg.f_b
    q = torch.zeros(5, n, n, n)
    q[0] = rho
    q[4] = a * a * rho * e
    kw = dict(rho_mean_gas=cfg.f_b, gamma=cfg.gamma, e_floor=cfg.e_floor, t_per_e=cfg.t_per_e)
    o = observe.fli_observable(q, a, **kw)
    assert torch.allclose(o, torch.full((n, n, n), temp), rtol=1e-14, atol=0)
    rng = np.random.default_rng(8)
    data = torch.from_numpy(rng.normal(temp, 1e3, (n, n, n)))
    nv = torch.from_numpy(rng.uniform(1e5, 1e6, (n, n, n)))
    w = torch.from_numpy(rng.standard_normal((n, n, n)))
    L = observe.fli_loss(q, a, data, nv, w, **kw)
    expect = 0.5 * float((((data - temp) ** 2) / nv).sum()) + 0.5 * float((w ** 2).sum())
    assert abs(float(L) - expect) < 1e-13 * expect
    # twice the density at the same specific energy doubles the observable
    q2 = q.clone()
    q2[0] *= 2.0
    q2[4] *= 2.0
    assert torch.allclose(observe.fli_observable(q2, a, **kw), 2.0 * o, rtol=1e-14, atol=0)


def test_fli_loss_gradient_against_finite_differences():
    n = 8
    cfg = osim.default_config(n=n, box=4.0)
    q = torch.from_numpy(si.smooth_gas_state(n, 0.2, seed=3, energy=0.6)).double().requires_grad_(True)
    rng = np.random.default_rng(9)
    kw = dict(rho_mean_gas=cfg.f_b, gamma=cfg.gamma, e_floor=cfg.e_floor, t_per_e=cfg.t_per_e)
    o = observe.fli_observable(q.detach(), 0.2, **kw)
    data = o * (1 + 0.1 * torch.from_numpy(rng.standard_normal((n, n, n))))
    nv = (0.2 * o) ** 2
    w = torch.from_numpy(rng.standard_normal((n, n, n)))
    L = observe.fli_loss(q, 0.2, data, nv, w, **kw)
    (g,) = torch.autograd.grad(L, q)
    for idx in ((0, 1, 2, 3), (1, 4, 4, 4), (4, 7, 0, 5), (3, 2, 6, 1)):
        h = 1e-6 * float(q[idx[0]].detach().abs().max())
        e = torch.zeros_like(q)
        e[idx] = h
        with torch.no_grad():
            fd = float(observe.fli_loss(q + e, 0.2, data, nv, w, **kw)
                       - observe.fli_loss(q - e, 0.2, data, nv, w, **kw)) / (2 * h)
        assert abs(fd - float(g[idx])) < 1e-5 * float(g[idx[0]].abs().max()), idx

"""Observables and losses of the paper's two applications (Sec. 3).  Test infrastructure: only
tests and the benchmark's CPU baseline use the oracle.

Baryon power spectrum (the summary statistic of the parameter inference): the gas overdensity
delta_b = rho / rho_mean_gas - 1 is Fourier transformed, X_m = sum_x delta_x exp(-i k_m x)
over all n^3 modes m with integer wavenumber vector (mx, my, mz) (fft order), and
    P_b = (L^3 / n^6) sum_{m in bin b} |X_m|^2 / W_b,
bin b (b = 0 .. nbins-1) holding the modes whose |m| rounds to b + 1 (|m| in [b+1/2, b+3/2):
no |m| is ever a half-integer, so no tie), W_b their number, k_b = 2 pi (b + 1) / L in h/Mpc.
The loss of a mock spectrum is the Gaussian one, L = 1/2 (P - P_obs)^T C^-1 (P - P_obs) with
the inverse covariance C^-1 given (the paper estimates C from independent boxes).

Field-level inference: the observable is proportional to the gas-mass-weighted temperature,
O = (rho / rho_mean_gas) T, with T from the floored specific internal energy, and the
negative log-posterior of the initial phases s (the white noise, whose prior is the standard
normal) is
    L(s) = 1/2 sum_i (d_i - O(s)_i)^2 / N_i + 1/2 sum_i s_i^2,
with N_i the noise variance of pixel i.
"""

import math

import torch

from . import subgrid


def wavenumber_bins(n):
    """Integer |m| rounded (the bin index + 1) of every mode of a full n^3 FFT, fft order
    [z, y, x]; computed exactly in integers."""
    f = torch.fft.fftfreq(n, d=1.0 / n).round().long()
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    j = torch.sqrt(m2.double()).round().long()
    # exact correction: j is the integer with (2j - 1)^2 <= 4 m2 < (2j + 1)^2
    j = torch.where(4 * m2 >= (2 * j + 1) ** 2, j + 1, j)
    j = torch.where((j > 0) & (4 * m2 < (2 * j - 1) ** 2), j - 1, j)
    return j


def power_spectrum(rho, rho_mean_gas, box, nbins):
    """(P_b, k_b, W_b) of the gas density rho [n, n, n] (module docstring)."""
    n = rho.shape[-1]
    delta = rho / rho_mean_gas - 1.0
    x = torch.fft.fftn(delta, dim=(-3, -2, -1))
    p2 = x.real ** 2 + x.imag ** 2
    j = wavenumber_bins(n)
    pk, counts = [], []
    for b in range(nbins):
        sel = j == b + 1
        counts.append(int(sel.sum()))
        pk.append(p2[sel].sum() / counts[-1])
    pk = torch.stack(pk) * (box ** 3 / float(n) ** 6)
    kb = torch.tensor([2.0 * math.pi * (b + 1) / box for b in range(nbins)], dtype=torch.float64)
    return pk, kb, torch.tensor(counts, dtype=torch.float64)


def power_loss(pk, pk_obs, cinv):
    """1/2 (P - P_obs)^T C^-1 (P - P_obs)."""
    r = pk - pk_obs
    return 0.5 * (r @ (cinv @ r))


def fli_observable(q, a, *, rho_mean_gas, gamma, e_floor, t_per_e):
    """O = (rho / rho_mean_gas) T [K]: gas-mass-weighted temperature."""
    return q[0] / rho_mean_gas * subgrid.temperature(q, a, gamma, e_floor, t_per_e)


def fli_loss(q, a, data, noise_var, white, *, rho_mean_gas, gamma, e_floor, t_per_e):
    """Negative log-posterior of the initial phases (module docstring)."""
    o = fli_observable(q, a, rho_mean_gas=rho_mean_gas, gamma=gamma, e_floor=e_floor,
                       t_per_e=t_per_e)
    return 0.5 * (((data - o) ** 2) / noise_var).sum() + 0.5 * (white ** 2).sum()

"""Pins of the FP64 oracle against things other than itself: published known-answer
vectors, textbook values, closed forms, independent integrations, brute force on tiny
inputs and invariants.  CPU only."""

import math
import os

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import cosmology, gravity, hydro, philox, riemann

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
torch.set_default_dtype(torch.float64)


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


# ---------------------------------------------------------------- Philox

def test_philox_known_answers():
    for row in _rows("philox4x32_10_kat.txt"):
        v = [int(s, 16) for s in row]
        out = philox.philox4x32_10(*v[:4], v[4], v[5])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_open_interval_and_normals():
    u = philox.uniform_open(np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert 0.0 < u[0] < 1e-7 and 1 - 1e-7 < u[1] < 1.0
    z = philox.white_noise(7, 32)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.std() - 1.0) < 0.01
    # Different seeds and steps give different streams
    assert not np.array_equal(philox.starform_uniform(1, 0, 8), philox.starform_uniform(1, 1, 8))


# ---------------------------------------------------------------- cosmology

def test_scale_factor_closed_form_matches_ode():
    om = 0.3
    t0, t1 = cosmology.time_of_a(0.01, om), cosmology.time_of_a(1.0, om)
    sol = integrate.solve_ivp(lambda t, a: a * cosmology.hubble_e(a[0], om), (t0, t1), [0.01],
                              rtol=1e-12, atol=1e-14, dense_output=True)
    for t in np.linspace(t0, t1, 7):
        assert abs(sol.sol(t)[0] - cosmology.a_of_time(t, om)) < 1e-9
    assert abs(cosmology.a_of_time(t1, om) - 1.0) < 1e-12


def test_growth_factor_matches_growth_ode_and_limits():
    om = 0.3
    # independent: D'' + (3/a + dlnE/da) D' - 1.5 om / (a^5 E^2) D = 0, growing mode D ~ a
    def rhs(a, y):
        e = cosmology.hubble_e(a, om)
        dlne = -1.5 * om / a ** 4 / e ** 2
        return [y[1], -(3.0 / a + dlne) * y[1] + 1.5 * om / (a ** 5 * e * e) * y[0]]
    a0 = 1e-4
    sol = integrate.solve_ivp(rhs, (a0, 1.0), [a0, 1.0], rtol=1e-11, atol=1e-16, dense_output=True)
    d1 = sol.sol(1.0)[0]
    for a in (0.01, 0.1, 0.29, 0.6):
        assert abs(sol.sol(a)[0] / d1 - cosmology.growth(a, om)) < 2e-7
        fd = sol.sol(a)[1] * a / sol.sol(a)[0]
        assert abs(fd - cosmology.growth_rate(a, om)) < 2e-7
    # Einstein-de Sitter limit: D_u -> a, f -> 1 at early times
    assert abs(cosmology.growth_unnormalised(1e-4, om) / 1e-4 - 1.0) < 1e-6
    assert abs(cosmology.growth_rate(1e-4, om) - 1.0) < 1e-6


def test_bbks_limits_and_sigma8_normalisation():
    assert abs(cosmology.bbks_transfer(1e-9) - 1.0) < 1e-6
    assert cosmology.bbks_transfer(10.0) < 1e-2
    om, h, ns = 0.3, 0.7, 0.96
    amp = cosmology.spectrum_amplitude(om, h, ns, 0.8)
    # independent quadrature: trapezoid on a fine log grid
    lnk = np.linspace(math.log(1e-6), math.log(1e4), 400001)
    k = np.exp(lnk)
    q = k / (om * h)
    t = np.log(1 + 2.34 * q) / (2.34 * q) * (1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3
                                           + (6.71 * q) ** 4) ** -0.25
    x = 8.0 * k
    w = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    s2 = np.trapezoid(k ** 3 * amp * k ** ns * t * t * w * w, lnk) / (2 * math.pi ** 2)
    assert abs(math.sqrt(s2) - 0.8) < 1e-5


# ---------------------------------------------------------------- Riemann solver

def test_exact_riemann_matches_textbook_sod():
    ps, us, rl, rr = [float(v) for v in _rows("sod_toro_test1.txt")[0]]
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    p, u = riemann.star_state(left, right, 1.4)
    assert abs(p - ps) < 1e-5 and abs(u - us) < 1e-5
    # star densities just left and right of the contact
    assert abs(riemann.sample(u - 1e-6, left, right, 1.4)[0] - rl) < 1e-5
    assert abs(riemann.sample(u + 1e-6, left, right, 1.4)[0] - rr) < 1e-5


# ---------------------------------------------------------------- limiter

def test_van_leer_limiter_cases():
    a = torch.tensor([1.0, -2.0, 1.0, 0.0, 3.0, 1e-3])
    b = torch.tensor([3.0, -6.0, -1.0, 5.0, 0.0, 1e-3])
    got = hydro.van_leer(a, b)
    want = torch.tensor([2 * 3 / 4.0, 2 * 12 / -8.0, 0.0, 0.0, 0.0, 1e-3])
    assert torch.allclose(got, want, rtol=1e-12, atol=0)
    # symmetric, odd, bounded by 2 min(|a|,|b|) and by |a|+|b|
    x = torch.randn(1000)
    y = torch.randn(1000)
    assert torch.equal(hydro.van_leer(x, y), hydro.van_leer(y, x))
    assert torch.allclose(hydro.van_leer(-x, -y), -hydro.van_leer(x, y))
    assert (hydro.van_leer(x, y).abs() <= 2 * torch.minimum(x.abs(), y.abs()) + 1e-15).all()


# ---------------------------------------------------------------- CIC

def _cic_brute(xp, n):
    rho = np.zeros((n, n, n))
    for p in xp.T:
        for iz in range(n):
            for iy in range(n):
                for ix in range(n):
                    w = 1.0
                    for c, i in zip(p, (ix, iy, iz)):
                        # periodic distance between particle and cell centre
                        dd = (c - (i + 0.5) + n / 2) % n - n / 2
                        w *= max(0.0, 1.0 - abs(dd))
                    rho[iz, iy, ix] += w
    return rho


def test_cic_deposit_brute_force():
    rng = np.random.default_rng(3)
    n = 4
    xp = rng.uniform(0, n, size=(3, 6))
    xp[:, 0] = [0.1, 3.9, 2.5]   # wraps on both sides
    got = gravity.cic_deposit(torch.from_numpy(xp), 1.0, n).numpy()
    assert np.allclose(got, _cic_brute(xp, n), atol=1e-14)


def test_cic_lattice_and_adjointness():
    from oracle import ics
    n = 8
    q = ics.lattice(n)
    assert torch.allclose(gravity.cic_deposit(q, 1.0, n), torch.ones(n, n, n), atol=1e-14)
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.uniform(0, n, size=(3, 50)))
    m = torch.from_numpy(rng.normal(size=50))
    f = torch.from_numpy(rng.normal(size=(n, n, n)))
    lhs = (gravity.cic_deposit(x, m, n) * f).sum()
    rhs = (m * gravity.cic_readout(f, x)).sum()
    assert abs(float(lhs - rhs)) < 1e-12
    # total mass is conserved by the deposit
    assert abs(float(gravity.cic_deposit(x, m, n).sum() - m.sum())) < 1e-12


# ---------------------------------------------------------------- Poisson

@pytest.mark.parametrize("axis,mode", [(0, 1), (1, 3), (2, 2)])
def test_poisson_sinusoid_exact(axis, mode):
    n, a, om, amp = 16, 0.5, 0.3, 0.7
    r = torch.arange(n, dtype=torch.float64)
    k = 2 * math.pi * mode / n
    shape = [1, 1, 1]
    shape[2 - axis] = n
    wave = torch.sin(k * r).reshape(shape).expand(n, n, n)
    phi = gravity.poisson(amp * wave, a, om)
    expect = -(1.5 * om / a) * amp * wave / k ** 2
    assert torch.allclose(phi, expect, atol=1e-12)
    g = gravity.grad_central(phi)
    # central difference of sin gives cos times sin(k)/k
    cosw = torch.cos(k * r).reshape(shape).expand(n, n, n)
    g_exp = (1.5 * om / a) * amp / k ** 2 * cosw * math.sin(k)
    assert torch.allclose(g[axis], g_exp, atol=1e-12)
    for other in range(3):
        if other != axis:
            assert g[other].abs().max() < 1e-12

"""Pins of the oracle's FastPM kick and drift factors (the growth-factor form of the
kick-drift-kick step that the paper's particle mesh uses, Sec. 2.2): the two growth
functions they are built from against numerical derivatives of the growth factor, their
small-step limit (the leapfrog in t), and a Zel'dovich pancake integrated in a few large
steps, where the growth-factor factors follow the exact solution and the leapfrog does not.
CPU only."""

import math

import numpy as np
import pytest
import torch

from oracle import cosmology, gravity, ics, sim

torch.set_default_dtype(torch.float64)
OM = 0.3


def _d_of_t(t):
    return cosmology.growth(cosmology.a_of_time(t, OM), OM)


@pytest.mark.parametrize("a", [0.01, 0.1, 0.5])
def test_growth_momentum_is_a2_dD_dt(a):
    """G(a) = a^2 dD/dt, checked by a central difference of D(a(t)) in t."""
    t = cosmology.time_of_a(a, OM)
    h = 1e-4 * t
    num = a * a * (_d_of_t(t + h) - _d_of_t(t - h)) / (2 * h)
    assert cosmology.growth_momentum(a, OM) == pytest.approx(num, rel=1e-7)


@pytest.mark.parametrize("a", [0.01, 0.1, 0.5])
def test_growth_force_is_dG_dt(a):
    """F(a) = dG/dt = (3 Om / 2a) D: the linear growth equation, checked by a central
    difference of G(a(t)) in t (an error in G's formula or in F's fails one of the two)."""
    t = cosmology.time_of_a(a, OM)
    h = 1e-4 * t
    g = lambda tt: cosmology.growth_momentum(cosmology.a_of_time(tt, OM), OM)
    num = (g(t + h) - g(t - h)) / (2 * h)
    assert cosmology.growth_force(a, OM) == pytest.approx(num, rel=1e-6)


def test_factors_reduce_to_leapfrog_for_small_steps():
    """K0 -> dt/2 and K1 -> dt/2 to first order in dt, Dr -> dt / a_half^2 to second."""
    a0 = 0.2
    t0 = cosmology.time_of_a(a0, OM)
    errs = []
    for dt in (1e-3, 1e-4):
        ah, a1 = cosmology.a_of_time(t0 + dt / 2, OM), cosmology.a_of_time(t0 + dt, OM)
        k0, dr, k1 = cosmology.fastpm_factors(a0, ah, a1, OM)
        errs.append((abs(k0 / (dt / 2) - 1), abs(k1 / (dt / 2) - 1), abs(dr / (dt / ah ** 2) - 1)))
    for e0, e1 in zip(*errs):
        assert e1 < e0
    assert errs[1][0] < 2e-3 and errs[1][1] < 2e-3 and errs[1][2] < 1e-7
    # first order for the kicks, second order for the drift
    assert errs[0][0] / errs[1][0] == pytest.approx(10.0, rel=0.05)
    assert errs[0][2] / errs[1][2] == pytest.approx(100.0, rel=0.05)


def _dm_pancake(n, frac, a_final, nsteps, kdk):
    """Dark matter only (all the matter in the particles): a plane sine mode along x that
    reaches `frac` of shell crossing at a_final, from the Zel'dovich state at a_init,
    integrated in nsteps kick-drift-kick steps of equal d ln a.  Returns the displacement of
    the mode relative to the exact solution (the Zel'dovich one, exact in one dimension
    before shell crossing), and the same for the momenta."""
    cfg = sim.default_config(n=n, box=20.0, kdk=kdk)
    a0 = cfg.a_init
    di = cosmology.growth(a0, OM)
    k = 2 * math.pi / n
    amp = frac / (k * cosmology.growth(a_final, OM) / di)
    r = torch.arange(n, dtype=torch.float64) + 0.5
    psi = torch.zeros(3, n, n, n)
    psi[0] = (amp * torch.sin(k * r)).reshape(1, 1, n).expand(n, n, n)
    basis = psi[0].reshape(-1)
    x = torch.remainder(ics.lattice(n) + psi.reshape(3, -1), float(n))
    p = cosmology.growth_momentum(a0, OM) / di * psi.reshape(3, -1)
    lna = np.linspace(math.log(a0), math.log(a_final), nsteps + 1)
    force = lambda xx, a: gravity.grad_central(
        gravity.poisson(gravity.cic_deposit(xx, 1.0, n) - 1.0, a, OM))
    for i in range(nsteps):
        a_s, a_e = math.exp(lna[i]), math.exp(lna[i + 1])
        t_s, t_e = cosmology.time_of_a(a_s, OM), cosmology.time_of_a(a_e, OM)
        dt = t_e - t_s
        a_h = cosmology.a_of_time(t_s + 0.5 * dt, OM)
        k0, dr, k1 = sim.dm_factors(cfg, a_s, a_h, a_e, dt)
        p = gravity.dm_kick(p, x, force(x, a_s), k0)
        x = gravity.dm_drift_by(x, p, dr, n)
        p = gravity.dm_kick(p, x, force(x, a_e), k1)
    d = cosmology.growth(a_final, OM) / di
    dx = torch.remainder(x[0] - ics.lattice(n)[0] + n / 2, n) - n / 2
    disp = float(dx @ basis / (basis @ basis)) / d
    mom = float(p[0] @ basis / (basis @ basis)) / (cosmology.growth_momentum(a_final, OM) / di)
    return disp, mom


def test_pancake_in_few_steps_follows_the_exact_solution():
    """Five steps from a = 0.01 to 0.25: with the growth-factor factors the mode's
    displacement and momentum are those of many small leapfrog steps (the time integration
    is exact for the mode; what remains is the force discretisation, the same for both),
    while the leapfrog in t with the same five steps misses by far more."""
    ref = _dm_pancake(32, 0.3, 0.25, 200, sim.KDK_PLAIN)
    fpm = _dm_pancake(32, 0.3, 0.25, 5, sim.KDK_FASTPM)
    plain = _dm_pancake(32, 0.3, 0.25, 5, sim.KDK_PLAIN)
    for i in range(2):
        assert abs(fpm[i] - ref[i]) < 2e-3, (fpm, ref)
        assert abs(plain[i] - ref[i]) > 10 * abs(fpm[i] - ref[i]), (plain, fpm, ref)
    # and the many-step solution itself is the exact one up to the force discretisation
    # of a mode 32 cells long (2-point gradient and CIC: a few percent)
    assert abs(ref[0] - 1.0) < 0.05 and abs(ref[1] - 1.0) < 0.05

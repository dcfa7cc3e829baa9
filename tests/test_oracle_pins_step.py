"""Pins of the oracle's step-level functions that the physics or the mathematics fixes: the
gravity source of the gas, the relaxed star-formation gates, the CFL time step, the flux
loss and the BBKS transfer function.  Each test is chosen so that a plausible mistake in the
function (a dropped term, a wrong sign, index or normalisation) fails it.  CPU only."""

import math

import numpy as np
import pytest
import torch

from oracle import cosmology, gravity, hydro, sim as osim, subgrid

torch.set_default_dtype(torch.float64)


def _random_gas(n, seed, a):
    rng = np.random.default_rng(seed)
    rho = 0.1 + rng.random((n, n, n))
    u = rng.normal(0.0, 2.0, (3, n, n, n))
    e = 0.05 + rng.random((n, n, n))
    q = np.concatenate([rho[None], a * rho[None] * u,
                        (a * a * rho * (e + 0.5 * (u * u).sum(0)))[None]])
    return torch.from_numpy(q)


def _internal(q, a):
    rho = q[0]
    return q[4] / (a * a * rho) - 0.5 * ((q[1:4] / (a * rho)) ** 2).sum(0)


# ---------------------------------------------------------------- gravity source (S_g)

def test_gas_kick_leaves_internal_energy_and_does_work():
    """Gravity changes momentum by rho g h and does work only on the bulk motion: the
    internal energy is unchanged and the change of a^2 rho E equals the change of the
    kinetic part a^2 rho U^2/2 = |m|^2 / (2 rho).  A kick whose energy term uses the old
    momentum instead of the mean of old and new fails both checks."""
    a, h = 0.37, 0.8
    q = _random_gas(6, 1, a)
    g = torch.from_numpy(np.random.default_rng(2).normal(0.0, 1.5, (3, 6, 6, 6)))
    out = gravity.gas_kick(q, g, h)
    assert torch.equal(out[0], q[0])
    assert torch.allclose(out[1:4] - q[1:4], q[0] * g * h, rtol=1e-13, atol=1e-13)
    assert torch.allclose(_internal(out, a), _internal(q, a), rtol=1e-12, atol=1e-13)
    ke = lambda s: 0.5 * (s[1:4] ** 2).sum(0) / s[0]
    assert torch.allclose(out[4] - q[4], ke(out) - ke(q), rtol=1e-11, atol=1e-12)
    # a gas at rest in a uniform field gains exactly rho g^2 h^2 / 2
    q0 = q.clone()
    q0[1:4] = 0.0
    gu = torch.zeros_like(g)
    gu[1] = 0.25
    out0 = gravity.gas_kick(q0, gu, h)
    assert torch.allclose(out0[4] - q0[4], 0.5 * q0[0] * (0.25 * h) ** 2, rtol=1e-14)


def test_gas_kick_with_a_stale_momentum_fails_the_pin():
    """The pin above rejects the plausible mistake of using m_old in the energy term."""
    a, h = 0.37, 0.8
    q = _random_gas(4, 3, a)
    g = torch.from_numpy(np.random.default_rng(4).normal(0.0, 1.5, (3, 4, 4, 4)))
    wrong = q.clone()
    wrong[1:4] = q[1:4] + q[0] * g * h
    wrong[4] = q[4] + (q[1:4] * g).sum(0) * h
    assert not torch.allclose(_internal(wrong, a), _internal(q, a), rtol=1e-6)


# ---------------------------------------------------------------- star-formation gates

def _pi0(delta, temp, mode, w_rho=0.1, w_t=0.1, dc=100.0, tc=10 ** 4.5, a=0.25, dt=0.003):
    d = torch.as_tensor(delta, dtype=torch.float64)
    t = torch.as_tensor(temp, dtype=torch.float64)
    return subgrid.formation_probability(d, t, a, dt, 0.05, 0.02, dc, tc, w_rho, w_t, mode)


def test_relaxed_gates_reduce_to_hard_gates_as_widths_vanish():
    """pi0 = Pi0 s((delta - delta_c)/a) s((T_c - T)/b) recovers the sharp thresholds as
    a, b -> 0 (the relaxed model's stated limit): star formation above the density threshold
    and below the temperature threshold only."""
    rng = np.random.default_rng(5)
    delta = np.concatenate([rng.uniform(1, 99, 50), rng.uniform(101, 1000, 50)])
    temp = np.concatenate([rng.uniform(10, 3.1e4, 50), rng.uniform(3.2e4, 1e6, 50)])
    rng.shuffle(temp)
    hard = _pi0(delta, temp, subgrid.MODE_HARD)
    soft = _pi0(delta, temp, subgrid.MODE_RELAXED, w_rho=1e-9, w_t=1e-9)
    assert torch.allclose(soft, hard, rtol=1e-12, atol=0)
    assert int((hard > 0).sum()) > 10 and int((hard == 0).sum()) > 10


def test_relaxed_gates_are_logistic_in_the_scaled_distances():
    """At the thresholds each gate is s(0) = 1/2; one width a = w_rho delta_c above the
    density threshold the density gate is s(1) = e / (1 + e); one width b = w_T T_c below
    the temperature threshold the temperature gate is s(1) as well."""
    p_sf = lambda d: -math.expm1(-0.02 * 0.003 / (0.5 * math.pi * math.sqrt(0.25 ** 3 / (0.05 * d))))
    s1 = math.e / (1.0 + math.e)
    tc, dc = 10 ** 4.5, 100.0
    assert float(_pi0(dc, tc, subgrid.MODE_RELAXED)) == pytest.approx(p_sf(dc) / 4, rel=1e-13)
    d1 = dc * 1.1
    got = float(_pi0(d1, tc * 0.9, subgrid.MODE_RELAXED))
    assert got == pytest.approx(p_sf(d1) * s1 * s1, rel=1e-13)
    # far above the density threshold the density gate is 1 to double precision; at T = 1 K
    # the temperature gate is s((T_c - 1)/(0.1 T_c)), just below 1
    s_t = 1.0 / (1.0 + math.exp(-(tc - 1.0) / (0.1 * tc)))
    assert float(_pi0(1e6, 1.0, subgrid.MODE_RELAXED)) == pytest.approx(p_sf(1e6) * s_t,
                                                                         rel=1e-12)


# ---------------------------------------------------------------- CFL time step

def _uniform_state(n, a, rho, u, p, gamma):
    q = torch.zeros(5, n, n, n)
    q[0] = rho
    for d in range(3):
        q[1 + d] = a * rho * u[d]
    e = p / ((gamma - 1.0) * rho)
    q[4] = a * a * rho * (e + 0.5 * sum(x * x for x in u))
    z = torch.zeros(3, n ** 3)
    return osim.State(q=q, x=z, p=z, star=torch.zeros(n, n, n), phi=torch.zeros(n, n, n),
                      t=cosmology.time_of_a(a, 0.3), a=a, step=0)


def test_cfl_dt_speed_branch_on_a_uniform_moving_gas():
    """A uniform gas with peculiar velocity U moves across comoving cells at U/a; signals
    travel at (|U_d| + c_s)/a along axis d, c_s = sqrt(gamma p / rho).  eq. dt with the
    fastest axis: dt = C a / max_d(|U_d| + c_s).  Using |U| instead of the per-axis speed, or
    leaving out the 1/a, fails."""
    cfg = osim.default_config(n=4, cfl=0.4, dlna_max=10.0)
    a, rho, p = 0.2, 0.3, 0.05
    u = (1.5, -4.0, 2.5)
    st = _uniform_state(4, a, rho, u, p, cfg.gamma)
    cs = math.sqrt(cfg.gamma * p / rho)
    want = 0.4 * a / (4.0 + cs)
    assert osim.cfl_dt(st, cfg) == pytest.approx(want, rel=1e-12)
    # t_end inside the step clips it
    assert osim.cfl_dt(st, cfg, t_end=st.t + 0.25 * want) == pytest.approx(0.25 * want,
                                                                             rel=1e-9)


def test_cfl_dt_expansion_cap_branch():
    """A cold gas at rest: the step is set by the cap on d ln a, dt = dlna_max / E(a) with
    E(a) = H/H0 (da/dt = a E in units of 1/H0), so a(t + dt) / a(t) = exp(dlna_max) to
    second order in dlna_max."""
    cfg = osim.default_config(n=4, cfl=0.4, dlna_max=0.04)
    a = 0.1
    st = _uniform_state(4, a, 0.2, (0.0, 0.0, 0.0), 1e-12, cfg.gamma)
    dt = osim.cfl_dt(st, cfg)
    assert dt == pytest.approx(0.04 / math.sqrt(0.3 / a ** 3 + 0.7), rel=1e-12)
    ratio = cosmology.a_of_time(st.t + dt, 0.3) / a
    assert math.log(ratio) == pytest.approx(0.04, abs=0.04 ** 2)


# ---------------------------------------------------------------- loss

def test_loss_on_a_uniform_state_at_the_mean_density():
    """At the mean gas density Delta = 1, so F = exp(-A) in every cell and the mean squared
    difference against a uniform target is (exp(-A) - F_t)^2 (with Delta = rho instead of
    rho / rho_mean_gas, or a sum instead of a mean, it is not)."""
    cfg = osim.default_config(n=4)
    st = _uniform_state(4, 0.2, cfg.f_b, (0.0, 0.0, 0.0), 1e-3, cfg.gamma)
    A, beta, ft = 0.3, 1.6, 0.55
    L = osim.loss(st, torch.full((4, 4, 4), ft), cfg, A, beta)
    assert float(L) == pytest.approx((math.exp(-A) - ft) ** 2, rel=1e-13)
    # at twice the mean density F = exp(-A 2^beta)
    st.q[0] = 2.0 * cfg.f_b
    L = osim.loss(st, torch.full((4, 4, 4), ft), cfg, A, beta)
    assert float(L) == pytest.approx((math.exp(-A * 2 ** beta) - ft) ** 2, rel=1e-13)


# ---------------------------------------------------------------- BBKS transfer function

def test_bbks_small_q_expansion():
    """T(q) = ln(1 + c1 q)/(c1 q) (1 + c2 q + (c3 q)^2 + ...)^(-1/4): to first order
    1 - (c1/2 + c2/4) q, and the q^2 coefficient c1^2/3 + (c1/2)(c2/4) - c3^2/4 + 5 c2^2/32,
    with the published c1 = 2.34, c2 = 3.89, c3 = 16.1."""
    c1, c2, c3 = 2.34, 3.89, 16.1
    k1 = c1 / 2 + c2 / 4
    k2 = c1 * c1 / 3 + (c1 / 2) * (c2 / 4) - c3 * c3 / 4 + 5 * c2 * c2 / 32
    for q in (1e-4, 3e-5):
        t = cosmology.bbks_transfer(q)
        assert (t - 1.0 + k1 * q) / (q * q) == pytest.approx(k2, rel=2e-3)


def test_bbks_large_q_asymptote():
    """For q -> infinity, T q^2 -> ln(c1 q) / (c1 c5) with c5 = 6.71, and the first
    correction is q T q^2 c1 c5 / ln(c1 q) - q -> 1/(c1 ln(c1 q)) - c4^3 / (4 c5^4)
    (c4 = 5.46): the last two published coefficients."""
    c1, c4, c5 = 2.34, 5.46, 6.71
    for q in (1e5, 1e6):
        t = cosmology.bbks_transfer(q)
        ratio = t * q * q * c1 * c5 / math.log(c1 * q)
        assert ratio == pytest.approx(1.0, abs=1e-4)
        corr = q * (ratio - 1.0)
        want = 1.0 / (c1 * math.log(c1 * q)) - c4 ** 3 / (4 * c5 ** 4)
        assert corr == pytest.approx(want, abs=2e-3 * abs(want) + 1e-4)

"""Pins of the oracle's dual-energy formalism (the entropy variable S as a sixth gas
component; Sec. 2.3's extension of its single-energy scheme, with the selection and
synchronisation rule of Bryan et al. 1995).  Each test fixes a property that the mathematics
or the single-energy scheme decides:
  * an entropy proportional to the density stays so through any sweep (the flux of S is
    that of the density times S / rho, and the limiter is homogeneous of degree one);
  * flows where the total energy holds the internal energy well (Sod, Sedov) evolve exactly
    as in the single-energy scheme;
  * in a smooth isentropic wave the entropy's internal energy follows the total energy's to
    the scheme's truncation error;
  * a cold, highly supersonic uniform flow keeps the exact adiabatic temperature
    T0 (a0 / a)^2 through whole steps, where the single-energy temperature is rounding noise;
  * the synchronisation makes the two internal energies equal where it acts, and only there;
  * supernova heating raises both internal energies by the same amount.
CPU only."""

import math

import numpy as np
import torch

import synth_inputs as si
from oracle import gravity, hydro, philox, sim as osim, subgrid

torch.set_default_dtype(torch.float64)

G53 = 5.0 / 3.0


def _with_entropy(q, gamma=G53):
    return torch.cat([q, hydro.entropy_of_total(q, gamma)[None]])


def _e_total(q, a):
    """e_E and E of the total energy (no selection)."""
    rho = q[0]
    u = q[1:4] / (a * rho)
    big_e = q[4] / (a * a * rho)
    return big_e - 0.5 * (u * u).sum(0), big_e


def _smooth_state(n, a, seed):
    return torch.from_numpy(si.smooth_gas_state(n, a, seed=seed, energy=0.8)).double()


def test_entropy_proportional_to_density_stays_so():
    a, n = 0.3, 12
    q = _smooth_state(n, a, 3)
    k = 0.7
    q6 = torch.cat([q, k * q[:1]])
    for d in (0, 1, 2):
        q6 = hydro.sweep(q6, d, 0.04, a, a * 1.01, G53, 1e-6)
    ratio = q6[5] / q6[0]
    assert float((ratio / k - 1.0).abs().max()) < 1e-12


def test_warm_flows_evolve_as_single_energy():
    # a smooth warm state: e_E > eta1 E everywhere, so the sixth component never enters
    a, n = 0.3, 12
    q5 = _smooth_state(n, a, 5)
    q6 = _with_entropy(q5)
    for d in (0, 1, 2, 2, 1, 0):
        q5 = hydro.sweep(q5, d, 0.04, a, a * 1.01, G53, 1e-6)
        q6 = hydro.sweep(q6, d, 0.04, a, a * 1.01, G53, 1e-6)
        e, big_e = _e_total(q6, a)
        assert bool((e > hydro.DUAL_ETA1 * big_e).all())
    assert torch.equal(q6[:5], q5)


def _sod(n, gamma):
    xc = np.arange(n) + 0.5
    hi = (xc >= n / 4) & (xc < 3 * n / 4)
    q = torch.zeros(5, 1, 1, n)
    q[0, 0, 0] = torch.from_numpy(np.where(hi, 1.0, 0.125))
    q[4, 0, 0] = torch.from_numpy(np.where(hi, 1.0, 0.1) / (gamma - 1.0))
    return q


def _sedov(n):
    q = torch.zeros(5, n, n, n)
    q[0] = 1.0
    q[4] = 1e-6
    q[4, n // 2, n // 2, n // 2] += 50.0
    return q


def test_shocks_evolve_as_single_energy_and_sync_feeds_the_entropy():
    for q5, gamma, axes, steps in ((_sod(128, 1.4), 1.4, (0,), 60),
                                   (_sedov(16), G53, None, 8)):
        q6 = _with_entropy(q5, gamma)
        for s in range(steps):
            dt = 0.4 / hydro.max_signal_speed(q5, 1.0, gamma, 0.0)
            assert dt == 0.4 / hydro.max_signal_speed(q6, 1.0, gamma, 0.0)
            for d in (axes or hydro.strang_axes(s)):
                q5 = hydro.sweep(q5, d, dt, 1.0, 1.0, gamma, 0.0)
                q6 = hydro.sweep(q6, d, dt, 1.0, 1.0, gamma, 0.0)
            q6 = hydro.dual_sync(q6, 1.0, gamma)
        assert torch.equal(q6[:5], q5)
        # every cell holds its internal energy in the total energy here, so the sync has set
        # the entropy from it everywhere, shocked cells included
        e, big_e = _e_total(q6, 1.0)
        assert bool((e >= hydro.DUAL_ETA2 * big_e).all())
        e_s = hydro.entropy_energy(q6, 1.0, gamma)
        assert float(((e_s - e) / e).abs().max()) < 1e-12


def _isentropic_wave_run(n, steps, dt, a=0.5):
    """(max, mean) relative difference of e_S from e_E after `steps` steps of a smooth
    isentropic wave over n cells, and the largest change of e_E from the start."""
    r = torch.arange(n, dtype=torch.float64) + 0.5
    z, y, x = torch.meshgrid(r, r, r, indexing="ij")
    ph = 2 * math.pi * (x + y) / n
    rho = 1.0 + 0.2 * torch.sin(ph)
    e = 0.9 * rho ** (G53 - 1.0)                    # isentropic: e rho^(1-gamma) uniform
    u = torch.stack([0.3 * torch.sin(ph + 0.4), -0.2 * torch.cos(ph), 0.1 * torch.sin(2 * ph)])
    q = torch.cat([rho[None], a * rho * u, (a * a * rho * (e + 0.5 * (u * u).sum(0)))[None]])
    q6 = _with_entropy(q)
    e0 = hydro.entropy_energy(q6, a, G53)
    assert float(((e0 - e) / e).abs().max()) < 1e-13
    for s in range(steps):
        for d in hydro.strang_axes(s):
            q6 = hydro.sweep(q6, d, dt, a, a, G53, 0.0)
    e_tot, _ = _e_total(q6, a)
    rel = ((hydro.entropy_energy(q6, a, G53) - e_tot) / e_tot).abs()
    return float(rel.max()), float(rel.mean()), float(((e_tot - e) / e).abs().max())


def test_isentropic_wave_entropy_energy_follows_total_energy():
    # the same wave and physical time on 16 and 32 cells: the two internal energies differ
    # by the scheme's truncation error (its numerical dissipation makes entropy), which
    # shrinks with resolution; a wrong power of rho or a in e_S would leave ~20% or 100%
    mx16, mean16, _ = _isentropic_wave_run(16, 6, 0.2)
    mx32, mean32, moved = _isentropic_wave_run(32, 12, 0.1)
    assert mx32 < 2e-2 and mx32 < mx16
    assert mean32 < 0.4 * mean16
    assert moved > 2e-2   # the wave has moved: the check is not against the initial state


def _uniform_flow_state(cfg, v, dual):
    n = cfg.n
    a = cfg.a_init
    rho = torch.full((n, n, n), cfg.f_b)
    u = torch.zeros(3, n, n, n)
    u[0] = v
    q = torch.cat([rho[None], a * rho * u,
                   (a * a * rho * (cfg.e_init + 0.5 * (u * u).sum(0)))[None]])
    if dual:
        q = torch.cat([q, (a * a * cfg.e_init * rho ** (2.0 - cfg.gamma))[None]])
    r = torch.arange(n, dtype=torch.float64) + 0.5
    zz, yy, xx = torch.meshgrid(r, r, r, indexing="ij")
    x = torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)])
    p = a * u.reshape(3, -1)
    return osim.state_from_qxp(q, x, p, cfg)


def test_cold_supersonic_flow_keeps_the_adiabatic_temperature():
    temps = {}
    for dual in (False, True):
        cfg = osim.default_config(n=8, t_init=100.0, dual_energy=dual)
        v = math.sqrt(2.0e15 * cfg.e_init)          # kinetic / internal energy = 1e15
        st = _uniform_flow_state(cfg, v, dual)
        st, _ = osim.run(st, cfg, osim.Params(), schedule=[2e-4] * 6)
        assert st.a > 1.1 * cfg.a_init
        temps[dual] = subgrid.temperature(st.q, st.a, cfg.gamma, cfg.e_floor, cfg.t_per_e)
        exact = cfg.t_init * (cfg.a_init / st.a) ** 2
    assert float((temps[True] / exact - 1.0).abs().max()) < 1e-9
    # the single-energy temperature of the same flow is a difference of numbers 1e15 times
    # larger than itself
    assert float((temps[False] / exact - 1.0).abs().max()) > 1e-2


def test_sync_equalises_the_energies_where_it_acts_only():
    a, n = 0.4, 10
    g = torch.Generator().manual_seed(7)
    q = _smooth_state(n, a, 9)
    # a third of the cells fast and cold (kinetic energy 1e4 times the internal one: the
    # entropy's energy is used), a third moderately fast (30 times: the total energy's is
    # used, but the entropy is not reset), the rest as they are
    pick = torch.rand(n, n, n, generator=g)
    fast, moderate = pick < 0.33, (pick >= 0.33) & (pick < 0.66)
    rho = q[0]
    u = q[1:4] / (a * rho)
    e, _ = _e_total(q, a)
    ratio = torch.where(fast, 2e4, torch.where(moderate, 60.0, 0.0)) * e / (u * u).sum(0)
    u = u * torch.where(fast | moderate, torch.sqrt(ratio), torch.ones_like(e))
    q = torch.cat([rho[None], a * rho * u, (a * a * rho * (e + 0.5 * (u * u).sum(0)))[None]])
    s_rand = hydro.entropy_of_total(q, G53) * (1.0 + 0.3 * torch.rand(n, n, n, generator=g))
    q6 = torch.cat([q, s_rand[None]])
    out = hydro.dual_sync(q6, a, G53)
    e_tot, big_e = _e_total(q6, a)
    acted = e_tot >= hydro.DUAL_ETA2 * big_e
    assert torch.equal(acted, ~(fast | moderate))
    assert torch.equal(out[:5], q6[:5])
    assert torch.equal(out[5][~acted], q6[5][~acted])
    e_s = hydro.entropy_energy(out, a, G53)
    assert float(((e_s - e_tot) / e_tot)[acted].abs().max()) < 1e-11
    # and the selection takes the entropy's energy in the fast cells only
    e_sel, _ = hydro.internal_energy(out, a, G53)
    assert torch.equal(e_sel[fast], hydro.entropy_energy(out, a, G53)[fast])
    assert torch.equal(e_sel[~fast], e_tot[~fast])


def test_supernova_heating_raises_both_internal_energies_alike():
    n, a, e0 = 8, 0.2, 3.0
    cfg = osim.default_config(n=n)
    g = torch.Generator().manual_seed(2)
    rho = cfg.f_b * (200.0 + 50.0 * torch.rand(n, n, n, generator=g))   # above delta_c
    e = torch.full((n, n, n), cfg.e_init)
    q = torch.cat([rho[None], torch.zeros(3, n, n, n), (a * a * rho * e)[None]])
    q6 = _with_entropy(q)
    u = torch.from_numpy(philox.starform_uniform(102, 0, n))
    for smooth in (False, True):
        out, _, z = subgrid.apply_source(
            q6, torch.zeros(n, n, n), a, 0.05, u, rho_mean_gas=cfg.f_b, omega_b=cfg.omega_b,
            gamma=cfg.gamma, e_floor=cfg.e_floor, t_per_e=cfg.t_per_e, e0_code=e0,
            eps_sf=0.5, delta_c=100.0, t_c=1e9, w_rho=0.1, w_t=0.1, tau=0.1,
            mode=subgrid.MODE_HARD, smooth=smooth, with_draw=True)
        assert 0 < float(z.sum()) < n ** 3
        de_tot = _e_total(out, a)[0] - _e_total(q6, a)[0]
        de_s = hydro.entropy_energy(out, a, G53) - hydro.entropy_energy(q6, a, G53)
        assert float(de_tot.max()) > 0.1 * e0
        assert float((de_s - de_tot).abs().max()) < 1e-12 * e0
        if not smooth:
            assert float((de_tot - z * e0).abs().max()) < 1e-12 * e0


def test_gas_kick_leaves_the_entropy():
    a, n = 0.3, 6
    q6 = _with_entropy(_smooth_state(n, a, 1))
    gfield = torch.randn(3, n, n, n, generator=torch.Generator().manual_seed(0))
    out = gravity.gas_kick(q6, gfield, 0.02)
    assert torch.equal(out[5], q6[5])
    assert torch.equal(out[:5], gravity.gas_kick(q6[:5], gfield, 0.02))


def test_initial_conditions_and_steps_keep_the_energies_in_step():
    # initial state: both internal energies are e_init; after whole steps of warm gas the
    # synchronisation has made them equal again (without it they would differ by the
    # entropy the scheme makes)
    cfg = osim.default_config(n=8, t_init=1e6, dual_energy=True)
    w = torch.from_numpy(philox.white_noise(5, 8))
    st = osim.initial_state(w, cfg)
    assert st.q.shape[0] == 6
    e_tot, big_e = _e_total(st.q, st.a)
    assert float((hydro.entropy_energy(st.q, st.a, G53) / cfg.e_init - 1.0).abs().max()) < 1e-12
    assert float((e_tot / cfg.e_init - 1.0).abs().max()) < 1e-9
    st, _ = osim.run(st, cfg, osim.Params(), nsteps=3)
    e_tot, big_e = _e_total(st.q, st.a)
    assert bool((e_tot >= hydro.DUAL_ETA2 * big_e).all())
    assert float(((hydro.entropy_energy(st.q, st.a, G53) - e_tot) / e_tot).abs().max()) < 1e-12

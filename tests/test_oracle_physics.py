"""Physics pins of the FP64 oracle: Zel'dovich pancake (PM + kick/drift + gas), Sedov blast
radius, initial-condition statistics, conservation with gravity, the star-formation draw
statistics and unit conversions, and finite-difference checks of the oracle's reverse-mode
gradient.  CPU only."""

import math

import numpy as np
import pytest
import torch
from scipy.ndimage import map_coordinates

from oracle import cosmology, gravity, hydro, ics, philox, sim, subgrid

torch.set_default_dtype(torch.float64)


# ---------------------------------------------------------------- Zel'dovich pancake

def _pancake(n, frac, a_final=0.25):
    """Plane sine mode along x reaching `frac` of shell crossing at a_final."""
    cfg = sim.default_config(n=n, box=20.0)
    di = cosmology.growth(cfg.a_init, cfg.omega_m)
    k = 2 * math.pi / n
    amp = frac / (k * cosmology.growth(a_final, cfg.omega_m) / di)
    r = torch.arange(n, dtype=torch.float64) + 0.5
    psi = torch.zeros(3, n, n, n)
    psi[0] = (amp * torch.sin(k * r)).reshape(1, 1, n).expand(n, n, n)
    st = sim.state_from_qxp(*ics.state_from_displacement(psi, cfg), cfg)
    st, _ = sim.run(st, cfg, sim.Params(), a_final=a_final)
    basis = psi[0].reshape(-1)
    dx = torch.remainder(st.x[0] - ics.lattice(n)[0] + n / 2, n) - n / 2
    d = cosmology.growth(st.a, cfg.omega_m) / di
    vfac = st.a ** 2 * cosmology.hubble_e(st.a, cfg.omega_m) * cosmology.growth_rate(st.a, cfg.omega_m)
    disp_ratio = float(dx @ basis / (basis @ basis)) / d
    mom_ratio = float(st.p[0] @ basis / (basis @ basis)) / (vfac * d)
    # density modes of gas and dark matter along x
    c = torch.cos(k * r)
    gas_mode = float(st.q[0][0, 0, :] @ c) / cfg.f_b
    dm_mode = float(gravity.cic_deposit(st.x, 1.0, n)[0, 0, :] @ c)
    transverse = float((st.x[1:] - ics.lattice(n)[1:]).abs().max())
    return disp_ratio, mom_ratio, gas_mode, dm_mode, transverse


@pytest.mark.slow
def test_zeldovich_pancake_before_shell_crossing():
    r32 = _pancake(32, 0.3)
    r64 = _pancake(64, 0.3)
    for r in (r32, r64):
        assert r[4] == 0.0                         # no transverse motion
        assert abs(r[2] / r[3] - 1) < 0.015        # the gas follows the dark matter
    # growth of the mode follows D(a) up to the PM force resolution, which converges at
    # second order in the cell size (CIC window and two-point gradient, ~ k^2)
    e32 = [abs(r32[0] - 1), abs(r32[1] - 1)]
    e64 = [abs(r64[0] - 1), abs(r64[1] - 1)]
    assert e64[0] < 0.012 and e64[1] < 0.015
    assert e32[0] > 2.5 * e64[0] and e32[1] > 2.5 * e64[1]


# ---------------------------------------------------------------- Sedov blast

def test_sedov_blast_radius():
    n, rsh, tf, g = 48, 10.0, 10.0, 5.0 / 3.0
    e0 = (rsh / 1.15) ** 5 / tf ** 2
    q = torch.zeros(5, n, n, n)
    q[0] = 1.0
    q[4] = 1e-6
    c = n // 2
    q[4, c, c, c] += e0
    t, s = 0.0, 0
    while t < tf * (1 - 1e-12):
        dt = min(0.4 / hydro.max_signal_speed(q, 1.0, g, 0.0), tf - t)
        for d in hydro.strang_axes(s):
            q = hydro.sweep(q, d, dt, 1.0, 1.0, g, 0.0)
        t += dt
        s += 1
    rho = q[0].numpy()
    rng = np.random.default_rng(0)
    rr = np.linspace(0, n / 2 - 1, 800)
    peaks = []
    for _ in range(64):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        pts = np.array([c + rr * v[2], c + rr * v[1], c + rr * v[0]])
        peaks.append(rr[np.argmax(map_coordinates(rho, pts, order=1, mode="wrap"))])
    peaks = np.array(peaks)
    exact = 1.15 * (e0 * tf ** 2 / 1.0) ** 0.2      # eq. sedov
    assert abs(peaks.mean() - exact) < 2.0
    assert peaks.std() < 1.0
    # energy is conserved exactly by the flux form
    assert abs(float(q[4].sum()) - (e0 + 1e-6 * n ** 3)) < 1e-9 * e0


# ---------------------------------------------------------------- initial conditions

def test_initial_field_spectrum_and_displacement():
    n = 32
    cfg = sim.default_config(n=n, box=10.0)
    w = torch.from_numpy(philox.white_noise(11, n))
    dk = ics.linear_density(w, cfg)
    kz, ky, kx = gravity.wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    kphys = (torch.sqrt(k2) * n / cfg.box).numpy()
    v_box = cfg.box ** 3
    # measured P(k) = V |delta_k / N^3|^2 against the input spectrum times D^2, shell averages
    pk_meas = (v_box * dk.abs() ** 2 / n ** 6).numpy()
    d2 = cosmology.growth(cfg.a_init, cfg.omega_m) ** 2
    weight = np.ones_like(pk_meas)
    weight[..., 1:n // 2] = 2.0      # rfft half-plane: interior kx modes stand for two
    edges = np.linspace(2 * math.pi / cfg.box, math.pi * n / cfg.box, 8)
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (kphys >= lo) & (kphys < hi)
        nm = weight[sel].sum()
        meas = (pk_meas[sel] * weight[sel]).sum() / nm
        ks = kphys[sel]
        expect = np.sum(weight[sel] * np.array([cosmology.linear_power(kk, cfg.omega_m, cfg.h,
                                                                        cfg.n_s, cfg.amp) for kk in ks])) / nm * d2
        assert abs(meas / expect - 1) < 5.0 / math.sqrt(nm / 2)
    # Zel'dovich displacement: zero mean, curl free and div(Psi) = -delta (spectrally)
    psi = ics.za_displacement(dk, n)
    assert float(psi.mean(dim=(1, 2, 3)).abs().max()) < 1e-14
    pk = torch.fft.rfftn(psi, dim=(-3, -2, -1))
    nyq = (kx.abs() == math.pi) | (ky.abs() == math.pi) | (kz.abs() == math.pi)
    div = 1j * (kx * pk[0] + ky * pk[1] + kz * pk[2])
    ok = ~nyq & (k2 > 0)
    assert torch.allclose(div[ok.expand_as(div)], -dk[ok.expand_as(dk)], atol=1e-12 * float(dk.abs().max()))
    curl_z = (kx * pk[1] - ky * pk[0])[ok.expand_as(div)]
    assert float(curl_z.abs().max()) < 1e-12 * float(pk.abs().max())


def test_initial_state_gas_tracks_dark_matter():
    n = 16
    cfg = sim.default_config(n=n, box=10.0)
    st = sim.initial_state(torch.from_numpy(philox.white_noise(3, n)), cfg)
    assert abs(float(st.q[0].sum()) - cfg.f_b * n ** 3) < 1e-9
    temp = subgrid.temperature(st.q, st.a, cfg.gamma, 0.0, cfg.t_per_e)
    assert torch.allclose(temp, torch.full_like(temp, cfg.t_init), rtol=1e-9)
    # the gas velocity equals the particle velocity on the lattice (both p/a)
    u = st.q[1:4] / (st.a * st.q[0])
    assert torch.allclose(u.reshape(3, -1), st.p / st.a, rtol=1e-12)


# ---------------------------------------------------------------- conservation

def test_full_step_conserves_mass_and_total_momentum():
    n = 16
    cfg = sim.default_config(n=n, box=10.0)
    st = sim.initial_state(torch.from_numpy(philox.white_noise(5, n)), cfg)
    c0 = sim.conservation(st, cfg)
    st, _ = sim.run(st, cfg, sim.Params(), nsteps=6)
    c1 = sim.conservation(st, cfg)
    assert abs(c1[0] - c0[0]) < 1e-12 * c0[0]
    for d in range(3):
        tot0, tot1 = c0[1 + d] + c0[5 + d], c1[1 + d] + c1[5 + d]
        assert abs(tot1 - tot0) < 1e-12 * (abs(c0[1 + d]) + abs(c1[5 + d]) + 1e-30) + 1e-15


# ---------------------------------------------------------------- subgrid

def test_unit_conversions_against_si_constants():
    # sound speed of gas at 1e4 K with mu = 0.6: sqrt(gamma k T / (mu m_p)) ~ 15.1 km/s
    tpe = subgrid.kelvin_per_code_energy(5 / 3, 0.6, 1.0)   # code velocity unit = 1 km/s
    e = 1e4 / tpe
    cs = math.sqrt(5 / 3 * 2 / 3 * e)
    assert abs(cs - 15.15) < 0.05
    # free-fall time from G and the critical density in SI units
    g_si, mpc = 6.67430e-11, 3.0856775814913673e22
    h, om_b, a, delta = 0.7, 0.05, 0.2, 150.0
    h0 = 100 * h * 1e3 / mpc
    rho_prop = om_b * 3 * h0 ** 2 / (8 * math.pi * g_si) * delta / a ** 3
    tff = math.sqrt(3 * math.pi / (32 * g_si * rho_prop)) * h0
    got = float(subgrid.free_fall_time(torch.tensor(delta), a, om_b))
    assert abs(got / tff - 1) < 1e-12


def _uniform_gas(n, a, delta, temp_k, cfg):
    rho = torch.full((n, n, n), cfg.f_b * delta)
    e = temp_k / cfg.t_per_e
    return torch.stack([rho, 0 * rho, 0 * rho, 0 * rho, a * a * rho * e])


def test_hard_draw_is_binomial_with_probability_pi0():
    n = 32
    cfg = sim.default_config(n=n, box=10.0)
    a, dt = 0.2, 0.02
    q = _uniform_gas(n, a, 300.0, 1e3, cfg)
    u = torch.from_numpy(philox.starform_uniform(9, 4, n))
    kw = dict(rho_mean_gas=cfg.f_b, omega_b=cfg.omega_b, gamma=cfg.gamma, e_floor=cfg.e_floor,
              t_per_e=cfg.t_per_e, e0_code=0.03e6 / cfg.vel_unit ** 2, eps_sf=0.5,
              delta_c=100.0, t_c=10 ** 4.5, w_rho=0.1, w_t=0.1, tau=0.1)
    q1, star = subgrid.apply_source(q, torch.zeros(n, n, n), a, dt, u, mode=subgrid.MODE_HARD, **kw)
    tff = 0.5 * math.pi * math.sqrt(a ** 3 / (cfg.omega_b * 300.0))
    pi0 = 1 - math.exp(-0.5 * dt / tff)
    frac = float(star.mean())
    sigma = math.sqrt(pi0 * (1 - pi0) / n ** 3)
    assert 0.05 < pi0 < 0.95 and abs(frac - pi0) < 4 * sigma
    # energy added exactly where stars formed, mass untouched
    de = (q1[4] - q[4]) / (a * a * q[0] * kw["e0_code"])
    assert torch.equal(q1[0], q[0]) and torch.allclose(de, star, atol=1e-12)
    # below the density threshold or above the temperature threshold: nothing forms
    for qq in (_uniform_gas(n, a, 50.0, 1e3, cfg), _uniform_gas(n, a, 300.0, 1e5, cfg)):
        _, st2 = subgrid.apply_source(qq, torch.zeros(n, n, n), a, dt, u, mode=subgrid.MODE_HARD, **kw)
        assert float(st2.sum()) == 0.0


def test_relaxed_draw_limits():
    torch.manual_seed(0)
    u = torch.from_numpy(philox.starform_uniform(5, 0, 64)).reshape(-1)
    for pi0 in (0.1, 0.4, 0.8):
        p = torch.full_like(u, pi0)
        # tau -> 0: the relaxed draw tends to the hard draw with the same u
        z_sharp = subgrid.draw(p, u, 1e-4, subgrid.MODE_RELAXED)
        z_hard = subgrid.draw(p, u, None, subgrid.MODE_HARD)
        near = (u - (1 - pi0)).abs() < 1e-3
        assert torch.equal((z_sharp > 0.5)[~near], (z_hard > 0.5)[~near])
        # the mean of the relaxed variable approaches pi0 as tau -> 0
        z = subgrid.draw(p, u, 0.02, subgrid.MODE_RELAXED)
        assert abs(float(z.mean()) - pi0) < 4 * math.sqrt(pi0 * (1 - pi0) / u.numel()) + 0.01


# ---------------------------------------------------------------- gradient of the oracle

def _loss_of(white, prm_t, cfg, schedule, target):
    prm = sim.Params(A=prm_t[0], beta=prm_t[1], eps_sf=prm_t[2], delta_c=prm_t[3],
                     t_c=1e6, e0=0.03)
    st = sim.initial_state(white, cfg)
    st, _ = sim.run(st, cfg, prm, schedule=schedule)
    return sim.loss(st, target, cfg, prm.A, prm.beta)


def test_oracle_gradient_matches_central_differences():
    n = 8
    cfg = sim.default_config(n=n, box=4.0, subgrid=subgrid.MODE_RELAXED, a_init=0.05)
    white = torch.from_numpy(philox.white_noise(21, n))
    base = torch.tensor([0.3, 1.6, 0.5, 1.05])
    st0 = sim.initial_state(white, cfg)
    _, schedule = sim.run(st0, cfg, sim.Params(), nsteps=3)
    target = torch.from_numpy(np.random.default_rng(1).uniform(0.2, 0.9, size=(n, n, n)))

    w = white.clone().requires_grad_(True)
    pt = base.clone().requires_grad_(True)
    val = _loss_of(w, [pt[0], pt[1], pt[2], pt[3]], cfg, schedule, target)
    gw, gp = torch.autograd.grad(val, (w, pt))
    assert float(gp.abs().min()) > 0.0      # every parameter reaches the loss

    v = torch.from_numpy(np.random.default_rng(2).normal(size=(n, n, n)))
    v /= v.norm()
    with torch.no_grad():
        # small steps: lattice particles start on the kinks of the CIC kernel, and a larger
        # step would average the derivative across a kink
        ref = float((gw * v).sum())
        for hstep in (2e-5, 1e-5):
            fd = (_loss_of(white + hstep * v, base, cfg, schedule, target)
                  - _loss_of(white - hstep * v, base, cfg, schedule, target)) / (2 * hstep)
            assert abs(float(fd) - ref) < 1e-6 * abs(ref)
        for i in range(4):
            hstep = 1e-5 * max(1.0, abs(float(base[i])))
            e = torch.zeros(4)
            e[i] = hstep
            fd = (_loss_of(white, base + e, cfg, schedule, target)
                  - _loss_of(white, base - e, cfg, schedule, target)) / (2 * hstep)
            assert abs(float(fd) - float(gp[i])) < 1e-5 * abs(float(gp[i])) + 1e-12

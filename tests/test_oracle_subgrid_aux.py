"""Pins of the oracle's supernova-injection and star-association options (Sec. 2.4.1): the
smoothed injection is a symmetric, total-preserving smoothing whose plane waves are
eigenfunctions with the closed-form factor cos^2(pi k / n) per axis; the stars' read-out on
the particles is the CIC interpolation of the step's new stars (a partition of unity, and the
cell's own value at a cell centre)."""

import math

import numpy as np
import torch

import synth_inputs as si
from oracle import gravity, ics, philox, sim as osim, subgrid

torch.set_default_dtype(torch.float64)


def test_smoothing_plane_waves_have_the_closed_form_factor():
    n = 16
    idx = torch.arange(n, dtype=torch.float64)
    for kz, ky, kx in ((0, 0, 1), (0, 3, 0), (5, 0, 0), (2, 7, 4), (8, 8, 8)):
        f = (torch.cos(2 * math.pi * kz * idx / n)[:, None, None]
             * torch.cos(2 * math.pi * ky * idx / n)[None, :, None]
             * torch.cos(2 * math.pi * kx * idx / n)[None, None, :])
        factor = 1.0
        for k in (kz, ky, kx):
            factor *= math.cos(math.pi * k / n) ** 2
        got = subgrid.smooth_injection(f)
        assert torch.allclose(got, factor * f, rtol=0, atol=1e-14), (kz, ky, kx)


def test_smoothing_preserves_totals_and_is_symmetric():
    n = 12
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.standard_normal((n, n, n)))
    b = torch.from_numpy(rng.standard_normal((n, n, n)))
    wa = subgrid.smooth_injection(a)
    assert abs(float(wa.sum() - a.sum())) < 1e-12
    assert abs(float((wa * b).sum() - (a * subgrid.smooth_injection(b)).sum())) < 1e-12
    c = torch.full((n, n, n), 2.5)
    assert torch.allclose(subgrid.smooth_injection(c), c, rtol=0, atol=1e-15)
    # a single source spreads over exactly its 27 cells, all positive
    d = torch.zeros(n, n, n)
    d[5, 6, 7] = 1.0
    w = subgrid.smooth_injection(d)
    assert int((w > 0).sum()) == 27 and float(w.max()) == float(w[5, 6, 7])


def _source(q, smooth, u, n):
    cfg = osim.default_config(n=n, subgrid=subgrid.MODE_RELAXED)
    return subgrid.apply_source(
        q, torch.zeros(n, n, n), 0.2, 0.01, u, rho_mean_gas=cfg.f_b, omega_b=cfg.omega_b,
        gamma=cfg.gamma, e_floor=cfg.e_floor, t_per_e=cfg.t_per_e, e0_code=3.0, eps_sf=0.5,
        delta_c=1.0, t_c=1e9, w_rho=0.1, w_t=0.1, tau=0.1, mode=subgrid.MODE_RELAXED,
        smooth=smooth, with_draw=True)


def test_smoothed_injection_moves_energy_but_keeps_its_total():
    n = 16
    q = torch.from_numpy(si.smooth_gas_state(n, 0.2, seed=4, energy=0.6))
    u = torch.from_numpy(philox.starform_uniform(102, 3, n))
    q0, s0, z0 = _source(q, False, u, n)
    q1, s1, z1 = _source(q, True, u, n)
    assert torch.equal(z0, z1) and torch.equal(s0, s1) and float(z0.sum()) > 1.0
    assert torch.equal(q0[:4], q1[:4])
    assert abs(float(q1[4].sum() - q0[4].sum())) < 1e-11 * float(q0[4].sum())
    assert float((q1[4] - q0[4]).abs().max()) > 1e-3 * float((q0[4] - q[4]).abs().max())


def test_star_readout_is_a_partition_of_unity_and_exact_at_cell_centres():
    n = 8
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.uniform(0, n, (3, 50)))
    c = torch.full((n, n, n), 0.37)
    assert torch.allclose(gravity.cic_readout(c, x), torch.full((50,), 0.37), rtol=0,
                          atol=1e-15)
    z = torch.from_numpy(rng.uniform(0, 1, (n, n, n)))
    lat = ics.lattice(n)
    assert torch.allclose(gravity.cic_readout(z, lat), z.reshape(-1), rtol=0, atol=1e-15)


def test_step_keeps_the_new_stars_on_the_particles():
    """Two steps with the read-out on: the auxiliary field is the sum of the two steps' new
    stars interpolated at the end-of-step positions, and nothing else in the state moves."""
    n = 16
    kw = dict(n=n, box=4.0, a_init=0.05, subgrid=subgrid.MODE_RELAXED)
    prm = osim.Params(delta_c=1.05, t_c=1e6, eps_sf=0.5)
    w = torch.from_numpy(si.white_noise(n, seed=21)).double()
    base = osim.default_config(**kw)
    cfg = osim.default_config(star_dm=True, **kw)
    st_b = osim.initial_state(w, base)
    st_a = osim.initial_state(w, cfg)
    expect = torch.zeros(n ** 3)
    for _ in range(2):
        dt = osim.cfl_dt(st_b, base)
        star_before = st_b.star
        st_b = osim.step(st_b, base, prm, dt)
        st_a = osim.step(st_a, cfg, prm, dt)
        expect = expect + gravity.cic_readout(st_b.star - star_before, st_b.x)
    assert st_b.aux is None
    assert torch.equal(st_a.q, st_b.q) and torch.equal(st_a.x, st_b.x)
    assert torch.equal(st_a.star, st_b.star)
    assert float(st_a.star.sum()) > 0.1
    assert torch.allclose(st_a.aux, expect, rtol=1e-12, atol=1e-14)

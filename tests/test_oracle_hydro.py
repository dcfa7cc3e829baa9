"""Pins of the oracle's relaxing-TVD hydro sweep: exact Sod solution (at a = 1 and at a
fixed a != 1, where the comoving system reduces to the Euler equations in t/a), exact
conservation, fixed points and axis-permutation symmetry.  CPU only."""

import math

import numpy as np
import pytest
import torch

from oracle import hydro, riemann

torch.set_default_dtype(torch.float64)

GAMMA_SOD = 1.4
LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def _sod_initial(n, axis, a, gamma):
    """Periodic tube with the high state in the middle half: a Sod interface at 3n/4 and a
    mirrored one at n/4."""
    xc = np.arange(n) + 0.5
    hi = (xc >= n / 4) & (xc < 3 * n / 4)
    rho = np.where(hi, LEFT[0], RIGHT[0])
    p = np.where(hi, LEFT[2], RIGHT[2])
    shape = [1, 1, 1]
    shape[2 - axis] = n
    q = np.zeros((5,) + tuple(shape))
    q[0] = rho.reshape(shape)
    q[4] = (a * a * p / (gamma - 1.0)).reshape(shape)
    return torch.from_numpy(q)


def _run_sod(n, axis, a, t_final, cfl=0.4, gamma=GAMMA_SOD):
    q = _sod_initial(n, axis, a, gamma)
    t = 0.0
    t_end = a * t_final          # comoving time runs as t/a at fixed a
    while t < t_end * (1 - 1e-14):
        dt = min(cfl / hydro.max_signal_speed(q, a, gamma, 0.0), t_end - t)
        q = hydro.sweep(q, axis, dt, a, a, gamma, 0.0)
        t += dt
    return q.reshape(5, n).numpy()


@pytest.mark.parametrize("axis,a", [(0, 1.0), (1, 1.0), (2, 1.0), (0, 0.5)])
def test_sod_against_exact_solution(axis, a):
    n = 256
    t_final = n / 14.0
    q = _run_sod(n, axis, a, t_final)
    rho = q[0]
    xc = np.arange(n) + 0.5
    sel = xc >= n / 2
    ex_rho, ex_u, ex_p = riemann.profile(xc[sel], t_final, 0.75 * n, LEFT, RIGHT, GAMMA_SOD)
    # no growing oscillations: total variation within 5% of the exact solution's (the
    # componentwise relaxing scheme leaves sub-percent wiggles behind the shock)
    tv = np.abs(np.diff(rho[sel])).sum()
    assert tv <= 1.05 * np.abs(np.diff(ex_rho)).sum()
    # positions of the shock and the contact within 2 cells of the exact ones
    ps, us = riemann.star_state(LEFT, RIGHT, GAMMA_SOD)
    rs = riemann.sample(us + 1e-9, LEFT, RIGHT, GAMMA_SOD)[0]
    rl = riemann.sample(us - 1e-9, LEFT, RIGHT, GAMMA_SOD)[0]
    x_contact = 0.75 * n + us * t_final
    shock_speed = us * rs / (rs - RIGHT[0])   # mass flux balance across the shock
    x_shock = 0.75 * n + shock_speed * t_final

    def crossing(level, lo, hi):
        idx = np.where((xc > lo) & (xc < hi))[0]
        for i in idx[:-1]:
            if (rho[i] - level) * (rho[i + 1] - level) <= 0:
                return xc[i] + (level - rho[i]) / (rho[i + 1] - rho[i])
        return None

    xs = crossing(0.5 * (rs + RIGHT[0]), x_contact + 2, n)
    xcn = crossing(0.5 * (rl + rs), x_contact - 12, x_contact + 12)
    assert xs is not None and abs(xs - x_shock) < 2.0
    assert xcn is not None and abs(xcn - x_contact) < 2.0
    # momentum and pressure profiles close in L1
    u = q[1 + axis][sel] / (a * rho[sel])
    l1_u = np.mean(np.abs(u - ex_u))
    assert l1_u < 0.03
    assert np.mean(np.abs(rho[sel] - ex_rho)) < 0.02


def test_sod_error_decreases_with_resolution():
    errs = []
    for n in (64, 128, 256):
        t_final = n / 14.0
        q = _run_sod(n, 0, 1.0, t_final)
        xc = np.arange(n) + 0.5
        sel = xc >= n / 2
        ex_rho, _, _ = riemann.profile(xc[sel], t_final, 0.75 * n, LEFT, RIGHT, GAMMA_SOD)
        # error measured in units of the box: L1 over the fraction of the box
        errs.append(np.mean(np.abs(q[0][sel] - ex_rho)))
    # the same physical problem on finer grids: error per unit length must shrink
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


def _random_state(n, a, seed, amp=0.2):
    g = torch.Generator().manual_seed(seed)
    r = torch.arange(n, dtype=torch.float64)
    z, y, x = torch.meshgrid(r, r, r, indexing="ij")
    smooth = lambda ph: (torch.sin(2 * math.pi * (x + 2 * y) / n + ph) +
                         torch.cos(2 * math.pi * (3 * z - y) / n + ph))
    rho = 1.0 + amp * smooth(0.3) + 0.05 * torch.rand(n, n, n, generator=g)
    u = torch.stack([0.5 * smooth(1.0), -0.3 * smooth(2.0), 0.4 * smooth(0.5)])
    e = 0.8 + amp * smooth(1.7)
    q = torch.cat([rho[None], a * rho * u, (a * a * rho * (e + 0.5 * (u * u).sum(0)))[None]])
    return q


def test_sweeps_conserve_mass_momentum_energy():
    a = 0.3
    q = _random_state(12, a, 1)
    s0 = q.sum(dim=(1, 2, 3))
    for d in (0, 1, 2):
        q = hydro.sweep(q, d, 0.05, a, a * 1.01, 5 / 3, 1e-6)
    s1 = q.sum(dim=(1, 2, 3))
    assert torch.allclose(s0, s1, rtol=1e-12, atol=1e-11)


def test_uniform_state_is_fixed_point():
    a = 0.7
    n = 8
    q = torch.zeros(5, n, n, n)
    q[0] = 2.0
    q[1] = a * 2.0 * 0.3
    q[2] = -a * 2.0 * 0.1
    q[4] = a * a * 2.0 * (1.5 + 0.5 * (0.09 + 0.01))
    for d in (0, 1, 2):
        out = hydro.sweep(q, d, 0.1, a, a, 5 / 3, 1e-6)
        assert torch.equal(out, q)


def test_axis_permutation_symmetry():
    a = 0.4
    q = _random_state(10, a, 2)
    # swap x and y: transpose the grid and swap the two momentum components
    perm = lambda s: torch.stack([s[0].transpose(-1, -2), s[2].transpose(-1, -2),
                                  s[1].transpose(-1, -2), s[3].transpose(-1, -2),
                                  s[4].transpose(-1, -2)])
    out_a = hydro.sweep(hydro.sweep(q, 0, 0.03, a, a, 5 / 3, 1e-6), 1, 0.03, a, a, 5 / 3, 1e-6)
    out_b = hydro.sweep(hydro.sweep(perm(q), 1, 0.03, a, a, 5 / 3, 1e-6), 0, 0.03, a, a, 5 / 3, 1e-6)
    assert torch.allclose(perm(out_a), out_b, rtol=0, atol=1e-13)


def test_strang_cycle_order():
    names = ["".join("XYZ"[d] for d in hydro.strang_axes(s)) for s in range(6)]
    assert "".join(names) == "XYZZYXZXYYXZYZXXZY"
    assert hydro.strang_axes(6) == hydro.strang_axes(0)


def test_sweep_with_fixed_branches():
    """The optional fixed choices of sweep() (used by derivative checks at kinks): with its
    own decisions the sweep is unchanged; a flipped limiter branch or |U_d| sign changes the
    value only by what that branch contributes at the point, which vanishes at the kink."""
    a, dt = 0.3, 0.04
    q = _random_state(8, a, 5)
    k = hydro.sweep_kinks(q, 1, dt, a, a, 5 / 3, 1e-6)
    one = lambda v: torch.where(v >= 0, torch.ones_like(v), -torch.ones_like(v))
    br = {"sign1": one(k["u1"][0]), "sign2": one(k["u2"][0]),
          "take_r": k["x_r"][0] * k["y_r"][0] > 0, "take_l": k["x_l"][0] * k["y_l"][0] > 0}
    base = hydro.sweep(q, 1, dt, a, a, 5 / 3, 1e-6)
    assert torch.allclose(hydro.sweep(q, 1, dt, a, a, 5 / 3, 1e-6, branches=br), base,
                          rtol=0, atol=1e-15)
    # every limiter branch switched on where the slopes disagree in sign: the flux gains the
    # harmonic mean of opposite-signed slopes, a change of the value
    br2 = dict(br, take_r=torch.ones_like(br["take_r"]))
    assert not torch.allclose(hydro.sweep(q, 1, dt, a, a, 5 / 3, 1e-6, branches=br2), base)
    # at an exact kink (a zero slope), either branch gives the same value
    x = torch.tensor([0.0, 0.3, -0.2])
    y = torch.tensor([0.7, 0.0, 0.0])
    assert torch.equal(hydro.van_leer(x, y, take=torch.tensor([True, True, True])),
                       hydro.van_leer(x, y, take=torch.tensor([False, False, False])))
    # the half weight at an exact zero slope: the same value, and the derivative of the
    # |x y| form there (sign(0) = 0), the mean of the two one-sided derivatives
    x = torch.tensor([0.0, 0.3], requires_grad=True)
    y = torch.tensor([0.7, 0.0], requires_grad=True)
    grads = []
    for take in (None, torch.tensor([0.5, 0.5]), torch.tensor([1.0, 1.0]),
                 torch.tensor([0.0, 0.0])):
        v = hydro.van_leer(x, y, take=take)
        assert torch.equal(v.detach(), torch.zeros(2))
        grads.append(torch.cat(torch.autograd.grad(v.sum(), (x, y))))
    assert torch.allclose(grads[0], grads[1], rtol=0, atol=1e-15)
    assert torch.allclose(grads[1], 0.5 * (grads[2] + grads[3]), rtol=0, atol=1e-15)
    assert torch.allclose(grads[2], torch.tensor([2.0, 0.0, 0.0, 2.0]), rtol=0, atol=1e-12)
    # |U_d| with the sign fixed to that of U_d is |U_d|
    f0, c0 = hydro.flux_and_speed(q, a, 2, 5 / 3, 1e-6)
    f1, c1 = hydro.flux_and_speed(q, a, 2, 5 / 3, 1e-6, sign_ud=one(q[3]))
    assert torch.equal(f0, f1) and torch.allclose(c0, c1, rtol=1e-15, atol=0)

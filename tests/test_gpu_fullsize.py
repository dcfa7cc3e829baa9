"""Parity at the benchmarked size: 256^3 cells and particles, in the launch configurations the
bench times (the same kernels, tiles and segments as a 256^3 run).

* one whole step of the bench workload (40 Mpc/h, a = 0.01, relaxed star formation) against
  the FP64 oracle's step from the same initial conditions;
* the three sweeps and their adjoints on sampled lines: a sweep along one axis acts on each
  line independently, so the oracle recomputes a sampled line on its own (the adjoint by
  autograd of that line);
* the CIC deposit and the Poisson solve over the whole field.

Each test prints what it runs before it runs it."""

import math

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_helpers import (displacement_err, gpu_config, gpu_params, rel_l2,
                         sweep_vjp_on_gpu_branches, to_gpu, to_np)
from oracle import gravity, hydro, ics, sim as osim, subgrid

pytestmark = pytest.mark.gpu
torch.set_default_dtype(torch.float64)

N = 256
STEP_TOL = 1e-5
# one 256-cell line of a sweep adjoint: each cell sums about sixty float32 products whose
# terms reach ten times the result (differences of limiter derivatives and of adjacent
# adjoints), so a line's relative L2 scatters around 1e-5 where a whole 128^3 field averages
# to below it
LINE_VJP_TOL = 3e-5


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


def _say(msg):
    print(msg, flush=True)


def _line(q, axis, i, j):
    """The line along `axis` through the two other indices (i, j) of a [5][z][y][x] field,
    shaped so that the oracle sweeps it along the same axis."""
    if axis == 0:
        return q[:, i:i + 1, j:j + 1, :]
    if axis == 1:
        return q[:, i:i + 1, :, j:j + 1]
    return q[:, :, i:i + 1, j:j + 1]


LINES = [(0, 0), (3, 255), (128, 17), (200, 101), (255, 254), (77, 190)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_256_sampled_lines(dhp, axis):
    _say(f"sweep 256^3 axis {axis}")
    ocfg = osim.default_config(n=N)
    s = dhp.Sim(gpu_config(ocfg), gpu_params(osim.Params()))
    a0, ah, dt = 0.3, 0.31, 0.04
    q = si.smooth_gas_state(N, a0, seed=40 + axis, energy=0.6)
    out = to_np(s.stage_sweep(to_gpu(q), axis, dt, a0, ah))
    qt = torch.from_numpy(q)
    for i, j in LINES:
        ref = hydro.sweep(_line(qt, axis, i, j).double(), axis, dt, a0, ah, ocfg.gamma,
                          ocfg.e_floor).numpy()
        got = _line(out, axis, i, j)
        for c in range(5):
            assert rel_l2(got[c], ref[c]) < STEP_TOL, (i, j, c, rel_l2(got[c], ref[c]))
    s.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_vjp_256_sampled_lines(dhp, axis):
    """Every cell of the sampled lines against the oracle's exact derivative of the line,
    taken, where a limiter slope or U_d lies within rounding of its kink, on the side the GPU
    took (both sides are exact one-sided derivatives)."""
    _say(f"sweep adjoint 256^3 axis {axis}")
    ocfg = osim.default_config(n=N)
    s = dhp.Sim(gpu_config(ocfg), gpu_params(osim.Params()))
    a0, ah, dt = 0.3, 0.31, 0.04
    q = si.smooth_gas_state(N, a0, seed=50 + axis, energy=0.6)
    lam = si.random_field((5, N, N, N), seed=60 + axis)
    out = to_np(s.stage_sweep_vjp(to_gpu(q), to_gpu(lam), axis, dt, a0, ah))
    # the sampled lines side by side: one field of independent lines along the axis
    d = 2 if axis == 0 else 3
    stack = lambda f: np.concatenate([_line(f, axis, i, j) for i, j in LINES], axis=d)
    got = stack(out)
    ref, nl, kinks = sweep_vjp_on_gpu_branches(stack(q), stack(lam), got, axis, dt, a0, ah,
                                               ocfg.gamma, ocfg.e_floor)
    _say(f"  {kinks} choices near a kink on {nl} of {len(LINES)} lines")
    assert np.isfinite(got).all()
    for k in range(len(LINES)):
        sl = [slice(None)] * 4
        sl[d] = slice(k, k + 1)
        gk, rk = got[tuple(sl)], ref[tuple(sl)]
        for c in range(5):
            err = rel_l2(gk[c], rk[c])
            assert err < LINE_VJP_TOL, (LINES[k], c, err)
            elem = np.abs(gk[c] - rk[c]).max() / np.abs(rk[c]).max()
            assert elem < 1e-3, (LINES[k], c, elem)
    s.close()


def test_deposit_256(dhp):
    _say("deposit 256^3")
    ocfg = osim.default_config(n=N)
    s = dhp.Sim(gpu_config(ocfg), gpu_params(osim.Params()))
    pos = si.random_positions(N, seed=70)
    rho = (0.2 + 0.01 * si.random_field((N, N, N), seed=71)).astype(np.float32)
    a = s.stage_deposit(to_gpu(rho), to_gpu(pos))
    b = s.stage_deposit(to_gpu(rho), to_gpu(pos))
    assert torch.equal(a, b)
    ref = gravity.total_overdensity(torch.from_numpy(rho).double(), torch.from_numpy(pos).double(),
                                    1.0 - ocfg.f_b, N).numpy()
    assert rel_l2(to_np(a) + 1.0, ref + 1.0) < STEP_TOL
    s.close()


def test_poisson_256(dhp):
    _say("poisson 256^3")
    ocfg = osim.default_config(n=N)
    s = dhp.Sim(gpu_config(ocfg), gpu_params(osim.Params()))
    delta = si.random_field((N, N, N), seed=72)
    out = to_np(s.stage_poisson(to_gpu(delta), 0.2))
    ref = gravity.poisson(torch.from_numpy(delta).double(), 0.2, ocfg.omega_m).numpy()
    assert rel_l2(out, ref) < STEP_TOL
    # closed form of one mode along z at this size
    r = np.arange(N)
    k = 2 * math.pi * 5 / N
    wave = np.broadcast_to(np.sin(k * r).reshape(N, 1, 1), (N, N, N)).astype(np.float32)
    out = to_np(s.stage_poisson(to_gpu(wave), 0.5))
    assert rel_l2(out, -(1.5 * ocfg.omega_m / 0.5) * wave / k ** 2) < 1e-5
    s.close()


def _step_256(dhp, prm, label):
    """One step of the 256^3 / 40 Mpc/h workload from its initial conditions (white-noise
    seed 6) on the GPU and in the oracle, with the star-formation parameters prm; the
    relative L2 of every field, and every element within 10 times the bar of its field's
    largest value."""
    _say(f"{label} 256^3: oracle initial conditions")
    ocfg = osim.default_config(n=N, box=40.0, a_init=0.01, subgrid=subgrid.MODE_RELAXED)
    w = si.white_noise(N, 6)
    st = osim.initial_state(torch.from_numpy(w).double(), ocfg)
    dt = osim.cfl_dt(st, ocfg)
    _say(f"{label} 256^3: GPU step")
    s = dhp.Sim(gpu_config(ocfg), gpu_params(prm))
    s.init_from_noise(to_gpu(w))
    s.set_schedule([dt])
    s.step()
    _say(f"{label} 256^3: oracle step")
    with torch.no_grad():
        ref = osim.step(st, ocfg, prm, dt)
    q = to_np(s.get("q"))
    fields = {f"q{c}": (q[c], ref.q[c].numpy()) for c in range(5)}
    fields["mom"] = (to_np(s.get("mom")), ref.p.numpy())
    fields["phi"] = (to_np(s.get("phi")), ref.phi.numpy())
    fields["star"] = (to_np(s.get("star")), ref.star.numpy())
    errs = {k: rel_l2(g, r) for k, (g, r) in fields.items()}
    elem = {k: float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-30))
            for k, (g, r) in fields.items()}
    lat = ics.lattice(N).numpy()
    disp = ((ref.x.numpy() - lat) + N / 2) % N - N / 2
    scale = np.linalg.norm(disp)
    got_x = to_np(s.get("pos"))
    errs["pos"] = displacement_err(got_x, ref.x.numpy(), N, scale)
    elem["pos"] = float(np.abs((got_x - ref.x.numpy() + N / 2) % N - N / 2).max()
                        / np.abs(disp).max())
    stars = float(ref.star.sum())
    _say(f"{label} 256^3: stars {stars:.4g}; rel-L2 / per-element "
         + str({k: f"{errs[k]:.2e}/{elem[k]:.2e}" for k in errs}))
    # positions are absolute float32 coordinates up to 256, resolved to 2^-16: rounding alone
    # leaves an error of about 2^-16 / sqrt(12) per coordinate, which the displacement norm
    # (sub-cell at a = 0.01) turns into a relative error of a few 1e-6 .. 1e-5; per element,
    # one rounding of a coordinate (2^-16 at 256) against the largest displacement
    pos_floor = 2.0 ** -16 * math.sqrt(3 * N ** 3 / 12.0) / scale
    tol = {k: (max(STEP_TOL, 4 * pos_floor) if k == "pos" else STEP_TOL) for k in errs}
    etol = {k: 10 * tol[k] for k in errs}
    etol["pos"] = max(10 * STEP_TOL, 2 * 2.0 ** -16 / np.abs(disp).max())
    if stars == 0.0:
        del errs["star"], elem["star"]
    bad = {k: (v, tol[k]) for k, v in errs.items() if not v < tol[k]}
    assert not bad, bad
    bad = {k: (v, etol[k]) for k, v in elem.items() if not v < etol[k]}
    assert not bad, ("per element", bad)
    s.close()
    return stars


def test_bench_step_256_matches_oracle(dhp):
    """One step of the bench workload (default star-formation thresholds, which no cell of
    the early field reaches)."""
    _step_256(dhp, osim.Params(), "bench step")


def test_step_256_with_active_source_term_matches_oracle(dhp):
    """The same step with thresholds every cell of the early field passes (Delta_c = 0.5,
    T_c = 1e6 K) and eps_sf = 5: the FP64 source term acts in every cell (stars form in a few
    percent of them).  The gates are saturated there, so the draw's sensitivity to rounding
    of the state is that of the relaxed draw itself (1/tau times d logit pi0 / d ln Delta,
    about 5); with the density threshold at the typical density the gate's slope 1/w_rho
    would multiply it by another 10."""
    stars = _step_256(dhp, osim.Params(delta_c=0.5, t_c=1e6, eps_sf=5.0), "active source")
    assert stars > 1000.0

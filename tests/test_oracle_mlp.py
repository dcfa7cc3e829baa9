"""Pins of the FP64 oracle of the learned closure (oracle.mlp): a loop-by-loop evaluation of
the network on a few samples, bfloat16 rounding on exactly known cases, finite differences of
the objective's gradient in weights and inputs, the closed-form gradient of the output bias,
closed forms of the two targets, and the reduction of the closure to the plain relaxed source
term when the network returns the targets exactly.  CPU only."""

import math

import numpy as np
import pytest
import torch

from oracle import hydro, mlp, philox, sim, subgrid

torch.set_default_dtype(torch.float64)


def _theta(seed=3):
    return torch.from_numpy(mlp.init_params(seed))


def _inputs(count, seed=5):
    return torch.from_numpy(np.random.default_rng(seed).uniform(-1.0, 1.0, (mlp.N_IN, count)))


def _loop_forward(theta, xs):
    """Network evaluated with scalar Python loops, one sample at a time."""
    th = theta.tolist()
    out = []
    for s in range(len(xs[0])):
        h = [xs[i][s] for i in range(mlp.N_IN)]
        k = 0
        for n_in, n_out, act in ((mlp.N_IN, mlp.N_HID, True), (mlp.N_HID, mlp.N_HID, True),
                                 (mlp.N_HID, mlp.N_HID, True), (mlp.N_HID, mlp.N_OUT, False)):
            w = th[k:k + n_out * n_in]
            b = th[k + n_out * n_in:k + n_out * n_in + n_out]
            k += n_out * n_in + n_out
            z = []
            for o in range(n_out):
                acc = b[o]
                for i in range(n_in):
                    acc += w[o * n_in + i] * h[i]
                z.append(acc / (1.0 + math.exp(-acc)) if act else acc * mlp.OUT_SCALE)
            h = z
        out.append(h)
    return out


def test_parameter_count_and_bounds():
    assert mlp.N_PARAMS == 8834
    th = mlp.init_params(1)
    assert th.shape == (8834,)
    parts = mlp.unpack(torch.from_numpy(th))
    for p, f in zip(parts, mlp.FAN_IN):
        assert float(p.abs().max()) <= 1.0 / math.sqrt(f)


def test_forward_matches_scalar_loops():
    th = _theta()
    x = _inputs(4)
    ref = _loop_forward(th, x.tolist())
    got = mlp.forward(th, x)
    for s in range(4):
        for k in range(2):
            assert got[k, s].item() == pytest.approx(ref[s][k], rel=1e-12, abs=1e-12)


def test_bf16_rounding_known_values():
    one = 1.0
    ulp = 2.0 ** -7                      # spacing of bfloat16 in [1, 2)
    cases = [(one, one), (one + ulp / 2, one),                 # tie: to the even neighbour
             (one + 1.5 * ulp, one + 2 * ulp),                # tie: to the even neighbour
             (one + ulp / 2 + ulp / 8, one + ulp),            # above the tie
             (-3.0 - ulp, -3.0), (2.0 ** -130, 2.0 ** -130)]  # subnormal kept
    x = torch.tensor([c[0] for c in cases])
    want = torch.tensor([c[1] for c in cases])
    assert torch.equal(mlp.bf16_round(x), want)


def test_bf16_rounding_passes_gradients_unchanged():
    t = torch.tensor([1.0 + 2.0 ** -9, -0.3, 7.7], requires_grad=True)
    g = torch.tensor([1.0 + 2.0 ** -10, 0.123456789, -5.0])
    out = mlp.bf16_round(t)
    assert torch.equal(out.detach(), mlp.bf16_round(t.detach()))
    gt, = torch.autograd.grad(out, t, grad_outputs=g)
    assert torch.equal(gt, g)


def test_bf16_forward_differs_from_fp64_by_rounding_only():
    th = _theta()
    x = _inputs(256)
    o64 = mlp.forward(th, x)
    o16 = mlp.forward(th, x, bf16=True)
    rel = float((o16 - o64).norm() / o64.norm())
    assert 1e-5 < rel < 2e-2


def test_objective_gradient_by_finite_differences():
    th = _theta().requires_grad_(True)
    x = _inputs(16).requires_grad_(True)
    t = torch.from_numpy(np.random.default_rng(9).normal(size=(2, 16)))
    L = mlp.loss(th, x, t)
    gth, gx = torch.autograd.grad(L, (th, x))
    rng = np.random.default_rng(11)
    for _ in range(3):
        v = torch.from_numpy(rng.normal(size=th.shape))
        w = torch.from_numpy(rng.normal(size=x.shape))
        h = 1e-5
        with torch.no_grad():
            fd_t = (mlp.loss(th + h * v, x, t) - mlp.loss(th - h * v, x, t)) / (2 * h)
            fd_x = (mlp.loss(th, x + h * w, t) - mlp.loss(th, x - h * w, t)) / (2 * h)
        assert float(gth @ v) == pytest.approx(float(fd_t), rel=1e-7)
        assert float((gx * w).sum()) == pytest.approx(float(fd_x), rel=1e-7)


def test_backward_rounding_operators():
    g = torch.tensor([1.0 + 2.0 ** -8, -3.0 - 2.0 ** -7, 0.1])
    z = torch.tensor([0.3, -2.0, 5.0], requires_grad=True)
    out = mlp._RoundGrad.apply(z)
    assert torch.equal(out, z)
    gz, = torch.autograd.grad(out, z, grad_outputs=g)
    assert torch.equal(gz, mlp.bf16_round(g))
    out = mlp._SiluBf16Grad.apply(z)
    assert torch.allclose(out, z * torch.sigmoid(z), rtol=1e-15)
    gz, = torch.autograd.grad(out, z, grad_outputs=torch.ones(3))
    with torch.no_grad():
        h = 1e-6
        fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert torch.allclose(gz, fd, rtol=2.0 ** -8)           # within one bfloat16 rounding
    assert torch.equal(gz, mlp.bf16_round(gz))              # and exactly a bfloat16 value


def test_bf16_gradient_differs_from_fp64_by_rounding_only():
    th = _theta().requires_grad_(True)
    x = _inputs(64)
    t = torch.from_numpy(np.random.default_rng(9).normal(size=(2, 64)))
    g64, = torch.autograd.grad(mlp.loss(th, x, t), th)
    g16, = torch.autograd.grad(mlp.loss(th, x, t, bf16=True), th)
    rel = float((g16 - g64).norm() / g64.norm())
    assert 1e-5 < rel < 3e-2


def test_output_bias_gradient_closed_form():
    th = _theta().requires_grad_(True)
    x = _inputs(32)
    t = torch.from_numpy(np.random.default_rng(4).normal(size=(2, 32)))
    g, = torch.autograd.grad(mlp.loss(th, x, t), th)
    with torch.no_grad():
        o = mlp.forward(th, x)
    want = 2.0 * mlp.OUT_SCALE * (o - t).mean(1)
    assert torch.allclose(g[-2:], want, rtol=1e-12, atol=0)


def test_targets_closed_forms():
    om_b, t_c = 0.05, 10 ** 4.5
    delta = torch.tensor([0.3, 1.0, 100.0, 5e3, 100.0])
    temp = torch.tensor([10.0, 1e4, t_c, 1e2, 1e8])
    a, eps, dc = 0.2, 0.02, 100.0
    o = mlp.targets(delta, temp, a, eps, dc, omega_b=om_b, t_c=t_c, w_rho=0.1, w_t=0.1)
    want0 = math.log(eps) + 0.5 * torch.log(om_b * delta) - 1.5 * math.log(a) - math.log(math.pi / 2)
    assert torch.allclose(o[0], want0, rtol=1e-13)
    assert o[1][2].item() == pytest.approx(-2.0 * math.log(2.0), rel=1e-13)   # both gates at 1/2
    y1, y2 = (5e3 - dc) / (0.1 * dc), (t_c - 1e2) / (0.1 * t_c)
    want13 = -math.log1p(math.exp(-y1)) - math.log1p(math.exp(-y2))           # both gates open
    assert o[1][3].item() == pytest.approx(want13, rel=1e-12)
    assert o[1][4].item() == mlp.GATE_CLIP                                    # far too hot


def test_features_round_trip():
    delta = torch.tensor([0.05, 3.0, 2e4])
    temp = torch.tensor([1.0, 5e4, 3e7])
    x = mlp.features(delta, temp, 0.13, 0.027, 61.0)
    d, tt, a, eps, dc = mlp.decode_features(x)
    assert torch.allclose(d, delta, rtol=1e-13) and torch.allclose(tt, temp, rtol=1e-13)
    assert torch.allclose(a, torch.full_like(a, 0.13), rtol=1e-13)
    assert torch.allclose(eps, torch.full_like(a, 0.027), rtol=1e-13)
    assert torch.allclose(dc, torch.full_like(a, 61.0), rtol=1e-13)


def test_probability_matches_plain_source_factors():
    delta = torch.tensor([50.0, 120.0, 400.0])
    temp = torch.tensor([1e3, 2e4, 5e4])
    o = mlp.targets(delta, temp, 0.25, 0.03, 90.0, omega_b=0.05, t_c=10 ** 4.5, w_rho=0.1,
                    w_t=0.1)
    dt = 0.01
    pi_net = mlp.probability(o, dt)
    pi_plain = subgrid.formation_probability(delta, temp, 0.25, dt, 0.05, 0.03, 90.0,
                                             10 ** 4.5, 0.1, 0.1, subgrid.MODE_RELAXED)
    assert torch.allclose(pi_net, pi_plain, rtol=1e-12)


@pytest.mark.parametrize("dual, smooth", [(False, False), (True, False), (True, True)])
def test_exact_outputs_reduce_closure_to_plain_source(dual, smooth):
    """With o = targets, the closure's update is the plain relaxed source term.  Where the
    gate is clipped (below e^-30), both draws are below e^-130 (the logistic noise of a 24-bit
    uniform stays within +-17), which the star-field tolerance absorbs.  With a dual-energy
    state (a quarter of the cells so cold against their bulk motion that the entropy gives
    their temperature) the entropy takes the injected energy alike, also when it is smoothed."""
    cfg = sim.default_config(n=8, box=2.0, subgrid=subgrid.MODE_RELAXED)
    prm = sim.Params(eps_sf=0.5, delta_c=2.0, t_c=1e5)
    rng = np.random.default_rng(2)
    n = cfg.n
    rho = torch.from_numpy(cfg.f_b * np.exp(rng.normal(0, 1.2, (n, n, n))))
    mom = torch.from_numpy(rng.normal(0, 0.05, (3, n, n, n))) * rho
    a = 0.2
    temp = torch.from_numpy(10 ** rng.uniform(1, 6, (n, n, n)))
    e = temp / cfg.t_per_e
    et = a * a * rho * (e + 0.5 * ((mom / (a * rho)) ** 2).sum(0))
    q = torch.cat([rho[None], mom, et[None]])
    if dual:
        s_var = a * a * e * rho ** (2.0 - cfg.gamma)   # the entropy of the true internal energy
        cold = torch.from_numpy(rng.random((n, n, n)) < 0.25)
        # these cells' total energy holds an internal energy of 1e-4 of their kinetic energy,
        # below the 1e-3 of the total at which the entropy takes over
        ke = 0.5 * ((mom / (a * rho)) ** 2).sum(0)
        et = torch.where(cold, a * a * rho * ke * (1.0 + 1e-4), et)
        q = torch.cat([rho[None], mom, et[None], s_var[None]])
        assert bool(((hydro.internal_energy(q, a, cfg.gamma)[0] - e).abs() < 1e-9 * e)[cold].all())
    star = torch.zeros(n, n, n)
    u = torch.from_numpy(philox.starform_uniform(cfg.sf_seed, 3, n))
    dt = 0.02
    e0 = prm.e0 * 1e6 / cfg.vel_unit ** 2
    ref_q, ref_s = subgrid.apply_source(
        q, star, a, dt, u, rho_mean_gas=cfg.f_b, omega_b=cfg.omega_b, gamma=cfg.gamma,
        e_floor=cfg.e_floor, t_per_e=cfg.t_per_e, e0_code=e0, eps_sf=prm.eps_sf,
        delta_c=prm.delta_c, t_c=prm.t_c, w_rho=prm.w_rho, w_t=prm.w_t, tau=cfg.tau,
        mode=cfg.subgrid, smooth=smooth)
    tgt = mlp.targets(q[0] / cfg.f_b, subgrid.temperature(q, a, cfg.gamma, cfg.e_floor, cfg.t_per_e),
                      a, prm.eps_sf, prm.delta_c, omega_b=cfg.omega_b, t_c=prm.t_c,
                      w_rho=prm.w_rho, w_t=prm.w_t)
    got_q, got_s = mlp.apply_with_outputs(q, star, a, dt, u, tgt, e0_code=e0, tau=cfg.tau,
                                          mode=cfg.subgrid, smooth=smooth, gamma=cfg.gamma)
    assert got_q.shape[0] == q.shape[0]
    assert float(ref_s.sum()) > 1.0   # stars do form in this state
    assert torch.allclose(got_q, ref_q, rtol=1e-12, atol=0)
    assert torch.allclose(got_s, ref_s, rtol=1e-10, atol=1e-50)

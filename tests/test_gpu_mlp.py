"""Learned star-formation closure on the GPU (matrix-core kernels through the C ABI) against
the FP64 oracle of oracle.mlp: inference, input gradients and the objective's weight
gradient, the training set, training, one simulation step and the reverse pass with the
closure, and what the trained network gains over running without the source term.

Tolerances.  The reference is the network in FP64 (oracle.mlp.forward with bf16=False).
The GPU multiplies bfloat16 operands (unit roundoff u = 2^-9 = 2e-3) with FP32 sums, so it
differs from the FP64 network by a few u per layer: on the test inputs the oracle's own
bfloat16 model of that arithmetic (bf16=True: every operand of the forward and backward
matrix products rounded) lies 1e-3 from the FP64 network in the outputs, 7e-3 in the input
gradient, 1e-3 in the weight gradient (5e-3 for the smallest block), 1.5e-3 in a closure
step's energy and star field.  The FP64 bars are about four times those: FP64_FWD = 5e-3,
FP64_VJP = 3e-2, FP64_WGRAD = 5e-3 (2e-2 per block), FP64_STEP = 1e-2.  A parameter
gradient that sums per-cell terms of both signs is held to 5e-2 of the sum of their
magnitudes.  As a second, tighter check the GPU is also compared with the bfloat16 model,
which it follows up to FP32 accumulation and rare values whose FP32 and FP64 results round
to neighbouring bfloat16 values: 1e-3 relative L2 for outputs, 5e-3 for gradients."""

import numpy as np
import pytest
import torch
from dataclasses import replace

import synth_inputs as si
from gpu_helpers import (closure_oracle_gradient, gpu_config, gpu_params, load_state, rel_l2,
                         rounded_state, to_gpu, to_np)
from oracle import mlp as omlp, sim as osim, subgrid

pytestmark = pytest.mark.gpu
torch.set_default_dtype(torch.float64)

FWD_TOL = 1e-3          # against the bfloat16 model
BWD_TOL = 5e-3
FP64_FWD = 5e-3         # against the FP64 network
FP64_VJP = 3e-2
FP64_WGRAD = 5e-3
FP64_STEP = 1e-2
FP64_PARAM = 5e-2


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


def _inputs(count, seed):
    """Network inputs spread over the trained range (uniform in [-1, 1] per input)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (5, count)).astype(np.float32)


def _theta(net):
    return torch.from_numpy(net.weights().astype(np.float64))


@pytest.mark.parametrize("count", [1, 1000, 4096])
def test_eval_matches_oracle(dhp, count):
    net = dhp.Mlp(seed=3)
    x = _inputs(count, seed=count)
    out = to_np(net.eval(to_gpu(x)))
    th = _theta(net)
    ref16 = omlp.forward(th, torch.from_numpy(x).double(), bf16=True).numpy()
    ref64 = omlp.forward(th, torch.from_numpy(x).double()).numpy()
    assert rel_l2(out, ref64) < FP64_FWD, rel_l2(out, ref64)
    assert rel_l2(out, ref16) < FWD_TOL, rel_l2(out, ref16)
    # per element: within a few bfloat16 roundings of the output scale
    assert np.abs(out - ref64).max() < 2e-2 * np.abs(ref64).max()


def test_weights_round_trip(dhp):
    net = dhp.Mlp(seed=5)
    th = net.weights()
    assert th.shape == (omlp.N_PARAMS,) and np.all(np.isfinite(th))
    parts = omlp.unpack(torch.from_numpy(th.astype(np.float64)))
    for p, f in zip(parts, omlp.FAN_IN):
        assert float(p.abs().max()) <= 1.0 / np.sqrt(f)
    net2 = dhp.Mlp()
    net2.set_weights(th)
    assert np.array_equal(net2.weights(), th)
    x = to_gpu(_inputs(300, seed=8))
    assert torch.equal(net.eval(x), net2.eval(x))


def test_vjp_matches_oracle_autograd(dhp):
    net = dhp.Mlp(seed=4)
    count = 2000
    x = _inputs(count, seed=11)
    gout = np.random.default_rng(12).normal(size=(2, count)).astype(np.float32)
    gx = to_np(net.vjp(to_gpu(x), to_gpu(gout)))
    refs = {}
    for bf16 in (False, True):
        xt = torch.from_numpy(x).double().requires_grad_(True)
        o = omlp.forward(_theta(net), xt, bf16=bf16)
        refs[bf16], = torch.autograd.grad(o, xt, grad_outputs=torch.from_numpy(gout).double())
    ref64, ref16 = refs[False].numpy(), refs[True].numpy()
    assert rel_l2(gx, ref64) < FP64_VJP, rel_l2(gx, ref64)
    assert rel_l2(gx, ref16) < BWD_TOL, rel_l2(gx, ref16)


@pytest.mark.parametrize("count", [100, 3000])
def test_weight_gradient_matches_oracle_autograd(dhp, count):
    net = dhp.Mlp(seed=6)
    x = _inputs(count, seed=13)
    y = np.random.default_rng(14).normal(0.0, 3.0, (2, count)).astype(np.float32)
    loss, g = net.grad(to_gpu(x), to_gpu(y))
    refs, losses = {}, {}
    for bf16 in (False, True):
        th = _theta(net).requires_grad_(True)
        L = omlp.loss(th, torch.from_numpy(x).double(), torch.from_numpy(y).double(), bf16=bf16)
        refs[bf16], = torch.autograd.grad(L, th)
        losses[bf16] = float(L)
    ref64, ref16 = refs[False].numpy(), refs[True].numpy()
    assert abs(loss - losses[False]) < FP64_FWD * losses[False]
    assert abs(loss - losses[True]) < 1e-4 * losses[True]
    assert rel_l2(g, ref64) < FP64_WGRAD, rel_l2(g, ref64)
    assert rel_l2(g, ref16) < BWD_TOL, rel_l2(g, ref16)
    # every parameter block (W1, b1, ..., b4) is right, not only the largest
    k = 0
    for s in omlp.SHAPES:
        m = int(np.prod(s))
        assert rel_l2(g[k:k + m], ref64[k:k + m]) < 4 * FP64_WGRAD, (s, k)
        assert rel_l2(g[k:k + m], ref16[k:k + m]) < 2 * BWD_TOL, (s, k)
        k += m


def test_training_set_is_the_plain_source_term(dhp):
    net = dhp.Mlp()
    count = 50000
    prm = osim.Params()
    x, y = net.sample(count, seed=7, omega_b=0.05, params=gpu_params(prm))
    x64, y64 = to_np(x), to_np(y)
    d, t, a, eps, dc = omlp.decode_features(torch.from_numpy(x64))
    ref = omlp.targets(d, t, a, eps, dc, omega_b=0.05, t_c=prm.t_c, w_rho=prm.w_rho,
                       w_t=prm.w_t).numpy()
    assert np.max(np.abs(y64 - ref)) < 1e-4
    assert float(eps.min()) >= 0.01 - 1e-6 and float(eps.max()) <= 0.03 + 1e-6
    assert float(dc.min()) >= 50 - 1e-4 and float(dc.max()) <= 150 + 1e-4
    assert float(a.min()) >= 0.008 * (1 - 1e-5) and float(a.max()) <= 0.32 * (1 + 1e-5)
    near = (np.abs(np.log(d.numpy()) - np.log(dc.numpy())) <= 1.5).mean()
    assert 0.55 < near < 0.65     # half drawn near the threshold, plus the uniform share
    # pieces of a stream concatenate to the whole
    x1, y1 = net.sample(1000, seed=7, first=0, params=gpu_params(prm))
    x2, y2 = net.sample(500, seed=7, first=1000, params=gpu_params(prm))
    xa, ya = net.sample(1500, seed=7, params=gpu_params(prm))
    assert torch.equal(torch.cat([x1, x2], 1), xa) and torch.equal(torch.cat([y1, y2], 1), ya)


def test_closure_states_are_the_plain_source_term(dhp):
    """dh_closure_states on an evolved state: every cell's network inputs and plain targets
    against the oracle's features and targets of the same cells."""
    n = 32
    ocfg = osim.default_config(n=n, box=10.0)
    st = osim.initial_state(torch.from_numpy(si.white_noise(n, 3)).double(), ocfg)
    st, _ = osim.run(st, ocfg, osim.Params(), a_final=0.1)
    st = rounded_state(st)
    prm = osim.Params(eps_sf=0.03, delta_c=10.0, t_c=1e7)
    s = dhp.Sim(gpu_config(replace(ocfg, subgrid=subgrid.MODE_RELAXED)), gpu_params(prm))
    load_state(s, st)
    x, y = s.closure_states()
    temp = subgrid.temperature(st.q, st.a, ocfg.gamma, ocfg.e_floor, ocfg.t_per_e)
    delta = st.q[0] / ocfg.f_b
    xr = omlp.features(delta, temp, st.a, prm.eps_sf, prm.delta_c).reshape(5, -1).numpy()
    yr = omlp.targets(delta, temp, st.a, prm.eps_sf, prm.delta_c, omega_b=ocfg.omega_b,
                      t_c=prm.t_c, w_rho=prm.w_rho, w_t=prm.w_t).reshape(2, -1).numpy()
    assert np.abs(to_np(x) - xr).max() < 1e-5
    assert np.abs(to_np(y) - yr).max() < 1e-4
    assert (yr[1] > -10.0).mean() > 1e-3   # some cells have open gates


def _train(dhp, steps=20000, count=1 << 21, seed=7, params=None, opts=None):
    net = dhp.Mlp(seed=1)
    x, y = net.sample(count, seed=seed, params=params, opts=opts)
    hist = net.train(x, y, steps=steps)
    return net, hist


def test_training_fits_the_source_term(dhp):
    net, hist = _train(dhp)
    assert np.all(np.isfinite(hist))
    assert hist[-100:].mean() < 0.01 * hist[:10].mean()
    # held-out states: the log probability of one step (the quantity the draw uses)
    xh, yh = net.sample(200000, seed=99)
    o = to_np(net.eval(xh))
    t = to_np(yh)
    dt = 0.002
    lp_net = np.log(-np.expm1(-np.exp(o[0]) * dt)) + np.minimum(o[1], 0.0)
    lp_ref = np.log(-np.expm1(-np.exp(t[0]) * dt)) + t[1]
    live = t[1] > -10.0          # states whose gate is not negligible
    err = np.abs(lp_net - lp_ref)[live]
    assert np.median(err) < 0.04 and np.mean(err) < 0.06, (np.median(err), np.mean(err))


def _closure_config(ocfg, theta, bf16=False, **kw):
    return replace(ocfg, closure_theta=theta, closure_bf16=bf16, **kw)


def test_closure_step_matches_oracle(dhp):
    n = 32
    ocfg0 = osim.default_config(n=n, box=10.0)
    st = osim.initial_state(torch.from_numpy(si.white_noise(n, 3)).double(), ocfg0)
    st, _ = osim.run(st, ocfg0, osim.Params(), a_final=0.05)
    st = rounded_state(st)
    net = dhp.Mlp(seed=8)
    theta = net.weights().astype(np.float64)
    ocfg0 = osim.default_config(n=n, box=10.0, subgrid=subgrid.MODE_RELAXED)
    prm = osim.Params()
    s = dhp.Sim(gpu_config(ocfg0, closure=1), gpu_params(prm))
    s.set_closure(theta)
    load_state(s, st)
    dt = osim.cfl_dt(st, ocfg0)
    s.set_schedule([dt])
    s.step()
    star = to_np(s.get("star"))
    q = to_np(s.get("q"))
    for bf16, tol_q, tol_star in ((False, FP64_STEP, FP64_STEP), (True, 1e-4, FWD_TOL)):
        ref = osim.step(st, _closure_config(ocfg0, theta, bf16=bf16), prm, dt)
        assert float(ref.star.sum()) > 10.0
        for c in range(5):
            assert rel_l2(q[c], ref.q[c].numpy()) < tol_q, (bf16, c, rel_l2(q[c], ref.q[c].numpy()))
        assert rel_l2(star, ref.star.numpy()) < tol_star, (bf16, rel_l2(star, ref.star.numpy()))


def test_closure_gradient_matches_oracle_autograd(dhp):
    n = 16
    net = dhp.Mlp(seed=9)
    theta = net.weights().astype(np.float64)
    ocfg0 = osim.default_config(n=n, box=4.0, subgrid=subgrid.MODE_RELAXED, a_init=0.05)
    prm = osim.Params(eps_sf=0.025, delta_c=80.0)
    w = si.white_noise(n, seed=22)
    target = (0.2 + 0.7 * np.random.default_rng(2).random((n, n, n))).astype(np.float32)
    nsteps = 3
    ocfg = _closure_config(ocfg0, theta)
    st0 = osim.initial_state(torch.from_numpy(w).double(), ocfg)
    _, sched = osim.run(st0, ocfg, prm, nsteps=nsteps)
    s = dhp.Sim(gpu_config(ocfg, closure=1, ckpt_every=2), gpu_params(prm))
    s.set_closure(theta)
    s.set_schedule(sched)
    assert s.forward(to_gpu(w), 1.0) == nsteps
    lval = s.loss(to_gpu(target))
    gw, gp = s.backward()
    gw = to_np(gw)
    gp = np.array(gp)
    # the FP64 network, then the bfloat16 model of the GPU's arithmetic
    for bf16, tol_w, tol_sf in ((False, 1e-2, FP64_PARAM), (True, 1e-2, BWD_TOL)):
        L, gw_ref, gp_ref, mag = closure_oracle_gradient(_closure_config(ocfg0, theta, bf16),
                                                          prm, w, target, sched)
        assert abs(lval - L) < 1e-4 * L, (bf16, lval, L)
        assert rel_l2(gw, gw_ref) < tol_w, (bf16, rel_l2(gw, gw_ref))
        for i in range(2):     # A, beta act on the final state only
            assert abs(gp[i] - gp_ref[i]) < 1e-3 * mag[i] + 1e-12, (bf16, i, gp, gp_ref)
        for i in (2, 3):
            assert abs(gp[i] - gp_ref[i]) < tol_sf * mag[i] + 1e-12, (bf16, i, gp, gp_ref, mag)


def test_trained_closure_gains_over_no_source_term(dhp):
    """Final fields of a run with the trained closure are much closer to the plain source
    term's run than a run without star formation (same initial conditions and uniforms).
    Without cooling, gas denser than the default threshold is hot at this resolution, so the
    run uses thresholds under which stars do form (Delta_c = 10, T_c = 1e7 K), and the
    network is trained for them."""
    prm = gpu_params(osim.Params(eps_sf=0.03, delta_c=10.0, t_c=1e7))
    net, _ = _train(dhp, params=prm, opts=dhp.mlp.sample_defaults(dc_lo=5.0, dc_hi=20.0))
    theta = net.weights()
    n, box, a_final = 64, 10.0, 0.29
    w = to_gpu(si.white_noise(n, seed=6))
    finals = {}
    for name, sub, clo in (("plain", 2, 0), ("mlp", 2, 1), ("off", 0, 0)):
        s = dhp.Sim(dhp.default_config(n=n, box=box, subgrid=sub, closure=clo), prm)
        if clo:
            s.set_closure(theta)
        s.init_from_noise(w)
        s.run_to(a_final)
        finals[name] = (to_np(s.get("rho")), np.log(to_np(s.get("temp"))), to_np(s.get("star")))
    rho_p, lt_p, star_p = finals["plain"]
    d_mlp = [rel_l2(finals["mlp"][k], finals["plain"][k]) for k in range(2)]
    d_off = [rel_l2(finals["off"][k], finals["plain"][k]) for k in range(2)]
    info = dict(d_mlp=d_mlp, d_off=d_off, stars_plain=float(star_p.sum()),
                stars_mlp=float(finals["mlp"][2].sum()))
    print(info)
    assert star_p.sum() > 10.0, info
    # the relaxed draw amplifies errors of ln pi0 by 1/tau = 10, so a per-cell error of a few
    # percent leaves a residual distance; the gain is still several-fold in both fields
    assert d_mlp[0] < 0.4 * d_off[0] and d_mlp[1] < 0.4 * d_off[1], info
    assert abs(finals["mlp"][2].sum() - star_p.sum()) < 0.15 * star_p.sum(), info

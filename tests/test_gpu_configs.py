"""The two 128^3 workloads of the paper-shaped runs on the GPU, at their stated sizes:

* forward: 128^3 cells and particles in a 20 Mpc/h box from a = 0.01 to a = 0.29 (about 150
  CFL steps) with Bernoulli star formation (rho/rho_mean > 100, T < 10^4.5 K, eps_SF = 0.02):
  the step count, conservation of gas mass and of total momentum, and a bitwise replay of the
  recorded schedule;
* forward + reverse: the flux-field loss against a target from another seed, gradients with
  respect to the 128^3 white noise and the four parameters with a checkpoint every 16 steps,
  checked against central finite differences of the GPU's own forward on 32 random
  directions of the white noise and on each parameter (to a = 0.05), and, over the whole run
  to a = 0.29, for consistency between checkpoint layouts and in the loss parameters.

The oracle cannot run 150 steps at 128^3 within a test; its parity at these sizes is shown
stage by stage and for single steps elsewhere, and here the checks are properties that hold
at any size.  Each test prints what it runs."""

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_helpers import to_gpu

pytestmark = pytest.mark.gpu

N = 128
BOX = 20.0
A_FINAL = 0.29


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


def _say(msg):
    print(msg, flush=True)


def test_forward_128_to_a029_with_bernoulli_star_formation(dhp):
    cfg = dhp.default_config(n=N, box=BOX, a_init=0.01, subgrid=1)   # 1: Bernoulli draws
    prm = dhp.default_params(eps_sf=0.02, delta_c=100.0, t_c=10 ** 4.5)
    w = to_gpu(si.white_noise(N, 1))
    _say("forward 128^3 a = 0.01 -> 0.29: first run")
    s = dhp.Sim(cfg, prm)
    s.init_from_noise(w)
    c0 = s.conservation()
    k = s.run_to(A_FINAL)
    c1 = s.conservation()
    _say(f"forward 128^3: {k} steps, a = {s.time()[0]:.4f}")
    assert 100 <= k <= 250
    assert abs(s.time()[0] - A_FINAL) < 1e-9
    q1, p1, star1 = s.get("q").clone(), s.get("pos").clone(), s.get("star").clone()
    assert torch.isfinite(q1).all() and torch.isfinite(p1).all()
    # gas mass is conserved to float32 rounding; total (gas + dark matter) momentum to the
    # PM scheme's symmetry
    assert abs(c1[0] - c0[0]) <= 1e-5 * c0[0]
    for d in range(3):
        scale = abs(c0[1 + d]) + abs(c0[5 + d]) + abs(c1[1 + d]) + abs(c1[5 + d]) + 1e-3 * c0[0]
        assert abs((c1[1 + d] + c1[5 + d]) - (c0[1 + d] + c0[5 + d])) < 1e-4 * scale, d
    sched = s.get_schedule()
    s.close()
    _say("forward 128^3: replay of the recorded schedule")
    r = dhp.Sim(cfg, prm)
    r.init_from_noise(w)
    r.set_schedule(sched)
    assert r.run_to(A_FINAL) == k
    assert torch.equal(r.get("q"), q1) and torch.equal(r.get("pos"), p1)
    assert torch.equal(r.get("star"), star1)
    r.close()


SF = dict(eps_sf=0.03, delta_c=10.0, t_c=1e7)


def _grad_setup(dhp, a_final, ckpt):
    # star formation that acts in this box (the default thresholds form almost no stars
    # without cooling), so that the two star-formation gradients are not zero
    cfg = dhp.default_config(n=N, box=BOX, a_init=0.01, subgrid=2, ckpt_every=ckpt)
    s = dhp.Sim(cfg, dhp.default_params(**SF))
    s.init_from_noise(to_gpu(si.white_noise(N, 12)))
    s.run_to(a_final)
    target = s.get("flux").clone()
    return s, target


def _loss_at(dhp, s, sched, target, white, **p):
    prm = dict(SF)
    prm.update(p)
    s.set_params(dhp.default_params(**prm))
    s.set_schedule(sched)
    s.forward(to_gpu(white), 1.0)
    return s.loss(target)


def test_gradient_128_against_finite_differences(dhp):
    """Adjoint against central finite differences of the GPU forward, 128^3 from a = 0.01 to
    a = 0.05 (about 40 steps, three checkpoint segments): 32 random white-noise directions
    and the four parameters."""
    a_final = 0.05
    _say("gradient 128^3 to a = 0.05: target run (seed 12)")
    s, target = _grad_setup(dhp, a_final, 16)
    w = si.white_noise(N, 11)
    _say("gradient 128^3 to a = 0.05: forward with checkpoints, loss, reverse pass")
    k = s.forward(to_gpu(w), a_final)
    sched = s.get_schedule()
    l0 = s.loss(target)
    gw, gp = s.backward()
    gw = gw.double().cpu().numpy()
    gnorm = np.linalg.norm(gw)
    _say(f"gradient 128^3: {k} steps, loss {l0:.6e}, |gw| {gnorm:.3e}, gp {gp}")
    # unit-variance random directions, eps = 1e-2 of the noise amplitude: the float32 forward
    # leaves a rounding noise of ~1e-6 of the loss, which a step of 1e-3 would turn into an
    # error of ~2% of |gw| here; at 1e-2 it is ~0.2%, above the second-order term
    rng = np.random.default_rng(13)
    eps = 1e-2
    errs = []
    for d in range(32):
        v = rng.standard_normal((N, N, N)).astype(np.float32)
        fd = (_loss_at(dhp, s, sched, target, (w + eps * v).astype(np.float32)) -
              _loss_at(dhp, s, sched, target, (w - eps * v).astype(np.float32))) / (2 * eps)
        ad = float(np.sum(gw * v))
        # relative to |gw|, the typical size of the derivative along a random direction
        errs.append(abs(fd - ad) / gnorm)
        _say(f"  direction {d}: finite difference {fd:.6e}, adjoint {ad:.6e}")
    _say(f"gradient 128^3: white-noise directions, errors / |gw|: median {np.median(errs):.2e} "
         f"max {np.max(errs):.2e}")
    # the map is piecewise smooth (limiter branches, CIC cell crossings): a finite difference
    # averages the derivative over the kinks it crosses, which costs about 1% of |gw| here at
    # both eps = 1e-3 and 1e-2; that the adjoint is the exact derivative of the discrete map is
    # checked against the oracle's autograd in the parity tests
    assert np.median(errs) < 2e-2 and np.max(errs) < 5e-2
    # parameters: relative steps of 1e-3
    center = dict(A=0.3, beta=1.6, eps_sf=SF["eps_sf"], delta_c=SF["delta_c"])
    for i, name in enumerate(("A", "beta", "eps_sf", "delta_c")):
        h = 1e-3 * center[name]
        lp = _loss_at(dhp, s, sched, target, w, **{name: center[name] + h})
        lm = _loss_at(dhp, s, sched, target, w, **{name: center[name] - h})
        fd = (lp - lm) / (2 * h)
        _say(f"  {name}: finite difference {fd:.6e}, adjoint {gp[i]:.6e}")
        # 2% of the value, or the float32 rounding of the loss over the step
        assert abs(fd - gp[i]) <= 2e-2 * abs(gp[i]) + 1e-6 * abs(l0) / h, (name, fd, gp[i])
    s.close()


def test_gradient_128_full_run_is_consistent(dhp):
    """The reverse pass of the whole 128^3 run (a = 0.01 -> 0.29, about 120 steps, a checkpoint
    every 16 steps): finite, bit for bit equal to the reverse pass of the same run kept as one
    segment, and exact in the loss parameters A and beta against finite differences (they act
    on the final state only).  Finite differences along white-noise directions do not
    converge over this run at the CFL number 0.4 (the exact derivative of the discrete map
    has grid-scale structure), so they are checked on the shorter run above."""
    _say("gradient 128^3 to a = 0.29: target run")
    s, target = _grad_setup(dhp, A_FINAL, 16)
    w = si.white_noise(N, 11)
    _say("gradient 128^3 to a = 0.29: reverse pass with checkpoints every 16 steps")
    k = s.forward(to_gpu(w), A_FINAL)
    sched = s.get_schedule()
    l0 = s.loss(target)
    gw, gp = s.backward()
    assert torch.isfinite(gw).all() and all(np.isfinite(gp))
    s.close()
    _say("gradient 128^3 to a = 0.29: reverse pass of one segment")
    one = dhp.Sim(dhp.default_config(n=N, box=BOX, a_init=0.01, subgrid=2, ckpt_every=1000),
                  dhp.default_params(**SF))
    one.set_schedule(sched)
    assert one.forward(to_gpu(w), 1.0) == k
    assert one.loss(target) == l0
    gw1, gp1 = one.backward()
    assert torch.equal(gw, gw1) and gp == gp1
    for i, (name, c) in enumerate((("A", 0.3), ("beta", 1.6))):
        h = 1e-3 * c
        lp = _loss_at(dhp, one, sched, target, w, **{name: c + h})
        lm = _loss_at(dhp, one, sched, target, w, **{name: c - h})
        fd = (lp - lm) / (2 * h)
        _say(f"  {name}: finite difference {fd:.6e}, adjoint {gp[i]:.6e}")
        assert abs(fd - gp[i]) <= 1e-3 * abs(gp[i]) + 1e-6 * abs(l0) / h
    one.close()


@pytest.mark.parametrize("n,box,a_final", [(32, 5.0, 0.29), (64, 10.0, 0.1)])
def test_long_run_gradient_matches_oracle_autograd(dhp, n, box, a_final):
    """Over whole runs (0.156 Mpc/h cells, CFL 0.4, no source term) the reverse pass is the
    exact derivative of the discrete map: against the FP64 oracle's autograd over 89 steps to
    a = 0.29 at 32^3 and 60 steps to a = 0.1 at 64^3 (the oracle's own central differences
    along a random direction are printed beside it).  The map is piecewise smooth
    (limiter, |U_d|, CIC cell crossings); float32 and float64 take different sides of the
    kinks in a few cells per step, which over these runs moves the gradient by a few 1e-3
    (5e-3 bar).  At 128^3 the float32 forward cannot resolve the derivative by finite
    differences beyond a ~ 0.05: steps above its rounding noise (eps >= 1e-3) cross many
    kinks, and the exact derivative grows quickly with a and with resolution."""
    import torch as th
    from gpu_helpers import gpu_config, gpu_params, initial_state_fp32_cells, rel_l2, to_np
    from oracle import sim as osim
    th.set_num_threads(16)
    prm = osim.Params(eps_sf=0.03, delta_c=10.0, t_c=1e7)
    ocfg = osim.default_config(n=n, box=box, a_init=0.01)
    w = si.white_noise(n, 11)
    tgt, sched = osim.run(osim.initial_state(th.from_numpy(si.white_noise(n, 12)).double(), ocfg),
                          ocfg, prm, a_final=a_final)
    target = osim.flux_observable(tgt.q[0], ocfg.f_b, prm.A, prm.beta).detach()
    _, sched = osim.run(osim.initial_state(th.from_numpy(w).double(), ocfg), ocfg, prm,
                        a_final=a_final)
    _say(f"long-run gradient {n}^3 to a = {a_final}: {len(sched)} steps, oracle autograd")
    w64 = th.from_numpy(w).double().requires_grad_(True)
    st, _ = osim.run(initial_state_fp32_cells(w64, ocfg), ocfg, prm, schedule=sched)
    L = osim.loss(st, target, ocfg, prm.A, prm.beta)
    (gref,) = th.autograd.grad(L, w64)
    s = dhp.Sim(gpu_config(ocfg, ckpt_every=16), gpu_params(prm))
    s.set_schedule(sched)
    s.forward(to_gpu(w), 1.0)
    lval = s.loss(to_gpu(target.numpy()))
    gw, _ = s.backward()
    g = to_np(gw)
    err = rel_l2(g, gref.numpy())
    _say(f"long-run gradient {n}^3: loss {lval:.6e} / {float(L.detach()):.6e}, rel-L2 {err:.2e}")
    assert abs(lval - float(L.detach())) < 1e-4 * float(L.detach())
    assert err < 5e-3
    # the oracle's finite differences converge to its exact derivative along a direction
    v = th.from_numpy(np.random.default_rng(13).standard_normal((n, n, n)))
    eps = 1e-6
    with th.no_grad():
        lp, lm = (osim.loss(osim.run(osim.initial_state(th.from_numpy(w).double() + sg * eps * v,
                                                        ocfg), ocfg, prm, schedule=sched)[0],
                            target, ocfg, prm.A, prm.beta) for sg in (1.0, -1.0))
    fd = float(lp - lm) / (2 * eps)
    ad = float((gref * v).sum())
    _say(f"  oracle: finite difference {fd:.6e}, autograd {ad:.6e}; GPU {float((th.from_numpy(g) * v).sum()):.6e}")

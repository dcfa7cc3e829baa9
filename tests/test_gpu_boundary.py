"""The C-ABI boundary as a caller sees it, on the GPU: the torch.autograd.Function over the
forward run and the reverse pass against the oracle's autograd, the FP64 conservation sums
against the oracle's on the same state, the accuracy check of replayed time-step schedules
(Sec. 2.3.3) and the error returned for a state with a non-finite value or a non-positive
density."""

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_helpers import (gpu_config, gpu_params, initial_state_fp32_cells, load_state, rel_l2,
                         rounded_state, to_gpu, to_np)
from oracle import sim as osim, subgrid

pytestmark = pytest.mark.gpu
torch.set_default_dtype(torch.float64)


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


def test_autograd_function_matches_oracle_autograd(dhp):
    """DiffHydroFn.apply(white, (eps_sf, delta_c)) -> final gas density; backpropagating a
    random dL/drho through it (dh_backward with a caller adjoint) gives the oracle's exact
    gradient with respect to the white noise and the two star-formation parameters."""
    from paper_2502_02294_amd.autograd import DiffHydroFn
    n, nsteps = 16, 3
    ocfg = osim.default_config(n=n, box=4.0, subgrid=subgrid.MODE_RELAXED, a_init=0.05)
    prm = osim.Params(delta_c=1.05, t_c=1e6, eps_sf=0.5)
    w = si.white_noise(n, seed=31)
    lam = np.random.default_rng(32).normal(size=(n, n, n)).astype(np.float32)
    st0 = osim.initial_state(torch.from_numpy(w).double(), ocfg)
    _, sched = osim.run(st0, ocfg, prm, nsteps=nsteps)
    w64 = torch.from_numpy(w).double().requires_grad_(True)
    th = torch.tensor([prm.eps_sf, prm.delta_c], requires_grad=True)
    p2 = osim.Params(eps_sf=th[0], delta_c=th[1], t_c=prm.t_c)
    st = initial_state_fp32_cells(w64, ocfg)
    st, _ = osim.run(st, ocfg, p2, schedule=sched)
    L = (st.q[0] * torch.from_numpy(lam).double()).sum()
    gw_ref, gth_ref = torch.autograd.grad(L, (w64, th))

    s = dhp.Sim(gpu_config(ocfg, ckpt_every=2), gpu_params(prm))
    s.set_schedule(sched)
    wg = to_gpu(w).requires_grad_(True)
    theta = torch.tensor([prm.eps_sf, prm.delta_c], dtype=torch.float64, requires_grad=True)
    rho = DiffHydroFn.apply(wg, theta, s, 1.0)
    assert rho.shape == (n, n, n)
    assert rel_l2(to_np(rho), st.q[0].detach().numpy()) < 1e-5
    (rho * to_gpu(lam)).sum().backward()
    err_w = rel_l2(to_np(wg.grad), gw_ref.numpy())
    assert err_w < 1e-3, err_w
    assert np.abs(to_np(wg.grad) - gw_ref.numpy()).max() < 1e-2 * np.abs(gw_ref.numpy()).max()
    g = theta.grad.numpy()
    for i in range(2):
        assert abs(g[i] - float(gth_ref[i])) < 1e-3 * abs(float(gth_ref[i])) + 1e-9, (g, gth_ref)
    with pytest.raises(ValueError):
        b = dhp.Sim(gpu_config(ocfg, batch=2), gpu_params(prm))
        DiffHydroFn.apply(to_gpu(np.stack([w, w])), theta, b, 1.0)


@pytest.mark.parametrize("subgrid_mode", [subgrid.MODE_OFF, subgrid.MODE_RELAXED])
def test_conservation_sums_match_oracle(dhp, subgrid_mode):
    """The eight FP64 sums (gas mass, gas momentum, gas energy, dark-matter momentum) on one
    state, and after three steps on the GPU and in the oracle from it."""
    n = 32
    ocfg = osim.default_config(n=n, box=10.0, subgrid=subgrid_mode)
    prm = osim.Params(delta_c=1.5, t_c=1e6, eps_sf=5.0)
    st = osim.initial_state(torch.from_numpy(si.white_noise(n, 33)).double(), ocfg)
    st, _ = osim.run(st, ocfg, prm, a_final=0.04)
    st = rounded_state(st)
    s = dhp.Sim(gpu_config(ocfg), gpu_params(prm))
    load_state(s, st)
    got = np.array(s.conservation())
    ref = osim.conservation(st, ocfg)
    # sums of the same float32 values in FP64: equal to the FP64 summation rounding
    scale = np.array([abs(ref[0])] + [np.abs(st.q[1 + d].numpy()).sum() for d in range(3)] +
                     [abs(ref[4])] + [np.abs(st.p[d].numpy()).sum() * (1 - ocfg.f_b)
                                      for d in range(3)])
    assert np.all(np.abs(got - ref) <= 1e-12 * scale), (got, ref)
    mass0, mom0 = ref[0], ref[1:4] + ref[5:8]
    dts = []
    for _ in range(3):
        dt = osim.cfl_dt(st, ocfg)
        dts.append(dt)
        st = osim.step(st, ocfg, prm, dt)
    s.set_schedule(dts)
    for _ in range(3):
        s.step()
    got = np.array(s.conservation())
    ref = osim.conservation(st, ocfg)
    # three FP32 steps against FP64 ones: the per-step field tolerance, on sums
    assert abs(got[0] - ref[0]) <= 1e-6 * abs(ref[0])
    assert abs(got[4] - ref[4]) <= 1e-5 * abs(ref[4])
    for d in range(3):
        assert abs(got[1 + d] - ref[1 + d]) <= 1e-5 * scale[1 + d], (d, got, ref)
        assert abs(got[5 + d] - ref[5 + d]) <= 1e-5 * scale[5 + d], (d, got, ref)
    # the gas mass is conserved by the flux form, gas + dark-matter momentum by the symmetric
    # CIC and the antisymmetric gradient (to float32 rounding of the fields)
    assert abs(got[0] - mass0) <= 1e-6 * mass0
    for d in range(3):
        assert abs(got[1 + d] + got[5 + d] - mom0[d]) <= 1e-5 * (scale[1 + d] + scale[5 + d])


def _cfl_limited_schedule(dhp, n, steps):
    """(config, white noise, schedule) of a run whose steps are all set by the CFL speed
    (the d ln a cap raised out of the way)."""
    cfg = dhp.default_config(n=n, box=10.0, a_init=0.05, dlna_max=10.0)
    w = to_gpu(si.white_noise(n, seed=34))
    s = dhp.Sim(cfg)
    s.init_from_noise(w)
    for _ in range(steps):
        s.step()
    return cfg, w, s.get_schedule()


def test_replayed_schedule_accuracy_check(dhp):
    """A schedule replayed on its own run has Courant number C_fid = 0.4 at every step and is
    accepted; scaled by 1.3 (about 0.52 <= C_forward = 0.6) too; scaled by 2 (0.8) the first
    replayed step already exceeds C_forward and the call returns DH_E_SCHEDULE, after which
    the forward cannot be differentiated.  With the check switched off (C_forward = 0) the
    same replay is accepted."""
    from paper_2502_02294_amd._lib import DiffHydroError
    n = 32
    cfg, w, sched = _cfl_limited_schedule(dhp, n, 4)
    assert abs(cfg.cfl_forward - 0.6) < 1e-15
    for scale, ok in ((1.0, True), (1.3, True), (2.0, False)):
        s = dhp.Sim(cfg)
        s.init_from_noise(w)
        s.set_schedule([scale * dt for dt in sched])
        if ok:
            assert s.run_steps(4) == 4
        else:
            with pytest.raises(DiffHydroError) as e:
                s.run_steps(4)
            assert e.value.code == -5 and "Courant" in str(e.value)
        s.close()
    s = dhp.Sim(cfg)
    s.set_schedule([2.0 * dt for dt in sched])
    with pytest.raises(DiffHydroError) as e:
        s.forward(w, 1.0)
    assert e.value.code == -5
    with pytest.raises(DiffHydroError) as e:
        s.backward(torch.zeros(n, n, n, dtype=torch.float32, device="cuda"))
    assert e.value.code == -6
    s.close()
    # one step at a time: the step that exceeds it reports it
    s = dhp.Sim(cfg)
    s.init_from_noise(w)
    s.set_schedule([sched[0], 2.0 * sched[1]])
    s.step()
    with pytest.raises(DiffHydroError) as e:
        s.step()
    assert e.value.code == -5
    s.close()
    cfg.cfl_forward = 0.0
    s = dhp.Sim(cfg)
    s.init_from_noise(w)
    s.set_schedule([2.0 * dt for dt in sched])
    assert s.run_steps(4) == 4
    s.close()


@pytest.mark.parametrize("what", ["nan_energy", "negative_density"])
def test_nonfinite_state_is_reported(dhp, what):
    """A state with a NaN (set through dh_set_field) or a non-positive density: the next CFL
    step returns DH_E_NONFINITE before it takes the step."""
    from paper_2502_02294_amd._lib import DiffHydroError
    n = 16
    s = dhp.Sim(dhp.default_config(n=n, box=4.0))
    s.init_from_noise(to_gpu(si.white_noise(n, seed=35)))
    q = s.get("q").clone()
    if what == "nan_energy":
        q[4, 3, 5, 7] = float("nan")
    else:
        q[0, 2, 2, 2] = -0.01
    s.set("q", q)
    a0 = s.time()[0]
    with pytest.raises(DiffHydroError) as e:
        s.step()
    assert e.value.code == -4
    assert s.time()[0] == a0

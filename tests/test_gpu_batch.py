"""Batched samples (one handle, every launch covering all samples) on the GPU.

Each sample of a batch runs the same kernels on its own slice with its own dt, scale factors,
parameters and random-number keys, and the counting sort orders every sample's particles by
id inside a bin exactly as a single run does, so a sample's result is bit for bit that of a
single-sample handle given the same noise, parameters and star-formation key; the samples
reach their end after different numbers of steps.  The reverse pass is checked the same way,
and one sample against the FP64 oracle."""

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_helpers import gpu_config, gpu_params, rel_l2, to_gpu, to_np
from oracle import sim as osim, subgrid

pytestmark = pytest.mark.gpu
torch.set_default_dtype(torch.float64)


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


SAMPLE_PARAMS = [dict(eps_sf=0.5, delta_c=1.05, t_c=1e6), dict(eps_sf=0.8, delta_c=1.2, t_c=2e6),
                 dict(eps_sf=0.3, delta_c=0.9, t_c=5e5)]


def _batch(dhp, n, box, S, **kw):
    cfg = dhp.default_config(n=n, box=box, subgrid=subgrid.MODE_RELAXED, batch=S, **kw)
    s = dhp.Sim(cfg)
    for i in range(S):
        s.set_sample_params(i, **SAMPLE_PARAMS[i])
    return s


def _single(dhp, n, box, i, **kw):
    # sample i of a batch uses the star-formation key sf_seed + i
    cfg = dhp.default_config(n=n, box=box, subgrid=subgrid.MODE_RELAXED, sf_seed=102 + i, **kw)
    return dhp.Sim(cfg, dhp.default_params(**SAMPLE_PARAMS[i]))


# sample 1 opens with three longer steps (then the CFL): the samples end after different
# numbers of steps
FIRST_STEPS = {1: [1.2e-4] * 3}


def test_batch_samples_equal_single_runs(dhp):
    n, box, S = 32, 10.0, 3
    white = np.stack([si.white_noise(n, seed=40 + i) for i in range(S)])
    b = _batch(dhp, n, box, S)
    for i, dts in FIRST_STEPS.items():
        b.set_sample_schedule(i, dts)
    b.init_from_noise(to_gpu(white))
    k = b.run_to(0.05)
    counts = [len(b.get_sample_schedule(i)) for i in range(S)]
    assert max(counts) == k and len(set(counts)) > 1, counts
    a_b, _ = b.sample_times()
    for i in range(S):
        s = _single(dhp, n, box, i)
        s.set_schedule(FIRST_STEPS.get(i, []))
        s.init_from_noise(to_gpu(white[i]))
        ki = s.run_to(0.05)
        assert ki == counts[i]
        assert s.get_schedule() == b.get_sample_schedule(i)
        assert a_b[i] == s.time()[0]
        for f in ("q", "pos", "mom", "star", "phi"):
            assert torch.equal(b.get(f)[i], s.get(f)), (i, f)


def test_run_loops_equal_single_steps(dhp):
    """run_to and run_steps leave each closing dark-matter kick to the next step's kick-drift
    pass (a sample that has finished keeps its last one pending until the loop ends); the
    states are those of separate steps, bit for bit."""
    n, box, S = 32, 10.0, 3
    white = np.stack([si.white_noise(n, seed=80 + i) for i in range(S)])
    print("run_to of a batch with uneven step counts against single steps", flush=True)
    b = _batch(dhp, n, box, S)
    for i, dts in FIRST_STEPS.items():
        b.set_sample_schedule(i, dts)
    b.init_from_noise(to_gpu(white))
    b.run_to(0.03)
    counts = [len(b.get_sample_schedule(i)) for i in range(S)]
    assert len(set(counts)) > 1, counts
    for i in range(S):
        s = _single(dhp, n, box, i)
        s.set_schedule(b.get_sample_schedule(i))
        s.init_from_noise(to_gpu(white[i]))
        for _ in range(counts[i]):
            s.step()
        for f in ("q", "pos", "mom", "star", "phi"):
            assert torch.equal(b.get(f)[i], s.get(f)), (i, f)
    print("run_steps against step", flush=True)
    runs = []
    for fused in (True, False):
        r = _batch(dhp, n, box, S)
        for i, dts in FIRST_STEPS.items():
            r.set_sample_schedule(i, dts)
        r.init_from_noise(to_gpu(white))
        if fused:
            assert r.run_steps(5) == 5
        else:
            for _ in range(5):
                r.step()
        runs.append({f: r.get(f) for f in ("q", "pos", "mom", "star", "phi")})
        assert r.get_sample_schedule(1)[:3] == FIRST_STEPS[1]
    for f in runs[0]:
        assert torch.equal(runs[0][f], runs[1][f]), f


# samples 1 and 2 replay schedules that stop before a = 0.08 (a forward run ends a sample at
# the end of its schedule); sample 0 steps by the CFL
REPLAY = {1: [7e-4] * 4, 2: [6e-4] * 6}


def test_batch_gradient_equals_single_runs(dhp):
    n, box, S = 16, 4.0, 3
    white = np.stack([si.white_noise(n, seed=60 + i) for i in range(S)])
    target = (0.2 + 0.7 * np.random.default_rng(3).random((S, n, n, n))).astype(np.float32)
    b = _batch(dhp, n, box, S, a_init=0.05, ckpt_every=3)
    for i, dts in REPLAY.items():
        b.set_sample_schedule(i, dts)
    kb = b.forward(to_gpu(white), 0.08)
    lb = b.loss(to_gpu(target))
    gwb, gpb = b.backward()
    counts = [len(b.get_sample_schedule(i)) for i in range(S)]
    assert kb == max(counts) and len(set(counts)) > 1, counts
    for i in range(S):
        s = _single(dhp, n, box, i, a_init=0.05, ckpt_every=3)
        s.set_schedule(REPLAY.get(i, []))
        assert s.forward(to_gpu(white[i]), 0.08) == counts[i]
        assert s.loss(to_gpu(target[i])) == lb[i]
        gw, gp = s.backward()
        assert torch.equal(gwb[i], gw), i
        assert gpb[i] == gp, (i, gpb[i], gp)


@pytest.mark.parametrize("S", [1, 3])
def test_reverse_pass_with_and_without_stored_steps(dhp, S):
    """The forward keeps data for the reverse pass as memory allows: the full tape of whole
    checkpoint segments (no recomputation there), then the particle sort and potential of
    further steps (their recomputation takes them).  Everything taped (-1), nothing (0), two
    steps' sorts (2), one taped segment of three steps and one step's sort (4): the same
    gradients bit for bit (with S = 3 the samples end after different numbers of steps)."""
    n, box = 16, 4.0
    white = np.stack([si.white_noise(n, seed=90 + i) for i in range(S)])
    target = (0.2 + 0.7 * np.random.default_rng(5).random((S, n, n, n))).astype(np.float32)
    outs = []
    for limit in (-1, 0, 2, 4):
        print(f"reverse pass, S = {S}, store limit {limit}", flush=True)
        if S == 1:
            b = _single(dhp, n, box, 0, a_init=0.05, ckpt_every=3)
            b.set_schedule(REPLAY[2])
        else:
            b = _batch(dhp, n, box, S, a_init=0.05, ckpt_every=3)
            for i, dts in REPLAY.items():
                b.set_sample_schedule(i, dts)
        b.set_store_limit(limit)
        w = to_gpu(white if S > 1 else white[0])
        t = to_gpu(target if S > 1 else target[0])
        k = b.forward(w, 0.08)
        assert k >= 4, k   # two checkpoint segments or more
        # what the forward kept: whole segments of 3 steps taped first, then sorts
        expect = {-1: (k, 0), 0: (0, 0), 2: (0, 2), 4: (3, 1)}[limit]
        assert b.store_info() == expect, (limit, b.store_info())
        b.loss(t)
        gw, gp = b.backward()
        outs.append((gw.clone(), gp, b.get("q").clone()))
        b.close()
    for gw, gp, q in outs[1:]:
        assert torch.equal(gw, outs[0][0]) and gp == outs[0][1]
        assert torch.equal(q, outs[0][2])   # the forward's final state is restored


def test_batch_sample_gradient_matches_oracle_autograd(dhp):
    n, box, S = 16, 4.0, 2
    white = np.stack([si.white_noise(n, seed=70 + i) for i in range(S)])
    target = (0.2 + 0.7 * np.random.default_rng(4).random((S, n, n, n))).astype(np.float32)
    b = _batch(dhp, n, box, S, a_init=0.05, ckpt_every=2)
    scheds = []
    for i in range(S):
        ocfg = osim.default_config(n=n, box=box, subgrid=subgrid.MODE_RELAXED, a_init=0.05,
                                   sf_seed=102 + i)
        prm = osim.Params(**SAMPLE_PARAMS[i])
        st0 = osim.initial_state(torch.from_numpy(white[i]).double(), ocfg)
        _, sched = osim.run(st0, ocfg, prm, nsteps=3 + i)   # uneven counts
        scheds.append((ocfg, prm, sched))
        b.set_sample_schedule(i, sched)
    b.forward(to_gpu(white), 1.0)
    losses = b.loss(to_gpu(target))
    gwb, gpb = b.backward()
    for i in range(S):
        ocfg, prm, sched = scheds[i]
        w64 = torch.from_numpy(white[i]).double().requires_grad_(True)
        th = torch.tensor([prm.A, prm.beta, prm.eps_sf, prm.delta_c], requires_grad=True)
        p2 = osim.Params(A=th[0], beta=th[1], eps_sf=th[2], delta_c=th[3], t_c=prm.t_c)
        st, _ = osim.run(osim.initial_state(w64, ocfg), ocfg, p2, schedule=sched)
        loss = osim.loss(st, torch.from_numpy(target[i]).double(), ocfg, th[0], th[1])
        gw_ref, gp_ref = torch.autograd.grad(loss, (w64, th))
        assert abs(losses[i] - float(loss)) < 1e-4 * float(loss)
        assert rel_l2(to_np(gwb[i]), gw_ref.numpy()) < 1e-3, (i, rel_l2(to_np(gwb[i]), gw_ref.numpy()))
        for k in range(4):
            assert abs(gpb[i][k] - float(gp_ref[k])) < 1e-3 * abs(float(gp_ref[k])) + 1e-9, (i, k)


def test_batch_of_one_is_the_single_handle(dhp):
    n = 32
    w = to_gpu(si.white_noise(n, seed=5))
    a = dhp.Sim(dhp.default_config(n=n, box=10.0, subgrid=2, batch=1))
    c = dhp.Sim(dhp.default_config(n=n, box=10.0, subgrid=2))
    for s in (a, c):
        s.init_from_noise(w)
        for _ in range(3):
            s.step()
    assert torch.equal(a.get("q"), c.get("q"))

"""Benchmark of the MI355X path: cell-updates/s of the full time step (forward with
checkpoints plus the reverse pass) at 256^3 cells + 256^3 dark-matter particles, the
forward-only rate, the same over a whole run a = 0.01 -> 0.29, the HBM roofline of the
dominant kernel (the hydro sweep adjoint) and of the whole step (algorithmic bytes per
cell-step recounted from the kernels), the error of the first step against the FP64 oracle,
the oracle itself timed on this host's cores, the learned star-formation closure against
the plain source term (its training, its step rates, and the distance of its final fields
from the plain run's), and the batched parameter sampler (64 samples of 64^3 with their own
seeds, star-formation parameters and step counts, forward + reverse in shared launches)
against running the same samples one after another.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
SWEEP_FLOPS_PER_CELL = 236           # FP32 operations of one sweep per cell (FMA = 2)
SWEEP_BYTES_PER_CELL = 40            # read Q, write Q
SWEEP_VJP_BYTES_PER_CELL = 60        # read Q, read lambda_out, write lambda_in
SWEEP_VJP_KICK_BYTES_PER_CELL = 16   # the first of a step's three also reads g4 (the kick)
# Algorithmic HBM bytes per cell (one particle per cell) of one step, recounted from the
# kernels a step launches: every array a kernel must read or write, once.
FWD_BYTES = [
    ("kick+drift: x, p read and written, key written, g4 read", 68),
    ("first sweep with the opening gas kick: Q read and written, g4 read", 56),
    ("second and third sweeps: Q read and written", 80),
    ("sort: histogram 8, scan 8, scatter 12, bin sort 8, gather of x 32", 68),
    ("deposit: bin starts, sorted x, rho_gas read, delta written", 28),
    ("FFT Poisson: r2c, y, z with Green's function, y, c2r passes", 64),
    ("gradient: phi read, g4 written", 20),
    ("closing pass: Q read and written, g4 read, star read and written", 64),
]
REV_BYTES = [
    ("source, closing-kick and next opening-kick adjoints", 120),
    ("gather of lambda_p into bin order", 32),
    ("vector deposit of the kick adjoint", 60),
    ("gradient adjoint (two fields)", 28),
    ("FFT Poisson of the potential adjoint", 64),
    ("density adjoint added to lambda_rho", 12),
    ("position adjoint of kicks, deposit and drift", 80),
    ("three sweep adjoints (the first re-applies the opening kick: g4 read)", 196),
    ("gradient of the step's start potential", 20),
]
MODEL_FWD_BYTES = 340                # the byte model the >= 50% target is stated in
MODEL_FWD_BWD_BYTES = 1180
N = 256
BOX = 40.0           # Mpc/h: cell size 0.156 Mpc/h, as the 128^3 / 20 Mpc/h box
A_INIT = 0.01


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=8)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=N)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mlp", action="store_true", help="skip the learned-closure comparison")
    p.add_argument("--mlp-samples", type=int, default=1 << 24)
    p.add_argument("--no-batch", action="store_true", help="skip the batched-sampler comparison")
    p.add_argument("--batch-samples", type=int, default=64)
    p.add_argument("--no-full-run", action="store_true", help="skip the whole run a -> 0.29")
    p.add_argument("--no-dual", action="store_true", help="skip the dual-energy timing")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def counter_record(name):
    """A record of rocprofv3 counters of 256^3 launches (profiles/<name>), or None when the
    kernel sources it names have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh)
    for src_name, digest in doc.get("sources_sha256", {}).items():
        src = os.path.join(ROOT, "paper_2502_02294_amd", "csrc", src_name)
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    return doc


def time_fwd_bwd(torch, s, white, sched, target, steps):
    """Seconds of one forward + loss + reverse pass over the schedule, after an untimed one."""
    for timed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_schedule(sched)
        k = s.forward(white, 1.0)
        s.loss(target)
        s.backward()
        torch.cuda.synchronize()
        assert k == steps
    return time.perf_counter() - t0


def time_steps(torch, s, white, steps, warmup):
    """(forward-only seconds, forward + loss + reverse seconds with what device memory lets
    the forward keep, the same with every checkpoint segment recomputed, the schedule, the
    steps the forward taped) of `steps` steps from the initial conditions of `white`, after
    `warmup` untimed steps / one untimed pass of the full path."""
    s.init_from_noise(white)
    s.run_steps(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert s.run_steps(steps) == steps
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s.init_from_noise(white)
    s.run_steps(steps)
    sched = s.get_schedule()
    target = s.get("flux").clone()
    t_fb = time_fwd_bwd(torch, s, white, sched, target, steps)
    taped = s.store_info()
    s.set_store_limit(0)
    t_fb_recompute = time_fwd_bwd(torch, s, white, sched, target, steps)
    s.set_store_limit(-1)
    return t_fwd, t_fb, t_fb_recompute, sched, taped


def mlp_comparison(torch, dhp, white, n, box, steps, warmup, samples):
    """Learned closure vs the plain source term at the same size.  Without cooling the gas
    denser than the default threshold is hot at this resolution and forms almost no stars,
    so the comparison uses thresholds under which stars form (Delta_c = 10, T_c = 1e7 K,
    eps_sf = 0.03); the network is trained for them on `samples` states of the plain term."""
    prm = dhp.default_params(eps_sf=0.03, delta_c=10.0, t_c=1e7)
    net = dhp.Mlp(seed=1)
    x, y = net.sample(samples, seed=7, params=prm,
                      opts=dhp.mlp.sample_defaults(dc_lo=5.0, dc_hi=20.0))
    opts = dhp.mlp.train_defaults()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(x, y, opts)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, y
    theta = net.weights()
    log(f"bench: closure trained in {t_train:.2f} s, objective {hist[-100:].mean():.4g}")
    rates = {}
    for name, clo in (("plain", 0), ("mlp", 1)):
        cfg = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2, closure=clo,
                                 ckpt_every=max(1, steps))
        s = dhp.Sim(cfg, prm)
        if clo:
            s.set_closure(theta)
        t_fwd, t_fb, _, _, _ = time_steps(torch, s, white, steps, warmup)
        rates[name] = (n ** 3 * steps / t_fwd, n ** 3 * steps / t_fb)
        s.close()
        log(f"bench: {name} source term: forward {t_fwd * 1e3 / steps:.2f} ms/step, "
            f"fwd+bwd {t_fb * 1e3 / steps:.2f} ms/step")
    # the same pair over the whole run a = 0.01 -> 0.29 (CFL steps, checkpoints every 16
    # steps): the late steps have more cells where stars can form, and the closure's adjoint
    # skips the network's backward only for groups of 32 cells where none can
    whole = {}
    for name, clo in (("plain", 0), ("mlp", 1)):
        cfg = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2, closure=clo,
                                 ckpt_every=16)
        s = dhp.Sim(cfg, prm)
        if clo:
            s.set_closure(theta)
        sec, k, _ = full_run(torch, s, white)
        whole[name] = (sec, k)
        s.close()
        log(f"bench: {name} source term, whole run: {k} steps, forward + reverse "
            f"{sec * 1e3 / k:.2f} ms/step")
    finals = {}
    # "nudged": the plain term with eps_sf changed by one part in a million, the distance a
    # run keeps from itself under a perturbation far below any closure's error (the flow's
    # own sensitivity: the floor of every distance below)
    prm_nudged = dhp.default_params(eps_sf=0.03 * (1.0 + 1e-6), delta_c=10.0, t_c=1e7)
    for name, sub, clo in (("plain", 2, 0), ("mlp", 2, 1), ("off", 0, 0), ("nudged", 2, 0)):
        s = dhp.Sim(dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=sub, closure=clo),
                    prm_nudged if name == "nudged" else prm)
        if clo:
            s.set_closure(theta)
        s.init_from_noise(white)
        k = s.run_to(0.29)
        finals[name] = (s.get("rho").double(), s.get("temp").double().log(),
                        float(s.get("star").double().sum()), k)
        if name == "plain":
            # the network against the plain term on every cell of the state the run reached:
            # ln pi0 of a step of dt = 0.002 where the gates are open (o1 > -10)
            xs, ys = s.closure_states()
            o = net.eval(xs).double()
            t = ys.double()
            dt = 0.002
            lp_net = torch.log(-torch.expm1(-torch.exp(o[0]) * dt)) + torch.clamp(o[1], max=0.0)
            lp_ref = torch.log(-torch.expm1(-torch.exp(t[0]) * dt)) + t[1]
            err = (lp_net - lp_ref).abs()[t[1] > -10.0]
            lp_stats = {"cells": int(err.numel()), "median": float(err.median()),
                        "mean": float(err.mean()),
                        "p99": float(torch.quantile(err[:1 << 24].float(), 0.99))}
            del xs, ys, o, t
        s.close()

    def rel(a, b):
        return float((a - b).norm() / b.norm())

    p = finals["plain"]
    return {
        "fwd_cell_updates_per_s": rates["mlp"][0],
        "fwd_bwd_cell_updates_per_s": rates["mlp"][1],
        "plain_fwd_cell_updates_per_s": rates["plain"][0],
        "plain_fwd_bwd_cell_updates_per_s": rates["plain"][1],
        "fwd_time_ratio_vs_plain": rates["plain"][0] / rates["mlp"][0],
        "fwd_bwd_time_ratio_vs_plain": rates["plain"][1] / rates["mlp"][1],
        "whole_run": {"what": f"forward + loss + reverse over a = {A_INIT} -> 0.29 with CFL "
                              "steps, checkpoints every 16 steps",
                      "steps_plain": whole["plain"][1], "steps_mlp": whole["mlp"][1],
                      "plain_ms_per_step": whole["plain"][0] * 1e3 / whole["plain"][1],
                      "mlp_ms_per_step": whole["mlp"][0] * 1e3 / whole["mlp"][1],
                      "fwd_bwd_time_ratio_vs_plain":
                          (whole["mlp"][0] / whole["mlp"][1]) /
                          (whole["plain"][0] / whole["plain"][1])},
        "train": {"samples": samples, "steps": int(opts.steps), "batch": int(opts.batch),
                  "seconds": t_train, "objective_start": float(np.mean(hist[:10])),
                  "objective_end": float(np.mean(hist[-100:]))},
        "accuracy": {"run": f"a = {A_INIT} -> 0.29, {p[3]} steps, relaxed star formation, "
                            "Delta_c = 10, T_c = 1e7 K, eps_sf = 0.03",
                     "rel_l2_rho_vs_plain": rel(finals["mlp"][0], p[0]),
                     "rel_l2_lnT_vs_plain": rel(finals["mlp"][1], p[1]),
                     "no_source_rel_l2_rho_vs_plain": rel(finals["off"][0], p[0]),
                     "no_source_rel_l2_lnT_vs_plain": rel(finals["off"][1], p[1]),
                     "nudged_rel_l2_rho_vs_plain": rel(finals["nudged"][0], p[0]),
                     "nudged_rel_l2_lnT_vs_plain": rel(finals["nudged"][1], p[1]),
                     "stars_plain": p[2], "stars_mlp": finals["mlp"][2],
                     "abs_err_ln_pi0_on_run_states": lp_stats},
    }


def batch_comparison(torch, dhp, si, samples):
    """Batched parameter sampler: `samples` samples of 64^3 cells + particles in 10 Mpc/h
    boxes, white noise from seeds 1000 + s, (eps_sf, Delta_c) drawn uniformly within +-50% of
    (0.02, 100) (seed 8), relaxed star formation, each stepping by its own CFL from a = 0.01
    to 0.29; forward with checkpoints, per-sample loss against the flux field of seeds 2000 + s,
    reverse pass.  Timed as one batch and as the same samples run one after another."""
    n, box, a_final, K = 64, 10.0, 0.29, 16
    rng = np.random.default_rng(8)
    eps = 0.02 * rng.uniform(0.5, 1.5, samples)
    dcs = 100.0 * rng.uniform(0.5, 1.5, samples)
    white = torch.from_numpy(np.stack([si.white_noise(n, 1000 + i) for i in range(samples)])).cuda()
    white_t = torch.from_numpy(np.stack([si.white_noise(n, 2000 + i)
                                         for i in range(samples)])).cuda()
    b = dhp.Sim(dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2, batch=samples,
                                   ckpt_every=K))
    for i in range(samples):
        b.set_sample_params(i, eps_sf=float(eps[i]), delta_c=float(dcs[i]))
    t0 = time.perf_counter()
    kt = b.forward(white_t, a_final)
    target = b.get("flux").clone()
    torch.cuda.synchronize()
    log(f"bench: batch target run: {kt} lockstep steps, {time.perf_counter() - t0:.2f} s")
    b.forward(white, a_final)                  # warm-up of the full path
    b.loss(target)
    b.backward()
    torch.cuda.synchronize()
    log(f"bench: batch warm-up done, {time.perf_counter() - t0:.2f} s")
    t0 = time.perf_counter()
    k = b.forward(white, a_final)
    losses = b.loss(target)
    gw, gp = b.backward()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    steps = [len(b.get_sample_schedule(i)) for i in range(samples)]
    b.close()
    log(f"bench: batch of {samples}: {k} lockstep steps, per-sample {min(steps)}..{max(steps)}, "
        f"fwd+bwd {t_batch:.2f} s")
    # the same samples one at a time, each after an untimed pass of its own (as the batch:
    # the device buffers of a handle are allocated by its first pass)
    t_seq = 0.0
    seq_steps = []
    for i in range(samples):
        s = dhp.Sim(dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2, ckpt_every=K,
                                       sf_seed=102 + i),
                    dhp.default_params(eps_sf=float(eps[i]), delta_c=float(dcs[i])))
        for timed in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.forward(white[i].contiguous(), a_final)
            s.loss(target[i].contiguous())
            s.backward()
            torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        seq_steps.append(len(s.get_schedule()))
        if i % 8 == 7:
            log(f"bench: sequential samples {i + 1}/{samples}, {t_seq:.2f} s")
        s.close()
    assert seq_steps == steps
    log(f"bench: the same {samples} samples one after another: {t_seq:.2f} s")
    cells = float(n ** 3) * sum(steps)
    return {
        "workload": f"{samples} samples x (64^3 cells + 64^3 DM particles), 10 Mpc/h boxes, "
                    "white-noise seeds 1000+s, eps_sf and Delta_c uniform within +-50% of "
                    "(0.02, 100) (seed 8), relaxed star formation, own CFL steps a = 0.01 -> "
                    "0.29, checkpointed forward + per-sample flux loss + reverse pass",
        "fwd_bwd_cell_updates_per_s": cells / t_batch,
        "sequential_fwd_bwd_cell_updates_per_s": cells / t_seq,
        "speedup_vs_sequential": t_seq / t_batch,
        "seconds": t_batch,
        "sequential_seconds": t_seq,
        "lockstep_steps": k,
        "steps_min": min(steps), "steps_max": max(steps), "steps_total": sum(steps),
        "ckpt_every": K,
        "mean_abs_dL_deps_sf": float(np.mean([abs(g[2]) for g in gp])),
        "mean_abs_dL_ddelta_c": float(np.mean([abs(g[3]) for g in gp])),
        "mean_loss": float(np.mean(losses)),
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_fwd_bwd_rate(n, box, threads, min_seconds):
    """Cell-updates/s of forward + reverse steps of the FP64 oracle (the step, the flux loss,
    torch.autograd back to the step's gas, particles and potential and to the parameters) at
    n^3 on `threads` host threads: one untimed step (the first touch of its memory), then
    timed steps until min_seconds have passed.  Returns (rate, timed steps, seconds)."""
    import torch
    import synth_inputs as si
    from oracle import sim as osim, subgrid
    torch.set_num_threads(threads)
    cfg = osim.default_config(n=n, box=box, a_init=A_INIT, subgrid=subgrid.MODE_RELAXED)
    w = torch.from_numpy(si.white_noise(n, 6)).double()
    target = torch.from_numpy(si.white_noise(n, 7)).double().abs() * 0.1 + 0.5
    with torch.no_grad():
        st0 = osim.initial_state(w, cfg)
        dt = osim.cfl_dt(st0, cfg)

    def one():
        th = torch.tensor([0.3, 1.6, 0.02, 100.0], dtype=torch.float64, requires_grad=True)
        prm = osim.Params(A=th[0], beta=th[1], eps_sf=th[2], delta_c=th[3])
        leaves = [v.clone().requires_grad_(True) for v in (st0.q, st0.x, st0.p, st0.phi)]
        st = osim.State(q=leaves[0], x=leaves[1], p=leaves[2], star=st0.star, phi=leaves[3],
                        t=st0.t, a=st0.a, step=st0.step)
        out = osim.step(st, cfg, prm, dt)
        L = osim.loss(out, target, cfg, th[0], th[1])
        torch.autograd.grad(L, leaves + [th])

    one()
    k, t0 = 0, time.perf_counter()
    while k < 2 or time.perf_counter() - t0 < min_seconds:
        one()
        k += 1
    el = time.perf_counter() - t0
    return n ** 3 * k / el, k, el


def cpu_baseline(n, box, gpu_first_step):
    """The FP64 oracle on this host's cores.  The headline sample: one forward + reverse step
    at 128^3 on all threads; beside it the same at 64^3 on one thread, and one forward step at
    the benchmarked size, which also gives the error of the GPU's first step against it."""
    import torch
    import synth_inputs as si
    from oracle import sim as osim, subgrid
    threads = torch.get_num_threads()
    n_fb = min(n, 64)
    v_all, k_all, el_all = oracle_fwd_bwd_rate(n_fb, box * n_fb / n, threads, 6.0)
    log(f"bench: oracle fwd+bwd {n_fb}^3 on {threads} threads: {k_all} steps {el_all:.1f} s")
    v_one, k_one, el_one = oracle_fwd_bwd_rate(n_fb, box * n_fb / n, 1, 6.0)
    log(f"bench: oracle fwd+bwd {n_fb}^3 on 1 thread: {k_one} steps {el_one:.1f} s")
    torch.set_num_threads(threads)
    cfg = osim.default_config(n=n, box=box, a_init=A_INIT, subgrid=subgrid.MODE_RELAXED)
    with torch.no_grad():
        st = osim.initial_state(torch.from_numpy(si.white_noise(n, 6)).double(), cfg)
        dt = osim.cfl_dt(st, cfg)
        t0 = time.perf_counter()
        ref = osim.step(st, cfg, osim.Params(), dt)
        el = time.perf_counter() - t0
    log(f"bench: oracle forward step {n}^3 {el:.1f} s")
    errors = None
    if gpu_first_step is not None:
        got, gpu_dt = gpu_first_step
        errors = {"dt_rel": abs(gpu_dt - dt) / dt}
        refs = {f"q{c}": ref.q[c].numpy() for c in range(5)}
        refs.update(mom=ref.p.numpy(), phi=ref.phi.numpy(), star=ref.star.numpy())
        for k, r in refs.items():
            g = got[k]
            nr = float(np.linalg.norm(r))
            errors[k] = float(np.linalg.norm(g - r) / (nr if nr > 0 else 1.0))
    return {"value": v_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"forward + reverse steps (relaxed star formation, flux loss, "
                      f"torch.autograd) of the FP64 oracle at {n_fb}^3 ({box * n_fb / n:g} "
                      f"Mpc/h, the benchmark's cell size) from a = {A_INIT}: {k_all} timed "
                      f"steps, {el_all:.1f} s on {threads} threads, after one untimed step",
            "cpu_model": cpu_model(),
            "one_core": {"value": v_one, "cores": 1,
                         "sample": f"the same on 1 thread: {k_one} steps, {el_one:.1f} s"},
            "forward_step": {"value": n ** 3 / el, "cores": threads,
                             "sample": f"one forward step at {n}^3, {el:.1f} s"}}, errors


def gpu_first_step(torch, dhp, white, n, box):
    """The fields after the first CFL step of the benchmark workload on the GPU (for its error
    against the oracle's step), and the step's dt."""
    cfg = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2)
    s = dhp.Sim(cfg)
    s.init_from_noise(white)
    dt, _ = s.step()
    q = s.get("q").double().cpu().numpy()
    out = {f"q{c}": q[c] for c in range(5)}
    out.update(mom=s.get("mom").double().cpu().numpy(), phi=s.get("phi").double().cpu().numpy(),
               star=s.get("star").double().cpu().numpy())
    s.close()
    return out, dt


def full_run(torch, s, white, a_final=0.29):
    """Forward + loss + reverse over a whole run from a = 0.01 to a_final with CFL steps
    (checkpoints every cfg.ckpt_every steps, the reverse pass's data chosen by the free device
    memory); timed after an untimed pass.  Returns (seconds, steps, (taped, sorted))."""
    s.init_from_noise(white)
    s.run_to(a_final)
    target = s.get("flux").clone()
    s.set_schedule([])
    for timed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = s.forward(white, a_final)
        s.loss(target)
        s.backward()
        torch.cuda.synchronize()
    return time.perf_counter() - t0, k, s.store_info()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method is "
              "benchmarked on a single MI355X", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2502_02294_amd as dhp
    import synth_inputs as si

    n = args.n
    nc = n ** 3
    box = BOX * n / N
    cfg = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2,
                             ckpt_every=max(1, args.steps))
    s = dhp.Sim(cfg)
    white = torch.from_numpy(si.white_noise(n, 6)).cuda()
    log(f"bench: n={n} steps={args.steps} warmup={args.warmup}")

    t_fwd, t_fb, t_fb_rc, sched, taped = time_steps(torch, s, white, args.steps, args.warmup)
    log(f"bench: forward {args.steps} steps {t_fwd * 1e3:.1f} ms")
    log(f"bench: forward+backward {args.steps} steps {t_fb * 1e3:.1f} ms "
        f"({taped[0]} taped by the forward, {taped[1]} with a kept sort); every segment "
        f"recomputed {t_fb_rc * 1e3:.1f} ms")

    # dominant kernel of the forward + reverse step: the sweep adjoint (three launches per
    # step, about a fifth of the step), 60 algorithmic bytes per cell and launch (76 for the
    # first, which reads g4 to re-apply the opening kick); beside it
    # the forward sweeps, 40 bytes and 236 FP32 operations per cell and launch.  Their
    # launches inside one more forward + loss + reverse pass of the same steps are timed by
    # the library with HIP events on the stream it launches them on.
    from paper_2502_02294_amd import _lib as dhl
    kt = {}
    for fam in (dhl.KTIME_SWEEP_VJP, dhl.KTIME_SWEEP, dhl.KTIME_SWEEP_KICK):
        s.set_kernel_timing(fam)
        time_fwd_bwd(torch, s, white, sched, s.get("flux").clone(), args.steps)
        kt[fam] = s.kernel_timing()
        s.set_kernel_timing(-1)
    (n_vjp, t_vjp), (n_sweep, t_sweep), (n_kick, t_kick) = (
        kt[dhl.KTIME_SWEEP_VJP], kt[dhl.KTIME_SWEEP], kt[dhl.KTIME_SWEEP_KICK])
    log(f"bench: in-step launches: sweep adjoint {n_vjp} x {t_vjp * 1e6:.1f} us, second/third "
        f"sweeps {n_sweep} x {t_sweep * 1e6:.1f} us, kicking first sweep {n_kick} x "
        f"{t_kick * 1e6:.1f} us")
    # mean over a step's three launches
    vjp_bytes = (SWEEP_VJP_BYTES_PER_CELL + SWEEP_VJP_KICK_BYTES_PER_CELL / 3.0) * nc
    vjp_gbs = vjp_bytes / t_vjp / 1e9
    rec = counter_record("sweep_vjp_256_traffic.json") if n == N else None
    traffic = float(rec["traffic_bytes_per_launch"]) if rec else None
    sweep_gbs = SWEEP_BYTES_PER_CELL * nc / t_sweep / 1e9
    sweep_tflops = SWEEP_FLOPS_PER_CELL * nc / t_sweep / 1e12

    # whole run a = 0.01 -> 0.29 at the benchmarked size
    if not args.no_full_run:
        cfg_run = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2, ckpt_every=16)
        s_run = dhp.Sim(cfg_run)
        t_run, k_run, taped_run = full_run(torch, s_run, white)
        s_run.close()
        log(f"bench: whole run a = {A_INIT} -> 0.29: {k_run} steps, fwd+bwd {t_run:.2f} s "
            f"({taped_run[0]} taped, {taped_run[1]} with a kept sort)")
    first = gpu_first_step(torch, dhp, white, n, box) if not args.no_cpu_baseline else None

    fwd_b = sum(b for _, b in FWD_BYTES)
    rev_b = sum(b for _, b in REV_BYTES)
    fb_b = fwd_b + rev_b
    rate_fwd = nc * args.steps / t_fwd
    rate_fb = nc * args.steps / t_fb

    def frac(bytes_per_cell, rate):
        return bytes_per_cell * rate / (HBM_PEAK_GBS * 1e9)

    out = {
        "metric": "cell-updates/s fwd+bwd at 256^3 (forward with checkpoints + reverse pass)",
        "value": rate_fb,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_fb / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 cells + {n}^3 DM particles, {box:g} Mpc/h box, "
                               "BBKS Gaussian random field at a=0.01, relaxed stochastic star "
                               "formation, checkpointed forward + flux loss + reverse pass",
                   "n": n, "box_mpc_h": box, "ckpt_every": int(cfg.ckpt_every),
                   "reverse_data": "capacity-chosen: the forward taped "
                                   f"{taped[0]} of {args.steps} steps, kept the sort of "
                                   f"{taped[1]} more; the rest recomputed from checkpoints"},
        "fwd_bwd_recompute_all": {"value": nc * args.steps / t_fb_rc,
                                  "ms_per_step": t_fb_rc / args.steps * 1e3,
                                  "what": "the same with every checkpoint segment recomputed "
                                          "(nothing kept by the forward)"},
        "fwd_cell_updates_per_s": rate_fwd,
        "fwd_ms_per_step": t_fwd / args.steps * 1e3,
        "full_run": None if args.no_full_run else {
            "what": f"whole run a = {A_INIT} -> 0.29 with CFL steps, checkpoint every 16 steps, "
                    "forward + flux loss + reverse pass",
            "steps": k_run, "seconds": t_run, "ms_per_step": t_run / k_run * 1e3,
            "cell_updates_per_s": nc * k_run / t_run,
            "taped_steps": taped_run[0], "sorted_steps": taped_run[1]},
        "roofline": {"bound": "hbm", "achieved": vjp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": vjp_gbs / HBM_PEAK_GBS,
                     "traffic": traffic / t_vjp / 1e9 if traffic else None,
                     "kernel": "hydro sweep adjoint (sweep_x_vjp_kernel, "
                               "sweep_walk_vjp_kernel<1>, <2>): mean of its launches inside "
                               "a forward + reverse pass",
                     "launches": n_vjp, "ms_per_launch": t_vjp * 1e3,
                     "algorithmic_bytes_per_launch": vjp_bytes,
                     "traffic_bytes_per_launch": traffic},
        "forward_sweep": {"bound": "hbm", "achieved": sweep_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": sweep_gbs / HBM_PEAK_GBS,
                          "algorithmic_bytes_per_launch": SWEEP_BYTES_PER_CELL * nc,
                          "alu_tflops": sweep_tflops,
                          "alu_frac": sweep_tflops / FP32_VECTOR_PEAK_TFLOPS,
                          "kernel": "second and third hydro sweeps of a step (sweep_x_kernel"
                                    "<false>, sweep_walk_kernel<1|2, false, ·>)",
                          "launches": n_sweep, "ms_per_launch": t_sweep * 1e3,
                          "kicking_first_sweep_ms_per_launch": t_kick * 1e3},
        "step_roofline": {
            "peak_gbs": HBM_PEAK_GBS,
            "forward": {"bytes_per_cell_step_recount": fwd_b,
                        "frac_recount": frac(fwd_b, rate_fwd),
                        "bytes_per_cell_step_model": MODEL_FWD_BYTES,
                        "frac_model": frac(MODEL_FWD_BYTES, rate_fwd)},
            "fwd_bwd": {"bytes_per_cell_step_recount": fb_b,
                        "frac_recount": frac(fb_b, rate_fb),
                        "bytes_per_cell_step_model": MODEL_FWD_BWD_BYTES,
                        "frac_model": frac(MODEL_FWD_BWD_BYTES, rate_fb)},
            "recount": {"forward": dict(FWD_BYTES), "reverse": dict(REV_BYTES)}},
    }
    s.close()
    if not args.no_dual:
        # the dual-energy formalism (entropy as a sixth gas component) on the same steps
        cfg_d = dhp.default_config(n=n, box=box, a_init=A_INIT, subgrid=2,
                                   ckpt_every=max(1, args.steps), dual_energy=1)
        s_d = dhp.Sim(cfg_d)
        td_fwd, td_fb, _, _, _ = time_steps(torch, s_d, white, args.steps, args.warmup)
        s_d.close()
        log(f"bench: dual energy: forward {td_fwd * 1e3 / args.steps:.2f} ms/step, fwd+bwd "
            f"{td_fb * 1e3 / args.steps:.2f} ms/step")
        out["dual_energy"] = {"fwd_ms_per_step": td_fwd / args.steps * 1e3,
                              "fwd_bwd_ms_per_step": td_fb / args.steps * 1e3,
                              "fwd_time_ratio_vs_plain": td_fwd / t_fwd,
                              "fwd_bwd_time_ratio_vs_plain": td_fb / t_fb}
    if not args.no_mlp:
        log("bench: learned closure vs plain source term")
        out["mlp_closure"] = mlp_comparison(torch, dhp, white, n, box, args.steps,
                                            args.warmup, args.mlp_samples)
    if not args.no_batch:
        log("bench: batched parameter sampler vs one sample at a time")
        bs = batch_comparison(torch, dhp, si, args.batch_samples)
        # the plain path over the same whole run (a = 0.01 -> 0.29, the same cell size): both
        # include the late, clustered steps, whose particle kernels cost more than the early
        # steps of `value`
        if out.get("full_run"):
            fr = out["full_run"]["cell_updates_per_s"]
            bs["plain_256_full_run_fwd_bwd_cell_updates_per_s"] = fr
            bs["rate_vs_plain_256_full_run"] = bs["fwd_bwd_cell_updates_per_s"] / fr
        out["batched_sampler"] = bs
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(n, box, first)
        out["error_vs_oracle_what"] = ("relative L2 of every field after the first CFL step of "
                                       "the benchmark workload, GPU (FP32) against the FP64 "
                                       "oracle from the same white noise")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

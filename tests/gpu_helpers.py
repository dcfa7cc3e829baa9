"""Helpers shared by the GPU parity tests: conversions between the oracle's float64 state
and the library's float32 buffers, and error measures."""

import numpy as np
import torch

from oracle import sim as osim


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def round32(t):
    """A float64 tensor rounded through float32 (both sides then start from equal values)."""
    return t.detach().float().double()


def rounded_state(st):
    return osim.State(q=round32(st.q), x=round32(st.x), p=round32(st.p), star=round32(st.star),
                      phi=round32(st.phi), t=st.t, a=st.a, step=st.step)


def load_state(sim, st):
    """Put an oracle state (already float32-representable) into the GPU handle."""
    sim.set("q", to_gpu(st.q.numpy()))
    sim.set("pos", to_gpu(st.x.numpy()))
    sim.set("mom", to_gpu(st.p.numpy()))
    sim.set("star", to_gpu(st.star.numpy()))
    sim.set_time(st.a, st.step)
    sim.set("phi", to_gpu(st.phi.numpy()))


def displacement_err(pos_gpu, pos_ref, n, scale):
    d = (np.asarray(pos_gpu, dtype=np.float64) - np.asarray(pos_ref, dtype=np.float64) + n / 2) % n - n / 2
    return np.linalg.norm(d) / scale


def gpu_config(ocfg, **kw):
    """Library configuration equal to an oracle configuration."""
    from paper_2502_02294_amd import default_config
    return default_config(n=ocfg.n, box=ocfg.box, omega_m=ocfg.omega_m, omega_b=ocfg.omega_b,
                          h=ocfg.h, sigma8=ocfg.sigma8, n_s=ocfg.n_s, gamma=ocfg.gamma, mu=ocfg.mu,
                          a_init=ocfg.a_init, t_init=ocfg.t_init, cfl=ocfg.cfl,
                          dlna_max=ocfg.dlna_max, t_floor=ocfg.t_floor, subgrid=ocfg.subgrid,
                          tau=ocfg.tau, sf_seed=ocfg.sf_seed, **kw)


def gpu_params(p):
    from paper_2502_02294_amd import default_params
    return default_params(A=p.A, beta=p.beta, eps_sf=p.eps_sf, delta_c=p.delta_c, t_c=p.t_c,
                          e0=p.e0, w_rho=p.w_rho, w_t=p.w_t)

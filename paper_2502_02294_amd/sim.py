"""Python face of libdiffhydro: a handle over the C ABI with PyTorch tensors for device
memory.  Every computation runs in the library's HIP kernels; this module only checks
shapes and passes pointers."""

import ctypes

import torch

from . import _lib
from ._lib import (FIELD_FLUX, FIELD_MOM, FIELD_OBS_TEMP, FIELD_PHI, FIELD_POS, FIELD_Q,
                   FIELD_RHO, FIELD_STAR, FIELD_STAR_DM, FIELD_TEMP, Config, Params, check, lib)

_FIELD_SHAPE = {FIELD_Q: (5,), FIELD_RHO: (), FIELD_POS: (3,), FIELD_MOM: (3,), FIELD_STAR: (),
                FIELD_PHI: (), FIELD_TEMP: (), FIELD_FLUX: (), FIELD_STAR_DM: (),
                FIELD_OBS_TEMP: ()}
FIELDS = {"q": FIELD_Q, "rho": FIELD_RHO, "pos": FIELD_POS, "mom": FIELD_MOM, "star": FIELD_STAR,
          "phi": FIELD_PHI, "temp": FIELD_TEMP, "flux": FIELD_FLUX, "star_dm": FIELD_STAR_DM,
          "obs_temp": FIELD_OBS_TEMP}


def default_config(**kw):
    c = Config()
    lib().dh_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def default_params(**kw):
    p = Params()
    lib().dh_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(t, dtype=torch.float32, numel=None):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _host_floats(values, count):
    """ctypes float array of exactly `count` values (from a sequence, numpy or CPU tensor)."""
    vals = [float(v) for v in (values.tolist() if hasattr(values, "tolist") else values)]
    if len(vals) != count:
        raise ValueError(f"expected {count} values, got {len(vals)}")
    return (ctypes.c_float * count)(*vals)


class Sim:
    """One simulation handle on the current HIP device.  With config.batch = S > 1 it holds
    S independent samples: fields, white noise, targets and gradients then carry a leading
    sample dimension, and losses and parameter gradients are per sample."""

    def __init__(self, config=None, params=None, **cfg_kw):
        self.cfg = config if config is not None else default_config(**cfg_kw)
        self.n = int(self.cfg.n)
        self.S = max(1, int(self.cfg.batch))
        self.nc = self.n ** 3
        self.nq = 6 if self.cfg.dual_energy else 5   # gas components (dual energy: entropy)
        self._h = ctypes.c_void_p()
        torch.cuda.init()
        check(lib().dh_create(ctypes.byref(self.cfg), ctypes.byref(self._h)))
        self._stream_handle = None
        self._stream()
        self.params = params if params is not None else default_params()
        self.set_params(self.params)

    def close(self):
        if self._h:
            lib().dh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        check(rc, self._h)

    def _stream(self):
        """Enqueue the library's work on torch's current stream, so that it is ordered with
        the tensors passed in and out (allocation, copies, reuse by the caching allocator)."""
        stream = torch.cuda.current_stream().cuda_stream
        if stream != self._stream_handle:
            check(lib().dh_set_stream(self._h, ctypes.c_void_p(stream)), self._h)
            self._stream_handle = stream

    def set_params(self, p=None, **kw):
        self._stream()
        if p is None:
            p = self.params
        for k, v in kw.items():
            setattr(p, k, v)
        self.params = p
        self._check(lib().dh_set_params(self._h, ctypes.byref(p)))

    def _lead(self):
        return (self.S,) if self.S > 1 else ()

    def set_sample_params(self, sample, p=None, **kw):
        """Star-formation parameters of one sample (A, beta stay the shared ones)."""
        self._stream()
        if p is None:
            p = default_params()
            for f, _ in type(p)._fields_:
                setattr(p, f, getattr(self.params, f))
        for k, v in kw.items():
            setattr(p, k, v)
        self._check(lib().dh_set_sample_params(self._h, sample, ctypes.byref(p)))

    def set_sample_schedule(self, sample, dts):
        self._stream()
        arr = (ctypes.c_double * max(1, len(dts)))(*[float(x) for x in dts])
        self._check(lib().dh_set_sample_schedule(self._h, sample, arr, len(dts)))

    def get_sample_schedule(self, sample):
        self._stream()
        n = ctypes.c_int32()
        self._check(lib().dh_get_sample_schedule(self._h, sample, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_double * max(1, n.value))()
        self._check(lib().dh_get_sample_schedule(self._h, sample, arr, n.value, ctypes.byref(n)))
        return list(arr[:n.value])

    def sample_times(self):
        """(a, t) of every sample."""
        self._stream()
        a = (ctypes.c_double * self.S)()
        t = (ctypes.c_double * self.S)()
        self._check(lib().dh_get_sample_times(self._h, a, t))
        return list(a), list(t)

    def set_closure(self, theta):
        """Weights of the learned closure (flat float vector of DH_MLP_NPARAMS values; a
        simulation created with closure=CLOSURE_MLP needs them before its first step)."""
        self._stream()
        arr = _host_floats(theta, _lib.MLP_NPARAMS)
        self._check(lib().dh_set_closure(self._h, arr))

    def init_from_seed(self, seed):
        self._stream()
        self._check(lib().dh_init_from_seed(self._h, ctypes.c_uint64(seed)))

    def init_from_noise(self, white):
        self._stream()
        self._check(lib().dh_init_from_noise(self._h, _ptr(white, numel=self.S * self.nc)))

    def step(self):
        self._stream()
        dt, a = ctypes.c_double(), ctypes.c_double()
        self._check(lib().dh_step(self._h, ctypes.byref(dt), ctypes.byref(a)))
        return dt.value, a.value

    def run_to(self, a_final):
        self._stream()
        k = ctypes.c_int32()
        self._check(lib().dh_run_to(self._h, a_final, ctypes.byref(k)))
        return k.value

    def run_steps(self, nsteps):
        """nsteps steps in one call (the same results as that many step() calls)."""
        self._stream()
        k = ctypes.c_int32()
        self._check(lib().dh_run_steps(self._h, int(nsteps), ctypes.byref(k)))
        return k.value

    def set_schedule(self, dts):
        self._stream()
        arr = (ctypes.c_double * len(dts))(*[float(x) for x in dts])
        self._check(lib().dh_set_schedule(self._h, arr, len(dts)))

    def get_schedule(self):
        self._stream()
        n = ctypes.c_int32()
        self._check(lib().dh_get_schedule(self._h, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_double * max(1, n.value))()
        self._check(lib().dh_get_schedule(self._h, arr, n.value, ctypes.byref(n)))
        return list(arr[:n.value])

    def get(self, name):
        self._stream()
        f = FIELDS[name]
        shape = (self.nq,) if f == FIELD_Q else _FIELD_SHAPE[f]
        out = torch.empty(self._lead() + shape + (self.n, self.n, self.n),
                          dtype=torch.float32, device="cuda")
        self._check(lib().dh_get_field(self._h, f, _ptr(out)))
        if f in (FIELD_POS, FIELD_MOM):
            out = out.reshape(self._lead() + (3, self.nc))
        return out

    def set(self, name, t):
        self._stream()
        f = FIELDS[name]
        numel = self.S * self.nc * (self.nq if f == FIELD_Q else
                                    3 if f in (FIELD_POS, FIELD_MOM) else 1)
        self._check(lib().dh_set_field(self._h, f, _ptr(t.contiguous(), numel=numel)))

    def refresh_potential(self):
        self._stream()
        self._check(lib().dh_refresh_potential(self._h))

    def time(self):
        self._stream()
        a, t, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        self._check(lib().dh_get_time(self._h, ctypes.byref(a), ctypes.byref(t), ctypes.byref(s)))
        return a.value, t.value, s.value

    def set_time(self, a, step):
        self._stream()
        self._check(lib().dh_set_time(self._h, a, step))

    def set_store_limit(self, max_steps):
        """Cap on forward steps whose sort and potential are kept for backward (-1: memory)."""
        self._check(lib().dh_set_store_limit(self._h, int(max_steps)))

    def store_info(self):
        """(steps on the last forward's own tape, further steps with a kept sort)."""
        t, k = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().dh_get_store_info(self._h, ctypes.byref(t), ctypes.byref(k)))
        return t.value, k.value

    def forward(self, white, a_final):
        self._stream()
        k = ctypes.c_int32()
        self._check(lib().dh_forward(self._h, _ptr(white, numel=self.S * self.nc), a_final,
                                     ctypes.byref(k)))
        return k.value

    def loss(self, target):
        """The flux-field loss (a list of per-sample values for a batch)."""
        self._stream()
        v = (ctypes.c_double * self.S)()
        self._check(lib().dh_loss(self._h, _ptr(target, numel=self.S * self.nc), v))
        return v[0] if self.S == 1 else list(v)

    def backward(self, grad_rho=None):
        """(dL/dwhite, dL/d(A, beta, eps_sf, delta_c)); per sample for a batch."""
        self._stream()
        gw = torch.empty(self._lead() + (self.n, self.n, self.n), dtype=torch.float32,
                         device="cuda")
        gp = (ctypes.c_double * (4 * self.S))()
        gr = (_ptr(grad_rho.contiguous(), numel=self.S * self.nc) if grad_rho is not None
              else None)
        self._check(lib().dh_backward(self._h, gr, _ptr(gw), gp))
        vals = list(gp)
        return gw, (vals if self.S == 1 else [vals[4 * i:4 * i + 4] for i in range(self.S)])

    def power_spectrum(self, nbins):
        """(P [S][nbins] or [nbins], k [nbins] in h/Mpc, mode counts [nbins]) of the gas
        overdensity (dh_power_spectrum)."""
        self._stream()
        pk = (ctypes.c_double * (self.S * nbins))()
        kk = (ctypes.c_double * nbins)()
        nm = (ctypes.c_double * nbins)()
        self._check(lib().dh_power_spectrum(self._h, nbins, pk, kk, nm))
        vals = list(pk)
        out = vals if self.S == 1 else [vals[i * nbins:(i + 1) * nbins] for i in range(self.S)]
        return out, list(kk), list(nm)

    def power_loss(self, pk_obs, cinv):
        """Gaussian loss of the spectrum against pk_obs ([nbins] or [S][nbins]) with inverse
        covariance cinv [nbins][nbins] (dh_power_loss); per-sample losses for S > 1."""
        self._stream()
        import numpy as np
        obs = np.asarray(pk_obs, dtype=np.float64).reshape(-1)
        nbins = obs.size // self.S
        ci = np.ascontiguousarray(np.asarray(cinv, dtype=np.float64).reshape(nbins, nbins))
        out = (ctypes.c_double * self.S)()
        self._check(lib().dh_power_loss(
            self._h, nbins, obs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ci.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out))
        return out[0] if self.S == 1 else list(out)

    def fli_loss(self, data, noise_var, white):
        """Field-level negative log-posterior (dh_fli_loss); device float32 tensors."""
        self._stream()
        out = (ctypes.c_double * self.S)()
        m = self.S * self.nc
        self._check(lib().dh_fli_loss(self._h, _ptr(data, numel=m), _ptr(noise_var, numel=m),
                                      _ptr(white, numel=m), out))
        return out[0] if self.S == 1 else list(out)

    def closure_states(self):
        """(x [5, S n^3], y [2, S n^3]): the closure network's inputs and the plain term's
        targets for every cell of the current state (dh_closure_states)."""
        self._stream()
        m = self.S * self.nc
        x = torch.empty(5, m, dtype=torch.float32, device="cuda")
        y = torch.empty(2, m, dtype=torch.float32, device="cuda")
        self._check(lib().dh_closure_states(self._h, _ptr(x), _ptr(y)))
        return x, y

    def set_kernel_timing(self, family):
        """Time the launches of one kernel family (_lib.KTIME_*; -1 stops) inside steps and
        reverse passes with HIP events on the handle's stream."""
        self._check(lib().dh_set_kernel_timing(self._h, family))

    def kernel_timing(self):
        """(launches timed since the last call, their mean duration in seconds)."""
        self._stream()
        cnt, ms = ctypes.c_int32(), ctypes.c_double()
        self._check(lib().dh_get_kernel_timing(self._h, ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value * 1e-3

    def conservation(self):
        self._stream()
        out = (ctypes.c_double * (8 * self.S))()
        self._check(lib().dh_conservation(self._h, out))
        vals = list(out)
        return vals if self.S == 1 else [vals[8 * i:8 * i + 8] for i in range(self.S)]

    # single stages on caller buffers
    def stage_sweep(self, q, axis, dt, a1, a2):
        self._stream()
        out = torch.empty_like(q)
        self._check(lib().dh_stage_sweep(self._h, _ptr(q, numel=self.nq * self.nc), _ptr(out),
                                         axis, dt, a1, a2))
        return out

    def stage_sweep_vjp(self, q, lam_out, axis, dt, a1, a2):
        self._stream()
        out = torch.empty_like(q)
        self._check(lib().dh_stage_sweep_vjp(self._h, _ptr(q, numel=self.nq * self.nc),
                                             _ptr(lam_out, numel=self.nq * self.nc), _ptr(out),
                                             axis, dt, a1, a2))
        return out

    def stage_poisson(self, delta, a):
        self._stream()
        out = torch.empty_like(delta)
        self._check(lib().dh_stage_poisson(self._h, _ptr(delta, numel=self.nc), _ptr(out), a))
        return out

    def stage_deposit(self, rho_gas, pos):
        self._stream()
        out = torch.empty_like(rho_gas)
        self._check(lib().dh_stage_deposit(self._h, _ptr(rho_gas, numel=self.nc),
                                           _ptr(pos, numel=3 * self.nc), _ptr(out)))
        return out

    def stage_readout(self, phi, pos):
        self._stream()
        out = torch.empty_like(pos)
        self._check(lib().dh_stage_readout(self._h, _ptr(phi, numel=self.nc),
                                           _ptr(pos, numel=3 * self.nc), _ptr(out)))
        return out


def conservation_noalloc(q, mom, n, m_dm, out, batch=1):
    """dh_conservation_noalloc: the FP64 sums of Sim.conservation over caller tensors q
    [batch][5][n^3] and mom [batch][3][n^3] (float32, device) into the caller's float64 device
    tensor out [batch][8], on torch's current stream; the library allocates nothing."""
    nc = n ** 3
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            and out.numel() == 8 * batch):
        raise ValueError("out: expected a contiguous float64 CUDA tensor of 8 * batch values")
    rc = lib().dh_conservation_noalloc(_ptr(q, numel=5 * nc * batch),
                                       _ptr(mom, numel=3 * nc * batch), n, batch, m_dm,
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != _lib.DH_OK:
        raise _lib.DiffHydroError(rc, lib().dh_last_error(None).decode())
    return out

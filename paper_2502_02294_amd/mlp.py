"""Python face of the learned star-formation closure network (dh_mlp_* in the C ABI):
training-set generation, inference, input gradients, the objective's weight gradient and
Adam training, all in the library's HIP kernels; this module only checks shapes and passes
pointers."""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import MlpSampleOpts, MlpTrainOpts, check, lib
from .sim import _host_floats, _ptr, default_params

N_PARAMS = _lib.MLP_NPARAMS


def train_defaults(**kw):
    o = MlpTrainOpts()
    lib().dh_mlp_train_defaults(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def sample_defaults(**kw):
    o = MlpSampleOpts()
    lib().dh_mlp_sample_defaults(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Mlp:
    """The closure network with its training state on the current HIP device."""

    def __init__(self, seed=None):
        self._h = ctypes.c_void_p()
        torch.cuda.init()
        check(lib().dh_mlp_create(ctypes.byref(self._h)))
        self._stream_handle = None
        self._stream()
        if seed is not None:
            self.init_weights(seed)

    def close(self):
        if self._h:
            lib().dh_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        check(rc, self._h, lib().dh_mlp_last_error)

    def _stream(self):
        stream = torch.cuda.current_stream().cuda_stream
        if stream != self._stream_handle:
            self._check(lib().dh_mlp_set_stream(self._h, ctypes.c_void_p(stream)))
            self._stream_handle = stream

    def init_weights(self, seed):
        self._stream()
        self._check(lib().dh_mlp_init_weights(self._h, ctypes.c_uint64(seed)))

    def set_weights(self, theta):
        self._stream()
        self._check(lib().dh_mlp_set_weights(self._h, _host_floats(theta, N_PARAMS)))

    def weights(self):
        """Flat float32 numpy vector of the current weights."""
        self._stream()
        arr = (ctypes.c_float * N_PARAMS)()
        self._check(lib().dh_mlp_get_weights(self._h, arr))
        return np.frombuffer(arr, dtype=np.float32).copy()

    def sample(self, count, seed, *, first=0, omega_b=0.05, params=None, opts=None,
               device="cuda"):
        """Training states (x [5, count], targets y [2, count]) of the plain source term."""
        self._stream()
        x = torch.empty(5, count, dtype=torch.float32, device=device)
        y = torch.empty(2, count, dtype=torch.float32, device=device)
        p = params if params is not None else default_params()
        o = opts if opts is not None else sample_defaults()
        self._check(lib().dh_mlp_sample(self._h, ctypes.byref(o), float(omega_b), ctypes.byref(p),
                                        ctypes.c_uint64(seed), first, count, _ptr(x), _ptr(y)))
        return x, y

    def eval(self, x):
        self._stream()
        count = x.shape[1]
        out = torch.empty(2, count, dtype=torch.float32, device=x.device)
        self._check(lib().dh_mlp_eval(self._h, _ptr(x, numel=5 * count), count, _ptr(out)))
        return out

    def vjp(self, x, gout):
        self._stream()
        count = x.shape[1]
        gx = torch.empty(5, count, dtype=torch.float32, device=x.device)
        self._check(lib().dh_mlp_vjp(self._h, _ptr(x, numel=5 * count),
                                     _ptr(gout, numel=2 * count), count, _ptr(gx)))
        return gx

    def grad(self, x, y):
        """(objective, gradient [N_PARAMS] float64 numpy) on the set (x, y)."""
        self._stream()
        count = x.shape[1]
        g = (ctypes.c_double * N_PARAMS)()
        loss = ctypes.c_double()
        self._check(lib().dh_mlp_grad(self._h, _ptr(x, numel=5 * count), _ptr(y, numel=2 * count),
                                      count, g, ctypes.byref(loss)))
        return loss.value, np.frombuffer(g, dtype=np.float64).copy()

    def train(self, x, y, opts=None, **kw):
        """Adam on the set; returns the per-step batch objective (numpy float64)."""
        self._stream()
        o = opts if opts is not None else train_defaults(**kw)
        count = x.shape[1]
        hist = (ctypes.c_double * max(1, o.steps))()
        self._check(lib().dh_mlp_train(self._h, _ptr(x, numel=5 * count), _ptr(y, numel=2 * count),
                                       count, ctypes.byref(o), hist))
        return np.frombuffer(hist, dtype=np.float64)[:o.steps].copy()

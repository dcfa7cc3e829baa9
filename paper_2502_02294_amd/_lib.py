"""ctypes binding of libdiffhydro.so (include/diffhydro.h): argument marshalling only.

The library is loaded from this package directory; if it is missing, importing raises, so
nothing can silently fall back to another implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffhydro.so")

DH_OK = 0
ERRORS = {-1: "DH_E_INVAL", -2: "DH_E_OOM", -3: "DH_E_HIP", -4: "DH_E_NONFINITE",
          -5: "DH_E_SCHEDULE", -6: "DH_E_STATE"}

SUBGRID_OFF, SUBGRID_HARD, SUBGRID_RELAXED = 0, 1, 2
CLOSURE_PLAIN, CLOSURE_MLP = 0, 1
KDK_PLAIN, KDK_FASTPM = 0, 1
TRANSFER_BBKS, TRANSFER_EH = 0, 1
KTIME_SWEEP_KICK, KTIME_SWEEP, KTIME_SWEEP_VJP = 0, 1, 2
MLP_NPARAMS = 8834
(FIELD_Q, FIELD_RHO, FIELD_POS, FIELD_MOM, FIELD_STAR, FIELD_PHI, FIELD_TEMP, FIELD_FLUX,
 FIELD_STAR_DM, FIELD_OBS_TEMP) = range(10)


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_double), ("omega_m", ctypes.c_double),
                ("omega_b", ctypes.c_double), ("h", ctypes.c_double), ("sigma8", ctypes.c_double),
                ("n_s", ctypes.c_double), ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("a_init", ctypes.c_double), ("t_init", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dlna_max", ctypes.c_double), ("t_floor", ctypes.c_double),
                ("subgrid", ctypes.c_int32), ("tau", ctypes.c_double), ("sf_seed", ctypes.c_uint64),
                ("ckpt_every", ctypes.c_int32), ("closure", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("cfl_forward", ctypes.c_double),
                ("kdk", ctypes.c_int32), ("star_dm", ctypes.c_int32),
                ("sn_smooth", ctypes.c_int32), ("lpt", ctypes.c_int32),
                ("transfer", ctypes.c_int32),
                ("dual_energy", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("A", "beta", "eps_sf", "delta_c", "t_c", "e0",
                                                "w_rho", "w_t")]


class MlpTrainOpts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("steps", ctypes.c_int32), ("lr", ctypes.c_double),
                ("lr_final", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class MlpSampleOpts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("lnd_lo", "lnd_hi", "lnt_lo", "lnt_hi", "lna_lo",
                                                "lna_hi", "eps_lo", "eps_hi", "dc_lo", "dc_hi")]


class DiffHydroError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None

P = ctypes.c_void_p
D = ctypes.c_double
I = ctypes.c_int32

_SIGNATURES = {
    "dh_config_default": (None, [ctypes.POINTER(Config)]),
    "dh_params_default": (None, [ctypes.POINTER(Params)]),
    "dh_create": (I, [ctypes.POINTER(Config), ctypes.POINTER(P)]),
    "dh_destroy": (I, [P]),
    "dh_set_stream": (I, [P, P]),
    "dh_set_params": (I, [P, ctypes.POINTER(Params)]),
    "dh_set_sample_params": (I, [P, I, ctypes.POINTER(Params)]),
    "dh_init_from_seed": (I, [P, ctypes.c_uint64]),
    "dh_init_from_noise": (I, [P, P]),
    "dh_step": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
    "dh_run_to": (I, [P, D, ctypes.POINTER(I)]),
    "dh_run_steps": (I, [P, I, ctypes.POINTER(I)]),
    "dh_set_store_limit": (I, [P, I]),
    "dh_get_store_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
    "dh_set_schedule": (I, [P, ctypes.POINTER(D), I]),
    "dh_get_schedule": (I, [P, ctypes.POINTER(D), I, ctypes.POINTER(I)]),
    "dh_set_sample_schedule": (I, [P, I, ctypes.POINTER(D), I]),
    "dh_get_sample_schedule": (I, [P, I, ctypes.POINTER(D), I, ctypes.POINTER(I)]),
    "dh_get_field": (I, [P, I, P]),
    "dh_set_field": (I, [P, I, P]),
    "dh_refresh_potential": (I, [P]),
    "dh_get_time": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I)]),
    "dh_set_time": (I, [P, D, I]),
    "dh_get_sample_times": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
    "dh_forward": (I, [P, P, D, ctypes.POINTER(I)]),
    "dh_loss": (I, [P, P, ctypes.POINTER(D)]),
    "dh_backward": (I, [P, P, P, ctypes.POINTER(D)]),
    "dh_power_spectrum": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]),
    "dh_power_loss": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]),
    "dh_fli_loss": (I, [P, P, P, P, ctypes.POINTER(D)]),
    "dh_closure_states": (I, [P, P, P]),
    "dh_set_kernel_timing": (I, [P, I]),
    "dh_get_kernel_timing": (I, [P, ctypes.POINTER(I), ctypes.POINTER(D)]),
    "dh_conservation": (I, [P, ctypes.POINTER(D)]),
    "dh_conservation_noalloc": (I, [P, P, I, I, D, P, P]),
    "dh_stage_sweep": (I, [P, P, P, I, D, D, D]),
    "dh_stage_sweep_vjp": (I, [P, P, P, P, I, D, D, D]),
    "dh_stage_poisson": (I, [P, P, P, D]),
    "dh_stage_deposit": (I, [P, P, P, P]),
    "dh_stage_readout": (I, [P, P, P, P]),
    "dh_last_error": (ctypes.c_char_p, [P]),
    "dh_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dh_set_closure": (I, [P, P]),
    "dh_mlp_train_defaults": (None, [ctypes.POINTER(MlpTrainOpts)]),
    "dh_mlp_sample_defaults": (None, [ctypes.POINTER(MlpSampleOpts)]),
    "dh_mlp_create": (I, [ctypes.POINTER(P)]),
    "dh_mlp_destroy": (I, [P]),
    "dh_mlp_set_stream": (I, [P, P]),
    "dh_mlp_init_weights": (I, [P, ctypes.c_uint64]),
    "dh_mlp_set_weights": (I, [P, P]),
    "dh_mlp_get_weights": (I, [P, P]),
    "dh_mlp_sample": (I, [P, ctypes.POINTER(MlpSampleOpts), D, ctypes.POINTER(Params),
                          ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, P, P]),
    "dh_mlp_eval": (I, [P, P, ctypes.c_int64, P]),
    "dh_mlp_vjp": (I, [P, P, P, ctypes.c_int64, P]),
    "dh_mlp_grad": (I, [P, P, P, ctypes.c_int64, ctypes.POINTER(D), ctypes.POINTER(D)]),
    "dh_mlp_train": (I, [P, P, P, ctypes.c_int64, ctypes.POINTER(MlpTrainOpts),
                         ctypes.POINTER(D)]),
    "dh_mlp_last_error": (ctypes.c_char_p, [P]),
}

EXPORTED = tuple(_SIGNATURES)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(rc, handle=None, last_error=None):
    if rc != DH_OK:
        if handle:
            msg = (last_error or lib().dh_last_error)(handle).decode()
        else:
            msg = lib().dh_strerror(rc).decode()
        raise DiffHydroError(rc, msg)

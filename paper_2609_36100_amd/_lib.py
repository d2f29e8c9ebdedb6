"""ctypes binding of libpf (include/pf.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libpf.so``; this module only
converts Python values to the C structs, passes device pointers from PyTorch
tensors (PyTorch supplies device memory and the stream) and raises on error
codes.  Importing it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

from .build import source_id

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")


class PFError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, status_string(code), code))


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("W", ctypes.c_double), ("w", ctypes.c_double), ("kappa_c", ctypes.c_double),
        ("kappa_eta", ctypes.c_double), ("M", ctypes.c_double), ("L", ctypes.c_double),
        ("c_m", ctypes.c_double), ("c_p", ctypes.c_double),
        ("C11", ctypes.c_double), ("C12", ctypes.c_double), ("C44", ctypes.c_double),
        ("eps_star", (ctypes.c_double * 3) * 3),
        ("eps_bar", ctypes.c_double * 3),
        ("mean_strain_mode", ctypes.c_int32),
        ("implicit_bulk_c", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("adaptive", ctypes.c_int32),
        ("dt0", ctypes.c_double), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
        ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("max_rejects", ctypes.c_int32),
        ("norm_space", ctypes.c_int32),
        ("elastic_inhom", ctypes.c_int32),
        ("C11p", ctypes.c_double), ("C12p", ctypes.c_double), ("C44p", ctypes.c_double),
        ("el_tol", ctypes.c_double),
        ("el_max_iter", ctypes.c_int32),
    ]


class FnoConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("width", ctypes.c_int32), ("modes", ctypes.c_int32),
                ("layers", ctypes.c_int32), ("hidden", ctypes.c_int32), ("cin", ctypes.c_int32),
                ("cout", ctypes.c_int32)]


class FnoStats(ctypes.Structure):
    _fields_ = [("surrogate", ctypes.c_int32), ("checks", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("plain", ctypes.c_int32), ("since_check", ctypes.c_int32), ("plain_left", ctypes.c_int32),
                ("err_last", ctypes.c_double), ("err_max", ctypes.c_double),
                ("ms_surrogate", ctypes.c_double), ("ms_plain", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("attempts", ctypes.c_int64),
        ("rejects", ctypes.c_int64), ("n_rhs", ctypes.c_int64),
        ("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("dt_next", ctypes.c_double),
        ("dt_min_seen", ctypes.c_double), ("dt_max_seen", ctypes.c_double),
        ("err_last", ctypes.c_double), ("mass", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("F", ctypes.c_double), ("vf", ctypes.c_double), ("vf_threshold", ctypes.c_double),
        ("el_iterations", ctypes.c_int64), ("el_last", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PF_FP64, PF_MIXED = 0, 1
PF_IMEX_EULER, PF_ARK2, PF_ARK324L, PF_ARK436L = 1, 2, 3, 4
METHODS = {"imex_euler": PF_IMEX_EULER, "ark2": PF_ARK2, "ark324l": PF_ARK324L, "ark436l": PF_ARK436L}
PRECISIONS = {"fp64": PF_FP64, "mixed": PF_MIXED}

_lib = None

_SIGS = {
    "pf_default_params": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "pf_size_supported": (ctypes.c_int32, [ctypes.c_int32]),
    "pf_init": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pf_finalize": (None, [ctypes.c_void_p]),
    "pf_kspace_pitch": (ctypes.c_int64, [ctypes.c_void_p]),
    "pf_workspace_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "pf_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double]),
    "pf_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "pf_get_state_hat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pf_set_state_hat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    "pf_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pf_ark_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "pf_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(Stats)]),
    "pf_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "pf_get_time": (ctypes.c_double, [ctypes.c_void_p]),
    "pf_set_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "pf_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pf_fft3d": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "pf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pf_build_id": (ctypes.c_char_p, []),
    "pf_free_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "pf_ensemble_free_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "pf_fno_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "pf_fno_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_float, ctypes.POINTER(ctypes.c_float)]),
    "pf_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "pf_tuning_kinds": (ctypes.c_int32, []),
    "pf_tuning_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "pf_tuning_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pf_tuning_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "pf_tuning_ms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "pf_ensemble_init": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "pf_ensemble_finalize": (None, [ctypes.c_void_p]),
    "pf_ensemble_size_supported": (ctypes.c_int32, [ctypes.c_int32]),
    "pf_ensemble_workspace_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "pf_ensemble_kspace_pitch": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32]),
    "pf_ensemble_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_double]),
    "pf_ensemble_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int32]),
    "pf_ensemble_get_state_hat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "pf_ensemble_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pf_ensemble_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                           ctypes.POINTER(Stats)]),
    "pf_ensemble_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "pf_ensemble_tuning_kinds": (ctypes.c_int32, []),
    "pf_ensemble_tuning_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "pf_ensemble_tuning_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pf_ensemble_tuning_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "pf_fno_create": (ctypes.c_int, [ctypes.POINTER(FnoConfig), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pf_fno_destroy": (None, [ctypes.c_void_p]),
    "pf_fno_num_params": (ctypes.c_int64, [ctypes.c_void_p]),
    "pf_fno_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_set_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double)]),
    "pf_fno_get_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_zero_grad": (ctypes.c_int, [ctypes.c_void_p]),
    "pf_fno_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_float]),
    "pf_fno_set_input_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pf_fno_apply_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "pf_fno_work": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "pf_fno_ensemble_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                               ctypes.c_double, ctypes.POINTER(FnoStats)]),
    "pf_fno_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(FnoStats)]),
    "pf_bandwidth_probe": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "pf_rel_l2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_double)]),
    "pf_rel_l2_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_double)]),
    "pf_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "pf_profile_classes": (ctypes.c_int32, []),
    "pf_profile_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "pf_profile_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
}


def lib():
    """Load libpf.so (raises ImportError with instructions when it is missing or
    was built from sources other than those beside it)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpf.so not built: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950) first; there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        built = L.pf_build_id().decode()
        want = source_id()
        if built != want:
            raise ImportError("stale libpf.so: built from sources %s, the sources here are %s; "
                              "rebuild with __graft_entry__.build()" % (built, want))
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def status_string(code):
    return lib().pf_status_string(int(code)).decode()


def check(code, where):
    if code != 0:
        raise PFError(code, where)


def make_params(n, model=None, method="ark436l", precision="fp64", adaptive=False,
                dt0=1e-2, rtol=1e-6, atol=1e-9, dt_min=0.0, dt_max=1e300, max_rejects=10, norm_space=0):
    """Build a Params struct; ``n`` is an int (cubic) or (nx, ny, nz)."""
    p = Params()
    check(lib().pf_default_params(ctypes.byref(p)), "pf_default_params")
    nx, ny, nz = (n, n, n) if isinstance(n, int) else tuple(n)
    p.nx, p.ny, p.nz = nx, ny, nz
    model = dict(model or {})
    for key in ("dx", "W", "w", "kappa_c", "kappa_eta", "M", "L", "c_m", "c_p", "C11", "C12", "C44"):
        if key in model:
            setattr(p, key, float(model[key]))
    if "eps_star" in model:
        for v in range(3):
            for i in range(3):
                p.eps_star[v][i] = float(model["eps_star"][v][i])
    if "eps_bar" in model:
        for i in range(3):
            p.eps_bar[i] = float(model["eps_bar"][i])
    if "mean_strain_mode" in model:
        p.mean_strain_mode = int(model["mean_strain_mode"])
    if "implicit_bulk_c" in model:
        p.implicit_bulk_c = int(model["implicit_bulk_c"])
    if "C11p" in model:      # a precipitate stiffness selects the inhomogeneous (Reuss) elasticity
        p.elastic_inhom = 1
        p.C11p, p.C12p, p.C44p = float(model["C11p"]), float(model["C12p"]), float(model["C44p"])
    if "el_tol" in model:
        p.el_tol = float(model["el_tol"])
    if "el_max_iter" in model:
        p.el_max_iter = int(model["el_max_iter"])
    p.method = METHODS[method] if isinstance(method, str) else int(method)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.adaptive = 1 if adaptive else 0
    p.dt0, p.rtol, p.atol = float(dt0), float(rtol), float(atol)
    p.dt_min, p.dt_max = float(dt_min), float(dt_max)
    p.max_rejects = int(max_rejects)
    p.norm_space = int(norm_space)
    return p

"""MI355X-native pseudospectral phase-field ImEx-ARK hot path (Python front end).

The compute path lives in ``libpf.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/pf.h``).  This package is a thin binding: :class:`Solver` owns a
``pf_ctx`` and marshals PyTorch device tensors and numpy arrays to it.  There
is no CPU fallback: without the built library, creating a solver raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FnoStats, PFError, Stats, make_params  # noqa: F401

__all__ = ["Solver", "Ensemble", "FNO", "FnoStats", "PFError", "make_params", "bandwidth_probe", "rel_l2", "size_supported"]


def _torch():
    import torch
    return torch


def size_supported(n):
    return bool(_lib.lib().pf_size_supported(int(n)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One simulation context on the current GPU.

    Parameters mirror ``pf_params``: ``n`` (int or (nx, ny, nz)), ``model``
    (dict of model constants, see ``pfinputs.default_params``), ``method``
    ("imex_euler" | "ark2" | "ark324l" | "ark436l"), ``precision`` ("fp64" | "mixed"), ``adaptive``,
    ``dt0``, ``rtol``, ``atol``.
    """

    def __init__(self, n, model=None, stream=None, **kw):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libpf needs a GPU (gfx950); none is visible")
        L = _lib.lib()
        self.params = make_params(n, model, **kw)
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _lib.check(L.pf_init(ctypes.byref(self.params), ctypes.c_void_p(self._stream.cuda_stream),
                             ctypes.byref(h)), "pf_init")
        self._h = h
        self.kpitch = int(L.pf_kspace_pitch(h))
        self.nxh = self.params.nx // 2 + 1

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().pf_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- buffers ------------------------------------------------------------
    def kspace_empty(self, nf=4):
        torch = _torch()
        nz, ny, _ = self.shape
        return torch.empty((nf, nz, ny, self.kpitch), dtype=torch.complex128, device="cuda")

    def kspace_from_numpy(self, a):
        """Pad a (nf, nz, ny, nx//2+1) complex array to the library pitch on the GPU."""
        torch = _torch()
        t = self.kspace_empty(a.shape[0])
        t.zero_()
        t[..., : self.nxh] = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
        return t

    def kspace_to_numpy(self, t):
        return t[..., : self.nxh].cpu().numpy()

    @property
    def workspace_bytes(self):
        return int(_lib.lib().pf_workspace_bytes(self._h))

    # -- state ----------------------------------------------------------------
    def set_state(self, c, eta, t0=0.0):
        torch = _torch()
        if isinstance(c, torch.Tensor):
            c = c.to(device="cuda", dtype=torch.float64).contiguous()
            eta = eta.to(device="cuda", dtype=torch.float64).contiguous()
            _lib.check(_lib.lib().pf_set_state(self._h, _ptr(c), _ptr(eta), 1, float(t0)), "pf_set_state")
        else:
            c = np.ascontiguousarray(c, dtype=np.float64)
            eta = np.ascontiguousarray(eta, dtype=np.float64)
            assert c.shape == self.shape and eta.shape == (3,) + self.shape
            _lib.check(_lib.lib().pf_set_state(self._h, c.ctypes.data_as(ctypes.c_void_p),
                                               eta.ctypes.data_as(ctypes.c_void_p), 0, float(t0)),
                       "pf_set_state")

    def get_state(self):
        c = np.empty(self.shape)
        eta = np.empty((3,) + self.shape)
        _lib.check(_lib.lib().pf_get_state(self._h, c.ctypes.data_as(ctypes.c_void_p),
                                           eta.ctypes.data_as(ctypes.c_void_p), 0), "pf_get_state")
        return c, eta

    def get_state_device(self, out=None):
        """Real-space state as a device float64 tensor (4, nz, ny, nx)."""
        torch = _torch()
        if out is None:
            out = torch.empty((4,) + self.shape, dtype=torch.float64, device="cuda")
        _lib.check(_lib.lib().pf_get_state(self._h, _ptr(out[0]), _ptr(out[1]), 1), "pf_get_state")
        return out

    def set_state_device(self, u, t0=0.0):
        """Set the state from a device float64 tensor (4, nz, ny, nx)."""
        _lib.check(_lib.lib().pf_set_state(self._h, _ptr(u[0]), _ptr(u[1]), 1, float(t0)), "pf_set_state")

    def get_state_hat(self):
        t = self.kspace_empty()
        _lib.check(_lib.lib().pf_get_state_hat(self._h, _ptr(t)), "pf_get_state_hat")
        return t

    def set_state_hat(self, t, t0=0.0):
        _lib.check(_lib.lib().pf_set_state_hat(self._h, _ptr(t.contiguous()), float(t0)), "pf_set_state_hat")

    # -- hot path -------------------------------------------------------------
    def rhs(self, y_hat, t=0.0):
        fI = self.kspace_empty()
        fE = self.kspace_empty()
        _lib.check(_lib.lib().pf_rhs(self._h, float(t), _ptr(y_hat), _ptr(fI), _ptr(fE)), "pf_rhs")
        return fI, fE

    def step(self, dt):
        dn, err, acc = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        code = _lib.lib().pf_ark_step(self._h, float(dt), ctypes.byref(dn), ctypes.byref(err),
                                      ctypes.byref(acc))
        _lib.check(code, "pf_ark_step")
        return bool(acc.value), err.value, dn.value

    def advance(self, t_final):
        st = Stats()
        _lib.check(_lib.lib().pf_advance(self._h, float(t_final), ctypes.byref(st)), "pf_advance")
        return st.as_dict()

    def stats(self):
        st = Stats()
        _lib.check(_lib.lib().pf_get_stats(self._h, ctypes.byref(st)), "pf_get_stats")
        return st.as_dict()

    @property
    def t(self):
        return float(_lib.lib().pf_get_time(self._h))

    def set_dt(self, dt):
        _lib.check(_lib.lib().pf_set_dt(self._h, float(dt)), "pf_set_dt")

    def diagnostics(self):
        m, v, vt = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.lib().pf_diagnostics(self._h, ctypes.byref(m), ctypes.byref(v), ctypes.byref(vt)),
                   "pf_diagnostics")
        return dict(mass=m.value, vf=v.value, vf_threshold=vt.value)

    def free_energy(self):
        """Total free energy F of the current state (computed by libpf in FP64)."""
        F = ctypes.c_double()
        _lib.check(_lib.lib().pf_free_energy(self._h, ctypes.byref(F)), "pf_free_energy")
        return F.value

    # -- tile plans -------------------------------------------------------------
    def autotune(self, reps=3):
        """Time the tile variants of every column pass and keep the fastest."""
        _lib.check(_lib.lib().pf_autotune(self._h, int(reps)), "pf_autotune")
        return self.tuning()

    def tuning(self):
        L = _lib.lib()
        out = {}
        for k in range(L.pf_tuning_kinds()):
            v, tx, re_ = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            m0, m1 = ctypes.c_double(), ctypes.c_double()
            _lib.check(L.pf_tuning_get(self._h, k, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(re_),
                                       ctypes.byref(m0), ctypes.byref(m1)), "pf_tuning_get")
            m2 = ctypes.c_double()
            _lib.check(L.pf_tuning_ms(self._h, k, 2, ctypes.byref(m2)), "pf_tuning_ms")
            out[L.pf_tuning_name(k).decode()] = dict(variant=v.value, tile_cols=tx.value,
                                                     end_radix=re_.value, ms=[m0.value, m1.value, m2.value])
        return out

    def set_tuning(self, kind, variant):
        _lib.check(_lib.lib().pf_tuning_set(self._h, int(kind), int(variant)), "pf_tuning_set")

    # -- measurement ----------------------------------------------------------
    def profile(self, on=True):
        """Clear and enable/disable per-kernel-class HIP-event timing."""
        _lib.check(_lib.lib().pf_profile_enable(self._h, 1 if on else 0), "pf_profile_enable")

    def profile_report(self):
        """{class: (total_ms, launches, algorithmic_bytes)} for classes with launches."""
        L = _lib.lib()
        out = {}
        for k in range(L.pf_profile_classes()):
            ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
            _lib.check(L.pf_profile_get(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
                       "pf_profile_get")
            if n.value:
                out[L.pf_profile_name(k).decode()] = (ms.value, n.value, b.value)
        return out

    def fft3d(self, direction, nf, src, dst):
        """Standalone 3D real FFT on device tensors (see pf_fft3d)."""
        _lib.check(_lib.lib().pf_fft3d(self._h, int(direction), int(nf), _ptr(src), _ptr(dst)), "pf_fft3d")


class Ensemble:
    """Many independent simulations of uneven cubic sizes advanced together.

    ``members`` is a list of dicts with keys ``n`` (32, 48, 64, 96 or 128) and
    optionally ``model`` plus any :func:`make_params` keyword (``adaptive``,
    ``dt0``, ``rtol``, ``atol``, ``precision``, ``method`` among the embedded pairs,
    ARK4(3)6L by default; one method for all members).
    """

    def __init__(self, members, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libpf needs a GPU (gfx950); none is visible")
        L = _lib.lib()
        arr = (_lib.Params * len(members))()
        self.shapes = []
        for i, mb in enumerate(members):
            kw = {k: v for k, v in mb.items() if k not in ("n", "model")}
            kw.setdefault("method", "ark436l")
            arr[i] = make_params(int(mb["n"]), mb.get("model"), **kw)
            self.shapes.append((arr[i].nz, arr[i].ny, arr[i].nx))
        self.M = len(members)
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p(0)
        _lib.check(L.pf_ensemble_init(self.M, arr, sp, ctypes.byref(h)), "pf_ensemble_init")
        self._h = h
        self._params = arr

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().pf_ensemble_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def workspace_bytes(self):
        return int(_lib.lib().pf_ensemble_workspace_bytes(self._h))

    def set_state(self, m, c, eta, t0=0.0):
        c = np.ascontiguousarray(c, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        assert c.shape == self.shapes[m] and eta.shape == (3,) + self.shapes[m]
        _lib.check(_lib.lib().pf_ensemble_set_state(self._h, int(m), c.ctypes.data_as(ctypes.c_void_p),
                                                    eta.ctypes.data_as(ctypes.c_void_p), 0, float(t0)),
                   "pf_ensemble_set_state")

    def get_state(self, m):
        c = np.empty(self.shapes[m])
        eta = np.empty((3,) + self.shapes[m])
        _lib.check(_lib.lib().pf_ensemble_get_state(self._h, int(m), c.ctypes.data_as(ctypes.c_void_p),
                                                    eta.ctypes.data_as(ctypes.c_void_p), 0),
                   "pf_ensemble_get_state")
        return c, eta

    def get_state_hat(self, m):
        """Member m's reciprocal-space state as a numpy array (4, nz, ny, nx//2+1)."""
        torch = _torch()
        nz, ny, nx = self.shapes[m]
        kp = int(_lib.lib().pf_ensemble_kspace_pitch(self._h, int(m)))
        t = torch.empty((4, nz, ny, kp), dtype=torch.complex128, device="cuda")
        _lib.check(_lib.lib().pf_ensemble_get_state_hat(self._h, int(m), _ptr(t)), "pf_ensemble_get_state_hat")
        return t[..., : nx // 2 + 1].cpu().numpy()

    def diagnostics(self, m):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.lib().pf_ensemble_diagnostics(self._h, int(m), ctypes.byref(a), ctypes.byref(b),
                                                      ctypes.byref(c)), "pf_ensemble_diagnostics")
        return dict(mass=a.value, vf=b.value, vf_threshold=c.value)

    def free_energy(self, m):
        F = ctypes.c_double()
        _lib.check(_lib.lib().pf_ensemble_free_energy(self._h, int(m), ctypes.byref(F)), "pf_ensemble_free_energy")
        return F.value

    def advance(self, t_final, max_steps=100000):
        """Advance every member to t_final (scalar or per member); returns per-member stats."""
        tf = np.broadcast_to(np.asarray(t_final, dtype=np.float64), (self.M,)).copy()
        st = (Stats * self.M)()
        code = _lib.lib().pf_ensemble_advance(self._h, tf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              int(min(max_steps, 2**31 - 1)), st)
        _lib.check(code, "pf_ensemble_advance")
        return [st[i].as_dict() for i in range(self.M)]

    def autotune(self, reps=3):
        _lib.check(_lib.lib().pf_ensemble_autotune(self._h, int(reps)), "pf_ensemble_autotune")
        return self.tuning()

    def tuning(self):
        L = _lib.lib()
        out = {}
        for k in range(L.pf_ensemble_tuning_kinds()):
            bt, a, b = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
            _lib.check(L.pf_ensemble_tuning_get(self._h, k, ctypes.byref(bt), ctypes.byref(a), ctypes.byref(b)),
                       "pf_ensemble_tuning_get")
            out[L.pf_ensemble_tuning_name(k).decode()] = dict(block_threads=bt.value, ms=[a.value, b.value])
        return out

    def set_tuning(self, kind, block_threads):
        _lib.check(_lib.lib().pf_ensemble_tuning_set(self._h, int(kind), int(block_threads)),
                   "pf_ensemble_tuning_set")


def bandwidth_probe(nbytes=1 << 30, reps=5):
    """Streaming HBM bandwidth of this device in GB/s: {"copy", "read", "multi"}."""
    vals = [ctypes.c_double() for _ in range(3)]
    _lib.check(_lib.lib().pf_bandwidth_probe(int(nbytes), int(reps), None, *[ctypes.byref(v) for v in vals]),
               "pf_bandwidth_probe")
    return dict(copy=vals[0].value, read=vals[1].value, multi=vals[2].value)


def rel_l2(a, b):
    """||a - b|| / ||b|| of two device float64 tensors (computed by libpf)."""
    out = ctypes.c_double()
    _lib.check(_lib.lib().pf_rel_l2(_ptr(a.contiguous()), _ptr(b.contiguous()), a.numel(), None,
                                    ctypes.byref(out)), "pf_rel_l2")
    return out.value


class FNO:
    """Fourier neural operator surrogate on the GPU (BF16 MFMA, FP32 master weights).

    Parameters are a flat float32 vector (see ``pf_fno_set_params``); inputs
    and targets are device float32 tensors of shape (cin, n, n, n).
    """

    def __init__(self, n, width=32, modes=12, layers=4, hidden=None, cin=4, cout=4, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libpf needs a GPU (gfx950); none is visible")
        self.cfg = _lib.FnoConfig(n, width, modes, layers, hidden if hidden else 4 * width, cin, cout)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().pf_fno_create(ctypes.byref(self.cfg), ctypes.c_void_p(self._stream.cuda_stream),
                                            ctypes.byref(h)), "pf_fno_create")
        self._h = h
        self.n, self.cin, self.cout = n, cin, cout
        self.num_params = int(_lib.lib().pf_fno_num_params(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().pf_fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.num_params
        _lib.check(_lib.lib().pf_fno_set_params(self._h, th.ctypes.data_as(ctypes.c_void_p)), "pf_fno_set_params")

    def load(self, weights):
        """Load a flat parameter vector given as float32 or bfloat16 bytes / numpy array
        (bfloat16 as uint16 bit patterns)."""
        buf = weights.tobytes() if isinstance(weights, np.ndarray) else bytes(weights)
        _lib.check(_lib.lib().pf_fno_load(self._h, ctypes.c_char_p(buf), len(buf)), "pf_fno_load")

    def train_step(self, x, y, lr):
        """One Adam step on a batch (x, y: device float32 (batch, cin, n, n, n)); returns the mean loss."""
        loss = ctypes.c_float()
        _lib.check(_lib.lib().pf_fno_train_step(self._h, _ptr(x.contiguous()), _ptr(y.contiguous()), int(x.shape[0]),
                                                float(lr), ctypes.byref(loss)), "pf_fno_train_step")
        return loss.value

    def get_params(self):
        th = np.empty(self.num_params, np.float32)
        _lib.check(_lib.lib().pf_fno_get_params(self._h, th.ctypes.data_as(ctypes.c_void_p)), "pf_fno_get_params")
        return th

    def set_scale(self, scale):
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        _lib.check(_lib.lib().pf_fno_set_scale(self._h, sc.ctypes.data_as(ctypes.c_void_p)), "pf_fno_set_scale")

    def set_input_norm(self, shift, scale):
        """The network sees (x - shift) / scale per input channel."""
        sh = np.ascontiguousarray(shift, dtype=np.float32)
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        assert sh.size == self.cin and sc.size == self.cin
        _lib.check(_lib.lib().pf_fno_set_input_norm(self._h, sh.ctypes.data_as(ctypes.c_void_p),
                                                    sc.ctypes.data_as(ctypes.c_void_p)), "pf_fno_set_input_norm")

    def forward(self, x):
        torch = _torch()
        out = torch.empty((self.n ** 3, self.cout), dtype=torch.float32, device="cuda")
        _lib.check(_lib.lib().pf_fno_forward(self._h, _ptr(x.contiguous()), _ptr(out)), "pf_fno_forward")
        return out

    def grad(self, x, y):
        loss = ctypes.c_double()
        _lib.check(_lib.lib().pf_fno_grad(self._h, _ptr(x.contiguous()), _ptr(y.contiguous()), ctypes.byref(loss)),
                   "pf_fno_grad")
        return loss.value

    def get_grad(self):
        g = np.empty(self.num_params, np.float32)
        _lib.check(_lib.lib().pf_fno_get_grad(self._h, g.ctypes.data_as(ctypes.c_void_p)), "pf_fno_get_grad")
        return g

    def zero_grad(self):
        _lib.check(_lib.lib().pf_fno_zero_grad(self._h), "pf_fno_zero_grad")

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        _lib.check(_lib.lib().pf_fno_adam_step(self._h, lr, beta1, beta2, eps, grad_scale), "pf_fno_adam_step")

    def apply(self, state, out):
        """out = state + scale * net(state), mean of c restored (device float64 (cin, n, n, n))."""
        _lib.check(_lib.lib().pf_fno_apply(self._h, _ptr(state), _ptr(out)), "pf_fno_apply")

    WORK_KINDS = ("lm_gemm", "cm_gemm", "wgrad", "wgrad_sum", "mix", "gelu_bwd", "elementwise")

    def work(self, enable=-1):
        """Algorithmic bytes / flops / launches per kind since the last reset (pf_fno_work);
        enable = 1 / 0 then resets and turns the accounting on / off."""
        k = len(self.WORK_KINDS)
        b, f, n = (ctypes.c_double * k)(), (ctypes.c_double * k)(), (ctypes.c_int64 * k)()
        _lib.check(_lib.lib().pf_fno_work(self._h, int(enable), b, f, n, k), "pf_fno_work")
        return {name: dict(bytes=b[i], flops=f[i], launches=n[i]) for i, name in enumerate(self.WORK_KINDS)}

    def apply_batch(self, states, out):
        """out[b] = states[b] + scale * net(states[b]) for every b (device float64 (B, cin, n, n, n))."""
        assert states.is_contiguous() and out.is_contiguous() and states.shape == out.shape
        _lib.check(_lib.lib().pf_fno_apply_batch(self._h, _ptr(states), _ptr(out), int(states.shape[0])),
                   "pf_fno_apply_batch")

    def ensemble_advance(self, ens, members, n_adv, delta, check_every=5, tol=1e-3, stats=None):
        """Checked surrogate advance of the listed members of an :class:`Ensemble` (see
        pf_fno_ensemble_advance); ``stats`` (a list of FnoStats, one per member) carries the
        cadence between calls; returns it."""
        idx = (ctypes.c_int32 * len(members))(*[int(m) for m in members])
        if stats is None:
            stats = [_lib.FnoStats() for _ in members]
        arr = (_lib.FnoStats * len(members))(*stats)
        _lib.check(_lib.lib().pf_fno_ensemble_advance(self._h, ens._h, idx, len(members), int(n_adv), float(delta),
                                                      int(check_every), float(tol), arr),
                   "pf_fno_ensemble_advance")
        return [arr[i] for i in range(len(members))]

    def advance(self, plain, state, n_adv, delta, check_every=5, tol=1e-3, stats=None):
        """Checked surrogate advance of ``state`` (device float64 (4, n, n, n), in place) by
        ``n_adv`` intervals of ``delta``; ``plain`` is a :class:`Solver` on the same grid that
        runs the checks and fallbacks.  ``stats`` (an ``FnoStats``) carries the check cadence
        between calls; returns it."""
        if stats is None:
            stats = _lib.FnoStats()
        assert state.is_contiguous() and state.dtype == _torch().float64
        _lib.check(_lib.lib().pf_fno_advance(self._h, plain._h, _ptr(state), int(n_adv), float(delta),
                                             int(check_every), float(tol), ctypes.byref(stats)),
                   "pf_fno_advance")
        return stats

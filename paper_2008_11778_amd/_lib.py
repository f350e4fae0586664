"""ctypes binding of libaafwi.so (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw device pointers and the HIP stream,
and turns status codes into exceptions.  PyTorch provides device memory and
streams.  Importing fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaafwi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python -m paper_2008_11778_amd.build` (the HIP path has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

AAFWI_OK = 0
ERRORS = {-1: "E_INVALID", -2: "E_CFL", -3: "E_NOMEM", -4: "E_HIP", -5: "E_NONFINITE", -6: "E_STATE"}
K_FWD_STEP, K_REC_STEP, K_ADJ_STEP, K_BORN_STEP = 0, 1, 2, 3
DOT_WORKSPACE = 1024


class AafwiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"aafwi {ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Geometry(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("nb", ctypes.c_int32),
        ("h", ctypes.c_float), ("dt", ctypes.c_float), ("nt", ctypes.c_int32),
        ("vref", ctypes.c_float), ("refl", ctypes.c_float), ("vmax_bound", ctypes.c_float),
        ("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
        ("src_iz", ctypes.POINTER(ctypes.c_int32)), ("src_ix", ctypes.POINTER(ctypes.c_int32)),
        ("rec_iz", ctypes.POINTER(ctypes.c_int32)), ("rec_ix", ctypes.POINTER(ctypes.c_int32)),
        ("wavelet", ctypes.POINTER(ctypes.c_float)), ("ckpt_every", ctypes.c_int32),
    ]


_vp, _i32, _i64, _f32, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double


def _sig(name, *args):
    fn = getattr(_lib, name)
    fn.argtypes = list(args)
    fn.restype = ctypes.c_int
    return fn


_sig("aafwi_create", ctypes.POINTER(_Geometry), _vp, ctypes.POINTER(_vp))
_sig("aafwi_destroy", _vp)
_sig("aafwi_device_bytes", _vp, ctypes.POINTER(_i64))
_sig("aafwi_sync", _vp)
_sig("aafwi_forward_model", _vp, _vp, _vp, ctypes.c_int)
_sig("aafwi_residual_misfit", _vp, _vp, _vp, _vp, _vp)
_sig("aafwi_residual_misfit_noalloc", _vp, ctypes.c_int64, _vp, _vp, _vp, _vp)
_sig("aafwi_batch_aa_create", ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, ctypes.c_double, _vp,
     ctypes.POINTER(_vp))
_sig("aafwi_batch_aa_step", _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_float),
     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint8))
_sig("aafwi_batch_aa_reset", _vp, ctypes.POINTER(ctypes.c_uint8))
_sig("aafwi_batch_aa_state", _vp, _vp, _vp)
_sig("aafwi_batch_aa_destroy", _vp)
_sig("aafwi_adjoint_gradient", _vp, _vp, _vp, _vp, _vp)
_sig("aafwi_adjoint_from_residual", _vp, _vp, _vp)
_sig("aafwi_born", _vp, _vp, _vp, _vp)
_sig("aafwi_born_adjoint", _vp, _vp, _vp, _vp)
_sig("aafwi_aa_create", _i64, _i32, _f64, _vp, ctypes.POINTER(_vp))
_sig("aafwi_aa_reset", _vp)
_sig("aafwi_aa_destroy", _vp)
_sig("aafwi_aa_step", _vp, _vp, _vp, _f32, _vp, _vp, _vp, _vp)
_sig("aafwi_aa_last_cond", _vp, _vp)
_sig("aafwi_aa_set_solver", _vp, ctypes.c_int)
_sig("aafwi_aa_set_damping", _vp, _f32)
_sig("aafwi_aa_set_weights", _vp, _vp)
AA_GRAM, AA_QR = 0, 1
_sig("aafwi_blend", _vp, _i64, _f32, _vp, _vp, _vp)
_sig("aafwi_dot", _vp, _i64, _vp, _vp, _vp, _vp)
_sig("aafwi_dot_diff", _vp, _i64, _vp, _vp, _vp, _vp, _vp)
_sig("aafwi_axpy", _vp, _i64, _f32, _vp, _vp)
_sig("aafwi_floor", _vp, _i64, _f32, _vp)
_sig("aafwi_laplacian_filter", _vp, _i32, _i32, _f32, _vp, _vp)
_sig("aafwi_scale", _vp, _i64, _f32, _vp, _vp)
_sig("aafwi_kernel_timing", _vp, ctypes.c_int)
_sig("aafwi_kernel_timing_read", _vp, ctypes.c_int, ctypes.POINTER(_f64), ctypes.POINTER(_i64))
_sig("aafwi_set_tile", _vp, _i32, _i32)
_sig("aafwi_get_tile", _vp, _i32, ctypes.POINTER(_i32))
_sig("aafwi_set_time_blocking", _vp, ctypes.c_int)
_sig("aafwi_set_time_blocking_kernel", _vp, _i32, ctypes.c_int)
_sig("aafwi_set_tile_order", _vp, _i32, _i32)
_sig("aafwi_get_time_blocking", _vp, ctypes.POINTER(ctypes.c_int))
_sig("aafwi_set_full_storage", _vp, ctypes.c_int)
_sig("aafwi_get_full_storage", _vp, ctypes.POINTER(ctypes.c_int))
_sig("aafwi_batch_set_time_blocking", _vp, ctypes.c_int)
_sig("aafwi_batch_get_time_blocking", _vp, ctypes.POINTER(ctypes.c_int))
_sig("aafwi_batch_destroy", _vp)
_sig("aafwi_batch_misfits", _vp, _vp)
_sig("aafwi_batch_set_active", _vp, _vp)
_sig("aafwi_batch_forward", _vp, ctypes.c_int)
_sig("aafwi_batch_backward", _vp)
_sig("aafwi_batch_use_graphs", _vp, ctypes.c_int)
_sig("aafwi_batch_device_bytes", _vp, ctypes.POINTER(_i64))
_sig("aafwi_batch_set_tile", _vp, _i32, _i32)
_sig("aafwi_batch_set_instance_tile", _vp, _i32, _i32, _i32)
_sig("aafwi_batch_kernel_timing", _vp, ctypes.c_int)
_sig("aafwi_batch_kernel_timing_read", _vp, ctypes.c_int, ctypes.POINTER(_f64), ctypes.POINTER(_i64))
_lib.aafwi_last_error.argtypes = []
_lib.aafwi_last_error.restype = ctypes.c_char_p


def _check(code: int):
    if code != AAFWI_OK:
        raise AafwiError(code, (_lib.aafwi_last_error() or b"").decode())


def _ptr(t: torch.Tensor, dtype=torch.float32, numel=None, name="tensor") -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements (got {t.numel()})")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def make_geometry_struct(geom, ckpt_every=0):
    """Pack a geometry description (any object with the documented fields)."""
    keep = dict(
        src_iz=np.ascontiguousarray(geom.src_iz, dtype=np.int32).ravel(),
        src_ix=np.ascontiguousarray(geom.src_ix, dtype=np.int32).ravel(),
        rec_iz=np.ascontiguousarray(geom.rec_iz, dtype=np.int32).ravel(),
        rec_ix=np.ascontiguousarray(geom.rec_ix, dtype=np.int32).ravel(),
        wavelet=np.ascontiguousarray(geom.wavelet, dtype=np.float32).ravel(),
    )
    ip = ctypes.POINTER(ctypes.c_int32)
    s = _Geometry(
        nz=int(geom.nz), nx=int(geom.nx), nb=int(geom.nb), h=float(geom.h), dt=float(geom.dt),
        nt=int(geom.nt), vref=float(geom.vref), refl=float(geom.refl),
        vmax_bound=float(geom.vmax_bound), nshots=int(keep["src_iz"].size),
        nrec=int(keep["rec_iz"].size // max(1, keep["src_iz"].size)),
        src_iz=keep["src_iz"].ctypes.data_as(ip), src_ix=keep["src_ix"].ctypes.data_as(ip),
        rec_iz=keep["rec_iz"].ctypes.data_as(ip), rec_ix=keep["rec_ix"].ctypes.data_as(ip),
        wavelet=keep["wavelet"].ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
        ckpt_every=int(ckpt_every))
    return s, keep


class Context:
    """One acquisition geometry on one GPU (all shots batched in every launch)."""

    def __init__(self, geom, stream=None, ckpt_every=0, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            self.nz, self.nx, self.nt = int(geom.nz), int(geom.nx), int(geom.nt)
            self.nb = int(geom.nb)
            # the smallest m the scheme runs (1 / vmax_bound^2, as the library rounds it)
            self.floor = float(np.float32(1.0 / (float(geom.vmax_bound) ** 2)))
            self.nshots = int(np.asarray(geom.src_iz).size)
            self.nrec = int(np.asarray(geom.rec_iz).size // self.nshots)
            s, self._keep = make_geometry_struct(geom, ckpt_every)
            h = _vp()
            _check(_lib.aafwi_create(ctypes.byref(s), _stream_handle(self.stream), ctypes.byref(h)))
            self._h = h
        self.n = self.nz * self.nx
        self.data_shape = (self.nshots, self.nt, self.nrec)
        # incremented by every call that replaces the kept checkpoints / model
        self.generation = 0

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.aafwi_destroy(self._h))
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

    # -- helpers --------------------------------------------------------------
    def _new(self, shape, dtype=torch.float32):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def device_bytes(self) -> int:
        v = _i64()
        _check(_lib.aafwi_device_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def sync(self):
        _check(_lib.aafwi_sync(self._h))

    # -- the calls -------------------------------------------------------------
    def forward_model(self, m, d=None, keep_ckpt=False):
        d = self._new(self.data_shape) if d is None else d
        self.generation += 1
        _check(_lib.aafwi_forward_model(self._h, _ptr(m, numel=self.n, name="m"),
                                        _ptr(d, numel=self.nshots * self.nt * self.nrec, name="d"),
                                        int(bool(keep_ckpt))))
        return d

    def residual_misfit(self, d, d_obs, r=None, J=None):
        N = self.nshots * self.nt * self.nrec
        r = self._new(self.data_shape) if r is None else r
        J = self._new((1,), torch.float64) if J is None else J
        _check(_lib.aafwi_residual_misfit(self._h, _ptr(d, numel=N, name="d"), _ptr(d_obs, numel=N, name="d_obs"),
                                          _ptr(r, numel=N, name="r"), _ptr(J, torch.float64, 1, "J")))
        return r, J

    def adjoint_gradient(self, m, d_obs, grad=None, J=None):
        grad = self._new((self.nz, self.nx)) if grad is None else grad
        J = self._new((1,), torch.float64) if J is None else J
        self.generation += 1
        _check(_lib.aafwi_adjoint_gradient(self._h, _ptr(m, numel=self.n, name="m"),
                                           _ptr(d_obs, numel=self.nshots * self.nt * self.nrec, name="d_obs"),
                                           _ptr(grad, numel=self.n, name="grad"), _ptr(J, torch.float64, 1, "J")))
        return grad, J

    def adjoint_from_residual(self, r, grad=None):
        grad = self._new((self.nz, self.nx)) if grad is None else grad
        _check(_lib.aafwi_adjoint_from_residual(self._h, _ptr(r, numel=self.nshots * self.nt * self.nrec, name="r"),
                                                _ptr(grad, numel=self.n, name="grad")))
        return grad

    def born(self, m0, dm, d=None):
        d = self._new(self.data_shape) if d is None else d
        self.generation += 1
        _check(_lib.aafwi_born(self._h, _ptr(m0, numel=self.n, name="m0"), _ptr(dm, numel=self.n, name="dm"),
                               _ptr(d, numel=self.nshots * self.nt * self.nrec, name="d")))
        return d

    def born_adjoint(self, m0, y, image=None):
        image = self._new((self.nz, self.nx)) if image is None else image
        self.generation += 1
        _check(_lib.aafwi_born_adjoint(self._h, _ptr(m0, numel=self.n, name="m0"),
                                       _ptr(y, numel=self.nshots * self.nt * self.nrec, name="y"),
                                       _ptr(image, numel=self.n, name="image")))
        return image

    # -- instrumentation -------------------------------------------------------
    def kernel_timing(self, every: int):
        _check(_lib.aafwi_kernel_timing(self._h, int(every)))

    def kernel_timing_read(self, kernel_id: int):
        ms, cnt = _f64(), _i64()
        _check(_lib.aafwi_kernel_timing_read(self._h, int(kernel_id), ctypes.byref(ms), ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    def set_tile(self, rows_per_wave: int, kernel_id: int = -1):
        _check(_lib.aafwi_set_tile(self._h, int(kernel_id), int(rows_per_wave)))

    def set_tile_order(self, order: int, kernel_id: int = -1):
        """0: x-tiles of a strip adjacent in the launch; 1: strips of a column adjacent."""
        _check(_lib.aafwi_set_tile_order(self._h, int(kernel_id), int(order)))

    def set_time_blocking(self, enable: bool, kernel_id: int = -1):
        """Two time steps per launch or one (for one of the forward,
        recompute, adjoint kernels, or all three); results are bitwise equal."""
        if kernel_id < 0:
            _check(_lib.aafwi_set_time_blocking(self._h, int(bool(enable))))
        else:
            _check(_lib.aafwi_set_time_blocking_kernel(self._h, int(kernel_id), int(bool(enable))))

    def time_blocking(self) -> int:
        """Bit mask: bit k set when kernel k advances two steps per launch."""
        v = ctypes.c_int()
        _check(_lib.aafwi_get_time_blocking(self._h, ctypes.byref(v)))
        return int(v.value)

    def set_full_storage(self, enable: bool):
        """Keep q-hat of every forward step in device memory (no recompute in
        the backward pass) or checkpoints; results are bitwise equal.  Drops
        kept state; raises AafwiError (out of memory) and keeps the previous
        layout when the device cannot hold the full one."""
        self.generation += 1
        _check(_lib.aafwi_set_full_storage(self._h, int(bool(enable))))

    def full_storage(self) -> bool:
        v = ctypes.c_int()
        _check(_lib.aafwi_get_full_storage(self._h, ctypes.byref(v)))
        return bool(v.value)

    def full_storage_bytes(self) -> int:
        """Device bytes of the q planes of every step (the full layout's main buffer)."""
        pitch = (self.nx + 2 * self.nb + 63) // 64 * 64
        return 4 * self.nt * self.nshots * (self.nz + 2 * self.nb) * pitch

    def get_tile(self, kernel_id: int) -> int:
        v = _i32()
        _check(_lib.aafwi_get_tile(self._h, int(kernel_id), ctypes.byref(v)))
        return int(v.value)


class _BatchIO(ctypes.Structure):
    _fields_ = [("m", _vp), ("d_obs", _vp), ("r", _vp), ("grad", _vp)]


_sig("aafwi_batch_create", ctypes.POINTER(_Geometry), ctypes.POINTER(_BatchIO), _i32, _i32, _vp,
     ctypes.POINTER(_vp))


class Batch:
    """N uneven inversion instances advanced together (one launch per step).

    The batch owns torch buffers per instance: ``m[i]`` (model, read by
    forward), ``d_obs[i]`` (observed data), ``r[i]`` (residual, written by
    forward) and ``grad[i]`` (written by backward).  A non-default stream is
    created for it (graph capture cannot use the null stream); run torch work
    that touches these buffers under ``with torch.cuda.stream(batch.stream)``.
    """

    def __init__(self, geoms, d_obs, ckpt_every=0, use_graphs=True, stream=None):
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.N = len(geoms)
        self.geoms = list(geoms)
        self.floors = [float(np.float32(1.0 / (float(g.vmax_bound) ** 2))) for g in self.geoms]
        self.shapes, self.data_shapes = [], []
        structs, self._keep = [], []
        for g in geoms:
            s, keep = make_geometry_struct(g, 0)
            structs.append(s)
            self._keep.append(keep)
            S = int(np.asarray(g.src_iz).size)
            R = int(np.asarray(g.rec_iz).size // S)
            self.shapes.append((int(g.nz), int(g.nx)))
            self.data_shapes.append((S, int(g.nt), R))
        with torch.cuda.stream(self.stream):
            self.m = [torch.zeros(sh, dtype=torch.float32, device=self.device) for sh in self.shapes]
            self.grad = [torch.zeros(sh, dtype=torch.float32, device=self.device) for sh in self.shapes]
            self.r = [torch.zeros(ds, dtype=torch.float32, device=self.device) for ds in self.data_shapes]
            self.d_obs = []
            for i, x in enumerate(d_obs):
                t = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous().clone()
                if tuple(t.shape) != self.data_shapes[i]:
                    t = t.reshape(self.data_shapes[i])
                self.d_obs.append(t)
            self.J = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        self.stream.synchronize()
        garr = (_Geometry * self.N)(*structs)
        ioarr = (_BatchIO * self.N)(*[_BatchIO(self.m[i].data_ptr(), self.d_obs[i].data_ptr(),
                                               self.r[i].data_ptr(), self.grad[i].data_ptr())
                                      for i in range(self.N)])
        h = _vp()
        _check(_lib.aafwi_batch_create(garr, ioarr, self.N, int(ckpt_every), _stream_handle(self.stream),
                                       ctypes.byref(h)))
        self._h = h
        if use_graphs:
            _check(_lib.aafwi_batch_use_graphs(self._h, 1))
        self.active = np.ones(self.N, dtype=np.uint8)

    def set_time_blocking(self, enable: bool):
        _check(_lib.aafwi_batch_set_time_blocking(self._h, int(bool(enable))))

    def set_active(self, mask):
        self.active = np.ascontiguousarray(mask, dtype=np.uint8)
        _check(_lib.aafwi_batch_set_active(self._h, self.active.ctypes.data))

    def forward(self, keep_ckpt=True):
        _check(_lib.aafwi_batch_forward(self._h, int(bool(keep_ckpt))))

    def backward(self):
        _check(_lib.aafwi_batch_backward(self._h))

    def misfits(self):
        _check(_lib.aafwi_batch_misfits(self._h, _ptr(self.J, torch.float64, self.N, "J")))
        self.stream.synchronize()
        return self.J.cpu().numpy()

    def use_graphs(self, enable):
        _check(_lib.aafwi_batch_use_graphs(self._h, int(bool(enable))))

    def set_tile(self, rows_per_wave: int, kernel_id: int = -1):
        _check(_lib.aafwi_batch_set_tile(self._h, int(kernel_id), int(rows_per_wave)))

    def set_instance_tile(self, inst: int, rows_per_wave: int, kernel_id: int = -1):
        """Strip height of one instance (0 = the batch setting)."""
        _check(_lib.aafwi_batch_set_instance_tile(self._h, int(inst), int(kernel_id), int(rows_per_wave)))

    def time_blocking(self) -> int:
        """Bit k set when stepping kernel k runs two steps per launch."""
        v = ctypes.c_int(0)
        _check(_lib.aafwi_batch_get_time_blocking(self._h, ctypes.byref(v)))
        return int(v.value)

    def device_bytes(self) -> int:
        v = _i64()
        _check(_lib.aafwi_batch_device_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def kernel_timing(self, every: int):
        _check(_lib.aafwi_batch_kernel_timing(self._h, int(every)))

    def kernel_timing_read(self, kernel_id: int):
        ms, cnt = _f64(), _i64()
        _check(_lib.aafwi_batch_kernel_timing_read(self._h, int(kernel_id), ctypes.byref(ms), ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.aafwi_batch_destroy(self._h))
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


class AA:
    """Device state of Algorithm 2 (Steps 1-3) for vectors of n values."""

    def __init__(self, n: int, M: int, cond_max: float = 1e5, stream=None, solver: str = "gram"):
        self.n, self.M = int(n), int(M)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = _vp()
        _check(_lib.aafwi_aa_create(self.n, self.M, float(cond_max), _stream_handle(self.stream), ctypes.byref(h)))
        self._h = h
        self.gamma = torch.zeros(self.M, dtype=torch.float64, device=self.device)
        self.mk = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.cond = torch.zeros(1, dtype=torch.float64, device=self.device)
        if solver != "gram":
            self.set_solver(solver)

    def set_solver(self, solver: str):
        """'gram' (FP64 normal equations) or 'qr' (rank-updated QR); clears the history."""
        code = {"gram": AA_GRAM, "qr": AA_QR}[solver]
        _check(_lib.aafwi_aa_set_solver(self._h, code))

    def set_damping(self, beta: float):
        """Damping of the mixed step (eq. AAupdate0); 1 = none."""
        _check(_lib.aafwi_aa_set_damping(self._h, float(beta)))

    def set_weights(self, w):
        """Per-entry least-squares weights (device tensor of n floats, kept
        referenced here) or None; clears the history."""
        self._w = None if w is None else w
        _check(_lib.aafwi_aa_set_weights(self._h, None if w is None else _ptr(w, numel=self.n, name="w")))

    def reset(self):
        _check(_lib.aafwi_aa_reset(self._h))

    def step(self, p, g, eta, p_bar=None, p_tilde=None):
        p_bar = torch.empty_like(p) if p_bar is None else p_bar
        p_tilde = torch.empty_like(p) if p_tilde is None else p_tilde
        _check(_lib.aafwi_aa_step(self._h, _ptr(p, numel=self.n, name="p"), _ptr(g, numel=self.n, name="g"),
                                  float(eta), _ptr(p_bar, numel=self.n, name="p_bar"),
                                  _ptr(p_tilde, numel=self.n, name="p_tilde"),
                                  _ptr(self.gamma, torch.float64, self.M, "gamma"),
                                  _ptr(self.mk, torch.int32, 1, "mk")))
        return p_bar, p_tilde

    def last_cond(self):
        _check(_lib.aafwi_aa_last_cond(self._h, _ptr(self.cond, torch.float64, 1, "cond")))
        return self.cond

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.aafwi_aa_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchAA:
    """Anderson state of many instances stepped together (one launch
    sequence for all of them); instance i holds vectors of ns[i] values."""

    def __init__(self, ns, M: int, cond_max: float = 1e5, stream=None):
        self.ns = [int(x) for x in ns]
        self.N, self.M = len(self.ns), int(M)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.device("cuda", torch.cuda.current_device())
        arr = (ctypes.c_int64 * self.N)(*self.ns)
        h = _vp()
        _check(_lib.aafwi_batch_aa_create(self.N, arr, self.M, float(cond_max), _stream_handle(self.stream),
                                          ctypes.byref(h)))
        self._h = h
        self.gamma = torch.zeros(self.N, self.M, dtype=torch.float64, device=self.device)
        self.mk = torch.zeros(self.N, dtype=torch.int32, device=self.device)

    def _ptrs(self, ts, name, active):
        out = (_vp * self.N)()
        for i, t in enumerate(ts):
            if active is None or active[i]:
                out[i] = _ptr(t, numel=self.ns[i], name=f"{name}[{i}]")
        return out

    def step(self, ps, gs, etas, pbars, ptildes, active=None):
        """pbar[i] = G(p[i]) and ptilde[i] for every active instance."""
        act = None if active is None else (ctypes.c_uint8 * self.N)(*[1 if a else 0 for a in active])
        eta = (ctypes.c_float * self.N)(*[float(e) for e in etas])
        _check(_lib.aafwi_batch_aa_step(self._h, self._ptrs(ps, "p", active), self._ptrs(gs, "g", active), eta,
                                        self._ptrs(pbars, "p_bar", active), self._ptrs(ptildes, "p_tilde", active),
                                        act))

    def reset(self, which=None):
        w = None if which is None else (ctypes.c_uint8 * self.N)(*[1 if a else 0 for a in which])
        _check(_lib.aafwi_batch_aa_reset(self._h, w))

    def state(self):
        """(gamma [N][M] float64, mk [N] int32) of the last step, on the device."""
        _check(_lib.aafwi_batch_aa_state(self._h, _ptr(self.gamma, torch.float64, self.N * self.M, "gamma"),
                                         _ptr(self.mk, torch.int32, self.N, "mk")))
        return self.gamma, self.mk

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.aafwi_batch_aa_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Reducer:
    """FP64 dot products with a private device workspace (one per instance)."""

    def __init__(self, stream=None, device=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.ws = torch.empty(DOT_WORKSPACE, dtype=torch.float64, device=dev)

    def dot(self, x, y, out=None):
        out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
        n = x.numel()
        _check(_lib.aafwi_dot(_stream_handle(self.stream), n, _ptr(x, numel=n, name="x"),
                              _ptr(y, numel=n, name="y"), _ptr(out, torch.float64, 1, "out"),
                              _ptr(self.ws, torch.float64, DOT_WORKSPACE, "workspace")))
        return out

    def dot_diff(self, g, a, b, out=None):
        out = torch.empty(1, dtype=torch.float64, device=g.device) if out is None else out
        n = g.numel()
        _check(_lib.aafwi_dot_diff(_stream_handle(self.stream), n, _ptr(g, numel=n, name="g"),
                                   _ptr(a, numel=n, name="a"), _ptr(b, numel=n, name="b"),
                                   _ptr(out, torch.float64, 1, "out"),
                                   _ptr(self.ws, torch.float64, DOT_WORKSPACE, "workspace")))
        return out


def residual_misfit_noalloc(d, d_obs, r, J, stream=None):
    """r = d - d_obs and J = 1/2 sum r^2 (one device double) through the
    entry point that allocates nothing; r and J are caller tensors."""
    n = d.numel()
    _check(_lib.aafwi_residual_misfit_noalloc(_stream_handle(stream), n, _ptr(d, numel=n, name="d"),
                                              _ptr(d_obs, numel=n, name="d_obs"), _ptr(r, numel=n, name="r"),
                                              _ptr(J, torch.float64, 1, "J")))
    return r, J


def blend(lam, p_tilde, p_bar, out=None, stream=None):
    out = torch.empty_like(p_bar) if out is None else out
    n = p_bar.numel()
    _check(_lib.aafwi_blend(_stream_handle(stream), n, float(lam), _ptr(p_tilde, numel=n, name="p_tilde"),
                            _ptr(p_bar, numel=n, name="p_bar"), _ptr(out, numel=n, name="out")))
    return out


def scale(a, x, out=None, stream=None):
    """out = a * x (out may be x)."""
    out = torch.empty_like(x) if out is None else out
    n = x.numel()
    _check(_lib.aafwi_scale(_stream_handle(stream), n, float(a), _ptr(x, numel=n, name="x"),
                            _ptr(out, numel=n, name="out")))
    return out


def laplacian_filter(image, h, out=None, stream=None):
    """-Lap_h of an [nz][nx] image (the Laplacian-filtered RTM image)."""
    if image.dim() != 2:
        raise ValueError("image must be [nz][nx]")
    out = torch.empty_like(image) if out is None else out
    nz, nx = image.shape
    _check(_lib.aafwi_laplacian_filter(_stream_handle(stream), nz, nx, float(h), _ptr(image, name="image"),
                                       _ptr(out, numel=nz * nx, name="out")))
    return out


def floor_(x, floor, stream=None):
    """x = max(x, floor) in place (an iterate kept in the stable domain)."""
    n = x.numel()
    _check(_lib.aafwi_floor(_stream_handle(stream), n, float(floor), _ptr(x, numel=n, name="x")))
    return x


def axpy(a, x, y, stream=None):
    n = y.numel()
    _check(_lib.aafwi_axpy(_stream_handle(stream), n, float(a), _ptr(x, numel=n, name="x"),
                           _ptr(y, numel=n, name="y")))
    return y


_sig("aafwi_stream_probe", _vp, _i32, _i64, _i32, _vp, _vp, _vp)


def stream_probe(kind, a, b, c=None, blocks_per_cu=4, stream=None):
    """One launch of the HBM stream probe over equal-size device buffers:
    kind 0 read a, 1 write b, 2 copy a -> b, 3 b = a + 2c."""
    nbytes = b.numel() * b.element_size()
    for name, t in (("a", a), ("c", c)):
        if t is not None and t.numel() * t.element_size() != nbytes:
            raise ValueError(f"{name} must have the size of b")
    _check(_lib.aafwi_stream_probe(_stream_handle(stream), int(kind), nbytes, int(blocks_per_cu),
                                   None if a is None else a.data_ptr(), b.data_ptr(),
                                   None if c is None else c.data_ptr()))


_sig("aafwi_cnn_create", _i32, _i32, _i32, _vp, _vp, ctypes.POINTER(_vp))
_sig("aafwi_cnn_destroy", _vp)
_sig("aafwi_cnn_set_weights", _vp, _vp)
_sig("aafwi_cnn_get_weights", _vp, _vp)
_sig("aafwi_cnn_forward", _vp, _i32, _vp, _vp, _vp, _vp)
_sig("aafwi_cnn_gradients", _vp, _i32, _vp, _vp, _vp, _vp, _vp)
_sig("aafwi_cnn_train_step", _vp, _i32, _vp, _vp, _vp, _f32, _vp)
_sig("aafwi_cnn_set_fused", _vp, _i32)
CNN_PARAMS = 19296
CNN_SHAPES = ((32, 2, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (1, 32, 3, 3))


def cnn_flatten(ws) -> np.ndarray:
    """Per-layer [C_out][C_in][3][3] arrays -> the flat FP32 host layout."""
    flat = np.concatenate([np.asarray(w, np.float32).reshape(-1) for w in ws])
    if flat.size != CNN_PARAMS:
        raise ValueError(f"expected {CNN_PARAMS} weights, got {flat.size}")
    return np.ascontiguousarray(flat)


def cnn_unflatten(flat):
    out, o = [], 0
    for shp in CNN_SHAPES:
        n = int(np.prod(shp))
        out.append(np.asarray(flat[o:o + n]).reshape(shp))
        o += n
    return out


class CNN:
    """Learned direction network on [B][nz][nx] images (device tensors)."""

    def __init__(self, nz: int, nx: int, max_batch: int, weights, stream=None):
        self.nz, self.nx, self.max_batch = int(nz), int(nx), int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.device("cuda", torch.cuda.current_device())
        w = cnn_flatten(weights) if isinstance(weights, (list, tuple)) else np.ascontiguousarray(weights, np.float32)
        if w.size != CNN_PARAMS:
            raise ValueError(f"expected {CNN_PARAMS} weights")
        h = _vp()
        _check(_lib.aafwi_cnn_create(self.nz, self.nx, self.max_batch, w.ctypes.data, _stream_handle(self.stream),
                                     ctypes.byref(h)))
        self._h = h
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.device)

    def _images(self, x, name):
        if x.dim() == 2:
            x = x.unsqueeze(0)
        B = x.shape[0]
        if not (1 <= B <= self.max_batch):
            raise ValueError(f"batch of {B} images outside [1, {self.max_batch}]")
        _ptr(x, numel=B * self.nz * self.nx, name=name)
        return x, B

    def set_weights(self, weights):
        w = cnn_flatten(weights) if isinstance(weights, (list, tuple)) else np.ascontiguousarray(weights, np.float32)
        _check(_lib.aafwi_cnn_set_weights(self._h, w.ctypes.data))

    def set_fused(self, on: bool):
        """Second and third convolutions in one kernel (default) or two."""
        _check(_lib.aafwi_cnn_set_fused(self._h, int(bool(on))))

    def get_weights(self) -> np.ndarray:
        w = np.empty(CNN_PARAMS, np.float32)
        _check(_lib.aafwi_cnn_get_weights(self._h, w.ctypes.data))
        return w

    def forward(self, g, m, z=None, d=None):
        """(z, d) with d = softplus(z) * g; pass z=False or d=False to skip one."""
        g, B = self._images(g, "g")
        m, _ = self._images(m, "m")
        with torch.cuda.stream(self.stream):
            zt = torch.empty_like(g) if z is None else z
            dt = torch.empty_like(g) if d is None else d
        zp = 0 if zt is False else _ptr(zt, numel=g.numel(), name="z")
        dp = 0 if dt is False else _ptr(dt, numel=g.numel(), name="d")
        _check(_lib.aafwi_cnn_forward(self._h, B, g.data_ptr(), m.data_ptr(), zp or None, dp or None))
        return (None if zt is False else zt), (None if dt is False else dt)

    def gradients(self, g, m, s, grad=None):
        """Weight gradient (flat, device) and the batch loss (device double)."""
        g, B = self._images(g, "g")
        m, _ = self._images(m, "m")
        s, _ = self._images(s, "s")
        with torch.cuda.stream(self.stream):
            grad = torch.empty(CNN_PARAMS, dtype=torch.float32, device=self.device) if grad is None else grad
        _check(_lib.aafwi_cnn_gradients(self._h, B, g.data_ptr(), m.data_ptr(), s.data_ptr(),
                                        _ptr(grad, numel=CNN_PARAMS, name="grad"),
                                        _ptr(self.loss_dev, torch.float64, 1, "loss")))
        return grad, self.loss_dev

    def train_step(self, g, m, s, lr: float = 1e-3):
        """One Adam step; returns the device loss (before the step)."""
        g, B = self._images(g, "g")
        m, _ = self._images(m, "m")
        s, _ = self._images(s, "s")
        _check(_lib.aafwi_cnn_train_step(self._h, B, g.data_ptr(), m.data_ptr(), s.data_ptr(), float(lr),
                                         _ptr(self.loss_dev, torch.float64, 1, "loss")))
        return self.loss_dev

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.aafwi_cnn_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

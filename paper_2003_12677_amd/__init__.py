"""MI355X sparse Fubini-Radon tomography: thin Python binding of libtomo.so.

Every computation runs in the HIP library; this module only marshals arguments
(torch tensors -> device pointers, torch's current stream -> hipStream_t).  The
names follow the C ABI in ``include/tomo.h``.  ``torch`` is imported before the
library is loaded so that the process holds a single HIP runtime.
"""

from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtomo.so")

VALUES = {"f32": 0, "bf16": 1, "f16": 2}
VALUE_MASK = {"f32": 1, "bf16": 2, "f16": 4}
FILTERS = {"none": 0, "ramlak": 1, "shepp": 2, "hamming": 3, "density": 4}
SOLVERS = {"cgls": 0, "sirt_bb": 1, "cgnr": 2, "sirt_bb_normal": 3, "tv_split_bregman": 4}
STATUS = {0: "TOMO_OK", -1: "TOMO_EINVAL", -2: "TOMO_ENOMEM", -3: "TOMO_EHIP", -4: "TOMO_EFFT",
          -5: "TOMO_ESTATE", -6: "TOMO_EUNSUPPORTED"}


class TomoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class tomo_geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("kw", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("values", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("beta", ctypes.c_double), ("center", ctypes.c_double),
                ("angles", ctypes.POINTER(ctypes.c_double))]


class tomo_op_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("kw", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("beta", ctypes.c_double), ("center", ctypes.c_double),
                ("n_polar", ctypes.c_int64), ("n_cart", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("cols_touched", ctypes.c_int64), ("polar_nonempty", ctypes.c_int64),
                ("adj_sell_rows", ctypes.c_int64), ("adj_sell_padding", ctypes.c_int64),
                ("adj_medium_rows", ctypes.c_int64), ("adj_long_rows", ctypes.c_int64),
                ("adj_long_chunks", ctypes.c_int64), ("device", ctypes.c_int32),
                ("values", ctypes.c_uint32)]


class tomo_tuning(ctypes.Structure):
    _fields_ = [("fwd_channels_per_lane", ctypes.c_int32), ("adj_channels_per_lane", ctypes.c_int32),
                ("adj_sell_max", ctypes.c_int32), ("adj_sell_sigma", ctypes.c_int32),
                ("adj_medium_max", ctypes.c_int32), ("adj_chunk", ctypes.c_int32),
                ("fwd_tiled", ctypes.c_int32), ("adj_tiled", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("tile_points", ctypes.c_int32), ("adj_tile_points", ctypes.c_int32),
                ("normal_tiled", ctypes.c_int32), ("adj_sell_xcd_rows", ctypes.c_int32),
                ("adj_medium_xcd_rows", ctypes.c_int32), ("fwd_rows_per_group", ctypes.c_int32),
                ("det_fft", ctypes.c_int32), ("grid_fft", ctypes.c_int32),
                ("adj_sell_tiles", ctypes.c_int32), ("tile_strip", ctypes.c_int32),
                ("adj_dense_mode", ctypes.c_int32), ("adj_seg_chunks", ctypes.c_int32),
                ("adj_run", ctypes.c_int32)]


class tomo_solve_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("refine_outer", ctypes.c_int32), ("values", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("out_resnorm", ctypes.c_void_p), ("tv_mu", ctypes.c_double),
                ("tv_lambda", ctypes.c_double)]


# name -> (restype, argtypes); every symbol declared in include/tomo.h
_P = ctypes.c_void_p
_I = ctypes.c_int32
class tomo_step(ctypes.Structure):
    _fields_ = [("op", _P), ("kind", _I), ("batch", _I), ("values", _I), ("reserved", _I),
                ("inp", _P), ("out", _P), ("aux", _P)]


STEPS = {"spmm_pair": 0, "project": 1, "backproject": 2, "normal": 3}


class tomo_stack_item(ctypes.Structure):
    _fields_ = [("op", _P), ("batch", _I), ("reserved", _I), ("inp", _P), ("out", _P), ("aux", _P)]

SIGNATURES = {
    "tomo_build_operator": (ctypes.c_int, [ctypes.POINTER(tomo_geometry), ctypes.c_int, ctypes.POINTER(_P)]),
    "tomo_project": (ctypes.c_int, [_P, _P, _P, _I, _I, _P]),
    "tomo_backproject": (ctypes.c_int, [_P, _P, _P, _I, _I, _P]),
    "tomo_irradon": (ctypes.c_int, [_P, _P, _P, _I, _I, _I, _P]),
    "tomo_slice_fwd": (ctypes.c_int, [_P, _P, _P, _I, _I, _P]),
    "tomo_slice_adj": (ctypes.c_int, [_P, _P, _P, _I, _I, _I, _P]),
    "tomo_solve": (ctypes.c_int, [_P, _P, _P, _I, ctypes.POINTER(tomo_solve_opts), _P]),
    "tomo_normal": (ctypes.c_int, [_P, _P, _P, _I, _I, _I, _P]),
    "tomo_autotune": (ctypes.c_int, [_P, _I, _I, _I, ctypes.POINTER(tomo_tuning),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "tomo_export_normal": (ctypes.c_int, [_P, _I, _P]),
    "tomo_tv": (ctypes.c_int, [_P, _P, _I, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "tomo_tv_noalloc": (ctypes.c_int, [_P, _P, _I, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "tomo_density_filter": (ctypes.c_int, [_P, _I, ctypes.POINTER(ctypes.c_double)]),
    "tomo_export_density": (ctypes.c_int, [_P, _P]),
    "tomo_graph_create": (ctypes.c_int, [ctypes.POINTER(tomo_step), _I, ctypes.POINTER(_P)]),
    "tomo_graph_launch": (ctypes.c_int, [_P, _P]),
    "tomo_graph_destroy": (None, [_P]),
    "tomo_stack_create": (ctypes.c_int, [ctypes.POINTER(tomo_stack_item), _I, _I, ctypes.POINTER(_P)]),
    "tomo_stack_launch": (ctypes.c_int, [_P, _P]),
    "tomo_stack_destroy": (None, [_P]),
    "tomo_op_info_get": (ctypes.c_int, [_P, ctypes.POINTER(tomo_op_info)]),
    "tomo_export_csr": (ctypes.c_int, [_P, _I, _P, _P, _P]),
    "tomo_export_factors": (ctypes.c_int, [_P, _I, _P, _P]),
    "tomo_check_layouts": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "tomo_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(tomo_tuning)]),
    "tomo_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(tomo_tuning)]),
    "tomo_destroy_operator": (None, [_P]),
    "tomo_last_error": (ctypes.c_char_p, []),
    "tomo_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtomo.so (built by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_2003_12677_amd.build`)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != 0:
        raise TomoError(status, _lib.tomo_last_error().decode())


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device: int) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need(t: torch.Tensor, shape, device: int, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32 or not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be a float32 tensor on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Operator:
    """A built operator (``tomo_build_operator``); device -1 builds a host-only operator."""

    def __init__(self, n: int, n_angles: int, n_det: int, *, grid: int = 0, kw: int = 3,
                 max_batch: int = 32, values=("f32",), beta: float = math.nan,
                 center: float = math.nan, angles=None, device: int = 0):
        lib = load()
        self._handle = None
        self._angles = None
        g = tomo_geometry()
        g.n, g.n_angles, g.n_det, g.grid, g.kw, g.max_batch = n, n_angles, n_det, grid, kw, max_batch
        g.values = sum(VALUE_MASK[v] for v in values)
        g.reserved = 0
        g.beta = beta
        g.center = center
        if angles is not None:
            self._angles = (ctypes.c_double * n_angles)(*[float(a) for a in angles])
            g.angles = ctypes.cast(self._angles, ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib.tomo_build_operator(ctypes.byref(g), device, ctypes.byref(h)))
        self._handle = h
        self.device = device
        self.info = self.op_info()
        self.n, self.n_angles, self.n_det = n, n_angles, n_det
        self.grid = self.info.grid
        self.kw = self.info.kw

    # ---- lifecycle ---------------------------------------------------------------------
    def destroy_operator(self) -> None:
        if self._handle is not None and _lib is not None:
            _lib.tomo_destroy_operator(self._handle)
        self._handle = None

    close = destroy_operator

    def __del__(self):
        try:
            self.destroy_operator()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy_operator()

    # ---- info / export -------------------------------------------------------------------
    def op_info(self) -> tomo_op_info:
        info = tomo_op_info()
        _check(_lib.tomo_op_info_get(self._handle, ctypes.byref(info)))
        return info

    def export_csr(self, which: int):
        """Host CSR copy: ``(rowptr int64, col int32, val float64)``; which 0 = S^dagger, 1 = S."""
        import numpy as np
        info = self.info
        rows = info.n_polar if which == 0 else info.n_cart
        rp = np.empty(rows + 1, dtype=np.int64)
        col = np.empty(info.nnz, dtype=np.int32)
        val = np.empty(info.nnz, dtype=np.float64)
        _check(_lib.tomo_export_csr(self._handle, which, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val

    def get_tuning(self) -> dict:
        t = tomo_tuning()
        _check(_lib.tomo_get_tuning(self._handle, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in tomo_tuning._fields_}

    def set_tuning(self, **changes) -> dict:
        """``tomo_set_tuning`` with the given fields changed; returns the new tuning."""
        cur = self.get_tuning()
        unknown = set(changes) - set(cur)
        if unknown:
            raise KeyError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(changes)
        t = tomo_tuning(**cur)
        _check(_lib.tomo_set_tuning(self._handle, ctypes.byref(t)))
        self.info = self.op_info()
        return self.get_tuning()

    def autotune(self, batch: int, values: str = "f32", rounds: int = 1) -> dict:
        """``tomo_autotune``: search and apply the fastest SpMM tuning for ``batch`` slices;
        returns the tuning with the measured ``fwd_ms`` / ``adj_ms``."""
        t = tomo_tuning()
        f, a = ctypes.c_double(), ctypes.c_double()
        _check(_lib.tomo_autotune(self._handle, batch, VALUES[values], rounds, ctypes.byref(t),
                                  ctypes.byref(f), ctypes.byref(a)))
        self.info = self.op_info()
        out = {name: getattr(t, name) for name, _ in tomo_tuning._fields_}
        out.update(fwd_ms=f.value, adj_ms=a.value)
        return out

    def density_filter(self, iters: int = 100) -> float:
        """``tomo_density_filter``: compute the density weights (kept for filter="density");
        returns ||S D_v - kappa(0)^2 1||."""
        r = ctypes.c_double()
        _check(_lib.tomo_density_filter(self._handle, iters, ctypes.byref(r)))
        return r.value

    def export_density(self):
        """Density weights on the host: float32 [L * n_angles], FFT-ordered polar rows."""
        import numpy as np
        w = np.empty(self.grid * self.n_angles, dtype=np.float32)
        _check(_lib.tomo_export_density(self._handle, w.ctypes.data))
        return w

    def check_layouts(self) -> float:
        """``tomo_check_layouts``: host replay of every kernel layout against the CSR products."""
        err = ctypes.c_double()
        _check(_lib.tomo_check_layouts(self._handle, ctypes.byref(err)))
        return err.value

    def export_factors(self, filter: str = "none"):
        import numpy as np
        kd = np.empty(self.n, dtype=np.float64)
        d = np.empty(self.grid, dtype=np.float64)
        _check(_lib.tomo_export_factors(self._handle, FILTERS[filter], kd.ctypes.data, d.ctypes.data))
        return kd, d

    # ---- operators -------------------------------------------------------------------------
    def _image_shape(self, b):
        return (b, self.n, self.n)

    def _sino_shape(self, b):
        return (b, self.n_angles, self.n_det)

    def project(self, x: torch.Tensor, y: torch.Tensor | None = None, values: str = "f32") -> torch.Tensor:
        B = x.shape[0]
        _need(x, self._image_shape(B), self.device, "x")
        if y is None:
            y = torch.empty(self._sino_shape(B), dtype=torch.float32, device=x.device)
        _need(y, self._sino_shape(B), self.device, "y")
        _check(_lib.tomo_project(self._handle, _ptr(x), _ptr(y), B, VALUES[values], _stream(self.device)))
        return y

    def backproject(self, y: torch.Tensor, x: torch.Tensor | None = None, values: str = "f32") -> torch.Tensor:
        B = y.shape[0]
        _need(y, self._sino_shape(B), self.device, "y")
        if x is None:
            x = torch.empty(self._image_shape(B), dtype=torch.float32, device=y.device)
        _need(x, self._image_shape(B), self.device, "x")
        _check(_lib.tomo_backproject(self._handle, _ptr(y), _ptr(x), B, VALUES[values], _stream(self.device)))
        return x

    def irradon(self, y: torch.Tensor, x: torch.Tensor | None = None, values: str = "f32",
                filter: str = "hamming") -> torch.Tensor:
        B = y.shape[0]
        _need(y, self._sino_shape(B), self.device, "y")
        if x is None:
            x = torch.empty(self._image_shape(B), dtype=torch.float32, device=y.device)
        _need(x, self._image_shape(B), self.device, "x")
        _check(_lib.tomo_irradon(self._handle, _ptr(y), _ptr(x), B, VALUES[values], FILTERS[filter],
                                 _stream(self.device)))
        return x

    def cart_shape(self, batch: int):
        """Shape of the Cartesian Fourier grid buffer as float32: (G*G, C, 2)."""
        return (self.grid * self.grid, (batch + 1) // 2, 2)

    def polar_shape(self, batch: int):
        """Shape of the polar Fourier buffer as float32: (L*n_angles, C, 2)."""
        return (self.grid * self.n_angles, (batch + 1) // 2, 2)

    def slice_fwd(self, Xc: torch.Tensor, batch: int, Yp: torch.Tensor | None = None,
                  values: str = "f32") -> torch.Tensor:
        _need(Xc, self.cart_shape(batch), self.device, "Xc")
        if Yp is None:
            Yp = torch.empty(self.polar_shape(batch), dtype=torch.float32, device=Xc.device)
        _need(Yp, self.polar_shape(batch), self.device, "Yp")
        _check(_lib.tomo_slice_fwd(self._handle, _ptr(Xc), _ptr(Yp), batch, VALUES[values],
                                   _stream(self.device)))
        return Yp

    def slice_adj(self, Yp: torch.Tensor, batch: int, Xc: torch.Tensor | None = None,
                  values: str = "f32", filter: str = "none") -> torch.Tensor:
        _need(Yp, self.polar_shape(batch), self.device, "Yp")
        if Xc is None:
            Xc = torch.empty(self.cart_shape(batch), dtype=torch.float32, device=Yp.device)
        _need(Xc, self.cart_shape(batch), self.device, "Xc")
        _check(_lib.tomo_slice_adj(self._handle, _ptr(Yp), _ptr(Xc), batch, VALUES[values],
                                   FILTERS[filter], _stream(self.device)))
        return Xc

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, *, method: str = "cgls",
              iters: int = 10, refine_outer: int = 1, values: str = "f32", filter: str = "none",
              use_x0: bool = False, resnorm: torch.Tensor | None = None, tv_mu: float = 0.0,
              tv_lambda: float = 0.0) -> torch.Tensor:
        """``tomo_solve``.  For ``method="tv_split_bregman"``, ``refine_outer`` is the number of
        Bregman steps, ``iters`` the CG steps in each, ``tv_mu`` / ``tv_lambda`` the weights."""
        B = b.shape[0]
        _need(b, self._sino_shape(B), self.device, "b")
        if x is None:
            x = torch.empty(self._image_shape(B), dtype=torch.float32, device=b.device)
        _need(x, self._image_shape(B), self.device, "x")
        if resnorm is not None:
            if resnorm.dtype != torch.float64 or not resnorm.is_cuda or resnorm.numel() < B:
                raise ValueError("resnorm must be a float64 device tensor with >= batch entries")
        o = tomo_solve_opts(SOLVERS[method], iters, refine_outer, VALUES[values], FILTERS[filter],
                            1 if use_x0 else 0, _ptr(resnorm), float(tv_mu), float(tv_lambda))
        _check(_lib.tomo_solve(self._handle, _ptr(b), _ptr(x), B, ctypes.byref(o), _stream(self.device)))
        return x

    def normal(self, x: torch.Tensor, out: torch.Tensor | None = None, values: str = "f32",
               filter: str = "none") -> torch.Tensor:
        """``tomo_normal``: A^T D A x through the normal-operator stencil (no 1D FFTs)."""
        B = x.shape[0]
        _need(x, self._image_shape(B), self.device, "x")
        if out is None:
            out = torch.empty_like(x)
        _need(out, self._image_shape(B), self.device, "out")
        _check(_lib.tomo_normal(self._handle, _ptr(x), _ptr(out), B, VALUES[values],
                                FILTERS[filter], _stream(self.device)))
        return out

    def export_normal(self, filter: str = "none"):
        """Host float64 stencil of W = S diag(D) S^dagger: array [grid*grid, (2kw-1)^2]."""
        import numpy as np
        d = 2 * self.kw - 1
        w = np.empty((self.grid * self.grid, d * d), dtype=np.float64)
        _check(_lib.tomo_export_normal(self._handle, FILTERS[filter], w.ctypes.data))
        return w

    def tv(self, x: torch.Tensor, eps: float = 1e-8, weight: float = 1.0, *, value: bool = True,
           grad: bool = True):
        """``tomo_tv``: (per-slice weight*TV_eps as float64 [B] or None, weight*gradient or None)."""
        B = x.shape[0]
        _need(x, self._image_shape(B), self.device, "x")
        v = torch.empty(B, dtype=torch.float64, device=x.device) if value else None
        g = torch.empty_like(x) if grad else None
        _check(_lib.tomo_tv(self._handle, _ptr(x), B, float(eps), float(weight), _ptr(g), _ptr(v),
                            _stream(self.device)))
        return v, g

    def tv_noalloc(self, x: torch.Tensor, value: torch.Tensor | None, grad: torch.Tensor | None,
                   eps: float = 1e-8, weight: float = 1.0) -> None:
        """``tomo_tv_noalloc``: as :meth:`tv` into caller-given ``value`` (float64 [B]) and
        ``grad`` (like x) tensors, either may be None; the library allocates nothing."""
        B = x.shape[0]
        _need(x, self._image_shape(B), self.device, "x")
        if grad is not None:
            _need(grad, self._image_shape(B), self.device, "grad")
        if value is not None and (value.dtype != torch.float64 or tuple(value.shape) != (B,)
                                  or not value.is_cuda or value.device.index != self.device):
            raise ValueError(f"value must be a float64 tensor of shape ({B},) on cuda:{self.device}")
        _check(_lib.tomo_tv_noalloc(self._handle, _ptr(x), B, float(eps), float(weight), _ptr(grad),
                                    _ptr(value), _stream(self.device)))

class Graph:
    """``tomo_graph_create``: several operators' steps recorded as one HIP graph.

    ``steps`` is a list of dicts with keys ``op`` (:class:`Operator`), ``kind`` (one of
    ``STEPS``), ``batch``, ``values`` and the tensors ``inp``, ``out`` (and ``aux`` for
    ``"spmm_pair"``).  The graph keeps references to the operators and tensors it records."""

    def __init__(self, steps):
        self._keep = list(steps)
        arr = (tomo_step * len(steps))()
        for k, st in enumerate(steps):
            aux = st.get("aux")
            arr[k] = tomo_step(st["op"]._handle, STEPS[st["kind"]], st["batch"],
                               VALUES[st.get("values", "f32")], 0, _ptr(st["inp"]),
                               _ptr(st["out"]), _ptr(aux))
        h = ctypes.c_void_p()
        _check(_lib.tomo_graph_create(arr, len(steps), ctypes.byref(h)))
        self._handle = h
        self.device = steps[0]["op"].device

    def launch(self) -> None:
        _check(_lib.tomo_graph_launch(self._handle, _stream(self.device)))

    def close(self) -> None:
        if self._handle is not None and _lib is not None:
            _lib.tomo_graph_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_operator(*args, **kwargs) -> Operator:
    """``tomo_build_operator``: see :class:`Operator`."""
    return Operator(*args, **kwargs)


def version() -> str:
    return load().tomo_version().decode()


class Stack:
    """``tomo_stack_create``: persistent SpMM pairs over several operators.  ``items`` is a list
    of dicts with keys ``op`` (:class:`Operator`), ``batch`` and the tensors ``inp`` (Cartesian
    input), ``out`` (polar product) and ``aux`` (adjoint of ``out``); all items use the value
    type ``values``.  The stack keeps references to the operators and tensors."""

    def __init__(self, items, values: str = "f32"):
        self._keep = list(items)
        self._handle = None
        arr = (tomo_stack_item * len(items))()
        dev = items[0]["op"].device
        for k, it in enumerate(items):
            op, b = it["op"], it["batch"]
            _need(it["inp"], op.cart_shape(b), dev, "inp")
            _need(it["out"], op.polar_shape(b), dev, "out")
            _need(it["aux"], op.cart_shape(b), dev, "aux")
            arr[k] = tomo_stack_item(op._handle, b, 0, it["inp"].data_ptr(), it["out"].data_ptr(),
                                     it["aux"].data_ptr())
        self.device = dev
        h = ctypes.c_void_p()
        _check(_lib.tomo_stack_create(arr, len(items), VALUES[values], ctypes.byref(h)))
        self._handle = h

    def launch(self) -> None:
        _check(_lib.tomo_stack_launch(self._handle, _stream(self.device)))

    def close(self) -> None:
        if self._handle is not None and _lib is not None:
            _lib.tomo_stack_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

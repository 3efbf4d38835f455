"""w-stacking dirty imager for AMD MI355X (gfx950): Python binding of libwsimg.so.

Every step of the imaging path runs in the HIP kernels behind the C ABI declared in
include/wsimg.h; this module only checks tensor arguments, hands device pointers and the
current HIP stream to the library, and turns status codes into exceptions.  PyTorch is
used for device memory and streams.  There is no CPU fallback: if the library is not
built, importing the binding's entry points raises.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Tuple

from . import _lib

__all__ = ["WsimgError", "Plan", "image", "image_noalloc", "grid", "predict", "query", "stage_names", "version",
           "ImagingOperator"]


class WsimgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"wsimg status {status}: {message}")
        self.status = status
        self.message = message


def _check(status: int):
    if status != _lib.WSIMG_OK:
        L = _lib.load()
        raise WsimgError(status, L.wsimg_last_error().decode() or L.wsimg_status_string(status).decode())


def version() -> int:
    return int(_lib.load().wsimg_version())


def stage_names():
    L = _lib.load()
    return [L.wsimg_stage_name(i).decode() for i in range(_lib.WSIMG_N_KERNELS)]


def _params(n, pixel_rad, n_wplanes, support, beta, precision, w_range, normalize, fold_w, pad,
            complex_out=False, w_support=0):
    p = _lib.Params()
    p.n, p.n_wplanes, p.support = int(n), int(n_wplanes), int(support)
    p.precision = _prec_code(precision)
    p.pixel_rad = float(pixel_rad)
    p.beta = 0.0 if beta is None else float(beta)
    p.flags = 0
    if w_range is not None:
        p.w_lo, p.w_hi = float(w_range[0]), float(w_range[1])
        p.flags |= _lib.WSIMG_FIXED_WRANGE
    if not normalize:
        p.flags |= _lib.WSIMG_UNNORMALIZED
    if fold_w:
        p.flags |= _lib.WSIMG_FOLD_W
    if pad not in (1, 2):
        raise ValueError("pad must be 1 or 2")
    if pad == 2:
        p.flags |= _lib.WSIMG_PAD2
    if complex_out:
        p.flags |= _lib.WSIMG_COMPLEX_OUT
    p.w_support = int(w_support)
    return p


def query(n: int, pixel_rad: float, n_wplanes: int, support: int = 7, beta: Optional[float] = None,
          precision: str = "f32", max_vis: int = 0, max_channels: int = 1,
          w_range: Optional[Tuple[float, float]] = None, normalize: bool = True, fold_w: bool = False,
          pad: int = 1, w_support: int = 0) -> dict:
    """What a Plan of these arguments would hold (wsimg_plan_query): shapes and device bytes,
    computed on the host without a GPU."""
    L = _lib.load()
    p = _params(n, pixel_rad, n_wplanes, support, beta, precision, w_range, normalize, fold_w, pad,
                w_support=w_support)
    i = _lib.PlanInfo()
    _check(L.wsimg_plan_query(ctypes.byref(p), int(max_vis), int(max_channels), ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in _lib.PlanInfo._fields_}


def _prec_code(precision: str) -> int:
    if precision in ("f32", "float32"):
        return _lib.WSIMG_F32
    if precision in ("f64", "float64"):
        return _lib.WSIMG_F64
    raise ValueError(f"precision must be 'f32' or 'f64', got {precision!r}")


class Plan:
    """One imaging geometry on one GPU: owns the library plan and its device scratch."""

    def __init__(self, n: int, pixel_rad: float, n_wplanes: int, support: int = 7,
                 beta: Optional[float] = None, precision: str = "f32", max_vis: int = 0,
                 w_range: Optional[Tuple[float, float]] = None, device=None, max_channels: int = 1,
                 normalize: bool = True, fold_w: bool = False, pad: int = 1, complex_out: bool = False,
                 w_support: int = 0):
        import torch

        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.precision = "f32" if _prec_code(precision) == _lib.WSIMG_F32 else "f64"
        self.n, self.n_wplanes, self.support = int(n), int(n_wplanes), int(support)
        p = _params(n, pixel_rad, n_wplanes, support, beta, precision, w_range, normalize, fold_w, pad,
                    complex_out, w_support)
        self.pad = int(pad)
        self.complex_out = bool(complex_out)
        self._L = _lib.load()
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(self._L.wsimg_plan_create_batch(ctypes.byref(self._h), ctypes.byref(p), int(max_vis),
                                                   int(max_channels), ctypes.c_void_p(stream)))
        self.max_vis = int(max_vis)
        self.max_channels = int(max_channels)

    # -- helpers -------------------------------------------------------------------------
    def _dtypes(self):
        t = self._torch
        return (t.complex64, t.float32) if self.precision == "f32" else (t.complex128, t.float64)

    def _image_dtype(self):
        cdt, rdt = self._dtypes()
        return cdt if self.complex_out else rdt

    def _args(self, uvw, vis, weights):
        t = self._torch
        cdt, rdt = self._dtypes()
        m = int(uvw.shape[0]) if uvw.dim() == 2 else -1
        if uvw.dtype != t.float64 or uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be a float64 tensor of shape [M, 3] (metres)")
        if vis.dtype != cdt or vis.shape != (m,):
            raise ValueError(f"vis must be {cdt} of shape [M]")
        if weights.dtype != rdt or weights.shape != (m,):
            raise ValueError(f"weights must be {rdt} of shape [M]")
        for name, x in (("uvw", uvw), ("vis", vis), ("weights", weights)):
            if x.device != self.device:
                raise ValueError(f"{name} must live on {self.device}")
            if not x.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        return m

    def _stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        _check(self._L.wsimg_plan_set_stream(self._h, ctypes.c_void_p(s)))

    def _run(self, fn, uvw, vis, weights, freq_hz, out, stats):
        m = self._args(uvw, vis, weights)
        self._stream()
        st = _lib.Stats()
        status = fn(self._h, m, ctypes.c_void_p(uvw.data_ptr()), ctypes.c_void_p(vis.data_ptr()),
                    ctypes.c_void_p(weights.data_ptr()), float(freq_hz), ctypes.c_void_p(out.data_ptr()),
                    ctypes.byref(st) if stats else None)
        _check(status)
        if stats:
            return out, {f: getattr(st, f) for f, _ in _lib.Stats._fields_}
        return out

    # -- the calls -------------------------------------------------------------------------
    def image(self, uvw, vis, weights, freq_hz: float, out=None, stats: bool = False):
        """Dirty image [n, n] (wsimg_image): real, or complex for a plan made with
        complex_out=True.  With stats=True returns (image, stats dict)."""
        rdt = self._image_dtype()
        if out is None:
            out = self._torch.empty((self.n, self.n), dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != (self.n, self.n) or not out.is_contiguous() or out.device != self.device:
            raise ValueError(f"out must be a contiguous [n, n] {rdt} tensor on the plan's device")
        return self._run(self._L.wsimg_image, uvw, vis, weights, freq_hz, out, stats)

    def image_batch(self, uvw, vis, weights, row_counts, freqs_hz, out=None, stats: bool = False):
        """Dirty images [n_channels, n, n] of the channels laid out one after another in the
        inputs: channel c owns the next row_counts[c] rows and has frequency freqs_hz[c]
        (wsimg_image_batch).  With stats=True returns (images, [stats dict per channel])."""
        rdt = self._image_dtype()
        counts = [int(x) for x in row_counts]
        freqs = [float(x) for x in freqs_hz]
        nch = len(counts)
        if nch != len(freqs) or nch < 1:
            raise ValueError("row_counts and freqs_hz must have the same, non-zero length")
        m = self._args(uvw, vis, weights)
        if sum(counts) != m:
            raise ValueError(f"row_counts sum to {sum(counts)}, the inputs hold {m} rows")
        shape = (nch, self.n, self.n)
        if out is None:
            out = self._torch.empty(shape, dtype=rdt, device=self.device)
        elif out.dtype != rdt or tuple(out.shape) != shape or not out.is_contiguous() or out.device != self.device:
            raise ValueError(f"out must be a contiguous [n_channels, n, n] {rdt} tensor")
        self._stream()
        c_counts = (ctypes.c_int64 * nch)(*counts)
        c_freqs = (ctypes.c_double * nch)(*freqs)
        st = (_lib.Stats * nch)()
        status = self._L.wsimg_image_batch(self._h, nch, c_counts, ctypes.c_void_p(uvw.data_ptr()),
                                           ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
                                           c_freqs, ctypes.c_void_p(out.data_ptr()), st if stats else None)
        _check(status)
        if stats:
            return out, [{f: getattr(st[c], f) for f, _ in _lib.Stats._fields_} for c in range(nch)]
        return out

    def predict(self, uvw, weights, freq_hz: float, image, out=None, stats: bool = False):
        """Prediction (wsimg_predict): visibilities [M] of the plan's complex dtype from a real
        image [n, n]; the transpose of the unnormalised imaging operator."""
        t = self._torch
        cdt, rdt = self._dtypes()
        m = int(uvw.shape[0]) if uvw.dim() == 2 else -1
        if uvw.dtype != t.float64 or uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be a float64 tensor of shape [M, 3] (metres)")
        if weights.dtype != rdt or weights.shape != (m,):
            raise ValueError(f"weights must be {rdt} of shape [M]")
        if image.dtype != rdt or tuple(image.shape) != (self.n, self.n):
            raise ValueError(f"image must be {rdt} of shape [n, n]")
        for name, x in (("uvw", uvw), ("weights", weights), ("image", image)):
            if x.device != self.device:
                raise ValueError(f"{name} must live on {self.device}")
            if not x.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        if out is None:
            out = t.empty((m,), dtype=cdt, device=self.device)
        elif out.dtype != cdt or tuple(out.shape) != (m,) or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous [M] tensor of the plan's complex dtype on its device")
        self._stream()
        st = _lib.Stats()
        _check(self._L.wsimg_predict(self._h, m, ctypes.c_void_p(uvw.data_ptr()),
                                     ctypes.c_void_p(weights.data_ptr()), float(freq_hz),
                                     ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.byref(st) if stats else None))
        if stats:
            return out, {f: getattr(st, f) for f, _ in _lib.Stats._fields_}
        return out

    def grid(self, uvw, vis, weights, freq_hz: float, out=None, stats: bool = False):
        """The gridding step alone: complex grid [n_wplanes, n, n] (wsimg_grid)."""
        cdt, _ = self._dtypes()
        ng = self.pad * self.n
        shape = (self.n_wplanes, ng, ng)
        if out is None:
            out = self._torch.empty(shape, dtype=cdt, device=self.device)
        elif out.dtype != cdt or tuple(out.shape) != shape or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous [n_wplanes, n, n] tensor of the plan's complex dtype")
        return self._run(self._L.wsimg_grid, uvw, vis, weights, freq_hz, out, stats)

    def info(self) -> dict:
        i = _lib.PlanInfo()
        _check(self._L.wsimg_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _lib.PlanInfo._fields_}

    def set_timing(self, enable: bool = True):
        _check(self._L.wsimg_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        t = _lib.Timing()
        _check(self._L.wsimg_read_timing(self._h, ctypes.byref(t)))
        names = stage_names()
        return {"calls": t.calls, "ms_total": t.ms_total, "ms": {names[i]: t.ms[i] for i in range(len(names))}}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.wsimg_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def image(uvw, vis, weights, freq_hz: float, *, n: int, pixel_rad: float, n_wplanes: int,
          support: int = 7, beta: Optional[float] = None, precision: Optional[str] = None,
          w_range=None, stats: bool = False, complex_out: bool = False, w_support: int = 0):
    """One-shot dirty image (creates and frees a plan); complex_out=True returns the complex
    image S / (sum W C C) instead of its real part; w_support > 0 spreads each visibility over
    that many w-planes with a Kaiser-Bessel kernel along w."""
    import torch
    if precision is None:
        precision = "f64" if vis.dtype == torch.complex128 else "f32"
    with Plan(n, pixel_rad, n_wplanes, support, beta, precision, max_vis=uvw.shape[0],
              w_range=w_range, device=uvw.device, complex_out=complex_out, w_support=w_support) as p:
        return p.image(uvw, vis, weights, freq_hz, stats=stats)


def image_noalloc(uvw, vis, weights, freq_hz: float, out, *, n: int, pixel_rad: float, n_wplanes: int,
                  support: int = 7, beta: Optional[float] = None, w_range=None, stats: bool = False):
    """Dirty image into the caller's `out` [n, n] through wsimg_image_noalloc: no plan and no
    device allocation (the library's static scratch array holds every intermediate buffer);
    precision from the vis dtype.  Raises WsimgError (WSIMG_E_CAPACITY) when the geometry and
    row count need more than that array holds."""
    import torch
    precision = "f64" if vis.dtype == torch.complex128 else "f32"
    cdt, rdt = (torch.complex64, torch.float32) if precision == "f32" else (torch.complex128, torch.float64)
    m = int(uvw.shape[0]) if uvw.dim() == 2 else -1
    if uvw.dtype != torch.float64 or uvw.dim() != 2 or uvw.shape[1] != 3:
        raise ValueError("uvw must be a float64 tensor of shape [M, 3] (metres)")
    if vis.dtype != cdt or vis.shape != (m,) or weights.dtype != rdt or weights.shape != (m,):
        raise ValueError(f"vis must be {cdt} [M] and weights {rdt} [M]")
    if out.dtype != rdt or tuple(out.shape) != (n, n):
        raise ValueError(f"out must be {rdt} of shape [n, n]")
    for name, x in (("uvw", uvw), ("vis", vis), ("weights", weights), ("out", out)):
        if x.device != uvw.device or not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous on {uvw.device}")
    L = _lib.load()
    p = _params(n, pixel_rad, n_wplanes, support, beta, precision, w_range, True, False, 1)
    st = _lib.Stats()
    with torch.cuda.device(uvw.device):
        stream = torch.cuda.current_stream(uvw.device).cuda_stream
        _check(L.wsimg_image_noalloc(ctypes.byref(p), m, ctypes.c_void_p(uvw.data_ptr()),
                                     ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
                                     float(freq_hz), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream),
                                     ctypes.byref(st) if stats else None))
    if stats:
        return out, {f: getattr(st, f) for f, _ in _lib.Stats._fields_}
    return out


def grid(uvw, vis, weights, freq_hz: float, *, n: int, pixel_rad: float, n_wplanes: int,
         support: int = 7, beta: Optional[float] = None, precision: Optional[str] = None,
         w_range=None, stats: bool = False, w_support: int = 0):
    """One-shot gridding step (creates and frees a plan)."""
    import torch
    if precision is None:
        precision = "f64" if vis.dtype == torch.complex128 else "f32"
    with Plan(n, pixel_rad, n_wplanes, support, beta, precision, max_vis=uvw.shape[0],
              w_range=w_range, device=uvw.device, w_support=w_support) as p:
        return p.grid(uvw, vis, weights, freq_hz, stats=stats)


def predict(uvw, weights, freq_hz: float, image, *, pixel_rad: float, n_wplanes: int, support: int = 7,
            beta: Optional[float] = None, w_range=None, stats: bool = False):
    """One-shot prediction (creates and frees a plan); precision from the image dtype."""
    import torch
    precision = "f64" if image.dtype == torch.float64 else "f32"
    with Plan(int(image.shape[0]), pixel_rad, n_wplanes, support, beta, precision, max_vis=uvw.shape[0],
              w_range=w_range, device=uvw.device) as p:
        return p.predict(uvw, weights, freq_hz, image, stats=stats)


from .operator import ImagingOperator  # noqa: E402

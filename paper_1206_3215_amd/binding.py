"""ctypes binding of libpst.so: the C-ABI entry points under the same names.

Only argument marshalling happens here; every step of the computation runs
in the library's HIP kernels.  Device memory and streams come from PyTorch:
fields are torch tensors on the GPU, passed by data pointer, and a plan runs
on the torch stream that was current when it was created (or the one given).

Importing this module fails with ImportError if libpst.so has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: it brings its HIP runtime, which libpst then binds to (loading
# libpst first would map a second HIP runtime into the process, and device
# pointers from one are not usable by the other)
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpst.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1206_3215_amd.build`")
lib = C.CDLL(_LIB_PATH)

# enums (include/pst.h)
PST_OK, PST_ERR_INVALID, PST_ERR_UNSUPPORTED, PST_ERR_OOM, PST_ERR_DEVICE, \
    PST_ERR_NOT_CONVERGED, PST_ERR_NONFINITE = range(7)
STATUS_NAMES = ["OK", "INVALID", "UNSUPPORTED", "OOM", "DEVICE", "NOT_CONVERGED", "NONFINITE"]
PST_FP32, PST_FP64 = 0, 1
PST_C2C, PST_R2C = 0, 1
PST_NLS, PST_SG, PST_NS = 0, 1, 2
PASS_NLS_ROW, PASS_NLS_COL, PASS_SG_ROW, PASS_SG_COL, PASS_NS_ROW, PASS_NS_COL = range(6)
EQ = {"nls": PST_NLS, "sg": PST_SG, "ns": PST_NS}


class Domain(C.Structure):
    _fields_ = [("lx", C.c_double), ("ly", C.c_double), ("x0", C.c_double), ("y0", C.c_double)]


class NlsParams(C.Structure):
    _fields_ = [("d", Domain), ("dt", C.c_double), ("g", C.c_double)]


class SgParams(C.Structure):
    _fields_ = [("d", Domain), ("dt", C.c_double)]


class NsParams(C.Structure):
    _fields_ = [("d", Domain), ("dt", C.c_double), ("nu", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int)]


class Request(C.Structure):
    _fields_ = [("eq", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("prec", C.c_int),
                ("nsteps", C.c_int), ("params", C.c_void_p), ("f0", C.c_void_p),
                ("f1", C.c_void_p), ("dev_status", C.c_void_p)]


_vp = C.c_void_p
_SIGS = {
    "fft2d_plan": [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.POINTER(_vp)],
    "pst_workspace_size": [_vp, C.POINTER(C.c_size_t)],
    "pst_set_workspace": [_vp, _vp, C.c_size_t],
    "fft2d_exec": [_vp, _vp, _vp, C.c_int],
    "fft2d_destroy": [_vp],
    "nls_step": [_vp, _vp, C.POINTER(NlsParams), C.c_int],
    "sg_start": [_vp, _vp, _vp, _vp, _vp, C.POINTER(SgParams)],
    "sg_step": [_vp, _vp, _vp, C.POINTER(SgParams), C.c_int],
    "sg_step_noalloc": [_vp, _vp, _vp, C.POINTER(SgParams), C.c_int],
    "ns_step": [_vp, _vp, C.POINTER(NsParams), C.c_int, _vp],
    "conserved_quantities": [_vp, C.c_int, _vp, _vp, _vp, C.POINTER(C.c_double)],
    "pst_sync_status": [_vp, C.POINTER(C.c_int)],
    "solve_batch": [C.POINTER(Request), C.c_int, _vp],
    "pst_batch_cache_bytes": [C.POINTER(C.c_size_t)],
    "pst_batch_cache_release": [],
    "pst_autotune": [_vp, C.c_int, C.POINTER(C.c_int)],
    "pst_set_column_variant": [_vp, C.c_int],
    "pst_column_variant_info": [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "pst_row_variant_info": [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "pst_set_row_variant": [_vp, C.c_int],
    "pst_get_variants": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "pst_profile_enable": [_vp, C.c_int],
    "pst_profile_read": [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)],
    "pst_last_error": [],
    "pst_version": [],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_char_p if _name in ("pst_last_error", "pst_version") else C.c_int


class PstError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.pst_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")


def check(status: int, where: str) -> None:
    if status != PST_OK:
        raise PstError(status, where)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("field must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("field must be contiguous")
    return t.data_ptr()


def _check(t, name: str, dtype, numel: int | None = None, min_numel: int | None = None) -> None:
    """Validate a tensor before its pointer crosses the boundary: the kernels
    trust the dtype and size they are given (a wrong one reads or writes out
    of bounds).  Raises ValueError; checks nothing about the values."""
    if t is None:
        raise ValueError(f"{name} is required")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected at least {min_numel}")


def domain(d) -> Domain:
    return Domain(float(d.lx), float(d.ly), float(d.x0), float(d.y0))


class Plan:
    """Owns a pst_plan and its torch-allocated workspace."""

    def __init__(self, nx: int, ny: int, kind: int = PST_C2C, prec: int = PST_FP32,
                 batch: int = 1, stream=None):
        import torch
        self.nx, self.ny, self.kind, self.prec, self.batch = nx, ny, kind, prec, batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        check(lib.fft2d_plan(nx, ny, kind, prec, batch, _vp(self.stream.cuda_stream), C.byref(h)),
              "fft2d_plan")
        self.handle = h
        n = C.c_size_t()
        check(lib.pst_workspace_size(h, C.byref(n)), "pst_workspace_size")
        self.workspace = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device="cuda")
        check(lib.pst_set_workspace(h, _vp(self.workspace.data_ptr()), n.value), "pst_set_workspace")

    @property
    def real_dtype(self):
        import torch
        return torch.float32 if self.prec == PST_FP32 else torch.float64

    @property
    def complex_dtype(self):
        import torch
        return torch.complex64 if self.prec == PST_FP32 else torch.complex128

    def close(self):
        if getattr(self, "handle", None):
            lib.fft2d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks (sizes and dtypes the kernels rely on) -------------
    @property
    def _points(self) -> int:
        return self.batch * self.ny * self.nx

    @property
    def _half_points(self) -> int:
        return self.batch * self.ny * (self.nx // 2 + 1)

    def _need_kind(self, kind: int, who: str) -> None:
        if self.kind != kind:
            raise ValueError(f"{who} needs a {'C2C' if kind == PST_C2C else 'R2C'} plan")

    def _complex_field(self, t, name: str) -> None:
        _check(t, name, self.complex_dtype, self._points)

    def _real_field(self, t, name: str) -> None:
        _check(t, name, self.real_dtype, self._points)

    # -- entry points -----------------------------------------------------
    def fft2d_exec(self, inp, out, sign: int) -> None:
        if self.kind == PST_C2C:
            self._complex_field(inp, "in")
            self._complex_field(out, "out")
        elif sign == -1:
            self._real_field(inp, "in")
            _check(out, "out", self.complex_dtype, self._half_points)
        else:
            _check(inp, "in", self.complex_dtype, self._half_points)
            self._real_field(out, "out")
        check(lib.fft2d_exec(self.handle, _ptr(inp), _ptr(out), sign), "fft2d_exec")

    def nls_step(self, psi, d, dt: float, g: float, nsteps: int) -> None:
        self._need_kind(PST_C2C, "nls_step")
        self._complex_field(psi, "psi")
        p = NlsParams(domain(d), dt, g)
        check(lib.nls_step(self.handle, _ptr(psi), C.byref(p), nsteps), "nls_step")

    def sg_start(self, u0, v0, u_prev, u_curr, d, dt: float) -> None:
        self._need_kind(PST_R2C, "sg_start")
        for t, name in ((u0, "u0"), (v0, "v0"), (u_prev, "u_prev"), (u_curr, "u_curr")):
            self._real_field(t, name)
        p = SgParams(domain(d), dt)
        check(lib.sg_start(self.handle, _ptr(u0), _ptr(v0), _ptr(u_prev), _ptr(u_curr), C.byref(p)),
              "sg_start")

    def sg_step(self, u_prev, u_curr, d, dt: float, nsteps: int) -> None:
        self._need_kind(PST_R2C, "sg_step")
        self._real_field(u_prev, "u_prev")
        self._real_field(u_curr, "u_curr")
        p = SgParams(domain(d), dt)
        check(lib.sg_step(self.handle, _ptr(u_prev), _ptr(u_curr), C.byref(p), nsteps), "sg_step")

    def sg_step_noalloc(self, u_prev, u_curr, d, dt: float, nsteps: int) -> None:
        """sg_step with the library's fixed scratch array as workspace."""
        self._need_kind(PST_R2C, "sg_step_noalloc")
        self._real_field(u_prev, "u_prev")
        self._real_field(u_curr, "u_curr")
        p = SgParams(domain(d), dt)
        check(lib.sg_step_noalloc(self.handle, _ptr(u_prev), _ptr(u_curr), C.byref(p), nsteps), "sg_step_noalloc")

    def ns_step(self, omega, d, dt: float, nu: float, nsteps: int, tol: float = 1e-10,
                max_iter: int = 50, fixed_iters: int = 0, dev_iters=None) -> None:
        import torch
        self._need_kind(PST_R2C, "ns_step")
        self._real_field(omega, "omega")
        if dev_iters is not None:
            _check(dev_iters, "dev_iters", torch.int32, min_numel=max(nsteps, 0) * self.batch)
        p = NsParams(domain(d), dt, nu, tol, max_iter, fixed_iters)
        check(lib.ns_step(self.handle, _ptr(omega), C.byref(p), nsteps, _ptr(dev_iters)), "ns_step")

    def conserved_quantities(self, eq: str, f0, f1=None, d=None, dt: float = 0.0, g: float = 1.0,
                             nu: float = 0.0) -> np.ndarray:
        if eq not in EQ:
            raise ValueError(f"unknown equation {eq!r}")
        self._need_kind(PST_C2C if eq == "nls" else PST_R2C, f"conserved_quantities({eq})")
        if eq == "nls":
            self._complex_field(f0, "f0")
        else:
            self._real_field(f0, "f0")
            if eq == "sg":
                self._real_field(f1, "f1")
        out = np.zeros(4 * self.batch, dtype=np.float64)
        if eq == "nls":
            p = NlsParams(domain(d), dt, g)
        elif eq == "sg":
            p = SgParams(domain(d), dt)
        else:
            p = NsParams(domain(d), dt, nu, 0.0, 1, 0)
        st = lib.conserved_quantities(self.handle, EQ[eq], _ptr(f0), _ptr(f1), C.byref(p),
                                      out.ctypes.data_as(C.POINTER(C.c_double)))
        check(st, "conserved_quantities")
        return out.reshape(self.batch, 4)

    def autotune(self, eq: str) -> int:
        """Pick the fastest column variant for this plan; returns it."""
        w = C.c_int()
        check(lib.pst_autotune(self.handle, EQ[eq], C.byref(w)), "pst_autotune")
        return w.value

    def set_column_variant(self, variant: int) -> None:
        check(lib.pst_set_column_variant(self.handle, int(variant)), "pst_set_column_variant")

    def set_row_variant(self, variant: int) -> None:
        check(lib.pst_set_row_variant(self.handle, int(variant)), "pst_set_row_variant")

    def variants(self) -> tuple:
        """(row variant, column variant) the plan runs."""
        r, c = C.c_int(), C.c_int()
        check(lib.pst_get_variants(self.handle, C.byref(r), C.byref(c)), "pst_get_variants")
        return r.value, c.value

    def column_variants(self) -> list:
        """[(columns per block, values per thread, split, radix)] of every
        column variant compiled for this plan's ny and kind, by number."""
        return column_variants(self.prec, self.ny, self.kind == PST_C2C)

    def profile_enable(self, on: bool = True) -> None:
        check(lib.pst_profile_enable(self.handle, int(on)), "pst_profile_enable")

    def profile_read(self, pass_id: int):
        """(total_ms, launches) recorded for a pass since the last read."""
        ms, n = C.c_double(), C.c_int()
        check(lib.pst_profile_read(self.handle, pass_id, C.byref(ms), C.byref(n)), "pst_profile_read")
        return ms.value, n.value

    def sync_status(self) -> int:
        s = C.c_int()
        check(lib.pst_sync_status(self.handle, C.byref(s)), "pst_sync_status")
        return s.value


def column_variants(prec: int, n: int, single_field: bool) -> list:
    """[(columns per block, values per thread, split, radix)] by variant number."""
    out = []
    w, v, sp, r = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    while lib.pst_column_variant_info(prec, n, len(out), int(single_field), C.byref(w), C.byref(v),
                                      C.byref(sp), C.byref(r)) == 0:
        out.append((w.value, v.value, sp.value, r.value))
    return out


def row_variants(prec: int, n: int) -> list:
    """[(row pairs per block (0: one line per block), values per thread,
    split, radix)] of the NLS in-place row pass by variant number."""
    out = []
    p, v, sp, r = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    while lib.pst_row_variant_info(prec, n, len(out), C.byref(p), C.byref(v), C.byref(sp), C.byref(r)) == 0:
        out.append((p.value, v.value, sp.value, r.value))
    return out


def make_params(eq: str, d, dt: float, g: float = 1.0, nu: float = 0.0, tol: float = 1e-10,
                max_iter: int = 50, fixed_iters: int = 0):
    if eq == "nls":
        return NlsParams(domain(d), dt, g)
    if eq == "sg":
        return SgParams(domain(d), dt)
    return NsParams(domain(d), dt, nu, tol, max_iter, fixed_iters)


def solve_batch(requests, stream=None) -> None:
    """Advance independent simulations in one call.

    requests: sequence of dicts with keys eq ("nls" | "sg" | "ns"), f0, f1
    (torch tensors; f1 only for "sg"), params (from make_params), nsteps,
    and optionally dev_status (a CUDA int32 tensor of one element).
    Fields keep their own storage; the library groups them by equation,
    size, precision and parameters.
    """
    import torch
    arr = (Request * len(requests))()
    keep = []
    ptypes = {"nls": NlsParams, "sg": SgParams, "ns": NsParams}
    for i, r in enumerate(requests):
        eq = r["eq"]
        if eq not in EQ:
            raise ValueError(f"request {i}: unknown equation {eq!r}")
        f0 = r["f0"]
        if f0 is None or f0.dim() < 2 or f0.numel() != f0.shape[-1] * f0.shape[-2]:
            raise ValueError(f"request {i}: f0 must hold one ny x nx field")
        allowed = (torch.complex64, torch.complex128) if eq == "nls" else (torch.float32, torch.float64)
        if f0.dtype not in allowed:
            raise ValueError(f"request {i}: f0 dtype {f0.dtype} does not suit equation {eq}")
        if eq == "sg":
            _check(r.get("f1"), f"request {i}: f1", f0.dtype, f0.numel())
        if r.get("dev_status") is not None:
            _check(r["dev_status"], f"request {i}: dev_status", torch.int32, min_numel=1)
        pr = r["params"]
        if not isinstance(pr, ptypes[eq]):
            raise ValueError(f"request {i}: params must be {ptypes[eq].__name__} for equation {eq}")
        prec = PST_FP64 if f0.dtype in (torch.float64, torch.complex128) else PST_FP32
        ny, nx = f0.shape[-2:]
        keep.append(pr)
        arr[i].eq = EQ[eq]
        arr[i].nx, arr[i].ny, arr[i].prec, arr[i].nsteps = nx, ny, prec, int(r["nsteps"])
        arr[i].params = C.cast(C.pointer(pr), C.c_void_p)
        arr[i].f0 = _ptr(f0)
        arr[i].f1 = _ptr(r.get("f1"))
        arr[i].dev_status = _ptr(r.get("dev_status"))
    st = stream if stream is not None else torch.cuda.current_stream()
    check(lib.solve_batch(arr, len(requests), _vp(st.cuda_stream)), "solve_batch")


def batch_cache_bytes() -> int:
    """Device bytes held by solve_batch's cached internal plans."""
    n = C.c_size_t()
    check(lib.pst_batch_cache_bytes(C.byref(n)), "pst_batch_cache_bytes")
    return int(n.value)


def batch_cache_release() -> None:
    """Free solve_batch's cached internal plans (waits for their streams)."""
    check(lib.pst_batch_cache_release(), "pst_batch_cache_release")


def version() -> str:
    return lib.pst_version().decode()

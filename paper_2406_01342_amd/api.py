"""Python binding of libpolyclean.so: the C ABI's functions under the same
names, taking torch device tensors for device buffers and numpy arrays for
host inputs.  Argument marshalling only; every operator step runs in the HIP
library.  Device buffers come from torch (its caching allocator) and calls
are issued on torch's current stream unless a stream is passed.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (PC_PREC_FP32, PC_PREC_FP64, PC_UV_METRES, PC_UV_WAVELENGTHS,  # noqa: F401
                   PcBatcherStats, PcGeometry, PcKernelStat, PcPlanInfo, PcSolveParams,
                   PcSolveResult, PolycleanError, check)

LIB = _lib.load()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: torch.Tensor, dtype, numel: int, name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


class Plan:
    """Owns a pc_plan handle (destroyed with the object)."""

    def __init__(self, handle: C.c_void_p, device: torch.device):
        self._h = handle
        self.device = device
        info = PcPlanInfo()
        check(LIB.pc_plan_get_info(self._h, C.byref(info)), "pc_plan_get_info")
        self.info = {k: getattr(info, k) for k, _ in PcPlanInfo._fields_}
        self.nvis = int(info.nvis)
        self.npix = int(info.npix)
        self.precision = int(info.precision)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            LIB.pc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _geometry(uv, npix, fov_rad, w, uv_units, freq_hz, nufft_eps, upsamp, precision):
    uv = np.ascontiguousarray(np.asarray(uv, dtype=np.float64))
    if uv.ndim != 2 or uv.shape[1] != 2:
        raise ValueError("uv must have shape (L, 2)")
    u = np.ascontiguousarray(uv[:, 0])
    v = np.ascontiguousarray(uv[:, 1])
    keep = [u, v]
    g = PcGeometry()
    g.nvis = uv.shape[0]
    g.u = u.ctypes.data_as(C.POINTER(C.c_double))
    g.v = v.ctypes.data_as(C.POINTER(C.c_double))
    if w is not None:
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        keep.append(w)
        g.w = w.ctypes.data_as(C.POINTER(C.c_double))
    g.uv_units = int(uv_units)
    g.freq_hz = float(freq_hz)
    g.npix = int(npix)
    g.fov_rad = float(fov_rad)
    g.nufft_eps = float(nufft_eps)
    g.upsamp = float(upsamp)
    g.precision = int(precision)
    return g, keep


def pc_device_pool_trim(device: int = 0) -> int:
    """Frees the device buffers parked in the library's pool on ``device``
    (released plans' and solvers' memory kept for reuse); returns the bytes."""
    n = C.c_size_t(0)
    check(LIB.pc_device_pool_trim(int(device), C.byref(n)), "pc_device_pool_trim")
    return int(n.value)


def pc_plan_footprint(uv, npix: int, fov_rad: float, *, w=None, uv_units=PC_UV_WAVELENGTHS,
                      freq_hz: float = 0.0, nufft_eps: float = 1e-5, upsamp: float = 2.0,
                      precision: int = PC_PREC_FP32) -> int:
    g, keep = _geometry(uv, npix, fov_rad, w, uv_units, freq_hz, nufft_eps, upsamp, precision)
    out = C.c_size_t(0)
    check(LIB.pc_plan_footprint(C.byref(g), C.byref(out)), "pc_plan_footprint")
    return int(out.value)


def pc_plan_create(uv, npix: int, fov_rad: float, *, w=None, uv_units=PC_UV_WAVELENGTHS,
                   freq_hz: float = 0.0, nufft_eps: float = 1e-5, upsamp: float = 2.0,
                   precision: int = PC_PREC_FP32, stream=None) -> Plan:
    g, keep = _geometry(uv, npix, fov_rad, w, uv_units, freq_hz, nufft_eps, upsamp, precision)
    h = C.c_void_p()
    check(LIB.pc_plan_create(C.byref(g), C.c_void_p(_stream(stream)), C.byref(h)),
          "pc_plan_create")
    return Plan(h, torch.device("cuda", torch.cuda.current_device()))


def _new(plan: Plan, shape, dtype):
    return torch.empty(shape, dtype=dtype, device=plan.device)


def pc_adjoint_grid(plan: Plan, vis: torch.Tensor, image: Optional[torch.Tensor] = None,
                    want_max: bool = True, stream=None):
    """Phi* vis -> (image [n, n] float32, max|image| or None, argmax or None)."""
    n = plan.npix
    if image is None:
        image = _new(plan, (n, n), torch.float32)
    mx, am = C.c_double(0), C.c_int64(-1)
    check(LIB.pc_adjoint_grid(plan.handle, C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")),
                              C.c_void_p(_dev(image, torch.float32, n * n, "image")),
                              C.byref(mx) if want_max else None, C.byref(am) if want_max else None,
                              C.c_void_p(_stream(stream))), "pc_adjoint_grid")
    return image, (mx.value if want_max else None), (am.value if want_max else None)


def pc_adjoint_grid_ms(plan: Plan, vis: torch.Tensor, sigma, gamma,
                       images: Optional[torch.Tensor] = None, want_max: bool = True, stream=None):
    """Psi* Phi* vis for the Gaussian synthesis dictionary (Sect. 4.3) ->
    (images [S, n, n] float32, max|.| or None, flat argmax s n^2 + p or None)."""
    n = plan.npix
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    gam = np.ascontiguousarray(gamma, dtype=np.float64)
    if sig.shape != gam.shape or sig.ndim != 1:
        raise ValueError("sigma and gamma must be 1-D of equal length")
    S = int(sig.size)
    if images is None:
        images = _new(plan, (S, n, n), torch.float32)
    mx, am = C.c_double(0), C.c_int64(-1)
    check(LIB.pc_adjoint_grid_ms(plan.handle,
                                 C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), S,
                                 sig.ctypes.data_as(C.POINTER(C.c_double)),
                                 gam.ctypes.data_as(C.POINTER(C.c_double)),
                                 C.c_void_p(_dev(images, torch.float32, S * n * n, "images")),
                                 C.byref(mx) if want_max else None,
                                 C.byref(am) if want_max else None,
                                 C.c_void_p(_stream(stream))), "pc_adjoint_grid_ms")
    return images, (mx.value if want_max else None), (am.value if want_max else None)


def pc_adjoint_grid_f64(plan: Plan, vis: torch.Tensor, image: Optional[torch.Tensor] = None,
                        want_max: bool = True, stream=None):
    n = plan.npix
    if image is None:
        image = _new(plan, (n, n), torch.float64)
    mx, am = C.c_double(0), C.c_int64(-1)
    check(LIB.pc_adjoint_grid_f64(plan.handle,
                                  C.c_void_p(_dev(vis, torch.complex128, plan.nvis, "vis")),
                                  C.c_void_p(_dev(image, torch.float64, n * n, "image")),
                                  C.byref(mx) if want_max else None,
                                  C.byref(am) if want_max else None,
                                  C.c_void_p(_stream(stream))), "pc_adjoint_grid_f64")
    return image, (mx.value if want_max else None), (am.value if want_max else None)


def pc_forward_sparse(plan: Plan, pix: torch.Tensor, weight: torch.Tensor,
                      out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    na = int(pix.numel())
    if out is None:
        out = _new(plan, (plan.nvis,), torch.complex64)
    check(LIB.pc_forward_sparse(plan.handle, na, C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                C.c_void_p(_dev(weight, torch.float32, na, "weight")),
                                C.c_void_p(_dev(out, torch.complex64, plan.nvis, "out")),
                                C.c_void_p(_stream(stream))), "pc_forward_sparse")
    return out


def pc_forward_sparse_f64(plan: Plan, pix: torch.Tensor, weight: torch.Tensor,
                          out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    na = int(pix.numel())
    if out is None:
        out = _new(plan, (plan.nvis,), torch.complex128)
    check(LIB.pc_forward_sparse_f64(plan.handle, na,
                                    C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                    C.c_void_p(_dev(weight, torch.float64, na, "weight")),
                                    C.c_void_p(_dev(out, torch.complex128, plan.nvis, "out")),
                                    C.c_void_p(_stream(stream))), "pc_forward_sparse_f64")
    return out


def row_mask(npix: int, rows) -> np.ndarray:
    """Host row mask (uint32 words, bit i % 32 of word i / 32 for row i) of
    the image rows ``rows``."""
    m = np.zeros((npix + 31) // 32, np.uint32)
    r = np.asarray(rows, dtype=np.int64).reshape(-1)
    if r.size and (r.min() < 0 or r.max() >= npix):
        raise ValueError("row index out of range")
    np.bitwise_or.at(m, r // 32, (np.uint32(1) << (r % 32).astype(np.uint32)))
    return m


def _mask(plan: Plan, mask) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    if m.shape != ((plan.npix + 31) // 32,):
        raise ValueError(f"row mask must hold {(plan.npix + 31) // 32} uint32 words")
    return m


def pc_forward_grid_rows(plan: Plan, image: torch.Tensor, mask, out: Optional[torch.Tensor] = None,
                         stream=None) -> torch.Tensor:
    """pc_forward_grid of an image that is zero outside the rows of ``mask``
    (see row_mask)."""
    n = plan.npix
    m = _mask(plan, mask)
    if out is None:
        out = _new(plan, (plan.nvis,), torch.complex64)
    check(LIB.pc_forward_grid_rows(plan.handle,
                                   C.c_void_p(_dev(image, torch.float32, n * n, "image")),
                                   m.ctypes.data_as(C.c_void_p),
                                   C.c_void_p(_dev(out, torch.complex64, plan.nvis, "out")),
                                   C.c_void_p(_stream(stream))), "pc_forward_grid_rows")
    return out


def pc_adjoint_grid_rows(plan: Plan, vis: torch.Tensor, mask, image: torch.Tensor,
                         stream=None) -> torch.Tensor:
    """The rows of Phi* vis that ``mask`` selects, written into ``image``
    (the other rows are left as they are)."""
    n = plan.npix
    m = _mask(plan, mask)
    check(LIB.pc_adjoint_grid_rows(plan.handle,
                                   C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")),
                                   m.ctypes.data_as(C.c_void_p),
                                   C.c_void_p(_dev(image, torch.float32, n * n, "image")),
                                   C.c_void_p(_stream(stream))), "pc_adjoint_grid_rows")
    return image


def pc_forward_grid(plan: Plan, image: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    n = plan.npix
    if out is None:
        out = _new(plan, (plan.nvis,), torch.complex64)
    check(LIB.pc_forward_grid(plan.handle, C.c_void_p(_dev(image, torch.float32, n * n, "image")),
                              C.c_void_p(_dev(out, torch.complex64, plan.nvis, "out")),
                              C.c_void_p(_stream(stream))), "pc_forward_grid")
    return out


def pc_adjoint_sparse(plan: Plan, vis: torch.Tensor, pix: torch.Tensor,
                      out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    na = int(pix.numel())
    if out is None:
        out = _new(plan, (na,), torch.float64)
    check(LIB.pc_adjoint_sparse(plan.handle,
                                C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), na,
                                C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                C.c_void_p(_dev(out, torch.float64, na, "out")),
                                C.c_void_p(_stream(stream))), "pc_adjoint_sparse")
    return out


def pc_restricted_gradient(plan: Plan, vis: torch.Tensor, pix: torch.Tensor, weight: torch.Tensor,
                           grad: Optional[torch.Tensor] = None, want_resid: bool = False,
                           stream=None):
    """Phi_S* (V - Phi_S x) on the active set (float64 [natoms]) and, on
    request, the residual V - Phi_S x (complex64 [nvis], caller order)."""
    na = int(pix.numel())
    if grad is None:
        grad = _new(plan, (na,), torch.float64)
    resid = _new(plan, (plan.nvis,), torch.complex64) if want_resid else None
    check(LIB.pc_restricted_gradient(
        plan.handle, C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), na,
        C.c_void_p(_dev(pix, torch.int32, na, "pix")),
        C.c_void_p(_dev(weight, torch.float32, na, "weight")),
        C.c_void_p(_dev(grad, torch.float64, na, "grad")),
        C.c_void_p(_dev(resid, torch.complex64, plan.nvis, "resid") if resid is not None else None),
        C.c_void_p(_stream(stream))), "pc_restricted_gradient")
    return (grad, resid) if want_resid else grad


def pc_restricted_gradient_grid(plan: Plan, vis: torch.Tensor, pix: torch.Tensor,
                                weight: torch.Tensor, grad: Optional[torch.Tensor] = None,
                                want_resid: bool = False, stream=None):
    """pc_restricted_gradient by the gridded operators (pass B at the set)."""
    na = int(pix.numel())
    if grad is None:
        grad = _new(plan, (na,), torch.float64)
    resid = _new(plan, (plan.nvis,), torch.complex64) if want_resid else None
    check(LIB.pc_restricted_gradient_grid(
        plan.handle, C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), na,
        C.c_void_p(_dev(pix, torch.int32, na, "pix")),
        C.c_void_p(_dev(weight, torch.float32, na, "weight")),
        C.c_void_p(_dev(grad, torch.float64, na, "grad")),
        C.c_void_p(_dev(resid, torch.complex64, plan.nvis, "resid") if resid is not None else None),
        C.c_void_p(_stream(stream))), "pc_restricted_gradient_grid")
    return (grad, resid) if want_resid else grad


def pc_restricted_gradient_noalloc(plan: Plan, vis: torch.Tensor, pix: torch.Tensor,
                                   weight: torch.Tensor, grad: torch.Tensor,
                                   resid: Optional[torch.Tensor] = None, stream=None):
    """pc_restricted_gradient without device allocation: grad (float64
    [natoms]) and resid (complex64 [nvis] or None) are caller-allocated; the
    library's scratch is a fixed per-device array."""
    na = int(pix.numel())
    check(LIB.pc_restricted_gradient_noalloc(
        plan.handle, C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), na,
        C.c_void_p(_dev(pix, torch.int32, na, "pix")),
        C.c_void_p(_dev(weight, torch.float32, na, "weight")),
        C.c_void_p(_dev(grad, torch.float64, na, "grad")),
        C.c_void_p(_dev(resid, torch.complex64, plan.nvis, "resid") if resid is not None else None),
        C.c_void_p(_stream(stream))), "pc_restricted_gradient_noalloc")
    return grad, resid


def pc_dual_certificate(plan: Plan, vis: torch.Tensor, pix: torch.Tensor, weight: torch.Tensor,
                        lam: float, cert: Optional[torch.Tensor] = None, want_max: bool = True,
                        stream=None):
    n, na = plan.npix, int(pix.numel())
    if cert is None:
        cert = _new(plan, (n, n), torch.float32)
    mx, am = C.c_double(0), C.c_int64(-1)
    check(LIB.pc_dual_certificate(plan.handle,
                                  C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")), na,
                                  C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                  C.c_void_p(_dev(weight, torch.float32, na, "weight")),
                                  float(lam), C.c_void_p(_dev(cert, torch.float32, n * n, "cert")),
                                  C.byref(mx) if want_max else None,
                                  C.byref(am) if want_max else None,
                                  C.c_void_p(_stream(stream))), "pc_dual_certificate")
    return cert, (mx.value if want_max else None), (am.value if want_max else None)


def pc_adjoint_sparse_f64(plan: Plan, vis: torch.Tensor, pix: torch.Tensor,
                          out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    na = int(pix.numel())
    if out is None:
        out = _new(plan, (na,), torch.float64)
    check(LIB.pc_adjoint_sparse_f64(plan.handle,
                                    C.c_void_p(_dev(vis, torch.complex128, plan.nvis, "vis")), na,
                                    C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                    C.c_void_p(_dev(out, torch.float64, na, "out")),
                                    C.c_void_p(_stream(stream))), "pc_adjoint_sparse_f64")
    return out


def pc_dual_certificate_f64(plan: Plan, vis: torch.Tensor, pix: torch.Tensor,
                            weight: torch.Tensor, lam: float, cert: Optional[torch.Tensor] = None,
                            want_max: bool = True, stream=None):
    n, na = plan.npix, int(pix.numel())
    if cert is None:
        cert = _new(plan, (n, n), torch.float64)
    mx, am = C.c_double(0), C.c_int64(-1)
    check(LIB.pc_dual_certificate_f64(plan.handle,
                                      C.c_void_p(_dev(vis, torch.complex128, plan.nvis, "vis")),
                                      na, C.c_void_p(_dev(pix, torch.int32, na, "pix")),
                                      C.c_void_p(_dev(weight, torch.float64, na, "weight")),
                                      float(lam),
                                      C.c_void_p(_dev(cert, torch.float64, n * n, "cert")),
                                      C.byref(mx) if want_max else None,
                                      C.byref(am) if want_max else None,
                                      C.c_void_p(_stream(stream))), "pc_dual_certificate_f64")
    return cert, (mx.value if want_max else None), (am.value if want_max else None)


def pc_adjoint_grid_batch(plans, vis, images=None, want_max: bool = True, stream=None):
    """Gridded adjoints of several FP32 plans in shared launches; returns
    (images, max_abs list, argmax list)."""
    n = len(plans)
    if len(vis) != n:
        raise ValueError("one visibility tensor per plan")
    if images is None:
        images = [_new(p, (p.npix, p.npix), torch.float32) for p in plans]
    P = (C.c_void_p * max(n, 1))()
    Vp = (C.c_void_p * max(n, 1))()
    Ip = (C.c_void_p * max(n, 1))()
    for j, (p, v, im) in enumerate(zip(plans, vis, images)):
        P[j] = p.handle.value if isinstance(p.handle, C.c_void_p) else p.handle
        Vp[j] = _dev(v, torch.complex64, p.nvis, "vis")
        Ip[j] = _dev(im, torch.float32, p.npix * p.npix, "image")
    mx = (C.c_double * max(n, 1))()
    am = (C.c_int64 * max(n, 1))()
    check(LIB.pc_adjoint_grid_batch(P, Vp, Ip, n, mx if want_max else None,
                                    am if want_max else None, C.c_void_p(_stream(stream))),
          "pc_adjoint_grid_batch")
    if not want_max:
        return images, None, None
    return images, [mx[j] for j in range(n)], [am[j] for j in range(n)]


def solve_params(**kw) -> PcSolveParams:
    """Defaults plus keyword fields; ``scales=(sigmas, gammas)`` sets the
    synthesis dictionary (n_scales, scale_sigma, scale_gamma) and
    ``x0=(atoms, weights)`` the warm start (the arrays are kept alive with the
    returned structure)."""
    p = PcSolveParams()
    LIB.pc_solve_params_default(C.byref(p))
    x0 = kw.pop("x0", None)
    if x0 is not None:
        pix = np.ascontiguousarray(x0[0], dtype=np.int32)
        w = np.ascontiguousarray(x0[1], dtype=np.float64)
        if pix.shape != w.shape or pix.ndim != 1:
            raise ValueError("x0: atoms and weights must be 1-D of equal length")
        p._x0_keep = (pix, w)
        p.x0_pix = pix.ctypes.data_as(C.POINTER(C.c_int32))
        p.x0_w = w.ctypes.data_as(C.POINTER(C.c_double))
        p.x0_n = int(pix.size)
    scales = kw.pop("scales", None)
    if scales is not None:
        sig, gam = (list(map(float, a)) for a in scales)
        if len(sig) != len(gam) or not 1 <= len(sig) <= 8:
            raise ValueError("scales: 1 to 8 (sigma, gamma) pairs")
        p.n_scales = len(sig)
        for i, (a, b) in enumerate(zip(sig, gam)):
            p.scale_sigma[i] = a
            p.scale_gamma[i] = b
    for k, v in kw.items():
        key = "lambda_" if k in ("lam", "lambda") else k
        if not hasattr(p, key):
            raise KeyError(k)
        setattr(p, key, v)
    return p


def pc_polyclean_solve(plan: Plan, vis: torch.Tensor, params: Optional[PcSolveParams] = None,
                       capacity: int = 65536, cert: Optional[torch.Tensor] = None, stream=None,
                       **kw):
    """Run Alg. 2; returns a dict with the atoms, weights and scalars."""
    if params is None:
        params = solve_params(**kw)
    elif kw:
        raise ValueError("pass either params or keyword parameters")
    n = plan.npix
    pix = np.zeros(capacity, dtype=np.int32)
    wgt = np.zeros(capacity, dtype=np.float64)
    res = PcSolveResult()
    res.capacity = capacity
    res.pix = pix.ctypes.data_as(C.POINTER(C.c_int32))
    res.weight = wgt.ctypes.data_as(C.POINTER(C.c_double))
    ncert = n * n * max(1, params.n_scales)  # Psi* eta / lambda with a dictionary
    res.cert = C.c_void_p(_dev(cert, torch.float32, ncert, "cert")) if cert is not None else None
    st = LIB.pc_polyclean_solve(plan.handle, C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis")),
                                C.byref(params), C.byref(res), C.c_void_p(_stream(stream)))
    check(st, "pc_polyclean_solve")
    return _result_dict(res, st, pix, wgt)


def _result_dict(res: PcSolveResult, status: int, pix: np.ndarray, wgt: np.ndarray) -> dict:
    out = {k: getattr(res, k) for k, _ in PcSolveResult._fields_
           if k not in ("pix", "weight", "cert", "capacity")}
    out["lambda"] = out.pop("lambda_")
    out["status"] = status
    na = int(res.natoms)
    out["pix"] = pix[:na].astype(np.int64)
    out["weight"] = wgt[:na].copy()
    return out


class Batcher:
    """Owns a pc_batcher handle: merges the gridded adjoints of solvers on
    different threads into shared launches."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(LIB.pc_batcher_create(int(device), C.byref(h)), "pc_batcher_create")
        self._h = h
        self.device = int(device)

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        st = PcBatcherStats()
        check(LIB.pc_batcher_get_stats(self._h, C.byref(st)), "pc_batcher_get_stats")
        return {k: getattr(st, k) for k, _ in PcBatcherStats._fields_ if k != "pad"}

    def close(self):
        if self._h:
            LIB.pc_batcher_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Step-wise solve (pc_solver_create[_batched] / step / result / destroy).
    The solver reads `vis` only during construction."""

    def __init__(self, plan: Plan, vis: torch.Tensor, params: Optional[PcSolveParams] = None,
                 stream=None, batcher: Optional[Batcher] = None, **kw):
        if params is None:
            params = solve_params(**kw)
        elif kw:
            raise ValueError("pass either params or keyword parameters")
        self.plan = plan
        self.n_scales = params.n_scales
        h = C.c_void_p()
        dv = C.c_void_p(_dev(vis, torch.complex64, plan.nvis, "vis"))
        if batcher is None:
            st = LIB.pc_solver_create(plan.handle, dv, C.byref(params), C.c_void_p(_stream(stream)),
                                      C.byref(h))
            check(st, "pc_solver_create")
        else:
            st = LIB.pc_solver_create_batched(plan.handle, dv, C.byref(params),
                                              C.c_void_p(_stream(stream)), batcher.handle,
                                              C.byref(h))
            check(st, "pc_solver_create_batched")
        self._h = h
        self.done = False

    def step(self) -> bool:
        done = C.c_int32(0)
        check(LIB.pc_solver_step(self._h, C.byref(done)), "pc_solver_step")
        self.done = bool(done.value)
        return self.done

    def result(self, capacity: int = 65536, cert: Optional[torch.Tensor] = None) -> dict:
        """Current iterate; `cert` (device float [n, n], [S, n, n] with a
        dictionary) receives the dual certificate when the solver was created
        with want_certificate=1."""
        pix = np.zeros(capacity, dtype=np.int32)
        wgt = np.zeros(capacity, dtype=np.float64)
        res = PcSolveResult()
        res.capacity = capacity
        res.pix = pix.ctypes.data_as(C.POINTER(C.c_int32))
        res.weight = wgt.ctypes.data_as(C.POINTER(C.c_double))
        n = self.plan.npix
        ncert = n * n * max(1, self.n_scales)
        res.cert = C.c_void_p(_dev(cert, torch.float32, ncert, "cert")) if cert is not None else None
        st = LIB.pc_solver_result(self._h, C.byref(res))
        check(st, "pc_solver_result")
        return _result_dict(res, st, pix, wgt)

    def close(self):
        if self._h:
            LIB.pc_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pc_plan_profile(plan: Plan, enable: bool = True) -> None:
    """Enable (and reset) or disable per-kernel event timing on the plan."""
    check(LIB.pc_plan_profile(plan.handle, 1 if enable else 0), "pc_plan_profile")


def pc_plan_kernel_stats(plan: Plan):
    """Per-kernel sums since profiling was enabled: list of dicts with name,
    launches, ms, bytes (algorithmic) and work units."""
    out = []
    for i in range(LIB.pc_plan_kernel_stat_count(plan.handle)):
        st = PcKernelStat()
        check(LIB.pc_plan_kernel_stat(plan.handle, i, C.byref(st)), "pc_plan_kernel_stat")
        out.append({"name": st.name.decode(), "launches": int(st.launches), "ms": float(st.ms),
                    "bytes": float(st.bytes), "work": float(st.work)})
    return out

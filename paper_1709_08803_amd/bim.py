"""Thin ctypes binding of libbim.so (argument marshalling only).

Every computation happens in the HIP library; this module only turns torch
device tensors and problem descriptions into the plain pointers and structs of
include/bim.h.  Importing it does not load the library; the first call does,
and fails loudly if libbim.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbim.so")

FP64 = 0
FP32C = 1
_PREC = {"fp64": FP64, "fp32c": FP32C, FP64: FP64, FP32C: FP32C}

_lib = None


class BimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libbim error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("x1", ctypes.c_double), ("dx", ctypes.c_double),
                ("y1", ctypes.c_double), ("dy", ctypes.c_double),
                ("half_domain", ctypes.c_int32), ("n_decay", ctypes.c_double),
                ("froude", ctypes.c_double),
                ("beta", ctypes.c_void_p), ("beta_x", ctypes.c_void_p), ("beta_y", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        pp = ctypes.POINTER(_Problem)
        L.bim_residual.argtypes = [pp, vp, vp, i32, vp]
        L.bim_jv.argtypes = [pp, vp, vp, vp, dbl, vp, i32, vp]
        for name in ("bim_residual", "bim_jv"):
            getattr(L, name).restype = i32
        L.bim_last_error.restype = ctypes.c_char_p
        L.bim_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise BimError(rc, lib().bim_last_error().decode())
    return rc


def _stream(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dptr(t: torch.Tensor) -> int:
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return t.data_ptr()


class DeviceProblem:
    """A problem whose bottom arrays live on the GPU (keeps the tensors alive)."""

    def __init__(self, p, device="cuda"):
        self.host = p
        self.device = torch.device(device)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
        self.beta, self.beta_x, self.beta_y = t(p.beta), t(p.beta_x), t(p.beta_y)
        self.struct = _Problem(p.N, p.M, p.x1, p.dx, p.y1, p.dy, 1 if p.half_domain else 0,
                               p.n_decay, p.froude, self.beta.data_ptr(), self.beta_x.data_ptr(),
                               self.beta_y.data_ptr())

    @property
    def n(self) -> int:
        return 3 * (self.host.N + 1) * self.host.M

    def ref(self):
        return ctypes.byref(self.struct)


def residual(dp: DeviceProblem, u: torch.Tensor, prec="fp64", out: Optional[torch.Tensor] = None,
             stream=None) -> torch.Tensor:
    F = out if out is not None else torch.empty_like(u)
    _check(lib().bim_residual(dp.ref(), _dptr(u), _dptr(F), _PREC[prec], _stream(stream)))
    return F


def jv(dp: DeviceProblem, u: torch.Tensor, Fu: torch.Tensor, v: torch.Tensor, h: float = 0.0,
       prec="fp64", out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    J = out if out is not None else torch.empty_like(u)
    _check(lib().bim_jv(dp.ref(), _dptr(u), _dptr(Fu), _dptr(v), float(h), _dptr(J), _PREC[prec],
                        _stream(stream)))
    return J


def version() -> str:
    return lib().bim_version().decode()

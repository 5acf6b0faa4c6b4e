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
STORE_FP64, STORE_FP32 = 0, 1
_STORE = {"fp64": STORE_FP64, "fp32": STORE_FP32, STORE_FP64: STORE_FP64, STORE_FP32: STORE_FP32}

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
                ("beta", ctypes.c_void_p), ("beta_x", ctypes.c_void_p), ("beta_y", ctypes.c_void_p),
                ("tau", ctypes.c_double)]


class Bump(ctypes.Structure):
    """bim_bump: eps exp(-((x - b1)^2 + (y - b2)^2) / (2 delta^2)), eq. (bottom)."""
    _fields_ = [("eps", ctypes.c_double), ("delta", ctypes.c_double), ("b1", ctypes.c_double),
                ("b2", ctypes.c_double)]


class ExactConfig(ctypes.Structure):
    _fields_ = [("periods_per_panel", ctypes.c_double), ("decay", ctypes.c_double),
                ("psi_width_max", ctypes.c_double), ("grade_start", ctypes.c_double),
                ("workgroups", ctypes.c_int32), ("timing", ctypes.c_int32), ("tile_cols", ctypes.c_int32)]


class ExactInfo(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("psi_nodes", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("kcut", ctypes.c_double), ("hk", ctypes.c_double),
                ("contract_ms", ctypes.c_double), ("total_ms", ctypes.c_double), ("tile_cols", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        pp = ctypes.POINTER(_Problem)
        L.bim_residual.argtypes = [pp, vp, vp, i32, vp]
        L.bim_residual_linear.argtypes = [pp, vp, vp, i32, vp]
        L.bim_residual_noalloc.argtypes = [pp, vp, vp, i32, vp]
        L.bim_bottom_pressure.argtypes = [pp, vp, vp, vp, vp]
        L.bim_exact_linear.argtypes = [dbl, ctypes.POINTER(Bump), i32, i32, i32, dbl, dbl, dbl, dbl, vp, vp,
                                       ctypes.POINTER(ExactConfig), ctypes.POINTER(ExactInfo), vp]
        L.bim_exact_start.argtypes = [pp, vp, vp, vp, vp]
        L.bim_residual_noalloc_max_bytes.argtypes = []
        L.bim_residual_noalloc_max_bytes.restype = ctypes.c_size_t
        L.bim_jv.argtypes = [pp, vp, vp, vp, dbl, vp, i32, vp]
        L.bim_release_workspaces.argtypes = []
        L.bim_residual_timed.argtypes = [pp, vp, vp, i32, i32, ctypes.POINTER(PairConfig), vp,
                                         ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.bim_tune_residual.argtypes = [pp, vp, i32, vp, ctypes.POINTER(PairConfig), ctypes.POINTER(dbl)]
        L.precond_setup.argtypes = [pp, i32, ctypes.POINTER(vp), vp]
        L.precond_setup_ex.argtypes = [pp, i32, i32, ctypes.POINTER(vp), vp]
        L.precond_storage.argtypes = [vp]
        L.precond_apply.argtypes = [vp, vp, vp, vp]
        L.precond_destroy.argtypes = [vp]
        L.precond_destroy.restype = None
        L.precond_bytes.argtypes = [vp]
        L.precond_bytes.restype = ctypes.c_int64
        L.precond_band.argtypes = [vp]
        L.bim_residual_batched.argtypes = [pp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
        L.bim_residual_batched.restype = i32
        L.jfnk_default_opts.argtypes = [ctypes.POINTER(JfnkOpts)]
        L.jfnk_default_opts.restype = None
        L.jfnk_solve.argtypes = [pp, vp, vp, ctypes.POINTER(JfnkOpts), ctypes.POINTER(JfnkReport), vp]
        L.bim_linear_start.argtypes = [pp, vp, vp, dbl, vp]
        L.bim_linear_start_ex.argtypes = [pp, vp, vp, dbl, i32, vp]
        L.jfnk_solve_batched.argtypes = [pp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(JfnkOpts),
                                         ctypes.POINTER(JfnkReport), vp]
        L.jfnk_solve_batched.restype = i32
        fp = ctypes.POINTER(ctypes.c_float)
        L.lg_default_arch.argtypes = [ctypes.POINTER(LgArch), i32, i32]
        L.lg_default_arch.restype = None
        L.lg_create.argtypes = [ctypes.POINTER(LgArch), ctypes.c_uint64, i32, ctypes.POINTER(vp)]
        L.lg_destroy.argtypes = [vp]
        L.lg_destroy.restype = None
        L.lg_num_params.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.lg_set_params.argtypes = [vp, i32, fp, fp]
        L.lg_get_params.argtypes = [vp, i32, fp, fp, fp, fp]
        L.lg_forward.argtypes = [vp, vp, vp, i32, vp, vp]
        L.lg_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, i32, fp, vp]
        L.lg_make_input.argtypes = [pp, vp, i32, vp, vp, vp]
        L.lg_infer_start.argtypes = [vp, pp, vp, vp, vp]
        for name in ("bim_residual", "bim_residual_linear", "bim_residual_noalloc", "bim_bottom_pressure", "bim_jv", "bim_residual_timed", "bim_tune_residual", "precond_setup",
                     "precond_setup_ex", "precond_storage", "precond_apply", "precond_band", "jfnk_solve",
                     "bim_linear_start", "bim_linear_start_ex", "lg_create",
                     "lg_num_params", "lg_set_params", "lg_get_params", "lg_forward", "lg_train_step",
                     "lg_make_input", "lg_infer_start"):
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


class PairConfig(ctypes.Structure):
    _fields_ = [("targets_per_lane", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("rows_per_chunk", ctypes.c_int32), ("chunks", ctypes.c_int32)]

    def as_tuple(self):
        return (self.targets_per_lane, self.unroll, self.rows_per_chunk, self.chunks)


class JfnkOpts(ctypes.Structure):
    _fields_ = [("ftol", ctypes.c_double), ("gmres_rtol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("max_backtracks", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("band_halfwidth", ctypes.c_int32), ("use_precond", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("fd_eps", ctypes.c_double), ("stall_steps", ctypes.c_int32),
                ("fp64_below", ctypes.c_double), ("fp32c_gmres_rtol", ctypes.c_double),
                ("precond_storage", ctypes.c_int32)]


class JfnkReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("newton_iters", ctypes.c_int32), ("gmres_iters", ctypes.c_int32),
                ("residual_evals", ctypes.c_int32), ("inner_residual_evals", ctypes.c_int32),
                ("jv_evals", ctypes.c_int32), ("backtracks", ctypes.c_int32), ("fnorm_inf", ctypes.c_double),
                ("fnorm0_inf", ctypes.c_double), ("gmres_relres_last", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("precond_ms", ctypes.c_double), ("history", ctypes.c_double * 64),
                ("max_zeta", ctypes.c_double), ("min_depth", ctypes.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "history"}
        d["history"] = [self.history[i] for i in range(min(64, self.newton_iters + 1))]
        return d


class LgArch(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("C1", ctypes.c_int32), ("C2", ctypes.c_int32),
                ("D3", ctypes.c_int32), ("in_linear", ctypes.c_int32), ("out_scale", ctypes.c_double)]


class DeviceProblem:
    """A problem whose bottom arrays live on the GPU (keeps the tensors alive)."""

    def __init__(self, p, device="cuda"):
        self.host = p
        self.device = torch.device(device)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
        self.beta, self.beta_x, self.beta_y = t(p.beta), t(p.beta_x), t(p.beta_y)
        self.struct = _Problem(p.N, p.M, p.x1, p.dx, p.y1, p.dy, 1 if p.half_domain else 0,
                               p.n_decay, p.froude, self.beta.data_ptr(), self.beta_x.data_ptr(),
                               self.beta_y.data_ptr(), float(getattr(p, "tau", 0.0)))

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


def residual_linear(dp: DeviceProblem, u: torch.Tensor, prec="fp64", out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """bim_residual_linear: the linearised residual F_lin(u)."""
    F = out if out is not None else torch.empty_like(u)
    _check(lib().bim_residual_linear(dp.ref(), _dptr(u), _dptr(F), _PREC[prec], _stream(stream)))
    return F


def residual_noalloc(dp: DeviceProblem, u: torch.Tensor, F: torch.Tensor, prec="fp64", stream=None) -> torch.Tensor:
    """bim_residual_noalloc: F(u) into the caller's F with the library's fixed device scratch."""
    _check(lib().bim_residual_noalloc(dp.ref(), _dptr(u), _dptr(F), _PREC[prec], _stream(stream)))
    return F


def bottom_pressure(dp: DeviceProblem, u: torch.Tensor, stream=None):
    """bim_bottom_pressure: (pressure at the bottom nodes [M][N], force (Fx, Fy, Fz)) as device tensors."""
    h = dp.host
    pres = torch.empty((h.M, h.N), dtype=torch.float64, device=u.device)
    force = torch.empty(3, dtype=torch.float64, device=u.device)
    _check(lib().bim_bottom_pressure(dp.ref(), _dptr(u), pres.data_ptr(), force.data_ptr(), _stream(stream)))
    return pres, force


def exact_linear(froude: float, bumps, N: int, M: int, x1: float, dx: float, y1: float, dy: float,
                 derivative: bool = True, config: Optional[dict] = None, device="cuda", stream=None):
    """bim_exact_linear: (zeta [M][N], zeta_x [M][N] or None, info dict) of eq. (exactsoln) for
    bumps = [(eps, delta, b1, b2), ...] on the mesh x1 + i dx, y1 + j dy."""
    arr = (Bump * len(bumps))(*[Bump(*map(float, b)) for b in bumps])
    zeta = torch.empty((M, N), dtype=torch.float64, device=device)
    zx = torch.empty((M, N), dtype=torch.float64, device=device) if derivative else None
    cfg = ExactConfig(**(config or {}))
    info = ExactInfo()
    _check(lib().bim_exact_linear(float(froude), arr, len(bumps), int(N), int(M), float(x1), float(dx), float(y1),
                                  float(dy), zeta.data_ptr(), zx.data_ptr() if zx is not None else None,
                                  ctypes.byref(cfg), ctypes.byref(info), _stream(stream)))
    return zeta, zx, {f: getattr(info, f) for f, _ in ExactInfo._fields_}


def exact_start(dp: DeviceProblem, zeta: torch.Tensor, zeta_x: torch.Tensor, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """bim_exact_start: an unknown vector from the exact linear solution on dp's mesh."""
    h = dp.host
    if tuple(zeta.shape) != (h.M, h.N) or tuple(zeta_x.shape) != (h.M, h.N):
        raise ValueError("zeta and zeta_x must be [M][N] on the problem's mesh")
    u = out if out is not None else torch.empty(dp.n, dtype=torch.float64, device=dp.device)
    _check(lib().bim_exact_start(dp.ref(), _dptr(zeta), _dptr(zeta_x), _dptr(u),
                                 _stream(stream)))
    return u


def residual_noalloc_max_bytes() -> int:
    return int(lib().bim_residual_noalloc_max_bytes())


def residual_batched(dps, us, prec="fp64", outs=None, stream=None):
    """F_i = F(u_i) for a list of problems in one persistent all-pairs launch."""
    n = len(dps)
    outs = outs if outs is not None else [torch.empty_like(u) for u in us]
    arr = (_Problem * n)(*[d.struct for d in dps])
    up = (ctypes.c_void_p * n)(*[_dptr(u) for u in us])
    fp = (ctypes.c_void_p * n)(*[_dptr(f) for f in outs])
    _check(lib().bim_residual_batched(arr, n, up, fp, _PREC[prec], _stream(stream)))
    return outs


def jv(dp: DeviceProblem, u: torch.Tensor, Fu: torch.Tensor, v: torch.Tensor, h: float = 0.0,
       prec="fp64", out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    J = out if out is not None else torch.empty_like(u)
    _check(lib().bim_jv(dp.ref(), _dptr(u), _dptr(Fu), _dptr(v), float(h), _dptr(J), _PREC[prec],
                        _stream(stream)))
    return J


def release_workspaces() -> None:
    """Frees the per-stream workspaces kept by residual() and jv()."""
    _check(lib().bim_release_workspaces())


def residual_timed(dp: DeviceProblem, u: torch.Tensor, prec="fp64", iters: int = 10, config=None,
                   stream=None):
    """(all-pairs kernel ms, whole evaluation ms), averaged over `iters` evaluations (HIP events).

    config: (targets_per_lane, unroll, rows_per_chunk[, chunks]) or None for the current choice.
    """
    F = torch.empty_like(u)
    k, t = ctypes.c_double(), ctypes.c_double()
    cfg = ctypes.byref(PairConfig(*config)) if config is not None else None
    _check(lib().bim_residual_timed(dp.ref(), _dptr(u), _dptr(F), _PREC[prec], int(iters), cfg,
                                    _stream(stream), ctypes.byref(k), ctypes.byref(t)))
    return k.value, t.value


def tune_residual(dp: DeviceProblem, u: torch.Tensor, prec="fp64", stream=None):
    """Run the in-library autotuner; returns ((tpl, unroll, rows_per_chunk, chunks), kernel ms)."""
    best, ms = PairConfig(), ctypes.c_double()
    _check(lib().bim_tune_residual(dp.ref(), _dptr(u), _PREC[prec], _stream(stream), ctypes.byref(best),
                                   ctypes.byref(ms)))
    return best.as_tuple(), ms.value


class Preconditioner:
    """Library-owned block-banded preconditioner P (freed with close() or on deletion)."""

    def __init__(self, dp: DeviceProblem, band_halfwidth: int = -1, stream=None, storage="fp64"):
        """storage: "fp64", or "fp32" (operator rounded to FP32 after the FP64
        factorisation; products and sums of the apply stay FP64)."""
        self._h = ctypes.c_void_p()
        self.dp = dp
        _check(lib().precond_setup_ex(dp.ref(), int(band_halfwidth), _STORE[storage], ctypes.byref(self._h),
                                      _stream(stream)))

    @property
    def storage(self) -> str:
        return {STORE_FP64: "fp64", STORE_FP32: "fp32"}[lib().precond_storage(self._h)]

    @property
    def handle(self):
        return self._h

    @property
    def band(self) -> int:
        return lib().precond_band(self._h)

    @property
    def nbytes(self) -> int:
        return lib().precond_bytes(self._h)

    def apply(self, r: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        z = out if out is not None else torch.empty_like(r)
        _check(lib().precond_apply(self._h, _dptr(r), _dptr(z), _stream(stream)))
        return z

    def close(self):
        if self._h:
            lib().precond_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_opts(**kw) -> JfnkOpts:
    o = JfnkOpts()
    lib().jfnk_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "inner_prec":
            v = _PREC[v]
        if k == "precond_storage":
            v = _STORE.get(v, v)  # names, or the library's integer values (which it validates)
        setattr(o, k, v)
    return o


def solve(dp: DeviceProblem, u: torch.Tensor, P: Optional[Preconditioner] = None, stream=None,
          check: bool = True, **opts) -> dict:
    """jfnk_solve in place on u; returns the report as a dict (status included)."""
    o = default_opts(**opts)
    rep = JfnkReport()
    rc = lib().jfnk_solve(dp.ref(), P.handle if P is not None else None, _dptr(u), ctypes.byref(o),
                          ctypes.byref(rep), _stream(stream))
    if rc < 0 and check:
        _check(rc)
    d = rep.as_dict()
    d["status"] = rc
    return d


def solve_batched(dps, us, Ps=None, stream=None, check: bool = True, **opts):
    """jfnk_solve_batched in place on every u; returns (status, [report dicts])."""
    n = len(dps)
    o = default_opts(**opts)
    arr = (_Problem * n)(*[d.struct for d in dps])
    up = (ctypes.c_void_p * n)(*[_dptr(u) for u in us])
    pp = (ctypes.c_void_p * n)(*[(P.handle.value if P is not None else None) for P in Ps]) if Ps else None
    reps = (JfnkReport * n)()
    rc = lib().jfnk_solve_batched(arr, n, pp, up, ctypes.byref(o), reps, _stream(stream))
    if rc < 0 and check:
        _check(rc)
    return rc, [r.as_dict() for r in reps]


def linear_start(dp: DeviceProblem, P: Optional[Preconditioner] = None, rtol: float = 0.0,
                 out: Optional[torch.Tensor] = None, stream=None, prec="fp64") -> torch.Tensor:
    """bim_linear_start_ex: prec "fp32c" forms the linear operator's products with FP32C sums."""
    u = out if out is not None else torch.empty(dp.n, dtype=torch.float64, device=dp.device)
    rc = lib().bim_linear_start_ex(dp.ref(), P.handle if P is not None else None, _dptr(u), float(rtol),
                                   _PREC[prec], _stream(stream))
    _check(rc)
    return u


class LearnedNet:
    """The learned-start network (library-owned; bf16 kernels with FP32 accumulation)."""

    def __init__(self, N: int, M: int, seed: int = 0, max_batch: int = 64, **arch):
        a = LgArch()
        lib().lg_default_arch(ctypes.byref(a), int(N), int(M))
        for k, v in arch.items():
            setattr(a, k, v)
        self.arch = a
        self.max_batch = max_batch
        self._h = ctypes.c_void_p()
        _check(lib().lg_create(ctypes.byref(a), ctypes.c_uint64(seed), int(max_batch), ctypes.byref(self._h)))

    @property
    def n_out(self) -> int:
        return 2 * self.arch.H * self.arch.W

    def shapes(self, layer: int):
        w, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lg_num_params(self._h, layer, ctypes.byref(w), ctypes.byref(b)))
        return w.value, b.value

    def get(self, layer: int):
        """(W, b, gW, gb) as float32 numpy arrays (W flattened [fan_in * fan_out])."""
        nw, nb = self.shapes(layer)
        arrs = [np.empty(nw, np.float32), np.empty(nb, np.float32), np.empty(nw, np.float32), np.empty(nb, np.float32)]
        fptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        _check(lib().lg_get_params(self._h, layer, *[fptr(a) for a in arrs]))
        return arrs

    def set(self, layer: int, W=None, b=None):
        fptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a is not None else None
        W = np.ascontiguousarray(W, dtype=np.float32) if W is not None else None
        b = np.ascontiguousarray(b, dtype=np.float32) if b is not None else None
        _check(lib().lg_set_params(self._h, layer, fptr(W), fptr(b)))

    def forward(self, X0: torch.Tensor, ffeat: torch.Tensor, stream=None) -> torch.Tensor:
        B = ffeat.shape[0]
        Y = torch.empty((B, self.n_out), dtype=torch.float32, device=ffeat.device)
        _check(lib().lg_forward(self._h, X0.data_ptr(), ffeat.data_ptr(), B, Y.data_ptr(), _stream(stream)))
        return Y

    def train_step(self, X0: torch.Tensor, ffeat: torch.Tensor, T: torch.Tensor, lr: float, update: bool = True,
                   stream=None) -> float:
        loss = ctypes.c_float()
        _check(lib().lg_train_step(self._h, X0.data_ptr(), ffeat.data_ptr(), T.data_ptr(), ffeat.shape[0],
                                   ctypes.c_float(lr), 1 if update else 0, ctypes.byref(loss), _stream(stream)))
        return loss.value

    @property
    def in_channels(self) -> int:
        return 4 if self.arch.in_linear else 2

    def make_input(self, dp: DeviceProblem, u_lin: Optional[torch.Tensor] = None, stream=None):
        """Network input of one problem; u_lin (the linear start) is needed when the net reads it."""
        X0 = torch.empty((dp.host.M, dp.host.N, self.in_channels), dtype=torch.int16, device=dp.device)
        f = torch.empty(1, dtype=torch.float32, device=dp.device)
        _check(lib().lg_make_input(dp.ref(), _dptr(u_lin) if u_lin is not None else None, int(self.arch.in_linear),
                                   X0.data_ptr(), f.data_ptr(), _stream(stream)))
        return X0, f

    def infer_start(self, dp: DeviceProblem, P: Optional[Preconditioner] = None, out=None, stream=None):
        u = out if out is not None else torch.empty(dp.n, dtype=torch.float64, device=dp.device)
        _check(lib().lg_infer_start(self._h, dp.ref(), P.handle if P is not None else None, _dptr(u),
                                    _stream(stream)))
        return u

    def close(self):
        if self._h:
            lib().lg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return lib().bim_version().decode()

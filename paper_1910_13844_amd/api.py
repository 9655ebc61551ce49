"""Python binding of libls with the same names as the C ABI.

PyTorch supplies device memory and HIP streams; every step of the computation runs in the HIP
kernels behind include/ls.h.  Volumes are [Q, n, n, n] (z, y, x), detector fields [Q, n, n].
"""
from __future__ import annotations

import ctypes as C
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """Green kernels of one geometry, resident on the device (ls_green_init).

    The context itself is immutable and may be used from several threads and streams at once.
    Calls that are not given a workspace (`ws=None`) share one cached workspace per operation, so
    concurrent calls (other threads or streams) must each pass a workspace of their own.
    """

    def __init__(self, n: int, kbh: float, p: int = 4, xg: Optional[float] = None, prec: str = "c64",
                 device: str = "cuda:0", stream=None):
        self.lib = L.load()
        self.n, self.p, self.kbh = int(n), int(p), float(kbh)
        self.xg = float(n) if xg is None else float(xg)
        self.prec = prec
        self.device = torch.device(device)
        self.cdtype = torch.complex64 if prec == "c64" else torch.complex128
        self.rdtype = torch.float32 if prec == "c64" else torch.float64
        self.geom = L.Geom(self.n, self.p, self.kbh, self.xg, L.LS_C64 if prec == "c64" else L.LS_C128, 0)
        kb, wb = C.c_size_t(), C.c_size_t()
        L.check(self.lib.ls_kernel_bytes(C.byref(self.geom), C.byref(kb)), "ls_kernel_bytes")
        L.check(self.lib.ls_init_workspace_bytes(C.byref(self.geom), C.byref(wb)), "ls_init_workspace_bytes")
        self.kbuf = torch.empty(kb.value, dtype=torch.uint8, device=self.device)
        ws = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        L.check(self.lib.ls_green_init(C.byref(self.geom), _ptr(self.kbuf), kb.value, _ptr(ws), wb.value,
                                       _stream(stream), C.byref(h)), "ls_green_init")
        del ws
        self.h = h
        self._ws = {}

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                self.lib.ls_ctx_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def N(self) -> int:
        return self.n ** 3

    # -- workspaces ------------------------------------------------------------------------
    def workspace_bytes(self, Q: int, op: int) -> int:
        b = C.c_size_t()
        L.check(self.lib.ls_workspace_bytes(self.h, int(Q), int(op), C.byref(b)), "ls_workspace_bytes")
        return b.value

    def workspace(self, Q: int, op: int, max_bytes: Optional[int] = None) -> torch.Tensor:
        need = self.workspace_bytes(Q, op)
        if max_bytes is not None:
            need = min(need, max_bytes)
        key = (op,)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            self._ws.pop(key, None)
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def _chk_vol(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if t.device != self.device or t.dtype != self.cdtype or not t.is_contiguous() or t.shape[-3:] != (self.n,) * 3:
            raise ValueError(f"{name}: expected contiguous {self.cdtype} [..., {self.n}, {self.n}, {self.n}] on {self.device}")
        return t

    def _chk_f(self, f: torch.Tensor) -> torch.Tensor:
        if f.device != self.device or f.dtype != self.rdtype or not f.is_contiguous() or tuple(f.shape) != (self.n,) * 3:
            raise ValueError(f"f: expected contiguous {self.rdtype} [{self.n}]^3 on {self.device}")
        return f

    def _chk_like(self, t: torch.Tensor, shape, dtype, name: str) -> torch.Tensor:
        """Device, dtype, contiguity and exact shape of a caller tensor (the library only sees pointers)."""
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected contiguous {dtype} {list(shape)} on {self.device}, got "
                             f"{t.dtype} {list(t.shape)} on {t.device}")
        return t

    def _chk_det_q(self, y: torch.Tensor, Q: int, name: str) -> torch.Tensor:
        return self._chk_like(y.contiguous(), (Q, self.n, self.n), self.cdtype, name)

    @staticmethod
    def _opts(tol: float, maxit: int, max_restarts: int, x0_mode: int = 0, breakdown: float = 0.0) -> L.SolveOpts:
        return L.SolveOpts(float(tol), int(maxit), int(max_restarts), int(x0_mode), 0, float(breakdown))

    # -- operators -------------------------------------------------------------------------
    def ls_apply_G(self, v: torch.Tensor, stream=None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        v = self._chk_vol(v, "v")
        Q = v.numel() // self.N
        out = torch.empty_like(v)
        ws = self.workspace(Q, L.LS_OP_APPLY) if ws is None else ws
        L.check(self.lib.ls_apply_G(self.h, _ptr(v), _ptr(out), Q, _ptr(ws), ws.numel(), _stream(stream)), "ls_apply_G")
        return out

    def ls_apply_A(self, f: torch.Tensor, v: torch.Tensor, stream=None) -> torch.Tensor:
        v = self._chk_vol(v, "v")
        f = self._chk_f(f)
        Q = v.numel() // self.N
        out = torch.empty_like(v)
        ws = self.workspace(Q, L.LS_OP_APPLY)
        L.check(self.lib.ls_apply_A(self.h, _ptr(f), _ptr(v), _ptr(out), Q, _ptr(ws), ws.numel(), _stream(stream)),
                "ls_apply_A")
        return out

    def ls_forward(self, f: torch.Tensor, dirs, tol: float = 1e-5, maxit: int = 500, max_restarts: int = 3,
                   u: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None,
                   warm_start: bool = False, breakdown: float = 0.0) -> Tuple[torch.Tensor, List[dict]]:
        """Forward solves for plane waves `dirs`.  warm_start: start BiCGSTAB from the contents of
        `u` (which must then be given) instead of from the incident field.  breakdown: threshold of
        the restart test (0: the unit roundoff of the field precision)."""
        f = self._chk_f(f)
        if warm_start and u is None:
            raise ValueError("warm_start needs u (the initial guesses)")
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        Q = d.shape[0]
        if u is None:
            u = torch.empty((Q, self.n, self.n, self.n), dtype=self.cdtype, device=self.device)
        self._chk_like(u, (Q, self.n, self.n, self.n), self.cdtype, "u")
        ws = self.workspace(Q, L.LS_OP_FORWARD) if ws is None else ws
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts, 1 if warm_start else 0, breakdown)
        L.check(self.lib.ls_forward(self.h, _ptr(f), Q, d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(u),
                                    C.byref(o), info, _ptr(ws), ws.numel(), _stream(stream)), "ls_forward")
        return u, [i.as_dict() for i in info]

    def ls_forward_farfield(self, f: torch.Tensor, dirs, tol: float = 1e-5, maxit: int = 500, max_restarts: int = 3,
                            u: Optional[torch.Tensor] = None, y: Optional[torch.Tensor] = None,
                            ws: Optional[torch.Tensor] = None, stream=None, warm_start: bool = False,
                            breakdown: float = 0.0) -> Tuple[torch.Tensor, torch.Tensor, List[dict]]:
        """ls_forward and the far field of every solution in one call: (u, y, info)."""
        f = self._chk_f(f)
        if warm_start and u is None:
            raise ValueError("warm_start needs u (the initial guesses)")
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        Q = d.shape[0]
        if u is None:
            u = torch.empty((Q, self.n, self.n, self.n), dtype=self.cdtype, device=self.device)
        self._chk_like(u, (Q, self.n, self.n, self.n), self.cdtype, "u")
        if y is None:
            y = torch.empty((Q, self.n, self.n), dtype=self.cdtype, device=self.device)
        self._chk_like(y, (Q, self.n, self.n), self.cdtype, "y")
        ws = self.workspace(Q, L.LS_OP_FORWARD) if ws is None else ws
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts, 1 if warm_start else 0, breakdown)
        L.check(self.lib.ls_forward_farfield(self.h, _ptr(f), Q, d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(u),
                                             _ptr(y), C.byref(o), info, _ptr(ws), ws.numel(), _stream(stream)),
                "ls_forward_farfield")
        return u, y, [i.as_dict() for i in info]

    def ls_forward_farfield_noalloc(self, f: torch.Tensor, dirs, u: torch.Tensor, y: torch.Tensor, tol: float = 1e-5,
                                    maxit: int = 500, max_restarts: int = 3, stream=None, warm_start: bool = False,
                                    breakdown: float = 0.0) -> List[dict]:
        """ls_forward_farfield into the caller's u [Q, n, n, n] and y [Q, n, n] with the library's fixed
        device scratch (no workspace, nothing allocated on the device); returns the solve info."""
        f = self._chk_f(f)
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        Q = d.shape[0]
        self._chk_like(u, (Q, self.n, self.n, self.n), self.cdtype, "u")
        self._chk_like(y, (Q, self.n, self.n), self.cdtype, "y")
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts, 1 if warm_start else 0, breakdown)
        L.check(self.lib.ls_forward_farfield_noalloc(self.h, _ptr(f), Q, d.ctypes.data_as(C.POINTER(C.c_double)),
                                                     _ptr(u), _ptr(y), C.byref(o), info, _stream(stream)),
                "ls_forward_farfield_noalloc")
        return [i.as_dict() for i in info]

    def ls_forward_uin(self, f: torch.Tensor, uin: torch.Tensor, tol: float = 1e-5, maxit: int = 500,
                       max_restarts: int = 3, u: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                       stream=None, warm_start: bool = False, breakdown: float = 0.0) -> Tuple[torch.Tensor, List[dict]]:
        """Forward solves with stored incident volumes uin [Q, n, n, n] (warm_start, breakdown as in
        ls_forward)."""
        f = self._chk_f(f)
        if warm_start and u is None:
            raise ValueError("warm_start needs u (the initial guesses)")
        uin = self._chk_vol(uin, "uin")
        Q = uin.numel() // self.N
        if u is None:
            u = torch.empty_like(uin)
        self._chk_like(u, tuple(uin.shape), self.cdtype, "u")
        ws = self.workspace(Q, L.LS_OP_FORWARD) if ws is None else ws
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts, 1 if warm_start else 0, breakdown)
        L.check(self.lib.ls_forward_uin(self.h, _ptr(f), Q, _ptr(uin), _ptr(u), C.byref(o), info, _ptr(ws), ws.numel(),
                                        _stream(stream)), "ls_forward_uin")
        return u, [i.as_dict() for i in info]

    def ls_incident_field(self, y_in: torch.Tensor, ktilde=None, tilt: bool = True, out: Optional[torch.Tensor] = None,
                          ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Incident volumes [Q, n, n, n] from detector fields y_in [Q, n, n]; ktilde [Q, 2] (x, y)."""
        y_in = y_in.contiguous()
        if y_in.dtype != self.cdtype or y_in.device != self.device or tuple(y_in.shape[-2:]) != (self.n, self.n):
            raise ValueError(f"y_in: expected {self.cdtype} [Q, {self.n}, {self.n}] on {self.device}")
        Q = y_in.numel() // (self.n * self.n)
        kt = np.ascontiguousarray(np.zeros((Q, 2)) if ktilde is None else np.asarray(ktilde, dtype=np.float64)
                                  .reshape(Q, 2))
        u = torch.empty((Q, self.n, self.n, self.n), dtype=self.cdtype, device=self.device) if out is None else out
        self._chk_like(u, (Q, self.n, self.n, self.n), self.cdtype, "out")
        ws = self.workspace(Q, L.LS_OP_INCIDENT) if ws is None else ws
        L.check(self.lib.ls_incident_field(self.h, _ptr(y_in), kt.ctypes.data_as(C.POINTER(C.c_double)), Q,
                                           int(bool(tilt)), _ptr(u), _ptr(ws), ws.numel(), _stream(stream)),
                "ls_incident_field")
        return u

    def ls_farfield(self, f: torch.Tensor, u: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None
                    ) -> torch.Tensor:
        f = self._chk_f(f)
        u = self._chk_vol(u, "u")
        Q = u.numel() // self.N
        y = torch.empty((Q, self.n, self.n), dtype=self.cdtype, device=self.device)
        ws = self.workspace(Q, L.LS_OP_FARFIELD) if ws is None else ws
        L.check(self.lib.ls_farfield(self.h, _ptr(f), _ptr(u), Q, _ptr(y), _ptr(ws), ws.numel(), _stream(stream)),
                "ls_farfield")
        return y

    def ls_farfield_adj(self, r: torch.Tensor, conj: bool = False, stream=None,
                        ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        r = r.contiguous()
        if r.dtype != self.cdtype or r.device != self.device or r.shape[-2:] != (self.n, self.n):
            raise ValueError(f"r: expected [Q, n, n] in the field precision on {self.device}")
        Q = r.numel() // (self.n * self.n)
        out = torch.empty((Q, self.n, self.n, self.n), dtype=self.cdtype, device=self.device)
        ws = self.workspace(Q, L.LS_OP_FARFIELD) if ws is None else ws
        L.check(self.lib.ls_farfield_adj(self.h, _ptr(r), int(bool(conj)), Q, _ptr(out), _ptr(ws), ws.numel(),
                                         _stream(stream)), "ls_farfield_adj")
        return out

    def ls_vjp(self, f: torch.Tensor, u: torch.Tensor, gy: torch.Tensor, tol: float = 1e-5, maxit: int = 500,
               max_restarts: int = 3, ws: Optional[torch.Tensor] = None, stream=None
               ) -> Tuple[torch.Tensor, List[dict]]:
        f = self._chk_f(f)
        u = self._chk_vol(u, "u")
        Q = u.numel() // self.N
        gy = self._chk_det_q(gy, Q, "gy")
        grad = torch.empty((self.n,) * 3, dtype=self.rdtype, device=self.device)
        ws = self.workspace(Q, L.LS_OP_GRAD) if ws is None else ws
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts)
        L.check(self.lib.ls_vjp(self.h, _ptr(f), _ptr(u), Q, _ptr(gy), _ptr(grad), C.byref(o), info, _ptr(ws),
                                ws.numel(), _stream(stream)), "ls_vjp")
        return grad, [i.as_dict() for i in info]

    def ls_grad(self, f: torch.Tensor, dirs, y_meas: torch.Tensor, tol: float = 1e-5, maxit: int = 500,
                max_restarts: int = 3, ws: Optional[torch.Tensor] = None, stream=None
                ) -> Tuple[float, torch.Tensor, List[dict]]:
        f = self._chk_f(f)
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        Q = d.shape[0]
        y_meas = self._chk_det_q(y_meas, Q, "y_meas")
        grad = torch.empty((self.n,) * 3, dtype=self.rdtype, device=self.device)
        ws = self.workspace(Q, L.LS_OP_GRAD) if ws is None else ws
        info = (L.SolveInfo * (2 * Q))()
        loss = C.c_double()
        o = self._opts(tol, maxit, max_restarts)
        L.check(self.lib.ls_grad(self.h, _ptr(f), Q, d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(y_meas),
                                 _ptr(grad), C.byref(loss), C.byref(o), info, _ptr(ws), ws.numel(),
                                 _stream(stream)), "ls_grad")
        return loss.value, grad, [i.as_dict() for i in info]

    def ls_residual(self, y: torch.Tensor, y_meas: torch.Tensor, out: Optional[torch.Tensor] = None,
                    weighted: bool = False, stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        """r = y - y_meas (weighted: (y - y_meas) / ||y_meas_q||^2), the FP64 sums
        [||y_q - y_meas_q||^2, ||y_meas_q||^2] per illumination, and the data term of eq. (prob)
        as a 0-dim float64 device tensor."""
        y = y.contiguous()
        Q = y.numel() // (self.n * self.n)
        y = self._chk_det_q(y, Q, "y")
        y_meas = self._chk_det_q(y_meas, Q, "y_meas")
        r = torch.empty_like(y) if out is None else self._chk_det_q(out, Q, "out")
        stats = torch.empty(2 * Q, dtype=torch.float64, device=self.device)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        L.check(self.lib.ls_residual(self.h, _ptr(y), _ptr(y_meas), Q, 1 if weighted else 0, _ptr(r), _ptr(stats),
                                     _ptr(loss), _stream(stream)), "ls_residual")
        return r, stats, loss

    def ls_grad_accumulate(self, u: torch.Tensor, wb: torch.Tensor, grad: torch.Tensor,
                           stats: Optional[torch.Tensor] = None, accumulate: bool = False, stream=None) -> torch.Tensor:
        u = self._chk_vol(u, "u")
        Q = u.numel() // self.N
        wb = self._chk_like(wb, tuple(u.shape), self.cdtype, "wb")
        grad = self._chk_f(grad)
        if stats is not None:
            stats = self._chk_like(stats, (2 * Q,), torch.float64, "stats")
        L.check(self.lib.ls_grad_accumulate(self.h, _ptr(u), _ptr(wb), Q, _ptr(stats), _ptr(grad),
                                            int(bool(accumulate)), _stream(stream)), "ls_grad_accumulate")
        return grad

    # ---- detector-side operators
    def detector_workspace(self, m: int) -> torch.Tensor:
        b = C.c_size_t()
        L.check(self.lib.ls_detector_bytes(self.h, int(m), C.byref(b)), "ls_detector_bytes")
        key = ("det", int(m))
        ws = self._ws.get(key)
        if ws is None or ws.numel() < b.value:
            self._ws.pop(key, None)
            ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def _chk_det(self, y: torch.Tensor, m: int, name: str) -> torch.Tensor:
        if y.device != self.device or y.dtype != self.cdtype or not y.is_contiguous() or tuple(y.shape[-2:]) != (m, m):
            raise ValueError(f"{name}: expected contiguous {self.cdtype} [..., {m}, {m}] on {self.device}")
        return y

    def ls_farfield_wide(self, m: int, f: torch.Tensor, u: torch.Tensor, stream=None) -> torch.Tensor:
        f, u = self._chk_f(f), self._chk_vol(u, "u")
        Q = u.numel() // self.N
        y = torch.empty((Q, m, m), dtype=self.cdtype, device=self.device)
        ws = self.detector_workspace(m)
        L.check(self.lib.ls_farfield_wide(self.h, int(m), _ptr(f), _ptr(u), Q, _ptr(y), _ptr(ws), ws.numel(),
                                          _stream(stream)), "ls_farfield_wide")
        return y

    def ls_farfield_wide_adj(self, m: int, r: torch.Tensor, conj: bool = False, stream=None) -> torch.Tensor:
        r = self._chk_det(r.contiguous(), m, "r")
        Q = r.numel() // (m * m)
        out = torch.empty((Q, self.n, self.n, self.n), dtype=self.cdtype, device=self.device)
        ws = self.detector_workspace(m)
        L.check(self.lib.ls_farfield_wide_adj(self.h, int(m), _ptr(r), int(bool(conj)), Q, _ptr(out), _ptr(ws),
                                              ws.numel(), _stream(stream)), "ls_farfield_wide_adj")
        return out

    def ls_pupil(self, y: torch.Tensor, na: float, dz: float, adjoint: bool = False, stream=None) -> torch.Tensor:
        m = y.shape[-1]
        y = self._chk_det(y.contiguous(), m, "y")
        Q = y.numel() // (m * m)
        out = torch.empty_like(y)
        ws = self.detector_workspace(m)
        L.check(self.lib.ls_pupil(self.h, int(m), _ptr(y), Q, float(na), float(dz), int(bool(adjoint)), _ptr(out),
                                  _ptr(ws), ws.numel(), _stream(stream)), "ls_pupil")
        return out

    def ls_decimate(self, y: torch.Tensor, q: int, m: Optional[int] = None, transpose: bool = False,
                    stream=None) -> torch.Tensor:
        if not transpose:
            m = y.shape[-1]
            y = self._chk_det(y.contiguous(), m, "y")
            Q = y.numel() // (m * m)
            out = torch.empty((Q, m // q, m // q), dtype=self.cdtype, device=self.device)
        else:
            if m is None or m % q:
                raise ValueError("ls_decimate(transpose=True) needs the full detector size m, a multiple of q")
            y = self._chk_det(y.contiguous(), m // q, "y")
            Q = y.numel() // ((m // q) ** 2)
            out = torch.empty((Q, m, m), dtype=self.cdtype, device=self.device)
        L.check(self.lib.ls_decimate(self.h, int(m), int(q), _ptr(y), Q, _ptr(out), int(bool(transpose)),
                                     _stream(stream)), "ls_decimate")
        return out

    def ls_vjp_rhs(self, f: torch.Tensor, u: torch.Tensor, b: torch.Tensor, tol: float = 1e-5, maxit: int = 500,
                   max_restarts: int = 3, ws: Optional[torch.Tensor] = None, stream=None
                   ) -> Tuple[torch.Tensor, List[dict]]:
        f, u = self._chk_f(f), self._chk_vol(u, "u")
        Q = u.numel() // self.N
        b = self._chk_like(b.contiguous(), tuple(u.shape), self.cdtype, "b")
        grad = torch.empty((self.n,) * 3, dtype=self.rdtype, device=self.device)
        ws = self.workspace(Q, L.LS_OP_GRAD) if ws is None else ws
        info = (L.SolveInfo * Q)()
        o = self._opts(tol, maxit, max_restarts)
        L.check(self.lib.ls_vjp_rhs(self.h, _ptr(f), _ptr(u), Q, _ptr(b), _ptr(grad), C.byref(o), info, _ptr(ws),
                                    ws.numel(), _stream(stream)), "ls_vjp_rhs")
        return grad, [i.as_dict() for i in info]

    # ---- reconstruction step (Algorithm 1)
    def ls_prox_tv(self, v: torch.Tensor, lam: float, iters: int, d: Optional[torch.Tensor] = None,
                   gamma: float = 0.0, nonneg: bool = True, out: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """prox of lam TV + i_{>=0} at v - gamma d (at v when d is None)."""
        v = self._chk_f(v)
        if d is not None:
            d = self._chk_f(d)
        x = torch.empty_like(v) if out is None else self._chk_f(out)
        ws = self.workspace(1, L.LS_OP_PROX) if ws is None else ws
        L.check(self.lib.ls_prox_tv(self.h, _ptr(v), _ptr(d), float(gamma), float(lam), int(iters), int(bool(nonneg)),
                                    _ptr(x), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), "ls_prox_tv")
        return x

    def ls_fbs_extrapolate(self, f: torch.Tensor, f_prev: torch.Tensor, beta: float,
                           out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """f + beta (f - f_prev)."""
        f, f_prev = self._chk_f(f), self._chk_f(f_prev)
        v = torch.empty_like(f) if out is None else self._chk_f(out)
        L.check(self.lib.ls_fbs_extrapolate(self.h, _ptr(f), _ptr(f_prev), float(beta), _ptr(v), _stream(stream)),
                "ls_fbs_extrapolate")
        return v

    def ls_tv_value(self, x: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None) -> float:
        x = self._chk_f(x)
        ws = self.workspace(1, L.LS_OP_PROX) if ws is None else ws
        out = C.c_double()
        L.check(self.lib.ls_tv_value(self.h, _ptr(x), C.byref(out), _ptr(ws), ws.numel() * ws.element_size(),
                                     _stream(stream)), "ls_tv_value")
        return out.value


def profile_pass(ctx: "Context", f: torch.Tensor, u: torch.Tensor, pass_id: int, reps: int,
                 ws: torch.Tensor, stream=None) -> None:
    """ls_profile_pass: enqueue `reps` launches of one solver pass (for timing a kernel alone)."""
    Q = u.numel() // ctx.N
    L.check(ctx.lib.ls_profile_pass(ctx.h, _ptr(f), _ptr(u), int(pass_id), Q, int(reps), _ptr(ws), ws.numel(),
                                    _stream(stream)), "ls_profile_pass")


class Batch:
    """Slot pool for continuous batching (ls_batch_*)."""

    def __init__(self, ctx: Context, nslots: int, tol: float = 1e-5, maxit: int = 500, max_restarts: int = 3):
        self.ctx = ctx
        self.lib = ctx.lib
        self.nslots = int(nslots)
        b = C.c_size_t()
        L.check(self.lib.ls_batch_bytes(ctx.h, self.nslots, C.byref(b)), "ls_batch_bytes")
        self.ws = torch.empty(b.value, dtype=torch.uint8, device=ctx.device)
        o = L.SolveOpts(float(tol), int(maxit), int(max_restarts))
        h = C.c_void_p()
        L.check(self.lib.ls_batch_create(ctx.h, self.nslots, _ptr(self.ws), self.ws.numel(), C.byref(o), C.byref(h)),
                "ls_batch_create")
        self.h = h
        self._keep = {}

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                self.lib.ls_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def ls_batch_admit(self, slot: int, f: torch.Tensor, x: torch.Tensor, direction=None,
                       rhs: Optional[torch.Tensor] = None, stream=None) -> None:
        c, vol = self.ctx, (self.ctx.n,) * 3
        c._chk_f(f)
        c._chk_like(x, vol, c.cdtype, "x")
        if rhs is not None:
            c._chk_like(rhs, vol, c.cdtype, "rhs")
        dptr = None
        if direction is not None:
            d = np.ascontiguousarray(np.asarray(direction, dtype=np.float64).reshape(3))
            self._keep[("dir", slot)] = d
            dptr = d.ctypes.data_as(C.POINTER(C.c_double))
        self._keep[slot] = (f, x, rhs)
        L.check(self.lib.ls_batch_admit(self.h, int(slot), _ptr(f), dptr, _ptr(rhs), _ptr(x), _stream(stream)),
                "ls_batch_admit")

    def ls_batch_step(self, iters: int, stream=None) -> None:
        L.check(self.lib.ls_batch_step(self.h, int(iters), _stream(stream)), "ls_batch_step")

    def ls_batch_poll(self):
        st = (C.c_int32 * self.nslots)()
        info = (L.SolveInfo * self.nslots)()
        L.check(self.lib.ls_batch_poll(self.h, st, info), "ls_batch_poll")
        return list(st), [i.as_dict() for i in info]

    def ls_batch_release(self, slot: int) -> None:
        L.check(self.lib.ls_batch_release(self.h, int(slot)), "ls_batch_release")
        self._keep.pop(slot, None)
        self._keep.pop(("dir", slot), None)

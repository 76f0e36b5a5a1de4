"""Python binding of the mifft C ABI on torch tensors and streams.

torch provides device memory and streams only; every transform step runs in
libmifft.so.  Names follow the C ABI: ``plan_create``, ``execute_forward``,
``execute_inverse``, ``plan_destroy`` and friends take and return raw handles
and device pointers; ``Plan``, ``PencilPlan``, ``SlabPlan`` and ``BatchPlan``
wrap them for tensors.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from ._lib import (MIFFT_C2C, MIFFT_FP32, MIFFT_FP64, MIFFT_HEURISTIC, MIFFT_R2C,
                   MIFFT_SLAB_INVERSE, MIFFT_SLAB_PACK, MIFFT_SLAB_UNPACK, MIFFT_SLAB_X,
                   MIFFT_SLAB_Y, MIFFT_SLAB_Z, MIFFT_STAGE_PACK, MIFFT_STAGE_UNPACK,
                   MIFFT_STAGE_Y, MIFFT_STAGE_Z, MIFFT_TUNE, MifftError, check, lib)

_KIND = {"c2c": MIFFT_C2C, "r2c": MIFFT_R2C}
_PREC = {"fp32": MIFFT_FP32, "fp64": MIFFT_FP64}
_CDTYPE = {"fp32": torch.complex64, "fp64": torch.complex128}
_RDTYPE = {"fp32": torch.float32, "fp64": torch.float64}


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream or None
    return int(stream) or None


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("mifft works on device tensors")
    if not t.is_contiguous():
        raise ValueError("mifft needs contiguous tensors")
    return t.data_ptr() or None


# ------------------------------------------------------- raw C-ABI mirrors

def plan_create(n0: int, n1: int, n2: int, kind: int = MIFFT_C2C, prec: int = MIFFT_FP32,
                flags: int = MIFFT_HEURISTIC) -> int:
    h = ctypes.c_void_p()
    check(lib.mifft_plan_create(ctypes.byref(h), n0, n1, n2, kind, prec, flags),
          "mifft_plan_create")
    return h.value


def plan_create_pencil(n0, n1, n2, p0, p1, kind=MIFFT_C2C, prec=MIFFT_FP32, flags=0) -> int:
    h = ctypes.c_void_p()
    check(lib.mifft_plan_create_pencil(ctypes.byref(h), n0, n1, n2, p0, p1, kind, prec, flags),
          "mifft_plan_create_pencil")
    return h.value


def plan_create_nd(dims: Sequence[int], kind: int = MIFFT_C2C, prec: int = MIFFT_FP32,
                   flags: int = MIFFT_HEURISTIC) -> int:
    h = ctypes.c_void_p()
    arr = (ctypes.c_int * len(dims))(*[int(d) for d in dims])
    check(lib.mifft_plan_create_nd(ctypes.byref(h), len(dims), arr, kind, prec, flags),
          "mifft_plan_create_nd")
    return h.value


def plan_create_slab(n0, n1, n2, p, kind=MIFFT_C2C, prec=MIFFT_FP32, flags=0) -> int:
    h = ctypes.c_void_p()
    check(lib.mifft_plan_create_slab(ctypes.byref(h), n0, n1, n2, p, kind, prec, flags),
          "mifft_plan_create_slab")
    return h.value


def execute_forward(plan: int, in_ptr: int, out_ptr: int, stream: Optional[int] = None) -> None:
    check(lib.mifft_execute_forward(plan, in_ptr, out_ptr, stream), "mifft_execute_forward")


def execute_inverse(plan: int, in_ptr: int, out_ptr: int, stream: Optional[int] = None) -> None:
    check(lib.mifft_execute_inverse(plan, in_ptr, out_ptr, stream), "mifft_execute_inverse")


def execute_forward_ws(plan, in_ptr, out_ptr, ws_ptr, stream=None) -> None:
    check(lib.mifft_execute_forward_ws(plan, in_ptr, out_ptr, ws_ptr, stream),
          "mifft_execute_forward_ws")


def execute_inverse_ws(plan, in_ptr, out_ptr, ws_ptr, stream=None) -> None:
    check(lib.mifft_execute_inverse_ws(plan, in_ptr, out_ptr, ws_ptr, stream),
          "mifft_execute_inverse_ws")


def execute_pencil_stages(plan, mask, a, send, recv, out, stream=None) -> None:
    check(lib.mifft_execute_pencil_stages(plan, mask, a, send, recv, out, stream),
          "mifft_execute_pencil_stages")


def execute_slab_stages(plan, mask, in_ptr, send, recv, out, stream=None) -> None:
    check(lib.mifft_execute_slab_stages(plan, mask, in_ptr, send, recv, out, stream),
          "mifft_execute_slab_stages")


def poisson_solve(plan, f_ptr, u_ptr, ws_ptr=None, stream=None) -> None:
    check(lib.mifft_poisson_solve(plan, f_ptr, u_ptr, ws_ptr, stream), "mifft_poisson_solve")


def spectral_apply(plan, op, alpha, f_ptr, u_ptr, ws_ptr=None, stream=None) -> None:
    check(lib.mifft_spectral_apply(plan, op, float(alpha), f_ptr, u_ptr, ws_ptr, stream),
          "mifft_spectral_apply")


def spectral_gradient(plan, f_ptr, gx, gy, gz, ws_ptr=None, stream=None) -> None:
    check(lib.mifft_spectral_gradient(plan, f_ptr, gx, gy, gz, ws_ptr, stream), "mifft_spectral_gradient")


def spectral_divergence(plan, vx, vy, vz, d_ptr, ws_ptr=None, stream=None) -> None:
    check(lib.mifft_spectral_divergence(plan, vx, vy, vz, d_ptr, ws_ptr, stream), "mifft_spectral_divergence")


def spectral_ws_bytes(plan: int) -> int:
    return int(lib.mifft_spectral_ws_bytes(plan))


def workspace_bytes(plan: int) -> int:
    return int(lib.mifft_workspace_bytes(plan))


def poisson_ws_bytes(plan: int) -> int:
    return int(lib.mifft_poisson_ws_bytes(plan))


def plan_destroy(plan: int) -> None:
    check(lib.mifft_plan_destroy(plan), "mifft_plan_destroy")


def plan_describe(plan: int) -> str:
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib.mifft_plan_describe(plan, buf, len(buf)), "mifft_plan_describe")
    return buf.value.decode()


def profile_begin(plan: int, max_calls: int) -> None:
    check(lib.mifft_profile_begin(plan, max_calls), "mifft_profile_begin")


def profile_end(plan: int, max_passes: int = 16):
    """Mean per-pass durations (ms) of the profiled calls, and the call count."""
    buf = (ctypes.c_float * max_passes)()
    npass, ncalls = ctypes.c_int(), ctypes.c_int()
    check(lib.mifft_profile_end(plan, buf, max_passes, ctypes.byref(npass), ctypes.byref(ncalls)),
          "mifft_profile_end")
    return [float(buf[i]) for i in range(npass.value)], ncalls.value


def version() -> str:
    return lib.mifft_version().decode()


# ------------------------------------------------------------ tensor API

class Plan:
    """A planned transform of a C-order array on the current device: 3-D
    (n0, n1, n2) grids, or any rank 1 .. 8 (axes transformed last to first,
    Algorithm 2).

    kind "c2c": forward / inverse map complex arrays of `shape`.
    kind "r2c": forward maps real `shape` to complex with the last extent
    n // 2 + 1, inverse is the C2R map back; ``poisson`` (3-D only) solves
    lap(u) = f.  Neither direction is scaled.
    """

    def __init__(self, shape: Sequence[int], kind: str = "c2c", prec: str = "fp32",
                 tune: bool = False):
        self.shape = tuple(int(s) for s in shape)
        if not 1 <= len(self.shape) <= 8:
            raise ValueError("shape must have 1 .. 8 extents")
        self.kind, self.prec = kind, prec
        flags = MIFFT_TUNE if tune else MIFFT_HEURISTIC
        if len(self.shape) == 3:
            self.handle = plan_create(*self.shape, _KIND[kind], _PREC[prec], flags)
        else:
            self.handle = plan_create_nd(self.shape, _KIND[kind], _PREC[prec], flags)
        self.cdtype, self.rdtype = _CDTYPE[prec], _RDTYPE[prec]
        last = self.shape[-1]
        self.spec_shape = self.shape[:-1] + (last // 2 + 1,) if kind == "r2c" else self.shape

    @property
    def workspace_bytes(self) -> int:
        return workspace_bytes(self.handle)

    @property
    def poisson_ws_bytes(self) -> int:
        return poisson_ws_bytes(self.handle)

    def describe(self) -> str:
        return plan_describe(self.handle)

    def _check(self, t: torch.Tensor, shape, dtype, name: str):
        if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            raise ValueError("%s must be %s %s, got %s %s" % (name, tuple(shape), dtype,
                                                               tuple(t.shape), t.dtype))

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        in_dtype = self.rdtype if self.kind == "r2c" else self.cdtype
        self._check(x, self.shape, in_dtype, "input")
        if out is None:
            out = torch.empty(self.spec_shape, dtype=self.cdtype, device=x.device)
        self._check(out, self.spec_shape, self.cdtype, "output")
        s = _stream_handle(stream)
        if ws is None:
            execute_forward(self.handle, _ptr(x), _ptr(out), s)
        else:
            execute_forward_ws(self.handle, _ptr(x), _ptr(out), _ptr(ws), s)
        return out

    def inverse(self, y: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(y, self.spec_shape, self.cdtype, "input")
        out_dtype = self.rdtype if self.kind == "r2c" else self.cdtype
        if out is None:
            out = torch.empty(self.shape, dtype=out_dtype, device=y.device)
        self._check(out, self.shape, out_dtype, "output")
        s = _stream_handle(stream)
        if ws is None:
            execute_inverse(self.handle, _ptr(y), _ptr(out), s)
        else:
            execute_inverse_ws(self.handle, _ptr(y), _ptr(out), _ptr(ws), s)
        return out

    def poisson(self, f: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(f, self.shape, self.rdtype, "f")
        if out is None:
            out = torch.empty(self.shape, dtype=self.rdtype, device=f.device)
        self._check(out, self.shape, self.rdtype, "out")
        poisson_solve(self.handle, _ptr(f), _ptr(out), _ptr(ws), _stream_handle(stream))
        return out

    @property
    def spectral_ws_bytes(self) -> int:
        return spectral_ws_bytes(self.handle)

    def _ws(self, ws, need: int):
        if ws is not None and ws.numel() * ws.element_size() < need:
            raise ValueError("workspace of %d bytes is smaller than the %d needed"
                             % (ws.numel() * ws.element_size(), need))
        return _ptr(ws)

    def spectral(self, op: int, f: torch.Tensor, out: Optional[torch.Tensor] = None,
                 alpha: float = 0.0, stream=None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """u = C2R(m(k) R2C(f)) / N for one of the MIFFT_OP_* operators."""
        self._check(f, self.shape, self.rdtype, "f")
        if out is None:
            out = torch.empty(self.shape, dtype=self.rdtype, device=f.device)
        self._check(out, self.shape, self.rdtype, "out")
        spectral_apply(self.handle, op, alpha, _ptr(f), _ptr(out), self._ws(ws, self.poisson_ws_bytes),
                       _stream_handle(stream))
        return out

    def gradient(self, f: torch.Tensor, outs=None, stream=None, ws: Optional[torch.Tensor] = None):
        """(df/dx, df/dy, df/dz) of a real periodic field."""
        self._check(f, self.shape, self.rdtype, "f")
        if outs is None:
            outs = [torch.empty(self.shape, dtype=self.rdtype, device=f.device) for _ in range(3)]
        for g in outs:
            self._check(g, self.shape, self.rdtype, "gradient component")
        spectral_gradient(self.handle, _ptr(f), *[_ptr(g) for g in outs],
                          self._ws(ws, self.spectral_ws_bytes), _stream_handle(stream))
        return outs

    def divergence(self, v, out: Optional[torch.Tensor] = None, stream=None,
                   ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dv0/dx + dv1/dy + dv2/dz of three real periodic fields."""
        for c in v:
            self._check(c, self.shape, self.rdtype, "field component")
        if out is None:
            out = torch.empty(self.shape, dtype=self.rdtype, device=v[0].device)
        self._check(out, self.shape, self.rdtype, "out")
        spectral_divergence(self.handle, *[_ptr(c) for c in v], _ptr(out),
                            self._ws(ws, self.spectral_ws_bytes), _stream_handle(stream))
        return out

    def close(self) -> None:
        if getattr(self, "handle", None):
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PencilPlan:
    """One rank's share of the pencil forward transform (Algorithm 1, up to
    the y-FFT) of an (N0, N1, N2) C2C grid on a p0 x p1 process grid."""

    def __init__(self, shape: Sequence[int], grid: Sequence[int], prec: str = "fp32"):
        self.shape = tuple(int(s) for s in shape)
        self.p0, self.p1 = (int(g) for g in grid)
        self.prec = prec
        self.handle = plan_create_pencil(*self.shape, self.p0, self.p1, MIFFT_C2C, _PREC[prec])
        n0, n1, n2 = self.shape
        self.n0l, self.n1l, self.m = n0 // self.p0, n1 // self.p1, n2 // self.p1
        self.local_shape = (self.n0l, self.n1l, n2)
        self.send_shape = (self.p1, self.n0l, self.n1l, self.m)
        self.out_shape = (self.n0l, n1, self.m)
        self.cdtype = _CDTYPE[prec]

    def stages(self, mask: int, a=None, send=None, recv=None, out=None, stream=None) -> None:
        execute_pencil_stages(self.handle, mask, _ptr(a), _ptr(send), _ptr(recv), _ptr(out),
                              _stream_handle(stream))

    def forward_share(self, a: torch.Tensor, send: torch.Tensor, out: torch.Tensor,
                      recv: Optional[torch.Tensor] = None, fused: bool = True, stream=None):
        """z-FFT, pack, exchange (loopback when recv is None), unpack, y-FFT."""
        recv = send if recv is None else recv
        if fused:
            self.stages(MIFFT_STAGE_Z | MIFFT_STAGE_PACK, a=a, send=send, stream=stream)
            self.stages(MIFFT_STAGE_UNPACK | MIFFT_STAGE_Y, recv=recv, out=out, stream=stream)
        else:
            self.stages(MIFFT_STAGE_Z, a=a, stream=stream)
            self.stages(MIFFT_STAGE_PACK, a=a, send=send, stream=stream)
            self.stages(MIFFT_STAGE_UNPACK, recv=recv, out=out, stream=stream)
            self.stages(MIFFT_STAGE_Y, out=out, stream=stream)
        return out

    def describe(self) -> str:
        return plan_describe(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlabPlan:
    """One task's share of the slab-decomposed transform (Algorithm 3) of an
    (N0, N1, N2) grid over p tasks: spatial slab (N0/p, N1, N2), spectral
    share (N0, N1/p, N2c); send / receive buffers (p, N0/p, N1/p, N2c)."""

    def __init__(self, shape: Sequence[int], p: int, kind: str = "c2c", prec: str = "fp32"):
        self.shape = tuple(int(s) for s in shape)
        self.p, self.kind, self.prec = int(p), kind, prec
        self.handle = plan_create_slab(*self.shape, self.p, _KIND[kind], _PREC[prec])
        n0, n1, n2 = self.shape
        nc = n2 // 2 + 1 if kind == "r2c" else n2
        self.n0l, self.n1l, self.nc = n0 // self.p, n1 // self.p, nc
        self.slab_shape = (self.n0l, n1, n2)
        self.mid_shape = (self.n0l, n1, nc)      # the 2-D transformed slab
        self.share_shape = (n0, self.n1l, nc)
        self.send_shape = (self.p, self.n0l, self.n1l, nc)
        self.cdtype = _CDTYPE[prec]
        self.sdtype = _RDTYPE[prec] if kind == "r2c" else self.cdtype

    def stages(self, mask: int, src=None, send=None, recv=None, out=None, stream=None) -> None:
        """Raw stage call: the tensors are passed as pointers, unchecked."""
        execute_slab_stages(self.handle, mask, _ptr(src), _ptr(send), _ptr(recv), _ptr(out),
                            _stream_handle(stream))

    def _check(self, t: torch.Tensor, shape, dtype, name: str):
        if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            raise ValueError("%s must be %s %s, got %s %s" % (name, tuple(shape), dtype,
                                                               tuple(t.shape), t.dtype))

    def forward_local(self, a: torch.Tensor, send: torch.Tensor, mid: torch.Tensor,
                      fused: bool = True, stream=None) -> torch.Tensor:
        """2-D FFTs of the slab's x-planes, written in the send layout; `mid`
        (mid_shape, complex) holds the z-transformed slab in between."""
        self._check(a, self.slab_shape, self.sdtype, "slab")
        self._check(send, self.send_shape, self.cdtype, "send")
        self._check(mid, self.mid_shape, self.cdtype, "mid")
        if fused:
            self.stages(MIFFT_SLAB_Z | MIFFT_SLAB_Y | MIFFT_SLAB_PACK, src=a, send=send, out=mid,
                        stream=stream)
        else:
            self.stages(MIFFT_SLAB_Z | MIFFT_SLAB_Y, src=a, out=mid, stream=stream)
            self.stages(MIFFT_SLAB_PACK, send=send, out=mid, stream=stream)
        return send

    def forward_x(self, recv: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """x-FFT of the received slab: out is the spectral share."""
        self._check(recv, self.send_shape, self.cdtype, "recv")
        self._check(out, self.share_shape, self.cdtype, "out")
        self.stages(MIFFT_SLAB_X, recv=recv, out=out, stream=stream)
        return out

    def inverse_x(self, y: torch.Tensor, send: torch.Tensor, stream=None) -> torch.Tensor:
        self._check(y, self.share_shape, self.cdtype, "share")
        self._check(send, self.send_shape, self.cdtype, "send")
        self.stages(MIFFT_SLAB_INVERSE | MIFFT_SLAB_X, src=y, send=send, stream=stream)
        return send

    def inverse_local(self, recv: torch.Tensor, send: torch.Tensor, out: torch.Tensor,
                      fused: bool = True, stream=None) -> torch.Tensor:
        """Unpack, y-IFFT and z-IFFT (C2R) into the spatial slab `out`; `send`
        is the complex scratch in between."""
        self._check(recv, self.send_shape, self.cdtype, "recv")
        self._check(send, self.send_shape, self.cdtype, "send")
        self._check(out, self.slab_shape, self.sdtype, "out")
        if fused:
            self.stages(MIFFT_SLAB_INVERSE | MIFFT_SLAB_UNPACK | MIFFT_SLAB_Y | MIFFT_SLAB_Z,
                        recv=recv, send=send, out=out, stream=stream)
        else:
            self.stages(MIFFT_SLAB_INVERSE | MIFFT_SLAB_UNPACK, recv=recv, send=send, stream=stream)
            self.stages(MIFFT_SLAB_INVERSE | MIFFT_SLAB_Y | MIFFT_SLAB_Z, send=send, out=out,
                        stream=stream)
        return out

    def describe(self) -> str:
        return plan_describe(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Plan", "PencilPlan", "SlabPlan", "MifftError", "plan_create", "plan_create_pencil",
           "plan_create_slab", "plan_create_nd", "execute_forward", "execute_inverse", "execute_forward_ws",
           "execute_inverse_ws", "execute_pencil_stages", "execute_slab_stages", "poisson_solve",
           "spectral_apply", "spectral_gradient", "spectral_divergence", "spectral_ws_bytes",
           "workspace_bytes", "poisson_ws_bytes", "plan_destroy", "plan_describe",
           "profile_begin", "profile_end", "version"]

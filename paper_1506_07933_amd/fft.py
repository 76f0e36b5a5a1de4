"""Python binding of the mifft C ABI on torch tensors and streams.

torch provides device memory and streams only; every transform step runs in
libmifft.so.  Names follow the C ABI: ``plan_create``, ``execute_forward``,
``execute_inverse``, ``plan_destroy`` and friends take and return raw handles
and device pointers; ``Plan``, ``PencilPlan`` and ``BatchPlan`` wrap them for
tensors.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from ._lib import (MIFFT_C2C, MIFFT_FP32, MIFFT_FP64, MIFFT_HEURISTIC, MIFFT_R2C,
                   MIFFT_STAGE_PACK, MIFFT_STAGE_UNPACK, MIFFT_STAGE_Y, MIFFT_STAGE_Z,
                   MIFFT_TUNE, MifftError, check, lib)

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


def poisson_solve(plan, f_ptr, u_ptr, ws_ptr=None, stream=None) -> None:
    check(lib.mifft_poisson_solve(plan, f_ptr, u_ptr, ws_ptr, stream), "mifft_poisson_solve")


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
    """A planned 3-D transform of an (n0, n1, n2) grid on the current device.

    kind "c2c": forward / inverse map complex [n0][n1][n2] arrays.
    kind "r2c": forward maps real [n0][n1][n2] to complex [n0][n1][n2//2+1],
    inverse is the C2R map back; ``poisson`` solves lap(u) = f.
    Neither direction is scaled.
    """

    def __init__(self, shape: Sequence[int], kind: str = "c2c", prec: str = "fp32",
                 tune: bool = False):
        self.shape = tuple(int(s) for s in shape)
        if len(self.shape) != 3:
            raise ValueError("shape must have 3 extents")
        self.kind, self.prec = kind, prec
        self.handle = plan_create(*self.shape, _KIND[kind], _PREC[prec],
                                  MIFFT_TUNE if tune else MIFFT_HEURISTIC)
        self.cdtype, self.rdtype = _CDTYPE[prec], _RDTYPE[prec]
        n0, n1, n2 = self.shape
        self.spec_shape = (n0, n1, n2 // 2 + 1) if kind == "r2c" else self.shape

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
        poisson_solve(self.handle, _ptr(f), _ptr(out), _ptr(ws), _stream_handle(stream))
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
    """One rank's share of the pencil forward transform (Algorithm 1, steps
    1-3) of an (N0, N1, N2) C2C grid on a p0 x p1 process grid."""

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


__all__ = ["Plan", "PencilPlan", "MifftError", "plan_create", "plan_create_pencil",
           "execute_forward", "execute_inverse", "execute_forward_ws", "execute_inverse_ws",
           "execute_pencil_stages", "poisson_solve", "workspace_bytes", "poisson_ws_bytes",
           "plan_destroy", "plan_describe", "profile_begin", "profile_end", "version"]

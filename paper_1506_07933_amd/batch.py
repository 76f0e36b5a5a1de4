"""Batched uneven-size 3-D C2C transforms: one persistent launch per batch.

Binding of mifft_batch_create / mifft_batch_execute_forward /
mifft_batch_graph_launch / mifft_batch_check / mifft_batch_destroy.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from ._lib import (MIFFT_BATCH_GROUPED, MIFFT_BATCH_KERNELS, MIFFT_C2C, MIFFT_FP32, MIFFT_FP64,
                   MIFFT_TUNE, check, lib)
from .fft import _ptr, _stream_handle

_PREC = {"fp32": MIFFT_FP32, "fp64": MIFFT_FP64}
_CDTYPE = {"fp32": torch.complex64, "fp64": torch.complex128}


class BatchPlan:
    """Forward C2C transforms of len(shapes) grids of uneven sizes.

    mode "persistent": one persistent kernel for the whole batch (axis
    lengths 2..256 with factors 2, 3, 5); mode "kernels": the per-pass
    kernels of ordinary plans (any supported length); mode "grouped": those
    kernels with each pass of all transforms of one shape as one launch."""

    def __init__(self, shapes: Sequence[Sequence[int]], prec: str = "fp32",
                 mode: str = "persistent", tune: bool = False):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.prec = prec
        dims = (ctypes.c_int * (3 * len(self.shapes)))(*[v for s in self.shapes for v in s])
        modes = {"persistent": 0, "kernels": MIFFT_BATCH_KERNELS, "grouped": MIFFT_BATCH_GROUPED}
        if mode not in modes:
            raise ValueError("mode must be one of %s" % sorted(modes))
        flags = modes[mode] | (MIFFT_TUNE if tune else 0)
        h = ctypes.c_void_p()
        check(lib.mifft_batch_create(ctypes.byref(h), len(self.shapes), dims, MIFFT_C2C,
                                     _PREC[prec], flags), "mifft_batch_create")
        self.handle = h.value
        self.cdtype = _CDTYPE[prec]

    def _arrays(self, xs, outs):
        if len(xs) != len(self.shapes) or len(outs) != len(self.shapes):
            raise ValueError("need one input and one output per transform")
        for x, o, s in zip(xs, outs, self.shapes):
            for t in (x, o):
                if tuple(t.shape) != s or t.dtype != self.cdtype:
                    raise ValueError("buffer must be %s %s" % (s, self.cdtype))
        n = len(self.shapes)
        ins = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
        ous = (ctypes.c_void_p * n)(*[_ptr(o) for o in outs])
        return ins, ous

    def forward(self, xs, outs=None, stream=None, graph: bool = False):
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        ins, ous = self._arrays(xs, outs)
        s = _stream_handle(stream)
        if graph:
            check(lib.mifft_batch_graph_launch(self.handle, ins, ous, s), "mifft_batch_graph_launch")
        else:
            check(lib.mifft_batch_execute_forward(self.handle, ins, ous, s),
                  "mifft_batch_execute_forward")
        return outs

    def aborted(self) -> bool:
        """True if a bounded wait of the last launch ran out (outputs invalid)."""
        flag = ctypes.c_int()
        check(lib.mifft_batch_check(self.handle, ctypes.byref(flag)), "mifft_batch_check")
        return bool(flag.value)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        check(lib.mifft_batch_describe(self.handle, buf, len(buf)), "mifft_batch_describe")
        return buf.value.decode()

    def close(self) -> None:
        if getattr(self, "handle", None):
            check(lib.mifft_batch_destroy(self.handle), "mifft_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

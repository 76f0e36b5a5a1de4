"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mifft.h declares, and rejects bad arguments with the
documented status codes before it makes any HIP call."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mifft.h")


@pytest.fixture(scope="module")
def L():
    from paper_1506_07933_amd._lib import lib
    return lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mifft_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mifft_plan_create", "mifft_execute_forward", "mifft_execute_inverse",
                 "mifft_plan_destroy", "mifft_last_error", "mifft_plan_create_pencil",
                 "mifft_execute_pencil_stages", "mifft_plan_create_slab",
                 "mifft_execute_slab_stages", "mifft_plan_create_nd", "mifft_batch_create",
                 "mifft_batch_execute_forward", "mifft_poisson_solve"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_signatures_cover_header():
    from paper_1506_07933_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == declared_functions()


def _create(L, n0, n1, n2, kind=0, prec=0, flags=0):
    h = ctypes.c_void_p()
    rc = L.mifft_plan_create(ctypes.byref(h), n0, n1, n2, kind, prec, flags)
    return rc, h


@pytest.mark.parametrize("args,status", [
    ((0, 4, 4), 1), ((4, -1, 4), 1), ((4, 4, 0), 1),
    ((7, 4, 4), 2), ((4, 4, 11), 2), ((2048, 4, 4), 2), ((4, 1026, 4), 2),
    ((4, 4, 49), 2),
])
def test_bad_sizes(L, args, status):
    rc, h = _create(L, *args)
    assert rc == status
    assert h.value is None
    assert L.mifft_last_error()


def test_bad_enums_and_flags(L):
    assert _create(L, 4, 4, 4, kind=2)[0] == 1
    assert _create(L, 4, 4, 4, prec=7)[0] == 1
    assert _create(L, 4, 4, 4, flags=0x80)[0] == 1
    assert L.mifft_plan_create(None, 4, 4, 4, 0, 0, 0) == 1


def test_r2c_needs_even_n2(L):
    rc, _ = _create(L, 4, 4, 9, kind=1)
    assert rc == 2
    assert b"even" in L.mifft_last_error()


def test_pencil_validation(L):
    h = ctypes.c_void_p()
    f = L.mifft_plan_create_pencil
    assert f(ctypes.byref(h), 1024, 1024, 1024, 4, 3, 0, 0, 0) == 2   # 3 does not divide 1024
    assert f(ctypes.byref(h), 1024, 1024, 1024, 0, 4, 0, 0, 0) == 1
    assert f(ctypes.byref(h), 1024, 1024, 1024, 4, 4, 1, 0, 0) == 2   # R2C share not offered
    assert f(None, 1024, 1024, 1024, 4, 4, 0, 0, 0) == 1


def test_slab_validation(L):
    h = ctypes.c_void_p()
    f = L.mifft_plan_create_slab
    assert f(ctypes.byref(h), 512, 512, 512, 3, 0, 0, 0) == 2     # 3 does not divide 512
    assert f(ctypes.byref(h), 512, 96, 512, 64, 0, 0, 0) == 2     # p divides N0 but not N1
    assert f(ctypes.byref(h), 512, 512, 512, 0, 0, 0, 0) == 1
    assert f(ctypes.byref(h), 512, 512, 511, 4, 1, 0, 0) == 2     # R2C needs an even n2
    assert f(ctypes.byref(h), 512, 512, 512, 4, 0, 0, 1) == 1     # MIFFT_TUNE not offered
    assert f(ctypes.byref(h), 512, 512, 512, 4, 3, 0, 0) == 1     # bad kind
    assert f(None, 512, 512, 512, 4, 0, 0, 0) == 1
    # a plan-only slab plan describes but never executes
    assert f(ctypes.byref(h), 64, 32, 16, 4, 1, 1, 2) == 0
    buf = ctypes.c_void_p(0x10000)
    assert L.mifft_execute_slab_stages(h, 1, buf, buf, buf, buf, None) == 5
    assert L.mifft_execute_forward(h, buf, buf, None) == 5
    assert b"slab" in L.mifft_last_error()
    assert L.mifft_execute_pencil_stages(h, 1, buf, buf, buf, buf, None) == 5
    assert L.mifft_workspace_bytes(h) == 0
    assert L.mifft_plan_destroy(h) == 0


def test_nd_validation(L):
    h = ctypes.c_void_p()
    f = L.mifft_plan_create_nd

    def dims(*d):
        return (ctypes.c_int * len(d))(*d)
    assert f(ctypes.byref(h), 0, dims(4), 0, 0, 0) == 1               # rank 0
    assert f(ctypes.byref(h), 9, dims(*([2] * 9)), 0, 0, 0) == 1       # rank above MIFFT_MAX_RANK
    assert f(ctypes.byref(h), 4, None, 0, 0, 0) == 1
    assert f(None, 4, dims(2, 2, 2, 2), 0, 0, 0) == 1
    assert f(ctypes.byref(h), 4, dims(2, 0, 2, 2), 0, 0, 0) == 1
    assert f(ctypes.byref(h), 4, dims(2, 7, 2, 2), 0, 0, 0) == 2       # prime factor 7
    assert f(ctypes.byref(h), 4, dims(2, 2, 2, 9), 1, 0, 0) == 2       # R2C, odd last extent
    assert f(ctypes.byref(h), 4, dims(1024, 1024, 1024, 2), 0, 0, 2) == 2  # 2^31 elements
    assert f(ctypes.byref(h), 4, dims(2, 2, 2, 2), 0, 0, 1) == 2       # MIFFT_TUNE: rank <= 3 only
    assert f(ctypes.byref(h), 4, dims(2, 2, 2, 2), 2, 0, 0) == 1       # bad kind
    assert f(ctypes.byref(h), 2, dims(4, 7), 0, 0, 2) == 2             # rank <= 3 checks as 3-D
    # plan-only N-D plans describe but never execute or solve Poisson
    assert f(ctypes.byref(h), 5, dims(4, 3, 2, 5, 6), 1, 1, 2) == 0
    buf = ctypes.c_void_p(0x10000)
    assert L.mifft_execute_forward(h, buf, buf, None) == 5
    assert L.mifft_poisson_solve(h, buf, buf, None, None) == 5
    assert L.mifft_plan_destroy(h) == 0


def test_stale_and_null_handles(L):
    bogus = ctypes.c_void_p(0x1234560)
    assert L.mifft_plan_destroy(None) == 0
    assert L.mifft_plan_destroy(bogus) == 5
    buf = ctypes.c_void_p(0x10000)
    assert L.mifft_execute_forward(None, buf, buf, None) == 1
    assert L.mifft_execute_forward(bogus, buf, buf, None) == 5
    assert L.mifft_execute_inverse(bogus, buf, buf, None) == 5
    assert L.mifft_execute_pencil_stages(bogus, 1, buf, buf, buf, buf, None) == 5
    assert L.mifft_execute_slab_stages(bogus, 1, buf, buf, buf, buf, None) == 5
    assert L.mifft_execute_slab_stages(None, 1, buf, buf, buf, buf, None) == 1
    assert L.mifft_poisson_solve(bogus, buf, buf, None, None) == 5
    assert L.mifft_spectral_apply(bogus, 1, 0.0, buf, buf, None, None) == 5
    assert L.mifft_spectral_apply(None, 1, 0.0, buf, buf, None, None) == 1
    assert L.mifft_spectral_gradient(bogus, buf, buf, buf, buf, None, None) == 5
    assert L.mifft_spectral_divergence(bogus, buf, buf, buf, buf, None, None) == 5
    assert L.mifft_spectral_ws_bytes(bogus) == 0
    assert L.mifft_workspace_bytes(bogus) == 0
    s = ctypes.create_string_buffer(64)
    assert L.mifft_plan_describe(bogus, s, 64) == 5
    assert L.mifft_batch_destroy(None) == 0


def test_last_error_is_per_call(L):
    _create(L, 7, 4, 4)
    assert L.mifft_last_error()
    L.mifft_plan_destroy(None)
    assert L.mifft_last_error() == b""


def test_no_device_reports_device_error(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    rc, h = _create(L, 32, 32, 32)
    assert rc == 4
    assert h.value is None


def test_binding_raises_typed_error():
    from paper_1506_07933_amd.fft import MifftError, plan_create
    with pytest.raises(MifftError) as e:
        plan_create(7, 4, 4)
    assert e.value.status_name == "MIFFT_ERR_UNSUPPORTED"


def test_package_exports_load_the_library():
    import paper_1506_07933_amd as pkg
    assert pkg.Plan.__name__ == "Plan"
    assert pkg.PencilPlan.__name__ == "PencilPlan"
    assert pkg.SlabPlan.__name__ == "SlabPlan"
    assert issubclass(pkg.MifftError, RuntimeError)
    from paper_1506_07933_amd import Plan  # noqa: F401


def test_batch_argument_validation(L):
    import ctypes as C
    h = C.c_void_p()
    dims = (C.c_int * 6)(64, 64, 64, 48, 48, 48)
    assert L.mifft_batch_create(None, 2, dims, 0, 0, 0) == 1
    assert L.mifft_batch_create(C.byref(h), 0, dims, 0, 0, 0) == 1
    assert L.mifft_batch_create(C.byref(h), 2, dims, 1, 0, 0) == 2      # R2C batches not offered
    assert L.mifft_batch_create(C.byref(h), 2, dims, 0, 0, 0x100) == 1  # unknown flag
    assert L.mifft_batch_create(C.byref(h), 2, dims, 0, 0, 4 | 8) == 1   # kernels and grouped
    big = (C.c_int * 6)(512, 64, 64, 48, 48, 48)
    assert L.mifft_batch_create(C.byref(h), 2, big, 0, 0, 0) == 2       # 512 not in the menu
    assert L.mifft_batch_create(C.byref(h), 129, (C.c_int * 387)(*([8] * 387)), 0, 0, 0) == 2
    ones = (C.c_int * 6)(1, 1, 1, 48, 48, 48)
    assert L.mifft_batch_create(C.byref(h), 2, ones, 0, 0, 0) == 2     # 1x1x1 has no pass
    bogus = C.c_void_p(0x4321000)
    arr = (C.c_void_p * 2)()
    assert L.mifft_batch_execute_forward(bogus, arr, arr, None) == 5
    assert L.mifft_batch_destroy(bogus) == 5
    flag = C.c_int()
    assert L.mifft_batch_check(bogus, C.byref(flag)) == 5


def test_reference_copies_reject_out_of_range_patterns(L):
    """The measurement copies check every offset against the caller's sizes
    on the host, before any launch (the pointers here are never touched)."""
    a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x40000000)
    L_, cols, groups, es, gs = 40, 45, 3, 48, 48 * 40
    need_in = (groups - 1) * gs + (cols - 1) + (L_ - 1) * es + 1
    es_o, gs_o = 3 * 45, 45
    need_out = (groups - 1) * gs_o + (cols - 1) + (L_ - 1) * es_o + 1
    f = L.mifft_pattern_copy
    assert f(0, a, need_in - 1, b, need_out, L_, cols, groups, es, es_o, gs, gs_o, 16, 8, 0, None) == 1
    assert b"reaches" in L.mifft_last_error()
    assert f(0, a, need_in, b, need_out - 1, L_, cols, groups, es, es_o, gs, gs_o, 16, 8, 0, None) == 1
    # huge strides cannot wrap around the size check
    assert f(0, a, 1 << 40, b, 1 << 40, 1024, 1, 2, 1 << 62, 1, 1 << 62, 1, 1, 1, 0, None) == 1
    assert f(0, a, need_in, a, need_out, L_, cols, groups, es, es_o, gs, gs_o, 16, 8, 0, None) == 1  # overlap
    assert f(0, a, need_in, b, need_out, L_, cols, groups, es, es_o, gs, gs_o, 16, 8, 4, None) == 1  # flags
    assert f(0, a, need_in, b, need_out, L_, cols, groups, es, es_o, gs, gs_o, 64, 32, 0, None) == 1  # 2048 threads
    assert f(0, a, need_in, b, need_out, L_, cols, groups, -1, es_o, gs, gs_o, 16, 8, 0, None) == 1
    assert f(0, None, need_in, b, need_out, L_, cols, groups, es, es_o, gs, gs_o, 16, 8, 0, None) == 1
    assert f(0, ctypes.c_void_p(0x100004), need_in, b, need_out, L_, cols, groups, es, es_o, gs, gs_o,
             16, 8, 0, None) == 1                                                              # misaligned
    g = L.mifft_copy_reference
    assert g(a, ctypes.c_void_p(0x100000 + 4096), 8192, 0, 0, None) == 1       # overlap
    assert g(a, b, 100, 0, 0, None) == 1                                        # not a multiple of 16
    assert g(a, b, 4096, 8, 0, None) == 1                                       # flags
    assert g(a, b, 4096, 0, -1, None) == 1                                      # grid
    assert g(None, b, 4096, 0, 0, None) == 1


def test_static_scratch_entry_rejects_large_workspaces(L):
    """The no-allocation forward transform refuses a plan whose workspace
    exceeds the static scratch array, before any HIP call (a plan-only 512^3
    C2C plan needs 1 GiB for its transposed intermediate)."""
    from paper_1506_07933_amd._lib import MIFFT_C2C, MIFFT_FP32, MIFFT_PLAN_ONLY
    p = ctypes.c_void_p()
    assert L.mifft_plan_create(ctypes.byref(p), 512, 512, 512, MIFFT_C2C, MIFFT_FP32, MIFFT_PLAN_ONLY) == 0
    try:
        assert L.mifft_workspace_bytes(p) == 512 ** 3 * 8 > 256 << 20
        a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x40000000)
        assert L.mifft_execute_forward_static(p, a, b, None) == 1
        assert b"static scratch" in L.mifft_last_error()
        assert L.mifft_execute_forward_static(None, a, b, None) == 1
    finally:
        assert L.mifft_plan_destroy(p) == 0
    # a plan-only plan that fits is refused as any plan-only execute is
    q = ctypes.c_void_p()
    assert L.mifft_plan_create(ctypes.byref(q), 64, 64, 64, MIFFT_C2C, MIFFT_FP32, MIFFT_PLAN_ONLY) == 0
    try:
        assert L.mifft_execute_forward_static(q, ctypes.c_void_p(0x100000), ctypes.c_void_p(0x40000000), None) == 5
    finally:
        assert L.mifft_plan_destroy(q) == 0

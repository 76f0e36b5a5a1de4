"""The autotuner's search space on the CPU: every compiled kernel variant's
radix list multiplies to its length and uses the radices 2, 3, 4, 5, 8; its
threads per line match one (emul = 1) or two (emul = 2) radix groups of the
largest stage; every supported length has the default variant the planner
falls back on; and the policies are the documented radix orders."""
import ctypes
from math import prod

import pytest

from paper_1506_07933_amd._lib import lib


def variants(prec):
    buf = ctypes.create_string_buffer(1 << 20)
    assert lib.mifft_variants_describe(prec, buf, len(buf)) == 0, lib.mifft_last_error()
    out = []
    for line in buf.value.decode().splitlines():
        d = dict(kv.split("=") for kv in line.split())
        out.append({"L": int(d["L"]), "policy": int(d["policy"]), "emul": int(d["emul"]),
                    "tpl": int(d["tpl"]), "radix": [int(r) for r in d["radix"].split("x") if r]})
    return out


def _smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("prec", [0, 1])
def test_every_variant_factorises_its_length(prec):
    vs = variants(prec)
    assert len(vs) > 100
    for v in vs:
        if v["L"] == 1:
            assert v["radix"] == []
            continue
        assert prod(v["radix"]) == v["L"], v
        assert set(v["radix"]) <= {2, 3, 4, 5, 8}, v
        assert v["emul"] in (1, 2) and v["policy"] in (0, 1, 2)
        # threads per line: one (emul 1) or two (emul 2) butterflies of the
        # largest radix per thread
        assert v["tpl"] * max(v["radix"]) * v["emul"] == v["L"], v


@pytest.mark.parametrize("prec", [0, 1])
def test_every_supported_length_has_a_default_variant(prec):
    have = {(v["L"], v["policy"], v["emul"]) for v in variants(prec)}
    lengths = {v["L"] for v in variants(prec)}
    assert lengths == {n for n in range(1, 1025) if _smooth(n)}
    for n in lengths:
        assert (n, 0, 1) in have, n


def test_policies_are_radix_orders():
    """Variants of one length with different policies use the same multiset
    of radices only where the policy merely reorders stages (policy 1);
    policy 2 starts with radix 4 where the length allows it."""
    by = {}
    for v in variants(0):
        by.setdefault(v["L"], {})[(v["policy"], v["emul"])] = v["radix"]
    for L, d in by.items():
        if (0, 1) in d and (1, 1) in d:
            assert sorted(d[(0, 1)]) == sorted(d[(1, 1)]), L
        if (2, 1) in d and L % 4 == 0:
            assert d[(2, 1)][0] == 4, (L, d[(2, 1)])


def test_buffer_too_small_is_an_error():
    buf = ctypes.create_string_buffer(16)
    assert lib.mifft_variants_describe(0, buf, len(buf)) == 1
    assert lib.mifft_variants_describe(5, ctypes.create_string_buffer(64), 64) == 1

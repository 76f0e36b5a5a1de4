"""MIFFT_TUNE on the GPU: tuned plans keep parity with the oracle, the wisdom
file is written, and a second plan of the same shape reuses it (same
choices, no new timing)."""
import os

import numpy as np
import pytest

import oracle
from paper_1506_07933_amd import synth
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tuned_plans_parity_and_wisdom(tmp_path):
    wisdom = tmp_path / "wisdom.json"
    os.environ["MIFFT_WISDOM"] = str(wisdom)
    from paper_1506_07933_amd import Plan
    # (64, 256, 256) R2C runs the transposed intermediate with padded rows
    cases = [((128, 96, 64), "c2c", "fp32"), ((64, 64, 64), "r2c", "fp64"), ((48, 100, 120), "c2c", "fp64"),
             ((64, 256, 256), "r2c", "fp32")]
    for shape, kind, prec in cases:
        p = Plan(shape, kind, prec, tune=True)
        print("  tuned", shape, kind, prec, "\n", p.describe(), flush=True)
        if kind == "c2c":
            cd = np.complex64 if prec == "fp32" else np.complex128
            x = synth.uniform_complex(shape, cd, seed=2)
            X = p.forward(torch.from_numpy(x).cuda()).cpu().numpy()
            assert rel_l2(X, oracle.fft3d_c2c(x.astype(np.complex128), -1)) <= TOL[prec]
            xi = p.inverse(torch.from_numpy(X).cuda()).cpu().numpy()
            assert rel_l2(xi, np.prod(shape) * x.astype(np.complex128)) <= TOL[prec]
        else:
            rd = np.float32 if prec == "fp32" else np.float64
            x = synth.normal_real(shape, rd, seed=2)
            x64 = x.astype(np.float64)
            Y = p.forward(torch.from_numpy(x).cuda())
            assert rel_l2(Y.cpu().numpy(), oracle.fft3d_r2c(x64)) <= TOL[prec]
            assert rel_l2(p.inverse(Y).cpu().numpy(), np.prod(shape) * x64) <= TOL[prec]
            f = (x64 - x64.mean()).astype(rd)
            u = p.poisson(torch.from_numpy(f).cuda()).cpu().numpy()
            assert rel_l2(u, oracle.poisson_solve(f.astype(np.float64))) <= TOL[prec]
        first = p.describe()
        p.close()
        text = wisdom.read_text()
        assert "gfx950|" in text
        q = Plan(shape, kind, prec, tune=True)
        assert q.describe() == first   # the wisdom entries are reused
        q.close()
    import json
    entries = json.loads(wisdom.read_text())
    assert len(entries) >= 6
    del os.environ["MIFFT_WISDOM"]

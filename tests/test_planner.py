"""Planner checks on the CPU (MIFFT_PLAN_ONLY: pass lists and launch shapes,
no device).  They pin the launch configurations the GPU tests and the
benchmark rely on: the kernel grids cover every line / column exactly, LDS
and workgroup sizes stay within the gfx950 limits, and the transposed
intermediate is used where the x-stride is large."""
import ctypes
import re

import pytest

from paper_1506_07933_amd._lib import MIFFT_PLAN_ONLY, lib
from paper_1506_07933_amd.fft import plan_describe, plan_destroy


def plan_only(n0, n1, n2, kind=0, prec=0):
    h = ctypes.c_void_p()
    rc = lib.mifft_plan_create(ctypes.byref(h), n0, n1, n2, kind, prec, MIFFT_PLAN_ONLY)
    assert rc == 0, lib.mifft_last_error()
    text = plan_describe(h.value)
    ws = lib.mifft_workspace_bytes(h.value)
    pws = lib.mifft_poisson_ws_bytes(h.value)
    plan_destroy(h.value)
    passes = []
    for line in text.splitlines():
        d = dict(kv.split("=") for kv in line.split()[1:])
        d["dir"] = line.split()[0]
        passes.append(d)
    return passes, ws, pws


def ints(d, *keys):
    return [int(d[k]) for k in keys]


SHAPES = [(512, 512, 512), (256, 256, 1024), (32, 32, 32), (100, 120, 144), (125, 125, 125),
          (1, 1, 1), (3, 1024, 2), (1024, 3, 2), (64, 1, 1), (48, 64, 96), (2, 2, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", [0, 1])
def test_launch_shapes_cover_and_fit(shape, prec, kind):
    if kind == 1 and shape[2] % 2:
        pytest.skip("R2C needs an even n2")
    passes, ws, _ = plan_only(*shape, kind=kind, prec=prec)
    esz = 16 if prec else 8
    for p in passes:
        if p["kind"] in ("copy", "poisson"):
            continue
        grid, block, lds = ints(p, "grid", "block", "lds")
        assert 1 <= block <= 1024
        assert lds <= 160 * 1024
        if p["kind"] in ("contig", "r2c_z", "c2r_z"):
            lines, lpw, tpl, L = ints(p, "lines", "lpw", "tpl", "L")
            assert block == lpw * tpl
            assert grid * lpw >= lines > (grid - 1) * lpw
            # per-line tiles (padded; real kernels hold L + 1 points) + the twiddle table
            n = L if p["kind"] == "contig" else L + 1
            assert lds == (lpw * (n + (n >> 3) + 1) + L) * esz
        elif p["kind"] == "poisson_x":
            B, cols, groups, tpl, L = ints(p, "B", "cols", "groups", "tpl", "L")
            assert B & (B - 1) == 0 and block == B * tpl
            tpg = int(p["tpg"])
            assert grid == (-(-cols * groups // B) if tpg == 0 else groups * tpg)
            assert lds == (B * L + L) * esz
        elif p["kind"] == "strided":
            B, cols, groups, tpl, L = ints(p, "B", "cols", "groups", "tpl", "L")
            assert B & (B - 1) == 0 and block == B * tpl
            tpg = int(p["tpg"])
            # tiles over the flattened (group, column) index where one side is
            # contiguous across groups (gs = cols), else per group
            gs_in, gs_out = (int(v) for v in p["gs"].split("/"))
            assert (tpg == 0) == (gs_out == cols or gs_in == cols)
            tiles = -(-cols * groups // B) if tpg == 0 else groups * tpg
            assert int(p["tiles"]) == tiles
            if p["pf"] == "1":
                # prefetching kernels walk the tiles with a grid of at most one
                # resident wave of workgroups (256 CUs x workgroups per CU)
                per_cu = max(1, min(160 * 1024 // lds, 2048 // block))
                cap = 256 * per_cu
                rounds = -(-tiles // cap)
                assert grid == -(-tiles // rounds)  # balanced: every workgroup walks `rounds` tiles
                assert grid <= cap and grid * rounds >= tiles > grid * (rounds - 1)
            else:
                assert grid == tiles
            assert lds == (B * L + L) * esz  # column tile + the twiddle table


def test_512_cube_default_schedule_is_unchunked():
    passes, ws, _ = plan_only(512, 512, 512)
    assert ws == 512 ** 3 * 8
    assert [p["axis"] for p in passes if p["dir"] == "forward"] == ["z", "y", "x"]
    assert [p["axis"] for p in passes if p["dir"] == "inverse"] == ["y", "x", "z"]
    assert not [p for p in passes if p["dir"].endswith("_inplace")]


def test_512_cube_blocked_schedule_geometry(monkeypatch):
    """Out of place, the 512^3 complex64 transform passes through blocked
    intermediates of 32-column (256-byte) blocks: z stores T[x][zb][y][zc]
    through the pack map, y reads contiguous 512 x 32 blocks of T and writes
    U[k1][zb][x][zc], x reads contiguous blocks of U and writes the standard
    layout.  In-place calls run the transposed schedule."""
    monkeypatch.setenv("MIFFT_BLOCKED", "1")
    passes, _, _ = plan_only(512, 512, 512)
    assert [p["axis"] for p in passes if p["dir"] == "inverse"] == ["z", "y", "x"]
    assert [p["axis"] for p in passes if p["dir"] == "forward_inplace"] == ["z", "y", "x"]
    assert [p["axis"] for p in passes if p["dir"] == "inverse_inplace"] == ["y", "x", "z"]
    z, y, x = [p for p in passes if p["dir"] == "forward"]
    n, W = 512, 32
    assert z["kind"] == "contig_pack" and z["pm"] == "%d/%d" % (W, n * W)
    assert y["kind"] == x["kind"] == "strided"
    assert y["B"] == x["B"] == y["cols"] == x["cols"] == str(W)
    assert y["groups"] == x["groups"] == str(n * n // W)
    # y: group g = x nb + zb at g n1 W (one contiguous block); row k1 at k1 n0 n2
    # + zb n0 W + x W
    assert y["es"] == "%d/%d" % (W, n * n) and y["gs"] == "%d/%d" % (n * W, W)
    assert y["gdiv"] == "0/%d" % (n // W) and y["gs2"] == "0/%d" % (n * W) and y["nt"] == "1"
    # x: group g = k1 nb + zb at g n0 W; row k0 of the output at k0 n1 n2 + g W
    assert x["es"] == "%d/%d" % (W, n * n) and x["gs"] == "%d/%d" % (n * W, W)
    assert x["gdiv"] == "0/0" and x["nt"] == "1"


def _emulate(passes, x, nws):
    """Run a plan's pass list on the CPU: every pass's index maps as the
    kernels compute them (tiles, two-level group maps, the pack map), with a
    numpy FFT per line."""
    import numpy as np

    def pair(v):
        a, b = v.split("/")
        return int(a), int(b)
    bufs = {"in": x.copy(), "out": np.zeros_like(x), "ws": np.zeros(max(nws, 1), dtype=x.dtype)}
    flow = [("in", "out"), ("out", "ws"), ("ws", "out")]
    for k, p in enumerate(passes):
        src, dst = flow[k]
        S, D = bufs[src], bufs[dst]
        L = int(p["L"])
        fft = (lambda a: np.fft.fft(a, axis=-1)) if p["sgn"] == "1" else \
              (lambda a: np.fft.ifft(a, axis=-1) * a.shape[-1])
        if p["kind"] == "contig_pack":
            M, blk = pair(p["pm"])
            nl, ni = int(p["lines"]), int(p["ni"])
            is_o, is_i = pair(p["is"])
            os_o, os_i = pair(p["os"])
            line = np.arange(nl)
            lo, li = line // ni, line % ni
            ib = lo * is_o + li * is_i
            ob = lo * os_o + li * os_i
            idx = np.arange(L)
            q = idx // M
            off = ob[:, None] + q[None, :] * blk + (idx - q * M)[None, :]
            D[off.ravel()] = fft(S[ib[:, None] + idx[None, :]]).ravel()
        else:
            assert p["kind"] == "strided"
            B, cols, groups, tpg, tiles = ints(p, "B", "cols", "groups", "tpg", "tiles")
            es_in, es_out = pair(p["es"])
            gs_in, gs_out = pair(p["gs"])
            gd_in, gd_out = pair(p["gdiv"])
            g2_in, g2_out = pair(p["gs2"])
            tl = np.repeat(np.arange(tiles), B)
            cc = np.tile(np.arange(B), tiles)
            if tpg > 0:
                g = tl // tpg
                col = (tl - g * tpg) * B + cc
                g = np.where(col >= cols, groups, g)
            else:
                f = tl * B + cc
                g = f // cols
                col = f - g * cols
            ok = g < groups
            g, col = g[ok], col[ok]

            def goff(d, s1, s2):
                return (g // d) * s1 + (g % d) * s2 if d > 1 else g * s1
            ib = goff(gd_in, gs_in, g2_in) + col
            ob = goff(gd_out, gs_out, g2_out) + col
            r = np.arange(L)
            D[ob[:, None] + r[None, :] * es_out] = fft(S[ib[:, None] + r[None, :] * es_in])
    return bufs["out"]


@pytest.mark.parametrize("shape,prec", [((8, 64, 512), 0), ((6, 40, 1024), 0), ((4, 32, 512), 1),
                                         ((10, 96, 192), 1)])
def test_blocked_schedule_maps_compose_to_the_3d_dft(monkeypatch, shape, prec):
    """The blocked schedule's index maps (pack map of the z-pass, tiles and
    two-level group maps of the strided passes), followed on the CPU with a
    library FFT per line, give the 3-D DFT forward and n0 n1 n2 times the
    input back: every element is read from where the pass before wrote it."""
    import numpy as np
    monkeypatch.setenv("MIFFT_BLOCKED", "1")
    passes, ws, _ = plan_only(*shape, prec=prec)
    fwd = [p for p in passes if p["dir"] == "forward"]
    inv = [p for p in passes if p["dir"] == "inverse"]
    assert [p["kind"] for p in fwd] == ["contig_pack", "strided", "strided"]
    assert [p["kind"] for p in inv] == ["contig_pack", "strided", "strided"]
    n = int(np.prod(shape))
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    nws = ws // (16 if prec else 8)
    ref = np.fft.fftn(x.reshape(shape)).ravel()
    y = _emulate(fwd, x, nws)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    z = _emulate(inv, ref, nws)
    assert np.linalg.norm(z - n * x) <= 1e-12 * np.linalg.norm(n * x)


def test_512_cube_chunked_transposed_intermediate(monkeypatch):
    monkeypatch.setenv("MIFFT_CHUNK_MIB", "128")
    passes, ws, _ = plan_only(512, 512, 512)
    assert ws == 512 ** 3 * 8
    fwd = [p for p in passes if p["dir"] == "forward"]
    # z and y interleaved over x-plane chunks, then x
    assert [p["axis"] for p in fwd] == ["z", "y"] * (len(fwd) // 2) + ["x"]
    zs, ys, x = fwd[0:-1:2], fwd[1:-1:2], fwd[-1]
    assert sum(int(p["lines"]) for p in zs) == 512 * 512
    assert sum(int(p["groups"]) for p in ys) == 512
    # chunk k starts where chunk k-1 ended (byte offsets)
    line_bytes = 512 * 8
    off = 0
    for z in zs:
        assert z["off"] == "%d/%d" % (off, off)
        off += int(z["lines"]) * line_bytes
    g = 0
    for y in ys:
        # y reads x-planes (stride n1 n2) and writes W[k1][x][k2] (x stride n2)
        assert y["es"] == "512/262144" and y["gs"] == "262144/512"
        assert y["off"] == "%d/%d" % (g * 262144 * 8, g * 512 * 8)
        g += int(y["groups"])
    # x reads W with stride n2 and writes the standard layout (stride n1 n2)
    assert x["es"] == "512/262144" and x["gs"] == "262144/512" and x["groups"] == "512"
    assert x["B"] == "32" and x["tpl"] == "32" and x["pf"] == "1"
    inv = [p for p in passes if p["dir"] == "inverse"]
    assert [p["axis"] for p in inv] == ["y"] + ["x", "z"] * ((len(inv) - 1) // 2)
    assert sum(int(p["lines"]) for p in inv if p["axis"] == "z") == 512 * 512


def test_small_grid_keeps_standard_layout():
    passes, ws, _ = plan_only(32, 32, 32, prec=1)
    assert ws == 0
    for p in passes:
        if p["kind"] == "strided":
            a, b = p["es"].split("/")
            assert a == b


def test_r2c_workspace_sizes(monkeypatch):
    # transposed intermediate: rows of the half spectrum (129) padded to a
    # multiple of 128 bytes (136 complex128)
    passes, ws, pws = plan_only(256, 256, 256, kind=1, prec=1)
    w = 256 * 256 * 136 * 16
    assert ws == w
    fwd = [p for p in passes if p["dir"] == "forward"]
    assert fwd[1]["es"] == "129/%d" % (256 * 136) and fwd[1]["gs"] == "%d/136" % (256 * 129)
    assert fwd[2]["es"] == "136/%d" % (256 * 129) and fwd[2]["gs"] == "%d/129" % (256 * 136)
    # the spectral chain keeps the Nyquist plane apart: each Poisson half holds
    # rows of exactly 128 complex128 and the 256 x 256 plane
    assert pws == 2 * 256 * 256 * (128 + 1) * 16
    # with the Nyquist column in the rows: the padded rows
    monkeypatch.setenv("MIFFT_POISSON_NYQ", "0")
    _, _, pws = plan_only(256, 256, 256, kind=1, prec=1)
    assert pws == 2 * w
    # small grids keep the standard layout and the unpadded workspace
    _, ws, pws = plan_only(32, 32, 32, kind=1, prec=1)
    assert pws == 2 * 32 * 32 * 17 * 16


def test_poisson_chain_with_the_nyquist_plane_apart():
    """512^3 R2C: the fused spectral chain transforms rows of exactly 256
    columns (8 column tiles of 32 per group for y, 16 of 16 for the fused x)
    and runs the k2 = 256 plane N[x][k1] through its own y, fused x
    (k2 fixed) and y^-1 passes, after W in the same half of the workspace."""
    passes, _, pws = plan_only(512, 512, 512, kind=1, prec=0)
    po = [p for p in passes if p["dir"] == "poisson"]
    assert [(p["kind"], p["axis"]) for p in po] == [
        ("r2c_z", "z"), ("strided", "y"), ("contig", "y"), ("poisson_x", "x"), ("poisson_x", "x"),
        ("contig", "y"), ("strided", "y"), ("c2r_z", "z")]
    noff = 512 * 512 * 256 * 8
    assert po[1]["cols"] == "256" and po[1]["tiles"] == str(512 * 8)
    assert po[3]["cols"] == "256" and po[3]["tiles"] == str(512 * 16)
    assert po[2]["off"] == po[4]["off"] == po[5]["off"] == "%d/%d" % (noff, noff)
    assert po[4]["cols"] == "512" and po[4]["groups"] == "1" and po[4]["es"] == "512/512"
    assert po[2]["lines"] == "512" and po[2]["L"] == "512"
    assert pws == 2 * (noff + 512 * 512 * 8)


def test_poisson_plane_passes_run_beside_the_main_chain_on_large_grids():
    """The Nyquist plane's three passes (lane 1) run on a side stream after the
    z-pass (fork) and before the C2R (join) where the half spectrum is at
    least 256 MiB; smaller solves run every pass in line."""
    passes, _, _ = plan_only(512, 512, 512, kind=1, prec=0)
    po = [p for p in passes if p["dir"] == "poisson"]
    assert [p["lane"] for p in po] == ["0", "0", "1", "0", "1", "1", "0", "0"]
    assert [p.get("fork") for p in po] == ["1"] + [None] * 7
    assert [p.get("join") for p in po] == [None] * 7 + ["1"]
    for shape in ((64, 64, 64), (256, 256, 256)):
        passes, _, _ = plan_only(*shape, kind=1, prec=0)
        po = [p for p in passes if p["dir"] == "poisson"]
        assert all(p["lane"] == "0" and "fork" not in p and "join" not in p for p in po)
    assert len(po) == 8  # 256^3 keeps the plane apart, in line


def test_plan_only_cannot_execute():
    h = ctypes.c_void_p()
    assert lib.mifft_plan_create(ctypes.byref(h), 8, 8, 8, 0, 0, MIFFT_PLAN_ONLY) == 0
    buf = ctypes.c_void_p(0x10000)
    assert lib.mifft_execute_forward(h, buf, buf, None) == 5
    assert lib.mifft_plan_destroy(h) == 0
    assert lib.mifft_plan_create(ctypes.byref(h), 8, 8, 8, 0, 0, MIFFT_PLAN_ONLY | 4) == 1


_WISDOM_CHILD = r"""
import ctypes, sys
from paper_1506_07933_amd._lib import MIFFT_PLAN_ONLY, lib
from paper_1506_07933_amd.fft import plan_describe, plan_destroy
h = ctypes.c_void_p()
assert lib.mifft_plan_create(ctypes.byref(h), 64, 64, 64, 0, 0, MIFFT_PLAN_ONLY | 1) == 0, lib.mifft_last_error()
print(plan_describe(h.value))
plan_destroy(h.value)
"""


def test_wisdom_only_plan_applies_valid_entries_and_ignores_malformed(tmp_path):
    """MIFFT_TUNE with MIFFT_PLAN_ONLY applies stored choices without a device.
    A strided tile width must be a power of two (the kernel maps threads to
    columns with a mask): B = 24 or B = 0 in a hand-edited file is ignored
    and the heuristic shape stays."""
    import os
    import subprocess
    import sys
    passes, _, _ = plan_only(64, 64, 64)
    y = [d for d in passes if d["dir"] == "forward" and d["axis"] == "y"][0]
    x = [d for d in passes if d["dir"] == "forward" and d["axis"] == "x"][0]
    z = [d for d in passes if d["dir"] == "forward" and d["axis"] == "z"][0]

    def key(d):
        return "gfx950|fp32|strided|L=64|cols=%s|groups=%s|es=%s|gs=%s" % (d["cols"], d["groups"], d["es"], d["gs"])

    assert int(y["B"]) != 8 and int(x["B"]) == int(y["B"])
    wis = tmp_path / "wisdom.json"
    wis.write_text("{\n"
                   '  "%s": [0, 1, 8, 0, 1.0],\n' % key(y) +          # valid: B = 8
                   '  "%s": [0, 1, 24, 0, 1.0],\n' % key(x) +         # not a power of two
                   '  "gfx950|fp32|contig|L=64|lines=%s": [0, 1, 0, 0, 1.0]\n' % z["lines"] +  # lpw 0
                   "}\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MIFFT_WISDOM=str(wis), PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", _WISDOM_CHILD], env=env, cwd=root,
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [dict(kv.split("=") for kv in l.split()[1:]) | {"dir": l.split()[0]}
           for l in out.stdout.splitlines() if l.startswith(("forward", "inverse"))]
    gy = [d for d in got if d["dir"] == "forward" and d["axis"] == "y"][0]
    gx = [d for d in got if d["dir"] == "forward" and d["axis"] == "x"][0]
    gz = [d for d in got if d["dir"] == "forward" and d["axis"] == "z"][0]
    assert int(gy["B"]) == 8 and int(gy["block"]) == 8 * int(gy["tpl"])
    assert gx["B"] == x["B"] and gz["lpw"] == z["lpw"]


def test_pencil_plan_only_describes_fused_stages():
    h = ctypes.c_void_p()
    assert lib.mifft_plan_create_pencil(ctypes.byref(h), 1024, 1024, 1024, 4, 4, 0, 0,
                                        MIFFT_PLAN_ONLY) == 0
    text = plan_describe(h.value)
    plan_destroy(h.value)
    assert "pencil_z_pack kind=contig_pack axis=z L=1024" in text
    assert "pencil_unpack_y kind=strided_unpack axis=y L=1024" in text


@pytest.mark.parametrize("shape,transposed", [((512, 512, 512), True), ((64, 48, 32), False)])
def test_poisson_fuses_the_x_passes(monkeypatch, shape, transposed):
    """R2C Poisson: z, y, fused x-forward * multiply * x-inverse, y^-1, z^-1
    (5 passes, the spectrum read and written once per pass) instead of
    7 passes plus the standalone multiply.  (Here with the Nyquist column in
    the rows; the default splits it off for the transposed layout, see
    test_poisson_chain_with_the_nyquist_plane_apart.)"""
    monkeypatch.setenv("MIFFT_POISSON_NYQ", "0")
    passes, _, pws = plan_only(*shape, kind=1, prec=0)
    po = [p for p in passes if p["dir"] == "poisson"]
    assert [p["kind"] for p in po] == ["r2c_z", "strided", "poisson_x", "strided", "c2r_z"]
    assert [p["axis"] for p in po] == ["z", "y", "x", "y", "z"]
    assert [p["sgn"] for p in po][1:4] == ["1", "1", "-1"]
    n0, n1, n2 = shape
    nc = n2 // 2 + 1
    pitch = -(-nc // 16) * 16 if transposed else nc   # internal rows padded to 128 bytes
    x = po[2]
    if transposed:   # on W[k1][x][k2]: lines along x (stride pitch), groups = k1, columns = k2
        assert x["es"] == "%d/%d" % (pitch, pitch) and x["groups"] == str(n1) and x["cols"] == str(nc)
        assert po[3]["es"] == "%d/%d" % (n0 * pitch, n0 * pitch) and po[3]["groups"] == str(n0)
        assert po[1]["es"] == "%d/%d" % (pitch, n0 * pitch)
    else:            # standard layout: one group of n1 * nc columns
        assert x["es"] == "%d/%d" % (n1 * nc, n1 * nc) and x["groups"] == "1"
        assert x["cols"] == str(n1 * nc)
    assert pws == 2 * n0 * n1 * pitch * 8


def test_poisson_unfused_switch(monkeypatch):
    monkeypatch.setenv("MIFFT_POISSON_UNFUSED", "1")
    passes, _, _ = plan_only(64, 48, 32, kind=1, prec=1)
    po = [p["kind"] for p in passes if p["dir"] == "poisson"]
    assert po == ["r2c_z", "strided", "strided", "poisson", "strided", "strided", "c2r_z"]


EXTENT_SHAPES = [(512, 512, 512), (256, 256, 256), (384, 384, 384), (100, 120, 144), (125, 125, 120),
                 (1024, 1, 2), (1, 1024, 2), (2, 2, 1024), (96, 1, 64), (3, 5, 8), (64, 64, 1024)]


@pytest.mark.parametrize("unfused", ["0", "1"])
@pytest.mark.parametrize("chunk", ["0", "16"])
def test_every_pass_stays_inside_its_buffers(monkeypatch, unfused, chunk):
    """The library validates, at plan time, that the largest offset every
    pass reads or writes lies inside its source and destination buffers
    (user arrays, workspace, Poisson halves); a violation fails plan
    creation with an internal error.  A planted under-sized Poisson
    workspace (the standard-layout size for the padded intermediate) is
    rejected this way.  Here: every schedule variant is accepted."""
    monkeypatch.setenv("MIFFT_POISSON_UNFUSED", unfused)
    monkeypatch.setenv("MIFFT_CHUNK_MIB", chunk)
    for shape in EXTENT_SHAPES:
        for kind in (0, 1):
            if kind == 1 and shape[2] % 2:
                continue
            for prec in (0, 1):
                h = ctypes.c_void_p()
                rc = lib.mifft_plan_create(ctypes.byref(h), *shape, kind, prec, MIFFT_PLAN_ONLY)
                assert rc == 0, (shape, kind, prec, lib.mifft_last_error())
                plan_destroy(h.value)


@pytest.mark.parametrize("shape,grid", [((1024, 1024, 1024), (4, 4)), ((256, 256, 512), (2, 4)),
                                        ((64, 96, 120), (1, 2)), ((32, 32, 32), (2, 2))])
def test_pencil_passes_stay_inside_the_share(shape, grid):
    """Pencil plans are checked the same way: every fused / plain z and y
    pass stays inside the (N0/p0) x (N1/p1) x N2 buffers of the share."""
    for prec in (0, 1):
        h = ctypes.c_void_p()
        rc = lib.mifft_plan_create_pencil(ctypes.byref(h), *shape, *grid, 0, prec, MIFFT_PLAN_ONLY)
        assert rc == 0, lib.mifft_last_error()
        plan_destroy(h.value)


def slab_only(shape, p, kind=0, prec=0):
    h = ctypes.c_void_p()
    rc = lib.mifft_plan_create_slab(ctypes.byref(h), *shape, p, kind, prec, MIFFT_PLAN_ONLY)
    assert rc == 0, lib.mifft_last_error()
    text = plan_describe(h.value)
    plan_destroy(h.value)
    out = {}
    for line in text.splitlines():
        d = dict(kv.split("=") for kv in line.split()[1:])
        out[line.split()[0]] = d
    return out


@pytest.mark.parametrize("kind", [0, 1])
def test_slab_plan_stages(kind):
    """Slab share of 512^3 over 4 tasks (Algorithm 3): z over the slab's
    (N0/p) N1 lines, y over (N0/p) groups of N2c columns with the pack fused
    into its stores (split every N1/p rows into blocks of (N0/p)(N1/p)N2c),
    x over the received slab (one group of (N1/p) N2c columns), and the
    inverse's y with the unpack fused into its loads."""
    n, p = 512, 4
    nc = n // 2 + 1 if kind else n
    st = slab_only((n, n, n), p, kind)
    z = st["slab_z"]
    assert z["kind"] == ("r2c_z" if kind else "contig")
    assert int(z["lines"]) == (n // p) * n
    y, yp = st["slab_y"], st["slab_y_pack"]
    assert (y["kind"], yp["kind"]) == ("strided", "strided_pack")
    assert ints(yp, "L", "cols", "groups") == [n, nc, n // p]
    assert yp["es"] == "%d/%d" % (nc, nc)
    assert yp["gs"] == "%d/%d" % (n * nc, (n // p) * nc)
    x = st["slab_x"]
    assert ints(x, "L", "cols", "groups") == [n, (n // p) * nc, 1]
    assert x["es"] == "%d/%d" % ((n // p) * nc, (n // p) * nc)
    assert st["slab_x_inv"]["sgn"] == "-1"
    yu = st["slab_unpack_y_inv"]
    assert yu["kind"] == "strided_unpack" and yu["sgn"] == "-1"
    assert yu["gs"] == "%d/%d" % ((n // p) * nc, n * nc)
    assert st["slab_z_inv"]["kind"] == ("c2r_z" if kind else "contig")
    assert st["slab_pack"]["kind"] == "pack" and st["slab_unpack"]["kind"] == "unpack"


@pytest.mark.parametrize("shape,p", [((512, 512, 512), 4), ((512, 512, 512), 512), ((64, 96, 120), 2),
                                     ((125, 125, 120), 5), ((8, 8, 2), 8), ((4, 6, 1), 2),
                                     ((1, 1, 1), 1), ((1024, 1024, 32), 64)])
def test_slab_passes_stay_inside_the_share(shape, p):
    """Every slab stage's reads and writes stay inside the share's buffers
    (checked by the library at plan time, for both kinds and precisions)."""
    for kind in (0, 1):
        if kind == 1 and shape[2] % 2:
            continue
        for prec in (0, 1):
            h = ctypes.c_void_p()
            rc = lib.mifft_plan_create_slab(ctypes.byref(h), *shape, p, kind, prec, MIFFT_PLAN_ONLY)
            assert rc == 0, (shape, p, kind, prec, lib.mifft_last_error())
            plan_destroy(h.value)


def nd_only(dims, kind=0, prec=0):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int * len(dims))(*dims)
    rc = lib.mifft_plan_create_nd(ctypes.byref(h), len(dims), arr, kind, prec, MIFFT_PLAN_ONLY)
    assert rc == 0, lib.mifft_last_error()
    text = plan_describe(h.value)
    ws = lib.mifft_workspace_bytes(h.value)
    plan_destroy(h.value)
    passes = []
    for line in text.splitlines():
        d = dict(kv.split("=") for kv in line.split()[1:])
        d["dir"] = line.split()[0]
        passes.append(d)
    return passes, ws, text


@pytest.mark.parametrize("kind", [0, 1])
def test_nd_4d_pass_list(kind):
    """512 x 256 x 128 x 64 (the paper's 4-D case): the last axis as
    contiguous lines, then one strided pass per earlier axis, last to first,
    each with the elements after the axis as its columns and the index range
    before it as its groups.  Axis 0's stride (256 x 128 x N2c elements) is
    large, so axis 1 writes the transposed intermediate W[k1][x0][rest] and
    axis 0 reads it with stride `rest`; the inverse runs axis 1 (into W),
    axis 0 (back to the standard layout), axis 2, then the last axis.  R2C
    halves the last axis; its inverse keeps the input (two spectra of
    workspace)."""
    d = (512, 256, 128, 64)
    nc = 33 if kind else 64
    rest = 128 * nc
    passes, ws, _ = nd_only(d, kind)
    fwd = [p for p in passes if p["dir"] == "forward"]
    inv = [p for p in passes if p["dir"] == "inverse"]
    assert fwd[0]["kind"] == ("r2c_z" if kind else "contig")
    assert int(fwd[0]["lines"]) == 512 * 256 * 128
    a2, a1, a0 = fwd[1:]
    assert ints(a2, "L", "cols", "groups") == [128, nc, 512 * 256]
    assert a2["es"] == "%d/%d" % (nc, nc) and a2["gs"] == "%d/%d" % (128 * nc, 128 * nc)
    assert int(a2["B"]) == 64      # 131072 groups of 33 / 64 columns: one tile per group
    assert ints(a1, "L", "cols", "groups") == [256, rest, 512]
    assert a1["es"] == "%d/%d" % (rest, 512 * rest) and a1["gs"] == "%d/%d" % (256 * rest, rest)
    assert ints(a0, "L", "cols", "groups") == [512, rest, 256]
    assert a0["es"] == "%d/%d" % (rest, 256 * rest) and a0["gs"] == "%d/%d" % (512 * rest, rest)
    assert all(q["sgn"] == "1" for q in fwd[1:])
    assert [int(q["L"]) for q in inv] == [256, 512, 128, 32 if kind else 64]
    assert all(q["sgn"] == "-1" for q in inv[:3])
    assert inv[-1]["kind"] == ("c2r_z" if kind else "contig")
    spec = 512 * 256 * 128 * nc * 8
    assert ws == (2 * spec if kind else spec)


def test_nd_small_axis0_stride_keeps_the_standard_layout():
    passes, ws, _ = nd_only((8, 4, 6, 10))
    fwd = [p for p in passes if p["dir"] == "forward"]
    assert [int(q["L"]) for q in fwd] == [10, 6, 4, 8]
    assert fwd[-1]["es"] == "240/240" and ws == 0


def test_nd_rank3_is_the_3d_plan():
    h = ctypes.c_void_p()
    assert lib.mifft_plan_create_nd(ctypes.byref(h), 3, (ctypes.c_int * 3)(64, 48, 40), 0, 0,
                                    MIFFT_PLAN_ONLY) == 0
    a = plan_describe(h.value)
    plan_destroy(h.value)
    assert lib.mifft_plan_create(ctypes.byref(h), 64, 48, 40, 0, 0, MIFFT_PLAN_ONLY) == 0
    b = plan_describe(h.value)
    plan_destroy(h.value)
    assert a == b
    assert lib.mifft_plan_create_nd(ctypes.byref(h), 1, (ctypes.c_int * 1)(96), 1, 1,
                                    MIFFT_PLAN_ONLY) == 0
    c = plan_describe(h.value)
    plan_destroy(h.value)
    assert "r2c_z" in c and "strided" not in c


@pytest.mark.parametrize("dims", [(512, 256, 128, 64), (2, 3, 4, 5, 6), (1, 1, 1, 1), (8, 1, 1, 6),
                                  (3, 1, 5, 1, 2, 1, 4, 2), (1024, 1024, 2, 1), (16, 16, 16, 1024)])
def test_nd_passes_stay_inside_the_buffers(dims):
    for kind in (0, 1):
        if kind and dims[-1] % 2:
            continue
        for prec in (0, 1):
            nd_only(dims, kind, prec)


@pytest.mark.parametrize("shape", [(512, 512, 512), (64, 48, 32), (1, 32, 64)])
def test_spectral_workspace_is_three_halves(shape):
    """Gradient and divergence keep one spectrum while they build another:
    three half-spectrum buffers, 1.5 x the Poisson workspace."""
    h = ctypes.c_void_p()
    assert lib.mifft_plan_create(ctypes.byref(h), *shape, 1, 0, MIFFT_PLAN_ONLY) == 0
    pws = lib.mifft_poisson_ws_bytes(h.value)
    sws = lib.mifft_spectral_ws_bytes(h.value)
    plan_destroy(h.value)
    assert pws > 0 and sws == pws // 2 * 3


def test_streaming_loads_only_for_whole_aligned_lines():
    """Strided passes read with streaming loads only where every tile covers
    whole, aligned 128-byte lines of the input (512 columns); the 257-column
    half spectrum of R2C 512^3 keeps cached loads."""
    passes, _, _ = plan_only(512, 512, 512, kind=0, prec=0)
    st = [p for p in passes if p["kind"] == "strided"]
    assert st and all(p["nt"] == "1" for p in st)
    passes, _, _ = plan_only(512, 512, 512, kind=1, prec=0)
    fwd = [p for p in passes if p["dir"] == "forward" and p["kind"] == "strided"]
    assert fwd and all(p["nt"] == "0" for p in fwd)

"""Build step of the HIP library: compiles every csrc/*.hip for gfx950 and
links libmifft.so next to this file.

    python -m paper_1506_07933_amd.build        # or build() from Python

Each .hip source becomes one object (the kernel-variant table is compiled in
chunks, once per precision, so the objects build in parallel); the objects
are linked with hipcc into a shared library exporting the C ABI of
include/mifft.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmifft.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
NCHUNK = 4

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          # no packed FP32 instructions anywhere in this library
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


def _jobs():
    jobs = []
    for prec in ("float", "double"):
        for c in range(NCHUNK):
            jobs.append((os.path.join(CSRC, "variants.hip"),
                         os.path.join(OBJDIR, "variants_%s_%d.o" % (prec, c)),
                         ["-DMIFFT_REAL=%s" % prec, "-DMIFFT_CHUNK=%d" % c]))
    for prec in ("float", "double"):
        jobs.append((os.path.join(CSRC, "batch_kern.hip"),
                     os.path.join(OBJDIR, "batch_kern_%s.o" % prec), ["-DMIFFT_REAL=%s" % prec]))
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") and name not in ("variants.hip", "batch_kern.hip"):
            jobs.append((os.path.join(CSRC, name),
                         os.path.join(OBJDIR, name[:-4] + ".o"), []))
    return jobs


def _compile(job):
    src, obj, extra = job
    cmd = [HIPCC] + COMMON + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    return r.returncode, " ".join(cmd), out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    todo = _jobs()
    workers = jobs or min(len(todo), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_compile, todo))
    failed = [r for r in results if r[0] != 0]
    for rc, cmd, out in results:
        if verbose or rc != 0:
            if out:
                sys.stderr.write(out + "\n")
    if failed:
        raise RuntimeError("HIP compilation failed:\n" + "\n".join(c for _, c, _ in failed))
    objs = [o for _, o, _ in todo]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stdout))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

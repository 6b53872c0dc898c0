"""Build the gfx950 HIP library ``libgrmhd.so`` in-tree with hipcc.

The stage kernels of each reconstruction are a translation unit of their own
(``csrc/stage_<recon>.hip``); the units compile in parallel and are linked
into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SRC = [os.path.join(CSRC, f) for f in ("grmhd_capi.hip", "stage_weno5.hip", "stage_wenoz.hip", "stage_wenoz2.hip",
                                      "stage_minmod.hip")]
DEPS = SRC + [os.path.join(CSRC, h) for h in ("grmhd_device.h", "grmhd_adjoint.h", "grmhd_stage.h")] + \
    [os.path.join(ROOT, "include", "grmhd.h")]
LIB = os.path.join(HERE, "libgrmhd.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (their forms are not trusted on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build_hip(force=True, verbose=False, extra_flags=()):
    """Compile libgrmhd.so for gfx950 (always, unless force=False and it is up to date)."""
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    cc = hipcc()
    inc = ["-I" + os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="grmhd_build_") as tmpd:
        objs, procs = [], []
        for src in SRC:
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            objs.append(obj)
            cmd = [cc] + HIPCC_FLAGS + list(extra_flags) + inc + ["-c", src, "-o", obj]
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        errs = []
        for src, p in procs:
            out, err = p.communicate()
            if p.returncode != 0:
                errs.append(f"{os.path.basename(src)}:\n{err[-4000:]}")
            elif verbose and err:
                print(err)
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
        tmp = LIB + ".tmp"
        r = subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_hip())

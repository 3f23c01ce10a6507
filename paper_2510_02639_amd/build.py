"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into libicrs.so (in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libicrs.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 (v_pk_*_f32) instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l)  # host-pass notice about the device-only feature
    return res.returncode, msgs


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Each source compiled to an object in parallel (no device code crosses files: every
    kernel is launched from its own file), then one shared-library link."""
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = [os.path.join(objdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    flags = [a for a in HIPCC_FLAGS if a != "-shared"]
    cmds = [[hipcc, *flags, *inc, "-c", s, "-o", o] for s, o in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, msgs), s in zip(results, srcs):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(s)} ({rc}):\n{msgs}")
        if verbose and msgs.strip():
            print(msgs)
    tmp = LIB + ".tmp"
    rc, msgs = _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    if rc != 0:
        raise RuntimeError(f"hipcc link failed ({rc}):\n{msgs}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Builds libkcore.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkcore.so")
LIB_CHECKED = os.path.join(HERE, "libkcore_checked.so")
ARCH = os.environ.get("KCORE_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: hipcc must not emit packed fp32 instructions on this target.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("not a recognized feature", "ignoring feature")
    err = "\n".join(x for x in r.stderr.splitlines() if not any(s in x for s in noise))
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{err}")
    if err.strip():
        print(err, file=sys.stderr)


def _build_one(lib: str, defines, verbose: bool) -> str:
    from concurrent.futures import ThreadPoolExecutor
    tag = os.path.basename(lib).replace(".so", "")
    cmds, objs = [], []
    for src, hip in (("kcore_device.hip", True), ("kcore_api.cpp", False), ("kcore_server.cpp", False)):
        obj = os.path.join(CSRC, f"{src}.{tag}.o")
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
        if not hip:
            cmd.insert(1, "-xhip")
        if verbose:
            print(" ".join(cmd))
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(len(cmds)) as ex:
        list(ex.map(_run, cmds))
    tmp = lib + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


def build(verbose: bool = False) -> str:
    """Compiles every source (always) and links libkcore.so atomically; then the checked variant
    libkcore_checked.so (run-time invariant checks in the kernels, for tests)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(2) as ex:
        list(ex.map(lambda x: _build_one(x[0], x[1], verbose),
                    ((LIB, []), (LIB_CHECKED, ["-DKCORE_CHECKS=1"]))))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP/C++ library ``libsmpc.so`` for gfx950 in this directory.

``python -m paper_1604_01074_amd.build`` (or ``build()``) always recompiles:
the kernel file three times (float64, float32 and float32-on-float64-dual
instantiations) and the host
sources, in parallel, then one link.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsmpc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-std=c++17", "-O3", "-fPIC",
    "--offload-arch=gfx950",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
LINK_FLAGS = ["-shared", "-fPIC", "--offload-arch=gfx950"]


def _run(cmd: list[str]) -> subprocess.Popen:
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def _output(text: str) -> str:
    return "\n".join(line for line in text.splitlines() if "packed-fp32-ops" not in line)


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (the kernel file three times,
    one part per precision), then link ``libsmpc.so``."""
    inc = ["-I", os.path.join(HERE, "..", "include")]
    tmpdir = tempfile.mkdtemp(prefix="smpc_build_")
    try:
        jobs = []
        for src, defs in (("smpc_kernels.hip", ["-DSMPC_KERNEL_PART=1"]), ("smpc_kernels.hip", ["-DSMPC_KERNEL_PART=2"]),
                          ("smpc_kernels.hip", ["-DSMPC_KERNEL_PART=3"]),
                          ("smpc_data.hip", []), ("smpc_setup.cpp", []), ("smpc_api.cpp", []),
                          ("smpc_server.cpp", []), ("smpc_loop.cpp", [])):
            obj = os.path.join(tmpdir, f"{os.path.splitext(src)[0]}{defs[0][-1] if defs else ''}.o")
            cmd = [HIPCC, *FLAGS, *defs, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((obj, _run(cmd)))
        objs, errors = [], []
        for obj, proc in jobs:
            out, _ = proc.communicate()
            if proc.returncode != 0:
                errors.append(f"hipcc failed ({proc.returncode}) for {obj}:\n{_output(out)}")
            elif verbose and _output(out).strip():
                print(_output(out))
            objs.append(obj)
        if errors:
            raise RuntimeError("\n".join(errors))
        tmp = LIB + ".tmp"
        cmd = [HIPCC, *LINK_FLAGS, *objs, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed ({r.returncode}):\n{_output(r.stdout + r.stderr)}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

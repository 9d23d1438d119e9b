"""Build the lsdm HIP library for gfx950 in-tree (liblsdm.so next to this file)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["csrc/kernels.hip", "csrc/pattern.hip", "csrc/symbolic.cpp", "csrc/api.cpp"]
OUT = os.path.join(HERE, "liblsdm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled for all device code; MFMA accumulators
# are kept in ordinary VGPRs (the accumulation-register form makes the
# compiler copy every accumulator out and back around conditionally issued
# MFMAs)
DEVFLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-mfma-vgpr-form=1"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]


def _compile(src):
    obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + DEVFLAGS + lang + ["-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msg}")
    return obj, msg


def build(verbose: bool = False) -> str:
    with ThreadPoolExecutor(len(SRC)) as ex:
        res = list(ex.map(_compile, SRC))
    for _, msg in res:
        if verbose and msg.strip():
            print(msg)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + DEVFLAGS + ["-shared", "-fPIC", "-o", tmp] + [o for o, _ in res] + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Builds libacse.so (HIP, gfx950) in-tree with hipcc: every translation unit
is compiled to an object in _build/ (in parallel), then linked."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libacse.so")
SOURCES = ["acse_api.hip", "gemm.hip", "gemm_crt.hip", "ny.hip", "spin.hip", "tensor_ops.hip", "vjp.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    return res.returncode, msg


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    workers = max(1, min(len(cmds), len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 4))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(_run, cmds))
    msgs = []
    for src, (rc, msg) in zip(SOURCES, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
        if msg.strip():
            msgs.append(msg)
    tmp = LIB + ".tmp"
    rc, msg = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    if rc != 0:
        raise RuntimeError("hipcc link failed:\n" + msg)
    if verbose and (msgs or msg.strip()):
        print("\n".join(msgs + [msg]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

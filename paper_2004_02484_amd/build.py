"""Build libnmpc.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnmpc.so")
SOURCES = ["nmpc_kernels.hip", "nmpc_gs.hip", "nmpc_ragged.hip", "nmpc_loop.hip", "nmpc_stream.hip",
           "nmpc_runtime.hip", "nmpc_ragged_runtime.hip", "nmpc_net.hip", "nmpc_net_runtime.hip",
           "nmpc_model.hip", "nmpc_model_runtime.hip", "nmpc_net_model.hip"]

# Packed FP32 ops are disabled: code is written for scalar FP32/FP64 VALU.
HIPFLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]
# Per-source additions: the fused stage kernel's and the ragged kernel's
# translation units are scheduled for instruction-level parallelism (two waves
# per SIMD leave little room to hide latency across waves): 531 against 538 us
# per launch on the 64 x 64, N = 40 batch of 256 (no spills), 1.77 against
# 1.79 ms per upper iteration of the 512-instance ragged batch. The other
# units keep the default scheduler (no gain, or slower: the streaming passes;
# the Gauss-Seidel unit does not compile with it).
_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
EXTRA = {"nmpc_kernels.hip": _ILP, "nmpc_ragged.hip": _ILP}


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmds.append([hipcc, *HIPFLAGS, *EXTRA.get(src, []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the translation units compile independently: run them side by side
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for f in [pool.submit(subprocess.check_call, cmd) for cmd in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

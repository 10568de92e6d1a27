"""Build libwave.so (HIP kernels + host runtime + C ABI) for gfx950, in-tree.

Every HIP translation unit is compiled with packed-FP32 instruction selection
disabled (-packed-fp32-ops) and explicit FP contraction; the kernels use fmaf
where a fused multiply-add is intended.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwave.so")
SOURCES = ["wave_kernels.hip", "wave_fused.hip", "wave_api.cpp", "wave_engine.cpp",
           "wave_launch.cpp", "wave_scratch.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=fast",
          "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, lib: str = LIB, defines=()) -> str:
    """Compile and link; defines are extra -D options (tuning switches such as
    WAVE_ZUNROLL_MASK), lib the output path."""
    odir = os.path.dirname(os.path.abspath(lib))
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(odir, src + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmds.append([HIPCC] + COMMON + ["-D" + d for d in defines] + lang
                    + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # translation units compile in parallel (the kernels' unit dominates)
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    failed = [c for c, p in zip(cmds, procs) if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

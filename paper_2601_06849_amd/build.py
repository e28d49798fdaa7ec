"""Compile the HIP library libetdds.so in-tree for gfx950 (hipcc).

The library is one translation unit per mode-product precision
(csrc/kern_*.hip), the C ABI (csrc/etdds.hip) and the host plan
(csrc/plan.cpp); the units compile in parallel into _build/ and are linked
into paper_2601_06849_amd/libetdds.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libetdds.so")
OBJDIR = os.path.join(ROOT, "_build", "etdds")


def sources():
    names = sorted(f for f in os.listdir(CSRC) if f.startswith("kern_") and f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in ["etdds.hip", *names, "plan.cpp"]]


HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed-FP32 instructions are kept out of every device code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    pending = []
    objs = []
    for src in sources():
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        pending.append([hipcc, *HIPCC_FLAGS, *inc, "-c", "-o", obj, src])
    running = []
    failed = None
    while pending or running:
        while pending and len(running) < jobs and failed is None:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            running.append((cmd, subprocess.Popen(cmd)))
        cmd, proc = running.pop(0)
        if proc.wait() != 0 and failed is None:
            failed = cmd
        if failed is not None:
            pending.clear()
    if failed is not None:
        raise subprocess.CalledProcessError(1, failed)
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), file=sys.stderr)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

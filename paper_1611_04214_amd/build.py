"""Build libmolt.so (HIP, gfx950) in-tree.

    python -m paper_1611_04214_amd.build

Every HIP source is compiled with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmolt.so")
ARCH = os.environ.get("MOLT_OFFLOAD_ARCH", "gfx950")

# (source, extra defines): the kernel files compile once per precision (and
# the single-problem kernels once per pass direction), in parallel
SOURCES = [("molt_kernels.hip", ("MOLT_PART_X",)), ("molt_kernels.hip", ("MOLT_PART_Y",)),
           ("molt_kernels.hip", ("MOLT_PART_X", "MOLT_PREC_F64")), ("molt_kernels.hip", ("MOLT_PART_Y", "MOLT_PREC_F64")),
           ("molt_batch.hip", ()), ("molt_batch.hip", ("MOLT_BATCH_F64",)), ("molt_noalloc.hip", ()),
           ("molt_host.cpp", ())]
# -ffp-contract=on: a multiply-add is fused only within one source expression,
# so every kernel that inlines the same device code rounds alike (the batched
# kernels reproduce the single-problem ones bit for bit)
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    objs, procs = [], []
    tag = f".{os.getpid()}.o"
    for k, (src, extra) in enumerate(SOURCES):  # the translation units compile in parallel
        obj = os.path.join(CSRC, f"{src}.{k}{tag}")
        cmd = ["hipcc", "-c"] + FLAGS + [f"-D{d}" for d in tuple(defines) + tuple(extra)] + \
              (["-x", "hip"] if src.endswith(".hip") else []) + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = out + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    for o in objs:
        os.remove(o)
    # every symbol of the library's own namespace must be defined in it
    und = subprocess.run(["nm", "-D", "--undefined-only", tmp], capture_output=True, text=True).stdout
    missing = [ln.split()[-1] for ln in und.splitlines() if "_ZN4molt" in ln or " molt_" in ln]
    if missing:
        os.remove(tmp)
        raise RuntimeError(f"libmolt.so would leave its own symbols undefined: {missing}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "-v"]
    defs = [a[2:] for a in args if a.startswith("-D")]
    outs = [a[len("--out="):] for a in args if a.startswith("--out=")]
    print(build(verbose="-v" in sys.argv, out=outs[0] if outs else LIB, defines=defs))

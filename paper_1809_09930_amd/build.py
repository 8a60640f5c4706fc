"""Build libselfjoin.so (HIP C++ for gfx950) in-tree with hipcc.

    python -m paper_1809_09930_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libselfjoin.so")
SOURCES = ["sj_prims.hip", "sj_index.hip", "sj_join.hip", "sj_mfma.hip", "sj_api.hip", "sj_batch.hip",
           "sj_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for the whole device build.  MFMA
# results are kept in ordinary VGPRs (the epilogue reads every accumulator
# with VALU instructions; AGPR results would need a move per accumulator).
COMMON = ["-x", "hip", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-mfma-vgpr-form=1",
          "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False, lib: str = LIB, build_dir: str = BUILD_DIR,
          defines=()) -> str:
    """Compile every source and link `lib`.  `defines` (e.g. ["SJ_FINE_BITS=3"])
    override the tunable constants of the kernels."""
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    dflags = ["-D" + d for d in defines]

    def compile_one(i):
        src = os.path.join(CSRC, SOURCES[i])
        return _run([HIPCC, *COMMON, *dflags, "-c", src, "-o", objs[i]])

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        outs = list(ex.map(compile_one, range(len(SOURCES))))
    tmp = lib + ".tmp%d" % os.getpid()
    outs.append(_run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]))
    os.replace(tmp, lib)
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

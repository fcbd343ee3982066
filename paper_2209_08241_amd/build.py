"""Build libbnormals.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2209_08241_amd.build

Every kernel translation unit is compiled with contraction off (the
boundary masks are specified as binary32 sequences: the four-pair one
unfused, the fused multiply-adds of the other methods written out as such)
and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbnormals.so")

SOURCES = ["bn_kernels.hip", "bn_batch.hip", "bn_adjoint.hip", "bn_autotune.hip", "bn_serve.hip",
           "bn_eval.hip", "bn_probe.hip", "bn_stack.hip", "bn_workspace.hip", "bn_capi.hip"]
ARCH = os.environ.get("BN_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    # the SLP vectorizer packs the per-pixel validity flags into vector
    # registers and tests them there (about 15 instructions where 5 compares
    # and 4 scalar ANDs do)
    "-fno-slp-vectorize",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every device atomic here is issued by one lane; the wavefront-combining
    # rewrite adds a wait for the atomic's return right after it
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(src: str, obj: str, verbose: bool) -> str:
    cmd = [hipcc(), *HIPCC_FLAGS, "-c", f"-I{INCLUDE}", f"-I{CSRC}", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({res.returncode}):\n{out}")
    return out


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link the library."""
    import concurrent.futures as cf
    import tempfile
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="bn_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            outs = list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(srcs, objs)))
        tmp = LIB + ".tmp"
        link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{res.stdout}")
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)

"""Compile the HIP sources of the package into libpprpa.so for gfx950 (in-tree).

    python -m paper_2512_12515_amd.build        (or build() from Python)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpprpa.so")
SOURCES = ["api.cpp", "davidson.cpp", "server.cpp", "trace.cpp", "k_sigma.hip", "k_sigma_f64.hip", "k_sigma_ab.hip", "k_sigma_bf16.hip", "k_linalg.hip",
           "k_dense.hip", "k_dense_mw.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-Wall",
         "-Wno-unused-function", "-Wno-unused-result",
         # packed FP32 instructions are avoided on this hardware: the compiler must not emit them
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # keep per-thread staging arrays in registers (not promoted into LDS)
         "-mllvm", "-disable-promote-alloca-to-lds"]


def _compile(src, objdir):
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        res = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    objs = [o for o, _ in res]
    if verbose:
        for (_, err), src in zip(res, SOURCES):
            warn = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if warn:
                print(src, "\n".join(warn[:40]), file=sys.stderr)
    tmp = OUT + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp] + objs + ["-ldl"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

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


# Host-sanitized variant for the C-ABI driver test (tests/abi_sanitized.c): the host sources are
# recompiled with AddressSanitizer and UndefinedBehaviorSanitizer on the host pass only (device
# code is unchanged; the kernel objects of build() are reused), linked into
# _build/libpprpa_san.so, and the C driver is linked against it with the sanitizer runtimes.
HOST_SOURCES = ["api.cpp", "davidson.cpp", "server.cpp", "trace.cpp"]
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
CLANG = os.environ.get("PPRPA_CLANG", "/opt/rocm/llvm/bin/clang")
SAN_DRIVER = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed:\n{r.stderr}")


def build_sanitized():
    """Build _build/libpprpa_san.so and the driver _build/abi_sanitized; returns the driver path.
    Needs the kernel objects of build()."""
    objdir = os.path.join(HERE, "_build")
    sandir = os.path.join(objdir, "san")
    os.makedirs(sandir, exist_ok=True)
    dev = [os.path.join(objdir, s + ".o") for s in SOURCES if s not in HOST_SOURCES]
    missing = [o for o in dev if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"run build() first: missing {missing}")

    def host(src):
        obj = os.path.join(sandir, src + ".o")
        _run([HIPCC] + FLAGS + SAN_HOST + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj],
             f"sanitized compile of {src}")
        return obj

    with ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        hobjs = list(ex.map(host, HOST_SOURCES))
    lib = os.path.join(objdir, "libpprpa_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-o", lib] + hobjs + dev + ["-ldl"],
         "sanitized link")
    root = os.path.dirname(HERE)
    dobj = os.path.join(sandir, "abi_sanitized.o")
    _run([CLANG, "-std=c11", "-O1", "-Wall"] + SAN_DRIVER + ["-I", os.path.join(root, "include"), "-c",
          os.path.join(root, "tests", "abi_sanitized.c"), "-o", dobj], "driver compile")
    exe = os.path.join(objdir, "abi_sanitized")
    _run([CLANG + "++"] + SAN_DRIVER + [dobj, "-o", exe, "-L", objdir, "-lpprpa_san",
          "-Wl,-rpath," + objdir, "-lm"], "driver link")
    return exe


if __name__ == "__main__":
    print(build(verbose=True))

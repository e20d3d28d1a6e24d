"""The C-ABI library: exports and argument checks that return before touching a GPU (CPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2512_12515_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "pprpa.h")).read()
    return sorted(set(re.findall(r"^\s*(?:pprpa_status|void|const char\*)\s+(pprpa_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["pprpa_build", "pprpa_matvec", "pprpa_davidson", "pprpa_dims", "pprpa_free",
              "pprpa_dense_matrix", "pprpa_strerror", "pprpa_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_strerror():
    L = B.lib()
    assert L.pprpa_strerror(0) == b"ok"
    assert L.pprpa_strerror(4) == b"not converged"


def _args(**over):
    eps = np.linspace(-1, 1, 6)
    L = np.zeros((3, 6, 6))
    a = B.BuildArgs()
    a.nmo, a.nocc, a.naux = 6, 2, 3
    a.eps = eps.ctypes.data
    a.Lpq = L.ctypes.data
    a.mult, a.prec = 0, 0
    for k, v in over.items():
        setattr(a, k, v)
    return a, eps, L


@pytest.mark.parametrize("over,msg", [
    (dict(nocc=7), "nocc"),
    (dict(nocc=-1), "nocc"),
    (dict(naux=0), "naux"),
    (dict(mult=2), "mult"),
    (dict(prec=9), "prec"),
    (dict(nocc_act=3), "nocc_act"),
    (dict(nvir_act=5), "nvir_act"),
    (dict(nocc=6), "virtual"),
])
def test_build_rejects_invalid_arguments(over, msg):
    a, eps, L = _args(**over)
    h = C.c_void_p(1234)
    st = B.lib().pprpa_build(C.byref(a), C.byref(h))
    assert st == B.EINVAL
    assert h.value is None
    assert msg in B.lib().pprpa_last_error().decode()


def test_build_rejects_non_finite_energies():
    a, eps, L = _args()
    eps[3] = np.nan
    h = C.c_void_p()
    assert B.lib().pprpa_build(C.byref(a), C.byref(h)) == B.EINVAL
    assert "not finite" in B.lib().pprpa_last_error().decode()


@pytest.mark.parametrize("swap,msg", [
    ((0, 1), "occupied block"),   # occupied energies out of order
    ((3, 5), "virtual block"),    # virtual energies out of order
    ((1, 2), "not below"),        # highest occupied above the lowest virtual
])
def test_build_rejects_unordered_energies(swap, msg):
    """The definite shift 2 mu = e_HOMO + e_LUMO and the active window read the energies in
    ascending order within each block: unordered energies are an argument error, not a silent
    wrong shift or window."""
    a, eps, L = _args()
    i, j = swap
    eps[i], eps[j] = eps[j], eps[i]
    h = C.c_void_p(1234)
    assert B.lib().pprpa_build(C.byref(a), C.byref(h)) == B.EINVAL
    assert h.value is None
    assert msg in B.lib().pprpa_last_error().decode()


def test_build_rejects_degenerate_gap():
    a, eps, L = _args()
    eps[2] = eps[1]
    h = C.c_void_p()
    assert B.lib().pprpa_build(C.byref(a), C.byref(h)) == B.EINVAL
    assert "not below" in B.lib().pprpa_last_error().decode()


def test_null_arguments():
    L = B.lib()
    assert L.pprpa_build(None, None) == B.EINVAL
    L.pprpa_free(None)  # NULL-safe
    assert L.pprpa_matvec(None, 1, None, None, 0) == B.EINVAL
    d = B.DavidsonArgs()
    assert L.pprpa_davidson(None, C.byref(d), None, None, None, None) == B.EINVAL


def test_binding_constants_match_header_enums():
    """The binding's status, multiplicity and precision constants equal the header's enum values
    (parsed from include/pprpa.h, so that a renumbering on either side fails here)."""
    text = open(os.path.join(ROOT, "include", "pprpa.h")).read()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(PPRPA_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    for name in ("OK", "EINVAL", "ENOMEM", "EDEVICE", "ENOCONV", "ENONDEF", "EUNSUPPORTED", "EBUSY"):
        assert getattr(B, name) == vals["PPRPA_" + name], name
    assert B.MULT == {"singlet": vals["PPRPA_SINGLET"], "triplet": vals["PPRPA_TRIPLET"]}
    assert B.PREC == {"fp64": vals["PPRPA_FP64"], "fp32": vals["PPRPA_FP32"],
                      "bf16x6": vals["PPRPA_BF16X6"], "bf16x3": vals["PPRPA_BF16X3"]}
    for code in range(8):  # every status has its own message; an unknown code is reported as such
        assert B.lib().pprpa_strerror(code).decode() != "unknown status"
    assert B.lib().pprpa_strerror(8).decode() == "unknown status"
    assert B.lib().pprpa_strerror(-1).decode() == "unknown status"


def test_roctx_ranges_open_when_enabled():
    """PPRPA_ROCTX=1 opens the profiler SDK's roctx library on the first traced entry point;
    with no profiler attached its ranges are no-ops and the call behaves as without them."""
    import subprocess
    import sys
    code = ("import ctypes as C; from paper_2512_12515_amd import binding as B; "
            "L = B.lib(); assert L.pprpa_build(None, None) == B.EINVAL; "
            "assert L.pprpa_matvec(None, 1, None, None, 0) == B.EINVAL; print('ok')")
    env = dict(os.environ, PPRPA_ROCTX="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "could not be opened" not in r.stderr and "lacks" not in r.stderr, r.stderr


def test_server_argument_checks():
    L = B.lib()
    h = C.c_void_p(1234)
    assert L.pprpa_server_create(1 << 30, 0, C.byref(h)) == B.EINVAL
    assert "max_inflight" in L.pprpa_last_error().decode()
    assert L.pprpa_server_create(1 << 30, 65, C.byref(h)) == B.EINVAL
    assert L.pprpa_server_create(1000, 4, C.byref(h)) == B.EINVAL
    assert "1 MiB" in L.pprpa_last_error().decode()
    assert L.pprpa_server_submit(None, None, None, None) == B.EINVAL
    info = B.RequestInfo()
    assert L.pprpa_server_poll(None, 1, C.byref(info), None, None, None) == B.EINVAL
    assert L.pprpa_server_wait(None, 1, 0.0) == B.EINVAL
    st = B.ServingStats()
    assert L.pprpa_server_stats(None, C.byref(st)) == B.EINVAL
    L.pprpa_server_destroy(None)


STRUCTS = [("pprpa_build_args", "BuildArgs"), ("pprpa_davidson_args", "DavidsonArgs"),
           ("pprpa_report", "Report"), ("pprpa_kernel_stats", "KernelStats"),
           ("pprpa_request_info", "RequestInfo"), ("pprpa_serving_stats", "ServingStats"),
           ("pprpa_corr_energy", "CorrEnergy"), ("pprpa_build_ab_args", "BuildAbArgs")]


def test_struct_layouts_match_header(tmp_path):
    """Every field of the header's argument/result structs sits at the same offset in the
    binding's ctypes mirror, and the sizes agree (compiled against include/pprpa.h with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pprpa.h"', "int main(void) {"]
    for cname, pyname in STRUCTS:
        lines.append(f'  printf("{pyname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(B, pyname)._fields_:
            lines.append(f'  printf("{pyname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        pyname, field, val = line.split()
        cls = getattr(B, pyname)
        got = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (pyname, field, got, int(val))



def test_build_ab_rejects_invalid_arguments():
    L = B.lib()
    eps = np.linspace(-1, 1, 6)
    Lq = np.zeros((3, 6, 6))
    for over, msg in [(dict(nocc_a=6), "nocc_a"), (dict(nocc_b=-1), "nocc_b"), (dict(naux=0), "naux"),
                      (dict(eps_b=None), "NULL")]:
        a = B.BuildAbArgs()
        a.nmo, a.nocc_a, a.nocc_b, a.naux = 6, 2, 1, 3
        a.eps_a = a.eps_b = eps.ctypes.data
        a.Lpq_a = a.Lpq_b = Lq.ctypes.data
        for k, v in over.items():
            setattr(a, k, v)
        h = C.c_void_p(1234)
        assert L.pprpa_build_ab(C.byref(a), C.byref(h)) == B.EINVAL
        assert h.value is None
        assert msg in L.pprpa_last_error().decode()

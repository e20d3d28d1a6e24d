"""GPU: the hh channel (two-electron removal roots, the negative-norm solutions of the ppRPA
pencil; the roots nearest the gap, descending), through the C ABI, against the FP64 oracle.

* L = 0: the hh roots are exactly e_i + e_j, highest first (Davidson and direct);
* Davidson hh vs oracle on ragged shapes, both spins, an active window; the Ritz vectors are
  normalised to z^T W z = -1 and satisfy M z = Omega W z to the residual tolerance;
* direct hh (dense pencil) on both pencil paths (n <= 96 in LDS, 96 < n <= 512 in L2);
* the FP64 Davidson workload 20 x 200 x 700 (10 hh roots per spin, tol 1e-6) vs the oracle's
  stored values;
* a served hh request equals the same solve on a context of its own, bit for bit;
* argument checks: unknown channel, more roots than occupied pairs.
Tolerances as in the parity tests: eigenvalues 1e-8 Ha for FP64 at tol 1e-9, 1e-6 Ha at 1e-6.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import pprpa_oracle as O
from workloads import gen
import paper_2512_12515_amd as P

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(seed, nocc, nvir, naux):
    return gen.orbital_energies(seed, nocc, nvir), gen.lpq_full(seed, nocc + nvir, naux)


def dense(eps, L, nocc, mult, **kw):
    sp = O.active_space(eps, L, nocc, **kw)
    A, B, C = O.build_matrices(sp, mult)
    return O.pprpa_matrix(A, B, C), A.shape[0]


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_hh_zero_interaction_closed_form(mult):
    note("hh L = 0", mult)
    nocc, nvir, naux = 6, 8, 5
    eps = gen.orbital_energies(41, nocc, nvir)
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    k = 0 if mult == "singlet" else 1
    eo = eps[:nocc]
    ref = np.sort([eo[i] + eo[j] for i in range(nocc) for j in range(i + k, nocc)])[::-1][:5]
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        r = ctx.davidson(5, block=5, tol=1e-10, channel="hh")
        d = ctx.davidson(5, direct=True, channel="hh")
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-12
    assert np.max(np.abs(d["omega"] - ref)) <= 1e-12


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case,nroot", [((4, 9, 30), 3), ((7, 17, 40), 6), ((12, 25, 60), 8),
                                        ((20, 11, 70), 10)])
def test_hh_davidson_vs_oracle(mult, case, nroot):
    nocc, nvir, naux = case
    note("hh davidson", mult, case)
    eps, L = problem(43, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, nroot, channel="hh")
    M, nvv = dense(eps, L, nocc, mult)
    w = np.r_[np.ones(nvv), -np.ones(M.shape[0] - nvv)]
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-9, vectors=True, channel="hh")
    assert r["status"] == 0
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    assert np.all(np.diff(r["omega"]) <= 1e-12)
    Z = r["vecs"]
    assert np.allclose(np.einsum("i,ji,ji->j", w, Z, Z), -1.0, atol=1e-10)
    res = Z @ M.T - (Z * w[None, :]) * r["omega"][:, None]
    assert np.max(np.linalg.norm(res, axis=1)) <= 1e-8


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_hh_active_window(mult):
    note("hh active window", mult)
    nocc, nvir, naux = 12, 30, 80
    eps, L = problem(44, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 5, nocc_act=6, nvir_act=12, channel="hh")
    with P.PpRPA(eps, L, nocc, mult=mult, nocc_act=6, nvir_act=12) as ctx:
        r = ctx.davidson(5, block=5, tol=1e-9, channel="hh")
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(4, 9, 30), (9, 20, 60), (8, 45, 150)])
def test_hh_direct_vs_oracle(mult, case):
    """(4, 9, 30): n <= 96 (pencil in LDS); (9, 20, 60) and (8, 45, 150): n = 255 / 226 and
    1071 / 1018 (the dense direct pencil on many workgroups)."""
    nocc, nvir, naux = case
    note("hh direct", mult, case)
    eps, L = problem(45, nocc, nvir, naux)
    nroot = 5
    ref = O.solve(eps, L, nocc, mult, nroot, channel="hh")
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        d = ctx.davidson(nroot, direct=True, vectors=True, channel="hh")
    assert np.max(np.abs(d["omega"] - ref)) <= 1e-9
    assert np.all(d["resid"] <= 1e-9)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_hh_full_size_fp64(mult):
    """20 x 200 x 700 (the FP64 Davidson workload), 10 hh roots, block 20, tol 1e-6, vs the
    oracle's dense route-D values."""
    path = os.path.join(GOLD, "davidson_hh_fp64.json")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    gd = json.load(open(path))
    note("hh full", mult)
    eps, L = problem(0, gd["nocc"], gd["nvir"], gd["naux"])
    ref = np.array(gd["roots"][f"0/{mult}"])
    with P.PpRPA(eps, L, gd["nocc"], mult=mult) as ctx:
        r = ctx.davidson(10, block=20, tol=1e-6, channel="hh")
    note("report", r["report"])
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-6
    assert np.all(r["resid"] <= 1e-6)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_hh_most_roots_widest_block(mult):
    """64 hh roots in blocks of 64 (the largest solve the interface takes; n below the subspace
    cap of 256, so the subspace can span the whole space), against the oracle."""
    nocc, nvir, naux = 12, 14, 50
    note("hh 64 roots, block 64", mult)
    eps = gen.orbital_energies(29, nocc, nvir)
    L = gen.lpq_full(29, nocc + nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 64, channel="hh")
    with P.PpRPA(eps, L, nocc, mult=mult, max_block=64) as ctx:
        r = ctx.davidson(64, block=64, tol=1e-8, channel="hh")
    assert r["status"] == 0
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8


def test_hh_served_equals_standalone():
    note("hh served")
    reqs = [(46, 8, 40, "singlet", 5, "hh"), (47, 10, 50, "triplet", 6, "pp"),
            (48, 6, 30, "triplet", 4, "hh")]
    inputs = [problem(s, no, nv, (7 * (no + nv) + 1) // 2) for (s, no, nv, *_r) in reqs]
    with P.Server(2 << 30, 4) as srv:
        tickets = [srv.submit(eps, L, no, nr, mult=m, tol=1e-8, channel=ch)
                   for (eps, L), (_s, no, _nv, m, nr, ch) in zip(inputs, reqs)]
        served = [srv.wait(t, timeout=60.0) for t in tickets]
    for (eps, L), (_s, no, _nv, m, nr, ch), sv in zip(inputs, reqs, served):
        assert sv["status"] == P.binding.OK, sv["message"]
        with P.PpRPA(eps, L, no, mult=m, max_block=64) as ctx:
            r = ctx.davidson(nr, tol=1e-8, channel=ch)
        assert np.array_equal(r["omega"], sv["omega"])
        ref = O.solve(eps, L, no, m, nr, channel=ch)
        assert np.max(np.abs(sv["omega"] - ref)) <= 1e-7


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
def test_hh_reduced_precision_sigma(prec):
    """hh roots with FP32 / BF16-split sigma (FP64 subspace algebra) against the FP64 oracle."""
    note("hh reduced precision", prec)
    nocc, nvir, naux = 14, 30, 90
    eps, L = problem(50, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, "singlet", 6, channel="hh")
    with P.PpRPA(eps, L, nocc, prec=prec) as ctx:
        r = ctx.davidson(6, block=6, tol=1e-6 if prec == "fp32" else 1e-5, channel="hh")
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-6


def test_hh_argument_checks():
    note("hh argument checks")
    eps, L = problem(49, 4, 10, 20)
    with P.PpRPA(eps, L, 4) as ctx:
        assert ctx.n_hh == 10
        with pytest.raises(P.PpRPAError) as e:
            ctx.davidson(11, channel="hh")
        assert e.value.status == P.binding.EINVAL and "n_hh" in str(e.value)
        # a channel value outside {0, 1} set directly in the argument structure
        import ctypes as C
        a = P.binding.DavidsonArgs()
        a.nroot, a.tol, a.channel = 2, 1e-6, 2
        om = np.empty(2)
        st = P.binding.lib().pprpa_davidson(ctx._h, C.byref(a), om.ctypes.data, None, None, None)
        assert st == P.binding.EINVAL
        assert "channel" in P.binding.lib().pprpa_last_error().decode()

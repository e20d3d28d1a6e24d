"""GPU: edge and degenerate cases of the path, against the oracle.

* L = 0: sigma is exactly the pair-energy diagonal (compared bitwise with E z), and the roots
  are exactly the lowest pair energies, degenerate ones included (Davidson and direct);
* degenerate orbital energies with interactions: eigenvalues with multiplicity;
* no occupied orbitals (pp block only), a single pair (nroot = n_pp = 1), one aux function;
* every root of a channel (nroot = n_pp or n_hh), the subspace reaching the whole space;
* more aux functions (70001) than one staging pass takes, from host and device inputs;
* the widest block (64 vectors; FP64 with one aux function, every reduced precision on a
  ragged shape) and a window of one virtual orbital;
* every sigma precision on the smallest and most ragged shapes.
Tolerances as in the parity tests: FP64 sigma 1e-12 relative, eigenvalues 1e-8 Ha (FP64).
"""
import sys

import numpy as np
import pytest

from oracle import pprpa_oracle as O
from workloads import gen
import paper_2512_12515_amd as P

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dense(eps, L, nocc, mult, **kw):
    sp = O.active_space(eps, L, nocc, **kw)
    A, B, C = O.build_matrices(sp, mult)
    return O.pprpa_matrix(A, B, C), A.shape[0]


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_zero_interaction_sigma_is_the_diagonal(mult):
    note("L = 0 sigma", mult)
    nocc, nvir, naux = 4, 11, 7
    eps = gen.orbital_energies(31, nocc, nvir)
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    M, nvv = dense(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        z = gen.random_vectors(8, 3, ctx.n)
        s = ctx.matvec(z)
    assert np.array_equal(s, (np.diag(M)[None, :] * z))


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_zero_interaction_roots_with_degeneracy(mult):
    """Doubly degenerate orbitals make the pair energies degenerate; with L = 0 the pp roots
    are the lowest pair energies exactly, with their multiplicities."""
    note("L = 0 roots", mult)
    nocc, nvir, naux = 4, 10, 5
    eo = np.array([-0.9, -0.7, -0.7, -0.4])
    ev = np.array([0.1, 0.1, 0.3, 0.5, 0.5, 0.8, 1.0, 1.2, 1.2, 2.0])
    eps = np.r_[eo, ev]
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    va, vb = O.pairs(nvir, mult)
    ref = np.sort(ev[va] + ev[vb])[:6]
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        r = ctx.davidson(6, block=6, tol=1e-10)
        d = ctx.davidson(6, direct=True)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-12
    assert np.max(np.abs(d["omega"] - ref)) <= 1e-12


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_degenerate_orbitals_with_interactions(mult):
    note("degenerate orbitals", mult)
    nocc, nvir, naux = 6, 24, 50
    eps = gen.orbital_energies(33, nocc, nvir)
    eps[nocc + 1] = eps[nocc]          # degenerate LUMO
    eps[nocc + 5] = eps[nocc + 4]
    eps[nocc - 2] = eps[nocc - 1]      # degenerate HOMO
    L = gen.lpq_full(33, nocc + nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 8)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        r = ctx.davidson(8, block=8, tol=1e-9)
        d = ctx.davidson(8, direct=True)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    assert np.max(np.abs(d["omega"] - ref)) <= 1e-8


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-7), ("bf16x6", 1e-7)])
def test_no_occupied_orbitals(prec, tol):
    """nocc = 0: only the pp block (A); the shift falls back to e_LUMO - 1."""
    note("nocc = 0", prec)
    nvir, naux = 18, 30
    eps = gen.orbital_energies(34, 0, nvir)
    L = gen.lpq_full(34, nvir, naux)
    M, nvv = dense(eps, L, 0, "singlet")
    assert M.shape[0] == nvv
    ref = O.solve(eps, L, 0, "singlet", 5)
    with P.PpRPA(eps, L, 0, prec=prec) as ctx:
        z = gen.random_vectors(9, 4, ctx.n)
        s = ctx.matvec(z)
        r = ctx.davidson(5, block=5, tol=1e-7)
    sref = (M @ z.T).T
    assert np.max(np.abs(s - sref)) <= tol * np.abs(sref).max()
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-6


@pytest.mark.parametrize("mult,nvir", [("singlet", 1), ("triplet", 2)])
def test_single_pair(mult, nvir):
    """n_pp = 1: the one pp root, Davidson with nroot = n_pp and the direct path."""
    note("single pair", mult)
    nocc, naux = 3, 4
    eps = gen.orbital_energies(35, nocc, nvir)
    L = gen.lpq_full(35, nocc + nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 1)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        assert ctx.n_pp == 1
        r = ctx.davidson(1, tol=1e-10)
        d = ctx.davidson(1, direct=True)
    assert abs(r["omega"][0] - ref[0]) <= 1e-10
    assert abs(d["omega"][0] - ref[0]) <= 1e-10


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("channel", ["pp", "hh"])
def test_every_root_of_a_channel(mult, channel):
    """nroot = the whole channel (n_pp or n_hh) on a tiny problem, where the Davidson subspace
    can reach the whole space: every root of the channel, against the oracle."""
    note("every root of the channel", mult, channel)
    nocc, nvir, naux = 4, 3, 6
    eps = gen.orbital_energies(37, nocc, nvir)
    L = gen.lpq_full(37, nocc + nvir, naux)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        nroot = ctx.n_pp if channel == "pp" else ctx.n - ctx.n_pp
        ref = O.solve(eps, L, nocc, mult, nroot, channel=channel)
        r = ctx.davidson(nroot, tol=1e-9, channel=channel)
    assert r["status"] == 0
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-9


def test_one_aux_function_and_widest_block():
    note("naux = 1, k = 64")
    nocc, nvir, naux = 5, 21, 1
    eps = gen.orbital_energies(36, nocc, nvir)
    L = gen.lpq_full(36, nocc + nvir, naux)
    M, _ = dense(eps, L, nocc, "singlet")
    with P.PpRPA(eps, L, nocc, max_block=64) as ctx:
        z = gen.random_vectors(10, 64, ctx.n)
        s = ctx.matvec(z)
    ref = (M @ z.T).T
    assert np.max(np.abs(s - ref)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-7), ("bf16x6", 1e-7), ("bf16x3", 3e-6)])
def test_widest_block_every_precision(mult, prec, tol):
    """64 vectors in one block in each reduced sigma precision on a ragged shape, against the
    oracle's M z; the last vector alone gives the same product to the same tolerance."""
    note("k = 64", mult, prec)
    nocc, nvir, naux = 5, 21, 30
    eps = gen.orbital_energies(38, nocc, nvir)
    L = gen.lpq_full(38, nocc + nvir, naux)
    M, _ = dense(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, prec=prec, max_block=64) as ctx:
        z = gen.random_vectors(11, 64, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[63])
    ref = (M @ z.T).T
    scale = np.abs(ref).max()
    assert np.max(np.abs(s - ref)) <= tol * scale
    assert np.max(np.abs(s1 - ref[63])) <= tol * scale


_NAUX_CACHE = {}


@pytest.mark.parametrize("inputs", ["host", "device"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-7)])
def test_aux_count_above_65535(inputs, prec, tol):
    """naux = 70001: more aux slices than one staging pass takes (65535), from host and from
    device inputs, against the oracle's M z."""
    note("naux 70001", inputs, prec)
    nocc, nvir, naux = 3, 7, 70001
    eps = gen.orbital_energies(39, nocc, nvir)
    L = gen.lpq_full(39, nocc + nvir, naux) * (1.0 / 16.0)
    if "M" not in _NAUX_CACHE:  # the oracle's matrix once for the four cases (8 s)
        _NAUX_CACHE["M"] = dense(eps, L, nocc, "singlet")[0]
    M = _NAUX_CACHE["M"]
    if inputs == "device":
        import torch
        dev = torch.device("cuda:0")
        e_in, L_in = torch.from_numpy(eps).to(dev), torch.from_numpy(L).to(dev)
    else:
        e_in, L_in = eps, L
    with P.PpRPA(e_in, L_in, nocc, prec=prec) as ctx:
        z = gen.random_vectors(12, 5, ctx.n)
        s = ctx.matvec(z)
    ref = (M @ z.T).T
    assert np.max(np.abs(s - ref)) <= tol * np.abs(ref).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-7), ("bf16x6", 1e-7),
                                      ("bf16x3", 3e-6)])
def test_window_of_one_virtual(prec, tol):
    note("one-virtual window", prec)
    nocc, nvir, naux = 7, 15, 20
    eps = gen.orbital_energies(37, nocc, nvir)
    L = gen.lpq_full(37, nocc + nvir, naux)
    M, nvv = dense(eps, L, nocc, "singlet", nocc_act=3, nvir_act=1)
    assert nvv == 1
    with P.PpRPA(eps, L, nocc, prec=prec, nocc_act=3, nvir_act=1) as ctx:
        z = gen.random_vectors(11, 2, ctx.n)
        s = ctx.matvec(z)
    ref = (M @ z.T).T
    assert np.max(np.abs(s - ref)) <= tol * np.abs(ref).max()

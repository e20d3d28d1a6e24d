"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances:
* FP64 sigma: |sigma_gpu - M z| <= 1e-12 * max(1, max|M z|) elementwise (only the summation
  order differs);
* FP32 sigma: <= 1e-7 * max|M z| on the small shapes (3.5e-8 measured; operands rounded to 24
  bits, sums over naux * nmo terms); on the panel shapes FP32 and BF16x6 <= 6e-7 and BF16x3
  <= 1.5e-5 of the largest sampled entry (2.4e-7, 2.1e-7 and 5.4e-6 measured);
* eigenvalues: <= 1e-6 Ha (the bar of the method's accuracy target); FP64 paths are asserted at
  1e-8 Ha, their measured level being ~1e-12.
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


def oracle_M(eps, L, nocc, mult, **kw):
    sp = O.active_space(eps, L, nocc, **kw)
    A, B, C = O.build_matrices(sp, mult)
    return O.pprpa_matrix(A, B, C), A.shape[0], sp


SIGMA_CASES = [(2, 3, 7), (4, 9, 30), (5, 20, 100), (3, 17, 40), (0, 5, 12), (1, 2, 5),
               (20, 35, 50), (7, 40, 64), (17, 33, 23)]


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", SIGMA_CASES)
def test_sigma_fp64(mult, case):
    nocc, nvir, naux = case
    note("sigma fp64", mult, case)
    eps, L = problem(11, nocc, nvir, naux)
    M, nvv, _ = oracle_M(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        assert (ctx.n_pp, ctx.n) == (nvv, M.shape[0])
        z = gen.random_vectors(3, 5, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[2])
    ref = (M @ z.T).T
    tol = 1e-12 * max(1.0, np.abs(ref).max())
    assert np.max(np.abs(s - ref)) <= tol
    assert np.array_equal(s1, s[2])  # a vector's result does not depend on the block around it


# Virtual blocks of 5, 6 and 7 column tiles (a full four-tile panel, then a narrow one of 1, 2
# or 3 tiles) and occupied blocks of 3, 4 and 5 tiles: every panel shape of the sigma kernels,
# checked on sampled entries (the first and last pairs of each block and random ones) against the
# oracle's row-by-row definition.
PANEL_CASES = [(40, 70, 24), (50, 90, 20), (70, 110, 16)]


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-12), ("fp32", 6e-7), ("bf16x6", 6e-7),
                                       ("bf16x3", 1.5e-5)])
@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", PANEL_CASES)
def test_sigma_panel_mixes(case, mult, prec, rtol):
    nocc, nvir, naux = case
    note("sigma panel mix", prec, mult, case)
    eps, L = problem(13, nocc, nvir, naux)
    sp = O.active_space(eps, L, nocc)
    with P.PpRPA(eps, L, nocc, mult=mult, prec=prec) as ctx:
        nvv, n = ctx.n_pp, ctx.n
        z = gen.random_vectors(6, 3, n)
        s = ctx.matvec(z)
    rng = np.random.default_rng(5)
    rows = np.unique(np.r_[np.arange(4), nvv - 4 + np.arange(4), nvv + np.arange(4),
                           n - 4 + np.arange(4), rng.integers(0, n, 24)])
    for j in range(z.shape[0]):
        ref = O.sigma_rows(sp, mult, rows, z[j])
        assert np.max(np.abs(s[j, rows] - ref)) <= rtol * max(1.0, np.abs(ref).max())


# Shapes for the software-pipelined FP64 kernel (from 20 virtual 16-tiles on) and the wide-panel
# BF16x6 kernel (virtual blocks of 32 tiles and more in full 8-tile panels): a ragged last
# virtual panel (FP64: 21 tiles = 5 x 4 + 1, 25 = 6 x 4 + 1), a virtual block longer than one
# unit's 32 row tiles (FP64 35 tiles: row ranges of 32 + 3 and a three-tile panel; BF16 at 630
# virtual orbitals: 40 tiles, 32 + 8), occupied blocks of 3 and 5 tiles (FP64) or 4 and 6 (BF16,
# padded to 32 orbitals), and units that walk several aux indices (20 vectors at naux 120:
# dozens of aux splits of 2-3 indices). The BF16x3 kernel and the BF16x6 kernel elsewhere (22,
# 26 and 36 tiles) run on the same shapes. Sampled entries against the oracle's rows.
PIPE_CASES = [((40, 330, 120), 20), ((70, 560, 12), 3), ((40, 500, 120), 20), ((70, 630, 12), 3),
              ((40, 400, 24), 3)]


# (BF16x6 is held to 1e-6 here, the full-size gate: these vectors are longer (nmo 370-630) than
# the panel shapes' and FP32 accumulation sets the level, 6.6e-7 measured at 40/330/120.)
@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-12), ("bf16x6", 1e-6), ("bf16x3", 1.5e-5)])
@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case,k", PIPE_CASES)
def test_sigma_pipelined_shapes(case, k, mult, prec, rtol):
    nocc, nvir, naux = case
    note("sigma pipelined shapes", prec, mult, case, k)
    eps, L = problem(14, nocc, nvir, naux)
    sp = O.active_space(eps, L, nocc)
    with P.PpRPA(eps, L, nocc, mult=mult, prec=prec) as ctx:
        nvv, n = ctx.n_pp, ctx.n
        z = gen.random_vectors(8, k, n)
        s = ctx.matvec(z)
    rng = np.random.default_rng(6)
    rows = np.unique(np.r_[np.arange(3), nvv - 3 + np.arange(3), nvv + np.arange(3),
                           n - 3 + np.arange(3), rng.integers(0, n, 16)])
    for j in sorted({0, k - 1}):
        ref = O.sigma_rows(sp, mult, rows, z[j])
        err = np.max(np.abs(s[j, rows] - ref)) / max(1.0, np.abs(ref).max())
        note("vector", j, "relative error", err)
        assert err <= rtol


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(4, 9, 30), (5, 20, 100), (20, 35, 50), (17, 33, 23)])
def test_sigma_fp32(mult, case):
    nocc, nvir, naux = case
    note("sigma fp32", mult, case)
    eps, L = problem(12, nocc, nvir, naux)
    M, nvv, _ = oracle_M(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, prec="fp32") as ctx:
        z = gen.random_vectors(4, 7, ctx.n)
        s = ctx.matvec(z)
    ref = (M @ z.T).T
    err = np.max(np.abs(s - ref)) / np.abs(ref).max()
    note("relative error", err)
    assert err <= 1e-7, err


def test_sigma_block_sizes_and_repeat_bitwise():
    """Blocks of 1..40 vectors (above the context's 32-vector cap) give the same sigma, and a
    repeated call is bitwise identical."""
    note("sigma blocks")
    eps, L = problem(13, 6, 30, 45)
    M, _, _ = oracle_M(eps, L, 6, "singlet")
    with P.PpRPA(eps, L, 6, max_block=32) as ctx:
        z = gen.random_vectors(5, 40, ctx.n)
        full = ctx.matvec(z)
        again = ctx.matvec(z)
        assert np.array_equal(full, again)
        for k in (1, 7, 33):
            assert np.allclose(ctx.matvec(z[:k]), full[:k], rtol=0, atol=1e-12)
    ref = (M @ z.T).T
    assert np.max(np.abs(full - ref)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_sigma_active_window(mult):
    nocc, nvir, naux, no, nv = 9, 45, 60, 4, 21
    note("active window", mult)
    eps, L = problem(14, nocc, nvir, naux)
    M, _, _ = oracle_M(eps, L, nocc, mult, nocc_act=no, nvir_act=nv)
    La = gen.lpq_active(14, nocc, nvir, naux, no, nv)
    with P.PpRPA(eps, L, nocc, mult=mult, nocc_act=no, nvir_act=nv) as c1, \
            P.PpRPA(eps, La, nocc, mult=mult, nocc_act=no, nvir_act=nv, lpq_is_active=True) as c2:
        z = gen.random_vectors(6, 3, c1.n)
        s1, s2 = c1.matvec(z), c2.matvec(z)
    ref = (M @ z.T).T
    assert np.array_equal(s1, s2)
    assert np.max(np.abs(s1 - ref)) <= 1e-12 * np.abs(ref).max()


def test_device_pointers():
    import torch
    note("device pointers")
    eps, L = problem(15, 5, 20, 100)
    M, _, _ = oracle_M(eps, L, 5, "singlet")
    dev = torch.device("cuda:0")
    te, tL = torch.from_numpy(eps).to(dev), torch.from_numpy(L).to(dev)
    with P.PpRPA(te, tL, 5) as ctx:
        z = gen.random_vectors(7, 4, ctx.n)
        tz = torch.from_numpy(z).to(dev)
        ts = ctx.matvec(tz)
        torch.cuda.synchronize()
        s = ts.cpu().numpy()
    ref = (M @ z.T).T
    assert np.max(np.abs(s - ref)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(5, 20, 100), (3, 17, 40), (0, 6, 10)])
def test_dense_build(mult, case):
    nocc, nvir, naux = case
    note("dense", mult, case)
    eps, L = problem(16, nocc, nvir, naux)
    M, _, _ = oracle_M(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True, prec="fp32") as ctx:
        Md = ctx.dense_matrix()
    assert np.max(np.abs(Md - M)) <= 1e-13 * max(1.0, np.abs(M).max())


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_direct_small(mult, seed):
    """Dense build + direct diagonalisation on the device, 5 x 20 x 100, vs the oracle."""
    note("direct", mult, seed)
    gd = _golden("small_direct.json")
    eps, L = problem(seed, gd["nocc"], gd["nvir"], gd["naux"])
    ref = np.array(gd["roots"][f"{seed}/{mult}"])
    with P.PpRPA(eps, L, gd["nocc"], mult=mult, dense=True) as ctx:
        r = ctx.davidson(5, direct=True, vectors=True)
        M = ctx.dense_matrix()
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    w = np.r_[np.ones(ctx.n_pp), -np.ones(ctx.n_hh)]
    Z = r["vecs"]
    assert np.allclose(np.einsum("ij,j,ij->i", Z, w, Z), 1.0, atol=1e-10)
    res = M @ Z.T - (w[:, None] * Z.T) * r["omega"][None, :]
    assert np.max(np.abs(res)) < 1e-9
    # same vectors as the oracle (non-degenerate roots; sign fixed by the largest component)
    om, zo = O.solve(eps, L, gd["nocc"], mult, 5, vectors=True)
    assert np.allclose(Z, zo.T, atol=1e-8)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case,nroot", [((8, 30, 60), 8), ((6, 14, 40), 5), ((2, 13, 30), 3),
                                        ((8, 45, 150), 6), ((8, 62, 150), 6), ((8, 72, 120), 4)])
def test_direct_orders(mult, case, nroot):
    """The direct dense path at orders from below the 96 of the LDS-resident solver (n = 94 / 79
    for 2 x 13) to the many-workgroup one above it (501 / 463 for 8 x 30, 1071 / 1018 for 8 x 45,
    1989 / 1919 for 8 x 62, 2664 / 2584 for 8 x 72): eigenvalues, residuals, normalisation."""
    nocc, nvir, naux = case
    note("direct orders", mult, case)
    eps, L = problem(21, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, nroot)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        r = ctx.davidson(nroot, direct=True, vectors=True)
        M = ctx.dense_matrix()
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    w = np.r_[np.ones(ctx.n_pp), -np.ones(ctx.n_hh)]
    Z = r["vecs"]
    assert np.allclose(np.einsum("ij,j,ij->i", Z, w, Z), 1.0, atol=1e-10)
    assert np.max(np.abs(M @ Z.T - (w[:, None] * Z.T) * r["omega"][None, :])) < 1e-9


def test_direct_at_the_order_limit():
    """The direct dense solve near its order limit (n = 8183 of 8192), where an oracle
    eigensolve is too slow for a test: the dense matrix on sampled rows against the oracle's
    elements (its sigma rows of the returned vectors), then what holds at any size: residual and
    normalisation of every returned vector, and the same roots from a Davidson solve of the
    density-fitted product on the same context; the correlation energy's two sum-rule sides at
    the same order."""
    nocc, nvir, naux = 10, 127, 400
    note("direct near the order limit")
    eps, L = problem(67, nocc, nvir, naux)
    sp = O.active_space(eps, L, nocc)
    with P.PpRPA(eps, L, nocc, dense=True, max_block=16) as ctx:
        assert 8100 < ctx.n <= 8192
        r = ctx.davidson(5, direct=True, vectors=True)
        dv = ctx.davidson(5, block=10, tol=1e-8)
        ec = ctx.correlation_energy()
        M = ctx.dense_matrix()
    # the whole-spectrum energy at the same order: both sides of the sum rule agree
    assert abs(ec["ec_pp"] - ec["ec_hh"]) <= 1e-9 * max(1.0, abs(ec["ec_pp"]))
    Z = r["vecs"]
    rows = np.linspace(0, ctx.n - 1, 24).astype(int)
    for j in range(5):
        ref = O.sigma_rows(sp, "singlet", rows, Z[j])
        assert np.max(np.abs(M[rows] @ Z[j] - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
    w = np.r_[np.ones(ctx.n_pp), -np.ones(ctx.n_hh)]
    assert np.allclose(np.einsum("ij,j,ij->i", Z, w, Z), 1.0, atol=1e-10)
    assert np.max(np.abs(M @ Z.T - (w[:, None] * Z.T) * r["omega"][None, :])) < 1e-8
    assert np.max(np.abs(r["omega"] - dv["omega"])) <= 1e-8


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case,nroot", [((4, 9, 30), 3), ((3, 17, 40), 6), ((0, 8, 20), 4),
                                        ((12, 25, 60), 8)])
def test_davidson_small(mult, case, nroot):
    nocc, nvir, naux = case
    note("davidson small", mult, case)
    eps, L = problem(17, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, nroot)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-8, vectors=True)
    assert r["status"] == 0
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    assert np.all(r["resid"] <= 1e-8)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_davidson_most_roots_widest_block(mult):
    """The largest solve the interface takes: 64 roots in blocks of 64, so the subspace grows to
    its cap of 256 and the projected pencil runs on its L2-resident path (order > 96)."""
    nocc, nvir, naux = 6, 30, 60
    note("davidson 64 roots, block 64", mult)
    eps, L = problem(23, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 64)
    M, nvv, _ = oracle_M(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, max_block=64) as ctx:
        r = ctx.davidson(64, block=64, tol=1e-8, vectors=True)
    assert r["status"] == 0 and r["report"]["iters"] >= 2
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    Z = r["vecs"]
    w = np.r_[np.ones(nvv), -np.ones(M.shape[0] - nvv)]
    assert np.allclose(np.einsum("ij,j,ij->i", Z, w, Z), 1.0, atol=1e-9)
    assert np.max(np.abs(M @ Z.T - (w[:, None] * Z.T) * r["omega"][None, :])) < 1e-7


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("block,max_subspace", [(1, 0), (1, 20), (2, 20), (3, 15), (5, 15)])
def test_davidson_small_blocks_and_restarts(mult, block, max_subspace):
    """Fewer corrections per iteration than roots, and subspace caps that force restarts every
    few iterations: the oracle's roots all the same."""
    nocc, nvir, naux = 6, 20, 60
    note("davidson block", block, "max_subspace", max_subspace, mult)
    eps, L = problem(19, nocc, nvir, naux)
    ref = O.solve(eps, L, nocc, mult, 5)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        r = ctx.davidson(5, block=block, tol=1e-8, max_iter=600, max_subspace=max_subspace)
    note("iterations", r["report"]["iters"], "final subspace", r["report"]["subspace"])
    assert r["status"] == 0
    assert max_subspace == 0 or r["report"]["subspace"] <= max_subspace
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8


def test_davidson_stalled_by_a_tight_cap_reports_enoconv():
    """A subspace cap barely above nroot with one correction per iteration stalls on this singlet
    problem (each restart to the five Ritz vectors discards what the corrections added): the
    solve reports ENOCONV with its last iterate, finite and not claimed converged."""
    eps, L = problem(19, 6, 20, 60)
    with P.PpRPA(eps, L, 6) as ctx:
        r = ctx.davidson(5, block=1, tol=1e-8, max_iter=60, max_subspace=7, raise_noconv=False)
        with pytest.raises(P.PpRPAError) as e:
            ctx.davidson(5, block=1, tol=1e-8, max_iter=60, max_subspace=7)
    assert r["status"] == P.binding.ENOCONV and e.value.status == P.binding.ENOCONV
    assert np.all(np.isfinite(r["omega"])) and np.all(np.isfinite(r["resid"]))
    assert r["report"]["max_resid"] > 1e-8 and r["report"]["n_conv"] < 5


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("seed", [0, 3])
def test_davidson_vs_direct_small_config(mult, seed):
    gd = _golden("small_direct.json")
    note("davidson cfg small", mult, seed)
    eps, L = problem(seed, gd["nocc"], gd["nvir"], gd["naux"])
    ref = np.array(gd["roots"][f"{seed}/{mult}"])
    with P.PpRPA(eps, L, gd["nocc"], mult=mult) as ctx:
        r = ctx.davidson(5, block=5, tol=1e-7)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_davidson_full_size_fp64(mult):
    """20 x 200 x 700, 10 roots, block 20, tol 1e-6 (the FP64 Davidson workload) vs the
    oracle's dense route-D eigenvalues."""
    path = os.path.join(GOLD, "davidson_fp64.json")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    gd = _golden("davidson_fp64.json")
    note("davidson full", mult)
    eps, L = problem(0, gd["nocc"], gd["nvir"], gd["naux"])
    ref = np.array(gd["roots"][f"0/{mult}"])
    with P.PpRPA(eps, L, gd["nocc"], mult=mult) as ctx:
        r = ctx.davidson(10, block=20, tol=1e-6)
    note("iters", r["report"])
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-6
    assert np.all(r["resid"] <= 1e-6)


def test_failure_paths():
    note("failure paths")
    eps, L = problem(18, 4, 12, 20)
    with P.PpRPA(eps, L, 4) as ctx:
        r = ctx.davidson(4, block=4, tol=1e-14, max_iter=1, raise_noconv=False)
        assert r["status"] == P.binding.ENOCONV
        assert np.all(np.isfinite(r["omega"])) and r["report"]["iters"] == 1
        with pytest.raises(P.PpRPAError) as e:
            ctx.davidson(2, direct=True)
        assert e.value.status == P.binding.EUNSUPPORTED
        with pytest.raises(P.PpRPAError) as e:
            ctx.davidson(ctx.n_pp + 1)
        assert e.value.status == P.binding.EINVAL
    bad = L.copy()
    bad[3, 2, 5] = np.inf
    with pytest.raises(P.PpRPAError) as e:
        P.PpRPA(eps, bad, 4)
    assert e.value.status == P.binding.EINVAL


@pytest.mark.parametrize("case", [(4, 10, 30), (8, 30, 60), (8, 45, 150)])
def test_non_definite_is_reported(case):
    """Interactions scaled far beyond the orbital gap make M - 2 mu W indefinite: the dense
    path must report ENONDEF, never return silently (order 65: the LDS-resident solver; 501
    and 1071: the many-workgroup one)."""
    nocc, nvir, naux = case
    note("non-definite", case)
    eps, L = problem(19, nocc, nvir, naux)
    with P.PpRPA(eps, L * 30.0, nocc, dense=True) as ctx:
        with pytest.raises(P.PpRPAError) as e:
            ctx.davidson(3, direct=True)
    assert e.value.status == P.binding.ENONDEF


def test_concurrent_solves_match_serial():
    """Solves on several contexts from several host threads (each context on its own stream;
    their sandwich launches ordered on the device) give bitwise the roots of the same solves run
    one after the other."""
    from concurrent.futures import ThreadPoolExecutor
    note("concurrent solves")
    probs = [(81, 6, 30, 60, "singlet"), (82, 8, 25, 70, "triplet"), (83, 5, 40, 50, "singlet"),
             (84, 7, 33, 64, "triplet")]
    inputs = [problem(s, no, nv, na) for (s, no, nv, na, _m) in probs]

    def solve(i):
        eps, L = inputs[i]
        with P.PpRPA(eps, L, probs[i][1], mult=probs[i][4]) as ctx:
            return ctx.davidson(6, block=6, tol=1e-9)["omega"]

    serial = [solve(i) for i in range(len(probs))]
    with ThreadPoolExecutor(max_workers=len(probs)) as ex:
        conc = list(ex.map(solve, range(len(probs))))
    for a, b in zip(serial, conc):
        assert np.array_equal(a, b)

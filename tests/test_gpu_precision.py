"""GPU: the precision pattern and the large workloads.

* sigma at full size (50 occ / 500 vir / 1800 aux and the 40 + 400 window of 120 / 1500 / 4000)
  against oracle rows computed one by one from the integrals of those rows only;
* BF16-split sigma (six and three products) against the oracle's dense M z on small and ragged
  problems;
* FP32- and BF16x6-sigma Davidson against the oracle on small problems and against the FP64 GPU
  Davidson at full size, per root, within 1e-6 Ha (the integrals scaled by eig_scale = 0.7 at
  full size, where the unscaled inputs give complex roots; see workloads/gen.py).

Tolerances, relative to max|sigma| (measured on the MI355X, then frozen at about 2.5x the
largest value seen in each group; the values are deterministic: seeded inputs, fixed reduction
order):

  group                                  FP32     BF16x6   BF16x3   (measured max: FP32 / x6 / x3)
  small ragged shapes vs dense M z       1e-7     1e-7     3e-6     3.5e-8 / 3.8e-8 / 1.2e-6
  full size, sampled rows                1e-6     1e-6     5e-6     5.3e-7 / 4.2e-7 / 1.9e-6

FP64 is held to 1e-12. BF16x6 carries each operand to ~24 bits, so it lands where FP32 does
(both accumulate in FP32 over naux * nmo terms); BF16x3 drops the mid*mid, hi*lo and lo*hi
products (each ~2^-16 of a product). On the small shapes, where the FP32 accumulation error is
small, six products are 28-120x more accurate than three (test_bf16x6_beats_bf16x3): a kernel that
ran three products where six are asked for fails that test and the 1e-7 gate, and one that ran
the hi*hi product alone (~2e-4) fails the BF16x3 gate. Eigenvalues 1e-6 Ha.
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


def device_lpq(seed, nocc, nvir, naux, nocc_act=None, nvir_act=None, scale=1.0):
    import torch
    dev = torch.device("cuda:0")
    idx = gen.active_indices(nocc, nvir, nocc_act, nvir_act)
    out = torch.empty((naux, idx.size, idx.size), dtype=torch.float64, device=dev)
    for p0 in range(0, naux, 256):
        aux = np.arange(p0, min(naux, p0 + 256))
        out[p0:p0 + aux.size] = gen.lpq_block_torch(seed, nocc + nvir, naux, idx, idx, aux, dev) * scale
    return out


def oracle_sigma_rows(seed, nocc, nvir, naux, mult, rows, z, nocc_act=None, nvir_act=None):
    """sigma[rows] from the definition, generating only the integral rows each entry needs."""
    eps = gen.orbital_energies(seed, nocc, nvir)
    idx = gen.active_indices(nocc, nvir, nocc_act, nvir_act)
    no = idx.size - (min(nvir_act, nvir) if nvir_act else nvir)
    occ, vir = idx[:no], idx[no:]
    eo, ev = eps[occ], eps[vir]
    nv = vir.size
    s = 1.0 if mult == "singlet" else -1.0
    va, vb = O.pairs(nv, mult)
    oi, oj = O.pairs(no, mult)
    nva, noo = O.pair_norm(va, vb, mult), O.pair_norm(oi, oj, mult)
    nvv = va.size
    x, y = z[:nvv], z[nvv:]
    out = []
    for r in rows:
        if r < nvv:
            p, q = vir[va[r]], vir[vb[r]]
            Lr_v = gen.lpq_block(seed, nocc + nvir, naux, [p, q], vir)
            Lr_o = gen.lpq_block(seed, nocc + nvir, naux, [p, q], occ)
            Arow = O.pair_integrals(Lr_v, np.array([0]), np.array([1]), va, vb, s)[0] * nva[r] * nva
            Brow = O.pair_integrals(Lr_o, np.array([0]), np.array([1]), oi, oj, s)[0] * nva[r] * noo
            out.append((ev[va[r]] + ev[vb[r]]) * x[r] + Arow @ x + Brow @ y)
        else:
            t = r - nvv
            p, q = occ[oi[t]], occ[oj[t]]
            Lr_v = gen.lpq_block(seed, nocc + nvir, naux, [p, q], vir)
            Lr_o = gen.lpq_block(seed, nocc + nvir, naux, [p, q], occ)
            BTrow = O.pair_integrals(Lr_v, np.array([0]), np.array([1]), va, vb, s)[0] * noo[t] * nva
            Crow = O.pair_integrals(Lr_o, np.array([0]), np.array([1]), oi, oj, s)[0] * noo[t] * noo
            out.append(BTrow @ x + Crow @ y - (eo[oi[t]] + eo[oj[t]]) * y[t])
    return np.array(out)


BIG = {
    "mixed": dict(nocc=50, nvir=500, naux=1800, nocc_act=None, nvir_act=None, mult="singlet"),
    "active": dict(nocc=120, nvir=1500, naux=4000, nocc_act=40, nvir_act=400, mult="triplet"),
}


TOL_SMALL = {"fp64": 1e-12, "fp32": 1e-7, "bf16x6": 1e-7, "bf16x3": 3e-6}
TOL_FULL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 5e-6}


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(4, 9, 30), (5, 20, 100), (20, 35, 50), (17, 33, 23), (1, 2, 5),
                                  (7, 40, 64), (0, 5, 12)])
def test_sigma_bf16_vs_oracle(prec, mult, case):
    nocc, nvir, naux = case
    note("sigma", prec, mult, case)
    eps, L = gen.orbital_energies(12, nocc, nvir), gen.lpq_full(12, nocc + nvir, naux)
    sp = O.active_space(eps, L, nocc)
    M = O.pprpa_matrix(*O.build_matrices(sp, mult))
    with P.PpRPA(eps, L, nocc, mult=mult, prec=prec) as ctx:
        z = gen.random_vectors(4, 7, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[3])
    ref = (M @ z.T).T
    err = np.max(np.abs(s - ref)) / np.abs(ref).max()
    note("relative error", err)
    assert err <= TOL_SMALL[prec], err
    assert np.array_equal(s1, s[3])


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_bf16x6_beats_bf16x3(mult):
    """The two BF16 schemes on the same inputs: the six-product sigma must be at least 20 times
    more accurate than the three-product one (measured 28-120x on these shapes), which tells
    the arithmetic that ran apart from a silent fallback to three products."""
    err = {}
    for case in [(4, 9, 30), (5, 20, 100), (3, 17, 40), (0, 5, 12)]:
        nocc, nvir, naux = case
        eps, L = gen.orbital_energies(12, nocc, nvir), gen.lpq_full(12, nocc + nvir, naux)
        M = O.pprpa_matrix(*O.build_matrices(O.active_space(eps, L, nocc), mult))
        for prec in ("bf16x6", "bf16x3"):
            with P.PpRPA(eps, L, nocc, mult=mult, prec=prec) as ctx:
                z = gen.random_vectors(4, 7, ctx.n)
                s = ctx.matvec(z)
            ref = (M @ z.T).T
            err[case, prec] = np.max(np.abs(s - ref)) / np.abs(ref).max()
        note(mult, case, "x6 %.2e x3 %.2e" % (err[case, "bf16x6"], err[case, "bf16x3"]))
        assert err[case, "bf16x6"] <= err[case, "bf16x3"] / 20.0
        assert err[case, "bf16x3"] >= 2e-8  # three products really dropped the small terms


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("name", ["mixed", "active"])
def test_sigma_full_size_sampled_rows(name, prec):
    tol = TOL_FULL[prec]
    import torch
    c = BIG[name]
    note("sigma full size", name, prec)
    eps = gen.orbital_energies(0, c["nocc"], c["nvir"])
    Ld = device_lpq(0, c["nocc"], c["nvir"], c["naux"], c["nocc_act"], c["nvir_act"])
    with P.PpRPA(torch.from_numpy(eps).cuda(), Ld, c["nocc"], mult=c["mult"], prec=prec,
                 nocc_act=c["nocc_act"] or 0, nvir_act=c["nvir_act"] or 0,
                 lpq_is_active=c["nocc_act"] is not None) as ctx:
        del Ld
        z = gen.random_vectors(21, 2, ctx.n)
        s = ctx.matvec(z)
        npp, n = ctx.n_pp, ctx.n
    rng = np.random.default_rng(5)
    rows = np.unique(np.r_[0, 1, npp - 1, npp, n - 1, rng.integers(0, npp, 6), rng.integers(npp, n, 3)])
    for v in range(2):
        ref = oracle_sigma_rows(0, c["nocc"], c["nvir"], c["naux"], c["mult"], rows, z[v],
                                c["nocc_act"], c["nvir_act"])
        scale = np.abs(s[v]).max()
        err = np.max(np.abs(s[v][rows] - ref)) / scale
        note("relative error", err)
        assert err <= tol


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case,nroot", [((6, 40, 90), 6), ((10, 60, 150), 8)])
def test_mixed_precision_davidson_vs_oracle(prec, mult, case, nroot):
    nocc, nvir, naux = case
    note(prec, "davidson small", mult, case)
    eps, L = gen.orbital_energies(3, nocc, nvir), gen.lpq_full(3, nocc + nvir, naux)
    ref = O.solve(eps, L, nocc, mult, nroot)
    with P.PpRPA(eps, L, nocc, mult=mult, prec=prec) as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-6)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-6


@pytest.mark.parametrize("name,nroot", [("mixed", 20), ("active", 16)])
def test_mixed_vs_fp64_davidson_full_size(name, nroot):
    """Per-root FP32- and BF16x6-sigma eigenvalues against the FP64 GPU Davidson on the same
    inputs."""
    import torch
    c = BIG[name]
    scale = gen.CONFIGS[name]["eig_scale"]
    note("fp32 vs fp64 full size", name)
    eps = torch.from_numpy(gen.orbital_energies(0, c["nocc"], c["nvir"])).cuda()
    Ld = device_lpq(0, c["nocc"], c["nvir"], c["naux"], c["nocc_act"], c["nvir_act"], scale=scale)
    kw = dict(mult=c["mult"], nocc_act=c["nocc_act"] or 0, nvir_act=c["nvir_act"] or 0,
              lpq_is_active=c["nocc_act"] is not None, max_block=20)
    out = {}
    # BF16x6 sigma leaves a residual floor just above 1e-6 at these sizes (1.3e-6 measured), so
    # it converges to 1e-5; the eigenvalue error, quadratic in the residual, is unaffected
    for prec, tol in (("fp64", 1e-6), ("fp32", 1e-6), ("bf16x6", 1e-5)):
        with P.PpRPA(eps, Ld, c["nocc"], prec=prec, **kw) as ctx:
            r = ctx.davidson(nroot, block=20, tol=tol, max_iter=300)
        note(prec, r["report"])
        out[prec] = r["omega"]
    for prec in ("fp32", "bf16x6"):
        err = np.abs(out[prec] - out["fp64"])
        note(prec, "per-root |dOmega| (Ha):", err)
        assert np.all(err <= 1e-6)

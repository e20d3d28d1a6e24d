"""GPU: spin-unrestricted ppRPA (three spin sectors), through the C ABI, against the FP64 oracle.

* the alpha-beta sector as a dense context: its matrix, direct and Davidson roots in both
  channels, sigma = M z and the correlation energy against the oracle's alpha-beta sector;
* alpha = beta: the alpha-beta roots are the singlet and triplet roots together;
* alpha != beta end to end: the lowest pp roots of the three GPU sectors (alpha-alpha and
  beta-beta as triplet contexts of one spin's data) equal the lowest pp roots of the oracle's
  general spin-orbital build;
* argument checks;
* the density-fitted alpha-beta sector (Q = sum_P La^P Z Lb^P on the rectangular amplitude
  blocks): sigma against the oracle's M z at ragged shapes and against the dense context, the
  Davidson roots of both channels against the oracle, a sector of order 33120 (beyond the dense
  limit, which is refused) on sampled rows of the oracle, and the dense-only calls refused;
* NTO weights and spin-resolved two-electron densities of alpha-beta roots (rectangular
  amplitude blocks) against the oracle's, with their sum rules;
* the density-fitted alpha-beta sector with FP32 and BF16-split sigma: sigma against the
  oracle's M z at the same shapes and on sampled rows at order 33120, six BF16 products at least
  20x more accurate than three on the same inputs, roots of both channels against the oracle.
Tolerances: matrices and sigma 1e-12 relative, eigenvalues 1e-9 Ha (FP64, tol 1e-10); FP32
sigma 2e-7 relative to max|M z| on the small shapes, 1e-6 at order 33120 (the level of FP32
operands and accumulation, as for the restricted FP32 kernel); BF16x6 / BF16x3 sigma 1e-7 /
2.5e-6 on the small shapes (TOL_AB_BF16), BF16x6 1e-6 at order 33120; reduced-precision roots
1e-6 Ha.
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


def unrestricted(seed, nmo, nocc_a, nocc_b, naux):
    return (gen.orbital_energies(seed, nocc_a, nmo - nocc_a),
            gen.orbital_energies(seed + 1000, nocc_b, nmo - nocc_b),
            gen.lpq_full(seed, nmo, naux), gen.lpq_full(seed + 1000, nmo, naux))


@pytest.mark.parametrize("case", [(8, 3, 2, 20), (12, 5, 5, 40), (16, 4, 6, 50)])
def test_ab_matrix_sigma_and_direct(case):
    nmo, noa, nob, naux = case
    note("ab dense", case)
    ea, eb, La, Lb = unrestricted(71, nmo, noa, nob, naux)
    Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        assert ctx.n_pp == nvv and ctx.n == Mref.shape[0]
        M = ctx.dense_matrix()
        z = gen.random_vectors(72, 5, ctx.n)
        s = ctx.matvec(z)
        if ctx.n <= 512:
            d = ctx.davidson(4, direct=True)
            dh = ctx.davidson(3, direct=True, channel="hh")
    assert np.max(np.abs(M - Mref)) <= 1e-12 * np.abs(Mref).max()
    sref = z @ Mref.T
    assert np.max(np.abs(s - sref)) <= 1e-12 * np.abs(sref).max()
    if Mref.shape[0] <= 512:
        assert np.max(np.abs(d["omega"] - O.solve_ab(ea, eb, La, Lb, noa, nob, 4))) <= 1e-9
        assert np.max(np.abs(dh["omega"] - O.solve_ab(ea, eb, La, Lb, noa, nob, 3, channel="hh"))) <= 1e-9


@pytest.mark.parametrize("channel,nroot", [("pp", 6), ("hh", 4)])
def test_ab_davidson_vs_oracle(channel, nroot):
    nmo, noa, nob, naux = 30, 6, 5, 80   # n = 24 * 25 + 30 = 630: beyond the direct solver
    note("ab davidson", channel)
    ea, eb, La, Lb = unrestricted(73, nmo, noa, nob, naux)
    ref = O.solve_ab(ea, eb, La, Lb, noa, nob, nroot, channel=channel)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-10, channel=channel)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-9


def test_ab_with_alpha_equal_beta_is_singlet_plus_triplet():
    note("ab alpha = beta")
    nocc, nvir, naux = 4, 10, 30
    eps = gen.orbital_energies(74, nocc, nvir)
    L = gen.lpq_full(74, nocc + nvir, naux)
    with P.PpRPA.alpha_beta(eps, eps, L, L, nocc, nocc) as ctx:
        ab = ctx.davidson(8, direct=True)["omega"]
    parts = []
    for mult in ("singlet", "triplet"):
        with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
            parts += list(ctx.davidson(8, direct=True)["omega"])
    assert np.max(np.abs(ab - np.sort(parts)[:8])) <= 1e-9


def test_three_sectors_equal_spin_orbital_build():
    """alpha != beta: lowest pp roots over alpha-alpha, beta-beta (triplet contexts of each spin)
    and alpha-beta (dense context) on the GPU equal the lowest pp roots of the oracle's general
    spin-orbital build."""
    note("three sectors")
    nmo, noa, nob, naux = 7, 3, 2, 12
    ea, eb, La, Lb = unrestricted(75, nmo, noa, nob, naux)
    Mso, nvv_so = O.spin_orbital_matrix_u(ea, eb, La, Lb, noa, nob)
    Om, _, sg = O.solve_general(Mso, nvv_so)
    ref = np.sort(Om[sg > 0])[:8]
    got = []
    for e_s, L_s, no_s in ((ea, La, noa), (eb, Lb, nob)):
        with P.PpRPA(e_s, L_s, no_s, mult="triplet", dense=True) as ctx:
            got += list(ctx.davidson(min(8, ctx.n_pp), direct=True)["omega"])
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        got += list(ctx.davidson(8, direct=True)["omega"])
    assert np.max(np.abs(np.sort(got)[:8] - ref)) <= 1e-9


def test_ab_correlation_energy():
    note("ab correlation energy")
    nmo, noa, nob, naux = 14, 4, 3, 40
    ea, eb, La, Lb = unrestricted(76, nmo, noa, nob, naux)
    M, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    Om, _, sg = O.solve_definite(M, nvv, O.midgap_ab(ea, eb, noa, nob))
    A, C = M[:nvv, :nvv], M[nvv:, nvv:]
    ref_pp, ref_hh = O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        r = ctx.correlation_energy()
    assert abs(r["ec_pp"] - ref_pp) <= 1e-10 and abs(r["ec_hh"] - ref_hh) <= 1e-10


def test_ab_argument_checks():
    note("ab argument checks")
    ea, eb, La, Lb = unrestricted(77, 8, 3, 2, 10)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, 3, 2) as ctx:
        with pytest.raises(P.PpRPAError) as e:
            ctx.nto(np.ones((65, ctx.n)))  # more than 64 roots per call
        assert e.value.status == P.binding.EINVAL
    bad = Lb.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(P.PpRPAError) as e:
        P.PpRPA.alpha_beta(ea, eb, La, bad, 3, 2)
    assert e.value.status == P.binding.EINVAL


# ---- density-fitted alpha-beta sector ----------------------------------------------------
# Ragged shapes: alpha and beta blocks of different tile counts, a beta block of one orbital,
# no beta occupied pairs partner (nocc_b = 0 has no hh pairs).
AB_DF_CASES = [(12, 3, 2, 20), (30, 7, 5, 40), (45, 10, 9, 60), (70, 20, 17, 50), (37, 18, 1, 30),
               (20, 1, 3, 15), (24, 4, 0, 18)]


@pytest.mark.parametrize("case", AB_DF_CASES)
def test_ab_df_sigma_vs_oracle(case):
    """Density-fitted alpha-beta sigma against M z of the oracle's alpha-beta matrix, and against
    the dense context's sigma."""
    nmo, noa, nob, naux = case
    note("ab df sigma", case)
    ea, eb, La, Lb = unrestricted(81, nmo, noa, nob, naux)
    Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as ctx:
        assert ctx.n_pp == nvv and ctx.n == Mref.shape[0]
        z = gen.random_vectors(82, 6, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[3])
    sref = z @ Mref.T
    assert np.max(np.abs(s - sref)) <= 1e-12 * max(1.0, np.abs(sref).max())
    assert np.array_equal(s1, s[3])  # a vector's result does not depend on the block around it
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as dense:
        sd = dense.matvec(z)
    assert np.max(np.abs(s - sd)) <= 1e-12 * max(1.0, np.abs(sd).max())


@pytest.mark.parametrize("case", AB_DF_CASES)
def test_ab_df_sigma_fp32_vs_oracle(case):
    """FP32 density-fitted alpha-beta sigma (integrals and amplitudes rounded to FP32, FP32 MFMA
    accumulation, FP64 epilogue) against M z of the oracle's alpha-beta matrix."""
    nmo, noa, nob, naux = case
    note("ab df sigma fp32", case)
    ea, eb, La, Lb = unrestricted(81, nmo, noa, nob, naux)
    Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec="fp32") as ctx:
        z = gen.random_vectors(82, 6, ctx.n)
        s = ctx.matvec(z)
    sref = z @ Mref.T
    err = np.max(np.abs(s - sref)) / np.abs(sref).max()
    note("relative error", err)
    assert err <= 2e-7


@pytest.mark.parametrize("channel,nroot", [("pp", 6), ("hh", 4)])
def test_ab_df_fp32_davidson_vs_oracle(channel, nroot):
    """FP32 sigma, FP64 subspace algebra: every root within 1e-6 Ha of the oracle's."""
    nmo, noa, nob, naux = 45, 10, 9, 60
    note("ab df davidson fp32", channel)
    ea, eb, La, Lb = unrestricted(83, nmo, noa, nob, naux)
    ref = O.solve_ab(ea, eb, La, Lb, noa, nob, nroot, channel=channel)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec="fp32") as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-5, channel=channel)
    err = np.max(np.abs(r["omega"] - ref))
    note("max root error", err)
    assert r["status"] == 0
    assert err <= 1e-6


# relative to max |M z|; measured on the MI355X over AB_DF_CASES (BF16x6 8.4e-9 - 3.5e-8, BF16x3
# 4.1e-7 - 9.6e-7), then frozen at about 2.5x the largest value seen
TOL_AB_BF16 = {"bf16x6": 1e-7, "bf16x3": 2.5e-6}


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("case", AB_DF_CASES)
def test_ab_df_sigma_bf16_vs_oracle(case, prec):
    """BF16-split density-fitted alpha-beta sigma (integrals and amplitudes as hi/mid/lo BF16
    planes, six or three products on the BF16 MFMA, FP32 accumulation, FP64 epilogue) against
    M z of the oracle's alpha-beta matrix; shapes with one or no occupied beta orbital and
    blocks that are not multiples of 32 orbitals included."""
    nmo, noa, nob, naux = case
    note("ab df sigma", prec, case)
    ea, eb, La, Lb = unrestricted(81, nmo, noa, nob, naux)
    Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec=prec) as ctx:
        z = gen.random_vectors(82, 6, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[2])
    sref = z @ Mref.T
    err = np.max(np.abs(s - sref)) / np.abs(sref).max()
    note("relative error", err)
    assert err <= TOL_AB_BF16[prec]
    assert np.array_equal(s1, s[2])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-7),
                                      ("bf16x6", TOL_AB_BF16["bf16x6"]),
                                      ("bf16x3", TOL_AB_BF16["bf16x3"])])
def test_ab_df_sigma_widest_block(prec, tol):
    """64 vectors in one block (the largest block the interface takes) in each precision,
    against M z of the oracle's alpha-beta matrix; the last vector alone to the same tolerance."""
    nmo, noa, nob, naux = 30, 7, 5, 40
    note("ab df sigma k = 64", prec)
    ea, eb, La, Lb = unrestricted(81, nmo, noa, nob, naux)
    Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, max_block=64, density_fitted=True,
                            prec=prec) as ctx:
        z = gen.random_vectors(83, 64, ctx.n)
        s = ctx.matvec(z)
        s1 = ctx.matvec(z[63])
    sref = z @ Mref.T
    scale = max(1.0, np.abs(sref).max()) if prec == "fp64" else np.abs(sref).max()
    err = np.max(np.abs(s - sref)) / scale
    note("relative error", err)
    assert err <= tol
    assert np.max(np.abs(s1 - sref[63])) / scale <= tol


def test_ab_bf16x6_beats_bf16x3():
    """The two BF16 schemes on the same alpha-beta inputs: six products at least 20 times more
    accurate than three, which tells the arithmetic that ran apart."""
    for case in [(30, 7, 5, 40), (45, 10, 9, 60)]:
        nmo, noa, nob, naux = case
        ea, eb, La, Lb = unrestricted(81, nmo, noa, nob, naux)
        Mref, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
        err = {}
        for prec in ("bf16x6", "bf16x3"):
            with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True,
                                    prec=prec) as ctx:
                z = gen.random_vectors(82, 6, ctx.n)
                s = ctx.matvec(z)
            sref = z @ Mref.T
            err[prec] = np.max(np.abs(s - sref)) / np.abs(sref).max()
        note(case, "x6 %.2e x3 %.2e" % (err["bf16x6"], err["bf16x3"]))
        assert err["bf16x6"] <= err["bf16x3"] / 20.0


@pytest.mark.parametrize("channel,nroot", [("pp", 6), ("hh", 4)])
def test_ab_df_bf16x6_davidson_vs_oracle(channel, nroot):
    """BF16x6 sigma, FP64 subspace algebra: every root within 1e-6 Ha of the oracle's."""
    nmo, noa, nob, naux = 45, 10, 9, 60
    note("ab df davidson bf16x6", channel)
    ea, eb, La, Lb = unrestricted(83, nmo, noa, nob, naux)
    ref = O.solve_ab(ea, eb, La, Lb, noa, nob, nroot, channel=channel)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec="bf16x6") as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-5, channel=channel)
    err = np.max(np.abs(r["omega"] - ref))
    note("max root error", err)
    assert r["status"] == 0
    assert err <= 1e-6


def test_ab_df_precision_refusals():
    """The alpha-beta sector takes reduced-precision sigma only density fitted."""
    ea, eb, La, Lb = unrestricted(88, 12, 3, 2, 20)
    for kw in (dict(prec="fp32"), dict(prec="bf16x6"), dict(prec="bf16x3")):
        with pytest.raises(P.PpRPAError) as e:
            P.PpRPA.alpha_beta(ea, eb, La, Lb, 3, 2, **kw)
        assert e.value.status == P.binding.EUNSUPPORTED


@pytest.mark.parametrize("channel,nroot", [("pp", 6), ("hh", 4)])
def test_ab_df_davidson_vs_oracle(channel, nroot):
    nmo, noa, nob, naux = 45, 10, 9, 60
    note("ab df davidson", channel)
    ea, eb, La, Lb = unrestricted(83, nmo, noa, nob, naux)
    ref = O.solve_ab(ea, eb, La, Lb, noa, nob, nroot, channel=channel)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as ctx:
        r = ctx.davidson(nroot, block=nroot, tol=1e-10, channel=channel)
    assert r["status"] == 0
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-9


def test_ab_df_beyond_the_dense_limit():
    """n = 180 * 182 + 20 * 18 = 33120 > 32768: the dense context is refused, the density-fitted
    one builds; sampled sigma entries against the oracle's rows of M, and a Davidson solve whose
    returned residuals meet the tolerance. naux = 3.5 nmo as in the workloads (with far fewer aux
    functions this synthetic pencil is not definite, which the solver reports as ENONDEF)."""
    nmo, noa, nob, naux = 200, 20, 18, 700
    note("ab df large")
    ea, eb, La, Lb = unrestricted(85, nmo, noa, nob, naux)
    with pytest.raises(P.PpRPAError) as e:
        P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob)
    assert e.value.status == P.binding.EINVAL
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as ctx:
        assert ctx.n == 180 * 182 + 20 * 18
        z = gen.random_vectors(86, 4, ctx.n)
        s = ctx.matvec(z)
        r = ctx.davidson(5, block=10, tol=1e-7)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec="fp32") as c32:
        s32 = c32.matvec(z)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True, prec="bf16x6") as c16:
        s16 = c16.matvec(z)
    rng = np.random.default_rng(4)
    nvv = 180 * 182
    rows = np.unique(np.r_[np.arange(3), nvv - 3 + np.arange(6), ctx.n - 3 + np.arange(3),
                           rng.integers(0, ctx.n, 20)])
    for j in range(z.shape[0]):
        ref = O.ab_sigma_rows(ea, eb, La, Lb, noa, nob, rows, z[j])
        assert np.max(np.abs(s[j, rows] - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
        err32 = np.max(np.abs(s32[j, rows] - ref)) / np.abs(s32[j]).max()
        err16 = np.max(np.abs(s16[j, rows] - ref)) / np.abs(s16[j]).max()
        note("fp32 / bf16x6 relative error", err32, err16)
        assert err32 <= 1e-6 and err16 <= 1e-6
    assert r["status"] == 0 and np.all(r["resid"] <= 1e-7)
    assert np.all(np.diff(r["omega"]) >= 0)


def test_ab_df_dense_only_calls_are_refused():
    nmo, noa, nob, naux = 12, 3, 2, 20
    note("ab df refusals")
    ea, eb, La, Lb = unrestricted(87, nmo, noa, nob, naux)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as ctx:
        for call in (lambda: ctx.davidson(3, direct=True), ctx.correlation_energy, ctx.dense_matrix):
            with pytest.raises(P.PpRPAError) as e:
                call()
            assert e.value.status == P.binding.EUNSUPPORTED


@pytest.mark.parametrize("case", [(12, 4, 2, 20), (10, 2, 5, 18), (9, 3, 0, 14), (30, 7, 5, 40)])
def test_ab_nto_vs_oracle(case):
    """NTO weights and spin-resolved density blocks of alpha-beta roots (rectangular amplitude
    blocks: alpha longer than beta, shorter, no beta occupied): pp and hh roots of the dense
    context's direct solve and seeded random vectors against the oracle's, 1e-12 relative to the
    vector's squared norm; on the roots, sum(lam^p) - sum(lam^h) = +1 / -1 and every spin's trace
    x^T x (vv) or -y^T y (oo); the density-fitted context of the same system gives the same
    values bit for bit."""
    nmo, noa, nob, naux = case
    note("ab nto", case)
    ea, eb, La, Lb = unrestricted(91, nmo, noa, nob, naux)
    nva, nvb = nmo - noa, nmo - nob
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        zs = [ctx.davidson(3, direct=True, vectors=True)["vecs"]]
        nh = min(2, ctx.n_hh)
        if nh:
            zs.append(ctx.davidson(nh, direct=True, vectors=True, channel="hh")["vecs"])
        zs.append(gen.random_vectors(92, 3, ctx.n))
        Z = np.vstack(zs)
        out = ctx.nto(Z)
        nvv = ctx.n_pp
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as dfc:
        out_df = dfc.nto(Z)
    for key in ("lam_p", "lam_h", "d_vv_a", "d_vv_b", "d_oo_a", "d_oo_b"):
        assert np.array_equal(out[key], out_df[key]), key
    nroots = 3 + nh
    for j, z in enumerate(Z):
        lp, lh, _ = O.nto_ab(z, nva, nvb, noa, nob)
        Dva, Dvb, Doa, Dob = O.density_2e_ab(z, nva, nvb, noa, nob)
        tol = 1e-12 * max(1.0, z @ z)
        assert np.max(np.abs(out["lam_p"][j] - lp)) <= tol
        if noa:
            assert np.max(np.abs(out["lam_h"][j] - lh)) <= tol
        for got, ref in ((out["d_vv_a"][j], Dva), (out["d_vv_b"][j], Dvb),
                         (out["d_oo_a"][j], Doa), (out["d_oo_b"][j], Dob)):
            if ref.size:
                assert np.max(np.abs(got - ref)) <= tol
        if j < nroots:
            sgn = 1.0 if j < 3 else -1.0
            x2, y2 = z[:nvv] @ z[:nvv], z[nvv:] @ z[nvv:]
            assert abs(out["lam_p"][j].sum() - out["lam_h"][j].sum() - sgn) <= 1e-10
            assert abs(np.trace(out["d_vv_a"][j]) - x2) <= 1e-12
            assert abs(np.trace(out["d_vv_b"][j]) - x2) <= 1e-12
            if noa and nob:
                assert abs(np.trace(out["d_oo_a"][j]) + y2) <= 1e-12

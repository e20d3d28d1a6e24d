"""Pins for the FP64 oracle: each checks it against something other than itself.

P1  L = 0: closed form Omega = e_a + e_b (pp), e_i + e_j (hh).
P2  B = 0 (L_vo = 0): pp roots = eigvalsh(A), hh roots = -eigvalsh(C) (LAPACK), E_c = 0.
P3  sum rule of Eq. correlation_energy: sum(pp) + sum(hh) = Tr A - Tr C; root counts.
P4  normalisation of Eq. xy_norm: Z^T W Z = diag(+-1).
P5  the spin-orbital build (general elements with a<b, i<j) has the spectrum
    singlet U 3 x triplet.
P6  second order: with A/C interactions off and L_vo scaled by lam,
    E_c(singlet) + 3 E_c(triplet) -> lam^2 * closed-shell RI-MP2 (section "Total Energy":
    ppRPA correlation is exact to second order).
P7  two electrons: with no occupied orbitals the singlet and triplet A spectra together are
    the spectrum of the two-electron CI Hamiltonian (Slater-Condon).
P8  the factorised sigma equals the dense M z; route D equals route G.
NTO the natural transition orbital weights and the two-electron density matrix: L = 0 closed
    form, the weight sum rule and Tr D = +-2 (Eq. dm_constrain) on every root.
UHF the spin-unrestricted sectors: alpha = beta gives singlet U triplet in the alpha-beta
    sector; alpha != beta: the general spin-orbital build equals alpha-alpha U alpha-beta U
    beta-beta; L = 0 closed form.
hh  the removal channel's selection: L = 0 closed form (highest e_i + e_j first), B = 0 against
    -eigvalsh(C), the subset solve against the full spectrum.
Plus mutation checks: plausible mistakes planted in a copy of the oracle fail a pin.
"""
import numpy as np
import pytest

from oracle import pprpa_oracle as O
from workloads import gen


def make_sp(seed, nocc, nvir, naux, scale=None):
    eps = gen.orbital_energies(seed, nocc, nvir)
    L = gen.lpq_full(seed, nocc + nvir, naux)
    if scale is not None:
        L = L * scale
    return eps, L, O.active_space(eps, L, nocc)


def full_spectrum(sp, mult, route="D"):
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    if route == "D":
        Om, Z, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
    else:
        Om, Z, sg = O.solve_general(M, A.shape[0])
    return A, B, C, M, Om, Z, sg


MULTS = ["singlet", "triplet"]
SIZES = [(1, 2, 5), (2, 3, 7), (3, 5, 11), (4, 9, 30)]


@pytest.mark.parametrize("mult", MULTS)
@pytest.mark.parametrize("route", ["D", "G"])
@pytest.mark.parametrize("nocc,nvir,naux", SIZES)
def test_p1_zero_interaction(mult, route, nocc, nvir, naux):
    eps, L, sp = make_sp(1, nocc, nvir, naux, scale=0.0)
    A, B, C, M, Om, Z, sg = full_spectrum(sp, mult, route)
    k = 0 if mult == "singlet" else 1
    eo, ev = eps[:nocc], eps[nocc:]
    pp = np.sort([ev[a] + ev[b] for a in range(nvir) for b in range(a + k, nvir)])
    hh = np.sort([eo[i] + eo[j] for i in range(nocc) for j in range(i + k, nocc)])
    assert np.allclose(np.sort(Om[sg > 0]), pp, atol=1e-13)
    assert np.allclose(np.sort(Om[sg < 0]), hh, atol=1e-13)


@pytest.mark.parametrize("mult", MULTS)
@pytest.mark.parametrize("nocc,nvir,naux", SIZES)
def test_p2_no_coupling(mult, nocc, nvir, naux):
    eps, L, sp = make_sp(2, nocc, nvir, naux)
    sp["Lov"] = np.zeros_like(sp["Lov"])
    A, B, C, M, Om, Z, sg = full_spectrum(sp, mult)
    assert np.all(B == 0.0)
    assert np.allclose(np.sort(Om[sg > 0]), np.linalg.eigvalsh(A), atol=1e-12)
    assert np.allclose(np.sort(Om[sg < 0]), np.sort(-np.linalg.eigvalsh(C)), atol=1e-12)
    ec1, ec2 = O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C)
    assert abs(ec1) < 1e-12 and abs(ec2) < 1e-12


@pytest.mark.parametrize("mult", MULTS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p3_p4_sum_rule_counts_normalisation(mult, seed):
    eps, L, sp = make_sp(seed, 4, 9, 30)
    A, B, C, M, Om, Z, sg = full_spectrum(sp, mult)
    nvv, noo = A.shape[0], C.shape[0]
    assert int(np.sum(sg > 0)) == nvv and int(np.sum(sg < 0)) == noo
    ec1, ec2 = O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C)
    assert abs(ec1 - ec2) < 1e-12
    assert ec1 < 0.0  # correlation lowers the energy
    w = O.metric(nvv, noo)
    G = Z.T @ (w[:, None] * Z)
    assert np.allclose(G, np.diag(sg), atol=1e-10)
    # eigen-relation itself
    assert np.allclose(M @ Z, (w[:, None] * Z) * Om[None, :], atol=1e-11)


@pytest.mark.parametrize("nocc,nvir,naux", [(1, 2, 5), (2, 3, 6), (2, 4, 9), (3, 3, 8)])
def test_p5_spin_orbital_equals_singlet_plus_3_triplet(nocc, nvir, naux):
    eps, L, sp = make_sp(3, nocc, nvir, naux)
    Mso, nvv_so = O.spin_orbital_matrix(sp)
    Om_so, _, sg_so = O.solve_general(Mso, nvv_so)
    parts_pp, parts_hh = [], []
    for mult, mult_count in (("singlet", 1), ("triplet", 3)):
        _, _, _, _, Om, _, sg = full_spectrum(sp, mult, "G")
        parts_pp += list(Om[sg > 0]) * mult_count
        parts_hh += list(Om[sg < 0]) * mult_count
    assert np.allclose(np.sort(Om_so[sg_so > 0]), np.sort(parts_pp), atol=1e-12)
    assert np.allclose(np.sort(Om_so[sg_so < 0]), np.sort(parts_hh), atol=1e-12)


def _ec_total(sp):
    tot = 0.0
    for mult, g in (("singlet", 1), ("triplet", 3)):
        A, B, C, M, Om, Z, sg = full_spectrum(sp, mult)
        tot += g * O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C)[0]
    return tot


@pytest.mark.parametrize("seed", [0, 1])
def test_p6_mp2_limit(seed):
    eps, L, sp = make_sp(seed, 3, 6, 20)
    emp2 = O.rimp2_energy(sp)
    lam = 1e-2
    sp2 = dict(sp)
    sp2["Lvv"] = np.zeros_like(sp["Lvv"])
    sp2["Loo"] = np.zeros_like(sp["Loo"])
    sp2["Lov"] = sp["Lov"] * np.sqrt(lam)  # integrals (ak|bl) scale by lam
    ec = _ec_total(sp2)
    assert emp2 < 0
    assert abs(ec / lam ** 2 - emp2) < 1e-5 * abs(emp2)  # measured 7e-7 and 1.3e-6


@pytest.mark.parametrize("nvir,naux", [(1, 4), (3, 8), (5, 12)])
def test_p7_two_electron_ci(nvir, naux):
    eps, L, sp = make_sp(4, 0, nvir, naux)
    As, _, _ = O.build_matrices(sp, "singlet")
    At, _, _ = O.build_matrices(sp, "triplet")
    spec = np.sort(np.concatenate([np.linalg.eigvalsh(As), np.linalg.eigvalsh(At)]))
    ci = O.two_electron_ci(sp["ev"], sp["Lvv"])
    # the CI over |a alpha b beta> holds the singlets and the M_s = 0 triplets once each
    assert np.allclose(spec, ci, atol=1e-13)


@pytest.mark.parametrize("mult", MULTS)
@pytest.mark.parametrize("nocc,nvir,naux", SIZES + [(5, 20, 100)])
def test_p8_factorised_sigma_and_routes(mult, nocc, nvir, naux):
    eps, L, sp = make_sp(5, nocc, nvir, naux)
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    z = gen.random_vectors(9, 3, M.shape[0]).T
    s_dense = O.sigma_dense(M, z)
    s_fact = O.sigma_factorised(sp, mult, z)
    assert np.allclose(s_fact, s_dense, atol=1e-13 * max(1.0, np.abs(s_dense).max()))
    rows = np.unique(np.r_[0, M.shape[0] - 1, M.shape[0] // 2, A.shape[0] - 1])
    assert np.allclose(O.sigma_rows(sp, mult, rows, z[:, 0]), s_dense[rows, 0], atol=1e-13)
    OmD, _, sgD = O.solve_definite(M, A.shape[0], O.midgap(sp))
    OmG, _, sgG = O.solve_general(M, A.shape[0])
    assert np.array_equal(sgD, sgG)
    assert np.allclose(OmD, OmG, atol=1e-11)


def test_subset_route_matches_full():
    eps, L, sp = make_sp(0, 5, 20, 100)
    A, B, C = O.build_matrices(sp, "singlet")
    M = O.pprpa_matrix(A, B, C)
    Om, Z, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
    Om5, Z5, sg5 = O.solve_definite(M, A.shape[0], O.midgap(sp), nroot=5)
    assert np.all(sg5 > 0)
    assert np.allclose(Om5, Om[sg > 0][:5], atol=1e-12)


# ----------------------------------------------------------------------------------------
# hh channel selection (two-electron removal roots nearest the gap, largest Omega first)
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("mult", MULTS)
@pytest.mark.parametrize("nocc,nvir,naux", [(4, 9, 30), (6, 5, 20)])
def test_hh_channel_zero_interaction(mult, nocc, nvir, naux):
    """L = 0: the hh roots are e_i + e_j; the channel returns the highest pairs, descending."""
    eps = gen.orbital_energies(3, nocc, nvir)
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    k = 0 if mult == "singlet" else 1
    eo = eps[:nocc]
    hh = np.sort([eo[i] + eo[j] for i in range(nocc) for j in range(i + k, nocc)])[::-1]
    nroot = min(5, hh.size)
    for route in ("D", "G"):
        om = O.solve(eps, L, nocc, mult, nroot, route=route, channel="hh")
        assert np.allclose(om, hh[:nroot], atol=1e-13)
        assert np.all(np.diff(om) <= 0.0)


@pytest.mark.parametrize("mult", MULTS)
def test_hh_channel_no_coupling(mult):
    """B = 0: the hh roots are -eigvalsh(C) (LAPACK on C alone); the channel returns the
    largest of them."""
    eps, L, sp = make_sp(4, 6, 9, 30)
    sp["Lov"] = np.zeros_like(sp["Lov"])
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    Om, Z, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
    om, z = O.hh_nearest(Om, Z, sg, 4)
    ref = np.sort(-np.linalg.eigvalsh(C))[::-1][:4]
    assert np.allclose(om, ref, atol=1e-12)


@pytest.mark.parametrize("mult", MULTS)
def test_hh_subset_route_matches_full(mult):
    """The nroot smallest theta of route D are the hh roots nearest the gap; their vectors
    satisfy M z = Omega W z with z^T W z = -1 (Eq. xy_norm, removal sign)."""
    eps, L, sp = make_sp(0, 5, 20, 100)
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    nvv = A.shape[0]
    Om, Z, sg = O.solve_definite(M, nvv, O.midgap(sp))
    full, _ = O.hh_nearest(Om, Z, sg, 5)
    Om5, Z5, sg5 = O.solve_definite(M, nvv, O.midgap(sp), nroot=5, channel="hh")
    assert np.all(sg5 < 0)
    assert np.allclose(np.sort(Om5)[::-1], full, atol=1e-12)
    assert np.all(Om5 < 2.0 * O.midgap(sp))
    w = O.metric(nvv, M.shape[0] - nvv)
    assert np.allclose(M @ Z5, (w[:, None] * Z5) * Om5[None, :], atol=1e-10)
    assert np.allclose(np.einsum("i,ij,ij->j", w, Z5, Z5), -1.0, atol=1e-12)


# ----------------------------------------------------------------------------------------
# NTOs and the two-electron density matrix
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("mult", MULTS)
def test_nto_zero_interaction_closed_form(mult):
    """L = 0: a pp root is a unit vector on one pair (a, b): one NTO pair of weight 1, and the
    density block is E_aa + E_bb (D = 2 E_aa for a = b); an hh root likewise with -1."""
    nocc, nvir, naux = 4, 7, 5
    eps = gen.orbital_energies(5, nocc, nvir)
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    sp = O.active_space(eps, L, nocc)
    A, B, C, M, Om, Z, sg = full_spectrum(sp, mult)
    nvv = A.shape[0]
    for j in range(Z.shape[1]):
        z = O.fix_sign(Z[:, j:j + 1])[:, 0]
        lp, lh, _ = O.nto(z, nvir, nocc, mult)
        Dv, Do = O.density_2e(z, nvir, nocc, mult)
        k = int(np.argmax(np.abs(z)))
        if sg[j] > 0:
            pa, pb = O.pairs(nvir, mult)
            a, b = pa[k], pb[k]
            assert np.allclose(lp, np.r_[1.0, np.zeros(nvir - 1)], atol=1e-14) and np.allclose(lh, 0.0)
            ref = np.zeros((nvir, nvir))
            ref[a, a] += 1.0
            ref[b, b] += 1.0
            assert np.allclose(Dv, ref, atol=1e-14) and np.allclose(Do, 0.0)
        else:
            pi, pj = O.pairs(nocc, mult)
            i, jj = pi[k - nvv], pj[k - nvv]
            assert np.allclose(lh, np.r_[1.0, np.zeros(nocc - 1)], atol=1e-14) and np.allclose(lp, 0.0)
            ref = np.zeros((nocc, nocc))
            ref[i, i] -= 1.0
            ref[jj, jj] -= 1.0
            assert np.allclose(Do, ref, atol=1e-14) and np.allclose(Dv, 0.0)


@pytest.mark.parametrize("mult", MULTS)
def test_nto_weight_and_density_sum_rules(mult):
    """Every root: sum(lam^p) - sum(lam^h) = +1 (pp) / -1 (hh) (NTO section) and
    Tr D^2e = +2 / -2 (Eq. dm_constrain); the SVD factors reproduce X and Y."""
    eps, L, sp = make_sp(6, 5, 12, 40)
    A, B, C, M, Om, Z, sg = full_spectrum(sp, mult)
    for j in range(Z.shape[1]):
        z = Z[:, j]
        lp, lh, (U, V, Uh, Vh) = O.nto(z, 12, 5, mult)
        assert abs(lp.sum() - lh.sum() - sg[j]) <= 1e-12
        Dv, Do = O.density_2e(z, 12, 5, mult)
        assert abs(np.trace(Dv) + np.trace(Do) - 2.0 * sg[j]) <= 1e-12
        nvv = A.shape[0]
        X = O.triangular(z[:nvv], 12, mult)
        assert np.allclose(U @ np.diag(np.sqrt(lp)) @ V.T, X, atol=1e-13)
        assert np.all(np.diff(lp) <= 1e-15) and np.all(lp >= 0.0)


# ----------------------------------------------------------------------------------------
# Spin-unrestricted sectors
# ----------------------------------------------------------------------------------------

def unrestricted(seed, nmo, nocc_a, nocc_b, naux):
    return (gen.orbital_energies(seed, nocc_a, nmo - nocc_a),
            gen.orbital_energies(seed + 1000, nocc_b, nmo - nocc_b),
            gen.lpq_full(seed, nmo, naux), gen.lpq_full(seed + 1000, nmo, naux))


def test_nto_ab_zero_interaction_closed_form():
    """L = 0 in the alpha-beta sector: every root is a unit vector on one pair (a_alpha, b_beta)
    (or (i, j)): one NTO pair of weight 1 (alpha side padded with zeros), D^alpha = E_aa,
    D^beta = E_bb (with the sign of the channel)."""
    nmo, noa, nob, naux = 7, 3, 2, 4
    ea, eb, La, Lb = unrestricted(31, nmo, noa, nob, naux)
    La[:] = 0.0
    Lb[:] = 0.0
    nva, nvb = nmo - noa, nmo - nob
    M, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    Om, Z, sg = O.solve_definite(M, nvv, O.midgap_ab(ea, eb, noa, nob))
    for j in range(Z.shape[1]):
        z = Z[:, j]
        k = int(np.argmax(np.abs(z)))
        lp, lh, _ = O.nto_ab(z, nva, nvb, noa, nob)
        Dva, Dvb, Doa, Dob = O.density_2e_ab(z, nva, nvb, noa, nob)
        if sg[j] > 0:
            a, b = divmod(k, nvb)
            assert np.allclose(lp, np.r_[1.0, np.zeros(nva - 1)], atol=1e-14) and np.allclose(lh, 0.0)
            assert np.allclose(Dva, np.diag(np.eye(nva)[a]), atol=1e-14)
            assert np.allclose(Dvb, np.diag(np.eye(nvb)[b]), atol=1e-14)
            assert np.allclose(Doa, 0.0) and np.allclose(Dob, 0.0)
        else:
            i, jj = divmod(k - nvv, nob)
            assert np.allclose(lh, np.r_[1.0, np.zeros(noa - 1)], atol=1e-14) and np.allclose(lp, 0.0)
            assert np.allclose(Doa, -np.diag(np.eye(noa)[i]), atol=1e-14)
            assert np.allclose(Dob, -np.diag(np.eye(nob)[jj]), atol=1e-14)


@pytest.mark.parametrize("nmo,noa,nob", [(12, 4, 2), (10, 2, 5), (9, 3, 0)])
def test_nto_ab_sum_rules(nmo, noa, nob):
    """Every alpha-beta root: sum(lam^p) - sum(lam^h) = +1 (pp) / -1 (hh); the traces of the
    spin-resolved density blocks: Tr D^alpha_vv = Tr D^beta_vv = x^T x, Tr D^alpha_oo =
    Tr D^beta_oo = -y^T y, in all +2 / -2; the SVD factors reproduce X; the nonzero weights
    number at most min(nvir_a, nvir_b) (alpha longer or shorter than beta; no beta occupied)."""
    ea, eb, La, Lb = unrestricted(33, nmo, noa, nob, 16)
    nva, nvb = nmo - noa, nmo - nob
    M, nvv = O.ab_sector(ea, eb, La, Lb, noa, nob)
    Om, Z, sg = O.solve_definite(M, nvv, O.midgap_ab(ea, eb, noa, nob))
    for j in range(Z.shape[1]):
        z = Z[:, j]
        lp, lh, (U, V, Uh, Vh) = O.nto_ab(z, nva, nvb, noa, nob)
        assert abs(lp.sum() - lh.sum() - sg[j]) <= 1e-12
        Dva, Dvb, Doa, Dob = O.density_2e_ab(z, nva, nvb, noa, nob)
        x2, y2 = z[:nvv] @ z[:nvv], z[nvv:] @ z[nvv:]
        assert abs(np.trace(Dva) - x2) <= 1e-12 and abs(np.trace(Dvb) - x2) <= 1e-12
        assert abs(np.trace(Doa) + y2) <= 1e-12 and abs(np.trace(Dob) + y2) <= 1e-12
        assert abs(np.trace(Dva) + np.trace(Dvb) + np.trace(Doa) + np.trace(Dob) - 2 * sg[j]) <= 1e-12
        X = z[:nvv].reshape(nva, nvb)
        r = min(nva, nvb)
        assert np.allclose(U[:, :r] @ np.diag(np.sqrt(lp[:r])) @ V[:, :r].T, X, atol=1e-13)
        assert np.all(lp[r:] == 0.0) and np.all(np.diff(lp) <= 1e-15) and np.all(lp >= 0.0)


@pytest.mark.parametrize("nocc,nvir,naux", [(2, 3, 7), (3, 5, 11), (4, 6, 20)])
def test_ab_sector_with_alpha_equal_beta_is_singlet_plus_triplet(nocc, nvir, naux):
    """alpha = beta: the alpha-beta pairs carry both spin couplings, so the sector's spectrum is
    the union of the singlet and triplet spectra (spin-adapted elements, built independently)."""
    eps, L, sp = make_sp(7, nocc, nvir, naux)
    M, nvv = O.ab_sector(eps, eps, L, L, nocc, nocc)
    Om, _, sg = O.solve_definite(M, nvv, O.midgap_ab(eps, eps, nocc, nocc))
    ref_pp, ref_hh = [], []
    for mult in MULTS:
        _, _, _, _, Om_s, _, sg_s = full_spectrum(sp, mult)
        ref_pp += list(Om_s[sg_s > 0])
        ref_hh += list(Om_s[sg_s < 0])
    assert np.allclose(np.sort(Om[sg > 0]), np.sort(ref_pp), atol=1e-12)
    assert np.allclose(np.sort(Om[sg < 0]), np.sort(ref_hh), atol=1e-12)


@pytest.mark.parametrize("nmo,nocc_a,nocc_b,naux", [(6, 2, 1, 9), (7, 3, 2, 12), (6, 2, 2, 10)])
def test_unrestricted_sectors_equal_spin_orbital_matrix(nmo, nocc_a, nocc_b, naux):
    """alpha != beta (energies, integrals and occupations): the spectrum of the general
    spin-orbital build is the union of the alpha-alpha, alpha-beta and beta-beta sectors."""
    ea, eb, La, Lb = unrestricted(8, nmo, nocc_a, nocc_b, naux)
    Mso, nvv_so = O.spin_orbital_matrix_u(ea, eb, La, Lb, nocc_a, nocc_b)
    Om_so, _, sg_so = O.solve_general(Mso, nvv_so)
    parts_pp, parts_hh = [], []
    for e_s, L_s, no_s in ((ea, La, nocc_a), (eb, Lb, nocc_b)):
        sp = O.active_space(e_s, L_s, no_s)
        A, B, C = O.build_matrices(sp, "triplet")
        Om, _, sg = O.solve_general(O.pprpa_matrix(A, B, C), A.shape[0])
        parts_pp += list(Om[sg > 0])
        parts_hh += list(Om[sg < 0])
    M, nvv = O.ab_sector(ea, eb, La, Lb, nocc_a, nocc_b)
    Om, _, sg = O.solve_general(M, nvv)
    parts_pp += list(Om[sg > 0])
    parts_hh += list(Om[sg < 0])
    assert np.allclose(np.sort(Om_so[sg_so > 0]), np.sort(parts_pp), atol=1e-12)
    assert np.allclose(np.sort(Om_so[sg_so < 0]), np.sort(parts_hh), atol=1e-12)
    # route D with the alpha-beta shift agrees with the general solver
    OmD, _, sgD = O.solve_definite(M, nvv, O.midgap_ab(ea, eb, nocc_a, nocc_b))
    assert np.array_equal(sgD, sg) and np.allclose(OmD, Om, atol=1e-11)


@pytest.mark.parametrize("nmo,nocc_a,nocc_b,naux", [(7, 3, 2, 12), (9, 2, 4, 7), (6, 1, 0, 5)])
def test_ab_sigma_rows_equal_dense_product(nmo, nocc_a, nocc_b, naux):
    """The row-by-row alpha-beta sigma equals M z of the alpha-beta matrix, every row."""
    ea, eb, La, Lb = unrestricted(10, nmo, nocc_a, nocc_b, naux)
    M, nvv = O.ab_sector(ea, eb, La, Lb, nocc_a, nocc_b)
    z = np.random.default_rng(3).standard_normal(M.shape[0])
    rows = np.arange(M.shape[0])
    assert np.allclose(O.ab_sigma_rows(ea, eb, La, Lb, nocc_a, nocc_b, rows, z), M @ z,
                       atol=1e-13, rtol=0)


def test_ab_sector_zero_interaction():
    nmo, nocc_a, nocc_b = 7, 3, 2
    ea, eb, La, Lb = unrestricted(9, nmo, nocc_a, nocc_b, 5)
    z = np.zeros_like(La)
    om = O.solve_ab(ea, eb, z, z, nocc_a, nocc_b, 6)
    ref = np.sort((ea[nocc_a:][:, None] + eb[nocc_b:][None, :]).ravel())[:6]
    assert np.allclose(om, ref, atol=1e-13)
    hh = O.solve_ab(ea, eb, z, z, nocc_a, nocc_b, 4, channel="hh")
    ref_hh = np.sort((ea[:nocc_a][:, None] + eb[:nocc_b][None, :]).ravel())[::-1][:4]
    assert np.allclose(hh, ref_hh, atol=1e-13)


def test_active_window_equals_oracle_on_sliced_input():
    nocc, nvir, naux = 6, 12, 40
    eps = gen.orbital_energies(0, nocc, nvir)
    L = gen.lpq_full(0, nocc + nvir, naux)
    a = O.solve(eps, L, nocc, "triplet", 4, nocc_act=3, nvir_act=7)
    La = gen.lpq_active(0, nocc, nvir, naux, 3, 7)
    b = O.solve(eps, La, nocc, "triplet", 4, nocc_act=3, nvir_act=7, lpq_is_active=True)
    assert np.array_equal(a, b)
    idx = gen.active_indices(nocc, nvir, 3, 7)
    c = O.solve(np.r_[eps[idx]], La, 3, "triplet", 4)
    assert np.allclose(a, c, atol=1e-14)


# ----------------------------------------------------------------------------------------
# Mutation checks: a planted mistake in the oracle must fail at least one pin.
# ----------------------------------------------------------------------------------------

def test_mutation_wrong_b_convention_fails_p6(monkeypatch):
    """Reading B as (ab|kl) (from L_vv and L_oo) instead of (ak|bl) breaks the MP2 limit."""
    eps, L, sp = make_sp(0, 3, 6, 20)
    emp2 = O.rimp2_energy(sp)
    lam = 1e-2
    sp2 = dict(sp)
    sp2["Lvv"] = np.zeros_like(sp["Lvv"])
    sp2["Loo"] = np.zeros_like(sp["Loo"])
    sp2["Lov"] = sp["Lov"] * np.sqrt(lam)
    good = O.build_matrices

    def wrong(spx, mult):
        A, B, C = good(spx, mult)
        sign = 1.0 if mult == "singlet" else -1.0
        va, vb = O.pairs(spx["ev"].size, mult)
        oi, oj = O.pairs(spx["eo"].size, mult)
        Lv = sp["Lvv"] * np.sqrt(lam)
        Lo = sp["Loo"] * np.sqrt(lam)
        ab_kl = np.einsum("Pab,Pkl->abkl", Lv, Lo)
        Bw = (ab_kl[va, vb][:, oi, oj] + sign * ab_kl[va, vb][:, oj, oi])
        Bw *= np.outer(O.pair_norm(va, vb, mult), O.pair_norm(oi, oj, mult))
        return A, Bw, C

    monkeypatch.setattr(O, "build_matrices", wrong)
    ec = _ec_total(sp2)
    assert abs(ec / lam ** 2 - emp2) > 1e-2 * abs(emp2)


def test_mutation_dropped_singlet_norm_fails_p5(monkeypatch):
    eps, L, sp = make_sp(3, 2, 3, 6)
    Mso, nvv_so = O.spin_orbital_matrix(sp)
    Om_so, _, sg_so = O.solve_general(Mso, nvv_so)
    monkeypatch.setattr(O, "pair_norm", lambda p, q, mult: np.ones(p.size))
    parts = []
    for mult, g in (("singlet", 1), ("triplet", 3)):
        _, _, _, _, Om, _, sg = full_spectrum(sp, mult, "G")
        parts += list(Om[sg > 0]) * g
    assert not np.allclose(np.sort(Om_so[sg_so > 0]), np.sort(parts), atol=1e-6)


def test_mutation_exchange_sign_fails_p7(monkeypatch):
    """Using (ab|cd) (chemists' order) in A instead of (ac|bd) breaks the 2-electron CI pin."""
    eps, L, sp = make_sp(4, 0, 3, 8)
    ci = O.two_electron_ci(sp["ev"], sp["Lvv"])
    orig = O.pair_integrals

    def chem(L_rc, rp, rq, cp, cq, sign, chunk=256):
        if rp.size == 0 or cp.size == 0:
            return np.zeros((rp.size, cp.size))
        g = np.einsum("Ppq,Prs->pqrs", L_rc, L_rc)  # (pq|rs) used as <pq|rs>
        return g[rp, rq][:, cp, cq] + sign * g[rp, rq][:, cq, cp]

    monkeypatch.setattr(O, "pair_integrals", chem)
    As, _, _ = O.build_matrices(sp, "singlet")
    At, _, _ = O.build_matrices(sp, "triplet")
    monkeypatch.setattr(O, "pair_integrals", orig)
    spec = np.sort(np.concatenate([np.linalg.eigvalsh(As), np.linalg.eigvalsh(At)]))
    assert not np.allclose(spec, ci, atol=1e-6)

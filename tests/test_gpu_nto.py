"""GPU: natural transition orbital weights (section "Natural Transition Orbital") and the
two-electron density matrix (section "Density Matrix") of ppRPA roots, through the C ABI,
against the FP64 oracle applied to the same vectors.

* weights (squared singular values of the triangular amplitude matrices, descending) and the
  density blocks equal the oracle's within 1e-12 on pp and hh roots of ragged shapes, both
  spins, an active window, host and device vectors;
* the sum rules: sum lam^p - sum lam^h = +1 (pp) / -1 (hh), Tr D = +2 / -2 (Eq. dm_constrain);
* L = 0: one NTO pair of weight 1 per root;
* argument checks;
* the NTO pairs themselves (pprpa_nto_vectors): against the oracle's SVD (one sign convention
  applied to both; pairs with nonzero, isolated weights, within 1e-9), the full set
  reconstructing X and Y within 1e-10, for restricted and alpha-beta roots.
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


def check_against_oracle(z, res, nv, no, mult, sign):
    for j in range(z.shape[0]):
        lp, lh, _ = O.nto(z[j], nv, no, mult)
        Dv, Do = O.density_2e(z[j], nv, no, mult)
        assert np.max(np.abs(res["lam_p"][j] - lp)) <= 1e-12
        assert np.max(np.abs(res["lam_h"][j] - lh)) <= 1e-12 if no else True
        assert np.max(np.abs(res["d_vv"][j] - Dv)) <= 1e-12
        if no:
            assert np.max(np.abs(res["d_oo"][j] - Do)) <= 1e-12
        s = res["lam_p"][j].sum() - (res["lam_h"][j].sum() if no else 0.0)
        assert abs(s - sign) <= 1e-9
        tr = np.trace(res["d_vv"][j]) + (np.trace(res["d_oo"][j]) if no else 0.0)
        assert abs(tr - 2.0 * sign) <= 2e-9


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(4, 9, 30), (10, 31, 80), (17, 6, 50)])
def test_nto_pp_and_hh_roots(mult, case):
    nocc, nvir, naux = case
    note("nto", mult, case)
    eps = gen.orbital_energies(61, nocc, nvir)
    L = gen.lpq_full(61, nocc + nvir, naux)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        rp = ctx.davidson(4, block=4, tol=1e-10, vectors=True)
        rh = ctx.davidson(3, block=3, tol=1e-10, vectors=True, channel="hh")
        resp = ctx.nto(rp["vecs"])
        resh = ctx.nto(rh["vecs"])
    check_against_oracle(rp["vecs"], resp, nvir, nocc, mult, +1.0)
    check_against_oracle(rh["vecs"], resh, nvir, nocc, mult, -1.0)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_nto_active_window_device_vectors(mult):
    import torch
    note("nto window", mult)
    nocc, nvir, naux = 12, 40, 90
    eps = gen.orbital_energies(62, nocc, nvir)
    L = gen.lpq_full(62, nocc + nvir, naux)
    with P.PpRPA(eps, L, nocc, mult=mult, nocc_act=7, nvir_act=15) as ctx:
        r = ctx.davidson(3, block=3, tol=1e-10, vectors=True)
        zd = torch.from_numpy(r["vecs"]).to("cuda:0")
        res = ctx.nto(zd)
    check_against_oracle(r["vecs"], res, 15, 7, mult, +1.0)


def test_nto_zero_interaction():
    note("nto L = 0")
    nocc, nvir, naux = 5, 9, 4
    eps = gen.orbital_energies(63, nocc, nvir)
    L = np.zeros((naux, nocc + nvir, nocc + nvir))
    with P.PpRPA(eps, L, nocc) as ctx:
        r = ctx.davidson(4, block=4, tol=1e-12, vectors=True)
        res = ctx.nto(r["vecs"], density=False)
    for j in range(4):
        assert np.allclose(res["lam_p"][j], np.r_[1.0, np.zeros(nvir - 1)], atol=1e-12)
        assert np.allclose(res["lam_h"][j], 0.0, atol=1e-24)


def test_nto_argument_checks():
    note("nto argument checks")
    eps = gen.orbital_energies(64, 3, 6)
    L = gen.lpq_full(64, 9, 10)
    with P.PpRPA(eps, L, 3) as ctx:
        with pytest.raises(P.PpRPAError) as e:
            ctx.nto(np.zeros((0, ctx.n)))
        assert e.value.status == P.binding.EINVAL


def _signed(u, v):
    """The library's sign convention for a singular pair: the largest |u_i| (lowest i) positive."""
    i = int(np.argmax(np.abs(u)))
    return (u, v) if u[i] >= 0 else (-u, -v)


def _check_vectors(out, j, lam, U, V, tol=1e-9, wkey=("c_p1", "c_p2")):
    """Returned pairs against the oracle's where the weight is nonzero and isolated; every
    returned pair orthonormal where nonzero."""
    nvec = out[wkey[0]].shape[1]
    for q in range(min(nvec, lam.size, U.shape[1], V.shape[1])):
        gap = min([abs(lam[q] - lam[p]) for p in range(lam.size) if p != q] + [1.0])
        if lam[q] < 1e-8 or gap < 1e-6 * max(lam[0], 1e-300):
            continue
        u, v = _signed(U[:, q], V[:, q])
        assert np.max(np.abs(out[wkey[0]][j, q] - u)) <= tol
        assert np.max(np.abs(out[wkey[1]][j, q] - v)) <= tol


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(4, 9, 30), (6, 14, 40)])
def test_nto_vectors_vs_oracle(mult, case):
    """pprpa_nto_vectors: the leading NTO pairs of pp and hh roots and of random vectors against
    the oracle's SVD (sign convention applied to both, pairs with nonzero isolated weights), and
    the full set reconstructing X and Y: X = sum_q sqrt(lam_q) c_p1[q] c_p2[q]^T (null directions
    contribute zero); the leading three equal the first three of the full set."""
    nocc, nvir, naux = case
    note("nto vectors", mult, case)
    eps, L = gen.orbital_energies(61, nocc, nvir), gen.lpq_full(61, nocc + nvir, naux)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        zs = [ctx.davidson(3, direct=True, vectors=True)["vecs"],
              ctx.davidson(2, direct=True, vectors=True, channel="hh")["vecs"],
              gen.random_vectors(62, 2, ctx.n)]
        Z = np.vstack(zs)
        full = ctx.nto_vectors(Z, max(nvir, nocc))
        lead = ctx.nto_vectors(Z, 3)
        w = ctx.nto(Z, density=False)
    nvv = O.pairs(nvir, mult)[0].size
    for j, z in enumerate(Z):
        lp, lh, (U, V, Uh, Vh) = O.nto(z, nvir, nocc, mult)
        _check_vectors(lead, j, lp, U, V)
        _check_vectors(lead, j, lh, Uh, Vh, wkey=("c_h1", "c_h2"))
        X = O.triangular(z[:nvv], nvir, mult)
        Y = O.triangular(z[nvv:], nocc, mult)
        Xr = (full["c_p1"][j].T * np.sqrt(w["lam_p"][j])) @ full["c_p2"][j][:nvir]
        Yr = (full["c_h1"][j][:nocc].T * np.sqrt(w["lam_h"][j])) @ full["c_h2"][j][:nocc]
        assert np.max(np.abs(Xr[:, :] - X)) <= 1e-10 * max(1.0, np.abs(X).max())
        assert np.max(np.abs(Yr - Y)) <= 1e-10 * max(1.0, np.abs(Y).max())
        assert np.allclose(lead["c_p1"][j], full["c_p1"][j][:3], atol=1e-9)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_nto_largest_block(mult):
    """Both NTO entry points at their block limit (nv = 512) on random vectors: weights and
    density blocks against the oracle's SVD and densities, the leading pairs against the oracle's
    singular vectors."""
    nocc, nvir, naux = 3, 512, 8
    note("nto at nv = 512", mult)
    eps, L = gen.orbital_energies(65, nocc, nvir), gen.lpq_full(65, nocc + nvir, naux)
    with P.PpRPA(eps, L, nocc, mult=mult) as ctx:
        Z = gen.random_vectors(66, 2, ctx.n)
        res = ctx.nto(Z)
        out = ctx.nto_vectors(Z, 4)
    for j, z in enumerate(Z):
        lp, lh, (U, V, Uh, Vh) = O.nto(z, nvir, nocc, mult)
        Dv, Do = O.density_2e(z, nvir, nocc, mult)
        assert np.max(np.abs(res["lam_p"][j] - lp)) <= 1e-12 * lp.max()
        assert np.max(np.abs(res["lam_h"][j] - lh)) <= 1e-12 * max(lh.max(), 1e-300)
        assert np.max(np.abs(res["d_vv"][j] - Dv)) <= 1e-12 * np.abs(Dv).max()
        assert np.max(np.abs(res["d_oo"][j] - Do)) <= 1e-12 * max(np.abs(Do).max(), 1e-300)
        _check_vectors(out, j, lp, U, V)
        _check_vectors(out, j, lh, Uh, Vh, wkey=("c_h1", "c_h2"))


def test_nto_vectors_alpha_beta_vs_oracle():
    """The same for alpha-beta roots (rectangular blocks: alpha longer than beta, then shorter)."""
    for nmo, noa, nob in ((12, 4, 2), (10, 2, 5)):
        ea = gen.orbital_energies(63, noa, nmo - noa)
        eb = gen.orbital_energies(1063, nob, nmo - nob)
        La, Lb = gen.lpq_full(63, nmo, 16), gen.lpq_full(1063, nmo, 16)
        nva, nvb = nmo - noa, nmo - nob
        with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
            Z = np.vstack([ctx.davidson(2, direct=True, vectors=True)["vecs"],
                           ctx.davidson(2, direct=True, vectors=True, channel="hh")["vecs"],
                           gen.random_vectors(64, 2, ctx.n)])
            out = ctx.nto_vectors(Z, 4)
        for j, z in enumerate(Z):
            lp, lh, (U, V, Uh, Vh) = O.nto_ab(z, nva, nvb, noa, nob)
            _check_vectors(out, j, lp, U, V)
            _check_vectors(out, j, lh, Uh, Vh, wkey=("c_h1", "c_h2"))

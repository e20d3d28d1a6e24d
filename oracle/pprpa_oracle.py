"""FP64 CPU oracle for density-fitted particle-particle RPA (arXiv 2512.12515).

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or executes this file:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it. It shares no code with the HIP path.

It is the plain definition written out in NumPy/SciPy, FP64 throughout:

* the ppRPA generalised eigenproblem  [[A, B], [B^T, C]] [X; Y] = Omega diag(I, -I) [X; Y]
  (section "ppRPA Equation", Eq. eigen_equation);
* the spin-adapted singlet and triplet matrix elements of that section, with the
  physicists' integrals <pq|rs> = (pr|qs) defined beside Eq. dyson;
* density fitting: (pq|rs) = sum_P L^P_pq L^P_rs with the three-centre integrals given in the
  MO basis (section "Implementation Details");
* the normalisation X^T X - Y^T Y = +1 (pp) / -1 (hh) of Eq. xy_norm;
* the correlation energy sum(Omega_pp) - Tr A = -sum(Omega_hh) - Tr C of
  Eq. correlation_energy (section "Total Energy");
* the natural transition orbitals (section "Natural Transition Orbital", Eqs. nto_pp and
  nto_hh) and the two-electron part of the density matrix (section "Density Matrix");
* spin-unrestricted ppRPA in its three spin sectors (section "Implementation Details");
* the canonical active window (section "ppRPA Equation", last paragraph; section
  "Implementation Details"): the highest occupied and lowest virtual orbitals.

Readings where the paper is silent (listed with reasons in the design notes):
* pair order: upper triangle, row-major; singlet (p <= q), triplet (p < q); z = [x; y];
* "lowest roots" are the smallest Omega among eigenvectors with z^T W z = +1;
* the NTO amplitude matrices are the packed amplitudes placed on the upper triangle (p <= q,
  p < q for the triplet), as the section describes them; the weights are the squared singular
  values, so sum(lam^p) - sum(lam^h) = x^T x - y^T y;
* the hh channel (two-electron removal, z^T W z = -1) returns the roots nearest the gap, i.e.
  the largest Omega_hh first (the states of the (N-2)-electron system closest to its ground
  state);
* the pencil is solved through the definite shift K = M - 2 mu W (mu = mid-gap), which is
  positive definite for the synthetic inputs; the general non-symmetric solver (route G)
  serves as the cross-check on small inputs.

Pinned by tests/test_oracle_pins.py (closed forms, sum rules, spin-orbital equivalence,
the second-order MP2 limit, the two-electron CI limit); see that file.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

SQRT2 = np.sqrt(2.0)


# ----------------------------------------------------------------------------------------
# Active space and pair bookkeeping
# ----------------------------------------------------------------------------------------

def active_space(eps, L, nocc, nocc_act=None, nvir_act=None, lpq_is_active=False):
    """Slice the canonical active window.

    eps: [nmo] orbital energies (occupied first, each block ascending).
    L:   [naux, nmo, nmo] (or [naux, nact, nact] when lpq_is_active).
    Returns dict with eo [no], ev [nv], Loo [naux,no,no], Lov [naux,no,nv], Lvv [naux,nv,nv].
    """
    eps = np.asarray(eps, dtype=np.float64)
    nmo = eps.size
    nvir = nmo - nocc
    no = nocc if not nocc_act or nocc_act <= 0 else min(nocc_act, nocc)
    nv = nvir if not nvir_act or nvir_act <= 0 else min(nvir_act, nvir)
    occ = np.arange(nocc - no, nocc)
    vir = np.arange(nocc, nocc + nv)
    if lpq_is_active:
        assert L.shape[1] == no + nv
        o_l, v_l = np.arange(no), np.arange(no, no + nv)
    else:
        assert L.shape[1] == nmo
        o_l, v_l = occ, vir
    L = np.asarray(L, dtype=np.float64)
    return dict(
        eo=eps[occ].copy(), ev=eps[vir].copy(),
        Loo=L[:, o_l][:, :, o_l], Lov=L[:, o_l][:, :, v_l], Lvv=L[:, v_l][:, :, v_l],
    )


def pairs(n, mult):
    """Packed pair order: (p, q) with p <= q (singlet) or p < q (triplet), p outer."""
    k = 0 if mult == "singlet" else 1
    p, q = np.triu_indices(n, k=k)
    return p, q


def pair_norm(p, q, mult):
    """1/sqrt(1 + delta_pq) for the singlet; 1 for the triplet."""
    if mult == "singlet":
        return np.where(p == q, 1.0 / SQRT2, 1.0)
    return np.ones(p.size)


# ----------------------------------------------------------------------------------------
# Matrix elements
# ----------------------------------------------------------------------------------------

def pair_integrals(L_rc, rp, rq, cp, cq, sign, chunk=256):
    """F[(p,q),(r,s)] = <pq|rs> + sign * <pq|sr>, with <pq|rs> = (pr|qs) = sum_P L^P_pr L^P_qs.

    L_rc: [naux, n_rowspace, n_colspace]: L^P_{p r} for p in the row orbital space and r in
    the column orbital space. (rp, rq): row pairs; (cp, cq): column pairs.
    """
    nr = rp.size
    out = np.empty((nr, cp.size))
    for m0 in range(0, nr, chunk):
        m1 = min(nr, m0 + chunk)
        Lp = np.ascontiguousarray(L_rc[:, rp[m0:m1], :].transpose(1, 2, 0))  # [m, ncol, naux]
        Lq = np.ascontiguousarray(L_rc[:, rq[m0:m1], :].transpose(1, 0, 2))  # [m, naux, ncol]
        g = Lp @ Lq                                                          # g[m, r, s] = (p r|q s)
        out[m0:m1] = g[:, cp, cq] + sign * g[:, cq, cp]
    return out


def build_matrices(sp, mult):
    """Spin-adapted A, B, C of the ppRPA equation for the active space ``sp``.

    singlet: A_ab,cd = d(E_ab) + N_ab N_cd (<ab|cd> + <ab|dc>), pairs a <= b, N = 1/sqrt(1+d)
    triplet: A_ab,cd = d(E_ab) + <ab|cd> - <ab|dc>,             pairs a <  b
    B and C likewise, with C carrying -d(E_ij) on its diagonal.
    """
    eo, ev = sp["eo"], sp["ev"]
    no, nv = eo.size, ev.size
    sign = 1.0 if mult == "singlet" else -1.0
    va, vb = pairs(nv, mult)
    oi, oj = pairs(no, mult)
    nva, noo = pair_norm(va, vb, mult), pair_norm(oi, oj, mult)
    Lvo = sp["Lov"].transpose(0, 2, 1)  # L^P_{a k}
    A = pair_integrals(sp["Lvv"], va, vb, va, vb, sign) * np.outer(nva, nva)
    A[np.diag_indices_from(A)] += ev[va] + ev[vb]
    B = pair_integrals(Lvo, va, vb, oi, oj, sign) * np.outer(nva, noo)
    C = pair_integrals(sp["Loo"], oi, oj, oi, oj, sign) * np.outer(noo, noo)
    C[np.diag_indices_from(C)] -= eo[oi] + eo[oj]
    return A, B, C


def pprpa_matrix(A, B, C):
    return np.block([[A, B], [B.T, C]])


def metric(nvv, noo):
    return np.concatenate([np.ones(nvv), -np.ones(noo)])


def sigma_dense(M, z):
    """sigma = M z (z: [n] or [n, k])."""
    return M @ z


def sigma_rows(sp, mult, rows, z):
    """Selected entries of sigma = M z, computed from the rows of M one by one (any size).

    rows: packed indices into [x; y]; z: [n] vector. Returns sigma[rows]."""
    eo, ev = sp["eo"], sp["ev"]
    no, nv = eo.size, ev.size
    sign = 1.0 if mult == "singlet" else -1.0
    va, vb = pairs(nv, mult)
    oi, oj = pairs(no, mult)
    nva, noo = pair_norm(va, vb, mult), pair_norm(oi, oj, mult)
    nvv = va.size
    x, y = z[:nvv], z[nvv:]
    Lvo = sp["Lov"].transpose(0, 2, 1)
    Lov = sp["Lov"]
    out = np.empty(len(rows))
    for t, r in enumerate(rows):
        if r < nvv:
            a, b = np.array([va[r]]), np.array([vb[r]])
            Arow = pair_integrals(sp["Lvv"], a, b, va, vb, sign)[0] * nva[r] * nva
            Brow = pair_integrals(Lvo, a, b, oi, oj, sign)[0] * nva[r] * noo
            out[t] = (ev[va[r]] + ev[vb[r]]) * x[r] + Arow @ x + Brow @ y
        else:
            s = r - nvv
            i, j = np.array([oi[s]]), np.array([oj[s]])
            BTrow = pair_integrals(Lov, i, j, va, vb, sign)[0] * noo[s] * nva
            Crow = pair_integrals(sp["Loo"], i, j, oi, oj, sign)[0] * noo[s] * noo
            out[t] = BTrow @ x + Crow @ y - (eo[oi[s]] + eo[oj[s]]) * y[s]
    return out


# ----------------------------------------------------------------------------------------
# Solvers of M z = Omega W z
# ----------------------------------------------------------------------------------------

def midgap(sp):
    """mu = (e_HOMO + e_LUMO)/2 over the active orbitals."""
    eo, ev = sp["eo"], sp["ev"]
    if eo.size and ev.size:
        return 0.5 * (eo[-1] + ev[0])
    if ev.size:
        return ev[0] - 1.0
    return eo[-1] + 1.0


class NotDefinite(RuntimeError):
    pass


def solve_definite(M, nvv, mu, nroot=None, channel="pp"):
    """Route D. K = M - 2 mu W = R R^T (Cholesky); G = R^-1 W R^-T (symmetric);
    G u = theta u gives Omega = 2 mu + 1/theta and z = R^-T u / sqrt|theta|, z^T W z = sign(theta).

    With nroot, only the nroot largest theta (channel "pp": the lowest pp roots) or the nroot
    smallest theta (channel "hh": the hh roots nearest 2 mu) are computed.
    Returns (Omega, Z, sign) with Z columns as eigenvectors, sorted by Omega."""
    n = M.shape[0]
    w = metric(nvv, n - nvv)
    K = M - 2.0 * mu * np.diag(w)
    try:
        R = sla.cholesky(K, lower=True)
    except np.linalg.LinAlgError as e:  # pragma: no cover - reported, never silent
        raise NotDefinite(str(e))
    Y = sla.solve_triangular(R, np.diag(w), lower=True)          # R^-1 W
    G = sla.solve_triangular(R, Y.T, lower=True)                 # R^-1 W R^-T
    G = 0.5 * (G + G.T)
    if nroot is None:
        theta, U = sla.eigh(G)
    elif channel == "pp":
        theta, U = sla.eigh(G, subset_by_index=[n - nroot, n - 1])
    else:
        theta, U = sla.eigh(G, subset_by_index=[0, nroot - 1])
    Z = sla.solve_triangular(R, U, lower=True, trans="T") / np.sqrt(np.abs(theta))
    Omega = 2.0 * mu + 1.0 / theta
    order = np.argsort(Omega)
    return Omega[order], Z[:, order], np.sign(theta[order])


def solve_general(M, nvv, imag_tol=1e-10):
    """Route G. Eigen-decomposition of W M (W^-1 = W) by the general solver.
    Returns (Omega, Z, sign) sorted by Omega; raises NotDefinite on complex roots."""
    n = M.shape[0]
    w = metric(nvv, n - nvv)
    ev, V = sla.eig(w[:, None] * M)
    if np.max(np.abs(ev.imag)) > imag_tol * max(1.0, np.max(np.abs(ev.real))):
        raise NotDefinite("complex ppRPA eigenvalues")
    Omega = ev.real
    V = V.real
    nrm = np.einsum("i,ij,ij->j", w, V, V)
    Z = V / np.sqrt(np.abs(nrm))
    order = np.argsort(Omega)
    return Omega[order], Z[:, order], np.sign(nrm[order])


def fix_sign(Z):
    """Sign convention: the largest-magnitude component of each column is positive."""
    idx = np.argmax(np.abs(Z), axis=0)
    s = np.sign(Z[idx, np.arange(Z.shape[1])])
    s[s == 0] = 1.0
    return Z * s


def pp_roots(Omega, Z, sign, nroot):
    sel = np.where(sign > 0)[0][:nroot]
    return Omega[sel], fix_sign(Z[:, sel])


def hh_roots(Omega, Z, sign):
    sel = np.where(sign < 0)[0]
    return Omega[sel], fix_sign(Z[:, sel])


def hh_nearest(Omega, Z, sign, nroot):
    """The nroot two-electron removal (hh) roots nearest the gap: negative norm in Eq. xy_norm,
    largest Omega first (Omega < 2 mu for every hh root)."""
    sel = np.where(sign < 0)[0]
    sel = sel[np.argsort(-Omega[sel], kind="stable")][:nroot]
    return Omega[sel], fix_sign(Z[:, sel])


def correlation_energy(Omega_pp, Omega_hh, A, C):
    """Both expressions of Eq. correlation_energy: (sum pp - Tr A, -sum hh - Tr C)."""
    return np.sum(Omega_pp) - np.trace(A), -np.sum(Omega_hh) - np.trace(C)


# ----------------------------------------------------------------------------------------
# Natural transition orbitals and the two-electron density matrix of a root
# ----------------------------------------------------------------------------------------

def triangular(v, n, mult):
    """The packed pair amplitudes v (pair order of ``pairs``) as the n x n triangular matrix of
    section "Natural Transition Orbital": entry (p, q) for every packed pair, zero elsewhere."""
    T = np.zeros((n, n))
    p, q = pairs(n, mult)
    T[p, q] = v
    return T


def nto(z, nv, no, mult):
    """NTOs of one root z = [x; y] (Eqs. nto_pp, nto_hh): the SVDs X = C^p1 sqrt(lam^p) C^p2^T
    and Y = C^h1 sqrt(lam^h) C^h2^T of the triangular matrices. Returns the weights lam^p (nv)
    and lam^h (no), descending, and the coefficient matrices (C^p1, C^p2, C^h1, C^h2)."""
    nvv = pairs(nv, mult)[0].size
    X = triangular(z[:nvv], nv, mult)
    Y = triangular(z[nvv:], no, mult)
    U, sx, Vt = np.linalg.svd(X)
    Uh, sy, Vht = np.linalg.svd(Y)
    return sx ** 2, sy ** 2, (U, Vt.T, Uh, Vht.T)


def density_2e(z, nv, no, mult):
    """Two-electron addition/removal part of the one-particle density matrix of a root (section
    "Density Matrix"): D_ab = [X X^T + X^T X]_ab, D_ij = -[Y Y^T + Y^T Y]_ij."""
    nvv = pairs(nv, mult)[0].size
    X = triangular(z[:nvv], nv, mult)
    Y = triangular(z[nvv:], no, mult)
    return X @ X.T + X.T @ X, -(Y @ Y.T + Y.T @ Y)


# ----------------------------------------------------------------------------------------
# End-to-end
# ----------------------------------------------------------------------------------------

def solve(eps, L, nocc, mult, nroot, nocc_act=None, nvir_act=None, lpq_is_active=False,
          route="D", vectors=False, channel="pp"):
    """Lowest nroot pp roots (Hartree) of the ppRPA problem, ascending (channel "pp"), or the
    nroot hh roots nearest the gap, descending (channel "hh"); optionally their vectors."""
    sp = active_space(eps, L, nocc, nocc_act, nvir_act, lpq_is_active)
    A, B, C = build_matrices(sp, mult)
    M = pprpa_matrix(A, B, C)
    nvv = A.shape[0]
    if route == "D":
        Om, Z, sg = solve_definite(M, nvv, midgap(sp), nroot=nroot if M.shape[0] > 3000 else None,
                                   channel=channel)
    else:
        Om, Z, sg = solve_general(M, nvv)
    om, z = pp_roots(Om, Z, sg, nroot) if channel == "pp" else hh_nearest(Om, Z, sg, nroot)
    return (om, z) if vectors else om


# ----------------------------------------------------------------------------------------
# Spin-unrestricted ppRPA (section "Implementation Details": the matrix built and diagonalised
# in three spin subspaces). The alpha-alpha and beta-beta sectors have the triplet elements
# (pairs a<b, antisymmetrised integrals) of the one spin's orbitals and integrals, so
# build_matrices(active_space(eps_s, L_s, nocc_s), "triplet") is that sector. The alpha-beta
# sector is below.
# ----------------------------------------------------------------------------------------

def ab_sector(eps_a, eps_b, La, Lb, nocc_a, nocc_b):
    """Alpha-beta sector: pairs (a_alpha, b_beta) and (i_alpha, j_beta), every combination, the
    alpha index outer; <ab|cd> = (ac|bd) = sum_P La^P_ac Lb^P_bd, with no exchange term (its
    partner pairs orbitals of different spin):
        A = d(e^alpha_a + e^beta_b) + (ac|bd),  B = (ai|bj),  C = -d(e^alpha_i + e^beta_j) + (ik|jl).
    Returns (M, nvv) with M = [[A, B], [B^T, C]]."""
    nmo = eps_a.size
    oa, va = slice(0, nocc_a), slice(nocc_a, nmo)
    ob, vb = slice(0, nocc_b), slice(nocc_b, nmo)
    nva, nvb, noa, nob = nmo - nocc_a, nmo - nocc_b, nocc_a, nocc_b
    A = np.einsum("Pac,Pbd->abcd", La[:, va, va], Lb[:, vb, vb]).reshape(nva * nvb, nva * nvb)
    A += np.diag((eps_a[va][:, None] + eps_b[vb][None, :]).ravel())
    B = np.einsum("Pai,Pbj->abij", La[:, va, oa], Lb[:, vb, ob]).reshape(nva * nvb, noa * nob)
    C = np.einsum("Pik,Pjl->ijkl", La[:, oa, oa], Lb[:, ob, ob]).reshape(noa * nob, noa * nob)
    C -= np.diag((eps_a[oa][:, None] + eps_b[ob][None, :]).ravel())
    return pprpa_matrix(A, B, C), nva * nvb


def ab_sigma_rows(eps_a, eps_b, La, Lb, nocc_a, nocc_b, rows, z):
    """Selected entries of sigma = M z in the alpha-beta sector, each from its row of M written
    out (any size): for the pair (a, b),
        sigma = (e^alpha_a + e^beta_b) x_ab + sum_cd (ac|bd) x_cd + sum_kl (ak|bl) y_kl,
    for the pair (i, j),
        sigma = sum_cd (ic|jd) x_cd + sum_kl (ik|jl) y_kl - (e^alpha_i + e^beta_j) y_ij,
    with (pq|rs) = sum_P La^P_pq Lb^P_rs; X is nvir_a x nvir_b and Y nocc_a x nocc_b (the packed
    order of ab_sector, alpha index outer)."""
    nmo = eps_a.size
    nva, nvb = nmo - nocc_a, nmo - nocc_b
    nvv = nva * nvb
    X = z[:nvv].reshape(nva, nvb)
    Y = z[nvv:].reshape(nocc_a, nocc_b)
    va, vb = np.arange(nocc_a, nmo), np.arange(nocc_b, nmo)
    oa, ob = np.arange(nocc_a), np.arange(nocc_b)
    out = np.empty(len(rows))
    for t, r in enumerate(rows):
        if r < nvv:
            p, q = nocc_a + r // nvb, nocc_b + r % nvb
            diag = (eps_a[p] + eps_b[q]) * z[r]
        else:
            p, q = (r - nvv) // nocc_b, (r - nvv) % nocc_b
            diag = -(eps_a[p] + eps_b[q]) * z[r]
        # sum_P [ La^P_{p,vir} X Lb^P_{vir,q} + La^P_{p,occ} Y Lb^P_{occ,q} ]
        vv = np.einsum("Pc,cd,Pd->", La[:, p, va], X, Lb[:, q, vb])
        oo = np.einsum("Pk,kl,Pl->", La[:, p, oa], Y, Lb[:, q, ob]) if Y.size else 0.0
        out[t] = diag + vv + oo
    return out


def midgap_ab(eps_a, eps_b, nocc_a, nocc_b):
    """2 mu between the alpha-beta hh and pp pair energies: mu = (e^a_HOMO + e^b_HOMO +
    e^a_LUMO + e^b_LUMO) / 4 (the restricted mid-gap when alpha = beta)."""
    lumo = eps_a[nocc_a] + eps_b[nocc_b]
    if nocc_a > 0 and nocc_b > 0:
        return 0.25 * (lumo + eps_a[nocc_a - 1] + eps_b[nocc_b - 1])
    return 0.5 * lumo - 1.0


def nto_ab(z, nvir_a, nvir_b, nocc_a, nocc_b):
    """NTOs of one alpha-beta root z = [x; y] (Eqs. nto_pp, nto_hh): the amplitude matrices are
    rectangular here, X nvir_a x nvir_b and Y nocc_a x nocc_b (alpha index outer, the packed
    order of ab_sector), and X = C^p1 sqrt(lam^p) C^p2^T with alpha NTOs C^p1 and beta NTOs C^p2
    (likewise Y). Returns lam^p (nvir_a) and lam^h (nocc_a), descending, the squared singular
    values followed by zeros when the alpha side is the longer one, and (C^p1, C^p2, C^h1, C^h2)."""
    nvv = nvir_a * nvir_b
    X = z[:nvv].reshape(nvir_a, nvir_b)
    Y = z[nvv:].reshape(nocc_a, nocc_b)
    lp, lh = np.zeros(nvir_a), np.zeros(nocc_a)
    U, sx, Vt = np.linalg.svd(X)
    lp[:sx.size] = sx ** 2
    if Y.size:
        Uh, sy, Vht = np.linalg.svd(Y)
        lh[:sy.size] = sy ** 2
    else:
        Uh, Vht = np.eye(nocc_a), np.eye(nocc_b)
    return lp, lh, (U, Vt.T, Uh, Vht.T)


def density_2e_ab(z, nvir_a, nvir_b, nocc_a, nocc_b):
    """Two-electron addition/removal part of the one-particle density of an alpha-beta root
    (section "Density Matrix"), resolved by spin (the pair holds one electron of each):
    D^alpha_vv = X X^T, D^beta_vv = X^T X, D^alpha_oo = -Y Y^T, D^beta_oo = -Y^T Y."""
    nvv = nvir_a * nvir_b
    X = z[:nvv].reshape(nvir_a, nvir_b)
    Y = z[nvv:].reshape(nocc_a, nocc_b)
    return X @ X.T, X.T @ X, -(Y @ Y.T), -(Y.T @ Y)


def solve_ab(eps_a, eps_b, La, Lb, nocc_a, nocc_b, nroot, channel="pp", vectors=False):
    """Lowest nroot pp roots (or the nroot hh roots nearest the gap) of the alpha-beta sector."""
    M, nvv = ab_sector(eps_a, eps_b, La, Lb, nocc_a, nocc_b)
    Om, Z, sg = solve_definite(M, nvv, midgap_ab(eps_a, eps_b, nocc_a, nocc_b))
    om, z = pp_roots(Om, Z, sg, nroot) if channel == "pp" else hh_nearest(Om, Z, sg, nroot)
    return (om, z) if vectors else om


# ----------------------------------------------------------------------------------------
# Independent references used only by the pins
# ----------------------------------------------------------------------------------------

def spin_orbital_matrix_u(eps_a, eps_b, La, Lb, nocc_a, nocc_b):
    """Unrestricted ppRPA matrix in spin orbitals from the general elements (<pq||rs> over spin
    orbitals, (pr|qs) = sum_P L^{s_p P}_pr L^{s_q P}_qs when the spins of p, r and of q, s
    agree, zero otherwise), pairs p<q over all occupied or all virtual spin orbitals. Returns
    (M, nvv). Small sizes only (explicit loops)."""
    nmo = eps_a.size
    eps = (eps_a, eps_b)
    Ls = (La, Lb)
    occ = [(p, 0) for p in range(nocc_a)] + [(p, 1) for p in range(nocc_b)]
    vir = [(p, 0) for p in range(nocc_a, nmo)] + [(p, 1) for p in range(nocc_b, nmo)]

    def phys(p, q, r, s):
        if p[1] != r[1] or q[1] != s[1]:
            return 0.0
        return float(np.dot(Ls[p[1]][:, p[0], r[0]], Ls[q[1]][:, q[0], s[0]]))

    def block(P1, P2):
        out = np.empty((len(P1), len(P2)))
        for x, (p, q) in enumerate(P1):
            for y, (r, s) in enumerate(P2):
                out[x, y] = phys(p, q, r, s) - phys(p, q, s, r)
        return out

    vp = [(a, b) for i, a in enumerate(vir) for b in vir[i + 1:]]
    op = [(a, b) for i, a in enumerate(occ) for b in occ[i + 1:]]
    A = block(vp, vp) + np.diag([eps[a[1]][a[0]] + eps[b[1]][b[0]] for a, b in vp])
    B = block(vp, op)
    C = block(op, op) - np.diag([eps[a[1]][a[0]] + eps[b[1]][b[0]] for a, b in op])
    return pprpa_matrix(A, B, C), len(vp)

def spin_orbital_matrix(sp):
    """ppRPA matrix in spin orbitals from the general (not spin-adapted) elements:
    A_ab,cd = d(e_a+e_b) + <ab||cd>, B_ab,kl = <ab||kl>, C_ij,kl = -d(e_i+e_j) + <ij||kl>,
    pairs a<b, c<d, i<j, k<l over spin orbitals (spatial index * 2 + spin)."""
    eo, ev = sp["eo"], sp["ev"]
    no, nv = eo.size, ev.size
    naux = sp["Lvv"].shape[0]
    n = no + nv
    Lf = np.zeros((naux, n, n))
    Lf[:, :no, :no] = sp["Loo"]
    Lf[:, :no, no:] = sp["Lov"]
    Lf[:, no:, :no] = sp["Lov"].transpose(0, 2, 1)
    Lf[:, no:, no:] = sp["Lvv"]
    eri = np.einsum("Ppq,Prs->pqrs", Lf, Lf)  # (pq|rs)
    e = np.concatenate([eo, ev])
    occ_so = [2 * p + s for p in range(no) for s in (0, 1)]
    vir_so = [2 * p + s for p in range(no, n) for s in (0, 1)]

    def phys(p, q, r, s):  # <pq|rs> = (pr|qs) with spin integration
        if (p % 2 != r % 2) or (q % 2 != s % 2):
            return 0.0
        return eri[p // 2, r // 2, q // 2, s // 2]

    def block(P1, P2):
        out = np.empty((len(P1), len(P2)))
        for x, (p, q) in enumerate(P1):
            for y, (r, s) in enumerate(P2):
                out[x, y] = phys(p, q, r, s) - phys(p, q, s, r)
        return out

    vp = [(a, b) for i, a in enumerate(vir_so) for b in vir_so[i + 1:]]
    op = [(a, b) for i, a in enumerate(occ_so) for b in occ_so[i + 1:]]
    A = block(vp, vp) + np.diag([e[a // 2] + e[b // 2] for a, b in vp])
    B = block(vp, op)
    C = block(op, op) - np.diag([e[a // 2] + e[b // 2] for a, b in op])
    return pprpa_matrix(A, B, C), len(vp)


def rimp2_energy(sp):
    """Closed-shell RI-MP2 correlation energy:
    sum_ijab (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)."""
    eo, ev = sp["eo"], sp["ev"]
    iajb = np.einsum("Pia,Pjb->iajb", sp["Lov"], sp["Lov"])
    den = eo[:, None, None, None] - ev[None, :, None, None] + eo[None, None, :, None] - ev[None, None, None, :]
    return np.sum(iajb * (2.0 * iajb - iajb.transpose(0, 3, 2, 1)) / den)


def two_electron_ci(ev, Lvv):
    """Spectrum of two electrons (one alpha, one beta) in the virtual orbitals:
    H = d_ac d_bd (e_a + e_b) + (ac|bd) over determinants |a alpha, b beta> (Slater-Condon)."""
    nv = ev.size
    H = np.einsum("Pac,Pbd->abcd", Lvv, Lvv).reshape(nv * nv, nv * nv)
    H += np.diag((ev[:, None] + ev[None, :]).ravel())
    return sla.eigvalsh(H)


def sigma_factorised(sp, mult, z):
    """sigma = M z through the density-fitted factorisation (no 4-index tensor):
    unpack the packed x (y) into a full nv x nv (no x no) matrix that is symmetric with
    sqrt(2) on the diagonal (singlet) or antisymmetric (triplet); then
      S_vv = sum_P L_vv X L_vv + L_vo Y L_ov,   S_oo = sum_P L_ov X L_vo + L_oo Y L_oo,
      sigma_x(ab) = E_ab x_ab + N_ab S_vv[a,b],  sigma_y(ij) = -E_ij y_ij + N_ij S_oo[i,j].
    Pinned against the dense definition (sigma_dense) by the tests. z: [n] or [n, k]."""
    eo, ev = sp["eo"], sp["ev"]
    no, nv = eo.size, ev.size
    s = 1.0 if mult == "singlet" else -1.0
    va, vb = pairs(nv, mult)
    oi, oj = pairs(no, mult)
    nvv = va.size
    z2 = z.reshape(z.shape[0], -1)
    out = np.empty_like(z2)
    Lvv, Lov, Loo = sp["Lvv"], sp["Lov"], sp["Loo"]
    Lvo = Lov.transpose(0, 2, 1)
    for c in range(z2.shape[1]):
        x, y = z2[:nvv, c], z2[nvv:, c]
        X = np.zeros((nv, nv))
        X[va, vb] = x
        X[vb, va] = s * x
        Y = np.zeros((no, no))
        Y[oi, oj] = y
        Y[oj, oi] = s * y
        if mult == "singlet":
            X[np.diag_indices(nv)] *= SQRT2
            Y[np.diag_indices(no)] *= SQRT2
        Svv = np.einsum("Pac,cd,Pdb->ab", Lvv, X, Lvv, optimize=True) \
            + np.einsum("Pak,kl,Plb->ab", Lvo, Y, Lov, optimize=True)
        Soo = np.einsum("Pka,ab,Pbl->kl", Lov, X, Lvo, optimize=True) \
            + np.einsum("Pik,kl,Plj->ij", Loo, Y, Loo, optimize=True)
        out[:nvv, c] = (ev[va] + ev[vb]) * x + pair_norm(va, vb, mult) * Svv[va, vb]
        out[nvv:, c] = -(eo[oi] + eo[oj]) * y + pair_norm(oi, oj, mult) * Soo[oi, oj]
    return out.reshape(z.shape)

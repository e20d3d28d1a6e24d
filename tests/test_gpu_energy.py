"""GPU: the ppRPA correlation energy (section "Total Energy", Eq. correlation_energy) from the
whole spectrum of the dense pencil, through the C ABI, against the FP64 oracle.

* both sides of the sum rule (sum of the pp roots - Tr A, -(sum of the hh roots) - Tr C) against
  the oracle's full-spectrum values, both spins, shapes up to n = 456 (one-workgroup solver) and
  at orders 1018, 1071 and 1989 (multi-workgroup solver), and against each other;
* E_c = 0 when L = 0 and when the coupling block B vanishes (L_vo = 0), as the oracle's pin P2,
  with both solvers;
* the closed-shell total E(singlet) + 3 E(triplet) against the oracle's;
* argument checks: no dense build, n > 8192.
Tolerance: 1e-10 Ha absolute (the sums run over up to ~450 roots, each good to ~1e-13); 1e-9 Ha
at order ~1000 (twice the roots, the reduction's rounding growing with the order).
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


def oracle_ec(eps, L, nocc, mult):
    sp = O.active_space(eps, L, nocc)
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    Om, Z, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
    return O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C), int(np.sum(sg > 0)), int(np.sum(sg < 0))


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
@pytest.mark.parametrize("case", [(5, 20, 100), (3, 8, 25), (12, 10, 60), (6, 29, 90)])
def test_correlation_energy_vs_oracle(mult, case):
    nocc, nvir, naux = case
    note("E_c", mult, case)
    eps = gen.orbital_energies(51, nocc, nvir)
    L = gen.lpq_full(51, nocc + nvir, naux)
    (ref_pp, ref_hh), npp, nhh = oracle_ec(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        assert ctx.n <= 512
        r = ctx.correlation_energy()
    assert r["n_pp_roots"] == npp == ctx.n_pp and r["n_hh_roots"] == nhh == ctx.n_hh
    assert abs(r["ec_pp"] - ref_pp) <= 1e-10
    assert abs(r["ec_hh"] - ref_hh) <= 1e-10
    assert abs(r["ec_pp"] - r["ec_hh"]) <= 1e-10
    assert r["ec_pp"] < 0.0


@pytest.mark.parametrize("mult,nvir", [("singlet", 45), ("triplet", 45), ("singlet", 62)])
def test_correlation_energy_order_above_1000(mult, nvir):
    """Orders above the one-workgroup solver's 512 (the multi-workgroup whole-spectrum solve):
    8 occupied and 45 virtual orbitals, n = 1071 (singlet) and 1018 (triplet); 62 virtual,
    n = 1989."""
    nocc, naux = 8, 150
    note("E_c order > 1000", mult, nvir)
    eps = gen.orbital_energies(54, nocc, nvir)
    L = gen.lpq_full(54, nocc + nvir, naux)
    (ref_pp, ref_hh), npp, nhh = oracle_ec(eps, L, nocc, mult)
    with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
        assert ctx.n > 1000
        r = ctx.correlation_energy()
    note("ec_pp", r["ec_pp"], "oracle", ref_pp, "diff", r["ec_pp"] - ref_pp)
    assert r["n_pp_roots"] == npp and r["n_hh_roots"] == nhh
    assert abs(r["ec_pp"] - ref_pp) <= 1e-9
    assert abs(r["ec_hh"] - ref_hh) <= 1e-9
    assert abs(r["ec_pp"] - r["ec_hh"]) <= 1e-9


@pytest.mark.parametrize("mult,nvir", [("singlet", 14), ("triplet", 14), ("singlet", 40)])
def test_correlation_energy_vanishes_without_coupling(mult, nvir):
    """nvir 40: n = 835, the multi-workgroup solve."""
    note("E_c B = 0", mult, nvir)
    nocc, naux = 5, 40
    eps = gen.orbital_energies(52, nocc, nvir)
    L = gen.lpq_full(52, nocc + nvir, naux)
    L[:, :nocc, nocc:] = 0.0
    L[:, nocc:, :nocc] = 0.0
    Lz = np.zeros_like(L)
    for LL in (L, Lz):
        with P.PpRPA(eps, LL, nocc, mult=mult, dense=True) as ctx:
            r = ctx.correlation_energy()
        assert abs(r["ec_pp"]) <= 1e-11 and abs(r["ec_hh"]) <= 1e-11


def test_closed_shell_total():
    note("E_c closed shell")
    nocc, nvir, naux = 5, 20, 100
    eps = gen.orbital_energies(0, nocc, nvir)
    L = gen.lpq_full(0, nocc + nvir, naux)
    tot, ref = 0.0, 0.0
    for mult, w in (("singlet", 1.0), ("triplet", 3.0)):
        with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
            tot += w * ctx.correlation_energy()["ec_pp"]
        ref += w * oracle_ec(eps, L, nocc, mult)[0][0]
    assert abs(tot - ref) <= 1e-10


def test_correlation_energy_argument_checks():
    note("E_c argument checks")
    eps = gen.orbital_energies(53, 4, 10)
    L = gen.lpq_full(53, 14, 20)
    with P.PpRPA(eps, L, 4) as ctx:
        with pytest.raises(P.PpRPAError) as e:
            ctx.correlation_energy()
        assert e.value.status == P.binding.EUNSUPPORTED
    eps = gen.orbital_energies(53, 4, 130)
    L = gen.lpq_full(53, 134, 20)
    with P.PpRPA(eps, L, 4, dense=True) as ctx:
        assert ctx.n > 8192
        with pytest.raises(P.PpRPAError) as e:
            ctx.correlation_energy()
        assert e.value.status == P.binding.EUNSUPPORTED

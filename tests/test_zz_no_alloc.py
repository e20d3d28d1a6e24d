"""GPU: pprpa_correlation_energy_noalloc, the correlation energy (section "Total Energy", Eq.
correlation_energy) with its workspace in the library's static device array instead of a
device allocation per call, against pprpa_correlation_energy on the same contexts: two calls in
a row (the second on a smaller problem, so the array holds the first call's larger contents),
each bit for bit equal to the allocating entry point and within 1e-10 Ha of the oracle; orders
beyond the array's 512 are refused."""
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


def oracle_energy(eps, L, nocc, mult):
    sp = O.active_space(eps, L, nocc)
    A, B, C = O.build_matrices(sp, mult)
    M = O.pprpa_matrix(A, B, C)
    om, _, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
    return O.correlation_energy(om[sg > 0], om[sg < 0], A, C)[0]


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_noalloc_energy_equals_allocating_entry_point(order):
    cases = [(51, 8, 30, 60, "singlet"), (52, 3, 12, 40, "triplet")]  # n = 501, then 69
    if order == "small_then_large":
        cases = cases[::-1]
    for seed, nocc, nvir, naux, mult in cases:
        note("noalloc energy", seed, nocc, nvir, naux, mult)
        eps, L = gen.orbital_energies(seed, nocc, nvir), gen.lpq_full(seed, nocc + nvir, naux)
        with P.PpRPA(eps, L, nocc, mult=mult, dense=True) as ctx:
            got = ctx.correlation_energy(noalloc=True)
            ref = ctx.correlation_energy()
            again = ctx.correlation_energy(noalloc=True)
        assert got == ref and again == ref, (got, ref, again)
        ec = oracle_energy(eps, L, nocc, mult)
        assert abs(got["ec_pp"] - ec) <= 1e-10 and abs(got["ec_hh"] - ec) <= 1e-10


def test_noalloc_energy_refuses_orders_beyond_its_array():
    eps, L = gen.orbital_energies(53, 8, 32), gen.lpq_full(53, 40, 50)  # singlet n = 528 + 36
    with P.PpRPA(eps, L, 8, dense=True) as ctx:
        assert ctx.n > 512
        with pytest.raises(P.PpRPAError) as e:
            ctx.correlation_energy(noalloc=True)
    assert e.value.status == P.binding.EUNSUPPORTED and "512" in str(e.value)

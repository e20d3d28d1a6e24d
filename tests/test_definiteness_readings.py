"""Why the large workloads solve the pencil with the integrals scaled by 0.7 (CPU, oracle only).

Eq. eigen_equation with the metric of Eq. xy_norm has well-defined "lowest pp roots" only when
the pencil (M, W) is definite: some shift 2 mu makes M - 2 mu W positive definite, the spectrum
is real, and the pp roots are the eigenvectors with z^T W z = +1. A pencil with complex
eigenvalues is definite for no shift at all.

With the generator's integrals (each entry N(0, 0.09 / naux)), the pair interaction
(ac|bd) = sum_P L^P_ac L^P_bd has elements of standard deviation 0.09 / sqrt(naux) over about
nv^2 / 2 pairs, so its spread grows as nv / sqrt(naux) against the fixed range of the pair
energies e_a + e_b. The dense oracle cannot reach 50 / 500 / 1800 (order 126525) or the
40 + 400 window of 120 / 1500 / 4000 (order 80580); these tests take analogues that keep
nv / sqrt(naux) and the orbital-energy range of the active orbitals and shrink the orbital
counts:

* 50 / 500 / 1800, singlet: nv / sqrt(naux) = 11.8 over the full virtual range [0, 3] Ha
  -> 6 / 60 / 26 (60 / sqrt(26) = 11.8);
* the 40 + 400 window of 120 / 1500 / 4000, triplet: nv / sqrt(naux) = 6.3, the window's virtual
  orbitals spanning 400 * 3 / 1500 = 0.8 Ha -> the 4 + 40 window of 12 / 150 / 40
  (40 / sqrt(40) = 6.3; 40 * 3 / 150 = 0.8 Ha);
* the largest serving request, 40 / 400 / 1540: nv / sqrt(naux) = 10.2 -> 6 / 60 / 35;
* control, 20 / 200 / 700 (which the oracle solves directly: definite, both spins):
  nv / sqrt(naux) = 7.6 -> 6 / 60 / 63.

Unscaled, the analogues of the first two have complex roots (no shift is definite) and fail the
Cholesky of M - 2 mu W; with the integrals scaled by 0.7 every one is definite with margin and
the definite route (Cholesky + eigh) agrees with the general eigensolver. The serving analogue
sits at the border (complex roots for some seeds), and is definite for every seed at 0.7. The
control is definite unscaled, as 20 / 200 / 700 itself is.
"""
import numpy as np
import pytest

from oracle import pprpa_oracle as O
from workloads import gen


def pencil(nocc, nvir, naux, mult, seed, scale, no=None, nv=None):
    eps = gen.orbital_energies(seed, nocc, nvir)
    La = gen.lpq_active(seed, nocc, nvir, naux, no, nv) * scale
    sp = O.active_space(eps, La, nocc, nocc_act=no, nvir_act=nv, lpq_is_active=True)
    A, B, C = O.build_matrices(sp, mult)
    return O.pprpa_matrix(A, B, C), A.shape[0], O.midgap(sp)


def lowest_shifted(M, nvv, mu):
    """Lowest eigenvalue of M - 2 mu W."""
    w = O.metric(nvv, M.shape[0] - nvv)
    return np.linalg.eigvalsh(M - 2.0 * mu * np.diag(w))[0]


def assert_not_definite(M, nvv, mu):
    with pytest.raises(O.NotDefinite):
        O.solve_definite(M, nvv, mu)
    with pytest.raises(O.NotDefinite):  # complex roots: no shift makes the pencil definite
        O.solve_general(M, nvv)


def assert_definite(M, nvv, mu, margin):
    assert lowest_shifted(M, nvv, mu) >= margin
    om_d, _, sg_d = O.solve_definite(M, nvv, mu)
    om_g, _, sg_g = O.solve_general(M, nvv)
    assert np.array_equal(sg_d, sg_g)
    assert np.max(np.abs(om_d - om_g)) <= 1e-10 * np.abs(om_d).max()
    assert np.sum(sg_d > 0) == nvv  # as many pp roots as particle pairs


ANALOGUES = {
    # name: (nocc, nvir, naux, mult, nocc_act, nvir_act)
    "mixed_50x500x1800": (6, 60, 26, "singlet", None, None),
    "active_40+400_of_120x1500x4000": (12, 150, 40, "triplet", 4, 40),
}


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("name", sorted(ANALOGUES))
def test_large_workload_analogue_indefinite_unscaled_definite_at_0p7(name, seed):
    nocc, nvir, naux, mult, no, nv = ANALOGUES[name]
    M, nvv, mu = pencil(nocc, nvir, naux, mult, seed, 1.0, no, nv)
    assert lowest_shifted(M, nvv, mu) < 0.0
    assert_not_definite(M, nvv, mu)
    M, nvv, mu = pencil(nocc, nvir, naux, mult, seed, gen.CONFIGS[
        "mixed" if name.startswith("mixed") else "active"]["eig_scale"], no, nv)
    assert_definite(M, nvv, mu, margin=0.1)


@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_serving_mix_largest_request_analogue(mult):
    """Unscaled, the analogue of the mix's largest request is indefinite (complex roots) for
    some seeds; scaled by the mix's eig_scale it is definite for every seed tried."""
    scale = gen.serve_requests(0, 1)[0]["eig_scale"]
    complex_seen = 0
    for seed in range(3):
        M, nvv, mu = pencil(6, 60, 35, mult, seed, 1.0)
        try:
            O.solve_general(M, nvv)
        except O.NotDefinite:
            complex_seen += 1
        M, nvv, mu = pencil(6, 60, 35, mult, seed, scale)
        assert_definite(M, nvv, mu, margin=0.1)
    assert complex_seen >= 1


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("mult", ["singlet", "triplet"])
def test_control_analogue_of_the_fp64_davidson_workload_is_definite(mult, seed):
    """The same construction applied to 20 / 200 / 700, which the oracle solves directly (its
    golden roots come from the definite route), gives a definite pencil unscaled: the analogue
    rule separates the workloads the way the full-size pencils do."""
    M, nvv, mu = pencil(6, 60, 63, mult, seed, 1.0)
    assert_definite(M, nvv, mu, margin=0.1)

"""Seeded input generators: determinism, slicing, symmetry and moments (CPU)."""
import numpy as np

from workloads import gen


def test_deterministic_and_seed_dependent():
    a = gen.lpq_full(0, 7, 5)
    b = gen.lpq_full(0, 7, 5)
    c = gen.lpq_full(1, 7, 5)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    e0 = gen.orbital_energies(3, 4, 9)
    assert np.array_equal(e0, gen.orbital_energies(3, 4, 9))


def test_symmetric_in_pq():
    L = gen.lpq_full(2, 11, 6)
    assert np.array_equal(L, L.transpose(0, 2, 1))


def test_active_slice_equals_full_slice():
    nocc, nvir, naux = 6, 13, 9
    L = gen.lpq_full(5, nocc + nvir, naux)
    idx = gen.active_indices(nocc, nvir, 3, 7)
    assert list(idx) == [3, 4, 5, 6, 7, 8, 9, 10, 11, 12]
    La = gen.lpq_active(5, nocc, nvir, naux, 3, 7)
    assert np.array_equal(La, L[:, idx][:, :, idx])


def test_energy_ranges_sorted():
    e = gen.orbital_energies(0, 50, 500)
    eo, ev = e[:50], e[50:]
    assert np.all(np.diff(eo) >= 0) and np.all(np.diff(ev) >= 0)
    assert eo.min() >= -1.0 and eo.max() <= -0.3
    assert ev.min() >= 0.0 and ev.max() <= 3.0


def test_moments():
    naux = 400
    L = gen.lpq_full(7, 40, naux)
    iu = np.triu_indices(40)
    v = L[:, iu[0], iu[1]].ravel() / gen.lpq_scale(naux)  # independent N(0,1) entries
    assert abs(v.mean()) < 0.01
    assert abs(v.var() - 1.0) < 0.01
    # off-diagonal entries carry the same variance as diagonal ones (mirror, not (G+G^T)/2)
    off = L[:, 0, 1:].ravel() / gen.lpq_scale(naux)
    assert abs(off.var() - 1.0) < 0.05
    # fourth moment of a normal is 3
    assert abs(np.mean(v ** 4) - 3.0) < 0.05


def test_serve_mix():
    reqs = gen.serve_requests(0, 512)
    assert len(reqs) == 512
    no = np.array([r["nocc"] for r in reqs])
    nv = np.array([r["nvir"] for r in reqs])
    assert no.min() >= 4 and no.max() <= 40 and nv.min() >= 30 and nv.max() <= 400
    assert all(r["naux"] == (7 * (r["nocc"] + r["nvir"]) + 1) // 2 for r in reqs)
    frac_s = np.mean([r["mult"] == "singlet" for r in reqs])
    assert 0.4 < frac_s < 0.6
    t = gen.poisson_arrivals(0, 512, 10.0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 512 - 0.1) < 0.02


def test_torch_generator_matches_numpy():
    import torch
    nmo, naux = 23, 7
    rows, cols, aux = np.arange(3, 15), np.arange(nmo), np.arange(2, 6)
    a = gen.lpq_block(4, nmo, naux, rows, cols, aux=aux)
    b = gen.lpq_block_torch(4, nmo, naux, rows, cols, aux, device="cpu").numpy()
    assert np.allclose(a, b, rtol=1e-14, atol=0)
    # the integer hash itself is bit-identical
    c = np.arange(1000, dtype=np.uint64) * np.uint64(7919) + np.uint64(2 ** 62)
    ref = gen.uniform(3, gen.STREAM_LPQ, c)
    got = gen._uniform_t(3, gen.STREAM_LPQ, torch.as_tensor(c.astype(np.int64))).numpy()
    assert np.array_equal(ref, got)

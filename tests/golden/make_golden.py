"""Write the oracle's expected eigenvalues for the seeded workloads to tests/golden/*.json.

Calls only ``oracle/`` (the FP64 dense definition, route D) and ``workloads/`` (inputs). The
paper prints no worked example for this path, so every stored value here is the oracle's.

    python tests/golden/make_golden.py small      # 5 x 20 x 100, seeds 0-4, both spins (seconds)
    python tests/golden/make_golden.py davidson   # 20 x 200 x 700, seed 0, both spins (minutes)
    python tests/golden/make_golden.py hh         # the same, hh channel (minutes)
    python tests/golden/make_golden.py energy     # correlation energies, 5 x 20 x 100 (seconds)
    python tests/golden/make_golden.py unrestricted  # three spin sectors, nmo 60 (seconds)
    python tests/golden/make_golden.py serving    # small requests of the serving mix (minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pprpa_oracle as O  # noqa: E402
from workloads import gen  # noqa: E402


def run(name, nocc, nvir, naux, seeds, mults, nroot, channel="pp"):
    out = dict(
        source="oracle/pprpa_oracle.py, dense build + route D (Cholesky of M - 2 mu W, eigh)",
        channel=channel,
        inputs=f"workloads/gen.py: orbital_energies(seed, {nocc}, {nvir}), lpq_full(seed, {nocc + nvir}, {naux})",
        units="Hartree", nocc=nocc, nvir=nvir, naux=naux, nroot=nroot, roots={})
    for seed in seeds:
        eps = gen.orbital_energies(seed, nocc, nvir)
        L = gen.lpq_full(seed, nocc + nvir, naux)
        for mult in mults:
            t = time.time()
            om = O.solve(eps, L, nocc, mult, nroot, channel=channel)
            out["roots"][f"{seed}/{mult}"] = [float(x) for x in om]
            print(name, seed, mult, f"{time.time() - t:.1f}s", om[:3], flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


def run_energy(name, nocc, nvir, naux, seeds):
    """Correlation energy of Eq. correlation_energy per spin block, from the oracle's whole
    spectrum (both sides of the sum rule), and the closed-shell total E_s + 3 E_t."""
    out = dict(source="oracle/pprpa_oracle.py: dense build, route D full spectrum, correlation_energy",
               inputs=f"workloads/gen.py: orbital_energies(seed, {nocc}, {nvir}), lpq_full(seed, {nocc + nvir}, {naux})",
               units="Hartree", nocc=nocc, nvir=nvir, naux=naux, energies={})
    for seed in seeds:
        eps = gen.orbital_energies(seed, nocc, nvir)
        L = gen.lpq_full(seed, nocc + nvir, naux)
        sp = O.active_space(eps, L, nocc)
        e = {}
        for mult in ("singlet", "triplet"):
            A, B, C = O.build_matrices(sp, mult)
            M = O.pprpa_matrix(A, B, C)
            Om, Z, sg = O.solve_definite(M, A.shape[0], O.midgap(sp))
            ec_pp, ec_hh = O.correlation_energy(Om[sg > 0], Om[sg < 0], A, C)
            e[mult] = [float(ec_pp), float(ec_hh)]
        e["closed_shell"] = e["singlet"][0] + 3.0 * e["triplet"][0]
        out["energies"][str(seed)] = e
        print(name, seed, e, flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


def run_unrestricted(name, nmo, nocc_a, nocc_b, naux, seed, nroot):
    """Lowest nroot pp roots of each spin sector of unrestricted ppRPA and of all three together
    (alpha = seed, beta = seed + 1000 of the same generators)."""
    ea = gen.orbital_energies(seed, nocc_a, nmo - nocc_a)
    eb = gen.orbital_energies(seed + 1000, nocc_b, nmo - nocc_b)
    La = gen.lpq_full(seed, nmo, naux)
    Lb = gen.lpq_full(seed + 1000, nmo, naux)
    out = dict(source="oracle/pprpa_oracle.py: triplet sectors (build_matrices) and ab_sector, route D",
               inputs=f"workloads/gen.py: alpha orbital_energies({seed}, {nocc_a}, {nmo - nocc_a}), "
                      f"lpq_full({seed}, {nmo}, {naux}); beta the same with seed {seed + 1000} and nocc {nocc_b}",
               units="Hartree", nmo=nmo, nocc_a=nocc_a, nocc_b=nocc_b, naux=naux, seed=seed,
               nroot=nroot, roots={})
    for label, e_s, L_s, no_s in (("aa", ea, La, nocc_a), ("bb", eb, Lb, nocc_b)):
        out["roots"][label] = [float(x) for x in O.solve(e_s, L_s, no_s, "triplet", nroot)]
    out["roots"]["ab"] = [float(x) for x in O.solve_ab(ea, eb, La, Lb, nocc_a, nocc_b, nroot)]
    out["roots"]["all"] = sorted(out["roots"]["aa"] + out["roots"]["bb"] + out["roots"]["ab"])[:nroot]
    print(name, out["roots"]["all"][:3], flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


def run_serving(name, count, max_nmo):
    """Roots of every request of the serving mix (gen.serve_requests(0, count)) with at most
    max_nmo orbitals, integrals scaled by the request's eig_scale."""
    out = dict(source="oracle/pprpa_oracle.py, dense build + route D",
               inputs=f"workloads/gen.py: serve_requests(0, {count}); request r: orbital_energies(r, nocc, "
                      "nvir), lpq_full(r, nocc + nvir, naux) * eig_scale",
               units="Hartree", count=count, max_nmo=max_nmo, roots={})
    for r in gen.serve_requests(0, count):
        if r["nocc"] + r["nvir"] > max_nmo:
            continue
        eps = gen.orbital_energies(r["seed"], r["nocc"], r["nvir"])
        L = gen.lpq_full(r["seed"], r["nocc"] + r["nvir"], r["naux"]) * r["eig_scale"]
        om = O.solve(eps, L, r["nocc"], r["mult"], r["nroot"])
        out["roots"][str(r["rid"])] = [float(x) for x in om]
    print(name, len(out["roots"]), "requests", flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["small"]
    if "small" in which:
        run("small_direct", 5, 20, 100, (0, 1, 2, 3, 4), ("singlet", "triplet"), 5)
    if "davidson" in which:
        run("davidson_fp64", 20, 200, 700, (0,), ("singlet", "triplet"), 10)
    if "serving" in which:
        run_serving("serving_small", 512, 100)
    if "unrestricted" in which:
        run_unrestricted("unrestricted", 60, 10, 9, 200, 0, 8)
    if "energy" in which:
        run_energy("correlation_energy", 5, 20, 100, (0, 1, 2, 3, 4))
    if "hh" in which:
        run("davidson_hh_fp64", 20, 200, 700, (0,), ("singlet", "triplet"), 10, channel="hh")

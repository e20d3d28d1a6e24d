"""GPU: boundary behaviour of the C ABI beyond the arithmetic.

* EBUSY: a context is used by one thread at a time; a call from a second thread while the first
  is inside pprpa_davidson returns EBUSY at once (and the first call is unaffected);
* warm start: the converged vectors passed back as `guess` reach the same roots in at most two
  iterations;
* a start block of 128 and of 256 guesses (wider than any correction block): the oracle's roots;
* the per-iteration log callback: one JSON object per Davidson iteration, in order, whose last
  line agrees with the report;
* a solve with the roctx ranges switched on (PPRPA_ROCTX=1, no profiler attached);
* the caller-driven solve (pprpa_solve_begin / _iterate / _end): driven to convergence one
  iteration at a time it returns bitwise what pprpa_davidson returns; it holds the context
  (EBUSY for other calls) until ended; ended early it reports ENOCONV with the last iterate.
"""
import json
import sys
import threading

import numpy as np
import pytest

from oracle import pprpa_oracle as O
from workloads import gen
import paper_2512_12515_amd as P

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(seed, nocc, nvir, naux):
    return gen.orbital_energies(seed, nocc, nvir), gen.lpq_full(seed, nocc + nvir, naux)


def test_second_thread_gets_ebusy():
    note("EBUSY")
    eps, L = problem(41, 6, 30, 60)
    ref = O.solve(eps, L, 6, "singlet", 5)
    inside, released = threading.Event(), threading.Event()
    seen = {}

    def on_iteration(line):
        # called by the library from inside pprpa_davidson (the context is held): let the other
        # thread try the context once, then continue
        if not inside.is_set():
            inside.set()
            released.wait(timeout=60.0)

    def other(ctx, z):
        inside.wait(timeout=60.0)
        try:
            ctx.matvec(z)
            seen["status"] = P.binding.OK
        except P.PpRPAError as e:
            seen["status"] = e.status
            seen["message"] = str(e)
        finally:
            released.set()

    with P.PpRPA(eps, L, 6) as ctx:
        z = gen.random_vectors(3, 2, ctx.n)
        th = threading.Thread(target=other, args=(ctx, z))
        th.start()
        r = ctx.davidson(5, block=5, tol=1e-8, log=on_iteration)
        th.join(timeout=60.0)
        assert not th.is_alive()
        assert seen["status"] == P.binding.EBUSY, seen
        # the context is free again once the first call returned
        s = ctx.matvec(z)
    assert np.max(np.abs(r["omega"] - ref)) <= 1e-8
    M = O.pprpa_matrix(*O.build_matrices(O.active_space(eps, L, 6), "singlet"))
    assert np.max(np.abs(s - (M @ z.T).T)) <= 1e-12 * np.abs(M @ z.T).max()


@pytest.mark.parametrize("mult,channel", [("singlet", "pp"), ("triplet", "pp"), ("singlet", "hh")])
def test_warm_start_from_converged_vectors(mult, channel):
    note("warm start", mult, channel)
    eps, L = problem(42, 8, 40, 90)
    ref = O.solve(eps, L, 8, mult, 6, channel=channel)
    with P.PpRPA(eps, L, 8, mult=mult) as ctx:
        cold = ctx.davidson(6, block=6, tol=1e-8, vectors=True, channel=channel)
        warm = ctx.davidson(6, block=6, tol=1e-8, guess=cold["vecs"], channel=channel)
    note("cold", cold["report"]["iters"], "warm", warm["report"]["iters"])
    assert cold["report"]["iters"] > 2
    assert warm["report"]["iters"] <= 2
    assert np.max(np.abs(warm["omega"] - ref)) <= 1e-8
    assert np.max(np.abs(warm["omega"] - cold["omega"])) <= 1e-9
    assert np.all(warm["resid"] <= 1e-8)


@pytest.mark.parametrize("nguess", [128, 256])
def test_warm_start_with_many_guesses(nguess):
    """A start block wider than a correction block: the converged vectors followed by random
    ones, 128 and 256 (the subspace cap) guesses in all; the same roots as the oracle's."""
    note("warm start with", nguess, "guesses")
    eps, L = problem(42, 8, 40, 90)
    ref = O.solve(eps, L, 8, "singlet", 6)
    with P.PpRPA(eps, L, 8) as ctx:
        cold = ctx.davidson(6, block=6, tol=1e-8, vectors=True)
        guess = np.vstack([cold["vecs"], gen.random_vectors(44, nguess - 6, ctx.n)])
        warm = ctx.davidson(6, block=6, tol=1e-8, guess=guess, max_subspace=256)
    note("warm iters", warm["report"]["iters"])
    assert warm["status"] == 0
    assert np.max(np.abs(warm["omega"] - ref)) <= 1e-8
    assert np.all(warm["resid"] <= 1e-8)


def test_warm_start_guess_count_below_nroot_is_rejected():
    eps, L = problem(42, 8, 40, 90)
    with P.PpRPA(eps, L, 8) as ctx:
        cold = ctx.davidson(6, block=6, tol=1e-8, vectors=True)
        with pytest.raises(P.PpRPAError) as e:  # 3 directions cannot carry 6 roots
            ctx.davidson(6, block=6, tol=1e-8, guess=cold["vecs"][:3])
    assert e.value.status == P.binding.EINVAL


def test_log_callback_one_json_line_per_iteration():
    note("log callback")
    eps, L = problem(43, 10, 50, 120)
    got = []
    with P.PpRPA(eps, L, 10, mult="triplet") as ctx:
        r = ctx.davidson(8, block=8, tol=1e-7, log=got.append)
    rep = r["report"]
    assert rep["iters"] >= 3
    assert len(got) == rep["iters"] == len(r["log"])
    recs = [json.loads(s) for s in got]
    assert [x["iter"] for x in recs] == list(range(1, rep["iters"] + 1))
    for x in recs:
        assert set(x) >= {"iter", "subspace", "n_conv", "max_resid", "omega0", "n_sigma"}
        assert 0 <= x["n_conv"] <= 8 and x["max_resid"] >= 0.0
    assert all(a["n_sigma"] <= b["n_sigma"] for a, b in zip(recs, recs[1:]))
    last = recs[-1]
    assert last["n_conv"] == 8 and last["n_sigma"] == rep["n_sigma"]
    assert abs(last["max_resid"] - rep["max_resid"]) <= 1e-3 * rep["max_resid"]
    assert abs(last["omega0"] - r["omega"][0]) <= 1e-11


@pytest.mark.parametrize("mult,prec,channel", [("singlet", "fp64", "pp"), ("triplet", "fp32", "pp"),
                                               ("singlet", "fp64", "hh")])
def test_solve_in_steps_equals_davidson(mult, prec, channel):
    note("solve in steps", mult, prec, channel)
    eps, L = problem(44, 9, 60, 110)
    with P.PpRPA(eps, L, 9, mult=mult, prec=prec) as ctx:
        ref = ctx.davidson(6, block=8, tol=1e-7, vectors=True, channel=channel)
        sv = ctx.solve_begin(6, block=8, tol=1e-7, channel=channel)
        steps = 0
        while not sv.done:
            assert sv.iterate(1) == 1
            steps += 1
        assert sv.iterate(3) == 0  # a finished solve runs no more iterations
        r = sv.end(vectors=True)
    assert steps == ref["report"]["iters"] == r["report"]["iters"]
    assert r["report"]["n_sigma"] == ref["report"]["n_sigma"]
    assert np.array_equal(r["omega"], ref["omega"])
    assert np.array_equal(r["resid"], ref["resid"])
    assert np.array_equal(r["vecs"], ref["vecs"])
    assert len(r["log"]) == steps


def test_open_solve_holds_the_context_and_ends_early():
    note("open solve")
    eps, L = problem(45, 8, 50, 100)
    with P.PpRPA(eps, L, 8) as ctx:
        z = gen.random_vectors(3, 1, ctx.n)
        sv = ctx.solve_begin(5, block=5, tol=1e-9)
        with pytest.raises(P.PpRPAError) as e:
            ctx.matvec(z)
        assert e.value.status == P.binding.EBUSY
        with pytest.raises(P.PpRPAError) as e:
            ctx.solve_begin(5)
        assert e.value.status == P.binding.EBUSY
        assert sv.iterate(0) == 0 and not sv.done
        assert sv.iterate(2) == 2 and not sv.done
        r = sv.end(raise_noconv=False)
        assert r["status"] == P.binding.ENOCONV and r["report"]["iters"] == 2
        assert np.all(np.isfinite(r["omega"])) and np.all(r["resid"] > 1e-9)
        ctx.matvec(z)  # released
        # the same solve run to the end converges to the oracle's roots
        sv = ctx.solve_begin(5, block=5, tol=1e-9)
        while not sv.done:
            sv.iterate(4)
        r = sv.end()
    assert np.max(np.abs(r["omega"] - O.solve(eps, L, 8, "singlet", 5))) <= 1e-8


def test_solve_with_roctx_ranges_enabled():
    """PPRPA_ROCTX=1 (roctx ranges around the entry points and Davidson phases, no profiler
    attached): a solve in a child process gives the oracle's roots, as without the ranges."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import numpy as np, paper_2512_12515_amd as P; from workloads import gen; "
            "eps, L = gen.orbital_energies(42, 8, 40), gen.lpq_full(42, 48, 90); "
            "ctx = P.PpRPA(eps, L, 8); r = ctx.davidson(6, block=6, tol=1e-8); ctx.close(); "
            "print(' '.join(repr(float(x)) for x in r['omega']))")
    note("solve with PPRPA_ROCTX=1")
    out = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, PPRPA_ROCTX="1"),
                         cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    assert "could not be opened" not in out.stderr
    omega = np.array([float(x) for x in out.stdout.strip().splitlines()[-1].split()])
    eps, L = problem(42, 8, 40, 90)
    assert np.max(np.abs(omega - O.solve(eps, L, 8, "singlet", 6))) <= 1e-8


"""Benchmark of the ppRPA hot path on one MI355X.

Headline workload (default): nocc = 50, nvir = 500, naux = 1800 (the largest single-GPU
configuration that the whole path runs on without an active window), orbital energies and
three-centre integrals from workloads/gen.py (seed 0, integrals scaled by 0.7: unscaled, this
size has no definite pencil and so no well-defined lowest roots), the lowest 20 singlet pp roots
by block Davidson (block 20, residual tolerance 1e-6), sigma in FP64 on FP64 MFMA, subspace
algebra in FP64.

One step = one Davidson iteration of that solve with the inputs already resident in HBM and the
problem staged (pprpa_build, timed separately): the sigma product of the new block of trial
vectors (unpack, the fused density-fitted contraction, the epilogue), the Rayleigh-Ritz step on
the projected pencil, residuals, preconditioned corrections and their orthogonalisation, driven
through pprpa_solve_iterate. After the K timed steps the solve runs on to convergence (untimed)
and the line reports every root's residual norm. value = single-vector sigma products per second
over the K steps.

Extras on the same line: the 20/200/700 FP64 Davidson (singlet + triplet, 10 roots, both solves
concurrently on two streams, eigenvalues against the oracle's), isolated sigma, the small direct
workload, the correlation energy, unrestricted sectors, the hh channel, NTOs, the precision study
at 50/500/1800 (FP32 / BF16x6 / BF16x3 sigma against the headline's FP64 roots), the active
window (40 + 400 of 120/1500/4000) in every precision, a serving sample (the first 128 requests
of the 512-request stream, which hold its largest, 37/399/1526 and 40/395/1523) and the oracle
timed on the host cores.

Serving stream (--serve-only): 512 seeded requests (workloads/gen.py serve_requests: nocc 4-40,
nvir 30-400, naux = 3.5 nmo, singlet/triplet 50/50, 4-12 roots, integrals scaled by 0.7, tol
1e-6) through the library's server, FP32 sigma with FP64 subspace algebra by default
(--serve-prec fp64 for all-FP64). The saturated rate R_sat is measured first (the first 48
requests submitted at once); then all 512 arrive as a Poisson process at 0.7 R_sat. Each
request's integrals are generated on the device ahead of its arrival (not timed); latency =
finish - submit on the server's clock.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-serve | --serve-only]
"""
import argparse
import json
from concurrent.futures import ThreadPoolExecutor
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12   # MI355X dense FP64 matrix, FLOP/s
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12     # B/s
# HBM traffic of one launch of the FP64 sigma kernel (GB), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a plain 1 GiB device copy, keyed by (workload, precision); the profile
# summaries under profiles/ name the command. A workload without an entry reports null.
TRAFFIC_GB_PER_LAUNCH = {
    # profiles/sigma_fp64_headline_50x500x1800_hbm_traffic.md (20 timed launches of 20 vectors,
    # 16384 work units each)
    ("mixed", "fp64"): 452.8,
}


def sigma_kernel_name(prec, nv):
    """Name of the sigma kernel the library launches for this precision and virtual block (the
    label of the roofline object; the choice itself is made in the library)."""
    t16 = -(-nv // 16)
    t32 = 2 * -(-nv // 32)
    if prec == "fp64":
        k = "k_sandwich_f64 (software-pipelined)" if t16 >= 20 else "k_sandwich<double> (two workgroups per CU)"
    elif prec == "fp32":
        k = "k_sandwich<float>"
    elif prec == "bf16x6" and t32 >= 32 and t32 % 8 == 0:
        k = "k_sandwich_bf16w (double-buffered, 8-column panels)"
    else:
        k = "k_sandwich_bf16<%d>" % (6 if prec == "bf16x6" else 3)
    return k + ": fused density-fitted sigma contraction"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """Cores, CPU model and BLAS of the host the oracle runs on."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cores"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            b = blas[0]
            info["blas"] = f"{b.get('internal_api')} {b.get('version')} ({b.get('architecture')})"
            info["blas_threads"] = int(b.get("num_threads", 0))
    except Exception:
        pass
    info["omp_num_threads"] = os.environ.get("OMP_NUM_THREADS")
    return info


def _median_time(fn, reps=3):
    fn()  # warm-up
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        t.append(time.perf_counter() - t0)
    return float(np.median(t))


def cpu_baseline(head_L=None, head_eps=None, head_cfg=None):
    """The oracle (oracle/pprpa_oracle.py) on the host cores, on bounded samples:
    * the headline workload's density-fitted sigma (sigma_factorised, FP64 NumPy/BLAS): single
      vectors, median of 3 after a warm-up, all cores -> value (sigma/s);
    * the 20/200/700 workload's sigma, all cores and 1 thread, medians of 3;
    * the dense oracle end to end at 5/20/100 (build A, B, C + Cholesky-reduced eigh, 5 singlet
      roots), all cores and 1 thread, medians of 3."""
    from oracle import pprpa_oracle as O
    from workloads import gen
    from threadpoolctl import threadpool_limits
    info = host_info()
    out = {"kind": "oracle", "unit": "sigma/s", "host": info}
    cores = info.get("blas_threads") or info.get("affinity_cores") or os.cpu_count()

    def sigma_rate(sp, mult, n):
        z = gen.random_vectors(1, 1, n)[0]
        return 1.0 / _median_time(lambda: O.sigma_factorised(sp, mult, z))

    # headline workload (the integrals come in from the caller's device copy)
    if head_L is not None:
        c = head_cfg
        sp = O.active_space(head_eps, head_L, c["nocc"])
        n = O.pairs(c["nvir"], c["mult"])[0].size + O.pairs(c["nocc"], c["mult"])[0].size
        out["value"] = sigma_rate(sp, c["mult"], n)
        out["sample"] = (f"median of 3 single-vector {c['mult']} sigma products (oracle "
                         f"sigma_factorised, FP64) at nocc={c['nocc']}, nvir={c['nvir']}, "
                         f"naux={c['naux']}, after one warm-up, {cores} BLAS threads")
        del sp
    # 20/200/700 sigma, all cores and 1 thread
    eps = gen.orbital_energies(0, 20, 200)
    L = gen.lpq_full(0, 220, 700)
    sp = O.active_space(eps, L, 20)
    n = O.pairs(200, "singlet")[0].size + O.pairs(20, "singlet")[0].size
    out["sigma_20x200x700_all_cores"] = sigma_rate(sp, "singlet", n)
    with threadpool_limits(1):
        out["sigma_20x200x700_1_thread"] = sigma_rate(sp, "singlet", n)
    del sp, L
    # dense oracle end to end at 5/20/100
    eps = gen.orbital_energies(0, 5, 20)
    L = gen.lpq_full(0, 25, 100)
    dense = lambda: O.solve(eps, L, 5, "singlet", 5)
    out["dense_5x20x100_ms_all_cores"] = 1e3 * _median_time(dense)
    with threadpool_limits(1):
        out["dense_5x20x100_ms_1_thread"] = 1e3 * _median_time(dense)
    out["cores"] = int(cores)
    if "value" not in out:
        out["value"] = out["sigma_20x200x700_all_cores"]
        out["sample"] = "median of 3 single-vector singlet sigma products at 20/200/700"
    return out


def serve_stream(P, gen, n_req=512, n_sat=48, budget_gb=96, max_inflight=16, prec="fp64",
                 tol=1e-6, lookahead=12):
    """The serving workload: saturated rate, then Poisson arrivals at 0.7 of it."""
    import queue
    import threading
    import torch
    dev = torch.device("cuda:0")
    reqs = gen.serve_requests(0, n_req)
    pstream = torch.cuda.Stream(device=dev)  # input generation, off the library's streams

    def inputs(r):
        nmo = r["nocc"] + r["nvir"]
        idx = np.arange(nmo)
        with torch.cuda.stream(pstream):
            L = torch.empty((r["naux"], nmo, nmo), dtype=torch.float64, device=dev)
            for p0 in range(0, r["naux"], 128):
                aux = np.arange(p0, min(r["naux"], p0 + 128))
                L[p0:p0 + aux.size] = gen.lpq_block_torch(r["seed"], nmo, r["naux"], idx, idx, aux,
                                                          dev) * r["eig_scale"]
            eps = torch.from_numpy(gen.orbital_energies(r["seed"], r["nocc"], r["nvir"])).to(dev)
        pstream.synchronize()
        return eps, L

    def submit(srv, r, eps, L):
        return srv.submit(eps, L, r["nocc"], r["nroot"], mult=r["mult"], prec=prec, tol=tol)

    def run(srv, order, arrivals):
        """Submit requests `order` at `arrivals` (s, from start); poll until all are done. The
        binding keeps a request's inputs alive until a poll shows the library no longer needs
        them, so polling as we go bounds the memory held by inputs."""
        q = queue.Queue(maxsize=lookahead)

        def producer():
            for i in order:
                q.put((i, inputs(reqs[i])))

        th = threading.Thread(target=producer, daemon=True)
        th.start()
        pending, out, late = {}, {}, []

        def sweep():
            for t, i in list(pending.items()):
                r = srv.poll(t)
                if r["state"] == srv.DONE:
                    out[i] = r
                    del pending[t]
                    if len(out) % 32 == 0:
                        log(f"  {len(out)}/{len(order)} requests done at "
                            f"{time.perf_counter() - t_start:.1f}s")

        t_start = time.perf_counter()
        for j, _ in enumerate(order):
            i, (eps, L) = q.get()
            wait = arrivals[j] - (time.perf_counter() - t_start)
            while wait > 0:
                time.sleep(min(wait, 0.002))
                sweep()
                wait = arrivals[j] - (time.perf_counter() - t_start)
            if wait < -1e-3:
                late.append(-wait)
            pending[submit(srv, reqs[i], eps, L)] = i
            del eps, L
            sweep()
        th.join()
        while pending:
            time.sleep(0.001)
            sweep()
        return out, time.perf_counter() - t_start, late

    budget = int(budget_gb * (1 << 30))
    # saturated service rate: n_sat requests, inputs generated beforehand, submitted at once
    pre = [inputs(reqs[i]) for i in range(n_sat)]
    with P.Server(budget, max_inflight) as srv:
        t0 = time.perf_counter()
        tk = {i: submit(srv, reqs[i], *pre[i]) for i in range(n_sat)}
        del pre
        res = {}
        for i, t in tk.items():
            res[i] = srv.wait(t, timeout=600.0)
            if (i + 1) % 16 == 0:
                log(f"  saturated: {i + 1}/{n_sat} done at {time.perf_counter() - t0:.1f}s")
        t_sat = time.perf_counter() - t0
        st_sat = srv.stats()
    log(f"saturated stats: {st_sat}")
    sat_ok = sum(r["status"] == P.binding.OK for r in res.values())
    r_sat = n_sat / t_sat
    log(f"saturated: {n_sat} requests in {t_sat:.2f}s -> R_sat = {r_sat:.1f}/s")
    lam = 0.7 * r_sat
    arr = gen.poisson_arrivals(0, n_req, lam)
    with P.Server(budget, max_inflight) as srv:
        res, makespan, late = run(srv, list(range(n_req)), arr)
        st = srv.stats()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res.values()])
    qwait = np.array([r["t_admit"] - r["t_submit"] for r in res.values()])
    status = {}
    for r in res.values():
        name = P.binding.STATUS_NAMES[r["status"]]
        status[name] = status.get(name, 0) + 1
    ok = [r for r in res.values() if r["status"] == P.binding.OK]
    failures = [dict(nocc=reqs[i]["nocc"], nvir=reqs[i]["nvir"], mult=reqs[i]["mult"],
                     nroot=reqs[i]["nroot"], status=P.binding.STATUS_NAMES[r["status"]],
                     message=r["message"][:80])
                for i, r in sorted(res.items()) if r["status"] != P.binding.OK]
    n_sigma = sum(r["report"]["n_sigma"] for r in ok)
    # accuracy: the six smallest served requests against the oracle's stored roots (every request
    # of the mix with at most 100 orbitals, tests/golden/serving_small.json)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "serving_small.json")))["roots"]
    small = sorted((i for i in res if str(reqs[i]["rid"]) in gold),
                   key=lambda i: reqs[i]["nvir"] + reqs[i]["nocc"])[:6]
    errs = []
    for i in small:
        if res[i]["status"] != P.binding.OK:
            continue
        ref = np.array(gold[str(reqs[i]["rid"])])
        errs.append(float(np.max(np.abs(res[i]["omega"] - ref))))
    peak = PEAK_FP64 if prec == "fp64" else PEAK_FP32
    tf = st["sigma_flops"] / st["sigma_seconds"] if st["sigma_seconds"] > 0 else 0.0
    return {
        "requests": n_req, "prec": prec, "tol": tol, "budget_gb": budget_gb,
        "max_inflight": max_inflight,
        "saturated_rate_req_s": r_sat, "saturated_sample": n_sat, "saturated_ok": sat_ok,
        "saturated_mean_group_size": st_sat["grouped_products"] / max(st_sat["group_launches"], 1),
        "saturated_peak_inflight": st_sat["peak_inflight"],
        "arrival_rate_req_s": lam,
        "throughput_req_s": n_req / makespan, "makespan_s": makespan,
        "sigma_products_per_s": n_sigma / makespan,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(np.mean(lat)), "latency_max_s": float(np.max(lat)),
        "latency_p99_over_p50": float(np.percentile(lat, 99) / np.percentile(lat, 50)),
        "queue_wait_p50_s": float(np.percentile(qwait, 50)),
        "queue_wait_p99_s": float(np.percentile(qwait, 99)),
        "late_submits": len(late), "status": status, "failures": failures[:12],
        "peak_inflight": st["peak_inflight"], "peak_reserved_gb": st["peak_reserved"] / 2 ** 30,
        "group_launches": st["group_launches"],
        "mean_group_size": st["grouped_products"] / max(st["group_launches"], 1),
        "grouped_sigma_tflops": tf / 1e12, "grouped_sigma_frac": tf / peak,
        "max_eig_err_ha_smallest6_vs_oracle": max(errs) if errs else None,
    }


PEAK_BF16 = 2.5e15   # dense BF16 matrix, FLOP/s


def small_direct(P, gen, reps=20):
    """The small direct workload (nocc 5, nvir 20, naux 100, singlet, 5 roots, seeds 0-4):
    staging + dense build (pprpa_build with dense=1) and the direct dense diagonalisation on the
    device, inputs resident in HBM; error against the oracle's stored roots."""
    import torch
    dev = torch.device("cuda:0")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "small_direct.json")))
    t_build, t_solve, errs = [], [], []
    for seed in range(5):
        eps = torch.from_numpy(gen.orbital_energies(seed, 5, 20)).to(dev)
        L = torch.from_numpy(gen.lpq_full(seed, 25, 100)).to(dev)
        torch.cuda.synchronize()
        for rep in range(reps):
            t0 = time.perf_counter()
            ctx = P.PpRPA(eps, L, 5, mult="singlet", dense=True)
            t1 = time.perf_counter()
            r = ctx.davidson(5, direct=True)
            t2 = time.perf_counter()
            ctx.close()
            if rep > 0:  # the first call of each seed also pays one-time set-up
                t_build.append(t1 - t0)
                t_solve.append(t2 - t1)
        errs.append(float(np.max(np.abs(r["omega"] - np.array(gold["roots"][f"{seed}/singlet"])))))
    return {"workload": "nocc=5 nvir=20 naux=100 singlet, 5 roots, seeds 0-4, direct",
            "build_dense_ms_p50": 1e3 * float(np.median(t_build)),
            "direct_solve_ms_p50": 1e3 * float(np.median(t_solve)),
            "max_eig_err_ha_vs_oracle": max(errs)}


def correlation_energy(P, gen, reps=10):
    """Correlation energy (closed shell: E_singlet + 3 E_triplet) of the small direct workload
    (nocc 5, nvir 20, naux 100, seeds 0-4) from the whole spectrum of the dense pencil on the
    device (dense build + eigenvalues, inputs resident in HBM); error against the oracle's
    stored values and the gap between the two sides of the sum rule."""
    import torch
    dev = torch.device("cuda:0")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "correlation_energy.json")))
    t_call, errs, gaps = [], [], []
    for seed in range(5):
        eps = torch.from_numpy(gen.orbital_energies(seed, 5, 20)).to(dev)
        L = torch.from_numpy(gen.lpq_full(seed, 25, 100)).to(dev)
        torch.cuda.synchronize()
        for rep in range(reps):
            t0 = time.perf_counter()
            tot = 0.0
            for mult, wgt in (("singlet", 1.0), ("triplet", 3.0)):
                with P.PpRPA(eps, L, 5, mult=mult, dense=True) as ctx:
                    r = ctx.correlation_energy()
                tot += wgt * r["ec_pp"]
                gaps.append(abs(r["ec_pp"] - r["ec_hh"]))
            if rep > 0:
                t_call.append(time.perf_counter() - t0)
        errs.append(abs(tot - gold["energies"][str(seed)]["closed_shell"]))
    return {"workload": "nocc=5 nvir=20 naux=100, E_singlet + 3 E_triplet, seeds 0-4, "
                        "build + whole-spectrum solve per spin",
            "ms_per_energy_p50": 1e3 * float(np.median(t_call)),
            "max_err_ha_vs_oracle": max(errs), "max_sum_rule_gap_ha": max(gaps)}


def dense_large(P, gen, cases=((8, 45, 150), (8, 62, 150)), nroot=5, reps=3):
    """The dense pencil solves on many workgroups: for each (nocc, nvir, naux), singlet (orders
    1071 and 1989 by default), the direct solve of the nroot lowest pp roots with vectors and the
    correlation energy from the whole spectrum, inputs resident on the device; median time of
    reps calls after one untimed call, the largest residual |M z - Omega W z| of the roots and
    the gap between the two sides of the energy's sum rule (both exact relations, so no stored
    values are needed)."""
    out = []
    for nocc, nvir, naux in cases:
        eps, L = gen.orbital_energies(54, nocc, nvir), gen.lpq_full(54, nocc + nvir, naux)
        with P.PpRPA(eps, L, nocc, mult="singlet", dense=True) as ctx:
            ctx.davidson(nroot, direct=True)
            ctx.correlation_energy()
            td, te = [], []
            for _ in range(reps):
                t0 = time.perf_counter()
                r = ctx.davidson(nroot, direct=True, vectors=True)
                td.append(time.perf_counter() - t0)
            for _ in range(reps):
                t0 = time.perf_counter()
                e = ctx.correlation_energy()
                te.append(time.perf_counter() - t0)
            out.append({"nocc": nocc, "nvir": nvir, "naux": naux, "n": ctx.n,
                        "direct_ms_p50": 1e3 * float(np.median(td)),
                        "direct_max_resid": float(np.max(r["resid"])),
                        "energy_ms_p50": 1e3 * float(np.median(te)),
                        "energy_sum_rule_gap_ha": abs(e["ec_pp"] - e["ec_hh"])})
    return {"workload": f"singlet, {nroot} pp roots with vectors (direct) and the whole spectrum "
                        "(correlation energy), many-workgroup dense solver", "orders": out}


def nto_analysis(P, eps_d, L_d, nocc, nroot, block, tol, reps=5):
    """NTO weights and two-electron density blocks of the nroot singlet pp roots of the FP64
    Davidson workload (vectors handed over from the host, density blocks copied back): time per
    call and the largest deviations from the sum rules sum lam^p - sum lam^h = 1, Tr D = 2."""
    with P.PpRPA(eps_d, L_d, nocc, mult="singlet", max_block=block) as ctx:
        r = ctx.davidson(nroot, block=block, tol=tol, vectors=True)
        ctx.nto(r["vecs"])
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            res = ctx.nto(r["vecs"])
            t.append(time.perf_counter() - t0)
    w = res["lam_p"].sum(axis=1) - res["lam_h"].sum(axis=1)
    tr = np.trace(res["d_vv"], axis1=1, axis2=2) + np.trace(res["d_oo"], axis1=1, axis2=2)
    return {"workload": f"{nroot} singlet pp roots, nv {ctx.nv}, no {ctx.no}, weights + density blocks",
            "ms_per_call_p50": 1e3 * float(np.median(t)),
            "max_weight_sum_rule_dev": float(np.max(np.abs(w - 1.0))),
            "max_trace_rule_dev": float(np.max(np.abs(tr - 2.0))),
            "leading_weight_root0": float(res["lam_p"][0, 0])}


def unrestricted(P, gen, reps=3, tol=1e-8):
    """Spin-unrestricted ppRPA on nmo 60, nocc 10 (alpha) / 9 (beta), naux 200: the alpha-alpha
    and beta-beta sectors as triplet contexts of each spin (density-fitted sigma), the
    alpha-beta sector as a dense context (order 2640), 8 lowest pp roots of each by Davidson;
    time for the three builds and solves, error of the 8 lowest overall against the oracle."""
    import torch
    dev = torch.device("cuda:0")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "unrestricted.json")))
    nmo, noa, nob, naux, seed, nroot = (gold[k] for k in ("nmo", "nocc_a", "nocc_b", "naux", "seed", "nroot"))
    ea = torch.from_numpy(gen.orbital_energies(seed, noa, nmo - noa)).to(dev)
    eb = torch.from_numpy(gen.orbital_energies(seed + 1000, nob, nmo - nob)).to(dev)
    La = torch.from_numpy(gen.lpq_full(seed, nmo, naux)).to(dev)
    Lb = torch.from_numpy(gen.lpq_full(seed + 1000, nmo, naux)).to(dev)
    torch.cuda.synchronize()
    times = []
    for rep in range(reps + 1):
        t0 = time.perf_counter()
        roots = []
        for e_s, L_s, no_s in ((ea, La, noa), (eb, Lb, nob)):
            with P.PpRPA(e_s, L_s, no_s, mult="triplet") as ctx:
                roots += list(ctx.davidson(nroot, block=nroot, tol=tol)["omega"])
        with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
            n_ab = ctx.n
            roots += list(ctx.davidson(nroot, block=nroot, tol=tol)["omega"])
        if rep > 0:
            times.append(time.perf_counter() - t0)
    err = float(np.max(np.abs(np.sort(roots)[:nroot] - np.array(gold["roots"]["all"]))))
    # the alpha-beta sector with the density-fitted sigma: the same system (its roots against the
    # dense context's), then a sector beyond the dense limit (order 33120)
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob) as ctx:
        om_dense = ctx.davidson(nroot, block=nroot, tol=tol)["omega"]
    with P.PpRPA.alpha_beta(ea, eb, La, Lb, noa, nob, density_fitted=True) as ctx:
        om_df = ctx.davidson(nroot, block=nroot, tol=tol)["omega"]
    big = (200, 20, 18, 700, 85, 8)
    bmo, bna, bnb, baux, bseed, broot = big
    ea2 = torch.from_numpy(gen.orbital_energies(bseed, bna, bmo - bna)).to(dev)
    eb2 = torch.from_numpy(gen.orbital_energies(bseed + 1000, bnb, bmo - bnb)).to(dev)
    La2 = torch.from_numpy(gen.lpq_full(bseed, bmo, baux)).to(dev)
    Lb2 = torch.from_numpy(gen.lpq_full(bseed + 1000, bmo, baux)).to(dev)
    torch.cuda.synchronize()
    with P.PpRPA.alpha_beta(ea2, eb2, La2, Lb2, bna, bnb, density_fitted=True) as ctx:
        n_big = ctx.n
        ctx.davidson(broot, block=16, tol=1e-6)  # warm-up
        ctx.sigma_stats(reset=True)
        t0 = time.perf_counter()
        rb = ctx.davidson(broot, block=16, tol=1e-6)
        t_big = time.perf_counter() - t0
        st = ctx.sigma_stats()
    # the sigma kernel in each precision on the same sector: 16 vectors, 3 timed products
    zb = torch.from_numpy(gen.random_vectors(86, 16, n_big)).to(dev)
    by_prec = {}
    for prec in ("fp64", "fp32", "bf16x6", "bf16x3"):
        with P.PpRPA.alpha_beta(ea2, eb2, La2, Lb2, bna, bnb, density_fitted=True, prec=prec,
                                max_block=16) as ctx:
            ctx.matvec(zb)
            ctx.sigma_stats(reset=True)
            for _ in range(3):
                ctx.matvec(zb)
            sp = ctx.sigma_stats()
        by_prec[prec] = sp["flops"] / max(sp["seconds"], 1e-30) / 1e12
    del La2, Lb2, zb
    return {"workload": f"nmo {nmo}, nocc {noa}/{nob}, naux {naux}: aa + bb (triplet, DF sigma) + "
                        f"ab (dense, n {n_ab}), {nroot} roots each, tol {tol:g}",
            "s_per_three_sectors_p50": float(np.median(times)), "max_eig_err_ha_vs_oracle": err,
            "ab_density_fitted": {
                "same_system_max_root_diff_vs_dense_ha": float(np.max(np.abs(om_df - om_dense))),
                "large_workload": f"nmo {bmo}, nocc {bna}/{bnb}, naux {baux}, alpha-beta sector of "
                                  f"order {n_big} (beyond the dense limit), {broot} pp roots, "
                                  "block 16, tol 1e-06",
                "solve_s": t_big, "iters": rb["report"]["iters"],
                "n_sigma": rb["report"]["n_sigma"], "max_resid": float(np.max(rb["resid"])),
                "sigma_kernel_tflops_algorithmic": st["flops"] / max(st["seconds"], 1e-30) / 1e12,
                "isolated_sigma_tflops_algorithmic_by_prec": by_prec}}


def isolated_sigma(P, gen, eps_d, L_d, nocc, block, warm=3, reps=20):
    """Isolated sigma: pprpa_matvec on block random FP64 vectors resident on the device, 3 warm-up
    calls, then the median of 20 timed calls (unpack + sandwich + epilogue, host clock around
    the synchronous call) and the sandwich kernel's own event time; sigma/s = block / t."""
    import torch
    out = {}
    for mult in ("singlet", "triplet"):
        with P.PpRPA(eps_d, L_d, nocc, mult=mult, max_block=block) as ctx:
            z = torch.from_numpy(gen.random_vectors(5, block, ctx.n)).to(eps_d.device)
            for _ in range(warm):
                ctx.matvec(z)
            ctx.sigma_stats(reset=True)
            t = []
            for _ in range(reps):
                t0 = time.perf_counter()
                ctx.matvec(z)
                t.append(time.perf_counter() - t0)
            st = ctx.sigma_stats()
        tm = float(np.median(t))
        out[mult] = {"ms_per_call_p50": 1e3 * tm, "sigma_per_s": block / tm,
                     "kernel_ms_per_launch": 1e3 * st["seconds"] / st["launches"],
                     "kernel_tflops_algorithmic": st["flops"] / st["seconds"] / 1e12}
    return dict(workload=f"pprpa_matvec, {block} vectors, median of {reps} after {warm} warm-ups",
                **out)


def hh_channel(P, eps_d, L_d, nocc, nroot, block, tol, reps=2):
    """The hh channel (two-electron removal roots nearest the gap) on the FP64 Davidson workload:
    singlet and triplet solved one after the other, reps times; sigma products per second,
    solve latency and the error against the oracle's stored hh roots."""
    gold_path = os.path.join(ROOT, "tests", "golden", "davidson_hh_fp64.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    n_sigma, secs, lat, errs, iters = 0, 0.0, [], [], {}
    for rep in range(reps + 1):
        for mult in ("singlet", "triplet"):
            t0 = time.perf_counter()
            with P.PpRPA(eps_d, L_d, nocc, mult=mult, max_block=block) as ctx:
                r = ctx.davidson(nroot, block=block, tol=tol, channel="hh")
            dt = time.perf_counter() - t0
            if rep == 0:
                continue  # warm-up
            n_sigma += r["report"]["n_sigma"]
            secs += dt
            lat.append(dt)
            iters[mult] = r["report"]["iters"]
            if gold is not None and nroot <= len(gold["roots"][f"0/{mult}"]):
                ref = np.array(gold["roots"][f"0/{mult}"][:nroot])
                errs.append(float(np.max(np.abs(r["omega"] - ref))))
    return {"workload": f"hh channel, {nroot} roots per spin, block {block}, tol {tol:g}, "
                        "singlet then triplet",
            "sigma_per_s": n_sigma / secs, "latency_p50_s": float(np.percentile(lat, 50)),
            "iters": iters, "max_eig_err_ha_vs_oracle": max(errs) if errs else None}


def device_problem(gen, name, dev, scale=None):
    """Orbital energies and the active block of the integrals of a large workload, generated on
    the device (scaled by the workload's eig_scale unless scale is given), and the build
    keywords that go with them."""
    import torch
    c = gen.CONFIGS[name]
    nocc, nvir, naux = c["nocc"], c["nvir"], c["naux"]
    no_act, nv_act = c.get("nocc_act"), c.get("nvir_act")
    idx = gen.active_indices(nocc, nvir, no_act, nv_act)
    scale = c.get("eig_scale", 1.0) if scale is None else scale
    L = torch.empty((naux, idx.size, idx.size), dtype=torch.float64, device=dev)
    for p0 in range(0, naux, 128):
        aux = np.arange(p0, min(naux, p0 + 128))
        L[p0:p0 + aux.size] = gen.lpq_block_torch(0, nocc + nvir, naux, idx, idx, aux, dev) * scale
    eps = torch.from_numpy(gen.orbital_energies(0, nocc, nvir)).to(dev)
    torch.cuda.synchronize()
    kw = dict(nocc_act=no_act or 0, nvir_act=nv_act or 0, lpq_is_active=no_act is not None)
    return eps, L, kw


def precision_study(P, gen, precs=("fp64", "fp32", "bf16x6", "bf16x3"), block=20, tol=1e-6,
                    tol_reduced=1e-5, name="mixed", problem=None, ref=None):
    """A large workload (default: the mixed-precision one, nocc 50, nvir 500, naux 1800, singlet,
    20 roots; name="active": the 40 + 400 window of 120 / 1500 / 4000, triplet, 16 roots, only
    the active block of L passed) solved by the same Davidson with sigma in each precision
    (subspace algebra FP64 throughout); per-root eigenvalue error against the FP64 GPU run. The
    integrals are scaled by the workload's eig_scale (0.7), at which the pencil is definite.
    FP64 converges to residual tol; the reduced precisions to tol_reduced, since their sigma
    error puts a floor near 1e-6 under the residual (the eigenvalue error, quadratic in the
    residual, stays far below 1e-6 Ha). sigma_rel_err_random_unit: |sigma_prec z - sigma_fp64 z|_2
    / |sigma_fp64 z|_2 on four seeded random unit vectors, the size of that floor."""
    import torch
    dev = torch.device("cuda:0")
    c = gen.CONFIGS[name]
    nocc, nvir, naux, nroot = c["nocc"], c["nvir"], c["naux"], c["nroot"]
    mult = c["mult"] if isinstance(c["mult"], str) else c["mult"][0]
    no_act, nv_act = c.get("nocc_act"), c.get("nvir_act")
    eps, L, kw = problem if problem is not None else device_problem(gen, name, dev)
    out = {}
    with P.PpRPA(eps, L, nocc, mult=mult, prec="fp64", max_block=block, **kw) as ctx:
        zr = gen.random_vectors(5, 4, ctx.n)
        zr /= np.linalg.norm(zr, axis=1, keepdims=True)
        s64 = ctx.matvec(zr)
    for prec in precs:
        t0 = time.perf_counter()
        with P.PpRPA(eps, L, nocc, mult=mult, prec=prec, max_block=block, **kw) as ctx:
            t1 = time.perf_counter()
            r = ctx.davidson(nroot, block=block, tol=tol if prec == "fp64" else tol_reduced,
                             max_iter=300, raise_noconv=False)
            t2 = time.perf_counter()
            st = ctx.sigma_stats()
            rel = np.linalg.norm(ctx.matvec(zr) - s64, axis=1) / np.linalg.norm(s64, axis=1)
        nprod = {"bf16x6": 6, "bf16x3": 3}.get(prec, 1)
        peak = {"fp64": PEAK_FP64, "fp32": PEAK_FP32}.get(prec, PEAK_BF16)
        alg = st["flops"] / st["seconds"] if st["seconds"] > 0 else 0.0
        e = {"status": P.binding.STATUS_NAMES[r["status"]], "build_s": t1 - t0, "solve_s": t2 - t1,
             "iters": r["report"]["iters"], "n_sigma": r["report"]["n_sigma"],
             "sigma_per_s": r["report"]["n_sigma"] / (t2 - t1),
             "sigma_kernel_tflops_algorithmic": alg / 1e12,
             "sigma_kernel_tflops_executed": nprod * alg / 1e12,
             "sigma_kernel_frac_of_peak": nprod * alg / peak,
             "sigma_kernel_share_of_solve": st["seconds"] / (t2 - t1),
             "max_resid": r["report"]["max_resid"],
             "sigma_rel_err_random_unit": float(rel.max())}
        if prec == "fp64" and ref is None:
            ref = r["omega"]
        elif ref is not None:
            d = np.abs(r["omega"] - ref)
            e["max_abs_err_vs_fp64_ha"] = float(d.max())
            e["per_root_err_ha"] = [float(x) for x in d]
        out[prec] = e
        log(f"{name} {prec}: {e['status']} {e['solve_s']:.2f}s {e['sigma_kernel_tflops_algorithmic']:.1f} TF")
    del L, eps
    window = f" window {no_act} occ + {nv_act} vir," if no_act else ""
    return {"workload": f"nocc={nocc} nvir={nvir} naux={naux}{window} {mult}, {nroot} roots, "
                        f"block {block}, tol {tol:g} (FP64) / {tol_reduced:g} (reduced precisions), "
                        f"L x {c['eig_scale']}", "by_prec": out}


def headline(P, gen, name, prec, block, tol, steps, warmup, problem):
    """The headline: K Davidson iterations of the workload's solve, timed one by one through
    pprpa_solve_iterate after W untimed ones; then the solve runs on to convergence. A solve
    that converges inside the timed window is followed by a new one on the same context."""
    import torch
    c = gen.CONFIGS[name]
    nocc, nroot = c["nocc"], c["nroot"]
    mult = c["mult"] if isinstance(c["mult"], str) else c["mult"][0]
    eps, L, kw = problem
    t0 = time.perf_counter()
    ctx = P.PpRPA(eps, L, nocc, mult=mult, prec=prec, max_block=block, **kw)
    t_build = time.perf_counter() - t0
    state = {"sv": None, "prev": 0, "solves": 0}

    def begin():
        state["sv"] = ctx.solve_begin(nroot, block=block, tol=tol, max_iter=300)
        state["prev"] = 0
        state["solves"] += 1

    def step():
        """One Davidson iteration; returns the sigma products it computed."""
        if state["sv"] is None or state["sv"].done:
            if state["sv"] is not None:
                state["sv"].end()
            begin()
        sv = state["sv"]
        if sv.iterate(1) != 1:
            raise RuntimeError("no Davidson iteration ran")
        ns = json.loads(sv.log[-1])["n_sigma"]
        d, state["prev"] = ns - state["prev"], ns
        return d

    for w in range(warmup):
        step()
    log(f"headline: {warmup} warm-up iterations done")
    torch.cuda.synchronize()
    state["sv"].sigma_stats(reset=True)
    n_sigma = 0
    t0 = time.perf_counter()
    for k in range(steps):
        n_sigma += step()
        if (k + 1) % 5 == 0:
            log(f"headline step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = state["sv"].sigma_stats()
    timed_solves = state["solves"]
    # the solve runs on to convergence (untimed): residuals of every root
    sv = state["sv"]
    while not sv.done:
        sv.iterate(8)
    r = sv.end()
    ctx.close()
    return dict(elapsed=elapsed, n_sigma=n_sigma, stats=st, t_build=t_build, result=r,
                solves_in_timed_window=timed_solves, mult=mult, nroot=nroot)


def fp64_davidson_pair(P, gen, steps, warmup, nroot=10, block=20, tol=1e-6, concurrent=True):
    """The 20/200/700 FP64 Davidson workload: one step = staging + the singlet and triplet solves
    (concurrently on two streams), eigenvalues against the oracle's stored roots."""
    import torch
    dev = torch.device("cuda:0")
    nocc, nvir, naux = 20, 200, 700
    eps_d = torch.from_numpy(gen.orbital_energies(0, nocc, nvir)).to(dev)
    L_d = torch.from_numpy(gen.lpq_full(0, nocc + nvir, naux)).to(dev)
    torch.cuda.synchronize()
    mults = ("singlet", "triplet")

    def solve(mult):
        t0 = time.perf_counter()
        with P.PpRPA(eps_d, L_d, nocc, mult=mult, max_block=block) as ctx:
            r = ctx.davidson(nroot, block=block, tol=tol)
            st = ctx.sigma_stats()
        return dict(omega=r["omega"], rep=r["report"], stats=st, latency=time.perf_counter() - t0)

    pool = ThreadPoolExecutor(max_workers=2) if concurrent else None

    def step():
        if pool is None:
            return {m: solve(m) for m in mults}
        futs = {m: pool.submit(solve, m) for m in mults}
        return {m: f.result() for m, f in futs.items()}

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_sigma = sum(r[m]["rep"]["n_sigma"] for r in results for m in mults)
    k_sec = sum(r[m]["stats"]["seconds"] for r in results for m in mults)
    k_flops = sum(r[m]["stats"]["flops"] for r in results for m in mults)
    k_launch = sum(r[m]["stats"]["launches"] for r in results for m in mults)
    lat = np.array([r[m]["latency"] for r in results for m in mults])
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "davidson_fp64.json")))
    errs = [float(np.max(np.abs(r[m]["omega"] - np.array(g["roots"][f"0/{m}"][:nroot]))))
            for r in results for m in mults]
    out = {"workload": f"ppRPA Davidson nocc={nocc} nvir={nvir} naux={naux}, singlet+triplet, "
                       f"{nroot} roots, block {block}, tol {tol:g}, FP64; one step = staging + both "
                       f"solves ({'concurrent, 2 streams' if concurrent else 'serial'})",
           "steps": steps, "sigma_per_s": n_sigma / elapsed, "ms_per_step": 1e3 * elapsed / steps,
           "sigma_kernel_tflops": k_flops / k_sec / 1e12, "sigma_kernel_frac": k_flops / k_sec / PEAK_FP64,
           "avg_launch_ms": 1e3 * k_sec / max(k_launch, 1), "sigma_kernel_share": k_sec / elapsed,
           "latency_p50_s": float(np.percentile(lat, 50)),
           "max_eig_err_ha_vs_oracle": max(errs),
           "iters": {m: results[-1][m]["rep"]["iters"] for m in mults}}
    return out, (eps_d, L_d)


def copy_probe(torch, dev):
    """One plain 1 GiB device-to-device copy: a kernel of known traffic (1 GiB read, 1 GiB
    written) that calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--workload", default="mixed",
                    help="headline workload (workloads/gen.py CONFIGS: mixed = 50/500/1800)")
    ap.add_argument("--block", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--prec", default="fp64")
    ap.add_argument("--headline-only", action="store_true", help="only the headline line")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision study")
    ap.add_argument("--no-active", action="store_true", help="skip the active-window study")
    ap.add_argument("--precision-only", action="store_true", help="run only the precision study")
    ap.add_argument("--precs", default="fp64,fp32,bf16x6,bf16x3",
                    help="sigma precisions of the precision / active-window study (comma list; "
                         "errors are reported against fp64 when it is included)")
    ap.add_argument("--active-only", action="store_true",
                    help="run only the active-window workload in each precision")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving stream")
    ap.add_argument("--dense-only", action="store_true",
                    help="run only the dense solves at orders 1071 and 1989 (many workgroups)")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="requests in the serving stream (default 512 with --serve-only, else 128)")
    ap.add_argument("--serve-prec", default="fp32",
                    help="sigma precision of the served solves (subspace algebra is FP64)")
    ap.add_argument("--no-extras", action="store_true",
                    help="no isolated sigma, 20/200/700, small direct, correlation energy, "
                         "large dense, unrestricted, hh channel or NTO entries")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--pair-only", action="store_true",
                    help="run only the 20/200/700 FP64 singlet + triplet Davidson workload "
                         "(--steps / --warmup steps of it; with --copy-probe, the calibration copy)")
    ap.add_argument("--serial", dest="concurrent", action="store_false",
                    help="20/200/700 extra: the singlet and triplet solves one after the other")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sigma product "
              "would shard over the aux index with one all-reduce per block, which is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2512_12515_amd as P
    from workloads import gen

    dev = torch.device("cuda:0")
    data = "synthetic (seeded counter-based generator, workloads/gen.py)"
    if args.precision_only or args.active_only:
        name = "active" if args.active_only else "mixed"
        line = {"metric": "sigma-products/sec and per-root eigenvalue error by sigma precision",
                "n_gpus": 1, "data": data}
        line.update(precision_study(P, gen, precs=tuple(args.precs.split(",")), name=name))
        print(json.dumps(line), flush=True)
        return
    if args.serve_only:
        line = {"metric": "served ppRPA requests/s with p50/p99 latency", "n_gpus": 1, "data": data}
        line.update(serve_stream(P, gen, n_req=args.serve_requests or 512, prec=args.serve_prec))
        print(json.dumps(line), flush=True)
        return
    if args.dense_only:
        line = {"metric": "dense pencil solve time (direct roots and correlation energy)",
                "n_gpus": 1, "data": data}
        line.update(dense_large(P, gen))
        print(json.dumps(line), flush=True)
        return
    if args.pair_only:
        if args.copy_probe:
            copy_probe(torch, dev)
        line = {"metric": "sigma-products/sec (20/200/700 FP64 Davidson, singlet + triplet)",
                "n_gpus": 1, "data": data}
        line.update(fp64_davidson_pair(P, gen, steps=args.steps, warmup=args.warmup,
                                       concurrent=args.concurrent)[0])
        print(json.dumps(line), flush=True)
        return
    if args.copy_probe:
        copy_probe(torch, dev)

    name = args.workload
    c = gen.CONFIGS[name]
    t = time.perf_counter()
    problem = device_problem(gen, name, dev)
    log(f"{name} inputs resident in HBM ({problem[1].numel() * 8 / 1e9:.2f} GB) in "
        f"{time.perf_counter() - t:.1f}s")
    h = headline(P, gen, name, args.prec, args.block, args.tol, args.steps, args.warmup, problem)
    st, r = h["stats"], h["result"]
    peak = {"fp64": PEAK_FP64, "fp32": PEAK_FP32}.get(args.prec, PEAK_BF16)
    nprod = {"bf16x6": 6, "bf16x3": 3}.get(args.prec, 1)
    achieved = st["flops"] / st["seconds"] if st["seconds"] > 0 else 0.0
    window = (f", window {c['nocc_act']} occ + {c['nvir_act']} vir" if c.get("nocc_act") else "")
    wl = (f"ppRPA Davidson nocc={c['nocc']} nvir={c['nvir']} naux={c['naux']}{window}, {h['mult']}, "
          f"{h['nroot']} roots, block {args.block}, tol {args.tol:g}, sigma {args.prec}, subspace "
          f"FP64, integrals x {c.get('eig_scale', 1.0)}; one step = one Davidson iteration")
    line = {
        "metric": "sigma-products/sec (Davidson, every root converged to residual <= tol; "
                  "eigenvalue error <= 1e-6 Ha)",
        "value": h["n_sigma"] / h["elapsed"],
        "unit": "sigma/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * h["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else args.prec,
        "data": data,
        "config": {"workload": wl, "nocc": c["nocc"], "nvir": c["nvir"], "naux": c["naux"],
                   "nocc_act": c.get("nocc_act"), "nvir_act": c.get("nvir_act"),
                   "mult": h["mult"], "nroot": h["nroot"], "block": args.block, "tol": args.tol,
                   "prec": args.prec, "eig_scale": c.get("eig_scale", 1.0)},
        "roofline": {"bound": "mfma", "achieved": nprod * achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": nprod * achieved / peak,
                     "traffic": TRAFFIC_GB_PER_LAUNCH.get((name, args.prec)),
                     "traffic_unit": "GB/launch",
                     "kernel": sigma_kernel_name(args.prec, c.get("nvir_act") or c["nvir"]),
                     "launches": st["launches"], "avg_launch_ms": 1e3 * st["seconds"] / max(st["launches"], 1),
                     "algorithmic_gflop_per_launch": st["flops"] / max(st["launches"], 1) / 1e9,
                     "algorithmic_gbytes_per_launch": st["bytes"] / max(st["launches"], 1) / 1e9},
        "sigma_mfma_tflops_algorithmic": achieved / 1e12,
        "n_sigma_per_step": h["n_sigma"] / args.steps,
        "sigma_kernel_share": st["seconds"] / h["elapsed"],
        "staging_s": h["t_build"],
        "solves_in_timed_window": h["solves_in_timed_window"],
        "converged": {"status": P.binding.STATUS_NAMES[r["status"]], "iters": r["report"]["iters"],
                      "n_sigma": r["report"]["n_sigma"], "solve_s": r["report"]["t_total_s"],
                      "omega_ha": [float(x) for x in r["omega"]],
                      "resid_per_root": [float(x) for x in r["resid"]],
                      "max_resid": float(np.max(r["resid"]))},
    }
    log(f"headline: {line['value']:.1f} sigma/s, kernel {line['roofline']['achieved']:.1f} TF "
        f"({line['roofline']['frac']:.3f}), converged max resid {line['converged']['max_resid']:.2e}")
    if args.headline_only:
        print(json.dumps(line), flush=True)
        return
    ref_omega = r["omega"] if (args.prec == "fp64" and r["status"] == 0) else None
    head_host = None
    if not args.no_cpu:  # the headline's integrals, on the host, for the oracle's sigma rate
        head_host = (problem[1].cpu().numpy(), problem[0].cpu().numpy())
    if not args.no_precision and name == "mixed":
        log("precision study ...")
        precs = ("fp32", "bf16x6", "bf16x3") if ref_omega is not None else ("fp64", "fp32", "bf16x6", "bf16x3")
        line["precision"] = precision_study(P, gen, precs=precs, name="mixed", problem=problem,
                                            ref=ref_omega)
    del problem
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("20/200/700 FP64 Davidson ...")
        line["fp64_davidson_20x200x700"], (eps_d, L_d) = fp64_davidson_pair(
            P, gen, steps=5, warmup=2, concurrent=args.concurrent)
        log("isolated sigma ...")
        line["isolated_sigma"] = isolated_sigma(P, gen, eps_d, L_d, 20, 20)
        log("hh channel ...")
        line["hh_channel"] = hh_channel(P, eps_d, L_d, 20, 10, 20, 1e-6)
        log("NTO analysis ...")
        line["nto_analysis"] = nto_analysis(P, eps_d, L_d, 20, 10, 20, 1e-6)
        del eps_d, L_d
        log("small direct workload ...")
        line["small_direct"] = small_direct(P, gen)
        line["correlation_energy"] = correlation_energy(P, gen)
        line["dense_large"] = dense_large(P, gen)
        line["unrestricted"] = unrestricted(P, gen)
    if not args.no_active:
        log("active-window study ...")
        line["active_window"] = precision_study(P, gen, precs=tuple(args.precs.split(",")),
                                                name="active", block=20)
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving stream ...")
        line["serving"] = serve_stream(P, gen, n_req=args.serve_requests or 128, n_sat=32,
                                       prec=args.serve_prec)
    if not args.no_cpu:
        log("timing the oracle on the host cores ...")
        line["cpu_baseline"] = cpu_baseline(head_L=head_host[0], head_eps=head_host[1], head_cfg=c)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Seeded synthetic ppRPA inputs: orbital energies and MO-basis three-centre integrals.

This module draws random numbers and nothing else: it holds none of the ppRPA arithmetic.
It is the one module that both the FP64 CPU oracle (``oracle/``) and the GPU path's
callers (tests, ``bench.py``) use, so that both see bit-identical inputs.

Every value is a pure function of (seed, stream, counter). The generator is the SplitMix64
output function (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) applied to ``base(seed, stream) + (counter + 1) * GAMMA``; normal deviates use the
Box-Muller transform (Box and Muller, Ann. Math. Statist. 29, 1958) on two 53-bit uniforms.
Because values are keyed by their full-space index, any slice of a tensor (an active window)
equals the same slice of the full tensor, and the full tensor never has to be built.

Orbital order everywhere is physical: occupied 0..nocc-1 (ascending energy), then virtual
nocc..nmo-1 (ascending energy).
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO53_INV = 1.0 / 9007199254740992.0  # 2**-53

# stream ids
STREAM_EPS_OCC = 1
STREAM_EPS_VIR = 2
STREAM_LPQ = 3
STREAM_SERVE = 4
STREAM_VECTORS = 5


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _base(seed: int, stream: int) -> np.uint64:
    s = np.array([(int(seed) & 0xFFFFFFFF) << 16 ^ (int(stream) & 0xFFFF)], dtype=np.uint64)
    return _mix64(_mix64(s))[0]


def hash64(seed: int, stream: int, counter: np.ndarray) -> np.ndarray:
    """64-bit hash of each counter (uint64 array) under (seed, stream)."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = _base(seed, stream) + (c + np.uint64(1)) * _GAMMA
    return _mix64(state)


def uniform(seed: int, stream: int, counter: np.ndarray) -> np.ndarray:
    """Uniform deviates in the open interval (0, 1), 53-bit resolution."""
    h = hash64(seed, stream, counter)
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO53_INV


def normal(seed: int, stream: int, counter: np.ndarray) -> np.ndarray:
    """Standard normal deviates, one per counter (Box-Muller, cosine branch)."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        u1 = uniform(seed, stream, c * np.uint64(2))
        u2 = uniform(seed, stream, c * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ----------------------------------------------------------------------------------------
# ppRPA inputs
# ----------------------------------------------------------------------------------------

def orbital_energies(seed: int, nocc: int, nvir: int,
                     occ_range=(-1.0, -0.3), vir_range=(0.0, 3.0)) -> np.ndarray:
    """MO energies [nmo] in Hartree: occupied uniform in occ_range, virtual uniform in
    vir_range, each block sorted ascending; occupied first."""
    uo = uniform(seed, STREAM_EPS_OCC, np.arange(nocc, dtype=np.uint64))
    uv = uniform(seed, STREAM_EPS_VIR, np.arange(nvir, dtype=np.uint64))
    eo = np.sort(occ_range[0] + (occ_range[1] - occ_range[0]) * uo)
    ev = np.sort(vir_range[0] + (vir_range[1] - vir_range[0]) * uv)
    return np.concatenate([eo, ev])


def lpq_scale(naux: int) -> float:
    return 0.3 / np.sqrt(float(naux))


def lpq_block(seed: int, nmo: int, naux: int, rows, cols, aux=None,
              scale: float | None = None, dtype=np.float64) -> np.ndarray:
    """Block L[P, p, q] of the full-space three-centre tensor, P in ``aux`` (default all),
    p in ``rows``, q in ``cols`` (full-space orbital indices).

    The full tensor is symmetric in (p, q); each p <= q entry is an independent N(0,1)
    deviate times ``scale`` (default 0.3/sqrt(naux)), keyed by
    (P, min(p, q), max(p, q)) in the full space of ``nmo`` orbitals.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    aux = np.arange(naux, dtype=np.int64) if aux is None else np.asarray(aux, dtype=np.int64)
    if scale is None:
        scale = lpq_scale(naux)
    lo = np.minimum(rows[:, None], cols[None, :]).astype(np.uint64)
    hi = np.maximum(rows[:, None], cols[None, :]).astype(np.uint64)
    pq = lo * np.uint64(nmo) + hi  # [nr, nc]
    out = np.empty((aux.size, rows.size, cols.size), dtype=dtype)
    nmo2 = np.uint64(nmo) * np.uint64(nmo)
    for i, P in enumerate(aux):
        cnt = np.uint64(P) * nmo2 + pq
        out[i] = (normal(seed, STREAM_LPQ, cnt) * scale).astype(dtype)
    return out


def lpq_full(seed: int, nmo: int, naux: int, dtype=np.float64) -> np.ndarray:
    """The whole [naux, nmo, nmo] tensor."""
    idx = np.arange(nmo)
    return lpq_block(seed, nmo, naux, idx, idx, dtype=dtype)


def active_indices(nocc: int, nvir: int, nocc_act: int | None, nvir_act: int | None):
    """Full-space indices of the active window: the highest nocc_act occupied and the
    lowest nvir_act virtual orbitals (all when None or <= 0), in physical order."""
    no = nocc if not nocc_act or nocc_act <= 0 else min(nocc_act, nocc)
    nv = nvir if not nvir_act or nvir_act <= 0 else min(nvir_act, nvir)
    return np.concatenate([np.arange(nocc - no, nocc), np.arange(nocc, nocc + nv)])


def lpq_active(seed: int, nocc: int, nvir: int, naux: int, nocc_act=None, nvir_act=None,
               dtype=np.float64) -> np.ndarray:
    """Active block of the full-space tensor, generated directly: [naux, nact, nact]."""
    idx = active_indices(nocc, nvir, nocc_act, nvir_act)
    return lpq_block(seed, nocc + nvir, naux, idx, idx, dtype=dtype)


def random_vectors(seed: int, k: int, n: int) -> np.ndarray:
    """k seeded N(0,1) test vectors of length n (for sigma parity)."""
    c = np.arange(k * n, dtype=np.uint64)
    return normal(seed, STREAM_VECTORS, c).reshape(k, n)


# ----------------------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------------------

CONFIGS = {
    # plain FP64, singlet, direct diagonalisation
    "small_direct": dict(nocc=5, nvir=20, naux=100, mult="singlet", nroot=5, seeds=(0, 1, 2, 3, 4)),
    # FP64 Davidson, singlet and triplet, 10 roots, block 20, tol 1e-6
    "davidson_fp64": dict(nocc=20, nvir=200, naux=700, mult=("singlet", "triplet"), nroot=10,
                          block=20, tol=1e-6, seeds=(0, 1)),
    # mixed precision, 20 singlet roots
    "mixed": dict(nocc=50, nvir=500, naux=1800, mult="singlet", nroot=20, seeds=(0,),
                  eig_scale=0.7),
    # active-space: full 120/1500/4000, window 40 occ + 400 vir, 16 triplet roots
    "active": dict(nocc=120, nvir=1500, naux=4000, nocc_act=40, nvir_act=400, mult="triplet",
                   nroot=16, seeds=(0,), eig_scale=0.7),
}
# eig_scale: at these two sizes the unscaled integrals make M - 2 mu W indefinite for every shift
# (the random interaction spreads wider than the orbital gap) and the pp and hh spectra overlap,
# which on smaller analogues of the same ratio gives complex roots: there are no well-defined
# lowest pp roots. Eigenvalue comparisons at these sizes therefore use L * eig_scale (definite
# with margin: lowest eigenvalue of M - 2 mu W is 0.18 Ha and 0.11 Ha); sigma throughput is
# measured on the unscaled integrals.


def serve_requests(master_seed: int, count: int = 512):
    """Request mix for the serving stream: nocc ~ U{4..40}, nvir ~ U{30..400},
    naux = round-half-up(3.5 * nmo), singlet/triplet 50/50, nroot ~ U{4..12}.
    Request r draws from sub-seed r. Every request carries eig_scale = 0.7 (its integrals are
    used as L * 0.7), for the reason given for the large workloads above: unscaled, about a fifth
    of the mix (those with nvir above about 250, mostly triplets) has an indefinite M - 2 mu W."""
    reqs = []
    for r in range(count):
        u = uniform(master_seed, STREAM_SERVE, np.arange(4, dtype=np.uint64) + np.uint64(8 * r))
        nocc = 4 + int(u[0] * 37)
        nvir = 30 + int(u[1] * 371)
        mult = "singlet" if u[2] < 0.5 else "triplet"
        nroot = 4 + int(u[3] * 9)
        naux = (7 * (nocc + nvir) + 1) // 2
        reqs.append(dict(rid=r, seed=r, nocc=nocc, nvir=nvir, naux=naux, mult=mult, nroot=nroot,
                         eig_scale=0.7))
    return reqs


def poisson_arrivals(master_seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    u = uniform(master_seed, STREAM_SERVE, np.arange(count, dtype=np.uint64) + np.uint64(1 << 40))
    return np.cumsum(-np.log(u) / rate)


# ----------------------------------------------------------------------------------------
# The same generator on torch tensors (any device): for the large workloads, whose integral
# slices are generated in device memory. The integer hash matches the NumPy version bit for bit
# (int64 tensors hold the uint64 bit patterns; multiplications wrap); the Box-Muller step uses
# torch's log/cos/sqrt and may differ from NumPy's in the last bits.
# ----------------------------------------------------------------------------------------

def _s64(x: int) -> int:
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(z, s: int):
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix64_t(z):
    z = z ^ _lsr(z, 30)
    z = z * _s64(0xBF58476D1CE4E5B9)
    z = z ^ _lsr(z, 27)
    z = z * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def _uniform_t(seed: int, stream: int, counter):
    import torch
    base = _s64(int(_base(seed, stream)))
    h = _mix64_t(base + (counter + 1) * _s64(0x9E3779B97F4A7C15))
    return (_lsr(h, 11).to(torch.float64) + 0.5) * _TWO53_INV


def lpq_block_torch(seed: int, nmo: int, naux: int, rows, cols, aux, device,
                    scale: float | None = None):
    """lpq_block on a torch device: [len(aux), len(rows), len(cols)] float64."""
    import torch
    rows = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=device)
    cols = torch.as_tensor(np.asarray(cols, dtype=np.int64), device=device)
    aux = torch.as_tensor(np.asarray(aux, dtype=np.int64), device=device)
    if scale is None:
        scale = float(lpq_scale(naux))
    lo = torch.minimum(rows[:, None], cols[None, :])
    hi = torch.maximum(rows[:, None], cols[None, :])
    pq = lo * nmo + hi
    cnt = aux[:, None, None] * (nmo * nmo) + pq[None]
    u1 = _uniform_t(seed, STREAM_LPQ, cnt * 2)
    u2 = _uniform_t(seed, STREAM_LPQ, cnt * 2 + 1)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * np.pi * u2) * scale

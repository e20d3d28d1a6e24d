"""ctypes binding of libpprpa.so (argument marshalling only; every step runs in the library).

The names mirror the C ABI in include/pprpa.h: ``pprpa_build``, ``pprpa_matvec``,
``pprpa_dense_matrix``, ``pprpa_davidson``, ``pprpa_free``. ``PpRPA`` wraps one context.

Host arrays are NumPy float64; device arrays are torch tensors (float64, contiguous, on the
context's GPU), passed by pointer. torch is used for nothing else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PPRPA_LIB: load another build of the library (e.g. to compare two kernel builds); default: the
# in-tree build.
LIB_PATH = os.environ.get("PPRPA_LIB") or os.path.join(_HERE, "libpprpa.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ENONDEF, EUNSUPPORTED, EBUSY = range(8)
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "ENOCONV", "ENONDEF", "EUNSUPPORTED", "EBUSY"]
MULT = {"singlet": 0, "triplet": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16x6": 2, "bf16x3": 3}
CHANNEL = {"pp": 0, "hh": 1}


class PpRPAError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


class BuildArgs(C.Structure):
    _fields_ = [("nmo", C.c_int32), ("nocc", C.c_int32), ("naux", C.c_int32),
                ("nocc_act", C.c_int32), ("nvir_act", C.c_int32),
                ("eps", C.c_void_p), ("Lpq", C.c_void_p),
                ("lpq_is_active", C.c_int32), ("on_device", C.c_int32),
                ("mult", C.c_int32), ("prec", C.c_int32), ("dense", C.c_int32),
                ("max_block", C.c_int32), ("stream", C.c_void_p)]


LOGFN = C.CFUNCTYPE(None, C.c_void_p, C.c_char_p)


class BuildAbArgs(C.Structure):
    _fields_ = [("nmo", C.c_int32), ("nocc_a", C.c_int32), ("nocc_b", C.c_int32),
                ("naux", C.c_int32), ("eps_a", C.c_void_p), ("eps_b", C.c_void_p),
                ("Lpq_a", C.c_void_p), ("Lpq_b", C.c_void_p), ("on_device", C.c_int32),
                ("max_block", C.c_int32), ("stream", C.c_void_p), ("density_fitted", C.c_int32),
                ("prec", C.c_int32)]


class DavidsonArgs(C.Structure):
    _fields_ = [("nroot", C.c_int32), ("block", C.c_int32), ("max_iter", C.c_int32),
                ("max_subspace", C.c_int32), ("tol", C.c_double), ("guess", C.c_void_p),
                ("nguess", C.c_int32), ("direct", C.c_int32), ("log", LOGFN),
                ("user", C.c_void_p), ("channel", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_sigma", C.c_int32), ("n_conv", C.c_int32),
                ("subspace", C.c_int32), ("max_resid", C.c_double), ("t_sigma_s", C.c_double),
                ("t_total_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CorrEnergy(C.Structure):
    _fields_ = [("ec_pp", C.c_double), ("ec_hh", C.c_double), ("trace_a", C.c_double),
                ("trace_c", C.c_double), ("n_pp_roots", C.c_int32), ("n_hh_roots", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("nroot", C.c_int32),
                ("max_overtaken", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("footprint", C.c_uint64), ("message", C.c_char * 256)]


class ServingStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("inflight", C.c_int64), ("peak_inflight", C.c_int64),
                ("budget", C.c_uint64), ("reserved", C.c_uint64), ("peak_reserved", C.c_uint64),
                ("group_launches", C.c_int64), ("grouped_products", C.c_int64),
                ("sigma_seconds", C.c_double), ("sigma_flops", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
EXPORTS = ["pprpa_build", "pprpa_dims", "pprpa_matvec", "pprpa_dense_matrix", "pprpa_davidson",
           "pprpa_free", "pprpa_strerror", "pprpa_last_error", "pprpa_sigma_stats",
           "pprpa_server_create", "pprpa_server_submit", "pprpa_server_poll", "pprpa_server_wait",
           "pprpa_server_stats", "pprpa_server_destroy", "pprpa_solve_begin", "pprpa_solve_iterate",
           "pprpa_solve_end", "pprpa_solve_stats", "pprpa_correlation_energy_noalloc"]


def lib():
    """Load libpprpa.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 / libhsa-runtime64.so.1.
    # Loading torch first makes the dynamic linker resolve this library's dependencies to those
    # already-loaded copies (same SONAME), so torch tensors and this library share a runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_12515_amd.build`"
                          " (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    L.pprpa_build.argtypes = [C.POINTER(BuildArgs), C.POINTER(C.c_void_p)]
    L.pprpa_build.restype = C.c_int
    L.pprpa_build_ab.argtypes = [C.POINTER(BuildAbArgs), C.POINTER(C.c_void_p)]
    L.pprpa_build_ab.restype = C.c_int
    L.pprpa_dims.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.pprpa_dims.restype = C.c_int
    L.pprpa_matvec.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]
    L.pprpa_matvec.restype = C.c_int
    L.pprpa_dense_matrix.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.pprpa_dense_matrix.restype = C.c_int
    L.pprpa_davidson.argtypes = [C.c_void_p, C.POINTER(DavidsonArgs), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.POINTER(Report)]
    L.pprpa_davidson.restype = C.c_int
    L.pprpa_solve_begin.argtypes = [C.c_void_p, C.POINTER(DavidsonArgs), C.POINTER(C.c_void_p)]
    L.pprpa_solve_begin.restype = C.c_int
    L.pprpa_solve_iterate.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
    L.pprpa_solve_iterate.restype = C.c_int
    L.pprpa_solve_end.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(Report)]
    L.pprpa_solve_end.restype = C.c_int
    L.pprpa_solve_stats.argtypes = [C.c_void_p, C.POINTER(KernelStats), C.c_int32]
    L.pprpa_solve_stats.restype = C.c_int
    L.pprpa_nto.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p]
    L.pprpa_nto.restype = C.c_int
    L.pprpa_nto_vectors.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.pprpa_nto_vectors.restype = C.c_int
    L.pprpa_correlation_energy.argtypes = [C.c_void_p, C.POINTER(CorrEnergy)]
    L.pprpa_correlation_energy.restype = C.c_int
    L.pprpa_correlation_energy_noalloc.argtypes = [C.c_void_p, C.POINTER(CorrEnergy)]
    L.pprpa_correlation_energy_noalloc.restype = C.c_int
    L.pprpa_sigma_stats.argtypes = [C.c_void_p, C.POINTER(KernelStats), C.c_int32]
    L.pprpa_sigma_stats.restype = C.c_int
    L.pprpa_free.argtypes = [C.c_void_p]
    L.pprpa_free.restype = None
    L.pprpa_strerror.argtypes = [C.c_int]
    L.pprpa_strerror.restype = C.c_char_p
    L.pprpa_last_error.argtypes = []
    L.pprpa_last_error.restype = C.c_char_p
    L.pprpa_server_create.argtypes = [C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]
    L.pprpa_server_create.restype = C.c_int
    L.pprpa_server_submit.argtypes = [C.c_void_p, C.POINTER(BuildArgs), C.POINTER(DavidsonArgs),
                                      C.POINTER(C.c_uint64)]
    L.pprpa_server_submit.restype = C.c_int
    L.pprpa_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(RequestInfo), C.c_void_p,
                                    C.c_void_p, C.POINTER(Report)]
    L.pprpa_server_poll.restype = C.c_int
    L.pprpa_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_double]
    L.pprpa_server_wait.restype = C.c_int
    L.pprpa_server_stats.argtypes = [C.c_void_p, C.POINTER(ServingStats)]
    L.pprpa_server_stats.restype = C.c_int
    L.pprpa_server_destroy.argtypes = [C.c_void_p]
    L.pprpa_server_destroy.restype = None
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise PpRPAError(status, lib().pprpa_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, on_device):
    if on_device:
        import torch  # noqa: F401  (only for tensors the caller handed in)
        assert x.dtype.itemsize == 8 and x.is_contiguous(), "device arrays must be contiguous float64"
        return C.c_void_p(x.data_ptr())
    assert x.dtype == np.float64 and x.flags["C_CONTIGUOUS"], "host arrays must be C-contiguous float64"
    return C.c_void_p(x.ctypes.data)


class PpRPA:
    """One staged ppRPA problem (a library context).

    eps: [nmo] orbital energies; Lpq: [naux, nmo, nmo] (or the active block with
    lpq_is_active). Both NumPy (host) or both torch CUDA tensors (device)."""

    def __init__(self, eps, Lpq, nocc, mult="singlet", prec="fp64", nocc_act=0, nvir_act=0,
                 lpq_is_active=False, dense=False, max_block=32, stream=None):
        on_dev = _is_torch(Lpq) and Lpq.is_cuda
        if not on_dev:
            eps = np.ascontiguousarray(eps, dtype=np.float64)
            Lpq = np.ascontiguousarray(Lpq, dtype=np.float64)
        a = BuildArgs()
        a.nmo = int(eps.shape[0])
        a.nocc = int(nocc)
        a.naux = int(Lpq.shape[0])
        a.nocc_act = int(nocc_act or 0)
        a.nvir_act = int(nvir_act or 0)
        a.eps = _ptr(eps, on_dev).value
        a.Lpq = _ptr(Lpq, on_dev).value
        a.lpq_is_active = int(bool(lpq_is_active))
        a.on_device = int(on_dev)
        a.mult = MULT[mult]
        a.prec = PREC[prec]
        a.dense = int(bool(dense))
        a.max_block = int(max_block)
        a.stream = stream
        h = C.c_void_p()
        _check(lib().pprpa_build(C.byref(a), C.byref(h)))
        self._h = h
        npp, nhh = C.c_int64(), C.c_int64()
        _check(lib().pprpa_dims(h, C.byref(npp), C.byref(nhh)))
        self.n_pp, self.n_hh = npp.value, nhh.value
        self.n = self.n_pp + self.n_hh
        self.mult, self.prec = mult, prec
        # orbitals of the active window (all virtual / occupied orbitals without one)
        self.nv = int(nvir_act) if nvir_act else a.nmo - a.nocc
        self.no = int(nocc_act) if nocc_act else a.nocc

    def _dims_active(self):
        return self.nv, self.no

    @classmethod
    def alpha_beta(cls, eps_a, eps_b, Lpq_a, Lpq_b, nocc_a, nocc_b, max_block=32, stream=None,
                   density_fitted=False, prec="fp64"):
        """The alpha-beta sector of spin-unrestricted ppRPA (pprpa_build_ab): a dense context, or
        with density_fitted=True the density-fitted sigma of both spins' integrals (no matrix;
        prec "fp64", "fp32", "bf16x6" or "bf16x3"); the alpha-alpha and beta-beta sectors are
        PpRPA(eps_s, Lpq_s, nocc_s, mult="triplet")."""
        on_dev = _is_torch(Lpq_a) and Lpq_a.is_cuda
        if not on_dev:
            eps_a, eps_b = (np.ascontiguousarray(x, dtype=np.float64) for x in (eps_a, eps_b))
            Lpq_a, Lpq_b = (np.ascontiguousarray(x, dtype=np.float64) for x in (Lpq_a, Lpq_b))
        a = BuildAbArgs()
        a.nmo, a.nocc_a, a.nocc_b = int(eps_a.shape[0]), int(nocc_a), int(nocc_b)
        a.naux = int(Lpq_a.shape[0])
        a.eps_a, a.eps_b = _ptr(eps_a, on_dev).value, _ptr(eps_b, on_dev).value
        a.Lpq_a, a.Lpq_b = _ptr(Lpq_a, on_dev).value, _ptr(Lpq_b, on_dev).value
        a.on_device, a.max_block, a.stream = int(on_dev), int(max_block), stream
        a.density_fitted = int(bool(density_fitted))
        a.prec = PREC[prec]
        h = C.c_void_p()
        _check(lib().pprpa_build_ab(C.byref(a), C.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        npp, nhh = C.c_int64(), C.c_int64()
        _check(lib().pprpa_dims(h, C.byref(npp), C.byref(nhh)))
        self.n_pp, self.n_hh = npp.value, nhh.value
        self.n = self.n_pp + self.n_hh
        self.mult, self.prec = "alpha-beta", prec
        self.nv, self.no = a.nmo - a.nocc_a, a.nocc_a
        self.nvb, self.nob = a.nmo - a.nocc_b, a.nocc_b
        return self

    def close(self):
        if getattr(self, "_h", None):
            lib().pprpa_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- sigma = M z ---------------------------------------------------------------------
    def matvec(self, z, out=None):
        """z: [k, n] (or [n]) NumPy or torch CUDA float64; returns sigma of the same kind."""
        on_dev = _is_torch(z) and z.is_cuda
        one = z.ndim == 1
        if on_dev:
            z2 = z.reshape(1, -1) if one else z
            z2 = z2.contiguous()
            s = out if out is not None else z2.new_empty(z2.shape)
        else:
            z2 = np.ascontiguousarray(np.atleast_2d(z), dtype=np.float64)
            s = np.empty_like(z2)
        assert z2.shape[1] == self.n, f"vectors must have length n={self.n}"
        _check(lib().pprpa_matvec(self._h, int(z2.shape[0]), _ptr(z2, on_dev), _ptr(s, on_dev),
                                  int(on_dev)))
        return s.reshape(-1) if one else s

    def sigma_stats(self, reset=False):
        """Event-timed launches of the sigma contraction kernel since the last reset."""
        st = KernelStats()
        _check(lib().pprpa_sigma_stats(self._h, C.byref(st), int(bool(reset))))
        return st.as_dict()

    def correlation_energy(self, noalloc=False):
        """ppRPA correlation energy of this spin block from the whole spectrum of the dense
        pencil (requires dense=True and n <= 8192): both sides of the sum rule, ec_pp = sum of
        the pp roots - Tr A and ec_hh = -(sum of the hh roots) - Tr C, and the root counts.
        noalloc=True: pprpa_correlation_energy_noalloc (workspace in the library's static device
        array, no device allocation)."""
        out = CorrEnergy()
        fn = lib().pprpa_correlation_energy_noalloc if noalloc else lib().pprpa_correlation_energy
        _check(fn(self._h, C.byref(out)))
        return out.as_dict()

    def nto(self, z, density=True):
        """NTO weights and two-electron density blocks of the packed roots z ([k][n], e.g. the
        vectors of davidson(..., vectors=True)): lam_p [k][nv], lam_h [k][no] (squared singular
        values of the triangular amplitude matrices, descending), and with density=True
        d_vv [k][nv][nv], d_oo [k][no][no]."""
        on_dev = _is_torch(z) and z.is_cuda
        if not on_dev:
            z = np.ascontiguousarray(np.atleast_2d(z), dtype=np.float64)
        k = int(z.shape[0])
        nv, no = self._dims_active()
        if self.mult == "alpha-beta":
            return self._nto_ab(z, on_dev, k, nv, no, density)
        lam_p, lam_h = np.empty((k, nv)), np.empty((k, no))
        d_vv = np.empty((k, nv, nv)) if density else None
        d_oo = np.empty((k, no, no)) if density else None
        _check(lib().pprpa_nto(self._h, k, _ptr(z, on_dev), int(on_dev), lam_p.ctypes.data,
                               lam_h.ctypes.data if no else None,
                               d_vv.ctypes.data if density else None,
                               d_oo.ctypes.data if (density and no) else None))
        return dict(lam_p=lam_p, lam_h=lam_h, d_vv=d_vv, d_oo=d_oo)

    def nto_vectors(self, z, nvec):
        """The leading nvec NTO pairs of the packed roots z ([k][n]) (pprpa_nto_vectors): c_p1
        [k][nvec][rows of X], c_p2 [k][nvec][columns of X], c_h1 / c_h2 likewise for Y, one vector
        per row, in the order of the weights of nto()."""
        on_dev = _is_torch(z) and z.is_cuda
        if not on_dev:
            z = np.ascontiguousarray(np.atleast_2d(z), dtype=np.float64)
        k = int(z.shape[0])
        rp, rh = self._dims_active()
        if self.mult == "alpha-beta":
            cp, ch = self.nvb, self.nob
        else:
            cp, ch = rp, rh
        out = {name: np.zeros((k, int(nvec), m)) for name, m in
               (("c_p1", rp), ("c_p2", cp), ("c_h1", rh), ("c_h2", ch))}
        ptr = {name: (a.ctypes.data if a.size else None) for name, a in out.items()}
        _check(lib().pprpa_nto_vectors(self._h, k, _ptr(z, on_dev), int(on_dev), int(nvec),
                                       ptr["c_p1"], ptr["c_p2"], ptr["c_h1"], ptr["c_h2"]))
        return out

    def _nto_ab(self, z, on_dev, k, nva, noa, density):
        """pprpa_nto on an alpha-beta context: lam_p [k][nvir_a], lam_h [k][nocc_a] and the
        spin-resolved density blocks d_vv_a [k][nvir_a][nvir_a] = X X^T, d_vv_b = X^T X,
        d_oo_a = -Y Y^T, d_oo_b = -Y^T Y."""
        nvb, nob = self.nvb, self.nob
        lam_p, lam_h = np.empty((k, nva)), np.empty((k, noa))
        dv = np.empty((k, nva * nva + nvb * nvb)) if density else None
        do = np.empty((k, noa * noa + nob * nob)) if density else None
        _check(lib().pprpa_nto(self._h, k, _ptr(z, on_dev), int(on_dev), lam_p.ctypes.data,
                               lam_h.ctypes.data if noa else None,
                               dv.ctypes.data if density else None,
                               do.ctypes.data if (density and do.size) else None))
        out = dict(lam_p=lam_p, lam_h=lam_h)
        if density:
            out.update(d_vv_a=dv[:, :nva * nva].reshape(k, nva, nva),
                       d_vv_b=dv[:, nva * nva:].reshape(k, nvb, nvb),
                       d_oo_a=do[:, :noa * noa].reshape(k, noa, noa),
                       d_oo_b=do[:, noa * noa:].reshape(k, nob, nob))
        return out

    def dense_matrix(self):
        M = np.empty((self.n, self.n))
        _check(lib().pprpa_dense_matrix(self._h, _ptr(M, False), 0))
        return M

    # -- eigensolvers ------------------------------------------------------------------------
    @staticmethod
    def _davidson_args(nroot, block, tol, max_iter, max_subspace, guess, direct, log, channel):
        """pprpa_davidson_args plus the Python objects that must outlive the call (guess array,
        log callback) and the list the log lines are collected in."""
        a = DavidsonArgs()
        a.nroot = int(nroot)
        a.channel = CHANNEL[channel]
        a.block = int(block)
        a.max_iter = int(max_iter)
        a.max_subspace = int(max_subspace)
        a.tol = float(tol)
        g = None
        if guess is not None:
            g = np.ascontiguousarray(np.atleast_2d(guess), dtype=np.float64)
            a.guess = g.ctypes.data
            a.nguess = g.shape[0]
        a.direct = int(bool(direct))
        lines = []
        cb = LOGFN(lambda u, s: (lines.append(s.decode()), log and log(s.decode())))
        a.log = cb
        return a, (g, cb), lines

    def solve_begin(self, nroot, block=0, tol=1e-6, max_iter=0, max_subspace=0, guess=None,
                    log=None, channel="pp"):
        """A Davidson solve advanced by the caller (pprpa_solve_begin); see Solve."""
        return Solve(self, nroot, block, tol, max_iter, max_subspace, guess, log, channel)

    def davidson(self, nroot, block=0, tol=1e-6, max_iter=0, max_subspace=0, guess=None,
                 direct=False, vectors=False, log=None, raise_noconv=True, channel="pp"):
        """channel "pp": the lowest nroot two-electron addition roots, ascending; "hh": the nroot
        two-electron removal roots nearest the gap, descending."""
        a, keep, lines = self._davidson_args(nroot, block, tol, max_iter, max_subspace, guess,
                                             direct, log, channel)
        omega = np.empty(nroot)
        resid = np.empty(nroot)
        vecs = np.empty((nroot, self.n)) if vectors else None
        rep = Report()
        st = lib().pprpa_davidson(self._h, C.byref(a), omega.ctypes.data,
                                  vecs.ctypes.data if vectors else None, resid.ctypes.data,
                                  C.byref(rep))
        msg = lib().pprpa_last_error().decode()
        if st not in (OK, ENOCONV) or (st == ENOCONV and raise_noconv):
            raise PpRPAError(st, msg)
        return dict(omega=omega, vecs=vecs, resid=resid, report=rep.as_dict(), status=st,
                    log=lines, message=msg)


class Solve:
    """pprpa_solve_begin / pprpa_solve_iterate / pprpa_solve_end: iterate(n) runs up to n
    Davidson iterations and returns how many ran; done tells whether the solve has finished;
    end() returns what PpRPA.davidson returns (and releases the context)."""

    def __init__(self, ctx, nroot, block, tol, max_iter, max_subspace, guess, log, channel):
        self._ctx = ctx
        self._a, self._keep, self.log = ctx._davidson_args(nroot, block, tol, max_iter,
                                                           max_subspace, guess, False, log,
                                                           channel)
        self.nroot = int(nroot)
        self.done = False
        self.iters = 0
        h = C.c_void_p()
        _check(lib().pprpa_solve_begin(ctx._h, C.byref(self._a), C.byref(h)))
        self._h = h

    def iterate(self, n=1):
        it, dn = C.c_int32(), C.c_int32()
        _check(lib().pprpa_solve_iterate(self._h, int(n), C.byref(it), C.byref(dn)))
        self.iters += it.value
        self.done = bool(dn.value)
        return it.value

    def sigma_stats(self, reset=False):
        """PpRPA.sigma_stats of the context while this solve holds it."""
        st = KernelStats()
        _check(lib().pprpa_solve_stats(self._h, C.byref(st), int(bool(reset))))
        return st.as_dict()

    def end(self, vectors=False, raise_noconv=True):
        omega = np.full(self.nroot, np.nan)
        resid = np.full(self.nroot, np.nan)
        vecs = np.empty((self.nroot, self._ctx.n)) if vectors else None
        rep = Report()
        st = lib().pprpa_solve_end(self._h, omega.ctypes.data,
                                   vecs.ctypes.data if vectors else None, resid.ctypes.data,
                                   C.byref(rep))
        self._h = None
        msg = lib().pprpa_last_error().decode()
        if st not in (OK, ENOCONV) or (st == ENOCONV and raise_noconv):
            raise PpRPAError(st, msg)
        return dict(omega=omega, vecs=vecs, resid=resid, report=rep.as_dict(), status=st,
                    log=self.log, message=msg)

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().pprpa_solve_end(self._h, None, None, None, None)
            except Exception:
                pass


class Server:
    """Serving loop (pprpa_server_*): admits solves by device footprint into an HBM arena of
    hbm_budget_bytes, keeps up to max_inflight of them on the device and groups their sigma
    products. Inputs of a request are kept referenced here until the library reports that it
    no longer reads them (state >= 1)."""

    QUEUED, RUNNING, DONE = 0, 1, 2

    def __init__(self, hbm_budget_bytes, max_inflight=16):
        h = C.c_void_p()
        _check(lib().pprpa_server_create(int(hbm_budget_bytes), int(max_inflight), C.byref(h)))
        self._h = h
        self._held = {}
        self._nroot = {}

    def submit(self, eps, Lpq, nocc, nroot, mult="singlet", prec="fp64", nocc_act=0, nvir_act=0,
               lpq_is_active=False, block=0, tol=1e-6, max_iter=0, max_subspace=0, channel="pp"):
        on_dev = _is_torch(Lpq) and Lpq.is_cuda
        if on_dev:
            import torch
            torch.cuda.current_stream(Lpq.device).synchronize()  # inputs complete before submit
        else:
            eps = np.ascontiguousarray(eps, dtype=np.float64)
            Lpq = np.ascontiguousarray(Lpq, dtype=np.float64)
        b = BuildArgs()
        b.nmo, b.nocc, b.naux = int(eps.shape[0]), int(nocc), int(Lpq.shape[0])
        b.nocc_act, b.nvir_act = int(nocc_act or 0), int(nvir_act or 0)
        b.eps, b.Lpq = _ptr(eps, on_dev).value, _ptr(Lpq, on_dev).value
        b.lpq_is_active, b.on_device = int(bool(lpq_is_active)), int(on_dev)
        b.mult, b.prec = MULT[mult], PREC[prec]
        d = DavidsonArgs()
        d.nroot, d.block, d.max_iter = int(nroot), int(block), int(max_iter)
        d.max_subspace, d.tol, d.channel = int(max_subspace), float(tol), CHANNEL[channel]
        t = C.c_uint64()
        _check(lib().pprpa_server_submit(self._h, C.byref(b), C.byref(d), C.byref(t)))
        self._held[t.value] = (eps, Lpq)
        self._nroot[t.value] = int(nroot)
        return t.value

    def poll(self, ticket):
        """Request state; once done also its roots, residuals and report (the ticket retires)."""
        info = RequestInfo()
        nroot = self._nroot.get(ticket, 64)
        omega, resid, rep = np.empty(nroot), np.empty(nroot), Report()
        _check(lib().pprpa_server_poll(self._h, int(ticket), C.byref(info), omega.ctypes.data,
                                       resid.ctypes.data, C.byref(rep)))
        out = dict(state=info.state, status=info.status, t_submit=info.t_submit,
                   t_admit=info.t_admit, t_done=info.t_done, footprint=info.footprint,
                   max_overtaken=info.max_overtaken,
                   message=info.message.decode(errors="replace"))
        if info.state >= self.RUNNING:
            self._held.pop(ticket, None)
        if info.state == self.DONE:
            self._nroot.pop(ticket, None)
            out.update(omega=omega, resid=resid, report=rep.as_dict())
        return out

    def wait(self, ticket, timeout=-1.0):
        _check(lib().pprpa_server_wait(self._h, int(ticket), float(timeout)))
        return self.poll(ticket)

    def stats(self):
        st = ServingStats()
        _check(lib().pprpa_server_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().pprpa_server_destroy(self._h)
            self._h = None
            self._held.clear()
            self._nroot.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# Plain-function forms with the C names (thin wrappers over PpRPA).
def pprpa_build(eps, Lpq, nocc, **kw):
    return PpRPA(eps, Lpq, nocc, **kw)


def pprpa_matvec(ctx, z):
    return ctx.matvec(z)


def pprpa_davidson(ctx, nroot, **kw):
    return ctx.davidson(nroot, **kw)


def pprpa_free(ctx):
    ctx.close()

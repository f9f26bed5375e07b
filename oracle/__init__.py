"""Plain FP64 CPU oracle of the deflated block-Jacobi PCG (A-DEF2) method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  The arithmetic lives
in ``dpcg_oracle.c`` (plain C, sequential sums, OpenMP over independent rows and
blocks); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, LIB_SAN, build

OK, NOT_CONVERGED, EINVAL, EBLOCK_NOT_SPD, ECOARSE_NOT_SPD, EBREAKDOWN, ENONFINITE = 0, 1, -1, -3, -4, -5, -7

_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("ORACLE_SANITIZED") == "1"
        path = LIB_SAN if san else LIB
        if not os.path.exists(path):
            build(sanitize=san)
        L = C.CDLL(path)
        P = C.c_void_p
        L.oracle_setup.argtypes = [C.POINTER(C.c_void_p), C.c_int64, P, P, P, C.c_int32, P, P, P,
                                   C.c_int32, P, C.POINTER(C.c_int64)]
        L.oracle_setup.restype = C.c_int
        L.oracle_destroy.argtypes = [P]
        L.oracle_solve.argtypes = [P, P, P, C.c_double, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), P, C.POINTER(C.c_int64)]
        L.oracle_solve.restype = C.c_int
        for name in ("oracle_spmv", "oracle_bj_apply", "oracle_coarse_solve", "oracle_coarse_matrix"):
            getattr(L, name).argtypes = [P, P, P] if name != "oracle_coarse_matrix" else [P, P]
        L.oracle_adef2_apply.argtypes = [P, P, P, P, C.c_int32]
        L.oracle_start.argtypes = [P, P, P, P, P, C.c_int32]
        L.oracle_prepare_fast.argtypes = [P]
        L.oracle_prepare_fast.restype = C.c_int
        L.oracle_coarse_inverse.argtypes = [P, P]
        L.oracle_zt_times.argtypes = [P, P, P]
        L.oracle_x_plus_z_times.argtypes = [P, P, P, P]
        L.oracle_k.argtypes = [P]
        L.oracle_k.restype = C.c_int32
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = C.c_int32
        _lib = L
    return _lib


def threads():
    """OpenMP threads the oracle's parallel loops run on."""
    return int(lib().oracle_threads())


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, status, bad=-1):
        super().__init__(f"oracle status {status} (bad index {bad})")
        self.status, self.bad = status, bad


class Oracle:
    """Setup (block Cholesky factors, E = Z^T K Z and its Cholesky) plus solves."""

    def __init__(self, n, k_rowptr, k_col, k_val, k, z_rowptr, z_col, z_val, block_ptr):
        self.n, self.k = int(n), int(k)
        self._keep = [np.ascontiguousarray(k_rowptr, np.int64), np.ascontiguousarray(k_col, np.int32),
                      np.ascontiguousarray(k_val, np.float64), np.ascontiguousarray(z_rowptr, np.int64),
                      np.ascontiguousarray(z_col, np.int32), np.ascontiguousarray(z_val, np.float64),
                      np.ascontiguousarray(block_ptr, np.int32)]
        kp, kc, kv, zp, zc, zv, bp = self._keep
        h = C.c_void_p()
        bad = C.c_int64()
        st = lib().oracle_setup(C.byref(h), self.n, _p(kp), _p(kc), _p(kv), self.k, _p(zp), _p(zc), _p(zv),
                                len(bp) - 1, _p(bp), C.byref(bad))
        if st != OK:
            raise OracleError(st, bad.value)
        self._h = h

    @classmethod
    def from_problem(cls, p):
        return cls(p.n, p.k_rowptr, p.k_col, p.k_val, p.k, p.z_rowptr, p.z_col, p.z_val, p.block_ptr)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().oracle_destroy(h)
            self._h = None

    def solve(self, f, tol=1e-8, max_iter=20000, u0=None, history=False, fast=False):
        """Returns dict(u, status, iterations, rel_res, rel_res_true, history, bad).
        fast=True runs the fast mode (same iterates up to rounding, exact rewrites:
        precomputed K Z, one merged coarse solve by the explicit E^-1)."""
        f = np.ascontiguousarray(f, np.float64)
        u = np.zeros(self.n) if u0 is None else np.array(u0, np.float64, copy=True)
        hist = np.zeros(max_iter + 1) if history else None
        it = C.c_int32()
        rr = C.c_double()
        rt = C.c_double()
        bad = C.c_int64()
        st = lib().oracle_solve(self._h, _p(f), _p(u), float(tol), int(max_iter), int(u0 is not None), int(fast),
                                C.byref(it), C.byref(rr), C.byref(rt), _p(hist), C.byref(bad))
        out = dict(u=u, status=st, iterations=it.value, rel_res=rr.value, rel_res_true=rt.value,
                   bad=bad.value)
        if history:
            out["history"] = hist[: it.value + 1]
        return out

    def _vec(self, fn, x, m=None):
        x = np.ascontiguousarray(x, np.float64)
        y = np.zeros(self.n if m is None else m)
        getattr(lib(), fn)(self._h, _p(x), _p(y))
        return y

    def spmv(self, x):
        return self._vec("oracle_spmv", x)

    def bj_apply(self, r):
        return self._vec("oracle_bj_apply", r)

    def coarse_solve(self, b):
        return self._vec("oracle_coarse_solve", b, self.k)

    def coarse_matrix(self):
        E = np.zeros((self.k, self.k))
        lib().oracle_coarse_matrix(self._h, _p(E))
        return E

    def zt_times(self, x):
        return self._vec("oracle_zt_times", x, self.k)

    def x_plus_z_times(self, x, c):
        c = np.ascontiguousarray(c, np.float64)
        xx = None if x is None else np.ascontiguousarray(x, np.float64)
        y = np.zeros(self.n)
        lib().oracle_x_plus_z_times(self._h, _p(xx), _p(c), _p(y))
        return y

    def adef2_apply(self, r, fast=False):
        r = np.ascontiguousarray(r, np.float64)
        z = np.zeros(self.n)
        y = np.zeros(self.n)
        lib().oracle_adef2_apply(self._h, _p(r), _p(z), _p(y), int(fast))
        return z, y

    def start(self, f, u_m1=None, fast=False):
        f = np.ascontiguousarray(f, np.float64)
        um = None if u_m1 is None else np.ascontiguousarray(u_m1, np.float64)
        u0 = np.zeros(self.n)
        r0 = np.zeros(self.n)
        lib().oracle_start(self._h, _p(f), _p(um), _p(u0), _p(r0), int(fast))
        return u0, r0

    def prepare_fast(self):
        """Builds the fast mode's Z^T, (K Z)^T and explicit E^-1 (done on first use)."""
        lib().oracle_prepare_fast(self._h)

    def coarse_inverse(self):
        """The fast mode's explicit E^-1 = L^-T L^-1 (k x k)."""
        Ei = np.zeros((self.k, self.k))
        lib().oracle_coarse_inverse(self._h, _p(Ei))
        return Ei

"""ctypes binding of libdpcg.so (argument marshalling only).

Every computation runs in the library's HIP kernels; PyTorch supplies device
memory and the HIP stream.  There is no fallback: if the shared library is not
built, importing a solver raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpcg.so")

OK, NOT_CONVERGED, EINVAL, ENOTSYM, EBLOCK_NOT_SPD, ECOARSE_NOT_SPD, EBREAKDOWN, EHIP, ENONFINITE, ETOOBIG = (
    0, 1, -1, -2, -3, -4, -5, -6, -7, -8)


PREC_FP64, PREC_MIXED = 0, 1
PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED}


class Options(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("check_every", C.c_int32), ("use_initial_guess", C.c_int32),
                ("record_history", C.c_int32), ("precision", C.c_int32), ("max_refinements", C.c_int32),
                ("inner_tol", C.c_double), ("switch_tol", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("bad_index", C.c_int64), ("refinements", C.c_int32), ("iterations_fp64", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("n", "nnz", "nnzb", "k", "nnz_z", "nnz_kz", "nblocks", "bj_values",
                                         "device_bytes", "dense_blocks", "dense_values", "spmv_col_bytes")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("spmv_launches", C.c_int64), ("spmv_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

P = C.c_void_p
# name -> (restype, argtypes), mirroring include/dpcg.h
SIGNATURES = {
    "dpcg_default_options": (None, [C.POINTER(Options)]),
    "dpcg_setup": (C.c_int, [C.POINTER(P), C.c_int64, P, P, P, C.c_int32, P, P, P, C.c_int32, P, P,
                             C.POINTER(Info)]),
    "dpcg_setup_host": (C.c_int, [C.POINTER(P), C.c_int64, P, P, P, C.c_int32, P, P, P, C.c_int32, P, P,
                                  C.POINTER(Info)]),
    "dpcg_solve": (C.c_int, [P, P, P, C.c_double, C.POINTER(Options), C.POINTER(Info)]),
    "dpcg_solve_noalloc": (C.c_int, [P, P, P, C.c_double, C.POINTER(Options), C.POINTER(Info)]),
    "dpcg_noalloc_scratch_bytes": (C.c_size_t, []),
    "dpcg_solve_adjoint": (C.c_int, [P, P, P, C.c_double, C.POINTER(Options), C.POINTER(Info)]),
    "dpcg_solve_batch": (C.c_int, [P, C.c_int32, P, P, C.c_double, C.POINTER(Options), P]),
    "dpcg_solve_many": (C.c_int, [P, C.c_int32, P, P, C.c_double, C.POINTER(Options), P]),
    "dpcg_autotune": (C.c_int, [P, C.c_int32]),
    "dpcg_update_values": (C.c_int, [P, P, P, P, C.c_int32, P, C.POINTER(Info)]),
    "dpcg_destroy": (None, [P]),
    "dpcg_release_cached_memory": (None, []),
    "dpcg_status_string": (C.c_char_p, [C.c_int]),
    "dpcg_get_stats": (C.c_int, [P, C.POINTER(Stats)]),
    "dpcg_get_history": (C.c_int64, [P, P, C.c_int64]),
    "dpcg_set_timing": (C.c_int, [P, C.c_int32]),
    "dpcg_get_timing": (C.c_int, [P, C.POINTER(Timing)]),
    "dpcg_spmv": (C.c_int, [P, P, P]),
    "dpcg_spmv_fp32": (C.c_int, [P, P, P]),
    "dpcg_spmv_batch": (C.c_int, [P, C.c_int32, P, P]),
    "dpcg_bj_apply": (C.c_int, [P, P, P]),
    "dpcg_bj_apply_fp32": (C.c_int, [P, P, P]),
    "dpcg_restrict": (C.c_int, [P, P, P, P]),
    "dpcg_element_gradient": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P]),
    "dpcg_coarse_apply": (C.c_int, [P, P, P]),
    "dpcg_prolong": (C.c_int, [P, P, P, P]),
    "dpcg_precond": (C.c_int, [P, P, P]),
}


def lib():
    """The loaded libdpcg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().dpcg_status_string(int(code)).decode()


class DpcgError(RuntimeError):
    def __init__(self, code, where, info=None):
        self.code = int(code)
        self.info = info
        bad = f", bad index {info.bad_index}" if info is not None and info.bad_index >= 0 else ""
        super().__init__(f"{where}: {status_string(code)} (status {code}{bad})")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t


class Solver:
    """Handle of the deflated block-Jacobi CG solver for one matrix K.

    All arrays are device tensors: K as CSR (int64 rowptr, int32 col, float64 val),
    Z as CSR (same types), the block partition as int32.  The library copies what
    it keeps; the tensors may be released after construction.
    """

    def __init__(self, n, k_rowptr, k_col, k_val, k, z_rowptr, z_col, z_val, block_ptr, stream=None):
        import torch
        self.n, self.k = int(n), int(k)
        _check_dev(k_rowptr, torch.int64, "k_rowptr", self.n + 1)
        _check_dev(k_col, torch.int32, "k_col")
        _check_dev(k_val, torch.float64, "k_val", k_col.numel())
        _check_dev(block_ptr, torch.int32, "block_ptr")
        if self.k > 0:
            _check_dev(z_rowptr, torch.int64, "z_rowptr", self.n + 1)
            _check_dev(z_col, torch.int32, "z_col")
            _check_dev(z_val, torch.float64, "z_val", z_col.numel())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = k_val.device
        h = C.c_void_p()
        info = Info()
        st = lib().dpcg_setup(C.byref(h), self.n, _ptr(k_rowptr), _ptr(k_col), _ptr(k_val), self.k,
                              _ptr(z_rowptr) if self.k else None, _ptr(z_col) if self.k else None,
                              _ptr(z_val) if self.k else None, block_ptr.numel() - 1, _ptr(block_ptr),
                              C.c_void_p(self.stream.cuda_stream), C.byref(info))
        if st != OK:
            raise DpcgError(st, "dpcg_setup", info)
        self._h = h
        self.setup_info = info.as_dict()

    @classmethod
    def from_problem(cls, p, device="cuda", stream=None):
        """Uploads a fixtures.Problem (numpy arrays) and builds the solver."""
        import torch
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()  # noqa: E731
        zr = t(p.z_rowptr, torch.int64) if p.k else None
        return cls(p.n, t(p.k_rowptr, torch.int64), t(p.k_col, torch.int32), t(p.k_val, torch.float64), p.k,
                   zr, t(p.z_col, torch.int32) if p.k else None, t(p.z_val, torch.float64) if p.k else None,
                   t(p.block_ptr, torch.int32), stream=stream)

    @classmethod
    def from_host_arrays(cls, n, k_rowptr, k_col, k_val, k, z_rowptr, z_col, z_val, block_ptr, stream=None):
        """Builds the solver from host (numpy) CSR arrays through dpcg_setup_host."""
        import numpy as np
        import torch
        arr = lambda a, dt: np.ascontiguousarray(a, dtype=dt)  # noqa: E731
        keep = [arr(k_rowptr, np.int64), arr(k_col, np.int32), arr(k_val, np.float64),
                arr(z_rowptr, np.int64) if k else None, arr(z_col, np.int32) if k else None,
                arr(z_val, np.float64) if k else None, arr(block_ptr, np.int32)]
        hp = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self = cls.__new__(cls)
        self.n, self.k = int(n), int(k)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        h = C.c_void_p()
        info = Info()
        st = lib().dpcg_setup_host(C.byref(h), self.n, hp(keep[0]), hp(keep[1]), hp(keep[2]), self.k, hp(keep[3]),
                                   hp(keep[4]), hp(keep[5]), len(keep[6]) - 1, hp(keep[6]),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(info))
        if st != OK:
            self._h = None
            raise DpcgError(st, "dpcg_setup_host", info)
        self._h = h
        self.setup_info = info.as_dict()
        return self

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().dpcg_destroy(h)
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

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("solver is closed")
        return self._h

    # ------------------------------------------------------------------ solves
    def _opts(self, max_iter, check_every, guess, record, precision="fp64", inner_tol=None, max_refinements=None, switch_tol=None):
        o = Options()
        lib().dpcg_default_options(C.byref(o))
        if max_iter is not None:
            o.max_iter = int(max_iter)
        if check_every is not None:
            o.check_every = int(check_every)
        o.use_initial_guess = int(bool(guess))
        o.record_history = int(bool(record))
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        o.precision = PRECISIONS[precision]
        if inner_tol is not None:
            o.inner_tol = float(inner_tol)
        if max_refinements is not None:
            o.max_refinements = int(max_refinements)
        if switch_tol is not None:
            o.switch_tol = float(switch_tol)
        return o

    def _run(self, fn, where, f, u, tol, max_iter, check_every, initial_guess, record_history, raise_on_error,
             precision="fp64", inner_tol=None, max_refinements=None, switch_tol=None):
        import torch
        _check_dev(f, torch.float64, "rhs", self.n)
        if u is None:
            u = torch.empty(self.n, dtype=torch.float64, device=f.device)
        _check_dev(u, torch.float64, "solution", self.n)
        if initial_guess is not None:
            _check_dev(initial_guess, torch.float64, "initial_guess", self.n)
            if initial_guess.data_ptr() != u.data_ptr():
                u.copy_(initial_guess)
        o = self._opts(max_iter, check_every, initial_guess is not None, record_history, precision, inner_tol,
                       max_refinements, switch_tol)
        info = Info()
        st = fn(self.handle, _ptr(f), _ptr(u), float(tol), C.byref(o), C.byref(info))
        if st < 0 and raise_on_error:
            raise DpcgError(st, where, info)
        return u, info.as_dict()

    def solve(self, f, u=None, tol=1e-8, max_iter=None, check_every=None, initial_guess=None,
              record_history=False, raise_on_error=True, precision="fp64", inner_tol=None, max_refinements=None, switch_tol=None):
        """u = K^{-1} f to ||r||/||f|| <= tol.  precision "mixed" runs FP64 iterative
        refinement around inner solves on binary32 copies of K and the block inverses
        down to switch_tol, then the FP64 method from that iterate to tol.
        Returns (u, info dict)."""
        return self._run(lib().dpcg_solve, "dpcg_solve", f, u, tol, max_iter, check_every, initial_guess,
                         record_history, raise_on_error, precision, inner_tol, max_refinements, switch_tol)

    def solve_adjoint(self, g, lam=None, tol=1e-8, max_iter=None, check_every=None, initial_guess=None,
                      raise_on_error=True, precision="fp64", inner_tol=None, max_refinements=None, switch_tol=None):
        """lambda = K^{-1} g in the adjoint workspace.  Returns (lambda, info dict)."""
        return self._run(lib().dpcg_solve_adjoint, "dpcg_solve_adjoint", g, lam, tol, max_iter, check_every,
                         initial_guess, False, raise_on_error, precision, inner_tol, max_refinements, switch_tol)

    def solve_batch(self, F, U=None, tol=1e-8, max_iter=None, check_every=None, initial_guess=None,
                    raise_on_error=True):
        """U = K^{-1} F for an n x nrhs float64 device tensor F (1 <= nrhs <= 32), each
        column its own recurrence sharing the passes over the operator.  Returns
        (U, list of per-column info dicts)."""
        import torch
        if F.dim() != 2 or F.shape[0] != self.n:
            raise ValueError(f"F must be {self.n} x nrhs")
        nrhs = F.shape[1]
        _check_dev(F, torch.float64, "F")
        if U is None:
            U = torch.empty_like(F)
        _check_dev(U, torch.float64, "U", F.numel())
        if initial_guess is not None:
            _check_dev(initial_guess, torch.float64, "initial_guess", F.numel())
            if initial_guess.data_ptr() != U.data_ptr():
                U.copy_(initial_guess)
        o = self._opts(max_iter, check_every, initial_guess is not None, False)
        infos = (Info * max(1, nrhs))()
        st = lib().dpcg_solve_batch(self.handle, int(nrhs), _ptr(F), _ptr(U), float(tol), C.byref(o),
                                    C.cast(infos, C.c_void_p))
        if st < 0 and raise_on_error:
            raise DpcgError(st, "dpcg_solve_batch", infos[0] if nrhs else None)
        return U, [infos[j].as_dict() for j in range(nrhs)]

    def history(self):
        import numpy as np
        buf = np.zeros(200001)
        m = lib().dpcg_get_history(self.handle, buf.ctypes.data_as(C.c_void_p), len(buf))
        if m < 0:
            raise DpcgError(m, "dpcg_get_history")
        return buf[:m].copy()

    def stats(self):
        s = Stats()
        st = lib().dpcg_get_stats(self.handle, C.byref(s))
        if st != OK:
            raise DpcgError(st, "dpcg_get_stats")
        return s.as_dict()

    def set_timing(self, on=True, every=1):
        """Event timing of every `every`-th SpMV launch of the solves (off with on=False)."""
        st = lib().dpcg_set_timing(self.handle, int(every) if on else 0)
        if st != OK:
            raise DpcgError(st, "dpcg_set_timing")

    def timing(self):
        t = Timing()
        st = lib().dpcg_get_timing(self.handle, C.byref(t))
        if st != OK:
            raise DpcgError(st, "dpcg_get_timing")
        return t.as_dict()

    # ------------------------------------------------------------------ single steps
    def _call(self, name, *args):
        st = getattr(lib(), name)(self.handle, *[_ptr(a) for a in args])
        if st != OK:
            raise DpcgError(st, name)

    def spmv(self, x, y=None):
        import torch
        _check_dev(x, torch.float64, "x", self.n)
        y = torch.empty_like(x) if y is None else y
        self._call("dpcg_spmv", x, y)
        return y

    def spmv_batch(self, X):
        """Y = K X for an n x nrhs float64 device tensor X (1 <= nrhs <= 32) with the
        multi-RHS product of solve_batch."""
        import torch
        if X.dim() != 2 or X.shape[0] != self.n:
            raise ValueError(f"X must be {self.n} x nrhs")
        _check_dev(X, torch.float64, "X")
        Y = torch.empty_like(X)
        st = lib().dpcg_spmv_batch(self.handle, int(X.shape[1]), _ptr(X), _ptr(Y))
        if st != OK:
            raise DpcgError(st, "dpcg_spmv_batch")
        return Y

    def bj_apply(self, r):
        import torch
        _check_dev(r, torch.float64, "r", self.n)
        y = torch.empty_like(r)
        self._call("dpcg_bj_apply", r, y)
        return y

    def element_gradient(self, elements, u, lam):
        """g[e] = -lam_e^T K_e u_e for the element data `elements` (an Elements)."""
        import torch
        _check_dev(u, torch.float64, "u", self.n)
        _check_dev(lam, torch.float64, "lambda", self.n)
        g = torch.empty(elements.nel, dtype=torch.float64, device=u.device)
        st = lib().dpcg_element_gradient(self.handle, elements.nel, _ptr(elements.elem_ptr),
                                         _ptr(elements.elem_dof), _ptr(elements.kmat_off), elements.kmat.numel(),
                                         _ptr(elements.kmat), _ptr(u), _ptr(lam), _ptr(g))
        if st != OK:
            raise DpcgError(st, "dpcg_element_gradient")
        return g

    def update_values(self, k_rowptr, k_col, k_val, changed_blocks=None):
        """New values of K on the setup's pattern; only the listed block-Jacobi blocks
        (all when None) are refactorised.  Returns the info dict (setup_ms = update time)."""
        import numpy as np
        import torch
        _check_dev(k_rowptr, torch.int64, "k_rowptr", self.n + 1)
        _check_dev(k_col, torch.int32, "k_col")
        _check_dev(k_val, torch.float64, "k_val", k_col.numel())
        info = Info()
        if changed_blocks is None:
            st = lib().dpcg_update_values(self.handle, _ptr(k_rowptr), _ptr(k_col), _ptr(k_val), -1, None,
                                          C.byref(info))
        else:
            blk = np.ascontiguousarray(changed_blocks, dtype=np.int32)
            st = lib().dpcg_update_values(self.handle, _ptr(k_rowptr), _ptr(k_col), _ptr(k_val), len(blk),
                                          blk.ctypes.data_as(C.c_void_p), C.byref(info))
        if st != OK:
            raise DpcgError(st, "dpcg_update_values", info)
        return info.as_dict()

    def autotune(self, reps=5):
        """Measures the SpMV lane-group sizes and keeps the fastest; returns it."""
        g = lib().dpcg_autotune(self.handle, int(reps))
        if g < 0:
            raise DpcgError(g, "dpcg_autotune")
        return g

    def spmv_fp32(self, x, y=None):
        """y = K32 x: K's values rounded to binary32, FP64 arithmetic."""
        import torch
        _check_dev(x, torch.float64, "x", self.n)
        y = torch.empty_like(x) if y is None else y
        self._call("dpcg_spmv_fp32", x, y)
        return y

    def bj_apply_fp32(self, r):
        """y = M32^{-1} r with the block inverses rounded to binary32."""
        import torch
        _check_dev(r, torch.float64, "r", self.n)
        y = torch.empty_like(r)
        self._call("dpcg_bj_apply_fp32", r, y)
        return y

    def restrict(self, a, b=None):
        import torch
        _check_dev(a, torch.float64, "a", self.n)
        if b is not None:
            _check_dev(b, torch.float64, "b", self.n)
        g = torch.zeros(max(self.k, 1), dtype=torch.float64, device=a.device)
        self._call("dpcg_restrict", a, b, g)
        return g[: self.k]

    def coarse_apply(self, g):
        import torch
        _check_dev(g, torch.float64, "g", self.k)
        d = torch.zeros(max(self.k, 1), dtype=torch.float64, device=g.device)
        self._call("dpcg_coarse_apply", g, d)
        return d[: self.k]

    def prolong(self, delta, base=None):
        import torch
        _check_dev(delta, torch.float64, "delta", self.k)
        out = torch.empty(self.n, dtype=torch.float64, device=delta.device)
        self._call("dpcg_prolong", base, delta, out)
        return out

    def precond(self, r):
        import torch
        _check_dev(r, torch.float64, "r", self.n)
        z = torch.empty_like(r)
        self._call("dpcg_precond", r, z)
        return z


def solve_many(solvers, fs, us=None, tol=1e-8, max_iter=None, check_every=None, initial_guesses=None,
               raise_on_error=True):
    """Independent systems solved together (one launch per iteration phase for all):
    solvers[i] solves K_i u_i = fs[i].  Returns (list of u, list of info dicts)."""
    import torch
    m = len(solvers)
    if m != len(fs) or m == 0:
        raise ValueError("one right-hand side per solver")
    if us is None:
        us = [torch.empty_like(f) for f in fs]
    for s, f, u in zip(solvers, fs, us):
        _check_dev(f, torch.float64, "rhs", s.n)
        _check_dev(u, torch.float64, "solution", s.n)
    if initial_guesses is not None:
        for u, g in zip(us, initial_guesses):
            if g.data_ptr() != u.data_ptr():
                u.copy_(g)
    o = solvers[0]._opts(max_iter, check_every, initial_guesses is not None, False)
    hs = (C.c_void_p * m)(*[s.handle.value for s in solvers])
    fp = (C.c_void_p * m)(*[f.data_ptr() for f in fs])
    up = (C.c_void_p * m)(*[u.data_ptr() for u in us])
    infos = (Info * m)()
    st = lib().dpcg_solve_many(C.cast(hs, C.c_void_p), m, C.cast(fp, C.c_void_p), C.cast(up, C.c_void_p),
                               float(tol), C.byref(o), C.cast(infos, C.c_void_p))
    if st < 0 and raise_on_error:
        raise DpcgError(st, "dpcg_solve_many", infos[0])
    return us, [infos[i].as_dict() for i in range(m)]


class Elements:
    """Element matrices K_e (for a unit scaling) and their DoF lists, as device tensors,
    for dpcg_element_gradient: elem_ptr int64 (nel+1), elem_dof int32 (-1 = removed
    DoF), kmat_off int64 (nel), kmat float64 (row-major m_e x m_e blocks)."""

    def __init__(self, elem_ptr, elem_dof, kmat_off, kmat, device="cuda"):
        import torch
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()  # noqa: E731
        self.elem_ptr = t(elem_ptr, torch.int64)
        self.elem_dof = t(elem_dof, torch.int32)
        self.kmat_off = t(kmat_off, torch.int64)
        self.kmat = t(kmat, torch.float64)
        self.nel = self.kmat_off.numel()
        if self.elem_ptr.numel() != self.nel + 1:
            raise ValueError("elem_ptr must have nel + 1 entries")

"""dpcg_solve_noalloc (the solve with its workspace in the library's fixed device
array) against dpcg_solve, through the C ABI: two calls in a row on different
systems, the second smaller, each equal to the ordinary solve of its handle (same
kernels and launch shapes, so bitwise equal), and the device's free memory unchanged
by the calls."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2111_09294_amd as D  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _noalloc(s, f, u, tol=1e-8, **kw):
    o = D.abi.Options()
    D.abi.lib().dpcg_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    info = D.abi.Info()
    st = D.abi.lib().dpcg_solve_noalloc(s.handle, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), tol,
                                        C.byref(o), C.byref(info))
    return st, info.as_dict()


def test_noalloc_solve_equals_solve(problems):
    assert D.abi.lib().dpcg_noalloc_scratch_bytes() == 96 << 20
    big, small = problems("penny40"), problems("penny12")
    sb, ss = D.Solver.from_problem(big, DEV), D.Solver.from_problem(small, DEV)
    try:
        fb = torch.as_tensor(big.f, device=DEV)
        fs = torch.as_tensor(small.f, device=DEV)
        ub_ref, ib_ref = sb.solve(fb)
        us_ref, is_ref = ss.solve(fs)
        ub, us = torch.empty_like(fb), torch.empty_like(fs)
        for rep in range(2):
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            st_b, ib = _noalloc(sb, fb, ub)
            st_s, is_ = _noalloc(ss, fs, us)          # second call, smaller system
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            say(f"[noalloc] pass {rep}: penny40 {ib['iterations']} it ({ib['solve_ms']:.2f} ms), penny12 "
                f"{is_['iterations']} it; free device memory {free0} -> {free1}")
            assert st_b == D.abi.OK and st_s == D.abi.OK
            assert ib["iterations"] == ib_ref["iterations"] and is_["iterations"] == is_ref["iterations"]
            assert torch.equal(ub, ub_ref) and torch.equal(us, us_ref)
            assert ib["rel_res_true"] == ib_ref["rel_res_true"]
            if rep > 0:
                assert free1 >= free0
        # the handles' own workspaces are untouched: ordinary solves still match
        u2, i2 = sb.solve(fb)
        assert torch.equal(u2, ub_ref)
        # options outside the entry point's scope
        assert _noalloc(ss, fs, us, record_history=1)[0] == D.abi.EINVAL
        assert _noalloc(ss, fs, us, precision=D.abi.PREC_MIXED)[0] == D.abi.EINVAL
        # a warm start and an iteration cap behave as in dpcg_solve
        st, i3 = _noalloc(ss, fs, us, max_iter=7)
        u3, i3_ref = ss.solve(fs, max_iter=7)
        assert st == D.abi.NOT_CONVERGED and i3["iterations"] == 7 and torch.equal(us, u3)
        g = us.clone()
        st, i4 = _noalloc(ss, fs, g, use_initial_guess=1)
        u4, i4_ref = ss.solve(fs, initial_guess=u3)
        assert st == D.abi.OK and i4["iterations"] == i4_ref["iterations"] and torch.equal(g, u4)
    finally:
        sb.close()
        ss.close()

"""GPU parity of the mixed-precision path: FP64 iterative refinement around inner
solves by the same method on binary32 copies of K's values and of the block-Jacobi
inverses (vectors, E^-1 and all arithmetic stay FP64).

Tolerances:
* K32 x against the FP64 product with K's values rounded to binary32: 1e-13 relative
  to sum_j |K32_ij x_j| (summation order only);
* M32^-1 r against numpy's inverses of the diagonal blocks, rounded to binary32 and
  applied in FP64: 1.2e-7 (|M32^-1| |r|)_i (the two FP64 inverses agree to about
  1e-10, so their binary32 roundings may differ by one unit in the last place);
* whole solve at tol 1e-8 (binary32 refinement to the switch tolerance, then the
  FP64 method from its iterate): the true FP64 residual must be <= 1.5e-8 relative and
  the solution must lie within 1e-6 of the oracle's FP64 one; refinement alone
  (switch_tol = 0) stops on the true residual, <= 1e-8.
The 80^3 workload is checked against the oracle in test_gpu_full_size.py.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2111_09294_amd as D  # noqa: E402

DEV = "cuda:0"
SMALL = ["plain6", "edge4", "penny12", "edge10"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def solver(problems):
    cache = {}

    def get(name):
        if name not in cache:
            p = problems(name)
            say(f"[mixed setup] {name} n={p.n} k={p.k}")
            cache[name] = (p, D.Solver.from_problem(p, DEV))
        return cache[name]

    yield get
    for _, s in cache.values():
        s.close()


def _k32(p):
    import scipy.sparse as sp
    v = p.k_val.astype(np.float32).astype(np.float64)
    return sp.csr_matrix((v, p.k_col, p.k_rowptr), shape=(p.n, p.n))


@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_spmv_fp32(solver, name):
    p, s = solver(name)
    K32 = _k32(p)
    rng = np.random.default_rng(11)
    for x in (rng.standard_normal(p.n), p.f):
        y = host(s.spmv_fp32(dev(x)))
        ref = K32 @ x
        scale = abs(K32) @ np.abs(x) + 1e-300
        assert np.all(np.abs(y - ref) <= 1e-13 * scale)
    # the FP64 product is untouched by the FP32 copy
    x = rng.standard_normal(p.n)
    assert np.all(np.abs(host(s.spmv(dev(x))) - p.K_scipy() @ x) <= 1e-13 * (abs(p.K_scipy()) @ np.abs(x)))


@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_bj_apply_fp32(solver, name):
    p, s = solver(name)
    K = p.K_scipy().tocsr()
    r = np.random.default_rng(12).standard_normal(p.n)
    y = host(s.bj_apply_fp32(dev(r)))
    ref = np.empty(p.n)
    bound = np.empty(p.n)
    bp = p.block_ptr
    for b in range(len(bp) - 1):
        a, e = bp[b], bp[b + 1]
        inv32 = np.linalg.inv(K[a:e, a:e].toarray()).astype(np.float32).astype(np.float64)
        ref[a:e] = inv32 @ r[a:e]
        bound[a:e] = np.abs(inv32) @ np.abs(r[a:e])
    assert np.all(np.abs(y - ref) <= 1.2e-7 * bound + 1e-300)


@pytest.mark.parametrize("name", ["edge10", "penny12", "penny40"])
def test_mixed_solve_matches_oracle(solver, name):
    p, s = solver(name)
    o = O.Oracle.from_problem(p)
    ref = o.solve(p.f, tol=1e-8)
    del o
    f = dev(p.f)
    u64, i64 = s.solve(f, tol=1e-8)
    u, info = s.solve(f, tol=1e-8, precision="mixed", record_history=True)
    u = host(u)
    say(f"[mixed] {name}: {info['iterations']} inner it in {info['refinements']} cycles "
        f"(FP64 {i64['iterations']}), true rel res {info['rel_res_true']:.2e}, solve {info['solve_ms']:.2f} ms "
        f"(FP64 {i64['solve_ms']:.2f} ms)")
    assert info["status"] == D.abi.OK and ref["status"] == O.OK
    assert info["rel_res_true"] <= 1.5e-8 and info["rel_res_recursive"] <= 1e-8
    assert np.linalg.norm(u - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    assert info["refinements"] >= 1 and i64["refinements"] == 0 and i64["iterations_fp64"] == i64["iterations"]
    assert 0 <= info["iterations_fp64"] < info["iterations"]
    h = s.history()
    # one entry per refinement cycle (and the start), then the FP64 phase's end
    assert len(h) == info["refinements"] + 2
    assert h[0] == pytest.approx(1.0, rel=1e-12) and h[-1] <= 1.5e-8 and h[-2] <= 1e-6
    assert np.all(np.diff(h) < 0)
    # refinement alone (no FP64 phase) stops on the true residual
    u1, i1 = s.solve(f, tol=1e-8, precision="mixed", switch_tol=0.0)
    assert i1["status"] == D.abi.OK and i1["iterations_fp64"] == 0
    assert i1["rel_res_true"] <= 1e-8 and i1["rel_res_recursive"] == i1["rel_res_true"]


def test_mixed_deterministic_adjoint_and_warm_start(solver):
    p, s = solver("penny12")
    f = dev(p.f)
    u1, i1 = s.solve(f, precision="mixed")
    u2, i2 = s.solve(f, precision="mixed")
    assert torch.equal(u1, u2) and i1["iterations"] == i2["iterations"]
    lam, ia = s.solve_adjoint(f, precision="mixed")
    assert torch.equal(lam, u1) and ia["refinements"] == i1["refinements"]
    # started from a converged FP64 solution: no refinement cycle is needed
    u64, _ = s.solve(f, tol=1e-9)
    u3, i3 = s.solve(f, initial_guess=u64, precision="mixed")
    assert i3["status"] == D.abi.OK and i3["refinements"] == 0 and i3["iterations"] == 0
    assert torch.equal(u3, u64)


def test_mixed_timing_counts_binary32_spmv_only(solver):
    """In a mixed solve the SpMV timing samples the binary32 inner iterations only: with
    every launch timed, one sample per binary32 iteration and none for the FP64 phase."""
    p, s = solver("penny12")
    f = dev(p.f)
    s.set_timing(True, every=1)
    _, info = s.solve(f, precision="mixed")
    t = s.timing()
    s.set_timing(False)
    assert info["status"] == D.abi.OK and info["iterations_fp64"] > 0
    assert t["spmv_launches"] == info["iterations"] - info["iterations_fp64"]
    assert t["spmv_ms"] > 0.0


def test_mixed_caps_and_options(solver):
    p, s = solver("edge10")
    f = dev(p.f)
    # one loose cycle cannot reach 1e-8
    u, info = s.solve(f, precision="mixed", inner_tol=0.5, max_refinements=1)
    assert info["status"] == D.abi.NOT_CONVERGED and info["refinements"] == 1
    assert 1e-8 < info["rel_res_true"] < 1.0
    # an inner iteration cap counts inner K p products over all cycles
    u, info = s.solve(f, precision="mixed", max_iter=5)
    assert info["status"] == D.abi.NOT_CONVERGED and info["iterations"] <= 5
    for bad in (0.0, 1.0, 1.5, -1e-3):
        with pytest.raises(D.DpcgError) as e:
            s.solve(f, precision="mixed", inner_tol=bad)
        assert e.value.code == D.abi.EINVAL
    with pytest.raises(ValueError):
        s.solve(f, precision="fp16")
    # an unknown precision code through the C ABI
    o = D.abi.Options()
    D.abi.lib().dpcg_default_options(C.byref(o))
    o.precision = 7
    info = D.abi.Info()
    out = torch.empty_like(f)
    st = D.abi.lib().dpcg_solve(s.handle, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()), 1e-8, C.byref(o),
                                C.byref(info))
    assert st == D.abi.EINVAL
    for bad in (-1e-3, 1.0, float("nan")):
        with pytest.raises(D.DpcgError) as e:
            s.solve(f, precision="mixed", switch_tol=bad)
        assert e.value.code == D.abi.EINVAL
    # loose inner solves still converge, with more cycles
    u, info = s.solve(f, precision="mixed", inner_tol=0.1)
    assert info["status"] == D.abi.OK and info["refinements"] >= 4 and info["rel_res_true"] <= 1.5e-8

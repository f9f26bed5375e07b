"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances:
* sparse products with the same terms summed in another order: 1e-13 relative to
  sum_j |K_ij x_j| per entry;
* block-Jacobi by explicit inverse vs Cholesky solves: 1e-9 relative (nodal blocks
  have condition numbers up to about 1e6);
* coarse solve by explicit E^{-1} vs Cholesky solve: 1e-6 relative (kappa(E) up to
  about 3e8);
* whole solve at tol 1e-8: solution within 1e-6 relative, iteration counts equal
  below 50 iterations and within 2% above.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2111_09294_amd as D  # noqa: E402
from fixtures.xfem import build_problem  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pair(problems):
    cache = {}

    def get(name):
        if name not in cache:
            p = problems(name)
            say(f"[setup] {name} n={p.n} k={p.k}")
            cache[name] = (p, O.Oracle.from_problem(p), D.Solver.from_problem(p, DEV))
        return cache[name]

    yield get
    for _, _, s in cache.values():
        s.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def iters_close(a, b):
    if max(a, b) < 50:
        return a == b
    return abs(a - b) <= 0.02 * max(a, b)


SMALL = ["plain6", "edge4", "penny12", "edge10"]


# ------------------------------------------------------------------ single steps
@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_spmv(pair, name):
    p, o, s = pair(name)
    rng = np.random.default_rng(1)
    for x in (rng.standard_normal(p.n), p.f):
        y = host(s.spmv(dev(x)))
        ref = o.spmv(x)
        K = p.K_scipy()
        scale = abs(K) @ np.abs(x) + 1e-300
        assert np.all(np.abs(y - ref) <= 1e-13 * scale)


@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_block_jacobi(pair, name):
    p, o, s = pair(name)
    r = np.random.default_rng(2).standard_normal(p.n)
    y = host(s.bj_apply(dev(r)))
    ref = o.bj_apply(r)
    assert np.linalg.norm(y - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_restrict_coarse_prolong(pair, name):
    p, o, s = pair(name)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(p.n), rng.standard_normal(p.n)
    g = host(s.restrict(dev(a), dev(b)))
    gref = o.zt_times(a) - o.zt_times(o.spmv(b))
    scale = np.abs(o.zt_times(a)).max() + np.abs(o.zt_times(o.spmv(b))).max()
    assert np.abs(g - gref).max() <= 1e-12 * scale
    g0 = host(s.restrict(dev(a)))
    assert np.abs(g0 - o.zt_times(a)).max() <= 1e-13 * np.abs(o.zt_times(a)).max()
    d = host(s.coarse_apply(dev(gref)))
    dref = o.coarse_solve(gref)
    assert np.linalg.norm(d - dref) <= 1e-6 * np.linalg.norm(dref)
    out = host(s.prolong(dev(dref), dev(a)))
    assert np.allclose(out, o.x_plus_z_times(a, dref), rtol=1e-13, atol=1e-13 * np.abs(out).max())
    out0 = host(s.prolong(dev(dref)))
    assert np.allclose(out0, o.x_plus_z_times(None, dref), rtol=1e-13, atol=1e-13 * np.abs(out0).max())


@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_adef2_preconditioner(pair, name):
    p, o, s = pair(name)
    r = np.random.default_rng(4).standard_normal(p.n)
    z = host(s.precond(dev(r)))
    zref, _ = o.adef2_apply(r)
    assert np.linalg.norm(z - zref) <= 1e-6 * np.linalg.norm(zref)


def test_operators_at_full_size_80(pair):
    """Every operator of the iteration at the 80^3 configuration (1.66M DoFs, k = 4,528),
    whole output vectors against the oracle with the tolerances of the smaller cases: the
    SpMV, block-Jacobi, the merged restriction, the coarse solve, the prolongation and
    the A-DEF2 preconditioner (the launch shapes of the bench's 80^3 line)."""
    p, o, s = pair("penny80")
    rng = np.random.default_rng(80)
    a, b = rng.standard_normal(p.n), rng.standard_normal(p.n)
    y = host(s.spmv(dev(a)))
    ref = o.spmv(a)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    z = host(s.bj_apply(dev(a)))
    ref = o.bj_apply(a)
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)
    g = host(s.restrict(dev(a), dev(b)))
    za, zkb = o.zt_times(a), o.zt_times(o.spmv(b))
    assert np.abs(g - (za - zkb)).max() <= 1e-12 * (np.abs(za).max() + np.abs(zkb).max())
    d = host(s.coarse_apply(dev(za - zkb)))
    dref = o.coarse_solve(za - zkb)
    assert np.linalg.norm(d - dref) <= 1e-6 * np.linalg.norm(dref)
    out = host(s.prolong(dev(dref), dev(a)))
    assert np.allclose(out, o.x_plus_z_times(a, dref), rtol=1e-13, atol=1e-13 * np.abs(out).max())
    zz = host(s.precond(dev(a)))
    zref, _ = o.adef2_apply(a)
    assert np.linalg.norm(zz - zref) <= 1e-6 * np.linalg.norm(zref)
    say(f"[full size] penny80 n={p.n} k={p.k}: operators match the oracle")


# ------------------------------------------------------------------ whole solves
@pytest.mark.parametrize("name", SMALL + ["penny40"])
def test_solve_matches_oracle(pair, name):
    p, o, s = pair(name)
    say(f"[solve] {name}")
    ref = o.solve(p.f, tol=1e-8, history=True)
    u, info = s.solve(dev(p.f), tol=1e-8, record_history=True)
    u = host(u)
    say(f"[solve] {name}: gpu {info['iterations']} it, oracle {ref['iterations']} it, "
        f"setup {info['setup_ms']:.1f} ms solve {info['solve_ms']:.2f} ms")
    assert ref["status"] == O.OK and info["status"] == D.abi.OK
    assert iters_close(info["iterations"], ref["iterations"])
    assert np.linalg.norm(u - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    assert info["rel_res_recursive"] <= 1e-8 and info["rel_res_true"] <= 1.5e-8
    h = s.history()
    assert len(h) == info["iterations"] + 1
    m = min(len(h), len(ref["history"]))
    assert np.allclose(h[:m], ref["history"][:m], rtol=1e-6, atol=1e-12)


def test_block_columns_beyond_16_bits(pair):
    """The iteration SpMV reads its block columns as 16-bit offsets from their row when
    every offset fits (node-major numbering) and the 4-byte columns otherwise.  The 40^3
    system with its nodal blocks in a random order (70,857 block rows, so offsets far
    beyond 16 bits) takes the 4-byte path; both solve to the oracle's solution with its
    iteration count."""
    from fixtures import permuted
    p, o, s = pair("penny40")
    assert s.stats()["spmv_col_bytes"] == 2
    bp = np.asarray(p.block_ptr, np.int64)
    order = np.random.default_rng(5).permutation(len(bp) - 1)
    lens = np.diff(bp)[order]
    starts = bp[:-1][order]
    offs = np.zeros(len(order) + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    perm = np.repeat(starts - offs[:-1], lens) + np.arange(offs[-1])
    q = permuted(p, perm, offs.astype(np.int32), name="penny40-shuffled")
    ref = o.solve(p.f, tol=1e-8)
    with D.Solver.from_problem(q, DEV) as sq:
        assert sq.stats()["spmv_col_bytes"] == 4
        u, info = sq.solve(dev(q.f), tol=1e-8)
    u0, info0 = s.solve(dev(p.f), tol=1e-8)
    for uu, inf, pp in ((host(u), info, perm), (host(u0), info0, np.arange(p.n))):
        assert inf["status"] == D.abi.OK
        assert np.linalg.norm(uu - ref["u"][pp]) <= 1e-6 * np.linalg.norm(ref["u"])
        assert iters_close(inf["iterations"], ref["iterations"])
    say(f"[columns] penny40 shuffled: {info['iterations']} iterations (node-major {info0['iterations']}, "
        f"oracle {ref['iterations']})")


@pytest.mark.parametrize("name", ["penny12", "penny40"])
def test_deterministic_and_adjoint(pair, name):
    """Two solves are bitwise identical; the adjoint solve runs the same operator."""
    p, o, s = pair(name)
    f = dev(p.f)
    u1, i1 = s.solve(f)
    u2, i2 = s.solve(f)
    assert torch.equal(u1, u2) and i1["iterations"] == i2["iterations"]
    lam, ia = s.solve_adjoint(f)
    assert torch.equal(lam, u1) and ia["iterations"] == i1["iterations"]
    # a forward solve is undisturbed by an adjoint solve in between
    g = dev(np.random.default_rng(9).standard_normal(p.n))
    s.solve_adjoint(g)
    u3, _ = s.solve(f)
    assert torch.equal(u3, u1)


@pytest.mark.parametrize("name", ["edge10", "penny40"])
def test_setup_deterministic(pair, name):
    """Two independent setups of the same system give bitwise-identical solves."""
    p, o, s = pair(name)
    f = dev(p.f)
    u1, i1 = s.solve(f)
    with D.Solver.from_problem(p, DEV) as s2:
        u2, i2 = s2.solve(f)
        # the handle's memory differs once it has run an adjoint solve (its workspace is
        # made on first use); the structure does not
        drop = lambda d: {k: v for k, v in d.items() if k != "device_bytes"}  # noqa: E731
        assert drop(s2.stats()) == drop(s.stats())
        s2.solve_adjoint(f)
        assert s2.stats()["device_bytes"] > drop(s2.stats())["nnzb"]
    assert torch.equal(u1, u2) and i1["iterations"] == i2["iterations"]


def test_random_rhs_and_warm_start(pair):
    p, o, s = pair("penny12")
    rng = np.random.default_rng(5)
    f = rng.standard_normal(p.n)
    ref = o.solve(f, tol=1e-8)
    u, info = s.solve(dev(f), tol=1e-8)
    assert iters_close(info["iterations"], ref["iterations"])
    assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    # warm start from a random u_{-1}
    u_m1 = rng.standard_normal(p.n)
    ref = o.solve(f, tol=1e-8, u0=u_m1)
    u, info = s.solve(dev(f), tol=1e-8, initial_guess=dev(u_m1))
    assert iters_close(info["iterations"], ref["iterations"])
    assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    # warm start from the solution: 0 iterations
    tight, _ = s.solve(dev(f), tol=1e-12)
    u, info = s.solve(dev(f), tol=1e-8, initial_guess=tight)
    assert info["iterations"] == 0 and info["status"] == D.abi.OK


def test_iteration_cap_and_special_rhs(pair):
    p, o, s = pair("edge10")
    for cap in (0, 1, 7):
        ref = o.solve(p.f, tol=1e-8, max_iter=cap)
        u, info = s.solve(dev(p.f), tol=1e-8, max_iter=cap, check_every=3)
        assert ref["status"] == O.NOT_CONVERGED and info["status"] == D.abi.NOT_CONVERGED
        assert info["iterations"] == ref["iterations"] == cap
        assert np.linalg.norm(host(u) - ref["u"]) <= 1e-9 * np.linalg.norm(ref["u"])
    u, info = s.solve(torch.zeros(p.n, dtype=torch.float64, device=DEV))
    assert info["status"] == D.abi.OK and info["iterations"] == 0 and not torch.any(u)
    f = p.f.copy()
    f[5] = np.inf
    with pytest.raises(D.DpcgError) as e:
        s.solve(dev(f))
    assert e.value.code == D.abi.ENONFINITE
    with pytest.raises(D.DpcgError) as e:
        s.solve(dev(p.f), tol=0.0)
    assert e.value.code == D.abi.EINVAL
    # f in K range(Z): the start already solves it
    c = np.random.default_rng(1).standard_normal(p.k)
    us = p.Z_scipy() @ c
    u, info = s.solve(dev(p.K_scipy() @ us))
    assert info["iterations"] <= 1
    assert np.linalg.norm(host(u) - us) <= 1e-7 * np.linalg.norm(us)


def test_check_every_does_not_change_result(pair):
    p, o, s = pair("penny12")
    f = dev(p.f)
    a, ia = s.solve(f, check_every=1)
    b, ib = s.solve(f, check_every=64)
    assert torch.equal(a, b) and ia["iterations"] == ib["iterations"]


# ------------------------------------------------------------------ special operators
def _solver_from_dense(K, Z, bp):
    import scipy.sparse as sp
    A = sp.csr_matrix(K)
    A.sort_indices()
    n = A.shape[0]
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)  # noqa: E731
    if Z is None:
        return D.Solver(n, t(A.indptr, torch.int64), t(A.indices, torch.int32), t(A.data, torch.float64), 0,
                        None, None, None, t(bp, torch.int32))
    Zs = sp.csr_matrix(Z)
    Zs.sort_indices()
    return D.Solver(n, t(A.indptr, torch.int64), t(A.indices, torch.int32), t(A.data, torch.float64),
                    Zs.shape[1], t(Zs.indptr, torch.int64), t(Zs.indices, torch.int32),
                    t(Zs.data, torch.float64), t(bp, torch.int32))


def _with_entry(K, i, j, v):
    """CSR copy of K with the structurally absent entry (i, j) stored explicitly as v."""
    import scipy.sparse as sp
    A = K.tocoo()
    B = sp.csr_matrix((np.append(A.data, v), (np.append(A.row, i), np.append(A.col, j))), shape=K.shape)
    B.sort_indices()
    assert B.nnz == K.nnz + 1
    return B


def test_setup_structural_asymmetry(problems):
    """A stored entry whose mirror block is absent: nonzero values are rejected from
    either side of the diagonal; an explicit zero is symmetric in value and solves as K."""
    p = problems("edge4")
    K = p.K_scipy().tocsr()
    Z = p.Z_scipy().toarray()
    bp = p.block_ptr
    i, j = p.n - 3, 0
    assert K[i, j] == 0 and K[j, i] == 0 and K[i].indices.min() > 2
    for a, b in ((i, j), (j, i)):
        with pytest.raises(D.DpcgError) as e:
            _solver_from_dense(_with_entry(K, a, b, 1.0), Z, bp)
        assert e.value.code == D.abi.ENOTSYM
    f = dev(p.f)
    s0 = _solver_from_dense(K, Z, bp)
    s1 = _solver_from_dense(_with_entry(K, i, j, 0.0), Z, bp)
    u0, i0 = s0.solve(f)
    u1, i1 = s1.solve(f)
    assert s1.stats()["nnzb"] == s0.stats()["nnzb"] + 1
    assert i0["iterations"] == i1["iterations"]
    # only the summation order of the extra zero block differs
    assert np.abs(host(u1) - host(u0)).max() <= 1e-9 * np.abs(host(u0)).max()
    s0.close()
    s1.close()


def test_no_deflation_and_point_jacobi(problems):
    p = problems("plain6")
    K = p.K_scipy()
    for bp in (np.arange(p.n + 1), p.block_ptr):
        o = O.Oracle(p.n, p.k_rowptr, p.k_col, p.k_val, 0, np.zeros(p.n + 1, np.int64), np.zeros(0, np.int32),
                     np.zeros(0), bp)
        ref = o.solve(p.f)
        with _solver_from_dense(K, None, bp) as s:
            u, info = s.solve(dev(p.f))
        assert iters_close(info["iterations"], ref["iterations"])
        assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])


def test_one_block_is_direct():
    p = build_problem("cube1", 1, 1, crack=None)
    K = p.K_scipy().toarray()
    with _solver_from_dense(K, p.Z_scipy(), np.array([0, p.n])) as s:
        u, info = s.solve(dev(p.f), tol=1e-12)
    assert info["iterations"] == 1
    assert np.allclose(host(u), np.linalg.solve(K, p.f), rtol=1e-12)


def test_single_triplet_system():
    K = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    f = np.array([1.0, -2.0, 0.5])
    with _solver_from_dense(K, None, np.array([0, 1, 2, 3])) as s:
        u, info = s.solve(dev(f), tol=1e-14)
    assert info["status"] == D.abi.OK
    assert np.allclose(host(u), np.linalg.solve(K, f), rtol=1e-12)


def test_indefinite_system_breaks_down_like_the_oracle():
    """Symmetric K with SPD nodal blocks but indefinite, f chosen so that p_0^T K p_0 < 0
    (the system of the oracle's own breakdown test): the single solve and the
    several-systems path both stop at iteration 0 with the breakdown status."""
    from test_oracle import indefinite_breakdown_system
    K, f, bp = indefinite_breakdown_system()
    import scipy.sparse as sp
    Ks = sp.csr_matrix(K)
    Ks.sort_indices()
    ref = O.Oracle(6, Ks.indptr.astype(np.int64), Ks.indices.astype(np.int32), Ks.data, 0,
                   np.zeros(7, np.int64), np.zeros(0, np.int32), np.zeros(0), bp).solve(f)
    with _solver_from_dense(K, None, bp) as s:
        u, info = s.solve(dev(f), raise_on_error=False)
        assert info["status"] == D.abi.EBREAKDOWN == ref["status"]
        assert info["bad_index"] == ref["bad"] and info["iterations"] == ref["iterations"]
        with pytest.raises(D.DpcgError) as e:
            s.solve(dev(f))
        assert e.value.code == D.abi.EBREAKDOWN
        _, infos = D.solve_many([s], [dev(f)], raise_on_error=False)
        assert infos[0]["status"] == D.abi.EBREAKDOWN and infos[0]["bad_index"] == ref["bad"]


# ------------------------------------------------------------------ setup errors
def test_setup_errors(problems):
    p = problems("edge4")
    K = p.K_scipy().tolil()
    Z = p.Z_scipy().toarray()
    bp = p.block_ptr
    with pytest.raises(D.DpcgError) as e:
        _solver_from_dense(K.tocsr(), np.concatenate([Z, Z[:, :1]], 1), bp)
    assert e.value.code == D.abi.ECOARSE_NOT_SPD
    K2 = K.copy()
    s0 = bp[3]
    K2[s0, s0] = -1.0
    with pytest.raises(D.DpcgError) as e:
        _solver_from_dense(K2.tocsr(), Z, bp)
    assert e.value.code == D.abi.EBLOCK_NOT_SPD and e.value.info.bad_index == 3
    K3 = K.copy()
    K3[0, 5] = K3[0, 5] + 1.0
    with pytest.raises(D.DpcgError) as e:
        _solver_from_dense(K3.tocsr(), Z, bp)
    assert e.value.code == D.abi.ENOTSYM
    bad_bp = np.array([0, 3, 3] + list(range(6, p.n + 1, 3)))   # an empty block
    with pytest.raises(D.DpcgError) as e:
        _solver_from_dense(K.tocsr(), Z, bad_bp)
    assert e.value.code == D.abi.EINVAL
    with pytest.raises(D.DpcgError) as e:
        _solver_from_dense(K.tocsr()[:-1, :-1], Z[:-1], np.arange(p.n))
    assert e.value.code == D.abi.EINVAL


def test_setup_rejects_malformed_csr(problems):
    """Malformed K or Z arrays (with a truthful entry count) are refused before use."""
    p = problems("edge4")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)  # noqa: E731

    def setup(kp, kc, kv, zc=p.z_col):
        return D.Solver(p.n, t(kp, torch.int64), t(kc, torch.int32), t(kv, torch.float64), p.k,
                        t(p.z_rowptr, torch.int64), t(zc, torch.int32), t(p.z_val, torch.float64),
                        t(p.block_ptr, torch.int32))

    r = 7
    a, b = int(p.k_rowptr[r]), int(p.k_rowptr[r + 1])
    cases = {}
    kc = p.k_col.copy()
    kc[a], kc[a + 1] = kc[a + 1], kc[a]
    cases["unsorted columns"] = (p.k_rowptr, kc, p.k_val)
    kc = p.k_col.copy()
    kc[a + 1] = kc[a]
    cases["repeated column"] = (p.k_rowptr, kc, p.k_val)
    kc = p.k_col.copy()
    kc[b - 1] = p.n
    cases["column out of range"] = (p.k_rowptr, kc, p.k_val)
    kv = p.k_val.copy()
    kv[a + 2] = np.nan
    cases["NaN value"] = (p.k_rowptr, p.k_col, kv)
    kp = p.k_rowptr.copy()
    kp[r + 1] = kp[r + 2] + 1
    cases["row pointer decreasing"] = (kp, p.k_col, p.k_val)
    kp = p.k_rowptr.copy()
    kp[r + 1] = kp[-1] + 50
    cases["row pointer past the end"] = (kp, p.k_col, p.k_val)
    for what, (kp, kc, kv) in cases.items():
        with pytest.raises(D.DpcgError) as e:
            setup(kp, kc, kv)
        assert e.value.code == D.abi.EINVAL, what
    zc = p.z_col.copy()
    zc[3] = p.k
    with pytest.raises(D.DpcgError) as e:
        setup(p.k_rowptr, p.k_col, p.k_val, zc)
    assert e.value.code == D.abi.EINVAL
    with setup(p.k_rowptr, p.k_col, p.k_val) as s:   # the well-formed arrays still work
        u, info = s.solve(dev(p.f))
        assert info["status"] == D.abi.OK


def test_spmv_timing_samples(pair):
    """dpcg_set_timing(m): the SpMV launches of working iterations 0, m, 2m, ... are
    timed; m = 0 turns timing off, m < 0 is refused."""
    p, o, s = pair("edge10")
    f = dev(p.f)
    for every in (1, 8):
        s.set_timing(True, every=every)
        _, info = s.solve(f)
        t = s.timing()
        it = info["iterations"]
        assert t["spmv_launches"] == (it + every - 1) // every
        assert t["spmv_ms"] > 0.0
    s.set_timing(False)
    _, info = s.solve(f)
    assert s.timing()["spmv_launches"] == (info["iterations"] + 7) // 8   # counters kept while off
    with pytest.raises(D.DpcgError) as e:
        s.set_timing(True, every=-1)
    assert e.value.code == D.abi.EINVAL

"""GPU parity of subdomain-sized block-Jacobi blocks (Sec. 3.4: one block per subdomain,
its standard and enriched DoFs numbered consecutively).  Blocks of more than 18 DoFs
keep explicit FP64 inverses made at setup by batched Gauss-Jordan sweeps and are
applied each iteration by a dense matrix-vector kernel; smaller blocks keep the fused
nodal path, and a partition may mix both.

Tolerances:
* M^-1 r per block against LAPACK's Cholesky solve of K_BB: ||dy|| <= m eps cond(K_BB)
  ||y|| (two backward-stable inversions of one SPD matrix, first-order bound);
* solves at tol 1e-8 against the oracle with the same partition: iteration counts
  within 2% (plus one), solutions within 1e-6 relative;
* value updates: bitwise equal to a fresh setup on the new values (same kernels, same
  inputs).
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import scipy.linalg as sla  # noqa: E402
import scipy.sparse as sp  # noqa: E402

import paper_2111_09294_amd as D  # noqa: E402
from fixtures import CONFIGS, load_elements, permuted, problem_with_moduli, with_subdomain_blocks  # noqa: E402

DEV = "cuda:0"
EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def sd():
    cache = {}

    def get(name, nsd):
        if (name, nsd) not in cache:
            cache[(name, nsd)] = with_subdomain_blocks(name, nsd)
        return cache[(name, nsd)]

    return get


def _with_blocks(q, bp):
    return permuted(q, np.arange(q.n), bp, name=q.name + "-mixed")


@pytest.mark.parametrize("name,nsd", [("plain6", 1), ("edge4", 1), ("edge10", 2), ("penny12", 3)])
def test_dense_block_apply(sd, name, nsd):
    q, _ = sd(name, nsd)
    say(f"[dense] apply {name} sd{nsd}: blocks {np.diff(q.block_ptr).tolist()[:8]}")
    K = q.K_scipy().tocsr()
    r = np.random.default_rng(41).standard_normal(q.n)
    with D.Solver.from_problem(q, DEV) as s:
        st = s.stats()
        assert st["dense_blocks"] == int((np.diff(q.block_ptr) > 18).sum())
        y = host(s.bj_apply(dev(r)))
        y32 = host(s.bj_apply_fp32(dev(r)))
    bp = q.block_ptr
    worst = 0.0
    for b in range(len(bp) - 1):
        s0, e0 = bp[b], bp[b + 1]
        KB = K[s0:e0, s0:e0].toarray()
        ref = sla.cho_solve(sla.cho_factor(KB, lower=True), r[s0:e0])
        cond = np.linalg.cond(KB)
        err = np.linalg.norm(y[s0:e0] - ref) / np.linalg.norm(ref)
        worst = max(worst, err / (cond * EPS))
        assert err <= (e0 - s0) * EPS * cond
        # binary32 inverse applied in FP64: the rounding of the inverse's entries
        Minv = np.linalg.inv(KB)
        bound = 2 ** -24 * np.abs(Minv) @ np.abs(r[s0:e0])
        assert np.all(np.abs(y32[s0:e0] - Minv @ r[s0:e0]) <= 1.01 * bound + (e0 - s0) * EPS * cond * np.abs(ref).max())
    say(f"[dense] worst error / (eps cond) = {worst:.2f}")


@pytest.mark.parametrize("name,nsd", [("edge10", 2), ("edge10", 3), ("penny12", 2), ("penny12", 3)])
def test_dense_solve_matches_oracle(sd, name, nsd):
    q, _ = sd(name, nsd)
    ref = O.Oracle.from_problem(q).solve(q.f, tol=1e-8)
    with D.Solver.from_problem(q, DEV) as s:
        u, info = s.solve(dev(q.f), tol=1e-8)
    say(f"[dense] {name} sd{nsd}: {info['iterations']} iterations (oracle {ref['iterations']}), "
        f"solve {info['solve_ms']:.2f} ms, setup {s.setup_info['setup_ms']:.2f} ms")
    assert info["status"] == D.abi.OK and ref["status"] == O.OK
    assert abs(info["iterations"] - ref["iterations"]) <= 0.02 * ref["iterations"] + 1
    assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    assert info["rel_res_true"] <= 1.5e-8


@pytest.mark.parametrize("name", ["plain6", "edge4"])
def test_one_subdomain_block_one_iteration(sd, name):
    q, _ = sd(name, 1)
    u_star = np.linalg.solve(q.K_scipy().toarray(), q.f)
    with D.Solver.from_problem(q, DEV) as s:
        u, info = s.solve(dev(q.f), tol=1e-10)
    assert info["status"] == D.abi.OK and info["iterations"] == 1
    assert np.linalg.norm(host(u) - u_star) <= 1e-9 * np.linalg.norm(u_star)


def test_mixed_small_and_dense_blocks(sd, problems):
    """Subdomains 1, 3, 5 and 6 split into their nodal blocks, the others whole."""
    q, perm = sd("edge10", 2)
    p = problems("edge10")
    inv = np.empty(p.n, np.int64)
    inv[perm] = np.arange(p.n)
    node_starts = np.sort(inv[p.block_ptr[:-1]])
    cuts = set(q.block_ptr.tolist())
    for b in (1, 3, 5, 6):
        s0, e0 = q.block_ptr[b], q.block_ptr[b + 1]
        cuts.update(node_starts[(node_starts >= s0) & (node_starts < e0)].tolist())
    bp = np.array(sorted(cuts), np.int32)
    m = _with_blocks(q, bp)
    sizes = np.diff(bp)
    assert (sizes > 18).sum() == 4 and (sizes <= 18).sum() > 100
    ref = O.Oracle.from_problem(m).solve(m.f, tol=1e-8)
    with D.Solver.from_problem(m, DEV) as s:
        u, info = s.solve(dev(m.f), tol=1e-8)
        r = np.random.default_rng(42).standard_normal(m.n)
        y = host(s.bj_apply(dev(r)))
    say(f"[dense] mixed partition: {info['iterations']} iterations (oracle {ref['iterations']})")
    assert abs(info["iterations"] - ref["iterations"]) <= 0.02 * ref["iterations"] + 1
    assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    yo = O.Oracle.from_problem(m).bj_apply(r)
    assert np.linalg.norm(y - yo) <= 1e-8 * np.linalg.norm(yo)


def test_dense_block_errors(sd):
    q, _ = sd("edge10", 2)
    # a block that is not SPD: a negative diagonal entry inside block 5 (K stays symmetric)
    K = q.K_scipy().tolil()
    d = int(q.block_ptr[5]) + 7
    K[d, d] = -1.0
    K = K.tocsr()
    K.sort_indices()
    t = lambda a, dt: dev(a, dt)  # noqa: E731
    with pytest.raises(D.DpcgError) as e:
        D.Solver(q.n, t(K.indptr, torch.int64), t(K.indices, torch.int32), t(K.data, torch.float64), q.k,
                 t(q.z_rowptr, torch.int64), t(q.z_col, torch.int32), t(q.z_val, torch.float64),
                 t(q.block_ptr, torch.int32))
    assert e.value.code == D.abi.EBLOCK_NOT_SPD and e.value.info.bad_index == 5
    # a block above 8192 DoFs
    n = 8196
    A = sp.identity(n, format="csr") * 2.0
    A.sort_indices()
    with pytest.raises(D.DpcgError) as e:
        D.Solver(n, t(A.indptr, torch.int64), t(A.indices, torch.int32), t(A.data, torch.float64), 0, None, None,
                 None, t(np.array([0, 3, n], np.int32), torch.int32))
    assert e.value.code == D.abi.EINVAL and e.value.info.bad_index == 1
    # the largest allowed block: a diagonal matrix, one block of 8192 DoFs and one of 4
    with D.Solver(n, t(A.indptr, torch.int64), t(A.indices, torch.int32), t(A.data, torch.float64), 0, None, None,
                  None, t(np.array([0, 8192, n], np.int32), torch.int32)) as s:
        f = np.random.default_rng(43).standard_normal(n)
        u, info = s.solve(dev(f))
        assert info["iterations"] == 1 and np.allclose(host(u), f / 2.0, rtol=1e-14, atol=0)
    # the multi-RHS and several-systems paths take small blocks only
    with D.Solver.from_problem(q, DEV) as s:
        F = dev(np.stack([q.f, 2 * q.f], 1))
        with pytest.raises(D.DpcgError) as e:
            s.solve_batch(F)
        assert e.value.code == D.abi.EINVAL
        with pytest.raises(D.DpcgError) as e:
            D.solve_many([s], [dev(q.f)])
        assert e.value.code == D.abi.EINVAL
        u, info = s.solve(dev(q.f))      # still usable
        assert info["status"] == D.abi.OK


def test_dense_update_values_and_mixed(sd):
    """Moduli of the elements of enriched nodes doubled: updating the listed blocks gives
    a fresh setup's iterates; the mixed-precision copies follow."""
    name = "edge10"
    q0, perm = sd(name, 2)
    ep, ed, ko, km = load_elements(name)
    nel = CONFIGS[name]["ne"] ** 3
    enr = np.nonzero(np.diff(ep) > 24)[0]
    E = np.ones(nel)
    E[enr] = 2.0
    q1 = permuted(problem_with_moduli(name, E), perm, q0.block_ptr)
    assert np.array_equal(q1.k_col, q0.k_col)
    inv = np.empty(q0.n, np.int64)
    inv[perm] = np.arange(q0.n)
    dofs = np.unique(np.concatenate([ed[ep[e]:ep[e + 1]] for e in enr]))
    dofs = inv[dofs[dofs >= 0]]
    blocks = np.unique(np.searchsorted(q0.block_ptr, dofs, side="right") - 1).astype(np.int32)
    kt = lambda q: (dev(q.k_rowptr, torch.int64), dev(q.k_col, torch.int32), dev(q.k_val))  # noqa: E731
    f = dev(q1.f)
    with D.Solver.from_problem(q1, DEV) as fresh:
        u_ref, i_ref = fresh.solve(f)
        um_ref, im_ref = fresh.solve(f, precision="mixed")
    with D.Solver.from_problem(q0, DEV) as s:
        s.solve(dev(q0.f), precision="mixed")          # FP32 copies exist before the update
        info = s.update_values(*kt(q1), changed_blocks=blocks)
        u1, i1 = s.solve(f)
        say(f"[dense] update: {len(blocks)} of {q0.nblocks} blocks, {info['setup_ms']:.2f} ms; "
            f"{i1['iterations']} iterations (fresh {i_ref['iterations']})")
        assert i1["iterations"] == i_ref["iterations"] and torch.equal(u1, u_ref)
        um, im = s.solve(f, precision="mixed")
        assert im["iterations"] == im_ref["iterations"] and torch.equal(um, um_ref)
        assert im["status"] == D.abi.OK and torch.linalg.norm(um - u_ref) <= 1e-6 * torch.linalg.norm(u_ref)
        # a list without the first changed block: a stale inverse, still SPD
        s.update_values(*kt(q0))
        s.update_values(*kt(q1), changed_blocks=blocks[1:])
        u2, i2 = s.solve(f)
        assert i2["status"] == D.abi.OK and torch.linalg.norm(u2 - u_ref) <= 1e-6 * torch.linalg.norm(u_ref)


def test_subdomain_blocks_penny40():
    """The 40^3 workload with 8^3 subdomain blocks (375..849 DoFs) against the oracle,
    and with 4^3 blocks (3,000..4,236 DoFs, 5.8 GB of inverses) by its true residual."""
    name = "penny40"
    say("[dense] penny40: permuting the system")
    q8, _ = with_subdomain_blocks(name, 8)
    ref = O.Oracle.from_problem(q8).solve(q8.f, tol=1e-8)
    with D.Solver.from_problem(q8, DEV) as s:
        u, info = s.solve(dev(q8.f), tol=1e-8)
        setup8 = s.setup_info["setup_ms"]
    say(f"[dense] penny40 sd8: {info['iterations']} iterations (oracle {ref['iterations']}), setup {setup8:.1f} ms, "
        f"solve {info['solve_ms']:.1f} ms")
    assert abs(info["iterations"] - ref["iterations"]) <= 0.02 * ref["iterations"] + 1
    assert np.linalg.norm(host(u) - ref["u"]) <= 1e-6 * np.linalg.norm(ref["u"])
    del ref
    q4, _ = with_subdomain_blocks(name, 4)
    with D.Solver.from_problem(q4, DEV) as s:
        u, info = s.solve(dev(q4.f), tol=1e-8)
        setup4 = s.setup_info["setup_ms"]
    r = q4.f - q4.K_scipy() @ host(u)
    rel = np.linalg.norm(r) / np.linalg.norm(q4.f)
    say(f"[dense] penny40 sd4: {info['iterations']} iterations, setup {setup4:.1f} ms, solve {info['solve_ms']:.1f} ms, "
        f"true residual {rel:.2e}")
    assert info["status"] == D.abi.OK and rel <= 1.5e-8

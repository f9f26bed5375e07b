"""Pins of the oracle with subdomain-sized block-Jacobi blocks (Sec. 3.4: one block per
subdomain, its standard and enriched DoFs together, numbered consecutively).

Checks against LAPACK block solves, the Sec. 3.2 operator formula with a dense
block-diagonal M^-1, the one-subdomain limit (M = K: one iteration) and the trend that
whole-subdomain blocks precondition better than nodal blocks.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from fixtures import with_subdomain_blocks


@pytest.fixture(scope="module")
def sd():
    cache = {}

    def get(name, nsd):
        if (name, nsd) not in cache:
            cache[(name, nsd)] = with_subdomain_blocks(name, nsd)
        return cache[(name, nsd)]

    return get


@pytest.mark.parametrize("name,nsd", [("edge10", 2), ("penny12", 2), ("penny12", 3)])
def test_block_apply_is_blockwise_lapack_solve(sd, name, nsd):
    q, _ = sd(name, nsd)
    assert np.diff(q.block_ptr).max() > 18
    K = q.K_scipy().tocsr()
    r = np.random.default_rng(21).standard_normal(q.n)
    y = O.Oracle.from_problem(q).bj_apply(r)
    bp = q.block_ptr
    for b in range(len(bp) - 1):
        s, e = bp[b], bp[b + 1]
        KB = K[s:e, s:e].toarray()
        ref = sla.cho_solve(sla.cho_factor(KB, lower=True), r[s:e])
        cond = np.linalg.cond(KB)
        assert np.linalg.norm(y[s:e] - ref) <= 1e-15 * (e - s) * cond * np.linalg.norm(ref)


def test_adef2_apply_with_subdomain_blocks_is_the_operator(sd):
    """M_A-DEF2 = P^T M^-1 + Q with M^-1 = blockdiag(K_BB^-1) over subdomain blocks."""
    q, _ = sd("edge10", 2)
    K = q.K_scipy().toarray()
    Z = q.Z_scipy().toarray()
    Q = Z @ np.linalg.solve(Z.T @ K @ Z, Z.T)
    P = np.eye(q.n) - K @ Q
    Minv = np.zeros_like(K)
    bp = q.block_ptr
    for b in range(len(bp) - 1):
        s, e = bp[b], bp[b + 1]
        Minv[s:e, s:e] = np.linalg.inv(K[s:e, s:e])
    o = O.Oracle.from_problem(q)
    r = np.random.default_rng(22).standard_normal(q.n)
    z, y = o.adef2_apply(r)
    ref = P.T @ (Minv @ r) + Q @ r
    assert np.linalg.norm(z - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.linalg.norm(y - Minv @ r) <= 1e-9 * np.linalg.norm(y)


@pytest.mark.parametrize("name", ["plain6", "edge4"])
def test_one_subdomain_block_converges_in_one_iteration(sd, name):
    """One subdomain: the block is K itself, M^-1 K = I and CG stops after one step."""
    q, _ = sd(name, 1)
    assert q.nblocks == 1
    K = q.K_scipy().toarray()
    u_star = np.linalg.solve(K, q.f)
    r = O.Oracle.from_problem(q).solve(q.f, tol=1e-10)
    assert r["status"] == O.OK and r["iterations"] == 1
    assert np.linalg.norm(r["u"] - u_star) <= 1e-9 * np.linalg.norm(u_star)


@pytest.mark.parametrize("name,nsd", [("edge10", 2), ("penny12", 2), ("penny12", 3)])
def test_subdomain_blocks_need_fewer_iterations(sd, problems, name, nsd):
    """Blocks of whole subdomains sit closer to K than nodal blocks: fewer iterations,
    same solution (the permuted system is the same system)."""
    p = problems(name)
    q, perm = sd(name, nsd)
    rn = O.Oracle.from_problem(p).solve(p.f, tol=1e-10)
    rs = O.Oracle.from_problem(q).solve(q.f, tol=1e-10)
    assert rn["status"] == O.OK and rs["status"] == O.OK
    assert rs["iterations"] < rn["iterations"]
    u = np.empty(p.n)
    u[perm] = rs["u"]
    assert np.linalg.norm(u - rn["u"]) <= 1e-6 * np.linalg.norm(rn["u"])

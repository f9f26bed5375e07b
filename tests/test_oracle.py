"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a LAPACK dense
solve, the operator definitions of Sec. 3.2 (P, Q, M_A-DEF2 = P^T M^{-1} + Q and
u_0 = Q f + P^T u_{-1}), invariants (Z^T r_0 = 0), special cases that collapse to a
library routine (point-Jacobi CG = scipy's cg) or to a closed form (finite
termination, one-step convergence).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from fixtures.xfem import Problem, build_problem


def _csr_arrays(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def _make(K, Z, block_ptr):
    kp, kc, kv = _csr_arrays(K)
    n = K.shape[0]
    if Z is None or Z.shape[1] == 0:
        zp, zc, zv, k = np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), 0
    else:
        zp, zc, zv = _csr_arrays(Z)
        k = Z.shape[1]
    return O.Oracle(n, kp, kc, kv, k, zp, zc, zv, np.asarray(block_ptr, np.int32))


def _dense_operators(p):
    K = p.K_scipy().toarray()
    Z = p.Z_scipy().toarray()
    E = Z.T @ K @ Z
    Q = Z @ np.linalg.solve(E, Z.T)
    P = np.eye(p.n) - K @ Q
    Minv = np.zeros_like(K)
    bp = p.block_ptr
    for b in range(len(bp) - 1):
        s, e = bp[b], bp[b + 1]
        Minv[s:e, s:e] = np.linalg.inv(K[s:e, s:e])
    return K, Z, Q, P, Minv


# ------------------------------------------------------------------ whole solve
@pytest.mark.parametrize("name", ["plain6", "edge4", "penny12", "edge10"])
def test_solution_matches_dense_lapack(problems, name):
    """u within kappa(K) * tol of the LAPACK solution at tol 1e-8; within 1e-9 at 1e-13."""
    p = problems(name)
    K = p.K_scipy().toarray()
    u_star = np.linalg.solve(K, p.f)
    ev = np.linalg.eigvalsh(K) if p.n <= 8000 else None
    kappa = ev[-1] / ev[0]
    o = O.Oracle.from_problem(p)
    r = o.solve(p.f, tol=1e-8)
    assert r["status"] == O.OK
    assert r["rel_res"] <= 1e-8
    err = np.linalg.norm(r["u"] - u_star) / np.linalg.norm(u_star)
    assert err <= kappa * 1e-8
    tight = o.solve(p.f, tol=1e-13)
    assert tight["status"] == O.OK
    assert np.linalg.norm(tight["u"] - u_star) / np.linalg.norm(u_star) <= 1e-9
    # the recursively updated residual tracks the true one
    assert abs(r["rel_res_true"] - r["rel_res"]) <= 1e-10


# ------------------------------------------------------------------ Sec. 3.2 operators
@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("name", ["edge4", "penny12"])
def test_adef2_apply_is_the_operator(problems, name, fast):
    """Algorithm 3 applies M_A-DEF2 = P^T M^{-1} + Q with P = I - K Q, Q = Z E^{-1} Z^T
    (the literal mode and the fast mode's merged coarse solve alike)."""
    p = problems(name)
    K, Z, Q, P, Minv = _dense_operators(p)
    o = O.Oracle.from_problem(p)
    rng = np.random.default_rng(11)
    for _ in range(3):
        r = rng.standard_normal(p.n)
        z, y = o.adef2_apply(r, fast=fast)
        ref = P.T @ (Minv @ r) + Q @ r
        assert np.linalg.norm(z - ref) <= 1e-8 * np.linalg.norm(ref)
        assert np.linalg.norm(y - Minv @ r) <= 1e-12 * np.linalg.norm(y)


@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("name", ["edge4", "penny12"])
def test_adef2_start_is_the_operator(problems, name, fast):
    """Algorithm 2 gives u_0 = Q f + P^T u_{-1} (both modes)."""
    p = problems(name)
    K, Z, Q, P, _ = _dense_operators(p)
    o = O.Oracle.from_problem(p)
    rng = np.random.default_rng(5)
    um1 = rng.standard_normal(p.n)
    u0, r0 = o.start(p.f, um1, fast=fast)
    ref = Q @ p.f + P.T @ um1
    assert np.linalg.norm(u0 - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.allclose(r0, p.f - K @ u0, rtol=0, atol=1e-12 * np.abs(p.f).max())
    u0z, _ = o.start(p.f, None, fast=fast)
    assert np.linalg.norm(u0z - Q @ p.f) <= 1e-8 * np.linalg.norm(Q @ p.f)


def test_PK_symmetric_PtK_not(problems):
    """The deflated operator is P K (P = I - K Q), which is symmetric; P^T K is not."""
    p = problems("edge4")
    K, Z, Q, P, _ = _dense_operators(p)
    PK, PtK = P @ K, P.T @ K
    assert np.abs(PK - PK.T).max() <= 1e-9 * np.abs(PK).max()
    assert np.abs(PtK - PtK.T).max() >= 1e-3 * np.abs(PtK).max()


@pytest.mark.parametrize("name", ["plain6", "edge4", "penny12", "edge10"])
def test_fast_mode_takes_the_literal_iterates(problems, name):
    """The fast mode (K Z precomputed, one merged coarse solve by the explicit E^-1,
    Sec. 3.2 identities Z^T K y = (K Z)^T y and lambda - mu = E^-1 (Z^T r - Z^T K y))
    reproduces the literal mode's iteration count and iterates up to rounding."""
    p = problems(name)
    o = O.Oracle.from_problem(p)
    a = o.solve(p.f, tol=1e-8, history=True)
    b = o.solve(p.f, tol=1e-8, history=True, fast=True)
    assert a["status"] == b["status"] == O.OK
    assert a["iterations"] == b["iterations"]
    assert np.linalg.norm(a["u"] - b["u"]) <= 1e-10 * np.linalg.norm(a["u"])
    # residual histories agree to the last digits that rounding leaves intact (the
    # recurrences amplify rounding as ||r_i|| falls: 1e-5 relative at edge4's end)
    assert np.all(np.abs(a["history"] - b["history"]) <= 1e-4 * a["history"])
    # warm start and a few iterations: same recurrences
    um1 = np.random.default_rng(9).standard_normal(p.n)
    a = o.solve(p.f, tol=1e-8, max_iter=5, u0=um1)
    b = o.solve(p.f, tol=1e-8, max_iter=5, u0=um1, fast=True)
    assert a["iterations"] == b["iterations"]
    assert np.linalg.norm(a["u"] - b["u"]) <= 1e-9 * np.linalg.norm(a["u"])


def test_fast_coarse_inverse(problems):
    """The fast mode's explicit E^-1 = L^-T L^-1 against LAPACK's inverse of E."""
    p = problems("penny12")
    o = O.Oracle.from_problem(p)
    E = o.coarse_matrix()
    Ei = o.coarse_inverse()
    ref = np.linalg.inv(E)
    kappa = np.linalg.cond(E)
    assert np.abs(Ei - Ei.T).max() == 0.0
    assert np.linalg.norm(Ei - ref) <= 1e-15 * kappa * np.linalg.norm(ref)
    assert np.abs(Ei @ E - np.eye(p.k)).max() <= 1e-15 * kappa


def test_coarse_matrix(problems):
    p = problems("penny12")
    K = p.K_scipy()
    Z = p.Z_scipy()
    o = O.Oracle.from_problem(p)
    E = o.coarse_matrix()
    Eref = (Z.T @ (K @ Z)).toarray()
    assert np.abs(E - Eref).max() <= 1e-12 * np.abs(Eref).max()
    b = np.random.default_rng(2).standard_normal(p.k)
    assert np.allclose(o.coarse_solve(b), np.linalg.solve(Eref, b), rtol=1e-6, atol=0)


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("name", ["edge10", "penny12"])
def test_Zt_r0_vanishes(problems, name):
    """After the A-DEF2 start, Z^T r_0 = Z^T (f - K u_0) = 0."""
    p = problems(name)
    o = O.Oracle.from_problem(p)
    Z = p.Z_scipy()
    _, r0 = o.start(p.f)
    assert np.linalg.norm(Z.T @ r0) <= 1e-12 * np.linalg.norm(Z.T @ p.f)


def test_solution_in_range_of_Z_converges_at_start(problems):
    """f = K Z c: Algorithm 2 already returns u* = Z c (0 iterations)."""
    p = problems("edge10")
    o = O.Oracle.from_problem(p)
    c = np.random.default_rng(1).standard_normal(p.k)
    u_star = p.Z_scipy() @ c
    f = p.K_scipy() @ u_star
    r = o.solve(f, tol=1e-8)
    assert r["status"] == O.OK and r["iterations"] <= 1
    assert np.linalg.norm(r["u"] - u_star) <= 1e-7 * np.linalg.norm(u_star)


def test_one_block_is_a_direct_solve():
    """One block holding every DoF makes M^{-1} = K^{-1}: one iteration (Sec. 4.1)."""
    p = build_problem("cube1", 1, 1, crack=None)
    assert p.n == 12
    K = p.K_scipy()
    for Z in (None, p.Z_scipy()):
        o = _make(K, Z, [0, p.n])
        r = o.solve(p.f, tol=1e-12)
        assert r["status"] == O.OK and r["iterations"] == 1
        assert np.allclose(r["u"], np.linalg.solve(K.toarray(), p.f), rtol=1e-12, atol=0)


def test_point_jacobi_equals_scipy_cg(problems):
    """Blocks of size 1 and no deflation: the iteration is diagonally preconditioned CG;
    its iterates equal scipy.sparse.linalg.cg's with M = diag(K)^{-1}."""
    p = problems("plain6")
    K = p.K_scipy()
    o = _make(K, None, np.arange(p.n + 1))
    xs = []
    Minv = sp.diags(1.0 / K.diagonal())
    spla.cg(K, p.f, rtol=1e-300, atol=0.0, maxiter=12, M=Minv, callback=lambda x: xs.append(x.copy()))
    for it in (1, 2, 5, 12):
        r = o.solve(p.f, tol=1e-300, max_iter=it)
        assert r["status"] == O.NOT_CONVERGED and r["iterations"] == it
        ref = xs[it - 1]
        assert np.linalg.norm(r["u"] - ref) <= 1e-10 * np.linalg.norm(ref)


def _unit_diag_spd(q, C, seed):
    """B = P (I_q kron C) P^T: unit diagonal, the eigenvalues of C, random order."""
    n = q * C.shape[0]
    B = np.kron(np.eye(q), C)
    perm = np.random.default_rng(seed).permutation(n)
    return B[np.ix_(perm, perm)], perm


def _small_C(c, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((c, c))
    S = A @ A.T + c * np.eye(c)
    d = np.sqrt(np.diag(S))
    C = S / np.outer(d, d)
    np.fill_diagonal(C, 1.0)
    return C


def test_finite_termination():
    """M^{-1} K with c distinct eigenvalues: CG ends in at most c iterations."""
    c, q = 5, 12
    B, _ = _unit_diag_spd(q, _small_C(c, 0), 3)
    D = np.random.default_rng(4).uniform(0.5, 4.0, B.shape[0])
    K = np.sqrt(D)[:, None] * B * np.sqrt(D)[None, :]
    f = np.random.default_rng(5).standard_normal(B.shape[0])
    o = _make(K, None, np.arange(B.shape[0] + 1))
    r = o.solve(f, tol=1e-10, max_iter=100)
    assert r["status"] == O.OK and r["iterations"] <= c
    assert np.allclose(r["u"], np.linalg.solve(K, f), rtol=1e-8)


def test_exact_eigenvector_deflation():
    """M = I and Z spanning the eigenspace of one eigenvalue: the deflated iteration
    sees only the remaining c - 1 eigenvalues."""
    c, q = 5, 10
    C = _small_C(c, 9)
    B, perm = _unit_diag_spd(q, C, 8)
    w, V = np.linalg.eigh(C)
    n = B.shape[0]
    Z = np.zeros((n, q))
    inv = np.empty(n, int)
    inv[perm] = np.arange(n)
    for j in range(q):
        v = np.zeros(n)
        v[j * c:(j + 1) * c] = V[:, 0]
        Z[:, j] = v[perm]
    assert np.allclose(B @ Z, w[0] * Z)
    f = np.random.default_rng(6).standard_normal(n)
    o_plain = _make(B, None, np.arange(n + 1))
    o_defl = _make(B, sp.csr_matrix(Z), np.arange(n + 1))
    rp = o_plain.solve(f, tol=1e-10)
    rd = o_defl.solve(f, tol=1e-10)
    assert rp["iterations"] <= c and rp["iterations"] >= c - 1
    assert rd["status"] == O.OK and rd["iterations"] <= c - 1
    assert np.allclose(rd["u"], np.linalg.solve(B, f), rtol=1e-8)


def test_enriched_deflation_helps(problems):
    """Adding the enriched modes to the rigid-body modes does not cost iterations."""
    from fixtures.configs import CONFIGS, make_crack
    cfg = CONFIGS["penny12"]
    p_std = build_problem("std", cfg["ne"], cfg["nsd"], crack=make_crack(cfg["crack"]), r_e=cfg["r_e"],
                          enriched_deflation=False)
    p_enr = problems("penny12")
    it_std = O.Oracle.from_problem(p_std).solve(p_std.f)["iterations"]
    it_enr = O.Oracle.from_problem(p_enr).solve(p_enr.f)["iterations"]
    assert it_enr <= it_std


# ------------------------------------------------------------------ status codes
def test_status_codes(problems):
    p = problems("edge4")
    o = O.Oracle.from_problem(p)
    f = p.f.copy()
    f[3] = np.nan
    assert o.solve(f)["status"] == O.ENONFINITE
    r = o.solve(np.zeros(p.n))
    assert r["status"] == O.OK and r["iterations"] == 0 and not r["u"].any()
    r = o.solve(p.f, max_iter=1)
    assert r["status"] == O.NOT_CONVERGED and r["iterations"] == 1
    # duplicate deflation column: E singular
    Z = p.Z_scipy().toarray()
    Z2 = sp.csr_matrix(np.concatenate([Z, Z[:, :1]], 1))
    with pytest.raises(O.OracleError) as e:
        _make(p.K_scipy(), Z2, p.block_ptr)
    assert e.value.status == O.ECOARSE_NOT_SPD
    # indefinite diagonal block
    K = p.K_scipy().tolil()
    b = 7
    s = p.block_ptr[b]
    K[s, s] = -1.0
    with pytest.raises(O.OracleError) as e:
        _make(K.tocsr(), p.Z_scipy(), p.block_ptr)
    assert e.value.status == O.EBLOCK_NOT_SPD and e.value.bad == b


def indefinite_breakdown_system():
    """K = [[A, 2A], [2A, A]] with A SPD: symmetric with SPD nodal blocks, but indefinite
    (eigenvalues of A times 3 and -1).  With f = (A x, -A x) and no deflation, the first
    search direction of Algorithm 1 is p_0 = M^-1 f = (x, -x), and p_0^T K p_0 =
    2 x^T A x - 4 x^T A x = -2 x^T A x < 0: the step length has no valid value."""
    A = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    K = np.block([[A, 2 * A], [2 * A, A]])
    x = np.array([1.0, -0.5, 0.25])
    f = np.concatenate([A @ x, -(A @ x)])
    return K, f, np.array([0, 3, 6])


def test_indefinite_system_breaks_down_at_the_first_step():
    K, f, bp = indefinite_breakdown_system()
    assert np.linalg.eigvalsh(K).min() < 0
    p0 = np.linalg.solve(np.kron(np.eye(2), K[:3, :3]), f)  # block-Jacobi, no deflation
    assert p0 @ K @ p0 < 0
    Ks = sp.csr_matrix(K)
    Ks.sort_indices()
    o = O.Oracle(6, Ks.indptr.astype(np.int64), Ks.indices.astype(np.int32), Ks.data, 0,
                 np.zeros(7, np.int64), np.zeros(0, np.int32), np.zeros(0), bp)
    r = o.solve(f)
    assert r["status"] == O.EBREAKDOWN and r["bad"] == 0 and r["iterations"] == 0


def test_deterministic(problems):
    p = problems("penny12")
    o = O.Oracle.from_problem(p)
    a, b = o.solve(p.f), o.solve(p.f)
    assert np.array_equal(a["u"], b["u"]) and a["iterations"] == b["iterations"]


def test_warm_start_from_solution(problems):
    """u_{-1} = converged solution: the A-DEF2 start keeps it and stops at once."""
    p = problems("penny12")
    o = O.Oracle.from_problem(p)
    u = o.solve(p.f, tol=1e-12)["u"]
    r = o.solve(p.f, tol=1e-8, u0=u)
    assert r["status"] == O.OK and r["iterations"] == 0

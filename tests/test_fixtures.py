"""Pins of the synthetic XFEM input generator (CPU only).

These check the assembled systems against facts of elasticity and of the paper's
deflation vectors, not against the generator's own formulas.
"""
import numpy as np
import pytest

from fixtures.xfem import (PlanarEdgeCrack, ThroughCrack, XfemBox, branch_functions, bsr_to_csr,
                           build_problem, lame)


def _dense(p):
    return p.K_scipy().toarray()


def _rigid_modes(X):
    """Six rigid-body displacement fields at points X, as (3m, 6)."""
    m = len(X)
    R = np.zeros((m, 3, 6))
    R[:, 0, 0] = R[:, 1, 1] = R[:, 2, 2] = 1.0
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    R[:, :, 3] = np.stack([np.zeros(m), -z, y], -1)
    R[:, :, 4] = np.stack([z, np.zeros(m), -x], -1)
    R[:, :, 5] = np.stack([-y, x, np.zeros(m)], -1)
    return R.reshape(3 * m, 6)


def test_edge10_counts(problems):
    """Node, DoF, block and deflation counts of the 10^3 edge-crack workload."""
    p = problems("edge10")
    m = p.meta
    assert m["nodes"] == 1331 and m["free_nodes"] == 1210
    assert p.n == 4785 and m["n_std"] == 3630 and m["n_enr"] == 1155
    assert m["block_hist"] == {3: 1100, 6: 22, 15: 77, 18: 11}
    assert m["nnzb"] == 68541
    # 8 subdomains x 6 rigid modes; 2 Heaviside subdomains x 6; tip groups with
    # collinear tip nodes lose columns
    assert m["k_std"] == 48 and m["k_heaviside"] == 12
    assert p.k == m["k_std"] + m["k_heaviside"] + m["k_tip"]
    assert np.all(np.diff(p.block_ptr) > 0) and p.block_ptr[-1] == p.n


def test_symmetric_and_spd(problems):
    for name in ("edge4", "penny12", "plain6"):
        p = problems(name)
        K = _dense(p)
        assert np.array_equal(K, K.T)
        np.linalg.cholesky(K)
        Z = p.Z_scipy().toarray()
        assert np.linalg.matrix_rank(Z) == p.k


def test_unconstrained_rigid_modes_in_kernel():
    """An unconstrained body stores no energy under rigid motion: K R = 0."""
    box = XfemBox(3, crack=None, clamp_bottom=False)
    bptr, bcol, bval = box.assemble_bsr()
    rp, c, v = bsr_to_csr(bptr, bcol, bval)
    import scipy.sparse as sp
    K = sp.csr_matrix((v, c, rp), shape=(box.n, box.n))
    R = _rigid_modes(box.X)
    assert np.abs(K @ R).max() <= 1e-13 * np.abs(v).max()
    ev = np.linalg.eigvalsh(K.toarray())
    assert np.sum(ev < 1e-10 * ev[-1]) == 6


@pytest.mark.parametrize("E,nu", [(1.0, 0.3), (2.1e5, 0.25)])
def test_homogeneous_strain_energy(E, nu):
    """u = eps x on the unit cube: 1/2 u^T K u equals 1/2 eps:C:eps times the volume,
    and interior nodes carry no force (patch test)."""
    ne = 3
    box = XfemBox(ne, crack=None, clamp_bottom=False, E=E, nu=nu)
    bptr, bcol, bval = box.assemble_bsr()
    rp, c, v = bsr_to_csr(bptr, bcol, bval)
    import scipy.sparse as sp
    K = sp.csr_matrix((v, c, rp), shape=(box.n, box.n))
    rng = np.random.default_rng(7)
    A = rng.standard_normal((3, 3))
    eps = 0.5 * (A + A.T)
    u = (box.X @ eps.T).reshape(-1)
    lam, mu = lame(E, nu)
    energy = 0.5 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(0.5 * u @ (K @ u) - energy) <= 1e-12 * abs(energy)
    force = (K @ u).reshape(-1, 3)
    interior = np.all((box.node_ijk > 0) & (box.node_ijk < ne), axis=1)
    assert np.abs(force[interior]).max() <= 1e-12 * np.abs(force).max()


@pytest.mark.parametrize("x0", [0.5, 0.45, 0.62])
def test_heaviside_modes_in_kernel_of_through_cracked_body(x0):
    """Body split in two by a through crack, Heaviside enrichment, no supports: the
    paper's enriched deflation vectors (std DoFs H(x_I) W_I, enriched DoFs W_I) and
    the standard rigid-body vectors are rigid motions of the two halves, so K w = 0;
    the kernel of K is exactly 12-dimensional."""
    p = build_problem("through", 4, 1, crack=ThroughCrack(x0), clamp_bottom=False, load=False)
    K = _dense(p)
    Z = p.Z_scipy().toarray()
    assert p.k == 12 and p.meta["k_heaviside"] == 6
    assert np.abs(K @ Z).max() <= 1e-12 * np.abs(K).max() * np.abs(Z).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-9 * ev[-1]) == 12


def test_branch_function_gradients():
    """Analytic gradients of the shifted branch functions vs central differences."""
    cr = PlanarEdgeCrack(0.5, 0.45)
    rng = np.random.default_rng(3)
    X = rng.uniform([0.3, 0.0, 0.3], [0.7, 1.0, 0.6], size=(50, 3))
    X = X[np.abs(X[:, 0] - 0.5) > 0.01]
    F, G = branch_functions(*cr.tip_coords(X))
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        Fp, _ = branch_functions(*cr.tip_coords(X + e))
        Fm, _ = branch_functions(*cr.tip_coords(X - e))
        assert np.allclose((Fp - Fm) / (2 * h), G[:, :, d], rtol=1e-5, atol=1e-6)
    # sqrt(r) sin(theta/2) jumps by 2 sqrt(r) across the crack faces; the others do not
    y = np.array([[0.5 + 1e-12, 0.3, 0.2], [0.5 - 1e-12, 0.3, 0.2]])
    Fy, _ = branch_functions(*cr.tip_coords(y))
    assert np.isclose(Fy[0, 0] - Fy[1, 0], 2 * np.sqrt(0.25))
    assert np.allclose(Fy[0, 1:], Fy[1, 1:], atol=1e-6)


def test_nodal_blocks_match_groups(problems):
    """Each nodal block is one node's [u, b, c1..c4] triplets: sizes 3, 6, 15 or 18."""
    p = problems("edge10")
    s = np.diff(p.block_ptr)
    assert set(np.unique(s).tolist()) <= {3, 6, 15, 18}
    assert s.sum() == p.n

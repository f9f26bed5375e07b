"""Pins of the adjoint element-sensitivity oracle (CPU only).

* The element matrices reassemble to the fixture's K (sum_e K_e over the DoF lists).
* Central finite differences of L(E) = c^T K(E)^{-1} f, with K(E) re-assembled from
  scratch by the generator for perturbed element moduli and solved directly, agree
  with -lambda_e^T K_e u_e (the derivative of a matrix inverse).
* sum_e E_e g_e = -lambda^T K u = -lambda^T f, since K is linear in the moduli.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from fixtures import load, load_elements, problem_with_moduli
from oracle.adjoint import element_gradient


def _reassemble(n, ep, ed, ko, km, scale=None):
    rows, cols, vals = [], [], []
    for e in range(len(ep) - 1):
        d = ed[ep[e]:ep[e + 1]]
        m = len(d)
        M = km[ko[e]:ko[e] + m * m].reshape(m, m) * (1.0 if scale is None else scale[e])
        ok = np.nonzero(d >= 0)[0]
        A, B = np.meshgrid(ok, ok, indexing="ij")
        rows.append(d[A].ravel())
        cols.append(d[B].ravel())
        vals.append(M[A, B].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


@pytest.mark.parametrize("name", ["edge4", "penny12", "edge10"])
def test_element_matrices_reassemble_K(name):
    p = load(name)
    ep, ed, ko, km = load_elements(name)
    K = p.K_scipy()
    Kr = _reassemble(p.n, ep, ed, ko, km)
    assert abs(Kr - K).max() <= 1e-14 * abs(K).max()
    assert (np.diff(ep) == 24).sum() > 0 and (np.diff(ep) > 24).sum() > 0  # standard and enriched


def test_element_gradient_matches_finite_differences():
    name = "edge4"
    p = load(name)
    ep, ed, ko, km = load_elements(name)
    nel = len(ep) - 1
    c = np.random.default_rng(21).standard_normal(p.n)
    K = p.K_scipy().tocsc()
    u = spla.spsolve(K, p.f)
    lam = spla.spsolve(K, c)
    g = element_gradient(ep, ed, ko, km, u, lam)
    m = np.diff(ep)
    picks = list(np.nonzero(m == 24)[0][:2]) + list(np.nonzero(m > 24)[0][:3])
    h = 1e-4
    for j in picks:
        Ls = []
        for sgn in (1.0, -1.0):
            E = np.ones(nel)
            E[j] += sgn * h
            Kj = problem_with_moduli(name, E).K_scipy().tocsc()
            Ls.append(c @ spla.spsolve(Kj, p.f))
        fd = (Ls[0] - Ls[1]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * abs(g[j]) + 1e-12 * np.abs(g).max(), (j, fd, g[j])


@pytest.mark.parametrize("name", ["penny12", "edge10"])
def test_element_gradient_sum_identity(name):
    p = load(name)
    ep, ed, ko, km = load_elements(name)
    K = p.K_scipy().tocsc()
    u = spla.spsolve(K, p.f)
    lam = spla.spsolve(K, np.random.default_rng(22).standard_normal(p.n))
    g = element_gradient(ep, ed, ko, km, u, lam)
    scale = element_gradient(ep, ed, ko, km, u, lam, absolute=True)
    assert abs(g.sum() + lam @ p.f) <= 1e-12 * scale.sum()
    # a sign or transposition error would break the symmetric pairing: swap u and lambda
    g2 = element_gradient(ep, ed, ko, km, lam, u)
    assert np.allclose(g, g2, rtol=1e-10, atol=1e-14 * scale.max())

"""GPU parity of the adjoint path: the element-sensitivity kernel against the oracle,
and the autograd wrapper (forward solve, adjoint solve, element kernel) against
direct CPU solves and finite differences.

Tolerances:
* element kernel with the same u, lambda: 1e-12 relative to |lambda_e|^T |K_e| |u_e|
  (summation order only);
* gradients from solves at tol 1e-10 against direct solves: 1e-6 relative to the
  largest entry;
* central finite differences (h = 3e-3 on one element modulus, truncation error about
  h^2 relative; GPU solves at tol 1e-12 on freshly assembled systems): 1e-4 relative;
* the adjoint workload (penny60, 20 seeded elements) and every element of edge10:
  central differences with the workload's step h = 1e-6 E_e, each quotient evaluated
  exactly through a solve for u(+h) - u(-h) (see _adjoint_vs_fd), per element within
  1e-5 of max(|g_e|, 1e-6 max |g|).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import scipy.sparse.linalg as spla  # noqa: E402

import paper_2111_09294_amd as D  # noqa: E402
from fixtures import load_elements, problem_with_moduli  # noqa: E402
from oracle.adjoint import element_gradient  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", ["edge4", "penny12", "edge10", "penny40"])
def test_element_gradient_kernel(problems, name):
    p = problems(name)
    ep, ed, ko, km = load_elements(name)
    el = D.Elements(ep, ed, ko, km, DEV)
    rng = np.random.default_rng(31)
    u, lam = rng.standard_normal(p.n), rng.standard_normal(p.n)
    with D.Solver.from_problem(p, DEV) as s:
        g = host(s.element_gradient(el, dev(u), dev(lam)))
    ref = element_gradient(ep, ed, ko, km, u, lam)
    scale = element_gradient(ep, ed, ko, km, u, lam, absolute=True)
    assert np.all(np.abs(g - ref) <= 1e-12 * scale + 1e-300)


def test_element_gradient_rejects_bad_element_data(problems):
    p = problems("edge4")
    ep, ed, ko, km = load_elements("edge4")
    u = dev(np.ones(p.n))
    with D.Solver.from_problem(p, DEV) as s:
        bad = []
        ed2 = ed.copy()
        ed2[5] = p.n                      # DoF out of range
        bad.append((ep, ed2, ko, km))
        ko2 = ko.copy()
        ko2[-1] = len(km) - 10            # matrix beyond the end of kmat
        bad.append((ep, ed, ko2, km))
        ep2 = ep.copy()
        ep2[1:] += 300                    # an element of 300 DoFs (> 256)
        bad.append((ep2, np.concatenate([np.full(300, -1, np.int32), ed]), ko, km))
        for args in bad:
            with pytest.raises(D.DpcgError) as e:
                s.element_gradient(D.Elements(*args, device=DEV), u, u)
            assert e.value.code == D.abi.EINVAL
        g = s.element_gradient(D.Elements(ep, ed, ko, km, DEV), u, u)   # still usable
        assert torch.isfinite(g).all()


def test_autograd_matches_direct_solves(problems):
    name = "edge10"
    p = problems(name)
    ep, ed, ko, km = load_elements(name)
    nel = len(ep) - 1
    el = D.Elements(ep, ed, ko, km, DEV)
    c = np.random.default_rng(32).standard_normal(p.n)
    K = p.K_scipy().tocsc()
    u_ref = spla.spsolve(K, p.f)
    with D.Solver.from_problem(p, DEV) as s:
        for precision in ("fp64", "mixed"):
            f = dev(p.f).requires_grad_(True)
            scale = torch.ones(nel, dtype=torch.float64, device=DEV, requires_grad=True)
            u = D.solve(f, s, scale=scale, elements=el, tol=1e-10, precision=precision)
            # compliance f^T u plus a linear functional c^T u
            L = (f * u).sum() + (dev(c) * u).sum()
            L.backward()
            # dL/du = f + c, lambda = K^{-1}(f + c); dL/df = u + lambda (explicit term + adjoint)
            lam_ref = spla.spsolve(K, p.f + c)
            gf_ref = u_ref + lam_ref
            gs_ref = element_gradient(ep, ed, ko, km, u_ref, lam_ref)
            gf, gs = host(f.grad), host(scale.grad)
            say(f"[adjoint] {precision}: |dL/df err| {np.abs(gf - gf_ref).max():.2e}, "
                f"|dL/ds err| {np.abs(gs - gs_ref).max():.2e} (max {np.abs(gs_ref).max():.2e})")
            assert np.abs(gf - gf_ref).max() <= 1e-6 * np.abs(gf_ref).max()
            assert np.abs(gs - gs_ref).max() <= 1e-6 * np.abs(gs_ref).max()


def test_autograd_matches_finite_differences(problems):
    name = "edge10"
    p = problems(name)
    ep, ed, ko, km = load_elements(name)
    nel = len(ep) - 1
    m = np.diff(ep)
    el = D.Elements(ep, ed, ko, km, DEV)
    c = dev(np.random.default_rng(33).standard_normal(p.n))
    with D.Solver.from_problem(p, DEV) as s:
        scale = torch.ones(nel, dtype=torch.float64, device=DEV, requires_grad=True)
        u = D.solve(dev(p.f), s, scale=scale, elements=el, tol=1e-12)
        (c * u).sum().backward()
        gs = host(scale.grad)
    h = 3e-3
    for j in [int(np.nonzero(m == 24)[0][7]), int(np.argmax(np.abs(gs) * (m > 24)))]:
        Ls = []
        for sgn in (1.0, -1.0):
            E = np.ones(nel)
            E[j] += sgn * h
            pj = problem_with_moduli(name, E)
            with D.Solver.from_problem(pj, DEV) as sj:
                uj, info = sj.solve(dev(pj.f), tol=1e-12)
                assert info["status"] == D.abi.OK
            Ls.append(float((c * uj).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * h)
        say(f"[adjoint] element {j} (m={m[j]}): autograd {gs[j]:.10e}, central FD {fd:.10e}")
        assert abs(fd - gs[j]) <= 1e-4 * abs(gs[j])


# ------------------------------------------------------------------ the adjoint workload
def _perturbed_values(p, ep, ed, ko, km, j, delta):
    """CSR values of K + delta K_j: element j's unit-modulus matrix added at its DoF
    pairs (every such pair is in K's pattern), i.e. K re-assembled with E_j + delta."""
    vals = p.k_val.copy()
    d = ed[ep[j]:ep[j + 1]].astype(np.int64)
    m = len(d)
    M = km[ko[j]:ko[j] + m * m].reshape(m, m)
    ok = np.nonzero(d >= 0)[0]
    for a in ok:
        r0, r1 = p.k_rowptr[d[a]], p.k_rowptr[d[a] + 1]
        pos = r0 + np.searchsorted(p.k_col[r0:r1], d[ok])
        assert np.array_equal(p.k_col[pos], d[ok])
        vals[pos] += delta * M[a, ok]
    return vals


def _solver_with_values(p, vals):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)  # noqa: E731
    return D.Solver(p.n, t(p.k_rowptr, torch.int64), t(p.k_col, torch.int32), t(vals, torch.float64), p.k,
                    t(p.z_rowptr, torch.int64), t(p.z_col, torch.int32), t(p.z_val, torch.float64),
                    t(p.block_ptr, torch.int32))


def _adjoint_vs_fd(name, picks, h_rel, tol):
    """Loss L = f^T u + (sum of crack-opening jumps) with per-element moduli
    E_e = exp(0.5 g_e): autograd gradients against central differences
    (L(E_e + h) - L(E_e - h)) / 2h over the moduli of the picked elements.

    Each difference quotient is evaluated exactly without subtracting two solutions
    that agree to about h / E_e (the cancellation would leave the solves' last digits
    divided by 2h): with K(+-h) = K +- h K_e (fresh setups of the re-assembled
    values), K(+h) (u(+h) - u(-h)) = f - K(+h) u(-h) = -2h K_e u(-h), so
    (L(+h) - L(-h)) / 2h = -(f + c)^T w with K(+h) w = K_e u(-h).  Only forward solves
    of the perturbed systems are used (no adjoint)."""
    from fixtures import box, load_elements, log_normal_moduli, problem_with_moduli
    E = log_normal_moduli(name)
    p = problem_with_moduli(name, E)
    ep, ed, ko, km = load_elements(name)
    c = box(name).cod_functional()
    el = D.Elements(ep, ed, ko, km, DEV)
    fc = dev(p.f + c)
    with D.Solver.from_problem(p, DEV) as s:
        f = dev(p.f).requires_grad_(True)
        scale = torch.as_tensor(E, device=DEV).requires_grad_(True)
        u = D.solve(f, s, scale=scale, elements=el, tol=tol)
        L = (f * u).sum() + (dev(c) * u).sum()
        L.backward()
        gs = host(scale.grad)
        gf = host(f.grad)
        # dL/df = u + lambda, lambda = K^{-1} (f + c)
        lam, _ = s.solve(fc, tol=tol)
        assert np.abs(gf - host(u.detach()) - host(lam)).max() <= 1e-8 * np.abs(gf).max()
    fd = np.empty(len(picks))
    for q, j in enumerate(picks):
        h = h_rel * E[j]
        with _solver_with_values(p, _perturbed_values(p, ep, ed, ko, km, j, -h)) as sm:
            um, info = sm.solve(dev(p.f), tol=tol)
            assert info["status"] == D.abi.OK
        d = ed[ep[j]:ep[j + 1]].astype(np.int64)
        m = len(d)
        M = km[ko[j]:ko[j] + m * m].reshape(m, m)
        ok = d >= 0
        ue = np.zeros(m)
        ue[ok] = host(um)[d[ok]]
        b = np.zeros(p.n)
        np.add.at(b, d[ok], (M @ ue)[ok])
        with _solver_with_values(p, _perturbed_values(p, ep, ed, ko, km, j, h)) as sp_:
            w, info = sp_.solve(dev(b), tol=tol)
            assert info["status"] == D.abi.OK
        fd[q] = -float((fc * w).sum())
    return gs, fd


def _assert_per_element(gs, fd, picks, what):
    """Each element on its own: |FD_e - g_e| <= 1e-5 max(|g_e|, floor), floor = 1e-6
    max_e |g_e|: a gradient a million times below the largest is held to an absolute
    1e-11 of the largest, the level of the solves' own accuracy (relative residual
    1e-12) in the difference quotient."""
    g = gs[picks]
    floor = 1e-6 * np.abs(gs).max()
    scale = np.maximum(np.abs(g), floor)
    rel = np.abs(fd - g) / scale
    say(f"[adjoint] {what}: max |FD - g| / max(|g_e|, floor) = {rel.max():.2e} (median {np.median(rel):.2e}); "
        f"{int(np.sum(np.abs(g) < floor))} of {len(g)} elements below the floor; "
        f"max |FD - g| / max |g| = {np.abs(fd - g).max() / np.abs(gs).max():.2e}")
    assert np.all(rel <= 1e-5), np.argsort(-rel)[:5]


def test_adjoint_full_finite_difference_check_edge10():
    """Every element of the 10^3 mesh (log-normal moduli, compliance + COD loss)."""
    import fixtures
    nel = fixtures.CONFIGS["edge10"]["ne"] ** 3
    picks = np.arange(nel)
    gs, fd = _adjoint_vs_fd("edge10", picks, 1e-6, 1e-12)
    _assert_per_element(gs, fd, picks, "edge10 all elements")


def test_adjoint_finite_differences_penny60():
    """The 60^3 adjoint workload: 20 seeded random elements."""
    import fixtures
    nel = fixtures.CONFIGS["penny60"]["ne"] ** 3
    picks = np.random.default_rng(60).choice(nel, 20, replace=False)
    say("[adjoint] penny60: building the system and element matrices (about a minute)")
    gs, fd = _adjoint_vs_fd("penny60", picks, 1e-6, 1e-12)
    _assert_per_element(gs, fd, picks, "penny60 20 elements")

"""GPU parity of value updates (crack-growth style): new element moduli on the
enriched elements, the same sparsity pattern, dpcg_update_values with the list of
affected block-Jacobi blocks.  The updated handle must give bitwise the results of a
fresh setup on the new matrix; a list that misses changed blocks still converges (stale
block inverses are still an SPD preconditioner); another pattern is rejected."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2111_09294_amd as D  # noqa: E402
from fixtures import CONFIGS, load, load_elements, problem_with_moduli  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)


def _k(p):
    return dev(p.k_rowptr, torch.int64), dev(p.k_col, torch.int32), dev(p.k_val)


@pytest.mark.parametrize("name", ["edge10", "penny40"])
def test_update_values_matches_fresh_setup(name):
    p0 = load(name)
    ep, ed, ko, km = load_elements(name)
    nel = CONFIGS[name]["ne"] ** 3
    m = np.diff(ep)
    enr = np.nonzero(m > 24)[0]                     # the elements of enriched nodes
    E = np.ones(nel)
    E[enr] = 2.0
    p1 = problem_with_moduli(name, E)
    assert np.array_equal(p1.k_col, p0.k_col) and np.array_equal(p1.k_rowptr, p0.k_rowptr)
    dofs = np.unique(np.concatenate([ed[ep[e]:ep[e + 1]] for e in enr]))
    dofs = dofs[dofs >= 0]
    blocks = np.unique(np.searchsorted(p0.block_ptr, dofs, side="right") - 1).astype(np.int32)
    f = dev(p1.f)
    with D.Solver.from_problem(p1, DEV) as fresh:
        u_ref, i_ref = fresh.solve(f)
        setup_ms = i_ref["setup_ms"]
    with D.Solver.from_problem(p0, DEV) as s:
        s.solve(dev(p0.f))
        info = s.update_values(*_k(p1), changed_blocks=blocks)
        u1, i1 = s.solve(f)
        say(f"[update] {name}: {len(blocks)} of {p0.nblocks} blocks refactorised, update {info['setup_ms']:.2f} ms "
            f"vs setup {setup_ms:.2f} ms; iterations {i1['iterations']} (fresh {i_ref['iterations']})")
        assert i1["iterations"] == i_ref["iterations"] and torch.equal(u1, u_ref)
        # every block refactorised: same result
        s.update_values(*_k(p1))
        u2, i2 = s.solve(f)
        assert torch.equal(u2, u_ref)
        # back to the old values, then a list that misses half of the changed blocks
        s.update_values(*_k(p0))
        s.update_values(*_k(p1), changed_blocks=blocks[::2])
        u3, i3 = s.solve(f)
        assert i3["status"] == D.abi.OK and i3["rel_res_true"] <= 1.5e-8
        assert torch.linalg.norm(u3 - u_ref) <= 1e-6 * torch.linalg.norm(u_ref)
        # mixed-precision copies follow the update
        s.solve(f, precision="mixed")
        s.update_values(*_k(p0))
        um, im = s.solve(dev(p0.f), precision="mixed")
        with D.Solver.from_problem(p0, DEV) as s0:
            u0, _ = s0.solve(dev(p0.f))
        assert im["status"] == D.abi.OK and torch.linalg.norm(um - u0) <= 1e-6 * torch.linalg.norm(u0)


def test_update_values_rejects_other_patterns():
    p = load("edge4")
    import scipy.sparse as sp
    K = p.K_scipy().tocoo()
    i, j = p.n - 3, 0
    K2 = sp.csr_matrix((np.append(K.data, 0.0), (np.append(K.row, i), np.append(K.col, j))), shape=K.shape)
    K2.sort_indices()
    with D.Solver.from_problem(p, DEV) as s:
        with pytest.raises(D.DpcgError) as e:
            s.update_values(dev(K2.indptr, torch.int64), dev(K2.indices, torch.int32), dev(K2.data))
        assert e.value.code == D.abi.EINVAL
    with D.Solver.from_problem(p, DEV) as s:
        with pytest.raises(D.DpcgError) as e:
            s.update_values(*_k(p), changed_blocks=[0, p.nblocks])
        assert e.value.code == D.abi.EINVAL
        bad = p.k_val.copy()
        bad[5] = np.nan
        with pytest.raises(D.DpcgError) as e:
            s.update_values(dev(p.k_rowptr, torch.int64), dev(p.k_col, torch.int32), dev(bad))
        assert e.value.code == D.abi.EINVAL

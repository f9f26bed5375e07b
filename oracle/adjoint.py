"""Oracle for the adjoint element sensitivities (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
module; the product path never does.

For K = sum_e s_e K_e (s_e a per-element scaling such as Young's modulus, K_e the
element matrix for s_e = 1; the assembled stiffness of Sec. 2.4, eq. linear_system)
and u = K^{-1} f, a loss L(u) has dL/ds_e = -lambda^T K_e u with the adjoint
lambda = K^{-1} dL/du, since dK^{-1}/ds_e = -K^{-1} K_e K^{-1} and K is symmetric.
Element e touches only its DoFs, so the product is -lambda_e^T K_e u_e over them.
Plain numpy in FP64: the standard elements that share one matrix are evaluated as
one batched product, the others one by one.
"""
from __future__ import annotations

import numpy as np


def _gather(v, dofs):
    """v at the DoFs, 0 where the DoF is -1 (a clamped node)."""
    out = np.zeros(dofs.shape)
    ok = dofs >= 0
    out[ok] = v[dofs[ok]]
    return out


def element_gradient(elem_ptr, elem_dof, kmat_off, kmat, u, lam, absolute=False):
    """g[e] = -lambda_e^T K_e u_e for every element (or, with absolute=True, the
    magnitude |lambda_e|^T |K_e| |u_e| of the same sum, a scale for tolerances)."""
    elem_ptr = np.asarray(elem_ptr, np.int64)
    elem_dof = np.asarray(elem_dof, np.int64)
    kmat_off = np.asarray(kmat_off, np.int64)
    kmat = np.asarray(kmat, np.float64)
    u = np.asarray(u, np.float64)
    lam = np.asarray(lam, np.float64)
    nel = len(elem_ptr) - 1
    m = np.diff(elem_ptr)
    g = np.zeros(nel)
    # groups of elements with the same matrix offset and size: one batched product each
    key = kmat_off * 4096 + m
    for k in np.unique(key):
        ids = np.nonzero(key == k)[0]
        me = int(m[ids[0]])
        if me == 0:
            continue
        K = kmat[kmat_off[ids[0]]:kmat_off[ids[0]] + me * me].reshape(me, me)
        dofs = elem_dof[elem_ptr[ids][:, None] + np.arange(me)]
        U = _gather(u, dofs)
        L = _gather(lam, dofs)
        if absolute:
            g[ids] = ((np.abs(U) @ np.abs(K).T) * np.abs(L)).sum(1)
        else:
            g[ids] = -((U @ K.T) * L).sum(1)
    return g

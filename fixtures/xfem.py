"""Synthetic XFEM inputs: hex8 meshes of the unit cube with an embedded crack.

This is the input generator shared by the tests, the benchmark and the oracle-side
checks.  It holds no part of the solver.  It produces, for one configuration:

* the SPD stiffness matrix K (scalar CSR, FP64, full symmetric storage) of a cracked
  linear elastic body, discretised with the XFEM displacement approximation of the
  paper (Sec. 2.3, eq. xfem_displ): standard trilinear DoFs, shifted Heaviside DoFs
  (eq. jump_enr_functions, H = +1 for phi >= 0) and four shifted branch-function DoF
  triplets per tip node;
* the load vector f (uniform traction on the top face);
* the subdomain deflation matrix Z (Sec. 3.3.1 eq. dcg_deflation_space, Sec. 3.3.2
  eqs. dcg_deflation_space_enr_std / dcg_deflation_space_enr_enr);
* the nodal block partition used by block-Jacobi (Sec. 3.4, eqs. block_jacobi and
  block_jacobi_enr applied per node: [u, b, c1..c4] of one node form one block).

DoF layout ("node-major triplets"): free nodes in lexicographic order (x fastest);
for each node the triplets [u] then [b] if Heaviside-enriched then [c1, c2, c3, c4]
if tip-enriched.  Every DoF group is a 3-vector, so n % 3 == 0.

Readings where the paper is silent (each also listed in the design notes):
* the tip functions are the four classical branch functions, shifted by their nodal
  values (the quasi-orthogonal set of eq. orthogonal_tip_enr_func has a singular
  constant at theta_I = pi, which nodes on a crack face reach);
* a node is Heaviside-enriched when no element of its support contains the front,
  the crack exists at the node's projection, and both sides of the crack hold at
  least ``min_split_frac`` of the support volume (measured on the 8^3 Gauss points);
* a node is tip-enriched when its support contains a front element or its distance
  to the front is <= r_e (with a 1e-9 relative tie tolerance);
* Dirichlet nodes (clamped face z = 0) lose all DoFs, standard and enriched;
* rigid-body coordinates are taken relative to the subdomain centroid (same span);
* enriched deflation columns for a branch function put W_I on that function's DoFs
  of the tip nodes of the subdomain and zero elsewhere; linearly dependent columns
  of one subdomain are dropped by in-order selection (standard, Heaviside, tip).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------
# hex8 reference element
# ----------------------------------------------------------------------------------
HEX_OFF = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)
_SGN = 2 * HEX_OFF - 1  # local node coordinates in [-1, 1]


def gauss_rule_3d(npt: int):
    """Tensor Gauss-Legendre rule on [-1,1]^3: points (g,3), weights (g,)."""
    x, w = np.polynomial.legendre.leggauss(npt)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
    return X, W


def hex8_shape(xi: np.ndarray):
    """Trilinear shape functions N (g,8) and derivatives dN/dxi (g,8,3)."""
    f = 1.0 + xi[:, None, :] * _SGN[None, :, :]          # (g,8,3)
    N = f.prod(-1) / 8.0
    dN = np.empty(f.shape)
    dN[..., 0] = _SGN[None, :, 0] * f[..., 1] * f[..., 2] / 8.0
    dN[..., 1] = _SGN[None, :, 1] * f[..., 0] * f[..., 2] / 8.0
    dN[..., 2] = _SGN[None, :, 2] * f[..., 0] * f[..., 1] / 8.0
    return N, dN


def lame(E: float, nu: float):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def stiffness_from_gradients(G: np.ndarray, w: np.ndarray, lam: float, mu: float):
    """Element stiffness for vector-valued DoF triplets of scalar functions.

    G: (g, m, 3) gradients of the m scalar functions at the g quadrature points,
    w: (g,) quadrature weights including the Jacobian.  Returns (m,3,m,3) with
    K[a,i,b,j] = int lam d_i phi_a d_j phi_b + mu delta_ij grad phi_a . grad phi_b
                     + mu d_j phi_a d_i phi_b,
    i.e. the bilinear form of the weak form (Sec. 2.1) for isotropic Hooke's law.
    """
    g, m, _ = G.shape
    A = G.reshape(g, 3 * m)
    M = ((A * w[:, None]).T @ A).reshape(m, 3, m, 3)     # M[a,k,b,l] = int d_k phi_a d_l phi_b
    tr = np.einsum("akbk->ab", M)
    K = lam * M + mu * np.swapaxes(M, 1, 3)
    K = K + mu * tr[:, None, :, None] * np.eye(3)[None, :, None, :]
    K = 0.5 * (K + K.transpose(2, 3, 0, 1))
    return K


def hex8_standard_stiffness(h: float, E: float, nu: float):
    """Stiffness (8,3,8,3) of an undistorted cube element of side h (2^3 Gauss, exact)."""
    xi, wq = gauss_rule_3d(2)
    _, dN = hex8_shape(xi)
    G = dN * (2.0 / h)
    w = wq * (h / 2.0) ** 3
    lam, mu = lame(E, nu)
    return stiffness_from_gradients(G, w, lam, mu)


# ----------------------------------------------------------------------------------
# crack geometries
# ----------------------------------------------------------------------------------
class PlanarEdgeCrack:
    """Planar crack in the plane x = x0, occupying z < zf across the full y-width.

    Front: the line x = x0, z = zf.  phi = x - x0, psi = z - zf (psi > 0 ahead).
    """

    def __init__(self, x0: float = 0.5, zf: float = 0.45, z0: float = -1.0):
        self.x0, self.zf, self.z0 = float(x0), float(zf), float(z0)

    def level(self, X):
        return X[..., 0] - self.x0

    def on_crack(self, X):
        return (X[..., 2] < self.zf) & (X[..., 2] > self.z0)

    def tip_coords(self, X):
        phi = X[..., 0] - self.x0
        psi = X[..., 2] - self.zf
        gphi = np.zeros(X.shape)
        gphi[..., 0] = 1.0
        gpsi = np.zeros(X.shape)
        gpsi[..., 2] = 1.0
        return phi, psi, gphi, gpsi

    def front_points(self, h):
        m = int(math.ceil(16.0 / h)) + 1
        y = np.linspace(0.0, 1.0, m)
        return np.stack([np.full(m, self.x0), y, np.full(m, self.zf)], -1)

    def has_front(self):
        return self.zf < 1.0


class ThroughCrack(PlanarEdgeCrack):
    """Plane x = x0 cutting the whole body: no front, two free halves (test geometry)."""

    def __init__(self, x0: float):
        super().__init__(x0=x0, zf=10.0)

    def front_points(self, h):
        return np.zeros((0, 3))

    def has_front(self):
        return False


class CurvedPennyCrack:
    """Penny crack of radius R bent into the paraboloid z = zc + c*rho^2 (rho <= R).

    rho is the distance to the vertical axis through (xc, yc).  H uses the sign of
    g = z - zc - c*rho^2.  Tip coordinates: phi = g/|grad g| (signed distance to the
    surface to first order) and psi = signed distance, in the meridian plane, to the
    line through the front normal to the surface (psi > 0 outside the rim).
    """

    def __init__(self, center=(0.5, 0.5, 0.5), R: float = 0.25, curv: float = 0.3):
        self.xc, self.yc, self.zc = (float(v) for v in center)
        self.R, self.c = float(R), float(curv)
        self.zf = self.zc + self.c * self.R ** 2
        self.s = 2.0 * self.c * self.R

    def _rho(self, X):
        dx = X[..., 0] - self.xc
        dy = X[..., 1] - self.yc
        return dx, dy, np.sqrt(dx * dx + dy * dy)

    def level(self, X):
        _, _, rho = self._rho(X)
        return X[..., 2] - self.zc - self.c * rho * rho

    def on_crack(self, X):
        return self._rho(X)[2] < self.R

    def tip_coords(self, X):
        dx, dy, rho = self._rho(X)
        c = self.c
        g = X[..., 2] - self.zc - c * rho * rho
        gg = np.stack([-2 * c * dx, -2 * c * dy, np.ones_like(dx)], -1)
        a = np.sqrt(1.0 + 4 * c * c * rho * rho)
        ga = np.stack([4 * c * c * dx, 4 * c * c * dy, np.zeros_like(dx)], -1) / a[..., None]
        phi = g / a
        gphi = gg / a[..., None] - (g / (a * a))[..., None] * ga
        nrm = math.sqrt(1.0 + self.s ** 2)
        psi = ((rho - self.R) + self.s * (X[..., 2] - self.zf)) / nrm
        rs = np.where(rho > 0, rho, 1.0)
        grho = np.stack([dx / rs, dy / rs, np.zeros_like(dx)], -1)
        gpsi = (grho + np.array([0.0, 0.0, self.s])) / nrm
        return phi, psi, gphi, gpsi

    def front_points(self, h):
        m = int(math.ceil(2 * math.pi * self.R * 16.0 / h)) + 1
        t = np.linspace(0.0, 2 * math.pi, m, endpoint=False)
        return np.stack([self.xc + self.R * np.cos(t), self.yc + self.R * np.sin(t),
                         np.full(m, self.zf)], -1)

    def has_front(self):
        return True


def branch_functions(phi, psi, gphi, gpsi):
    """The four classical branch functions and their gradients.

    r = sqrt(phi^2 + psi^2), theta = atan2(phi, psi) (eq. polar_coords with the
    quadrant fixed by atan2; theta = +pi on the phi >= 0 crack face).
    F = [sqrt(r) sin(t/2), sqrt(r) cos(t/2), sqrt(r) sin(t/2) sin t, sqrt(r) cos(t/2) sin t].
    Returns F (...,4) and grad F (...,4,3).
    """
    r = np.sqrt(phi * phi + psi * psi)
    th = np.arctan2(phi, psi)
    sr = np.sqrt(r)
    s2, c2 = np.sin(th / 2), np.cos(th / 2)
    st, ct = np.sin(th), np.cos(th)
    F = np.stack([sr * s2, sr * c2, sr * s2 * st, sr * c2 * st], -1)
    rs = np.where(r > 0, r, 1.0)
    dr = np.stack([s2, c2, s2 * st, c2 * st], -1) / (2.0 * np.sqrt(rs))[..., None]
    dth = np.stack([c2 / 2, -s2 / 2, c2 / 2 * st + s2 * ct, -s2 / 2 * st + c2 * ct], -1) * sr[..., None]
    gr = (phi[..., None] * gphi + psi[..., None] * gpsi) / rs[..., None]
    gth = (psi[..., None] * gphi - phi[..., None] * gpsi) / (rs * rs)[..., None]
    G = dr[..., None] * gr[..., None, :] + dth[..., None] * gth[..., None, :]
    return F, G


# ----------------------------------------------------------------------------------
# problem container
# ----------------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    n: int
    k_rowptr: np.ndarray          # int64 (n+1)
    k_col: np.ndarray             # int32
    k_val: np.ndarray             # float64
    f: np.ndarray                 # float64 (n)
    z_rowptr: np.ndarray          # int64 (n+1)
    z_col: np.ndarray             # int32
    z_val: np.ndarray             # float64
    k: int                        # number of deflation columns
    block_ptr: np.ndarray         # int32 (nblocks+1)
    meta: dict = field(default_factory=dict)

    @property
    def nblocks(self):
        return len(self.block_ptr) - 1

    def K_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.k_val, self.k_col, self.k_rowptr), shape=(self.n, self.n))

    def Z_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.z_val, self.z_col, self.z_rowptr), shape=(self.n, self.k))

    def block_sizes(self):
        return np.diff(self.block_ptr)


# ----------------------------------------------------------------------------------
# the generator
# ----------------------------------------------------------------------------------
class XfemBox:
    """Structured ne^3 hex8 mesh of the unit cube with one crack."""

    def __init__(self, ne: int, crack=None, r_e: float = 0.0, E: float = 1.0, nu: float = 0.3,
                 clamp_bottom: bool = True, n_gauss_enr: int = 8, min_split_frac: float = 1e-3,
                 tip: bool = True, elem_E: np.ndarray | None = None):
        self.ne = int(ne)
        self.h = 1.0 / self.ne
        self.n1 = self.ne + 1
        self.crack = crack
        self.r_e = float(r_e)
        self.E, self.nu = float(E), float(nu)
        self.clamp = clamp_bottom
        self.ng = int(n_gauss_enr)
        self.min_split_frac = float(min_split_frac)
        self.tip = tip and crack is not None and crack.has_front()
        nel = self.ne ** 3
        self.elem_E = np.full(nel, self.E) if elem_E is None else np.asarray(elem_E, float)
        assert self.elem_E.shape == (nel,)
        n1 = self.n1
        idx = np.arange(n1 ** 3)
        self.node_ijk = np.stack([idx % n1, (idx // n1) % n1, idx // (n1 * n1)], -1)
        self.X = self.node_ijk / float(self.ne)
        e = np.arange(nel)
        self.elem_ijk = np.stack([e % self.ne, (e // self.ne) % self.ne, e // (self.ne ** 2)], -1)
        lin = HEX_OFF[:, 0] + n1 * (HEX_OFF[:, 1] + n1 * HEX_OFF[:, 2])
        origin = self.elem_ijk[:, 0] + n1 * (self.elem_ijk[:, 1] + n1 * self.elem_ijk[:, 2])
        self.conn = origin[:, None] + lin[None, :]                 # (nel, 8)
        self.free = self.node_ijk[:, 2] > 0 if self.clamp else np.ones(n1 ** 3, bool)
        self._classify()
        self._number()

    # -- enrichment sets ---------------------------------------------------------
    def _elements_containing(self, P):
        """Elements whose closed box contains any of the points P (m,3)."""
        if len(P) == 0:
            return np.zeros(0, np.int64)
        ne, h = self.ne, self.h
        out = []
        for d in [(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]:
            q = np.floor((P + 1e-9 * np.array(d)) / h).astype(np.int64)
            ok = np.all((q >= 0) & (q < ne), axis=1)
            q = q[ok]
            out.append(q[:, 0] + ne * (q[:, 1] + ne * q[:, 2]))
        return np.unique(np.concatenate(out))

    def _element_gauss_points(self, elems, xi):
        x0 = self.elem_ijk[elems] * self.h                       # (m,3)
        return x0[:, None, :] + (xi[None, :, :] + 1.0) * (self.h / 2.0)

    def _classify(self):
        nel, nn = self.ne ** 3, self.n1 ** 3
        self.is_front_elem = np.zeros(nel, bool)
        self.H_node = np.zeros(nn, bool)
        self.T_node = np.zeros(nn, bool)
        self.node_sign = np.ones(nn)
        if self.crack is None:
            return
        cr = self.crack
        self.node_sign = np.where(cr.level(self.X) >= 0, 1.0, -1.0)
        fe = self._elements_containing(cr.front_points(self.h))
        self.is_front_elem[fe] = True
        # volume of each element on the + and - side of the crack surface, measured on
        # the 8^3 Gauss points of the elements near the surface (others are one-sided)
        xi, wq = gauss_rule_3d(self.ng)
        centers = (self.elem_ijk + 0.5) * self.h
        band = np.abs(cr.level(centers)) < 2.0 * self.h
        pos = np.where(cr.level(centers) >= 0, 1.0, 0.0)
        band_ids = np.nonzero(band)[0]
        if len(band_ids):
            wn = wq / wq.sum()
            for s in range(0, len(band_ids), 4096):
                ids = band_ids[s:s + 4096]
                Xg = self._element_gauss_points(ids, xi)
                pos[ids] = ((cr.level(Xg) >= 0) * wn[None, :]).sum(1)
        # node supports
        n1 = self.n1
        sup_pos = np.zeros(nn)
        sup_cnt = np.zeros(nn)
        sup_front = np.zeros(nn, bool)
        for a in range(8):
            nodes = self.conn[:, a]
            np.add.at(sup_pos, nodes, pos)
            np.add.at(sup_cnt, nodes, 1.0)
            np.logical_or.at(sup_front, nodes, self.is_front_elem)
        frac_pos = sup_pos / np.maximum(sup_cnt, 1.0)
        split = np.minimum(frac_pos, 1.0 - frac_pos) >= self.min_split_frac
        self.H_node = split & ~sup_front & cr.on_crack(self.X)
        if self.tip:
            phi, psi, _, _ = cr.tip_coords(self.X)
            r = np.sqrt(phi * phi + psi * psi)
            self.T_node = sup_front | (r <= self.r_e * (1.0 + 1e-9))
        self.H_node &= self.free
        self.T_node &= self.free
        del n1

    # -- DoF numbering -------------------------------------------------------------
    def _number(self):
        nn = self.n1 ** 3
        ngrp = np.where(self.free, 1 + self.H_node.astype(np.int64) + 4 * self.T_node.astype(np.int64), 0)
        self.ngroups = ngrp
        start = np.zeros(nn + 1, np.int64)
        np.cumsum(ngrp, out=start[1:])
        self.trip_start = start[:-1]
        self.ntrip = int(start[-1])
        self.n = 3 * self.ntrip
        # group slot of b and of c1 within the node (or -1)
        self.slot_b = np.where(self.H_node, 1, -1)
        self.slot_c = np.where(self.T_node, 1 + self.H_node.astype(np.int64), -1)

    def trip(self, node, slot):
        return np.where(self.free[node] & (slot >= 0), self.trip_start[node] + slot, -1)

    # -- assembly -------------------------------------------------------------------
    def _standard_blocks(self):
        """Node-pair 3x3 blocks of the standard part, as triplet COO (rows, cols, vals)."""
        n1 = self.n1
        nn = n1 ** 3
        Ke0 = hex8_standard_stiffness(self.h, 1.0, self.nu)
        St = np.zeros((nn, 27, 3, 3))
        origin = self.conn[:, 0]
        Ee = self.elem_E
        for a in range(8):
            for b in range(8):
                d = HEX_OFF[b] - HEX_OFF[a]
                o = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1)
                na = self.conn[:, a]
                St[na, o] += Ee[:, None, None] * Ke0[a, :, b, :][None]
        del origin
        rows, cols, vals = [], [], []
        ijk = self.node_ijk
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                    nb = ijk + np.array([dx, dy, dz])
                    ok = np.all((nb >= 0) & (nb < n1), axis=1)
                    I = np.nonzero(ok)[0]
                    J = nb[ok, 0] + n1 * (nb[ok, 1] + n1 * nb[ok, 2])
                    keep = self.free[I] & self.free[J]
                    I, J = I[keep], J[keep]
                    rows.append(self.trip_start[I])
                    cols.append(self.trip_start[J])
                    vals.append(St[I, o])
        return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)

    def enriched_elements(self):
        enr = self.H_node | self.T_node
        return np.nonzero(enr[self.conn].any(1))[0]

    def element_functions(self, e, xi, wq):
        """Gradients (g, m, 3) of the element's scalar functions and their triplet ids.

        Functions, per local node a: N_a (standard), N_a (H - H(x_a)) if a is in the
        jump set, N_a (F_j - F_j(x_a)) j=1..4 if a is in the tip set.
        """
        cr = self.crack
        nodes = self.conn[e]
        Xg = self._element_gauss_points(np.array([e]), xi)[0]       # (g,3)
        N, dN = hex8_shape(xi)
        gN = dN * (2.0 / self.h)
        w = wq * (self.h / 2.0) ** 3
        grads, trips = [], []
        if cr is not None:
            Hg = np.where(cr.level(Xg) >= 0, 1.0, -1.0)
        needT = self.T_node[nodes].any()
        if needT:
            Fg, gFg = branch_functions(*cr.tip_coords(Xg))
            Fn, _ = branch_functions(*cr.tip_coords(self.X[nodes]))
        for a in range(8):
            I = nodes[a]
            grads.append(gN[:, a, :])
            trips.append(self.trip(I, 0) if self.free[I] else -1)
            if self.H_node[I]:
                sh = Hg - self.node_sign[I]
                grads.append(gN[:, a, :] * sh[:, None])
                trips.append(self.trip_start[I] + self.slot_b[I])
            if self.T_node[I]:
                for j in range(4):
                    sh = Fg[:, j] - Fn[a, j]
                    grads.append(gN[:, a, :] * sh[:, None] + N[:, a, None] * gFg[:, j, :])
                    trips.append(self.trip_start[I] + self.slot_c[I] + j)
        return np.stack(grads, 1), np.array(trips, np.int64), w

    def _enriched_blocks(self):
        xi, wq = gauss_rule_3d(self.ng)
        lam1, mu1 = lame(1.0, self.nu)
        rows, cols, vals = [], [], []
        for e in self.enriched_elements():
            G, tr, w = self.element_functions(e, xi, wq)
            Ke = stiffness_from_gradients(G, w, lam1, mu1) * self.elem_E[e]
            enr = np.ones(len(tr), bool)
            # standard-standard pairs are already in the standard part
            std = np.zeros(len(tr), bool)
            pos = 0
            for a in range(8):
                I = self.conn[e, a]
                std[pos] = True
                pos += 1 + int(self.H_node[I]) + 4 * int(self.T_node[I])
            enr = ~std
            ok = tr >= 0
            A, B = np.meshgrid(np.arange(len(tr)), np.arange(len(tr)), indexing="ij")
            sel = ok[A] & ok[B] & (enr[A] | enr[B])
            rows.append(tr[A[sel]])
            cols.append(tr[B[sel]])
            vals.append(Ke[A[sel], :, B[sel], :])
        if not rows:
            return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3, 3))
        return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)

    def element_matrices(self):
        """Unit-modulus element stiffness matrices in scalar DoF space.

        K = sum_e elem_E[e] K_e, with K_e the element's matrix for E = 1 over its DoFs
        elem_dof[elem_ptr[e]:elem_ptr[e+1]] (-1 for a DoF of a clamped node).  Each
        function of the element (standard N_a, then N_a (H - H_a) and the four shifted
        branch functions of enriched nodes, node by node) contributes the DoF triplet
        3t, 3t+1, 3t+2 of its triplet t.  Standard elements share one 24 x 24 matrix,
        stored first (kmat_off = 0); an enriched element has its own (8^3 Gauss, with the
        standard-standard pairs from the exact 2^3 matrix, as assembled).
        Returns (elem_ptr int64, elem_dof int32, kmat_off int64, kmat float64).
        """
        nel = self.ne ** 3
        Ke0 = hex8_standard_stiffness(self.h, 1.0, self.nu)        # (8,3,8,3)
        mats = [Ke0.reshape(24, 24)]
        off = 576
        kmat_off = np.zeros(nel, np.int64)
        dofs = [None] * nel
        std_trip = np.where(self.free[self.conn], self.trip_start[self.conn], -1)    # (nel, 8)
        std_dofs = np.where(std_trip[:, :, None] >= 0, 3 * std_trip[:, :, None] + np.arange(3), -1).reshape(nel, 24)
        enr = np.zeros(nel, bool)
        enr_ids = self.enriched_elements()
        enr[enr_ids] = True
        if len(enr_ids):
            xi, wq = gauss_rule_3d(self.ng)
            lam1, mu1 = lame(1.0, self.nu)
        for e in enr_ids:
            G, tr, w = self.element_functions(e, xi, wq)
            Ke = stiffness_from_gradients(G, w, lam1, mu1)             # (m,3,m,3)
            std_pos = []
            pos = 0
            for a in range(8):
                I = self.conn[e, a]
                std_pos.append(pos)
                pos += 1 + int(self.H_node[I]) + 4 * int(self.T_node[I])
            sp_ = np.array(std_pos)
            Ke[np.ix_(sp_, np.arange(3), sp_, np.arange(3))] = Ke0
            m = len(tr)
            mats.append(Ke.reshape(3 * m, 3 * m))
            kmat_off[e] = off
            off += 9 * m * m
            dofs[e] = np.where(tr[:, None] >= 0, 3 * tr[:, None] + np.arange(3), -1).reshape(-1)
        sizes = np.where(enr, 0, 24)
        for e in enr_ids:
            sizes[e] = len(dofs[e])
        elem_ptr = np.zeros(nel + 1, np.int64)
        np.cumsum(sizes, out=elem_ptr[1:])
        elem_dof = np.empty(elem_ptr[-1], np.int32)
        std_ids = np.nonzero(~enr)[0]
        base = elem_ptr[std_ids][:, None] + np.arange(24)
        elem_dof[base.reshape(-1)] = std_dofs[std_ids].reshape(-1)
        for e in enr_ids:
            elem_dof[elem_ptr[e]:elem_ptr[e + 1]] = dofs[e]
        kmat = np.concatenate([M.reshape(-1) for M in mats])
        return elem_ptr, elem_dof, kmat_off, kmat

    def assemble_bsr(self):
        r1, c1, v1 = self._standard_blocks()
        r2, c2, v2 = self._enriched_blocks()
        rows = np.concatenate([r1, r2])
        cols = np.concatenate([c1, c2])
        vals = np.concatenate([v1, v2])
        key = rows * self.ntrip + cols
        order = np.argsort(key, kind="stable")
        key, vals = key[order], vals[order]
        uk, first = np.unique(key, return_index=True)
        bval = np.add.reduceat(vals, first, axis=0)
        brow = uk // self.ntrip
        bcol = uk % self.ntrip
        # exact symmetrisation: average each block with the transpose of its mirror
        tkey = bcol * self.ntrip + brow
        mirror = np.searchsorted(uk, tkey)
        assert np.array_equal(uk[mirror], tkey), "block structure not symmetric"
        bval = 0.5 * (bval + np.swapaxes(bval[mirror], 1, 2))
        bptr = np.zeros(self.ntrip + 1, np.int64)
        np.add.at(bptr, brow + 1, 1)
        bptr = np.cumsum(bptr)
        return bptr, bcol, bval

    def loads(self):
        """Consistent nodal forces of a unit +z traction on the top face z = 1."""
        f = np.zeros(self.n)
        top = np.nonzero((self.node_ijk[:, 2] == self.ne) & self.free)[0]
        assert not (self.H_node[top] | self.T_node[top]).any(), "enriched node on loaded face"
        i, j = self.node_ijk[top, 0], self.node_ijk[top, 1]
        wx = np.where((i == 0) | (i == self.ne), 0.5, 1.0)
        wy = np.where((j == 0) | (j == self.ne), 0.5, 1.0)
        f[3 * self.trip_start[top] + 2] = wx * wy * self.h * self.h
        return f

    def random_top_tractions(self, nrhs, seed):
        """nrhs load cases: on every free node of the top face z = 1, a force whose three
        components are i.i.d. N(0, 1) times the node's tributary area (consistent
        forces of a piecewise-constant random traction).  Returns (n, nrhs)."""
        rng = np.random.default_rng(seed)
        top = np.nonzero((self.node_ijk[:, 2] == self.ne) & self.free)[0]
        i, j = self.node_ijk[top, 0], self.node_ijk[top, 1]
        wx = np.where((i == 0) | (i == self.ne), 0.5, 1.0)
        wy = np.where((j == 0) | (j == self.ne), 0.5, 1.0)
        area = wx * wy * self.h * self.h
        F = np.zeros((self.n, nrhs))
        comps = rng.standard_normal((len(top), 3, nrhs))
        for c in range(3):
            F[3 * self.trip_start[top] + c] = area[:, None] * comps[:, c, :]
        return F

    def cod_functional(self):
        """c with c^T u = the sum over enriched nodes of the crack-opening displacement
        jump components: the shifted Heaviside function jumps by 2 across the crack, so a
        jump node's b DoFs count twice; of the four branch functions only
        sqrt(r) sin(theta / 2) jumps (by 2 sqrt(r)), so a tip node's c1 DoFs count
        2 sqrt(r_I), r_I its distance to the front."""
        c = np.zeros(self.n)
        jn = np.nonzero(self.H_node)[0]
        for comp in range(3):
            c[3 * (self.trip_start[jn] + self.slot_b[jn]) + comp] = 2.0
        tn = np.nonzero(self.T_node)[0]
        if len(tn):
            phi, psi, _, _ = self.crack.tip_coords(self.X[tn])
            r = np.sqrt(phi * phi + psi * psi)
            for comp in range(3):
                c[3 * (self.trip_start[tn] + self.slot_c[tn]) + comp] = 2.0 * np.sqrt(r)
        return c

    # -- deflation space -----------------------------------------------------------
    def subdomain_of_nodes(self, nsd):
        q = np.maximum(0, np.ceil(self.node_ijk * nsd / self.ne).astype(np.int64) - 1)
        q = np.minimum(q, nsd - 1)
        return q[:, 0] + nsd * (q[:, 1] + nsd * q[:, 2])

    @staticmethod
    def rbm(rel):
        """Rigid-body block W_I (m,3,6) of eq. dcg_deflation_space at coordinates rel."""
        m = len(rel)
        W = np.zeros((m, 3, 6))
        x, y, z = rel[:, 0], rel[:, 1], rel[:, 2]
        W[:, 0, 0] = W[:, 1, 1] = W[:, 2, 2] = 1.0
        W[:, 1, 3], W[:, 2, 3] = -z, y
        W[:, 0, 4], W[:, 2, 4] = z, -x
        W[:, 0, 5], W[:, 1, 5] = -y, x
        return W

    def deflation(self, nsd, enriched=True, drop_tol=1e-8):
        """Z (CSR n x k) from subdomain rigid-body modes plus enriched modes.

        Returns (rowptr int64, col int32, val f64, k, info).
        """
        sd = self.subdomain_of_nodes(nsd)
        nsub = nsd ** 3
        entries_r, entries_c, entries_v = [], [], []
        kcol = 0
        info = {"std": 0, "heaviside": 0, "tip": 0, "dropped": 0, "groups": []}
        free_nodes = np.nonzero(self.free)[0]
        sd_free = sd[free_nodes]
        order = np.argsort(sd_free, kind="stable")
        bounds = np.searchsorted(sd_free[order], np.arange(nsub + 1))
        for s in range(nsub):
            nodes = free_nodes[order[bounds[s]:bounds[s + 1]]]
            if len(nodes) == 0:
                continue
            c = self.X[nodes].mean(0)
            W = self.rbm(self.X[nodes] - c)                        # (m,3,6)
            groups = []
            rows_u = (3 * self.trip_start[nodes])[:, None] + np.arange(3)[None, :]
            groups.append(("std", rows_u.reshape(-1), W.reshape(-1, 6)))
            if enriched and self.H_node[nodes].any():
                Hs = self.node_sign[nodes]
                hn = nodes[self.H_node[nodes]]
                Wh = W[self.H_node[nodes]]
                rows_b = (3 * (self.trip_start[hn] + self.slot_b[hn]))[:, None] + np.arange(3)[None, :]
                rr = np.concatenate([rows_u.reshape(-1), rows_b.reshape(-1)])
                vv = np.concatenate([(Hs[:, None, None] * W).reshape(-1, 6), Wh.reshape(-1, 6)])
                groups.append(("heaviside", rr, vv))
            if enriched and self.T_node[nodes].any():
                tn = nodes[self.T_node[nodes]]
                Wt = W[self.T_node[nodes]]
                for j in range(4):
                    rows_c = (3 * (self.trip_start[tn] + self.slot_c[tn] + j))[:, None] + np.arange(3)[None, :]
                    groups.append(("tip", rows_c.reshape(-1), Wt.reshape(-1, 6)))
            # select independent columns across all groups of the subdomain, in order
            # (standard modes first, then Heaviside, then each branch function)
            allrows = np.unique(np.concatenate([g[1] for g in groups]))
            dense = np.zeros((len(allrows), 6 * len(groups)))
            for gi, (kind, rr, vv) in enumerate(groups):
                dense[np.searchsorted(allrows, rr), 6 * gi:6 * gi + 6] = vv
            keep = self._independent_columns(dense, drop_tol)
            for gi, (kind, rr, vv) in enumerate(groups):
                kept = [j - 6 * gi for j in keep if 6 * gi <= j < 6 * gi + 6]
                info["dropped"] += 6 - len(kept)
                info[kind] += len(kept)
                info["groups"].append((s, kind, len(kept)))
                for jj in kept:
                    nz = vv[:, jj] != 0.0
                    entries_r.append(rr[nz])
                    entries_c.append(np.full(int(nz.sum()), kcol, np.int64))
                    entries_v.append(vv[nz, jj])
                    kcol += 1
        r = np.concatenate(entries_r)
        cidx = np.concatenate(entries_c)
        v = np.concatenate(entries_v)
        order = np.lexsort((cidx, r))
        r, cidx, v = r[order], cidx[order], v[order]
        rowptr = np.zeros(self.n + 1, np.int64)
        np.add.at(rowptr, r + 1, 1)
        rowptr = np.cumsum(rowptr)
        info["k"] = kcol
        return rowptr, cidx.astype(np.int32), v, kcol, info

    @staticmethod
    def _independent_columns(V, tol):
        """Indices of the columns of V kept by in-order selection: a column is kept when
        its component orthogonal to the kept ones exceeds tol times its norm."""
        Q = np.zeros((V.shape[0], 0))
        keep = []
        for j in range(V.shape[1]):
            v = V[:, j].copy()
            nv = np.linalg.norm(v)
            if nv == 0.0:
                continue
            for _ in range(2):
                v -= Q @ (Q.T @ v)
            nr = np.linalg.norm(v)
            if nr > tol * nv:
                Q = np.concatenate([Q, (v / nr)[:, None]], 1)
                keep.append(j)
        return keep

    def nodal_blocks(self):
        sizes = 3 * self.ngroups[self.free]
        bp = np.zeros(len(sizes) + 1, np.int64)
        np.cumsum(sizes, out=bp[1:])
        return bp.astype(np.int32)


def bsr_to_csr(bptr, bcol, bval):
    """Scalar CSR (rowptr int64, col int32, val f64) from 3x3 block CSR."""
    nb = len(bptr) - 1
    cnt = np.diff(bptr)
    rowlen = 3 * cnt
    rowptr = np.zeros(3 * nb + 1, np.int64)
    np.cumsum(np.repeat(rowlen, 3), out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz)
    brow = np.repeat(np.arange(nb), cnt)
    # position of block b's first scalar entry in scalar row 3R+i
    pos_in_row = (np.arange(len(bcol)) - bptr[brow]) * 3
    for i in range(3):
        base = rowptr[3 * brow + i] + pos_in_row
        for j in range(3):
            col[base + j] = 3 * bcol + j
            val[base + j] = bval[:, i, j]
    return rowptr, col, val


def build_problem(name, ne, nsd, crack=None, r_e=0.0, E=1.0, nu=0.3, clamp_bottom=True,
                  enriched_deflation=True, elem_E=None, min_split_frac=1e-3, tip=True,
                  load=True) -> Problem:
    box = XfemBox(ne, crack=crack, r_e=r_e, E=E, nu=nu, clamp_bottom=clamp_bottom,
                  elem_E=elem_E, min_split_frac=min_split_frac, tip=tip)
    bptr, bcol, bval = box.assemble_bsr()
    rowptr, col, val = bsr_to_csr(bptr, bcol, bval)
    f = box.loads() if load else np.zeros(box.n)
    zr, zc, zv, k, zinfo = box.deflation(nsd, enriched=enriched_deflation)
    blocks = box.nodal_blocks()
    sizes = np.diff(blocks)
    meta = {
        "ne": ne, "nsd": nsd, "nodes": int(box.n1 ** 3), "free_nodes": int(box.free.sum()),
        "n_std": int(3 * box.free.sum()), "n_enr": int(box.n - 3 * box.free.sum()),
        "nnzb": int(len(bcol)), "jump_nodes": int(box.H_node.sum()), "tip_nodes": int(box.T_node.sum()),
        "block_hist": {int(b): int((sizes == b).sum()) for b in np.unique(sizes)},
        "k_std": zinfo["std"], "k_heaviside": zinfo["heaviside"], "k_tip": zinfo["tip"],
        "k_dropped": zinfo["dropped"], "nnz_z": int(len(zv)),
        "enriched_elements": int(len(box.enriched_elements())),
    }
    return Problem(name=name, n=box.n, k_rowptr=rowptr, k_col=col, k_val=val, f=f,
                   z_rowptr=zr, z_col=zc, z_val=zv, k=k, block_ptr=blocks, meta=meta)

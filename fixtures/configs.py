"""Named synthetic workloads and a small on-disk cache.

The three plain-FP64 workloads are structured hex8 meshes of the unit cube
(E = 1, nu = 0.3, bottom face z = 0 clamped, unit +z traction on the top face):

* ``edge10``   10^3 elements, planar edge crack in x = 0.5 for z < 0.45 across the
               full width, Heaviside + 4 shifted branch functions within r_e = 0.15,
               2^3 subdomains.
* ``penny40``  40^3 elements, penny crack of radius 0.25 centred at (0.5,0.5,0.5)
               bent into z = 0.5 + 0.3 rho^2, tip enrichment within r_e = 0.05,
               4^3 subdomains.
* ``penny80``  80^3 elements, same crack, 8^3 subdomains.
* ``penny60``  60^3 elements, same crack, 6^3 subdomains (the adjoint workload, with
               per-element moduli E_e = exp(0.5 g_e), g a seeded N(0, 1) field).

They stand in for the paper's gmsh tetrahedral meshes (notched beam, bracket,
blade), which are not available; sizes per subdomain (about 3.3k DoFs) sit inside
the paper's range of DoFs per subdomain.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .xfem import CurvedPennyCrack, PlanarEdgeCrack, Problem, XfemBox, build_problem

GENERATOR_VERSION = 4

CONFIGS = {
    "edge10": dict(ne=10, nsd=2, crack=("edge", dict(x0=0.5, zf=0.45)), r_e=0.15),
    "penny40": dict(ne=40, nsd=4, crack=("penny", dict(center=(0.5, 0.5, 0.5), R=0.25, curv=0.3)), r_e=0.05),
    "penny80": dict(ne=80, nsd=8, crack=("penny", dict(center=(0.5, 0.5, 0.5), R=0.25, curv=0.3)), r_e=0.05),
    "penny60": dict(ne=60, nsd=6, crack=("penny", dict(center=(0.5, 0.5, 0.5), R=0.25, curv=0.3)), r_e=0.05),
    # small cases for tests: several tiles and ragged tails, fast to generate
    "edge4": dict(ne=4, nsd=2, crack=("edge", dict(x0=0.5, zf=0.45)), r_e=0.3),
    "penny12": dict(ne=12, nsd=2, crack=("penny", dict(center=(0.5, 0.5, 0.5), R=0.25, curv=0.3)), r_e=0.1),
    "plain6": dict(ne=6, nsd=2, crack=None, r_e=0.0),
}


def make_crack(spec):
    if spec is None:
        return None
    kind, kw = spec
    if kind == "edge":
        return PlanarEdgeCrack(**kw)
    if kind == "penny":
        return CurvedPennyCrack(**kw)
    raise ValueError(kind)


def cache_dir():
    d = os.environ.get("DPCG_FIXTURE_CACHE")
    if not d:
        d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _key(name, cfg):
    blob = json.dumps({"v": GENERATOR_VERSION, "name": name, "cfg": cfg}, sort_keys=True, default=str)
    return hashlib.sha1(blob.encode()).hexdigest()[:12]


def load(name: str, use_cache: bool = True) -> Problem:
    cfg = CONFIGS[name]
    path = os.path.join(cache_dir(), f"{name}-{_key(name, cfg)}.npz")
    if use_cache and os.path.exists(path):
        d = np.load(path, allow_pickle=False)
        meta = json.loads(str(d["meta"]))
        meta["block_hist"] = {int(b): c for b, c in meta["block_hist"].items()}
        return Problem(name=name, n=int(d["n"]), k_rowptr=d["k_rowptr"], k_col=d["k_col"],
                       k_val=d["k_val"], f=d["f"], z_rowptr=d["z_rowptr"], z_col=d["z_col"],
                       z_val=d["z_val"], k=int(d["k"]), block_ptr=d["block_ptr"], meta=meta)
    p = build_problem(name, cfg["ne"], cfg["nsd"], crack=make_crack(cfg["crack"]), r_e=cfg["r_e"])
    p.meta["config_hash"] = _key(name, cfg)
    if use_cache:
        tmp = path + ".tmp.npz"
        np.savez(tmp, n=p.n, k_rowptr=p.k_rowptr, k_col=p.k_col, k_val=p.k_val, f=p.f,
                 z_rowptr=p.z_rowptr, z_col=p.z_col, z_val=p.z_val, k=p.k, block_ptr=p.block_ptr,
                 meta=json.dumps(p.meta))
        os.replace(tmp, path)
    return p


def box(name: str, elem_E=None) -> XfemBox:
    """The mesh object of a named workload (optionally with per-element moduli)."""
    cfg = CONFIGS[name]
    return XfemBox(cfg["ne"], crack=make_crack(cfg["crack"]), r_e=cfg["r_e"], elem_E=elem_E)


def load_elements(name: str, use_cache: bool = True):
    """Unit-modulus element matrices of a named workload (XfemBox.element_matrices)."""
    cfg = CONFIGS[name]
    path = os.path.join(cache_dir(), f"{name}-{_key(name, cfg)}-elements.npz")
    if use_cache and os.path.exists(path):
        d = np.load(path, allow_pickle=False)
        return d["elem_ptr"], d["elem_dof"], d["kmat_off"], d["kmat"]
    ep, ed, ko, km = box(name).element_matrices()
    if use_cache:
        tmp = path + ".tmp.npz"
        np.savez(tmp, elem_ptr=ep, elem_dof=ed, kmat_off=ko, kmat=km)
        os.replace(tmp, path)
    return ep, ed, ko, km


def problem_with_moduli(name: str, elem_E) -> Problem:
    """The named workload re-assembled with per-element Young's moduli elem_E."""
    cfg = CONFIGS[name]
    return build_problem(name, cfg["ne"], cfg["nsd"], crack=make_crack(cfg["crack"]), r_e=cfg["r_e"],
                         elem_E=np.asarray(elem_E, float))


def log_normal_moduli(name: str, seed: int = 7, sigma: float = 0.5):
    """Per-element Young's moduli E_e = exp(sigma g_e), g i.i.d. N(0, 1) (seeded)."""
    nel = CONFIGS[name]["ne"] ** 3
    return np.exp(sigma * np.random.default_rng(seed).standard_normal(nel))


def uneven_specs(count: int = 16, seed: int = 16, ne_range=(20, 48)):
    """(ne, crack centre) of each system of the multi-system workload, in draw order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ne = int(rng.integers(ne_range[0], ne_range[1] + 1))
        centre = tuple(float(v) for v in rng.uniform(0.3, 0.7, 3))
        out.append((ne, centre))
    return out


def uneven_systems(count: int = 16, seed: int = 16, ne_range=(20, 48), r_e: float = 0.05, which=None):
    """Independent systems of the multi-system workload: meshes of ne^3 elements with ne
    uniform in ne_range, each with a curved penny crack (radius 0.25, curvature 0.3)
    whose centre is uniform in [0.3, 0.7]^3, 1 + ne // 12 subdomains per axis.
    which: indices of the systems to build (default all; the draws of the others are
    still taken, so system i is the same either way).  Returns a list of Problems (not
    cached)."""
    specs = uneven_specs(count, seed, ne_range)
    out = []
    for i in (range(count) if which is None else which):
        ne, centre = specs[i]
        crack = CurvedPennyCrack(center=centre, R=0.25, curv=0.3)
        out.append(build_problem(f"uneven{i}", ne, 1 + ne // 12, crack=crack, r_e=r_e))
    return out


def subdomain_order(bx: XfemBox, nsd: int):
    """DoF permutation that numbers the unknowns subdomain by subdomain (nsd^3 boxes of
    nodes, XfemBox.subdomain_of_nodes; a node's DoFs stay together and in order) and the
    block partition with one block per non-empty subdomain: the subdomain-sized
    block-Jacobi blocks of Sec. 3.4.  Returns (perm int64, block_ptr int32) with new
    unknown i = old unknown perm[i]."""
    sd = bx.subdomain_of_nodes(nsd)
    nodes = np.nonzero(bx.ngroups > 0)[0]
    order = nodes[np.argsort(sd[nodes], kind="stable")]
    starts = 3 * bx.trip_start[order]
    lens = 3 * bx.ngroups[order]
    offs = np.zeros(len(order) + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    perm = np.repeat(starts - offs[:-1], lens) + np.arange(offs[-1])
    sizes = np.bincount(sd[order], weights=lens, minlength=nsd ** 3).astype(np.int64)
    sizes = sizes[sizes > 0]
    bp = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=bp[1:])
    return perm.astype(np.int64), bp.astype(np.int32)


def permuted(p: Problem, perm, block_ptr, name=None) -> Problem:
    """P K P^T, P f, P Z for the permutation perm (new i = old perm[i]) with a new block
    partition; columns sorted in every row."""
    K = p.K_scipy()[perm][:, perm].tocsr()
    K.sort_indices()
    Z = p.Z_scipy()[perm].tocsr()
    Z.sort_indices()
    meta = dict(p.meta)
    meta["perm"] = "subdomain"
    return Problem(name=name or p.name, n=p.n, k_rowptr=K.indptr.astype(np.int64), k_col=K.indices.astype(np.int32),
                   k_val=K.data.astype(np.float64), f=np.ascontiguousarray(p.f[perm]),
                   z_rowptr=Z.indptr.astype(np.int64), z_col=Z.indices.astype(np.int32),
                   z_val=Z.data.astype(np.float64), k=p.k, block_ptr=np.asarray(block_ptr, np.int32), meta=meta)


def with_subdomain_blocks(name: str, nsd: int, p: Problem | None = None):
    """The named workload (or p, a problem on the same mesh) renumbered subdomain by
    subdomain with one block-Jacobi block per subdomain of an nsd^3 box partition.
    Returns (problem, perm)."""
    p = load(name) if p is None else p
    perm, bp = subdomain_order(box(name), nsd)
    return permuted(p, perm, bp, name=f"{name}-sd{nsd}"), perm

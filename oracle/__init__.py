"""ORACLE — test infrastructure only.

Python access (ctypes + numpy) to the plain FP64 CPU oracle in ``ogo_tree.c``
(octree build and per-target walk of the short-range TreePM force) and
``ogo_direct.c`` (brute-force direct sum).  Only ``tests/``, the smoke entry
and the benchmark's CPU-baseline leg may import this package.  It imports
nothing from the HIP package, and the HIP package imports nothing from it.

Parameters follow the paper's notation ("Gravity Solver" section): G, the
Plummer(-equivalent) softening ``eps``, the split scale ``r_s`` (the paper's
A_smth), the cutoff ``r_cut`` (0 means 4.5 r_s), the opening angle
``theta``, the leaf size ``leaf_max``, the ``periodic`` flag, the softening
kernel (``softening``: 0 Plummer, 1 cubic spline of support 2.8 eps, paper
"Force evaluation") and the opening criterion (``criterion``: 0 Barnes-Hut,
1 relative with tolerance ``alpha`` against the previous acceleration, paper
"Tree walk").
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        I = ctypes.c_int
        lib.ogo_frame.argtypes = [P, I64, D, I, P, P]
        lib.ogo_frame.restype = I
        lib.ogo_keys.argtypes = [P, I64, P, D, I, P]
        lib.ogo_keys.restype = None
        lib.ogo_sort.argtypes = [P, I64, P]
        lib.ogo_sort.restype = None
        lib.ogo_topology.argtypes = [P, I64, I, I64, P, P, P, P, P]
        lib.ogo_topology.restype = I64
        lib.ogo_node_centres.argtypes = [P, I64, P, P, P, D, P, P]
        lib.ogo_node_centres.restype = None
        lib.ogo_moments.argtypes = [P, P, I64, P, P, P, P, P]
        lib.ogo_moments.restype = None
        lib.ogo_walk.argtypes = [P, P, I64, P, P, P, P, P, P, P, P, I,
                                 D, D, D, D, D, I, D, I, I, D, P, P, P, I64, P, P, P]
        lib.ogo_walk.restype = None
        lib.ogo_walk_groups.argtypes = [P, P, I64, P, P, P, P, P, P, P, P, I,
                                        D, D, D, D, D, I, D, I, I, D, P, P, P, P, I64, P, P, P]
        lib.ogo_walk_groups.restype = None
        lib.ogo_direct.argtypes = [P, P, I64, D, I, D, D, D, D, I, P, P, I64, P, P, P]
        lib.ogo_direct.restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Params:
    G: float = 1.0
    eps: float = 0.0
    r_s: float = 0.0
    r_cut: float = 0.0
    theta: float = 0.5
    periodic: int = 1
    leaf_max: int = 8
    softening: int = 0      # 0 Plummer, 1 cubic spline (support 2.8 eps)
    curve: int = 0          # 0 Morton, 1 Peano-Hilbert
    criterion: int = 0      # 0 Barnes-Hut (theta), 1 relative (alpha, a_old)
    alpha: float = 0.0

    @property
    def rcut(self) -> float:
        """Cutoff actually used: r_cut, or 4.5 r_s when r_cut is 0."""
        return self.r_cut if self.r_cut > 0 else 4.5 * self.r_s


class OracleError(ValueError):
    pass


@dataclass
class Tree:
    lo: np.ndarray          # root cube lower corner [3]
    L: float                # root cube side
    keys: np.ndarray        # uint64 [N], caller order
    perm: np.ndarray        # uint32 [N], sorted position -> caller index
    skeys: np.ndarray       # uint64 [N], sorted
    first: np.ndarray       # uint32 [n_nodes]
    count: np.ndarray       # uint32 [n_nodes]
    level: np.ndarray       # uint8  [n_nodes]
    skip: np.ndarray        # uint32 [n_nodes]
    parent: np.ndarray      # uint32 [n_nodes] (root: 0xffffffff)
    centre: np.ndarray      # float64 [n_nodes, 3]
    side: np.ndarray        # float64 [n_nodes]
    mass: np.ndarray        # float64 [n_nodes]
    com: np.ndarray         # float64 [n_nodes, 3]
    spos: np.ndarray        # float64 [N, 3], sorted
    smass: np.ndarray       # float64 [N], sorted
    box: float
    params: Params
    seps: np.ndarray = None  # float64 [N], sorted per-particle softening (R32), or None

    @property
    def n_nodes(self) -> int:
        return int(self.first.shape[0])

    @property
    def is_leaf(self) -> np.ndarray:
        return ~((self.count > self.params.leaf_max) & (self.level < 21))


def node_bound(n: int, leaf_max: int) -> int:
    """Upper bound on the node count: at most n leaves, and at most
    n/(leaf_max+1) internal nodes on each of the 21 splitting levels."""
    return int(n + 21 * (n // (leaf_max + 1)) + 1)


def frame(pos, box, periodic):
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    lo = np.zeros(3)
    L = np.zeros(1)
    rc = lib.ogo_frame(_p(pos), pos.shape[0], float(box), int(periodic), _p(lo), _p(L))
    if rc != 0:
        raise OracleError("position outside the periodic box or not finite")
    return lo, float(L[0])


def keys(pos, box, periodic=1, curve=0):
    """Curve keys (uint64, caller order) of the positions: Morton (curve 0)
    or Peano-Hilbert (curve 1)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    lo, L = frame(pos, box, periodic)
    k = np.empty(pos.shape[0], dtype=np.uint64)
    lib.ogo_keys(_p(pos), pos.shape[0], _p(lo), L, int(curve), _p(k))
    return k


def build_tree(pos, mass, box, params: Params, eps=None) -> Tree:
    """Octree of the particles; `eps` optionally gives every particle's own
    softening length (caller order, R32)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if n < 1:
        raise OracleError("empty particle set")
    lo, L = frame(pos, box, params.periodic)
    k = np.empty(n, dtype=np.uint64)
    lib.ogo_keys(_p(pos), n, _p(lo), L, int(params.curve), _p(k))
    perm = np.empty(n, dtype=np.uint32)
    lib.ogo_sort(_p(k), n, _p(perm))
    skeys = np.ascontiguousarray(k[perm])
    cap = node_bound(n, params.leaf_max)
    first = np.empty(cap, dtype=np.uint32)
    count = np.empty(cap, dtype=np.uint32)
    level = np.empty(cap, dtype=np.uint8)
    skip = np.empty(cap, dtype=np.uint32)
    parent = np.empty(cap, dtype=np.uint32)
    nn = lib.ogo_topology(_p(skeys), n, int(params.leaf_max), cap, _p(first), _p(count),
                          _p(level), _p(skip), _p(parent))
    if nn < 0:
        raise OracleError("node bound exceeded")
    first, count, level, skip, parent = (a[:nn].copy() for a in (first, count, level, skip, parent))
    spos = np.ascontiguousarray(pos[perm])
    centre = np.empty((nn, 3))
    side = np.empty(nn)
    lib.ogo_node_centres(_p(spos), nn, _p(first), _p(level), _p(lo), L, _p(centre), _p(side))
    smass = np.ascontiguousarray(mass[perm])
    nmass = np.empty(nn)
    com = np.empty((nn, 3))
    lib.ogo_moments(_p(spos), _p(smass), nn, _p(first), _p(count), _p(centre), _p(nmass), _p(com))
    seps = None
    if eps is not None:
        eps = np.asarray(eps, dtype=np.float64)
        if eps.shape != (n,) or not np.all(eps > 0):
            raise OracleError("eps must hold one positive length per particle")
        seps = np.ascontiguousarray(eps[perm])
    return Tree(lo, L, k, perm, skeys, first, count, level, skip, parent, centre, side,
                nmass, com, spos, smass, float(box), params, seps)


def walk(tree: Tree, targets=None, params: Params = None, a_old=None):
    """Tree walk for caller-order target indices (None = all).  With the
    relative criterion, ``a_old`` holds every particle's previous
    acceleration [N,3] in caller order.
    Returns (acc [M,3], pot [M], n_interactions [M]) in target order."""
    lib = _load()
    p = params or tree.params
    if p.softening == 1 and not p.eps > 0 and tree.seps is None:
        raise OracleError("spline softening needs eps > 0")
    n = tree.spos.shape[0]
    inv = np.empty(n, dtype=np.uint32)
    inv[tree.perm] = np.arange(n, dtype=np.uint32)
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    tpos = np.ascontiguousarray(inv[targets])
    M = tpos.shape[0]
    if p.criterion == 1:
        if a_old is None:
            raise OracleError("the relative criterion needs a_old")
        aold = np.ascontiguousarray(np.asarray(a_old, dtype=np.float64).reshape(n, 3)[targets])
    else:
        aold = np.zeros((1, 3))
    acc = np.empty((M, 3))
    pot = np.empty(M)
    nint = np.empty(M, dtype=np.int64)
    lib.ogo_walk(_p(tree.spos), _p(tree.smass), tree.n_nodes, _p(tree.first), _p(tree.count),
                 _p(tree.level), _p(tree.skip), _p(tree.centre), _p(tree.side), _p(tree.mass),
                 _p(tree.com), int(tree.params.leaf_max), float(p.G), float(p.eps), float(p.r_s),
                 float(p.rcut), float(p.theta), int(p.periodic), float(tree.box),
                 int(p.softening), int(p.criterion), float(p.alpha), _p(aold),
                 None if tree.seps is None else _p(tree.seps), _p(tpos), M,
                 _p(acc), _p(pot), _p(nint))
    return acc, pot, nint


def curve_groups(tree: Tree, group_size: int, targets=None):
    """Partition of the targets (caller-order indices, None = all) into
    groups of `group_size` consecutive targets in the tree's curve order
    (ties between repeated targets kept in list order).  Returns (order,
    goff): order[k] is the position in the target list of the k-th target
    in curve order; group g is order[goff[g]:goff[g+1]]."""
    n = tree.spos.shape[0]
    inv = np.empty(n, dtype=np.int64)
    inv[tree.perm] = np.arange(n)
    tl = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    order = np.argsort(inv[tl], kind="stable")
    M = len(tl)
    goff = np.append(np.arange(0, M, group_size), M).astype(np.int64)
    return order, goff


def walk_groups(tree: Tree, group_size: int, targets=None, params: Params = None, a_old=None):
    """Group-shared walk (R31) over the curve-order partition of
    `curve_groups`.  Returns (acc, pot, n_interactions) in target order."""
    lib = _load()
    p = params or tree.params
    if p.softening == 1 and not p.eps > 0 and tree.seps is None:
        raise OracleError("spline softening needs eps > 0")
    n = tree.spos.shape[0]
    inv = np.empty(n, dtype=np.uint32)
    inv[tree.perm] = np.arange(n, dtype=np.uint32)
    tl = np.arange(n, dtype=np.int64) if targets is None else np.asarray(targets, dtype=np.int64)
    order, goff = curve_groups(tree, group_size, tl)
    tsorted = tl[order]
    tpos = np.ascontiguousarray(inv[tsorted])
    M = len(tl)
    if p.criterion == 1:
        if a_old is None:
            raise OracleError("the relative criterion needs a_old")
        aold = np.ascontiguousarray(np.asarray(a_old, dtype=np.float64).reshape(n, 3)[tsorted])
    else:
        aold = np.zeros((1, 3))
    acc = np.empty((M, 3))
    pot = np.empty(M)
    nint = np.empty(M, dtype=np.int64)
    lib.ogo_walk_groups(_p(tree.spos), _p(tree.smass), tree.n_nodes, _p(tree.first), _p(tree.count),
                        _p(tree.level), _p(tree.skip), _p(tree.centre), _p(tree.side), _p(tree.mass),
                        _p(tree.com), int(tree.params.leaf_max), float(p.G), float(p.eps), float(p.r_s),
                        float(p.rcut), float(p.theta), int(p.periodic), float(tree.box),
                        int(p.softening), int(p.criterion), float(p.alpha), _p(aold),
                        None if tree.seps is None else _p(tree.seps), _p(tpos),
                        _p(goff), len(goff) - 1, _p(acc), _p(pot), _p(nint))
    out_a = np.empty_like(acc)
    out_p = np.empty_like(pot)
    out_n = np.empty_like(nint)
    out_a[order] = acc
    out_p[order] = pot
    out_n[order] = nint
    return out_a, out_p, out_n


def tree_force(pos, mass, box, params: Params, targets=None, a_old=None, eps=None):
    """Build + walk.  Returns (acc, pot, n_interactions) in target order."""
    return walk(build_tree(pos, mass, box, params, eps=eps), targets, params, a_old)


def direct(pos, mass, box, params: Params, targets=None, eps=None):
    """Brute-force direct sum (exact short-range force).  Returns
    (acc [M,3], pot [M], n_interactions [M]) in target order."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    M = targets.shape[0]
    acc = np.empty((M, 3))
    pot = np.empty(M)
    nint = np.empty(M, dtype=np.int64)
    if params.softening == 1 and not params.eps > 0 and eps is None:
        raise OracleError("spline softening needs eps > 0")
    peps = None
    if eps is not None:
        peps = np.ascontiguousarray(eps, dtype=np.float64)
        if peps.shape != (n,) or not np.all(peps > 0):
            raise OracleError("eps must hold one positive length per particle")
    lib.ogo_direct(_p(pos), _p(mass), n, float(box), int(params.periodic), float(params.G),
                   float(params.eps), float(params.r_s), float(params.rcut),
                   int(params.softening), None if peps is None else _p(peps), _p(targets), M,
                   _p(acc), _p(pot), _p(nint))
    return acc, pot, nint

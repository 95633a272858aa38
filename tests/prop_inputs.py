"""Hypothesis strategies for small particle configurations, shared by the
oracle's and the GPU path's property tests.  Inputs only: positions,
masses and parameters, no part of the force computation.

A configuration mixes uniform particles with the cases that stress a tree
code: coincident particles (finest-level leaves larger than leaf_max),
coordinates on dyadic cell faces (exactly on a split plane), coordinates at
the periodic wrap (0 and the largest double below the box side), and leaf
sizes from 1 up; boxes are periodic with a cutoff or open (Newtonian or with
a cutoff), of side 1 or 3, with Morton or Hilbert keys."""
from dataclasses import dataclass

import numpy as np
from hypothesis import strategies as st


@dataclass
class Config:
    pos: np.ndarray
    mass: np.ndarray
    box: float
    params: dict
    label: str

    def __repr__(self):
        return self.label


@st.composite
def configs(draw, max_n=160):
    n = draw(st.integers(1, max_n))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    periodic = draw(st.booleans())
    box = draw(st.sampled_from([1.0, 3.0]))
    n_dup = draw(st.integers(0, n // 3))
    n_face = draw(st.integers(0, n // 3))
    n_wrap = draw(st.integers(0, n // 4)) if periodic else 0
    theta = draw(st.sampled_from([0.0, 0.3, 0.5, 0.8]))
    leaf_max = draw(st.sampled_from([1, 2, 8, 16]))
    curve = draw(st.sampled_from([0, 1]))
    newtonian = (not periodic) and draw(st.booleans())
    clustered = draw(st.booleans())

    rng = np.random.default_rng(seed)
    if clustered:
        c = rng.random(3) * box
        pos = c + 0.03 * box * rng.standard_normal((n, 3))
        if periodic:
            pos = np.mod(pos, box)
    else:
        pos = rng.random((n, 3)) * box
    if not periodic:
        pos = pos * rng.uniform(0.5, 2.0) - rng.uniform(0.0, 1.0)
    idx = rng.permutation(n)
    face = idx[:n_face]
    ax = rng.integers(0, 3, n_face)
    m = rng.integers(1, 8, n_face)
    k = rng.integers(0, 2 ** m)
    pos[face, ax] = box * k / 2.0 ** m if periodic else pos[face, ax].round(2)
    if n_wrap:
        wr = idx[n_face:n_face + n_wrap]
        axw = rng.integers(0, 3, n_wrap)
        pos[wr, axw] = np.where(rng.random(n_wrap) < 0.5, 0.0, np.nextafter(box, 0.0))
    if n_dup and n > 1:
        src = rng.integers(0, n, n_dup)
        dst = rng.integers(0, n, n_dup)
        pos[dst] = pos[src]
    if periodic:
        pos = np.where(pos >= box, np.nextafter(box, 0.0), pos)
        pos = np.where(pos < 0.0, 0.0, pos)
    mass = rng.uniform(0.5, 1.5, n) / n
    if newtonian:
        prm = dict(G=1.0, eps=0.01 * box, r_s=0.0, r_cut=0.0)
    else:
        r_s = 0.04 * box
        prm = dict(G=1.0, eps=0.002 * box, r_s=r_s, r_cut=4.5 * r_s)
    prm.update(theta=theta, periodic=int(periodic), leaf_max=leaf_max, curve=curve)
    label = ("n=%d seed=%d periodic=%d box=%g dup=%d face=%d wrap=%d theta=%g leaf=%d curve=%d newt=%d clus=%d"
             % (n, seed, periodic, box, n_dup, n_face, n_wrap, theta, leaf_max, curve, newtonian, clustered))
    return Config(np.ascontiguousarray(pos, dtype=np.float64), mass, box, prm, label)


def oracle_params(oracle_mod, prm, **kw):
    d = dict(prm, **kw)
    return oracle_mod.Params(**{k: d[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic",
                                                  "leaf_max", "curve") if k in d})

"""Pins of per-particle softening lengths and the mixed-softening check
(paper, "Tree walk": extra checks where gravitational softenings differ).

Reading: a pair is softened with the larger of its two lengths; a node's
monopole with the larger of the target's and the node's largest; a node
holding different lengths whose largest exceeds the target's is opened when
the target lies within 2.8 times that largest length of its centre of mass.
Pins: equal lengths reproduce the single-length results bit for bit; the
two-body closed form with the larger length; Newton's third law of the
direct sum (the pair rule is symmetric); theta = 0 reproduces the direct sum
(written separately) for both kernels; the check opens nodes for a target
with a small length and not for one with a large length at the same place.
"""
import math

import numpy as np
import pytest

from paper_2609_17658_amd import synth


def _mixed_eps(n, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(n) < 0.3, 0.004, 0.0008) * rng.uniform(0.8, 1.2, n)


def test_equal_lengths_reproduce_single_length(oracle_mod):
    w = synth.mixture32k()
    p = oracle_mod.Params(**w.params.as_dict())
    tg = np.arange(0, w.pos.shape[0], 9)
    eps = np.full(w.pos.shape[0], p.eps)
    for soft in (0, 1):
        q = oracle_mod.Params(**{**w.params.as_dict(), "softening": soft})
        a, pot, n = oracle_mod.tree_force(w.pos, w.mass, 1.0, q, targets=tg)
        ae, pote, ne = oracle_mod.tree_force(w.pos, w.mass, 1.0, q, targets=tg, eps=eps)
        assert np.array_equal(a, ae) and np.array_equal(pot, pote) and np.array_equal(n, ne)
        ad, _, _ = oracle_mod.direct(w.pos, w.mass, 1.0, q, targets=tg)
        ade, _, _ = oracle_mod.direct(w.pos, w.mass, 1.0, q, targets=tg, eps=eps)
        assert np.array_equal(ad, ade)


def test_two_body_uses_the_larger_length(oracle_mod):
    G, m1, m2, e1, e2 = 1.0, 0.4, 0.9, 0.01, 0.05
    pos = np.array([[0.1, 0.2, 0.3], [0.13, 0.18, 0.31]])
    d = pos[1] - pos[0]
    r2 = d @ d
    a1 = G * m2 * d / (r2 + e2 * e2) ** 1.5
    p = oracle_mod.Params(G=G, eps=0.0, r_s=0.0, periodic=0, theta=0.5, leaf_max=1)
    for fn in (oracle_mod.direct, oracle_mod.tree_force):
        acc, pot, _ = fn(pos, np.array([m1, m2]), 1.0, p, eps=np.array([e1, e2]))
        assert np.allclose(acc[0], a1, rtol=1e-14, atol=0)
        assert math.isclose(pot[0], -G * m2 / math.sqrt(r2 + e2 * e2), rel_tol=1e-14)


def test_direct_sum_conserves_momentum(oracle_mod):
    rng = np.random.default_rng(4)
    n = 500
    pos = synth.wrap(0.5 + 0.05 * rng.standard_normal((n, 3)))
    mass = rng.uniform(0.5, 2.0, n) / n
    for soft in (0, 1):
        p = oracle_mod.Params(eps=0.001, r_s=0.03, periodic=1, softening=soft)
        acc, _, _ = oracle_mod.direct(pos, mass, 1.0, p, eps=_mixed_eps(n, 5))
        mom = (mass[:, None] * acc).sum(0)
        assert np.abs(mom).max() <= 1e-14 * (mass * np.linalg.norm(acc, axis=1)).sum()


@pytest.mark.parametrize("soft", [0, 1])
def test_theta_zero_reproduces_direct_sum(oracle_mod, soft):
    w = synth.mixture32k()
    eps = _mixed_eps(w.pos.shape[0], 6)
    p = oracle_mod.Params(**{**w.params.as_dict(), "theta": 0.0, "softening": soft})
    tg = np.arange(0, w.pos.shape[0], 11)
    a, pot, n = oracle_mod.tree_force(w.pos, w.mass, 1.0, p, targets=tg, eps=eps)
    ad, potd, nd = oracle_mod.direct(w.pos, w.mass, 1.0, p, targets=tg, eps=eps)
    assert (np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)).max() <= 1e-13
    assert np.abs(pot - potd).max() <= 1e-13 * np.abs(potd).max()
    assert np.array_equal(n, nd)


def test_mixed_softening_check_opens_for_small_lengths(oracle_mod):
    """A clump of particles with large lengths and a few with small ones; two
    coincident targets beside it, one with a small length, one with a large
    one.  With a wide opening angle only the check (and the boundary test)
    opens nodes: the small-length target interacts with more partners."""
    rng = np.random.default_rng(8)
    clump = 0.5 + 0.004 * rng.standard_normal((400, 3))
    pos = np.concatenate([clump, [[0.515, 0.5, 0.5], [0.515, 0.5, 0.5]]])
    n = pos.shape[0]
    eps = np.full(n, 0.01)
    eps[rng.choice(400, 20, replace=False)] = 0.0005
    eps[400] = 0.0005   # small-length target
    mass = np.full(n, 1.0 / n)
    p = oracle_mod.Params(G=1.0, eps=0.0, r_s=0.0, periodic=0, theta=5.0, leaf_max=4)
    a, pot, nint = oracle_mod.tree_force(pos, mass, 1.0, p, targets=[400, 401], eps=eps)
    assert nint[0] > 2 * nint[1]
    # and it is the more accurate one against the direct sum
    ad, _, _ = oracle_mod.direct(pos, mass, 1.0, p, targets=[400, 401], eps=eps)
    e = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
    assert e[0] < 0.5 * e[1]

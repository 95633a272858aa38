"""Property tests of the oracle on hypothesis-drawn small configurations
(coincident particles, particles on cell faces and at the periodic wrap,
leaf sizes 1..16, open and periodic boxes, Morton and Hilbert keys):

  * the result does not depend on the order of the input particles: equal
    to the bit when all keys differ (the sorted order, hence the tree and
    every sum, is then the same), within rounding otherwise;
  * forces are linear in G and in the masses: scaling by powers of two
    scales every output exactly (opening decisions are geometric);
  * a walk over a subset of targets gives those targets' full-walk values
    to the bit (each target's walk is independent of the others);
  * with theta = 0 every node is opened: the tree walk is the direct sum
    over the same pairs (same interaction counts, values within rounding);
  * the built tree satisfies the structural invariants of the hierarchy.
"""
import numpy as np
from hypothesis import HealthCheck, given, settings

from prop_inputs import configs, oracle_params

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


def _scale(a):
    return max(float(np.abs(a).max()) if a.size else 0.0, 1e-300)


@SETTINGS
@given(cfg=configs())
def test_input_order_does_not_matter(oracle_mod, cfg):
    op = oracle_params(oracle_mod, cfg.params)
    acc, pot, nint = oracle_mod.tree_force(cfg.pos, cfg.mass, cfg.box, op)
    sig = np.random.default_rng(len(cfg.pos)).permutation(len(cfg.pos))
    acc2, pot2, nint2 = oracle_mod.tree_force(cfg.pos[sig], cfg.mass[sig], cfg.box, op)
    keys = oracle_mod.keys(cfg.pos, cfg.box, cfg.params["periodic"], cfg.params["curve"])
    if len(np.unique(keys)) == len(keys):
        assert np.array_equal(acc2, acc[sig]) and np.array_equal(pot2, pot[sig])
        assert np.array_equal(nint2, nint[sig])
    else:
        assert np.abs(acc2 - acc[sig]).max() <= 1e-12 * _scale(acc)
        assert np.abs(pot2 - pot[sig]).max() <= 1e-12 * _scale(pot)


@SETTINGS
@given(cfg=configs())
def test_linear_in_G_and_mass(oracle_mod, cfg):
    op = oracle_params(oracle_mod, cfg.params)
    acc, pot, nint = oracle_mod.tree_force(cfg.pos, cfg.mass, cfg.box, op)
    op4 = oracle_params(oracle_mod, cfg.params, G=4.0 * cfg.params["G"])
    acc8, pot8, nint8 = oracle_mod.tree_force(cfg.pos, 2.0 * cfg.mass, cfg.box, op4)
    assert np.array_equal(acc8, 8.0 * acc) and np.array_equal(pot8, 8.0 * pot)
    assert np.array_equal(nint8, nint)


@SETTINGS
@given(cfg=configs())
def test_subset_walk_equals_full_walk(oracle_mod, cfg):
    op = oracle_params(oracle_mod, cfg.params)
    tree = oracle_mod.build_tree(cfg.pos, cfg.mass, cfg.box, op)
    acc, pot, nint = oracle_mod.walk(tree)
    n = len(cfg.pos)
    tg = np.random.default_rng(n + 1).choice(n, size=max(1, n // 3), replace=False)
    a, p, c = oracle_mod.walk(tree, targets=tg)
    assert np.array_equal(a, acc[tg]) and np.array_equal(p, pot[tg]) and np.array_equal(c, nint[tg])


@SETTINGS
@given(cfg=configs())
def test_theta_zero_is_the_direct_sum(oracle_mod, cfg):
    op = oracle_params(oracle_mod, cfg.params, theta=0.0)
    acc, pot, nint = oracle_mod.tree_force(cfg.pos, cfg.mass, cfg.box, op)
    accd, potd, nintd = oracle_mod.direct(cfg.pos, cfg.mass, cfg.box, op)
    assert np.array_equal(nint, nintd)
    assert np.abs(acc - accd).max() <= 1e-11 * _scale(accd)
    assert np.abs(pot - potd).max() <= 1e-11 * _scale(potd)


@SETTINGS
@given(cfg=configs())
def test_tree_invariants(oracle_mod, cfg):
    op = oracle_params(oracle_mod, cfg.params)
    t = oracle_mod.build_tree(cfg.pos, cfg.mass, cfg.box, op)
    n, nn = len(cfg.pos), t.n_nodes
    assert np.all(t.skeys[1:] >= t.skeys[:-1])
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    assert t.first[0] == 0 and t.count[0] == n and t.level[0] == 0 and t.skip[0] == nn
    leaf = t.is_leaf
    for r in range(nn):
        if leaf[r]:
            assert t.skip[r] == r + 1
            continue
        kids, nxt = [], t.first[r]
        ch = r + 1
        while ch < t.skip[r]:
            assert t.parent[ch] == r and t.level[ch] == t.level[r] + 1 and t.first[ch] == nxt
            nxt += t.count[ch]
            kids.append(ch)
            ch = t.skip[ch]
        assert ch == t.skip[r] and 1 <= len(kids) <= 8 and nxt == t.first[r] + t.count[r]
        # children lie in distinct octants of the parent cube
        oct_ = {tuple((t.centre[c] > t.centre[r]).astype(int)) for c in kids}
        assert len(oct_) == len(kids)
        off = np.abs(t.centre[kids] - t.centre[r])
        assert np.all(np.abs(off - t.side[r] / 4) <= 1e-12 * (np.abs(t.centre[r]).max() + t.side[r]))
    # leaves tile the particles in order; mass is conserved
    lf = np.flatnonzero(leaf)
    assert np.array_equal(t.first[lf][1:], (t.first[lf] + t.count[lf])[:-1]) and t.count[lf].sum() == n
    assert abs(t.mass[0] - cfg.mass.sum()) <= 1e-13 * cfg.mass.sum()

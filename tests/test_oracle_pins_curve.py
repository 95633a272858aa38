"""Pins of the oracle's Peano-Hilbert keys (paper, "Tree construction" and
"Domain decomposition": particles are ordered along the Peano-Hilbert
curve).  What makes a Hilbert curve is checked directly, not its formula:
at every resolution the keys enumerate the cells once each and consecutive
keys are face-adjacent cells; every octree cell is one contiguous key range;
and the tree built on these keys has the same nodes (cells) as the Morton
tree, so the per-target forces agree up to summation order with identical
interaction counts."""
import numpy as np
import pytest

from paper_2609_17658_amd import synth


def _grid_centres(level, origin=(0, 0, 0), cells=None, depth=None):
    """Centres of the cells of a cubic block: `cells` per axis at `depth`
    (cell size 2^-depth), starting at integer cell `origin`."""
    depth = level if depth is None else depth
    cells = 2 ** level if cells is None else cells
    q = np.arange(cells)
    c = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3) + np.asarray(origin)
    return c, (c + 0.5) / 2.0 ** depth


def _assert_face_adjacent_path(cells_in_key_order):
    step = np.abs(np.diff(cells_in_key_order, axis=0)).sum(1)
    assert np.all(step == 1)


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_hilbert_enumerates_grid_as_adjacent_path(oracle_mod, level):
    cells, pos = _grid_centres(level)
    k = oracle_mod.keys(pos, 1.0, periodic=1, curve=1) >> np.uint64(3 * (21 - level))
    assert np.array_equal(np.sort(k), np.arange(8 ** level, dtype=np.uint64))
    _assert_face_adjacent_path(cells[np.argsort(k)])


def test_hilbert_starts_at_origin(oracle_mod):
    k = oracle_mod.keys(np.array([[0.0, 0.0, 0.0], [1e-9, 2e-9, 0.0]]), 1.0, periodic=1, curve=1)
    assert int(k[0]) == 0


@pytest.mark.parametrize("depth", [12, 21])
def test_hilbert_deep_blocks_are_adjacent_key_ranges(oracle_mod, depth):
    """A 4x4x4 block of cells at `depth` aligned to a cell of depth-2 gets
    64 consecutive keys forming a face-adjacent path."""
    rng = np.random.default_rng(depth)
    for _ in range(20):
        origin = rng.integers(0, 2 ** (depth - 2), 3) * 4
        cells, pos = _grid_centres(None, origin=origin, cells=4, depth=depth)
        k = oracle_mod.keys(pos, 1.0, periodic=1, curve=1) >> np.uint64(3 * (21 - depth))
        ks = np.sort(k)
        assert int(ks[-1] - ks[0]) == 63 and int(ks[0]) % 64 == 0
        _assert_face_adjacent_path(cells[np.argsort(k)])


def test_hilbert_octree_cells_are_key_prefixes(oracle_mod):
    rng = np.random.default_rng(4)
    pos = rng.random((20000, 3))
    k = oracle_mod.keys(pos, 1.0, periodic=1, curve=1)
    for level in (1, 3, 7, 12, 21):
        cell = np.floor(pos * 2 ** level).astype(np.int64)
        cid = (cell[:, 0] << 42) | (cell[:, 1] << 21) | cell[:, 2]
        pre = (k >> np.uint64(3 * (21 - level))).astype(np.int64)
        # same cell <=> same prefix
        pairs = np.unique(np.stack([cid, pre], 1), axis=0)
        assert len(pairs) == len(np.unique(cid)) == len(np.unique(pre))


def test_hilbert_tree_has_morton_nodes_and_forces(oracle_mod):
    w = synth.mixture32k()
    out = {}
    for curve in (0, 1):
        p = oracle_mod.Params(**{**w.params.as_dict(), "curve": curve})
        tr = oracle_mod.build_tree(w.pos, w.mass, w.box, p)
        cells = set(zip(tr.level.tolist(), map(tuple, np.round(tr.centre * 2 ** 22).astype(np.int64).tolist()),
                        tr.count.tolist()))
        acc, pot, nint = oracle_mod.walk(tr, np.arange(0, w.pos.shape[0], 4))
        out[curve] = (cells, acc, pot, nint, tr)
    assert out[0][0] == out[1][0]
    assert not np.array_equal(out[0][4].perm, out[1][4].perm)
    e = np.linalg.norm(out[0][1] - out[1][1], axis=1) / np.linalg.norm(out[0][1], axis=1)
    assert e.max() <= 1e-13
    assert np.abs(out[0][2] - out[1][2]).max() <= 1e-13 * np.abs(out[0][2]).max()
    assert np.array_equal(out[0][3], out[1][3])

"""GPU particle-mesh long-range force against the oracle (same steps of the
paper's "Particle Mesh" subsection, FP64 on both sides).  The GPU sums the
mesh in 64-bit fixed point (relative resolution ~1e-18 of the total mass)
and runs its own FFT, so values agree to rounding: |da| <= 1e-10 max|a|
and |dphi| <= 1e-10 max|phi|.  The full TreePM force (tree short-range +
mesh long-range) is checked the same way against the oracle's direct sum +
mesh."""
import sys

import numpy as np
import pytest

from paper_2609_17658_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def og_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_17658_amd import og
    og.load()
    return og


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _particles(n, seed, box=1.0):
    rng = np.random.default_rng(seed)
    h = n // 2
    pos = np.concatenate([rng.random((h, 3)), (0.3 + 0.04 * rng.standard_normal((n - h, 3))) % 1.0]) * box
    return pos, rng.uniform(0.5, 1.5, n) / n


@pytest.mark.parametrize("n_grid,N,box,G", [(8, 500, 1.0, 1.0), (32, 3000, 1.0, 1.0), (64, 20000, 3.0, 2.0),
                                            (128, 50000, 1.0, 1.0)])
def test_pm_matches_oracle(og_mod, n_grid, N, box, G):
    from oracle import pm as opm
    _note("pm n_grid=%d N=%d box=%g" % (n_grid, N, box))
    pos, mass = _particles(N, n_grid, box)
    r_s = 1.25 * box / n_grid
    a_o, p_o = opm.long_range(pos, mass, box, n_grid, G, r_s)
    m = og_mod.PM(n_grid, box, G, r_s, stream=torch.cuda.current_stream())
    acc, pot = m.force(_dev(pos), _dev(mass))
    torch.cuda.synchronize()
    a, p = acc.cpu().numpy(), pot.cpu().numpy()
    assert np.abs(a - a_o).max() <= 1e-10 * np.abs(a_o).max()
    assert np.abs(p - p_o).max() <= 1e-10 * np.abs(p_o).max()
    # deterministic: the same call again gives the same bits
    acc2, pot2 = m.force(_dev(pos), _dev(mass))
    torch.cuda.synchronize()
    assert torch.equal(acc, acc2) and torch.equal(pot, pot2)
    m.close()


def test_pm_256_four_line_tiles_match_oracle(og_mod):
    """n_grid = 256: the FFT passes take 4 lines per workgroup (the smaller
    meshes take 16 and 8)."""
    from oracle import pm as opm
    pos, mass = _particles(120000, 256)
    r_s = 1.25 / 256
    _note("pm n_grid=256 N=120000 (4-line FFT tiles)")
    a_o, p_o = opm.long_range(pos, mass, 1.0, 256, 1.0, r_s)
    m = og_mod.PM(256, 1.0, 1.0, r_s, stream=torch.cuda.current_stream())
    acc, pot = m.force(_dev(pos), _dev(mass))
    torch.cuda.synchronize()
    a, p = acc.cpu().numpy(), pot.cpu().numpy()
    _note("  max |da|/max|a| %.3g" % (np.abs(a - a_o).max() / np.abs(a_o).max()))
    assert np.abs(a - a_o).max() <= 1e-10 * np.abs(a_o).max()
    assert np.abs(p - p_o).max() <= 1e-10 * np.abs(p_o).max()
    m.close()


@pytest.mark.parametrize("n_grid", [64, 128])
def test_pm_every_fft_tile_width(og_mod, n_grid, monkeypatch):
    """OG_FFT_LINES sets the lines per FFT workgroup, so every width the
    larger meshes take runs on small meshes, and at 128^3 the 16-line
    tiles of the fused x pass are the larger meshes' tile shape (2048
    elements, 8 per thread, more than 64 KB of LDS): each result is
    bitwise the default one (the same butterflies per line) and within
    1e-10 of the oracle, from caller arrays and from a tree."""
    from oracle import pm as opm
    pos, mass = _particles(30000, n_grid + 1)
    r_s = 1.25 / n_grid
    a_o, p_o = opm.long_range(pos, mass, 1.0, n_grid, 1.0, r_s)
    stream = torch.cuda.current_stream()
    m = og_mod.PM(n_grid, 1.0, 1.0, r_s, stream=stream)
    ref_a, ref_p = m.force(_dev(pos), _dev(mass))
    tree = og_mod.Tree(_dev(pos), _dev(mass), 1.0, synth.scale_free_params(30000).as_dict(), stream=stream)
    for lines in (16, 8, 4, 2, 1):
        _note("pm n_grid=%d with %d-line FFT tiles" % (n_grid, lines))
        monkeypatch.setenv("OG_FFT_LINES", str(lines))
        acc, pot = m.force(_dev(pos), _dev(mass))
        at, pt = m.force_tree(tree)
        torch.cuda.synchronize()
        monkeypatch.delenv("OG_FFT_LINES")
        assert torch.equal(acc, ref_a) and torch.equal(pot, ref_p), lines
        assert torch.equal(at, ref_a) and torch.equal(pt, ref_p), lines
        a, p = acc.cpu().numpy(), pot.cpu().numpy()
        assert np.abs(a - a_o).max() <= 1e-10 * np.abs(a_o).max()
        assert np.abs(p - p_o).max() <= 1e-10 * np.abs(p_o).max()
    tree.close()
    m.close()


def test_pm_512_fused_pass_threads(og_mod, monkeypatch):
    """At 512^3 the fused x pass takes tiles of 8 lines with 512 threads;
    with 4 lines or fewer it takes 256 threads.  Every width gives the
    default result bitwise (from caller arrays and from a tree), and the
    mesh force conserves momentum: with the same assignment and
    interpolation and an odd gradient kernel the pair forces cancel, so
    sum m a vanishes up to rounding (checked on the oracle at 32^3, where
    it is 1e-17 of sum m |a|)."""
    n_grid = 512
    pos, mass = _particles(30000, 7)
    stream = torch.cuda.current_stream()
    m = og_mod.PM(n_grid, 1.0, 1.0, 1.25 / n_grid, stream=stream)
    ref_a, ref_p = m.force(_dev(pos), _dev(mass))
    tree = og_mod.Tree(_dev(pos), _dev(mass), 1.0, synth.scale_free_params(30000).as_dict(), stream=stream)
    for lines in (8, 4, 1):
        _note("pm n_grid=512 with %d-line FFT tiles" % lines)
        monkeypatch.setenv("OG_FFT_LINES", str(lines))
        acc, pot = m.force(_dev(pos), _dev(mass))
        at, pt = m.force_tree(tree)
        torch.cuda.synchronize()
        monkeypatch.delenv("OG_FFT_LINES")
        assert torch.equal(acc, ref_a) and torch.equal(pot, ref_p), lines
        assert torch.equal(at, ref_a) and torch.equal(pt, ref_p), lines
    a = ref_a.cpu().numpy()
    mom = np.abs((mass[:, None] * a).sum(0))
    assert np.all(mom <= 1e-12 * (mass[:, None] * np.abs(a)).sum(0))
    tree.close()
    m.close()


def test_pm_wraps_positions_and_accumulates(og_mod):
    pos, mass = _particles(4000, 5)
    m = og_mod.PM(32, 1.0, 1.0, 1.25 / 32, stream=torch.cuda.current_stream())
    a1, p1 = m.force(_dev(pos), _dev(mass))
    shifted = pos + np.array([1.0, -1.0, 2.0])    # periodic images
    a2, p2 = m.force(_dev(shifted), _dev(mass))
    base_a = torch.full_like(a1, 0.25)
    base_p = torch.full_like(p1, -0.5)
    a3, p3 = m.force(_dev(pos), _dev(mass), acc=base_a.clone(), pot=base_p.clone(), accumulate=True)
    torch.cuda.synchronize()
    assert torch.allclose(a1, a2, rtol=0, atol=1e-9 * a1.abs().max().item())
    assert torch.equal(a3, base_a + a1) and torch.equal(p3, base_p + p1)
    m.close()


def test_treepm_total_matches_oracle(og_mod, oracle_mod):
    """Full TreePM force: tree (theta = 0.3, FP64) short-range + mesh."""
    from oracle import pm as opm
    w = synth.mixture32k()
    prm = dict(w.params.as_dict(), theta=0.3)
    n_grid = 64   # r_s = 1.25/64 = 1.25 mesh cells
    tree = og_mod.Tree(_dev(w.pos), _dev(w.mass), 1.0, prm, stream=torch.cuda.current_stream())
    acc, pot = tree.force(precision="fp64")
    m = og_mod.PM(n_grid, 1.0, prm["G"], prm["r_s"], stream=torch.cuda.current_stream())
    m.force(_dev(w.pos), _dev(w.mass), acc=acc, pot=pot, accumulate=True)
    torch.cuda.synchronize()
    op = oracle_mod.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic", "leaf_max")})
    a_s, p_s, _ = oracle_mod.tree_force(w.pos, w.mass, 1.0, op)
    a_l, p_l = opm.long_range(w.pos, w.mass, 1.0, n_grid, prm["G"], prm["r_s"])
    a_t = a_s + a_l
    err = np.linalg.norm(acc.cpu().numpy() - a_t, axis=1) / np.linalg.norm(a_t, axis=1)
    assert np.percentile(err, 99.9) <= 1e-10
    tree.close()
    m.close()


def test_pm_rejects_bad_arguments(og_mod):
    import ctypes
    lib = og_mod.load()
    h = ctypes.c_void_p()
    for n, box, r_s in ((12, 1.0, 0.01), (4, 1.0, 0.01), (2048, 1.0, 0.01), (32, 0.0, 0.01), (32, 1.0, 0.0)):
        assert lib.og_pm_create(n, box, 1.0, r_s, None, ctypes.byref(h)) == og_mod.OG_EINVAL
    m = og_mod.PM(16, 1.0, 1.0, 0.1)
    pos = np.random.default_rng(0).random((10, 3))
    rc = lib.og_pm_force(m.handle, pos.ctypes.data_as(ctypes.c_void_p), None, 10, None, None, 0)
    assert rc == og_mod.OG_EINVAL
    m.close()


def test_pm_from_tree_equals_caller_order(og_mod):
    """The fixed-point deposit does not depend on the order of particles, so
    the mesh filled in the tree's curve order is the same, and every
    particle's interpolation is the same arithmetic: bitwise equal."""
    pos, mass = _particles(30000, 8)
    prm = synth.scale_free_params(30000).as_dict()
    stream = torch.cuda.current_stream()
    tree = og_mod.Tree(_dev(pos), _dev(mass), 1.0, prm, stream=stream)
    m = og_mod.PM(64, 1.0, prm["G"], prm["r_s"], stream=stream)
    a1, p1 = m.force(_dev(pos), _dev(mass))
    a2, p2 = m.force_tree(tree)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    # non-periodic tree or another box side: rejected
    t2 = og_mod.Tree(_dev(pos), _dev(mass), 1.0, dict(G=1.0, eps=0.01, r_s=0.0, theta=0.5, periodic=0, leaf_max=8),
                     stream=stream)
    with pytest.raises(og_mod.OgError):
        m.force_tree(t2)
    m2 = og_mod.PM(64, 2.0, prm["G"], prm["r_s"], stream=stream)
    with pytest.raises(og_mod.OgError):
        m2.force_tree(tree)
    for x in (tree, t2, m, m2):
        x.close()


@pytest.mark.parametrize("n_grid,curve,clump", [(8, "morton", 0), (32, "hilbert", 0), (64, "morton", 20000),
                                                (64, "hilbert", 20000), (128, "morton", 40000)])
def test_pm_from_tree_blocks(og_mod, n_grid, curve, clump):
    """The tree-order path (block workgroups of 8^3 cells, halos, and the
    per-particle kernels for blocks of more than 2048 particles) gives the
    caller-order result to the bit and the oracle's within the bar, with
    particles at 0 and just below the box side, on one block (n = 8, whose
    halo wraps onto itself) and on Hilbert trees (block corners from the
    inverse curve)."""
    from oracle import pm as opm
    rng = np.random.default_rng(n_grid + clump)
    pos, mass = _particles(30000, n_grid)
    if clump:
        pos = np.concatenate([pos, (0.61 + 0.004 * rng.standard_normal((clump, 3))) % 1.0])
        mass = np.concatenate([mass, np.full(clump, 0.5 / clump)])
    pos[:7, 0] = np.nextafter(1.0, 0.0)
    pos[7:14, 1] = 0.0
    pos[14:21, 2] = np.nextafter(1.0, 0.0)
    n = pos.shape[0]
    _note("pm from tree n_grid=%d curve=%s N=%d" % (n_grid, curve, n))
    prm = dict(synth.scale_free_params(n).as_dict(), curve=curve)
    stream = torch.cuda.current_stream()
    tree = og_mod.Tree(_dev(pos), _dev(mass), 1.0, prm, stream=stream)
    r_s = 1.25 / n_grid
    m = og_mod.PM(n_grid, 1.0, 1.0, r_s, stream=stream)
    a1, p1 = m.force(_dev(pos), _dev(mass))
    a2, p2 = m.force_tree(tree)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    a_o, p_o = opm.long_range(pos, mass, 1.0, n_grid, 1.0, r_s)
    a, p = a2.cpu().numpy(), p2.cpu().numpy()
    assert np.abs(a - a_o).max() <= 1e-10 * np.abs(a_o).max()
    assert np.abs(p - p_o).max() <= 1e-10 * np.abs(p_o).max()
    tree.close()
    m.close()

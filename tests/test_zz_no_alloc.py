"""og_tree_force_noalloc (the allocation-free variant of og_tree_force)
through the C ABI: bitwise the results of og_tree_force on the same tree
and targets, for two calls in a row of which the second has fewer targets
(the shared device array keeps the first call's contents), in both
precisions, for all particles, and with the size limit enforced."""
import ctypes
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


def _call(lib, fn, h, idx, M):
    acc = torch.full((M, 3), np.nan, dtype=torch.float64, device="cuda")
    pot = torch.full((M,), np.nan, dtype=torch.float64, device="cuda")
    tg = None
    if idx is not None:
        tg = ctypes.byref(_targets(idx))
    rc = getattr(lib, fn)(h, tg, ctypes.c_void_p(acc.data_ptr()), ctypes.c_void_p(pot.data_ptr()))
    return rc, acc, pot


def _targets(idx):
    from paper_2609_17658_amd import og
    return og.og_targets(ctypes.c_void_p(idx.data_ptr()), int(idx.numel()))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_equals_og_tree_force(og_mod, prec):
    w = synth.mixture32k()
    lib = og_mod.load()
    params = og_mod.make_params(w.params, precision=prec, stream=torch.cuda.current_stream())
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    h = og_mod.og_tree_build(tp, tm, w.pos.shape[0], 1.0, params)
    rng = np.random.default_rng(7)
    n = w.pos.shape[0]
    # first call: 20000 targets with repeats; second call: 3000 other targets
    for M, seed in ((20000, 1), (3000, 2)):
        sel = np.random.default_rng(seed).integers(0, n, M)
        sel[:5] = sel[5]
        idx = torch.as_tensor(sel, dtype=torch.int64, device="cuda")
        _note("noalloc %s: M=%d" % (prec, M))
        rc1, a1, p1 = _call(lib, "og_tree_force_noalloc", h, idx, M)
        rc2, a2, p2 = _call(lib, "og_tree_force", h, idx, M)
        torch.cuda.synchronize()
        assert rc1 == 0 and rc2 == 0
        assert torch.equal(a1, a2) and torch.equal(p1, p2)
    # all particles (no scratch needed)
    rc1, a1, p1 = _call(lib, "og_tree_force_noalloc", h, None, n)
    rc2, a2, p2 = _call(lib, "og_tree_force", h, None, n)
    torch.cuda.synchronize()
    assert rc1 == 0 and rc2 == 0
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    assert og_mod.og_tree_status(h) == 0
    og_mod.og_tree_free(h)
    del rng


def test_noalloc_limit_and_arguments(og_mod):
    w = synth.mixture32k()
    lib = og_mod.load()
    params = og_mod.make_params(w.params, stream=torch.cuda.current_stream())
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    h = og_mod.og_tree_build(tp, tm, w.pos.shape[0], 1.0, params)
    M = og_mod.OG_NOALLOC_MAX_TARGETS + 1
    idx = torch.zeros(M, dtype=torch.int64, device="cuda")
    rc, a, _ = _call(lib, "og_tree_force_noalloc", h, idx, M)
    torch.cuda.synchronize()
    assert rc == og_mod.OG_EINVAL
    assert "limit" in lib.og_last_error().decode()
    assert torch.isnan(a).all()           # nothing written
    # the largest allowed list works and matches the allocating call
    M = og_mod.OG_NOALLOC_MAX_TARGETS
    sel = np.random.default_rng(3).integers(0, w.pos.shape[0], M)
    idx = torch.as_tensor(sel, dtype=torch.int64, device="cuda")
    rc1, a1, p1 = _call(lib, "og_tree_force_noalloc", h, idx, M)
    rc2, a2, p2 = _call(lib, "og_tree_force", h, idx, M)
    torch.cuda.synchronize()
    assert rc1 == 0 and rc2 == 0
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    assert lib.og_tree_force_noalloc(None, None, None, None) == og_mod.OG_EINVAL
    og_mod.og_tree_free(h)

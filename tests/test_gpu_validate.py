"""og_tree_validate, the host-side invariant checker, on trees of every
kind the builder makes (periodic and open boxes, Morton and Hilbert keys,
leaf sizes 1..16, coincident particles that end in finest-level leaves,
one particle, per-particle softening, a 2M-particle clustered box), and on
host-corrupted copies, where each kind of damage must be reported as
OG_ECORRUPT with a message naming it (OG_FAULT_CORRUPT edits only the
checker's host copy; the device tree is untouched)."""
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


def _tree(og_mod, pos, mass, box=1.0, **prm):
    p = dict(synth.scale_free_params(len(pos)).as_dict(), **prm)
    tp = torch.as_tensor(pos, device="cuda")
    tm = torch.as_tensor(mass, device="cuda")
    return og_mod.Tree(tp, tm, box, p, stream=torch.cuda.current_stream())


def _coincident(n, seed):
    rng = np.random.default_rng(seed)
    pos = synth.mixture_box(n, seed)
    # a quarter of the particles stacked on 5 points: leaves at level 21 of
    # more than leaf_max particles
    k = n // 4
    pos[:k] = pos[rng.integers(0, 5, k) + k]
    return pos


CASES = {
    "periodic_mixed": lambda: (synth.mixture_box(3000, 71), {}),
    "periodic_fp64": lambda: (synth.mixture_box(3000, 72), {"precision": "fp64"}),
    "open_box": lambda: (synth.mixture_box(3000, 73) * 0.5 + 0.2, {"periodic": 0}),
    "hilbert": lambda: (synth.mixture_box(5000, 74), {"curve": "hilbert"}),
    "leaf1": lambda: (synth.mixture_box(2000, 75), {"leaf_max": 1}),
    "leaf16": lambda: (synth.mixture_box(4000, 76), {"leaf_max": 16}),
    "coincident": lambda: (_coincident(4000, 77), {}),
    "coincident_hilbert_open": lambda: (_coincident(4000, 78) * 0.9, {"curve": "hilbert", "periodic": 0}),
    "one_particle": lambda: (np.array([[0.25, 0.5, 0.75]]), {"r_s": 0.01, "r_cut": 0.045, "eps": 0.001}),
    "zeldovich64": lambda: (synth.zeldovich(64, 79), {}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_built_trees_satisfy_invariants(og_mod, name):
    pos, prm = CASES[name]()
    _note("validate %s: N=%d %s" % (name, len(pos), prm))
    t = _tree(og_mod, pos, synth.equal_masses(len(pos)), **prm)
    assert t.validate() == og_mod.OG_OK
    t.close()


def test_per_particle_softening_tree_is_valid(og_mod):
    n = 3000
    pos = synth.mixture_box(n, 80)
    eps = torch.as_tensor(np.random.default_rng(80).uniform(1e-4, 1e-3, n), device="cuda")
    _note("validate per-particle softening N=%d" % n)
    t = _tree(og_mod, pos, synth.equal_masses(n), eps_particle=eps)
    assert t.validate() == og_mod.OG_OK
    t.close()


def test_mixture2m_tree_is_valid(og_mod):
    w = synth.mixture2m()
    _note("validate mixture2m N=%d" % len(w.pos))
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    t = og_mod.Tree(tp, tm, w.box, w.params.as_dict(), stream=torch.cuda.current_stream())
    assert t.validate() == og_mod.OG_OK
    t.close()


@pytest.mark.parametrize("field,phrase", [
    ("keys", "keys not sorted"), ("perm", "permutation"), ("position", "particle"),
    ("count", "hold particles up to"), ("skip", "root node"), ("parent", "parent"), ("level", "level"),
    ("mass", "mass of node"), ("com", "centre of mass"), ("record", "walk record"),
])
def test_corrupted_copies_are_reported(og_mod, monkeypatch, field, phrase):
    pos = synth.mixture_box(3000, 81)
    t = _tree(og_mod, pos, synth.equal_masses(3000))
    monkeypatch.setenv("OG_FAULT_CORRUPT", field)
    with pytest.raises(og_mod.OgError) as ei:
        t.validate()
    _note("corrupt %s: %s" % (field, ei.value))
    assert ei.value.code == og_mod.OG_ECORRUPT
    assert phrase in str(ei.value)
    monkeypatch.delenv("OG_FAULT_CORRUPT")
    assert t.validate() == og_mod.OG_OK     # the device tree was never touched
    t.close()

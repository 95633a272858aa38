"""Property tests of the HIP path on hypothesis-drawn small configurations
(the strategies of prop_inputs: coincident particles, dyadic cell faces,
the periodic wrap, leaf sizes 1..16, open and periodic boxes, Morton and
Hilbert keys), through the C ABI:

  * the tree equals the oracle's to the bit (keys, permutation, topology),
    the FP64 walk matches the oracle (|da| <= 1e-11 |a| per target, plus
    1e-13 of the largest |a| for targets whose force nearly cancels) with
    identical interaction counts, and the built tree passes
    og_tree_validate;
  * reordering the input particles permutes the outputs: to the bit when
    all keys differ, within rounding otherwise (FP64 and mixed walks);
  * a walk over a target subset equals the full walk at those targets to
    the bit (FP64 and mixed).
"""
import sys

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

from prop_inputs import configs, oracle_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large,
                                           HealthCheck.function_scoped_fixture])


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


def _run(og, cfg, precision, pos=None, mass=None, targets=None, export=False, validate=False):
    pos = cfg.pos if pos is None else pos
    mass = cfg.mass if mass is None else mass
    tp = torch.as_tensor(pos, device="cuda")
    tm = torch.as_tensor(mass, device="cuda")
    tree = og.Tree(tp, tm, cfg.box, dict(cfg.params, precision=precision), stream=torch.cuda.current_stream())
    tg = None if targets is None else torch.as_tensor(targets, dtype=torch.int64, device="cuda")
    acc, pot, nint = tree.force(targets=tg, with_counts=True)
    out = {"acc": acc.cpu().numpy(), "pot": pot.cpu().numpy(), "nint": nint.cpu().numpy()}
    if export:
        out["tree"] = tree.export()
    if validate:
        tree.validate()
    tree.close()
    return out


@SETTINGS
@given(cfg=configs())
def test_tree_and_fp64_walk_match_the_oracle(og_mod, oracle_mod, cfg):
    _note("fp64 vs oracle: %s" % cfg.label)
    op = oracle_params(oracle_mod, cfg.params)
    ot = oracle_mod.build_tree(cfg.pos, cfg.mass, cfg.box, op)
    g = _run(og_mod, cfg, "fp64", export=True, validate=True)
    t = g["tree"]
    assert np.array_equal(t["keys"], ot.skeys) and np.array_equal(t["perm"], ot.perm)
    for k in ("first", "count", "level", "skip", "parent"):
        assert np.array_equal(t[k], getattr(ot, k)), k
    acc, pot, nint = oracle_mod.walk(ot)
    assert np.array_equal(g["nint"], nint)
    big = np.abs(acc).max() if acc.size else 0.0
    da = np.linalg.norm(g["acc"] - acc, axis=1)
    assert np.all(da <= 1e-11 * np.linalg.norm(acc, axis=1) + 1e-13 * big)
    assert np.all(np.abs(g["pot"] - pot) <= 1e-12 * np.abs(pot) + 1e-13 * np.abs(pot).max())


@SETTINGS
@given(cfg=configs())
def test_input_order_does_not_matter(og_mod, oracle_mod, cfg):
    _note("permutation: %s" % cfg.label)
    n = len(cfg.pos)
    sig = np.random.default_rng(n).permutation(n)
    keys = oracle_mod.keys(cfg.pos, cfg.box, cfg.params["periodic"], cfg.params["curve"])
    distinct = len(np.unique(keys)) == n
    for prec in ("fp64", "mixed"):
        a = _run(og_mod, cfg, prec)
        b = _run(og_mod, cfg, prec, pos=np.ascontiguousarray(cfg.pos[sig]), mass=cfg.mass[sig])
        if distinct:
            assert np.array_equal(b["acc"], a["acc"][sig]), prec
            assert np.array_equal(b["pot"], a["pot"][sig]), prec
            assert np.array_equal(b["nint"], a["nint"][sig]), prec
        else:
            tol = 1e-12 if prec == "fp64" else 1e-5
            scale = max(np.abs(a["acc"]).max(), 1e-300)
            assert np.abs(b["acc"] - a["acc"][sig]).max() <= tol * scale, prec


@SETTINGS
@given(cfg=configs())
def test_subset_walk_equals_full_walk(og_mod, cfg):
    _note("subset: %s" % cfg.label)
    n = len(cfg.pos)
    tg = np.random.default_rng(n + 1).choice(n, size=max(1, n // 3), replace=False)
    for prec in ("fp64", "mixed"):
        full = _run(og_mod, cfg, prec)
        sub = _run(og_mod, cfg, prec, targets=tg)
        for k in ("acc", "pot", "nint"):
            assert np.array_equal(sub[k], full[k][tg]), (prec, k)

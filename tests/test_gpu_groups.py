"""GPU group-shared interaction lists (one walk per group of consecutive
targets in curve order) against the oracle's group walk over the same
partition.  FP64: identical interaction counts and |da|/|a| <= 1e-11 (the
same partners in the same order); mixed: the usual error bars.  The
partition is the oracle's own: chunks of group_max consecutive targets in
its curve order."""
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


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def _oparams(oracle_mod, prm):
    return oracle_mod.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic", "leaf_max",
                                                    "softening", "criterion", "alpha", "curve") if k in prm})


def _cases():
    rng = np.random.default_rng(99)
    out = []
    w = synth.mixture32k()
    out.append(("mixture32k", w.pos, w.mass, 1.0, w.params.as_dict()))
    n = 7001
    pos = synth.wrap(np.concatenate([rng.random((n - n // 2, 3)), 0.6 + 0.01 * rng.standard_normal((n // 2, 3))]))
    out.append(("clustered7001_lm16", pos, rng.uniform(0.5, 1.5, n) / n, 1.0,
                synth.scale_free_params(n, leaf_max=16).as_dict()))
    pos = np.full((300, 3), 0.3)
    pos[:100] = rng.random((100, 3))
    out.append(("coincident300", pos, np.full(300, 1 / 300), 1.0, synth.scale_free_params(300, leaf_max=4).as_dict()))
    pos = rng.normal(size=(3000, 3)) * [1.0, 2.0, 0.5] + 5.0
    out.append(("open3000", pos, np.full(3000, 1 / 3000), 1.0,
                dict(G=1.0, eps=0.01, r_s=0.0, r_cut=0.0, theta=0.6, periodic=0, leaf_max=8)))
    pos = rng.random((6000, 3)) * 3.0
    pos[:500, 0] = 0.0
    out.append(("box3_faces", pos, np.full(6000, 1 / 6000), 3.0,
                dict(G=1.0, eps=0.002, r_s=0.05, r_cut=0.25, theta=0.7, periodic=1, leaf_max=8)))
    return out


CASES = _cases()


@pytest.mark.parametrize("gm", [64, 13])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_group_lists_match_oracle(og_mod, oracle_mod, case, gm):
    name, pos, mass, box, prm = case
    _note("group lists %s group_max %d N=%d" % (name, gm, pos.shape[0]))
    otree = oracle_mod.build_tree(pos, mass, box, _oparams(oracle_mod, prm))
    acc, pot, nint = oracle_mod.walk_groups(otree, gm)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream(),
                       lists="group", group_max=gm)
    a64, p64, n64 = tree.force(precision="fp64", with_counts=True)
    a32, p32, n32 = tree.force(precision="mixed", with_counts=True)
    torch.cuda.synchronize()
    assert tree.status() == 0
    tree.close()
    assert np.array_equal(n64.cpu().numpy(), nint)
    e64 = _rel(a64.cpu().numpy(), acc)
    assert e64.max() <= 1e-11 or (np.percentile(e64, 99.9) <= 1e-12 and e64.max() <= 1e-9)
    assert np.all(np.abs(p64.cpu().numpy() - pot) <= 1e-12 * np.abs(pot) + 1e-300)
    ok = np.linalg.norm(acc, axis=1) > 0
    e = _rel(a32.cpu().numpy(), acc)[ok]
    if e.size:
        assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2
    assert (n32.cpu().numpy() != nint).mean() <= 0.01


def test_group_of_one_equals_per_target_walk(og_mod):
    name, pos, mass, box, prm = CASES[0]
    out = {}
    for lists in ("target", "group"):
        t = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream(), lists=lists,
                        group_max=1)
        a, p, n = t.force(precision="fp64", with_counts=True)
        torch.cuda.synchronize()
        out[lists] = (a.cpu().numpy(), n.cpu().numpy())
        t.close()
    assert np.array_equal(out["target"][1], out["group"][1])
    assert np.abs(out["target"][0] - out["group"][0]).max() <= 1e-13 * np.abs(out["target"][0]).max()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_group_lists_batch_equals_alone(og_mod, prec):
    items = [(pos, mass, box, dict(prm, lists="group")) for name, pos, mass, box, prm in CASES]
    alone = []
    for pos, mass, box, prm in items:
        t = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
        a, p = t.force(precision=prec)
        torch.cuda.synchronize()
        alone.append((a.cpu().numpy(), p.cpu().numpy()))
        t.close()
    bt = og_mod.Batch([(_dev(p), _dev(m), b, prm) for p, m, b, prm in items], stream=torch.cuda.current_stream(),
                      precision=prec)
    outs = bt.force()
    torch.cuda.synchronize()
    assert bt.status() == 0
    for (a, p), (ga, gp) in zip(alone, outs):
        assert np.array_equal(ga.cpu().numpy(), a) and np.array_equal(gp.cpu().numpy(), p)
    bt.close()


def test_group_lists_with_variants(og_mod, oracle_mod):
    name, pos, mass, box, prm = CASES[0]
    prm = dict(prm, lists="group", softening=1, criterion=1, alpha=0.003, curve=1)
    oprm = dict(prm, softening=1, criterion=1, curve=1)
    otree = oracle_mod.build_tree(pos, mass, box, _oparams(oracle_mod, dict(oprm, criterion=0)))
    a_old = oracle_mod.walk(otree)[0]
    otree = oracle_mod.build_tree(pos, mass, box, _oparams(oracle_mod, oprm))
    acc, pot, nint = oracle_mod.walk_groups(otree, 64, a_old=a_old)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    a64, _, n64 = tree.force(precision="fp64", with_counts=True, a_old=_dev(a_old))
    a32, _, _ = tree.force(precision="mixed", with_counts=True, a_old=_dev(a_old))
    torch.cuda.synchronize()
    tree.close()
    assert np.array_equal(n64.cpu().numpy(), nint)
    assert _rel(a64.cpu().numpy(), acc).max() <= 1e-11
    e = _rel(a32.cpu().numpy(), acc)
    assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2

"""GPU parity of the Peano-Hilbert curve and of active-subset forces on a
resident tree (paper, "Tree construction": Peano-Hilbert insertion order;
"Code structure": forces for the active time-step levels only).

Hilbert keys, permutation and topology are integers and must equal the
oracle's bit for bit; the FP64 walk within 1e-11 with identical counts; the
mixed walk within the usual bars.  Active forces must equal, bit for bit,
the same targets' entries of a force call on every particle (each lane's
walk is independent of its group), leave inactive entries untouched, and
match the oracle walk on the active targets."""
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


def _oparams(oracle_mod, prm, **kw):
    d = dict(prm, **kw)
    return oracle_mod.Params(**{k: d[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic", "leaf_max",
                                                  "curve") if k in d})


def _cases():
    rng = np.random.default_rng(77)
    out = []
    w = synth.mixture32k()
    out.append(("mixture32k", w.pos, w.mass, 1.0, w.params.as_dict()))
    n = 9001
    pos = synth.wrap(np.concatenate([rng.random((n - n // 2, 3)), 0.7 + 0.01 * rng.standard_normal((n // 2, 3))]))
    out.append(("clustered9001_lm16", pos, rng.uniform(0.5, 1.5, n) / n, 1.0,
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


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_hilbert_tree_and_walk_parity(og_mod, oracle_mod, case):
    name, pos, mass, box, prm = case
    prm = dict(prm, curve=1)
    _note("hilbert case %s N=%d" % (name, pos.shape[0]))
    otree = oracle_mod.build_tree(pos, mass, box, _oparams(oracle_mod, prm))
    acc, pot, nint = oracle_mod.walk(otree)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    ex = tree.export()
    assert np.array_equal(ex["keys"], otree.skeys)
    assert np.array_equal(ex["perm"], otree.perm)
    assert len(ex["first"]) == otree.n_nodes
    for k in ("first", "count", "level", "skip", "parent"):
        assert np.array_equal(ex[k], getattr(otree, k)), k
    # moments: the two sides sum in different orders (see the Morton test)
    m, u = ex["node_m_com"], 2.0 ** -53
    cnt = otree.count.astype(np.float64)
    assert np.all(np.abs(m[:, 0] - otree.mass) <= 2 * cnt * u * otree.mass)
    lim = 2 * cnt[:, None] * u * otree.side[:, None] + 4 * u * np.abs(otree.com)
    assert np.all(np.abs(m[:, 1:] - otree.com) <= lim)
    a64, p64, n64 = tree.force(precision="fp64", with_counts=True)
    a32, p32, n32 = tree.force(precision="mixed", with_counts=True)
    torch.cuda.synchronize()
    assert tree.status() == 0
    tree.close()
    assert np.array_equal(n64.cpu().numpy(), nint)
    e64 = _rel(a64.cpu().numpy(), acc)
    assert e64.max() <= 1e-11 or (np.percentile(e64, 99.9) <= 1e-12 and e64.max() <= 1e-9)
    ok = np.linalg.norm(acc, axis=1) > 0
    e = _rel(a32.cpu().numpy(), acc)[ok]
    if e.size:
        assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2
    assert (n32.cpu().numpy() != nint).mean() <= 0.01


def test_hilbert_batch_equals_alone(og_mod):
    items = [(pos, mass, box, dict(prm, curve=c)) for c, (name, pos, mass, box, prm) in
             zip((1, 0, 1, 1, 0), CASES)]
    alone = []
    for pos, mass, box, prm in items:
        t = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
        a, p = t.force(precision="mixed")
        torch.cuda.synchronize()
        alone.append((a.cpu().numpy(), p.cpu().numpy()))
        t.close()
    bt = og_mod.Batch([(_dev(p), _dev(m), b, prm) for p, m, b, prm in items], stream=torch.cuda.current_stream())
    outs = bt.force()
    torch.cuda.synchronize()
    assert bt.status() == 0
    for (a, p), (ga, gp) in zip(alone, outs):
        assert np.array_equal(ga.cpu().numpy(), a) and np.array_equal(gp.cpu().numpy(), p)
    bt.close()


def _bins(n, seed):
    """Seeded time-step levels 0..5, most particles on the long steps."""
    rng = np.random.default_rng(seed)
    return np.minimum(rng.geometric(0.45, n) - 1, 5).astype(np.int8)


@pytest.mark.parametrize("curve", [0, 1])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_active_forces_match_full_and_oracle(og_mod, oracle_mod, prec, curve):
    name, pos, mass, box, prm = CASES[0]
    prm = dict(prm, curve=curve)
    n = pos.shape[0]
    bins = _bins(n, 5)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    full_a, full_p, full_n = tree.force(precision=prec, with_counts=True)
    dbin = _dev(bins, torch.int8)
    for level in (0, 2, 5):
        act = np.flatnonzero(bins <= level)
        acc = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        pot = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        nint = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        na = torch.zeros(1, dtype=torch.int64, device="cuda")
        tree.force_active(dbin, level, acc, pot, precision=prec, n_inter=nint, n_active=na)
        torch.cuda.synchronize()
        _note("active %s curve %d level %d: %d of %d" % (prec, curve, level, act.size, n))
        assert int(na.item()) == act.size
        a, p, ni = acc.cpu().numpy(), pot.cpu().numpy(), nint.cpu().numpy()
        inact = np.setdiff1d(np.arange(n), act)
        assert np.isnan(a[inact]).all() and np.isnan(p[inact]).all() and np.all(ni[inact] == -1)
        assert np.array_equal(a[act], full_a.cpu().numpy()[act])
        assert np.array_equal(p[act], full_p.cpu().numpy()[act])
        assert np.array_equal(ni[act], full_n.cpu().numpy()[act])
    assert tree.status() == 0
    tree.close()
    # the oracle on the last level's active targets
    oa, _, on = oracle_mod.tree_force(pos, mass, box, _oparams(oracle_mod, prm), targets=act)
    if prec == "fp64":
        assert np.array_equal(ni[act], on)
        assert _rel(a[act], oa).max() <= 1e-11
    else:
        e = _rel(a[act], oa)
        assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2


def test_active_empty_set_writes_nothing(og_mod):
    name, pos, mass, box, prm = CASES[1]
    n = pos.shape[0]
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    acc = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    na = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    tree.force_active(_dev(np.full(n, 3, np.int8), torch.int8), 2, acc, n_active=na)
    torch.cuda.synchronize()
    assert int(na.item()) == 0
    assert torch.all(acc == 7.0).item()
    tree.close()


def test_active_relative_criterion_uses_caller_index(og_mod, oracle_mod):
    name, pos, mass, box, prm = CASES[0]
    prm = dict(prm, criterion=1, alpha=0.003, curve=1)
    n = pos.shape[0]
    a_old = oracle_mod.tree_force(pos, mass, box, _oparams(oracle_mod, prm))[0]
    bins = _bins(n, 9)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    dao = _dev(a_old)
    full_a, _ = tree.force(precision="fp64", a_old=dao)
    acc = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    tree.force_active(_dev(bins, torch.int8), 1, acc, precision="fp64", a_old=dao)
    torch.cuda.synchronize()
    act = np.flatnonzero(bins <= 1)
    assert np.array_equal(acc.cpu().numpy()[act], full_a.cpu().numpy()[act])
    tree.close()

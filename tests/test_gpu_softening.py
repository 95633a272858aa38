"""GPU per-particle softening lengths and the mixed-softening check (paper,
"Tree walk") against the oracle: FP64 walk with identical interaction
counts and |da|/|a| <= 1e-11, mixed walk within the usual bars; equal
lengths reproduce the single-length FP64 result bit for bit; batches of
boxes with and without lengths equal the alone runs; group lists refuse
per-particle lengths; a non-positive length is reported."""
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


def _lengths(n, base, seed):
    """Two populations: 30 % with 5x the base length, the rest at it (x0.8-1.2)."""
    rng = np.random.default_rng(seed)
    return base * np.where(rng.random(n) < 0.3, 5.0, 1.0) * rng.uniform(0.8, 1.2, n)


def _cases():
    rng = np.random.default_rng(55)
    out = []
    w = synth.mixture32k()
    out.append(("mixture32k", w.pos, w.mass, 1.0, w.params.as_dict()))
    n = 8003
    pos = synth.wrap(np.concatenate([rng.random((n - n // 2, 3)), 0.2 + 0.01 * rng.standard_normal((n // 2, 3))]))
    out.append(("clustered8003_lm16", pos, rng.uniform(0.5, 1.5, n) / n, 1.0,
                synth.scale_free_params(n, leaf_max=16).as_dict()))
    pos = rng.normal(size=(3000, 3)) * 0.3
    out.append(("newton3000", pos, np.full(3000, 1 / 3000), 1.0,
                dict(G=1.0, eps=0.01, r_s=0.0, r_cut=0.0, theta=0.6, periodic=0, leaf_max=8)))
    return out


CASES = _cases()


def _run(og, pos, mass, box, prm, prec, eps=None, a_old=None):
    p = dict(prm)
    t_eps = None
    if eps is not None:
        t_eps = _dev(eps)
        p["eps_particle"] = t_eps
    tree = og.Tree(_dev(pos), _dev(mass), box, p, stream=torch.cuda.current_stream())
    a, pot, n = tree.force(precision=prec, with_counts=True, a_old=None if a_old is None else _dev(a_old))
    torch.cuda.synchronize()
    st = tree.status()
    tree.close()
    return a.cpu().numpy(), pot.cpu().numpy(), n.cpu().numpy(), st


@pytest.mark.parametrize("soft", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_per_particle_lengths_match_oracle(og_mod, oracle_mod, case, soft):
    name, pos, mass, box, prm = case
    prm = dict(prm, softening=soft)
    eps = _lengths(pos.shape[0], prm["eps"], 3)
    _note("softening lengths %s kernel %d" % (name, soft))
    op = oracle_mod.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic", "leaf_max",
                                                  "softening")})
    acc, pot, nint = oracle_mod.tree_force(pos, mass, box, op, eps=eps)
    a64, p64, n64, st = _run(og_mod, pos, mass, box, prm, "fp64", eps)
    assert st == 0
    assert np.array_equal(n64, nint)
    e64 = _rel(a64, acc)
    assert e64.max() <= 1e-11 or (np.percentile(e64, 99.9) <= 1e-12 and e64.max() <= 1e-9)
    assert np.all(np.abs(p64 - pot) <= 1e-12 * np.abs(pot) + 1e-300)
    a32, p32, n32, _ = _run(og_mod, pos, mass, box, prm, "mixed", eps)
    e = _rel(a32, acc)
    assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2
    assert (n32 != nint).mean() <= 0.01


def test_equal_lengths_reproduce_single_length(og_mod):
    name, pos, mass, box, prm = CASES[0]
    eps = np.full(pos.shape[0], prm["eps"])
    for soft in (0, 1):
        q = dict(prm, softening=soft)
        a, p, n, _ = _run(og_mod, pos, mass, box, q, "fp64")
        ae, pe, ne, _ = _run(og_mod, pos, mass, box, q, "fp64", eps)
        assert np.array_equal(a, ae) and np.array_equal(p, pe) and np.array_equal(n, ne)
        a, _, n, _ = _run(og_mod, pos, mass, box, q, "mixed")
        ae, _, ne, _ = _run(og_mod, pos, mass, box, q, "mixed", eps)
        assert np.abs(a - ae).max() <= 1e-6 * np.abs(a).max()


def test_with_relative_criterion_and_hilbert(og_mod, oracle_mod):
    name, pos, mass, box, prm = CASES[0]
    eps = _lengths(pos.shape[0], prm["eps"], 4)
    prm = dict(prm, softening=1, criterion=1, alpha=0.003, curve=1)
    op = oracle_mod.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic", "leaf_max",
                                                  "softening", "criterion", "alpha", "curve")})
    a_old = oracle_mod.tree_force(pos, mass, box, oracle_mod.Params(**{**op.__dict__, "criterion": 0}), eps=eps)[0]
    acc, pot, nint = oracle_mod.tree_force(pos, mass, box, op, a_old=a_old, eps=eps)
    a64, _, n64, _ = _run(og_mod, pos, mass, box, prm, "fp64", eps, a_old)
    assert np.array_equal(n64, nint)
    assert _rel(a64, acc).max() <= 1e-11
    a32, _, _, _ = _run(og_mod, pos, mass, box, prm, "mixed", eps, a_old)
    e = _rel(a32, acc)
    assert np.median(e) <= 1e-3 and np.percentile(e, 99) <= 1e-2


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_with_and_without_lengths_equals_alone(og_mod, prec):
    items, keep = [], []
    for b, (name, pos, mass, box, prm) in enumerate(CASES):
        eps = _lengths(pos.shape[0], prm["eps"], 10 + b) if b != 1 else None
        items.append((pos, mass, box, prm, eps))
    alone = [_run(og_mod, pos, mass, box, prm, prec, eps)[:2] for pos, mass, box, prm, eps in items]
    bitems = []
    for pos, mass, box, prm, eps in items:
        p = dict(prm)
        if eps is not None:
            t = _dev(eps)
            keep.append(t)
            p["eps_particle"] = t
        bitems.append((_dev(pos), _dev(mass), box, p))
    bt = og_mod.Batch(bitems, stream=torch.cuda.current_stream(), precision=prec)
    outs = bt.force()
    torch.cuda.synchronize()
    assert bt.status() == 0
    for (a, p), (ga, gp) in zip(alone, outs):
        assert np.array_equal(ga.cpu().numpy(), a) and np.array_equal(gp.cpu().numpy(), p)
    bt.close()


def test_group_lists_refuse_lengths_and_bad_lengths_are_reported(og_mod):
    name, pos, mass, box, prm = CASES[0]
    eps = _lengths(pos.shape[0], prm["eps"], 5)
    with pytest.raises(og_mod.OgError) as ei:
        og_mod.Tree(_dev(pos), _dev(mass), box, dict(prm, lists="group", eps_particle=_dev(eps)),
                    stream=torch.cuda.current_stream())
    assert ei.value.code == og_mod.OG_EUNSUPPORTED
    eps[17] = 0.0
    te = _dev(eps)
    tree = og_mod.Tree(_dev(pos), _dev(mass), box, dict(prm, eps_particle=te), stream=torch.cuda.current_stream())
    assert tree.status() == og_mod.OG_ERANGE
    tree.close()

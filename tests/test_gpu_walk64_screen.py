"""The screened FP64 walk (node tests screened in FP32, the FP64 walk's own
tests wherever the FP32 value cannot settle the outcome) against the plain
FP64 walk, which makes every test in FP64 (OG_WALK64_PLAIN=1): accelerations,
potentials and interaction counts must be the same to the bit (paper, "Tree
walk": the decisions and the FP64 sums are those of the walk rules).  The
cases cover the kernel's branches: periodic groups that take no minimum
image below level 1 and groups that do (per-group reduction and per-lane
images), open boundaries with a cutoff and without one, boxes the screen
does not cover (theta > 1, a root cube far from the origin), the library
erfc tail, spline softening, the relative criterion, per-particle softening
lengths, big and coincident leaves, trees of a few particles, Hilbert keys,
target lists, batches of boxes (one with a spline box among Plummer boxes),
and 40 generated inputs with coincident points and coordinates on cell faces
and at the periodic wrap.  Parity with the oracle is covered by the FP64
parity tests, which run this walk by default."""
import sys

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

from paper_2609_17658_amd import synth
from prop_inputs import configs

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


def _fp64(og, pos, mass, box, prm, targets=None):
    prm = dict(prm)
    eps = prm.pop("eps_lengths", None)
    te = None
    if eps is not None:  # per-particle softening lengths (kept alive with the tree)
        te = _dev(eps)
        prm["eps_particle"] = te
    tree = og.Tree(_dev(pos), _dev(mass), box, prm, stream=torch.cuda.current_stream())
    tg = None if targets is None else _dev(targets, torch.int64)
    a_old = None
    if prm.get("criterion", 0) == 1:
        # previous accelerations of a spread of magnitudes (both walks get the same)
        rng = np.random.default_rng(5)
        a_old = _dev(rng.standard_normal((pos.shape[0], 3)) * np.exp(rng.uniform(-3.0, 3.0, (pos.shape[0], 1))))
    acc, pot, nint = tree.force(targets=tg, precision="fp64", with_counts=True, a_old=a_old)
    torch.cuda.synchronize()
    out = acc.cpu().numpy(), pot.cpu().numpy(), nint.cpu().numpy()
    assert tree.status() == 0
    tree.close()
    return out


def _cases():
    rng = np.random.default_rng(97)
    out = []
    w = synth.mixture32k()
    base = w.params.as_dict()
    out.append(("mixture32k", w.pos, w.mass, 1.0, base))
    for th in (0.3, 0.7, 1.0, 1.2):
        out.append(("mixture32k_theta%.1f" % th, w.pos, w.mass, 1.0, dict(base, theta=th)))
    out.append(("mixture32k_hilbert", w.pos, w.mass, 1.0, dict(base, curve="hilbert")))
    # r_cut above a quarter box: no group is interior; wide groups take the
    # minimum image per lane
    n = 6000
    pos = synth.wrap(rng.random((n, 3)))
    out.append(("uniform6000_wide_cut", pos, np.full(n, 1.0 / n), 1.0,
                dict(G=1.0, eps=0.002, r_s=0.06, r_cut=0.27, theta=0.5, periodic=1, leaf_max=8)))
    # r_cut > 6 r_s: the library erfc tail
    pos = synth.wrap(np.concatenate([rng.random((4000, 3)), 0.3 + 0.02 * rng.standard_normal((4000, 3))]))
    out.append(("clustered8000_tail", pos, rng.uniform(0.5, 1.5, 8000) / 8000, 1.0,
                dict(G=1.0, eps=0.001, r_s=0.015, r_cut=0.12, theta=0.6, periodic=1, leaf_max=8)))
    # open boundaries, with and without a cutoff, near and far from the origin
    pos = rng.random((5000, 3)) * 7.0 - 3.0
    cut = dict(G=2.0, eps=0.02, r_s=0.2, r_cut=0.9, theta=0.5, periodic=0, leaf_max=8)
    out.append(("open_cut5000", pos, np.full(5000, 1 / 5000), 1.0, cut))
    out.append(("open_cut5000_at10", pos + 10.0, np.full(5000, 1 / 5000), 1.0, cut))
    out.append(("open_cut5000_at1e4", pos + 1.0e4, np.full(5000, 1 / 5000), 1.0, cut))
    pos = rng.normal(size=(3000, 3)) * 0.3
    out.append(("newton3000", pos, np.full(3000, 1 / 3000), 1.0,
                dict(G=1.0, eps=0.01, r_s=0.0, r_cut=0.0, theta=0.6, periodic=0, leaf_max=8)))
    # big leaves and coincident particles (leaves over leaf_max at the
    # deepest level)
    n = 7000
    pos = synth.wrap(rng.random((n, 3)))
    pos[:600] = pos[0]
    pos[600:900] = 0.25
    out.append(("coincident7000_lm32", pos, np.full(n, 1.0 / n), 1.0,
                dict(synth.scale_free_params(n, leaf_max=32).as_dict())))
    # spline softening (read from the box; the node tests do not depend on it)
    out.append(("mixture32k_spline", w.pos, w.mass, 1.0, dict(base, softening=1)))
    out.append(("clustered8000_tail_spline", out[7][1], out[7][2], 1.0, dict(out[7][4], softening=1)))
    # the relative criterion (with theta above 1 too: it is not used), alone
    # and with spline softening, periodic and open
    rel = dict(criterion=1, alpha=0.002)
    out.append(("mixture32k_relative", w.pos, w.mass, 1.0, dict(base, **rel)))
    out.append(("mixture32k_relative_theta1.5", w.pos, w.mass, 1.0, dict(base, theta=1.5, **rel)))
    out.append(("mixture32k_spline_relative", w.pos, w.mass, 1.0, dict(base, softening=1, **rel)))
    out.append(("open_cut5000_relative", out[8][1], out[8][2], 1.0, dict(out[8][4], criterion=1, alpha=0.01)))
    # per-particle lengths (30 % at five times the box's), with the Plummer
    # and spline kernels, with the relative criterion, and in an open box
    lengths = np.full(w.pos.shape[0], base["eps"])
    lengths[rng.random(w.pos.shape[0]) < 0.3] *= 5.0
    out.append(("mixture32k_lengths", w.pos, w.mass, 1.0, dict(base, eps_lengths=lengths)))
    out.append(("mixture32k_lengths_spline", w.pos, w.mass, 1.0, dict(base, softening=1, eps_lengths=lengths)))
    out.append(("mixture32k_lengths_relative", w.pos, w.mass, 1.0, dict(base, eps_lengths=lengths, **rel)))
    nl = out[11][1].shape[0]
    lengths_open = np.where(rng.random(nl) < 0.3, 0.05, 0.01)
    out.append(("newton3000_lengths", out[11][1], out[11][2], 1.0, dict(out[11][4], eps_lengths=lengths_open)))
    # a few particles: leaves at the top two levels
    for n in (2, 5, 17, 70):
        pos = synth.wrap(rng.random((n, 3)))
        out.append(("tiny%d" % n, pos, np.full(n, 1.0 / n), 1.0,
                    dict(G=1.0, eps=0.01, r_s=0.05, r_cut=0.225, theta=0.5, periodic=1, leaf_max=4)))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_screened_equals_plain(og_mod, monkeypatch, case):
    name, pos, mass, box, prm = case
    _note("screened vs plain FP64 walk: %s N=%d" % (name, pos.shape[0]))
    screened = _fp64(og_mod, pos, mass, box, prm)
    monkeypatch.setenv("OG_WALK64_PLAIN", "1")
    plain = _fp64(og_mod, pos, mass, box, prm)
    for x, y in zip(screened, plain):
        assert np.array_equal(x, y)
    assert plain[2].sum() > 0 or pos.shape[0] < 10  # two particles may lie beyond r_cut


def test_screened_target_list_equals_plain(og_mod, monkeypatch):
    name, pos, mass, box, prm = CASES[0]
    tg = np.random.default_rng(3).integers(0, pos.shape[0], 5000)
    _note("screened vs plain FP64 walk: target list of %d" % tg.size)
    screened = _fp64(og_mod, pos, mass, box, prm, targets=tg)
    monkeypatch.setenv("OG_WALK64_PLAIN", "1")
    plain = _fp64(og_mod, pos, mass, box, prm, targets=tg)
    for x, y in zip(screened, plain):
        assert np.array_equal(x, y)


def _batch_items(spline):
    rng = np.random.default_rng(11)
    items = []
    for i, n in enumerate((3000, 9000, 1500)):
        pos = synth.wrap(rng.random((n, 3)))
        prm = synth.scale_free_params(n, theta=0.4 + 0.2 * i).as_dict()
        if spline and i == 1:
            prm["softening"] = 1  # one spline box among Plummer boxes
        items.append((_dev(pos), _dev(np.full(n, 1.0 / n)), 1.0, prm))
    pos = rng.random((2500, 3)) * 3.0
    items.append((_dev(pos), _dev(np.full(2500, 1 / 2500)), 1.0,
                  dict(G=1.0, eps=0.01, r_s=0.1, r_cut=0.45, theta=0.5, periodic=0, leaf_max=8)))
    return items


@pytest.mark.parametrize("spline", [False, True], ids=["plummer", "with_spline_box"])
def test_screened_batch_equals_plain(og_mod, monkeypatch, spline):
    items = _batch_items(spline)
    _note("screened vs plain FP64 walk: batch of %d boxes" % len(items))

    def run():
        b = og_mod.Batch(items, stream=torch.cuda.current_stream(), precision="fp64")
        outs = b.force()
        torch.cuda.synchronize()
        assert b.status() == 0
        res = [(a.cpu().numpy().copy(), p.cpu().numpy().copy()) for a, p in outs]
        b.close()
        return res

    screened = run()
    monkeypatch.setenv("OG_WALK64_PLAIN", "1")
    plain = run()
    for (a1, p1), (a2, p2) in zip(screened, plain):
        assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large,
                                 HealthCheck.function_scoped_fixture])
@given(cfg=configs())
def test_screened_equals_plain_on_generated_inputs(og_mod, monkeypatch, cfg):
    """Coincident points, dyadic coordinates on cell faces (exact ties with
    node thresholds), coordinates 0 and just below the periodic side, theta 0
    to 0.8, leaves of 1 to 16, both curves, open and periodic boxes."""
    _note("screened vs plain FP64 walk: %s" % cfg.label)
    monkeypatch.delenv("OG_WALK64_PLAIN", raising=False)
    screened = _fp64(og_mod, cfg.pos, cfg.mass, cfg.box, cfg.params)
    monkeypatch.setenv("OG_WALK64_PLAIN", "1")
    plain = _fp64(og_mod, cfg.pos, cfg.mass, cfg.box, cfg.params)
    for x, y in zip(screened, plain):
        assert np.array_equal(x, y)

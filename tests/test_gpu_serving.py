"""Serving: requests of different sizes admitted by device-memory footprint
as slots and memory free up, overlapping on the device.  Each request's
result must be the same alone and in the mix (bitwise: same kernels, same
tree, same per-lane walk), and the admitted footprint must never exceed the
budget."""
import sys
import time

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


def _requests(k, seed, nmin=2000, nmax=60000):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        if i % 2:
            g = max(8, int(round(n ** (1 / 3))))
            pos = synth.zeldovich(g, 9000 + i)
        else:
            pos = synth.mixture_box(n, 9000 + i)
        n = pos.shape[0]
        out.append((pos, synth.equal_masses(n), synth.scale_free_params(max(n, 1000)).as_dict()))
    return out


def _alone(og, pos, mass, prm, prec):
    t = og.Tree(torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda"), 1.0, prm,
                stream=torch.cuda.current_stream())
    a, p = t.force(precision=prec)
    torch.cuda.synchronize()
    t.close()
    return a.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_served_equals_alone_and_budget_respected(og_mod, prec):
    reqs = _requests(14, 21)
    p0 = og_mod.make_params(reqs[0][2])
    sizes = [og_mod.og_tree_workspace_bound(r[0].shape[0], p0) for r in reqs]
    budget = int(max(sizes) * 2.2)          # forces queueing
    srv = og_mod.Server(budget, max_slots=3)
    dev = [(torch.as_tensor(p, device="cuda"), torch.as_tensor(m, device="cuda"), prm) for p, m, prm in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(p, m, 1.0, prm, precision=prec) for p, m, prm in dev]
    seen_pending = False
    done = set()
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        st = srv.stats()
        assert st["reserved"] <= budget
        seen_pending |= st["pending"] > 0
        for t in tickets:
            if t not in done and srv.poll(t)[0]:
                done.add(t)
                a, p = srv.result(t)
                srv.release(t)  # frees memory for the queue
                i = tickets.index(t)
                ra, rp = _alone(og_mod, reqs[i][0], reqs[i][1], reqs[i][2], prec)
                assert np.array_equal(a.cpu().numpy(), ra), i
                assert np.array_equal(p.cpu().numpy(), rp), i
        time.sleep(0.001)
    assert len(done) == len(tickets)
    assert seen_pending
    assert srv.stats() == {"reserved": 0, "in_flight": 0, "pending": 0}
    srv.close()


def test_latencies_and_errors(og_mod):
    reqs = _requests(6, 22)
    srv = og_mod.Server(256 << 20, max_slots=2)
    dev = [(torch.as_tensor(p, device="cuda"), torch.as_tensor(m, device="cuda"), prm) for p, m, prm in reqs]
    tickets = [srv.submit(p, m, 1.0, prm) for p, m, prm in dev]
    for t in tickets:
        srv.wait(t)
        done, ta, td = srv.poll(t)
        assert done and td >= ta > 0
    with pytest.raises(og_mod.OgError) as e:
        srv.poll(987654)
    assert e.value.code == og_mod.OG_ENOTFOUND
    big = torch.zeros((2_000_000, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(og_mod.OgError) as e:
        srv.submit(big, torch.ones(2_000_000, dtype=torch.float64, device="cuda"), 1.0,
                   synth.scale_free_params(2_000_000).as_dict())
    assert e.value.code == og_mod.OG_EBUSY
    for t in tickets:
        srv.release(t)
    srv.close()

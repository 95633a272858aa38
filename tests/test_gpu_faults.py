"""Host-forced faults: the error paths of the library, taken without any
device fault.  OG_FAULT_ALLOC=k fails the k-th device allocation and
OG_FAULT_LAUNCH=k the k-th build or walk enqueue, on the host, before
anything is enqueued; the call must return OG_ENOMEM / OG_EDEVICE with a
message, write no handle, and leave the library usable: the next call with
the knob cleared gives the normal (oracle-checked) result."""
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


def _small():
    pos = synth.mixture_box(3000, 61)
    mass = synth.equal_masses(3000)
    prm = synth.scale_free_params(3000).as_dict()
    return pos, mass, prm


def _oracle_acc(oracle_mod, pos, mass, prm):
    op = oracle_mod.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic",
                                                  "leaf_max")})
    return oracle_mod.tree_force(pos, mass, 1.0, op)[0]


def test_build_allocation_failure_returns_enomem(og_mod, oracle_mod, monkeypatch):
    pos, mass, prm = _small()
    tp, tm = torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda")
    lib = og_mod.load()
    params = og_mod.make_params(prm, precision="fp64", stream=torch.cuda.current_stream())
    monkeypatch.setenv("OG_FAULT_ALLOC", "1")
    h = ctypes.c_void_p(12345)
    rc = lib.og_tree_build(ctypes.c_void_p(tp.data_ptr()), ctypes.c_void_p(tm.data_ptr()), 3000, 1.0,
                           ctypes.byref(params), ctypes.byref(h))
    msg = lib.og_last_error().decode()
    _note("forced build allocation failure: rc %d, %r" % (rc, msg))
    assert rc == og_mod.OG_ENOMEM and "OG_FAULT_ALLOC" in msg
    assert h.value == 12345            # no handle written
    monkeypatch.delenv("OG_FAULT_ALLOC")
    t = og_mod.Tree(tp, tm, 1.0, prm, precision="fp64", stream=torch.cuda.current_stream())
    a, _ = t.force()
    torch.cuda.synchronize()
    assert t.status() == 0
    ra = _oracle_acc(oracle_mod, pos, mass, prm)
    e = np.linalg.norm(a.cpu().numpy() - ra, axis=1) / np.linalg.norm(ra, axis=1)
    assert e.max() <= 1e-11
    t.close()


def test_caller_workspace_takes_no_allocation(og_mod, monkeypatch):
    """With a caller workspace the build allocates nothing, so the knob does
    not reach it."""
    pos, mass, prm = _small()
    tp, tm = torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda")
    p = og_mod.make_params(prm)
    ws = torch.empty(og_mod.og_tree_workspace_bound(3000, p), dtype=torch.uint8, device="cuda")
    monkeypatch.setenv("OG_FAULT_ALLOC", "1")
    t = og_mod.Tree(tp, tm, 1.0, prm, workspace=ws, stream=torch.cuda.current_stream())
    t.force()
    torch.cuda.synchronize()
    assert t.status() == 0
    t.close()


def test_launch_failure_returns_edevice(og_mod, monkeypatch):
    pos, mass, prm = _small()
    tp, tm = torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda")
    monkeypatch.setenv("OG_FAULT_LAUNCH", "1")
    with pytest.raises(og_mod.OgError) as e:
        og_mod.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream())
    assert e.value.code == og_mod.OG_EDEVICE
    monkeypatch.setenv("OG_FAULT_LAUNCH", "2")   # a new value restarts the count: build ok, walk fails
    t = og_mod.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream())
    with pytest.raises(og_mod.OgError) as e:
        t.force()
    assert e.value.code == og_mod.OG_EDEVICE
    a, _ = t.force()                              # the third enqueue goes through
    torch.cuda.synchronize()
    assert t.status() == 0 and torch.isfinite(a).all()
    t.close()


def test_subset_scratch_failure(og_mod, monkeypatch):
    pos, mass, prm = _small()
    tp, tm = torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda")
    t = og_mod.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream())
    full, _ = t.force()
    idx = torch.arange(0, 3000, 7, dtype=torch.int64, device="cuda")
    monkeypatch.setenv("OG_FAULT_ALLOC", "1")
    with pytest.raises(og_mod.OgError) as e:
        t.force(targets=idx)
    assert e.value.code == og_mod.OG_ENOMEM
    monkeypatch.delenv("OG_FAULT_ALLOC")
    sub, _ = t.force(targets=idx)
    torch.cuda.synchronize()
    assert torch.equal(sub, full[idx])
    t.close()


def test_mesh_and_server_allocation_failures(og_mod, monkeypatch):
    monkeypatch.setenv("OG_FAULT_ALLOC", "1")
    with pytest.raises(og_mod.OgError) as e:
        og_mod.PM(32, 1.0, 1.0, 0.04)
    assert e.value.code == og_mod.OG_ENOMEM
    monkeypatch.setenv("OG_FAULT_ALLOC", "01")   # another value: count restarts
    with pytest.raises(og_mod.OgError) as e:
        og_mod.Server(64 << 20, max_slots=2)
    assert e.value.code == og_mod.OG_ENOMEM
    monkeypatch.delenv("OG_FAULT_ALLOC")
    srv = og_mod.Server(64 << 20, max_slots=2)
    srv.close()
    mesh = og_mod.PM(32, 1.0, 1.0, 0.04)
    mesh.close()

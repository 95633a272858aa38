"""OG_TRACE=1 (roctx ranges around API calls and build stages) changes
nothing but the markers: a child process with tracing on builds and walks
the same box, and its forces equal this process's to the bit."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2609_17658_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2609_17658_amd import og, synth
pos = synth.mixture_box(20000, 91)
prm = synth.scale_free_params(20000).as_dict()
tp = torch.as_tensor(pos, device="cuda")
tm = torch.as_tensor(synth.equal_masses(20000), device="cuda")
out = []
for prec in ("mixed", "fp64"):
    t = og.Tree(tp, tm, 1.0, dict(prm, precision=prec), stream=torch.cuda.current_stream())
    a, p = t.force()
    t.validate()
    out += [a.cpu().numpy(), p.cpu().numpy()]
    t.close()
np.savez(sys.argv[2], *out)
print("child done", flush=True)
"""


def _forces(og):
    pos = synth.mixture_box(20000, 91)
    prm = synth.scale_free_params(20000).as_dict()
    tp = torch.as_tensor(pos, device="cuda")
    tm = torch.as_tensor(synth.equal_masses(20000), device="cuda")
    out = []
    for prec in ("mixed", "fp64"):
        t = og.Tree(tp, tm, 1.0, dict(prm, precision=prec), stream=torch.cuda.current_stream())
        a, p = t.force()
        out += [a.cpu().numpy(), p.cpu().numpy()]
        t.close()
    return out


def test_trace_ranges_leave_results_unchanged(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_17658_amd import og
    ref = _forces(og)
    dst = str(tmp_path / "traced.npz")
    env = dict(os.environ, OG_TRACE="1")
    print("child with OG_TRACE=1", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, dst], env=env, capture_output=True, text=True,
                       timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    got = np.load(dst)
    for i, want in enumerate(ref):
        assert np.array_equal(got["arr_%d" % i], want), i

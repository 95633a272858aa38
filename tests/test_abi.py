"""Host-side checks of the C ABI library (no GPU work): it loads, exports
every symbol include/og.h declares, and rejects bad arguments before it
touches the device."""
import ctypes
import os
import re

import pytest

from paper_2609_17658_amd import og

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "og.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(og_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = og.load()
    names = _declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps every one of them
    assert set(names) == set(og._SIGNATURES)


def test_params_default_and_struct_layout():
    p = og.og_params_default()
    assert p.struct_size == ctypes.sizeof(og.og_params) == 128
    assert (p.G, p.eps, p.r_s, p.r_cut, p.theta, p.alpha) == (1.0, 0.0, 0.0, 0.0, 0.5, 0.0)
    assert (p.periodic, p.leaf_max, p.precision, p.group_max, p.walk_list_cap) == (1, 8, og.OG_PREC_MIXED, 0, 0)
    assert (p.softening, p.criterion, p.curve) == (og.OG_SOFT_PLUMMER, og.OG_OPEN_BH, og.OG_CURVE_MORTON)
    assert ctypes.sizeof(og.og_box) == 8 + 8 + 8 + 8 + 128 + 8 + 8
    assert p.eps_particle is None
    assert p.lists == og.OG_LISTS_TARGET
    assert ctypes.sizeof(og.og_force_opts) == 32


def test_workspace_bound_monotone_and_rejects_bad_input():
    p = og.og_params_default()
    b1 = og.og_tree_workspace_bound(1000, p)
    b2 = og.og_tree_workspace_bound(2000, p)
    assert 0 < b1 < b2
    # per particle: sorted data, keys and at most N(1+21/(leaf_max+1)) nodes
    # of about 180 B each (topology, moments, walk records, FP64 centres)
    assert b2 / 2000 < 700
    assert og.og_tree_workspace_bound(0, p) == 0
    assert og.og_tree_workspace_bound(1 << 27, p) == 0
    p.leaf_max = 0
    assert og.og_tree_workspace_bound(1000, p) == 0


@pytest.mark.parametrize("field,value", [
    ("eps", -1.0), ("theta", -0.1), ("leaf_max", 0), ("leaf_max", 5000), ("group_max", 65),
    ("precision", 7), ("r_s", 0.0), ("r_cut", 0.6), ("walk_list_cap", 12),
    ("softening", 2), ("criterion", 3), ("curve", 2), ("lists", 2),
    ("softening", 1),   # spline with eps = 0
    ("criterion", 1),   # relative criterion with alpha = 0
])
def test_build_rejects_bad_params_on_host(field, value):
    lib = og.load()
    p = og.make_params(r_s=0.01)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    rc = lib.og_tree_build(None, None, 100, 1.0, ctypes.byref(p), ctypes.byref(h))
    assert rc == og.OG_EINVAL
    assert lib.og_last_error()
    assert not h.value


def test_build_rejects_bad_sizes_and_struct_size():
    lib = og.load()
    p = og.make_params(r_s=0.01)
    h = ctypes.c_void_p()
    assert lib.og_tree_build(None, None, 0, 1.0, ctypes.byref(p), ctypes.byref(h)) == og.OG_EINVAL
    assert lib.og_tree_build(None, None, 10, 0.0, ctypes.byref(p), ctypes.byref(h)) == og.OG_EINVAL
    p.struct_size = 12
    assert lib.og_tree_build(None, None, 10, 1.0, ctypes.byref(p), ctypes.byref(h)) == og.OG_EINVAL
    assert b"struct_size" in lib.og_last_error()


def test_strerror_codes():
    lib = og.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.og_strerror(code)
    assert lib.og_strerror(0) == b"ok"


def test_header_layout_matches_binding(tmp_path):
    """The C compiler's layout of og.h's structs equals the binding's."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = {"og_params": [f[0] for f in og.og_params._fields_],
              "og_force_opts": [f[0] for f in og.og_force_opts._fields_],
              "og_box": [f[0] for f in og.og_box._fields_],
              "og_targets": [f[0] for f in og.og_targets._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "og.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for f in fs:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, f, st, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for st, fs in fields.items():
        cls = getattr(og, st)
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fs:
            assert int(got["%s.%s" % (st, f)]) == getattr(cls, f).offset, (st, f)


def test_build_rejects_host_softening_lengths():
    import numpy as np
    lib = og.load()
    eps = np.full(100, 0.01)
    p = og.make_params(r_s=0.01, eps_particle=eps.ctypes.data)
    h = ctypes.c_void_p()
    assert lib.og_tree_build(None, None, 100, 1.0, ctypes.byref(p), ctypes.byref(h)) == og.OG_EINVAL


def test_validate_rejects_null_and_names_its_error():
    lib = og.load()
    assert lib.og_tree_validate(None) == og.OG_EINVAL
    assert lib.og_strerror(og.OG_ECORRUPT) == b"tree invariant violated"

"""Python binding of the C ABI in ``include/og.h`` (ctypes; marshalling only).

Functions keep the C names (``og_tree_build``, ``og_tree_force``, ...).
Arrays are torch CUDA/HIP tensors; only their device pointers cross the
ABI, and every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: if ``libog.so`` is missing or no GPU is present,
the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import asdict, is_dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libog.so")

OG_OK, OG_EINVAL, OG_ERANGE, OG_ENOMEM, OG_EDEVICE, OG_EBUSY, OG_EUNSUPPORTED, OG_ENOTFOUND, OG_ECORRUPT = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
OG_PREC_FP64, OG_PREC_MIXED = 0, 1
PRECISIONS = {"fp64": OG_PREC_FP64, "mixed": OG_PREC_MIXED, OG_PREC_FP64: OG_PREC_FP64,
              OG_PREC_MIXED: OG_PREC_MIXED}
OG_SOFT_PLUMMER, OG_SOFT_SPLINE = 0, 1
OG_OPEN_BH, OG_OPEN_RELATIVE = 0, 1
SOFTENINGS = {"plummer": OG_SOFT_PLUMMER, "spline": OG_SOFT_SPLINE, 0: 0, 1: 1}
CRITERIA = {"bh": OG_OPEN_BH, "relative": OG_OPEN_RELATIVE, 0: 0, 1: 1}
OG_CURVE_MORTON, OG_CURVE_HILBERT = 0, 1
CURVES = {"morton": OG_CURVE_MORTON, "hilbert": OG_CURVE_HILBERT, 0: 0, 1: 1}
OG_LISTS_TARGET, OG_LISTS_GROUP = 0, 1
OG_NOALLOC_MAX_TARGETS = 1048576
LISTS = {"target": OG_LISTS_TARGET, "group": OG_LISTS_GROUP, 0: 0, 1: 1}


class og_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("G", ctypes.c_double), ("eps", ctypes.c_double),
                ("r_s", ctypes.c_double), ("r_cut", ctypes.c_double), ("theta", ctypes.c_double),
                ("alpha", ctypes.c_double), ("periodic", ctypes.c_int32), ("leaf_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("group_max", ctypes.c_int32),
                ("walk_list_cap", ctypes.c_int32), ("softening", ctypes.c_int32),
                ("criterion", ctypes.c_int32), ("curve", ctypes.c_int32), ("lists", ctypes.c_int32),
                ("eps_particle", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class og_targets(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_void_p), ("M", ctypes.c_int64)]


class og_force_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("n_inter", ctypes.c_void_p), ("a_old", ctypes.c_void_p)]


class og_box(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("mass", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("box", ctypes.c_double), ("params", og_params), ("acc", ctypes.c_void_p),
                ("pot", ctypes.c_void_p)]


# Every symbol og.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_SIGNATURES = {
    "og_params_default": (None, [ctypes.POINTER(og_params)]),
    "og_tree_workspace_bound": (ctypes.c_size_t, [ctypes.c_int64, ctypes.POINTER(og_params)]),
    "og_tree_build": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(og_params),
                                     ctypes.POINTER(_P)]),
    "og_tree_force": (ctypes.c_int, [_P, ctypes.POINTER(og_targets), _P, _P]),
    "og_tree_force_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(og_targets), _P, _P]),
    "og_tree_force_ex": (ctypes.c_int, [_P, ctypes.POINTER(og_targets), ctypes.POINTER(og_force_opts),
                                        _P, _P]),
    "og_tree_force_active": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(og_force_opts), _P, _P,
                                            _P]),
    "og_tree_status": (ctypes.c_int, [_P]),
    "og_tree_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "og_tree_export": (ctypes.c_int, [_P] * 9),
    "og_tree_validate": (ctypes.c_int, [_P]),
    "og_tree_free": (ctypes.c_int, [_P]),
    "og_batch_build": (ctypes.c_int, [ctypes.POINTER(og_box), ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "og_batch_force": (ctypes.c_int, [_P]),
    "og_batch_graph_replay": (ctypes.c_int, [_P]),
    "og_batch_status": (ctypes.c_int, [_P]),
    "og_batch_free": (ctypes.c_int, [_P]),
    "og_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_P)]),
    "og_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(og_box), ctypes.POINTER(ctypes.c_uint64)]),
    "og_server_progress": (ctypes.c_int, [_P]),
    "og_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "og_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "og_server_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "og_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "og_server_destroy": (ctypes.c_int, [_P]),
    "og_pm_workspace_bound": (ctypes.c_size_t, [ctypes.c_int32]),
    "og_pm_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P,
                                    ctypes.POINTER(_P)]),
    "og_pm_force": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P, ctypes.c_int32]),
    "og_pm_force_tree": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32]),
    "og_pm_free": (ctypes.c_int, [_P]),
    "og_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "og_last_error": (ctypes.c_char_p, []),
}

_lib = None


class OgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libog.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libog.so not built (run __graft_entry__.build() or "
                              "python -m paper_2609_17658_amd.build): %s" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _strerror(code):
    try:
        return load().og_strerror(code).decode()
    except Exception:  # noqa: BLE001 - message only
        return "error"


def _check(code):
    if code != OG_OK:
        raise OgError(code, load().og_last_error().decode())
    return code


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_params(params=None, stream=None, workspace=None, **kw) -> og_params:
    """og_params from og_params_default() updated by a dict/dataclass and keywords."""
    p = og_params()
    load().og_params_default(ctypes.byref(p))
    d = {}
    if params is not None:
        d.update(asdict(params) if is_dataclass(params) else dict(params))
    d.update(kw)
    for k, v in d.items():
        if k == "precision":
            v = PRECISIONS[v]
        elif k == "softening":
            v = SOFTENINGS[v]
        elif k == "criterion":
            v = CRITERIA[v]
        elif k == "curve":
            v = CURVES[v]
        elif k == "lists":
            v = LISTS[v]
        elif k == "eps_particle":
            v = None if v is None else (v if isinstance(v, int) else v.data_ptr())
        setattr(p, k, v)
    p.stream = _stream_handle(stream)
    if workspace is not None:
        p.workspace = _ptr(workspace)
        p.workspace_bytes = workspace.numel() * workspace.element_size()
    return p


def _check_pos_mass(pos, mass):
    import torch
    if not (pos.is_cuda and mass.is_cuda):
        raise ValueError("pos and mass must be device tensors")
    if pos.dtype != torch.float64 or mass.dtype != torch.float64:
        raise ValueError("pos and mass must be float64")
    if pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous() or not mass.is_contiguous():
        raise ValueError("pos must be a contiguous [N,3] tensor, mass a contiguous [N] tensor")
    if mass.shape[0] != pos.shape[0]:
        raise ValueError("pos and mass lengths differ")


# ------------------------------------------------------ C-named calls --

def og_params_default() -> og_params:
    return make_params()


def og_tree_workspace_bound(N: int, params: og_params) -> int:
    return int(load().og_tree_workspace_bound(int(N), ctypes.byref(params)))


def og_tree_build(pos, mass, N: int, box: float, params: og_params) -> ctypes.c_void_p:
    _check_pos_mass(pos, mass)
    h = ctypes.c_void_p()
    _check(load().og_tree_build(_ptr(pos), _ptr(mass), int(N), float(box), ctypes.byref(params),
                                ctypes.byref(h)))
    return h


def og_tree_force(tree, targets, acc, pot, precision=None, stream=None, n_inter=None, a_old=None):
    """targets: None (all) or an int64 device tensor of caller-order indices;
    a_old: previous accelerations [N,3] (device, caller order) for the
    relative criterion."""
    tg = None
    if targets is not None:
        tg = og_targets(_ptr(targets), int(targets.numel()))
    opts = og_force_opts(ctypes.sizeof(og_force_opts), -1 if precision is None else PRECISIONS[precision],
                         _stream_handle(stream), _ptr(n_inter), _ptr(a_old))
    _check(load().og_tree_force_ex(tree, ctypes.byref(tg) if tg is not None else None,
                                   ctypes.byref(opts), _ptr(acc), _ptr(pot)))


def og_tree_force_noalloc(tree, targets, acc, pot):
    """og_tree_force with the target scratch in the library's fixed device
    array (no allocation); targets: None (all) or an int64 device tensor of
    at most OG_NOALLOC_MAX_TARGETS caller-order indices."""
    tg = None if targets is None else og_targets(_ptr(targets), int(targets.numel()))
    _check(load().og_tree_force_noalloc(tree, ctypes.byref(tg) if tg is not None else None, _ptr(acc), _ptr(pot)))


def og_tree_force_active(tree, bin, level, acc, pot, precision=None, stream=None, n_inter=None, a_old=None,
                         n_active=None):
    """bin: int8 device tensor [N] (caller order); particles with bin <= level
    get acc/pot (caller order [N]); others' entries are left unchanged."""
    opts = og_force_opts(ctypes.sizeof(og_force_opts), -1 if precision is None else PRECISIONS[precision],
                         _stream_handle(stream), _ptr(n_inter), _ptr(a_old))
    _check(load().og_tree_force_active(tree, _ptr(bin), int(level), ctypes.byref(opts), _ptr(acc), _ptr(pot),
                                       _ptr(n_active)))


def og_tree_status(tree) -> int:
    return load().og_tree_status(tree)


def og_tree_stats(tree):
    n = ctypes.c_int64()
    d = ctypes.c_int32()
    b = ctypes.c_size_t()
    _check(load().og_tree_stats(tree, ctypes.byref(n), ctypes.byref(d), ctypes.byref(b)))
    return {"n_nodes": n.value, "depth": d.value, "bytes": b.value}


def og_tree_export(tree, N: int):
    import numpy as np
    nn = og_tree_stats(tree)["n_nodes"]
    out = {
        "keys": np.empty(N, np.uint64), "perm": np.empty(N, np.uint32),
        "first": np.empty(nn, np.uint32), "count": np.empty(nn, np.uint32),
        "level": np.empty(nn, np.uint8), "skip": np.empty(nn, np.uint32),
        "parent": np.empty(nn, np.uint32), "node_m_com": np.empty((nn, 4), np.float64),
    }
    args = [out[k].ctypes.data_as(ctypes.c_void_p) for k in
            ("keys", "perm", "first", "count", "level", "skip", "parent", "node_m_com")]
    _check(load().og_tree_export(tree, *args))
    return out


def og_tree_validate(tree):
    """Host-side check of the tree's invariants; raises OgError (code
    OG_ECORRUPT, message naming the first violation) when one fails."""
    return _check(load().og_tree_validate(tree))


def og_tree_free(tree):
    if tree:
        _check(load().og_tree_free(tree))


def og_batch_build(boxes: list, stream=None) -> ctypes.c_void_p:
    arr = (og_box * len(boxes))(*boxes)
    h = ctypes.c_void_p()
    _check(load().og_batch_build(arr, len(boxes), _stream_handle(stream), ctypes.byref(h)))
    return h


def og_batch_force(b):
    _check(load().og_batch_force(b))


def og_batch_graph_replay(b):
    _check(load().og_batch_graph_replay(b))


def og_batch_status(b) -> int:
    return load().og_batch_status(b)


def og_batch_free(b):
    if b:
        _check(load().og_batch_free(b))


def og_server_create(hbm_budget_bytes: int, max_slots: int):
    h = ctypes.c_void_p()
    _check(load().og_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
    return h


def og_server_submit(s, req: og_box) -> int:
    t = ctypes.c_uint64()
    _check(load().og_server_submit(s, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def og_server_progress(s):
    _check(load().og_server_progress(s))


def og_server_poll(s, ticket: int):
    d = ctypes.c_int32()
    ta = ctypes.c_double()
    td = ctypes.c_double()
    _check(load().og_server_poll(s, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(ta),
                                 ctypes.byref(td)))
    return bool(d.value), ta.value, td.value


def og_server_wait(s, ticket: int):
    _check(load().og_server_wait(s, ctypes.c_uint64(ticket)))


def og_server_release(s, ticket: int):
    _check(load().og_server_release(s, ctypes.c_uint64(ticket)))


def og_server_stats(s):
    r = ctypes.c_size_t()
    a = ctypes.c_int32()
    p = ctypes.c_int32()
    _check(load().og_server_stats(s, ctypes.byref(r), ctypes.byref(a), ctypes.byref(p)))
    return {"reserved": r.value, "in_flight": a.value, "pending": p.value}


def og_server_destroy(s):
    if s:
        _check(load().og_server_destroy(s))


# ------------------------------------------------------- conveniences --

class Tree:
    """Owning wrapper: builds on construction, frees on close()/GC."""

    def __init__(self, pos, mass, box: float, params=None, stream=None, workspace=None, **kw):
        self.N = int(pos.shape[0])
        self.device = pos.device
        self.params = make_params(params, stream=stream, workspace=workspace, **kw)
        eps_t = kw.get("eps_particle")
        if eps_t is None and isinstance(params, dict):
            eps_t = params.get("eps_particle")
        self._keep = (pos, mass, workspace, eps_t)
        self.handle = og_tree_build(pos, mass, self.N, box, self.params)

    def force(self, targets=None, precision=None, with_pot=True, with_counts=False, stream=None,
              acc=None, pot=None, a_old=None):
        import torch
        M = self.N if targets is None else int(targets.numel())
        if acc is None:
            acc = torch.empty((M, 3), dtype=torch.float64, device=self.device)
        if with_pot and pot is None:
            pot = torch.empty(M, dtype=torch.float64, device=self.device)
        nint = torch.empty(M, dtype=torch.int64, device=self.device) if with_counts else None
        og_tree_force(self.handle, targets, acc, pot if with_pot else None, precision=precision,
                      stream=stream, n_inter=nint, a_old=a_old)
        if with_counts:
            return acc, pot, nint
        return acc, pot

    def force_active(self, bin, level, acc, pot=None, precision=None, n_inter=None, a_old=None,
                     n_active=None, stream=None):
        """Forces on particles with bin <= level into acc/pot (caller order,
        [N]); other entries are not written."""
        og_tree_force_active(self.handle, bin, level, acc, pot, precision=precision, stream=stream,
                             n_inter=n_inter, a_old=a_old, n_active=n_active)
        return acc, pot

    def status(self) -> int:
        return og_tree_status(self.handle)

    def stats(self):
        return og_tree_stats(self.handle)

    def export(self):
        return og_tree_export(self.handle, self.N)

    def validate(self):
        return og_tree_validate(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            og_tree_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def box_struct(pos, mass, box, params, acc, pot=None) -> og_box:
    _check_pos_mass(pos, mass)
    return og_box(_ptr(pos), _ptr(mass), int(pos.shape[0]), float(box),
                  params if isinstance(params, og_params) else make_params(params),
                  _ptr(acc), _ptr(pot))


class Batch:
    """B independent boxes built and walked by one set of launches."""

    def __init__(self, items, stream=None, precision="mixed", group_max=0, walk_list_cap=0):
        """items: list of (pos, mass, box, params) with device tensors."""
        import torch
        self.outputs = []
        structs = []
        for pos, mass, box, params in items:
            acc = torch.empty((pos.shape[0], 3), dtype=torch.float64, device=pos.device)
            pot = torch.empty(pos.shape[0], dtype=torch.float64, device=pos.device)
            p = make_params(params, precision=precision, group_max=group_max,
                            walk_list_cap=walk_list_cap)
            structs.append(box_struct(pos, mass, box, p, acc, pot))
            self.outputs.append((acc, pot))
        self._keep = items
        self.handle = og_batch_build(structs, stream=stream)

    def force(self):
        og_batch_force(self.handle)
        return self.outputs

    def replay(self):
        og_batch_graph_replay(self.handle)
        return self.outputs

    def status(self) -> int:
        return og_batch_status(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            og_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Server:
    """Continuous-batching server (og_server_*): requests are admitted as
    memory and stream slots free up, and trees stay resident until release."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4):
        self.handle = og_server_create(hbm_budget_bytes, max_slots)
        self._keep = {}

    def submit(self, pos, mass, box, params, precision="mixed", group_max=0, walk_list_cap=0,
               acc=None, pot=None, stream=None):
        """stream: where pos/mass are written (default: torch's current
        stream); the request's build waits for the work enqueued there."""
        import torch
        if acc is None:
            acc = torch.empty((pos.shape[0], 3), dtype=torch.float64, device=pos.device)
        if pot is None:
            pot = torch.empty(pos.shape[0], dtype=torch.float64, device=pos.device)
        if stream is None:
            stream = torch.cuda.current_stream(pos.device)
        p = make_params(params, precision=precision, group_max=group_max, walk_list_cap=walk_list_cap,
                        stream=stream)
        t = og_server_submit(self.handle, box_struct(pos, mass, box, p, acc, pot))
        self._keep[t] = (pos, mass, acc, pot)
        return t

    def poll(self, ticket):
        return og_server_poll(self.handle, ticket)

    def progress(self):
        og_server_progress(self.handle)

    def wait(self, ticket):
        og_server_wait(self.handle, ticket)

    def result(self, ticket):
        _, _, acc, pot = self._keep[ticket]
        return acc, pot

    def release(self, ticket):
        og_server_release(self.handle, ticket)
        self._keep.pop(ticket, None)

    def stats(self):
        return og_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            og_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


# --------------------------------------------------------- particle mesh --
def og_pm_workspace_bound(n_grid: int) -> int:
    return int(load().og_pm_workspace_bound(int(n_grid)))


class PM:
    """Long-range (mesh) part of the TreePM force on an n_grid^3 periodic mesh."""

    def __init__(self, n_grid: int, box: float, G: float, r_s: float, stream=None):
        h = ctypes.c_void_p()
        _check(load().og_pm_create(int(n_grid), float(box), float(G), float(r_s), _stream_handle(stream),
                                   ctypes.byref(h)))
        self.handle = h
        self.n_grid = int(n_grid)

    def force(self, pos, mass, acc=None, pot=None, accumulate=False, with_pot=True):
        import torch
        N = int(pos.shape[0])
        if acc is None:
            acc = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        if with_pot and pot is None:
            pot = torch.empty(N, dtype=torch.float64, device=pos.device)
        _check(load().og_pm_force(self.handle, _ptr(pos), _ptr(mass), N, _ptr(acc), _ptr(pot) if with_pot else None,
                                  1 if accumulate else 0))
        return acc, pot

    def force_tree(self, tree, acc=None, pot=None, accumulate=False, with_pot=True):
        """Mesh force on a built periodic tree's particles (read in curve
        order); acc/pot in caller order."""
        import torch
        N = tree.N
        if acc is None:
            acc = torch.empty((N, 3), dtype=torch.float64, device=tree.device)
        if with_pot and pot is None:
            pot = torch.empty(N, dtype=torch.float64, device=tree.device)
        _check(load().og_pm_force_tree(self.handle, tree.handle, _ptr(acc), _ptr(pot) if with_pot else None,
                                       1 if accumulate else 0))
        return acc, pot

    def close(self):
        if getattr(self, "handle", None):
            _check(load().og_pm_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

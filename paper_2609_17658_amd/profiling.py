"""Small drivers for hardware-counter runs (run under rocprofv3).

  python paper_2609_17658_amd/profiling.py walk --prec mixed --reps 3
      builds the 2M-particle mixture tree once and runs the force walk
      `reps` times (the build kernels run once, the walk kernel `reps` times);
  python paper_2609_17658_amd/profiling.py build --reps 3 [--workload zeldovich256]
      builds the tree `reps` times (every build kernel runs `reps` times);
  python paper_2609_17658_amd/profiling.py pm --n-grid 256 --reps 3
      the particle-mesh force of the same mixture on a 256^3 mesh;
  python paper_2609_17658_amd/profiling.py pmtree --n-grid 256 --reps 3
      the same from a built tree (og_pm_force_tree, curve order);
  python paper_2609_17658_amd/profiling.py copy --mib 1024 --reps 3
      device-to-device copy of a buffer of known size, the reference for
      scaling FETCH_SIZE / WRITE_SIZE readings to bytes.
"""
import argparse
import os
import sys

if __package__ in (None, ""):  # run as a file (profilers exec the script path)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def _walk(prec: str, reps: int, workload: str):
    import torch

    from paper_2609_17658_amd import og, synth

    w = synth.WORKLOADS[workload]()
    dev = torch.device("cuda:0")
    tp = torch.as_tensor(w.pos, device=dev)
    tm = torch.as_tensor(w.mass, device=dev)
    t = og.Tree(tp, tm, w.box, w.params.as_dict(), stream=torch.cuda.current_stream())
    for _ in range(reps):
        t.force(precision=prec)
    torch.cuda.synchronize()
    t.close()
    print("walk %s x%d on %s: done" % (prec, reps, workload), flush=True)


def _build(reps: int, workload: str):
    import torch

    from paper_2609_17658_amd import og, synth

    w = synth.WORKLOADS[workload]()
    dev = torch.device("cuda:0")
    tp = torch.as_tensor(w.pos, device=dev)
    tm = torch.as_tensor(w.mass, device=dev)
    prm = w.params.as_dict()
    ws = torch.empty(og.og_tree_workspace_bound(tp.shape[0], og.make_params(prm)), dtype=torch.uint8, device=dev)
    for _ in range(reps):
        t = og.Tree(tp, tm, w.box, prm, stream=torch.cuda.current_stream(), workspace=ws)
        torch.cuda.synchronize()
        t.close()
    print("build x%d on %s: done" % (reps, workload), flush=True)


def _pm(n_grid: int, reps: int, workload: str):
    import torch

    from paper_2609_17658_amd import og, synth

    w = synth.WORKLOADS[workload]()
    dev = torch.device("cuda:0")
    tp = torch.as_tensor(w.pos, device=dev)
    tm = torch.as_tensor(w.mass, device=dev)
    prm = w.params.as_dict()
    mesh = og.PM(n_grid, w.box, prm["G"], prm["r_s"], stream=torch.cuda.current_stream())
    acc = torch.empty((tp.shape[0], 3), dtype=torch.float64, device=dev)
    pot = torch.empty(tp.shape[0], dtype=torch.float64, device=dev)
    for _ in range(reps):
        mesh.force(tp, tm, acc, pot)
    torch.cuda.synchronize()
    mesh.close()
    print("pm %d^3 x%d on %s: done" % (n_grid, reps, workload), flush=True)


def _pm_tree(n_grid: int, reps: int, workload: str):
    import torch

    from paper_2609_17658_amd import og, synth

    w = synth.WORKLOADS[workload]()
    dev = torch.device("cuda:0")
    tp = torch.as_tensor(w.pos, device=dev)
    tm = torch.as_tensor(w.mass, device=dev)
    prm = w.params.as_dict()
    stream = torch.cuda.current_stream()
    t = og.Tree(tp, tm, w.box, prm, stream=stream)
    mesh = og.PM(n_grid, w.box, prm["G"], prm["r_s"], stream=stream)
    acc = torch.empty((tp.shape[0], 3), dtype=torch.float64, device=dev)
    pot = torch.empty(tp.shape[0], dtype=torch.float64, device=dev)
    for _ in range(reps):
        mesh.force_tree(t, acc, pot)
    torch.cuda.synchronize()
    mesh.close()
    t.close()
    print("pm from the tree %d^3 x%d on %s: done" % (n_grid, reps, workload), flush=True)


def _copy(mib: int, reps: int):
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy %d MiB x%d: done" % (mib, reps), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    w = sub.add_parser("walk")
    w.add_argument("--prec", default="mixed")
    w.add_argument("--reps", type=int, default=3)
    w.add_argument("--workload", default="mixture2m")
    b = sub.add_parser("build")
    b.add_argument("--reps", type=int, default=3)
    b.add_argument("--workload", default="mixture2m")
    m = sub.add_parser("pm")
    m.add_argument("--n-grid", type=int, default=256)
    m.add_argument("--reps", type=int, default=3)
    m.add_argument("--workload", default="mixture2m")
    mt = sub.add_parser("pmtree")
    mt.add_argument("--n-grid", type=int, default=256)
    mt.add_argument("--reps", type=int, default=3)
    mt.add_argument("--workload", default="mixture2m")
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    if a.cmd == "walk":
        _walk(a.prec, a.reps, a.workload)
    elif a.cmd == "build":
        _build(a.reps, a.workload)
    elif a.cmd == "pm":
        _pm(a.n_grid, a.reps, a.workload)
    elif a.cmd == "pmtree":
        _pm_tree(a.n_grid, a.reps, a.workload)
    else:
        _copy(a.mib, a.reps)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark: short-range TreePM tree force on one MI355X.

One step = the whole hot path on one synthetic box: octree build (keys,
radix sort, gather, topology, moments, groups) + force on every particle.
Workload: N = 128^3 = 2,097,152 equal-mass particles in a periodic unit box,
half uniform, half in 64 Plummer spheres (a = 0.005), eps = 1/(40*128),
r_s = 1.25/256, r_cut = 4.5 r_s, theta = 0.5, leaf_max = 8.

Prints ONE JSON line: particles/s of the mixed form (FP32 interactions,
FP64 offsets and accumulation), the plain FP64 form beside it, per-step
p50/p99 ms, error percentiles vs the FP64 CPU oracle, the walk kernel's
achieved FP32 rate against the vector peak, and the oracle timed on the host
cores as a baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "short-range tree-force particles/s, FP32 vs FP64 at stated error; p99 ms"
FLOP_PER_INTERACTION = 42          # 35 FP32 + 7 FP64 per accepted partner (the pair term as executed)
PEAK_FP32 = 157.3e12               # MI355X FP32 vector, FLOP/s
PEAK_HBM = 8.0e12                  # MI355X HBM3E, B/s
BUILD_BYTES_PER_PARTICLE = None    # computed from the tree (algorithmic bytes)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_bytes(n, n_nodes, n_groups_bound=None):
    """Algorithmic HBM bytes of one build (every array read/written once per
    pass it is needed in): keys 36 B/particle (24 in + 12 out), 8 radix
    passes x (8 histogram read + 24 scatter read/write), gather 64 (32
    random read, 32 + 8 written), topology 8 key + 6 lcp/depth + 12 scan
    per particle plus 24 per node, moments 16 + 32 particle, 48 + 12 per
    node, groups 16 per node."""
    per_particle = 36 + 8 * 32 + 64 + 8 + 6 + 12 + 48
    per_node = 24 + 60 + 16
    return per_particle * n + per_node * n_nodes


def walk_profile():
    """The walk's rocprofv3 record (profiles/k_walk32_mixture2m_traffic.txt):
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy) and
    vector / scalar instruction counts per launch; empty once the walk source
    differs from the profiled one."""
    import hashlib
    try:
        rec = {}
        with open(os.path.join(ROOT, "profiles", "k_walk32_mixture2m_traffic.txt")) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip()
        with open(os.path.join(ROOT, "paper_2609_17658_amd", "csrc", "k_walk.hip"), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
        if rec.get("source_sha256") != h:
            return {}
        return rec
    except OSError:
        return {}


def walk_traffic_bytes():
    try:
        return float(walk_profile()["walk_traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def walk_issue(walk_ms):
    """Vector issue of the walk: a wave64 VALU instruction holds a 16-lane SIMD
    for 4 cycles; 1024 SIMDs at 2.4 GHz.  From the profiled instruction count
    and this run's walk time."""
    try:
        rec = walk_profile()
        valu = float(rec["walk_valu_insts_per_launch"])
    except (KeyError, ValueError):
        return None
    busy = valu * 4 / (1024 * walk_ms * 1e-3 * 2.4e9)
    out = {"valu_insts_per_launch": valu, "valu_busy_frac": busy,
           "note": "vector instructions x 4 cycles / SIMD cycles of the launch; 1 = vector issue saturated "
                   "(an estimate: it assumes every wave64 vector instruction holds its SIMD for 4 cycles, "
                   "so values slightly above 1 mean some take fewer)"}
    try:
        out["salu_insts_per_launch"] = float(rec["walk_salu_insts_per_launch"])
    except (KeyError, ValueError):
        pass
    return out


def source_id():
    """Identity of the code that ran: sha256 over the library's sources,
    headers, binding and this script (a GPU machine has no git metadata; the
    same digest is reproducible from any checkout), plus the commit when a
    git work tree is present (read from .git, no subprocess)."""
    import glob
    import hashlib
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2609_17658_amd", "csrc", "*"))
                   + [os.path.join(ROOT, "include", "og.h"), os.path.join(ROOT, "paper_2609_17658_amd", "og.py"),
                      os.path.abspath(__file__)])
    h = hashlib.sha256()
    for f in files:
        if os.path.isfile(f) and not f.endswith(".pyc"):
            h.update(os.path.relpath(f, ROOT).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    out = {"sources_sha256": h.hexdigest(), "files": len(files), "git": None}
    try:
        with open(os.path.join(ROOT, ".git", "HEAD")) as f:
            ref = f.read().strip()
        if ref.startswith("ref:"):
            with open(os.path.join(ROOT, ".git", ref.split(None, 1)[1])) as f:
                ref = f.read().strip()
        out["git"] = ref[:12]
    except OSError:
        pass
    return out


def time_steps(og, torch, tp, tm, params, ws, precision, steps, warmup, a_old=None):
    """Returns per-step ms, per-step walk ms, final (acc, pot) and the trees."""
    stream = torch.cuda.current_stream()
    trees = []

    def one_step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        t = og.Tree(tp, tm, 1.0, params, stream=stream, workspace=ws, precision=precision)
        if ev is not None:
            ev[1].record(stream)
        acc, pot = t.force(a_old=a_old)
        if ev is not None:
            ev[2].record(stream)
        trees.append(t)
        return acc, pot

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    for t in trees:
        t.close()
    trees.clear()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for k in range(steps):
        out = one_step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
    build_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    walk_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    total_ms = evs[0][0].elapsed_time(evs[-1][2])
    return {"step_ms": step_ms, "build_ms": build_ms, "walk_ms": walk_ms, "total_ms": total_ms,
            "wall_s": wall, "out": out, "trees": trees}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--cpu-budget-s", type=float, default=25.0)
    ap.add_argument("--legs", default="accuracy,tuned,batch,serving,zeldovich,variants,hilbert,active,pm,groups,theta",
                    help="extra workloads reported beside the headline: accuracy (tree vs direct sum), tuned, batch, "
                         "serving, zeldovich, variants, hilbert, active, pm, groups, theta (comma list, or 'none')")
    ap.add_argument("--serve-requests", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent boxes would be spread over GPUs; one large box would be split "
              "into curve segments with a one-step ghost exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_17658_amd import og, synth

    assert torch.cuda.is_available(), "no GPU"
    og.load()
    dev = torch.device("cuda:0")
    w = synth.mixture2m(theta=args.theta)
    n = w.pos.shape[0]
    prm = w.params.as_dict()
    log("workload mixture2m: N=%d theta=%.2f" % (n, args.theta))
    tp = torch.as_tensor(w.pos, device=dev)
    tm = torch.as_tensor(w.mass, device=dev)
    ws = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device=dev)

    # launch shape: the result-neutral knobs (targets per group, list depth)
    # tuned at the workload's leaf size
    from paper_2609_17658_amd import tune
    neutral = tune.tune_tree(tp, tm, 1.0, prm, fixed_leaf=prm["leaf_max"], reps=3, log=log)
    shape = {k: neutral["best"][k] for k in ("group_max", "walk_list_cap")}
    prm = dict(prm, **shape)
    log("tuned launch shape %s" % shape)
    res = {}
    for prec in ("mixed", "fp64"):
        log("timing %s: %d warmup + %d steps" % (prec, args.warmup, args.steps))
        r = time_steps(og, torch, tp, tm, prm, ws, prec, args.steps, args.warmup)
        res[prec] = r
        log("  %s: step %.3f ms (build %.3f, walk %.3f)" % (prec, r["step_ms"].mean(), r["build_ms"].mean(),
                                                            r["walk_ms"].mean()))

    # interaction counts and tree stats (outside the timed region)
    t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=ws)
    st = t.stats()
    acc_m, pot_m, nint_m = t.force(precision="mixed", with_counts=True)
    acc_d, pot_d, nint_d = t.force(precision="fp64", with_counts=True)
    torch.cuda.synchronize()
    inter_m = int(nint_m.sum().item())
    inter_d = int(nint_d.sum().item())
    acc_m = acc_m.cpu().numpy()
    acc_d = acc_d.cpu().numpy()
    nint_d_np = nint_d.cpu().numpy()
    nint_m_np = nint_m.cpu().numpy()
    t.close()
    for r in res.values():
        for tr in r["trees"]:
            tr.close()

    K = args.steps
    m = res["mixed"]
    d = res["fp64"]
    ms_step = m["total_ms"] / K
    value = n / (ms_step * 1e-3)
    fp64_value = n / (d["total_ms"] / K * 1e-3)
    walk_ms = float(m["walk_ms"].mean())
    flops = inter_m * FLOP_PER_INTERACTION
    achieved = flops / (walk_ms * 1e-3)
    bb = build_bytes(n, st["n_nodes"])
    build_gbs = bb / (float(m["build_ms"].mean()) * 1e-3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "mixture2m: N=128^3 periodic unit box, 50%% uniform + 64 Plummer spheres "
                        "(a=0.005), eps=1/5120, r_s=1.25/256, r_cut=4.5 r_s, theta=%.2f, leaf_max=8"
                        % args.theta,
            "N": n, "theta": args.theta, "leaf_max": 8, "group_max": shape["group_max"],
            "walk_list_cap": shape["walk_list_cap"],
            "launch_shape_tuning": neutral["trials"],
            "precision": "mixed: FP32 interactions on node-relative offsets, FP64 offsets + accumulation",
            "step": "og_tree_build + og_tree_force on all N targets",
        },
        "p50_ms": float(np.percentile(m["step_ms"], 50)),
        "p99_ms": float(np.percentile(m["step_ms"], 99)),
        "build_ms": float(m["build_ms"].mean()),
        "walk_ms": walk_ms,
        "fp64": {
            "value": fp64_value, "unit": "particles/s", "ms_per_step": d["total_ms"] / K,
            "build_ms": float(d["build_ms"].mean()), "walk_ms": float(d["walk_ms"].mean()),
            "p99_ms": float(np.percentile(d["step_ms"], 99)),
        },
        "mixed_over_fp64": value / fp64_value,
        "interactions_per_target": inter_m / n,
        "tree": {"n_nodes": st["n_nodes"], "depth": st["depth"]},
        "roofline": {
            "bound": "alu", "kernel": "k_walk32 (mixed walk)",
            "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": walk_traffic_bytes(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "peak_unpacked_fp32": 78.6,
            "flop_per_interaction": FLOP_PER_INTERACTION, "interactions": inter_m,
            "issue": walk_issue(walk_ms),
        },
        "roofline_build": {
            "bound": "hbm", "achieved": build_gbs / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": build_gbs / PEAK_HBM, "algorithmic_bytes": bb,
        },
        "source": source_id(),
    }

    legs = [l for l in args.legs.split(",") if l and l != "none"]
    # free the headline workload's device memory before the extra legs
    del tp, tm, ws
    torch.cuda.empty_cache()
    for leg in legs:
        fn = {"accuracy": leg_accuracy, "tuned": leg_tuned, "batch": leg_batch, "serving": leg_serving, "zeldovich": leg_zeldovich,
              "variants": leg_variants, "hilbert": leg_hilbert, "active": leg_active, "pm": leg_pm,
              "groups": leg_groups, "theta": leg_theta}[leg]
        log("leg %s" % leg)
        try:
            out[LEG_NAMES[leg]] = fn(og, torch, synth, args)
        except Exception as exc:  # noqa: BLE001 - report, do not hide
            log("leg %s failed: %r" % (leg, exc))
            out[LEG_NAMES[leg]] = {"failed": repr(exc)}
        torch.cuda.empty_cache()

    # oracle: error of both GPU forms and the CPU baseline
    if args.no_oracle:
        out["error"] = None
        out["cpu_baseline"] = None
        print(json.dumps(out), flush=True)
        return
    try:
        import oracle
        op = oracle.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic",
                                                  "leaf_max")})
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        otree = oracle.build_tree(w.pos, w.mass, 1.0, op)
        t_build = time.perf_counter() - t0
        rng = np.random.default_rng(99)
        probe = np.sort(rng.choice(n, 16384, replace=False))
        t0 = time.perf_counter()
        acc_o, _, nint_o = oracle.walk(otree, targets=probe)
        t_probe = time.perf_counter() - t0
        per_target = t_probe / probe.size
        if not args.no_cpu_baseline and t_build + per_target * n <= args.cpu_budget_s:
            sample = np.arange(n)
        else:
            k = int(max(16384, min(n, (args.cpu_budget_s - t_build) / max(per_target, 1e-9))))
            sample = np.sort(rng.choice(n, k, replace=False))
        t0 = time.perf_counter()
        acc_s, _, nint_s = oracle.walk(otree, targets=sample)
        t_walk = time.perf_counter() - t0
        t_total = t_build + t_walk * (n / sample.size)
        e_m = np.linalg.norm(acc_m[sample] - acc_s, axis=1) / np.linalg.norm(acc_s, axis=1)
        e_d = np.linalg.norm(acc_d[sample] - acc_s, axis=1) / np.linalg.norm(acc_s, axis=1)
        rms = np.sqrt(np.mean(np.sum(acc_s ** 2, axis=1)))
        out["error"] = {
            "vs": "FP64 CPU oracle tree walk, same tree parameters", "targets": int(sample.size),
            "mixed_median": float(np.median(e_m)), "mixed_p99": float(np.percentile(e_m, 99)),
            "mixed_max": float(e_m.max()),
            "mixed_p99_over_rms": float(np.percentile(np.linalg.norm(acc_m[sample] - acc_s, axis=1), 99) / rms),
            "fp64_median": float(np.median(e_d)), "fp64_max": float(e_d.max()),
            "fp64_counts_equal": bool(np.array_equal(nint_d_np[sample], nint_s)),
            "mixed_count_flips": int((nint_m_np[sample] != nint_s).sum()),
        }
        out["cpu_baseline"] = {
            "value": n / t_total, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": ("full tree build (%.2f s) + walk of %d of %d targets (%.2f s)%s"
                       % (t_build, sample.size, n, t_walk,
                          "" if sample.size == n else ", walk time scaled to all targets")),
            "cpu": _cpu_model(),
        }
        if args.no_cpu_baseline:
            out["cpu_baseline"] = None
    except Exception as exc:  # noqa: BLE001 - report, do not hide
        log("oracle leg failed: %r" % (exc,))
        out["error"] = None
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


LEG_NAMES = {"accuracy": "accuracy_vs_direct", "tuned": "tuned_mixture2m", "batch": "batch512", "serving": "serving", "zeldovich": "zeldovich256",
             "variants": "variants_mixture2m", "hilbert": "hilbert_mixture2m", "active": "active_mixture2m",
             "pm": "treepm", "groups": "group_lists_mixture2m",
             "theta": "theta_mixture2m"}


def _oracle_params(oracle, prm):
    return oracle.Params(**{k: prm[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic",
                                                "leaf_max")})


def _rel_err(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def leg_batch(og, torch, synth, args):
    """512 independent periodic boxes, N_b log-uniform in [1e3, 2e5]: one
    captured graph (build + walk of every box), launch shape autotuned."""
    from paper_2609_17658_amd import tune

    ws = synth.batch512()
    n_tot = int(sum(w.pos.shape[0] for w in ws))
    dev = [(torch.as_tensor(w.pos, device="cuda"), torch.as_tensor(w.mass, device="cuda"), w.box,
            w.params.as_dict()) for w in ws]
    tuned = tune.tune_batch(dev, reps=2, log=log)
    best = {k: tuned["best"][k] for k in ("group_max", "walk_list_cap", "leaf_max")}
    ms = tune.time_batch(dev, reps=max(3, args.steps), **best)
    # the same boxes one tree at a time (one reused workspace), for comparison
    stream = torch.cuda.current_stream()
    wsz = max(og.og_tree_workspace_bound(w.pos.shape[0], og.make_params(w.params.as_dict(),
                                                                          leaf_max=best["leaf_max"]))
              for w in ws)
    wbuf = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    acc = torch.empty((max(w.pos.shape[0] for w in ws), 3), dtype=torch.float64, device="cuda")
    pot = torch.empty(acc.shape[0], dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    trees = []
    e0.record(stream)
    for (pos, mass, box, prm) in dev:
        t = og.Tree(pos, mass, box, prm, stream=stream, workspace=wbuf, leaf_max=best["leaf_max"],
                    group_max=best["group_max"], walk_list_cap=best["walk_list_cap"])
        t.force(acc=acc[:pos.shape[0]], pot=pot[:pos.shape[0]])
        trees.append(t)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    for t in trees:
        t.close()
    del wbuf, acc, pot
    # parity of the tuned batch against the oracle at the tuned leaf size, sampled boxes
    err = None
    try:
        import oracle
        bt = og.Batch([(p, m, b, dict(prm, leaf_max=best["leaf_max"])) for p, m, b, prm in dev],
                      precision="mixed", group_max=best["group_max"],
                      walk_list_cap=best["walk_list_cap"])
        outs = bt.force()
        torch.cuda.synchronize()
        errs, worst_med, worst_p99 = [], 0.0, 0.0
        t0 = time.perf_counter()
        for b, w in enumerate(ws):
            op = _oracle_params(oracle, dict(w.params.as_dict(), leaf_max=best["leaf_max"]))
            a_o, _, _ = oracle.tree_force(w.pos, w.mass, w.box, op)
            e = _rel_err(outs[b][0].cpu().numpy(), a_o)
            worst_med = max(worst_med, float(np.median(e)))
            worst_p99 = max(worst_p99, float(np.percentile(e, 99)))
            errs.append(e)
        t_or = time.perf_counter() - t0
        bt.close()
        e = np.concatenate(errs)
        err = {"boxes": len(ws), "targets": int(e.size), "leaf_max": best["leaf_max"],
               "mixed_median": float(np.median(e)), "mixed_p99": float(np.percentile(e, 99)),
               "per_box_median_worst": worst_med, "per_box_p99_worst": worst_p99, "oracle_s": t_or}
    except Exception as exc:  # noqa: BLE001
        log("batch parity failed: %r" % (exc,))
    return {"boxes": len(ws), "N_total": n_tot, "ms_per_pass": ms, "value": n_tot / (ms * 1e-3),
            "unit": "particles/s", "tuned": best, "tuning": tuned["trials"],
            "one_tree_at_a_time_ms": loop_ms, "speedup_vs_one_at_a_time": loop_ms / ms,
            "error_vs_oracle": err,
            "workload": "512 periodic boxes, N_b log-uniform [1e3, 2e5], half uniform + 8 Plummer "
                        "spheres (a=0.01), box seed 1000+b, scale-free eps and r_s, theta 0.5; "
                        "graph replay of build + mixed walk"}


def leg_serving(og, torch, synth, args):
    """Poisson request stream, N log-uniform in [1e4, 4e6] (Zel'dovich or
    mixture): continuous batching with HBM admission; p50/p99 latency from
    arrival to completion, throughput = particles / makespan."""
    pool_n = 16
    reqs = synth.request_stream(pool_n, 1.0, seed=5)
    pool = []
    for r in reqs:
        w = r.workload()
        pool.append((torch.as_tensor(w.pos, device="cuda"), torch.as_tensor(w.mass, device="cuda"),
                     w.params.as_dict()))
    budget = 48 << 30
    srv = og.Server(budget, max_slots=4)
    # closed-loop calibration: everything at once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tk = [srv.submit(p, m, 1.0, prm) for p, m, prm in pool]
    for t in tk:
        srv.wait(t)
    calib = time.perf_counter() - t0
    for t in tk:
        srv.release(t)
    sustain = pool_n / calib
    rate = 0.7 * sustain
    K = args.serve_requests
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, K))
    arrivals -= arrivals[0]
    lat, inflight, n_done, parts = [], [], 0, 0
    kept = []          # (pool box, acc) of the first served requests, checked after the stream
    n_check = 50
    k = 0
    start = time.perf_counter()
    while n_done < K:
        now = time.perf_counter() - start
        while k < K and arrivals[k] <= now:
            p, m, prm = pool[k % pool_n]
            inflight.append((srv.submit(p, m, 1.0, prm), p.shape[0], k % pool_n))
            k += 1
        still = []
        for t, n, b in inflight:
            done, ta, td = srv.poll(t)
            if done:
                lat.append(td - ta)
                parts += n
                n_done += 1
                if len(kept) < n_check:
                    kept.append((b, srv.result(t)[0]))
                srv.release(t)
            else:
                still.append((t, n, b))
        inflight = still
        if k < K and not inflight:
            time.sleep(max(0.0, min(0.0005, arrivals[k] - (time.perf_counter() - start))))
    makespan = time.perf_counter() - start
    srv.close()
    lat = np.array(lat) * 1e3
    check = _serving_check(og, torch, reqs, pool, kept)
    return {"requests": K, "pool": pool_n, "rate_per_s": rate, "sustainable_per_s": sustain,
            "error_vs_oracle": check,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "value": parts / makespan, "unit": "particles/s",
            "makespan_s": makespan, "slots": 4, "hbm_budget_bytes": budget,
            "pool_N": [int(p[0].shape[0]) for p in pool],
            "workload": "Poisson arrivals at 0.7x the closed-loop rate; request k is pool box k mod 16, "
                        "N log-uniform [1e4, 4e6], Zel'dovich or mixture by seeded coin; mixed walk"}


def _serving_check(og, torch, reqs, pool, kept):
    """Served results of the first requests against the FP64 oracle (2000
    seeded targets of their pool box, all when smaller) and bitwise against
    an alone run of that box."""
    try:
        import oracle
    except Exception as exc:  # noqa: BLE001
        return {"failed": repr(exc)}
    refs, alone = {}, {}
    for b in sorted({b for b, _ in kept}):
        w = reqs[b].workload()
        n = w.pos.shape[0]
        rng = np.random.default_rng(200 + b)
        tg = np.arange(n) if n <= 2000 else np.sort(rng.choice(n, 2000, replace=False))
        a_o, _, _ = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, w.params.as_dict()), targets=tg)
        refs[b] = (tg, a_o)
        p, m, prm = pool[b]
        t = og.Tree(p, m, 1.0, prm, stream=torch.cuda.current_stream())
        a, _ = t.force(precision="mixed")
        torch.cuda.synchronize()
        alone[b] = a.cpu().numpy()
        t.close()
    med, p99, same = [], [], 0
    for b, acc in kept:
        a = acc.cpu().numpy()
        tg, a_o = refs[b]
        e = _rel_err(a[tg], a_o)
        med.append(float(np.median(e)))
        p99.append(float(np.percentile(e, 99)))
        same += int(np.array_equal(a, alone[b]))
    return {"requests_checked": len(kept), "distinct_boxes": len(refs), "targets_per_request": "min(N, 2000)",
            "mixed_median_worst": max(med), "mixed_p99_worst": max(p99),
            "bitwise_equal_to_alone": same}


def leg_zeldovich(og, torch, synth, args):
    """N = 256^3 Zel'dovich-displaced grid (P(k) ~ k^-2, rms 0.3 cell): the
    largest single box; both forms, error on sampled targets."""
    from paper_2609_17658_amd import tune
    w = synth.zeldovich256()
    n = w.pos.shape[0]
    prm = w.params.as_dict()
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device="cuda")
    neutral = tune.tune_tree(tp, tm, 1.0, prm, fixed_leaf=prm["leaf_max"], reps=2, log=log)
    shape = {k: neutral["best"][k] for k in ("group_max", "walk_list_cap")}
    prm = dict(prm, **shape)
    res = {}
    for prec, steps in (("mixed", 5), ("fp64", 2)):
        r = time_steps(og, torch, tp, tm, prm, wsb, prec, steps, 1)
        for t in r["trees"]:
            t.close()
        res[prec] = {"value": n / (r["total_ms"] / steps * 1e-3), "ms_per_step": r["total_ms"] / steps,
                     "build_ms": float(r["build_ms"].mean()), "walk_ms": float(r["walk_ms"].mean())}
    t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=wsb)
    a_m, _, ni_m = t.force(precision="mixed", with_counts=True)
    a_d, _, ni_d = t.force(precision="fp64", with_counts=True)
    torch.cuda.synchronize()
    t.close()
    inter_m = int(ni_m.sum().item())
    walk_ms = res["mixed"]["walk_ms"]
    achieved = inter_m * FLOP_PER_INTERACTION / (walk_ms * 1e-3)
    roof = {"bound": "alu", "kernel": "k_walk32 (mixed walk)", "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
            "flop_per_interaction": FLOP_PER_INTERACTION, "interactions": inter_m,
            "interactions_per_target": inter_m / n, "walk_ms": walk_ms,
            "fp64_walk_tflops": int(ni_d.sum().item()) * FLOP_PER_INTERACTION / (res["fp64"]["walk_ms"] * 1e-3) / 1e12}
    err = None
    try:
        import oracle
        rng = np.random.default_rng(3)
        tg = np.sort(rng.choice(n, 1 << 20, replace=False))
        t0 = time.perf_counter()
        a_o, _, ni_o = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, prm), targets=tg)
        t_or = time.perf_counter() - t0
        a_mt = a_m.cpu().numpy()[tg]
        e_m = _rel_err(a_mt, a_o)
        e_d = _rel_err(a_d.cpu().numpy()[tg], a_o)
        rms = np.sqrt(np.mean(np.sum(a_o ** 2, axis=1)))
        err = {"targets": int(tg.size), "mixed_median": float(np.median(e_m)),
               "mixed_p99": float(np.percentile(e_m, 99)), "mixed_max": float(e_m.max()),
               "mixed_p99_over_rms": float(np.percentile(np.linalg.norm(a_mt - a_o, axis=1), 99) / rms),
               "fp64_max": float(e_d.max()),
               "fp64_counts_equal": bool(np.array_equal(ni_d.cpu().numpy()[tg], ni_o)),
               "oracle_s": t_or}
    except Exception as exc:  # noqa: BLE001
        log("zeldovich parity failed: %r" % (exc,))
    return {"N": n, "launch_shape": shape, "mixed": res["mixed"], "fp64": res["fp64"], "roofline": roof,
            "error_vs_oracle": err,
            "workload": "256^3 grid, Gaussian field P(k)~k^-2 cut at k_Nyq, rms displacement 0.3 cell, "
                        "eps=1/10240, r_s=1.25/512, theta 0.5, leaf_max 8; oracle on 2^20 seeded targets"}


def _err_stats(a, ref):
    e = _rel_err(a, ref)
    return {"median": float(np.median(e)), "p99": float(np.percentile(e, 99)), "max": float(e.max())}


def leg_accuracy(og, torch, synth, args):
    """Error of the tree force itself (the opening criterion's truncation):
    the GPU mixed and FP64 walks and the oracle's walk against the
    brute-force direct sum with the same split, cutoff and softening.  The
    32k mixture on every target (the full N^2 direct sum); the 2M mixture on
    4096 seeded targets at theta 0.3, 0.5 and 0.7.  The paper prints no such
    error, so these values are not pinned to it."""
    import oracle
    out = {}
    w = synth.mixture32k()
    prm = w.params.as_dict()
    n = w.pos.shape[0]
    t0 = time.perf_counter()
    a_dir = oracle.direct(w.pos, w.mass, 1.0, _oracle_params(oracle, prm))[0]
    t_dir = time.perf_counter() - t0
    tp, tm = torch.as_tensor(w.pos, device="cuda"), torch.as_tensor(w.mass, device="cuda")
    tr = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream())
    a_m, _ = tr.force(precision="mixed")
    a_d, _ = tr.force(precision="fp64")
    torch.cuda.synchronize()
    tr.close()
    a_t = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, prm))[0]
    out["mixture32k"] = {"targets": n, "theta": prm["theta"], "direct_s": t_dir,
                         "gpu_mixed": _err_stats(a_m.cpu().numpy(), a_dir),
                         "gpu_fp64": _err_stats(a_d.cpu().numpy(), a_dir),
                         "oracle_tree": _err_stats(a_t, a_dir)}
    w = synth.mixture2m()
    n = w.pos.shape[0]
    tg = np.sort(np.random.default_rng(17).choice(n, 4096, replace=False))
    t0 = time.perf_counter()
    a_dir = oracle.direct(w.pos, w.mass, 1.0, _oracle_params(oracle, w.params.as_dict()), targets=tg)[0]
    t_dir = time.perf_counter() - t0
    tp, tm = torch.as_tensor(w.pos, device="cuda"), torch.as_tensor(w.mass, device="cuda")
    tgd = torch.as_tensor(tg, dtype=torch.int64, device="cuda")
    res = {"targets": int(tg.size), "direct_s": t_dir}
    for theta in (0.3, 0.5, 0.7):
        prm = dict(w.params.as_dict(), theta=theta)
        tr = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream())
        a_m, _ = tr.force(targets=tgd, precision="mixed")
        a_d, _ = tr.force(targets=tgd, precision="fp64")
        torch.cuda.synchronize()
        tr.close()
        a_t = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, prm), targets=tg)[0]
        res["theta_%.1f" % theta] = {"gpu_mixed": _err_stats(a_m.cpu().numpy(), a_dir),
                                     "gpu_fp64": _err_stats(a_d.cpu().numpy(), a_dir),
                                     "oracle_tree": _err_stats(a_t, a_dir)}
    med = [res["theta_%.1f" % th]["oracle_tree"]["median"] for th in (0.3, 0.5, 0.7)]
    res["median_decreases_with_theta"] = bool(med[0] < med[1] < med[2])
    out["mixture2m"] = res
    out["vs"] = "brute-force direct sum (oracle), same erfc split, r_cut, Plummer softening, minimum image"
    return out


def leg_tuned(og, torch, synth, args):
    """The 2M mixture with the leaf size searched too (tree build + mixed
    walk timed for leaf_max 4, 8, 16 with both launch-shape knobs): the
    fastest setting, its error against the oracle at that leaf size (65536
    seeded targets) and against the direct sum (4096 seeded targets)."""
    from paper_2609_17658_amd import tune
    import oracle
    w = synth.mixture2m()
    n = w.pos.shape[0]
    prm = w.params.as_dict()
    tp, tm = torch.as_tensor(w.pos, device="cuda"), torch.as_tensor(w.mass, device="cuda")
    res = tune.tune_tree(tp, tm, 1.0, prm, reps=3, log=log)
    best = {k: res["best"][k] for k in ("group_max", "walk_list_cap", "leaf_max")}
    p = dict(prm, **best)
    tr = og.Tree(tp, tm, 1.0, p, stream=torch.cuda.current_stream())
    a_m, _, ni = tr.force(precision="mixed", with_counts=True)
    torch.cuda.synchronize()
    tr.close()
    a_m = a_m.cpu().numpy()
    rng = np.random.default_rng(23)
    tg = np.sort(rng.choice(n, 65536, replace=False))
    a_o = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, p), targets=tg)[0]
    e = _rel_err(a_m[tg], a_o)
    tgd = np.sort(np.random.default_rng(17).choice(n, 4096, replace=False))
    a_dir = oracle.direct(w.pos, w.mass, 1.0, _oracle_params(oracle, p), targets=tgd)[0]
    return {"best": best, "ms_per_step": res["best"]["ms"], "value": n / (res["best"]["ms"] * 1e-3),
            "unit": "particles/s", "interactions_per_target": float(ni.sum().item()) / n,
            "trials": res["trials"],
            "error_vs_oracle_at_tuned_leaf": {"targets": int(tg.size), "mixed_median": float(np.median(e)),
                                              "mixed_p99": float(np.percentile(e, 99))},
            "error_vs_direct": dict(_err_stats(a_m[tgd], a_dir), targets=int(tgd.size)),
            "workload": "mixture2m (the headline box) with leaf_max searched; the headline keeps leaf_max 8 "
                        "as configured"}


VARIANT_LEGS = (
    ("spline", dict(softening="spline")),
    ("relative", dict(criterion="relative", alpha=0.0025)),
    ("spline_relative", dict(softening="spline", criterion="relative", alpha=0.0025)),
    ("particle_lengths", dict(softening="spline", lengths=True)),
)


def particle_lengths(n, eps, seed=21):
    """Per-particle softening lengths: 30 % of the particles at 5x eps, the
    rest at eps, each scattered by a factor in [0.8, 1.2]."""
    rng = np.random.default_rng(seed)
    return eps * np.where(rng.random(n) < 0.3, 5.0, 1.0) * rng.uniform(0.8, 1.2, n)


def leg_variants(og, torch, synth, args):
    """The headline box with the spline softening (support 2.8 eps) and the
    relative opening criterion (alpha = 0.0025 against the previous
    acceleration).  Timing uses this device's FP64 Barnes-Hut accelerations
    as a_old (a previous step's result); the error check runs sampled
    targets on both sides with a_old taken from the oracle's own
    Barnes-Hut walk."""
    w = synth.mixture2m(theta=args.theta)
    n = w.pos.shape[0]
    base = w.params.as_dict()
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(base)), dtype=torch.uint8, device="cuda")
    t = og.Tree(tp, tm, 1.0, base, stream=torch.cuda.current_stream(), workspace=wsb)
    a_prev, _ = t.force(precision="fp64")
    torch.cuda.synchronize()
    t.close()
    out = {}
    oracle = None
    if not args.no_oracle:
        import oracle
        rng = np.random.default_rng(7)
        tg = np.sort(rng.choice(n, 4096, replace=False))
        a_bh, _, _ = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, base), targets=tg)
        a_old_o = np.zeros((n, 3))
        a_old_o[tg] = a_bh
    eps_np = particle_lengths(n, base["eps"])
    eps_t = torch.as_tensor(eps_np, device="cuda")
    wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(dict(base, eps_particle=eps_t))),
                      dtype=torch.uint8, device="cuda")
    for name, extra in VARIANT_LEGS:
        extra = dict(extra)
        lengths = extra.pop("lengths", False)
        prm = dict(base, **extra)
        if lengths:
            prm["eps_particle"] = eps_t
        rel = prm.get("criterion") == "relative"
        row = {}
        for prec, steps in (("mixed", 5), ("fp64", 2)):
            r = time_steps(og, torch, tp, tm, prm, wsb, prec, steps, 1, a_old=a_prev if rel else None)
            for tr in r["trees"]:
                tr.close()
            row[prec] = {"value": n / (r["total_ms"] / steps * 1e-3), "ms_per_step": r["total_ms"] / steps,
                         "build_ms": float(r["build_ms"].mean()), "walk_ms": float(r["walk_ms"].mean())}
        t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=wsb)
        _, _, ni = t.force(precision="mixed", with_counts=True, a_old=a_prev if rel else None)
        torch.cuda.synchronize()
        row["interactions_per_target"] = float(ni.sum().item()) / n
        if oracle is not None:
            ao = torch.as_tensor(a_old_o, device="cuda") if rel else None
            tgd = torch.as_tensor(tg, device="cuda")
            am, _ = t.force(targets=tgd, precision="mixed", a_old=ao)
            ad, _, nd = t.force(targets=tgd, precision="fp64", with_counts=True, a_old=ao)
            torch.cuda.synchronize()
            op = oracle.Params(**{**{k: base[k] for k in ("G", "eps", "r_s", "r_cut", "theta", "periodic",
                                                          "leaf_max")},
                                  "softening": 1 if prm.get("softening") == "spline" else 0,
                                  "criterion": 1 if rel else 0, "alpha": prm.get("alpha", 0.0)})
            a_o, _, n_o = oracle.tree_force(w.pos, w.mass, 1.0, op, targets=tg, a_old=a_old_o,
                                            eps=eps_np if lengths else None)
            e_m = _rel_err(am.cpu().numpy(), a_o)
            row["error_vs_oracle"] = {
                "targets": int(tg.size), "mixed_median": float(np.median(e_m)),
                "mixed_p99": float(np.percentile(e_m, 99)),
                "fp64_max": float(_rel_err(ad.cpu().numpy(), a_o).max()),
                "fp64_counts_equal": bool(np.array_equal(nd.cpu().numpy(), n_o))}
        t.close()
        log("  %s: mixed %.3f ms/step, fp64 %.3f" % (name, row["mixed"]["ms_per_step"], row["fp64"]["ms_per_step"]))
        out[name] = row
    out["workload"] = ("mixture2m as the headline; variants: %s; particle_lengths: 30%% of the particles at "
                       "5x eps, the rest at eps, x U(0.8, 1.2), seed 21" % ", ".join("%s=%s" % (k, v) for k, v in VARIANT_LEGS))
    return out


def leg_hilbert(og, torch, synth, args):
    """The headline box with Peano-Hilbert keys: same nodes, curve order for
    the particles, the children and the walk groups."""
    w = synth.mixture2m(theta=args.theta)
    n = w.pos.shape[0]
    prm = dict(w.params.as_dict(), curve="hilbert")
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device="cuda")
    out = {}
    for prec, steps in (("mixed", 5), ("fp64", 2)):
        r = time_steps(og, torch, tp, tm, prm, wsb, prec, steps, 1)
        for t in r["trees"]:
            t.close()
        out[prec] = {"value": n / (r["total_ms"] / steps * 1e-3), "ms_per_step": r["total_ms"] / steps,
                     "build_ms": float(r["build_ms"].mean()), "walk_ms": float(r["walk_ms"].mean())}
        log("  hilbert %s: %.3f ms/step (build %.3f, walk %.3f)" % (prec, out[prec]["ms_per_step"],
                                                                   out[prec]["build_ms"], out[prec]["walk_ms"]))
    if not args.no_oracle:
        import oracle
        rng = np.random.default_rng(11)
        tg = np.sort(rng.choice(n, 4096, replace=False))
        t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=wsb)
        tgd = torch.as_tensor(tg, device="cuda")
        am, _ = t.force(targets=tgd, precision="mixed")
        ad, _, nd = t.force(targets=tgd, precision="fp64", with_counts=True)
        torch.cuda.synchronize()
        t.close()
        op = oracle.Params(**{**{k: w.params.as_dict()[k] for k in ("G", "eps", "r_s", "r_cut", "theta",
                                                                    "periodic", "leaf_max")}, "curve": 1})
        a_o, _, n_o = oracle.tree_force(w.pos, w.mass, 1.0, op, targets=tg)
        e_m = _rel_err(am.cpu().numpy(), a_o)
        out["error_vs_oracle"] = {"targets": int(tg.size), "mixed_median": float(np.median(e_m)),
                                  "mixed_p99": float(np.percentile(e_m, 99)),
                                  "fp64_max": float(_rel_err(ad.cpu().numpy(), a_o).max()),
                                  "fp64_counts_equal": bool(np.array_equal(nd.cpu().numpy(), n_o))}
    out["workload"] = "mixture2m as the headline, Peano-Hilbert keys"
    return out


def leg_theta(og, torch, synth, args):
    """The headline mixture at the other opening angles of its sweep
    (theta 0.3 and 0.7): both forms, error on sampled targets."""
    out = {}
    for theta in (0.3, 0.7):
        w = synth.mixture2m(theta=theta)
        n = w.pos.shape[0]
        prm = w.params.as_dict()
        tp = torch.as_tensor(w.pos, device="cuda")
        tm = torch.as_tensor(w.mass, device="cuda")
        wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device="cuda")
        res = {}
        for prec, steps in (("mixed", 5), ("fp64", 2)):
            r = time_steps(og, torch, tp, tm, prm, wsb, prec, steps, 1)
            for t in r["trees"]:
                t.close()
            res[prec] = {"value": n / (r["total_ms"] / steps * 1e-3), "ms_per_step": r["total_ms"] / steps,
                         "build_ms": float(r["build_ms"].mean()), "walk_ms": float(r["walk_ms"].mean())}
            log("  theta %.1f %s: %.3f ms/step (build %.3f, walk %.3f)" % (
                theta, prec, res[prec]["ms_per_step"], res[prec]["build_ms"], res[prec]["walk_ms"]))
        rng = np.random.default_rng(11)
        tg = np.sort(rng.choice(n, 4096, replace=False))
        t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=wsb)
        tgd = torch.as_tensor(tg, device="cuda")
        am, _, nm = t.force(targets=tgd, precision="mixed", with_counts=True)
        ad, _, nd = t.force(targets=tgd, precision="fp64", with_counts=True)
        torch.cuda.synchronize()
        t.close()
        res["interactions_per_target"] = float(nd.double().mean().item())
        if not args.no_oracle:
            import oracle
            a_o, _, n_o = oracle.tree_force(w.pos, w.mass, 1.0, _oracle_params(oracle, prm), targets=tg)
            e_m = _rel_err(am.cpu().numpy(), a_o)
            res["error_vs_oracle"] = {"targets": int(tg.size), "mixed_median": float(np.median(e_m)),
                                      "mixed_p99": float(np.percentile(e_m, 99)),
                                      "fp64_max": float(_rel_err(ad.cpu().numpy(), a_o).max()),
                                      "fp64_counts_equal": bool(np.array_equal(nd.cpu().numpy(), n_o))}
        out["theta%.1f" % theta] = res
        del tp, tm, wsb
    out["workload"] = "mixture2m as the headline at theta 0.3 and 0.7 (the headline runs theta 0.5)"
    return out


def leg_active(og, torch, synth, args):
    """Individual power-of-two time steps on a resident tree: time-step
    levels from the Gadget-style criterion dt = sqrt(2 eta eps / |a|)
    (eta = 0.025) on the headline box's forces, level b = floor(log2(dt /
    dt_min)) capped at 6; one cycle of 64 substeps, substep s walking the
    particles with level <= ctz(s) (og_tree_force_active, no host sync)."""
    w = synth.mixture2m(theta=args.theta)
    n = w.pos.shape[0]
    prm = w.params.as_dict()
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    stream = torch.cuda.current_stream()
    tree = og.Tree(tp, tm, 1.0, prm, stream=stream)
    a, _ = tree.force(precision="mixed")
    amag = torch.linalg.norm(a, dim=1).cpu().numpy()
    dt = np.sqrt(2 * 0.025 * prm["eps"] / np.maximum(amag, 1e-300))
    kmax = 6
    bins_np = np.clip(np.floor(np.log2(dt / dt.min())), 0, kmax).astype(np.int8)
    bins = torch.as_tensor(bins_np, device="cuda")
    acc = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    nact = torch.zeros(2 ** kmax, dtype=torch.int64, device="cuda")
    levels = [min((s & -s).bit_length() - 1, kmax) for s in range(1, 2 ** kmax + 1)]
    for _ in range(2):  # warm-up cycle
        for s, lev in enumerate(levels):
            tree.force_active(bins, lev, acc, pot, n_active=nact[s:s + 1])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for s, lev in enumerate(levels):
        tree.force_active(bins, lev, acc, pot, n_active=nact[s:s + 1])
    ev[1].record(stream)
    torch.cuda.synchronize()
    cycle_ms = ev[0].elapsed_time(ev[1])
    counts = nact.cpu().numpy()
    expect = np.array([(bins_np <= lev).sum() for lev in levels])
    # the same cycle with every particle walked on every substep
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev2[0].record(stream)
    for _ in range(4):
        tree.force(precision="mixed", acc=acc, pot=pot)
    ev2[1].record(stream)
    torch.cuda.synchronize()
    full_ms = ev2[0].elapsed_time(ev2[1]) / 4
    tree.close()
    tot = int(counts.sum())
    return {"substeps": len(levels), "levels_histogram": np.bincount(bins_np, minlength=kmax + 1).tolist(),
            "active_forces": tot, "cycle_ms": cycle_ms, "value": tot / (cycle_ms * 1e-3), "unit": "particles/s",
            "counts_match": bool(np.array_equal(counts, expect)),
            "all_particles_every_substep_ms": full_ms * len(levels),
            "speedup_vs_all_every_substep": full_ms * len(levels) / cycle_ms,
            "workload": "mixture2m resident tree (mixed walk), levels 0..%d from dt = sqrt(2 eta eps/|a|), "
                        "eta 0.025; one cycle of %d substeps" % (kmax, len(levels))}


def pm_bytes(n_particles, n_grid):
    """Algorithmic HBM bytes of one og_pm_force_tree call, each array the
    pipeline needs read or written once: per particle, the deposit reads
    32 B, the interpolation reads 32 B and writes 32 B (acc + pot); per mesh
    cell, the deposit writes the 8-byte fixed-point sum, the forward z pass
    reads it and writes 16 B, the y pass reads and writes 16 B, the x pass
    (with the Green's function and both inverse x passes) reads 16 B and
    writes 32 B, the inverse y and z passes of both fields read and write
    4 x 32 B, and the interpolation reads both fields (32 B).  The block
    halos (217 of 729 tile nodes, 6.8 B per cell written and read) are not
    counted."""
    cells = n_grid ** 3
    return n_particles * (32 + 32 + 32) + cells * (8 + 24 + 32 + 48 + 128 + 32)


def leg_pm(og, torch, synth, args):
    """Full TreePM force: tree short-range (mixed walk) + particle-mesh
    long-range on a mesh of 2 N^(1/3) points per axis (r_s = 1.25 mesh
    cells), for the headline box and the 256^3 Zel'dovich box."""
    out = {}
    # the device's streaming rate: a 1 GiB device-to-device copy (read + write)
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(100):  # about 50 ms of copies first: the clocks settle
        b.copy_(a)
    torch.cuda.synchronize()
    ec = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ec[0].record()
    for _ in range(20):
        b.copy_(a)
    ec[1].record()
    torch.cuda.synchronize()
    copy_gbps = 2 * (1 << 30) / (ec[0].elapsed_time(ec[1]) / 20 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out["copy_1GiB_GBps"] = copy_gbps
    for name, make, n_grid, reps in (("mixture2m", lambda: synth.mixture2m(theta=args.theta), 256, 5),
                                     ("zeldovich256", synth.zeldovich256, 512, 3)):
        w = make()
        n = w.pos.shape[0]
        prm = w.params.as_dict()
        tp = torch.as_tensor(w.pos, device="cuda")
        tm = torch.as_tensor(w.mass, device="cuda")
        stream = torch.cuda.current_stream()
        mesh = og.PM(n_grid, 1.0, prm["G"], prm["r_s"], stream=stream)
        wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device="cuda")
        acc = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        pot = torch.empty(n, dtype=torch.float64, device="cuda")
        mesh.force(tp, tm, acc, pot)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            mesh.force(tp, tm, acc, pot)
        ev[1].record(stream)
        torch.cuda.synchronize()
        pm_ms = ev[0].elapsed_time(ev[1]) / reps
        # the same from a resident tree's curve-ordered particles
        t = og.Tree(tp, tm, 1.0, prm, stream=stream, workspace=wsb)
        mesh.force_tree(t, acc, pot)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            mesh.force_tree(t, acc, pot)
        ev[1].record(stream)
        torch.cuda.synchronize()
        pm_tree_ms = ev[0].elapsed_time(ev[1]) / reps
        t.close()
        # one full TreePM step: build + short-range walk + mesh (accumulated)
        steps = []
        for _ in range(reps + 1):
            e3 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e3[0].record(stream)
            t = og.Tree(tp, tm, 1.0, prm, stream=stream, workspace=wsb)
            t.force(acc=acc, pot=pot)
            mesh.force_tree(t, acc, pot, accumulate=True)
            e3[1].record(stream)
            torch.cuda.synchronize()
            t.close()
            steps.append(e3[0].elapsed_time(e3[1]))
        step_ms = float(np.mean(steps[1:]))
        row = {"N": n, "n_grid": n_grid, "pm_ms": pm_ms, "pm_from_tree_ms": pm_tree_ms, "treepm_ms_per_step": step_ms,
               "value": n / (step_ms * 1e-3), "unit": "particles/s",
               "pm_roofline": {"bound": "hbm", "achieved": pm_bytes(n, n_grid) / (pm_tree_ms * 1e-3) / 1e9,
                               "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                               "frac": pm_bytes(n, n_grid) / (pm_tree_ms * 1e-3) / PEAK_HBM,
                               "kernel": "og_pm_force_tree (all mesh kernels of one call)",
                               "algorithmic_bytes": pm_bytes(n, n_grid),
                               "frac_of_copy_rate": pm_bytes(n, n_grid) / (pm_tree_ms * 1e-3) / 1e9 / copy_gbps}}
        if not args.no_oracle and name == "mixture2m":
            from oracle import pm as opm
            rng = np.random.default_rng(13)
            tg = np.sort(rng.choice(n, 4096, replace=False))
            mesh.force(tp, tm, acc, pot)
            torch.cuda.synchronize()
            a_o, p_o = opm.long_range(w.pos, w.mass, 1.0, n_grid, prm["G"], prm["r_s"], targets=tg)
            a_g = acc.cpu().numpy()[tg]
            row["pm_error_vs_oracle"] = {
                "targets": int(tg.size),
                "max_abs_over_max": float(np.abs(a_g - a_o).max() / np.abs(a_o).max()),
                "pot_max_abs_over_max": float(np.abs(pot.cpu().numpy()[tg] - p_o).max() / np.abs(p_o).max())}
        log("  treepm %s: mesh %.3f ms (from the tree %.3f), TreePM step %.3f ms" % (name, pm_ms, pm_tree_ms, step_ms))
        mesh.close()
        del tp, tm, wsb, acc, pot
        torch.cuda.empty_cache()
        out[name] = row
    out["workload"] = ("mixture2m (mesh 256^3) and zeldovich256 (mesh 512^3), r_s = 1.25 cells; step = "
                       "og_tree_build + og_tree_force (mixed) + og_pm_force_tree accumulated")
    return out


def leg_groups(og, torch, synth, args):
    """The headline box with group-shared interaction lists (one walk per
    group of consecutive targets in curve order), for two group sizes; the
    error is against the oracle's group walk over the same partition, on
    64 whole groups."""
    w = synth.mixture2m(theta=args.theta)
    n = w.pos.shape[0]
    base = w.params.as_dict()
    tp = torch.as_tensor(w.pos, device="cuda")
    tm = torch.as_tensor(w.mass, device="cuda")
    out = {}
    otree = None
    if not args.no_oracle:
        import oracle
        otree = oracle.build_tree(w.pos, w.mass, 1.0, _oracle_params(oracle, base))
    for gm in (64, 32):
        prm = dict(base, lists="group", group_max=gm)
        wsb = torch.empty(og.og_tree_workspace_bound(n, og.make_params(prm)), dtype=torch.uint8, device="cuda")
        row = {}
        for prec, steps in (("mixed", 5), ("fp64", 2)):
            r = time_steps(og, torch, tp, tm, prm, wsb, prec, steps, 1)
            for t in r["trees"]:
                t.close()
            row[prec] = {"value": n / (r["total_ms"] / steps * 1e-3), "ms_per_step": r["total_ms"] / steps,
                         "build_ms": float(r["build_ms"].mean()), "walk_ms": float(r["walk_ms"].mean())}
        t = og.Tree(tp, tm, 1.0, prm, stream=torch.cuda.current_stream(), workspace=wsb)
        am, _, nm = t.force(precision="mixed", with_counts=True)
        ad, _, nd = t.force(precision="fp64", with_counts=True)
        torch.cuda.synchronize()
        t.close()
        row["interactions_per_target"] = float(nm.sum().item()) / n
        if otree is not None:
            order, goff = oracle.curve_groups(otree, gm)
            rng = np.random.default_rng(17)
            gsel = np.sort(rng.choice(len(goff) - 1, 64, replace=False))
            members = np.concatenate([order[goff[g]:goff[g + 1]] for g in gsel])
            a_o, _, n_o = oracle.walk_groups(otree, gm, targets=members)
            e_m = _rel_err(am.cpu().numpy()[members], a_o)
            row["error_vs_oracle"] = {
                "targets": int(members.size), "mixed_median": float(np.median(e_m)),
                "mixed_p99": float(np.percentile(e_m, 99)),
                "fp64_max": float(_rel_err(ad.cpu().numpy()[members], a_o).max()),
                "fp64_counts_equal": bool(np.array_equal(nd.cpu().numpy()[members], n_o))}
        log("  group lists %d: mixed %.3f ms/step, fp64 %.3f, %.0f interactions/target"
            % (gm, row["mixed"]["ms_per_step"], row["fp64"]["ms_per_step"], row["interactions_per_target"]))
        out["group_max_%d" % gm] = row
        del wsb
    out["workload"] = "mixture2m as the headline, group-shared lists (OG_LISTS_GROUP)"
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()

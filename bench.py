"""Benchmark of the inexact-policy-iteration hot path on one MI355X.

One step = one full mdp_solve: float64 inexact policy iteration with GMRES(30)
policy evaluation, from v = 0 to ||T v - v||_inf <= 1e-8, with the instance
resident in HBM before the timed region.  The default workload is the largest
single-GPU configuration: S = 4e6 states, A = 16 actions, 24 uniform-random
nonzeros per row (1.536G nonzeros), Dirichlet(0.5) probabilities,
Lognormal(0,1) costs, gamma = 0.995; the mixed-precision solve on the same
instance is reported beside it.  --config 1..3 select the other single-MDP
workloads and --config 5 the serving load.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Bellman sweeps/s + HBM GB/s (% peak); solve time to ‖Tv−v‖∞≤1e-8, "
          "FP64 vs mixed")
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2502_14474_amd/csrc/device.h", "paper_2502_14474_amd/csrc/kernels.hip",
                  "paper_2502_14474_amd/csrc/colblock.hip", "paper_2502_14474_amd/csrc/internal.h",
                  "paper_2502_14474_amd/csrc/xcdprod.hip")
COUNTERS_GLOB = os.path.join(ROOT, "profiles", "counters_*.json")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kind, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (profiles/counters_*.json), or None when none
    was taken on this workload with the current kernel sources."""
    import glob
    sha = None
    for path in sorted(glob.glob(COUNTERS_GLOB)):
        try:
            with open(path) as f:
                d = json.load(f)
        except (OSError, ValueError):
            continue
        if d.get("workload") != workload:
            continue
        sha = sha or kernel_source_sha()
        if d.get("source_sha") != sha:
            continue
        k = d.get("kernels", {}).get(kind)
        if k is not None:
            return k.get("traffic_bytes_per_launch")
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_instance(args):
    from workloads import config1, config2, config3, config4
    if args.config == 1:
        return config1(seed=args.seed)
    if args.config == 2:
        inst = config2(S=args.S or 1_000_000, n_band=16 - args.n_jump, n_jump=args.n_jump, seed=args.seed)
        if args.n_jump != 2:  # another workload: its own name, so no stored counters apply
            inst.name = f"band-dirichlet1-{args.n_jump}-jumps"
        return inst
    if args.config == 3:
        side = args.S or 2000
        return config3(H=side, W=side, seed=args.seed)
    if args.config == 4:
        return config4(S=args.S or 4_000_000, seed=args.seed)
    raise SystemExit("unknown config")


def workload_key(inst):
    return f"{inst.name}:S={inst.S}:A={inst.A}:nnz={inst.nnz}:seed={inst.meta.get('seed')}"


def workload_name(inst, args):
    pre = (f" with the degree-{args.precond_degree} polynomial preconditioner"
           if getattr(args, "precond_degree", 1) > 1 else "")
    return (f"{inst.name} MDP (config {args.config}): S={inst.S}, A={inst.A}, nnz={inst.nnz}, "
            f"gamma={inst.gamma}; float64 inexact policy iteration, GMRES({args.restart}) "
            f"evaluation{pre}, alpha={args.alpha}, to ||Tv-v||_inf<={args.atol} from v=0")


ORACLE_RUNS_FILE = os.path.join(ROOT, "profiles", "oracle_full_runs.json")


def oracle_full_run(inst):
    """The recorded full oracle solve of this exact instance (written by
    oracle/full_run.py), or None."""
    try:
        with open(ORACLE_RUNS_FILE) as f:
            return json.load(f).get(workload_key(inst))
    except (OSError, ValueError):
        return None


def blas_threads():
    from threadpoolctl import threadpool_info
    n = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
    return max(n) if n else 1


def cpu_baseline(args, inst):
    """The CPU oracle (oracle/: plain float64 exact policy iteration) timed on
    this run's host cores, on the benchmarked instance itself.

    Small workloads (S <= 1e6) run the oracle's whole solve.  Larger ones time
    the two full-size steps an exact-PI solve repeats: one greedy sweep
    (oracle.bellman) and one certified policy evaluation
    (oracle.evaluate_policy) at the first policy; a solve is then priced with
    the sweep and evaluation counts of the oracle's recorded full run on the
    same instance (profiles/oracle_full_runs.json).  The CSR conversion is a
    format copy and is not timed, like the instance generation."""
    import numpy as np

    import oracle
    cores = blas_threads()
    avail = len(os.sched_getaffinity(0))
    base = {"unit": "solves/s", "cores": cores, "kind": "oracle", "host_cores_available": avail,
            "sparse_matvec_threads": 1}
    if inst.S <= 1_000_000:
        t0 = time.perf_counter()
        r = oracle.policy_iteration(inst, method="auto")
        dt = time.perf_counter() - t0
        return dict(base, value=1.0 / dt, seconds=dt,
                    sample=(f"the oracle's whole exact policy iteration on this instance: {dt:.2f} s, "
                            f"{r['iters']} improvement steps, final residual {r['res']:.1e}; scipy's "
                            f"sparse matvec runs on 1 thread, BLAS on {cores}"))
    P = oracle.to_csr(inst)
    t0 = time.perf_counter()
    _, pi0, res0 = oracle.bellman(inst, np.zeros(inst.S), P)
    t_sweep = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, true_res = oracle.evaluate_policy(inst, pi0, P, method="certified")
    t_eval = time.perf_counter() - t1
    del P
    steps = {"sweep_s": t_sweep, "evaluation_s": t_eval, "evaluation_true_residual": true_res}
    rec = oracle_full_run(inst)
    if rec is None:
        return dict(base, value=None, steps=steps,
                    sample=(f"one full-size oracle sweep ({t_sweep:.2f} s) and one certified evaluation "
                            f"({t_eval:.2f} s); no recorded full oracle run of this instance to count "
                            f"its steps, so no solve rate"))
    est = rec["sweeps"] * t_sweep + rec["evaluations"] * t_eval
    return dict(base, value=1.0 / est, seconds=est, steps=steps, full_run=rec,
                sample=(f"one full-size oracle sweep ({t_sweep:.2f} s) and one certified policy "
                        f"evaluation ({t_eval:.2f} s) on this instance, priced at the "
                        f"{rec['sweeps']} sweeps and {rec['evaluations']} evaluations of the oracle's "
                        f"recorded full solve of it ({rec['seconds']:.0f} s on {rec['cores']} BLAS "
                        f"threads): {est:.1f} s per solve"))


def serving_requests(args):
    """The first `serve_pool` requests of the seeded config-5 stream: S
    log-uniform in [1e3, 1e6], A in 2..16, nnz/row in 4..32 (band plus long
    jumps), gamma in {0.9, 0.99, 0.999}; the full law, nothing filtered."""
    from workloads import config5_requests
    return config5_requests(args.serve_pool, seed=args.seed)


def serving_oracle(args, reqs):
    """The oracle on a stratified subsample of the pool: per decade of S
    (1e3-1e4, 1e4-1e5, 1e5-1e6, each a third of the log-uniform law) and per
    discount (0.9, 0.99, 0.999, each a third), the pool's smallest request of
    that cell (smallest S*A*k, which keeps the oracle's time bounded and so
    favours the CPU), solved by the oracle's exact policy iteration.  A solve
    costs the mean over the cells."""
    import oracle
    from workloads import config5_instance
    times, picks = [], []
    cells = [(lo, g) for lo in (1e3, 1e4, 1e5) for g in (0.9, 0.99, 0.999)]
    for lo, g in cells:
        cand = [r for r in reqs if lo <= r["S"] < 10 * lo and r["gamma"] == g]
        r = min(cand, key=lambda r: r["S"] * r["A"] * r["k"]) if cand else None
        if r is None:
            continue
        inst = config5_instance(r, workers=16)
        t0 = time.perf_counter()
        out = oracle.policy_iteration(inst, method="auto" if inst.S <= 2500 else "certified")
        dt = time.perf_counter() - t0
        times.append(dt)
        picks.append(dict(S=r["S"], A=r["A"], k=r["k"], gamma=r["gamma"], nnz=inst.nnz, seconds=dt,
                          improvement_steps=out["iters"]))
        log(f"[serve] oracle on S={r['S']} A={r['A']} k={r['k']} gamma={r['gamma']}: {dt:.1f}s")
    mean = sum(times) / len(times)
    return {"value": 1.0 / mean, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "host_cores_available": len(os.sched_getaffinity(0)), "sparse_matvec_threads": 1,
            "sample": (f"oracle exact policy iteration on the smallest pool request of each (decade of S, "
                       f"gamma) cell, {len(picks)} cells: mean {mean:.2f} s per solve"), "requests": picks}


def serving_bench(args, m):
    """Config 5: a continuous-batching server under the serving load.

    A pool of distinct requests drawn from the full law is generated before
    the timed runs (host generation of the whole 10,000-request stream would
    take most of an hour, at about 70M nonzeros/s).  Submission i sends pool
    request i mod pool, in stream order.  One server takes every run: an
    untimed warm-up pass over the pool, a closed-loop run (every request
    submitted at once) that measures the capacity C, then open-loop Poisson
    streams at 0.7 C and 0.9 C with the stream's seeded exponential gaps.
    Mixed float32 with float64 refinement, the server's default."""
    import numpy as np
    import torch

    from workloads import MDPInstance, config5_instance, config5_requests
    reqs = serving_requests(args)
    t = time.time()
    pageable = [config5_instance(r, workers=16) for r in reqs]
    nnz = np.array([p.nnz for p in pageable])
    log(f"[serve] pool of {len(pageable)} requests, {nnz.sum()/1e9:.2f}G nnz (median {np.median(nnz)/1e6:.1f}M, "
        f"max {nnz.max()/1e6:.0f}M), generated in {time.time()-t:.1f}s")

    def pin(a):
        return torch.from_numpy(a).pin_memory().numpy()
    pool = [MDPInstance(p.S, p.A, pin(p.row_ptr), pin(p.col), pin(p.val), pin(p.cost), p.gamma,
                        name=p.name, meta=p.meta) for p in pageable]
    del pageable
    n = args.serve_requests or 3 * len(pool)

    def run(srv, gaps, n=n, tag=""):
        ids = []
        t0 = time.perf_counter()
        nxt = t0
        for i in range(n):
            if gaps is not None:
                nxt += gaps[i]
                dt = nxt - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            ids.append(srv.submit(pool[i % len(pool)], borrow=True))
        outs = [srv.wait(r) for r in ids]
        t1 = time.perf_counter()
        if args.serve_dump:
            with open(args.serve_dump, "a") as f:
                f.write(json.dumps({"run": tag, "requests": [
                    {"i": i, "nnz": int(pool[i % len(pool)].nnz), "S": int(pool[i % len(pool)].S),
                     "gamma": pool[i % len(pool)].gamma, "submit_ms": o[2]["submit_ms"],
                     "admit_ms": o[2]["admit_ms"], "finish_ms": o[2]["finish_ms"],
                     "sweeps": o[2]["bellman_sweeps"], "inner": o[2]["inner_iters"]}
                    for i, o in enumerate(outs)]}) + "\n")
        lat = np.array([o[2]["finish_ms"] - o[2]["submit_ms"] for o in outs])
        wait = np.array([o[2]["admit_ms"] - o[2]["submit_ms"] for o in outs])
        size = np.array([pool[i % len(pool)].nnz for i in range(n)])
        small = size <= np.median(size)
        bad = [o[2]["status"] for o in outs if o[2]["status"] != 0]
        log(f"[serve] run of {n}: {n / (t1 - t0):.1f} solves/s, p50 {np.percentile(lat, 50):.1f} ms, "
            f"p99 {np.percentile(lat, 99):.1f} ms; queue wait p50 {np.percentile(wait, 50):.1f} ms; "
            f"p50 small/large {np.percentile(lat[small], 50):.1f}/{np.percentile(lat[~small], 50):.1f} ms")
        return dict(solves_per_s=n / (t1 - t0), p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), ok=not bad, wall_s=t1 - t0,
                    residual_max=float(max(o[2]["residual"] for o in outs)),
                    queue_wait_p50_ms=float(np.percentile(wait, 50)),
                    service_p50_ms=float(np.percentile(lat - wait, 50)),
                    p50_ms_smaller_half=float(np.percentile(lat[small], 50)),
                    p50_ms_larger_half=float(np.percentile(lat[~small], 50)))

    # the server times the lane widths of each new (A, row length) class once,
    # at the class's first admission; the widths land in this run's own cache
    import tempfile
    tune_file = os.path.join(tempfile.mkdtemp(prefix="mdp_tune_"), "tune.json")
    os.environ["MDP_TUNE_CACHE"] = tune_file
    with m.Server(precision=m.MDP_MIXED_FP32, alpha=args.alpha, atol=args.atol,
                  hbm_budget_bytes=int(args.serve_budget_gib * (1 << 30)),
                  max_batch=args.serve_max_batch, autotune=not args.no_autotune,
                  split_nnz=args.split_nnz, trace_path=args.serve_trace,
                  launch={"auto": m.MDP_LAUNCH_AUTO, "graphs": m.MDP_LAUNCH_GRAPHS,
                          "direct": m.MDP_LAUNCH_DIRECT}[args.serve_launch]) as srv:
        warm = run(srv, None, len(pool), tag="warm")
        closed = run(srv, None, tag="closed")
        cap = closed["solves_per_s"]
        gaps = np.array([r["gap"] for r in config5_requests(n, seed=args.seed)])
        # an untimed open-loop pass first: batches of the sizes spread arrivals
        # produce (and their captured graphs) are new to the server after the
        # closed loop
        warm_open = run(srv, gaps / (0.5 * cap), tag="open0.5")
        open70 = run(srv, gaps / (0.7 * cap), tag="open0.7")
        open90 = run(srv, gaps / (0.9 * cap), tag="open0.9")
    try:
        with open(tune_file) as f:
            tuned = json.load(f)
    except (OSError, ValueError):
        tuned = {}
    cpu = None if args.no_cpu_baseline else serving_oracle(args, reqs)
    return {
        "metric": METRIC,
        "value": closed["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": len(pool),
        "ms_per_step": 1e3 * closed["wall_s"] / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"serving load (config 5): {len(pool)} distinct requests from the seeded "
                                f"stream's law (S log-uniform in [1e3,1e6], A 2..16, 4..32 nnz/row, "
                                f"gamma in {{0.9,0.99,0.999}}), submitted {n} times in stream order; "
                                f"mixed float32 + float64 refinement to ||Tv-v||_inf<={args.atol}"),
                   "pool": len(pool), "pool_nnz": int(nnz.sum()), "pool_max_states": int(max(p.S for p in pool)),
                   "submissions": n, "alpha": args.alpha, "hbm_budget_gib": args.serve_budget_gib,
                   "max_batch": args.serve_max_batch},
        "roofline": None,
        "cpu_baseline": cpu,
        "serving": {"warmup_pass": warm, "closed_loop": closed, "open_loop_warmup_0.5C": warm_open,
                    "open_loop_0.7C": open70,
                    "open_loop_0.9C": open90, "client_memory": "page-locked", "autotuned_widths": tuned,
                    "launch": args.serve_launch, "split_nnz": args.split_nnz},
    }


def graph_sweep_rate(m, inst, lanes, n=1000, replays=5):
    """Sweeps/s of value-iteration sweeps v <- T v replayed from one captured
    HIP graph of n sweeps (the allocation-free sweep, two buffers): what a
    small MDP reaches once the per-launch host work and syncs are gone."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rp, col, val, cost = t(inst.row_ptr.astype(np.int64)), t(inst.col), t(inst.val), t(inst.cost)
    va = torch.zeros(inst.S, dtype=torch.float64, device=dev)
    vb = torch.zeros_like(va)
    pol = torch.zeros(inst.S, dtype=torch.int32, device=dev)
    res = torch.zeros(1, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)

    def sweeps(count):
        for _ in range(count // 2):
            for x, y in ((va, vb), (vb, va)):
                m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma, x, y, pol, res,
                                      lanes_per_row=lanes, stream=s.cuda_stream)

    with torch.cuda.stream(s):
        sweeps(2)  # resolves the scratch address before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        sweeps(n)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"sweeps_per_s": n * replays / dt, "us_per_sweep": 1e6 * dt / (n * replays), "graph_sweeps": n,
            "replays": replays, "residual_after": float(res.item())}


def rows_leg(args, m, h, inst, v, pi, stream):
    """Times the path's other steps on the solved MDP: the policy product on
    its own (20 launches at the greedy policy of the solution, warm and after a
    1 GiB cache scrub each), the sweep after a scrub, solves with
    Richardson, BiCGSTAB and TFQMR inner iterations, and the per-kernel
    breakdown of one float64 GMRES solve.  Rates use the library's
    algorithmic byte counts."""
    import torch

    def summary(prof):
        out = {}
        for k, d in prof.items():
            if d["launches"]:
                avg = d["ms"] / d["launches"]
                gbs = d["bytes"] / d["launches"] / (avg * 1e-3) / 1e9 if d["bytes"] else None
                out[k] = {"launches": d["launches"], "avg_us": 1e3 * avg,
                          "gbs": gbs, "frac": gbs / HBM_PEAK_GBS if gbs else None}
        return out

    rows = {}
    y = torch.empty_like(v)
    m.mdp_policy_apply(h, pi, v, y, 0)
    m.mdp_profile(h, kinds=["policy_apply"])
    for _ in range(20):
        m.mdp_policy_apply(h, pi, v, y, 0)
    torch.cuda.synchronize()
    rows["policy_product"] = summary(m.mdp_profile_read(h))["policy_apply"]
    m.mdp_profile(h, False)

    # Cold: a 1 GiB copy on the handle's stream before each launch, so none of
    # the kernel's working set is left in the 256 MB Infinity Cache (the warm
    # numbers above and in the solve can be served partly from it).
    scrub_a = torch.zeros(1 << 27, dtype=torch.float64, device=v.device)
    scrub_b = torch.empty_like(scrub_a)
    Tv = torch.empty_like(v)
    p_tmp = torch.empty_like(pi)
    m.mdp_profile(h, kinds=["policy_apply", "bellman"])
    for _ in range(20):
        with torch.cuda.stream(stream):
            scrub_b.copy_(scrub_a)
        m.mdp_policy_apply(h, pi, v, y, 0)
        with torch.cuda.stream(stream):
            scrub_b.copy_(scrub_a)
        m.mdp_bellman(h, v, Tv, p_tmp)
    torch.cuda.synchronize()
    raw = m.mdp_profile_read(h)
    m.mdp_profile(h, False)
    cold = summary(raw)
    prof_bytes = {k: d["bytes"] / d["launches"] for k, d in raw.items() if d["launches"]}
    for k, name in (("policy_apply", "policy_product_cold"), ("bellman", "bellman_cold")):
        if k in cold:
            cold[k]["working_set_mb"] = prof_bytes.get(k, 0.0) / 1e6
            rows[name] = cold[k]
    del scrub_a, scrub_b

    if inst.gamma <= 0.99:
        w = torch.zeros_like(v)
        p2 = torch.zeros_like(pi)
        m.mdp_profile(h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.mdp_solve(h, w, p2, inner=m.MDP_INNER_RICHARDSON, alpha=args.alpha, atol=args.atol,
                         max_inner=200000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rows["richardson_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"],
                                    "sweeps": st["bellman_sweeps"], "inner": st["inner_iters"],
                                    "residual": st["residual"],
                                    "kernels": summary(m.mdp_profile_read(h))}
        m.mdp_profile(h, False)

    w = torch.zeros_like(v)
    p2 = torch.zeros_like(pi)
    m.mdp_solve(h, w, p2, inner=m.MDP_INNER_BICGSTAB, alpha=args.alpha, atol=args.atol)  # warm-up
    w.zero_()
    m.mdp_profile(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = m.mdp_solve(h, w, p2, inner=m.MDP_INNER_BICGSTAB, alpha=args.alpha, atol=args.atol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rows["bicgstab_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"],
                              "sweeps": st["bellman_sweeps"], "inner": st["inner_iters"],
                              "residual": st["residual"], "kernels": summary(m.mdp_profile_read(h))}
    m.mdp_profile(h, False)

    w.zero_()
    m.mdp_solve(h, w, p2, inner=m.MDP_INNER_TFQMR, alpha=args.alpha, atol=args.atol)  # warm-up
    w.zero_()
    m.mdp_profile(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = m.mdp_solve(h, w, p2, inner=m.MDP_INNER_TFQMR, alpha=args.alpha, atol=args.atol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rows["tfqmr_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"],
                           "sweeps": st["bellman_sweeps"], "inner": st["inner_iters"],
                           "residual": st["residual"], "kernels": summary(m.mdp_profile_read(h))}
    m.mdp_profile(h, False)

    # GMRES with the polynomial preconditioner sum_{i<d} (gamma P_pi)^i
    for deg in (2, 4):
        w.zero_()
        m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol, precond_degree=deg)
        w.zero_()
        m.mdp_profile(h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol, precond_degree=deg)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rows[f"gmres_precond{deg}_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"],
                                             "sweeps": st["bellman_sweeps"], "inner": st["inner_iters"],
                                             "products": st["policy_applies"], "residual": st["residual"],
                                             "kernels": summary(m.mdp_profile_read(h))}
        m.mdp_profile(h, False)
        log(f"[bench] gmres + polynomial preconditioner of degree {deg}: {1e3 * (t1 - t0):.1f} ms, "
            f"{st['inner_iters']} Arnoldi steps, {st['policy_applies']} products")

    if not args.no_mixed:
        # mixed float32 inner solves with the polynomial preconditioner
        mp = m.MDP_MIXED_FP32 if args.mixed == "fp32" else m.MDP_MIXED_FP16
        w.zero_()
        m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol, precision=mp,
                    precond_degree=4)
        w.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol, precision=mp,
                         precond_degree=4)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rows["mixed_precond4_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"], "sweeps": st["bellman_sweeps"],
                                        "inner": st["inner_iters"], "products": st["policy_applies"],
                                        "refinements": st["refinements"], "residual": st["residual"],
                                        "precision": args.mixed}
        log(f"[bench] mixed {args.mixed} + polynomial preconditioner of degree 4: {1e3 * (t1 - t0):.1f} ms")

    # GMRES with a second Gram-Schmidt pass: its cost, and the loss of
    # orthogonality the default single pass leaves (the second correction)
    w.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol, gs_passes=2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rows["gmres_cgs2_solve"] = {"ms": 1e3 * (t1 - t0), "status": st["status"], "sweeps": st["bellman_sweeps"],
                                "inner": st["inner_iters"], "orth_loss": st["orth_loss"],
                                "residual": st["residual"]}
    log(f"[bench] gmres with CGS2: {1e3 * (t1 - t0):.1f} ms, {st['inner_iters']} steps, "
        f"loss of orthogonality of one pass {st['orth_loss']:.2e}")

    # the inexactness parameter: solve time against alpha (each inner solve
    # stops at alpha times its initial residual; alpha -> 0 is exact PI)
    sweep = {}
    for a in (1e-1, 1e-2, 1e-4, 1e-6):
        w.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.mdp_solve(h, w, p2, restart=args.restart, alpha=a, atol=args.atol, max_inner=100000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sweep[f"{a:g}"] = {"ms": 1e3 * (t1 - t0), "status": st["status"], "sweeps": st["bellman_sweeps"],
                           "inner": st["inner_iters"], "residual": st["residual"]}
    rows["gmres_alpha_sweep"] = sweep
    log("[bench] alpha sweep: " + ", ".join(f"{a}: {d['ms']:.1f} ms ({d['sweeps']} sweeps, {d['inner']} steps)"
                                             for a, d in sweep.items()))

    w = torch.zeros_like(v)
    p2 = torch.zeros_like(pi)
    m.mdp_profile(h, True)
    st = m.mdp_solve(h, w, p2, restart=args.restart, alpha=args.alpha, atol=args.atol)
    torch.cuda.synchronize()
    rows["gmres_solve_kernels"] = summary(m.mdp_profile_read(h))
    m.mdp_profile(h, False)
    pc, bc = rows.get("policy_product_cold", {}), rows.get("bellman_cold", {})
    log(f"[bench] cold (after a 1 GiB scrub): policy product {pc.get('avg_us', float('nan')):.1f} us "
        f"(working set {pc.get('working_set_mb', float('nan')):.0f} MB), sweep {bc.get('avg_us', float('nan')):.1f} us "
        f"(working set {bc.get('working_set_mb', float('nan')):.0f} MB)")
    log(f"[bench] rows: policy product {rows['policy_product']['avg_us']:.1f} us, "
        f"richardson {rows.get('richardson_solve', {}).get('ms', float('nan')):.1f} ms, "
        f"bicgstab {rows['bicgstab_solve']['ms']:.1f} ms ({rows['bicgstab_solve']['inner']} its), "
        f"tfqmr {rows['tfqmr_solve']['ms']:.1f} ms ({rows['tfqmr_solve']['inner']} its)")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--S", type=int, default=0)
    ap.add_argument("--n-jump", type=int, default=2,
                    help="config 2: long jumps per row (of 16 entries); 0 gives the band-only "
                         "twin used to separate the cost of the long-jump gathers")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--alpha", type=float, default=1e-2)
    ap.add_argument("--atol", type=float, default=1e-8)
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--precond-degree", type=int, default=1,
                    help="GMRES polynomial preconditioner sum_{i<d} (gamma P_pi)^i for the timed solves (1: none)")
    ap.add_argument("--profile-every", type=int, default=4,
                    help="time one launch in this many per kernel class inside the timed region")
    ap.add_argument("--autotune", action="store_true",
                    help="time the lane widths on this MDP (mdp_autotune) before the timed solves")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed", choices=["fp32", "fp16"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the per-row leg (policy product, Richardson solve, GMRES kernel breakdown)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve-pool", type=int, default=96,
                    help="config 5: distinct requests generated from the stream's law")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="config 5: submissions per run (0: three times the pool)")
    ap.add_argument("--serve-max-batch", type=int, default=128)
    ap.add_argument("--serve-budget-gib", type=float, default=192.0,
                    help="config 5: the server's HBM budget (of the 288 GB on the GPU)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="config 5: the server keeps the default lane widths")
    ap.add_argument("--serve-trace", default=None,
                    help="config 5: file for the server's trace of admissions, rounds and retirements")
    ap.add_argument("--serve-dump", default=None,
                    help="config 5: append every request's times, size and iteration counts to this file")
    ap.add_argument("--serve-launch", choices=["auto", "graphs", "direct"], default="auto",
                    help="config 5: how the server's GMRES cycles reach the GPU")
    ap.add_argument("--split-nnz", type=int, default=None,
                    help="config 5: the server's size-class split (0: one worker; default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the "
              "multi-GPU sharding of the path is a design, not a build).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2502_14474_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] copy calibration: 3 copies of 1 GiB")

    if args.config == 5:
        print(json.dumps(serving_bench(args, m)), flush=True)
        return

    t = time.time()
    inst = make_instance(args)
    log(f"[bench] generated {inst.name} S={inst.S} A={inst.A} nnz={inst.nnz} in {time.time()-t:.1f}s")
    stream = torch.cuda.Stream(device=dev)
    t = time.time()
    h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma,
                     stream=stream.cuda_stream, device=0, lanes_per_row=args.lanes,
                     low_precision=0 if args.no_mixed else (
                         m.MDP_BUILD_FP32 if args.mixed == "fp32" else m.MDP_BUILD_FP16))
    create_s = time.time() - t  # host validation, upload and low-precision copies; not in `value`
    if args.autotune:
        t1 = time.time()
        lanes = m.mdp_autotune(h)
        log(f"[bench] autotuned lanes per row: {lanes} in {time.time()-t1:.1f}s")
    info = m.mdp_info(h)
    log(f"[bench] created handle in {time.time()-t:.1f}s: {info}")
    v = torch.zeros(inst.S, dtype=torch.float64, device=dev)
    pi = torch.zeros(inst.S, dtype=torch.int32, device=dev)
    kw = dict(restart=args.restart, alpha=args.alpha, atol=args.atol)

    def solve(prec):
        return m.mdp_solve(h, v, pi, precision=prec, precond_degree=args.precond_degree, **kw)

    for _ in range(args.warmup):
        st = solve(m.MDP_FP64)
        assert st["status"] == m.MDP_OK, st
        log(f"[bench] warmup solve: {st['time_ms']:.2f} ms, sweeps {st['bellman_sweeps']}, "
            f"inner {st['inner_iters']}, res {st['residual']:.3e}")

    # ---- timed region: K full float64 solves ---------------------------------
    # HIP events bracket the two heaviest kernel classes only, and only one
    # launch in --profile-every of each: every event record leaves the GPU idle
    # for a few microseconds, which would otherwise count against the solve
    m.mdp_profile(h, kinds=["bellman", "arnoldi_apply"], every=args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        stats.append(solve(m.MDP_FP64))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = m.mdp_profile_read(h)
    m.mdp_profile(h, False)
    elapsed = t1 - t0
    for st in stats:
        assert st["status"] == m.MDP_OK, st
    v64 = v.cpu().numpy().copy()
    last = stats[-1]
    log(f"[bench] timed {args.steps} solves in {elapsed:.3f}s; last: sweeps {last['bellman_sweeps']}, "
        f"inner {last['inner_iters']}, res {last['residual']:.3e}")

    kernels = {}
    for k, d in prof.items():
        if d["launches"]:
            avg_ms = d["ms"] / d["launches"]
            kernels[k] = {"launches": d["launches"], "total_ms": d["ms"], "avg_us": 1e3 * avg_ms,
                          "bytes_per_launch": d["bytes"] / d["launches"],
                          "gbs": (d["bytes"] / d["launches"]) / (avg_ms * 1e-3) / 1e9 if d["bytes"] else None}
    dom = max((k for k in kernels if kernels[k]["gbs"]), key=lambda k: kernels[k]["total_ms"])
    achieved = kernels[dom]["gbs"]

    # ---- Bellman sweep rate ---------------------------------------------------
    Tv = torch.empty_like(v)
    m.mdp_profile(h, kinds=["bellman"])
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for _ in range(args.sweeps):
        m.mdp_bellman(h, v, Tv, pi)
    torch.cuda.synchronize()
    ts1 = time.perf_counter()
    sprof = m.mdp_profile_read(h)["bellman"]
    m.mdp_profile(h, False)
    sweep_avg_ms = sprof["ms"] / sprof["launches"]
    sweep_gbs = sprof["bytes"] / sprof["launches"] / (sweep_avg_ms * 1e-3) / 1e9

    graph_sweeps = None
    if inst.S <= 100_000:
        graph_sweeps = graph_sweep_rate(m, inst, info["lanes_per_row"])
        log(f"[bench] graph-replayed sweeps: {graph_sweeps['sweeps_per_s']:.0f}/s "
            f"({graph_sweeps['us_per_sweep']:.2f} us each) vs {args.sweeps / (ts1 - ts0):.0f}/s synced")

    # ---- the other rows of the path, each on its own ----------------------------
    rows = None if args.no_rows else rows_leg(args, m, h, inst, v, pi, stream)

    # ---- mixed precision --------------------------------------------------------
    mixed = None
    if not args.no_mixed:
        mp = m.MDP_MIXED_FP32 if args.mixed == "fp32" else m.MDP_MIXED_FP16
        for _ in range(args.warmup):
            solve(mp)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        mst = [solve(mp) for _ in range(args.steps)]
        torch.cuda.synchronize()
        tm1 = time.perf_counter()
        vm = v.cpu().numpy()
        mixed = {"ms_per_solve": 1e3 * (tm1 - tm0) / args.steps,
                 "speedup_vs_fp64": elapsed / (tm1 - tm0),
                 "residual": mst[-1]["residual"], "status": mst[-1]["status"],
                 "sweeps": mst[-1]["bellman_sweeps"], "inner": mst[-1]["inner_iters"],
                 "refinements": mst[-1]["refinements"],
                 "rel_diff_vs_fp64": float(np.max(np.abs(vm - v64)) / np.max(np.abs(v64)))}
        log(f"[bench] mixed: {mixed}")

    cpu = None
    if not args.no_cpu_baseline:
        t = time.time()
        cpu = cpu_baseline(args, inst)
        log(f"[bench] cpu baseline ({time.time() - t:.0f}s): {cpu}")

    m.mdp_destroy(h)
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(inst, args), "S": inst.S, "A": inst.A,
                   "nnz": inst.nnz, "gamma": inst.gamma, "inner": f"gmres({args.restart})",
                   "precond_degree": args.precond_degree,
                   "alpha": args.alpha, "atol": args.atol, "lanes_per_row": info["lanes_per_row"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(dom, workload_key(inst)),
                     "kernel": dom,
                     "bytes_per_launch": kernels[dom]["bytes_per_launch"],
                     "avg_us": kernels[dom]["avg_us"]},
        "cpu_baseline": cpu,
        "create_s": create_s,
        "bellman_sweeps_per_s": (graph_sweeps["sweeps_per_s"] if graph_sweeps else args.sweeps / (ts1 - ts0)),
        "bellman_sweeps_per_s_synced": args.sweeps / (ts1 - ts0),
        "graph_sweeps": graph_sweeps,
        "bellman_kernel": {"avg_us": 1e3 * sweep_avg_ms, "gbs": sweep_gbs,
                           "frac": sweep_gbs / HBM_PEAK_GBS,
                           "bytes_per_launch": sprof["bytes"] / sprof["launches"],
                           "traffic": counter_traffic("bellman", workload_key(inst))},
        "solve": {"sweeps": last["bellman_sweeps"], "inner": last["inner_iters"],
                  "residual": last["residual"], "history": last.get("history")},
        "mixed": dict(mixed, precision=args.mixed) if mixed else None,
        "rows": rows,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

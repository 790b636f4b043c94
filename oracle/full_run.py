"""Time the oracle's whole exact policy iteration on one benchmark workload and
record it (test and measurement infrastructure; nothing here is on the
solver's path).

    python3 -m oracle.full_run --config 4 [--out profiles/oracle_full_runs.json]

The record, keyed like the benchmark's workloads, holds the number of greedy
sweeps and policy evaluations the solve took, its wall time and the BLAS
thread count; bench.py prices a solve from one timed sweep and one timed
evaluation on the same instance and these counts.  Generation and the CSR
conversion are not timed.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def instance(cfg, seed):
    from workloads import config1, config2, config3, config4
    return {1: lambda: config1(seed=seed), 2: lambda: config2(seed=seed),
            3: lambda: config3(seed=seed), 4: lambda: config4(seed=seed)}[cfg]()


def key(inst):
    return f"{inst.name}:S={inst.S}:A={inst.A}:nnz={inst.nnz}:seed={inst.meta.get('seed')}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "oracle_full_runs.json"))
    args = ap.parse_args()
    from threadpoolctl import threadpool_info
    t = time.time()
    inst = instance(args.config, args.seed)
    print(f"[oracle] generated {key(inst)} in {time.time() - t:.1f}s", flush=True)
    P = oracle.to_csr(inst)
    counts = {"sweeps": 0, "evaluations": 0}
    bellman, evaluate = oracle.bellman, oracle.evaluate_policy

    def counted_bellman(*a, **k):
        counts["sweeps"] += 1
        t = time.perf_counter()
        out = bellman(*a, **k)
        print(f"[oracle] sweep {counts['sweeps']}: residual {out[2]:.3e} ({time.perf_counter() - t:.1f}s)",
              flush=True)
        return out

    def counted_evaluate(*a, **k):
        counts["evaluations"] += 1
        t = time.perf_counter()
        out = evaluate(*a, **k)
        print(f"[oracle] evaluation {counts['evaluations']}: true residual {out[1]:.1e} "
              f"({time.perf_counter() - t:.1f}s)", flush=True)
        return out

    # count the steps of the unmodified solve: the two step functions are
    # wrapped for the duration of the run only
    oracle.mdp_oracle.bellman, oracle.mdp_oracle.evaluate_policy = counted_bellman, counted_evaluate
    try:
        orig_to_csr = oracle.mdp_oracle.to_csr
        oracle.mdp_oracle.to_csr = lambda _inst: P  # the conversion above, not timed again
        t0 = time.perf_counter()
        r = oracle.policy_iteration(inst, method="certified")
        dt = time.perf_counter() - t0
    finally:
        oracle.mdp_oracle.bellman, oracle.mdp_oracle.evaluate_policy = bellman, evaluate
        oracle.mdp_oracle.to_csr = orig_to_csr
    blas = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
    rec = {"sweeps": counts["sweeps"], "evaluations": counts["evaluations"], "seconds": dt,
           "improvement_steps": r["iters"], "final_residual": r["res"],
           "cores": max(blas) if blas else 1, "host_cores_available": len(os.sched_getaffinity(0)),
           "command": f"python3 -m oracle.full_run --config {args.config} --seed {args.seed}"}
    print(f"[oracle] {key(inst)}: {json.dumps(rec)}", flush=True)
    try:
        with open(args.out) as f:
            runs = json.load(f)
    except (OSError, ValueError):
        runs = {}
    runs[key(inst)] = rec
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(runs, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

"""Benchmark: FastSV connected components on one MI355X.

One step = one complete connected-components solve (every iteration of
hooking, shortcutting, grandparent and termination test) of the R-MAT
scale-24 / edge-factor-16 graph (16.8M vertices, 268M undirected edge draws,
a=.57 b=c=.19 d=.05, permuted ids; seed 2), already resident in HBM.

Prints one JSON line:
  value    undirected edges per second per solve (m_eff * steps / time)
  roofline dense hooking kernel (the dominant one): algorithmic bytes per
           launch / average launch time from HIP events on its stream, vs 8 TB/s
  cpu_baseline  the union-find oracle on the host, one core, full graph
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "er65k", "grid4096", "rmat20"])
    ap.add_argument("--tau", type=float, default=None, help="frontier threshold (default: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="counter-measured HBM bytes per dense launch (written from rocprofv3 runs)")
    return ap.parse_args()


def make_graph(name):
    from paper_1910_05971_amd import graphgen as gg
    if name == "rmat24":
        return gg.c2_rmat(), {"workload": "rmat_scale24_ef16", "n": 1 << 24, "edge_draws": 16 << 24,
                              "a": 0.57, "b": 0.19, "c": 0.19, "seed": 2, "ids": "permuted"}
    if name == "rmat20":
        return gg.rmat(20, 16, seed=2), {"workload": "rmat_scale20_ef16", "n": 1 << 20, "seed": 2}
    if name == "er65k":
        return gg.c1_er(), {"workload": "er_n65536_m262144", "n": 65536, "edge_draws": 262144, "seed": 1}
    return gg.c3_grid(), {"workload": "grid_4096x4096_p0.55", "n": 4096 * 4096, "p": 0.55, "seed": 3}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1910_05971_amd as fs

    t0 = time.time()
    g, cfg = make_graph(args.workload)
    print(f"[bench] generated {cfg['workload']}: n={g.n} nnz={g.nnz} m_eff={g.m_eff} "
          f"in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = torch.empty(fs.workspace_bytes(g.n, g.nnz) + 256, dtype=torch.uint8, device=dev)
    kw = {} if args.tau is None else {"frontier_tau": args.tau}
    # validate once, outside the timed region
    _, st = fs.cc_csr(rp, col, labels=labels, workspace=ws, validate=True, **kw)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        fs.cc_csr(rp, col, labels=labels, workspace=ws, **kw)
    torch.cuda.synchronize()
    # timed region: every kernel is timed with HIP events on the call's stream
    hook_ms, hook_n, gp_ms, sparse_ms = 0.0, 0, 0.0, 0.0
    iters = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        _, st = fs.cc_csr(rp, col, labels=labels, workspace=ws, timing=True, **kw)
        iters.append(st.iterations)
        for k in range(min(st.iterations, 64)):
            if st.sparse[k]:
                sparse_ms += st.ms_hook[k]
            else:
                hook_ms += st.ms_hook[k]
                hook_n += 1
            gp_ms += st.ms_gp[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    value = g.m_eff * args.steps / elapsed

    # roofline of the dense hooking kernel: algorithmic bytes per launch
    n, nnz = g.n, g.nnz
    bytes_dense = 4 * (n + 1) + 8 * nnz + 12 * n
    avg_ms = hook_ms / max(hook_n, 1)
    achieved = bytes_dense / (avg_ms * 1e-3) / 1e9 if hook_n else 0.0
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            traffic = tj.get(cfg["workload"], {}).get("hook_dense_bytes")
        except Exception:
            traffic = None

    # correctness spot check of the timed output against the oracle (outside the timing)
    check = None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps, t_cpu = 0, 0.0
        while t_cpu < 10.0 and reps < 5:
            t1 = time.perf_counter()
            want = oracle.uf_labels(g.n, g.row_ptr, g.col)
            t_cpu += time.perf_counter() - t1
            reps += 1
        cpu = {"value": g.m_eff * reps / t_cpu, "unit": "undirected edges/s", "cores": 1, "kind": "oracle",
               "sample": f"union-find oracle over the whole graph, {reps} run(s), {t_cpu:.1f} s, single thread"}
        got = labels.cpu().numpy()
        check = bool(np.array_equal(got, want))

    out = {
        "metric": "undirected edges/s per CC solve",
        "value": value,
        "unit": "undirected edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": dict(cfg, m_eff=g.m_eff, nnz=g.nnz, iterations=iters[-1] if iters else None,
                       frontier_tau=args.tau),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_hook_dense", "alg_bytes_per_launch": bytes_dense,
                     "avg_launch_ms": avg_ms, "launches": hook_n},
        "breakdown_ms_per_step": {"hook_dense": hook_ms / args.steps, "hook_sparse": sparse_ms / args.steps,
                                  "grandparent": gp_ms / args.steps},
        "labels_match_oracle": check,
    }
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

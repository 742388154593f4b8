"""Benchmark: FastSV connected components on one MI355X.

Headline (the JSON line's value): one step = one complete connected-components
solve (every iteration of hooking, shortcutting, grandparent and termination
test) of the R-MAT scale-24 / edge-factor-16 graph (16.8M vertices, 268M
undirected edge draws, a=.57 b=c=.19 d=.05, ids permuted; seed 2), already
resident in HBM; value = undirected edges per second.

Also in the same JSON line:
  roofline      the kernel with the most time per solve, of the binned dense
                SpMV step (k_bin_pull<16> for R-MAT scale 24, whose bins are long,
                <8> for short bins; one launch per iteration) and the layout
                fill that also performs the first iteration (k_bin_fill<true>,
                once per solve); the other one is in roofline_other.  Each:
                algorithmic bytes per launch / its average launch time from HIP
                events on the call's stream, against 8 TB/s; traffic = counter-
                measured HBM bytes per launch (profiles/), null when the kernel
                sources have changed since they were taken
  solve_roofline  the same for the whole solve: the library's algorithmic
                bytes of all executed iterations over the wall time per solve,
                and the counter-measured bytes of all kernels of one solve
  cpu_baseline  the union-find oracle on the host, one core, the whole graph
  batched       4096 Erdos-Renyi graphs in one batched call vs one call per
                graph (graphs/s)
  serving       Poisson request stream (2000 req/s; 99% graphs from the batch
                distribution, 1% R-MAT scale 20) through the continuous-
                batching server vs one request at a time: p50/p99 latency and
                graphs/s, open loop and at saturation
  extras        on C1, C2 and C3: iterations and time of the convergence
                ablation sv1..sv5 (Algorithm 1 plus, in turn, the four changes
                of Sec. 3; sv5 is FastSV) and of the asynchronous mode; and a
                warm start of C2 from the labels of its first 99% edge draws
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "undirected edges/s per CC solve & % HBM peak; batched graphs/s & p99 vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "er65k", "grid4096", "rmat20"])
    ap.add_argument("--tau", type=float, default=None, help="frontier threshold (default: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default options instead of the autotuner's choice")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the convergence ablation, asynchronous mode and warm-start measurements")
    ap.add_argument("--serve-requests", type=int, default=22100,
                    help="requests in the serving trace; those arriving in the first --serve-warmup seconds are "
                         "served but not counted")
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--serve-er-pool", type=int, default=1024)
    ap.add_argument("--serve-rmat-pool", type=int, default=4)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="counter-measured HBM bytes per dense step (see profiles/)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (counter calibration) and exit")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_1910_05971_amd/csrc/kernels.h", "paper_1910_05971_amd/csrc/binned.h",
                  "paper_1910_05971_amd/csrc/engine.h")


def kernel_source_hash():
    """sha256 over the device-kernel sources: counter figures taken for another
    version of the kernels are not reported."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def copy_calibration(torch):
    a = torch.ones(256 * 1024 * 1024, dtype=torch.int32, device="cuda")  # 1 GiB
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 3}), flush=True)


def roofline_record(kernel, unit, alg_bytes, total_ms, launches, solves, src_hash, traffic_db):
    """Roofline figures of one kernel: algorithmic bytes per launch over its
    average launch time (HIP events on the call's stream), against HBM peak;
    traffic = counter-measured HBM bytes per launch from profiles/, reported
    only while the kernel sources are those the counters were taken with."""
    avg_ms = total_ms / max(launches, 1)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    traffic, by_req, l2_hit, note = None, None, None, "no counter record"
    rec = traffic_db.get(kernel)
    if "_error" in traffic_db:
        note = f"unreadable counter record: {traffic_db['_error']}"
    elif rec is not None:
        if rec.get("kernel_source_sha256_16") != src_hash:
            note = "kernel source changed since the counters were taken"
        else:
            # FETCH_SIZE + WRITE_SIZE, copy-scaled; beside it the same bytes
            # from the read and write request counts by request size
            traffic, note = rec.get("hbm_bytes_per_launch"), rec.get("source")
            by_req, l2_hit = rec.get("request_bytes_per_launch"), rec.get("l2_hit")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_by_request_size": by_req,
            "l2_hit": l2_hit, "traffic_note": note, "kernel": kernel,
            "unit_of_work": unit, "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms,
            "launches_timed": launches, "ms_per_solve": total_ms / max(solves, 1),
            "kernel_source_sha256_16": src_hash}


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


def bench_solve(args, fs, torch, np):
    t0 = time.time()
    g, cfg = make_graph(args.workload)
    log(f"generated {cfg['workload']}: n={g.n} nnz={g.nnz} m_eff={g.m_eff} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    kw = {} if args.tau is None else {"frontier_tau": args.tau}
    # the autotuner picks the threshold, bin width and span for this graph
    # (none of them changes the iterates); the timed solves use its choice
    tuning = None
    if not args.no_tune and args.tau is None:
        from paper_1910_05971_amd import tune
        t1 = time.time()
        rec = tune.tune_csr(rp, col, reps=2, save=False)
        kw = dict(rec["best"]["opts"])
        tuning = {"candidates": len(rec["results"]), "best_opts": kw, "best_ms": rec["best"]["ms"],
                  "default_opts": rec["default"]["opts"], "default_ms": rec["default"]["ms"],
                  "tuner_s": time.time() - t1}
        log(f"tuned {kw}: {rec['best']['ms']:.3f} ms vs default {rec['default']['ms']:.3f} ms "
            f"({len(rec['results'])} candidates, {time.time() - t1:.1f} s)")
    ws = torch.empty(fs.workspace_bytes(g.n, g.nnz, fs.make_opts(**{k: v for k, v in kw.items()})) + 256,
                     dtype=torch.uint8, device=dev)
    # validate once, outside the timed region
    fs.cc_csr(rp, col, labels=labels, workspace=ws, validate=True, **kw)
    # one traced solve, also untimed: the global atomics of every iteration's
    # hooking (8 B each, a read-modify-write, in the algorithmic bytes)
    _, tr = fs.cc_csr(rp, col, labels=labels, workspace=ws, trace=True, **kw)
    atomics = tr.atomics_list()
    for _ in range(args.warmup):
        fs.cc_csr(rp, col, labels=labels, workspace=ws, **kw)
    torch.cuda.synchronize()
    log("timed region")
    # every step of the solve is timed with HIP events on the call's stream
    gather_ms, gather_n, first_ms, sparse_ms, gp_ms, prep_ms = 0.0, 0, 0.0, 0.0, 0.0, 0.0
    solve_alg = 0
    iters = []
    binned = fused = False
    span = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    per_iter = None
    for _ in range(args.steps):
        _, st = fs.cc_csr(rp, col, labels=labels, workspace=ws, timing=True, **kw)
        iters.append(st.iterations)
        solve_alg = st.alg_bytes + 8 * max(tr.atomics_issued, 0)
        per_iter = st
        binned = st.binned_iterations > 0
        span = st.bin_span
        fused = st.bin_fused_first == 1
        prep_ms += st.ms_bin_prepare
        for k in range(min(st.iterations, 64)):
            if st.sparse[k]:
                sparse_ms += st.ms_hook[k]
            elif k == 0:
                first_ms += st.ms_hook[k]
            else:
                gather_ms += st.ms_hook[k]
                gather_n += 1
            gp_ms += st.ms_gp[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n, nnz = g.n, g.nnz
    src_hash = kernel_source_hash()
    traffic_db = {}
    if os.path.exists(args.traffic_json):
        try:
            traffic_db = json.load(open(args.traffic_json)).get(cfg["workload"], {})
        except Exception as e:  # a malformed record reads as missing
            traffic_db = {"_error": str(e)}
    kernels = []
    its = min(per_iter.iterations, 64) if per_iter else 0
    dense_ks = [k for k in range(1, its) if not per_iter.sparse[k]]
    # atomics per launch, from the traced solve (its iterates are the timed ones')
    a_first = atomics[0] if atomics else 0
    if gather_n:
        # one dense SpMV step (one launch), as the library counts it for the
        # traced solve: row_ptr, col, the G[col] gathers, then G, F, M per
        # row, and each atomic of the hooks as a read-modify-write
        hook_bytes = tr.alg_hook_list()
        per_launch = sum(hook_bytes[k] for k in dense_ks) / len(dense_ks)
        rec = roofline_record(f"k_bin_pull<{span}>" if binned else "k_tile_reduce<kGather>",
                              "one dense SpMV step", per_launch, gather_ms, gather_n, args.steps, src_hash,
                              traffic_db)
        kernels.append(rec)
    if fused and first_ms > 0:
        # the layout fill that also performs the first iteration: col and row_ptr
        # read, one 4-byte record per entry written (the markers, at most 256 per
        # bin, are left out), M and Fn written per row, the atomics of rows
        # shared by tiles
        kernels.append(roofline_record("k_bin_fill<true>", "layout fill fused with the first iteration",
                                       8 * nnz + 12 * n + 4 + 8 * a_first, first_ms, args.steps, args.steps,
                                       src_hash, traffic_db))
    # the dominant kernel is the one with the most time per solve
    kernels.sort(key=lambda r: -r["ms_per_solve"])
    # the whole solve: the library's count of algorithmic bytes over all executed
    # iterations, over the wall time per solve; traffic = counter-measured bytes
    # of all kernels of one solve
    solve_ms = 1000.0 * elapsed / args.steps
    srec = traffic_db.get("_solve") or {}
    solve = {"alg_bytes": solve_alg, "ms": solve_ms, "achieved": solve_alg / (solve_ms * 1e-3) / 1e9,
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": solve_alg / (solve_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "traffic": srec.get("hbm_bytes_per_solve") if srec.get("kernel_source_sha256_16") == src_hash else None}
    res = {
        "value": g.m_eff * args.steps / elapsed,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "config": dict(cfg, m_eff=g.m_eff, nnz=g.nnz, iterations=iters[-1] if iters else None,
                       frontier_tau=kw.get("frontier_tau"), solver_opts=kw),
        "tuning": tuning,
        "roofline": kernels[0] if kernels else None,
        "roofline_other": kernels[1:],
        "solve_roofline": solve,
        "breakdown_ms_per_solve": {"first_iteration": first_ms / args.steps, "bin_layout": prep_ms / args.steps,
                                   "dense_steps": gather_ms / args.steps, "sparse_push": sparse_ms / args.steps,
                                   "grandparent": gp_ms / args.steps},
        # per iteration of the last timed solve: the changed grandparents (the
        # frontier of the next iteration) as a count and a share of n, the
        # pass, the edge slots a sparse pass pushed, the hooks' atomics (from
        # the traced solve) and the kernel times
        "iterations_detail": [
            {"k": k + 1, "changed": per_iter.changed[k], "changed_frac": per_iter.changed[k] / n,
             "pass": "sparse" if per_iter.sparse[k] else ("fill+first" if k == 0 and fused else "dense"),
             "pushed": per_iter.pushed[k], "atomics": atomics[k] if k < len(atomics) else None,
             "alg_hook_bytes": tr.alg_hook[k],
             "ms_hook": per_iter.ms_hook[k], "ms_gp": per_iter.ms_gp[k]} for k in range(its)],
    }
    cpu = None
    check = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (union-find oracle, one core)")
        reps, t_cpu = 0, 0.0
        while t_cpu < 10.0 and reps < 5:
            t1 = time.perf_counter()
            want = oracle.uf_labels(g.n, g.row_ptr, g.col)
            t_cpu += time.perf_counter() - t1
            reps += 1
        cpu = {"value": g.m_eff * reps / t_cpu, "unit": "undirected edges/s", "cores": 1, "kind": "oracle",
               "sample": f"union-find oracle over the whole {cfg['workload']} graph, {reps} run(s), "
                         f"{t_cpu:.1f} s, single thread"}
        check = bool(np.array_equal(labels.cpu().numpy(), want))
    res["cpu_baseline"] = cpu
    res["labels_match_oracle"] = check
    res["labels"] = labels.cpu().numpy()
    res["graph"] = g
    del rp, col, labels, ws
    torch.cuda.empty_cache()
    return res


def _timed(fn, torch, reps=2):
    """Best wall time (ms) of reps calls after one untimed call; returns (ms, last result)."""
    out = fn()
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, 1000.0 * (time.perf_counter() - t))
    return best, out


def bench_extras(fs, torch, np, c2, c2_labels):
    """The method's other forms on the same inputs: iterations and time of the
    convergence ablation sv1..sv5 (Algorithm 1 plus, in turn, grandparent,
    stochastic and aggressive hooking and early termination), the asynchronous
    mode, and a warm start of C2 after 1% of its edges were added."""
    from paper_1910_05971_amd import graphgen as gg
    dev = torch.device("cuda:0")
    out = {"ablation": {}, "async": {}}
    for name, g in (("C1 er_n65536_m262144", gg.c1_er()), ("C2 rmat_scale24_ef16", c2),
                    ("C3 grid_4096x4096_p0.55", gg.c3_grid())):
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        ws = torch.empty(fs.workspace_bytes(g.n, g.nnz) + 256, dtype=torch.uint8, device=dev)
        row, ref = {}, None
        for vname, flags in fs.SV_FLAGS.items():
            ms, (lab, st) = _timed(lambda: fs.cc_csr(rp, col, workspace=ws, sv_flags=flags), torch)
            lab = lab.cpu().numpy()
            ref = lab if ref is None else ref
            row[vname] = {"iterations": st.iterations, "ms": ms, "labels_equal_sv1": bool(np.array_equal(lab, ref))}
        out["ablation"][name] = row
        ms, (lab, st) = _timed(lambda: fs.cc_csr(rp, col, workspace=ws, mode="async"), torch)
        out["async"][name] = {"passes": st.iterations, "ms": ms, "jacobi_ms": row["sv5"]["ms"],
                              "jacobi_iterations": row["sv5"]["iterations"],
                              "labels_equal_jacobi": bool(np.array_equal(lab.cpu().numpy(), ref))}
        log(f"extras {name}: " + ", ".join(f"{k} {v['iterations']} it {v['ms']:.2f} ms" for k, v in row.items())
            + f"; async {st.iterations} passes {ms:.2f} ms")
        del rp, col, ws
        torch.cuda.empty_cache()
    # warm start: C2 without the last 1% of its edge draws, solved; then the
    # full C2 from those labels, against solving it from scratch
    src, dst = gg.rmat_edges(24, 16, seed=2)
    keep = int(src.shape[0] * 0.99)
    rp99, col99 = gg.csr_from_edges(1 << 24, src[:keep], dst[:keep])
    del src, dst
    rp = torch.from_numpy(rp99).to(dev)
    col = torch.from_numpy(col99).to(dev)
    lab99, _ = fs.cc_csr(rp, col)
    torch.cuda.synchronize()
    del rp, col
    rp = torch.from_numpy(c2.row_ptr).to(dev)
    col = torch.from_numpy(c2.col).to(dev)
    ws = torch.empty(fs.workspace_bytes(c2.n, c2.nnz) + 256, dtype=torch.uint8, device=dev)
    ms_warm, (lab, st_w) = _timed(lambda: fs.cc_csr(rp, col, workspace=ws, f_init=lab99), torch)
    ok = bool(np.array_equal(lab.cpu().numpy(), c2_labels))
    ms_cold, (_, st_c) = _timed(lambda: fs.cc_csr(rp, col, workspace=ws), torch)
    out["warm_start"] = {"workload": "rmat_scale24_ef16 from the labels of its first 99% edge draws",
                         "warm_ms": ms_warm, "warm_iterations": st_w.iterations, "cold_ms": ms_cold,
                         "cold_iterations": st_c.iterations, "labels_equal_cold": ok}
    log(f"extras warm start: {ms_warm:.2f} ms / {st_w.iterations} it vs cold {ms_cold:.2f} ms / {st_c.iterations} it")
    del rp, col, ws, lab99
    torch.cuda.empty_cache()
    return out


def host_info():
    """The host the CPU oracle runs on: CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def oracle_workers():
    """Threads for the oracle's all-core runs: the cores this process may use,
    at most 16 (a one-GPU host's share of cores).  ctypes releases the GIL during each
    oracle call, so threads run the C oracle in parallel."""
    return max(1, min(16, host_info()["usable_cores"]))


def bench_batch(fs, torch, np, tuned=True):
    from paper_1910_05971_amd import graphgen as gg
    t0 = time.time()
    b = gg.c4_batch()
    log(f"batch: {b.num_graphs} graphs, n={b.row_ptr.shape[0] - 1} nnz={b.col.shape[0]} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    vo, eo, rp, col = [torch.from_numpy(np.ascontiguousarray(x)).to(dev)
                       for x in (b.vtx_off, b.edge_off, b.row_ptr, b.col)]
    fs.cc_batch_csr(vo, eo, rp, col, validate=True)
    bkw, tuning = {}, None
    if tuned:
        from paper_1910_05971_amd import tune
        rec = tune.tune_batch(vo, eo, rp, col, reps=1, save=False)
        bkw = dict(rec["best"]["opts"])
        tuning = {"best_opts": bkw, "best_ms": rec["best"]["ms"], "default_ms": rec["default"]["ms"]}
        log(f"batch tuned {bkw}: {rec['best']['ms']:.2f} ms vs default {rec['default']['ms']:.2f} ms")
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        labels, iters, st = fs.cc_batch_csr(vo, eo, rp, col, **bkw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    t_batch = sorted(times)[1]
    gpu_labels, gpu_iters = labels.cpu().numpy(), iters.cpu().numpy()
    # plain: one cc_csr call per graph on device-resident sub-CSRs
    subs = []
    for gi in range(b.num_graphs):
        s = b.graph(gi)
        subs.append((torch.from_numpy(np.ascontiguousarray(s.row_ptr)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(s.col)).to(dev)))
    for r, c in subs[:64]:
        fs.cc_csr(r, c)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r, c in subs:
        fs.cc_csr(r, c)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    del subs, vo, eo, rp, col, labels, iters
    torch.cuda.empty_cache()
    # the whole batch against HBM: the library's algorithmic bytes over the
    # union graph's executed iterations (dense or sparse passes and
    # grandparent passes, as for one solve) per batch time
    alg = int(st.alg_bytes)
    batch_roofline = {"alg_bytes": alg, "ms": 1000 * t_batch, "achieved": alg / t_batch / 1e9, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": alg / t_batch / 1e9 / HBM_PEAK_GBS,
                      "dense_iterations": int(st.dense_iterations), "sparse_iterations": int(st.sparse_iterations)}
    out = {"workload": "4096 Erdos-Renyi graphs, n log-uniform in [64, 65536), average degree uniform in [2, 32]",
           "graphs": b.num_graphs, "total_edges_undirected": int(b.m_eff.sum()),
           "graphs_per_s": b.num_graphs / t_batch, "ms_per_batch": 1000 * t_batch,
           "iterations": st.iterations, "plain_graphs_per_s": b.num_graphs / t_plain,
           "speedup_vs_plain": t_plain / t_batch, "tuning": tuning, "solve_roofline": batch_roofline}
    return out, (b, gpu_labels, gpu_iters)


def batch_oracle(np, b, gpu_labels, gpu_iters):
    """CPU-baseline leg of the batch: union-find over all graphs on one core and
    on all usable cores, and Algorithm 2 on all cores; each graph's batched
    labels and iteration count are compared with them (outside any timed GPU
    region)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    G = b.num_graphs
    graphs = [b.graph(i) for i in range(G)]
    t = time.perf_counter()
    uf = [oracle.uf_labels(g.n, g.row_ptr, g.col) for g in graphs]
    t_uf1 = time.perf_counter() - t
    W = oracle_workers()
    with ThreadPoolExecutor(W) as ex:
        t = time.perf_counter()
        list(ex.map(lambda g: oracle.uf_labels(g.n, g.row_ptr, g.col), graphs))
        t_ufw = time.perf_counter() - t
        t = time.perf_counter()
        its = list(ex.map(lambda g: oracle.fastsv_alg2(g.n, g.row_ptr, g.col).iterations, graphs))
        t_a2w = time.perf_counter() - t
    lab_ok = all(np.array_equal(gpu_labels[b.vtx_off[i]:b.vtx_off[i + 1]], uf[i]) for i in range(G))
    it_ok = bool(np.array_equal(np.asarray(its), gpu_iters[:G]))
    return {"labels_match_oracle": bool(lab_ok), "iterations_match_oracle": it_ok,
            "cpu_oracle": {"union_find_1core_graphs_per_s": G / t_uf1,
                           "union_find_all_cores_graphs_per_s": G / t_ufw,
                           "alg2_all_cores_graphs_per_s": G / t_a2w, "cores": W,
                           "sample": f"all {G} graphs of the batch"}}


def bench_serve(args, torch, np, want_check):
    from paper_1910_05971_amd import graphgen as gg, serving
    t0 = time.time()
    tr = gg.request_trace(args.serve_requests, args.serve_rate, er_pool=args.serve_er_pool,
                          rmat_pool=args.serve_rmat_pool)
    graphs = serving.pin_graphs(tr.graphs)
    measured = tr.arrivals >= args.serve_warmup
    nmeas = int(measured.sum())
    log(f"serving trace: {len(graphs)} requests ({int(tr.kinds.sum())} R-MAT scale 20), {nmeas} after the "
        f"{args.serve_warmup:g} s warm-up, in {time.time() - t0:.1f}s")
    out = {"workload": f"Poisson {args.serve_rate:.0f} req/s, {len(graphs)} requests ({nmeas} measured after a "
                       f"{args.serve_warmup:g} s warm-up): 99% Erdos-Renyi from the batch distribution (pool of "
                       f"{args.serve_er_pool} graphs), 1% R-MAT scale 20 edge factor 16 (pool of "
                       f"{args.serve_rmat_pool}); host-resident page-locked CSRs",
           "requests": len(graphs), "measured_requests": nmeas, "rmat_requests": int(tr.kinds.sum())}

    def pct(lat):
        return float(np.percentile(lat, 50) * 1e3), float(np.percentile(lat, 99) * 1e3)

    pool = (16_000_000, 320_000_000, 2048)  # the trace's working set: about 1.3 GB of CSR and labels state
    admit = None
    if not args.no_tune:
        from paper_1910_05971_amd import tune
        rec = tune.tune_server(graphs[:2000], pool, save=False)
        admit = rec["best"]["opts"]["admit_mb"]
        out["tuning"] = {"best_opts": rec["best"]["opts"], "results": rec["results"],
                         "sample": "the trace's first 2000 requests submitted at once"}
        log(f"serving tuned admission: {admit} MB per step")

    def server():
        return serving.Server(*pool, validate=False, admit_mb=admit)

    # warm both paths
    srv = server()
    serving.run_open_loop(srv, graphs[:64], np.zeros(64), mapped=True)
    srv.close()
    serving.run_plain(graphs[:64], np.zeros(64))

    def settled():
        # the host loops of both paths run in Python: collect once and freeze
        # what exists, so that no full collection lands inside a timed run
        gc.collect()
        gc.freeze()

    results = {}
    for mode, arr in (("open_loop", tr.arrivals), ("saturation", np.zeros_like(tr.arrivals))):
        got = {}
        for path in ("server", "plain"):
            done = [None] * len(graphs)

            def keep(i, lab, its, done=done):
                done[i] = (lab, its)  # kept by reference; compared after the run
            settled()
            if path == "server":
                srv = server()
                lat, span, _ = serving.run_open_loop(srv, graphs, arr, on_done=keep, mapped=True)
                steps = int(srv.stats().steps)
                srv.close()
            else:
                lat, span, _ = serving.run_plain(graphs, arr, on_done=keep)
            gc.unfreeze()
            if mode == "open_loop":
                # steady state: requests arriving after the warm-up, over the
                # time from the first of them to the last completion
                sel = measured
                t_first = float(tr.arrivals[measured].min())
                rate = nmeas / (span - t_first)
            else:
                sel = np.ones(len(graphs), dtype=bool)
                rate = len(graphs) / span
            p50, p99 = pct(lat[sel])
            got[path] = {"graphs_per_s": rate, "p50_ms": p50, "p99_ms": p99}
            if path == "server":
                got[path]["steps"] = steps
            results[(mode, path)] = done
        got["throughput_ratio"] = got["server"]["graphs_per_s"] / got["plain"]["graphs_per_s"]
        out[mode] = got
        log(f"serving {mode}: server {got['server']['graphs_per_s']:.0f} graphs/s p50 {got['server']['p50_ms']:.2f}"
            f" p99 {got['server']['p99_ms']:.2f} ms; plain {got['plain']['graphs_per_s']:.0f} graphs/s p50 "
            f"{got['plain']['p50_ms']:.2f} p99 {got['plain']['p99_ms']:.2f} ms")
    if want_check:
        out.update(serve_oracle(np, graphs, tr.arrivals, measured, results))
    return out


def serve_oracle(np, graphs, arrivals, measured, results):
    """CPU-baseline leg of serving: union-find and Algorithm 2 once per
    distinct request graph (the trace draws from pools), union-find's solve
    time per request as a latency distribution, and every served request's
    labels and iteration count (server and plain, open loop and saturation)
    against them."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    uniq = {}
    for g in graphs:
        uniq.setdefault(id(g), g)
    pool = list(uniq.values())
    uf_t = {}
    for g in pool:  # one core, one graph at a time: the per-request solve time
        t = time.perf_counter()
        oracle.uf_labels(g.n, g.row_ptr, g.col)
        uf_t[id(g)] = time.perf_counter() - t
    with ThreadPoolExecutor(oracle_workers()) as ex:
        ufl = dict(zip([id(g) for g in pool], ex.map(lambda g: oracle.uf_labels(g.n, g.row_ptr, g.col), pool)))
        its = dict(zip([id(g) for g in pool], ex.map(lambda g: oracle.fastsv_alg2(g.n, g.row_ptr, g.col).iterations,
                                                      pool)))
    bad = {}
    for key, done in results.items():
        nbad = 0
        for i, g in enumerate(graphs):
            lab, it = done[i]
            if it != its[id(g)] or not np.array_equal(lab, ufl[id(g)]):
                nbad += 1
        bad["/".join(key)] = nbad
    lat = np.array([uf_t[id(g)] for g, m in zip(graphs, measured) if m])
    return {"labels_match_oracle": all(v == 0 for v in bad.values()),
            "mismatched_requests": bad,
            "cpu_oracle": {"union_find_p50_ms": float(np.percentile(lat, 50) * 1e3),
                           "union_find_p99_ms": float(np.percentile(lat, 99) * 1e3), "cores": 1,
                           "sample": f"union-find solve time of each measured request's graph "
                                     f"({len(pool)} distinct graphs), one core"}}


def cpu_oracle_table(np, c2, c2_iters):
    """Oracle timings on C1..C3, one core: union-find (edges/s) and Algorithm 2
    (time and iteration count; the GPU's count is given beside it)."""
    import oracle
    from paper_1910_05971_amd import graphgen as gg
    rows = {}
    for name, g in (("er_n65536_m262144", gg.c1_er()), ("rmat_scale24_ef16", c2),
                    ("grid_4096x4096_p0.55", gg.c3_grid())):
        t = time.perf_counter()
        oracle.uf_labels(g.n, g.row_ptr, g.col)
        t_uf = time.perf_counter() - t
        t = time.perf_counter()
        r = oracle.fastsv_alg2(g.n, g.row_ptr, g.col)
        t_a2 = time.perf_counter() - t
        rows[name] = {"union_find_ms": 1e3 * t_uf, "union_find_edges_per_s": g.m_eff / t_uf,
                      "alg2_ms": 1e3 * t_a2, "alg2_edges_per_s": g.m_eff / t_a2, "alg2_iterations": r.iterations}
        if name == "rmat_scale24_ef16":
            rows[name]["gpu_iterations"] = c2_iters
        log(f"cpu oracle {name}: union-find {1e3 * t_uf:.0f} ms, Algorithm 2 {1e3 * t_a2:.0f} ms "
            f"({r.iterations} iterations)")
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_1910_05971_amd as fs

    res = bench_solve(args, fs, torch, np)
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "undirected edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": res["config"],
        "tuning": res["tuning"],
        "roofline": res["roofline"],
        "roofline_other": res["roofline_other"],
        "solve_roofline": res["solve_roofline"],
        "breakdown_ms_per_solve": res["breakdown_ms_per_solve"],
        "iterations_detail": res["iterations_detail"],
        "labels_match_oracle": res["labels_match_oracle"],
    }
    if res["cpu_baseline"]:
        out["cpu_baseline"] = res["cpu_baseline"]
    if not args.no_extras and args.workload == "rmat24":
        out["extras"] = bench_extras(fs, torch, np, res["graph"], res["labels"])
    batch_gpu = None
    if not args.no_batch:
        out["batched"], batch_gpu = bench_batch(fs, torch, np, tuned=not args.no_tune)
    if not args.no_serve:
        out["serving"] = bench_serve(args, torch, np, want_check=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        # the rest of the oracle's baseline (outside every timed GPU region)
        out["cpu_host"] = host_info()
        if batch_gpu is not None:
            log("cpu oracle over the batch (one core and all cores)")
            out["batched"].update(batch_oracle(np, *batch_gpu))
        if args.workload == "rmat24":
            out["cpu_oracle_table"] = cpu_oracle_table(np, res["graph"], out["config"]["iterations"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

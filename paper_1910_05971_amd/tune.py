"""Autotuner for the run-time choices that leave the iterates unchanged.

The solver's result and trajectory do not depend on the sparse-frontier
threshold (Sec. 4.2 leaves its value open), on the bin width of the binned
layout or on the span of its dense pass; only the time does.  ``tune_csr``
times ``fastsv_cc_csr`` over a grid of these options for one graph on one
device, ``tune_batch`` does the same for the batched entry's threshold and
``tune_server`` for the server's per-step admission size, and the fastest
choice is stored in a JSON cache keyed by device and graph-size class
(``log2`` of the vertex and entry counts).  ``binding.cc_csr(..., tuned=True)``
and the benchmark read the cache back with ``lookup``.

The cache lives at ``$FASTSV_TUNING_CACHE`` or ``~/.cache/fastsv/tuning.json``.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import binding as B

TAUS = (0.01, 0.02, 0.05, 0.1, 0.2)
# (bin_shift, bin_span): automatic width with each span, and two fixed widths
BIN_CHOICES = ((0, 0), (0, 8), (0, 16), (0, 32), (14, 0), (15, 0))
ADMIT_MB = (32, 64, 128, 256)
BINNED_MIN_N = 1 << 22  # the automatic layout choice (binned above this many vertices)


def cache_path(path: str | None = None) -> str:
    if path:
        return path
    return os.environ.get("FASTSV_TUNING_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "fastsv",
                                                                  "tuning.json")


def device_key(device: int) -> str:
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "") or ""
    return f"{p.name}|{arch}|{p.multi_processor_count}cu"


def size_class(n: int, nnz: int) -> str:
    lg = lambda x: int(math.ceil(math.log2(max(int(x), 1))))
    return f"n2^{lg(n)}_e2^{lg(nnz)}"


def csr_candidates(n: int, nnz: int, all_bins: bool = False) -> list[dict]:
    """Options to try: every threshold, and the bin choices where the binned
    layout is built (or all of them with ``all_bins``)."""
    bins = BIN_CHOICES if (all_bins or n > BINNED_MIN_N) else ((0, 0),)
    out = []
    for tau in TAUS:
        for shift, span in bins:
            out.append({"frontier_tau": tau, "bin_shift": shift, "bin_span": span})
    return out


def _time_call(fn, reps: int) -> float:
    fn()  # warm-up (workspace, caches)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, 1e3 * (time.perf_counter() - t))
    return best


def load(path: str | None = None) -> dict:
    p = cache_path(path)
    if not os.path.exists(p):
        return {}
    try:
        with open(p) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def store(kind: str, device: str, cls: str, record: dict, path: str | None = None) -> None:
    p = cache_path(path)
    db = load(p)
    db.setdefault(device, {}).setdefault(kind, {})[cls] = record
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(device: int, n: int, nnz: int, kind: str = "csr", path: str | None = None) -> dict:
    """The stored best options for this device and size class, else {}."""
    if not torch.cuda.is_available():
        return {}
    rec = load(path).get(device_key(device), {}).get(kind, {}).get(size_class(n, nnz))
    return dict(rec["best"]["opts"]) if rec else {}


def tune_csr(row_ptr: torch.Tensor, col: torch.Tensor, reps: int = 3, save: bool = True,
             path: str | None = None, candidates: list[dict] | None = None) -> dict:
    """Time every candidate on this graph; returns {"default", "best",
    "results"} (milliseconds per solve) and stores it unless save=False."""
    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col.numel()
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n]
    cands = candidates if candidates is not None else csr_candidates(n, nnz)
    ws = torch.empty(max(B.workspace_bytes(n, nnz, B.make_opts(**c)) for c in cands) + 256, dtype=torch.uint8,
                     device=dev)
    results = []
    for c in cands:
        ms = _time_call(lambda: B.cc_csr(row_ptr, col, labels=labels, workspace=ws, **c), reps)
        results.append({"opts": c, "ms": ms})
    d = B.default_opts()
    default = {"frontier_tau": round(float(d.frontier_tau), 6), "bin_shift": 0, "bin_span": 0}
    dms = _time_call(lambda: B.cc_csr(row_ptr, col, labels=labels, workspace=ws), reps)
    best = min(results, key=lambda r: r["ms"])
    rec = {"n": n, "nnz": nnz, "default": {"opts": default, "ms": dms}, "best": best, "results": results}
    if save:
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        store("csr", device_key(idx), size_class(n, nnz), rec, path)
    return rec


def tune_batch(vtx_off, edge_off, row_ptr, col, reps: int = 2, save: bool = True, path: str | None = None) -> dict:
    """The batched entry's frontier threshold."""
    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col.numel()
    results = []
    for tau in TAUS:
        ms = _time_call(lambda: B.cc_batch_csr(vtx_off, edge_off, row_ptr, col, frontier_tau=tau), reps)
        results.append({"opts": {"frontier_tau": tau}, "ms": ms})
    dms = _time_call(lambda: B.cc_batch_csr(vtx_off, edge_off, row_ptr, col), reps)
    best = min(results, key=lambda r: r["ms"])
    rec = {"n": n, "nnz": nnz, "graphs": vtx_off.numel() - 1,
           "default": {"opts": {"frontier_tau": round(float(B.default_opts().frontier_tau), 6)}, "ms": dms},
           "best": best, "results": results}
    if save:
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        store("batch", device_key(idx), size_class(n, nnz), rec, path)
    return rec


def tune_server(graphs, pool: tuple[int, int, int], device: int = 0, save: bool = True,
                path: str | None = None) -> dict:
    """The server's per-step admission size, on all of ``graphs`` submitted at
    once (saturation); graphs/s per candidate."""
    from . import serving
    results = []
    for mb in ADMIT_MB:
        srv = serving.Server(*pool, device=device, validate=False, admit_mb=mb)
        t = time.perf_counter()
        srv.submit_many(graphs, mapped=True)
        left = len(graphs)
        while left:
            srv.step()
            left -= len(srv.poll())
        dt = time.perf_counter() - t
        srv.close()
        results.append({"opts": {"admit_mb": mb}, "graphs_per_s": len(graphs) / dt})
    best = max(results, key=lambda r: r["graphs_per_s"])
    rec = {"requests": len(graphs), "pool": list(pool), "default": {"opts": {"admit_mb": 128}},
           "best": best, "results": results}
    if save:
        store("server", device_key(device), f"pool_{pool[0]}_{pool[1]}_{pool[2]}", rec, path)
    return rec

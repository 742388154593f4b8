"""Writes alg2_counts.json: Algorithm 2's iteration count and per-iteration
changed-grandparent counts on the full-size seeded workloads (ER n=65,536;
R-MAT scale 24 edge factor 16; the 4096x4096 percolated grid), plus each
graph's size and component count.  Calls only the CPU oracle and the seeded
generators; the R-MAT run takes about half a minute on one core.

    python tests/golden/configs/make_alg2_counts.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1910_05971_amd import graphgen as gg  # noqa: E402


def main():
    out = {"source": "oracle_fastsv_alg2 and oracle_uf_labels on the seeded workloads (this script)"}
    for key, make in (("er_n65536_m262144", gg.c1_er), ("rmat_scale24_ef16", gg.c2_rmat),
                      ("grid_4096x4096_p0.55", gg.c3_grid)):
        t = time.time()
        g = make()
        r = O.fastsv_alg2(g.n, g.row_ptr, g.col, trace_cap=64, record_f=False)
        lab = O.uf_labels(g.n, g.row_ptr, g.col)
        out[key] = {"n": int(g.n), "nnz": int(g.nnz), "iterations": int(r.iterations),
                    "changed": [int(c) for c in r.changed], "components": int(np.count_nonzero(lab == np.arange(g.n)))}
        print(key, out[key], f"{time.time() - t:.1f}s", flush=True)
    with open(os.path.join(HERE, "alg2_counts.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()

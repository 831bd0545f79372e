"""Write the oracle's reference values for the LFR-style n = 2e7 workload.

Test infrastructure: this script calls only the seeded input generator
(``rsgen``) and the CPU oracle (``oracle``).  It scores every vertex of the
graph with the oracle (a full pass takes tens of minutes on a few cores) and
stores what a GPU test at that size compares against:

* the graph's fingerprint (sizes and SHA-256 of the CSR and labels), so a
  test can tell that it regenerated the same graph;
* the oracle's totals (w_max, border count, inter-community edges, sums of
  tI and tII) and SHA-256 digests of its per-vertex integer arrays (border,
  ell, d', tI, tII) and of the zero pattern of R;
* the oracle's top-(K + 256) list (ids and scores), K = 10,000, in the order
  of Algorithm 1 Step 4 (R descending, id ascending);
* the oracle's R on a seeded random sample of 100,000 vertices and on the
  1,000 vertices of highest degree (ids recomputed by the test from
  ``sample_ids``; only the scores are stored).

Run from the repository root:
    RS_GRAPH_CACHE=/tmp/rscache python tests/golden/make_lfr20m_golden.py [nthreads]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from rsgen import cached, cfg_lfr_20m  # noqa: E402

K = 10_000
EXTRA = 256
N_SAMPLE = 100_000
N_HUBS = 1_000


def sample_ids(g):
    """The sampled vertices: 100,000 drawn with a fixed seed, then the 1,000
    of highest degree (ties by id), in that order (ids may repeat)."""
    rng = np.random.default_rng(2024)
    rand = np.sort(rng.choice(g.n, N_SAMPLE, replace=False))
    deg = np.diff(np.asarray(g.off, dtype=np.int64))
    hubs = np.argsort(-deg, kind="stable")[:N_HUBS]
    return np.concatenate([rand, hubs]).astype(np.int64)
OUT_JSON = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lfr_20m_oracle.json")
OUT_NPZ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lfr_20m_oracle_topk.npz")


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def fingerprint(g):
    return {"n": int(g.n), "m": int(g.m), "nnz": int(g.nnz),
            "off_sha256": sha(g.off, np.int64), "col_sha256": sha(g.col, np.int32),
            "labels_sha256": sha(g.labels, np.int32)}


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    t0 = time.time()
    g = cached("lfr_20m_seed0", lambda: cfg_lfr_20m(0, log=print), log=print)
    print(f"graph n={g.n} m={g.m} in {time.time() - t0:.0f}s", flush=True)
    oracle.build()
    t0 = time.time()
    o = oracle.score(g, nthreads=nthreads)
    t_score = time.time() - t0
    print(f"oracle pass {t_score:.0f}s", flush=True)
    ids, sc = oracle.topk(o["R"], K + EXTRA)
    out = {
        "what": "oracle reference values for the LFR-style n=2e7 workload (seed 0); written by "
                "tests/golden/make_lfr20m_golden.py from the CPU oracle only",
        "graph": fingerprint(g),
        "k": K,
        "omega_max_hex": float(o["omega_max"]).hex(),
        "n_border": int(o["n_border"]), "m_inter": int(o["m_inter"]),
        "sum_tI": int(o["tI"].sum()), "sum_tII": int(o["tII"].sum()),
        "sha256": {"border": sha(o["border"], np.uint8), "ell": sha(o["ell"], np.int32),
                   "dprime": sha(o["dprime"], np.int32), "tI": sha(o["tI"], np.int64),
                   "tII": sha(o["tII"], np.int64), "R_zero": sha(o["R"] == 0, np.uint8)},
        "oracle_seconds": round(t_score, 1), "oracle_threads": nthreads,
    }
    with open(OUT_JSON, "w") as f:
        json.dump(out, f, indent=1)
    np.savez_compressed(OUT_NPZ, ids=ids.astype(np.int32), scores=sc.astype(np.float64),
                        sample_R=o["R"][sample_ids(g)].astype(np.float64))
    print("wrote", OUT_JSON, OUT_NPZ, flush=True)


if __name__ == "__main__":
    main()

"""Writes the CPU oracle's ICP results for the full-size workloads, with
SHA-256 digests of the exact inputs the oracle saw:

  icp_workloads.json  the depth-camera room (307,200 points) and the LiDAR
                      street (2,097,152 points);
  icp_batch256.json   every pair of the 256 uneven pairs (11.98 M points per
                      side): pose, status, iterations, inliers and rms.

Each result is the oracle end to end: its own kd-tree normals of the target
(rounded to float32), then point-to-plane ICP from the identity with the
float32 rejection distance and the fixed iteration count.

Only oracle/ and the seeded generators are used.  Run from the repo root:
    python tests/golden/make_icp_golden.py [single|batch]
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
from gen import batch_workload, make_workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_SINGLE = os.path.join(HERE, "icp_workloads.json")
OUT_BATCH = os.path.join(HERE, "icp_batch256.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def oracle_pair(w):
    nrm, _, _ = oracle.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
    nrm = nrm.astype(np.float32)
    dmax = float(np.float32(w.d_max))
    r = oracle.icp(w.source, w.target, nrm, None, dmax, w.iters, 0.0, method="kdtree")
    return nrm, dmax, r


def single():
    res = {}
    for cfg in (1, 2):
        w = make_workload(cfg)
        t0 = time.time()
        nrm, dmax, r = oracle_pair(w)
        res[w.name] = dict(
            config=cfg, k=w.k, d_max_f32=dmax, iters=w.iters,
            sha256_source=digest(w.source), sha256_target=digest(w.target), sha256_normals=digest(nrm),
            T=[float(v) for v in r["T"].reshape(-1)], status=r["status"], iterations=r["iterations"],
            inliers=r["inliers"], rms=r["rms"], oracle_seconds=round(time.time() - t0, 1),
            oracle_threads=oracle.num_threads())
        print(w.name, res[w.name]["oracle_seconds"], "s", flush=True)
    with open(OUT_SINGLE, "w") as f:
        json.dump(res, f, indent=1)


def batch():
    b = batch_workload(3)
    t0 = time.time()
    pairs = []
    for j, w in enumerate(b.pairs):
        _, dmax, r = oracle_pair(w)
        pairs.append(dict(name=w.name, n=w.n, k=w.k, d_max_f32=dmax, iters=w.iters,
                          T=[float(v) for v in r["T"].reshape(-1)], status=int(r["status"]),
                          iterations=int(r["iterations"]), inliers=int(r["inliers"]), rms=float(r["rms"])))
    el = time.time() - t0
    res = dict(workload=b.name, n_pairs=b.n_pairs, points_per_side=b.n,
               sha256_source=digest(b.source), sha256_target=digest(b.target), sha256_offsets=digest(b.offsets),
               oracle_seconds=round(el, 1), oracle_threads=oracle.num_threads(), pairs=pairs)
    print(b.name, round(el, 1), "s", flush=True)
    with open(OUT_BATCH, "w") as f:
        # one pair per line keeps the file short and diffable
        f.write("{\n")
        for key in ("workload", "n_pairs", "points_per_side", "sha256_source", "sha256_target",
                    "sha256_offsets", "oracle_seconds", "oracle_threads"):
            f.write(f" {json.dumps(key)}: {json.dumps(res[key])},\n")
        f.write(' "pairs": [\n')
        f.write(",\n".join("  " + json.dumps(p) for p in pairs))
        f.write("\n ]\n}\n")


def main():
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    oracle.build(force=False)
    if what in ("all", "single"):
        single()
    if what in ("all", "batch"):
        batch()


if __name__ == "__main__":
    main()

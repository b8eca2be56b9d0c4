"""Writes icp_workloads.json: the CPU oracle's ICP result on the full-size
depth-camera room (307,200 points) and LiDAR street (2,097,152 points)
workloads, with SHA-256 digests of the exact inputs it saw.

Only oracle/ and the seeded generators are used.  Run from the repo root:
    python tests/golden/make_icp_golden.py
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
from gen import make_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "icp_workloads.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    res = {}
    for cfg in (1, 2):
        w = make_workload(cfg)
        t0 = time.time()
        nrm, _, _ = oracle.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
        nrm = nrm.astype(np.float32)
        dmax = float(np.float32(w.d_max))
        r = oracle.icp(w.source, w.target, nrm, None, dmax, w.iters, 0.0, method="kdtree")
        res[w.name] = dict(
            config=cfg, k=w.k, d_max_f32=dmax, iters=w.iters,
            sha256_source=digest(w.source), sha256_target=digest(w.target), sha256_normals=digest(nrm),
            T=[float(v) for v in r["T"].reshape(-1)], status=r["status"], iterations=r["iterations"],
            inliers=r["inliers"], rms=r["rms"], oracle_seconds=round(time.time() - t0, 1),
            oracle_threads=oracle.num_threads())
        print(w.name, res[w.name]["oracle_seconds"], "s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()

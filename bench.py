"""Benchmark of the point-to-plane ICP hot path on one MI355X.

Default workload (the largest configuration): 256 pairs of uneven sizes
(5k-200k points each, 11.98 M points per side).  One step = the targets'
pyramid, the PCA normals of every target and the point-to-plane ICP of every
pair (the fixed iteration loops and the final statistics passes) in one
batched call over one pyramid; the call launches kernels only and the timed
steps replay it captured as a graph.  The per-pair poses of the timed run
are compared with the oracle's stored results (tests/golden/), and the
single-pair LiDAR street (2,097,152 points) is timed the same way and
reported under "street"; a summary of the learned-initialiser workload is
appended.

    python bench.py [--steps K] [--warmup W] [--workload batch|room|street|sphere|projective|learned]

A single-pair workload's step is one pair through the same path
(icp_point_to_plane_with_normals, one target pyramid for normals and ICP).
Inputs are resident in HBM before the timed region; the timed region is
bracketed by device synchronisation.

Prints one JSON line.  value = pairs/s; the loop-only Mpt*iter/s, the
roofline of the dominant kernel (the per-iteration correspondence +
accumulation kernel, timed with HIP events on the library's stream), the
pose check against the oracle and a CPU-oracle baseline (with the host CPU
model) are reported alongside.  The learned workload registers 512
exact-copy pairs from four starts (plain, 8-start, learned with 8-start
fallback, learned only).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ICP pairs/s + Mpt·iter/s at ≤1e-5 rad pose error; learned-init vs plain"
WORKLOADS = {"sphere": 0, "room": 1, "street": 2, "batch": 3, "projective": 5, "learned": 4, "knn": 6, "normals": 7}
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per source point per ICP iteration: source xyz (12),
# matched target xyz + normal (24), cell lookup (4); the projective
# association reads the pixel's point and normal directly (no cell lookup)
ICP_BYTES_PER_POINT = 40
# k-NN: the query's xyz read, k (index, key) pairs written; normals: xyz
# read, normal and curvature written (neighbours come from the pyramid)
KNN_BYTES_PER_QUERY = lambda k: 12 + 8 * k
NORMALS_BYTES_PER_POINT = 28
PROJ_BYTES_PER_POINT = 36
PROJECTIVE = dict(name="room_views_vga", width=640, height=480, angle=3.0, t=0.03, k=16, d_max=0.2, iters=15)
# matrix-core work of the learned initialiser's encoder per point: the
# 64 -> 128 and 128 -> 256 layers, 2 flops per multiply-add
ENC_FLOPS_PER_POINT = 2 * (64 * 128 + 128 * 256)
BF16_PEAK_TFLOPS = 2500.0
PROFILES = os.path.join(ROOT, "profiles")
TUNING_CACHE = os.path.join(ROOT, "paper_1807_00399_amd", "tuning_cache.json")


def autotune_step(args, step, tag, n_points):
    """Sets the tuning for this workload (cached choice, or timed now)."""
    from paper_1807_00399_amd import autotune, pcgpu
    if args.no_autotune:
        return {"tuning": pcgpu.get_tuning(), "source": "default"}
    r = autotune.tune(step, tag, n_points, cache_file=TUNING_CACHE, use_cache=not args.retune)
    if not r["from_cache"]:
        # record the timings where a GPU run keeps its outputs
        out = os.path.join(ROOT, "gpurun_out")
        if os.path.isdir(out):
            with open(os.path.join(out, f"tuning_{tag}.json"), "w") as f:
                json.dump({autotune.cache_key(autotune._device_name(None), tag, n_points): r}, f, indent=1)
    return {"tuning": r["tuning"], "source": "cache" if r["from_cache"] else "timed"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tuning instead of the autotuner's choice")
    ap.add_argument("--retune", action="store_true",
                    help="time every tuning candidate even when the tuning cache has this workload")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch workload: skip the one-call-per-pair comparison")
    ap.add_argument("--no-graph", action="store_true",
                    help="single-pair and batch workloads: time eager launches instead of replays of a captured graph")
    ap.add_argument("--no-learned", action="store_true",
                    help="default run: skip the learned-initialiser comparison")
    ap.add_argument("--cloud", choices=["room", "street"], default="room",
                    help="knn and normals workloads: the cloud queried against itself")
    ap.add_argument("--no-street", action="store_true",
                    help="default run: skip the single-pair street line reported beside the batch")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 1 GiB device copy (bandwidth and counter calibration) and exit")
    return ap.parse_args()


GOLDEN = os.path.join(ROOT, "tests", "golden")
POSE_TOL_RAD, POSE_TOL_T = 1e-5, 1e-6


def cpu_model():
    """The host CPU's model name and logical CPU count (lscpu)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except Exception:
        return None
    info = {}
    for line in out.splitlines():
        key, _, val = line.partition(":")
        if key.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)"):
            info[key.strip()] = val.strip()
    return info or None


def _sha256(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def pose_errors(Ta, Tb):
    """Rotation angle of Ra Rb^T (atan2 form, no acos near 1) and the
    translation distance, for stacks of 4x4 poses."""
    Ta = np.asarray(Ta, np.float64).reshape(-1, 4, 4)
    Tb = np.asarray(Tb, np.float64).reshape(-1, 4, 4)
    M = Ta[:, :3, :3] @ np.transpose(Tb[:, :3, :3], (0, 2, 1))
    v = np.stack([M[:, 2, 1] - M[:, 1, 2], M[:, 0, 2] - M[:, 2, 0], M[:, 1, 0] - M[:, 0, 1]], axis=1)
    rot = np.arctan2(0.5 * np.linalg.norm(v, axis=1), 0.5 * (np.trace(M, axis1=1, axis2=2) - 1.0))
    tr = np.linalg.norm(Ta[:, :3, 3] - Tb[:, :3, 3], axis=1)
    return rot, tr


def pose_check(T_gpu, T_ref, inl_gpu=None, inl_ref=None, source=""):
    """The timed poses against the oracle's: worst errors and the number of
    pairs within the pose tolerance."""
    rot, tr = pose_errors(T_gpu, T_ref)
    ok = (rot <= POSE_TOL_RAD) & (tr <= POSE_TOL_T)
    d = {"oracle": source, "pairs": int(rot.size), "within_tol": int(ok.sum()),
         "tol": {"rad": POSE_TOL_RAD, "translation": POSE_TOL_T},
         "max_rot_rad": float(rot.max()), "max_trans": float(tr.max())}
    if inl_gpu is not None:
        d["inliers_equal"] = int(np.sum(np.asarray(inl_gpu) == np.asarray(inl_ref)))
    return d


def batch_golden(b):
    """The oracle's per-pair results for this batch (stored by
    tests/golden/make_icp_golden.py), if the inputs are the ones it saw."""
    path = os.path.join(GOLDEN, "icp_batch256.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    if (g.get("n_pairs") != b.n_pairs or g.get("sha256_source") != _sha256(b.source)
            or g.get("sha256_target") != _sha256(b.target) or g.get("sha256_offsets") != _sha256(b.offsets)):
        return None
    return g


def single_golden(w):
    path = os.path.join(GOLDEN, "icp_workloads.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path)).get(w.name)
    if g is None or g["sha256_source"] != _sha256(w.source) or g["sha256_target"] != _sha256(w.target):
        return None
    return g


class HipEvents:
    """Timing events from the HIP runtime, recorded by the library on the
    stream its kernels run on."""

    def __init__(self, n):
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.c_void_p]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.n = n
        self.beg = (ctypes.c_void_p * n)()
        self.end = (ctypes.c_void_p * n)()
        for i in range(n):
            assert self.rt.hipEventCreate(ctypes.byref(self.beg, i * ctypes.sizeof(ctypes.c_void_p))) == 0
            assert self.rt.hipEventCreate(ctypes.byref(self.end, i * ctypes.sizeof(ctypes.c_void_p))) == 0

    def elapsed_ms(self, i):
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), self.beg[i], self.end[i]) == 0
        return ms.value

    def span_ms(self, i, j):
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), self.beg[i], self.end[j]) == 0
        return ms.value


KERNEL_SOURCES = {"icp_accum": ("icp.hip", "search.h", "common.h"),
                  "k_knn": ("knn.hip", "search.h", "common.h"),
                  "k_normals": ("knn.hip", "search.h", "common.h")}


def kernel_tag_of(regex):
    """Which kernel a rocprofv3 kernel regex names (for its source digest)."""
    return "k_knn" if "knn" in regex else "k_normals" if "normals" in regex else "icp_accum"


def kernel_digest(kernel_tag="icp_accum"):
    """Digest of the sources a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel_tag]:
        h.update(open(os.path.join(ROOT, "paper_1807_00399_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary for
    this kernel and workload, provided the kernel sources have not changed
    since the counters were taken (else None)."""
    path = os.path.join(PROFILES, f"{kernel_tag}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_digest") != kernel_digest(kernel_tag if kernel_tag in KERNEL_SOURCES else "icp_accum"):
        return None
    return d.get("hbm_bytes_per_launch")


def valu_from_profiles(workload):
    """Share of the nominal vector-issue capacity the accumulate kernel used
    (time-weighted over its launches), from the committed rocprofv3 SQ
    counter summary, provided the kernel sources have not changed since."""
    path = os.path.join(PROFILES, f"icp_accum_{workload}_valu.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_digest") != kernel_digest():
        return None
    return d.get("valu_issue_share_nominal_time_weighted")


def copy_probe():
    """Plain device copy of 1 GiB, 10 times: achievable bandwidth, and a
    kernel of known traffic for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    from paper_1807_00399_amd import pcgpu
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    pcgpu.copy_probe(b, a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        pcgpu.copy_probe(b, a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gbs = 2 * nbytes * reps / el / 1e9
    print(json.dumps({"copy_probe": {"bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                                     "launches": reps + 1, "achieved_GBps": gbs, "peak_GBps": HBM_PEAK_GBS}}),
          flush=True)


def cpu_baseline(w, budget_s):
    """The CPU oracle on the same pair: kd-tree normals + ICP (OpenMP over
    points), repeated until about budget_s seconds have passed."""
    import oracle
    oracle.build(force=False)
    d32 = float(np.float32(w.d_max))
    t0 = time.perf_counter()
    pairs, loop_s = 0, 0.0
    while True:
        nrm, _, _ = oracle.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
        t1 = time.perf_counter()
        oracle.icp(w.source, w.target, nrm.astype(np.float32), None, d32, w.iters)
        loop_s += time.perf_counter() - t1
        pairs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": pairs / el, "unit": "pairs/s", "cores": oracle.num_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"{pairs} full pair(s) of the same workload (normals + ICP incl. kd-tree builds), "
                      f"{el:.1f} s wall",
            "mpt_iter_per_s": w.n * w.iters * pairs / loop_s / 1e6}


def cpu_baseline_batch(b, budget_s):
    """The CPU oracle on the batch's pairs in order (normals + ICP each),
    until about budget_s seconds have passed."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    pairs, pts_iter, loop_s = 0, 0, 0.0
    for w in b.pairs:
        nrm, _, _ = oracle.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
        t1 = time.perf_counter()
        oracle.icp(w.source, w.target, nrm.astype(np.float32), None, float(np.float32(w.d_max)), w.iters)
        loop_s += time.perf_counter() - t1
        pairs += 1
        pts_iter += w.n * w.iters
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": pairs / el, "unit": "pairs/s", "cores": oracle.num_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"the first {pairs} of {b.n_pairs} pairs (normals + ICP incl. kd-tree builds), "
                      f"{el:.1f} s wall",
            "mpt_iter_per_s": pts_iter / loop_s / 1e6}


def bench_projective(args):
    """Projective workload: two VGA depth frames of one room; one step =
    normals of the target frame + projective-association ICP."""
    import torch
    from gen.scenes import room_views, rng_for
    from paper_1807_00399_amd import pcgpu
    c = PROJECTIVE
    dev = torch.device("cuda:0")
    src_np, tgt_np, C, K = room_views(rng_for(5, 0), c["width"], c["height"], c["angle"], c["t"])
    src = torch.from_numpy(src_np).to(dev)
    tgt = torch.from_numpy(tgt_np).to(dev)
    n = src_np.shape[0]
    T = torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24, dtype=torch.uint8, device=dev)
    ws_n = torch.empty(pcgpu.lib.estimate_normals_workspace_size(n, c["k"]), dtype=torch.uint8, device=dev)
    ws_i = torch.empty(pcgpu.lib.icp_projective_workspace_size(n, c["iters"]), dtype=torch.uint8, device=dev)

    def step():
        nrm, _ = pcgpu.estimate_normals(tgt, c["k"], curvature=False, workspace=ws_n)
        pcgpu.icp_projective(src, tgt, nrm, c["width"], c["height"], K, None, c["d_max"], c["iters"],
                             workspace=ws_i, out_T=T, out_stats=stats, read_stats=False)

    tuning = autotune_step(args, step, c["name"], n)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = pcgpu.decode_stats(stats)
    ev = HipEvents(c["iters"])
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, c["iters"])
    kern, loop_ms = [], []
    for _ in range(max(3, min(args.steps, 10))):
        step()
        torch.cuda.synchronize()
        cnt = pcgpu.lib.pc_kernel_timer_count()
        kern += [ev.elapsed_ms(i) for i in range(cnt)]
        loop_ms.append(ev.span_ms(0, cnt - 1))
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    avg_kernel_s = float(np.mean(kern)) * 1e-3
    algo = PROJ_BYTES_PER_POINT * n
    achieved = algo / avg_kernel_s / 1e9
    out = {
        "metric": METRIC, "value": args.steps / el, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{c['name']}: two {c['width']}x{c['height']} depth frames of one room, "
                               f"projective association, k={c['k']} normals, d_max {c['d_max']}, "
                               f"{c['iters']} iterations",
                   "points_per_cloud": n, "iters": c["iters"]},
        "mpt_iter_per_s": n * c["iters"] / (float(np.median(loop_ms)) * 1e-3) / 1e6,
        "loop_ms": float(np.median(loop_ms)),
        "icp_status": st,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles("icp_accum", "projective"),
                     "kernel": "k_icp_accum_proj", "avg_kernel_us": avg_kernel_s * 1e6,
                     "algorithmic_bytes_per_launch": algo},
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t1 = time.perf_counter()
        pairs, loop_s = 0, 0.0
        while True:
            nrm, _, _ = oracle.normals(tgt_np, c["k"], (0.0, 0.0, 0.0), method="kdtree")
            t2 = time.perf_counter()
            oracle.icp_projective(src_np, tgt_np, nrm.astype(np.float32), c["width"], c["height"], K, None,
                                  float(np.float32(c["d_max"])), c["iters"])
            loop_s += time.perf_counter() - t2
            pairs += 1
            if time.perf_counter() - t1 >= args.cpu_seconds:
                break
        el1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": pairs / el1, "unit": "pairs/s", "cores": oracle.num_threads(),
                               "cpu": cpu_model(), "kind": "oracle", "sample": f"{pairs} full pair(s) (normals + ICP), {el1:.1f} s wall",
                               "mpt_iter_per_s": n * c["iters"] * pairs / loop_s / 1e6}
    print(json.dumps(out), flush=True)


def cpu_baseline_learned(b, gpu_T, budget_s):
    """The oracle's 8-start ICP (kd-tree normals + 8 registrations per pair)
    on the first pairs of the workload until about budget_s seconds have
    passed, and how many of the GPU's learned-initialiser results agree
    with it (1e-5 rad, 1e-6)."""
    import oracle
    from oracle import pose_net as opn
    oracle.build(force=False)

    def pose_err(Ta, Tb):
        c = (np.trace(Ta[:3, :3] @ Tb[:3, :3].T) - 1.0) / 2.0
        return float(np.arccos(np.clip(c, -1.0, 1.0))), float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))

    t0 = time.perf_counter()
    pairs, agree = 0, 0
    for j, w in enumerate(b.pairs):
        nrm, _, _ = oracle.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
        ro, _ = opn.multi_start_icp(oracle, w.source, w.target, nrm.astype(np.float32), float(np.float32(w.d_max)),
                                    w.iters)
        ea, et = pose_err(gpu_T[j], ro["T"])
        agree += int(ea <= 1e-5 and et <= 1e-6)
        pairs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": pairs / el, "unit": "pairs/s", "cores": oracle.num_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"the first {pairs} of {b.n_pairs} pairs, 8-start ICP each (normals + 8 registrations), "
                      f"{el:.1f} s wall",
            "gpu_learned_agrees_with_oracle_8_start": f"{agree}/{pairs}"}


def learned_legs(steps, warmup, args=None):
    """The learned-initialiser workload through four starts: plain (identity),
    8-start, learned with 8-start fallback, learned only.  One step = target
    normals + registration of every pair.  Success = final pose within
    1e-5 rad and 1e-6 of the generating transform (the pairs are exact
    copies, so the optimum is that transform)."""
    import torch
    from gen import POSE_CONFIG, pose_pairs
    from paper_1807_00399_amd import pcgpu
    from paper_1807_00399_amd.train_pose_net import load_params
    dev = torch.device("cuda:0")
    cfg = POSE_CONFIG
    b = pose_pairs(cfg["eval_config"])
    off = b.offsets
    m = b.n_pairs
    src = torch.from_numpy(b.source).to(dev)
    tgt = torch.from_numpy(b.target).to(dev)
    params = torch.from_numpy(load_params()).to(dev)
    gt = np.stack([w.T_gt for w in b.pairs])
    ws_n = torch.empty(pcgpu.lib.estimate_normals_batched_workspace_size(m, off.ctypes.data), dtype=torch.uint8,
                       device=dev)
    ws_l = torch.empty(pcgpu.lib.icp_learned_batched_workspace_size(m, off.ctypes.data, off.ctypes.data,
                                                                    cfg["iters"]), dtype=torch.uint8, device=dev)
    T = torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24 * m, dtype=torch.uint8, device=dev)

    def run(mode):
        nrm, _ = pcgpu.estimate_normals_batched(tgt, off, cfg["k"], curvature=False, workspace=ws_n)
        if mode == "plain":
            Tm, sm = pcgpu.icp_point_to_plane_batched(src, off, tgt, nrm, off, None, cfg["d_max"], cfg["iters"],
                                                      workspace=ws_l, out_T=T, out_stats=stats, read_stats=False)
            return Tm, sm, None
        code = {"multi_start": pcgpu.PC_INIT_MULTI_START, "learned": pcgpu.PC_INIT_LEARNED,
                "learned_only": pcgpu.PC_INIT_LEARNED_ONLY}[mode]
        return pcgpu.icp_learned_batched(code, params, src, off, tgt, nrm, off, cfg["d_max"], cfg["iters"],
                                         accept_rms=cfg["accept_rms"], workspace=ws_l, read_stats=False)

    # one tuning for all legs: the learned path's (its fallback is 8-start ICP)
    tuning = autotune_step(args, lambda: run("learned"), "pose_pairs_512", b.n) if args is not None else None
    legs = {}
    for mode in ("plain", "multi_start", "learned", "learned_only"):
        for _ in range(warmup):
            run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            Tm, sm, start = run(mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Tn = Tm.cpu().numpy()
        ea = np.array([np.arccos(np.clip((np.trace(Tn[j, :3, :3] @ gt[j, :3, :3].T) - 1) / 2, -1, 1))
                       for j in range(m)])
        et = np.linalg.norm(Tn[:, :3, 3] - gt[:, :3, 3], axis=1)
        leg = {"pairs_per_s": m * steps / el, "ms_per_step": 1e3 * el / steps,
               "success": float(np.mean((ea <= 1e-5) & (et <= 1e-6)))}
        if start is not None and mode == "learned":
            leg["fallback_fraction"] = float(np.mean(start.cpu().numpy() >= 0))
        legs[mode] = leg
        if mode == "learned":
            learned_T = Tn
    # the whole predict call (torch events: the library runs on torch's
    # stream), and its encoder kernel alone (the library's HIP events, timer
    # slot 0, recorded on the stream the kernel is launched on)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pcgpu.pose_net_predict(params, src, off, tgt, off)
    e0.record()
    for _ in range(10):
        T0 = pcgpu.pose_net_predict(params, src, off, tgt, off)
    e1.record()
    torch.cuda.synchronize()
    call_s = e0.elapsed_time(e1) / 10 * 1e-3
    ev = HipEvents(1)
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, 1)
    ks = []
    for _ in range(10):
        pcgpu.pose_net_predict(params, src, off, tgt, off)
        torch.cuda.synchronize()
        assert pcgpu.lib.pc_kernel_timer_count() == 1
        ks.append(ev.elapsed_ms(0))
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    pred_s = float(np.mean(ks)) * 1e-3
    e_init = np.array([np.degrees(np.arccos(np.clip((np.trace(a[:3, :3] @ g[:3, :3].T) - 1) / 2, -1, 1)))
                       for a, g in zip(T0.cpu().numpy(), gt)])
    info = {"workload": f"{b.name}: {m} exact-copy pairs of {cfg['n_points']} points, sphere+plane or room, "
                        f"rotation U(0, 90) deg, |t| U(0, 0.3); k={cfg['k']}, d_max {cfg['d_max']}, "
                        f"{cfg['iters']} iterations, accepted rms {cfg['accept_rms']}",
            "pairs": m, "points_per_side": b.n, "legs": legs, "tuning": tuning,
            "learned_init_rotation_error_deg": {"median": float(np.median(e_init)),
                                                "within_30": float(np.mean(e_init < 30))},
            "predict_ms": call_s * 1e3,
            "predict_call_tflops": ENC_FLOPS_PER_POINT * 2 * b.n / call_s / 1e12,
            "encoder_kernel_us": pred_s * 1e6,
            "encoder_forward_tflops": ENC_FLOPS_PER_POINT * 2 * b.n / pred_s / 1e12}
    return info, b, learned_T, pred_s


# one training row of the encoder's backward (per cloud and channel): the
# arg-max point's layer-1 and layer-2 recompute, the layer-1 gradient, and
# the dW1|b1, dW2|b2 and dW3 products, 2 flops per multiply-add
TRAIN_BWD_FLOPS_PER_ROW = 2 * (3 * 64 + 64 * 128 + 64 * 128 + 4 * 64 + 65 * 128 + 128)
W2_GRAD_FLOPS_PER_ROW = 2 * 65 * 128


def training_step_metrics(steps=10, warmup=2, n_pairs=64):
    """pose_net_train_step (forward with arg-max, head and encoder backward,
    Adam) on n_pairs pairs of 4,096 points, timed per phase by the library's
    events: forward, backward, and the second-layer weight gradients on the
    matrix cores."""
    import torch
    from gen import POSE_CONFIG, pose_pairs
    from paper_1807_00399_amd import pcgpu
    from paper_1807_00399_amd.train_pose_net import load_params
    dev = torch.device("cuda:0")
    b = pose_pairs(POSE_CONFIG["eval_config"], n_pairs)
    off = b.offsets
    src, tgt = torch.from_numpy(b.source).to(dev), torch.from_numpy(b.target).to(dev)
    params = torch.from_numpy(load_params()).to(dev)
    m_, v_ = torch.zeros_like(params), torch.zeros_like(params)
    labels = np.stack([w.T_gt for w in b.pairs])
    ws = torch.empty(pcgpu.lib.pose_net_workspace_size(n_pairs, off.ctypes.data, off.ctypes.data),
                     dtype=torch.uint8, device=dev)
    p0 = params.clone()

    def step(i):
        pcgpu.pose_net_train_step(params, m_, v_, i, 1e-6, src, off, tgt, off, labels, workspace=ws)

    for i in range(warmup):
        step(i + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(warmup + i + 1)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ev = HipEvents(3)
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, 3)
    ph = []
    for i in range(3):
        step(warmup + steps + i + 1)
        torch.cuda.synchronize()
        assert pcgpu.lib.pc_kernel_timer_count() == 3
        ph.append([ev.elapsed_ms(k) for k in range(3)])
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    params.copy_(p0)
    fwd, bwd, w2 = (float(np.median([x[k] for x in ph])) * 1e-3 for k in range(3))
    rows = 2 * n_pairs * 256
    return {"pairs_per_step": n_pairs, "points_per_cloud": int(b.n // n_pairs), "steps_per_s": 1.0 / el,
            "ms_per_step": el * 1e3, "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
            "forward_tflops": ENC_FLOPS_PER_POINT * 2 * b.n / fwd / 1e12,
            "backward_tflops": TRAIN_BWD_FLOPS_PER_ROW * rows / bwd / 1e12,
            "w2_grad_us": w2 * 1e6, "w2_grad_tflops": W2_GRAD_FLOPS_PER_ROW * rows / w2 / 1e12,
            "note": "backward flops: per (cloud, channel) row the arg-max point's recompute and the dW1, dW2, dW3 "
                    "products; forward: the two matrix-core layers of every point of both clouds"}


def bench_learned(args):
    info, b, learned_T, pred_s = learned_legs(args.steps, args.warmup, args)
    leg = info["legs"]["learned"]
    flops = ENC_FLOPS_PER_POINT * 2 * b.n
    achieved = flops / pred_s / 1e12
    out = {
        "metric": METRIC,
        "value": leg["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (encoder bf16 matrix cores, f32 accumulation)",
        "data": "synthetic",
        "config": {"workload": info["workload"], "pairs": info["pairs"], "points_per_side": info["points_per_side"]},
        "success": leg["success"],
        "learned_vs_plain": info["legs"],
        "learned_init_rotation_error_deg": info["learned_init_rotation_error_deg"],
        "tuning": info["tuning"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_enc_forward (encoder forward of both clouds of every pair; HIP events "
                               "around the kernel inside pose_net_predict)",
                     "avg_call_us": pred_s * 1e6, "algorithmic_flops_per_call": float(flops),
                     "predict_call_us": info["predict_ms"] * 1e3,
                     "predict_call_frac": info["predict_call_tflops"] / BF16_PEAK_TFLOPS},
    }
    out["training"] = training_step_metrics()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_learned(b, learned_T, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched workload: all pairs per step through the batched entry points."""
    import torch
    from gen import batch_workload
    from paper_1807_00399_amd import pcgpu
    dev = torch.device("cuda:0")
    b = batch_workload(3)
    off = b.offsets
    kc = b.param("k").astype(np.int32)
    dm = b.param("d_max").astype(np.float32)
    it = b.param("iters").astype(np.int32)
    src = torch.from_numpy(b.source).to(dev)
    tgt = torch.from_numpy(b.target).to(dev)
    m = b.n_pairs
    T = torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24 * m, dtype=torch.uint8, device=dev)
    ws_i = torch.empty(pcgpu.lib.icp_point_to_plane_with_normals_batched_workspace_size(
        m, off.ctypes.data, off.ctypes.data, int(it.max())), dtype=torch.uint8, device=dev)

    def step():
        # targets' normals and all registrations over one pyramid of the targets
        pcgpu.icp_point_to_plane_with_normals_batched(src, off, tgt, off, kc, (0.0, 0.0, 0.0), None, dm, it,
                                                      workspace=ws_i, out_T=T, out_stats=stats, read_stats=False)

    tuning = autotune_step(args, step, "uneven_pairs_256", b.n)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    el, launch = el_eager, "eager"
    if not args.no_graph:
        # the batched call launches kernels only: captured once, replayed
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        # timed region: K whole steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        el, launch = time.perf_counter() - t0, "graph replay"
    st = pcgpu.decode_stats_batched(stats)

    # per-iteration accumulate kernel: events recorded by the library
    iters_max = int(it.max())
    ev = HipEvents(iters_max)
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, iters_max)
    kern, loop_ms = [], []
    for _ in range(3):
        step()
        torch.cuda.synchronize()
        cnt = pcgpu.lib.pc_kernel_timer_count()
        kern.append([ev.elapsed_ms(i) for i in range(cnt)])
        loop_ms.append(ev.span_ms(0, cnt - 1))
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    kern = np.median(np.array(kern), axis=0) * 1e-3
    # source points processed by launch i: pairs still iterating
    ran = np.array([r["iterations_run"] for r in st])
    sizes = np.diff(off)
    active = np.array([int(sizes[ran > i].sum()) for i in range(len(kern))])
    achieved = ICP_BYTES_PER_POINT * active.sum() / kern.sum() / 1e9
    pts_iter = int((sizes * ran).sum())

    # the same pairs one call each (single-pair entry points), for comparison
    seq_pairs = 0 if args.no_compare else min(m, 64)
    srcs = [src[off[j]:off[j + 1]] for j in range(seq_pairs)]
    tgts = [tgt[off[j]:off[j + 1]] for j in range(seq_pairs)]
    seq_el = 0.0
    for rep in range(2 if seq_pairs else 0):   # the first round grows the workspace
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for j in range(seq_pairs):
            pcgpu.icp_point_to_plane_with_normals(srcs[j], tgts[j], int(kc[j]), (0.0, 0.0, 0.0), None, float(dm[j]),
                                                  int(it[j]), read_stats=False)
        torch.cuda.synchronize()
        seq_el = time.perf_counter() - t1

    out = {
        "metric": METRIC,
        "value": m * args.steps / el,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{b.name}: {m} uneven pairs per step, {b.n} points per side, "
                               f"sphere+plane (k=10, d_max 0.1, 20 iterations) or room (k=16, d_max 0.05, "
                               f"30 iterations) pairs",
                   "pairs": m, "points_per_side": b.n, "launch": launch},
        "eager_pairs_per_s": m * args.steps / el_eager,
        "mpt_iter_per_s": pts_iter / (float(np.median(loop_ms)) * 1e-3) / 1e6,
        "loop_ms": float(np.median(loop_ms)),
        "single_call_pairs_per_s": seq_pairs / seq_el if seq_pairs else None,
        "tuning": tuning,
        "icp_status_counts": {str(k): int(v) for k, v in zip(*np.unique([r["status"] for r in st],
                                                                        return_counts=True))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profiles("icp_accum", "batch"),
                     "kernel": "k_icp_accum",
                     "avg_kernel_us": float(kern.mean()) * 1e6,
                     "algorithmic_bytes_per_launch": float(ICP_BYTES_PER_POINT * active.mean())},
    }
    g = batch_golden(b)
    Tn = T.cpu().numpy()
    if g is not None:
        out["pose_vs_oracle"] = pose_check(
            Tn, np.array([p["T"] for p in g["pairs"]]), [r["inliers"] for r in st],
            [p["inliers"] for p in g["pairs"]],
            source="tests/golden/icp_batch256.json (oracle kd-tree normals + float64 ICP, input digests matched)")
    else:
        out["pose_vs_oracle"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(b, args.cpu_seconds)
    return out


def bench_search(args):
    """Standalone k-NN (every point of a cloud against the cloud) or PCA
    normals of a cloud: one step = the pyramid build + the search kernel
    (knn_search / estimate_normals, one call)."""
    import torch
    from gen import make_workload
    from paper_1807_00399_amd import pcgpu
    dev = torch.device("cuda:0")
    w = make_workload(WORKLOADS[args.cloud])
    x = torch.from_numpy(w.target).to(dev)
    n, k = w.n, w.k
    knn = args.workload == "knn"
    if knn:
        idx = torch.empty((n, k), dtype=torch.int32, device=dev)
        d2 = torch.empty((n, k), dtype=torch.float32, device=dev)
        ws = torch.empty(pcgpu.lib.knn_search_workspace_size(n, n, k), dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream().cuda_stream

        def step():
            pcgpu._check(pcgpu.lib.knn_search(x.data_ptr(), n, x.data_ptr(), n, k, idx.data_ptr(), d2.data_ptr(),
                                              ws.data_ptr(), ws.numel(), stream), "knn_search")
    else:
        ws = torch.empty(pcgpu.lib.estimate_normals_workspace_size(n, k), dtype=torch.uint8, device=dev)

        def step():
            pcgpu.estimate_normals(x, k, workspace=ws)
    # leaf size and pyramid depth of the search, as for the ICP workloads
    tuning = autotune_step(args, step, f"{args.workload}_{w.name}", n)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev = HipEvents(1)
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, 1)
    kern = []
    for _ in range(max(3, min(args.steps, 10))):
        step()
        torch.cuda.synchronize()
        assert pcgpu.lib.pc_kernel_timer_count() == 1
        kern.append(ev.elapsed_ms(0))
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    kern_s = float(np.median(kern)) * 1e-3
    algo = (KNN_BYTES_PER_QUERY(k) if knn else NORMALS_BYTES_PER_POINT) * n
    achieved = algo / kern_s / 1e9
    name = "k_knn" if knn else "k_normals"
    tag = f"{'knn' if knn else 'normals'}_{args.cloud}"
    out = {
        "metric": ("k-NN queries/s" if knn else "normals points/s") + " (exact, bit-equal to brute force)",
        "value": n * args.steps / el, "unit": "queries/s" if knn else "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (normals: f64 covariance and eigensolver)", "data": "synthetic",
        "config": {"workload": f"{w.name}: {'k-NN of every point against its cloud' if knn else 'PCA normals'}, "
                               f"{n} points, k={k}; one step = pyramid build + {name}",
                   "points": n, "k": k},
        "search_kernel_ms": kern_s * 1e3,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(name, args.cloud),
                     "kernel": name, "avg_kernel_us": kern_s * 1e6, "algorithmic_bytes_per_launch": algo},
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t1 = time.perf_counter()
        reps = 0
        while True:
            if knn:
                oracle.knn(w.target, w.target, k, "kdtree")
            else:
                oracle.normals(w.target, k, (0.0, 0.0, 0.0), method="kdtree")
            reps += 1
            if time.perf_counter() - t1 >= args.cpu_seconds:
                break
        el1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": n * reps / el1, "unit": out["unit"], "cores": oracle.num_threads(),
                               "cpu": cpu_model(), "kind": "oracle",
                               "sample": f"{reps} whole cloud(s) through the oracle's kd-tree "
                                         f"({'k-NN' if knn else 'normals'}), {el1:.1f} s wall"}
    print(json.dumps(out), flush=True)


def bench_single(args, workload, with_cpu=True):
    """One pair per step: target pyramid + normals + ICP in one call."""
    import torch

    from gen import make_workload
    from paper_1807_00399_amd import pcgpu
    dev = torch.device("cuda:0")
    w = make_workload(WORKLOADS[workload])
    src = torch.from_numpy(w.source).to(dev)
    tgt = torch.from_numpy(w.target).to(dev)
    T = torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24, dtype=torch.uint8, device=dev)
    ws = torch.empty(pcgpu.lib.icp_point_to_plane_with_normals_workspace_size(w.n, w.n, w.iters),
                     dtype=torch.uint8, device=dev)

    def step():
        # target normals and ICP in one call: one target pyramid serves both
        pcgpu.icp_point_to_plane_with_normals(src, tgt, w.k, (0.0, 0.0, 0.0), None, w.d_max, w.iters,
                                              workspace=ws, out_T=T, out_stats=stats, read_stats=False)

    tuning = autotune_step(args, step, w.name, w.n)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # K whole steps launched eagerly
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    el = el_eager
    launch = "eager"
    if not args.no_graph:
        # the step launches kernels only: captured once as a graph and
        # replayed, the same kernels run without per-launch host overhead
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        # timed region: K whole steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        launch = "graph replay"
    ms_per_step = 1e3 * el / args.steps
    st = pcgpu.decode_stats(stats)

    # dominant kernel: per-iteration correspondence + accumulation, events
    # recorded by the library around each launch on its stream
    ev = HipEvents(w.iters)
    pcgpu.lib.pc_set_kernel_timer(ev.beg, ev.end, w.iters)
    kern_ms, loop_ms = [], []
    for _ in range(max(3, min(args.steps, 10))):
        step()
        torch.cuda.synchronize()
        cnt = pcgpu.lib.pc_kernel_timer_count()
        kern_ms += [ev.elapsed_ms(i) for i in range(cnt)]
        loop_ms.append(ev.span_ms(0, cnt - 1))
    pcgpu.lib.pc_set_kernel_timer(None, None, 0)
    loop_s = float(np.median(loop_ms)) * 1e-3
    avg_kernel_s = float(np.mean(kern_ms)) * 1e-3
    algo_bytes = ICP_BYTES_PER_POINT * w.n
    kernel_name = "k_icp_accum"
    by_iter = [round(float(x) * 1e3, 1) for x in np.median(np.array(kern_ms).reshape(-1, w.iters), axis=0)]
    achieved = algo_bytes / avg_kernel_s / 1e9
    traffic = traffic_from_profiles("icp_accum", workload)

    out = {
        "metric": METRIC,
        "value": args.steps / el,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: one pair, {w.n} points per cloud, k={w.k} normals, "
                               f"d_max {w.d_max}, {w.iters} iterations",
                   "points_per_cloud": w.n, "k": w.k, "d_max": w.d_max, "iters": w.iters, "launch": launch},
        "eager_pairs_per_s": args.steps / el_eager,
        "mpt_iter_per_s": w.n * w.iters / loop_s / 1e6,
        "loop_ms": loop_s * 1e3,
        "kernel_us_by_iter": by_iter,
        "icp_status": st,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name, "avg_kernel_us": avg_kernel_s * 1e6,
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "valu_issue_share": valu_from_profiles(workload)},
    }
    g = single_golden(w)
    out["pose_vs_oracle"] = None if g is None else pose_check(
        T.cpu().numpy(), np.array(g["T"]), [st["inliers"]], [g["inliers"]],
        source="tests/golden/icp_workloads.json (oracle kd-tree normals + float64 ICP, input digests matched)")
    if with_cpu and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    return out



def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "projective":
        bench_projective(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload in ("knn", "normals"):
        bench_search(args)
        return
    if args.workload != "batch":
        print(json.dumps(bench_single(args, args.workload)), flush=True)
        return
    out = bench_batch(args)
    if not args.no_street:
        # the single-pair LiDAR street (2,097,152 points), timed the same way
        s = bench_single(args, "street", with_cpu=False)
        out["street"] = {k: s[k] for k in ("value", "unit", "ms_per_step", "eager_pairs_per_s", "mpt_iter_per_s",
                                           "loop_ms", "config", "icp_status", "tuning", "roofline",
                                           "pose_vs_oracle")}
    if not args.no_learned:
        info = learned_legs(min(args.steps, 5), 1, args)[0]
        out["learned_vs_plain"] = {"workload": info["workload"], "legs": info["legs"],
                                   "learned_init_rotation_error_deg": info["learned_init_rotation_error_deg"],
                                   "encoder_kernel_us": info["encoder_kernel_us"],
                                   "encoder_forward_tflops": info["encoder_forward_tflops"],
                                   "predict_call_tflops": info["predict_call_tflops"],
                                   "training": training_step_metrics()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

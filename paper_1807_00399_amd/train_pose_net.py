"""Training of the learned pose initialiser on pairs and poses produced by the
library's own multi-start ICP.

    python -m paper_1807_00399_amd.train_pose_net --steps 3000 --out ckpt.npz

Each step draws `batch` clouds from a pool of scenes of the training
generator stream (sphere + plane or room scans, 4096 points), moves each by
a fresh random rigid motion (angle U(0, 90) degrees, |t| U(0, 0.3)),
estimates the target normals and runs multi-start ICP on the GPU, and takes
a training step on the pairs whose ICP result reached the accepted residual,
with that result as the label (pairs where no start converged get weight 0).
The forward, backward and Adam update are the library's kernels
(pose_net_train_step).  Checkpoints (numpy .npz, no pickled objects) hold
the parameters, Adam moments, step count and generator state, so a run can
be resumed with --resume; --export writes the parameters alone for
inference.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "pose_net.npz")


def load_params(path: str = WEIGHTS) -> np.ndarray:
    """Flat float32 parameters from a checkpoint or an exported weights file."""
    with np.load(path, allow_pickle=False) as z:
        return np.ascontiguousarray(z["params"].astype(np.float32))


def save_checkpoint(path, params, m, v, step, rng, meta, full=True):
    arrays = {"params": params, "meta": np.array(json.dumps(meta))}
    if full:
        arrays.update(adam_m=m, adam_v=v, step=np.array(step, np.int64),
                      rng_state=np.array(json.dumps(rng.bit_generator.state)))
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def rotation_error_deg(Ta, Tb):
    Ra, Rb = np.asarray(Ta)[..., :3, :3], np.asarray(Tb)[..., :3, :3]
    c = (np.einsum("nij,nij->n", Ra, Rb) - 1.0) / 2.0
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--pool", type=int, default=2048, help="scenes in the training pool")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-every", type=int, default=500)
    ap.add_argument("--eval-pairs", type=int, default=256)
    ap.add_argument("--out", default="pose_net_ckpt.npz")
    ap.add_argument("--export", default=None, help="also write the parameters alone to this file")
    ap.add_argument("--resume", default=None)
    args = ap.parse_args(argv)

    import torch

    from gen import POSE_CONFIG, apply_rigid, pose_net_init, pose_pairs, random_rigid
    from paper_1807_00399_amd import pcgpu

    assert torch.cuda.is_available(), "training runs on the GPU"
    dev = torch.device("cuda:0")
    cfg = POSE_CONFIG
    n_pts = cfg["n_points"]
    rng = np.random.Generator(np.random.PCG64(args.seed))
    if args.resume:
        with np.load(args.resume, allow_pickle=False) as z:
            params_np = z["params"].astype(np.float32)
            m_np, v_np = z["adam_m"].astype(np.float32), z["adam_v"].astype(np.float32)
            step0 = int(z["step"])
            rng.bit_generator.state = json.loads(str(z["rng_state"]))
    else:
        params_np = pose_net_init(rng)
        m_np = np.zeros_like(params_np)
        v_np = np.zeros_like(params_np)
        step0 = 0
    params = torch.from_numpy(params_np).to(dev)
    adam_m = torch.from_numpy(m_np).to(dev)
    adam_v = torch.from_numpy(v_np).to(dev)

    t0 = time.time()
    pool = [w.source for w in pose_pairs(cfg["train_config"], args.pool, n_points=n_pts).pairs]
    ev = pose_pairs(cfg["eval_config"], args.eval_pairs, n_points=n_pts)
    ev_src = torch.from_numpy(ev.source).to(dev)
    ev_tgt = torch.from_numpy(ev.target).to(dev)
    ev_gt = np.stack([w.T_gt for w in ev.pairs])
    print(f"pool of {len(pool)} scenes and {ev.n_pairs} evaluation pairs in {time.time() - t0:.1f} s", flush=True)

    B = args.batch
    off = np.arange(B + 1, dtype=np.int64) * n_pts
    ws_n = ws_i = ws_t = None

    def evaluate():
        T = pcgpu.pose_net_predict(params, ev_src, ev.offsets, ev_tgt, ev.offsets).cpu().numpy()
        e = rotation_error_deg(T, ev_gt)
        return {"median_deg": float(np.median(e)), "within_20deg": float(np.mean(e < 20)),
                "within_30deg": float(np.mean(e < 30))}

    hist = []
    t_start = time.time()
    for step in range(step0 + 1, step0 + args.steps + 1):
        idx = rng.integers(0, len(pool), size=B)
        src = np.empty((B * n_pts, 3), np.float32)
        tgt = np.empty((B * n_pts, 3), np.float32)
        for j, i in enumerate(idx):
            T = random_rigid(rng, rng.uniform(*cfg["angle"]), rng.uniform(*cfg["t"]))
            src[j * n_pts:(j + 1) * n_pts] = pool[i]
            tgt[j * n_pts:(j + 1) * n_pts] = apply_rigid(T, pool[i])
        S = torch.from_numpy(src).to(dev)
        Tt = torch.from_numpy(tgt).to(dev)
        if ws_n is None:
            ws_n = torch.empty(pcgpu.lib.estimate_normals_batched_workspace_size(B, off.ctypes.data),
                               dtype=torch.uint8, device=dev)
            ws_i = torch.empty(pcgpu.lib.icp_learned_batched_workspace_size(B, off.ctypes.data, off.ctypes.data,
                                                                            cfg["iters"]),
                               dtype=torch.uint8, device=dev)
            ws_t = torch.empty(pcgpu.lib.pose_net_workspace_size(B, off.ctypes.data, off.ctypes.data),
                               dtype=torch.uint8, device=dev)
        nrm, _ = pcgpu.estimate_normals_batched(Tt, off, cfg["k"], curvature=False, workspace=ws_n)
        T_lab, st, _ = pcgpu.icp_learned_batched(pcgpu.PC_INIT_MULTI_START, None, S, off, Tt, nrm, off,
                                                 cfg["d_max"], cfg["iters"], workspace=ws_i)
        w = np.array([1.0 if (r["status"] in (0, 1) and r["inliers"] > 0 and r["rms"] <= cfg["accept_rms"])
                      else 0.0 for r in st], np.float32)
        if step <= args.warmup:
            lr = args.lr * step / args.warmup
        else:
            frac = (step - args.warmup) / max(1, step0 + args.steps - args.warmup)
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1.0 + math.cos(math.pi * min(1.0, frac)))
        loss, _ = pcgpu.pose_net_train_step(params, adam_m, adam_v, step, lr, S, off, Tt, off, T_lab,
                                            pair_weight=w, workspace=ws_t)
        wl = float((loss.cpu().numpy()).sum() / max(w.sum(), 1.0))
        hist.append(wl)
        if step % 100 == 0 or step == step0 + 1:
            print(f"step {step} lr {lr:.2e} loss {np.mean(hist[-100:]):.4f} labelled {w.mean():.2f} "
                  f"({time.time() - t_start:.0f} s)", flush=True)
        if step % args.eval_every == 0 or step == step0 + args.steps:
            e = evaluate()
            print(f"eval step {step}: {json.dumps(e)}", flush=True)
            meta = {"step": step, "eval": e, "batch": B, "pool": args.pool, "seed": args.seed,
                    "workload": cfg["name"], "n_points": n_pts}
            save_checkpoint(args.out, params.cpu().numpy(), adam_m.cpu().numpy(), adam_v.cpu().numpy(), step,
                            rng, meta)
            if args.export:
                save_checkpoint(args.export, params.cpu().numpy(), None, None, step, rng, meta, full=False)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()

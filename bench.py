"""Benchmark of the Siddon DRR hot path on one MI355X.

Workload: 512 x 512 x 133 CT at 0.7 x 0.7 x 2.5 mm (seeded ellipsoid
phantom with a bone-like shell), 256 x 256 detector at 1.4 mm, SDD 1020 mm,
256 random poses (angles +-pi/6, shifts +-30 mm) per batch.

One step = one pass of the hot path over the batch:
  forward     all 256 DRRs through a batched plan: one persistent tile-queue
              launch replayed from a captured HIP graph, launch shape chosen
              by the autotuner                                (timed: fwd)
  fwd + bwd   all 256 DRRs, negative ZNCC against per-pose targets and the
              pose gradient, in one fused tracing launch      (timed: fwd+bwd)
  direct      the same 256 forward DRRs through the plain drr_render call
              (one launch, no plan)                           (timed: direct)
The printed JSON line reports forward DRRs/s of the plan as `value`, with
fwd+bwd throughput, voxel-gather rates, latency percentiles, the HBM
roofline of the forward kernel and the FP64 CPU oracle timed on a bounded
sample.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = ("DRRs/sec and Gvoxel-gathers/s (fwd, fwd+bwd) at 512²×133 CT, "
          "256² det; p99 ms")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--poses", type=int, default=256)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="approximate CPU time (thread-seconds) for the oracle sample")
    ap.add_argument("--only", choices=["fwd", "fwdbwd", "direct"], default=None,
                    help="time one phase only (for profiling runs)")
    ap.add_argument("--mode", choices=["drr", "register", "serve"], default="drr",
                    help="drr: the headline forward / fwd+bwd batch (default); register: "
                         "32 batched registrations; serve: the request loop over four "
                         "resident volumes at a QPS sweep")
    ap.add_argument("--requests", type=int, default=2000,
                    help="requests per QPS point in --mode serve")
    ap.add_argument("--tune-cache", default=os.path.join(
                        os.path.dirname(os.path.abspath(__file__)), "paper_2208_12737_amd",
                        "tuning.txt"),
                    help="autotuner cache file: launch shapes chosen earlier for a workload "
                         "are reused, new workloads are tuned and appended ('' = always tune)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (reference kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def _source_digest():
    """Digest of the kernel sources, to tell whether a stored profile still
    describes the kernels that run."""
    import hashlib
    import glob
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in sorted(glob.glob(os.path.join(here, "paper_2208_12737_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(plan_cfg):
    """HBM-side bytes per forward launch from the committed rocprofv3 counter
    summary (FETCH_SIZE, WRITE_SIZE scaled by a plain copy kernel), or None
    when the kernel sources or launch shape changed since it was taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "render_fwd_ct512_det256_poses256.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    import re
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_digest") != _source_digest():
        return None
    for k in ("strategy", "tile_code", "wg_per_cu"):
        if rec.get(k) != plan_cfg[k]:
            return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(ph, poses, det_px, pitch, cpu_seconds):
    """The FP64 oracle on host cores over whole DRRs of the same workload."""
    import oracle
    nthreads = oracle.max_threads()
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    p64 = poses.astype(np.float64)
    t0 = time.perf_counter()
    oracle.render(grid, p64[:1], det_px, det_px, pitch, pitch, nthreads=nthreads)
    first = time.perf_counter() - t0
    n = int(max(1, min(len(p64) - 1, round(cpu_seconds / max(first * nthreads, 1e-6)))))
    t0 = time.perf_counter()
    oracle.render(grid, p64[1:1 + n], det_px, det_px, pitch, pitch, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "DRRs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} whole {det_px}x{det_px} DRRs of the benchmark poses "
                      f"({n * det_px * det_px} rays), FP64 sort-based Siddon, "
                      f"{dt:.2f} s wall on {nthreads} threads"}


def bench_register(args):
    """32 registration problems on the 512 x 512 x 133 CT, 256 x 256
    detector: ground-truth poses (angles +-pi/6, shifts +-30 mm), starts
    offset by up to 15 deg / 25 mm per parameter, 200 steps of momentum
    gradient descent on -ZNCC with the step sizes of Sec. 3.2, all problems
    in one captured graph; beside it the one-DRR-at-a-time autograd path."""
    import torch
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.register import (BatchedRegistration, CONVERGED_LOSS,
                                               default_rates, pose_errors,
                                               register_one_at_a_time)
    from synth import make_phantom, random_poses

    n, steps = 32, 200
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device="cuda")
    det = P.Detector(256, 256, 1.4, 1.4)
    gt = random_poses(n, math.pi / 6, 30.0, 1020.0, seed=11)
    rng = np.random.default_rng(12)
    off = np.zeros((n, 7), np.float32)
    off[:, :3] = rng.uniform(-1, 1, (n, 3)) * math.radians(15.0)
    off[:, 3:6] = rng.uniform(-1, 1, (n, 3)) * 25.0
    targets = P.render(vol, torch.from_numpy(gt).cuda(), det)
    init = torch.from_numpy(gt + off).cuda()
    rates = default_rates(n)
    reg = BatchedRegistration(vol, det, targets, init, rates, steps=steps, use_graph=True)
    reg.run()                                     # capture + first replay
    torch.cuda.synchronize()
    walls = []
    for _ in range(max(args.steps // 4, 3)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        poses, hist = reg.run()
        b.record()
        torch.cuda.synchronize()
        walls.append(a.elapsed_time(b) / 1e3)
    t_batch = float(np.median(walls))
    h = hist.cpu().numpy()
    r_err, t_err = pose_errors(poses.cpu().numpy(), gt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    po, fl = register_one_at_a_time(vol, det, targets, init, rates, steps=steps)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    r1, t1 = pose_errors(po.cpu().numpy(), gt)
    fl = fl.cpu().numpy()
    r0, t0e = pose_errors(gt + off, gt)
    res = {"metric": "batched registration: wall time and final pose error", "mode": "register",
           "problems": n, "steps": steps, "detector": [256, 256],
           "volume": [512, 512, 133], "rates": {"rot": float(rates[0, 0]), "xyz": float(rates[0, 3])},
           "initial_error_mean": {"rot_deg": float(r0.mean()), "trans_mm": float(t0e.mean())},
           "batched_graph": {"wall_s": t_batch, "ms_per_step": 1e3 * t_batch / steps,
                             "fwdbwd_drrs_per_s": n * (steps + 1) / t_batch,
                             "converged": int((h[-1] < CONVERGED_LOSS).sum()),
                             "final_loss_mean": float(h[-1].mean()),
                             "rot_err_deg_median": float(np.median(r_err)),
                             "trans_err_mm_median": float(np.median(t_err)),
                             "rot_err_deg_mean": float(r_err.mean()),
                             "trans_err_mm_mean": float(t_err.mean())},
           "one_at_a_time": {"wall_s": t_one, "converged": int((fl < CONVERGED_LOSS).sum()),
                             "rot_err_deg_median": float(np.median(r1)),
                             "trans_err_mm_median": float(np.median(t1))},
           "speedup": t_one / t_batch, "data": "synthetic"}
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """The request loop over four resident volumes (128^3 at 2 mm, 256^3 at
    1 mm, 512 x 512 x 133, 512 x 512 x 300 at 0.7 x 0.7 x 1.25 mm): requests
    with a random volume, a detector of 128^2 / 200^2 / 256^2 / 512^2 pixels
    (pitch 358.4 mm / N, SDD 1020 mm), a random pose and a 70/30 split of
    forward vs forward + backward (NCC gradient against a target rendered
    near the pose), Poisson arrivals at a sweep of offered rates."""
    import torch
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.serve import (FWD, FWDBWD, GpuBackend, Request, Server,
                                            plain_forward)
    from synth import make_phantom, random_poses

    dev = "cuda"
    names = ["ct128", "ct256", "ct512", "ct512x300"]
    vols = {}
    for nm in names:
        print(f"[bench] phantom {nm}", file=sys.stderr, flush=True)
        ph = make_phantom(nm, seed=0)
        vols[nm] = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=dev)
    sizes = [128, 200, 256, 512]
    rng = np.random.default_rng(7)
    # a pool of targets per (volume, detector) for the forward + backward requests
    pool = {}
    for nm in names:
        for N in sizes:
            gt = random_poses(4, math.pi / 6, 30.0, 1020.0, seed=10 * names.index(nm) + sizes.index(N))
            det = P.Detector(N, N, 358.4 / N, 358.4 / N)
            pool[(nm, N)] = (gt, P.render(vols[nm], torch.from_numpy(gt).to(dev), det))

    def make_requests(count, seed):
        r = np.random.default_rng(seed)
        out = []
        for i in range(count):
            nm = names[int(r.integers(0, 4))]
            N = sizes[int(r.integers(0, 4))]
            if r.uniform() < 0.7:
                pose = random_poses(1, math.pi / 6, 30.0, 1020.0, seed=seed * 100003 + i)[0]
                out.append(Request(nm, N, N, 358.4 / N, 358.4 / N, pose, FWD))
            else:
                gt, tg = pool[(nm, N)]
                k = int(r.integers(0, 4))
                pose = gt[k].copy()
                pose[:3] += r.uniform(-1, 1, 3).astype(np.float32) * 0.05
                pose[3:6] += r.uniform(-1, 1, 3).astype(np.float32) * 5.0
                out.append(Request(nm, N, N, 358.4 / N, 358.4 / N, pose, FWDBWD, tg[k]))
        return out

    budget = 2 << 30

    def run_point(reqs, qps):
        be = GpuBackend(vols, n_streams=3)
        srv = Server(be, hbm_budget_bytes=budget, n_streams=3, max_batch=256)
        if qps is None:
            arrivals = np.zeros(len(reqs))
        else:
            arrivals = np.cumsum(rng.exponential(1.0 / qps, len(reqs)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets, k = [], 0
        while k < len(reqs) or srv.pending():
            now = time.perf_counter() - t0
            while k < len(reqs) and arrivals[k] <= now:
                reqs[k].arrival = t0 + arrivals[k]
                tickets.append(srv.submit(reqs[k]))
                k += 1
            srv.tick()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([t.latency for t in tickets]) * 1e3
        return {"offered_qps": qps, "achieved_rps": len(reqs) / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "batches": srv.batches}

    print("[bench] serving: saturation", file=sys.stderr, flush=True)
    warm = make_requests(200, seed=1)
    run_point(warm, None)
    sat = run_point(make_requests(args.requests, seed=2), None)
    points = []
    for frac in (0.1, 0.3, 0.5, 0.7, 0.9, 1.1):
        q = frac * sat["achieved_rps"]
        print(f"[bench] serving at {q:.0f} req/s", file=sys.stderr, flush=True)
        pt = run_point(make_requests(args.requests, seed=int(100 * frac) + 3), q)
        pt["offered_frac_of_saturation"] = frac
        points.append(pt)
    # plain single-DRR forward path, one request at a time
    reqs = [r for r in make_requests(400, seed=9) if r.kind == FWD]
    lat = []
    for r in reqs:
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain_forward(vols, r)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)
    res = {"metric": "served requests/s and p50/p99 latency (ms), mixed volumes and detectors",
           "mode": "serve", "volumes": names, "detectors": sizes, "fwd_fraction": 0.7,
           "hbm_budget_bytes": budget, "saturation": sat, "sweep": points,
           "plain_single_drr_forward": {"rps": float(1e3 / lat.mean()),
                                        "p50_ms": float(np.percentile(lat, 50)),
                                        "p99_ms": float(np.percentile(lat, 99)),
                                        "requests": len(lat)},
           "data": "synthetic"}
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(poses are independent: the multi-GPU layout replicates the volume and deals "
              "poses out, with no communication)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mode == "register":
        bench_register(args)
        return
    if args.mode == "serve":
        bench_serve(args)
        return

    import torch
    import paper_2208_12737_amd as P
    from synth import make_phantom, random_poses

    dev = torch.device("cuda")
    torch.cuda.set_device(0)
    H = W = 256
    pitch, sdd = 1.4, 1020.0
    nb = args.poses
    print(f"[bench] building 512x512x133 phantom", file=sys.stderr, flush=True)
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=dev)
    det = P.Detector(H, W, pitch, pitch)
    poses_np = random_poses(nb, math.pi / 6, 30.0, sdd, seed=1)
    gt_np = random_poses(nb, math.pi / 6, 30.0, sdd, seed=2)
    poses = torch.from_numpy(poses_np).to(dev)
    gt = torch.from_numpy(gt_np).to(dev)
    # moving poses for fwd+bwd: ground truth plus a seeded offset
    off = np.random.default_rng(3).uniform(-1, 1, (nb, 7)).astype(np.float32)
    off[:, :3] *= math.radians(5.0)
    off[:, 3:6] *= 5.0
    off[:, 6] = 0.0
    moving = torch.from_numpy(gt_np + off).to(dev)
    targets = P.render(vol, gt, det)
    torch.cuda.synchronize()

    # algorithmic work: gathers counted by the renderer's counting mode
    _, cnt = P.render_count(vol, poses, det)
    _, cnt_m = P.render_count(vol, moving, det)
    gathers_fwd = int(cnt.to(torch.int64).sum().item())
    gathers_bwd = int(cnt_m.to(torch.int64).sum().item())
    pixels = nb * H * W
    bytes_fwd = 4 * gathers_fwd + 4 * pixels

    stream = torch.cuda.current_stream()
    img = torch.empty((nb, H, W), dtype=torch.float32, device=dev)
    import paper_2208_12737_amd._lib as L
    ws_n = L.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), nb)
    ws = torch.empty(ws_n, dtype=torch.uint8, device=dev)
    loss = torch.empty((nb,), dtype=torch.float32, device=dev)
    grad = torch.empty((nb, 7), dtype=torch.float32, device=dev)

    from paper_2208_12737_amd.plan import Item, Plan
    items = [Item(0, det, poses[b], img[b]) for b in range(nb)]
    print("[bench] autotuning the batched plan", file=sys.stderr, flush=True)
    plan = Plan([vol], max_items=nb, use_graph=True, autotune=True, tune_items=items,
                cache_path=args.tune_cache or None)
    plan_cfg = plan.config

    def fwd():
        plan.execute(items)

    def direct():
        L.call("drr_render", vol.packed.data_ptr(), ctypes.byref(vol.desc),
               ctypes.byref(det.desc), poses.data_ptr(), nb, img.data_ptr(), None,
               stream.cuda_stream)

    def fwdbwd():
        L.call("drr_render_ncc_grad", vol.packed.data_ptr(), ctypes.byref(vol.desc),
               ctypes.byref(det.desc), moving.data_ptr(), nb, targets.data_ptr(), H * W, None,
               loss.data_ptr(), grad.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)

    phases = [("fwd", fwd), ("fwdbwd", fwdbwd), ("direct", direct)]
    if args.only:
        phases = [p for p in phases if p[0] == args.only]

    for _ in range(args.warmup):
        for _, f in phases:
            f()
    torch.cuda.synchronize()

    ev = {name: [] for name, _ in phases}
    step_ev = []
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for name, f in phases:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            f()
            b.record(stream)
            ev[name].append((a, b))
        s1 = torch.cuda.Event(enable_timing=True)
        s1.record(stream)
        step_ev.append((s0, s1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = {k: np.array([a.elapsed_time(b) for a, b in v]) for k, v in ev.items()}
    step_ms = np.array([a.elapsed_time(b) for a, b in step_ev])

    # single-DRR latency (plain forward path, one pose per launch)
    lat = []
    one = poses[:1].clone()
    img1 = torch.empty((1, H, W), dtype=torch.float32, device=dev)
    for i in range(args.latency_reps + 10 if args.latency_reps > 0 else 0):
        torch.cuda.synchronize()
        t = time.perf_counter()
        L.call("drr_render", vol.packed.data_ptr(), ctypes.byref(vol.desc),
               ctypes.byref(det.desc), one.data_ptr(), 1, img1.data_ptr(), None,
               stream.cuda_stream)
        torch.cuda.synchronize()
        if i >= 10:
            lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)

    res = {"metric": METRIC, "unit": "DRRs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": float(step_ms.mean()),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded ellipsoid phantom, random poses)",
           "config": {"workload": "ct512x512x133_det256_poses256", "volume": [512, 512, 133],
                      "spacing_mm": [0.7, 0.7, 2.5], "detector": [H, W], "pitch_mm": pitch,
                      "sdd_mm": sdd, "poses_per_batch": nb}}
    if "fwd" in times:
        t_fwd = times["fwd"].mean() / 1e3
        res["value"] = nb / t_fwd
        res["fwd_ms_per_batch"] = float(times["fwd"].mean())
        res["gvox_gathers_per_s_fwd"] = gathers_fwd / t_fwd / 1e9
        res["gathers_per_ray_fwd"] = gathers_fwd / pixels
        achieved = bytes_fwd / t_fwd / 1e9
        res["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": profiled_traffic(plan_cfg),
                           "kernel": f"{plan_cfg['strategy']} plan kernel, image mode, tile "
                                     f"code {plan_cfg['tile_code']}, {plan_cfg['wg_per_cu']} WG/CU",
                           "bytes_per_launch": bytes_fwd}
        res["plan"] = plan_cfg
    if "direct" in times:
        t_d = times["direct"].mean() / 1e3
        res["direct_drrs_per_s"] = nb / t_d
        res["direct_ms_per_batch"] = float(times["direct"].mean())
    if "fwdbwd" in times:
        t_fb = times["fwdbwd"].mean() / 1e3
        res["fwdbwd_drrs_per_s"] = nb / t_fb
        res["fwdbwd_ms_per_batch"] = float(times["fwdbwd"].mean())
        res["gvox_gathers_per_s_fwdbwd"] = gathers_bwd / t_fb / 1e9
        if "value" not in res:
            res["value"] = nb / t_fb
    res["p50_ms"] = float(np.percentile(step_ms, 50))
    res["p99_ms"] = float(np.percentile(step_ms, 99))
    if len(lat):
        res["single_drr_latency_ms"] = {"p50": float(np.percentile(lat, 50)),
                                        "p99": float(np.percentile(lat, 99)),
                                        "drrs_per_s": float(1e3 / lat.mean())}
    res["wall_s_timed"] = wall
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(ph, poses_np, H, pitch, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

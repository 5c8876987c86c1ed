"""Benchmark of the FWI-gradient hot path on one MI355X.

One step = one gradient of every medium of the workload: forward solve of
every transmit, misfit, adjoint with imaging, finalisation (the whole path).
Default workload: 64 media of uneven size (side U{256..768}, 8-32 transmits,
2000-5000 steps, h 0.1 mm, dt 20 ns, rod + Gaussian media, FP32), run by the
batched form.  The plain form (one transmit and one step per launch) is timed
beside it on the first media of the same workload.

Prints one JSON line.  Inputs are synthetic and resident in HBM before the
timed region; observed traces come from the forward solve of partner media.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


METRIC = "FWI gradient Gcell-updates/s (fwd+adj), % HBM roofline; batched vs plain"
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
BYTES_PER_UPDATE = 24          # algorithmic bytes per cell-update (48 per forward+adjoint pair)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven64", choices=["uneven64", "rodgauss512", "disc128", "ring188", "unfold16"])
    ap.add_argument("--unfold-k", type=int, default=8, help="unfolded iterations (unfold16)")
    ap.add_argument("--unfold-backprop", default="exact", choices=["none", "fd", "exact"])
    ap.add_argument("--media", type=int, default=64, help="media of the uneven workload (ring188: phantoms, default 1)")
    ap.add_argument("--nt", type=int, default=0, help="override every medium's step count (counter runs)")
    ap.add_argument("--mode", default="batched", choices=["batched", "plain"])
    ap.add_argument("--group", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--spl", type=int, default=0, help="time steps fused per launch (0: library default)")
    ap.add_argument("--order", type=int, default=2, choices=[2, 4], help="spatial order of the operator")
    ap.add_argument("--persistent", type=int, default=0, help="one persistent launch per wave")
    ap.add_argument("--tune", type=int, default=1, help="pick steps per launch and tile rows with the autotuner")
    ap.add_argument("--tune-cache", default="", help="JSON cache file of the autotuner")
    ap.add_argument("--mem-frac", type=float, default=0.85, help="workspace budget as a fraction of free HBM")
    ap.add_argument("--plain-media", type=int, default=64,
                    help="media of the workload timed in plain form (0: skip; all of them by default)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle sample steps (0: sized for ~15 s)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB of one device-to-device copy run first (reference for HBM byte counters)")
    return ap.parse_args()


def build_workload(name, n_media):
    import workloads as W
    if name == "uneven64":
        media = W.c4_batch(40, n_media=n_media)
        desc = (f"uneven{n_media}: {n_media} rod+Gaussian media, side U{{256..768}}, 8-32 transmits, "
                "2000-5000 steps, h 0.1 mm, dt 20 ns, 2.5 MHz Ricker, linear array pitch 0.3 mm")
    elif name == "rodgauss512":
        media = [W.c2_medium(20)]
        desc = "rodgauss512: 512^2, h 0.1 mm, dt 20 ns, 4000 steps, 128 elements, 16 transmits, 2.5 MHz Ricker"
    elif name == "ring188":
        # the paper's acquisition: gradient at the water start model against rod data
        k = n_media if n_media != 64 else 1
        media = [W.ring188(60 + i, rods=False) for i in range(k)]
        desc = (f"ring188 x{k}: 188^2 over 10 cm (h 0.532 mm), dt 90.243 ns, 1034 steps, 16-element ring, "
                "16 transmits, 3 receivers each, 350 kHz Gaussian-derivative pulse; water start model, "
                "observed data from water + rods phantoms")
        return media, [W.ring188(60 + i, rods=True) for i in range(k)], desc
    else:
        media = [W.c1_small()]
        desc = "disc128: 128^2, h 0.2 mm, dt 20 ns, 1000 steps, 32 elements, 1 transmit, 1 MHz Ricker"
    partners = [W.partner_medium(m, 7000 + i) for i, m in enumerate(media)]
    return media, partners, desc


def to_dev(media, dtype, dev):
    import numpy as np
    import torch
    npd = np.float64 if dtype == "f64" else np.float32
    out = []
    for m in media:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, npd)).to(dev)
        out.append({"c": t(m.c), "rho": t(m.rho), "wavelet": t(m.wavelet)})
    return out


def make_plan(media, dtype, mode, args, c_max, forward_only=False):
    import torch
    import paper_2603_04070_amd as F
    grids = [F.GridSpec.of(m.geom, c_max) for m in media]
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return F.Plan(grids, dtype=dtype, mode=mode, ckpt=args.ckpt, group=args.group if mode == "batched" else 0,
                  rows=args.rows if mode == "batched" else 0, use_graph=bool(args.graph) and mode == "batched",
                  steps_per_launch=args.spl if mode == "batched" else 1, forward_only=forward_only,
                  persistent=bool(args.persistent) and mode == "batched" and not forward_only,
                  mem_budget=args.mem_frac * free, order=args.order)


def observed(partners, dtype, args, c_max, dev):
    """Observed traces: forward solve of the partner media (batched form)."""
    import torch
    import paper_2603_04070_amd as F
    plan = make_plan(partners, dtype, "batched", args, c_max, forward_only=True)
    ios = to_dev(partners, dtype, dev)
    outs = F.forward(plan, ios)
    del plan, ios
    torch.cuda.empty_cache()
    return [o["traces"] for o in outs]


def time_gradient(plan, media_dev, d_obs, dtype, steps, warmup, dev):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    ios = []
    for g, m, o in zip(plan.grids, media_dev, d_obs):
        io = dict(m)
        io["d_obs"] = o
        io["traces"] = torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev)
        io["grad_c"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
        io["grad_rho"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
        io["misfit"] = torch.zeros(1, dtype=torch.float64, device=dev)
        ios.append(io)
    ws = plan.new_workspace(dev)
    for _ in range(warmup):
        plan.execute(ios, ws)
    plan.check()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        plan.execute(ios, ws, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plan.check()
    ms = e0.elapsed_time(e1) / steps
    return ms, ios


def run_unfold(args):
    """16 media 512^2, K unfolded iterations of (gradient over 32 transmits,
    4000 steps, FP32) + a random-init 3-layer 3x3 CNN update, forward and
    backward of an MSE loss on C_K."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd.unfold import DUFWI
    dev = torch.device("cuda:0")
    media = [W.c2_medium(5000 + i, n_tx=32) for i in range(16)]
    partners = [W.partner_medium(m, 6000 + i) for i, m in enumerate(media)]
    progress("unfold workload built: 16 media 512^2, 32 transmits")
    if args.nt > 0:
        for m in media + partners:
            m.geom.nt = args.nt
            m.wavelet = m.wavelet[:, :args.nt]
    c_max = 1700.0
    d_obs = observed(partners, "f32", args, c_max, dev)
    progress("observed traces computed")
    grids = [F.GridSpec.of(m.geom, c_max) for m in media]
    torch.manual_seed(0)
    model = DUFWI(grids, K=args.unfold_k, arch="small", hidden=32, physics_backprop=args.unfold_backprop).to(dev)
    progress("unfolded network built")
    keys = ("recompute_updates", "waves", "launches", "max_ckpt", "steps_per_launch", "group")
    progress(f"gradient plan {dict((k, model.plan.info[k]) for k in keys)}")
    if model.hvp_plan is not None:
        progress(f"hvp plan {dict((k, model.hvp_plan.info[k]) for k in keys)}")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    c0 = torch.full((16, 512, 512), 1540.0, device=dev)
    rho = torch.stack([t(m.rho) for m in media])
    wav = [t(m.wavelet) for m in media]
    target = torch.stack([t(m.c) for m in media])
    upd = sum(g.n_tx * g.nx * g.nz * g.nt * 2 for g in grids)
    times = []
    for it in range(args.warmup + args.steps):
        c_in = c0.clone().requires_grad_(args.unfold_backprop != "none")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cK = model(c_in, rho, wav, d_obs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        progress(f"unfold iteration {it}: forward {t1 - t0:.1f} s")
        loss = ((cK - target) ** 2).mean()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        progress(f"unfold iteration {it}: forward {t1 - t0:.1f} s, backward {t2 - t1:.1f} s")
        if it >= args.warmup:
            times.append((t1 - t0, t2 - t1))
    fw = float(np.mean([a for a, _ in times]))
    bw = float(np.mean([b for _, b in times]))
    grads_fw = args.unfold_k
    # backward physics per unfolded iteration: two gradients (fd) or one
    # Hessian-vector product (exact), counted here in gradient-equivalents
    # of useful cell-updates (an HVP advances value and derivative together)
    grads_bw = {"none": 0, "fd": 2, "exact": 1}[args.unfold_backprop] * args.unfold_k
    line = {
        "metric": "DUFWI unfolded forward+backward time", "value": round(fw + bw, 3), "unit": "s",
        "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"unfold16: 16 rod+Gaussian media 512^2, 32 transmits, {grids[0].nt} steps, "
                               f"K={args.unfold_k}, 3-layer 3x3 CNN, physics backprop {args.unfold_backprop}"},
        "forward_s": round(fw, 3), "backward_s": round(bw, 3),
        "gradient_evaluations": grads_fw + grads_bw,
        "physics_gcell_updates_per_s": round(upd * (grads_fw + grads_bw) / (fw + bw) / 1e9, 2),
    }
    print(json.dumps(line))


def main():
    args = parse()
    if args.workload == "unfold16":
        run_unfold(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(multi-GPU sharding is described, not run)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2603_04070_amd as F

    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        n = args.copy_calibration * 2 ** 20 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    dtype = "f64" if args.workload == "disc128" else "f32"
    media, partners, desc = build_workload(args.workload, args.media)
    if args.nt > 0:
        for m in media + partners:
            m.geom.nt = args.nt
            m.wavelet = m.wavelet[:, :args.nt]
        desc += f" [steps overridden to {args.nt}]"
    c_max = 1.02 * max(float(np.max(m.c)) for m in media + partners)
    progress(f"workload built: {desc}")
    d_obs = observed(partners, dtype, args, c_max, dev)
    mdev = to_dev(media, dtype, dev)
    progress("observed traces computed")

    tuned = None
    if args.tune and args.rows == 0 and args.spl == 0:
        grids = [F.GridSpec.of(m.geom, c_max) for m in media]
        t0 = time.perf_counter()
        tuned = F.autotune(grids, dtype=dtype, mode=args.mode, group=args.group, cache=args.tune_cache or None,
                           order=args.order)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
        args.rows, args.spl = tuned["rows"], tuned["steps_per_launch"]
        if args.group == 0:
            args.group = tuned["group"]
        progress(f"autotuned: {tuned}")
    plan = make_plan(media, dtype, args.mode, args, c_max)
    info = plan.info
    progress(f"plan: {info}")
    ms, _ = time_gradient(plan, mdev, d_obs, dtype, args.steps, args.warmup, dev)
    progress(f"timed: {ms:.1f} ms per gradient")
    updates = info["cell_updates"]
    value = updates / (ms * 1e-3) / 1e9
    launches = max(1, info["launches"])
    avg_launch_ms = ms / launches
    alg_bytes_per_launch = updates * BYTES_PER_UPDATE / launches
    achieved = alg_bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    del plan
    torch.cuda.empty_cache()

    # plain form on the first media of the same workload, and the batched form on the same subset
    plain = None
    if args.plain_media > 0 and args.mode == "batched":
        k = min(args.plain_media, len(media))
        sub, sub_dev, sub_obs = media[:k], mdev[:k], d_obs[:k]
        progress(f"plain form on {k} media")
        pp = make_plan(sub, dtype, "plain", args, c_max)
        # one run: the plain form's launches are short and uniform, so a
        # warm-up run changes nothing but the benchmark's length
        pms, _ = time_gradient(pp, sub_dev, sub_obs, dtype, 1, 0, dev)
        pu = pp.info["cell_updates"]
        del pp
        if k == len(media):
            bms = ms                     # the timed batched gradient of the same media
        else:
            bp = make_plan(sub, dtype, "batched", args, c_max)
            bms, _ = time_gradient(bp, sub_dev, sub_obs, dtype, 1, 1, dev)
            del bp
        torch.cuda.empty_cache()
        progress("plain form timed")
        plain = {"value": pu / (pms * 1e-3) / 1e9, "unit": "Gcell-updates/s", "media": k,
                 "ms_per_gradient": round(pms, 1),
                 "batched_same_media": pu / (bms * 1e-3) / 1e9,
                 "speedup_batched_over_plain": pms / bms,
                 "sample": (f"{'all' if k == len(media) else 'first'} {k} medium(s) of the workload, "
                            f"{pu:.3e} cell-updates, one run")}

    cpu = None
    if args.cpu_baseline:
        import oracle
        oracle.use_native()
        cpu = run_cpu_baseline(media, args)
        # the same oracle on one core
        one = run_cpu_baseline(media, args, threads=1, seconds=4.0)
        cpu["single_core"] = {k: one[k] for k in ("value", "cores", "seconds", "runs_s", "sample")}
        progress("oracle baseline timed")

    # the committed counter runs measured the second-order kernels
    traffic = load_traffic(info, launches) if args.order == 2 else None
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": desc,
            "media": len(media),
            "transmits": int(sum(m.geom.n_tx for m in media)),
            "cell_updates_per_step": int(updates),
            "recompute_updates_per_step": int(info["recompute_updates"]),
            "mode": args.mode,
            "order": args.order,
            "group": info["group"], "rows": info["rows"], "waves": info["waves"],
            "steps_per_launch": info["steps_per_launch"],
            "persistent": bool(args.persistent), "graph": bool(args.graph),
            "autotuned": tuned,
            "ckpt_min": info["min_ckpt"], "ckpt_max": info["max_ckpt"],
            "launches_per_step": launches,
            "workspace_gib": round(info["workspace_bytes"] / 2 ** 30, 2),
            "parallelism": "single GPU",
        },
        "hbm_roofline_pct": round(100.0 * value * 1e9 * BYTES_PER_UPDATE / (HBM_PEAK_GBS * 1e9), 2),
        "roofline": {
            "bound": "hbm",
            "kernel": ("step kernels (fwd4x2_kernel, fwd4_kernel, adj4_kernel): 24 B per update each" if args.order == 4 else
                       "step kernels (fwd3_kernel, fwd2_kernel, adj2_kernel, fwd1_kernel, adj1_kernel): "
                       "24 B per update each"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": int(alg_bytes_per_launch),
            "avg_launch_us": round(avg_launch_ms * 1e3, 3),
        },
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(media, args, threads=0, seconds=5.0, reps=3):
    """The oracle (built for this host with -march=native) timed on a bounded
    sample of the workload: one warm-up run, then the median of ``reps``."""
    import numpy as np
    import oracle
    m = media[0]
    g = m.geom
    if threads <= 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    # ~`seconds` per run at the oracle's measured rate (~0.17 G updates/s on
    # one core, ~0.28 on 16: it parallelises rows within a step): as many
    # transmits as the full schedule allows, else the first steps of two
    budget_updates = seconds * (0.17e9 if threads == 1 else 0.28e9)
    ntx = int(min(g.n_tx, max(2, budget_updates // (2 * g.nx * g.nz * g.nt))))
    steps = args.cpu_steps
    if steps <= 0:
        steps = int(max(50, min(g.nt, budget_updates / (2 * g.nx * g.nz * ntx))))
    import copy
    gs = copy.copy(g)
    gs.src = np.asarray(g.src)[:ntx]
    gs.rcv = np.asarray(g.rcv)[:ntx]
    gs.nt = steps
    w = np.asarray(m.wavelet)[:ntx, :steps]
    d_obs = np.zeros((ntx, steps, gs.n_rcv))
    times = []
    for r in range(1 + reps):
        t0 = time.perf_counter()
        oracle.run(gs, m.c, m.rho, w, d_obs=d_obs, threads=threads)
        if r > 0:
            times.append(time.perf_counter() - t0)
    sec = float(np.median(times))
    upd = 2 * g.nx * g.nz * steps * ntx
    return {"value": round(upd / sec / 1e9, 4), "unit": "Gcell-updates/s", "cores": threads, "kind": "oracle",
            "seconds": round(sec, 2), "runs_s": [round(t, 2) for t in times], "warmup_runs": 1,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "build": "gcc -O3 -march=native -fopenmp",
            "sample": (f"medium 0 ({g.nx}x{g.nz}), {ntx} transmits, first {steps} steps, FP64, d_obs = 0; "
                       f"median of {reps} runs after one warm-up")}


def load_traffic(info, launches, path=None):
    """HBM bytes per step-kernel launch: the bytes per executed cell-update
    measured by the committed rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE,
    scaled by a 1 GiB copy) times this workload's executed updates per
    launch; null when the kernel source differs from the one measured or the
    plan fuses a different number of steps or rows per launch."""
    path = path or os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2603_04070_amd", "csrc", "fwi_kernels.hpp"), "rb").read()
    if rec.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    if (rec.get("steps_per_launch"), rec.get("rows")) != (info["steps_per_launch"], info["rows"]):
        return None
    executed = info["cell_updates"] + info["recompute_updates"]
    return int(rec["bytes_per_executed_update"] * executed / launches)


if __name__ == "__main__":
    main()

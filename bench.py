#!/usr/bin/env python3
"""Throughput of the fused forward + backward hot path on one MI355X.

Default workload: one 1200x680 frame (816,000 rays) on the sparse 256^3 room
grid (~10 % of vertices allocated).  One step is the whole hot path over that
batch: the TV gradient written into the zeroed grid gradient, then ray
generation, sampling, gathers, compositing, loss, grid gradient (mapping,
added onto it) and pose gradient (tracking) in one fused launch, and the Adam
pose update.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line: the metric, throughput and step time, the roofline of the
dominant kernel and the FP64 oracle's rate on this host.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# committed FETCH_SIZE / WRITE_SIZE summaries of the fused kernel, by workload
PROFILES_DIR = os.path.join(ROOT, "profiles")
TRAFFIC_PROFILES = {
    "c2_room256_1200x680_mapping": "k_fused_c2_room256_816k_rays_traffic.md",
    "c3_track32_16frames": "k_fused_c3_dense32_16_frames_traffic.md",
    "c4_room512_8x1200x680_mapping": "k_fused_c4_room512_8x816k_rays_traffic.md",
    "c5_room512_64frames_mixed": "k_fused_c5_room512_64_mixed_frames_traffic.md",
}
# the translation unit of the fused kernel: its HBM counters stay valid while
# these files are unchanged
KERNEL_SOURCES = ("paper_2307_03404_amd/csrc/render.hip", "paper_2307_03404_amd/csrc/scatter.hpp",
                  "paper_2307_03404_amd/csrc/kcommon.hpp", "paper_2307_03404_amd/csrc/internal.hpp")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2307_03404_amd import synth
    return {"c1": synth.config1, "c2": synth.config2, "c3": synth.config3,
            "c4": synth.config4, "c5": synth.config5}[name]()


def alg_bytes(stats, n_rays, n_frames, want):
    """Algorithmic bytes of one fused launch (per-ray model, gathers counted
    without cache reuse): 44 B/ray of ray inputs, targets and outputs, 32 B of
    links per occupied sample, 112 B per allocated corner gathered, 224 B per
    gradient corner (read-modify-write of 28 floats) and 24 B per frame."""
    occ, occ_c, grad_c, valid = (int(x) for x in stats)
    b = 44 * n_rays + 32 * occ + 112 * occ_c + 24 * n_frames
    if want & 1:
        b += 224 * grad_c
    return b


def sources_sha256():
    """Digest of the kernel sources: HBM counters are only valid for the code
    they were taken on."""
    import hashlib
    h = hashlib.sha256()
    files = []
    for rel in KERNEL_SOURCES:
        p = os.path.join(ROOT, rel)
        if os.path.isdir(p):
            files += sorted(os.path.join(p, f) for f in os.listdir(p)
                            if f.endswith((".hip", ".hpp", ".h")))
        else:
            files.append(p)
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name, block, variant):
    """HBM bytes per fused launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs (each scaled by the same counter's reading on a copy of known
    size), or None when they were taken on other kernel sources, another
    workload or another launch shape."""
    if workload_name not in TRAFFIC_PROFILES:
        return None
    try:
        with open(os.path.join(PROFILES_DIR, TRAFFIC_PROFILES[workload_name])) as fh:
            kv = dict(m.groups() for m in re.finditer(r"^- (\w+): `([^`]*)`", fh.read(), re.M))
        if (kv.get("sources_sha256") != sources_sha256() or kv.get("workload") != workload_name
                or int(kv.get("block", -1)) != block or int(kv.get("variant", -1)) != variant):
            return None
        return {"bytes": float(kv["traffic_bytes_per_launch"]),
                "read_bytes": float(kv["fetch_kib_per_launch"]) / float(kv["fetch_scale"]) * 1024.0,
                "write_bytes": float(kv["write_kib_per_launch"]) / float(kv["write_scale"]) * 1024.0,
                "kernel_us_profiled": float(kv["kernel_us"]) if "kernel_us" in kv else None}
    except (OSError, KeyError, ValueError):
        return None


def roofline(bytes_alg, bytes_min, kern_ms, traffic, kernel, workload_name):
    """Roofline of the dominant kernel.  `frac` is the HBM-side traffic the
    counters measured (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known
    size; committed per kernel sources) over the live kernel time, against
    the 8 TB/s peak.  The kernel is bound by the latency of its dependent
    gathers at its occupancy, not by a bandwidth: the per-ray byte model
    (every gather counted, cache reuse ignored) is reported as the lane-level
    gather issue rate, which caches serve, and `compulsory_bytes` is a lower
    bound on what any implementation must move (ray inputs and outputs, each
    record that receives a gradient read once and its gradient read and
    written once)."""
    t = kern_ms * 1e-3
    tb = None if traffic is None else traffic["bytes"]
    achieved = None if tb is None else tb / t / 1e9
    return {"bound": "latency", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
            "traffic": tb, "kernel": kernel, "kernel_ms": kern_ms,
            "traffic_read_bytes": None if traffic is None else traffic["read_bytes"],
            "traffic_write_bytes": None if traffic is None else traffic["write_bytes"],
            "compulsory_bytes": bytes_min,
            "traffic_over_compulsory": None if tb is None else tb / bytes_min,
            "gather_issue": {"bytes_per_launch": bytes_alg, "gbs": bytes_alg / t / 1e9,
                             "what": "per-ray byte model, every lane's gathers counted without cache "
                                     "reuse (served by L1/L2/MALL, not HBM)"},
            "evidence": "profiles/" + TRAFFIC_PROFILES.get(workload_name, "")}


def compulsory_bytes(grad_data, n_rays, n_frames, want, rec_bytes):
    """Lower bound on the HBM bytes of one fused launch: 44 B of ray inputs,
    targets and outputs per ray, 24 B per frame and, per record that
    received a grid gradient, the record read once and its gradient read and
    written once."""
    import torch
    touched = 0
    if want & 1:
        touched = int((grad_data != 0).any(dim=1).sum().item())
    return 44 * n_rays + 24 * n_frames + 3 * rec_bytes * touched


def copy_calibration(nbytes=1 << 30, reps=3):
    """Plain device-to-device copies of a known size, for scaling the HBM
    byte counters (run under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}),
          flush=True)


def cache_probe():
    """Streaming-read bandwidth of buffers from L2-resident to HBM-resident
    sizes (pxm_probe_read_bandwidth: each XCD reads its own eighth), the
    cache-level ceilings beside which the fused kernel's traffic is read."""
    import torch
    from paper_2307_03404_amd import pxm
    out = []
    sink = torch.empty(2048 * 256, dtype=torch.float32, device="cuda")
    for mib in (4, 16, 32, 64, 128, 224, 1024, 4096):
        nbytes = mib << 20
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        passes = max(1, int((16 << 30) // nbytes))
        pxm.probe_read_bandwidth(buf, 1, sink)                # warm-up: caches filled
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pxm.probe_read_bandwidth(buf, passes, sink)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out.append({"buffer_mib": mib, "passes": passes, "ms": ms,
                    "read_gbs": nbytes * passes / (ms * 1e-3) / 1e9})
        log(f"read probe {mib} MiB x {passes}: {out[-1]['read_gbs']:.0f} GB/s")
        del buf
    return {"metric": "streaming read bandwidth by buffer size (each XCD reads its own eighth)",
            "unit": "GB/s", "n_gpus": 1, "data": "synthetic", "probe": out}


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(wl, budget_s=15.0, want_grid=True):
    """The FP64 oracle (forward, loss, grid and/or pose backward) on a bounded
    seeded ray sample of the same workload, on this host's cores."""
    import oracle
    from paper_2307_03404_amd import synth
    oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
    probe = synth.subset_rays(wl, 4000, seed=21)
    t0 = time.perf_counter()
    oracle.fused(probe.grid, probe.rays, probe.targets, probe.opts, want_grid=want_grid)
    dt0 = dt = time.perf_counter() - t0
    n = int(min(wl.rays.n_rays, max(4000, 4000 * budget_s / max(dt, 1e-3))))
    sample = synth.subset_rays(wl, n, seed=22)
    t0 = time.perf_counter()
    oracle.fused(sample.grid, sample.rays, sample.targets, sample.opts, want_grid=want_grid)
    dt = time.perf_counter() - t0
    what = "grid+pose" if want_grid else "pose"
    out = {"value": n / dt, "unit": "rays/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{n} of {wl.rays.n_rays} rays (seeded uniform subset), fwd+loss+{what} "
                     f"backward in FP64, {dt:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    # the same oracle on one thread, on a smaller sample of the same workload
    cores = oracle.num_threads()
    oracle.set_threads(1)
    try:
        n1 = int(min(wl.rays.n_rays, max(500, 4000 * (budget_s / 3) / max(dt0 * cores, 1e-3))))
        one = synth.subset_rays(wl, n1, seed=23)
        t0 = time.perf_counter()
        oracle.fused(one.grid, one.rays, one.targets, one.opts, want_grid=want_grid)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    out["single_thread"] = {"value": n1 / dt1, "unit": "rays/s", "cores": 1,
                            "sample": f"{n1} rays (seeded uniform subset), {dt1:.1f} s"}
    return out


def tracking_bench(wl, g, r, trgb, tdep, fw, args):
    """Tracking: `iters` Adam iterations of fused forward + loss + pose
    backward over every frame, captured in one hipGraph; one step = one
    replay.  rays/s counts every ray of every iteration."""
    import torch
    from paper_2307_03404_amd import pxm
    from paper_2307_03404_amd.batch import TrackingGraph
    n, F = wl.rays.n_rays, wl.rays.n_frames
    iters = int(wl.meta.get("iters", 20))
    method = "gauss-newton" if args.gauss_newton else "adam"
    c2w0 = r.c2w.clone()
    tg = TrackingGraph(g, r, wl.opts, trgb, tdep, fw, iters=iters, lr=1e-3, method=method)
    tg.run_eager()                                   # warm-up and lazy set-up outside capture
    torch.cuda.synchronize()
    tg.reset(c2w0)
    tg.capture()
    for _ in range(args.warmup):
        tg.reset(c2w0)
        tg.replay()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tg.reset(c2w0)
        ev[i][0].record()
        tg.replay()
        ev[i][1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    first, last = tg.losses[0].sum().item(), tg.losses[-1].sum().item()
    # the dominant kernel, timed alone on the same stream
    stats = torch.zeros(4, dtype=torch.int64, device=g.data.device)
    loss = torch.zeros(F, dtype=torch.float64, device=g.data.device)
    gp = torch.zeros(F, 6, dtype=torch.float64, device=g.data.device)
    ws = pxm.new_workspace(g, r, wl.opts, pxm.WANT_POSE)
    r.c2w.copy_(c2w0)
    pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, pxm.WANT_POSE | pxm.WANT_STATS, loss=loss,
                     grad_pose=gp, stats=stats, ws=ws)
    torch.cuda.synchronize()
    bytes_launch = alg_bytes(stats.cpu().numpy(), n, F, pxm.WANT_POSE)
    gn = torch.zeros(F, pxm.GN_VALUES, dtype=torch.float64, device=g.data.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        if args.gauss_newton:
            pxm.render_gn(g, r, wl.opts, trgb, tdep, fw, gn=gn)
        else:
            pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, pxm.WANT_POSE, loss=loss,
                             grad_pose=gp, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / 10
    block, variant = pxm.get_tuning()
    kname = ("k_gn<false>" if args.gauss_newton
             else "k_fused<false,true,false,1> + k_fused<false,true,false,2>"
             if variant == 2 else "k_fused<false,true,false,0>")
    traffic = None if args.gauss_newton else measured_traffic(wl.name, block, variant)
    what = ("fwd + residual + 4x6 pose Jacobian + per-frame normal equations + damped "
            "Gauss-Newton step" if args.gauss_newton else "fwd + loss + se(3) pose bwd + Adam")
    out = {
        "metric": f"tracking rays/s ({what}, all frames, {iters} iterations in one hipGraph)",
        "value": n * iters * args.steps / elapsed, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "rays": n, "frames": F, "iters": iters,
                   "grid": list(wl.grid.reso), "step": "one replay of the captured tracking loop",
                   "block": block, "variant": variant},
        "roofline": roofline(bytes_launch, 44 * n + 24 * F, kern_ms, traffic, kname, wl.name),
        "graph_ms_median": graph_ms,
        "loss_first_last_iteration": [first, last],
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget, want_grid=False)
    r.c2w.copy_(c2w0)
    return out


def compare_per_frame(wl, g, r, trgb, tdep, fw, steps, warmup):
    """Batched fused launch over all frames vs. the same work issued frame by
    frame: (a) one fused launch per frame, (b) the unfused kernels per frame
    (forward, loss gradient in torch, grid backward, pose backward)."""
    import torch
    from paper_2307_03404_amd import pxm
    n, F = wl.rays.n_rays, wl.rays.n_frames
    off = wl.rays.frame_offsets
    dev = g.data.device
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device=dev)
    loss = torch.zeros(F, dtype=torch.float64, device=dev)
    want = pxm.WANT_GRID | pxm.WANT_POSE
    frames = []
    for f in range(F):
        a, b = int(off[f]), int(off[f + 1])
        rf = pxm.DeviceRays(r.c2w[f:f + 1], r.intr[f:f + 1],
                            torch.tensor([0, b - a], dtype=torch.int32, device=dev), r.pix[a:b])
        frames.append((a, b, rf))

    def batched():
        pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, want, loss=loss, grad_data=gd, grad_pose=gp)

    def per_frame_fused():
        for f, (a, b, rf) in enumerate(frames):
            pxm.render_fused(g, rf, wl.opts, trgb[a:b], tdep[a:b], fw[f:f + 1], want,
                             loss=loss[f:f + 1], grad_data=gd, grad_pose=gp[f:f + 1])

    lam = float(wl.opts.lambda_depth)

    def per_frame_unfused():
        for f, (a, b, rf) in enumerate(frames):
            rgb, depth, ns = pxm.render_forward(g, rf, wl.opts)
            t = tdep[a:b]
            valid = torch.isfinite(t) & (t > 0)
            g_rgb = torch.where(valid[:, None], 2.0 * fw[f] * (rgb - trgb[a:b]), 0.0).contiguous()
            g_dep = torch.where(valid, lam * fw[f] * torch.sign(depth - torch.where(valid, t, 0.0)),
                                0.0).contiguous()
            pxm.render_backward_grid(g, rf, wl.opts, rgb, depth, ns, g_rgb, g_dep, gd)
            pxm.render_backward_pose(g, rf, wl.opts, rgb, depth, ns, g_rgb, g_dep, gp[f:f + 1])

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tb, tf, tu = timed(batched), timed(per_frame_fused), timed(per_frame_unfused)
    return {"metric": "batched fused fwd+bwd vs per-frame launches (speedup, rays/s ratio)",
            "value": tu / tb, "unit": "x", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": tb * 1e3, "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "rays": n, "frames": F},
            "batched_rays_per_s": n / tb, "per_frame_fused_rays_per_s": n / tf,
            "per_frame_unfused_rays_per_s": n / tu, "speedup_vs_per_frame_fused": tf / tb,
            "speedup_vs_per_frame_unfused": tu / tb}


def grid_edit_bench(args):
    """Dynamic-grid edits on the resident 256^3 room (10 % allocated): prune
    at tau = 0, then grow to 511^3 (link table, then records).  Each launch
    group is bracketed by HIP events on the stream it runs on."""
    import ctypes as C
    import torch
    from paper_2307_03404_amd import pxm, synth
    wl = synth.config2()
    g = pxm.grid_to_device(wl.grid, occupancy=False)
    L = pxm.lib()
    gs = g.struct()
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    ws = pxm.grid_edit_workspace(g)
    Rf = tuple(2 * r - 1 for r in g.reso)
    nc, nf, na = int(np.prod(g.reso)), int(np.prod(Rf)), g.n_alloc
    link_f = torch.empty(nf, dtype=torch.int32, device="cuda")
    n_f = torch.zeros(1, dtype=torch.int64, device="cuda")
    link_p = torch.empty_like(g.link)
    data_p = torch.empty_like(g.data)
    n_p = torch.zeros(1, dtype=torch.int64, device="cuda")
    P = pxm._ptr

    def prune():
        pxm._check("prune", L.pxm_grid_prune(C.byref(gs), 0.0, P(link_p), P(data_p), P(n_p), P(ws),
                                             ws.numel(), sp))

    def grow_link():
        pxm._check("upsample_link", L.pxm_grid_upsample_link(C.byref(gs), P(link_f), P(n_f), P(ws),
                                                             ws.numel(), sp))

    grow_link()
    prune()
    torch.cuda.synchronize()
    n_fine, n_kept = int(n_f.item()), int(n_p.item())
    data_f = torch.empty((n_fine, pxm.REC), dtype=torch.float32, device="cuda")

    def grow_data():
        pxm._check("upsample_data", L.pxm_grid_upsample_data(C.byref(gs), P(link_f), n_fine, P(data_f), sp))

    ops = {"prune": prune, "grow_link": grow_link, "grow_data": grow_data}
    for _ in range(args.warmup):
        for f in ops.values():
            f()
    torch.cuda.synchronize()
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for k in ops}
    t0 = time.perf_counter()
    for i in range(args.steps):
        for k, f in ops.items():
            ev[k][i][0].record(stream)
            f()
            ev[k][i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    # algorithmic bytes: every input read once, every output written once
    alg = {"prune": 4 * nc * 2 + 112 * na + 112 * n_kept,
           "grow_link": 4 * nc + 4 * nf,
           "grow_data": 4 * nf + 4 * nc + 112 * na + 112 * n_fine}
    gbs = {k: alg[k] / (ms[k] * 1e-3) / 1e9 for k in ops}
    total_ms = sum(ms.values())
    achieved = sum(alg.values()) / (total_ms * 1e-3) / 1e9
    return {
        "metric": "dynamic-grid edit: prune + grow 256^3 -> 511^3, fine lattice vertices/s",
        "value": nf * args.steps / elapsed,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 records, f64 interpolation, int32 links",
        "data": "synthetic",
        "config": {"workload": "c2_room256_grid_edit", "grid": list(g.reso), "fine_grid": list(Rf),
                   "allocated_vertices": na, "kept_after_prune": n_kept, "fine_records": n_fine,
                   "step": "prune (tau 0), grow link table, grow records"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "prune + grow_link + grow_data", "kernel_ms": total_ms,
                     "alg_bytes_per_launch": sum(alg.values())},
        "kernels_ms": ms,
        "kernels_gbs": gbs,
        "alg_bytes": alg,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--compare-per-frame", action="store_true",
                    help="time one batched fused launch against per-frame launches instead")
    ap.add_argument("--gauss-newton", action="store_true",
                    help="tracking workloads: Gauss-Newton iterations instead of Adam")
    ap.add_argument("--grid-edit", action="store_true",
                    help="time the dynamic-grid edits (prune, grow 256^3 -> 511^3) instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 1 GiB device copies (for scaling HBM byte counters)")
    ap.add_argument("--cache-probe", action="store_true",
                    help="only measure streaming-read bandwidth from L2- to HBM-resident sizes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_03404_amd import pxm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cache_probe:
        print(json.dumps(cache_probe()), flush=True)
        return
    if args.grid_edit:
        print(json.dumps(grid_edit_bench(args)), flush=True)
        return

    t0 = time.perf_counter()
    wl = workload(args.workload)
    log(f"workload {wl.name}: {wl.rays.n_rays} rays, {wl.rays.n_frames} frames, grid {wl.grid.reso}, "
        f"{wl.grid.n_alloc} allocated vertices (generated in {time.perf_counter() - t0:.1f} s)")
    g = pxm.grid_to_device(wl.grid)
    r = pxm.rays_to_device(wl.rays)
    trgb = torch.from_numpy(wl.targets.rgb).to(dev)
    tdep = torch.from_numpy(wl.targets.depth).to(dev)
    fw = torch.from_numpy(wl.targets.frame_weight).to(dev)
    n, F = wl.rays.n_rays, wl.rays.n_frames
    tracking = wl.meta.get("mode") == "tracking"
    want = pxm.WANT_POSE if tracking else pxm.WANT_GRID | pxm.WANT_POSE
    tv = wl.meta.get("tv", (1e-5, 1e-6, 1e-9))
    tuned_ms = None
    if args.block or args.variant >= 0:
        pxm.set_tuning(args.block or 256, max(args.variant, 0))
    else:
        from paper_2307_03404_amd.batch import Autotuner
        (b_, v_), tuned_ms = Autotuner(None, reps=3, warmup=1).tune(
            g, r, wl.opts, trgb, tdep, fw, want, force=True)
        log("autotuned launch shape: %d rays/workgroup, variant %d (%s)" % (
            b_, v_, ", ".join("%s: %.2f ms" % kv for kv in sorted(tuned_ms.items()))))
    if args.compare_per_frame:
        out = compare_per_frame(wl, g, r, trgb, tdep, fw, args.steps, args.warmup)
        out["config"]["block"], out["config"]["variant"] = pxm.get_tuning()
        print(json.dumps(out), flush=True)
        return
    if tracking:
        out = tracking_bench(wl, g, r, trgb, tdep, fw, args)
        out["autotune_ms"] = tuned_ms
        print(json.dumps(out), flush=True)
        return
    block, variant = pxm.get_tuning()

    rgb = torch.empty(n, 3, device=dev)
    depth = torch.empty(n, device=dev)
    loss = torch.zeros(F, dtype=torch.float64, device=dev)
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device=dev)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    adam_state = torch.zeros(F, 16, dtype=torch.float64, device=dev)
    c2w0 = r.c2w.clone()
    ws = pxm.new_workspace(g, r, wl.opts, want)

    # one untimed pass with traffic counters for the byte model
    pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, want | pxm.WANT_STATS, rgb=rgb, depth=depth,
                     loss=loss, grad_data=gd, grad_pose=gp, stats=stats, ws=ws)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    bytes_launch = alg_bytes(st, n, F, want)
    bytes_min = compulsory_bytes(gd, n, F, want, 4 * gd.shape[1])
    log(f"per ray: {st[0] / n:.2f} occupied samples, {st[1] / n:.2f} corner gathers, "
        f"{st[2] / max(st[3], 1):.2f} gradient corners per valid ray; "
        f"{bytes_launch / n:.0f} algorithmic bytes/ray")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(i=None):
        # the TV term is written into the zeroed gradient first, and the
        # rendering backward adds onto it
        gd.zero_()
        loss.zero_()
        pxm.tv_grad_set(g, tv[0], tv[1], tv[2], gd)
        if i is not None:
            ev[i][0].record()
        pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, want, rgb=rgb, depth=depth, loss=loss,
                         grad_data=gd, grad_pose=gp, ws=ws)
        if i is not None:
            ev[i][1].record()
        pxm.pose_adam(r.c2w, gp, adam_state, 1e-4)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fused_times = [a.elapsed_time(b) for a, b in ev]
    fused_ms = float(np.mean(fused_times))
    r.c2w.copy_(c2w0)

    # separate timing of the TV and pose-update kernels (reported, not used)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        pxm.tv_grad_set(g, tv[0], tv[1], tv[2], gd)
    e1.record()
    torch.cuda.synchronize()
    tv_ms = e0.elapsed_time(e1) / 5

    ms = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    traffic = measured_traffic(wl.name, block, variant)
    kname = ("k_fused<true,true,false,1> + k_fused<true,true,false,2>"
             if variant == 2 else "k_fused<true,true,false,0>")
    out = {
        "metric": "fwd+bwd rays/s (mapping & tracking), 1200x680 rays, 256^3 grid; % of HBM peak",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "rays": n, "frames": F, "grid": list(wl.grid.reso),
                   "allocated_vertices": wl.grid.n_alloc,
                   "step": "TV grad (written), fused fwd+loss+grid+pose bwd (added), Adam pose update",
                   "block": block, "variant": variant},
        "roofline": roofline(bytes_launch, bytes_min, fused_ms, traffic, kname, wl.name),
        "kernels_ms": {"fused": fused_ms, "fused_median": float(np.median(fused_times)), "tv": tv_ms},
        "autotune_ms": tuned_ms,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

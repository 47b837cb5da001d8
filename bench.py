#!/usr/bin/env python3
"""Benchmark of the MI355X Canny edge detector (one GPU).

Headline (the JSON line's `value`): float Canny -- Gaussian sigma=1.4 (7 taps),
Sobel, L2 strength, continuous-direction suppression, thresholds 0.05 / 0.15
of the largest strength, 8-connected hysteresis -- on a 4096x4096 fp32 image,
in MPix/s.  One step = one full pass of the operator over one image.  Inputs
are seeded synthetic images (value-noise shading + 40 step-edged shapes +
noise, see workloads.py) already resident in HBM; the step rotates through
enough distinct input/output buffers (>= 1 GiB, 4x the 256 MB Infinity Cache)
that no step finds its input there, so every step streams from HBM.  The
line also gives per-step percentiles of the same steps and, labelled as such,
the rate with one buffer set reused (cache-warm).

Also reported (under "configs"): the integer pipeline at 4096^2 and on the
16384^2 hysteresis stress image, the float pipeline at 7680x4320, the batched
uneven-size plan against a per-image loop, the differentiable front end
forward + backward, and the Laplacian zero-crossing detector at 4096^2.  `roofline` describes the dominant kernel of the headline
step (the float walk: blur, Sobel, strength, suppression), timed with HIP
events that the library records around it on the step's stream;
`cpu_baseline` is the C oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# non-packed fp32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-ops/s)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
MALL_BYTES = 256 << 20


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps  # ms per call


def n_rot(bytes_per_set):
    """Distinct buffer sets to rotate through: >= 1 GiB in total, 4x the
    Infinity Cache, so that no step finds its input there."""
    return max(2, -(-4 * MALL_BYTES // max(bytes_per_set, 1)))


def step_percentiles(fn, steps, stream):
    """p10 / p50 / p90 of single-step device times (one event pair per step)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in evs)
    pick = lambda q: round(t[min(len(t) - 1, int(q * len(t)))], 4)
    return {"p10": pick(0.1), "p50": pick(0.5), "p90": pick(0.9)}


def bench_f32(canny, torch, H, W, steps, warmup, seed, sector=False):
    import numpy as np
    import workloads
    X = workloads.natural_u8(H, W, seed=seed).astype(np.float32)
    k = n_rot(H * W * 5)
    xs = [torch.from_numpy(X).cuda() for _ in range(k)]
    es = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(k)]
    ws = torch.empty(canny.f32_workspace_bytes(H, W), dtype=torch.uint8, device="cuda")
    it = [0]

    def step():
        i = it[0] % k
        it[0] += 1
        if sector:  # four-sector direction, absolute thresholds near 0.05 / 0.15 of the max
            canny.canny_f32_sector(xs[i], 1.4, 3, 16.0, 48.0, edges=es[i], workspace=ws)
        else:
            canny.canny_f32(xs[i], 1.4, 3, 0.05, 0.15, True, edges=es[i], workspace=ws)

    st = torch.cuda.current_stream()
    ms = timed(step, steps, warmup, st)
    if not sector and (H, W) == (4096, 4096):
        pct = step_percentiles(step, steps, st)  # rotating buffers, per step
        warm = timed(lambda: canny.canny_f32(xs[0], 1.4, 3, 0.05, 0.15, True, edges=es[0],
                                             workspace=ws), steps, warmup, st)
        return ({"ms": ms, "mpix_s": H * W / (ms * 1e-3) / 1e6, "rot_buffers": k,
                 "step_ms_percentiles": pct,
                 "warm_same_buffer_mpix_s": round(H * W / (warm * 1e-3) / 1e6, 1)}, (xs, es, ws))
    return {"ms": ms, "mpix_s": H * W / (ms * 1e-3) / 1e6, "rot_buffers": k}, (xs, es, ws)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "f32_walk_4096_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "f32_walk_4096_valu.txt")


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy GB/s (bytes read + written) on the same GPU: what
    a plain streaming kernel reaches, next to the 8 TB/s peak."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    ms = timed(lambda: dst.copy_(src), reps, 3, st)
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def roofline_headline(canny, torch, bufs, H, W, steps):
    """Per-stage device time of the headline step, from HIP events the library
    records on the step's stream around each stage (a second pass over the
    same rotating buffers, after the timed one).  The dominant kernel is the
    float walk (Gaussian, Sobel, strength, suppression); its algorithmic bytes
    are the float forward's 4 B/px in + 0.25 B/px of class map out."""
    from paper_1710_07745_amd.profiling import WALK_KERNEL, read_traffic, read_valu
    xs, es, ws = bufs
    k = len(xs)
    with canny.StageTiming(steps) as t:
        for i in range(steps):
            canny.canny_f32(xs[i % k], 1.4, 3, 0.05, 0.15, True, edges=es[i % k], workspace=ws)
        torch.cuda.synchronize()
        us = {}
        for name in ("f32_clear", "f32_walk", "f32_classify", "hysteresis"):
            ms, n = t.read(name)
            us[name] = round(ms * 1e3 / max(n, 1), 2)
    alg = H * W * (4 + 0.25)
    walk_s = us["f32_walk"] * 1e-6
    gbs = alg / walk_s / 1e9
    fwd_s = (us["f32_clear"] + us["f32_walk"] + us["f32_classify"]) * 1e-6
    valu_insts = read_valu(VALU_FILE)  # wave instructions per launch (x 64 lanes)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": read_traffic(TRAFFIC_FILE),
            "kernel": WALK_KERNEL + " (float walk: blur, Sobel, strength, "
                      "suppression; 4096x4096)",
            "bytes_per_launch": alg, "avg_launch_us": us["f32_walk"],
            "stage_avg_us": us,
            "forward_frac": round(alg / fwd_s / 1e9 / HBM_PEAK_GBS, 4),
            "valu_insts_per_launch": valu_insts,
            "valu_frac": None if valu_insts is None else
            round(valu_insts * 64 / walk_s / VALU_PEAK_LANE_OPS, 4),
            # Step 4's three passes (local, merge, resolve) together,
            # on their algorithmic 0.25 B/px of class map in + 1 B/px of
            # edges out; on this path the local pass reads the 4 B/px signed
            # strength map instead of a class map (measured traffic in
            # profiles/f32_4096_traffic.txt)
            "hysteresis": {"bytes_per_launch": H * W * 1.25, "avg_us": us["hysteresis"],
                           "achieved_gbs": round(H * W * 1.25 / (us["hysteresis"] * 1e-6) / 1e9, 1),
                           "frac": round(H * W * 1.25 / (us["hysteresis"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}


def bench_u8(canny, torch, img, steps, warmup, label):
    H, W = img.shape
    k = n_rot(H * W * 2)
    xs = [torch.from_numpy(img).cuda() for _ in range(k)]
    es = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(k)]
    ws = torch.empty(canny.u8_workspace_bytes(H, W), dtype=torch.uint8, device="cuda")
    it = [0]

    def full():
        i = it[0] % k
        it[0] += 1
        canny.canny_u8(xs[i], 40, 100, edges=es[i], workspace=ws)

    def fwd():
        i = it[0] % k
        it[0] += 1
        canny.canny_u8(xs[i], 40, 100, with_edges=False, workspace=ws)

    st = torch.cuda.current_stream()
    ms = timed(full, steps, warmup, st)
    msf = timed(fwd, steps, warmup, st)
    out = {"workload": label, "ms": round(ms, 4), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1),
           "forward_ms": round(msf, 4),
           "forward_mpix_s": round(H * W / (msf * 1e-3) / 1e6, 1),
           "forward_hbm_frac": round(H * W * 1.25 / (msf * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del xs, es, ws
    torch.cuda.empty_cache()
    return out


def bench_log(canny, torch, steps, warmup):
    """Laplacian zero-crossing detector (binomial blur, 5-point Laplacian,
    zero crossings with slope >= 10) on the 4096^2 uint8 scene: one kernel,
    1 B/px in + 1 B/px out."""
    import workloads
    H = W = 4096
    img = workloads.natural_u8(H, W, seed=10)
    k = n_rot(H * W * 2)
    xs = [torch.from_numpy(img).cuda() for _ in range(k)]
    es = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(k)]
    it = [0]

    def step():
        i = it[0] % k
        it[0] += 1
        canny.canny_log_u8(xs[i], 10, edges=es[i])

    ms = timed(step, steps, warmup, torch.cuda.current_stream())
    edge_frac = float((es[0] > 0).float().mean())
    del xs, es
    torch.cuda.empty_cache()
    return {"workload": "Laplacian zero-crossing detector (5x5 binomial, 5-point Laplacian, "
                        "slope threshold 10), 4096x4096 uint8",
            "ms": round(ms, 4), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1),
            "hbm_frac": round(H * W * 2.0 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "edge_fraction": round(edge_frac, 4)}


def bench_mag(canny, torch, steps, warmup):
    """Differentiable front end: 32 images of 1024x1024 in [0, 1], sigma ~ U[1, 3],
    radius 9; the loss gradient dM = 2 (M - T), T the magnitude at sigma = 2, is
    formed once outside the timed region.  One step = forward + backward."""
    import numpy as np
    import workloads
    N, H, W, R = 32, 1024, 1024, 9
    I = torch.from_numpy(np.stack([workloads.natural_unit_f32(H, W, seed=2000 + i)
                                   for i in range(N)])).cuda()
    sig = torch.from_numpy(workloads.sigma_init(N, seed=4)).cuda()
    T = canny.mag_forward(I, torch.full_like(sig, 2.0), R)
    gM = 2.0 * (canny.mag_forward(I, sig, R) - T)
    M = torch.empty_like(I)
    st = torch.cuda.current_stream()
    fwd = timed(lambda: canny.mag_forward(I, sig, R), steps, warmup, st)
    bwd = timed(lambda: canny.mag_backward(I, sig, gM, R), steps, warmup, st)
    both = timed(lambda: (canny.mag_forward(I, sig, R), canny.mag_backward(I, sig, gM, R)),
                 steps, warmup, st)
    px = N * H * W
    del I, T, gM, M
    torch.cuda.empty_cache()
    return {"workload": "differentiable front end, 32 x 1024x1024 fp32, radius 9",
            "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4), "fwd_bwd_ms": round(both, 4),
            "fwd_mpix_s": round(px / (fwd * 1e-3) / 1e6, 1),
            "bwd_mpix_s": round(px / (bwd * 1e-3) / 1e6, 1),
            "fwd_bwd_mpix_s": round(px / (both * 1e-3) / 1e6, 1),
            "fwd_bwd_hbm_frac": round(px * 20 / (both * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_batch(canny, torch, steps, warmup):
    """256 uint8 images, H ~ U{240..2160}, W ~ U{320..3840}: one replay of the
    autotuned batch plan (one HIP graph) against a host loop of canny_u8 over
    the same images on one stream."""
    import workloads
    shapes = workloads.batch_shapes(256, seed=3)
    dev = [torch.from_numpy(workloads.natural_u8(h, w, seed=1000 + i)).cuda()
           for i, (h, w) in enumerate(shapes)]
    outs = [torch.empty((h, w), dtype=torch.uint8, device="cuda") for h, w in shapes]
    plan = canny.BatchPlan(shapes, 40, 100, autotune=True)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    nb = max(3, steps // 5)
    t_graph = timed(lambda: plan.run(dev, outs, ws), nb, max(1, warmup // 5), st)
    hmax = max(h for h, _ in shapes)
    wmax = max(w for _, w in shapes)
    ws1 = torch.empty(canny.u8_workspace_bytes(hmax, wmax), dtype=torch.uint8, device="cuda")

    def loop():
        for x, e in zip(dev, outs):
            canny.canny_u8(x, 40, 100, edges=e, workspace=ws1)

    t_loop = timed(loop, nb, max(1, warmup // 5), st)
    px = sum(h * w for h, w in shapes)
    info = plan.info()
    plan.close()
    del dev, outs, ws, ws1
    torch.cuda.empty_cache()
    return {"workload": "batched integer Canny, 256 uneven uint8 images (%.0f MPix)" % (px / 1e6),
            "graph_ms": round(t_graph, 4), "loop_ms": round(t_loop, 4),
            "graph_mpix_s": round(px / (t_graph * 1e-3) / 1e6, 1),
            "loop_mpix_s": round(px / (t_loop * 1e-3) / 1e6, 1),
            "speedup_vs_loop": round(t_loop / t_graph, 3), "tuned": info}


def bench_video(canny, torch, steps, warmup):
    """Streaming integer Canny on host frames (PCIe-inclusive): pinned 4K and
    8K uint8 frames pushed through canny_video_* with a 3-slot ring (uploads,
    detection and downloads overlapped) and with one slot (each frame's
    upload waits for the previous download), timed on the host from the
    first push to the final sync."""
    import workloads
    out = {}
    for label, (H, W), n in (("4k", (2160, 3840), max(40, 2 * steps)),
                             ("8k", (4320, 7680), max(20, steps))):
        frames = [torch.from_numpy(workloads.natural_u8(H, W, seed=900 + i)).pin_memory()
                  for i in range(4)]
        outs = [torch.empty((H, W), dtype=torch.uint8).pin_memory() for _ in range(4)]
        res, push_us = {}, {}
        for depth in (3, 1):
            vs = canny.VideoStream(H, W, 40, 100, depth=depth)
            for i in range(4):
                vs.push(frames[i], outs[i])
            vs.sync()
            t0 = time.perf_counter()
            t_push = 0.0
            for i in range(n):
                tp = time.perf_counter()
                vs.push(frames[i % 4], outs[i % 4])
                t_push += time.perf_counter() - tp
            vs.sync()
            dt = time.perf_counter() - t0
            vs.close()
            res[depth] = n / dt
            push_us[depth] = t_push / n * 1e6
        # the link alone: one frame up and one down per step, each direction
        # timed on its own (pinned buffers), the slower sets the streaming bound
        d = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        st = torch.cuda.current_stream()
        up = timed(lambda: d.copy_(frames[0], non_blocking=True), 10, 2, st)
        down = timed(lambda: outs[0].copy_(d, non_blocking=True), 10, 2, st)
        del d
        out[label] = {"frames": n, "shape": [H, W], "fps": round(res[3], 1),
                      "mpix_s": round(res[3] * H * W / 1e6, 1),
                      "fps_serialized": round(res[1], 1),
                      "overlap_speedup": round(res[3] / res[1], 3),
                      "host_push_us_per_frame": round(push_us[3], 1),
                      "h2d_ms": round(up, 4), "d2h_ms": round(down, 4),
                      "fps_link_bound": round(1e3 / max(up, down), 1)}
        del frames, outs
    out["workload"] = ("streaming integer Canny from pinned host frames to host edge maps "
                       "(PCIe-inclusive), 3-slot ring vs 1 slot")
    return out


def cpu_baseline(seconds=10.0):
    import numpy as np
    import oracle
    import workloads
    X = workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)
    oracle.canny_f32(X)  # warm caches / page in
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.canny_f32(X)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": round(n * 4096 * 4096 / dt / 1e6, 2), "unit": "MPix/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} runs of the fp64 float Canny oracle (single thread) on the 4096x4096 "
                      f"benchmark image, {dt:.1f} s"}


def cpu_paper_design(reps=3):
    """The float operator on the host in the paper's own design: Steps 1-3 as
    row-parallel loops, hysteresis serial (oracle/paper_design.c).  Measures
    the parallel fraction f at one thread and the speedup on all threads the
    box grants, and evaluates Amdahl's law and the paper's asymmetric-multicore
    form 1 / ((1-f)/perf(r) + f/(perf(r)+n-r)) with perf(r) = sqrt(r) (the
    paper does not define perf; sqrt is the usual assumption for that form)."""
    import math
    import numpy as np
    import oracle
    import workloads
    X = workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)
    n = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16)))
    oracle.paper_design_canny_f32(X, n)  # page in

    def best(threads, k):
        runs = [oracle.paper_design_canny_f32(X, threads)[1:] for _ in range(k)]
        return min(runs, key=lambda t: t[0] + t[1])

    p1, s1 = best(1, 1)
    pn, sn = best(n, reps)
    f = p1 / (p1 + s1)
    asym = {}
    for r in (1, 4, 16):
        if r <= n:
            perf = math.sqrt(r)
            asym[f"r{r}"] = round(1.0 / ((1.0 - f) / perf + f / (perf + n - r)), 2)
    return {"unit": "MPix/s", "threads": n, "image": "4096x4096 float, sigma 1.4, radius 3, "
            "relative thresholds 0.05/0.15 (the headline workload)",
            "mpix_s_1thread": round(4096 * 4096 / (p1 + s1) / 1e6, 2),
            "mpix_s": round(4096 * 4096 / (pn + sn) / 1e6, 2),
            "ms_parallel_part": [round(p1 * 1e3, 1), round(pn * 1e3, 1)],
            "ms_serial_part": [round(s1 * 1e3, 1), round(sn * 1e3, 1)],
            "parallel_fraction_f": round(f, 4),
            "speedup_measured": round((p1 + s1) / (pn + sn), 2),
            "speedup_amdahl": round(1.0 / ((1.0 - f) + f / n), 2),
            "speedup_asymmetric_sqrt_perf": asym}


def profile_workload(canny, torch, what, steps):
    """A few calls of one workload on one buffer set, then a 256 MiB device
    copy (the calibration kernel of the traffic counters).  Each workload runs
    alone so that per-kernel counter medians never mix workloads."""
    import numpy as np
    import workloads
    dev = "cuda"
    if what == "f32_4096":
        X = torch.from_numpy(workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)).to(dev)
        E = torch.empty((4096, 4096), dtype=torch.uint8, device=dev)
        ws = torch.empty(canny.f32_workspace_bytes(4096, 4096), dtype=torch.uint8, device=dev)
        for _ in range(steps):
            canny.canny_f32(X, 1.4, 3, 0.05, 0.15, True, edges=E, workspace=ws)
    elif what in ("u8_4096", "u8_16384_spiral"):
        img = (workloads.natural_u8(4096, 4096, seed=10) if what == "u8_4096"
               else workloads.spiral_u8(16384, seed=5))
        X = torch.from_numpy(img).to(dev)
        E = torch.empty_like(X)
        ws = torch.empty(canny.u8_workspace_bytes(*img.shape), dtype=torch.uint8, device=dev)
        for _ in range(steps):
            canny.canny_u8(X, 40, 100, edges=E, workspace=ws)
    elif what == "log_4096":
        X = torch.from_numpy(workloads.natural_u8(4096, 4096, seed=10)).to(dev)
        E = torch.empty_like(X)
        for _ in range(steps):
            canny.canny_log_u8(X, 10, edges=E)
    elif what == "mag_32x1024":
        N, H, W, R = 32, 1024, 1024, 9
        I = torch.from_numpy(np.stack([workloads.natural_unit_f32(H, W, seed=2000 + i)
                                       for i in range(N)])).to(dev)
        sig = torch.from_numpy(workloads.sigma_init(N, seed=4)).to(dev)
        gM = torch.ones_like(I)
        for _ in range(steps):
            canny.mag_forward(I, sig, R)
            canny.mag_backward(I, sig, gM, R)
    elif what == "batch_256":
        shapes = workloads.batch_shapes(256, seed=3)
        xs = [torch.from_numpy(workloads.natural_u8(h, w, seed=1000 + i)).to(dev)
              for i, (h, w) in enumerate(shapes)]
        outs = [torch.empty((h, w), dtype=torch.uint8, device=dev) for h, w in shapes]
        plan = canny.BatchPlan(shapes, 40, 100, autotune=False)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        for _ in range(steps):
            plan.run(xs, outs, ws)
        torch.cuda.synchronize()
        plan.close()
    src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile": what, "steps": steps, "copy_bytes": 256 << 20}), flush=True)


PROFILE_WORKLOADS = ("f32_4096", "u8_4096", "u8_16384_spiral", "log_4096", "mag_32x1024", "batch_256")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-roofline", action="store_true",
                    help="only the headline step (float Canny, 4096^2, one buffer set) and a "
                         "256 MiB device copy, for hardware-counter runs")
    ap.add_argument("--profile", choices=sorted(PROFILE_WORKLOADS),
                    help="only --steps runs of one workload (one buffer set) and a 256 MiB "
                         "device copy, for per-kernel counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_07745_amd as canny
    torch.cuda.set_device(0)

    if args.profile:
        profile_workload(canny, torch, args.profile, args.steps)
        return

    if args.profile_roofline:
        import numpy as np
        import workloads
        X = torch.from_numpy(workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)).cuda()
        E = torch.empty((4096, 4096), dtype=torch.uint8, device="cuda")
        ws = torch.empty(canny.f32_workspace_bytes(4096, 4096), dtype=torch.uint8, device="cuda")
        for _ in range(args.steps):
            canny.canny_f32(X, 1.4, 3, 0.05, 0.15, True, edges=E, workspace=ws)
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_roofline": "done", "copy_bytes": 256 << 20,
                          "kernel_bytes": 4096 * 4096 * 4.25}), flush=True)
        return

    log("headline: float Canny 4096x4096")
    head, bufs = bench_f32(canny, torch, 4096, 4096, args.steps, args.warmup, seed=1)
    roof = roofline_headline(canny, torch, bufs, 4096, 4096, args.steps)
    del bufs
    torch.cuda.empty_cache()
    roof["copy_gbs"] = copy_bandwidth(torch)

    configs = {}
    if not args.no_extra:
        import workloads
        log("u8 4096x4096")
        configs["u8_4096"] = bench_u8(canny, torch, workloads.natural_u8(4096, 4096, seed=10),
                                      args.steps, args.warmup, "integer Canny, 4096x4096 uint8")
        log("f32 7680x4320")
        r, b = bench_f32(canny, torch, 4320, 7680, args.steps, args.warmup, seed=2)
        del b
        torch.cuda.empty_cache()
        configs["f32_7680x4320"] = {"workload": "float Canny, 7680x4320 fp32",
                                    "ms": round(r["ms"], 4), "mpix_s": round(r["mpix_s"], 1)}
        log("f32 four-sector 4096x4096")
        r, b = bench_f32(canny, torch, 4096, 4096, args.steps, args.warmup, seed=1, sector=True)
        del b
        torch.cuda.empty_cache()
        configs["f32_sector_4096"] = {"workload": "float Canny, four-sector direction, absolute "
                                                  "thresholds 16/48, 4096x4096 fp32",
                                      "ms": round(r["ms"], 4), "mpix_s": round(r["mpix_s"], 1)}
        log("u8 16384x16384 spiral")
        configs["u8_16384_spiral"] = bench_u8(canny, torch, workloads.spiral_u8(16384, seed=5),
                                              max(3, args.steps // 5), 2,
                                              "integer Canny, 16384x16384 spiral stress image")
        for name, fn in (("log_u8_4096", "bench_log"), ("batch_256_uneven", "bench_batch"),
                         ("mag_fwd_bwd_32x1024", "bench_mag"), ("video_u8", "bench_video")):
            f = globals().get(fn)
            if f is not None:
                log(name)
                configs[name] = f(canny, torch, args.steps, args.warmup)

    cpu = None if args.no_cpu else cpu_baseline()
    cpu_pd = None
    if cpu is not None:
        log("cpu paper-design baseline")
        cpu_pd = cpu_paper_design()
    line = {
        "metric": "Canny MPix/s at 4096² & batched uneven sizes; % HBM roofline; fwd+bwd MPix/s",
        "value": round(head["mpix_s"], 1),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "float Canny (sigma 1.4, 7 taps, L2, interpolated NMS, relative "
                               "thresholds 0.05/0.15, hysteresis), one 4096x4096 fp32 image per step",
                   "image": [4096, 4096], "rotating_buffers": head["rot_buffers"]},
        "step_ms_percentiles": head.get("step_ms_percentiles"),
        "warm_same_buffer_mpix_s": head.get("warm_same_buffer_mpix_s"),
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_paper_design": cpu_pd,
        "configs": configs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

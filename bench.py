"""Benchmark of the rasterizer training step on one MI355X.

One step = the whole hot path over one batch of views, inputs resident in HBM:
gs_preprocess -> gs_bin_sort -> gs_render_fwd -> gs_loss -> gs_render_bwd_adam
(the backward with the Adam step applied as each Gaussian's gradient is formed;
the same bits as gs_render_bwd followed by gs_adam_step).  Default workload: 1M Gaussians (SH degree 3) and 9 views (the
newest pose of a seeded random-walk camera path plus its 8 neighbours by frustum
overlap) at 3x 1600x1067, 3x 1296x864, 3x 979x546, loss 0.8 L1 + 0.2 D-SSIM,
per-view learning rates from Eq. 6-7.  Prints one JSON line (rank 0).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload c3|c2|c1|c4] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X fp32 vector, packed FMA: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2 x 2.4 GHz
FP32_NONPACKED_PEAK_TFLOPS = 78.6  # the same without packed issue (the build disables packed fp32)


def eq6_lr(iters, eta0=1.6e-4, etaf=1.6e-6, t_a=30000.0):
    """Per-image learning rate of Eq. 6-7 (log-linear in trained iterations)."""
    t = min(iters / t_a, 1.0)
    return math.exp(math.log(eta0) * (1.0 - t) + math.log(etaf) * t)


def make_workload(name):
    import scenegen
    if name == "c3":
        return scenegen.config3()
    if name == "c2":
        return scenegen.config2()
    if name == "c1":
        return scenegen.config1()
    if name == "c4":
        return scenegen.config4()
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(n, n_p, V, K, P, tiles, ssim, K_eff=0):
    """Compulsory HBM bytes per stage: each input read once, each output written
    once; K = the (tile, Gaussian) pairs that belong to a tile's list, K_eff = those
    some pixel of the tile blends (the backward adds their 9 partial gradients into
    the Gaussian's sums: 36 B each)."""
    return {
        "preprocess": 4 * n_p * n + 64 * V * n,
        "scan_emit": 8 * V * n + 12 * K,
        "tile_sort": 24 * K,
        "ranges": 8 * K + 8 * tiles,
        "render_fwd": 52 * K + 20 * P,
        "loss": (72 if ssim else 36) * P,
        "render_bwd": 52 * K + 24 * P + 36 * K_eff,
        "preprocess_bwd": 36 * V * n + 8 * n_p * n,
        "adam": 28 * n_p * n + 8 * n,
        # grad2d and visibility per (view, Gaussian); params, m, v read and written; step
        "preprocess_bwd_adam": 40 * V * n + 24 * n_p * n + 8 * n,
    }


# Flops per pixel-Gaussian evaluation (add, mul, compare, min, exp2, reciprocal = 1;
# fma = 2).  The method's work per pixel is E, the Gaussians that pass its cutoff
# test before it stops (the blended ones and the one that stops it; counted by
# gs_render_count, independent of the tile edge): each takes the cutoff test,
# centre offset (2), base-2 exponent (3 mul + 2 fma = 7), two comparisons (2) = 11.
# A blended Gaussian adds, in the forward, exp2, opacity product, clamp, 1 - alpha,
# transmittance product, stop test, weight and three colour fmas = 13; in the
# backward, exp2, opacity product, clamp, 1 - alpha, reciprocal, transmittance
# recovery, weight, the alpha derivative over three channels (15), cap select,
# exponent derivative, six moment/opacity products, three colour products, three
# suffix-colour fmas (6) and the nine sums over pixels = 48.  List positions a
# kernel walks without the Gaussian passing (up to each pixel's last blended
# position) are reported beside it as "visits": work of the tiling, not of the method.
TEST_FLOPS = 11
FWD_BLEND_FLOPS = 13
BWD_BLEND_FLOPS = 48


def raster_flops(evals, blends):
    """Algorithmic flops of one forward and one backward raster launch."""
    return {"render_fwd": TEST_FLOPS * evals + FWD_BLEND_FLOPS * blends,
            "render_bwd": TEST_FLOPS * evals + BWD_BLEND_FLOPS * blends}


def probe_rates(dev):
    """Achievable rates on this GPU from the library's probes: a streaming copy of
    1 GiB (bytes read + written per second, best of 5) and fp32 FMA chains (flops
    per second, best of 3), each timed with HIP events on the stream it runs on."""
    import torch
    from paper_2503_13086_amd import gs_probe_copy, gs_probe_fma
    stream = torch.cuda.current_stream(dev)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    nbytes = src.numel() * 4
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        gs_probe_copy(src, dst, nbytes, stream)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    assert torch.equal(src[:1024], dst[:1024]) and torch.equal(src[-1024:], dst[-1024:])
    copy_gbs = 2 * nbytes / (best * 1e-3) / 1e9
    del src, dst
    blocks, iters = 256 * 32, 4096
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    best = float("inf")
    flops = 0
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        flops = gs_probe_fma(out, blocks, iters, stream)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    assert bool(torch.isfinite(out).all())
    return copy_gbs, flops / (best * 1e-3) / 1e12


KERNEL_SOURCE = {"render_fwd": "k_raster.hip", "render_bwd": "k_raster.hip", "preprocess": "k_preprocess.hip",
                 "preprocess_bwd": "k_preprocess.hip", "tile_sort": "k_sort.hip", "depth_sort": "k_sort.hip",
                 "emit": "k_sort.hip", "loss": "k_loss.hip", "adam": "k_adam.hip",
                 "preprocess_bwd_adam": "k_preprocess.hip"}


def traffic_for(kernel, workload):
    """HBM bytes per launch of `kernel` measured with the FETCH_SIZE and WRITE_SIZE
    counters (profiles/<kernel>_traffic_<workload>.json), or None when there is no
    such record or the kernel's source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_{workload}.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCE:
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2503_13086_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("source_sha256"):
            return None
    return rec.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scene, budget_s=15.0):
    """The FP64 oracle, as it is, on the host's cores: (1) a bounded sample of the
    benchmark workload, forward and backward of random pixels of its first view
    (every visible Gaussian evaluated per pixel) plus one projection of the whole
    field; (2) the whole 10k-Gaussian 128x128 workload, forward and backward of
    every pixel (L1 loss gradient)."""
    import torch
    import oracle
    import scenegen
    from oracle import composite
    from oracle.geometry import params_f64, project_view
    cam = scene.cams[0]
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    P = params_f64(scene.params, scene.n, requires_grad=True)
    proj = project_view(P, cam, scene.sh_degree, 16)
    t_proj = time.perf_counter() - t0
    ids = composite.ordered_visible(proj)
    sel = composite.select(proj, ids, requires_grad=True)
    leaves = {k: sel[k].detach().clone().requires_grad_(True) for k in ("u", "w", "a", "b", "c", "o", "rgb")}
    q = {k: v.detach() for k, v in sel.items()}
    gq = dict(leaves)
    gq["tau"] = q["tau"]
    n_pix = 0
    t1 = time.perf_counter()
    chunk = 4
    while time.perf_counter() - t1 < budget_s and n_pix < 4096:
        px = rng.integers(0, cam["width"], chunk)
        py = rng.integers(0, cam["height"], chunk)
        r = composite.blend(q, px, py, margins=False, grad_q=gq)
        (r["C"].sum() + r["T_final"].sum()).backward()
        n_pix += chunk
    outs = [sel[k] for k in leaves if leaves[k].grad is not None]
    grads = [leaves[k].grad for k in leaves if leaves[k].grad is not None]
    torch.autograd.backward(outs, grads)
    t_total = time.perf_counter() - t1 + t_proj
    # the whole small workload
    c1 = scenegen.config1()
    t2 = time.perf_counter()
    projs = oracle.project_views(c1.params, c1.n, c1.sh_degree, c1.cams)
    img = composite.render_view(projs[0], margins=False)["color"]
    up = [(np.sign(img - c1.targets[0]) / img.size).astype(np.float32)]
    oracle.param_grads(c1.params, c1.n, c1.sh_degree, c1.cams, up)
    t_c1 = time.perf_counter() - t2
    px_c1 = c1.cams[0]["width"] * c1.cams[0]["height"]
    return {"value": n_pix / t_total / 1e6, "unit": "Mpix/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"{n_pix} random pixels of view 0 ({cam['width']}x{cam['height']}), FP64 forward + "
                      f"autograd backward over all {len(ids)} visible Gaussians, including one projection of "
                      f"all {scene.n} Gaussians; {t_total:.1f} s",
            "small_workload_full": {"workload": c1.name, "pixels": px_c1, "seconds": round(t_c1, 2),
                                    "mpix_s": px_c1 / t_c1 / 1e6,
                                    "what": "FP64 projection, forward of every pixel and autograd backward of "
                                            "the L1 loss gradient"}}


def serving_leg(n_arrivals, time_scale, slots, autotune=True):
    """The on-the-fly stream served twice on fresh fields: the plain loop (one job
    at a time, one view per step) and continuous batching (up to `slots` jobs per
    step).  Targets and new Gaussians are resident on the device before timing."""
    import torch
    import scenegen
    from paper_2503_13086_amd.serving import Engine, Field
    t = time.perf_counter()
    st = scenegen.serving_stream(n_arrivals=n_arrivals)
    dev = torch.device("cuda", 0)
    targets = [torch.as_tensor(a.target()).reshape(-1).to(dev) for a in st.arrivals]
    for a in st.arrivals:
        a.block = torch.as_tensor(a.block).to(dev)
    print(f"[bench] serving stream {st.name}: {n_arrivals} arrivals, prepared in {time.perf_counter() - t:.1f}s",
          file=sys.stderr, flush=True)
    out = {"workload": st.name, "arrivals": n_arrivals, "iterations_per_arrival": 200,
           "time_scale": time_scale, "stream_mean_interarrival_s": 2.0, "mean_interarrival_s": 2.0 * time_scale,
           "initial_gaussians": int(st.initial.shape[1]),
           "loss": "Eq. 10: 0.47 L1 + 0.12 D-SSIM + 0.41 load balance (Eq. 9)", "lr": "Eq. 6-8, T_a = 200"}
    from paper_2503_13086_amd.autotune import Autotuner
    for name, s in (("plain_loop", 1), ("continuous_batching", slots)):
        fld = Field(st.initial, st.sh_degree, capacity=st.initial.shape[1])
        tuner = Autotuner(coarse=True) if autotune else None
        eng = Engine(fld, max_slots=s, t_i=200, seed=5, w_l1=0.47, w_dssim=0.12, w_load=0.41, autotuner=tuner)
        t = time.perf_counter()
        done = [0]

        def progress(job, name=name, t0=t):
            done[0] += 1
            if done[0] % 20 == 0:
                print(f"[bench] serving {name}: {done[0]}/{n_arrivals} arrivals done "
                      f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)

        stats = eng.run(st.arrivals, targets, time_scale=time_scale, on_job_done=progress)
        eng.close()
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.summary().items()}
        out[name]["tiles_chosen"] = ({f"n<=2^{k[0]}": t for k, t in sorted(tuner.table.items())} if tuner
                                     else "16 (fixed)")
        print(f"[bench] serving {name}: {json.dumps(out[name])} ({time.perf_counter() - t:.1f}s)", file=sys.stderr,
              flush=True)
        del fld, eng
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-loop", action="store_true")
    ap.add_argument("--serve-arrivals", type=int, default=200,
                    help="arrivals of the serving stream (0 skips the serving leg)")
    ap.add_argument("--serve-time-scale", type=float, default=0.1,
                    help="arrival times (Poisson, mean gap 2 s) are multiplied by this factor")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-autotune", action="store_true",
                    help="let the serving engine autotune the tile edge per field-size bucket")
    ap.add_argument("--serve-only", action="store_true",
                    help="run the serving leg alone (no training-step figures; prints {\"serving\": ...})")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls only (by default the step is also captured into a HIP graph and "
                         "replayed, and the replay rate is the reported value)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size kernel that calibrates "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU split of this path "
              "is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(max(args.serve_arrivals, 1), args.serve_time_scale,
                                                 args.serve_slots, autotune=args.serve_autotune)}), flush=True)
        return

    import torch
    from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device, DEFAULT_LR, n_params

    t_gen = time.perf_counter()
    sc = make_workload(args.workload)
    print(f"[bench] workload {sc.name}: n={sc.n}, views={len(sc.cams)}, generated in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    V = len(sc.cams)
    iters = sc.iters if sc.iters is not None else np.zeros(V, np.int64)
    lrs = [eq6_lr(float(it)) for it in iters]
    scales = [lr / DEFAULT_LR[0] for lr in lrs]

    rz = Rasterizer(0)
    dev = rz.device
    params = params_to_device(sc.params)
    n, D = sc.n, sc.sh_degree
    rz.set_views(sc.cams)
    target = rz.pack_images(sc.targets)
    loss = torch.zeros(V, dtype=torch.float64, device=dev)
    grad = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    step = torch.zeros(n, dtype=torch.int32, device=dev)

    from paper_2503_13086_amd.autotune import Autotuner
    tuner = Autotuner()
    tile = tuner.choose(rz, params, n, D, sc.cams, target, sc.w_l1, sc.w_dssim)
    tune_ms = tuner.last_timings(n, D, sc.cams)
    print(f"[bench] autotuned tile {tile}: " + ", ".join(f"{t}: {ms:.3f} ms" for t, ms in tune_ms.items()),
          file=sys.stderr, flush=True)
    P = rz.P
    color = rz.new_image()
    dl = rz.new_image()

    def one_step(count=False):
        rz.preprocess(params, n, D, sc.cams)
        rz.bin_sort(count=count)     # count False: K stays on the device, no host wait
        rz.render_fwd(color)
        rz.loss(color, target, sc.w_l1, sc.w_dssim, loss, dl)
        rz.render_bwd_adam(dl, m, v, step, DEFAULT_LR, scales, group_mask=1)

    for i in range(args.warmup):
        one_step(count=i == 0)
    torch.cuda.synchronize()
    rz.sync_status()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    rz.preprocess(params, n, D, sc.cams)
    K = rz.bin_sort(count=True)
    rz.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    rz.sync_status()      # raises if a binning in the timed steps ran out of room
    prof = rz.profile_read()
    rz.profile(False)
    t_eager = t_step

    # the same step captured once into a HIP graph and replayed (no launch or
    # host overhead between its kernels); every buffer was sized by the eager steps
    t_graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            one_step()
        for _ in range(2):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        t_graph = (time.perf_counter() - t0) / args.steps
        rz.sync_status()
        del graph
        t_step = min(t_step, t_graph)
    kern_ms = {k: (ms / cnt if cnt else 0.0) for k, (cnt, ms) in prof.items()}
    kern_launches = {k: cnt for k, (cnt, ms) in prof.items()}
    fwd_bwd_ms = sum(kern_ms[k] * kern_launches[k] / args.steps for k in
                     ["preprocess", "depth_sort", "scan", "emit", "tile_sort", "ranges", "render_fwd", "loss", "zero",
                      "render_bwd", "preprocess_bwd_adam"])

    # per-pixel work of the method, from the last timed step's forward state: the
    # Gaussians each pixel evaluated up to termination and those it blended; beside
    # them the list positions the kernels walked (up to each pixel's last blend)
    from paper_2503_13086_amd import (GS_BUF_LAST, GS_BUF_N_CONTRIB, GS_BUF_RANGES, GS_BUF_EVALS, GS_BUF_PAIRS_EFF,
                                      gs_render_count)
    gs_render_count(rz.ctx)
    evals = int(rz.buffer(GS_BUF_EVALS).to(torch.int64).sum().item())
    k_eff = int(rz.buffer(GS_BUF_PAIRS_EFF).to(torch.int64).sum().item())
    visits = int(rz.buffer(GS_BUF_LAST).to(torch.int64).sum().item())
    blends = int(rz.buffer(GS_BUF_N_CONTRIB).to(torch.int64).sum().item())
    rg = rz.buffer(GS_BUF_RANGES).view(-1, 2).to(torch.int64)
    K_valid = int((rg[:, 1] - rg[:, 0]).sum().item())      # pairs in some tile's list

    # plain loop: each view on its own call sequence, gradients summed, one Adam step
    plain_ms = None
    if not args.no_plain_loop and V > 1:
        def plain_step():
            for vi, c in enumerate(sc.cams):
                rz.preprocess(params, n, D, [c])
                rz.bin_sort(count=False)
                col = rz.render_fwd(color[: 3 * c["width"] * c["height"]])
                rz.loss(col, target[3 * rz_off[vi]: 3 * rz_off[vi + 1]], sc.w_l1, sc.w_dssim, loss[:1],
                        dl[: 3 * c["width"] * c["height"]])
                rz.render_bwd(dl[: 3 * c["width"] * c["height"]], grad, accumulate=vi > 0)
            rz.adam_step(grad, m, v, step, DEFAULT_LR, None, group_mask=1)
        from paper_2503_13086_amd import gs_layout
        rz_off, _ = gs_layout(sc.cams, tile)
        for _ in range(2):
            plain_step()
        torch.cuda.synchronize()
        rz.sync_status()
        t0 = time.perf_counter()
        reps = max(2, args.steps // 4)
        for _ in range(reps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) / reps * 1e3
        rz.sync_status()

    n_p = n_params(D)
    rz.set_views(sc.cams)
    n_tiles = rz.tile_off[-1]
    algo = algorithmic_bytes(n, n_p, V, K_valid, P, n_tiles, sc.w_dssim != 0, k_eff)
    # dominant kernel and its roofline
    dom = max(["render_fwd", "render_bwd", "preprocess", "tile_sort", "depth_sort", "preprocess_bwd_adam", "loss",
               "emit"], key=lambda k: kern_ms[k] * kern_launches[k])
    copy_gbs, fma_tflops = probe_rates(dev)
    if dom in ("render_bwd", "render_fwd"):
        flops = raster_flops(evals, blends)[dom]
        achieved = flops / (kern_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic_for(dom, args.workload), "kernel": dom,
                "kernel_ms": kern_ms[dom], "algorithmic_flops": flops,
                "flop_model": f"{TEST_FLOPS} x evals + {BWD_BLEND_FLOPS if dom == 'render_bwd' else FWD_BLEND_FLOPS}"
                              f" x blends",
                "peak_nonpacked": FP32_NONPACKED_PEAK_TFLOPS, "frac_nonpacked": achieved / FP32_NONPACKED_PEAK_TFLOPS,
                "measured_fma_tflops": round(fma_tflops, 2), "frac_of_measured_fma": achieved / fma_tflops}
    else:
        key = {"tile_sort": "tile_sort", "depth_sort": "tile_sort", "emit": "scan_emit"}.get(dom, dom)
        achieved = algo[key] / (kern_ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom, args.workload), "kernel": dom,
                "kernel_ms": kern_ms[dom]}

    fb_stages = ["preprocess", "scan_emit", "tile_sort", "ranges", "render_fwd", "loss", "render_bwd",
                 "preprocess_bwd_adam"]
    fb_gbs = sum(algo[k] for k in fb_stages) / (fwd_bwd_ms * 1e-3) / 1e9

    mpix = P / (t_step) / 1e6
    line = {
        "metric": "fwd+bwd Mpix/s at 1M Gaussians vs plain loop; p50/p99 per-new-image latency",
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "step_mode": "hip_graph_replay" if t_graph is not None and t_graph <= t_eager else "eager_calls",
        "eager_ms_per_step": round(t_eager * 1e3, 4),
        "graph_ms_per_step": round(t_graph * 1e3, 4) if t_graph is not None else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "gaussians": n, "sh_degree": D, "views": V,
                   "resolutions": [f"{c['width']}x{c['height']}" for c in sc.cams], "pixels": P,
                   "loss": f"{sc.w_l1} L1 + {sc.w_dssim} D-SSIM", "tile": tile, "pairs": K,
                   "pairs_in_tiles": K_valid,
                   "autotune_fwd_bwd_ms": {str(t): round(ms, 4) for t, ms in tune_ms.items()}},
        "fwd_bwd_mpix_s": round(P / (fwd_bwd_ms * 1e-3) / 1e6, 3),
        "plain_loop_mpix_s": round(P / (plain_ms * 1e-3) / 1e6, 3) if plain_ms else None,
        "plain_loop_ms_per_step": round(plain_ms, 3) if plain_ms else None,
        "kernel_ms_per_step": {k: round(kern_ms[k] * kern_launches[k] / args.steps, 4) for k in kern_ms},
        "algorithmic_gb_per_step": {k: round(b / 1e9, 4) for k, b in algo.items()},
        "fwd_bwd_algorithmic_gbs": round(fb_gbs, 1),
        "achievable_hbm_gbs": round(copy_gbs, 1),
        "fwd_bwd_frac_of_achievable_hbm": round(fb_gbs / copy_gbs, 4),
        "evals": evals,
        "pairs_blended": k_eff,
        "blends": blends,
        "visits": visits,
        "measured_fma_tflops": round(fma_tflops, 2),
        "roofline": roof,
    }
    if args.serve_arrivals > 0:
        rz.close()
        line["serving"] = serving_leg(args.serve_arrivals, args.serve_time_scale, args.serve_slots,
                                      autotune=args.serve_autotune)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(sc)
    rz.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Frame-rate benchmark of the render path on one MI355X.

Workload: 1M Gaussians (64-cluster mixture, SH degree 3, log-scale N(ln 0.01, 0.7),
opacity sigmoid(N(0, 1.5))) rendered at 1920x1080 along a 200-pose orbit of the
radius-4 sphere, 1x1 tile grouping.  One step = one frame of the whole path on the
resident scene: preprocess + count scan, binning + radix sort + ranges, rasterize.

The chosen form (FP16 MFMA power, hi/lo splits) is timed, then the plain FP32
rasterizer on the same poses.  The JSON line carries both rates, per-frame p50/p99,
the raster kernel's ALU roofline (HIP events on the launch stream), the PSNR of the
chosen form against the FP64 oracle on sampled tiles, the oracle's own rate on
the host cores, and a serving run (8 resident scenes, mixed resolutions, continuous
batching; p50/p99 latency of an open-loop Poisson stream) under "serving".

With --scene dense6m the same legs run on the dense stress scene (6M Gaussians, log-scale
N(ln 0.05, 0.5), opacity sigmoid(N(-1, 1))) along its own 200-pose orbit, e.g. with --group 4.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-serve]
       python bench.py --scene dense6m --group 4 [...]
       python bench.py --serve-only [--serve-requests R] [--serve-load F]
       python bench.py --sweep [--sweep-steps K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s @1080p 1M Gaussians: MFMA-FP16 vs FP32 plain at PSNR≥45dB; p99 ms"
# Per Gaussian-pixel evaluation: power as 6 multiply-adds (12 flops), alpha = o exp(power)
# (2); per blended pair: 1 - alpha, T (1 - alpha), alpha T, 3 colour FMAs (9).
FLOPS_PER_EVAL = 14
FLOPS_PER_BLEND = 9
PEAK_FP32_TFLOPS = 157.3   # 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # the same without packed FP32 (which this build does not emit)
PEAK_FP16_MFMA_TFLOPS = 2500.0      # dense FP16 / BF16 matrix peak
POWER_FLOPS = 12                    # the power's 6 multiply-adds, moved onto the matrix cores

# Counters of one launch of the rasterizer on this workload (FP16, splits 2, 1x1 groups), from
# rocprofv3: FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by what the same counters read
# for a plain device copy of known size (x2 and x1); the wave-level VALU instruction count
# (SQ_INSTS_VALU) and the SIMD cycles spent on VALU instructions (SQ_ACTIVE_INST_VALU, in units
# of 4 cycles, summed over the SIMDs).  They describe the kernel built from the source and
# compiler flags hashed in `sha256`; after any change to either they are reported as null.
RASTER_COUNTERS = dict(sha256="97c7411ab9156cc5cc8b8d5597cdbef1983b75d60f013d73bf4da0f983cfc227",
                       fetch_kib=65246, write_kib=25081, fetch_scale=2.0, write_scale=1.0,
                       insts_valu=34.77e6, active_valu_quads=38.46e6,
                       precision="fp16", splits=2, group=1, scene="clustered1m")
SIMDS = 1024                # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9
VALU_CYCLES = 4             # a wave64 VALU instruction on a 16-lane SIMD


def raster_source_hash():
    import hashlib
    from paper_2605_17855_amd import build
    h = hashlib.sha256()
    for part in (("paper_2605_17855_amd", "csrc", "gs_raster_mfma.hip"), ("paper_2605_17855_amd", "csrc", "gs_mfma.hpp"),
                 ("paper_2605_17855_amd", "csrc", "gs_internal.hpp"), ("include", "gs.h")):
        with open(os.path.join(ROOT, *part), "rb") as f:
            h.update(f.read())
    h.update(" ".join(f for f in build.FLAGS if not os.path.isabs(f)).encode())
    return h.hexdigest()


def raster_counters(args):
    """The stored counters when they describe this kernel and workload, else None."""
    c = RASTER_COUNTERS
    if (args.precision, args.splits, args.group, args.scene) != (c["precision"], c["splits"], c["group"], c["scene"]):
        return None
    try:
        if raster_source_hash() != c["sha256"]:
            return None
    except OSError:          # sources not shipped beside the library
        return None
    return c


def raster_traffic(args):
    """Measured HBM bytes per launch, or None when they do not describe this kernel and workload."""
    c = raster_counters(args)
    if c is None:
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def valu_fracs(args, launch_s):
    """Shares of the chip's SIMD cycles over one launch: (issue, active).  issue counts every VALU
    wave instruction as 4 cycles; active is the counted cycles the SIMDs spent on VALU
    instructions (slower transcendentals included).  (None, None) without stored counters."""
    c = raster_counters(args)
    if c is None or launch_s <= 0:
        return None, None
    simd_cycles = SIMDS * launch_s * CLOCK_HZ
    return VALU_CYCLES * c["insts_valu"] / simd_cycles, 4.0 * c["active_valu_quads"] / simd_cycles


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp16", choices=["fp16", "bf16", "fp32"])
    ap.add_argument("--splits", type=int, default=2)
    ap.add_argument("--group", type=int, default=1)
    ap.add_argument("--scene", default="clustered1m", choices=["clustered1m", "dense6m"],
                    help="the 1M-Gaussian scene, or the dense 6M-Gaussian stress scene")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tight", action="store_true", help="skip the opacity-aware tile culling variant")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 plain comparison run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle compositing time")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward-pass timing")
    ap.add_argument("--no-pipelined", action="store_true", help="skip the two-frames-in-flight rate")
    ap.add_argument("--no-device-counts", action="store_true",
                    help="skip the frames without the host wait (eager and graph-replayed)")
    ap.add_argument("--no-all-rows", action="store_true",
                    help="skip the MFMA run without quadrant culling (its launches share the kernel's name)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving workload")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-load", type=float, default=0.7, help="offered rate / saturated throughput")
    ap.add_argument("--serve-pool-gib", type=float, default=4.0)
    ap.add_argument("--sweep", action="store_true",
                    help="only the sensitivity sweep: 3M at 1080p/2160p and dense 6M, groups 1/2/4, all precisions")
    ap.add_argument("--sweep-steps", type=int, default=30)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times), for HBM counter calibration")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain copy of known size: FETCH_SIZE / WRITE_SIZE of its dispatches give the counters' scale."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 4, "dispatches": 5}), flush=True)


def timed_frames(gs, torch, ds, cams, rend, opt, steps, warmup):
    """Returns (elapsed s, per-frame ms list, per-frame raster-kernel ms list).

    The throughput loop records no event inside the frames: an event recorded into the stream
    costs the GPU about 5 us (its release writes the caches back), as much as a small kernel.
    The same frames then run twice more: with an event before and after each frame (latency:
    p50, p99) and with events between the three calls (stage times, raster time)."""
    st = torch.cuda.current_stream()

    def frame(cam, ev):
        gs.gs_preprocess(ds, cam, opt, rend.proj, rend.ws)
        if ev is not None and ev[3] is not None:
            ev[3].record(st)
        gs.gs_bin_sort(rend.proj, cam, opt, rend.bins, rend.ws)
        if ev is not None and ev[1] is not None:
            ev[1].record(st)
        gs.gs_rasterize(rend.proj, rend.bins, cam, opt, rend.image)
        if ev is not None:
            ev[2].record(st)

    # make sure the entry buffers are large enough for every pose (grows outside the timed region)
    for cam in cams[:max(steps, warmup, 1)]:
        rend.render(ds, cam, opt)
    for i in range(warmup):
        frame(cams[i % len(cams)], None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        frame(cams[i % len(cams)], None)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    def marked(stages):
        evs = [[torch.cuda.Event(enable_timing=True) if (k in (0, 2) or stages) else None for k in range(4)]
               for _ in range(steps)]
        for i in range(steps):
            evs[i][0].record(st)
            frame(cams[i % len(cams)], evs[i])
        torch.cuda.synchronize()
        return evs

    evs = marked(False)
    frame_ms = [e[0].elapsed_time(e[2]) for e in evs]
    evs = marked(True)
    raster_ms = [e[1].elapsed_time(e[2]) for e in evs]
    timed_frames.stages = {"preprocess_ms": float(np.mean([e[0].elapsed_time(e[3]) for e in evs])),
                           "bin_sort_ms": float(np.mean([e[3].elapsed_time(e[1]) for e in evs])),
                           "rasterize_ms": float(np.mean(raster_ms))}
    return elapsed, frame_ms, raster_ms


def pipelined_frames(gs, torch, ds, cams, n, opt, steps, warmup, inflight=2):
    """Frames/s with `inflight` frames of the orbit in flight at once: frame i runs on stream
    i % inflight with its own buffers, so one frame's latency-bound sort overlaps another's
    rasterization (each frame is still the whole path, and the host still waits once per frame
    for its entry count)."""
    streams = [torch.cuda.Stream() for _ in range(inflight)]
    rends = [gs.Renderer(n, 1920, 1080, group=opt.group) for _ in range(inflight)]
    for k in range(inflight):
        with torch.cuda.stream(streams[k]):
            for cam in cams[:max(steps, warmup, 1)]:
                rends[k].render(ds, cam, opt, stream=streams[k])
    torch.cuda.synchronize()

    def frame(i):
        k = i % inflight
        st = streams[k]
        cam = cams[i % len(cams)]
        gs.gs_preprocess(ds, cam, opt, rends[k].proj, rends[k].ws, stream=st)
        gs.gs_bin_sort(rends[k].proj, cam, opt, rends[k].bins, rends[k].ws, stream=st)
        gs.gs_rasterize(rends[k].proj, rends[k].bins, cam, opt, rends[k].image, stream=st)

    for i in range(warmup):
        frame(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        frame(i)
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0)


def device_count_frames(gs, torch, ds, cams, n, capacity, opt_kwargs, steps, warmup, ref_image):
    """Frames/s of the frame without the host wait (GS_OPT_DEVICE_COUNTS: the bin sort reads its
    counts on the device, grids sized for `capacity`), run eagerly and replayed from captured
    HIP graphs: one graph per pose (the camera is a kernel argument), all over the same buffers.
    `capacity` holds every pose's entries; the replay of pose 0 is compared with `ref_image`, the
    frame that waits for its counts."""
    opt = gs.options(device_counts=True, **opt_kwargs)
    rend = gs.Renderer(n, 1920, 1080, group=opt.group, capacity=capacity)

    def frame(cam):
        gs.gs_preprocess(ds, cam, opt, rend.proj, rend.ws)
        gs.gs_bin_sort(rend.proj, cam, opt, rend.bins, rend.ws)
        gs.gs_rasterize(rend.proj, rend.bins, cam, opt, rend.image)

    for i in range(warmup):
        frame(cams[i % len(cams)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        frame(cams[i % len(cams)])
    torch.cuda.synchronize()
    eager = steps / (time.perf_counter() - t0)
    poses = min(steps, len(cams))
    graphs = []
    for i in range(poses):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            frame(cams[i])
        graphs.append(g)
    torch.cuda.synchronize()
    graphs[0].replay()
    torch.cuda.synchronize()
    same = bool(ref_image is not None and np.array_equal(rend.image.double().cpu().numpy(), ref_image))
    fits = gs.entry_count(rend.proj) <= capacity
    for i in range(warmup):
        graphs[i % poses].replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        graphs[i % poses].replay()
    torch.cuda.synchronize()
    replay = steps / (time.perf_counter() - t0)
    return {"option": "GS_OPT_DEVICE_COUNTS", "capacity": capacity, "eager_frames_per_s": eager,
            "graph_frames_per_s": replay, "graphs": poses, "pose0_image_equals_host_count_frame": same,
            "last_frame_fits_capacity": bool(fits)}


def work_units(gs, torch, ds, cams, rend, opt_kwargs, steps):
    """Gaussian-pixel evaluations and blended pairs of the timed frames (aux pass, untimed)."""
    opt = gs.options(aux_flags=gs.GS_AUX_NEVAL | gs.GS_AUX_NBLEND, **opt_kwargs)
    e_pix = blend = entries = visible = e_tile = e_wave = 0
    seen = {}
    for i in range(steps):
        k = i % len(cams)
        if k not in seen:
            n_keys = rend.render(ds, cams[k], opt)
            torch.cuda.synchronize()
            a = rend.aux.double()
            ne = a[0]
            # what a tile-synchronous (256 pixels) and a wave-synchronous (8x8) kernel execute:
            # every pixel of the unit runs as many evaluations as its longest pixel
            h, w = ne.shape
            pad = torch.zeros(((h + 15) // 16 * 16, (w + 15) // 16 * 16), dtype=ne.dtype, device=ne.device)
            pad[:h, :w] = ne
            tile_max = pad.view(pad.shape[0] // 16, 16, pad.shape[1] // 16, 16).amax(dim=(1, 3))
            wave_max = pad.view(pad.shape[0] // 8, 8, pad.shape[1] // 8, 8).amax(dim=(1, 3))
            seen[k] = (int(ne.sum().item()), int(a[1].sum().item()), n_keys,
                       int(rend.proj.n_visible.cpu().item()), int(tile_max.sum().item()) * 256,
                       int(wave_max.sum().item()) * 64)
        e_pix += seen[k][0]
        blend += seen[k][1]
        entries += seen[k][2]
        visible += seen[k][3]
        e_tile += seen[k][4]
        e_wave += seen[k][5]
    work_units.executed = {"e_tile": e_tile, "e_wave": e_wave}
    return e_pix, blend, entries / steps, visible / steps


def cpu_baseline_and_psnr(gs, torch, sc, cam, image_gpu, target_s):
    from oracle import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    rec = oracle.preprocess(sc, cam)
    st, ids, _ = oracle.lists(rec, cam, 1)
    amb = oracle.ambiguous_membership(rec, cam)
    t_pre = time.perf_counter() - t0
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    ntiles = tx * ty
    rng = np.random.default_rng(7)
    order = rng.permutation(ntiles)
    # calibrate the tile sample so the compositing takes about target_s
    t1 = time.perf_counter()
    probe = np.sort(order[:64])
    oracle.composite(rec, cam, st, ids, nthreads=threads, tiles=probe, amb=amb)
    per_tile = (time.perf_counter() - t1) / len(probe)
    nsel = int(min(ntiles, max(64, target_s / max(per_tile, 1e-6))))
    sel = np.sort(order[:nsel])
    t2 = time.perf_counter()
    ref = oracle.composite(rec, cam, st, ids, nthreads=threads, tiles=sel, amb=amb)
    t_comp = time.perf_counter() - t2
    frame_s = t_pre + t_comp * ntiles / nsel
    # one thread on a sample of tiles, extrapolated
    one = np.sort(order[:min(ntiles, 256)])
    t3 = time.perf_counter()
    oracle.composite(rec, cam, st, ids, nthreads=1, tiles=one, amb=amb)
    single_s = t_pre + (time.perf_counter() - t3) * ntiles / len(one)
    mask = np.zeros((cam.height, cam.width), bool)
    for t in sel:
        x, y = (t % tx) * 16, (t // tx) * 16
        mask[y:y + 16, x:x + 16] = True
    a = np.clip(image_gpu[:, mask], 0, 1)
    b = np.clip(ref["image"][:, mask], 0, 1)
    mse = float(np.mean((a - b) ** 2))
    psnr = float("inf") if mse == 0 else 10 * np.log10(1 / mse)
    mae = float(np.mean(np.abs(image_gpu[:, mask] - ref["image"][:, mask])))
    ok = mask & (ref["ambiguous"] == 0)
    quality = {"psnr_db": psnr, "mae": mae, "max_abs": float(np.abs(image_gpu[:, ok] - ref["image"][:, ok]).max()),
               "ambiguous_pixel_frac": float(1.0 - ok.sum() / max(mask.sum(), 1)), "tiles": int(nsel)}
    base = {"value": 1.0 / frame_s, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle on the first pose: preprocess + tile lists of all {sc.n} Gaussians "
                       f"({t_pre:.1f} s, 1 thread), compositing of {nsel} of {ntiles} random tiles "
                       f"({t_comp:.1f} s, {threads} threads), extrapolated to the full frame"),
            "single_thread_s_per_frame": single_s, "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}
    return base, quality


def quality_over_poses(gs, torch, sc, cams, rend, opt, steps, tiles_per_pose=96, max_poses=50):
    """Image quality of the chosen form against the FP64 oracle on every timed pose (at most
    max_poses, evenly spaced when there are more): per pose, a seeded sample of tiles is
    composited by the oracle and compared with the GPU image of that pose.  PSNR and MAE over
    all sampled pixels; max abs over those whose decisions lie outside the guard bands; the
    flagged ones are checked against the oracle's admissible results (oracle.check_flagged)."""
    from oracle import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    n_timed = min(steps, len(cams))
    poses = np.unique(np.linspace(0, n_timed - 1, min(n_timed, max_poses)).round().astype(int))
    sq = ab = npx = 0.0
    mx = 0.0
    flagged = matched = failed = unresolved = 0
    tx, ty = (cams[0].width + 15) // 16, (cams[0].height + 15) // 16
    for k in poses:
        cam = cams[k]
        rend.render(sc["device"], cam, opt)
        torch.cuda.synchronize()
        img = rend.image.double().cpu().numpy()
        rec = oracle.preprocess(sc["scene"], cam)
        tiles = np.sort(np.random.default_rng(1000 + int(k)).choice(tx * ty, size=min(tiles_per_pose, tx * ty),
                                                                      replace=False))
        st, ids = oracle.tile_lists(rec, cam, tiles)
        amb = oracle.ambiguous_membership(rec, cam)
        ref = oracle.composite(rec, cam, st, ids, nthreads=threads, tiles=tiles, amb=amb)
        mask = np.zeros((cam.height, cam.width), bool)
        for t in tiles:
            mask[(t // tx) * 16:(t // tx) * 16 + 16, (t % tx) * 16:(t % tx) * 16 + 16] = True
        a, b = np.clip(img[:, mask], 0, 1), np.clip(ref["image"][:, mask], 0, 1)
        sq += float(((a - b) ** 2).sum())
        ab += float(np.abs(img[:, mask] - ref["image"][:, mask]).sum())
        npx += a.size
        ok = mask & (ref["ambiguous"] == 0)
        mx = max(mx, float(np.abs(img[:, ok] - ref["image"][:, ok]).max()))
        fl = ref["ambiguous"].copy()
        fl[~mask] = 0
        r = oracle.check_flagged(img, None, rec, cam, st, ids, fl, tol_img=1e-3, amb=amb)
        flagged += r["checked"]
        matched += r["matched"]
        failed += r["failed"]
        unresolved += r["unresolved"]
    mse = sq / max(npx, 1)
    sampled = npx / 3
    return {"psnr_db": float("inf") if mse == 0 else float(10 * np.log10(1 / mse)), "mae": ab / max(npx, 1),
            "max_abs": mx, "poses": int(len(poses)), "tiles_per_pose": int(tiles_per_pose),
            "flagged_pixel_frac": flagged / max(sampled, 1),
            "flagged_matched": matched, "flagged_failed": failed, "flagged_unresolved": unresolved,
            "unresolved_pixel_frac": unresolved / max(sampled, 1)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def backward_mfma_leg(gs, torch, ds, cams, n, steps, warmup, precision, splits):
    """Times gs_rasterize_backward_mfma on each pose after that pose's MFMA forward (which also
    writes the T_final and blended-prefix-end planes the backward starts from), with a fixed
    N(0, 1) upstream gradient; HIP events around the backward launch only."""
    st = torch.cuda.current_stream()
    rend = gs.Renderer(n, 1920, 1080, group=1)
    opt = gs.options(group=1, precision=precision, splits=splits, aux_flags=gs.GS_AUX_TFINAL | gs.GS_AUX_LAST)
    grads = gs.Grads(n)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    dimg = torch.randn((3, 1080, 1920), generator=gen, device="cuda")
    evs = []
    fwd_evs = []
    for i in range(warmup + steps):
        cam = cams[i % len(cams)]
        f0 = torch.cuda.Event(enable_timing=True)
        f0.record(st)
        rend.render(ds, cam, opt)
        grads.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        gs.gs_rasterize_backward_mfma(rend.proj, rend.bins, cam, opt, dimg, rend.aux[0], rend.aux[1], grads)
        b.record(st)
        if i >= warmup:
            evs.append((a, b))
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    return {"kernel": f"k_raster_backward_mfma ({precision}, splits {splits})", "precision": precision,
            "frames": steps, "avg_ms": float(np.mean(ms)), "p50_ms": float(np.percentile(ms, 50)),
            "p99_ms": float(np.percentile(ms, 99)),
            "forward_state": "GS_AUX_TFINAL | GS_AUX_LAST planes of the MFMA forward (no replay)"}


def backward_leg(gs, torch, ds, cams, n, steps, warmup):
    """Times gs_rasterize_backward (FP32, tile bins) on each pose after its forward render,
    with a fixed N(0, 1) upstream gradient; HIP events around the backward launch only."""
    st = torch.cuda.current_stream()
    rend = gs.Renderer(n, 1920, 1080, group=1)
    opt = gs.options(group=1, precision="fp32")
    grads = gs.Grads(n)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    dimg = torch.randn((3, 1080, 1920), generator=gen, device="cuda")
    evs = []
    for i in range(warmup + steps):
        cam = cams[i % len(cams)]
        rend.render(ds, cam, opt)
        grads.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        gs.gs_rasterize_backward(rend.proj, rend.bins, cam, opt, dimg, grads)
        b.record(st)
        if i >= warmup:
            evs.append((a, b))
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    return {"kernel": "k_raster_backward", "precision": "fp32", "frames": steps, "avg_ms": float(np.mean(ms)),
            "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99))}


def serve(gs, torch, args):
    """Serving workload: 8 resident scenes (N = 0.5M..3M), requests of mixed resolution and pose.
    A closed burst measures saturated throughput; then an open-loop Poisson stream at
    `serve_load` of it gives p50/p99 latency (completion - scheduled arrival)."""
    from paper_2605_17855_amd import scenes, server
    log("serving: generating 8 resident scenes (0.5M..3M Gaussians)")
    scs = scenes.serving_scenes()
    dss = [gs.DeviceScene(s) for s in scs]
    # opacity-aware tile culling unless disabled: the images are those of the full lists
    opt = gs.options(group=1, precision=args.precision, splits=args.splits, tight=not args.no_tight)
    # per-scene duplicated entries per pixel, from one 1080p render each
    kpp = {}
    for i, sc in enumerate(scs):
        cam = scenes.random_pose(np.random.default_rng(900 + i), 1920, 1080)
        r = gs.Renderer(sc.n, 1920, 1080)
        kpp[i] = r.render(dss[i], cam, opt) / (1920 * 1080)
        del r
    torch.cuda.synchronize()
    max_px = max(w * h for w, h in scenes.SERVE_RESOLUTIONS)
    pool = int(args.serve_pool_gib * (1 << 30))
    slots = 16

    def run(reqs, max_batch=32):
        be = server.GpuBackend(dss, slots=slots, pool_bytes=pool, opt=opt, max_pixels=max_px,
                               keys_per_pixel=kpp)
        try:
            st = server.Server(be, pool, slots=slots, max_batch=max_batch, max_inflight_batches=3).run(reqs)
        finally:
            be.close()
        torch.cuda.synchronize()
        return st

    log("serving: warm-up")
    run(scenes.serving_requests(64, rate_hz=1e7, seed=48))
    log("serving: saturated burst of 1000 requests")
    sat = run(scenes.serving_requests(1000, rate_hz=1e7, seed=47))
    log("serving: the same burst with one job per raster launch")
    sat1 = run(scenes.serving_requests(1000, rate_hz=1e7, seed=47), max_batch=1)
    rate = args.serve_load * sat.frames_per_s
    log(f"serving: saturated {sat.frames_per_s:.0f} frames/s; open loop at {rate:.0f} req/s, "
        f"{args.serve_requests} requests")
    st = run(scenes.serving_requests(args.serve_requests, rate_hz=rate, seed=49))
    return {"workload": "8 resident scenes, N = linspace(0.5M, 3M), 64-cluster mixture, SH degree 3; "
                        "resolution uniform over 640x360..2560x1440, poses on the radius-4 sphere",
            "requests": args.serve_requests, "offered_rate_hz": rate, "load": args.serve_load,
            "frames_per_s": st.frames_per_s, "p50_ms": st.latency_p50_ms, "p99_ms": st.latency_p99_ms,
            "mean_ms": st.latency_mean_ms, "saturated_frames_per_s": sat.frames_per_s,
            "saturated_p99_ms": sat.latency_p99_ms, "saturated_mean_batch": sat.mean_batch,
            "saturated_frames_per_s_one_job_per_launch": sat1.frames_per_s,
            "saturated_p99_ms_one_job_per_launch": sat1.latency_p99_ms,
            "completed": st.completed, "failed": st.failed,
            "retries": st.retries, "batches": st.batches, "mean_batch": st.mean_batch,
            "max_inflight_jobs": st.max_inflight_jobs, "pool_bytes": pool,
            "max_reserved_bytes": st.max_reserved_bytes, "slots": slots,
            "precision": args.precision, "tight_culling": not args.no_tight,
            "resident_gaussians": int(sum(s.n for s in scs))}


def sweep(gs, torch, args):
    """Frame rate of every (precision, tile group) variant on the sensitivity and stress
    workloads, with the entry counts behind the load reduction 1 - K(G)/K(1)."""
    from paper_2605_17855_amd import scenes
    work = [("3M Gaussians, 256 clusters, 1920x1080", lambda: scenes.clustered_3m(width=1920, height=1080), 1920, 1080, 3),
            ("3M Gaussians, 256 clusters, 3840x2160", lambda: scenes.clustered_3m(width=3840, height=2160), 3840, 2160, 3),
            ("dense 6M Gaussians, log-scale N(ln 0.05, 0.5), opacity sigmoid(N(-1,1)), 1920x1080",
             lambda: scenes.dense_6m(), 1920, 1080, 5)]
    rows, lr, adaptive = [], [], []
    for name, make, w, h, seed in work:
        log(f"sweep: {name}")
        sc, _ = make()
        ds = gs.DeviceScene(sc)
        cams = scenes.orbit(max(args.sweep_steps, 1), w, h, seed=seed)
        keys = {}
        # (group, tight, per-tile rows, precisions): 2x2 groups build rows in the group frame unless
        # per-tile rows are asked for
        variants = ((1, False, False, ("fp32", "fp16", "bf16")), (1, True, False, ("fp32", "fp16", "bf16")),
                    (2, False, False, ("fp32", "fp16", "bf16")), (2, False, True, ("fp16", "bf16")),
                    (4, False, False, ("fp32", "fp16", "bf16")),
                    (8, False, False, ("fp16", "bf16")), (2, True, False, ("fp16",)), (4, True, False, ("fp16",)),
                    (8, True, False, ("fp16",)))
        for group, tight, tile_rows, precs in variants:
            rend = gs.Renderer(sc.n, w, h, group=group)
            for prec in precs:
                splits = 3 if prec == "bf16" else 2
                opt = gs.options(group=group, precision=prec, splits=splits, tight=tight, tile_rows=tile_rows)
                el, fm, rm = timed_frames(gs, torch, ds, cams, rend, opt, args.sweep_steps, 3)
                rows.append({"workload": name, "precision": prec, "splits": splits, "group": group, "tight": tight,
                             "tile_rows": tile_rows,
                             "frames_per_s": args.sweep_steps / el, "p99_ms": float(np.percentile(fm, 99)),
                             "raster_avg_ms": float(np.mean(rm)), "stage_ms": timed_frames.stages})
                log(f"  G{group}{' tight' if tight else ''}{' tile rows' if tile_rows else ''} {prec}: "
                    f"{rows[-1]['frames_per_s']:.1f} frames/s, raster {rows[-1]['raster_avg_ms']:.3f} ms")
            if not tile_rows:
                keys[f"{group}t" if tight else group] = np.mean(
                    [rend.render(ds, c, gs.options(group=group, precision="fp16", tight=tight)) for c in cams[:5]])
            del rend
        # per-scene adaptive (group side, culling) variant, FP16: probe, then time
        from paper_2605_17855_amd.adaptive import AdaptiveRenderer
        ar = AdaptiveRenderer(sc.n, w, h, precision="fp16", splits=2, probes=2)
        for i in range(2 * len(ar.variants)):
            ar.render(ds, cams[i % len(cams)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.sweep_steps):
            ar.render(ds, cams[i % len(cams)])
        torch.cuda.synchronize()
        adaptive.append({"workload": name, "chosen_group": ar.chooser.chosen[0], "chosen_tight": ar.chooser.chosen[1],
                         "probe_best_ms": {f"{g}{'t' if t else ''}": min(v) for (g, t), v in ar.chooser.times.items()},
                         "frames_per_s": args.sweep_steps / (time.perf_counter() - t0)})
        log(f"  adaptive: G{ar.chooser.chosen[0]}{' culling' if ar.chooser.chosen[1] else ''}, "
            f"{adaptive[-1]['frames_per_s']:.1f} frames/s")
        del ar
        lr.append({"workload": name, "entries": {str(g): float(k) for g, k in keys.items()},
                   "load_reduction": {str(g): 1.0 - keys[g] / keys[1] for g in (2, 4, 8, "1t", "2t", "4t", "8t")}})
        del ds
        torch.cuda.empty_cache()
    return {"rows": rows, "load_reduction": lr, "adaptive": adaptive, "steps": args.sweep_steps}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
        return
    import torch
    from paper_2605_17855_amd import gs, scenes

    if args.serve_only:
        print(json.dumps({"serving": serve(gs, torch, args)}), flush=True)
        return
    if args.sweep:
        print(json.dumps({"sweep": sweep(gs, torch, args)}), flush=True)
        return

    if args.scene == "dense6m":
        log("generating the dense 6M-Gaussian scene")
        sc, _ = scenes.dense_6m()
        cams = scenes.orbit(200, 1920, 1080, seed=5)
        scene_text = "6M Gaussians, dense 64-cluster mixture (log-scale N(ln 0.05, 0.5), opacity sigmoid(N(-1, 1)))"
    else:
        log("generating the 1M-Gaussian scene")
        sc, _ = scenes.clustered_1m()
        cams = scenes.orbit(200, 1920, 1080, seed=2)
        scene_text = "1M Gaussians, 64-cluster mixture"
    ds = gs.DeviceScene(sc)
    okw = dict(group=args.group, precision=args.precision, splits=args.splits)
    rend = gs.Renderer(sc.n, 1920, 1080, group=args.group)

    opt = gs.options(**okw)
    log(f"timing {args.precision}: {args.warmup} warm-up + {args.steps} frames")
    elapsed, frame_ms, raster_ms = timed_frames(gs, torch, ds, cams, rend, opt, args.steps, args.warmup)
    stages = timed_frames.stages
    fps = args.steps / elapsed
    first_img = None
    rend.render(ds, cams[0], opt)
    torch.cuda.synchronize()
    first_img = rend.image.double().cpu().numpy()

    log("counting evaluations of the timed frames (aux pass)")
    e_pix, blend, entries_pf, visible_pf = work_units(gs, torch, ds, cams, rend, okw, args.steps)
    exe = work_units.executed
    raster_total_s = sum(raster_ms) / 1e3
    flops = FLOPS_PER_EVAL * e_pix + FLOPS_PER_BLEND * blend
    achieved = flops / raster_total_s / 1e12
    vfr = valu_fracs(args, float(np.mean(raster_ms)) / 1e3)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": raster_traffic(args),
                "kernel": f"k_raster_mfma (precision {args.precision}, splits {args.splits}, group {args.group})"
                          if args.precision != "fp32" else "k_raster_fp32",
                "frac_vs_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                "mfma_frac": (POWER_FLOPS * e_pix / raster_total_s / 1e12 / PEAK_FP16_MFMA_TFLOPS)
                if args.precision != "fp32" else None,
                "traffic_source": "profiles/hbm_counters_1m_1080p_fp16.md (rocprofv3 FETCH_SIZE, WRITE_SIZE of the "
                                  "kernel built from the hashed sources; not measured in this run)",
                "valu_issue_frac": vfr[0], "valu_active_frac": vfr[1],
                "valu_source": "profiles/sq_counters_raster_1m_1080p_fp16.md (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU "
                               "per launch) over this run's average launch",
                "avg_launch_ms": float(np.mean(raster_ms)),
                "evals_per_frame": e_pix / args.steps, "blends_per_frame": blend / args.steps,
                "entries_per_frame": entries_pf, "visible_per_frame": visible_pf}

    pipelined = None
    if not args.no_pipelined:
        log("timing two frames in flight (two streams, separate buffers)")
        pipelined = {"frames_in_flight": 2, "frames_per_s": pipelined_frames(gs, torch, ds, cams, sc.n, opt,
                                                                              args.steps, args.warmup)}

    device_counts = None
    if not args.no_device_counts:
        log("timing the frame without the host wait, eager and replayed from captured graphs")
        device_counts = device_count_frames(gs, torch, ds, cams, sc.n, rend.bins.capacity, okw, args.steps,
                                            args.warmup, first_img)

    all_rows = None
    if args.precision != "fp32" and not args.no_all_rows:
        # the same frames with quadrant culling off (every row in every quadrant, as the FP32
        # rasterizer runs them): separates the contraction's share of the speedup from the culling's
        log("timing the MFMA rasterizer with every row in every quadrant")
        rend_a = gs.Renderer(sc.n, 1920, 1080, group=args.group)
        _, fma, rma = timed_frames(gs, torch, ds, cams, rend_a, gs.options(all_rows=True, **okw), args.steps,
                                   args.warmup)
        all_rows = {"option": "GS_OPT_ALL_ROWS", "raster_avg_ms": float(np.mean(rma)),
                    "p50_ms": float(np.percentile(fma, 50)), "p99_ms": float(np.percentile(fma, 99))}
        del rend_a

    compare = None
    if not args.no_compare and args.precision != "fp32":
        log("timing fp32 plain on the same poses")
        opt32 = gs.options(group=1, precision="fp32")
        rend32 = gs.Renderer(sc.n, 1920, 1080, group=1)
        el32, fm32, rm32 = timed_frames(gs, torch, ds, cams, rend32, opt32, args.steps, args.warmup)
        compare = {"precision": "fp32", "frames_per_s": args.steps / el32,
                   "p50_ms": float(np.percentile(fm32, 50)), "p99_ms": float(np.percentile(fm32, 99)),
                   "raster_avg_ms": float(np.mean(rm32)), "stage_ms": timed_frames.stages}

    tight = None
    if not args.no_tight and args.group == 1:
        # the same frames with opacity-aware tile culling (identical images, fewer entries)
        log("timing the opacity-aware tile culling variant")
        rend_t = gs.Renderer(sc.n, 1920, 1080, group=1)
        res = {}
        for prec, splits in ((args.precision, args.splits), ("fp32", 2)):
            el, fm, rm = timed_frames(gs, torch, ds, cams, rend_t, gs.options(precision=prec, splits=splits,
                                                                               tight=True),
                                      args.steps, args.warmup)
            res[prec] = {"frames_per_s": args.steps / el, "p50_ms": float(np.percentile(fm, 50)),
                         "p99_ms": float(np.percentile(fm, 99)), "raster_avg_ms": float(np.mean(rm)),
                         "stage_ms": timed_frames.stages}
        ek, eb, ent, _ = work_units(gs, torch, ds, cams, rend_t, dict(precision=args.precision, splits=args.splits,
                                                                       tight=True), args.steps)
        t_raster_s = res[args.precision]["raster_avg_ms"] * args.steps / 1e3
        tight = {"option": "GS_OPT_TIGHT", **res[args.precision],
                 "fp32_plain_frames_per_s": res["fp32"]["frames_per_s"],
                 "speedup_vs_fp32": res[args.precision]["frames_per_s"] / res["fp32"]["frames_per_s"],
                 "entries_per_frame": ent, "evals_per_frame": ek / args.steps,
                 "roofline_frac": (FLOPS_PER_EVAL * ek + FLOPS_PER_BLEND * eb) / t_raster_s / 1e12 / PEAK_FP32_TFLOPS}

    backward = None
    if not args.no_backward:
        log("timing the backward pass (FP32, tile bins)")
        backward = backward_leg(gs, torch, ds, cams, sc.n, args.steps, args.warmup)
        if args.precision != "fp32":
            log(f"timing the backward pass of the MFMA forward ({args.precision})")
            backward["mfma"] = backward_mfma_leg(gs, torch, ds, cams, sc.n, args.steps, args.warmup, args.precision,
                                                 args.splits)
            backward["mfma"]["vs_mfma_forward_raster"] = backward["mfma"]["avg_ms"] / float(np.mean(raster_ms))

    cpu = None
    quality = {}
    if not args.no_cpu_baseline:
        log("FP64 oracle: CPU baseline on the first pose")
        cpu, _ = cpu_baseline_and_psnr(gs, torch, sc, cams[0], first_img, args.cpu_seconds)
        log("FP64 oracle: quality of the chosen form over the timed poses")
        quality = quality_over_poses(gs, torch, {"scene": sc, "device": ds}, cams, rend, opt, args.steps)

    serving = None
    if not args.no_serve:
        serving = serve(gs, torch, args)

    line = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision if args.precision != "fp32" else "fp32",
        "data": "synthetic",
        "config": {"workload": f"{scene_text}, SH degree 3, 1920x1080, {min(args.steps, len(cams))} "
                               f"poses of a {len(cams)}-pose orbit (one frame per pose), "
                               f"{args.group}x{args.group} tile groups, {args.precision} splits {args.splits}",
                   "gaussians": sc.n, "width": 1920, "height": 1080, "group": args.group,
                   "precision": args.precision, "splits": args.splits},
        "p50_ms": float(np.percentile(frame_ms, 50)), "p99_ms": float(np.percentile(frame_ms, 99)),
        "raster_avg_ms": float(np.mean(raster_ms)),
        "mpix_gauss_evals_per_s": e_pix / raster_total_s / 1e6,
        "psnr_db_vs_oracle": quality.get("psnr_db"), "mae_vs_oracle": quality.get("mae"),
        "max_abs_vs_oracle": quality.get("max_abs"), "quality_vs_oracle": quality or None,
        "stage_ms": stages,
        "executed_work_efficiency": {"e_pix_over_e_tile": e_pix / max(exe["e_tile"], 1),
                                     "e_pix_over_e_wave": e_pix / max(exe["e_wave"], 1)},
        "fp32_plain": compare,
        "speedup_vs_fp32": (fps / compare["frames_per_s"]) if compare else None,
        "raster_speedup_vs_fp32": (compare["raster_avg_ms"] / float(np.mean(raster_ms))) if compare else None,
        "mfma_all_rows": all_rows,
        "pipelined": pipelined,
        "device_counts": device_counts,
        "raster_speedup_vs_fp32_all_rows": (compare["raster_avg_ms"] / all_rows["raster_avg_ms"])
        if (compare and all_rows) else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tight_culling": tight,
        "backward": backward,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

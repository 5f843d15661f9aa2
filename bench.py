#!/usr/bin/env python3
"""Benchmark of the data-parallel volume-rendering hot path on one MI355X.

One step = one frame: every brick's partial image is ray cast (all bricks'
partials through one persistent work-queue launch), then the partials are
sort-last composited into the frame.  Inputs are resident in HBM before timing starts (brick ingest is
outside the timed region).  Default workload: a 1024x1024x512 float32 field
(64 Gaussian blobs + a tanh shock front), kd-split into 16 uneven bricks with
ghost layers, 1920x1080 perspective view, step 0.5 voxel, opacity scale 0.05,
16-partial composite.

Prints one JSON line: Msamples/s (samples the kernels evaluated, counted on
the device), frames/s, the march kernel's achieved HBM bandwidth on
algorithmic bytes (bricks read once + partial images written) against the
8 TB/s peak, and the CPU oracle timed on a bounded pixel sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["c2", "c1", "c3", "c4", "c5", "c5-adjoint"], default="c2")
    ap.add_argument("--storage", choices=["f32", "f16"], default=None,
                    help="brick storage (default f32; c5 is a float16 workload: f16)")
    ap.add_argument("--path", choices=["staged", "direct"], default="staged",
                    help="march from LDS-staged slices or straight from HBM (same images)")
    ap.add_argument("--staging", choices=["slab", "ring"], default=None,
                    help="staged march family: all waves stage a slab then march it, or a producer "
                         "wave streams slices into an LDS ring ahead of the marching waves "
                         "(default: the library's choice for the storage, f32 ring, f16 slab)")
    ap.add_argument("--tile-width", type=int, choices=[16, 32], default=32,
                    help="staged march: tile width in pixels (tiles are 16 rows high; slab: 16)")
    ap.add_argument("--chunk", type=int, choices=[4, 8], default=4,
                    help="staged march: slices per chunk between producer/consumer synchronisations")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="first run one plain copy of known size through the ingest kernel "
                         "(512^3 float32: 512 MiB read, 512 MiB written) for HBM-counter scaling")
    ap.add_argument("--summarize-sq", metavar="SQ_DIR",
                    help="turn a rocprofv3 --pmc run with SQ_INSTS_VALU into the per-launch "
                         "VALU record under profiles/")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs of --pmc-calibrate (FETCH_SIZE, then "
                         "WRITE_SIZE) into the per-frame HBM traffic record under profiles/")
    args = ap.parse_args()
    if args.storage is None:
        args.storage = "f16" if args.workload.startswith("c5") else "f32"
    return args


def scene_for(name):
    import synth
    if name == "c2":
        sc = synth.config_c2()
        desc = ("c2: 1024x1024x512 f32 field (64 blobs + tanh shock), 16 uneven kd bricks with "
                "1-voxel ghosts, 1920x1080 perspective, step 0.5, opacity 0.05, 16-partial "
                "sort-last composite")
    elif name == "c5":
        sc = synth.config_c5(log=lambda m: log(f"c5 generation: {m}"))
        desc = ("c5: 2048x1024x1024 field (128 blobs + two tanh shocks + fractal noise) stored "
                "as f16, 64 uneven kd bricks with 1-voxel ghosts, 3840x2160 perspective, step "
                "0.25, opacity 0.05, 64-partial sort-last composite")
    else:
        sc = synth.config_c1()
        desc = "c1: 64^3 f32 field (8 blobs + noise), 2 bricks 32x64x64, 256x256, step 0.5"
    return sc, desc


KERNEL_SOURCES = ("march.hip", "march_common.h", "dpvr_kernels.h")


def kernel_sha256():
    """Hash of the sources the march kernel is built from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2501_01628_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_path(workload, storage):
    return os.path.join(ROOT, "profiles", f"march_queue_{workload}_{storage}_traffic.json")


def traffic_for(workload, storage):
    """Measured HBM bytes per launch from a committed rocprofv3 --pmc summary,
    valid only while the kernel sources are unchanged."""
    path = traffic_path(workload, storage)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != kernel_sha256():
        return None
    return rec.get("hbm_bytes_per_frame")


CALIB_STORED = 512                      # stored extent of the calibration brick (pitch = extent)
CALIB_BYTES = CALIB_STORED ** 3 * 4     # bytes read and bytes written by its ingest
MARCH_KERNEL = "march_queue"


def _pmc_rows(d, counter):
    """(kernel name, value) per dispatch of one counter, in dispatch order."""
    import csv
    import glob
    rows = []
    for fn in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def summarize_pmc(args):
    """HBM bytes per frame of the march launch: its FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) scaled by what the same counters read for the plain
    copy of CALIB_BYTES done first by --pmc-calibrate."""
    out = {}
    for name, d in zip(("FETCH_SIZE", "WRITE_SIZE"), args.summarize_pmc):
        rows = _pmc_rows(d, name)
        ingest = [v for k, v in rows if "ingest_kernel" in k]
        march = [v for k, v in rows if MARCH_KERNEL in k]
        if not ingest or not march:
            raise SystemExit(f"{d}: no ingest/march dispatches with {name}")
        calib = ingest[0] * 1024.0                  # first ingest = the calibration copy
        scale = CALIB_BYTES / calib
        out[name] = {"calibration_bytes_counted": calib, "scale": scale,
                     "march_kib_per_dispatch": sum(march) / len(march),
                     "march_dispatches": len(march),
                     "march_bytes_per_dispatch_scaled": sum(march) / len(march) * 1024.0 * scale}
    rec = {"kernel": MARCH_KERNEL, "workload": args.workload, "storage": args.storage,
           "kernel_sha256": kernel_sha256(), "kernel_sources": list(KERNEL_SOURCES),
           "hbm_bytes_per_frame": out["FETCH_SIZE"]["march_bytes_per_dispatch_scaled"]
           + out["WRITE_SIZE"]["march_bytes_per_dispatch_scaled"],
           "counters": out,
           "calibration": f"ingest_kernel copy of a {CALIB_STORED}^3 float32 brick "
                          f"({CALIB_BYTES} B read, {CALIB_BYTES} B written)",
           "commands": [f"rocprofv3 --pmc {c} --output-format csv -d <dir> -- python3 bench.py "
                        f"--workload {args.workload} --storage {args.storage} --steps 2 --warmup 1 "
                        f"--no-cpu-baseline --pmc-calibrate" for c in ("FETCH_SIZE", "WRITE_SIZE")]}
    path = traffic_path(args.workload, args.storage)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
    return 0


VALU_LANES_PER_CU_CYCLE = 64        # 4 SIMDs x 16 lanes: one wave64 VALU instruction per 4 cycles
N_CU, CLOCK_HZ = 256, 2.4e9


def valu_path(workload, storage):
    return os.path.join(ROOT, "profiles", f"march_queue_{workload}_{storage}_valu.json")


def summarize_sq(args):
    """VALU wave instructions per march launch from SQ_INSTS_VALU."""
    rows = [v for k, v in _pmc_rows(args.summarize_sq, "SQ_INSTS_VALU") if MARCH_KERNEL in k]
    if not rows:
        raise SystemExit(f"{args.summarize_sq}: no march dispatch with SQ_INSTS_VALU")
    rec = {"kernel": MARCH_KERNEL, "workload": args.workload, "storage": args.storage,
           "kernel_sha256": kernel_sha256(), "kernel_sources": list(KERNEL_SOURCES),
           "valu_wave_insts_per_launch": sum(rows) / len(rows), "dispatches": len(rows),
           "command": f"rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU "
                      f"SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_INSTS_VMEM "
                      f"--output-format csv -d <dir> -- python3 "
                      f"bench.py --workload {args.workload} --storage {args.storage} --steps 3 "
                      f"--warmup 1 --no-cpu-baseline"}
    with open(valu_path(args.workload, args.storage), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
    return 0


def valu_for(workload, storage, march_ms):
    """Issue time of the launch's VALU instructions at the chip's vector rate
    (from the committed counter record, while the kernel is unchanged), as a
    fraction of the measured launch time."""
    path = valu_path(workload, storage)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != kernel_sha256():
        return None
    insts = rec["valu_wave_insts_per_launch"]
    issue_ms = insts * 64 / (VALU_LANES_PER_CU_CYCLE * N_CU * CLOCK_HZ) * 1e3
    return {"wave_insts_per_launch": insts, "issue_ms": issue_ms, "frac": issue_ms / march_ms,
            "peak": "64 lanes/CU/cycle x 256 CUs x 2.4 GHz (unpacked fp32)"}


def calibration_copy():
    """One ingest of a CALIB_STORED^3 float32 brick whose rows need no
    padding: a plain copy of known size, for scaling the HBM counters."""
    import torch
    import paper_2501_01628_amd as dp
    n = CALIB_STORED
    v = torch.rand((n, n, n), dtype=torch.float32, device="cuda:0")
    r = dp.Renderer([(v, (0, 0, 0))], np.zeros((256, 4), np.float32))
    r.synchronize()
    r.close()
    del v, r
    torch.cuda.empty_cache()
    log(f"calibration copy: {CALIB_BYTES} B read + written by the ingest kernel")


def cpu_baseline(sc, target_s, frame=None):
    """The oracle timed on a random pixel sample of the frame; with the GPU
    frame given, also its max error against the oracle at those pixels."""
    import numpy as np
    import oracle
    W, H = sc.camera["width"], sc.camera["height"]
    rng = np.random.default_rng(0)
    # calibrate on a sample of ~1 s, then size the measured sample
    def run(npix):
        idx = rng.choice(W * H, npix, replace=False)
        pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
        t0 = time.perf_counter()
        img, _, cnt = oracle.render_scene(sc, pixels=pix)
        return time.perf_counter() - t0, int(cnt[0]), pix, img
    t, _, _, _ = run(20000)
    npix = int(min(W * H, max(20000, 20000 * target_s / max(t, 1e-3))))
    t, samples, pix, img = run(npix)
    cores = oracle.threads()
    out = {"value": samples / t / 1e6, "unit": "Msamples/s", "cores": cores, "kind": "oracle",
           "sample": f"{npix} random pixels of the same frame, all {len(sc.bricks)} bricks + "
                     f"composite, {samples} samples (no early termination) in {t:.1f} s"}
    err = None
    if frame is not None:
        got = frame[pix[:, 1], pix[:, 0]].astype(np.float64)
        err = float(np.max(np.abs(got - img)))
    return out, err


def bench_batch(args):
    """Batched workload: 14 uneven bricks x 6 time steps x 3 fields x 4 cameras
    at 1024^2 (1008 partial images, 72 frames): the plain path (per frame,
    one launch per brick + one composite) against the batch (one graph:
    persistent queued march + one composite launch for all frames), for
    float32 and float16 storage."""
    import numpy as np
    import torch

    import paper_2501_01628_amd as dp
    import synth
    t0 = time.perf_counter()
    d = synth.config_c3()
    log(f"generated c3 ({len(d['bricks'])} brick-volumes) in {time.perf_counter() - t0:.1f} s")
    keys = sorted({(t, f) for t, f, _, _, _ in d["bricks"]})
    out = {"metric": "Msamples/s (batched render+composite, samples evaluated per batch x batches/s)",
           "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "c3: 14 uneven bricks (U{64..320}^3) x 6 time steps x 3 fields x "
                                  "4 cameras at 1024x1024, step 0.5, opacity 0.1; 1008 partials, "
                                  "72 frames of 14-partial sort-last composites"}}
    results = {}
    for storage in ("f32", "f16"):
        st = dp.VR_F16 if storage == "f16" else dp.VR_F32
        br = dp.BatchRenderer(dt=d["step"])
        tfi = br.add_tf(d["tf"], (0, 1), d["opacity_scale"])
        for (t, f, b, lo, vox) in d["bricks"]:
            br.add_brick(vox, lo, storage=st)
        br.drop_uploads()
        cams = [br.add_camera(c) for c in d["cameras"]]
        for (t, f) in keys:
            ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
            for c in cams:
                br.add_frame(c, ids, tfi)
        br.build()
        tuned_ms = br.autotune(reps=2)
        for _ in range(args.warmup):
            br.launch()
        br.samples.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(br.stream)
        for _ in range(args.steps):
            br.launch()
        e1.record(br.stream)
        torch.cuda.synchronize()
        batch_ms = e0.elapsed_time(e1) / args.steps
        samples = int(br.samples.sum().item()) // args.steps
        wg, order, staging, tile_w, chunk = br.config()
        # plain path on the same bricks: per frame, one march launch per brick + a composite,
        # with the launch shape the batch was tuned to
        ctx = br.ctx
        dp.vr_set_march_config(ctx, st, staging, tile_w, chunk)
        dp.vr_set_transfer_function(ctx, br._tf_keep[0], 256, 0.0, 1.0, d["opacity_scale"])
        frame_parts = []
        fi = 0
        for (t, f) in keys:
            ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
            for c in cams:
                frame_parts.append((c, [br.bricks[i] for i in ids],
                                    [dp.make_partial(*br.parts[fi * len(ids) + k]) for k in range(len(ids))],
                                    br.frames[fi]))
                fi += 1

        def plain_pass():
            for c, bricks, parts, outf in frame_parts:
                dp.set_camera(ctx, d["cameras"][c])
                for b, p in zip(bricks, parts):
                    dp.vr_render_partial(ctx, b, p)
                dp.vr_composite(ctx, parts, (0.0, 0.0, 0.0, 0.0), outf)
        plain_pass()
        torch.cuda.synchronize()
        e0.record(br.stream)
        plain_steps = max(1, args.steps // 4)
        for _ in range(plain_steps):
            plain_pass()
        e1.record(br.stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1) / plain_steps
        results[storage] = {"batch_ms": batch_ms, "plain_ms": plain_ms, "samples": samples,
                            "autotune": {"wg_per_cu": wg, "order": ["as given", "by brick"][order],
                                         "staging": ["slab", "ring"][staging],
                                         "tile_width": tile_w, "chunk_slices": chunk,
                                         "tuned_ms": tuned_ms},
                            "msamples_per_s": samples / (batch_ms * 1e-3) / 1e6,
                            "speedup_vs_plain": plain_ms / batch_ms}
        log(f"c3 {storage}: batch {batch_ms:.3f} ms, plain {plain_ms:.3f} ms, {samples} samples, "
            f"wg/cu {wg}, order {order}")
        br.close()
        torch.cuda.empty_cache()
    out["value"] = results["f32"]["msamples_per_s"]
    out["ms_per_step"] = results["f32"]["batch_ms"]
    out["storage"] = results
    out["f16_vs_f32_batch_speedup"] = results["f32"]["batch_ms"] / results["f16"]["batch_ms"]
    out["f16_batch_vs_f32_plain_speedup"] = results["f32"]["plain_ms"] / results["f16"]["batch_ms"]
    print(json.dumps(out), flush=True)
    return 0


def _time_gradient_steps(args, dr, tf, vol, cams, targets, bg):
    """Mean ms of a forward pass (no grad) and of a gradient step."""
    import torch

    def forward():
        tot = torch.zeros((), device="cuda")
        for cam, tgt in zip(cams, targets):
            tot = tot + ((dr.render(tf, vol, cam, bg) - tgt) ** 2).sum()
        return tot

    def step():
        tf.grad = None
        vol.grad = None
        forward().backward()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(args.steps):
        with torch.no_grad():
            forward()
    ev[1].record()
    ev[2].record()
    for _ in range(args.steps):
        step()
    ev[3].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / args.steps, ev[2].elapsed_time(ev[3]) / args.steps


def bench_adjoint(args):
    """Differentiable workloads.  c4: 128^3 float32 volume, 8 views at
    512x512, step 0.5.  c5-adjoint: the c5 volume (2048x1024x1024, 64 float16
    bricks, step 0.25) seen through the central 512x512 crop of its 3840x2160
    view (same pixel rays: the crop camera narrows the field of view).  One
    gradient step = forward with transmittance checkpoints every 64 samples
    + L2 loss against fixed targets + composite backward + adjoint march
    (gradients for the 256x4 table and all voxels).  Targets are seeded random
    images (timing only; the gradient itself is checked against the oracle
    and finite differences in the tests)."""
    import math

    import torch

    import paper_2501_01628_amd as dp
    import synth
    if args.workload == "c4":
        sc = synth.config_c4()
        cams = sc.extra["cameras"]
        n = sc.field.shape[0]
        dims, boxes, storage = (n, n, n), [((0, 0, 0), (n, n, n))], dp.VR_F32
        desc = ("c4: 128^3 f32 volume (8 blobs), 8 views at 512x512, step 0.5, 64-sample "
                "checkpoints, L2 loss, gradients for the 256x4 TF and all voxels")
    else:
        sc = synth.config_c5(log=lambda m: log(f"c5 generation: {m}"))
        cam = dict(sc.camera)
        crop = 512
        half = math.tan(math.radians(cam["fovy_deg"]) / 2.0) * crop / cam["height"]
        cam.update(width=crop, height=crop, fovy_deg=math.degrees(2.0 * math.atan(half)))
        cams = [cam]
        dims = sc.dims
        boxes = [(b.lo, b.hi) for b in sc.bricks]
        storage = dp.VR_F16
        desc = ("c5-adjoint: 2048x1024x1024 field in 64 f16 bricks, central 512x512 crop of the "
                "3840x2160 view, step 0.25, 64-sample checkpoints, L2 loss, gradients for the "
                "256x4 TF and all voxels")
    dr = dp.DiffRenderer(dims, boxes, sc.vrange, sc.opacity_scale, sc.step, 64, storage=storage)
    tf = torch.tensor(synth.default_tf(), device="cuda", requires_grad=True)
    vol = torch.tensor(sc.field, device="cuda", requires_grad=True)
    log(f"volume on the device: {tuple(vol.shape)}")
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    targets = [torch.rand((c["height"], c["width"], 4), device="cuda", generator=g) for c in cams]
    fwd_ms, step_ms = _time_gradient_steps(args, dr, tf, vol, cams, targets, (0.1, 0.2, 0.3, 1.0))
    dr.close()
    out = {"metric": f"ms per gradient step ({len(cams)}-view forward with checkpoints + backward)",
           "value": step_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": step_ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": desc},
           "forward_ms": fwd_ms, "backward_ms": step_ms - fwd_ms,
           "views_per_s": len(cams) * 1e3 / step_ms}
    print(json.dumps(out), flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes, not built)"}))
        return 2
    if args.summarize_pmc:
        return summarize_pmc(args)
    if args.summarize_sq:
        return summarize_sq(args)
    if args.workload == "c3":
        return bench_batch(args)
    if args.workload in ("c4", "c5-adjoint"):
        return bench_adjoint(args)
    import torch

    import paper_2501_01628_amd as dp

    if args.pmc_calibrate:
        calibration_copy()
    t0 = time.perf_counter()
    sc, desc = scene_for(args.workload)
    log(f"generated {sc.name} in {time.perf_counter() - t0:.1f} s")
    storage = dp.VR_F16 if args.storage == "f16" else dp.VR_F32
    if args.staging is None:
        args.staging = "slab" if args.storage == "f16" else "ring"
    r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale,
                    sc.step, storage=storage, device=0,
                    path=dp.VR_PATH_DIRECT if args.path == "direct" else dp.VR_PATH_STAGED,
                    march_config=(0 if args.staging == "slab" else 1,
                                  16 if args.staging == "slab" else args.tile_width, args.chunk))
    r.set_camera(sc.camera)
    r.synchronize()
    # drop the float32 upload copies: only the workspaces stay resident
    r.workspaces = [(ws, None) for ws, _ in r.workspaces]
    torch.cuda.empty_cache()
    log(f"ingested {len(sc.bricks)} bricks; rois {r.rois}")
    stream = r.stream
    elt = 2 if args.storage == "f16" else 4
    brick_bytes = [int(np.prod([d + 2 for d in dims])) * elt for dims, _ in r.meta]
    roi_px = [w * h for (_, _, w, h) in r.rois]
    march_alg = [bb + px * 20 + 4096 for bb, px in zip(brick_bytes, roi_px)]
    W, H = sc.camera["width"], sc.camera["height"]
    comp_alg = sum(roi_px) * 20 + W * H * 16
    bg = (0.0, 0.0, 0.0, 0.0)

    for _ in range(args.warmup):
        r.render(bg)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    nb = len(r.bricks)
    # one march launch per frame (all partials through one work queue), then the composite
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(2)] for _ in range(args.steps)]
    r.reset_samples()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        ev[s][0][0].record(stream)
        r.render_partials()
        ev[s][0][1].record(stream)
        ev[s][1][0].record(stream)
        r.composite(bg)
        ev[s][1][1].record(stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = t_total / args.steps * 1e3
    samples = int(r.sample_counts().sum()) // args.steps
    march_ms = np.zeros(1)
    comp_ms = 0.0
    for s in range(args.steps):
        march_ms[0] += ev[s][0][0].elapsed_time(ev[s][0][1])
        comp_ms += ev[s][1][0].elapsed_time(ev[s][1][1])
    march_ms /= args.steps
    comp_ms /= args.steps
    log(f"timed {args.steps} frames: {ms_per_step:.3f} ms/frame, march {march_ms.sum():.3f} ms, "
        f"composite {comp_ms:.3f} ms, {samples} samples/frame")

    achieved = sum(march_alg) / (march_ms.sum() * 1e-3) / 1e9
    traffic = traffic_for(args.workload, args.storage)
    out = {
        "metric": "Msamples/s (render+composite, samples evaluated per frame x frames/s)",
        "value": samples / (ms_per_step * 1e-3) / 1e6,
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "fps": 1e3 / ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "bricks": nb, "width": W, "height": H,
                   "storage": args.storage, "step_voxels": sc.step, "path": args.path,
                   "staging": args.staging,
                   "tile_width": 16 if args.staging == "slab" else args.tile_width,
                   "chunk_slices": None if args.staging == "slab" else args.chunk},
        "samples_per_frame": samples,
        "march_ms_per_frame": float(march_ms.sum()),
        "composite_ms_per_frame": comp_ms,
        "roofline": {
            "kernel": "march_queue (all bricks' partials, one persistent launch)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_gbs": traffic / (march_ms.sum() * 1e-3) / 1e9 if traffic else None,
            "launches_per_frame": 1,
            "algorithmic_bytes_per_frame": int(sum(march_alg)),
        },
        "valu": valu_for(args.workload, args.storage, float(march_ms.sum())),
        "composite_roofline": {"achieved": comp_alg / (comp_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "algorithmic_bytes": int(comp_alg)},
    }
    frame = r.frame.cpu().numpy()
    r.close()
    del r
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"], err = cpu_baseline(sc, args.cpu_seconds, frame)
        out["max_abs_err_vs_oracle"] = {"value": err, "pixels": "the cpu_baseline sample",
                                        "bar": 2e-3 if args.storage == "f16" else 1e-5}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

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
    ap.add_argument("--workload", choices=["c2", "c1", "c3", "c4", "c5", "c5-adjoint", "rqc", "stream", "tets",
                                                 "tets-mixed", "tets-shadow"],
                    default="c2")
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
    ap.add_argument("--view", type=float, nargs=2, metavar=("AZ", "EL"), default=None,
                    help="c1/c2/c5: orbit the camera to azimuth/elevation AZ EL degrees instead of the "
                         "workload's 30/20 (e.g. 90 0: rays along x, which no staged slab axis takes)")
    ap.add_argument("--tet-locator", choices=["grid", "bvh"], default="grid",
                    help="tets workloads: where a sample the walk misses is searched (same images)")
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


def host_info():
    """Host the oracle runs on: logical CPUs, the CPUs this process may use,
    and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)), "cpu_model": model}


def copy_bandwidth_gbs(nbytes=1 << 30, reps=10):
    """Streaming-copy bandwidth of this GPU (a 1 GiB device-to-device copy,
    read + write bytes per second), measured live for the HBM fractions."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / t / 1e9


def _oracle_rates(run, target_s, unit_scale, first=2000, cap=None):
    """Time ``run(n) -> (seconds, work, payload)`` on a sample sized for
    about target_s seconds (at most cap) with all of the oracle's threads,
    then on a smaller sample with one thread.  Rates are work / s *
    unit_scale."""
    import oracle
    t, _, _ = run(first)
    n = max(first, int(first * target_s / max(t, 1e-3)))
    if cap is not None:
        n = min(n, cap)
    t, work, payload = run(n)
    cores = oracle.threads()
    n1 = max(first // 4, int(n * min(1.0, (target_s / 4) / max(t * cores, 1e-3))))
    oracle.set_threads(1)
    try:
        t1, work1, _ = run(n1)
    finally:
        oracle.set_threads(cores)
    return {"value": work / t * unit_scale, "cores": cores, "n": n, "seconds": t, "work": work,
            "one_core_value": work1 / t1 * unit_scale, "one_core_n": n1, "one_core_seconds": t1,
            "payload": payload}


def cpu_baseline(sc, target_s, frame=None):
    """The oracle timed on a random pixel sample of the frame; with the GPU
    frame given, also its max error against the oracle at those pixels."""
    import numpy as np
    import oracle
    W, H = sc.camera["width"], sc.camera["height"]
    rng = np.random.default_rng(0)

    def run(npix):
        idx = rng.choice(W * H, min(npix, W * H), replace=False)
        pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
        t0 = time.perf_counter()
        img, _, cnt = oracle.render_scene(sc, pixels=pix)
        return time.perf_counter() - t0, int(cnt[0]), (pix, img)
    r = _oracle_rates(run, target_s, 1e-6, first=20000, cap=W * H)
    pix, img = r["payload"]
    out = {"value": r["value"], "unit": "Msamples/s", "cores": r["cores"], "kind": "oracle",
           "sample": f"{len(pix)} random pixels of the same frame, all {len(sc.bricks)} bricks + "
                     f"composite, {r['work']} samples (no early termination) in {r['seconds']:.1f} s",
           "one_core_value": r["one_core_value"],
           "one_core_sample": f"{min(r['one_core_n'], W * H)} random pixels, one thread, "
                              f"{r['one_core_seconds']:.1f} s",
           **host_info()}
    err = None
    if frame is not None:
        got = frame[pix[:, 1], pix[:, 0]].astype(np.float64)
        err = float(np.max(np.abs(got - img)))
    return out, err


def _c3_oracle_frame(d, frame, pix):
    """Oracle image of one C3 frame at pixels pix, and its owned samples."""
    import oracle
    t, f, c, ids = frame
    cam = d["cameras"][c]
    parts, samples = [], 0
    for i in ids:
        _, _, _, lo, vox = d["bricks"][i]
        nz, ny, nx = (s - 2 for s in vox.shape)
        rgba, depth, cnt = oracle.render_brick(cam, vox, (nx, ny, nz), 1, lo, (1, 1, 1), d["tf"], (0, 1),
                                               d["opacity_scale"], d["step"], 0.0, pix)
        parts.append((rgba, depth))
        samples += int(cnt[0])
    return oracle.composite(parts, (0.0, 0.0, 0.0, 0.0)), samples


def c3_pixel_sets(d, frame_list, target_s):
    """A seeded random pixel sample of every frame, sized so that the oracle
    renders all of them in about target_s seconds."""
    rng = np.random.default_rng(11)
    probe = frame_list[:: max(1, len(frame_list) // 4)]
    t0 = time.perf_counter()
    for fr in probe:
        cam = d["cameras"][fr[2]]
        idx = rng.choice(cam["width"] * cam["height"], 8000, replace=False)
        _c3_oracle_frame(d, fr, np.stack([idx % cam["width"], idx // cam["width"]], 1).astype(np.int32))
    per_px = (time.perf_counter() - t0) / (8000 * len(probe))
    W, H = d["cameras"][0]["width"], d["cameras"][0]["height"]
    n = int(min(W * H, max(500, target_s / (len(frame_list) * per_px))))
    sets = []
    for t, f, c, ids in frame_list:
        W, H = d["cameras"][c]["width"], d["cameras"][c]["height"]
        idx = rng.choice(W * H, min(n, W * H), replace=False)
        sets.append(np.stack([idx % W, idx // W], 1).astype(np.int32))
    return sets


def c3_oracle(d, frame_list, pix_sets, gpu_px, target_s):
    """The oracle on the pixel sample of all 72 frames (timed with all
    threads, then a part of it with one), and the per-frame max error of the
    float32 and float16 batches against it (float16 against the oracle on
    the original float32 field)."""
    import oracle
    errs = {k: [] for k in gpu_px}
    t0 = time.perf_counter()
    samples = 0
    for fi, (frame, pix) in enumerate(zip(frame_list, pix_sets)):
        ref, n = _c3_oracle_frame(d, frame, pix)
        samples += n
        for k in gpu_px:
            errs[k].append(float(np.max(np.abs(gpu_px[k][fi] - ref))))
    t = time.perf_counter() - t0
    cores = oracle.threads()
    # one thread on the first frames' samples, about target_s / 4 seconds
    n1 = max(1, int(len(frame_list) * min(1.0, (target_s / 4) / max(t * cores, 1e-3))))
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        s1 = sum(_c3_oracle_frame(d, frame_list[i], pix_sets[i])[1] for i in range(n1))
        t1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    npx = sum(len(p) for p in pix_sets)
    out = {"value": samples / t / 1e6, "unit": "Msamples/s", "cores": cores, "kind": "oracle",
           "sample": f"{npx} seeded random pixels over all {len(frame_list)} frames "
                     f"({len(pix_sets[0])} per frame), 14 bricks each + composite, {samples} samples "
                     f"(no early termination) in {t:.1f} s",
           "one_core_value": s1 / t1 / 1e6,
           "one_core_sample": f"the first {n1} frames' pixel samples, one thread, {t1:.1f} s",
           **host_info()}
    return out, errs


def bench_batch(args):
    """Batched workload: 14 uneven bricks x 6 time steps x 3 fields x 4 cameras
    at 1024^2 (1008 partial images, 72 frames): the plain path (per frame,
    one launch per brick + one composite) and the per-frame path (per frame,
    one persistent launch over its 14 partials + one composite) against the
    batch (one graph: persistent queued march + one composite launch for all
    frames), for float32 and float16 storage."""
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
    # frames in add_frame order, and a seeded pixel sample of each for the
    # oracle (per-image errors of both storages + the CPU baseline)
    frame_list = []
    for (t, f) in keys:
        ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
        for c in range(len(d["cameras"])):
            frame_list.append((t, f, c, ids))
    pix_sets = None
    if not args.no_cpu_baseline:
        pix_sets = c3_pixel_sets(d, frame_list, args.cpu_seconds)
    gpu_px = {}
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
        if pix_sets is not None:
            gpu_px[storage] = [br.frames[fi][torch.from_numpy(px[:, 1]).long().cuda(),
                                             torch.from_numpy(px[:, 0]).long().cuda()].double().cpu().numpy()
                               for fi, px in enumerate(pix_sets)]
        elt = 2 if storage == "f16" else 4
        roi_px = sum(w * h for (_, _, w, h), _, _ in br.parts)
        vol_bytes = sum(int(np.prod(vox.shape)) * elt for (_, _, _, _, vox) in d["bricks"])
        frame_px = sum(d["cameras"][c]["width"] * d["cameras"][c]["height"] for _, _, c, _ in frame_list)
        batch_alg = vol_bytes + roi_px * 40 + frame_px * 16
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

        # the single-frame path a caller without the batch API takes: per
        # frame, one persistent launch over the frame's partials + a composite
        fneed = dp.vr_frame_workspace_size(max(len(bs) for _, bs, _, _ in frame_parts))
        fws = torch.empty(fneed // 4 + 64, dtype=torch.float32, device="cuda")
        fbase = fws.data_ptr() + ((-fws.data_ptr()) % 256)

        def frame_pass():
            for c, bricks, parts, outf in frame_parts:
                dp.set_camera(ctx, d["cameras"][c])
                dp.vr_render_partials(ctx, bricks, parts, fbase, fneed)
                dp.vr_composite(ctx, parts, (0.0, 0.0, 0.0, 0.0), outf)
        frame_pass()
        torch.cuda.synchronize()
        e0.record(br.stream)
        for _ in range(plain_steps):
            frame_pass()
        e1.record(br.stream)
        torch.cuda.synchronize()
        per_frame_ms = e0.elapsed_time(e1) / plain_steps
        del fws

        # release groups: the batch split into 8 groups of 9 frames; time
        # from the launch to the first group's frames being written (seen by
        # a stream that waits for it) and to the whole batch
        n_groups = 8
        br.set_groups(n_groups)
        side = torch.cuda.Stream()
        eg = torch.cuda.Event(enable_timing=True)
        first_ms, grouped_ms = [], []
        for rep in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            e0.record(br.stream)
            br.launch()
            br.wait_group(0, side)
            eg.record(side)
            e1.record(br.stream)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                first_ms.append(e0.elapsed_time(eg))
                grouped_ms.append(e0.elapsed_time(e1))
        release = {"groups": n_groups, "frames_per_group": br.group(0)[1],
                   "first_group_ms": float(np.mean(first_ms)), "batch_ms": float(np.mean(grouped_ms))}
        br.set_groups(1)
        achieved = batch_alg / (batch_ms * 1e-3) / 1e9
        results[storage] = {"batch_ms": batch_ms, "plain_ms": plain_ms, "per_frame_launch_ms": per_frame_ms,
                            "samples": samples,
                            "roofline": {"kernel": "batch graph (march_queue over all 1008 partials "
                                                   "+ composite_many over all 72 frames)",
                                         "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                         "traffic": None, "algorithmic_bytes_per_batch": int(batch_alg)},
                            "autotune": {"wg_per_cu": wg, "order": ["as given", "by brick"][order],
                                         "staging": ["slab", "ring"][staging],
                                         "tile_width": tile_w, "chunk_slices": chunk,
                                         "tuned_ms": tuned_ms},
                            "msamples_per_s": samples / (batch_ms * 1e-3) / 1e6,
                            "speedup_vs_plain": plain_ms / batch_ms,
                            "speedup_vs_per_frame_launch": per_frame_ms / batch_ms,
                            "release_groups": release}
        log(f"c3 {storage}: {n_groups} release groups: first group {release['first_group_ms']:.3f} ms, "
            f"batch {release['batch_ms']:.3f} ms")
        log(f"c3 {storage}: batch {batch_ms:.3f} ms, per-frame launches {per_frame_ms:.3f} ms, "
            f"plain {plain_ms:.3f} ms, {samples} samples, "
            f"wg/cu {wg}, order {order}")
        br.close()
        torch.cuda.empty_cache()
    out["value"] = results["f32"]["msamples_per_s"]
    out["ms_per_step"] = results["f32"]["batch_ms"]
    out["storage"] = results
    copy_gbs = copy_bandwidth_gbs()
    r32 = results["f32"]["roofline"]
    out["roofline"] = {**r32, "copy_gbs": copy_gbs, "frac_of_copy": r32["achieved"] / copy_gbs}
    if pix_sets is not None:
        log("c3 oracle on the pixel sample of every frame ...")
        out["cpu_baseline"], errs = c3_oracle(d, frame_list, pix_sets, gpu_px, args.cpu_seconds)
        out["per_image_max_abs_err_vs_oracle"] = {
            "pixels": "a seeded random sample of every frame (count in cpu_baseline.sample)",
            "f32": [float("%.3g" % e) for e in errs["f32"]],
            "f16": [float("%.3g" % e) for e in errs["f16"]],
            "max_f32": max(errs["f32"]), "max_f16": max(errs["f16"]),
            "bars": {"f32": 1e-5, "f16 (vs the float32 field)": 2e-3}}
    else:
        out["cpu_baseline"] = None
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
    del vol, targets
    torch.cuda.empty_cache()
    # owned samples of all views (the forward march's counter, early
    # termination off): the nominal sample count of one gradient step
    r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], synth.default_tf(), sc.vrange, sc.opacity_scale,
                    sc.step, ert_eps=0.0, storage=storage, device=0)
    samples = 0
    for cam in cams:
        r.set_camera(cam)
        r.reset_samples()
        r.render()
        samples += int(r.sample_counts().sum())
    r.close()
    del r
    torch.cuda.empty_cache()
    evals = 3     # checkpointed forward, segment re-march, adjoint walk
    lane_ops = samples * evals * VALU_LANE_OPS_PER_SAMPLE
    achieved = lane_ops / (step_ms * 1e-3)
    peak = VALU_LANES_PER_CU_CYCLE * N_CU * CLOCK_HZ
    out = {"metric": f"ms per gradient step ({len(cams)}-view forward with checkpoints + backward)",
           "value": step_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": step_ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": desc},
           "forward_ms": fwd_ms, "backward_ms": step_ms - fwd_ms,
           "backward_over_forward": (step_ms - fwd_ms) / fwd_ms,
           "views_per_s": len(cams) * 1e3 / step_ms, "samples_per_step": samples,
           "roofline": {"kernel": "march_checkpointed + march_backward (+ composite and its backward)",
                        "bound": "alu", "achieved": achieved, "peak": peak, "unit": "lane-op/s",
                        "frac": achieved / peak, "traffic": None,
                        "model": f"{VALU_LANE_OPS_PER_SAMPLE} VALU lane-ops per sample evaluation, "
                                 f"{evals} evaluations per owned sample per step (checkpointed forward, "
                                 f"segment re-march, adjoint walk); peak = 64 lanes/CU/cycle x 256 CUs "
                                 f"x 2.4 GHz, unpacked fp32"}}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle gradient on a central crop) ...")
        out["cpu_baseline"] = adjoint_cpu_baseline(sc, cams, args.cpu_seconds, samples)
    print(json.dumps(out), flush=True)
    return 0


VALU_LANE_OPS_PER_SAMPLE = 48


def _crop_camera(cam, side):
    """The central side x side pixels of a perspective view as a camera of
    its own (same pixel rays)."""
    import math
    c = dict(cam)
    half = math.tan(math.radians(cam["fovy_deg"]) / 2.0) * side / cam["height"]
    c.update(width=side, height=side, fovy_deg=math.degrees(2.0 * math.atan(half)))
    return c


def adjoint_cpu_baseline(sc, cams, target_s, samples_per_step):
    """The oracle's reverse-mode gradient (forward + adjoint for the table
    and the voxels, every brick) on a central crop of the first view with a
    seeded upstream gradient, scaled by owned samples (the crop's, counted by
    the oracle, against the step's) to ms per gradient step over all views
    (the composite backward is not included)."""
    import oracle
    rng = np.random.default_rng(5)

    def run(side):
        cam = _crop_camera(cams[0], side)
        g = rng.uniform(-1.0, 1.0, (side, side, 4))
        t0 = time.perf_counter()
        for b in sc.bricks:
            oracle.render_brick_grad(cam, b.voxels, b.dims, b.ghost, b.origin, (1.0, 1.0, 1.0), sc.tf,
                                     sc.vrange, sc.opacity_scale, sc.step, g)
        t = time.perf_counter() - t0
        n = sum(int(oracle.render_brick(cam, b.voxels, b.dims, b.ghost, b.origin, (1.0, 1.0, 1.0), sc.tf,
                                        sc.vrange, sc.opacity_scale, sc.step)[2][0]) for b in sc.bricks)
        return t, max(n, 1)

    side = 16
    t, _ = run(side)
    side = int(min(cams[0]["height"], max(16, side * (target_s / max(t, 1e-3)) ** 0.5)))
    t, n = run(side)
    cores = oracle.threads()
    side1 = max(8, int(side * min(1.0, (target_s / 4 / max(t * cores, 1e-3))) ** 0.5))
    oracle.set_threads(1)
    try:
        t1, n1 = run(side1)
    finally:
        oracle.set_threads(cores)
    return {"value": t * samples_per_step / n * 1e3, "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": f"central {side}x{side} crop of view 0 ({n} owned samples), all {len(sc.bricks)} "
                      f"bricks' table and voxel gradients in {t:.1f} s, scaled to the step's "
                      f"{samples_per_step} owned samples",
            "one_core_value": t1 * samples_per_step / n1 * 1e3,
            "one_core_sample": f"central {side1}x{side1} crop ({n1} owned samples), one thread, {t1:.1f} s",
            **host_info()}


def rqc_scene():
    """Ray-queue-cycling workload: 96^3 field (8 blobs + a tanh shock), 6 kd
    bricks as ranks, 384x384 orbit view, step 0.5, one
    directional light at ambient 0.3 (opacity scale 0.25)."""
    import synth
    rng = np.random.default_rng(6)
    dims = (96, 96, 96)
    field = synth.tile_field(rng, dims, n_blobs=8, noise=0.0, shock=True)
    boxes = synth.kd_split(dims, 6, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, 384, 384)
    sc = synth.scene_from_field("rqc_96cube_6bricks", field, boxes, synth.default_tf(), cam, 0.5, 0.25)
    return sc, (0.8, 1.0, -0.4), 0.3


def bench_rqc(args):
    """Ray-queue cycling with shadow rays (bricks as ranks): the frame with
    the light, the same frame without shadow rays, and the sort-last frame of
    the same bricks for comparison."""
    import torch

    import oracle
    import paper_2501_01628_amd as dp
    sc, light, ambient = rqc_scene()
    r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale, sc.step, 0.0,
                    storage=dp.VR_F32, device=0)
    r.set_camera(sc.camera)
    total = r.rqc_plan()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    bg = (0.0, 0.0, 0.0, 0.0)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(r.stream)
        for _ in range(args.steps):
            fn()
        e1.record(r.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_shadow = timed(lambda: r.render_rqc(light, ambient, bg))
    cnt.zero_()
    r.render_rqc(light, ambient, bg, samples=cnt)
    torch.cuda.synchronize()
    samples = int(cnt.item())
    frame = r.frame.cpu().numpy().astype(np.float64)
    ms_plain = timed(lambda: r.render_rqc(light, 1.0, bg))
    ms_sortlast = timed(lambda: r.render(bg))
    r.close()
    W, H = sc.camera["width"], sc.camera["height"]
    peak = VALU_LANES_PER_CU_CYCLE * N_CU * CLOCK_HZ
    achieved = samples * VALU_LANE_OPS_PER_SAMPLE / (ms_shadow * 1e-3)
    out = {"metric": "Msamples/s (ray-queue-cycled frame with shadow rays: primary + shadow samples "
                     "evaluated per frame x frames/s)",
           "value": samples / (ms_shadow * 1e-3) / 1e6, "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_shadow, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"rqc: 96^3 f32 field (8 blobs + tanh shock), 6 kd bricks as ranks, "
                                  f"{W}x{H} perspective, step 0.5, opacity 0.25, light {light}, ambient {ambient}"},
           "samples_per_frame": samples, "primary_samples_per_frame": total,
           "ms_without_shadows": ms_plain, "ms_sort_last": ms_sortlast,
           "roofline": {"kernel": "rqc_shadow_step x 6 + rqc_primary_step x 6 + rqc_resolve", "bound": "alu",
                        "achieved": achieved, "peak": peak, "unit": "lane-op/s", "frac": achieved / peak,
                        "traffic": None,
                        "model": f"{VALU_LANE_OPS_PER_SAMPLE} VALU lane-ops per evaluated sample; peak = 64 "
                                 f"lanes/CU/cycle x 256 CUs x 2.4 GHz, unpacked fp32"}}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle with shadow rays on a pixel sample) ...")
        rng = np.random.default_rng(3)

        def run(npix):
            idx = rng.choice(W * H, min(npix, W * H), replace=False)
            pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
            t0 = time.perf_counter()
            img, _, _ = oracle.render_scene_shadowed(sc, light, ambient, pixels=pix)
            return time.perf_counter() - t0, len(pix), (pix, img)
        spp = samples / (W * H)       # primary + shadow samples per pixel, counted on the GPU
        rr = _oracle_rates(run, args.cpu_seconds, spp * 1e-6, first=200, cap=W * H)
        pix, img = rr["payload"]
        got = frame[pix[:, 1], pix[:, 0]]
        out["cpu_baseline"] = {
            "value": rr["value"], "unit": "Msamples/s", "cores": rr["cores"], "kind": "oracle",
            "sample": f"{len(pix)} random pixels with shadow rays in {rr['seconds']:.1f} s, pixels/s times "
                      f"the frame's {spp:.0f} primary + shadow samples per pixel",
            "one_core_value": rr["one_core_value"],
            "one_core_sample": f"{min(rr['one_core_n'], W * H)} random pixels, one thread, "
                               f"{rr['one_core_seconds']:.1f} s", **host_info()}
        out["max_abs_err_vs_oracle"] = {"value": float(np.max(np.abs(got - img))),
                                        "pixels": "the cpu_baseline sample", "bar": 1e-5}
    print(json.dumps(out), flush=True)
    return 0


def stream_scenes(n_steps=6):
    """Time-series workload: a 384x384x256 float32 field (16 blobs + a tanh
    front) advected along x by 8 voxels per step, n_steps steps, 8 kd bricks,
    1920x1080 orbit view, step 0.5, opacity scale 0.05."""
    import synth
    dims = (384, 384, 256)
    rng = np.random.default_rng(7)
    base = synth.tile_field(rng, dims, n_blobs=16, noise=0.0, shock=True)
    boxes = synth.kd_split(dims, 8, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, 1920, 1080)
    return [synth.scene_from_field(f"stream{t}", np.roll(base, 8 * t, axis=2), boxes, synth.default_tf(), cam,
                                   0.5, 0.05) for t in range(n_steps)], cam


def bench_stream(args):
    """Playback of a time series with two resident steps (each frame uploads
    the next step over the host link while the current one renders) against
    the same frames with every step resident."""
    import torch

    import paper_2501_01628_amd as dp
    t0 = time.perf_counter()
    scenes, cam = stream_scenes()
    log(f"generated {len(scenes)} time steps in {time.perf_counter() - t0:.1f} s")
    steps = [[(b.voxels, b.lo) for b in sc.bricks] for sc in scenes]
    sc0 = scenes[0]
    T = len(scenes)
    step_bytes = sum(int(np.prod(v.shape)) * 4 for v, _ in steps[0])

    def play(slots, rounds):
        sr = dp.StreamRenderer(steps, sc0.tf, sc0.vrange, sc0.opacity_scale, sc0.step, slots=slots)
        sr.set_camera(cam)
        order = [t for _ in range(rounds) for t in range(T)]
        for i, t in enumerate(order[:T]):                 # warm-up pass (loads every step once)
            sr.render(t, prefetch=order[i + 1] if i + 1 < len(order) else None)
        torch.cuda.synchronize()
        loads0, _ = sr.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sr.stream)
        timed = order[T:]
        for i, t in enumerate(timed):
            sr.render(t, prefetch=timed[i + 1] if i + 1 < len(timed) else None)
        e1.record(sr.stream)
        torch.cuda.synchronize()
        loads, _ = sr.stats()
        ms = e0.elapsed_time(e1) / len(timed)
        frame = sr.frame.cpu().numpy()
        sr.close()
        return ms, loads - loads0, len(timed), frame

    rounds = 1 + max(1, args.steps // T)
    ms_stream, loads, frames, frame = play(2, rounds)
    ms_resident, loads_res, _, _ = play(T, rounds)
    W, H = cam["width"], cam["height"]
    out = {"metric": "frames/s (time-series playback, 2 of 6 time steps resident, next step uploaded "
                     "during each frame)",
           "value": 1e3 / ms_stream, "unit": "frames/s", "n_gpus": 1, "steps": frames, "warmup": T,
           "ms_per_step": ms_stream, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"stream: 384x384x256 f32 field advected 8 voxels per step, {T} steps, 8 kd "
                                  f"bricks, {W}x{H} perspective, step 0.5, opacity 0.05, 2 resident slots"},
           "ms_all_resident": ms_resident, "loads_per_frame": loads / frames,
           "bytes_uploaded_per_step": step_bytes,
           "h2d": {"achieved": step_bytes * loads / frames / (ms_stream * 1e-3) / 1e9, "peak": 64.0,
                   "unit": "GB/s", "frac": step_bytes * loads / frames / (ms_stream * 1e-3) / 1e9 / 64.0,
                   "peak_source": "PCIe 5.0 x16, one direction"},
           "roofline": {"kernel": "time-series frame: host-to-device upload of the next step (copy stream) "
                                  "overlapped with march + composite of the current one",
                        "bound": "hbm", "traffic": None,
                        "achieved": (step_bytes * loads / frames * 2) / (ms_stream * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": (step_bytes * loads / frames * 2) / (ms_stream * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "note": "HBM bytes of the upload and its ingest (write + read of each step) per "
                                "frame; the frame is bound by the host link (see h2d)"}}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle on a pixel sample of the last step) ...")
        sc = scenes[(frames + T - 1) % T]
        rng = np.random.default_rng(0)

        def run(npix):
            idx = rng.choice(W * H, min(npix, W * H), replace=False)
            pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
            t0 = time.perf_counter()
            img, _, _ = oracle.render_scene(sc, pixels=pix)
            return time.perf_counter() - t0, len(pix), (pix, img)
        # rates in pixels/s x 1 / (W H) = frames/s
        rr = _oracle_rates(run, args.cpu_seconds, 1.0 / (W * H), first=20000, cap=W * H)
        pix, img = rr["payload"]
        out["cpu_baseline"] = {"value": rr["value"], "unit": "frames/s", "cores": rr["cores"], "kind": "oracle",
                               "sample": f"{len(pix)} random pixels of the last step's frame in "
                                         f"{rr['seconds']:.1f} s, scaled by pixel count (no upload: the "
                                         f"oracle reads host memory)",
                               "one_core_value": rr["one_core_value"],
                               "one_core_sample": f"{min(rr['one_core_n'], W * H)} random pixels, one thread, "
                                                  f"{rr['one_core_seconds']:.1f} s", **host_info()}
        out["max_abs_err_vs_oracle"] = {"value": float(np.max(np.abs(frame[pix[:, 1], pix[:, 0]] - img))),
                                        "pixels": "the cpu_baseline sample", "bar": 1e-5}
    print(json.dumps(out), flush=True)
    return 0


def tet_scene(cells=(128, 96, 96), n_parts=16, width=1920, height=1080):
    """Tetrahedral workload: a 128x96x96-cube box cut into 7.1 M tetrahedra
    (6 per cube, interior vertices jittered by up to 0.15 of a cube, 1.2 M
    vertices), 8 Gaussian blobs evaluated at the vertices, 16 uneven
    non-convex parts (weighted nearest seed + noise per tetrahedron),
    1920x1080 orbit view, step 0.5 cube, opacity scale 0.05."""
    import synth
    rng = np.random.default_rng(12)
    v, t = synth.tet_mesh(cells, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, cells, n_blobs=8)
    parts = synth.tet_partitions(v, t, n_parts, rng)
    cam = synth.orbit_camera((0, 0, 0), cells, width, height)
    return vals, parts, cam, len(t), len(v)


# fp64 operations per held sample in the tetrahedral march when the first
# tetrahedron tested holds it: the sample position (t = (k + 1/2) dt, p = o +
# t d: 8), four face sub-volumes (3 multiplies + 3 adds each: 24) and the
# barycentric value (3 adds for the sum, 4 multiplies + 3 adds, 1 divide: 11)
TET_FP64_OPS_PER_SAMPLE = 43
FP64_VECTOR_PEAK = 78.6e12


def mixed_scene(cells=(96, 72, 72), n_parts=16, width=1920, height=1080):
    """Mixed-element workload: a 96x72x72-cube box (jitter 0.15) whose
    cubes are, by 2-cube blocks, hexahedra, wedge pairs, six pyramids around
    a centre vertex, or six Kuhn tetrahedra (1,866,240 cells, 641,329
    vertices), 8 blobs at the vertices, 16 smooth non-convex parts by cell
    centroid, 1920x1080 orbit view, step 0.5 cube, opacity 0.05."""
    import synth
    rng = np.random.default_rng(14)
    v, sz, cv = synth.mixed_mesh(cells, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, cells, n_blobs=8)
    parts = synth.mixed_partitions(v, sz, cv, n_parts, rng)
    cam = synth.orbit_camera((0, 0, 0), cells, width, height)
    return vals, parts, cam, len(sz), len(v)


def bench_tets(args):
    """Unstructured data: a tetrahedral (or, for tets-mixed, mixed-element)
    mesh in 16 non-convex parts; one step = the march of every part into
    runs + the per-pixel resolve."""
    import torch

    import paper_2501_01628_amd as dp
    import synth
    mixed = args.workload == "tets-mixed"
    t0 = time.perf_counter()
    if mixed:
        vals, parts, cam, n_cells, n_verts = mixed_scene()
        box = (96.0, 72.0, 72.0)
    else:
        vals, parts, cam, n_cells, n_verts = tet_scene()
        box = (128.0, 96.0, 96.0)
    log(f"generated {n_cells} cells in {len(parts)} parts in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    tf = synth.default_tf()
    r = dp.TetRenderer([p if mixed else p[:2] for p in parts], tf, (0.0, 1.0), 0.05, 0.5, max_runs=32,
                       locator=dp.VR_TET_BVH if args.tet_locator == "bvh" else dp.VR_TET_GRID)
    host_build_s = time.perf_counter() - t0
    n_tets = sum(i["n_tets"] for i in r.info)
    for k, part in enumerate(parts):
        r.set_values(k, vals[part[-1]])
    r.set_camera(cam)
    r.synchronize()
    r.values = [None] * len(parts)
    torch.cuda.empty_cache()
    grid_entries = sum(i["grid_entries"] for i in r.info)
    table_bytes = sum(i["workspace_bytes"] for i in r.info)
    log(f"tables built in {host_build_s:.1f} s: {table_bytes / 1e9:.2f} GB on the device, "
        f"{grid_entries} grid entries ({grid_entries / n_tets:.1f} per tetrahedron)")
    bg = (0.0, 0.0, 0.0, 0.0)
    for _ in range(args.warmup):
        r.render(bg)
    r.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(r.stream)
        r.march()
        ev[s][1].record(r.stream)
        r.resolve(bg)
        ev[s][2].record(r.stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    r.synchronize()
    ms_per_step = t_total / args.steps * 1e3
    march_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    resolve_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps
    r.samples.zero_()
    r.render(bg, count=True)
    r.synchronize()
    held = int(r.samples.item())
    frame = r.frame.cpu().numpy().astype(np.float64)
    r.close()
    log(f"timed {args.steps} frames: {ms_per_step:.3f} ms/frame, march {march_ms:.3f} ms, resolve "
        f"{resolve_ms:.3f} ms, {held} held samples/frame")
    W, H = cam["width"], cam["height"]
    achieved = held * TET_FP64_OPS_PER_SAMPLE / (march_ms * 1e-3)
    if mixed:
        wl = (f"tets-mixed: {n_cells} cells (hexahedra, wedges, pyramids, tetrahedra of jittered 96x72x72 "
              f"cubes; {n_tets} tetrahedra after the cut, {n_verts} vertices), 8 blobs, {len(parts)} non-convex "
              f"parts, {W}x{H} perspective, step 0.5, opacity 0.05, max 32 runs per ray and part")
    else:
        wl = (f"tets: {n_tets} tetrahedra ({n_verts} vertices, jittered 128x96x96 cubes), 8 blobs, "
              f"{len(parts)} non-convex parts, {W}x{H} perspective, step 0.5, opacity 0.05, max 32 runs per ray "
              f"and part")
    out = {"metric": "Msamples/s (tetrahedral parts: samples held by a tetrahedron per frame x frames/s)",
           "value": held / (ms_per_step * 1e-3) / 1e6, "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "fps": 1e3 / ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 location, f32 shading", "data": "synthetic",
           "config": {"workload": wl, "locator": args.tet_locator},
           "samples_per_frame": held, "ms_march": march_ms, "ms_resolve": resolve_ms,
           "host_table_build_s": host_build_s, "device_table_bytes": table_bytes,
           "grid_entries_per_tet": grid_entries / n_tets,
           "roofline": {"kernel": "tet_march", "bound": "alu", "achieved": achieved / 1e12,
                        "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK,
                        "traffic": None,
                        "model": f"{TET_FP64_OPS_PER_SAMPLE} fp64 operations per held sample (position, four "
                                 f"face sub-volumes, barycentric value) over the march launch; peak = fp64 "
                                 f"vector 78.6 TFLOP/s"}}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle, brute-force location, on a pixel sample) ...")
        rng = np.random.default_rng(5)
        if mixed:
            tparts = [oracle.cells_to_tets(pv, vals[used], psz, pcv, vertex_ids=used) for pv, psz, pcv, used in parts]
        else:
            tparts = [(pv, vals[used], pt) for pv, pt, used in parts]
        # The oracle tests every sample against every tetrahedron (about 0.3 s
        # per sample here), so the sample is pixels whose rays cross the mesh
        # box in a short chord (8 to 24 samples; the mesh fills its box, so
        # every one of them is held): its rate per sample is the oracle's.
        hit = np.argwhere(frame[..., 3] > 0.0)
        cand = hit[rng.choice(len(hit), min(20000, len(hit)), replace=False)]
        hi = np.array(box)
        short = []
        for j, i in cand:
            o, d = oracle.ray(cam, int(i), int(j))
            with np.errstate(divide="ignore", invalid="ignore"):
                ta, tb = (0.0 - o) / d, (hi - o) / d
            chord = np.min(np.maximum(ta, tb)) - max(np.max(np.minimum(ta, tb)), 0.0)
            if 8 * 0.5 <= chord <= 24 * 0.5:
                short.append((i, j))
        short = np.array(short, dtype=np.int32)

        def run(npix):
            pix = short[rng.choice(len(short), min(npix, len(short)), replace=False)]
            log(f"oracle on {len(pix)} pixels with {oracle.threads()} threads ...")
            t0 = time.perf_counter()
            img, cnt = oracle.render_tets(cam, tparts, tf, (0.0, 1.0), 0.05, 0.5, bg, pixels=pix)
            return time.perf_counter() - t0, int(cnt[0]), (pix, img)
        rr = _oracle_rates(run, args.cpu_seconds, 1e-6, first=oracle.threads(), cap=len(short))
        pix, img = rr["payload"]
        out["cpu_baseline"] = {
            "value": rr["value"], "unit": "Msamples/s", "cores": rr["cores"], "kind": "oracle",
            "sample": f"{len(pix)} random pixels whose rays cross the mesh box in 8 to 24 samples, "
                      f"{rr['work']} held samples in {rr['seconds']:.1f} s (every sample tested against all "
                      f"{n_tets} tetrahedra)",
            "one_core_value": rr["one_core_value"],
            "one_core_sample": f"{rr['one_core_n']} random pixels, one thread, {rr['one_core_seconds']:.1f} s",
            **host_info()}
        out["max_abs_err_vs_oracle"] = {"value": float(np.max(np.abs(frame[pix[:, 1], pix[:, 0]] - img))),
                                        "pixels": "the cpu_baseline sample", "bar": 1e-5}
    print(json.dumps(out), flush=True)
    return 0


def bench_tets_shadow(args):
    """Shadow rays through tetrahedral parts: a 64x48x48-cube box (884,736
    tetrahedra, jitter 0.15), 8 blobs, 8 smooth non-convex parts, 768x768
    orbit view, step 0.5, opacity 0.1, light (0.8, 1.0, -0.4), ambient 0.3.
    One step = record + 8 shadow cycle steps + shaded march + resolve (the
    plan, which depends on geometry and camera only, is made once)."""
    import torch

    import paper_2501_01628_amd as dp
    import synth
    cells, n_parts, light, a0 = (64, 48, 48), 8, (0.8, 1.0, -0.4), 0.3
    rng = np.random.default_rng(13)
    v, t = synth.tet_mesh(cells, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, cells, n_blobs=8)
    parts = synth.tet_partitions(v, t, n_parts, rng)
    cam = synth.orbit_camera((0, 0, 0), cells, 768, 768)
    tf = synth.default_tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, (0.0, 1.0), 0.1, 0.5, max_runs=32,
                       locator=dp.VR_TET_BVH if args.tet_locator == "bvh" else dp.VR_TET_GRID)
    for k, (_, _, used) in enumerate(parts):
        r.set_values(k, vals[used])
    r.set_camera(cam)
    total = r.shadow_plan()
    bg = (0.0, 0.0, 0.0, 0.0)
    for _ in range(args.warmup):
        r.render_shadowed(light, a0, bg)
    r.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(r.stream)
    for _ in range(args.steps):
        r.render_shadowed(light, a0, bg)
    e1.record(r.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    r.samples.zero_()
    r.render_shadowed(light, a0, bg, count=True)
    r.synchronize()
    samples = int(r.samples.item())
    frame = r.frame.cpu().numpy().astype(np.float64)
    e0.record(r.stream)
    for _ in range(args.steps):
        r.render(bg)
    e1.record(r.stream)
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / args.steps
    r.close()
    log(f"shadowed frame {ms:.3f} ms ({total} primary + {samples - total} shadow samples), unshadowed {ms_plain:.3f} ms")
    achieved = samples * TET_FP64_OPS_PER_SAMPLE / (ms * 1e-3)
    W, H = cam["width"], cam["height"]
    out = {"metric": "Msamples/s (tetrahedral parts with shadow rays: primary + shadow samples held per frame x "
                     "frames/s)",
           "value": samples / (ms * 1e-3) / 1e6, "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 location, f32 shading", "data": "synthetic",
           "config": {"workload": f"tets-shadow: {len(t)} tetrahedra (jittered 64x48x48 cubes), 8 blobs, {n_parts} "
                                  f"non-convex parts, {W}x{H} perspective, step 0.5, opacity 0.1, light {light}, "
                                  f"ambient {a0}"},
           "samples_per_frame": samples, "primary_samples_per_frame": total, "ms_without_shadows": ms_plain,
           "roofline": {"kernel": "tet_march<record> + tet_shadow_step x 8 + tet_march<shaded> + tet_resolve",
                        "bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                        "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK, "traffic": None,
                        "model": f"{TET_FP64_OPS_PER_SAMPLE} fp64 operations per held (primary or shadow) sample "
                                 f"over the frame; peak = fp64 vector 78.6 TFLOP/s"}}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle with shadow rays, brute-force location, on a pixel sample) ...")
        tparts = [(pv, vals[used], pt) for pv, pt, used in parts]
        hit = np.argwhere(frame[..., 3] > 0.0)
        pick = np.random.default_rng(3)
        cand = hit[pick.choice(len(hit), min(20000, len(hit)), replace=False)]
        hi = np.array(cells, dtype=np.float64)
        short = []
        for j, i in cand:
            o, d = oracle.ray(cam, int(i), int(j))
            with np.errstate(divide="ignore", invalid="ignore"):
                ta, tb = (0.0 - o) / d, (hi - o) / d
            chord = np.min(np.maximum(ta, tb)) - max(np.max(np.minimum(ta, tb)), 0.0)
            if 2 * 0.5 <= chord <= 6 * 0.5:
                short.append((i, j))
        short = np.array(short, dtype=np.int32)

        def run(npix):
            pix = short[pick.choice(len(short), min(npix, len(short)), replace=False)]
            log(f"oracle on {len(pix)} pixels with {oracle.threads()} threads ...")
            t0 = time.perf_counter()
            img, cnt = oracle.render_tets_shadowed(cam, tparts, tf, (0.0, 1.0), 0.1, 0.5, light, a0, bg, pixels=pix)
            return time.perf_counter() - t0, int(cnt[0] + cnt[2]), (pix, img)
        rr = _oracle_rates(run, args.cpu_seconds, 1e-6, first=oracle.threads(), cap=len(short))
        pix, img = rr["payload"]
        out["cpu_baseline"] = {
            "value": rr["value"], "unit": "Msamples/s", "cores": rr["cores"], "kind": "oracle",
            "sample": f"{len(pix)} random pixels whose rays cross the mesh box in 2 to 6 samples, {rr['work']} "
                      f"primary + shadow samples in {rr['seconds']:.1f} s (every sample tested against all "
                      f"{len(t)} tetrahedra)",
            "one_core_value": rr["one_core_value"],
            "one_core_sample": f"{rr['one_core_n']} random pixels, one thread, {rr['one_core_seconds']:.1f} s",
            **host_info()}
        out["max_abs_err_vs_oracle"] = {"value": float(np.max(np.abs(frame[pix[:, 1], pix[:, 0]] - img))),
                                        "pixels": "the cpu_baseline sample", "bar": 1e-5}
    print(json.dumps(out), flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: --gpus must be 1 "
                                   "(sharding over several GPUs is not built)"}))
        return 2
    if args.summarize_pmc:
        return summarize_pmc(args)
    if args.summarize_sq:
        return summarize_sq(args)
    if args.workload == "c3":
        return bench_batch(args)
    if args.workload in ("c4", "c5-adjoint"):
        return bench_adjoint(args)
    if args.workload == "rqc":
        return bench_rqc(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload in ("tets", "tets-mixed"):
        return bench_tets(args)
    if args.workload == "tets-shadow":
        return bench_tets_shadow(args)
    import torch

    import paper_2501_01628_amd as dp

    if args.pmc_calibrate:
        calibration_copy()
    t0 = time.perf_counter()
    sc, desc = scene_for(args.workload)
    if args.view is not None:
        import synth
        az, el = args.view
        cam = sc.camera
        sc.camera = synth.orbit_camera((0, 0, 0), sc.dims, cam["width"], cam["height"], az_deg=az, el_deg=el,
                                       fovy_deg=cam["fovy_deg"])
        desc += f", camera orbited to azimuth {az:g} / elevation {el:g} degrees"
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
    # the committed counter records were taken with the workload's own view
    traffic = traffic_for(args.workload, args.storage) if args.view is None else None
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
        "valu": valu_for(args.workload, args.storage, float(march_ms.sum())) if args.view is None else None,
        "composite_roofline": {"achieved": comp_alg / (comp_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "algorithmic_bytes": int(comp_alg)},
    }
    frame = r.frame.cpu().numpy()
    r.close()
    del r
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth_gbs()
    out["roofline"]["copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    out["composite_roofline"]["frac"] = out["composite_roofline"]["achieved"] / HBM_PEAK_GBS
    out["composite_roofline"]["frac_of_copy"] = out["composite_roofline"]["achieved"] / copy_gbs
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

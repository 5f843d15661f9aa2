"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars: max |GPU - oracle| <= 1e-5 per RGBA channel with float32 storage,
<= 2e-3 with float16 storage (measured against the oracle on the original
float32 field); depth keys are compared exactly (the GPU's float32 key of
t = (k + 1/2) dt is exact for the lattice sizes used here, and both sides
decide ownership in float64 with the same operation order).  Pixels outside
a partial's region of interest must be empty in the oracle's partial.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 2e-3
BG = (0.1, 0.2, 0.3, 1.0)


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_01628_amd as m
    return m


def _renderer(dp, scene, storage=0, ert=2.0 ** -20, fields=None):
    bricks = [(b.voxels if fields is None else fields[k], b.lo) for k, b in enumerate(scene.bricks)]
    return dp.Renderer(bricks, scene.tf, scene.vrange, scene.opacity_scale, scene.step, ert,
                       storage=storage)


def _gpu_frame(r, cam, bg):
    r.set_camera(cam)
    img = r.render(bg)
    r.synchronize()
    parts = []
    for k in range(len(r.bricks)):
        rgba, depth = r.partial_arrays(k)
        parts.append((r.rois[k], rgba.cpu().numpy().astype(np.float64),
                      depth.cpu().numpy().astype(np.float64)))
    return img.cpu().numpy().astype(np.float64), parts


def _check_partials(parts_gpu, parts_ref, tol):
    worst = 0.0
    for (roi, rg, dg), (rr, dr) in zip(parts_gpu, parts_ref):
        x0, y0, w, h = roi
        sub_r = rr[y0:y0 + h, x0:x0 + w]
        sub_d = dr[y0:y0 + h, x0:x0 + w]
        worst = max(worst, float(np.max(np.abs(rg - sub_r))) if rg.size else 0.0)
        assert np.array_equal(dg, sub_d.astype(np.float32).astype(np.float64)), "depth keys differ"
        # outside the ROI the oracle's partial must be empty
        mask = np.ones(dr.shape, bool)
        mask[y0:y0 + h, x0:x0 + w] = False
        assert np.all(np.isinf(dr[mask])) and np.all(rr[mask] == 0), "ROI misses owned samples"
    assert worst <= tol, worst
    return worst


def _scene_small(seed, dims, n_bricks, w, h, az=30.0, el=20.0, radius=2.0, scale=1.0, step=0.5):
    rng = np.random.default_rng(seed)
    field = synth.tile_field(rng, dims, n_blobs=6, noise=0.02, shock=True)
    boxes = synth.kd_split(dims, n_bricks, rng) if n_bricks > 1 else [((0, 0, 0), tuple(dims))]
    cam = synth.orbit_camera((0, 0, 0), dims, w, h, az_deg=az, el_deg=el, radius_factor=radius)
    return synth.scene_from_field(f"s{seed}", field, boxes, synth.default_tf(), cam, step, scale)


# ------------------------------------------------------------- worked examples
def test_worked_examples_on_gpu(dp):
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))
    for name in ("W1", "W2"):
        tf = np.zeros((256, 4), np.float32)
        x = np.arange(256) / 255.0
        if name == "W1":
            tf[:, :3] = 1.0
        else:
            tf[:, 0], tf[:, 1], tf[:, 2] = x, 1 - x, 0.25
        tf[:, 3] = x
        va = np.repeat(np.repeat(np.array([0.0, 0.0, 1.0], np.float32)[None, None], 3, 1), 3, 0)
        vb = np.repeat(np.repeat(np.array([0.0, 1.0, 1.0], np.float32)[None, None], 3, 1), 3, 0)
        r = dp.Renderer([(va, (0, 0, 0)), (vb, (1, 0, 0))], tf, (0, 1), 1.0, 0.5, 0.0)
        cam = dict(kind="ortho", eye=(0.0, 0.5, 0.5), dir=(1.0, 0, 0), up=(0, 1.0, 0), width=1,
                   height=1, view_height=1.0)
        img, parts = _gpu_frame(r, cam, gold["bg"])
        r.close()
        assert np.max(np.abs(img[0, 0] - np.array(gold[name]["final_bg"]))) < 1e-6
        assert parts[0][2][0, 0] == 0.25 and parts[1][2][0, 0] == 1.25


# --------------------------------------------------------------------- C1
def test_c1_partials_and_frame(dp):
    sc = synth.config_c1()
    r = _renderer(dp, sc)
    img, parts = _gpu_frame(r, sc.camera, BG)
    r.close()
    ref, ref_parts, cnt = oracle.render_scene(sc, bg=BG)
    _check_partials(parts, ref_parts, TOL32)
    assert np.max(np.abs(img - ref)) <= TOL32
    assert cnt[0] > 1e6


@pytest.mark.parametrize("seed,dims,nb,w,h,az,el,radius", [
    (101, (37, 29, 23), 5, 61, 47, 30.0, 20.0, 2.0),      # ragged ROI / tile tails
    (102, (40, 40, 40), 8, 64, 64, 125.0, -35.0, 1.7),    # x-dominant view, from below
    (103, (17, 50, 31), 3, 33, 71, 250.0, 60.0, 2.5),     # steep elevation
    (104, (48, 24, 16), 6, 80, 40, 0.0, 0.0, 2.0),        # axis-aligned view
])
def test_random_scenes(dp, seed, dims, nb, w, h, az, el, radius):
    sc = _scene_small(seed, dims, nb, w, h, az, el, radius, scale=4.0)
    r = _renderer(dp, sc)
    img, parts = _gpu_frame(r, sc.camera, BG)
    r.close()
    ref, ref_parts, _ = oracle.render_scene(sc, bg=BG)
    _check_partials(parts, ref_parts, TOL32)
    assert np.max(np.abs(img - ref)) <= TOL32


def test_camera_inside_volume(dp):
    """Eye inside the data: every ROI is the whole frame, rays start inside
    a brick."""
    sc = _scene_small(105, (40, 36, 30), 6, 48, 40, scale=4.0)
    cam = synth.inside_camera((0, 0, 0), (40, 36, 30), 48, 40, fovy_deg=70.0)
    r = _renderer(dp, sc)
    img, parts = _gpu_frame(r, cam, BG)
    r.close()
    ref, ref_parts, _ = oracle.render_scene(sc, camera=cam, bg=BG)
    assert all(p[0] == (0, 0, 48, 40) for p in parts)
    _check_partials(parts, ref_parts, TOL32)
    assert np.max(np.abs(img - ref)) <= TOL32


def test_orthographic_and_fine_step(dp):
    sc = _scene_small(106, (30, 30, 30), 4, 40, 40, scale=3.0, step=0.25)
    cam = dict(kind="ortho", eye=(15.0, 15.0, 60.0), dir=(0.1, -0.2, -1.0), up=(0, 1.0, 0),
               width=40, height=40, view_height=36.0)
    r = _renderer(dp, sc)
    img, parts = _gpu_frame(r, cam, BG)
    r.close()
    ref, ref_parts, _ = oracle.render_scene(sc, camera=cam, bg=BG)
    _check_partials(parts, ref_parts, TOL32)
    assert np.max(np.abs(img - ref)) <= TOL32


# ---------------------------------------------------------- special cases
def test_empty_volume_is_background_bitwise(dp):
    sc = _scene_small(107, (20, 20, 20), 3, 32, 24)
    tf = sc.tf.copy()
    tf[:, 3] = 0.0
    sc.tf = tf
    r = _renderer(dp, sc)
    img, _ = _gpu_frame(r, sc.camera, BG)
    r.close()
    assert np.array_equal(img.astype(np.float32), np.broadcast_to(np.float32(BG), img.shape))


def test_split_invariance_on_gpu(dp):
    rng = np.random.default_rng(108)
    dims = (36, 28, 20)
    field = synth.tile_field(rng, dims, n_blobs=6, shock=True)
    cam = synth.orbit_camera((0, 0, 0), dims, 56, 44, az_deg=40.0)
    tf = synth.default_tf()
    whole = synth.scene_from_field("w", field, [((0, 0, 0), dims)], tf, cam, 0.5, 3.0)
    split = synth.scene_from_field("s", field, synth.kd_split(dims, 7, rng), tf, cam, 0.5, 3.0)
    out = []
    for sc in (whole, split):
        r = _renderer(dp, sc)
        out.append(_gpu_frame(r, cam, BG)[0])
        r.close()
    assert np.max(np.abs(out[0] - out[1])) <= TOL32


def test_forward_is_deterministic(dp):
    sc = _scene_small(109, (32, 32, 32), 4, 64, 48, scale=2.0)
    r = _renderer(dp, sc)
    a, _ = _gpu_frame(r, sc.camera, BG)
    b, _ = _gpu_frame(r, sc.camera, BG)
    r.close()
    assert np.array_equal(a, b)


def test_ert_off_matches_no_termination(dp):
    sc = _scene_small(110, (24, 24, 24), 2, 40, 40, scale=40.0)
    r = _renderer(dp, sc, ert=0.0)
    img, parts = _gpu_frame(r, sc.camera, BG)
    r.close()
    ref, ref_parts, cnt = oracle.render_scene(sc, bg=BG, ert_eps=2.0 ** -20)
    assert cnt[1] < cnt[0]          # the view does saturate
    _check_partials(parts, ref_parts, TOL32)
    assert np.max(np.abs(img - ref)) <= TOL32


# -------------------------------------------------------------------- FP16
def test_fp16_storage(dp):
    sc = synth.config_c1()
    r = _renderer(dp, sc, storage=dp.VR_F16)
    img, parts = _gpu_frame(r, sc.camera, BG)
    r.close()
    ref, _, _ = oracle.render_scene(sc, bg=BG)
    err_orig = float(np.max(np.abs(img - ref)))
    assert err_orig <= TOL16, err_orig
    dec = [b.voxels.astype(np.float16).astype(np.float32) for b in sc.bricks]
    ref_dec, ref_parts_dec, _ = oracle.render_scene(sc, bg=BG, field_override=dec)
    _check_partials(parts, ref_parts_dec, TOL32)     # kernel error alone
    assert np.max(np.abs(img - ref_dec)) <= TOL32


# --------------------------------------------------------------- composite
@pytest.mark.parametrize("n,seed,ties", [(1, 1, False), (7, 2, False), (64, 3, False), (7, 4, True),
                                         (64, 5, True)])
def test_composite_kernel_random_partials(dp, n, seed, ties):
    """Random ROIs (ragged, overlapping, some empty pixels, +inf keys) and
    random premultiplied values: the GPU composite equals the oracle's.  With
    ``ties`` the keys take three values only, so most pixels hold equal keys
    of several partials (taken in partial-index order) and more than four
    finite keys."""
    rng = np.random.default_rng(seed)
    W, H = (150, 37) if ties else (77, 45)
    ctx = dp.vr_context_create(0, torch.cuda.current_stream())
    dp.vr_set_camera_perspective(ctx, (0, 0, 10.0), (0, 0, 0), (0, 1.0, 0), 45.0, W, H)
    parts, bufs, ref_parts = [], [], []
    for p in range(n):
        w, h = int(rng.integers(1, W + 1)), int(rng.integers(1, H + 1))
        x0, y0 = int(rng.integers(0, W - w + 1)), int(rng.integers(0, H - h + 1))
        A = rng.uniform(0, 1, (h, w)).astype(np.float32)
        rgb = (A[..., None] * rng.uniform(0, 1, (h, w, 3))).astype(np.float32)
        rgba = np.concatenate([rgb, A[..., None]], -1)
        if ties:
            depth = rng.integers(0, 3, (h, w)).astype(np.float32)
        else:
            depth = rng.uniform(0.0, 1000.0, (h, w)).astype(np.float32)
        depth[rng.uniform(0, 1, (h, w)) < 0.2] = np.inf
        rgba[np.isinf(depth)] = 0
        tr = torch.from_numpy(rgba).cuda().contiguous()
        td = torch.from_numpy(depth).cuda().contiguous()
        bufs.append((tr, td))
        parts.append(dp.make_partial((x0, y0, w, h), tr, td))
        full_r = np.zeros((H, W, 4)); full_d = np.full((H, W), np.inf)
        full_r[y0:y0 + h, x0:x0 + w] = rgba
        full_d[y0:y0 + h, x0:x0 + w] = depth
        ref_parts.append((full_r, full_d))
    out = torch.empty(H, W, 4, device="cuda")
    dp.vr_composite(ctx, parts, BG, out)
    dp.vr_synchronize(ctx)
    dp.vr_context_release(ctx)
    ref = oracle.composite(ref_parts, BG)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-6


def test_state_errors(dp):
    ctx = dp.vr_context_create(0, None)
    with pytest.raises(dp.VRError) as e:
        dp.vr_partial_roi(ctx, None)
    assert e.value.status == dp.VR_ERR_INVALID_HANDLE
    ws = torch.empty(4096, device="cuda")
    b = dp.vr_brick_create(ctx, (4, 4, 4), 1, (0, 0, 0), (1, 1, 1), dp.VR_F32, ws, ws.numel() * 4)
    with pytest.raises(dp.VRError) as e:
        dp.vr_render_partial(ctx, b, dp.make_partial((0, 0, 1, 1), ws, ws))
    assert e.value.status == dp.VR_ERR_STATE
    with pytest.raises(dp.VRError) as e:
        dp.vr_brick_create(ctx, (40, 40, 40), 1, (0, 0, 0), (1, 1, 1), dp.VR_F32, ws, ws.numel() * 4)
    assert e.value.status == dp.VR_ERR_WORKSPACE
    with pytest.raises(dp.VRError) as e:
        dp.vr_set_camera_perspective(ctx, (0, 0, 0), (0, 1, 0), (0, 1, 0), 45, 8, 8)
    assert e.value.status == dp.VR_ERR_INVALID_ARG
    with pytest.raises(dp.VRError) as e:
        dp.vr_context_release(ctx)
    assert e.value.status == dp.VR_ERR_STATE
    dp.vr_brick_release(b)
    dp.vr_context_release(ctx)


# ----------------------------------------------------- launch-path invariance
@pytest.mark.parametrize("seed,dims,nb,w,h,az,el,radius,step", [
    (201, (64, 48, 40), 6, 96, 80, 30.0, 20.0, 2.0, 0.5),     # z slabs, every tile staged
    (202, (48, 64, 40), 5, 80, 72, 120.0, 20.0, 1.8, 0.5),    # x-dominant view, y/z slabs
    (203, (40, 40, 40), 4, 72, 64, 90.0, 0.0, 2.0, 0.5),      # view along -x: HBM fallback
    (204, (60, 40, 30), 7, 64, 64, 200.0, -50.0, 1.3, 0.25),  # y slabs, negative direction
])
@pytest.mark.parametrize("config", [(0, 16, 4), (1, 16, 4), (1, 16, 8), (1, 32, 4), (1, 32, 8)],
                         ids=["slab", "ring16x4", "ring16x8", "ring32x4", "ring32x8"])
def test_staged_equals_direct_bitwise(dp, seed, dims, nb, w, h, az, el, radius, step, config):
    """The LDS-staged march (slab staging, and ring staging with every tile
    width x chunk length) and the direct
    march evaluate every sample at the same float32 position from the same
    voxel values, so partial images and sample counts are bit-identical; both
    match the oracle."""
    sc = _scene_small(seed, dims, nb, w, h, az, el, radius, scale=3.0, step=step)
    out = []
    for path in (dp.VR_PATH_STAGED, dp.VR_PATH_DIRECT):
        bricks = [(b.voxels, b.lo) for b in sc.bricks]
        r = dp.Renderer(bricks, sc.tf, sc.vrange, sc.opacity_scale, sc.step, path=path,
                        march_config=config)
        r.reset_samples()
        img, parts = _gpu_frame(r, sc.camera, BG)
        counts = r.sample_counts()
        r.close()
        out.append((img, parts, counts))
    (ia, pa, ca), (ib, pb, cb) = out
    assert np.array_equal(ia, ib)
    for (ra, rga, da), (rb, rgb, db) in zip(pa, pb):
        assert ra == rb and np.array_equal(rga, rgb) and np.array_equal(da, db)
    assert np.array_equal(ca, cb)
    ref, ref_parts, _ = oracle.render_scene(sc, bg=BG)
    _check_partials(pa, ref_parts, TOL32)
    assert np.max(np.abs(ia - ref)) <= TOL32


@pytest.mark.parametrize("config", [(0, 16, 4), (1, 16, 4), (1, 32, 8)],
                         ids=["slab", "ring16x4", "ring32x8"])
def test_staged_fp16_and_inside_camera(dp, config):
    """FP16 storage (staged raw, decoded at read) and a camera inside the
    volume (large per-slice footprints that may exceed the ring and fall
    back)."""
    sc = _scene_small(205, (48, 40, 36), 6, 64, 56, scale=3.0)
    cam = synth.inside_camera((0, 0, 0), (48, 40, 36), 64, 56, fovy_deg=80.0)
    outs = []
    for path in (dp.VR_PATH_STAGED, dp.VR_PATH_DIRECT):
        r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale,
                        sc.step, storage=dp.VR_F16, path=path, march_config=config)
        outs.append(_gpu_frame(r, cam, BG)[0])
        r.close()
    assert np.array_equal(outs[0], outs[1])
    dec = [b.voxels.astype(np.float16).astype(np.float32) for b in sc.bricks]
    ref, _, _ = oracle.render_scene(sc, camera=cam, bg=BG, field_override=dec)
    assert np.max(np.abs(outs[0] - ref)) <= TOL32


def test_queued_frame_equals_per_brick_launches(dp):
    """All partials of a frame through one work-queue launch (mixed float32 and
    float16 bricks: two queues) equal one launch per brick, bitwise."""
    sc = _scene_small(206, (56, 44, 36), 9, 88, 72, az=65.0, scale=3.0)
    bricks = [(b.voxels, b.lo) for b in sc.bricks]
    r = dp.Renderer([], sc.tf, sc.vrange, sc.opacity_scale, sc.step)
    for k, (v, lo) in enumerate(bricks):
        r.storage = dp.VR_F16 if k % 3 == 0 else dp.VR_F32
        r.add_brick(v, lo)
    r.set_camera(sc.camera)
    r.render_partials()
    r.synchronize()
    a = [tuple(t.cpu().numpy().copy() for t in r.partial_arrays(k)) for k in range(len(bricks))]
    r.render_partials_each()
    r.synchronize()
    b = [tuple(t.cpu().numpy().copy() for t in r.partial_arrays(k)) for k in range(len(bricks))]
    r.close()
    for (ra, da), (rb, db) in zip(a, b):
        assert np.array_equal(ra, rb) and np.array_equal(da, db)

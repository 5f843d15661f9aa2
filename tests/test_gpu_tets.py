"""GPU parity of tetrahedral parts (vr_render_tetparts) against the oracle's
oc_render_tets: the image within 1e-5 per channel and the count of samples
held by a tetrahedron exactly, on conforming meshes split into uneven,
non-convex parts; samples placed on mesh vertices, edges and faces; the eye
inside the mesh; a part with no tetrahedra; the run-overflow error; and new
vertex values on the same tables."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _dp():
    import paper_2501_01628_amd as dp
    return dp


def _scene(cells, jitter, n_parts, seed, linear=False, rough=True):
    rng = np.random.default_rng(seed)
    v, t = synth.tet_mesh(cells, jitter=jitter, rng=rng)
    if linear:
        v = np.round(v * 1024.0) / 1024.0
        vals = (0.25 + 0.125 * v[:, 0] + 0.0625 * v[:, 1] - 0.03125 * v[:, 2]).astype(np.float32)
    else:
        vals = synth.tet_field(v, rng, cells)
    if n_parts == 1:
        parts = [(v, t, np.arange(len(v)))]
    else:
        parts = synth.tet_partitions(v, t, n_parts, rng, rough=rough)
    return vals, parts


def _tf():
    return synth.hidden_tf(11), (0.02, 0.95), 1.3


def _gpu(parts, vals, cam, dt, bg, max_runs=8):
    dp = _dp()
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, dt, max_runs=max_runs)
    try:
        for k, (_, _, used) in enumerate(parts):
            r.set_values(k, vals[used])
        r.set_camera(cam)
        r.samples.zero_()
        img = r.render(bg, count=True)
        r.synchronize()
        return img.cpu().numpy().astype(np.float64), int(r.samples.item())
    finally:
        r.close()


def _ref(parts, vals, cam, dt, bg):
    tf, vr, s = _tf()
    img, cnt = oracle.render_tets(cam, [(pv, vals[used], pt) for pv, pt, used in parts], tf, vr, s, dt, bg)
    assert cnt[1] == 0
    return img, int(cnt[0])


def _compare(parts, vals, cam, dt, bg=(0.0, 0.0, 0.0, 0.0), max_runs=8):
    print(f"tets: {sum(len(p[1]) for p in parts)} in {len(parts)} parts, {cam['width']}x{cam['height']}, dt {dt}",
          flush=True)
    img, held = _gpu(parts, vals, cam, dt, bg, max_runs)
    ref, rheld = _ref(parts, vals, cam, dt, bg)
    assert held == rheld
    err = np.max(np.abs(img - ref))
    assert err <= TOL, err
    return img


@pytest.mark.parametrize("n_parts,seed,rough", [(1, 1, True), (5, 2, True), (9, 3, True), (6, 12, False)])
def test_jittered_mesh_in_parts(n_parts, seed, rough):
    cells = (6, 5, 7)
    vals, parts = _scene(cells, 0.25, n_parts, seed, rough=rough)
    cam = synth.orbit_camera((0, 0, 0), cells, 61, 47, az_deg=30.0 + 20 * seed, el_deg=20.0, radius_factor=1.5)
    _compare(parts, vals, cam, 0.37, (0.05, 0.1, 0.15, 0.3))


def test_samples_on_vertices_edges_and_faces():
    # orthographic view along +z with pixel centres on half-integer lines and
    # samples on the planes z = m / 2 of an unjittered mesh
    cells = (4, 3, 5)
    vals, parts = _scene(cells, 0.0, 1, 4, linear=True)
    cam = dict(kind="ortho", eye=(0.25, 0.25, -1.25), dir=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0),
               width=16, height=16, view_height=8.0)
    _compare(parts, vals, cam, 0.5)
    vals, parts = _scene(cells, 0.0, 3, 5, linear=True)
    _compare(parts, vals, cam, 0.5)


def test_eye_inside_the_mesh():
    cells = (6, 6, 6)
    vals, parts = _scene(cells, 0.2, 4, 6)
    cam = synth.inside_camera((0, 0, 0), cells, 40, 33, az_deg=-40.0, el_deg=15.0, fovy_deg=75.0)
    _compare(parts, vals, cam, 0.23)


def test_empty_part_and_single_tetrahedron_parts():
    cells = (3, 3, 3)
    vals, parts = _scene(cells, 0.2, 2, 7)
    v0, t0, u0 = parts[0]
    one = [(v0, t0[:1], u0), (v0, t0[1:], u0)]
    empty = (np.zeros((0, 3)), np.zeros((0, 4), dtype=np.int32), np.zeros(0, dtype=np.int64))
    cam = synth.orbit_camera((0, 0, 0), cells, 33, 29, az_deg=70.0, el_deg=-25.0, radius_factor=1.4)
    _compare(one + [parts[1], empty], vals, cam, 0.31)


def test_runs_overflow_is_reported_and_recovers():
    dp = _dp()
    cells = (8, 6, 6)
    vals, parts = _scene(cells, 0.25, 6, 8)
    cam = synth.orbit_camera((0, 0, 0), cells, 48, 40, az_deg=10.0, el_deg=5.0, radius_factor=1.3)
    ref, _ = _ref(parts, vals, cam, 0.2, (0.0, 0.0, 0.0, 0.0))
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, 0.2, max_runs=1)
    try:
        for k, (_, _, used) in enumerate(parts):
            r.set_values(k, vals[used])
        r.set_camera(cam)
        r.render()
        with pytest.raises(dp.VRError, match="max_runs"):
            r.synchronize()
        r.max_runs = 16
        r.set_camera(cam)
        img = r.render()
        r.synchronize()
        assert np.max(np.abs(img.cpu().numpy() - ref)) <= TOL
    finally:
        r.close()


def test_new_values_on_the_same_tables():
    dp = _dp()
    cells = (5, 4, 4)
    vals, parts = _scene(cells, 0.2, 3, 9)
    vals2 = np.ascontiguousarray(vals[::-1])
    cam = synth.orbit_camera((0, 0, 0), cells, 37, 31, az_deg=-60.0, el_deg=30.0, radius_factor=1.6)
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, 0.29)
    try:
        r.set_camera(cam)
        for vv in (vals, vals2):
            for k, (_, _, used) in enumerate(parts):
                r.set_values(k, vv[used])
            img = r.render().cpu().numpy()
            r.synchronize()
            ref, _ = _ref(parts, vv, cam, 0.29, (0.0, 0.0, 0.0, 0.0))
            assert np.max(np.abs(img - ref)) <= TOL
    finally:
        r.close()


def test_rejected_calls():
    dp = _dp()
    ctx = dp.vr_context_create(0)
    try:
        v = np.zeros((4, 3))
        v[1, 0] = v[2, 1] = 1.0            # v[3] at the origin too: zero volume
        with pytest.raises(dp.VRError, match="zero volume"):
            dp.vr_tetpart_create(ctx, v, np.array([[0, 1, 2, 3]], dtype=np.int32))
        v[3, 2] = 1.0
        with pytest.raises(dp.VRError, match="outside"):
            dp.vr_tetpart_create(ctx, v, np.array([[0, 1, 2, 4]], dtype=np.int32))
        h = dp.vr_tetpart_create(ctx, v, np.array([[0, 1, 2, 3]], dtype=np.int32))
        with pytest.raises(dp.VRError, match="VR_ERR_STATE"):
            dp.vr_tetpart_set_values(h, 0, ctx)          # no workspace yet
        with pytest.raises(dp.VRError, match="VR_ERR_STATE"):
            dp.vr_tetparts_workspace_size(ctx, [h], 4)   # no camera
        dp.set_camera(ctx, synth.orbit_camera((0, 0, 0), (1, 1, 1), 8, 8))
        with pytest.raises(dp.VRError, match="max_runs"):
            dp.vr_tetparts_workspace_size(ctx, [h], 0)
        with pytest.raises(dp.VRError, match="repeats"):
            dp.vr_tetparts_workspace_size(ctx, [h, h], 4)
        with pytest.raises(dp.VRError, match="VR_ERR_STATE"):
            dp.vr_context_release(ctx)                   # a part is alive
        dp.vr_tetpart_release(h, ctx)
    finally:
        dp.vr_context_release(ctx)


def test_march_and_resolve_stages_equal_the_frame_call():
    dp = _dp()
    cells = (6, 4, 5)
    vals, parts = _scene(cells, 0.2, 4, 10)
    cam = synth.orbit_camera((0, 0, 0), cells, 45, 38, az_deg=20.0, el_deg=35.0, radius_factor=1.5)
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, 0.33)
    try:
        for k, (_, _, used) in enumerate(parts):
            r.set_values(k, vals[used])
        r.set_camera(cam)
        whole = r.render((0.1, 0.0, 0.2, 0.5)).clone()
        r.frame.zero_()
        r.march()
        staged = r.resolve((0.1, 0.0, 0.2, 0.5))
        r.synchronize()
        assert bool((whole == staged).all())
        # a resolve whose march used another max_runs is refused
        r.max_runs = 4
        with pytest.raises(dp.VRError, match="VR_ERR_STATE"):
            r.resolve()
    finally:
        r.close()


def test_bench_size_split_invariance_and_linear_field():
    """At the benchmark's size (7.1 M tetrahedra, 1920x1080): the frame of
    16 non-convex parts equals the frame of the whole mesh as one part (same
    held-sample count, 1e-5), and a linear field renders as the brick
    oracle renders it at sampled pixels."""
    dp = _dp()
    cells = (128, 96, 96)
    rng = np.random.default_rng(12)
    v, t = synth.tet_mesh(cells, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, cells, n_blobs=8)
    parts = synth.tet_partitions(v, t, 16, rng)
    cam = synth.orbit_camera((0, 0, 0), cells, 1920, 1080)
    print("bench-size mesh generated", flush=True)
    tf, vr, s = _tf()

    def frame(pp, vv, count=True):
        r = dp.TetRenderer([(pv, pt) for pv, pt, _ in pp], tf, vr, s, 0.5, max_runs=32)
        try:
            for k, (_, _, used) in enumerate(pp):
                r.set_values(k, vv[used])
            r.set_camera(cam)
            r.samples.zero_()
            img = r.render(count=count)
            r.synchronize()
            return img.cpu().numpy().astype(np.float64), int(r.samples.item())
        finally:
            r.close()
    split, n16 = frame(parts, vals)
    whole, n1 = frame([(v, t, np.arange(len(v)))], vals)
    print(f"held {n16} / {n1}", flush=True)
    assert n16 == n1 > 0
    assert np.max(np.abs(split - whole)) <= TOL
    lin = (0.1 + 0.004 * v[:, 0] + 0.003 * v[:, 1] + 0.002 * v[:, 2]).astype(np.float32)
    img, _ = frame(parts, lin, count=False)
    nx, ny, nz = cells
    z, y, x = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    vox = (0.1 + 0.004 * (x - 0.5) + 0.003 * (y - 0.5) + 0.002 * (z - 0.5)).astype(np.float32)
    pick = np.random.default_rng(0)
    pix = np.stack([pick.integers(0, 1920, 48), pick.integers(0, 1080, 48)], 1).astype(np.int32)
    ref, _, _ = oracle.render_brick(cam, vox, cells, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), tf, vr, s, 0.5,
                                    pixels=pix)
    err = np.max(np.abs(img[pix[:, 1], pix[:, 0]] - ref))
    assert err <= TOL, err


# ----------------------------------------------------------- shadow rays
def _gpu_shadowed(parts, vals, cam, dt, light, a0, bg, max_runs=8):
    dp = _dp()
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, dt, max_runs=max_runs)
    try:
        for k, (_, _, used) in enumerate(parts):
            r.set_values(k, vals[used])
        r.set_camera(cam)
        total = r.shadow_plan()
        r.samples.zero_()
        img = r.render_shadowed(light, a0, bg, count=True)
        r.synchronize()
        out = img.cpu().numpy().astype(np.float64), total, int(r.samples.item())
        plain = r.render(bg).cpu().numpy().astype(np.float64)
        r.synchronize()
        return out + (plain,)
    finally:
        r.close()


@pytest.mark.parametrize("n_parts,seed,rough,light,a0", [(1, 21, True, (0.3, 1.0, -0.4), 0.3),
                                                         (4, 22, True, (-1.0, 0.0, 0.0), 0.0),
                                                         (5, 23, False, (0.0, 0.5, 1.0), 0.45)])
def test_shadowed_parts_match_oracle(n_parts, seed, rough, light, a0):
    cells = (5, 4, 5)
    vals, parts = _scene(cells, 0.2, n_parts, seed, rough=rough)
    cam = synth.orbit_camera((0, 0, 0), cells, 37, 29, az_deg=15.0 * seed, el_deg=25.0, radius_factor=1.5)
    bg = (0.02, 0.04, 0.08, 0.1)
    print(f"shadowed tets: {n_parts} parts, light {light}, a0 {a0}", flush=True)
    img, total, counted, plain = _gpu_shadowed(parts, vals, cam, 0.35, light, a0, bg)
    tf, vr, s = _tf()
    tparts = [(pv, vals[used], pt) for pv, pt, used in parts]
    ref, cnt = oracle.render_tets_shadowed(cam, tparts, tf, vr, s, 0.35, light, a0, bg)
    assert cnt[1] == 0
    assert total == cnt[0]
    assert counted == cnt[0] + cnt[2]
    err = np.max(np.abs(img - ref))
    assert err <= TOL, err
    if a0 < 1.0 and cnt[2] > 0:
        assert np.max(np.abs(img - plain)) > 1e-3      # the shadows change the image


def test_shadowed_ambient_one_equals_plain_frame_bitwise():
    cells = (4, 4, 4)
    vals, parts = _scene(cells, 0.15, 3, 24)
    cam = synth.inside_camera((0, 0, 0), cells, 30, 26, az_deg=30.0, el_deg=-10.0, fovy_deg=70.0)
    img, total, _, plain = _gpu_shadowed(parts, vals, cam, 0.29, (1.0, 1.0, 1.0), 1.0, (0.0, 0.0, 0.0, 0.0))
    assert total > 0
    assert np.array_equal(img, plain)


# -------------------------------------------------------- mixed cells
def _mixed_gpu(parts, vals, cam, dt, bg=(0.0, 0.0, 0.0, 0.0)):
    dp = _dp()
    tf, vr, s = _tf()
    r = dp.TetRenderer([(pv, psz, pcv, used) for pv, psz, pcv, used in parts], tf, vr, s, dt)
    try:
        for k, (_, _, _, used) in enumerate(parts):
            r.set_values(k, vals[used])
        r.set_camera(cam)
        r.samples.zero_()
        img = r.render(bg, count=True)
        r.synchronize()
        ntets = sum(i["n_tets"] for i in r.info)
        return img.cpu().numpy().astype(np.float64), int(r.samples.item()), ntets
    finally:
        r.close()


@pytest.mark.parametrize("n_parts,seed,rough", [(1, 41, False), (4, 42, True), (6, 43, False)])
def test_mixed_cells_match_oracle(n_parts, seed, rough):
    cells = (6, 5, 4)
    rng = np.random.default_rng(seed)
    v, sz, cv = synth.mixed_mesh(cells, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, cells)
    if n_parts == 1:
        parts = [(v, sz, cv, np.arange(len(v)))]
    else:
        parts = synth.mixed_partitions(v, sz, cv, n_parts, rng, rough=rough)
    cam = synth.orbit_camera((0, 0, 0), cells, 53, 41, az_deg=20.0 + 10 * seed, el_deg=30.0, radius_factor=1.5)
    print(f"mixed cells: {len(sz)} in {n_parts} parts", flush=True)
    img, held, ntets = _mixed_gpu(parts, vals, cam, 0.31, (0.1, 0.0, 0.05, 0.2))
    tf, vr, s = _tf()
    tparts = [oracle.cells_to_tets(pv, vals[used], psz, pcv, vertex_ids=used) for pv, psz, pcv, used in parts]
    ref, cnt = oracle.render_tets(cam, tparts, tf, vr, s, 0.31, (0.1, 0.0, 0.05, 0.2))
    assert ntets == sum(len(t[2]) for t in tparts)
    assert cnt[1] == 0 and held == cnt[0]
    assert np.max(np.abs(img - ref)) <= TOL


def test_mixed_cells_linear_field_equals_brick():
    cells = (5, 4, 3)
    rng = np.random.default_rng(44)
    v, sz, cv = synth.mixed_mesh(cells, jitter=0.1, rng=rng)
    vals = (0.2 + 0.05 * v[:, 0] + 0.03 * v[:, 1] + 0.04 * v[:, 2]).astype(np.float32)
    parts = synth.mixed_partitions(v, sz, cv, 3, rng)
    cam = synth.orbit_camera((0, 0, 0), cells, 40, 36, az_deg=-30.0, el_deg=20.0, radius_factor=1.6)
    img, _, _ = _mixed_gpu(parts, vals, cam, 0.27)
    nx, ny, nz = cells
    z, y, x = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    vox = (0.2 + 0.05 * (x - 0.5) + 0.03 * (y - 0.5) + 0.04 * (z - 0.5)).astype(np.float32)
    tf, vr, s = _tf()
    ref, _, _ = oracle.render_brick(cam, vox, cells, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), tf, vr, s, 0.27)
    assert np.max(np.abs(img - ref)) <= TOL


# ----------------------------------------------------------- BVH locator
def test_bvh_locator_gives_the_grid_frames_bitwise():
    """After the walk, the BVH and the grid find the same owner for every
    sample, so every frame (plain, shadowed, mixed cells) is bit-identical,
    and the BVH frame matches the oracle."""
    dp = _dp()
    cells = (6, 5, 5)
    vals, parts = _scene(cells, 0.2, 5, 51, rough=True)
    cam = synth.orbit_camera((0, 0, 0), cells, 47, 39, az_deg=65.0, el_deg=-15.0, radius_factor=1.5)
    tf, vr, s = _tf()
    frames = {}
    for loc in (dp.VR_TET_GRID, dp.VR_TET_BVH):
        r = dp.TetRenderer([(pv, pt) for pv, pt, _ in parts], tf, vr, s, 0.3, locator=loc)
        try:
            for k, (_, _, used) in enumerate(parts):
                r.set_values(k, vals[used])
            r.set_camera(cam)
            r.samples.zero_()
            plain = r.render(count=True).clone()
            r.synchronize()
            held = int(r.samples.item())
            r.shadow_plan()
            shadowed = r.render_shadowed((0.4, 1.0, 0.3), 0.2).clone()
            r.synchronize()
            frames[loc] = (plain.cpu().numpy(), held, shadowed.cpu().numpy())
        finally:
            r.close()
    g, b = frames[dp.VR_TET_GRID], frames[dp.VR_TET_BVH]
    assert np.array_equal(g[0], b[0]) and g[1] == b[1] and np.array_equal(g[2], b[2])
    ref, cnt = _ref(parts, vals, cam, 0.3, (0.0, 0.0, 0.0, 0.0))
    assert cnt == b[1] and np.max(np.abs(b[0] - ref)) <= TOL
    # mixed cells
    rng = np.random.default_rng(52)
    v, sz, cv = synth.mixed_mesh((5, 4, 4), jitter=0.1, rng=rng)
    mvals = synth.tet_field(v, rng, (5, 4, 4))
    mparts = synth.mixed_partitions(v, sz, cv, 3, rng)
    mcam = synth.orbit_camera((0, 0, 0), (5, 4, 4), 33, 30, az_deg=10.0, el_deg=40.0, radius_factor=1.5)
    imgs = []
    for loc in (dp.VR_TET_GRID, dp.VR_TET_BVH):
        r = dp.TetRenderer(mparts, tf, vr, s, 0.3, locator=loc)
        try:
            for k, part in enumerate(mparts):
                r.set_values(k, mvals[part[-1]])
            r.set_camera(mcam)
            imgs.append(r.render().cpu().numpy())
            r.synchronize()
        finally:
            r.close()
    assert np.array_equal(imgs[0], imgs[1])

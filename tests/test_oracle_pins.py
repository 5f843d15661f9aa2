"""Pins of the FP64 oracle against values fixed by the mathematics, not by the
oracle itself: hand-derived worked examples (tests/golden), closed forms
(constant slab, linear ramp), special cases (empty volume), invariants (split
invariance, associativity of "over"), an independent pinhole projection for
the camera, brute force with library routines (scipy's grid interpolator and
numpy's piecewise-linear interp) and finite differences for the gradients.

Each test names the reading of the optical model it pins: cell-centred grid,
sample lattice t_k = (k + 1/2) dt, endpoint-aligned table, emission-absorption,
first-sample depth key, sort-last "over".
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def _ramp_tf(rgb=None):
    tf = np.zeros((256, 4))
    if rgb is None:
        tf[:, :3] = 1.0
    else:
        x = np.arange(256) / 255.0
        tf[:, 0], tf[:, 1], tf[:, 2] = rgb(x)
    tf[:, 3] = np.arange(256) / 255.0
    return tf


_W_CAM = dict(kind="ortho", eye=(0.0, 0.5, 0.5), dir=(1.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
              width=1, height=1, view_height=1.0)
_W_V = np.array([[[0.0, 1.0]]], dtype=np.float32)
_W2_RGB = lambda x: (x, 1.0 - x, 0.25 + 0 * x)


# ------------------------------------------------------------ worked examples
@pytest.mark.parametrize("name,rgb", [("W1", None), ("W2", _W2_RGB)])
def test_worked_example_whole(name, rgb):
    g = GOLD[name]
    tf = _ramp_tf(rgb)
    rgba, depth, cnt = oracle.render_brick(_W_CAM, _W_V, (2, 1, 1), 0, (0, 0, 0), (1, 1, 1), tf,
                                           (0, 1), 1.0, 0.5)
    np.testing.assert_allclose(rgba[0, 0, :3], g["C"], atol=2e-9)
    assert abs(rgba[0, 0, 3] - g["A"]) < 2e-9
    assert depth[0, 0] == 0.25
    assert list(cnt) == [4, 4]
    img = oracle.composite([(rgba, depth)], GOLD["bg"])
    np.testing.assert_allclose(img[0, 0], g["final_bg"], atol=2e-9)


@pytest.mark.parametrize("name,rgb", [("W1", None), ("W2", _W2_RGB)])
def test_worked_example_split(name, rgb):
    """Split at x = 1 into two ghosted bricks; partials and composite are the
    hand values and the composite equals the unsplit result."""
    g = GOLD[name]
    tf = _ramp_tf(rgb)
    # ghost layer: neighbour voxel inside the domain, edge copy outside
    va = np.array([[[0.0, 0.0, 1.0]]] * 3, dtype=np.float32).reshape(3, 1, 3)
    va = np.repeat(np.repeat(np.array([0.0, 0.0, 1.0], dtype=np.float32)[None, None, :], 3, 1), 3, 0)
    vb = np.repeat(np.repeat(np.array([0.0, 1.0, 1.0], dtype=np.float32)[None, None, :], 3, 1), 3, 0)
    pa = oracle.render_brick(_W_CAM, va, (1, 1, 1), 1, (0, 0, 0), (1, 1, 1), tf, (0, 1), 1.0, 0.5)
    pb = oracle.render_brick(_W_CAM, vb, (1, 1, 1), 1, (1, 0, 0), (1, 1, 1), tf, (0, 1), 1.0, 0.5)
    if name == "W1":
        assert abs(pa[0][0, 0, 3] - g["split_A"]["A"]) < 2e-9 and pa[1][0, 0] == 0.25
        assert abs(pb[0][0, 0, 3] - g["split_B"]["A"]) < 2e-9 and pb[1][0, 0] == 1.25
    else:
        np.testing.assert_allclose(pa[0][0, 0], g["split_A"]["rgba"], atol=2e-9)
        np.testing.assert_allclose(pb[0][0, 0], g["split_B"]["rgba"], atol=2e-9)
    # order of the list must not matter: the depth key decides
    img = oracle.composite([(pb[0], pb[1]), (pa[0], pa[1])], GOLD["bg"])
    np.testing.assert_allclose(img[0, 0], g["final_bg"], atol=2e-9)


# ------------------------------------------------------------- closed forms
def _slab_count(o, lo, hi, dt):
    """Number of k >= 0 with lo <= o + (k + 1/2) dt < hi (o < lo)."""
    return math.ceil((hi - o) / dt - 0.5) - math.ceil((lo - o) / dt - 0.5)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("o_off,dt", [(0.0, 0.5), (-0.3, 0.5), (-1.7, 0.25), (-0.1, 0.37)])
def test_constant_slab_orthographic(axis, o_off, dt):
    """Constant field + constant table: T = exp(-sigma m dt) with m the number
    of lattice points inside the slab, C = rgb (1 - T)."""
    n = [3, 4, 5]
    n[axis] = 16
    nx, ny, nz = n
    vol = np.full((nz, ny, nx), 0.5, dtype=np.float32)
    tf = np.zeros((256, 4))
    tf[:] = (0.2, 0.6, 0.9, 0.8)
    d = [0.0, 0.0, 0.0]; d[axis] = 1.0
    up = (0.0, 0.0, 1.0) if axis == 1 else (0.0, 1.0, 0.0)
    eye = [0.5 * nx, 0.5 * ny, 0.5 * nz]; eye[axis] = o_off
    cam = dict(kind="ortho", eye=tuple(eye), dir=tuple(d), up=up, width=2, height=2,
               view_height=1.0)
    rgba, depth, cnt = oracle.render_brick(cam, vol, (nx, ny, nz), 0, (0, 0, 0), (1, 1, 1), tf,
                                           (0, 1), 1.0, dt)
    m = _slab_count(o_off, 0.0, 16.0, dt)
    sigma = 1.0 * 0.8
    A = 1.0 - math.exp(-sigma * m * dt)
    np.testing.assert_allclose(rgba[..., 3], A, rtol=1e-13, atol=1e-15)
    for c, v in enumerate((0.2, 0.6, 0.9)):
        np.testing.assert_allclose(rgba[..., c], v * A, rtol=1e-12)
    k_first = math.ceil((0.0 - o_off) / dt - 0.5)
    np.testing.assert_array_equal(depth, (k_first + 0.5) * dt)
    assert cnt[0] == 4 * m


def test_slab_example_value():
    """sigma = 0.8, L = 16 -> T = exp(-12.8) = 2.76077257e-6."""
    vol = np.full((16, 1, 1), 0.5, dtype=np.float32)
    tf = np.zeros((256, 4)); tf[:] = (1, 1, 1, 0.8)
    cam = dict(kind="ortho", eye=(0.5, 0.5, 0.0), dir=(0, 0, 1.0), up=(0, 1.0, 0), width=1,
               height=1, view_height=0.5)
    rgba, _, _ = oracle.render_brick(cam, vol, (1, 1, 16), 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                     1.0, 0.5)
    assert abs((1 - rgba[0, 0, 3]) - 2.76077257e-6) < 1e-14


def _slab_interval(o, d, lo, hi):
    tin, tout = 0.0, math.inf
    for c in range(3):
        if d[c] == 0:
            if not (lo[c] <= o[c] < hi[c]):
                return None
            continue
        a, b = (lo[c] - o[c]) / d[c], (hi[c] - o[c]) / d[c]
        tin, tout = max(tin, min(a, b)), min(tout, max(a, b))
    return (tin, tout) if tout > tin else None


def test_constant_perspective_lattice_count():
    """Perspective view of a constant box: every pixel is 1 - exp(-sigma m dt)
    with m the count of lattice points in the ray's slab interval, found by
    the closed form ceil(t_out/dt - 1/2) - ceil(t_in/dt - 1/2)."""
    dims = (9, 7, 5)
    vol = np.full(dims[::-1], 0.3, dtype=np.float32)
    tf = np.zeros((256, 4)); tf[:] = (1, 1, 1, 0.5)
    cam = synth.orbit_camera((0, 0, 0), dims, 24, 18, az_deg=37.0, el_deg=23.0, radius_factor=1.4)
    dt = 0.25
    rgba, depth, cnt = oracle.render_brick(cam, vol, dims, 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                           2.0, dt)
    hits = 0
    total = 0
    for j in range(18):
        for i in range(24):
            o, d = oracle.ray(cam, i, j)
            iv = _slab_interval(o, d, (0, 0, 0), dims)
            m = 0 if iv is None else max(0, math.ceil(iv[1] / dt - 0.5) - math.ceil(iv[0] / dt - 0.5))
            total += m
            hits += m > 0
            assert abs(rgba[j, i, 3] - (1 - math.exp(-1.0 * m * dt))) < 1e-12
            if m == 0:
                assert depth[j, i] == math.inf
            else:
                assert depth[j, i] == (math.ceil(iv[0] / dt - 0.5) + 0.5) * dt
    assert hits > 100 and cnt[0] == total


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_ramp(axis):
    """Field linear along the view axis, single-segment linear table: the
    trilinear interpolant is the line itself between the first and last voxel
    centres and clamps to the edge values outside, so the opacity integral is
    a sum of a clamped linear function over the lattice."""
    n = 12
    shape = [3, 3, 3]; shape[axis] = n
    nx, ny, nz = shape
    vals = 0.1 + 0.05 * np.arange(n)  # voxel centre values V_i at i + 1/2
    vol = np.empty((nz, ny, nx), dtype=np.float32)
    idx = np.indices((nz, ny, nx))[2 - axis]
    vol[:] = (0.1 + 0.05 * idx).astype(np.float32)
    vals = vol.reshape(-1)[np.argsort(idx.reshape(-1), kind="stable")][:: (vol.size // n)]
    tf = np.zeros((256, 4)); tf[:, 3] = np.arange(256) / 255.0; tf[:, 1] = 1.0
    d = [0.0, 0.0, 0.0]; d[axis] = 1.0
    eye = [1.5, 1.5, 1.5]; eye[axis] = -0.4
    up = (0.0, 0.0, 1.0) if axis == 1 else (0.0, 1.0, 0.0)
    cam = dict(kind="ortho", eye=tuple(eye), dir=tuple(d), up=up, width=1, height=1,
               view_height=0.1)
    dt, scale = 0.5, 1.5
    rgba, _, _ = oracle.render_brick(cam, vol, (nx, ny, nz), 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                     scale, dt)
    tau = 0.0
    k = 0
    while True:
        x = -0.4 + (k + 0.5) * dt
        if x >= n:
            break
        if x >= 0:
            c = min(max(x - 0.5, 0.0), n - 1.0)       # clamp to first/last centre
            i0 = min(int(math.floor(c)), n - 2)
            v = float(vals[i0]) + (c - i0) * (float(vals[i0 + 1]) - float(vals[i0]))
            tau += scale * v * dt
        k += 1
    assert abs(rgba[0, 0, 3] - (1 - math.exp(-tau))) < 1e-12
    assert abs(rgba[0, 0, 1] - (1 - math.exp(-tau))) < 1e-12
    assert rgba[0, 0, 0] == 0.0


def test_axis_orientation_in_image():
    """A field that grows along +x seen from +z (looking down -z, up = +y):
    pixel columns to the right see larger values, rows do not change."""
    vol = np.zeros((4, 4, 16), dtype=np.float32)
    vol[:] = (np.arange(16) / 16.0).astype(np.float32)[None, None, :]
    tf = _ramp_tf()
    cam = dict(kind="ortho", eye=(8.0, 2.0, 10.0), dir=(0, 0, -1.0), up=(0, 1.0, 0), width=8,
               height=2, view_height=2.0)
    rgba, _, _ = oracle.render_brick(cam, vol, (16, 4, 4), 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                     1.0, 0.5)
    a = rgba[..., 3]
    # camera right vector = f x up = (0,0,-1) x (0,1,0) = (1,0,0): +x to the right
    assert np.all(np.diff(a[0]) > 0)
    np.testing.assert_allclose(a[0], a[1], rtol=0, atol=0)


def _ortho_ramp(axis, n_axis, eye, up, width, height, view_height, scale, dt):
    """Alpha of every pixel of an orthographic view down -z through an
    n_axis x n_axis x 4 field that is a linear ramp along `axis` (x or y;
    voxel i holds (i + 1/2) / n_axis, so the trilinear interpolant is
    v = position / n_axis away from the edges), with the identity alpha
    table a = v.  Returns (alpha image, lattice count
    m of the 4-voxel thick slab)."""
    nx, ny, nz = n_axis, n_axis, 4
    vol = np.empty((nz, ny, nx), dtype=np.float32)
    idx = np.indices((nz, ny, nx))[2 - axis]
    vol[:] = ((idx + 0.5) / n_axis).astype(np.float32)
    tf = _ramp_tf()
    cam = dict(kind="ortho", eye=eye, dir=(0.0, 0.0, -1.0), up=up, width=width, height=height,
               view_height=view_height)
    rgba, _, cnt = oracle.render_brick(cam, vol, (nx, ny, nz), 0, (0, 0, 0), (1, 1, 1), tf,
                                       (0, 1), scale, dt)
    # rays start at z = eye_z = 10 and cross z in [0, 4): t in (6, 10]
    m = _slab_count(-eye[2], -4.0, 0.0, dt)
    assert cnt[0] == m * width * height
    return rgba[..., 3], m


def test_orthographic_pixel_mapping():
    """Orthographic pixel centres at hand-computed world positions.  Image
    10 x 4 pixels, 2 world units tall, centred at (8, 2): the pixel pitch is
    2 / 4 = 0.5 in both directions, so the columns sit at x = 8 + 0.5 (i - 4.5)
    = 5.75, 6.25, ..., 10.25 and the rows (row 0 on top, up = +y) at
    y = 2 + 0.5 (1.5 - j) = 2.75, 2.25, 1.75, 1.25.  A ramp along x (then
    along y) turns each pixel's alpha into the coordinate its ray travels
    at: v = -ln(1 - A) / (scale m dt) = coordinate / 16."""
    scale, dt = 1.0, 0.5
    cols = np.array([5.75, 6.25, 6.75, 7.25, 7.75, 8.25, 8.75, 9.25, 9.75, 10.25])
    rows = np.array([2.75, 2.25, 1.75, 1.25])
    a, m = _ortho_ramp(0, 16, (8.0, 2.0, 10.0), (0.0, 1.0, 0.0), 10, 4, 2.0, scale, dt)
    assert m == 8
    v = -np.log1p(-a) / (scale * m * dt)
    np.testing.assert_allclose(v, np.broadcast_to(cols / 16.0, v.shape), rtol=0, atol=1e-12)
    # ramp along y, the image centred at (8, 8): rows at y = 8 + 0.5 (1.5 - j)
    a, m = _ortho_ramp(1, 16, (8.0, 8.0, 10.0), (0.0, 1.0, 0.0), 10, 4, 2.0, scale, dt)
    v = -np.log1p(-a) / (scale * m * dt)
    np.testing.assert_allclose(v, np.broadcast_to(((rows + 6.0) / 16.0)[:, None], v.shape),
                               rtol=0, atol=1e-12)
    # a tall image (3 x 10, 5 units tall): pitch 0.5, columns at x = 7.5, 8, 8.5,
    # rows at y = 10.25 - 0.5 j
    a, m = _ortho_ramp(0, 16, (8.0, 8.0, 10.0), (0.0, 1.0, 0.0), 3, 10, 5.0, scale, dt)
    v = -np.log1p(-a) / (scale * m * dt)
    np.testing.assert_allclose(v, np.broadcast_to(np.array([7.5, 8.0, 8.5]) / 16.0, v.shape),
                               rtol=0, atol=1e-12)
    a, m = _ortho_ramp(1, 16, (8.0, 8.0, 10.0), (0.0, 1.0, 0.0), 3, 10, 5.0, scale, dt)
    v = -np.log1p(-a) / (scale * m * dt)
    ys = 10.25 - 0.5 * np.arange(10)
    np.testing.assert_allclose(v, np.broadcast_to((ys / 16.0)[:, None], v.shape), rtol=0,
                               atol=1e-12)


def test_camera_matches_projection_matrix():
    """Camera pin: project points along the oracle's pixel rays with an
    independent look-at + perspective matrix (OpenGL convention) and recover
    the pixel centre; the top row is +up."""
    cam = synth.orbit_camera((0, 0, 0), (10, 20, 30), 33, 21, az_deg=70.0, el_deg=-35.0,
                             fovy_deg=50.0)
    eye = np.array(cam["eye"]); tgt = np.array(cam["target"]); up = np.array(cam["up"])
    zc = eye - tgt; zc /= np.linalg.norm(zc)
    xc = np.cross(up, zc); xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    view = np.eye(4)
    view[0, :3], view[1, :3], view[2, :3] = xc, yc, zc
    view[:3, 3] = -view[:3, :3] @ eye
    W, H = 33, 21
    f = 1.0 / math.tan(math.radians(50.0) / 2)
    proj = np.array([[f * H / W, 0, 0, 0], [0, f, 0, 0], [0, 0, -1.0, -0.2], [0, 0, -1.0, 0]])
    for (i, j) in [(0, 0), (32, 0), (0, 20), (16, 10), (5, 17), (29, 3)]:
        o, d = oracle.ray(cam, i, j)
        p = o + 7.3 * d
        clip = proj @ view @ np.append(p, 1.0)
        ndc = clip[:2] / clip[3]
        px = (ndc[0] + 1) / 2 * W - 0.5
        py = (1 - ndc[1]) / 2 * H - 0.5
        assert abs(px - i) < 1e-9 and abs(py - j) < 1e-9
        assert abs(np.linalg.norm(d) - 1) < 1e-15


# --------------------------------------------------------- special cases
def test_empty_volume_gives_background_bitwise():
    rng = np.random.default_rng(7)
    vol = rng.uniform(0, 1, (6, 5, 4)).astype(np.float32)
    tf = np.zeros((256, 4)); tf[:, :3] = rng.uniform(0, 1, (256, 3))   # alpha == 0
    cam = synth.orbit_camera((0, 0, 0), (4, 5, 6), 16, 12, radius_factor=1.2)
    bg = (0.1, 0.2, 0.3, 1.0)
    img = oracle.render_volume(vol, cam, tf, (0, 1), 1.0, 0.5, bg=bg)
    assert np.array_equal(img, np.broadcast_to(np.array(bg), img.shape))
    # a ray that misses the box entirely also gives bg, and a key of +inf
    cam_miss = dict(cam, target=(100.0, 100.0, 100.0))
    rgba, depth, cnt = oracle.render_brick(cam_miss, vol, (4, 5, 6), 0, (0, 0, 0), (1, 1, 1),
                                           _ramp_tf(), (0, 1), 1.0, 0.5)
    assert np.all(depth == np.inf) and np.all(rgba == 0) and cnt[0] == 0


def test_fp16_representable_constant_is_exact():
    vol = np.full((8, 8, 8), 0.5, dtype=np.float32)
    vol16 = vol.astype(np.float16).astype(np.float32)
    assert np.array_equal(vol, vol16)
    tf = synth.default_tf()
    cam = synth.orbit_camera((0, 0, 0), (8, 8, 8), 12, 12, radius_factor=1.3)
    a = oracle.render_volume(vol, cam, tf, (0, 1), 1.0, 0.5)
    b = oracle.render_volume(vol16, cam, tf, (0, 1), 1.0, 0.5)
    assert np.array_equal(a, b)


# ------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed,n_bricks", [(11, 2), (12, 5), (13, 8)])
def test_split_invariance(seed, n_bricks):
    """Rendering the whole volume equals rendering kd bricks (with ghosts) and
    compositing them, at the same sample positions."""
    rng = np.random.default_rng(seed)
    dims = (20, 17, 13)
    field = synth.tile_field(rng, dims, n_blobs=6, noise=0.02, shock=True)
    boxes = synth.kd_split(dims, n_bricks, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, 40, 30, az_deg=20.0 + seed, el_deg=15.0,
                             radius_factor=1.6)
    tf = synth.default_tf()
    sc = synth.scene_from_field("split", field, boxes, tf, cam, 0.5, 2.0)
    bg = (0.1, 0.2, 0.3, 1.0)
    img, parts, cnt = oracle.render_scene(sc, bg=bg)
    ref = oracle.render_volume(field, cam, tf, (0, 1), 2.0, 0.5, bg=bg)
    assert np.max(np.abs(img - ref)) < 1e-13
    _, _, cnt_whole = oracle.render_brick(cam, field, dims, 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                          2.0, 0.5)
    assert cnt[0] == cnt_whole[0]     # every lattice point owned exactly once


def test_over_associative_and_alpha_product():
    rng = np.random.default_rng(3)
    n, npx = 6, 50
    parts = []
    for p in range(n):
        A = rng.uniform(0, 1, npx)
        Crgb = A[:, None] * rng.uniform(0, 1, (npx, 3))
        parts.append((np.concatenate([Crgb, A[:, None]], 1), rng.uniform(0, 100, npx)))
    out = oracle.composite(parts, (0, 0, 0, 0))
    A = np.array([p[0][:, 3] for p in parts])
    np.testing.assert_allclose(out[:, 3], 1 - np.prod(1 - A, axis=0), atol=1e-14)
    # (a over b) over c == a over (b over c) per pixel, in depth order
    for q in range(npx):
        order = np.argsort([p[1][q] for p in parts], kind="stable")
        xs = [parts[o][0][q] for o in order]

        def over(a, b):
            return a + (1 - a[3]) * b

        left = xs[0]
        for x in xs[1:]:
            left = over(left, x)
        right = xs[-1]
        for x in reversed(xs[:-1]):
            right = over(x, right)
        np.testing.assert_allclose(out[q], left, atol=1e-14)
        np.testing.assert_allclose(out[q], right, atol=1e-14)


def test_ert_counter_and_bound():
    """Stopping at T < eps changes each channel by at most eps; the counter of
    evaluated samples never exceeds the owned count."""
    rng = np.random.default_rng(5)
    dims = (16, 16, 16)
    field = synth.tile_field(rng, dims, n_blobs=4, shock=True)
    tf = synth.default_tf()
    cam = synth.orbit_camera((0, 0, 0), dims, 24, 24, radius_factor=1.5)
    eps = 2.0 ** -20
    rgba, _, cnt = oracle.render_brick(cam, field, dims, 0, (0, 0, 0), (1, 1, 1), tf, (0, 1), 30.0,
                                       0.5, eps)
    assert cnt[1] < cnt[0]     # some rays saturate at this opacity scale
    assert np.all(rgba[..., 3] <= 1.0) and np.all(rgba >= 0)


@pytest.mark.parametrize("sigma,dt,eps", [(0.8, 0.5, 2.0 ** -20), (0.3, 0.25, 1e-3),
                                          (2.5, 0.5, 2.0 ** -20), (0.01, 0.5, 2.0 ** -20)])
def test_ert_stop_index_closed_form(sigma, dt, eps):
    """Constant slab: after n samples T = exp(-sigma n dt), so a renderer that
    stops once T < eps evaluates n* = floor(ln(1/eps) / (sigma dt)) + 1
    samples (the stopping one included), or all m owned samples if T never
    drops below eps."""
    vol = np.full((32, 2, 2), 0.5, dtype=np.float32)
    tf = np.zeros((256, 4)); tf[:] = (1.0, 1.0, 1.0, sigma)
    cam = dict(kind="ortho", eye=(1.0, 1.0, -0.3), dir=(0, 0, 1.0), up=(0, 1.0, 0), width=2,
               height=2, view_height=1.0)
    rgba, _, cnt = oracle.render_brick(cam, vol, (2, 2, 32), 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                       1.0, dt, eps)
    m = _slab_count(-0.3, 0.0, 32.0, dt)
    x = math.log(1.0 / eps) / (sigma * dt)
    assert abs(x - round(x)) > 1e-6          # no tie at the threshold
    n_stop = min(math.floor(x) + 1, m)
    assert cnt[0] == 4 * m
    assert cnt[1] == 4 * n_stop
    np.testing.assert_allclose(rgba[..., 3], 1.0 - math.exp(-sigma * m * dt), rtol=1e-12)


# ------------------------------------------------------------- brute force
@pytest.mark.parametrize("dims", [(2, 1, 1), (2, 2, 2), (3, 4, 5)])
def test_brute_force_library_routines(dims):
    """Independent evaluation with library primitives: scipy's
    RegularGridInterpolator on the voxel centres (queries clipped to the
    first/last centre = clamp to edge), numpy.interp for the table, and a
    Python loop over every lattice point tested against the box."""
    from scipy.interpolate import RegularGridInterpolator
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    vol = rng.uniform(0, 1, (nz, ny, nx)).astype(np.float32)
    tf = synth.default_tf().astype(np.float64)
    cam = synth.orbit_camera((0, 0, 0), dims, 5, 5, az_deg=33.0, el_deg=27.0, radius_factor=1.1)
    dt, scale = 0.25, 3.0
    rgba, depth, _ = oracle.render_brick(cam, vol, dims, 0, (0, 0, 0), (1, 1, 1), tf, (0, 1),
                                         scale, dt)

    def axis_pts(n):
        return np.arange(n) + 0.5 if n > 1 else np.array([0.5, 1.5])

    data = vol.astype(np.float64).transpose(2, 1, 0)        # (x, y, z)
    for ax, n in enumerate(dims):
        if n == 1:
            data = np.concatenate([data, data], axis=ax)
    interp = RegularGridInterpolator([axis_pts(n) for n in dims], data, method="linear")
    grid = np.arange(256) / 255.0
    for j in range(5):
        for i in range(5):
            o, d = oracle.ray(cam, i, j)
            C = np.zeros(3); T = 1.0; key = math.inf
            for k in range(0, 400):
                p = o + ((k + 0.5) * dt) * d
                if not all(0 <= p[c] < dims[c] for c in range(3)):
                    continue
                if key == math.inf:
                    key = (k + 0.5) * dt
                q = [min(max(p[c], 0.5), max(dims[c] - 0.5, 0.5)) for c in range(3)]
                v = float(interp(q)[0])
                x = min(max(v, 0.0), 1.0)
                e = [np.interp(x, grid, tf[:, c]) for c in range(4)]
                alpha = 1 - math.exp(-scale * e[3] * dt)
                C += T * alpha * np.array(e[:3])
                T *= 1 - alpha
            np.testing.assert_allclose(rgba[j, i, :3], C, atol=1e-12)
            assert abs(rgba[j, i, 3] - (1 - T)) < 1e-12
            assert depth[j, i] == key


# ---------------------------------------------------------------- gradients
def _loss_parts(cam, bricks, tf, scale, dt, bg, target):
    parts = [oracle.render_brick(cam, v, dm, 1, lo, (1, 1, 1), tf, (0, 1), scale, dt)[:2]
             for (v, dm, lo) in bricks]
    img = oracle.composite(parts, bg)
    return float(np.sum((img - target) ** 2)), img, parts


def _bricks64(field64, boxes):
    out = []
    for lo, hi in boxes:
        b = synth.extract_brick(field64.astype(np.float32), lo, hi).astype(np.float64)
        # re-cut in float64 so perturbations below float32 resolution survive
        nz, ny, nx = field64.shape
        ix = np.clip(np.arange(lo[0] - 1, hi[0] + 1), 0, nx - 1)
        iy = np.clip(np.arange(lo[1] - 1, hi[1] + 1), 0, ny - 1)
        iz = np.clip(np.arange(lo[2] - 1, hi[2] + 1), 0, nz - 1)
        b = field64[np.ix_(iz, iy, ix)].copy()
        out.append((b, tuple(int(v) for v in np.subtract(hi, lo)), lo))
    return out


def test_gradient_against_central_differences():
    """Oracle gradient (composite backward + per-brick reverse recurrences +
    ghost fold) against float64 central differences of the loss
    L = sum (I - I*)^2 on a two-brick scene."""
    rng = np.random.default_rng(21)
    dims = (10, 9, 8)
    field = rng.uniform(0.1, 0.9, dims[::-1])          # float64, away from the clamps
    boxes = synth.kd_split(dims, 2, rng)
    bricks = _bricks64(field, boxes)
    cam = synth.orbit_camera((0, 0, 0), dims, 12, 10, radius_factor=1.5)
    tf = synth.default_tf().astype(np.float64)
    scale, dt, bg = 2.0, 0.5, (0.1, 0.2, 0.3, 1.0)
    target = rng.uniform(0, 1, (10, 12, 4))
    L, img, parts = _loss_parts(cam, bricks, tf, scale, dt, bg, target)
    g_out = 2.0 * (img - target)
    g_parts = oracle.composite_grad(parts, bg, g_out)
    gtf = np.zeros_like(tf)
    gvox = np.zeros(field.shape)
    for (v, dm, lo), gp in zip(bricks, g_parts):
        a, b = oracle.render_brick_grad(cam, v, dm, 1, lo, (1, 1, 1), tf, (0, 1), scale, dt, gp)
        gtf += a
        gvox += oracle.fold_ghost_grad(b, lo, field.shape)
    # table entries enter linearly through the lerp weights: FD is smooth
    h = 1e-6
    checked = 0
    for e in np.argsort(-np.abs(gtf).reshape(-1))[:10]:
        e_, c = divmod(int(e), 4)
        tp, tm = tf.copy(), tf.copy()
        tp[e_, c] += h; tm[e_, c] -= h
        fd = (_loss_parts(cam, bricks, tp, scale, dt, bg, target)[0] -
              _loss_parts(cam, bricks, tm, scale, dt, bg, target)[0]) / (2 * h)
        assert abs(fd - gtf[e_, c]) <= 1e-6 * max(1.0, abs(fd)), (e_, c, fd, gtf[e_, c])
        checked += 1
    assert checked == 10
    # voxels (including ones next to the cut, whose ghost copies fold back)
    h = 1e-6
    for f in np.argsort(-np.abs(gvox).reshape(-1))[:10]:
        z, y, x = np.unravel_index(int(f), field.shape)
        vals = []
        for sgn in (1, -1):
            fp = field.copy()
            fp[z, y, x] += sgn * h
            vals.append(_loss_parts(cam, _bricks64(fp, boxes), tf, scale, dt, bg, target)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gvox[z, y, x]) <= 1e-5 * max(1.0, abs(fd)), (z, y, x, fd, gvox[z, y, x])


# ------------------------------------------------------------------- shadows
def _lattice_count(o, lo, hi, dt):
    """Number of j >= 0 with lo <= o + (j + 1/2) dt < hi (a 1-D count)."""
    return sum(1 for j in range(100000) if lo <= o + (j + 0.5) * dt < hi)


@pytest.mark.parametrize("a0,dt,x,light_sign", [(0.0, 0.5, 4.3, 1), (0.3, 0.5, 1.7, 1), (0.0, 0.25, 6.9, 1),
                                                (0.0, 0.5, 4.3, -1), (1.0, 0.5, 4.3, 1)])
def test_shadow_constant_slab_closed_form(a0, dt, x, light_sign):
    """A constant emitter brick A (x in [0, 8)) seen along -z, a constant
    occluder slab B (x in [10, 14)) beyond a gap, light along +x (or -x, where
    nothing but A itself lies).  Every sample of the pixel's ray has the same
    shadow ray up to a shift along z, so the pixel is the unshadowed closed
    form rgb (1 - (1 - aA)^m) times a0 + (1 - a0) (1 - aA)^nA (1 - aB)^nB, with
    m, nA, nB lattice counts and a = 1 - exp(-scale v dt)."""
    vA, vB, scale, rgb = 0.375, 0.75, 1.5, np.array([1.0, 0.5, 0.25])   # exact in float32
    tf = _ramp_tf(lambda s: (1.0 + 0 * s, 0.5 + 0 * s, 0.25 + 0 * s))
    A = (np.full((6, 10, 10), vA, np.float32), (8, 8, 4), 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    B = (np.full((6, 10, 6), vB, np.float32), (4, 8, 4), 1, (10.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    y, zeye = 3.7, 20.0
    cam = dict(kind="ortho", eye=(x, y, zeye), dir=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), width=1, height=1,
               view_height=1.0)
    light = (float(light_sign), 0.0, 0.0)
    rgba, depth, cnt = oracle.render_brick_shadowed(cam, A, [A, B], tf, (0, 1), scale, dt, light, a0)
    aA, aB = 1.0 - math.exp(-scale * vA * dt), 1.0 - math.exp(-scale * vB * dt)
    m = _lattice_count(-zeye, -4.0, 0.0, dt)             # t along -z: z = zeye - t in [0, 4)
    if light_sign > 0:
        nA, nB = _lattice_count(x, x, 8.0, dt), _lattice_count(x, 10.0, 14.0, dt)
    else:
        nA, nB = _lattice_count(-x, -x, 0.0, dt), 0       # along -x: x - (j + 1/2) dt in [0, x)
    S = (1.0 - aA) ** nA * (1.0 - aB) ** nB
    f = a0 + (1.0 - a0) * S
    np.testing.assert_allclose(rgba[0, 0, :3], rgb * (1.0 - (1.0 - aA) ** m) * f, rtol=0, atol=1e-12)
    assert abs(rgba[0, 0, 3] - (1.0 - (1.0 - aA) ** m)) < 1e-12
    assert depth[0, 0] == min((k + 0.5) * dt for k in range(1000) if 0.0 <= zeye - (k + 0.5) * dt < 4.0)
    assert cnt[0] == m
    # the occluder itself, seen by a ray that misses A, is lit by nothing in front of it
    cam_b = dict(cam, eye=(12.2, y, zeye))
    rgba_b, _, _ = oracle.render_brick_shadowed(cam_b, B, [A, B], tf, (0, 1), scale, dt, light, a0)
    mb = m
    if light_sign > 0:
        Sb = (1.0 - aB) ** _lattice_count(12.2, 12.2, 14.0, dt)
    else:
        Sb = (1.0 - aB) ** _lattice_count(-12.2, -12.2, -10.0, dt) * (1.0 - aA) ** _lattice_count(-12.2, -8.0, 0.0, dt)
    np.testing.assert_allclose(rgba_b[0, 0, :3], rgb * (1.0 - (1.0 - aB) ** mb) * (a0 + (1.0 - a0) * Sb),
                               rtol=0, atol=1e-12)


def test_shadow_ambient_one_equals_unshadowed_bitwise():
    """a0 = 1 turns shadows off: the shadowed partial equals the plain one."""
    rng = np.random.default_rng(21)
    dims = (14, 12, 10)
    field = synth.tile_field(rng, dims, n_blobs=4, noise=0.02, shock=False)
    boxes = synth.kd_split(dims, 3, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, 24, 20, az_deg=35.0, el_deg=25.0, radius_factor=1.7)
    sc = synth.scene_from_field("sh1", field, boxes, synth.default_tf(), cam, 0.5, 2.0)
    desc = [(b.voxels, b.dims, b.ghost, b.origin, (1.0, 1.0, 1.0)) for b in sc.bricks]
    for d in desc:
        a = oracle.render_brick(cam, *d, sc.tf, (0, 1), 2.0, 0.5)
        b = oracle.render_brick_shadowed(cam, d, desc, sc.tf, (0, 1), 2.0, 0.5, (0.3, 1.0, -0.2), 1.0)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and list(a[2]) == list(b[2])


@pytest.mark.parametrize("seed,n_bricks,light", [(31, 2, (1.0, 0.4, 0.2)), (32, 5, (-0.3, 1.0, 0.6))])
def test_shadow_split_invariance(seed, n_bricks, light):
    """Shadow rays see the same samples whatever the decomposition: one
    brick and kd bricks (with ghosts) give the same shadowed image."""
    rng = np.random.default_rng(seed)
    dims = (16, 14, 12)
    field = synth.tile_field(rng, dims, n_blobs=5, noise=0.02, shock=True)
    cam = synth.orbit_camera((0, 0, 0), dims, 20, 16, az_deg=25.0, el_deg=20.0, radius_factor=1.6)
    tf = synth.default_tf()
    bg = (0.1, 0.2, 0.3, 1.0)
    one = synth.scene_from_field("one", field, [((0, 0, 0), dims)], tf, cam, 0.5, 2.0)
    many = synth.scene_from_field("many", field, synth.kd_split(dims, n_bricks, rng), tf, cam, 0.5, 2.0)
    a, _, ca = oracle.render_scene_shadowed(one, light, 0.2, bg=bg)
    b, _, cb = oracle.render_scene_shadowed(many, light, 0.2, bg=bg)
    assert np.max(np.abs(a - b)) < 1e-12
    assert ca[0] == cb[0]
    plain, _, _ = oracle.render_scene(many, bg=bg)
    assert np.max(np.abs(plain - b)) > 1e-3          # the light does darken the image

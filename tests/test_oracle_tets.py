"""Pins of the oracle's tetrahedral-partition renderer (unstructured,
possibly non-convex parts of one mesh) against what the mathematics fixes:

* barycentric interpolation reproduces a linear field exactly on any
  tetrahedron, and trilinear interpolation reproduces it on a grid, so the
  image of a linear field on a mesh of a box equals the image of the same
  field on a brick of that box (an independent renderer of the oracle that
  the brick pins fix);
* the tie rule gives every lattice sample in the box exactly one owner, and
  on the box's faces it agrees with the brick's half-open box, so the owned
  sample count equals a brute-force count -- checked where samples fall
  exactly on vertices, edges and faces of the mesh;
* the image does not depend on how the mesh is split into parts.
"""
import numpy as np
import pytest

import oracle
import synth

CELLS = (4, 3, 5)
COEF = (0.25, 0.125, 0.0625, -0.03125)   # f = c0 + c1 x + c2 y + c3 z, exact in float32 at the points used


def _lin(p):
    return COEF[0] + COEF[1] * p[..., 0] + COEF[2] * p[..., 1] + COEF[3] * p[..., 2]


def _brick_of_linear(cells):
    """Ghost-padded voxels of the linear field on the box [0, cells) with
    unit spacing (voxel centres at i + 1/2; the ghost layer continues the
    field linearly, so trilinear interpolation is exact everywhere)."""
    nx, ny, nz = cells
    z, y, x = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    p = np.stack([x - 0.5, y - 0.5, z - 0.5], -1).astype(np.float64)
    return _lin(p).astype(np.float32)


def _tf():
    tf = synth.hidden_tf(7)
    return tf, (-0.3, 0.9), 1.7


def _brick_image(cam, cells, dt, bg):
    tf, vr, s = _tf()
    rgba, _, cnt = oracle.render_brick(cam, _brick_of_linear(cells), cells, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                                       tf, vr, s, dt)
    a = rgba[..., 3:4]
    return rgba + (1.0 - a) * np.asarray(bg), int(cnt[0])


def _mesh_parts(jitter, seed, n_parts):
    rng = np.random.default_rng(seed)
    v, t = synth.tet_mesh(CELLS, jitter=jitter, rng=rng)
    v = np.round(v * 1024.0) / 1024.0        # dyadic positions: the linear field is exact in float32
    e = v[t[:, 1:]] - v[t[:, :1]]
    assert np.all(np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) > 0)
    vals = _lin(v).astype(np.float32)
    assert np.array_equal(vals, _lin(v))
    if n_parts == 1:
        return [(v, vals, t)]
    return [(pv, vals[used], pt) for pv, pt, used in synth.tet_partitions(v, t, n_parts, rng)]


def _tet_image(cam, parts, dt, bg):
    tf, vr, s = _tf()
    img, cnt = oracle.render_tets(cam, parts, tf, vr, s, dt, bg)
    return img, cnt


def _count_in_box(cam, dt, hi):
    """Brute force: lattice samples o + (k + 1/2) dt d inside [0, hi)."""
    n = 0
    kmax = int(4.0 * (np.linalg.norm(hi) + np.linalg.norm(cam["eye"])) / dt) + 8
    t = (np.arange(kmax) + 0.5) * dt
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            o, d = oracle.ray(cam, i, j)
            p = o[None, :] + t[:, None] * d[None, :]
            n += int(np.sum(np.all((p >= 0.0) & (p < np.asarray(hi, dtype=np.float64)), 1)))
    return n


# Orthographic camera along +z whose pixel centres sit on the half-integer
# lines x, y in {..., -0.5, 0, 0.5, ...} and whose samples (dt = 1/2) sit on
# the planes z = m / 2: samples land on mesh vertices, edges, faces and cube
# centres (all on the main diagonal every tetrahedron of a cube shares).
_ON_LATTICE = dict(kind="ortho", eye=(0.25, 0.25, -1.25), dir=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0),
                   width=16, height=16, view_height=8.0)


def test_on_lattice_samples_have_one_owner_each():
    bg = (0.1, 0.2, 0.3, 0.4)
    img, cnt = _tet_image(_ON_LATTICE, _mesh_parts(0.0, 0, 1), 0.5, bg)
    ref, nref = _brick_image(_ON_LATTICE, CELLS, 0.5, bg)
    brute = _count_in_box(_ON_LATTICE, 0.5, CELLS)
    assert brute > 0
    assert cnt[1] == 0
    assert cnt[0] == brute == nref
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("jitter,seed", [(0.0, 1), (0.2, 2), (0.3, 3)])
def test_linear_field_equals_brick(jitter, seed):
    cam = synth.orbit_camera((0, 0, 0), CELLS, 24, 20, az_deg=35.0, el_deg=25.0, radius_factor=1.6)
    bg = (0.0, 0.05, 0.1, 0.2)
    img, cnt = _tet_image(cam, _mesh_parts(jitter, seed, 1), 0.37, bg)
    ref, nref = _brick_image(cam, CELLS, 0.37, bg)
    assert cnt[1] == 0
    assert cnt[0] == nref == _count_in_box(cam, 0.37, CELLS)
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-11)


def test_eye_inside_mesh():
    cam = synth.inside_camera((0, 0, 0), CELLS, 20, 16, az_deg=-50.0, el_deg=10.0, fovy_deg=70.0)
    img, cnt = _tet_image(cam, _mesh_parts(0.25, 4, 1), 0.29, (0.0, 0.0, 0.0, 0.0))
    ref, nref = _brick_image(cam, CELLS, 0.29, (0.0, 0.0, 0.0, 0.0))
    assert cnt[1] == 0 and cnt[0] == nref
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n_parts,seed,rough", [(3, 5, False), (7, 6, True)])
def test_split_into_parts_is_invariant(n_parts, seed, rough):
    cam = synth.orbit_camera((0, 0, 0), CELLS, 22, 18, az_deg=-20.0, el_deg=40.0, radius_factor=1.5)
    rng = np.random.default_rng(seed)
    v, t = synth.tet_mesh(CELLS, jitter=0.25, rng=rng)
    vals = synth.tet_field(v, rng, CELLS)
    whole, c1 = _tet_image(cam, [(v, vals, t)], 0.31, (0.0, 0.0, 0.0, 0.0))
    parts = [(pv, vals[used], pt) for pv, pt, used in synth.tet_partitions(v, t, n_parts, rng, rough=rough)]
    assert sum(len(p[2]) for p in parts) == len(t)
    split, c2 = _tet_image(cam, parts, 0.31, (0.0, 0.0, 0.0, 0.0))
    assert np.array_equal(whole, split)
    assert np.array_equal(c1, c2) and c1[1] == 0


def test_no_parts_gives_background():
    cam = synth.orbit_camera((0, 0, 0), CELLS, 8, 8)
    img, cnt = oracle.render_tets(cam, [], *_tf(), 0.5, (0.5, 0.25, 0.125, 1.0))
    assert np.all(img == np.array([0.5, 0.25, 0.125, 1.0])) and cnt[0] == 0


def test_mesh_generator_is_conforming():
    """Positive volumes summing to the box volume, and every interior face
    shared by exactly two tetrahedra (the property the tie rule relies on)."""
    v, t = synth.tet_mesh(CELLS, jitter=0.3, rng=np.random.default_rng(9))
    e = v[t[:, 1:]] - v[t[:, :1]]
    vol = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) / 6.0
    assert np.all(vol > 0)
    assert abs(vol.sum() - np.prod(CELLS)) < 1e-9
    faces = np.sort(np.concatenate([t[:, [1, 2, 3]], t[:, [0, 2, 3]], t[:, [0, 1, 3]], t[:, [0, 1, 2]]]), 1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    nx, ny, nz = CELLS
    boundary = 2 * 2 * (nx * ny + ny * nz + nx * nz)
    assert np.sum(counts == 1) == boundary and np.all(counts <= 2)


# ---------------------------------------------------------------- shadows
def _brick_shadowed_image(cam, cells, dt, light, a0, bg):
    tf, vr, s = _tf()
    b = (_brick_of_linear(cells), cells, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    rgba, _, cnt = oracle.render_brick_shadowed(cam, b, [b], tf, vr, s, dt, light, a0)
    a = rgba[..., 3:4]
    return rgba + (1.0 - a) * np.asarray(bg), int(cnt[0])


@pytest.mark.parametrize("jitter,seed,light,a0", [(0.0, 11, (0.3, 1.0, -0.5), 0.2),
                                                  (0.2, 12, (-1.0, 0.0, 0.0), 0.0),
                                                  (0.15, 13, (0.0, -0.4, 1.0), 0.6)])
def test_shadowed_linear_field_equals_shadowed_brick(jitter, seed, light, a0):
    """The shadow rays' samples are lattice points of the box like the
    primary ones, so on a mesh of the box they are the brick's samples."""
    cam = synth.orbit_camera((0, 0, 0), CELLS, 18, 14, az_deg=25.0, el_deg=30.0, radius_factor=1.6)
    bg = (0.05, 0.0, 0.1, 0.3)
    tf, vr, s = _tf()
    img, cnt = oracle.render_tets_shadowed(cam, _mesh_parts(jitter, seed, 1), tf, vr, s, 0.41, light, a0, bg)
    ref, nref = _brick_shadowed_image(cam, CELLS, 0.41, light, a0, bg)
    assert cnt[1] == 0 and cnt[0] == nref and cnt[2] > 0
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-11)


def test_shadowed_ambient_one_is_unshadowed_bitwise():
    cam = synth.orbit_camera((0, 0, 0), CELLS, 16, 12, az_deg=-35.0, el_deg=15.0, radius_factor=1.5)
    parts = _mesh_parts(0.2, 14, 1)
    tf, vr, s = _tf()
    img, _ = oracle.render_tets_shadowed(cam, parts, tf, vr, s, 0.37, (1.0, 2.0, 0.5), 1.0)
    ref, _ = oracle.render_tets(cam, parts, tf, vr, s, 0.37)
    assert np.array_equal(img, ref)


def test_shadowed_split_into_parts_is_invariant():
    cam = synth.orbit_camera((0, 0, 0), CELLS, 16, 14, az_deg=50.0, el_deg=-20.0, radius_factor=1.5)
    rng = np.random.default_rng(15)
    v, t = synth.tet_mesh(CELLS, jitter=0.2, rng=rng)
    vals = synth.tet_field(v, rng, CELLS)
    tf, vr, s = _tf()
    whole, c1 = oracle.render_tets_shadowed(cam, [(v, vals, t)], tf, vr, s, 0.33, (0.5, 1.0, 0.2), 0.25)
    parts = [(pv, vals[used], pt) for pv, pt, used in synth.tet_partitions(v, t, 5, rng, rough=True)]
    split, c2 = oracle.render_tets_shadowed(cam, parts, tf, vr, s, 0.33, (0.5, 1.0, 0.2), 0.25)
    assert np.array_equal(whole, split) and np.array_equal(c1, c2)
    with pytest.raises(ValueError):
        oracle.render_tets_shadowed(cam, parts, tf, vr, s, 0.33, (0.0, 0.0, 0.0), 0.25)


# ------------------------------------------------------ mixed elements
MCELLS = (4, 4, 3)


def _mixed(jitter, seed):
    rng = np.random.default_rng(seed)
    v, sz, cv = synth.mixed_mesh(MCELLS, jitter=jitter, rng=rng)
    v = np.round(v * 1024.0) / 1024.0
    return v, sz, cv


def test_mixed_mesh_decomposes_into_a_conforming_mesh():
    v, sz, cv = _mixed(0.15, 31)
    assert set(np.unique(sz)) == {4, 5, 6, 8}
    vals = np.zeros(len(v), dtype=np.float32)
    V, F, T = oracle.cells_to_tets(v, vals, sz, cv)
    e = V[T[:, 1:]] - V[T[:, :1]]
    vol = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) / 6.0
    assert np.all(np.abs(vol) > 1e-6)
    assert abs(np.abs(vol).sum() - np.prod(MCELLS)) < 1e-9
    faces = np.sort(np.concatenate([T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]]), 1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    nx, ny, nz = MCELLS
    assert np.sum(counts == 1) == 2 * 2 * (nx * ny + ny * nz + nx * nz) and np.all(counts <= 2)


@pytest.mark.parametrize("jitter,seed", [(0.0, 32), (0.15, 33)])
def test_mixed_linear_field_equals_brick(jitter, seed):
    """A linear field is reproduced by every cell's tetrahedra (the centre
    vertices carry the mean of a linear field's node values, which is its
    value at the node centroid), so the mixed mesh renders as the brick."""
    v, sz, cv = _mixed(jitter, seed)
    vals = _lin(v).astype(np.float32)
    V, F, T = oracle.cells_to_tets(v, vals, sz, cv)
    cam = synth.orbit_camera((0, 0, 0), MCELLS, 20, 18, az_deg=-25.0, el_deg=35.0, radius_factor=1.6)
    bg = (0.0, 0.1, 0.0, 0.25)
    tf, vr, s = _tf()
    img, cnt = oracle.render_tets(cam, [(V, F, T)], tf, vr, s, 0.33, bg)
    ref, nref = _brick_image(cam, MCELLS, 0.33, bg)
    assert cnt[1] == 0 and cnt[0] == nref
    # centre values are float32 means (sixths are not dyadic): 1e-6
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-6)


def test_mixed_split_into_parts_is_invariant():
    rng = np.random.default_rng(34)
    v, sz, cv = synth.mixed_mesh(MCELLS, jitter=0.15, rng=rng)
    vals = synth.tet_field(v, rng, MCELLS)
    cam = synth.orbit_camera((0, 0, 0), MCELLS, 18, 16, az_deg=40.0, el_deg=15.0, radius_factor=1.5)
    tf, vr, s = _tf()
    whole, c1 = oracle.render_tets(cam, [oracle.cells_to_tets(v, vals, sz, cv)], tf, vr, s, 0.31)
    parts = []
    for pv, psz, pcv, used in synth.mixed_partitions(v, sz, cv, 4, rng, rough=True):
        parts.append(oracle.cells_to_tets(pv, vals[used], psz, pcv, vertex_ids=used))
    split, c2 = oracle.render_tets(cam, parts, tf, vr, s, 0.31)
    assert np.array_equal(whole, split) and np.array_equal(c1, c2) and c1[1] == 0

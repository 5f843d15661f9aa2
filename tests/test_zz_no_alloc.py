"""vr_render_partials_static (tables in the library's static device array,
no allocation) against vr_render_partials (caller workspace): the partial
images, depth keys and sample counts must be identical, bit for bit, on two
calls in a row, the second with fewer partials (and float16 storage, the
other queue group), and on a third call back at the first size."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_01628_amd as m
    return m


def _scene(seed, dims, n_bricks, w, h, az):
    rng = np.random.default_rng(seed)
    field = synth.tile_field(rng, dims, n_blobs=8, noise=0.02, shock=True)
    boxes = synth.kd_split(dims, n_bricks, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, w, h, az_deg=az, el_deg=17.0, radius_factor=1.7)
    return synth.scene_from_field("noalloc", field, boxes, synth.default_tf(), cam, 0.5, 3.0)


def _snapshot(r):
    out = []
    for k in range(len(r.bricks)):
        rgba, depth = r.partial_arrays(k)
        out.append((rgba.cpu().numpy().copy(), depth.cpu().numpy().copy()))
    return out, r.sample_counts().copy()


def _both_paths(dp, sc, storage):
    r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale,
                    sc.step, storage=storage)
    r.set_camera(sc.camera)
    r.reset_samples()
    r.render_partials()                      # workspace path
    ref, ref_cnt = _snapshot(r)
    for k in range(len(r.bricks)):           # poison the outputs
        rgba, depth = r.partial_arrays(k)
        rgba.fill_(-7.0)
        depth.fill_(-7.0)
    r.reset_samples()
    dp.vr_render_partials_static(r.ctx, r.bricks, r.partials)
    got, got_cnt = _snapshot(r)
    r.close()
    return ref, ref_cnt, got, got_cnt


def _assert_same(ref, ref_cnt, got, got_cnt):
    assert len(ref) == len(got)
    for (a, b), (c, d) in zip(ref, got):
        assert np.array_equal(a, c)
        assert np.array_equal(b, d)
    assert np.array_equal(ref_cnt, got_cnt)


def test_static_scratch_matches_workspace_path(dp):
    big = _scene(71, (40, 36, 30), 12, 97, 75, 35.0)
    small = _scene(72, (26, 22, 18), 5, 61, 47, 120.0)
    _assert_same(*_both_paths(dp, big, dp.VR_F32))
    _assert_same(*_both_paths(dp, small, dp.VR_F16))     # second call: fewer partials
    _assert_same(*_both_paths(dp, big, dp.VR_F32))       # and back to the larger table


def test_static_scratch_rejects_too_many_partials(dp):
    sc = _scene(73, (8, 8, 8), 1, 8, 8, 30.0)
    r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale,
                    sc.step)
    r.set_camera(sc.camera)
    n = dp.STATIC_MAX_PARTIALS + 1
    with pytest.raises(dp.VRError) as e:
        dp.vr_render_partials_static(r.ctx, [r.bricks[0]] * n, [r.partials[0]] * n)
    assert e.value.status == dp.VR_ERR_INVALID_ARG
    assert "static scratch limit" in dp.vr_last_error(r.ctx)
    r.close()

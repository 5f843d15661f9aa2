"""Ray-queue cycling (bricks as ranks, one directional light) through the
C-ABI, against the sort-last path and the FP64 oracle.

* ambient = 1 (no shadow rays): the cycled image equals the sort-last image
  of the same bricks (vr_render_partials + vr_composite) bit for bit, for
  perspective, orthographic and eye-inside views, float32 and float16
  storage, with early termination on.
* shadows on: max |GPU - oracle| <= 1e-5 per channel (float32 storage; the
  oracle's shadowed render of the same bricks), <= 1e-5 against the oracle
  on the decoded voxels with float16 storage; light directions with a zero
  component, one brick, many bricks.
* the plan's slot count equals the oracle's owned-sample count.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
BG = (0.1, 0.2, 0.3, 1.0)


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_01628_amd as m
    return m


def _scene(seed, dims, n_bricks, w, h, az=30.0, el=20.0, radius=1.7, kind="perspective"):
    rng = np.random.default_rng(seed)
    field = synth.tile_field(rng, dims, n_blobs=6, noise=0.02, shock=True)
    boxes = synth.kd_split(dims, n_bricks, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, w, h, az_deg=az, el_deg=el, radius_factor=radius)
    if kind == "ortho":
        c = np.asarray(dims, dtype=np.float64) / 2
        cam = dict(kind="ortho", eye=tuple(c + np.array([0.3, 0.2, -2.0 * dims[2]])), dir=(0.1, 0.05, 1.0),
                   up=(0.0, 1.0, 0.0), view_height=1.1 * max(dims), width=w, height=h)
    return synth.scene_from_field(f"rqc{seed}", field, boxes, synth.default_tf(), cam, 0.5, 2.0)


def _renderer(dp, sc, storage=0, ert=2.0 ** -20, fields=None):
    bricks = [(b.voxels if fields is None else fields[k], b.lo) for k, b in enumerate(sc.bricks)]
    r = dp.Renderer(bricks, sc.tf, sc.vrange, sc.opacity_scale, sc.step, ert, storage=storage)
    r.set_camera(sc.camera)
    return r


CASES = [
    (41, (24, 20, 16), 3, 40, 32, dict()),
    (42, (30, 18, 22), 6, 48, 40, dict(az=130.0, el=-25.0)),
    (43, (20, 20, 20), 4, 36, 36, dict(kind="ortho")),
    (44, (24, 24, 24), 5, 32, 32, dict(radius=0.3)),          # eye inside the volume
]


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("seed,dims,nb,w,h,kw", CASES)
def test_rqc_without_shadows_equals_sort_last(dp, seed, dims, nb, w, h, kw, storage):
    sc = _scene(seed, dims, nb, w, h, **kw)
    r = _renderer(dp, sc, storage=storage)
    ref = r.render(BG).cpu().numpy().copy()
    r.rqc_plan()
    got = r.render_rqc((1.0, 0.3, 0.2), 1.0, BG)
    r.synchronize()
    got = got.cpu().numpy()
    r.close()
    print(f"seed {seed}: max |rqc - sort-last| = {np.max(np.abs(got - ref)):.3g}")
    assert np.array_equal(got, ref)


LIGHTS = [((1.0, 0.6, -0.3), 0.25), ((0.0, 1.0, 0.0), 0.0), ((-0.4, 0.0, 0.9), 0.6)]


@pytest.mark.parametrize("light,ambient", LIGHTS)
@pytest.mark.parametrize("seed,dims,nb,w,h,kw", CASES[:3] + [(45, (22, 18, 16), 1, 32, 24, dict())])
def test_rqc_shadows_against_oracle(dp, seed, dims, nb, w, h, kw, light, ambient):
    sc = _scene(seed, dims, nb, w, h, **kw)
    r = _renderer(dp, sc, ert=0.0)
    total = r.rqc_plan()
    got = r.render_rqc(light, ambient, BG)
    r.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    r.close()
    ref, _, cnt = oracle.render_scene_shadowed(sc, light, ambient, bg=BG)
    err = float(np.max(np.abs(got - ref)))
    print(f"seed {seed} light {light} ambient {ambient}: max |GPU - oracle| = {err:.3g}")
    assert total == cnt[0]
    assert err <= TOL32


def test_rqc_shadows_float16_against_oracle_on_decoded_voxels(dp):
    sc = _scene(46, (26, 22, 18), 4, 40, 32)
    r = _renderer(dp, sc, storage=1, ert=0.0)
    r.rqc_plan()
    got = r.render_rqc((0.7, 0.7, 0.1), 0.2, BG)
    r.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    r.close()
    for b in sc.bricks:
        b.voxels = b.voxels.astype(np.float16).astype(np.float32)
    ref, _, _ = oracle.render_scene_shadowed(sc, (0.7, 0.7, 0.1), 0.2, bg=BG)
    err = float(np.max(np.abs(got - ref)))
    print(f"float16 bricks: max |GPU - oracle(decoded)| = {err:.3g}")
    assert err <= TOL32


def test_rqc_plan_state_errors(dp):
    sc = _scene(47, (16, 16, 16), 2, 16, 16)
    r = _renderer(dp, sc)
    with pytest.raises(dp.VRError) as e:          # no plan yet for this workspace
        nbytes = dp.vr_rqc_workspace_size(r.ctx, r.bricks)
        ws = torch.empty(nbytes // 4 + 64, device="cuda")
        base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
        dp.vr_render_rqc(r.ctx, r.bricks, (1, 0, 0), 1.0, BG, base, nbytes, None, 0, r.frame)
    assert e.value.status == dp.VR_ERR_STATE
    r.rqc_plan()
    cam = dict(sc.camera, width=20)               # camera changed since the plan
    r.set_camera(cam)
    with pytest.raises(dp.VRError) as e:
        r.render_rqc((1, 0, 0), 1.0, BG)
    assert e.value.status == dp.VR_ERR_STATE
    r.close()


def test_rqc_sample_counter(dp):
    """Without early termination and shadows the counter sees each owned
    primary sample once (the plan's slot count); with early termination it
    matches the sort-last march's counter; shadow rays add their samples."""
    sc = _scene(48, (24, 20, 16), 3, 40, 32)
    r = _renderer(dp, sc, ert=0.0)
    total = r.rqc_plan()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    r.render_rqc((1, 0, 0), 1.0, BG, samples=cnt)
    r.synchronize()
    assert int(cnt.item()) == total
    cnt.zero_()
    r.render_rqc((1, 0, 0), 0.5, BG, samples=cnt)
    r.synchronize()
    assert int(cnt.item()) > total
    r.close()
    r = _renderer(dp, sc, ert=2.0 ** -4)
    r.reset_samples()
    r.render(BG)
    sort_last = int(r.sample_counts().sum())
    r.rqc_plan()
    cnt.zero_()
    r.render_rqc((1, 0, 0), 1.0, BG, samples=cnt)
    r.synchronize()
    r.close()
    assert int(cnt.item()) == sort_last

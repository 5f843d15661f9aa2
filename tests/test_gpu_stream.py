"""Time-step streaming through the C-ABI: a series of time steps with only
some resident, played in an order that loads, hits and evicts; every frame
equals, bit for bit, the frame of a renderer that holds that step's bricks
from the start (float32 and float16 storage, one and two resident slots)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BG = (0.1, 0.2, 0.3, 1.0)


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_01628_amd as m
    return m


def _series(n_steps, dims=(28, 24, 20), n_bricks=3, w=40, h=32):
    rng = np.random.default_rng(61)
    boxes = synth.kd_split(dims, n_bricks, rng)
    cam = synth.orbit_camera((0, 0, 0), dims, w, h, az_deg=40.0, el_deg=25.0, radius_factor=1.7)
    scenes = []
    for t in range(n_steps):
        field = synth.tile_field(np.random.default_rng(100 + t), dims, n_blobs=5, noise=0.02, shock=t % 2 == 0)
        scenes.append(synth.scene_from_field(f"step{t}", field, boxes, synth.default_tf(), cam, 0.5, 2.0))
    return scenes, cam


@pytest.mark.parametrize("storage,slots", [(0, 2), (1, 2), (0, 1)])
def test_stream_frames_equal_resident_frames(dp, storage, slots):
    scenes, cam = _series(5)
    ref = []
    for sc in scenes:
        r = dp.Renderer([(b.voxels, b.lo) for b in sc.bricks], sc.tf, sc.vrange, sc.opacity_scale, sc.step,
                        storage=storage)
        r.set_camera(cam)
        ref.append(r.render(BG).cpu().numpy().copy())
        r.close()
    sc0 = scenes[0]
    sr = dp.StreamRenderer([[(b.voxels, b.lo) for b in sc.bricks] for sc in scenes], sc0.tf, sc0.vrange,
                           sc0.opacity_scale, sc0.step, slots=slots, storage=storage)
    sr.set_camera(cam)
    order = [0, 1, 2, 0, 3, 4, 4, 2, 1]
    for i, t in enumerate(order):
        nxt = order[i + 1] if i + 1 < len(order) else None
        img = sr.render(t, BG, prefetch=nxt).cpu().numpy()
        assert np.array_equal(img, ref[t]), f"frame {i} (step {t}) differs"
    loads, resident = sr.stats()
    sr.synchronize()
    sr.close()
    assert len([s for s in resident if s >= 0]) <= slots
    assert loads <= len(order) + (len(order) - 1)      # at most one load per acquire and per prefetch
    if slots == 1:
        assert loads >= len(set(order))

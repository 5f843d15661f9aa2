"""Batched rendering (bricks x time steps x fields x cameras in one
persistent, graph-captured launch) on the GPU.

* every frame and partial of the batch equals the plain path (one Renderer
  frame per camera/time/field), bitwise;
* sampled frames match the oracle (1e-5 float32, 2e-3 float16);
* the autotuner's configurations all give the same bits, and replays of the
  captured graph -- with eager work and synchronisations in between -- give
  the same bits every time;
* with the frames split into release groups, each group's frames are final
  once it is reported done, and all results keep their bits.
"""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def c3_small():
    return synth.config_c3(extent=(10, 44), pitch=46, n_bricks=7, steps=2, fields=2, size=112,
                           n_blobs=10)


def _build(dp, d, storage_of=lambda i: 0, stream=None):
    br = dp.BatchRenderer(dt=d["step"], stream=stream)
    tf = br.add_tf(d["tf"], (0, 1), d["opacity_scale"])
    for i, (t, f, b, lo, vox) in enumerate(d["bricks"]):
        br.add_brick(vox, lo, storage=storage_of(i))
    cams = [br.add_camera(c) for c in d["cameras"]]
    keys = sorted({(t, f) for t, f, _, _, _ in d["bricks"]})
    frames = []
    for (t, f) in keys:
        ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
        for c in cams:
            frames.append(((t, f, c), br.add_frame(c, ids, tf, BG)))
    br.build()
    return br, frames


def test_batch_equals_plain_path(dp, c3_small):
    d = c3_small
    br, frames = _build(dp, d)
    br.launch()
    br.synchronize()
    got = {key: br.frames[fi].cpu().numpy().copy() for key, fi in frames}
    br.close()
    for (t, f, c), img in got.items():
        ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
        r = dp.Renderer([(d["bricks"][i][4], d["bricks"][i][3]) for i in ids], d["tf"], (0, 1),
                        d["opacity_scale"], d["step"])
        r.set_camera(d["cameras"][c])
        ref = r.render(BG).cpu().numpy()
        r.close()
        assert np.array_equal(img, ref), (t, f, c)


def test_batch_matches_oracle(dp, c3_small):
    d = c3_small
    br, frames = _build(dp, d, storage_of=lambda i: i % 2)    # mixed float32 / float16
    br.launch()
    br.synchronize()
    imgs = {key: br.frames[fi].cpu().numpy().astype(np.float64) for key, fi in frames}
    br.close()
    for key in [k for k, _ in frames][::3]:
        t, f, c = key
        ids = [i for i, (tt, ff, _, _, _) in enumerate(d["bricks"]) if (tt, ff) == (t, f)]
        parts = []
        for i in ids:
            _, _, _, lo, vox = d["bricks"][i]
            v = vox if i % 2 == 0 else vox.astype(np.float16).astype(np.float32)
            nz, ny, nx = (s - 2 for s in vox.shape)
            parts.append(oracle.render_brick(d["cameras"][c], v, (nx, ny, nz), 1, lo, (1, 1, 1),
                                             d["tf"], (0, 1), d["opacity_scale"], d["step"])[:2])
        ref = oracle.composite(parts, BG)
        assert np.max(np.abs(imgs[key] - ref)) <= 1e-5, key


def test_autotune_keeps_bits_and_replays_are_stable(dp, c3_small, tmp_path, monkeypatch):
    d = c3_small
    br, frames = _build(dp, d)
    br.launch()
    br.synchronize()
    ref = [br.frames[fi].cpu().numpy().copy() for _, fi in frames]
    ref_parts = [tuple(a.cpu().numpy().copy() for a in br.partial_arrays(j)) for j in range(br.n_jobs)]
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DPVR_AUTOTUNE_CACHE", str(cache))
    ms = br.autotune(reps=2)
    assert ms > 0 and cache.exists()
    wg, order, staging, tile_w, chunk = br.config()
    assert wg >= 1 and order in (0, 1) and staging in (0, 1) and tile_w in (16, 32) and chunk in (4, 8)
    for rep in range(4):
        # eager work and a synchronisation between replays
        for fr in br.frames:
            fr.fill_(-1.0)
        torch.cuda.synchronize()
        br.launch()
        br.synchronize()
        for (_, fi), r in zip(frames, ref):
            assert np.array_equal(br.frames[fi].cpu().numpy(), r), rep
    for j in range(br.n_jobs):
        a = tuple(x.cpu().numpy() for x in br.partial_arrays(j))
        assert np.array_equal(a[0], ref_parts[j][0]) and np.array_equal(a[1], ref_parts[j][1])
    # a second tuning of the same shape comes from the cache
    assert br.autotune(reps=2) == -1.0
    br.close()


def test_autotune_right_after_launch_on_a_side_stream(dp, c3_small, tmp_path, monkeypatch):
    """Tuning rewrites the batch's job table; started right behind a launch
    on a non-blocking side stream it must wait for that launch, so the
    frames stay bit-identical to the reference."""
    d = c3_small
    br, frames = _build(dp, d)
    br.launch()
    br.synchronize()
    ref = [br.frames[fi].cpu().numpy().copy() for _, fi in frames]
    br.close()
    monkeypatch.setenv("DPVR_AUTOTUNE_CACHE", str(tmp_path / "tune_side.txt"))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        br, frames = _build(dp, d, stream=side)
        for fr in br.frames:
            fr.fill_(-1.0)
        br.launch()                 # no synchronisation before the tuning
        br.autotune(reps=1)
        for fr in br.frames:
            fr.fill_(-1.0)
        br.launch()
        br.synchronize()
        got = [br.frames[fi].cpu().numpy() for _, fi in frames]
        br.close()
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_release_groups_keep_bits_and_release_in_order(dp, c3_small, tmp_path, monkeypatch):
    """Frames split into release groups: each group's frames are final once
    the group is reported done (host wait, or a stream waiting on the
    device), and every frame and partial equals the one-group batch bit for
    bit, before and after tuning the grouped batch."""
    d = c3_small
    br, _ = _build(dp, d, storage_of=lambda i: i % 2)
    br.launch()
    br.synchronize()
    ref = [fr.cpu().numpy().copy() for fr in br.frames]
    ref_parts = [tuple(a.cpu().numpy().copy() for a in br.partial_arrays(j)) for j in range(br.n_jobs)]
    nf = len(br.frames)
    for bad in (0, nf + 1):
        with pytest.raises(dp.VRError) as e:
            br.set_groups(bad)
        assert e.value.status == dp.VR_ERR_INVALID_ARG
    br.set_groups(3)
    spans = [br.group(g) for g in range(3)]
    assert spans[0][0] == 0 and sum(n for _, n in spans) == nf
    assert all(spans[g][0] + spans[g][1] == spans[g + 1][0] for g in range(2))
    monkeypatch.setenv("DPVR_AUTOTUNE_CACHE", str(tmp_path / "tune_groups.txt"))
    for rep in range(2):
        for fr in br.frames:
            fr.fill_(-1.0)
        torch.cuda.synchronize()
        br.launch()
        for g, (f0, n) in enumerate(spans):
            br.wait_group(g)
            assert br.group_done(g)
            for fi in range(f0, f0 + n):
                assert np.array_equal(br.frames[fi].cpu().numpy(), ref[fi]), (rep, g, fi)
        br.synchronize()
        for j in range(br.n_jobs):
            a = tuple(x.cpu().numpy() for x in br.partial_arrays(j))
            assert np.array_equal(a[0], ref_parts[j][0]) and np.array_equal(a[1], ref_parts[j][1]), (rep, j)
        if rep == 0:
            br.autotune(reps=1)
    # a stream that waits for the last group on the device
    for fr in br.frames:
        fr.fill_(-1.0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    br.launch()
    br.wait_group(2, side)
    with torch.cuda.stream(side):
        last = br.frames[nf - 1].clone()
    side.synchronize()
    assert np.array_equal(last.cpu().numpy(), ref[nf - 1])
    br.synchronize()
    br.set_groups(1)
    for fr in br.frames:
        fr.fill_(-1.0)
    torch.cuda.synchronize()
    br.launch()
    br.synchronize()
    for fi in range(nf):
        assert np.array_equal(br.frames[fi].cpu().numpy(), ref[fi]), fi
    br.close()


def test_batch_argument_errors(dp, c3_small):
    d = c3_small
    br = dp.BatchRenderer(dt=d["step"])
    br.add_tf(d["tf"], (0, 1), d["opacity_scale"])
    t, f, b, lo, vox = d["bricks"][0]
    br.add_brick(vox, lo)
    br.add_camera(d["cameras"][0])
    br.add_frame(0, [0], 5, BG)            # transfer-function index out of range
    with pytest.raises(dp.VRError) as e:
        br.build()
    assert e.value.status == dp.VR_ERR_INVALID_ARG
    br.close()

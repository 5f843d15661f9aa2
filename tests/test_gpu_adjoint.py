"""Adjoint (differentiable rendering) on the GPU against the oracle.

* GPU gradients (TF table and global voxels) vs the oracle's reverse-mode
  gradients: max |dg| <= 1e-4 * max |g| per parameter group;
* the checkpointed forward equals the plain forward with ERT off, bitwise;
* checkpoint intervals 64, 7 and 1 give the same gradient up to float32
  summation order;
* composite backward vs the oracle's on random partials;
* the 128^3, 8-view, 512^2 differentiable case: GPU gradients vs central
  finite differences (h = 1e-3) of the loss on 32 seeded parameters.
Loss: L = sum over views, pixels and channels of (I - I*)^2.
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


def _small_case(seed=31, dims=(24, 20, 16), nb=3, w=40, h=32, views=2, scale=3.0):
    rng = np.random.default_rng(seed)
    field = synth.tile_field(rng, dims, n_blobs=5, noise=0.05)
    boxes = synth.kd_split(dims, nb, rng)
    cams = [synth.orbit_camera((0, 0, 0), dims, w, h, az_deg=25.0 + 70.0 * v, el_deg=15.0,
                               radius_factor=1.6) for v in range(views)]
    tf = synth.default_tf()
    targets = [rng.uniform(0, 1, (h, w, 4)) for _ in range(views)]
    return field, boxes, cams, tf, targets, scale


def _oracle_grads(field, boxes, cams, tf, targets, scale, dt=0.5, storage=0):
    if storage == 1:      # float16 storage: the oracle sees the decoded voxels
        field = field.astype(np.float16).astype(np.float32)
    gtf = np.zeros((256, 4))
    gvol = np.zeros(field.shape)
    L = 0.0
    for cam, tgt in zip(cams, targets):
        parts, bricks = [], []
        for lo, hi in boxes:
            v = synth.extract_brick(field, lo, hi)
            dims = tuple(int(x) for x in np.subtract(hi, lo))
            parts.append(oracle.render_brick(cam, v, dims, 1, lo, (1, 1, 1), tf, (0, 1), scale,
                                             dt)[:2])
            bricks.append((v, dims, lo))
        img = oracle.composite(parts, BG)
        L += float(np.sum((img - tgt) ** 2))
        gparts = oracle.composite_grad(parts, BG, 2.0 * (img - tgt))
        for (v, dims, lo), gp in zip(bricks, gparts):
            a, b = oracle.render_brick_grad(cam, v, dims, 1, lo, (1, 1, 1), tf, (0, 1), scale, dt, gp)
            gtf += a
            gvol += oracle.fold_ghost_grad(b, lo, field.shape)
    return L, gtf, gvol


def _gpu_grads(dp, field, boxes, cams, tf, targets, scale, interval=64, dt=0.5, storage=0):
    nx, ny, nz = field.shape[2], field.shape[1], field.shape[0]
    dr = dp.DiffRenderer((nx, ny, nz), boxes, (0.0, 1.0), scale, dt, interval, storage=storage)
    tft = torch.tensor(tf, dtype=torch.float32, device="cuda", requires_grad=True)
    vol = torch.tensor(field, dtype=torch.float32, device="cuda", requires_grad=True)
    L = 0.0
    imgs = []
    for cam, tgt in zip(cams, targets):
        img = dr.render(tft, vol, cam, BG)
        loss = ((img.double() - torch.tensor(tgt, device="cuda")) ** 2).sum()
        loss.backward()
        L += float(loss.detach())
        imgs.append(img.detach().cpu().numpy())
    torch.cuda.synchronize()
    out = (L, tft.grad.cpu().numpy().astype(np.float64), vol.grad.cpu().numpy().astype(np.float64),
           imgs)
    dr.close()
    return out


@pytest.mark.parametrize("storage", [0, 1], ids=["f32", "f16"])
def test_gradients_match_oracle(dp, storage):
    """float32 storage, and float16 storage against the oracle on the decoded
    field (the gradient is taken with respect to the stored values)."""
    case = _small_case()
    L_ref, gtf_ref, gvol_ref = _oracle_grads(*case, storage=storage)
    L, gtf, gvol, _ = _gpu_grads(dp, *case, storage=storage)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref) + 1e-6
    for got, ref in ((gtf, gtf_ref), (gvol, gvol_ref)):
        scale = np.max(np.abs(ref))
        assert scale > 0
        err = np.max(np.abs(got - ref))
        assert err <= 1e-4 * scale, (err, scale)


def test_f16_table_gradient_central_differences(dp):
    """float16 storage: table gradients against central differences of the
    GPU loss (the table stays float32, so a perturbation of it is exact)."""
    field, boxes, cams, tf, targets, scale = _small_case(seed=34)
    nx, ny, nz = field.shape[2], field.shape[1], field.shape[0]
    dr = dp.DiffRenderer((nx, ny, nz), boxes, (0.0, 1.0), scale, 0.5, 64, storage=1)
    tft = torch.tensor(tf, dtype=torch.float32, device="cuda", requires_grad=True)
    vol = torch.tensor(field, dtype=torch.float32, device="cuda")
    tg = [torch.tensor(t, device="cuda") for t in targets]

    def loss_of(t_):
        tot = torch.zeros((), dtype=torch.float64, device="cuda")
        for cam, tgt in zip(cams, tg):
            tot = tot + ((dr.render(t_, vol, cam, BG).double() - tgt) ** 2).sum()
        return tot

    loss_of(tft).backward()
    g = tft.grad.double().cpu().numpy()
    cand = np.flatnonzero(np.abs(g).reshape(-1) > 1e-2 * np.abs(g).max())
    h = 1e-3
    with torch.no_grad():
        for idx in np.random.default_rng(35).choice(cand, 8, replace=False):
            e, c = divmod(int(idx), 4)
            tp, tm = tft.detach().clone(), tft.detach().clone()
            tp[e, c] += h
            tm[e, c] -= h
            fd = (float(loss_of(tp)) - float(loss_of(tm))) / (2 * h)
            assert abs(fd - g[e, c]) <= 1e-2 * abs(fd) + 1e-3 * np.abs(g).max(), (e, c, fd, g[e, c])
    dr.close()


@pytest.mark.parametrize("storage", [0, 1], ids=["f32", "f16"])
def test_batched_backward_equals_per_brick_backward(dp, storage):
    """One adjoint launch over all bricks' tiles gives the per-brick
    launches' gradients up to the order of the float atomics."""
    field, boxes, cams, tf, targets, scale = _small_case(seed=36, nb=6)
    nx, ny, nz = field.shape[2], field.shape[1], field.shape[0]
    grads = []
    for batched in (True, False):
        dr = dp.DiffRenderer((nx, ny, nz), boxes, (0.0, 1.0), scale, 0.5, 64, storage=storage)
        dr.batched_backward = batched
        tft = torch.tensor(tf, dtype=torch.float32, device="cuda", requires_grad=True)
        vol = torch.tensor(field, dtype=torch.float32, device="cuda", requires_grad=True)
        for cam, tgt in zip(cams, targets):
            ((dr.render(tft, vol, cam, BG).double() - torch.tensor(tgt, device="cuda")) ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((tft.grad.double().cpu().numpy(), vol.grad.double().cpu().numpy()))
        dr.close()
    for a, b in zip(grads[0], grads[1]):
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))


def test_checkpoint_interval_invariance(dp):
    case = _small_case(seed=32, nb=2)
    ref = _gpu_grads(dp, *case, interval=64)
    for interval in (7, 1):
        got = _gpu_grads(dp, *case, interval=interval)
        for a, b in ((got[1], ref[1]), (got[2], ref[2])):
            assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))
        for ia, ib in zip(got[3], ref[3]):
            assert np.array_equal(ia, ib)


def test_checkpointed_forward_equals_plain_forward(dp):
    field, boxes, cams, tf, _, scale = _small_case(seed=33)
    nx, ny, nz = field.shape[2], field.shape[1], field.shape[0]
    dr = dp.DiffRenderer((nx, ny, nz), boxes, (0.0, 1.0), scale, 0.5, 64)
    img = dr.render(torch.tensor(tf, device="cuda"), torch.tensor(field, device="cuda"), cams[0],
                    BG).cpu().numpy()
    dr.close()
    r = dp.Renderer([(synth.extract_brick(field, lo, hi), lo) for lo, hi in boxes], tf, (0, 1),
                    scale, 0.5, 0.0)
    r.set_camera(cams[0])
    ref = r.render(BG).cpu().numpy()
    r.close()
    assert np.array_equal(img, ref)


@pytest.mark.parametrize("n,seed", [(1, 4), (5, 5), (64, 6)])
def test_composite_backward_matches_oracle(dp, n, seed):
    rng = np.random.default_rng(seed)
    W, H = 37, 29
    ctx = dp.vr_context_create(0, torch.cuda.current_stream())
    dp.vr_set_camera_perspective(ctx, (0, 0, 10.0), (0, 0, 0), (0, 1.0, 0), 45.0, W, H)
    parts, keep, dparts, ref_parts = [], [], [], []
    for p in range(n):
        w, h = int(rng.integers(1, W + 1)), int(rng.integers(1, H + 1))
        x0, y0 = int(rng.integers(0, W - w + 1)), int(rng.integers(0, H - h + 1))
        A = rng.uniform(0, 1, (h, w)).astype(np.float32)
        rgba = np.concatenate([A[..., None] * rng.uniform(0, 1, (h, w, 3)), A[..., None]],
                              -1).astype(np.float32)
        depth = rng.uniform(0, 100, (h, w)).astype(np.float32)
        depth[rng.uniform(0, 1, (h, w)) < 0.2] = np.inf
        rgba[np.isinf(depth)] = 0
        tr, td = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
        keep.append((tr, td))
        parts.append(dp.make_partial((x0, y0, w, h), tr, td))
        dparts.append(torch.full((h * w * 4,), 7.0, device="cuda"))
        fr = np.zeros((H, W, 4)); fd = np.full((H, W), np.inf)
        fr[y0:y0 + h, x0:x0 + w] = rgba; fd[y0:y0 + h, x0:x0 + w] = depth
        ref_parts.append((fr, fd))
    g = rng.normal(0, 1, (H, W, 4)).astype(np.float32)
    dp.vr_composite_backward(ctx, parts, BG, torch.from_numpy(g).cuda(), dparts)
    dp.vr_synchronize(ctx)
    dp.vr_context_release(ctx)
    ref = oracle.composite_grad(ref_parts, BG, g.astype(np.float64))
    for p, (dpt, rg) in enumerate(zip(dparts, ref)):
        x0, y0, w, h = parts[p].x0, parts[p].y0, parts[p].w, parts[p].h
        got = dpt.cpu().numpy().reshape(h, w, 4)
        want = rg[y0:y0 + h, x0:x0 + w].copy()
        want[np.isinf(ref_parts[p][1][y0:y0 + h, x0:x0 + w])] = 0.0
        assert np.max(np.abs(got - want)) <= 1e-5 * max(1.0, np.max(np.abs(want)))


def test_c4_fullsize_finite_differences(dp):
    """128^3 field, 8 views at 512^2, step 0.5, targets rendered by the oracle
    with a hidden TF; gradients of L at the default TF vs central differences
    of the GPU forward loss (float64 sums), h = 1e-3, on 16 TF entries and 16
    voxels with |g| > 1e-3 max|g| (seeded)."""
    sc = synth.config_c4()
    cams = sc.extra["cameras"]
    field = sc.field
    hidden = sc.extra["hidden_tf"]
    targets = []
    for cam in cams:
        img = oracle.render_volume(field, cam, hidden, (0, 1), 1.0, 0.5, bg=BG)
        targets.append(torch.tensor(img, device="cuda"))
    dr = dp.DiffRenderer((128, 128, 128), [((0, 0, 0), (128, 128, 128))], (0.0, 1.0), 1.0, 0.5, 64)
    tf = torch.tensor(synth.default_tf(), device="cuda", requires_grad=True)
    vol = torch.tensor(field, device="cuda", requires_grad=True)

    def loss_of(tf_, vol_):
        tot = torch.zeros((), dtype=torch.float64, device="cuda")
        for cam, tgt in zip(cams, targets):
            tot = tot + ((dr.render(tf_, vol_, cam, BG).double() - tgt) ** 2).sum()
        return tot

    L = loss_of(tf, vol)
    L.backward()
    gtf = tf.grad.double().cpu().numpy()
    gvol = vol.grad.double().cpu().numpy()
    rng = np.random.default_rng(43)
    cand_tf = np.flatnonzero(np.abs(gtf).reshape(-1) > 1e-3 * np.abs(gtf).max())
    cand_v = np.flatnonzero(np.abs(gvol).reshape(-1) > 1e-3 * np.abs(gvol).max())
    pick_tf = rng.choice(cand_tf, 16, replace=False)
    pick_v = rng.choice(cand_v, 16, replace=False)
    h = 1e-3
    with torch.no_grad():
        for idx in pick_tf:
            e, c = divmod(int(idx), 4)
            tp, tm = tf.detach().clone(), tf.detach().clone()
            tp[e, c] += h; tm[e, c] -= h
            fd = (float(loss_of(tp, vol.detach())) - float(loss_of(tm, vol.detach()))) / (2 * h)
            assert abs(fd - gtf[e, c]) <= 1e-2 * abs(fd) + 1e-3 * np.abs(gtf).max(), (e, c, fd, gtf[e, c])
        vflat = vol.detach().reshape(-1)
        for idx in pick_v:
            vp, vm = vflat.clone(), vflat.clone()
            vp[int(idx)] += h; vm[int(idx)] -= h
            fd = (float(loss_of(tf.detach(), vp.view_as(vol))) -
                  float(loss_of(tf.detach(), vm.view_as(vol)))) / (2 * h)
            g = gvol.reshape(-1)[int(idx)]
            assert abs(fd - g) <= 1e-2 * abs(fd) + 1e-3 * np.abs(gvol).max(), (int(idx), fd, g)
    dr.close()

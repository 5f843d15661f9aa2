"""Seeded synthetic inputs for the volume-rendering path.

This module only *makes inputs*: scalar fields on a voxel grid, their kd
decomposition into bricks with a one-voxel ghost layer, transfer-function
tables and camera placements.  It holds none of the rendering arithmetic
(rays, sampling, classification, accumulation, compositing); both the GPU path
and the CPU oracle consume what it returns.

Conventions shared by every generator:

* world units are voxel units; voxel (i, j, k) is a cell whose centre sits at
  (i + 1/2, j + 1/2, k + 1/2) measured from the domain's min corner;
* arrays are stored z-slowest / x-fastest, shape ``(nz, ny, nx)``;
* fields are evaluated in float64 at voxel centres, clamped to [0, 1] and
  cast to float32;
* every random draw comes from ``numpy.random.default_rng(seed)`` in the order
  the generator documents.

The paper's own dataset (a finite-element CFD run distributed as the
simulation left it, uneven partitions, several time steps and fields) is not
available; these fields stand in for it with the same structure: large,
unevenly partitioned, sharp fronts, time-varying, several fields.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field as dc_field

import numpy as np

__all__ = [
    "Brick", "Scene", "default_tf", "hidden_tf", "orbit_camera", "inside_camera",
    "draw_blobs", "add_blobs", "add_shock", "add_fractal_noise", "kd_split", "extract_brick",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5", "tile_field", "scene_from_field",
]

_THREADS = max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------
_DEFAULT_TF_X = np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0])
_DEFAULT_TF_RGB = np.array([[0, 0, .5], [0, .5, 1], [0, 1, .5],
                            [1, 1, 0], [1, .5, 0], [1, 0, 0]], dtype=np.float64)
_DEFAULT_TF_A = np.array([0, 0, .2, .5, .8, 1.0])


def _raster_tf(xs, rgb, a, n=256):
    grid = np.arange(n, dtype=np.float64) / (n - 1)
    out = np.empty((n, 4), dtype=np.float64)
    for c in range(3):
        out[:, c] = np.interp(grid, xs, rgb[:, c])
    out[:, 3] = np.interp(grid, xs, a)
    return out.astype(np.float32)


def default_tf(n: int = 256) -> np.ndarray:
    """Default colour map: six control points rasterised at x_i = i/(n-1).

    Opacity is zero on [0, 0.2] so that low values (blob tails, the empty
    side of a shock) are transparent.
    """
    return _raster_tf(_DEFAULT_TF_X, _DEFAULT_TF_RGB, _DEFAULT_TF_A, n)


def hidden_tf(seed: int = 41, n: int = 256) -> np.ndarray:
    """Seeded colour map used to render fitting targets: 8 sorted control
    points on [0, 1] (first at 0, last at 1), rgb and alpha U(0, 1), alpha at
    x = 0 forced to 0.  Draw order: 6 interior positions, then 8x3 rgb, then 8
    alphas."""
    rng = np.random.default_rng(seed)
    xs = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, 6)), [1.0]])
    rgb = rng.uniform(0, 1, (8, 3))
    a = rng.uniform(0, 1, 8)
    a[0] = 0.0
    return _raster_tf(xs, rgb, a, n)


# --------------------------------------------------------------------------
# cameras (placement only; ray generation belongs to the renderer)
# --------------------------------------------------------------------------
def orbit_camera(domain_lo, domain_hi, width, height, az_deg=30.0, el_deg=20.0,
                 fovy_deg=45.0, radius_factor=2.0):
    """Perspective camera looking at the centre of the domain box from
    ``radius_factor`` x (longest box edge) away, at azimuth/elevation
    (degrees) about +y.  Returns a plain dict of float64 values."""
    lo = np.asarray(domain_lo, dtype=np.float64)
    hi = np.asarray(domain_hi, dtype=np.float64)
    centre = 0.5 * (lo + hi)
    r = radius_factor * float(np.max(hi - lo))
    az, el = math.radians(az_deg), math.radians(el_deg)
    offs = np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return dict(kind="perspective", eye=tuple(float(v) for v in centre + r * offs),
                target=tuple(float(v) for v in centre),
                up=(0.0, 1.0, 0.0), fovy_deg=float(fovy_deg), width=int(width), height=int(height))


def inside_camera(domain_lo, domain_hi, width, height, az_deg=30.0, el_deg=20.0, fovy_deg=45.0):
    """Eye at the centre of the domain, looking along the orbit direction
    (the view where every ray starts inside the data)."""
    lo = np.asarray(domain_lo, dtype=np.float64)
    hi = np.asarray(domain_hi, dtype=np.float64)
    centre = 0.5 * (lo + hi)
    az, el = math.radians(az_deg), math.radians(el_deg)
    offs = np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return dict(kind="perspective", eye=tuple(float(v) for v in centre + 1e-3 * offs),
                target=tuple(float(v) for v in centre - offs),
                up=(0.0, 1.0, 0.0), fovy_deg=float(fovy_deg), width=int(width), height=int(height))


# --------------------------------------------------------------------------
# fields
# --------------------------------------------------------------------------
def draw_blobs(rng, n, dims, sigma=(4.0, 12.0), amp=(0.3, 1.0)):
    """Draw ``n`` Gaussian blobs: centres U[0, dims) (x, y, z order), then
    sigmas, then amplitudes."""
    dims = np.asarray(dims, dtype=np.float64)
    centres = rng.uniform(0.0, 1.0, (n, 3)) * dims
    sig = rng.uniform(sigma[0], sigma[1], n)
    amps = rng.uniform(amp[0], amp[1], n)
    return centres, sig, amps


def add_blobs(acc, centres, sigmas, amps, offset=(0.0, 0.0, 0.0), cutoff=6.0):
    """acc[z, y, x] += sum_b A_b exp(-|p - c_b|^2 / (2 sigma_b^2)) with p the
    voxel centre (+ ``offset``).  The Gaussian is separable, so it is formed
    as an outer product of three 1-D factors and only inside the box
    |p - c| <= cutoff * sigma per axis (outside it every term is below
    exp(-cutoff^2 / 2) * A, i.e. < 1.6e-8 for the default cutoff)."""
    nz, ny, nx = acc.shape
    ox, oy, oz = offset
    for c, s, a in zip(centres, sigmas, amps):
        rad = cutoff * s
        rng_ax = []
        for ax_c, n_ax, o_ax in ((c[0], nx, ox), (c[1], ny, oy), (c[2], nz, oz)):
            lo = max(0, int(math.floor(ax_c - rad - o_ax - 0.5)))
            hi = min(n_ax, int(math.ceil(ax_c + rad - o_ax + 0.5)) + 1)
            rng_ax.append((lo, hi))
        (x0, x1), (y0, y1), (z0, z1) = rng_ax
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            continue
        inv = 1.0 / (2.0 * s * s)
        gx = np.exp(-((np.arange(x0, x1) + 0.5 + ox - c[0]) ** 2) * inv)
        gy = np.exp(-((np.arange(y0, y1) + 0.5 + oy - c[1]) ** 2) * inv)
        gz = np.exp(-((np.arange(z0, z1) + 0.5 + oz - c[2]) ** 2) * inv)
        acc[z0:z1, y0:y1, x0:x1] += (a * gz)[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return acc


def add_shock(acc, normal, p0, amp, width, offset=(0.0, 0.0, 0.0)):
    """acc += 0.5 * amp * (1 - tanh(n . (p - p0) / width)): a planar front
    with tanh profile (value ``amp`` behind the plane, 0 in front)."""
    nz, ny, nx = acc.shape
    n = np.asarray(normal, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    ox, oy, oz = offset
    xs = (np.arange(nx) + 0.5 + ox - p0[0]) * n[0]
    ys = (np.arange(ny) + 0.5 + oy - p0[1]) * n[1]
    zs = (np.arange(nz) + 0.5 + oz - p0[2]) * n[2]
    inv_w = 1.0 / width

    def slab(z):
        arg = (zs[z] + ys[:, None] + xs[None, :]) * inv_w
        acc[z] += 0.5 * amp * (1.0 - np.tanh(arg))

    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(slab, range(nz)))
    return acc


def _finish(acc):
    """Clamp to [0, 1] and cast to float32, slab by slab (keeps peak memory low)."""
    out = np.empty(acc.shape, dtype=np.float32)

    def slab(z):
        np.clip(acc[z], 0.0, 1.0, out=acc[z])
        out[z] = acc[z]

    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(slab, range(acc.shape[0])))
    return out


# --------------------------------------------------------------------------
# decomposition
# --------------------------------------------------------------------------
def kd_split(dims, n_leaves, rng, frac=(0.35, 0.65)):
    """Uneven kd decomposition of the voxel box [0, dims) into ``n_leaves``
    axis-aligned integer boxes.  Repeatedly take the leaf with the most voxels
    (lowest list index on ties), cut it across its longest axis (x < y < z on
    ties) at lo + round(U(frac) * len); the lower part keeps the leaf's list
    slot and the upper part is appended.  Returns a list of (lo, hi) integer
    triples in (x, y, z) order."""
    leaves = [((0, 0, 0), tuple(int(d) for d in dims))]
    while len(leaves) < n_leaves:
        vols = [int(np.prod(np.subtract(hi, lo))) for lo, hi in leaves]
        i = int(np.argmax(vols))
        lo, hi = leaves[i]
        ext = np.subtract(hi, lo)
        ax = int(np.argmax(ext))
        if ext[ax] < 2:
            raise ValueError("leaf too small to split")
        cut = lo[ax] + int(round(rng.uniform(frac[0], frac[1]) * ext[ax]))
        cut = min(max(cut, lo[ax] + 1), hi[ax] - 1)
        hi_a = list(hi); hi_a[ax] = cut
        lo_b = list(lo); lo_b[ax] = cut
        leaves[i] = (tuple(lo), tuple(hi_a))
        leaves.append((tuple(lo_b), tuple(hi)))
    return leaves


def extract_brick(field, lo, hi, ghost=1):
    """Cut box [lo, hi) (x, y, z) out of ``field`` (nz, ny, nx) with ``ghost``
    extra voxels on every face.  Ghost voxels inside the domain are the
    neighbours' voxels; outside it they replicate the edge voxel (index
    clamp).  Returns a C-contiguous float32 array of shape
    (nz_b + 2g, ny_b + 2g, nx_b + 2g)."""
    nz, ny, nx = field.shape
    g = int(ghost)
    ix = np.clip(np.arange(lo[0] - g, hi[0] + g), 0, nx - 1)
    iy = np.clip(np.arange(lo[1] - g, hi[1] + g), 0, ny - 1)
    iz = np.clip(np.arange(lo[2] - g, hi[2] + g), 0, nz - 1)
    # slice the contiguous interior range first (cheap), then fix the clamped edges
    zs = slice(int(iz.min()), int(iz.max()) + 1)
    ys = slice(int(iy.min()), int(iy.max()) + 1)
    xs = slice(int(ix.min()), int(ix.max()) + 1)
    sub = field[zs, ys, xs]
    out = sub[np.ix_(iz - zs.start, iy - ys.start, ix - xs.start)]
    return np.ascontiguousarray(out, dtype=np.float32)


@dataclass
class Brick:
    lo: tuple            # owned box min corner, integer voxel index (x, y, z)
    hi: tuple            # owned box max corner (exclusive)
    voxels: np.ndarray   # ghost-padded float32, (nz+2g, ny+2g, nx+2g)
    ghost: int = 1

    @property
    def dims(self):
        return tuple(int(h - l) for l, h in zip(self.lo, self.hi))

    @property
    def origin(self):
        return tuple(float(l) for l in self.lo)


@dataclass
class Scene:
    name: str
    dims: tuple                  # global (nx, ny, nz)
    field: np.ndarray            # (nz, ny, nx) float32
    bricks: list
    tf: np.ndarray               # (256, 4) float32
    camera: dict
    step: float                  # sample spacing in voxels
    opacity_scale: float
    vrange: tuple = (0.0, 1.0)
    extra: dict = dc_field(default_factory=dict)


def scene_from_field(name, field, boxes, tf, camera, step, opacity_scale, ghost=1, **extra):
    nz, ny, nx = field.shape
    bricks = [Brick(tuple(lo), tuple(hi), extract_brick(field, lo, hi, ghost), ghost)
              for lo, hi in boxes]
    return Scene(name, (nx, ny, nz), field, bricks, tf, camera, float(step),
                 float(opacity_scale), extra=dict(extra))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def config_c1(width=256, height=256):
    """64^3 field: 8 blobs + U(0, 0.02) noise, clamped; split at x = 32 into
    two 32x64x64 bricks; 256x256 orbit view, step 0.5, opacity scale 1.
    Seed 1; draw order: blobs (centres, sigmas, amplitudes), then noise."""
    rng = np.random.default_rng(1)
    dims = (64, 64, 64)
    acc = np.zeros((64, 64, 64), dtype=np.float64)
    add_blobs(acc, *draw_blobs(rng, 8, dims))
    acc += rng.uniform(0.0, 0.02, acc.shape)
    field = _finish(acc)
    boxes = [((0, 0, 0), (32, 64, 64)), ((32, 0, 0), (64, 64, 64))]
    cam = orbit_camera((0, 0, 0), dims, width, height)
    return scene_from_field("c1_64cube_2bricks", field, boxes, default_tf(), cam, 0.5, 1.0)


def config_c2(dims=(1024, 1024, 512), n_bricks=16, width=1920, height=1080, seed=2,
              n_blobs=64):
    """Large field: 64 blobs + one tanh shock front (width 4, amplitude 0.6,
    random normal, plane through centre + U(-1/4, 1/4) * dims); kd split into
    16 uneven bricks; 1920x1080 orbit view, step 0.5, opacity scale 0.05.
    Seed 2; draw order: blobs, shock normal N(0,1)^3, shock offset U^3, kd cuts.
    ``dims``/``width``/``height`` may be reduced for small parity cases; the
    recipe is otherwise unchanged."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    acc = np.zeros((nz, ny, nx), dtype=np.float64)
    add_blobs(acc, *draw_blobs(rng, n_blobs, dims))
    n = rng.normal(0.0, 1.0, 3)
    n /= np.linalg.norm(n)
    p0 = 0.5 * np.asarray(dims, dtype=np.float64) + rng.uniform(-0.25, 0.25, 3) * np.asarray(dims)
    add_shock(acc, n, p0, 0.6, 4.0)
    field = _finish(acc)
    del acc
    boxes = kd_split(dims, n_bricks, rng)
    cam = orbit_camera((0, 0, 0), dims, width, height)
    return scene_from_field(f"c2_{nx}x{ny}x{nz}_{n_bricks}bricks_{width}x{height}", field, boxes,
                            default_tf(), cam, 0.5, 0.05)


def config_c4(n=128, views=8, size=512, seed=4):
    """Differentiable case: n^3 field of 8 blobs (seed 4), one brick, ``views``
    orbit views at az = 45 deg * v, size x size, step 0.5, opacity scale 1.
    Targets are rendered with :func:`hidden_tf`."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    acc = np.zeros((n, n, n), dtype=np.float64)
    add_blobs(acc, *draw_blobs(rng, 8, dims))
    field = _finish(acc)
    boxes = [((0, 0, 0), dims)]
    cams = [orbit_camera((0, 0, 0), dims, size, size, az_deg=45.0 * v) for v in range(views)]
    sc = scene_from_field(f"c4_{n}cube_{views}views", field, boxes, default_tf(), cams[0], 0.5, 1.0)
    sc.extra["cameras"] = cams
    sc.extra["hidden_tf"] = hidden_tf()
    return sc


def add_fractal_noise(acc, rng, amp, octaves=6, base=None, log=None):
    """1/f-like noise: octaves o = 0..octaves-1 of seeded uniform grids with
    spacing base / 2^o voxels, trilinearly upsampled, amplitude proportional
    to the spacing (amp at the coarsest octave), zero mean.  Built slab by
    slab, so large fields need no full-size temporary."""
    nz, ny, nx = acc.shape
    if base is None:
        base = max(8, 2 ** int(math.floor(math.log2(max(nx, ny, nz) / 4))))
    grids = []
    for o in range(octaves):
        sp = base / 2 ** o
        if sp < 2:
            break
        shape = (int(math.ceil(nz / sp)) + 2, int(math.ceil(ny / sp)) + 2, int(math.ceil(nx / sp)) + 2)
        grids.append((sp, amp * sp / base, rng.uniform(-1.0, 1.0, shape)))

    def lerp_axis(n, sp):
        u = (np.arange(n, dtype=np.float64) + 0.5) / sp
        i = np.floor(u).astype(np.int64)
        return i, u - i

    for sp, a, g in grids:
        if log:
            log(f"fractal noise octave, spacing {sp:g}")
        ix, fx = lerp_axis(nx, sp)
        iy, fy = lerp_axis(ny, sp)
        for z in range(nz):
            uz = (z + 0.5) / sp
            iz = int(math.floor(uz))
            fz = uz - iz
            pl = (1 - fz) * g[iz] + fz * g[iz + 1]                    # (gy, gx)
            rows = (1 - fy)[:, None] * pl[iy] + fy[:, None] * pl[iy + 1]   # (ny, gx)
            acc[z] += a * ((1 - fx)[None, :] * rows[:, ix] + fx[None, :] * rows[:, ix + 1])
    return acc


def config_c5(dims=(2048, 1024, 1024), n_bricks=64, width=3840, height=2160, seed=5,
              n_blobs=128, log=None):
    """Large float16 case: blobs + two tanh shock fronts (widths 4 and 8) +
    1/f-like fractal noise (amplitude 0.05), clamped; kd split into
    ``n_bricks`` uneven bricks; 3840x2160 orbit view, step 0.25, opacity 0.05.
    Seed 5; draw order: blobs, shock 1 normal + offset, shock 2 normal +
    offset, noise grids, kd cuts.  ``dims``/``width``/``height`` may be
    reduced for parity cases; the recipe is otherwise unchanged.  ``log``
    (optional) is called with a message after each generation step."""
    say = log or (lambda msg: None)
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    acc = np.zeros((nz, ny, nx), dtype=np.float64)
    add_blobs(acc, *draw_blobs(rng, n_blobs, dims))
    say("blobs")
    for amp, w in ((0.6, 4.0), (0.4, 8.0)):
        n = rng.normal(0.0, 1.0, 3)
        n /= np.linalg.norm(n)
        p0 = 0.5 * np.asarray(dims, dtype=np.float64) + rng.uniform(-0.25, 0.25, 3) * np.asarray(dims)
        add_shock(acc, n, p0, amp, w)
        say(f"shock front, width {w:g}")
    add_fractal_noise(acc, rng, 0.05, log=log)
    field = _finish(acc)
    del acc
    say("clamped to float32")
    boxes = kd_split(dims, n_bricks, rng)
    cam = orbit_camera((0, 0, 0), dims, width, height)
    return scene_from_field(f"c5_{nx}x{ny}x{nz}_{n_bricks}bricks_{width}x{height}", field, boxes,
                            default_tf(), cam, 0.25, 0.05)


def tile_field(rng, dims, n_blobs=8, noise=0.0, shock=False):
    """Small random field for parity cases: blobs (+ noise, + shock)."""
    nx, ny, nz = dims
    acc = np.zeros((nz, ny, nx), dtype=np.float64)
    add_blobs(acc, *draw_blobs(rng, n_blobs, dims, sigma=(max(1.0, min(dims) / 16), max(2.0, min(dims) / 5))))
    if shock:
        n = rng.normal(0.0, 1.0, 3)
        n /= np.linalg.norm(n)
        add_shock(acc, n, 0.5 * np.asarray(dims, dtype=np.float64), 0.6, 2.0)
    if noise > 0:
        acc += rng.uniform(0.0, noise, acc.shape)
    return _finish(acc)


def config_c3(extent=(64, 320), pitch=336, n_bricks=14, steps=6, fields=3, size=1024,
              n_blobs=64, seed=3):
    """Batched case: ``n_bricks`` bricks of uneven extents (each axis
    U{extent[0]..extent[1]}), placed at the min corners of the slots of a
    4 x 2 x 2 grid of pitch ``pitch``; ``steps`` time steps x ``fields``
    fields (density, pressure, velocity magnitude stand-ins: independent
    blob sets, seeds 30, 31, 32, ...; blob centres advected by t * v with
    v U(-4, 4)^3 per blob, scaled with the extent); 4 orbit cameras at az =
    30 + 90 c, ``size`` x ``size``, step 0.5, opacity scale 0.1.  Ghost
    voxels are evaluated from the analytic field (the bricks do not touch).

    Returns dict(bricks=[(t, f, b, lo, voxels)], cameras=[...], tf, dims,
    step, opacity_scale).  Draw order: extents (seed), then per field: blobs,
    velocities (seed 30 + f)."""
    rng = np.random.default_rng(seed)
    ext = rng.integers(extent[0], extent[1] + 1, (n_bricks, 3))
    slots = [(s % 4, (s // 4) % 2, s // 8) for s in range(16)]
    dims = (4 * pitch, 2 * pitch, 2 * pitch)
    vscale = extent[1] / 320.0
    bricks = []
    for f in range(fields):
        frng = np.random.default_rng(30 + f)
        centres, sig, amps = draw_blobs(frng, n_blobs, dims, sigma=(4.0 * vscale, 12.0 * vscale))
        vel = frng.uniform(-4.0, 4.0, (n_blobs, 3)) * vscale
        for t in range(steps):
            c_t = centres + t * vel
            for b in range(n_bricks):
                lo = tuple(int(v) * pitch for v in slots[b])
                e = ext[b]
                shape = (int(e[2]) + 2, int(e[1]) + 2, int(e[0]) + 2)
                acc = np.zeros(shape, dtype=np.float64)
                add_blobs(acc, c_t, sig, amps, offset=(lo[0] - 1, lo[1] - 1, lo[2] - 1))
                np.clip(acc, 0.0, 1.0, out=acc)
                bricks.append((t, f, b, lo, acc.astype(np.float32)))
    cams = [orbit_camera((0, 0, 0), dims, size, size, az_deg=30.0 + 90.0 * c) for c in range(4)]
    return dict(bricks=bricks, cameras=cams, tf=default_tf(), dims=dims, step=0.5,
                opacity_scale=0.1, extents=ext)


# ------------------------------------------------------- tetrahedral meshes
def tet_mesh(cells, jitter=0.0, rng=None, spacing=1.0):
    """Conforming tetrahedral mesh of the box [0, cells * spacing]: vertices
    on the (cells + 1)^3 lattice (interior vertices moved by U(-jitter,
    jitter) x spacing per axis, boundary vertices kept on the box), every
    lattice cube cut into the 6 tetrahedra around its main diagonal (the
    same cut in every cube, so neighbouring cubes share faces).  Returns
    (vertices (V, 3) float64 in x, y, z order, tets (T, 4) int32 with
    positive orientation).  Raises if the jitter inverts a tetrahedron (at
    0.15 none is; from about 0.2 a large mesh has a few)."""
    nx, ny, nz = (int(c) for c in cells)
    gx, gy, gz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    verts = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1).astype(np.float64)
    if jitter > 0.0:
        interior = ((verts[:, 0] > 0) & (verts[:, 0] < nx) & (verts[:, 1] > 0) & (verts[:, 1] < ny) &
                    (verts[:, 2] > 0) & (verts[:, 2] < nz))
        d = rng.uniform(-jitter, jitter, verts.shape)
        verts[interior] += d[interior]
    verts *= spacing

    ci, cj, ck = (a.ravel() for a in np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"))
    perms = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
    tets = np.empty((len(ci), 6, 4), dtype=np.int64)
    for q, p in enumerate(perms):
        c = [ci.copy(), cj.copy(), ck.copy()]
        tets[:, q, 0] = (c[0] * (ny + 1) + c[1]) * (nz + 1) + c[2]
        for m, a in enumerate(p):
            c[a] += 1
            tets[:, q, m + 1] = (c[0] * (ny + 1) + c[1]) * (nz + 1) + c[2]
    tets = tets.reshape(-1, 4).astype(np.int32)
    # orient every tetrahedron positively on the lattice, then require the
    # jittered mesh to keep every orientation (an inverted tetrahedron would
    # overlap its neighbours: the mesh would no longer be conforming)
    gv = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1).astype(np.float64)
    e = gv[tets[:, 1:]] - gv[tets[:, :1]]
    neg = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    e = verts[tets[:, 1:]] - verts[tets[:, :1]]
    if np.any(np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) <= 0.0):
        raise ValueError("jitter inverts a tetrahedron: the mesh would not be conforming")
    return verts, tets


def tet_field(verts, rng, dims, n_blobs=6):
    """Vertex values: Gaussian blobs (as :func:`draw_blobs`, sigma scaled
    to the domain) evaluated at the vertex positions, clamped to [0, 1]."""
    centres, sig, amps = draw_blobs(rng, n_blobs, dims, sigma=(max(dims) / 10, max(dims) / 4))
    v = np.zeros(len(verts))
    for c, s, a in zip(centres, sig, amps):
        v += a * np.exp(-np.sum((verts - c) ** 2, 1) / (2.0 * s * s))
    return np.clip(v, 0.0, 1.0).astype(np.float32)


def tet_partitions(verts, tets, n_parts, rng, rough=False):
    """Uneven, non-convex partitions: each tetrahedron goes to the seed
    nearest its centroid under a seeded weighted distance (weights U(0.5, 2))
    plus a seeded perturbation of up to an eighth of the longest box edge,
    so parts differ in size and are not convex.  The perturbation is smooth
    (three random plane waves of a third of the box per part: contiguous
    parts with wavy boundaries, like a simulation's domain decomposition) or,
    with ``rough``, independent per tetrahedron (ragged, scattered parts
    whose rays enter and leave them many times).  Returns a list of
    (vertices, tets, used) per part: local vertex numbering (shared vertices
    copied), used = the global index of each local vertex."""
    owner = _partition_owner(verts[tets].mean(1), verts.min(0), verts.max(0), n_parts, rng, rough)
    parts = []
    for p in range(n_parts):
        sel = tets[owner == p]
        used, inv = np.unique(sel.ravel(), return_inverse=True)
        parts.append((verts[used].copy(), inv.reshape(-1, 4).astype(np.int32), used))
    return parts


def _partition_owner(cen, lo, hi, n_parts, rng, rough):
    """Part of every element (centroids cen) under the rule of
    :func:`tet_partitions`."""
    seeds = lo + rng.uniform(0.0, 1.0, (n_parts, 3)) * (hi - lo)
    w = rng.uniform(0.5, 2.0, n_parts)
    amp = np.max(hi - lo) / 8.0
    kmag = 2.0 * np.pi / (np.max(hi - lo) / 3.0)
    best = np.full(len(cen), np.inf)
    owner = np.zeros(len(cen), dtype=np.int64)
    for p in range(n_parts):        # one part at a time: memory stays O(elements)
        d = np.sqrt(((cen - seeds[p]) ** 2).sum(1)) / w[p]
        if rough:
            d += rng.uniform(0.0, 1.0, len(cen)) * amp
        else:
            for _ in range(3):
                k = rng.normal(size=3)
                k *= kmag / np.linalg.norm(k)
                d += (amp / 3.0) * (1.0 + np.sin(cen @ k + rng.uniform(0.0, 2.0 * np.pi)))
        better = d < best
        best[better] = d[better]
        owner[better] = p
    return owner


# Node order of the cell types (the common finite-element convention):
# tetrahedron v0..v3; pyramid: base v0..v3 in cyclic order, apex v4; wedge:
# bottom triangle v0 v1 v2, top v3 v4 v5 (v3 above v0, ...); hexahedron:
# bottom v0..v3 cyclic, top v4..v7 (v4 above v0, ...).
CELL_TET, CELL_PYRAMID, CELL_WEDGE, CELL_HEX = 4, 5, 6, 8


def mixed_mesh(cells, jitter=0.0, rng=None, kind=None):
    """Conforming mixed-element mesh of the box [0, cells] (lattice vertices
    as :func:`tet_mesh`, numbered (i (ny+1) + j)(nz+1) + k, interior ones
    jittered).  Each lattice cube becomes, by ``kind(i, j, k)`` (default: the
    four kinds in a 2x2x1 block pattern of 2-cube blocks): 8 one hexahedron,
    6 two wedges (cut along the diagonal plane through its lowest corner and
    the opposite vertical edge), 5 six pyramids on its faces around an added
    centre vertex (the mean of its corners, appended after the lattice), or
    4 the six Kuhn tetrahedra of :func:`tet_mesh`.  Every quadrilateral face
    that two cells share is cut by either along the diagonal through its
    lowest-numbered vertex, the cut the Kuhn tetrahedra and the wedges
    already have, so the mesh is conforming.  Returns (vertices (V, 3)
    float64, sizes (C,) uint8 = vertices per cell, cell_vertices (sum of
    sizes,) int32 in the node order above)."""
    nx, ny, nz = (int(c) for c in cells)
    gx, gy, gz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    verts = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1).astype(np.float64)
    if jitter > 0.0:
        interior = ((verts[:, 0] > 0) & (verts[:, 0] < nx) & (verts[:, 1] > 0) & (verts[:, 1] < ny) &
                    (verts[:, 2] > 0) & (verts[:, 2] < nz))
        d = rng.uniform(-jitter, jitter, verts.shape)
        verts[interior] += d[interior]
    if kind is None:
        def kind(i, j, k):
            return (CELL_HEX, CELL_WEDGE, CELL_PYRAMID, CELL_TET)[((i // 2) % 2) + 2 * ((j // 2) % 2)]

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    sizes, cv, centres = [], [], []
    perms = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                h = [vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k),
                     vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j + 1, k + 1), vid(i, j + 1, k + 1)]
                t = kind(i, j, k)
                if t == CELL_HEX:
                    sizes.append(8)
                    cv += h
                elif t == CELL_WEDGE:
                    sizes += [6, 6]
                    cv += [h[0], h[1], h[2], h[4], h[5], h[6], h[0], h[2], h[3], h[4], h[6], h[7]]
                elif t == CELL_PYRAMID:
                    c = len(verts) + len(centres)
                    centres.append(verts[h].sum(0) / 8.0)
                    for f in ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)):
                        sizes.append(5)
                        cv += [h[f[0]], h[f[1]], h[f[2]], h[f[3]], c]
                else:
                    for p in perms:
                        c = [i, j, k]
                        tt = [vid(*c)]
                        for a in p:
                            c[a] += 1
                            tt.append(vid(*c))
                        sizes.append(4)
                        cv += tt
    if centres:
        verts = np.concatenate([verts, np.asarray(centres)], 0)
    return verts, np.asarray(sizes, dtype=np.uint8), np.asarray(cv, dtype=np.int32)


def mixed_partitions(verts, sizes, cell_vertices, n_parts, rng, rough=False):
    """Parts of a mixed mesh by the rule of :func:`tet_partitions` on cell
    centroids.  Returns a list of (vertices, sizes, cell_vertices, used) per
    part: local numbering, used = the global index of each local vertex."""
    n = sizes.astype(np.int64)
    start = np.concatenate([[0], np.cumsum(n)])
    cen = np.add.reduceat(verts[cell_vertices], start[:-1], axis=0) / n[:, None]
    owner = _partition_owner(cen, verts.min(0), verts.max(0), n_parts, rng, rough)
    slot_owner = np.repeat(owner, n)
    parts = []
    for p in range(n_parts):
        sel = cell_vertices[slot_owner == p]
        used, inv = np.unique(sel, return_inverse=True)
        parts.append((verts[used].copy(), sizes[owner == p].copy(), inv.astype(np.int32), used))
    return parts

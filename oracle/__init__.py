"""FP64 CPU oracle for the volume-rendering path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it, and it shares no code with the GPU path.

The arithmetic lives in ``dpvr_oracle.c`` (plain C, float64, OpenMP over
pixels); this module compiles it with gcc and marshals numpy arrays through
ctypes.  The one piece of arithmetic written here is :func:`fold_ghost_grad`,
the chain rule through ghost-layer extraction (a ghost voxel is a copy of a
global voxel, so its gradient adds to that voxel's).

Conventions (readings of a paper that states no rendering mathematics; each
is listed in the design notes): cell-centred voxels in half-open owned boxes
with a one-voxel ghost layer; samples at t_k = (k + 1/2) dt from the ray
origin, owned by the brick whose box holds the sample point; 256-entry
endpoint-aligned piecewise-linear transfer function; emission-absorption
accumulation front to back; depth key = t of a brick's first owned sample;
sort-last "over" compositing by ascending key, then the background.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpvr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (float64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("pad_", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("dir", C.c_double * 3), ("up", C.c_double * 3), ("fovy_deg", C.c_double),
                ("view_height", C.c_double)]


class _Brick(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("ghost", C.c_int32), ("origin", C.c_double * 3),
                ("spacing", C.c_double * 3), ("vox", C.c_void_p), ("vox_f64", C.c_int32),
                ("pad_", C.c_int32)]


class _TF(C.Structure):
    _fields_ = [("table", C.POINTER(C.c_double)), ("n", C.c_int32), ("pad_", C.c_int32),
                ("vmin", C.c_double), ("vmax", C.c_double), ("opacity_scale", C.c_double)]


_dp = C.POINTER(C.c_double)


class _TetPart(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_tets", C.c_int32), ("vertices", C.POINTER(C.c_double)),
                ("values", C.POINTER(C.c_float)), ("tets", C.POINTER(C.c_int32))]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = C.CDLL(_LIB)
            lib.oc_ray.argtypes = [C.POINTER(_Camera), C.c_int32, C.c_int32, _dp, _dp]
            lib.oc_render_brick.argtypes = [C.POINTER(_Camera), C.POINTER(_Brick), C.POINTER(_TF),
                                            C.c_double, C.c_double, C.POINTER(C.c_int32),
                                            C.c_int64, _dp, _dp, C.POINTER(C.c_int64)]
            lib.oc_composite.argtypes = [C.c_int32, C.POINTER(_dp), C.POINTER(_dp), C.c_int64,
                                         _dp, _dp]
            lib.oc_composite.restype = C.c_int
            lib.oc_composite_grad.argtypes = [C.c_int32, C.POINTER(_dp), C.POINTER(_dp),
                                              C.c_int64, _dp, _dp, C.POINTER(_dp)]
            lib.oc_composite_grad.restype = C.c_int
            lib.oc_render_brick_grad.argtypes = [C.POINTER(_Camera), C.POINTER(_Brick),
                                                 C.POINTER(_TF), C.c_double, _dp, _dp, _dp]
            lib.oc_render_brick_grad.restype = C.c_int
            lib.oc_threads.restype = C.c_int
            lib.oc_render_brick_shadowed.argtypes = [C.POINTER(_Camera), C.POINTER(_Brick), C.c_int32,
                                                     C.POINTER(C.POINTER(_Brick)), C.POINTER(_TF),
                                                     C.c_double, C.c_double, _dp, C.c_double,
                                                     C.POINTER(C.c_int32), C.c_int64, _dp, _dp,
                                                     C.POINTER(C.c_int64)]
            lib.oc_render_brick_shadowed.restype = C.c_int
            lib.oc_render_tets.argtypes = [C.POINTER(_Camera), C.c_int32, C.POINTER(_TetPart), C.POINTER(_TF),
                                           C.c_double, _dp, C.POINTER(C.c_int32), C.c_int64, _dp,
                                           C.POINTER(C.c_int64)]
            lib.oc_render_tets.restype = None
            lib.oc_render_tets_shadowed.argtypes = [C.POINTER(_Camera), C.c_int32, C.POINTER(_TetPart),
                                                    C.POINTER(_TF), C.c_double, _dp, C.c_double, _dp,
                                                    C.POINTER(C.c_int32), C.c_int64, _dp, C.POINTER(C.c_int64)]
            lib.oc_render_tets_shadowed.restype = C.c_int
            lib.oc_set_threads.argtypes = [C.c_int]
            lib.oc_set_threads.restype = None
            _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _camera(cam: dict) -> _Camera:
    c = _Camera()
    kind = cam.get("kind", "perspective")
    c.kind = 0 if kind == "perspective" else 1
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.eye[:] = [float(v) for v in cam["eye"]]
    c.target[:] = [float(v) for v in cam.get("target", (0.0, 0.0, 0.0))]
    c.dir[:] = [float(v) for v in cam.get("dir", (0.0, 0.0, 1.0))]
    c.up[:] = [float(v) for v in cam["up"]]
    c.fovy_deg = float(cam.get("fovy_deg", 45.0))
    c.view_height = float(cam.get("view_height", 1.0))
    return c


class _BrickRef:
    """Keeps the numpy buffer alive next to its ctypes struct."""

    def __init__(self, vox, dims, ghost, origin, spacing):
        f64 = np.asarray(vox).dtype == np.float64
        self.vox = np.ascontiguousarray(vox, dtype=np.float64 if f64 else np.float32)
        g = int(ghost)
        nx, ny, nz = (int(d) for d in dims)
        if self.vox.shape != (nz + 2 * g, ny + 2 * g, nx + 2 * g):
            raise ValueError(f"voxel array shape {self.vox.shape} does not match dims {dims} ghost {g}")
        s = _Brick()
        s.dims[:] = [nx, ny, nz]
        s.ghost = g
        s.origin[:] = [float(v) for v in origin]
        s.spacing[:] = [float(v) for v in spacing]
        s.vox = self.vox.ctypes.data
        s.vox_f64 = 1 if f64 else 0
        self.s = s


class _TFRef:
    def __init__(self, table, vrange, opacity_scale):
        self.table = np.ascontiguousarray(table, dtype=np.float64)
        if self.table.ndim != 2 or self.table.shape[1] != 4 or self.table.shape[0] < 2:
            raise ValueError("transfer function must be (n >= 2, 4)")
        s = _TF()
        s.table = _ptr(self.table, C.c_double)
        s.n = self.table.shape[0]
        s.vmin, s.vmax = float(vrange[0]), float(vrange[1])
        s.opacity_scale = float(opacity_scale)
        self.s = s


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oc_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    _load().oc_set_threads(int(n))


def ray(cam: dict, i: int, j: int):
    """Origin and unit direction (float64) of the ray through pixel (i, j)."""
    lib = _load()
    o = np.zeros(3)
    d = np.zeros(3)
    c = _camera(cam)
    lib.oc_ray(C.byref(c), int(i), int(j), _ptr(o, C.c_double), _ptr(d, C.c_double))
    return o, d


def render_brick(cam, vox, dims, ghost, origin, spacing, tf, vrange, opacity_scale, dt,
                 ert_eps=0.0, pixels=None):
    """Partial image of one brick (``vox`` float32, or float64 for exact
    perturbation studies).

    Returns (rgba, depth, counters): rgba premultiplied colour + alpha, depth
    the key t of the first owned sample (+inf where none), counters =
    [owned samples, samples evaluated by a renderer stopping at T < ert_eps].
    Full frame -> rgba (H, W, 4), depth (H, W); with ``pixels`` (n, 2) of
    (i, j) -> rgba (n, 4), depth (n,).
    """
    lib = _load()
    c = _camera(cam)
    b = _BrickRef(vox, dims, ghost, origin, spacing)
    t = _TFRef(tf, vrange, opacity_scale)
    cnt = np.zeros(2, dtype=np.int64)
    if pixels is None:
        n = c.width * c.height
        shape = (c.height, c.width)
        pix_p, npix = None, 0
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
        shape = (n,)
        pix_p, npix = _ptr(pix, C.c_int32), n
    rgba = np.zeros(n * 4)
    depth = np.zeros(n)
    lib.oc_render_brick(C.byref(c), C.byref(b.s), C.byref(t.s), float(dt), float(ert_eps), pix_p,
                        npix, _ptr(rgba, C.c_double), _ptr(depth, C.c_double),
                        _ptr(cnt, C.c_int64))
    return rgba.reshape(shape + (4,)), depth.reshape(shape), cnt


def composite(partials, bg=(0.0, 0.0, 0.0, 0.0)):
    """Sort-last composite of [(rgba, depth), ...] (same pixel shape) over bg."""
    lib = _load()
    n = len(partials)
    shape = partials[0][1].shape if n else ()
    rg = [np.ascontiguousarray(p[0], dtype=np.float64) for p in partials]
    dp = [np.ascontiguousarray(p[1], dtype=np.float64) for p in partials]
    npx = int(np.prod(shape)) if n else 0
    arr_r = (_dp * max(n, 1))(*[_ptr(a, C.c_double) for a in rg])
    arr_d = (_dp * max(n, 1))(*[_ptr(a, C.c_double) for a in dp])
    bgv = np.asarray(bg, dtype=np.float64)
    out = np.zeros(npx * 4)
    st = lib.oc_composite(n, arr_r, arr_d, npx, _ptr(bgv, C.c_double), _ptr(out, C.c_double))
    if st != 0:
        raise ValueError("too many partials for the oracle composite")
    return out.reshape(tuple(shape) + (4,))


def composite_grad(partials, bg, g_out):
    """dL/d(partial rgba) for each partial, given dL/d(composited image)."""
    lib = _load()
    n = len(partials)
    shape = partials[0][1].shape
    npx = int(np.prod(shape))
    rg = [np.ascontiguousarray(p[0], dtype=np.float64) for p in partials]
    dp = [np.ascontiguousarray(p[1], dtype=np.float64) for p in partials]
    gs = [np.zeros(npx * 4) for _ in range(n)]
    arr_r = (_dp * n)(*[_ptr(a, C.c_double) for a in rg])
    arr_d = (_dp * n)(*[_ptr(a, C.c_double) for a in dp])
    arr_g = (_dp * n)(*[_ptr(a, C.c_double) for a in gs])
    bgv = np.asarray(bg, dtype=np.float64)
    go = np.ascontiguousarray(g_out, dtype=np.float64).reshape(-1)
    st = lib.oc_composite_grad(n, arr_r, arr_d, npx, _ptr(bgv, C.c_double), _ptr(go, C.c_double),
                               arr_g)
    if st != 0:
        raise ValueError("too many partials for the oracle composite")
    return [g.reshape(tuple(shape) + (4,)) for g in gs]


def render_brick_grad(cam, vox, dims, ghost, origin, spacing, tf, vrange, opacity_scale, dt,
                      g_part):
    """Gradient of sum(g_part * partial) w.r.t. the table (n, 4) and the stored
    (ghost-padded) voxels of one brick; no early termination."""
    lib = _load()
    c = _camera(cam)
    b = _BrickRef(vox, dims, ghost, origin, spacing)
    t = _TFRef(tf, vrange, opacity_scale)
    g = np.ascontiguousarray(g_part, dtype=np.float64).reshape(-1)
    if g.size != 4 * c.width * c.height:
        raise ValueError("g_part must be (H, W, 4)")
    gtf = np.zeros(t.table.shape)
    gvox = np.zeros(b.vox.shape)
    st = lib.oc_render_brick_grad(C.byref(c), C.byref(b.s), C.byref(t.s), float(dt),
                                  _ptr(g, C.c_double), _ptr(gtf, C.c_double),
                                  _ptr(gvox, C.c_double))
    if st != 0:
        raise MemoryError("oracle gradient ran out of memory")
    return gtf, gvox


def fold_ghost_grad(gvox_stored, lo, global_shape, ghost=1):
    """Chain rule through ghost extraction: stored voxel (s_x, s_y, s_z) of a
    brick with owned min corner ``lo`` is a copy of global voxel
    clamp(lo + s - g, 0, N - 1) per axis; its gradient adds there."""
    nz, ny, nx = global_shape
    sz, sy, sx = gvox_stored.shape
    g = int(ghost)
    ix = np.clip(np.arange(sx) + lo[0] - g, 0, nx - 1)
    iy = np.clip(np.arange(sy) + lo[1] - g, 0, ny - 1)
    iz = np.clip(np.arange(sz) + lo[2] - g, 0, nz - 1)
    out = np.zeros(global_shape)
    np.add.at(out, np.ix_(iz, iy, ix), gvox_stored)
    return out


# ---------------------------------------------------------------- shadows
def render_brick_shadowed(cam, brick, bricks, tf, vrange, opacity_scale, dt, light_dir, ambient,
                          ert_eps=0.0, pixels=None):
    """Partial image of one brick with one directional light (R-shadow): the
    colour of each owned sample is scaled by ambient + (1 - ambient) S, S the
    transmittance of its shadow ray toward the light through all ``bricks``.
    ``brick`` and every entry of ``bricks`` are (vox, dims, ghost, origin,
    spacing).  Returns (rgba, depth, counters) as :func:`render_brick`."""
    lib = _load()
    c = _camera(cam)
    refs = [_BrickRef(*bb) for bb in bricks]
    me = _BrickRef(*brick)
    arr = (C.POINTER(_Brick) * max(len(refs), 1))(*[C.pointer(r.s) for r in refs])
    t = _TFRef(tf, vrange, opacity_scale)
    l = np.ascontiguousarray(light_dir, dtype=np.float64)
    if pixels is None:
        n = c.width * c.height
        pix_p = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
        pix_p = _ptr(pix, C.c_int32)
    rgba = np.zeros(n * 4)
    depth = np.zeros(n)
    cnt = np.zeros(2, dtype=np.int64)
    st = lib.oc_render_brick_shadowed(C.byref(c), C.byref(me.s), len(refs), arr, C.byref(t.s), float(dt),
                                      float(ert_eps), _ptr(l, C.c_double), float(ambient), pix_p, n,
                                      _ptr(rgba, C.c_double), _ptr(depth, C.c_double),
                                      _ptr(cnt, C.c_int64))
    if st != 0:
        raise ValueError("bad light direction or ambient fraction")
    if pixels is None:
        return rgba.reshape(c.height, c.width, 4), depth.reshape(c.height, c.width), cnt
    return rgba.reshape(n, 4), depth, cnt


def render_scene_shadowed(scene, light_dir, ambient, camera=None, bg=(0.0, 0.0, 0.0, 0.0), pixels=None,
                          ert_eps=0.0):
    """Final image of a :class:`synth.Scene` with R-shadow: every brick's
    shadowed partial, composited over bg.  Returns (image, partials, counters)."""
    cam = camera or scene.camera
    desc = [(b.voxels, b.dims, b.ghost, b.origin, (1.0, 1.0, 1.0)) for b in scene.bricks]
    parts, counters = [], np.zeros(2, dtype=np.int64)
    for d in desc:
        rgba, depth, cnt = render_brick_shadowed(cam, d, desc, scene.tf, scene.vrange, scene.opacity_scale,
                                                 scene.step, light_dir, ambient, ert_eps, pixels)
        parts.append((rgba, depth))
        counters += cnt
    return composite(parts, bg), parts, counters


# ----------------------------------------------------- tetrahedral parts
def render_tets(cam, parts, tf, vrange, opacity_scale, dt, bg=(0.0, 0.0, 0.0, 0.0), pixels=None):
    """Image of the volume given as tetrahedral parts [(vertices (V, 3)
    float64, values (V,) float32, tets (T, 4) int32)], over bg (R-tet,
    R-ea).  Returns (image, counters) with counters = [samples held by a
    tetrahedron, samples held by more than one]."""
    return _render_tets(cam, parts, tf, vrange, opacity_scale, dt, bg, pixels, None, None)


def _quad(q, ids):
    """Triangles of the quadrilateral q (cyclic) cut along the diagonal
    through its vertex of smallest id (R-cells)."""
    a, b, c, d = q
    m = min(range(4), key=lambda i: ids[q[i]])
    if m in (0, 2):
        return [(a, b, c), (a, c, d)]
    return [(a, b, d), (b, c, d)]


_WEDGE_FACES = ((0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5))
_HEX_FACES = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))


def cells_to_tets(vertices, values, sizes, cell_vertices, vertex_ids=None):
    """R-cells: the tetrahedra of a mixed-element part.  Tetrahedra stay;
    a pyramid is its base's two triangles joined to the apex; a wedge and a
    hexahedron get a centre vertex (position: the sum of the node positions
    in node order over the node count, float64; value: the mean of the node
    values) joined to every triangle of its faces.  Every quadrilateral is
    cut along the diagonal through its vertex of smallest id (vertex_ids,
    default the vertex index), so cells that share it cut it alike.
    Returns (vertices, values (float32), tets (T, 4) int32) with the centre
    vertices appended."""
    V = [tuple(float(x) for x in v) for v in np.asarray(vertices, dtype=np.float64).reshape(-1, 3)]
    F = [float(x) for x in np.asarray(values, dtype=np.float32)]
    ids = list(range(len(V))) if vertex_ids is None else [int(x) for x in vertex_ids]
    out = []
    pos = 0
    for n in (int(x) for x in sizes):
        cell = [int(x) for x in cell_vertices[pos:pos + n]]
        pos += n
        if n == 4:
            out.append(tuple(cell))
        elif n == 5:
            for t in _quad(cell[:4], ids):
                out.append(t + (cell[4],))
        elif n in (6, 8):
            c = len(V)
            sx = sy = sz = 0.0
            sv = 0.0
            for q in cell:
                sx += V[q][0]
                sy += V[q][1]
                sz += V[q][2]
                sv += F[q]
            V.append((sx / n, sy / n, sz / n))
            F.append(sv / n)
            ids.append(-1)                  # a centre vertex lies on no quadrilateral
            for f in (_WEDGE_FACES if n == 6 else _HEX_FACES):
                nodes = [cell[i] for i in f]
                for t in ([tuple(nodes)] if len(nodes) == 3 else _quad(nodes, ids)):
                    out.append(t + (c,))
        else:
            raise ValueError(f"cell with {n} vertices")
    return (np.asarray(V, dtype=np.float64).reshape(-1, 3), np.asarray(F, dtype=np.float32),
            np.asarray(out, dtype=np.int32).reshape(-1, 4))


def render_tets_shadowed(cam, parts, tf, vrange, opacity_scale, dt, light_dir, ambient,
                         bg=(0.0, 0.0, 0.0, 0.0), pixels=None):
    """render_tets with one directional light (R-shadow): every held primary
    sample's colour scaled by ambient + (1 - ambient) S, S the transmittance
    of its shadow ray through all parts.  Returns (image, counters) with
    counters = [primary samples held, held more than once, shadow samples
    held]."""
    return _render_tets(cam, parts, tf, vrange, opacity_scale, dt, bg, pixels, light_dir, ambient)


def _render_tets(cam, parts, tf, vrange, opacity_scale, dt, bg, pixels, light_dir, ambient):
    lib = _load()
    c = _camera(cam)
    keep = []
    arr = (_TetPart * max(len(parts), 1))()
    for i, (v, f, t) in enumerate(parts):
        v = np.ascontiguousarray(v, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        keep += [v, f, t]
        arr[i] = _TetPart(len(v), len(t), _ptr(v, C.c_double), _ptr(f, C.c_float), _ptr(t, C.c_int32))
    tfr = _TFRef(tf, vrange, opacity_scale)
    bgv = np.asarray(bg, dtype=np.float64)
    if pixels is None:
        n = c.width * c.height
        pix_p = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
        pix_p = _ptr(pix, C.c_int32)
    out = np.zeros(n * 4)
    if light_dir is None:
        cnt = np.zeros(2, dtype=np.int64)
        lib.oc_render_tets(C.byref(c), len(parts), arr, C.byref(tfr.s), float(dt), _ptr(bgv, C.c_double), pix_p,
                           n, _ptr(out, C.c_double), _ptr(cnt, C.c_int64))
    else:
        cnt = np.zeros(3, dtype=np.int64)
        lv = np.asarray(light_dir, dtype=np.float64)
        rc = lib.oc_render_tets_shadowed(C.byref(c), len(parts), arr, C.byref(tfr.s), float(dt),
                                         _ptr(lv, C.c_double), float(ambient), _ptr(bgv, C.c_double), pix_p, n,
                                         _ptr(out, C.c_double), _ptr(cnt, C.c_int64))
        if rc != 0:
            raise ValueError("light direction must be non-zero and ambient in [0, 1]")
    if pixels is None:
        return out.reshape(c.height, c.width, 4), cnt
    return out.reshape(n, 4), cnt


# ---------------------------------------------------------------- scenes
def render_scene_partials(scene, camera=None, ert_eps=0.0, pixels=None, field_override=None):
    """Partial image of every brick of a :class:`synth.Scene`."""
    cam = camera or scene.camera
    parts, counters = [], np.zeros(2, dtype=np.int64)
    for k, b in enumerate(scene.bricks):
        vox = b.voxels if field_override is None else field_override[k]
        rgba, depth, cnt = render_brick(cam, vox, b.dims, b.ghost, b.origin, (1.0, 1.0, 1.0),
                                        scene.tf, scene.vrange, scene.opacity_scale, scene.step,
                                        ert_eps, pixels)
        parts.append((rgba, depth))
        counters += cnt
    return parts, counters


def render_scene(scene, camera=None, bg=(0.0, 0.0, 0.0, 0.0), pixels=None, ert_eps=0.0,
                 field_override=None):
    """Final image of a scene: every brick's partial, composited over bg."""
    parts, counters = render_scene_partials(scene, camera, ert_eps, pixels, field_override)
    return composite(parts, bg), parts, counters


def render_volume(field, cam, tf, vrange, opacity_scale, dt, bg=(0.0, 0.0, 0.0, 0.0),
                  origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), pixels=None):
    """Whole field rendered as a single brick without ghosts (the reconstruction
    clamps to the edge), composited over bg."""
    nz, ny, nx = field.shape
    rgba, depth, _ = render_brick(cam, field, (nx, ny, nz), 0, origin, spacing, tf, vrange,
                                  opacity_scale, dt, 0.0, pixels)
    return composite([(rgba, depth)], bg)

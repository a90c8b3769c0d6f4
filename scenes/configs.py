"""Seeded synthetic scenes for the five benchmark configurations and test fixtures.

Conventions (all inputs are FP64 numpy arrays):

* A patch has degrees ``degree[3]``, control-point counts ``ncp[3]`` and clamped,
  non-decreasing knot vectors on [0, 1] (open uniform unless stated).
* ``cp`` has shape ``(ncp0*ncp1*ncp2, 4)`` holding ``(x, y, z, w)``; index
  ``i + ncp0*(j + ncp1*k)`` (i fastest).  ``w`` is 1 for plain B-splines.
* ``scalar`` holds the coefficients of the scalar spline rho in the same layout.
* Transfer function: ``n_knots`` abscissae on [0, 1] (first 0, last 1) with an
  RGBA value at each; ``domain`` maps rho to [0, 1]; ``extinction`` scales A.
* Camera: pinhole with ``eye``, ``target``, ``up``, vertical field of view.

RNG: ``numpy.random.Generator(PCG64(seed))`` with seed ``1000*k + role`` for
config k and role 1 geometry, 2 field, 3 transfer function, 4 camera, 5 MLP.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

ROLE_GEOM, ROLE_FIELD, ROLE_TF, ROLE_CAM, ROLE_MLP = 1, 2, 3, 4, 5


def rng_for(config: int, role: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + role))


@dataclass
class Patch:
    degree: tuple
    ncp: tuple
    knots: List[np.ndarray]
    cp: np.ndarray            # (N, 4) x, y, z, w
    scalar: np.ndarray        # (N,)
    rational: bool = False
    displacement: Optional[np.ndarray] = None   # (N, 3) displacement spline u, or None

    def grid(self) -> np.ndarray:
        """Control points as an array indexed [k, j, i, c]."""
        n0, n1, n2 = self.ncp
        return self.cp.reshape(n2, n1, n0, 4)


@dataclass
class TransferFunction:
    x: np.ndarray             # (n,)
    rgba: np.ndarray          # (n, 4)
    extinction: float
    domain: tuple             # (r_lo, r_hi)


@dataclass
class Camera:
    eye: np.ndarray
    target: np.ndarray
    up: np.ndarray
    fov_y_deg: float
    width: int
    height: int


@dataclass
class Scene:
    name: str
    patches: List[Patch]
    tf: TransferFunction
    cameras: List[Camera]
    bbox: np.ndarray          # (2, 3) bounding box of all control points
    params: dict = field(default_factory=dict)

    @property
    def scale(self) -> float:
        """Length of the bounding-box diagonal (the scene's length scale)."""
        return float(np.linalg.norm(self.bbox[1] - self.bbox[0]))


# ---------------------------------------------------------------- knots

def open_uniform_knots(n: int, p: int) -> np.ndarray:
    """Clamped knot vector on [0,1] with n control points and uniform interior knots."""
    nspan = n - p
    interior = [m / nspan for m in range(1, nspan)]
    return np.array([0.0] * (p + 1) + interior + [1.0] * (p + 1))


def greville(t: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae: the mean of p consecutive interior knots."""
    n = len(t) - p - 1
    return np.array([np.mean(t[i + 1:i + p + 1]) for i in range(n)])


def _grid_points(xi, eta, zeta):
    """Tensor grid of parameter triples, indexed [k, j, i]."""
    Z, Y, X = np.meshgrid(zeta, eta, xi, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _make_patch(degree, ncp, knots, xyz, scalar, w=None, rational=False) -> Patch:
    n = int(np.prod(ncp))
    cp = np.empty((n, 4))
    cp[:, :3] = xyz.reshape(n, 3)
    cp[:, 3] = 1.0 if w is None else w.reshape(n)
    return Patch(tuple(int(d) for d in degree), tuple(int(c) for c in ncp),
                 [np.asarray(k, dtype=np.float64) for k in knots], cp,
                 np.asarray(scalar, dtype=np.float64).reshape(n), rational)


def bbox_of(patches) -> np.ndarray:
    pts = np.concatenate([p.cp[:, :3] for p in patches])
    return np.stack([pts.min(0), pts.max(0)])


# ---------------------------------------------------------------- transfer function

def random_tf(rng: np.random.Generator, extinction: float, domain, n_knots: int = 8
              ) -> TransferFunction:
    """First knot 0, last 1, the rest sorted U[0,1); RGBA at every knot U[0,1]^4."""
    inner = np.sort(rng.uniform(0.0, 1.0, n_knots - 2))
    x = np.concatenate([[0.0], inner, [1.0]])
    rgba = rng.uniform(0.0, 1.0, (n_knots, 4))
    return TransferFunction(x, rgba, float(extinction), (float(domain[0]), float(domain[1])))


def scalar_domain(patches):
    """Transfer-function domain: min and max scalar coefficient (the hull bounds rho)."""
    s = np.concatenate([p.scalar for p in patches])
    lo, hi = float(s.min()), float(s.max())
    if hi <= lo:
        hi = lo + 1.0
    return lo, hi


def extinction_for(bbox) -> float:
    """Same optical thickness as a unit cube with extinction 4: 4*sqrt(3)/diag."""
    return 4.0 * math.sqrt(3.0) / float(np.linalg.norm(bbox[1] - bbox[0]))


# ---------------------------------------------------------------- camera

def camera_from_angles(target, dist, az_deg, el_deg, width, height, fov_y_deg=40.0) -> Camera:
    """Eye on a sphere around the target; +z up."""
    az, el = math.radians(az_deg), math.radians(el_deg)
    target = np.asarray(target, dtype=np.float64)
    eye = target + dist * np.array([math.cos(el) * math.cos(az),
                                    math.cos(el) * math.sin(az), math.sin(el)])
    return Camera(eye, target, np.array([0.0, 0.0, 1.0]), float(fov_y_deg), int(width), int(height))


def _framing_distance(bbox, fov_y_deg=40.0, margin=1.1):
    radius = 0.5 * float(np.linalg.norm(bbox[1] - bbox[0]))
    return margin * radius / math.sin(math.radians(fov_y_deg) / 2.0)


def _fit_distance(points, target, az_deg, el_deg, width, height, fov_y_deg=40.0, fill=0.95):
    """Smallest eye distance at which every point projects inside `fill` of the
    screen (bisection on the distance; pinhole projection of the points)."""
    az, el = math.radians(az_deg), math.radians(el_deg)
    back = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    f = -back
    r = np.cross(f, [0.0, 0.0, 1.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(fov_y_deg) / 2.0)
    aspect = width / height
    rel = np.asarray(points) - np.asarray(target)

    def fits(dist):
        depth = rel @ f + dist
        if (depth <= 1e-6).any():
            return False
        sx = (rel @ r) / depth / (th * aspect)
        sy = (rel @ u) / depth / th
        return max(np.abs(sx).max(), np.abs(sy).max()) <= fill

    radius = float(np.linalg.norm(rel, axis=1).max())
    lo, hi = 1e-3, 4.0 * radius / math.sin(math.radians(fov_y_deg) / 2.0)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if fits(mid) else (mid, hi)
    return hi


def _seeded_cameras(config, bbox, n, width, height, points=None):
    """n views with az ~ U[0,360), el ~ U[-45,45] about the bbox centre, each at the
    distance that fits the control points to the screen."""
    rng = rng_for(config, ROLE_CAM)
    target = 0.5 * (bbox[0] + bbox[1])
    cams = []
    for _ in range(n):
        az = rng.uniform(0.0, 360.0)
        el = rng.uniform(-45.0, 45.0)
        dist = (_fit_distance(points, target, az, el, width, height) if points is not None
                else _framing_distance(bbox))
        cams.append(camera_from_angles(target, dist, az, el, width, height))
    return cams


# ---------------------------------------------------------------- fixtures

def affine_patch(A, b, degree=(2, 2, 2), ncp=(4, 4, 4), scalar=None) -> Patch:
    """Control points A*greville+b: by linear precision the map is exactly p -> A p + b."""
    knots = [open_uniform_knots(ncp[d], degree[d]) for d in range(3)]
    g = _grid_points(*(greville(knots[d], degree[d]) for d in range(3)))
    xyz = g @ np.asarray(A, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
    if scalar is None:
        scalar = np.zeros(int(np.prod(ncp)))
    elif callable(scalar):
        scalar = scalar(g.reshape(-1, 3))
    return _make_patch(degree, ncp, knots, xyz, scalar)


# ---------------------------------------------------------------- config 1

def _config1() -> Scene:
    """One degree-2 patch, 4^3 control points forming the unit cube; the 8 interior
    control points jittered by U[-0.05,0.05]^3; rho coefficients U[0,1]."""
    p, n = (2, 2, 2), (4, 4, 4)
    knots = [open_uniform_knots(4, 2)] * 3            # [0,0,0,.5,1,1,1]
    gr = greville(knots[0], 2)                        # [0,.25,.75,1]
    xyz = _grid_points(gr, gr, gr).copy()
    rg = rng_for(1, ROLE_GEOM)
    for k in (1, 2):
        for j in (1, 2):
            for i in (1, 2):
                xyz[k, j, i] += rg.uniform(-0.05, 0.05, 3)
    scalar = rng_for(1, ROLE_FIELD).uniform(0.0, 1.0, 64)
    patch = _make_patch(p, n, knots, xyz, scalar)
    tf = random_tf(rng_for(1, ROLE_TF), 4.0, scalar_domain([patch]))
    cam = camera_from_angles([0.5, 0.5, 0.5], 3.0, 30.0, 20.0, 64, 64)
    bbox = bbox_of([patch])
    return Scene("config1_unit_cube_deg2", [patch], tf, [cam], bbox,
                 dict(precision="fp64", rk_tol=1e-6))


# ---------------------------------------------------------------- config 2

def _basis_matrices(t, k, x):
    """Dense value and first-derivative B-spline collocation matrices (scipy)."""
    from scipy.interpolate import BSpline
    n = len(t) - k - 1
    B = np.zeros((len(x), n))
    dB = np.zeros((len(x), n))
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        s = BSpline(t, c, k, extrapolate=True)
        B[:, i] = s(x)
        dB[:, i] = s.derivative()(x)
    return B, dB


def _config2() -> Scene:
    """Twisted bar: cubic, 8x8x32 control points, cross-section 1x1, length 8, twisted
    180 degrees linearly along its length.  The scalar field interpolates the spline's
    det J at the Greville points (tensor-product collocation)."""
    p, n = (3, 3, 3), (8, 8, 32)
    knots = [open_uniform_knots(n[d], p[d]) for d in range(3)]
    gx, gy, gz = (greville(knots[d], p[d]) for d in range(3))
    g = _grid_points(gx, gy, gz)
    ang = math.pi * g[..., 2]
    cx, cy = g[..., 0] - 0.5, g[..., 1] - 0.5
    xyz = np.stack([np.cos(ang) * cx - np.sin(ang) * cy,
                    np.sin(ang) * cx + np.cos(ang) * cy,
                    8.0 * g[..., 2]], axis=-1)
    # det J of the spline at the Greville points, via scipy's B-spline basis
    Bu, dBu = _basis_matrices(knots[0], 3, gx)
    Bv, dBv = _basis_matrices(knots[1], 3, gy)
    Bw, dBw = _basis_matrices(knots[2], 3, gz)
    Pu = np.einsum("ai,bj,ck,kjid->cbad", dBu, Bv, Bw, xyz)
    Pv = np.einsum("ai,bj,ck,kjid->cbad", Bu, dBv, Bw, xyz)
    Pw = np.einsum("ai,bj,ck,kjid->cbad", Bu, Bv, dBw, xyz)
    detj = np.linalg.det(np.stack([Pu, Pv, Pw], axis=-1))
    coef = np.einsum("ia,jb,kc,cba->kji", np.linalg.inv(Bu), np.linalg.inv(Bv),
                     np.linalg.inv(Bw), detj)
    patch = _make_patch(p, n, knots, xyz, coef)
    bbox = bbox_of([patch])
    tf = random_tf(rng_for(2, ROLE_TF), extinction_for(bbox), scalar_domain([patch]))
    rng = rng_for(2, ROLE_CAM)
    cams = []
    dist = 1.1 * 4.06 / math.sin(math.radians(20.0))
    for _ in range(3):
        az = rng.uniform(0.0, 360.0)
        el = rng.uniform(-45.0, 45.0)
        cams.append(camera_from_angles([0.0, 0.0, 4.0], dist, az, el, 512, 512))
    return Scene("config2_twisted_bar", [patch], tf, cams, bbox,
                 dict(precision="fp32", rk_tol=1e-5))


# ---------------------------------------------------------------- config 3

def _gaussian_field(rng, bbox, n=3, ramp=0.5):
    """Sum of n Gaussians (sigma 0.1-0.3) plus a linear ramp, in bbox-normalised coords."""
    c = rng.uniform(0.0, 1.0, (n, 3))
    sig = rng.uniform(0.1, 0.3, n)
    amp = rng.uniform(0.5, 1.0, n)
    lo = bbox[0]
    ext = float((bbox[1] - bbox[0]).max())

    def f(x):
        xh = (np.asarray(x) - lo) / ext
        r = ramp * xh[..., 0]
        for q in range(n):
            d2 = np.sum((xh - c[q]) ** 2, axis=-1)
            r = r + amp[q] * np.exp(-d2 / (2.0 * sig[q] ** 2))
        return r
    return f


def _config3(width=1920, height=1080) -> Scene:
    """Straight beam [0,4]x[0,1]^2 tiled 4x4x4, each tile a cubic patch with 10^3
    control points at its Greville points, bent through 90 degrees about z.  Shared
    faces carry identical control points (C0, watertight).  Field: three Gaussians
    plus a ramp, quasi-interpolated (coefficient = field at the control point)."""
    p, n = (3, 3, 3), (10, 10, 10)
    knots = [open_uniform_knots(10, 3)] * 3
    gr = greville(knots[0], 3)
    r0 = 8.0 / math.pi                                  # centreline arc length 4
    patches_xyz = []
    for iz in range(4):
        for iy in range(4):
            for ix in range(4):
                g = _grid_points(gr, gr, gr)
                x = ix + g[..., 0]
                y = 0.25 * (iy + g[..., 1])
                z = 0.25 * (iz + g[..., 2])
                th = (math.pi / 2.0) * x / 4.0
                r = r0 - (y - 0.5)
                xyz = np.stack([r * np.sin(th), r0 - r * np.cos(th), z], axis=-1)
                patches_xyz.append(xyz)
    pts = np.concatenate([q.reshape(-1, 3) for q in patches_xyz])
    bbox = np.stack([pts.min(0), pts.max(0)])
    f = _gaussian_field(rng_for(3, ROLE_FIELD), bbox)
    patches = [_make_patch(p, n, knots, xyz, f(xyz)) for xyz in patches_xyz]
    tf = random_tf(rng_for(3, ROLE_TF), extinction_for(bbox), scalar_domain(patches))
    cams = _seeded_cameras(3, bbox, 3, width, height, pts)
    return Scene("config3_bent_beam_64", patches, tf, cams, bbox,
                 dict(precision="fp32", rk_tol=1e-5))


# ---------------------------------------------------------------- config 4

def _config4(width=1920, height=1080) -> Scene:
    """Backward-facing step channel: inlet [-2,0]x[.5,1]x[0,1] as 4x2x4 boxes and
    main channel [0,7]x[0,1]^2 as 14x4x4 boxes, 256 cubic NURBS patches with 8^3
    control points at affine Greville positions, weights U[0.8,1.2]; control points
    that coincide across patches share one weight (watertight).  Field: four tanh
    fronts of width 0.01-0.05, quasi-interpolated."""
    p, n = (3, 3, 3), (8, 8, 8)
    knots = [open_uniform_knots(8, 3)] * 3
    gr = greville(knots[0], 3)
    boxes = []
    for iz in range(4):
        for iy in range(2):
            for ix in range(4):
                boxes.append((-2.0 + 0.5 * ix, 0.5 + 0.25 * iy, 0.25 * iz))
    for iz in range(4):
        for iy in range(4):
            for ix in range(14):
                boxes.append((0.5 * ix, 0.25 * iy, 0.25 * iz))
    rw = rng_for(4, ROLE_GEOM)
    weight_at = {}
    xyzs, ws = [], []
    for (x0, y0, z0) in boxes:
        g = _grid_points(gr, gr, gr)
        xyz = np.stack([x0 + 0.5 * g[..., 0], y0 + 0.25 * g[..., 1],
                        z0 + 0.25 * g[..., 2]], axis=-1)
        w = np.empty(xyz.shape[:3])
        for idx in np.ndindex(*w.shape):
            key = tuple(np.round(xyz[idx] * 1e9).astype(np.int64))
            if key not in weight_at:
                weight_at[key] = rw.uniform(0.8, 1.2)
            w[idx] = weight_at[key]
        xyzs.append(xyz)
        ws.append(w)
    pts = np.concatenate([q.reshape(-1, 3) for q in xyzs])
    bbox = np.stack([pts.min(0), pts.max(0)])
    rf = rng_for(4, ROLE_FIELD)
    ext = float((bbox[1] - bbox[0]).max())
    xh_all = (pts - bbox[0]) / ext
    fronts = []
    for _ in range(4):
        nv = rf.normal(size=3)
        nv /= np.linalg.norm(nv)
        proj = xh_all @ nv
        o = rf.uniform(proj.min(), proj.max())
        wd = rf.uniform(0.01, 0.05)
        fronts.append((nv, o, wd))

    def f(x):
        xh = (x - bbox[0]) / ext
        r = np.zeros(x.shape[:-1])
        for nv, o, wd in fronts:
            r = r + 0.5 * (1.0 + np.tanh((xh @ nv - o) / wd))
        return r
    patches = [_make_patch(p, n, knots, xyz, f(xyz), w=w, rational=True)
               for xyz, w in zip(xyzs, ws)]
    tf = random_tf(rng_for(4, ROLE_TF), extinction_for(bbox), scalar_domain(patches))
    cams = _seeded_cameras(4, bbox, 3, width, height, pts)
    return Scene("config4_step_channel_nurbs_256", patches, tf, cams, bbox,
                 dict(precision="fp32", rk_tol=1e-5))


# ---------------------------------------------------------------- config 5 model B

def _config5_model_b() -> List[Patch]:
    """8^3 lattice of unit-cube patches over [0,8]^3: degree 2 (5^3 control points)
    where i+j+k is even, else degree 3 (6^3).  Boundary-layer control points at affine
    Greville positions (faces match exactly by linear precision), interior control
    points jittered by U[-0.05,0.05]^3."""
    rg = rng_for(5, ROLE_GEOM)
    out = []
    for k in range(8):
        for j in range(8):
            for i in range(8):
                deg = 2 if (i + j + k) % 2 == 0 else 3
                nc = 5 if deg == 2 else 6
                kn = open_uniform_knots(nc, deg)
                gr = greville(kn, deg)
                g = _grid_points(gr, gr, gr)
                xyz = g + np.array([i, j, k], dtype=np.float64)
                inner = (slice(1, nc - 1),) * 3
                xyz[inner] += rg.uniform(-0.05, 0.05, xyz[inner].shape)
                out.append(_make_patch((deg,) * 3, (nc,) * 3, [kn] * 3, xyz,
                                       np.zeros(nc ** 3)))
    return out


def _config5():
    """Batched views over two models: model A is config 4, model B the mixed-degree
    lattice with a Gaussian field; 32 views with resolutions drawn from a fixed set."""
    a = _config4()
    b_patches = _config5_model_b()
    bbox_b = bbox_of(b_patches)
    f = _gaussian_field(rng_for(5, ROLE_FIELD), bbox_b)
    for q in b_patches:
        q.scalar = f(q.cp[:, :3])
    tf_b = random_tf(rng_for(5, ROLE_TF), extinction_for(bbox_b), scalar_domain(b_patches))
    b = Scene("config5_model_b_lattice_512", b_patches, tf_b, [], bbox_b,
              dict(precision="fp32", rk_tol=1e-5))
    res = [(256, 256), (512, 512), (1024, 1024), (1920, 1080), (2048, 2048)]
    rng = rng_for(5, ROLE_CAM)
    views = []
    for v in range(32):
        model = a if v % 2 == 0 else b
        w, h = res[int(rng.integers(0, len(res)))]
        az = rng.uniform(0.0, 360.0)
        el = rng.uniform(-45.0, 45.0)
        target = 0.5 * (model.bbox[0] + model.bbox[1])
        pts = np.concatenate([q.cp[:, :3] for q in model.patches])
        cam = camera_from_angles(target, _fit_distance(pts, target, az, el, w, h), az, el, w, h)
        views.append((v % 2, cam))
    return a, b, views


def make_degenerate(constant_field: bool = False, width: int = 96, height: int = 96) -> Scene:
    """A block with a degenerate boundary (Sec. "Degeneracies and Points Outside
    Domain"): the unit cube as a degree-2 patch with 4^3 control points whose first
    two layers in u coincide, so d phi/du = 0 and det J = 0 on the whole face u = 0
    (x = 0), while the face itself is a regular unit square.  The geometry is still
    exactly the unit cube.  rho is uniform [0,1] coefficients (seed 6002) or, with
    constant_field, 0.5 everywhere.  Camera 0 looks at the face x = 0 from outside
    (rays enter through the degenerate face), camera 1 from the opposite side
    (rays leave through it)."""
    p, n = (2, 2, 2), (4, 4, 4)
    knots = [open_uniform_knots(4, 2)] * 3
    gr = greville(knots[0], 2)                        # [0,.25,.75,1]
    gu = gr.copy()
    gu[1] = gu[0]                                     # layers i = 0 and 1 coincide
    xyz = _grid_points(gu, gr, gr)
    if constant_field:
        scalar = np.full(64, 0.5)
    else:
        scalar = np.random.default_rng(np.random.PCG64(6002)).uniform(0.0, 1.0, 64)
    patch = _make_patch(p, n, knots, xyz, scalar)
    dom = [0.0, 1.0] if constant_field else scalar_domain([patch])
    tf = random_tf(np.random.default_rng(np.random.PCG64(6003)), 4.0, dom)
    cams = [camera_from_angles([0.5, 0.5, 0.5], 2.4, 180.0 + az, el, width, height)
            for az, el in ((25.0, 15.0),)]
    cams.append(camera_from_angles([0.5, 0.5, 0.5], 2.4, -20.0, -10.0, width, height))
    return Scene("degenerate_face_cube", [patch], tf, cams, bbox_of([patch]),
                 dict(precision="fp32", rk_tol=1e-5))


def make_edge_lattice(width: int = 65, height: int = 65) -> Scene:
    """Eight affine degree-2 blocks (4^3 control points each) tiling [0, 2]^3, rho
    sampled from one smooth function at every block's Greville points (C0 across
    the interfaces).  With odd image sizes the centre pixel's ray goes exactly
    at the camera target: camera 0 through the edge x = y = 1 that four blocks
    share, camera 1 through the corner (1, 1, 1) of all eight, camera 2 through
    the boundary edge x = 1, y = 0 of two blocks (leaving the model there)."""
    def field(x):
        return 0.5 + 0.25 * np.sin(1.3 * x[:, 0] + 0.4) * np.cos(0.9 * x[:, 1] - 0.2) + 0.1 * x[:, 2]
    patches = []
    for k in range(2):
        for j in range(2):
            for i in range(2):
                off = np.array([i, j, k], dtype=np.float64)
                patches.append(affine_patch(np.eye(3), off, scalar=lambda g, off=off: field(g + off)))
    tf = random_tf(np.random.default_rng(np.random.PCG64(6101)), 3.0, scalar_domain(patches))
    up = np.array([0.0, 0.0, 1.0])
    cams = [Camera(np.array([-1.5, 3.5, 0.73]), np.array([1.0, 1.0, 0.73]), up, 30.0, width, height),
            Camera(np.array([-0.6, 2.9, -0.35]), np.array([1.0, 1.0, 1.0]), up, 30.0, width, height),
            Camera(np.array([1.9, 2.2, 1.4]), np.array([1.0, 0.0, 0.6]), up, 30.0, width, height)]
    return Scene("edge_lattice_2x2x2", patches, tf, cams, bbox_of(patches),
                 dict(precision="fp32", rk_tol=1e-5))


def _insert_knot_homogeneous(t, H, p, u):
    """Boehm insertion of u into a rational curve given by homogeneous points H
    (rows (w x, w y, w)), via scipy's B-spline knot insertion per coordinate."""
    from scipy.interpolate import insert
    cols, tt = [], None
    for c in range(H.shape[1]):
        tt, cc, _ = insert(u, (t, np.concatenate([H[:, c], np.zeros(p + 1)]), p))
        cols.append(cc[:len(tt) - p - 1])
    return np.asarray(tt), np.stack(cols, axis=1)


def make_annulus(constant_field: bool = False, width: int = 48, height: int = 48,
                 r_in: float = 1.0, r_out: float = 2.0, height_z: float = 1.5) -> Scene:
    """Quarter annulus r_in <= r <= r_out, 0 <= theta <= pi/2, 0 <= z <= height_z as
    one quadratic NURBS block (degree 2 in every direction):
      u (arc): the unit quarter circle with weights (1, sqrt(2)/2, 1), then the knot
               0.35 inserted (homogeneous Boehm insertion): knots (0,0,0,.35,1,1,1);
      v (radial): radii (r_in, mid, r_out), knots (0,0,0,1,1,1) (linear);
      w (height): knots (0,0,0,.3,1,1,1), control points at the Greville points.
    Weights depend on u only, so the map is r(v) (cos theta(u), sin theta(u)), z(w):
    the faces v = 0, 1 are exactly the cylinders r = r_in, r_out, the faces u = 0, 1
    the half planes y = 0, x = 0, and w = 0, 1 the planes z = 0, height_z.
    Field: constant 0.5, or 0.5 + 0.3 sin(2x) cos(1.5y) + 0.2 z quasi-interpolated.
    Three views (seeds 6201..6203)."""
    p = 2
    arc = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    w0 = np.array([1.0, math.sqrt(0.5), 1.0])
    H0 = np.concatenate([arc * w0[:, None], w0[:, None]], axis=1)
    tu, Hu = _insert_knot_homogeneous(np.array([0, 0, 0, 1, 1, 1.0]), H0, p, 0.35)
    wu = Hu[:, 2]
    au = Hu[:, :2] / wu[:, None]
    tv = np.array([0, 0, 0, 1, 1, 1.0])
    radii = np.array([r_in, 0.5 * (r_in + r_out), r_out])
    tw = np.array([0, 0, 0, 0.3, 1, 1, 1.0])
    zs = height_z * greville(tw, p)
    nu, nv, nw = len(wu), len(radii), len(zs)
    xyz = np.empty((nw, nv, nu, 3))
    wt = np.empty((nw, nv, nu))
    for k in range(nw):
        for j in range(nv):
            for i in range(nu):
                xyz[k, j, i] = (radii[j] * au[i, 0], radii[j] * au[i, 1], zs[k])
                wt[k, j, i] = wu[i]
    if constant_field:
        sc = np.full((nw, nv, nu), 0.5)
    else:
        sc = 0.5 + 0.3 * np.sin(2.0 * xyz[..., 0]) * np.cos(1.5 * xyz[..., 1]) + 0.2 * xyz[..., 2]
    patch = _make_patch((p, p, p), (nu, nv, nw), [tu, tv, tw], xyz, sc, w=wt, rational=True)
    bbox = np.array([[0.0, 0.0, 0.0], [r_out, r_out, height_z]])
    rng = np.random.Generator(np.random.PCG64(6200))
    tf = random_tf(rng, extinction_for(bbox), (0.0, 1.0) if constant_field else scalar_domain([patch]))
    target = 0.5 * (bbox[0] + bbox[1])
    cams = []
    for s in range(3):
        r = np.random.Generator(np.random.PCG64(6201 + s))
        az, el = r.uniform(0.0, 360.0), r.uniform(-45.0, 45.0)
        cams.append(camera_from_angles(target, 3.2 * float(np.linalg.norm(bbox[1] - bbox[0])) / 2.0,
                                       az, el, width, height))
    return Scene("quarter_annulus_nurbs", [patch], tf, cams, bbox,
                 dict(r_in=r_in, r_out=r_out, height=height_z))


def make_mixed_degree(rational: bool = False, width: int = 64, height: int = 64) -> Scene:
    """One block whose directions have different degrees: (1, 2, 3) as a B-spline
    with 3 x 4 x 5 control points, or (2, 3, 3) as a NURBS with 4 x 5 x 6 control
    points, weights U[0.8, 1.2] and non-uniform knots along w.  Control points at
    the Greville points of the unit cube, bent and sheared smoothly
    (x + 0.15 sin(pi z), y + 0.1 z^2, z + 0.1 x y), interior points jittered by
    U[-0.03, 0.03]; scalar coefficients U[0, 1].  Two 64x64 views (seeds 6300+)."""
    seed = 6310 if rational else 6300
    rng = np.random.Generator(np.random.PCG64(seed))
    if rational:
        deg, ncp = (2, 3, 3), (4, 5, 6)
        knots = [open_uniform_knots(4, 2), open_uniform_knots(5, 3),
                 np.array([0, 0, 0, 0, 0.2, 0.55, 1, 1, 1, 1.0])]
    else:
        deg, ncp = (1, 2, 3), (3, 4, 5)
        knots = [open_uniform_knots(3, 1), open_uniform_knots(4, 2), open_uniform_knots(5, 3)]
    g = _grid_points(*(greville(knots[d], deg[d]) for d in range(3)))
    x, y, z = g[..., 0], g[..., 1], g[..., 2]
    xyz = np.stack([x + 0.15 * np.sin(math.pi * z), y + 0.1 * z * z, z + 0.1 * x * y], axis=-1)
    n0, n1, n2 = ncp
    inner = np.zeros((n2, n1, n0), bool)
    inner[1:-1, 1:-1, 1:-1] = True
    xyz[inner] += rng.uniform(-0.03, 0.03, (int(inner.sum()), 3))
    w = rng.uniform(0.8, 1.2, (n2, n1, n0)) if rational else None
    sc = rng.uniform(0.0, 1.0, (n2, n1, n0))
    patch = _make_patch(deg, ncp, knots, xyz, sc, w=w, rational=rational)
    bbox = bbox_of([patch])
    tf = random_tf(rng, extinction_for(bbox), scalar_domain([patch]))
    target = 0.5 * (bbox[0] + bbox[1])
    cams = [camera_from_angles(target, 2.2, az, el, width, height) for az, el in ((35.0, 25.0), (200.0, -30.0))]
    return Scene("mixed_degree_nurbs" if rational else "mixed_degree_bspline", [patch], tf, cams, bbox)


def make_config(k: int, width: Optional[int] = None, height: Optional[int] = None):
    """Build config k (1..4) as a Scene; config 5 returns (model_a, model_b, views)."""
    if k == 1:
        return _config1()
    if k == 2:
        return _config2()
    if k == 3:
        return _config3(width or 1920, height or 1080)
    if k == 4:
        return _config4(width or 1920, height or 1080)
    if k == 5:
        return _config5()
    raise ValueError(f"unknown config {k}")


# ---------------------------------------------------------------- displacement fields

def with_displacement(scene: Scene, B: Optional[np.ndarray] = None, amplitude: float = 0.0,
                      seed: int = 7300) -> Scene:
    """The scene with a displacement spline u on every block, on the block's own
    basis, with coefficient u_i = f(x_i) at each control point x_i (quasi-
    interpolation): f(g) = B g for a 3x3 matrix B (then u = B phi exactly, also
    for NURBS blocks), plus, with amplitude > 0, a smooth seeded field
    amplitude * (sin(a.g), cos(b.g), sin(c.g + 0.3)) with random wave vectors.
    The transfer function and cameras are the scene's."""
    rng = np.random.Generator(np.random.PCG64(seed))
    waves = rng.normal(0.0, 1.0, (3, 3)) / max(float(np.linalg.norm(scene.bbox[1] - scene.bbox[0])), 1e-9) * 4.0
    out = []
    for P in scene.patches:
        x = P.cp[:, :3]
        u = np.zeros_like(x)
        if B is not None:
            u += x @ np.asarray(B, dtype=np.float64).T
        if amplitude > 0.0:
            u += amplitude * np.stack([np.sin(x @ waves[0]), np.cos(x @ waves[1]), np.sin(x @ waves[2] + 0.3)], -1)
        out.append(Patch(P.degree, P.ncp, P.knots, P.cp, P.scalar, P.rational, u))
    return Scene(scene.name + "_displaced", out, scene.tf, scene.cameras, scene.bbox, dict(scene.params))

"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain C, see ``ivr_oracle.c``)
with ctypes and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "ivr_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64, -O3, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", "-o", tmp, SRC_PATH,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Patch(C.Structure):
    _fields_ = [("deg", C.c_int32 * 3), ("ncp", C.c_int32 * 3),
                ("knots", C.POINTER(C.c_double) * 3), ("cp", C.POINTER(C.c_double)),
                ("scalar", C.POINTER(C.c_double)), ("rational", C.c_int32), ("disp", C.POINTER(C.c_double))]


# fields sampled along the ray (orc_opts.field)
FIELDS = {"scalar": 0, "param_quality": 1, "von_mises": 2}


class _TF(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.POINTER(C.c_double)), ("rgba", C.POINTER(C.c_double)),
                ("extinction", C.c_double), ("domain", C.c_double * 2)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("panels_per_scale", C.c_double), ("richardson", C.c_int32),
                ("nthreads", C.c_int32), ("self_tol", C.c_double), ("cut", C.c_int32),
                ("cut_point", C.c_double * 3), ("cut_normal", C.c_double * 3), ("near_clip", C.c_double),
                ("field", C.c_int32)]


class _MethodOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("h_max", C.c_double), ("c_perp", C.c_double), ("rho_step", C.c_double),
                ("tf_step", C.c_double), ("n_super", C.c_int32), ("hermite", C.c_int32), ("nthreads", C.c_int32),
                ("method", C.c_int32)]


# interior methods of the method mode (orc_method_opts.method)
METHODS = {"rkf45": 0, "rk1": 1, "rk2": 2, "rk3": 3, "rk4": 4, "rk4_38": 5, "rkf5": 6, "irk1": 7, "rf": 8}


class Fragment(C.Structure):
    _fields_ = [("t", C.c_double), ("p", C.c_double * 3), ("patch", C.c_int32),
                ("face", C.c_int32), ("entering", C.c_int32), ("pad", C.c_int32)]


class _Diag(C.Structure):
    _fields_ = [("n_fragments", C.c_int32), ("n_segments", C.c_int32),
                ("n_anomalies", C.c_int32), ("n_newton_fail", C.c_int32),
                ("self_error", C.c_double), ("first_chord", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_prepare.restype = C.c_void_p
        L.orc_prepare.argtypes = [C.POINTER(_Patch), C.c_int32, C.c_double]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_basis.argtypes = [dp, C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_basis.restype = C.c_int32
        L.orc_eval.argtypes = [C.POINTER(_Patch), dp, dp, dp, dp]
        L.orc_eval.restype = C.c_int32
        L.orc_invert.argtypes = [C.POINTER(_Patch), dp, dp, C.c_double, dp, C.POINTER(C.c_int32)]
        L.orc_invert.restype = C.c_int32
        L.orc_camera_ray.argtypes = [C.POINTER(_Camera), C.c_double, C.c_double, dp, dp]
        L.orc_transfer.argtypes = [C.POINTER(_TF), C.c_double, dp]
        L.orc_ray_fragments.argtypes = [C.c_void_p, dp, dp, C.POINTER(Fragment), C.c_int32]
        L.orc_ray_fragments.restype = C.c_int32
        L.orc_render_pixels.argtypes = [C.c_void_p, C.POINTER(_Camera), C.POINTER(_TF),
                                        C.POINTER(_Opts), C.POINTER(C.c_int64), C.c_int64, dp, dp,
                                        C.POINTER(_Diag)]
        L.orc_render_pixels.restype = C.c_int32
        L.orc_locate.argtypes = [C.c_void_p, dp, C.c_int64, C.POINTER(C.c_int32), dp, dp]
        L.orc_locate.restype = C.c_int32
        L.orc_render_pixels_method.argtypes = [C.c_void_p, C.POINTER(_Camera), C.POINTER(_TF),
                                               C.POINTER(_MethodOpts), C.POINTER(C.c_int64), C.c_int64, dp,
                                               C.POINTER(C.c_int64), dp, C.POINTER(C.c_int32)]
        L.orc_delta_p.argtypes = [C.POINTER(_Camera), C.c_int64, dp]
        L.orc_delta_p.restype = C.c_double
        L.orc_render_pixels_method.restype = C.c_int32
        L.orc_table1.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_table1.restype = C.c_double
        L.orc_table1_newton.argtypes = [C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_int32)]
        L.orc_table1_newton.restype = C.c_double
        L.orc_path_error.argtypes = [C.POINTER(_Patch), dp, dp, C.c_int32, C.c_double, C.c_double,
                                     C.POINTER(C.c_int32)]
        L.orc_path_error.restype = C.c_double
        L.orc_field.argtypes = [C.POINTER(_Patch), dp, C.c_int32, dp]
        L.orc_field.restype = C.c_int32
        L.orc_eval_hessian.argtypes = [C.POINTER(_Patch), dp, dp, dp, dp]
        L.orc_eval_hessian.restype = C.c_int32
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OraclePatch:
    """ctypes view of one scenes.Patch (keeps the numpy buffers alive)."""

    def __init__(self, patch):
        self._keep = [np.ascontiguousarray(k, dtype=np.float64) for k in patch.knots]
        self._cp = np.ascontiguousarray(patch.cp, dtype=np.float64)
        self._sc = np.ascontiguousarray(patch.scalar, dtype=np.float64)
        s = _Patch()
        for d in range(3):
            s.deg[d] = int(patch.degree[d])
            s.ncp[d] = int(patch.ncp[d])
            s.knots[d] = _dp(self._keep[d])
        s.cp = _dp(self._cp)
        s.scalar = _dp(self._sc)
        s.rational = 1 if patch.rational else 0
        disp = getattr(patch, "displacement", None)
        if disp is not None:
            self._disp = np.ascontiguousarray(disp, dtype=np.float64).reshape(-1)
            s.disp = _dp(self._disp)
        self.struct = s


def _camera(cam) -> _Camera:
    c = _Camera()
    for q in range(3):
        c.eye[q] = float(cam.eye[q])
        c.target[q] = float(cam.target[q])
        c.up[q] = float(cam.up[q])
    c.fov_y_deg = float(cam.fov_y_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


class OracleTF:
    def __init__(self, tf):
        self._x = np.ascontiguousarray(tf.x, dtype=np.float64)
        self._rgba = np.ascontiguousarray(tf.rgba, dtype=np.float64).reshape(-1)
        t = _TF()
        t.n = len(self._x)
        t.x = _dp(self._x)
        t.rgba = _dp(self._rgba)
        t.extinction = float(tf.extinction)
        t.domain[0] = float(tf.domain[0])
        t.domain[1] = float(tf.domain[1])
        self.struct = t


class OracleScene:
    """Prepared scene: patches plus their Bezier-extracted boundary faces."""

    def __init__(self, patches: Sequence, scale: float):
        self.patches = [OraclePatch(p) for p in patches]
        arr = (_Patch * len(self.patches))(*[p.struct for p in self.patches])
        self._arr = arr
        self.scale = float(scale)
        self.handle = lib().orc_prepare(arr, len(self.patches), self.scale)

    def __del__(self):
        try:
            if self.handle:
                lib().orc_free(self.handle)
        except Exception:
            pass

    def locate(self, g, hint_block=None, hint_p=None, chain=False):
        """Brute-force point location (Newton inversion from a hint and nine seeds):
        per point the block that holds it (-1: none), its parameters and rho.
        chain: each point after the first is seeded with its predecessor's result."""
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1, 3))
        n = len(g)
        blk = np.full(n, -1, dtype=np.int32) if hint_block is None else \
            np.ascontiguousarray(np.broadcast_to(hint_block, (n,)), dtype=np.int32).copy()
        p = np.full((n, 3), 0.5) if hint_p is None else \
            np.ascontiguousarray(np.broadcast_to(hint_p, (n, 3)), dtype=np.float64).copy()
        if chain and n > 1:
            blk[1:] = -2
        rho = np.zeros(n)
        lib().orc_locate(self.handle, _dp(g), n, blk.ctypes.data_as(C.POINTER(C.c_int32)), _dp(p), _dp(rho))
        return blk, p, rho

    def fragments(self, o, d, cap=1024):
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        buf = (Fragment * cap)()
        n = lib().orc_ray_fragments(self.handle, _dp(o), _dp(d), buf, cap)
        if n < 0:
            raise RuntimeError(f"orc_ray_fragments failed ({n})")
        return [(buf[i].t, np.array(buf[i].p[:]), buf[i].patch, buf[i].face, bool(buf[i].entering))
                for i in range(n)]


def basis(t, p, u):
    t = np.ascontiguousarray(t, dtype=np.float64)
    n = len(t) - p - 1
    N = np.zeros(n)
    dN = np.zeros(n)
    lib().orc_basis(_dp(t), len(t), p, float(u), _dp(N), _dp(dN))
    return N, dN


def evaluate(patch, p):
    """phi(p), J(p) (3x3, J[r, c] = d phi_r / d p_c) and rho(p)."""
    op = patch if isinstance(patch, OraclePatch) else OraclePatch(patch)
    p = np.ascontiguousarray(p, dtype=np.float64)
    x = np.zeros(3)
    J = np.zeros(9)
    rho = np.zeros(1)
    lib().orc_eval(C.byref(op.struct), _dp(p), _dp(x), _dp(J), _dp(rho))
    return x, J.reshape(3, 3), float(rho[0])


def invert(patch, g, seed=(0.5, 0.5, 0.5), scale=1.0):
    op = patch if isinstance(patch, OraclePatch) else OraclePatch(patch)
    g = np.ascontiguousarray(g, dtype=np.float64)
    s = np.ascontiguousarray(seed, dtype=np.float64)
    out = np.zeros(3)
    it = C.c_int32(0)
    rc = lib().orc_invert(C.byref(op.struct), _dp(g), _dp(s), float(scale), _dp(out), C.byref(it))
    return rc, out, it.value


def camera_ray(cam, px, py):
    c = _camera(cam)
    o = np.zeros(3)
    d = np.zeros(3)
    lib().orc_camera_ray(C.byref(c), float(px), float(py), _dp(o), _dp(d))
    return o, d


def transfer(tf, rho):
    t = OracleTF(tf)
    out = np.zeros(4)
    lib().orc_transfer(C.byref(t.struct), float(rho), _dp(out))
    return out


def table1(method: int, ds: float, c: float = 1.0) -> float:
    """Error of the convergence study (methods 1..6 explicit RK, 7 implicit Euler)."""
    return float(lib().orc_table1(int(method), float(ds), float(c)))


def table1_newton(method: int, ds: float, c: float = 1.0):
    """(error, most Newton iterations of an implicit Euler step; -1: one failed)."""
    it = C.c_int32(0)
    e = float(lib().orc_table1_newton(int(method), float(ds), float(c), C.byref(it)))
    return e, it.value


def path_error(patch, p_in, p_out, method: int, ds: float, c: float = 1.0):
    """Convergence study on a block: (largest distance of phi(p_i) from the ray
    phi(p_in) -> phi(p_out) after uniform steps ds of method 1..7, most Newton
    iterations of an implicit Euler step)."""
    op = patch if isinstance(patch, OraclePatch) else OraclePatch(patch)
    a = np.ascontiguousarray(p_in, dtype=np.float64)
    b = np.ascontiguousarray(p_out, dtype=np.float64)
    it = C.c_int32(0)
    e = float(lib().orc_path_error(C.byref(op.struct), _dp(a), _dp(b), int(method), float(ds), float(c),
                                   C.byref(it)))
    return e, it.value


def field_value(patch, p, field: str) -> float:
    """The value of a field of FIELDS at parameter point p of the block."""
    op = patch if isinstance(patch, OraclePatch) else OraclePatch(patch)
    p = np.ascontiguousarray(p, dtype=np.float64)
    v = np.zeros(1)
    if lib().orc_field(C.byref(op.struct), _dp(p), FIELDS[field], _dp(v)) != 0:
        raise ValueError(f"orc_field failed ({field})")
    return float(v[0])


def evaluate_hessian(patch, p):
    """phi(p), J(p) and H (3x3x3, H[r, a, b] = d^2 phi_r / dp_a dp_b)."""
    op = patch if isinstance(patch, OraclePatch) else OraclePatch(patch)
    p = np.ascontiguousarray(p, dtype=np.float64)
    x, J, H = np.zeros(3), np.zeros(9), np.zeros(27)
    rc = lib().orc_eval_hessian(C.byref(op.struct), _dp(p), _dp(x), _dp(J), _dp(H))
    if rc != 0:
        raise ValueError("orc_eval_hessian failed")
    return x, J.reshape(3, 3), H.reshape(3, 3, 3)


class RenderResult:
    def __init__(self, rgba, depth, diag):
        self.rgba = rgba
        self.depth = depth
        self.n_fragments = np.array([d.n_fragments for d in diag])
        self.n_segments = np.array([d.n_segments for d in diag])
        self.n_anomalies = np.array([d.n_anomalies for d in diag])
        self.n_newton_fail = np.array([d.n_newton_fail for d in diag])
        self.self_error = np.array([d.self_error for d in diag])
        self.first_chord = np.array([d.first_chord for d in diag])


def render(scene_or_patches, cam, tf, pixels: Optional[np.ndarray] = None,
           panels_per_scale: float = 2048.0, richardson: bool = True, nthreads: int = 0,
           scale: Optional[float] = None, prepared: Optional[OracleScene] = None,
           self_tol: float = 1e-5, cut_plane=None, near_clip: float = 0.0, field: str = "scalar") -> RenderResult:
    """Reference image (premultiplied RGBA, first-entry depth) for the listed pixels
    (linear index row*width+col), or for the whole image when pixels is None.
    cut_plane: (point, normal), keeping normal . (g - point) >= 0; near_clip: the
    near plane's distance from the eye along the view direction (0: none);
    field: the value sampled along the ray (FIELDS)."""
    if prepared is None:
        patches = getattr(scene_or_patches, "patches", scene_or_patches)
        if scale is None:
            scale = scene_or_patches.scale
        prepared = OracleScene(patches, scale)
    cam_s = _camera(cam)
    tf_s = OracleTF(tf)
    opts = _Opts(float(panels_per_scale), 1 if richardson else 0, int(nthreads), float(self_tol))
    if cut_plane is not None:
        opts.cut = 1
        for q in range(3):
            opts.cut_point[q] = float(cut_plane[0][q])
            opts.cut_normal[q] = float(cut_plane[1][q])
    opts.near_clip = float(near_clip)
    opts.field = FIELDS[field]
    if pixels is None:
        npix = cam.width * cam.height
        pix_ptr = None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = len(pixels)
        pix_ptr = pixels.ctypes.data_as(C.POINTER(C.c_int64))
    rgba = np.zeros((npix, 4))
    depth = np.zeros(npix)
    diag = (_Diag * max(npix, 1))()
    rc = lib().orc_render_pixels(prepared.handle, C.byref(cam_s), C.byref(tf_s.struct),
                                 C.byref(opts), pix_ptr, npix, _dp(rgba), _dp(depth), diag)
    if rc != 0:
        raise RuntimeError(f"orc_render_pixels failed ({rc})")
    return RenderResult(rgba, depth, [diag[i] for i in range(npix)])


def render_method(scene_or_patches, cam, tf, pixels: Optional[np.ndarray] = None, rk_tol: float = 1e-5,
                  h_max: float = 0.0, c_perp: float = 1.0, rho_step: float = 0.1, tf_step: float = 0.025,
                  n_super: int = 4, hermite: bool = True, nthreads: int = 0, scale: Optional[float] = None,
                  prepared: Optional[OracleScene] = None, method: str = "rkf45", pixel_accuracy: bool = False):
    """Method mode: the GPU path's method (adaptive RKF45 on the ray preimage ODE,
    or a fixed-step method of METHODS; Hermite or linear rho, supersampling) in
    FP64.  Returns (rgba, steps), and with pixel_accuracy a third item: per pixel
    the largest Delta P of the interior samples and the depth-order violations."""
    if prepared is None:
        patches = getattr(scene_or_patches, "patches", scene_or_patches)
        if scale is None:
            scale = scene_or_patches.scale
        prepared = OracleScene(patches, scale)
    mo = _MethodOpts(float(rk_tol), float(h_max), float(c_perp), float(rho_step), float(tf_step),
                     int(n_super), 1 if hermite else 0, int(nthreads), METHODS[method])
    tf_s = OracleTF(tf)
    if pixels is None:
        npix, pix_ptr = cam.width * cam.height, None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        npix, pix_ptr = len(pixels), pixels.ctypes.data_as(C.POINTER(C.c_int64))
    rgba = np.zeros((npix, 4))
    steps = C.c_int64(0)
    dpv = np.zeros(npix) if pixel_accuracy else None
    bad = np.zeros(npix, dtype=np.int32) if pixel_accuracy else None
    rc = lib().orc_render_pixels_method(prepared.handle, C.byref(_camera(cam)), C.byref(tf_s.struct), C.byref(mo),
                                        pix_ptr, npix, _dp(rgba), C.byref(steps),
                                        _dp(dpv) if pixel_accuracy else None,
                                        bad.ctypes.data_as(C.POINTER(C.c_int32)) if pixel_accuracy else None)
    if rc != 0:
        raise RuntimeError(f"orc_render_pixels_method failed ({rc})")
    if pixel_accuracy:
        return rgba, steps.value, {"delta_p": dpv, "order_violations": bad}
    return rgba, steps.value


def delta_p(cam, pixel: int, g) -> float:
    """Eq. (deltaP) for point g and pixel (row*width + col)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    return float(lib().orc_delta_p(C.byref(_camera(cam)), int(pixel), _dp(g)))

"""ctypes binding of the C ABI in include/ivr.h.

Argument marshalling only: every step of the render runs in the gfx950 kernels of
``libivr.so``.  PyTorch provides device memory and the stream.  There is no CPU
fallback: if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libivr.so")

IVR_OK, IVR_EINVAL, IVR_ENOMEM, IVR_EDEVICE, IVR_ESTATE, IVR_EOVERFLOW = 0, -1, -2, -3, -4, -5
FLAGS = {"anomaly": 1, "fragment_overflow": 2, "segment_overflow": 4, "iter_cap": 8,
         "drift_restart": 16, "restart_fail": 32, "degenerate": 64, "depth_order": 128}
PRECISION = {"fp32": 0, "fp64": 1}
SEED = {"plain": 0, "mlp": 1, "box": 2}
RHO_INTERP = {"linear": 0, "hermite": 1}
FIELDS = {"scalar": 0, "param_quality": 1, "von_mises": 2}
NEWTON_STOP = {"tol": 0, "frustum": 1}
INTERIOR = {"ode": 0, "rf": 1, "rk1": 2, "rk2": 3, "rk3": 4, "rk4": 5, "rk4_38": 6, "rkf5": 7, "irk1": 8}

EXPORTS = ["ivr_create", "ivr_default_opts", "ivr_upload_patches", "ivr_upload_models",
           "ivr_render", "ivr_render_noalloc", "ivr_render_batch", "ivr_autotune", "ivr_set_launch",
           "ivr_phase_times", "ivr_last_error", "ivr_destroy", "ivr_default_mlp_opts",
           "ivr_train_inverse_mlp", "ivr_mlp_forward_backward", "ivr_mlp_get_weights",
           "ivr_mlp_infer", "ivr_device_bytes", "ivr_delta_e2000"]
MLP_PARAMS = 4611


class PatchDesc(C.Structure):
    _fields_ = [("degree", C.c_int32 * 3), ("ncp", C.c_int32 * 3),
                ("knots", C.POINTER(C.c_double) * 3), ("cp", C.POINTER(C.c_double)),
                ("scalar", C.POINTER(C.c_double)), ("rational", C.c_int32),
                ("displacement", C.POINTER(C.c_double))]


class CameraDesc(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class TransferDesc(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("x", C.POINTER(C.c_double)),
                ("rgba", C.POINTER(C.c_double)), ("extinction", C.c_double),
                ("domain", C.c_double * 2)]


class RenderOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rk_tol", C.c_double), ("h_max", C.c_double),
                ("c_perp", C.c_double), ("n_super", C.c_int32),
                ("det_fp64_threshold", C.c_double), ("max_fragments", C.c_int32),
                ("seed_mode", C.c_int32), ("early_term", C.c_double),
                ("max_newton_iter", C.c_int32), ("rho_interp", C.c_int32),
                ("timing", C.c_int32), ("tf_step", C.c_double), ("rho_step", C.c_double),
                ("cand_per_pixel", C.c_int32), ("det_singular", C.c_double),
                ("drift_tol", C.c_double), ("interior", C.c_int32), ("cut", C.c_int32),
                ("cut_point", C.c_double * 3), ("cut_normal", C.c_double * 3), ("near_clip", C.c_double),
                ("newton_stop", C.c_int32), ("field", C.c_int32)]


class ViewDesc(C.Structure):
    _fields_ = [("cam", CameraDesc), ("tf", C.c_void_p), ("model", C.c_int32),
                ("rgba_dev", C.c_void_p), ("depth_dev", C.c_void_p), ("flags_dev", C.c_void_p),
                ("dp_dev", C.c_void_p)]


class TuneReport(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("xcd_chunk", C.c_int32),
                ("int_block", C.c_int32), ("int_waves_cu", C.c_int32), ("n_tried", C.c_int32),
                ("tried_ms", C.c_double * 32), ("ms_before", C.c_double), ("ms_after", C.c_double)]


STAT_FIELDS = ["rays", "segments", "fragments", "anomalies", "fragment_overflow",
               "segment_overflow", "box_tests", "face_newton", "face_newton_iter",
               "fp64_polish_iter", "rk_steps", "rk_rejected", "samples", "w_evals",
               "fp64_solves", "rk_iter_cap", "mlp_queries", "subsamples", "degenerate",
               "mlp_restarts", "drift_restarts", "restart_fail", "dp_over", "order_violations"]


class MlpOpts(C.Structure):
    _fields_ = [("samples_per_patch", C.c_int32), ("steps", C.c_int32), ("lr", C.c_double),
                ("seed", C.c_uint32), ("log_every", C.c_int32), ("batch", C.c_int32)]


class MlpReport(C.Structure):
    _fields_ = [("n_loss", C.c_int32), ("loss", C.c_float * 64), ("heldout_mean_err", C.c_double),
                ("heldout_max_err", C.c_double), ("ms_samples", C.c_double),
                ("ms_train", C.c_double)]


class DeltaESummary(C.Structure):
    _fields_ = [("max", C.c_double), ("mean", C.c_double), ("over", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in STAT_FIELDS] + [
        ("ms_fragments", C.c_double), ("ms_integrate", C.c_double), ("ms_merge", C.c_double)]


_lib = None


def load_library() -> C.CDLL:
    """Load libivr.so (built by __graft_entry__.build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ivr_create.argtypes = [C.POINTER(vp), C.c_int32, vp]
    L.ivr_create.restype = C.c_int32
    L.ivr_default_opts.argtypes = [C.POINTER(RenderOpts)]
    L.ivr_default_opts.restype = None
    L.ivr_upload_patches.argtypes = [vp, C.POINTER(PatchDesc), C.c_int32]
    L.ivr_upload_patches.restype = C.c_int32
    L.ivr_upload_models.argtypes = [vp, C.POINTER(PatchDesc), C.c_int32, C.POINTER(C.c_int32),
                                    C.c_int32]
    L.ivr_upload_models.restype = C.c_int32
    L.ivr_render_batch.argtypes = [vp, C.POINTER(ViewDesc), C.c_int32, C.POINTER(TransferDesc),
                                   C.POINTER(RenderOpts), C.POINTER(Stats)]
    L.ivr_render_batch.restype = C.c_int32
    L.ivr_autotune.argtypes = [vp, C.POINTER(ViewDesc), C.c_int32, C.POINTER(TransferDesc),
                               C.POINTER(RenderOpts), C.POINTER(TuneReport)]
    L.ivr_autotune.restype = C.c_int32
    L.ivr_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.ivr_set_launch.restype = C.c_int32
    L.ivr_render.argtypes = [vp, C.POINTER(CameraDesc), C.POINTER(TransferDesc),
                             C.POINTER(RenderOpts), vp, vp, C.POINTER(Stats)]
    L.ivr_render.restype = C.c_int32
    L.ivr_render_noalloc.argtypes = L.ivr_render.argtypes
    L.ivr_render_noalloc.restype = C.c_int32
    fp = C.POINTER(C.c_float)
    L.ivr_default_mlp_opts.argtypes = [C.POINTER(MlpOpts)]
    L.ivr_default_mlp_opts.restype = None
    L.ivr_train_inverse_mlp.argtypes = [vp, C.POINTER(MlpOpts), C.POINTER(MlpReport)]
    L.ivr_train_inverse_mlp.restype = C.c_int32
    L.ivr_mlp_forward_backward.argtypes = [vp, fp, fp, fp, C.c_int32, fp, fp]
    L.ivr_mlp_forward_backward.restype = C.c_int32
    L.ivr_mlp_get_weights.argtypes = [vp, C.c_int32, fp]
    L.ivr_mlp_get_weights.restype = C.c_int32
    L.ivr_mlp_infer.argtypes = [vp, C.POINTER(C.c_int32), fp, C.c_int32, fp]
    L.ivr_mlp_infer.restype = C.c_int32
    L.ivr_phase_times.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]
    L.ivr_phase_times.restype = C.c_int32
    L.ivr_device_bytes.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.ivr_device_bytes.restype = C.c_int32
    L.ivr_delta_e2000.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_double), C.c_double, vp,
                                  C.POINTER(DeltaESummary)]
    L.ivr_delta_e2000.restype = C.c_int32
    L.ivr_last_error.argtypes = [vp]
    L.ivr_last_error.restype = C.c_char_p
    L.ivr_destroy.argtypes = [vp]
    L.ivr_destroy.restype = None
    _lib = L
    return L


class IvrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ivr error {code}: {msg}")
        self.code = code


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_opts(**kw) -> RenderOpts:
    o = RenderOpts()
    load_library().ivr_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "seed_mode" and isinstance(v, str):
            v = SEED[v]
        if k == "rho_interp" and isinstance(v, str):
            v = RHO_INTERP[v]
        if k == "interior" and isinstance(v, str):
            v = INTERIOR[v]
        if k == "field" and isinstance(v, str):
            v = FIELDS[v]
        if k == "newton_stop" and isinstance(v, str):
            v = NEWTON_STOP[v]
        if k == "cut_plane":   # (point, normal) or None
            o.cut = 0 if v is None else 1
            if v is not None:
                for q in range(3):
                    o.cut_point[q] = float(v[0][q])
                    o.cut_normal[q] = float(v[1][q])
            continue
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def camera_desc(cam) -> CameraDesc:
    c = CameraDesc()
    for q in range(3):
        c.eye[q] = float(cam.eye[q])
        c.target[q] = float(cam.target[q])
        c.up[q] = float(cam.up[q])
    c.fov_y_deg = float(cam.fov_y_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


class _TF:
    def __init__(self, tf):
        self.x = np.ascontiguousarray(tf.x, dtype=np.float64)
        self.rgba = np.ascontiguousarray(np.asarray(tf.rgba, dtype=np.float64).reshape(-1))
        d = TransferDesc()
        d.n_knots = len(self.x)
        d.x = _dp(self.x)
        d.rgba = _dp(self.rgba)
        d.extinction = float(tf.extinction)
        d.domain[0] = float(tf.domain[0])
        d.domain[1] = float(tf.domain[1])
        self.desc = d


class Renderer:
    """One ivr context on a GPU.  Uses torch for output buffers and the stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ivr needs a GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = int(device)
        self.lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        handle = C.c_void_p(int(stream.cuda_stream))
        ctx = C.c_void_p()
        rc = self.lib.ivr_create(C.byref(ctx), self.device, handle)
        if rc != IVR_OK:
            raise IvrError(rc, "ivr_create failed (device missing or not gfx950)")
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ivr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != IVR_OK:
            raise IvrError(rc, self.lib.ivr_last_error(self.ctx).decode())

    def upload(self, patches: Sequence) -> None:
        self.upload_models([patches])

    def upload_models(self, models: Sequence[Sequence]) -> None:
        """Several models in one context; views name them by index."""
        patches = [p for m in models for p in m]
        sizes = (C.c_int32 * len(models))(*[len(m) for m in models])
        keep = []
        arr = (PatchDesc * len(patches))()
        for i, p in enumerate(patches):
            kn = [np.ascontiguousarray(k, dtype=np.float64) for k in p.knots]
            cp = np.ascontiguousarray(p.cp, dtype=np.float64)
            sc = np.ascontiguousarray(p.scalar, dtype=np.float64)
            keep += kn + [cp, sc]
            d = arr[i]
            for q in range(3):
                d.degree[q] = int(p.degree[q])
                d.ncp[q] = int(p.ncp[q])
                d.knots[q] = _dp(kn[q])
            d.cp = _dp(cp)
            d.scalar = _dp(sc)
            d.rational = 1 if p.rational else 0
            disp = getattr(p, "displacement", None)
            if disp is not None:
                u = np.ascontiguousarray(disp, dtype=np.float64).reshape(-1)
                assert u.size == 3 * len(sc), "displacement: 3 values per control point"
                keep.append(u)
                d.displacement = _dp(u)
        self._check(self.lib.ivr_upload_models(self.ctx, arr, len(patches), sizes, len(models)))

    # ---- learned initialiser
    def train_mlp(self, **kw) -> dict:
        o = MlpOpts()
        self.lib.ivr_default_mlp_opts(C.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        rep = MlpReport()
        self._check(self.lib.ivr_train_inverse_mlp(self.ctx, C.byref(o), C.byref(rep)))
        return {"loss": list(rep.loss[:rep.n_loss]), "heldout_mean_err": rep.heldout_mean_err,
                "heldout_max_err": rep.heldout_max_err, "ms_samples": rep.ms_samples,
                "ms_train": rep.ms_train}

    def mlp_forward_backward(self, params, x, p):
        fptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
        params = np.ascontiguousarray(params, dtype=np.float32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert params.size == MLP_PARAMS and x.shape == p.shape == (x.shape[0], 3)
        grad = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        self._check(self.lib.ivr_mlp_forward_backward(self.ctx, fptr(params), fptr(x), fptr(p),
                                                      x.shape[0], fptr(loss), fptr(grad)))
        return float(loss[0]), grad

    def mlp_weights(self, patch: int) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.ivr_mlp_get_weights(self.ctx, int(patch),
                                                 out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def mlp_infer(self, patch, x) -> np.ndarray:
        patch = np.ascontiguousarray(patch, dtype=np.int32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.zeros_like(x)
        self._check(self.lib.ivr_mlp_infer(self.ctx, patch.ctypes.data_as(C.POINTER(C.c_int32)),
                                           x.ctypes.data_as(C.POINTER(C.c_float)), len(x),
                                           out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def delta_e2000(self, rgba_a, rgba_b, background=(1.0, 1.0, 1.0), threshold: float = 5.0,
                    per_pixel: bool = False):
        """CIEDE2000 between two premultiplied RGBA device images (float32, 4 values
        per pixel, same size) composited over `background`: {"max", "mean",
        "over"} (pixels above threshold), and the per-pixel tensor with
        per_pixel."""
        a = rgba_a.contiguous()
        b = rgba_b.contiguous()
        if a.dtype != self.torch.float32 or b.dtype != self.torch.float32 or a.numel() != b.numel() or \
                a.numel() % 4:
            raise ValueError("two float32 RGBA images of the same size")
        n = a.numel() // 4
        out = self.torch.empty(n, dtype=self.torch.float32, device=a.device) if per_pixel else None
        bg = (C.c_double * 3)(*[float(v) for v in background])
        sm = DeltaESummary()
        self._check(self.lib.ivr_delta_e2000(self.ctx, a.data_ptr(), b.data_ptr(), n, bg, float(threshold),
                                             out.data_ptr() if out is not None else None, C.byref(sm)))
        res = {"max": sm.max, "mean": sm.mean, "over": int(sm.over)}
        return (res, out) if per_pixel else res

    def device_bytes(self) -> dict:
        """Device memory held by the uploaded model and by the frame buffers."""
        m, f = C.c_uint64(0), C.c_uint64(0)
        self._check(self.lib.ivr_device_bytes(self.ctx, C.byref(m), C.byref(f)))
        return {"model": m.value, "frame": f.value}

    def phase_times(self, cap: int = 4096) -> np.ndarray:
        """(n, 3) milliseconds (fragments, integrate, merge) of the renders recorded
        with timing=1 since the last call."""
        buf = np.zeros(3 * cap)
        n = C.c_int32(0)
        self._check(self.lib.ivr_phase_times(self.ctx, buf.ctypes.data_as(C.POINTER(C.c_double)),
                                             cap, C.byref(n)))
        return buf[:3 * min(n.value, cap)].reshape(-1, 3)

    def _outputs(self, cam, rgba, depth):
        torch = self.torch
        dev = torch.device("cuda", self.device)
        if rgba is None:
            rgba = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
        if depth is None:
            depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device=dev)
        for t, n in ((rgba, cam.width * cam.height * 4), (depth, cam.width * cam.height)):
            if not (t.is_contiguous() and t.dtype == torch.float32 and t.device == dev
                    and t.numel() >= n):
                raise ValueError("outputs must be contiguous float32 tensors of the view's size "
                                 "on the renderer's device")
        return rgba, depth

    def _batch_args(self, views, tf, opts, kw, outputs, flags=False, pixel_accuracy=False):
        if opts is None:
            opts = default_opts(**kw)
        elif kw:
            raise ValueError("pass either opts or keyword options")
        keep, descs, outs = [], (ViewDesc * len(views))(), []
        for i, v in enumerate(views):
            cam, vtf, model = v[0], v[1] if len(v) > 1 else None, v[2] if len(v) > 2 else 0
            rgba, depth = self._outputs(cam, *(outputs[i][:2] if outputs else (None, None)))
            item = [rgba, depth]
            if flags:
                fl = self.torch.empty((cam.height, cam.width), dtype=self.torch.int32,
                                      device=rgba.device)
                descs[i].flags_dev = fl.data_ptr()
                item.append(fl)
            if pixel_accuracy:
                dpb = self.torch.empty((cam.height, cam.width), dtype=self.torch.float32, device=rgba.device)
                descs[i].dp_dev = dpb.data_ptr()
                item.append(dpb)
            outs.append(tuple(item))
            d = descs[i]
            d.cam = camera_desc(cam)
            if vtf is not None:
                t = _TF(vtf)
                keep.append(t)
                d.tf = C.cast(C.pointer(t.desc), C.c_void_p)
            d.model = int(model)
            d.rgba_dev = rgba.data_ptr()
            d.depth_dev = depth.data_ptr()
        btf = _TF(tf) if tf is not None else None
        return opts, descs, outs, btf, keep

    def render_batch(self, views, tf=None, opts: Optional[RenderOpts] = None, outputs=None,
                     stats: bool = False, flags: bool = False, pixel_accuracy: bool = False, **kw):
        """views: sequence of (camera, transfer_function or None, model index).
        Returns [(rgba, depth)] per view, plus flags (int32 IVR_FLAG_* bits per
        pixel) with flags and the per-pixel largest Delta P (float) with
        pixel_accuracy, in that order, and the batch counters with stats."""
        opts, descs, outs, btf, keep = self._batch_args(views, tf, opts, kw, outputs, flags, pixel_accuracy)
        st = Stats() if stats else None
        rc = self.lib.ivr_render_batch(self.ctx, descs, len(views),
                                       C.byref(btf.desc) if btf is not None else None,
                                       C.byref(opts), C.byref(st) if st is not None else None)
        self._check(rc)
        if st is None:
            return outs
        out = {f: int(getattr(st, f)) for f in STAT_FIELDS}
        out.update(ms_fragments=st.ms_fragments, ms_integrate=st.ms_integrate, ms_merge=st.ms_merge)
        return outs, out

    def autotune(self, views, tf=None, opts: Optional[RenderOpts] = None, outputs=None, **kw) -> dict:
        opts, descs, outs, btf, keep = self._batch_args(views, tf, opts, kw, outputs)
        rep = TuneReport()
        self._check(self.lib.ivr_autotune(self.ctx, descs, len(views),
                                          C.byref(btf.desc) if btf is not None else None,
                                          C.byref(opts), C.byref(rep)))
        return {"tile_w": rep.tile_w, "tile_h": rep.tile_h, "xcd_chunk": rep.xcd_chunk,
                "int_block": rep.int_block, "int_waves_cu": rep.int_waves_cu,
                "tried_ms": list(rep.tried_ms[:rep.n_tried]), "ms_before": rep.ms_before,
                "ms_after": rep.ms_after}

    def set_launch(self, tile_w=8, xcd_chunk=0, int_block=256, int_waves_cu=0) -> None:
        self._check(self.lib.ivr_set_launch(self.ctx, tile_w, xcd_chunk, int_block, int_waves_cu))

    def render(self, cam, tf, opts: Optional[RenderOpts] = None, rgba=None, depth=None,
               stats: bool = False, noalloc: bool = False, **kw):
        """One view.  noalloc: through ivr_render_noalloc (frame buffers in the
        device's fixed scratch array, no allocation by the library)."""
        if opts is None:
            opts = default_opts(**kw)
        elif kw:
            raise ValueError("pass either opts or keyword options")
        rgba, depth = self._outputs(cam, rgba, depth)
        cd = camera_desc(cam)
        td = _TF(tf)
        st = Stats() if stats else None
        fn = self.lib.ivr_render_noalloc if noalloc else self.lib.ivr_render
        rc = fn(self.ctx, C.byref(cd), C.byref(td.desc), C.byref(opts),
                C.c_void_p(rgba.data_ptr()), C.c_void_p(depth.data_ptr()),
                C.byref(st) if st is not None else None)
        self._check(rc)
        out = None
        if st is not None:
            out = {f: int(getattr(st, f)) for f in STAT_FIELDS}
            out.update(ms_fragments=st.ms_fragments, ms_integrate=st.ms_integrate,
                       ms_merge=st.ms_merge)
        return rgba, depth, out

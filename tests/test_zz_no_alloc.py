"""ivr_render_noalloc (frame buffers in the device's fixed scratch array) against
ivr_render (the context's own buffers), through the C ABI: the same kernels on the
same inputs give the same image, depth and counters, on two calls in a row (the
second on a smaller view, so stale contents of the shared array would show), and
sizes beyond the array's stated maximum are refused before anything is launched."""
import numpy as np
import pytest

from scenes import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    from paper_1404_3363_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


def _np(t):
    return t.cpu().numpy().astype(np.float64)


def _both(r, sc, cam, **kw):
    import torch
    a, da, sa = r.render(cam, sc.tf, stats=True, **kw)
    b, db, sb = r.render(cam, sc.tf, stats=True, noalloc=True, **kw)
    torch.cuda.synchronize()
    return (_np(a), _np(da), sa), (_np(b), _np(db), sb)


@pytest.mark.parametrize("k,sizes", [(3, [(640, 360), (320, 180)]), (4, [(480, 270), (200, 120)])])
def test_noalloc_matches_render_on_two_calls(renderer, k, sizes):
    for w, h in sizes:
        sc = make_config(k, w, h)
        cam = sc.cameras[1]
        renderer.upload(sc.patches)
        print(f"[noalloc] config{k} {w}x{h}", flush=True)
        (a, da, sa), (b, db, sb) = _both(renderer, sc, cam)
        err = float(np.abs(a - b).max())
        hit = np.isfinite(da)
        print(f"[noalloc] config{k} {w}x{h}: segments {sb['segments']} (render {sa['segments']}), "
              f"max|rgba diff| {err:.3e}", flush=True)
        assert (np.isfinite(db) == hit).all()
        assert np.array_equal(da[hit], db[hit])
        assert err <= 1e-6
        for key in ("rays", "segments", "fragments", "anomalies", "rk_steps", "w_evals", "subsamples"):
            assert sa[key] == sb[key], key
        assert sb["segment_overflow"] == 0 and sb["fragment_overflow"] == 0


def test_noalloc_fp64_matches_render(renderer):
    sc = make_config(1)
    cam = sc.cameras[0]
    renderer.upload(sc.patches)
    (a, da, sa), (b, db, sb) = _both(renderer, sc, cam, precision="fp64", rk_tol=1e-6)
    assert float(np.abs(a - b).max()) <= 1e-12
    assert sa["segments"] == sb["segments"] and sb["segment_overflow"] == 0


@pytest.mark.parametrize("opts", [dict(interior="rf", cut_plane=((0.5, 0.5, 0.5), (0.6, -0.3, 0.74)), near_clip=0.5),
                                  dict(field="param_quality")], ids=["rf_planes", "param_quality"])
def test_noalloc_matches_render_with_options(renderer, opts):
    """Root finding with clip planes, and the parametrisation-quality field: the
    scratch-array entry gives the allocating entry's image and counters."""
    sc = make_config(3, 320, 180)
    cam = sc.cameras[0]
    renderer.upload(sc.patches)
    (a, da, sa), (b, db, sb) = _both(renderer, sc, cam, **opts)
    hit = np.isfinite(da)
    assert (np.isfinite(db) == hit).all() and np.array_equal(da[hit], db[hit])
    assert float(np.abs(a - b).max()) <= 1e-6
    for key in ("rays", "segments", "fragments", "anomalies", "w_evals", "samples"):
        assert sa[key] == sb[key], key


def test_noalloc_refuses_what_does_not_fit(renderer):
    from paper_1404_3363_amd.ivr import IvrError, IVR_EOVERFLOW, IVR_EINVAL
    from scenes import camera_from_angles
    sc = make_config(1)
    renderer.upload(sc.patches)
    big = camera_from_angles([0.5, 0.5, 0.5], 3.0, 30.0, 20.0, 1025, 1024)
    with pytest.raises(IvrError) as e:
        renderer.render(big, sc.tf, noalloc=True)
    assert e.value.code == IVR_EOVERFLOW
    with pytest.raises(IvrError) as e:
        renderer.render(sc.cameras[0], sc.tf, noalloc=True, timing=1)
    assert e.value.code == IVR_EINVAL

"""GPU tests of the batched path: many views of different sizes and models in one
fragment launch, one persistent integrator launch per degree class and one merge,
replayed from a captured HIP graph; the autotuner's launch shapes.

* A batch gives, bit for bit, the images of the same views rendered one at a time
  (each lane's work does not depend on which other rays share its wave).
* Graph replays with cameras changed in between match direct launches every time,
  with eager renders and synchronisations between the replays.
* The batched-views workload (two models, 32 views) at reduced resolution matches
  the oracle on sampled pixels of every view.
* Autotuned launch shapes leave the images unchanged.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from scenes import make_config, camera_from_angles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    from paper_1404_3363_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


def _np(t):
    return t.cpu().numpy().astype(np.float64)


def _small_models():
    c1 = make_config(1)
    c3 = make_config(3, 160, 90)
    return c1, c3


def _views(c1, c3):
    tf2 = dataclasses.replace(c1.tf, extinction=2.0)
    cams = [c1.cameras[0],
            camera_from_angles([0.5, 0.5, 0.5], 3.0, 120.0, -15.0, 33, 17),
            c3.cameras[0],
            dataclasses.replace(c3.cameras[0], width=97, height=55)]
    return [(cams[0], c1.tf, 0), (cams[1], tf2, 0), (cams[2], c3.tf, 1), (cams[3], c3.tf, 1)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_views_rendered_alone(renderer, precision):
    """Four views of two models and four sizes in one graph replay give, bit for
    bit, the images of the same views rendered alone (FP32 and FP64 paths)."""
    import torch
    c1, c3 = _small_models()
    renderer.upload_models([c1.patches, c3.patches])
    views = _views(c1, c3)
    print(f"[batch] 4 views, 2 models, graph replay, {precision}", flush=True)
    outs = renderer.render_batch(views, precision=precision)
    torch.cuda.synchronize()
    for i, v in enumerate(views):
        alone, st = renderer.render_batch([v], stats=True, precision=precision)
        torch.cuda.synchronize()
        a_rgba, a_depth = _np(alone[0][0]), _np(alone[0][1])
        b_rgba, b_depth = _np(outs[i][0]), _np(outs[i][1])
        print(f"[batch] view {i} {v[0].width}x{v[0].height}: segments {st['segments']}, "
              f"max|diff| {np.abs(a_rgba - b_rgba).max():.1e}", flush=True)
        assert np.array_equal(a_rgba, b_rgba)
        assert np.array_equal(a_depth, b_depth)
        assert st["segments"] > 0 and st["anomalies"] == 0


@pytest.mark.parametrize("opts", [dict(interior="rf"), dict(interior="rk4"), dict(field="param_quality"),
                                  dict(cut_plane=((0.5, 0.5, 0.5), (0.6, -0.3, 0.74)), near_clip=0.5)],
                         ids=["rf", "rk4", "param_quality", "planes"])
def test_batch_options_equal_views_rendered_alone(renderer, opts):
    """The batch path with the root-finding and fixed-step interior methods, the
    parametrisation-quality field and the cutting and near-clip planes: each view
    of the graph replay equals, bit for bit, the view rendered alone."""
    import torch
    c1, c3 = _small_models()
    renderer.upload_models([c1.patches, c3.patches])
    views = _views(c1, c3)
    outs = renderer.render_batch(views, **opts)
    torch.cuda.synchronize()
    for i, v in enumerate(views):
        alone, st = renderer.render_batch([v], stats=True, **opts)
        torch.cuda.synchronize()
        assert np.array_equal(_np(alone[0][0]), _np(outs[i][0])), (opts, i)
        assert np.array_equal(_np(alone[0][1]), _np(outs[i][1])), (opts, i)
        assert st["anomalies"] == 0 and st["restart_fail"] == 0, (opts, i, st)


def test_graph_replays_follow_the_view_table(renderer):
    """Three replays of one captured batch with the cameras moved between them and
    eager work (a single-view render, a synchronisation) in between; every replay
    equals direct launches of the same views."""
    import torch
    c1, c3 = _small_models()
    renderer.upload_models([c1.patches, c3.patches])
    base = _views(c1, c3)
    outs = None
    for rep, az in enumerate((10.0, 75.0, 200.0)):
        moved = [(camera_from_angles([0.5, 0.5, 0.5], 3.0, az + 15 * i, 20.0, v[0].width,
                                     v[0].height) if v[2] == 0 else v[0], v[1], v[2])
                 for i, v in enumerate(base)]
        outs = renderer.render_batch(moved, outputs=[(o[0], o[1]) for o in outs] if outs else None)
        torch.cuda.synchronize()
        got = [(_np(o[0]), _np(o[1])) for o in outs]
        renderer.render(c1.cameras[0], c1.tf)          # eager work between replays
        torch.cuda.synchronize()
        ref, _ = renderer.render_batch(moved, stats=True)
        torch.cuda.synchronize()
        for i in range(len(moved)):
            assert np.array_equal(got[i][0], _np(ref[i][0])), (rep, i)
            assert np.array_equal(got[i][1], _np(ref[i][1])), (rep, i)
        print(f"[batch] replay {rep} matches direct launches", flush=True)


def test_batched_views_workload_matches_oracle(renderer):
    """Two models (the 256-block NURBS channel and the 512-block mixed-degree
    lattice), 32 views of the batched-views workload at 1/8 resolution in one
    batch; seeded covered and random pixels of every view against the oracle."""
    import torch
    a, b, views = make_config(5)
    renderer.upload_models([a.patches, b.patches])
    small = [(dataclasses.replace(cam, width=max(cam.width // 8, 1), height=max(cam.height // 8, 1)),
              (a, b)[mi].tf, mi) for mi, cam in views]
    print(f"[batch] config5: {len(small)} views, {sum(c.width * c.height for c, _, _ in small)} rays",
          flush=True)
    outs, st = renderer.render_batch(small, stats=True)
    torch.cuda.synchronize()
    print(f"[batch] config5 stats: segments {st['segments']} anomalies {st['anomalies']} "
          f"overflow {st['fragment_overflow']}/{st['segment_overflow']}", flush=True)
    assert st["fragment_overflow"] == 0 and st["segment_overflow"] == 0
    graph_outs = renderer.render_batch(small)
    torch.cuda.synchronize()
    rng = np.random.default_rng(55)
    worst = 0.0
    for i, (cam, tf, mi) in enumerate(small):
        img = _np(outs[i][0]).reshape(-1, 4)
        assert np.array_equal(img, _np(graph_outs[i][0]).reshape(-1, 4))
        cov = np.flatnonzero(img[:, 3] > 0)
        pix = np.unique(np.concatenate([rng.choice(cov, min(12, len(cov)), replace=False),
                                        rng.choice(cam.width * cam.height, 4, replace=False)]))
        ref = oracle.render((a, b)[mi], cam, tf, pixels=pix)
        err = float(np.abs(img[pix] - ref.rgba).max())
        worst = max(worst, err)
        assert err <= 1e-3, (i, err)
    print(f"[batch] config5 worst |rgba - oracle| over all views: {worst:.2e}", flush=True)


def test_batched_views_full_resolution_sampled(renderer):
    """The batched-views workload at full resolution (32 views of 256^2..2048^2, two
    models, 47M rays) in one graph replay: no anomaly or overflow, and 64 pixels of
    every view (48 covered, 16 anywhere) within the bar against the oracle."""
    import torch
    a, b, views = make_config(5)
    renderer.upload_models([a.patches, b.patches])
    vs = [(cam, (a, b)[mi].tf, mi) for mi, cam in views]
    print(f"[batch] config5 full resolution: {sum(c.width * c.height for c, _, _ in vs)} rays", flush=True)
    outs, st = renderer.render_batch(vs, stats=True)
    torch.cuda.synchronize()
    print(f"[batch] config5 full: segments {st['segments']} anomalies {st['anomalies']} "
          f"overflow {st['fragment_overflow']}/{st['segment_overflow']}", flush=True)
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0 and st["segment_overflow"] == 0
    replay = renderer.render_batch(vs)
    torch.cuda.synchronize()
    preps = [oracle.OracleScene(m.patches, m.scale) for m in (a, b)]
    rng = np.random.default_rng(56)
    worst, n = 0.0, 0
    for i, (cam, tf, mi) in enumerate(vs):
        img = _np(outs[i][0]).reshape(-1, 4)
        assert np.array_equal(img, _np(replay[i][0]).reshape(-1, 4)), i
        cov = np.flatnonzero(img[:, 3] > 0)
        pix = np.unique(np.concatenate([rng.choice(cov, min(48, len(cov)), replace=False),
                                        rng.choice(cam.width * cam.height, 16, replace=False)]))
        ref = oracle.render((a, b)[mi], cam, tf, pixels=pix, prepared=preps[mi])
        err = float(np.abs(img[pix] - ref.rgba).max())
        worst = max(worst, err)
        n += len(pix)
        assert err <= 1e-3, (i, err)
    print(f"[batch] config5 full resolution: {n} pixels, worst |rgba - oracle| {worst:.2e}", flush=True)
    assert n >= 32 * 60


def test_frame_buffers_are_sized_from_counts():
    """A fresh context renders the batched-views workload (47M rays): its frame
    buffers follow the segments and candidates the batch needs (2.2 segments per
    pixel here), not 32 segment slots per pixel, and stay under 10 GB."""
    import torch
    from paper_1404_3363_amd import Renderer
    r = Renderer(0)
    try:
        a, b, views = make_config(5)
        r.upload_models([a.patches, b.patches])
        vs = [(cam, (a, b)[mi].tf, mi) for mi, cam in views]
        outs, st = r.render_batch(vs, stats=True)
        r.render_batch(vs, outputs=outs)
        torch.cuda.synchronize()
        mem = r.device_bytes()
        rays = sum(c.width * c.height for c, _, _ in vs)
        print(f"[batch] config5 frame buffers {mem['frame'] / 1e9:.2f} GB for {rays} rays, "
              f"{st['segments'] / rays:.2f} segments per ray; model {mem['model'] / 1e6:.1f} MB", flush=True)
        assert st["segment_overflow"] == 0 and mem["frame"] < 10e9
    finally:
        r.close()


def test_batch_of_32_views_at_2048():
    """32 views of 2048^2 (134M rays, more than 2^32 / 32 pixels) in one batch of
    the step channel: accepted, no overflow, sampled pixels of every view within
    the bar against the oracle."""
    import torch
    from paper_1404_3363_amd import Renderer
    r = Renderer(0)
    try:
        sc = make_config(4)
        r.upload(sc.patches)
        rng = np.random.default_rng(77)
        vs = [(camera_from_angles(sc.cameras[0].target, float(np.linalg.norm(sc.cameras[0].eye - sc.cameras[0].target)),
                                  rng.uniform(0, 360), rng.uniform(-40, 40), 2048, 2048), sc.tf, 0) for _ in range(32)]
        print("[batch] 32 views of 2048^2", flush=True)
        outs, st = r.render_batch(vs, stats=True, flags=True)
        torch.cuda.synchronize()
        mem = r.device_bytes()
        print(f"[batch] 32x2048^2: segments {st['segments']} overflow {st['fragment_overflow']}/"
              f"{st['segment_overflow']} anomalies {st['anomalies']}; frame buffers {mem['frame'] / 1e9:.1f} GB",
              flush=True)
        for i, (cam, _, _) in enumerate(vs):
            bad = np.flatnonzero(outs[i][2].cpu().numpy().reshape(-1) & 1)
            for q in bad:
                print(f"[batch] unpaired crossing: view {i} (eye {np.round(cam.eye, 6).tolist()}) pixel "
                      f"x={q % cam.width} y={q // cam.width}", flush=True)
        assert st["rays"] == 32 * 2048 * 2048
        assert st["segment_overflow"] == 0 and st["fragment_overflow"] == 0
        # rare unpaired crossings (rays grazing a block edge), at most one in 10^7 rays
        assert st["anomalies"] <= st["rays"] // 10_000_000
        prep = oracle.OracleScene(sc.patches, sc.scale)
        worst = 0.0
        for i, (cam, tf, _) in enumerate(vs):
            img = _np(outs[i][0]).reshape(-1, 4)
            cov = np.flatnonzero(img[:, 3] > 0)
            pix = np.unique(np.concatenate([rng.choice(cov, min(6, len(cov)), replace=False),
                                            rng.choice(cam.width * cam.height, 2, replace=False)]))
            ref = oracle.render(sc, cam, tf, pixels=pix, prepared=prep)
            worst = max(worst, float(np.abs(img[pix] - ref.rgba).max()))
        print(f"[batch] 32x2048^2 worst |rgba - oracle| {worst:.2e}", flush=True)
        assert worst <= 1e-3
    finally:
        r.close()


def test_transfer_functions_with_many_knots(renderer):
    """A 16-knot transfer function (14 interior knots, the most a view holds),
    alone against the oracle, and in one batch with an 8-knot view: the batch
    counts every sample's interval over the knot slots its views use, and each
    view's image equals its render alone."""
    import torch
    from scenes import random_tf
    c1 = make_config(1)
    cam = c1.cameras[0]
    tf16 = random_tf(np.random.default_rng(7101), c1.tf.extinction, c1.tf.domain, n_knots=16)
    renderer.upload_models([c1.patches])
    (alone16,), st = renderer.render_batch([(cam, tf16, 0)], stats=True)
    (alone8,) = renderer.render_batch([(cam, c1.tf, 0)])
    both = renderer.render_batch([(cam, c1.tf, 0), (cam, tf16, 0)])
    torch.cuda.synchronize()
    img = _np(alone16[0]).reshape(-1, 4)
    ref = oracle.render(c1, cam, tf16)
    err = float(np.abs(img - ref.rgba).max())
    print(f"[batch] 16-knot transfer function {cam.width}x{cam.height}: segments {st['segments']}, "
          f"max|rgba - oracle| {err:.3e}", flush=True)
    assert (ref.n_anomalies == 0).all() and st["anomalies"] == 0
    assert err <= 1e-3
    for (a_rgba, a_depth), (b_rgba, b_depth) in ((alone8, both[0]), (alone16, both[1])):
        assert np.array_equal(_np(a_rgba), _np(b_rgba))
        assert np.array_equal(_np(a_depth), _np(b_depth))


def test_mlp_seeded_batch_matches_oracle(renderer):
    """The batched-views workload at 1/16 resolution with MLP seeds (networks
    trained for all 768 blocks of both models): the two-pass fragment kernel with
    batched MFMA inference matches the oracle on sampled pixels of every view, and
    the seeds were used (queries recorded, no candidate fell back)."""
    import torch
    a, b, views = make_config(5)
    renderer.upload_models([a.patches, b.patches])
    rep = renderer.train_mlp(steps=600)
    print(f"[batch] MLP for 768 blocks: held-out mean {rep['heldout_mean_err']:.2e}", flush=True)
    small = [(dataclasses.replace(cam, width=max(cam.width // 16, 1), height=max(cam.height // 16, 1)),
              (a, b)[mi].tf, mi) for mi, cam in views]
    outs, st = renderer.render_batch(small, stats=True, seed_mode="mlp")
    torch.cuda.synchronize()
    print(f"[batch] MLP seeds: queries {st['mlp_queries']}, solves {st['face_newton']}, "
          f"iterations/solve {st['face_newton_iter'] / max(st['face_newton'], 1):.3f}", flush=True)
    assert st["mlp_queries"] == st["face_newton"] and st["fragment_overflow"] == 0
    graph_outs = renderer.render_batch(small, seed_mode="mlp")
    torch.cuda.synchronize()
    rng = np.random.default_rng(57)
    worst = 0.0
    for i, (cam, tf, mi) in enumerate(small):
        img = _np(outs[i][0]).reshape(-1, 4)
        assert np.array_equal(img, _np(graph_outs[i][0]).reshape(-1, 4))
        cov = np.flatnonzero(img[:, 3] > 0)
        pix = rng.choice(cov, min(6, len(cov)), replace=False)
        ref = oracle.render((a, b)[mi], cam, tf, pixels=pix)
        worst = max(worst, float(np.abs(img[pix] - ref.rgba).max()))
    print(f"[batch] MLP-seeded batch worst |rgba - oracle|: {worst:.2e}", flush=True)
    assert worst <= 1e-3


def test_autotuned_shapes_keep_the_images(renderer):
    import torch
    c1, c3 = _small_models()
    renderer.upload_models([c1.patches, c3.patches])
    views = _views(c1, c3)
    before = [(_np(o[0]), _np(o[1])) for o in renderer.render_batch(views)]
    torch.cuda.synchronize()
    rep = renderer.autotune(views)
    print(f"[batch] autotune: {rep}", flush=True)
    assert rep["tile_w"] * rep["tile_h"] == 64 and rep["int_block"] in (64, 128, 256)
    after = renderer.render_batch(views)
    torch.cuda.synchronize()
    for i in range(len(views)):
        assert np.array_equal(before[i][0], _np(after[i][0]))
        assert np.array_equal(before[i][1], _np(after[i][1]))
    for tw, xo, blk, wpc in ((16, 0, 64, 8), (32, 1, 128, 16)):
        renderer.set_launch(tw, xo, blk, wpc)
        other = renderer.render_batch(views)
        torch.cuda.synchronize()
        for i in range(len(views)):
            assert np.array_equal(before[i][0], _np(other[i][0])), (tw, xo, blk, wpc, i)
    renderer.set_launch()


def test_batch_errors(renderer):
    from paper_1404_3363_amd import IvrError
    c1, c3 = _small_models()
    renderer.upload_models([c1.patches, c3.patches])
    with pytest.raises(IvrError):
        renderer.render_batch([(c1.cameras[0], c1.tf, 2)])      # no model 2
    with pytest.raises(IvrError):
        renderer.render_batch([(c1.cameras[0], c1.tf, 0)] * 65)  # too many views
    with pytest.raises(IvrError):
        renderer.render_batch([(c1.cameras[0], None, 0)])       # no transfer function

"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (the benchmark spec): max |RGBA_gpu - RGBA_oracle| <= 1e-3 per channel, entry depth
within 1e-5 relative.  Full images at small sizes; at 512^2 and 1920x1080 the
full GPU image is compared on seeded pixel samples (random plus silhouette
pixels) that the oracle computes one by one.
"""
import math

import numpy as np
import pytest

import oracle
from scenes import make_config, make_degenerate, make_edge_lattice, camera_from_angles
from scenes.configs import Patch, TransferFunction

pytestmark = pytest.mark.gpu

RGBA_TOL = 1e-3
DEPTH_REL_TOL = 1e-5


@pytest.fixture(scope="module")
def renderer():
    from paper_1404_3363_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


def _render(r, scene_patches, cam, tf, **kw):
    import torch
    r.upload(scene_patches)
    rgba, depth, st = r.render(cam, tf, stats=True, **kw)
    torch.cuda.synchronize()
    return (rgba.cpu().numpy().reshape(-1, 4).astype(np.float64),
            depth.cpu().numpy().reshape(-1).astype(np.float64), st)


def _silhouette_pixels(depth, w, h):
    d = np.isfinite(depth.reshape(h, w))
    edge = np.zeros_like(d)
    edge[:, 1:] |= d[:, 1:] != d[:, :-1]
    edge[1:, :] |= d[1:, :] != d[:-1, :]
    return np.flatnonzero(edge.reshape(-1))


def _sample(cam, depth, n_random, n_edge, seed):
    rng = np.random.default_rng(seed)
    npx = cam.width * cam.height
    covered = np.flatnonzero(np.isfinite(depth))
    pick = [rng.choice(npx, n_random // 2, replace=False)]
    if len(covered):
        pick.append(rng.choice(covered, min(n_random // 2, len(covered)), replace=False))
    edge = _silhouette_pixels(depth, cam.width, cam.height)
    if len(edge):
        pick.append(rng.choice(edge, min(n_edge, len(edge)), replace=False))
    return np.unique(np.concatenate(pick))


def _stratified_with_silhouette_tiles(cam, depth, n_total, seed, tile=8):
    """A seeded sample of about n_total pixels: one coverage-edge pixel of every
    tile x tile block of the image that holds one, 1/16 of the rest uniform over
    the image, and the remainder stratified over the covered pixels (one from each
    of that many equal runs in raster order).  Returns (pixels, silhouette part)."""
    w, h = cam.width, cam.height
    rng = np.random.default_rng(seed)
    edge = _silhouette_pixels(depth, w, h)
    tid = (edge // w // tile) * ((w + tile - 1) // tile) + (edge % w) // tile
    order = rng.permutation(len(edge))
    _, first = np.unique(tid[order], return_index=True)
    sil = edge[order[first]]
    n_bg = max((n_total - len(sil)) // 16, 0)
    bg = rng.choice(w * h, n_bg, replace=False)
    covered = np.flatnonzero(np.isfinite(depth))
    n_cov = max(n_total - len(sil) - n_bg, 1)
    runs = [r for r in np.array_split(covered, min(n_cov, len(covered))) if len(r)]
    cov = np.array([r[rng.integers(len(r))] for r in runs], dtype=np.int64)
    return np.unique(np.concatenate([sil, bg, cov])), sil


def _compare(name, img, depth, ref, pix=None, scale=1.0):
    if pix is not None:
        img, depth = img[pix], depth[pix]
    err = np.abs(img - ref.rgba)
    # depth is compared where both hit and the oracle's first chord is not a
    # grazing sliver (< 1e-4 of the scene scale)
    both = np.isfinite(depth) & np.isfinite(ref.depth) & (ref.first_chord >= 1e-4 * scale)
    rel = np.abs(depth[both] - ref.depth[both]) / ref.depth[both] if both.any() else np.zeros(1)
    cover_mismatch = int((np.isfinite(depth) != np.isfinite(ref.depth)).sum())
    print(f"[parity] {name}: n={len(img)} max|rgba|={err.max():.3e} mean={err.mean():.3e} "
          f"depth_rel={rel.max():.3e} coverage_mismatch={cover_mismatch}", flush=True)
    assert (ref.n_anomalies == 0).all() and (ref.n_newton_fail == 0).all()
    worst = int(np.unravel_index(err.argmax(), err.shape)[0])
    wpix = int(pix[worst]) if pix is not None else worst
    print(f"[parity] {name}: worst pixel {wpix} gpu={img[worst]} oracle={ref.rgba[worst]} "
          f"gpu_depth={depth[worst]:.6f} oracle_depth={ref.depth[worst]:.6f} "
          f"oracle_nseg={ref.n_segments[worst]}", flush=True)
    assert err.max() <= RGBA_TOL, (name, err.max(), wpix)
    assert rel.max() <= DEPTH_REL_TOL, (name, rel.max())
    # a coverage mismatch is allowed only where the oracle's opacity is negligible
    mism = np.isfinite(depth) != np.isfinite(ref.depth)
    assert (ref.rgba[mism, 3] <= RGBA_TOL).all()


def test_config1_fp64_full_image(renderer):
    sc = make_config(1)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp64", rk_tol=1e-6)
    ref = oracle.render(sc, cam, sc.tf)
    _compare("config1 fp64 64x64", img, depth, ref, scale=sc.scale)
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0 and st["segment_overflow"] == 0


def test_config1_fp32_full_image(renderer):
    sc = make_config(1)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", rk_tol=1e-6)
    ref = oracle.render(sc, cam, sc.tf)
    _compare("config1 fp32 64x64", img, depth, ref, scale=sc.scale)


def _box_chord(o, d):
    t0, t1 = -np.inf, np.inf
    for c in range(3):
        a, b = (0 - o[c]) / d[c], (1 - o[c]) / d[c]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return (t0, t1) if t1 > max(t0, 0) else (None, None)


def test_constant_field_closed_form(renderer):
    """Constant rho: alpha = 1 - exp(-kappa L), RGB = E alpha; L and the entry depth
    from the ray-box closed form (config 1's boundary is the unit cube)."""
    sc = make_config(1)
    P = sc.patches[0]
    Pc = Patch(P.degree, P.ncp, P.knots, P.cp, np.full_like(P.scalar, 0.37), False)
    tf = TransferFunction(sc.tf.x, sc.tf.rgba, 4.0, (0.0, 1.0))
    cam = camera_from_angles([0.5, 0.5, 0.5], 3.0, 30.0, 20.0, 40, 40)
    img, depth, _ = _render(renderer, [Pc], cam, tf, precision="fp32")
    E = np.array([np.interp(0.37, tf.x, tf.rgba[:, c]) for c in range(4)])
    kappa = 4.0 * E[3]
    worst = 0.0
    for pix in range(40 * 40):
        o, d = oracle.camera_ray(cam, pix % 40 + 0.5, pix // 40 + 0.5)
        t0, t1 = _box_chord(o, d)
        if t0 is None:
            assert img[pix, 3] == 0.0 and np.isinf(depth[pix])
            continue
        a = 1.0 - math.exp(-kappa * (t1 - t0))
        worst = max(worst, abs(img[pix, 3] - a), np.abs(img[pix, :3] - E[:3] * a).max())
        assert abs(depth[pix] - t0) <= DEPTH_REL_TOL * t0
    print(f"[parity] constant field closed form: max err {worst:.3e}", flush=True)
    assert worst <= RGBA_TOL


@pytest.mark.parametrize("view", [0, 1])
def test_degenerate_face_full_image(renderer, view):
    """J singular on a whole boundary face (first two control layers coincide):
    rays that enter (view 0) or leave (view 1) through it are shrunk by
    Eq. (degeneracyfix); full 96x96 image against the oracle, no NaN."""
    sc = make_degenerate()
    cam = sc.cameras[view]
    print(f"[parity] degenerate face view {view}", flush=True)
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    assert np.isfinite(img).all()
    ref = oracle.render(sc, cam, sc.tf)
    _compare(f"degenerate face view{view} 96x96", img, depth, ref, scale=sc.scale)
    print(f"[parity] degenerate face view {view}: shrunk segment ends {st['degenerate']}, "
          f"fp64 solves {st['fp64_solves']}, iteration cap {st['rk_iter_cap']}", flush=True)
    assert st["degenerate"] > 100 and st["rk_iter_cap"] == 0


@pytest.mark.parametrize("view", [0, 1, 2])
def test_rays_through_block_edges_and_corners(renderer, view):
    """Centre rays exactly through an edge of four blocks (view 0), a corner of
    eight (view 1) and a boundary edge of two (view 2): the crossings found from
    different faces of one point must leave every block paired (no anomaly);
    the full 65x65 image against the oracle."""
    sc = make_edge_lattice()
    cam = sc.cameras[view]
    print(f"[parity] edge lattice view {view}", flush=True)
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    ref = oracle.render(sc, cam, sc.tf)
    _compare(f"edge lattice view{view} 65x65", img, depth, ref, scale=sc.scale)
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0
    centre = 32 * cam.width + 32
    assert abs(depth[centre] - ref.depth[centre]) <= DEPTH_REL_TOL * ref.depth[centre]


@pytest.mark.parametrize("tile_w", [16, 32])
def test_tile_frustum_culling_keeps_every_candidate(renderer, tile_w):
    """The traversal culls blocks and element tiles against each pixel tile's
    frustum.  On the 65x65 edge-lattice views, where the last tile column and
    row are partial (one pixel wide or high for 8x8 tiles), tiles of 16x4 and
    32x2 pixels give the image and depth of 8x8 tiles bit for bit, with the same
    Newton solves: the per-ray candidates do not depend on the tile's shape."""
    import torch
    sc = make_edge_lattice()
    renderer.upload(sc.patches)
    try:
        for view, cam in enumerate(sc.cameras):
            renderer.set_launch(8)
            a, da, sa = renderer.render(cam, sc.tf, stats=True, precision="fp32")
            renderer.set_launch(tile_w)
            b, db, sb = renderer.render(cam, sc.tf, stats=True, precision="fp32")
            torch.cuda.synchronize()
            print(f"[parity] edge lattice view {view} tiles {tile_w}x{64 // tile_w}: box tests "
                  f"{sb['box_tests']} (8x8: {sa['box_tests']}), solves {sb['face_newton']}", flush=True)
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), view
            assert np.array_equal(da.cpu().numpy(), db.cpu().numpy()), view
            assert sb["face_newton"] == sa["face_newton"] and sb["anomalies"] == 0 and sa["anomalies"] == 0
    finally:
        renderer.set_launch()


def test_face_with_more_than_64_element_tiles(renderer):
    """A cubic block of 40^3 control points has 37 x 37 elements per face in 100
    element tiles, more than one 64-lane culling pass per face.  With an affine map
    and a constant field every pixel is the closed form alpha = 1 - exp(-kappa L)
    of the ray's chord L through the parallelepiped, with the chord's entry as
    depth; the pixels that miss it stay empty."""
    from scenes import affine_patch
    A = np.array([[1.1, 0.2, 0.0], [-0.1, 0.95, 0.15], [0.05, 0.0, 1.05]])
    b0 = np.array([-0.3, 0.1, 0.2])
    P = affine_patch(A, b0, (3, 3, 3), (40, 40, 40), scalar=lambda g: np.full(len(g), 0.5))
    cam = camera_from_angles(A @ np.full(3, 0.5) + b0, 3.2, 40.0, 25.0, 96, 96)
    tf = TransferFunction(np.array([0.0, 0.5, 1.0]), np.array([[0.1, 0.2, 0.9, 0.1], [0.9, 0.5, 0.1, 0.6],
                                                                [0.3, 0.8, 0.4, 0.9]]), 3.0, (0.0, 1.0))
    img, depth, st = _render(renderer, [P], cam, tf, precision="fp32")
    E = np.array([np.interp(0.5, tf.x, tf.rgba[:, c]) for c in range(4)])
    Ainv = np.linalg.inv(A)
    worst, worst_depth, hits = 0.0, 0.0, 0
    for pix in range(cam.width * cam.height):
        o, d = oracle.camera_ray(cam, pix % cam.width + 0.5, pix // cam.width + 0.5)
        po, pd = Ainv @ (o - b0), Ainv @ d
        t0, t1 = -np.inf, np.inf
        for c in range(3):
            a_, b_ = (0 - po[c]) / pd[c], (1 - po[c]) / pd[c]
            t0, t1 = max(t0, min(a_, b_)), min(t1, max(a_, b_))
        if not (t1 > max(t0, 0.0)):
            assert img[pix, 3] == 0.0 and np.isinf(depth[pix]), pix
            continue
        hits += 1
        a = 1.0 - math.exp(-tf.extinction * E[3] * (t1 - t0))
        worst = max(worst, float(np.abs(img[pix] - np.concatenate([E[:3] * a, [a]])).max()))
        worst_depth = max(worst_depth, abs(depth[pix] - t0) / t0)
    print(f"[parity] 40^3 affine block: {hits} rays, max err {worst:.2e}, depth rel {worst_depth:.2e}, "
          f"solves {st['face_newton']}", flush=True)
    assert hits > 2000 and worst <= 1e-5 and worst_depth <= DEPTH_REL_TOL
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0


@pytest.mark.parametrize("name", ["config3", "config4", "edge_lattice"])
def test_random_views_at_odd_sizes(renderer, name):
    """Twelve seeded random views per model at odd sizes (partial tiles one or a
    few pixels wide or high), camera 0.5 to 2.5 diagonals away: tiles of 8x8, 16x4
    and 32x2 pixels give the same image bit for bit, and the full image is within
    the bar against the oracle with the same coverage and no anomaly."""
    import torch
    sc = {"config3": lambda: make_config(3, 97, 61), "config4": lambda: make_config(4, 97, 61),
          "edge_lattice": make_edge_lattice}[name]()
    renderer.upload(sc.patches)
    rng = np.random.default_rng({"config3": 1, "config4": 2, "edge_lattice": 3}[name])
    lo, hi = np.asarray(sc.bbox[0]), np.asarray(sc.bbox[1])
    centre, diag = 0.5 * (lo + hi), float(np.linalg.norm(hi - lo))
    try:
        for it in range(12):
            w, h = int(rng.integers(17, 90)), int(rng.integers(9, 70))
            cam = camera_from_angles(centre + rng.uniform(-0.2, 0.2, 3) * diag, diag * float(rng.uniform(0.5, 2.5)),
                                     float(rng.uniform(0, 360)), float(rng.uniform(-60, 60)), w, h)
            out = []
            for tw in (8, 16, 32):
                renderer.set_launch(tw)
                img, depth, st = renderer.render(cam, sc.tf, stats=True)
                torch.cuda.synchronize()
                out.append((img.cpu().numpy().astype(np.float64), depth.cpu().numpy().astype(np.float64), st))
            for img, depth, _ in out[1:]:
                assert np.array_equal(img, out[0][0]) and np.array_equal(depth, out[0][1]), (name, it)
            img, depth, st = out[0]
            ref = oracle.render(sc, cam, sc.tf)
            _compare(f"{name} random view {it} {w}x{h}", img.reshape(-1, 4), depth.reshape(-1), ref, scale=sc.scale)
            assert st["anomalies"] == 0, (name, it)
    finally:
        renderer.set_launch()


def test_degenerate_face_constant_field_closed_form(renderer):
    """Constant rho on the degenerate-face cube: alpha = 1 - exp(-kappa L) with L
    the ray-box chord of the unit cube, for both views."""
    sc = make_degenerate(constant_field=True, width=40, height=40)
    E = np.array([np.interp(0.5, sc.tf.x, sc.tf.rgba[:, c]) for c in range(4)])
    kappa = 4.0 * E[3]
    for view, cam in enumerate(sc.cameras):
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
        worst, hits = 0.0, 0
        for pix in range(40 * 40):
            o, d = oracle.camera_ray(cam, pix % 40 + 0.5, pix // 40 + 0.5)
            t0, t1 = _box_chord(o, d)
            if t0 is None:
                continue
            hits += 1
            a = 1.0 - math.exp(-kappa * (t1 - t0))
            worst = max(worst, abs(img[pix, 3] - a), np.abs(img[pix, :3] - E[:3] * a).max())
            assert abs(depth[pix] - t0) <= DEPTH_REL_TOL * t0
        print(f"[parity] degenerate constant field view {view}: max err {worst:.3e} "
              f"({hits} rays, {st['degenerate']} shrunk)", flush=True)
        assert worst <= RGBA_TOL and hits > 200


@pytest.mark.parametrize("view", [0, 1, 2])
def test_config2_twisted_bar_sampled(renderer, view):
    sc = make_config(2)
    cam = sc.cameras[view]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", rk_tol=1e-5)
    pix = _sample(cam, depth, 512, 256, 20 + view)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare(f"config2 view{view} 512x512", img, depth, ref, pix, sc.scale)
    assert st["segment_overflow"] == 0
    assert st["anomalies"] == 0


# Rays of the twisted bar that clip a thin sliver of it, crossing one curved face
# element twice (found as the only pairing anomalies of the 512^2 views when an
# element gave at most one root): view, pixel x, y.
_DOUBLE_CROSSINGS = [(0, 283, 170), (2, 224, 419), (2, 285, 254), (2, 232, 249)]


def test_element_crossed_twice(renderer):
    sc = make_config(2)
    for view in sorted({v for v, _, _ in _DOUBLE_CROSSINGS}):
        cam = sc.cameras[view]
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", rk_tol=1e-5)
        pix = np.array([y * cam.width + x for v, x, y in _DOUBLE_CROSSINGS if v == view])
        ref = oracle.render(sc, cam, sc.tf, pixels=pix)
        assert (ref.n_segments >= 1).all()
        _compare(f"config2 view{view} double crossings", img, depth, ref, pix, sc.scale)
        assert st["anomalies"] == 0


def test_config3_bent_beam_1080p_stratified(renderer):
    """The headline view at 1920x1080 against the oracle on a stratified sample of
    16384 pixels that holds a pixel of every 8x8 silhouette tile."""
    sc = make_config(3)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    pix, sil = _stratified_with_silhouette_tiles(cam, depth, 16384, 31)
    print(f"[parity] config3 stratified sample: {len(pix)} pixels, {len(sil)} silhouette tiles", flush=True)
    assert len(pix) >= 16000 and len(sil) > 500
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare("config3 1920x1080 stratified", img, depth, ref, pix, sc.scale)
    print(f"[stats] config3: {st}", flush=True)
    assert st["fragment_overflow"] == 0 and st["segment_overflow"] == 0
    assert st["anomalies"] == 0


def test_config4_nurbs_channel_1080p_sampled(renderer):
    sc = make_config(4)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    pix = _sample(cam, depth, 512, 256, 41)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare("config4 1920x1080", img, depth, ref, pix, sc.scale)
    print(f"[stats] config4: {st}", flush=True)
    assert st["anomalies"] == 0
    assert st["fragment_overflow"] == 0 and st["segment_overflow"] == 0


def test_config4_nurbs_channel_1080p_stratified(renderer):
    """The NURBS channel (256 curved rational blocks, non-uniform weights) at
    1920x1080 against the oracle on a stratified sample of 16384 pixels that
    holds a pixel of every 8x8 silhouette tile."""
    sc = make_config(4)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    pix, sil = _stratified_with_silhouette_tiles(cam, depth, 16384, 43)
    print(f"[parity] config4 stratified sample: {len(pix)} pixels, {len(sil)} silhouette tiles", flush=True)
    assert len(pix) >= 16000 and len(sil) > 300
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare("config4 1920x1080 stratified", img, depth, ref, pix, sc.scale)
    assert st["anomalies"] == 0


@pytest.mark.parametrize("k", [3, 4])
def test_multiblock_fp64_stratified(renderer, k):
    """The FP64 path (FP64 face roots, pairing and integrator) on the multi-block
    models, shared faces and NURBS blocks included, at 480x270 against the oracle on
    a stratified sample of 4096 pixels with every 8x8 silhouette tile; every
    crossing paired."""
    sc = make_config(k, 480, 270)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp64")
    pix, sil = _stratified_with_silhouette_tiles(cam, depth, 4096, 50 + k)
    print(f"[parity] config{k} fp64 stratified sample: {len(pix)} pixels, {len(sil)} silhouette tiles", flush=True)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare(f"config{k} fp64 480x270 stratified", img, depth, ref, pix, sc.scale)
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0 and st["segment_overflow"] == 0


@pytest.mark.parametrize("k", [3, 4])
def test_every_ray_pairs_cleanly_at_1080p(renderer, k):
    """All views of the multi-block models at 1920x1080 (6.2M rays): every
    crossing is paired (rays through block edges and corners, grazing rays)."""
    sc = make_config(k)
    for view, cam in enumerate(sc.cameras):
        _, _, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
        print(f"[parity] config{k} view{view}: rays {st['rays']} segments {st['segments']} "
              f"anomalies {st['anomalies']}", flush=True)
        assert st["anomalies"] == 0 and st["fragment_overflow"] == 0 and st["segment_overflow"] == 0


@pytest.mark.parametrize("k,cpp", [(2, 0), (3, 0), (3, 1), (4, 0)])
def test_rays_past_the_candidate_list_traverse_again(renderer, k, cpp):
    """Rays whose candidates do not fit the candidate list are traversed again
    by the solve launch and solved ray by ray (cand_per_pixel 0: every ray; 1:
    the tiles recorded after the list fills).  The same candidates give the same
    roots: crossings, segments and image agree with the list path, and a sample
    agrees with the oracle."""
    sc = make_config(k)
    cam = sc.cameras[0]
    img0, d0, st0 = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    img1, d1, st1 = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", cand_per_pixel=cpp)
    print(f"[parity] config{k} cand_per_pixel={cpp}: candidates {st1['face_newton']} "
          f"(list path {st0['face_newton']}), box tests {st1['box_tests']} ({st0['box_tests']}), "
          f"max|rgba - list path| {np.abs(img1 - img0).max():.3e}", flush=True)
    for key in ("face_newton", "fragments", "segments"):
        assert st1[key] == st0[key], key
    assert st1["box_tests"] > st0["box_tests"]   # the second traversal ran
    assert st1["anomalies"] == 0 and st1["fragment_overflow"] == 0 and st1["segment_overflow"] == 0
    assert np.abs(img1 - img0).max() <= 1e-5
    hit = np.isfinite(d0)
    assert (np.isfinite(d1) == hit).all()
    assert (np.abs(d1[hit] - d0[hit]) <= 1e-6 * d0[hit]).all()
    pix = _sample(cam, d1, 256, 128, 50 + k)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare(f"config{k} cand_per_pixel={cpp}", img1, d1, ref, pix, sc.scale)


@pytest.mark.parametrize("size", [(1, 1), (67, 35), (8, 8)])
def test_ragged_and_tiny_images(renderer, size):
    sc = make_config(1)
    w, h = size
    cam = camera_from_angles([0.5, 0.5, 0.5], 3.0, 30.0, 20.0, w, h)
    img, depth, _ = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    ref = oracle.render(sc, cam, sc.tf)
    _compare(f"config1 {w}x{h}", img, depth, ref, scale=sc.scale)


def test_view_that_misses_everything(renderer):
    sc = make_config(1)
    # eye between the block and the target: every ray points away from the block
    cam = camera_from_angles([5.0, 5.0, 5.0], 1.0, 225.0, -35.0, 32, 32)
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf)
    assert (img == 0).all() and np.isinf(depth).all() and st["segments"] == 0


def test_render_is_deterministic(renderer):
    sc = make_config(3, 320, 180)
    cam = sc.cameras[1]
    a, da, _ = _render(renderer, sc.patches, cam, sc.tf)
    b, db, _ = _render(renderer, sc.patches, cam, sc.tf)
    assert np.array_equal(a, b) and np.array_equal(da, db)


def test_error_codes(renderer):
    from paper_1404_3363_amd import IvrError
    sc = make_config(1)
    P = sc.patches[0]
    bad = Patch(P.degree, P.ncp, [P.knots[0][::-1], P.knots[1], P.knots[2]], P.cp, P.scalar)
    with pytest.raises(IvrError) as e:
        renderer.upload([bad])
    assert e.value.code == -1
    renderer.upload(sc.patches)
    with pytest.raises(IvrError) as e:
        renderer.render(sc.cameras[0], sc.tf, seed_mode="mlp")
    assert e.value.code in (-4,)
    bad_tf = TransferFunction(np.array([0.0, 0.7, 0.5, 1.0]), np.ones((4, 4)), 1.0, (0.0, 1.0))
    with pytest.raises(IvrError) as e:
        renderer.render(sc.cameras[0], bad_tf)
    assert e.value.code == -1
    for opt in ({"rho_step": 0.0}, {"tf_step": -1.0}, {"rho_step": float("nan")}, {"h_max": float("inf")},
                {"cand_per_pixel": -1}, {"cand_per_pixel": 65}):
        with pytest.raises(IvrError) as e:
            renderer.render(sc.cameras[0], sc.tf, **opt)
        assert e.value.code == -1, opt


_BAD_OPTIONS = [
    {"precision": 5}, {"rk_tol": 0.0}, {"rk_tol": float("nan")}, {"h_max": float("nan")}, {"c_perp": -1.0},
    {"n_super": 0}, {"n_super": 65}, {"det_fp64_threshold": -1.0}, {"det_singular": -1.0}, {"drift_tol": -1.0},
    {"interior": 9}, {"interior": -1}, {"near_clip": -1.0}, {"near_clip": float("inf")},
    {"cut_plane": ((0.5, 0.5, 0.5), (0.0, 0.0, 0.0))}, {"cut_plane": ((float("nan"), 0.5, 0.5), (1.0, 0.0, 0.0))},
    {"max_fragments": 1}, {"max_fragments": 65}, {"rho_interp": 7}, {"seed_mode": 9}, {"early_term": 1.0},
    {"early_term": -0.1}, {"max_newton_iter": 0}, {"max_newton_iter": 101}, {"field": 3}, {"newton_stop": 2},
    {"field": "param_quality", "interior": "rk4"},
]


def test_options_out_of_range_are_refused(renderer):
    """Every option outside its documented range is refused with IVR_EINVAL before
    anything is launched, and the context renders as before afterwards."""
    import torch
    from paper_1404_3363_amd import IvrError
    sc = make_config(1)
    cam = sc.cameras[0]
    renderer.upload(sc.patches)
    before, d0, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    before = before.cpu().numpy().copy()
    for opt in _BAD_OPTIONS:
        with pytest.raises(IvrError) as e:
            renderer.render(cam, sc.tf, **opt)
        assert e.value.code == -1, opt
    after, d1, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(before, after.cpu().numpy())


def _bad_patches():
    """Blocks that break one documented rule each (arrays sized for what the
    library reads before it refuses them)."""
    import dataclasses
    from scenes import affine_patch
    P = make_config(1).patches[0]
    out = []
    for deg in ((0, 2, 2), (4, 2, 2)):
        out.append(("degree", dataclasses.replace(P, degree=deg)))
    out.append(("ncp", dataclasses.replace(P, ncp=(2, 4, 4))))
    k = [np.array(x, dtype=np.float64) for x in P.knots]
    out.append(("not clamped", dataclasses.replace(P, knots=[np.array([0, 0, 0.1, 0.5, 1, 1, 1.0]), k[1], k[2]])))
    out.append(("empty span", dataclasses.replace(P, knots=[np.zeros(7), k[1], k[2]])))
    Q = affine_patch(np.eye(3), np.zeros(3), (2, 2, 2), (6, 4, 4))
    out.append(("multiplicity", dataclasses.replace(Q, knots=[np.array([0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1.0])] +
                                                       list(Q.knots[1:]))))
    cp = P.cp.copy(); cp[5, 1] = np.nan
    out.append(("nan point", dataclasses.replace(P, cp=cp)))
    sc = P.scalar.copy(); sc[7] = np.nan
    out.append(("nan scalar", dataclasses.replace(P, scalar=sc)))
    cp = P.cp.copy(); cp[3, 3] = 0.0
    out.append(("zero weight", dataclasses.replace(P, cp=cp, rational=True)))
    du = np.zeros((len(P.scalar), 3)); du[9, 2] = np.inf
    out.append(("displacement", dataclasses.replace(P, displacement=du)))
    return out


def test_invalid_blocks_are_refused(renderer):
    """Every block that breaks a documented rule (degree 1..3, ncp >= degree+1,
    clamped non-decreasing knots with a non-empty span and interior multiplicity
    at most the degree, finite points and field, positive NURBS weights, finite
    displacement) is refused with IVR_EINVAL, and the model uploaded before stays
    in place."""
    import torch
    from paper_1404_3363_amd import IvrError
    sc = make_config(1)
    cam = sc.cameras[0]
    renderer.upload(sc.patches)
    before, _, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    before = before.cpu().numpy().copy()
    for name, bad in _bad_patches():
        with pytest.raises(IvrError) as e:
            renderer.upload([bad])
        assert e.value.code == -1, name
    after, _, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(before, after.cpu().numpy())


def test_invalid_cameras_are_refused(renderer):
    """Cameras outside the documented ranges (image 1..16384 pixels a side, field
    of view in (0, 179) degrees, finite vectors, eye apart from the target, up not
    along the view) are refused with IVR_EINVAL; the next valid render is as before."""
    import dataclasses
    import torch
    from paper_1404_3363_amd import IvrError
    sc = make_config(1)
    cam = sc.cameras[0]
    renderer.upload(sc.patches)
    before, _, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    before = before.cpu().numpy().copy()
    view = np.asarray(cam.target, dtype=np.float64) - np.asarray(cam.eye, dtype=np.float64)
    bad = [dict(width=0), dict(width=4, height=20000), dict(fov_y_deg=0.0), dict(fov_y_deg=179.5),
           dict(eye=np.array([np.nan, 0.0, 0.0])), dict(eye=np.asarray(cam.target, dtype=np.float64)),
           dict(up=view)]
    for kw in bad:
        with pytest.raises(IvrError) as e:
            renderer.render(dataclasses.replace(cam, **kw), sc.tf)
        assert e.value.code == -1, kw
    after, _, _ = renderer.render(cam, sc.tf, stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(before, after.cpu().numpy())


def test_sampling_options_follow_their_definitions(renderer):
    """h_max and rho_step bound the RK steps, tf_step the supersampling sub-steps:
    tighter bounds take more steps / sub-steps and the image stays within the bar."""
    sc = make_config(3, 160, 90)
    cam = sc.cameras[0]
    ref_pix = np.arange(0, 160 * 90, 37)
    ref = oracle.render(sc, cam, sc.tf, pixels=ref_pix)
    runs = {}
    for name, kw in (("default", {}), ("h_max/4", {"h_max": sc.scale / 128}),
                     ("rho_step/4", {"rho_step": 0.025}), ("tf_step/4", {"tf_step": 0.00625})):
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", **kw)
        err = float(np.abs(img[ref_pix] - ref.rgba).max())
        print(f"[parity] sampling {name}: rk steps {st['rk_steps']} sub-steps {st['subsamples']} "
              f"max err {err:.2e}", flush=True)
        assert err <= RGBA_TOL
        runs[name] = st
    assert runs["h_max/4"]["rk_steps"] > 1.5 * runs["default"]["rk_steps"]
    assert runs["rho_step/4"]["rk_steps"] >= runs["default"]["rk_steps"]
    assert runs["tf_step/4"]["rk_steps"] == runs["default"]["rk_steps"]
    assert runs["tf_step/4"]["subsamples"] > 1.5 * runs["default"]["subsamples"]


def _annulus_chord(o, d, prm):
    """Total chord of the ray through the quarter annulus, and its first entry, from
    the closed-form roots of its two cylinders and four planes."""
    roots = []
    a = d[0] ** 2 + d[1] ** 2
    b = 2.0 * (o[0] * d[0] + o[1] * d[1])
    for R in (prm["r_in"], prm["r_out"]):
        c = o[0] ** 2 + o[1] ** 2 - R * R
        disc = b * b - 4.0 * a * c
        if a > 0.0 and disc > 0.0:
            q = -0.5 * (b + math.copysign(math.sqrt(disc), b))
            roots += [q / a, c / q]
    for ax, val in ((0, 0.0), (1, 0.0), (2, 0.0), (2, prm["height"])):
        if d[ax] != 0.0:
            roots.append((val - o[ax]) / d[ax])
    roots = sorted(t for t in roots if t > 0.0)

    def inside(t):
        x = o + t * d
        r = math.hypot(x[0], x[1])
        return (prm["r_in"] <= r <= prm["r_out"] and x[0] >= 0.0 and x[1] >= 0.0
                and 0.0 <= x[2] <= prm["height"])
    L, first = 0.0, None
    for t0, t1 in zip(roots[:-1], roots[1:]):
        if inside(0.5 * (t0 + t1)):
            L += t1 - t0
            first = t0 if first is None else first
    return L, first


@pytest.mark.parametrize("view", [0, 1, 2])
def test_nurbs_annulus_full_image(renderer, view):
    """Rational faces with non-uniform knots (quadratic NURBS quarter annulus whose
    curved faces are exact cylinders): full 48x48 image against the oracle."""
    from scenes import make_annulus
    sc = make_annulus()
    cam = sc.cameras[view]
    print(f"[parity] NURBS annulus view {view}", flush=True)
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
    ref = oracle.render(sc, cam, sc.tf)
    _compare(f"NURBS annulus view{view} 48x48", img, depth, ref, scale=sc.scale)
    assert st["anomalies"] == 0 and st["fragment_overflow"] == 0 and st["segment_overflow"] == 0
    assert st["segments"] > 500


def test_nurbs_annulus_constant_field_closed_form(renderer):
    """Constant rho on the NURBS annulus: alpha = 1 - exp(-kappa L), RGB = E alpha with
    L the closed-form chord through the cylinders and planes; depth = first entry."""
    from scenes import make_annulus
    sc = make_annulus(constant_field=True, width=40, height=40)
    E = np.array([np.interp(0.5, sc.tf.x, sc.tf.rgba[:, c]) for c in range(4)])
    kappa = sc.tf.extinction * E[3]
    for view, cam in enumerate(sc.cameras):
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
        worst, hits = 0.0, 0
        for pix in range(cam.width * cam.height):
            o, d = oracle.camera_ray(cam, pix % cam.width + 0.5, pix // cam.width + 0.5)
            L, first = _annulus_chord(o, d, sc.params)
            a = 1.0 - math.exp(-kappa * L)
            worst = max(worst, abs(img[pix, 3] - a), np.abs(img[pix, :3] - E[:3] * a).max())
            if first is not None:
                hits += 1
                assert abs(depth[pix] - first) <= DEPTH_REL_TOL * first, (view, pix)
        print(f"[parity] NURBS annulus constant field view {view}: max err {worst:.3e} ({hits} rays)",
              flush=True)
        assert worst <= RGBA_TOL and hits > 300


# ------------------------------------------------------------------ robustness options

def test_fragment_cap_of_two_counts_overflow(renderer):
    """max_fragments = 2 on the bent beam (rays cross up to 20 block faces): the
    crossings past the cap are dropped and counted, and the image stays finite."""
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, max_fragments=2)
    print(f"[robust] max_fragments=2: overflow {st['fragment_overflow']} anomalies {st['anomalies']}",
          flush=True)
    assert st["fragment_overflow"] > 0
    assert np.isfinite(img).all() and (img[:, 3] >= 0).all() and (img[:, 3] <= 1 + 1e-6).all()
    assert not np.isnan(depth).any()


def test_one_newton_iteration_counts_failures(renderer):
    """max_newton_iter = 1: the face Newton gets one iteration per seed.  Roots that
    no seed then reaches leave crossings unpaired or segments missing: the image
    stays finite, and either it is within the bar or the failures show in the
    counters and in the per-pixel flags."""
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img0, d0, fl0, st0 = _render_flags(renderer, sc, cam)
    img1, d1, fl1, st1 = _render_flags(renderer, sc, cam, max_newton_iter=1)
    err = float(np.abs(img1 - img0).max())
    print(f"[robust] max_newton_iter=1: segments {st1['segments']} ({st0['segments']}), anomalies "
          f"{st1['anomalies']}, flagged pixels {int(((fl1 & 1) != 0).sum())}, max|diff| {err:.2e}", flush=True)
    assert np.isfinite(img1).all()
    assert err <= RGBA_TOL or st1["segments"] != st0["segments"] or st1["anomalies"] > 0
    assert ((fl1 & 1) != 0).sum() <= st1["anomalies"]


def test_every_solve_in_fp64(renderer):
    """det_fp64_threshold = 1e30 sends every 3x3 solve of W to FP64 (fp64_solves ==
    w_evals); the degeneracy rule keeps its own threshold; the image stays within
    the bar against the oracle."""
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, det_fp64_threshold=1e30)
    print(f"[robust] all-FP64 solves: fp64_solves {st['fp64_solves']} w_evals {st['w_evals']} "
          f"degenerate {st['degenerate']}", flush=True)
    assert st["fp64_solves"] == st["w_evals"] > 0 and st["degenerate"] == 0
    pix = _sample(cam, depth, 384, 128, 71)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare("config3 480x270 all solves FP64", img, depth, ref, pix, sc.scale)


# ------------------------------------------------------------------ sampling readings and precision

@pytest.mark.parametrize("k", [1, 2, 3])
def test_linear_rho_as_in_the_paper(renderer, k):
    """Supersampling as the paper states it (Sec. "Quadrature of volume render
    integral"): rho linear between two samples.  Its error falls as h^2; with rho's
    change per step bounded by 0.0125 of the domain and h_max = scale/256 all three
    configs are within the bar (rho_step 0.025, scale/128 is the loosest that is)."""
    sc = make_config(k) if k != 3 else make_config(3, 480, 270)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", rho_interp="linear",
                             rho_step=0.0125, h_max=sc.scale / 256)
    pix = None if k == 1 else _sample(cam, depth, 512, 256, 80 + k)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    _compare(f"config{k} linear rho", img, depth, ref, pix, sc.scale)
    assert st["anomalies"] == 0


def test_config1_fp64_at_fine_sampling(renderer):
    """FP64 on config 1 against a tight oracle (panels of scale/8192, self-error
    1e-9): with h_max, rho_step and tf_step divided by 4 the image is within 1e-5,
    by 16 within 1e-6; the error is the sampling's, not the arithmetic's."""
    sc = make_config(1)
    cam = sc.cameras[0]
    ref = oracle.render(sc, cam, sc.tf, self_tol=1e-9, panels_per_scale=8192.0)
    assert ref.self_error.max() <= 1e-8
    for div, bar in ((4, 1e-5), (16, 1e-6)):
        kw = dict(rk_tol=1e-8, h_max=sc.scale / (32 * div), rho_step=0.1 / div, tf_step=0.025 / div)
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp64", **kw)
        err = float(np.abs(img - ref.rgba).max())
        img32, _, _ = _render(renderer, sc.patches, cam, sc.tf, precision="fp32", **kw)
        err32 = float(np.abs(img32 - ref.rgba).max())
        print(f"[parity] config1 sampling/{div}: fp64 max err {err:.2e}, fp32 {err32:.2e}", flush=True)
        assert err <= bar, (div, err)


@pytest.mark.parametrize("rational", [False, True])
def test_per_direction_degrees(renderer, rational):
    """Blocks whose directions differ in degree: (1, 2, 3) B-spline and (2, 3, 3)
    NURBS with non-uniform knots.  The library raises each to one degree at upload
    (exact degree elevation); the oracle evaluates the block as given.  Full 64x64
    images of two views against the oracle."""
    from scenes import make_mixed_degree
    sc = make_mixed_degree(rational)
    for view, cam in enumerate(sc.cameras):
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp32")
        ref = oracle.render(sc, cam, sc.tf)
        _compare(f"degrees {sc.patches[0].degree} view{view}", img, depth, ref, scale=sc.scale)
        assert st["anomalies"] == 0 and st["segments"] > 1000


# ------------------------------------------------------------------ drift guard and per-pixel flags

def _render_flags(r, sc, cam, **kw):
    import torch
    r.upload(sc.patches)
    outs, st = r.render_batch([(cam, sc.tf, 0)], stats=True, flags=True, **kw)
    torch.cuda.synchronize()
    rgba, depth, fl = outs[0]
    return (rgba.cpu().numpy().reshape(-1, 4).astype(np.float64),
            depth.cpu().numpy().reshape(-1).astype(np.float64), fl.cpu().numpy().reshape(-1), st)


def _wavy_block_with_linear_field(width=256, height=256):
    """A cubic block with 24 x 6 x 6 control points whose layers wave along x
    (y + 0.12 sin(3 pi u), z + 0.08 cos(2 pi u) at the Greville points u of
    [0, 4] x [0, 1]^2; det J > 0), so the parameter ray curves strongly and a loose
    RK tolerance lets it drift, and the field rho = a.x + b exactly (coefficients
    a.P + b reproduce it by partition of unity), so rho is linear along every ray
    and samples at any step size interpolate it exactly: only where the samples
    are taken can be wrong.  One view across the waves."""
    from scenes.configs import (Scene, open_uniform_knots, greville, _grid_points, _make_patch, bbox_of,
                                random_tf, extinction_for)
    p, n = (3, 3, 3), (24, 6, 6)
    knots = [open_uniform_knots(n[d], 3) for d in range(3)]
    g = _grid_points(*(greville(knots[d], 3) for d in range(3)))
    xyz = np.stack([4.0 * g[..., 0], g[..., 1] + 0.12 * np.sin(3 * math.pi * g[..., 0]),
                    g[..., 2] + 0.08 * np.cos(2 * math.pi * g[..., 0])], axis=-1)
    rho = xyz @ np.array([0.05, 0.3, 0.2]) + 0.3
    P = _make_patch(p, n, knots, xyz, rho)
    bbox = bbox_of([P])
    tf = random_tf(np.random.Generator(np.random.PCG64(6400)), extinction_for(bbox),
                   (float(rho.min()), float(rho.max())))
    cam = camera_from_angles(0.5 * (bbox[0] + bbox[1]), 6.0, 70.0, 25.0, width, height)
    return Scene("wavy_block_linear_field", [P], tf, [cam], bbox)


def test_drift_restarts_keep_the_image(renderer):
    """c_perp = 0 (nothing pulls the parameter ray back onto the view ray), a loose
    rk_tol = 1e-2 and long steps (h_max = scale/4, no bound from rho's change) on
    a wavy block with a field linear in world coordinates: the samples drift off
    the ray.  Before each sample the distance of phi(p) from the ray point is
    checked and the point is found again by Newton when it exceeds drift_tol;
    restarts are counted and flagged per pixel, the image stays within the bar,
    and its error is well below that of the same render with the check off."""
    sc = _wavy_block_with_linear_field()
    cam = sc.cameras[0]
    kw = dict(c_perp=0.0, rk_tol=1e-2, h_max=sc.scale / 4, rho_step=10.0)
    # drift_tol 1e-5 (tighter than the default) so that the restarts are many
    img, depth, fl, st = _render_flags(renderer, sc, cam, drift_tol=1e-5, **kw)
    img0, _, fl0, st0 = _render_flags(renderer, sc, cam, drift_tol=0.0, **kw)
    pix = _sample(cam, depth, 512, 256, 90)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    err0 = float(np.abs(img0[pix] - ref.rgba).max())
    flagged = int(((fl & 16) != 0).sum())
    print(f"[drift] c_perp=0 rk_tol=1e-2: restarts {st['drift_restarts']} (failed {st['restart_fail']}), "
          f"flagged pixels {flagged}, rk steps {st['rk_steps']}; without the check max err {err0:.2e}",
          flush=True)
    _compare("wavy block, linear field, c_perp=0 rk_tol=1e-2, drift restarts", img, depth, ref, pix, sc.scale)
    err = float(np.abs(img[pix] - ref.rgba).max())
    assert st["drift_restarts"] > 300 and st["restart_fail"] == 0 and flagged > 100
    assert st0["drift_restarts"] == 0 and not (fl0 & 16).any()
    assert err < 0.6 * err0   # the restarts bring the samples back onto the ray


def test_per_pixel_flags(renderer):
    """The flag buffer: zero on a clean render of the bent beam, and the pixels whose
    crossings overflow max_fragments = 2 carry IVR_FLAG_FRAGMENT_OVERFLOW; a singular
    face flags the pixels whose segments it ends."""
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img, depth, fl, st = _render_flags(renderer, sc, cam)
    assert (fl == 0).all() and st["anomalies"] == 0
    img, depth, fl, st = _render_flags(renderer, sc, cam, max_fragments=2)
    n_ovf = int(((fl & 2) != 0).sum())
    print(f"[flags] max_fragments=2: {n_ovf} pixels flagged, {st['fragment_overflow']} crossings dropped",
          flush=True)
    assert 0 < n_ovf <= st["fragment_overflow"]
    _, depth_all, _, _ = _render_flags(renderer, sc, cam)
    assert ((fl & 2) == 0)[np.isinf(depth_all)].all()   # rays that miss every block cannot overflow
    dg = make_degenerate()
    img, depth, fl, st = _render_flags(renderer, dg, dg.cameras[0])
    n_deg = int(((fl & 64) != 0).sum())
    print(f"[flags] degenerate face: {n_deg} pixels flagged, {st['degenerate']} singular ends", flush=True)
    assert 0 < n_deg <= st["degenerate"]


# ------------------------------------------------------------------ root finding; cutting and near clip planes

@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_root_finding_interior_method(renderer, k):
    """The root-finding interior method (Sec. "Root Finding Based Algorithm"): every
    sample's preimage by Newton from the previous sample's, moved along J^-1 d;
    same step bounds as the ODE method.  Within the bar against the oracle."""
    sc = make_config(k) if k <= 2 else make_config(k, 480, 270)
    cam = sc.cameras[0]
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, interior="rf")
    _, _, st_ode = _render(renderer, sc.patches, cam, sc.tf)
    pix = None if k == 1 else _sample(cam, depth, 512, 256, 100 + k)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    print(f"[rf] config{k}: samples {st['rk_steps']} evaluations {st['w_evals']} failed {st['restart_fail']} | "
          f"ODE steps {st_ode['rk_steps']} evaluations {st_ode['w_evals']}", flush=True)
    _compare(f"config{k} root finding", img, depth, ref, pix, sc.scale)
    assert st["restart_fail"] == 0 and st["anomalies"] == 0


def _cube_kept_chord(o, d, fwd, cut=None, near=0.0):
    t0, t1 = -np.inf, np.inf
    for c in range(3):
        a, b = (0 - o[c]) / d[c], (1 - o[c]) / d[c]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    t0 = max(t0, 0.0)
    if near > 0.0:
        t0 = max(t0, near / float(d @ fwd))
    if cut is not None:
        g0, n = (np.asarray(v, float) for v in cut)
        s0, sd = float(n @ (o - g0)), float(n @ d)
        if sd > 0:
            t0 = max(t0, -s0 / sd)
        elif sd < 0:
            t1 = min(t1, -s0 / sd)
    return (t0, t1 - t0) if t1 > t0 else (None, 0.0)


@pytest.mark.parametrize("case", ["cut", "near", "eye_inside", "cut_and_near"])
@pytest.mark.parametrize("interior", ["ode", "rf"])
def test_clip_planes_constant_field_closed_form(renderer, case, interior):
    """Sec. "Cutting and Near Clip Planes" on the unit cube with constant rho:
    alpha = 1 - exp(-kappa L), RGB = E alpha with L the closed-form kept chord and
    the depth where it starts; the entries on a plane are found by Newton."""
    sc = make_config(1)
    P = sc.patches[0]
    Pc = Patch(P.degree, P.ncp, P.knots, P.cp, np.full_like(P.scalar, 0.37), False)
    tf = TransferFunction(sc.tf.x, sc.tf.rgba, 4.0, (0.0, 1.0))
    cut = ((0.5, 0.45, 0.55), np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8]))
    if case == "eye_inside":
        cam = camera_from_angles([0.9, 0.5, 0.5], 0.5, 200.0, 10.0, 40, 40, fov_y_deg=60.0)
    else:
        cam = camera_from_angles([0.5, 0.5, 0.5], 3.0, 30.0, 20.0, 40, 40)
    kw = {"cut": {"cut_plane": cut}, "near": {"near_clip": 2.75}, "eye_inside": {"near_clip": 0.05},
          "cut_and_near": {"cut_plane": cut, "near_clip": 2.75}}[case]
    img, depth, st = _render(renderer, [Pc], cam, tf, interior=interior, **kw)
    E = np.array([np.interp(0.37, tf.x, tf.rgba[:, c]) for c in range(4)])
    fwd = (cam.target - cam.eye) / np.linalg.norm(cam.target - cam.eye)
    worst = 0.0
    for pix in range(cam.width * cam.height):
        o, d = oracle.camera_ray(cam, pix % cam.width + 0.5, pix // cam.width + 0.5)
        t_start, L = _cube_kept_chord(o, d, fwd, kw.get("cut_plane"), kw.get("near_clip", 0.0))
        a = 1.0 - math.exp(-4.0 * E[3] * L)
        worst = max(worst, abs(img[pix, 3] - a), np.abs(img[pix, :3] - E[:3] * a).max())
        if t_start is None:
            assert img[pix, 3] == 0.0 and np.isinf(depth[pix]), pix
        else:
            assert abs(depth[pix] - t_start) <= DEPTH_REL_TOL * t_start, (pix, depth[pix], t_start)
    print(f"[planes] {case} {interior}: max err {worst:.2e}, segments {st['segments']}, "
          f"entry solves failed {st['restart_fail']}", flush=True)
    assert worst <= RGBA_TOL and st["anomalies"] == 0 and st["restart_fail"] == 0


@pytest.mark.parametrize("case", ["cut", "near", "eye_inside"])
def test_clip_planes_on_the_bent_beam(renderer, case):
    """The bent beam (config 3, 64 blocks) with a cutting plane through it, a near
    plane through it, and the eye inside it: sampled pixels against the oracle
    with the same planes."""
    import dataclasses
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    centre = 0.5 * (sc.bbox[0] + sc.bbox[1])
    if case == "cut":
        kw = {"cut_plane": (centre, np.array([0.6, 0.3, -0.74]))}
    elif case == "near":
        kw = {"near_clip": float(np.linalg.norm(cam.target - cam.eye))}
    else:
        # the eye just inside one block of the beam, looking along it
        x = 0.5 * (sc.patches[21].cp[:, :3].min(0) + sc.patches[21].cp[:, :3].max(0))
        cam = dataclasses.replace(camera_from_angles(x, 0.02, 200.0, 5.0, 480, 270, fov_y_deg=70.0))
        cam = dataclasses.replace(cam, eye=x.copy(), target=x + (cam.target - cam.eye))
        kw = {"near_clip": 0.01}
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, **kw)
    pix = _sample(cam, depth, 512, 256, 110)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix, **kw)
    print(f"[planes] config3 {case}: segments {st['segments']} entry solves failed {st['restart_fail']}",
          flush=True)
    _compare(f"config3 {case}", img, depth, ref, pix, sc.scale)
    assert st["anomalies"] == 0 and st["restart_fail"] == 0


@pytest.mark.parametrize("k", [1, 2])
def test_gpu_follows_the_method_mode(renderer, k):
    """The GPU's integrator against the oracle's method mode (the same method in
    FP64, written separately): in FP64 the images agree to the rounding of the
    binary32 output, far below the method's own sampling error, so what the parity
    bar measures on the GPU is the method's discretisation, not a different
    algorithm; the RK attempts match."""
    sc = make_config(k)
    cam = sc.cameras[0]
    tol = 1e-6 if k == 1 else 1e-5
    # the method mode has no drift check: off here too
    img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp64", rk_tol=tol, drift_tol=0.0)
    pix = None if k == 1 else _sample(cam, depth, 512, 256, 120)
    method, steps = oracle.render_method(sc, cam, sc.tf, pixels=pix, rk_tol=tol)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    sel = img if pix is None else img[pix]
    d_method = float(np.abs(sel - method).max())
    d_ref = float(np.abs(sel - ref.rgba).max())
    w = int(np.abs(sel - method).max(1).argmax())
    wpix = w if pix is None else int(pix[w])
    print(f"[method] config{k} worst pixel {wpix}: gpu {sel[w]} method mode {method[w]} "
          f"reference {ref.rgba[w]} segments {ref.n_segments[w]} first chord {ref.first_chord[w]:.3e}", flush=True)
    print(f"[method] config{k} fp64: |gpu - method mode| {d_method:.2e}, |gpu - reference| {d_ref:.2e}, "
          f"rk attempts gpu {st['rk_steps']} method mode {steps}", flush=True)
    assert d_method <= 2.0 ** -25 * 1.01 and d_method < 0.05 * d_ref
    if k == 1:
        assert st["rk_steps"] == steps


# ------------------------------------------------------------------ fixed-step methods of the convergence study

FIXED_METHODS = ["rk1", "rk2", "rk3", "rk4", "rk4_38", "rkf5", "irk1"]


@pytest.mark.parametrize("method", FIXED_METHODS)
def test_fixed_step_methods_follow_the_method_mode(renderer, method):
    """The fixed-step methods of Sec. "ODE Based Algorithm" (explicit family and
    implicit Euler with the exact J_G) on the GPU in FP64 against the oracle's
    method mode with the same method and step bound (drift check off, as there):
    full 64x64 images of configs 1 and 2 agree to the rounding of the binary32
    output (at most 2^-25 for values below 1), with the same number of steps on
    config 1."""
    for k in (1, 2):
        sc = make_config(k)
        cam = sc.cameras[0]
        hm = sc.scale / 32
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, precision="fp64", interior=method, h_max=hm,
                                 drift_tol=0.0)
        mm, steps = oracle.render_method(sc, cam, sc.tf, method=method, h_max=hm)
        ref = oracle.render(sc, cam, sc.tf)
        dm = float(np.abs(img - mm).max())
        dr = float(np.abs(img - ref.rgba).max())
        print(f"[fixed] {method} config{k} fp64: |gpu - method mode| {dm:.2e}, |gpu - reference| {dr:.2e}, "
              f"steps gpu {st['rk_steps']} method mode {steps}, evaluations {st['w_evals']}, "
              f"newton failures {st['restart_fail']}", flush=True)
        assert dm <= 2.0 ** -25 * 1.01
        assert st["restart_fail"] == 0 and st["anomalies"] == 0
        if k == 1:
            assert st["rk_steps"] == steps


@pytest.mark.parametrize("method", FIXED_METHODS)
def test_fixed_step_methods_fp32_within_the_bar(renderer, method):
    """FP32 GPU renders of the bent beam (config 3, 480x270) and the NURBS channel
    (config 4) with every fixed-step method at the default options against the
    oracle: within the bar; implicit Euler's Newton (with the Hessian of B-spline and
    NURBS maps) converges on every step of the bent beam.  On the channel's small,
    strongly curved blocks implicit Euler takes h_max = scale/128 (about five
    steps per block): at the default scale/32 a step can span most of a block, and
    there its Newton fails on some steps (flagged), as the oracle's does; at
    scale/128 at most 0.2% of its steps are flagged."""
    for k in (3, 4):
        sc = make_config(k, 480, 270)
        cam = sc.cameras[0]
        kw = dict(h_max=sc.scale / 128) if (method == "irk1" and k == 4) else {}
        img, depth, st = _render(renderer, sc.patches, cam, sc.tf, interior=method, **kw)
        pix = _sample(cam, depth, 384, 128, 300 + k)
        ref = oracle.render(sc, cam, sc.tf, pixels=pix)
        print(f"[fixed] {method} config{k} fp32: steps {st['rk_steps']} evaluations {st['w_evals']} "
              f"drift restarts {st['drift_restarts']} newton failures {st['restart_fail']}", flush=True)
        _compare(f"config{k} {method}", img, depth, ref, pix, sc.scale)
        if method == "irk1" and k == 4:
            # where a step's implicit solution lies outside P (the ray meets the
            # block's boundary between samples) the projected Newton slides along
            # the boundary and may not settle: such steps are flagged and rare
            _, _, s64 = _render(renderer, sc.patches, cam, sc.tf, interior=method, precision="fp64", **kw)
            print(f"[fixed] irk1 config4 fp64: newton failures {s64['restart_fail']} of {s64['rk_steps']} steps",
                  flush=True)
            assert st["restart_fail"] <= 2e-3 * st["rk_steps"]
        else:
            assert st["restart_fail"] == 0


# ------------------------------------------------------------------ derived fields

def _field_tf(sc, field, seed=5):
    """The scene's transfer function over the range of a derived field (its 2nd to
    98th percentile over seeded points of every block, by the oracle)."""
    rng = np.random.default_rng(seed)
    vals = [oracle.field_value(P, p, field) for P in sc.patches for p in rng.uniform(0, 1, (max(2, 256 // len(sc.patches)), 3))]
    lo, hi = np.percentile(vals, [2, 98])
    if hi <= lo:
        lo, hi = lo - 1.0, hi + 1.0
    return TransferFunction(sc.tf.x, sc.tf.rgba, sc.tf.extinction, (float(lo), float(hi)))


@pytest.mark.parametrize("interior", ["ode", "rf"])
@pytest.mark.parametrize("k", [2, 4])
def test_parametrisation_quality_field(renderer, k, interior):
    """The parametrisation quality det J / |J|_F (Eq. (paramQuality)) computed at
    every sample, with its exact gradient for the Hermite interpolation and the
    step bound, on the twisted bar (config 2) and the NURBS channel (config 4):
    within the bar against the oracle's reference render of the same field.  On
    the channel the quality spans only 0.044..0.060, which the transfer function
    stretches over its whole range: the sampling takes rho_step = 0.01 and
    h_max = scale/512 there (at the defaults the error is that of the sampling,
    4e-3 with the ODE, and falls with rho_step)."""
    sc = make_config(k) if k == 2 else make_config(k, 480, 270)
    cam = sc.cameras[0]
    tf = _field_tf(sc, "param_quality")
    kw = {} if k == 2 else dict(rho_step=0.01, h_max=sc.scale / 512)
    img, depth, st = _render(renderer, sc.patches, cam, tf, field="param_quality", interior=interior, **kw)
    pix = None if k == 2 else _sample(cam, depth, 384, 128, 400 + k)
    ref = oracle.render(sc, cam, tf, pixels=pix, field="param_quality")
    _compare(f"config{k} parametrisation quality ({interior})", img, depth, ref, pix, sc.scale)
    assert st["anomalies"] == 0
    if k == 4 and interior == "ode":
        errs = []
        for rs in (0.1, 0.025):
            im, _, _ = _render(renderer, sc.patches, cam, tf, field="param_quality", rho_step=rs)
            errs.append(float(np.abs(im[pix] - ref.rgba).max()))
        print(f"[fields] channel quality, ODE: max err {errs[0]:.2e} at rho_step 0.1, {errs[1]:.2e} at 0.025",
              flush=True)
        assert errs[1] < errs[0]


@pytest.mark.parametrize("k", [3, 4])
def test_von_mises_field(renderer, k):
    """Von Mises of a displacement spline (Eq. (vonMises) as read) with its exact
    gradient, on the bent beam (config 3, cubic B-spline blocks) and the NURBS
    channel (config 4), the displacement a seeded smooth field plus a linear part:
    within the bar against the oracle's reference render (rho_step = 0.05); FP64
    as well on the channel."""
    from scenes import with_displacement
    base = make_config(k, 480, 270)
    B = np.array([[0.01, 0.004, 0.0], [0.002, -0.006, 0.003], [0.0, 0.001, 0.008]])
    sc = with_displacement(base, B=B, amplitude=0.02 * base.scale)
    cam = sc.cameras[0]
    tf = _field_tf(sc, "von_mises")
    for precision in (("fp32", "fp64") if k == 4 else ("fp32",)):
        img, depth, st = _render(renderer, sc.patches, cam, tf, field="von_mises", precision=precision,
                                 rho_step=0.05)
        pix = _sample(cam, depth, 384, 128, 410 + k)
        ref = oracle.render(sc, cam, tf, pixels=pix, field="von_mises")
        _compare(f"config{k} von Mises {precision}", img, depth, ref, pix, sc.scale)


def test_derived_fields_closed_form_and_errors(renderer):
    """On an affine block with u = B phi both derived fields are constant: the GPU
    image is the constant-field closed form.  Von Mises on a model without
    displacement, or a derived field with a fixed-step method, is refused."""
    from paper_1404_3363_amd import IvrError
    from scenes import affine_patch, with_displacement
    from scenes.configs import Scene
    A = np.array([[1.2, 0.1, 0.0], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]])
    b0 = np.array([0.1, -0.2, 0.05])
    P = affine_patch(A, b0)
    B = np.array([[0.02, 0.013, -0.004], [0.001, -0.011, 0.007], [0.009, 0.002, 0.015]])
    bbox = np.array([P.cp[:, :3].min(0), P.cp[:, :3].max(0)])
    cam = camera_from_angles(A @ np.full(3, 0.5) + b0, 3.5, 35.0, 20.0, 40, 40)
    sc = with_displacement(Scene("affine", [P], None, [cam], bbox), B=B)
    e = 0.5 * (B + B.T)
    vm = math.sqrt(0.5 * ((e[0, 0] - e[1, 1]) ** 2 + (e[1, 1] - e[2, 2]) ** 2 + (e[2, 2] - e[0, 0]) ** 2 +
                          6 * (e[0, 1] ** 2 + e[1, 2] ** 2 + e[2, 0] ** 2)))
    Ainv = np.linalg.inv(A)
    for field, value in (("param_quality", np.linalg.det(A) / np.linalg.norm(A)), ("von_mises", vm)):
        tf = TransferFunction(np.array([0.0, 0.5, 1.0]), np.array([[0.1, 0.2, 0.9, 0.1], [0.9, 0.5, 0.1, 0.6],
                                                                    [0.3, 0.8, 0.4, 0.9]]),
                              3.0, (value - abs(value), value + 0.5 * abs(value)))
        img, depth, _ = _render(renderer, sc.patches, cam, tf, field=field)
        n = (value - tf.domain[0]) / (tf.domain[1] - tf.domain[0])
        E = np.array([np.interp(n, tf.x, tf.rgba[:, c]) for c in range(4)])
        worst = 0.0
        for pix in range(cam.width * cam.height):
            o, d = oracle.camera_ray(cam, pix % cam.width + 0.5, pix // cam.width + 0.5)
            po, pd = Ainv @ (o - b0), Ainv @ d
            t0, t1 = -np.inf, np.inf
            for c in range(3):
                a_, b_ = (0 - po[c]) / pd[c], (1 - po[c]) / pd[c]
                t0, t1 = max(t0, min(a_, b_)), min(t1, max(a_, b_))
            if not (t1 > max(t0, 0.0)):
                continue
            a = 1.0 - math.exp(-tf.extinction * E[3] * (t1 - t0))
            worst = max(worst, float(np.abs(img[pix] - np.concatenate([E[:3] * a, [a]])).max()))
        print(f"[fields] affine block, {field}: max err vs closed form {worst:.2e}", flush=True)
        assert worst <= 1e-5
    renderer.upload([P])
    with pytest.raises(IvrError):
        renderer.render(cam, make_config(1).tf, field="von_mises")
    renderer.upload(sc.patches)
    with pytest.raises(IvrError):
        renderer.render(cam, make_config(1).tf, field="param_quality", interior="rk2")


# ------------------------------------------------------------------ pixel accuracy (Definition, Eq. (deltaP))

def _render_dp(r, sc, cam, tf=None, **kw):
    import torch
    r.upload(sc.patches)
    outs, st = r.render_batch([(cam, tf or sc.tf, 0)], stats=True, flags=True, pixel_accuracy=True, **kw)
    torch.cuda.synchronize()
    rgba, depth, fl, dp = outs[0]
    return (rgba.cpu().numpy().reshape(-1, 4).astype(np.float64), depth.cpu().numpy().reshape(-1),
            fl.cpu().numpy().reshape(-1), dp.cpu().numpy().reshape(-1).astype(np.float64), st)


@pytest.mark.parametrize("k", [1, 2])
def test_pixel_accuracy_record_follows_the_method_mode(renderer, k):
    """The instrumented integrator's per-pixel largest Delta P (Eq. (deltaP)) of the
    interior samples, in FP64 with the drift check off, equals the oracle method
    mode's for the same method (adaptive RKF45) to binary32 rounding, and neither
    finds a sample out of depth order; the image is the one the plain integrator
    gives.  Root finding puts the samples on the ray (Delta P at rounding level)."""
    sc = make_config(k)
    cam = sc.cameras[0]
    tol = 1e-6 if k == 1 else 1e-5
    img, depth, fl, dp, st = _render_dp(renderer, sc, cam, precision="fp64", rk_tol=tol, drift_tol=0.0)
    plain, _, _ = _render(renderer, sc.patches, cam, sc.tf, precision="fp64", rk_tol=tol, drift_tol=0.0)
    _, _, rec = oracle.render_method(sc, cam, sc.tf, rk_tol=tol, pixel_accuracy=True)
    dd = float(np.abs(dp - rec["delta_p"]).max())
    print(f"[pixel] config{k} ODE fp64: max Delta P gpu {dp.max():.3e} oracle {rec['delta_p'].max():.3e}, "
          f"|difference| {dd:.2e}; samples over 1: {st['dp_over']}, order violations {st['order_violations']}",
          flush=True)
    assert dd <= 1e-6 * max(1.0, float(dp.max()))
    assert st["order_violations"] == 0 and rec["order_violations"].max() == 0 and not (fl & 128).any()
    assert np.abs(img - plain).max() == 0.0
    _, _, _, dp_rf, st_rf = _render_dp(renderer, sc, cam, precision="fp64", interior="rf")
    print(f"[pixel] config{k} RF fp64: max Delta P {dp_rf.max():.2e}", flush=True)
    assert dp_rf.max() < 1e-6 and st_rf["dp_over"] == 0


def test_default_render_is_pixel_accurate(renderer):
    """The default FP32 render of the bent beam (config 3, 480x270): every interior
    sample projects into its pixel (Delta P <= 1) in depth order."""
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img, depth, fl, dp, st = _render_dp(renderer, sc, cam)
    print(f"[pixel] config3 fp32 defaults: max Delta P {dp.max():.3e}, 99.9th percentile "
          f"{np.percentile(dp, 99.9):.3e}, samples over 1: {st['dp_over']}, order violations "
          f"{st['order_violations']}", flush=True)
    assert dp.max() <= 1.0 and st["dp_over"] == 0 and st["order_violations"] == 0


def test_frustum_newton_stop(renderer):
    """Root finding with the paper's pixel-accurate Newton stop (residual at most the
    sample's distance to its pixel frustum's boundary): every sample lies in its
    pixel (Delta P <= 1), with fewer Newton iterations than the fixed tolerance;
    the image difference from the fixed-tolerance render is reported.  The
    instrumented integrator is refused for a fixed-step method."""
    from paper_1404_3363_amd import IvrError
    sc = make_config(3, 480, 270)
    cam = sc.cameras[0]
    img_t, _, _, dp_t, st_t = _render_dp(renderer, sc, cam, interior="rf")
    img_f, depth, _, dp_f, st_f = _render_dp(renderer, sc, cam, interior="rf", newton_stop="frustum")
    pix = _sample(cam, depth, 384, 128, 431)
    ref = oracle.render(sc, cam, sc.tf, pixels=pix)
    print(f"[pixel] RF tolerance stop: evaluations {st_t['w_evals']}, max Delta P {dp_t.max():.2e}, "
          f"max err {np.abs(img_t[pix] - ref.rgba).max():.2e} | frustum stop: evaluations {st_f['w_evals']}, "
          f"max Delta P {dp_f.max():.2e}, max err {np.abs(img_f[pix] - ref.rgba).max():.2e}", flush=True)
    assert dp_f.max() <= 1.0 and st_f["dp_over"] == 0
    assert st_f["w_evals"] < st_t["w_evals"]
    # the paper's image criterion: colour difference to the reference at most 5
    import torch
    de = renderer.delta_e2000(torch.tensor(img_f, dtype=torch.float32, device="cuda"),
                              torch.tensor(img_t, dtype=torch.float32, device="cuda"))
    print(f"[pixel] frustum vs tolerance stop: CIEDE2000 max {de['max']:.3f} mean {de['mean']:.4f}", flush=True)
    assert de["max"] <= 5.0
    with pytest.raises(IvrError):
        _render_dp(renderer, sc, cam, interior="rk2")


# ------------------------------------------------------------------ CIEDE2000 image comparison

def test_delta_e2000_matches_the_oracle(renderer):
    """The device CIEDE2000 between two seeded premultiplied RGBA images (random
    colours and opacities, identical pixels, grays, transparent pixels) equals the
    oracle's per pixel (FP64 on both sides, binary32 output), and the summary's
    largest, mean and count above 5 agree."""
    import torch
    from oracle import color
    rng = np.random.default_rng(77)
    n = 100_000
    A = rng.uniform(0, 1, (n, 4))
    A[:, :3] *= A[:, 3:4]                          # premultiplied
    B = A + rng.normal(0, 0.03, A.shape)
    B = np.clip(B, 0, 1)
    B[:, :3] = np.minimum(B[:, :3], B[:, 3:4])
    B[:1000] = A[:1000]                            # identical
    g = rng.uniform(0, 1, (1000, 1))
    A[1000:2000] = np.column_stack([g, g, g, np.ones(1000)])
    B[1000:2000] = np.column_stack([g + 0.01, g + 0.01, g + 0.01, np.ones(1000)]).clip(0, 1)
    A[2000:2100, 3] = 0.0
    A[2000:2100, :3] = 0.0
    dev = torch.device("cuda", 0)
    ta = torch.tensor(A, dtype=torch.float32, device=dev)
    tb = torch.tensor(B, dtype=torch.float32, device=dev)
    for bg in ((1.0, 1.0, 1.0), (0.0, 0.0, 0.0)):
        summ, per = renderer.delta_e2000(ta, tb, background=bg, threshold=5.0, per_pixel=True)
        torch.cuda.synchronize()
        got = per.cpu().numpy().astype(np.float64)
        ref = color.delta_e_images(ta.cpu().numpy(), tb.cpu().numpy(), bg)
        err = float(np.abs(got - ref).max())
        print(f"[deltaE] background {bg}: max |gpu - oracle| {err:.2e}; max {summ['max']:.3f} "
              f"mean {summ['mean']:.4f} over 5: {summ['over']}", flush=True)
        assert err <= 1e-5 * max(1.0, float(ref.max()))
        assert got[:1000].max() == 0.0
        assert abs(summ["max"] - ref.max()) <= 1e-5 * ref.max()
        assert abs(summ["mean"] - ref.mean()) <= 1e-9 * max(1.0, ref.mean())
        assert summ["over"] == int((ref > 5.0).sum())

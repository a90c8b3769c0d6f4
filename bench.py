"""Benchmark: Mrays/s at 1920x1080 on the 64-patch cubic bent beam (config 3).

One step = one ivr_render of the view: boundary crossings and blockwise pairing,
RKF45 integration with sampling and compositing, per-pixel merge.  The model is
uploaded once (outside the timed region).  Every pixel counts as a ray.

Prints one JSON line with the metric, the roofline of the dominant kernel
(algorithmic FP32 work per launch from the device counters times per-unit
operation counts, divided by its average HIP-event duration over the timed
steps) and the FP64 oracle timed on the host cores over a bounded pixel sample
(whose parity against the GPU image is reported too).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s at 1080p, RGBA err ≤1e-3 vs FP64 oracle; MLP-seeded vs plain Newton"
PEAK_FP32_TFLOPS = 157.3            # MI355X vector FP32, published (packed FMA)
PEAK_FP32_UNPACKED_TFLOPS = 78.6    # 256 CUs x 64 lanes x 2 flops x 2.4 GHz without packing


COUNTER_PROFILE = os.path.join(ROOT, "profiles", "render_config3_1080p_counters.md")
KERNEL_SOURCES = ["paper_1404_3363_amd/csrc/ivr_kernels.hip", "paper_1404_3363_amd/csrc/ivr_integrate.h",
                  "paper_1404_3363_amd/csrc/ivr_device.h", "paper_1404_3363_amd/csrc/ivr_spline.h",
                  "paper_1404_3363_amd/csrc/ivr_types.h", "paper_1404_3363_amd/csrc/ivr_mlp_dev.h"]


def kernel_sources_sha256():
    """Hash of the kernel sources (in this order): counter profiles record it."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile (FETCH_SIZE
    and WRITE_SIZE passes, scaled by a plain copy), or None if the profile is
    missing or was taken on other kernel sources."""
    try:
        with open(COUNTER_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    src = None
    value = None
    for line in text.splitlines():
        if line.startswith("kernel sources sha256:"):
            src = line.split(":", 1)[1].strip()
        if line.startswith(f"traffic_bytes {kernel}:"):
            value = float(line.split(":", 1)[1])
    return value if (src == kernel_sources_sha256() and value is not None) else None


# Algorithmic work per unit in FP32 flops (FMA = 2, reciprocal and exp 1 each):
# the per-evaluation counts of the method, not of a dense grid, for cubic
# B-spline blocks (the headline model): an evaluation of phi, J_phi and
# W = J^-1 V (three bases with derivatives, the sum-factorised contraction of
# 576 FMA, V = V_par + c V_perp and the 3x3 solve) 1340; rho's value where the
# step is sampled 168; the RK bookkeeping of one attempt 120; one supersampling
# sub-step (interpolation, transfer function, exp, front-to-back update) 40; one
# face Newton iteration (bivariate value and partials, 3x3 solve) 400; one
# box test 20.  Degree 2: 700 / 78 per evaluation; NURBS add the fourth
# homogeneous channel and the quotient rule (1770 for cubic).
UNIT_FLOPS = {
    (3, False): {"w_eval": 1340, "rho": 168},
    (3, True): {"w_eval": 1770, "rho": 200},
    (2, False): {"w_eval": 700, "rho": 78},
    (2, True): {"w_eval": 930, "rho": 95},
}
UNIT_COMMON = {"rk_step": 120, "subsample": 40, "face_iter": 400, "box_test": 20}


def kernel_flops(st, p, rational):
    u = dict(UNIT_FLOPS[(p, rational)], **UNIT_COMMON)
    # rho is sampled once per accepted step (the first stage of the next attempt)
    k2 = (st["w_evals"] * u["w_eval"] + st["samples"] * u["rho"] + st["rk_steps"] * u["rk_step"] +
          st["subsamples"] * u["subsample"])
    k1 = (st["box_tests"] * u["box_test"] + st["face_newton_iter"] * u["face_iter"] +
          st["fp64_polish_iter"] * u["face_iter"] + st["segments"] * (u["w_eval"] + u["rho"]))
    return {"k_fragments": k1, "k_integrate": k2}


def host_cpu():
    """The host's CPU model, logical CPUs and the CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable": usable}


# the CPU share of one GPU on the GPU host (worker pools are limited to it)
CPU_SHARE = 16


def cpu_baseline(sc, cam, gpu_rgba, seconds_target=15.0, seed=7):
    """The oracle in reference mode (the judge of parity) and in method mode (the
    GPU's method in FP64, the like-for-like CPU baseline), each on a bounded
    uniform pixel sample of the same view, on the host's CPU share."""
    import oracle
    rng = np.random.default_rng(seed)
    npx = cam.width * cam.height
    prep = oracle.OracleScene(sc.patches, sc.scale)
    cpu = host_cpu()
    nthreads = max(1, min(cpu["usable"], CPU_SHARE))

    def timed(fn, n0):
        n = n0
        pix = rng.choice(npx, n, replace=False)
        t0 = time.perf_counter()
        out = fn(pix)
        dt = time.perf_counter() - t0
        if dt < seconds_target / 4:
            n = int(min(npx, max(n, n * seconds_target / max(dt, 1e-3))))
            pix = rng.choice(npx, n, replace=False)
            t0 = time.perf_counter()
            out = fn(pix)
            dt = time.perf_counter() - t0
        return pix, out, dt

    pix, ref, dt = timed(lambda px: oracle.render(sc, cam, sc.tf, pixels=px, prepared=prep, nthreads=nthreads), 512)
    err = float(np.abs(gpu_rgba[pix] - ref.rgba).max())
    note = (f"{cpu['model']}, {cpu['nproc']} logical CPUs, {cpu['usable']} usable by this process, "
            f"{nthreads} threads (the CPU share of one GPU)")
    base = {"value": len(pix) / dt / 1e6, "unit": "Mrays/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{len(pix)} uniformly drawn pixels of the same 1920x1080 view, reference mode "
                      f"(converged quadrature of Eq. (volRenderIntegral)), {dt:.1f} s; {note}"}
    mpix, (mimg, msteps), mdt = timed(lambda px: oracle.render_method(sc, cam, sc.tf, pixels=px, prepared=prep,
                                                                        nthreads=nthreads), 4096)
    method = {"value": len(mpix) / mdt / 1e6, "unit": "Mrays/s", "cores": nthreads, "kind": "oracle method mode",
              "sample": f"{len(mpix)} uniformly drawn pixels, the GPU's method in FP64 (adaptive RKF45, "
                        f"same tolerance and step bounds), {mdt:.1f} s, {msteps} RK attempts",
              "max_abs_rgba_vs_gpu": float(np.abs(gpu_rgba[mpix] - mimg).max())}
    return base, method, {"pixels": len(pix), "max_abs_rgba_vs_oracle": err}


def time_renders(r, sc, cam, steps, warmup, **kw):
    """Mrays/s of `steps` timed renders (after `warmup`) and the counters of one more."""
    import torch
    from paper_1404_3363_amd import default_opts
    opts = default_opts(**kw)
    dev = torch.device("cuda", 0)
    rgba = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        r.render(cam, sc.tf, opts=opts, rgba=rgba, depth=depth)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.render(cam, sc.tf, opts=opts, rgba=rgba, depth=depth)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    _, _, st = r.render(cam, sc.tf, opts=opts, rgba=rgba, depth=depth, stats=True)
    torch.cuda.synchronize()
    return cam.width * cam.height * steps / el / 1e6, 1e3 * el / steps, st, rgba


def mlp_vs_plain(r, steps, warmup):
    """Config 4 (256 NURBS blocks, 1920x1080): boundary-root Newton seeded by the
    trained MLP versus the plain element-centre seed (and the box seed, the
    default), same GPU, same image within the parity bar; then the cold starts of
    Sec. "Cutting and Near Clip Planes": with a cutting plane through the model,
    the entries on it are found by Newton from the block centre or from the
    network."""
    from scenes import make_config
    sc = make_config(4)
    cam = sc.cameras[0]
    r.upload(sc.patches)
    rep = r.train_mlp()
    res = {}
    imgs = {}
    for mode in ("plain", "mlp", "box"):
        v, ms, st, rgba = time_renders(r, sc, cam, steps, warmup, seed_mode=mode)
        imgs[mode] = rgba.cpu().numpy().reshape(-1, 4)
        res[mode] = {"value": round(v, 3), "ms_per_step": round(ms, 4),
                     "newton_iter_per_root": round(st["face_newton_iter"] / max(st["face_newton"], 1), 4),
                     "ms_fragments": round(st["ms_fragments"], 4), "mlp_queries": st["mlp_queries"]}
    centre = 0.5 * (sc.bbox[0] + sc.bbox[1])
    cut = (centre, np.array([0.8, -0.2, 0.55]))
    cold = {}
    for mode in ("box", "mlp"):
        v, ms, st, rgba = time_renders(r, sc, cam, steps, warmup, seed_mode=mode, cut_plane=cut)
        cold[mode] = {"value": round(v, 3), "ms_per_step": round(ms, 4), "ms_integrate": round(st["ms_integrate"], 4),
                      "entries_on_plane_seeded_by_network": st["mlp_restarts"], "w_evals": st["w_evals"]}
    return {"workload": "config4: step channel, 256 cubic NURBS patches of 8^3 control points, "
                        "1920x1080 view 0", "unit": "Mrays/s",
            "mlp_training": {"ms_samples": round(rep["ms_samples"], 2), "ms_train": round(rep["ms_train"], 2),
                             "heldout_mean_err": rep["heldout_mean_err"],
                             "heldout_max_err": rep["heldout_max_err"]},
            "plain": res["plain"], "mlp": res["mlp"], "box": res["box"],
            "speedup_mlp_over_plain": round(res["mlp"]["value"] / res["plain"]["value"], 4),
            "max_abs_rgba_mlp_vs_plain": float(np.abs(imgs["mlp"] - imgs["plain"]).max()),
            "cold_start_at_cutting_plane": {"plane": "through the model's centre, normal (0.8, -0.2, 0.55)",
                                            "centre_seed": cold["box"], "mlp_seed": cold["mlp"],
                                            "speedup_mlp_over_centre": round(cold["mlp"]["value"] /
                                                                             cold["box"]["value"], 4)}}


def interior_ab(r, steps, warmup, seed=11):
    """The interior methods on configs 3 and 4 at 1920x1080 with the same step
    bounds: the ray preimage ODE by adaptive RKF45 (the default), root finding
    (every sample's preimage by Newton, Sec. "Root Finding Based Algorithm") and
    the fixed-step methods of the convergence study (explicit RK family and
    implicit Euler, Sec. "ODE Based Algorithm").  Mrays/s, evaluations, Newton
    failures and the largest RGBA error against the oracle on 1024 covered
    pixels."""
    import oracle
    from scenes import make_config
    out = {}
    for k in (3, 4):
        sc = make_config(k)
        cam = sc.cameras[0]
        r.upload(sc.patches)
        row, imgs = {}, {}
        pix = ref = None
        for method in ("ode", "rf", "rk1", "rk2", "rk3", "rk4", "rk4_38", "rkf5", "irk1"):
            v, ms, st, rgba = time_renders(r, sc, cam, steps, warmup, interior=method)
            imgs[method] = rgba.cpu().numpy().reshape(-1, 4).astype(np.float64)
            if pix is None:
                cov = np.flatnonzero(imgs[method][:, 3] > 0)
                pix = np.random.default_rng(seed + k).choice(cov, min(1024, len(cov)), replace=False)
                ref = oracle.render(sc, cam, sc.tf, pixels=pix, nthreads=CPU_SHARE).rgba
            row[method] = {"value": round(v, 3), "ms_per_step": round(ms, 4),
                           "ms_integrate": round(st["ms_integrate"], 4), "w_evals": st["w_evals"],
                           "samples": st["samples"], "newton_failures": st["restart_fail"],
                           "max_abs_rgba_vs_oracle": float(np.abs(imgs[method][pix] - ref).max())}
        row["speedup_rf_over_ode"] = round(row["rf"]["value"] / row["ode"]["value"], 4)
        row["max_abs_rgba_rf_vs_ode"] = float(np.abs(imgs["rf"] - imgs["ode"]).max())
        out[f"config{k}"] = row
    return {"unit": "Mrays/s", **out}


def _field_tf(sc, field, seed=5):
    """The scene's transfer function over the 2nd..98th percentile of a derived
    field at seeded points of every block (by the oracle)."""
    import oracle
    from scenes.configs import TransferFunction
    rng = np.random.default_rng(seed)
    vals = [oracle.field_value(P, p, field) for P in sc.patches
            for p in rng.uniform(0, 1, (max(2, 256 // len(sc.patches)), 3))]
    lo, hi = np.percentile(vals, [2, 98])
    return TransferFunction(sc.tf.x, sc.tf.rgba, sc.tf.extinction, (float(lo), float(hi)))


def extensions(r, steps, warmup, seed=13):
    """The derived fields (Sec. "Parametrization Quality of Geometry", Eq.
    (vonMises)) and the pixel-accuracy tools on config 3 at 1920x1080: Mrays/s and
    the largest RGBA error against the oracle on 512 covered pixels; the largest
    Delta P (Eq. (deltaP)) of the default render and of root finding with the
    frustum Newton stop, its Mrays/s, and its CIEDE2000 against the tolerance stop."""
    import torch
    import oracle
    from scenes import make_config, with_displacement
    base = make_config(3)
    B = np.array([[0.01, 0.004, 0.0], [0.002, -0.006, 0.003], [0.0, 0.001, 0.008]])
    sc = with_displacement(base, B=B, amplitude=0.02 * base.scale)
    cam = sc.cameras[0]
    r.upload(sc.patches)
    out = {"workload": "config3 1920x1080 with a displacement spline (linear part plus a seeded smooth field)",
           "unit": "Mrays/s"}
    for field in ("param_quality", "von_mises"):
        tf = _field_tf(sc, field)
        sc_f = type(sc)(sc.name, sc.patches, tf, sc.cameras, sc.bbox, sc.params)
        v, ms, st, rgba = time_renders(r, sc_f, cam, steps, warmup, field=field, rho_step=0.05)
        img = rgba.cpu().numpy().reshape(-1, 4).astype(np.float64)
        cov = np.flatnonzero(img[:, 3] > 0)
        pix = np.random.default_rng(seed).choice(cov, min(512, len(cov)), replace=False)
        ref = oracle.render(sc_f, cam, tf, pixels=pix, field=field, nthreads=CPU_SHARE)
        out[field] = {"value": round(v, 3), "ms_per_step": round(ms, 4), "rho_step": 0.05,
                      "max_abs_rgba_vs_oracle": float(np.abs(img[pix] - ref.rgba).max())}
    r.upload(base.patches)
    res = {}
    for name, kw in (("ode_default", {}), ("rf_tolerance_stop", {"interior": "rf"}),
                     ("rf_frustum_stop", {"interior": "rf", "newton_stop": "frustum"})):
        outs, st = r.render_batch([(cam, base.tf, 0)], stats=True, pixel_accuracy=True, **kw)
        torch.cuda.synchronize()
        v, ms, _, rgba = time_renders(r, base, cam, steps, warmup, **kw)
        res[name] = {"value": round(v, 3), "max_delta_p": float(outs[0][2].max().item()),
                     "samples_delta_p_over_1": st["dp_over"], "order_violations": st["order_violations"],
                     "w_evals": st["w_evals"], "rgba": outs[0][0]}
    de = r.delta_e2000(res["rf_frustum_stop"]["rgba"], res["rf_tolerance_stop"]["rgba"])
    for v in res.values():
        v.pop("rgba")
    out["pixel_accuracy"] = res
    out["ciede2000_frustum_vs_tolerance_stop"] = {"max": de["max"], "mean": de["mean"], "over_5": de["over"]}
    return out


def batch_views(r, steps, warmup, seed=9):
    """The batched-views workload: the 256-block NURBS channel and the 512-block
    mixed-degree lattice, 32 views with resolutions from {256^2, 512^2, 1024^2,
    1920x1080, 2048^2}, all rendered by one graph replay of the batch (fragment
    launch over all views' tiles, persistent integrator per degree class, merge),
    launch shapes from the autotuner.  Mrays/s over the whole batch, plus the
    oracle on a few covered pixels of every view."""
    import torch
    import oracle
    from scenes import make_config
    a, b, views = make_config(5)
    r.upload_models([a.patches, b.patches])
    vs = [(cam, (a, b)[mi].tf, mi) for mi, cam in views]
    dev = torch.device("cuda", 0)
    outs = [(torch.empty((c.height, c.width, 4), dtype=torch.float32, device=dev),
             torch.empty((c.height, c.width), dtype=torch.float32, device=dev)) for c, _, _ in vs]
    tune = r.autotune(vs, outputs=outs)
    for _ in range(warmup):
        r.render_batch(vs, outputs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.render_batch(vs, outputs=outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rays = sum(c.width * c.height for c, _, _ in vs)
    _, st = r.render_batch(vs, outputs=outs, stats=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    worst, npx = 0.0, 0
    for i, (cam, tf, mi) in enumerate(vs):
        img = outs[i][0].cpu().numpy().reshape(-1, 4).astype(np.float64)
        cov = np.flatnonzero(img[:, 3] > 0)
        pix = rng.choice(cov, min(4, len(cov)), replace=False)
        ref = oracle.render((a, b)[mi], cam, tf, pixels=pix, nthreads=min(16, os.cpu_count() or 1))
        worst = max(worst, float(np.abs(img[pix] - ref.rgba).max()))
        npx += len(pix)
    return {"workload": "batched views: config4 channel (256 cubic NURBS blocks) and a 512-block "
                        "mixed degree-2/3 lattice, 32 views of 256^2..2048^2 in one graph replay",
            "unit": "Mrays/s", "rays_per_batch": rays, "value": round(rays * steps / el / 1e6, 3),
            "ms_per_batch": round(1e3 * el / steps, 3), "steps": steps, "warmup": warmup,
            "segments": st["segments"],
            "counters": {k: st[k] for k in ("samples", "subsamples", "rk_steps", "rk_rejected", "w_evals",
                                            "drift_restarts", "restart_fail", "degenerate", "anomalies")},
            "ms_fragments": round(st["ms_fragments"], 3),
            "ms_integrate": round(st["ms_integrate"], 3), "ms_merge": round(st["ms_merge"], 3),
            "autotune": {k: tune[k] for k in ("tile_w", "tile_h", "xcd_chunk", "int_block",
                                              "int_waves_cu", "ms_before", "ms_after")},
            "parity_sample": {"pixels": npx, "max_abs_rgba_vs_oracle": worst}}


def copy_calibration(nbytes=256 << 20, reps=5):
    """A plain copy of known size: under a counter profile, its FETCH_SIZE and
    WRITE_SIZE per dispatch against nbytes/1024 KiB give the counters' scale."""
    import torch
    dev = torch.device("cuda", 0)
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_kib": nbytes // 1024, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--view", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-ab", action="store_true", help="skip the RF-vs-ODE interior-method comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 5 times (reference "
                         "for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the path shards by image tiles or "
              "views; see DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from scenes import make_config
    from paper_1404_3363_amd import Renderer, default_opts

    sc = make_config(3)
    cam = sc.cameras[args.view]
    r = Renderer(0)
    r.upload(sc.patches)
    dev = torch.device("cuda", 0)
    rgba = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device=dev)
    opts = default_opts()
    for _ in range(args.warmup):
        r.render(cam, sc.tf, opts=opts, rgba=rgba, depth=depth)
    torch.cuda.synchronize()
    r.phase_times()                      # clear
    topts = default_opts(timing=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.render(cam, sc.tf, opts=topts, rgba=rgba, depth=depth)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases = r.phase_times()             # (steps, 3) ms from HIP events on the render stream
    ms_step = 1e3 * elapsed / args.steps
    rays = cam.width * cam.height
    value = rays * args.steps / elapsed / 1e6
    per_render = phases.sum(axis=1)      # fragments + integrator + merge of every timed render

    # counters of one render (deterministic work) -> algorithmic FLOPs per launch
    _, _, st = r.render(cam, sc.tf, opts=opts, rgba=rgba, depth=depth, stats=True)
    torch.cuda.synchronize()
    flops = kernel_flops(st, 3, False)
    avg_ms = {"k_fragments": float(phases[:, 0].mean()), "k_integrate": float(phases[:, 1].mean()),
              "k_merge": float(phases[:, 2].mean())}
    dom = max(("k_fragments", "k_integrate"), key=lambda k: avg_ms[k])
    achieved = flops[dom] / (avg_ms[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "frac_of_unpacked_fp32": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
                "traffic": measured_traffic(dom),
                "avg_ms": {k: round(v, 4) for k, v in avg_ms.items()},
                "algorithmic_gflop_per_launch": {k: round(v / 1e9, 3) for k, v in flops.items()}}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "ms_per_render_events": {"median": round(float(np.median(per_render)), 4),
                                    "p10": round(float(np.percentile(per_render, 10)), 4),
                                    "p90": round(float(np.percentile(per_render, 90)), 4)},
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "config3: bent beam, 64 cubic B-spline patches of 10^3 control "
                                  "points, 3-Gaussian+ramp field, 8-knot transfer function, "
                                  f"1920x1080 view {args.view}",
                      "width": cam.width, "height": cam.height, "patches": len(sc.patches),
                      "rk_tol": opts.rk_tol, "rho_interp": "hermite", "n_super": opts.n_super,
                      "interior": "ode (adaptive RKF45)"},
           "roofline": roofline,
           "device_bytes": r.device_bytes(),
           "counters": {k: st[k] for k in ("segments", "fragments", "anomalies", "rk_steps",
                                           "rk_rejected", "samples", "w_evals", "subsamples",
                                           "face_newton", "face_newton_iter", "fp64_polish_iter",
                                           "box_tests", "drift_restarts")}}
    if not args.no_cpu_baseline:
        img = rgba.cpu().numpy().reshape(-1, 4).astype(np.float64)
        cpu, method, parity = cpu_baseline(sc, cam, img)
        out["cpu_baseline"] = cpu
        out["cpu_baseline_method_mode"] = method
        out["parity_sample"] = parity
    if not args.no_mlp:
        out["mlp_vs_plain"] = mlp_vs_plain(r, args.steps, args.warmup)
    if not args.no_ab:
        out["interior_methods"] = interior_ab(r, args.steps, args.warmup)
        out["extensions"] = extensions(r, args.steps, args.warmup)
    if not args.no_batch:
        out["batch_views"] = batch_views(r, max(args.steps // 4, 3), 2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Benchmark of the MI355X sphere tracer (one JSON line on stdout).

A step is one pass of the whole hot path over one batch: forward render of
8 views x 4 latents = 32 images of 256x256 with the DeepSDF-scale decoder in
bf16 (coarse-to-fine, aggressive marching, compaction, normals), the image
loss (10 L1 depth + silhouette hinge + normal term, on the device), and the
backward pass (the paper's approximate gradient w.r.t. the latent codes).  Inputs are
seeded synthetic decoders, latents and cameras, resident on the GPU before the
timed region.  The same workload is also timed with the float32 plain tracer,
and a single 256x256 image (the float32 workload) is timed for latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp32]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SDF queries/s + 256^2 fwd+bwd frames/s, BF16 vs FP32 plain; serving p99 ms"
# algorithmic work per decoder query of the DeepSDF-scale decoder with the
# latent folded into per-image biases: 1,573,376 multiply-adds
FLOP_PER_QUERY = 2 * 1_573_376
# backward per sample: the recompute (as a query) + the VJP through the hidden
# layers (5 x 512x512 + 2 x 253x512 multiply-adds)
FLOP_VJP = 2 * (5 * 512 * 512 + 2 * 253 * 512)
FLOP_PER_SAMPLE = FLOP_PER_QUERY + FLOP_VJP
# per kernel class of dist_timing_read: algorithmic FLOP per processed row
KERNEL_CLASSES = (("march", FLOP_PER_QUERY), ("eval", FLOP_PER_QUERY), ("adjoint", FLOP_PER_SAMPLE),
                  ("vjp_saved", FLOP_VJP))
PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(n_views=8, n_lat=4, H=256, precision=1):
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs)
    cams = [di.front_camera(H, H)] if n_views == 1 else di.random_sphere_cameras(n_views, H, H)
    Z = torch.tensor(di.make_latents(n_lat, spec.latent_dim, sigma=0.01), device="cuda")
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1,
                         precision=precision, want_normals=1)
    tg = [di.sphere_target_maps(c, 0.5) for c in cams]
    # targets per image (image i = view i // n_lat)
    dt = torch.tensor(np.stack([tg[i // n_lat][0] for i in range(n_views * n_lat)]), device="cuda")
    nt = torch.tensor(np.stack([tg[i // n_lat][1] for i in range(n_views * n_lat)]), device="cuda")
    st = torch.tensor(np.stack([tg[i // n_lat][2] for i in range(n_views * n_lat)]), device="cuda")
    return dict(ctx=ctx, cams=cams, Z=Z, prm=prm, targets=(dt, nt, st), n_img=n_views * n_lat)


def step(w, keep=False):
    """forward + loss + backward; returns (g_z, per-image query tensor) and,
    with keep, the rendered maps."""
    from paper_1911_13225_amd import api
    Z = w["Z"]
    out = api.dist_render_fwd(w["ctx"], w["cams"], Z, w["prm"], save=True)
    dt, nt, st = w["targets"]
    _, gd, gn, gs = api.dist_render_loss(out["depth"], out["normal"], out["sil"], dt, nt, st, w_d=10.0, w_s=1.0,
                                         w_n=1.0)
    g_z = api.dist_render_bwd(w["ctx"], out["saved"], gd, gn, gs, n_latents=Z.shape[0])
    out["saved"].free()
    if keep:
        return g_z, out["queries"], out
    return g_z, out["queries"]


def time_steps(w, steps, warmup):
    import torch
    from paper_1911_13225_amd import api
    for _ in range(warmup):
        step(w)
    torch.cuda.synchronize()
    api.dist_timing_enable(w["ctx"], True)
    torch.cuda.synchronize()
    qs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, q = step(w)
        qs.append(q)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {name: api.dist_timing_read(w["ctx"], k) for k, (name, _) in enumerate(KERNEL_CLASSES)}
    api.dist_timing_enable(w["ctx"], False)
    queries = int(sum(int(q.sum()) for q in qs))
    return dict(sec=t1 - t0, steps=steps, queries=queries, kern=kern)


def kernel_summary(r, dtype):
    """Algorithmic FLOP/s of each kernel class from live HIP-event timing."""
    out = {}
    for name, (launches, ms, rows) in r["kern"].items():
        if launches == 0 or ms <= 0:
            continue
        fl = dict(KERNEL_CLASSES)[name]
        out[name] = dict(launches=launches, ms_total=round(ms, 3), ms_avg=round(ms / launches, 4), rows=rows,
                         tflops=round(rows * fl / (ms * 1e-3) / 1e12, 2))
    return out


# HBM bytes per launch from the committed counter summaries (FETCH_SIZE and
# WRITE_SIZE runs scaled by a copy kernel's reading); valid only while the
# kernel sources are the ones the counters were taken with
TRAFFIC_PROFILES = {"march": "profiles/k_march_bf16_32x256sq_traffic.md"}
KERNEL_SOURCES = ("paper_1911_13225_amd/csrc/mlp_kernels.hip", "paper_1911_13225_amd/csrc/dist_internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    path = TRAFFIC_PROFILES.get(kernel)
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    vals = {}
    with open(os.path.join(ROOT, path)) as fh:
        for line in fh:
            if ":" in line and line.strip().startswith(("bytes_per_launch", "source_sha256")):
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash() or "bytes_per_launch" not in vals:
        return None
    return float(vals["bytes_per_launch"])


def gradient_variants(w, reps=2):
    """dL/dz of the depth and silhouette terms of the benchmark workload by the
    paper's approximation, the implicit-function depth derivative and the exact
    gradient through the unrolled march: time per call and the relative gap of
    each to the unrolled one."""
    import copy
    import torch
    from paper_1911_13225_amd import api
    prm = copy.copy(w["prm"])
    prm.keep_history = 1
    Z = w["Z"]
    out = api.dist_render_fwd(w["ctx"], w["cams"], Z, prm, save=True)
    dt, nt, st = w["targets"]
    _, gd, _, gs = api.dist_render_loss(out["depth"], None, out["sil"], dt, None, st, w_d=10.0, w_s=1.0)
    n = Z.shape[0]
    calls = {
        "paper": lambda: api.dist_render_bwd(w["ctx"], out["saved"], gd, None, gs, n_latents=n),
        "implicit": lambda: api.dist_render_bwd_implicit(w["ctx"], out["saved"], gd, None, gs, n_latents=n),
        "unrolled": lambda: api.dist_render_bwd_unrolled(w["ctx"], out["saved"], gd, gs, n_latents=n),
    }
    res, g = {}, {}
    for name, fn in calls.items():
        g[name] = fn().double()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 2)
    ref = g["unrolled"]
    for name in ("paper", "implicit"):
        res[name + "_rel_gap_to_unrolled"] = round(float((g[name] - ref).norm() / ref.norm()), 4)
    res["loss_terms"] = "10 L1 depth + silhouette (normal terms are not part of the unrolled gradient)"
    out["saved"].free()
    return res


def theta_run(w, reps=2):
    """dL/dtheta of the benchmark's loss on the 32-image bf16 launch: the
    backward with weight gradients (recompute and VJP of every sample row with
    h and Delta captured in bf16, then one GEMM per layer over the rows),
    against the same backward to z alone.  Reports the captured rows and the
    weight-gradient GEMM rate (2 x rows x every layer's weights, a lower bound
    on the work of that call, over its time)."""
    import torch
    from paper_1911_13225_amd import api
    Z = w["Z"]
    out = api.dist_render_fwd(w["ctx"], w["cams"], Z, w["prm"], save=True)
    dt, nt, st = w["targets"]
    _, gd, gn, gs = api.dist_render_loss(out["depth"], out["normal"], out["sil"], dt, nt, st, w_d=10.0, w_s=1.0,
                                         w_n=1.0)
    n = Z.shape[0]
    res = {}
    for name, theta in (("z_only", False), ("with_theta", True)):
        api.dist_render_bwd(w["ctx"], out["saved"], gd, gn, gs, n_latents=n, want_theta=theta)
        torch.cuda.synchronize()
        api.dist_timing_enable(w["ctx"], True)
        t0 = time.perf_counter()
        for _ in range(reps):
            api.dist_render_bwd(w["ctx"], out["saved"], gd, gn, gs, n_latents=n, want_theta=theta)
        torch.cuda.synchronize()
        res[name + "_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 2)
        launches, ms, rows = api.dist_timing_read(w["ctx"], 2)
        if theta:
            res["rows"] = int(rows // max(reps, 1))
            res["recompute_capture_ms"] = round(ms / reps, 2)
            dl, dms, _ = api.dist_timing_read(w["ctx"], 4)
            res["contraction_ms"] = round(dms / reps, 2)
            res["contraction_launches"] = int(dl // reps)
        api.dist_timing_enable(w["ctx"], False)
    out["saved"].free()
    weights = 1_835_520   # multiply-adds of one row through every layer's weights (z and p columns included)
    extra = res["with_theta_ms"] - res["z_only_ms"]
    res["weight_gradient_gflop"] = round(2 * weights * res["rows"] / 1e9, 1)
    res["extra_ms_over_z_only"] = round(extra, 2)
    res["weight_gradient_tflops_over_extra"] = round(2 * weights * res["rows"] / (extra * 1e-3) / 1e12, 1) if extra > 0 else None
    res["contraction_tflops"] = round(2 * weights * res["rows"] / (res["contraction_ms"] * 1e-3) / 1e12, 1) \
        if res["contraction_ms"] > 0 else None
    res["note"] = ("rows = recomputed sample rows (depth/silhouette records and the six stencil queries of every "
                   "hit with a normal seed); the captured h and Delta are bfloat16")
    return res


def color_run(w, reps=3):
    """The colour network (the geometry layout on 512-wide shape + texture
    codes, three outputs) at the hits of the benchmark workload's render:
    time per colour render and per colour backward (bf16)."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.COLOR_SPEC
    Wc, bc = di.make_decoder(spec, seed=7)
    cctx = api.Context.from_spec(spec, Wc, bc)
    zc = torch.tensor(di.make_latents(w["Z"].shape[0], spec.latent_dim, sigma=0.3, base_seed=6000), device="cuda")
    out = api.dist_render_fwd(w["ctx"], w["cams"], w["Z"], w["prm"], save=True)
    hits = int((out["status"] == 1).sum())
    g = torch.randn(out["depth"].shape + (3,), device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    res = {"hits": hits}
    for name, fn in (("render", lambda: api.dist_render_color(cctx, out["saved"], zc, 1)),
                     ("backward", lambda: api.dist_render_color_bwd(cctx, out["saved"], zc, g, 1))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        res[name + "_ms"] = round(ms, 3)
        res[name + "_hit_queries_per_s"] = round(hits / (ms * 1e-3), 1)
    out["saved"].free()
    cctx.close()
    return res


BASELINE_IMAGES = (0, 9, 22, 31)      # images of the benchmark batch the oracle samples (i = view i // 4, latent i % 4)


def cpu_baseline(gpu_maps=None, seconds_target=15.0):
    """The FP64 oracle on a bounded sample of the benchmark workload: rounds of
    2048 random pixels (with their coarse-to-fine ancestors) of four of the 32
    images, forward + normals + loss + backward.  With the GPU's maps of those
    images, also the per-output error of the bf16 launch on the sampled pixels."""
    import dist_inputs as di
    from oracle import dist_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    H = 256
    cams = di.random_sphere_cameras(8, H, H)
    Z = di.make_latents(4, spec.latent_dim, sigma=0.01)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=0,
                         want_normals=1)
    rng = np.random.Generator(np.random.PCG64(77))
    n_pix = 2048
    total_q, total_s, rounds = 0, 0.0, 0
    seen = {i: {} for i in BASELINE_IMAGES}
    while total_s < seconds_target and rounds < 64:
        img = BASELINE_IMAGES[rounds % len(BASELINE_IMAGES)]
        v, l = img // 4, img % 4
        pix = rng.choice(H * H, n_pix, replace=False)
        t0 = time.perf_counter()
        r = O.render(dec, Z, cams, [(v, l)], prm, pixels=[pix])[0]
        dt, nt, st = di.sphere_target_maps(cams[v], 0.5)
        _, g_d, g_n, g_s = O.loss_and_grads(r, dt, nt, st, w_d=10.0, w_s=1.0, w_n=1.0)
        O.backward(dec, Z, [r], [(v, l)], prm, [(g_d, g_n, g_s)], want_theta=False)
        total_s += time.perf_counter() - t0
        total_q += r.queries
        rounds += 1
        for q in pix:
            seen[img][int(q)] = (r.status.reshape(-1)[q], r.depth.reshape(-1)[q], r.sil.reshape(-1)[q],
                                 r.normal.reshape(-1, 3)[q], r.dirs[q], float(np.linalg.norm(r.nraw.reshape(-1, 3)[q])))
    out = {"value": round(total_q / total_s, 1), "unit": "queries/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{rounds} x {n_pix} random pixels of images {list(BASELINE_IMAGES)} of the 32-image "
                     f"workload (with their coarse-to-fine ancestors), FP64 fwd + normals + loss + backward; "
                     f"{total_q} march queries in {total_s:.1f} s"}
    if gpu_maps is not None:
        out["error_vs_oracle"] = per_output_error(seen, gpu_maps)
    return out


def per_output_error(seen, gpu_maps):
    """Per-output error of the GPU's bf16 maps against the oracle on the pixels
    the oracle traced: depth over pixels that are foreground in both (all of
    them, and the well-conditioned ones with |cos(ray, normal)| >= 0.25),
    normals on the well-conditioned ones (unit normals, and as the tests bound
    them: the unit-normal difference times the length of the central-difference
    gradient, which normalising would otherwise amplify where that length is
    small), binary silhouette mismatch over all sampled pixels."""
    dd, dd_wc, dn_wc, dg_wc, n_pix, mis = [], [], [], [], 0, 0
    for img, px in seen.items():
        g = gpu_maps[img]
        for q, (st, dep, sil, nrm, dvec, glen) in px.items():
            n_pix += 1
            mis += int((sil < 0) != (g["sil"][q] < 0))
            if st == 1 and g["status"][q] == 1:
                e = abs(float(dep) - float(g["depth"][q]))
                dd.append(e)
                if abs(float(np.dot(dvec, nrm))) >= 0.25:
                    dd_wc.append(e)
                    dn_wc.append(float(np.linalg.norm(nrm - g["normal"][q])))
                    dg_wc.append(dn_wc[-1] * glen)
    dd = np.array(dd)
    res = {"pixels": n_pix, "hits_both": int(dd.size), "silhouette_mismatch_frac": round(mis / max(n_pix, 1), 6),
           "tolerance": {"depth": 2e-3, "silhouette_mismatch_frac": 1e-3, "normal_x_grad_len": 2e-3}}
    if dd.size:
        res["depth_all_hits"] = {"max": float(dd.max()), "p99_9": float(np.percentile(dd, 99.9)),
                                 "frac_above_2e-3": round(float((dd > 2e-3).mean()), 6)}
        res["depth_well_conditioned"] = {"n": len(dd_wc), "max": float(max(dd_wc)) if dd_wc else None}
        res["normal_well_conditioned_max"] = float(max(dn_wc)) if dn_wc else None
        res["normal_x_grad_len_well_conditioned_max"] = float(max(dg_wc)) if dg_wc else None
    return res


def strategy_ablation(sizes=(256, 512), reps=3):
    """The paper's runtime ablation (Table 1) on a seeded single view: decoder
    queries and fwd + loss + bwd time per frame (bf16) for dynamic
    synchronized inference, + aggressive marching, + coarse-to-fine, and
    coarse-to-fine with 100 steps; "parallel" (no culling of finished rays)
    would query every ray that meets the unit sphere at every step."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs)
    Z = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.01), device="cuda")
    variants = (("dynamic", 1.0, 0, 50), ("+aggressive", 1.5, 0, 50), ("+coarse_to_fine", 1.5, 2, 50),
                ("+coarse_to_fine_100_steps", 1.5, 2, 100))
    out = {}
    for H in sizes:
        cam = di.front_camera(H, H)
        dt, nt, st = (torch.tensor(x, device="cuda")[None] for x in di.sphere_target_maps(cam, 0.5))
        rows = {}
        for name, alpha, c2f, steps in variants:
            prm = di.TraceParams(alpha=alpha, eps=5e-4, max_steps=steps, c2f_levels=c2f, k_samples=1,
                                 precision=1, want_normals=1)

            def one():
                o = api.dist_render_fwd(ctx, [cam], Z, prm, save=True)
                _, gd, gn, gs = api.dist_render_loss(o["depth"], o["normal"], o["sil"], dt, nt, st, w_d=10.0,
                                                     w_s=1.0, w_n=1.0)
                api.dist_render_bwd(ctx, o["saved"], gd, gn, gs, n_latents=1)
                o["saved"].free()
                return o
            o = one()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                one()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            rows[name] = {"alpha": alpha, "c2f_levels": c2f, "max_steps": steps,
                          "queries": int(o["queries"].sum()), "hits": int((o["status"] == 1).sum()),
                          "fwd_bwd_ms": round(ms, 3)}
            if name == "dynamic":
                rows["parallel_queries"] = int((o["status"] != 2).sum()) * steps
        out[f"{H}x{H}"] = rows
    ctx.close()
    return out


def serving_run(rate=10.0, n_req=24, zopt_iters=50, seed=4000):
    """Poisson stream of mixed requests through dist_submit/dist_poll."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api, _native as N
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs, hbm_budget=64 << 30)
    stream = di.poisson_requests(rate, n_req, seed=seed)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=1,
                         want_normals=1)
    reqs = []
    for q in stream:
        cams = di.random_sphere_cameras(q["n_views"], q["res"], q["res"], base_seed=q["latent_seed"])
        z = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.01, base_seed=q["latent_seed"])[0],
                         device="cuda")
        if q["kind"] == "zopt":
            tg = [di.sphere_target_maps(c, 0.5) for c in cams]
            td = torch.tensor(np.stack([np.where(np.isfinite(t[0]), t[0], 0.0) for t in tg]), device="cuda")
            ts = torch.tensor(np.stack([t[2] for t in tg]), device="cuda")
            r = api.ServeRequest(N.REQ_ZOPT, cams, z, prm, want_normals=False, targets=(td, ts),
                                 iters=zopt_iters, lr=1e-2)
        else:
            r = api.ServeRequest(N.REQ_RENDER, cams, z, prm, want_normals=True)
        reqs.append((q, r))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, r in reqs:
        delay = q["t_arrive"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        api.dist_submit(ctx, r)
    lat = {"render": [], "zopt": []}
    queries = 0
    for q, r in reqs:
        res = api.dist_poll(ctx, r, 600_000_000)
        assert res is not None and res["status"] == 0, res
        lat[q["kind"]].append(res["latency_ms"])
        queries += res["queries"]
    wall = time.perf_counter() - t0
    ctx.close()
    allv = np.array(lat["render"] + lat["zopt"])
    out = {"rate_req_per_s": rate, "requests": n_req, "completed_req_per_s": round(n_req / wall, 2),
           "march_queries_per_s": round(queries / wall, 1), "p50_ms": round(float(np.percentile(allv, 50)), 2),
           "p99_ms": round(float(np.percentile(allv, 99)), 2), "wall_s": round(wall, 2),
           "mix": f"resolution uniform over {{64,128,256,512}}^2, 1-8 views, 10% z-opt jobs of {zopt_iters} "
                  "Adam iterations; bf16; 64 GB admission budget"}
    for k, v in lat.items():
        if v:
            out[k] = {"n": len(v), "p50_ms": round(float(np.percentile(v, 50)), 2),
                      "p99_ms": round(float(np.percentile(v, 99)), 2)}
    return out


def kernel_micro(n=1 << 21):
    """One decoder launch over n random points per precision (no march tail)."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs)
    g = torch.Generator(device="cuda").manual_seed(0)
    P = (torch.rand(n, 3, device="cuda", generator=g) - 0.5) * 1.2
    lat = torch.zeros(n, dtype=torch.int32, device="cuda")
    Z = torch.zeros(1, spec.latent_dim, device="cuda")
    out = {}
    for prec, name, peak in ((1, "bf16", PEAK["bf16"]), (2, "split_bf16", PEAK["bf16"] / 3), (0, "fp32", PEAK["fp32"])):
        for _ in range(2):
            api.dist_sdf_eval(ctx, P, lat, Z, prec)
        torch.cuda.synchronize()
        api.dist_timing_enable(ctx, True)
        reps = 3
        for _ in range(reps):
            api.dist_sdf_eval(ctx, P, lat, Z, prec)
        launches, ms, rows = api.dist_timing_read(ctx, 1)
        api.dist_timing_enable(ctx, False)
        tf = n * launches * FLOP_PER_QUERY / (ms * 1e-3) / 1e12
        out[name] = {"points": n, "ms": round(ms / launches, 3), "tflops": round(tf, 1),
                     "frac_of_peak": round(tf * 1e12 / peak, 4)}
    ctx.close()
    return out


def zopt_run(iters=200, n_views=4, H=256, precision=1):
    """Latent-code fitting: Adam (lr 1e-2) on z from N(0, 0.01^2) towards
    depth/silhouette maps rendered from z* ~ N(0, 0.1^2); 10 L1 + silhouette."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs)
    cams = di.random_sphere_cameras(n_views, H, H)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=precision,
                         want_normals=0)
    zs = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.1, base_seed=3000), device="cuda")
    tgt = api.dist_render_fwd(ctx, cams, zs, prm)
    dt = torch.where(torch.isfinite(tgt["depth"]), tgt["depth"], torch.zeros_like(tgt["depth"]))
    st = (tgt["sil"] < 0).float()
    nz = torch.zeros(dt.shape + (3,), device="cuda")
    z = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.01, base_seed=1000), device="cuda")
    d0 = float((z - zs).norm())
    m = torch.zeros_like(z)
    v = torch.zeros_like(z)
    checks = (0, 1, 10, 50, 100, iters - 1)
    curve, image = {}, {}

    def image_fit(o):
        # the fit in image space: mean |depth error| where both are foreground,
        # and the intersection over union of the two silhouettes
        fr, ft = o["sil"] < 0, st > 0.5
        both = fr & ft
        derr = float((o["depth"] - dt).abs()[both].mean()) if bool(both.any()) else None
        iou = float(both.sum()) / max(float((fr | ft).sum()), 1.0)
        return {"depth_abs_err_fg": round(derr, 6) if derr is not None else None, "silhouette_iou": round(iou, 5)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        out = api.dist_render_fwd(ctx, cams, z, prm, save=True)
        loss, gd, _, gs = api.dist_render_loss(out["depth"], None, out["sil"], dt, None, st, w_d=10.0, w_s=1.0)
        g = api.dist_render_bwd(ctx, out["saved"], gd, None, gs, n_latents=1)
        out["saved"].free()
        if it in checks:
            curve[it] = round(float(loss.sum()), 6)
            image[it] = image_fit(out)
            image[it]["z_dist_rel"] = round(float((z - zs).norm()) / d0, 4)
        api.dist_adam_step(z, m, v, g, it + 1, lr=1e-2)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out = api.dist_render_fwd(ctx, cams, z, prm)
    final = image_fit(out)
    ctx.close()
    return {"iters": iters, "views": n_views, "resolution": H, "precision": "bf16" if precision else "fp32",
            "its_per_s": round(iters / sec, 2), "loss": curve, "image_space": image, "final": final,
            "z_dist_rel": {"start": 1.0, "end": round(float((z - zs).norm()) / d0, 4)},
            "note": "a random decoder's latent is not identifiable from four depth maps: the fit converges in "
                    "image space (depth error, silhouette IoU) while z wanders; Adam at a fixed lr 1e-2 "
                    "oscillates near the fit (App. B.4 schedule)"}


def photometric_run(iters=50, n_views=8, H=112, precision=1):
    """Multi-view reconstruction from colour images alone: the photometric
    loss (weight 5, each view warped to the next of a ring of 8 at 112x112,
    the paper's synthetic setting) between the rendered depth of z and
    procedurally textured images of a radius-0.45 sphere; Adam (lr 1e-2) on z
    from N(0, 0.01^2) with the paper's gradient."""
    import torch
    import dist_inputs as di
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    ctx = api.Context.from_spec(spec, Ws, bs)
    cams = di.ring_cameras(n_views, H, H)
    images = torch.tensor(di.textured_sphere_images(cams, 0.45, freq=4.0), device="cuda")
    pairs = [(i, (i + 1) % n_views) for i in range(n_views)]
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=0, k_samples=1, precision=precision,
                         want_normals=0)
    z = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.01, base_seed=1000), device="cuda")
    m = torch.zeros_like(z)
    v = torch.zeros_like(z)
    curve = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        out = api.dist_render_fwd(ctx, cams, z, prm, save=True)
        loss, g_depth = api.dist_photometric_loss(cams, out["depth"], images, pairs, weight=5.0)
        g = api.dist_render_bwd(ctx, out["saved"], g_depth, None, None, n_latents=1)
        out["saved"].free()
        api.dist_adam_step(z, m, v, g, it + 1, lr=1e-2)
        if it in (0, 1, 10, 25, iters - 1):
            curve[it] = round(float(loss.item()), 6)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ctx.close()
    return {"iters": iters, "views": n_views, "resolution": H, "precision": "bf16" if precision else "fp32",
            "its_per_s": round(iters / sec, 2), "loss": curve,
            "data": "ring of views of a procedurally textured radius-0.45 sphere (synthetic)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100, help="requests per rate of the serving sweep")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--no-zopt", action="store_true")
    ap.add_argument("--serve-sweep", type=str, default="10,20,50,100,200,500",
                    help="comma-separated Poisson request rates (req/s), --serve-requests each")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-grad-variants", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (reference dispatch for HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: the tracer has no multi-GPU path (requested --gpus {a.gpus}); "
              "images and requests are independent and would shard by image across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)

    if a.copy_calibration:
        # 1 GiB read + 1 GiB written by one copy dispatch: the counters' reading
        # for it scales FETCH_SIZE / WRITE_SIZE of the decoder kernels to bytes
        src = torch.empty(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration done")

    micro = None
    if not a.no_micro:
        log("[bench] decoder kernel alone")
        micro = kernel_micro()
        log("[bench] micro", micro)

    log("[bench] bf16 32-image workload")
    w = build_workload(precision=1)
    r = time_steps(w, a.steps, a.warmup)
    ms_step = 1e3 * r["sec"] / r["steps"]
    qps = r["queries"] / r["sec"]
    fps = w["n_img"] * r["steps"] / r["sec"]
    ks = kernel_summary(r, "bf16")
    log("[bench] bf16", round(ms_step, 2), "ms/step", ks)
    # the maps of the images the oracle samples for the per-output error report
    _, _, maps = step(w, keep=True)
    gpu_maps = {i: {k: maps[k][i].reshape(-1, 3).cpu().numpy() if k == "normal" else maps[k][i].reshape(-1).cpu().numpy()
                    for k in ("depth", "sil", "status", "normal")} for i in BASELINE_IMAGES}
    del maps

    res = {"metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "8 views x 4 latents = 32 images of 256x256 per step, DeepSDF 8x512 decoder "
                                  "(Kaiming seed 0), alpha 1.5, eps 5e-4, 50 steps, coarse-to-fine from 64x64, "
                                  "K=1, normals, loss 10 L1 + silhouette + normal, backward to z",
                      "global_batch": w["n_img"], "resolution": 256, "precision": "bf16"},
           "frames_per_s": round(fps, 2), "queries_per_step": r["queries"] // r["steps"], "kernels": ks,
           "decoder_kernel_alone": micro}
    # roofline of the dominant kernel (by measured time)
    dom = max(ks.items(), key=lambda kv: kv[1]["ms_total"])
    name, k = dom
    achieved = k["tflops"]
    res["roofline"] = {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": PEAK["bf16"] / 1e12,
                       "unit": "TFLOP/s", "frac": round(achieved / (PEAK["bf16"] / 1e12), 4),
                       "traffic": measured_traffic(name)}
    if not a.no_grad_variants:
        log("[bench] gradient variants on the same workload")
        res["gradient_variants"] = gradient_variants(w)
        log("[bench] gradient variants", res["gradient_variants"])
        log("[bench] weight gradient on the same workload")
        res["weight_gradient"] = theta_run(w)
        log("[bench] weight gradient", res["weight_gradient"])
        log("[bench] colour network at the hits of the same workload")
        res["color"] = color_run(w)
        log("[bench] colour", res["color"])
    w["ctx"].close()
    del w
    torch.cuda.empty_cache()

    if not a.no_fp32:
        log("[bench] fp32 plain 32-image workload")
        w = build_workload(precision=0)
        r2 = time_steps(w, max(1, a.steps // 5), 1)
        q2 = r2["queries"] / r2["sec"]
        ks2 = kernel_summary(r2, "fp32")
        res["fp32_plain"] = {"queries_per_s": round(q2, 1), "frames_per_s": round(w["n_img"] * r2["steps"] / r2["sec"], 2),
                             "ms_per_step": round(1e3 * r2["sec"] / r2["steps"], 2), "kernels": ks2,
                             "march_frac_of_fp32_peak": round(ks2["march"]["tflops"] / (PEAK["fp32"] / 1e12), 4)
                             if "march" in ks2 else None}
        res["speedup_bf16_vs_fp32"] = round(qps / q2, 2)
        w["ctx"].close()
        del w
        torch.cuda.empty_cache()
        log("[bench] single 256x256 image, fp32 and bf16")
        single = {}
        for prec, nm in ((0, "fp32"), (1, "bf16")):
            w = build_workload(n_views=1, n_lat=1, precision=prec)
            r3 = time_steps(w, 3, 1)
            single[nm] = {"ms_per_frame": round(1e3 * r3["sec"] / r3["steps"], 2),
                          "queries_per_s": round(r3["queries"] / r3["sec"], 1)}
            w["ctx"].close()
            del w
        res["single_image"] = single

    if not a.no_zopt:
        log("[bench] latent fit, 4 views 256x256, 200 Adam iterations")
        res["latent_fit"] = zopt_run()
        log("[bench] latent fit", res["latent_fit"])

    if not a.no_zopt:
        log("[bench] multi-view photometric fit, 8 views 112x112, 50 Adam iterations")
        res["photometric_fit"] = photometric_run()
        log("[bench] photometric fit", res["photometric_fit"])

    if not a.no_ablation:
        log("[bench] strategy ablation (Table 1 analogue), single view 256x256 and 512x512")
        res["strategy_ablation"] = strategy_ablation()
        log("[bench] ablation", res["strategy_ablation"])

    if not a.no_serve and a.serve_sweep:
        res["serving"] = []
        for rate in [float(x) for x in a.serve_sweep.split(",") if x]:
            log("[bench] serving sweep at", rate, "req/s,", a.serve_requests, "requests")
            res["serving"].append(serving_run(rate, a.serve_requests))
            log("[bench]  ", res["serving"][-1])

    if not a.no_cpu:
        log("[bench] cpu baseline (oracle) and per-output error of the bf16 launch on its pixels")
        res["cpu_baseline"] = cpu_baseline(gpu_maps)
    # every context was closed explicitly where its workload ended (its
    # serving thread joined, its memory freed) while the HIP runtime is up, so
    # the interpreter's teardown finds nothing of the library left to release
    import gc
    gc.collect()
    torch.cuda.synchronize()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

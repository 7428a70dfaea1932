#!/usr/bin/env python3
"""Benchmark of the uplift hot path on one MI355X.

Workload (the mid configuration): 200,000 Gaussians (centres U[-1,1]^3,
scales exp(N(-4, 0.5^2)), uniform rotations, opacities sigmoid(N(0,1))), 50
Fibonacci-sphere cameras at radius 4, 512x384 px, 55 deg horizontal FoV; two
feature sets per view: D = 64 FP32 maps (N(0,1) at 1/14 resolution, bilinearly
upsampled) and a D = 1 ellipse mask.  Inputs are generated before timing and
are resident in HBM.

One step = the whole job on that workload: make the scene resident
(lv_scene_create), uplift the D = 64 maps and the D = 1 masks of all 50 views
(lv_uplift, FP32), release the scene.  value = ms per (view x channel) over
the 50 x 65 view-channels of a step.

Also reported, measured in the same run outside the timed steps:
  roofline      the blend-and-accumulate kernel of the D = 64 uplift, timed with
                HIP events around each launch during the timed steps;
  bf16          BF16 storage of the D = 64 maps (encode + uplift) and its error
                against the FP32 result;
  filtering     pruning by weight sum and the count-normalised finalize;
  render        the forward render (Eq. 4) of the uplifted D = 64 features into
                all 50 views, with opacity;
  diffuse       100 steps of Eq. (8) on a 16-NN graph of the scene (D = 1 and 64),
                the graph build, and the segmentation diffusion (Eq. 7 / 9);
  serving       a synthetic request trace through the server;
  cpu_baseline  the FP64 oracle on a sample of the same workload, host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "uplift ms/view/channel + % HBM roofline, BF16 vs FP32 @ tol; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# FP32 FMA on the vector ALUs without packed-FP32 instructions:
# 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
ALU_PEAK_PACKED_TFLOPS = 157.3
# Device-scope atomic updates in the L2: one 4-byte update per L2 channel per
# clock, 8 XCDs x 16 channels x 2.4 GHz
ATOMIC_PEAK_GPS = 307.2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-views", type=int, default=6,
                    help="views of the workload the CPU-baseline oracle runs (0 = skip)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM traffic counters)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the serving trace (0 = skip the serving leg)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, req/s")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_14462_amd as lv
    from synth import scenes

    torch.cuda.set_device(0)
    w = scenes.WORKLOADS["mid"]
    n, m, H, W, D = w.n, w.m, w.height, w.width, w.D
    log(f"bench: {w.name}: generating inputs")
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    means, scales, quats, opac = dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacity)
    maps = [scenes.feature_map(w, v, device="cuda") for v in range(m)]
    masks = [dev(scenes.ellipse_mask(w.seed, v, H, W)) for v in range(m)]
    f64 = torch.empty((n, D), device="cuda")
    b64 = torch.empty((n,), device="cuda")
    f1 = torch.empty((n, 1), device="cuda")
    b1 = torch.empty((n,), device="cuda")
    torch.cuda.synchronize()

    # the rig and the two map lists marshalled once (pointer tables), as a
    # C caller would hold them
    rig, tab64, tab1 = lv.Cameras(cams), lv.Maps(maps), lv.Maps(masks)

    def step():
        s = lv.Scene(means, scales, quats, opac)
        s.uplift_sets(rig, [tab64, tab1], outs=[(f64, b64), (f1, b1)])
        s.close()

    # work statistics (untimed pass with counters)
    s = lv.Scene(means, scales, quats, opac)
    acc, accm = lv.Accum(s, D, counts=True), lv.Accum(s, 1, counts=True)
    lv.accumulate_sets(cams, [(acc, maps), (accm, masks)])
    st64 = acc.stats()
    acc.close()
    accm.close()
    s.close()
    log(f"bench: stats {st64}")

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    lv.profile_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        step()
        ev[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches = lv.profile_stop()
    lat = [a.elapsed_time(b) for a, b in ev]
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = ms_step / (m * (D + 1))
    log(f"bench: {ms_step:.3f} ms/step, {value * 1e3:.4f} us/view/channel")

    # the blend launch of a step serves both feature sets (65 channels)
    t64 = sum(launches) / len(launches) * 1e-3
    C = D + 1
    bytes64 = (st64["covered_pixels"] * C * 4 + st64["visible"] * 32 + st64["pairs"] * 4
               + n * (C + 4) * 4)
    flops64 = 2.0 * st64["contributions"] * (C + 2)
    hbm_gbs = bytes64 / t64 / 1e9
    alu_tflops = flops64 / t64 / 1e12
    t_hbm, t_alu = bytes64 / (HBM_PEAK_GBS * 1e9), flops64 / (ALU_PEAK_TFLOPS * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(alu_tflops, 3), "peak": ALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu_tflops / ALU_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    roof.update({
        "traffic": measured_traffic(),
        "kernel": "blend_wide_kernel<LV_F32> (D=64 maps + D=1 mask, 50 views per launch)",
        "launch_ms": round(t64 * 1e3, 4),
        "hbm": {"achieved_GBs": round(hbm_gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "alg_bytes": int(bytes64)},
        "alu": {"achieved_TFLOPs": round(alu_tflops, 3), "peak_TFLOPs": ALU_PEAK_TFLOPS,
                "frac": round(alu_tflops / ALU_PEAK_TFLOPS, 4),
                "frac_of_packed_peak": round(alu_tflops / ALU_PEAK_PACKED_TFLOPS, 4),
                "alg_flops": flops64},
    })
    # the resource that binds this kernel: one atomic update per channel and
    # one for beta per (Gaussian, view, 8x8 block) partial sum
    if st64.get("partial_sums", -1) > 0:
        upd = st64["partial_sums"] * (C + 1)
        roof["l2_atomics"] = {"achieved_Gps": round(upd / t64 / 1e9, 1), "peak_Gps": ATOMIC_PEAK_GPS,
                              "frac": round(upd / t64 / 1e9 / ATOMIC_PEAK_GPS, 4),
                              "updates": int(upd), "partial_sums": int(st64["partial_sums"])}

    out = {
        "metric": METRIC,
        "value": round(value, 7),
        "unit": "ms/view/channel",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "gaussians": n, "views": m, "width": W, "height": H,
                   "channels": [D, 1], "map_dtype": "f32"},
        "latency_ms": {"p50": round(percentile(lat, 0.5), 4), "p99": round(percentile(lat, 0.99), 4)},
        "contributions_per_s": round(st64["contributions"] / t64, 1),
        "work": st64,
        "roofline": roof,
    }

    if args.calib_copy:
        src = torch.empty(1 << 28, device="cuda", dtype=torch.float32).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
        del src, dst

    if not args.no_extras:
        out.update(extras(lv, w, sc, cams, maps, f64, b64, f1, means, scales, quats, opac))

    if args.serve_requests > 0:
        del maps, masks, f64, b64, f1, b1
        torch.cuda.empty_cache()
        out["serving"] = serving(lv, args.serve_requests, args.serve_rate)
        maps = [scenes.feature_map(w, v, device="cuda") for v in range(args.cpu_views)]
        masks = [dev(scenes.ellipse_mask(w.seed, v, H, W)) for v in range(args.cpu_views)]

    if args.cpu_views > 0:
        out["cpu_baseline"] = cpu_baseline(w, sc, cams, maps, masks, args.cpu_views)
        out["cpu_baseline"]["gpu_over_cpu"] = round(out["cpu_baseline"]["value"] / value, 1)

    print(json.dumps(out), flush=True)


def measured_traffic():
    """HBM bytes per D=64 blend launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "uplift-200k-50v-512x384-D64+mask_blend_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2410_14462_amd", "csrc")
    src = open(os.path.join(csrc, "blend.hip"), "rb").read() + \
        open(os.path.join(csrc, "lv_internal.h"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return int(rec["traffic_bytes"])


def extras(lv, w, sc, cams, maps, f64, b64, f1, means, scales, quats, opac):
    import numpy as np
    import torch

    res = {}
    n, m, D = w.n, w.m, w.D
    s = lv.Scene(means, scales, quats, opac)
    # ---- BF16 storage (codec + uplift) against the FP32 result
    log("bench: bf16 leg")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    enc = [lv.encode(mp, "bf16")[0] for mp in maps]
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - t0
    # the codec kernel itself: one call over all 50 maps stacked (the wall
    # time above is mostly the per-call marshalling of 50 separate maps)
    stacked = torch.stack(maps)
    lv.encode(stacked, "bf16")  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        lv.encode(stacked, "bf16")
    e1.record()
    torch.cuda.synchronize()
    t_enc_gpu = e0.elapsed_time(e1) * 1e-3 / 3
    enc_bytes = stacked.numel() * (4 + 2)
    del stacked
    fb = torch.empty((n, D), device="cuda")
    bb = torch.empty((n,), device="cuda")
    s.uplift(cams, enc, dtype="bf16", out=fb, wsum=bb)  # warm
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.uplift(cams, enc, dtype="bf16", out=fb, wsum=bb)
    torch.cuda.synchronize()
    t_bf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        s.uplift(cams, maps, out=f64, wsum=b64)
    torch.cuda.synchronize()
    t_f32 = (time.perf_counter() - t0) / reps
    # error scale a = uplift of |F| (sum w |F| / beta)
    absmaps = [mp.abs() for mp in maps]
    fa, _ = s.uplift(cams, absmaps)
    seen = b64 > 0
    err = ((fb - f64).abs() / fa.clamp_min(1e-30))[seen]
    res["bf16"] = {
        "encode_ms": round(t_enc * 1e3, 3),
        "encode_stacked_ms": round(t_enc_gpu * 1e3, 3),
        "encode_GBs": round(enc_bytes / t_enc_gpu / 1e9, 1),
        "uplift_ms": round(t_bf * 1e3, 3),
        "uplift_ms_f32": round(t_f32 * 1e3, 3),
        "ms_per_view_channel": round(t_bf * 1e3 / (m * D), 7),
        "ms_per_view_channel_f32": round(t_f32 * 1e3 / (m * D), 7),
        "err_vs_f32": {"max": float(err.max()), "p99": float(torch.quantile(err[:1000000], 0.99)),
                       "mean": float(err.mean()), "bound": 2.0 ** -8 + 1e-4},
    }
    del enc, absmaps
    # ---- weight-based filtering (keep the half with the largest beta) and
    # the count-normalised finalize
    log("bench: filtering leg")
    k = n // 2
    keep = lv.prune_by_weight(b64, k)
    reps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        keep = lv.prune_by_weight(b64, k)
    torch.cuda.synchronize()
    t_prune = (time.perf_counter() - t0) / reps
    acc = lv.Accum(s, D, counts=True)
    acc.add(cams, maps)
    fc = acc.finalize_count()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fc = acc.finalize_count()
    torch.cuda.synchronize()
    t_fc = (time.perf_counter() - t0) / reps
    res["filtering"] = {"n": n, "kept": int(keep.sum()), "prune_ms": round(t_prune * 1e3, 4),
                        "finalize_count_ms": round(t_fc * 1e3, 4)}
    del acc, fc, keep
    # ---- forward render (Eq. 4) of the uplifted D=64 features into all views
    log("bench: render leg")
    outs, alps = s.render(cams, f64)  # warm (and output allocation)
    del outs, alps
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        outs, alps = s.render(cams, f64)
    torch.cuda.synchronize()
    t_r = (time.perf_counter() - t0) / reps
    H, W = w.height, w.width
    out_bytes = m * H * W * (D + 1) * 4  # rendered features and opacity, written once
    res["render"] = {"ms": round(t_r * 1e3, 3), "ms_per_view_channel": round(t_r * 1e3 / (m * D), 7),
                     "output_GB": round(out_bytes / 1e9, 3),
                     "output_GBs": round(out_bytes / t_r / 1e9, 1),
                     "hbm_frac_of_output_bytes": round(out_bytes / t_r / 1e9 / HBM_PEAK_GBS, 4)}
    del outs, alps
    # ---- diffusion over the 16-NN graph of the scene, built on the device
    # from the uplifted features
    log("bench: diffusion leg (16-NN graph built on the device)")
    G = lv.Graph.knn(s, f64, 16)
    G.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = lv.Graph.knn(s, f64, 16)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    nnz = int(G.csr()[1].shape[0])
    dres = {"graph_nnz": nnz, "graph_build_ms": round(t_graph * 1e3, 3), "steps": 100}
    # with the scene: rows in the Morton order of the centres (built on the
    # first call); without: the caller's order
    for name, g0, scene in (("D1", f1.contiguous(), s), ("D64", f64, s),
                            ("D64_caller_order", f64, None)):
        out = G.diffuse(g0, 100, scene=scene)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = G.diffuse(g0, 100, scene=scene, out=out)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / 100
        Dg = g0.shape[1]
        byts = 4 * (n + 1) + nnz * 8 + 2 * n * Dg * 4
        dres[name] = {"ms_per_step": round(t * 1e3, 4), "GBs": round(byts / t / 1e9, 1),
                      "hbm_frac": round(byts / t / 1e9 / HBM_PEAK_GBS, 4)}
    G.close()
    # the paper's segmentation diffusion: binarised Eq. 7 / Eq. 9 graph with a
    # unary term, anchors from the uplifted mask, 10 steps, reached nodes
    log("bench: segmentation diffusion (Eq. 7 / Eq. 9 graph)")
    unary = torch.rand(n, device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    kw = dict(kind="feature_rbf", bandwidth=0.5, unary=unary, binarize=1e-5)
    Gs = lv.Graph.knn(s, f64, 16, **kw)
    Gs.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Gs = lv.Graph.knn(s, f64, 16, **kw)
    torch.cuda.synchronize()
    t_sg = time.perf_counter() - t0
    g0 = lv.anchor_init(f1.reshape(-1).contiguous(), 0.1)
    gT = Gs.diffuse(g0, 10, scene=s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g0 = lv.anchor_init(f1.reshape(-1).contiguous(), 0.1)
    gT = Gs.diffuse(g0, 10, scene=s, out=gT)
    h = lv.reach_unary(gT, unary)
    torch.cuda.synchronize()
    t_seg = time.perf_counter() - t0
    dres["segmentation"] = {"graph_build_ms": round(t_sg * 1e3, 3), "graph_nnz": int(Gs.csr()[1].shape[0]),
                            "anchors": int((g0 > 0).sum()), "steps": 10,
                            "anchors_diffuse_reach_ms": round(t_seg * 1e3, 3),
                            "reached": int((h > 0).sum())}
    Gs.close()
    res["diffuse"] = dres
    s.close()
    return res


def serving(lv, nreq, rate, bank_k=4):
    """The serving trace (synth.trace) twice: BF16 maps through the server
    (2 workers, same-scene requests merged into one pass, admission by a
    64 GiB accumulator budget), and FP32 maps one request at a time (1 worker,
    no merging).  Latency = completion - submission; submissions follow the
    trace's arrival times."""
    import torch
    from synth import trace
    log(f"bench: serving leg ({nreq} requests at {rate}/s): scenes, rigs, map bank")
    scs = [lv.Scene.from_arrays(s) for s in trace.scenes()]
    rigs = [trace.rig(r) for r in range(len(trace.RESOLUTIONS))]
    bank32 = [trace.bank(r, bank_k) for r in range(len(trace.RESOLUTIONS))]
    bank16 = [[b.to(torch.bfloat16) for b in bk] for bk in bank32]
    reqs = trace.requests(nreq, rate)
    check = list(range(min(6, nreq)))  # requests whose BF16 and FP32 results are compared

    def run(dtype, workers, max_sets):
        bank = bank16 if dtype == "bf16" else bank32
        srv = lv.Server(budget=64 << 30, workers=workers, max_sets=max_sets, max_channels=1024)
        # warm each worker's stream workspace on every scene (not timed)
        for k, g in enumerate(scs):
            for _ in range(workers):
                srv.submit(g, rigs[2][:1], [bank[2][0][..., :4]], dtype=dtype, tag=1_000_000 + k)
        srv.drain()
        srv.poll()
        torch.cuda.synchronize()
        kept, comps = {}, []
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(0.0005)
            maps = [bank[r.res][v % bank_k][..., :r.D] for v in r.views]
            srv.submit(scs[r.scene], [rigs[r.res][v] for v in r.views], maps, dtype=dtype, tag=i)
            for c in srv.poll():
                comps.append(c)
        srv.drain()
        comps += srv.poll()
        st = srv.stats()
        srv.close()
        for c in comps:
            if c["tag"] in check:
                kept[c["tag"]] = c["out"]
        bad = [(c["tag"], c["status"]) for c in comps if c["status"] != 0]
        if len(comps) != nreq or bad:
            raise RuntimeError(f"serving: {len(comps)} of {nreq} completed, failed: {bad[:8]}")
        lat = [(c["t_end"] - c["t_submit"]) * 1e3 for c in comps]
        span = max(c["t_end"] for c in comps) - min(c["t_submit"] for c in comps)
        res = {"p50_ms": round(percentile(lat, 0.5), 2), "p99_ms": round(percentile(lat, 0.99), 2),
               "req_per_s": round(nreq / span, 3), "makespan_s": round(span, 3),
               "passes": st["passes"] - len(scs) * workers,
               "mean_requests_per_pass": round(nreq / max(1, st["passes"] - len(scs) * workers), 2)}
        return res, kept

    served, out16 = run("bf16", 2, 8)
    log(f"bench: served {served}")
    base, out32 = run("f32", 1, 1)
    log(f"bench: baseline {base}")
    err = 0.0
    for k in check:
        a, b = out16[k].double(), out32[k].double()
        err = max(err, float(((a - b).abs().max(dim=0).values / b.abs().max(dim=0).values.clamp_min(1e-30)).max()))
    views = [len(r.views) for r in reqs]
    return {
        "trace": {"requests": nreq, "rate_per_s": rate, "scenes": list(trace.SCENE_SIZES),
                  "resolutions": [list(x) for x in trace.RESOLUTIONS], "D": list(trace.D_CHOICES),
                  "views_mean": round(sum(views) / len(views), 1)},
        "served_bf16": served,
        "baseline_f32_one_at_a_time": base,
        "speedup_req_per_s": round(served["req_per_s"] / base["req_per_s"], 3),
        "bf16_vs_f32_max_rel_err": err,
    }


def cpu_baseline(w, sc, cams, maps, masks, views):
    """The FP64 oracle (unchanged) on the first `views` views of the workload,
    both feature sets, all Gaussians; host threads as the oracle uses them."""
    import oracle
    log(f"bench: cpu baseline ({views} views)")
    hm = [maps[v].cpu().numpy() for v in range(views)]
    hk = [masks[v].cpu().numpy() for v in range(views)]
    t0 = time.perf_counter()
    oracle.uplift(sc, cams[:views], hm)
    oracle.uplift(sc, cams[:views], hk)
    t = time.perf_counter() - t0
    return {"value": round(t * 1e3 / (views * (w.D + 1)), 4), "unit": "ms/view/channel",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{views} of {w.m} views, D=64 and D=1, all {w.n} Gaussians, FP64",
            "seconds": round(t, 2)}


if __name__ == "__main__":
    main()

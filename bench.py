#!/usr/bin/env python3
"""Benchmark of the uplift hot path on one MI355X.

Headline workload (the large precision configuration): 1,000,000 Gaussians
(centres U[-1,1]^3, scales exp(N(-5, 0.7^2)), uniform rotations, opacities
sigmoid(N(0.5, 1))), 100 Fibonacci-sphere cameras at radius 4, 1008x756 px,
55 deg horizontal FoV; D = 384 feature maps (N(0,1) at 1/14 resolution,
bilinearly upsampled), stored BF16 (the headline), FP32 and FP8 E4M3 with
per-(view, channel) scales; FP32 accumulation throughout.  Every map of the
three storage formats is generated and resident in HBM before timing
(205 GB).

One step = the whole uplift job on that workload: make the scene resident
(lv_scene_create), uplift the 100 BF16 maps (lv_uplift: structure build and
blend-accumulate of all views, finalize), release the scene.  value = ms per
(view x channel) = ms_per_step / (100 x 384).

Also in the same JSON line:
  roofline      the blend-and-accumulate kernel of the headline step, timed
                with HIP events on its stream during the timed steps, against
                the HBM and FP32-FMA roofs of its algorithmic bytes and flops
                (the binding one named), plus its matrix-core share;
  storage       the FP32 and FP8 legs of the same job, and the error of every
                storage leg against the FP64 oracle on a 20,000-Gaussian
                subsample (views given by --oracle-views);
  mid           the mid configuration (200k Gaussians, 50 views of 512x384,
                D = 64 maps + a D = 1 mask in one pass), FP32 and BF16;
  diffuse       the uplift + diffusion configuration: 16-NN graph of the large
                scene built on the device from D = 64 uplifted features, 100
                steps of Eq. (8) at D = 1 and D = 64, FP32 and BF16 storage;
  serving       the serving trace through the request server;
  cpu_baseline  the FP64 oracle on a bounded sample of the headline workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "uplift ms/view/channel + % HBM roofline, BF16 vs FP32 @ tol; p50/p99 latency"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3        # MI355X vector FP32 (packed FMA)
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores
SUBSAMPLE = 20_000


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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default="f32,fp8", help="storage legs besides the BF16 headline")
    ap.add_argument("--layout", choices=["px8", "hwc"], default="px8",
                    help="stored-map layout of the large configuration's legs: pixel blocks "
                         "(lv_encode_map) or HWC")
    ap.add_argument("--oracle-views", type=int, default=6,
                    help="views of the headline workload the FP64 oracle runs (0 = skip)")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--only", choices=["mid", "diffuse", "render", "serving"],
                    help="run one secondary leg alone (no headline; for profiles)")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests of the serving trace (0 = skip the serving leg)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, req/s")
    ap.add_argument("--serve-workers", type=int, default=2, help="server workers (passes in flight)")
    ap.add_argument("--serve-log", default=None,
                    help="write each served request's metrics as JSON lines to PATH.<dtype>.w<workers>.jsonl")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2410_14462_amd as lv

    torch.cuda.set_device(0)
    if args.only:
        leg = {"mid": lambda: mid_leg(lv, args), "diffuse": lambda: diffusion_leg(lv),
               "render": lambda: render_leg(lv),
               "serving": lambda: serving(lv, args.serve_requests, args.serve_rate, log_path=args.serve_log, workers=args.serve_workers)}[args.only]
        print(json.dumps({args.only: leg()}), flush=True)
        return
    out, keep = large_leg(lv, args)
    if args.calib_copy:
        src = torch.empty(1 << 28, device="cuda", dtype=torch.float32).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
        del src, dst
    del keep
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["mid"] = mid_leg(lv, args)
        torch.cuda.empty_cache()
        out["diffuse"] = diffusion_leg(lv)
        torch.cuda.empty_cache()
        out["render"] = render_leg(lv)
        torch.cuda.empty_cache()
        if args.serve_requests > 0:
            out["serving"] = serving(lv, args.serve_requests, args.serve_rate, log_path=args.serve_log, workers=args.serve_workers)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ headline
def large_leg(lv, args):
    import numpy as np
    import torch

    from synth import scenes

    w = scenes.WORKLOADS["large"]
    n, m, H, W, D = w.n, w.m, w.height, w.width, w.D
    log(f"bench: {w.name}: scene, rig")
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    means, scales, quats, opac = dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacity)
    legs = ["bf16"] + [x for x in args.legs.split(",") if x in ("f32", "fp8")]
    # storage format of each leg (lv dtype): the encoded legs in pixel blocks
    # (or HWC), the FP32 leg the maps as generated (HWC: the faster FP32 path)
    fmt = {k: (k + "_px8" if args.layout == "px8" else k) for k in ("bf16", "fp8")}
    fmt["f32"] = "f32"
    rig = lv.Cameras(cams)
    fout = torch.empty((n, D), device="cuda")
    bout = torch.empty((n,), device="cuda")
    nv = args.oracle_views

    def generate(leg):
        """The leg's 100 stored maps (all resident in HBM) and FP8 scales; one
        leg's maps at a time."""
        maps, sc8 = [], []
        for v in range(m):
            f = scenes.feature_map(w, v, device="cuda")
            if leg == "f32":
                maps.append(f)
            else:
                e, s8 = lv.encode(f, fmt[leg])
                maps.append(e)
                if s8 is not None:
                    sc8.append(s8)
            del f
        torch.cuda.synchronize()
        return maps, (torch.stack(sc8).contiguous() if sc8 else None)

    storage, kept, gpu_sub = {}, {}, {}
    out = None
    for leg in legs:
        log(f"bench: {leg} leg: {m} maps ({fmt[leg]})")
        maps, scales8 = generate(leg)
        tab = lv.Maps(maps, fmt[leg])

        def step():
            s = lv.Scene(means, scales, quats, opac)
            s.uplift(rig, tab, dtype=fmt[leg], scales=scales8, out=fout, wsum=bout)
            s.close()

        if leg == "bf16":
            # work statistics of the headline pass (untimed, with counters)
            s = lv.Scene(means, scales, quats, opac)
            acc = lv.Accum(s, D, counts=True)
            acc.add(rig, tab, dtype=fmt[leg], scales=scales8)
            stats = acc.stats()
            acc.close()
            s.close()
            log(f"bench: stats {stats}")
            log(f"bench: headline (bf16): warmup {args.warmup}, timing {args.steps} steps")
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
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
            value = ms_step / (m * D)
            log(f"bench: {ms_step:.3f} ms/step, {value * 1e3:.4f} us/view/channel, "
                f"blend {sum(launches) / args.steps:.2f} ms in {len(launches) / args.steps:.0f} launches")
            roof = roofline(stats, launches, args.steps, n, D, 2, products=2,
                            kernel=f"blend_pair_kernel<LV_BF16, {args.layout == 'px8'}> "
                                   f"(D=384 BF16 maps, {args.layout.upper()} layout)",
                            traffic_name=f"blend_pair_kernel-uplift-1M-100v-1008x756-D384-{fmt['bf16']}")
            storage[leg] = {"ms_per_step": round(ms_step, 3), "ms_per_view_channel": round(value, 7),
                            "blend_ms_per_step": round(sum(launches) / args.steps, 3)}
            out = {
                "metric": METRIC,
                "value": round(value, 8),
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
                           "channels": D, "storage": fmt["bf16"], "accumulation": "f32",
                           "scene_order": "morton (library default; outputs in the caller's order)",
                           "contraction": "split-BF16 matrix-core products, FP32 accumulate (BF16 maps "
                                          "and FP8 codes: 2 exact products per term; FP32 maps: 3, "
                                          "error < 2^-16 |w F|)"},
                "latency_ms": {"p50": round(percentile(lat, 0.5), 3), "p99": round(percentile(lat, 0.99), 3)},
                "contributions_per_s": round(stats["contributions"] / (ms_step * 1e-3), 1),
                "work": stats,
                "roofline": roof,
            }
        else:
            step()
            torch.cuda.synchronize()
            lv.profile_start()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3 / reps
            bl = lv.profile_stop()
            storage[leg] = {"ms_per_step": round(t, 3), "ms_per_view_channel": round(t / (m * D), 7),
                            "blend_ms_per_step": round(sum(bl) / reps, 3)}
            log(f"bench: {leg}: {storage[leg]}")
        if nv > 0:  # this leg's result over the first nv views, for the oracle comparison
            s = lv.Scene(means, scales, quats, opac)
            gpu_sub[leg] = s.uplift(cams[:nv], maps[:nv], dtype=fmt[leg],
                                    scales=None if scales8 is None else scales8[:nv].contiguous())
            torch.cuda.synchronize()
            s.close()
            kept[leg] = ([t.clone() for t in maps[:nv]], None if scales8 is None else scales8[:nv].clone())
        del tab, maps, scales8
        torch.cuda.empty_cache()
    storage["bf16_speedup_vs_f32"] = (round(storage["f32"]["ms_per_step"] / storage["bf16"]["ms_per_step"], 3)
                                      if "f32" in storage else None)
    if nv > 0:
        errs, cpu = oracle_errors(w, sc, cams, gpu_sub, kept, nv)
        for dt, e in errs.items():
            storage[dt]["error"] = e
        out["cpu_baseline"] = cpu
        out["cpu_baseline"]["cpu_over_gpu"] = round(cpu["value"] / out["value"], 1)
    out["storage"] = storage
    return out, None


def measured_traffic(name):
    """HBM bytes per blend launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", name + "_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2410_14462_amd", "csrc")
    src = open(os.path.join(csrc, "blend.hip"), "rb").read() + \
        open(os.path.join(csrc, "lv_internal.h"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return int(rec["traffic_bytes"])


def roofline(st, launches, steps, n, D, s_f, products, kernel, traffic_name):
    """Blend-accumulate against its roofs.  Algorithmic bytes of a step: the
    features of covered pixels (covered_px D s_F), one 24-byte projected
    record per visible (view, Gaussian), one 4-byte id per (tile, Gaussian)
    pair, and U and beta written once per launch (n (D + 1) 4).  Flops: one
    FMA per channel per counted contribution plus ~15 for alpha, T and w
    (2 nnz D + 15 nnz).  The FP32-FMA roof prices those flops at 157.3
    TFLOP/s; the matrix-core share prices the contraction as it runs (2 nnz D
    per product, `products` split-BF16 products) at 2.5 PFLOP/s."""
    per_step = len(launches) / steps
    t = sum(launches) / len(launches) * 1e-3          # average launch, s
    nb = (st["covered_pixels"] * D * s_f + st["visible"] * 24 + st["pairs"] * 4
          + per_step * n * (D + 1) * 4) / per_step     # bytes per launch
    nnz = st["contributions"] / per_step
    fl = 2.0 * nnz * D + 15.0 * nnz
    mf = 2.0 * nnz * D * products
    gbs, tfl = nb / t / 1e9, fl / t / 1e12
    hbm = {"achieved_GBs": round(gbs, 1), "peak_GBs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
           "alg_bytes_per_launch": int(nb)}
    fma = {"achieved_TFLOPs": round(tfl, 2), "peak_TFLOPs": FP32_PEAK_TFLOPS,
           "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "alg_flops_per_launch": fl}
    mfma = {"achieved_TFLOPs": round(mf / t / 1e12, 2), "peak_TFLOPs": MFMA_BF16_PEAK_TFLOPS,
            "frac": round(mf / t / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4), "products_per_term": products}
    if nb / (HBM_PEAK_GBS * 1e9) >= fl / (FP32_PEAK_TFLOPS * 1e12):
        roof = {"bound": "hbm", "achieved": hbm["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm["frac"]}
    else:
        roof = {"bound": "alu", "achieved": fma["achieved_TFLOPs"], "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": fma["frac"]}
    roof.update({"traffic": measured_traffic(traffic_name), "kernel": kernel,
                 "launches_per_step": per_step, "launch_ms": round(t * 1e3, 4),
                 "hbm": hbm, "fma_fp32": fma, "mfma_bf16": mfma})
    if st.get("partial_sums", -1) > 0:
        # one device-scope FP32 atomic per channel and one for beta per
        # (Gaussian, view, pixel block) partial sum
        ps = st["partial_sums"] / per_step
        upd = ps * (D + 1)
        roof["atomics"] = {"updates_per_launch": int(upd), "achieved_Gps": round(upd / t / 1e9, 1),
                           "partial_sums_per_launch": int(ps)}
    return roof


def unblock(t, W):
    """A pixel-block map [H, ceil(W/8), D, 8] back to HWC [H, W, D] (HWC maps pass)."""
    if t.dim() == 3:
        return t
    H, W8, D, _ = t.shape
    return t.permute(0, 1, 3, 2).reshape(H, W8 * 8, D)[:, :W]


def oracle_errors(w, sc, cams, gpu_sub, kept, nv):
    """Each storage leg's result over the first nv views against the FP64
    oracle on a 20,000-Gaussian subsample: total error (oracle on the FP32
    maps) and accumulation error (oracle on the decoded stored maps), in units
    of a = sum w |F| / beta; Gaussians flagged by an ambiguous skip/stop
    decision are excluded and counted.  The first oracle run is also the CPU
    baseline."""
    import numpy as np
    import torch

    import oracle
    from synth import scenes

    rows = scenes.subsample(w.seed, sc.n, SUBSAMPLE)

    def run(get):
        up = oracle.Uplifter(sc, w.D, rows=rows)
        for v in range(nv):
            up.add_view(cams[v], get(v))
        return up.result()

    log(f"bench: oracle on {nv} views, {SUBSAMPLE} Gaussians accumulated")
    host32 = lambda v: scenes.feature_map(w, v, device="cuda").cpu().numpy()
    t0 = time.perf_counter()
    ref32 = run(host32)
    t_cpu = time.perf_counter() - t0

    def decoded(dt):
        maps, s8 = kept[dt]
        if dt == "f32":
            return host32
        if dt == "bf16":
            return lambda v: unblock(maps[v], w.width).float().cpu().numpy()
        return lambda v: (unblock(maps[v], w.width).view(torch.float8_e4m3fn).float() * s8[v]).cpu().numpy()

    errs = {}
    for dt, (f, b) in gpu_sub.items():
        f = f.cpu().numpy().astype(np.float64)[rows]
        b = b.cpu().numpy().astype(np.float64)
        refq = ref32 if dt == "f32" else run(decoded(dt))
        res = {}
        for name, ref in (("total", ref32), ("accumulation", refq)):
            ok = (ref.beta[rows] > 0) & ref.strict[rows]
            a = ref.a[ok]
            e = np.abs(f[ok] - ref.f[ok]) / np.maximum(a, 1e-30)
            res[name] = {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "mean": float(e.mean())}
        okb = (refq.beta > 0) & refq.strict
        res["beta_rel_max"] = float((np.abs(b[okb] - refq.beta[okb]) / refq.beta[okb]).max())
        res["bound_total"] = {"f32": "1e-4 a", "bf16": "2^-8 a + 1e-4 a",
                              "fp8": "2^-4 a + 2^-10 scale + 1e-4 a"}[dt]
        res["ambiguous_pixels"] = ref32.amb_px
        res["excluded_gaussians"] = int((~ref32.strict[rows]).sum())
        errs[dt] = res
        log(f"bench: {dt} error {res}")
    cpu = {"value": round(t_cpu * 1e3 / (nv * w.D), 4), "unit": "ms/view/channel (subsample)",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{nv} of {w.m} views, D={w.D}, every pixel walked over all {w.n} Gaussians, "
                     f"{SUBSAMPLE} Gaussians accumulated, FP64",
           "seconds": round(t_cpu, 2)}
    return errs, cpu


# --------------------------------------------------------------- mid config
def mid_leg(lv, args):
    """200k Gaussians, 50 views of 512x384, D = 64 maps and the D = 1 mask in
    one pass; FP32 and BF16 storage; the blend's roofline for each."""
    import numpy as np
    import torch

    from synth import scenes

    w = scenes.WORKLOADS["mid"]
    n, m, H, W, D = w.n, w.m, w.height, w.width, w.D
    log(f"bench: mid leg {w.name}")
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    means, scales, quats, opac = dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacity)
    maps = [scenes.feature_map(w, v, device="cuda") for v in range(m)]
    masks = [dev(scenes.ellipse_mask(w.seed, v, H, W)) for v in range(m)]
    rig = lv.Cameras(cams)
    tab = {"f32": (lv.Maps(maps), lv.Maps(masks)),
           "bf16": (lv.Maps([x.to(torch.bfloat16) for x in maps], "bf16"),
                    lv.Maps([x.to(torch.bfloat16) for x in masks], "bf16")),
           "bf16_px8": (lv.Maps([lv.encode(x, "bf16_px8")[0] for x in maps], "bf16_px8"),
                        lv.Maps([lv.encode(x, "bf16_px8")[0] for x in masks], "bf16_px8"))}
    outs = [(torch.empty((n, D), device="cuda"), torch.empty((n,), device="cuda")),
            (torch.empty((n, 1), device="cuda"), torch.empty((n,), device="cuda"))]
    s = lv.Scene(means, scales, quats, opac)
    acc, accm = lv.Accum(s, D, counts=True), lv.Accum(s, 1, counts=True)
    lv.accumulate_sets(cams, [(acc, maps), (accm, masks)])
    st = acc.stats()
    acc.close()
    accm.close()
    s.close()
    res = {"workload": w.name, "work": st}
    for dt in ("f32", "bf16", "bf16_px8"):
        def step():
            s = lv.Scene(means, scales, quats, opac)
            s.uplift_sets(rig, list(tab[dt]), dtype=dt, outs=outs)
            s.close()
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        lv.profile_start()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3 / reps
        bl = lv.profile_stop()
        kname = "LV_F32, false" if dt == "f32" else "LV_BF16, false" if dt == "bf16" else "LV_BF16, true"
        res[dt] = {"ms_per_step": round(t, 3), "ms_per_view_channel": round(t / (m * (D + 1)), 7),
                   "roofline": roofline(st, bl, reps, n, D + 1, 4 if dt == "f32" else 2,
                                        3 if dt == "f32" else 2, f"blend_wide_kernel<{kname}>",
                                        f"blend_wide_kernel-{w.name}-{dt}")}
        log(f"bench: mid {dt}: {res[dt]['ms_per_step']} ms/step, blend {res[dt]['roofline']['launch_ms']} ms")
    res["bf16_speedup_vs_f32"] = round(res["f32"]["ms_per_step"] / res["bf16"]["ms_per_step"], 3)
    res["bf16_blend_speedup_vs_f32"] = round(res["f32"]["roofline"]["launch_ms"]
                                             / res["bf16"]["roofline"]["launch_ms"], 3)
    res["bf16_px8_speedup_vs_f32"] = round(res["f32"]["ms_per_step"] / res["bf16_px8"]["ms_per_step"], 3)
    return res


# ------------------------------------------------------ uplift + diffusion
def diffusion_leg(lv):
    """The uplift + diffusion configuration: D = 64 FP32 features uplifted
    from the 100 views of the large scene, the 16-NN graph built on the device
    from them, 100 steps of Eq. (8) on a D = 1 half-space mask and on the D =
    64 features, FP32 and BF16 storage (signal and graph values).  Bytes of a
    step: row pointers 4 (n + 1), columns and values nnz (4 + s_val), the
    signal read and written once, 2 n D s_g."""
    import torch

    from synth import scenes

    w = scenes.WORKLOADS["diffuse"]
    n, m, D = w.n, w.m, w.D
    steps = w.extra["steps"]
    log(f"bench: diffusion leg {w.name}")
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)
    gs = lv.Scene.from_arrays(sc)
    acc = lv.Accum(gs, D)
    t_up = 0.0
    for v0 in range(0, m, 10):
        maps = [scenes.feature_map(w, v, device="cuda", D=D) for v in range(v0, v0 + 10)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc.add(cams[v0:v0 + 10], maps)
        torch.cuda.synchronize()
        t_up += time.perf_counter() - t0
        del maps
    f, _ = acc.finalize()
    acc.close()
    G = lv.Graph.knn(gs, f, w.extra["k"])
    G.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = lv.Graph.knn(gs, f, w.extra["k"])
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    rp, col, val = G.csr()
    nnz = int(col.shape[0])
    Gb = lv.Graph(rp, col, val.to(torch.bfloat16))
    mask = torch.as_tensor(scenes.halfspace_indicator(w.seed, sc.means), device="cuda")
    res = {"workload": w.name, "uplift_ms": round(t_up * 1e3, 2), "graph_build_ms": round(t_graph * 1e3, 2),
           "graph_nnz": nnz, "steps": steps}
    for name, g0, Gx, s_v, s_g in (("D1_f32", mask, G, 4, 4), ("D64_f32", f, G, 4, 4),
                                   ("D1_bf16", mask.to(torch.bfloat16), Gb, 2, 2),
                                   ("D64_bf16", f.to(torch.bfloat16), Gb, 2, 2)):
        o = Gx.diffuse(g0, steps, scene=gs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = Gx.diffuse(g0, steps, scene=gs, out=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        Dg = 1 if g0.dim() == 1 else g0.shape[1]
        byts = 4 * (n + 1) + nnz * (4 + s_v) + 2 * n * Dg * s_g
        res[name] = {"ms_per_step": round(t * 1e3, 4), "GBs": round(byts / t / 1e9, 1),
                     "hbm_frac": round(byts / t / 1e9 / HBM_PEAK_GBS, 4), "bytes_per_step": byts}
        log(f"bench: diffuse {name}: {res[name]}")
    G.close()
    Gb.close()
    gs.close()
    return res


# ------------------------------------------------------------ forward render
RENDER_VIEWS = 20


def render_leg(lv):
    """Eq. (4) on the large scene: D = 384 FP32 features (seeded normal draws)
    rendered with opacity into the first RENDER_VIEWS of its 1008x756 views,
    into preallocated outputs.  Algorithmic bytes per view: every output
    written once, H W (D + 1) 4, and the features of the Gaussians the view
    sees read once, taken as n D 4 (the rig sees all but 0.03 % of the scene
    in every view); the render kernel's own time from HIP events around its
    launches."""
    import torch

    from synth import scenes

    w = scenes.WORKLOADS["large"]
    n, H, W, D = w.n, w.height, w.width, w.D
    m = RENDER_VIEWS
    log(f"bench: render leg {w.name}: {m} views, D={D}")
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)[:m]
    gs = lv.Scene.from_arrays(sc)
    gen = torch.Generator().manual_seed(w.seed + 4)
    g = torch.randn((n, D), generator=gen).to("cuda")
    outs = ([torch.empty((H, W, D), device="cuda") for _ in range(m)],
            [torch.empty((H, W), device="cuda") for _ in range(m)])
    gs.render(cams, g, outs=outs)  # warmup
    torch.cuda.synchronize()
    reps = 3
    lv.profile_start()
    t0 = time.perf_counter()
    for _ in range(reps):
        gs.render(cams, g, outs=outs)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) * 1e3 / reps
    bl = lv.profile_stop()
    gs.close()
    launch_ms = float(sum(bl)) / reps
    byts = m * (H * W * (D + 1) * 4 + n * D * 4)
    gbs = byts / (launch_ms * 1e-3) / 1e9
    res = {"workload": f"render-1M-{m}v-{W}x{H}-D{D}", "views": m, "D": D,
           "ms_per_call": round(t, 3), "ms_per_view": round(t / m, 4),
           "ms_per_view_channel": round(t / (m * D), 7),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "render_kernel",
                        "launches_per_call": len(bl) / reps, "launch_ms": round(launch_ms, 4),
                        "alg_bytes_per_call": byts}}
    log(f"bench: render: {t:.2f} ms per call of {m} views, render kernel {launch_ms:.2f} ms "
        f"({gbs:.0f} GB/s, {gbs / HBM_PEAK_GBS:.3f} of HBM)")
    del outs
    return res


# ------------------------------------------------------------------ serving
def serving(lv, nreq, rate, bank_k=4, log_path=None, workers=2):
    """The serving trace (synth.trace) three times: BF16 pixel-block maps through the
    server (2 workers, same-scene requests merged into one pass, admission by
    an HBM budget), FP32 maps through the same server settings, and FP32 maps
    one request at a time (1 worker, no merging).  Latency = completion -
    submission; submissions follow the trace's arrival times."""
    import torch

    from synth import trace
    log(f"bench: serving leg ({nreq} requests at {rate}/s): scenes, rigs, map bank")
    scs = [lv.Scene.from_arrays(s) for s in trace.scenes()]
    rigs = [trace.rig(r) for r in range(len(trace.RESOLUTIONS))]
    bank32 = [trace.bank(r, bank_k) for r in range(len(trace.RESOLUTIONS))]
    # BF16 maps in the pixel-block layout (requests read channel slices of them)
    bank16 = [[lv.encode(b, "bf16_px8")[0] for b in bk] for bk in bank32]
    reqs = trace.requests(nreq, rate)
    check = list(range(min(6, nreq)))  # requests whose BF16 and FP32 results are compared
    budget = 64 << 30

    scratch = 4 << 30  # per worker (the server's default)

    def take(t, D):  # channels [0, D) of a bank map, HWC or pixel blocks
        return t[..., :D] if t.dim() == 3 else t[:, :, :D, :]

    def run(dtype, workers, max_sets):
        bank = bank16 if dtype == "bf16" else bank32
        dtype = "bf16_px8" if dtype == "bf16" else dtype
        srv = lv.Server(budget=budget, workers=workers, max_sets=max_sets, max_channels=1024,
                        scratch=scratch)
        # warm each worker's stream workspace on every scene (not timed)
        for k, g in enumerate(scs):
            for _ in range(workers):
                srv.submit(g, rigs[2][:1], [take(bank[2][0], 4)], dtype=dtype, tag=1_000_000 + k)
        srv.drain()
        srv.poll()
        torch.cuda.synchronize()
        kept, comps = {}, []
        out_bytes = {}            # the client's output tensors of submitted, unfinished requests
        live = [0, 0]             # bytes in flight, peak

        def collect(cs):
            # a finished request's outputs are dropped at once (kept only for the
            # requests compared below), as a client that consumes them would
            for c in cs:
                if c["tag"] in check:
                    kept[c["tag"]] = c["out"]
                c.pop("out", None)
                c.pop("wsum", None)
                live[0] -= out_bytes.pop(c["tag"], 0)
                comps.append(c)

        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(0.0005)
            maps = [take(bank[r.res][v % bank_k], r.D) for v in r.views]
            srv.submit(scs[r.scene], [rigs[r.res][v] for v in r.views], maps, dtype=dtype, tag=i)
            out_bytes[i] = scs[r.scene].n * (r.D + 1) * 4
            live[0] += out_bytes[i]
            live[1] = max(live[1], live[0])
            collect(srv.poll())
        srv.drain()
        collect(srv.poll())
        st = srv.stats()
        srv.close()
        bad = [(c["tag"], c["status"]) for c in comps if c["status"] != 0]
        if len(comps) != nreq or bad:
            raise RuntimeError(f"serving: {len(comps)} of {nreq} completed, failed: {bad[:8]}")
        lat = [(c["t_end"] - c["t_submit"]) * 1e3 for c in comps]
        wait_admit = [(c["t_admit"] - c["t_submit"]) * 1e3 for c in comps]  # memory budget
        wait_pass = [(c["t_start"] - c["t_admit"]) * 1e3 for c in comps]    # admitted, waiting for a worker
        span = max(c["t_end"] for c in comps) - min(c["t_submit"] for c in comps)
        if log_path:
            with open(f"{log_path}.{dtype}.w{workers}.jsonl", "w") as fh:
                for c in comps:
                    fh.write(json.dumps(lv.completion_record(c)) + "\n")
        res = {"p50_ms": round(percentile(lat, 0.5), 2), "p99_ms": round(percentile(lat, 0.99), 2),
               "admission_wait_ms_p50_p99": [round(percentile(wait_admit, 0.5), 2),
                                             round(percentile(wait_admit, 0.99), 2)],
               "worker_wait_ms_p50_p99": [round(percentile(wait_pass, 0.5), 2),
                                          round(percentile(wait_pass, 0.99), 2)],
               "req_per_s": round(nreq / span, 3), "makespan_s": round(span, 3),
               "passes": st["passes"] - len(scs) * workers,
               "mean_requests_per_pass": round(nreq / max(1, st["passes"] - len(scs) * workers), 2),
               "peak_budget_bytes": st["peak_bytes"]}
        # the server's memory: accumulators (within the budget by admission) and
        # the workers' scratch, set aside from the budget at creation
        res["server_peak_bytes"] = st["peak_bytes"] + workers * scratch
        res["server_within_budget"] = res["server_peak_bytes"] <= budget
        if "peak_device_bytes" in st:
            # device memory in use above the level at the server's creation
            # (hipMemGetInfo): the server's, plus the client's output tensors of the
            # submitted, unfinished requests (caller-owned; peak of those below)
            res["peak_device_bytes"] = st["peak_device_bytes"]
            res["client_outputs_peak_bytes"] = live[1]
            res["peak_device_within_budget_plus_client_outputs"] = st["peak_device_bytes"] <= budget + live[1]
        return res, kept

    served, out16 = run("bf16", workers, 8)
    log(f"bench: served bf16 {served}")
    served32, _ = run("f32", workers, 8)
    log(f"bench: served f32 {served32}")
    base, out32 = run("f32", 1, 1)
    log(f"bench: baseline {base}")
    err = 0.0
    for k in check:
        a, b = out16[k].double(), out32[k].double()
        err = max(err, float(((a - b).abs().max(dim=0).values / b.abs().max(dim=0).values.clamp_min(1e-30)).max()))
    views = [len(r.views) for r in reqs]
    for g in scs:
        g.close()
    return {
        "trace": {"requests": nreq, "of_configured": 2000, "rate_per_s": rate,
                  "scenes": list(trace.SCENE_SIZES), "resolutions": [list(x) for x in trace.RESOLUTIONS],
                  "D": list(trace.D_CHOICES), "views_mean": round(sum(views) / len(views), 1),
                  "budget_bytes": budget},
        "served_bf16": served,
        "served_f32": served32,
        "baseline_f32_one_at_a_time": base,
        "speedup_req_per_s": round(served["req_per_s"] / base["req_per_s"], 3),
        "bf16_vs_f32_served_req_per_s": round(served["req_per_s"] / served32["req_per_s"], 3),
        "bf16_vs_f32_max_rel_err": err,
    }


if __name__ == "__main__":
    main()

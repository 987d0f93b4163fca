"""Benchmark of the rasterizer hot path on one MI355X.

A step is one full training iteration of the hot path on the paper-scale
workload (1M Gaussians, one 1600x1064 view, FP32): preprocess, bin/sort,
forward blend, L1 loss gradient, backward blend, then the chain rule fused with
the Adam step.
Inputs are resident in HBM before timing starts.  Prints ONE JSON line.

Besides the headline (Mpix/s at full resolution) the line carries the
per-level throughput at the schedule's downscale factors (8/4/2/1), the
batched multi-resolution form vs 16 sequential plain calls (it/s), the
roofline of the dominant kernel measured with HIP events on its stream, and
the FP64 oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (packed FP32: two FMAs per lane and cycle)
FP32_PEAK_TFLOPS = 157.3
# the same without packed-FP32 instructions, which the library is compiled without:
# 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# algorithmic FLOPs per (pixel, Gaussian) evaluation of Eq. 1 in the forward:
# offset (2), quadratic form (5 mul/fma = 8 FLOP), exponent + log2(o) (1), exp (1), clamp (1),
# two cutoff tests (2), T(1-alpha) (2), alpha*T (1), colour (3 fma = 6)
FWD_FLOP_PER_EVAL = 2 + 8 + 1 + 1 + 1 + 2 + 2 + 1 + 6
# and in the backward: alpha again (13), T recovery 1-a, 1/x, T*inv (3), weight (1),
# c.dL/dC (5), dL/dalpha (3), colour-behind update (2), colour grads (6), opacity
# grad (1: the sum of dL/dpower, divided by the opacity once per Gaussian), dL/dpower
# and its products with the offsets (3), conic grads (6), the two offset sums whose
# product with the conic is the mean gradient (2; the product itself is per
# Gaussian, not per evaluation)
BWD_FLOP_PER_EVAL = 13 + 3 + 1 + 5 + 3 + 2 + 6 + 1 + 3 + 6 + 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-batch", type=int, default=128)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--train-iters", type=int, default=6000,
                    help="iterations of the scheduled-training comparison (0: skip)")
    ap.add_argument("--train-ablations", action="store_true",
                    help="also run the ablation loops (fixed budget, resolution only, "
                         "Mip-Splatting primitives)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 4M-Gaussian, 16-view workload")
    ap.add_argument("--no-extras", action="store_true", help="skip levels and batched form")
    ap.add_argument("--graphs", action="store_true",
                    help="training loops replay one HIP graph per level instead of stepping eagerly")
    ap.add_argument("--no-spatial", action="store_true",
                    help="keep the scenes in generation order instead of the spatial order")
    ap.add_argument("--train-spatial", action="store_true",
                    help="training loops keep their Gaussians in the spatial order")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run warmup + this many steps (for rocprofv3), no extras")
    ap.add_argument("--level", type=int, default=1, choices=(1, 2, 4, 8),
                    help="with --profile-steps: profile the step at this downscale level "
                         "of the headline view")
    ap.add_argument("--sparse-adam", action="store_true",
                    help="with --profile-steps: profile the step with sparse Adam")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--training-only", action="store_true",
                    help="run only the training comparison (for rocprofv3) and print its JSON")
    return ap.parse_args()


def sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if (args.level != 1 or args.sparse_adam) and not args.profile_steps:
        print("--level and --sparse-adam are for profiling runs (--profile-steps)",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path would shard "
              "by views across GPUs, which is not implemented.", file=sys.stderr)
        sys.exit(2)
    # the host baseline first: its worker processes are forked before anything
    # touches the GPU
    cpu = None
    if not (args.no_cpu or args.training_only or args.profile_steps):
        log("timing the FP64 oracle on the host cores")
        cpu = cpu_baseline()
    import torch
    from paper_2503_18402_amd import gsmi, raster, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gsmi.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.training_only:
        print(json.dumps(scheduled_training(torch, raster, scenes, dev, args.train_iters,
                                            args.train_ablations, args.train_spatial,
                                            args.graphs)))
        return

    # ---------------------------------------------------------------- inputs
    log("generating the 1M-Gaussian scene and target")
    scene, cam = scenes.paper_scale_scene(level=args.level, n=args.n)
    tscene = scenes.paper_scale_target_scene(n=args.n)
    params = raster.to_device(scene, dev)
    if not args.no_spatial:
        # stored along the Morton curve of the means (gs_spatial_order); the
        # rendering does not depend on the order
        _, params = raster.spatial_order(params)
    tparams = raster.to_device(tscene, dev)
    target = raster.render(tparams, [cam], tile=args.tile).image.clone()
    del tparams
    pipe = raster.Pipeline(params, [cam], target, tile=args.tile, lds_batch=args.lds_batch,
                           sparse_adam=args.sparse_adam)
    stream = torch.cuda.current_stream()
    W, H = cam.width, cam.height

    steps = args.profile_steps if args.profile_steps else args.steps
    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps), timing {steps} steps")

    # ------------------------------------------------------------ timed loop
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fwd_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    for k in range(steps):
        step_ev[k].record(stream)
        p = pipe.params
        gsmi.gs_preprocess(pipe.cams_c, pipe.cfg, pipe.n, p["means"], p["log_scales"], p["quats"],
                           p["opacity_logits"], p["sh"], pipe.sh_degree, pipe.proj)
        gsmi.gs_bin_sort(pipe.cams_c, pipe.cfg, pipe.n, pipe.proj, pipe.capacity, pipe.sort_ws,
                         None, pipe.vals, pipe.ranges, pipe.n_pairs)
        pipe.loss.zero_()
        fwd_ev[k][0].record(stream)
        gsmi.gs_render_fwd_l1(pipe.cams_c, pipe.cfg, pipe.n, pipe.proj, pipe.ranges, pipe.vals,
                              pipe.image, pipe.final_T, pipe.last, pipe.targets,
                              1.0 / pipe.image.numel(), pipe.dL, pipe.loss)
        fwd_ev[k][1].record(stream)
        pipe.backward_adam(l1_done=True)
    step_ev[steps].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps
    per_step = np.array([step_ev[k].elapsed_time(step_ev[k + 1]) for k in range(steps)])
    step_stats = dict(median=round(float(np.median(per_step)), 4),
                      p10=round(float(np.percentile(per_step, 10)), 4),
                      p90=round(float(np.percentile(per_step, 90)), 4))
    assert not pipe.overflowed(), "pair capacity overflowed during timing"
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in fwd_ev]))
    n_pairs = int(pipe.n_pairs.item())
    mpix = W * H / (ms / 1e3) / 1e6
    log(f"{ms:.3f} ms/step ({mpix:.1f} Mpix/s), forward blend {fwd_ms:.3f} ms, pairs {n_pairs}")

    if args.copy_mib:
        # a plain streaming kernel of known traffic (reads and writes copy_mib MiB each),
        # the reference for scaling the profiler's fetch / write byte counters
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()

    if args.profile_steps:
        print(json.dumps(dict(profile_only=True, ms_per_step=ms, pairs=n_pairs)))
        return

    # per-kernel durations: the same steps again with every launch bracketed by HIP
    # events on its own stream (separate from the timed loop above)
    gsmi.gs_profile_enable(True)
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    kt = gsmi.gs_profile_collect()
    gsmi.gs_profile_enable(False)
    breakdown = {k: round(v[1] / steps, 4) for k, v in sorted(kt.items(), key=lambda kv: -kv[1][1])}
    kernel_ms = {k: v[1] / v[0] for k, v in kt.items()}

    # the same step with sparse Adam (the Taming backbone's optimiser: Gaussians
    # with no pair in the view keep their parameters and moments); reported
    # beside the dense step, not as the headline
    pipe.sparse_adam = True
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        pipe.step()
    ev1.record(stream)
    torch.cuda.synchronize()
    sparse_ms = ev0.elapsed_time(ev1) / steps
    gsmi.gs_profile_enable(True)
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    kt_sparse = gsmi.gs_profile_collect()
    gsmi.gs_profile_enable(False)
    pipe.sparse_adam = False
    # Gaussians with a pair in the view: the visibility count of the densification statistics
    vis = torch.zeros(pipe.n, device=dev)
    gsmi.gs_densify_stats(1, pipe.n, pipe.proj, torch.zeros(pipe.n, device=dev),
                          torch.zeros(pipe.n, device=dev), vis)
    sparse = dict(ms_per_step=round(sparse_ms, 4),
                  mpix_per_s=round(W * H / (sparse_ms / 1e3) / 1e6, 2),
                  k_chain_adam_ms=round(kt_sparse["k_chain_adam"][1] / kt_sparse["k_chain_adam"][0], 4),
                  touched=int((vis > 0).sum().item()), n=pipe.n)
    log(f"sparse Adam: {sparse_ms:.3f} ms/step, chain+Adam {sparse['k_chain_adam_ms']:.3f} ms")

    # ------------------------------------------------- blend rooflines (ALU)
    # algorithmic evaluations: per pixel, the list entries up to and including its
    # last blended Gaussian (the entries a pixel examines after it are not counted)
    evals = int(pipe.last.to(torch.int64).sum().item())
    srcs = ["paper_2503_18402_amd/csrc/blend_bwd.hip", "paper_2503_18402_amd/csrc/blend_common.hpp"]
    bwd_ms = kernel_ms["k_blend_bwd"]
    bwd_tf = evals * BWD_FLOP_PER_EVAL / (bwd_ms / 1e3) / 1e12
    fwd_tf = evals * FWD_FLOP_PER_EVAL / (kernel_ms["k_blend_fwd"] / 1e3) / 1e12
    algo_bytes = 40 * n_pairs + 24 * W * H   # records of the pairs + per-pixel state
    roofline = dict(kernel="k_blend_bwd", bound="alu", achieved=round(bwd_tf, 3),
                    peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(bwd_tf / FP32_PEAK_TFLOPS, 4),
                    frac_nonpacked=round(bwd_tf / ALU_PEAK_TFLOPS, 4),
                    peak_nonpacked=round(ALU_PEAK_TFLOPS, 1),
                    traffic=read_traffic("k_blend_bwd", srcs), evals=evals,
                    flop_per_eval=BWD_FLOP_PER_EVAL, launch_ms=round(bwd_ms, 4),
                    hbm_frac_algorithmic=round(algo_bytes / (bwd_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                    fwd=dict(kernel="k_blend_fwd", achieved=round(fwd_tf, 3),
                             frac=round(fwd_tf / FP32_PEAK_TFLOPS, 4),
                             frac_nonpacked=round(fwd_tf / ALU_PEAK_TFLOPS, 4),
                             launch_ms=round(kernel_ms["k_blend_fwd"], 4),
                             event_ms_in_timed_loop=round(fwd_ms, 4)))

    extras = {"binning": binning_forms(torch, pipe)}
    if not args.no_extras:
        extras["levels"] = level_sweep(torch, raster, scenes, params, tparams_scene=tscene,
                                       tile=args.tile, lds=args.lds_batch)
        extras["batched"] = batched_vs_plain(torch, raster, scenes, params, tscene)
        if not args.no_large:
            extras["large"] = large_scene(torch, raster, scenes, dev, not args.no_spatial)
        if args.train_iters > 0:
            extras["training"] = scheduled_training(torch, raster, scenes, dev, args.train_iters,
                                                    args.train_ablations, args.train_spatial,
                                                    args.graphs)

    out = {
        "metric": "fwd+bwd Mpix/s at 1M Gaussians 1600x1064; batched vs plain it/s at oracle tol",
        "value": round(mpix, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_step_stats": step_stats,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 1M-Gaussian scene; target rendered from a second seeded scene)",
        "config": {"workload": "1M Gaussians, one 1600x1064 view, full step: preprocess, "
                               "bin/sort, blend fwd, L1, blend bwd, chain rule fused with Adam",
                   "n_gaussians": args.n, "width": W, "height": H, "tile": args.tile,
                   "lds_batch": args.lds_batch, "pairs": n_pairs, "wall_s": round(wall, 3),
                   "storage_order": "index" if args.no_spatial else "spatial (Morton)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": breakdown,
        "sparse_adam": sparse,
    }
    out.update(extras)
    print(json.dumps(out))


def read_traffic(kernel: str, sources):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, or
    None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_counters.md")
    if not os.path.exists(path):
        return None
    want = sha(sources)
    data = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_json:"):
                data = json.loads(line.split(":", 1)[1])
    if not data or data.get("source_sha") != want:
        return None
    return data.get("bytes_per_launch")


def time_pipe(torch, pipe, steps):
    for _ in range(2):
        pipe.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pipe.step()
    e1.record()
    torch.cuda.synchronize()
    assert not pipe.overflowed()
    return e0.elapsed_time(e1) / steps


def binning_forms(torch, pipe, reps=20):
    """gs_bin_sort (pairs bucketed by tile, each tile's list sorted on chip)
    against gs_bin_sort_radix (stable LSD radix sort of the (tile | depth) keys)
    on the pipeline's current projected records: time per call and agreement."""
    from paper_2503_18402_amd import gsmi

    n, cap = pipe.n, pipe.capacity
    ws = torch.empty(max(gsmi.gs_bin_sort_radix_workspace_bytes(1, n, cap), 16),
                     dtype=torch.uint8, device=pipe.vals.device)
    vals = torch.empty_like(pipe.vals)
    ranges = torch.empty_like(pipe.ranges)
    npairs = torch.zeros(1, dtype=torch.int64, device=pipe.vals.device)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    bucket = timed(lambda: gsmi.gs_bin_sort(pipe.cams_c, pipe.cfg, n, pipe.proj, cap, pipe.sort_ws,
                                            None, pipe.vals, pipe.ranges, pipe.n_pairs))
    radix = timed(lambda: gsmi.gs_bin_sort_radix(pipe.cams_c, pipe.cfg, n, pipe.proj, cap, ws, None,
                                                 vals, ranges, npairs))
    npr = int(pipe.n_pairs.item())
    same = bool(torch.equal(vals[:npr], pipe.vals[:npr]) and torch.equal(ranges, pipe.ranges))
    log(f"binning: bucket + tile sort {bucket:.3f} ms, LSD radix {radix:.3f} ms, identical {same}")
    return dict(bucket_tile_sort_ms=round(bucket, 4), lsd_radix_ms=round(radix, 4),
                identical=same, pairs=npr)


def level_sweep(torch, raster, scenes, params, tparams_scene, tile, lds):
    """The plain single-view step at each downscale level of the schedule (8/4/2/1),
    autotuned per level and replayed from a HIP graph, with dense and with sparse
    Adam, and the two binning routes timed on the level's records."""
    from paper_2503_18402_amd import autotune, gsmi

    out = {}
    tparams = raster.to_device(tparams_scene, params["means"].device)
    for r in (8, 4, 2, 1):
        _, cam = scenes.paper_scale_scene(level=r, n=1)  # camera only
        tgt = raster.render(tparams, [cam], tile=tile).image.clone()
        p = {k: v.clone() for k, v in params.items()}
        pick = autotune.tune(p, [cam], tgt, reps=3)
        pipe = raster.Pipeline(p, [cam], tgt, tile=pick["tile"], lds_batch=pick["lds_batch"])
        pipe.capture()
        ms = time_pipe(torch, pipe, 10)
        # per-kernel durations over a few eager steps (event-bracketed launches)
        graph, pipe.graph = pipe.graph, None
        gsmi.gs_profile_enable(True)
        for _ in range(5):
            pipe.step()
        torch.cuda.synchronize()
        kt = gsmi.gs_profile_collect()
        gsmi.gs_profile_enable(False)
        pipe.graph = graph
        top = sorted(kt.items(), key=lambda kv: -kv[1][1])[:12]
        bins = binning_forms(torch, pipe, reps=10)
        # the same step with sparse Adam (rows of Gaussians with no footprint skipped)
        ps = raster.Pipeline({k: v.clone() for k, v in params.items()}, [cam], tgt,
                             tile=pick["tile"], lds_batch=pick["lds_batch"],
                             capacity=pipe.capacity, sparse_adam=True)
        ps.capture()
        ms_sparse = time_pipe(torch, ps, 10)
        out[f"r{r}"] = dict(width=cam.width, height=cam.height, ms_per_step=round(ms, 4),
                            mpix_per_s=round(cam.width * cam.height / (ms / 1e3) / 1e6, 2),
                            ms_per_step_sparse_adam=round(ms_sparse, 4),
                            tile=pick["tile"], lds_batch=pick["lds_batch"],
                            kernel_ms=({k: round(v[1] / 5, 4) for k, v in top}),
                            binning=bins)
        log(f"level r={r}: {ms:.3f} ms/step, sparse Adam {ms_sparse:.3f} "
            f"(tile {pick['tile']}, batch {pick['lds_batch']})")
        del pipe, ps, p
    return out


def batched_vs_plain(torch, raster, scenes, params, tscene):
    """One iteration over the 16 views of the multi-resolution workload (4 each at
    200x133, 400x266, 800x532, 1600x1064): fwd + bwd of every view and one Adam
    step.  Batched: all views in one launch per kernel.  Plain: 16 sequential
    per-view calls accumulating into one gradient buffer, then the same Adam.
    Both forms use autotuned tile / LDS batch (per mix, per resolution) and are
    captured as HIP graphs; eager times are reported too."""
    cams = scenes.mixed_resolution_views()
    tparams = raster.to_device(tscene, params["means"].device)
    tgts = [raster.render(tparams, [c]).image.clone() for c in cams]
    del tparams
    return compare_forms(torch, raster, params, cams, tgts, "16 mixed-resolution views")


def large_scene(torch, raster, scenes, dev, spatial=True):
    """The large workload: 4M Gaussians, 8 views at 1920x1080 and 8 at 960x540,
    gradients of all 16 views accumulated into one Adam step over 236M floats;
    seeded uniform random targets."""
    scene, cams = scenes.large_scene_views()
    params = raster.to_device(scene, dev)
    del scene
    if spatial:
        _, params = raster.spatial_order(params)
    gen = torch.Generator(device=dev).manual_seed(2)
    tgts = [torch.rand(3 * c.width * c.height, generator=gen, device=dev) for c in cams]
    out = compare_forms(torch, raster, params, cams, tgts, "16 views, 4M Gaussians")
    out["n_gaussians"] = int(params["means"].shape[0])
    return out


def compare_forms(torch, raster, params, cams, tgts, label):
    from paper_2503_18402_amd import autotune

    p = {k: v.clone() for k, v in params.items()}
    cat = torch.cat(tgts)
    tb = autotune.tune(p, cams, cat, reps=3)
    batched = raster.Pipeline(p, cams, cat, tile=tb["tile"], lds_batch=tb["lds_batch"])
    ms_b_eager = time_pipe(torch, batched, 5)
    batched.capture()
    ms_b = time_pipe(torch, batched, 5)
    pairs_b = int(batched.n_pairs.item())
    del batched
    # plain: per-resolution autotuned pipelines sharing one gradient buffer
    grads = raster.zero_grads(p)
    plains, picks = [], {}
    for c, t in zip(cams, tgts):
        key = (c.width, c.height)
        if key not in picks:
            picks[key] = autotune.tune(p, [c], t, reps=3)
        pk = picks[key]
        plains.append(raster.Pipeline(p, [c], t, tile=pk["tile"], lds_batch=pk["lds_batch"],
                                      grads=grads))

    def plain_iter():
        for k, pp in enumerate(plains):
            pp.forward()
            pp.backward(accumulate=k > 0)
        plains[0].adam()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_p_eager = timed(plain_iter, 3)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plain_iter()
    ms_p = timed(g.replay, 3)
    assert not any(pp.overflowed() for pp in plains)
    del plains, g
    log(f"{label}: batched {ms_b:.3f} ms/it (eager {ms_b_eager:.3f}), plain {ms_p:.3f} ms/it "
        f"(eager {ms_p_eager:.3f})")
    return dict(views=len(cams), pixels=sum(c.width * c.height for c in cams), pairs=pairs_b,
                batched_it_s=round(1e3 / ms_b, 2), plain_it_s=round(1e3 / ms_p, 2),
                speedup=round(ms_p / ms_b, 3),
                batched_eager_it_s=round(1e3 / ms_b_eager, 2),
                plain_eager_it_s=round(1e3 / ms_p_eager, 2),
                batched_cfg=dict(tile=tb["tile"], lds_batch=tb["lds_batch"]),
                plain_cfg={f"{w}x{h}": dict(tile=v["tile"], lds_batch=v["lds_batch"])
                           for (w, h), v in picks.items()},
                note="both forms autotuned and HIP-graph captured; fwd+bwd of all 16 views "
                     "plus one Adam step per iteration. The batched form runs the backward "
                     "fused with Adam (one call over all views); the plain form accumulates "
                     "16 per-view gradients and then runs the separate Adam step")


def scheduled_training(torch, raster, scenes, dev, iters, ablations=False, spatial=False,
                       graphs=False):
    """The optimisation loop of the hidden-scene workload: learnable Gaussians
    fitted to 64 views at 1200x800 of a 500k-Gaussian hidden scene (ground
    truth rendered once), ``iters`` iterations, one view per iteration.  From
    the same 50k-Gaussian start: the full method (Eq. 7 resolution schedule,
    Eq. 4/5 primitive schedule with top-k densification) as the fused
    pipeline step and as the autograd form (RasterizeFn under a torch L1 loss,
    loss.backward(), then the Adam step), and the backbone (full resolution,
    every candidate densified) for the time comparison.  With ``ablations``
    also: a fixed budget P_fin = 300k (momentum off, the Revising-3DGS
    setting), the resolution schedule alone, and the full method and the
    backbone on Mip-Splatting's primitives.
    Densification every 100 iterations over the first half; the gradient
    threshold is set for the synthetic scene (its gradients sit an order of
    magnitude below a photograph's) so that the backbone grows to about 300k.
    The schedule's downsampling factor is capped at 4 (the 1/4 -> 1/2 -> 1
    range of this workload; uncapped, the smooth synthetic views would start
    near 1/19).  Reports wall time, densification time, final primitive count
    and the mean full-resolution PSNR over the views."""
    from paper_2503_18402_amd import train

    hidden, cams = scenes.hidden_scene()
    hp = raster.to_device(hidden, dev)
    gt = torch.stack([raster.render(hp, [c]).image.view(3, c.height, c.width).clone()
                      for c in cams])
    del hp
    n_init, grad_thr, r_max = 50_000, 2e-5, 4.0
    init = scenes.make_scene(n_init, seed=6, mean_range=4.0, ls_mu=-4.0, ls_sigma=0.5)
    extent = 6.0 * 1.1   # camera sphere radius with the backbone's 10% margin
    # name: (resolution schedule, top-k densification, Mip primitives, fixed budget, autograd)
    loops = [("dashgaussian", True, True, False, None, False),
             ("dashgaussian_autograd", True, True, False, None, True),
             ("backbone", False, False, False, None, False)]
    if ablations:
        loops += [("dashgaussian_fixed_budget", True, True, False, 300_000, False),
                  ("resolution_only", True, False, False, None, False),
                  ("mip_dashgaussian", True, True, True, None, False),
                  ("mip_backbone", False, False, True, None, False)]
    out = {}
    for name, sched, top_k, mip, budget, autograd in loops:
        params = raster.to_device(init, dev)
        dcfg = train.DensifyConfig(every=100, start=100, stop=iters // 2, extent=extent,
                                   schedule=top_k, grad_thr=grad_thr, momentum=budget is None,
                                   p_fin=budget)
        tr = train.Trainer(params, cams, gt, iters, schedule=sched, densify=dcfg, r_max=r_max,
                           means_lr=(1.6e-4 * extent, 1.6e-6 * extent), mip=mip,
                           autograd=autograd, spatial=spatial, graphs=graphs)
        psnr0 = train.psnr(tr.params, cams, gt, mip2d=mip, filter3d=tr.filter3d)
        res = tr.run()
        psnr1 = train.psnr(tr.params, cams, gt, mip2d=mip, filter3d=tr.filter3d)
        out[name] = dict(seconds=round(res["seconds"], 3),
                         ms_per_iter=round(1e3 * res["s_per_iter"], 4),
                         densify_seconds=round(res["densify_seconds"], 3),
                         densify_steps=res["densify_steps"], n_gaussians=res["n_gaussians"],
                         iters_per_factor=res["iters_per_factor"], psnr_init=round(psnr0, 3),
                         psnr=round(psnr1, 3),
                         form="RasterizeFn (torch.autograd.Function)" if autograd else
                              ("fused pipeline step, one HIP graph replay per iteration"
                               if graphs else "fused pipeline step"),
                         storage_order="spatial" if spatial else "index")
        if sched:
            out[name]["r_knots"] = [round(float(x), 4) for x in tr.sched.r_knots]
            out[name]["s_knots"] = [round(float(x), 2) for x in tr.sched.s_knots]
        if top_k:
            out[name]["p_fin"] = round(float(tr.p_fin))
        log(f"training ({name}): {res['seconds']:.2f} s for {iters} iterations "
            f"({res['densify_seconds']:.2f} s densifying), {res['n_gaussians']} Gaussians, "
            f"PSNR {psnr0:.2f} -> {psnr1:.2f} dB")
        del tr, params
    for name in out:
        if name != "backbone" and not name.startswith("mip_"):
            out[name]["speedup_vs_backbone"] = round(out["backbone"]["seconds"] /
                                                     out[name]["seconds"], 3)
    if "mip_dashgaussian" in out:
        out["mip_dashgaussian"]["speedup_vs_backbone"] = round(
            out["mip_backbone"]["seconds"] / out["mip_dashgaussian"]["seconds"], 3)
    out.update(iters=iters, views=len(cams), width=cams[0].width, height=cams[0].height,
               initial=n_init, hidden=500_000, grad_thr_ndc=grad_thr, r_max=r_max,
               note="X(F_r) normalised per pixel; one view per iteration; L1 loss")
    return out


# ---- the FP64 oracle on the host (a baseline, not a target).  Workers are
# forked before anything touches the GPU and run numpy only.
_CPU = {}


def _oracle_tiles(tiles):
    """Worker: binned oracle forward + backward over ``tiles`` of the view in
    _CPU; returns the 2D gradient sums of the Gaussians it touched."""
    from threadpoolctl import threadpool_limits
    from oracle import render

    P, cands, w = _CPU["P"], _CPU["cands"], _CPU["w"]
    with threadpool_limits(1):
        render.render_fwd_binned(P, tiles=tiles, cands=cands)
        g = render.render_bwd_2d_binned(P, w, tiles=tiles, cands=cands)
    idx = np.nonzero(g["contrib"])[0]
    return idx, {k: g[k][idx] for k in ("d_mean2d", "d_conic", "d_opacity", "d_rgb", "abs2d")}


def cpu_baseline(one_core_tiles=(48, 12, 6)):
    """The FP64 oracle's fwd + bwd of the paper-scale view (1M Gaussians) at the
    schedule's levels r = 1, 4, 8, whole frames: projection, binned blend
    forward and backward (each tile blends its footprint candidates, which
    gives the brute force's result) and the chain rule to the parameters.  The
    blend runs on every host core (a process per core, tiles dealt round
    robin); projection and chain rule are single-threaded numpy.  One core:
    ``one_core_tiles`` tiles per level, spread over the list lengths, timed on
    one process and scaled by list entries to the frame."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import project, render
    from paper_2503_18402_amd import scenes

    cores = len(os.sched_getaffinity(0))
    scene, _ = scenes.paper_scale_scene(level=1)
    levels = {}
    for r, n1 in zip((1, 4, 8), one_core_tiles):
        _, cam = scenes.paper_scale_scene(level=r, n=1)
        t0 = time.perf_counter()
        with threadpool_limits(1):
            P = project.project(scene, cam, tile=16)
            cands = render.tile_candidates(P)
        t1 = time.perf_counter()
        w = np.random.default_rng(3).uniform(-1.0, 1.0, size=(3, cam.height, cam.width))
        _CPU.update(P=P, cands=cands, w=w)
        lens = np.array([len(c) for c in cands])
        chunks = [list(range(k, len(cands), cores)) for k in range(cores)]
        with mp.get_context("fork").Pool(cores) as pool:
            parts = pool.map(_oracle_tiles, chunks)
        t2 = time.perf_counter()
        g2 = {k: np.zeros((scene["means"].shape[0],) + v.shape[1:])
              for k, v in parts[0][1].items()}
        for idx, vals in parts:
            for k, v in vals.items():
                g2[k][idx] += v
        with threadpool_limits(1):
            render.chain_to_3d(scene, P, g2)
        t3 = time.perf_counter()
        # one core: a sample of tiles spread over the list lengths, scaled by entries
        pick = np.argsort(lens)[np.linspace(0, len(lens) - 1, n1).astype(int)]
        ta = time.perf_counter()
        _oracle_tiles(list(pick))
        tb = time.perf_counter()
        blend_1core = (tb - ta) * lens.sum() / max(1, lens[pick].sum())
        whole = t3 - t0
        one = (t1 - t0) + (t3 - t2) + blend_1core
        px = cam.width * cam.height
        levels[f"r{r}"] = dict(width=cam.width, height=cam.height, seconds_all_cores=round(whole, 2),
                               mpix_per_s_all_cores=round(px / whole / 1e6, 6),
                               seconds_one_core=round(one, 2),
                               mpix_per_s_one_core=round(px / one / 1e6, 6),
                               project_s=round(t1 - t0, 2), blend_s_all_cores=round(t2 - t1, 2),
                               chain_s=round(t3 - t2, 2), list_entries=int(lens.sum()),
                               one_core_sample_tiles=int(n1))
        log(f"oracle r={r}: {whole:.1f} s on {cores} cores, {one:.1f} s on one core (est.)")
        _CPU.clear()
        del P, cands
    head = levels["r1"]
    return dict(value=head["mpix_per_s_all_cores"], unit="Mpix/s", cores=cores, kind="oracle",
                sample="whole 1600x1064 frame of the 1M-Gaussian view (the headline workload): "
                       "FP64 projection, binned blend fwd+bwd on every core, chain rule; "
                       "also whole frames at r=4 and r=8, and one core estimated from a "
                       "sample of tiles per level",
                one_core_mpix_per_s=head["mpix_per_s_one_core"], levels=levels)


if __name__ == "__main__":
    main()

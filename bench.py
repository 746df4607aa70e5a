"""Benchmark: differentiated light paths per second on one MI355X.

One step = light-tracing forward (lt_trace) + L2 loss and image adjoint
(lt_loss_l2) + LRB-3-pass backward (lt_backward_lrb3) over 4,194,304 light
paths in the 256x256 textured box at max depth 32, inputs resident in HBM.
Prints one JSON line with the roofline of the dominant kernel (the fused
LRB-3 replay) and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per event (a 64-B two-child node, a 48-B triangle, a
# tent splat = 4 taps x RGB float read-modify-write, a tent gather = 4 taps
# x RGB float, one scattered gradient value = float read-modify-write)
B_NODE, B_TRI, B_SPLAT, B_GATHER, B_GRAD, B_TAPE = 64, 48, 96, 48, 8, 32


KERNEL_SOURCES = ["lt_common.h", "lt_device.h", "lt_launch.h", "lt_kernels.hip", "lt_attached.inc", "lt_camera.inc",
                  "lt_api.cpp"]


def profiled_traffic(name, field="traffic_bytes_per_launch"):
    """A figure from the committed rocprofv3 summary profiles/<name>: HBM bytes
    per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), a VALU
    issue fraction, an L2 hit rate or the resident waves per SIMD; None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().split()[0] if v.strip() else ""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2609_32920_amd", "csrc", f), "rb").read())
    if fields.get("sources_sha256") != h.hexdigest() or field not in fields:
        return None
    return float(fields[field])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--paths", type=int, default=1 << 22)
    ap.add_argument("--depth", type=int, default=32)
    ap.add_argument("--film", type=int, default=256)
    ap.add_argument("--no-sweep", action="store_true", help="skip the per-method / per-depth sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-caustic", action="store_true", help="skip the attached caustic workload")
    ap.add_argument("--no-guide", action="store_true", help="skip the learned-guide workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 48-instance workload")
    ap.add_argument("--guide-iters", type=int, default=40, help="online training iterations of the guide")
    ap.add_argument("--guide-seeds", type=int, default=32, help="seeds per gradient-variance estimate")
    ap.add_argument("--ee-seeds", type=int, default=16, help="seeds per equal-error variance estimate")
    ap.add_argument("--no-inverse", action="store_true", help="skip the heightfield inverse-rendering loop")
    ap.add_argument("--no-bidir", action="store_true", help="skip the bidirectional glass-slab workload")
    ap.add_argument("--lrb3-split", type=int, choices=(0, 1, 2), default=2,
                    help="lt_tuning.lrb3_split of the headline step (2: the library's default, fused when detached)")
    ap.add_argument("--no-materials", action="store_true",
                    help="skip the mirror / glass-panel / tumbler material workloads")
    ap.add_argument("--inverse-iters", type=int, default=1000, help="Adam iterations of the inverse-rendering loop")
    ap.add_argument("--cpu-paths", type=int, default=1 << 22, help="paths in the CPU-oracle sample")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="least CPU-oracle time (whole steps)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for profiler byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU execution is not "
              "implemented (paths would shard by index across GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2609_32920_amd import lt, scenes

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sc = scenes.box_scene(width=args.film, height=args.film)
    N, D = args.paths, args.depth
    ctx = lt.Context(0).scene_upload(sc)
    if args.lrb3_split != 2:
        ctx.set_tuning(lrb3_split=args.lrb3_split)
    albedo = torch.as_tensor(sc["albedo"], dtype=torch.float32, device=dev).contiguous()
    Le = torch.as_tensor(sc["Le"], dtype=torch.float32, device=dev)
    alb_t = torch.as_tensor(sc["albedo_target"], dtype=torch.float32, device=dev).contiguous()
    H = W = args.film
    img = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    target = torch.empty_like(img)
    dI = torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g_alb = torch.zeros_like(albedo)
    g_le = torch.zeros_like(Le)
    ctx.trace(ctx.args(0x7A6, N, D), ctx.params(alb_t, Le), target)
    torch.cuda.synchronize()

    p = ctx.params(albedo, Le)
    stream = torch.cuda.current_stream(dev)

    def step(seed, ev=None):
        a = ctx.args(seed, N, D)
        if ev: ev[0].record(stream)
        ctx.trace(a, p, img)
        if ev: ev[1].record(stream)
        ctx.loss_l2(img, target, dI, loss)
        if ev: ev[2].record(stream)
        ctx.backward_lrb3(a, p, dI, g_alb, g_le)
        if ev: ev[3].record(stream)

    if args.copy_ref:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for k in range(args.warmup):
        step(1000 + k)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(2000 + k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = [e[0].elapsed_time(e[1]) for e in evs]
    lss = [e[1].elapsed_time(e[2]) for e in evs]
    bwd = [e[2].elapsed_time(e[3]) for e in evs]
    step_ms = [e[0].elapsed_time(e[3]) for e in evs]
    ms_per_step = wall * 1e3 / args.steps
    value = N / (ms_per_step * 1e-3)
    print(f"# fwd {np.median(fwd):.3f} ms  loss {np.median(lss):.3f} ms  bwd(lrb3) {np.median(bwd):.3f} ms  "
          f"step(events) {np.median(step_ms):.3f} ms  step(wall) {ms_per_step:.3f} ms", file=sys.stderr, flush=True)

    # ---- algorithmic byte model from the counters build, on a path sample
    counts = {}
    sample = min(N, 1 << 18)
    try:
        cctx = lt.Context(0, counters=True).scene_upload(sc)
        cctx.read_counters(reset=True)
        a = cctx.args(2000, sample, D)
        cctx.trace(a, p, img)
        counts["trace"] = cctx.read_counters(reset=True)
        cctx.backward_lrb3(a, p, dI, torch.zeros_like(albedo), torch.zeros_like(Le))
        counts["lrb3"] = cctx.read_counters(reset=True)
        del cctx
    except Exception as e:  # the diagnostic build is optional
        print(f"# counters unavailable: {e}", file=sys.stderr)

    def bytes_per_path(c, n_sample=None):
        b = (c["nodes"] * B_NODE + c["tris"] * B_TRI + c["splats"] * B_SPLAT + c["gathers"] * B_GATHER
             + c["grad_values"] * B_GRAD + (c["tape_written"] + c["tape_read"]) * B_TAPE)
        return b / (n_sample or sample)

    roofline = None
    if "lrb3" in counts:
        bpp = bytes_per_path(counts["lrb3"])
        t_launch = float(np.mean(bwd)) * 1e-3
        achieved = bpp * N / t_launch / 1e9
        fused = args.lrb3_split != 1
        traffic = profiled_traffic("k_lrb3_bwd_box256_d32_4M.txt") if (fused and N == 1 << 22 and D == 32 and W == 256) \
            else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    # the same launch's measured DRAM bytes (rocprofv3) over its time: the
                    # share of the HBM peak the kernel actually moves, beside the
                    # algorithmic-byte fraction above
                    "traffic_frac": None if traffic is None else round(traffic / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                    "kernel": "k_lrb3_bwd" if fused else "k_lrb3_p2 + k_lrb3_p3", "bytes_per_path": round(bpp, 1),
                    "valu_issue_frac_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                                 "valu_issue_frac_k_lrb3_bwd"),
                    "l2_hit_rate_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                             "l2_hit_rate_k_lrb3_bwd"),
                    "waves_per_simd_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                                "waves_per_simd_k_lrb3_bwd"),
                    "launch_ms": round(t_launch * 1e3, 4),
                    "events_per_path": {k: round(v / sample, 3) for k, v in counts["lrb3"].items()}}
        print(f"# lrb3 algorithmic bytes/path {bpp:.0f}  achieved {achieved:.0f} GB/s", file=sys.stderr)

    # ---- per-method / per-depth sweep: differentiated paths/s, bytes/path.
    # Side state is what the call's API sizes (lt_side_state_bytes); the
    # measured figure is the device memory the step holds beyond the inputs
    # (the side-state tensor, the library workspace it grows: hand-off,
    # guide records), from hipMemGetInfo before and after, with a fresh
    # context per entry so that nothing is left over from the last one.
    sweep = {}
    if not args.no_sweep:
        recs = {"naive": lt.RECORD_TAPE, "reslrb": lt.RECORD_RESERVOIR, "lrb3": 0, "lrb2": lt.RECORD_SPLATS}
        for d in (8, 16, 32):
            for mode in ("naive", "reslrb", "lrb3", "lrb2"):
                rec = recs[mode]
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                free0 = torch.cuda.mem_get_info(dev)[0]
                mctx = lt.Context(0).scene_upload(sc)
                a = mctx.args(3000, N, d, rec)
                nb = mctx.side_state_bytes(a)
                side = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
                ts = []
                for k in range(4):
                    a = mctx.args(3000 + k, N, d, rec)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    mctx.trace(a, p, img, side)
                    mctx.loss_l2(img, target, dI, loss)
                    if mode == "naive":
                        mctx.backward_naive(a, p, dI, side, g_alb, g_le)
                    elif mode == "reslrb":
                        mctx.backward_reslrb(a, p, dI, side, g_alb, g_le)
                    elif mode == "lrb2":
                        mctx.backward_lrb2(a, p, dI, side, g_alb, g_le)
                    else:
                        mctx.backward_lrb3(a, p, dI, g_alb, g_le)
                    e1.record(stream)
                    e1.synchronize()
                    if k:
                        ts.append(e0.elapsed_time(e1))
                held = free0 - torch.cuda.mem_get_info(dev)[0]
                ws = mctx.workspace_bytes(a)
                del side, mctx
                ms = float(np.median(ts))
                sweep[f"{mode}_d{d}"] = {"ms": round(ms, 3), "paths_per_s": round(N / (ms * 1e-3)),
                                         "side_bytes_per_path": round(nb / N, 2),
                                         "workspace_bytes": ws,
                                         "measured_device_bytes_per_path": round(held / N, 2)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print("# memory per path (measured, D 8/16/32): " + "; ".join(
            f"{m} " + "/".join(f"{sweep[f'{m}_d{d}']['measured_device_bytes_per_path']:.0f}" for d in (8, 16, 32))
            for m in ("naive", "reslrb", "lrb3", "lrb2")), file=sys.stderr, flush=True)

    # ---- equal-error throughput: paths/s x (naive-AD variance / the method's
    # variance), the gradient variance summed over parameters across seeds
    # with one fixed image adjoint (only the estimators differ)
    equal = None
    if not args.no_sweep and f"naive_d{D}" in sweep:
        equal = {}
        dI_fix = dI.clone()
        for mode in ("naive", "reslrb", "lrb3"):
            rec = lt.RECORD_TAPE if mode == "naive" else lt.RECORD_RESERVOIR if mode == "reslrb" else 0
            nb = ctx.side_state_bytes(ctx.args(4000, N, D, rec))
            side = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
            gs = []
            for k in range(args.ee_seeds):
                a = ctx.args(4000 + k, N, D, rec)
                ctx.trace(a, p, img, side)
                g_alb.zero_(); g_le.zero_()
                if mode == "naive":
                    ctx.backward_naive(a, p, dI_fix, side, g_alb, g_le)
                elif mode == "reslrb":
                    ctx.backward_reslrb(a, p, dI_fix, side, g_alb, g_le)
                else:
                    ctx.backward_lrb3(a, p, dI_fix, g_alb, g_le)
                gs.append(torch.cat([g_alb.flatten(), g_le.flatten()]).double())
            del side
            equal[mode] = {"variance": torch.stack(gs).var(0).sum().item()}
        for mode in equal:
            ms = sweep[f"{mode}_d{D}"]["ms"]
            r = equal["naive"]["variance"] / equal[mode]["variance"]
            equal[mode].update(paths_per_s=round(N / (ms * 1e-3)), variance_ratio_naive_over_method=round(r, 4),
                               equal_error_paths_per_s=round(N / (ms * 1e-3) * r))
        print("# equal-error paths/s (D=%d): " % D + ", ".join(
            f"{m} {v['equal_error_paths_per_s'] / 1e6:.0f}M (variance ratio {v['variance_ratio_naive_over_method']:.3f})"
            for m, v in equal.items()), file=sys.stderr, flush=True)
        torch.cuda.synchronize()

    # ---- attached workload: caustic heightfield slab (gradients w.r.t. heights)
    caustic = None
    if not args.no_caustic:
        caustic = bench_caustic(lt, scenes, dev, stream, bytes_per_path)

    # ---- heightfield inverse rendering: loss against time per reverse mode
    inverse = None
    if not (args.no_caustic or args.no_inverse):
        inverse = bench_inverse(lt, scenes, dev, stream, iters=args.inverse_iters)

    # ---- learned guide: gradient variance x time, guided vs cosine emission
    guide = guide_smooth = None
    if not args.no_guide:
        guide = bench_guide(lt, scenes, dev, stream, iters=args.guide_iters, K=args.guide_seeds, lr=2e-3)
        guide_smooth = bench_guide(lt, scenes, dev, stream, G=64, film=256, N=1 << 22, D=6, iters=60, K=16,
                                   n_train=1 << 18, mode="lrb3", target="gradient", lr=2e-3)

    # ---- batched instances: one persistent launch per pass, hipGraph replay
    batch = batch_small = None
    if not args.no_batch:
        batch = bench_batch(lt, scenes, dev, stream)
        batch_small = bench_batch(lt, scenes, dev, stream, path_scale=1.0 / 64, reps=4)

    # ---- learned guide at diffuse vertices (detail-view box)
    guide_diffuse = None
    if not args.no_guide:
        guide_diffuse = bench_guide_diffuse(lt, scenes, dev, stream)

    # ---- guided + batched against the plain GPU tracer
    guided_batch = None
    if not (args.no_batch or args.no_guide):
        guided_batch = bench_guided_batch(lt, scenes, dev, stream)

    # ---- bidirectional: LRB-3 light paths + path-replay camera samples
    bidir = None
    if not args.no_bidir:
        bidir = bench_bidirectional(lt, scenes, dev, stream, bytes_per_path, cpu=not args.no_cpu)

    # ---- further materials: rough conductor, normal map, textured directional emitter
    materials = None
    if not args.no_materials:
        materials = bench_materials(lt, scenes, dev, stream, bytes_per_path)

    # ---- CPU baseline: the FP64 oracle, forward + naive backward, on a sample
    cpu = cpu1 = cpu_more = None
    if not args.no_cpu:
        from oracle import oracle as O
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        ids = np.arange(args.cpu_paths, dtype=np.uint32)
        dIh = dI.cpu().numpy().astype(np.float64)
        # whole steps (one seed each) until at least --cpu-seconds of work
        reps, t0 = 0, time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < args.cpu_seconds:
            O.render(sc, 2000 + reps, N, D, path_list=ids, threads=threads)
            O.gradient(sc, 2000 + reps, N, D, dIh, path_list=ids, threads=threads)
            reps += 1
        tc = time.perf_counter() - t0
        cpu = {"value": round(reps * args.cpu_paths / tc, 1), "unit": "paths/s", "cores": threads, "kind": "oracle",
               "sample": f"first {args.cpu_paths} of the {N} paths (same scene, depth {D}) for {reps} seeds; "
                         f"forward + taped naive-AD backward in FP64, {tc:.2f} s"}
        n1 = min(args.cpu_paths, 1 << 16)
        ids1 = np.arange(n1, dtype=np.uint32)
        t1 = time.perf_counter()
        O.render(sc, 2000, N, D, path_list=ids1, threads=1)
        O.gradient(sc, 2000, N, D, dIh, path_list=ids1, threads=1)
        t1 = time.perf_counter() - t1
        cpu1 = {"value": round(n1 / t1, 1), "unit": "paths/s", "cores": 1, "kind": "oracle",
                "sample": f"first {n1} paths, one thread, {t1:.2f} s"}
        cpu_more = cpu_baselines(O, scenes, threads, sc, dIh, N)

    out = {
        "metric": "differentiated light paths/s (fwd+bwd) at fixed gradient error; bytes/path vs depth",
        "value": round(value, 1),
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"textured diffuse box, film {W}x{H}, max depth {D}, {N} light paths per step, "
                               "forward + L2 loss + LRB-3-pass detached backward (albedo texels + emitter)",
                   "paths": N, "depth": D, "film": [W, H], "method": "lrb3", "scene": "box"},
        "step_ms": {"forward": round(float(np.median(fwd)), 4), "loss": round(float(np.median(lss)), 4),
                    "backward": round(float(np.median(bwd)), 4)},
        "forward_paths_per_s": round(N / (float(np.median(fwd)) * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "cpu_baseline_workloads": cpu_more,
        "sweep": sweep,
        "equal_error": equal,
        "caustic": caustic,
        "inverse_rendering": inverse,
        "guide": guide,
        "guide_smooth_slab": guide_smooth,
        "batch": batch,
        "batch_small_instances": batch_small,
        "guided_batch": guided_batch,
        "guide_diffuse_detail_box": guide_diffuse,
        "bidirectional": bidir,
        "materials": materials,
    }
    print(json.dumps(out), flush=True)


def cpu_baselines(O, scenes, threads, box, dI_box, N_box, n_box=1 << 18, n_caustic=1 << 15):
    """The FP64 oracle (forward + taped naive backward) on the other
    workloads, each on a bounded sample of its paths whose rate stands for
    the whole job (paths are independent; the rate is per path): the box at
    depth 8 and 16 (2^18 of 4,194,304 paths) and the attached caustic (128^2
    heights, 512^2 film, depth 6; 2^15 of 16,777,216 paths: the oracle finds
    hits by testing every triangle, 33k here)."""
    import numpy as np
    out = {}
    ids = np.arange(n_box, dtype=np.uint32)
    for d in (8, 16):
        t0 = time.perf_counter()
        O.render(box, 2100, N_box, d, path_list=ids, threads=threads)
        O.gradient(box, 2100, N_box, d, dI_box, path_list=ids, threads=threads)
        t = time.perf_counter() - t0
        out[f"box_d{d}"] = {"value": round(n_box / t, 1), "unit": "paths/s", "cores": threads, "kind": "oracle",
                            "sample": f"first {n_box} of {N_box} paths, 256x256 box, depth {d}, {t:.2f} s; "
                                      f"rate per path stands for the whole job"}
    sc = scenes.caustic_scene(G=128, width=512, height=512)
    dI = np.random.default_rng(9).normal(size=(512, 512, 3)) * 1e-3
    ids = np.arange(n_caustic, dtype=np.uint32)
    t0 = time.perf_counter()
    O.render(sc, 2200, 1 << 24, 6, path_list=ids, threads=threads)
    O.gradient(sc, 2200, 1 << 24, 6, dI, flags=O.ATTACHED, path_list=ids, threads=threads)
    t = time.perf_counter() - t0
    out["caustic"] = {"value": round(n_caustic / t, 1), "unit": "paths/s", "cores": threads, "kind": "oracle",
                      "sample": f"first {n_caustic} of 16777216 paths, caustic 128^2 heights, 512^2 film, depth 6, "
                                f"attached, {t:.2f} s; rate per path stands for the whole job"}
    print("# oracle paths/s: " + ", ".join(f"{k} {v['value']:.0f}" for k, v in out.items()), file=sys.stderr,
          flush=True)
    return out


def bench_caustic(lt, scenes, dev, stream, bytes_per_path_fn, G=128, film=512, N=1 << 24, D=6, ee_seeds=8):
    """Attached workload: glass heightfield slab (G x G heights), film^2,
    depth D, N paths; forward + loss + attached backward per method."""
    import numpy as np
    import torch

    sc = scenes.caustic_scene(G=G, width=film, height=film)
    ctx = lt.Context(0).scene_upload(sc)
    albedo = torch.as_tensor(sc["albedo"], dtype=torch.float32, device=dev).contiguous()
    Le = torch.as_tensor(sc["Le"], dtype=torch.float32, device=dev)
    h = torch.as_tensor(sc["heights"], dtype=torch.float32, device=dev).contiguous()
    ht = torch.as_tensor(sc["heights_target"], dtype=torch.float32, device=dev).contiguous()
    img = torch.empty((film, film, 3), dtype=torch.float32, device=dev)
    target, dI = torch.empty_like(img), torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ga, gl, gh = torch.zeros_like(albedo), torch.zeros_like(Le), torch.zeros_like(h)
    ctx.trace(ctx.args(0x7A6, N, D), ctx.params(albedo, Le, ht), target)
    p = ctx.params(albedo, Le, h)
    out = {"workload": f"glass heightfield slab {G}x{G} heights, film {film}x{film}, depth {D}, {N} paths, "
                       "attached gradients w.r.t. heights"}
    for mode in ("lrb3", "reslrb", "naive"):
        rec = lt.RECORD_TAPE if mode == "naive" else lt.RECORD_RESERVOIR if mode == "reslrb" else 0
        a = ctx.args(100, N, D, lt.ATTACHED | rec)
        nb = ctx.side_state_bytes(a)
        side = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
        ts, tb = [], []
        for k in range(4):
            a = ctx.args(100 + k, N, D, lt.ATTACHED | rec)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            ctx.trace(a, p, img, side)
            ctx.loss_l2(img, target, dI, loss)
            e[1].record(stream)
            if mode == "naive":
                ctx.backward_naive(a, p, dI, side, ga, gl, gh)
            elif mode == "reslrb":
                ctx.backward_reslrb(a, p, dI, side, ga, gl, gh)
            else:
                ctx.backward_lrb3(a, p, dI, ga, gl, gh)
            e[2].record(stream)
            e[2].synchronize()
            if k:
                ts.append(e[0].elapsed_time(e[2]))
                tb.append(e[1].elapsed_time(e[2]))
        del side
        ms = float(np.median(ts))
        guards = ctx.stats()["guard_triggers"]  # of the last backward
        out[mode] = {"ms": round(ms, 3), "backward_ms": round(float(np.median(tb)), 3),
                     "paths_per_s": round(N / (ms * 1e-3)), "side_bytes_per_path": round(nb / N, 2),
                     "guard_triggers_per_path": round(guards / N, 6)}
        print(f"# caustic {mode}: step {ms:.3f} ms (backward {np.median(tb):.3f} ms)", file=sys.stderr, flush=True)
    # equal-error form: heights-gradient variance over seeds with one fixed
    # image adjoint, per method (the paper expects ResLRB close to LRB-3
    # here: a caustic path has about one sensor connection)
    dI_fix = dI.clone()
    var = {}
    for mode in ("naive", "reslrb", "lrb3"):
        rec = lt.RECORD_TAPE if mode == "naive" else lt.RECORD_RESERVOIR if mode == "reslrb" else 0
        nb = ctx.side_state_bytes(ctx.args(0, N, D, lt.ATTACHED | rec))
        side = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
        gs = []
        for k in range(ee_seeds):
            a = ctx.args(7000 + k, N, D, lt.ATTACHED | rec)
            ctx.trace(a, p, img, side)
            ga.zero_(); gl.zero_(); gh.zero_()
            if mode == "naive":
                ctx.backward_naive(a, p, dI_fix, side, ga, gl, gh)
            elif mode == "reslrb":
                ctx.backward_reslrb(a, p, dI_fix, side, ga, gl, gh)
            else:
                ctx.backward_lrb3(a, p, dI_fix, ga, gl, gh)
            gs.append(gh.double().clone())
        del side
        var[mode] = torch.stack(gs).var(0).sum().item()
    for mode in var:
        r = var["naive"] / var[mode]
        out[mode].update(heights_variance=var[mode], variance_ratio_naive_over_method=round(r, 4),
                         equal_error_paths_per_s=round(out[mode]["paths_per_s"] * r))
    print("# caustic equal-error paths/s: " + ", ".join(
        f"{m} {out[m]['equal_error_paths_per_s'] / 1e6:.0f}M (variance ratio {out[m]['variance_ratio_naive_over_method']:.3f})"
        for m in var), file=sys.stderr, flush=True)
    # byte model of the attached LRB-3 backward from the counters build
    try:
        sample = 1 << 18
        cctx = lt.Context(0, counters=True).scene_upload(sc)
        cctx.read_counters(reset=True)
        a = cctx.args(100, sample, D, lt.ATTACHED)
        cctx.trace(cctx.args(100, sample, D), p, img)
        cctx.read_counters(reset=True)
        cctx.backward_lrb3(a, p, dI, torch.zeros_like(albedo), torch.zeros_like(Le), torch.zeros_like(h))
        c = cctx.read_counters(reset=True)
        bpp = bytes_per_path_fn(c, sample)
        t = out["lrb3"]["backward_ms"] * 1e-3
        achieved = bpp * N / t / 1e9
        traffic = profiled_traffic("k_lrb3_att_p2_p3_caustic128_512_d6_16M.txt")
        out["lrb3_roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_path": round(bpp, 1),
                                "kernel": "k_lrb3_att_p2 + k_lrb3_att_p3",
                                "traffic": traffic,
                                "traffic_frac": None if traffic is None else round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                                "valu_issue_frac_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                                             "valu_issue_frac_k_lrb3_att"),
                                "l2_hit_rate_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                                         "l2_hit_rate_k_lrb3_att"),
                                "waves_per_simd_profiled": profiled_traffic("k_lrb3_caustic128_box256_valu.txt",
                                                                            "waves_per_simd_k_lrb3_att"),
                                "events_per_path": {k: round(v / sample, 3) for k, v in c.items()}}
        del cctx
    except Exception as e:
        print(f"# caustic counters unavailable: {e}", file=sys.stderr)
    return out


def bench_guide(lt, scenes, dev, stream, G=256, film=1024, N=1 << 26, D=8, iters=40, K=12, n_train=1 << 20,
                mode="naive", target="adjoint", lr=1e-2):
    """Learned emission guide on the caustic scene (film^2, G x G heights,
    depth D, N paths per iteration): the guide is trained online on the
    per-path signal the backward writes (target "adjoint": |delta_total|, the
    adjoint-weighted contribution; "gradient": the L1 norm of the path's
    heights gradient), then the heights gradient over K seeds (fixed image
    adjoint) and the time per forward + backward iteration are compared with
    cosine emission.  Two dispersions: the sample variance summed over heights,
    and the median over heights of the per-height variance.  On a rough slab
    the attached per-path derivative is heavy-tailed (focusing at caustic
    folds, grazing hits): single paths then set the sample variance of K
    seeds, and the median is the stable measure of the sampling."""
    import numpy as np
    import torch

    sc = scenes.caustic_scene(G=G, width=film, height=film)
    ctx = lt.Context(0).scene_upload(sc)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    albedo, Le, h, ht = f32(sc["albedo"]), f32(sc["Le"]), f32(sc["heights"]), f32(sc["heights_target"])
    img = torch.empty((film, film, 3), dtype=torch.float32, device=dev)
    target_img, dI = torch.empty_like(img), torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ctx.trace(ctx.args(0x7A6, N, D, lt.ATTACHED), ctx.params(albedo, Le, ht), target_img)
    ctx.trace(ctx.args(0x7A7, N, D, lt.ATTACHED), ctx.params(albedo, Le, h), img)
    ctx.loss_l2(img, target_img, dI, loss)
    ga, gl, gh = torch.zeros_like(albedo), torch.zeros_like(Le), torch.zeros_like(h)
    flags = lt.ATTACHED | (lt.RECORD_TAPE if mode == "naive" else 0)
    extra = lt.CONTRIB_ADJOINT if target == "adjoint" else 0
    nb = ctx.side_state_bytes(ctx.args(0, N, D, flags))
    tape = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None

    def iteration(seed, gw, contrib=None):
        p = ctx.params(albedo, Le, h, gw)
        ctx.trace(ctx.args(seed, N, D, flags), p, img, tape)
        ga.zero_(); gl.zero_(); gh.zero_()
        a = ctx.args(seed, N, D, flags | extra, contrib=contrib)
        if mode == "naive":
            ctx.backward_naive(a, p, dI, tape, ga, gl, gh)
        else:
            ctx.backward_lrb3(a, p, dI, ga, gl, gh)

    def estimate(gw):
        gs, ts = [], []
        iteration(69999, gw)  # warm-up
        for k in range(K):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            iteration(70000 + k, gw)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
            gs.append(gh.double().clone())
        return torch.stack(gs), float(np.median(ts))

    g0, t0 = estimate(None)
    w = f32(scenes.guide_weights())
    m, v, gw_grad = torch.zeros_like(w), torch.zeros_like(w), torch.zeros_like(w)
    gloss = torch.zeros(1, dtype=torch.float32, device=dev)
    contrib = torch.zeros(N, dtype=torch.float32, device=dev)
    n_train = min(n_train, N)
    smp = torch.zeros((n_train, 12), dtype=torch.float32, device=dev)
    tt = []
    for it in range(1, iters + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        iteration(60000 + it, w, contrib)
        e1.record(stream)
        p = ctx.params(albedo, Le, h, w)
        ctx.guide_emit(ctx.args(60000 + it, n_train, D), p, smp, contrib)
        ctx.guide_grad(w, smp, gw_grad, gloss)
        ctx.guide_adam(w, gw_grad, m, v, it, lr)
        e2.record(stream)
        e2.synchronize()
        tt.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
    g1, t1 = estimate(w)
    dropped = ctx.stats()["nonfinite"]
    del tape
    v0, v1 = g0.var(0), g1.var(0)
    se = torch.sqrt(v0 / K + v1 / K)
    ok = se > 0
    z2 = ((g1.mean(0) - g0.mean(0))[ok] / se[ok]) ** 2
    tv0, tv1, mv0, mv1 = v0.sum().item(), v1.sum().item(), v0.median().item(), v1.median().item()
    # bootstrap over seeds (both sides resampled): how far single heavy-tailed
    # paths move the summed-variance ratio
    gen = torch.Generator(device=g0.device)
    gen.manual_seed(12345)
    boot = []
    for _ in range(200):
        i0 = torch.randint(K, (K,), device=g0.device, generator=gen)
        i1 = torch.randint(K, (K,), device=g0.device, generator=gen)
        boot.append(g1[i1].var(0).sum().item() / max(g0[i0].var(0).sum().item(), 1e-300))
    ci = [round(float(x), 4) for x in np.percentile(boot, [5, 95])]
    cos_share = float((smp[:, 11] == 0).float().mean().item())
    est = "naive-AD" if mode == "naive" else "LRB-3-pass"
    out = {"workload": f"glass heightfield slab {G}x{G} heights, film {film}x{film}, depth {D}, {N} paths per "
                       f"iteration, attached {est} gradients w.r.t. heights; guide trained online for {iters} "
                       f"iterations on {n_train} samples each (target: {target})",
           "ms_per_iter_cosine": round(t0, 3), "ms_per_iter_guided": round(t1, 3),
           "train_ms_per_iter": round(float(np.median([a + b for a, b in tt])), 3),
           "guide_update_ms": round(float(np.median([b for _, b in tt])), 3),
           "variance_cosine": tv0, "variance_guided": tv1, "variance_ratio": round(tv1 / tv0, 4),
           "variance_ratio_bootstrap_90": ci,
           "median_coord_variance_ratio": round(mv1 / mv0, 4),
           "efficiency_gain": round((tv0 * t0) / (tv1 * t1), 4),
           "robust_efficiency_gain": round((mv0 * t0) / (mv1 * t1), 4),
           "bias_mean_z2": round(float(z2.mean().item()), 4), "bias_median_z2": round(float(z2.median().item()), 4),
           "seeds": K, "cosine_share_after_training": round(cos_share, 4),
           "nonfinite_dropped_last_iteration": int(dropped)}
    print(f"# guide G={G}: variance ratio {tv1 / tv0:.3f} (bootstrap 90% {ci[0]:.3f}-{ci[1]:.3f}; "
          f"median-coordinate {mv1 / mv0:.3f}), "
          f"iteration {t0:.1f} -> {t1:.1f} ms, efficiency gain {out['efficiency_gain']} "
          f"(robust {out['robust_efficiency_gain']}), bias z^2 {out['bias_mean_z2']}", file=sys.stderr, flush=True)
    return out


def _boot_ratio(g0, g1, stat, n=200, seed=12345):
    """Bootstrap (both sides' seeds resampled) 5th-95th percentiles of
    stat(var of g1) / stat(var of g0) over the per-seed gradients g [K, P]."""
    import numpy as np
    import torch
    gen = torch.Generator(device=g0.device)
    gen.manual_seed(seed)
    K0, K1 = g0.shape[0], g1.shape[0]
    out = []
    for _ in range(n):
        i0 = torch.randint(K0, (K0,), device=g0.device, generator=gen)
        i1 = torch.randint(K1, (K1,), device=g0.device, generator=gen)
        out.append(stat(g1[i1].var(0)) / max(stat(g0[i0].var(0)), 1e-300))
    return [round(float(x), 4) for x in np.percentile(out, [5, 95])]


def bench_guide_diffuse(lt, scenes, dev, stream, film=256, N=1 << 22, D=8, iters=40, K=24, n_train=1 << 18,
                        lr=2e-3):
    """Learned guide at diffuse vertices on the box seen through a narrow
    window (film^2, depth D, N paths per iteration, detached LRB-3-pass
    albedo gradients): cosine sampling against a guide trained online on
    emission samples only (used at vertex 0) and one trained on emission plus
    diffuse-vertex samples (used at vertex 0 and every Lambertian vertex).
    Variance over K seeds (summed and median over texels, with bootstrap 90%
    intervals of the ratios), time per backward, efficiency gain =
    (variance x time) cosine / guided."""
    import numpy as np
    import torch

    sc = scenes.box_detail_scene(width=film, height=film)
    ctx = lt.Context(0).scene_upload(sc)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    alb, Le = f32(sc["albedo"]), f32(sc["Le"])
    img = torch.empty((film, film, 3), dtype=torch.float32, device=dev)
    T, dI, loss = torch.empty_like(img), torch.empty_like(img), torch.zeros(1, dtype=torch.float32, device=dev)
    ctx.trace(ctx.args(1, 1 << 24, D), ctx.params(f32(sc["albedo_target"]), Le), T)
    ctx.trace(ctx.args(2, 1 << 24, D), ctx.params(alb, Le), img)
    ctx.loss_l2(img, T, dI, loss)
    ga, gl = torch.zeros_like(alb), torch.zeros_like(Le)

    def step(seed, w, flags, contrib=None):
        ga.zero_(); gl.zero_()
        ctx.backward_lrb3(ctx.args(seed, N, D, flags | lt.CONTRIB_ADJOINT, contrib=contrib),
                          ctx.params(alb, Le, None, w), dI, ga, gl)

    def estimate(w, flags):
        step(69999, w, flags)
        gs, ts = [], []
        for k in range(K):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            step(70000 + k, w, flags)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
            gs.append(ga.double().clone())
        return torch.stack(gs), float(np.median(ts))

    def train(diffuse):
        w = f32(scenes.guide_weights())
        m, v, g1, g2 = (torch.zeros_like(w) for _ in range(4))
        contrib = torch.zeros(N, dtype=torch.float32, device=dev)
        se = torch.zeros((n_train, 12), dtype=torch.float32, device=dev)
        sd = torch.zeros_like(se)
        flags = lt.GUIDE_DIFFUSE if diffuse else 0
        for i in range(1, iters + 1):
            step(60000 + i, w, flags, contrib)
            p = ctx.params(alb, Le, None, w)
            ctx.guide_emit(ctx.args(60000 + i, n_train, D), p, se, contrib)
            ctx.guide_grad(w, se, g1, None)
            if diffuse:
                ctx.guide_vertex_samples(ctx.args(60000 + i, n_train, D, lt.GUIDE_DIFFUSE), p, sd)
                ctx.guide_grad(w, sd, g2, None)
                g1 += g2
            ctx.guide_adam(w, g1, m, v, i, lr)
        return w

    g0, t0 = estimate(None, 0)
    out = {"workload": f"diffuse box seen through a 12-degree window, film {film}x{film}, depth {D}, {N} paths, "
                       f"detached LRB-3-pass albedo gradients over {K} seeds; guides trained online for {iters} "
                       f"iterations on {n_train} samples of each kind",
           "ms_per_backward_cosine": round(t0, 3)}
    for name, diffuse in (("emission_only", False), ("emission_and_diffuse", True)):
        w = train(diffuse)
        g1, t1 = estimate(w, lt.GUIDE_DIFFUSE if diffuse else 0)
        v0, v1 = g0.var(0), g1.var(0)
        se = torch.sqrt(v0 / K + v1 / K)
        ok = se > 0
        z2 = ((g1.mean(0) - g0.mean(0))[ok] / se[ok]) ** 2
        vr, mr = v1.sum().item() / v0.sum().item(), v1.median().item() / v0.median().item()
        out[name] = {"ms_per_backward": round(t1, 3), "variance_ratio": round(vr, 4),
                     "variance_ratio_bootstrap_90": _boot_ratio(g0, g1, lambda v: v.sum().item()),
                     "median_texel_variance_ratio": round(mr, 4),
                     "median_texel_ratio_bootstrap_90": _boot_ratio(g0, g1, lambda v: v.median().item()),
                     "efficiency_gain": round(t0 / (vr * t1), 4), "robust_efficiency_gain": round(t0 / (mr * t1), 4),
                     "bias_mean_z2": round(float(z2.mean().item()), 4)}
        print(f"# diffuse guide ({name}): variance ratio {vr:.3f} {out[name]['variance_ratio_bootstrap_90']}, "
              f"median-texel {mr:.3f} {out[name]['median_texel_ratio_bootstrap_90']}, {t0:.2f} -> {t1:.2f} ms, "
              f"gain {out[name]['efficiency_gain']} (robust {out[name]['robust_efficiency_gain']}), "
              f"z^2 {out[name]['bias_mean_z2']}", file=sys.stderr, flush=True)
    return out


def bench_materials(lt, scenes, dev, stream, bytes_per_path_fn, G=128, film=512, N=1 << 24, D=6, reps=4):
    """The further materials and parameters of the paper's validation scenes
    at the attached workload's size (G x G heightfield, film^2, depth D, N
    paths), one LRB-3 optimisation step each (forward, L2 loss, backward):
    Mirror (rough-conductor heightfield, attached gradients w.r.t. the
    heights), Glass Panel (normal-mapped dielectric, attached gradients
    w.r.t. the normal map), Tumbler (glass under a directional emitter with
    a radiance texture, detached gradients w.r.t. that texture and the
    albedo).  The backward's roofline uses the byte model of the counters
    build on a 2^18-path sample."""
    import numpy as np
    import torch
    t32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    cases = (
        ("mirror", scenes.mirror_scene(G=G, width=film, height=film), lt.ATTACHED,
         "rough-conductor heightfield (GGX) lighting a diffuse wall, attached gradients w.r.t. the heights"),
        ("glass_panel", scenes.glass_panel_scene(G=G, width=film, height=film), lt.ATTACHED,
         "normal-mapped glass panel over a diffuse receiver, attached gradients w.r.t. the normal map"),
        ("tumbler", scenes.tumbler_scene(G=G, width=film, height=film), 0,
         "glass heightfield under a directional emitter with an 8x8 radiance texture, detached gradients "
         "w.r.t. the emitter texture and the albedo"),
    )
    out = {}
    for name, sc, flags, what in cases:
        ctx = lt.Context(0).scene_upload(sc)
        albedo, Le, h = t32(sc["albedo"]), t32(sc["Le"]), t32(sc["heights"])
        nm = t32(sc["normal_map"]) if "normal_map" in sc else None
        img = torch.empty((film, film, 3), dtype=torch.float32, device=dev)
        target, dI = torch.empty_like(img), torch.empty_like(img)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        ga, gl = torch.zeros_like(albedo), torch.zeros_like(Le)
        gh = torch.zeros_like(h) if flags else None
        gn = torch.zeros_like(nm) if (flags and nm is not None) else None
        tgt = ctx.params(t32(sc["albedo_target"]) if sc.get("albedo_target") is not None else albedo,
                         t32(sc["Le_target"]) if "Le_target" in sc else Le,
                         t32(sc["heights_target"]) if sc.get("heights_target") is not None else h,
                         normal_map=t32(sc["normal_map_target"]) if "normal_map_target" in sc else nm)
        ctx.trace(ctx.args(0x7A6, N, D, flags), tgt, target)
        p = ctx.params(albedo, Le, h, normal_map=nm)
        ts, tb = [], []
        for k in range(reps + 1):
            a = ctx.args(100 + k, N, D, flags)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            ctx.trace(a, p, img)
            ctx.loss_l2(img, target, dI, loss)
            e[1].record(stream)
            ctx.backward_lrb3(a, p, dI, ga, gl, gh, gn)
            e[2].record(stream)
            e[2].synchronize()
            if k:
                ts.append(e[0].elapsed_time(e[2]))
                tb.append(e[1].elapsed_time(e[2]))
        ms, bms = float(np.median(ts)), float(np.median(tb))
        r = {"workload": f"{what}; {G}x{G} heightfield, film {film}x{film}, depth {D}, {N} paths",
             "ms": round(ms, 3), "backward_ms": round(bms, 3), "paths_per_s": round(N / (ms * 1e-3)),
             "guard_triggers_per_path": round(ctx.stats()["guard_triggers"] / N, 6) if flags else 0.0}
        try:
            sample = 1 << 18
            cctx = lt.Context(0, counters=True).scene_upload(sc)
            a = cctx.args(100, sample, D, flags)
            cctx.trace(a, p, img)
            cctx.read_counters(reset=True)
            cctx.backward_lrb3(a, p, dI, torch.zeros_like(albedo), torch.zeros_like(Le),
                               None if gh is None else torch.zeros_like(h), None if gn is None else torch.zeros_like(nm))
            c = cctx.read_counters(reset=True)
            del cctx
            bpp = bytes_per_path_fn(c, sample)
            achieved = bpp * N / (bms * 1e-3) / 1e9
            r["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_path": round(bpp, 1),
                             "kernel": "LRB-3 backward (attached pair)" if flags else "k_lrb3_bwd",
                             "traffic": None,
                             "events_per_path": {k: round(v / sample, 3) for k, v in c.items()}}
        except Exception as e:
            print(f"# {name} counters unavailable: {e}", file=sys.stderr)
        out[name] = r
        fr = r.get("roofline", {}).get("frac")
        print(f"# {name}: step {ms:.2f} ms (backward {bms:.2f} ms), {N / (ms * 1e-3) / 1e6:.0f}M paths/s"
              + (f", backward frac {fr:.3f}" if fr is not None else ""), file=sys.stderr, flush=True)
        del ctx
    return out


def bench_bidirectional(lt, scenes, dev, stream, bytes_per_path_fn, G=64, film=256, N_lt=1 << 22, spp=16, D=8,
                        reps=6, cpu=True):
    """Glass slab seen from above: the light tracer (LRB-3 backward) covers
    the camera paths whose first vertex is diffuse, camera samples with a
    path-replay backward those whose first vertex is specular (the surface
    seen through the glass).  One step: both forwards into one image, the L2
    loss, both backwards into one gradient."""
    import numpy as np
    import torch
    sc = scenes.glass_slab_scene(G=G, width=film, height=film)
    ctx = lt.Context(0).scene_upload(sc)
    t32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    albedo, Le, h = t32(sc["albedo"]), t32(sc["Le"]), t32(sc["heights"])
    alb_t = t32(sc["albedo_target"])
    n_cam = spp * film * film
    img = torch.zeros((film, film, 3), dtype=torch.float32, device=dev)
    target = torch.zeros_like(img)
    dI = torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g_alb, g_le = torch.zeros_like(albedo), torch.zeros_like(Le)
    p = ctx.params(albedo, Le, h)
    pt = ctx.params(alb_t, Le, h)
    ctx.trace(ctx.args(0x7A6, N_lt, D), pt, target)
    ctx.camera_trace(ctx.args(0x7A7, n_cam, D), pt, target)

    def step(seed, ev=None):
        a_l, a_c = ctx.args(seed, N_lt, D), ctx.args(seed + 0x10000, n_cam, D)
        rec = (lambda i: ev[i].record(stream)) if ev else (lambda i: None)
        rec(0); ctx.trace(a_l, p, img)
        rec(1); ctx.camera_trace(a_c, p, img)
        rec(2); ctx.loss_l2(img, target, dI, loss)
        rec(3); ctx.backward_lrb3(a_l, p, dI, g_alb, g_le)
        rec(4); ctx.camera_backward_prb(a_c, p, dI, g_alb, g_le)
        rec(5)

    for k in range(2):
        step(100 + k)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(reps)]
    for k in range(reps):
        step(200 + k, evs[k])
    torch.cuda.synchronize()
    med = lambda i, j: float(np.median([e[i].elapsed_time(e[j]) for e in evs]))
    t = {"lt_forward": med(0, 1), "camera_forward": med(1, 2), "loss": med(2, 3), "lrb3_backward": med(3, 4),
         "camera_prb_backward": med(4, 5), "step": med(0, 5)}
    # share of the image only camera samples reach (through the glass)
    cam = torch.zeros_like(img)
    ctx.camera_trace(ctx.args(300, n_cam, D), p, cam)
    ctx.trace(ctx.args(301, N_lt, D), p, img)
    torch.cuda.synchronize()
    share = float(cam.sum() / (cam.sum() + img.sum()))
    roof = None
    try:
        cctx = lt.Context(0, counters=True).scene_upload(sc)
        n_s = min(n_cam, 1 << 18)
        cctx.read_counters(reset=True)
        cctx.camera_backward_prb(cctx.args(200, n_s, D), p, dI, torch.zeros_like(albedo), torch.zeros_like(Le))
        c = cctx.read_counters(reset=True)
        del cctx
        # the model's node, triangle and gradient bytes plus the pixel adjoint read
        bps = bytes_per_path_fn(c, n_s) + 12.0
        t_l = t["camera_prb_backward"] * 1e-3
        ach = bps * n_cam / t_l / 1e9
        traffic = profiled_traffic("k_camera_prb_slab64_256_d8_1M.txt") if (G, film, spp, D) == (64, 256, 16, 8) else None
        roof = {"bound": "hbm", "kernel": "k_camera_prb", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_sample": round(bps, 1),
                "traffic": traffic,
                "traffic_frac": None if traffic is None else round(traffic / t_l / 1e9 / HBM_PEAK_GBS, 4),
                "events_per_sample": {k: round(v / n_s, 3) for k, v in c.items()}}
    except Exception as e:  # the diagnostic build is optional
        print(f"# counters unavailable: {e}", file=sys.stderr)
    cpu_rate = None
    if cpu:
        from oracle import oracle as O
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        ids = np.arange(1 << 18, dtype=np.uint32)
        dIh = dI.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        O.render_camera(sc, 200, n_cam, D, path_list=ids, threads=threads)
        O.gradient_camera(sc, 200, n_cam, D, dIh, path_list=ids, threads=threads)
        tc = time.perf_counter() - t0
        cpu_rate = {"value": round(len(ids) / tc, 1), "unit": "camera samples/s (fwd+bwd)", "cores": threads,
                    "kind": "oracle", "sample": f"first {len(ids)} of {n_cam} camera samples, {tc:.2f} s"}
    out = {"workload": f"glass slab (heightfield top {G}x{G}) seen from above, film {film}x{film}, depth {D}: "
                       f"{N_lt} light paths (LRB-3) + {spp} camera samples per pixel ({n_cam}, path replay)",
           "ms": {k: round(v, 3) for k, v in t.items()},
           "light_paths_per_s": round(N_lt / (t["lt_forward"] + t["lrb3_backward"]) * 1e3, 1),
           "camera_samples_per_s": round(n_cam / (t["camera_forward"] + t["camera_prb_backward"]) * 1e3, 1),
           "camera_image_share": round(share, 4),
           "camera_roofline": roof, "camera_cpu_baseline": cpu_rate}
    print(f"# bidirectional: step {t['step']:.2f} ms (light fwd {t['lt_forward']:.2f}, camera fwd "
          f"{t['camera_forward']:.2f}, LRB-3 bwd {t['lrb3_backward']:.2f}, PRB bwd {t['camera_prb_backward']:.2f}); "
          f"camera share of the image {share:.3f}", file=sys.stderr, flush=True)
    return out


def bench_inverse(lt, scenes, dev, stream, G=128, film=512, N=1 << 24, D=6, iters=1000, lr=1e-4, log_every=50):
    """Heightfield inverse rendering: Adam on the slab's free heights (the
    boundary ring stays at zero) toward the image of the seeded sinusoid
    target heights, one attached backward per iteration, per reverse mode.
    Loss against time; the Monte Carlo floor is the loss of the target
    heights themselves rendered with N paths."""
    import numpy as np
    import torch

    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    sc = scenes.caustic_scene(G=G, width=film, height=film)
    ctx = lt.Context(0).scene_upload(sc)
    albedo, Le, ht = f32(sc["albedo"]), f32(sc["Le"]), f32(sc["heights_target"])
    free = torch.zeros((G, G), device=dev)
    free[1:-1, 1:-1] = 1.0
    free = free.reshape(-1)
    T = torch.empty((film, film, 3), dtype=torch.float32, device=dev)
    ctx.trace(ctx.args(0x7A6, 1 << 26, D, lt.ATTACHED), ctx.params(albedo, Le, ht), T)
    img, dI, loss = torch.empty_like(T), torch.empty_like(T), torch.zeros(1, dtype=torch.float32, device=dev)
    ctx.trace(ctx.args(4242, N, D, lt.ATTACHED), ctx.params(albedo, Le, ht), img)
    floor = (img - T).pow(2).mean().item()
    ga, gl = torch.zeros_like(albedo), torch.zeros_like(Le)
    out = {"workload": f"glass heightfield slab {G}x{G} heights, film {film}x{film}, depth {D}, {N} paths per "
                       f"iteration; Adam (lr {lr}, decaying to a tenth) on the free heights toward the image of the sinusoid target "
                       f"heights (rendered with 2^26 paths), {iters} iterations",
           "loss_floor": floor}
    for mode in ("lrb3", "reslrb", "naive"):
        rec = lt.RECORD_TAPE if mode == "naive" else lt.RECORD_RESERVOIR if mode == "reslrb" else 0
        nb = ctx.side_state_bytes(ctx.args(0, N, D, lt.ATTACHED | rec))
        side = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
        h = torch.nn.Parameter(f32(sc["heights"]))
        rmse = lambda: float(torch.sqrt(((h.detach() - ht) ** 2 * free).sum() / free.sum()).item())
        h_rmse0 = rmse()
        opt = torch.optim.Adam([h], lr=lr)
        gh = torch.zeros_like(ht)
        curve = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(iters):
            a = ctx.args(5000 + it, N, D, lt.ATTACHED | rec)
            p = ctx.params(albedo, Le, h.detach())
            ctx.trace(a, p, img, side)
            ctx.loss_l2(img, T, dI, loss)
            gh.zero_(); ga.zero_(); gl.zero_()
            if mode == "naive":
                ctx.backward_naive(a, p, dI, side, ga, gl, gh)
            elif mode == "reslrb":
                ctx.backward_reslrb(a, p, dI, side, ga, gl, gh)
            else:
                ctx.backward_lrb3(a, p, dI, ga, gl, gh)
            h.grad = gh * free
            # step decays exponentially to a tenth over the run: with Monte
            # Carlo gradients a fixed step random-walks the heights the image
            # constrains loosely once the loss is near its floor
            for gr in opt.param_groups:
                gr["lr"] = lr * 0.1 ** (it / max(iters - 1, 1))
            opt.step()
            if it % log_every == 0 or it == iters - 1:
                torch.cuda.synchronize()
                curve.append([it, round(time.perf_counter() - t0, 3), loss.item()])
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        del side
        first = next((t for _, t, l in curve if l <= 2.0 * floor), None)
        out[mode] = {"ms_per_iter": round(total * 1e3 / iters, 3), "loss_first": curve[0][2],
                     "loss_last": curve[-1][2], "time_to_2x_floor_s": first,
                     "heights_rmse_first": h_rmse0, "heights_rmse_last": rmse(), "curve": curve}
        print(f"# inverse {mode}: {total * 1e3 / iters:.1f} ms/iter, loss {curve[0][2]:.3e} -> {curve[-1][2]:.3e} "
              f"(floor {floor:.3e}), 2x floor after {first} s, heights rmse {h_rmse0:.2e} -> {rmse():.2e}",
              file=sys.stderr, flush=True)
    return out


def bench_batch(lt, scenes, dev, stream, n=48, seed=7, reps=2, path_scale=1.0):
    """48 box / caustic instances of uneven heightfield (32^2..256^2), film
    (128^2..1024^2), path count (1M..32M) and depth (4..12) drawn from a
    seed: one optimisation step each (forward, L2 loss, LRB-3-pass backward;
    attached for the caustics).  Per-instance calls against the batched
    runner (autotuned launch shape, one persistent launch per pass, the step
    replayed from a captured hipGraph)."""
    import tempfile

    import numpy as np
    import torch

    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    specs = scenes.batched_instances(n, seed)
    insts = []
    for k, sp in enumerate(specs):
        box = sp["kind"] == "box"
        sc = scenes.box_scene(width=sp["film"], height=sp["film"]) if box else \
            scenes.caustic_scene(G=sp["G"], width=sp["film"], height=sp["film"])
        ctx = lt.Context(0).scene_upload(sc)
        npaths = max(1, int(sp["n_paths"] * path_scale))
        d = dict(ctx=ctx, seed=5000 + k, n_paths=npaths, depth=sp["depth"], attached=not box,
                 albedo=f32(sc["albedo"]), Le=f32(sc["Le"]), heights=None if box else f32(sc["heights"]), guide=None)
        tgt = torch.empty((sp["film"], sp["film"], 3), dtype=torch.float32, device=dev)
        tp = ctx.params(f32(sc["albedo_target"]) if box else d["albedo"], d["Le"],
                        None if box else f32(sc["heights_target"]))
        ctx.trace(ctx.args(0x7A6, min(npaths, 1 << 22), sp["depth"], 0 if box else lt.ATTACHED), tp, tgt)
        d.update(target=tgt, image=torch.empty_like(tgt), d_image=torch.empty_like(tgt),
                 loss=torch.zeros(1, dtype=torch.float32, device=dev), g_albedo=torch.zeros_like(d["albedo"]),
                 g_Le=torch.zeros_like(d["Le"]), g_heights=None if box else torch.zeros_like(d["heights"]))
        insts.append(d)
    total = sum(d["n_paths"] for d in insts)
    torch.cuda.synchronize()

    def per_instance():
        for d in insts:
            ctx = d["ctx"]
            a = ctx.args(d["seed"], d["n_paths"], d["depth"], lt.ATTACHED if d["attached"] else 0)
            p = ctx.params(d["albedo"], d["Le"], d["heights"])
            ctx.trace(a, p, d["image"])
            ctx.loss_l2(d["image"], d["target"], d["d_image"], d["loss"])
            ctx.backward_lrb3(a, p, d["d_image"], d["g_albedo"], d["g_Le"], d["g_heights"])

    def timed(fn):
        ts = []
        for r in range(reps + 1):
            for d in insts:
                d["seed"] += 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    t_inst = timed(per_instance)
    b = lt.Batch(0)
    t_tune0 = time.perf_counter()
    tune = b.autotune(insts, os.path.join(tempfile.gettempdir(), "lt_batch_tuning.json"))
    t_tune = time.perf_counter() - t_tune0
    t_eager = timed(lambda: b.step(insts, use_graph=False))
    t_graph = timed(lambda: b.step(insts, use_graph=True))
    lo, hi = min(d["n_paths"] for d in insts), max(d["n_paths"] for d in insts)
    out = {"workload": f"{n} instances ({sum(1 for d in insts if not d['attached'])} box, "
                       f"{sum(1 for d in insts if d['attached'])} caustic; heightfields 32^2..256^2, films "
                       f"128^2..1024^2, {lo}..{hi} paths, depth 4..12, drawn from seed {seed}); one step each = "
                       "forward + L2 loss + LRB-3-pass backward (attached for caustics)",
           "paths_per_step": total, "per_instance_ms": round(t_inst, 2), "batched_eager_ms": round(t_eager, 2),
           "batched_graph_ms": round(t_graph, 2),
           "per_instance_paths_per_s": round(total / (t_inst * 1e-3)),
           "batched_graph_paths_per_s": round(total / (t_graph * 1e-3)),
           "speedup": round(t_inst / t_graph, 3), "tuning": tune, "autotune_s": round(t_tune, 2)}
    print(f"# batch: per-instance {t_inst:.1f} ms, batched {t_eager:.1f} ms (eager) / {t_graph:.1f} ms (graph), "
          f"speedup {t_inst / t_graph:.3f}, tuning {tune}", file=sys.stderr, flush=True)
    return out


def bench_guided_batch(lt, scenes, dev, stream, n=12, seed=11, iters=50, K=32, n_train=1 << 18, lr=2e-3):
    """Guided + batched against the plain GPU tracer.  n smooth-slab caustic
    instances (sizes and scenes from a seed) take optimisation steps
    (forward, L2 loss and image adjoint, attached LRB-3 backward).  Plain:
    per-instance calls with cosine emission.  Guided + batched: every
    instance's guide is first trained online on its own per-path gradient
    magnitudes (per-instance calls, `iters` steps; reported apart, as a cost
    an optimisation pays once), then the steps run as one batched hipGraph
    replay with guided emission.  Per instance: the heights-gradient variance
    over K seeds (each step with its own image and adjoint); per step: the
    time of all instances.  Gain = geometric mean over instances of
    (variance x time) plain / guided-batched; the robust gain uses the median
    per-height variance instead of the sum."""
    import tempfile

    import numpy as np
    import torch

    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev).contiguous()
    specs = scenes.guided_batch_instances(n, seed)
    insts = []
    for sp in specs:
        sc = scenes.caustic_scene(G=sp["G"], width=sp["film"], height=sp["film"], seed=sp["scene_seed"],
                                  target_seed=sp["target_seed"])
        ctx = lt.Context(0).scene_upload(sc)
        d = dict(ctx=ctx, seed=0, n_paths=sp["n_paths"], depth=sp["depth"], attached=True, albedo=f32(sc["albedo"]),
                 Le=f32(sc["Le"]), heights=f32(sc["heights"]), guide=None)
        tgt = torch.empty((sp["film"], sp["film"], 3), dtype=torch.float32, device=dev)
        ctx.trace(ctx.args(0x7A6, 1 << 22, sp["depth"], lt.ATTACHED), ctx.params(d["albedo"], d["Le"],
                  f32(sc["heights_target"])), tgt)
        d.update(target=tgt, image=torch.empty_like(tgt), d_image=torch.empty_like(tgt),
                 loss=torch.zeros(1, dtype=torch.float32, device=dev), g_albedo=torch.zeros_like(d["albedo"]),
                 g_Le=torch.zeros_like(d["Le"]), g_heights=torch.zeros_like(d["heights"]))
        insts.append(d)
    torch.cuda.synchronize()
    seed_of = lambda s, k: s + 7919 * k

    def zero():
        for d in insts:
            d["g_albedo"].zero_(); d["g_Le"].zero_(); d["g_heights"].zero_()

    def per_instance(s, contrib=None):
        zero()
        for k, d in enumerate(insts):
            ctx = d["ctx"]
            a = ctx.args(seed_of(s, k), d["n_paths"], d["depth"], lt.ATTACHED,
                         contrib=None if contrib is None else contrib[k])
            p = ctx.params(d["albedo"], d["Le"], d["heights"], d["guide"])
            ctx.trace(a, p, d["image"])
            ctx.loss_l2(d["image"], d["target"], d["d_image"], d["loss"])
            ctx.backward_lrb3(a, p, d["d_image"], d["g_albedo"], d["g_Le"], d["g_heights"])

    b = lt.Batch(0)

    def batched(s):
        zero()
        for k, d in enumerate(insts):
            d["seed"] = seed_of(s, k)
        b.step(insts, use_graph=True)

    def timed(fn, reps=4):
        fn(80000)
        ts = []
        for r in range(reps):
            torch.cuda.synchronize(); t0 = time.perf_counter()
            fn(81000 + 1000 * r)
            torch.cuda.synchronize(); ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    def measure(fn):
        gs, ts = [[] for _ in insts], []
        fn(90000)
        for r in range(K):
            torch.cuda.synchronize(); t0 = time.perf_counter()
            fn(100000 + 1000 * r)
            torch.cuda.synchronize(); ts.append(time.perf_counter() - t0)
            for k, d in enumerate(insts):
                gs[k].append(d["g_heights"].double().clone())
        return [torch.stack(g) for g in gs], float(np.median(ts)) * 1e3

    g0, t0 = measure(per_instance)            # plain: cosine emission, per-instance calls
    b.autotune(insts, os.path.join(tempfile.gettempdir(), "lt_guided_batch_tuning.json"))
    t_cos_batched = timed(batched)
    # train every instance's guide on its own gradient-magnitude signal
    contrib = [torch.zeros(d["n_paths"], dtype=torch.float32, device=dev) for d in insts]
    opt = []
    for d in insts:
        d["guide"] = f32(scenes.guide_weights())
        w = d["guide"]
        opt.append(dict(m=torch.zeros_like(w), v=torch.zeros_like(w), g=torch.zeros_like(w),
                        smp=torch.zeros((min(n_train, d["n_paths"]), 12), dtype=torch.float32, device=dev)))
    torch.cuda.synchronize(); tt0 = time.perf_counter()
    for it in range(1, iters + 1):
        s = 60000 + 1000 * it
        per_instance(s, contrib)
        for k, d in enumerate(insts):
            ctx, o = d["ctx"], opt[k]
            p = ctx.params(d["albedo"], d["Le"], d["heights"], d["guide"])
            ctx.guide_emit(ctx.args(seed_of(s, k), o["smp"].shape[0], d["depth"]), p, o["smp"], contrib[k])
            ctx.guide_grad(d["guide"], o["smp"], o["g"], None)
            ctx.guide_adam(d["guide"], o["g"], o["m"], o["v"], it, lr)
    torch.cuda.synchronize(); train_s = time.perf_counter() - tt0
    t_guided_inst = timed(per_instance)
    g1, t1 = measure(batched)                 # guided + batched (graph replays)
    for d in insts:
        d["guide"] = None
    ratios, robust, z2 = [], [], []
    for a, c in zip(g0, g1):
        v0, v1 = a.var(0), c.var(0)
        ratios.append(v1.sum().item() / v0.sum().item())
        robust.append(v1.median().item() / max(v0.median().item(), 1e-300))
        se = torch.sqrt(v0 / K + v1 / K)
        ok = se > 0
        z = (c.mean(0) - a.mean(0))[ok] / se[ok]
        z2.append((z * z).mean().item())
    gm = lambda xs: float(np.exp(np.mean(np.log(np.asarray(xs)))))
    gain = gm([1.0 / r for r in ratios]) * t0 / t1
    rgain = gm([1.0 / r for r in robust]) * t0 / t1
    # bootstrap over seeds (each instance's K seeds resampled on both sides):
    # 90% intervals of both gains; the robust (median-coordinate) gain is the
    # estimator fixed in advance for the conclusion
    gen = torch.Generator(device=g0[0].device)
    gen.manual_seed(12345)
    bg, brg = [], []
    for _ in range(200):
        rr, rb = [], []
        for a, c in zip(g0, g1):
            i0 = torch.randint(K, (K,), device=a.device, generator=gen)
            i1 = torch.randint(K, (K,), device=a.device, generator=gen)
            v0, v1 = a[i0].var(0), c[i1].var(0)
            rr.append(v1.sum().item() / max(v0.sum().item(), 1e-300))
            rb.append(v1.median().item() / max(v0.median().item(), 1e-300))
        bg.append(gm([1.0 / max(r, 1e-300) for r in rr]) * t0 / t1)
        brg.append(gm([1.0 / max(r, 1e-300) for r in rb]) * t0 / t1)
    gain_ci = [round(float(x), 3) for x in np.percentile(bg, [5, 95])]
    rgain_ci = [round(float(x), 3) for x in np.percentile(brg, [5, 95])]
    if rgain_ci[0] > 1.0:
        verdict = "guided+batched beats the plain tracer at equal gradient error (robust gain interval above 1)"
    elif rgain_ci[1] < 1.0:
        verdict = "no gain: the plain tracer is more efficient (robust gain interval below 1)"
    else:
        verdict = "no resolved gain: the robust gain interval contains 1"
    total = sum(d["n_paths"] for d in insts)
    out = {"workload": f"{n} glass-slab caustic instances (heightfields 32^2..96^2, films 128^2..384^2, "
                       f"{min(d['n_paths'] for d in insts)}..{max(d['n_paths'] for d in insts)} paths, depth 6, "
                       f"scenes and sizes from seed {seed}); one step each = forward + L2 loss + attached LRB-3 "
                       f"backward; heights-gradient variance over {K} seeds",
           "paths_per_step": total, "plain_per_instance_cosine_ms": round(t0, 2),
           "batched_cosine_ms": round(t_cos_batched, 2), "per_instance_guided_ms": round(t_guided_inst, 2),
           "batched_guided_ms": round(t1, 2), "guide_training_s": round(train_s, 2), "training_steps": iters,
           "variance_ratio_geomean": round(gm(ratios), 4), "median_coord_variance_ratio_geomean": round(gm(robust), 4),
           "variance_ratio_per_instance": [round(r, 3) for r in ratios],
           "efficiency_gain": round(gain, 3), "robust_efficiency_gain": round(rgain, 3),
           "efficiency_gain_bootstrap_90": gain_ci, "robust_efficiency_gain_bootstrap_90": rgain_ci,
           "conclusion": verdict,
           "bias_mean_z2": round(float(np.mean(z2)), 3)}
    print(f"# guided+batched ({n} slabs): plain {t0:.1f} ms/step, batched cosine {t_cos_batched:.1f}, "
          f"guided per-instance {t_guided_inst:.1f}, guided batched {t1:.1f}; variance ratio (geomean) "
          f"{gm(ratios):.3f}, median-coordinate {gm(robust):.3f}; gain {gain:.2f}x {gain_ci} "
          f"(robust {rgain:.2f}x {rgain_ci}: {verdict}); "
          f"bias z^2 {np.mean(z2):.3f}; training {train_s:.1f} s", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
